#!/usr/bin/env python3
"""K3 bubble throughput on one MI355X: split-FP32 vs FP64 MFMA at rel err <= 1e-6.

Workload (the headline configuration): channel-a bubble B_a(Gamma, Gamma) of the
particle-hole symmetric Anderson model, U = 1, T = 0.1, Delta = 1, N = 201 points per
frequency axis (tangent grid on [-20, 20]), 2001 Gauss-Legendre nodes for the v''
integral; Gamma = Gamma_0 + second-order K1 in all three channels + 1e-3 complex Gaussian
noise on every class entry (seed 0).  One step = one kqft_bubble call producing all four
asymptotic classes (propagator pairs, vertex gathers, GEMMs, epilogue) with the vertex
resident in HBM.  Algorithmic work per step:
    F = 2 * N * 8 * (4N + 4) * 4 Nq * (4N + 4)   real flops (= 16.81 TFLOP).
`value` is F / (ms per step) of the split-FP32 path when its error against the FP64
path is <= 1e-6, otherwise of the FP64 path.  The split-FP32 path is the lowest rung of the
split ladder: operands rounded once to FP32 (no hi*lo correction products), FP32 MFMA with
FP32 partial sums over 128 complex terms promoted to FP64.

Prints one JSON line.  --gpus above 1 is rejected: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K3 bubble GFLOP/s & % MFMA peak: split-FP32 vs FP64 at rel err ≤1e-6, 1 GPU"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
KERNEL_SRC = os.path.join(ROOT, "paper_2405_20996_amd", "csrc", "kqft_kernels.hip")
# HBM bytes per GEMM launch from two rocprofv3 --pmc passes over this workload (FETCH_SIZE
# x 2.000 and WRITE_SIZE x 1.000, the factors that make a 1 GiB device copy read and write
# 1 GiB), valid for the GEMM source they were taken on (first 16 hex digits of the SHA-256
# of the kernel file's GEMM section) and the batch of 67 transfer frequencies.
MEASURED_TRAFFIC = {
    "zgemm_f32_kernel": {"src": "629fd9fe3706776f", "omega_batch": 67, "n": 201, "nq": 2001,
                         "read_bytes": 67.352e9, "write_bytes": 1.446e9},
}


def kernel_src_digest() -> str:
    """Digest of the split-FP32 GEMM kernel's source (its section of the kernel file)."""
    import hashlib
    with open(KERNEL_SRC, "r", encoding="utf-8") as f:
        src = f.read()
    a = src.index("// ======================================================================== split-FP32 GEMM")
    b = src.index("// The two combinations' products of the GEMM's tile range into the classes", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def measured_traffic(kernel, n, nq, omega_batch):
    m = MEASURED_TRAFFIC.get(kernel)
    if not m or (m["n"], m["nq"], m["omega_batch"]) != (n, nq, omega_batch) or m["src"] != kernel_src_digest():
        return None
    return round(m["read_bytes"] + m["write_bytes"], 0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_flops(n, nq, n_w=None):
    n_w = n if n_w is None else n_w
    return 2.0 * n_w * 8.0 * (4 * n + 4) * 4.0 * nq * (4 * n + 4)


def seeded_vertex(K, torch, dev, n, q, P, U, noise):
    """PT2 seed (K1 of the bare bubble in each channel) plus the seeded noise on every class."""
    g = K.Grid(n)
    bare = K.Vertex(g, U)
    chans = []
    for r in range(3):
        k1 = K.bubble(r, bare, bare, P, q, class_mask=K.K1).K1
        c = K.Channel(1.0, *[torch.from_numpy(noise[r][x]).to(dev) for x in K.CLASSES])
        c.K1 = c.K1 + k1
        chans.append(c)
    return K.Vertex(g, U, chans)


def small_workload(K, torch, dev, seed_noise, with_cpu):
    """The channel-a bubble (all classes) at N = 31, Nq = 201, seeded as the headline workload:
    GPU time per call on both paths (median of 10 after 3 warm-ups), and with the oracle its
    whole-array max-norm errors and the oracle's time on all host cores and on one core."""
    import numpy as np
    n1, nq1, U, T, Dl = 31, 201, 1.0, 0.1, 1.0
    noise = seed_noise(n1, 0)
    q, P = K.Quad(nq1), K.Propagator(Dl, T)
    V = seeded_vertex(K, torch, dev, n1, q, P, U, noise)
    res = {"workload": f"channel-a bubble (K1, K2, K2', K3), N={n1}, Nq={nq1}, same seeding as the headline",
           "gflop": round(algorithmic_flops(n1, nq1) / 1e9, 3)}
    outs = {}
    for name, prec in (("fp64", K.FP64), ("split", K.SPLIT_FP32)):
        out = K.alloc_channel(n1)
        for _ in range(3):
            K.bubble(0, V, V, P, q, precision=prec, out=out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            K.bubble(0, V, V, P, q, precision=prec, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[f"gpu_ms_{name}"] = round(1e3 * float(np.median(ts)), 3)
        outs[name] = out
    if with_cpu:
        import oracle as O
        from threadpoolctl import threadpool_limits
        og, oq, op = O.Grid(n1), O.Quad(nq1), O.Prop(Dl, T)
        ov = O.seeded_vertex(og, U, op, oq, noise)
        t0 = time.perf_counter()
        ref = O.bubble(0, ov, ov, op, oq)
        res["oracle_seconds_all_cores"] = round(time.perf_counter() - t0, 3)
        res["oracle_cores"] = len(os.sched_getaffinity(0))
        with threadpool_limits(limits=1, user_api="openmp"):
            t0 = time.perf_counter()
            O.bubble(0, ov, ov, op, oq)
            res["oracle_seconds_one_core"] = round(time.perf_counter() - t0, 3)
        for name, out in outs.items():
            res[f"rel_err_vs_oracle_{name}"] = max(
                float(np.abs(getattr(out, c).cpu().numpy() - getattr(ref, c)).max() / np.abs(getattr(ref, c)).max())
                for c in K.CLASSES)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=201)
    ap.add_argument("--nq", type=int, default=2001)
    ap.add_argument("--omega-batch", type=int, default=67)
    ap.add_argument("--cpu-points", type=int, default=0, help="oracle sample size (0 = about 20 s of CPU work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["both", "split", "fp64"], default="both")
    ap.add_argument("--overlap", action="store_true",
                    help="run the gathers of the next batch concurrently with the current GEMM")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a device-to-device copy of 1 GiB three times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (the bubble shards over transfer frequencies "
              "across GPUs by design, but no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": nbytes, "copy_write_bytes": nbytes, "launches": 3}), flush=True)
        return

    from paper_2405_20996_amd import kqft as K
    from workload import seed_noise

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n, nq, U, T, Dl = args.n, args.nq, 1.0, 0.1, 1.0
    log(f"workload n={n} nq={nq}: generating seeded noise")
    t0 = time.time()
    noise = seed_noise(n, 0)
    log(f"noise ready in {time.time() - t0:.1f}s; uploading")
    g, q, P = K.Grid(n), K.Quad(nq), K.Propagator(Dl, T)
    V = seeded_vertex(K, torch, dev, n, q, P, U, noise)
    chans = V.ch
    torch.cuda.synchronize()
    log("vertex resident on the device")

    F = algorithmic_flops(n, nq)
    results = {}
    outs = {}
    precs = {"split": K.SPLIT_FP32, "fp64": K.FP64}
    order = ["split", "fp64"] if args.only == "both" else [args.only]
    for name in order:
        prec = precs[name]
        out = K.alloc_channel(n)
        for _ in range(args.warmup):
            K.bubble(0, V, V, P, q, precision=prec, omega_batch=args.omega_batch, out=out, overlap=args.overlap)
        torch.cuda.synchronize()
        K.profile(True)
        t0 = time.perf_counter()
        for i in range(args.steps):
            K.bubble(0, V, V, P, q, precision=prec, omega_batch=args.omega_batch, out=out, overlap=args.overlap)
            log(f"{name} step {i + 1}/{args.steps} enqueued")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        prof = K.profile_read()
        K.profile(False)
        gemm_ms, gemm_launches = prof["gemm"]
        gemm_ms_step = gemm_ms / args.steps
        dtype = "f32" if name == "split" else "f64"
        results[name] = {
            "ms_per_step": dt * 1e3,
            "gflops": F / dt / 1e9,
            "gemm_ms_per_step": gemm_ms_step,
            "gemm_launches_per_step": gemm_launches // args.steps,
            "gemm_avg_launch_ms": gemm_ms / max(gemm_launches, 1),
            "gemm_tflops": F / (gemm_ms_step * 1e-3) / 1e12,
            "gather_ms_per_step": prof["gather"][0] / args.steps,
            "pi_ms_per_step": prof["pi"][0] / args.steps,
            "unmix_ms_per_step": prof["reduce"][0] / args.steps,
            "dtype": dtype,
        }
        outs[name] = out
        log(f"{name}: {dt * 1e3:.1f} ms/step, {F / dt / 1e12:.2f} TFLOP/s; GEMM {gemm_ms_step:.1f} ms, "
            f"gather {prof['gather'][0] / args.steps:.1f} ms, pi {prof['pi'][0] / args.steps:.1f} ms")

    # accuracy of the split path against the FP64 path (parity-tested against the oracle)
    err = {}
    if "split" in outs and "fp64" in outs:
        for c in K.CLASSES:
            a, b = getattr(outs["split"], c), getattr(outs["fp64"], c)
            err[c] = float((a - b).abs().max() / b.abs().max())
        log(f"split vs fp64 max-norm relative errors: {err}")
    # Sigma(v) and chi(w) from the bubble's vertex: Gamma' = Gamma_0 + gamma_a' + the seed's p and t
    # channels, with gamma_a' = the bubble of each path; the SDE's own bubble in the same path,
    # its loop and the chi reduction in FP64.  Errors of the split path against the FP64 path.
    derived = {}
    sd_err = {}
    for name, out in outs.items():
        Vd = K.Vertex(g, U, [out, chans[1], chans[2]])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, chi = K.sde(Vd, P, q, q, precision=precs[name], omega_batch=args.omega_batch)
        torch.cuda.synchronize()
        derived[name] = (sig, chi, time.perf_counter() - t0)
        log(f"{name}: Sigma and chi of the updated vertex in {derived[name][2]:.2f} s")
    if "split" in derived and "fp64" in derived:
        (s32, c32, _), (s64, c64, _) = derived["split"], derived["fp64"]

        def chi_r(c):  # chi^R(w) = u^T chi^X(w) v, u on pairs {00, 11}, v on {01, 10}
            m = c[0].reshape(-1, 4, 4)
            return m[:, [0, 3]][:, :, [1, 2]].sum(dim=(1, 2))

        sd_err = {"Sigma": float((s32 - s64).abs().max() / s64.abs().max()),
                  "SigmaR": float((s32[:, 1] - s64[:, 1]).abs().max() / s64[:, 1].abs().max()),
                  "chi_pair": float((c32 - c64).abs().max() / c64.abs().max()),
                  "chiR": float((chi_r(c32) - chi_r(c64)).abs().max() / chi_r(c64).abs().max())}
        log(f"split vs fp64, Sigma and chi of the updated vertex: {sd_err}")
    split_ok = bool(err) and max(err.values()) <= 1e-6
    head = "split" if (split_ok or args.only == "split") else "fp64"
    if args.only == "fp64":
        head = "fp64"
    hr = results[head]

    # roofline of the dominant kernel (the GEMM), timed with events on the launch stream
    peak = PEAK_TFLOPS[hr["dtype"]]
    # The GEMMs multiply complex numbers with three real products (6 executed flops per complex
    # multiply-add against the 8 algorithmic ones), so the MFMA units execute 3/4 of `achieved`.
    roofline = {"bound": "mfma", "achieved": round(hr["gemm_tflops"], 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(hr["gemm_tflops"] / peak, 4),
                "traffic": measured_traffic("zgemm_f32_kernel" if head == "split" else "zgemm_f64_kernel", n, nq,
                                            args.omega_batch),
                "kernel": "zgemm_f32_kernel" if head == "split" else "zgemm_f64_kernel",
                "per_launch": {"algorithmic_flop": F / max(hr["gemm_launches_per_step"], 1),
                               "avg_ms": round(hr["gemm_avg_launch_ms"], 4)},
                "executed_flop_per_complex_mac": 6,
                "executed_frac": round(0.75 * hr["gemm_tflops"] / peak, 4),
                "frac_note": "frac counts 8 algorithmic flops per complex multiply-add; the MFMAs execute 6 "
                             "(three real products), so frac may exceed 1 while executed_frac stays below it"}

    # CPU baseline: the FP64 oracle on a bounded sample of the same outputs
    cpu = None
    oracle_err = None
    if not args.no_cpu_baseline:
        import oracle as O
        og, oq, op = O.Grid(n), O.Quad(nq), O.Prop(Dl, T)
        ov = O.seeded_vertex(og, U, op, oq, noise)
        rng = np.random.default_rng(1)
        npts = args.cpu_points
        cores = len(os.sched_getaffinity(0))
        if npts <= 0:  # size the sample to 10-30 s of CPU work
            m = 8 * cores
            probe = np.stack([np.full(m, 8), rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, n, m)], 1)
            t0 = time.perf_counter()
            O.bubble_points(0, ov, ov, op, oq, probe)
            per = (time.perf_counter() - t0) / m
            # the probe overestimates the per-block time (start-up); aim at 15-20 s measured
            npts = int(max(64, min(400000, 45.0 / max(per, 1e-7))))
        pts = np.stack([np.full(npts, 8), rng.integers(0, n, npts), rng.integers(0, n, npts),
                        rng.integers(0, n, npts)], 1)
        pts[: min(8, npts), 0] = [1, 2, 4, 8, 1, 2, 4, 8][: min(8, npts)]
        log(f"oracle sample: up to {npts} output blocks on {cores} cores, in chunks, stopping after about 40 s")
        t0 = time.perf_counter()
        chunk = max(64, npts // 20)
        refs, done = [], 0
        while done < npts:
            refs.append(O.bubble_points(0, ov, ov, op, oq, pts[done:done + chunk]))
            done = min(npts, done + chunk)
            el = time.perf_counter() - t0
            log(f"oracle sample: {done} blocks in {el:.1f} s")
            if el > 40.0:
                break
        tc = time.perf_counter() - t0
        npts = done
        pts = pts[:done]
        ref = np.concatenate(refs)
        flops_per_block = 2.0 * 8 * 16 * 4 * nq
        cpu_model = "unknown"
        try:
            with open("/proc/cpuinfo", encoding="utf-8") as f:
                for ln in f:
                    if ln.startswith("model name"):
                        cpu_model = ln.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        cpu = {"value": round(npts * flops_per_block / tc / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
               "kind": "oracle", "seconds": round(tc, 2), "cpu_model": cpu_model,
               "sample": f"{npts} random (w, v, v') output blocks (4x4 Keldysh x 2 spins) of the same "
                         f"channel-a bubble, mostly K3, at n={n}, nq={nq}"}
        # parity of both GPU paths on the sample (denominator: max-norm of the full FP64 array),
        # one indexed read per class
        oracle_err = {}
        den = outs.get("fp64", next(iter(outs.values())))
        mx = {c: float(getattr(den, c).abs().max()) for c in ("K1", "K2", "K2p", "K3")}
        for name, out in outs.items():
            worst = 0.0
            for cls, c in ((1, "K1"), (2, "K2"), (4, "K2p"), (8, "K3")):
                sel = pts[:, 0] == cls
                if not sel.any():
                    continue
                p_ = torch.as_tensor(pts[sel], device=out.K1.device, dtype=torch.long)
                if cls == 8:
                    gv = out.K3[:, p_[:, 1], p_[:, 2], p_[:, 3]]
                elif cls == 2:
                    gv = out.K2[:, p_[:, 1], p_[:, 2]]
                elif cls == 4:
                    gv = out.K2p[:, p_[:, 1], p_[:, 3]]
                else:
                    gv = out.K1[:, p_[:, 1]]
                g_ = gv.permute(1, 0, 2).cpu().numpy()
                worst = max(worst, float(np.abs(g_ - ref[sel]).max()) / mx[c])
            oracle_err[name] = worst
        log(f"sampled relative error vs oracle: {oracle_err}")

    small = small_workload(K, torch, dev, seed_noise, not args.no_cpu_baseline)
    log(f"small workload: {small}")

    line = {
        "metric": METRIC,
        "value": round(hr["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hr["dtype"],
        "data": "synthetic",
        "config": {"workload": f"channel-a K3 bubble, SIAM at particle-hole symmetry, N={n}, Nq={nq}, U=1, "
                               f"T=0.1, Delta=1, PT2 seed + 1e-3 noise (seed 0)",
                   "n": n, "nq": nq, "channel": "a", "omega_batch": args.omega_batch,
                   "algorithmic_tflop_per_step": round(F / 1e12, 4), "path": head,
                   "overlap": args.overlap},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paths": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "split_vs_fp64_rel_err": err,
        "split_vs_fp64_sigma_chi_rel_err": sd_err,
        "sigma_chi_seconds": {k: round(v[2], 3) for k, v in derived.items()},
        "sampled_rel_err_vs_oracle": oracle_err,
        "small_workload": small,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
