// kqft_api.hip -- C ABI of the MI355X Keldysh bubble library: validation, context and
// workspace management, grid/quadrature tables, and the orchestration of the kernels
// for kqft_bubble, kqft_sde, kqft_mloop_step and kqft_bubble_adjoint.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>


#include "kqft.h"
#include "kqft_launch.h"

using namespace kqft;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(KQFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct kqft_ctx {
  int device = 0;
  std::map<std::tuple<int, double, double, int>, double*> grids;
  std::map<std::tuple<int, int, double, double>, std::pair<double*, double*>> quads;
  DevBuf panels[2], pi[2], phi, chi_part, lstore[2][3], adj, tab[2][2];
  // internal streams (default priority, non-blocking): vertex gathers and GEMMs of
  // consecutive transfer-frequency batches overlap, ordered by events
  hipStream_t sg = nullptr, sm = nullptr;
  DevBuf adjw, dkf[2][3], phigrad, pq, pqsig, pqred, vtab[3], flow, flowml, ctmp, flowred, pqx, adapt, sdep, mf, mftmp,
      mfflow, mftail;
  // multiloop adjoint / tangent: recomputed insertions, cotangent accumulators and the
  // extra cotangents of the stored left insertions (two orders each, per channel)
  DevBuf mlrec[2][3], mlbar[2][3], mlext[2][3], mlscr;
  DevBuf gemmP;  // GEMM products of one batch, both spin combinations (FP64 entries)
  DevBuf chi_proj;  // susceptibility: grid projection of Pi and the own-channel part
  // autotuned transfer-frequency batch per (n, nq, precision), used when opts.omega_batch = 0
  std::map<std::tuple<int, int, int>, int> tuned_nb;
  std::vector<hipEvent_t> events;
  size_t next_event = 0;
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
};

// Optional event bracketing of one launch (kind: 0 Pi, 1 gather, 2 GEMM, 3 reductions).
struct ProfScope {
  kqft_ctx* c;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(kqft_ctx* c_, int kind_, hipStream_t s_) : c(c_), kind(kind_), s(s_) {
    if (c && c->prof && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      c->ev[kind].emplace_back(a, b);
    }
  }
};

// ------------------------------------------------------------------ host tables
// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton iteration on the
// Legendre three-term recurrence.
static void gl_nodes(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      dp = n * (z * p1 - p2) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p1 = 1.0, p2 = 0.0;
    for (int j = 1; j <= n; ++j) {
      double p3 = p2;
      p2 = p1;
      p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    dp = n * (z * p1 - p2) / (z * z - 1.0);
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

static int get_grid(kqft_ctx* ctx, const kqft_grid& g, const double** out) {
  auto key = std::make_tuple(g.n, g.L, g.a, g.map);
  auto it = ctx->grids.find(key);
  if (it != ctx->grids.end()) {
    *out = it->second;
    return KQFT_OK;
  }
  std::vector<double> v(g.n);
  const double th = aux_of(g.map, g.L / g.a);
  for (int i = 0; i < g.n; ++i) v[i] = g.a * freq_of(g.map, (-1.0 + 2.0 * i / (g.n - 1)) * th);
  // The algebraic map's inverse goes as sqrt(|v|) at zero, so a frequency sum that should
  // vanish must vanish exactly: its nodes are made exactly odd.
  if (g.map == KQFT_GRID_ALGEBRAIC)
    for (int i = 0; i < g.n / 2; ++i) v[g.n - 1 - i] = -v[i];
  double* d = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(double) * g.n));
  HIP_TRY(hipMemcpy(d, v.data(), sizeof(double) * g.n, hipMemcpyHostToDevice));
  ctx->grids[key] = d;
  *out = d;
  return KQFT_OK;
}

static int get_quad(kqft_ctx* ctx, const kqft_quad& q, const double** qv, const double** qw) {
  auto key = std::make_tuple(q.n, q.map, q.L, q.a);
  auto it = ctx->quads.find(key);
  if (it == ctx->quads.end()) {
    std::vector<double> y, gw, v(q.n), w(q.n);
    gl_nodes(q.n, y, gw);
    const double th = q.map == KQFT_QUAD_TAN_FINITE ? atan(q.L / q.a) : 0.5 * M_PI;
    for (int k = 0; k < q.n; ++k) {
      const double c = cos(y[k] * th);
      v[k] = q.a * tan(y[k] * th);
      w[k] = gw[k] * q.a * th / (c * c);
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * 2 * q.n));
    HIP_TRY(hipMemcpy(d, v.data(), sizeof(double) * q.n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d + q.n, w.data(), sizeof(double) * q.n, hipMemcpyHostToDevice));
    it = ctx->quads.emplace(key, std::make_pair(d, d + q.n)).first;
  }
  *qv = it->second.first;
  *qw = it->second.second;
  return KQFT_OK;
}

// device bytes held by the workspaces of every context of the process, and their peak
static std::atomic<size_t> g_ws_bytes{0}, g_ws_peak{0};

static void free_buf(DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    g_ws_bytes -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

static int ensure(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return KQFT_OK;
  if (b.p) (void)hipDeviceSynchronize();  // the old buffer may still be read by work of an earlier call
  free_buf(b);
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(KQFT_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  const size_t now = (g_ws_bytes += bytes);
  size_t pk = g_ws_peak.load();
  while (now > pk && !g_ws_peak.compare_exchange_weak(pk, now)) {
  }
  return KQFT_OK;
}

// Keldysh flat-index permutation between channel pair orders.  Leg slots of the
// (row first, row second, col first, col second) pair entries, legs 0..3 = 1', 2', 1, 2.
static const int kPairLegs[3][4] = {{0, 3, 2, 1}, {0, 1, 2, 3}, {1, 3, 0, 2}};
static int init_tables() {
  static bool done = false;
  if (done) return KQFT_OK;
  int perm[3][3][16];
  for (int r = 0; r < 3; ++r)
    for (int r2 = 0; r2 < 3; ++r2)
      for (int f = 0; f < 16; ++f) {
        int al[4];
        const int bits[4] = {(f >> 3) & 1, (f >> 2) & 1, (f >> 1) & 1, f & 1};
        for (int s = 0; s < 4; ++s) al[kPairLegs[r][s]] = bits[s];
        const int* p = kPairLegs[r2];
        perm[r][r2][f] = 4 * (2 * al[p[0]] + al[p[1]]) + (2 * al[p[2]] + al[p[3]]);
      }
  HIP_TRY(upload_perm(&perm[0][0][0]));
  done = true;
  return KQFT_OK;
}

// ------------------------------------------------------------------ conversions
static bool same_grid(const kqft_grid& a, const kqft_grid& b) {
  return a.n == b.n && a.L == b.L && a.a == b.a && a.map == b.map;
}

static int check_grid(const kqft_grid& g, const char* what) {
  if (g.n < 2 || !(g.L > 0) || !(g.a > 0) || !std::isfinite(g.L) || !std::isfinite(g.a))
    return fail(KQFT_ESHAPE, std::string("invalid grid: ") + what);
  // the kernels index table records (n^3 + 2n^2 + n per table) in 32 bits; a K3 class at
  // n = 600 already takes 110 GB per channel
  if (g.n > 600) return fail(KQFT_ESHAPE, std::string("grid of more than 600 points: ") + what);
  if (g.map != KQFT_GRID_TAN && g.map != KQFT_GRID_ALGEBRAIC)
    return fail(KQFT_EINVAL, std::string("unknown grid map: ") + what);
  return KQFT_OK;
}

static DVert to_dvert(const kqft_vertex& v) {
  DVert d;
  d.r0 = v.r0;
  d.g = make_dgrid(v.grid.n, v.grid.L, v.grid.a, v.grid.map);
  for (int r = 0; r < 3; ++r) {
    d.ch[r].coef = v.ch[r].coef;
    d.ch[r].K[0] = (const double2*)v.ch[r].K1;
    d.ch[r].K[1] = (const double2*)v.ch[r].K2;
    d.ch[r].K[2] = (const double2*)v.ch[r].K2p;
    d.ch[r].K[3] = (const double2*)v.ch[r].K3;
    if (d.ch[r].coef == 0.0)
      for (int c = 0; c < 4; ++c) d.ch[r].K[c] = nullptr;
  }
  return d;
}

static int to_dprop(const kqft_propagator& p, DProp& d) {
  if (!(p.T > 0) || !(p.Delta > 0)) return fail(KQFT_EINVAL, "propagator needs T > 0 and Delta > 0");
  if (p.reg < KQFT_REG_DELTA || p.reg > KQFT_REG_NU) return fail(KQFT_EINVAL, "unknown regulator");
  if ((p.reg == KQFT_REG_U || p.reg == KQFT_REG_NU) && !(p.lam > 0))
    return fail(KQFT_EINVAL, "the interaction and frequency regulators need lam > 0");
  if ((p.dSigR == nullptr) != (p.dSigK == nullptr))
    return fail(KQFT_EINVAL, "Sigma_dot needs both dSigR and dSigK");
  d.Delta = p.Delta;
  d.T = p.T;
  d.eps = p.eps;
  d.SigR = (const double2*)p.SigR;
  d.SigK = (const double2*)p.SigK;
  d.reg = p.reg;
  d.lam = p.lam;
  d.dSigR = (const double2*)p.dSigR;
  d.dSigK = (const double2*)p.dSigK;
  if (!std::isfinite(p.deps)) return fail(KQFT_EINVAL, "deps must be finite");
  d.deps = p.deps;
  if (p.SigR || p.SigK || p.dSigR) {
    int rc = check_grid(p.sgrid, "propagator self-energy grid");
    if (rc) return rc;
    d.sg = make_dgrid(p.sgrid.n, p.sgrid.L, p.sgrid.a, p.sgrid.map);
  } else {
    d.sg = make_dgrid(2, 1.0, 1.0, 0);
  }
  return KQFT_OK;
}

// Spin combinations per channel (rows: combination 0, 1; columns: X, Y) that turn the
// spin sums of the three bubbles into two independent products P0, P1, and the inverse
// map back to (X, Y) including the channel prefactor (+1, 1/2, -1):
//   a: X Pi X, (X+2Y) Pi (X+2Y)  ->  X = P0,            Y = (P1 - P0)/2
//   p: (X+Y) Pi (X+Y), (X-Y) Pi (X-Y) -> X = (P0+P1)/4, Y = (P0-P1)/4
//   t: Y Pi Y, (2X+Y) Pi (2X+Y)  ->  X = (P0 - P1)/2,   Y = -P0
static const double kMix[3][4] = {{1, 0, 1, 2}, {1, 1, 1, -1}, {0, 1, 2, 1}};
static const double kUnmix[3][4] = {{1, 0, -0.5, 0.5}, {0.25, 0.25, 0.25, -0.25}, {0.5, -0.5, -1, 0}};

// ------------------------------------------------------------------ bubble core
struct BubbleOut {
  double2* K1;
  double2* K2;
  double2* K2p;
  double2* K3;
};

static size_t panel_bytes_per_w(int n, int nq, int precision) {
  const size_t M = 4 * (size_t)(n + 1);
  const size_t nq_pad = (size_t)((nq + 7) / 8) * 8;
  const size_t Kp = 4 * nq_pad;
  const size_t elt = precision == KQFT_FP64 ? 16 : 8;
  return 4 * M * Kp * elt;  // two spin combinations x (A + B^T)
}

static int next_event(kqft_ctx* ctx, hipEvent_t* ev) {
  if (ctx->next_event == ctx->events.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->events.push_back(e);
  }
  *ev = ctx->events[ctx->next_event++];
  return KQFT_OK;
}

static int ensure_streams(kqft_ctx* ctx) {
  if (!ctx->sg) HIP_TRY(hipStreamCreateWithFlags(&ctx->sg, hipStreamNonBlocking));
  if (!ctx->sm) HIP_TRY(hipStreamCreateWithFlags(&ctx->sm, hipStreamNonBlocking));
  return KQFT_OK;
}

static bool same_channel(const kqft_chvert& a, const kqft_chvert& b) {
  return a.coef != 0.0 && b.coef != 0.0 && a.K1 == b.K1 && a.K2 == b.K2 && a.K2p == b.K2p && a.K3 == b.K3;
}

// Fused K1+K2+K2'+K3 tables of the channels other than r that carry a K3 class; the
// right side reuses the left side's table when both point at the same arrays.
// Tables of the two other channels (r + 1, r + 2) in channel r's Keldysh order, with r's spin
// combinations and the channel coefficients applied, for each side of the bubble.  The right
// side shares a left table when its channel is the same (arrays and coefficient).
struct SideTables {
  const void* T[2] = {nullptr, nullptr};
};

// Table of channel r2 (classes c) in channel r's order into `out`.
static TableArgs table_args(int r, int r2, const kqft_chvert& c, int n, void* out) {
  TableArgs ta;
  memset(&ta, 0, sizeof ta);
  ta.n = n;
  ta.r = r;
  ta.r2 = r2;
  ta.coef = c.coef;
  for (int u = 0; u < 4; ++u) ta.mix[u] = kMix[r][u];
  ta.K[0] = (const double2*)c.K1;
  ta.K[1] = (const double2*)c.K2;
  ta.K[2] = (const double2*)c.K2p;
  ta.K[3] = (const double2*)c.K3;
  ta.out = out;
  return ta;
}
static bool table_active(const kqft_chvert& c) { return c.coef != 0.0 && (c.K1 || c.K2 || c.K2p || c.K3); }

static int build_tables(kqft_ctx* ctx, int r, const kqft_vertex& L, const kqft_vertex& R, bool f32,
                        SideTables& tl, SideTables& tr, hipStream_t s) {
  const size_t n = L.grid.n;
  const size_t bytes = (n * n * n + 2 * n * n + n) * 32 * (f32 ? sizeof(float2) : sizeof(double2));
  const kqft_vertex* side[2] = {&L, &R};
  SideTables* out[2] = {&tl, &tr};
  for (int sd = 0; sd < 2; ++sd)
    for (int d = 0; d < 2; ++d) {
      const int r2 = (r + 1 + d) % 3;
      out[sd]->T[d] = nullptr;
      const kqft_chvert& c = side[sd]->ch[r2];
      if (!table_active(c)) continue;
      if (sd == 1 && same_channel(L.ch[r2], c) && tl.T[d]) {
        tr.T[d] = tl.T[d];
        continue;
      }
      int rc = ensure(ctx->tab[sd][d], bytes);
      if (rc) return rc;
      {
        ProfScope ps(ctx, 1, s);
        launch_table(table_args(r, r2, c, (int)n, ctx->tab[sd][d].p), f32, s);
      }
      out[sd]->T[d] = ctx->tab[sd][d].p;
    }
  return KQFT_OK;
}

static GatherArgs make_gather(int r, int nb, int iw0, int nq, int nq_pad, int lo, int cnt, long Kp,
                              const kqft_vertex& V, const SideTables& T, const double* nodes, const double* qv,
                              const double2* pi, void* P0, void* P1) {
  GatherArgs g;
  memset(&g, 0, sizeof g);
  g.r = r;
  g.nb = nb;
  g.iw0 = iw0;
  g.nq = nq;
  g.nq_pad = nq_pad;
  g.lo = lo;
  g.cnt = cnt;
  g.Kp = Kp;
  g.g = make_dgrid(V.grid.n, V.grid.L, V.grid.a, V.grid.map);
  g.r0 = V.r0;
  const kqft_chvert& c = V.ch[r];
  g.coef = c.coef;
  if (c.coef != 0.0) {
    g.K[0] = (const double2*)c.K1;
    g.K[1] = (const double2*)c.K2;
    g.K[2] = (const double2*)c.K2p;
    g.K[3] = (const double2*)c.K3;
  }
  g.T[0] = T.T[0];
  g.T[1] = T.T[1];
  for (int u = 0; u < 4; ++u) g.mix[u] = kMix[r][u];
  g.nodes = nodes;
  g.qv = qv;
  g.pi = pi;
  g.P0 = P0;
  g.P1 = P1;
  return g;
}

static int bubble_core(kqft_ctx* ctx, int r, const kqft_vertex& L, const kqft_vertex& R, const kqft_propagator& G,
                       int kind, const kqft_quad& q, const kqft_opts& o, const BubbleOut& out, hipStream_t s,
                       double scale = 1.0) {
  int rc;
  const int n = L.grid.n;
  if ((rc = init_tables())) return rc;
  if ((rc = ensure_streams(ctx))) return rc;
  const double *nodes, *qv, *qw;
  if ((rc = get_grid(ctx, L.grid, &nodes))) return rc;
  if ((rc = get_quad(ctx, q, &qv, &qw))) return rc;
  DProp P;
  if ((rc = to_dprop(G, P))) return rc;
  const int nq = q.n;
  const int nq_pad = ((nq + 7) / 8) * 8;  // multiple of 8 so 4*nq_pad divides by the K block
  const long Kp = 4L * nq_pad;
  const int M = 4 * (n + 1);
  const bool f32 = o.precision == KQFT_SPLIT_FP32;
  const size_t elt = f32 ? 8 : 16;
  // output class ranges -> panel row / column ranges
  const int mask = o.class_mask & KQFT_KALL;
  const bool main_rows = mask & (KQFT_K3 | KQFT_K2), border_row = mask & (KQFT_K2P | KQFT_K1);
  const bool main_cols = mask & (KQFT_K3 | KQFT_K2P), border_col = mask & (KQFT_K2 | KQFT_K1);
  const int ilo = main_rows ? 0 : n, ihi = border_row ? n : n - 1;
  const int jlo = main_cols ? 0 : n, jhi = border_col ? n : n - 1;
  // batch of transfer frequencies (two panel buffers in flight)
  const size_t per_w = panel_bytes_per_w(n, nq, o.precision);
  int nb = o.omega_batch > 0 ? o.omega_batch : (int)std::max<size_t>(1, ((size_t)4 << 30) / per_w);
  if (o.omega_batch <= 0) {
    auto it = ctx->tuned_nb.find(std::make_tuple(n, nq, o.precision));
    if (it != ctx->tuned_nb.end()) nb = it->second;
  }
  nb = std::min(nb, n);
  {
    // A schedule of several transfer-frequency batches (gathers of the next batch ordered
    // after the GEMM of the previous one across the two internal streams) crashed the
    // runtime's graph instantiation when captured; a one-batch schedule captures and replays
    // bit for bit.  Under capture only the latter is accepted.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone && nb < n)
      return fail(KQFT_EINVAL, "under stream capture a bubble must run in one transfer-frequency batch "
                               "(omega_batch >= n)");
  }
  const size_t pbytes = (size_t)M * Kp * elt;  // one panel of one transfer frequency
  for (int x = 0; x < 2; ++x) {
    if ((rc = ensure(ctx->panels[x], 4 * pbytes * nb))) return rc;
    if ((rc = ensure(ctx->pi[x], (size_t)nb * nq * 256))) return rc;
  }
  // the two combinations' products of a batch (GEMM and unmix run in order on sm)
  const size_t prod = (size_t)nb * M * M * sizeof(double2);
  if (main_rows && (rc = ensure(ctx->gemmP, 2 * prod))) return rc;
  SideTables TL, TR;
  ctx->next_event = 0;
  hipEvent_t start;
  if ((rc = next_event(ctx, &start))) return rc;
  HIP_TRY(hipEventRecord(start, s));
  HIP_TRY(hipStreamWaitEvent(ctx->sg, start, 0));
  HIP_TRY(hipStreamWaitEvent(ctx->sm, start, 0));
  if (main_rows || main_cols)
    if ((rc = build_tables(ctx, r, L, R, f32, TL, TR, ctx->sg))) return rc;
  std::vector<hipEvent_t> gemm_done;
  int batch = 0;
  for (int iw0 = 0; iw0 < n; iw0 += nb, ++batch) {
    const int cnt = std::min(nb, n - iw0);
    const int x = batch & 1;
    char* base = (char*)ctx->panels[x].p;
    void* A0 = base;
    void* A1 = base + pbytes * nb;
    void* B0 = base + 2 * pbytes * nb;
    void* B1 = base + 3 * pbytes * nb;
    double2* pib = (double2*)ctx->pi[x].p;
    if (!o.overlap && batch >= 1) HIP_TRY(hipStreamWaitEvent(ctx->sg, gemm_done[batch - 1], 0));
    if (batch >= 2) HIP_TRY(hipStreamWaitEvent(ctx->sg, gemm_done[batch - 2], 0));
    PiArgs pa{r, kind, cnt, nq, iw0, P, nodes, qv, qw, pib};
    {
      ProfScope ps(ctx, 0, ctx->sg);
      launch_pi(pa, ctx->sg);
    }
    GatherArgs ga = make_gather(r, cnt, iw0, nq, nq_pad, ilo, ihi - ilo + 1, Kp, L, TL, nodes, qv, pib, A0, A1);
    {
      ProfScope ps(ctx, 1, ctx->sg);
      launch_gather(ga, true, f32, ctx->sg);
    }
    GatherArgs gb = make_gather(r, cnt, iw0, nq, nq_pad, jlo, jhi - jlo + 1, Kp, R, TR, nodes, qv, nullptr, B0, B1);
    {
      ProfScope ps(ctx, 1, ctx->sg);
      launch_gather(gb, false, f32, ctx->sg);
    }
    hipEvent_t gdone, mdone;
    if ((rc = next_event(ctx, &gdone)) || (rc = next_event(ctx, &mdone))) return rc;
    HIP_TRY(hipEventRecord(gdone, ctx->sg));
    HIP_TRY(hipStreamWaitEvent(ctx->sm, gdone, 0));
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.A[0] = A0;
    g.A[1] = A1;
    g.B[0] = B0;
    g.B[1] = B1;
    g.strideA = g.strideB = (long)M * Kp;
    g.M = M;
    g.Kp = (int)Kp;
    g.tm0 = (4 * ilo) / 64;
    g.tms = (4 * (ihi + 1) + 63) / 64 - g.tm0;
    g.tn0 = (4 * jlo) / 64;
    g.tns = (4 * (jhi + 1) + 63) / 64 - g.tn0;
    g.nb = cnt;
    g.r = r;
    g.n = n;
    g.iw0 = iw0;
    g.beta = o.beta;
    g.cmask = mask;
    for (int u = 0; u < 4; ++u) g.unmix[u] = scale * kUnmix[r][u];  // output scale folded in
    g.K1 = out.K1;
    g.K2 = out.K2;
    g.K2p = out.K2p;
    g.K3 = out.K3;
    if (main_rows) {
      g.P[0] = (double2*)ctx->gemmP.p;
      g.P[1] = (double2*)((char*)ctx->gemmP.p + prod);
    }
    if (!main_rows) {  // only the border row block: a streaming row product, no GEMM tile
      ProfScope ps(ctx, 2, ctx->sm);
      launch_rowpanel(g, o.precision, ctx->sm);
    } else {
      {
        ProfScope ps(ctx, 2, ctx->sm);
        launch_gemm(g, o.precision, ctx->sm);
      }
      {
        ProfScope ps(ctx, 3, ctx->sm);
        launch_unmix(g, ctx->sm);
      }
    }
    HIP_TRY(hipEventRecord(mdone, ctx->sm));
    gemm_done.push_back(mdone);
  }
  // the caller's stream resumes after the last GEMM (which followed every gather)
  HIP_TRY(hipStreamWaitEvent(s, gemm_done.back(), 0));
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

static int check_vertex(const kqft_vertex* v, const char* what) {
  if (!v) return fail(KQFT_EINVAL, std::string(what) + " is NULL");
  return check_grid(v->grid, what);
}

static int check_common(kqft_ctx* ctx, const kqft_propagator* G, const kqft_quad* q, const kqft_opts* o) {
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!G || !q || !o) return fail(KQFT_EINVAL, "propagator, quadrature and options must be given");
  if (q->n < 1 || (q->map != KQFT_QUAD_TAN_FINITE && q->map != KQFT_QUAD_TAN_INFINITE) ||
      (q->map == KQFT_QUAD_TAN_FINITE && !(q->L > 0)) || !(q->a > 0))
    return fail(KQFT_ESHAPE, "invalid quadrature");
  if (o->precision != KQFT_FP64 && o->precision != KQFT_SPLIT_FP32) return fail(KQFT_EINVAL, "unknown precision");
  if (o->beta != 0 && o->beta != 1) return fail(KQFT_EINVAL, "beta must be 0 or 1");
  if (o->omega_batch < 0) return fail(KQFT_EINVAL, "omega_batch must be >= 0");
  if (o->overlap != 0 && o->overlap != 1) return fail(KQFT_EINVAL, "overlap must be 0 or 1");
  return KQFT_OK;
}

// ------------------------------------------------------------------ adjoint core

// Reverse pass of one bubble: FP64, or with the two transposed products per transfer frequency
// on FP32 MFMA (precision KQFT_SPLIT_FP32).  dr0_left / dr0_right / dDelta: device doubles that
// receive the accumulated cotangents (dr0_left may equal dr0_right).
static int adjoint_core(kqft_ctx* ctx, int r, const kqft_vertex& L, const kqft_vertex& R, const kqft_propagator& G,
                        int kind, const kqft_quad& q, const kqft_chout& dout, const kqft_chout* dleft,
                        const kqft_chout* dright, double* dr0_left, double* dr0_right, double* dDelta,
                        hipStream_t s, int precision = KQFT_FP64) {
  int rc;
  const int n = L.grid.n;
  if ((rc = init_tables())) return rc;
  const double *nodes, *qv, *qw;
  if ((rc = get_grid(ctx, L.grid, &nodes))) return rc;
  if ((rc = get_quad(ctx, q, &qv, &qw))) return rc;
  DProp P;
  if ((rc = to_dprop(G, P))) return rc;
  const int nq = q.n;
  const int nq_pad = ((nq + 7) / 8) * 8;
  const long Kp = 4L * nq_pad;
  const long M = 4L * (n + 1);
  // per transfer frequency: raw L (2), A (2), B (2), conj dA (2), conj dB (2), conj dP (2), Pi
  const size_t pan = (size_t)M * Kp * 16, dpan = (size_t)M * M * 16, pib = (size_t)nq * 256;
  const size_t per_w = 10 * pan + 2 * dpan + pib;
  int nb = (int)std::max<size_t>(1, ((size_t)3 << 30) / per_w);
  nb = std::min(nb, n);
  if ((rc = ensure(ctx->adjw, per_w * nb))) return rc;
  char* w = (char*)ctx->adjw.p;
  double2* Lr[2] = {(double2*)w, (double2*)(w + pan * nb)};
  double2* Ap[2] = {(double2*)(w + 2 * pan * nb), (double2*)(w + 3 * pan * nb)};
  double2* Bp[2] = {(double2*)(w + 4 * pan * nb), (double2*)(w + 5 * pan * nb)};
  double2* GA[2] = {(double2*)(w + 6 * pan * nb), (double2*)(w + 7 * pan * nb)};
  double2* GB[2] = {(double2*)(w + 8 * pan * nb), (double2*)(w + 9 * pan * nb)};
  double2* Dp[2] = {(double2*)(w + 10 * pan * nb), (double2*)(w + 10 * pan * nb + dpan * nb)};
  double2* pi = (double2*)(w + 10 * pan * nb + 2 * dpan * nb);
  DVert VL = to_dvert(L), VR = to_dvert(R);
  SideTables TL, TR;
  if ((rc = build_tables(ctx, r, L, R, false, TL, TR, s))) return rc;
  // fused cotangent tables of the other channels (zeroed), un-fused into the classes at the end
  const kqft_vertex* side[2] = {&L, &R};
  const kqft_chout* dside[2] = {dleft, dright};
  AdjScatterArgs sa[2];
  const size_t fbytes = (size_t)2 * n * n * n * 16 * 16;
  for (int sd = 0; sd < 2; ++sd) {
    memset(&sa[sd], 0, sizeof sa[sd]);
    for (int r2 = 0; r2 < 3; ++r2) {
      const kqft_chout& d = dside[sd][r2];
      const bool active = side[sd]->ch[r2].coef != 0.0;
      sa[sd].dK[r2][0] = active ? (double2*)d.K1 : nullptr;
      sa[sd].dK[r2][1] = active ? (double2*)d.K2 : nullptr;
      sa[sd].dK[r2][2] = active ? (double2*)d.K2p : nullptr;
      sa[sd].dK[r2][3] = active ? (double2*)d.K3 : nullptr;
      sa[sd].dKf[r2] = nullptr;
      if (r2 != r && active && d.K3) {
        if ((rc = ensure(ctx->dkf[sd][r2], fbytes))) return rc;
        HIP_TRY(hipMemsetAsync(ctx->dkf[sd][r2].p, 0, fbytes, s));
        sa[sd].dKf[r2] = (double2*)ctx->dkf[sd][r2].p;
      }
    }
  }
  for (int iw0 = 0; iw0 < n; iw0 += nb) {
    const int cnt = std::min(nb, n - iw0);
    PiArgs pa{r, kind, cnt, nq, iw0, P, nodes, qv, qw, pi};
    launch_pi(pa, s);
    GatherArgs ga = make_gather(r, cnt, iw0, nq, nq_pad, 0, n + 1, Kp, L, TL, nodes, qv, nullptr, Lr[0], Lr[1]);
    launch_gather(ga, true, false, s);
    ApplyPiArgs ap{n, cnt, nq, nq_pad, Kp, pi, Lr[0], Lr[1], Ap[0], Ap[1]};
    launch_apply_pi(ap, s);
    GatherArgs gb = make_gather(r, cnt, iw0, nq, nq_pad, 0, n + 1, Kp, R, TR, nodes, qv, nullptr, Bp[0], Bp[1]);
    launch_gather(gb, false, false, s);
    DPanelArgs dp{n, cnt, iw0, {kUnmix[r][0], kUnmix[r][1], kUnmix[r][2], kUnmix[r][3]},
                  (const double2*)dout.K1, (const double2*)dout.K2, (const double2*)dout.K2p,
                  (const double2*)dout.K3, Dp[0], Dp[1]};
    launch_dpanel(dp, s);
    for (int c = 0; c < 2; ++c) {
      // conj(dA) = conj(dP) . B^T-panel and conj(dB) (as a B^T panel) = conj(dP)^T . A, per
      // transfer frequency, on the project's FP64 MFMA GEMM (row-major operands)
      ZgemmArgs za;
      memset(&za, 0, sizeof za);
      za.M = (int)M;
      za.N = (int)Kp;
      za.K = (int)M;
      za.batch = cnt;
      za.A = Dp[c];
      za.lda = M;
      za.strideA = M * M;
      za.ldb = za.ldc = Kp;
      za.strideB = za.strideC = M * Kp;
      ZgemmArgs zb = za;
      za.B = Bp[c];
      za.C = GA[c];
      za.TA = 0;
      zb.B = Ap[c];
      zb.C = GB[c];
      zb.TA = 1;
      {
        ProfScope ps(ctx, 2, s);
        if (precision == KQFT_SPLIT_FP32) {
          launch_zgemm_nn_f32(za, s);
          launch_zgemm_nn_f32(zb, s);
        } else {
          launch_zgemm_nn(za, s);
          launch_zgemm_nn(zb, s);
        }
      }
    }
    AdjScatterArgs al = sa[0];
    al.r = r;
    al.nb = cnt;
    al.iw0 = iw0;
    al.nq = nq;
    al.Kp = Kp;
    al.V = VL;
    al.nodes = nodes;
    al.qv = qv;
    al.pi = pi;
    al.G0 = GA[0];
    al.G1 = GA[1];
    for (int x = 0; x < 4; ++x) al.mix[x] = kMix[r][x];
    al.dr0 = dr0_left;
    launch_adj_left(al, s);
    AdjScatterArgs ar = sa[1];
    ar.r = r;
    ar.nb = cnt;
    ar.iw0 = iw0;
    ar.nq = nq;
    ar.Kp = Kp;
    ar.V = VR;
    ar.nodes = nodes;
    ar.qv = qv;
    ar.pi = nullptr;
    ar.G0 = GB[0];
    ar.G1 = GB[1];
    for (int x = 0; x < 4; ++x) ar.mix[x] = kMix[r][x];
    ar.dr0 = dr0_right;
    launch_adj_right(ar, s);
    DPiArgs di{r, kind, cnt, nq, iw0, n, Kp, P, nodes, qv, qw, Lr[0], Lr[1], GA[0], GA[1], dDelta};
    launch_dpi(di, s);
  }
  for (int sd = 0; sd < 2; ++sd)
    for (int r2 = 0; r2 < 3; ++r2)
      if (sa[sd].dKf[r2]) {
        UnfuseArgs ua{n, sa[sd].dKf[r2], sa[sd].dK[r2][0], sa[sd].dK[r2][1], sa[sd].dK[r2][2], nullptr};
        launch_unfuse(ua, s);
        // the K3 class takes the table itself
        UnfuseArgs u3{n, sa[sd].dKf[r2], nullptr, nullptr, nullptr, sa[sd].dK[r2][3]};
        launch_unfuse(u3, s);
      }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

// ------------------------------------------------------------------ C ABI
// Susceptibility of channel r of the vertex `gamma` into chi [2][n][16] (arguments checked).
// Device buffers of one susceptibility evaluation: grid nodes, quadrature nodes and weights,
// the other channels' target-order tables (nullptr = inactive), Pi and the block partials of
// nb transfer frequencies.
struct ChiBufs {
  const double* nodes;
  const double* qv;
  const double* qw;
  const void* T[2];
  double2* pi;
  double2* partial;
  double2* pt;   // grid projection of Pi, [nb][n + 1][16] (nullptr: own channel in the pair loop)
  double2* own;  // [nb][2][16]
  int nb;
  int f32;  // tables in FP32
};
// bytes per transfer frequency of the grid projection (Pt and the own part)
static size_t chi_proj_bytes(int n) { return ((size_t)(n + 1) * 16 + 32) * sizeof(double2); }

// chi_r of `gamma` into chi [2][n][16] in batches of b.nb transfer frequencies.  prof: the
// context whose profiling flag brackets the launches (nullptr: none).
static void chi_run(kqft_ctx* prof, int r, const kqft_vertex& gamma, const DProp& P, int nq, const ChiBufs& b,
                    double* chi, hipStream_t s) {
  const int n = gamma.grid.n;
  for (int iw0 = 0; iw0 < n; iw0 += b.nb) {
    const int cnt = std::min(b.nb, n - iw0);
    PiArgs pa{r, KQFT_PI_GG, cnt, nq, iw0, P, b.nodes, b.qv, b.qw, b.pi};
    {
      ProfScope ps(prof, 0, s);
      launch_pi(pa, s);
    }
    ChiArgs ca;
    memset(&ca, 0, sizeof ca);
    ca.r = r;
    ca.nq = nq;
    ca.nb = cnt;
    ca.iw0 = iw0;
    ca.g = make_dgrid(n, gamma.grid.L, gamma.grid.a, gamma.grid.map);
    ca.r0 = gamma.r0;
    const kqft_chvert& own = gamma.ch[r];
    ca.coef = own.coef;
    if (own.coef != 0.0) {
      ca.K[0] = (const double2*)own.K1;
      ca.K[1] = (const double2*)own.K2;
      ca.K[2] = (const double2*)own.K2p;
      ca.K[3] = (const double2*)own.K3;
    }
    ca.T[0] = b.T[0];
    ca.T[1] = b.T[1];
    for (int u = 0; u < 4; ++u) ca.mix[u] = kMix[r][u];
    ca.nodes = b.nodes;
    ca.qv = b.qv;
    ca.pi = b.pi;
    ca.partial = b.partial;
    ca.out = (double2*)chi;
    ca.f32 = b.f32;
    if (b.pt) {
      ca.pt = b.pt;
      ca.own = b.own;
    }
    {
      ProfScope ps(prof, 3, s);
      launch_chi(ca, s);
    }
  }
}

static int chi_core(kqft_ctx* ctx, int r, const kqft_vertex& gamma, const DProp& P, const double* nodes,
                    const kqft_quad& q_bubble, double* chi, hipStream_t s, bool f32 = false) {
  int rc;
  const int n = gamma.grid.n;
  ChiBufs b;
  memset(&b, 0, sizeof b);
  b.nodes = nodes;
  b.f32 = f32;
  if ((rc = get_quad(ctx, q_bubble, &b.qv, &b.qw))) return rc;
  const int nq = q_bubble.n;
  const int nblk = chi_blocks(nq);
  b.nb = std::max(1, std::min(n, (int)((256L << 20) / ((long)nq * 256))));
  if ((rc = ensure(ctx->pi[0], (size_t)b.nb * nq * 256))) return rc;
  if ((rc = ensure(ctx->chi_part, (size_t)b.nb * nblk * 32 * 16))) return rc;
  b.pi = (double2*)ctx->pi[0].p;
  b.partial = (double2*)ctx->chi_part.p;
  if (n <= kChiProjMaxN) {
    if ((rc = ensure(ctx->chi_proj, (size_t)b.nb * chi_proj_bytes(n)))) return rc;
    b.pt = (double2*)ctx->chi_proj.p;
    b.own = b.pt + (size_t)b.nb * (n + 1) * 16;
  }
  // the two other channels in channel r's Keldysh order with its spin combinations
  SideTables tabs, unused;
  if ((rc = build_tables(ctx, r, gamma, gamma, f32, tabs, unused, s))) return rc;
  b.T[0] = tabs.T[0];
  b.T[1] = tabs.T[1];
  chi_run(ctx, r, gamma, P, nq, b, chi, s);
  return KQFT_OK;
}

// Sigma (and chi when given) of the vertex `gamma` (the body of kqft_sde; arguments checked).
static int sde_core(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q_bubble,
                    const kqft_quad* q_loop, const kqft_opts* opts, double* sigma, double* chi, hipStream_t s) {
  int rc;
  const int n = gamma->grid.n;
  // Phi = B_a(Gamma_0, Gamma): classes K1 and K2' only
  const size_t k1b = (size_t)2 * n * 16 * 16, k2b = (size_t)2 * n * n * 16 * 16;
  if ((rc = ensure(ctx->phi, k1b + k2b))) return rc;
  double2* phiK1 = (double2*)ctx->phi.p;
  double2* phiK2p = (double2*)((char*)ctx->phi.p + k1b);
  kqft_vertex bare;
  memset(&bare, 0, sizeof bare);
  bare.r0 = gamma->r0;
  bare.grid = gamma->grid;
  kqft_opts o = *opts;
  o.class_mask = KQFT_K1 | KQFT_K2P;
  o.beta = 0;
  BubbleOut po{phiK1, nullptr, phiK2p, nullptr};
  if ((rc = bubble_core(ctx, KQFT_CH_A, bare, *gamma, *G, KQFT_PI_GG, *q_bubble, o, po, s))) return rc;
  const double *nodes, *qv, *qw;
  if ((rc = get_grid(ctx, gamma->grid, &nodes))) return rc;
  if ((rc = get_quad(ctx, *q_loop, &qv, &qw))) return rc;
  DProp P;
  if ((rc = to_dprop(*G, P))) return rc;
  LoopArgs la{make_dgrid(n, gamma->grid.L, gamma->grid.a, gamma->grid.map), P, 0, q_loop->n, nodes, qv, qw, phiK1, phiK2p,
              (double2*)sigma};
  {
    ProfScope ps(ctx, 3, s);
    launch_loop(la, s);
  }
  if (chi && (rc = chi_core(ctx, KQFT_CH_A, *gamma, P, nodes, *q_bubble, chi, s, opts->precision == KQFT_SPLIT_FP32)))
    return rc;
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

// ------------------------------------------------------------------ parquet
// Right-hand sides of the parquet equations for the state `V` (Sec. parquet solver): the
// symmetrized Bethe-Salpeter equations gamma_r' = 1/2 [B_r(I_r, Gamma) + B_r(Gamma, I_r)],
// I_r = Gamma without channel r, and Sigma' from the Schwinger-Dyson equation.
static int vloop_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, int kind, const kqft_quad& q,
                      double* out, hipStream_t s);
static void lincomb_n(double2* out, const double2* x, int nt, const double2* const* k, const double* c, size_t count,
                      hipStream_t s);

// Sigma as the mean of the three forms of the SDE (its two inner lines read as an a, a p or a
// t bubble).  The t-form equals the a-form for every crossing-symmetric vertex (the crossing
// 1 <-> 2 maps the one closure onto the other in the discrete scheme), which the states of the
// parquet solver are; so Sigma = (2 Sigma_a + Sigma_p) / 3 with
// Sigma_p = -L(B_p(Gamma_0, Gamma), G), B_p carrying its prefactor 1/2.
static int sde_mean_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, const kqft_quad& qb,
                         const kqft_quad& ql, const kqft_opts& opts, double* sigma, hipStream_t s) {
  int rc;
  if ((rc = sde_core(ctx, &V, &G, &qb, &ql, &opts, sigma, nullptr, s))) return rc;
  const int n = V.grid.n;
  const size_t k1b = (size_t)2 * n * 16 * 16;
  double2* phiK1 = (double2*)ctx->phi.p;  // sized by sde_core for K1 and K2'
  double2* phiK2p = (double2*)((char*)ctx->phi.p + k1b);
  kqft_vertex bare;
  memset(&bare, 0, sizeof bare);
  bare.r0 = V.r0;
  bare.grid = V.grid;
  kqft_opts o = opts;
  o.class_mask = KQFT_K1 | KQFT_K2P;
  o.beta = 0;
  BubbleOut po{phiK1, nullptr, phiK2p, nullptr};
  if ((rc = bubble_core(ctx, KQFT_CH_P, bare, V, G, KQFT_PI_GG, qb, o, po, s))) return rc;
  kqft_vertex pv;
  memset(&pv, 0, sizeof pv);
  pv.grid = V.grid;
  pv.ch[KQFT_CH_P] = kqft_chvert{1.0, (const double*)phiK1, nullptr, (const double*)phiK2p, nullptr};
  if ((rc = ensure(ctx->sdep, (size_t)n * 4 * sizeof(double2)))) return rc;
  if ((rc = vloop_core(ctx, pv, G, KQFT_LINE_G, ql, (double*)ctx->sdep.p, s))) return rc;
  const double2* k[2] = {(const double2*)sigma, (const double2*)ctx->sdep.p};
  const double c[2] = {2.0 / 3.0, -1.0 / 3.0};
  lincomb_n((double2*)sigma, nullptr, 2, k, c, (size_t)n * 4, s);
  return KQFT_OK;
}

static int parquet_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, const kqft_quad& qb,
                        const kqft_quad& ql, const kqft_opts& opts, const BubbleOut out[3], double* sigma_out,
                        hipStream_t s, int sde_forms = 1) {
  int rc;
  kqft_opts o = opts;
  o.class_mask = KQFT_KALL;
  for (int r = 0; r < 3; ++r) {
    kqft_vertex I = V;
    I.ch[r] = kqft_chvert{0.0, nullptr, nullptr, nullptr, nullptr};
    o.beta = 0;
    if ((rc = bubble_core(ctx, r, I, V, G, KQFT_PI_GG, qb, o, out[r], s, 0.5))) return rc;
    o.beta = 1;
    if ((rc = bubble_core(ctx, r, V, I, G, KQFT_PI_GG, qb, o, out[r], s, 0.5))) return rc;
  }
  if (sde_forms == 3) return sde_mean_core(ctx, V, G, qb, ql, opts, sigma_out, s);
  return sde_core(ctx, &V, &G, &qb, &ql, &opts, sigma_out, nullptr, s);
}

// max over the arrays of max|f - x| / max|f| (each array reduced on the device, the last
// step on the host after a stream synchronisation)
static int rel_change(kqft_ctx* ctx, const std::vector<std::pair<const double2*, const double2*>>& xf,
                      const std::vector<size_t>& counts, hipStream_t s, double* out) {
  const int nblk = 256;
  int rc;
  if ((rc = ensure(ctx->pqred, xf.size() * nblk * 2 * sizeof(double)))) return rc;
  double* part = (double*)ctx->pqred.p;
  for (size_t a = 0; a < xf.size(); ++a) launch_maxdiff(xf[a].first, xf[a].second, counts[a], part + a * nblk * 2, nblk, s);
  std::vector<double> h(xf.size() * nblk * 2);
  HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double worst = 0.0;
  for (size_t a = 0; a < xf.size(); ++a) {
    double md = 0.0, mf = 0.0;
    for (int b = 0; b < nblk; ++b) {
      md = std::max(md, h[(a * nblk + b) * 2]);
      mf = std::max(mf, h[(a * nblk + b) * 2 + 1]);
    }
    if (mf > 0.0) worst = std::max(worst, md / mf);
    else if (md > 0.0) worst = std::max(worst, 1.0);
  }
  *out = worst;
  return KQFT_OK;
}

// out = x + sum_{j < nt} c_j k_j (x may be null), in launches of at most six terms; out may
// alias x, and alias a k_j only when nt <= 6 (one launch, each entry read before it is written)
static void lincomb_n(double2* out, const double2* x, int nt, const double2* const* k, const double* c, size_t count,
                     hipStream_t s) {
  int j0 = 0;
  do {
    LinComb a;
    memset(&a, 0, sizeof a);
    a.out = out;
    a.x = j0 == 0 ? x : out;
    a.nt = std::min(6, nt - j0);
    a.count = count;
    for (int j = 0; j < a.nt; ++j) {
      a.k[j] = k[j0 + j];
      a.c[j] = c[j0 + j];
    }
    launch_lincomb(a, s);
    j0 += 6;
  } while (j0 < nt);
}

// Re <a_i, b_i> for several pairs over count entries: per-block partials on the device, summed
// on the host in block order after one stream synchronisation.
static int dots(kqft_ctx* ctx, const std::vector<std::pair<const double2*, const double2*>>& ab, size_t count,
                hipStream_t s, std::vector<double>& out) {
  const int nblk = 256;
  int rc;
  if ((rc = ensure(ctx->pqred, std::max<size_t>(ab.size(), 1) * nblk * sizeof(double)))) return rc;
  double* part = (double*)ctx->pqred.p;
  for (size_t i = 0; i < ab.size(); ++i) launch_dot(ab[i].first, ab[i].second, count, part + i * nblk, nblk, s);
  std::vector<double> h(ab.size() * nblk);
  HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out.assign(ab.size(), 0.0);
  for (size_t i = 0; i < ab.size(); ++i)
    for (int b = 0; b < nblk; ++b) out[i] += h[i * nblk + b];
  return KQFT_OK;
}

// Solve A x = b (m x m, row-major) by Gaussian elimination with partial pivoting; false if
// a pivot vanishes.
static bool solve_small(std::vector<double> A, std::vector<double> b, int m, std::vector<double>& x) {
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (fabs(A[(size_t)r * m + col]) > fabs(A[(size_t)piv * m + col])) piv = r;
    if (A[(size_t)piv * m + col] == 0.0) return false;
    if (piv != col) {
      for (int c = 0; c < m; ++c) std::swap(A[(size_t)piv * m + c], A[(size_t)col * m + c]);
      std::swap(b[piv], b[col]);
    }
    for (int r = col + 1; r < m; ++r) {
      const double f = A[(size_t)r * m + col] / A[(size_t)col * m + col];
      for (int c = col; c < m; ++c) A[(size_t)r * m + c] -= f * A[(size_t)col * m + c];
      b[r] -= f * b[col];
    }
  }
  x.assign(m, 0.0);
  for (int r = m - 1; r >= 0; --r) {
    double t = b[r];
    for (int c = r + 1; c < m; ++c) t -= A[(size_t)r * m + c] * x[c];
    x[r] = t / A[(size_t)r * m + r];
  }
  return true;
}

// Loop of a full vertex (tables of all three channels in the a-channel order with the spin
// combination 2X + Y), arguments checked by the caller.
static int vloop_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, int kind, const kqft_quad& q,
                      double* out, hipStream_t s) {
  int rc;
  if ((rc = init_tables())) return rc;
  const size_t n = V.grid.n;
  const double* nodes;
  const double *qv, *qw;
  if ((rc = get_grid(ctx, V.grid, &nodes))) return rc;
  if ((rc = get_quad(ctx, q, &qv, &qw))) return rc;
  DProp P;
  if ((rc = to_dprop(G, P))) return rc;
  VLoopArgs la;
  memset(&la, 0, sizeof la);
  const size_t bytes = (n * n * n + 2 * n * n + n) * 32 * sizeof(double2);
  for (int r2 = 0; r2 < 3; ++r2) {
    const kqft_chvert& c = V.ch[r2];
    if (c.coef == 0.0 || (!c.K1 && !c.K2 && !c.K2p && !c.K3)) continue;
    if ((rc = ensure(ctx->vtab[r2], bytes))) return rc;
    TableArgs ta;
    memset(&ta, 0, sizeof ta);
    ta.n = (int)n;
    ta.r = KQFT_CH_A;
    ta.r2 = r2;
    ta.coef = c.coef;
    ta.mix[0] = 2.0;  // slot 0: 2X + Y; slot 1 unused
    ta.mix[1] = 1.0;
    ta.K[0] = (const double2*)c.K1;
    ta.K[1] = (const double2*)c.K2;
    ta.K[2] = (const double2*)c.K2p;
    ta.K[3] = (const double2*)c.K3;
    ta.out = ctx->vtab[r2].p;
    launch_table(ta, false, s);
    la.T[r2] = ctx->vtab[r2].p;
  }
  la.g = make_dgrid((int)n, V.grid.L, V.grid.a, V.grid.map);
  la.P = P;
  la.kind = kind;
  la.nq = q.n;
  la.r0 = V.r0;
  la.nodes = nodes;
  la.qv = qv;
  la.qw = qw;
  la.out = (double2*)out;
  {
    ProfScope ps(ctx, 3, s);
    launch_vloop(la, s);
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

extern "C" {

const char* kqft_last_error(void) { return g_err.c_str(); }

int kqft_ctx_create(kqft_ctx** ctx, int device) {
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(KQFT_EINVAL, "no such HIP device");
  HIP_TRY(hipSetDevice(device));
  kqft_ctx* c = new kqft_ctx();
  c->device = device;
  *ctx = c;
  int rc = init_tables();
  if (rc) {
    delete c;
    *ctx = nullptr;
  }
  return rc;
}

int kqft_ctx_destroy(kqft_ctx* ctx) {
  if (!ctx) return KQFT_OK;
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->grids) (void)hipFree(kv.second);
  for (auto& kv : ctx->quads) (void)hipFree(kv.second.first);
  DevBuf* bufs[] = {&ctx->panels[0], &ctx->panels[1], &ctx->pi[0], &ctx->pi[1], &ctx->phi, &ctx->chi_part,
                    &ctx->adj};
  for (DevBuf* b : bufs)
    if (b->p) free_buf(*b);
  for (auto& row : ctx->lstore)
    for (auto& b : row)
      if (b.p) free_buf(b);
  for (auto& row : ctx->tab)
    for (auto& b : row)
      if (b.p) free_buf(b);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (auto& row : ctx->dkf)
    for (auto& b : row)
      if (b.p) free_buf(b);
  free_buf(ctx->adjw);
  for (DevBuf* b : {&ctx->pq, &ctx->pqsig, &ctx->pqred, &ctx->vtab[0], &ctx->vtab[1], &ctx->vtab[2], &ctx->flow,
                    &ctx->flowml, &ctx->ctmp, &ctx->flowred, &ctx->pqx, &ctx->adapt, &ctx->sdep, &ctx->mf, &ctx->mftmp,
                    &ctx->mfflow, &ctx->mftail})
    if (b->p) free_buf(*b);
  free_buf(ctx->phigrad);
  for (auto* set : {&ctx->mlrec, &ctx->mlbar, &ctx->mlext})
    for (auto& row : *set)
      for (auto& b : row) free_buf(b);
  free_buf(ctx->mlscr);
  free_buf(ctx->gemmP);
  free_buf(ctx->chi_proj);
  if (ctx->sg) (void)hipStreamDestroy(ctx->sg);
  if (ctx->sm) (void)hipStreamDestroy(ctx->sm);
  delete ctx;
  return KQFT_OK;
}

int kqft_ctx_profile(kqft_ctx* ctx, int enable) {
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  double ms[4];
  int cnt[4];
  kqft_ctx_profile_read(ctx, ms, cnt);
  ctx->prof = enable != 0;
  return KQFT_OK;
}

int kqft_ctx_profile_read(kqft_ctx* ctx, double* ms, int* launches) {
  if (!ctx || !ms || !launches) return fail(KQFT_EINVAL, "NULL argument");
  int rc = KQFT_OK;
  for (int k = 0; k < 4; ++k) {
    ms[k] = 0.0;
    launches[k] = (int)ctx->ev[k].size();
    for (auto& e : ctx->ev[k]) {
      float t = 0.f;
      if (hipEventSynchronize(e.second) != hipSuccess || hipEventElapsedTime(&t, e.first, e.second) != hipSuccess)
        rc = fail(KQFT_EDEVICE, "event timing failed");
      ms[k] += t;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    ctx->ev[k].clear();
  }
  return rc;
}

size_t kqft_bubble_workspace(int n, int nq, int omega_batch, int precision) {
  if (n < 2 || nq < 1) return 0;
  const size_t per_w = panel_bytes_per_w(n, nq, precision);
  int nb = omega_batch > 0 ? omega_batch : (int)std::max<size_t>(1, ((size_t)4 << 30) / per_w);
  nb = std::min(nb, n);
  // two panel buffers, two propagator-pair buffers, up to four target-order class tables
  const size_t nn = n;
  const size_t table = (nn * nn * nn + 2 * nn * nn + nn) * 32 * (precision == KQFT_SPLIT_FP32 ? 8 : 16);
  // the per-combination products of one batch (FP64 entries on both paths)
  const size_t prod = 2 * (size_t)nb * 16 * (4 * nn + 4) * (4 * nn + 4);
  return 2 * (per_w + (size_t)nq * 256) * nb + 4 * table + prod;
}

int kqft_bubble(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                const kqft_chout* out, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if (channel < 0 || channel > 2) return fail(KQFT_EINVAL, "channel must be 0 (a), 1 (p) or 2 (t)");
  if (pi_kind != KQFT_PI_GG && pi_kind != KQFT_PI_DOT) return fail(KQFT_EINVAL, "unknown propagator pair");
  if ((rc = check_vertex(left, "left vertex")) || (rc = check_vertex(right, "right vertex"))) return rc;
  if (!same_grid(left->grid, right->grid)) return fail(KQFT_ESHAPE, "left and right vertices must share one grid");
  if (!out) return fail(KQFT_EINVAL, "out is NULL");
  const int m = opts->class_mask & KQFT_KALL;
  if (m == 0) return fail(KQFT_EINVAL, "class_mask selects no class");
  if (((m & KQFT_K1) && !out->K1) || ((m & KQFT_K2) && !out->K2) || ((m & KQFT_K2P) && !out->K2p) ||
      ((m & KQFT_K3) && !out->K3))
    return fail(KQFT_EINVAL, "an output class selected by class_mask is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  BubbleOut o{(double2*)out->K1, (double2*)out->K2, (double2*)out->K2p, (double2*)out->K3};
  return bubble_core(ctx, channel, *left, *right, *G, pi_kind, *q, *opts, o, (hipStream_t)stream);
}

int kqft_bubble_tune(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                     const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                     const kqft_chout* out, size_t max_workspace, int* omega_batch, double* ms, void* stream) {
  int rc;
  if (!omega_batch) return fail(KQFT_EINVAL, "omega_batch is NULL");
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if ((rc = check_vertex(left, "left vertex")) || (rc = check_vertex(right, "right vertex"))) return rc;
  const int n = left->grid.n;
  kqft_opts o = *opts;
  o.beta = 0;  // the outputs are scratch while tuning
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  // candidates: the whole grid and its halves, thirds, ... down to about 8 frequencies
  std::vector<int> cand;
  for (int parts : {1, 2, 3, 4, 6, 8, 12, 16}) {
    const int nb = (n + parts - 1) / parts;
    if (!cand.empty() && cand.back() == nb) continue;
    if (nb < 8 && !cand.empty()) break;
    if (max_workspace && kqft_bubble_workspace(n, q->n, nb, o.precision) > max_workspace) continue;
    cand.push_back(nb);
  }
  if (cand.empty()) return fail(KQFT_ENOMEM, "no transfer-frequency batch fits the workspace limit");
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = cand[0];
  float best_ms = 1e30f;
  for (int nb : cand) {
    o.omega_batch = nb;
    if ((rc = kqft_bubble(ctx, channel, left, right, G, pi_kind, q, &o, out, stream))) break;  // warm-up, sizes
    float t = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess || (rc = kqft_bubble(ctx, channel, left, right, G, pi_kind, q, &o, out,
                                                                 stream)) ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      if (!rc) rc = fail(KQFT_EDEVICE, "event timing failed while tuning");
      break;
    }
    if (t < best_ms) {
      best_ms = t;
      best = nb;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  ctx->tuned_nb[std::make_tuple(n, q->n, o.precision)] = best;
  *omega_batch = best;
  if (ms) *ms = best_ms;
  return KQFT_OK;
}

// Gauss-Lobatto-Kronrod rules on [-1, 1] (Sec. Frequency integration).  GL4 and its 7-point
// Kronrod extension in closed form; the 13-point extension (the GLK7 nodes plus three new
// symmetric pairs, exact for even degrees up to 18) from its moment equations: weights by a
// linear solve of the moments of degree 0..12, the new nodes by Newton on those of degree
// 14, 16, 18.  Nodes ascending.
struct GlkRules {
  double x7[7], w4[7], w7[7], x13[13], w13[13];
  bool ok = false;
};
static bool glk13_weights(const double pos[7], double wpos[7]) {
  std::vector<double> A(49), b(7), x;
  for (int k = 0; k < 7; ++k) {
    for (int c = 0; c < 7; ++c) A[(size_t)k * 7 + c] = (pos[c] == 0.0 ? 1.0 : 2.0) * pow(pos[c], 2.0 * k);
    b[k] = 2.0 / (2.0 * k + 1.0);
  }
  if (!solve_small(A, b, 7, x)) return false;
  for (int c = 0; c < 7; ++c) wpos[c] = x[c];
  return true;
}
static const GlkRules& glk_rules() {
  static GlkRules R;
  if (R.ok) return R;
  const double s5 = 1.0 / sqrt(5.0), s23 = sqrt(2.0 / 3.0);
  const double x7[7] = {-1.0, -s23, -s5, 0.0, s5, s23, 1.0};
  const double w4[7] = {1.0 / 6.0, 0.0, 5.0 / 6.0, 0.0, 5.0 / 6.0, 0.0, 1.0 / 6.0};
  const double w7[7] = {11.0 / 210.0, 72.0 / 245.0, 125.0 / 294.0, 16.0 / 35.0, 125.0 / 294.0, 72.0 / 245.0,
                        11.0 / 210.0};
  for (int k = 0; k < 7; ++k) {
    R.x7[k] = x7[k];
    R.w4[k] = w4[k];
    R.w7[k] = w7[k];
  }
  double t[3] = {0.94, 0.64, 0.24};  // the new positive nodes
  auto resid = [&](const double tt[3], double out[3], double wpos[7], double pos[7]) -> bool {
    const double p[7] = {0.0, s5, s23, 1.0, tt[0], tt[1], tt[2]};
    for (int c = 0; c < 7; ++c) pos[c] = p[c];
    if (!glk13_weights(pos, wpos)) return false;
    for (int q = 0; q < 3; ++q) {
      const double k = 14.0 + 2.0 * q;
      double m = 0.0;
      for (int c = 0; c < 7; ++c) m += (pos[c] == 0.0 ? 1.0 : 2.0) * wpos[c] * pow(pos[c], k);
      out[q] = m - 2.0 / (k + 1.0);
    }
    return true;
  };
  double wpos[7], pos[7], r0[3];
  for (int itn = 0; itn < 60; ++itn) {
    if (!resid(t, r0, wpos, pos)) return R;
    if (fabs(r0[0]) + fabs(r0[1]) + fabs(r0[2]) < 1e-16) break;
    std::vector<double> J(9), rhs(3), dx;
    for (int c = 0; c < 3; ++c) {
      double tp[3] = {t[0], t[1], t[2]}, tm[3] = {t[0], t[1], t[2]}, rp[3], rm[3], wd[7], pd[7];
      tp[c] += 1e-7;
      tm[c] -= 1e-7;
      if (!resid(tp, rp, wd, pd) || !resid(tm, rm, wd, pd)) return R;
      for (int q = 0; q < 3; ++q) J[(size_t)q * 3 + c] = (rp[q] - rm[q]) / 2e-7;
    }
    for (int q = 0; q < 3; ++q) rhs[q] = r0[q];
    if (!solve_small(J, rhs, 3, dx)) return R;
    for (int c = 0; c < 3; ++c) t[c] -= dx[c];
  }
  if (!resid(t, r0, wpos, pos)) return R;
  // ascending nodes: -pos (descending magnitude), 0, +pos
  std::vector<std::pair<double, double>> nw;
  for (int c = 0; c < 7; ++c) {
    nw.push_back({pos[c], wpos[c]});
    if (pos[c] != 0.0) nw.push_back({-pos[c], wpos[c]});
  }
  std::sort(nw.begin(), nw.end());
  if (nw.size() != 13) return R;
  for (int k = 0; k < 13; ++k) {
    R.x13[k] = nw[k].first;
    R.w13[k] = nw[k].second;
  }
  R.ok = true;
  return R;
}

int kqft_bubble_adaptive(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                         const kqft_propagator* G, int pi_kind, const kqft_quad* q, double eps, const kqft_opts* opts,
                         const kqft_chout* out, kqft_adapt_info* info, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if (channel < 0 || channel > 2) return fail(KQFT_EINVAL, "channel must be 0 (a), 1 (p) or 2 (t)");
  if (pi_kind != KQFT_PI_GG && pi_kind != KQFT_PI_DOT) return fail(KQFT_EINVAL, "unknown propagator pair");
  if (q->map != KQFT_QUAD_TAN_FINITE) return fail(KQFT_EINVAL, "the adaptive bubble integrates over [-L, L]");
  if (!(eps > 0)) return fail(KQFT_EINVAL, "eps must be positive");
  if ((rc = check_vertex(left, "left vertex")) || (rc = check_vertex(right, "right vertex"))) return rc;
  if (!same_grid(left->grid, right->grid)) return fail(KQFT_ESHAPE, "left and right vertices must share one grid");
  if (!out) return fail(KQFT_EINVAL, "out is NULL");
  const int msk = opts->class_mask & KQFT_KALL;
  if (msk == 0) return fail(KQFT_EINVAL, "class_mask selects no class");
  if (((msk & KQFT_K1) && !out->K1) || ((msk & KQFT_K2) && !out->K2) || ((msk & KQFT_K2P) && !out->K2p) ||
      ((msk & KQFT_K3) && !out->K3))
    return fail(KQFT_EINVAL, "an output class selected by class_mask is NULL");
  const GlkRules& gr = glk_rules();
  if (!gr.ok) return fail(KQFT_EDEVICE, "Gauss-Lobatto-Kronrod rule construction failed");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int r = channel, n = left->grid.n;
  if ((rc = init_tables())) return rc;
  const double* nodes;
  if ((rc = get_grid(ctx, left->grid, &nodes))) return rc;
  DProp P;
  if ((rc = to_dprop(*G, P))) return rc;
  SideTables TL, TR;
  if ((rc = build_tables(ctx, r, *left, *right, false, TL, TR, s))) return rc;
  // outputs in the order K1, K2, K2', K3 of the selected classes
  const long long cnts[4] = {n, (long long)n * n, (long long)n * n, (long long)n * n * n};
  const int bits[4] = {KQFT_K1, KQFT_K2, KQFT_K2P, KQFT_K3};
  double2* outs[4] = {(double2*)out->K1, (double2*)out->K2, (double2*)out->K2p, (double2*)out->K3};
  long long nout_tot = 0;
  AdaptArgs A;
  memset(&A, 0, sizeof A);
  for (int c = 0; c < 4; ++c) {
    A.cstart[c] = (int)nout_tot;
    A.ccount[c] = (msk & bits[c]) ? (int)cnts[c] : 0;
    nout_tot += A.ccount[c];
    A.K[c] = (msk & bits[c]) ? outs[c] : nullptr;
    if (msk & bits[c]) HIP_TRY(hipMemsetAsync(outs[c], 0, 2 * (size_t)cnts[c] * 16 * sizeof(double2), s));
  }
  if (nout_tot > (1LL << 28)) return fail(KQFT_ESHAPE, "too many outputs for the adaptive bubble");
  // outputs in batches of at most 8192, each refined to the end before the next: one
  // generation's list then holds at most 2048 intervals per output on average
  const long long cap = 1LL << 24;
  const long long bsz = std::min<long long>(nout_tot, 8192);
  // device memory: two rules (78 doubles), scale per output, two work lists, counters
  const size_t rule_b = 2 * 39 * sizeof(double), scale_b = (size_t)nout_tot * sizeof(double);
  const size_t list_b = (size_t)cap * sizeof(AdaptItem);
  const size_t off_scale = 1024, off_l0 = off_scale + ((scale_b + 255) / 256) * 256, off_l1 = off_l0 + list_b,
               off_cnt = off_l1 + list_b;
  if ((rc = ensure(ctx->adapt, off_cnt + 256))) return rc;
  char* base = (char*)ctx->adapt.p;
  double* rules = (double*)base;
  double* scale = (double*)(base + off_scale);
  AdaptItem* lists[2] = {(AdaptItem*)(base + off_l0), (AdaptItem*)(base + off_l1)};
  int* counters = (int*)(base + off_cnt);  // next count, overflow
  std::vector<double> hr(78, 0.0);
  for (int k = 0; k < 13; ++k) {
    hr[k] = gr.x13[k];
    hr[13 + k] = gr.w13[k];
  }
  for (int k = 0; k < 7; ++k) {
    hr[39 + k] = gr.x7[k];
    hr[39 + 13 + k] = gr.w4[k];
    hr[39 + 26 + k] = gr.w7[k];
  }
  HIP_TRY(hipMemcpyAsync(rules, hr.data(), rule_b, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(counters, 0, 2 * sizeof(int), s));
  A.L = make_gather(r, 1, 0, 0, 0, 0, 0, 0, *left, TL, nodes, nullptr, nullptr, nullptr, nullptr);
  A.R = make_gather(r, 1, 0, 0, 0, 0, 0, 0, *right, TR, nodes, nullptr, nullptr, nullptr, nullptr);
  A.P = P;
  A.r = r;
  A.kind = pi_kind;
  A.n = n;
  for (int u = 0; u < 4; ++u) A.unmix[u] = kUnmix[r][u];
  A.qa = q->a;
  A.qth = atan(q->L / q->a);
  A.eps = eps;
  A.min_width = 1e-12;
  A.max_depth = 40;
  A.scale = scale;
  A.nout = counters;
  A.overflow = counters + 1;
  A.cap = (int)cap;
  int gens_max = 0;
  long long accepted = 0, evals = 0;
  std::vector<AdaptItem> init((size_t)bsz);
  for (long long o0 = 0; o0 < nout_tot; o0 += bsz) {
    const long long nb = std::min(bsz, nout_tot - o0);
    for (long long o = 0; o < nb; ++o) init[(size_t)o] = AdaptItem{-1.0, 1.0, (int)(o0 + o), 0};
    HIP_TRY(hipMemcpyAsync(lists[0], init.data(), (size_t)nb * sizeof(AdaptItem), hipMemcpyHostToDevice, s));
    // error scales: GLK13 over the whole interval of every output of the batch
    A.phase = 0;
    A.nn = 13;
    A.rule = rules;
    A.in = lists[0];
    A.nin = (int)nb;
    A.out = lists[1];
    launch_adaptive(A, s);
    HIP_TRY(hipGetLastError());
    evals += 13 * nb;
    // generations of GL4 / GLK7 steps
    A.phase = 1;
    A.nn = 7;
    A.rule = rules + 39;
    int cur = 0, gens = 0;
    long long nin = nb;
    while (nin > 0) {
      if (gens > A.max_depth + 1) return fail(KQFT_ENOCONV, "adaptive bubble did not terminate");
      HIP_TRY(hipMemsetAsync(counters, 0, sizeof(int), s));
      A.in = lists[cur];
      A.nin = (int)nin;
      A.out = lists[cur ^ 1];
      launch_adaptive(A, s);
      HIP_TRY(hipGetLastError());
      int hc[2];
      HIP_TRY(hipMemcpyAsync(hc, counters, sizeof hc, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (hc[1]) return fail(KQFT_ENOMEM, "adaptive work list overflow");
      evals += 7 * nin;
      accepted += nin - hc[0] / 6;
      nin = hc[0];
      cur ^= 1;
      ++gens;
    }
    gens_max = std::max(gens_max, gens);
  }
  if (info) {
    info->intervals = accepted;
    info->generations = gens_max;
    info->evaluations = evals;
  }
  return KQFT_OK;
}

int kqft_sde(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q_bubble,
             const kqft_quad* q_loop, const kqft_opts* opts, double* sigma, double* chi, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q_bubble, opts))) return rc;
  if (!q_loop || q_loop->n < 1) return fail(KQFT_ESHAPE, "invalid loop quadrature");
  if (chi && q_bubble->n > 46340) return fail(KQFT_ESHAPE, "chi needs q_bubble->n <= 46340");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!sigma) return fail(KQFT_EINVAL, "sigma is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  return sde_core(ctx, gamma, G, q_bubble, q_loop, opts, sigma, chi, (hipStream_t)stream);
}

int kqft_chi(kqft_ctx* ctx, int channel, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
             double* chi, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (channel < KQFT_CH_A || channel > KQFT_CH_T) return fail(KQFT_EINVAL, "channel must be 0, 1 or 2");
  if (!G || !q) return fail(KQFT_EINVAL, "propagator and quadrature must be given");
  if (q->n < 1 || (q->map != KQFT_QUAD_TAN_FINITE && q->map != KQFT_QUAD_TAN_INFINITE) ||
      (q->map == KQFT_QUAD_TAN_FINITE && !(q->L > 0)) || !(q->a > 0))
    return fail(KQFT_ESHAPE, "invalid quadrature");
  if (q->n > 46340) return fail(KQFT_ESHAPE, "chi needs q->n <= 46340");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!chi) return fail(KQFT_EINVAL, "chi is NULL");
  DProp P;
  if ((rc = to_dprop(*G, P))) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  const double* nodes;
  if ((rc = get_grid(ctx, gamma->grid, &nodes))) return rc;
  const hipStream_t s = (hipStream_t)stream;
  if ((rc = chi_core(ctx, channel, *gamma, P, nodes, *q, chi, s))) return rc;
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

static int check_mprop(const kqft_mprop& G) {
  if (!(G.Delta > 0)) return fail(KQFT_EINVAL, "Delta must be positive");
  if (G.reg != KQFT_REG_DELTA && G.reg != KQFT_REG_U) return fail(KQFT_EINVAL, "unknown Matsubara regulator");
  if (G.reg == KQFT_REG_U && !(G.lam > 0)) return fail(KQFT_EINVAL, "the interaction regulator needs lam > 0");
  if (G.sigma_N < 0 || ((G.sigma || G.dsigma) && G.sigma_N == 0)) return fail(KQFT_ESHAPE, "invalid self-energy box");
  return KQFT_OK;
}

static MGatherArgs mf_side(const kqft_mgrid& g, int channel, int kind, int Nq, const kqft_mvertex& v,
                           const kqft_mprop& G) {
  MGatherArgs a;
  memset(&a, 0, sizeof a);
  a.r = channel;
  a.M = g.M;
  a.N = g.N;
  a.Nq = Nq;
  a.kind = kind;
  a.T = g.T;
  a.Delta = G.Delta;
  a.sigma = (const double2*)G.sigma;
  a.dsigma = (const double2*)G.dsigma;
  a.Ns = (G.sigma || G.dsigma) ? G.sigma_N : 0;
  a.U = v.U;
  a.reg = G.reg;
  a.lam = G.lam;
  for (int r = 0; r < 3; ++r)
    a.ch[r] = MChan{v.ch[r].coef, {(const double2*)v.ch[r].K1, (const double2*)v.ch[r].K2,
                                   (const double2*)v.ch[r].K2p, (const double2*)v.ch[r].K3}};
  for (int u = 0; u < 4; ++u) a.mix[u] = kMix[channel][u];
  return a;
}

int kqft_loop_matsubara(kqft_ctx* ctx, const kqft_mvertex* gamma, const kqft_mprop* G, int kind, int Nl,
                        double* out, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!gamma || !G || !out) return fail(KQFT_EINVAL, "vertex, propagator and out must be given");
  if (kind < KQFT_LINE_G || kind > KQFT_LINE_GSG) return fail(KQFT_EINVAL, "kind must be a KQFT_LINE_* value");
  if (kind == KQFT_LINE_GSG && !G->dsigma) return fail(KQFT_EINVAL, "the G Sigma_dot G line needs Sigma_dot");
  if (gamma->grid.M < 0 || gamma->grid.N < 1 || Nl < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1, Nl >= 1");
  if (!(gamma->grid.T > 0)) return fail(KQFT_EINVAL, "T must be positive");
  if ((rc = check_mprop(*G))) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  launch_mf_vloop(mf_side(gamma->grid, KQFT_CH_A, 0, 1, *gamma, *G), kind, Nl, (double2*)out, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

// digamma and trigamma for x > 0: upward recurrence to x >= 10, then the asymptotic series in
// 1/x^2 with Bernoulli-number coefficients (Abramowitz and Stegun 6.3.18, 6.4.12)
static double digamma_pos(double x) {
  double r = 0.0;
  while (x < 10.0) {
    r -= 1.0 / x;
    x += 1.0;
  }
  const double f = 1.0 / (x * x);
  return r + std::log(x) - 0.5 / x -
         f * (1.0 / 12 - f * (1.0 / 120 - f * (1.0 / 252 - f * (1.0 / 240 - f * (1.0 / 132)))));
}
static double trigamma_pos(double x) {
  double r = 0.0;
  while (x < 10.0) {
    r += 1.0 / (x * x);
    x += 1.0;
  }
  const double f = 1.0 / (x * x);
  return r + 1.0 / x + 0.5 * f + f / x * (1.0 / 6 - f * (1.0 / 30 - f * (1.0 / 42 - f * (1.0 / 30 - f * (5.0 / 66)))));
}

// T sum over every n'' of the bare Pi_r(m, n''), G_0 = 1/(i nu + i Delta sgn nu): for a and t the
// n'' where both frequencies share a sign sum to digamma differences (twice the same value by
// the reflection n'' -> -n'' - 1 - m), the |m| mixed terms are added; p is minus a (G_0 odd).
static double mf_bare_bubble_sum(int r, int m, double Delta, double T) {
  const int ma = std::abs(m);
  const double d = Delta / (2.0 * M_PI * T), c = 1.0 / (4.0 * M_PI * M_PI * T * T);
  const double same = c * (ma == 0 ? trigamma_pos(0.5 + d) : (digamma_pos(0.5 + ma + d) - digamma_pos(0.5 + d)) / ma);
  double mixed = 0.0;
  for (int n = -ma; n < 0; ++n)
    mixed += 1.0 / (((2.0 * (n + ma) + 1.0) * M_PI * T + Delta) * ((2.0 * n + 1.0) * M_PI * T - Delta));
  const double sa = -T * (2.0 * same + mixed);
  return r == KQFT_CH_P ? -sa : sa;
}

int kqft_regrid(kqft_ctx* ctx, const kqft_grid* src, const kqft_grid* dst, const kqft_chout* gamma_in,
                const double* sigma_in, const kqft_chout* gamma_out, double* sigma_out, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!src || !dst) return fail(KQFT_EINVAL, "both grids must be given");
  if ((rc = check_grid(*src, "source grid")) || (rc = check_grid(*dst, "destination grid"))) return rc;
  if ((gamma_in == nullptr) != (gamma_out == nullptr) || (sigma_in == nullptr) != (sigma_out == nullptr))
    return fail(KQFT_EINVAL, "inputs and outputs must be given together");
  if (!gamma_in && !sigma_in) return fail(KQFT_EINVAL, "nothing to regrid");
  if (gamma_in)
    for (int r = 0; r < 3; ++r) {
      const double* iv[4] = {gamma_in[r].K1, gamma_in[r].K2, gamma_in[r].K2p, gamma_in[r].K3};
      const double* ov[4] = {gamma_out[r].K1, gamma_out[r].K2, gamma_out[r].K2p, gamma_out[r].K3};
      for (int c = 0; c < 4; ++c) {
        if ((iv[c] == nullptr) != (ov[c] == nullptr))
          return fail(KQFT_EINVAL, "a class must be given on both sides or on neither");
        if (iv[c] && iv[c] == ov[c]) return fail(KQFT_EINVAL, "regridding cannot run in place");
      }
    }
  if (sigma_in && sigma_in == sigma_out) return fail(KQFT_EINVAL, "regridding cannot run in place");
  const double* nodes = nullptr;
  HIP_TRY(hipSetDevice(ctx->device));
  if ((rc = get_grid(ctx, *dst, &nodes))) return rc;
  hipStream_t s = (hipStream_t)stream;
  RegridArgs a;
  memset(&a, 0, sizeof a);
  a.src = make_dgrid(src->n, src->L, src->a, src->map);
  a.dst = nodes;
  a.nd = dst->n;
  if (gamma_in)
    for (int r = 0; r < 3; ++r) {
      const double* iv[4] = {gamma_in[r].K1, gamma_in[r].K2, gamma_in[r].K2p, gamma_in[r].K3};
      double* ov[4] = {gamma_out[r].K1, gamma_out[r].K2, gamma_out[r].K2p, gamma_out[r].K3};
      const int dims[4] = {1, 2, 2, 3};
      for (int c = 0; c < 4; ++c) {
        if (!iv[c]) continue;
        a.dims = dims[c];
        a.nspin = 2;
        a.ncomp = 16;
        a.in = (const double2*)iv[c];
        a.out = (double2*)ov[c];
        launch_regrid(a, s);
      }
    }
  if (sigma_in) {
    a.dims = 1;
    a.nspin = 1;
    a.ncomp = 4;
    a.in = (const double2*)sigma_in;
    a.out = (double2*)sigma_out;
    launch_regrid(a, s);
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

int kqft_chi_matsubara(kqft_ctx* ctx, int channel, const kqft_mvertex* gamma, const kqft_mprop* G, int Nq,
                       double* chi, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!gamma || !G || !chi) return fail(KQFT_EINVAL, "vertex, propagator and chi must be given");
  if (channel < KQFT_CH_A || channel > KQFT_CH_T) return fail(KQFT_EINVAL, "channel must be 0, 1 or 2");
  if (gamma->grid.M < 0 || gamma->grid.N < 1 || Nq < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1, Nq >= 1");
  if (Nq > 16384) return fail(KQFT_ESHAPE, "chi needs Nq <= 16384");
  if (!(gamma->grid.T > 0)) return fail(KQFT_EINVAL, "T must be positive");
  if ((rc = check_mprop(*G))) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  launch_mf_chi(mf_side(gamma->grid, channel, 0, Nq, *gamma, *G), (double2*)chi, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

int kqft_bubble_matsubara(kqft_ctx* ctx, int channel, const kqft_mvertex* left, const kqft_mvertex* right,
                          const kqft_mprop* G, int pi_kind, int Nq, int tails, const kqft_chout* out, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!left || !right || !G || !out) return fail(KQFT_EINVAL, "vertices, propagator and outputs must be given");
  if (channel < KQFT_CH_A || channel > KQFT_CH_T) return fail(KQFT_EINVAL, "channel must be 0, 1 or 2");
  if (pi_kind != KQFT_PI_GG && pi_kind != KQFT_PI_DOT) return fail(KQFT_EINVAL, "unknown bubble kind");
  if (tails != 0 && (tails != 1 || pi_kind != KQFT_PI_GG))
    return fail(KQFT_EINVAL, "tails must be 0 or 1, and 1 only for the bubble G G");
  if (tails && G && G->reg != KQFT_REG_DELTA)
    return fail(KQFT_EINVAL, "the analytic tails need the unregulated G_0 (reg = KQFT_REG_DELTA)");
  const kqft_mgrid g = left->grid;
  if (g.M < 0 || g.N < 1 || Nq < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1, Nq >= 1");
  if (right->grid.M != g.M || right->grid.N != g.N || right->grid.T != g.T)
    return fail(KQFT_ESHAPE, "left and right must share the Matsubara grid");
  if (!(g.T > 0)) return fail(KQFT_EINVAL, "T must be positive");
  if ((rc = check_mprop(*G))) return rc;
  if (!out->K1 || !out->K2 || !out->K2p || !out->K3) return fail(KQFT_EINVAL, "all four output classes are required");
  const long R = 2L * g.N + 1, Kw = 2L * Nq, nbos = 2L * g.M + 1;
  if (R * Kw > (1L << 30) || R * R > (1L << 30)) return fail(KQFT_ESHAPE, "Matsubara panels too large");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // per bosonic frequency: A and B for two combinations, C for two
  const size_t per_m = (size_t)(4 * R * Kw + 2 * R * R) * sizeof(double2);
  const long nb = std::max(1L, std::min(nbos, (long)((size_t)(512u << 20) / per_m)));
  if (nb * R * Kw > (1L << 31) - 1) return fail(KQFT_ESHAPE, "Matsubara panels too large");
  if ((rc = ensure(ctx->mf, (size_t)nb * per_m))) return rc;
  double2* base = (double2*)ctx->mf.p;
  double2* A[2] = {base, base + (size_t)nb * R * Kw};
  double2* B[2] = {base + 2 * (size_t)nb * R * Kw, base + 3 * (size_t)nb * R * Kw};
  double2* Cm[2] = {base + 4 * (size_t)nb * R * Kw, base + 4 * (size_t)nb * R * Kw + (size_t)nb * R * R};
  auto side = [&](const kqft_mvertex& v, double2* const* P, int m0, int cnt) {
    MGatherArgs a = mf_side(g, channel, pi_kind, Nq, v, *G);
    a.m0 = m0;
    a.nb = cnt;
    a.P[0] = P[0];
    a.P[1] = P[1];
    return a;
  };
  for (int m0 = -g.M; m0 <= g.M; m0 += (int)nb) {
    const int cnt = (int)std::min<long>(nb, g.M - m0 + 1);
    {
      ProfScope ps(ctx, 1, s);
      launch_mf_left(side(*left, A, m0, cnt), s);
      launch_mf_right(side(*right, B, m0, cnt), s);
    }
    // C = A B per bosonic frequency and combination on the project's FP64 MFMA GEMM
    for (int c = 0; c < 2; ++c) {
      ZgemmArgs z;
      memset(&z, 0, sizeof z);
      z.A = A[c];
      z.B = B[c];
      z.C = Cm[c];
      z.M = (int)R;
      z.N = (int)R;
      z.K = (int)Kw;
      z.batch = cnt;
      z.lda = Kw;
      z.ldb = R;
      z.ldc = R;
      z.strideA = R * Kw;
      z.strideB = R * Kw;
      z.strideC = R * R;
      ProfScope ps(ctx, 2, s);
      launch_zgemm_nn(z, s);
    }
    MEpiArgs e;
    memset(&e, 0, sizeof e);
    e.M = g.M;
    e.N = g.N;
    e.m0 = m0;
    e.nb = cnt;
    for (int u = 0; u < 4; ++u) e.unmix[u] = kUnmix[channel][u];
    e.C[0] = Cm[0];
    e.C[1] = Cm[1];
    e.K[0] = (double2*)out->K1;
    e.K[1] = (double2*)out->K2;
    e.K[2] = (double2*)out->K2p;
    e.K[3] = (double2*)out->K3;
    {
      ProfScope ps(ctx, 3, s);
      launch_mf_epilogue(e, s);
    }
  }
  if (tails) {  // the bare sum beyond each window, with the large-frequency vertices
    std::vector<double2> t(nbos);
    for (int m = -g.M; m <= g.M; ++m) {
      const int sm = channel == KQFT_CH_P ? -m : m;
      const int x = -2 * Nq - sm;
      const int lo = x >= 0 ? (x + 1) / 2 : -((-x) / 2);
      const int len = 2 * Nq - ((m & 1) ? 1 : 0);
      std::complex<double> w = 0.0;
      for (int k = lo; k < lo + len; ++k) {
        const int k1 = channel == KQFT_CH_P ? k : k + m, k2 = channel == KQFT_CH_P ? m - k - 1 : k;
        auto g0 = [&](int n) {
          const double v = (2.0 * n + 1.0) * M_PI * g.T;
          return 1.0 / std::complex<double>(0.0, v + (v > 0.0 ? G->Delta : -G->Delta));
        };
        w += g.T * g0(k1) * g0(k2);
      }
      const std::complex<double> tm = mf_bare_bubble_sum(channel, m, G->Delta, g.T) - w;
      t[m + g.M] = make_double2(tm.real(), tm.imag());
    }
    if ((rc = ensure(ctx->mftail, (size_t)nbos * sizeof(double2)))) return rc;
    HIP_TRY(hipMemcpyAsync(ctx->mftail.p, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    MTailArgs ta;
    memset(&ta, 0, sizeof ta);
    ta.M = g.M;
    ta.N = g.N;
    ta.t = (const double2*)ctx->mftail.p;
    for (int u = 0; u < 4; ++u) {
      ta.mix[u] = kMix[channel][u];
      ta.unmix[u] = kUnmix[channel][u];
    }
    ta.UL = left->U;
    ta.UR = right->U;
    const kqft_chvert &cl = left->ch[channel], &cr = right->ch[channel];
    ta.L = MChan{cl.coef, {(const double2*)cl.K1, (const double2*)cl.K2, (const double2*)cl.K2p, (const double2*)cl.K3}};
    ta.R = MChan{cr.coef, {(const double2*)cr.K1, (const double2*)cr.K2, (const double2*)cr.K2p, (const double2*)cr.K3}};
    ta.K[0] = (double2*)out->K1;
    ta.K[1] = (double2*)out->K2;
    ta.K[2] = (double2*)out->K2p;
    ta.K[3] = (double2*)out->K3;
    launch_mf_tail(ta, s);
    HIP_TRY(hipStreamSynchronize(s));  // t lives on the host until the copy has run
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

int kqft_sde_matsubara(kqft_ctx* ctx, const kqft_mvertex* gamma, const kqft_mprop* G, int Nq, int Nl,
                       double* sigma_out, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!gamma || !G || !sigma_out) return fail(KQFT_EINVAL, "vertex, propagator and sigma_out must be given");
  if (Nl < 1) return fail(KQFT_ESHAPE, "need Nl >= 1");
  const kqft_mgrid g = gamma->grid;
  if (g.M < 0 || g.N < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // Phi = B_a(Gamma_0, Gamma): all four classes into the scratch (K2 and K3 vanish)
  const size_t nb = 2 * (size_t)g.M + 1, nf = 2 * (size_t)g.N;
  const size_t c1 = 2 * nb, c2 = 2 * nb * nf, c3 = 2 * nb * nf * nf;
  if ((rc = ensure(ctx->phi, (c1 + 2 * c2 + c3) * sizeof(double2)))) return rc;
  double2* ph = (double2*)ctx->phi.p;
  kqft_chout po{(double*)ph, (double*)(ph + c1), (double*)(ph + c1 + c2), (double*)(ph + c1 + 2 * c2)};
  kqft_mvertex bare;
  memset(&bare, 0, sizeof bare);
  bare.grid = g;
  bare.U = gamma->U;
  if ((rc = kqft_bubble_matsubara(ctx, KQFT_CH_A, &bare, gamma, G, KQFT_PI_GG, Nq, 0, &po, stream))) return rc;
  MLoopArgs la;
  memset(&la, 0, sizeof la);
  la.M = g.M;
  la.N = g.N;
  la.Nl = Nl;
  la.T = g.T;
  la.Delta = G->Delta;
  la.reg = G->reg;
  la.lam = G->lam;
  la.sigma = (const double2*)G->sigma;
  la.Ns = G->sigma ? G->sigma_N : 0;
  la.K1 = ph;
  la.K2p = ph + c1 + c2;
  la.out = (double2*)sigma_out;
  {
    ProfScope ps(ctx, 3, s);
    launch_mf_loop(la, s);
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

static int fixed_point_core(kqft_ctx* ctx, size_t stc, double2* xb, double2* g, const kqft_parquet_opts& po,
                            const std::function<int()>& eval, const std::function<int(double*)>& residual,
                            double* residuals, int* iterations, hipStream_t s);

int kqft_parquet_solve_matsubara(kqft_ctx* ctx, const kqft_mgrid* grid, double U, double Delta, int Nq, int Nl,
                                 const kqft_parquet_opts* popts, const kqft_chout* gamma, double* sigma,
                                 double* residuals, int* iterations, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!grid || !popts || !gamma || !sigma || !iterations)
    return fail(KQFT_EINVAL, "grid, options, gamma, sigma and iterations must be given");
  const kqft_mgrid g = *grid;
  if (g.M < 0 || g.N < 1 || Nq < 1 || Nl < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1, Nq >= 1, Nl >= 1");
  if (!(g.T > 0) || !(Delta > 0)) return fail(KQFT_EINVAL, "T and Delta must be positive");
  const kqft_parquet_opts po = *popts;
  if (!(po.alpha > 0) || po.alpha > 1 || po.max_iterations < 1)
    return fail(KQFT_EINVAL, "need 0 < alpha <= 1, max_iterations >= 1");
  if (po.anderson_depth < 0 || po.anderson_depth > 32) return fail(KQFT_EINVAL, "need 0 <= anderson_depth <= 32");
  if (po.reduce_alpha && (!(po.alpha_min > 0) || po.alpha_min > po.alpha))
    return fail(KQFT_EINVAL, "need 0 < alpha_min <= alpha");
  if (po.hartree != 0 || (po.sde_forms != 0 && po.sde_forms != 1))
    return fail(KQFT_EINVAL, "the Matsubara solver takes the symmetric model and the a-channel SDE");
  for (int r = 0; r < 3; ++r)
    if (!gamma[r].K1 || !gamma[r].K2 || !gamma[r].K2p || !gamma[r].K3)
      return fail(KQFT_EINVAL, "gamma arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int m = po.anderson_depth;
  const size_t nb = 2 * (size_t)g.M + 1, nf = 2 * (size_t)g.N;
  const size_t cnt[4] = {2 * nb, 2 * nb * nf, 2 * nb * nf, 2 * nb * nf * nf};
  const size_t chc = cnt[0] + cnt[1] + cnt[2] + cnt[3];
  const size_t stc = 3 * chc + nf;  // channels a, p, t (K1, K2, K2', K3), Sigma [2N]
  if ((rc = ensure(ctx->pq, stc * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx->pqx, (size_t)(4 + 2 * m) * stc * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx->mftmp, chc * sizeof(double2)))) return rc;
  double2* gb = (double2*)ctx->pq.p;
  double2* xb = (double2*)ctx->pqx.p;
  double2* tmp = (double2*)ctx->mftmp.p;
  auto cls = [&](double2* base, int r, int c) {
    size_t off = (size_t)r * chc;
    for (int u = 0; u < c; ++u) off += cnt[u];
    return base + off;
  };
  auto chout = [&](double2* base) {
    return kqft_chout{(double*)base, (double*)(base + cnt[0]), (double*)(base + cnt[0] + cnt[1]),
                      (double*)(base + cnt[0] + cnt[1] + cnt[2])};
  };
  double2* xsig = xb + 3 * chc;
  // PT2 start: gamma_r = B_r(Gamma_0, Gamma_0) (K1 only), Sigma^(2) = SDE(Gamma_0), bare G
  kqft_mvertex bare;
  memset(&bare, 0, sizeof bare);
  bare.grid = g;
  bare.U = U;
  const kqft_mprop G0{Delta, nullptr, 0, nullptr};
  for (int r = 0; r < 3; ++r) {
    const kqft_chout o = chout(cls(xb, r, 0));
    if ((rc = kqft_bubble_matsubara(ctx, r, &bare, &bare, &G0, KQFT_PI_GG, Nq, 0, &o, stream))) return rc;
  }
  if ((rc = kqft_sde_matsubara(ctx, &bare, &G0, Nq, Nl, (double*)xsig, stream))) return rc;
  kqft_mvertex V;
  memset(&V, 0, sizeof V);
  V.grid = g;
  V.U = U;
  for (int r = 0; r < 3; ++r)
    V.ch[r] = kqft_chvert{1.0, (const double*)cls(xb, r, 0), (const double*)cls(xb, r, 1),
                          (const double*)cls(xb, r, 2), (const double*)cls(xb, r, 3)};
  const kqft_mprop Gs{Delta, (const double*)xsig, g.N, nullptr};
  std::vector<std::pair<const double2*, const double2*>> xf;
  std::vector<size_t> counts;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      xf.push_back({cls(xb, r, c), cls(gb, r, c)});
      counts.push_back(cnt[c]);
    }
  xf.push_back({xsig, gb + 3 * chc});
  counts.push_back(nf);
  // F: gamma_r' = 1/2 [B_r(I_r, Gamma) + B_r(Gamma, I_r)], Sigma' = SDE(Gamma) with the state's Sigma
  auto eval = [&]() -> int {
    for (int r = 0; r < 3; ++r) {
      kqft_mvertex I = V;
      I.ch[r] = kqft_chvert{0.0, nullptr, nullptr, nullptr, nullptr};
      const kqft_chout o1 = chout(cls(gb, r, 0)), o2 = chout(tmp);
      if ((rc = kqft_bubble_matsubara(ctx, r, &I, &V, &Gs, KQFT_PI_GG, Nq, 0, &o1, stream))) return rc;
      if ((rc = kqft_bubble_matsubara(ctx, r, &V, &I, &Gs, KQFT_PI_GG, Nq, 0, &o2, stream))) return rc;
      const double2* k[2] = {cls(gb, r, 0), tmp};
      const double c[2] = {0.5, 0.5};
      lincomb_n(cls(gb, r, 0), nullptr, 2, k, c, chc, s);
    }
    return kqft_sde_matsubara(ctx, &V, &Gs, Nq, Nl, (double*)(gb + 3 * chc), stream);
  };
  auto residual = [&](double* res) { return rel_change(ctx, xf, counts, s, res); };
  if ((rc = fixed_point_core(ctx, stc, xb, gb, po, eval, residual, residuals, iterations, s))) return rc;
  for (int r = 0; r < 3; ++r) {
    double* dst[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(dst[c], cls(xb, r, c), cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(sigma, xsig, nf * sizeof(double2), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

static double flow_lambda(int reg, double t);
static double flow_t(int reg, double lam);
static double flow_dlambda_dt(int reg, double t);

// Cash-Karp embedded pair (Cash and Karp 1990): nodes, stage matrix, fifth- and fourth-order weights.
static const double kCkC[6] = {0.0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1.0, 7.0 / 8};
static const double kCkA[6][5] = {{0, 0, 0, 0, 0},
                                  {1.0 / 5, 0, 0, 0, 0},
                                  {3.0 / 40, 9.0 / 40, 0, 0, 0},
                                  {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
                                  {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
                                  {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}};
static const double kCkB5[6] = {37.0 / 378, 0.0, 250.0 / 621, 125.0 / 594, 0.0, 512.0 / 1771};
static const double kCkB4[6] = {2825.0 / 27648, 0.0, 18575.0 / 48384, 13525.0 / 55296, 277.0 / 14336, 1.0 / 4};

int kqft_mfrg_flow_matsubara(kqft_ctx* ctx, const kqft_mgrid* grid, double U, double Lambda_i, double Lambda_f,
                             int reg, double Delta, int steps, int nloops, int Nq, int Nl, int katanin, int se_iterations, double se_tol_abs,
                             double se_tol_rel, int adaptive, double ode_tol_abs, double ode_tol_rel, int max_steps,
                             const kqft_chout* gamma, double* sigma, double* lambdas, kqft_flow_info* info,
                             void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!grid || !gamma || !sigma) return fail(KQFT_EINVAL, "grid, gamma and sigma must be given");
  const kqft_mgrid g = *grid;
  if (g.M < 0 || g.N < 1 || Nq < 1 || Nl < 1) return fail(KQFT_ESHAPE, "need M >= 0, N >= 1, Nq >= 1, Nl >= 1");
  if (reg != KQFT_REG_DELTA && reg != KQFT_REG_U) return fail(KQFT_EINVAL, "the Matsubara flow runs in Delta or U");
  if (!(g.T > 0) || !(Lambda_i > 0) || !(Lambda_f > 0) || (reg == KQFT_REG_U && !(Delta > 0)))
    return fail(KQFT_EINVAL, "need T > 0, a positive flow parameter and Delta > 0");
  if (reg == KQFT_REG_DELTA && (Lambda_i > 1e6 || Lambda_f > 1e6))
    return fail(KQFT_EINVAL, "Delta-flow parameter beyond the reparametrisation's range");
  if (steps < 1 || nloops < 1) return fail(KQFT_EINVAL, "need steps >= 1 and nloops >= 1");
  if (se_iterations < 0 || !(se_tol_abs >= 0) || !(se_tol_rel >= 0))
    return fail(KQFT_EINVAL, "self-energy correction settings must be non-negative");
  if (adaptive != 0 && adaptive != 1) return fail(KQFT_EINVAL, "adaptive must be 0 or 1");
  if (adaptive && (max_steps < 1 || !(ode_tol_abs >= 0) || !(ode_tol_rel >= 0) || !(ode_tol_abs + ode_tol_rel > 0)))
    return fail(KQFT_EINVAL, "adaptive steps need max_steps >= 1 and positive tolerances");
  for (int r = 0; r < 3; ++r)
    if (!gamma[r].K1 || !gamma[r].K2 || !gamma[r].K2p || !gamma[r].K3)
      return fail(KQFT_EINVAL, "gamma arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const size_t nb = 2 * (size_t)g.M + 1, nf = 2 * (size_t)g.N;
  const size_t cnt[4] = {2 * nb, 2 * nb * nf, 2 * nb * nf, 2 * nb * nf * nf};
  const size_t chc = cnt[0] + cnt[1] + cnt[2] + cnt[3];
  const size_t stc = 3 * chc + nf;
  const bool corr = se_iterations > 0 && nloops >= 3;
  // states: Y, stage input, then the RK4 stage derivative and accumulator, or y4 and the six
  // Cash-Karp stage derivatives; insertions; centre sums; two scratch channels; Sigma-sized
  // work arrays; the step-error partial maxima
  const int nst = adaptive ? 9 : 4;
  const int nblk = (int)std::min<size_t>(1024, (stc + 255) / 256);
  const size_t total = (size_t)nst * stc + (size_t)nloops * 3 * chc + 2 * chc + 2 * chc + 6 * nf + nblk;
  if ((rc = ensure(ctx->mfflow, total * sizeof(double2)))) return rc;
  double2* base = (double2*)ctx->mfflow.p;
  double2 *Y = base, *yt = base + stc, *kd = base + 2 * stc, *ys = base + 3 * stc;
  double2* ml = base + (size_t)nst * stc;
  double2* cen = ml + (size_t)nloops * 3 * chc;
  double2 *t1 = cen + 2 * chc, *t2 = t1 + chc;
  double2* ax = t2 + chc;
  double2 *sd1 = ax, *tb = ax + nf, *sdt = ax + 2 * nf, *snew = ax + 3 * nf, *sdk = ax + 4 * nf;
  double* red = (double*)(ax + 6 * nf);
  kqft_flow_info inf;
  memset(&inf, 0, sizeof inf);
  int status = KQFT_OK;
  auto cls = [&](double2* b0, int c) {
    size_t off = 0;
    for (int u = 0; u < c; ++u) off += cnt[u];
    return b0 + off;
  };
  auto chout = [&](double2* b0) {
    return kqft_chout{(double*)b0, (double*)cls(b0, 1), (double*)cls(b0, 2), (double*)cls(b0, 3)};
  };
  auto chvert = [&](double coef, double2* b0) {
    return kqft_chvert{coef, (const double*)b0, (const double*)cls(b0, 1), (const double*)cls(b0, 2),
                       (const double*)cls(b0, 3)};
  };
  auto ins = [&](int l, int r) { return ml + ((size_t)l * 3 + r) * chc; };
  auto add_into = [&](double2* dst, const double2* src, size_t count) {
    const double2* k[2] = {dst, src};
    const double c[2] = {1.0, 1.0};
    lincomb_n(dst, nullptr, 2, k, c, count, s);
  };
  auto rhs = [&](double t, double2* yb, double2* kout) -> int {
    int e;
    const double lam = flow_lambda(reg, t);
    ++inf.rhs_evaluations;
    // the propagator at the flow parameter: Delta = lam, or G_0 -> lam G_0 at fixed Delta
    auto prop = [&](const double* sg, const double* dsg) {
      kqft_mprop p{reg == KQFT_REG_U ? Delta : lam, sg, g.N, dsg, reg, reg == KQFT_REG_U ? lam : 1.0};
      return p;
    };
    kqft_mvertex V;
    memset(&V, 0, sizeof V);
    V.grid = g;
    V.U = U;
    for (int r = 0; r < 3; ++r) V.ch[r] = chvert(1.0, yb + (size_t)r * chc);
    const kqft_mprop G = prop((const double*)(yb + 3 * chc), nullptr);
    // Sigma_dot^(1) = -L(Gamma, S)
    if ((e = kqft_loop_matsubara(ctx, &V, &G, KQFT_LINE_S, Nl, (double*)sd1, stream))) return e;
    launch_axpby(sd1, -1.0, sd1, 0.0, sd1, nf, s);
    launch_axpby(sdk, 1.0, sd1, 0.0, sd1, nf, s);
    for (int it = 0;;) {
      const kqft_mprop Gk = prop((const double*)(yb + 3 * chc), katanin ? (const double*)sdk : nullptr);
      for (int l = 0; l < nloops; ++l)
        for (int r = 0; r < 3; ++r) {
          const kqft_chout o = chout(ins(l, r));
          if (l == 0) {
            if ((e = kqft_bubble_matsubara(ctx, r, &V, &V, &Gk, KQFT_PI_DOT, Nq, 0, &o, stream))) return e;
            continue;
          }
          kqft_mvertex rbar;
          memset(&rbar, 0, sizeof rbar);
          rbar.grid = g;
          for (int r2 = 0; r2 < 3; ++r2)
            if (r2 != r) rbar.ch[r2] = chvert(1.0, ins(l - 1, r2));
          const kqft_chout o1 = chout(t1);
          if ((e = kqft_bubble_matsubara(ctx, r, &rbar, &V, &Gk, KQFT_PI_GG, Nq, 0, &o, stream))) return e;
          if ((e = kqft_bubble_matsubara(ctx, r, &V, &rbar, &Gk, KQFT_PI_GG, Nq, 0, &o1, stream))) return e;
          add_into(ins(l, r), t1, chc);
          if (l >= 2) {  // centre: B_r(Gamma, B_r(gdot_rbar^(l-2), Gamma))
            kqft_mvertex rbar2;
            memset(&rbar2, 0, sizeof rbar2);
            rbar2.grid = g;
            for (int r2 = 0; r2 < 3; ++r2)
              if (r2 != r) rbar2.ch[r2] = chvert(1.0, ins(l - 2, r2));
            const kqft_chout o2 = chout(t2);
            if ((e = kqft_bubble_matsubara(ctx, r, &rbar2, &V, &Gk, KQFT_PI_GG, Nq, 0, &o2, stream))) return e;
            kqft_mvertex inner;
            memset(&inner, 0, sizeof inner);
            inner.grid = g;
            inner.ch[r] = chvert(1.0, t2);
            if ((e = kqft_bubble_matsubara(ctx, r, &V, &inner, &Gk, KQFT_PI_GG, Nq, 0, &o1, stream))) return e;
            add_into(ins(l, r), t1, chc);
            if (corr && r < 2) {
              if (l == 2) {
                HIP_TRY(hipMemcpyAsync(cen + (size_t)r * chc, t1, chc * sizeof(double2), hipMemcpyDeviceToDevice, s));
              } else {
                add_into(cen + (size_t)r * chc, t1, chc);
              }
            }
          }
        }
      if (!corr) break;
      // Sigma_dot_tbar = -L(centre_a + centre_p, G); Sigma_dot_t = -L(Gamma, G Sigma_dot_tbar G)
      kqft_mvertex Vc;
      memset(&Vc, 0, sizeof Vc);
      Vc.grid = g;
      for (int r = 0; r < 2; ++r) Vc.ch[r] = chvert(1.0, cen + (size_t)r * chc);
      if ((e = kqft_loop_matsubara(ctx, &Vc, &G, KQFT_LINE_G, Nl, (double*)tb, stream))) return e;
      launch_axpby(tb, -1.0, tb, 0.0, tb, nf, s);
      const kqft_mprop Gt = prop((const double*)(yb + 3 * chc), (const double*)tb);
      if ((e = kqft_loop_matsubara(ctx, &V, &Gt, KQFT_LINE_GSG, Nl, (double*)sdt, stream))) return e;
      const double2* ks[2] = {tb, sdt};
      const double cs[2] = {1.0, -1.0};
      lincomb_n(snew, sd1, 2, ks, cs, nf, s);
      // max-norms of the change and of the new value (host, Sigma-sized)
      std::vector<double2> ha(nf), hb(nf);
      HIP_TRY(hipMemcpyAsync(ha.data(), sdk, nf * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(hb.data(), snew, nf * sizeof(double2), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double md = 0.0, mv = 0.0;
      for (size_t i = 0; i < nf; ++i) {
        md = std::max(md, std::hypot(hb[i].x - ha[i].x, hb[i].y - ha[i].y));
        mv = std::max(mv, std::hypot(hb[i].x, hb[i].y));
      }
      ++it;
      ++inf.se_iterations;
      launch_axpby(sdk, 1.0, snew, 0.0, snew, nf, s);
      if (md <= se_tol_abs + se_tol_rel * mv || it >= se_iterations) break;
    }
    // Gamma_dot = sum over the loop orders, Sigma_dot; times dLambda/dt
    const double dl = flow_dlambda_dt(reg, t);
    for (int r = 0; r < 3; ++r) {
      std::vector<const double2*> ks;
      std::vector<double> cs;
      for (int l = 0; l < nloops; ++l) {
        ks.push_back(ins(l, r));
        cs.push_back(dl);
      }
      lincomb_n(kout + (size_t)r * chc, nullptr, nloops, ks.data(), cs.data(), chc, s);
    }
    launch_axpby(kout + 3 * chc, dl, sdk, 0.0, sdk, nf, s);
    return KQFT_OK;
  };
  for (int r = 0; r < 3; ++r) {
    const double* src[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(cls(Y + (size_t)r * chc, c), src[c], cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(Y + 3 * chc, sigma, nf * sizeof(double2), hipMemcpyDeviceToDevice, s));
  const double ti = flow_t(reg, Lambda_i), tf = flow_t(reg, Lambda_f);
  int nrec = 0;
  auto record = [&](double t) {
    if (lambdas) lambdas[nrec] = flow_lambda(reg, t);
    ++nrec;
  };
  record(ti);
  const double h = (tf - ti) / steps;
  for (int k = 0; k < steps && !adaptive; ++k) {  // classical RK4
    const double ta = ti + k * h;
    const double2* kk[1] = {kd};
    double c[1];
    if ((rc = rhs(ta, Y, kd))) return rc;
    c[0] = h / 6.0;
    lincomb_n(ys, Y, 1, kk, c, stc, s);
    c[0] = h / 2.0;
    lincomb_n(yt, Y, 1, kk, c, stc, s);
    if ((rc = rhs(ta + h / 2.0, yt, kd))) return rc;
    c[0] = h / 3.0;
    lincomb_n(ys, ys, 1, kk, c, stc, s);
    c[0] = h / 2.0;
    lincomb_n(yt, Y, 1, kk, c, stc, s);
    if ((rc = rhs(ta + h / 2.0, yt, kd))) return rc;
    c[0] = h / 3.0;
    lincomb_n(ys, ys, 1, kk, c, stc, s);
    c[0] = h;
    lincomb_n(yt, Y, 1, kk, c, stc, s);
    if ((rc = rhs(ta + h, yt, kd))) return rc;
    c[0] = h / 6.0;
    lincomb_n(Y, ys, 1, kk, c, stc, s);
    ++inf.accepted;
    record(ti + (k + 1) * h);
  }
  if (adaptive) {  // Cash-Karp, advancing with the fourth-order solution (as the Keldysh flow)
    double2* y4 = base + 2 * stc;
    double2* K[6];
    for (int k = 0; k < 6; ++k) K[k] = base + (size_t)(3 + k) * stc;
    const double dir = tf >= ti ? 1.0 : -1.0;
    double t = ti, hh = (tf - ti) / steps;
    bool have_k1 = false, done = false;
    std::vector<double> hr(nblk);
    for (int trial = 0; trial < max_steps && !done; ++trial) {
      const bool last = (t + hh - tf) * dir >= 0.0;
      if (last) hh = tf - t;
      if (!have_k1) {
        if ((rc = rhs(t, Y, K[0]))) return rc;
        have_k1 = true;
      }
      for (int i = 1; i < 6; ++i) {
        double c[5];
        for (int j = 0; j < i; ++j) c[j] = hh * kCkA[i][j];
        lincomb_n(yt, Y, i, K, c, stc, s);
        if ((rc = rhs(t + kCkC[i] * hh, yt, K[i]))) return rc;
      }
      double c4[6], ce[6];
      for (int j = 0; j < 6; ++j) {
        c4[j] = hh * kCkB4[j];
        ce[j] = hh * (kCkB5[j] - kCkB4[j]);
      }
      lincomb_n(y4, Y, 6, K, c4, stc, s);
      lincomb_n(yt, nullptr, 6, K, ce, stc, s);
      launch_errnorm(yt, Y, y4, ode_tol_abs, ode_tol_rel, stc, red, nblk, s);
      HIP_TRY(hipMemcpyAsync(hr.data(), red, (size_t)nblk * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double err = 0.0;
      for (int b = 0; b < nblk; ++b) err = std::max(err, hr[b]);
      if (err <= 1.0) {
        std::swap(Y, y4);
        t = last ? tf : t + hh;
        have_k1 = false;
        ++inf.accepted;
        record(t);
        if (last) done = true;
        hh *= err == 0.0 ? 5.0 : std::min(5.0, 0.9 * pow(err, -0.2));
      } else {
        ++inf.rejected;
        hh *= std::max(0.1, 0.9 * pow(err, -0.25));
      }
    }
    if (!done) status = fail(KQFT_ENOCONV, "flow step limit reached before Lambda_f");
  }
  for (int r = 0; r < 3; ++r) {
    double* dst[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(dst[c], cls(Y + (size_t)r * chc, c), cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(sigma, Y + 3 * chc, nf * sizeof(double2), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipGetLastError());
  if (info) *info = inf;
  return status;
}

int kqft_loop(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, int kind, const kqft_quad* q,
              double* out, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!G || !q) return fail(KQFT_EINVAL, "propagator and quadrature must be given");
  if (q->n < 1 || (q->map != KQFT_QUAD_TAN_FINITE && q->map != KQFT_QUAD_TAN_INFINITE) ||
      (q->map == KQFT_QUAD_TAN_FINITE && !(q->L > 0)) || !(q->a > 0))
    return fail(KQFT_ESHAPE, "invalid quadrature");
  if (kind < KQFT_LINE_G || kind > KQFT_LINE_GSG) return fail(KQFT_EINVAL, "kind must be a KQFT_LINE_* value");
  if (kind == KQFT_LINE_GSG && !G->dSigR && G->deps == 0.0)
    return fail(KQFT_EINVAL, "the G Sigma_dot G line needs Sigma_dot");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!out) return fail(KQFT_EINVAL, "out is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  return vloop_core(ctx, *gamma, *G, kind, *q, out, (hipStream_t)stream);
}

static int mloop_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, const kqft_quad& q, int nloops,
                      kqft_opts o, const std::function<BubbleOut(int, int)>& dview, const BubbleOut* centre,
                      hipStream_t s, bool keep_last_left = false);

// <n_sigma> = 1/2 + (1/2 pi) sum_j w_j tanh(v_j/2T) Im G^R(v_j) at level E (Eq. Hartree with the
// spectral sum rule for the constant half); device partial sums, host total
static int occupation(kqft_ctx* ctx, const kqft_propagator& G, double E, const kqft_quad& q, hipStream_t s,
                      double* n_out) {
  int rc;
  const double *qv, *qw;
  if ((rc = get_quad(ctx, q, &qv, &qw))) return rc;
  kqft_propagator Ge = G;
  Ge.eps = E;
  DProp P;
  if ((rc = to_dprop(Ge, P))) return rc;
  const int nblk = std::max(1, std::min(64, (q.n + 255) / 256));
  if ((rc = ensure(ctx->flowred, std::max(ctx->flowred.bytes, (size_t)nblk * sizeof(double))))) return rc;
  double* part = (double*)ctx->flowred.p;
  launch_occupation(P, qv, qw, q.n, part, nblk, s);
  std::vector<double> h(nblk);
  HIP_TRY(hipMemcpyAsync(h.data(), part, (size_t)nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += h[b];
  *n_out = 0.5 + t / (2.0 * M_PI);
  return KQFT_OK;
}

// Hartree term, one shot (sigma_H in -> U n) or self-consistent by bisection on [0, U].
static int hartree_core(kqft_ctx* ctx, double U, double eps_d, const kqft_propagator& G, const kqft_quad& q,
                        bool self_consistent, double tol, double* sigma_H, int* evals, hipStream_t s) {
  int rc;
  double n = 0.0;
  int ev = 0;
  if (!self_consistent) {
    if ((rc = occupation(ctx, G, eps_d + *sigma_H, q, s, &n))) return rc;
    *sigma_H = U * n;
    ev = 1;
  } else {
    double lo = 0.0, hi = U;
    while (hi - lo > tol && ev < 200) {
      const double mid = 0.5 * (lo + hi);
      if ((rc = occupation(ctx, G, eps_d + mid, q, s, &n))) return rc;
      if (mid - U * n > 0.0)
        hi = mid;
      else
        lo = mid;
      ++ev;
    }
    *sigma_H = 0.5 * (lo + hi);
  }
  if (evals) *evals = ev;
  return KQFT_OK;
}

int kqft_hartree(kqft_ctx* ctx, double U, double eps_d, const kqft_propagator* G, const kqft_quad* q,
                 int self_consistent, double tol, double* sigma_H, int* iterations, void* stream) {
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!G || !q || !sigma_H) return fail(KQFT_EINVAL, "propagator, quadrature and sigma_H must be given");
  if (q->n < 1 || (q->map != KQFT_QUAD_TAN_FINITE && q->map != KQFT_QUAD_TAN_INFINITE) ||
      (q->map == KQFT_QUAD_TAN_FINITE && !(q->L > 0)) || !(q->a > 0))
    return fail(KQFT_ESHAPE, "invalid quadrature");
  if (G->reg != KQFT_REG_DELTA || G->dSigR || G->deps != 0.0)
    return fail(KQFT_EINVAL, "the Hartree term takes the plain propagator");
  if (!(U >= 0)) return fail(KQFT_EINVAL, "the bracketing needs U >= 0");
  if (self_consistent && !(tol > 0)) return fail(KQFT_EINVAL, "tol must be positive");
  HIP_TRY(hipSetDevice(ctx->device));
  return hartree_core(ctx, U, eps_d, *G, *q, self_consistent != 0, tol, sigma_H, iterations, (hipStream_t)stream);
}

// Flow parameter of the ODE (Sec. "Details on the ODE-solver"): the Delta-flow runs in t with
// Lambda(t) = 5 t|t| / sqrt(1 - t^2), the other flows in Lambda itself.
static double flow_lambda(int reg, double t) { return reg == KQFT_REG_DELTA ? 5.0 * t * fabs(t) / sqrt(1.0 - t * t) : t; }
static double flow_t(int reg, double lam) {
  if (reg != KQFT_REG_DELTA) return lam;
  const double l2 = lam * lam;  // 25 t^4 + Lambda^2 t^2 - Lambda^2 = 0
  return copysign(sqrt((-l2 + sqrt(l2 * l2 + 100.0 * l2)) / 50.0), lam);
}
static double flow_dlambda_dt(int reg, double t) {
  return reg == KQFT_REG_DELTA ? 5.0 * fabs(t) * (2.0 - t * t) / pow(1.0 - t * t, 1.5) : 1.0;
}

// Anderson step (Walker and Ni 2011) on a small host vector of interleaved complex values, over
// the real inner product: x_next = x + alpha f - sum_i gamma_i (dG_i - (1 - alpha) dF_i), f = g - x,
// with the columns of the last `depth` calls and gamma from the shifted normal equations.
struct HostAnderson {
  int depth;
  double alpha;
  std::vector<std::vector<double>> dF, dG;
  std::vector<double> fprev, gprev;
  bool has_prev = false;
  HostAnderson(int d, double a) : depth(d), alpha(a) {}
  bool step(const std::vector<double>& x, const std::vector<double>& g, std::vector<double>& out) {
    const size_t m = x.size();
    std::vector<double> f(m);
    for (size_t e = 0; e < m; ++e) f[e] = g[e] - x[e];
    if (depth > 0 && has_prev) {
      std::vector<double> a(m), b(m);
      for (size_t e = 0; e < m; ++e) {
        a[e] = f[e] - fprev[e];
        b[e] = g[e] - gprev[e];
      }
      dF.push_back(a);
      dG.push_back(b);
      if ((int)dF.size() > depth) {
        dF.erase(dF.begin());
        dG.erase(dG.begin());
      }
    }
    fprev = f;
    gprev = g;
    has_prev = true;
    out.resize(m);
    for (size_t e = 0; e < m; ++e) out[e] = x[e] + alpha * f[e];
    const int nc = (int)dF.size();
    if (nc == 0) return true;
    std::vector<double> A((size_t)nc * nc), bb(nc), gam;
    double dmax = 0.0;
    for (int i = 0; i < nc; ++i) {
      for (int j = 0; j < nc; ++j) {
        double t = 0.0;
        for (size_t e = 0; e < m; ++e) t += dF[i][e] * dF[j][e];
        A[(size_t)i * nc + j] = t;
      }
      double t = 0.0;
      for (size_t e = 0; e < m; ++e) t += dF[i][e] * f[e];
      bb[i] = t;
      dmax = std::max(dmax, A[(size_t)i * nc + i]);
    }
    for (int i = 0; i < nc; ++i) A[(size_t)i * nc + i] += 1e-14 * dmax;
    if (!solve_small(A, bb, nc, gam)) return false;
    for (int i = 0; i < nc; ++i)
      for (size_t e = 0; e < m; ++e) out[e] -= gam[i] * (dG[i][e] - (1.0 - alpha) * dF[i][e]);
    return true;
  }
};


int kqft_mfrg_flow(kqft_ctx* ctx, const kqft_grid* grid, double U, double T, double Lambda_i, double Lambda_f,
                   int steps, int nloops, const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                   const kqft_flow_opts* flow, const kqft_chout* gamma, double* sigma, double* lambdas,
                   kqft_flow_info* info, void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (!flow) return fail(KQFT_EINVAL, "flow options must be given");
  if (!grid || (rc = check_grid(*grid, "grid"))) return grid ? rc : fail(KQFT_EINVAL, "grid is NULL");
  const kqft_flow_opts fo = *flow;
  if (fo.reg < KQFT_REG_DELTA || fo.reg > KQFT_REG_NU) return fail(KQFT_EINVAL, "unknown regulator");
  const double Dphys = fo.reg == KQFT_REG_DELTA ? Lambda_i : fo.Delta;
  if (!(T > 0) || !(Dphys > 0)) return fail(KQFT_EINVAL, "T and Delta must be positive");
  if (!(Lambda_i > 0) || !(Lambda_f > 0)) return fail(KQFT_EINVAL, "the flow parameter must stay positive");
  if (fo.reg == KQFT_REG_DELTA && (Lambda_i > 1e6 || Lambda_f > 1e6))
    return fail(KQFT_EINVAL, "Delta-flow parameter beyond the reparametrisation's range");
  kqft_propagator Gc;
  memset(&Gc, 0, sizeof Gc);
  Gc.Delta = Dphys;
  Gc.T = T;
  Gc.sgrid = *grid;
  if ((rc = check_common(ctx, &Gc, q_bubble, opts))) return rc;
  if (!q_loop || q_loop->n < 1) return fail(KQFT_ESHAPE, "invalid loop quadrature");
  if (steps < 1 || nloops < 1) return fail(KQFT_EINVAL, "need steps >= 1 and nloops >= 1");
  if (fo.se_iterations < 0 || !(fo.se_tol_abs >= 0) || !(fo.se_tol_rel >= 0) || fo.se_anderson < 0 ||
      fo.se_anderson > 32)
    return fail(KQFT_EINVAL, "self-energy correction settings must be non-negative (Anderson depth <= 32)");
  if (fo.adaptive && (fo.max_steps < 1 || !(fo.ode_tol_abs >= 0) || !(fo.ode_tol_rel >= 0) ||
                      !(fo.ode_tol_abs + fo.ode_tol_rel > 0)))
    return fail(KQFT_EINVAL, "adaptive steps need max_steps >= 1 and positive tolerances");
  if (fo.asymmetric != 0 && fo.asymmetric != 1) return fail(KQFT_EINVAL, "asymmetric must be 0 or 1");
  const bool aam = fo.asymmetric == 1;
  if (aam && (!std::isfinite(fo.eps_d) || !std::isfinite(fo.sigma_inf)))
    return fail(KQFT_EINVAL, "eps_d and sigma_inf must be finite");
  if (!gamma || !sigma) return fail(KQFT_EINVAL, "gamma and sigma must be given");
  for (int r = 0; r < 3; ++r)
    if (!gamma[r].K1 || !gamma[r].K2 || !gamma[r].K2p || !gamma[r].K3)
      return fail(KQFT_EINVAL, "gamma arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = grid->n;
  const size_t c1 = (size_t)2 * n * 16, c2 = (size_t)2 * n * n * 16, c3 = (size_t)2 * n * n * n * 16;
  const size_t cnt[4] = {c1, c2, c2, c3};
  const size_t chc = c1 + 2 * c2 + c3;  // complex entries of one channel
  // of the state: channels a, p, t (K1, K2, K2', K3), Sigma, and Sigma_inf (asymmetric)
  const size_t stc = 3 * chc + (size_t)4 * n + (aam ? 1 : 0);
  const bool corr = fo.se_iterations > 0 && nloops >= 3;
  // states: Y, stage input, y4 and six stage derivatives (adaptive) or one (RK4) plus the
  // RK4 accumulator; then Sigma-sized work arrays and two centre sums
  const int nst = fo.adaptive ? 9 : 4;
  const size_t aux = (size_t)30 * n;
  if ((rc = ensure(ctx->flow, ((size_t)nst * stc + aux + (corr ? 2 * chc : 0)) * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx->flowml, (size_t)nloops * 3 * chc * sizeof(double2)))) return rc;
  const int nblk = (int)std::min<size_t>(1024, (stc + 255) / 256);
  if ((rc = ensure(ctx->flowred, (size_t)2 * nblk * sizeof(double)))) return rc;
  double2* buf = (double2*)ctx->flow.p;
  double2* st[9];
  for (int k = 0; k < nst; ++k) st[k] = buf + (size_t)k * stc;
  double2* ax = buf + (size_t)nst * stc;
  double2 *sigR = ax, *sigK = ax + n, *dsR = ax + 2 * n, *dsK = ax + 3 * n, *tR = ax + 4 * n, *tK = ax + 5 * n;
  double2 *sd1 = ax + 6 * n, *tb = ax + 10 * n, *sdt = ax + 14 * n, *snew = ax + 18 * n;
  double2 *stat = ax + 22 * n, *ra = ax + 26 * n;  // asymptotic loop, 1 on retarded and advanced
  double2* cen = ax + aux;
  double2* ml = (double2*)ctx->flowml.p;
  double* red = (double*)ctx->flowred.p;
  auto cls = [&](double2* base, int r, int c) {
    size_t off = (size_t)r * chc;
    for (int u = 0; u < c; ++u) off += cnt[u];
    return base + off;
  };
  auto sig_of = [&](double2* base) { return base + 3 * chc; };
  auto sinf_of = [&](double2* base) { return base + 3 * chc + (size_t)4 * n; };
  auto chan_view = [&](double2* b0) { return BubbleOut{b0, b0 + c1, b0 + c1 + c2, b0 + c1 + 2 * c2}; };
  auto lincomb = [&](double2* out, const double2* x, int nt, const double2* const* k, const double* c, size_t count) {
    LinComb a;
    memset(&a, 0, sizeof a);
    a.out = out;
    a.x = x;
    a.nt = nt;
    a.count = count;
    for (int j = 0; j < nt; ++j) {
      a.k[j] = k[j];
      a.c[j] = c[j];
    }
    launch_lincomb(a, s);
  };
  // max-norms (change, value) of f - x and f over count entries, on the host
  auto maxdiff = [&](const double2* x, const double2* f, size_t count, double& md, double& mf) -> int {
    const int nb = (int)std::min<size_t>(1024, (count + 255) / 256);
    launch_maxdiff(x, f, count, red, nb, s);
    std::vector<double> h((size_t)2 * nb);
    HIP_TRY(hipMemcpyAsync(h.data(), red, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    md = mf = 0.0;
    for (int b = 0; b < nb; ++b) {
      md = std::max(md, h[2 * (size_t)b]);
      mf = std::max(mf, h[2 * (size_t)b + 1]);
    }
    return KQFT_OK;
  };
  auto read_real = [&](const double2* p, double* out) -> int {
    double2 h;
    HIP_TRY(hipMemcpyAsync(&h, p, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = h.x;
    return KQFT_OK;
  };
  auto write_real = [&](double2* p, double v) -> int {
    const double2 h = make_double2(v, 0.0);
    HIP_TRY(hipMemcpyAsync(p, &h, sizeof h, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return KQFT_OK;
  };
  // asymptotic value of -L(V, X): the loop of the bare vertex and K1_t, K2_t of V (the part
  // that does not depend on the external frequency in the loop's legs); ds = its real
  // retarded component, the same at every grid point (read at the first)
  auto static_part = [&](const kqft_vertex& V, const kqft_propagator& Gx, int kind, double* ds) -> int {
    int e;
    kqft_vertex Vs;
    memset(&Vs, 0, sizeof Vs);
    Vs.r0 = V.r0;
    Vs.grid = V.grid;
    const kqft_chvert& t = V.ch[KQFT_CH_T];
    Vs.ch[KQFT_CH_T] = kqft_chvert{t.coef, t.K1, t.K2, nullptr, nullptr};
    if ((e = vloop_core(ctx, Vs, Gx, kind, *q_loop, (double*)stat, s))) return e;
    double v;
    if ((e = read_real(stat + 1, &v))) return e;
    *ds = -v;
    return KQFT_OK;
  };
  if (aam) {
    std::vector<double2> h((size_t)4 * n);
    for (int i = 0; i < n; ++i) {
      h[4 * (size_t)i] = h[4 * (size_t)i + 3] = make_double2(0.0, 0.0);
      h[4 * (size_t)i + 1] = h[4 * (size_t)i + 2] = make_double2(1.0, 0.0);
    }
    HIP_TRY(hipMemcpyAsync(ra, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  kqft_flow_info inf;
  memset(&inf, 0, sizeof inf);
  // derivative dY/dt of the state yb at flow time t into kout
  auto rhs = [&](double t, double2* yb, double2* kout) -> int {
    int e;
    const double lam = flow_lambda(fo.reg, t);
    ++inf.rhs_evaluations;
    launch_sigma_split(n, sig_of(yb), sigR, sigK, s);
    kqft_propagator G;
    memset(&G, 0, sizeof G);
    G.Delta = fo.reg == KQFT_REG_DELTA ? lam : fo.Delta;
    G.T = fo.reg == KQFT_REG_T ? lam : T;
    G.reg = fo.reg;
    G.lam = (fo.reg == KQFT_REG_U || fo.reg == KQFT_REG_NU) ? lam : 1.0;
    G.sgrid = *grid;
    G.SigR = (const double*)sigR;
    G.SigK = (const double*)sigK;
    if (aam) {
      double si;
      if ((e = read_real(sinf_of(yb), &si))) return e;
      G.eps = fo.eps_d + si;
    }
    kqft_vertex V;
    memset(&V, 0, sizeof V);
    V.r0 = U;
    V.grid = *grid;
    for (int r = 0; r < 3; ++r)
      V.ch[r] = kqft_chvert{1.0, (const double*)cls(yb, r, 0), (const double*)cls(yb, r, 1),
                            (const double*)cls(yb, r, 2), (const double*)cls(yb, r, 3)};
    auto dview = [&](int l, int r) { return chan_view(ml + ((size_t)l * 3 + r) * chc); };
    double2* sd = sig_of(kout);
    // one-loop self-energy flow Sigma_dot^(1) = -L(Gamma, S)
    if ((e = vloop_core(ctx, V, G, KQFT_LINE_S, *q_loop, (double*)sd1, s))) return e;
    launch_axpby(sd1, -1.0, sd1, 0.0, sd1, (size_t)4 * n, s);
    double ds1 = 0.0, ds = 0.0;  // d Sigma_inf (asymmetric)
    if (aam) {
      if ((e = static_part(V, G, KQFT_LINE_S, &ds1))) return e;
      const double2* kr[1] = {ra};
      const double cr[1] = {-ds1};
      lincomb(sd1, sd1, 1, kr, cr, (size_t)4 * n);
      ds = ds1;
    }
    launch_axpby(sd, 1.0, sd1, 0.0, sd1, (size_t)4 * n, s);
    BubbleOut centre[2] = {chan_view(cen), chan_view(cen + chc)};
    HostAnderson mixer(fo.se_anderson, 1.0);
    for (int it = 0;;) {
      kqft_propagator Gk = G;
      if (fo.katanin) {
        launch_sigma_split(n, sd, dsR, dsK, s);
        Gk.dSigR = (const double*)dsR;
        Gk.dSigK = (const double*)dsK;
        Gk.deps = ds;
      }
      if ((e = mloop_core(ctx, V, Gk, *q_bubble, nloops, *opts, dview, corr ? centre : nullptr, s))) return e;
      if (!corr) break;
      // Sigma_dot_tbar = -L(centre_a + centre_p, G); Sigma_dot_t = -L(Gamma, G Sigma_dot_tbar G)
      kqft_vertex Vc;
      memset(&Vc, 0, sizeof Vc);
      Vc.grid = *grid;
      for (int r = 0; r < 2; ++r)
        Vc.ch[r] = kqft_chvert{1.0, (const double*)centre[r].K1, (const double*)centre[r].K2,
                               (const double*)centre[r].K2p, (const double*)centre[r].K3};
      if ((e = vloop_core(ctx, Vc, G, KQFT_LINE_G, *q_loop, (double*)tb, s))) return e;
      launch_axpby(tb, -1.0, tb, 0.0, tb, (size_t)4 * n, s);
      launch_sigma_split(n, tb, tR, tK, s);
      kqft_propagator Gt = G;
      Gt.dSigR = (const double*)tR;
      Gt.dSigK = (const double*)tK;
      if ((e = vloop_core(ctx, V, Gt, KQFT_LINE_GSG, *q_loop, (double*)sdt, s))) return e;
      double dst = 0.0;  // asymptotic part of Sigma_dot_t (the centre-term loop has none)
      if (aam && (e = static_part(V, Gt, KQFT_LINE_GSG, &dst))) return e;
      const double2* ks[3] = {tb, sdt, ra};
      const double cs[3] = {1.0, -1.0, -dst};
      lincomb(snew, sd1, aam ? 3 : 2, ks, cs, (size_t)4 * n);
      const double dnew = ds1 + dst;
      double md, mf;
      if ((e = maxdiff(sd, snew, (size_t)4 * n, md, mf))) return e;
      if (aam) {
        md = std::max(md, fabs(dnew - ds));
        mf = std::max(mf, fabs(dnew));
      }
      ++it;
      ++inf.se_iterations;
      if (md <= fo.se_tol_abs + fo.se_tol_rel * mf || it >= fo.se_iterations || fo.se_anderson == 0) {
        launch_axpby(sd, 1.0, snew, 0.0, snew, (size_t)4 * n, s);
        ds = dnew;
        if (md <= fo.se_tol_abs + fo.se_tol_rel * mf || it >= fo.se_iterations) break;
        continue;
      }
      // Anderson step on the host (4n complex values, and d Sigma_inf)
      const size_t m = (size_t)8 * n + (aam ? 2 : 0);
      std::vector<double> hx(m), hg(m), hn;
      HIP_TRY(hipMemcpyAsync(hx.data(), sd, (size_t)8 * n * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(hg.data(), snew, (size_t)8 * n * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (aam) {
        hx[8 * (size_t)n] = ds;
        hg[8 * (size_t)n] = dnew;
        hx[8 * (size_t)n + 1] = hg[8 * (size_t)n + 1] = 0.0;
      }
      if (!mixer.step(hx, hg, hn)) return fail(KQFT_ENOCONV, "singular Anderson system in the self-energy corrections");
      if (aam) ds = hn[8 * (size_t)n];
      HIP_TRY(hipMemcpyAsync(sd, hn.data(), (size_t)8 * n * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    // Gamma_dot = sum over the loop orders; everything times dLambda/dt
    const double dl = flow_dlambda_dt(fo.reg, t);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 4; ++c) {
        double2* dst = cls(kout, r, c);
        for (int l0 = 0; l0 < nloops; l0 += 6) {
          const int nt = std::min(6, nloops - l0);
          const double2* ks[6];
          double cs[6];
          for (int j = 0; j < nt; ++j) {
            ks[j] = cls(ml + (size_t)(l0 + j) * 3 * chc, r, c);
            cs[j] = dl;
          }
          lincomb(dst, l0 == 0 ? nullptr : dst, nt, ks, cs, cnt[c]);
        }
      }
    if (dl != 1.0) launch_axpby(sd, dl, sd, 0.0, sd, (size_t)4 * n, s);
    if (aam && (e = write_real(sinf_of(kout), dl * ds))) return e;
    return KQFT_OK;
  };
  // the user's state into Y
  double2* Y = st[0];
  for (int r = 0; r < 3; ++r) {
    const double* src[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(cls(Y, r, c), src[c], cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(sig_of(Y), sigma, (size_t)4 * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (aam && (rc = write_real(sinf_of(Y), fo.sigma_inf))) return rc;
  const double ti = flow_t(fo.reg, Lambda_i), tf = flow_t(fo.reg, Lambda_f);
  int nl = 0;
  auto record = [&](double t) {
    if (lambdas) lambdas[nl] = flow_lambda(fo.reg, t);
    ++nl;
  };
  record(ti);
  int status = KQFT_OK;
  if (!fo.adaptive) {
    double2 *yt = st[1], *kd = st[2], *ys = st[3];
    const double h = (tf - ti) / steps;
    for (int k = 0; k < steps; ++k) {
      const double ta = ti + k * h;
      const double2* kk[1] = {kd};
      double c[1];
      if ((rc = rhs(ta, Y, kd))) return rc;
      c[0] = h / 6.0;
      lincomb(ys, Y, 1, kk, c, stc);
      c[0] = h / 2.0;
      lincomb(yt, Y, 1, kk, c, stc);
      if ((rc = rhs(ta + h / 2.0, yt, kd))) return rc;
      c[0] = h / 3.0;
      lincomb(ys, ys, 1, kk, c, stc);
      c[0] = h / 2.0;
      lincomb(yt, Y, 1, kk, c, stc);
      if ((rc = rhs(ta + h / 2.0, yt, kd))) return rc;
      c[0] = h / 3.0;
      lincomb(ys, ys, 1, kk, c, stc);
      c[0] = h;
      lincomb(yt, Y, 1, kk, c, stc);
      if ((rc = rhs(ta + h, yt, kd))) return rc;
      c[0] = h / 6.0;
      lincomb(Y, ys, 1, kk, c, stc);
      ++inf.accepted;
      record(ti + (k + 1) * h);
    }
  } else {
    double2 *yt = st[1], *y4 = st[2], *K[6];
    for (int k = 0; k < 6; ++k) K[k] = st[3 + k];
    const double dir = tf >= ti ? 1.0 : -1.0;
    double t = ti, h = (tf - ti) / steps;
    bool have_k1 = false, done = false;
    std::vector<double> hr(nblk);
    for (int trial = 0; trial < fo.max_steps && !done; ++trial) {
      const bool last = (t + h - tf) * dir >= 0.0;
      if (last) h = tf - t;
      if (!have_k1) {
        if ((rc = rhs(t, Y, K[0]))) return rc;
        have_k1 = true;
      }
      for (int i = 1; i < 6; ++i) {
        double c[5];
        for (int j = 0; j < i; ++j) c[j] = h * kCkA[i][j];
        lincomb(yt, Y, i, K, c, stc);
        if ((rc = rhs(t + kCkC[i] * h, yt, K[i]))) return rc;
      }
      double c4[6], ce[6];
      for (int j = 0; j < 6; ++j) {
        c4[j] = h * kCkB4[j];
        ce[j] = h * (kCkB5[j] - kCkB4[j]);
      }
      lincomb(y4, Y, 6, K, c4, stc);
      lincomb(yt, nullptr, 6, K, ce, stc);
      launch_errnorm(yt, Y, y4, fo.ode_tol_abs, fo.ode_tol_rel, stc, red, nblk, s);
      HIP_TRY(hipMemcpyAsync(hr.data(), red, (size_t)nblk * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double err = 0.0;
      for (int b = 0; b < nblk; ++b) err = std::max(err, hr[b]);
      if (err <= 1.0) {
        std::swap(Y, y4);
        st[2] = y4;
        t = last ? tf : t + h;
        have_k1 = false;
        ++inf.accepted;
        record(t);
        if (last) done = true;
        h *= err == 0.0 ? 5.0 : std::min(5.0, 0.9 * pow(err, -0.2));
      } else {
        ++inf.rejected;
        h *= std::max(0.1, 0.9 * pow(err, -0.25));
      }
    }
    if (!done) status = fail(KQFT_ENOCONV, "flow step limit reached before Lambda_f");
  }
  // Y back to the user's arrays
  for (int r = 0; r < 3; ++r) {
    double* dst[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(dst[c], cls(Y, r, c), cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(sigma, sig_of(Y), (size_t)4 * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (aam && (rc = read_real(sinf_of(Y), &inf.sigma_inf))) return rc;
  HIP_TRY(hipGetLastError());
  if (info) *info = inf;
  return status;
}

int kqft_parquet_iteration(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G,
                           const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                           const kqft_chout* gamma_out, double* sigma_out, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q_bubble, opts))) return rc;
  if (!q_loop || q_loop->n < 1) return fail(KQFT_ESHAPE, "invalid loop quadrature");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!gamma_out || !sigma_out) return fail(KQFT_EINVAL, "gamma_out and sigma_out must be given");
  for (int r = 0; r < 3; ++r)
    if (!gamma_out[r].K1 || !gamma_out[r].K2 || !gamma_out[r].K2p || !gamma_out[r].K3)
      return fail(KQFT_EINVAL, "gamma_out arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  BubbleOut out[3];
  for (int r = 0; r < 3; ++r)
    out[r] = BubbleOut{(double2*)gamma_out[r].K1, (double2*)gamma_out[r].K2, (double2*)gamma_out[r].K2p,
                       (double2*)gamma_out[r].K3};
  return parquet_core(ctx, *gamma, *G, *q_bubble, *q_loop, *opts, out, sigma_out, (hipStream_t)stream);
}

// Fixed-point iteration x = F(x) of a device state vector of stc complex entries (Sec. parquet
// solver): per iteration eval() writes g = F(x) for x = xb and residual() returns the relative
// change; then x <- x + alpha f - sum_i gamma_i (dG_i - (1 - alpha) dF_i), f = g - x, with the
// Anderson columns of the last m iterations and gamma from the shifted normal equations over
// the real inner product; a growing residual halves alpha (reduce_alpha) and clears the
// columns.  xb holds x, f, the previous f and g and the 2m columns (stc entries each).
static int fixed_point_core(kqft_ctx* ctx, size_t stc, double2* xb, double2* g, const kqft_parquet_opts& po,
                            const std::function<int()>& eval, const std::function<int(double*)>& residual,
                            double* residuals, int* iterations, hipStream_t s) {
  int rc;
  const int m = po.anderson_depth;
  double2 *fr = xb + stc, *fprev = xb + 2 * stc, *gprev = xb + 3 * stc;
  std::vector<double2*> dF(m), dG(m);
  for (int i = 0; i < m; ++i) {
    dF[i] = xb + (size_t)(4 + i) * stc;
    dG[i] = xb + (size_t)(4 + m + i) * stc;
  }
  double alpha = po.alpha, prev_res = 0.0;
  int ncol = 0, head = 0, it = 0;
  bool have_prev = false;
  for (; it < po.max_iterations;) {
    if ((rc = eval())) return rc;
    double res = 0.0;
    if ((rc = residual(&res))) return rc;
    {  // f = g - x
      const double2* k[2] = {g, xb};
      const double c[2] = {1.0, -1.0};
      lincomb_n(fr, nullptr, 2, k, c, stc, s);
    }
    if (po.reduce_alpha && it > 0 && res > prev_res) {
      alpha = std::max(0.5 * alpha, po.alpha_min);
      ncol = 0;
    } else if (m > 0 && have_prev) {  // newest columns dF = f - f_prev, dG = g - g_prev
      const int slot = head % m;
      const double2* k[2] = {fr, fprev};
      const double c[2] = {1.0, -1.0};
      lincomb_n(dF[slot], nullptr, 2, k, c, stc, s);
      const double2* kg[2] = {g, gprev};
      lincomb_n(dG[slot], nullptr, 2, kg, c, stc, s);
      ++head;
      ncol = std::min(ncol + 1, m);
    }
    if (m > 0) {
      HIP_TRY(hipMemcpyAsync(fprev, fr, stc * sizeof(double2), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(gprev, g, stc * sizeof(double2), hipMemcpyDeviceToDevice, s));
      have_prev = true;
    }
    // x <- x + alpha f - sum_i gamma_i (dG_i - (1 - alpha) dF_i)
    std::vector<const double2*> ks{fr};
    std::vector<double> cs{alpha};
    if (ncol > 0) {
      std::vector<int> cols;
      for (int i = 0; i < ncol; ++i) cols.push_back((head - ncol + i) % m);  // oldest first
      std::vector<std::pair<const double2*, const double2*>> ab;
      for (int i = 0; i < ncol; ++i)
        for (int j = 0; j <= i; ++j) ab.push_back({dF[cols[i]], dF[cols[j]]});
      for (int i = 0; i < ncol; ++i) ab.push_back({dF[cols[i]], fr});
      std::vector<double> d;
      if ((rc = dots(ctx, ab, stc, s, d))) return rc;
      std::vector<double> A((size_t)ncol * ncol), b(ncol), gam;
      size_t q = 0;
      for (int i = 0; i < ncol; ++i)
        for (int j = 0; j <= i; ++j, ++q) A[(size_t)i * ncol + j] = A[(size_t)j * ncol + i] = d[q];
      double dmax = 0.0;
      for (int i = 0; i < ncol; ++i) {
        b[i] = d[q + i];
        dmax = std::max(dmax, A[(size_t)i * ncol + i]);
      }
      for (int i = 0; i < ncol; ++i) A[(size_t)i * ncol + i] += 1e-14 * dmax;
      if (!solve_small(A, b, ncol, gam)) return fail(KQFT_ENOCONV, "singular Anderson system");
      for (int i = 0; i < ncol; ++i) {
        ks.push_back(dG[cols[i]]);
        cs.push_back(-gam[i]);
        ks.push_back(dF[cols[i]]);
        cs.push_back(gam[i] * (1.0 - alpha));
      }
    }
    lincomb_n(xb, xb, (int)ks.size(), ks.data(), cs.data(), stc, s);
    if (residuals) residuals[it] = res;
    prev_res = res;
    ++it;
    if (res < po.tol) break;
  }
  *iterations = it;
  return KQFT_OK;
}

int kqft_parquet_solve(kqft_ctx* ctx, const kqft_grid* grid, double U, double Delta, double T,
                       const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                       const kqft_parquet_opts* popts, const kqft_chout* gamma, double* sigma, double* sigma_H,
                       double* residuals, int* iterations, void* stream) {
  int rc;
  if (!grid || (rc = check_grid(*grid, "grid"))) return grid ? rc : fail(KQFT_EINVAL, "grid is NULL");
  kqft_propagator G0;
  memset(&G0, 0, sizeof G0);
  G0.Delta = Delta;
  G0.T = T;
  G0.sgrid = *grid;
  if ((rc = check_common(ctx, &G0, q_bubble, opts))) return rc;
  if (!q_loop || q_loop->n < 1) return fail(KQFT_ESHAPE, "invalid loop quadrature");
  if (!(Delta > 0) || !(T > 0)) return fail(KQFT_EINVAL, "Delta and T must be positive");
  if (!popts) return fail(KQFT_EINVAL, "solver options must be given");
  const kqft_parquet_opts po = *popts;
  if (!(po.alpha > 0) || po.alpha > 1 || po.max_iterations < 1)
    return fail(KQFT_EINVAL, "need 0 < alpha <= 1, max_iterations >= 1");
  if (po.anderson_depth < 0 || po.anderson_depth > 32) return fail(KQFT_EINVAL, "need 0 <= anderson_depth <= 32");
  if (po.reduce_alpha && (!(po.alpha_min > 0) || po.alpha_min > po.alpha))
    return fail(KQFT_EINVAL, "need 0 < alpha_min <= alpha");
  if (po.sde_forms != 0 && po.sde_forms != 1 && po.sde_forms != 3) return fail(KQFT_EINVAL, "sde_forms must be 1 or 3");
  const int forms = po.sde_forms == 3 ? 3 : 1;
  const bool aam = po.hartree != 0;
  if (aam) {
    const kqft_quad& qh = po.q_hartree;
    if (qh.n < 1 || (qh.map != KQFT_QUAD_TAN_FINITE && qh.map != KQFT_QUAD_TAN_INFINITE) ||
        (qh.map == KQFT_QUAD_TAN_FINITE && !(qh.L > 0)) || !(qh.a > 0))
      return fail(KQFT_ESHAPE, "invalid Hartree quadrature");
    if (!(U >= 0) || !(po.hartree_tol > 0)) return fail(KQFT_EINVAL, "the Hartree term needs U >= 0 and tol > 0");
  }
  if (!gamma || !sigma || !iterations) return fail(KQFT_EINVAL, "gamma, sigma and iterations must be given");
  for (int r = 0; r < 3; ++r)
    if (!gamma[r].K1 || !gamma[r].K2 || !gamma[r].K2p || !gamma[r].K3)
      return fail(KQFT_EINVAL, "gamma arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = grid->n, m = po.anderson_depth;
  const size_t c1 = (size_t)2 * n * 16, c2 = (size_t)2 * n * n * 16, c3 = (size_t)2 * n * n * n * 16;
  const size_t cnt[4] = {c1, c2, c2, c3};
  const size_t chc = c1 + 2 * c2 + c3;
  // state: channels a, p, t (K1, K2, K2', K3), Sigma, and Sigma_H for the asymmetric model
  const size_t stc = 3 * chc + (size_t)4 * n + (aam ? 1 : 0);
  // g = F(x) in pq; x, f, the previous f and g, and 2m Anderson columns in pqx
  if ((rc = ensure(ctx->pq, stc * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx->pqx, (size_t)(4 + 2 * m) * stc * sizeof(double2)))) return rc;
  if ((rc = ensure(ctx->pqsig, (size_t)2 * n * sizeof(double2)))) return rc;
  double2* g = (double2*)ctx->pq.p;
  double2* xb = (double2*)ctx->pqx.p;
  auto cls = [&](double2* base, int r, int c) {
    size_t off = (size_t)r * chc;
    for (int u = 0; u < c; ++u) off += cnt[u];
    return base + off;
  };
  auto chan_out = [&](double2* base, int r) {
    return BubbleOut{cls(base, r, 0), cls(base, r, 1), cls(base, r, 2), cls(base, r, 3)};
  };
  double2* xsig = xb + 3 * chc;
  double2* sigR = (double2*)ctx->pqsig.p;
  double2* sigK = sigR + n;
  // PT2 start: K1_r = B_r(Gamma_0, Gamma_0), Sigma^(2) = SDE(Gamma_0) with the bare propagator
  kqft_vertex bare;
  memset(&bare, 0, sizeof bare);
  bare.r0 = U;
  bare.grid = *grid;
  for (int r = 0; r < 3; ++r)
    for (int c = 1; c < 4; ++c) HIP_TRY(hipMemsetAsync(cls(xb, r, c), 0, cnt[c] * sizeof(double2), s));
  double sH = 0.5 * U;
  if (aam) {  // self-consistent Hartree term of the bare level, into the state
    if ((rc = hartree_core(ctx, U, po.eps_d, G0, po.q_hartree, true, po.hartree_tol, &sH, nullptr, s))) return rc;
    G0.eps = po.eps_d + sH;
    const double2 hv = make_double2(sH, 0.0);
    HIP_TRY(hipMemcpyAsync(xsig + 4 * n, &hv, sizeof hv, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  kqft_opts o = *opts;
  o.beta = 0;
  o.class_mask = KQFT_K1;
  for (int r = 0; r < 3; ++r) {
    BubbleOut k1{cls(xb, r, 0), nullptr, nullptr, nullptr};
    if ((rc = bubble_core(ctx, r, bare, bare, G0, KQFT_PI_GG, *q_bubble, o, k1, s))) return rc;
  }
  G0.sgrid = kqft_grid{2, 1.0, 1.0};
  if ((rc = sde_core(ctx, &bare, &G0, q_bubble, q_loop, opts, (double*)xsig, nullptr, s))) return rc;
  kqft_vertex V;
  memset(&V, 0, sizeof V);
  V.r0 = U;
  V.grid = *grid;
  for (int r = 0; r < 3; ++r)
    V.ch[r] = kqft_chvert{1.0, (const double*)cls(xb, r, 0), (const double*)cls(xb, r, 1),
                          (const double*)cls(xb, r, 2), (const double*)cls(xb, r, 3)};
  kqft_propagator Gs;
  memset(&Gs, 0, sizeof Gs);
  Gs.Delta = Delta;
  Gs.T = T;
  Gs.sgrid = *grid;
  Gs.SigR = (const double*)sigR;
  Gs.SigK = (const double*)sigK;
  BubbleOut F[3] = {chan_out(g, 0), chan_out(g, 1), chan_out(g, 2)};
  std::vector<std::pair<const double2*, const double2*>> xf;
  std::vector<size_t> counts;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      xf.push_back({cls(xb, r, c), cls(g, r, c)});
      counts.push_back(cnt[c]);
    }
  xf.push_back({xsig, g + 3 * chc});
  counts.push_back((size_t)n * 4);
  if (aam) {
    xf.push_back({xsig + 4 * n, g + 3 * chc + 4 * n});
    counts.push_back(1);
  }
  auto eval = [&]() -> int {
    launch_sigma_split(n, xsig, sigR, sigK, s);
    if (aam) {  // the state's Hartree term sets the level
      double2 hv;
      HIP_TRY(hipMemcpyAsync(&hv, xsig + 4 * n, sizeof hv, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      Gs.eps = po.eps_d + hv.x;
      double h = hv.x;
      kqft_propagator Gh = Gs;
      if ((rc = hartree_core(ctx, U, po.eps_d, Gh, po.q_hartree, false, 0.0, &h, nullptr, s))) return rc;
      const double2 hn = make_double2(h, 0.0);
      HIP_TRY(hipMemcpyAsync(g + 3 * chc + 4 * n, &hn, sizeof hn, hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    if ((rc = parquet_core(ctx, V, Gs, *q_bubble, *q_loop, *opts, F, (double*)(g + 3 * chc), s, forms))) return rc;
    return KQFT_OK;
  };
  auto residual = [&](double* res) { return rel_change(ctx, xf, counts, s, res); };
  if ((rc = fixed_point_core(ctx, stc, xb, g, po, eval, residual, residuals, iterations, s))) return rc;
  // the state back into the caller's arrays
  for (int r = 0; r < 3; ++r) {
    double* dst[4] = {gamma[r].K1, gamma[r].K2, gamma[r].K2p, gamma[r].K3};
    for (int c = 0; c < 4; ++c)
      HIP_TRY(hipMemcpyAsync(dst[c], cls(xb, r, c), cnt[c] * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(sigma, xsig, (size_t)4 * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (aam) {
    double2 hv;
    HIP_TRY(hipMemcpyAsync(&hv, xsig + 4 * n, sizeof hv, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    sH = hv.x;
  }
  if (sigma_H) *sigma_H = sH;
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

// Multiloop insertions of one parameter point into dview(l - 1, r) (Eqs. 1l, 2l, 3l).  With
// `centre` (two outputs, channels a and p), the centre terms of those channels are also
// summed over l >= 3 into centre[0], centre[1] (written when nloops >= 3).  dview(l - 1, .)
// is read only while order l + 1 is formed, so a caller may map the orders onto two
// alternating buffers.  keep_last_left: the left insertions of the last order (nloops >= 2)
// stay in ctx->lstore[nloops & 1] as well.
static int mloop_core(kqft_ctx* ctx, const kqft_vertex& V, const kqft_propagator& G, const kqft_quad& q, int nloops,
                      kqft_opts o, const std::function<BubbleOut(int, int)>& dview, const BubbleOut* centre,
                      hipStream_t s, bool keep_last_left) {
  int rc;
  o.class_mask = KQFT_KALL;
  const int n = V.grid.n;
  const size_t c1 = (size_t)2 * n * 16, c2 = (size_t)2 * n * n * 16, c3 = (size_t)2 * n * n * n * 16;
  const size_t s1 = c1 * sizeof(double2), s2 = c2 * sizeof(double2), s3 = c3 * sizeof(double2);
  const size_t chb = s1 + 2 * s2 + s3;
  // left insertions of the previous and the current order, per channel
  if (nloops >= 3 || (keep_last_left && nloops >= 2))
    for (int x = 0; x < 2; ++x)
      for (int r = 0; r < 3; ++r)
        if ((rc = ensure(ctx->lstore[x][r], chb))) return rc;
  if (centre && nloops >= 3 && (rc = ensure(ctx->ctmp, chb))) return rc;
  auto view_of = [&](void* p) {
    char* b = (char*)p;
    return BubbleOut{(double2*)b, (double2*)(b + s1), (double2*)(b + s1 + s2), (double2*)(b + s1 + 2 * s2)};
  };
  // out = a x + b y, class by class
  auto comb = [&](const BubbleOut& out, double a, const BubbleOut& x, double b, const BubbleOut& y) {
    launch_axpby(out.K1, a, x.K1, b, y.K1, c1, s);
    launch_axpby(out.K2, a, x.K2, b, y.K2, c2, s);
    launch_axpby(out.K2p, a, x.K2p, b, y.K2p, c2, s);
    launch_axpby(out.K3, a, x.K3, b, y.K3, c3, s);
  };
  for (int l = 1; l <= nloops; ++l) {
    const int cur = l & 1, prev = cur ^ 1;
    for (int r = 0; r < 3; ++r) {
      BubbleOut dst = dview(l - 1, r);
      if (l == 1) {
        o.beta = 0;
        if ((rc = bubble_core(ctx, r, V, V, G, KQFT_PI_DOT, q, o, dst, s))) return rc;
        continue;
      }
      kqft_vertex rbar;
      memset(&rbar, 0, sizeof rbar);
      rbar.grid = V.grid;
      for (int r2 = 0; r2 < 3; ++r2) {
        if (r2 == r) continue;
        const BubbleOut d = dview(l - 2, r2);
        rbar.ch[r2] = kqft_chvert{1.0, (const double*)d.K1, (const double*)d.K2, (const double*)d.K2p,
                                  (const double*)d.K3};
      }
      // left insertion: into dst, and kept for the next order's centre term
      o.beta = 0;
      if ((rc = bubble_core(ctx, r, rbar, V, G, KQFT_PI_GG, q, o, dst, s))) return rc;
      if ((l + 1 <= nloops || keep_last_left) && l >= 2) {
        BubbleOut lv = view_of(ctx->lstore[cur][r].p);
        HIP_TRY(hipMemcpyAsync(lv.K1, dst.K1, s1, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(lv.K2, dst.K2, s2, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(lv.K2p, dst.K2p, s2, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(lv.K3, dst.K3, s3, hipMemcpyDeviceToDevice, s));
      }
      o.beta = 1;
      const bool own_centre = l >= 3 && centre && r < 2;  // the centre term is wanted on its own
      if (l >= 3 && !own_centre) {
        // right insertion + centre term = B_r(Gamma, gdot_rbar^(l-1) + gdot_{r,L}^(l-1)): the
        // bubble is linear in its right vertex, so one bubble of the combined vertex (the other
        // channels from order l-1, channel r the stored left insertion) replaces two
        BubbleOut lv = view_of(ctx->lstore[prev][r].p);
        kqft_vertex rc_vert = rbar;
        rc_vert.ch[r] = kqft_chvert{1.0, (const double*)lv.K1, (const double*)lv.K2, (const double*)lv.K2p,
                                    (const double*)lv.K3};
        if ((rc = bubble_core(ctx, r, V, rc_vert, G, KQFT_PI_GG, q, o, dst, s))) return rc;
        continue;
      }
      if ((rc = bubble_core(ctx, r, V, rbar, G, KQFT_PI_GG, q, o, dst, s))) return rc;
      if (own_centre) {  // centre term B_r(Gamma, gdot_{r,L}^(l-1)), kept apart for the Sigma_dot corrections
        BubbleOut lv = view_of(ctx->lstore[prev][r].p);
        kqft_vertex lvert;
        memset(&lvert, 0, sizeof lvert);
        lvert.grid = V.grid;
        lvert.ch[r] = kqft_chvert{1.0, (const double*)lv.K1, (const double*)lv.K2, (const double*)lv.K2p,
                                  (const double*)lv.K3};
        BubbleOut ct = view_of(ctx->ctmp.p);
        o.beta = 0;
        if ((rc = bubble_core(ctx, r, V, lvert, G, KQFT_PI_GG, q, o, ct, s))) return rc;
        comb(dst, 1.0, dst, 1.0, ct);
        if (l == 3)
          comb(centre[r], 1.0, ct, 0.0, ct);
        else
          comb(centre[r], 1.0, centre[r], 1.0, ct);
      }
    }
  }
  return KQFT_OK;
}

int kqft_mloop_step(kqft_ctx* ctx, int n_points, const kqft_vertex* gamma, const kqft_propagator* G,
                    const kqft_quad* q, int nloops, const kqft_opts* opts, const kqft_chout* dgamma,
                    void* stream) {
  int rc;
  if (!ctx) return fail(KQFT_EINVAL, "ctx is NULL");
  if (n_points < 1 || nloops < 1 || !gamma || !G || !q || !dgamma || !opts)
    return fail(KQFT_EINVAL, "mloop_step needs n_points >= 1, nloops >= 1 and non-NULL arrays");
  for (int p = 0; p < n_points; ++p) {
    if ((rc = check_common(ctx, &G[p], &q[p], opts))) return rc;
    if ((rc = check_grid(gamma[p].grid, "gamma"))) return rc;
    for (int l = 0; l < nloops; ++l)
      for (int r = 0; r < 3; ++r) {
        const kqft_chout& d = dgamma[((size_t)p * nloops + l) * 3 + r];
        if (!d.K1 || !d.K2 || !d.K2p || !d.K3) return fail(KQFT_EINVAL, "dgamma arrays must all be given");
      }
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  for (int p = 0; p < n_points; ++p) {
    auto dview = [&](int l, int r) {
      const kqft_chout& d = dgamma[((size_t)p * nloops + l) * 3 + r];
      return BubbleOut{(double2*)d.K1, (double2*)d.K2, (double2*)d.K2p, (double2*)d.K3};
    };
    if ((rc = mloop_core(ctx, gamma[p], G[p], q[p], nloops, *opts, dview, nullptr, s))) return rc;
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

// The adjoints differentiate the Delta-regulated propagator without Sigma_dot only.
static int check_adjoint_prop(const kqft_propagator& G) {
  if (G.reg != KQFT_REG_DELTA || G.dSigR || G.dSigK || G.deps != 0.0)
    return fail(KQFT_EINVAL, "adjoints take the Delta-regulated propagator without Sigma_dot");
  return KQFT_OK;
}

int kqft_bubble_adjoint(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                        const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                        const kqft_chout* dout, const kqft_chout* dleft, const kqft_chout* dright, double* dscal,
                        void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if ((rc = check_adjoint_prop(*G))) return rc;
  if (channel < 0 || channel > 2) return fail(KQFT_EINVAL, "channel must be 0 (a), 1 (p) or 2 (t)");
  if (pi_kind != KQFT_PI_GG && pi_kind != KQFT_PI_DOT) return fail(KQFT_EINVAL, "unknown propagator pair");
  if ((rc = check_vertex(left, "left vertex")) || (rc = check_vertex(right, "right vertex"))) return rc;
  if (!same_grid(left->grid, right->grid)) return fail(KQFT_ESHAPE, "left and right vertices must share one grid");
  if (!dout || !dleft || !dright || !dscal) return fail(KQFT_EINVAL, "dout, dleft, dright and dscal must be given");
  HIP_TRY(hipSetDevice(ctx->device));
  return adjoint_core(ctx, channel, *left, *right, *G, pi_kind, *q, *dout, dleft, dright, dscal, dscal + 1,
                      dscal + 2, (hipStream_t)stream, opts->precision);
}

int kqft_sde_adjoint(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q_bubble,
                     const kqft_quad* q_loop, const kqft_opts* opts, const double* dsigma, const kqft_chout* dgamma,
                     double* dscal, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q_bubble, opts))) return rc;
  if ((rc = check_adjoint_prop(*G))) return rc;
  if (!q_loop || q_loop->n < 1) return fail(KQFT_ESHAPE, "invalid loop quadrature");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!dsigma || !dgamma || !dscal) return fail(KQFT_EINVAL, "dsigma, dgamma and dscal must be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = gamma->grid.n;
  // recompute Phi = B_a(Gamma_0, Gamma) (classes K1, K2')
  const size_t k1b = (size_t)2 * n * 16 * 16, k2b = (size_t)2 * n * n * 16 * 16;
  if ((rc = ensure(ctx->phi, k1b + k2b))) return rc;
  if ((rc = ensure(ctx->phigrad, k1b + k2b))) return rc;
  double2* phiK1 = (double2*)ctx->phi.p;
  double2* phiK2p = (double2*)((char*)ctx->phi.p + k1b);
  double2* dK1 = (double2*)ctx->phigrad.p;
  double2* dK2p = (double2*)((char*)ctx->phigrad.p + k1b);
  kqft_vertex bare;
  memset(&bare, 0, sizeof bare);
  bare.r0 = gamma->r0;
  bare.grid = gamma->grid;
  kqft_opts o = *opts;
  o.precision = KQFT_FP64;
  o.class_mask = KQFT_K1 | KQFT_K2P;
  o.beta = 0;
  o.overlap = 0;
  BubbleOut po{phiK1, nullptr, phiK2p, nullptr};
  if ((rc = bubble_core(ctx, KQFT_CH_A, bare, *gamma, *G, KQFT_PI_GG, *q_bubble, o, po, s))) return rc;
  // loop adjoint: dSigma -> dPhi, dDelta
  const double *nodes, *qv, *qw;
  if ((rc = get_grid(ctx, gamma->grid, &nodes))) return rc;
  if ((rc = get_quad(ctx, *q_loop, &qv, &qw))) return rc;
  DProp P;
  if ((rc = to_dprop(*G, P))) return rc;
  HIP_TRY(hipMemsetAsync(ctx->phigrad.p, 0, k1b + k2b, s));
  LoopAdjArgs la{make_dgrid(n, gamma->grid.L, gamma->grid.a, gamma->grid.map), P, q_loop->n, nodes, qv, qw, phiK1, phiK2p,
                 (const double2*)dsigma, dK1, dK2p, dscal + 1};
  launch_loop_adjoint(la, s);
  // bubble adjoint of Phi: the bare vertex on the left carries gamma->r0 as well
  kqft_chout dphi{(double*)dK1, nullptr, (double*)dK2p, nullptr};
  kqft_chout none[3];
  memset(none, 0, sizeof none);
  return adjoint_core(ctx, KQFT_CH_A, bare, *gamma, *G, KQFT_PI_GG, *q_bubble, dphi, none, dgamma, dscal, dscal,
                      dscal + 1, s);
}


// Views of the four classes of one channel packed back to back in a buffer.
static BubbleOut class_view(void* p, int n) {
  const size_t s1 = (size_t)2 * n * 16 * sizeof(double2), s2 = (size_t)2 * n * n * 16 * sizeof(double2);
  char* b = (char*)p;
  return BubbleOut{(double2*)b, (double2*)(b + s1), (double2*)(b + s1 + s2), (double2*)(b + s1 + 2 * s2)};
}
static kqft_chout chout_of(const BubbleOut& v) {
  return kqft_chout{(double*)v.K1, (double*)v.K2, (double*)v.K2p, (double*)v.K3};
}
static kqft_chvert chvert_of(const BubbleOut& v, double coef = 1.0) {
  return kqft_chvert{coef, (const double*)v.K1, (const double*)v.K2, (const double*)v.K2p, (const double*)v.K3};
}
// dst (+)= src class by class; a NULL src class counts as zero
static int copy_classes(const BubbleOut& dst, const kqft_chout& src, int n, bool add, hipStream_t s) {
  const size_t c[4] = {(size_t)2 * n * 16, (size_t)2 * n * n * 16, (size_t)2 * n * n * 16, (size_t)2 * n * n * n * 16};
  double2* d[4] = {dst.K1, dst.K2, dst.K2p, dst.K3};
  const double2* x[4] = {(const double2*)src.K1, (const double2*)src.K2, (const double2*)src.K2p,
                         (const double2*)src.K3};
  for (int k = 0; k < 4; ++k) {
    if (x[k])
      launch_axpby(d[k], 1.0, x[k], add ? 1.0 : 0.0, add ? d[k] : x[k], c[k], s);
    else if (!add)
      HIP_TRY(hipMemsetAsync(d[k], 0, c[k] * sizeof(double2), s));
  }
  return KQFT_OK;
}

int kqft_mloop_adjoint(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
                       int nloops, const kqft_opts* opts, const kqft_chout* dgdot, const kqft_chout* dgamma,
                       double* dscal, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if ((rc = check_adjoint_prop(*G))) return rc;
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (nloops < 1) return fail(KQFT_EINVAL, "nloops must be >= 1");
  if (!dgdot || !dgamma || !dscal) return fail(KQFT_EINVAL, "dgdot, dgamma and dscal must be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = gamma->grid.n;
  const size_t chb = ((size_t)2 * n * 16 + (size_t)4 * n * n * 16 + (size_t)2 * n * n * n * 16) * sizeof(double2);
  const int depth = nloops >= 2 ? 2 : 0;
  for (int x = 0; x < depth; ++x)
    for (int r = 0; r < 3; ++r)
      if ((rc = ensure(ctx->mlrec[x][r], chb)) || (rc = ensure(ctx->mlbar[x][r], chb)) ||
          (rc = ensure(ctx->mlext[x][r], chb)))
        return rc;
  if ((rc = ensure(ctx->mlscr, 4 * sizeof(double)))) return rc;
  double* dr0_drop = (double*)ctx->mlscr.p;  // r0 cotangents of insertion vertices (r0 = 0, no parameter)
  kqft_opts o = *opts;  // recomputed insertions and transposed products in opts->precision
  const int prec = o.precision;
  o.class_mask = KQFT_KALL;
  o.beta = 0;
  o.overlap = 0;
  auto rec = [&](int l0, int r) { return class_view(ctx->mlrec[l0 & 1][r].p, n); };  // order l0 + 1
  auto bar = [&](int l0, int r) { return class_view(ctx->mlbar[l0 & 1][r].p, n); };
  auto ext = [&](int l0, int r) { return class_view(ctx->mlext[l0 & 1][r].p, n); };
  kqft_chout none[3];
  memset(none, 0, sizeof none);
  // cotangent accumulators of the top order: the caller's cotangents (NULL classes = 0)
  if (nloops >= 2)
    for (int r = 0; r < 3; ++r) {
      if ((rc = copy_classes(bar(nloops - 1, r), dgdot[(size_t)(nloops - 1) * 3 + r], n, false, s))) return rc;
      if ((rc = copy_classes(ext(nloops - 1, r), kqft_chout{}, n, false, s))) return rc;
    }
  for (int l = nloops; l >= 2; --l) {
    // recompute orders 1..l-1 (two alternating buffers) and the left insertions of order l-1
    auto dview = [&](int l0, int r) { return rec(l0, r); };
    if ((rc = mloop_core(ctx, *gamma, *G, *q, l - 1, o, dview, nullptr, s, true))) return rc;
    // accumulators of order l-1: the caller's cotangents, zero extras
    for (int r = 0; r < 3; ++r) {
      if ((rc = copy_classes(bar(l - 2, r), dgdot[(size_t)(l - 2) * 3 + r], n, false, s))) return rc;
      if ((rc = copy_classes(ext(l - 2, r), kqft_chout{}, n, false, s))) return rc;
    }
    for (int r = 0; r < 3; ++r) {
      // gdot_rbar^(l-1): the other two channels of order l-1; their cotangents accumulate
      kqft_vertex rbar;
      memset(&rbar, 0, sizeof rbar);
      rbar.grid = gamma->grid;
      kqft_chout drbar[3];
      memset(drbar, 0, sizeof drbar);
      for (int r2 = 0; r2 < 3; ++r2) {
        if (r2 == r) continue;
        rbar.ch[r2] = chvert_of(rec(l - 2, r2));
        drbar[r2] = chout_of(bar(l - 2, r2));
      }
      const BubbleOut dtot = bar(l - 1, r);
      // left insertion L_r^l = B_r(rbar, Gamma): cotangent = that of the order plus the one the
      // centre term of order l+1 passed back (already summed into ext)
      const BubbleOut dl = ext(l - 1, r);
      if ((rc = copy_classes(dl, chout_of(dtot), n, true, s))) return rc;
      if ((rc = adjoint_core(ctx, r, rbar, *gamma, *G, KQFT_PI_GG, *q, chout_of(dl), drbar, dgamma, dr0_drop,
                             dscal, dscal + 1, s, prec)))
        return rc;
      // right insertion B_r(Gamma, rbar)
      if ((rc = adjoint_core(ctx, r, *gamma, rbar, *G, KQFT_PI_GG, *q, chout_of(dtot), dgamma, drbar, dscal,
                             dr0_drop, dscal + 1, s, prec)))
        return rc;
      if (l >= 3) {  // centre term B_r(Gamma, L_r^(l-1)): its right cotangent goes to L_r^(l-1)
        kqft_vertex lv;
        memset(&lv, 0, sizeof lv);
        lv.grid = gamma->grid;
        lv.ch[r] = chvert_of(class_view(ctx->lstore[(l - 1) & 1][r].p, n));
        kqft_chout dlv[3];
        memset(dlv, 0, sizeof dlv);
        dlv[r] = chout_of(ext(l - 2, r));
        if ((rc = adjoint_core(ctx, r, *gamma, lv, *G, KQFT_PI_GG, *q, chout_of(dtot), dgamma, dlv, dscal,
                               dr0_drop, dscal + 1, s, prec)))
          return rc;
      }
    }
  }
  // order 1: B_r(Gamma, Gamma; Pidot); its cotangent is the caller's plus what order 2 passed down
  for (int r = 0; r < 3; ++r) {
    kqft_chout d1 = dgdot[r];
    if (nloops >= 2) d1 = chout_of(bar(0, r));
    if (!d1.K1 && !d1.K2 && !d1.K2p && !d1.K3) continue;
    if (nloops < 2) {  // the caller's cotangent may leave classes NULL: give the adjoint zeros
      if ((rc = ensure(ctx->mlbar[0][r], chb))) return rc;
      if ((rc = copy_classes(class_view(ctx->mlbar[0][r].p, n), d1, n, false, s))) return rc;
      d1 = chout_of(class_view(ctx->mlbar[0][r].p, n));
    }
    if ((rc = adjoint_core(ctx, r, *gamma, *gamma, *G, KQFT_PI_DOT, *q, d1, dgamma, dgamma, dscal, dscal,
                           dscal + 1, s, prec)))
      return rc;
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

int kqft_mloop_jvp(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_vertex* tangent, const kqft_propagator* G,
                   const kqft_quad* q, int nloops, const kqft_opts* opts, const kqft_chout* out,
                   const kqft_chout* dout, void* stream) {
  int rc;
  if ((rc = check_common(ctx, G, q, opts))) return rc;
  if ((rc = check_vertex(gamma, "gamma")) || (rc = check_vertex(tangent, "tangent"))) return rc;
  if (!same_grid(gamma->grid, tangent->grid)) return fail(KQFT_ESHAPE, "gamma and its tangent must share one grid");
  if (nloops < 1 || !out || !dout) return fail(KQFT_EINVAL, "jvp needs nloops >= 1, out and dout");
  for (int k = 0; k < nloops * 3; ++k)
    if (!out[k].K1 || !out[k].K2 || !out[k].K2p || !out[k].K3 || !dout[k].K1 || !dout[k].K2 || !dout[k].K2p ||
        !dout[k].K3)
      return fail(KQFT_EINVAL, "out and dout arrays must all be given");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = gamma->grid.n;
  const size_t chb = ((size_t)2 * n * 16 + (size_t)4 * n * n * 16 + (size_t)2 * n * n * n * 16) * sizeof(double2);
  const size_t cls[4] = {(size_t)2 * n * 16, (size_t)2 * n * n * 16, (size_t)2 * n * n * 16,
                         (size_t)2 * n * n * n * 16};
  if (nloops >= 3)
    for (int x = 0; x < 2; ++x)
      for (int r = 0; r < 3; ++r)
        if ((rc = ensure(ctx->mlrec[x][r], chb)) || (rc = ensure(ctx->mlbar[x][r], chb))) return rc;
  kqft_opts o = *opts;
  o.class_mask = KQFT_KALL;
  o.overlap = 0;
  auto view = [&](const kqft_chout* a, int l0, int r) {
    const kqft_chout& c = a[(size_t)l0 * 3 + r];
    return BubbleOut{(double2*)c.K1, (double2*)c.K2, (double2*)c.K2p, (double2*)c.K3};
  };
  auto keep = [&](DevBuf (&buf)[2][3], int l, int r, const BubbleOut& src) -> int {
    const BubbleOut d = class_view(buf[l & 1][r].p, n);
    const double2* x[4] = {src.K1, src.K2, src.K2p, src.K3};
    double2* y[4] = {d.K1, d.K2, d.K2p, d.K3};
    for (int k = 0; k < 4; ++k)
      HIP_TRY(hipMemcpyAsync(y[k], x[k], cls[k] * sizeof(double2), hipMemcpyDeviceToDevice, s));
    return KQFT_OK;
  };
  // B(L, R) and its tangent B(dL, R) + B(L, dR) at the fixed propagator (bilinear bubble)
  auto bub = [&](int r, const kqft_vertex& L, const kqft_vertex& dL, const kqft_vertex& R, const kqft_vertex& dR,
                 int kind, const BubbleOut& o1, const BubbleOut& d1, int beta) -> int {
    int e;
    o.beta = beta;
    if ((e = bubble_core(ctx, r, L, R, *G, kind, *q, o, o1, s))) return e;
    if ((e = bubble_core(ctx, r, dL, R, *G, kind, *q, o, d1, s))) return e;
    o.beta = 1;
    return bubble_core(ctx, r, L, dR, *G, kind, *q, o, d1, s);
  };
  for (int l = 1; l <= nloops; ++l) {
    for (int r = 0; r < 3; ++r) {
      const BubbleOut o1 = view(out, l - 1, r), d1 = view(dout, l - 1, r);
      if (l == 1) {
        if ((rc = bub(r, *gamma, *tangent, *gamma, *tangent, KQFT_PI_DOT, o1, d1, 0))) return rc;
        continue;
      }
      kqft_vertex rb, drb;
      memset(&rb, 0, sizeof rb);
      memset(&drb, 0, sizeof drb);
      rb.grid = drb.grid = gamma->grid;
      for (int r2 = 0; r2 < 3; ++r2) {
        if (r2 == r) continue;
        rb.ch[r2] = chvert_of(view(out, l - 2, r2));
        drb.ch[r2] = chvert_of(view(dout, l - 2, r2));
      }
      if ((rc = bub(r, rb, drb, *gamma, *tangent, KQFT_PI_GG, o1, d1, 0))) return rc;  // left
      if (l + 1 <= nloops && l >= 2)  // kept for the centre term of order l + 1
        if ((rc = keep(ctx->mlrec, l, r, o1)) || (rc = keep(ctx->mlbar, l, r, d1))) return rc;
      if ((rc = bub(r, *gamma, *tangent, rb, drb, KQFT_PI_GG, o1, d1, 1))) return rc;  // right
      if (l >= 3) {  // centre B_r(Gamma, L_r^(l-1))
        kqft_vertex lv, dlv;
        memset(&lv, 0, sizeof lv);
        memset(&dlv, 0, sizeof dlv);
        lv.grid = dlv.grid = gamma->grid;
        lv.ch[r] = chvert_of(class_view(ctx->mlrec[(l - 1) & 1][r].p, n));
        dlv.ch[r] = chvert_of(class_view(ctx->mlbar[(l - 1) & 1][r].p, n));
        if ((rc = bub(r, *gamma, *tangent, lv, dlv, KQFT_PI_GG, o1, d1, 1))) return rc;
      }
    }
  }
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

int kqft_workspace_bytes(size_t* current, size_t* peak) {
  if (!current && !peak) return fail(KQFT_EINVAL, "current and peak are both NULL");
  if (current) *current = g_ws_bytes.load();
  if (peak) *peak = g_ws_peak.load();
  return KQFT_OK;
}

int kqft_workspace_reset_peak(void) {
  g_ws_peak.store(g_ws_bytes.load());
  return KQFT_OK;
}


}  // extern "C"

// ------------------------------------------------------------------ allocation-free chi
// Static scratch of kqft_chi_noalloc: one copy per device, held until the process ends.  In
// host code `scratch` is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that address
// is handed to kernels.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_of_current_device(void** ptr) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(KQFT_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KQFT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return KQFT_OK;
}

extern "C" {

int kqft_chi_noalloc(int channel, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
                     double* chi, void* stream) {
  int rc;
  if (channel < KQFT_CH_A || channel > KQFT_CH_T) return fail(KQFT_EINVAL, "channel must be 0, 1 or 2");
  if (!G || !q) return fail(KQFT_EINVAL, "propagator and quadrature must be given");
  if (q->n < 1 || (q->map != KQFT_QUAD_TAN_FINITE && q->map != KQFT_QUAD_TAN_INFINITE) ||
      (q->map == KQFT_QUAD_TAN_FINITE && !(q->L > 0)) || !(q->a > 0))
    return fail(KQFT_ESHAPE, "invalid quadrature");
  if (q->n > 46340) return fail(KQFT_ESHAPE, "chi needs q->n <= 46340");
  if ((rc = check_vertex(gamma, "gamma"))) return rc;
  if (!chi) return fail(KQFT_EINVAL, "chi is NULL");
  DProp P;
  if ((rc = to_dprop(*G, P))) return rc;
  void* base = nullptr;
  if ((rc = scratch_of_current_device(&base))) return rc;
  const int r = channel, n = gamma->grid.n, nq = q->n, nblk = chi_blocks(nq);
  // layout: grid nodes | quadrature nodes, weights | tables of the active other channels |
  // Pi and block partials of nb transfer frequencies (256-byte aligned pieces)
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t tbytes = ((size_t)n * n * n + 2 * (size_t)n * n + n) * 32 * sizeof(double2);
  size_t fixed = up(n * sizeof(double)) + 2 * up(nq * sizeof(double));
  bool act[2];
  for (int d = 0; d < 2; ++d) {
    act[d] = table_active(gamma->ch[(r + 1 + d) % 3]);
    if (act[d]) fixed += up(tbytes);
  }
  const bool proj = n <= kChiProjMaxN;
  const size_t per_w = (size_t)nq * 256 + (size_t)nblk * 32 * sizeof(double2) + (proj ? chi_proj_bytes(n) : 0);
  const long nb = fixed + up(per_w) + 512 <= kScratchBytes ? (long)((kScratchBytes - fixed - 512) / per_w) : 0;
  if (nb < 1)
    return fail(KQFT_ENOMEM, "kqft_chi_noalloc: n = " + std::to_string(n) + ", nq = " + std::to_string(nq) +
                                 " needs " + std::to_string(fixed + per_w) +
                                 " bytes of scratch; the static maximum is " + std::to_string(kScratchBytes));
  char* p = (char*)base;
  ChiBufs b;
  memset(&b, 0, sizeof b);
  double* nodes = (double*)p;
  p += up(n * sizeof(double));
  double* qv = (double*)p;
  p += up(nq * sizeof(double));
  double* qw = (double*)p;
  p += up(nq * sizeof(double));
  b.nodes = nodes;
  b.qv = qv;
  b.qw = qw;
  const hipStream_t s = (hipStream_t)stream;
  for (int d = 0; d < 2; ++d)
    if (act[d]) {
      const int r2 = (r + 1 + d) % 3;
      launch_table(table_args(r, r2, gamma->ch[r2], n, p), false, s);
      b.T[d] = p;
      p += up(tbytes);
    }
  b.nb = (int)std::min<long>(n, nb);
  b.pi = (double2*)p;
  p += up((size_t)b.nb * nq * 256);
  b.partial = (double2*)p;
  p += up((size_t)b.nb * nblk * 32 * sizeof(double2));
  if (proj) {
    b.pt = (double2*)p;
    b.own = b.pt + (size_t)b.nb * (n + 1) * 16;
  }
  launch_grid_nodes(n, gamma->grid.map, gamma->grid.a, aux_of(gamma->grid.map, gamma->grid.L / gamma->grid.a), nodes,
                    s);
  launch_quad_nodes(nq, q->a, q->map == KQFT_QUAD_TAN_FINITE ? atan(q->L / q->a) : 0.5 * M_PI, qv, qw, s);
  chi_run(nullptr, r, *gamma, P, nq, b, chi, s);
  HIP_TRY(hipGetLastError());
  return KQFT_OK;
}

}  // extern "C"
