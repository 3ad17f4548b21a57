// kqft_kernels.hip -- CDNA4 (gfx950) kernels of the Keldysh bubble path.
//
//   pi_kernel          Pi_r(w, v''_k) * w_k / (2 pi i) for a batch of transfer frequencies
//   table_kernel       the other channels' classes in the bubble channel's Keldysh order
//   gather_left        A panel:  rows (i, row) x cols (k, m) = Gamma_L-part(w, v_i, v''_k) . Pi_k
//   gather_right       B^T panel: rows (j, col) x cols (k, m) = Gamma_R-part(w, v''_k, v'_j)
//   zgemm_f64 / _f32   C = A . B per (w, spin combination) on MFMA, bordered epilogue
//                      that de-diagonalises the spin combinations into X/Y and writes
//                      K3 (main block), K2 (last column), K2' (last row), K1 (corner)
//   adaptive_kernel    adaptive Gauss-Lobatto-Kronrod bubble, one wavefront per output interval
//   loop_kernel        Schwinger-Dyson loop reduction
//   vloop_kernel       loop of a full vertex (all channels through tables) with G, S or G s G
//   chi_kernel         susceptibility double sum of one channel (table gathers + Pi contractions)
//   parquet / flow helpers: sigma_split, maxdiff, axpby, lincomb, errnorm, dot, mix,
//                      occupation (Hartree term)
//   adjoint kernels    reverse pass of the bubble and of the Schwinger-Dyson loop
//
// The bubble (Eq. B_a and the BSEs of the paper) is written as one Keldysh-blocked
// complex matrix product per transfer frequency: the 4x4 Keldysh matrices of the
// paper's vectorised integrand become the innermost dimension of the product, the
// v'' quadrature its contraction index, and the asymptotic-class split of the
// vertex a border of one extra block row and column.
#include <algorithm>

#include "kqft_internal.h"
#include "kqft_launch.h"

namespace kqft {

__constant__ int c_perm[3][3][16];

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// ======================================================================== Pi
__global__ __launch_bounds__(256) void pi_kernel(PiArgs a) {
  long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)a.nb * a.nq;
  if (tid >= total) return;
  int b = (int)(tid / a.nq), k = (int)(tid % a.nq);
  double w = a.wnodes[a.iw0 + b];
  double vq = a.qv[k];
  double f3, f4;
  if (a.r == 1) {
    f3 = 0.5 * w + vq;
    f4 = 0.5 * w - vq;
  } else {
    f3 = vq + 0.5 * w;
    f4 = vq - 0.5 * w;
  }
  double2 g3[4], g4[4];
  propagator(a.P, 0, f3, g3);
  propagator(a.P, 0, f4, g4);
  double2 s3[4], s4[4];
  if (a.kind == 1) {
    propagator(a.P, 1, f3, s3);
    propagator(a.P, 1, f4, s4);
  }
  double2 wgt = make_double2(0.0, -a.qw[k] * (0.5 / M_PI));  // w_k / (2 pi i)
  double2* out = a.out + ((size_t)b * a.nq + k) * 16;
  for (int a3 = 0; a3 < 2; ++a3)
    for (int a3p = 0; a3p < 2; ++a3p)
      for (int a4 = 0; a4 < 2; ++a4)
        for (int a4p = 0; a4p < 2; ++a4p) {
          int rp, cp;
          if (a.r == 0) {  // (a3, a4' | a3', a4)
            rp = 2 * a3 + a4p;
            cp = 2 * a3p + a4;
          } else if (a.r == 1) {  // (a3, a4 | a3', a4')
            rp = 2 * a3 + a4;
            cp = 2 * a3p + a4p;
          } else {  // (a4', a3 | a3', a4)
            rp = 2 * a4p + a3;
            cp = 2 * a3p + a4;
          }
          double2 v;
          if (a.kind == 0)
            v = cmul(g3[2 * a3 + a3p], g4[2 * a4 + a4p]);
          else
            v = cadd(cmul(s3[2 * a3 + a3p], g4[2 * a4 + a4p]), cmul(g3[2 * a3 + a3p], s4[2 * a4 + a4p]));
          out[4 * rp + cp] = cmul(wgt, v);
        }
}

// ======================================================================== target-order tables
// For a bubble in channel r every other channel r2 is tabulated once per call in r's
// Keldysh order, with r's spin combinations and r2's coefficient applied:
//   rec(f, c) = coef_{r2} * sum_s mix[c][s] * K_{r2, s}[perm_{r -> r2}(f)],
// one record of 32 values (16 flat indices f x 2 combinations c) per grid cell, for
//   F3[w][v][v'] = K1 + K2 + K2' + K3   (all three arguments on the grid)
//   F2v[w][v]    = K1 + K2              (v' off the grid)
//   F2p[w][v']   = K1 + K2'             (v off the grid)
//   F1[w]        = K1                   (v and v' off the grid)
// stored back to back.  Absent classes count as zero.  Inside a record, (f, c) sits where
// lane l of an 8-lane group finds (f = l, l + 8; c = 0, 1) with 16-byte loads that cover
// whole cache lines across the group:
//   FP32 record (256 B): float2 position 2f + c
//   FP64 record (512 B): double2 position 16 (f / 8) + 8c + f % 8
__host__ __device__ inline int rec_pos(int f, int c, bool f32) {
  return f32 ? 2 * f + c : 16 * (f >> 3) + 8 * c + (f & 7);
}
__device__ inline void st2(double2* p, double2 v) { *p = v; }
__device__ inline void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// Record indices in 32 bits: grids have at most 600 points (checked at the entry points), so
// 16 threads per record stay below 2^32.
template <class TT> __global__ __launch_bounds__(256) void table_kernel(TableArgs a) {
  const unsigned n = a.n, n2 = n * n, n3 = n2 * n;
  const unsigned total = (n3 + 2 * n2 + n) * 16;
  const bool f32 = sizeof(TT) == sizeof(float2);
  for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int f = (int)(e & 15);
    const unsigned rec = e >> 4;
    unsigned w, v = 0, vp = 0;
    bool has_v = false, has_vp = false;
    if (rec < n3) {
      const unsigned wv = rec / n;
      vp = rec - wv * n;
      w = wv / n;
      v = wv - w * n;
      has_v = has_vp = true;
    } else if (rec < n3 + n2) {
      w = (rec - n3) / n;
      v = rec - n3 - w * n;
      has_v = true;
    } else if (rec < n3 + 2 * n2) {
      w = (rec - n3 - n2) / n;
      vp = rec - n3 - n2 - w * n;
      has_vp = true;
    } else {
      w = rec - n3 - 2 * n2;
    }
    const int pf = c_perm[a.r][a.r2][f];
    double2 xy[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      double2 x = czero();
      const size_t sw = (size_t)s * n + w;
      if (a.K[0]) x = cadd(x, a.K[0][sw * 16 + pf]);
      if (has_v && a.K[1]) x = cadd(x, a.K[1][(sw * n + v) * 16 + pf]);
      if (has_vp && a.K[2]) x = cadd(x, a.K[2][(sw * n + vp) * 16 + pf]);
      if (has_v && has_vp && a.K[3]) x = cadd(x, a.K[3][((sw * n + v) * n + vp) * 16 + pf]);
      xy[s] = x;
    }
    TT* out = (TT*)a.out + (size_t)rec * 32;
    double2 cv[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double m0 = a.coef * a.mix[2 * c], m1 = a.coef * a.mix[2 * c + 1];
      cv[c] = make_double2(m0 * xy[0].x + m1 * xy[1].x, m0 * xy[0].y + m1 * xy[1].y);
    }
    if constexpr (sizeof(TT) == sizeof(float2)) {
      // (f, 0) and (f, 1) are adjacent in an FP32 record: one 16-byte store
      *reinterpret_cast<float4*>(out + rec_pos(f, 0, true)) =
          make_float4((float)cv[0].x, (float)cv[0].y, (float)cv[1].x, (float)cv[1].y);
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c) st2(out + rec_pos(f, c, f32), cv[c]);
    }
  }
}

// ======================================================================== gathers
// One 8-lane group per panel item (transfer frequency w, fermionic index i or j, node k).
// Lane l accumulates the spin combinations c = 0, 1 of the flat indices f = l and f = l + 8
// (channel r order): acc = {(l, 0), (l, 1), (l + 8, 0), (l + 8, 1)}.

// one tap of a table record, weight wgt
__device__ inline void rec_tap(const float2* rec, int l, double wgt, double2 acc[4]) {
  const float4* p = reinterpret_cast<const float4*>(rec);
  const float4 u = p[l], v = p[8 + l];
  acc[0] = make_double2(fma(wgt, (double)u.x, acc[0].x), fma(wgt, (double)u.y, acc[0].y));
  acc[1] = make_double2(fma(wgt, (double)u.z, acc[1].x), fma(wgt, (double)u.w, acc[1].y));
  acc[2] = make_double2(fma(wgt, (double)v.x, acc[2].x), fma(wgt, (double)v.y, acc[2].y));
  acc[3] = make_double2(fma(wgt, (double)v.z, acc[3].x), fma(wgt, (double)v.w, acc[3].y));
}
__device__ inline void rec_tap(const double2* rec, int l, double wgt, double2 acc[4]) {
  acc[0] = cfma(wgt, rec[l], acc[0]);
  acc[1] = cfma(wgt, rec[8 + l], acc[1]);
  acc[2] = cfma(wgt, rec[16 + l], acc[2]);
  acc[3] = cfma(wgt, rec[24 + l], acc[3]);
}

// Other channel from its tables at cell (iw, iv, ivp) with weights (tw, tv, tvp); an index
// of -1 marks an argument off the grid.
template <class TT>
__device__ inline void table_taps(const TT* T, int n, int iw, double tw, int iv, double tv, int ivp, double tvp,
                                  int l, double2 acc[4]) {
  if (iw < 0) return;
  const size_t nn = n, n2 = nn * nn, n3 = n2 * nn;
#pragma unroll
  for (int cw = 0; cw < 2; ++cw) {
    const double ww = cw ? tw : 1.0 - tw;
    const size_t w = (size_t)iw + cw;
    if (iv >= 0 && ivp >= 0) {
#pragma unroll
      for (int cv = 0; cv < 2; ++cv)
#pragma unroll
        for (int cp = 0; cp < 2; ++cp)
          rec_tap(T + ((w * nn + iv + cv) * nn + ivp + cp) * 32, l,
                  ww * (cv ? tv : 1.0 - tv) * (cp ? tvp : 1.0 - tvp), acc);
    } else if (iv >= 0) {
#pragma unroll
      for (int cv = 0; cv < 2; ++cv) rec_tap(T + (n3 + w * nn + iv + cv) * 32, l, ww * (cv ? tv : 1.0 - tv), acc);
    } else if (ivp >= 0) {
#pragma unroll
      for (int cp = 0; cp < 2; ++cp)
        rec_tap(T + (n3 + n2 + w * nn + ivp + cp) * 32, l, ww * (cp ? tvp : 1.0 - tvp), acc);
    } else {
      rec_tap(T + (n3 + 2 * n2 + w) * 32, l, ww, acc);
    }
  }
}

// Own-channel class entry (channel order, both spins) for f = l, l + 8:
// xy = {X(l), X(l + 8), Y(l), Y(l + 8)} += wgt * entry; sstride = spin stride in double2.
__device__ inline void own_tap(const double2* p, size_t sstride, int l, double wgt, double2 xy[4]) {
  xy[0] = cfma(wgt, p[l], xy[0]);
  xy[1] = cfma(wgt, p[8 + l], xy[1]);
  xy[2] = cfma(wgt, p[sstride + l], xy[2]);
  xy[3] = cfma(wgt, p[sstride + 8 + l], xy[3]);
}

// acc += combinations (mix) of coef * xy, plus the bare vertex when r0 != 0
__device__ inline void own_mix(double c, const double mix[4], int l, double r0, const double2 xy[4],
                               double2 acc[4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = l + 8 * h;
    const double2 X = xy[h], Y = xy[2 + h];
    const double bare = bare_odd(f) ? 0.5 * r0 : 0.0;  // X_R = -r0/2, Y_R = +r0/2 on odd f
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const double m0 = mix[2 * cc], m1 = mix[2 * cc + 1];
      acc[2 * h + cc].x += c * (m0 * X.x + m1 * Y.x) + (m1 - m0) * bare;
      acc[2 * h + cc].y += c * (m0 * X.y + m1 * Y.y);
    }
  }
}

// Seven grid locations per item, one per lane, shared across the 8-lane group:
// slot 0 = v'' (own channel), slots 1-3 / 4-6 = (w, v, v') of channels r + 1 / r + 2.
// loc[j] = cell index (-1 off the grid), wt[j] = weight of the upper node.
__device__ inline void group_locate(const GatherArgs& a, int l, bool others, double w, double v, double vp,
                                    double vq, int loc[7], double wt[7]) {
  double arg = vq;
  if (others && l >= 1 && l <= 6) {
    double L[4];
    legs_of(a.r, w, v, vp, L);
    const int d = l <= 3 ? 1 : 2, which = (l - 1) % 3;
    double w2, v2, vp2;
    params_of((a.r + d) % 3, L, w2, v2, vp2);
    arg = which == 0 ? w2 : (which == 1 ? v2 : vp2);
  }
  int ic;
  double tc;
  if (!dgrid_locate(a.g, arg, ic, tc)) {
    ic = -1;
    tc = 0.0;
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    loc[j] = __shfl(ic, j, 8);
    wt[j] = __shfl(tc, j, 8);
  }
}

template <int Q> __device__ inline double quad_bcast(double v) {
  constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);  // quad_perm [Q, Q, Q, Q]
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int Q> __device__ inline void pi_step(const double2 acc[4], double2 P, double2 s[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 x = make_double2(quad_bcast<Q>(acc[u].x), quad_bcast<Q>(acc[u].y));
    s[u] = cadd(s[u], cmul(x, P));
  }
}

// (acc . Pi)[row, m] for m = l % 4 from the quad's four q (pk = Pi entries of one node)
__device__ inline void apply_pi(const double2* pk, int q4, double2 acc[4]) {
  const double2 P0 = pk[q4], P1 = pk[4 + q4], P2 = pk[8 + q4], P3 = pk[12 + q4];
  double2 s[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) s[u] = czero();
  pi_step<0>(acc, P0, s);
  pi_step<1>(acc, P1, s);
  pi_step<2>(acc, P2, s);
  pi_step<3>(acc, P3, s);
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = s[u];
}

template <class T> __device__ inline void store_c(T* p, double2 v);
template <> __device__ inline void store_c<double2>(double2* p, double2 v) { *p = v; }
template <> __device__ inline void store_c<float2>(float2* p, double2 v) {
  *p = make_float2((float)v.x, (float)v.y);
}

// Left factor of one (w_iw, v_i, v'') for the lanes of an 8-lane group: Gamma_L - Gamma_L^inf
// at (w, v_i, v'') when main, else Gamma_L^inf(w, v''); lane l gets rows l/4 and 2 + l/4 at
// column l%4 for both spin combinations: acc = {c0 row h, c1 row h, c0 row 2+h, c1 row 2+h}.
template <class T>
__device__ __forceinline__ void left_vals(const GatherArgs& a, int l, int iw, int i, bool main, double vq,
                                          double2 acc[4]) {
  const int n = a.g.n;
  const double w = a.nodes[iw];
  int loc[7];
  double wt[7];
  group_locate(a, l, main, w, main ? a.nodes[i] : 0.0, vq, vq, loc, wt);
  double2 xy[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = xy[u] = czero();
  const size_t nn = n, n2 = nn * nn, n3 = n2 * nn;
  const int j0 = loc[0];
  const double t = wt[0];
  if (main) {  // Gamma_L - Gamma_L^inf: own K2(w, v_i) + K3(w, v_i, v''), the other channels
    if (a.coef != 0.0) {
      if (a.K[1]) own_tap(a.K[1] + ((size_t)iw * nn + i) * 16, n2 * 16, l, 1.0, xy);
      if (a.K[3] && j0 >= 0) {
        const double2* p = a.K[3] + (((size_t)iw * nn + i) * nn + j0) * 16;
        own_tap(p, n3 * 16, l, 1.0 - t, xy);
        own_tap(p + 16, n3 * 16, l, t, xy);
      }
      own_mix(a.coef, a.mix, l, 0.0, xy, acc);
    }
#pragma unroll
    for (int d = 0; d < 2; ++d)
      if (a.T[d])
        table_taps((const T*)a.T[d], n, loc[1 + 3 * d], wt[1 + 3 * d], loc[2 + 3 * d], wt[2 + 3 * d],
                   loc[3 + 3 * d], wt[3 + 3 * d], l, acc);
  } else {  // Gamma_L^inf(w, v'') = R + own K1(w) + K2'(w, v'')
    if (a.coef != 0.0) {
      if (a.K[0]) own_tap(a.K[0] + (size_t)iw * 16, nn * 16, l, 1.0, xy);
      if (a.K[2] && j0 >= 0) {
        const double2* p = a.K[2] + ((size_t)iw * nn + j0) * 16;
        own_tap(p, n2 * 16, l, 1.0 - t, xy);
        own_tap(p + 16, n2 * 16, l, t, xy);
      }
    }
    own_mix(a.coef, a.mix, l, a.r0, xy, acc);
  }
}

// Right factor of one (w_iw, v'', v'_j): Gamma_R - Gamma_R^inf at (w, v'', v'_j) when main, else
// Gamma_R^inf(w, v''); lane l gets column l%4 of rows e = l/4 and 2 + l/4, both combinations:
// acc = {c0 row h, c1 row h, c0 row 2+h, c1 row 2+h}.
template <class T>
__device__ __forceinline__ void right_vals(const GatherArgs& a, int l, int iw, int j, bool main, double vq,
                                           double2 acc[4]) {
  const int n = a.g.n;
  const double w = a.nodes[iw];
  int loc[7];
  double wt[7];
  group_locate(a, l, main, w, vq, main ? a.nodes[j] : 0.0, vq, loc, wt);
  double2 xy[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = xy[u] = czero();
  const size_t nn = n, n2 = nn * nn, n3 = n2 * nn;
  const int i0 = loc[0];
  const double t = wt[0];
  if (main) {  // Gamma_R - Gamma_R^inf: own K2'(w, v'_j) + K3(w, v'', v'_j), the other channels
    if (a.coef != 0.0) {
      if (a.K[2]) own_tap(a.K[2] + ((size_t)iw * nn + j) * 16, n2 * 16, l, 1.0, xy);
      if (a.K[3] && i0 >= 0) {
        const double2* p = a.K[3] + (((size_t)iw * nn + i0) * nn + j) * 16;
        own_tap(p, n3 * 16, l, 1.0 - t, xy);
        own_tap(p + nn * 16, n3 * 16, l, t, xy);
      }
      own_mix(a.coef, a.mix, l, 0.0, xy, acc);
    }
#pragma unroll
    for (int d = 0; d < 2; ++d)
      if (a.T[d])
        table_taps((const T*)a.T[d], n, loc[1 + 3 * d], wt[1 + 3 * d], loc[2 + 3 * d], wt[2 + 3 * d],
                   loc[3 + 3 * d], wt[3 + 3 * d], l, acc);
  } else {  // Gamma_R^inf(w, v'') = R + own K1(w) + K2(w, v'')
    if (a.coef != 0.0) {
      if (a.K[0]) own_tap(a.K[0] + (size_t)iw * 16, nn * 16, l, 1.0, xy);
      if (a.K[1] && i0 >= 0) {
        const double2* p = a.K[1] + ((size_t)iw * nn + i0) * 16;
        own_tap(p, n2 * 16, l, 1.0 - t, xy);
        own_tap(p + 16, n2 * 16, l, t, xy);
      }
    }
    own_mix(a.coef, a.mix, l, a.r0, xy, acc);
  }
}

// A panel: row (i, row) x column (k, m) = sum_q (Gamma_L - Gamma_L^inf)(w, v_i, v''_k)[row, q]
// Pi_k[q, m] for i < n, Gamma_L^inf(w, v''_k) Pi_k on the border row block i = n; without
// Pi (a.pi == nullptr) the raw left factor.  Lane l holds rows l/4 and 2 + l/4, column l%4.
template <class T> __global__ __launch_bounds__(256) void gather_left_kernel(GatherArgs a) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = (int)(tid & 7);
  long item = tid >> 3;
  const int k = (int)(item % a.nq_pad);
  item /= a.nq_pad;
  const int il = (int)(item % a.cnt);
  const int b = (int)(item / a.cnt);
  if (b >= a.nb) return;  // whole groups: nq_pad, cnt and the block size are multiples of 8
  const int n = a.g.n, i = a.lo + il, iw = a.iw0 + b, h = l >> 2, q4 = l & 3;
  const size_t M = 4 * (size_t)(n + 1);
  const size_t off0 = ((size_t)b * M + 4 * (size_t)i + h) * a.Kp + 4 * (size_t)k + q4;
  const size_t off1 = off0 + 2 * a.Kp;
  T* o0 = (T*)a.P0;
  T* o1 = (T*)a.P1;
  if (k >= a.nq) {
    store_c(o0 + off0, czero());
    store_c(o1 + off0, czero());
    store_c(o0 + off1, czero());
    store_c(o1 + off1, czero());
    return;
  }
  double2 acc[4];
  left_vals<T>(a, l, iw, i, i < n, a.qv[k], acc);
  if (a.pi != nullptr) apply_pi(a.pi + ((size_t)b * a.nq + k) * 16, q4, acc);  // (Gamma_L . Pi_k)
  store_c(o0 + off0, acc[0]);
  store_c(o1 + off0, acc[1]);
  store_c(o0 + off1, acc[2]);
  store_c(o1 + off1, acc[3]);
}

// B^T panel: row (j, col) x column (k, e) = (Gamma_R - Gamma_R^inf)(w, v''_k, v'_j)[e, col]
// for j < n, Gamma_R^inf(w, v''_k)[e, col] on the border block j = n.  Lane l holds
// column l%4, rows e = l/4 and 2 + l/4.
template <class T> __global__ __launch_bounds__(256) void gather_right_kernel(GatherArgs a) {
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = (int)(tid & 7);
  long item = tid >> 3;
  const int k = (int)(item % a.nq_pad);
  item /= a.nq_pad;
  const int jl = (int)(item % a.cnt);
  const int b = (int)(item / a.cnt);
  if (b >= a.nb) return;
  const int n = a.g.n, j = a.lo + jl, iw = a.iw0 + b, h = l >> 2, q4 = l & 3;
  const size_t Ncol = 4 * (size_t)(n + 1);
  const size_t off0 = ((size_t)b * Ncol + 4 * (size_t)j + q4) * a.Kp + 4 * (size_t)k + h;
  const size_t off1 = off0 + 2;
  T* o0 = (T*)a.P0;
  T* o1 = (T*)a.P1;
  double2 acc[4];
  if (k < a.nq) {
    right_vals<T>(a, l, iw, j, j < n, a.qv[k], acc);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = czero();
  }
  if constexpr (sizeof(T) == sizeof(float2)) {
    // FP32 panels: lanes l and l ^ 4 (rows e = h, h + 2 of one column) trade one value per
    // combination so that each stores the two adjacent entries e = 2h, 2h + 1 as one 16-byte
    // store; the group's stores then cover whole 32-byte column runs of each panel row.
    float2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = make_float2((float)acc[u].x, (float)acc[u].y);
    const float2 s0 = h ? v[0] : v[2], s1 = h ? v[1] : v[3];
    const float2 r0 = make_float2(__shfl_xor(s0.x, 4), __shfl_xor(s0.y, 4));
    const float2 r1 = make_float2(__shfl_xor(s1.x, 4), __shfl_xor(s1.y, 4));
    const float4 c0 = h ? make_float4(r0.x, r0.y, v[2].x, v[2].y) : make_float4(v[0].x, v[0].y, r0.x, r0.y);
    const float4 c1 = h ? make_float4(r1.x, r1.y, v[3].x, v[3].y) : make_float4(v[1].x, v[1].y, r1.x, r1.y);
    const size_t offs = ((size_t)b * Ncol + 4 * (size_t)j + q4) * a.Kp + 4 * (size_t)k + 2 * h;
    *reinterpret_cast<float4*>(o0 + offs) = c0;
    *reinterpret_cast<float4*>(o1 + offs) = c1;
  } else {
    store_c(o0 + off0, acc[0]);
    store_c(o1 + off0, acc[1]);
    store_c(o0 + off1, acc[2]);
    store_c(o1 + off1, acc[3]);
  }
}

// ======================================================================== adaptive bubble
// Gauss-Lobatto-Kronrod integration per output (Sec. Frequency integration), breadth first:
// every work item (output o, interval [ya, yb] of the auxiliary variable y of the tangent
// map v'' = qa tan(y qth)) is one wavefront; its 8-lane groups evaluate the rule's nodes
// (left factor . Pi, right factor, the 4x4 product per spin combination, as the panels and
// the GEMM do for fixed nodes), the groups are summed, and the combinations are unmixed to
// X, Y.  Phase 0 stores the error scale of the output (GLK13 on the item's interval);
// phase 1 compares GL4 with GLK7 and either adds GLK7 into the outputs (FP64 atomics) or
// appends the six subintervals between the GLK7 nodes to the next work list.

__device__ inline double2 sel4(const double2 g[4], int k) {
  return k == 0 ? g[0] : (k == 1 ? g[1] : (k == 2 ? g[2] : g[3]));
}

// Pi_r[e][q4] (e = 0..3) at (w, v'') times 1/(2 pi i), the column this lane multiplies with
__device__ inline void pi_column(const DProp& P, int r, int kind, double w, double vq, int q4, double2 col[4]) {
  double f3, f4;
  if (r == 1) {
    f3 = 0.5 * w + vq;
    f4 = 0.5 * w - vq;
  } else {
    f3 = vq + 0.5 * w;
    f4 = vq - 0.5 * w;
  }
  double2 g3[4], g4[4], s3[4], s4[4];
  propagator(P, 0, f3, g3);
  propagator(P, 0, f4, g4);
  if (kind == 1) {
    propagator(P, 1, f3, s3);
    propagator(P, 1, f4, s4);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int a3, a3p, a4, a4p;
    if (r == 0) {  // rows (a3, a4'), columns (a3', a4)
      a3 = e >> 1;
      a4p = e & 1;
      a3p = q4 >> 1;
      a4 = q4 & 1;
    } else if (r == 1) {  // rows (a3, a4), columns (a3', a4')
      a3 = e >> 1;
      a4 = e & 1;
      a3p = q4 >> 1;
      a4p = q4 & 1;
    } else {  // rows (a4', a3), columns (a3', a4)
      a4p = e >> 1;
      a3 = e & 1;
      a3p = q4 >> 1;
      a4 = q4 & 1;
    }
    const int i3 = 2 * a3 + a3p, i4 = 2 * a4 + a4p;
    double2 v = cmul(sel4(g3, i3), sel4(g4, i4));
    if (kind == 1) v = cadd(cmul(sel4(s3, i3), sel4(g4, i4)), cmul(sel4(g3, i3), sel4(s4, i4)));
    col[e] = make_double2(v.y * (0.5 / M_PI), -v.x * (0.5 / M_PI));  // v / (2 pi i)
  }
}

__device__ inline void apply_pi_col(const double2 col[4], double2 acc[4]) {
  double2 s[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) s[u] = czero();
  pi_step<0>(acc, col[0], s);
  pi_step<1>(acc, col[1], s);
  pi_step<2>(acc, col[2], s);
  pi_step<3>(acc, col[3], s);
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = s[u];
}

__device__ inline double cabs2(double2 z) { return hypot(z.x, z.y); }

__global__ __launch_bounds__(256) void adaptive_kernel(AdaptArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int item = blockIdx.x * 4 + wave;
  if (item >= a.nin) return;  // whole wavefronts leave together; no block-level barrier follows
  const int grp = lane >> 3, l = lane & 7, h = l >> 2, q4 = l & 3;
  const AdaptItem it = a.in[item];
  int cls = 0, rel = it.o;
  for (int c = 0; c < 4; ++c)
    if (a.ccount[c] > 0 && it.o >= a.cstart[c] && it.o < a.cstart[c] + a.ccount[c]) {
      cls = c;
      rel = it.o - a.cstart[c];
    }
  const int n = a.n;
  int iw, i = 0, j = 0;
  if (cls == 0) {
    iw = rel;
  } else if (cls == 1) {
    iw = rel / n;
    i = rel % n;
  } else if (cls == 2) {
    iw = rel / n;
    j = rel % n;
  } else {
    iw = rel / (n * n);
    i = (rel / n) % n;
    j = rel % n;
  }
  const bool mainl = cls == 1 || cls == 3, mainr = cls == 2 || cls == 3;
  const double w = a.L.nodes[iw];
  const double m = 0.5 * (it.ya + it.yb), hw = 0.5 * (it.yb - it.ya);
  double2 Ia[4], Ib[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) Ia[u] = Ib[u] = czero();
  double fmx = 0.0;
  for (int base = 0; base < a.nn; base += 8) {
    const int node = base + grp;
    if (node >= a.nn) continue;  // uniform over the 8-lane group
    const double y = m + hw * a.rule[node];
    const double vq = a.qa * tan(y * a.qth);
    const double cy = cos(y * a.qth);
    const double jac = a.qa * a.qth / (cy * cy);
    double2 lv[4], rv[4], col[4];
    left_vals<double2>(a.L, l, iw, i, mainl, vq, lv);
    pi_column(a.P, a.r, a.kind, w, vq, q4, col);
    apply_pi_col(col, lv);
    right_vals<double2>(a.R, l, iw, j, mainr, vq, rv);
    double2 C[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) C[u] = czero();
#pragma unroll
    for (int e = 0; e < 4; ++e) {  // C[row, q4] += (L Pi)[row, e] R[e, q4], per combination
      const int sl = 4 * h + e, sr = 4 * (e & 1) + q4;
      double2 lp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) lp[u] = make_double2(__shfl(lv[u].x, sl, 8), __shfl(lv[u].y, sl, 8));
      const double2 ra = make_double2(__shfl(rv[e < 2 ? 0 : 2].x, sr, 8), __shfl(rv[e < 2 ? 0 : 2].y, sr, 8));
      const double2 rb = make_double2(__shfl(rv[e < 2 ? 1 : 3].x, sr, 8), __shfl(rv[e < 2 ? 1 : 3].y, sr, 8));
      C[0] = cadd(C[0], cmul(lp[0], ra));
      C[1] = cadd(C[1], cmul(lp[1], rb));
      C[2] = cadd(C[2], cmul(lp[2], ra));
      C[3] = cadd(C[3], cmul(lp[3], rb));
    }
    const double fa = hw * jac * a.rule[13 + node], fb = hw * jac * a.rule[26 + node];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Ia[u] = cadd(Ia[u], cscale(fa, C[u]));
      Ib[u] = cadd(Ib[u], cscale(fb, C[u]));
    }
    // size of the integrand (times the Jacobian) in X, Y, for a vanishing error scale
    const double2 X0 = cadd(cscale(a.unmix[0], C[0]), cscale(a.unmix[1], C[1]));
    const double2 Y0 = cadd(cscale(a.unmix[2], C[0]), cscale(a.unmix[3], C[1]));
    const double2 X1 = cadd(cscale(a.unmix[0], C[2]), cscale(a.unmix[1], C[3]));
    const double2 Y1 = cadd(cscale(a.unmix[2], C[2]), cscale(a.unmix[3], C[3]));
    fmx = fmax(fmx, jac * fmax(fmax(cabs2(X0), cabs2(Y0)), fmax(cabs2(X1), cabs2(Y1))));
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) {
      Ia[u].x += __shfl_xor(Ia[u].x, off);
      Ia[u].y += __shfl_xor(Ia[u].y, off);
      Ib[u].x += __shfl_xor(Ib[u].x, off);
      Ib[u].y += __shfl_xor(Ib[u].y, off);
    }
  // X, Y of this lane's two flat indices f = 4h + q4 (row h) and 8 + 4h + q4 (row 2 + h)
  double2 Xa[2], Ya[2], Xb[2], Yb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    Xa[t] = cadd(cscale(a.unmix[0], Ia[2 * t]), cscale(a.unmix[1], Ia[2 * t + 1]));
    Ya[t] = cadd(cscale(a.unmix[2], Ia[2 * t]), cscale(a.unmix[3], Ia[2 * t + 1]));
    Xb[t] = cadd(cscale(a.unmix[0], Ib[2 * t]), cscale(a.unmix[1], Ib[2 * t + 1]));
    Yb[t] = cadd(cscale(a.unmix[2], Ib[2 * t]), cscale(a.unmix[3], Ib[2 * t + 1]));
  }
  if (a.phase == 0) {
    double sc = fmax(fmax(cabs2(Xa[0]), cabs2(Ya[0])), fmax(cabs2(Xa[1]), cabs2(Ya[1])));
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      sc = fmax(sc, __shfl_xor(sc, off));
      fmx = fmax(fmx, __shfl_xor(fmx, off));
    }
    if (sc == 0.0) sc = (it.yb - it.ya) * fmx;
    if (sc == 0.0) sc = 1.0;
    if (lane == 0) a.scale[it.o] = sc;
    return;
  }
  double err = fmax(fmax(cabs2(csub(Xb[0], Xa[0])), cabs2(csub(Yb[0], Ya[0]))),
                    fmax(cabs2(csub(Xb[1], Xa[1])), cabs2(csub(Yb[1], Ya[1]))));
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) err = fmax(err, __shfl_xor(err, off));
  const bool accept = err <= a.eps * a.scale[it.o] || it.yb - it.ya < a.min_width || it.depth >= a.max_depth;
  if (accept) {
    if (lane < 8) {
      const size_t nn = n;
      size_t base;
      if (cls == 0)
        base = (size_t)iw;
      else if (cls == 1)
        base = (size_t)iw * nn + i;
      else if (cls == 2)
        base = (size_t)iw * nn + j;
      else
        base = ((size_t)iw * nn + i) * nn + j;
      const size_t sstride = cls == 0 ? nn : (cls == 3 ? nn * nn * nn : nn * nn);
      double2* out = cls == 0 ? a.K[0] : (cls == 1 ? a.K[1] : (cls == 2 ? a.K[2] : a.K[3]));
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const size_t f = 8 * t + 4 * h + q4;
        double* px = (double*)(out + base * 16 + f);
        double* py = (double*)(out + (sstride + base) * 16 + f);
        atomicAdd(px, Xb[t].x);
        atomicAdd(px + 1, Xb[t].y);
        atomicAdd(py, Yb[t].x);
        atomicAdd(py + 1, Yb[t].y);
      }
    }
  } else if (lane == 0) {
    const int pos = atomicAdd(a.nout, 6);
    if (pos + 6 <= a.cap) {
      double yk[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) yk[k] = m + hw * a.rule[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        AdaptItem c;
        c.ya = yk[k];
        c.yb = yk[k + 1];
        c.o = it.o;
        c.depth = it.depth + 1;
        a.out[pos + k] = c;
      }
    } else {
      atomicMax(a.overflow, 1);
    }
  }
}

// ======================================================================== epilogue
// Undo the spin diagonalisation (channel prefactors +1, 1/2, -1 included) and store
// the element at panel position (row, col) of transfer frequency iw into its class.
__device__ inline void epilogue_store(const GemmArgs& g, int b, int row, int col, double2 P0, double2 P1) {
  const int n = g.n;
  const int Mtot = 4 * (n + 1);
  if (row >= Mtot || col >= Mtot) return;
  // (X, Y) = unmix . (P0, P1), the inverse combination with the channel prefactor
  double2 X = make_double2(g.unmix[0] * P0.x + g.unmix[1] * P1.x, g.unmix[0] * P0.y + g.unmix[1] * P1.y);
  double2 Y = make_double2(g.unmix[2] * P0.x + g.unmix[3] * P1.x, g.unmix[2] * P0.y + g.unmix[3] * P1.y);
  const int i = row >> 2, j = col >> 2, f = 4 * (row & 3) + (col & 3);
  const int iw = g.iw0 + b;
  double2* base;
  size_t sstride;
  size_t off;
  if (i < n && j < n) {
    if (!(g.cmask & 8) || !g.K3) return;
    base = g.K3;
    sstride = (size_t)n * n * n * 16;
    off = (((size_t)iw * n + i) * n + j) * 16 + f;
  } else if (i < n) {
    if (!(g.cmask & 2) || !g.K2) return;
    base = g.K2;
    sstride = (size_t)n * n * 16;
    off = ((size_t)iw * n + i) * 16 + f;
  } else if (j < n) {
    if (!(g.cmask & 4) || !g.K2p) return;
    base = g.K2p;
    sstride = (size_t)n * n * 16;
    off = ((size_t)iw * n + j) * 16 + f;
  } else {
    if (!(g.cmask & 1) || !g.K1) return;
    base = g.K1;
    sstride = (size_t)n * 16;
    off = (size_t)iw * 16 + f;
  }
  double2* px = base + off;
  double2* py = base + sstride + off;
  if (g.beta) {
    X = cadd(X, *px);
    Y = cadd(Y, *py);
  }
  *px = X;
  *py = Y;
}

// Workgroups are dispatched round-robin over the eight XCDs (block id mod 8), each with
// its own L2.  Give every XCD a contiguous range of logical tiles -- consecutive tiles of
// one transfer frequency, row-major -- so that the workgroups sharing an A row strip or a
// B column strip run on the same XCD at the same time and reuse it from that L2 (padding
// blocks of the last XCD find a transfer frequency index >= nb and exit).
constexpr int kXcds = 8;

// ======================================================================== FP64 GEMM
// One spin combination per workgroup (grid = both combinations x tiles, combination-major,
// XCD-spread as the split kernel), 64x64 complex tile, four waves of 32x32 on
// v_mfma_f64_16x16x4f64 (lane l: A row l%16 / k l/16, B k l/16 / col l%16, D rows 4v + l/16,
// col l%16); three real products per complex multiply-add (Gauss), as in the split-FP32
// kernel.  K blocks of 16 complex through a single LDS buffer (34 KB), so three workgroups
// share a CU; waves raise their issue priority while they run MFMAs; a wave whose 32-row or
// 32-column block lies wholly past the ragged edge skips its MFMAs.  The combination's product
// goes to the workspace P[c][w][row][col]; unmix_kernel undoes the spin diagonalisation.
namespace f64g {
constexpr int BM = 64, BK = 16, LDP = BM + 2;
}

__global__ __launch_bounds__(256, 3) void zgemm_f64_kernel(GemmArgs g) {
  using namespace f64g;
  __shared__ double sA[2][BK][LDP];
  __shared__ double sB[2][BK][LDP];
  const int tiles = g.tms * g.tns;
  const int total = 2 * g.nb * tiles;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  const int c = logical >= g.nb * tiles ? 1 : 0;  // combination-major order
  logical -= c * g.nb * tiles;
  const int b = logical / tiles;
  if (b >= g.nb) return;
  const int t = logical - b * tiles;
  const int tm = g.tm0 + t / g.tns, tn = g.tn0 + t % g.tns;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const int Mtot = g.M, Kp = g.Kp;
  const int arow = min(tm * BM + lrow, Mtot - 1);
  const int brow = min(tn * BM + lrow, Mtot - 1);
  const int nk = Kp / BK;
  const bool live = tm * BM + wm * 32 < Mtot && tn * BM + wn * 32 < Mtot;
  const double2* Ap = (const double2*)g.A[c] + (size_t)b * g.strideA + (size_t)arow * Kp + lk;
  const double2* Bp = (const double2*)g.B[c] + (size_t)b * g.strideB + (size_t)brow * Kp + lk;
  d4 p[3][2][2];  // Gauss products ar br, ai bi, (ar + ai)(br + bi)
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) p[x][mb][nb] = d4{0.0, 0.0, 0.0, 0.0};
  double2 ra[4], rb[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    ra[e] = Ap[e];
    rb[e] = Bp[e];
  }
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sA[0][lk + e][lrow] = ra[e].x;
      sA[1][lk + e][lrow] = ra[e].y;
      sB[0][lk + e][lrow] = rb[e].x;
      sB[1][lk + e][lrow] = rb[e].y;
    }
  };
  stash();
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    if (kb + 1 < nk) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ra[e] = Ap[(size_t)(kb + 1) * BK + e];
        rb[e] = Bp[(size_t)(kb + 1) * BK + e];
      }
    }
    if (live) {
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        double ar[2], ai[2], br[2], bi[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          ar[mb] = sA[0][kr][wm * 32 + mb * 16 + (lane & 15)];
          ai[mb] = sA[1][kr][wm * 32 + mb * 16 + (lane & 15)];
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          br[nb] = sB[0][kr][wn * 32 + nb * 16 + (lane & 15)];
          bi[nb] = sB[1][kr][wn * 32 + nb * 16 + (lane & 15)];
        }
        double sa[2], sb[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          sa[u] = ar[u] + ai[u];
          sb[u] = br[u] + bi[u];
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            p[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[mb], br[nb], p[0][mb][nb], 0, 0, 0);
            p[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[mb], bi[nb], p[1][mb][nb], 0, 0, 0);
            p[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[mb], sb[nb], p[2][mb][nb], 0, 0, 0);
          }
      }
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();  // every wave is done with this block
    if (kb + 1 < nk) stash();
    __syncthreads();
  }
  double2* P = g.P[c] + (size_t)b * Mtot * Mtot;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tm * BM + wm * 32 + mb * 16 + 4 * v + (lane >> 4);
        const int col = tn * BM + wn * 32 + nb * 16 + (lane & 15);
        const double re = p[0][mb][nb][v] - p[1][mb][nb][v];
        const double im = p[2][mb][nb][v] - p[0][mb][nb][v] - p[1][mb][nb][v];
        if (row < Mtot && col < Mtot) P[(size_t)row * Mtot + col] = make_double2(re, im);
      }
}

// ======================================================================== split-FP32 GEMM
// FP32 operands on v_mfma_f32_32x32x2f32, one spin combination per workgroup (grid = both
// combinations x tiles), 64x64 complex tile, four waves of 32x32 complex (lane l: A row l%32 /
// k l/32; D rows 8(v/4) + 4(l/32) + v%4, col l%32).  K blocks of 32 complex staged through a
// single LDS buffer of (re, im) pairs -- 33 KB, so three workgroups share a CU and one's MFMAs
// cover another's staging and barriers -- with the next block's global loads in registers and
// each step's LDS operands read one step ahead; waves raise their issue priority while they
// run MFMAs.  A wave whose 32-row or 32-column block lies past the ragged edge skips its MFMAs.  Complex products by three real products (Gauss): P1 = ar br,
// P2 = ai bi, P3 = (ar + ai)(br + bi), Re = P1 - P2, Im = P3 - P1 - P2 -- 6 instead of 8 real
// flops per complex multiply-add.  FP32 partial sums over four K blocks (128 complex terms),
// promoted to FP64.  The combination's product goes to the workspace P[c][w][row][col];
// unmix_kernel then undoes the spin diagonalisation into the classes.
namespace f32g {
constexpr int BM = 64, BK = 32, LDP = BM + 1;  // odd pitch: conflict-free transposed LDS stores
constexpr int PROMO = 4;                      // K blocks per FP64 promotion
}

__global__ __launch_bounds__(256, 3) void zgemm_f32_kernel(GemmArgs g) {
  using namespace f32g;
  __shared__ float2 sA[BK][LDP];  // (re, im) pairs: one 8-byte LDS access per operand and step
  __shared__ float2 sB[BK][LDP];
  const int tiles = g.tms * g.tns;
  const int total = 2 * g.nb * tiles;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  const int c = logical >= g.nb * tiles ? 1 : 0;  // combination-major order
  logical -= c * g.nb * tiles;
  const int b = logical / tiles;
  if (b >= g.nb) return;
  const int t = logical - b * tiles;
  const int tm = g.tm0 + t / g.tns, tn = g.tn0 + t % g.tns;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lrow = tid >> 2, lk = (tid & 3) * 8;
  const int Mtot = g.M, Kp = g.Kp;
  const int arow = min(tm * BM + lrow, Mtot - 1);
  const int brow = min(tn * BM + lrow, Mtot - 1);
  const int nk = Kp / BK;
  const int am = wm * 32 + (lane & 31), bn = wn * 32 + (lane & 31);
  // a wave whose 32-row or 32-column block lies wholly past the ragged edge of the product
  // only helps stage the operands (its MFMAs would produce discarded entries)
  const bool live = tm * BM + wm * 32 < Mtot && tn * BM + wn * 32 < Mtot;
  double acc[2][16];  // [re/im][v]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[x][v] = 0.0;
  const float2* Ap = (const float2*)g.A[c] + (size_t)b * g.strideA + (size_t)arow * Kp + lk;
  const float2* Bp = (const float2*)g.B[c] + (size_t)b * g.strideB + (size_t)brow * Kp + lk;
  float2 ra[8], rb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    ra[e] = Ap[e];
    rb[e] = Bp[e];
  }
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      sA[lk + e][lrow] = ra[e];
      sB[lk + e][lrow] = rb[e];
    }
  };
  stash();
  __syncthreads();
  f16v p1, p2, p3;
#pragma unroll
  for (int v = 0; v < 16; ++v) p1[v] = p2[v] = p3[v] = 0.f;
  for (int kb = 0; kb < nk; ++kb) {
    if (kb + 1 < nk) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        ra[e] = Ap[(size_t)(kb + 1) * BK + e];
        rb[e] = Bp[(size_t)(kb + 1) * BK + e];
      }
    }
    if (live) {
      __builtin_amdgcn_s_setprio(1);  // waves in their MFMA phase issue ahead of staging waves
      float ar[2], ai[2], br[2], bi[2];
      {
        const float2 x = sA[lane >> 5][am], y = sB[lane >> 5][bn];
        ar[0] = x.x;
        ai[0] = x.y;
        br[0] = y.x;
        bi[0] = y.y;
      }
#pragma unroll
      for (int kk = 0; kk < BK / 2; ++kk) {
        const int cur = kk & 1, nx = cur ^ 1;
        if (kk + 1 < BK / 2) {
          const int kr = (kk + 1) * 2 + (lane >> 5);
          const float2 x = sA[kr][am], y = sB[kr][bn];
          ar[nx] = x.x;
          ai[nx] = x.y;
          br[nx] = y.x;
          bi[nx] = y.y;
        }
        p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[cur], br[cur], p1, 0, 0, 0);
        p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[cur], bi[cur], p2, 0, 0, 0);
        p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[cur] + ai[cur], br[cur] + bi[cur], p3, 0, 0, 0);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();  // every wave is done with this block
    if (kb + 1 < nk) stash();
    __syncthreads();
    if (kb % PROMO == PROMO - 1 || kb + 1 == nk) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[0][v] += (double)(p1[v] - p2[v]);
        acc[1][v] += (double)(p3[v] - p1[v] - p2[v]);
        p1[v] = p2[v] = p3[v] = 0.f;
      }
    }
  }
  double2* P = g.P[c] + (size_t)b * Mtot * Mtot;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = tm * BM + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int col = tn * BM + wn * 32 + (lane & 31);
    if (row < Mtot && col < Mtot) P[(size_t)row * Mtot + col] = make_double2(acc[0][v], acc[1][v]);
  }
}

// The two combinations' products of the GEMM's tile range into the classes (epilogue_store).
__global__ __launch_bounds__(256) void unmix_kernel(GemmArgs g) {
  const int Mtot = g.M;
  const int r0 = g.tm0 * 64, r1 = min((g.tm0 + g.tms) * 64, Mtot);
  const int c0 = g.tn0 * 64, c1 = min((g.tn0 + g.tns) * 64, Mtot);
  const long rows = r1 - r0, cols = c1 - c0;
  const long total = (long)g.nb * rows * cols;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int col = c0 + (int)(e % cols);
    const int row = r0 + (int)((e / cols) % rows);
    const int b = (int)(e / (cols * rows));
    const size_t off = ((size_t)b * Mtot + row) * Mtot + col;
    epilogue_store(g, b, row, col, g.P[0][off], g.P[1][off]);
  }
}

// ======================================================================== border-row product
// A bubble whose outputs are only the classes of the border row block (K1 and K2': the bare
// vertex or another constant-in-v vertex on the left, as in the Schwinger-Dyson bubble
// B_a(Gamma_0, Gamma)) needs the four rows 4n .. 4n+3 of C = A B only.  One wavefront per
// output column and transfer frequency streams the B^T panel row once (HBM-bound: the panel is
// read exactly once) against the four A rows (L2-resident, shared by every column), both
// spin combinations, products and sums in FP64 (FP32 panels widened), a fixed-order wavefront
// reduction, and stores through the bubble epilogue -- instead of a 64-row GEMM tile of which
// 60 rows are discarded.
template <class T> __global__ __launch_bounds__(256) void rowpanel_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = g.tn0 * 64 + blockIdx.x * 4 + wave;
  const int b = blockIdx.y;
  const int c1 = min((g.tn0 + g.tns) * 64, g.M);
  if (col >= c1) return;  // whole wavefronts
  const size_t rowA = 4 * (size_t)g.n;
  double2 acc[2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int h = 0; h < 4; ++h) acc[c][h] = czero();
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T* A = (const T*)g.A[c] + (size_t)b * g.strideA + rowA * g.Kp;
    const T* B = (const T*)g.B[c] + (size_t)b * g.strideB + (size_t)col * g.Kp;
    for (int k = lane; k < g.Kp; k += 64) {
      const T bv = B[k];
      const double2 y = make_double2((double)bv.x, (double)bv.y);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const T av = A[(size_t)h * g.Kp + k];
        acc[c][h] = cadd(acc[c][h], cmul(make_double2((double)av.x, (double)av.y), y));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        acc[c][h].x += __shfl_xor(acc[c][h].x, o);
        acc[c][h].y += __shfl_xor(acc[c][h].y, o);
      }
  if (lane < 4) {
    double2 p0 = acc[0][0], p1 = acc[1][0];
#pragma unroll
    for (int h = 1; h < 4; ++h)
      if (lane == h) {
        p0 = acc[0][h];
        p1 = acc[1][h];
      }
    epilogue_store(g, b, (int)rowA + lane, col, p0, p1);
  }
}

void launch_rowpanel(const GemmArgs& g, int precision, hipStream_t s) {
  const int cols = min((g.tn0 + g.tns) * 64, g.M) - g.tn0 * 64;
  dim3 grid((unsigned)((cols + 3) / 4), (unsigned)g.nb);
  if (precision == 0)
    hipLaunchKernelGGL(rowpanel_kernel<double2>, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(rowpanel_kernel<float2>, grid, dim3(256), 0, s, g);
}

// ======================================================================== general complex GEMM
// C[b] = op(A[b]) . B[b] in FP64 complex on v_mfma_f64_16x16x4f64, row-major operands:
// op(A)[m][k] = A[m][k] (TA = false, lda = row length of A) or A[k][m] (TA = true), B[k][n],
// C[m][n] overwritten.  Arbitrary M, N, K (edges zero-filled and masked).  64x64 complex
// tile per 256-thread workgroup, four waves of 32x32, K blocks of 16 staged through a single
// LDS buffer [k][m|n] (34 KB: three workgroups per CU), three real products per complex
// multiply-add (Gauss), tiles of one
// batch entry row-major and spread over the XCDs as in the bubble GEMMs.  Used by the
// adjoint's transposed products and the Matsubara bubble.
__global__ __launch_bounds__(256, 3) void zgemm_nn_kernel(ZgemmArgs g) {
  using namespace f64g;
  __shared__ double sA[2][BK][LDP];  // single buffer: three workgroups per CU
  __shared__ double sB[2][BK][LDP];
  const int tiles = g.tiles_m * g.tiles_n;
  const int total = g.batch * tiles;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  const int b = logical / tiles;
  if (b >= g.batch) return;
  const int t = logical - b * tiles;
  const int tm = t / g.tiles_n, tn = t % g.tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const double2* A = g.A + (size_t)b * g.strideA;
  const double2* B = g.B + (size_t)b * g.strideB;
  // global -> register staging: four consecutive complex entries per thread per operand
  // A, TA = false: row m = tm*64 + tid/4, k = 4 (tid % 4) + e;  TA = true: k = tid/16, m = tm*64 + 4 (tid % 16) + e
  // B: k = tid/16, n = tn*64 + 4 (tid % 16) + e
  const int a_r = g.TA ? tid >> 4 : tid >> 2, a_c = g.TA ? (tid & 15) * 4 : (tid & 3) * 4;
  const int b_k = tid >> 4, b_n = (tid & 15) * 4;
  double2 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int m, k;
      if (g.TA) {
        k = k0 + a_r;
        m = tm * BM + a_c + e;
      } else {
        m = tm * BM + a_r;
        k = k0 + a_c + e;
      }
      ra[e] = (m < g.M && k < g.K) ? (g.TA ? A[(size_t)k * g.lda + m] : A[(size_t)m * g.lda + k]) : czero();
      const int kb = k0 + b_k, nb = tn * BM + b_n + e;
      rb[e] = (kb < g.K && nb < g.N) ? B[(size_t)kb * g.ldb + nb] : czero();
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = g.TA ? a_r : a_c + e, mm = g.TA ? a_c + e : a_r;
      sA[0][kk][mm] = ra[e].x;
      sA[1][kk][mm] = ra[e].y;
      sB[0][b_k][b_n + e] = rb[e].x;
      sB[1][b_k][b_n + e] = rb[e].y;
    }
  };
  d4 p[3][2][2];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) p[x][mb][nb] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = (g.K + BK - 1) / BK;
  // a wave whose 32-row or 32-column block lies wholly past the edge of C skips its MFMAs
  const bool live = tm * BM + wm * 32 < g.M && tn * BM + wn * 32 < g.N;
  load(0);
  stash();
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    if (kb + 1 < nk) load((kb + 1) * BK);
    if (live) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        double ar[2], ai[2], br[2], bi[2], sa[2], sb[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          ar[u] = sA[0][kr][wm * 32 + u * 16 + (lane & 15)];
          ai[u] = sA[1][kr][wm * 32 + u * 16 + (lane & 15)];
          br[u] = sB[0][kr][wn * 32 + u * 16 + (lane & 15)];
          bi[u] = sB[1][kr][wn * 32 + u * 16 + (lane & 15)];
          sa[u] = ar[u] + ai[u];
          sb[u] = br[u] + bi[u];
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            p[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[mb], br[nb], p[0][mb][nb], 0, 0, 0);
            p[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[mb], bi[nb], p[1][mb][nb], 0, 0, 0);
            p[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[mb], sb[nb], p[2][mb][nb], 0, 0, 0);
          }
      }
    }
    __syncthreads();  // every wave is done with this block
    if (kb + 1 < nk) stash();
    __syncthreads();
  }
  double2* C = g.C + (size_t)b * g.strideC;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tm * BM + wm * 32 + mb * 16 + 4 * v + (lane >> 4);
        const int col = tn * BM + wn * 32 + nb * 16 + (lane & 15);
        if (row < g.M && col < g.N)
          C[(size_t)row * g.ldc + col] =
              make_double2(p[0][mb][nb][v] - p[1][mb][nb][v], p[2][mb][nb][v] - p[0][mb][nb][v] - p[1][mb][nb][v]);
      }
}

// The same product with FP64 operands rounded to FP32 as they are staged into LDS (the split
// path's rung: FP32 operands, no hi/lo correction), v_mfma_f32_32x32x2f32 with FP32 partial
// sums over 64 complex terms promoted to FP64, FP64 output.  K blocks of 32; one 32x32
// complex block per wave (lane l: A row l%32 / k l/32; D rows 8(v/4) + 4(l/32) + v%4, col l%32).
__global__ __launch_bounds__(256, 2) void zgemm_nn_f32_kernel(ZgemmArgs g) {
  using namespace f32g;
  __shared__ float sA[2][2][BK][LDP];
  __shared__ float sB[2][2][BK][LDP];
  const int tiles = g.tiles_m * g.tiles_n;
  const int total = g.batch * tiles;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  const int b = logical / tiles;
  if (b >= g.batch) return;
  const int t = logical - b * tiles;
  const int tm = t / g.tiles_n, tn = t % g.tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const double2* A = g.A + (size_t)b * g.strideA;
  const double2* B = g.B + (size_t)b * g.strideB;
  // A, TA = false: m = tm*64 + tid/4, k = 8 (tid % 4) + e;  TA = true: k = tid/8, m = tm*64 + 8 (tid % 8) + e
  // B: k = tid/8, n = tn*64 + 8 (tid % 8) + e
  const int a_r = g.TA ? tid >> 3 : tid >> 2, a_c = g.TA ? (tid & 7) * 8 : (tid & 3) * 8;
  const int b_k = tid >> 3, b_n = (tid & 7) * 8;
  float2 ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int m, k;
      if (g.TA) {
        k = k0 + a_r;
        m = tm * BM + a_c + e;
      } else {
        m = tm * BM + a_r;
        k = k0 + a_c + e;
      }
      const double2 x =
          (m < g.M && k < g.K) ? (g.TA ? A[(size_t)k * g.lda + m] : A[(size_t)m * g.lda + k]) : czero();
      ra[e] = make_float2((float)x.x, (float)x.y);
      const int kb = k0 + b_k, nb = tn * BM + b_n + e;
      const double2 y = (kb < g.K && nb < g.N) ? B[(size_t)kb * g.ldb + nb] : czero();
      rb[e] = make_float2((float)y.x, (float)y.y);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = g.TA ? a_r : a_c + e, mm = g.TA ? a_c + e : a_r;
      sA[buf][0][kk][mm] = ra[e].x;
      sA[buf][1][kk][mm] = ra[e].y;
      sB[buf][0][b_k][b_n + e] = rb[e].x;
      sB[buf][1][b_k][b_n + e] = rb[e].y;
    }
  };
  const int am = wm * 32 + (lane & 31), bn = wn * 32 + (lane & 31);
  double acc[2][16];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[x][v] = 0.0;
  f16v p1, p2, p3;
  const int nk = (g.K + BK - 1) / BK;
  load(0);
  stash(0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if ((kb & 1) == 0)
#pragma unroll
      for (int v = 0; v < 16; ++v) p1[v] = p2[v] = p3[v] = 0.f;
    if (kb + 1 < nk) load((kb + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int kr = kk * 2 + (lane >> 5);
      const float ar = sA[buf][0][kr][am], ai = sA[buf][1][kr][am];
      const float br = sB[buf][0][kr][bn], bi = sB[buf][1][kr][bn];
      p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, p1, 0, 0, 0);
      p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, p2, 0, 0, 0);
      p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar + ai, br + bi, p3, 0, 0, 0);
    }
    if (kb + 1 < nk) stash(buf ^ 1);
    __syncthreads();
    if ((kb & 1) == 1 || kb + 1 == nk)  // FP32 partial sums of 64 complex terms -> FP64
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[0][v] += (double)(p1[v] - p2[v]);
        acc[1][v] += (double)(p3[v] - p1[v] - p2[v]);
      }
  }
  double2* C = g.C + (size_t)b * g.strideC;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = tm * BM + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int col = tn * BM + wn * 32 + (lane & 31);
    if (row < g.M && col < g.N) C[(size_t)row * g.ldc + col] = make_double2(acc[0][v], acc[1][v]);
  }
}

void launch_zgemm_nn_f32(ZgemmArgs g, hipStream_t s) {
  g.tiles_m = (g.M + 63) / 64;
  g.tiles_n = (g.N + 63) / 64;
  const long total = (long)g.batch * g.tiles_m * g.tiles_n;
  const long grid = (total + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(zgemm_nn_f32_kernel, dim3((unsigned)grid), dim3(256), 0, s, g);
}

void launch_zgemm_nn(ZgemmArgs g, hipStream_t s) {
  g.tiles_m = (g.M + 63) / 64;
  g.tiles_n = (g.N + 63) / 64;
  const long total = (long)g.batch * g.tiles_m * g.tiles_n;
  const long grid = (total + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(zgemm_nn_kernel, dim3((unsigned)grid), dim3(256), 0, s, g);
}

// ======================================================================== SDE loop
// Sigma^{a1'|a1}(v_i) = -1/2 sum_j w_j/(2 pi i) sum_{a2,a2'} [2 Phi^X + Phi^Y]
//   (w = v_i - v_j, v' = (v_i + v_j)/2) G^{a2|a2'}(v_j);  Phi = K1(w) + K2'(w, v').
// One workgroup per output frequency; shuffle + LDS reduction in FP64.
__global__ __launch_bounds__(256) void loop_kernel(LoopArgs a) {
  const int i = blockIdx.x;
  const int n = a.g.n;
  const double v = a.nodes[i];
  double2 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = czero();
  for (int jq = threadIdx.x; jq < a.nq; jq += blockDim.x) {
    const double vq = a.qv[jq];
    int iw;
    double tw;
    if (!dgrid_locate(a.g, v - vq, iw, tw)) continue;
    int ip = 0;
    double tp = 0.0;
    const bool inp = dgrid_locate(a.g, 0.5 * (v + vq), ip, tp);
    double2 Mx[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) Mx[f] = czero();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double sw = s ? 1.0 : 2.0;  // spin sum 2X + Y
#pragma unroll
      for (int cw = 0; cw < 2; ++cw) {
        const double ww = sw * (cw ? tw : 1.0 - tw);
        if (a.K1) {
          const double2* p = a.K1 + ((size_t)s * n + iw + cw) * 16;
#pragma unroll
          for (int f = 0; f < 16; ++f) Mx[f] = cfma(ww, p[f], Mx[f]);
        }
        if (inp && a.K2p) {
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2) {
            const double wv = ww * (c2 ? tp : 1.0 - tp);
            const double2* p = a.K2p + (((size_t)s * n + iw + cw) * n + ip + c2) * 16;
#pragma unroll
            for (int f = 0; f < 16; ++f) Mx[f] = cfma(wv, p[f], Mx[f]);
          }
        }
      }
    }
    double2 G[4];
    propagator(a.P, a.kind, vq, G);
    const double2 wgt = make_double2(0.0, 0.5 * a.qw[jq] * (0.5 / M_PI));  // -1/2 * w/(2 pi i)
#pragma unroll
    for (int a1p = 0; a1p < 2; ++a1p)
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1) {
        double2 s = czero();
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int a2p = 0; a2p < 2; ++a2p) {
            const int f = 4 * (2 * a1p + a2) + (2 * a1 + a2p);
            s = cadd(s, cmul(Mx[f], G[2 * a2 + a2p]));
          }
        acc[2 * a1p + a1] = cadd(acc[2 * a1p + a1], cmul(wgt, s));
      }
  }
  // reduction over the workgroup
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      acc[c].x += __shfl_xor(acc[c].x, o);
      acc[c].y += __shfl_xor(acc[c].y, o);
    }
  __shared__ double2 red[4][4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wave][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    double2 s = czero();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = cadd(s, red[w][c]);
    a.out[(size_t)i * 4 + c] = s;
  }
}

// ======================================================================== vertex loop
// L(Gamma, X)^{a1'|a1}(v_i) = sum_j w_j/(2 pi i) sum_{a2,a2'} [2 Gamma^X + Gamma^Y]
//   (legs v_i, v_j | v_i, v_j) X^{a2|a2'}(v_j),  X = G (kind 0) or S (kind 1),
// the loop function of a full vertex (Sec. "loop"): bare part plus the three channels, each
// read from its table at (w, v, v') = (v_i - v_j, (v_i + v_j)/2, (v_i + v_j)/2) in its own
// parametrization.  One workgroup per output frequency, one 8-lane group per node v_j.
__global__ __launch_bounds__(256) void vloop_kernel(VLoopArgs a) {
  const int i = blockIdx.x;
  const int l8 = threadIdx.x & 7, grp = threadIdx.x >> 3, ngrp = blockDim.x >> 3;
  const int n = a.g.n;
  const double v = a.nodes[i];
  double2 acc[4];  // output (a1', a1) at index 2 a1' + a1
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = czero();
  for (int j = grp; j < a.nq; j += ngrp) {
    const double vq = a.qv[j];
    double L[4];
    legs_of(0, v - vq, 0.5 * (v + vq), 0.5 * (v + vq), L);
    // slots: 0, 1 = (w, v) of channel a (v' = v there); 2-4 / 5-7 = (w, v, v') of p / t
    double arg;
    if (l8 < 2) {
      arg = l8 == 0 ? v - vq : 0.5 * (v + vq);
    } else {
      const int d = l8 <= 4 ? 1 : 2, which = (l8 - 2) % 3;
      double w2, v2, vp2;
      params_of(d, L, w2, v2, vp2);
      arg = which == 0 ? w2 : (which == 1 ? v2 : vp2);
    }
    int ic;
    double tc;
    if (!dgrid_locate(a.g, arg, ic, tc)) {
      ic = -1;
      tc = 0.0;
    }
    double2 g4[4];
    propagator(a.P, a.kind, vq, g4);
    double2 gam[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) gam[u] = czero();
    if (a.T[0]) {
      const int iw = __shfl(ic, 0, 8), iv = __shfl(ic, 1, 8);
      const double tw = __shfl(tc, 0, 8), tv = __shfl(tc, 1, 8);
      table_taps((const double2*)a.T[0], n, iw, tw, iv, tv, iv, tv, l8, gam);
    }
#pragma unroll
    for (int d = 0; d < 2; ++d)
      if (a.T[1 + d]) {
        const int s0 = 2 + 3 * d;
        table_taps((const double2*)a.T[1 + d], n, __shfl(ic, s0, 8), __shfl(tc, s0, 8), __shfl(ic, s0 + 1, 8),
                   __shfl(tc, s0 + 1, 8), __shfl(ic, s0 + 2, 8), __shfl(tc, s0 + 2, 8), l8, gam);
      }
    const double2 wgt = make_double2(0.0, -a.qw[j] * (0.5 / M_PI));  // w_j / (2 pi i)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = l8 + 8 * h;  // a-channel order: row (a1', a2), column (a1, a2')
      const int a1p = f >> 3, a2 = (f >> 2) & 1, a1 = (f >> 1) & 1, a2p = f & 1;
      double2 x = gam[2 * h];  // 2X + Y of the channels
      if (bare_odd(f)) x.x -= 0.5 * a.r0;  // 2 X_R + Y_R = -r0/2 on odd f
      const double2 gp = a2 ? (a2p ? g4[3] : g4[2]) : (a2p ? g4[1] : g4[0]);
      const double2 val = cmul(cmul(x, gp), wgt);
      const int idx = 2 * a1p + a1;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c == idx) acc[c] = cadd(acc[c], val);  // register-resident: no indexed store
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      acc[c].x += __shfl_xor(acc[c].x, o);
      acc[c].y += __shfl_xor(acc[c].y, o);
    }
  __shared__ double2 red[4][4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wave][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < 4) {
    double2 s = czero();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = cadd(s, red[w][threadIdx.x]);
    a.out[(size_t)i * 4 + threadIdx.x] = s;
  }
}

// ======================================================================== chi
// chi_r^c(w)[p, m] = sum_k Pi_k[p, m]
//   + sum_{k,l} sum_{row,q} Pi_k[p, row] Gamma_c(w; v''_k, v''_l)[row, q] Pi_l[q, m]
// for channel r's two spin combinations c, Pi (channel r) with the weights folded in.
// One 8-lane group per node pair (k, l), grid-stride over the pairs of one transfer
// frequency.  Lane l8 evaluates the full vertex (bare part, own classes, the other channels
// through their target-order tables) at f = l8, l8 + 8 -- rows l8/4 and 2 + l8/4, column
// q = l8 % 4 -- multiplies by Pi_l from the right through quad broadcasts and by Pi_k from
// the left for its two rows.  Per-lane partial sums, reduced over the block in a fixed tree;
// chi_finalize_kernel adds the per-block partials in fixed order (deterministic).
template <class TT> __global__ __launch_bounds__(256) void chi_kernel(ChiArgs a) {
  const int b = blockIdx.y, iw = a.iw0 + b;
  const int l8 = threadIdx.x & 7, h = l8 >> 2, q4 = l8 & 3;
  // 32-bit indices: the host keeps nq * nq below 2^31
  const unsigned grp = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const unsigned ngrp = (gridDim.x * blockDim.x) >> 3;
  const unsigned total = (unsigned)a.nq * (unsigned)a.nq;
  const int n = a.g.n;
  const size_t nn = n, n2 = nn * nn, n3 = n2 * nn;
  const double w = a.nodes[iw];
  const double2* pis = a.pi + (size_t)b * a.nq * 16;
  double2 part[2][4];  // [combination][p] for m = q4, rows h and 2 + h
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int p = 0; p < 4; ++p) part[c][p] = czero();
  for (unsigned t = grp; t < total; t += ngrp) {
    const int kq = (int)(t / (unsigned)a.nq), lq = (int)(t - (unsigned)kq * (unsigned)a.nq);
    const double vk = a.qv[kq], vl = a.qv[lq];
    // grid locations: lane 0 v''_k, lane 1 v''_l, lanes 2-4 / 5-7 (w, v, v') of channels
    // r + 1 / r + 2
    double arg = l8 == 0 ? vk : vl;
    if (l8 >= 2) {
      double L[4];
      legs_of(a.r, w, vk, vl, L);
      const int d = l8 <= 4 ? 1 : 2, which = (l8 - 2) % 3;
      double w2, v2, vp2;
      params_of((a.r + d) % 3, L, w2, v2, vp2);
      arg = which == 0 ? w2 : (which == 1 ? v2 : vp2);
    }
    int ic;
    double tc;
    if (!dgrid_locate(a.g, arg, ic, tc)) {
      ic = -1;
      tc = 0.0;
    }
    const int i0 = __shfl(ic, 0, 8), j0 = __shfl(ic, 1, 8);
    const double ti = __shfl(tc, 0, 8), tj = __shfl(tc, 1, 8);
    double2 acc[4], xy[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = xy[u] = czero();
    if (a.coef != 0.0) {  // own channel: K1(w) + K2(w, v''_k) + K2'(w, v''_l) + K3(w, v''_k, v''_l)
      if (a.K[0]) own_tap(a.K[0] + (size_t)iw * 16, nn * 16, l8, 1.0, xy);
      if (a.K[1] && i0 >= 0) {
        const double2* p = a.K[1] + ((size_t)iw * nn + i0) * 16;
        own_tap(p, n2 * 16, l8, 1.0 - ti, xy);
        own_tap(p + 16, n2 * 16, l8, ti, xy);
      }
      if (a.K[2] && j0 >= 0) {
        const double2* p = a.K[2] + ((size_t)iw * nn + j0) * 16;
        own_tap(p, n2 * 16, l8, 1.0 - tj, xy);
        own_tap(p + 16, n2 * 16, l8, tj, xy);
      }
      if (a.K[3] && i0 >= 0 && j0 >= 0) {
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
          const double2* p = a.K[3] + (((size_t)iw * nn + i0 + ci) * nn + j0) * 16;
          const double wi = ci ? ti : 1.0 - ti;
          own_tap(p, n3 * 16, l8, wi * (1.0 - tj), xy);
          own_tap(p + 16, n3 * 16, l8, wi * tj, xy);
        }
      }
    }
    own_mix(a.coef, a.mix, l8, a.r0, xy, acc);
#pragma unroll
    for (int d = 0; d < 2; ++d)
      if (a.T[d]) {
        const int s0 = 2 + 3 * d;
        table_taps((const TT*)a.T[d], n, __shfl(ic, s0, 8), __shfl(tc, s0, 8), __shfl(ic, s0 + 1, 8),
                   __shfl(tc, s0 + 1, 8), __shfl(ic, s0 + 2, 8), __shfl(tc, s0 + 2, 8), l8, acc);
      }
    apply_pi(pis + (size_t)lq * 16, q4, acc);  // (Gamma . Pi_l)[row, m]
    const double2* pk = pis + (size_t)kq * 16;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double2 P0 = pk[4 * p + h], P1 = pk[4 * p + 2 + h];
      part[0][p] = cadd(part[0][p], cadd(cmul(P0, acc[0]), cmul(P1, acc[2])));
      part[1][p] = cadd(part[1][p], cadd(cmul(P0, acc[1]), cmul(P1, acc[3])));
    }
  }
  // rows h = 0, 1 (lanes l8, l8 ^ 4), then the eight groups of the wave
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int o = 4; o < 64; o <<= 1) {
        part[c][p].x += __shfl_xor(part[c][p].x, o);
        part[c][p].y += __shfl_xor(part[c][p].y, o);
      }
  __shared__ double2 red[4][32];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < 4)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int p = 0; p < 4; ++p) red[wave][c * 16 + 4 * p + lane] = part[c][p];
  __syncthreads();
  if (threadIdx.x < 32) {
    double2 s = czero();
    for (int wv = 0; wv < 4; ++wv) s = cadd(s, red[wv][threadIdx.x]);
    a.partial[((size_t)b * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = s;
  }
}

// out[c][w][f] = sum of the block partials (fixed order) + sum_k Pi_k[f] (+ the own part)
__global__ void chi_finalize_kernel(ChiArgs a, int nblk) {
  const int b = blockIdx.x;  // transfer frequency within the batch
  const int e = threadIdx.x; // 0..31 = c*16 + f
  if (e >= 32) return;
  double2 s = czero();
  for (int k = 0; k < nblk; ++k) s = cadd(s, a.partial[((size_t)b * nblk + k) * 32 + e]);
  const int c = e >> 4, f = e & 15;
  const double2* pis = a.pi + (size_t)b * a.nq * 16;
  for (int k = 0; k < a.nq; ++k) s = cadd(s, pis[(size_t)k * 16 + f]);
  if (a.own) s = cadd(s, a.own[((size_t)b * 2 + c) * 16 + f]);
  a.out[((size_t)c * a.g.n + a.iw0 + b) * 16 + f] = s;
}

// The own channel r enters chi at (w; v''_k, v''_l) through its classes, each linear in the
// loop frequencies on the grid: K(v''_k) = sum_i c_ki K_i with the interpolation weights c_ki
// (two per k, zero beyond the grid).  So its part of sum_{k,l} Pi_k Gamma Pi_l is
//   sum_{i,j} Pt_i K3_ij Pt_j + (sum_i Pt_i K2_i) Pibar + Pibar (sum_j K2'_j Pt_j) + Pibar (K1 + R) Pibar
// with Pt_i = sum_k c_ki Pi_k and Pibar = sum_k Pi_k -- the same discrete sum reordered, O(n^2)
// instead of O(nq^2) per transfer frequency.
// chi_proj_kernel: block (node i or n, batch entry b), 64 threads = 16 entries x 4 parts of k.
__global__ __launch_bounds__(64) void chi_proj_kernel(ChiArgs a) {
  __shared__ double2 red[4][16];
  const int i = blockIdx.x, b = blockIdx.y, n = a.g.n;
  const int f = threadIdx.x & 15, part = threadIdx.x >> 4;
  const double2* pis = a.pi + (size_t)b * a.nq * 16;
  int klo = 0, khi = a.nq - 1;
  if (i < n) {  // loop nodes between the neighbouring grid nodes (sorted), widened by one
    const double lo = i > 0 ? a.nodes[i - 1] : -1e300, hi = i + 1 < n ? a.nodes[i + 1] : 1e300;
    int x = 0, y = a.nq;
    while (x < y) {  // first k with v''_k >= lo
      const int m = (x + y) >> 1;
      if (a.qv[m] < lo) x = m + 1; else y = m;
    }
    klo = max(x - 1, 0);
    x = 0;
    y = a.nq;
    while (x < y) {  // first k with v''_k > hi
      const int m = (x + y) >> 1;
      if (a.qv[m] <= hi) x = m + 1; else y = m;
    }
    khi = min(x, a.nq - 1);
  }
  double2 acc = czero();
  for (int k = klo + part; k <= khi; k += 4) {
    double w = 1.0;
    if (i < n) {
      int ic;
      double tc;
      if (!dgrid_locate(a.g, a.qv[k], ic, tc)) continue;
      w = ic == i ? 1.0 - tc : (ic + 1 == i ? tc : 0.0);
      if (w == 0.0) continue;
    }
    acc = cfma(w, pis[(size_t)k * 16 + f], acc);
  }
  red[part][f] = acc;
  __syncthreads();
  if (part == 0)
    a.pt[((size_t)b * (n + 1) + i) * 16 + f] = cadd(cadd(red[0][f], red[1][f]), cadd(red[2][f], red[3][f]));
}

// own-channel class entry f of combination c at (iw, i, j): coef (mix0 X + mix1 Y)
__device__ inline double2 own_combo(const double2* K, size_t sstride, size_t off, double coef, double m0, double m1) {
  const double2 X = K[off], Y = K[sstride + off];
  return make_double2(coef * (m0 * X.x + m1 * Y.x), coef * (m0 * X.y + m1 * Y.y));
}

// chi_own_kernel: block (combination c, batch entry b), 256 threads; dynamic LDS of
// (2n + 1) x 16 complex: Pt (n + 1 rows, the last Pibar) and W_j = sum_i Pt_i K3_ij + Pibar K2'_j.
__global__ __launch_bounds__(256) void chi_own_kernel(ChiArgs a) {
  extern __shared__ double2 lds[];
  const int c = blockIdx.x, b = blockIdx.y, n = a.g.n, iw = a.iw0 + b;
  double2* Pt = lds;                   // [n + 1][16]
  double2* W = lds + (size_t)(n + 1) * 16;  // [n][16]
  __shared__ double2 V[16];            // sum_i Pt_i K2_i + Pibar (K1 + R)
  for (int e = threadIdx.x; e < (n + 1) * 16; e += blockDim.x) Pt[e] = a.pt[(size_t)b * (n + 1) * 16 + e];
  __syncthreads();
  const double m0 = a.mix[2 * c], m1 = a.mix[2 * c + 1];
  const size_t nn = n, n2 = nn * nn, n3 = n2 * nn;
  const double2* Pb = Pt + (size_t)n * 16;
  for (int e = threadIdx.x; e < n * 16; e += blockDim.x) {
    const int j = e >> 4, p = (e >> 2) & 3, q = e & 3;
    double2 s = czero();
    if (a.coef != 0.0) {
      if (a.K[3])
        for (int i = 0; i < n; ++i)
#pragma unroll
          for (int row = 0; row < 4; ++row)
            s = cadd(s, cmul(Pt[i * 16 + 4 * p + row],
                             own_combo(a.K[3], n3 * 16, (((size_t)iw * nn + i) * nn + j) * 16 + 4 * row + q, a.coef, m0,
                                       m1)));
      if (a.K[2])
#pragma unroll
        for (int row = 0; row < 4; ++row)
          s = cadd(s, cmul(Pb[4 * p + row],
                           own_combo(a.K[2], n2 * 16, ((size_t)iw * nn + j) * 16 + 4 * row + q, a.coef, m0, m1)));
    }
    W[e] = s;
  }
  if (threadIdx.x < 16) {
    const int p = threadIdx.x >> 2, q = threadIdx.x & 3;
    double2 s = czero();
    if (a.coef != 0.0 && a.K[1])
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int row = 0; row < 4; ++row)
          s = cadd(s, cmul(Pt[i * 16 + 4 * p + row],
                           own_combo(a.K[1], n2 * 16, ((size_t)iw * nn + i) * 16 + 4 * row + q, a.coef, m0, m1)));
#pragma unroll
    for (int row = 0; row < 4; ++row) {
      const int f = 4 * row + q;
      double2 k1 = (a.coef != 0.0 && a.K[0]) ? own_combo(a.K[0], nn * 16, (size_t)iw * 16 + f, a.coef, m0, m1) : czero();
      if (bare_odd(f)) k1.x += (m1 - m0) * 0.5 * a.r0;  // the bare vertex R in combination c
      s = cadd(s, cmul(Pb[4 * p + row], k1));
    }
    V[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int p = threadIdx.x >> 2, m = threadIdx.x & 3;
    double2 s = czero();
    for (int j = 0; j < n; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) s = cadd(s, cmul(W[j * 16 + 4 * p + q], Pt[j * 16 + 4 * q + m]));
#pragma unroll
    for (int q = 0; q < 4; ++q) s = cadd(s, cmul(V[4 * p + q], Pb[4 * q + m]));
    a.own[((size_t)b * 2 + c) * 16 + threadIdx.x] = s;
  }
}

// ======================================================================== parquet helpers
// Sigma^R and Sigma^K (contiguous, for the propagator) from a self-energy [n][4]
__global__ void sigma_split_kernel(int n, const double2* sigma, double2* sigR, double2* sigK) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  sigR[i] = sigma[4 * i + 1];
  sigK[i] = sigma[4 * i + 0];
}

// per block: max |f - x| and max |f| over its grid-stride share of `count` entries
__global__ __launch_bounds__(256) void maxdiff_kernel(const double2* x, const double2* f, size_t count,
                                                      double* partial) {
  double md = 0.0, mf = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const double2 a = x[e], b = f[e];
    md = fmax(md, hypot(b.x - a.x, b.y - a.y));
    mf = fmax(mf, hypot(b.x, b.y));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    md = fmax(md, __shfl_xor(md, o));
    mf = fmax(mf, __shfl_xor(mf, o));
  }
  __shared__ double red[4][2];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[wave][0] = md;
    red[wave][1] = mf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0][0], b = red[0][1];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      a = fmax(a, red[w][0]);
      b = fmax(b, red[w][1]);
    }
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = b;
  }
}

// out = a x + b y (out may alias x or y)
__global__ __launch_bounds__(256) void axpby_kernel(double2* out, double a, const double2* x, double b,
                                                    const double2* y, size_t count) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const double2 u = x[e], v = y[e];
    out[e] = make_double2(fma(a, u.x, b * v.x), fma(a, u.y, b * v.y));
  }
}

// out = x + sum_{j < nt} c_j k_j (x may be null; out may alias x or any k_j)
__global__ __launch_bounds__(256) void lincomb_kernel(LinComb a) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.count; e += (size_t)gridDim.x * blockDim.x) {
    double2 acc = a.x ? a.x[e] : czero();
    for (int j = 0; j < a.nt; ++j) {
      const double2 u = a.k[j][e];
      acc = make_double2(fma(a.c[j], u.x, acc.x), fma(a.c[j], u.y, acc.y));
    }
    a.out[e] = acc;
  }
}

// Step error of the embedded Runge-Kutta pair: per-block max of |e| / (atol + rtol max(|y|, |y4|)),
// zero where e is zero; a NaN or infinite entry counts as +inf (fmax alone would drop NaN).
__global__ __launch_bounds__(256) void errnorm_kernel(const double2* err, const double2* y, const double2* y4,
                                                      double atol, double rtol, size_t count, double* partial) {
  double m = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const double2 d = err[e], u = y[e], w = y4[e];
    const double ad = hypot(d.x, d.y);
    double r = ad == 0.0 ? 0.0 : ad / (atol + rtol * fmax(hypot(u.x, u.y), hypot(w.x, w.y)));
    if (!(r <= 1.7976931348623157e308)) r = __builtin_inf();
    m = fmax(m, r);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = fmax(b, red[w]);
    partial[blockIdx.x] = b;
  }
}

// Per-block partial sums of Re <a, b> = sum_e (a.x b.x + a.y b.y); fixed grid and order.
__global__ __launch_bounds__(256) void dot_kernel(const double2* a, const double2* b, size_t count, double* partial) {
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const double2 u = a[e], v = b[e];
    acc = fma(u.x, v.x, fma(u.y, v.y, acc));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    partial[blockIdx.x] = t;
  }
}

// Per-block partial sums of w_j tanh(v_j/2T) Im G^R(v_j) over the quadrature nodes: the occupation
// of the Hartree term is 1/2 + (this sum)/(2 pi); fixed grid and order.
__global__ __launch_bounds__(256) void occupation_kernel(DProp P, const double* nodes, const double* weights, int nq,
                                                         double* partial) {
  double acc = 0.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nq; j += gridDim.x * blockDim.x) {
    const double v = nodes[j];
    double2 m[4];
    propagator(P, 0, v, m);
    acc = fma(weights[j] * tanh(v / (2.0 * P.T)), m[2].y, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    partial[blockIdx.x] = t;
  }
}

// linear mixing x <- x + alpha (f - x)
__global__ __launch_bounds__(256) void mix_kernel(double2* x, const double2* f, size_t count, double alpha) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const double2 a = x[e], b = f[e];
    x[e] = make_double2(fma(alpha, b.x - a.x, a.x), fma(alpha, b.y - a.y, a.y));
  }
}

// ======================================================================== adjoint
// Reverse pass of the bubble: the cotangent panel conj(dP) is built from the class
// cotangents (transpose of the epilogue), the two transposed products are batched
// ZGEMMs, and the kernels below scatter through Pi and the interpolation taps (the
// transpose of the gathers) and reduce dPi into the Delta-derivative.

__device__ inline void atomic_c(double2* p, double2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

__device__ inline void pi_index(int r, int a3, int a3p, int a4, int a4p, int& rp, int& cp) {
  if (r == 0) {
    rp = 2 * a3 + a4p;
    cp = 2 * a3p + a4;
  } else if (r == 1) {
    rp = 2 * a3 + a4;
    cp = 2 * a3p + a4p;
  } else {
    rp = 2 * a4p + a3;
    cp = 2 * a3p + a4;
  }
}

__global__ __launch_bounds__(256) void dpanel_kernel(DPanelArgs a) {
  const int n = a.n;
  const long M = 4L * (n + 1);
  const long total = (long)a.nb * M * M;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long C = e % M, R = (e / M) % M;
    const int b = (int)(e / (M * M));
    const int i = (int)(R >> 2), j = (int)(C >> 2), f = 4 * (int)(R & 3) + (int)(C & 3);
    const size_t iw = (size_t)(a.iw0 + b);
    const double2* base;
    size_t sstride, off;
    if (i < n && j < n) {
      base = a.dK3;
      sstride = (size_t)n * n * n * 16;
      off = ((iw * n + i) * n + j) * 16 + f;
    } else if (i < n) {
      base = a.dK2;
      sstride = (size_t)n * n * 16;
      off = (iw * n + i) * 16 + f;
    } else if (j < n) {
      base = a.dK2p;
      sstride = (size_t)n * n * 16;
      off = (iw * n + j) * 16 + f;
    } else {
      base = a.dK1;
      sstride = (size_t)n * 16;
      off = iw * 16 + f;
    }
    double2 dX = base ? base[off] : czero();
    double2 dY = base ? base[sstride + off] : czero();
    double2 p0 = make_double2(a.unmix[0] * dX.x + a.unmix[2] * dY.x, a.unmix[0] * dX.y + a.unmix[2] * dY.y);
    double2 p1 = make_double2(a.unmix[1] * dX.x + a.unmix[3] * dY.x, a.unmix[1] * dX.y + a.unmix[3] * dY.y);
    const size_t o = ((size_t)b * M + R) * M + C;
    a.D0[o] = cconj(p0);
    a.D1[o] = cconj(p1);
  }
}

// One thread per panel entry (row, k, m): the lane loads its own raw entry L[row][(k, m)]
// (coalesced), takes the quad's four q through quad-permute broadcasts, and writes
// A[row][(k, m)] = sum_q L[row][(k, q)] Pi_k[q][m].
__global__ __launch_bounds__(256) void apply_pi_kernel(ApplyPiArgs a) {
  const long M = 4L * (a.n + 1);
  const long total = (long)a.nb * M * a.Kp;  // Kp = 4 nq_pad: whole quads of entries
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int km = (int)(e % a.Kp), k = km >> 2, m = km & 3;
    const long R = (e / a.Kp) % M;
    const int b = (int)(e / (a.Kp * M));
    const size_t off = ((size_t)b * M + R) * a.Kp + km;
    const bool real = k < a.nq;  // padding nodes: zero (uniform per quad)
    const double2 x0 = real ? a.L0[off] : czero(), x1 = real ? a.L1[off] : czero();
    double2 s0 = czero(), s1 = czero();
    const double2* pk = a.pi + ((size_t)b * a.nq + (real ? k : 0)) * 16;
    double2 p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = real ? pk[4 * q + m] : czero();
#define KQFT_APPLY_Q(Q)                                                                        \
    {                                                                                          \
      const double2 l0 = make_double2(quad_bcast<Q>(x0.x), quad_bcast<Q>(x0.y));               \
      const double2 l1 = make_double2(quad_bcast<Q>(x1.x), quad_bcast<Q>(x1.y));               \
      s0 = cadd(s0, cmul(l0, p[Q]));                                                           \
      s1 = cadd(s1, cmul(l1, p[Q]));                                                           \
    }
    KQFT_APPLY_Q(0)
    KQFT_APPLY_Q(1)
    KQFT_APPLY_Q(2)
    KQFT_APPLY_Q(3)
#undef KQFT_APPLY_Q
    a.A0[off] = s0;
    a.A1[off] = s1;
  }
}

// Transpose of the gathers, accumulated along runs of loop nodes.  One wavefront per (row
// block i of the left panel or column block j of the right panel, transfer frequency, chunk of
// consecutive loop nodes); lane = (other channel h, spin s, Keldysh index rc of the block's
// row or column, entry e) = 2 x 2 x 4 x 4.  Each lane carries one cotangent stream d_k (the
// conj(dA) panel times conj(Pi_k) on the left, conj(dB) on the right, recombined into spin s)
// and walks the chunk's nodes in order.  Consecutive nodes share the interpolation cell of the
// other channel a few at a time and the own-channel cell about ten at a time, so the weighted
// values are summed in registers per cell corner and reach memory (FP64 atomics) only when the
// cell changes -- and then only the corners the next cell does not share, when it is one node
// further along one axis -- and at the end of the chunk; arguments off the grid (the partial classes) go
// to memory at once.  The own channel's class that does not depend on the loop node (K2 / K2'
// of the main blocks, K1 of the border) and the bare vertex's cotangent are summed over the
// chunk.

struct Corner8 {  // register accumulators of the current cell of one lane's target table
  int iw = -1, iv = 0, ivp = 0;
  double2 c[8];
};

// cell (iw, iv, ivp) of a table of n^3 records of 16 entries per spin; x = corner 4cw + 2cv + cp
__device__ __forceinline__ void flush8(double2* T, int n, int s, int f, const Corner8& q) {
  if (q.iw < 0) return;
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    const int cw = x >> 2, cv = (x >> 1) & 1, cp = x & 1;
    const size_t rec = (((size_t)s * n + q.iw + cw) * n + q.iv + cv) * n + q.ivp + cp;
    atomic_c(T + rec * 16 + f, q.c[x]);
  }
}

// one corner x of the current cell to memory
__device__ __forceinline__ void flush1(double2* T, int n, int s, int f, const Corner8& q, int x) {
  const int cw = x >> 2, cv = (x >> 1) & 1, cp = x & 1;
  const size_t rec = (((size_t)s * n + q.iw + cw) * n + q.iv + cv) * n + q.ivp + cp;
  atomic_c(T + rec * 16 + f, q.c[x]);
}

// move the accumulators to cell (jw, jv, jvp).  After a step of one node along one axis the
// four corners the two cells share keep their sums and only the other four go to memory;
// otherwise all eight do.  (Corner indices stay compile-time constants: selects, no indexed
// register array.)
__device__ __forceinline__ void move8(double2* T, int n, int s, int f, Corner8& q, int jw, int jv, int jvp) {
  const int dw = jw - q.iw, dv = jv - q.iv, dp = jvp - q.ivp;
  const bool valid = q.iw >= 0;
  int sw = 0, sv = 0, sp = 0;
  if (valid && dv == 0 && dp == 0 && (dw == 1 || dw == -1))
    sw = dw;
  else if (valid && dw == 0 && dp == 0 && (dv == 1 || dv == -1))
    sv = dv;
  else if (valid && dw == 0 && dv == 0 && (dp == 1 || dp == -1))
    sp = dp;
  if (valid) {
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const bool bw = x & 4, bv = x & 2, bp = x & 1;
      const bool kept = (sw > 0 && bw) || (sw < 0 && !bw) || (sv > 0 && bv) || (sv < 0 && !bv) ||
                        (sp > 0 && bp) || (sp < 0 && !bp);
      if (!kept) flush1(T, n, s, f, q, x);
    }
  }
  double2 nc[8];
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    double2 v = czero();
    if (x & 4) {
      if (sw < 0) v = q.c[x & 3];
    } else {
      if (sw > 0) v = q.c[x | 4];
    }
    if (x & 2) {
      if (sv < 0) v = q.c[x & 5];
    } else {
      if (sv > 0) v = q.c[x | 2];
    }
    if (x & 1) {
      if (sp < 0) v = q.c[x & 6];
    } else {
      if (sp > 0) v = q.c[x | 1];
    }
    nc[x] = v;
  }
#pragma unroll
  for (int x = 0; x < 8; ++x) q.c[x] = nc[x];
  q.iw = jw;
  q.iv = jv;
  q.ivp = jvp;
}

// partial classes of another channel (an argument off the grid, or no fused table): the
// transpose of the table taps into K1, K2, K2', K3 at once, as in the forward tables
__device__ inline void scatter_partial(double2* const dK[4], int n, int s, int f, int iw, double tw, bool inv,
                                       int iv, double tv, bool invp, int ivp, double tvp, double2 d) {
#pragma unroll
  for (int cw = 0; cw < 2; ++cw) {
    const double ww = cw ? tw : 1.0 - tw;
    const size_t sw = (size_t)s * n + iw + cw;
    if (dK[0]) atomic_c(dK[0] + sw * 16 + f, cscale(ww, d));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (inv && dK[1]) atomic_c(dK[1] + (sw * n + iv + c) * 16 + f, cscale(ww * (c ? tv : 1.0 - tv), d));
      if (invp && dK[2]) atomic_c(dK[2] + (sw * n + ivp + c) * 16 + f, cscale(ww * (c ? tvp : 1.0 - tvp), d));
      if (inv && invp && dK[3])
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2)
          atomic_c(dK[3] + ((sw * n + iv + c) * n + ivp + c2) * 16 + f,
                   cscale(ww * (c ? tv : 1.0 - tv) * (c2 ? tvp : 1.0 - tvp), d));
    }
  }
}

template <bool LEFT>
__global__ __launch_bounds__(256) void adj_run_kernel(AdjScatterArgs a, int chunk) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = lane & 3, rc = (lane >> 2) & 3, s = (lane >> 4) & 1, h = lane >> 5;
  const int i = blockIdx.x, b = blockIdx.y;
  const int k0 = (blockIdx.z * 4 + wv) * chunk;
  if (k0 >= a.nq) return;  // a whole wavefront; the kernel has no barriers
  const int k1 = min(a.nq, k0 + chunk);
  const int n = a.V.g.n, iw = a.iw0 + b, r = a.r;
  const size_t M = 4 * (size_t)(n + 1), nn = n;
  const double w = a.nodes[iw];
  const bool mainb = i < n;
  // entry of the lane in the own channel's Keldysh order (row rc / column rc of the block)
  const int fo = LEFT ? 4 * rc + e : 4 * e + rc;
  const double co = a.V.ch[r].coef;
  double2* const* dKo = a.dK[r];
  // own class along the loop node: K3 (main) or K2' (left border) / K2 (right border)
  double2* tapT = nullptr;
  size_t tapBase = 0, tapStep = 16;
  // own class constant along the loop node: K2 / K2' (main) or K1 (border)
  double2* cT = nullptr;
  size_t cOff = 0;
  if (co != 0.0 && h == 0) {
    if (mainb) {
      tapT = dKo[3];
      tapBase = LEFT ? ((((size_t)s * nn + iw) * nn + i) * nn) * 16 : ((((size_t)s * nn + iw) * nn) * nn + i) * 16;
      tapStep = LEFT ? 16 : nn * 16;
      cT = LEFT ? dKo[1] : dKo[2];
      cOff = (((size_t)s * nn + iw) * nn + i) * 16;
    } else {
      tapT = LEFT ? dKo[2] : dKo[1];
      tapBase = (((size_t)s * nn + iw) * nn) * 16;
      tapStep = 16;
      cT = dKo[0];
      cOff = ((size_t)s * nn + iw) * 16;
    }
  }
  int tj = -1;  // current own cell (node index along v'')
  double2 t0 = czero(), t1 = czero(), cacc = czero();
  double racc = 0.0;
  const bool bare = !mainb && bare_odd(fo) && h == 0;
  // other channel r + 1 + h (main blocks only)
  const int r2 = (r + 1 + h) % 3;
  const double co2 = a.V.ch[r2].coef;
  const bool oth = mainb && co2 != 0.0;
  const int f2 = c_perm[r][r2][fo];
  double2* const dKf2 = a.dKf[r2];
  Corner8 q;
#pragma unroll
  for (int x = 0; x < 8; ++x) q.c[x] = czero();
  const double vfix = a.nodes[min(i, n - 1)];
  for (int k = k0; k < k1; ++k) {
    const size_t off = ((size_t)b * M + 4 * (size_t)i + rc) * a.Kp + 4 * (size_t)k;
    double2 l0, l1;
    if (LEFT) {
      const double2* pk = a.pi + ((size_t)b * a.nq + k) * 16;
      l0 = l1 = czero();
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double2 cp = cconj(pk[4 * e + m]);
        l0 = cadd(l0, cmul(cconj(a.G0[off + m]), cp));
        l1 = cadd(l1, cmul(cconj(a.G1[off + m]), cp));
      }
    } else {
      l0 = cconj(a.G0[off + e]);
      l1 = cconj(a.G1[off + e]);
    }
    const double m0 = s ? a.mix[1] : a.mix[0], m1 = s ? a.mix[3] : a.mix[2];
    const double2 d = make_double2(m0 * l0.x + m1 * l1.x, m0 * l0.y + m1 * l1.y);
    const double vq = a.qv[k];
    if (bare) racc += (s ? 0.5 : -0.5) * d.x;
    if (cT) cacc = cfma(co, d, cacc);
    if (tapT) {
      int j0;
      double t;
      if (dgrid_locate(a.V.g, vq, j0, t)) {
        if (j0 != tj) {  // a step of one node keeps the shared corner's sum
          if (tj >= 0 && j0 == tj + 1) {
            atomic_c(tapT + tapBase + (size_t)tj * tapStep + fo, t0);
            t0 = t1;
            t1 = czero();
          } else if (tj >= 0 && j0 == tj - 1) {
            atomic_c(tapT + tapBase + (size_t)(tj + 1) * tapStep + fo, t1);
            t1 = t0;
            t0 = czero();
          } else {
            if (tj >= 0) {
              atomic_c(tapT + tapBase + (size_t)tj * tapStep + fo, t0);
              atomic_c(tapT + tapBase + (size_t)(tj + 1) * tapStep + fo, t1);
            }
            t0 = t1 = czero();
          }
          tj = j0;
        }
        t0 = cfma(co * (1.0 - t), d, t0);
        t1 = cfma(co * t, d, t1);
      }
    }
    if (oth) {
      double L[4];
      if (LEFT)
        legs_of(r, w, vfix, vq, L);
      else
        legs_of(r, w, vq, vfix, L);
      double w2, v2, vp2;
      params_of(r2, L, w2, v2, vp2);
      int jw, jv = 0, jvp = 0;
      double tw, tv = 0.0, tvp = 0.0;
      if (dgrid_locate(a.V.g, w2, jw, tw)) {
        const bool inv = dgrid_locate(a.V.g, v2, jv, tv);
        const bool invp = dgrid_locate(a.V.g, vp2, jvp, tvp);
        const double2 dc = cscale(co2, d);
        if (inv && invp && dKf2) {
          if (jw != q.iw || jv != q.iv || jvp != q.ivp) move8(dKf2, n, s, f2, q, jw, jv, jvp);
#pragma unroll
          for (int x = 0; x < 8; ++x) {
            const double wt = ((x >> 2) ? tw : 1.0 - tw) * (((x >> 1) & 1) ? tv : 1.0 - tv) * ((x & 1) ? tvp : 1.0 - tvp);
            q.c[x] = cfma(wt, dc, q.c[x]);
          }
        } else {
          scatter_partial(a.dK[r2], n, s, f2, jw, tw, inv, jv, tv, invp, jvp, tvp, dc);
        }
      }
    }
  }
  if (oth && dKf2) flush8(dKf2, n, s, f2, q);
  if (tapT && tj >= 0) {
    atomic_c(tapT + tapBase + (size_t)tj * tapStep + fo, t0);
    atomic_c(tapT + tapBase + (size_t)(tj + 1) * tapStep + fo, t1);
  }
  if (cT) atomic_c(cT + cOff + fo, cacc);
  if (!mainb && a.dr0) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) racc += __shfl_xor(racc, o);
    if (lane == 0) atomicAdd(a.dr0, racc);
  }
}

// dPi_k[q][m] = sum_c sum_rows conj(L_c[row][(k,q)]) dA_c[row][(k,m)], then
// dDelta += Re sum conj(dPi_k/dDelta) dPi_k with dPi_k/dDelta by the product rule.
__global__ __launch_bounds__(256) void dpi_kernel(DPiArgs a) {
  __shared__ double2 red[4][16];
  const int k = blockIdx.x, b = blockIdx.y;
  const long M = 4L * (a.n + 1);
  double2 acc[16];
#pragma unroll
  for (int f = 0; f < 16; ++f) acc[f] = czero();
  for (long R = threadIdx.x; R < M; R += blockDim.x) {
    const size_t off = ((size_t)b * M + R) * a.Kp + 4 * (size_t)k;
    double2 l0[4], l1[4], g0[4], g1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      l0[q] = cconj(a.L0[off + q]);
      l1[q] = cconj(a.L1[off + q]);
      g0[q] = cconj(a.G0[off + q]);
      g1[q] = cconj(a.G1[off + q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[4 * q + m] = cadd(acc[4 * q + m], cadd(cmul(l0[q], g0[m]), cmul(l1[q], g1[m])));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < 16; ++f) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      acc[f].x += __shfl_xor(acc[f].x, o);
      acc[f].y += __shfl_xor(acc[f].y, o);
    }
    if (lane == 0) red[wave][f] = acc[f];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double2 dpi[16];
  for (int f = 0; f < 16; ++f) dpi[f] = cadd(cadd(red[0][f], red[1][f]), cadd(red[2][f], red[3][f]));
  const double w = a.wnodes[a.iw0 + b], vq = a.qv[k];
  double f3, f4;
  if (a.r == 1) {
    f3 = 0.5 * w + vq;
    f4 = 0.5 * w - vq;
  } else {
    f3 = vq + 0.5 * w;
    f4 = vq - 0.5 * w;
  }
  double2 G3[4], S3[4], G4[4], S4[4], dS3[4], dS4[4];
  propagator_dDelta(a.P, 0, f3, G3, S3);
  propagator_dDelta(a.P, 0, f4, G4, S4);
  if (a.kind == 1) {
    double2 t3[4], t4[4];
    propagator_dDelta(a.P, 1, f3, t3, dS3);
    propagator_dDelta(a.P, 1, f4, t4, dS4);
  }
  const double2 wgt = make_double2(0.0, -a.qw[k] * (0.5 / M_PI));
  double sum = 0.0;
  for (int a3 = 0; a3 < 2; ++a3)
    for (int a3p = 0; a3p < 2; ++a3p)
      for (int a4 = 0; a4 < 2; ++a4)
        for (int a4p = 0; a4p < 2; ++a4p) {
          int rp, cp;
          pi_index(a.r, a3, a3p, a4, a4p, rp, cp);
          const int x = 2 * a3 + a3p, y = 2 * a4 + a4p;
          double2 d;
          if (a.kind == 0)
            d = cadd(cmul(S3[x], G4[y]), cmul(G3[x], S4[y]));
          else
            d = cadd(cadd(cmul(dS3[x], G4[y]), cscale(2.0, cmul(S3[x], S4[y]))), cmul(G3[x], dS4[y]));
          d = cmul(wgt, d);
          const double2 g = dpi[4 * rp + cp];
          sum += d.x * g.x + d.y * g.y;  // Re(conj(d) g)
        }
  atomicAdd(a.dDelta, sum);
}

__global__ __launch_bounds__(256) void unfuse_kernel(UnfuseArgs a, int cls) {
  const size_t n = a.n;
  size_t total;
  if (cls == 3) total = 2 * n * n * n * 16;
  else total = 2 * n * n * 16;  // K2, K2' (K1: unfuse_k1_kernel)
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t f = e & 15;
    if (cls == 3) {
      a.dK3[e] = cadd(a.dK3[e], a.dKf[e]);
      continue;
    }
    double2 s = czero();
    if (cls == 1) {  // K2[s][w][v]: sum over v'
      const size_t swv = e >> 4;
      for (size_t vp = 0; vp < n; ++vp) s = cadd(s, a.dKf[(swv * n + vp) * 16 + f]);
      a.dK2[e] = cadd(a.dK2[e], s);
    } else {  // K2'[s][w][v']: sum over v
      const size_t vp = (e >> 4) % n, sw = (e >> 4) / n;
      for (size_t v = 0; v < n; ++v) s = cadd(s, a.dKf[((sw * n + v) * n + vp) * 16 + f]);
      a.dK2p[e] = cadd(a.dK2p[e], s);
    }
  }
}


// K1[s][w] += sum over (v, v') of the fused table: one workgroup per (s, w), sixteen slices of
// the n^2 records per entry f, summed in a fixed order (deterministic).
__global__ __launch_bounds__(256) void unfuse_k1_kernel(UnfuseArgs a) {
  __shared__ double2 part[16][16];
  const int f = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const size_t n = a.n, n2 = n * n, sw = blockIdx.x;
  const double2* src = a.dKf + sw * n2 * 16 + f;
  double2 acc = czero();
  for (size_t q = sl; q < n2; q += 16) acc = cadd(acc, src[q * 16]);
  part[sl][f] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    double2 t = czero();
#pragma unroll
    for (int x = 0; x < 16; ++x) t = cadd(t, part[x][f]);
    a.dK1[sw * 16 + f] = cadd(a.dK1[sw * 16 + f], t);
  }
}

// Transpose of loop_kernel.  With M = 2 Phi^X + Phi^Y and c = 2 a1' + a1:
//   dM[f(a1',a2',a1,a2)] = conj(wgt G^{a2|a2'}) dSigma[c],  dPhi^X = 2 dM, dPhi^Y = dM,
//   dG^{a2|a2'} = sum_c conj(wgt M[f]) dSigma[c],  dDelta += Re conj(S^{a2|a2'}) dG.
__global__ __launch_bounds__(256) void loop_adjoint_kernel(LoopAdjArgs a) {
  const int i = blockIdx.x;
  const int n = a.g.n;
  const double v = a.nodes[i];
  double2 ds[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) ds[c] = a.dsig[(size_t)i * 4 + c];
  double dD = 0.0;
  for (int jq = threadIdx.x; jq < a.nq; jq += blockDim.x) {
    const double vq = a.qv[jq];
    int iw;
    double tw;
    if (!dgrid_locate(a.g, v - vq, iw, tw)) continue;
    int ip = 0;
    double tp = 0.0;
    const bool inp = dgrid_locate(a.g, 0.5 * (v + vq), ip, tp);
    double2 Gm[4], Sm[4];
    propagator_dDelta(a.P, 0, vq, Gm, Sm);
    const double2 wgt = make_double2(0.0, 0.5 * a.qw[jq] * (0.5 / M_PI));
    // Phi at the point (for dG) and dM
    double2 Mx[16], dM[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) Mx[f] = czero();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double sw = s ? 1.0 : 2.0;
#pragma unroll
      for (int cw = 0; cw < 2; ++cw) {
        const double ww = sw * (cw ? tw : 1.0 - tw);
        if (a.K1) {
          const double2* p = a.K1 + ((size_t)s * n + iw + cw) * 16;
#pragma unroll
          for (int f = 0; f < 16; ++f) Mx[f] = cfma(ww, p[f], Mx[f]);
        }
        if (inp && a.K2p)
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2) {
            const double2* p = a.K2p + (((size_t)s * n + iw + cw) * n + ip + c2) * 16;
            const double wv = ww * (c2 ? tp : 1.0 - tp);
#pragma unroll
            for (int f = 0; f < 16; ++f) Mx[f] = cfma(wv, p[f], Mx[f]);
          }
      }
    }
#pragma unroll
    for (int a1p = 0; a1p < 2; ++a1p)
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int a2p = 0; a2p < 2; ++a2p) {
            const int f = 4 * (2 * a1p + a2) + (2 * a1 + a2p);
            const double2 d = ds[2 * a1p + a1];
            dM[f] = cmul(cconj(cmul(wgt, Gm[2 * a2 + a2p])), d);
            const double2 dg = cmul(cconj(cmul(wgt, Mx[f])), d);
            dD += Sm[2 * a2 + a2p].x * dg.x + Sm[2 * a2 + a2p].y * dg.y;
          }
    for (int s = 0; s < 2; ++s) {
      const double sw = s ? 1.0 : 2.0;
      for (int cw = 0; cw < 2; ++cw) {
        const double ww = sw * (cw ? tw : 1.0 - tw);
        if (a.dK1) {
          double2* p = a.dK1 + ((size_t)s * n + iw + cw) * 16;
          for (int f = 0; f < 16; ++f) atomic_c(p + f, cscale(ww, dM[f]));
        }
        if (inp && a.dK2p)
          for (int c2 = 0; c2 < 2; ++c2) {
            double2* p = a.dK2p + (((size_t)s * n + iw + cw) * n + ip + c2) * 16;
            const double wv = ww * (c2 ? tp : 1.0 - tp);
            for (int f = 0; f < 16; ++f) atomic_c(p + f, cscale(wv, dM[f]));
          }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dD += __shfl_xor(dD, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(a.dDelta, dD);
}

// ======================================================================== launchers
static inline unsigned blocks_for(long threads, int bs) { return (unsigned)((threads + bs - 1) / bs); }

hipError_t upload_perm(const int* host_perm) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_perm), host_perm, sizeof(int) * 3 * 3 * 16);
}

void launch_table(const TableArgs& a, bool f32, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(table_kernel<float2>, dim3(8192), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(table_kernel<double2>, dim3(8192), dim3(256), 0, s, a);
}
void launch_pi(const PiArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(pi_kernel, dim3(blocks_for((long)a.nb * a.nq, 256)), dim3(256), 0, s, a);
}
void launch_gather(const GatherArgs& a, bool left, bool f32, hipStream_t s) {
  const long threads = (long)a.nb * a.cnt * a.nq_pad * 8;
  dim3 grid(blocks_for(threads, 256));
  if (left) {
    if (f32)
      hipLaunchKernelGGL(gather_left_kernel<float2>, grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(gather_left_kernel<double2>, grid, dim3(256), 0, s, a);
  } else {
    if (f32)
      hipLaunchKernelGGL(gather_right_kernel<float2>, grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(gather_right_kernel<double2>, grid, dim3(256), 0, s, a);
  }
}
void launch_gemm(const GemmArgs& g, int precision, hipStream_t s) {
  const int total = g.nb * g.tms * g.tns;
  dim3 grid2((unsigned)(((2 * total + kXcds - 1) / kXcds) * kXcds));  // both combinations
  if (precision == 0)
    hipLaunchKernelGGL(zgemm_f64_kernel, grid2, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(zgemm_f32_kernel, grid2, dim3(256), 0, s, g);
}
void launch_unmix(const GemmArgs& g, hipStream_t s) { hipLaunchKernelGGL(unmix_kernel, dim3(4096), dim3(256), 0, s, g); }
void launch_loop(const LoopArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(loop_kernel, dim3(a.g.n), dim3(256), 0, s, a);
}
void launch_vloop(const VLoopArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(vloop_kernel, dim3(a.g.n), dim3(256), 0, s, a);
}
void launch_chi(const ChiArgs& a, hipStream_t s) {
  const int nblk = chi_blocks(a.nq);
  ChiArgs pl = a;  // the pair loop: without the own channel and the bare vertex when projected
  if (a.own) {
    const size_t lds = (size_t)(2 * a.g.n + 1) * 16 * sizeof(double2);
    (void)hipFuncSetAttribute((const void*)chi_own_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(chi_proj_kernel, dim3(a.g.n + 1, a.nb), dim3(64), 0, s, a);
    hipLaunchKernelGGL(chi_own_kernel, dim3(2, a.nb), dim3(256), lds, s, a);
    pl.coef = 0.0;
    pl.r0 = 0.0;
    for (int u = 0; u < 4; ++u) pl.K[u] = nullptr;
  }
  if (a.f32)
    hipLaunchKernelGGL(chi_kernel<float2>, dim3(nblk, a.nb), dim3(256), 0, s, pl);
  else
    hipLaunchKernelGGL(chi_kernel<double2>, dim3(nblk, a.nb), dim3(256), 0, s, pl);
  hipLaunchKernelGGL(chi_finalize_kernel, dim3(a.nb), dim3(64), 0, s, a, nblk);
}
void launch_loop_adjoint(const LoopAdjArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(loop_adjoint_kernel, dim3(a.g.n), dim3(256), 0, s, a);
}
void launch_dpanel(const DPanelArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dpanel_kernel, dim3(4096), dim3(256), 0, s, a);
}
void launch_apply_pi(const ApplyPiArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(apply_pi_kernel, dim3(4096), dim3(256), 0, s, a);
}
// about 8192 wavefronts per launch, chunks of at least 32 loop nodes
static void adj_run_grid(const AdjScatterArgs& a, dim3& grid, int& chunk) {
  const long units = (long)(a.V.g.n + 1) * a.nb;
  const long want = std::max<long>(1, std::min<long>((a.nq + 31) / 32, (8192 + units - 1) / units));
  chunk = (int)((a.nq + want - 1) / want);
  const int nchunks = (a.nq + chunk - 1) / chunk;
  grid = dim3(a.V.g.n + 1, a.nb, (nchunks + 3) / 4);
}
void launch_adj_left(const AdjScatterArgs& a, hipStream_t s) {
  dim3 grid;
  int chunk;
  adj_run_grid(a, grid, chunk);
  hipLaunchKernelGGL(adj_run_kernel<true>, grid, dim3(256), 0, s, a, chunk);
}
void launch_adj_right(const AdjScatterArgs& a, hipStream_t s) {
  dim3 grid;
  int chunk;
  adj_run_grid(a, grid, chunk);
  hipLaunchKernelGGL(adj_run_kernel<false>, grid, dim3(256), 0, s, a, chunk);
}
void launch_dpi(const DPiArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(dpi_kernel, dim3(a.nq, a.nb), dim3(256), 0, s, a);
}
void launch_unfuse(const UnfuseArgs& a, hipStream_t s) {
  if (a.dK3) hipLaunchKernelGGL(unfuse_kernel, dim3(4096), dim3(256), 0, s, a, 3);
  if (a.dK2) hipLaunchKernelGGL(unfuse_kernel, dim3(1024), dim3(256), 0, s, a, 1);
  if (a.dK2p) hipLaunchKernelGGL(unfuse_kernel, dim3(1024), dim3(256), 0, s, a, 2);
  if (a.dK1) hipLaunchKernelGGL(unfuse_k1_kernel, dim3(2 * a.n), dim3(256), 0, s, a);
}
void launch_sigma_split(int n, const double2* sigma, double2* sigR, double2* sigK, hipStream_t s) {
  hipLaunchKernelGGL(sigma_split_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, sigma, sigR, sigK);
}
void launch_maxdiff(const double2* x, const double2* f, size_t count, double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(maxdiff_kernel, dim3(nblk), dim3(256), 0, s, x, f, count, partial);
}
void launch_axpby(double2* out, double a, const double2* x, double b, const double2* y, size_t count,
                  hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(2048), dim3(256), 0, s, out, a, x, b, y, count);
}
void launch_occupation(const DProp& P, const double* nodes, const double* weights, int nq, double* partial, int nblk,
                       hipStream_t s) {
  hipLaunchKernelGGL(occupation_kernel, dim3(nblk), dim3(256), 0, s, P, nodes, weights, nq, partial);
}
void launch_adaptive(const AdaptArgs& a, hipStream_t s) {
  if (a.nin > 0) hipLaunchKernelGGL(adaptive_kernel, dim3((a.nin + 3) / 4), dim3(256), 0, s, a);
}
void launch_dot(const double2* a, const double2* b, size_t count, double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(nblk), dim3(256), 0, s, a, b, count, partial);
}
__global__ __launch_bounds__(256) void regrid_kernel(RegridArgs a) {
  const long nd = a.nd, ns = a.src.n;
  long outer = a.nspin;
  for (int d = 0; d < a.dims; ++d) outer *= nd;
  const long total = outer * a.ncomp;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % a.ncomp);
    long rest = e / a.ncomp;
    int idx[3] = {0, 0, 0};
    for (int d = a.dims - 1; d >= 0; --d) {
      idx[d] = (int)(rest % nd);
      rest /= nd;
    }
    const long sp = rest;  // spin block
    int i0[3] = {0, 0, 0};
    double t[3] = {0.0, 0.0, 0.0};
    bool in = true;
    for (int d = 0; d < a.dims; ++d) in = in && dgrid_locate(a.src, a.dst[idx[d]], i0[d], t[d]);
    double2 acc = czero();
    if (in) {
      for (int corner = 0; corner < (1 << a.dims); ++corner) {
        double w = 1.0;
        long off = sp;
        for (int d = 0; d < a.dims; ++d) {
          const int up = (corner >> d) & 1;
          w *= up ? t[d] : 1.0 - t[d];
          off = off * ns + i0[d] + up;
        }
        acc = cfma(w, a.in[off * a.ncomp + c], acc);
      }
    }
    a.out[e] = acc;
  }
}

void launch_regrid(const RegridArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(regrid_kernel, dim3(2048), dim3(256), 0, s, a);
}

void launch_lincomb(const LinComb& a, hipStream_t s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(2048), dim3(256), 0, s, a);
}
void launch_errnorm(const double2* err, const double2* y, const double2* y4, double atol, double rtol, size_t count,
                    double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(errnorm_kernel, dim3(nblk), dim3(256), 0, s, err, y, y4, atol, rtol, count, partial);
}
void launch_mix(double2* x, const double2* f, size_t count, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(mix_kernel, dim3(2048), dim3(256), 0, s, x, f, count, alpha);
}
int chi_blocks(int nq) { return (int)std::min<long>(512, std::max<long>(1, ((long)nq * nq + 255) / 256)); }

// ======================================================================== grids on the device
// Frequency-grid nodes v_i = a f(x_i theta), x_i = -1 + 2i/(n-1) (the algebraic map exactly
// odd: the upper half mirrors the lower), and the tangent-mapped Gauss-Legendre rule: the
// same recurrences as the host tables, evaluated on the device so that a caller without
// host-to-device staging can have them in its own buffer.
__global__ void grid_nodes_kernel(int n, int map, double a, double theta, double* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool mirror = map == 1 && i >= n - n / 2;
  const int j = mirror ? n - 1 - i : i;
  const double x = a * freq_of(map, (-1.0 + 2.0 * j / (n - 1)) * theta);
  v[i] = mirror ? -x : x;
}

__global__ void quad_nodes_kernel(int nq, double a, double th, double* qv, double* qw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (nq + 1) / 2) return;
  double z = cos(M_PI * (i + 0.75) / (nq + 0.5)), dp = 1.0;
  for (int it = 0; it < 100; ++it) {  // Newton on the Legendre recurrence
    double p1 = 1.0, p2 = 0.0;
    for (int j = 1; j <= nq; ++j) {
      const double p3 = p2;
      p2 = p1;
      p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    dp = nq * (z * p1 - p2) / (z * z - 1.0);
    const double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) < 1e-16) break;
  }
  double p1 = 1.0, p2 = 0.0;
  for (int j = 1; j <= nq; ++j) {
    const double p3 = p2;
    p2 = p1;
    p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
  }
  dp = nq * (z * p1 - p2) / (z * z - 1.0);
  const double gw = 2.0 / ((1.0 - z * z) * dp * dp);
  const bool centre = (nq & 1) && i == nq / 2;
  const double y = centre ? 0.0 : z;
  const double c = cos(y * th), v = a * tan(y * th), w = gw * a * th / (c * c);
  qv[nq - 1 - i] = v;
  qw[nq - 1 - i] = w;
  qv[i] = -v;
  qw[i] = w;
}

void launch_grid_nodes(int n, int map, double a, double theta, double* v, hipStream_t s) {
  hipLaunchKernelGGL(grid_nodes_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, map, a, theta, v);
}
void launch_quad_nodes(int nq, double a, double th, double* qv, double* qw, hipStream_t s) {
  hipLaunchKernelGGL(quad_nodes_kernel, dim3(blocks_for((nq + 1) / 2, 64)), dim3(64), 0, s, nq, a, th, qv, qw);
}

// ======================================================================== Matsubara formalism
// Leg indices (n1', n2', n1, n2) of channel r's (m, n, n') and back, every leg fermionic:
//   a: n2 = n, n1' = n + m, n2' = n', n1 = n' + m;  p: n1' = n, n2' = m - n - 1, n1 = n',
//   n2 = m - n' - 1;  t: n2 = n, n2' = n + m, n1' = n', n1 = n' + m.
__device__ inline void mf_legs(int r, int m, int n, int np, int L[4]) {
  if (r == 0) {
    L[0] = n + m; L[1] = np; L[2] = np + m; L[3] = n;
  } else if (r == 1) {
    L[0] = n; L[1] = m - n - 1; L[2] = np; L[3] = m - np - 1;
  } else {
    L[0] = np; L[1] = n + m; L[2] = np + m; L[3] = n;
  }
}
__device__ inline void mf_params(int r, const int L[4], int& m, int& n, int& np) {
  if (r == 0) {
    m = L[0] - L[3]; n = L[3]; np = L[1];
  } else if (r == 1) {
    m = L[0] + L[1] + 1; n = L[0]; np = L[2];
  } else {
    m = L[1] - L[3]; n = L[3]; np = L[0];
  }
}

// selected classes (bit 0 K1, 1 K2, 2 K2', 3 K3) of one channel at its own (m, n, n'), zero
// outside the boxes: XY = {X, Y}
__device__ inline void mf_chan(const MChan& c, int M, int N, int m, int n, int np, int parts, double2 XY[2]) {
  if (c.coef == 0.0 || m < -M || m > M) return;
  const size_t nb = 2 * (size_t)M + 1, nf = 2 * (size_t)N, im = (size_t)(m + M);
  const bool in_n = n >= -N && n < N, in_np = np >= -N && np < N;
  double2 acc[2] = {czero(), czero()};
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    if ((parts & 1) && c.K[0]) acc[sp] = cadd(acc[sp], c.K[0][sp * nb + im]);
    if ((parts & 2) && c.K[1] && in_n) acc[sp] = cadd(acc[sp], c.K[1][(sp * nb + im) * nf + (n + N)]);
    if ((parts & 4) && c.K[2] && in_np) acc[sp] = cadd(acc[sp], c.K[2][(sp * nb + im) * nf + (np + N)]);
    if ((parts & 8) && c.K[3] && in_n && in_np)
      acc[sp] = cadd(acc[sp], c.K[3][((sp * nb + im) * nf + (n + N)) * nf + (np + N)]);
    XY[sp] = cfma(c.coef, acc[sp], XY[sp]);
  }
}

// the other two channels of the full vertex at channel r's (m, n, n')
__device__ inline void mf_others(const MGatherArgs& a, int m, int n, int np, double2 XY[2]) {
  int L[4];
  mf_legs(a.r, m, n, np, L);
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    const int r2 = (a.r + d) % 3;
    int m2, n2, np2;
    mf_params(r2, L, m2, n2, np2);
    mf_chan(a.ch[r2], a.M, a.N, m2, n2, np2, 15, XY);
  }
}

// G(i nu_n) = 1/(i nu_n + i Delta sgn(nu_n) - Sigma(n))
__device__ inline double2 mf_G(const MGatherArgs& a, int n) {
  const double v = (2.0 * n + 1.0) * M_PI * a.T;
  double2 sg = czero();
  if (a.sigma && n >= -a.Ns && n < a.Ns) sg = a.sigma[n + a.Ns];
  const double d0 = (v + (v > 0.0 ? a.Delta : -a.Delta)) * (a.reg ? 1.0 / a.lam : 1.0);
  return cinv(make_double2(-sg.x, d0 - sg.y));
}

// X(n) of the lines: 0 G, 1 S = -i sgn(nu) G^2 + G Sigma_dot G, 2 G Sigma_dot G
__device__ inline double2 mf_line(const MGatherArgs& a, int n, int line) {
  const double2 g = mf_G(a, n);
  if (line == 0) return g;
  double2 ds = czero();
  if (a.dsigma && n >= -a.Ns && n < a.Ns) ds = a.dsigma[n + a.Ns];
  const double2 gsg = cmul(cmul(g, ds), g);
  if (line == 2) return gsg;
  const double2 g2 = cmul(g, g);
  if (a.reg) {  // G G_0^-1 G / lam^2 with G_0^-1 = i (nu + Delta sgn nu)
    const double v = (2.0 * n + 1.0) * M_PI * a.T;
    const double w = (v + (v > 0.0 ? a.Delta : -a.Delta)) / (a.lam * a.lam);
    return cadd(make_double2(-w * g2.y, w * g2.x), gsg);
  }
  const double sg = (2.0 * n + 1.0) > 0.0 ? 1.0 : -1.0;
  return cadd(make_double2(sg * g2.y, -sg * g2.x), gsg);  // -i sgn G^2
}

// first index and length of channel r's window |2n'' + 1 + s m| <= 2 Nq - 1 (s = -1 for p)
__device__ inline int mf_window_lo(int r, int m, int Nq) {
  const int sm = r == 1 ? -m : m;
  const int x = -2 * Nq - sm;  // 2 lo >= -(2Nq - 1) - 1 - s m
  return (x >= 0) ? (x + 1) / 2 : -((-x) / 2);
}
__device__ inline int mf_window_len(int m, int Nq) { return 2 * Nq - ((m & 1) ? 1 : 0); }

__global__ __launch_bounds__(256) void mf_left_kernel(MGatherArgs a) {
  const int R = 2 * a.N + 1, Kw = 2 * a.Nq;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)R * Kw;
  if (tid >= per * a.nb) return;
  const int b = (int)(tid / per), rem = (int)(tid - (long)b * per), i = rem / Kw, k = rem - i * Kw;
  const int m = a.m0 + b;
  const size_t off = (size_t)b * per + (size_t)i * Kw + k;
  if (k >= mf_window_len(m, a.Nq)) {
    a.P[0][off] = czero();
    a.P[1][off] = czero();
    return;
  }
  const int nq = mf_window_lo(a.r, m, a.Nq) + k;
  const int k1 = a.r == 1 ? nq : nq + m, k2 = a.r == 1 ? m - nq - 1 : nq;
  const double2 pi = a.kind == 1 ? cadd(cmul(mf_line(a, k1, 1), mf_G(a, k2)), cmul(mf_G(a, k1), mf_line(a, k2, 1)))
                                 : cmul(mf_G(a, k1), mf_G(a, k2));
  double2 XY[2] = {czero(), czero()};
  if (i < 2 * a.N) {  // L - L^inf: own K2(m, n) + K3(m, n, n''), the other channels
    const int n = i - a.N;
    mf_chan(a.ch[a.r], a.M, a.N, m, n, nq, 2 | 8, XY);
    mf_others(a, m, n, nq, XY);
  } else {  // L^inf = Gamma_0 + own K1(m) + K2'(m, n'')
    XY[0] = make_double2(-a.U, 0.0);
    XY[1] = make_double2(a.U, 0.0);
    mf_chan(a.ch[a.r], a.M, a.N, m, 0, nq, 1 | 4, XY);
  }
  const double2 p = cscale(a.T, pi);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double2 v = cadd(cscale(a.mix[2 * c], XY[0]), cscale(a.mix[2 * c + 1], XY[1]));
    a.P[c][off] = cmul(v, p);
  }
}

__global__ __launch_bounds__(256) void mf_right_kernel(MGatherArgs a) {
  const int R = 2 * a.N + 1, Kw = 2 * a.Nq;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)R * Kw;
  if (tid >= per * a.nb) return;
  const int b = (int)(tid / per), rem = (int)(tid - (long)b * per), k = rem / R, j = rem - k * R;
  const int m = a.m0 + b;
  const size_t off = (size_t)b * per + (size_t)k * R + j;
  if (k >= mf_window_len(m, a.Nq)) {
    a.P[0][off] = czero();
    a.P[1][off] = czero();
    return;
  }
  const int nq = mf_window_lo(a.r, m, a.Nq) + k;
  double2 XY[2] = {czero(), czero()};
  if (j < 2 * a.N) {  // R - R^inf: own K2'(m, n') + K3(m, n'', n'), the other channels
    const int np = j - a.N;
    mf_chan(a.ch[a.r], a.M, a.N, m, nq, np, 4 | 8, XY);
    mf_others(a, m, nq, np, XY);
  } else {  // R^inf = Gamma_0 + own K1(m) + K2(m, n'')
    XY[0] = make_double2(-a.U, 0.0);
    XY[1] = make_double2(a.U, 0.0);
    mf_chan(a.ch[a.r], a.M, a.N, m, nq, 0, 1 | 2, XY);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) a.P[c][off] = cadd(cscale(a.mix[2 * c], XY[0]), cscale(a.mix[2 * c + 1], XY[1]));
}

__global__ __launch_bounds__(256) void mf_epilogue_kernel(MEpiArgs a) {
  const int R = 2 * a.N + 1, nf = 2 * a.N;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)R * R;
  if (tid >= per * a.nb) return;
  const int b = (int)(tid / per), rem = (int)(tid - (long)b * per), i = rem / R, j = rem - i * R;
  const double2 P0 = a.C[0][tid], P1 = a.C[1][tid];
  const double2 XY[2] = {cadd(cscale(a.unmix[0], P0), cscale(a.unmix[1], P1)),
                         cadd(cscale(a.unmix[2], P0), cscale(a.unmix[3], P1))};
  const size_t nb = 2 * (size_t)a.M + 1, im = (size_t)(a.m0 + b + a.M);
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    if (i < nf && j < nf) {
      if (a.K[3]) a.K[3][((sp * nb + im) * nf + i) * nf + j] = XY[sp];
    } else if (i < nf) {
      if (a.K[1]) a.K[1][(sp * nb + im) * nf + i] = XY[sp];
    } else if (j < nf) {
      if (a.K[2]) a.K[2][(sp * nb + im) * nf + j] = XY[sp];
    } else {
      if (a.K[0]) a.K[0][sp * nb + im] = XY[sp];
    }
  }
}

// one thread per output frequency; the sum runs in a fixed order (deterministic)
__global__ __launch_bounds__(256) void mf_loop_kernel(MLoopArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * a.N) return;
  const int n = i - a.N;
  const size_t nb = 2 * (size_t)a.M + 1, nf = 2 * (size_t)a.N;
  double2 acc = czero();
  for (int k = -a.Nl; k < a.Nl; ++k) {
    const int m = n - k;
    if (m < -a.M || m > a.M) continue;
    const size_t im = (size_t)(m + a.M);
    double2 X = a.K1[im], Y = a.K1[nb + im];
    if (k >= -a.N && k < a.N) {
      X = cadd(X, a.K2p[im * nf + (k + a.N)]);
      Y = cadd(Y, a.K2p[(nb + im) * nf + (k + a.N)]);
    }
    const double v = (2.0 * k + 1.0) * M_PI * a.T;
    double2 sg = czero();
    if (a.sigma && k >= -a.Ns && k < a.Ns) sg = a.sigma[k + a.Ns];
    const double d0 = (v + (v > 0.0 ? a.Delta : -a.Delta)) * (a.reg ? 1.0 / a.lam : 1.0);
    const double2 g = cinv(make_double2(-sg.x, d0 - sg.y));
    acc = cadd(acc, cmul(cadd(cscale(2.0, X), Y), g));
  }
  a.out[i] = cscale(-0.5 * a.T, acc);
}

// one wavefront per output frequency: the lanes stride over the summation index, then a
// fixed-order LDS reduction (deterministic)
__global__ __launch_bounds__(64) void mf_vloop_kernel(MGatherArgs a, int line, int Nl, double2* out) {
  const int i = blockIdx.x;
  const int n = i - a.N;
  double2 acc = czero();
  for (int k = -Nl + (int)threadIdx.x; k < Nl; k += 64) {
    // legs (n, k | n, k) in channel a: m = n - k, n_a = k, n'_a = k
    const int m = n - k;
    double2 XY[2] = {make_double2(-a.U, 0.0), make_double2(a.U, 0.0)};
    mf_chan(a.ch[0], a.M, a.N, m, k, k, 15, XY);
    mf_others(a, m, k, k, XY);
    acc = cadd(acc, cmul(cadd(cscale(2.0, XY[0]), XY[1]), mf_line(a, k, line)));
  }
  __shared__ double2 red[64];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = cscale(a.T, red[0]);
}

void launch_mf_vloop(const MGatherArgs& v, int line, int Nl, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(mf_vloop_kernel, dim3((unsigned)(2 * v.N)), dim3(64), 0, s, v, line, Nl, out);
}

void launch_mf_loop(const MLoopArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mf_loop_kernel, dim3((unsigned)((2 * a.N + 255) / 256)), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void mf_tail_kernel(MTailArgs a) {
  const int R = 2 * a.N + 1, nf = 2 * a.N;
  const long per = (long)R * R;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nbos = 2L * a.M + 1;
  if (tid >= per * nbos) return;
  const int im = (int)(tid / per), rem = (int)(tid - (long)im * per), i = rem / R, j = rem - i * R;
  const int m = im - a.M;
  // left row: K2(m, n_i) for i < 2N, Gamma_0 + K1(m) on the border; right column alike with K2'
  double2 lxy[2] = {czero(), czero()}, rxy[2] = {czero(), czero()};
  if (i < nf) {
    mf_chan(a.L, a.M, a.N, m, i - a.N, 0, 2, lxy);
  } else {
    lxy[0] = make_double2(-a.UL, 0.0);
    lxy[1] = make_double2(a.UL, 0.0);
    mf_chan(a.L, a.M, a.N, m, 0, 0, 1, lxy);
  }
  if (j < nf) {
    mf_chan(a.R, a.M, a.N, m, 0, j - a.N, 4, rxy);
  } else {
    rxy[0] = make_double2(-a.UR, 0.0);
    rxy[1] = make_double2(a.UR, 0.0);
    mf_chan(a.R, a.M, a.N, m, 0, 0, 1, rxy);
  }
  double2 P[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double2 l = cadd(cscale(a.mix[2 * c], lxy[0]), cscale(a.mix[2 * c + 1], lxy[1]));
    const double2 r = cadd(cscale(a.mix[2 * c], rxy[0]), cscale(a.mix[2 * c + 1], rxy[1]));
    P[c] = cmul(cmul(l, a.t[im]), r);
  }
  const double2 XY[2] = {cadd(cscale(a.unmix[0], P[0]), cscale(a.unmix[1], P[1])),
                         cadd(cscale(a.unmix[2], P[0]), cscale(a.unmix[3], P[1]))};
  const size_t nb = (size_t)nbos;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    double2* o;
    if (i < nf && j < nf) {
      o = a.K[3] + ((sp * nb + im) * nf + i) * nf + j;
    } else if (i < nf) {
      o = a.K[1] + (sp * nb + im) * nf + i;
    } else if (j < nf) {
      o = a.K[2] + (sp * nb + im) * nf + j;
    } else {
      o = a.K[0] + sp * nb + im;
    }
    *o = cadd(*o, XY[sp]);
  }
}

__global__ __launch_bounds__(256) void mf_chi_kernel(MGatherArgs a, double2* out) {
  const int im = blockIdx.x, m = im - a.M;
  const int lo = mf_window_lo(a.r, m, a.Nq), len = mf_window_len(m, a.Nq);
  auto pi = [&](int k) {
    const int nq = lo + k;
    const int k1 = a.r == 1 ? nq : nq + m, k2 = a.r == 1 ? m - nq - 1 : nq;
    return cscale(a.T, cmul(mf_G(a, k1), mf_G(a, k2)));
  };
  double2 acc[2] = {czero(), czero()};
  const int pairs = len * len;
  for (int t = threadIdx.x; t < pairs; t += blockDim.x) {
    const int k = t / len, l = t - k * len;
    double2 XY[2] = {make_double2(-a.U, 0.0), make_double2(a.U, 0.0)};
    mf_chan(a.ch[a.r], a.M, a.N, m, lo + k, lo + l, 15, XY);
    mf_others(a, m, lo + k, lo + l, XY);
    const double2 pp = cmul(pi(k), pi(l));
#pragma unroll
    for (int c = 0; c < 2; ++c)
      acc[c] = cadd(acc[c], cmul(pp, cadd(cscale(a.mix[2 * c], XY[0]), cscale(a.mix[2 * c + 1], XY[1]))));
  }
  for (int t = threadIdx.x; t < len; t += blockDim.x) {  // the bare term T sum_k Pi
    const double2 p = pi(t);
    acc[0] = cadd(acc[0], p);
    acc[1] = cadd(acc[1], p);
  }
  __shared__ double2 red[2][256];
  red[0][threadIdx.x] = acc[0];
  red[1][threadIdx.x] = acc[1];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] = cadd(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = cadd(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[im] = red[0][0];
    out[(2 * a.M + 1) + im] = red[1][0];
  }
}

void launch_mf_chi(const MGatherArgs& v, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(mf_chi_kernel, dim3((unsigned)(2 * v.M + 1)), dim3(256), 0, s, v, out);
}

void launch_mf_tail(const MTailArgs& a, hipStream_t s) {
  const long total = (long)(2 * a.N + 1) * (2 * a.N + 1) * (2L * a.M + 1);
  hipLaunchKernelGGL(mf_tail_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
}

void launch_mf_left(const MGatherArgs& a, hipStream_t s) {
  const long total = (long)(2 * a.N + 1) * (2 * a.Nq) * a.nb;
  hipLaunchKernelGGL(mf_left_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
}
void launch_mf_right(const MGatherArgs& a, hipStream_t s) {
  const long total = (long)(2 * a.N + 1) * (2 * a.Nq) * a.nb;
  hipLaunchKernelGGL(mf_right_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
}
void launch_mf_epilogue(const MEpiArgs& a, hipStream_t s) {
  const long total = (long)(2 * a.N + 1) * (2 * a.N + 1) * a.nb;
  hipLaunchKernelGGL(mf_epilogue_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
}

}  // namespace kqft
