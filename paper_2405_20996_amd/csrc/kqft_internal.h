// kqft_internal.h -- device-side data model and helpers of the MI355X Keldysh
// bubble library (gfx950).  Conventions are those documented in include/kqft.h.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace kqft {

// ------------------------------------------------------------------ complex
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cfma(double s, double2 a, double2 acc) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}
__host__ __device__ inline double2 czero() { return make_double2(0.0, 0.0); }

// ------------------------------------------------------------------ grids
// Grids v_i = a f(x_i theta), x_i = -1 + 2i/(n-1), f(theta) = L/a.  map 0: f = tan;
// map 1: f(W) = W|W|/sqrt(1 - W^2), the algebraic grid of Sec. "Frequency grids".
// aux_of inverts f: W^2 = u solves u^2 + y^2 u - y^2 = 0, taken as 2|y|/(|y| + sqrt(y^2 + 4))
// (no cancellation at large |y|).
__host__ __device__ inline double aux_of(int map, double y) {
  if (map == 0) return atan(y);
  const double ay = fabs(y);
  return copysign(sqrt(2.0 * ay / (ay + sqrt(ay * ay + 4.0))), y);
}
__host__ __device__ inline double freq_of(int map, double w) {
  if (map == 0) return tan(w);
  return w * fabs(w) / sqrt((1.0 - w) * (1.0 + w));
}
struct DGrid {
  int n, map;
  double a, inv_a, inv_theta, half_nm1;
};
inline DGrid make_dgrid(int n, double L, double a, int map) {
  DGrid g;
  g.n = n;
  g.map = map;
  g.a = a;
  g.inv_a = 1.0 / a;
  g.inv_theta = 1.0 / aux_of(map, L / a);
  g.half_nm1 = 0.5 * (n - 1);
  return g;
}
// Cell of v on the auxiliary variable x = aux_of(v/a)/theta: returns false outside
// [-1, 1] (relative slack 1e-10 keeps the end nodes inside), else i0 in [0, n-2] and
// the linear weight t of node i0+1.
__device__ inline bool dgrid_locate(const DGrid& g, double v, int& i0, double& t) {
  double x = aux_of(g.map, v * g.inv_a) * g.inv_theta;
  if (fabs(x) > 1.0 + 1e-10) return false;
  x = fmin(fmax(x, -1.0), 1.0);
  double s = (x + 1.0) * g.half_nm1;
  int i = (int)floor(s);
  i = min(max(i, 0), g.n - 2);
  i0 = i;
  t = s - (double)i;
  return true;
}

// ------------------------------------------------------------------ vertex
struct DChan {
  double coef;
  const double2* K[4];  // K1, K2, K2p, K3
};
struct DVert {
  double r0;
  DGrid g;
  DChan ch[3];
};

// ------------------------------------------------------------------ propagator
struct DProp {
  double Delta, T, eps;
  DGrid sg;
  const double2* SigR;
  const double2* SigK;
  int reg;     // regulator: 0 Delta, 1 interaction (lam), 2 temperature, 3 frequency (lam)
  double lam;
  const double2* dSigR;  // Sigma_dot on sg (Katanin, G Sigma_dot G), or null
  const double2* dSigK;
  double deps;  // real constant added to Sigma_dot^R (the flow of the level), 0 if none
};

__device__ inline double2 sigma_at(const DGrid& g, const double2* arr, double v) {
  if (arr == nullptr) return czero();
  int i0;
  double t;
  if (!dgrid_locate(g, v, i0, t)) return czero();
  double2 a = arr[i0], b = arr[i0 + 1];
  return make_double2((1.0 - t) * a.x + t * b.x, (1.0 - t) * a.y + t * b.y);
}

__device__ inline double2 cinv(double2 a) {
  const double d = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * d, -a.y * d);
}

// Keldysh matrix m[2*a + a'] = X^{a|a'} of
//   kind 0: G;  kind 1: S = dG/dLambda at fixed Sigma (+ G Sigma_dot G with Sigma_dot);
//   kind 2: G Sigma_dot G.
// With D = v - eps + i Delta and br = Sigma^K - G_0^{-1,K} (G^K = G^R br G^A), per regulator
//   Delta:       G^R = 1/(D - Sigma),         S^R = -i (G^R)^2,             dbr = -2i tanh
//   interaction: G^R = lam/(D - lam Sigma),   S^R = D/(D - lam Sigma)^2,    br, dbr with Delta/lam
//   temperature: G^R = 1/(D - Sigma),         S^R = 0,                      dbr = -2i Delta dtanh/dT
//   frequency:   G^R = Th/(D - Th Sigma),     S^R = -i D (Th^2/v)/(D - Th Sigma)^2,
//                Th = v/(v + i lam), Im G_0^{-1,R} = Delta + lam (v - eps)/v
// and S^K = S^R br G^A + G^R dbr G^A + G^R br S^A.
__device__ inline void propagator(const DProp& P, int kind, double v, double2 m[4]) {
  const double th = tanh(v / (2.0 * P.T));
  const double2 sR = sigma_at(P.sg, P.SigR, v);
  const double2 sK = P.SigK ? sigma_at(P.sg, P.SigK, v) : make_double2(0.0, 2.0 * th * sR.y);
  const double2 D = make_double2(v - P.eps, P.Delta);
  double2 GR, SR, br, dbr;
  if (P.reg == 1) {
    const double2 d = cinv(csub(D, cscale(P.lam, sR)));
    GR = cscale(P.lam, d);
    SR = cmul(D, cmul(d, d));
    br = make_double2(sK.x, sK.y - 2.0 * th * P.Delta / P.lam);
    dbr = make_double2(0.0, 2.0 * th * P.Delta / (P.lam * P.lam));
  } else if (P.reg == 2) {
    GR = cinv(csub(D, sR));
    SR = czero();
    const double dth = -(v / (2.0 * P.T * P.T)) * (1.0 - th * th);
    br = make_double2(sK.x, sK.y - 2.0 * th * P.Delta);
    dbr = make_double2(0.0, -2.0 * dth * P.Delta);
  } else if (P.reg == 3) {
    const double L = P.lam, dd = v * v + L * L, idd = 1.0 / dd;
    const double2 theta = make_double2(v * v * idd, -v * L * idd);
    const double2 t2v = make_double2(v * (v * v - L * L) * idd * idd, -2.0 * v * v * L * idd * idd);
    const double th_v = v == 0.0 ? 0.5 / P.T : th / v;
    const double2 d = cinv(csub(D, cmul(theta, sR)));
    GR = cmul(theta, d);
    const double2 q = cmul(cmul(D, t2v), cmul(d, d));
    SR = make_double2(q.y, -q.x);  // -i q
    br = make_double2(sK.x, sK.y - 2.0 * th * P.Delta - 2.0 * L * (v - P.eps) * th_v);
    dbr = make_double2(0.0, -2.0 * (v - P.eps) * th_v);
  } else {
    GR = cinv(csub(D, sR));
    const double2 g2 = cmul(GR, GR);
    SR = make_double2(g2.y, -g2.x);  // -i (G^R)^2
    br = make_double2(sK.x, sK.y - 2.0 * th * P.Delta);
    dbr = make_double2(0.0, -2.0 * th);
  }
  const double2 GA = cconj(GR);
  const double2 GK = cmul(cmul(GR, br), GA);
  double2 R = czero(), K = czero();
  if (kind == 0) {
    R = GR;
    K = GK;
  } else if (kind == 1) {
    R = SR;
    K = cadd(cadd(cmul(cmul(SR, br), GA), cmul(cmul(GR, dbr), GA)), cmul(cmul(GR, br), cconj(SR)));
  }
  if (kind != 0 && (P.dSigR || P.deps != 0.0)) {
    const double2 dR = cadd(sigma_at(P.sg, P.dSigR, v), make_double2(P.deps, 0.0));
    const double2 dK = sigma_at(P.sg, P.dSigK, v);
    R = cadd(R, cmul(cmul(GR, dR), GR));
    K = cadd(K, cadd(cadd(cmul(cmul(GR, dR), GK), cmul(cmul(GR, dK), GA)), cmul(cmul(GK, cconj(dR)), GA)));
  }
  m[0] = czero();
  m[1] = cconj(R);
  m[2] = R;
  m[3] = K;
}

// (Adjoint paths: the Delta regulator without Sigma_dot only.)
// Value m and Delta-derivative dm (at fixed Sigma) of G (kind 0: dm = S) or of the
// single-scale propagator S (kind 1: dm = dS/dDelta).  With br = Sigma^K - 2 i Delta tanh:
//   dS^R = -2 (G^R)^3,  dS^K = dS^R br G^A + 2 S^R br S^A + G^R br dS^A
//                               + 2 (-2 i tanh)(S^R G^A + G^R S^A).
__device__ inline void propagator_dDelta(const DProp& P, int kind, double v, double2 m[4], double2 dm[4]) {
  double th = tanh(v / (2.0 * P.T));
  double2 sR = sigma_at(P.sg, P.SigR, v);
  double2 sK = P.SigK ? sigma_at(P.sg, P.SigK, v) : make_double2(0.0, 2.0 * th * sR.y);
  double dr = v - P.eps - sR.x, di = P.Delta - sR.y;
  double inv = 1.0 / (dr * dr + di * di);
  double2 GR = make_double2(dr * inv, -di * inv);
  double2 GA = cconj(GR);
  double2 br = make_double2(sK.x, sK.y - 2.0 * th * P.Delta);
  double2 dbr = make_double2(0.0, -2.0 * th);
  double2 SR = cmul(make_double2(0.0, -1.0), cmul(GR, GR));
  double2 SA = cconj(SR);
  double2 SK = cadd(cadd(cmul(cmul(SR, br), GA), cmul(cmul(GR, dbr), GA)), cmul(cmul(GR, br), SA));
  m[0] = czero();
  dm[0] = czero();
  if (kind == 0) {
    m[1] = GA;
    m[2] = GR;
    m[3] = cmul(cmul(GR, br), GA);
    dm[1] = SA;
    dm[2] = SR;
    dm[3] = SK;
    return;
  }
  double2 dSR = cscale(-2.0, cmul(GR, cmul(GR, GR)));
  double2 dSA = cconj(dSR);
  double2 dSK = cadd(cadd(cmul(cmul(dSR, br), GA), cscale(2.0, cmul(cmul(SR, br), SA))),
                     cadd(cmul(cmul(GR, br), dSA), cscale(2.0, cmul(dbr, cadd(cmul(SR, GA), cmul(GR, SA))))));
  m[1] = SA;
  m[2] = SR;
  m[3] = SK;
  dm[1] = dSA;
  dm[2] = dSR;
  dm[3] = dSK;
}

// ------------------------------------------------------------------ channels
// Leg frequencies (n1', n2', n1, n2) of channel r at (w, v, v') and back.
__device__ inline void legs_of(int r, double w, double v, double vp, double L[4]) {
  double h = 0.5 * w;
  if (r == 0) {
    L[0] = v + h; L[3] = v - h; L[2] = vp + h; L[1] = vp - h;
  } else if (r == 1) {
    L[0] = h + v; L[1] = h - v; L[2] = h + vp; L[3] = h - vp;
  } else {
    L[1] = v + h; L[3] = v - h; L[2] = vp + h; L[0] = vp - h;
  }
}
__device__ inline void params_of(int r, const double L[4], double& w, double& v, double& vp) {
  if (r == 0) {
    w = L[0] - L[3]; v = 0.5 * (L[0] + L[3]); vp = 0.5 * (L[2] + L[1]);
  } else if (r == 1) {
    w = L[0] + L[1]; v = 0.5 * (L[0] - L[1]); vp = 0.5 * (L[2] - L[3]);
  } else {
    w = L[1] - L[3]; v = 0.5 * (L[1] + L[3]); vp = 0.5 * (L[0] + L[2]);
  }
}

// Bare-vertex Keldysh table entry: nonzero iff the four leg indices have an odd sum,
// which is the parity of popcount(row pair) + popcount(column pair) in any channel.
__host__ __device__ inline bool bare_odd(int f) {
  int row = f >> 2, col = f & 3;
  return (((row >> 1) + (row & 1) + (col >> 1) + (col & 1)) & 1) != 0;
}

// flat-index permutation from channel r's pair order to channel r2's, filled on the host
extern __constant__ int c_perm[3][3][16];

struct Workspace;  // host side

}  // namespace kqft
