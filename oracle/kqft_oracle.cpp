// kqft_oracle.cpp -- plain, slow, FP64 CPU oracle of the real-frequency Keldysh
// bubble / Schwinger-Dyson / susceptibility hot path of the KeldyshQFT method
// (Ritz, Ge, Walter, Aguirre, von Delft, Kugler, arXiv:2405.20996).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no code,
// header or table with the HIP path; it is written from the paper's equations
// and the conventions listed below, with plain nested loops in the order the
// definitions are stated (no blocking, no spin diagonalisation, no GEMM).
//
// Conventions (the paper defers the parametrised formulas to its companion
// paper; these are the readings adopted here):
//  * Keldysh indices alpha in {0,1} (paper: 1,2).  Propagator matrix
//    G^{a|a'}: G^{0|0}=0, G^{0|1}=G^A, G^{1|0}=G^R, G^{1|1}=G^K.
//  * Bare vertex (parquet approximation R = Gamma_0, Sec. "Diagrammatic
//    many-body theory"): Gamma_0^{a1'a2'|a1a2} = -r0/2 when a1'+a2'+a1+a2 is
//    odd, else 0; spin components X0 = that table, Y0 = -X0.
//  * Spin (SU(2), Sec. "Symmetries"): Gamma_{s1's2'|s1s2} =
//    X d(s1',s1) d(s2',s2) + Y d(s1',s2) d(s2',s1); X = Gamma_{up dn|up dn},
//    Y = Gamma_{up dn|dn up}.  Both are stored, in every channel, defined on
//    the legs, so no spin permutation is needed between channels.
//  * Channel parametrisations (legs 1',2' outgoing, 1,2 incoming):
//      a: w = n1'-n2,  v = (n1'+n2)/2,  v' = (n1+n2')/2
//      p: w = n1'+n2', v = (n1'-n2')/2, v' = (n1-n2)/2
//      t: w = n2'-n2,  v = (n2'+n2)/2,  v' = (n1'+n1)/2
//    Keldysh 4x4 pair order (row pair | column pair), pair = 2*first+second:
//      a: (a1',a2 | a1,a2'),  p: (a1',a2' | a1,a2),  t: (a2',a2 | a1',a1)
//  * Bubbles in compound-index form (Eq. B_a and the BSEs, with channel
//    prefactors a: +1, p: +1/2, t: -1) and integration measure dv''/(2 pi i)
//    (the measure of the Hartree formula):
//      g_a(1'2'|12) =  +  G_L(1',4'|3,2) G(3|3') G(4|4') G_R(3',2'|1,4)
//      g_p(1'2'|12) = 1/2 G_L(1',2'|3,4) G(3|3') G(4|4') G_R(3',4'|1,2)
//      g_t(1'2'|12) =  -  G_L(4',2'|3,2) G(3|3') G(4|4') G_R(1',3'|1,4)
//  * Frequency grids: v_i = a tan(x_i atan(L/a)), x_i = -1 + 2i/(n-1)
//    (a tangent map of an equidistant auxiliary grid, in the spirit of the
//    paper's non-linear grid, Sec. "Frequency grids").  Linear interpolation
//    on the auxiliary variable x (the paper's preferred "linear_on_aux"),
//    value 0 outside the grid (the paper ignores tails beyond the largest grid
//    point, Sec. "Asymptotic corrections to frequency integrals").
//  * Quadrature: Gauss-Legendre nodes on [-1,1], mapped by the same tangent
//    map to [-L,L] (map 0) or by v = b tan(pi y/2) to the real line (map 1).
//
// Every floating value is FP64; the value type S is either double or a
// forward-mode dual number (value, derivative) used for exact derivatives of
// the discrete forward map with respect to U and Delta.

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

// ---------------------------------------------------------------- scalars
struct Dual {
  double v, d;
};
static inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
static inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
static inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
static inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
static inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
static inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
static inline Dual mk(double x, Dual*) { return {x, 0.0}; }
static inline double mk(double x, double*) { return x; }

template <class S> struct Cx {
  S re, im;
};
template <class S> static inline Cx<S> operator+(Cx<S> a, Cx<S> b) { return {a.re + b.re, a.im + b.im}; }
template <class S> static inline Cx<S> operator-(Cx<S> a, Cx<S> b) { return {a.re - b.re, a.im - b.im}; }
template <class S> static inline Cx<S> operator*(Cx<S> a, Cx<S> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class S> static inline Cx<S> operator*(double s, Cx<S> a) { return {s * a.re, s * a.im}; }
template <class S> static inline Cx<S> conj(Cx<S> a) { return {a.re, S(-a.im)}; }
template <class S> static inline Cx<S> inv(Cx<S> a) {
  S den = a.re * a.re + a.im * a.im;
  return {a.re / den, S(-a.im) / den};
}
template <class S> static inline Cx<S> czero() {
  S z = mk(0.0, (S*)nullptr);
  return {z, z};
}
// multiply by a plain complex number (c_re + i c_im)
template <class S> static inline Cx<S> cmul(double c_re, double c_im, Cx<S> a) {
  return {c_re * a.re - c_im * a.im, c_re * a.im + c_im * a.re};
}

// ---------------------------------------------------------------- ABI structs
extern "C" {
// one channel's reducible vertex gamma_r, asymptotic classes on the vertex grid;
// arrays are complex (2 doubles; 4 doubles for the dual variant), layouts
// K1[s][w][16], K2[s][w][v][16], K2p[s][w][v'][16], K3[s][w][v][v'][16], s in {X,Y};
// Keldysh flat index 4*row_pair+col_pair in the channel's own pair order.
typedef struct {
  double coef;
  const double* K1;
  const double* K2;
  const double* K2p;
  const double* K3;
} OCh;
// vertex = Gamma_0(r0) + sum_r coef_r gamma_r, all classes on one grid (n, L, a, map)
typedef struct {
  double r0, dr0;
  int n;
  double L, a;
  OCh ch[3];
  int map;
} OVert;
// propagator: G^R = 1/(v - eps + i Delta - Sigma^R(v)),
// G^K = G^R [Sigma^K - 2 i Delta tanh(v/2T)] G^A; Sigma optional on its own grid.
// reg selects the flow parameter Lambda of S = dG/dLambda at fixed Sigma (Sec. "Flow
// schemes"): 0 Delta (Lambda = Delta), 1 interaction flow (G_0 -> Lambda G_0, Lambda = lam),
// 2 temperature (Lambda = T), 3 frequency regulator Theta = v/(v + i lam) (Lambda = lam).
// dSigR/dSigK: optional Sigma_dot on the Sigma grid (Katanin: S -> S + G Sigma_dot G);
// deps: a frequency-independent real part of Sigma_dot^R (the flow of the level eps), added to
// dSigR in the G Sigma_dot G line.
typedef struct {
  double Delta, dDelta, T, eps;
  int sn;
  double sL, sa;
  const double* SigR;
  const double* SigK;
  int reg;
  double lam;
  const double* dSigR;
  const double* dSigK;
  double deps;
  int smap;  // map of the Sigma grid
} OProp;
// quadrature: n Gauss-Legendre nodes, map 0 = tangent onto [-L, L] with scale a,
// map 1 = v = a tan(pi y / 2) onto the real line; map 2 = the n nodes of the tangent grid
// (n, L, a) themselves with trapezoid weights on its auxiliary variable (a rule whose nodes
// are grid points, so that a vertex stored on that grid is read back without interpolation).
typedef struct {
  int n, map;
  double L, a;
} OQuad;
}

// ---------------------------------------------------------------- grids
// Sec. "Frequency grids": an equidistant auxiliary variable mapped to frequencies.
// map 0 (tangent): v = a tan(W); map 1 (the paper's non-linear map): v = a W |W| / sqrt(1 - W^2),
// W in (-1, 1).  Both are odd and increasing; the grid takes W_i = x_i theta with x_i
// equidistant in [-1, 1] and theta the W of v = L.
static double map_forward(int map, double W) {
  if (map == 0) return std::tan(W);
  return W * std::fabs(W) / std::sqrt(1.0 - W * W);
}
// inverse of map_forward for y = v/a: map 1 solves y^2 (1 - W^2) = W^4 for W^2 (the positive
// root of the quadratic u^2 + y^2 u - y^2, written as 2|y| / (|y| + sqrt(y^2 + 4)))
static double map_inverse(int map, double y) {
  if (map == 0) return std::atan(y);
  const double ay = std::fabs(y);
  const double u = 2.0 * ay / (ay + std::sqrt(ay * ay + 4.0));
  return y < 0 ? -std::sqrt(u) : std::sqrt(u);
}
struct Grid {
  int n;
  double L, a, theta;
  int map;
};
static Grid make_grid(int n, double L, double a, int map = 0) {
  return Grid{n, L, a, map_inverse(map, L / a), map};
}
// The algebraic grid is taken exactly odd (v_{n-1-i} = -v_i): its auxiliary variable grows as
// sqrt(|v|) at zero, so sums of nodes that vanish must vanish exactly (the W of a rounding
// residue of 1e-17 would be 3e-9).
static double grid_node(const Grid& g, int i) {
  if (g.map == 1 && 2 * i > g.n - 1) return -grid_node(g, g.n - 1 - i);
  double x = -1.0 + 2.0 * i / (g.n - 1);
  return g.a * map_forward(g.map, x * g.theta);
}
// Locate v on the auxiliary variable x = W(v/a)/theta; false if outside [-L, L]
// (with a relative tolerance of 1e-10 on x so that grid end points count as inside).
static bool grid_locate(const Grid& g, double v, int& i0, double& t) {
  double x = map_inverse(g.map, v / g.a) / g.theta;
  if (x > 1.0 + 1e-10 || x < -1.0 - 1e-10) return false;
  if (x > 1.0) x = 1.0;
  if (x < -1.0) x = -1.0;
  double s = (x + 1.0) * 0.5 * (g.n - 1);
  int i = (int)std::floor(s);
  if (i < 0) i = 0;
  if (i > g.n - 2) i = g.n - 2;
  i0 = i;
  t = s - i;
  return true;
}

// Gauss-Legendre nodes and weights on [-1,1] by Newton iteration on P_n.
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static void make_quad(const OQuad& q, std::vector<double>& nu, std::vector<double>& wt) {
  nu.resize(q.n);
  wt.resize(q.n);
  if (q.map == 2) {
    // trapezoid rule in x on the grid's own nodes: v = a tan(x theta), dv = a theta sec^2 dx
    Grid g = make_grid(q.n, q.L, q.a, 0);
    const double h = 2.0 / (q.n - 1);
    for (int k = 0; k < q.n; ++k) {
      double x = -1.0 + 2.0 * k / (q.n - 1);
      double c = std::cos(x * g.theta);
      nu[k] = grid_node(g, k);
      wt[k] = ((k == 0 || k == q.n - 1) ? 0.5 : 1.0) * h * q.a * g.theta / (c * c);
    }
    return;
  }
  std::vector<double> y(q.n), gw(q.n);
  gauss_legendre(q.n, y.data(), gw.data());
  for (int k = 0; k < q.n; ++k) {
    if (q.map == 0) {
      double th = std::atan(q.L / q.a);
      double c = std::cos(y[k] * th);
      nu[k] = q.a * std::tan(y[k] * th);
      wt[k] = gw[k] * q.a * th / (c * c);
    } else {
      double h = 0.5 * M_PI;
      double c = std::cos(y[k] * h);
      nu[k] = q.a * std::tan(y[k] * h);
      wt[k] = gw[k] * q.a * h / (c * c);
    }
  }
}

// ---------------------------------------------------------------- propagator
// Sigma on its grid, linear interpolation on the auxiliary variable; zero outside.
template <class S>
static Cx<S> sigma_interp(const OProp& P, const double* arr, double v) {
  Cx<S> z = czero<S>();
  if (!arr) return z;
  Grid g = make_grid(P.sn, P.sL, P.sa, P.smap);
  int i0;
  double t;
  if (!grid_locate(g, v, i0, t)) return z;
  const Cx<S>* a = (const Cx<S>*)arr;
  return (1.0 - t) * a[i0] + t * a[i0 + 1];
}

template <class S> static S param_delta(const OProp& P);
template <> double param_delta<double>(const OProp& P) { return P.Delta; }
template <> Dual param_delta<Dual>(const OProp& P) { return Dual{P.Delta, P.dDelta}; }

template <class S> static Cx<S> lift(double re, double im) {
  return Cx<S>{mk(re, (S*)nullptr), mk(im, (S*)nullptr)};
}

// Keldysh matrix g[a][a'] of
//   kind 0: G, with G^R = 1/(G_0^{-1,R} - Sigma^R), G^K = G^R [Sigma^K - G_0^{-1,K}] G^A and
//           G_0^{-1,K} = 2 i tanh(v/2T) Im G_0^{-1,R} (the bath in equilibrium);
//   kind 1: the single-scale propagator S = dG/dLambda at fixed Sigma of the regulator reg,
//           plus G Sigma_dot G when Sigma_dot is given (Katanin substitution);
//   kind 2: G Sigma_dot G alone.
// G_0^{-1,R} per regulator, with D = v - eps + i Delta:  Delta: D;  interaction: D / lam;
// temperature: D (the flow enters through tanh);  frequency: D (v + i lam) / v.
template <class S> static void propagator(const OProp& P, int kind, double v, Cx<S> g[2][2]) {
  S Dl = param_delta<S>(P);
  S zero = mk(0.0, (S*)nullptr);
  double th = std::tanh(v / (2.0 * P.T));
  Cx<S> sR = sigma_interp<S>(P, P.SigR, v);
  Cx<S> sK;
  if (P.SigK) {
    sK = sigma_interp<S>(P, P.SigK, v);
  } else {  // equilibrium FDR for the self-energy: Sigma^K = 2 i tanh Im Sigma^R
    sK = Cx<S>{zero, 2.0 * th * sR.im};
  }
  const Cx<S> Dc = Cx<S>{mk(v - P.eps, (S*)nullptr), Dl};
  Cx<S> GR, SR, br, dbr;  // br = Sigma^K - G_0^{-1,K}, dbr = -dG_0^{-1,K}/dLambda
  if (P.reg == 1) {
    const double L = P.lam;
    const Cx<S> d = inv(Dc - L * sR);
    GR = L * d;
    SR = Dc * d * d;  // d/dL [L / (D - L Sigma)] = D / (D - L Sigma)^2
    br = Cx<S>{sK.re, sK.im - (2.0 * th / L) * Dl};
    dbr = Cx<S>{zero, (2.0 * th / (L * L)) * Dl};
  } else if (P.reg == 2) {
    GR = inv(Dc - sR);
    SR = czero<S>();
    const double dth = -(v / (2.0 * P.T * P.T)) * (1.0 - th * th);  // d tanh(v/2T) / dT
    br = Cx<S>{sK.re, sK.im - 2.0 * th * Dl};
    dbr = Cx<S>{zero, (-2.0 * dth) * Dl};
  } else if (P.reg == 3) {
    const double L = P.lam;
    // Theta = v / (v + i L) and Theta^2 / v = v / (v + i L)^2, finite at v = 0
    const double dd = v * v + L * L;
    const Cx<S> theta = lift<S>(v * v / dd, -v * L / dd);
    const Cx<S> t2v = lift<S>(v * (v * v - L * L) / (dd * dd), -2.0 * v * v * L / (dd * dd));
    const double th_v = v == 0.0 ? 1.0 / (2.0 * P.T) : th / v;  // tanh(v/2T) / v
    const Cx<S> d = inv(Dc - theta * sR);
    GR = theta * d;
    SR = cmul(0.0, -1.0, Dc * t2v * d * d);
    // Im G_0^{-1,R} = Delta + lam (v - eps) / v, its lam-derivative (v - eps) / v
    br = Cx<S>{sK.re, sK.im - 2.0 * th * Dl - mk(2.0 * L * (v - P.eps) * th_v, (S*)nullptr)};
    dbr = lift<S>(0.0, -2.0 * (v - P.eps) * th_v);
  } else {
    GR = inv(Dc - sR);
    SR = cmul(0.0, -1.0, GR * GR);  // d/dDelta 1/(D - Sigma) = -i G^2
    br = Cx<S>{sK.re, sK.im - 2.0 * th * Dl};
    dbr = lift<S>(0.0, -2.0 * th);
  }
  const Cx<S> GA = conj(GR);
  const Cx<S> GK = GR * br * GA;
  Cx<S> R = czero<S>(), K = czero<S>();
  if (kind == 0) {
    R = GR;
    K = GK;
  }
  if (kind == 1) {  // product rule on G^K = G^R br G^A
    R = SR;
    K = SR * br * GA + GR * dbr * GA + GR * br * conj(SR);
  }
  if ((kind == 1 || kind == 2) && (P.dSigR || P.deps != 0.0)) {
    // G Sigma_dot G: R = G^R s^R G^R, K = G^R s^R G^K + G^R s^K G^A + G^K s^A G^A
    const Cx<S> dR = sigma_interp<S>(P, P.dSigR, v) + lift<S>(P.deps, 0.0);
    const Cx<S> dK = sigma_interp<S>(P, P.dSigK, v);
    R = R + GR * dR * GR;
    K = K + GR * dR * GK + GR * dK * GA + GK * conj(dR) * GA;
  }
  g[0][0] = czero<S>();
  g[0][1] = conj(R);
  g[1][0] = R;
  g[1][1] = K;
}

// ---------------------------------------------------------------- channels
// Leg frequencies (n1', n2', n1, n2) from channel parameters and back.
static void legs_from(int r, double w, double v, double vp, double L[4]) {
  // L[0]=n1', L[1]=n2', L[2]=n1, L[3]=n2
  if (r == 0) {  // a
    L[0] = v + w / 2;
    L[3] = v - w / 2;
    L[2] = vp + w / 2;
    L[1] = vp - w / 2;
  } else if (r == 1) {  // p
    L[0] = w / 2 + v;
    L[1] = w / 2 - v;
    L[2] = w / 2 + vp;
    L[3] = w / 2 - vp;
  } else {  // t
    L[1] = v + w / 2;
    L[3] = v - w / 2;
    L[2] = vp + w / 2;
    L[0] = vp - w / 2;
  }
}
static void params_from(int r, const double L[4], double& w, double& v, double& vp) {
  if (r == 0) {
    w = L[0] - L[3];
    v = 0.5 * (L[0] + L[3]);
    vp = 0.5 * (L[2] + L[1]);
  } else if (r == 1) {
    w = L[0] + L[1];
    v = 0.5 * (L[0] - L[1]);
    vp = 0.5 * (L[2] - L[3]);
  } else {
    w = L[1] - L[3];
    v = 0.5 * (L[1] + L[3]);
    vp = 0.5 * (L[0] + L[2]);
  }
}
// Keldysh leg indices (a1', a2', a1, a2) of a flat index f in channel r's pair order.
static void legs_of_flat(int r, int f, int al[4]) {
  int row = f / 4, col = f % 4;
  int x = row / 2, y = row % 2, z = col / 2, u = col % 2;
  if (r == 0) {  // rows (a1',a2), cols (a1,a2')
    al[0] = x; al[3] = y; al[2] = z; al[1] = u;
  } else if (r == 1) {  // rows (a1',a2'), cols (a1,a2)
    al[0] = x; al[1] = y; al[2] = z; al[3] = u;
  } else {  // rows (a2',a2), cols (a1',a1)
    al[1] = x; al[3] = y; al[0] = z; al[2] = u;
  }
}
static int flat_of_legs(int r, const int al[4]) {
  int row, col;
  if (r == 0) {
    row = 2 * al[0] + al[3];
    col = 2 * al[2] + al[1];
  } else if (r == 1) {
    row = 2 * al[0] + al[1];
    col = 2 * al[2] + al[3];
  } else {
    row = 2 * al[1] + al[3];
    col = 2 * al[0] + al[2];
  }
  return 4 * row + col;
}

// ---------------------------------------------------------------- vertex
template <class S> struct Vtx {
  S r0;
  Grid g;
  double coef[3];
  const Cx<S>* K[3][4];  // [channel][class]
};
template <class S> static S param_r0(const OVert& V);
template <> double param_r0<double>(const OVert& V) { return V.r0; }
template <> Dual param_r0<Dual>(const OVert& V) { return Dual{V.r0, V.dr0}; }

template <class S> static Vtx<S> make_vtx(const OVert& V) {
  Vtx<S> o;
  o.r0 = param_r0<S>(V);
  o.g = make_grid(V.n, V.L, V.a, V.map);
  for (int r = 0; r < 3; ++r) {
    o.coef[r] = V.ch[r].coef;
    o.K[r][0] = (const Cx<S>*)V.ch[r].K1;
    o.K[r][1] = (const Cx<S>*)V.ch[r].K2;
    o.K[r][2] = (const Cx<S>*)V.ch[r].K2p;
    o.K[r][3] = (const Cx<S>*)V.ch[r].K3;
  }
  return o;
}

enum { P_R = 1, P_K1 = 2, P_K2 = 4, P_K2P = 8, P_K3 = 16, P_OTHER = 32, P_ALL = 63 };

// Evaluate the classes of channel rr at its own parameters (w, v, vp) by
// multilinear interpolation on the auxiliary grid; out[s][16] accumulates.
template <class S>
static void add_channel_classes(const Vtx<S>& V, int rr, double w, double v, double vp, unsigned cls,
                                double c, Cx<S> out[2][16]) {
  const Grid& g = V.g;
  int n = g.n;
  int iw, iv, ivp;
  double tw, tv, tvp;
  if (!grid_locate(g, w, iw, tw)) return;  // every class vanishes outside the bosonic grid
  bool inv_ = grid_locate(g, v, iv, tv);
  bool invp = grid_locate(g, vp, ivp, tvp);
  for (int s = 0; s < 2; ++s) {
    for (int cw = 0; cw < 2; ++cw) {
      double ww = cw ? tw : 1.0 - tw;
      int jw = iw + cw;
      if ((cls & P_K1) && V.K[rr][0]) {
        const Cx<S>* A = V.K[rr][0] + ((size_t)s * n + jw) * 16;
        for (int f = 0; f < 16; ++f) out[s][f] = out[s][f] + (c * ww) * A[f];
      }
      for (int cv = 0; cv < 2; ++cv) {
        double wv = cv ? tv : 1.0 - tv;
        if ((cls & P_K2) && V.K[rr][1] && inv_) {
          const Cx<S>* A = V.K[rr][1] + (((size_t)s * n + jw) * n + iv + cv) * 16;
          for (int f = 0; f < 16; ++f) out[s][f] = out[s][f] + (c * ww * wv) * A[f];
        }
        double wvp = cv ? tvp : 1.0 - tvp;
        if ((cls & P_K2P) && V.K[rr][2] && invp) {
          const Cx<S>* A = V.K[rr][2] + (((size_t)s * n + jw) * n + ivp + cv) * 16;
          for (int f = 0; f < 16; ++f) out[s][f] = out[s][f] + (c * ww * wvp) * A[f];
        }
        if ((cls & P_K3) && V.K[rr][3] && inv_ && invp) {
          for (int cvp = 0; cvp < 2; ++cvp) {
            double wvp2 = cvp ? tvp : 1.0 - tvp;
            const Cx<S>* A = V.K[rr][3] + ((((size_t)s * n + jw) * n + iv + cv) * n + ivp + cvp) * 16;
            for (int f = 0; f < 16; ++f) out[s][f] = out[s][f] + (c * ww * wv * wvp2) * A[f];
          }
        }
      }
    }
  }
}

// Full (or partial) vertex in channel r's parametrisation and pair order.
// parts: P_R = bare vertex; P_K1..P_K3 = own-channel classes; P_OTHER = the two
// other channels (all their classes), reached through the leg frequencies.
template <class S>
static void eval_vertex(const Vtx<S>& V, int r, double w, double v, double vp, unsigned parts,
                        Cx<S> X[16], Cx<S> Y[16]) {
  Cx<S> out[2][16];
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 16; ++f) out[s][f] = czero<S>();
  if (parts & P_R) {
    for (int f = 0; f < 16; ++f) {
      int al[4];
      legs_of_flat(r, f, al);
      if ((al[0] + al[1] + al[2] + al[3]) % 2 == 1) {
        S val = -0.5 * V.r0;
        out[0][f] = out[0][f] + Cx<S>{val, mk(0.0, (S*)nullptr)};
        out[1][f] = out[1][f] - Cx<S>{val, mk(0.0, (S*)nullptr)};
      }
    }
  }
  unsigned own = parts & (P_K1 | P_K2 | P_K2P | P_K3);
  if (own && V.coef[r] != 0.0) add_channel_classes(V, r, w, v, vp, own, V.coef[r], out);
  if (parts & P_OTHER) {
    double L[4];
    legs_from(r, w, v, vp, L);
    for (int rr = 0; rr < 3; ++rr) {
      if (rr == r || V.coef[rr] == 0.0) continue;
      double w2, v2, vp2;
      params_from(rr, L, w2, v2, vp2);
      Cx<S> tmp[2][16];
      for (int s = 0; s < 2; ++s)
        for (int f = 0; f < 16; ++f) tmp[s][f] = czero<S>();
      add_channel_classes(V, rr, w2, v2, vp2, P_K1 | P_K2 | P_K2P | P_K3, V.coef[rr], tmp);
      for (int f = 0; f < 16; ++f) {
        int al[4];
        legs_of_flat(r, f, al);
        int f2 = flat_of_legs(rr, al);
        out[0][f] = out[0][f] + tmp[0][f2];
        out[1][f] = out[1][f] + tmp[1][f2];
      }
    }
  }
  for (int f = 0; f < 16; ++f) {
    X[f] = out[0][f];
    Y[f] = out[1][f];
  }
}

// ---------------------------------------------------------------- bubble
// Pi_r at transfer frequency w and loop frequency vq, as a 4x4 pair matrix in
// channel r's internal pair order (Eq. B_a and the BSEs written in pair form).
template <class S>
static void bubble_pi(const OProp& P, int r, int kind, double w, double vq, Cx<S> Pi[16]) {
  double f3, f4;  // frequencies of propagators G(3|3') and G(4|4')
  if (r == 1) {
    f3 = w / 2 + vq;
    f4 = w / 2 - vq;
  } else {
    f3 = vq + w / 2;
    f4 = vq - w / 2;
  }
  Cx<S> g3[2][2], g4[2][2], s3[2][2], s4[2][2];
  propagator<S>(P, 0, f3, g3);
  propagator<S>(P, 0, f4, g4);
  if (kind == 1) {
    propagator<S>(P, 1, f3, s3);
    propagator<S>(P, 1, f4, s4);
  }
  for (int a3 = 0; a3 < 2; ++a3)
    for (int a3p = 0; a3p < 2; ++a3p)
      for (int a4 = 0; a4 < 2; ++a4)
        for (int a4p = 0; a4p < 2; ++a4p) {
          int rp, cp;
          if (r == 0) {  // Pi_a[(a3,a4'),(a3',a4)]
            rp = 2 * a3 + a4p;
            cp = 2 * a3p + a4;
          } else if (r == 1) {  // Pi_p[(a3,a4),(a3',a4')]
            rp = 2 * a3 + a4;
            cp = 2 * a3p + a4p;
          } else {  // Pi_t[(a4',a3),(a3',a4)]
            rp = 2 * a4p + a3;
            cp = 2 * a3p + a4;
          }
          Cx<S> val;
          if (kind == 0)
            val = g3[a3][a3p] * g4[a4][a4p];
          else  // differentiated bubble: S G + G S
            val = s3[a3][a3p] * g4[a4][a4p] + g3[a3][a3p] * s4[a4][a4p];
          Pi[4 * rp + cp] = val;
        }
}

template <class S> static void matmul4(const Cx<S> A[16], const Cx<S> B[16], Cx<S> C[16]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      Cx<S> acc = czero<S>();
      for (int k = 0; k < 4; ++k) acc = acc + A[4 * i + k] * B[4 * k + j];
      C[4 * i + j] = acc;
    }
}

// Literal spin sums of the three bubbles (derived from the compound-index forms with
// the SU(2) spin structure), including the channel prefactor.
template <class S>
static void spin_sums(int r, const Cx<S>* LX, const Cx<S>* LY, const Cx<S>* Pi, const Cx<S>* RX,
                      const Cx<S>* RY, Cx<S> oX[16], Cx<S> oY[16]) {
  Cx<S> LXY[16], RXY[16], T1[16], T2[16], T3[16];
  for (int f = 0; f < 16; ++f) {
    LXY[f] = LX[f] + LY[f];
    RXY[f] = RX[f] + RY[f];
  }
  auto prod = [&](const Cx<S>* A, const Cx<S>* B, Cx<S>* C) {
    Cx<S> M[16];
    matmul4(A, Pi, M);
    matmul4(M, B, C);
  };
  if (r == 0) {  // a: X = X Pi X ; Y = (X+Y) Pi Y + Y Pi (X+Y)
    prod(LX, RX, T1);
    prod(LXY, RY, T2);
    prod(LY, RXY, T3);
    for (int f = 0; f < 16; ++f) {
      oX[f] = T1[f];
      oY[f] = T2[f] + T3[f];
    }
  } else if (r == 1) {  // p: X = 1/2 (X Pi X + Y Pi Y) ; Y = 1/2 (X Pi Y + Y Pi X)
    prod(LX, RX, T1);
    prod(LY, RY, T2);
    for (int f = 0; f < 16; ++f) oX[f] = 0.5 * (T1[f] + T2[f]);
    prod(LX, RY, T1);
    prod(LY, RX, T2);
    for (int f = 0; f < 16; ++f) oY[f] = 0.5 * (T1[f] + T2[f]);
  } else {  // t: X = -[X Pi (X+Y) + (X+Y) Pi X] ; Y = -Y Pi Y
    prod(LX, RXY, T1);
    prod(LXY, RX, T2);
    prod(LY, RY, T3);
    for (int f = 0; f < 16; ++f) {
      oX[f] = -1.0 * (T1[f] + T2[f]);
      oY[f] = -1.0 * T3[f];
    }
  }
}

enum { C_K1 = 1, C_K2 = 2, C_K2P = 4, C_K3 = 8 };

// Left factor of the bubble in channel r at (w, v_i, v''): the part that depends on
// v ("rem", gives K3/K2) or the v -> infinity limit ("inf", gives K2'/K1).
template <class S>
static void left_factor(const Vtx<S>& V, int r, double w, double v, double vq, bool inf, Cx<S>* X, Cx<S>* Y) {
  if (inf)
    eval_vertex(V, r, w, 0.0, vq, P_R | P_K1 | P_K2P, X, Y);
  else
    eval_vertex(V, r, w, v, vq, P_K2 | P_K3 | P_OTHER, X, Y);
}
template <class S>
static void right_factor(const Vtx<S>& V, int r, double w, double vq, double vp, bool inf, Cx<S>* X, Cx<S>* Y) {
  if (inf)
    eval_vertex(V, r, w, vq, 0.0, P_R | P_K1 | P_K2, X, Y);
  else
    eval_vertex(V, r, w, vq, vp, P_K2P | P_K3 | P_OTHER, X, Y);
}

// B_r(left, right) on the left vertex's grid; outputs overwritten for selected classes.
template <class S>
static void bubble_full(int r, const OVert& Lv, const OVert& Rv, const OProp& P, int kind, const OQuad& q,
                        int cmask, Cx<S>* K1, Cx<S>* K2, Cx<S>* K2p, Cx<S>* K3) {
  Vtx<S> VL = make_vtx<S>(Lv), VR = make_vtx<S>(Rv);
  int n = VL.g.n;
  std::vector<double> qv, qw;
  make_quad(q, qv, qw);
  int nq = q.n;
#pragma omp parallel for schedule(dynamic)
  for (int iw = 0; iw < n; ++iw) {
    double w = grid_node(VL.g, iw);
    // Pi_k * w_k/(2 pi i) for every loop node
    std::vector<Cx<S>> Pi((size_t)nq * 16);
    for (int k = 0; k < nq; ++k) {
      bubble_pi<S>(P, r, kind, w, qv[k], &Pi[(size_t)k * 16]);
      for (int f = 0; f < 16; ++f) Pi[(size_t)k * 16 + f] = cmul(0.0, -qw[k] / (2.0 * M_PI), Pi[(size_t)k * 16 + f]);
    }
    // left factors for rows i = 0..n-1 and the infinite row i = n; right factors likewise.
    // Only the rows the selected classes use are built: finite-v rows for K3/K2 (left)
    // and K3/K2' (right); row slot of i is i, or 0 when only the infinite row is kept.
    bool need_l = cmask & (C_K3 | C_K2), need_r = cmask & (C_K3 | C_K2P);
    size_t nl = need_l ? n + 1 : 1, nr = need_r ? n + 1 : 1;
    std::vector<Cx<S>> LX(nl * nq * 16), LY(LX.size()), RX(nr * nq * 16), RY(RX.size());
    auto lslot = [&](int i) { return need_l ? (size_t)i : 0; };
    auto rslot = [&](int j) { return need_r ? (size_t)j : 0; };
    for (int i = 0; i <= n; ++i) {
      double v = i < n ? grid_node(VL.g, i) : 0.0;
      for (int k = 0; k < nq; ++k) {
        if (i == n || need_l) {
          size_t o = (lslot(i) * nq + k) * 16;
          left_factor(VL, r, w, v, qv[k], i == n, &LX[o], &LY[o]);
        }
        if (i == n || need_r) {
          size_t o = (rslot(i) * nq + k) * 16;
          right_factor(VR, r, w, qv[k], v, i == n, &RX[o], &RY[o]);
        }
      }
    }
    for (int i = 0; i <= n; ++i)
      for (int j = 0; j <= n; ++j) {
        int cls = (i < n && j < n) ? C_K3 : (i < n) ? C_K2 : (j < n) ? C_K2P : C_K1;
        if (!(cmask & cls)) continue;
        Cx<S> aX[16], aY[16];
        for (int f = 0; f < 16; ++f) aX[f] = aY[f] = czero<S>();
        for (int k = 0; k < nq; ++k) {
          Cx<S> tX[16], tY[16];
          size_t ol = (lslot(i) * nq + k) * 16, orr = (rslot(j) * nq + k) * 16;
          spin_sums<S>(r, &LX[ol], &LY[ol], &Pi[(size_t)k * 16], &RX[orr], &RY[orr], tX, tY);
          for (int f = 0; f < 16; ++f) {
            aX[f] = aX[f] + tX[f];
            aY[f] = aY[f] + tY[f];
          }
        }
        for (int s = 0; s < 2; ++s) {
          Cx<S>* dst;
          if (cls == C_K3)
            dst = K3 + ((((size_t)s * n + iw) * n + i) * n + j) * 16;
          else if (cls == C_K2)
            dst = K2 + (((size_t)s * n + iw) * n + i) * 16;
          else if (cls == C_K2P)
            dst = K2p + (((size_t)s * n + iw) * n + j) * 16;
          else
            dst = K1 + ((size_t)s * n + iw) * 16;
          for (int f = 0; f < 16; ++f) dst[f] = s ? aY[f] : aX[f];
        }
      }
  }
}

// Selected output entries: pts[p] = (class in {1,2,4,8}, iw, i, j); out[p][2][16].
template <class S>
static void bubble_points(int r, const OVert& Lv, const OVert& Rv, const OProp& P, int kind, const OQuad& q,
                          int npts, const int* pts, Cx<S>* out) {
  Vtx<S> VL = make_vtx<S>(Lv), VR = make_vtx<S>(Rv);
  int n = VL.g.n;
  std::vector<double> qv, qw;
  make_quad(q, qv, qw);
  int nq = q.n;
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < npts; ++p) {
    int cls = pts[4 * p], iw = pts[4 * p + 1], i = pts[4 * p + 2], j = pts[4 * p + 3];
    bool linf = (cls == C_K2P || cls == C_K1), rinf = (cls == C_K2 || cls == C_K1);
    double w = grid_node(VL.g, iw);
    double v = linf ? 0.0 : grid_node(VL.g, i);
    double vp = rinf ? 0.0 : grid_node(VL.g, j);
    Cx<S> aX[16], aY[16];
    for (int f = 0; f < 16; ++f) aX[f] = aY[f] = czero<S>();
    for (int k = 0; k < nq; ++k) {
      Cx<S> Pi[16], LX[16], LY[16], RX[16], RY[16], tX[16], tY[16];
      bubble_pi<S>(P, r, kind, w, qv[k], Pi);
      for (int f = 0; f < 16; ++f) Pi[f] = cmul(0.0, -qw[k] / (2.0 * M_PI), Pi[f]);
      left_factor(VL, r, w, v, qv[k], linf, LX, LY);
      right_factor(VR, r, w, qv[k], vp, rinf, RX, RY);
      spin_sums<S>(r, LX, LY, Pi, RX, RY, tX, tY);
      for (int f = 0; f < 16; ++f) {
        aX[f] = aX[f] + tX[f];
        aY[f] = aY[f] + tY[f];
      }
    }
    for (int f = 0; f < 16; ++f) {
      out[(size_t)p * 32 + f] = aX[f];
      out[(size_t)p * 32 + 16 + f] = aY[f];
    }
  }
}

// Integrand of the bubble at output (cls, iw, i, j) and loop frequencies vq[k]: the summand of
// bubble_points with Pi / (2 pi i) and no quadrature weight; out[p][k][2][16].
static void bubble_integrand(int r, const OVert& Lv, const OVert& Rv, const OProp& P, int kind, int npts,
                             const int* pts, int nv, const double* vq, Cx<double>* out) {
  Vtx<double> VL = make_vtx<double>(Lv), VR = make_vtx<double>(Rv);
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < npts; ++p) {
    int cls = pts[4 * p], iw = pts[4 * p + 1], i = pts[4 * p + 2], j = pts[4 * p + 3];
    bool linf = (cls == C_K2P || cls == C_K1), rinf = (cls == C_K2 || cls == C_K1);
    double w = grid_node(VL.g, iw);
    double v = linf ? 0.0 : grid_node(VL.g, i);
    double vp = rinf ? 0.0 : grid_node(VL.g, j);
    for (int k = 0; k < nv; ++k) {
      Cx<double> Pi[16], LX[16], LY[16], RX[16], RY[16], tX[16], tY[16];
      bubble_pi<double>(P, r, kind, w, vq[k], Pi);
      for (int f = 0; f < 16; ++f) Pi[f] = cmul(0.0, -1.0 / (2.0 * M_PI), Pi[f]);
      left_factor(VL, r, w, v, vq[k], linf, LX, LY);
      right_factor(VR, r, w, vq[k], vp, rinf, RX, RY);
      spin_sums<double>(r, LX, LY, Pi, RX, RY, tX, tY);
      Cx<double>* o = out + ((size_t)p * nv + k) * 32;
      for (int f = 0; f < 16; ++f) {
        o[f] = tX[f];
        o[16 + f] = tY[f];
      }
    }
  }
}

// ---------------------------------------------------------------- brute force
// Full vertex Gamma(1'2'|12) from leg quantum numbers (Keldysh al, spin sg in
// {0=up,1=down}, frequencies nu), summing every channel through its own
// parametrisation; SU(2) structure X d(s1',s1)d(s2',s2) + Y d(s1',s2)d(s2',s1).
template <class S>
static Cx<S> vertex_legs(const Vtx<S>& V, const int al[4], const int sg[4], const double nu[4]) {
  double dX = (sg[0] == sg[2] && sg[1] == sg[3]) ? 1.0 : 0.0;
  double dY = (sg[0] == sg[3] && sg[1] == sg[2]) ? 1.0 : 0.0;
  Cx<S> acc = czero<S>();
  if ((al[0] + al[1] + al[2] + al[3]) % 2 == 1) {
    S val = -0.5 * V.r0;
    acc = acc + Cx<S>{(dX - dY) * val, mk(0.0, (S*)nullptr)};
  }
  for (int rr = 0; rr < 3; ++rr) {
    if (V.coef[rr] == 0.0) continue;
    double w, v, vp;
    params_from(rr, nu, w, v, vp);
    Cx<S> tmp[2][16];
    for (int s = 0; s < 2; ++s)
      for (int f = 0; f < 16; ++f) tmp[s][f] = czero<S>();
    add_channel_classes(V, rr, w, v, vp, P_K1 | P_K2 | P_K2P | P_K3, V.coef[rr], tmp);
    int f = flat_of_legs(rr, al);
    acc = acc + dX * tmp[0][f] + dY * tmp[1][f];
  }
  return acc;
}

// Total bubble output gamma_r(1'2'|12) for external legs at channel parameters
// (w, v, vp), by the 8-fold compound-index sum of the defining formula.
// out[s][16]: s in {X, Y}, flat Keldysh index in channel r's pair order.
template <class S>
static void bubble_brute(int r, const OVert& Lv, const OVert& Rv, const OProp& P, int kind, const OQuad& q,
                         double w, double v, double vp, Cx<S> out[32]) {
  Vtx<S> VL = make_vtx<S>(Lv), VR = make_vtx<S>(Rv);
  std::vector<double> qv, qw;
  make_quad(q, qv, qw);
  double pref = r == 0 ? 1.0 : (r == 1 ? 0.5 : -1.0);
  const int sgX[4] = {0, 1, 0, 1};  // (s1',s2',s1,s2) = up dn | up dn
  const int sgY[4] = {0, 1, 1, 0};  // up dn | dn up
  double ext[4];
  legs_from(r, w, v, vp, ext);  // n1', n2', n1, n2
  for (int s = 0; s < 2; ++s) {
    const int* sg = s ? sgY : sgX;
    for (int f = 0; f < 16; ++f) {
      int al[4];
      legs_of_flat(r, f, al);
      Cx<S> acc = czero<S>();
      for (int k = 0; k < q.n; ++k) {
        double vq = qv[k];
        // internal propagator frequencies: G(3|3') at n3, G(4|4') at n4
        double n3, n4;
        if (r == 1) {
          n3 = w / 2 + vq;
          n4 = w / 2 - vq;
        } else {
          n3 = vq + w / 2;
          n4 = vq - w / 2;
        }
        Cx<S> g3[2][2], g4[2][2], s3[2][2], s4[2][2];
        propagator<S>(P, 0, n3, g3);
        propagator<S>(P, 0, n4, g4);
        if (kind == 1) {
          propagator<S>(P, 1, n3, s3);
          propagator<S>(P, 1, n4, s4);
        }
        for (int b3 = 0; b3 < 2; ++b3)
          for (int b3p = 0; b3p < 2; ++b3p)
            for (int b4 = 0; b4 < 2; ++b4)
              for (int b4p = 0; b4p < 2; ++b4p)
                for (int s3s = 0; s3s < 2; ++s3s)
                  for (int s4s = 0; s4s < 2; ++s4s) {
                    Cx<S> gg = kind == 0 ? g3[b3][b3p] * g4[b4][b4p]
                                         : s3[b3][b3p] * g4[b4][b4p] + g3[b3][b3p] * s4[b4][b4p];
                    // legs (1', 2', 1, 2) of the left and right vertices
                    int aL[4], sL[4], aR[4], sR[4];
                    double nL[4], nR[4];
                    if (r == 0) {  // G_L(1',4'|3,2) G_R(3',2'|1,4)
                      int a_[4] = {al[0], b4p, b3, al[3]};
                      int s_[4] = {sg[0], s4s, s3s, sg[3]};
                      double n_[4] = {ext[0], n4, n3, ext[3]};
                      int b_[4] = {b3p, al[1], al[2], b4};
                      int t_[4] = {s3s, sg[1], sg[2], s4s};
                      double m_[4] = {n3, ext[1], ext[2], n4};
                      memcpy(aL, a_, sizeof aL); memcpy(sL, s_, sizeof sL); memcpy(nL, n_, sizeof nL);
                      memcpy(aR, b_, sizeof aR); memcpy(sR, t_, sizeof sR); memcpy(nR, m_, sizeof nR);
                    } else if (r == 1) {  // G_L(1',2'|3,4) G_R(3',4'|1,2)
                      int a_[4] = {al[0], al[1], b3, b4};
                      int s_[4] = {sg[0], sg[1], s3s, s4s};
                      double n_[4] = {ext[0], ext[1], n3, n4};
                      int b_[4] = {b3p, b4p, al[2], al[3]};
                      int t_[4] = {s3s, s4s, sg[2], sg[3]};
                      double m_[4] = {n3, n4, ext[2], ext[3]};
                      memcpy(aL, a_, sizeof aL); memcpy(sL, s_, sizeof sL); memcpy(nL, n_, sizeof nL);
                      memcpy(aR, b_, sizeof aR); memcpy(sR, t_, sizeof sR); memcpy(nR, m_, sizeof nR);
                    } else {  // G_L(4',2'|3,2) G_R(1',3'|1,4)
                      int a_[4] = {b4p, al[1], b3, al[3]};
                      int s_[4] = {s4s, sg[1], s3s, sg[3]};
                      double n_[4] = {n4, ext[1], n3, ext[3]};
                      int b_[4] = {al[0], b3p, al[2], b4};
                      int t_[4] = {sg[0], s3s, sg[2], s4s};
                      double m_[4] = {ext[0], n3, ext[2], n4};
                      memcpy(aL, a_, sizeof aL); memcpy(sL, s_, sizeof sL); memcpy(nL, n_, sizeof nL);
                      memcpy(aR, b_, sizeof aR); memcpy(sR, t_, sizeof sR); memcpy(nR, m_, sizeof nR);
                    }
                    Cx<S> gl = vertex_legs(VL, aL, sL, nL);
                    Cx<S> gr = vertex_legs(VR, aR, sR, nR);
                    acc = acc + gl * gg * gr * cmul(0.0, -qw[k] / (2.0 * M_PI), Cx<S>{mk(1.0, (S*)nullptr), mk(0.0, (S*)nullptr)});
                  }
      }
      out[s * 16 + f] = pref * acc;
    }
  }
}

// ---------------------------------------------------------------- loop / SDE
// Loop L(G, G)(1'|1) = sum_{2,2'} int dv''/(2 pi i) Gamma(1',2'|1,2) G(2|2') with the
// spin sum over sigma_2 (gives 2X + Y), Gamma read in the a channel at
// w = v - v'', v_a = v'_a = (v + v'')/2.  out[i][4] = Sigma^{a1'|a1}, index 2*a1'+a1,
// at the vertex grid nodes.  kind selects G (0) or S (1) on the loop line.
template <class S>
static void loop_full(const OVert& Gv, const OProp& P, int kind, const OQuad& q, Cx<S>* out) {
  Vtx<S> V = make_vtx<S>(Gv);
  int n = V.g.n;
  std::vector<double> qv, qw;
  make_quad(q, qv, qw);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < n; ++i) {
    double v = grid_node(V.g, i);
    Cx<S> acc[4];
    for (int c = 0; c < 4; ++c) acc[c] = czero<S>();
    for (int k = 0; k < q.n; ++k) {
      double vq = qv[k];
      Cx<S> X[16], Y[16], g[2][2];
      eval_vertex(V, 0, v - vq, 0.5 * (v + vq), 0.5 * (v + vq), P_ALL, X, Y);
      propagator<S>(P, kind, vq, g);
      Cx<S> m = cmul(0.0, -qw[k] / (2.0 * M_PI), Cx<S>{mk(1.0, (S*)nullptr), mk(0.0, (S*)nullptr)});
      for (int a1p = 0; a1p < 2; ++a1p)
        for (int a1 = 0; a1 < 2; ++a1)
          for (int a2 = 0; a2 < 2; ++a2)
            for (int a2p = 0; a2p < 2; ++a2p) {
              int al[4] = {a1p, a2p, a1, a2};
              int f = flat_of_legs(0, al);
              Cx<S> sp = 2.0 * X[f] + Y[f];
              acc[2 * a1p + a1] = acc[2 * a1p + a1] + sp * g[a2][a2p] * m;
            }
    }
    for (int c = 0; c < 4; ++c) out[(size_t)i * 4 + c] = acc[c];
  }
}

// ---------------------------------------------------------------- susceptibility
// chi_a^c(w) = Pibar + sum_{k,l} Pi_k Gamma_a^c(w; v''_k, v''_l) Pi_l with Pi_k carrying
// w_k/(2 pi i); c = 0: X, c = 1: D = X + 2Y.  out[c][iw][16].
template <class S>
static void chi_full(const OVert& Gv, const OProp& P, const OQuad& q, Cx<S>* out, int nw = -1,
                     const int* wlist = nullptr, int r = 0) {
  Vtx<S> V = make_vtx<S>(Gv);
  int n = V.g.n;
  std::vector<double> qv, qw;
  make_quad(q, qv, qw);
  int nq = q.n;
  // all transfer frequencies, or the listed ones (out then holds [2][nw][16])
  const int cnt = nw < 0 ? n : nw;
  const int ostride = nw < 0 ? n : nw;
#pragma omp parallel for schedule(dynamic)
  for (int ii = 0; ii < cnt; ++ii) {
    const int iw = wlist ? wlist[ii] : ii;
    double w = grid_node(V.g, iw);
    std::vector<Cx<S>> Pi((size_t)nq * 16);
    for (int k = 0; k < nq; ++k) {
      bubble_pi<S>(P, r, 0, w, qv[k], &Pi[(size_t)k * 16]);
      for (int f = 0; f < 16; ++f) Pi[(size_t)k * 16 + f] = cmul(0.0, -qw[k] / (2.0 * M_PI), Pi[(size_t)k * 16 + f]);
    }
    // the channel's two spin combinations: a: X, X + 2Y (spin, density); p: X + Y, X - Y;
    // t: Y, 2X + Y
    const double cx[3][2] = {{1.0, 1.0}, {1.0, 1.0}, {0.0, 2.0}};
    const double cy[3][2] = {{0.0, 2.0}, {1.0, -1.0}, {1.0, 1.0}};
    for (int c = 0; c < 2; ++c) {
      Cx<S> acc[16];
      for (int f = 0; f < 16; ++f) acc[f] = czero<S>();
      for (int k = 0; k < nq; ++k)
        for (int f = 0; f < 16; ++f) acc[f] = acc[f] + Pi[(size_t)k * 16 + f];
      for (int k = 0; k < nq; ++k)
        for (int l = 0; l < nq; ++l) {
          Cx<S> X[16], Y[16], G[16], M[16], T[16];
          eval_vertex(V, r, w, qv[k], qv[l], P_ALL, X, Y);
          for (int f = 0; f < 16; ++f) G[f] = cx[r][c] * X[f] + cy[r][c] * Y[f];
          matmul4(&Pi[(size_t)k * 16], G, M);
          matmul4(M, &Pi[(size_t)l * 16], T);
          for (int f = 0; f < 16; ++f) acc[f] = acc[f] + T[f];
        }
      for (int f = 0; f < 16; ++f) out[((size_t)c * ostride + ii) * 16 + f] = acc[f];
    }
  }
}

// ---------------------------------------------------------------- C ABI
extern "C" {

void oracle_grid_nodes(int n, double L, double a, int map, double* nodes) {
  Grid g = make_grid(n, L, a, map);
  for (int i = 0; i < n; ++i) nodes[i] = grid_node(g, i);
}
void oracle_gauss_legendre(int n, double* x, double* w) { gauss_legendre(n, x, w); }
void oracle_quad(const OQuad* q, double* nodes, double* weights) {
  std::vector<double> v, w;
  make_quad(*q, v, w);
  for (int k = 0; k < q->n; ++k) {
    nodes[k] = v[k];
    weights[k] = w[k];
  }
}
int oracle_grid_locate(int n, double L, double a, int map, double v, int* i0, double* t) {
  Grid g = make_grid(n, L, a, map);
  return grid_locate(g, v, *i0, *t) ? 1 : 0;
}

// g[p][4] = G^{00}, G^{01}, G^{10}, G^{11} at nu[p]
void oracle_propagator(int dual, const OProp* P, int kind, int npts, const double* nu, double* g) {
  for (int p = 0; p < npts; ++p) {
    if (dual) {
      Cx<Dual> m[2][2];
      propagator<Dual>(*P, kind, nu[p], m);
      Cx<Dual>* o = (Cx<Dual>*)g + (size_t)p * 4;
      o[0] = m[0][0]; o[1] = m[0][1]; o[2] = m[1][0]; o[3] = m[1][1];
    } else {
      Cx<double> m[2][2];
      propagator<double>(*P, kind, nu[p], m);
      Cx<double>* o = (Cx<double>*)g + (size_t)p * 4;
      o[0] = m[0][0]; o[1] = m[0][1]; o[2] = m[1][0]; o[3] = m[1][1];
    }
  }
}

void oracle_bubble_integrand(int r, const OVert* L, const OVert* R, const OProp* P, int kind, int npts,
                             const int* pts, int nv, const double* vq, double* out) {
  bubble_integrand(r, *L, *R, *P, kind, npts, pts, nv, vq, (Cx<double>*)out);
}

void oracle_bubble_pi(int dual, const OProp* P, int r, int kind, double w, double vq, double* out16) {
  if (dual)
    bubble_pi<Dual>(*P, r, kind, w, vq, (Cx<Dual>*)out16);
  else
    bubble_pi<double>(*P, r, kind, w, vq, (Cx<double>*)out16);
}

// vertex in channel r at (w, v, vp): out[2][16] (X, Y)
void oracle_vertex_eval(int dual, const OVert* V, int r, unsigned parts, int npts, const double* wvv, double* out) {
  for (int p = 0; p < npts; ++p) {
    if (dual) {
      Vtx<Dual> v = make_vtx<Dual>(*V);
      Cx<Dual>* o = (Cx<Dual>*)out + (size_t)p * 32;
      eval_vertex(v, r, wvv[3 * p], wvv[3 * p + 1], wvv[3 * p + 2], parts, o, o + 16);
    } else {
      Vtx<double> v = make_vtx<double>(*V);
      Cx<double>* o = (Cx<double>*)out + (size_t)p * 32;
      eval_vertex(v, r, wvv[3 * p], wvv[3 * p + 1], wvv[3 * p + 2], parts, o, o + 16);
    }
  }
}

// vertex from explicit legs: al[4], sg[4], nu[4] per point -> out[p] complex
void oracle_vertex_legs(const OVert* V, int npts, const int* al, const int* sg, const double* nu, double* out) {
  Vtx<double> v = make_vtx<double>(*V);
  for (int p = 0; p < npts; ++p) {
    Cx<double> c = vertex_legs(v, al + 4 * p, sg + 4 * p, nu + 4 * p);
    out[2 * p] = c.re;
    out[2 * p + 1] = c.im;
  }
}

int oracle_bubble(int dual, int r, const OVert* L, const OVert* R, const OProp* P, int kind, const OQuad* q,
                  int cmask, double* K1, double* K2, double* K2p, double* K3) {
  if (r < 0 || r > 2 || L->n != R->n || L->n < 2 || q->n < 1) return -1;
  if (dual)
    bubble_full<Dual>(r, *L, *R, *P, kind, *q, cmask, (Cx<Dual>*)K1, (Cx<Dual>*)K2, (Cx<Dual>*)K2p, (Cx<Dual>*)K3);
  else
    bubble_full<double>(r, *L, *R, *P, kind, *q, cmask, (Cx<double>*)K1, (Cx<double>*)K2, (Cx<double>*)K2p,
                        (Cx<double>*)K3);
  return 0;
}

int oracle_bubble_points(int dual, int r, const OVert* L, const OVert* R, const OProp* P, int kind,
                         const OQuad* q, int npts, const int* pts, double* out) {
  if (r < 0 || r > 2 || L->n != R->n) return -1;
  if (dual)
    bubble_points<Dual>(r, *L, *R, *P, kind, *q, npts, pts, (Cx<Dual>*)out);
  else
    bubble_points<double>(r, *L, *R, *P, kind, *q, npts, pts, (Cx<double>*)out);
  return 0;
}

int oracle_bubble_brute(int r, const OVert* L, const OVert* R, const OProp* P, int kind, const OQuad* q, double w,
                        double v, double vp, double* out) {
  bubble_brute<double>(r, *L, *R, *P, kind, *q, w, v, vp, (Cx<double>*)out);
  return 0;
}

int oracle_loop(int dual, const OVert* G, const OProp* P, int kind, const OQuad* q, double* out) {
  if (dual)
    loop_full<Dual>(*G, *P, kind, *q, (Cx<Dual>*)out);
  else
    loop_full<double>(*G, *P, kind, *q, (Cx<double>*)out);
  return 0;
}

int oracle_chi_points(const OVert* G, const OProp* P, const OQuad* q, int nw, const int* wlist, double* out) {
  chi_full<double>(*G, *P, *q, (Cx<double>*)out, nw, wlist, 0);
  return 0;
}

int oracle_chi_channel(int r, const OVert* G, const OProp* P, const OQuad* q, int nw, const int* wlist, double* out) {
  if (r < 0 || r > 2) return -1;
  chi_full<double>(*G, *P, *q, (Cx<double>*)out, nw, wlist, r);
  return 0;
}

int oracle_chi(int dual, const OVert* G, const OProp* P, const OQuad* q, double* out) {
  if (dual)
    chi_full<Dual>(*G, *P, *q, (Cx<Dual>*)out);
  else
    chi_full<double>(*G, *P, *q, (Cx<double>*)out);
  return 0;
}

}  // extern "C"
