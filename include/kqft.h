/*
 * kqft.h -- C ABI of the MI355X Keldysh bubble / Schwinger-Dyson library.
 *
 * Method: real-frequency Keldysh diagrammatics of the single-impurity Anderson
 * model in the parquet approximation (Ritz, Ge, Walter, Aguirre, von Delft,
 * Kugler, arXiv:2405.20996).  The library computes the numerical bottleneck of
 * that method -- bubble integrals of two four-point vertices (Eq. B_a and the
 * Bethe-Salpeter equations), the loop/Schwinger-Dyson self-energy (Eq. SDE,
 * Sec. "The loop function"), susceptibilities (Sec. "Susceptibilities"), the
 * multiloop flow insertions (Eqs. 1l-3l of the mfRG section) and the adjoint of
 * the bubble -- on one AMD Instinct MI355X (gfx950), and the algorithms around it:
 * the parquet solver (mixing, Anderson acceleration, the three forms of the SDE), the
 * mfRG flow (regulators, Katanin substitution, self-energy corrections, Cash-Karp step
 * control), the asymmetric model (Hartree term, parquet solver and flow with the
 * self-energy's asymptotic value), susceptibilities of every channel, the bubble with
 * adaptive Gauss-Lobatto-Kronrod integration, the paper's algebraic frequency grid and the
 * regridding of a state between grids, and the finite-temperature Matsubara formalism
 * (bubble with analytic tails, SDE, loop, susceptibilities, parquet solver, hybridization
 * and interaction flows).
 *
 * Conventions shared by every entry point
 *   Keldysh basis: rotated, alpha in {0,1}; G^{0|0}=0, G^{0|1}=G^A, G^{1|0}=G^R,
 *     G^{1|1}=G^K; Sigma^{0|0}=Sigma^K, Sigma^{0|1}=Sigma^R, Sigma^{1|0}=Sigma^A.
 *   Bare vertex Gamma_0 (parquet approximation R = Gamma_0): -r0/2 on the
 *     Keldysh components with an odd index sum; spin X0 = Gamma_0, Y0 = -Gamma_0.
 *   Spin components (SU(2)): X = Gamma_{up dn|up dn}, Y = Gamma_{up dn|dn up}.
 *   Channel parameters (legs 1',2' outgoing, 1,2 incoming):
 *     a: w = n1'-n2, v = (n1'+n2)/2, v' = (n1+n2')/2
 *     p: w = n1'+n2', v = (n1'-n2')/2, v' = (n1-n2)/2
 *     t: w = n2'-n2, v = (n2'+n2)/2, v' = (n1'+n1)/2
 *   Keldysh 4x4 pair order (row pair | column pair), pair = 2*first + second,
 *     flat index 4*row + col:  a (a1',a2 | a1,a2'), p (a1',a2' | a1,a2),
 *     t (a2',a2 | a1',a1).
 *   Frequency grids (Sec. "Frequency grids"): n nodes equidistant in an
 *     auxiliary variable x_i = -1 + 2i/(n-1) mapped onto [-L, L]; all classes
 *     share one grid.  map KQFT_GRID_TAN: v_i = a*tan(x_i*atan(L/a));
 *     map KQFT_GRID_ALGEBRAIC (the paper's non-linear grid): v = a W|W|/sqrt(1-W^2)
 *     at W_i = W_L x_i, W_L < 1 the auxiliary value of v = L, so v ~ W^2 near zero
 *     and the extent is finite.
 *   Interpolation: linear in the auxiliary variable per axis (the paper's
 *     "linear_on_aux"); a class is zero where any argument lies outside [-L, L].
 *   Complex arrays: interleaved (re, im) doubles, C order, Keldysh innermost:
 *     K1[s][w][16], K2[s][w][v][16], K2p[s][w][v'][16], K3[s][w][v][v'][16],
 *     s = 0 (X), 1 (Y).
 *
 * Memory and errors
 *   Array arguments are device pointers (hipMalloc'd or from the caller's
 *   allocator) unless stated otherwise; the caller owns them and they must stay
 *   valid until the work enqueued on `stream` has completed.  Structs are host
 *   memory, read during the call only.  A NULL class pointer means "this class
 *   is zero".  The library owns only the workspace inside a kqft_ctx.
 *   Every function returns KQFT_OK (0) or a negative code; kqft_last_error()
 *   gives a message for the calling thread.  Host-side checks (sizes, enums,
 *   NULL outputs) run before anything is enqueued.  `stream` is a hipStream_t
 *   (NULL = the default stream).  A kqft_ctx is not thread-safe: use one per
 *   stream.
 *
 * Graph capture
 *   kqft_bubble and kqft_mloop_step enqueue no host synchronisation and no memset;
 *   after one call with the same sizes (workspace grown, grids and quadratures
 *   cached) they allocate nothing, so a call on a capturing stream records into the
 *   graph -- the library's internal streams join through events recorded on
 *   `stream` -- and the graph replays it (pointers as captured).  Under capture each
 *   bubble must run in one transfer-frequency batch (opts->omega_batch >= n, or an
 *   automatic or tuned batch covering the grid): a multi-batch schedule is rejected
 *   with KQFT_EINVAL (its capture crashed the runtime's graph instantiation).  The solvers, the
 *   flow, the Hartree term, the adaptive bubble and the adjoints synchronise or
 *   clear memory and are not to be captured.
 */
#ifndef KQFT_H
#define KQFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KQFT_OK = 0,
  KQFT_EINVAL = -1,  /* bad enum, NULL where not allowed */
  KQFT_ESHAPE = -2,  /* inconsistent grid / quadrature sizes */
  KQFT_ENOMEM = -3,  /* workspace allocation failed */
  KQFT_EDEVICE = -4, /* HIP runtime error */
  KQFT_ENOCONV = -5  /* an iteration or step limit was reached (flow step control) */
};
enum { KQFT_CH_A = 0, KQFT_CH_P = 1, KQFT_CH_T = 2 };
/* arithmetic of the bubble contraction: FP64 MFMA, or KQFT_SPLIT_FP32, the lowest rung of
   the split-precision ladder: every panel operand (vertex times Pi, formed in FP64) is rounded
   once to FP32 -- its hi part; the lo remainder is dropped, no hi*lo correction products are
   formed -- and multiplied on FP32 MFMA with FP32 partial sums over 128 complex terms promoted
   to FP64 between them.  Max-norm error about 3.3e-7 of the FP64 result at N = 201, within the
   1e-6 bound, so the compensated rungs (extra hi*lo + lo*hi products) are not built. */
enum { KQFT_FP64 = 0, KQFT_SPLIT_FP32 = 1 };
/* propagator pair: Pi = G G, or the differentiated Pidot = S G + G S with the
   single-scale propagator S = dG/dLambda at fixed Sigma of the propagator's regulator
   (S + G Sigma_dot G when the propagator carries Sigma_dot: Katanin substitution) */
enum { KQFT_PI_GG = 0, KQFT_PI_DOT = 1 };
/* regulators (Sec. "Flow schemes"), the flow parameter Lambda of S = dG/dLambda:
   DELTA: Lambda = Delta;  U: G_0 -> Lambda G_0 (interaction flow, Lambda = lam);
   T: Lambda = T (temperature flow);  NU: G_0 -> Theta G_0, Theta = v / (v + i lam) (lam > 0) */
enum { KQFT_REG_DELTA = 0, KQFT_REG_U = 1, KQFT_REG_T = 2, KQFT_REG_NU = 3 };
/* line of a loop (kqft_loop): G, the single-scale propagator (with Katanin, if Sigma_dot is
   given), or G Sigma_dot G */
enum { KQFT_LINE_G = 0, KQFT_LINE_S = 1, KQFT_LINE_GSG = 2 };
/* asymptotic classes of a bubble output */
enum { KQFT_K1 = 1, KQFT_K2 = 2, KQFT_K2P = 4, KQFT_K3 = 8, KQFT_KALL = 15 };
/* quadrature maps: Gauss-Legendre nodes y in [-1,1] mapped to v = a tan(y atan(L/a))
   (onto [-L, L]) or to v = a tan(pi y / 2) (onto the real line) */
enum { KQFT_QUAD_TAN_FINITE = 0, KQFT_QUAD_TAN_INFINITE = 1 };

/* frequency-grid maps (auxiliary variable -> frequency) */
enum { KQFT_GRID_TAN = 0, KQFT_GRID_ALGEBRAIC = 1 };

typedef struct {
  int n;    /* points, odd recommended (v = 0 is then a node), 2 <= n <= 600 (KQFT_ESHAPE) */
  double L; /* extent: nodes span [-L, L]; L and a finite and positive, else KQFT_ESHAPE */
  double a; /* map scale */
  int map;  /* KQFT_GRID_TAN (0, a zero-initialised grid) or KQFT_GRID_ALGEBRAIC; another value:
               KQFT_EINVAL.  Left and right vertices of a bubble must agree in n, L, a and map. */
} kqft_grid;

typedef struct {
  int n;   /* Gauss-Legendre nodes */
  int map; /* KQFT_QUAD_TAN_FINITE or KQFT_QUAD_TAN_INFINITE */
  double L, a;
} kqft_quad;

/* one channel gamma_r: coef * (K1 + K2 + K2' + K3), device arrays (NULL = 0) */
typedef struct {
  double coef;
  const double* K1;
  const double* K2;
  const double* K2p;
  const double* K3;
} kqft_chvert;

/* a four-point vertex Gamma = Gamma_0(r0) + sum_r gamma_r on one grid
   (parquet decomposition, Sec. "Diagrammatic many-body theory") */
typedef struct {
  double r0;
  kqft_grid grid;
  kqft_chvert ch[3];
} kqft_vertex;

/* propagator (Sec. "The Propagator class", Sec. "Flow schemes"):
     G^R = 1/(G_0^{-1,R}(v) - Sigma^R(v)),  G^K = G^R [Sigma^K - G_0^{-1,K}] G^A,
     G_0^{-1,K} = 2 i tanh(v/2T) Im G_0^{-1,R}  (bath in equilibrium),
   G_0^{-1,R} = v - eps + i Delta (reg DELTA and T), (v - eps + i Delta) / lam (reg U),
   (v - eps + i Delta)(v + i lam) / v (reg NU).  SigR/SigK are optional device arrays of n
   complex values on sgrid (NULL SigR: Sigma = 0; NULL SigK with SigR given: equilibrium
   FDR Sigma^K = 2i tanh(v/2T) Im Sigma^R).  dSigR/dSigK: optional Sigma_dot on sgrid (both
   or neither); with them the single-scale line becomes S + G Sigma_dot G (Katanin) and the
   GSG line of a loop is G Sigma_dot G,
     (G s G)^R = G^R s^R G^R,  (G s G)^K = G^R s^R G^K + G^R s^K G^A + G^K s^A G^A;
   deps, a real constant added to s^R and s^A at every frequency (the flow of the level eps),
   enters the same lines (alone too, without dSigR/dSigK).
   A zero-initialised struct (reg 0, no Sigma_dot) is the plain Delta-regulated propagator. */
typedef struct {
  double Delta, T, eps;
  kqft_grid sgrid;
  const double* SigR;
  const double* SigK;
  int reg;    /* KQFT_REG_* */
  double lam; /* regulator parameter of reg U (> 0) and NU (> 0); unused otherwise */
  const double* dSigR;
  const double* dSigK;
  double deps; /* 0 unless the level flows (asymmetric model) */
} kqft_propagator;

/* output classes of one channel (device arrays, layouts as above; NULL = skip) */
typedef struct {
  double* K1;
  double* K2;
  double* K2p;
  double* K3;
} kqft_chout;

typedef struct {
  int precision;   /* KQFT_FP64 or KQFT_SPLIT_FP32 */
  int class_mask;  /* KQFT_K* bits of the outputs to compute */
  int beta;        /* 0: overwrite outputs, 1: add into them */
  int omega_batch; /* transfer frequencies per panel batch, 0 = automatic */
  int overlap;     /* 0: panel gathers and GEMMs of consecutive transfer-frequency batches run
                      one after the other (the faster schedule on gfx950: both kernels want
                      the whole chip); 1: the gathers of the next batch run concurrently with
                      the current GEMM on a second internal stream */
} kqft_opts;

typedef struct kqft_ctx kqft_ctx;

/* Create a context bound to HIP device `device` (workspace, cached grids). */
int kqft_ctx_create(kqft_ctx** ctx, int device);
int kqft_ctx_destroy(kqft_ctx* ctx);
/* Message of the last error on the calling thread ("" if none). */
const char* kqft_last_error(void);
/* Kernel timing for measurement: while enabled, every kernel launch of the library is
   bracketed by HIP events on the caller's stream.  kqft_ctx_profile_read synchronises
   those events and returns, per kernel kind (0 = propagator pair, 1 = gather, 2 = GEMM,
   3 = loop / susceptibility reductions and the GEMMs' unmix epilogue), the summed
   milliseconds and the launch counts,
   then clears them.  ms and launches: host arrays of 4. */
int kqft_ctx_profile(kqft_ctx* ctx, int enable);
int kqft_ctx_profile_read(kqft_ctx* ctx, double* ms, int* launches);
/* Workspace bytes a call of kqft_bubble with these sizes will hold. */
size_t kqft_bubble_workspace(int n, int nq, int omega_batch, int precision);

/*
 * kqft_bubble -- B_r(left, right) = left o Pi_r o right (Eq. B_a; p and t analogous
 * with prefactors +1/2 and -1, Eqs. BSE), the sum over internal Keldysh and spin
 * indices done before the frequency integral (Sec. "The bubble_function"):
 *
 *   gamma_r(w, v, v') = pref_r sum_k w_k/(2 pi i) Gamma_L(w, v, v''_k) Pi_r(w, v''_k)
 *                                                 Gamma_R(w, v''_k, v')
 *
 * with the literal spin sums of the compound-index bubbles and the v'' integral
 * replaced by the quadrature q.  The result is split into asymptotic classes
 * (Sec. "The Vertex classes"): K3 from the parts of Gamma_L, Gamma_R that depend on
 * the external fermionic frequency, K2 / K2' from one such part, K1 from neither.
 * Outputs are written on left->grid (left and right must share it) for the
 * classes in opts->class_mask, overwritten (beta = 0) or accumulated (beta = 1).
 * Unlike the paper's bubble_function, the result is not implicitly added to an
 * existing vertex.
 * Arguments: channel KQFT_CH_*; pi_kind KQFT_PI_*; out: device arrays of the
 * selected classes (others may be NULL).  Errors: KQFT_EINVAL, KQFT_ESHAPE,
 * KQFT_ENOMEM, KQFT_EDEVICE.
 */
int kqft_bubble(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                const kqft_chout* out, void* stream);

/*
 * kqft_sde -- dynamic self-energy from the Schwinger-Dyson equation (Eq. SDE, a-channel
 * form) and the a-channel susceptibilities (Sec. "Susceptibilities"):
 *
 *   Phi = B_a(Gamma_0, Gamma)  (classes K1, K2'; q_bubble),
 *   Sigma^{a1'|a1}(v_i) = -1/2 sum_j w_j/(2 pi i) sum_{a2,a2'} [2 Phi^X + Phi^Y]
 *                           (w = v_i - v_j, v' = (v_i + v_j)/2) G^{a2|a2'}(v_j)   (q_loop),
 *   chi_a^c(w) = Pibar_a(w) + sum_{k,l} Pi_k Gamma_a^c(w; v''_k, v''_l) Pi_l,
 *                c = X (transverse spin) and D = X + 2Y (density)             (q_bubble).
 *
 * The Hartree term of the rotated-basis loop, -L(Gamma_0, G) = U(<n> - 1/2), vanishes at
 * particle-hole symmetry and its constant U/2 is part of G (Sec. "Hartree-Fock"); Sigma
 * is the dynamic part.  sigma: device [n][4] complex (index 2*a1' + a1) on gamma->grid;
 * chi: device [2][n][16] complex or NULL (when given, q_bubble->n <= 46340, else
 * KQFT_ESHAPE).  FP64 throughout (the contraction inside Phi uses opts->precision).
 */
int kqft_sde(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q_bubble,
             const kqft_quad* q_loop, const kqft_opts* opts, double* sigma, double* chi, void* stream);

/*
 * kqft_chi -- the pair-space susceptibility of one channel (Sec. "Susceptibilities": legs of
 * the vertex contracted in pairs, here in channel r = `channel`):
 *
 *   chi_r^c(w) = sum_k Pi_r,k(w) + sum_{k,l} Pi_r,k(w) Gamma_r^c(w; v''_k, v''_l) Pi_r,l(w),
 *
 * Pi_r,k the 4x4 Keldysh pair-space bubble G G of channel r at v''_k times w_k/(2 pi i)
 * (q), products of 4x4 matrices in channel r's pair order, and Gamma_r^c the full vertex
 * (bare part, channel r's own classes, the two other channels) in channel r's
 * parametrization and spin combination c: a: X (transverse spin), X + 2Y (density);
 * p: X + Y, X - Y; t: Y, 2X + Y.  chi: device [2][n][16] complex on gamma->grid (c, w, pair
 * entry 4*row + col), written completely.  FP64 throughout.  KQFT_EINVAL for a NULL
 * argument or a channel outside 0..2, KQFT_ESHAPE for an invalid quadrature or q->n > 46340
 * (the double sum is indexed in 32 bits).  channel = KQFT_CH_A gives kqft_sde's chi.
 */
int kqft_chi(kqft_ctx* ctx, int channel, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
             double* chi, void* stream);

/* ---------------------------------------------------------------- Matsubara formalism
 * Finite temperature, imaginary frequencies (the paper's code also runs its diagrammatic
 * functions with Matsubara sums; Sec. "Vectorization": the sums as matrix products).
 * Frequencies nu_n = (2n + 1) pi T, Omega_m = 2 m pi T; legs of channel r's (m, n, n'), every
 * leg fermionic:  a: n2 = n, n1' = n + m, n2' = n', n1 = n' + m;  p: n1' = n,
 * n2' = m - n - 1, n1 = n', n2 = m - n' - 1;  t: n2 = n, n2' = n + m, n1' = n', n1 = n' + m.
 * Classes (no Keldysh index): K1[s][m], K2[s][m][n], K2p[s][m][n'], K3[s][m][n][n'], s = X, Y,
 * m in [-M, M] (index m + M), n, n' in [-N, N) (index n + N), complex, zero outside. */
typedef struct {
  int M;    /* bosonic box [-M, M], M >= 0 */
  int N;    /* fermionic box [-N, N), N >= 1 */
  double T; /* temperature > 0 */
} kqft_mgrid;

/* Gamma = Gamma_0 + sum_r coef_r gamma_r with X0 = -U, Y0 = +U */
typedef struct {
  kqft_mgrid grid;
  double U;
  kqft_chvert ch[3];
} kqft_mvertex;

/* G(i nu_n) = 1/(i nu_n + i Delta sgn(nu_n) - Sigma(n)) (level 0: particle-hole symmetric model
   with U/2 absorbed); sigma: device complex on n in [-sigma_N, sigma_N) or NULL.  The flow
   parameter is Delta (reg KQFT_REG_DELTA, 0): S = dG/dDelta at fixed Sigma = -i sgn(nu) G^2;
   or lam (reg KQFT_REG_U, the interaction flow of Sec. "Flow schemes"): G_0 -> lam G_0, so
   G = 1/(G_0^-1/lam - Sigma) and S = dG/dlam at fixed Sigma = G G_0^-1 G / lam^2 (lam > 0);
   plus G Sigma_dot G with dsigma (device complex on the same box, or NULL).  Another reg:
   KQFT_EINVAL. */
typedef struct {
  double Delta;
  const double* sigma;
  int sigma_N;
  const double* dsigma;
  int reg;
  double lam;
} kqft_mprop;

/*
 * kqft_bubble_matsubara -- B_r(left, right) in the Matsubara formalism:
 *   B_r(m; n, n') = pref_r T sum_{n''} left(m; n, n'') Pi_r(m, n'') right(m; n'', n')
 * (pi_kind KQFT_PI_GG: Pi = G G; KQFT_PI_DOT: Pi_dot = S G + G S with S of kqft_mprop).
 * tails = 1 (Pi = G G only; Sec. "asymptotic corrections", the analytic-tails option) adds the
 * summands beyond the window through the bare bubble, whose full sum is known in closed form
 * (digamma functions): t(m) = that sum minus the window's bare sum, times the vertices' values
 * at large n'' (left Gamma_0 + K1 + K2(m, n), right Gamma_0 + K1 + K2'(m, n') of the channel),
 * split over the classes like the bubble itself.
 * with the spin sums of the real-frequency bubble (the same two combinations per channel,
 * prefactors +1, 1/2, -1), Pi_a = Pi_t = G(n'' + m) G(n''), Pi_p = G(n'') G(m - n'' - 1), the
 * sum over the window |2n'' + 1 + s m| <= 2 Nq - 1 (s = +1 for a and t, -1 for p; symmetric
 * about the bubble's centre, no tail correction), and the asymptotic classes as in kqft_bubble
 * (L^inf = Gamma_0 + K1 + K2' of the own channel at (m, n''), R^inf = Gamma_0 + K1 + K2):
 * K3 = (L - L^inf) Pi (R - R^inf), K2 = (L - L^inf) Pi R^inf, K2' = L^inf Pi (R - R^inf),
 * K1 = L^inf Pi R^inf.  The product per bosonic frequency and combination is a complex
 * (2N + 1) x 2Nq x (2N + 1) GEMM (the library's FP64 MFMA GEMM, batched over m).  left and right on
 * the same grid; out: all four classes (device, overwritten).  FP64.  KQFT_EINVAL for NULL
 * arguments, a bad channel or non-positive T / Delta; KQFT_ESHAPE for mismatched grids, M < 0,
 * N < 1, Nq < 1 or sizes whose panels exceed 2^31 entries.
 */
int kqft_bubble_matsubara(kqft_ctx* ctx, int channel, const kqft_mvertex* left, const kqft_mvertex* right,
                          const kqft_mprop* G, int pi_kind, int Nq, int tails, const kqft_chout* out, void* stream);

/*
 * kqft_loop_matsubara -- the loop of a full Matsubara vertex (bare part, every channel at its own
 * parameters): L(Gamma, X)(n) = T sum_{n'} [2X + Y](legs n, n' | n, n') X(n'), |2n' + 1| <=
 * 2 Nl - 1, X = G, S (+ G Sigma_dot G with dsigma) or G Sigma_dot G (KQFT_LINE_G, _S, _GSG).
 * out: device [2N] complex.  FP64.  KQFT_EINVAL / KQFT_ESHAPE as kqft_bubble_matsubara.
 */
int kqft_loop_matsubara(kqft_ctx* ctx, const kqft_mvertex* gamma, const kqft_mprop* G, int kind, int Nl,
                        double* out, void* stream);

/*
 * kqft_regrid -- a state's classes and self-energy carried from grid `src` onto grid `dst` by the
 * interpolation every lookup uses (Sec. Interpolation routines: multilinear on the auxiliary
 * variable; zero where an argument lies outside src's extent), e.g. to rescale the frequency
 * grids between segments of a hybridization flow (Sec. Frequency grids).  gamma_in/gamma_out:
 * three channels, classes in the vertex layouts on src resp. dst (a NULL class is skipped and
 * must be NULL on both sides); sigma_in/sigma_out: [n][4] complex on src resp. dst, or both NULL.
 * Inputs are read only; outputs are overwritten and must not alias the inputs.  FP64, enqueued
 * on `stream`.  KQFT_EINVAL for missing or aliased arguments, KQFT_ESHAPE for invalid grids.
 */
int kqft_regrid(kqft_ctx* ctx, const kqft_grid* src, const kqft_grid* dst, const kqft_chout* gamma_in,
                const double* sigma_in, const kqft_chout* gamma_out, double* sigma_out, void* stream);

/*
 * kqft_chi_matsubara -- susceptibility of channel r (`channel`) in the Matsubara formalism:
 *   chi_r^c(m) = T sum_k Pi_r(m, k) + T^2 sum_{k,l} Pi_r(m, k) Gamma_r^c(m; k, l) Pi_r(m, l)
 * over the bubble's window (Nq), the full vertex in channel r's parameters and spin combination
 * c (a: X, X + 2Y; p: X + Y, X - Y; t: Y, 2X + Y).  chi: device [2][2M + 1] complex.  FP64.
 * KQFT_ESHAPE also for Nq > 16384 (the pair count is indexed in 32 bits).
 */
int kqft_chi_matsubara(kqft_ctx* ctx, int channel, const kqft_mvertex* gamma, const kqft_mprop* G, int Nq,
                       double* chi, void* stream);

/*
 * kqft_sde_matsubara -- the Schwinger-Dyson self-energy in the Matsubara formalism (a-channel
 * form, Hartree part absorbed at particle-hole symmetry):
 *   Phi = B_a(Gamma_0, Gamma) (kqft_bubble_matsubara, window Nq; classes K1 and K2'),
 *   Sigma(n) = -1/2 T sum_{n'} [2 Phi^X + Phi^Y](m = n - n', n', n') G(n'),  |2n' + 1| <= 2 Nl - 1,
 * for n in [-N, N); Phi is zero outside its boxes (take M >= N + Nl to keep every term).
 * sigma_out: device [2N] complex (index n + N).  FP64.  Errors as kqft_bubble_matsubara, and
 * KQFT_ESHAPE for Nl < 1.
 */
int kqft_sde_matsubara(kqft_ctx* ctx, const kqft_mvertex* gamma, const kqft_mprop* G, int Nq, int Nl,
                       double* sigma_out, void* stream);

/*
 * kqft_loop -- the loop function of a full vertex (Sec. "loop": the self-energy-like
 * contraction of a vertex with one propagator line):
 *   L(Gamma, X)^{a1'|a1}(v_i) = sum_j w_j/(2 pi i) sum_{a2,a2'} [2 Gamma^X + Gamma^Y]
 *                                 (legs v_i, v_j | v_i, v_j) X^{a2|a2'}(v_j),
 * X = G (KQFT_LINE_G), the single-scale propagator S = dG/dLambda at fixed Sigma of G's
 * regulator, plus G Sigma_dot G when G carries Sigma_dot (KQFT_LINE_S), or G Sigma_dot G
 * alone (KQFT_LINE_GSG, needs Sigma_dot);
 * Gamma = Gamma_0(r0) + sum_r coef_r gamma_r, every channel read at its own parameters.
 * The one-loop self-energy flow is Sigma_dot = -L(Gamma, S).  out: device [n][4] complex
 * (index 2*a1' + a1) on gamma->grid.  FP64.
 */
int kqft_loop(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, int kind, const kqft_quad* q,
              double* out, void* stream);

/* what an adaptive bubble did */
typedef struct {
  long long intervals;   /* accepted intervals, summed over the outputs */
  int generations;       /* refinement generations */
  long long evaluations; /* integrand evaluations (nodes x outputs, the error scales included) */
} kqft_adapt_info;

/*
 * kqft_bubble_adaptive -- the bubble B_r(left, right) of kqft_bubble with the loop integral
 * done by adaptive Gauss-Lobatto-Kronrod quadrature per output entry (Sec. "Frequency
 * integration") instead of a fixed Gauss-Legendre rule.  For every selected output (class,
 * w, v, v') the vector of its 32 entries (16 Keldysh x X, Y) is integrated over the auxiliary
 * variable y in [-1, 1] of q's tangent map v'' = q->a tan(y atan(q->L / q->a)) (q->map must
 * be KQFT_QUAD_TAN_FINITE; q->n is unused) with the Jacobian: I_s = GLK13 over [-1, 1] sets
 * the error scale max|I_s| ((b - a) max|F| at its nodes if that vanishes, else 1); an
 * interval is accepted with its GLK7 value when max|GLK7 - GL4| <= eps max|I_s|, narrower
 * than 1e-12 or 40 subdivisions deep, else split at the seven GLK7 nodes into six.  The work
 * proceeds breadth first over batches of up to 8192 outputs (one wavefront per output
 * interval, one synchronisation per generation).  FP64; outputs
 * overwritten for the classes of opts->class_mask (precision, beta, omega_batch ignored).
 * info (host, or NULL).  Errors as kqft_bubble, KQFT_ENOMEM when one generation of a batch
 * exceeds 2^24 intervals (two such lists of 24 bytes per interval are held), KQFT_ENOCONV
 * when the refinement does not end.
 */
int kqft_bubble_adaptive(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                         const kqft_propagator* G, int pi_kind, const kqft_quad* q, double eps, const kqft_opts* opts,
                         const kqft_chout* out, kqft_adapt_info* info, void* stream);

/*
 * kqft_hartree -- Hartree term of the impurity level eps_d (Sec. "Hartree-Fock", Eq. Hartree):
 *   Sigma_H = U <n_sigma>,   <n_sigma> = 1/2 + (1/2 pi) int dv tanh(v/2T) Im G_H^R(v),
 *   G_H^R(v) = 1/(v - eps_d - Sigma_H + i Delta - Sigma^R_dyn(v))
 * (Eq. Hartree with G^< = -2i n_F Im G^R in equilibrium, n_F = (1 - tanh(v/2T))/2, and the
 * spectral sum rule int A = 1 for the constant half, which keeps <n> = 1/2 exact at
 * particle-hole symmetry for a self-energy given on a grid), integrated with the quadrature q
 * (use KQFT_QUAD_TAN_INFINITE: the integrand has Lorentzian tails).  G supplies Delta, T and the
 * optional dynamic self-energy (SigR on sgrid); G->eps is replaced by eps_d + Sigma_H; the
 * regulator must be KQFT_REG_DELTA without Sigma_dot.
 *   self_consistent = 0: one shot; *sigma_H in: the Hartree term inside G_H, out: U <n>.
 *   self_consistent = 1: bisection of f(x) = x - U n(eps_d + x) on [0, U] (f is increasing,
 *   f(0) <= 0 <= f(U)) until the bracket is narrower than tol; *sigma_H out: the midpoint.
 * U >= 0, tol > 0 (self-consistent).  iterations (host, or NULL): evaluations of <n>.
 * Synchronises `stream` once per evaluation.  FP64.
 */
int kqft_hartree(kqft_ctx* ctx, double U, double eps_d, const kqft_propagator* G, const kqft_quad* q,
                 int self_consistent, double tol, double* sigma_H, int* iterations, void* stream);

/* options of kqft_mfrg_flow */
typedef struct {
  int reg;               /* KQFT_REG_*: the flow parameter */
  double Delta;          /* hybridization of the flows other than the Delta-flow */
  int katanin;           /* 1: the differentiated bubble uses S + G Sigma_dot G; 0: S */
  int se_iterations;     /* multiloop self-energy corrections (nloops >= 3): at most this many
                            iterations per right-hand side; 0: none */
  double se_tol_abs;     /* stop when max|Sigma_dot_new - Sigma_dot| <= abs + rel max|Sigma_dot_new| */
  double se_tol_rel;
  int se_anderson;       /* Anderson depth of the correction iterations (0: plain iteration;
                            else the next iterate is the Anderson step with mixing factor 1 over
                            the last se_anderson iterations, as in kqft_parquet_solve) */
  int adaptive;          /* 0: classical RK4 in `steps` equal steps; 1: Cash-Karp step control */
  double ode_tol_abs;    /* accept a step when max_i |e_i| / (abs + rel max(|y_i|, |y4_i|)) <= 1 */
  double ode_tol_rel;
  int max_steps;         /* accepted + rejected steps (adaptive); KQFT_ENOCONV beyond */
  int asymmetric;        /* 0: particle-hole symmetric model (level 0, Hartree U/2 absorbed);
                            1: asymmetric model (Sec. "Hartree-Fock", Sec. "The loop function"):
                            the level of G is eps_d + Sigma_inf, Sigma_inf the self-energy's
                            asymptotic value (real, beyond the grid), one more state entry */
  double eps_d;          /* bare level (asymmetric) */
  double sigma_inf;      /* initial Sigma_inf (asymmetric; e.g. the Hartree term of kqft_hartree) */
} kqft_flow_opts;

/* what a flow did */
typedef struct {
  int accepted;          /* accepted steps */
  int rejected;          /* rejected trial steps */
  int rhs_evaluations;   /* right-hand sides evaluated */
  int se_iterations;     /* self-energy correction iterations, summed over the right-hand sides */
  double sigma_inf;      /* final Sigma_inf (asymmetric; 0 otherwise) */
} kqft_flow_info;

/*
 * kqft_mfrg_flow -- multiloop fRG flow (Sec. "mfRG", Sec. "Details on the ODE-solver",
 * Sec. "Flow schemes") of the state (Gamma = Gamma_0(U) + sum_r gamma_r, Sigma) from
 * Lambda_i to Lambda_f.  Right-hand side at Lambda, with G dressed by the state's Sigma:
 *   Sigma_dot^(1) = -L(Gamma, S)                         (one-loop self-energy flow),
 *   Gamma_dot     = sum_{l <= nloops} gdot^(l)          (the insertions of kqft_mloop_step,
 *                   the l = 1 bubble along S + G Sigma_dot G with katanin, else S),
 * and with se_iterations > 0 and nloops >= 3, iterated from there:
 *   Sigma_dot_tbar = -L(sum_l (gdot_{a,C}^(l) + gdot_{p,C}^(l)), G)   (centre terms),
 *   Sigma_dot_t    = -L(Gamma, G Sigma_dot_tbar G),
 *   Sigma_dot      = Sigma_dot^(1) + Sigma_dot_tbar + Sigma_dot_t,
 * re-evaluating Gamma_dot with each new Sigma_dot until the change is within tolerance.
 * The ODE runs in t with Lambda(t) = 5 t|t| / sqrt(1 - t^2) for the Delta-flow and
 * Lambda = t otherwise; classical RK4 in `steps` equal steps in t, or Cash-Karp advancing
 * the fourth-order solution with the first trial step (t_f - t_i)/steps, growth by
 * min(5, 0.9 err^-1/5) after an accepted and shrinkage by max(0.1, 0.9 err^-1/4) after a
 * rejected step, the last step cut to land on t_f.
 * Asymmetric model (asymmetric = 1): Sigma = Sigma_inf + sigma with the real constant Sigma_inf
 * carried as the level (G_0 at eps_d + Sigma_inf) and sigma on the grid, zero beyond it.
 * Every loop L(Gamma, X) above also yields its asymptotic value: the loop of the part of Gamma
 * that does not depend on the external frequency in the loop's legs (v, v_j | v, v_j) -- the
 * bare vertex and the t-channel classes K1_t(0) and K2_t(0, v_j), the t channel sitting at
 * transfer frequency 0 -- the same at every v; d Sigma_inf takes minus its real retarded part,
 * and the grid values of that loop minus the same constant (retarded and advanced components)
 * go to sigma_dot.  The G Sigma_dot G lines carry the constant as the flow of the level
 * (kqft_propagator.deps).  The correction loop of the centre terms has no such part.
 * State in/out: gamma[3] (the three channels, all four classes, device) and sigma (device
 * [n][4], Sigma^K at index 0 and Sigma^R at 1, on grid).  lambdas (host, capacity
 * max_steps + 1 for adaptive, steps + 1 otherwise, or NULL): the accepted Lambda values,
 * starting with Lambda_i; info (host, or NULL).  Bubbles in opts->precision, loops FP64.
 * Synchronises `stream` once per trial step (adaptive) and per correction iteration.
 * Working memory: 9 (adaptive) or 4 states plus nloops x 3 channels.
 */
int kqft_mfrg_flow(kqft_ctx* ctx, const kqft_grid* grid, double U, double T, double Lambda_i, double Lambda_f,
                   int steps, int nloops, const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                   const kqft_flow_opts* flow, const kqft_chout* gamma, double* sigma, double* lambdas,
                   kqft_flow_info* info, void* stream);

/*
 * kqft_mfrg_flow_matsubara -- the mfRG flow (Sec. "mfRG") in the Matsubara formalism with the
 * hybridization as flow parameter (Delta from Lambda_i to Lambda_f; the ODE in t with
 * Delta = 5 t|t| / sqrt(1 - t^2); with reg = KQFT_REG_U the interaction flow G_0 -> Lambda G_0
 * at the fixed hybridization `Delta` (unused otherwise), the ODE in Lambda itself): classical RK4 in `steps` equal steps, or with adaptive = 1
 * the Cash-Karp step control of kqft_mfrg_flow (tolerances ode_tol_abs/ode_tol_rel on the
 * whole state, first trial step (t_f - t_i)/steps, at most max_steps trial steps, else
 * KQFT_ENOCONV with the state where it stopped)):
 *   Sigma_dot^(1) = -L(Gamma, S)                         (kqft_loop_matsubara, window Nl),
 *   Gamma_dot     = sum_{l <= nloops} gdot^(l): l = 1 B_r(Gamma, Gamma; Pi_dot) along S
 *                   (+ G Sigma_dot G with katanin), l = 2 B_r(gdot_rbar, Gamma) + B_r(Gamma,
 *                   gdot_rbar), l >= 3 also B_r(Gamma, B_r(gdot_rbar^(l-2), Gamma))   (window Nq),
 * and with se_iterations > 0 and nloops >= 3 the corrections Sigma_dot_tbar = -L(sum of the
 * a and p centre terms, G), Sigma_dot_t = -L(Gamma, G Sigma_dot_tbar G), Sigma_dot = Sigma_dot^(1)
 * + Sigma_dot_tbar + Sigma_dot_t, iterated until max|change| <= abs + rel max|Sigma_dot| or
 * se_iterations times.  State in/out: gamma[3] (device classes on grid) and sigma (device [2N]).
 * lambdas (host, capacity max_steps + 1 for adaptive, steps + 1 otherwise, or NULL): the
 * accepted Delta values from Lambda_i; info (host, or NULL): step and evaluation counts
 * (sigma_inf unused).  FP64.  Synchronises `stream` once per correction iteration and per
 * trial step (adaptive).
 */
int kqft_mfrg_flow_matsubara(kqft_ctx* ctx, const kqft_mgrid* grid, double U, double Lambda_i, double Lambda_f,
                             int reg, double Delta, int steps, int nloops, int Nq, int Nl, int katanin, int se_iterations, double se_tol_abs,
                             double se_tol_rel, int adaptive, double ode_tol_abs, double ode_tol_rel, int max_steps,
                             const kqft_chout* gamma, double* sigma, double* lambdas, kqft_flow_info* info,
                             void* stream);

/*
 * kqft_parquet_iteration -- right-hand sides of the parquet equations (Sec. "parquet
 * solver"; BSEs and Eq. SDE) for the state (gamma, Sigma in G):
 *   gamma_r' = 1/2 [B_r(I_r, Gamma) + B_r(Gamma, I_r)],  I_r = Gamma without channel r
 *              (the symmetrized Bethe-Salpeter equations, r = a, p, t),
 *   Sigma'   = the Schwinger-Dyson self-energy of Gamma (a-channel form, as kqft_sde),
 * Gamma = Gamma_0(r0) + sum_r coef_r gamma_r.  gamma_out[3]: device arrays of the three
 * channels (all four classes required; must not alias the inputs); sigma_out: device
 * [n][4] complex.  Bubbles in opts->precision, Sigma in FP64.
 */
int kqft_parquet_iteration(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G,
                           const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                           const kqft_chout* gamma_out, double* sigma_out, void* stream);

/* options of kqft_parquet_solve (Sec. "parquet solver": mixing, Anderson acceleration) */
typedef struct {
  double alpha;        /* mixing factor, 0 < alpha <= 1 */
  int max_iterations;  /* >= 1 */
  double tol;          /* stop after the update of the first iteration with residual < tol */
  int anderson_depth;  /* m: 0 = linear mixing, else Anderson acceleration over the last m
                          iterations (0 <= m <= 32) */
  int reduce_alpha;    /* 1: an iteration whose residual exceeds the previous one halves alpha
                          (not below alpha_min) and clears the Anderson history */
  double alpha_min;    /* 0 < alpha_min <= alpha when reduce_alpha */
  int hartree;         /* 0: level 0 (particle-hole symmetric model, Sigma_H = U/2 absorbed);
                          1: asymmetric model with level eps_d + Sigma_H (Sec. "Hartree-Fock") */
  double eps_d;        /* bare level (hartree = 1) */
  kqft_quad q_hartree; /* quadrature of the occupation (hartree = 1; full-line map) */
  double hartree_tol;  /* bracket width of the self-consistent Hartree term of the PT2 start */
  int sde_forms;       /* 1 (or 0): the self-energy from the a-channel form of the SDE (as
                          kqft_sde); 3: the mean of the SDE's three forms (Sec. "parquet solver"),
                          its two inner lines read as an a, a p or a t bubble:
                            Sigma_a = -1/2 L(B_a(Gamma_0, Gamma), G),
                            Sigma_p = -L(B_p(Gamma_0, Gamma), G),
                            Sigma_t = +1/2 (B_t(Gamma_0, Gamma) closed between its legs 2 and 1');
                          the t-form equals the a-form for the crossing-symmetric states of the
                          solver, which evaluates (2 Sigma_a + Sigma_p) / 3.  Any other value:
                          KQFT_EINVAL */
} kqft_parquet_opts;

/*
 * kqft_parquet_solve -- parquet solver (Sec. "parquet solver"): starts from the PT2 state
 * (gamma_r = K1_r = B_r(Gamma_0, Gamma_0), Sigma = SDE(Gamma_0) with the bare propagator),
 * then iterates the fixed point x = F(x) of the state x = (three channels, Sigma), F being
 * kqft_parquet_iteration with the propagator dressed by the state's Sigma (Sigma^R and
 * Sigma^K on `grid`, Delta and T of the bath, eps = 0).  Per iteration k: g = F(x_k),
 * f = g - x_k, residual r_k = max over arrays of max|f| / max|g|; then
 *   x_{k+1} = x_k + alpha f - sum_i gamma_i (dG_i - (1 - alpha) dF_i)
 * with the Anderson columns dF_i, dG_i (differences of f and g between consecutive
 * iterations, the last m of them) and gamma solving the normal equations
 * (dF^T dF + eps I) gamma = dF^T f over the real inner product Re <a, b> of the state
 * vectors, eps = 1e-14 max_i (dF^T dF)_ii (Walker and Ni 2011); no columns: linear mixing.
 * With hartree = 1 (asymmetric model) the level of G is eps_d + Sigma_H: the PT2 start uses
 * the self-consistent Sigma_H of the bare level (kqft_hartree), the state carries Sigma_H as
 * one more entry, and F updates it once per iteration by the one-shot Hartree term of the
 * state's propagator (its Sigma and Sigma_H); its relative change enters the residual.
 * gamma[3] (device, out): the channels of the final state; sigma (device [n][4], out);
 * sigma_H (host, out, or NULL): the final Hartree term (U/2 with hartree = 0); residuals
 * (host [max_iterations] or NULL); iterations (host, out).  Synchronises `stream` once per
 * iteration.  Working memory: (3 + 2m) states besides F(x).
 */
int kqft_parquet_solve(kqft_ctx* ctx, const kqft_grid* grid, double U, double Delta, double T,
                       const kqft_quad* q_bubble, const kqft_quad* q_loop, const kqft_opts* opts,
                       const kqft_parquet_opts* popts, const kqft_chout* gamma, double* sigma, double* sigma_H,
                       double* residuals, int* iterations, void* stream);

/*
 * kqft_parquet_solve_matsubara -- the parquet solver (kqft_parquet_solve: PT2 start, mixing or
 * Anderson acceleration, automatic reduction of alpha, residual = max over the arrays of
 * max|F(x) - x| / max|F(x)|) in the Matsubara formalism: F is the symmetrized Bethe-Salpeter
 * equations with kqft_bubble_matsubara (window Nq) and the SDE of kqft_sde_matsubara (loop
 * window Nl), G dressed by the state's Sigma on [-N, N).  popts: alpha, max_iterations, tol,
 * anderson_depth, reduce_alpha, alpha_min; hartree must be 0 and sde_forms 0 or 1
 * (KQFT_EINVAL otherwise).  gamma[3] (device, out; classes on grid), sigma (device [2N], out),
 * residuals (host [max_iterations] or NULL), iterations (host, out).  FP64.  Synchronises
 * `stream` once per iteration.  Working memory: (5 + 2m) states and one channel.
 */
int kqft_parquet_solve_matsubara(kqft_ctx* ctx, const kqft_mgrid* grid, double U, double Delta, int Nq, int Nl,
                                 const kqft_parquet_opts* popts, const kqft_chout* gamma, double* sigma,
                                 double* residuals, int* iterations, void* stream);

/*
 * kqft_mloop_step -- multiloop insertions of the mfRG flow (Eqs. 1l, 2l, 3l) for
 * n_points independent parameter points (ragged sizes allowed):
 *   l = 1:  gdot_r = B_r(Gamma, Gamma; Pidot),
 *   l = 2:  gdot_r = B_r(gdot_rbar, Gamma) + B_r(Gamma, gdot_rbar),
 *   l >= 3: gdot_r = L + R + B_r(Gamma, gdot_{r,L}^(l-1)),
 * with gdot_rbar the sum of the two channels other than r at the previous order and
 * the centre term reusing the stored left insertion of order l-1 (which equals
 * B_r(gdot_rbar^(l-2), Gamma)); R and the centre term are evaluated as one bubble of the
 * combined right vertex gdot_rbar^(l-1) + gdot_{r,L}^(l-1) (the bubble is linear in it).  Delta-flow single-scale propagator, no Katanin term.
 * gamma, G, q: host arrays of n_points structs.  dgamma: host array of
 * n_points * nloops * 3 kqft_chout (point-major, then order, then channel) whose
 * device arrays (all four classes required) receive each order's sum of insertions.
 */
int kqft_mloop_step(kqft_ctx* ctx, int n_points, const kqft_vertex* gamma, const kqft_propagator* G,
                    const kqft_quad* q, int nloops, const kqft_opts* opts, const kqft_chout* dgamma,
                    void* stream);

/*
 * kqft_bubble_adjoint -- vector-Jacobian product of kqft_bubble (not in the paper).
 * Given the cotangent `dout` of the four output classes (PyTorch convention: for a real
 * loss L and complex z, dz = dL/dRe z + i dL/dIm z), accumulates
 *   dleft[r]  += dL/d(class arrays of left's channel r)   (r = 0..2, NULL entries skipped),
 *   dright[r] += dL/d(class arrays of right's channel r),
 *   dscal[0] += dL/d left->r0,  dscal[1] += dL/d right->r0,  dscal[2] += dL/d G->Delta,
 * where class-array cotangents already include the channel coefficient.  The A/B panels
 * are recomputed (checkpointing) rather than stored.  Dynamic self-energies inside G
 * are held fixed.  dleft, dright: host arrays of 3 kqft_chout with device pointers;
 * dscal: device array of 3 doubles.  The transposed products conj(dA) = conj(dP) B^T and
 * conj(dB) = conj(dP)^T A per transfer frequency run on the library's own MFMA GEMM, in FP64,
 * or with opts->precision = KQFT_SPLIT_FP32 on FP32 MFMA (operands rounded to FP32, partial
 * sums of 64 terms promoted to FP64); everything else in FP64.  The scatter into class arrays
 * uses FP64 atomics (summation order not deterministic).
 */
int kqft_bubble_adjoint(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                        const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                        const kqft_chout* dout, const kqft_chout* dleft, const kqft_chout* dright,
                        double* dscal, void* stream);

/*
 * kqft_sde_adjoint -- vector-Jacobian product of the self-energy of kqft_sde (not in the
 * paper).  Given dsigma (device [n][4] complex, cotangent of sigma), accumulates
 *   dgamma[r] += dL/d(class arrays of gamma's channel r),
 *   dscal[0] += dL/d gamma->r0 (through both Gamma_0 of the Schwinger-Dyson bubble and gamma),
 *   dscal[1] += dL/d G->Delta.
 * Phi is recomputed.  dgamma: host array of 3 kqft_chout; dscal: device array of 2 doubles.
 */
int kqft_sde_adjoint(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q_bubble,
                     const kqft_quad* q_loop, const kqft_opts* opts, const double* dsigma, const kqft_chout* dgamma,
                     double* dscal, void* stream);

/*
 * kqft_mloop_adjoint -- vector-Jacobian product of kqft_mloop_step for one parameter point
 * (not in the paper; the forward map is the multiloop recursion of Eqs. 1l, 2l, 3l with the
 * Delta-flow single-scale propagator, no Katanin term).  Given the cotangents dgdot[l][r]
 * (host array of nloops * 3 kqft_chout, order-major; a NULL class counts as zero) of the
 * insertions gdot_r^(l) that kqft_mloop_step returns, accumulates
 *   dgamma[r] += dL/d(class arrays of gamma's channel r)   (host array of 3; NULL classes skipped),
 *   dscal[0]  += dL/d gamma->r0,   dscal[1] += dL/d G->Delta   (device array of 2 doubles),
 * PyTorch's convention for complex cotangents.  The insertions are not stored: going down
 * from l = nloops, orders 1..l-1 are recomputed (checkpointing) into two alternating
 * order buffers, and every bubble of order l is reversed with kqft_bubble_adjoint's kernels --
 * the left insertion B_r(gdot_rbar^(l-1), Gamma) with the cotangent of its order plus the one
 * the centre term of order l+1 passes back, the right insertion B_r(Gamma, gdot_rbar^(l-1)),
 * and the centre term B_r(Gamma, gdot_{r,L}^(l-1)); the cotangents of gdot_rbar^(l-1) are
 * accumulated into the order below.  Recomputes sum_{l < nloops} l orders of insertions.
 * Working memory: 6 channel buffers of cotangents, 6 of recomputed insertions (each
 * 2(n + 2n^2 + n^3) x 16 complex), plus the bubble adjoint's workspace.  Recomputed
 * insertions and transposed products in opts->precision, the rest in FP64; same propagator
 * restrictions and atomics as kqft_bubble_adjoint.
 */
int kqft_mloop_adjoint(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
                       int nloops, const kqft_opts* opts, const kqft_chout* dgdot, const kqft_chout* dgamma,
                       double* dscal, void* stream);

/*
 * kqft_mloop_jvp -- Jacobian-vector product of kqft_mloop_step for one parameter point along
 * a tangent of the vertex at a fixed propagator (not in the paper).  The insertions are
 * multilinear in Gamma (Eqs. 1l, 2l, 3l: every bubble is bilinear), so the tangent of each
 * bubble B(L, R) is B(dL, R) + B(L, dR) and the recursion carries the tangents of the
 * lower orders and of the stored left insertions along.  tangent: a vertex on gamma's grid
 * holding d r0 and the class tangents (channel coefficients as in gamma).  out, dout: host
 * arrays of nloops * 3 kqft_chout (order-major, all four classes given) receiving the
 * insertions (as kqft_mloop_step) and their tangents.  Bubbles in opts->precision.
 */
int kqft_mloop_jvp(kqft_ctx* ctx, const kqft_vertex* gamma, const kqft_vertex* tangent, const kqft_propagator* G,
                   const kqft_quad* q, int nloops, const kqft_opts* opts, const kqft_chout* out,
                   const kqft_chout* dout, void* stream);

/*
 * kqft_bubble_tune -- autotuner of the bubble's schedule (not in the paper): times kqft_bubble
 * with the given arguments for transfer-frequency batches of the whole grid divided into 1, 2,
 * 3, 4, 6, 8, 12 or 16 parts, down to about 8 frequencies (those whose workspace, kqft_bubble_workspace, stays
 * within max_workspace bytes; 0 = no limit), one warm-up and one timed call each, and keeps the
 * fastest in the context for (n, q->n, opts->precision): from then on every bubble of that
 * shape with opts->omega_batch = 0 -- kqft_bubble, kqft_mloop_step, the solvers and the flows --
 * uses it.  Returns it in *omega_batch and its time in *ms (may be NULL).  `out` is
 * overwritten (scratch while tuning; beta is ignored).  Synchronises `stream`; not to be
 * captured.
 */
int kqft_bubble_tune(kqft_ctx* ctx, int channel, const kqft_vertex* left, const kqft_vertex* right,
                     const kqft_propagator* G, int pi_kind, const kqft_quad* q, const kqft_opts* opts,
                     const kqft_chout* out, size_t max_workspace, int* omega_batch, double* ms, void* stream);

/*
 * kqft_chi_noalloc -- kqft_chi for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * susceptibility chi_r (same kernels, same arguments and layout of chi, no context), with
 * every buffer the kernels need beyond gamma, G and chi -- grid nodes, quadrature nodes and
 * weights (computed on the device), the other channels' target-order tables, Pi and the block
 * partials -- carved out of one static device array of 64 MiB (kept per device until the
 * process ends; the first call on a device looks its address up).  It calls no hipMalloc,
 * hipFree or allocating library routine.  The transfer frequencies run in batches sized to
 * what the array leaves; a vertex whose tables and one transfer frequency do not fit
 * (about n^3 + 2 n^2 + n <= 65000 with both other channels active, e.g. n <= 39) returns
 * KQFT_ENOMEM with the sizes in kqft_last_error().  Every call on a device shares that
 * device's array and leaves its contents behind; nothing in it needs to start at zero.
 * Calls that overlap on one device (two streams, or two host threads) race on the array:
 * order them on one stream.  Launches on `stream` only; no host synchronisation.
 */
int kqft_chi_noalloc(int channel, const kqft_vertex* gamma, const kqft_propagator* G, const kqft_quad* q,
                     double* chi, void* stream);

/* Device bytes held by the library's workspaces (every context of the process): current
   and peak since the library was loaded or the last kqft_workspace_reset_peak.  Either
   pointer may be NULL, not both. */
int kqft_workspace_bytes(size_t* current, size_t* peak);

/* Restart the peak of kqft_workspace_bytes at the current bytes (to measure one workload's
   peak in a process that ran others before).  Always returns KQFT_OK. */
int kqft_workspace_reset_peak(void);

#ifdef __cplusplus
}
#endif
#endif /* KQFT_H */
