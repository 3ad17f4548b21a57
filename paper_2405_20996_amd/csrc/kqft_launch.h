// kqft_launch.h -- kernel argument blocks and launchers (host <-> kernel contract).
#pragma once
#include "kqft_internal.h"

namespace kqft {

struct PiArgs {
  int r, kind, nb, nq, iw0;
  DProp P;
  const double* wnodes;  // transfer-frequency grid nodes
  const double* qv;
  const double* qw;
  double2* out;  // [nb][nq][16], Pi * w_k / (2 pi i)
};

struct GatherArgs {
  int r, nb, iw0, nq, nq_pad, lo, cnt;  // rows/cols lo .. lo+cnt-1 (index n = border)
  long Kp;                              // panel leading dimension (complex)
  DGrid g;
  double r0;
  double coef;          // own channel coefficient
  const double2* K[4];  // own channel K1, K2, K2', K3 (FP64, channel order; nullptr = absent)
  const void* T[2];     // tables of channels r + 1, r + 2 (nullptr = inactive)
  double mix[4];        // spin combination: c0 = mix0 X + mix1 Y, c1 = mix2 X + mix3 Y
  const double* nodes;  // vertex grid nodes
  const double* qv;
  const double2* pi;  // left gather: Pi * w / (2 pi i); nullptr = raw left factor
  void* P0;           // panel of spin combination 0 ([nb][4(n+1)][Kp])
  void* P1;           // combination 1
};

// target-order class tables of channel r2 for a bubble in channel r
struct TableArgs {
  int n, r, r2;
  double coef;
  double mix[4];
  const double2* K[4];  // K1, K2, K2', K3 of channel r2 (nullptr = absent)
  void* out;            // F3 [n^3] | F2v [n^2] | F2p [n^2] | F1 [n] records of 32 values
};

// C[b] = op(A[b]) . B[b], complex FP64, row-major (see zgemm_nn_kernel)
struct ZgemmArgs {
  const double2* A;
  const double2* B;
  double2* C;
  long lda, ldb, ldc;
  long strideA, strideB, strideC;
  int M, N, K, batch;
  int TA;                // op(A) = A^T when 1
  int tiles_m, tiles_n;  // set by the launcher
};
void launch_zgemm_nn(ZgemmArgs g, hipStream_t s);
void launch_zgemm_nn_f32(ZgemmArgs g, hipStream_t s);

struct GemmArgs {
  const void* A[2];
  const void* B[2];
  long strideA, strideB;  // complex elements per transfer frequency
  int M, Kp;              // M = 4(n+1) rows and columns; Kp padded contraction length
  int tm0, tms, tn0, tns; // tile ranges
  int nb;
  int r, n, iw0, beta, cmask;
  double unmix[4];  // X = u0 P0 + u1 P1, Y = u2 P0 + u3 P1 (channel prefactor included)
  double2* K1;
  double2* K2;
  double2* K2p;
  double2* K3;
  double2* P[2];  // split path: per-combination products [nb][M][M] (workspace)
};

struct LoopArgs {
  DGrid g;
  DProp P;
  int kind, nq;
  const double* nodes;
  const double* qv;
  const double* qw;
  const double2* K1;
  const double2* K2p;
  double2* out;  // [n][4]
};

// loop of a full vertex: all three channels through tables in the a-channel order with the
// spin combination 2X + Y in slot c = 0
struct VLoopArgs {
  DGrid g;
  DProp P;
  int kind, nq;
  double r0;
  const void* T[3];  // FP64 tables of channels a, p, t (nullptr = inactive)
  const double* nodes;
  const double* qv;
  const double* qw;
  double2* out;  // [n][4]
};

struct ChiArgs {
  int r;  // channel of the susceptibility
  int nq, nb, iw0;
  DGrid g;
  double r0;
  double coef;          // channel r coefficient
  const double2* K[4];  // channel r K1, K2, K2', K3 (nullptr = absent)
  const void* T[2];     // FP64 target-order tables of channels r + 1 and r + 2 (nullptr = inactive)
  double mix[4];        // channel r's spin combinations
  const double* nodes;
  const double* qv;
  const double2* pi;  // [nb][nq][16], channel r, Pi = G G, weights folded
  double2* partial;   // [nb][nblk][32]
  double2* out;       // [2][n][16]
  int f32;            // tables in FP32 (float2 records) instead of FP64
  // own channel and bare vertex through the grid projection (chi_proj / chi_own kernels):
  // pt[b][i][16] = sum_k c_ki Pi_k (i < n; c_ki the interpolation weight of node i at v''_k),
  // pt[b][n][16] = sum_k Pi_k; own[b][c][16] their contribution to chi (nullptr: own channel
  // and bare vertex evaluated in the pair loop instead)
  double2* pt;
  double2* own;
};
// largest grid whose projection fits the own-channel kernel's LDS
constexpr int kChiProjMaxN = 300;


// ------------------------------------------------------------------ adjoint
// cotangent panel D'_c[(i,row),(j,col)] = conj(dP_c), dP_c from the class cotangents
struct DPanelArgs {
  int n, nb, iw0;
  double unmix[4];
  const double2* dK1;
  const double2* dK2;
  const double2* dK2p;
  const double2* dK3;
  double2* D0;
  double2* D1;
};
// A = L . Pi from a raw left panel
struct ApplyPiArgs {
  int n, nb, nq, nq_pad;
  long Kp;
  const double2* pi;
  const double2* L0;
  const double2* L1;
  double2* A0;
  double2* A1;
};
struct AdjScatterArgs {
  int r, nb, iw0, nq;
  long Kp;
  DVert V;
  const double* nodes;
  const double* qv;
  const double2* pi;      // left side only: Pi * w/(2 pi i)
  const double2* G0;      // conj(dA_c) (left) or conj(dB_c) (right) panels
  const double2* G1;
  double mix[4];
  double2* dK[3][4];      // class cotangent targets of this side (NULL = not requested)
  double2* dKf[3];        // fused cotangent tables of the other channels (NULL = per class)
  double* dr0;            // cotangent of this side's r0
};
struct DPiArgs {
  int r, kind, nb, nq, iw0, n;
  long Kp;
  DProp P;
  const double* wnodes;
  const double* qv;
  const double* qw;
  const double2* L0;  // raw left panels
  const double2* L1;
  const double2* G0;  // conj(dA_c) panels
  const double2* G1;
  double* dDelta;
};
struct UnfuseArgs {
  int n;
  const double2* dKf;
  double2* dK1;
  double2* dK2;
  double2* dK2p;
  double2* dK3;
};
// loop adjoint: dSigma -> cotangents of Phi's K1/K2' (atomics) and dDelta
struct LoopAdjArgs {
  DGrid g;
  DProp P;
  int nq;
  const double* nodes;
  const double* qv;
  const double* qw;
  const double2* K1;   // Phi
  const double2* K2p;
  const double2* dsig; // [n][4]
  double2* dK1;
  double2* dK2p;
  double* dDelta;
};
void launch_loop_adjoint(const LoopAdjArgs& a, hipStream_t s);
void launch_dpanel(const DPanelArgs& a, hipStream_t s);
void launch_apply_pi(const ApplyPiArgs& a, hipStream_t s);
void launch_adj_left(const AdjScatterArgs& a, hipStream_t s);
void launch_adj_right(const AdjScatterArgs& a, hipStream_t s);
void launch_dpi(const DPiArgs& a, hipStream_t s);
void launch_unfuse(const UnfuseArgs& a, hipStream_t s);

hipError_t upload_perm(const int* host_perm);
void launch_table(const TableArgs& a, bool f32, hipStream_t s);
void launch_pi(const PiArgs& a, hipStream_t s);
void launch_gather(const GatherArgs& a, bool left, bool f32, hipStream_t s);
void launch_gemm(const GemmArgs& g, int precision, hipStream_t s);
// split path: the two combinations' products into the classes (after launch_gemm, same stream)
void launch_unmix(const GemmArgs& g, hipStream_t s);
// only the border row block (rows 4n .. 4n+3) of C = A B, both precisions, through the epilogue
void launch_rowpanel(const GemmArgs& g, int precision, hipStream_t s);
void launch_loop(const LoopArgs& a, hipStream_t s);
void launch_vloop(const VLoopArgs& a, hipStream_t s);
void launch_chi(const ChiArgs& a, hipStream_t s);  // projection + own part (when a.own) + pair loop + finalize
int chi_blocks(int nq);
void launch_grid_nodes(int n, int map, double a, double theta, double* v, hipStream_t s);
void launch_quad_nodes(int nq, double a, double th, double* qv, double* qw, hipStream_t s);
void launch_sigma_split(int n, const double2* sigma, double2* sigR, double2* sigK, hipStream_t s);
void launch_maxdiff(const double2* x, const double2* f, size_t count, double* partial, int nblk, hipStream_t s);
void launch_mix(double2* x, const double2* f, size_t count, double alpha, hipStream_t s);
// out = x + sum_{j < nt} c_j k_j over count complex entries (x may be null, nt <= 6)
struct LinComb {
  double2* out;
  const double2* x;
  const double2* k[6];
  double c[6];
  int nt;
  size_t count;
};
void launch_lincomb(const LinComb& a, hipStream_t s);
// out[s][i1..id][c] = the multilinear interpolation (on src's auxiliary variable) of
// in[s][..][c] at the destination nodes (dims 1..3 frequency axes, nspin leading blocks,
// ncomp complex components innermost); zero where any argument lies outside src's extent
struct RegridArgs {
  DGrid src;
  const double* dst;  // destination nodes [nd]
  int nd, dims, nspin, ncomp;
  const double2* in;
  double2* out;
};
void launch_regrid(const RegridArgs& a, hipStream_t s);
// adaptive bubble: one work item = one output and one interval of the auxiliary variable
struct AdaptItem {
  double ya, yb;
  int o, depth;
};
struct AdaptArgs {
  GatherArgs L, R;  // left / right factors (FP64 tables; panel fields unused)
  DProp P;
  int r, kind, n;
  int phase;                 // 0: error scale from the rule's nodes and weights a; 1: a (GL4) vs b (GLK7)
  int nn;                    // nodes of the rule
  const double* rule;        // device: nodes [13], weights a [13], weights b [13]
  int cstart[4], ccount[4];  // output ranges of K1, K2, K2', K3 (count 0: not computed)
  double unmix[4];           // combinations -> X, Y with the channel prefactor
  double qa, qth;            // v'' = qa tan(y qth), y in [-1, 1]
  double eps, min_width;
  int max_depth;
  const AdaptItem* in;
  int nin;
  AdaptItem* out;  // next work list
  int* nout;
  int cap;
  int* overflow;
  double* scale;     // per output
  double2* K[4];     // outputs, accumulated
};
void launch_adaptive(const AdaptArgs& a, hipStream_t s);
// per-block partial sums of w_j tanh(v_j/2T) Im G^R(v_j) (P.eps is the level)
void launch_occupation(const DProp& P, const double* nodes, const double* weights, int nq, double* partial, int nblk,
                       hipStream_t s);
// per-block partial sums of Re <a, b> over count complex entries (nblk blocks)
void launch_dot(const double2* a, const double2* b, size_t count, double* partial, int nblk, hipStream_t s);
void launch_errnorm(const double2* err, const double2* y, const double2* y4, double atol, double rtol, size_t count,
                    double* partial, int nblk, hipStream_t s);
void launch_axpby(double2* out, double a, const double2* x, double b, const double2* y, size_t count,
                  hipStream_t s);

// ------------------------------------------------------------------ Matsubara formalism
// One channel on the Matsubara boxes: K1[s][m], K2[s][m][n], K2'[s][m][n'], K3[s][m][n][n'],
// m in [-M, M], n, n' in [-N, N) (nullptr = absent).
struct MChan {
  double coef;
  const double2* K[4];
};
// Panels of one side of a Matsubara bubble for the bosonic indices m = m0 + b, b < nb:
// left A_c[b][i][k] (i < 2N: (L - L^inf)(m, n_i, n''_k) T Pi(m, n''_k); i = 2N: L^inf T Pi),
// right B_c[b][k][j] (j < 2N: (R - R^inf)(m, n''_k, n'_j); j = 2N: R^inf), k < 2 Nq over the
// window of channel r's bubble (zero past its end), c = 0, 1 the spin combinations of P[c].
struct MGatherArgs {
  int r, M, N, Nq, m0, nb;
  int kind;  // 0: Pi = G G; 1: Pi_dot = S G + G S (S = dG/dDelta + G Sigma_dot G)
  double T, Delta;
  const double2* sigma;   // G's self-energy on n in [-Ns, Ns), or null
  const double2* dsigma;  // Sigma_dot on the same box (Katanin), or null
  int Ns;
  double U;  // bare vertex X0 = -U, Y0 = +U
  int reg;     // 0: G_0^-1 = i nu + i Delta sgn nu; 1: G_0 -> lam G_0 (interaction flow)
  double lam;
  MChan ch[3];
  double mix[4];
  double2* P[2];
};
// C_c[b][i][j] (i, j <= 2N) -> classes of channel r at m = m0 + b (unmix with the prefactor)
struct MEpiArgs {
  int M, N, m0, nb;
  double unmix[4];
  const double2* C[2];
  double2* K[4];
};
// Sigma(n) = -1/2 T sum_{n'} [2 Phi^X + Phi^Y](m = n - n', n', n') G(n') for n in [-N, N), n' in
// [-Nl, Nl), Phi = K1 + K2' of an a-channel object on the boxes
struct MLoopArgs {
  int M, N, Nl;
  double T, Delta;
  int reg;  // as MGatherArgs
  double lam;
  const double2* sigma;  // G's self-energy on [-Ns, Ns), or null
  int Ns;
  const double2* K1;
  const double2* K2p;
  double2* out;
};
void launch_mf_loop(const MLoopArgs& a, hipStream_t s);
// L(Gamma, X)(n) = T sum_{n'} [2X + Y](legs n, n' | n, n') X(n') for n in [-N, N), n' in
// [-Nl, Nl), the full vertex of v (bare part, all channels and classes), X = G, S or G
// Sigma_dot G (line 0, 1, 2); v.r = 0
void launch_mf_vloop(const MGatherArgs& v, int line, int Nl, double2* out, hipStream_t s);
// analytic tails of a Matsubara bubble: adds, per m, the bubble of the large-frequency vertices
// (left Gamma_0 + K1 + K2(m, n), right Gamma_0 + K1 + K2'(m, n') of channel r) with the scalar
// t(m) (the bare sum beyond the window) to the four classes; v0 / v1 carry the two sides
struct MTailArgs {
  int M, N;
  const double2* t;  // [2M + 1]
  double mix[4], unmix[4];
  double UL, UR;
  MChan L, R;  // channel r of each side
  double2* K[4];
};
void launch_mf_tail(const MTailArgs& a, hipStream_t s);
// chi_r^c(m) = T sum_k Pi(m, k) + T^2 sum_{k,l} Pi(m, k) Gamma_r^c(m; k, l) Pi(m, l) over channel
// r's window for every m in [-M, M]: one workgroup per m, fixed reduction order; out [2][2M+1]
void launch_mf_chi(const MGatherArgs& v, double2* out, hipStream_t s);
void launch_mf_left(const MGatherArgs& a, hipStream_t s);
void launch_mf_right(const MGatherArgs& a, hipStream_t s);
void launch_mf_epilogue(const MEpiArgs& a, hipStream_t s);

}  // namespace kqft
