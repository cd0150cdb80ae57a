// Launch interface of the gfx950 kernels (host-callable, HIP types only).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qmc {

// Optional per-launch timing (qmc_profile_enable): a launch site opens a
// ProfScope naming the kernel; events are recorded on the launch stream.
bool prof_on();
void prof_push(const char* name, hipEvent_t a, hipEvent_t b);
struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  const char* name;
  hipStream_t st;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    if (prof_on() && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
      if (hipEventRecord(a, st) != hipSuccess) a = nullptr;
    } else {
      a = nullptr;
    }
  }
  ~ProfScope() {
    if (a && hipEventRecord(b, st) == hipSuccess) prof_push(name, a, b);
  }
};

// Compute kinds of the GEMM: operands and accumulation.
enum GemmKind { GK_F64 = 0, GK_F32 = 1, GK_BF16 = 2 };

// Y = act(X W + bias) (+ Res), over jet rows grouped per electron (or per pair).
//   Row r of X lives at X + (r / xrpw) * xws + (r % xrpw) * ldx (same for Y/Res
//   with yrpw/yws/ldy).  W(k, n) = W[k * ldw + n], or W[n * ldw + k] when transw.
//   Jet rows (vmode = 0): groups of Rp rows: row 0 value, rows 1..T tangents,
//   row T+1 Laplacian, the rest zero padding.  vmode = 1: every row a value row.
//   act: 0 linear, 1 tanh (propagated through the jet).
struct GemmArgs {
  const void* X;
  int64_t ldx, xrpw, xws;
  const void* W;
  int64_t ldw;
  const void* bias;
  const void* Res;
  void* Y;
  int64_t ldy, yrpw, yws;
  int64_t rows;
  int K, Ncols;
  int Rp, T, act, vmode;
  int transw;
  const void* aux;  // act == 2: out = acc * (1 - aux^2), aux addressed like Y (tanh backward)
  // electron jets: rows [W][N][Rp] also receive add5 [W][N][5][Ncols] before the activation, at
  // the value row, the 3 rows of the electron's own coordinates and the Laplacian row (N = nel)
  const void* add5;
  int nel;
  // tile choice: 0 = default, else 1 + bits (bit 0: 32-wide K stages for float32, bit 1: half-height
  // value and edge tiles, bit 2: persistent grid, bit 3: float32 on the bf16 matrix cores with
  // three-piece operands)
  int tile;
};

hipError_t launch_gemm(GemmKind kind, const GemmArgs& a, hipStream_t st);

// Geometry of a walker chunk: dense pair distances and unit vectors (float64).
//   r: [W][N][3]; ee: [W][N][N][4] (d, ux, uy, uz of r_i - r_j); en: [W][N][M][4];
//   vpot[W] = potential energy (+ vnn).
struct SysDev {
  int N, M, nup, ndn, T, Rp, K, D, ndet, nenv, P0, P1, P2;
  double dmax, vnn;
  double ee_cusp;  // alpha of the electron-electron cusp factor (0: none)
  int full_det;    // one N x N determinant per p instead of one per spin
  double Z[64];
  double R[64 * 3];
};

// Determinant matrices of spin s's stage (order; 0 when the stage has none), orbitals per
// determinant of spin s's orbital map, and the first matrix row of spin s's electrons.  With the
// full determinant, stage 0 holds the N x N matrices of both spins and stage 1 is empty.
__host__ __device__ inline int det_dim(const SysDev& s, int sp) {
  return s.full_det ? (sp ? 0 : s.N) : (sp ? s.ndn : s.nup);
}
__host__ __device__ inline int orb_count(const SysDev& s, int sp) { return s.full_det ? s.N : (sp ? s.ndn : s.nup); }
__host__ __device__ inline int det_row0(const SysDev& s, int sp) { return s.full_det && sp ? s.nup : 0; }

// Compute units of the current device (queried once per device, thread-safe; 256 if the query fails).
int device_cus();

// Fused edge filters w(d) = tanh(rho(d) U1 + a1) U2 + a2 on MFMA (float32, width 128 or 256, at most 16
// basis functions) for every pair of one edge type, from the geometry to the filter rows.
struct EdgeMlpArgs {
  const float *U1, *a1, *U2, *a2;
  const double *ee, *en;  // geometry of the walker chunk (layouts as launch_geometry writes them)
  float* out;             // [pairs][D] value rows, or [pairs][4][D] univariate jets (rows 0-2 written)
  float* zout;            // optional, value rows only: the hidden layer tanh(rho U1 + a1), [pairs][D]
  int64_t pairs;          // walkers x pairs of this type
  int type;               // 0 same-spin, 1 up-down, 2 electron-nucleus
  int jet;
  const float* feat;      // optional edge features in place of the radial basis of the distance:
                          // [pairs][K] values, or [pairs][4][K] univariate jets (rows 0-2 read)
};
bool edge_mlp_supported(const SysDev& s);
hipError_t launch_edge_mlp(const SysDev& s, const EdgeMlpArgs& a, hipStream_t st);
// the filters of n (1..3) edge types in one launch (all value rows or all jets), the blocks split
// among the types in proportion to their tiles
hipError_t launch_edge_mlp_types(const SysDev& s, const EdgeMlpArgs* a, int n, hipStream_t st);

hipError_t launch_geometry(const SysDev& s, const double* r, int64_t W, double* ee, double* en,
                           double* vpot, hipStream_t st);

template <typename S>
hipError_t launch_rbf(const SysDev& s, int type, const double* ee, const double* en, int64_t W, int jet,
                      S* rho, hipStream_t st);

template <typename S>
hipError_t launch_init_features(const SysDev& s, const double* ee, const double* en, int64_t W, int jet,
                                S* x0, hipStream_t st);

template <typename S>
hipError_t launch_aggregate(const SysDev& s, const S* h, const S* wsame, const S* wopp, const S* wnuc,
                            const S* Y, const double* ee, const double* en, int64_t W, int jet, S* m,
                            hipStream_t st);

// Jet mode writes [W][N][Rp][2D] (same-spin, opposite-spin messages); value mode writes [W][N][3D]
// including the nuclear message.  launch_nuc_message: nuclear messages with jets, [W][N][5][D].
template <typename S>
hipError_t launch_nuc_message(const SysDev& s, const S* wnuc, const S* Y, const double* en, int64_t W, S* out,
                              hipStream_t st);

template <typename S>
hipError_t launch_envelope(const SysDev& s, int spin, const S* phi, const S* pi, const S* sigma,
                           const double* en, int64_t W, int jet, S* ajet, hipStream_t st);

// Determinants of A-jets: one problem per (walker, spin, det).
//   ajet: per walker [spin][det][rows][n][n] (rows = T + 2 padded to Rp, or 1).
//   ainv (optional): A^-1 per spin block, [spin][W][det][n][n] (spin 1 after all of spin 0).
template <typename S>
hipError_t launch_det(const SysDev& s, const S* ajet, int64_t W, int jet, double* ld, double* sg,
                      double* g, double* lap, double* ainv, hipStream_t st);

// Generic batched determinant jets (float64), one n x n problem per matrix.
// Achievable peaks (float32, bf16 and float64 MFMA TFLOP/s; copy GB/s read + written) measured on the
// device with the caller's scratch buffer; synchronises the stream.
hipError_t measure_peaks(void* scratch, size_t bytes, double* out, hipStream_t st);
hipError_t launch_det_generic(int64_t nmat, int n, int ntan, const double* jets, double* ld,
                              double* sg, double* g, double* lap, hipStream_t st);

template <typename S>
hipError_t launch_combine(const SysDev& s, const S* c, const double* ld, const double* sg,
                          const double* g, const double* dlap, const double* vpot, const double* ee, const S* jas,
                          int64_t W, int jet, double* logpsi, double* sign, double* grad, double* lap, double* eloc,
                          hipStream_t st);
// Learnable Jastrow factor: out[w][q][d] = sum_i f[w][i][q][d] (R rows per electron); the scalar
// output layer out[row] = x[row] . W2 (+ b2 on value rows, every R-th row); in the backward
// go[w] = gbar[w], zb[w][d] = gbar[w] W2[d] (1 - h[w][d]^2); and fbar[w][i][d] += fs[w][d].
template <typename S>
hipError_t launch_sum_electrons(int64_t W, int N, int R, int D, const S* f, S* out, hipStream_t st);
template <typename S>
hipError_t launch_jastrow_out(int64_t rows, int R, int D, const S* x, const S* W2, const S* b2, S* out,
                              hipStream_t st);
template <typename S>
hipError_t launch_jastrow_bwd(int64_t W, int D, const double* gbar, const S* W2, const S* h, S* zb, S* go,
                              hipStream_t st);
template <typename S>
hipError_t launch_add_bcast(int64_t W, int N, int D, const S* fs, S* fbar, hipStream_t st);

hipError_t launch_propose(const double* r, const double* noise, double step, int64_t n, double* rp,
                          hipStream_t st);
hipError_t launch_accept(int64_t W, int N3, const double* rp, const double* lp_prop, const double* u,
                         double* r, double* logpsi, uint8_t* accepted, hipStream_t st);
// Clipped local energies of one system's n walkers (median-centred window of half-width
// width x mean absolute deviation; mode 0 hard, 1 logarithmic soft); out may equal e.
hipError_t launch_clip(const double* e, double* out, int64_t n, double width, int mode, hipStream_t st);
// Langevin step: drift proposal (one thread per electron) and Hastings acceptance (one per walker);
// rp, gp [W][N][3] and lpp [W] are the proposal, its gradient and its log|psi|.
hipError_t launch_propose_mala(const SysDev& s, const double* r, const double* g, const double* noise, double step,
                               int damp, int64_t W, double* rp, hipStream_t st);
hipError_t launch_accept_mala(const SysDev& s, int64_t W, const double* rp, const double* gp, const double* lpp,
                              const double* noise, const double* u, double step, int damp, double* r, double* g,
                              double* logpsi, uint8_t* accepted, hipStream_t st);

// ---------------------------------------------------------------- backward

// part[split][m][n] = sum_{rows r of the split} X[r][m] G[r][n] (m = Kin: ones, bias)
// then gW[m][n] += sum_split (m < Kin), gb[n] += bias row.  Rows addressed like GemmArgs.
struct WgradArgs {
  const void* X;
  int64_t ldx, xrpw, xws;
  const void* G;
  int64_t ldg, grpw, gws;
  int64_t rows;
  int Kin, Nout, ones;
  double* part;           // partial sums, [split][Kin + ones][Nout]
  int64_t part_elems;     // capacity of part (elements); the launcher picks the splits within it
  int64_t rows_per_split;  // set by launch_wgrad
};
hipError_t launch_wgrad(GemmKind kind, const WgradArgs& a, double* gW, int64_t ldgw, double* gb, hipStream_t st);

template <typename S>
hipError_t launch_tanh_bwd(int64_t n, const S* ybar, const S* t, S* z, hipStream_t st);
template <typename S>
hipError_t launch_add(int64_t n, const S* a, const S* b, S* o, hipStream_t st);
hipError_t launch_fill(int64_t n, double v, double* p, hipStream_t st);
// Position gradient by the reverse pass: distance cotangents of the edge filters (rhobar [pairs][K]),
// of the initial features (x0bar [N][(M+2)K] per walker) and of the envelopes, accumulated into
// dee [W][N][N] (i < j) and den [W][N][M]; then rbar [W][N][3] (with the cusp factor's gradient).
template <typename S>
hipError_t launch_pair_dbar(const SysDev& s, int type, const S* rhobar, const double* ee, const double* en, int64_t W,
                            double* dee, double* den, hipStream_t st);
template <typename S>
hipError_t launch_init_dbar(const SysDev& s, const S* x0bar, const double* ee, const double* en, int64_t W,
                            double* dee, double* den, hipStream_t st);
template <typename S>
hipError_t launch_env_dbar(const SysDev& s, int spin, const double* lbar, const double* ainv, const S* phi,
                           const S* pi, const S* sg, const double* en, int64_t W, double* den, hipStream_t st);
hipError_t launch_positions_bar(const SysDev& s, const double* ee, const double* en, const double* dee,
                                const double* den, const double* lp, int64_t W, double* out, hipStream_t st);
template <typename S>
hipError_t launch_sgd(int64_t n, double lr, const S* grad, S* params, hipStream_t st);
template <typename S>
hipError_t launch_cast(int64_t n, const double* src, S* dst, hipStream_t st);
hipError_t launch_rowsum(const double* src, int64_t R, int64_t C, int64_t ld, double* dst, double* scratch,
                         int64_t scratch_elems, hipStream_t st);
// Mean of the finite e[W] (stats[0]; count in stats[1] and, when n_finite is given, *n_finite) and the
// loss weights g[w] = 2 (e[w] - mean) / count (0 for non-finite e[w]); e_mean (may be NULL) receives the mean.
hipError_t launch_loss_weights(const double* e, int64_t W, double* stats, double* g, double* e_mean,
                               int64_t* n_finite, hipStream_t st);
template <typename S>
hipError_t launch_combine_bwd(const SysDev& s, const S* c, const double* ld, const double* sg, const double* gbar,
                              int64_t W, double* lbar, double* cpart, hipStream_t st);
template <typename S>
hipError_t launch_orb_bwd(const SysDev& s, int spin, const double* lbar, const double* ainv, const S* phi,
                          const S* pi, const S* sg, const double* en, int64_t W, S* phibar, double* pipart,
                          double* sgpart, hipStream_t st);
template <typename S>
hipError_t launch_agg_bwd(const SysDev& s, const S* mbar, const S* h, const S* wsame, const S* wopp, const S* wnuc,
                          const S* Y, int64_t W, S* hbar, S* wbs, S* wbo, S* wbn, double* ypart, hipStream_t st);

}  // namespace qmc
