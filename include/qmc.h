/*
 * qmc.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * real-space deep variational quantum Monte Carlo: batched evaluation of a
 * graph-network wave function over many walkers, its exact gradient and
 * Laplacian by forward propagation, the local energy, a random-walk
 * Metropolis step and the VMC loss gradient.
 *
 * The quantities follow the paper (arXiv 2307.14123, DeepQMC):
 *   - Hamiltonian inputs Z_I, R_I and the potential: molecular Hamiltonian,
 *     Sec. II.A (the constant nucleus-nucleus repulsion is added when
 *     qmc_ansatz.include_vnn is set).
 *   - Spin convention: electrons 0..n_up-1 are spin-up, Sec. II.B.
 *   - Ansatz: generalised Slater determinants (Sec. II.C) with graph-network
 *     electron embeddings (Sec. III.A), orbitals times isotropic exponential
 *     envelopes (Sec. III.B), spin-factorised determinants (Sec. III.C), in
 *     the log domain (Sec. III.E).
 *   - Local energy E_loc = -1/2 sum_i (Delta_i log|psi| + |grad_i log|psi||^2)
 *     + V, Sec. IV.B.
 *   - Loss gradient 2 E[(E_loc - L) grad_theta log|psi|], Sec. IV.A.
 *   - Random-walk Metropolis sampler, Sec. V.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   Memory: every array argument except the qmc_system / qmc_ansatz host
 *     arrays is DEVICE memory owned by the caller.  The library never keeps a
 *     pointer past the call.  Workspace `ws` is caller-allocated device memory
 *     of at least qmc_workspace_size(plan, op) bytes, 256-byte aligned.
 *   Layout: row-major, walker-major.  For a plan over several systems the
 *     walker arrays are the concatenation of each system's block (system 0
 *     first) and `params` is the concatenation of each system's blob.
 *   Types: positions r, noise, u, logpsi, sign, grad, lap, e_loc, cotangent
 *     and e_mean are double.  `params` and `grad_params` are double for a
 *     QMC_FP64 plan and float for QMC_FP32 / QMC_BF16_MIXED plans.
 *   Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Calls enqueue work and return without synchronising; outputs
 *     are valid once the stream reaches that point.
 *   Errors: arguments are validated on the host before anything is enqueued;
 *     a failed validation returns a status and launches nothing.  HIP launch
 *     failures return QMC_ERR_HIP.  Nothing aborts and no exception crosses
 *     the ABI.  Numerical anomalies are data: psi = 0 gives sign 0 and
 *     logpsi = -inf, and an undefined local energy is NaN.
 *   Concurrency: a plan is immutable after creation; concurrent calls on
 *     different streams with different workspaces are safe, except on a
 *     plan created with QMC_PLAN_CONCURRENT_SYSTEMS (its internal streams
 *     are shared by all calls).
 */
#ifndef QMC_H_
#define QMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One molecule (Sec. II.A): n_nuc nuclei with charges[n_nuc] and
 * coords[n_nuc][3] in bohr (host arrays, copied by qmc_plan_create), n_up
 * spin-up electrons followed by n_down spin-down electrons. */
typedef struct qmc_system {
  int32_t n_nuc;
  const double* charges;
  const double* coords;
  int32_t n_up;
  int32_t n_down;
} qmc_system;

/* Hyper-parameters of the ansatz (Sec. III).  version must be 1.
 *   n_rbf, rbf_dmax : Gaussian radial basis of distances, centres
 *                     k*rbf_dmax/(n_rbf-1), width rbf_dmax/(n_rbf-1)
 *   init_layers     : tanh layers of the electron-node initialisation
 *   width           : embedding width D
 *   mp_layers       : message-passing interaction layers
 *   n_det           : determinants
 *   n_env           : envelope exponents per (orbital, nucleus)
 *   include_vnn     : add sum_{I<J} Z_I Z_J / R_IJ to the potential
 *   ee_cusp         : alpha > 0 multiplies psi by the fixed electron-electron
 *                     cusp factor exp(gamma) of Sec. III.D, taken as
 *                     gamma = sum_{i<j} -c_ij alpha^2 / (alpha + r_ij) with
 *                     c_ij = 1/4 (same spin) or 1/2 (opposite spin), whose
 *                     slope at r_ij = 0 is c_ij for every alpha; 0 = none.
 *                     It has no parameters: gradients of log|psi| with respect
 *                     to the blob do not change.
 *   jastrow         : 1 multiplies psi by the learnable Jastrow factor exp(J)
 *                     of Sec. III.D, J = tanh(s W1 + b1) W2 + b2 with
 *                     s = sum_i f_i the sum of the final electron embeddings
 *                     (an MLP of one hidden layer of width D); 0 = none.
 *   full_det        : 1 takes one N x N determinant per p over both spins
 *                     (Sec. III.C, full-determinant equation): each spin's
 *                     orbital map gives N orbitals, row i of A^p is electron i
 *                     (up electrons first); needs N <= 32.  0 = spin-factorized
 *                     determinants.
 *   edge_update     : 1 updates the edge features in every interaction layer
 *                     after the first (Sec. III.A, edge update), per edge
 *                     type: f_e^l = tanh(f_e^(l-1) Ve^l + ce^l), f_e^0 the
 *                     radial basis; the filters of layer l read f_e^l.  0 =
 *                     the basis is reused in every layer. */
typedef struct qmc_ansatz {
  int32_t version;
  int32_t n_rbf;
  double rbf_dmax;
  int32_t init_layers;
  int32_t width;
  int32_t mp_layers;
  int32_t n_det;
  int32_t n_env;
  int32_t include_vnn;
  double ee_cusp;
  int32_t jastrow;
  int32_t full_det;
  int32_t edge_update;
} qmc_ansatz;

typedef enum qmc_precision {
  QMC_FP64 = 0,        /* every stage in float64 */
  QMC_FP32 = 1,        /* embedding/orbital jets in float32, determinants,
                          geometry and combination in float64 */
  QMC_BF16_MIXED = 2,  /* as QMC_FP32, but the embedding GEMMs take bf16
                          operands with float32 accumulation */
  QMC_BF16_VALUE = 3   /* bf16 operands only in the forwards of value rows
                          (log|psi| for Metropolis, the loss gradient and
                          qmc_logpsi_grad); the jets of the local energy stay
                          float32 */
} qmc_precision;

typedef enum qmc_status {
  QMC_OK = 0,
  QMC_ERR_INVALID_ARGUMENT = 1,
  QMC_ERR_UNSUPPORTED = 2,
  QMC_ERR_WORKSPACE_TOO_SMALL = 3,
  QMC_ERR_HIP = 4,
  QMC_ERR_INTERNAL = 5
} qmc_status;

/* Operation codes for qmc_workspace_size. */
enum {
  QMC_OP_LOGPSI = 0,
  QMC_OP_LOCAL_ENERGY = 1,
  QMC_OP_METROPOLIS = 2,
  QMC_OP_LOGPSI_VJP = 3,
  QMC_OP_LOSS_GRAD = 4,
  QMC_OP_MALA = 5,
  QMC_OP_LOGPSI_GRAD = 6
};

typedef struct qmc_plan qmc_plan;

/* Number of scalar parameters of the ansatz blob for one system, or a
 * negative value if the arguments are invalid.  Host only, pure.
 * Blob order (matrices stored [in][out] so that a layer is y = x W + b):
 *   init.W1[(M+2)K][D] init.b1[D], then init.Wl[D][D] init.bl[D] for l>=2;
 *   per interaction layer: for t in (same, opp, nuc): U1[K][D] a1[D]
 *     U2[D][D] a2[D] (then, with edge_update, in layers after the first:
 *     Ve[K][K] ce[K]); then Wh[D][D] bh[D] Y[M][D] Wg[3D][D] bg[D];
 *   per spin with n_sigma > 0, with n_o = n_sigma (or N with full_det):
 *     Worb[D][n_det*n_o] borb[n_det*n_o] pi[n_det][n_o][M][n_env]
 *     sigma[n_det][n_o][M][n_env];
 *   c[n_det]; then, with jastrow = 1: jas.W1[D][D] jas.b1[D] jas.W2[D][1]
 *   jas.b2[1]. */
int64_t qmc_param_count(const qmc_system* system, const qmc_ansatz* ansatz);

/* Plan flags.
 * QMC_PLAN_CONCURRENT_SYSTEMS: a multi-system plan runs the kernel sequence
 *   of every system on its own stream owned by the plan, forked from and
 *   joined back to the caller's stream with events, so that the systems
 *   (molecules of different sizes) share the device; captured into a graph,
 *   the whole batch is one graph launch.  Each system then has its own
 *   workspace region (the workspace is the sum over systems instead of the
 *   maximum).  Calls on such a plan must not overlap (one caller stream at a
 *   time, in host order).
 * QMC_PLAN_AUTOTUNE: qmc_plan_create times the candidate GEMM tiles (K-step,
 *   tile height, persistent grid, and for float32 GEMMs the float32 form on
 *   the bf16 matrix cores with three-piece operands, whose error is at the
 *   float32 level) on the current device for every system's
 *   jet, value, edge and backward GEMM shapes and keeps the fastest.  This
 *   allocates device memory transiently and synchronises the device. */
enum { QMC_PLAN_CONCURRENT_SYSTEMS = 1u, QMC_PLAN_AUTOTUNE = 2u };

/* Create a plan for n_systems systems with walkers_per_system[s] walkers
 * each (host arrays).  flags: a combination of QMC_PLAN_* (0 for none);
 * unknown bits are an invalid argument.  On success *out owns the plan;
 * release it with qmc_plan_destroy.  Without flags this is host only: no
 * device memory is allocated and nothing is launched.  With flags it creates
 * streams and events on the current device (QMC_ERR_HIP if that fails). */
qmc_status qmc_plan_create(qmc_plan** out, const qmc_system* systems, int32_t n_systems,
                           const int64_t* walkers_per_system, const qmc_ansatz* ansatz,
                           qmc_precision precision, uint32_t flags);

/* As qmc_plan_create, with every system's walkers processed in chunks of at
 * most max_chunk_walkers walkers (0 = no cap; negative is an invalid
 * argument).  Chunks run one after another on the same workspace, so the cap
 * bounds the workspace of every operation; results do not depend on it.
 * Without a cap (and below the cap) the plan still halves a system's chunk
 * until the local-energy workspace of one chunk is at most 24 GiB. */
qmc_status qmc_plan_create_ex(qmc_plan** out, const qmc_system* systems, int32_t n_systems,
                              const int64_t* walkers_per_system, const qmc_ansatz* ansatz,
                              qmc_precision precision, uint32_t flags, int64_t max_chunk_walkers);

qmc_status qmc_plan_destroy(qmc_plan* plan);

/* Walkers per chunk of system s (the last chunk holds the remainder).  Host
 * only. */
qmc_status qmc_plan_chunk_walkers(const qmc_plan* plan, int32_t s, int64_t* walkers);

/* GEMM tile choice of system s, one entry per GEMM class (electron jets,
 * value rows, edge jets, backward value rows): 0 = built-in default, else
 * 1 + bits (bit 0: 32-wide K steps, bit 1: 64-row tiles, bit 2: persistent
 * grid, bit 3: float32 operands split into three bf16 pieces on the bf16
 * matrix cores).  Host only. */
qmc_status qmc_plan_tiles(const qmc_plan* plan, int32_t s, int32_t tiles[4]);

/* Bytes of workspace that operation `op` (QMC_OP_*) needs. */
qmc_status qmc_workspace_size(const qmc_plan* plan, int32_t op, size_t* bytes);

/* Total walkers, electrons of system s, and parameters of the whole plan. */
qmc_status qmc_plan_info(const qmc_plan* plan, int64_t* total_walkers, int64_t* total_params,
                         int64_t* total_positions);

/* sign psi and log|psi| (Sec. III.E) of every walker.
 *   r[W][N][3] -> logpsi[W], sign[W] (sign in {-1, 0, +1}). */
qmc_status qmc_logpsi(const qmc_plan* plan, const void* params, const double* r, double* logpsi,
                      double* sign, void* ws, size_t ws_bytes, void* stream);

/* Local energy (Sec. IV.B) with exact derivatives over all 3N coordinates:
 *   r[W][N][3] -> logpsi[W], sign[W], grad[W][N][3] = grad log|psi|,
 *   lap[W] = Laplacian of log|psi|, e_loc[W].
 * Any output pointer except e_loc may be NULL. */
qmc_status qmc_local_energy(const qmc_plan* plan, const void* params, const double* r,
                            double* logpsi, double* sign, double* grad, double* lap, double* e_loc,
                            void* ws, size_t ws_bytes, void* stream);

/* Size of the device array that qmc_local_energy_noalloc uses as its
 * workspace (64 MiB; one array per device, held from the library's load
 * until the process ends). */
#define QMC_NOALLOC_SCRATCH_BYTES (64u << 20)

/* qmc_local_energy for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same outputs from the same kernels, with the workspace
 * taken from the library's own scratch array instead of a caller buffer.  It
 * calls no allocator.  The plan's local-energy workspace,
 * qmc_workspace_size(plan, QMC_OP_LOCAL_ENERGY), must be at most
 * QMC_NOALLOC_SCRATCH_BYTES (create the plan with qmc_plan_create_ex and a
 * max_chunk_walkers small enough); otherwise QMC_ERR_WORKSPACE_TOO_SMALL is
 * returned, nothing is launched, and qmc_last_error() states both sizes.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, or host threads) race and must be
 * serialised by the caller.  The array keeps the last call's contents; the
 * local energy does not depend on what its workspace holds on entry (as for
 * the caller's ws of qmc_local_energy), so nothing is cleared between calls. */
qmc_status qmc_local_energy_noalloc(const qmc_plan* plan, const void* params, const double* r, double* logpsi,
                                    double* sign, double* grad, double* lap, double* e_loc, void* stream);

/* One random-walk Metropolis step (Sec. V): r' = r + step * noise, accepted
 * iff log(u) < 2 (log|psi(r')| - logpsi) in float64.  r and logpsi are
 * in/out and change only for accepted walkers; logpsi must hold log|psi(r)|
 * on entry.  noise[W][N][3] ~ N(0,1), u[W] in [0,1), accepted[W] in {0,1}
 * (accepted may be NULL). */
qmc_status qmc_metropolis_step(const qmc_plan* plan, const void* params, double* r,
                               double* logpsi, const double* noise, const double* u, double step,
                               uint8_t* accepted, void* ws, size_t ws_bytes, void* stream);

/* log|psi| and its gradient over the electron coordinates by the value
 * forward and one reverse pass (no Laplacian): logpsi[W], grad[W][N][3]
 * (NaN where log|psi| is not finite).  Equal to the logpsi and grad outputs
 * of qmc_local_energy up to rounding. */
qmc_status qmc_logpsi_grad(const qmc_plan* plan, const void* params, const double* r, double* logpsi,
                           double* grad, void* ws, size_t ws_bytes, void* stream);

/* One Metropolis-adjusted Langevin step (Sec. V, Langevin sampler).  With
 * tau = step^2 the proposal is r' = (r + tau D(r)) + step * noise, where the
 * drift D is grad log|psi| (damp = 0) or, with damp = 1, each electron's
 * gradient v shortened near its nearest nucleus I (charge Z, distance d):
 *   a = 1/2 + (Z d)^2 / (10 (4 + (Z d)^2)),
 *   v_bar = v * 2 / (1 + sqrt(1 + 2 a |v|^2 tau)),
 * then scaled down so that tau |v_bar| <= d (the step-size correction near
 * nuclei of Sec. V, taken in the drift-limit form of Umrigar, Nightingale and
 * Runge, J. Chem. Phys. 99, 2865 (1993), angular term at its mean).  The
 * proposal is accepted iff, in float64,
 *   log(u) < 2 (l' - l) + |noise|^2 / 2 - |noise + step (D(r) + D(r'))|^2 / 2
 * (the Metropolis-Hastings ratio of the two Gaussian proposal densities);
 * a non-finite l' or gradient rejects.  l' and its gradient come from the
 * value forward and one reverse pass (as qmc_logpsi_grad computes them).
 * r[W][N][3], logpsi[W] (log|psi(r)|) and grad[W][N][3] (grad log|psi(r)|,
 * as returned by qmc_logpsi_grad or qmc_local_energy) are in/out and change
 * only for accepted walkers.  noise[W][N][3] ~ N(0,1),
 * u[W] in [0,1), accepted[W] in {0,1} (may be NULL).  step must be finite
 * and >= 0; damp must be 0 or 1. */
qmc_status qmc_mala_step(const qmc_plan* plan, const void* params, double* r, double* logpsi,
                         double* grad, const double* noise, const double* u, double step,
                         int32_t damp, uint8_t* accepted, void* ws, size_t ws_bytes, void* stream);

/* Clipped local energies for the loss gradient (Sec. IV.D): per system, over
 * its finite e_loc, mu = median (the mean of the two middle values for an
 * even count) and sigma = width * mean |e_loc - mu|; mode 0 (hard) clamps to
 * [mu - sigma, mu + sigma]; mode 1 (soft) leaves the window unchanged and maps
 * a value outside it to mu +- sigma (1 + log(|e - mu| / sigma)).  Non-finite
 * values pass through, and so does everything when sigma is not positive.
 * e_loc[W] and e_out[W] are device arrays (e_out may equal e_loc); width
 * must be finite and > 0.  Pass e_out to qmc_loss_grad; energy estimates use
 * the unclipped values. */
qmc_status qmc_clip_local_energy(const qmc_plan* plan, const double* e_loc, double* e_out, double width,
                                 int32_t mode, void* stream);

/* Vector-Jacobian product of log|psi| with respect to the parameters:
 *   grad_params[P] = sum_w cotangent[w] * d log|psi_w| / d params. */
qmc_status qmc_logpsi_vjp(const qmc_plan* plan, const void* params, const double* r,
                          const double* cotangent, void* grad_params, void* ws, size_t ws_bytes,
                          void* stream);

/* VMC loss gradient (Sec. IV.A): over the walkers of each system whose
 * e_loc is finite, e_mean = their mean local energy (float64) and
 *   grad_params = (2 / W_f) sum_w (e_loc[w] - e_mean) d log|psi_w| / d params.
 * e_loc[W] is an input (as returned by qmc_local_energy); e_mean[n_systems]
 * is a device output (may be NULL).  Walkers with a non-finite e_loc (psi = 0,
 * coincident particles) are left out of e_mean and of the sum; their count is
 * reported in the workspace header: when the call has completed on the
 * stream, ws begins with int64_t n_finite[n_systems], the number W_f of
 * walkers of each system that entered the estimator (0 gives e_mean = NaN
 * and a zero gradient).  The header is the first
 * roundup(8 n_systems, 256) bytes of ws and is included in
 * qmc_workspace_size(plan, QMC_OP_LOSS_GRAD). */
qmc_status qmc_loss_grad(const qmc_plan* plan, const void* params, const double* r,
                         const double* e_loc, void* grad_params, double* e_mean, void* ws,
                         size_t ws_bytes, void* stream);

/* Determinant stage on caller-given orbital-matrix jets, for one spin block:
 * for each of n_mat matrices A (n x n) with derivative matrices over n_tan
 * coordinates and a Laplacian matrix, stored jets[n_mat][n_tan + 2][n][n]
 * (row 0 = A, rows 1..n_tan = dA/dx_c, row n_tan+1 = sum_c d2A/dx_c^2),
 * computes log|det A|, its sign, d log|det A| / dx_c = tr(A^-1 dA_c) and
 * Delta log|det A| = tr(A^-1 lapA) - sum_c tr((A^-1 dA_c)^2) (Jacobi's
 * formula; the log-domain determinant of Sec. III.E).  All device float64:
 * logdet[n_mat], sign[n_mat], grad[n_mat][n_tan], lap[n_mat]. */
qmc_status qmc_det_jets(int64_t n_mat, int32_t n, int32_t n_tan, const double* jets,
                        double* logdet, double* sign, double* grad, double* lap, void* stream);

/* Optimizer step of a training iteration (plain gradient descent on the
 * parameter blob, Sec. IV.A): params[i] -= lr * grad[i] for i < n, computed
 * in float64 (product and difference each rounded, no fused multiply-add)
 * and rounded to the io dtype of the precision (float64 for
 * QMC_FP64, float32 otherwise).  params, grad: device, n elements each
 * (grad as written by qmc_loss_grad); enqueued on stream.  Invalid
 * arguments (n < 0, null pointers with n > 0, non-finite lr, unknown
 * precision) return QMC_ERR_INVALID_ARGUMENT and launch nothing. */
qmc_status qmc_sgd_update(int32_t precision, void* params, const void* grad, int64_t n, double lr,
                          void* stream);

/* Achievable device peaks, the denominators of measured roofline fractions:
 * peaks[0..2] = MFMA TFLOP/s of float32 16x16x4, bf16 16x16x32 and float64
 * 16x16x4 instructions (register operands, independent accumulation chains,
 * every compute unit busy), peaks[3] = GB/s of a plain device copy (bytes
 * read + bytes written) between the two halves of scratch.  scratch: device
 * buffer owned by the caller, 16-byte aligned, 64 MiB to 16 GiB (its contents
 * are overwritten; 512 MiB or more measures HBM rather than cache); peaks:
 * host double[4].  Synchronises the stream (it times itself with HIP events
 * on it); a measurement utility, not part of the method. */
qmc_status qmc_measure_peaks(void* scratch, size_t scratch_bytes, double* peaks, void* stream);

/* Launch timing for measurement.  While enabled (process-wide), every kernel
 * launch is bracketed by a pair of HIP events on its stream.
 * qmc_profile_report waits for the recorded events and writes one line per
 * kernel, "name launches total_ms\n", into buf (host, len bytes); reset != 0
 * clears the records.  Not safe to call concurrently with launches from
 * other host threads. */
qmc_status qmc_profile_enable(int32_t on);
qmc_status qmc_profile_report(char* buf, size_t len, int32_t reset);

const char* qmc_status_str(qmc_status status);

/* Text of the calling thread's last QMC_ERR_HIP: the HIP error name and the
 * failing launch or call ("" before the first failure).  Static storage owned
 * by the library, valid until the thread's next failing call. */
const char* qmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H_ */
