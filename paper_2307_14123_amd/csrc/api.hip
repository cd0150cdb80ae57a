// C-ABI entry points: validate on the host, then enqueue the kernel sequence
// of each system and walker chunk on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "plan.h"

namespace qmc {

// ---------------------------------------------------------------- launch timing
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;

bool prof_on() { return g_prof_on; }
void prof_push(const char* name, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back({name, a, b});
}

static SysDev make_dev(const Plan& P, const SysPlan& s) {
  SysDev d;
  std::memset(&d, 0, sizeof(d));
  d.N = s.N;
  d.M = s.M;
  d.nup = s.nup;
  d.ndn = s.ndn;
  d.T = s.T;
  d.Rp = s.Rp;
  d.K = P.ans.n_rbf;
  d.D = P.ans.width;
  d.ndet = P.ans.n_det;
  d.nenv = P.ans.n_env;
  d.P0 = s.P[0];
  d.P1 = s.P[1];
  d.P2 = s.P[2];
  d.dmax = P.ans.rbf_dmax;
  d.vnn = P.ans.include_vnn ? s.vnn : 0.0;
  d.ee_cusp = P.ans.ee_cusp;
  d.full_det = P.ans.full_det;
  for (int I = 0; I < s.M; ++I) {
    d.Z[I] = s.Z[I];
    for (int x = 0; x < 3; ++x) d.R[3 * I + x] = s.R[3 * I + x];
  }
  return d;
}

// The last HIP failure of this thread: error name, the failing call and its line.
static thread_local char g_last_error[512];

static qmc_status hip_failed(hipError_t e, const char* call, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s at api.hip:%d in %s", hipGetErrorName(e), line, call);
  return QMC_ERR_HIP;
}

#define CK(x)                                                   \
  do {                                                          \
    hipError_t e_ = (x);                                        \
    if (e_ != hipSuccess) return hip_failed(e_, #x, __LINE__);  \
  } while (0)

// Kind of the embedding GEMMs: value_rows for the log|psi| forwards (value rows only).
static GemmKind embed_kind(qmc_precision p, bool value_rows) {
  if (p == QMC_FP64) return GK_F64;
  if (p == QMC_BF16_MIXED || (p == QMC_BF16_VALUE && value_rows)) return GK_BF16;
  return GK_F32;
}
// float32 plans whose edge filters of this pass run in the fused float32 kernel
static bool fused_edges(const Plan& P, bool value_rows) {
  return P.prec == QMC_FP32 || (P.prec == QMC_BF16_VALUE && !value_rows);
}
static GemmKind orbital_kind(qmc_precision p) { return p == QMC_FP64 ? GK_F64 : GK_F32; }

// GEMM with the plan's tile choice for its class (electron jets, edge jets, value rows, backward).
static hipError_t gemm(const SysPlan& s, GemmKind kind, GemmArgs a, hipStream_t st) {
  const int cls = !a.vmode ? (a.Rp == 4 ? TILE_EDGE : TILE_JET) : (a.transw ? TILE_BWD : TILE_VAL);
  if (a.tile == 0) a.tile = s.tile[cls];
  return launch_gemm(kind, a, st);
}

static GemmArgs dense(const void* X, int64_t ldx, const void* W, int64_t ldw, const void* bias, void* Y, int64_t ldy,
                      int64_t rows, int K, int Ncols, int Rp, int T, int act, int vmode) {
  GemmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.X = X;
  a.ldx = ldx;
  a.xrpw = rows;
  a.xws = 0;
  a.W = W;
  a.ldw = ldw;
  a.bias = bias;
  a.Res = nullptr;
  a.Y = Y;
  a.ldy = ldy;
  a.yrpw = rows;
  a.yws = 0;
  a.rows = rows;
  a.K = K;
  a.Ncols = Ncols;
  a.Rp = Rp;
  a.T = T;
  a.act = act;
  a.vmode = vmode;
  a.transw = 0;
  return a;
}

struct Outs {
  double* logpsi;
  double* sign;
  double* grad;
  double* lap;
  double* eloc;
};

// Forward pass of one walker chunk: jet = 1 propagates value, 3N tangent and
// Laplacian rows (local energy); jet = 0 propagates values only (log|psi|).
template <typename S>
static qmc_status forward_chunk(const Plan& P, const SysPlan& s, const S* prm, const double* r, int64_t wc, int jet,
                                const Workspace& L, char* ws, const Outs& out, hipStream_t st) {
  const SysDev dv = make_dev(P, s);
  const int64_t N = s.N, M = s.M, D = P.ans.width, K = P.ans.n_rbf, ND = P.ans.n_det;
  const int Rp = jet ? s.Rp : 1, Re = jet ? 4 : 1, vm = jet ? 0 : 1;
  const GemmKind gk = embed_kind(P.prec, !jet), ok = orbital_kind(P.prec);
  double* ee = (double*)(ws + L.geom);
  double* en = ee + wc * N * N * 4;
  double* vpot = (double*)(ws + L.vpot);
  S* rho[3];
  S* ehid[3];
  S* wj[3];
  for (int t = 0; t < 3; ++t) {
    rho[t] = (S*)(ws + L.rho[t]);
    ehid[t] = (S*)(ws + L.ehid[t]);
    wj[t] = (S*)(ws + L.wjet[t]);
  }
  S* x0 = (S*)(ws + L.x0);
  S* f = (S*)(ws + L.f);
  S* h = (S*)(ws + L.h);
  S* m = (S*)(ws + L.m);
  S* ajet = (S*)(ws + L.ajet);
  double* dld = (double*)(ws + L.dld);
  double* dsg = (double*)(ws + L.dsg);
  double* dg = (double*)(ws + L.dg);
  double* dlap = (double*)(ws + L.dlap);
  const ParamOffsets& O = s.off;

  CK(launch_geometry(dv, r, wc, ee, en, jet ? vpot : nullptr, st));
  // float32 plans of width 128 or 256 evaluate each edge filter in one fused kernel from the distances
  // (with edge updates, the updated features of later layers are read from memory instead)
  const bool fused = std::is_same<S, float>::value && fused_edges(P, !jet) && edge_mlp_supported(dv);
  if (P.ans.mp_layers > 0 && (!fused || P.ans.edge_update))
    for (int t = 0; t < 3; ++t) CK(launch_rbf<S>(dv, t, ee, en, wc, jet, rho[t], st));
  CK(launch_init_features<S>(dv, ee, en, wc, jet, x0, st));
  const int64_t rows = wc * N * Rp;
  const int F = (int)((M + 2) * K);
  CK(gemm(s, gk, dense(x0, F, prm + O.initW[0], D, prm + O.initb[0], f, D, rows, F, (int)D, Rp, s.T, 1, vm), st));
  for (int l = 1; l < P.ans.init_layers; ++l) {
    CK(gemm(s, gk, dense(f, D, prm + O.initW[l], D, prm + O.initb[l], h, D, rows, (int)D, (int)D, Rp, s.T, 1, vm),
                   st));
    S* tmp = f;
    f = h;
    h = tmp;
  }
  S* fe[3] = {rho[0], rho[1], rho[2]};  // the edge features the filters read
  for (int l = 0; l < P.ans.mp_layers; ++l) {
    const auto& Ly = O.mp[l];
    EdgeMlpArgs eb[3];  // the fused filters of this layer, one launch for all types
    int ne = 0;
    for (int t = 0; t < 3; ++t) {
      const int64_t re = wc * s.P[t] * Re;
      if (re == 0) continue;
      if (Ly.Ve[t] >= 0) {
        // edge-feature update f_e <- tanh(f_e Ve + ce), univariate jets (4 rows an edge) or values
        S* nx = fe[t] == rho[t] ? (S*)(ws + L.rho2[t]) : rho[t];
        CK(gemm(s, gk, dense(fe[t], K, prm + Ly.Ve[t], K, prm + Ly.ce[t], nx, K, re, (int)K, (int)K, Re, 1, 1, vm),
                st));
        fe[t] = nx;
      }
      if constexpr (std::is_same<S, float>::value) {
        if (fused) {
          eb[ne++] = EdgeMlpArgs{prm + Ly.U1[t], prm + Ly.a1[t], prm + Ly.U2[t], prm + Ly.a2[t], ee, en, wj[t],
                                 nullptr, wc * s.P[t], t, jet, Ly.Ve[t] >= 0 ? (const float*)fe[t] : nullptr};
          continue;
        }
      }
      CK(gemm(s, gk, dense(fe[t], K, prm + Ly.U1[t], D, prm + Ly.a1[t], ehid[t], D, re, (int)K, (int)D, Re, 1, 1, vm),
                     st));
      CK(gemm(s, gk, dense(ehid[t], D, prm + Ly.U2[t], D, prm + Ly.a2[t], wj[t], D, re, (int)D, (int)D, Re, 1, 0, vm),
                     st));
    }
    if (ne > 0) CK(launch_edge_mlp_types(dv, eb, ne, st));
    CK(gemm(s, gk, dense(f, D, prm + Ly.Wh, D, prm + Ly.bh, h, D, rows, (int)D, (int)D, Rp, s.T, 0, vm), st));
    CK(launch_aggregate<S>(dv, h, wj[0], wj[1], wj[2], prm + Ly.Y, ee, en, wc, jet, m, st));
    if (jet) {
      // electron messages [W][N][Rp][2D]; the nuclear message has 5 nonzero jet rows per electron:
      // its product with the nuclear block of W_g is formed on those rows and added before the tanh
      S* mn5 = (S*)(ws + L.mn5);
      S* zn5 = (S*)(ws + L.zn5);
      CK(launch_nuc_message<S>(dv, wj[2], prm + Ly.Y, en, wc, mn5, st));
      CK(gemm(s, gk, dense(mn5, D, prm + Ly.Wg + 2 * D * D, D, nullptr, zn5, D, wc * N * 5, (int)D, (int)D, 1, 0, 0,
                               1), st));
      GemmArgs g = dense(m, 2 * D, prm + Ly.Wg, D, prm + Ly.bg, f, D, rows, (int)(2 * D), (int)D, Rp, s.T, 1, vm);
      g.Res = f;
      g.add5 = zn5;
      g.nel = (int)N;
      CK(gemm(s, gk, g, st));
    } else {
      GemmArgs g = dense(m, 3 * D, prm + Ly.Wg, D, prm + Ly.bg, f, D, rows, (int)(3 * D), (int)D, Rp, s.T, 1, vm);
      g.Res = f;
      CK(gemm(s, gk, g, st));
    }
  }
  // learnable Jastrow exponent J = tanh(s W1 + b1) W2 + b2 of the summed embeddings s = sum_i f_i,
  // with jets (the sum of the electrons' jet rows is the jet of s); h and m are free here
  S* jas = nullptr;
  if (P.ans.jastrow) {
    jas = (S*)(ws + L.jas);
    CK(launch_sum_electrons<S>(wc, (int)N, Rp, (int)D, f, h, st));
    CK(gemm(s, gk, dense(h, D, prm + O.jW1, D, prm + O.jb1, m, D, wc * Rp, (int)D, (int)D, Rp, s.T, 1, vm), st));
    CK(launch_jastrow_out<S>(wc * Rp, Rp, (int)D, m, prm + O.jW2, prm + O.jb2, jas, st));
  }
  int64_t off_e = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t n = s.nsig(sp), no = s.norb(sp);  // electrons of this spin, orbitals per determinant
    if (n == 0) continue;
    GemmArgs a = dense(f + off_e * Rp * D, D, prm + O.orbW[sp], ND * no, prm + O.orbb[sp], (S*)(ws + L.phi[sp]),
                       ND * no, wc * n * Rp, (int)D, (int)(ND * no), Rp, s.T, 0, vm);
    a.xrpw = n * Rp;
    a.xws = N * Rp * D;
    CK(gemm(s, ok, a, st));
    CK(launch_envelope<S>(dv, sp, (S*)(ws + L.phi[sp]), prm + O.pi[sp], prm + O.sigma[sp], en, wc, jet, ajet, st));
    off_e += n;
  }
  CK(launch_det<S>(dv, ajet, wc, jet, dld, dsg, dg, dlap, nullptr, st));
  CK(launch_combine<S>(dv, prm + O.c, dld, dsg, dg, dlap, vpot, ee, jas, wc, jet, out.logpsi, out.sign, out.grad, out.lap,
                       out.eloc, st));
  return QMC_OK;
}

static bool ws_ok(const Plan& P, int op, const void* ws, size_t ws_bytes) {
  if (!ws) return false;
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return false;
  return ws_bytes >= workspace_bytes(P, op);
}

static int64_t pos_offset(const Plan& P, const SysPlan& s) {
  int64_t pos = 0;
  for (const auto& t : P.sys) {
    if (&t == &s) break;
    pos += t.W * t.N * 3;
  }
  return pos;
}

// Runs f(si, stream, workspace) for every system: in order on the caller's stream, or, for a plan
// with concurrent systems, each on the plan's stream of that system (with its own workspace
// region) between a fork event recorded on the caller's stream and a join event it waits for.
template <class F>
static qmc_status for_systems(const Plan& P, int op, char* ws, hipStream_t st, F f) {
  if (!P.concurrent()) {
    for (size_t si = 0; si < P.sys.size(); ++si) {
      const qmc_status e = f(si, st, ws + sys_ws_offset(P, op, si));
      if (e != QMC_OK) return e;
    }
    return QMC_OK;
  }
  CK(hipEventRecord((hipEvent_t)P.fork, st));
  qmc_status err = QMC_OK;
  for (size_t si = 0; si < P.sys.size(); ++si) {
    hipStream_t ss = (hipStream_t)P.streams[si];
    if (err == QMC_OK && hipStreamWaitEvent(ss, (hipEvent_t)P.fork, 0) != hipSuccess) err = QMC_ERR_HIP;
    if (err == QMC_OK) err = f(si, ss, ws + sys_ws_offset(P, op, si));
    // every side stream joins back, also after an error, so that a stream capture stays well formed
    if (hipEventRecord((hipEvent_t)P.joins[si], ss) != hipSuccess ||
        hipStreamWaitEvent(st, (hipEvent_t)P.joins[si], 0) != hipSuccess)
      err = QMC_ERR_HIP;
  }
  return err;
}

template <typename S>
static qmc_status run_forward(const Plan& P, const void* params, const double* r, const Outs& o, int jet, char* ws,
                              hipStream_t st) {
  const int op = jet ? QMC_OP_LOCAL_ENERGY : QMC_OP_LOGPSI;
  return for_systems(P, op, ws, st, [&](size_t si, hipStream_t ss, char* wsb) -> qmc_status {
    const SysPlan& s = P.sys[si];
    const S* prm = (const S*)params + s.param_offset;
    for (int64_t w0 = 0; w0 < s.W; w0 += s.Wc) {
      const int64_t wc = std::min<int64_t>(s.Wc, s.W - w0);
      const int64_t wg = s.walker_offset + w0;  // global walker index
      const Workspace L = workspace_layout(P, s, op, wc);
      Outs oc;
      oc.logpsi = o.logpsi ? o.logpsi + wg : nullptr;
      oc.sign = o.sign ? o.sign + wg : nullptr;
      oc.grad = o.grad ? o.grad + pos_offset(P, s) + w0 * s.T : nullptr;
      oc.lap = o.lap ? o.lap + wg : nullptr;
      oc.eloc = o.eloc ? o.eloc + wg : nullptr;
      const double* rc = r + pos_offset(P, s) + w0 * s.N * 3;
      const qmc_status e = forward_chunk<S>(P, s, prm, rc, wc, jet, L, wsb, oc, ss);
      if (e != QMC_OK) return e;
    }
    return QMC_OK;
  });
}

template <typename S>
static qmc_status run_metropolis(const Plan& P, const void* params, double* r, double* logpsi, const double* noise,
                                 const double* u, double step, uint8_t* accepted, char* ws, hipStream_t st) {
  return for_systems(P, QMC_OP_METROPOLIS, ws, st, [&](size_t si, hipStream_t ss, char* wsb) -> qmc_status {
    const SysPlan& s = P.sys[si];
    const S* prm = (const S*)params + s.param_offset;
    const int64_t pos = pos_offset(P, s);
    for (int64_t w0 = 0; w0 < s.W; w0 += s.Wc) {
      const int64_t wc = std::min<int64_t>(s.Wc, s.W - w0);
      const int64_t wg = s.walker_offset + w0;
      const Workspace L = workspace_layout(P, s, QMC_OP_METROPOLIS, wc);
      double* rp = (double*)(wsb + L.lp_prop);
      double* lpp = rp + wc * s.N * 3;
      const int64_t off = pos + w0 * s.N * 3;
      CK(launch_propose(r + off, noise + off, step, wc * s.N * 3, rp, ss));
      Outs oc;
      std::memset(&oc, 0, sizeof(oc));
      oc.logpsi = lpp;
      const qmc_status e = forward_chunk<S>(P, s, prm, rp, wc, 0, L, wsb, oc, ss);
      if (e != QMC_OK) return e;
      CK(launch_accept(wc, s.N * 3, rp, lpp, u + wg, r + off, logpsi + wg, accepted ? accepted + wg : nullptr, ss));
    }
    return QMC_OK;
  });
}


// ---------------------------------------------------------------- parameter backward

static WgradArgs wg(const void* X, int64_t ldx, const void* G, int64_t ldg, int64_t rows, int Kin, int Nout,
                    const BwdWorkspace& B, char* ws) {
  WgradArgs a;
  std::memset(&a, 0, sizeof(a));
  a.X = X;
  a.ldx = ldx;
  a.xrpw = rows;
  a.xws = 0;
  a.G = G;
  a.ldg = ldg;
  a.grpw = rows;
  a.gws = 0;
  a.rows = rows;
  a.Kin = Kin;
  a.Nout = Nout;
  a.ones = 1;
  a.part = (double*)(ws + B.wpart);
  a.part_elems = B.wpart_elems;
  return a;
}

// Value-only forward of one chunk that keeps every layer's activations.
template <typename S>
static qmc_status forward_stash(const Plan& P, const SysPlan& s, const S* prm, const double* r, int64_t wc,
                                const BwdWorkspace& B, char* ws, hipStream_t st) {
  const SysDev dv = make_dev(P, s);
  const int64_t N = s.N, M = s.M, D = P.ans.width, K = P.ans.n_rbf, ND = P.ans.n_det;
  const int L = P.ans.mp_layers, L0 = P.ans.init_layers;
  const GemmKind gk = embed_kind(P.prec, true), ok = orbital_kind(P.prec);
  const ParamOffsets& O = s.off;
  double* ee = (double*)(ws + B.geom);
  double* en = ee + wc * N * N * 4;
  auto F_ = [&](size_t base, int64_t blk, int l) { return (S*)(ws + base + size_t(blk) * l); };
  CK(launch_geometry(dv, r, wc, ee, en, nullptr, st));
  if (L > 0)
    for (int t = 0; t < 3; ++t) CK(launch_rbf<S>(dv, t, ee, en, wc, 0, (S*)(ws + B.rho[t]), st));
  S* x0 = (S*)(ws + B.x0);
  CK(launch_init_features<S>(dv, ee, en, wc, 0, x0, st));
  const int64_t rows = wc * N;
  const int Fd = (int)((M + 2) * K);
  CK(gemm(s, gk, dense(x0, Fd, prm + O.initW[0], D, prm + O.initb[0], F_(B.finit, B.blk_f, 0), D, rows, Fd,
                           (int)D, 1, 0, 1, 1), st));
  for (int l = 1; l < L0; ++l)
    CK(gemm(s, gk, dense(F_(B.finit, B.blk_f, l - 1), D, prm + O.initW[l], D, prm + O.initb[l],
                             F_(B.finit, B.blk_f, l), D, rows, (int)D, (int)D, 1, 0, 1, 1), st));
  S* fprev = F_(B.finit, B.blk_f, L0 - 1);
  for (int l = 0; l < L; ++l) {
    const auto& Ly = O.mp[l];
    EdgeMlpArgs eb[3];  // the fused filters of this layer, one launch for all types
    int ne = 0;
    for (int t = 0; t < 3; ++t) {
      const int64_t re = wc * s.P[t];
      if (re == 0) continue;
      S* eh = F_(B.ehid[t], B.blk_e[t], l);
      S* wv = F_(B.wv[t], B.blk_e[t], l);
      // edge features of this layer: the radial basis, or its update (every layer's is kept)
      S* fe = F_(B.rho[t], B.blk_r[t], Ly.Ve[t] >= 0 ? l : 0);
      if (Ly.Ve[t] >= 0)
        CK(gemm(s, gk, dense(F_(B.rho[t], B.blk_r[t], l - 1), K, prm + Ly.Ve[t], K, prm + Ly.ce[t], fe, K, re, (int)K,
                             (int)K, 1, 0, 1, 1), st));
      if constexpr (std::is_same<S, float>::value) {
        if (fused_edges(P, true) && edge_mlp_supported(dv)) {
          // the hidden layer is kept for the backward
          eb[ne++] = EdgeMlpArgs{prm + Ly.U1[t], prm + Ly.a1[t], prm + Ly.U2[t], prm + Ly.a2[t], ee, en, wv, eh, re, t,
                                 0, Ly.Ve[t] >= 0 ? (const float*)fe : nullptr};
          continue;
        }
      }
      CK(gemm(s, gk, dense(fe, K, prm + Ly.U1[t], D, prm + Ly.a1[t], eh, D, re, (int)K, (int)D, 1, 0, 1, 1), st));
      CK(gemm(s, gk, dense(eh, D, prm + Ly.U2[t], D, prm + Ly.a2[t], wv, D, re, (int)D, (int)D, 1, 0, 0, 1), st));
    }
    if (ne > 0) CK(launch_edge_mlp_types(dv, eb, ne, st));
    S* h = F_(B.hst, B.blk_f, l);
    S* m = F_(B.mst, B.blk_m, l);
    S* t = F_(B.tst, B.blk_f, l);
    S* fo = F_(B.fst, B.blk_f, l);
    CK(gemm(s, gk, dense(fprev, D, prm + Ly.Wh, D, prm + Ly.bh, h, D, rows, (int)D, (int)D, 1, 0, 0, 1), st));
    CK(launch_aggregate<S>(dv, h, F_(B.wv[0], B.blk_e[0], l), F_(B.wv[1], B.blk_e[1], l), F_(B.wv[2], B.blk_e[2], l),
                           prm + Ly.Y, ee, en, wc, 0, m, st));
    CK(gemm(s, gk, dense(m, 3 * D, prm + Ly.Wg, D, prm + Ly.bg, t, D, rows, (int)(3 * D), (int)D, 1, 0, 1, 1), st));
    CK(launch_add<S>(rows * D, fprev, t, fo, st));
    fprev = fo;
  }
  if (P.ans.jastrow) {
    CK(launch_sum_electrons<S>(wc, (int)N, 1, (int)D, fprev, (S*)(ws + B.jsum), st));
    CK(gemm(s, gk, dense((S*)(ws + B.jsum), D, prm + O.jW1, D, prm + O.jb1, (S*)(ws + B.jhid), D, wc, (int)D, (int)D,
                         1, 0, 1, 1), st));
  }
  int64_t off_e = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t n = s.nsig(sp), no = s.norb(sp);
    if (n == 0) continue;
    GemmArgs a = dense(fprev + off_e * D, D, prm + O.orbW[sp], ND * no, prm + O.orbb[sp], (S*)(ws + B.phi[sp]),
                       ND * no, wc * n, (int)D, (int)(ND * no), 1, 0, 0, 1);
    a.xrpw = n;
    a.xws = N * D;
    CK(gemm(s, ok, a, st));
    CK(launch_envelope<S>(dv, sp, (S*)(ws + B.phi[sp]), prm + O.pi[sp], prm + O.sigma[sp], en, wc, 0,
                          (S*)(ws + B.aval), st));
    off_e += n;
  }
  CK(launch_det<S>(dv, (S*)(ws + B.aval), wc, 0, (double*)(ws + B.dld), (double*)(ws + B.dsg), nullptr, nullptr,
                   (double*)(ws + B.ainv), st));
  return QMC_OK;
}

// Cotangent gbar[wc] on log|psi| of the chunk -> accumulate parameter gradients into gacc (float64).
// With rbar given, the pass computes the position gradient [wc][N][3] instead of the parameter
// gradients (lp: log|psi| of the chunk, for the non-finite flag).
template <typename S>
static qmc_status backward_chunk(const Plan& P, const SysPlan& s, const S* prm, const double* gbar, int64_t wc,
                                 const BwdWorkspace& B, char* ws, hipStream_t st, double* rbar = nullptr,
                                 const double* lp = nullptr) {
  const bool pg = rbar == nullptr;  // parameter gradients
  const SysDev dv = make_dev(P, s);
  const int64_t N = s.N, M = s.M, D = P.ans.width, K = P.ans.n_rbf, ND = P.ans.n_det;
  const int L = P.ans.mp_layers, L0 = P.ans.init_layers;
  const GemmKind bk = P.prec == QMC_FP64 ? GK_F64 : GK_F32;
  const ParamOffsets& O = s.off;
  double* gacc = (double*)(ws + B.gacc);
  double* ee = (double*)(ws + B.geom);
  double* en = ee + wc * N * N * 4;
  double* dee = (double*)(ws + B.dee);
  double* den = (double*)(ws + B.den);
  if (!pg) {
    CK(launch_fill(wc * N * N, 0.0, dee, st));
    CK(launch_fill(wc * N * M, 0.0, den, st));
  }
  auto F_ = [&](size_t base, int64_t blk, int l) { return (S*)(ws + base + size_t(blk) * l); };
  const int64_t rows = wc * N;
  double* lbar = (double*)(ws + B.lbar);
  double* cpart = (double*)(ws + B.cpart);
  CK(launch_combine_bwd<S>(dv, prm + O.c, (double*)(ws + B.dld), (double*)(ws + B.dsg), gbar, wc, lbar, cpart, st));
  if (pg) CK(launch_rowsum(cpart, wc, ND, ND, gacc + O.c, (double*)(ws + B.wpart), B.wpart_elems, st));
  // Jastrow exponent: its cotangent is gbar itself (log|psi| = determinant part + J)
  S* jfs = nullptr;
  if (P.ans.jastrow) {
    S* jhid = (S*)(ws + B.jhid);
    S* jzb = (S*)(ws + B.jzb);
    S* jgo = (S*)(ws + B.jgo);
    jfs = (S*)(ws + B.jfs);
    CK(launch_jastrow_bwd<S>(wc, (int)D, gbar, prm + O.jW2, jhid, jzb, jgo, st));
    if (pg) {
      CK(launch_wgrad(bk, wg(jhid, D, jgo, 1, wc, (int)D, 1, B, ws), gacc + O.jW2, 1, gacc + O.jb2, st));
      CK(launch_wgrad(bk, wg((S*)(ws + B.jsum), D, jzb, D, wc, (int)D, (int)D, B, ws), gacc + O.jW1, D,
                      gacc + O.jb1, st));
    }
    GemmArgs gj = dense(jzb, D, prm + O.jW1, D, nullptr, jfs, D, wc, (int)D, (int)D, 1, 0, 0, 1);
    gj.transw = 1;
    CK(gemm(s, bk, gj, st));
  }
  S* fL = L > 0 ? F_(B.fst, B.blk_f, L - 1) : F_(B.finit, B.blk_f, L0 - 1);
  S* fbar = (S*)(ws + B.fbar);
  S* fbar2 = (S*)(ws + B.fbar2);
  int64_t off_e = 0;
  const double* ainv = (double*)(ws + B.ainv);
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t n = s.nsig(sp);
    if (n == 0) continue;
    const int64_t ncol = ND * s.norb(sp);
    S* phib = (S*)(ws + B.phibar[sp]);
    double* pip = (double*)(ws + B.pipart);
    double* sgp = (double*)(ws + B.sgpart);
    // inverses of this spin's matrices (with the full determinant both spins share the N x N ones)
    const double* ai = ainv + (sp && !s.full_det ? wc * ND * s.nup * s.nup : 0);
    CK(launch_orb_bwd<S>(dv, sp, lbar, ai, (S*)(ws + B.phi[sp]), prm + O.pi[sp], prm + O.sigma[sp], en, wc, phib, pip,
                         sgp, st));
    if (pg) {
      const int64_t ne = ncol * M * P.ans.n_env;
      CK(launch_rowsum(pip, wc, ne, ne, gacc + O.pi[sp], (double*)(ws + B.wpart), B.wpart_elems, st));
      CK(launch_rowsum(sgp, wc, ne, ne, gacc + O.sigma[sp], (double*)(ws + B.wpart), B.wpart_elems, st));
      WgradArgs a = wg(fL + off_e * D, D, phib, ncol, wc * n, (int)D, (int)ncol, B, ws);
      a.xrpw = n;
      a.xws = N * D;
      CK(launch_wgrad(bk, a, gacc + O.orbW[sp], ncol, gacc + O.orbb[sp], st));
    } else {
      CK(launch_env_dbar<S>(dv, (int)sp, lbar, ai, (S*)(ws + B.phi[sp]), prm + O.pi[sp], prm + O.sigma[sp], en, wc,
                            den, st));
    }
    GemmArgs g = dense(phib, ncol, prm + O.orbW[sp], ncol, nullptr, fbar + off_e * D, D, wc * n, (int)ncol, (int)D, 1, 0,
                       0, 1);
    g.transw = 1;
    g.yrpw = n;
    g.yws = N * D;
    CK(gemm(s, bk, g, st));
    off_e += n;
  }
  // the summed embedding's cotangent reaches every electron
  if (jfs) CK(launch_add_bcast<S>(wc, (int)N, (int)D, jfs, fbar, st));
  S* zbar = (S*)(ws + B.zbar);
  S* hbar = (S*)(ws + B.hbar);
  S* mbar = (S*)(ws + B.mbar);
  S* ebar = (S*)(ws + B.ebar);
  for (int l = L - 1; l >= 0; --l) {
    const auto& Ly = O.mp[l];
    S* fin = l == 0 ? F_(B.finit, B.blk_f, L0 - 1) : F_(B.fst, B.blk_f, l - 1);
    CK(launch_tanh_bwd<S>(rows * D, fbar, F_(B.tst, B.blk_f, l), zbar, st));
    if (pg)
      CK(launch_wgrad(bk, wg(F_(B.mst, B.blk_m, l), 3 * D, zbar, D, rows, (int)(3 * D), (int)D, B, ws), gacc + Ly.Wg,
                      D, gacc + Ly.bg, st));
    GemmArgs gm = dense(zbar, D, prm + Ly.Wg, D, nullptr, mbar, 3 * D, rows, (int)D, (int)(3 * D), 1, 0, 0, 1);
    gm.transw = 1;
    CK(gemm(s, bk, gm, st));
    S* wb[3] = {(S*)(ws + B.wbar[0]), (S*)(ws + B.wbar[1]), (S*)(ws + B.wbar[2])};
    double* yp = (double*)(ws + B.ypart);
    CK(launch_agg_bwd<S>(dv, mbar, F_(B.hst, B.blk_f, l), F_(B.wv[0], B.blk_e[0], l), F_(B.wv[1], B.blk_e[1], l),
                         F_(B.wv[2], B.blk_e[2], l), prm + Ly.Y, wc, hbar, wb[0], wb[1], wb[2], yp, st));
    if (pg) {
      CK(launch_rowsum(yp, wc, M * D, M * D, gacc + Ly.Y, (double*)(ws + B.wpart), B.wpart_elems, st));
      CK(launch_wgrad(bk, wg(fin, D, hbar, D, rows, (int)D, (int)D, B, ws), gacc + Ly.Wh, D, gacc + Ly.bh, st));
    }
    GemmArgs gh = dense(hbar, D, prm + Ly.Wh, D, nullptr, fbar2, D, rows, (int)D, (int)D, 1, 0, 0, 1);
    gh.transw = 1;
    gh.Res = fbar;
    CK(gemm(s, bk, gh, st));
    std::swap(fbar, fbar2);
    for (int t = 0; t < 3; ++t) {
      const int64_t re = wc * s.P[t];
      if (re == 0) continue;
      S* eh = F_(B.ehid[t], B.blk_e[t], l);
      if (pg)
        CK(launch_wgrad(bk, wg(eh, D, wb[t], D, re, (int)D, (int)D, B, ws), gacc + Ly.U2[t], D, gacc + Ly.a2[t],
                        st));
      GemmArgs ge = dense(wb[t], D, prm + Ly.U2[t], D, nullptr, ebar, D, re, (int)D, (int)D, 1, 0, 2, 1);
      ge.transw = 1;
      ge.aux = eh;
      CK(gemm(s, bk, ge, st));
      const bool upd = Ly.Ve[t] >= 0;  // this layer's edge features are an update of the previous layer's
      S* fe = F_(B.rho[t], B.blk_r[t], upd ? l : 0);
      if (pg)
        CK(launch_wgrad(bk, wg(fe, K, ebar, D, re, (int)K, (int)D, B, ws), gacc + Ly.U1[t], D, gacc + Ly.a1[t], st));
      if (!pg || upd) {
        // edge-feature cotangents rhobar = ebar U1^T, plus what the next layer's update carried back
        S* rb = (S*)(ws + B.rhobar);
        S* carry = (S*)(ws + B.ecarry[t]);
        GemmArgs gr = dense(ebar, D, prm + Ly.U1[t], D, nullptr, rb, K, re, (int)D, (int)K, 1, 0, 0, 1);
        gr.transw = 1;
        if (l + 1 < L && O.mp[l + 1].Ve[t] >= 0 && (!pg || l >= 1)) gr.Res = carry;
        CK(gemm(s, bk, gr, st));
        if (upd) {
          // through f_e^l = tanh(f_e^(l-1) Ve + ce): pre-activation cotangent (in ebar's space), the
          // update's weights, and the cotangent of f_e^(l-1) when a lower layer still needs it
          S* zb = ebar;
          CK(launch_tanh_bwd<S>(re * K, rb, fe, zb, st));
          if (pg)
            CK(launch_wgrad(bk, wg(F_(B.rho[t], B.blk_r[t], l - 1), K, zb, K, re, (int)K, (int)K, B, ws),
                            gacc + Ly.Ve[t], K, gacc + Ly.ce[t], st));
          if (!pg || l >= 2) {
            GemmArgs gc = dense(zb, K, prm + Ly.Ve[t], K, nullptr, carry, K, re, (int)K, (int)K, 1, 0, 0, 1);
            gc.transw = 1;
            CK(gemm(s, bk, gc, st));
          }
        } else if (!pg) {
          CK(launch_pair_dbar<S>(dv, t, rb, ee, en, wc, dee, den, st));
        }
      }
    }
  }
  for (int l = L0 - 1; l >= 0; --l) {
    S* out = F_(B.finit, B.blk_f, l);
    CK(launch_tanh_bwd<S>(rows * D, fbar, out, zbar, st));
    const int Fd = (int)((M + 2) * K);
    if (l == 0) {
      if (pg) {
        CK(launch_wgrad(bk, wg((S*)(ws + B.x0), Fd, zbar, D, rows, Fd, (int)D, B, ws), gacc + O.initW[0], D,
                        gacc + O.initb[0], st));
      } else {
        // initial-feature cotangents x0bar = zbar W1^T, then the distances
        S* xb = (S*)(ws + B.x0bar);
        GemmArgs gx = dense(zbar, D, prm + O.initW[0], D, nullptr, xb, Fd, rows, (int)D, Fd, 1, 0, 0, 1);
        gx.transw = 1;
        CK(gemm(s, bk, gx, st));
        CK(launch_init_dbar<S>(dv, xb, ee, en, wc, dee, den, st));
      }
    } else {
      if (pg)
        CK(launch_wgrad(bk, wg(F_(B.finit, B.blk_f, l - 1), D, zbar, D, rows, (int)D, (int)D, B, ws),
                        gacc + O.initW[l], D, gacc + O.initb[l], st));
      GemmArgs gi = dense(zbar, D, prm + O.initW[l], D, nullptr, fbar2, D, rows, (int)D, (int)D, 1, 0, 0, 1);
      gi.transw = 1;
      CK(gemm(s, bk, gi, st));
      std::swap(fbar, fbar2);
    }
  }
  if (!pg) CK(launch_positions_bar(dv, ee, en, dee, den, lp, wc, rbar, st));
  return QMC_OK;
}

// log|psi| and its position gradient of one chunk by the value forward and one reverse pass
// (r: the chunk's positions; lp [wc] and grad [wc][N][3] outputs).
template <typename S>
static qmc_status grad_chunk(const Plan& P, const SysPlan& s, const S* prm, const double* r, int64_t wc,
                             const BwdWorkspace& B, char* ws, double* lp, double* grad, hipStream_t st) {
  const qmc_status e = forward_stash<S>(P, s, prm, r, wc, B, ws, st);
  if (e != QMC_OK) return e;
  const SysDev dv = make_dev(P, s);
  const ParamOffsets& O = s.off;
  S* jv = nullptr;
  if (P.ans.jastrow) {
    jv = (S*)(ws + B.jval);
    CK(launch_jastrow_out<S>(wc, 1, P.ans.width, (const S*)(ws + B.jhid), prm + O.jW2, prm + O.jb2, jv, st));
  }
  CK(launch_combine<S>(dv, prm + O.c, (double*)(ws + B.dld), (double*)(ws + B.dsg), nullptr, nullptr, nullptr,
                       (double*)(ws + B.geom), jv, wc, 0, lp, nullptr, nullptr, nullptr, nullptr, st));
  double* ones = (double*)(ws + B.ones);
  CK(launch_fill(wc, 1.0, ones, st));
  return backward_chunk<S>(P, s, prm, ones, wc, B, ws, st, grad, lp);
}

template <typename S>
static qmc_status run_logpsi_grad(const Plan& P, const void* params, const double* r, double* logpsi, double* grad,
                                  char* ws, hipStream_t st) {
  return for_systems(P, QMC_OP_LOGPSI_GRAD, ws, st, [&](size_t si, hipStream_t ss, char* wsb) -> qmc_status {
    const SysPlan& s = P.sys[si];
    const S* prm = (const S*)params + s.param_offset;
    const BwdWorkspace B0 = bwd_layout(P, s, s.Wc);
    const int64_t pos = pos_offset(P, s);
    for (int64_t w0 = 0; w0 < s.W; w0 += s.Wc) {
      const int64_t wc = std::min<int64_t>(s.Wc, s.W - w0);
      const qmc_status e = grad_chunk<S>(P, s, prm, r + pos + w0 * s.N * 3, wc, B0, wsb,
                                         logpsi + s.walker_offset + w0, grad + pos + w0 * s.N * 3, ss);
      if (e != QMC_OK) return e;
    }
    return QMC_OK;
  });
}

// One Langevin step: drift proposal, log|psi| and its gradient at the proposal by the reverse pass,
// Hastings acceptance.
template <typename S>
static qmc_status run_mala(const Plan& P, const void* params, double* r, double* logpsi, double* grad,
                           const double* noise, const double* u, double step, int damp, uint8_t* accepted, char* ws,
                           hipStream_t st) {
  return for_systems(P, QMC_OP_MALA, ws, st, [&](size_t si, hipStream_t ss, char* wsb) -> qmc_status {
    const SysPlan& s = P.sys[si];
    const SysDev dv = make_dev(P, s);
    const S* prm = (const S*)params + s.param_offset;
    const BwdWorkspace B0 = bwd_layout(P, s, s.Wc);
    const int64_t pos = pos_offset(P, s);
    for (int64_t w0 = 0; w0 < s.W; w0 += s.Wc) {
      const int64_t wc = std::min<int64_t>(s.Wc, s.W - w0);
      const int64_t wg = s.walker_offset + w0;
      double* rp = (double*)(wsb + B0.prop);
      double* gp = rp + wc * s.N * 3;
      double* lpp = gp + wc * s.N * 3;
      const int64_t off = pos + w0 * s.N * 3;
      CK(launch_propose_mala(dv, r + off, grad + off, noise + off, step, damp, wc, rp, ss));
      const qmc_status e = grad_chunk<S>(P, s, prm, rp, wc, B0, wsb, lpp, gp, ss);
      if (e != QMC_OK) return e;
      CK(launch_accept_mala(dv, wc, rp, gp, lpp, noise + off, u + wg, step, damp, r + off, grad + off, logpsi + wg,
                            accepted ? accepted + wg : nullptr, ss));
    }
    return QMC_OK;
  });
}

// cot: per-walker cotangent (VJP) or nullptr with e_loc given (loss gradient).
template <typename S>
static qmc_status run_backward(const Plan& P, const void* params, const double* r, const double* cot,
                               const double* e_loc, void* grad, double* e_mean, char* ws, hipStream_t st) {
  const int op = cot ? QMC_OP_LOGPSI_VJP : QMC_OP_LOSS_GRAD;
  return for_systems(P, op, ws, st, [&](size_t si, hipStream_t ss, char* wsb) -> qmc_status {
    const SysPlan& s = P.sys[si];
    const S* prm = (const S*)params + s.param_offset;
    const BwdWorkspace B0 = bwd_layout(P, s, s.Wc);
    double* gacc = (double*)(wsb + B0.gacc);
    CK(launch_fill(s.off.total, 0.0, gacc, ss));
    const double* gall;
    if (cot) {
      gall = cot + s.walker_offset;
    } else {
      double* gb = (double*)(wsb + B0.gbar);
      // the workspace header receives the system's count of finite local energies
      CK(launch_loss_weights(e_loc + s.walker_offset, s.W, (double*)(wsb + B0.stats), gb,
                             e_mean ? e_mean + si : nullptr, (int64_t*)ws + si, ss));
      gall = gb;
    }
    for (int64_t w0 = 0; w0 < s.W; w0 += s.Wc) {
      const int64_t wc = std::min<int64_t>(s.Wc, s.W - w0);
      // the layout depends only on the chunk size through sizes; keep the full-chunk offsets so
      // that gacc / gbar / stats stay at fixed places
      const qmc_status e1 = forward_stash<S>(P, s, prm, r + pos_offset(P, s) + w0 * s.N * 3, wc, B0, wsb, ss);
      if (e1 != QMC_OK) return e1;
      const qmc_status e2 = backward_chunk<S>(P, s, prm, gall + w0, wc, B0, wsb, ss);
      if (e2 != QMC_OK) return e2;
    }
    CK(launch_cast<S>(s.off.total, gacc, (S*)grad + s.param_offset, ss));
    return QMC_OK;
  });
}

// ---------------------------------------------------------------- plan device set-up

// Mean time of 3 launches after one warm-up launch (ms), or a negative value if the launch fails.
static float time_gemm(GemmKind kind, const GemmArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (launch_gemm(kind, a, st) != hipSuccess) return -1.f;
  if (hipEventRecord(e0, st) != hipSuccess) return -1.f;
  for (int i = 0; i < 3; ++i)
    if (launch_gemm(kind, a, st) != hipSuccess) return -1.f;
  float ms = 0.f;
  if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    return -1.f;
  return ms / 3.f;
}

// Times the tile candidates of every system's four GEMM classes on representative shapes (at most
// 2^20 rows each, zero operands) and keeps the fastest in SysPlan::tile.
static qmc_status autotune(Plan& P) {
  const size_t E = act_bytes(P.prec);
  const int64_t D = P.ans.width, cap = int64_t(1) << 20;
  const size_t xb = size_t(cap) * 2 * D * E, wb = size_t(3 * D) * D * E, yb = size_t(cap) * D * E;
  void *X = nullptr, *Wm = nullptr, *B = nullptr, *Y = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  qmc_status err = QMC_OK;
  if (hipMalloc(&X, xb) != hipSuccess || hipMalloc(&Wm, wb) != hipSuccess || hipMalloc(&B, D * E) != hipSuccess ||
      hipMalloc(&Y, yb) != hipSuccess || hipMemset(X, 0, xb) != hipSuccess || hipMemset(Wm, 0, wb) != hipSuccess ||
      hipMemset(B, 0, D * E) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    err = QMC_ERR_HIP;
  const bool f32 = P.prec == QMC_FP32 || P.prec == QMC_BF16_VALUE;
  // K-step (bit 0) and persistent grids (bit 2) are float32 options; the three-piece bf16 form (bit 3)
  // is a candidate at width 256 and above, where the matrix cores bound the wide products (at width 128
  // the products are bound elsewhere and the form gains nothing)
  const bool x3 = f32 && D >= 256;
  std::vector<int> jet_bits = f32 ? std::vector<int>{0, 1, 4, 5} : std::vector<int>{0};
  std::vector<int> row_bits = f32 ? std::vector<int>{0, 1, 2, 3, 4, 6} : std::vector<int>{0, 2};
  if (x3) {
    jet_bits.insert(jet_bits.end(), {8, 12});
    row_bits.insert(row_bits.end(), {8, 10, 12, 14});
  }
  for (auto& s : P.sys) {
    if (err != QMC_OK) break;
    const int64_t pmax = std::max<int64_t>(1, std::max(s.P[0], std::max(s.P[1], s.P[2])));
    for (int cls = 0; cls < 4 && err == QMC_OK; ++cls) {
      GemmArgs a = dense(X, D, Wm, D, B, Y, D, 1, (int)D, (int)D, 1, 0, 0, 1);
      if (cls == TILE_JET) {
        a = dense(X, 2 * D, Wm, D, B, Y, D, std::min(cap, s.Wc * s.N * s.Rp) / s.Rp * s.Rp, (int)(2 * D), (int)D,
                  s.Rp, s.T, 1, 0);
      } else if (cls == TILE_EDGE) {
        a = dense(X, D, Wm, D, B, Y, D, std::min(cap, s.Wc * pmax * 4) / 4 * 4, (int)D, (int)D, 4, 1, 1, 0);
      } else if (cls == TILE_VAL && fused_edges(P, true) && edge_mlp_supported(make_dev(P, s))) {
        // the value-row edge filters run fused: the node products dominate, the message product
        // (K = 3D) the most
        // (rows x 3D inputs within the 2D x cap buffer)
        a = dense(X, 3 * D, Wm, D, B, Y, D, std::min(cap * 2 / 3, s.Wc * s.N), (int)(3 * D), (int)D, 1, 0, 1, 1);
      } else {
        a = dense(X, D, Wm, D, B, Y, D, std::min(cap, s.Wc * pmax), (int)D, (int)D, 1, 0, 0, 1);
        a.transw = cls == TILE_BWD;
      }
      if (a.rows <= 0) continue;
      // the kind these shapes run in: jets and edge jets as the local energy, value rows as the
      // log|psi| forwards, the backward's data products in the backward kind
      const GemmKind gk = cls == TILE_BWD ? (P.prec == QMC_FP64 ? GK_F64 : GK_F32)
                                          : embed_kind(P.prec, cls == TILE_VAL);
      float best = 1e30f;
      int pick = 0;
      for (int bits : (cls == TILE_JET ? jet_bits : row_bits)) {
        a.tile = bits + 1;
        const float t = time_gemm(gk, a, st, e0, e1);
        if (t < 0.f) {
          err = QMC_ERR_HIP;
          break;
        }
        if (t < best) {
          best = t;
          pick = bits + 1;
        }
      }
      s.tile[cls] = pick;
    }
  }
  if (st) (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (X) (void)hipFree(X);
  if (Wm) (void)hipFree(Wm);
  if (B) (void)hipFree(B);
  if (Y) (void)hipFree(Y);
  return err;
}

qmc_status plan_device_init(Plan& P) {
  if (P.concurrent()) {
    hipEvent_t f = nullptr;
    if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess) return QMC_ERR_HIP;
    P.fork = f;
    for (size_t si = 0; si < P.sys.size(); ++si) {
      hipStream_t s = nullptr;
      hipEvent_t j = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return QMC_ERR_HIP;
      P.streams.push_back(s);
      if (hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) return QMC_ERR_HIP;
      P.joins.push_back(j);
    }
  }
  if (P.flags & QMC_PLAN_AUTOTUNE) return autotune(P);
  return QMC_OK;
}

void plan_device_release(Plan& P) {
  for (void* s : P.streams) (void)hipStreamDestroy((hipStream_t)s);
  for (void* e : P.joins) (void)hipEventDestroy((hipEvent_t)e);
  if (P.fork) (void)hipEventDestroy((hipEvent_t)P.fork);
  P.streams.clear();
  P.joins.clear();
  P.fork = nullptr;
}

// ---------------------------------------------------------------- local energy without allocation
//
// The workspace of qmc_local_energy_noalloc: one array per device, held by the loaded code object
// until the process ends.  In host code its name is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[QMC_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

// Device address of this device's scratch array (resolved on the first call on the device).
static qmc_status scratch_address(void** out) {
  int dev = 0;
  CK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return QMC_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return QMC_ERR_INTERNAL;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QMC_OK;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

qmc_status qmc_logpsi(const qmc_plan* plan, const void* params, const double* r, double* logpsi, double* sign,
                      void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !logpsi) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_LOGPSI, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_LOGPSI)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.logpsi = logpsi;
  o.sign = sign;
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64) return run_forward<double>(plan->p, params, r, o, 0, (char*)ws, st);
  return run_forward<float>(plan->p, params, r, o, 0, (char*)ws, st);
}

qmc_status qmc_local_energy(const qmc_plan* plan, const void* params, const double* r, double* logpsi, double* sign,
                            double* grad, double* lap, double* e_loc, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !e_loc) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_LOCAL_ENERGY, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_LOCAL_ENERGY)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  Outs o = {logpsi, sign, grad, lap, e_loc};
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64) return run_forward<double>(plan->p, params, r, o, 1, (char*)ws, st);
  return run_forward<float>(plan->p, params, r, o, 1, (char*)ws, st);
}

qmc_status qmc_local_energy_noalloc(const qmc_plan* plan, const void* params, const double* r, double* logpsi,
                                    double* sign, double* grad, double* lap, double* e_loc, void* stream) {
  if (!plan || !params || !r || !e_loc) return QMC_ERR_INVALID_ARGUMENT;
  const size_t need = workspace_bytes(plan->p, QMC_OP_LOCAL_ENERGY);
  if (need > size_t(QMC_NOALLOC_SCRATCH_BYTES)) {
    snprintf(g_last_error, sizeof(g_last_error),
             "qmc_local_energy_noalloc: the plan's local-energy workspace (%zu bytes) exceeds the %zu-byte scratch "
             "array; create the plan with a smaller max_chunk_walkers",
             need, size_t(QMC_NOALLOC_SCRATCH_BYTES));
    return QMC_ERR_WORKSPACE_TOO_SMALL;
  }
  void* ws = nullptr;
  const qmc_status e = scratch_address(&ws);
  if (e != QMC_OK) return e;
  Outs o = {logpsi, sign, grad, lap, e_loc};
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64) return run_forward<double>(plan->p, params, r, o, 1, (char*)ws, st);
  return run_forward<float>(plan->p, params, r, o, 1, (char*)ws, st);
}

qmc_status qmc_metropolis_step(const qmc_plan* plan, const void* params, double* r, double* logpsi,
                               const double* noise, const double* u, double step, uint8_t* accepted, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !logpsi || !noise || !u) return QMC_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(step) || step < 0) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_METROPOLIS, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_METROPOLIS)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64)
    return run_metropolis<double>(plan->p, params, r, logpsi, noise, u, step, accepted, (char*)ws, st);
  return run_metropolis<float>(plan->p, params, r, logpsi, noise, u, step, accepted, (char*)ws, st);
}

qmc_status qmc_logpsi_grad(const qmc_plan* plan, const void* params, const double* r, double* logpsi, double* grad,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !logpsi || !grad) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_LOGPSI_GRAD, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_LOGPSI_GRAD)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64) return run_logpsi_grad<double>(plan->p, params, r, logpsi, grad, (char*)ws, st);
  return run_logpsi_grad<float>(plan->p, params, r, logpsi, grad, (char*)ws, st);
}

qmc_status qmc_mala_step(const qmc_plan* plan, const void* params, double* r, double* logpsi, double* grad,
                         const double* noise, const double* u, double step, int32_t damp, uint8_t* accepted, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !logpsi || !grad || !noise || !u) return QMC_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(step) || step < 0 || (damp != 0 && damp != 1)) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_MALA, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_MALA)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64)
    return run_mala<double>(plan->p, params, r, logpsi, grad, noise, u, step, damp, accepted, (char*)ws, st);
  return run_mala<float>(plan->p, params, r, logpsi, grad, noise, u, step, damp, accepted, (char*)ws, st);
}

qmc_status qmc_logpsi_vjp(const qmc_plan* plan, const void* params, const double* r, const double* cotangent,
                          void* grad_params, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !cotangent || !grad_params) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_LOGPSI_VJP, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_LOGPSI_VJP)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64)
    return run_backward<double>(plan->p, params, r, cotangent, nullptr, grad_params, nullptr, (char*)ws, st);
  return run_backward<float>(plan->p, params, r, cotangent, nullptr, grad_params, nullptr, (char*)ws, st);
}

qmc_status qmc_loss_grad(const qmc_plan* plan, const void* params, const double* r, const double* e_loc,
                         void* grad_params, double* e_mean, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !params || !r || !e_loc || !grad_params) return QMC_ERR_INVALID_ARGUMENT;
  if (!ws_ok(plan->p, QMC_OP_LOSS_GRAD, ws, ws_bytes)) {
    if (ws && ws_bytes < workspace_bytes(plan->p, QMC_OP_LOSS_GRAD)) return QMC_ERR_WORKSPACE_TOO_SMALL;
    return QMC_ERR_INVALID_ARGUMENT;
  }
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.prec == QMC_FP64)
    return run_backward<double>(plan->p, params, r, nullptr, e_loc, grad_params, e_mean, (char*)ws, st);
  return run_backward<float>(plan->p, params, r, nullptr, e_loc, grad_params, e_mean, (char*)ws, st);
}

qmc_status qmc_det_jets(int64_t n_mat, int32_t n, int32_t n_tan, const double* jets, double* logdet, double* sign,
                        double* grad, double* lap, void* stream) {
  if (n_mat < 0 || n < 1 || n > 32 || n_tan < 0 || n_tan > 4096) return QMC_ERR_INVALID_ARGUMENT;
  if (n_mat == 0) return QMC_OK;
  if (!jets || !logdet || !sign || !lap || (n_tan > 0 && !grad)) return QMC_ERR_INVALID_ARGUMENT;
  CK(launch_det_generic(n_mat, n, n_tan, jets, logdet, sign, grad, lap, (hipStream_t)stream));
  return QMC_OK;
}

const char* qmc_last_error(void) { return g_last_error; }

qmc_status qmc_clip_local_energy(const qmc_plan* plan, const double* e_loc, double* e_out, double width, int32_t mode,
                                 void* stream) {
  if (!plan || !e_loc || !e_out || !std::isfinite(width) || width <= 0 || (mode != 0 && mode != 1))
    return QMC_ERR_INVALID_ARGUMENT;
  for (const auto& s : plan->p.sys)
    CK(launch_clip(e_loc + s.walker_offset, e_out + s.walker_offset, s.W, width, mode, (hipStream_t)stream));
  return QMC_OK;
}

qmc_status qmc_sgd_update(int32_t precision, void* params, const void* grad, int64_t n, double lr, void* stream) {
  if (n < 0 || (n > 0 && (!params || !grad)) || !std::isfinite(lr)) return QMC_ERR_INVALID_ARGUMENT;
  if (precision != QMC_FP64 && precision != QMC_FP32 && precision != QMC_BF16_MIXED && precision != QMC_BF16_VALUE)
    return QMC_ERR_INVALID_ARGUMENT;
  if (n == 0) return QMC_OK;
  if (precision == QMC_FP64)
    CK(launch_sgd<double>(n, lr, (const double*)grad, (double*)params, (hipStream_t)stream));
  else
    CK(launch_sgd<float>(n, lr, (const float*)grad, (float*)params, (hipStream_t)stream));
  return QMC_OK;
}

qmc_status qmc_measure_peaks(void* scratch, size_t scratch_bytes, double* peaks, void* stream) {
  if (!scratch || !peaks || scratch_bytes < (size_t(64) << 20) || scratch_bytes > (size_t(16) << 30) ||
      (reinterpret_cast<uintptr_t>(scratch) & 15) != 0)
    return QMC_ERR_INVALID_ARGUMENT;
  CK(measure_peaks(scratch, scratch_bytes, peaks, (hipStream_t)stream));
  return QMC_OK;
}

}  // extern "C"

extern "C" {

qmc_status qmc_profile_enable(int32_t on) {
  g_prof_on = on != 0;
  return QMC_OK;
}

qmc_status qmc_profile_report(char* buf, size_t len, int32_t reset) {
  if (!buf || len == 0) return QMC_ERR_INVALID_ARGUMENT;
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs = g_prof;
    if (reset) g_prof.clear();
  }
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<long> cnt;
  for (const auto& r : recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return QMC_ERR_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return QMC_ERR_HIP;
    size_t k = 0;
    for (; k < names.size(); ++k)
      if (names[k] == r.name) break;
    if (k == names.size()) {
      names.push_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[k] += t;
    cnt[k] += 1;
    if (reset) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
  std::string out;
  for (size_t k = 0; k < names.size(); ++k) {
    char line[256];
    snprintf(line, sizeof(line), "%s %ld %.6f\n", names[k].c_str(), cnt[k], ms[k]);
    out += line;
  }
  if (out.size() + 1 > len) return QMC_ERR_WORKSPACE_TOO_SMALL;
  memcpy(buf, out.c_str(), out.size() + 1);
  return QMC_OK;
}

}  // extern "C"
