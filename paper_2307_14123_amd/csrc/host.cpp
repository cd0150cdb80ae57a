// Host-side part of the qmc library: parameter layout, plan creation,
// argument validation and workspace sizing.  No HIP calls here (the device set-up of plans created
// with flags lives in the HIP part: plan_device_init), so that this
// translation unit can be exercised on a machine without a GPU.
#include <cmath>
#include <cstring>
#include <new>

#include "plan.h"

namespace qmc {

static int64_t take(int64_t& cur, int64_t n) {
  int64_t o = cur;
  cur += n;
  return o;
}

bool compute_offsets(const qmc_system& s, const qmc_ansatz& a, ParamOffsets* off) {
  const int64_t M = s.n_nuc, K = a.n_rbf, D = a.width;
  int64_t cur = 0;
  for (int l = 0; l < 8; ++l) off->initW[l] = off->initb[l] = -1;
  off->initW[0] = take(cur, (M + 2) * K * D);
  off->initb[0] = take(cur, D);
  for (int l = 1; l < a.init_layers; ++l) {
    off->initW[l] = take(cur, D * D);
    off->initb[l] = take(cur, D);
  }
  off->mp.assign(a.mp_layers, ParamOffsets::Layer{});
  for (int l = 0; l < a.mp_layers; ++l) {
    auto& L = off->mp[l];
    for (int t = 0; t < 3; ++t) {
      L.U1[t] = take(cur, K * D);
      L.a1[t] = take(cur, D);
      L.U2[t] = take(cur, D * D);
      L.a2[t] = take(cur, D);
      L.Ve[t] = L.ce[t] = -1;
      if (a.edge_update && l >= 1) {
        L.Ve[t] = take(cur, K * K);
        L.ce[t] = take(cur, K);
      }
    }
    L.Wh = take(cur, D * D);
    L.bh = take(cur, D);
    L.Y = take(cur, M * D);
    L.Wg = take(cur, 3 * D * D);
    L.bg = take(cur, D);
  }
  const int ns[2] = {s.n_up, s.n_down};
  for (int sp = 0; sp < 2; ++sp) {
    if (ns[sp] == 0) {
      off->orbW[sp] = off->orbb[sp] = off->pi[sp] = off->sigma[sp] = -1;
      continue;
    }
    const int64_t n = a.full_det ? int64_t(s.n_up) + s.n_down : ns[sp];  // orbitals per determinant
    off->orbW[sp] = take(cur, D * a.n_det * n);
    off->orbb[sp] = take(cur, a.n_det * n);
    off->pi[sp] = take(cur, a.n_det * n * M * a.n_env);
    off->sigma[sp] = take(cur, a.n_det * n * M * a.n_env);
  }
  off->c = take(cur, a.n_det);
  off->jW1 = off->jb1 = off->jW2 = off->jb2 = -1;
  if (a.jastrow) {
    off->jW1 = take(cur, D * D);
    off->jb1 = take(cur, D);
    off->jW2 = take(cur, D);
    off->jb2 = take(cur, 1);
  }
  off->total = cur;
  return true;
}

size_t act_bytes(qmc_precision p) { return p == QMC_FP64 ? 8 : 4; }

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Workspace workspace_layout(const Plan& p, const SysPlan& s, int op, int64_t wc) {
  Workspace w;
  std::memset(&w, 0, sizeof(w));
  size_t cur = 0;
  auto alloc = [&](size_t bytes) {
    size_t o = cur;
    cur = align256(cur + bytes);
    return o;
  };
  const bool jet = (op == QMC_OP_LOCAL_ENERGY);
  const size_t E = act_bytes(p.prec);
  const int64_t N = s.N, M = s.M, D = p.ans.width, K = p.ans.n_rbf, ND = p.ans.n_det;
  const int64_t Rp = jet ? s.Rp : 1, Rpe = jet ? 4 : 1;
  w.geom = alloc(size_t(wc) * (N * N + N * M) * 4 * 8);
  w.vpot = alloc(size_t(wc) * 8);
  for (int t = 0; t < 3; ++t) {
    w.rho[t] = alloc(size_t(wc) * s.P[t] * Rpe * K * E);
    w.rho2[t] = alloc(p.ans.edge_update ? size_t(wc) * s.P[t] * Rpe * K * E : 0);
    w.ehid[t] = alloc(size_t(wc) * s.P[t] * Rpe * D * E);
    w.wjet[t] = alloc(size_t(wc) * s.P[t] * Rpe * D * E);
  }
  w.x0 = alloc(size_t(wc) * N * Rp * (M + 2) * K * E);
  w.f = alloc(size_t(wc) * N * Rp * D * E);
  w.h = alloc(size_t(wc) * N * Rp * D * E);
  w.m = alloc(size_t(wc) * N * Rp * (jet ? 2 : 3) * D * E);
  w.mn5 = alloc(jet ? size_t(wc) * N * 5 * D * E : 0);
  w.zn5 = alloc(jet ? size_t(wc) * N * 5 * D * E : 0);
  const int64_t nsq = s.det_sq();
  for (int sp = 0; sp < 2; ++sp) w.phi[sp] = alloc(size_t(wc) * s.nsig(sp) * Rp * ND * s.norb(sp) * E);
  w.ajet = alloc(size_t(wc) * ND * Rp * nsq * E);
  w.dld = alloc(size_t(wc) * 2 * ND * 8);
  w.dsg = alloc(size_t(wc) * 2 * ND * 8);
  w.dg = alloc(size_t(wc) * 2 * ND * (jet ? s.T : 1) * 8);
  w.dlap = alloc(size_t(wc) * 2 * ND * 8);
  if (op == QMC_OP_METROPOLIS) {
    w.lp_prop = alloc(size_t(wc) * (N * 3 + 1) * 8);  // proposal [wc][N][3], then its log|psi| [wc]
  }
  w.jas = alloc(p.ans.jastrow ? size_t(wc) * Rp * E : 0);

  w.total = cur;
  return w;
}

BwdWorkspace bwd_layout(const Plan& p, const SysPlan& s, int64_t wc) {
  BwdWorkspace b;
  std::memset(&b, 0, sizeof(b));
  size_t cur = 0;
  auto alloc = [&](size_t bytes) {
    size_t o = cur;
    cur = align256(cur + bytes);
    return o;
  };
  const size_t E = act_bytes(p.prec);
  const int64_t N = s.N, M = s.M, D = p.ans.width, K = p.ans.n_rbf, ND = p.ans.n_det;
  const int64_t L = p.ans.mp_layers, L0 = p.ans.init_layers, F = (M + 2) * K;
  const int64_t nsq = s.det_sq();
  int64_t nmax = 0, pmax = 0;  // nmax: most orbitals per determinant of a spin map
  for (int sp = 0; sp < 2; ++sp)
    if (s.nsig(sp) > 0 && s.norb(sp) > nmax) nmax = s.norb(sp);
  for (int t = 0; t < 3; ++t)
    if (s.P[t] > pmax) pmax = s.P[t];
  b.geom = alloc(size_t(wc) * (N * N + N * M) * 4 * 8);
  for (int t = 0; t < 3; ++t) {
    b.blk_e[t] = int64_t(align256(size_t(wc) * s.P[t] * D * E));
    b.blk_r[t] = int64_t(align256(size_t(wc) * s.P[t] * K * E));
    b.rho[t] = alloc(size_t(b.blk_r[t]) * (p.ans.edge_update && L > 1 ? L : 1));
    b.ecarry[t] = alloc(p.ans.edge_update ? size_t(wc) * s.P[t] * K * E : 0);
    b.ehid[t] = alloc(size_t(b.blk_e[t]) * (L > 0 ? L : 1));
    b.wv[t] = alloc(size_t(b.blk_e[t]) * (L > 0 ? L : 1));
  }
  b.blk_f = int64_t(align256(size_t(wc) * N * D * E));
  b.blk_m = int64_t(align256(size_t(wc) * N * 3 * D * E));
  b.x0 = alloc(size_t(wc) * N * F * E);
  b.finit = alloc(size_t(b.blk_f) * L0);
  b.fst = alloc(size_t(b.blk_f) * (L > 0 ? L : 1));
  b.hst = alloc(size_t(b.blk_f) * (L > 0 ? L : 1));
  b.mst = alloc(size_t(b.blk_m) * (L > 0 ? L : 1));
  b.tst = alloc(size_t(b.blk_f) * (L > 0 ? L : 1));
  for (int sp = 0; sp < 2; ++sp) b.phi[sp] = alloc(size_t(wc) * s.nsig(sp) * ND * s.norb(sp) * E);
  b.aval = alloc(size_t(wc) * ND * nsq * E);
  b.dld = alloc(size_t(wc) * 2 * ND * 8);
  b.dsg = alloc(size_t(wc) * 2 * ND * 8);
  b.ainv = alloc(size_t(wc) * ND * nsq * 8);
  b.gbar = alloc(size_t(s.W) * 8);
  b.stats = alloc(2 * 8);
  b.lbar = alloc(size_t(wc) * ND * 8);
  b.cpart = alloc(size_t(wc) * ND * 8);
  for (int sp = 0; sp < 2; ++sp) b.phibar[sp] = alloc(size_t(wc) * s.nsig(sp) * ND * s.norb(sp) * E);
  b.pipart = alloc(size_t(wc) * ND * nmax * M * p.ans.n_env * 8);
  b.sgpart = alloc(size_t(wc) * ND * nmax * M * p.ans.n_env * 8);
  b.fbar = alloc(size_t(b.blk_f));
  b.fbar2 = alloc(size_t(b.blk_f));
  b.zbar = alloc(size_t(b.blk_f));
  b.hbar = alloc(size_t(b.blk_f));
  b.mbar = alloc(size_t(b.blk_m));
  for (int t = 0; t < 3; ++t) b.wbar[t] = alloc(size_t(wc) * s.P[t] * D * E);
  b.ebar = alloc(size_t(wc) * pmax * D * E);
  b.ypart = alloc(size_t(wc) * M * D * 8);
  b.rows_per_split = 1024;
  const int64_t rmax = wc * (N > pmax ? N : pmax);
  b.max_split = int((rmax + b.rows_per_split - 1) / b.rows_per_split);
  int64_t kin = 3 * D;
  if (F > kin) kin = F;
  int64_t nout = D;
  if (ND * nmax > nout) nout = ND * nmax;
  b.wpart_elems = int64_t(b.max_split) * (kin + 1) * nout;
  {
    // the same scratch serves the row sums: chunks of 64 walkers x one walker's columns
    const int64_t rs = ((wc + 63) / 64) * (ND * nmax * M * p.ans.n_env + M * D + ND);
    if (rs > b.wpart_elems) b.wpart_elems = rs;
  }
  b.wpart = alloc(size_t(b.wpart_elems) * 8);
  b.gacc = alloc(size_t(s.off.total) * 8);
  const size_t jb = p.ans.jastrow ? size_t(wc) * D * E : 0;
  b.jsum = alloc(jb);
  b.jhid = alloc(jb);
  b.jzb = alloc(jb);
  b.jfs = alloc(jb);
  b.jgo = alloc(p.ans.jastrow ? size_t(wc) * E : 0);
  b.dee = alloc(size_t(wc) * N * N * 8);
  b.den = alloc(size_t(wc) * N * M * 8);
  b.rhobar = alloc(size_t(wc) * pmax * K * E);
  b.x0bar = alloc(size_t(wc) * N * F * E);
  b.ones = alloc(size_t(wc) * 8);
  b.lpv = alloc(size_t(wc) * 8);
  b.jval = alloc(size_t(wc) * E);
  b.prop = alloc(size_t(wc) * (2 * N * 3 + 1) * 8);
  b.total = cur;
  return b;
}

static size_t sys_bytes(const Plan& p, int op, const SysPlan& s) {
  return (op == QMC_OP_LOGPSI_VJP || op == QMC_OP_LOSS_GRAD || op == QMC_OP_LOGPSI_GRAD || op == QMC_OP_MALA)
             ? bwd_layout(p, s, s.Wc).total
                                                              : workspace_layout(p, s, op, s.Wc).total;
}

size_t ws_header_bytes(const Plan& p, int op) {
  return op == QMC_OP_LOSS_GRAD ? align256(sizeof(int64_t) * p.sys.size()) : 0;
}

size_t sys_ws_offset(const Plan& p, int op, size_t si) {
  size_t off = ws_header_bytes(p, op);
  if (!p.concurrent()) return off;
  for (size_t k = 0; k < si; ++k) off += align256(sys_bytes(p, op, p.sys[k]));
  return off;
}

size_t workspace_bytes(const Plan& p, int op) {
  size_t mx = 0, sum = 0;
  for (const auto& s : p.sys) {
    const size_t b = sys_bytes(p, op, s);
    if (b > mx) mx = b;
    sum += align256(b);
  }
  return ws_header_bytes(p, op) + (p.concurrent() ? sum : mx) + 256;
}

static bool valid_system(const qmc_system* s) {
  if (!s || s->n_nuc < 1 || s->n_nuc > 64 || !s->charges || !s->coords) return false;
  if (s->n_up < 0 || s->n_down < 0 || s->n_up + s->n_down < 1) return false;
  if (s->n_up + s->n_down > 64) return false;
  for (int i = 0; i < s->n_nuc; ++i) {
    if (!(s->charges[i] > 0) || !std::isfinite(s->charges[i])) return false;
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(s->coords[3 * i + x])) return false;
  }
  return true;
}

static bool valid_ansatz(const qmc_ansatz* a) {
  if (!a || a->version != 1) return false;
  if (a->n_rbf < 2 || a->n_rbf > 64 || !(a->rbf_dmax > 0) || !std::isfinite(a->rbf_dmax)) return false;
  if (a->init_layers < 1 || a->init_layers > 8) return false;
  if (a->width < 1 || a->width > 1024) return false;
  if (a->mp_layers < 0 || a->mp_layers > 16) return false;
  if (a->n_det < 1 || a->n_det > 64 || a->n_env < 1 || a->n_env > 32) return false;
  if (a->include_vnn != 0 && a->include_vnn != 1) return false;
  if (!std::isfinite(a->ee_cusp) || a->ee_cusp < 0) return false;
  if (a->jastrow != 0 && a->jastrow != 1) return false;
  if (a->full_det != 0 && a->full_det != 1) return false;
  if (a->edge_update != 0 && a->edge_update != 1) return false;
  return true;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

int64_t qmc_param_count(const qmc_system* system, const qmc_ansatz* ansatz) {
  if (!valid_system(system) || !valid_ansatz(ansatz)) return -1;
  ParamOffsets off;
  compute_offsets(*system, *ansatz, &off);
  return off.total;
}

qmc_status qmc_plan_create(qmc_plan** out, const qmc_system* systems, int32_t n_systems,
                           const int64_t* walkers_per_system, const qmc_ansatz* ansatz,
                           qmc_precision precision, uint32_t flags) {
  return qmc_plan_create_ex(out, systems, n_systems, walkers_per_system, ansatz, precision, flags, 0);
}

qmc_status qmc_plan_create_ex(qmc_plan** out, const qmc_system* systems, int32_t n_systems,
                              const int64_t* walkers_per_system, const qmc_ansatz* ansatz,
                              qmc_precision precision, uint32_t flags, int64_t max_chunk_walkers) {
  if (!out) return QMC_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (max_chunk_walkers < 0) return QMC_ERR_INVALID_ARGUMENT;
  if (!systems || n_systems < 1 || n_systems > 4096 || !walkers_per_system) return QMC_ERR_INVALID_ARGUMENT;
  if (!valid_ansatz(ansatz)) return QMC_ERR_INVALID_ARGUMENT;
  if (precision != QMC_FP64 && precision != QMC_FP32 && precision != QMC_BF16_MIXED && precision != QMC_BF16_VALUE)
    return QMC_ERR_INVALID_ARGUMENT;
  if (flags & ~uint32_t(QMC_PLAN_CONCURRENT_SYSTEMS | QMC_PLAN_AUTOTUNE)) return QMC_ERR_INVALID_ARGUMENT;
  // the bf16 MFMA path works on K in steps of 32 and the jet GEMM tiles on 16-wide
  // column blocks; both handle any width, so no further restriction here.
  qmc_plan* plan = new (std::nothrow) qmc_plan;
  if (!plan) return QMC_ERR_INTERNAL;
  Plan& P = plan->p;
  P.ans = *ansatz;
  P.prec = precision;
  P.flags = flags;
  P.total_walkers = 0;
  P.total_params = 0;
  P.max_chunk_bytes = int64_t(24) << 30;
  for (int32_t k = 0; k < n_systems; ++k) {
    const qmc_system* s = &systems[k];
    if (!valid_system(s) || walkers_per_system[k] < 1 || walkers_per_system[k] > (int64_t(1) << 24)) {
      delete plan;
      return QMC_ERR_INVALID_ARGUMENT;
    }
    SysPlan sp;
    sp.M = s->n_nuc;
    sp.nup = s->n_up;
    sp.ndn = s->n_down;
    sp.N = s->n_up + s->n_down;
    sp.full_det = ansatz->full_det;
    if (sp.full_det && sp.N > 32) {  // the determinant kernels hold a matrix row per lane of a 32-lane group
      delete plan;
      return QMC_ERR_UNSUPPORTED;
    }
    sp.Z.assign(s->charges, s->charges + sp.M);
    sp.R.assign(s->coords, s->coords + 3 * sp.M);
    sp.vnn = 0;
    for (int I = 0; I < sp.M; ++I)
      for (int J = 0; J < I; ++J) {
        const double dx = sp.R[3 * I] - sp.R[3 * J], dy = sp.R[3 * I + 1] - sp.R[3 * J + 1],
                     dz = sp.R[3 * I + 2] - sp.R[3 * J + 2];
        const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
        if (!(d > 0)) {
          delete plan;
          return QMC_ERR_INVALID_ARGUMENT;  // coincident nuclei
        }
        sp.vnn += sp.Z[I] * sp.Z[J] / d;
      }
    sp.W = walkers_per_system[k];
    sp.walker_offset = P.total_walkers;
    sp.param_offset = P.total_params;
    compute_offsets(*s, *ansatz, &sp.off);
    sp.T = 3 * sp.N;
    sp.Rp = ((sp.T + 2) + 15) / 16 * 16;
    sp.P[TYPE_SAME] = sp.nup * (sp.nup - 1) / 2 + sp.ndn * (sp.ndn - 1) / 2;
    sp.P[TYPE_OPP] = sp.nup * sp.ndn;
    sp.P[TYPE_NUC] = sp.N * sp.M;
    sp.Wc = sp.W;
    for (int c = 0; c < 4; ++c) sp.tile[c] = 0;
    P.total_walkers += sp.W;
    P.total_params += sp.off.total;
    P.sys.push_back(sp);
  }
  // walker chunks: at most max_chunk_walkers (when given), and halved until the largest workspace
  // (local energy) fits max_chunk_bytes
  for (auto& sp : P.sys) {
    int64_t wc = sp.W;
    if (max_chunk_walkers > 0 && wc > max_chunk_walkers) wc = max_chunk_walkers;
    while (wc > 64 && workspace_layout(P, sp, QMC_OP_LOCAL_ENERGY, wc).total > size_t(P.max_chunk_bytes))
      wc = (wc + 1) / 2;
    sp.Wc = wc;
  }
  if (flags) {
    const qmc_status e = plan_device_init(P);
    if (e != QMC_OK) {
      plan_device_release(P);
      delete plan;
      return e;
    }
  }
  *out = plan;
  return QMC_OK;
}

qmc_status qmc_plan_destroy(qmc_plan* plan) {
  if (!plan) return QMC_ERR_INVALID_ARGUMENT;
  plan_device_release(plan->p);
  delete plan;
  return QMC_OK;
}

qmc_status qmc_plan_chunk_walkers(const qmc_plan* plan, int32_t s, int64_t* walkers) {
  if (!plan || !walkers || s < 0 || s >= (int32_t)plan->p.sys.size()) return QMC_ERR_INVALID_ARGUMENT;
  *walkers = plan->p.sys[s].Wc;
  return QMC_OK;
}

qmc_status qmc_plan_tiles(const qmc_plan* plan, int32_t s, int32_t tiles[4]) {
  if (!plan || !tiles || s < 0 || s >= (int32_t)plan->p.sys.size()) return QMC_ERR_INVALID_ARGUMENT;
  for (int c = 0; c < 4; ++c) tiles[c] = plan->p.sys[s].tile[c];
  return QMC_OK;
}

qmc_status qmc_workspace_size(const qmc_plan* plan, int32_t op, size_t* bytes) {
  if (!plan || !bytes || op < QMC_OP_LOGPSI || op > QMC_OP_LOGPSI_GRAD) return QMC_ERR_INVALID_ARGUMENT;
  *bytes = workspace_bytes(plan->p, op);
  return QMC_OK;
}

qmc_status qmc_plan_info(const qmc_plan* plan, int64_t* total_walkers, int64_t* total_params,
                         int64_t* total_positions) {
  if (!plan) return QMC_ERR_INVALID_ARGUMENT;
  int64_t pos = 0;
  for (const auto& s : plan->p.sys) pos += s.W * s.N * 3;
  if (total_walkers) *total_walkers = plan->p.total_walkers;
  if (total_params) *total_params = plan->p.total_params;
  if (total_positions) *total_positions = pos;
  return QMC_OK;
}

const char* qmc_status_str(qmc_status s) {
  switch (s) {
    case QMC_OK: return "QMC_OK";
    case QMC_ERR_INVALID_ARGUMENT: return "QMC_ERR_INVALID_ARGUMENT";
    case QMC_ERR_UNSUPPORTED: return "QMC_ERR_UNSUPPORTED";
    case QMC_ERR_WORKSPACE_TOO_SMALL: return "QMC_ERR_WORKSPACE_TOO_SMALL";
    case QMC_ERR_HIP: return "QMC_ERR_HIP";
    case QMC_ERR_INTERNAL: return "QMC_ERR_INTERNAL";
  }
  return "QMC_ERR_UNKNOWN";
}

}  // extern "C"
