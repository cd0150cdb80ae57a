// Internal plan structures of the qmc library (host side, no HIP types).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/qmc.h"

namespace qmc {

// Offsets (in elements, relative to the system's blob) of every tensor.
struct ParamOffsets {
  int64_t initW[8], initb[8];  // init layers 1..L0 (index l-1)
  struct Layer {
    int64_t U1[3], a1[3], U2[3], a2[3];  // edge filters: 0 same, 1 opp, 2 nuc
    int64_t Ve[3], ce[3];                // edge-feature update (layers after the first), -1 without
    int64_t Wh, bh, Y, Wg, bg;
  };
  std::vector<Layer> mp;
  int64_t orbW[2], orbb[2], pi[2], sigma[2];  // -1 when that spin block is empty
  int64_t c;
  int64_t jW1, jb1, jW2, jb2;  // learnable Jastrow MLP, -1 without it
  int64_t total;
};

enum { TYPE_SAME = 0, TYPE_OPP = 1, TYPE_NUC = 2 };

// Everything one system needs at launch time.
struct SysPlan {
  int M, N, nup, ndn;
  std::vector<double> Z, R;  // R: [M][3]
  double vnn;
  int64_t W;              // walkers of this system
  int64_t walker_offset;  // first walker in the concatenated walker arrays
  int64_t param_offset;   // first element of this system's blob
  ParamOffsets off;
  int T;                  // tangents 3N
  int Rp;                 // jet rows per electron, padded: roundup(3N + 2, 16)
  int P[3];               // pairs per edge type: same-spin (unordered), up-down, electron-nucleus
  int64_t Wc;             // walkers per launch sequence (chunk)
  int tile[4];            // GEMM tile choice per class (TILE_*): 0 default, else 1 + tile bits
  int full_det;
  int nsig(int s) const { return s == 0 ? nup : ndn; }
  // orbitals per determinant of spin s's orbital map, and the order of the determinants' matrices
  int norb(int s) const { return full_det ? N : nsig(s); }
  int64_t det_sq() const { return full_det ? int64_t(N) * N : int64_t(nup) * nup + int64_t(ndn) * ndn; }
};

enum { TILE_JET = 0, TILE_VAL = 1, TILE_EDGE = 2, TILE_BWD = 3 };

struct Plan {
  qmc_ansatz ans;
  qmc_precision prec;
  uint32_t flags;
  std::vector<SysPlan> sys;
  int64_t total_walkers;
  int64_t total_params;
  int64_t max_chunk_bytes;
  // QMC_PLAN_CONCURRENT_SYSTEMS: one stream per system, a fork event and one join event per system
  // (HIP handles, created and destroyed by plan_device_init / plan_device_release)
  std::vector<void*> streams, joins;
  void* fork = nullptr;
  bool concurrent() const { return (flags & QMC_PLAN_CONCURRENT_SYSTEMS) && sys.size() > 1; }
};

// Byte offsets of the buffers one chunk of one system uses (forward ops).
struct Workspace {
  size_t geom, vpot;
  size_t rho[3], ehid[3], wjet[3];
  size_t rho2[3];  // the updated edge features (with edge updates: ping-pong with rho)
  size_t x0, f, h, m, mn5, zn5;
  size_t phi[2], ajet;
  size_t dld, dsg, dg, dlap;
  size_t lp_prop;
  size_t jas;  // Jastrow exponent jets [wc][Rp] (value rows: [wc])
  size_t total;
};

// Buffers of the parameter backward: a value-only forward that keeps every
// layer's activations (stash), then the cotangents.  Per-layer arrays hold L
// consecutive blocks.
struct BwdWorkspace {
  // stash
  size_t geom, rho[3], ehid[3], wv[3], x0, finit, fst, hst, mst, tst, phi[2], aval, dld, dsg, ainv;
  int64_t blk_e[3], blk_f, blk_m;  // bytes of one layer block (edges per type, node rows, messages)
  // cotangents
  size_t gbar, stats, lbar, cpart, phibar[2], pipart, sgpart, fbar, fbar2, zbar, hbar, mbar, wbar[3], ebar, ypart;
  size_t wpart, gacc;
  size_t jsum, jhid, jzb, jfs, jgo;  // Jastrow: summed embeddings, hidden layer, their cotangents, J cotangent
  // position gradient: distance cotangents (e-e [N][N], e-n [N][M]), radial-basis and initial-feature
  // cotangents, the unit cotangent, log|psi|, the Jastrow value; Langevin proposals (positions,
  // their gradient, log|psi|)
  size_t dee, den, rhobar, x0bar, ones, lpv, jval, prop;
  size_t ecarry[3];      // with edge updates: cotangent of a layer's edge features from the next layer
  int64_t blk_r[3];      // bytes of one layer's edge features (rho holds every layer's with edge updates)
  int64_t wpart_elems;
  int64_t rows_per_split;
  int max_split;
  size_t total;
};

bool compute_offsets(const qmc_system& s, const qmc_ansatz& a, ParamOffsets* off);
size_t act_bytes(qmc_precision p);
// jet = true: value, 3N tangent and Laplacian rows; false: value rows only.
Workspace workspace_layout(const Plan& p, const SysPlan& s, int op, int64_t wc);
BwdWorkspace bwd_layout(const Plan& p, const SysPlan& s, int64_t wc);
size_t workspace_bytes(const Plan& p, int op);
// Bytes at the start of the workspace of op that hold documented outputs (the loss gradient's
// per-system count of finite local energies), before the systems' regions.
size_t ws_header_bytes(const Plan& p, int op);
// Byte offset of system si's workspace region: the header, plus the regions of the systems before si
// when the plan runs systems concurrently.
size_t sys_ws_offset(const Plan& p, int op, size_t si);
// Streams, events and autotuning of a plan created with flags (device code, in the HIP part).
qmc_status plan_device_init(Plan& p);
void plan_device_release(Plan& p);

}  // namespace qmc

struct qmc_plan {
  qmc::Plan p;
};
