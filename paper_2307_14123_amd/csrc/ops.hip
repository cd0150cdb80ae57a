// Element-wise and per-walker kernels of the local-energy path (gfx950).
//
// Jets: every activation carries rows (value, d/dx_c for the 3N electron
// coordinates c = 3j + a, Laplacian), padded to Rp rows.  Functions of one
// distance are propagated as univariate jets in the distance (value, first,
// second derivative) and expanded here with the chain rule:
//   e-e distance d_ij: grad_i d = u_ij, grad_j d = -u_ij, |grad d|^2 = 2, lap d = 4/d
//   e-n distance d_iI: grad_i d = u_iI,                  |grad d|^2 = 1, lap d = 2/d
// with u the unit vector of r_i - r_j (or r_i - R_I).
#include <cmath>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"
#include "pairs.h"

namespace qmc {

// pair helpers (radial basis, pair indexing) live in pairs.h

// ---------------------------------------------------------------- geometry

__global__ void geometry_kernel(SysDev s, const double* __restrict__ r, int64_t W, double* __restrict__ ee,
                                double* __restrict__ en) {
  const int NN = s.N + s.M;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * s.N * NN) return;
  const int64_t w = t / (s.N * NN);
  const int rem = (int)(t % (s.N * NN));
  const int i = rem / NN, jj = rem % NN;
  const double* ri = r + (w * s.N + i) * 3;
  double o[3];
  double* dst;
  if (jj < s.N) {
    const double* rj = r + (w * s.N + jj) * 3;
    for (int x = 0; x < 3; ++x) o[x] = ri[x] - rj[x];
    dst = ee + ((w * s.N + i) * s.N + jj) * 4;
  } else {
    const int I = jj - s.N;
    for (int x = 0; x < 3; ++x) o[x] = ri[x] - s.R[3 * I + x];
    dst = en + ((w * s.N + i) * s.M + I) * 4;
  }
  const double d = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
  const double inv = (jj == i) ? 0.0 : 1.0 / d;
  dst[0] = d;
  dst[1] = o[0] * inv;
  dst[2] = o[1] * inv;
  dst[3] = o[2] * inv;
}

// V = sum_{i<j} 1/d_ij - sum_{i,I} Z_I / d_iI + V_nn, one thread per walker
__global__ void potential_kernel(SysDev s, const double* __restrict__ r, int64_t W, double* __restrict__ vpot) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double* rw = r + w * s.N * 3;
  double v = 0.0;
  for (int i = 0; i < s.N; ++i) {
    const double x = rw[3 * i], y = rw[3 * i + 1], z = rw[3 * i + 2];
    for (int I = 0; I < s.M; ++I) {
      const double dx = x - s.R[3 * I], dy = y - s.R[3 * I + 1], dz = z - s.R[3 * I + 2];
      v -= s.Z[I] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    for (int j = 0; j < i; ++j) {
      const double dx = x - rw[3 * j], dy = y - rw[3 * j + 1], dz = z - rw[3 * j + 2];
      v += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  vpot[w] = v + s.vnn;
}

hipError_t launch_geometry(const SysDev& s, const double* r, int64_t W, double* ee, double* en, double* vpot,
                           hipStream_t st) {
  ProfScope ps("geometry_kernel", st);
  const int64_t n = W * s.N * (s.N + s.M);
  hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, r, W, ee, en);
  if (vpot)
    hipLaunchKernelGGL(potential_kernel, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s, r, W, vpot);
  return hipGetLastError();
}

// ---------------------------------------------------------------- radial basis jets per edge

template <typename S>
__global__ void rbf_kernel(SysDev s, int type, const double* __restrict__ ee, const double* __restrict__ en,
                           int64_t W, int jet, S* __restrict__ rho) {
  const int P = type == 0 ? s.P0 : (type == 1 ? s.P1 : s.P2);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * P * s.K) return;
  const int k = (int)(t % s.K);
  const int64_t wp = t / s.K;
  const int64_t w = wp / P;
  const int p = (int)(wp % P);
  int i, j;
  decode_pair(s, type, p, i, j);
  const double d = (type == 2) ? en[((w * s.N + i) * s.M + j) * 4] : ee[((w * s.N + i) * s.N + j) * 4];
  double r0, r1, r2;
  // value rows take the float32 exponential; jets, which carry the local energy, the float64 one
  if (jet)
    rbf3(d, k, rbf_spacing(s.dmax, s.K), (s.K - 1) / s.dmax, r0, r1, r2);
  else
    rbf3_as<S>(d, k, rbf_spacing(s.dmax, s.K), (s.K - 1) / s.dmax, r0, r1, r2);
  if (jet) {
    S* o = rho + wp * 4 * s.K + k;
    o[0] = (S)r0;
    o[s.K] = (S)r1;
    o[2 * s.K] = (S)r2;
    o[3 * s.K] = (S)0;
  } else {
    rho[wp * s.K + k] = (S)r0;
  }
}

template <typename S>
hipError_t launch_rbf(const SysDev& s, int type, const double* ee, const double* en, int64_t W, int jet, S* rho,
                      hipStream_t st) {
  const int P = type == 0 ? s.P0 : (type == 1 ? s.P1 : s.P2);
  const int64_t n = W * P * s.K;
  if (n == 0) return hipSuccess;
  ProfScope ps("rbf_kernel", st);
  hipLaunchKernelGGL(rbf_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, type, ee, en, W, jet,
                     rho);
  return hipGetLastError();
}

// ---------------------------------------------------------------- electron-node input features

// x_i = [rho(d_i1) .. rho(d_iM), mean_same rho(d_ij), mean_opp rho(d_ij)] with jets over all 3N coordinates
template <typename S>
__global__ void init_features_kernel(SysDev s, const double* __restrict__ ee, const double* __restrict__ en,
                                     int64_t W, int jet, S* __restrict__ x0) {
  const int F = (s.M + 2) * s.K;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * s.N * F) return;
  const int f = (int)(t % F);
  const int64_t wi = t / F;
  const int i = (int)(wi % s.N);
  const int64_t w = wi / s.N;
  const int Rp = jet ? s.Rp : 1;
  S* out = x0 + wi * Rp * F + f;
  const int K = s.K;
  if (f < s.M * K) {
    const int I = f / K, k = f % K;
    const double* g = en + ((w * s.N + i) * s.M + I) * 4;
    double r0, r1, r2;
    // value rows take the float32 exponential; jets, which carry the local energy, the float64 one
    if (jet)
      rbf3(g[0], k, rbf_spacing(s.dmax, K), (K - 1) / s.dmax, r0, r1, r2);
    else
      rbf3_as<S>(g[0], k, rbf_spacing(s.dmax, K), (K - 1) / s.dmax, r0, r1, r2);
    out[0] = (S)r0;
    if (!jet) return;
    for (int q = 1; q < Rp; ++q) {
      double v = 0.0;
      if (q <= s.T) {
        const int c = q - 1;
        if (c / 3 == i) v = r1 * g[1 + c % 3];
      } else if (q == s.T + 1) {
        v = r2 + 2.0 * r1 / g[0];
      }
      out[(int64_t)q * F] = (S)v;
    }
    return;
  }
  const int blk = (f - s.M * K) / K;  // 0 same, 1 opposite
  const int k = (f - s.M * K) % K;
  const bool up = i < s.nup;
  // members of the set: same spin (j != i) or opposite spin
  const bool same_set = (blk == 0);
  const int lo = (up == same_set) ? 0 : s.nup;
  const int hi = (up == same_set) ? s.nup : s.N;
  const int cnt = (hi - lo) - (same_set ? 1 : 0);
  const double inv = cnt > 0 ? 1.0 / cnt : 0.0;
  const double* eei = ee + (w * s.N + i) * s.N * 4;
  double val = 0.0, gs[3] = {0, 0, 0}, lap = 0.0;
  const double sp = rbf_spacing(s.dmax, K), isp = (K - 1) / s.dmax;
  if (!jet) {
    for (int j = lo; j < hi; ++j) {
      if (j == i) continue;
      double r0, r1, r2;
      rbf3_as<S>(eei[j * 4], k, sp, isp, r0, r1, r2);
      val += r0;
    }
    out[0] = (S)(val * inv);
    return;
  }
  for (int j = lo; j < hi; ++j) {
    if (j == i) continue;
    double r0, r1, r2;
    const double* g = eei + j * 4;
    rbf3(g[0], k, sp, isp, r0, r1, r2);
    val += r0;
    for (int a = 0; a < 3; ++a) gs[a] += r1 * g[1 + a];
    lap += 2.0 * r2 + 4.0 * r1 / g[0];
  }
  out[0] = (S)(val * inv);
  for (int q = 1; q < Rp; ++q) {
    double v = 0.0;
    if (q <= s.T && cnt > 0) {
      const int c = q - 1, j = c / 3, a = c % 3;
      if (j == i) {
        v = gs[a] * inv;
      } else if (j >= lo && j < hi) {
        const double* g = eei + j * 4;
        double r0, r1, r2;
        rbf3(g[0], k, sp, isp, r0, r1, r2);
        v = -r1 * g[1 + a] * inv;
      }
    } else if (q == s.T + 1) {
      v = lap * inv;
    }
    out[(int64_t)q * F] = (S)v;
  }
}

template <typename S>
hipError_t launch_init_features(const SysDev& s, const double* ee, const double* en, int64_t W, int jet, S* x0,
                                hipStream_t st) {
  ProfScope ps("init_features_kernel", st);
  const int64_t n = W * s.N * (s.M + 2) * s.K;
  hipLaunchKernelGGL(init_features_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, ee, en, W,
                     jet, x0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- message aggregation

// Electron messages with jets: m_i = [mean_{j same} w_same(d_ij) h_j, mean_{j opp} w_opp(d_ij) h_j]
// propagated with the product rule, written as [W][N][Rp][2D].  (The nuclear
// message is nonzero in 5 jet rows only and is handled by nuc_message_kernel.)
//
// Block: one walker, a chunk of DC columns and a part of its receiver groups
// (all of them unless DC columns x all groups exceed 512 threads: then the
// groups are split over `parts` adjacent blocks of gpb groups each, which read
// the same sender rows).  Thread: one column d and one group of up to RG
// receivers of the same spin.  The group's filter values
// w(d_ij) for every sender stay in registers in fixed sender slots (up
// electrons, then down electrons, NS slots each; empty slots hold weight 0 and
// read a valid row, so the sums have no branches), and same/opposite follows
// from the receivers' spin.  The senders' jet rows are read one row q at a
// time, the next row (and the operands of its moving-sender correction)
// fetched while the current one is used; every output row is written once.
// Tangent row c = 3k + a gets, besides sum_j w_ij dh_j/dx_c:
//   k == i:  sum_j h_j w'_ij u_ij[a]          (dd_ij/dr_i = u_ij)
//   k != i:  -h_k w'_ik u_ik[a]               (dd_ik/dr_k = -u_ik)
// and the Laplacian row adds sum_j h_j (2 w'' + 4 w'/d) + 2 sum_c dw/dx_c dh_j/dx_c.
// Everything that involves the receiver's own coordinates (its own tangent
// rows, the Laplacian row's h_j terms and the cross terms of its own rows) is
// gathered once before the row loop; the cross terms of the moving senders
// accumulate while the rows stream past.
template <typename S, int NS, int RG>
__global__ __launch_bounds__(512) void aggregate_kernel(SysDev s, const S* __restrict__ h,
                                                        const S* __restrict__ wsame, const S* __restrict__ wopp,
                                                        const double* __restrict__ ee, int DC, int nch, int parts,
                                                        int gpb, S* __restrict__ m) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int OPP = 1 << 30;
  const int N = s.N, D = s.D, Rp = s.Rp, T = s.T, nup = s.nup, ndn = s.ndn;
  const int64_t w = blockIdx.x / ((int64_t)nch * parts);
  const int cp = (int)(blockIdx.x - w * nch * parts), chunk = cp / parts, part = cp - chunk * parts;
  S* gu = (S*)smem;                  // [N][N][4]: d_ij, unit vector of r_i - r_j
  int* pt = (int*)(gu + N * N * 4);  // [N][N]: pair index within its type, | OPP for an up-down pair
  for (int e = threadIdx.x; e < N * N * 4; e += blockDim.x) gu[e] = (S)ee[w * N * N * 4 + e];
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e - (e / N) * N;
    int v = 0;
    if (i != j) {
      int type;
      const int p = ee_pair(s, i, j, type);
      v = type ? (p | OPP) : p;
    }
    pt[e] = v;
  }
  __syncthreads();
  const int dr = chunk * DC + (int)(threadIdx.x % DC), gl = threadIdx.x / DC, g = part * gpb + gl;
  const int ngu = (nup + RG - 1) / RG, ngd = (ndn + RG - 1) / RG;
  // threads past the last column or group compute nothing (cnt = 0) but meet the barriers
  const bool live = dr < D && gl < gpb && g < ngu + ngd;
  const int d = min(dr, D - 1);
  const bool up = g < ngu;
  const int i0 = up ? g * RG : nup + (g - ngu) * RG;
  const int cnt = live ? min(RG, (up ? nup : N) - i0) : 0;
  const int nsame = (up ? nup : ndn) - 1, nopp = up ? ndn : nup;
  const S inv_s = nsame > 0 ? S(1) / S(nsame) : S(0), inv_o = nopp > 0 ? S(1) / S(nopp) : S(0);
  // row r (0 value, 1 first, 2 second derivative) of the filter jet of pair (i, j), column d
  auto wrow = [&](int i, int j, int r) -> S {
    const int v = pt[i * N + j];
    return (v & OPP) ? wopp[((w * s.P1 + (v & (OPP - 1))) * 4 + r) * (int64_t)D + d]
                     : wsame[((w * s.P0 + v) * 4 + r) * (int64_t)D + d];
  };
  // sender of slot sl, clamped to a valid electron for empty slots (their weights are zero)
  auto sender = [&](int sl) { return sl < NS ? min(sl, N - 1) : min(nup + sl - NS, N - 1); };
  S wv[RG][2 * NS];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int sl = 0; sl < 2 * NS; ++sl) {
      const int j = sender(sl);
      const bool ok = r < cnt && (sl < NS ? sl < nup : sl - NS < ndn) && j != i0 + r;
      wv[r][sl] = ok ? wrow(i0 + r, j, 0) : S(0);
    }
  const S* hb = h + w * N * (int64_t)Rp * D + d;  // h_j row q: hb[(j * Rp + q) * D]
  S* mb = m + w * N * (int64_t)Rp * 2 * D + d;    // m_i row q: mb[(i * Rp + q) * 2D], opposite at + D
  // Terms that involve a receiver's own coordinates, gathered once per thread: the sender sums of
  // its own tangent rows (ts, to: same-spin, opposite-spin senders), and the Laplacian row's
  // sum_j h_j (2 w'' + 4 w'/d) plus the cross terms 2 w'_ij u_ij . dh_j/dr_i (in lxs, lxo; the
  // cross terms of the other electrons' rows are added while the rows stream past).
  S lxs[RG], lxo[RG], ts[RG][3], to[RG][3];
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    lxs[r] = lxo[r] = 0;
    ts[r][0] = ts[r][1] = ts[r][2] = to[r][0] = to[r][1] = to[r][2] = 0;
    if (r >= cnt) continue;
    const int i = i0 + r;
#pragma unroll 2
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      const S w1 = wrow(i, j, 1), w2 = wrow(i, j, 2), h0 = hb[(int64_t)j * Rp * D];
      const S* gij = gu + (i * N + j) * 4;
      S lx = h0 * (S(2) * w2 + S(4) * w1 / gij[0]), t[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const S cw = w1 * gij[1 + c];
        t[c] = h0 * cw;
        lx += S(2) * cw * hb[((int64_t)j * Rp + 1 + 3 * i + c) * D];
      }
      if ((j < nup) == up) {
        lxs[r] += lx;
        ts[r][0] += t[0];
        ts[r][1] += t[1];
        ts[r][2] += t[2];
      } else {
        lxo[r] += lx;
        to[r][0] += t[0];
        to[r][1] += t[1];
        to[r][2] += t[2];
      }
    }
  }
  S hv[2 * NS];
  auto fetch = [&](int q, S* dst) {
#pragma unroll
    for (int sl = 0; sl < 2 * NS; ++sl) dst[sl] = hb[((int64_t)sender(sl) * Rp + q) * D];
  };
  // operands of the moving-sender correction of a tangent row (sender kk): w'_ik of every receiver,
  // h_k value row and h_k row q
  S cwp[RG], ch0 = 0, chq = 0;
  auto fetch_corr = [&](int q, int kk, S* wp, S& h0, S& hq) {
#pragma unroll
    for (int r = 0; r < RG; ++r) wp[r] = (r < cnt && i0 + r != kk) ? wrow(i0 + r, kk, 1) : S(0);
    h0 = hb[(int64_t)kk * Rp * D];
    hq = hb[((int64_t)kk * Rp + q) * D];
  };
#pragma unroll
  for (int r = 0; r < RG; ++r) cwp[r] = 0;
  fetch(0, hv);
  int k = 0, a = 0;  // electron and coordinate of tangent row q (q >= 1)
  for (int q = 0; q <= T + 1; ++q) {
    S nv[2 * NS], nwp[RG], nh0 = 0, nhq = 0;
    if (q <= T) fetch(q + 1, nv);
    if (q + 1 <= T) fetch_corr(q + 1, q / 3, nwp, nh0, nhq);  // tangent row q + 1 moves electron q / 3
    S ms[RG], mo[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      S au = 0, ad = 0;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        au += wv[r][sl] * hv[sl];
        ad += wv[r][NS + sl] * hv[NS + sl];
      }
      ms[r] = up ? au : ad;
      mo[r] = up ? ad : au;
    }
    if (q >= 1 && q <= T) {
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        if (r >= cnt) continue;
        const int i = i0 + r;
        if (k == i) {
          // d(d_ij)/dr_i = u_ij for every sender j: gathered before the rows
          ms[r] += a == 0 ? ts[r][0] : (a == 1 ? ts[r][1] : ts[r][2]);
          mo[r] += a == 0 ? to[r][0] : (a == 1 ? to[r][1] : to[r][2]);
        } else {
          // d(d_ik)/dr_k = -u_ik: only sender k moves with this coordinate
          const S cw = cwp[r] * gu[(i * N + k) * 4 + 1 + a];
          const S t0 = -ch0 * cw;
          const S t1 = S(-2) * cw * chq;
          if ((k < nup) == up) {
            ms[r] += t0;
            lxs[r] += t1;
          } else {
            mo[r] += t0;
            lxo[r] += t1;
          }
        }
      }
      if (++a == 3) {
        a = 0;
        ++k;
      }
    } else if (q == T + 1) {
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        ms[r] += lxs[r];
        mo[r] += lxo[r];
      }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r)
      if (r < cnt) {
        S* o = mb + ((int64_t)(i0 + r) * Rp + q) * 2 * D;
        // streaming stores: the messages are not read again here, so they should not take L2 lines
        // from the sender rows that the other receiver groups of the block are about to read
        __builtin_nontemporal_store(ms[r] * inv_s, o);
        __builtin_nontemporal_store(mo[r] * inv_o, o + D);
      }
#pragma unroll
    for (int sl = 0; sl < 2 * NS; ++sl) hv[sl] = nv[sl];
#pragma unroll
    for (int r = 0; r < RG; ++r) cwp[r] = nwp[r];
    ch0 = nh0;
    chq = nhq;
    // the receiver groups of a block read the same sender rows: a barrier every 8 rows keeps them
    // close enough for the rows to be found in L2 by the later groups
    if ((q & 7) == 7) __syncthreads();
  }
  // padding rows
  for (int q = T + 2; q < Rp; ++q)
#pragma unroll
    for (int r = 0; r < RG; ++r)
      if (r < cnt) {
        S* o = mb + ((int64_t)(i0 + r) * Rp + q) * 2 * D;
        __builtin_nontemporal_store(S(0), o);
        __builtin_nontemporal_store(S(0), o + D);
      }
}

// The same messages for larger spin blocks (more than 8 electrons per spin):
// one receiver per thread would fetch every sender row once per receiver, so
// here the block stages RC rows of all senders (its column chunk) in LDS and
// every receiver thread reads them from there.  Filter values stay in
// registers in sender slots; the moving-sender correction of the next row is
// fetched one row ahead.
template <typename S, int NS, int RC>
__global__ __launch_bounds__(512) void aggregate_lds_kernel(SysDev s, const S* __restrict__ h,
                                                            const S* __restrict__ wsame, const S* __restrict__ wopp,
                                                            const double* __restrict__ ee, int DC, int nch,
                                                            S* __restrict__ m) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int OPP = 1 << 30;
  const int N = s.N, D = s.D, Rp = s.Rp, T = s.T, nup = s.nup, ndn = s.ndn;
  const int64_t w = blockIdx.x / nch;
  const int chunk = blockIdx.x - (int)(w * nch);
  const int c0 = chunk * DC;
  S* gu = (S*)smem;                     // [N][N][4]: d_ij, unit vector of r_i - r_j
  S* hs = gu + N * N * 4;               // [RC][2NS][DC]: rows q0.. of every sender slot (zero if empty)
  S* h0s = hs + RC * 2 * NS * DC;       // [2NS][DC]: value rows
  int* pt = (int*)(h0s + 2 * NS * DC);  // [N][N]: pair index within its type, | OPP for an up-down pair
  const int nt = blockDim.x;
  const S* hw = h + w * N * (int64_t)Rp * D;  // h_j row q: hw[(j * Rp + q) * D + d]
  auto sender = [&](int sl) { return sl < NS ? (sl < nup ? sl : -1) : (sl - NS < ndn ? nup + sl - NS : -1); };
  auto slot_of = [&](int j) { return j < nup ? j : NS + (j - nup); };
  for (int e = threadIdx.x; e < N * N * 4; e += nt) gu[e] = (S)ee[w * N * N * 4 + e];
  for (int e = threadIdx.x; e < N * N; e += nt) {
    const int i = e / N, j = e - (e / N) * N;
    int v = 0;
    if (i != j) {
      int type;
      const int p = ee_pair(s, i, j, type);
      v = type ? (p | OPP) : p;
    }
    pt[e] = v;
  }
  for (int e = threadIdx.x; e < 2 * NS * DC; e += nt) {
    const int sl = e / DC, x = e - (e / DC) * DC, j = sender(sl);
    h0s[e] = (j >= 0 && c0 + x < D) ? hw[(int64_t)j * Rp * D + c0 + x] : S(0);
  }
  __syncthreads();
  const int dd = threadIdx.x % DC, i = threadIdx.x / DC, d = min(c0 + dd, D - 1);
  const bool active = c0 + dd < D && i < N;  // idle threads still stage rows and meet the barriers
  const bool up = i < nup;
  const int nsame = (up ? nup : ndn) - 1, nopp = up ? ndn : nup;
  const S inv_s = nsame > 0 ? S(1) / S(nsame) : S(0), inv_o = nopp > 0 ? S(1) / S(nopp) : S(0);
  auto wrow = [&](int ii, int j, int r) -> S {
    const int v = pt[ii * N + j];
    return (v & OPP) ? wopp[((w * s.P1 + (v & (OPP - 1))) * 4 + r) * (int64_t)D + d]
                     : wsame[((w * s.P0 + v) * 4 + r) * (int64_t)D + d];
  };
  S wv[2 * NS];
#pragma unroll
  for (int sl = 0; sl < 2 * NS; ++sl) {
    const int j = sender(sl);
    wv[sl] = (active && j >= 0 && j != i) ? wrow(i, j, 0) : S(0);
  }
  S* mb = m + (w * N + min(i, N - 1)) * (int64_t)Rp * 2 * D + d;  // row q of receiver i: mb[q * 2D]
  // own-coordinate terms gathered once (as in aggregate_kernel)
  S lxs = 0, lxo = 0, ts[3] = {0, 0, 0}, to[3] = {0, 0, 0};
  if (active) {
#pragma unroll 2
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      const S w1 = wrow(i, j, 1), w2 = wrow(i, j, 2), h0 = h0s[slot_of(j) * DC + dd];
      const S* gij = gu + (i * N + j) * 4;
      S lx = h0 * (S(2) * w2 + S(4) * w1 / gij[0]), t[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const S cw = w1 * gij[1 + c];
        t[c] = h0 * cw;
        lx += S(2) * cw * hw[((int64_t)j * Rp + 1 + 3 * i + c) * D + d];
      }
      if ((j < nup) == up) {
        lxs += lx;
        ts[0] += t[0];
        ts[1] += t[1];
        ts[2] += t[2];
      } else {
        lxo += lx;
        to[0] += t[0];
        to[1] += t[1];
        to[2] += t[2];
      }
    }
  }
  S cwp = 0;  // w'_ik of the moving sender of the current tangent row
  int k = 0, a = 0;
  for (int q0 = 0; q0 <= T + 1; q0 += RC) {
    if (q0 > 0) __syncthreads();  // the previous rows are consumed
    for (int e = threadIdx.x; e < RC * 2 * NS * DC; e += nt) {
      const int x = e % DC, sq = e / DC, sl = sq % (2 * NS), qq = sq / (2 * NS), j = sender(sl);
      hs[e] = (j >= 0 && q0 + qq <= T + 1 && c0 + x < D) ? hw[((int64_t)j * Rp + q0 + qq) * D + c0 + x] : S(0);
    }
    __syncthreads();
    if (!active) continue;
    const int qe = min(RC, T + 2 - q0);
    for (int qq = 0; qq < qe; ++qq) {
      const int q = q0 + qq;
      // w'_ik for tangent row q + 1 (electron q / 3), fetched ahead
      const int kn = q / 3;
      const S nwp = (q + 1 <= T && kn != i) ? wrow(i, kn, 1) : S(0);
      const S* hq = hs + qq * 2 * NS * DC + dd;  // sender slot sl of row q: hq[sl * DC]
      S au = 0, ad = 0;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        au += wv[sl] * hq[sl * DC];
        ad += wv[NS + sl] * hq[(NS + sl) * DC];
      }
      S ms = up ? au : ad, mo = up ? ad : au;
      if (q >= 1 && q <= T) {
        if (k == i) {
          // d(d_ij)/dr_i = u_ij for every sender j: gathered before the rows
          ms += a == 0 ? ts[0] : (a == 1 ? ts[1] : ts[2]);
          mo += a == 0 ? to[0] : (a == 1 ? to[1] : to[2]);
        } else {
          // d(d_ik)/dr_k = -u_ik: only sender k moves with this coordinate
          const S cw = cwp * gu[(i * N + k) * 4 + 1 + a];
          const S t0 = -h0s[slot_of(k) * DC + dd] * cw;
          const S t1 = S(-2) * cw * hq[slot_of(k) * DC];
          if ((k < nup) == up) {
            ms += t0;
            lxs += t1;
          } else {
            mo += t0;
            lxo += t1;
          }
        }
        if (++a == 3) {
          a = 0;
          ++k;
        }
      } else if (q == T + 1) {
        ms += lxs;
        mo += lxo;
      }
      S* o = mb + (int64_t)q * 2 * D;
      o[0] = ms * inv_s;
      o[D] = mo * inv_o;
      cwp = nwp;
    }
  }
  if (active)
    for (int q = T + 2; q < Rp; ++q) {
      S* o = mb + (int64_t)q * 2 * D;
      o[0] = 0;
      o[D] = 0;
    }
}

// Nuclear messages with jets.  m_nuc_i = mean_I w_nuc(d_iI) Y_I depends on r_i
// only, so its jet is nonzero in 5 rows: value, the 3 coordinates of electron
// i, Laplacian (e-n distance: |grad d|^2 = 1, lap d = 2/d).  Output
// [W][N][5][D], one thread per (walker, electron, column).
template <typename S>
__global__ void nuc_message_kernel(SysDev s, const S* __restrict__ wnuc, const S* __restrict__ Y,
                                   const double* __restrict__ en, int64_t W, S* __restrict__ out) {
  const int N = s.N, D = s.D, M = s.M;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * N * D) return;
  const int d = (int)(t % D);
  const int64_t wi = t / D;
  S v = 0, g[3] = {0, 0, 0}, l = 0;
  for (int I = 0; I < M; ++I) {
    const S* wn = wnuc + ((wi * M + I) * 4) * (int64_t)D + d;  // pair (i, I) of walker w: index wi*M + I
    const double* ge = en + (wi * M + I) * 4;
    const S y = Y[I * D + d];
    v += wn[0] * y;
    for (int a = 0; a < 3; ++a) g[a] += wn[D] * (S)ge[1 + a] * y;
    l += (wn[2 * D] + S(2) * wn[D] / (S)ge[0]) * y;
  }
  const S invM = S(1) / S(M);
  S* o = out + wi * 5 * (int64_t)D + d;
  o[0] = v * invM;
  o[D] = g[0] * invM;
  o[2 * D] = g[1] * invM;
  o[3 * D] = g[2] * invM;
  o[4 * D] = l * invM;
}

template <typename S>
hipError_t launch_nuc_message(const SysDev& s, const S* wnuc, const S* Y, const double* en, int64_t W, S* out,
                              hipStream_t st) {
  const int64_t n = W * s.N * s.D;
  ProfScope ps("nuc_message_kernel", st);
  hipLaunchKernelGGL(nuc_message_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, wnuc, Y, en, W,
                     out);
  return hipGetLastError();
}

// Value rows only (log|psi| without derivatives).  Block: one walker, or for walkers of more than
// 2048 (receiver, column) outputs a chunk of 1024 of them, so that large walkers spread over several
// blocks (more loads in flight).  The senders' features are staged in LDS (when they fit) with a table of pair
// indices and types; each thread produces (receiver, column) outputs, so the filter values are
// read once per ordered pair with consecutive columns.
template <typename S>
__global__ __launch_bounds__(256) void aggregate_value_kernel(SysDev s, const S* __restrict__ h,
                                                              const S* __restrict__ wsame,
                                                              const S* __restrict__ wopp,
                                                              const S* __restrict__ wnuc,
                                                              const S* __restrict__ Y, int stage, int nck,
                                                              int cs, S* __restrict__ m) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = s.N, D = s.D, M = s.M;
  const int64_t w = blockIdx.x / nck;
  const int ck = (int)(blockIdx.x - w * nck);
  constexpr int OPP = 1 << 30;
  int* po = (int*)smem;               // [N][N]: pair index, | OPP for an up-down pair
  S* hs = (S*)(smem + ((N * N * sizeof(int) + 15) / 16) * 16);  // [N][D] when staged
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e - (e / N) * N;
    int v = 0;
    if (i != j) {
      int type;
      const int p = ee_pair(s, i, j, type);
      v = type ? (p | OPP) : p;
    }
    po[e] = v;
  }
  const S* hw = h + w * N * (int64_t)D;
  if (stage)
    for (int e = threadIdx.x; e < N * D; e += blockDim.x) hs[e] = hw[e];
  __syncthreads();
  const S* hsrc = stage ? hs : hw;
  const S* wsw = wsame + w * s.P0 * (int64_t)D;
  const S* wow = wopp + w * s.P1 * (int64_t)D;
  const S* wnw = wnuc + w * s.P2 * (int64_t)D;
  const int o_end = min(N * D, (ck + 1) * cs);
  for (int o = ck * cs + threadIdx.x; o < o_end; o += blockDim.x) {
    const int i = o / D, d = o - (o / D) * D;
    const bool up = i < s.nup;
    const int nsame = (up ? s.nup : s.ndn) - 1;
    const int nopp = up ? s.ndn : s.nup;
    // senders of each spin block in one branch-free loop (independent loads in flight)
    const int ls = up ? 0 : s.nup, hs_ = up ? s.nup : N, lo = up ? s.nup : 0, ho = up ? N : s.nup;
    S ms = 0, mo = 0;
#pragma unroll 4
    for (int j = ls; j < hs_; ++j) {
      const S wgt = j == i ? S(0) : wsw[(int64_t)po[i * N + j] * D + d];
      ms += wgt * hsrc[j * D + d];
    }
#pragma unroll 4
    for (int j = lo; j < ho; ++j) mo += wow[(int64_t)(po[i * N + j] & (OPP - 1)) * D + d] * hsrc[j * D + d];
    S nuc = 0;
    for (int I = 0; I < M; ++I) nuc += wnw[(int64_t)(i * M + I) * D + d] * Y[I * D + d];
    S* row = m + (w * N + i) * 3 * (int64_t)D + d;
    row[0] = nsame > 0 ? ms / S(nsame) : S(0);
    row[D] = nopp > 0 ? mo / S(nopp) : S(0);
    row[2 * D] = nuc / S(M);
  }
}

// Value messages for spin blocks of at most NS electrons: a thread per (walker, column) holds the
// walker's sender features and every receiver's two sums in registers and reads each unordered pair's
// filter once, adding it to both of its receivers (the pair order, a ascending and then b, gives each
// receiver its senders in ascending order, as aggregate_value_kernel sums them).  Each filter row is
// read from memory exactly once, with consecutive columns across the wavefront.
template <typename S, int NS>
__global__ __launch_bounds__(256) void aggregate_value_pairs_kernel(SysDev s, const S* __restrict__ h,
                                                                    const S* __restrict__ wsame,
                                                                    const S* __restrict__ wopp,
                                                                    const S* __restrict__ wnuc,
                                                                    const S* __restrict__ Y, int64_t W,
                                                                    S* __restrict__ m) {
  const int N = s.N, D = s.D, M = s.M, nup = s.nup, ndn = s.ndn;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = t / D;
  const int d = (int)(t - w * D);
  if (w >= W) return;
  // sender slots: up electrons 0..NS-1, down electrons NS..2NS-1 (zero past the block)
  S hv[2 * NS], ms[2 * NS], mo[2 * NS];
  const S* hw = h + w * N * (int64_t)D + d;
#pragma unroll
  for (int sl = 0; sl < 2 * NS; ++sl) {
    const bool ok = sl < NS ? sl < nup : sl - NS < ndn;
    const S r = hw[ok ? (int64_t)(sl < NS ? sl : nup + sl - NS) * D : 0];
    hv[sl] = ok ? r : S(0);
    ms[sl] = mo[sl] = S(0);
  }
  const S* ws = wsame + w * s.P0 * (int64_t)D + d;
  const S* wo = wopp + w * s.P1 * (int64_t)D + d;
  // Every slot pair issues its load (slot pairs outside the spin blocks read the walker's first
  // feature row instead and take a zero weight), so that the loads of a thread are independent of
  // branches and all in flight together.
  // same-spin pairs (a, b), a < b, of the up block, then of the down block (pair indices as ee_pair)
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = a + 1; b < NS; ++b) {
      const bool ok = b < nup;
      const S r = *(ok ? ws + (int64_t)(a * (2 * nup - a - 1) / 2 + (b - a - 1)) * D : hw);
      const S x = ok ? r : S(0);
      ms[a] += x * hv[b];
      ms[b] += x * hv[a];
    }
  const int dn0 = nup * (nup - 1) / 2;
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = a + 1; b < NS; ++b) {
      const bool ok = b < ndn;
      const S r = *(ok ? ws + (int64_t)(dn0 + a * (2 * ndn - a - 1) / 2 + (b - a - 1)) * D : hw);
      const S x = ok ? r : S(0);
      ms[NS + a] += x * hv[NS + b];
      ms[NS + b] += x * hv[NS + a];
    }
  // up-down pairs (a, b): index a * ndn + b
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) {
      const bool ok = a < nup && b < ndn;
      const S r = *(ok ? wo + (int64_t)(a * ndn + b) * D : hw);
      const S x = ok ? r : S(0);
      mo[a] += x * hv[NS + b];
      mo[NS + b] += x * hv[a];
    }
  const S* wn = wnuc + w * s.P2 * (int64_t)D + d;
#pragma unroll
  for (int sl = 0; sl < 2 * NS; ++sl) {
    const bool up = sl < NS;
    const int li = up ? sl : sl - NS;
    if (li >= (up ? nup : ndn)) continue;
    const int i = up ? li : nup + li;
    const int nsame = (up ? nup : ndn) - 1, nopp = up ? ndn : nup;
    S nuc = 0;
    for (int I = 0; I < M; ++I) nuc += wn[(int64_t)(i * M + I) * D] * Y[I * D + d];
    S* row = m + (w * N + i) * 3 * (int64_t)D + d;
    row[0] = nsame > 0 ? ms[sl] / S(nsame) : S(0);
    row[D] = nopp > 0 ? mo[sl] / S(nopp) : S(0);
    row[2 * D] = nuc / S(M);
  }
}

// Raises a kernel's dynamic-LDS limit above 64 KB, once per device (the attribute is a per-device
// setting; done[dev] keeps the largest size set so far).
static hipError_t allow_lds(const void* fn, size_t lds, size_t* done) {
  if (lds <= 64 * 1024) return hipSuccess;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidValue;
  // under one lock: callers on several host threads never lower a limit another has just raised
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (lds <= done[dev]) return hipSuccess;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return hipErrorInvalidValue;
  done[dev] = lds;
  return hipSuccess;
}

template <typename S, int NS>
static hipError_t agg_launch(const SysDev& s, const S* h, const S* ws, const S* wo, const double* ee, int64_t W, S* m,
                             hipStream_t st) {
  constexpr int RG = (NS <= 24 && sizeof(S) == 4) ? 2 : 1;  // receivers per thread (register budget)
  const int ngroups = (s.nup + RG - 1) / RG + (s.ndn + RG - 1) / RG;
  // columns per block: the largest power of two up to 64 with all groups in at most 512 threads, but
  // not below 32 (128-byte row segments per load): more groups go to `parts` blocks of gpb each
  int DC = 64;
  while (DC > 1 && (DC >= 2 * s.D || (DC > 32 && DC * ngroups > 512))) DC >>= 1;
  const int nch = (s.D + DC - 1) / DC;
  const size_t lds = (size_t)s.N * s.N * 4 * sizeof(S) + (size_t)s.N * s.N * sizeof(int);
  static size_t lds_set[64] = {};
  const hipError_t le = allow_lds((const void*)aggregate_kernel<S, NS, RG>, lds, lds_set);
  if (le != hipSuccess) return le;
  // receiver parts: the fewest that reach the most busy threads per compute unit (resident blocks x
  // threads with a group, on average over the parts), as the kernel's occupancy gives them for each
  // block size; every extra part re-reads the walker's sender rows (3 % per part)
  // (the choice depends only on the device and the shape: it is kept per (device, N, D, nup), so the
  // occupancy queries run on the first launch of a shape only)
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, int> chosen;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidValue;
  const auto key = std::make_tuple(dev, s.N, s.D, s.nup);
  int parts = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    const auto it = chosen.find(key);
    if (it != chosen.end()) parts = it->second;
  }
  if (parts == 0) {
    parts = 1;
    long best = -1;
    for (int p = 1; p <= 8 && p <= ngroups; ++p) {
      const int gp = (ngroups + p - 1) / p;
      if (DC * gp > 512) continue;
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, aggregate_kernel<S, NS, RG>, DC * gp, lds) != hipSuccess)
        occ = 1;
      const long busy = (long)std::max(occ, 1) * DC * ngroups * 100 / ((long)p * (100 + 3 * (p - 1)));
      if (busy > best) {
        best = busy;
        parts = p;
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    chosen[key] = parts;
  }
  const int gpb = (ngroups + parts - 1) / parts;
  ProfScope ps("aggregate_kernel", st);
  // blocks of one walker are adjacent, so they run together and share its rows in L2
  hipLaunchKernelGGL((aggregate_kernel<S, NS, RG>), dim3((unsigned)(W * nch * parts)), dim3(DC * gpb), lds, st, s, h,
                     ws, wo, ee, DC, nch, parts, gpb, m);
  return hipGetLastError();
}

template <typename S, int NS>
static hipError_t agg_lds_launch(const SysDev& s, const S* h, const S* ws, const S* wo, const double* ee, int64_t W,
                                 S* m, hipStream_t st) {
  constexpr int RC = 4;  // sender rows staged per step
  // columns per block: the largest power of two up to 64 with one thread per receiver in at most 512 threads
  int DC = 64;
  while (DC > 1 && (DC >= 2 * s.D || DC * s.N > 512)) DC >>= 1;
  const int nch = (s.D + DC - 1) / DC;
  const size_t lds = ((size_t)s.N * s.N * 4 + (size_t)RC * 2 * NS * DC + (size_t)2 * NS * DC) * sizeof(S) +
                     (size_t)s.N * s.N * sizeof(int);
  static size_t lds_set[64] = {};
  const hipError_t le = allow_lds((const void*)aggregate_lds_kernel<S, NS, RC>, lds, lds_set);
  if (le != hipSuccess) return le;
  ProfScope ps("aggregate_kernel", st);
  hipLaunchKernelGGL((aggregate_lds_kernel<S, NS, RC>), dim3((unsigned)(W * nch)), dim3(DC * s.N), lds, st, s, h,
                     ws, wo, ee, DC, nch, m);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_aggregate(const SysDev& s, const S* h, const S* wsame, const S* wopp, const S* wnuc, const S* Y,
                            const double* ee, const double* /*en: the nuclear messages need no geometry here*/,
                            int64_t W, int jet, S* m, hipStream_t st) {
  if (W <= 0) return hipSuccess;
  if (!jet) {
    const int nsp = std::max(s.nup, s.ndn);
    if (nsp <= 8) {
      const int64_t n = W * s.D;
      ProfScope ps("aggregate_value_kernel", st);
      if (nsp <= 4)
        hipLaunchKernelGGL((aggregate_value_pairs_kernel<S, 4>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s,
                           h, wsame, wopp, wnuc, Y, W, m);
      else
        hipLaunchKernelGGL((aggregate_value_pairs_kernel<S, 8>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s,
                           h, wsame, wopp, wnuc, Y, W, m);
      return hipGetLastError();
    }
    const size_t tab = ((size_t)s.N * s.N * sizeof(int) + 15) / 16 * 16;
    const size_t hb = (size_t)s.N * s.D * sizeof(S);
    const int stage = tab + hb <= 64 * 1024;
    const int cs = s.N * s.D > 2048 ? 1024 : s.N * s.D;  // outputs per block
    const int nck = (s.N * s.D + cs - 1) / cs;
    ProfScope ps("aggregate_value_kernel", st);
    hipLaunchKernelGGL(aggregate_value_kernel<S>, dim3((unsigned)(W * nck)), dim3(256), tab + (stage ? hb : 0), st, s,
                       h, wsame, wopp, wnuc, Y, stage, nck, cs, m);
    return hipGetLastError();
  }
  // template on the larger spin block
  const int ns = std::max(s.nup, s.ndn);
  if (ns <= 4) return agg_launch<S, 4>(s, h, wsame, wopp, ee, W, m, st);
  if (ns <= 8) return agg_launch<S, 8>(s, h, wsame, wopp, ee, W, m, st);
  // float32: the streaming kernel up to 32 electrons per spin (two receivers per thread up to 24,
  // one above); float64 above 8 electrons per spin stages the senders' rows in LDS (register budget)
  if constexpr (sizeof(S) == 4) {
    if (ns <= 12) return agg_launch<S, 12>(s, h, wsame, wopp, ee, W, m, st);
    if (ns <= 16) return agg_launch<S, 16>(s, h, wsame, wopp, ee, W, m, st);
  }
  if constexpr (sizeof(S) == 4) {
    if (ns <= 20) return agg_launch<S, 20>(s, h, wsame, wopp, ee, W, m, st);
    if (ns <= 24) return agg_launch<S, 24>(s, h, wsame, wopp, ee, W, m, st);
    if (ns <= 32) return agg_launch<S, 32>(s, h, wsame, wopp, ee, W, m, st);
  }
  if (ns <= 16) return agg_lds_launch<S, 16>(s, h, wsame, wopp, ee, W, m, st);
  if (ns <= 24) return agg_lds_launch<S, 24>(s, h, wsame, wopp, ee, W, m, st);
  if (ns <= 32) return agg_lds_launch<S, 32>(s, h, wsame, wopp, ee, W, m, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- orbitals x envelopes

// A[a][k] = phi_k(r_a) * sum_{I,beta} pi exp(-sigma d_aI), jets by the product rule.
// Output per walker: [spin][det][row][a][k] (this launch fills one spin block).
//
// One determinant per block; a thread per (walker, electron a, orbital k).  The
// envelope weights of the determinant go through LDS a chunk of nuclei at a time, laid out
// [nucleus][exponent][orbital] as (pi, sigma) pairs, so that the lanes of a wave (consecutive
// orbitals, then electrons) read consecutive or identical pairs.  For jets the exponentials of
// one nucleus are summed as s1 = sum sigma e and s2 = sum sigma^2 e before they meet the
// direction u of that nucleus: grad = -sum_I u_I s1_I, Laplacian term sum_I (s2_I - 2 s1_I / d_I).
template <typename S>
__global__ __launch_bounds__(256) void envelope_kernel(SysDev s, int spin, const S* __restrict__ phi,
                                                       const S* __restrict__ pi, const S* __restrict__ sg,
                                                       const double* __restrict__ en, int64_t W, int jet, int ic,
                                                       S* __restrict__ ajet) {
  // arithmetic in the plan's activation type (float64 only for the FP64 plan)
  using T = S;
  typedef S S2 __attribute__((ext_vector_type(2)));
  extern __shared__ __align__(16) unsigned char esm[];
  S2* tab = (S2*)esm;
  const int n = spin ? s.ndn : s.nup;
  const int i0 = spin ? s.nup : 0;
  const int Rp = jet ? s.Rp : 1;
  // n electrons (rows) of this spin, no orbitals (columns) per determinant, matrices of order dim
  // starting at row row0 (dim = no = n and row0 = 0 for spin-factorized determinants)
  const int no = orb_count(s, spin), dim = s.full_det ? s.N : n;
  const int row0 = det_row0(s, spin);
  const int nn = n * no, nb = s.nenv, M = s.M;
  // block b runs on XCD b % 8 (round-robin dispatch): the determinants of one chunk of
  // (walker, electron, orbital) triples are consecutive blocks of one XCD, so the orbital rows they
  // share (every determinant's columns side by side) are read from HBM once and then from that XCD's L2
  const int64_t nx = (W * nn + 255) / 256;
  const int64_t b = blockIdx.x, rr = b >> 3;
  const int p = (int)(rr % s.ndet);
  const int64_t xc = (rr / s.ndet) * 8 + (b & 7);
  if (xc >= nx) return;  // the whole block: before any barrier
  const int64_t t = xc * 256 + threadIdx.x;
  const bool live = t < W * nn;
  const int64_t w = live ? t / nn : 0;
  const int r = live ? (int)(t - w * nn) : 0;
  const int a = r / no, k = r - a * no;
  const int i = i0 + a;
  const double* g = en + (w * s.N + i) * M * 4;
  T e0 = 0, eg[3] = {0, 0, 0}, el = 0;
  for (int I0 = 0; I0 < M; I0 += ic) {
    const int ni = min(ic, M - I0);
    __syncthreads();  // the previous chunk has been read
    for (int e = threadIdx.x; e < no * ni * nb; e += 256) {
      const int kk = e / (ni * nb), j = e - kk * (ni * nb);
      const int64_t src = ((int64_t)(p * no + kk) * M + I0) * nb + j;
      tab[j * no + kk] = S2{pi[src], sg[src]};
    }
    __syncthreads();
    if (!live) continue;
    for (int I = 0; I < ni; ++I) {
      const T d = (T)g[(I0 + I) * 4];
      T s1 = 0, s2 = 0;
      for (int b = 0; b < nb; ++b) {
        const S2 ps = tab[(I * nb + b) * no + k];
        const T e = ps.x * exp(-ps.y * d);
        e0 += e;
        s1 += ps.y * e;
        s2 += ps.y * ps.y * e;
      }
      if (jet) {
        for (int x = 0; x < 3; ++x) eg[x] -= (T)g[(I0 + I) * 4 + 1 + x] * s1;
        el += s2 - T(2) * s1 / d;
      }
    }
  }
  if (!live) return;
  const int ncol = s.ndet * no;
  const S* ph = phi + ((w * n + a) * Rp) * (int64_t)ncol + p * no + k;
  const int d0 = det_dim(s, 0), d1 = det_dim(s, 1);
  const int64_t wstride = (int64_t)s.ndet * Rp * (d0 * d0 + d1 * d1);
  const int64_t soff = spin && !s.full_det ? (int64_t)s.ndet * Rp * d0 * d0 : 0;
  S* out = ajet + w * wstride + soff + ((int64_t)p * Rp * dim + row0 + a) * dim + k;
  const T p0 = ph[0];
  out[0] = (S)(p0 * e0);
  if (!jet) return;
  const int64_t rs = (int64_t)dim * dim;
  const int own = 1 + 3 * i;  // tangent rows of this electron's own coordinates
  for (int q = 1; q < Rp; ++q) {
    T v = 0;
    if (q <= s.T) {
      v = (T)ph[(int64_t)q * ncol] * e0;
      if (q >= own && q < own + 3) v += p0 * eg[q - own];
    } else if (q == s.T + 1) {
      v = (T)ph[(int64_t)q * ncol] * e0 + p0 * el;
      for (int x = 0; x < 3; ++x) v += T(2) * (T)ph[(int64_t)(own + x) * ncol] * eg[x];
    }
    out[q * rs] = (S)v;
  }
}

template <typename S>
hipError_t launch_envelope(const SysDev& s, int spin, const S* phi, const S* pi, const S* sigma, const double* en,
                           int64_t W, int jet, S* ajet, hipStream_t st) {
  const int n = spin ? s.ndn : s.nup;
  const int no = orb_count(s, spin);
  const int64_t cnt = W * n * no;
  if (cnt == 0) return hipSuccess;
  // nuclei per LDS chunk: at most 32 KB of (pi, sigma) pairs
  const size_t per = (size_t)no * s.nenv * 2 * sizeof(S);
  const int ic = (int)std::max<size_t>(1, std::min<size_t>(s.M, 32768 / per));
  const size_t lds = per * ic;
  const int64_t nx8 = ((cnt + 255) / 256 + 7) / 8 * 8;  // row chunks, rounded up to whole XCD rounds
  if (lds > 65536 || nx8 * s.ndet > INT32_MAX) return hipErrorInvalidValue;
  ProfScope ps(jet ? "envelope_kernel<jet>" : "envelope_kernel<val>", st);
  hipLaunchKernelGGL(envelope_kernel<S>, dim3((unsigned)(nx8 * s.ndet)), dim3(256), lds, st, s, spin, phi, pi, sigma,
                     en, W, jet, ic, ajet);
  return hipGetLastError();
}

// ---------------------------------------------------------------- determinants (float64)

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Determinants with G lanes per n x n problem (G = 8, 16 or 32, G >= n): lane r
// holds row r of A (and of the growing inverse) in registers, so the
// elimination needs no barrier: the pivot of each column is found with a
// butterfly over the group, and the pivot row reaches the other lanes by
// shuffles.  Rows are never swapped; a lane that has served as pivot for column
// c is marked used and, in Gauss-Jordan form, ends up holding row c of A^-1.
// log|det A| is the sum of log|pivot|, its sign the product of the pivot signs
// and of the permutation's sign (parity of its inversions).
//
// Jets: for every tangent t the rows of dA_t go through LDS, lane r forms row
// c(r) of X = A^-1 dA_t, d log|det| = tr X (group sum), and the Laplacian is
// tr(A^-1 lapA) - sum_t tr(X^2), the product of X's rows and columns taken
// through a second LDS tile.
constexpr int DMAX = 32;

template <int G>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

template <int G>
__device__ inline int group_sum_int(int v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename S, int G, bool INV>
__global__ __launch_bounds__(256) void det_kernel(const S* __restrict__ src, int64_t stride_outer, int n_inner,
                                                  int64_t stride_inner, int64_t nprob, int n, int ntan, int jet,
                                                  int64_t out_outer, int64_t out_off, double* __restrict__ ld,
                                                  double* __restrict__ sg, double* __restrict__ gout,
                                                  double* __restrict__ lapout, double* __restrict__ ainv) {
  extern __shared__ __align__(16) unsigned char dsm[];
  const int lane = threadIdx.x & 63;
  const int r = lane & (G - 1);
  const int base = lane - r;
  const int slot = threadIdx.x / G;  // problem slot in the block
  const int64_t pb = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const bool live = pb < nprob;
  const int64_t o = live ? pb / n_inner : 0;
  const int in = live ? (int)(pb % n_inner) : 0;
  const S* A = src + o * stride_outer + in * stride_inner;
  const int64_t oi = o * out_outer + out_off + in;
  const int nn = n * n;
  const bool row = live && r < n;

  double a[G], v[G];
#pragma unroll
  for (int c = 0; c < G; ++c) {
    a[c] = (row && c < n) ? (double)A[r * n + c] : 0.0;
    v[c] = (INV && row && c == r) ? 1.0 : 0.0;
  }
  bool used = !row;  // padding lanes never serve as pivot
  int cp = r;        // column this lane was pivot for
  double logdet = 0.0, sgn = 1.0;
  bool singular = false;
  // one elimination step for column col; every array index is a compile-time constant once the
  // loops over c are unrolled, so the rows stay in registers even where the loop over col is not
  // unrolled (32-lane groups)
  auto eliminate = [&](int col) {
    double acol = 0.0;
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c == col) acol = a[c];
    // pivot: largest |a[col]| over the unused rows (NaN counts as largest; smallest row on ties)
    double key = used ? -1.0 : (acol != acol ? INFINITY : fabs(acol));
    int idx = r;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const double ok = __shfl_xor(key, off);
      const int oid = __shfl_xor(idx, off);
      if (ok > key || (ok == key && oid < idx)) {
        key = ok;
        idx = oid;
      }
    }
    if (!(key > 0.0)) singular = true;
    const double pv = __shfl(acol, base + idx);
    const double pvs = key > 0.0 ? pv : 1.0;
    logdet += log(fabs(pv));
    if (pv < 0) sgn = -sgn;
    const double rinv = 1.0 / pvs;
    const bool me = r == idx;
    // Gauss-Jordan eliminates every other row, LU only the rows below (the unused ones); the pivot
    // row's entries arrive one column at a time, so no copy of the row is held
    const bool upd = !me && (INV || !used);
    const double f = acol * rinv;
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const double pc = __shfl(a[c], base + idx);
      if (c > col) {
        if (me) {
          if (INV) a[c] *= rinv;
        } else if (upd) {
          a[c] -= f * pc;
        }
      }
    }
    if (INV) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const double pc = __shfl(v[c], base + idx);
        v[c] = me ? v[c] * rinv : v[c] - f * pc;
      }
    }
    if (me) {
      used = true;
      cp = col;
    }
  };
  if constexpr (G <= 16) {
#pragma unroll
    for (int col = 0; col < G; ++col) {
      if (col >= n) break;
      // pivot: largest |a[col]| over the unused rows (NaN counts as largest; smallest row on ties)
      double key = used ? -1.0 : (a[col] != a[col] ? INFINITY : fabs(a[col]));
      int idx = r;
#pragma unroll
      for (int off = 1; off < G; off <<= 1) {
        const double ok = __shfl_xor(key, off);
        const int oid = __shfl_xor(idx, off);
        if (ok > key || (ok == key && oid < idx)) {
          key = ok;
          idx = oid;
        }
      }
      if (!(key > 0.0)) singular = true;
      const double pv = __shfl(a[col], base + idx);
      const double pvs = key > 0.0 ? pv : 1.0;
      logdet += log(fabs(pv));
      if (pv < 0) sgn = -sgn;
      const double rinv = 1.0 / pvs;
      const bool me = r == idx;
      double prow[G], pvrow[G];
#pragma unroll
      for (int c = col + 1; c < G; ++c) prow[c] = __shfl(a[c], base + idx);
      if (INV) {
#pragma unroll
        for (int c = 0; c < G; ++c) pvrow[c] = __shfl(v[c], base + idx);
      }
      if (me) {
        used = true;
        cp = col;
        if (INV) {
#pragma unroll
          for (int c = col + 1; c < G; ++c) a[c] *= rinv;
#pragma unroll
          for (int c = 0; c < G; ++c) v[c] *= rinv;
        }
      } else if (INV || !used) {
        // Gauss-Jordan eliminates every other row, LU only the rows below (the unused ones)
        const double f = a[col] * rinv;
#pragma unroll
        for (int c = col + 1; c < G; ++c) a[c] -= f * prow[c];
        if (INV) {
#pragma unroll
          for (int c = 0; c < G; ++c) v[c] -= f * pvrow[c];
        }
      }
    }
  } else {
    for (int col = 0; col < n; ++col) eliminate(col);
  }
  // sign of the permutation row -> column: parity of its inversions
  int inv_cnt = 0;
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const int cj = __shfl(cp, base + j);
    if (j > r && j < n && r < n && cj < cp) ++inv_cnt;
  }
  inv_cnt = group_sum_int<G>(inv_cnt);
  if (inv_cnt & 1) sgn = -sgn;
  if (live && r == 0) {
    ld[oi] = singular ? -INFINITY : logdet;
    sg[oi] = singular ? 0.0 : sgn;
  }
  if (!INV) return;
  if (ainv && row) {
    double* dst = ainv + pb * (int64_t)nn + (int64_t)cp * n;
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < n) dst[c] = singular ? 0.0 : v[c];
  }
  if (!jet) return;
  // LDS per problem slot: dA tile [n][G] (type S), X tile [n][n+1] (double)
  // dA tile: rows of G columns (zero beyond n, so the row reads are whole aligned vectors), slots
  // 4 elements apart beyond that (the groups of a wave read different slots)
  const int ld1 = n + 1, slot_stride = n * G + 4;
  S* dsl = (S*)dsm + (size_t)slot * slot_stride;
  double* xsl = (double*)(dsm + (((size_t)(blockDim.x / G) * slot_stride * sizeof(S) + 15) / 16) * 16) +
                (size_t)slot * n * ld1;
  double qacc = 0.0;
  S nxt[G];
#pragma unroll
  for (int c = 0; c < G; ++c) nxt[c] = (row && c < n && ntan > 0) ? A[(int64_t)nn + r * n + c] : S(0);
  for (int t = 0; t < ntan; ++t) {
    if (row) {
#pragma unroll
      for (int c = 0; c < G; ++c) dsl[r * G + c] = nxt[c];
    }
    if (t + 1 < ntan) {
      const S* q = A + (int64_t)(2 + t) * nn + r * n;
#pragma unroll
      for (int c = 0; c < G; ++c) nxt[c] = (row && c < n) ? q[c] : S(0);
    }
    __syncthreads();
    // row cp of X = A^-1 dA_t
    double x[G];
#pragma unroll
    for (int b = 0; b < G; ++b) x[b] = 0.0;
    if (row) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (k >= n) break;
        const double vk = v[k];
#pragma unroll
        for (int b = 0; b < G; ++b) x[b] += vk * (double)dsl[k * G + b];
      }
#pragma unroll
      for (int b = 0; b < G; ++b)
        if (b < n) xsl[cp * ld1 + b] = x[b];
    }
    double dg = 0.0;
#pragma unroll
    for (int b = 0; b < G; ++b)
      if (b == cp) dg = x[b];
    dg = group_sum<G>(row ? dg : 0.0);
    if (live && r == 0) gout[oi * ntan + t] = singular ? 0.0 : dg;
    __syncthreads();
    if (row) {
#pragma unroll
      for (int b = 0; b < G; ++b)
        if (b < n) qacc += x[b] * xsl[b * ld1 + cp];
    }
  }
  // tr(A^-1 lapA): row cp of A^-1 against column cp of lapA
  double tr = 0.0;
  if (row) {
    const S* lsrc = A + (int64_t)(1 + ntan) * nn;
#pragma unroll
    for (int b = 0; b < G; ++b)
      if (b < n) tr += v[b] * (double)lsrc[b * n + cp];
  }
  const double lap = group_sum<G>(tr - qacc);
  if (live && r == 0) lapout[oi] = singular ? 0.0 : lap;
}

static int det_group(int n) { return n <= 8 ? 8 : (n <= 16 ? 16 : 32); }

// Launches the variant for n; LDS: the dA and X tiles of every problem slot (jets only).
template <typename S>
static hipError_t det_dispatch(const S* src, int64_t stride_outer, int n_inner, int64_t stride_inner, int64_t nprob,
                               int n, int ntan, int jet, int64_t out_outer, int64_t out_off, double* ld, double* sg,
                               double* g, double* lap, double* ainv, hipStream_t st) {
  if (n < 1 || n > DMAX) return hipErrorInvalidValue;
  if (nprob <= 0) return hipSuccess;
  const int G = det_group(n);
  const int threads = G == 8 ? 256 : (G == 16 ? 128 : 64);
  const int slots = threads / G;
  const int64_t blocks = (nprob + slots - 1) / slots;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const bool inv = jet || ainv;
  const size_t lds = jet ? ((size_t)slots * (n * G + 4) * sizeof(S) + 15) / 16 * 16 + (size_t)slots * n * (n + 1) * 8
                         : 0;
#define QMC_DET(GG, II)                                                                                       \
  hipLaunchKernelGGL((det_kernel<S, GG, II>), dim3((unsigned)blocks), dim3(threads), lds, st, src, stride_outer, \
                     n_inner, stride_inner, nprob, n, ntan, jet, out_outer, out_off, ld, sg, g, lap, ainv)
  if (G == 8) {
    if (inv) QMC_DET(8, true); else QMC_DET(8, false);
  } else if (G == 16) {
    if (inv) QMC_DET(16, true); else QMC_DET(16, false);
  } else {
    if (inv) QMC_DET(32, true); else QMC_DET(32, false);
  }
#undef QMC_DET
  return hipGetLastError();
}

template <typename S>
hipError_t launch_det(const SysDev& s, const S* ajet, int64_t W, int jet, double* ld, double* sg, double* g,
                      double* lap, double* ainv, hipStream_t st) {
  const int Rp = jet ? s.Rp : 1;
  const int d0 = det_dim(s, 0);
  const int64_t wstride = (int64_t)s.ndet * Rp * (d0 * d0 + det_dim(s, 1) * det_dim(s, 1));
  for (int spin = 0; spin < 2; ++spin) {
    const int n = det_dim(s, spin);
    if (n == 0) continue;
    if (n > DMAX) return hipErrorInvalidValue;
    const int64_t soff = spin ? (int64_t)s.ndet * Rp * d0 * d0 : 0;
    ProfScope ps(jet ? "det_kernel<jet>" : "det_kernel<val>", st);
    const hipError_t e =
        det_dispatch<S>(ajet + soff, wstride, s.ndet, (int64_t)Rp * n * n, W * s.ndet, n, s.T, jet,
                        (int64_t)2 * s.ndet, (int64_t)spin * s.ndet, ld, sg, g, lap,
                        ainv ? ainv + (spin ? (int64_t)W * s.ndet * d0 * d0 : 0) : nullptr, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_det_generic(int64_t nmat, int n, int ntan, const double* jets, double* ld, double* sg, double* g,
                              double* lap, hipStream_t st) {
  if (n < 1 || n > DMAX) return hipErrorInvalidValue;
  return det_dispatch<double>(jets, (int64_t)(ntan + 2) * n * n, 1, (int64_t)0, nmat, n, ntan, 1, (int64_t)1,
                              (int64_t)0, ld, sg, g, lap, nullptr, st);
}

// ---------------------------------------------------------------- combination and local energy

// psi = sum_p c_p det_p^up det_p^down in the log domain; with weights
// w_p = c_p D_p / psi: grad log|psi| = sum_p w_p grad l_p,
// Delta psi / psi = sum_p w_p (Delta l_p + |grad l_p|^2),
// E_loc = -1/2 Delta psi / psi + V.  One wavefront per walker.
// With the electron-electron cusp factor exp(gamma), gamma = sum_{i<j} -c_ij a^2 / (a + r_ij),
// log|psi| gains gamma, grad gains grad gamma, and Delta psi / psi gains
// Delta gamma + 2 grad l . grad gamma + |grad gamma|^2 (l the determinant part), with
// gamma' = c a^2 / (a + r)^2, gamma'' = -2 c a^2 / (a + r)^3, grad_i gamma = sum_j gamma'(r_ij) u_ij
// and Delta gamma = sum_{i<j} 2 (gamma'' + 2 gamma' / r_ij).
template <typename S>
__global__ __launch_bounds__(64) void combine_kernel(SysDev s, const S* __restrict__ c, const double* __restrict__ ld,
                                                     const double* __restrict__ sg, const double* __restrict__ g,
                                                     const double* __restrict__ dlap, const double* __restrict__ vpot,
                                                     const double* __restrict__ ee, const S* __restrict__ jas,
                                                     int jet, double* __restrict__ logpsi,
                                                     double* __restrict__ sign,
                                                     double* __restrict__ grad, double* __restrict__ lap,
                                                     double* __restrict__ eloc) {
  const int64_t w = blockIdx.x;
  const int lane = threadIdx.x;
  const int nd = s.ndet;
  const bool has[2] = {det_dim(s, 0) > 0, det_dim(s, 1) > 0};
  double mx = -INFINITY;
  for (int p = 0; p < nd; ++p) {
    double l = 0.0;
    for (int sp = 0; sp < 2; ++sp)
      if (has[sp]) l += ld[(w * 2 + sp) * nd + p];
    if (l > mx) mx = l;
  }
  if (!(mx > -INFINITY)) mx = 0.0;
  double S_ = 0.0;
  for (int p = 0; p < nd; ++p) {
    double l = 0.0, sgn = (double)c[p];
    for (int sp = 0; sp < 2; ++sp)
      if (has[sp]) {
        l += ld[(w * 2 + sp) * nd + p];
        sgn *= sg[(w * 2 + sp) * nd + p];
      }
    if (sgn != 0.0) S_ += sgn * exp(l - mx);
  }
  const double sgnpsi = S_ > 0 ? 1.0 : (S_ < 0 ? -1.0 : 0.0);
  // electron-electron cusp factor: its value and Laplacian over the pairs i < j
  const int N = s.N;
  const bool cusp = s.ee_cusp > 0.0 && N > 1;
  const double ca2 = s.ee_cusp * s.ee_cusp;
  const double* eew = ee + w * (int64_t)N * N * 4;  // [N][N][4]: r_ij, unit vector of r_i - r_j
  double gam = 0.0, glap = 0.0;
  if (cusp) {
    for (int e = lane; e < N * N; e += 64) {
      const int i = e / N, j = e - (e / N) * N;
      if (j <= i) continue;
      const double d = eew[4 * e];
      const double cij = ((i < s.nup) == (j < s.nup)) ? 0.25 : 0.5;
      const double q = 1.0 / (s.ee_cusp + d);
      gam -= cij * ca2 * q;
      const double g1 = cij * ca2 * q * q, g2 = -2.0 * g1 * q;
      glap += 2.0 * (g2 + 2.0 * g1 / d);
    }
    gam = wave_sum(gam);
    glap = wave_sum(glap);
  }
  // learnable Jastrow exponent: jet rows [Rp] per walker (value rows: one)
  const S* jw = jas ? jas + w * (int64_t)(jet ? s.Rp : 1) : nullptr;
  if (jw) {
    gam += (double)jw[0];
    if (jet) glap += (double)jw[s.T + 1];
  }
  const double lp = mx + log(fabs(S_)) + gam;
  if (lane == 0) {
    if (logpsi) logpsi[w] = lp;
    if (sign) sign[w] = sgnpsi;
  }
  if (!jet) return;
  const double invS = 1.0 / S_;
  double Apart = 0.0, Bpart = 0.0, Cpart = 0.0;
  for (int cc = lane; cc < s.T; cc += 64) {
    double gc = 0.0, a2 = 0.0;
    for (int p = 0; p < nd; ++p) {
      double l = 0.0, sgn = (double)c[p], gp = 0.0;
      for (int sp = 0; sp < 2; ++sp)
        if (has[sp]) {
          const int64_t o = (w * 2 + sp) * nd + p;
          l += ld[o];
          sgn *= sg[o];
          gp += g[o * s.T + cc];
        }
      const double wp = sgn != 0.0 ? sgn * exp(l - mx) * invS : 0.0;
      gc += wp * gp;
      a2 += wp * gp * gp;
    }
    Apart += a2;
    Bpart += gc * gc;
    if (cusp || jw) {
      // d gamma / d x_cc: the pairs of electron i = cc / 3, coordinate cc % 3, and the Jastrow row
      double dg = jw ? (double)jw[1 + cc] : 0.0;
      if (cusp) {
        const int i = cc / 3, a = cc - 3 * (cc / 3);
        for (int j = 0; j < N; ++j) {
          if (j == i) continue;
          const double* pij = eew + 4 * (i * N + j);
          const double cij = ((i < s.nup) == (j < s.nup)) ? 0.25 : 0.5;
          const double q = 1.0 / (s.ee_cusp + pij[0]);
          dg += cij * ca2 * q * q * pij[1 + a];
        }
      }
      Cpart += 2.0 * gc * dg + dg * dg;
      gc += dg;
    }
    if (grad) grad[w * s.T + cc] = sgnpsi != 0.0 ? gc : NAN;
  }
  const double A = wave_sum(Apart), B = wave_sum(Bpart), C = wave_sum(Cpart);
  if (lane == 0) {
    double lsum = 0.0;
    for (int p = 0; p < nd; ++p) {
      double l = 0.0, sgn = (double)c[p], dl = 0.0;
      for (int sp = 0; sp < 2; ++sp)
        if (has[sp]) {
          const int64_t o = (w * 2 + sp) * nd + p;
          l += ld[o];
          sgn *= sg[o];
          dl += dlap[o];
        }
      if (sgn != 0.0) lsum += sgn * exp(l - mx) * invS * dl;
    }
    const double ok = sgnpsi != 0.0 ? 1.0 : NAN;
    if (lap) lap[w] = ok * (lsum + A - B + glap);
    // an undefined local energy (psi = 0, or a coincident pair where the potential is singular) is NaN
    const double e = ok * (-0.5 * (lsum + A + glap + C) + vpot[w]);
    if (eloc) eloc[w] = isfinite(e) ? e : NAN;
  }
}

template <typename S>
hipError_t launch_combine(const SysDev& s, const S* c, const double* ld, const double* sg, const double* g,
                          const double* dlap, const double* vpot, const double* ee, const S* jas, int64_t W, int jet,
                          double* logpsi, double* sign, double* grad, double* lap, double* eloc, hipStream_t st) {
  ProfScope ps("combine_kernel", st);
  hipLaunchKernelGGL(combine_kernel<S>, dim3((unsigned)W), dim3(64), 0, st, s, c, ld, sg, g, dlap, vpot, ee, jas,
                     jet, logpsi, sign, grad, lap, eloc);
  return hipGetLastError();
}

// ---------------------------------------------------------------- learnable Jastrow factor

template <typename S>
__global__ void sum_electrons_kernel(int64_t W, int N, int R, int D, const S* __restrict__ f, S* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)R * D;
  if (t >= W * per) return;
  const int64_t w = t / per, qd = t - w * per;
  const S* src = f + w * N * per + qd;
  S acc = 0;
  for (int i = 0; i < N; ++i) acc += src[i * per];
  out[t] = acc;
}

// one wavefront per row: lanes stride the D columns, then a butterfly sum
template <typename S>
__global__ __launch_bounds__(256) void jastrow_out_kernel(int64_t rows, int R, int D, const S* __restrict__ x,
                                                          const S* __restrict__ W2, const S* __restrict__ b2,
                                                          S* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const S* xr = x + row * D;
  float acc32 = 0.0f;
  double acc64 = 0.0;
  for (int d = lane; d < D; d += 64) {
    if constexpr (sizeof(S) == 8)
      acc64 += (double)xr[d] * (double)W2[d];
    else
      acc32 += (float)xr[d] * (float)W2[d];
  }
  double v = sizeof(S) == 8 ? acc64 : (double)acc32;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) out[row] = (S)(v + (row % R == 0 ? (double)b2[0] : 0.0));
}

template <typename S>
__global__ void jastrow_bwd_kernel(int64_t W, int D, const double* __restrict__ gbar, const S* __restrict__ W2,
                                   const S* __restrict__ h, S* __restrict__ zb, S* __restrict__ go) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * D) return;
  const int64_t w = t / D;
  const int d = (int)(t - w * D);
  const double g = gbar[w];
  const double hv = (double)h[t];
  zb[t] = (S)(g * (double)W2[d] * (1.0 - hv * hv));
  if (d == 0) go[w] = (S)g;
}

template <typename S>
__global__ void add_bcast_kernel(int64_t W, int N, int D, const S* __restrict__ fs, S* __restrict__ fbar) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * N * D) return;
  const int64_t w = t / ((int64_t)N * D);
  const int d = (int)(t % D);
  fbar[t] += fs[w * D + d];
}

template <typename S>
hipError_t launch_sum_electrons(int64_t W, int N, int R, int D, const S* f, S* out, hipStream_t st) {
  const int64_t n = W * R * D;
  if (n == 0) return hipSuccess;
  ProfScope ps("jastrow_sum_kernel", st);
  hipLaunchKernelGGL(sum_electrons_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, N, R, D, f,
                     out);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_jastrow_out(int64_t rows, int R, int D, const S* x, const S* W2, const S* b2, S* out,
                              hipStream_t st) {
  if (rows == 0) return hipSuccess;
  ProfScope ps("jastrow_out_kernel", st);
  hipLaunchKernelGGL(jastrow_out_kernel<S>, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, rows, R, D, x, W2,
                     b2, out);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_jastrow_bwd(int64_t W, int D, const double* gbar, const S* W2, const S* h, S* zb, S* go,
                              hipStream_t st) {
  const int64_t n = W * D;
  if (n == 0) return hipSuccess;
  ProfScope ps("jastrow_bwd_kernel", st);
  hipLaunchKernelGGL(jastrow_bwd_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, D, gbar, W2, h,
                     zb, go);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_add_bcast(int64_t W, int N, int D, const S* fs, S* fbar, hipStream_t st) {
  const int64_t n = W * N * D;
  if (n == 0) return hipSuccess;
  ProfScope ps("jastrow_bcast_kernel", st);
  hipLaunchKernelGGL(add_bcast_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, N, D, fs, fbar);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Metropolis

__global__ void propose_kernel(const double* __restrict__ r, const double* __restrict__ noise, double step, int64_t n,
                               double* __restrict__ rp) {
  // product and sum rounded separately (no fused multiply-add), so the
  // proposal is the same float64 value a host computes as r + (step * noise)
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) rp[t] = r[t] + step * noise[t];
}

__global__ void accept_kernel(int64_t W, int N3, const double* __restrict__ rp, const double* __restrict__ lpp,
                              const double* __restrict__ u, double* __restrict__ r, double* __restrict__ logpsi,
                              uint8_t* __restrict__ accepted) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const bool acc = log(u[w]) < 2.0 * (lpp[w] - logpsi[w]);
  if (acc) {
    for (int x = 0; x < N3; ++x) r[w * N3 + x] = rp[w * N3 + x];
    logpsi[w] = lpp[w];
  }
  if (accepted) accepted[w] = acc ? 1 : 0;
}

// ---------------------------------------------------------------- Langevin (MALA)

// Drift of one electron at x with gradient v = grad_i log|psi| and time step tau: v itself, or
// with damping v * 2 / (1 + sqrt(1 + 2 a |v|^2 tau)), a = 1/2 + (Z d)^2 / (10 (4 + (Z d)^2)) for
// the nearest nucleus (lowest index on ties), scaled so that the drift step tau |v| stays <= d.
__device__ inline void langevin_drift(const SysDev& s, const double* x, const double* v, double tau, int damp,
                                      double D[3]) {
#pragma clang fp contract(off)
  D[0] = v[0];
  D[1] = v[1];
  D[2] = v[2];
  if (!damp) return;
  double d = INFINITY, Z = 0.0;
  for (int I = 0; I < s.M; ++I) {
    const double a0 = x[0] - s.R[3 * I], a1 = x[1] - s.R[3 * I + 1], a2 = x[2] - s.R[3 * I + 2];
    const double dI = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
    if (dI < d) {
      d = dI;
      Z = s.Z[I];
    }
  }
  const double zd = Z * d, zd2 = zd * zd;
  const double a = 0.5 + zd2 / (10.0 * (4.0 + zd2));
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double f = 2.0 / (1.0 + sqrt(1.0 + 2.0 * a * v2 * tau));
  for (int c = 0; c < 3; ++c) D[c] = v[c] * f;
  const double len = tau * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
  if (len > d) {
    const double cap = d / len;
    for (int c = 0; c < 3; ++c) D[c] = D[c] * cap;
  }
}

// r' = (r + tau D(r)) + step * xi, tau = step^2, one thread per electron.
__global__ void propose_mala_kernel(SysDev s, const double* __restrict__ r, const double* __restrict__ g,
                                    const double* __restrict__ noise, double step, int damp, int64_t n,
                                    double* __restrict__ rp) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double tau = step * step;
  double x[3], v[3], D[3];
  for (int c = 0; c < 3; ++c) {
    x[c] = r[3 * t + c];
    v[c] = g[3 * t + c];
  }
  langevin_drift(s, x, v, tau, damp, D);
  for (int c = 0; c < 3; ++c) rp[3 * t + c] = (x[c] + tau * D[c]) + step * noise[3 * t + c];
}

// Hastings acceptance, one thread per walker:
//   log a = 2 (l' - l) + |xi|^2 / 2 - |xi + step (D(r) + D(r'))|^2 / 2, accepted iff log u < log a.
__global__ void accept_mala_kernel(SysDev s, int64_t W, const double* __restrict__ rp, const double* __restrict__ gp,
                                   const double* __restrict__ lpp, const double* __restrict__ noise,
                                   const double* __restrict__ u, double step, int damp, double* __restrict__ r,
                                   double* __restrict__ g, double* __restrict__ logpsi,
                                   uint8_t* __restrict__ accepted) {
#pragma clang fp contract(off)
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double tau = step * step;
  const int64_t base = w * s.N * 3;
  double fwd = 0.0, back = 0.0;
  for (int i = 0; i < s.N; ++i) {
    const int64_t o = base + 3 * i;
    double D0[3], D1[3];
    langevin_drift(s, r + o, g + o, tau, damp, D0);
    langevin_drift(s, rp + o, gp + o, tau, damp, D1);
    for (int c = 0; c < 3; ++c) {
      const double xi = noise[o + c];
      const double b = xi + step * (D0[c] + D1[c]);
      fwd += xi * xi;
      back += b * b;
    }
  }
  const double la = 2.0 * (lpp[w] - logpsi[w]) + 0.5 * fwd - 0.5 * back;
  const bool acc = log(u[w]) < la;
  if (acc) {
    for (int x = 0; x < 3 * s.N; ++x) {
      r[base + x] = rp[base + x];
      g[base + x] = gp[base + x];
    }
    logpsi[w] = lpp[w];
  }
  if (accepted) accepted[w] = acc ? 1 : 0;
}

hipError_t launch_propose_mala(const SysDev& s, const double* r, const double* g, const double* noise, double step,
                               int damp, int64_t W, double* rp, hipStream_t st) {
  ProfScope ps("propose_mala_kernel", st);
  const int64_t n = W * s.N;
  hipLaunchKernelGGL(propose_mala_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, r, g, noise, step,
                     damp, n, rp);
  return hipGetLastError();
}

hipError_t launch_accept_mala(const SysDev& s, int64_t W, const double* rp, const double* gp, const double* lpp,
                              const double* noise, const double* u, double step, int damp, double* r, double* g,
                              double* logpsi, uint8_t* accepted, hipStream_t st) {
  ProfScope ps("accept_mala_kernel", st);
  hipLaunchKernelGGL(accept_mala_kernel, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s, W, rp, gp, lpp,
                     noise, u, step, damp, r, g, logpsi, accepted);
  return hipGetLastError();
}

hipError_t launch_propose(const double* r, const double* noise, double step, int64_t n, double* rp, hipStream_t st) {
  ProfScope ps("propose_kernel", st);
  hipLaunchKernelGGL(propose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, r, noise, step, n, rp);
  return hipGetLastError();
}

hipError_t launch_accept(int64_t W, int N3, const double* rp, const double* lp_prop, const double* u, double* r,
                         double* logpsi, uint8_t* accepted, hipStream_t st) {
  ProfScope ps("accept_kernel", st);
  hipLaunchKernelGGL(accept_kernel, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, W, N3, rp, lp_prop, u, r,
                     logpsi, accepted);
  return hipGetLastError();
}

// explicit instantiations
#define QMC_INST(S)                                                                                             \
  template hipError_t launch_rbf<S>(const SysDev&, int, const double*, const double*, int64_t, int, S*,         \
                                    hipStream_t);                                                               \
  template hipError_t launch_init_features<S>(const SysDev&, const double*, const double*, int64_t, int, S*,    \
                                              hipStream_t);                                                     \
  template hipError_t launch_aggregate<S>(const SysDev&, const S*, const S*, const S*, const S*, const S*,      \
                                          const double*, const double*, int64_t, int, S*, hipStream_t);         \
  template hipError_t launch_nuc_message<S>(const SysDev&, const S*, const S*, const double*, int64_t, S*,      \
                                            hipStream_t);                                                       \
  template hipError_t launch_envelope<S>(const SysDev&, int, const S*, const S*, const S*, const double*,       \
                                         int64_t, int, S*, hipStream_t);                                        \
  template hipError_t launch_det<S>(const SysDev&, const S*, int64_t, int, double*, double*, double*, double*, \
                                    double*, hipStream_t);                                                             \
  template hipError_t launch_combine<S>(const SysDev&, const S*, const double*, const double*, const double*,    \
                                        const double*, const double*, const double*, const S*, int64_t, int,    \
                                        double*, double*, double*, double*, double*, hipStream_t);              \
  template hipError_t launch_sum_electrons<S>(int64_t, int, int, int, const S*, S*, hipStream_t);               \
  template hipError_t launch_jastrow_out<S>(int64_t, int, int, const S*, const S*, const S*, S*, hipStream_t);  \
  template hipError_t launch_jastrow_bwd<S>(int64_t, int, const double*, const S*, const S*, S*, S*,            \
                                            hipStream_t);                                                        \
  template hipError_t launch_add_bcast<S>(int64_t, int, int, const S*, S*, hipStream_t);
QMC_INST(double)
QMC_INST(float)

}  // namespace qmc
