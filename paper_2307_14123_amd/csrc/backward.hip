// Backward (vector-Jacobian product of log|psi| with respect to the
// parameters) and the loss-gradient helpers, gfx950.
//
// With cotangent g_w on log|psi_w|: through the log-sum-exp over determinants
// (Sec. III.E) each determinant log gets g_w * w_p with w_p = c_p D_p / psi,
// and c_p gets g_w D_p / psi; d log|det A| / dA = A^-T (Jacobi's formula), so
// the orbital matrix cotangent is g_w w_p A^-T; A = phi * env splits into
// phi_bar = A_bar * env and env_bar = A_bar * phi; linear layers give
// W_bar = x^T y_bar, b_bar = sum y_bar, x_bar = y_bar W^T; tanh gives
// z_bar = t_bar (1 - t^2).  Parameter gradients are sums over walkers and
// electrons: they are formed as split-row MFMA reductions whose partial sums
// are added in float64 in a fixed order (deterministic).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "kernels.h"
#include "pairs.h"

namespace qmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- weight gradients

// part[split][m][n] = sum over this split's rows r of X[r][m] * G[r][n]
// (m = Kin is a virtual column of ones when a.ones: the bias gradient).
template <int KIND>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  using S = typename std::conditional<KIND == GK_F64, double, float>::type;
  using Acc = typename std::conditional<KIND == GK_F64, d4, f4>::type;
  constexpr int BM = 64, BN = 64, BR = 16;
  __shared__ S Xs[BR][BM + 4];
  __shared__ S Gs[BR][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int split = blockIdx.z;
  const int64_t r0 = (int64_t)split * a.rows_per_split;
  const int64_t r1 = r0 + a.rows_per_split < a.rows ? r0 + a.rows_per_split : a.rows;
  const S* X = (const S*)a.X;
  const S* G = (const S*)a.G;
  const int Mtot = a.Kin + (a.ones ? 1 : 0);
  Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;
  const int lr = tid / 16, lc = (tid % 16) * 4;  // loader: row lr, 4 columns from lc
  for (int64_t rb = r0; rb < r1; rb += BR) {
    const int64_t r = rb + lr;
    const bool rv = r < r1;
    const S* xr = X + (rv ? (r / a.xrpw) * a.xws + (r % a.xrpw) * a.ldx : 0);
    const S* gr = G + (rv ? (r / a.grpw) * a.gws + (r % a.grpw) * a.ldg : 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + lc + e, n = n0 + lc + e;
      S xv = 0, gv = 0;
      if (rv) {
        if (m < a.Kin)
          xv = xr[m];
        else if (m == a.Kin && a.ones)
          xv = 1;
        if (n < a.Nout) gv = gr[n];
      }
      Xs[lr][lc + e] = xv;
      Gs[lr][lc + e] = gv;
    }
    __syncthreads();
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int kq = 0; kq < BR / 4; ++kq) {
      S av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = Xs[kq * 4 + g][wm * 32 + i * 16 + c];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Gs[kq * 4 + g][wn * 32 + j * 16 + c];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (KIND == GK_F64)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = (KIND == GK_F64) ? g + 4 * e : 4 * g + e;
        const int m = m0 + wm * 32 + i * 16 + row;
        const int n = n0 + wn * 32 + j * 16 + c;
        if (m < Mtot && n < a.Nout) a.part[((int64_t)split * Mtot + m) * a.Nout + n] = (double)acc[i][j][e];
      }
}

// float32 weight gradients with whole-width tiles: a block owns a BM x 128 tile of W_bar for
// one split of the rows, so every input row is read by one block per output tile (D = 128:
// once).  Rows stream through LDS 32 at a time in two stages (the next rows are loaded into
// registers while the current ones feed the MFMAs, one barrier per step); float4 loads.
// The bias gradient (column sums of G) is accumulated by the first row of tiles from the
// same LDS rows, so the output tile carries no extra row of ones.
template <int BM>
__global__ __launch_bounds__(256) void wgrad_f32_kernel(WgradArgs a) {
  constexpr int BN = 128, BR = 32;
  constexpr int WGM = BM == 128 ? 2 : 1, WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int XL = BM + 4, GL = BN + 4;
  constexpr int XV = BR * BM / 4 / 256, GV = BR * BN / 4 / 256;
  __shared__ __attribute__((aligned(16))) float Xs[2][BR * XL];
  __shared__ __attribute__((aligned(16))) float Gs[2][BR * GL];
  __shared__ float bsum[2][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int g = lane >> 4, c = lane & 15;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int split = blockIdx.z;
  const int64_t r0 = (int64_t)split * a.rows_per_split;
  const int64_t r1 = r0 + a.rows_per_split < a.rows ? r0 + a.rows_per_split : a.rows;
  const float* X = (const float*)a.X;
  const float* G = (const float*)a.G;
  const bool bias = a.ones && blockIdx.x == 0;
  const int Mtot = a.Kin + (a.ones ? 1 : 0);
  float* part = (float*)a.part;  // float32 partial sums: each is a float32 MFMA accumulation, stored exactly

  f4 xv[XV], gv[GV];
  auto load = [&](int64_t rb) {
#pragma unroll
    for (int i = 0; i < XV; ++i) {
      const int f = tid + 256 * i, row = f / (BM / 4), m = m0 + 4 * (f % (BM / 4));
      const int64_t r = rb + row;
      f4 v = {0.f, 0.f, 0.f, 0.f};
      if (r < r1 && m < a.Kin) {
        const uint32_t q = (uint32_t)r / (uint32_t)a.xrpw, rem = (uint32_t)r - q * (uint32_t)a.xrpw;
        v = *(const f4*)(X + (int64_t)q * a.xws + (int64_t)rem * a.ldx + m);
      }
      xv[i] = v;
    }
#pragma unroll
    for (int i = 0; i < GV; ++i) {
      const int f = tid + 256 * i, row = f / (BN / 4), n = n0 + 4 * (f % (BN / 4));
      const int64_t r = rb + row;
      f4 v = {0.f, 0.f, 0.f, 0.f};
      if (r < r1 && n < a.Nout) {
        const uint32_t q = (uint32_t)r / (uint32_t)a.grpw, rem = (uint32_t)r - q * (uint32_t)a.grpw;
        v = *(const f4*)(G + (int64_t)q * a.gws + (int64_t)rem * a.ldg + n);
      }
      gv[i] = v;
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int i = 0; i < XV; ++i) {
      const int f = tid + 256 * i;
      *(f4*)&Xs[st][(f / (BM / 4)) * XL + 4 * (f % (BM / 4))] = xv[i];
    }
#pragma unroll
    for (int i = 0; i < GV; ++i) {
      const int f = tid + 256 * i;
      *(f4*)&Gs[st][(f / (BN / 4)) * GL + 4 * (f % (BN / 4))] = gv[i];
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float bs = 0.f;
  const int bcol = tid & (BN - 1), bhalf = tid >> 7;
  if (r0 < r1) {
    load(r0);
    store(0);
  }
  __syncthreads();
  int st = 0;
  for (int64_t rb = r0; rb < r1; rb += BR) {
    const bool more = rb + BR < r1;
    if (more) load(rb + BR);
#pragma unroll
    for (int kq = 0; kq < BR / 4; ++kq) {
      float av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = Xs[st][(4 * kq + g) * XL + wm * WTM + 16 * i + c];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = Gs[st][(4 * kq + g) * GL + wn * WTN + 16 * j + c];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (bias) {
#pragma unroll
      for (int rr = 0; rr < BR / 2; ++rr) bs += Gs[st][(bhalf * (BR / 2) + rr) * GL + bcol];
    }
    if (more) store(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * WTM + 16 * i + 4 * g + e;
        const int n = n0 + wn * WTN + 16 * j + c;
        if (m < a.Kin && n < a.Nout) part[((int64_t)split * Mtot + m) * a.Nout + n] = acc[i][j][e];
      }
  if (bias) {
    bsum[bhalf][bcol] = bs;
    __syncthreads();
    const int n = n0 + tid;
    if (tid < BN && n < a.Nout) part[((int64_t)split * Mtot + a.Kin) * a.Nout + n] = bsum[0][tid] + bsum[1][tid];
  }
}

// gW[m][n] += sum_split part (m < Kin), gb[n] += row Kin (bias).  Four waves per 64 outputs,
// wave q summing splits q, q + 4, ...; the four sums are added in a fixed order (deterministic).
template <typename P>
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const P* __restrict__ part, int nsplit, int Kin, int ones,
                                                           int Nout, double* __restrict__ gW, int64_t ldgw,
                                                           double* __restrict__ gb) {
  __shared__ double red[4][64];
  const int Mtot = Kin + (ones ? 1 : 0);
  const int64_t tot = (int64_t)Mtot * Nout;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (t < tot) {
#pragma unroll 4
    for (int k = q; k < nsplit; k += 4) s += (double)part[(int64_t)k * tot + t];
  }
  red[q][lane] = s;
  __syncthreads();
  if (q != 0 || t >= tot) return;
  s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  const int m = (int)(t / Nout), n = (int)(t % Nout);
  if (m < Kin)
    gW[(int64_t)m * ldgw + n] += s;
  else
    gb[n] += s;
}

static bool wgrad_f32_tiles_ok(const WgradArgs& a) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return a.Kin % 4 == 0 && a.Nout % 4 == 0 && a.ldx % 4 == 0 && a.ldg % 4 == 0 && a.xws % 4 == 0 &&
         a.gws % 4 == 0 && al(a.X) && al(a.G) && a.xrpw > 0 && a.grpw > 0 && a.xrpw <= INT32_MAX &&
         a.grpw <= INT32_MAX && a.rows <= INT32_MAX;
}

hipError_t launch_wgrad(GemmKind kind, const WgradArgs& a0, double* gW, int64_t ldgw, double* gb, hipStream_t st) {
  if (a0.rows <= 0) return hipSuccess;
  WgradArgs a = a0;
  const int Mtot = a.Kin + (a.ones ? 1 : 0);
  const bool tiles = kind == GK_F32 && wgrad_f32_tiles_ok(a);
  const int bm = !tiles ? 64 : (a.Kin <= 32 ? 32 : (a.Kin <= 64 ? 64 : 128));
  const int mt = tiles ? (a.Kin + bm - 1) / bm : (Mtot + 63) / 64;
  const int nt = tiles ? (a.Nout + 127) / 128 : (a.Nout + 63) / 64;
  // splits: about two blocks per compute unit, at least 256 rows each, within the partial-sum buffer
  // float32 tiles store float32 partials: twice as many fit
  const int64_t cap = (tiles ? 2 * a.part_elems : a.part_elems) / ((int64_t)Mtot * a.Nout);
  static const int per_cu = [] {
    const char* e = std::getenv("QMC_WGRAD_BLOCKS_PER_CU");  // tuning knob, default 2
    const int v = e ? std::atoi(e) : 2;
    return v >= 1 && v <= 8 ? v : 2;
  }();
  int64_t nsplit = std::min<int64_t>((per_cu * device_cus() + mt * nt - 1) / (mt * nt), (a.rows + 255) / 256);
  nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, cap));
  a.rows_per_split = ((a.rows + nsplit - 1) / nsplit + 31) / 32 * 32;
  nsplit = (a.rows + a.rows_per_split - 1) / a.rows_per_split;
  if (cap < 1 || nsplit > cap || nsplit > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)mt, (unsigned)nt, (unsigned)nsplit);
  {
    ProfScope ps(kind == GK_F64 ? "wgrad_kernel<f64>" : "wgrad_kernel<f32>", st);
    if (kind == GK_F64)
      hipLaunchKernelGGL(wgrad_kernel<GK_F64>, grid, dim3(256), 0, st, a);
    else if (!tiles)
      hipLaunchKernelGGL(wgrad_kernel<GK_F32>, grid, dim3(256), 0, st, a);
    else if (bm == 32)
      hipLaunchKernelGGL(wgrad_f32_kernel<32>, grid, dim3(256), 0, st, a);
    else if (bm == 64)
      hipLaunchKernelGGL(wgrad_f32_kernel<64>, grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(wgrad_f32_kernel<128>, grid, dim3(256), 0, st, a);
  }
  const int64_t n = (int64_t)Mtot * a.Nout;
  ProfScope ps("wgrad_reduce_kernel", st);
  if (tiles)
    hipLaunchKernelGGL(wgrad_reduce_kernel<float>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st,
                       (const float*)a.part, (int)nsplit, a.Kin, a.ones, a.Nout, gW, ldgw, gb);
  else
    hipLaunchKernelGGL(wgrad_reduce_kernel<double>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st,
                       (const double*)a.part, (int)nsplit, a.Kin, a.ones, a.Nout, gW, ldgw, gb);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small element-wise kernels

template <typename S>
__global__ void tanh_bwd_kernel(int64_t n, const S* __restrict__ ybar, const S* __restrict__ t, S* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = ybar[i] * (S(1) - t[i] * t[i]);
}

template <typename S>
__global__ void add_kernel(int64_t n, const S* __restrict__ a, const S* __restrict__ b, S* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] + b[i];
}

__global__ void fill_kernel(int64_t n, double v, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename S>
__global__ void cast_kernel(int64_t n, const double* __restrict__ src, S* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (S)src[i];
}

// params[i] -= lr * grad[i] (the optimizer step of a training iteration: plain gradient descent)
template <typename S>
__global__ void sgd_kernel(int64_t n, double lr, const S* __restrict__ grad, S* __restrict__ params) {
#pragma clang fp contract(off)  // a product, then a difference, each rounded (no fused multiply-add)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double step = lr * (double)grad[i];
    params[i] = (S)((double)params[i] - step);
  }
}

template <typename S>
hipError_t launch_sgd(int64_t n, double lr, const S* grad, S* params, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  ProfScope ps("sgd_kernel", st);
  hipLaunchKernelGGL(sgd_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, lr, grad, params);
  return hipGetLastError();
}
template hipError_t launch_sgd<float>(int64_t, double, const float*, float*, hipStream_t);
template hipError_t launch_sgd<double>(int64_t, double, const double*, double*, hipStream_t);

// dst[c] += sum_r src[r * ld + c]: rows split in chunks of 64 (one thread per
// (chunk, column)), then the chunk sums are added in chunk order.
__global__ void rowsum_partial_kernel(const double* __restrict__ src, int64_t R, int64_t C, int64_t ld,
                                      double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (c >= C) return;
  const int64_t r0 = k * 64, r1 = r0 + 64 < R ? r0 + 64 : R;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += src[r * ld + c];
  part[k * C + c] = s;
}

__global__ void rowsum_final_kernel(const double* __restrict__ part, int64_t nchunk, int64_t C,
                                    double* __restrict__ dst) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double s = 0.0;
  for (int64_t k = 0; k < nchunk; ++k) s += part[k * C + c];
  dst[c] += s;
}

template <typename S>
hipError_t launch_tanh_bwd(int64_t n, const S* ybar, const S* t, S* z, hipStream_t st) {
  ProfScope ps("tanh_bwd_kernel", st);
  hipLaunchKernelGGL(tanh_bwd_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ybar, t, z);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_add(int64_t n, const S* a, const S* b, S* o, hipStream_t st) {
  ProfScope ps("add_kernel", st);
  hipLaunchKernelGGL(add_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b, o);
  return hipGetLastError();
}
hipError_t launch_fill(int64_t n, double v, double* p, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  ProfScope ps("fill_kernel", st);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, p);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_cast(int64_t n, const double* src, S* dst, hipStream_t st) {
  ProfScope ps("cast_kernel", st);
  hipLaunchKernelGGL(cast_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src, dst);
  return hipGetLastError();
}
hipError_t launch_rowsum(const double* src, int64_t R, int64_t C, int64_t ld, double* dst, double* scratch,
                         int64_t scratch_elems, hipStream_t st) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const int64_t nchunk = (R + 63) / 64;
  if (nchunk * C > scratch_elems || nchunk > 65535) return hipErrorInvalidValue;
  ProfScope ps("rowsum_kernel", st);
  hipLaunchKernelGGL(rowsum_partial_kernel, dim3((unsigned)((C + 127) / 128), (unsigned)nchunk), dim3(128), 0, st, src,
                     R, C, ld, scratch);
  hipLaunchKernelGGL(rowsum_final_kernel, dim3((unsigned)((C + 127) / 128)), dim3(128), 0, st, scratch, nchunk, C, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------- loss-gradient weights

// stats[0] = mean of the finite e_loc, stats[1] = their count.  One block,
// fixed per-thread order and tree reduction: deterministic.
__global__ __launch_bounds__(1024) void emean_kernel(const double* __restrict__ e, int64_t W, double* __restrict__ stats,
                                                     int64_t* __restrict__ nfin) {
  __shared__ double ss[1024];
  __shared__ double sc[1024];
  double s = 0.0, c = 0.0;
  for (int64_t w = threadIdx.x; w < W; w += 1024) {
    const double v = e[w];
    if (isfinite(v)) {
      s += v;
      c += 1.0;
    }
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sc[threadIdx.x] += sc[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = sc[0] > 0 ? ss[0] / sc[0] : NAN;
    stats[1] = sc[0];
    if (nfin) *nfin = (int64_t)sc[0];
  }
}

// ---------------------------------------------------------------- clipped local energies

// Order-preserving map of a finite double onto uint64 keys, and back.
__device__ inline uint64_t order_key(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double key_value(uint64_t k) {
  const uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)u);
}

// Fixed-order block sum over 1024 threads (deterministic).
__device__ inline double block_sum_1024(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One block per system: the median of the finite values by an 8-pass radix select on order keys
// (256-bin LDS histograms), the mean absolute deviation from it (fixed-order sums), then
// hard: clamp to [mu - sigma, mu + sigma]; soft: outside the window mu +- sigma (1 + log(|E - mu| / sigma)).
// Non-finite values pass through; so does everything when sigma is not positive.
__global__ __launch_bounds__(1024) void clip_kernel(const double* __restrict__ e, double* __restrict__ out, int64_t n,
                                                    double width, int mode) {
  __shared__ unsigned hist[256];
  __shared__ double red[1024];
  __shared__ int sh_digit;
  __shared__ unsigned long long sh_rank;
  const int tid = threadIdx.x;
  double c = 0.0;
  for (int64_t i = tid; i < n; i += 1024) c += isfinite(e[i]) ? 1.0 : 0.0;
  const double cnt = block_sum_1024(c, red);
  double mu = 0.0, sigma = 0.0;
  if (cnt > 0) {
    const unsigned long long m = (unsigned long long)cnt;
    auto select = [&](unsigned long long k) -> double {
      uint64_t prefix = 0, mask = 0;
      for (int shift = 56; shift >= 0; shift -= 8) {
        if (tid < 256) hist[tid] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < n; i += 1024) {
          const double x = e[i];
          if (!isfinite(x)) continue;
          const uint64_t key = order_key(x);
          if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1u);
        }
        __syncthreads();
        if (tid == 0) {
          unsigned long long acc = 0;
          int d = 0;
          for (; d < 255; ++d) {
            if (acc + hist[d] > k) break;
            acc += hist[d];
          }
          sh_digit = d;
          sh_rank = k - acc;
        }
        __syncthreads();
        prefix |= (uint64_t)sh_digit << shift;
        mask |= (uint64_t)0xFF << shift;
        k = sh_rank;
        __syncthreads();
      }
      return key_value(prefix);
    };
    const double lo = select((m - 1) / 2);
    mu = (m & 1) ? lo : (lo + select(m / 2)) * 0.5;
    double a = 0.0;
    for (int64_t i = tid; i < n; i += 1024) {
      const double x = e[i];
      if (isfinite(x)) a += fabs(x - mu);
    }
    sigma = width * (block_sum_1024(a, red) / cnt);
  }
  const bool clip = cnt > 0 && sigma > 0.0;
  for (int64_t i = tid; i < n; i += 1024) {
    const double x = e[i];
    double y = x;
    if (clip && isfinite(x)) {
      if (mode == 0) {
        y = fmin(fmax(x, mu - sigma), mu + sigma);
      } else {
        const double dv = fabs(x - mu);
        if (dv > sigma) y = mu + copysign(sigma * (1.0 + log(dv / sigma)), x - mu);
      }
    }
    out[i] = y;
  }
}

hipError_t launch_clip(const double* e, double* out, int64_t n, double width, int mode, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  ProfScope ps("clip_kernel", st);
  hipLaunchKernelGGL(clip_kernel, dim3(1), dim3(1024), 0, st, e, out, n, width, mode);
  return hipGetLastError();
}

// g_w = 2 (e_w - mean) / count for finite e_w, else 0
__global__ void gbar_kernel(const double* __restrict__ e, const double* __restrict__ stats, int64_t W,
                            double* __restrict__ g) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double v = e[w];
  g[w] = (isfinite(v) && stats[1] > 0) ? 2.0 * (v - stats[0]) / stats[1] : 0.0;
}

hipError_t launch_loss_weights(const double* e, int64_t W, double* stats, double* g, double* e_mean,
                               int64_t* n_finite, hipStream_t st) {
  {
    ProfScope ps("emean_kernel", st);
    hipLaunchKernelGGL(emean_kernel, dim3(1), dim3(1024), 0, st, e, W, stats, n_finite);
  }
  if (e_mean) {
    if (hipMemcpyAsync(e_mean, stats, sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return hipErrorUnknown;
  }
  ProfScope ps("gbar_kernel", st);
  hipLaunchKernelGGL(gbar_kernel, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, st, e, stats, W, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------- combination backward

// lbar[w][p] = g_w * w_p (cotangent of each determinant log, both spins);
// cpart[w][p] = g_w * D_p / psi (cotangent of c_p, summed over walkers later).
template <typename S>
__global__ void combine_bwd_kernel(SysDev s, const S* __restrict__ c, const double* __restrict__ ld,
                                   const double* __restrict__ sg, const double* __restrict__ gbar, int64_t W,
                                   double* __restrict__ lbar, double* __restrict__ cpart) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
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
  const double gw = gbar[w];
  for (int p = 0; p < nd; ++p) {
    double l = 0.0, sd = 1.0;
    for (int sp = 0; sp < 2; ++sp)
      if (has[sp]) {
        l += ld[(w * 2 + sp) * nd + p];
        sd *= sg[(w * 2 + sp) * nd + p];
      }
    const double dpsi = (sd != 0.0 && S_ != 0.0 && gw != 0.0) ? sd * exp(l - mx) / S_ : 0.0;  // D_p / psi
    lbar[w * nd + p] = gw * (double)c[p] * dpsi;
    cpart[w * nd + p] = gw * dpsi;
  }
}

template <typename S>
hipError_t launch_combine_bwd(const SysDev& s, const S* c, const double* ld, const double* sg, const double* gbar,
                              int64_t W, double* lbar, double* cpart, hipStream_t st) {
  ProfScope ps("combine_bwd_kernel", st);
  hipLaunchKernelGGL(combine_bwd_kernel<S>, dim3((unsigned)((W + 127) / 128)), dim3(128), 0, st, s, c, ld, sg, gbar,
                     W, lbar, cpart);
  return hipGetLastError();
}

// ---------------------------------------------------------------- orbitals x envelopes backward

// One thread per (walker, det, orbital k) of spin block `spin`: loops over the
// electrons a of the block.  A_bar[a][k] = lbar_p * (A^-1)[k][a];
// phi_bar = A_bar * env (written per electron row), and the envelope weights
// and exponents collect env_bar * exp(-sigma d) and -env_bar * pi * d * exp(-sigma d).
template <typename S>
__global__ __launch_bounds__(128) void orb_bwd_kernel(SysDev s, int spin, const double* __restrict__ lbar,
                                                     const double* __restrict__ ainv, const S* __restrict__ phi,
                                                     const S* __restrict__ pi, const S* __restrict__ sg,
                                                     const double* __restrict__ en, int64_t W,
                                                     S* __restrict__ phibar, double* __restrict__ pipart,
                                                     double* __restrict__ sgpart) {
  // envelope values in the plan's activation type (as in the forward); sums in float64
  using T = S;
  // n electrons of this spin, no orbitals per determinant, matrices of order dim with this spin's
  // rows from row0 (spin-factorized: no = dim = n, row0 = 0)
  const int n = spin ? s.ndn : s.nup;
  const int no = orb_count(s, spin), dim = s.full_det ? s.N : n, row0 = det_row0(s, spin);
  const int i0 = spin ? s.nup : 0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * s.ndet * no) return;
  const int k = (int)(t % no);
  const int p = (int)((t / no) % s.ndet);
  const int64_t w = t / ((int64_t)no * s.ndet);
  const int ncol = s.ndet * no;
  const double lb = lbar[w * s.ndet + p];
  const double* Ai = ainv + ((w * s.ndet + p) * dim) * (int64_t)dim;  // [dim][dim]
  const double* gw = en + (w * s.N + i0) * s.M * 4;                    // electron a of this spin: gw + a * M * 4
  const S* phw = phi + (w * n) * (int64_t)ncol + p * no + k;           // row a: phw[a * ncol]
  const S* pik = pi + ((int64_t)p * no + k) * s.M * s.nenv;
  const S* sgk = sg + ((int64_t)p * no + k) * s.M * s.nenv;
  // One pass over (nucleus, exponent), each exponential evaluated once per electron: it feeds the
  // envelope of electron a (for phi_bar = Abar * env, Abar = lbar A^-T) and the pi_bar, sigma_bar
  // sums over the electrons of the spin block.  The spin block has at most 32 electrons (the
  // determinant limit), so its per-electron values stay in registers.
  constexpr int AMAX = 32;
  double eba[AMAX];
  T enva[AMAX];
#pragma unroll
  for (int a = 0; a < AMAX; ++a) {
    enva[a] = 0;
    eba[a] = a < n ? lb * Ai[k * dim + row0 + a] * (double)phw[(int64_t)a * ncol] : 0.0;
  }
  double* pp = pipart + t * (int64_t)(s.M * s.nenv);
  double* sp = sgpart + t * (int64_t)(s.M * s.nenv);
  for (int I = 0; I < s.M; ++I)
    for (int b = 0; b < s.nenv; ++b) {
      const T pw = pik[I * s.nenv + b], sgm = sgk[I * s.nenv + b];
      double ap = 0.0, as = 0.0;
#pragma unroll
      for (int a = 0; a < AMAX; ++a) {
        if (a < n) {
          const T d = (T)gw[a * s.M * 4 + I * 4];
          const T e = exp(-sgm * d);
          enva[a] += pw * e;
          const double ex = (double)e;
          ap += eba[a] * ex;
          as -= eba[a] * (double)pw * (double)d * ex;
        }
      }
      pp[I * s.nenv + b] = ap;
      sp[I * s.nenv + b] = as;
    }
#pragma unroll
  for (int a = 0; a < AMAX; ++a)
    if (a < n) phibar[(w * n + a) * (int64_t)ncol + p * no + k] = (S)(lb * Ai[k * dim + row0 + a] * (double)enva[a]);
}

template <typename S>
hipError_t launch_orb_bwd(const SysDev& s, int spin, const double* lbar, const double* ainv, const S* phi,
                          const S* pi, const S* sg, const double* en, int64_t W, S* phibar, double* pipart,
                          double* sgpart, hipStream_t st) {
  const int64_t cnt = (spin ? s.ndn : s.nup) > 0 ? W * s.ndet * orb_count(s, spin) : 0;
  if (cnt == 0) return hipSuccess;
  ProfScope ps("orb_bwd_kernel", st);
  hipLaunchKernelGGL(orb_bwd_kernel<S>, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, st, s, spin, lbar, ainv,
                     phi, pi, sg, en, W, phibar, pipart, sgpart);
  return hipGetLastError();
}

// ---------------------------------------------------------------- message aggregation backward

__device__ inline int ee_pair_b(const SysDev& s, int i, int j, int& type) {
  const bool ui = i < s.nup, uj = j < s.nup;
  if (ui != uj) {
    type = 1;
    const int a = ui ? i : j, b = ui ? j : i;
    return a * s.ndn + (b - s.nup);
  }
  type = 0;
  int a = i < j ? i : j, b = i < j ? j : i;
  int n = s.nup, off = 0;
  if (!ui) {
    n = s.ndn;
    a -= s.nup;
    b -= s.nup;
    off = s.nup * (s.nup - 1) / 2;
  }
  return off + a * (2 * n - a - 1) / 2 + (b - a - 1);
}

// Block per walker, thread per column d.  With mbar = [m_same, m_opp, m_nuc] cotangents:
//   h_bar_j   = sum_i (1/n(i)) w(d_ij) m_bar_type(i,j),_i
//   w_bar_ij  = (1/n(i)) m_bar_i h_j + (1/n(j)) m_bar_j h_i      (unordered e-e pair)
//   w_bar_iI  = m_bar_nuc_i Y_I / M,   Y_bar_I += sum_i w_iI m_bar_nuc_i / M
template <typename S>
__global__ void agg_bwd_kernel(SysDev s, const S* __restrict__ mbar, const S* __restrict__ h,
                               const S* __restrict__ wsame, const S* __restrict__ wopp, const S* __restrict__ wnuc,
                               const S* __restrict__ Y, S* __restrict__ hbar, S* __restrict__ wbs,
                               S* __restrict__ wbo, S* __restrict__ wbn, double* __restrict__ ypart) {
  const int64_t w = blockIdx.x;
  const int N = s.N, D = s.D, M = s.M;
  const S* mb = mbar + w * N * 3 * (int64_t)D;
  const S* hw = h + w * N * (int64_t)D;
  auto inv_n = [&](int i, int type) -> S {
    const bool up = i < s.nup;
    const int n = type == 0 ? (up ? s.nup : s.ndn) - 1 : (up ? s.ndn : s.nup);
    return n > 0 ? S(1) / S(n) : S(0);
  };
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    for (int j = 0; j < N; ++j) {
      S acc = 0;
      for (int i = 0; i < N; ++i) {
        if (i == j) continue;
        int type;
        const int p = ee_pair_b(s, i, j, type);
        const S wv = type ? wopp[(w * s.P1 + p) * D + d] : wsame[(w * s.P0 + p) * D + d];
        acc += inv_n(i, type) * wv * mb[(int64_t)i * 3 * D + type * D + d];
      }
      hbar[(w * N + j) * D + d] = acc;
    }
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        int type;
        const int p = ee_pair_b(s, i, j, type);
        const S v = inv_n(i, type) * mb[(int64_t)i * 3 * D + type * D + d] * hw[(int64_t)j * D + d] +
                    inv_n(j, type) * mb[(int64_t)j * 3 * D + type * D + d] * hw[(int64_t)i * D + d];
        if (type)
          wbo[(w * s.P1 + p) * D + d] = v;
        else
          wbs[(w * s.P0 + p) * D + d] = v;
      }
    const S invM = S(1) / S(M);
    for (int I = 0; I < M; ++I) {
      double yp = 0.0;
      const S yv = Y[I * D + d];
      for (int i = 0; i < N; ++i) {
        const S mn = mb[(int64_t)i * 3 * D + 2 * D + d];
        const int64_t pe = (w * s.P2 + i * M + I) * D + d;
        wbn[pe] = mn * yv * invM;
        yp += (double)(wnuc[pe] * mn * invM);
      }
      ypart[(w * M + I) * D + d] = yp;
    }
  }
}

template <typename S>
hipError_t launch_agg_bwd(const SysDev& s, const S* mbar, const S* h, const S* wsame, const S* wopp, const S* wnuc,
                          const S* Y, int64_t W, S* hbar, S* wbs, S* wbo, S* wbn, double* ypart, hipStream_t st) {
  ProfScope ps("agg_bwd_kernel", st);
  const int threads = s.D < 256 ? ((s.D + 63) / 64) * 64 : 256;
  hipLaunchKernelGGL(agg_bwd_kernel<S>, dim3((unsigned)W), dim3(threads), 0, st, s, mbar, h, wsame, wopp, wnuc, Y,
                     hbar, wbs, wbo, wbn, ypart);
  return hipGetLastError();
}

// ---------------------------------------------------------------- position gradient (reverse pass)
//
// d log|psi| / d r through the distances: every feature depends on the positions only through
// d_ij and d_iI, so the cotangents of the radial bases, of the envelopes and of the cusp factor are
// gathered per distance (dee[w][i][j] for i < j, den[w][i][I]) and then mapped to the positions
// with the unit vectors: rbar_i = sum_j dbar_ij u_ij + sum_I dbar_iI u_iI.

// edge filters of one type: dbar += sum_k rhobar[pair][k] drho_k / dd
template <typename S>
__global__ void pair_dbar_kernel(SysDev s, int type, const S* __restrict__ rhobar, const double* __restrict__ ee,
                                 const double* __restrict__ en, int64_t W, double* __restrict__ dee,
                                 double* __restrict__ den) {
  const int P = type == 0 ? s.P0 : (type == 1 ? s.P1 : s.P2);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * P) return;
  const int64_t w = t / P;
  const int p = (int)(t - w * P);
  int i, j;
  decode_pair(s, type, p, i, j);
  const double d = type == 2 ? en[((w * s.N + i) * s.M + j) * 4] : ee[((w * s.N + i) * s.N + j) * 4];
  const double sp = rbf_spacing(s.dmax, s.K), inv = (s.K - 1) / s.dmax;
  double acc = 0.0;
  for (int k = 0; k < s.K; ++k) {
    double r0, r1, r2;
    rbf3(d, k, sp, inv, r0, r1, r2);
    acc += (double)rhobar[t * s.K + k] * r1;
  }
  if (type == 2)
    den[(w * s.N + i) * s.M + j] += acc;
  else
    dee[(w * s.N + i) * s.N + j] += acc;  // i < j
}

// initial features x0 = [rho(d_iI) per nucleus, mean same-spin rho(d_ij), mean opposite-spin rho(d_ij)]:
// threads over (w, i, I) for the e-n block and (w, i < j) for the two means (both ends of a pair)
template <typename S>
__global__ void init_dbar_kernel(SysDev s, const S* __restrict__ x0bar, const double* __restrict__ ee,
                                 const double* __restrict__ en, int64_t W, double* __restrict__ dee,
                                 double* __restrict__ den) {
  const int N = s.N, M = s.M, K = s.K, F = (M + 2) * K;
  const int per = N * M + N * N;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * per) return;
  const int64_t w = t / per;
  const int e = (int)(t - w * per);
  const double sp = rbf_spacing(s.dmax, K), inv = (K - 1) / s.dmax;
  if (e < N * M) {
    const int i = e / M, I = e - (e / M) * M;
    const double d = en[((w * N + i) * M + I) * 4];
    const S* xb = x0bar + (w * N + i) * (int64_t)F + I * K;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
      double r0, r1, r2;
      rbf3(d, k, sp, inv, r0, r1, r2);
      acc += (double)xb[k] * r1;
    }
    den[(w * N + i) * M + I] += acc;
    return;
  }
  const int q = e - N * M, i = q / N, j = q - (q / N) * N;
  if (j <= i) return;
  const bool ui = i < s.nup, uj = j < s.nup, same = ui == uj;
  const int blk = same ? 0 : 1;
  // members of each end's set: same spin without itself, or the other spin
  const int ci = same ? (ui ? s.nup : s.ndn) - 1 : (ui ? s.ndn : s.nup);
  const int cj = same ? (uj ? s.nup : s.ndn) - 1 : (uj ? s.ndn : s.nup);
  const double d = ee[((w * N + i) * N + j) * 4];
  const S* xi = x0bar + (w * N + i) * (int64_t)F + (M + blk) * K;
  const S* xj = x0bar + (w * N + j) * (int64_t)F + (M + blk) * K;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    double r0, r1, r2;
    rbf3(d, k, sp, inv, r0, r1, r2);
    acc += ((double)xi[k] / ci + (double)xj[k] / cj) * r1;
  }
  dee[(w * N + i) * N + j] += acc;
}

// envelopes: dA[a][k] / dd_aI = phi_k(a) sum_b (-sigma pi exp(-sigma d)), weighted by
// Abar = lbar_p (A_p^-1)^T; thread per (w, electron a of this spin, nucleus I)
template <typename S>
__global__ void env_dbar_kernel(SysDev s, int spin, const double* __restrict__ lbar, const double* __restrict__ ainv,
                                const S* __restrict__ phi, const S* __restrict__ pi, const S* __restrict__ sg,
                                const double* __restrict__ en, int64_t W, double* __restrict__ den) {
  const int n = spin ? s.ndn : s.nup;
  const int no = orb_count(s, spin), dim = s.full_det ? s.N : n, row0 = det_row0(s, spin);
  const int i0 = spin ? s.nup : 0;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * n * s.M) return;
  const int I = (int)(t % s.M);
  const int64_t wa = t / s.M;
  const int a = (int)(wa % n);
  const int64_t w = wa / n;
  const int ncol = s.ndet * no;
  const double d = en[((w * s.N + i0 + a) * s.M + I) * 4];
  double acc = 0.0;
  for (int p = 0; p < s.ndet; ++p) {
    const double lb = lbar[w * s.ndet + p];
    const double* Ai = ainv + ((w * s.ndet + p) * dim) * (int64_t)dim;
    for (int k = 0; k < no; ++k) {
      const int64_t o = (((int64_t)p * no + k) * s.M + I) * s.nenv;
      double de = 0.0;
      for (int b = 0; b < s.nenv; ++b) {
        const double sgm = (double)sg[o + b];
        de -= sgm * (double)pi[o + b] * exp(-sgm * d);
      }
      acc += lb * Ai[k * dim + row0 + a] * (double)phi[(w * n + a) * (int64_t)ncol + p * no + k] * de;
    }
  }
  den[(w * s.N + i0 + a) * s.M + I] += acc;
}

// positions: rbar_i = sum_j dbar_ij u_ij + sum_I dbar_iI u_iI (+ the cusp factor's gradient); NaN
// where log|psi| is not finite
__global__ void positions_bar_kernel(SysDev s, const double* __restrict__ ee, const double* __restrict__ en,
                                     const double* __restrict__ dee, const double* __restrict__ den,
                                     const double* __restrict__ lp, int64_t W, double* __restrict__ out) {
  const int N = s.N, M = s.M;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * N) return;
  const int64_t w = t / N;
  const int i = (int)(t - w * N);
  double g[3] = {0.0, 0.0, 0.0};
  const double a = s.ee_cusp, a2 = a * a;
  for (int j = 0; j < N; ++j) {
    if (j == i) continue;
    const double* e = ee + ((w * N + i) * N + j) * 4;
    double db = i < j ? dee[(w * N + i) * N + j] : dee[(w * N + j) * N + i];
    if (a > 0.0) {
      const double c = ((i < s.nup) == (j < s.nup)) ? 0.25 : 0.5;
      const double q = 1.0 / (a + e[0]);
      db += c * a2 * q * q;
    }
    for (int x = 0; x < 3; ++x) g[x] += db * e[1 + x];
  }
  for (int I = 0; I < M; ++I) {
    const double* e = en + ((w * N + i) * M + I) * 4;
    const double db = den[(w * N + i) * M + I];
    for (int x = 0; x < 3; ++x) g[x] += db * e[1 + x];
  }
  const bool ok = isfinite(lp[w]);
  for (int x = 0; x < 3; ++x) out[t * 3 + x] = ok ? g[x] : NAN;
}

template <typename S>
hipError_t launch_pair_dbar(const SysDev& s, int type, const S* rhobar, const double* ee, const double* en, int64_t W,
                            double* dee, double* den, hipStream_t st) {
  const int P = type == 0 ? s.P0 : (type == 1 ? s.P1 : s.P2);
  const int64_t n = W * P;
  if (n == 0) return hipSuccess;
  ProfScope ps("pair_dbar_kernel", st);
  hipLaunchKernelGGL(pair_dbar_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, type, rhobar, ee, en,
                     W, dee, den);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_init_dbar(const SysDev& s, const S* x0bar, const double* ee, const double* en, int64_t W,
                            double* dee, double* den, hipStream_t st) {
  const int64_t n = W * (s.N * s.M + s.N * s.N);
  if (n == 0) return hipSuccess;
  ProfScope ps("init_dbar_kernel", st);
  hipLaunchKernelGGL(init_dbar_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, x0bar, ee, en, W,
                     dee, den);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_env_dbar(const SysDev& s, int spin, const double* lbar, const double* ainv, const S* phi,
                           const S* pi, const S* sg, const double* en, int64_t W, double* den, hipStream_t st) {
  const int64_t n = W * (spin ? s.ndn : s.nup) * s.M;
  if (n == 0) return hipSuccess;
  ProfScope ps("env_dbar_kernel", st);
  hipLaunchKernelGGL(env_dbar_kernel<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, spin, lbar, ainv, phi,
                     pi, sg, en, W, den);
  return hipGetLastError();
}

hipError_t launch_positions_bar(const SysDev& s, const double* ee, const double* en, const double* dee,
                                const double* den, const double* lp, int64_t W, double* out, hipStream_t st) {
  const int64_t n = W * s.N;
  if (n == 0) return hipSuccess;
  ProfScope ps("positions_bar_kernel", st);
  hipLaunchKernelGGL(positions_bar_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, ee, en, dee, den,
                     lp, W, out);
  return hipGetLastError();
}

#define QMC_BWD_INST(S)                                                                                           \
  template hipError_t launch_tanh_bwd<S>(int64_t, const S*, const S*, S*, hipStream_t);                          \
  template hipError_t launch_add<S>(int64_t, const S*, const S*, S*, hipStream_t);                               \
  template hipError_t launch_pair_dbar<S>(const SysDev&, int, const S*, const double*, const double*, int64_t,    \
                                          double*, double*, hipStream_t);                                          \
  template hipError_t launch_init_dbar<S>(const SysDev&, const S*, const double*, const double*, int64_t, double*, \
                                          double*, hipStream_t);                                                   \
  template hipError_t launch_env_dbar<S>(const SysDev&, int, const double*, const double*, const S*, const S*,     \
                                         const S*, const double*, int64_t, double*, hipStream_t);                               \
  template hipError_t launch_cast<S>(int64_t, const double*, S*, hipStream_t);                                   \
  template hipError_t launch_combine_bwd<S>(const SysDev&, const S*, const double*, const double*, const double*, \
                                            int64_t, double*, double*, hipStream_t);                              \
  template hipError_t launch_orb_bwd<S>(const SysDev&, int, const double*, const double*, const S*, const S*,     \
                                        const S*, const double*, int64_t, S*, double*, double*, hipStream_t);     \
  template hipError_t launch_agg_bwd<S>(const SysDev&, const S*, const S*, const S*, const S*, const S*,          \
                                        const S*, int64_t, S*, S*, S*, S*, double*, hipStream_t);
QMC_BWD_INST(double)
QMC_BWD_INST(float)

}  // namespace qmc
