// MFMA GEMM over jet rows with a fused tanh-jet epilogue (gfx950).
//
// A layer y = x W + b applied to a jet (value, gradient rows, Laplacian row)
// maps every row through W and adds b to the value row only.  The tanh that
// follows needs, per (electron, column), the sum over gradient rows of the
// squared pre-activation: t = tanh(z0), grad t = t' grad z,
// lap t = t' lap z + t'' |grad z|^2 with t' = 1 - t^2, t'' = -2 t t'.
// Tiles therefore hold whole row groups (BM is a multiple of the group size).
//
// Main loop: 256 threads, block tile BM x 128, each of the 4 waves owns all
// BM rows of 32 output columns.  Two LDS stages; the next K-slice is fetched
// into registers while the MFMAs consume the current stage (one barrier per
// K-step).  Operand loads are branch-free 16-byte loads whenever K is a
// multiple of the K-step and the operands are 16-byte aligned; otherwise a
// bounds-checked path is taken.
//
// LDS layouts: A [BM][BK+4] (k contiguous: one 16-byte read gives a lane the
// operands of four f32/f64 MFMAs); B [BK][128+4] (columns contiguous, written
// straight from coalesced row loads of W; a lane reads its four k values with
// four scalar reads).  For bf16 both tiles are k-contiguous ([rows][k],
// [columns][k]) so that a lane's eight k values are one 16-byte read.
//
// Epilogue: each wave stages its accumulator tile in LDS transposed
// ([column][row]), then every lane takes one output column and a run of whole
// row groups (or a part of one group, with the |grad z|^2 partial sums
// combined by cross-lane shuffles).  Rows are walked in order, so the bias,
// the five-row nuclear term, the residual and the output are read and written
// as row segments shared by 32 (16 for f64) lanes.
//
// MFMA shapes: f64 v_mfma_f64_16x16x4, f32 v_mfma_f32_16x16x4, bf16
// v_mfma_f32_16x16x32 (operands rounded to bf16, float accumulation), and
// float32 on the bf16 matrix cores (tile bit 3, "f32x3"): every operand x is
// split into three round-to-nearest bf16 pieces x = x0 + x1 + x2 (x0 = bf16(x),
// x1 = bf16(x - x0), x2 = bf16(x - x0 - x1); the differences are exact in
// float32 and the pieces represent x within 2^-24 |x|), and each product is the
// sum of the six piece products of order at most 2, exact in float32 and
// accumulated in float32 by v_mfma_f32_16x16x32_bf16, smallest first; the
// omitted products add up to at most about 2^-23 |x y|, so the result has
// float32-level error.  Six 16-cycle MFMAs replace eight 32-cycle float32 ones
// per 32 k.  A is split once per element when the tile is stored (three bf16
// planes in LDS, k-contiguous), B's fragment once per K-step by the wave that
// owns its columns (float32 in LDS, k-contiguous); one LDS stage (two barriers
// per K-step) keeps the block at the float32 kernel's LDS size.  The
// 16x16 accumulator layouts: f32/bf16: lane l, element i -> row 4*(l/16)+i,
// column l%16; f64: row (l/16)+4*i, column l%16.  Operand layout: lane l
// supplies row (A) / column (B) l%16 and the k-slice selected by l/16; A and
// B use the same k assignment, so the contraction does not depend on how the
// hardware orders k inside a lane.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <type_traits>

#include "act.h"
#include "kernels.h"

namespace qmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int GK_F32X3 = 3;  // float32 operands on bf16 matrix cores (three-piece split)

// Splits x into three bf16 pieces (round to nearest each): x0 + x1 + x2 = x within 2^-24 |x|.
__device__ inline void split3(float x, __bf16& x0, __bf16& x1, __bf16& x2) {
  x0 = (__bf16)x;
  const float r1 = x - (float)x0;
  x1 = (__bf16)r1;
  x2 = (__bf16)(r1 - (float)x1);
}

template <int KIND> struct GT;
template <> struct GT<GK_F64> {
  using S = double;
  using Acc = d4;
  using L = double;  // LDS element
};
template <> struct GT<GK_F32> {
  using S = float;
  using Acc = f4;
  using L = float;
};
template <> struct GT<GK_BF16> {
  using S = float;
  using Acc = f4;
  using L = __bf16;
};
template <> struct GT<GK_F32X3> {
  using S = float;
  using Acc = f4;
  using L = __bf16;  // the A planes; B stays float32 in LDS
};

template <typename S> struct V4;
template <> struct V4<float> {
  using T = float4;
};
template <> struct V4<double> {
  using T = double4;
};

__device__ inline double dtanh(double x) { return tanh(x); }
__device__ inline float dtanh(float x) { return tanh_f32(x); }

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// EPI: 0 value rows, 1 univariate edge jets (groups of 4 rows), 2 electron jets (groups of Rp = 16*bpg rows)
template <int KIND, int MB, int EPI, int BKT, bool PERSIST>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  using G = GT<KIND>;
  using S = typename G::S;
  using Acc = typename G::Acc;
  using L = typename G::L;
  using Vec = typename V4<S>::T;
  constexpr int BK = BKT;
  constexpr int BM = 16 * MB;
  constexpr int BN = 128;
  constexpr bool BF = (KIND == GK_BF16);
  constexpr bool X3 = (KIND == GK_F32X3);
  constexpr bool KC = BF || X3;  // k-contiguous tiles ([rows][k], [columns][k])
  constexpr int APAD = KC ? 8 : 4;
  constexpr int ALD = BK + APAD;
  constexpr int BLD = BF ? BK + 8 : (X3 ? BK + 4 : BN + 4);
  constexpr int ASZ = BM * ALD;  // one A stage (X3: one of the three planes)
  constexpr int BSZ = KC ? BN * BLD : BK * BLD;
  // epilogue staging: per wave NCP columns x CLD rows per pass
  constexpr int NPASS = (KIND == GK_F64) ? 2 : 1;
  constexpr int NCP = 32 / NPASS;  // columns staged per pass
  constexpr int LPC = 64 / NCP;    // lanes sharing one column
  constexpr int CLD = BM + 4;
  constexpr int STAGE_BYTES = X3 ? 3 * ASZ * 2 + BSZ * 4 : 2 * (ASZ + BSZ) * (int)sizeof(L);
  constexpr int C_BYTES = 4 * NCP * CLD * (int)sizeof(S);
  __shared__ __attribute__((aligned(16))) char smem[cmax(STAGE_BYTES, C_BYTES)];
  L* const As = (L*)smem;
  L* const Bs = As + 2 * ASZ;
  float* const Bf = (float*)(smem + 3 * ASZ * 2);  // X3: B stage [BN][BLD]

  constexpr int AV = BM * BK / 4, BV = BK * BN / 4;
  constexpr int NA = (AV + 255) / 256, NB = (BV + 255) / 256;
  constexpr int AKV = BK / 4;  // vectors per A row

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // one row tile; a persistent launch walks the row tiles with a grid stride
  auto row_tile = [&](int64_t bx) {
    const int64_t m0 = bx * BM;
    const int n0 = blockIdx.y * BN;
    const S* __restrict__ X = (const S*)a.X;
    const S* __restrict__ Wt = (const S*)a.W;
    const bool kfull = (a.K % BK) == 0;
    const bool avec = (a.ldx % 4 == 0) && ((a.xws % 4) == 0) &&
                      ((reinterpret_cast<uintptr_t>(X) % (4 * sizeof(S))) == 0);
    const bool bvec = (a.ldw % 4 == 0) && (reinterpret_cast<uintptr_t>(Wt) % (4 * sizeof(S)) == 0);
    // Fast path: every operand load is an unconditional 16-byte load.  Rows past the end and
    // columns past Ncols are clamped to the last valid ones; their products land only in outputs
    // that the epilogue does not store (rows are checked per row, jet groups are whole).
    const bool fast = kfull && avec && bvec && (a.Ncols % 4 == 0) && (a.K % 4 == 0);

    // fixed row pointers of this thread's A slots
    const S* arow[NA];
    bool aval[NA];
    int arr[NA], akk[NA];
  #pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + 256 * u;
      arr[u] = v / AKV;
      akk[u] = (v % AKV) * 4;
      const int64_t r = m0 + arr[u];
      aval[u] = (v < AV) && (r < a.rows);
      const uint32_t rr = (uint32_t)(r < a.rows ? r : a.rows - 1), rpw = (uint32_t)a.xrpw;
      const uint32_t qb = rr / rpw;
      arow[u] = X + (int64_t)qb * a.xws + (int64_t)(rr - qb * rpw) * a.ldx;
    }
    S ra[NA][4], rb[NB][4];

    // B slot v: float32/float64 with W row-major (k, n): 4 consecutive columns of row k;
    // transposed W and bf16: 4 consecutive k of column n
    int bkk[NB], bnn[NB];
    {
      const bool tr = KC || a.transw;
  #pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int v = tid + 256 * u;
        bkk[u] = tr ? (v / BN) * 4 : v / (BN / 4);
        bnn[u] = tr ? v % BN : (v % (BN / 4)) * 4;
      }
    }

    // MODE 0: bounds-checked loads; 1: fast, W row-major; 2: fast, W transposed
    auto load_tiles = [&](int k0, auto mode_tag) {
      constexpr int MODE = decltype(mode_tag)::value;
  #pragma unroll
      for (int u = 0; u < NA; ++u) {
        if (tid + 256 * u >= AV) continue;
        const int k = k0 + akk[u];
        if (MODE != 0 || (aval[u] && avec && k + 3 < a.K)) {
          const Vec t = *(const Vec*)(arow[u] + k);
          ra[u][0] = t.x;
          ra[u][1] = t.y;
          ra[u][2] = t.z;
          ra[u][3] = t.w;
        } else {
  #pragma unroll
          for (int e = 0; e < 4; ++e) ra[u][e] = (aval[u] && k + e < a.K) ? arow[u][k + e] : S(0);
        }
      }
  #pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int v = tid + 256 * u;
        if (v >= BV) continue;
        const int kg = k0 + bkk[u];
        int ng = n0 + bnn[u];
        if (MODE == 1 || (MODE == 0 && !a.transw)) {
          if constexpr (!KC) {
            // 4 consecutive columns of W row kg
            if (MODE == 1) ng = ng < a.Ncols ? ng : a.Ncols - 4;
            const S* src = Wt + (int64_t)kg * a.ldw + ng;
            if (MODE == 1 || (bvec && kg < a.K && ng + 3 < a.Ncols)) {
              const Vec t = *(const Vec*)src;
              rb[u][0] = t.x;
              rb[u][1] = t.y;
              rb[u][2] = t.z;
              rb[u][3] = t.w;
            } else {
  #pragma unroll
              for (int e = 0; e < 4; ++e) rb[u][e] = (kg < a.K && ng + e < a.Ncols) ? src[e] : S(0);
            }
          } else {
            // 4 consecutive k of column ng (strided by ldw)
            if (MODE == 1) ng = ng < a.Ncols ? ng : a.Ncols - 1;
            const S* src = Wt + (int64_t)kg * a.ldw + ng;
  #pragma unroll
            for (int e = 0; e < 4; ++e)
              rb[u][e] = (MODE == 1 || (ng < a.Ncols && kg + e < a.K)) ? src[(int64_t)e * a.ldw] : S(0);
          }
        } else {
          // 4 consecutive k of W^T column ng
          if (MODE == 2) ng = ng < a.Ncols ? ng : a.Ncols - 1;
          const S* src = Wt + (int64_t)ng * a.ldw + kg;
          if (MODE == 2 || (bvec && ng < a.Ncols && kg + 3 < a.K)) {
            const Vec t = *(const Vec*)src;
            rb[u][0] = t.x;
            rb[u][1] = t.y;
            rb[u][2] = t.z;
            rb[u][3] = t.w;
          } else {
  #pragma unroll
            for (int e = 0; e < 4; ++e) rb[u][e] = (ng < a.Ncols && kg + e < a.K) ? src[e] : S(0);
          }
        }
      }
    };
    auto store_tiles = [&](int buf) {
  #pragma unroll
      for (int u = 0; u < NA; ++u) {
        if (tid + 256 * u >= AV) continue;
        L* dst = &As[buf * ASZ + arr[u] * ALD + akk[u]];
        if constexpr (X3) {
  #pragma unroll
          for (int e = 0; e < 4; ++e) split3(ra[u][e], dst[e], dst[ASZ + e], dst[2 * ASZ + e]);
        } else if constexpr (BF) {
  #pragma unroll
          for (int e = 0; e < 4; ++e) dst[e] = (L)ra[u][e];
        } else {
          *(Vec*)dst = Vec{ra[u][0], ra[u][1], ra[u][2], ra[u][3]};
        }
      }
  #pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int v = tid + 256 * u;
        if (v >= BV) continue;
        const int kk = bkk[u], nn = bnn[u];
        if constexpr (X3) {
          *(Vec*)&Bf[nn * BLD + kk] = Vec{rb[u][0], rb[u][1], rb[u][2], rb[u][3]};
        } else if constexpr (BF) {
          L* dst = &Bs[buf * BSZ + nn * BLD + kk];
  #pragma unroll
          for (int e = 0; e < 4; ++e) dst[e] = (L)rb[u][e];
        } else {
          if (!a.transw) {
            *(Vec*)&Bs[buf * BSZ + kk * BLD + nn] = Vec{rb[u][0], rb[u][1], rb[u][2], rb[u][3]};
          } else {
  #pragma unroll
            for (int e = 0; e < 4; ++e) Bs[buf * BSZ + (kk + e) * BLD + nn] = rb[u][e];
          }
        }
      }
    };

    Acc acc[MB][2];
  #pragma unroll
    for (int i = 0; i < MB; ++i)
  #pragma unroll
      for (int j = 0; j < 2; ++j)
  #pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

    const int g = lane >> 4, c = lane & 15;
    const int nk = (a.K + BK - 1) / BK;

    auto mainloop = [&](auto mode_tag) {
      load_tiles(0, mode_tag);
      store_tiles(0);
      __syncthreads();
      if constexpr (X3) {
        for (int kt = 0; kt < nk; ++kt) {
          if (kt + 1 < nk) load_tiles((kt + 1) * BK, mode_tag);
          // the wave's two B fragments (columns wave*32 + nb*16 + c, k = 8g .. 8g + 7), split once
          bf16x8 bp[2][3];
  #pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            const float* src = &Bf[(wave * 32 + nb * 16 + c) * BLD + 8 * g];
            const f4 lo = *(const f4*)src, hi = *(const f4*)(src + 4);
  #pragma unroll
            for (int j = 0; j < 8; ++j) {
              __bf16 p0, p1, p2;
              split3(j < 4 ? lo[j] : hi[j - 4], p0, p1, p2);
              bp[nb][0][j] = p0;
              bp[nb][1][j] = p1;
              bp[nb][2][j] = p2;
            }
          }
  #pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const int ao = (mb * 16 + c) * ALD + 8 * g;
            const bf16x8 a0 = *(const bf16x8*)&As[ao], a1 = *(const bf16x8*)&As[ASZ + ao],
                         a2 = *(const bf16x8*)&As[2 * ASZ + ao];
            // smallest products first; two independent chains (nb) interleaved
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bp[nb][0], acc[mb][nb], 0, 0, 0);
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bp[nb][1], acc[mb][nb], 0, 0, 0);
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bp[nb][2], acc[mb][nb], 0, 0, 0);
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bp[nb][0], acc[mb][nb], 0, 0, 0);
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bp[nb][1], acc[mb][nb], 0, 0, 0);
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bp[nb][0], acc[mb][nb], 0, 0, 0);
          }
          if (kt + 1 < nk) {
            __syncthreads();  // every wave is done with the stage
            store_tiles(0);
          }
          __syncthreads();
        }
        return;
      }
      for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load_tiles((kt + 1) * BK, mode_tag);
        const L* Ac = As + cur * ASZ;
        const L* Bc = Bs + cur * BSZ;
        if constexpr (BF) {
          bf16x8 bv[2];
  #pragma unroll
          for (int nb = 0; nb < 2; ++nb) bv[nb] = *(const bf16x8*)&Bc[(wave * 32 + nb * 16 + c) * BLD + 8 * g];
  #pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const bf16x8 av = *(const bf16x8*)&Ac[(mb * 16 + c) * ALD + 8 * g];
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nb], acc[mb][nb], 0, 0, 0);
          }
        } else {
          // lane group g supplies k = 4g + kq at MFMA step kq (the same order for A and B)
  #pragma unroll
          for (int k4 = 0; k4 < BK / 16; ++k4) {
            S bq[2][4];
  #pragma unroll
            for (int nb = 0; nb < 2; ++nb)
  #pragma unroll
              for (int kq = 0; kq < 4; ++kq) bq[nb][kq] = Bc[(k4 * 16 + 4 * g + kq) * BLD + wave * 32 + nb * 16 + c];
  #pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
              const Vec av = *(const Vec*)&Ac[(mb * 16 + c) * ALD + k4 * 16 + 4 * g];
  #pragma unroll
              for (int nb = 0; nb < 2; ++nb) {
                if constexpr (KIND == GK_F64) {
                  acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bq[nb][0], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bq[nb][1], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.z, bq[nb][2], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.w, bq[nb][3], acc[mb][nb], 0, 0, 0);
                } else {
                  acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bq[nb][0], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bq[nb][1], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bq[nb][2], acc[mb][nb], 0, 0, 0);
                  acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bq[nb][3], acc[mb][nb], 0, 0, 0);
                }
              }
            }
          }
        }
        if (kt + 1 < nk) store_tiles(cur ^ 1);
        __syncthreads();
      }
    };
    if (fast && !a.transw)
      mainloop(std::integral_constant<int, 1>{});
    else if (fast)
      mainloop(std::integral_constant<int, 2>{});
    else
      mainloop(std::integral_constant<int, 0>{});

    // ---------------- epilogue ----------------
    // The loop ended with a barrier after the last LDS reads, so the stage buffers can be reused.
    const S* __restrict__ bias = (const S*)a.bias;
    const S* __restrict__ Res = (const S*)a.Res;
    const S* __restrict__ Aux = (const S*)a.aux;
    S* __restrict__ Y = (S*)a.Y;
    S* const Cw = (S*)smem + wave * NCP * CLD;
    const int cl = lane % NCP, sub = lane / NCP;

  #pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      if (pass > 0) __syncthreads();  // the previous pass's reads are done
  #pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        if (NPASS == 2 && nb != pass) continue;
        const int ccol = (NPASS == 1 ? nb * 16 : 0) + c;
  #pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          if constexpr (KIND == GK_F64) {
  #pragma unroll
            for (int i = 0; i < 4; ++i) Cw[ccol * CLD + mb * 16 + g + 4 * i] = acc[mb][nb][i];
          } else {
            *(f4*)&Cw[ccol * CLD + mb * 16 + 4 * g] = acc[mb][nb];
          }
        }
      }
      __syncthreads();

      const int col = n0 + wave * 32 + pass * NCP + cl;
      const bool cvalid = col < a.Ncols;
      const S b = (bias && cvalid) ? bias[col] : S(0);
      const S* Cc = Cw + cl * CLD;

      if constexpr (EPI == 0 || EPI == 1) {
        // a run of R0 consecutive rows per lane
        constexpr int R0 = BM / LPC;
        const int64_t rs = m0 + sub * R0;
        const uint32_t rpw = (uint32_t)a.yrpw;
        uint32_t qb = (uint32_t)rs / rpw, rem = (uint32_t)rs - qb * rpw;
        auto next_off = [&]() {
          const int64_t off = (int64_t)qb * a.yws + (int64_t)rem * a.ldy + col;
          if (++rem == rpw) {
            rem = 0;
            ++qb;
          }
          return off;
        };
        if (cvalid) {
          if constexpr (EPI == 0) {
  #pragma unroll 4
            for (int r = 0; r < R0; ++r) {
              if (rs + r >= a.rows) break;
              const int64_t off = next_off();
              const S z = Cc[sub * R0 + r] + b;
              S o = a.act == 1 ? dtanh(z) : z;
              if (a.act == 2) {
                const S t = Aux[off];
                o *= S(1) - t * t;
              }
              if (Res) o += Res[off];
              Y[off] = o;
            }
          } else {
            // univariate jets: groups of 4 rows (value, first, second derivative, pad)
            for (int r = 0; r < R0; r += 4) {
              if (rs + r >= a.rows) break;
              const S z0 = Cc[sub * R0 + r] + b, z1 = Cc[sub * R0 + r + 1], z2 = Cc[sub * R0 + r + 2];
              S o[4] = {z0, z1, z2, S(0)};
              if (a.act) {
                const S t = dtanh(z0), t1 = S(1) - t * t, t2 = S(-2) * t * t1;
                o[0] = t;
                o[1] = t1 * z1;
                o[2] = t1 * z2 + t2 * z1 * z1;
              }
  #pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int64_t off = next_off();
                Y[off] = Res ? o[e] + Res[off] : o[e];
              }
            }
          }
        }
      } else {
        // EPI == 2: groups of Rp rows; a lane takes whole groups, or one part of a group when the
        // tile has fewer groups than lanes per column
        const int Rp = a.Rp, T = a.T;
        const int Gt = BM / Rp;                    // groups in the tile (1, 2, 4 or 8)
        const int PPG = Gt >= LPC ? 1 : LPC / Gt;  // lanes per group
        const int GPL = Gt >= LPC ? Gt / LPC : 1;  // groups per lane
        const int rpp = Rp / PPG;
        const S* __restrict__ A5 = (const S*)a.add5;
        for (int j = 0; j < GPL; ++j) {
          const int grp = PPG == 1 ? sub + LPC * j : sub / PPG;
          const int part = PPG == 1 ? 0 : sub % PPG;
          const int qlo = part * rpp;
          const int64_t rg = m0 + (int64_t)grp * Rp;  // first row of the group
          const bool gvalid = cvalid && rg < a.rows;
          const int64_t gidx = rg / Rp;
          const int el = A5 ? (int)(gidx % a.nel) : -1;
          const S* Cg = Cc + grp * Rp;
          // One pass over the group's rows: the value row gives t, t' and t''; a gradient row's
          // output needs only t', so it is written as its pre-activation is read, while the
          // squares are summed for the Laplacian row, which is written last.  The bias enters the
          // value row only; the nuclear five-row term enters the value row, the electron's own
          // three coordinate rows and the Laplacian row.
          S ssq = 0, t = 0, t1 = 1, t2 = 0, a5c0 = 0, a5c1 = 0, a5c2 = 0, a5l = 0;
          int q5 = -8;  // first own-coordinate row of the group's electron
          int64_t base = 0;
          if (gvalid) {
            S z0 = Cg[0] + b;
            if (A5) {
              const S* a5 = A5 + gidx * 5 * a.Ncols + col;
              z0 += a5[0];
              a5c0 = a5[a.Ncols];
              a5c1 = a5[2 * a.Ncols];
              a5c2 = a5[3 * a.Ncols];
              a5l = a5[4 * a.Ncols];
              q5 = 1 + 3 * el;
            }
            t = z0;
            if (a.act) {
              t = dtanh(z0);
              t1 = S(1) - t * t;
              t2 = S(-2) * t * t1;
            }
            const uint32_t rpw = (uint32_t)a.yrpw;
            const uint32_t qb = (uint32_t)rg / rpw;
            base = (int64_t)qb * a.yws + (int64_t)((uint32_t)rg - qb * rpw) * a.ldy + col;
            // runs of 4 rows: the residual loads of a run are issued before its outputs are formed
            for (int q0 = qlo; q0 < qlo + rpp; q0 += 4) {
              S rv[4] = {S(0), S(0), S(0), S(0)};
              if (Res) {
  #pragma unroll
                for (int u = 0; u < 4; ++u) rv[u] = Res[base + (int64_t)(q0 + u) * a.ldy];
              }
  #pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int q = q0 + u;
                S z = Cg[q];
                const int d5 = q - q5;
                if (d5 >= 0 && d5 < 3) z += d5 == 0 ? a5c0 : (d5 == 1 ? a5c1 : a5c2);
                S o = 0;
                if (q == 0) {
                  o = t;
                } else if (q <= T) {
                  ssq += z * z;
                  o = t1 * z;
                }
                if (q != T + 1) Y[base + (int64_t)q * a.ldy] = o + rv[u];
              }
            }
          }
          for (int o = 1; o < PPG; o <<= 1) ssq += __shfl_xor(ssq, NCP * o);
          if (gvalid && T + 1 >= qlo && T + 1 < qlo + rpp) {
            const int64_t off = base + (int64_t)(T + 1) * a.ldy;
            S o = t1 * (Cg[T + 1] + a5l) + t2 * ssq;
            if (Res) o += Res[off];
            Y[off] = o;
          }
        }
      }
    }
  };
  if constexpr (PERSIST) {
    const int64_t nbx = (a.rows + BM - 1) / BM;
    for (int64_t bx = blockIdx.x; bx < nbx; bx += gridDim.x) {
      if (bx != (int64_t)blockIdx.x) __syncthreads();  // the previous tile's epilogue reads are done
      row_tile(bx);
    }
  } else {
    row_tile(blockIdx.x);
  }
}

struct GemmNames {
  char n[4][17][3][40];
};

static const char* gemm_name(int kind, int mb, int epi) {
  static const GemmNames names = [] {
    const char* kn[4] = {"f64", "f32", "bf16", "f32x3"};
    const char* en[3] = {"val", "edge", "jet"};
    GemmNames g;
    for (int k = 0; k < 4; ++k)
      for (int m = 0; m < 17; ++m)
        for (int e = 0; e < 3; ++e) snprintf(g.n[k][m][e], 40, "gemm_kernel<%s,%d,%s>", kn[k], m, en[e]);
    return g;
  }();
  return names.n[kind][mb][epi];
}

int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n > 0) return n;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  cache[dev].store(n, std::memory_order_relaxed);
  return n;
}

template <int KIND, int MB, int EPI, int BKT, bool PERSIST>
static hipError_t launch_grid(const GemmArgs& a, hipStream_t st) {
  ProfScope ps(gemm_name(KIND, MB, EPI), st);
  constexpr int BM = 16 * MB;
  const int64_t nbx = (a.rows + BM - 1) / BM;
  const unsigned gy = (unsigned)((a.Ncols + 127) / 128);
  int64_t gx = nbx;
  if constexpr (PERSIST) {
    // as many blocks as fit on the device at once, each walking row tiles with a grid stride (the
    // kernel's resident blocks per compute unit, queried once per device)
    static std::atomic<int> occ_cache[64];
    int dev = 0, occ = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) occ = occ_cache[dev].load(std::memory_order_relaxed);
    if (occ < 1) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gemm_kernel<KIND, MB, EPI, BKT, true>, 256, 0) !=
              hipSuccess ||
          occ < 1)
        occ = 1;
      if (dev >= 0 && dev < 64) occ_cache[dev].store(occ, std::memory_order_relaxed);
    }
    const int64_t slots = (int64_t)occ * device_cus() / gy;
    gx = std::max<int64_t>(1, std::min<int64_t>(nbx, slots));
  }
  hipLaunchKernelGGL((gemm_kernel<KIND, MB, EPI, BKT, PERSIST>), dim3((unsigned)gx, gy), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Persistent variants are instantiated for float32 only (the other kinds ignore the bit).
template <int KIND, int MB, int EPI, int BKT>
static hipError_t launch_mb(const GemmArgs& a, bool persist, hipStream_t st) {
  if constexpr (KIND == GK_F32 || KIND == GK_F32X3)
    if (persist) return launch_grid<KIND, MB, EPI, BKT, true>(a, st);
  return launch_grid<KIND, MB, EPI, BKT, false>(a, st);
}

// Tile choice (GemmArgs::tile - 1 when nonzero, or QMC_GEMM_TILE=<bits> for tuning runs): bit 0
// selects 32-wide K stages for float32, bit 1 half-height (64-row) value and edge tiles, bit 2 a
// persistent grid (float32), bit 3 float32 on the bf16 matrix cores (three-piece operands, 32-wide
// K stages).  The default takes half-height tiles when full ones would give fewer than 4
// blocks per compute unit.
static int tile_bits(const GemmArgs& a) {
  static const int env = [] {
    const char* e = getenv("QMC_GEMM_TILE");
    return e ? atoi(e) & 15 : -1;
  }();
  if (env >= 0) return env;
  if (a.tile > 0) return (a.tile - 1) & 15;
  const int64_t blocks = ((a.rows + 127) / 128) * ((a.Ncols + 127) / 128);
  return (a.vmode || a.Rp == 4) && blocks < 4 * 256 ? 2 : 0;
}

template <int KIND, int BKT>
static hipError_t launch_kind_bk(const GemmArgs& a, int bits, hipStream_t st) {
  const bool half = (bits & 2) != 0, persist = (bits & 4) != 0;
  if (a.vmode)
    return half ? launch_mb<KIND, 4, 0, BKT>(a, persist, st) : launch_mb<KIND, 8, 0, BKT>(a, persist, st);
  if (a.Rp == 4)
    return half ? launch_mb<KIND, 4, 1, BKT>(a, persist, st) : launch_mb<KIND, 8, 1, BKT>(a, persist, st);
  // a tile holds whole jet groups: as many as fit in 128 rows, or one group of up to 208 rows
  // (3N + 2 rows for up to 64 electrons)
  if (a.Rp % 16 != 0 || a.Rp > 208) return hipErrorInvalidValue;
  const int bpg = a.Rp / 16;
  switch (bpg <= 8 ? bpg * (8 / bpg) : bpg) {
    case 5: return launch_mb<KIND, 5, 2, BKT>(a, persist, st);
    case 6: return launch_mb<KIND, 6, 2, BKT>(a, persist, st);
    case 7: return launch_mb<KIND, 7, 2, BKT>(a, persist, st);
    case 8: return launch_mb<KIND, 8, 2, BKT>(a, persist, st);
    case 9: return launch_mb<KIND, 9, 2, BKT>(a, persist, st);
    case 10: return launch_mb<KIND, 10, 2, BKT>(a, persist, st);
    case 11: return launch_mb<KIND, 11, 2, BKT>(a, persist, st);
    case 12: return launch_mb<KIND, 12, 2, BKT>(a, persist, st);
    case 13: return launch_mb<KIND, 13, 2, BKT>(a, persist, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(GemmKind kind, const GemmArgs& a, hipStream_t st) {
  if (a.rows <= 0 || a.Ncols <= 0) return hipSuccess;
  // row indices and rows-per-block are handled in 32 bits inside the kernel
  if (a.rows >= (int64_t(1) << 31) || a.xrpw <= 0 || a.yrpw <= 0 || a.xrpw >= (int64_t(1) << 31) ||
      a.yrpw >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  if (!a.vmode && a.Rp == 4 && (a.T != 1 || a.rows % 4 != 0 || a.yrpw % 4 != 0)) return hipErrorInvalidValue;
  // electron jets: whole groups of Rp rows, none straddling an output row block
  if (!a.vmode && a.Rp != 4 && (a.Rp < 16 || a.rows % a.Rp != 0 || a.yrpw % a.Rp != 0)) return hipErrorInvalidValue;
  if (a.act == 2 && (!a.vmode || !a.aux)) return hipErrorInvalidValue;
  if (a.add5 && (a.vmode || a.Rp < 16 || a.nel < 1 || a.xrpw != a.rows || a.yrpw != a.rows))
    return hipErrorInvalidValue;
  const int bits = tile_bits(a);
  switch (kind) {
    case GK_F64: return launch_kind_bk<GK_F64, 16>(a, bits, st);
    case GK_F32:
      if (bits & 8) return launch_kind_bk<GK_F32X3, 32>(a, bits, st);
      return (bits & 1) ? launch_kind_bk<GK_F32, 32>(a, bits, st) : launch_kind_bk<GK_F32, 16>(a, bits, st);
    case GK_BF16: return launch_kind_bk<GK_BF16, 32>(a, bits, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qmc
