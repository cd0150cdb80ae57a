// MFMA GEMM over jet rows with a fused tanh-jet epilogue (gfx950).
//
// A layer y = x W + b applied to a jet (value, gradient rows, Laplacian row)
// maps every row through W and adds b to the value row only.  The tanh that
// follows needs, per (electron, column), the sum over gradient rows of the
// squared pre-activation: t = tanh(z0), grad t = t' grad z,
// lap t = t' lap z + t'' |grad z|^2 with t' = 1 - t^2, t'' = -2 t t'.
// Tiles therefore hold whole row groups (BM is a multiple of the group
// size) so that this reduction stays inside one wavefront: each wave owns all
// BM rows of its 32 output columns, reduces its own accumulator rows and
// finishes with two cross-lane shuffles.
//
// MFMA shapes: f64 v_mfma_f64_16x16x4, f32 v_mfma_f32_16x16x4, bf16
// v_mfma_f32_16x16x32 (operands rounded to bf16, float accumulation).  The
// 16x16 accumulator layouts: f32/bf16: lane l, element i -> row 4*(l/16)+i,
// column l%16; f64: row (l/16)+4*i, column l%16.  Operand layout: lane l supplies row (A) / column (B) l%16 and the
// k-slice selected by l/16; A and B use the same k assignment, so the
// contraction is independent of how the hardware orders k within a lane.
#include "kernels.h"

namespace qmc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND> struct GT;
template <> struct GT<GK_F64> {
  using S = double;
  using Acc = d4;
  using L = double;  // LDS element
  static constexpr int BK = 16;
};
template <> struct GT<GK_F32> {
  using S = float;
  using Acc = f4;
  using L = float;
  static constexpr int BK = 16;
};
template <> struct GT<GK_BF16> {
  using S = float;
  using Acc = f4;
  using L = __bf16;
  static constexpr int BK = 32;
};

__device__ inline double dtanh(double x) { return tanh(x); }
__device__ inline float dtanh(float x) { return tanhf(x); }

template <int KIND, int MB>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  using G = GT<KIND>;
  using S = typename G::S;
  using Acc = typename G::Acc;
  using L = typename G::L;
  constexpr int BK = G::BK;
  constexpr int BM = 16 * MB;
  constexpr int BN = 128;
  constexpr int APAD = (KIND == GK_BF16) ? 8 : 1;
  constexpr int BPAD = (KIND == GK_BF16) ? 8 : 16;
  // A tile [BM][BK+APAD]; B tile [BK][BN+BPAD] (f32/f64) or transposed [BN][BK+BPAD] (bf16)
  __shared__ L As[BM * (BK + APAD)];
  __shared__ L Bs[(KIND == GK_BF16) ? BN * (BK + BPAD) : BK * (BN + BPAD)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const S* __restrict__ X = (const S*)a.X;
  const S* __restrict__ Wt = (const S*)a.W;

  // each thread loads a fixed column kk of the A tile for rows rbase + s*RSTEP
  constexpr int RSTEP = 256 / BK;
  constexpr int APASS = BM / RSTEP;
  const int akk = tid % BK;
  const int arow0 = tid / BK;
  const S* xrow[APASS];
  bool rvalid[APASS];
#pragma unroll
  for (int s = 0; s < APASS; ++s) {
    const int64_t r = m0 + arow0 + s * RSTEP;
    rvalid[s] = r < a.rows;
    const int64_t rr = rvalid[s] ? r : 0;
    xrow[s] = X + (rr / a.xrpw) * a.xws + (rr % a.xrpw) * a.ldx;
  }

  Acc acc[MB][2];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  for (int k0 = 0; k0 < a.K; k0 += BK) {
    const int k = k0 + akk;
#pragma unroll
    for (int s = 0; s < APASS; ++s) {
      S v = (rvalid[s] && k < a.K) ? xrow[s][k] : S(0);
      As[(arow0 + s * RSTEP) * (BK + APAD) + akk] = (L)v;
    }
    for (int e = tid; e < BK * BN; e += 256) {
      int kk, n;
      if (a.transw) {
        n = e / BK;
        kk = e % BK;
      } else {
        kk = e / BN;
        n = e % BN;
      }
      const int kg = k0 + kk, ng = n0 + n;
      S v = 0;
      if (kg < a.K && ng < a.Ncols) v = a.transw ? Wt[(int64_t)ng * a.ldw + kg] : Wt[(int64_t)kg * a.ldw + ng];
      if (KIND == GK_BF16)
        Bs[n * (BK + BPAD) + kk] = (L)v;
      else
        Bs[kk * (BN + BPAD) + n] = (L)v;
    }
    __syncthreads();
    if constexpr (KIND == GK_BF16) {
      const int g = lane >> 4, c = lane & 15;
      bf16x8 bv[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        bv[nb] = *(const bf16x8*)&Bs[(wave * 32 + nb * 16 + c) * (BK + BPAD) + 8 * g];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const bf16x8 av = *(const bf16x8*)&As[(mb * 16 + c) * (BK + APAD) + 8 * g];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nb], acc[mb][nb], 0, 0, 0);
      }
    } else {
      const int g = lane >> 4, c = lane & 15;
#pragma unroll
      for (int kq = 0; kq < BK / 4; ++kq) {
        L bv[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bv[nb] = Bs[(kq * 4 + g) * (BN + BPAD) + wave * 32 + nb * 16 + c];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const L av = As[(mb * 16 + c) * (BK + APAD) + kq * 4 + g];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            if constexpr (KIND == GK_F64)
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[nb], acc[mb][nb], 0, 0, 0);
            else
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[nb], acc[mb][nb], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // ---------------- epilogue ----------------
  // row (inside a 16-row block) of accumulator element i of this lane
  auto rowof = [&](int g, int i) -> int { return KIND == GK_F64 ? g + 4 * i : 4 * g + i; };
  const S* __restrict__ bias = (const S*)a.bias;
  const S* __restrict__ Res = (const S*)a.Res;
  S* __restrict__ Y = (S*)a.Y;
  const int g4 = lane >> 4;
  const int c16 = lane & 15;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = n0 + wave * 32 + nb * 16 + c16;
    const bool cvalid = col < a.Ncols;
    const S b = (bias && cvalid) ? bias[col] : S(0);
    S out[MB][4];
    if (a.vmode) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const S z = acc[mb][nb][i] + b;
          out[mb][i] = a.act == 1 ? dtanh(z) : z;
        }
    } else if (a.Rp == 4) {
      // univariate jets: groups of 4 rows (value, first, second derivative, pad)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        if constexpr (KIND == GK_F64) {
          // element i of lane group g4 holds row 4*i + g4: the group is spread over the 4 lane groups
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const S z0 = __shfl(acc[mb][nb][i], c16) + b, z1 = __shfl(acc[mb][nb][i], c16 + 16),
                    z2 = __shfl(acc[mb][nb][i], c16 + 32);
            S o0 = z0, o1 = z1, o2 = z2;
            if (a.act) {
              const S t = dtanh(z0), t1 = S(1) - t * t, t2 = S(-2) * t * t1;
              o0 = t;
              o1 = t1 * z1;
              o2 = t1 * z2 + t2 * z1 * z1;
            }
            out[mb][i] = g4 == 0 ? o0 : (g4 == 1 ? o1 : (g4 == 2 ? o2 : S(0)));
          }
        } else {
          // one lane holds a whole group
          const S z0 = acc[mb][nb][0] + b, z1 = acc[mb][nb][1], z2 = acc[mb][nb][2];
          if (a.act) {
            const S t = dtanh(z0), t1 = S(1) - t * t, t2 = S(-2) * t * t1;
            out[mb][0] = t;
            out[mb][1] = t1 * z1;
            out[mb][2] = t1 * z2 + t2 * z1 * z1;
          } else {
            out[mb][0] = z0;
            out[mb][1] = z1;
            out[mb][2] = z2;
          }
          out[mb][3] = 0;
        }
      }
    } else {
      // groups of Rp = 16*bpg rows spanning whole 16-row blocks
      const int bpg = a.Rp >> 4;
      S ssq[MB], z0b[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        S s = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = (mb * 16 + rowof(g4, i)) % a.Rp;
          if (q >= 1 && q <= a.T) s += acc[mb][nb][i] * acc[mb][nb][i];
        }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        ssq[mb] = s;
        z0b[mb] = __shfl(acc[mb][nb][0], c16) + b;  // row 0 of this block (value row if block starts a group)
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int grp = mb / bpg;
        S S2 = 0, z0 = 0;
#pragma unroll
        for (int mq = 0; mq < MB; ++mq) {
          if (mq / bpg == grp) S2 += ssq[mq];
          if (mq == grp * bpg) z0 = z0b[mq];
        }
        S t = z0, t1 = 1, t2 = 0;
        if (a.act) {
          t = dtanh(z0);
          t1 = S(1) - t * t;
          t2 = S(-2) * t * t1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = (mb * 16 + rowof(g4, i)) % a.Rp;
          S o;
          if (q == 0)
            o = t;
          else if (q <= a.T)
            o = t1 * acc[mb][nb][i];
          else if (q == a.T + 1)
            o = t1 * acc[mb][nb][i] + t2 * S2;
          else
            o = 0;
          out[mb][i] = o;
        }
      }
    }
    if (cvalid) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t r = m0 + mb * 16 + rowof(g4, i);
          if (r < a.rows) {
            const int64_t off = (r / a.yrpw) * a.yws + (r % a.yrpw) * a.ldy + col;
            S o = out[mb][i];
            if (a.act == 2) {
              const S t = ((const S*)a.aux)[off];
              o *= S(1) - t * t;
            }
            if (Res) o += Res[off];
            Y[off] = o;
          }
        }
    }
  }
}

static const char* gemm_name(int kind, int mb) {
  static const char* names[3][9] = {
      {"", "", "", "", "", "gemm_kernel<f64,5>", "gemm_kernel<f64,6>", "gemm_kernel<f64,7>", "gemm_kernel<f64,8>"},
      {"", "", "", "", "", "gemm_kernel<f32,5>", "gemm_kernel<f32,6>", "gemm_kernel<f32,7>", "gemm_kernel<f32,8>"},
      {"", "", "", "", "", "gemm_kernel<bf16,5>", "gemm_kernel<bf16,6>", "gemm_kernel<bf16,7>",
       "gemm_kernel<bf16,8>"}};
  return names[kind][mb];
}

template <int KIND, int MB>
static hipError_t launch_mb(const GemmArgs& a, hipStream_t st) {
  ProfScope ps(gemm_name(KIND, MB), st);
  constexpr int BM = 16 * MB;
  dim3 grid((unsigned)((a.rows + BM - 1) / BM), (unsigned)((a.Ncols + 127) / 128));
  hipLaunchKernelGGL((gemm_kernel<KIND, MB>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_kind(const GemmArgs& a, hipStream_t st) {
  int mb = 8;
  if (!a.vmode && a.Rp != 4) {
    if (a.Rp % 16 != 0 || a.Rp > 128) return hipErrorInvalidValue;
    const int bpg = a.Rp / 16;
    mb = bpg * (8 / bpg);
  }
  switch (mb) {
    case 5: return launch_mb<KIND, 5>(a, st);
    case 6: return launch_mb<KIND, 6>(a, st);
    case 7: return launch_mb<KIND, 7>(a, st);
    case 8: return launch_mb<KIND, 8>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm(GemmKind kind, const GemmArgs& a, hipStream_t st) {
  if (a.rows <= 0 || a.Ncols <= 0) return hipSuccess;
  if (!a.vmode && a.Rp == 4 && a.T != 1) return hipErrorInvalidValue;
  if (a.act == 2 && (!a.vmode || !a.aux)) return hipErrorInvalidValue;
  switch (kind) {
    case GK_F64: return launch_kind<GK_F64>(a, st);
    case GK_F32: return launch_kind<GK_F32>(a, st);
    case GK_BF16: return launch_kind<GK_BF16>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qmc
