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
// Pipeline: two LDS stages; the next K-slice is fetched from global memory
// into registers (16-byte vectors where the layout allows) while the MFMAs
// consume the current stage, so each K-step needs one barrier.
//
// MFMA shapes: f64 v_mfma_f64_16x16x4, f32 v_mfma_f32_16x16x4, bf16
// v_mfma_f32_16x16x32 (operands rounded to bf16, float accumulation).  The
// 16x16 accumulator layouts: f32/bf16: lane l, element i -> row 4*(l/16)+i,
// column l%16; f64: row (l/16)+4*i, column l%16.  Operand layout: lane l
// supplies row (A) / column (B) l%16 and the k-slice selected by l/16; A and
// B use the same k assignment, so the contraction does not depend on how the
// hardware orders k inside a lane.
#include <cstdio>

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

template <typename S> struct V4;
template <> struct V4<float> {
  using T = float4;
};
template <> struct V4<double> {
  using T = double4;
};

__device__ inline double dtanh(double x) { return tanh(x); }
__device__ inline float dtanh(float x) { return tanhf(x); }

// EPI: 0 value rows, 1 univariate edge jets (groups of 4 rows), 2 electron jets (groups of Rp = 16*bpg rows)
template <int KIND, int MB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  using G = GT<KIND>;
  using S = typename G::S;
  using Acc = typename G::Acc;
  using L = typename G::L;
  using Vec = typename V4<S>::T;
  constexpr int BK = G::BK;
  constexpr int BM = 16 * MB;
  constexpr int BN = 128;
  constexpr int APAD = (KIND == GK_BF16) ? 8 : (KIND == GK_F64 ? 1 : 4);
  constexpr int BPAD = (KIND == GK_BF16) ? 8 : 16;
  constexpr int ALD = BK + APAD;  // A tile row stride
  constexpr int BLD = (KIND == GK_BF16) ? BK + BPAD : BN + BPAD;
  constexpr int ASZ = BM * ALD;
  constexpr int BSZ = (KIND == GK_BF16) ? BN * BLD : BK * BLD;
  __shared__ L As[2][ASZ];
  __shared__ L Bs[2][BSZ];

  // global -> register slots: A has BM*BK/4 vectors, B has BK*BN/4
  constexpr int AV = BM * BK / 4, BV = BK * BN / 4;
  constexpr int NA = (AV + 255) / 256, NB = (BV + 255) / 256;
  constexpr int AKV = BK / 4;  // vectors per A row

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const S* __restrict__ X = (const S*)a.X;
  const S* __restrict__ Wt = (const S*)a.W;
  const bool avec = (a.ldx % 4 == 0) && (a.K % 4 == 0) && ((a.xws % 4) == 0) &&
                    ((reinterpret_cast<uintptr_t>(X) % (4 * sizeof(S))) == 0);
  const bool bvec = (a.ldw % 4 == 0) && (reinterpret_cast<uintptr_t>(Wt) % (4 * sizeof(S)) == 0) &&
                    (a.transw ? (a.K % 4 == 0) : (a.Ncols % 4 == 0));

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
    const int64_t rr = aval[u] ? r : 0;
    arow[u] = X + (rr / a.xrpw) * a.xws + (rr % a.xrpw) * a.ldx;
  }
  S ra[NA][4], rb[NB][4];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int k = k0 + akk[u];
      if (aval[u] && avec && k + 3 < a.K) {
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
      if (!a.transw) {
        const int kk = v / (BN / 4), n = (v % (BN / 4)) * 4;
        const int kg = k0 + kk, ng = n0 + n;
        const S* src = Wt + (int64_t)kg * a.ldw + ng;
        if (bvec && kg < a.K && ng + 3 < a.Ncols) {
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
        const int n = v / (BK / 4), kk = (v % (BK / 4)) * 4;
        const int kg = k0 + kk, ng = n0 + n;
        const S* src = Wt + (int64_t)ng * a.ldw + kg;
        if (bvec && ng < a.Ncols && kg + 3 < a.K) {
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
#pragma unroll
      for (int e = 0; e < 4; ++e) As[buf][arr[u] * ALD + akk[u] + e] = (L)ra[u][e];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + 256 * u;
      if (v >= BV) continue;
      if (!a.transw) {
        const int kk = v / (BN / 4), n = (v % (BN / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (KIND == GK_BF16)
            Bs[buf][(n + e) * BLD + kk] = (L)rb[u][e];
          else
            Bs[buf][kk * BLD + n + e] = (L)rb[u][e];
        }
      } else {
        const int n = v / (BK / 4), kk = (v % (BK / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (KIND == GK_BF16)
            Bs[buf][n * BLD + kk + e] = (L)rb[u][e];
          else
            Bs[buf][(kk + e) * BLD + n] = (L)rb[u][e];
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
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
    const L* Ac = As[cur];
    const L* Bc = Bs[cur];
    if constexpr (KIND == GK_BF16) {
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
#pragma unroll
      for (int kq = 0; kq < BK / 4; ++kq) {
        L bv[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bv[nb] = Bc[(kq * 4 + g) * BLD + wave * 32 + nb * 16 + c];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const L av = Ac[(mb * 16 + c) * ALD + kq * 4 + g];
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
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  // ---------------- epilogue ----------------
  // row (inside a 16-row block) of accumulator element i of this lane
  auto rowof = [&](int gg, int i) -> int { return KIND == GK_F64 ? gg + 4 * i : 4 * gg + i; };
  const S* __restrict__ bias = (const S*)a.bias;
  const S* __restrict__ Res = (const S*)a.Res;
  S* __restrict__ Y = (S*)a.Y;
  const int g4 = g;
  const int c16 = c;
  // jet groups spanning whole 16-row blocks: block mb is block (mb % bpg) of group mb / bpg
  int qbase[MB], grp[MB];
  const int bpg = (EPI == 2) ? (a.Rp >> 4) : 1;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    grp[mb] = mb / bpg;
    qbase[mb] = (mb - grp[mb] * bpg) * 16;
  }
  auto emit = [&](int mb, int i, int col, S o) {
    const int64_t r = m0 + mb * 16 + rowof(g4, i);
    if (r < a.rows && col < a.Ncols) {
      const int64_t off = (r / a.yrpw) * a.yws + (r % a.yrpw) * a.ldy + col;
      if (a.act == 2) {
        const S t = ((const S*)a.aux)[off];
        o *= S(1) - t * t;
      }
      if (Res) o += Res[off];
      Y[off] = o;
    }
  };
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = n0 + wave * 32 + nb * 16 + c16;
    const bool cvalid = col < a.Ncols;
    const S b = (bias && cvalid) ? bias[col] : S(0);
    if constexpr (EPI == 0) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const S z = acc[mb][nb][i] + b;
          emit(mb, i, col, a.act == 1 ? dtanh(z) : z);
        }
    } else if constexpr (EPI == 1) {
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
            emit(mb, i, col, g4 == 0 ? o0 : (g4 == 1 ? o1 : (g4 == 2 ? o2 : S(0))));
          }
        } else {
          // one lane holds a whole group
          const S z0 = acc[mb][nb][0] + b, z1 = acc[mb][nb][1], z2 = acc[mb][nb][2];
          S o0 = z0, o1 = z1, o2 = z2;
          if (a.act) {
            const S t = dtanh(z0), t1 = S(1) - t * t, t2 = S(-2) * t * t1;
            o0 = t;
            o1 = t1 * z1;
            o2 = t1 * z2 + t2 * z1 * z1;
          }
          emit(mb, 0, col, o0);
          emit(mb, 1, col, o1);
          emit(mb, 2, col, o2);
          emit(mb, 3, col, S(0));
        }
      }
    } else {
      // EPI == 2: groups of Rp = 16*bpg rows spanning whole 16-row blocks
      S ssq[MB], z0b[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        S sq = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = qbase[mb] + rowof(g4, i);
          if (q >= 1 && q <= a.T) sq += acc[mb][nb][i] * acc[mb][nb][i];
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        ssq[mb] = sq;
        z0b[mb] = __shfl(acc[mb][nb][0], c16) + b;  // row 0 of this block (the value row when it starts a group)
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        S S2 = 0, z0 = 0;
#pragma unroll
        for (int mq = 0; mq < MB; ++mq) {
          if (grp[mq] == grp[mb]) S2 += ssq[mq];
          if (grp[mq] == grp[mb] && qbase[mq] == 0) z0 = z0b[mq];
        }
        S t = z0, t1 = 1, t2 = 0;
        if (a.act) {
          t = dtanh(z0);
          t1 = S(1) - t * t;
          t2 = S(-2) * t * t1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = qbase[mb] + rowof(g4, i);
          S o;
          if (q == 0)
            o = t;
          else if (q <= a.T)
            o = t1 * acc[mb][nb][i];
          else if (q == a.T + 1)
            o = t1 * acc[mb][nb][i] + t2 * S2;
          else
            o = 0;
          emit(mb, i, col, o);
        }
      }
    }
  }
}

static const char* gemm_name(int kind, int mb, int epi) {
  static const char* kn[3] = {"f64", "f32", "bf16"};
  static const char* en[3] = {"val", "edge", "jet"};
  static char names[3][9][3][40];
  static bool init = false;
  if (!init) {
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 9; ++m)
        for (int e = 0; e < 3; ++e) snprintf(names[k][m][e], 40, "gemm_kernel<%s,%d,%s>", kn[k], m, en[e]);
    init = true;
  }
  return names[kind][mb][epi];
}

template <int KIND, int MB, int EPI>
static hipError_t launch_mb(const GemmArgs& a, hipStream_t st) {
  ProfScope ps(gemm_name(KIND, MB, EPI), st);
  constexpr int BM = 16 * MB;
  dim3 grid((unsigned)((a.rows + BM - 1) / BM), (unsigned)((a.Ncols + 127) / 128));
  hipLaunchKernelGGL((gemm_kernel<KIND, MB, EPI>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_kind(const GemmArgs& a, hipStream_t st) {
  if (a.vmode) return launch_mb<KIND, 8, 0>(a, st);
  if (a.Rp == 4) return launch_mb<KIND, 8, 1>(a, st);
  if (a.Rp % 16 != 0 || a.Rp > 128) return hipErrorInvalidValue;
  const int bpg = a.Rp / 16;
  switch (bpg * (8 / bpg)) {
    case 5: return launch_mb<KIND, 5, 2>(a, st);
    case 6: return launch_mb<KIND, 6, 2>(a, st);
    case 7: return launch_mb<KIND, 7, 2>(a, st);
    case 8: return launch_mb<KIND, 8, 2>(a, st);
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
