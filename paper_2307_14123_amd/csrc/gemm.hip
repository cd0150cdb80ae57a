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
// Both operand tiles keep k contiguous in LDS ([rows][k] and [columns][k]),
// so one 16-byte LDS read gives a lane its operands of four f32/f64 MFMAs.
//
// MFMA shapes: f64 v_mfma_f64_16x16x4, f32 v_mfma_f32_16x16x4, bf16
// v_mfma_f32_16x16x32 (operands rounded to bf16, float accumulation).  The
// 16x16 accumulator layouts: f32/bf16: lane l, element i -> row 4*(l/16)+i,
// column l%16; f64: row (l/16)+4*i, column l%16.  Operand layout: lane l
// supplies row (A) / column (B) l%16 and the k-slice selected by l/16; A and
// B use the same k assignment, so the contraction does not depend on how the
// hardware orders k inside a lane.
#include <cstdio>
#include <cstdlib>
#include <cstring>

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
template <int KIND, int MB, int EPI, int BKT>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  using G = GT<KIND>;
  using S = typename G::S;
  using Acc = typename G::Acc;
  using L = typename G::L;
  using Vec = typename V4<S>::T;
  constexpr int BK = BKT;
  constexpr int BM = 16 * MB;
  constexpr int BN = 128;
  // A tile [BM][BK+pad] and B tile stored transposed [BN][BK+pad]: k is contiguous in both, so a
  // lane reads its operands for several MFMAs with one 16-byte LDS load
  constexpr int APAD = (KIND == GK_BF16) ? 8 : 4;
  constexpr int ALD = BK + APAD;
  constexpr int BLD = BK + APAD;
  constexpr int ASZ = BM * ALD;
  constexpr int BSZ = BN * BLD;
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
    const uint32_t rr = aval[u] ? (uint32_t)r : 0u, rpw = (uint32_t)a.xrpw;
    const uint32_t qb = rr / rpw;
    arow[u] = X + (int64_t)qb * a.xws + (int64_t)(rr - qb * rpw) * a.ldx;
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
      const int n = v % BN, kk = (v / BN) * 4;  // 4 consecutive k of output column n
      const int kg = k0 + kk, ng = n0 + n;
      if (!a.transw) {
        const S* src = Wt + (int64_t)kg * a.ldw + ng;
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[u][e] = (ng < a.Ncols && kg + e < a.K) ? src[(int64_t)e * a.ldw] : S(0);
      } else {
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
      L* dst = &As[buf][arr[u] * ALD + akk[u]];
      if constexpr (KIND == GK_BF16) {
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
      const int n = v % BN, kk = (v / BN) * 4;
      L* dst = &Bs[buf][n * BLD + kk];
      if constexpr (KIND == GK_BF16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = (L)rb[u][e];
      } else {
        *(Vec*)dst = Vec{rb[u][0], rb[u][1], rb[u][2], rb[u][3]};
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
      // lane group g supplies k = 4g + kq at MFMA step kq (the same order for A and B)
#pragma unroll
      for (int k4 = 0; k4 < BK / 16; ++k4) {
        Vec bv[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bv[nb] = *(const Vec*)&Bc[(wave * 32 + nb * 16 + c) * BLD + k4 * 16 + 4 * g];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const Vec av = *(const Vec*)&Ac[(mb * 16 + c) * ALD + k4 * 16 + 4 * g];
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            if constexpr (KIND == GK_F64) {
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv[nb].x, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv[nb].y, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.z, bv[nb].z, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.w, bv[nb].w, acc[mb][nb], 0, 0, 0);
            } else {
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[nb].x, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv[nb].y, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv[nb].z, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv[nb].w, acc[mb][nb], 0, 0, 0);
            }
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
  // global row group and electron (group mod nel) of each 16-row block, for add5
  int64_t gidx[MB];
  int gel[MB];
  if (EPI == 2 && a.add5) {
    const uint32_t g0 = (uint32_t)m0 / (uint32_t)a.Rp;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      gidx[mb] = (int64_t)g0 + grp[mb];
      gel[mb] = (int)((g0 + (uint32_t)grp[mb]) % (uint32_t)a.nel);
    }
  } else {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      gidx[mb] = 0;
      gel[mb] = 0;
    }
  }
  // output row offsets of this lane's 4*MB rows: one 32-bit division per 16-row block, then
  // stepping through the rows (rows of one lane are consecutive for f32/bf16, 4 apart for f64)
  int64_t yoff[MB][4];
  bool yval[MB][4];
  {
    const uint32_t rpw = (uint32_t)a.yrpw;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t r0 = m0 + mb * 16 + rowof(g4, 0);
      const uint32_t rr = (uint32_t)r0;
      uint32_t qb = rr / rpw, rem = rr - qb * rpw;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        yval[mb][i] = (r0 + (rowof(g4, i) - rowof(g4, 0))) < a.rows;
        yoff[mb][i] = (int64_t)qb * a.yws + (int64_t)rem * a.ldy;
        const uint32_t step = (uint32_t)(rowof(g4, 1) - rowof(g4, 0));
        rem += step;
        while (rem >= rpw) {
          rem -= rpw;
          ++qb;
        }
      }
    }
  }
  auto emit = [&](int mb, int i, int col, S o) {
    if (yval[mb][i] && col < a.Ncols) {
      const int64_t off = yoff[mb][i] + col;
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
      if (a.add5 && cvalid) {
        // the 5 nonzero rows of a term that depends on the electron's own position only
        const S* A5 = (const S*)a.add5;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int e = gel[mb];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = qbase[mb] + rowof(g4, i);
            int k5 = -1;
            if (q == 0)
              k5 = 0;
            else if (q == a.T + 1)
              k5 = 4;
            else if (q >= 1 && q <= a.T && (q - 1) / 3 == e)
              k5 = 1 + (q - 1) % 3;
            if (k5 >= 0 && yval[mb][i]) acc[mb][nb][i] += A5[(gidx[mb] * 5 + k5) * a.Ncols + col];
          }
        }
      }
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
  static char names[3][17][3][40];
  static bool init = false;
  if (!init) {
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 17; ++m)
        for (int e = 0; e < 3; ++e) snprintf(names[k][m][e], 40, "gemm_kernel<%s,%d,%s>", kn[k], m, en[e]);
    init = true;
  }
  return names[kind][mb][epi];
}

template <int KIND, int MB, int EPI, int BKT>
static hipError_t launch_mb(const GemmArgs& a, hipStream_t st) {
  ProfScope ps(gemm_name(KIND, MB, EPI), st);
  constexpr int BM = 16 * MB;
  dim3 grid((unsigned)((a.rows + BM - 1) / BM), (unsigned)((a.Ncols + 127) / 128));
  hipLaunchKernelGGL((gemm_kernel<KIND, MB, EPI, BKT>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// Tile choice: rows per tile (MB blocks of 16) and K per pipeline stage.
// QMC_GEMM_TILE=<mbmul>,<bk> overrides it for tuning runs: mbmul doubles the
// row blocks of jet tiles (and of value/edge tiles), bk in {16, 32}.
static int tile_mul() {
  static int v = -1;
  if (v < 0) {
    v = 1;
    if (const char* e = getenv("QMC_GEMM_TILE")) v = atoi(e) == 2 ? 2 : 1;
  }
  return v;
}
static int tile_bk(int def) {
  static int v = -1;
  if (v < 0) {
    v = 0;
    if (const char* e = getenv("QMC_GEMM_TILE"))
      if (const char* c = strchr(e, ',')) v = atoi(c + 1) == 32 ? 32 : (atoi(c + 1) == 16 ? 16 : 0);
  }
  return v ? v : def;
}

template <int KIND, int BKT>
static hipError_t launch_kind_bk(const GemmArgs& a, hipStream_t st) {
  constexpr bool WIDE = (KIND == GK_F32);  // larger tiles are only instantiated for float32
  const int mul = WIDE ? tile_mul() : 1;
  if (a.vmode) {
    if constexpr (WIDE)
      if (mul == 2) return launch_mb<KIND, 16, 0, BKT>(a, st);
    return launch_mb<KIND, 8, 0, BKT>(a, st);
  }
  if (a.Rp == 4) {
    if constexpr (WIDE)
      if (mul == 2) return launch_mb<KIND, 16, 1, BKT>(a, st);
    return launch_mb<KIND, 8, 1, BKT>(a, st);
  }
  if (a.Rp % 16 != 0 || a.Rp > 128) return hipErrorInvalidValue;
  const int bpg = a.Rp / 16;
  int mb = bpg * (8 / bpg);
  if constexpr (WIDE) {
    if (mul == 2) {
      switch (mb) {
        case 5: return launch_mb<KIND, 10, 2, BKT>(a, st);
        case 6: return launch_mb<KIND, 12, 2, BKT>(a, st);
        case 7: return launch_mb<KIND, 14, 2, BKT>(a, st);
        case 8: return launch_mb<KIND, 16, 2, BKT>(a, st);
      }
    }
  }
  switch (mb) {
    case 5: return launch_mb<KIND, 5, 2, BKT>(a, st);
    case 6: return launch_mb<KIND, 6, 2, BKT>(a, st);
    case 7: return launch_mb<KIND, 7, 2, BKT>(a, st);
    case 8: return launch_mb<KIND, 8, 2, BKT>(a, st);
  }
  return hipErrorInvalidValue;
}

template <int KIND>
static hipError_t launch_kind(const GemmArgs& a, hipStream_t st) {
  if constexpr (KIND == GK_F32) {
    if (tile_bk(16) == 32) return launch_kind_bk<KIND, 32>(a, st);
    return launch_kind_bk<KIND, 16>(a, st);
  } else if constexpr (KIND == GK_BF16) {
    return launch_kind_bk<KIND, 32>(a, st);
  } else {
    return launch_kind_bk<KIND, 16>(a, st);
  }
}

hipError_t launch_gemm(GemmKind kind, const GemmArgs& a, hipStream_t st) {
  if (a.rows <= 0 || a.Ncols <= 0) return hipSuccess;
  // row indices and rows-per-block are handled in 32 bits inside the kernel
  if (a.rows >= (int64_t(1) << 31) || a.xrpw <= 0 || a.yrpw <= 0 || a.xrpw >= (int64_t(1) << 31) ||
      a.yrpw >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  if (!a.vmode && a.Rp == 4 && a.T != 1) return hipErrorInvalidValue;
  if (a.act == 2 && (!a.vmode || !a.aux)) return hipErrorInvalidValue;
  if (a.add5 && (a.vmode || a.Rp < 16 || a.nel < 1 || a.xrpw != a.rows || a.yrpw != a.rows))
    return hipErrorInvalidValue;
  switch (kind) {
    case GK_F64: return launch_kind<GK_F64>(a, st);
    case GK_F32: return launch_kind<GK_F32>(a, st);
    case GK_BF16: return launch_kind<GK_BF16>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qmc
