// Fused edge filters on MFMA (float32, width 128 or 256, at most 16 radial basis
// functions): for every pair of one edge type,
//   w(d) = tanh(rho(d) U1 + a1) U2 + a2,
// from the pair distance to the filter row in one kernel, as a value row or
// as a univariate jet in d (rows value, first and second derivative; a 16-row
// tile holds the jets of 5 pairs).
//
// The first layer is computed transposed, Z^T = U1^T rho^T (+ a1 through a
// constant basis function on the value row), so that each lane's accumulator
// (rows 4*(l/16)+i, column l%16 of the 16x16 tile) holds the hidden units
// 16*hb + 4*(l/16) + i of pair row l%16: exactly the A-operand slice the
// second layer's MFMA wants from that lane (row l%16, k = 4*(l/16) + step).
// The hidden layer never leaves the registers.  For jets the tanh is
// propagated across the three rows of a pair (lanes 3p'..3p'+2 of a 16-lane
// group) with shuffles: t = tanh(z0), t' z1, t' z2 + t'' z1^2.
//
// At width 128 the second layer runs on bf16 matrix cores with float32 accuracy: each
// operand x is split into three bf16 pieces x = x0 + x1 + x2 (x0 = bf16(x), x1 = bf16(x - x0),
// x2 = bf16(x - x0 - x1), round to nearest; the differences are exact in float32, |x1| <= 2^-8 |x|,
// |x2| <= 2^-16 |x| and |x - x0 - x1 - x2| <= 2^-24 |x|), and the product is the sum of the six
// piece products whose orders add up to at most 2 (each exact in float32, accumulated in float32
// by the MFMA; the three omitted ones add up to at most about 2^-23 |x y|): float32-level error.
// The order-0 product goes to one accumulator, the five corrections to two others, added at the end.
// Six v_mfma_f32_16x16x32_bf16 replace eight v_mfma_f32_16x16x4f32 per 32 hidden units, at
// 16 instead of 32 cycles each.  The lane holding z for hidden units 16 hb + 4 g + i of
// pair row c supplies k-slots 8 g + 4 (hb mod 2) + i of the MFMA covering hb = 2 m, 2 m + 1, and
// U2's three pieces are stored in LDS in that k order (16-byte chunks XOR-swizzled by column).
//
// A persistent grid keeps U2 (transposed, 16-byte chunks XOR-swizzled by row
// against LDS bank conflicts) and U1, a1, a2 in LDS, one copy per block; each wave takes 16 pair
// rows at a time.  At width 128 the second layer forms one 16-column block at a time (three
// accumulators and three U2 fragments live), which keeps the kernel within 168 registers: blocks of
// 12 waves, three per SIMD (two 16-column blocks at a time needed 174-194 registers, two waves per
// SIMD; value rows 5 % and jets 13 % slower).  At width 256, 8 waves, two per SIMD.  A launch
// writes 128 output columns from c0 on: width 256 takes two launches, each
// recomputing the 256 hidden units (the half of U2 it needs fills 128 KB of LDS).  The radial
// basis takes its exponent in float64 and the exponential of its fractional part
// in float32 (rbf3_f32); tanh is the float32 form of act.h.
#include <algorithm>
#include <cstring>

#include "act.h"
#include "kernels.h"
#include "pairs.h"

namespace qmc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int ED = 128;  // output columns per launch

// Gaussian basis function k of the distance d and its first two derivatives in d.  The offset, its
// square and the base-2 exponent y = -x^2 log2(e) are formed in float64 (d up to tens of bohr loses
// no digits to the centre's cancellation), y is split into an integer n and a fraction f in [0, 1),
// and only 2^f is evaluated in float32 (the hardware exp2), then scaled by 2^n: the value carries
// about one float32 rounding at any argument.  The float64 exponential it replaces was the largest
// VALU cost per pair.  A NaN distance gives NaN; exponents below -200 give 0.
__device__ inline void rbf3_f32(double d, int k, double s, double inv_s, float& r0, float& r1, float& r2) {
  const double x = (d - k * s) * inv_s;
  double y = -(x * x) * 1.4426950408889634;  // log2(e)
  if (y < -200.0) y = -200.0;
  const double fl = floor(y);
  const float xf = (float)x, is = (float)inv_s;
  const float e = ldexpf(__builtin_amdgcn_exp2f((float)(y - fl)), (int)fl);
  r0 = e;
  r1 = -2.f * xf * is * e;
  r2 = (4.f * xf * xf - 2.f) * (is * is) * e;
}

// EH: hidden (and full output) width, 128 or 256; c0: first output column of this launch
// Up to three edge types in one launch: blocks [0, b1) take type slot 0, [b1, b2) slot 1, [b2, grid)
// slot 2, each walking its type's tiles with a stride of its own block count.
struct EdgeMlpBatch {
  EdgeMlpArgs t[3];
  int b1, b2;
};

// Splits x into three bf16 pieces (round to nearest each): x0 + x1 + x2 = x within 2^-27 |x|.
__device__ inline void split3(float x, __bf16& x0, __bf16& x1, __bf16& x2) {
  x0 = (__bf16)x;
  const float r1 = x - (float)x0;
  x1 = (__bf16)r1;
  x2 = (__bf16)(r1 - (float)x1);
}

template <int JET, int NW, int EH>
__global__ __launch_bounds__(64 * NW) void edge_mlp_kernel(SysDev s, EdgeMlpBatch B, int c0) {
  constexpr bool SPLIT = EH == 128;  // second layer on bf16 matrix cores with three-piece operands
  const int slot = (int)blockIdx.x < B.b1 ? 0 : ((int)blockIdx.x < B.b2 ? 1 : 2);
  const int bstart = slot == 0 ? 0 : (slot == 1 ? B.b1 : B.b2);
  const int bcount = (slot == 0 ? B.b1 : (slot == 1 ? B.b2 : (int)gridDim.x)) - bstart;
  // (selected field by field: the slot is uniform, and no copy of the batch goes to scratch)
  const EdgeMlpArgs a = slot == 0 ? B.t[0] : (slot == 1 ? B.t[1] : B.t[2]);
  // float32: U2^T (n, k), 4-float chunk (k/4) ^ (n & 7); split: three bf16 planes of U2^T (n, k'),
  // k' the MFMA k order, 8-element chunk (k'/8) ^ (n & 15)
  __shared__ __attribute__((aligned(16))) char u2raw[SPLIT ? 3 * ED * EH * 2 : ED * EH * 4];
  __shared__ __attribute__((aligned(16))) float u1t[EH * 16];  // U1^T (k, r), r < 16
  __shared__ float a1s[EH], a2s[ED];
  float* u2t = (float*)u2raw;
  __bf16* u2b = (__bf16*)u2raw;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int K = s.K;
  const double rs = rbf_spacing(s.dmax, K), ris = (K - 1) / s.dmax;
  for (int e = tid; e < ED * EH; e += 64 * NW) {
    const int k = e / ED, n = e - k * ED;
    const float v = a.U2[(int64_t)k * EH + c0 + n];
    if constexpr (SPLIT) {
      // hidden unit k = 32 m + 16 h + 4 gg + i sits at k-slot 8 gg + 4 h + i of block m
      const int m = k >> 5, h = (k >> 4) & 1, gg = (k >> 2) & 3, i = k & 3;
      const int ch = (4 * m + gg) ^ (n & 15);
      const int at = n * EH + ch * 8 + 4 * h + i;
      __bf16 p0, p1, p2;
      split3(v, p0, p1, p2);
      u2b[at] = p0;
      u2b[ED * EH + at] = p1;
      u2b[2 * ED * EH + at] = p2;
    } else {
      u2t[n * EH + (((k >> 2) ^ (n & 7)) << 2) + (k & 3)] = v;
    }
  }
  for (int e = tid; e < EH * 16; e += 64 * NW) {
    const int k = e >> 4, r = e & 15;
    u1t[e] = r < K ? a.U1[r * EH + k] : 0.f;
  }
  for (int e = tid; e < EH; e += 64 * NW) a1s[e] = a.a1[e];
  for (int e = tid; e < ED; e += 64 * NW) a2s[e] = a.a2[c0 + e];
  __syncthreads();

  const int P = a.type == 0 ? s.P0 : (a.type == 1 ? s.P1 : s.P2);
  // a tile holds 16 value rows, or the jets of 5 pairs (rows 3p .. 3p + 2; row 15 idle)
  constexpr int PPT = JET ? 5 : 16;
  const int64_t ntiles = (a.pairs + PPT - 1) / PPT;
  const int pc = JET ? c / 3 : c;           // pair of this lane's row within the tile
  const int e = JET ? c - 3 * pc : 0;       // its jet entry: value, first, second derivative
  // distance of this lane's pair row in a tile (0 for idle rows and with precomputed features)
  auto pair_distance = [&](int64_t tl) -> double {
    const int64_t pr = tl * PPT + pc;
    if ((JET && c >= 15) || pr >= a.pairs || a.feat) return 0.0;
    const int64_t w = pr / P;
    const int pi = (int)(pr - w * P);
    int i, j;
    decode_pair(s, a.type, pi, i, j);
    return a.type == 2 ? a.en[((w * s.N + i) * s.M + j) * 4] : a.ee[((w * s.N + i) * s.N + j) * 4];
  };
  const int64_t tstride = (int64_t)bcount * NW;
  int64_t tile = (int64_t)((int)blockIdx.x - bstart) * NW + wave;
  // the next tile's distance is loaded one tile ahead, so its gather latency hides behind the MFMAs
  double dnext = tile < ntiles ? pair_distance(tile) : 0.0;
  for (; tile < ntiles; tile += tstride) {
    const int64_t p0 = tile * PPT;
    const double d = dnext;
    if (tile + tstride < ntiles) dnext = pair_distance(tile + tstride);
    // ---- this lane's pair row (column c of the first layer)
    const int64_t pr = p0 + pc;
    const bool rowok = (!JET || c < 15) && pr < a.pairs;
    float rb[4] = {0.f, 0.f, 0.f, 0.f};
    if (rowok) {
      if (a.feat) {
        // precomputed edge features (an updated edge feature, Sec. III.A)
        const float* fr = a.feat + (JET ? pr * 4 + e : pr) * K;
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
          if (4 * g + kq < K) rb[kq] = fr[4 * g + kq];
      } else {
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const int r = 4 * g + kq;
          if (r < K) {
            float r0, r1, r2;
            rbf3_f32(d, r, rs, ris, r0, r1, r2);
            rb[kq] = e == 0 ? r0 : (e == 1 ? r1 : r2);
          }
        }
      }
    }
    const float bias_in = (g == 0 && e == 0) ? 1.f : 0.f;  // constant basis function of the value row
    // ---- first layer: z^T blocks of 16 hidden units
    f4 z[EH / 16];
#pragma unroll
    for (int hb = 0; hb < EH / 16; ++hb) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      const f4 ua = *(const f4*)&u1t[(16 * hb + c) * 16 + 4 * g];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.x, rb[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.y, rb[1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.z, rb[2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.w, rb[3], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(g == 0 ? a1s[16 * hb + c] : 0.f, bias_in, acc, 0, 0, 0);
      z[hb] = acc;
    }
    // ---- tanh (through the jet of a pair's three rows); the idle row 15 borrows pair 4's lanes
    const int qbase = (lane & 48) + 3 * (pc < 4 ? pc : 4);  // lane of row 0 of this lane's pair
#pragma unroll
    for (int hb = 0; hb < EH / 16; ++hb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float zi = z[hb][i];
        if constexpr (JET) {
          const float z0 = __shfl(zi, qbase), z1 = __shfl(zi, qbase + 1), z2 = __shfl(zi, qbase + 2);
          const float t = tanh_f32(z0), t1 = 1.f - t * t, t2 = -2.f * t * t1;
          z[hb][i] = e == 0 ? t : (e == 1 ? t1 * z1 : t1 * z2 + t2 * z1 * z1);
        } else {
          z[hb][i] = tanh_f32(zi);
        }
      }
    if (!JET && a.zout && rowok && c0 == 0) {
#pragma unroll
      for (int hb = 0; hb < EH / 16; ++hb) *(f4*)&a.zout[pr * EH + 16 * hb + 4 * g] = z[hb];
    }
    if constexpr (SPLIT) {
      // ---- second layer on bf16 matrix cores: operand pieces of the 32 hidden units of block m
      bf16x8 zp[3][EH / 32];
#pragma unroll
      for (int m = 0; m < EH / 32; ++m)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 p0, p1, p2;
          split3(z[2 * m + (j >> 2)][j & 3], p0, p1, p2);
          zp[0][m][j] = p0;
          zp[1][m][j] = p1;
          zp[2][m][j] = p2;
        }
#pragma unroll 1
      for (int nb = 0; nb < ED / 16; ++nb) {
        f4 h0 = {0.f, 0.f, 0.f, 0.f}, la0 = h0, lb0 = h0;
        const int n0 = 16 * nb + c;
#pragma unroll
        for (int m = 0; m < EH / 32; ++m) {
          const int o0 = n0 * EH + (((4 * m + g) ^ (n0 & 15)) << 3);
          bf16x8 b0[3];
#pragma unroll
          for (int p = 0; p < 3; ++p) b0[p] = *(const bf16x8*)&u2b[p * ED * EH + o0];
          lb0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[2][m], b0[0], lb0, 0, 0, 0);
          la0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[1][m], b0[0], la0, 0, 0, 0);
          lb0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[1][m], b0[1], lb0, 0, 0, 0);
          la0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[0][m], b0[1], la0, 0, 0, 0);
          lb0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[0][m], b0[2], lb0, 0, 0, 0);
          h0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(zp[0][m], b0[0], h0, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 4 * g + i;
          const int rp = JET ? r / 3 : r, re = JET ? r - 3 * rp : 0;
          const int64_t op = p0 + rp;
          if ((JET && r == 15) || op >= a.pairs) continue;
          const int64_t orow = JET ? op * 4 + re : op;
          a.out[orow * EH + c0 + n0] = (h0[i] + (la0[i] + lb0[i])) + (re == 0 ? a2s[n0] : 0.f);
        }
      }
      continue;
    }
    // ---- second layer, two 16-column blocks at a time
#pragma unroll 1
    for (int nb = 0; nb < ED / 16; nb += 2) {
      f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
      const int n0 = 16 * nb + c, n1 = n0 + 16;
#pragma unroll
      for (int hb = 0; hb < EH / 16; ++hb) {
        const int ch = 4 * hb + g;
        const f4 b0 = *(const f4*)&u2t[n0 * EH + ((ch ^ (n0 & 7)) << 2)];
        const f4 b1 = *(const f4*)&u2t[n1 * EH + ((ch ^ (n1 & 7)) << 2)];
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][0], b0.x, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][0], b1.x, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][1], b0.y, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][1], b1.y, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][2], b0.z, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][2], b1.z, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][3], b0.w, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(z[hb][3], b1.w, acc1, 0, 0, 0);
      }
      // lane holds tile rows 4g + i, columns n0 / n1; a2 goes to value rows only.  Jets are stored
      // as [pair][4][D] (rows value, first, second derivative; the fourth row is not written)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * g + i;
        const int rp = JET ? r / 3 : r, re = JET ? r - 3 * rp : 0;
        const int64_t op = p0 + rp;
        if ((JET && r == 15) || op >= a.pairs) continue;
        const int64_t orow = JET ? op * 4 + re : op;
        a.out[orow * EH + c0 + n0] = acc0[i] + (re == 0 ? a2s[n0] : 0.f);
        a.out[orow * EH + c0 + n1] = acc1[i] + (re == 0 ? a2s[n1] : 0.f);
      }
    }
  }
}

bool edge_mlp_supported(const SysDev& s) { return (s.D == 128 || s.D == 256) && s.K >= 2 && s.K <= 16; }

hipError_t launch_edge_mlp(const SysDev& s, const EdgeMlpArgs& a, hipStream_t st) {
  return launch_edge_mlp_types(s, &a, 1, st);
}

hipError_t launch_edge_mlp_types(const SysDev& s, const EdgeMlpArgs* a, int n, hipStream_t st) {
  if (!edge_mlp_supported(s) || n < 1 || n > 3) return hipErrorInvalidValue;
  EdgeMlpBatch B;
  std::memset(&B, 0, sizeof(B));
  int64_t tiles[3] = {0, 0, 0}, total = 0;
  int m = 0;  // slots with pairs
  for (int i = 0; i < n; ++i) {
    if (a[i].pairs < 0 || a[i].type < 0 || a[i].type > 2 || a[i].jet != a[0].jet) return hipErrorInvalidValue;
    if (a[i].pairs == 0) continue;
    B.t[m] = a[i];
    tiles[m] = a[i].jet ? (a[i].pairs + 4) / 5 : (a[i].pairs + 15) / 16;
    total += tiles[m++];
  }
  if (m == 0) return hipSuccess;
  const int jet = a[0].jet;
  const int cus = device_cus();
  // blocks of w waves share one copy of their type's weights in LDS (105 KB at width 128, 146 KB at
  // 256); as many blocks as fit per compute unit, split among the types in proportion to their tiles
  // (at least one each, at most one per w tiles), each type's blocks walking its tiles with a stride
  auto go = [&](auto kern, int w, int c0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * w, 0) != hipSuccess || occ < 1) occ = 1;
    const int64_t cap = (int64_t)occ * cus;
    int64_t nb[3] = {0, 0, 0}, sum = 0;
    for (int i = 0; i < m; ++i) {
      nb[i] = std::max<int64_t>(1, std::min<int64_t>((tiles[i] + w - 1) / w, cap * tiles[i] / total));
      sum += nb[i];
    }
    B.b1 = (int)nb[0];
    B.b2 = (int)(nb[0] + nb[1]);
    hipLaunchKernelGGL(kern, dim3((unsigned)sum), dim3(64 * w), 0, st, s, B, c0);
  };
  ProfScope ps(jet ? "edge_mlp_kernel<jet>" : "edge_mlp_kernel<val>", st);
  if (s.D == 256) {
    // the 256 hidden units take 64 more registers: two waves per SIMD
    for (int c0 = 0; c0 < 256; c0 += ED) {
      if (jet)
        go(edge_mlp_kernel<1, 8, 256>, 8, c0);
      else
        go(edge_mlp_kernel<0, 8, 256>, 8, c0);
    }
  } else if (jet) {
    // one 16-column block at a time in the second layer: within 168 registers, three waves per SIMD
    go(edge_mlp_kernel<1, 12, 128>, 12, 0);
  } else {
    go(edge_mlp_kernel<0, 12, 128>, 12, 0);
  }
  return hipGetLastError();
}

}  // namespace qmc
