// ddfb.hip -- the DDFB denoiser (arXiv 2511.00870, Sec. II-B1 Example 3,
// Eqs. (ddfb_operator) and (dfb_operator:T)): K unrolled iterations of a
// dual forward-backward scheme,
//   u_0 = W_K v,
//   u_k = HT(u_{k-1} + gamma_k W_k P(v - W_k^* u_{k-1})),   k = 1 .. K-1,
//   D(v) = P(v - gamma_K W_K^* u_{K-1}),
// with W_k a 3x3 convolution from 1 to F channels (zero padding), W_k^* its
// adjoint, P the projection onto [0,1] and HT the clip to [-thresh, thresh];
// every map is zero outside the image.  The sampler takes G = v - D(v).
//
// Each u_k is a per-channel function of v and the one-channel maps
// b_j = P(v - W_j^* u_{j-1}), j = 1 .. k:
//   u_k[c](p) = HT(u_{k-1}[c](p) + gamma_k (w_k[c] * b_k)(p)),
// which reads only the 3x3 neighbourhood of p.  So only the maps b_j are
// kept (4 bytes per pixel each); stage k (one launch) recomputes u_{k-1} on
// its 30 x 30 tile plus a one-pixel ring from v and b_1 .. b_{k-1}, forms the
// adjoint's per-tap partial sums s_tap(p) = sum_c w_k[c][tap] u_{k-1}[c](p),
// exchanges them through LDS and writes b_k (or G for k = K).  Recomputing u
// costs 9 multiply-adds per channel and layer; storing it would move 2 x 4F
// bytes per pixel and layer.  F <= 64.
#include "device_common.h"
#include "kernels.h"

namespace pnp {

namespace {
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kDdThreads = 256;
constexpr int kDdWin = kDdTile + 4;       // v and b maps: core +- 2
constexpr int kDdReg = kDdTile + 2;       // partial sums: core +- 1
static_assert(kDdReg * kDdReg == 4 * kDdThreads, "four region pixels per thread");
}  // namespace

// KM >= K: register budget for the A fragments of W_1 .. W_{K-1}
//
// Matrix-core form of one stage.  Every contraction of the stage is a small
// GEMM over 16-pixel groups on v_mfma_f32_16x16x4_f32 (FP32 inputs, FP32
// accumulation): for the 16 pixels of a group (half a row of the 32 x 32
// region) and the 64 channels as four 16-row blocks,
//   u_0 = W_K v:          A = W_K (channels x taps), B = v at the 9 taps (3 K steps
//                         of 4 taps, the last padded with zero weights);
//   u_j += gamma_j W_j b_j, then HT: the same, with A = gamma_j W_j, accumulating
//                         into u, and the clip on the accumulator registers;
//   s = W_k^* u:          A = the taps x channels transpose (9 taps padded to 16
//                         rows), B = u itself: the accumulator register r of
//                         channel block mb holds, in lane group q, channel
//                         16 mb + 4 q + r, which is exactly a B operand whose
//                         K index q stands for that channel, so u never moves.
// u_0 carries no hard-tanh, so u_1 = HT(W_K v + gamma_1 W_1 b_1) is one sum over
// 18 taps (v's nine, then b_1's nine): 5 K steps instead of 3 + 3.
// Lane layout of the 16x16x4 f32 MFMA: A lane l = (row l % 16, k l / 16),
// B lane l = (k l / 16, column l % 16), D lane l register r = (row 4 (l / 16)
// + r, column l % 16).
template <int KM, int MB>
__global__ __launch_bounds__(kDdThreads, KM <= 4 ? 3 : 2) void ddfb_stage_kernel(DdfbArgs a) {
  __shared__ float smap[KM][kDdWin * kDdWin];
  // tap (dy, dx)'s partial sums on the 30 x 30 block of region positions the
  // core's adjoint reads: rows 2 - dy .. 31 - dy, columns 2 - dx .. 31 - dx
  __shared__ float spart[9][kDdTile * kDdTile];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const int k = a.stage, K = a.K, F = a.F;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q4 = lane >> 4, l16 = lane & 15;
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  // the maps' windows: every load issued before the first is stored (the
  // maps carry a zero border of two pixels; lanes past the window read its
  // first element and drop it)
  constexpr int NQ = (kDdWin * kDdWin + kDdThreads - 1) / kDdThreads;
  float mv[KM][NQ];
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m >= k) break;
    const PNP_GLOBAL float *src = gp(m == 0 ? j.x[t & 1] : j.dmaps + (int64_t)(m - 1) * j.dstride);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q0 = tid + i * kDdThreads, q = q0 < kDdWin * kDdWin ? q0 : 0;
      const int Y = tl.y0 - 2 + q / kDdWin, X = tl.x0 - 2 + q % kDdWin;
      mv[m][i] = src[(int64_t)(Y + B) * P + (X + B)];
    }
  }
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m >= k) break;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = tid + i * kDdThreads;
      if (q < kDdWin * kDdWin) smap[m][q] = mv[m][i];
    }
  }
  // A fragments: MB blocks of 16 channels (channels from F on have zero
  // weights, so their u stays zero and adds nothing).  A01: the 18-tap
  // chain of u_0 and the first update (K step s, lane group q4: slot
  // 4 s + q4, v's tap for slots 0..8, b_1's for 9..17, zero weights beyond
  // and for b_1 when k = 1); AJ[m - 2]: the updates m = 2 .. k - 1.  A slot
  // with a zero weight reads tap (0, 0) of v, a finite value, so it adds an
  // exact zero and needs no select.
  const PNP_GLOBAL float *w = gp(a.w);
  float A01[MB][5], AJ[KM > 2 ? KM - 2 : 1][MB][3], AP[MB][4];
  int toff[3], toff01[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int t = 4 * s + q4, tp = t < 9 ? t : t - 9;
    const bool used = t < 18 && (t < 9 || k >= 2);
    toff01[s] = used ? (t < 9 ? 0 : kDdWin * kDdWin) + (tp / 3) * kDdWin + tp % 3 : 0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int c = 16 * mb + l16;
      const bool ok = used && c < F;
      A01[mb][s] = !ok ? 0.0f
                   : t < 9 ? w[((int64_t)(K - 1) * F + c) * 9 + tp]
                           : a.gamma[0] * w[(int64_t)c * 9 + tp];
    }
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int tp = 4 * s + q4;
    toff[s] = tp < 9 ? (tp / 3) * kDdWin + tp % 3 : 0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int c = 16 * mb + l16;
      const bool ok = tp < 9 && c < F;
#pragma unroll
      for (int m = 2; m < KM; ++m)
        AJ[m - 2][mb][s] = (m < k && ok) ? a.gamma[m - 1] * w[((int64_t)(m - 1) * F + c) * 9 + tp]
                                         : 0.0f;
    }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * mb + 4 * q4 + r;
      AP[mb][r] = (l16 < 9 && c < F) ? w[((int64_t)(k - 1) * F + c) * 9 + l16] : 0.0f;
    }
  __syncthreads();
  const float th = a.thresh;
  // 64 groups of 16 pixels (row ri, half h) of the 32 x 32 region, 16 per
  // wave, two at a time (the two halves of one row): two independent chains
  // for the matrix cores, and the transpose contraction split over MB
  // accumulators summed at the end instead of one chain of 4 MB steps
  for (int ri = 8 * wave; ri < 8 * wave + 8; ++ri) {
    f32x4 acc[2][MB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[h][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int base = ri * kDdWin + l16;            // window position of tap (0, 0), half 0
    // u_0 (k = 1: three K steps), or u_0 + gamma_1 W_1 b_1 and its clip
    const int ns01 = k >= 2 ? 5 : 3;
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      if (s >= ns01) break;                          // uniform
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float bv = (&smap[0][0])[base + 16 * h + toff01[s]];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[h][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A01[mb][s], bv, acc[h][mb], 0, 0, 0);
      }
    }
    if (k >= 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][mb][r] = __builtin_amdgcn_fmed3f(acc[h][mb][r], -th, th);
    }
#pragma unroll
    for (int m = 2; m < KM; ++m) {
      if (m >= k) break;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float bv = smap[m][base + 16 * h + toff[s]];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[h][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(AJ[m - 2][mb][s], bv, acc[h][mb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][mb][r] = __builtin_amdgcn_fmed3f(acc[h][mb][r], -th, th);
    }
    // u is zero outside the image
    const int Y = tl.y0 - 1 + ri;
    f32x4 sp[2][MB];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int X = tl.x0 - 1 + 16 * h + l16;
      const bool inside = Y >= 0 && Y < j.ny && X >= 0 && X < j.nx;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        sp[h][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sp[h][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(AP[mb][r], inside ? acc[h][mb][r] : 0.0f,
                                                           sp[h][mb], 0, 0, 0);
      }
    }
    // lane (q4, l16) holds taps 4 q4 .. 4 q4 + 3 of pixel 16 h + l16
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 tot = sp[h][0];
#pragma unroll
      for (int mb = 1; mb < MB; ++mb) tot += sp[h][mb];
      const int col = 16 * h + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tap = 4 * q4 + r, dy = tap / 3, dx = tap % 3;
        const int pr = ri - 2 + dy, pc = col - 2 + dx;
        if (tap < 9 && (unsigned)pr < (unsigned)kDdTile && (unsigned)pc < (unsigned)kDdTile)
          spart[tap][pr * kDdTile + pc] = tot[r];
      }
    }
  }
  __syncthreads();
  // adjoint on the core: (W^* u)(q) = sum_tap s_tap(q + (1 - dy, 1 - dx))
  for (int q = tid; q < kDdTile * kDdTile; q += kDdThreads) {
    const int ci = q / kDdTile, cc = q % kDdTile;
    if (ci >= tl.h || cc >= tl.w) continue;
    float out = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) out += spart[i][q];
    const float v = smap[0][(ci + 2) * kDdWin + cc + 2];
    const int Y = tl.y0 + ci, X = tl.x0 + cc;
    if (k < K) {
      gp(j.dmaps + (int64_t)(k - 1) * j.dstride)[(int64_t)(Y + B) * P + (X + B)] =
          fminf(fmaxf(v - out, 0.0f), 1.0f);
    } else {
      const float D = fminf(fmaxf(v - a.gamma[K - 1] * out, 0.0f), 1.0f);
      gp(j.G)[(int64_t)Y * j.nx + X] = v - D;
    }
  }
}

template <int KM>
static hipError_t launch_ddfb_km(const DdfbArgs &a, int n_tiles, hipStream_t s) {
  switch ((a.F + 15) / 16) {
    case 1: hipLaunchKernelGGL((ddfb_stage_kernel<KM, 1>), dim3(n_tiles), dim3(kDdThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((ddfb_stage_kernel<KM, 2>), dim3(n_tiles), dim3(kDdThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL((ddfb_stage_kernel<KM, 3>), dim3(n_tiles), dim3(kDdThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((ddfb_stage_kernel<KM, 4>), dim3(n_tiles), dim3(kDdThreads), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_ddfb_stage(const DdfbArgs &a, int n_tiles, hipStream_t s) {
  if (a.F < 1 || a.F > 64 || a.K < 1 || a.K > kMaxDdfbLayers) return hipErrorInvalidValue;
  return a.K <= 4 ? launch_ddfb_km<4>(a, n_tiles, s) : launch_ddfb_km<kMaxDdfbLayers>(a, n_tiles, s);
}

}  // namespace pnp
