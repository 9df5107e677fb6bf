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
// its tile plus a one-pixel ring from v and b_1 .. b_{k-1}, forms the
// adjoint's per-tap partial sums s_tap(p) = sum_c w_k[c][tap] u_{k-1}[c](p)
// in registers, exchanges them through LDS and writes b_k (or G for k = K).
// Recomputing u costs 9 FMAs per channel and layer; storing it would move
// 2 x 4F bytes per pixel and layer.
#include "device_common.h"
#include "kernels.h"

namespace pnp {

namespace {
constexpr int kDdThreads = 256;
constexpr int kDdWin = kDdTile + 4;       // v and b maps: core +- 2
constexpr int kDdReg = kDdTile + 2;       // partial sums: core +- 1
static_assert(kDdReg * kDdReg == 4 * kDdThreads, "four region pixels per thread");
}  // namespace

// KM >= K: register budget for the stencils of v and b_1 .. b_{K-1}
template <int KM>
__global__ __launch_bounds__(kDdThreads) void ddfb_stage_kernel(DdfbArgs a) {
  __shared__ float smap[KM][kDdWin * kDdWin];
  __shared__ float spart[9][kDdReg * kDdReg];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const int k = a.stage, K = a.K, F = a.F;
  const int tid = threadIdx.x;
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  // windows of v (map 0) and b_1 .. b_{k-1} (maps 1 .. k-1), zero outside the image
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m >= k) break;
    const PNP_GLOBAL float *src = gp(m == 0 ? j.x[t & 1] : j.dmaps + (int64_t)(m - 1) * j.dstride);
    for (int q = tid; q < kDdWin * kDdWin; q += kDdThreads) {
      const int Y = tl.y0 - 2 + q / kDdWin, X = tl.x0 - 2 + q % kDdWin;
      smap[m][q] = src[(int64_t)(Y + B) * P + (X + B)];
    }
  }
  __syncthreads();
  const PNP_CONST float *w = cp(a.w);
  const PNP_CONST float *wK = w + (size_t)(K - 1) * F * 9;        // W_K: u_0 = W_K v
  const PNP_CONST float *wa = w + (size_t)(k - 1) * F * 9;        // adjoint of this stage
  const float th = a.thresh;
  for (int pass = 0; pass < 4; ++pass) {
    const int q = tid + kDdThreads * pass;
    const int ri = q / kDdReg, rc = q % kDdReg;
    const int Y = tl.y0 - 1 + ri, X = tl.x0 - 1 + rc;
    float s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = 0.0f;
    if (Y >= 0 && Y < j.ny && X >= 0 && X < j.nx) {      // u is zero outside the image
      float st[KM][9];
#pragma unroll
      for (int m = 0; m < KM; ++m)
#pragma unroll
        for (int i = 0; i < 9; ++i)
          st[m][i] = m < k ? smap[m][(ri + i / 3) * kDdWin + rc + i % 3] : 0.0f;
      for (int c = 0; c < F; ++c) {
        float u = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) u = fmaf(wK[c * 9 + i], st[0][i], u);
#pragma unroll
        for (int m = 1; m < KM; ++m) {
          if (m >= k) break;
          const PNP_CONST float *wm = w + ((size_t)(m - 1) * F + c) * 9;
          float acc = 0.0f;
#pragma unroll
          for (int i = 0; i < 9; ++i) acc = fmaf(wm[i], st[m][i], acc);
          u = __builtin_amdgcn_fmed3f(fmaf(a.gamma[m - 1], acc, u), -th, th);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) s[i] = fmaf(wa[c * 9 + i], u, s[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) spart[i][q] = s[i];
  }
  __syncthreads();
  // adjoint on the core: (W^* u)(q) = sum_tap s_tap(q + (1 - dy, 1 - dx))
  for (int q = tid; q < kDdTile * kDdTile; q += kDdThreads) {
    const int ci = q / kDdTile, cc = q % kDdTile;
    if (ci >= tl.h || cc >= tl.w) continue;
    float out = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i)
      out += spart[i][(ci + 2 - i / 3) * kDdReg + (cc + 2 - i % 3)];
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

hipError_t launch_ddfb_stage(const DdfbArgs &a, int n_tiles, hipStream_t s) {
  if (a.K <= 4)
    hipLaunchKernelGGL(ddfb_stage_kernel<4>, dim3(n_tiles), dim3(kDdThreads), 0, s, a);
  else
    hipLaunchKernelGGL(ddfb_stage_kernel<kMaxDdfbLayers>, dim3(n_tiles), dim3(kDdThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace pnp
