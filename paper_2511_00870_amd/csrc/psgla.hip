// psgla.hip -- splitting variables held as chain state (arXiv 2511.00870,
// Eq. (sgs_pnp_ula_psgla:psgla) and the z-update of Algorithm 1) and the
// total-variation prior (Sec. III-B2).
//
// PSGLA z-step, after the x-update has written x^(t+1), per pixel p:
//   z1 <- prox_{kappa f}( z1 - (kappa/rho) (z1 - eta m (K x)_p) + sqrt(2 kappa) zeta1 )
//         with f = KL(y_p || .) (Poisson, Sec. III-A3) or (y_p - .)^2/(2 sigma^2);
//         at unobserved pixels (m = 0) f is absent and the prox is the identity;
//   z2 <- max( z2 - (kappa2/rho2) (z2 - x_p) + sqrt(2 kappa2) zeta2, 0 )
//         (f2 = indicator of R+ on the second block, Sec. III-B1 (ii)).
// TV through AXDA (Sec. III-B2, Eq. (tv_prior)): z = (zh, zv) ~ D x with
// f = beta ||.||_{2,1}:
//   prior term of the x-step: (1/rho) D^T (D x - z), evaluated at x^(t) and
//   z^(t) before the update (it takes the place of the denoiser's G);
//   z-step: z <- prox_{kappa beta ||.||}( z - (kappa/rho)(z - D x) + sqrt(2 kappa) zeta ),
//   the block soft threshold of each pixel's two components.
// D is the forward difference, zero in the last column (horizontal) and the
// last row (vertical).  Noise of the z-steps: the three Box-Muller draws of
// the pixel at counter t+1 (zeta1 / zeta_h from the sine branch of the first
// pair, zeta2 / zeta_v from the cosine branch of the second).
//
// Every z buffer is updated in place: a z-step reads only its own pixel of
// z and x^(t+1), which no kernel writes meanwhile.
#include "device_common.h"
#include "kernels.h"

namespace pnp {

namespace {
constexpr int kZThreads = 256;

// prox of kappa (u - y log u) on u >= 0: the non-negative root of
// u^2 - (v - kappa) u - kappa y = 0, in a form without cancellation
__device__ __forceinline__ float prox_kl(float v, float y, float kappa) {
  const float b = v - kappa;
  const float s = __builtin_sqrtf(b * b + 4.0f * kappa * y);
  return b >= 0.0f ? 0.5f * (b + s) : (2.0f * kappa * y) / (s - b);
}
}  // namespace

// One workgroup per 32 x 64 tile: x^(t+1) on the core +- r into LDS, K x on
// the core, then the z-steps of the core pixels.  Large blurs (JobDesc::big)
// take K x from JobDesc::res, computed beforehand by the whole-image pass.
// Every global read of the tile is issued before the first wait: the x window
// into registers, then z1, y, the mask, z2 and (large blurs) K x of the
// thread's eight core pixels; lanes past the tile read a valid address and
// drop the value.
__global__ __launch_bounds__(kZThreads) void zstep_psgla_kernel(UpdateArgs a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;            // x^(t) is the new iterate
  const bool big = j.big;
  const int r = big ? 0 : j.r, L = 2 * r + 1;
  constexpr int TH = kUpdTileH, TW = kUpdTileW, NT = kZThreads;
  constexpr int XQ = ((TH + 2 * kMaxR) * (TW + 2 * kMaxR) + NT - 1) / NT;
  constexpr int CQ = TH * TW / NT;
  const int WH = TH + 2 * r, WW = TW + 2 * r;
  float *sx = smem;                                  // WH x WW
  float *sh = sx + WH * WW;                          // WH x TW (row pass)
  constexpr int KMAX = (2 * kMaxR + 1) * (2 * kMaxR + 1);
  __shared__ float sku[2 * kMaxR + 1], skv[2 * kMaxR + 1], skern[KMAX];
  const int tid = threadIdx.x;
  const bool sep = !big && j.separable;
  const PNP_GLOBAL float *xin = gp(j.x[t & 1]);
  const int B = j.xborder;
  const int64_t xpitch = j.xpitch;
  const int wy = tl.y0 - r, wx = tl.x0 - r;
  float xw[XQ];
#pragma unroll
  for (int k = 0; k < XQ; ++k) {
    const int q0 = tid + NT * k, q = q0 < WH * WW ? q0 : 0;
    const int i = q / WW, c = q % WW;
    xw[k] = xin[(int64_t)(wy + i + B) * xpitch + (wx + c + B)];
  }
  const PNP_GLOBAL float *yb = gp(j.y);
  PNP_GLOBAL float *z1 = gp(j.z1);
  PNP_GLOBAL float *z2 = gp(j.has_z2 ? j.z2 : j.z1);
  const PNP_GLOBAL uint8_t *mk = gp(j.has_mask ? j.mask : reinterpret_cast<const uint8_t *>(j.y));
  const PNP_GLOBAL float *kxb = gp(big ? j.res : j.z1);
  float zo[CQ], yv[CQ], wo[CQ], kxv[CQ];
  uint32_t mraw[CQ];
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = tid + NT * k, i = q / TW, c = q % TW;
    const int ii = i < tl.h ? i : 0, cc = c < tl.w ? c : 0;
    const int Y = tl.y0 + ii, X = tl.x0 + cc;
    const int64_t pp = (int64_t)(Y + B) * xpitch + (X + B);
    zo[k] = z1[pp];
    yv[k] = yb[pp];
    mraw[k] = mk[pp];
    wo[k] = z2[pp];
    kxv[k] = big ? kxb[(int64_t)(Y + j.r) * j.rpitch + (X + j.r)] : 0.0f;
  }
  if (sep) {
    if (tid < L) {
      sku[tid] = gp(j.ku)[tid];
      skv[tid] = gp(j.kv)[tid];
    }
  } else if (!big) {
    for (int q = tid; q < L * L; q += NT) skern[q] = gp(j.kern)[q];
  }
#pragma unroll
  for (int k = 0; k < XQ; ++k) {
    const int q = tid + NT * k;
    if (NT * k < WH * WW && q < WH * WW) sx[q] = xw[k];
  }
  __syncthreads();
  if (sep) {
    for (int q = tid; q < WH * TW; q += NT) {
      const int i = q / TW, c = q % TW;
      const float *row = sx + i * WW + c + 2 * r;
      float acc = 0.0f;
      for (int k = 0; k < L; ++k) acc = fmaf(skv[k], row[-k], acc);
      sh[q] = acc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = tid + NT * k;
    const int i = q / TW, c = q % TW;
    if (i >= tl.h || c >= tl.w) continue;
    float kx = kxv[k];
    const int Y = tl.y0 + i, X = tl.x0 + c;
    if (sep) {
      for (int kk = 0; kk < L; ++kk) kx = fmaf(sku[kk], sh[(i + 2 * r - kk) * TW + c], kx);
    } else if (!big) {
      for (int a2 = 0; a2 < L; ++a2)
        for (int kk = 0; kk < L; ++kk)
          kx = fmaf(skern[a2 * L + kk], sx[(i + 2 * r - a2) * WW + (c + 2 * r - kk)], kx);
    }
    const int64_t pp = (int64_t)(Y + B) * xpitch + (X + B);
    const float mv = j.has_mask ? (float)mraw[k] : 1.0f;
    float g0, g1, g2;
    gauss_triple(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, g0, g1, g2);
    float v = zo[k] - j.za1 * (zo[k] - j.eta * (mv * kx)) + j.zs1 * g1;
    if (mv != 0.0f)
      v = j.poisson ? prox_kl(v, yv[k], j.zkappa) : (j.zsig2 * v + j.zkappa * yv[k]) / (j.zsig2 + j.zkappa);
    z1[pp] = v;
    if (j.has_z2) {
      const float w = wo[k] - j.za2 * (wo[k] - sx[(i + r) * WW + (c + r)]) + j.zs2 * g2;
      z2[pp] = fmaxf(w, 0.0f);
    }
  }
}

// The TV prior term of the x-step on the tile's pixels:
//   G = (1/rho) D^T (D x - z),
//   (D^T w)_p = [j >= 1] w_h(p - 1) - [j < nx-1] w_h(p) + [i >= 1] w_v(p - nx) - [i < ny-1] w_v(p)
// with w = D x - z (D x zero in the last column / row).  x, zh and zv carry a
// zero border of at least two pixels, so every neighbour's address is valid:
// the thread's eight pixels issue all their reads before the first use.
__global__ __launch_bounds__(kZThreads) void tv_prior_kernel(UpdateArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *x = gp(j.x[t & 1]);
  const PNP_GLOBAL float *zh = gp(j.z1);
  const PNP_GLOBAL float *zv = gp(j.z2);
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  constexpr int CQ = kUpdTileH * kUpdTileW / kZThreads;
  float xc[CQ], xl[CQ], xr[CQ], xu[CQ], xd[CQ], hl[CQ], hc[CQ], vu[CQ], vc[CQ];
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = threadIdx.x + kZThreads * k, i = q / kUpdTileW, c = q % kUpdTileW;
    const int ii = i < tl.h ? i : 0, cc = c < tl.w ? c : 0;
    const int64_t pp = (int64_t)(tl.y0 + ii + B) * P + (tl.x0 + cc + B);
    xc[k] = x[pp];
    xl[k] = x[pp - 1];
    xr[k] = x[pp + 1];
    xu[k] = x[pp - P];
    xd[k] = x[pp + P];
    hl[k] = zh[pp - 1];
    hc[k] = zh[pp];
    vu[k] = zv[pp - P];
    vc[k] = zv[pp];
  }
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = threadIdx.x + kZThreads * k, i = q / kUpdTileW, c = q % kUpdTileW;
    if (i >= tl.h || c >= tl.w) continue;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    float v = 0.0f;
    if (X >= 1) v += (xc[k] - xl[k]) - hl[k];
    if (X + 1 < j.nx) v -= (xr[k] - xc[k]) - hc[k];
    if (Y >= 1) v += (xc[k] - xu[k]) - vu[k];
    if (Y + 1 < j.ny) v -= (xd[k] - xc[k]) - vc[k];
    gp(j.G)[(int64_t)Y * j.nx + X] = v * j.inv_rho;
  }
}

// TV z-step from x^(t+1) (x^(t) for the new t); reads first, as above
__global__ __launch_bounds__(kZThreads) void zstep_tv_kernel(UpdateArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *x = gp(j.x[t & 1]);
  PNP_GLOBAL float *zh = gp(j.z1);
  PNP_GLOBAL float *zv = gp(j.z2);
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  constexpr int CQ = kUpdTileH * kUpdTileW / kZThreads;
  float xc[CQ], xr[CQ], xd[CQ], ho[CQ], vo[CQ];
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = threadIdx.x + kZThreads * k, i = q / kUpdTileW, c = q % kUpdTileW;
    const int ii = i < tl.h ? i : 0, cc = c < tl.w ? c : 0;
    const int64_t pp = (int64_t)(tl.y0 + ii + B) * P + (tl.x0 + cc + B);
    xc[k] = x[pp];
    xr[k] = x[pp + 1];
    xd[k] = x[pp + P];
    ho[k] = zh[pp];
    vo[k] = zv[pp];
  }
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = threadIdx.x + kZThreads * k, i = q / kUpdTileW, c = q % kUpdTileW;
    if (i >= tl.h || c >= tl.w) continue;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    const int64_t pp = (int64_t)(Y + B) * P + (X + B);
    const float dh = X + 1 < j.nx ? xr[k] - xc[k] : 0.0f;
    const float dv = Y + 1 < j.ny ? xd[k] - xc[k] : 0.0f;
    float g0, g1, g2;
    gauss_triple(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, g0, g1, g2);
    float vh = ho[k] - j.za1 * (ho[k] - dh) + j.zs1 * g1;
    float vv = vo[k] - j.za1 * (vo[k] - dv) + j.zs1 * g2;
    const float nrm = __builtin_sqrtf(vh * vh + vv * vv);
    const float f = nrm > j.zkappa ? 1.0f - j.zkappa / nrm : 0.0f;
    zh[pp] = vh * f;
    zv[pp] = vv * f;
  }
}

size_t zstep_lds_bytes(int r) {
  const int WH = kUpdTileH + 2 * r, WW = kUpdTileW + 2 * r;
  return sizeof(float) * ((size_t)WH * WW + (size_t)WH * kUpdTileW);
}

hipError_t launch_zstep_psgla(const UpdateArgs &a, int n_tiles, int max_r, hipStream_t s) {
  const size_t lds = zstep_lds_bytes(max_r);
  static size_t attr = 0;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&zstep_psgla_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  hipLaunchKernelGGL(zstep_psgla_kernel, dim3(n_tiles), dim3(kZThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_tv_prior(const UpdateArgs &a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL(tv_prior_kernel, dim3(n_tiles), dim3(kZThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zstep_tv(const UpdateArgs &a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL(zstep_tv_kernel, dim3(n_tiles), dim3(kZThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace pnp
