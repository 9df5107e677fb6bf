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
__global__ __launch_bounds__(kZThreads) void zstep_psgla_kernel(UpdateArgs a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;            // x^(t) is the new iterate
  const bool big = j.big;
  const int r = big ? 0 : j.r, L = 2 * r + 1;
  constexpr int TH = kUpdTileH, TW = kUpdTileW, NT = kZThreads;
  const int WH = TH + 2 * r, WW = TW + 2 * r;
  float *sx = smem;                                  // WH x WW
  float *sh = sx + WH * WW;                          // WH x TW (row pass)
  constexpr int KMAX = (2 * kMaxR + 1) * (2 * kMaxR + 1);
  __shared__ float sku[2 * kMaxR + 1], skv[2 * kMaxR + 1], skern[KMAX];
  const int tid = threadIdx.x;
  const bool sep = !big && j.separable;
  if (sep) {
    if (tid < L) {
      sku[tid] = gp(j.ku)[tid];
      skv[tid] = gp(j.kv)[tid];
    }
  } else if (!big) {
    for (int q = tid; q < L * L; q += NT) skern[q] = gp(j.kern)[q];
  }
  const PNP_GLOBAL float *xin = gp(j.x[t & 1]);
  const int B = j.xborder;
  const int64_t xpitch = j.xpitch;
  const int wy = tl.y0 - r, wx = tl.x0 - r;
  for (int q = tid; q < WH * WW; q += NT) {
    const int i = q / WW, c = q % WW;
    sx[q] = xin[(int64_t)(wy + i + B) * xpitch + (wx + c + B)];
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
  const PNP_GLOBAL float *yb = gp(j.y);
  const PNP_GLOBAL uint8_t *mk = gp(j.mask);
  PNP_GLOBAL float *z1 = gp(j.z1);
  PNP_GLOBAL float *z2 = gp(j.z2);
  for (int q = tid; q < TH * TW; q += NT) {
    const int i = q / TW, c = q % TW;
    if (i >= tl.h || c >= tl.w) continue;
    float kx = 0.0f;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    if (big) {
      kx = gp(j.res)[(int64_t)(Y + j.r) * j.rpitch + (X + j.r)];
    } else if (sep) {
      for (int k = 0; k < L; ++k) kx = fmaf(sku[k], sh[(i + 2 * r - k) * TW + c], kx);
    } else {
      for (int a2 = 0; a2 < L; ++a2)
        for (int k = 0; k < L; ++k)
          kx = fmaf(skern[a2 * L + k], sx[(i + 2 * r - a2) * WW + (c + 2 * r - k)], kx);
    }
    const int64_t pp = (int64_t)(Y + B) * xpitch + (X + B);
    const float mv = j.has_mask ? (float)mk[pp] : 1.0f;
    float g0, g1, g2;
    gauss_triple(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, g0, g1, g2);
    const float zo = z1[pp];
    float v = zo - j.za1 * (zo - j.eta * (mv * kx)) + j.zs1 * g1;
    if (mv != 0.0f) {
      const float yv = yb[pp];
      v = j.poisson ? prox_kl(v, yv, j.zkappa) : (j.zsig2 * v + j.zkappa * yv) / (j.zsig2 + j.zkappa);
    }
    z1[pp] = v;
    if (j.has_z2) {
      const float wo = z2[pp];
      const float w = wo - j.za2 * (wo - sx[(i + r) * WW + (c + r)]) + j.zs2 * g2;
      z2[pp] = fmaxf(w, 0.0f);
    }
  }
}

// The TV prior term of the x-step on the tile's pixels:
//   G = (1/rho) D^T (D x - z),
//   (D^T w)_p = [j >= 1] w_h(p - 1) - [j < nx-1] w_h(p) + [i >= 1] w_v(p - nx) - [i < ny-1] w_v(p)
// with w = D x - z (D x zero in the last column / row).
__global__ __launch_bounds__(kZThreads) void tv_prior_kernel(UpdateArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *x = gp(j.x[t & 1]);
  const PNP_GLOBAL float *zh = gp(j.z1);
  const PNP_GLOBAL float *zv = gp(j.z2);
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  for (int q = threadIdx.x; q < kUpdTileH * kUpdTileW; q += kZThreads) {
    const int i = q / kUpdTileW, c = q % kUpdTileW;
    if (i >= tl.h || c >= tl.w) continue;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    const int64_t pp = (int64_t)(Y + B) * P + (X + B);
    const float xc = x[pp];
    float v = 0.0f;
    if (X >= 1) v += (xc - x[pp - 1]) - zh[pp - 1];
    if (X + 1 < j.nx) v -= (x[pp + 1] - xc) - zh[pp];
    if (Y >= 1) v += (xc - x[pp - P]) - zv[pp - P];
    if (Y + 1 < j.ny) v -= (x[pp + P] - xc) - zv[pp];
    gp(j.G)[(int64_t)Y * j.nx + X] = v * j.inv_rho;
  }
}

// TV z-step from x^(t+1) (x^(t) for the new t)
__global__ __launch_bounds__(kZThreads) void zstep_tv_kernel(UpdateArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *x = gp(j.x[t & 1]);
  PNP_GLOBAL float *zh = gp(j.z1);
  PNP_GLOBAL float *zv = gp(j.z2);
  const int B = j.xborder;
  const int64_t P = j.xpitch;
  for (int q = threadIdx.x; q < kUpdTileH * kUpdTileW; q += kZThreads) {
    const int i = q / kUpdTileW, c = q % kUpdTileW;
    if (i >= tl.h || c >= tl.w) continue;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    const int64_t pp = (int64_t)(Y + B) * P + (X + B);
    const float xc = x[pp];
    const float dh = X + 1 < j.nx ? x[pp + 1] - xc : 0.0f;
    const float dv = Y + 1 < j.ny ? x[pp + P] - xc : 0.0f;
    float g0, g1, g2;
    gauss_triple(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, g0, g1, g2);
    const float ho = zh[pp], vo = zv[pp];
    float vh = ho - j.za1 * (ho - dh) + j.zs1 * g1;
    float vv = vo - j.za1 * (vo - dv) + j.zs1 * g2;
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
