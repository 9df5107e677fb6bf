// update.hip -- the fused memory-bound part of one PnP-ULA iteration.
//
// For every 32 x 64 tile of a block (arXiv 2511.00870, Algorithm 1, the
// x-update lines, with the z-update folded in):
//   1. read the tile's window x^(t) on [core +- 2r] from the previous iterate
//      (the block's ghost region is an overlapping read of device memory);
//   2. K x on core +- r (separable row/column passes when K = u v^T);
//   3. residual on core +- r, zero outside the image:
//        rho == 0:  m (K x - y)
//        rho > 0 :  m (K x - z),  z^(t) = (rho y + sigma^2 m K x)/(rho + sigma^2)
//                                       + sqrt(rho sigma^2/(rho + sigma^2)) zeta
//                   i.e. m (rho/(rho+sigma^2) (K x - y) - zsd zeta); z^(0) = 0.
//      The generator is keyed by the global pixel, so overlapping tiles draw
//      the same zeta and z never needs to be stored;
//   4. K^T of the residual on the core;
//   5. x^(t+1) = x - delta g - (alpha delta/eps) G + (delta/lambda)(clip x - x)
//                + sqrt(2 delta) xi,   g = K^T res / s2;
//   6. after burn-in, Welford update of the FP32 window mean / M2 and, when
//      the window is full, the Chan-Golub-LeVeque merge into the FP64 maps.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace pnp {

typedef float upd_f32x4 __attribute__((ext_vector_type(4)));

// Position (i, c) in the (32 + 2r) x (64 + 2r) residual region of the q-th
// residual pixel: the 32 x 64 core first, in the core's own row-major order
// (so a thread's core pixels in the residual pass are its pixels in the
// update and their noise stays in registers), then the ring: r rows above,
// r rows below, then the r columns on either side of each core row.
__device__ __forceinline__ void upd_res_pix(int q, int r, int RW, int &i, int &c) {
  constexpr int TH = kUpdTileH, TW = kUpdTileW;
  if (q < TH * TW) {
    i = q / TW + r;
    c = q % TW + r;
    return;
  }
  const int u = q - TH * TW, band = r * RW;
  if (u < 2 * band) {
    const int v = u < band ? u : u - band;
    i = (u < band ? 0 : TH + r) + v / RW;
    c = v % RW;
  } else {
    const int v = u - 2 * band, cc = v % (2 * r);
    i = r + v / (2 * r);
    c = cc < r ? cc : cc + TW;
  }
}

// RT > 0: every tile's blur half-width is RT (window sizes, divisions and
// tap loops become compile-time constants); RT = 0: read per job.
// MODE 0: the residual uses y (rho = 0) or the exact z draw (rho > 0);
// MODE 1: PSGLA chains, z1 and z2 held as state (JobDesc::zmode 1): the
// residual is m (eta m K x - z1), read in place of y, and the data gradient
// gains (x - z2)/rho2 on the core.
template <int RT, int MODE>
__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void fused_update_kernel(UpdateArgs a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const int r = RT > 0 ? RT : j.r, L = 2 * r + 1;
  constexpr int TH = kUpdTileH, TW = kUpdTileW, NT = kUpdThreads;
  // per-thread register budgets (r <= RM): residual region and core
  constexpr int RM = RT > 0 ? RT : kMaxR;
  constexpr int RQ = ((TH + 2 * RM) * (TW + 2 * RM) + NT - 1) / NT;
  constexpr int CQ = TH * TW / NT;
  constexpr int XQ = ((TH + 4 * RM) * (TW + 4 * RM) + NT - 1) / NT;
  // 16-byte slots of the x window (fixed widths: its rows are TW + 4r wide,
  // a multiple of 4) and the registers holding either form of the window
  constexpr int XQ4 = ((TH + 4 * RM) * (TW + 4 * RM) / 4 + NT - 1) / NT;
  constexpr int XS = XQ > 4 * XQ4 ? XQ : 4 * XQ4;
  const int WH = TH + 4 * r, WW = TW + 4 * r;       // x window
  const int RH = TH + 2 * r, RW = TW + 2 * r;       // K x / residual region
  float *sx = smem;                                  // WH x WW
  float *sh = sx + WH * WW;                          // WH x RW  (row pass of x)
  float *sres = sh + WH * RW;                        // RH x RW
  // RH x TW (row pass of the residual): reuses the row pass of x, whose last
  // reader (the residual pass) ends at the barrier before it is written
  float *shr = sh;
  const int tid = threadIdx.x;
  const PNP_GLOBAL float *xin = gp(j.x[t & 1]);
  const int B = j.xborder;
  const int64_t s = t + 1 - j.burn_in;              // sample number of x^(t+1)
  const bool stats = s >= 1;
  int nw = 0;
  bool merge = false;
  if (stats) {
    nw = (int)((s - j.wbase - 1) % j.wwin) + 1;
    merge = nw == j.wwin;
  }

  // blur taps, staged in LDS once per workgroup: their loads go first.  A
  // non-separable kernel (at most 17 x 17 = 289 taps, fewer than the row
  // pass buffer's 32 x 64 floats) lives in the row pass buffer, which only
  // the separable passes use.
  __shared__ float sku[2 * kMaxR + 1], skv[2 * kMaxR + 1];
  float *skern = sh;
  const bool sep = j.separable;
  const int nk = sep ? L : L * L;
  float tap0, tap1;
  {
    const PNP_GLOBAL float *k0 = gp(sep ? j.ku : j.kern);
    const PNP_GLOBAL float *k1 = gp(sep ? j.kv : j.kern);
    const int i0 = tid < nk ? tid : 0;
    const int i1 = sep ? i0 : (tid + NT < nk ? tid + NT : 0);
    tap0 = k0[i0];
    tap1 = k1[i1];
  }

  // 0. issue every global read of the tile up front: the x window, y and
  //    mask on the residual region, G and the Welford window on the core
  //    (no branch around a load: out-of-range lanes read a valid address and
  //    ignore the value, so the waits fall where the values are used)
  const int wy = tl.y0 - 2 * r, wx = tl.x0 - 2 * r;
  const int64_t xpitch = j.xpitch;
  // 16-byte loads when the window's rows start 16-byte aligned (uniform:
  // the tile's first column, the border and the pitch decide it)
  const bool xvec = RT > 0 && ((wx + B) & 3) == 0 && (xpitch & 3) == 0;
  float xv[XS];
  if (xvec) {
    constexpr int WW4 = RT > 0 ? (TW + 4 * RT) / 4 : 1;
#pragma unroll
    for (int k = 0; k < XQ4; ++k) {
      const int q0 = tid + NT * k, q = q0 < WH * WW4 ? q0 : 0;
      const int i = q / WW4, c4 = q % WW4;
      const upd_f32x4 v = *reinterpret_cast<const PNP_GLOBAL upd_f32x4 *>(
          xin + (wy + i + B) * xpitch + (wx + B + 4 * c4));
      xv[4 * k] = v.x;
      xv[4 * k + 1] = v.y;
      xv[4 * k + 2] = v.z;
      xv[4 * k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int q0 = tid + NT * k, q = q0 < WH * WW ? q0 : 0;
      const int i = q / WW, c = q % WW;
      xv[k] = xin[(wy + i + B) * xpitch + (wx + c + B)];
    }
  }
  const PNP_GLOBAL float *yb = gp(MODE == 1 ? j.z1 : j.y);
  const PNP_GLOBAL uint8_t *mk = gp(j.has_mask ? j.mask : reinterpret_cast<const uint8_t *>(j.y));
  float yv[RQ];
  uint32_t mraw[RQ];
#pragma unroll
  for (int k = 0; k < RQ; ++k) {
    const int q0 = tid + NT * k, q = q0 < RH * RW ? q0 : 0;
    int ri, rc;
    upd_res_pix(q, r, RW, ri, rc);
    const int Y = tl.y0 - r + ri, X = tl.x0 - r + rc;
    const int64_t pidx = (Y + B) * xpitch + (X + B);   // inside the padded buffer
    yv[k] = yb[pidx];
    mraw[k] = mk[pidx];
  }
  float gv[CQ], wmv[CQ], wm2v[CQ];
  float z2v[MODE == 1 ? CQ : 1];
  const bool z2on = MODE == 1 && j.has_z2;
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = tid + NT * k;
    const int i = q / TW, c = q % TW;
    const int64_t p = (i < tl.h && c < tl.w) ? (int64_t)(tl.y0 + i) * j.nx + tl.x0 + c : 0;
    gv[k] = gp(j.G)[p];
    if (MODE == 1) {
      const int ii = i < tl.h ? i : 0, cc = c < tl.w ? c : 0;
      z2v[k] = z2on ? gp(j.z2)[(int64_t)(tl.y0 + ii + B) * xpitch + (tl.x0 + cc + B)] : 0.0f;
    }
    wmv[k] = wm2v[k] = 0.0f;
    if (stats && nw > 1) {                           // uniform
      wmv[k] = gp(j.wmean)[p];
      wm2v[k] = gp(j.wm2)[p];
    }
  }

  // 1. blur taps and the window of x^(t) into LDS (their loads went first)
  if (sep) {
    if (tid < L) {
      sku[tid] = tap0;
      skv[tid] = tap1;
    }
  } else {
    if (tid < nk) skern[tid] = tap0;
    if (tid + NT < nk) skern[tid + NT] = tap1;
  }
  if (xvec) {
#pragma unroll
    for (int k = 0; k < XQ4; ++k) {
      const int q = tid + NT * k;
      if (4 * q < WH * WW)
        *reinterpret_cast<upd_f32x4 *>(sx + 4 * q) =
            upd_f32x4{xv[4 * k], xv[4 * k + 1], xv[4 * k + 2], xv[4 * k + 3]};
    }
  } else {
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int q = tid + NT * k;
      if (NT * k < WH * WW && q < WH * WW) sx[q] = xv[k];
    }
  }
  __syncthreads();

  // 2. K x on the residual region
  if (j.separable) {
    for (int q = tid; q < WH * RW; q += NT) {
      const int i = q / RW, c = q % RW;
      const float *row = sx + i * WW + c + 2 * r;
      float acc = 0.0f;
      for (int k = 0; k < L; ++k) acc = fmaf(skv[k], row[-k], acc);
      sh[q] = acc;
    }
    __syncthreads();
  }
  // 3. residual (zero outside the image); the noise xi of the thread's core
  //    pixels (residual pixels k < CQ) is kept for the update
  const int split = j.split;
  const bool draw = split && t >= 1;
  static_assert(NT * CQ == TH * TW, "the core's residual pixels come first, CQ per thread");
  float xir[CQ];
#pragma unroll
  for (int k = 0; k < RQ; ++k) {
    const int q = tid + NT * k;
    if (q >= RH * RW) break;
    int i, c;
    upd_res_pix(q, r, RW, i, c);
    float kx = 0.0f;
    if (j.separable) {
      for (int kk = 0; kk < L; ++kk) kx = fmaf(sku[kk], sh[(i + 2 * r - kk) * RW + c], kx);
    } else {
      for (int a2 = 0; a2 < L; ++a2)
        for (int kk = 0; kk < L; ++kk)
          kx = fmaf(skern[a2 * L + kk], sx[(i + 2 * r - a2) * WW + (c + 2 * r - kk)], kx);
    }
    const int Y = tl.y0 - r + i, X = tl.x0 - r + c;
    const float mv = j.has_mask ? (float)mraw[k] : 1.0f;
    float res = 0.0f;
    if (Y >= 0 && Y < j.ny && X >= 0 && X < j.nx) {
      if (MODE == 1) {
        res = mv * (j.eta * (mv * kx) - yv[k]);             // yv holds z1
      } else if (!split) {
        res = mv * (kx - yv[k]);
      } else if (!draw) {
        res = mv * kx;                                      // z^(0) = 0
      } else {
        float xi, zeta;
        gauss_pair(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, xi, zeta);
        res = mv * (j.zmix * (kx - yv[k]) - j.zsd * zeta);
        if (k < CQ) xir[k] = xi;
      }
    }
    sres[i * RW + c] = res;
  }
  __syncthreads();

  // 4. K^T res on the core
  if (j.separable) {
    for (int q = tid; q < RH * TW; q += NT) {
      const int i = q / TW, c = q % TW;
      const float *row = sres + i * RW + c;
      float acc = 0.0f;
      for (int k = 0; k < L; ++k) acc = fmaf(skv[k], row[k], acc);
      shr[q] = acc;
    }
    __syncthreads();
  }

  // 5./6. update, statistics
  PNP_GLOBAL float *xout = gp(j.x[(t + 1) & 1]);
  const float inv_nw = stats ? 1.0f / (float)nw : 0.0f;
  const int64_t na_i = j.nbase + (s - j.wbase - nw);       // merged before this window
  const double n_a = (double)na_i, n_b = (double)nw;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int q = tid + NT * k;
    const int i = q / TW, c = q % TW;
    if (i >= tl.h || c >= tl.w) continue;
    float ktr = 0.0f;
    if (j.separable) {
      for (int kk = 0; kk < L; ++kk) ktr = fmaf(sku[kk], shr[(i + kk) * TW + c], ktr);
    } else {
      for (int a2 = 0; a2 < L; ++a2)
        for (int kk = 0; kk < L; ++kk)
          ktr = fmaf(skern[a2 * L + kk], sres[(i + a2) * RW + (c + kk)], ktr);
    }
    const int Y = tl.y0 + i, X = tl.x0 + c;
    const int64_t p = (int64_t)Y * j.nx + X;
    float xi;
    if (draw) {
      xi = xir[k];
    } else {
      float zeta_unused;
      gauss_pair(j.key0, j.key1, j.chain, p, t, xi, zeta_unused);
    }
    const float xo = sx[(i + 2 * r) * WW + (c + 2 * r)];
    const float proj = fminf(fmaxf(xo, 0.0f), 1.0f);
    float gdat = ktr * j.inv_s2;
    if (MODE == 1 && z2on) gdat += (xo - z2v[k]) * j.inv_rho2;
    float xn = xo - j.delta * gdat - j.cprior * gv[k] + j.cproj * (proj - xo) + j.sq2d * xi;
    bad |= !isfinite(xn);
    if (j.xpos) xn = fmaxf(xn, 0.0f);                      // prox of the indicator of R+
    xout[(int64_t)(Y + B) * j.xpitch + (X + B)] = xn;
    if (stats) {
      float m = wmv[k], M = wm2v[k];                       // zero when the window starts
      const float d = xn - m;
      m = fmaf(d, inv_nw, m);
      M = fmaf(d, xn - m, M);
      if (merge) {
        const double n = n_a + n_b;
        const double ma = na_i > 0 ? gp(j.mean)[p] : 0.0;
        const double Ma = na_i > 0 ? gp(j.m2)[p] : 0.0;
        const double dl = (double)m - ma;
        gp(j.mean)[p] = ma + dl * (n_b / n);
        gp(j.m2)[p] = Ma + (double)M + dl * dl * (n_a * n_b / n);
      } else {
        gp(j.wmean)[p] = m;
        gp(j.wm2)[p] = M;
      }
    }
  }
  if (bad) gp(j.flag)[0] = 1;
}

// The update and statistics of step 5./6. when the data gradient comes
// precomputed (JobDesc::gdat: large blurs, whose blur and adjoint run as
// separate whole-image passes).  One workgroup per 32 x 64 tile.
__global__ __launch_bounds__(256) void update_pointwise_kernel(UpdateArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const int B = j.xborder;
  const int64_t xpitch = j.xpitch;
  const int64_t s = t + 1 - j.burn_in;
  const bool stats = s >= 1;
  int nw = 0;
  bool merge = false;
  if (stats) {
    nw = (int)((s - j.wbase - 1) % j.wwin) + 1;
    merge = nw == j.wwin;
  }
  const float inv_nw = stats ? 1.0f / (float)nw : 0.0f;
  const int64_t na_i = j.nbase + (s - j.wbase - nw);
  const double n_a = (double)na_i, n_b = (double)nw;
  const PNP_GLOBAL float *xin = gp(j.x[t & 1]);
  PNP_GLOBAL float *xout = gp(j.x[(t + 1) & 1]);
  const bool z2on = j.zmode == 1 && j.has_z2;
  bool bad = false;
  for (int q = threadIdx.x; q < kUpdTileH * kUpdTileW; q += 256) {
    const int i = q / kUpdTileW, c = q % kUpdTileW;
    if (i >= tl.h || c >= tl.w) continue;
    const int Y = tl.y0 + i, X = tl.x0 + c;
    const int64_t p = (int64_t)Y * j.nx + X, pp = (int64_t)(Y + B) * xpitch + (X + B);
    const float xo = xin[pp];
    float gdat = gp(j.gdat)[p];
    if (z2on) gdat += (xo - gp(j.z2)[pp]) * j.inv_rho2;
    float xi, zeta_unused;
    gauss_pair(j.key0, j.key1, j.chain, p, t, xi, zeta_unused);
    const float proj = fminf(fmaxf(xo, 0.0f), 1.0f);
    float xn = xo - j.delta * gdat - j.cprior * gp(j.G)[p] + j.cproj * (proj - xo) + j.sq2d * xi;
    bad |= !isfinite(xn);
    if (j.xpos) xn = fmaxf(xn, 0.0f);
    xout[pp] = xn;
    if (stats) {
      float m = nw > 1 ? gp(j.wmean)[p] : 0.0f, M = nw > 1 ? gp(j.wm2)[p] : 0.0f;
      const float d = xn - m;
      m = fmaf(d, inv_nw, m);
      M = fmaf(d, xn - m, M);
      if (merge) {
        const double n = n_a + n_b;
        const double ma = na_i > 0 ? gp(j.mean)[p] : 0.0;
        const double Ma = na_i > 0 ? gp(j.m2)[p] : 0.0;
        const double dl = (double)m - ma;
        gp(j.mean)[p] = ma + dl * (n_b / n);
        gp(j.m2)[p] = Ma + (double)M + dl * dl * (n_a * n_b / n);
      } else {
        gp(j.wmean)[p] = m;
        gp(j.wm2)[p] = M;
      }
    }
  }
  if (bad) gp(j.flag)[0] = 1;
}

hipError_t launch_update_pointwise(const UpdateArgs &a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL(update_pointwise_kernel, dim3(n_tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Merge a partially filled FP32 window (nw samples on top of n_a merged
// ones) into the FP64 statistics of one job.
__global__ __launch_bounds__(256) void welford_flush_kernel(JobDesc j, double n_a, double n_b) {
  const int64_t n_pix = (int64_t)j.ny * j.nx;
  const double n = n_a + n_b;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n_pix;
       p += (int64_t)gridDim.x * 256) {
    const double ma = n_a > 0 ? gp(j.mean)[p] : 0.0;
    const double Ma = n_a > 0 ? gp(j.m2)[p] : 0.0;
    const double dl = (double)gp(j.wmean)[p] - ma;
    gp(j.mean)[p] = ma + dl * (n_b / n);
    gp(j.m2)[p] = Ma + (double)gp(j.wm2)[p] + dl * dl * (n_a * n_b / n);
  }
}

// MMSE estimate and pixel variance of one job into FP32 device arrays
// (either may be null): mean = mu, var = M2 / (n - 1) (0 when n < 2)
__global__ __launch_bounds__(256) void stats_out_kernel(JobDesc j, int64_t n, float *mean,
                                                        float *var) {
  const int64_t n_pix = (int64_t)j.ny * j.nx;
  const double inv = n >= 2 ? 1.0 / (double)(n - 1) : 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n_pix;
       p += (int64_t)gridDim.x * 256) {
    if (mean) mean[p] = n >= 1 ? (float)gp(j.mean)[p] : 0.0f;
    if (var) var[p] = (float)(gp(j.m2)[p] * inv);
  }
}

hipError_t launch_stats_out(const JobDesc &j, int64_t n, float *mean, float *var, hipStream_t s) {
  const int64_t n_pix = (int64_t)j.ny * j.nx;
  int blocks = (int)std::min<int64_t>((n_pix + 255) / 256, 8192);
  hipLaunchKernelGGL(stats_out_kernel, dim3(blocks), dim3(256), 0, s, j, n, mean, var);
  return hipGetLastError();
}

// max |p[i]| over n floats into *out (float bits; all values >= 0 so the
// unsigned order is the float order)
__global__ __launch_bounds__(256) void amax_kernel(const float *p, size_t n, uint32_t *out) {
  float m = 0.0f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    m = fmaxf(m, fabsf(p[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

hipError_t launch_amax(const float *p, size_t n, uint32_t *out, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(amax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, out);
  return hipGetLastError();
}

size_t update_lds_bytes(int r) {
  const int TH = kUpdTileH, TW = kUpdTileW;
  const int WH = TH + 4 * r, WW = TW + 4 * r, RH = TH + 2 * r, RW = TW + 2 * r;
  // the residual's row pass shares the x row pass's buffer (RH x TW <= WH x RW),
  // which also holds a non-separable kernel's taps
  return sizeof(float) * ((size_t)WH * WW + (size_t)WH * RW + (size_t)RH * RW);
}

template <int RT, int MODE>
static hipError_t launch_update_t(const UpdateArgs &a, int n_tiles, int max_r, hipStream_t s) {
  const size_t lds = update_lds_bytes(max_r);
  static size_t attr = 0;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fused_update_kernel<RT, MODE>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  hipLaunchKernelGGL((fused_update_kernel<RT, MODE>), dim3(n_tiles), dim3(kUpdThreads), lds, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_fused_update(const UpdateArgs &a, int n_tiles, int max_r, bool uniform_r,
                               int mode, hipStream_t s) {
  if (mode == 1) {
    if (uniform_r && max_r == 4) return launch_update_t<4, 1>(a, n_tiles, max_r, s);
    return launch_update_t<0, 1>(a, n_tiles, max_r, s);
  }
  if (uniform_r) {
    switch (max_r) {                             // the blur sizes 5, 7 and 9
      case 2: return launch_update_t<2, 0>(a, n_tiles, max_r, s);
      case 3: return launch_update_t<3, 0>(a, n_tiles, max_r, s);
      case 4: return launch_update_t<4, 0>(a, n_tiles, max_r, s);
      default: break;
    }
  }
  return launch_update_t<0, 0>(a, n_tiles, max_r, s);
}

hipError_t launch_welford_flush(const JobDesc &j, double n_a, double n_b, hipStream_t s) {
  const int64_t n_pix = (int64_t)j.ny * j.nx;
  int blocks = (int)((n_pix + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(welford_flush_kernel, dim3(blocks), dim3(256), 0, s, j, n_a, n_b);
  return hipGetLastError();
}

}  // namespace pnp
