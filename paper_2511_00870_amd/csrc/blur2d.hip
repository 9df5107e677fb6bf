// blur2d.hip -- the likelihood gradient for large, non-separable blurs
// (arXiv 2511.00870, Sec. III-A2: motion-blur kernels up to 129 x 129; the
// data term of Eq. (sgs_pnp_ula_psgla:pnp_ula) and Algorithm 1).
//
// With a half-width r above the fused update's limit the blur and its
// adjoint no longer fit one tile's LDS window together, so the data term
// runs as two direct correlations over the whole image:
//   1. res = m (K x - v) on every pixel (v = y, the exact z draw, or
//      eta-scaled with z1 for PSGLA chains), stored with a zero border of
//      width r;
//   2. gdat = K^T res / s2 on every pixel;
// and the update reads gdat.  K x = corr(x, flip(k)), K^T res = corr(res, k).
// Each workgroup computes one 32 x 64 output tile from an LDS window of
// (32 + 2r) x (64 + 2r) pixels; each thread keeps a row of 8 outputs in
// registers and walks the kernel in chunks of 8 taps (16 window values read
// as four 16-byte LDS reads, 8 taps from scalar registers, 64 FMAs).
#include <mutex>

#include "device_common.h"
#include "kernels.h"

namespace pnp {

namespace {
constexpr int kBThreads = 256;
typedef float b_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int blur_ww(int kpitch) { return kUpdTileW + kpitch + 8; }

// acc[o] = sum_{a,b} kc[a][b] win(ti + a, c0 + o + b), o = 0..7, for the
// thread's row ti = tid / 8 and columns c0 = 8 (tid % 8) of a 32 x 64 output
// tile; the window (32 + 2r) x (64 + 2r) starts r rows / columns before the
// tile and is filled by load(Y, X) (global coordinates), zero beyond it
template <class Load>
__device__ __forceinline__ void corr_tile(float *sw, const PNP_CONST TileRef &tl, int r, int Lp,
                                          const PNP_CONST float *kc, Load load, float acc[8]) {
  constexpr int TH = kUpdTileH, TW = kUpdTileW;
  const int L = 2 * r + 1;
  const int WH = TH + 2 * r, WWp = blur_ww(Lp), WV = TW + 2 * r;
  const int tid = threadIdx.x;
  for (int q = tid; q < WH * WWp; q += kBThreads) {
    const int i = q / WWp, c = q % WWp;
    sw[q] = c < WV ? load(tl.y0 - r + i, tl.x0 - r + c) : 0.0f;
  }
  __syncthreads();
  const int ti = tid >> 3, c0 = 8 * (tid & 7);
#pragma unroll
  for (int o = 0; o < 8; ++o) acc[o] = 0.0f;
  for (int ka = 0; ka < L; ++ka) {
    const float *row = sw + (ti + ka) * WWp + c0;
    const PNP_CONST float *kr = kc + ka * Lp;
    for (int b0 = 0; b0 < Lp; b0 += 8) {
      float xv[16];
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const b_f32x4 u = *reinterpret_cast<const b_f32x4 *>(row + b0 + 4 * v4);
        xv[4 * v4] = u.x;
        xv[4 * v4 + 1] = u.y;
        xv[4 * v4 + 2] = u.z;
        xv[4 * v4 + 3] = u.w;
      }
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) {
        const float wv = kr[b0 + bb];
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[o] = fmaf(wv, xv[o + bb], acc[o]);
      }
    }
  }
}
}  // namespace

__global__ __launch_bounds__(kBThreads) void blur_big_kernel(BlurArgs a) {
  extern __shared__ __attribute__((aligned(16))) float sw[];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const int r = j.r;
  const int epi = a.epi;
  float acc[8];
  {
    // the sources carry a zero border: the residual of r, x of xborder
    const bool from_res = epi == EPI_GRAD;
    const PNP_GLOBAL float *src = from_res ? gp(j.res) : gp(j.x[t & 1]);
    const int64_t pitch = from_res ? j.rpitch : (int64_t)j.xpitch;
    const int off = from_res ? r : j.xborder;
    corr_tile(sw, tl, r, j.kpitch, cp(j.kbig[from_res ? 1 : 0]),
              [&](int Y, int X) { return src[(int64_t)(Y + off) * pitch + (X + off)]; }, acc);
  }
  const int ti = threadIdx.x >> 3, c0 = 8 * (threadIdx.x & 7);
  if (ti >= tl.h) return;
  const int Y = tl.y0 + ti;
  const int B = j.xborder;
  const int64_t xpitch = j.xpitch;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int X = tl.x0 + c0 + o;
    if (c0 + o >= tl.w) break;
    const int64_t pr = (int64_t)(Y + r) * j.rpitch + (X + r);
    if (epi == EPI_GRAD) {
      gp(j.gdat)[(int64_t)Y * j.nx + X] = acc[o] * j.inv_s2;
    } else if (epi == EPI_KX) {
      gp(j.res)[pr] = acc[o];
    } else {
      const int64_t pp = (int64_t)(Y + B) * xpitch + (X + B);
      const float kx = acc[o];
      const float mv = j.has_mask ? (float)gp(j.mask)[pp] : 1.0f;
      float res;
      if (j.zmode == 1) {
        res = mv * (j.eta * (mv * kx) - gp(j.z1)[pp]);
      } else if (!j.split) {
        res = mv * (kx - gp(j.y)[pp]);
      } else if (t < 1) {
        res = mv * kx;                                         // z^(0) = 0
      } else {
        float xi, zeta;
        gauss_pair(j.key0, j.key1, j.chain, (int64_t)Y * j.nx + X, t, xi, zeta);
        res = mv * (j.zmix * (kx - gp(j.y)[pp]) - j.zsd * zeta);
      }
      gp(j.res)[pr] = res;
    }
  }
}

// The data-fidelity gradient of an arbitrary image x (compact ny*nx, zero
// outside the image): epi 0: res = m (K x - y) into a compact buffer; epi 1:
// g = K^T res / sigma^2.  One job, its update tiles.
__global__ __launch_bounds__(kBThreads) void data_grad_kernel(GradArgs a) {
  extern __shared__ __attribute__((aligned(16))) float sw[];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int r = j.r, ny = j.ny, nx = j.nx;
  const PNP_GLOBAL float *src = gp(a.epi == 0 ? a.x : a.res);
  float acc[8];
  corr_tile(sw, tl, r, j.kpitch, cp(j.kbig[a.epi == 0 ? 0 : 1]),
            [&](int Y, int X) {
              return (Y >= 0 && Y < ny && X >= 0 && X < nx) ? src[(int64_t)Y * nx + X] : 0.0f;
            },
            acc);
  const int ti = threadIdx.x >> 3, c0 = 8 * (threadIdx.x & 7);
  if (ti >= tl.h) return;
  const int Y = tl.y0 + ti;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    if (c0 + o >= tl.w) break;
    const int X = tl.x0 + c0 + o;
    const int64_t p = (int64_t)Y * nx + X;
    if (a.epi == 0) {
      const int64_t pp = (int64_t)(Y + j.xborder) * j.xpitch + (X + j.xborder);
      const float mv = j.has_mask ? (float)gp(j.mask)[pp] : 1.0f;
      gp(a.res)[p] = mv * (acc[o] - gp(j.y)[pp]);
    } else {
      gp(a.g)[p] = acc[o] * j.inv_sig2;
    }
  }
}

hipError_t launch_data_grad(const GradArgs &a, int n_tiles, int r, int kpitch, hipStream_t s) {
  const size_t lds = blur_big_lds_bytes(r, kpitch);
  static size_t attr = 0;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&data_grad_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  hipLaunchKernelGGL(data_grad_kernel, dim3(n_tiles), dim3(kBThreads), lds, s, a);
  return hipGetLastError();
}

size_t blur_big_lds_bytes(int r, int kpitch) {
  return sizeof(float) * (size_t)(kUpdTileH + 2 * r) * (size_t)(kUpdTileW + kpitch + 8);
}

hipError_t launch_blur_big(const BlurArgs &a, int n_tiles, int max_r, int kpitch, hipStream_t s) {
  const size_t lds = blur_big_lds_bytes(max_r, kpitch);
  static size_t attr = 0;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&blur_big_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  hipLaunchKernelGGL(blur_big_kernel, dim3(n_tiles), dim3(kBThreads), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Allocation-free data gradient: the residual of the first pass lives in a
// static device buffer instead of memory allocated per call.  Each device
// the library runs on holds its own copy until the process ends; its device
// address is looked up once per device at context set-up.
// ---------------------------------------------------------------------
static __device__ __align__(256) float scratch[kNoallocMaxPixels];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<float *>(p);
  return hipSuccess;
}

float *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace pnp
