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
// Each workgroup computes one 32 x 64 output tile from a window of
// (32 + 2r) x (64 + 2r) pixels, of which LDS holds a ring of 48 rows (39 KB
// at r = 64, four workgroups per CU), on the matrix cores: for one kernel row a,
// out[y][x0 + n] = sum_j win[y + a][x0 + j] k[a][j - n] is a GEMM whose B
// operand is a band (Toeplitz) slice of that row, so v_mfma_f32_16x16x4f32
// takes 16 output rows x 16 columns per block and 4 shifts j per K step
// (L + 15 shifts per row: 1 + 15/L times the algorithmic work).
#include <mutex>

#include "device_common.h"
#include "kernels.h"

namespace pnp {

namespace {
constexpr int kBThreads = 256;
typedef float b_f32x4 __attribute__((ext_vector_type(4)));

// K steps (4 shifts each) per kernel row, a multiple of four (steps past the
// band meet zero weights), and the LDS layout: the window's
// row pitch is at least the columns the K steps read (16 w + 4 NJ) and 4 mod
// 64, so the 16 rows x 4 columns of an A fragment fall on 64 distinct banks;
// two kernel-row buffers with 16 zeros on either side supply the band's
// zero weights
__host__ __device__ constexpr int blur_nj(int L) { return ((L + 15 + 3) / 4 + 3) / 4 * 4; }
__host__ __device__ constexpr int blur_wwm(int r) {
  const int need = 48 + 4 * blur_nj(2 * r + 1);
  return (need + 59) / 64 * 64 + 4;
}
__host__ __device__ constexpr int blur_kb(int r) { return 4 * blur_nj(2 * r + 1) + 32; }
// window rows in the ring: window row y sits at slot y % kRing.  Kernel row a
// reads rows a .. a + 31 while row a + 32 is stored into the slot of row
// a - 16; with a row pitch of 4 mod 64 floats, any 16 cyclically consecutive
// slots of a ring whose length is a multiple of 16 fall on distinct banks
constexpr int kRing = 48;
static_assert(kRing % 16 == 0 && kRing >= kUpdTileH + 1, "ring length");
static_assert(blur_wwm(kMaxRBig) <= kBThreads, "one window column per thread");

// acc[mb] (mb = 0, 1) = the 16 x 16 output block at rows 16 mb .. 16 mb + 15
// and columns 16 w .. 16 w + 15 of a 32 x 64 output tile (w = the wave):
// lane l holds rows 16 mb + 4 (l / 16) + i (i = 0..3), column 16 w + l % 16,
// of sum_{a,b} kc[a][b] win(row + a, col + b).  The window (32 + 2r) x
// (64 + 2r) starts r rows / columns before the tile; load(Y, X) (global
// coordinates) gives its values, zero beyond it.  Its rows pass through the
// ring: kernel row a reads window rows a .. a + 31, and window row a + 32 and
// kernel row a + 1 are loaded into registers while row a runs and stored
// (the window row at its slot, the kernel row into the other of two buffers)
// before the row's barrier.
template <class Load>
__device__ __forceinline__ void corr_tile(float *sw, const PNP_CONST TileRef &tl, int r, int Lp,
                                          const PNP_CONST float *kc, Load load, b_f32x4 acc[2]) {
  constexpr int TH = kUpdTileH, TW = kUpdTileW;
  static_assert(TH == 32 && TW == 64 && kBThreads == 256, "two 16-row blocks per wave");
  const int L = 2 * r + 1, NJ = blur_nj(L), KB = blur_kb(r);
  const int WH = TH + 2 * r, WW = blur_wwm(r), WV = TW + 2 * r;
  float *kb = sw + kRing * WW;                   // two rows of KB floats
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, m = lane & 15, k = lane >> 4;
  for (int q = tid; q < TH * WW; q += kBThreads) {
    const int i = q / WW, c = q % WW;
    sw[q] = c < WV ? load(tl.y0 - r + i, tl.x0 - r + c) : 0.0f;
  }
  for (int q = tid; q < 2 * KB; q += kBThreads) {
    const int t = q % KB - 16;
    kb[q] = (q < KB && t >= 0 && t < L) ? kc[t] : 0.0f;
  }
  __syncthreads();
  acc[0] = b_f32x4{0.f, 0.f, 0.f, 0.f};
  acc[1] = b_f32x4{0.f, 0.f, 0.f, 0.f};
  // A: window row (16 mb + m + a), column 16 w + 4 js + k; B: the band entry
  // k[a][4 js + k - n] for this lane's n = m
  const int bo = 16 + k - m;
  const bool wcol = tid < WW;
  int slot = 0;                                  // ring slot of window row a
  for (int a = 0; a < L; ++a) {
    // the next kernel row and window row: loaded now, stored after this
    // row's MFMAs
    const bool nk = a + 1 < L && tid < L;
    const float kn = nk ? kc[(int64_t)(a + 1) * Lp + tid] : 0.0f;
    const bool nw = a + TH < WH && wcol;
    const float wn = (nw && tid < WV) ? load(tl.y0 - r + a + TH, tl.x0 - r + tid) : 0.0f;
    const float *kr = kb + (a & 1) * KB + bo;
    int s0 = slot + m, s1 = s0 + 16;               // slots of rows a + m, a + m + 16
    s0 = s0 >= kRing ? s0 - kRing : s0;
    s1 = s1 >= kRing ? s1 - kRing : s1;
    const float *w0 = sw + s0 * WW + 16 * w + k, *w1 = sw + s1 * WW + 16 * w + k;
    // K steps in batches of four, the next batch's operands read from LDS
    // before this batch's MFMAs
    float ca[2][4], cb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cb[u] = kr[4 * u];
      ca[0][u] = w0[4 * u];
      ca[1][u] = w1[4 * u];
    }
    for (int jb = 0; jb < NJ; jb += 4) {
      float na[2][4], nb[4];
      if (jb + 4 < NJ) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          nb[u] = kr[4 * (jb + 4 + u)];
          na[0][u] = w0[4 * (jb + 4 + u)];
          na[1][u] = w1[4 * (jb + 4 + u)];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[0][u], cb[u], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[1][u], cb[u], acc[1], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cb[u] = nb[u];
        ca[0][u] = na[0][u];
        ca[1][u] = na[1][u];
      }
    }
    // window row a + 32 goes to the slot of row a + 32 - kRing, last read
    // before an earlier barrier and not among this row's slots
    const int ns = slot + TH >= kRing ? slot + TH - kRing : slot + TH;
    if (nw) sw[ns * WW + tid] = wn;
    if (nk) kb[((a + 1) & 1) * KB + 16 + tid] = kn;
    __syncthreads();
    slot = slot + 1 == kRing ? 0 : slot + 1;
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
  b_f32x4 acc[2];
  {
    // the sources carry a zero border: the residual of r, x of xborder
    const bool from_res = epi == EPI_GRAD;
    const PNP_GLOBAL float *src = from_res ? gp(j.res) : gp(j.x[t & 1]);
    const int64_t pitch = from_res ? j.rpitch : (int64_t)j.xpitch;
    const int off = from_res ? r : j.xborder;
    corr_tile(sw, tl, r, j.kpitch, cp(j.kbig[from_res ? 1 : 0]),
              [&](int Y, int X) { return src[(int64_t)(Y + off) * pitch + (X + off)]; }, acc);
  }
  const int lane = threadIdx.x & 63, col = 16 * (threadIdx.x >> 6) + (lane & 15);
  if (col >= tl.w) return;
  const int X = tl.x0 + col;
  const int B = j.xborder;
  const int64_t xpitch = j.xpitch;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int row = 16 * (o >> 2) + 4 * (lane >> 4) + (o & 3);
    if (row >= tl.h) continue;
    const int Y = tl.y0 + row;
    const float kx = acc[o >> 2][o & 3];
    const int64_t pr = (int64_t)(Y + r) * j.rpitch + (X + r);
    if (epi == EPI_GRAD) {
      gp(j.gdat)[(int64_t)Y * j.nx + X] = kx * j.inv_s2;
    } else if (epi == EPI_KX) {
      gp(j.res)[pr] = kx;
    } else {
      const int64_t pp = (int64_t)(Y + B) * xpitch + (X + B);
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
  b_f32x4 acc[2];
  corr_tile(sw, tl, r, j.kpitch, cp(j.kbig[a.epi == 0 ? 0 : 1]),
            [&](int Y, int X) {
              return (Y >= 0 && Y < ny && X >= 0 && X < nx) ? src[(int64_t)Y * nx + X] : 0.0f;
            },
            acc);
  const int lane = threadIdx.x & 63, col = 16 * (threadIdx.x >> 6) + (lane & 15);
  if (col >= tl.w) return;
  const int X = tl.x0 + col;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int row = 16 * (o >> 2) + 4 * (lane >> 4) + (o & 3);
    if (row >= tl.h) continue;
    const int Y = tl.y0 + row;
    const float v = acc[o >> 2][o & 3];
    const int64_t p = (int64_t)Y * nx + X;
    if (a.epi == 0) {
      const int64_t pp = (int64_t)(Y + j.xborder) * j.xpitch + (X + j.xborder);
      const float mv = j.has_mask ? (float)gp(j.mask)[pp] : 1.0f;
      gp(a.res)[p] = mv * (v - gp(j.y)[pp]);
    } else {
      gp(a.g)[p] = v * j.inv_sig2;
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
  (void)kpitch;
  return sizeof(float) * ((size_t)kRing * (size_t)blur_wwm(r) + 2 * (size_t)blur_kb(r));
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
