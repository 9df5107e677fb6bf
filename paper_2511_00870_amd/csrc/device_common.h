// device_common.h -- data layout shared by the host runtime and the gfx950
// kernels of the PnP-ULA sampler: per-chain job descriptors, tile lists,
// the Philox4x32-10 generator and the bf16 / e4m3 conversions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pnp {

enum Fmt : int { FMT_F32 = 0, FMT_BF16 = 1, FMT_E4M3 = 2 };

constexpr int kMaxR = 8;           // largest blur half-width (L <= 17)
constexpr int kUpdTileH = 32;      // fused-update tile (rows x cols) and workgroup size
constexpr int kUpdTileW = 64;
constexpr int kUpdThreads = 512;
constexpr int kConvTileW = 32;     // convolution tiles are TH x 32 pixels
constexpr int kPairTileH = 14;     // e4m3 pair kernel: output tiles of 14 x 30
constexpr int kPairTileW = 30;
constexpr int kPairWsTileH = 9;   // split-layer pair kernel: output tiles of 9 x 30
constexpr int kPair8WsTileH = 20; // e4m3 split-layer pair kernel: output tiles of 20 x 30
constexpr int kDdTile = 30;        // DDFB stage kernel: output tiles of 30 x 30
constexpr int kMaxDdfbLayers = 8;  // DDFB iterations K
constexpr int kMaxRBig = 64;       // largest blur half-width (L <= 129)

// One chain resident on the device.  All images live in padded row-major
// buffers whose zero border is never written, so stencils read it as the
// zero boundary of the operators.
struct JobDesc {
  int32_t ny, nx;          // image size
  int32_t xpitch;          // floats per row of the x / y / mask buffers
  int32_t xborder;         // zero border (rows and columns) of those buffers
  int32_t apitch;          // pixels per row of the activation buffers (border 1)
  int32_t r;               // blur half-width
  int32_t separable;       // blur kernel = u v^T
  int32_t has_mask;
  int32_t split;           // rho > 0
  int32_t burn_in;
  int32_t wwin;            // Welford window
  int32_t arows;           // rows of the activation buffers (border 1, then slack)
  int64_t t_offset;        // this chain's t = tick + t_offset
  int64_t wbase;           // sample number of the last out-of-band merge point
                           // (flush, restore or state change); windows of wwin
                           // samples are merged from there on
  int64_t nbase;           // FP64 sample count at that point
  // buffers (device)
  float *x[2];             // ping-pong x^(t): x[t & 1] holds x^(t)
  const float *y;          // padded observation
  const uint8_t *mask;     // padded {0,1} mask or null
  void *act[4];            // activation buffers (channels-last, border 1); each
                           // holds one storage format (two per format in use)
  float *G;                // ny*nx denoiser output (compact)
  float *wmean, *wm2;      // FP32 Welford window (compact)
  double *mean, *m2;       // FP64 merged statistics (compact)
  int32_t *flag;           // non-finite flag
  float *S;                // last layer fused into the last middle layer: per pixel 12
                           // floats, the 9 per-tap partial dot products (zero border 1,
                           // row pitch nx + 2 records; one trash record at the end)
  const float *kern;       // L*L blur (2-D path)
  const float *ku, *kv;    // separable factors k[a][c] = ku[a] kv[c]
  // coefficients, computed in FP64 on the host and rounded once
  float delta;             // Langevin step
  float cprior;            // alpha delta / eps
  float cproj;             // delta / lambda
  float sq2d;              // sqrt(2 delta)
  float inv_s2;            // 1/sigma^2 (rho == 0) or 1/rho
  float zmix;              // rho / (rho + sigma^2): Hx - z = zmix (Hx - y) - zsd zeta
  float zsd;               // sqrt(rho sigma^2 / (rho + sigma^2))
  float inv_sig2;          // 1/sigma^2 (the data-gradient entry point)
  uint32_t key0, key1, chain, pad2;
  // ---- splitting variables held as chain state, and the other priors ----
  // zmode 1: PSGLA z-steps (Eq. (sgs_pnp_ula_psgla:psgla)): z1 ~ eta m K x with
  //   the data term (Gaussian, or Poisson KL(y || .)) as f, and optionally z2 ~ x
  //   with the indicator of R+; the x-step's data gradient is
  //   eta K^T m (eta m K x - z1)/rho + (x - z2)/rho2.
  // zmode 2: TV prior through AXDA (Sec. III-B2): z = (zh, zv) ~ D x with
  //   beta ||.||_{2,1}; the x-step adds (1/rho) D^T (D x - z) (held in G) and
  //   ends with the projection onto R+.
  int32_t zmode;
  int32_t poisson;         // z1's data term is KL(y || .) (else Gaussian)
  int32_t has_z2;          // second block z2
  int32_t xpos;            // the x-update ends with max(., 0)
  float *z1, *z2;          // padded like x (zero border); TV: zh, zv
  float eta;               // operator scale of the PSGLA residual
  float za1, zs1;          // z1 (TV: z) step: kappa/rho and sqrt(2 kappa)
  float za2, zs2;          // z2 step: kappa2/rho2 and sqrt(2 kappa2)
  float zkappa;            // prox parameter: kappa (TV: kappa beta)
  float zsig2;             // Gaussian data term of z1: sigma^2
  float inv_rho2;          // 1/rho2
  float inv_rho;           // TV: 1/rho of the coupling term
  float pad3;
  // large blur (half-width above kMaxR): the residual m (K x - v) on the whole
  // image, padded with a zero border of width r (row pitch rpitch floats)
  float *res;
  int64_t rpitch;
  float *gdat;             // large blur: the data gradient K^T res / s2 (compact)
  const float *kbig[2];    // large blur: [0] the kernel flipped, [1] as is; rows of
                           // kpitch floats (a multiple of 8, zero padded)
  int32_t kpitch;
  int32_t big;             // blur half-width above kMaxR
  // DDFB prior: maps b_1 .. b_{K-1} of the unrolled dual forward-backward
  // iterations, padded like x (zero border), dstride floats apart
  float *dmaps;
  int64_t dstride;
};

// A rectangle of one job's image: rows [y0, y0+h), cols [x0, x0+w).
// 32-bit fields only: kernels read it with scalar loads.
struct TileRef {
  int32_t job;
  int32_t y0, x0;
  int32_t h, w;
  int32_t pad[3];
};

// Pointers read out of a JobDesc are generic pointers to the compiler, and
// generic (flat) memory instructions also count against the LDS wait counter:
// a kernel waiting for its LDS reads would wait for every outstanding flat load
// too.  Device code therefore re-types them to the global address space.
#define PNP_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ PNP_GLOBAL T *gp(T *p) {
  return (PNP_GLOBAL T *)p;
}
// Descriptors (tile lists, JobDesc) are never written by a kernel; read
// through the constant address space, uniform reads of them become scalar
// loads, which a kernel can wait on without waiting for its outstanding
// vector-memory loads and stores.
#define PNP_CONST __attribute__((address_space(4)))
template <class T> __device__ __forceinline__ const PNP_CONST T *cp(const T *p) {
  return (const PNP_CONST T *)p;
}

// Tile of a one-workgroup-per-tile launch.  Workgroups are dispatched round
// robin over the 8 XCDs (workgroup b runs on XCD b mod 8); each XCD is given
// a contiguous run of the block-major tile list, so the halo rows that
// neighbouring tiles share are read once into that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, rem = n & 7, x = b & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

// --------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (X0..X3) -> (hi(M1 X2) ^ X1 ^ K0, lo(M1 X2), hi(M0 X0) ^ X3 ^ K1, lo(M0 X0))
// with the key bumped by (W0, W1) between rounds.
// --------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product each (v_mad_u64_u32) instead of a low and
    // a high multiply
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Two standard normals of pixel p at iteration t: (cos, sin) Box-Muller
// branches on 24-bit uniforms, exact in FP32.
__device__ __forceinline__ void gauss_pair(uint32_t key0, uint32_t key1, uint32_t chain,
                                           int64_t p, int64_t t, float &xi, float &zeta) {
  uint4 c = make_uint4((uint32_t)p, (uint32_t)t, chain, (uint32_t)((uint64_t)p >> 32));
  uint4 w = philox4x32_10(c, key0, key1);
  const float u1 = (float)((w.x >> 8) + 1u) * 5.9604644775390625e-8f;  // 2^-24
  const float u2 = (float)(w.y >> 8) * 5.9604644775390625e-8f;
  // hardware transcendentals: v_log_f32 (log2), v_sqrt_f32, and v_sin_f32 /
  // v_cos_f32, whose argument is in revolutions, so sin(2 pi u2) takes u2
  // as is (|error| ~1e-7, far below the noise scale's effect on x)
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  xi = rad * __builtin_amdgcn_cosf(u2);
  zeta = rad * __builtin_amdgcn_sinf(u2);
}

// Three standard normals of pixel p at counter t (the z-steps): the cosine
// and sine branches of the pair above from words (w0, w1), and the cosine
// branch of a second Box-Muller pair from (w2, w3).
__device__ __forceinline__ void gauss_triple(uint32_t key0, uint32_t key1, uint32_t chain,
                                             int64_t p, int64_t t, float &g0, float &g1,
                                             float &g2) {
  uint4 c = make_uint4((uint32_t)p, (uint32_t)t, chain, (uint32_t)((uint64_t)p >> 32));
  uint4 w = philox4x32_10(c, key0, key1);
  const float u1 = (float)((w.x >> 8) + 1u) * 5.9604644775390625e-8f;
  const float u2 = (float)(w.y >> 8) * 5.9604644775390625e-8f;
  const float u3 = (float)((w.z >> 8) + 1u) * 5.9604644775390625e-8f;
  const float u4 = (float)(w.w >> 8) * 5.9604644775390625e-8f;
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  const float rad2 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u3));
  g0 = rad * __builtin_amdgcn_cosf(u2);
  g1 = rad * __builtin_amdgcn_sinf(u2);
  g2 = rad2 * __builtin_amdgcn_cosf(u4);
}

// --------------------------------------------------------------------
// bf16 and OCP e4m3fn conversions (round to nearest even; e4m3 saturates)
// --------------------------------------------------------------------
// gfx950 converts in hardware (v_cvt_pk_bf16_f32, round to nearest even; a
// NaN stays a quiet NaN)
typedef __attribute__((ext_vector_type(2))) float pnp_f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 pnp_bf16x2;
__device__ __forceinline__ uint16_t f32_to_bf16(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
// two values: the low half holds lo
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(pnp_f32x2{lo, hi}, pnp_bf16x2));
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}
__device__ __forceinline__ float round_bf16(float v) { return bf16_to_f32(f32_to_bf16(v)); }

__device__ __forceinline__ uint8_t f32_to_e4m3_sw(float v) {
  // branch-free (selects only): NaN -> 0x7f, |v| >= 448 -> 448 (0x7e),
  // |v| < 2^-6 -> subnormal step 2^-9, else round to 3 mantissa bits (RNE)
  const uint32_t u = __float_as_uint(v);
  const uint32_t sign = (u >> 24) & 0x80u;
  const float a = fabsf(v);
  uint32_t b = __float_as_uint(a);
  b += 0x7ffffu + ((b >> 20) & 1u);
  const uint32_t normal = (((b >> 23) - 120u) << 3) | ((b >> 20) & 7u);
  const uint32_t sub = (uint32_t)rintf(a * 512.0f);          // 0..8 (8 = 2^-6)
  uint32_t r = a < 0.015625f ? sub : normal;
  r = a >= 448.0f ? 0x7eu : r;
  r = a != a ? 0x7fu : r;
  return (uint8_t)(sign | r);
}
// gfx950's v_cvt_pk_fp8_f32 (OCP e4m3, round to nearest even) on inputs
// clamped to +-448 gives the same codes as the rounding above for every
// finite float (checked exhaustively for |v| <= 1024; beyond, both give
// 448); NaN inputs take the rounding above
__device__ __forceinline__ float e4m3_clamp(float v) { return __builtin_amdgcn_fmed3f(v, -448.0f, 448.0f); }
__device__ __forceinline__ uint8_t f32_to_e4m3(float v) {
  const uint8_t h = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(v), 0.0f, 0, false) & 0xff);
  return v != v ? f32_to_e4m3_sw(v) : h;
}
// four values, the first in the low byte
__device__ __forceinline__ uint32_t pack_e4m3x4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), e4m3_clamp(b), 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(c), e4m3_clamp(d), w, true);
  uint32_t r = (uint32_t)w;
  if (a != a || b != b || c != c || d != d)
    r = (uint32_t)f32_to_e4m3_sw(a) | ((uint32_t)f32_to_e4m3_sw(b) << 8) |
        ((uint32_t)f32_to_e4m3_sw(c) << 16) | ((uint32_t)f32_to_e4m3_sw(d) << 24);
  return r;
}
// four values known not to be NaN (e.g. after a ReLU taken with fmaxf,
// which returns the non-NaN operand): no fallback branch
// ReLU and e4m3 of four values already multiplied by the activation scale's
// inverse: the clamp to [0, 448] is the ReLU and the saturation at once
__device__ __forceinline__ float e4m3_relu_clamp(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 448.0f); }
__device__ __forceinline__ uint32_t pack_e4m3x4_relu(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_relu_clamp(a), e4m3_relu_clamp(b), 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_relu_clamp(c), e4m3_relu_clamp(d), w, true);
  return (uint32_t)w;
}
__device__ __forceinline__ uint32_t pack_e4m3x4_nonan(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(a), e4m3_clamp(b), 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp(c), e4m3_clamp(d), w, true);
  return (uint32_t)w;
}
__device__ __forceinline__ float e4m3_to_f32(uint8_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u;
  float v = (e == 0) ? (float)m * 0.001953125f                 // m 2^-9
                     : __uint_as_float(((e + 120u) << 23) | (m << 20));
  return (c & 0x80) ? -v : v;
}

}  // namespace pnp
