// conv.hip -- the denoiser's 3x3 convolution layers on gfx950.
//
// Denoiser (arXiv 2511.00870, Sec. II-B1, Eqs. (feedforward_cnn) and
// (cnn:convolution), Example 2): G = T_K o ... o T_1 with
// T_k(v) = eta_k(W_k * v + b_k), 3x3 kernels, zero ("half") padding at every
// layer, ReLU on layers 1..K-1, identity on layer K, channels 1 -> F -> F -> 1.
//
// Layout: each layer's output is a channels-last image with a one-pixel zero
// border that is never written, so every layer reads its zero padding from
// memory.  Each layer of every block reads the block's core plus a one-pixel
// ghost ring of the previous layer's output (the per-layer exchange of Sec.
// II-B2, as an overlapping read of device memory).
//
// Middle layers (F -> F) are implicit GEMMs on the matrix cores:
//   out[c_out][pixel] = sum_{tap, c_in} W[c_out][tap][c_in] * in[pixel + tap][c_in]
// with the weights as the MFMA A operand (16 output channels per block) and
// the activations as the B operand (16 pixels per block).  A persistent
// workgroup keeps the layer's weights in LDS (fragment order, repacked on the
// host), stages (TH+2) x 34 input pixels per TH x 32 tile in LDS and
// prefetches the next tile into registers while the current one computes.
//   FP32: v_mfma_f32_16x16x4_f32, K grouped 16 channels per 16-byte read.
//   BF16: v_mfma_f32_16x16x32_bf16, 32 channels per step.
//   E4M3: v_mfma_f32_16x16x128_f8f6f4, two taps x 64 channels per step (the
//         tenth tap slot has zero weights).
// First (1 -> F) and last (F -> 1) layers are small VALU stencils.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace pnp {

constexpr int kNwLowp = 8;      // waves of the generic middle-layer kernel for bf16 / e4m3 input
constexpr int kPair8Wpe = 2;    // waves per SIMD the e4m3 pair kernel is compiled for

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;
// native 16-byte vector: a first-class IR type, so arrays of it stay in
// registers (HIP's uint4 struct is copied with memcpy and can be left in
// private memory)
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

template <int FMT> struct FmtInfo;
template <> struct FmtInfo<FMT_F32>  { static constexpr int bytes = 4; };
template <> struct FmtInfo<FMT_BF16> { static constexpr int bytes = 2; };
template <> struct FmtInfo<FMT_E4M3> { static constexpr int bytes = 1; };

// store/load one activation value in a format (scale already applied)
template <int FMT> __device__ __forceinline__ void store_act(void *p, float v);
template <> __device__ __forceinline__ void store_act<FMT_F32>(void *p, float v) {
  *reinterpret_cast<float *>(p) = v;
}
template <> __device__ __forceinline__ void store_act<FMT_BF16>(void *p, float v) {
  *reinterpret_cast<uint16_t *>(p) = f32_to_bf16(v);
}
template <> __device__ __forceinline__ void store_act<FMT_E4M3>(void *p, float v) {
  *reinterpret_cast<uint8_t *>(p) = f32_to_e4m3(v);
}

template <int FMT> __device__ __forceinline__ float load_act(const void *p);
template <> __device__ __forceinline__ float load_act<FMT_F32>(const void *p) {
  return *reinterpret_cast<const float *>(p);
}
template <> __device__ __forceinline__ float load_act<FMT_BF16>(const void *p) {
  return bf16_to_f32(*reinterpret_cast<const uint16_t *>(p));
}
template <> __device__ __forceinline__ float load_act<FMT_E4M3>(const void *p) {
  return e4m3_to_f32(*reinterpret_cast<const uint8_t *>(p));
}

// value as it enters a layer of format FMT (inv_scale = 1/s for e4m3)
template <int FMT> __device__ __forceinline__ float quant_in(float v, float inv_scale);
template <> __device__ __forceinline__ float quant_in<FMT_F32>(float v, float) { return v; }
template <> __device__ __forceinline__ float quant_in<FMT_BF16>(float v, float) {
  return round_bf16(v);
}
template <> __device__ __forceinline__ float quant_in<FMT_E4M3>(float v, float inv_scale) {
  return e4m3_to_f32(f32_to_e4m3(v * inv_scale));
}

// pack 4 consecutive output channels of one pixel and store them (P is a
// byte pointer into LDS or global memory)
typedef __attribute__((ext_vector_type(2))) unsigned int u32x2;
typedef __attribute__((ext_vector_type(2))) short i16x2;
typedef __attribute__((ext_vector_type(4))) short i16x4;
// ReLU of two packed bf16 values: as signed 16-bit integers the negative
// ones (sign bit set) are below zero
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t u) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(i16x2, u), i16x2{0, 0}));
}
template <int FMT, class P> __device__ __forceinline__ void store4(P *p, f32x4 v, float inv_s) {
  if constexpr (FMT == FMT_F32) {
    *reinterpret_cast<f32x4 *>(p) = v;
  } else if constexpr (FMT == FMT_BF16) {
    u32x2 w;
    w.x = pack_bf16x2(v[0], v[1]);
    w.y = pack_bf16x2(v[2], v[3]);
    *reinterpret_cast<u32x2 *>(p) = w;
  } else {
    const uint32_t w = pack_e4m3x4(v[0] * inv_s, v[1] * inv_s, v[2] * inv_s, v[3] * inv_s);
    *reinterpret_cast<uint32_t *>(p) = w;
  }
}

// ---------------------------------------------------------------------
// First layer: 1 -> F.  The tile's x window ((TH+2) x 34, rounded to the
// layer's input format) is staged in LDS; each lane owns one 16-byte group
// of output channels (weights, bias and scale in registers) and walks the
// tile's pixels, so consecutive lanes write consecutive bytes.
// ---------------------------------------------------------------------
template <int IN_FMT, int OUT_FMT, int F>
__global__ __launch_bounds__(256) void conv_first_kernel(ConvArgs a) {
  constexpr int OB = FmtInfo<OUT_FMT>::bytes;
  constexpr int CG = 16 / OB;                  // channels per lane
  constexpr int NG = F / CG;                   // lanes per pixel
  constexpr int PPP = 256 / NG;                // pixels per pass
  constexpr int WW = kConvTileW + 2;
  constexpr int XQ = (18 * WW + 255) / 256;     // window loads per thread (16-row tiles)
  __shared__ float sx[18 * WW];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *xb = gp(j.x[t & 1]);
  const int WH = tl.h + 2, B = j.xborder;
  const int64_t xpitch = j.xpitch;
  // all window loads in flight at once (out-of-range lanes read the origin)
  float xv[XQ];
#pragma unroll
  for (int k = 0; k < XQ; ++k) {
    const int q0 = (int)threadIdx.x + 256 * k, q = q0 < WH * WW ? q0 : 0;
    const int i = q / WW, c = q % WW;
    xv[k] = xb[(tl.y0 - 1 + i + B) * xpitch + (tl.x0 - 1 + c + B)];
  }
#pragma unroll
  for (int k = 0; k < XQ; ++k) {
    const int q = (int)threadIdx.x + 256 * k;
    if (q < WH * WW) sx[q] = quant_in<IN_FMT>(xv[k], a.in_inv_scale);
  }
  const int grp = threadIdx.x % NG, slot = threadIdx.x / NG;
  float w[CG][9], sc[CG], bi[CG];
#pragma unroll
  for (int cc = 0; cc < CG; ++cc) {
#pragma unroll
    for (int k = 0; k < 9; ++k) w[cc][k] = a.wf32[(grp * CG + cc) * 9 + k];
    sc[cc] = a.oscale[grp * CG + cc];
    bi[cc] = a.bias[grp * CG + cc];
  }
  __syncthreads();
  PNP_GLOBAL uint8_t *out = gp(reinterpret_cast<uint8_t *>(j.act[a.out_slot]));
  const int npix = (int)tl.h * tl.w;
  for (int pix = slot; pix < npix; pix += PPP) {
    const int r = pix / tl.w, c = pix % tl.w;
    float q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) q[k] = sx[(r + k / 3) * WW + c + k % 3];
    float v[CG];
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc = fmaf(w[cc][k], q[k], acc);
      float o = acc * sc[cc] + bi[cc];
      if (a.relu) o = fmaxf(o, 0.0f);
      v[cc] = o;
    }
    PNP_GLOBAL uint8_t *dst = out + ((int64_t)(tl.y0 + r + 1) * j.apitch + (tl.x0 + c + 1)) * (F * OB) +
                   grp * 16;
    u32x4 pk;
    if constexpr (OUT_FMT == FMT_F32) {
#pragma unroll
      for (int e = 0; e < 4; ++e) pk[e] = __float_as_uint(v[e]);
    } else if constexpr (OUT_FMT == FMT_BF16) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pk[e] = pack_bf16x2(v[2 * e], v[2 * e + 1]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pk[e] = pack_e4m3x4(v[4 * e] * a.out_inv_scale, v[4 * e + 1] * a.out_inv_scale,
                            v[4 * e + 2] * a.out_inv_scale, v[4 * e + 3] * a.out_inv_scale);
    }
    *reinterpret_cast<PNP_GLOBAL u32x4 *>(dst) = pk;
  }
}

// ---------------------------------------------------------------------
// First layer 1 -> 64 with e4m3 output on the matrix cores, as the e4m3 pair
// kernel's fused first layer computes it (so the codes are the same): x and
// the weights rounded to bf16, one v_mfma_f32_16x16x16_bf16 per 16 pixels and
// 16 channels with K slot 4g + e holding tap (g, e) (zero weights for g or
// e = 3), then fma with the scale and bias that already carry the output's
// inverse activation scale, ReLU and saturation in one clamp, e4m3.  Per
// 16 x 32 tile: the x window (18 x 34) as bf16 in LDS; wave w takes output
// rows 4w .. 4w + 3, two 16-pixel blocks per row.  A lane's four results
// (channels 16 mb + 4g .. + 3 of pixel l16, mb = 0..3) go through one 32-lane
// and one 16-lane swap per pair of registers, after which lane group g holds
// channels 16g .. 16g + 15 of its pixel: one 16-byte store per lane, 1 KB
// contiguous per wave and block.  Each workgroup walks the tiles of its XCD's
// contiguous range (the grid is a multiple of 8 and dispatched round-robin over
// the XCDs), with the weights read once and the next tile's x window loaded
// while the current tile is computed.
__global__ __launch_bounds__(256) void conv_first8_kernel(ConvArgs a) {
  constexpr int TW = kConvTileW, XW = TW + 2, XH = 18;
  constexpr int XQ = (XH * XW + 255) / 256;
  static_assert(TW == 32, "two 16-pixel blocks per tile row");
  __shared__ uint16_t sx[XH * XW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int n = a.n_tiles, xcd = blockIdx.x & 7, q8 = n >> 3, rem = n & 7;
  const int cnt = q8 + (xcd < rem ? 1 : 0), base = xcd * q8 + (xcd < rem ? xcd : rem);
  const int step = gridDim.x >> 3;
  int i = blockIdx.x >> 3;
  if (i >= cnt) return;                          // uniform over the workgroup
  // A fragments (rows: 16 channels of block mb; K slot 4g + e: tap (g, e)),
  // scale and bias of this lane's 4 channels per block
  i16x4 A0[4];
  f32x4 sc[4], bi[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      A0[mb][e] = __builtin_bit_cast(
          short, f32_to_bf16(g < 3 && e < 3 ? a.first_w[(16 * mb + l16) * 9 + 3 * g + e] : 0.0f));
      const int c = 16 * mb + 4 * g + e;
      sc[mb][e] = a.first_oscale[c] * a.first_out_inv_scale;
      bi[mb][e] = a.first_bias[c] * a.first_out_inv_scale;
    }
  }
  // the x window of tile t into registers (rows past the tile read its first row)
  float xv[XQ];
  auto load_x = [&](int t) {
    const PNP_CONST TileRef &tl = cp(a.tiles)[t];
    const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
    const PNP_GLOBAL float *xb = gp(j.x[(a.tick + j.t_offset) & 1]);
    const int B = j.xborder;
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int q0 = tid + 256 * k, q = q0 < XH * XW ? q0 : 0;
      const int r = q / XW, c = q % XW;
      const int rr = r < tl.h + 2 ? r : 0;
      xv[k] = xb[(int64_t)(tl.y0 - 1 + rr + B) * j.xpitch + (tl.x0 - 1 + c + B)];
    }
  };
  const int gr = g < 3 ? g : 2;                  // lane group 3 reads a valid row (zero weights)
  int t = base + i;
  load_x(t);
  for (;;) {
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int q = tid + 256 * k;
      if (q < XH * XW) sx[q] = f32_to_bf16(xv[k]);
    }
    __syncthreads();                             // window in place
    const int inext = i + step;
    if (inext < cnt) load_x(base + inext);       // uniform
    const PNP_CONST TileRef &tl = cp(a.tiles)[t];
    const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
    PNP_GLOBAL uint8_t *out = gp(reinterpret_cast<uint8_t *>(j.act[a.out_slot]));
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int r = 4 * wave + o;
      if (r >= tl.h) break;                        // uniform
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint16_t *xp = sx + (r + gr) * XW + 16 * h + l16;
        i16x4 Bx;
        Bx[0] = (short)xp[0];
        Bx[1] = (short)xp[1];
        Bx[2] = (short)xp[2];
        Bx[3] = 0;
        uint32_t v[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0[mb], Bx, f32x4{0.f, 0.f, 0.f, 0.f},
                                                                  0, 0, 0);
          v[mb] = pack_e4m3x4_relu(fmaf(d[0], sc[mb][0], bi[mb][0]), fmaf(d[1], sc[mb][1], bi[mb][1]),
                                   fmaf(d[2], sc[mb][2], bi[mb][2]), fmaf(d[3], sc[mb][3], bi[mb][3]));
        }
        const auto s02 = __builtin_amdgcn_permlane32_swap(v[0], v[2], false, false);
        const auto s13 = __builtin_amdgcn_permlane32_swap(v[1], v[3], false, false);
        const auto t01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
        const auto t23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
        const int c = 16 * h + l16;
        if (c < tl.w) {
          PNP_GLOBAL uint8_t *dst =
              out + ((int64_t)(tl.y0 + r + 1) * j.apitch + (tl.x0 + c + 1)) * 64 + 16 * g;
          *reinterpret_cast<PNP_GLOBAL u32x4 *>(dst) = u32x4{t01[0], t01[1], t23[0], t23[1]};
        }
      }
    }
    if (inext >= cnt) break;                     // uniform
    __syncthreads();                             // window read before it is replaced
    i = inext;
    t = base + i;
  }
}

hipError_t launch_conv_first8(const ConvArgs &a, int n_wg, hipStream_t s) {
  if (a.tile_rows < 1 || a.tile_rows > 16 || n_wg < 8 || n_wg % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(conv_first8_kernel, dim3(n_wg), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Last layer: F -> 1 (no activation); writes G (FP32, compact).  Every pixel
// of the tile's input window is read from memory once: a lane owns one
// 16-byte chunk of its channels (those channels' weights for all 9 taps in
// registers) and forms 9 per-tap partial dot products.  The lanes of a pixel
// combine them with a reduce-scatter of cross-lane exchanges, so each lane
// ends with whole sums for a subset of taps, and park them in LDS.  An output
// pixel is then the sum over taps of its neighbours' parked values.
// ---------------------------------------------------------------------
template <int FMT> __device__ __forceinline__ void decode16(u32x4 raw, float *v);
template <> __device__ __forceinline__ void decode16<FMT_F32>(u32x4 raw, float *v) {
  v[0] = __uint_as_float(raw.x); v[1] = __uint_as_float(raw.y);
  v[2] = __uint_as_float(raw.z); v[3] = __uint_as_float(raw.w);
}
template <> __device__ __forceinline__ void decode16<FMT_BF16>(u32x4 raw, float *v) {
  const uint32_t u[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[2 * e] = __uint_as_float(u[e] << 16);
    v[2 * e + 1] = __uint_as_float(u[e] & 0xffff0000u);
  }
}
template <> __device__ __forceinline__ void decode16<FMT_E4M3>(u32x4 raw, float *v) {
  const uint32_t u[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[4 * e + k] = e4m3_to_f32((uint8_t)(u[e] >> (8 * k)));
}

template <int IN_FMT, int F>
__global__ __launch_bounds__(256) void conv_last_kernel(ConvArgs a) {
  constexpr int IB = FmtInfo<IN_FMT>::bytes;
  constexpr int PIXB = F * IB;
  constexpr int NCH = PIXB / 16;               // lanes per pixel (power of two, <= 64)
  constexpr int EPC = 16 / IB;                 // channels per lane
  constexpr int IW = kConvTileW + 2, IHM = 18; // largest window (16-row tiles)
  static_assert((NCH & (NCH - 1)) == 0 && NCH <= 64 && 256 % NCH == 0, "lanes per pixel");
  __shared__ float sp[9][IHM * IW];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const PNP_GLOBAL uint8_t *in = gp(reinterpret_cast<const uint8_t *>(j.act[a.in_slot]));
  const int ch = threadIdx.x % NCH;
  float w[EPC][9];
#pragma unroll
  for (int e = 0; e < EPC; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) w[e][k] = a.wf32[(ch * EPC + e) * 9 + k];
  const int IH = tl.h + 2, WW = tl.w + 2, NQ = IH * WW * NCH;
  const int64_t apitch = j.apitch;
  constexpr int U = 8;                         // loads in flight per thread
  for (int q0 = 0; q0 < NQ; q0 += 256 * U) {   // uniform trip count: all lanes exchange
    u32x4 raw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int qa = q0 + 256 * u + (int)threadIdx.x, q = qa < NQ ? qa : ch;
      const int pix = q / NCH, row = pix / WW, col = pix % WW;
      raw[u] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          in + ((tl.y0 + row) * apitch + (tl.x0 + col)) * PIXB + ch * 16);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (q0 + 256 * u >= NQ) break;           // uniform
      const int q = q0 + 256 * u + (int)threadIdx.x;
      const bool ok = q < NQ;
      const int pix = q / NCH, row = pix / WW, col = pix % WW;
      float v[8], v8 = 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = 0.0f;
      if (ok) {
        float xv[EPC];
        decode16<IN_FMT>(raw[u], xv);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = fmaf(w[e][k], xv[e], v[k]);
          v8 = fmaf(w[e][8], xv[e], v8);
        }
      }
      // reduce-scatter of taps 0..7 over the NCH lanes of the pixel; tap 8 is
      // all-reduced.  Afterwards this lane holds taps base .. base + n - 1.
      int n = 8, base = 0;
#pragma unroll
      for (int off = NCH / 2; off >= 1; off >>= 1) {
        if (n > 1) {
          const bool hi = (ch & off) != 0;
          n >>= 1;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (k < n) {
              const float keep = hi ? v[n + k] : v[k];
              const float send = hi ? v[k] : v[n + k];
              v[k] = keep + __shfl_xor(send, off);
            }
          }
          if (hi) base += n;
        } else {
          v[0] += __shfl_xor(v[0], off);
        }
        v8 += __shfl_xor(v8, off);
      }
      // with more than 8 lanes per pixel, groups of NCH/8 lanes share a tap
      constexpr int DUP = NCH > 8 ? NCH / 8 : 1;
      if (ok && (ch % DUP) == 0) {
        const int at = row * IW + col;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < n) sp[base + k][at] = v[k];
        if (ch == 0) sp[8][at] = v8;
      }
    }
  }
  __syncthreads();
  const float sc = a.oscale[0], bi = a.bias[0];
  const int npix = (int)tl.h * tl.w;
  for (int pix = threadIdx.x; pix < npix; pix += 256) {
    const int r = pix / tl.w, c = pix % tl.w;
    float acc = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc += sp[tap][(r + tap / 3) * IW + c + tap % 3];
    gp(j.G)[(int64_t)(tl.y0 + r) * j.nx + tl.x0 + c] = acc * sc + bi;
  }
}

// Last layer for bf16 input on the matrix cores: the per-tap partial dot
// products s_tap(p) = sum_c w[c][tap] in[p][c] of every window pixel p are
// one small GEMM (M = 9 taps padded to 16, K = F channels, N = pixels), read
// straight from memory into B fragments: lane (g, l16) of a 16-pixel block
// holds channels 8g..8g+7 (+32 per K step) of pixel l16.  The 9 useful rows
// of each result block are parked in LDS and summed over the taps as in the
// VALU form above.
template <int F>
__global__ __launch_bounds__(256) void conv_last_mfma_kernel(ConvArgs a) {
  constexpr int PIXB = F * 2, KS = F / 32;     // bytes per pixel, K steps
  constexpr int IW = kConvTileW + 2, IHM = 18, NPIX = IHM * IW;
  constexpr int NB = (NPIX + 15) / 16, BPW = (NB + 3) / 4;   // blocks, blocks per wave
  __shared__ float sp[9][NPIX];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const PNP_GLOBAL uint8_t *in = gp(reinterpret_cast<const uint8_t *>(j.act[a.in_slot]));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int WW = tl.w + 2, np = (tl.h + 2) * WW;
  const int64_t apitch = j.apitch;
  // every load of this wave first (out-of-window lanes read pixel 0)
  u32x4 raw[BPW][KS];
#pragma unroll
  for (int u = 0; u < BPW; ++u) {
    const int q0 = (wave + 4 * u) * 16 + l16, q = q0 < np ? q0 : 0;
    const int row = q / WW, col = q % WW;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      raw[u][ks] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          in + ((tl.y0 + row) * apitch + (tl.x0 + col)) * PIXB + (ks * 4 + g) * 16);
  }
  // A fragments: row l16 = tap (zero past 8), channels 32 ks + 8 g .. +7
  bf16x8 A[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      A[ks][e] = (__bf16)(l16 < 9 ? a.wf32[(32 * ks + 8 * g + e) * 9 + l16] : 0.0f);
#pragma unroll
  for (int u = 0; u < BPW; ++u) {
    const int blk = wave + 4 * u;
    if (blk * 16 >= np) break;                 // uniform
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks], __builtin_bit_cast(bf16x8, raw[u][ks]),
                                                    acc, 0, 0, 0);
    const int q = blk * 16 + l16;
    if (q < np) {
      // this lane holds taps 4g .. 4g+3 of pixel q
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * g + i < 9) sp[4 * g + i][(q / WW) * IW + q % WW] = acc[i];
    }
  }
  __syncthreads();
  const float sc = a.oscale[0], bi = a.bias[0];
  const int npix = tl.h * tl.w;
  for (int pix = tid; pix < npix; pix += 256) {
    const int r = pix / tl.w, c = pix % tl.w;
    float acc = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc += sp[tap][(r + tap / 3) * IW + c + tap % 3];
    gp(j.G)[(int64_t)(tl.y0 + r) * j.nx + tl.x0 + c] = acc * sc + bi;
  }
}

// single 1 -> 1 layer (K = 1): reads x^(t) (FP32), writes G
__global__ __launch_bounds__(256) void conv_single_kernel(ConvArgs a) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const PNP_GLOBAL float *xb = gp(j.x[t & 1]);
  const int npix = (int)tl.h * tl.w;
  for (int pix = threadIdx.x; pix < npix; pix += blockDim.x) {
    const int r = pix / tl.w, c = pix % tl.w;
    const int Y = tl.y0 + r, X = tl.x0 + c;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int dy = k / 3, dx = k % 3;
      acc = fmaf(a.wf32[k],
                 xb[(int64_t)(Y + dy - 1 + j.xborder) * j.xpitch + (X + dx - 1 + j.xborder)],
                 acc);
    }
    gp(j.G)[(int64_t)Y * j.nx + X] = acc * a.oscale[0] + a.bias[0];
  }
}

// ---------------------------------------------------------------------
// Middle layers: F -> F on MFMA.
// ---------------------------------------------------------------------
// What a persistent conv kernel needs of one tile, held in registers.
// Output lanes of a partial tile store to a trash pixel (last slack row and
// column of the activation buffer, which no kernel reads), so every tile
// issues the same stores: the memory counters the compiler waits on then
// count exactly, and no wait for a tile's loads includes its stores.
struct MidTile {
  int y0, x0, h, w;
  int64_t apitch, trash;      // pixels per row; pixel index of the trash pixel
  const PNP_GLOBAL uint8_t *in;
  PNP_GLOBAL uint8_t *out;
  // fused first layer: x^(t) (padded, zero border xb), and the image size
  const PNP_GLOBAL float *x;
  int64_t xpitch;
  int xb, ny, nx;
  // fused last layer: per-tap partial records (12 floats, zero border 1)
  PNP_GLOBAL float *S;
};
__device__ __forceinline__ MidTile mid_tile(const ConvArgs &a, int ti) {
  const PNP_CONST TileRef &tl = cp(a.tiles)[ti];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  MidTile c;
  c.y0 = tl.y0;
  c.x0 = tl.x0;
  c.h = tl.h;
  c.w = tl.w;
  c.apitch = j.apitch;
  c.trash = (int64_t)j.arows * j.apitch - 1;
  c.in = gp(reinterpret_cast<const uint8_t *>(j.act[a.in_slot]));
  c.out = gp(reinterpret_cast<uint8_t *>(j.act[a.out_slot]));
  c.x = gp(j.x[(a.tick + j.t_offset) & 1]);
  c.xpitch = j.xpitch;
  c.xb = j.xborder;
  c.ny = j.ny;
  c.nx = j.nx;
  c.S = gp(j.S);
  return c;
}

template <int IN_FMT, int F>
struct MidCfg {
  static constexpr int IB = FmtInfo<IN_FMT>::bytes;
  static constexpr int PIXB = F * IB;            // bytes of one input pixel
  static constexpr int PSTR = PIXB + 16;         // LDS pixel stride (bank spread)
  static constexpr int CPP = PIXB / 16;          // 16-byte chunks per pixel
  static constexpr int MB = F / 16;              // 16-channel output blocks
  static constexpr int NSTEP = IN_FMT == FMT_E4M3 ? 5 : 9 * (IN_FMT == FMT_F32 ? F / 16 : F / 32);
  static constexpr int FRAGB = IN_FMT == FMT_E4M3 ? 32 : 16;   // A bytes per lane
  static constexpr int NCH = (IN_FMT == FMT_F32 && F == 64) ? 3 : 1;  // weight chunks
  static constexpr int STEPS_PER_CH = NSTEP / NCH;
  static constexpr int WBYTES = STEPS_PER_CH * MB * 64 * FRAGB;
};

template <int IN_FMT, int OUT_FMT, int F, int NW>
struct MidLayout {
  using C = MidCfg<IN_FMT, F>;
  static constexpr int TH = 2 * NW, TW = kConvTileW;
  static constexpr int IH = TH + 2, IW = TW + 2;
  static constexpr int OB = FmtInfo<OUT_FMT>::bytes;
  static constexpr int OPIXB = F * OB;               // bytes of one output pixel
  static constexpr int OSTR = OPIXB + 16;            // LDS stride of staged outputs
  static constexpr int IN_BYTES = IH * IW * C::PSTR;
  static constexpr int OUT_BYTES = TH * TW * OSTR;
  static constexpr int TILE_BYTES = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
  static constexpr int LDS_BYTES = TILE_BYTES + C::WBYTES + 2 * F * 4;   // + scale, bias
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <int IN_FMT, int OUT_FMT, int F, int NW>
__global__ __launch_bounds__(NW * 64) void conv_mid_kernel(ConvArgs a) {
  using C = MidCfg<IN_FMT, F>;
  using Lo = MidLayout<IN_FMT, OUT_FMT, F, NW>;
  constexpr int TH = Lo::TH, IW = Lo::IW;
  constexpr int NT = NW * 64;
  constexpr int NCHUNK = Lo::IH * IW * C::CPP;
  constexpr int NLOAD = (NCHUNK + NT - 1) / NT;
  constexpr int OB = Lo::OB;
  constexpr int MB = C::MB;
  // fragment types and per-step operand counts
  using AT = typename std::conditional<IN_FMT == FMT_BF16, bf16x8,
             typename std::conditional<IN_FMT == FMT_F32, f32x4, i32x8>::type>::type;

  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;                 // input tile, then staged output tile
  uint8_t *lds_w = lds + Lo::TILE_BYTES;
  float *lds_osc = reinterpret_cast<float *>(lds_w + C::WBYTES);
  float *lds_bias = lds_osc + F;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;

  // contiguous tile ranges per XCD (workgroups are dispatched round-robin
  // over the 8 XCDs): neighbouring tiles share their halo rows in one L2
  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  auto load_weights = [&](int chunk) {
    const PNP_GLOBAL u32x4 *src = gp(reinterpret_cast<const u32x4 *>(
        reinterpret_cast<const uint8_t *>(a.wblob) + (size_t)chunk * C::WBYTES));
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_w);
    for (int i = tid; i < C::WBYTES / 16; i += NT) dst[i] = src[i];
  };
  for (int i = tid; i < F; i += NT) {
    lds_osc[i] = gp(a.oscale)[i];
    lds_bias[i] = gp(a.bias)[i];
  }

  u32x4 pre[NLOAD];
  auto issue_loads = [&](const MidTile &tl) {
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q0 = tid + i * NT, q = q0 < NCHUNK ? q0 : 0;
      const int pix = q / C::CPP, c = q % C::CPP;
      const int row = pix / IW, col = pix % IW;
      pre[i] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          tl.in + ((int64_t)(tl.y0 + row) * tl.apitch + (tl.x0 + col)) * C::PIXB + c * 16);
    }
  };
  auto store_lds = [&]() {
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q = tid + i * NT;
      if (q < NCHUNK) {
        const int pix = q / C::CPP, c = q % C::CPP;
        *reinterpret_cast<u32x4 *>(lds_in + pix * C::PSTR + c * 16) = pre[i];
      }
    }
  };

  // pixel of N block nb for this lane, relative to the input tile origin
  auto in_pix = [&](int nb, int tap) {
    const int dy = tap / 3, dx = tap % 3;
    return (2 * wave + (nb >> 1) + dy) * IW + (nb & 1) * 16 + l16 + dx;
  };
  // operands of K step `sl` (index within the LDS-resident weight chunk)
  auto load_step = [&](int step, int sl, AT (&A)[MB], AT (&B)[4]) {
    const uint8_t *wf = lds_w + (size_t)sl * MB * 64 * C::FRAGB + lane * C::FRAGB;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      A[mb] = *reinterpret_cast<const AT *>(wf + mb * 64 * C::FRAGB);
    if constexpr (IN_FMT == FMT_BF16) {
      const int tap = step / (F / 32), half = step % (F / 32);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        B[nb] = *reinterpret_cast<const bf16x8 *>(lds_in + in_pix(nb, tap) * C::PSTR +
                                                   (half * 4 + g) * 16);
    } else if constexpr (IN_FMT == FMT_F32) {
      const int tap = step / (F / 16), ss = step % (F / 16);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        B[nb] = *reinterpret_cast<const f32x4 *>(lds_in + in_pix(nb, tap) * C::PSTR +
                                                  (ss * 4 + g) * 16);
    } else {  // e4m3: taps 2*step (lane groups 0,1) and 2*step+1 (2,3); slot 9 -> tap 8
      const int tap_raw = 2 * step + (g >> 1);
      const int tap = tap_raw > 8 ? 8 : tap_raw;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const uint8_t *src = lds_in + in_pix(nb, tap) * C::PSTR + (g & 1) * 32;
        const u32x4 lo = *reinterpret_cast<const u32x4 *>(src);
        const u32x4 hi = *reinterpret_cast<const u32x4 *>(src + 16);
        B[nb] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
    }
  };
  auto mma_step = [&](const AT (&A)[MB], const AT (&B)[4], f32x4 (&acc)[MB][4]) {
    if constexpr (IN_FMT == FMT_BF16) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mb], B[nb], acc[mb][nb], 0, 0, 0);
    } else if constexpr (IN_FMT == FMT_F32) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < 4; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mb][e], B[nb][e], acc[mb][nb],
                                                               0, 0, 0);
    } else {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              A[mb], B[nb], acc[mb][nb], 0, 0, 0, 0, 0, 0);
    }
  };

  if (C::NCH == 1) load_weights(0);
  // tile descriptors run two tiles ahead of the tile being computed, so no
  // load issued after a tile's output stores is waited on before the next
  // tile's stores (loads and stores share one completion counter)
  int ti = t_begin + slot;
  MidTile tl = mid_tile(a, ti < t_end ? ti : t_begin);
  MidTile nxt = mid_tile(a, ti + per_xcd < t_end ? ti + per_xcd : t_begin);
  if (ti < t_end) issue_loads(tl);

  while (ti < t_end) {
    __syncthreads();          // previous tile's output staging has been read
    store_lds();
    __syncthreads();
    const int tn = ti + per_xcd, tnn = tn + per_xcd;
    if (tn < t_end) issue_loads(nxt);  // overlaps with the MFMA work below
    const MidTile after = mid_tile(a, tnn < t_end ? tnn : t_begin);

    f32x4 acc[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll 1
    for (int ch = 0; ch < C::NCH; ++ch) {
      if (C::NCH > 1) {
        __syncthreads();
        load_weights(ch);
        __syncthreads();
      }
      // two-stage register pipeline: the next step's LDS reads are issued
      // before the current step's MFMAs
      AT A0[MB], B0[4], A1[MB], B1[4];
      load_step(ch * C::STEPS_PER_CH, 0, A0, B0);
#pragma unroll 1
      for (int sl = 0; sl < C::STEPS_PER_CH; sl += 2) {
        const int step = ch * C::STEPS_PER_CH + sl;
        if (sl + 1 < C::STEPS_PER_CH) load_step(step + 1, sl + 1, A1, B1);
        mma_step(A0, B0, acc);
        if (sl + 1 < C::STEPS_PER_CH) {
          if (sl + 2 < C::STEPS_PER_CH) load_step(step + 2, sl + 2, A0, B0);
          mma_step(A1, B1, acc);
        }
      }
    }

    // epilogue: scale, bias, ReLU, round to the next layer's format, stage
    // the tile in LDS (over the consumed input tile), then store whole
    // pixels with 16-byte lanes
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int r = 2 * wave + (nb >> 1), c = (nb & 1) * 16 + l16;
      uint8_t *dst = lds_in + (r * kConvTileW + c) * Lo::OSTR;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        // 4 consecutive output channels of this lane
        const f32x4 osc = *reinterpret_cast<const f32x4 *>(lds_osc + mb * 16 + 4 * g);
        const f32x4 bia = *reinterpret_cast<const f32x4 *>(lds_bias + mb * 16 + 4 * g);
        f32x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float o = acc[mb][nb][e] * osc[e] + bia[e];
          if (a.relu) o = fmaxf(o, 0.0f);
          v[e] = o;
        }
        store4<OUT_FMT>(dst + (mb * 16 + 4 * g) * OB, v, a.out_inv_scale);
      }
    }
    __syncthreads();
    {
      PNP_GLOBAL uint8_t *out = tl.out;
      constexpr int CPPO = Lo::OPIXB / 16;
      constexpr int NQ = TH * kConvTileW * CPPO;
#pragma unroll
      for (int q0 = 0; q0 < NQ; q0 += NT) {
        const int q = q0 + tid;
        const int pix = q / CPPO, c16 = q % CPPO;
        const int r = pix / kConvTileW, c = pix % kConvTileW;
        if (q < NQ) {
          const int64_t px = (r < tl.h && c < tl.w)
                                 ? (int64_t)(tl.y0 + r + 1) * tl.apitch + (tl.x0 + c + 1)
                                 : tl.trash;
          *reinterpret_cast<PNP_GLOBAL u32x4 *>(out + px * Lo::OPIXB + c16 * 16) =
              *reinterpret_cast<const u32x4 *>(lds_in + pix * Lo::OSTR + c16 * 16);
        }
      }
    }
    tl = nxt;
    nxt = after;
    ti = tn;
  }
}

// ---------------------------------------------------------------------
// Middle layers, row-reuse form (bf16 in and out, F = 64).  One persistent
// workgroup of 4 waves per CU, one wave per SIMD; the layer's weights stay in
// LDS in fragment order and the 16 x 32 tile's (18 x 34)-pixel input window
// is staged beside them.  Wave w owns output rows 4w..4w+3 (all 32 columns,
// all 64 channels: 32 accumulator blocks).  For one horizontal tap dx and one
// 32-channel half kh of the input, the B fragment of input row ir serves the
// three vertical taps dy (output row ir - dy), so every B fragment is read
// from LDS once per (dx, kh) instead of once per tap: half the LDS traffic
// of the two-rows-per-wave form.
// ---------------------------------------------------------------------
struct RrLayout {
  static constexpr int F = 64, MB = 4, PIXB = 128, CPP = 8;
  static constexpr int TH = 16, TW = kConvTileW, IH = TH + 2, IW = TW + 2;
  static constexpr int ROWS = 4;                              // output rows per wave
  static constexpr int NSTEP = 18;                            // 9 taps x 2 channel halves
  static constexpr int WBYTES = NSTEP * MB * 64 * 16;
  static constexpr int IN_BYTES = IH * IW * PIXB;
  static constexpr int OUT_BYTES = TH * TW * PIXB;
  static constexpr int TILE_BYTES = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
  static constexpr int EPI_BYTES = F * 4;                     // bias
  // fused first layer: x window (TH+4) x (TW+4) as bf16, and its bias
  static constexpr int XH = TH + 4, XW = TW + 4, XBYTES = XH * XW * 2;
  static constexpr int LDS_BYTES = TILE_BYTES + WBYTES + EPI_BYTES;
  static constexpr int A0BYTES = MB * 64 * 16;                // first-layer A fragments
  static constexpr int FIRST_BYTES = XBYTES + F * 4 + A0BYTES;
  static constexpr int ALBYTES = 2 * 64 * 16;                  // last-layer A fragments
  static constexpr int lds_bytes(bool first, bool last) {
    return LDS_BYTES + (first ? FIRST_BYTES : 0) + (last ? ALBYTES : 0);
  }
};
static_assert(RrLayout::lds_bytes(true, true) <= 160 * 1024, "LDS");
// LDS byte offset of 16-byte chunk k of pixel p: pixels are 128 bytes with no
// padding and the chunks of a pixel are permuted by the pixel's low 3 bits,
// so 8 lanes reading the same chunk of 8 consecutive pixels hit 8 different
// bank groups (a padded stride conflicts two ways at full LDS rate).
__device__ __forceinline__ int rr_off(int p, int k) { return p * 128 + ((k ^ (p & 7)) << 4); }

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void conv_mid_rr_kernel(ConvArgs a) {
  using Lo = RrLayout;
  constexpr int NT = 256, MB = Lo::MB, IW = Lo::IW, ROWS = Lo::ROWS;
  constexpr int NCHUNK = Lo::IH * IW * Lo::CPP;
  constexpr int NLOAD = (NCHUNK + NT - 1) / NT;

  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_w = lds + Lo::TILE_BYTES;
  float *lds_bias = reinterpret_cast<float *>(lds_w + Lo::WBYTES);
  uint16_t *lds_x = reinterpret_cast<uint16_t *>(lds_bias + Lo::F);     // FIRST only
  float *lds_bias0 = reinterpret_cast<float *>(lds_x + Lo::XH * Lo::XW);  // FIRST only
  uint8_t *lds_a0 = reinterpret_cast<uint8_t *>(lds_bias0 + Lo::F);        // FIRST only
  uint8_t *lds_al = lds + Lo::LDS_BYTES + (FIRST ? Lo::FIRST_BYTES : 0);  // LAST only
  constexpr int NX = Lo::XH * Lo::XW, XQ = (NX + NT - 1) / NT;
  constexpr int NWIN = Lo::IH * IW, NB0 = (NWIN + 15) / 16, BPW0 = (NB0 + 3) / 4;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;

  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  {
    const PNP_GLOBAL u32x4 *src = gp(reinterpret_cast<const u32x4 *>(a.wblob));
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_w);
    for (int i = tid; i < Lo::WBYTES / 16; i += NT) dst[i] = src[i];
    if (tid < Lo::F) lds_bias[tid] = gp(a.bias)[tid];
    if (FIRST && tid < Lo::F) lds_bias0[tid] = gp(a.first_bias)[tid];
  }
  // fused first layer: A fragments (rows = its 64 output channels in blocks of
  // 16, K = its 9 taps padded to 16) in LDS, fragment order
  if constexpr (FIRST) {
    if (wave == 0) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        i16x4 f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = 4 * g + e;
          f[e] = __builtin_bit_cast(short, f32_to_bf16(t < 9 ? gp(a.first_w)[(mb * 16 + l16) * 9 + t]
                                                             : 0.0f));
        }
        *reinterpret_cast<i16x4 *>(lds_a0 + (mb * 64 + lane) * 16) = f;
      }
    }
  }

  u32x4 pre[FIRST ? 1 : NLOAD];
  float prex[FIRST ? XQ : 1];
  // load i of the next tile's window (one 16-byte chunk per lane); with the
  // fused last layer the empty asm keeps the compiler from hoisting 20
  // loop-invariant lane offsets into registers for the whole tile loop
  // (which would spill)
  auto issue_load = [&](const MidTile &c, int i) {
    int q0 = tid + i * NT;
    if constexpr (LAST) asm volatile("" : "+v"(q0));
    const int q = q0 < NCHUNK ? q0 : 0;
    const int pix = q / Lo::CPP, k = q % Lo::CPP;
    const int row = pix / IW, col = pix % IW;
    pre[i] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
        c.in + ((int64_t)(c.y0 + row) * c.apitch + (c.x0 + col)) * Lo::PIXB + k * 16);
  };
  auto issue_loads = [&](const MidTile &c) {
    if constexpr (FIRST) {
      // x window: image rows y0-2 .. y0+TH+1, columns x0-2 .. x0+TW+1
#pragma unroll
      for (int i = 0; i < XQ; ++i) {
        const int q0 = tid + i * NT, q = q0 < NX ? q0 : 0;
        const int xr = q / Lo::XW, xc = q % Lo::XW;
        prex[i] = c.x[(int64_t)(c.y0 - 2 + xr + c.xb) * c.xpitch + (c.x0 - 2 + xc + c.xb)];
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q0 = tid + i * NT, q = q0 < NCHUNK ? q0 : 0;
      const int pix = q / Lo::CPP, k = q % Lo::CPP;
      const int row = pix / IW, col = pix % IW;
      pre[i] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          c.in + ((int64_t)(c.y0 + row) * c.apitch + (c.x0 + col)) * Lo::PIXB + k * 16);
    }
  };

  // branch-free: lanes past the window loaded chunk 0 and store it there
  // again (the same bytes the lane that owns chunk 0 stores)
  auto store_lds = [&]() {
    if constexpr (FIRST) {
#pragma unroll
      for (int i = 0; i < XQ; ++i) {
        const int q0 = tid + i * NT, q = q0 < NX ? q0 : 0;
        lds_x[q] = f32_to_bf16(prex[i]);
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q0 = tid + i * NT, q = q0 < NCHUNK ? q0 : 0;
      *reinterpret_cast<u32x4 *>(lds_in + rr_off(q / Lo::CPP, q % Lo::CPP)) = pre[i];
    }
  };

  // fused last layer: A fragments (rows = the 9 taps padded to 16, K = the 64
  // input channels in two steps) in LDS, fragment order
  if constexpr (LAST) {
    if (wave == 1) {
#pragma unroll
      for (int kh = 0; kh < 2; ++kh) {
        bf16x8 f;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          f[e] = (__bf16)(l16 < 9 ? gp(a.last_w)[(32 * kh + 8 * g + e) * 9 + l16] : 0.0f);
        *reinterpret_cast<bf16x8 *>(lds_al + (kh * 64 + lane) * 16) = f;
      }
    }
  }

  // Fused first layer on the staged x window: the 64-channel output of every
  // window pixel (an MFMA per 16-pixel block and 16 channels; K = the 9 taps),
  // + bias, ReLU, bf16, written into the layer input window; window pixels
  // outside the image are the next layer's zero padding.
  auto layer0 = [&](const MidTile &c) {
    // the A fragments and biases of the four channel blocks, read once per
    // tile (the window stores below would otherwise make the compiler read
    // them again for every block)
    i16x4 A0s[MB];
    f32x4 bias_s[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      bias_s[mb] = *reinterpret_cast<const f32x4 *>(lds_bias0 + mb * 16 + 4 * g);
      A0s[mb] = *reinterpret_cast<const i16x4 *>(lds_a0 + (mb * 64 + lane) * 16);
    }
#pragma unroll
    for (int u = 0; u < BPW0; ++u) {
      const int blk = wave + 4 * u;
      if (blk >= NB0) break;                                  // uniform
      const int q0 = blk * 16 + l16, q = q0 < NWIN ? q0 : 0;
      const int wr = q / IW, wc = q % IW;
      i16x4 Bx;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int t = 4 * g + e;
        const int tt = t < 9 ? t : 0;
        const uint16_t v = lds_x[(wr + tt / 3) * Lo::XW + wc + tt % 3];
        Bx[e] = (short)(t < 9 ? v : (uint16_t)0);
      }
      const int Y = c.y0 - 1 + wr, X = c.x0 - 1 + wc;
      const bool inside = Y >= 0 && Y < c.ny && X >= 0 && X < c.nx;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0s[mb], Bx, bias_s[mb], 0, 0, 0);
        u32x2 w;
        w.x = inside ? relu_bf16x2(pack_bf16x2(d[0], d[1])) : 0u;
        w.y = inside ? relu_bf16x2(pack_bf16x2(d[2], d[3])) : 0u;
        if (q0 < NWIN)
          *reinterpret_cast<u32x2 *>(lds_in + rr_off(q, 2 * mb + (g >> 1)) + 8 * (g & 1)) = w;
      }
    }
  };

  // Every iteration issues the same memory operations in the same order:
  // the next tile's loads (a real tile's, or any valid tile's on the last
  // iteration), the MFMAs, this tile's stores, then the LDS copy of the
  // loads.  The copy therefore waits for the loads only, never for the
  // stores (loads and stores share one in-order completion counter).  Tile
  // descriptors are read two tiles ahead, as scalar loads.
  int ti = t_begin + slot;
  if (ti >= t_end) return;                       // uniform over the workgroup
  MidTile cur = mid_tile(a, ti);
  MidTile nxt = mid_tile(a, ti + per_xcd < t_end ? ti + per_xcd : t_begin);
  issue_loads(cur);
  store_lds();
  __syncthreads();
  if constexpr (FIRST) {
    layer0(cur);
    __syncthreads();
  }

  while (true) {
    const int tn = ti + per_xcd, tnn = tn + per_xcd;
    // the next tile's loads are issued a few per pipeline stage below (all at
    // once, they would wait behind this tile's predecessor's stores in the
    // memory pipeline and hold up the first MFMAs)
    if constexpr (FIRST) issue_loads(nxt);
    const MidTile after = mid_tile(a, tnn < t_end ? tnn : t_begin);
    __builtin_amdgcn_sched_barrier(0);

    // accumulators start at the bias (this kernel runs layers whose output
    // scale is 1 and that end in ReLU)
    f32x4 acc[MB][ROWS][2];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const f32x4 bia = *reinterpret_cast<const f32x4 *>(lds_bias + mb * 16 + 4 * g);
#pragma unroll
      for (int o = 0; o < ROWS; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[mb][o][h] = bia;
    }

    // this lane's B column inside the window: pixel (ROWS*wave + ir, 16h + dx + l16)
    const int bpix = (ROWS * wave) * IW + l16;
    const uint8_t *abase = lds_w + lane * 16;
    // Software pipeline over 36 stages (6 (dx, kh) iterations x 6 input
    // rows): the B fragments of the stage PD ahead and the next iteration's
    // A fragments are read from LDS while this stage's MFMAs run.
    // Scheduling barriers keep each stage's reads ahead of its MFMAs.
    constexpr int NIT = 6, NR = ROWS + 2, NSTG = NIT * NR, PD = 3;
    bf16x8 Ab[2][3][MB], Bb[PD + 1][2];
    auto load_a = [&](int it, int dy) {
      const int dx = it >> 1, kh = it & 1;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        Ab[it & 1][dy][mb] = *reinterpret_cast<const bf16x8 *>(
            abase + (((3 * dy + dx) * 2 + kh) * MB + mb) * 1024);
    };
    auto load_b = [&](int stg) {
      const int it = stg / NR, ir = stg % NR, dx = it >> 1, kh = it & 1;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        Bb[stg % (PD + 1)][h] = *reinterpret_cast<const bf16x8 *>(
            lds_in + rr_off(bpix + ir * IW + 16 * h + dx, kh * 4 + g));
    };
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) load_a(0, dy);
#pragma unroll
    for (int k = 0; k < PD; ++k) load_b(k);
#pragma unroll
    for (int stg = 0; stg < NSTG; ++stg) {
      const int it = stg / NR, ir = stg % NR;
      if (stg + PD < NSTG) load_b(stg + PD);
      if (it + 1 < NIT && ir >= 2 && ir <= 4) load_a(it + 1, ir - 2);
      if constexpr (!FIRST) {
        constexpr int LPS = 1;                  // global loads per stage
#pragma unroll
        for (int i = stg * LPS; i < (stg + 1) * LPS; ++i)
          if (i < NLOAD) issue_load(nxt, i);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int o = ir - dy;
        if (o < 0 || o >= ROWS) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[mb][o][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                Ab[it & 1][dy][mb], Bb[stg % (PD + 1)][h], acc[mb][o][h], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }

    // epilogue: round to bf16, ReLU on the rounded pairs (as signed 16-bit
    // integers: a negative bf16 is a negative int16), stage the tile over the
    // consumed input window, then store whole pixels with 16-byte lanes
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int o = 0; o < ROWS; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4 v = acc[mb][o][h];
          u32x2 w;
          w.x = relu_bf16x2(pack_bf16x2(v[0], v[1]));
          w.y = relu_bf16x2(pack_bf16x2(v[2], v[3]));
          const int p = (ROWS * wave + o) * Lo::TW + 16 * h + l16;
          // channels mb*16 + 4g .. +3: chunk 2mb + g/2, bytes 8(g&1) .. +7
          *reinterpret_cast<u32x2 *>(lds_in + rr_off(p, 2 * mb + (g >> 1)) + 8 * (g & 1)) = w;
        }
    __syncthreads();
    if constexpr (LAST) {
      // the last layer's per-tap partials of every pixel of the tile, from the
      // staged (bf16, ReLU) outputs: one record of 12 floats per pixel (taps
      // 9..11 have zero weights), written with one 16-byte store per lane of
      // lane groups 0-2
      const bf16x8 AL0 = *reinterpret_cast<const bf16x8 *>(lds_al + lane * 16);
      const bf16x8 AL1 = *reinterpret_cast<const bf16x8 *>(lds_al + (64 + lane) * 16);
      const int64_t spitch = cur.nx + 2, strash = (int64_t)(cur.ny + 2) * spitch;
#pragma unroll
      for (int o = 0; o < ROWS; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = ROWS * wave + o, c = 16 * h + l16, p = r * Lo::TW + c;
          const bf16x8 B0 = *reinterpret_cast<const bf16x8 *>(lds_in + rr_off(p, g));
          const bf16x8 B1 = *reinterpret_cast<const bf16x8 *>(lds_in + rr_off(p, 4 + g));
          f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL0, B0, f32x4{0.f, 0.f, 0.f, 0.f},
                                                            0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL1, B1, d, 0, 0, 0);
          // this lane: taps 4g .. 4g+3 of pixel l16 of the block
          const int64_t rec = (r < cur.h && c < cur.w)
                                  ? (int64_t)(cur.y0 + r + 1) * spitch + (cur.x0 + c + 1)
                                  : strash;
          if (g < 3) *reinterpret_cast<PNP_GLOBAL f32x4 *>(cur.S + rec * 12 + 4 * g) = d;
        }
    } else {
      constexpr int NQ = Lo::TH * Lo::TW * Lo::CPP, NS = NQ / NT;
      u32x4 st[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int q = i * NT + tid;
        st[i] = *reinterpret_cast<const u32x4 *>(lds_in + rr_off(q / Lo::CPP, q % Lo::CPP));
      }
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int q = i * NT + tid;
        const int pix = q / Lo::CPP, k = q % Lo::CPP;
        const int r = pix / Lo::TW, c = pix % Lo::TW;
        const int64_t px = (r < cur.h && c < cur.w)
                               ? (int64_t)(cur.y0 + r + 1) * cur.apitch + (cur.x0 + c + 1)
                               : cur.trash;
        *reinterpret_cast<PNP_GLOBAL u32x4 *>(cur.out + px * Lo::PIXB + k * 16) = st[i];
      }
    }
    __syncthreads();                             // staged outputs are read
    store_lds();
    __syncthreads();
    if constexpr (FIRST) {
      layer0(nxt);
      __syncthreads();
    }
    if (tn >= t_end) break;
    cur = nxt;
    nxt = after;
    ti = tn;
  }
}

// calls fn(std::integral_constant<int, i>) for i = I .. N-1 in order (a loop
// unrolled by construction, whatever its body's size)
template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

// ---------------------------------------------------------------------
// Two bf16 middle layers per kernel with the layers on separate waves.
// Eight waves per workgroup: waves 0-3 run layer A of tile i (input window
// -> intermediate) while waves 4-7 run layer B of tile i-1 (intermediate ->
// memory); the intermediate is double-buffered in LDS.  Each wave keeps the
// A fragments of one layer only (72 VGPRs), so two waves share a SIMD and
// the epilogue, loads and barriers of one overlap the MFMAs of the other.
// Output tiles are 9 x 30 (input window 13 x 34, intermediate 11 x 32): the
// input window and two intermediates take 153 KB of LDS.  The layer-A waves
// also load the next tile's window (moving those loads to the layer-B waves,
// which have fewer MFMAs, spills registers).  Wave w & 3 owns output
// channels 16 (w & 3) .. + 15 of its layer and keeps their A fragments in
// registers for the whole kernel, so LDS holds activations only.
//
// Within a layer, work runs input row by input row: the B fragment of input
// row ir serves output rows ir, ir-1 and ir-2 (taps dy = 0, 1, 2), so output
// row o is complete after input row o + 2 and four accumulator row slots
// suffice.  The intermediate holds the tile plus a one-pixel ring (bf16,
// ReLU, and zero at positions outside the image, which is layer B's zero
// padding), computed from the input window; window positions beyond the
// one-pixel zero border of the activation buffer read the border.
// ---------------------------------------------------------------------
struct PairWsLayout {
  static constexpr int F = 64, PIXB = 128, CPP = 8, NSTEP = 18, NTG = 256;
  static constexpr int TH = kPairWsTileH, TW = kPairTileW;
  static constexpr int MH = TH + 2, MW = TW + 2, IH = TH + 4, IW = TW + 4;
  static constexpr int IN_BYTES = IH * IW * PIXB;
  static constexpr int MID_BYTES = MH * IW * PIXB;
  static constexpr int LDS_BYTES = IN_BYTES + 2 * MID_BYTES + 2 * F * 4;
  static constexpr int NLOAD = IH + 1;          // row loads + one load for columns 32, 33
};
static_assert(PairWsLayout::MW == 32 && PairWsLayout::IW == 34 &&
                  PairWsLayout::LDS_BYTES <= 160 * 1024,
              "split-layer pair layout");

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void conv_pair_ws_kernel(ConvArgs a) {
  using Lo = PairWsLayout;
  constexpr int IW = Lo::IW, NLOAD = Lo::NLOAD;
  constexpr int NIT = 6, PD = 1;                  // (dx, kh) steps per row; B reads ahead
                                                  // (one step: two measured 0.7% slower)
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_mid = lds + Lo::IN_BYTES;          // two buffers of MID_BYTES
  float *lds_bias = reinterpret_cast<float *>(lds_mid + 2 * Lo::MID_BYTES);   // [layer][64]

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2, wq = wave & 3;       // layer (0: A, 1: B), channel block
  const int g = lane >> 4, l16 = lane & 15;
  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  bf16x8 W[Lo::NSTEP];
  {
    const PNP_GLOBAL bf16x8 *wsrc = gp(reinterpret_cast<const bf16x8 *>(grp ? a.wblob2 : a.wblob));
#pragma unroll
    for (int s = 0; s < Lo::NSTEP; ++s) W[s] = wsrc[(s * 4 + wq) * 64 + lane];
  }
  if (tid < Lo::F) lds_bias[tid] = gp(a.bias)[tid];
  else if (tid < 2 * Lo::F) lds_bias[tid] = gp(a.bias2)[tid - Lo::F];
  // the intermediates' columns MW .. IW-1 are read only for the two padding
  // output columns and never written: zero both buffers once
  for (int i = tid; i < 2 * Lo::MID_BYTES / 16; i += 2 * Lo::NTG)
    reinterpret_cast<u32x4 *>(lds_mid)[i] = u32x4{0u, 0u, 0u, 0u};

  // Window loads by the layer-A waves (256 lanes), 16 bytes per lane: load r
  // < IH is window row r, lane (c = tid / 8, k = tid % 8) taking chunk k of
  // column c < 32; the last load takes the pixels of columns 32 and 33
  // (lanes past them repeat one, storing the bytes its owner stores).
  // Window pixel (r, c) is image pixel (y0 - 2 + r, x0 - 2 + c); positions
  // beyond the one-pixel zero border read the border.
  const int lc = (tid & 255) >> 3, lk = tid & 7;
  auto lane_col = [&](const MidTile &c) -> uint32_t {
    const int X = min(max(c.x0 - 2 + lc, -1), c.nx) + 1;
    return (uint32_t)X * Lo::PIXB + (uint32_t)lk * 16u;
  };
  constexpr int NEDGE = 2 * Lo::IH;               // pixels in columns 32 and 33
  auto load_chunk = [&](const MidTile &c, uint32_t lcol, auto ic) -> u32x4 {
    constexpr int i = decltype(ic)::value;
    if constexpr (i < Lo::IH) {
      const int Y = min(max(c.y0 - 2 + i, -1), c.ny) + 1;
      return *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          c.in + (int64_t)Y * c.apitch * Lo::PIXB + lcol);
    } else {
      const int e0 = (i - Lo::IH) * 32 + lc, e = e0 < NEDGE ? e0 : (lc & 15);
      const int Y = min(max(c.y0 - 2 + (e >> 1), -1), c.ny) + 1;
      const int X = min(max(c.x0 + 30 + (e & 1), -1), c.nx) + 1;
      return *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
          c.in + ((int64_t)Y * c.apitch + X) * Lo::PIXB + lk * 16);
    }
  };
  auto put_chunk = [&](auto ic, const u32x4 &v) {
    constexpr int i = decltype(ic)::value;
    if constexpr (i < Lo::IH) {
      const int off = (lc << 7) + ((lk ^ ((2 * (i & 3) + lc) & 7)) << 4);
      *reinterpret_cast<u32x4 *>(lds_in + i * IW * Lo::PIXB + off) = v;
    } else {
      const int e0 = (i - Lo::IH) * 32 + lc, e = e0 < NEDGE ? e0 : (lc & 15);
      *reinterpret_cast<u32x4 *>(lds_in + rr_off((e >> 1) * IW + 32 + (e & 1), lk)) = v;
    }
  };
  static_assert(NEDGE <= 32 && NEDGE >= 16, "edge loads");

  int tA = t_begin + slot;
  if (tA >= t_end) return;                       // uniform over the workgroup
  MidTile dA = mid_tile(a, tA), dB = dA;
  u32x4 pre[NLOAD];
  if (grp == 0) {
    const uint32_t lcol = lane_col(dA);
    static_for<0, NLOAD>([&](auto ic) { pre[decltype(ic)::value] = load_chunk(dA, lcol, ic); });
    static_for<0, NLOAD>([&](auto ic) { put_chunk(ic, pre[decltype(ic)::value]); });
  }
  // base[m][kh]: the lane's part of the swizzled address of chunk 4kh + g of
  // pixel c + l16 for c = m (mod 8)
  int bl[8][2];
#pragma unroll
  for (int m = 0; m < 8; ++m)
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      int v = 128 * l16 + (((4 * kh + g) ^ ((m + l16) & 7)) << 4);
      asm volatile("" : "+v"(v));
      bl[m][kh] = v;
    }
  __syncthreads();

  const int hb = g & 1, cpos = 16 * hb + l16;     // this lane's pixel after the swap
  bool haveB = false;
  int it = 0;
  while (true) {
    const bool haveA = tA < t_end;                // uniform
    const int tAn = tA + per_xcd;
    const MidTile dAn = mid_tile(a, tAn < t_end ? tAn : t_begin);
    f32x4 acc[4][2];
    bf16x8 Bb[PD + 1][2];

    auto layer = [&](const int (&base)[8][2], auto NRc, auto BIc, auto ep, auto pf) {
      constexpr int NR = decltype(NRc)::value, NO = NR - 2, NSTG = NR * NIT;
      constexpr int BI = decltype(BIc)::value;
      auto load_b = [&](auto stc) {
        constexpr int stg = decltype(stc)::value;
        constexpr int ir = stg / NIT, it2 = stg % NIT, dx = it2 >> 1, kh = it2 & 1;
        static_for<0, 2>([&](auto hc) {
          constexpr int c = ir * IW + 16 * decltype(hc)::value + dx;
          Bb[stg % (PD + 1)][decltype(hc)::value] =
              *reinterpret_cast<const bf16x8 *>(lds + base[c & 7][kh] + 128 * c);
        });
      };
      static_for<0, PD>(load_b);
      static_for<0, NSTG>([&](auto stc) {
        constexpr int stg = decltype(stc)::value;
        constexpr int ir = stg / NIT, it2 = stg % NIT, dx = it2 >> 1, kh = it2 & 1;
        if constexpr (stg + PD < NSTG) load_b(std::integral_constant<int, stg + PD>{});
        pf(stc);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (it2 == 0 && ir < NO) {
          const f32x4 bia = *reinterpret_cast<const f32x4 *>(lds_bias + BI * Lo::F + 16 * wq + 4 * g);
          acc[ir & 3][0] = bia;
          acc[ir & 3][1] = bia;
        }
        static_for<0, 3>([&](auto dyc) {
          constexpr int dy = decltype(dyc)::value, o = ir - dy;
          if constexpr (o >= 0 && o < NO) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
              acc[o & 3][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  W[(3 * dy + dx) * 2 + kh], Bb[stg % (PD + 1)][h], acc[o & 3][h], 0, 0, 0);
          }
        });
        if constexpr (it2 == 1 && ir >= 3 && ir - 3 < NO) ep(std::integral_constant<int, ir - 3>{});
        __builtin_amdgcn_sched_barrier(0);
      });
      static_for<(NR - 3 > 0 ? NR - 3 : 0), NO>(ep);
    };
    // bf16, ReLU, then halves swapped between neighbouring 16-lane rows: each
    // lane holds 8 channels of one pixel (block 0 for even rows, 1 for odd)
    auto pack_row = [&](auto oc) -> u32x4 {
      constexpr int o = decltype(oc)::value;
      u32x2 w[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 v = acc[o & 3][h];
        w[h].x = relu_bf16x2(pack_bf16x2(v[0], v[1]));
        w[h].y = relu_bf16x2(pack_bf16x2(v[2], v[3]));
      }
      const auto sx = __builtin_amdgcn_permlane16_swap(w[0].x, w[1].x, false, false);
      const auto sy = __builtin_amdgcn_permlane16_swap(w[0].y, w[1].y, false, false);
      return u32x4{sx[0], sy[0], sx[1], sy[1]};
    };

    if (grp == 0) {
      if (haveA) {
        // layer A of tile tA: intermediate rows into buffer it & 1, zero
        // outside the image; the next tile's window is loaded meanwhile
        uint8_t *mid = lds_mid + (it & 1) * Lo::MID_BYTES;
        const uint32_t in_x = (unsigned)(dA.x0 - 1 + cpos) < (unsigned)dA.nx ? ~0u : 0u;
        const uint32_t lcol_n = lane_col(dAn);
        auto epA = [&](auto oc) {
          constexpr int o = decltype(oc)::value;
          const uint32_t in_y = (unsigned)(dA.y0 - 1 + o) < (unsigned)dA.ny ? ~0u : 0u;
          const uint32_t keep = in_y & in_x;
          u32x4 q = pack_row(oc);
          q &= u32x4{keep, keep, keep, keep};
          *reinterpret_cast<u32x4 *>(mid + rr_off(o * IW + cpos, 2 * wq + (g >> 1))) = q;
        };
        auto pfA = [&](auto stc) {
          constexpr int stg = decltype(stc)::value;
          if constexpr (stg >= 4 && stg < 4 + NLOAD)
            pre[stg - 4] = load_chunk(dAn, lcol_n, std::integral_constant<int, stg - 4>{});
        };
        layer(bl, std::integral_constant<int, Lo::IH>{}, std::integral_constant<int, 0>{}, epA,
              pfA);
      }
    } else {
      if (haveB) {
        // layer B of the previous tile from buffer (it - 1) & 1 to memory;
        // lanes outside the tile (and the padding columns) store to the trash
        int bm[8][2];
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
          for (int kh = 0; kh < 2; ++kh) {
            int v = bl[m][kh] + Lo::IN_BYTES + ((it - 1) & 1) * Lo::MID_BYTES;
            asm volatile("" : "+v"(v));
            bm[m][kh] = v;
          }
        const int64_t lane_b = 32 * wq + 16 * (g >> 1);
        const int64_t trash_b = dB.trash * Lo::PIXB + lane_b;
        const int64_t col_b = (int64_t)(dB.x0 + cpos + 1) * Lo::PIXB + lane_b;
        const int64_t ok_c = cpos < dB.w ? -1 : 0;
        auto epB = [&](auto oc) {
          constexpr int o = decltype(oc)::value;
          const int64_t ok = (o < dB.h ? -1 : 0) & ok_c;
          const int64_t roff = (int64_t)(dB.y0 + o + 1) * dB.apitch * Lo::PIXB;
          const u32x4 q = pack_row(oc);
          const int64_t bo = ((col_b + roff) & ok) | (trash_b & ~ok);
          *reinterpret_cast<PNP_GLOBAL u32x4 *>(dB.out + bo) = q;
        };
        auto pfB = [&](auto) {};
        layer(bm, std::integral_constant<int, Lo::MH>{}, std::integral_constant<int, 1>{}, epB,
              pfB);
      }
    }
    __syncthreads();                             // intermediate written / read, window read
    if (!haveA) break;                           // uniform: the last tile's layer B is done
    if (grp == 0) static_for<0, NLOAD>([&](auto ic) { put_chunk(ic, pre[decltype(ic)::value]); });
    __syncthreads();                             // next window in place
    dB = dA;
    haveB = true;
    dA = dAn;
    tA = tAn;
    ++it;
  }
}

// ---------------------------------------------------------------------
// Middle layers, row-reuse form for e4m3 input (F = 64; output e4m3 or
// bf16).  v_mfma_scale_f32_16x16x128_f8f6f4 takes K = 128 = two taps of 64
// channels: lane groups 0-1 carry one tap, groups 2-3 another.  Pairing the
// horizontal taps as (dx 0, dx 1) and (dx 2, none) keeps both halves of a B
// fragment in the same input row, so, as in the bf16 kernel, one B fragment
// of input row ir serves the three vertical taps.  Two pairs x three dy are
// six K steps (three zero tap slots: 12 slots for 9 taps).  One persistent
// workgroup of 4 waves per CU, wave w owns output rows 4w..4w+3.
// ---------------------------------------------------------------------
template <int OUT_FMT>
struct Rr8Layout {
  static constexpr int F = 64, MB = 4, PIXB = 64, CPP = 4;
  static constexpr int TH = 16, TW = kConvTileW, IH = TH + 2, IW = TW + 2;
  static constexpr int ROWS = 4;
  static constexpr int WBYTES = 6 * MB * 64 * 32;
  static constexpr int IN_BYTES = IH * IW * PIXB;
  static constexpr int OPIXB = F * FmtInfo<OUT_FMT>::bytes, OCPP = OPIXB / 16;
  static constexpr int OUT_BYTES = TH * TW * OPIXB;
  static constexpr int TILE_BYTES = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
  static constexpr int LDS_BYTES = TILE_BYTES + WBYTES + 2 * F * 4;   // + scale, bias
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};
// 64-byte e4m3 pixels: chunk k of pixel p, permuted by bits 2..3 of p so that
// lanes reading one chunk of 16 consecutive pixels spread over the banks
__device__ __forceinline__ int rr8_off(int p, int k) { return p * 64 + ((k ^ ((p >> 2) & 3)) << 4); }

template <int OUT_FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void conv_mid_rr8_kernel(ConvArgs a) {
  using Lo = Rr8Layout<OUT_FMT>;
  constexpr int NT = 256, MB = Lo::MB, IW = Lo::IW, ROWS = Lo::ROWS;
  constexpr int NCHUNK = Lo::IH * IW * Lo::CPP;
  constexpr int NLOAD = (NCHUNK + NT - 1) / NT;

  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_w = lds + Lo::TILE_BYTES;
  float *lds_osc = reinterpret_cast<float *>(lds_w + Lo::WBYTES);
  float *lds_bias = lds_osc + Lo::F;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;

  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  {
    const PNP_GLOBAL u32x4 *src = gp(reinterpret_cast<const u32x4 *>(a.wblob_rr));
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_w);
    for (int i = tid; i < Lo::WBYTES / 16; i += NT) dst[i] = src[i];
    if (tid < Lo::F) {
      lds_osc[tid] = gp(a.oscale)[tid];
      lds_bias[tid] = gp(a.bias)[tid];
    }
  }

  u32x4 pre[NLOAD];
  auto issue_load = [&](const MidTile &c, int i) {
    const int q0 = tid + i * NT, q = q0 < NCHUNK ? q0 : 0;
    const int pix = q / Lo::CPP, k = q % Lo::CPP;
    const int row = pix / IW, col = pix % IW;
    pre[i] = *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
        c.in + ((int64_t)(c.y0 + row) * c.apitch + (c.x0 + col)) * Lo::PIXB + k * 16);
  };
  auto store_lds = [&]() {
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q0 = tid + i * NT, q = q0 < NCHUNK ? q0 : 0;
      *reinterpret_cast<u32x4 *>(lds_in + rr8_off(q / Lo::CPP, q % Lo::CPP)) = pre[i];
    }
  };

  int ti = t_begin + slot;
  if (ti >= t_end) return;                       // uniform over the workgroup
  MidTile cur = mid_tile(a, ti);
  MidTile nxt = mid_tile(a, ti + per_xcd < t_end ? ti + per_xcd : t_begin);
#pragma unroll
  for (int i = 0; i < NLOAD; ++i) issue_load(cur, i);
  store_lds();
  __syncthreads();

  // A fragments of step (P, dy): 32 bytes per lane
  const uint8_t *abase = lds_w + lane * 32;
  i32x8 Ab[3][MB];
  auto load_a = [&](int P, int dy) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const uint8_t *src = abase + ((P * 3 + dy) * MB + mb) * 2048;
      const u32x4 lo = *reinterpret_cast<const u32x4 *>(src);
      const u32x4 hi = *reinterpret_cast<const u32x4 *>(src + 16);
      Ab[dy][mb] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                         (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
  };
  // slots of dy 0 and 1 hold pair 0 when a tile starts (see the schedule below)
  load_a(0, 0);
  load_a(0, 1);

  while (true) {
    const int tn = ti + per_xcd, tnn = tn + per_xcd;
    const MidTile after = mid_tile(a, tnn < t_end ? tnn : t_begin);
    __builtin_amdgcn_sched_barrier(0);

    f32x4 acc[MB][ROWS][2];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int o = 0; o < ROWS; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[mb][o][h] = f32x4{0.f, 0.f, 0.f, 0.f};

    // this lane's B column: pixel (ROWS*wave + ir, 16h + l16 + dx), 32 bytes at
    // chunk 2(g&1); dx = first tap of the pair for groups 0-1, second for 2-3
    // (pair 1's second tap has zero weights: any pixel of the row will do)
    const int bpix = (ROWS * wave) * IW + l16;
    constexpr int NR = ROWS + 2, NSTG = 2 * NR, PD = 2;
    i32x8 Bb[PD + 1][2];
    auto load_b = [&](int stg) {
      const int P = stg / NR, ir = stg % NR;
      const int dx = (g < 2) ? (P == 0 ? 0 : 2) : (P == 0 ? 1 : 2);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = bpix + ir * IW + 16 * h + dx;
        const u32x4 lo = *reinterpret_cast<const u32x4 *>(lds_in + rr8_off(p, 2 * (g & 1)));
        const u32x4 hi = *reinterpret_cast<const u32x4 *>(lds_in + rr8_off(p, 2 * (g & 1) + 1));
        Bb[stg % (PD + 1)][h] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
    };
#pragma unroll
    for (int k = 0; k < PD; ++k) load_b(k);
    // 12 stages (pair P, input row ir).  A slots: dy 2 is loaded at (P, 0)
    // (last used at the previous pair's row 5); dy 0 and 1 for the next pair
    // at (P, 4) and (P, 5), after their last use at rows 3 and 4.
#pragma unroll
    for (int stg = 0; stg < NSTG; ++stg) {
      const int P = stg / NR, ir = stg % NR;
      if (stg + PD < NSTG) load_b(stg + PD);
      if (ir == 0) load_a(P, 2);
      if (ir == 4) load_a(P ^ 1, 0);
      if (ir == 5) load_a(P ^ 1, 1);
      if (stg < NLOAD) issue_load(nxt, stg);      // the next tile's window, one per stage
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int o = ir - dy;
        if (o < 0 || o >= ROWS) continue;
        // dy 0 / 1 slots were refilled at rows 4 / 5 of this pair, after
        // their last use (rows 3 / 4): the MFMAs below run before the refill
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[mb][o][h] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                Ab[dy][mb], Bb[stg % (PD + 1)][h], acc[mb][o][h], 0, 0, 0, 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = NSTG; i < NLOAD; ++i) issue_load(nxt, i);

    // epilogue: scale, bias, ReLU, round to the output format, stage the tile
    // over the consumed input window, store whole pixels with 16-byte lanes
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const f32x4 osc = *reinterpret_cast<const f32x4 *>(lds_osc + mb * 16 + 4 * g);
      const f32x4 bia = *reinterpret_cast<const f32x4 *>(lds_bias + mb * 16 + 4 * g);
#pragma unroll
      for (int o = 0; o < ROWS; ++o)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = fmaxf(fmaf(acc[mb][o][h][e], osc[e], bia[e]), 0.0f);
          const int p = (ROWS * wave + o) * Lo::TW + 16 * h + l16;
          if constexpr (OUT_FMT == FMT_BF16) {
            u32x2 w;
            w.x = pack_bf16x2(v[0], v[1]);
            w.y = pack_bf16x2(v[2], v[3]);
            *reinterpret_cast<u32x2 *>(lds_in + rr_off(p, 2 * mb + (g >> 1)) + 8 * (g & 1)) = w;
          } else {
            const float is = a.out_inv_scale;
            const uint32_t w = pack_e4m3x4(v[0] * is, v[1] * is, v[2] * is, v[3] * is);
            *reinterpret_cast<uint32_t *>(lds_in + rr8_off(p, mb) + 4 * g) = w;
          }
        }
    }
    __syncthreads();
    {
      constexpr int NQ = Lo::TH * Lo::TW * Lo::OCPP, NS = NQ / NT;
      u32x4 st[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int q = i * NT + tid, p = q / Lo::OCPP, k = q % Lo::OCPP;
        st[i] = *reinterpret_cast<const u32x4 *>(
            lds_in + (OUT_FMT == FMT_BF16 ? rr_off(p, k) : rr8_off(p, k)));
      }
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int q = i * NT + tid;
        const int pix = q / Lo::OCPP, k = q % Lo::OCPP;
        const int r = pix / Lo::TW, c = pix % Lo::TW;
        const int64_t px = (r < cur.h && c < cur.w)
                               ? (int64_t)(cur.y0 + r + 1) * cur.apitch + (cur.x0 + c + 1)
                               : cur.trash;
        *reinterpret_cast<PNP_GLOBAL u32x4 *>(cur.out + px * Lo::OPIXB + k * 16) = st[i];
      }
    }
    __syncthreads();                             // staged outputs are read
    store_lds();
    __syncthreads();
    if (tn >= t_end) break;
    cur = nxt;
    nxt = after;
    ti = tn;
  }
}

// ---------------------------------------------------------------------
// Two consecutive e4m3 middle layers (F = 64, ReLU, e4m3 in and out) in one
// persistent kernel: the bf16 pair kernel's tiles, order and prefetch with
// 64-byte pixels.  v_mfma_scale_f32_16x16x128_f8f6f4 takes K = 128 = two
// taps of 64 channels; as in the single-layer e4m3 kernel the horizontal
// taps are paired as (dx 0, dx 1) and (dx 2, zero weights), so an input row
// takes two steps P, each serving the three vertical taps.  Output-channel
// scales, bias and ReLU apply in the epilogue; each layer's output is rounded
// to e4m3 with the next layer's activation scale.  LDS pixels are 64 bytes,
// unpadded, and chunk c (16 bytes) of the pixel in window column col sits at
// c ^ bit 2 of col.  A 16-byte LDS access is served in four passes of 16
// lanes (lane bit 5 and the parity of lane bits 2..4 pick the pass; the bank
// is the address mod 256, 64 banks of 4 bytes, as measured with the bank
// conflict counter).  A pass of a B read holds two lane groups, with chunks c
// and c + 2, each at columns that share their residue mod 4 in fours (col,
// col + 4, col + 8, col + 12): the swizzle gives those 16 reads 16 distinct
// 16-byte slots.  Both windows fit in 80 KB, so two workgroups can share a CU.
// ---------------------------------------------------------------------
struct Pair8Layout {
  static constexpr int F = 64, PIXB = 64, CPP = 4, NT = 256;
  static constexpr int TH = kPairTileH, TW = kPairTileW;
  static constexpr int MH = TH + 2, MW = TW + 2;
  static constexpr int IH = TH + 4, IW = TW + 4;
  static constexpr int IN_BYTES = IH * IW * PIXB;
  static constexpr int MID_BYTES = MH * IW * PIXB;
  static constexpr int LDS_BYTES = IN_BYTES + MID_BYTES + 4 * F * 4;  // scale, bias per layer
  static constexpr int NCHUNK = IH * IW * CPP, NLOAD = (NCHUNK + NT - 1) / NT;
  static constexpr int NL1 = NLOAD / 2, NL2 = NLOAD - NL1;
  // fused first layer: x window (IH + 2) x (IW + 2) as bf16, its scale and bias
  static constexpr int XH = IH + 2, XW = IW + 2, NX = XH * XW, XQ = (NX + NT - 1) / NT;
  static constexpr int FIRST_BYTES = NX * 2 + 2 * F * 4;
  static constexpr int lds_bytes(bool first) { return LDS_BYTES + (first ? FIRST_BYTES : 0); }
  // fused last layer: per-row partial sums of the 4 waves (2 blocks, lane
  // groups 0-2 = taps 0..11, 16 bytes per lane) in a ring of 3 rows, placed
  // in the part of the input window that only the second prefetch half fills
  static constexpr int STG_ROW = 4 * 2 * 48 * 16, STG_OFF = NL1 * 64 * PIXB;
  static_assert(STG_OFF + 3 * STG_ROW <= IN_BYTES, "last-layer ring");
};
static_assert(Pair8Layout::MW == 32 && Pair8Layout::lds_bytes(true) <= 80 * 1024,
              "e4m3 pair layout: two workgroups per CU");
// LDS byte offset of 16-byte chunk c (channels 16c .. 16c+15) of the pixel
// in window column col whose row-major window index is p
__device__ __forceinline__ constexpr int p8_off(int p, int col, int c) {
  return p * Pair8Layout::PIXB + ((c ^ ((col >> 2) & 1)) << 4);
}


// OUT2: storage format of the second layer's output (e4m3, or bf16 when the
// next layer reads bf16, e.g. the last layer).  LAST: the second layer feeds
// the network's last layer (64 -> 1, bf16), and instead of its activations
// the kernel writes that layer's per-tap partial sums (JobDesc::S, 12 floats
// per pixel, zero border of one record), as the bf16 last-middle kernel does:
// per output row each wave multiplies its 16 channels (rounded to bf16 after
// ReLU) by the last layer's weights on the matrix core (M = 9 taps padded to
// 16, K = 16 channels), the four waves' partials meet in LDS, and after a
// barrier 96 lanes add them and store the records.  FIRST (only with LAST, in
// the four-layer network whose one pair is both first and last): the
// network's first layer (1 -> 64, bf16 weights, e4m3 output) is computed per
// tile from x into the input window, as a phase before layer A, instead of
// reading its output from memory: each wave takes its 16 channels for every
// window pixel, one MFMA per 16 pixels (K = the 9 taps padded to 16), then
// scale, bias, ReLU and e4m3 as conv_first8_kernel does; window pixels
// outside the image are set to zero (the next layer's padding).
template <int OUT2, bool FIRST, bool LAST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPair8Wpe, kPair8Wpe)))
void conv_pair8_kernel(ConvArgs a) {
  using Lo = Pair8Layout;
  constexpr int NT = Lo::NT, IW = Lo::IW, NL1 = Lo::NL1, NL2 = Lo::NL2;
  constexpr int NP = 2, PD = 2;                   // steps per input row; B reads ahead
  static_assert(!FIRST || LAST, "the first layer rides only in the pair that also feeds the last layer");
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_mid = lds + Lo::IN_BYTES;
  float *lds_ep = reinterpret_cast<float *>(lds_mid + Lo::MID_BYTES);  // [layer][scale | bias]
  uint16_t *lds_x = reinterpret_cast<uint16_t *>(lds + Lo::LDS_BYTES);   // FIRST only
  float *lds_ep0 = reinterpret_cast<float *>(lds_x + Lo::NX);             // FIRST: scale | bias

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  // this wave's A fragments of both layers: step (P, dy), block `wave`, 32 B
  i32x8 WA[3 * NP], WB[3 * NP];
  {
    const PNP_GLOBAL u32x4 *wa = gp(reinterpret_cast<const u32x4 *>(a.wblob_rr));
    const PNP_GLOBAL u32x4 *wb = gp(reinterpret_cast<const u32x4 *>(a.wblob2));
#pragma unroll
    for (int s = 0; s < 3 * NP; ++s) {
      const int i = ((s * 4 + wave) * 64 + lane) * 2;
      const u32x4 a0 = wa[i], a1 = wa[i + 1], b0 = wb[i], b1 = wb[i + 1];
      WA[s] = i32x8{(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
      WB[s] = i32x8{(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
    }
  }
  // Per-channel scale and bias of each layer.  Where the output is e4m3 they
  // are stored times the next layer's inverse activation scale, a power of
  // two, so fma(v, scale, bias) is the scaled value exactly (rounding commutes
  // with a power-of-two factor) and the epilogue is one fma and one clamp.
  {
    const float *src = tid < 64 ? a.oscale : tid < 128 ? a.bias : tid < 192 ? a.oscale2 : a.bias2;
    const float is = tid < 128 ? a.out_inv_scale : (OUT2 == FMT_E4M3 ? a.out_inv_scale2 : 1.0f);
    lds_ep[tid] = gp(src)[tid & 63] * is;
    if (FIRST && tid < 128)
      lds_ep0[tid] = gp(tid < 64 ? a.first_oscale : a.first_bias)[tid & 63] * a.first_out_inv_scale;
  }
  // fused first layer: this wave's A fragment (rows = its 16 channels, K =
  // the 9 taps padded to 16: lane group g holds taps 4g .. 4g+3) and the
  // lane's tap offsets in the x window relative to the pixel's own
  // fused last layer: this wave's A fragment (rows = the 9 taps padded to
  // 16, K = its 16 channels: lane group g holds channels 16 wave + 4g ..)
  i16x4 AL;
  if constexpr (LAST) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      AL[e] = __builtin_bit_cast(
          short, f32_to_bf16(l16 < 9 ? gp(a.last_w)[(16 * wave + 4 * g + e) * 9 + l16] : 0.0f));
  }
  // fused first layer: this wave's A fragment, rows = its 16 channels; K slot
  // 4g + e holds tap (dy, dx) = (g, e) for g, e < 3 and a zero weight
  // otherwise, so that lane group g reads kernel row g of the x window at the
  // immediate offsets 0, 1, 2
  i16x4 A0;
  if constexpr (FIRST) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      A0[e] = __builtin_bit_cast(
          short, f32_to_bf16(g < 3 && e < 3 ? gp(a.first_w)[(16 * wave + l16) * 9 + 3 * g + e] : 0.0f));
  }
  // the intermediate's columns MW .. IW-1 are read only for the two padding
  // output columns and never written: zero the buffer once
  for (int i = tid; i < Lo::MID_BYTES / 16; i += NT)
    reinterpret_cast<u32x4 *>(lds_mid)[i] = u32x4{0u, 0u, 0u, 0u};

  // Window loads: load i takes pixels 64i .. 64i+63 of the window (row-major,
  // IW per row), lane (tid / 4, chunk tid % 4); lanes past the window repeat
  // a pixel of load 0 (storing the bytes its owner stores).  Positions beyond
  // the one-pixel zero border read the border.
  auto win_pix = [&](int i) {
    int q0 = 64 * i + (tid >> 2);
    asm volatile("" : "+v"(q0));
    return q0 < Lo::IH * IW ? q0 : ((tid >> 2) & 31);
  };
  auto load_chunk = [&](const MidTile &c, int i) -> u32x4 {
    const int q = win_pix(i);
    const int r = q / IW, col = q % IW;
    const int Y = min(max(c.y0 - 2 + r, -1), c.ny) + 1, X = min(max(c.x0 - 2 + col, -1), c.nx) + 1;
    return *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
        c.in + ((int64_t)Y * c.apitch + X) * Lo::PIXB + (tid & 3) * 16);
  };
  auto put_chunk = [&](int i, const u32x4 &v) {
    const int q = win_pix(i);
    *reinterpret_cast<u32x4 *>(lds_in + p8_off(q, q % IW, tid & 3)) = v;
  };
  static_assert(Lo::NLOAD * 64 >= Lo::IH * Lo::IW && Lo::NLOAD <= 2 * NL2, "window loads");

  // fused first layer: x window rows y0-3 .. y0+TH+2, columns x0-3 ..
  // x0+TW+2, clamped to the image and its zero ring (positions outside the
  // image only feed window pixels that are set to zero)
  auto load_x = [&](const MidTile &c, int i) -> float {
    int q0 = tid + i * NT;
    asm volatile("" : "+v"(q0));
    const int q = q0 < Lo::NX ? q0 : 0;
    const int r = q / Lo::XW, col = q % Lo::XW;
    const int Y = min(max(c.y0 - 3 + r, -1), c.ny), X = min(max(c.x0 - 3 + col, -1), c.nx);
    return c.x[(int64_t)(Y + c.xb) * c.xpitch + (X + c.xb)];
  };
  auto put_x = [&](int i, float v) {
    const int q = tid + i * NT;
    if (q < Lo::NX) lds_x[q] = f32_to_bf16(v);
  };
  // Block blk covers window pixels 16 blk .. 16 blk + 15 (row-major); this
  // lane's pixel (l0_wr, l0_wc) and the x-window element of its tap row,
  // l0_xa, step by 16 pixels per block.  l0_reset starts them from an opaque
  // value, which keeps the compiler from holding every block's addresses
  // across the tile loop.
  constexpr int NWIN0 = Lo::IH * IW, NB0 = (NWIN0 + 15) / 16, NTAIL0 = NWIN0 - 16 * (NB0 - 1);
  int l0_wc = 0, l0_wr = 0, l0_xa = 0, l0_xa0 = 0;
  f32x4 sc0 = {}, bi0 = {};
  auto l0_reset = [&]() {
    l0_wc = l16;
    l0_wr = 0;
    l0_xa = (g < 3 ? g : 2) * Lo::XW + l16;
    asm volatile("" : "+v"(l0_wc), "+v"(l0_wr), "+v"(l0_xa));
    l0_xa0 = l0_xa;                              // the tail's lanes past the window read here
  };
  auto l0_block = [&](const MidTile &c, auto blkc) {
    constexpr int blk = decltype(blkc)::value;
    if constexpr (blk > 0) {
      l0_wc += 16;
      const bool wrap = l0_wc >= IW;
      l0_wc = wrap ? l0_wc - IW : l0_wc;
      l0_wr += wrap ? 1 : 0;
      l0_xa += wrap ? 16 + (Lo::XW - IW) : 16;
    }
    const bool tail_out = blk == NB0 - 1 && l16 >= NTAIL0;
    const uint16_t *xp = lds_x + (tail_out ? l0_xa0 : l0_xa);
    i16x4 Bx;
    Bx[0] = (short)xp[0];
    Bx[1] = (short)xp[1];
    Bx[2] = (short)xp[2];
    Bx[3] = 0;
    const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0, Bx, f32x4{0.f, 0.f, 0.f, 0.f},
                                                            0, 0, 0);
    const bool inside = (unsigned)(c.y0 - 2 + l0_wr) < (unsigned)c.ny &&
                        (unsigned)(c.x0 - 2 + l0_wc) < (unsigned)c.nx;
    uint32_t w = pack_e4m3x4_relu(fmaf(d[0], sc0[0], bi0[0]), fmaf(d[1], sc0[1], bi0[1]),
                                  fmaf(d[2], sc0[2], bi0[2]), fmaf(d[3], sc0[3], bi0[3]));
    w = inside ? w : 0u;
    if (!tail_out)
      *reinterpret_cast<uint32_t *>(lds_in + (16 * blk + l16) * Lo::PIXB + 4 * g +
                                    ((wave ^ ((l0_wc >> 2) & 1)) << 4)) = w;
  };
  auto layer0 = [&](const MidTile &c) {
    l0_reset();
    static_for<0, NB0>([&](auto b) { l0_block(c, b); });
  };

  int ti = t_begin + slot;
  if (ti >= t_end) return;                       // uniform over the workgroup
  MidTile cur = mid_tile(a, ti);
  MidTile nxt = mid_tile(a, ti + per_xcd < t_end ? ti + per_xcd : t_begin);
  u32x4 pre[NL2];
  float prex[FIRST ? Lo::XQ : 1];
  if constexpr (FIRST) {
#pragma unroll
    for (int i = 0; i < Lo::XQ; ++i) prex[i] = load_x(cur, i);
#pragma unroll
    for (int i = 0; i < Lo::XQ; ++i) put_x(i, prex[i]);
    __syncthreads();
    sc0 = *reinterpret_cast<const f32x4 *>(lds_ep0 + 16 * wave + 4 * g);
    bi0 = *reinterpret_cast<const f32x4 *>(lds_ep0 + Lo::F + 16 * wave + 4 * g);
    layer0(cur);
  } else {
#pragma unroll
    for (int i = 0; i < NL1; ++i) pre[i] = load_chunk(cur, i);
#pragma unroll
    for (int i = 0; i < NL1; ++i) put_chunk(i, pre[i]);
#pragma unroll
    for (int i = 0; i < NL2; ++i) pre[i] = load_chunk(cur, NL1 + i);
#pragma unroll
    for (int i = 0; i < NL2; ++i) put_chunk(NL1 + i, pre[i]);
  }
  __syncthreads();

  // B fragment of step P at window row ir, block h: this lane's pixel is in
  // column 16h + q, q = dx + l16 with dx = the tap its lane group carries,
  // 32 bytes at channel 32(g&1): chunks 2(g&1) (lo) and 2(g&1) + 1 (hi).
  // Column 16h + q swizzles as column q, so the address is 64 (ir*IW + 16h)
  // (an immediate) plus base[P][lo/hi] (per lane).
  int base_in[NP][2], base_mid[NP][2];
#pragma unroll
  for (int P = 0; P < NP; ++P)
#pragma unroll
    for (int hl = 0; hl < 2; ++hl) {
      const int q = ((g < 2) ? (P == 0 ? 0 : 2) : (P == 0 ? 1 : 2)) + l16;
      int v = p8_off(q, q, 2 * (g & 1) + hl), u = v + Lo::IN_BYTES;
      asm volatile("" : "+v"(v), "+v"(u));
      base_in[P][hl] = v;
      base_mid[P][hl] = u;
    }

  while (true) {
    const int tn = ti + per_xcd, tnn = tn + per_xcd;
    const MidTile after = mid_tile(a, tnn < t_end ? tnn : t_begin);
    f32x4 acc[4][2];
    i32x8 Bb[PD + 1][2];

    auto layer = [&](const int (&base)[NP][2], const i32x8 *W, auto NRc, auto ep, auto pf) {
      constexpr int NR = decltype(NRc)::value, NO = NR - 2, NSTG = NR * NP;
      auto load_b = [&](auto stc) {
        constexpr int stg = decltype(stc)::value;
        constexpr int ir = stg / NP, P = stg % NP;
        static_for<0, 2>([&](auto hc) {
          constexpr int c = (ir * IW + 16 * decltype(hc)::value) * Lo::PIXB;
          const u32x4 lo = *reinterpret_cast<const u32x4 *>(lds + base[P][0] + c);
          const u32x4 hi = *reinterpret_cast<const u32x4 *>(lds + base[P][1] + c);
          Bb[stg % (PD + 1)][decltype(hc)::value] =
              i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        });
      };
      static_for<0, PD>(load_b);
      static_for<0, NSTG>([&](auto stc) {
        constexpr int stg = decltype(stc)::value;
        constexpr int ir = stg / NP, P = stg % NP;
        if constexpr (stg + PD < NSTG) load_b(std::integral_constant<int, stg + PD>{});
        pf(stc);
        if constexpr (P == 0 && ir < NO) {
          acc[ir & 3][0] = f32x4{0.f, 0.f, 0.f, 0.f};
          acc[ir & 3][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        static_for<0, 3>([&](auto dyc) {
          constexpr int dy = decltype(dyc)::value, o = ir - dy;
          if constexpr (o >= 0 && o < NO) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
              acc[o & 3][h] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                  W[P * 3 + dy], Bb[stg % (PD + 1)][h], acc[o & 3][h], 0, 0, 0, 0, 0, 0);
          }
        });
        // output row ir - 3 finished one input row ago
        if constexpr (P == 0 && ir >= 3 && ir - 3 < NO) ep(std::integral_constant<int, ir - 3>{});
        __builtin_amdgcn_sched_barrier(0);
      });
      static_for<(NR - 3 > 0 ? NR - 3 : 0), NO>(ep);
    };

    // Epilogue: scale and bias (both already times the next layer's inverse
    // activation scale), ReLU, e4m3; then halves are swapped between
    // neighbouring 16-lane rows so that each lane holds 8 channels (8 bytes)
    // of one pixel: block 0's for even rows, block 1's for odd rows.
    auto pack_row = [&](auto oc, int layer_i) -> u32x2 {
      constexpr int o = decltype(oc)::value;
      const float *ep = lds_ep + layer_i * 2 * Lo::F;
      const f32x4 osc = *reinterpret_cast<const f32x4 *>(ep + 16 * wave + 4 * g);
      const f32x4 bia = *reinterpret_cast<const f32x4 *>(ep + Lo::F + 16 * wave + 4 * g);
      uint32_t w[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 v = acc[o & 3][h];
        w[h] = pack_e4m3x4_relu(fmaf(v[0], osc[0], bia[0]), fmaf(v[1], osc[1], bia[1]),
                                fmaf(v[2], osc[2], bia[2]), fmaf(v[3], osc[3], bia[3]));
      }
      const auto s = __builtin_amdgcn_permlane16_swap(w[0], w[1], false, false);
      return u32x2{s[0], s[1]};
    };
    const int cpos = 16 * (g & 1) + l16;         // column of this lane's pixel after the swap
    const int cbyte = 16 * wave + 8 * (g >> 1);  // its 8 channels inside the pixel
    // the same 8 channels in the swizzled intermediate (+ 64 o IW for row o)
    const int mid_w = p8_off(cpos, cpos, wave) + 8 * (g >> 1);

    // layer A: intermediate rows into LDS (zero outside the image)
    const uint32_t in_x = (unsigned)(cur.x0 - 1 + cpos) < (unsigned)cur.nx ? ~0u : 0u;
    auto epA = [&](auto oc) {
      constexpr int o = decltype(oc)::value;
      const uint32_t in_y = (unsigned)(cur.y0 - 1 + o) < (unsigned)cur.ny ? ~0u : 0u;  // uniform
      const uint32_t keep = in_y & in_x;
      u32x2 q = pack_row(oc, 0);
      q &= u32x2{keep, keep};
      *reinterpret_cast<u32x2 *>(lds_mid + o * IW * Lo::PIXB + mid_w) = q;
    };
    auto pfA = [&](auto stc) {
      constexpr int stg = decltype(stc)::value;
      if constexpr (!FIRST && stg >= 4 && stg < 4 + NL1) pre[stg - 4] = load_chunk(nxt, stg - 4);
    };
    layer(base_in, WA, std::integral_constant<int, Lo::IH>{}, epA, pfA);
    __syncthreads();                             // intermediate written, window read
    if constexpr (!FIRST) {
#pragma unroll
      for (int i = 0; i < NL1; ++i) put_chunk(i, pre[i]);
    }

    // layer B: the tile's rows to memory; lanes outside the tile (and the
    // two padding columns) store to the trash pixel.  bf16 output: 128-byte
    // pixels, this lane's 8 channels are 16 bytes at 32 wave + 16 (g >> 1).
    constexpr int OPIXB = OUT2 == FMT_BF16 ? 2 * Lo::PIXB : Lo::PIXB;
    const int obyte = OUT2 == FMT_BF16 ? 2 * cbyte : cbyte;
    const int64_t trash_b = cur.trash * OPIXB + obyte;
    const int64_t col_b = (int64_t)(cur.x0 + cpos + 1) * OPIXB + obyte;
    const int64_t ok_c = cpos < cur.w ? -1 : 0;
    const int64_t spitch = cur.nx + 2, strash = (int64_t)(cur.ny + 2) * spitch;
    auto epB = [&](auto oc) {
      constexpr int o = decltype(oc)::value;
      const int64_t ok = (o < cur.h ? -1 : 0) & ok_c;
      const int64_t roff = (int64_t)(cur.y0 + o + 1) * cur.apitch * OPIXB;
      const int64_t bo = ((col_b + roff) & ok) | (trash_b & ~ok);
      if constexpr (LAST) {
        const float *ep = lds_ep + 2 * Lo::F;
        const f32x4 osc = *reinterpret_cast<const f32x4 *>(ep + 16 * wave + 4 * g);
        const f32x4 bia = *reinterpret_cast<const f32x4 *>(ep + Lo::F + 16 * wave + 4 * g);
        uint8_t *ring = lds_in + Lo::STG_OFF + (o % 3) * Lo::STG_ROW;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4 v = acc[o & 3][h];
          i16x4 bv;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            bv[e] = __builtin_bit_cast(short, f32_to_bf16(fmaxf(fmaf(v[e], osc[e], bia[e]), 0.0f)));
          // taps 4g .. 4g+3 of pixel l16 of block h, over this wave's channels
          const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(AL, bv, f32x4{0.f, 0.f, 0.f, 0.f},
                                                                  0, 0, 0);
          if (g < 3)
            *reinterpret_cast<f32x4 *>(ring + ((wave * 2 + h) * 48 + 16 * g + l16) * 16) = d;
        }
        __syncthreads();
        if (tid < 96) {                          // (block, tap group, pixel) per lane
          const int h = tid / 48, r = tid % 48, c = 16 * h + (r & 15);
          f32x4 sum = *reinterpret_cast<const f32x4 *>(ring + (h * 48 + r) * 16);
#pragma unroll
          for (int w = 1; w < 4; ++w)
            sum += *reinterpret_cast<const f32x4 *>(ring + ((w * 2 + h) * 48 + r) * 16);
          const int64_t rec = (o < cur.h && c < cur.w)
                                  ? (int64_t)(cur.y0 + o + 1) * spitch + (cur.x0 + c + 1)
                                  : strash;
          *reinterpret_cast<PNP_GLOBAL f32x4 *>(cur.S + rec * 12 + 4 * (r >> 4)) = sum;
        }
      } else if constexpr (OUT2 == FMT_BF16) {
        const float *ep = lds_ep + 2 * Lo::F;
        const f32x4 osc = *reinterpret_cast<const f32x4 *>(ep + 16 * wave + 4 * g);
        const f32x4 bia = *reinterpret_cast<const f32x4 *>(ep + Lo::F + 16 * wave + 4 * g);
        u32x2 w[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4 v = acc[o & 3][h];
          w[h].x = pack_bf16x2(fmaxf(fmaf(v[0], osc[0], bia[0]), 0.0f),
                               fmaxf(fmaf(v[1], osc[1], bia[1]), 0.0f));
          w[h].y = pack_bf16x2(fmaxf(fmaf(v[2], osc[2], bia[2]), 0.0f),
                               fmaxf(fmaf(v[3], osc[3], bia[3]), 0.0f));
        }
        const auto sx = __builtin_amdgcn_permlane16_swap(w[0].x, w[1].x, false, false);
        const auto sy = __builtin_amdgcn_permlane16_swap(w[0].y, w[1].y, false, false);
        *reinterpret_cast<PNP_GLOBAL u32x4 *>(cur.out + bo) = u32x4{sx[0], sy[0], sx[1], sy[1]};
      } else {
        *reinterpret_cast<PNP_GLOBAL u32x2 *>(cur.out + bo) = pack_row(oc, 1);
      }
    };
    auto pfB = [&](auto stc) {
      constexpr int stg = decltype(stc)::value;
      if constexpr (FIRST) {
        if constexpr (stg >= 1 && stg < 1 + Lo::XQ) prex[stg - 1] = load_x(nxt, stg - 1);
      } else {
        if constexpr (stg >= 1 && stg < 1 + NL2) pre[stg - 1] = load_chunk(nxt, NL1 + stg - 1);
      }
    };
    layer(base_mid, WB, std::integral_constant<int, Lo::MH>{}, epB, pfB);
    if constexpr (LAST) __syncthreads();         // the last row's partials are summed
    if constexpr (FIRST) {
      // the x window is read by layer0 only, long done
#pragma unroll
      for (int i = 0; i < Lo::XQ; ++i) put_x(i, prex[i]);
    } else if constexpr (!FIRST) {
#pragma unroll
      for (int i = 0; i < NL2; ++i) put_chunk(NL1 + i, pre[i]);
    }
    __syncthreads();                             // next window in place, intermediate read
    if (tn >= t_end) break;
    cur = nxt;
    nxt = after;
    ti = tn;
    if constexpr (FIRST) {
      layer0(cur);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------
// Two consecutive e4m3 middle layers on separate waves, with the taps packed
// without zero slots.  Waves 0-3 run layer A of tile i and waves 4-7 layer B
// of tile i-1 from the other half of a double-buffered intermediate, as in
// the bf16 split-layer kernel; each wave holds one layer's A fragments for
// its 16 output channels.  K = 128 of v_mfma_scale_f32_16x16x128_f8f6f4 is two
// (tap, 64 channels) units.  The units of the window are numbered row-major,
// idx = 3 ir + dx (window row ir, horizontal tap dx), and B fragment m
// carries units 2m (lane groups 0-1) and 2m + 1 (groups 2-3), so no B
// fragment has an empty half.  Output row o needs units 3o .. 3o + 8: the
// five fragments floor(3o/2) .. floor((3o + 8)/2), with A fragment
// j = 2m - 3o + 1, which holds taps j - 1 and j of the 3x3 kernel (zero
// weights for taps outside 0..8).  Five K steps per row and layer for the
// nine taps, ten A fragments per layer.  LDS pixels as in the one-group e4m3
// pair kernel (64 bytes; chunk c at c ^ bit 2 of the column).
// ---------------------------------------------------------------------
struct Pair8WsLayout {
  static constexpr int F = 64, PIXB = 64, CPP = 4, NTG = 256, NA = 10;
  static constexpr int TH = kPair8WsTileH, TW = kPairTileW;
  static constexpr int MH = TH + 2, MW = TW + 2, IH = TH + 4, IW = TW + 4;
  static constexpr int IN_BYTES = IH * IW * PIXB;
  static constexpr int MID_BYTES = MH * IW * PIXB;
  static constexpr int LDS_BYTES = IN_BYTES + 2 * MID_BYTES + 4 * F * 4;   // + scale, bias per layer
  static constexpr int NCHUNK = IH * IW * CPP, NLOAD = (NCHUNK + NTG - 1) / NTG;
};
static_assert(Pair8WsLayout::MW == 32 && Pair8WsLayout::IW == 34 && Pair8WsLayout::TH % 2 == 0 &&
                  Pair8WsLayout::LDS_BYTES <= 160 * 1024 && Pair8WsLayout::PIXB == Pair8Layout::PIXB,
              "e4m3 split-layer pair layout");

// first and last B fragment of output row o
__host__ __device__ constexpr int p8s_first(int o) { return (3 * o) / 2; }
__host__ __device__ constexpr int p8s_last(int o) { return (3 * o + 8) / 2; }
// row o holds accumulator slot o % NS from its first fragment until its
// epilogue E fragments after its last: no two rows live at once may share one
constexpr bool p8s_slots_ok(int NR, int NS, int E) {
  const int NO = NR - 2, NF = 3 * NR / 2;
  for (int m = 0; m <= NF + E; ++m)
    for (int o1 = 0; o1 < NO; ++o1)
      for (int o2 = o1 + 1; o2 < NO; ++o2)
        if (o1 % NS == o2 % NS && p8s_first(o1) <= m && m <= p8s_last(o1) + E &&
            p8s_first(o2) <= m && m <= p8s_last(o2) + E)
          return false;
  return true;
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void conv_pair8_ws_kernel(ConvArgs a) {
  using Lo = Pair8WsLayout;
  constexpr int IW = Lo::IW, NLOAD = Lo::NLOAD;
  constexpr int NS = 4, E = 1, PD = 1;            // accumulator slots; epilogue delay; B reads ahead
  static_assert(p8s_slots_ok(Lo::IH, NS, E) && p8s_slots_ok(Lo::MH, NS, E), "accumulator slots");
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_mid = lds + Lo::IN_BYTES;          // two buffers of MID_BYTES
  float *lds_ep = reinterpret_cast<float *>(lds_mid + 2 * Lo::MID_BYTES);   // [layer][scale | bias]

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2, wq = wave & 3;       // layer (0: A, 1: B), channel block
  const int g = lane >> 4, l16 = lane & 15;
  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  i32x8 W[Lo::NA];
  {
    const PNP_GLOBAL u32x4 *w = gp(reinterpret_cast<const u32x4 *>(grp ? a.wblob2 : a.wblob_rr));
#pragma unroll
    for (int j = 0; j < Lo::NA; ++j) {
      const int i = ((j * 4 + wq) * 64 + lane) * 2;
      const u32x4 w0 = w[i], w1 = w[i + 1];
      W[j] = i32x8{(int)w0.x, (int)w0.y, (int)w0.z, (int)w0.w, (int)w1.x, (int)w1.y, (int)w1.z, (int)w1.w};
    }
  }
  // per-channel scale and bias of each layer, times the next layer's inverse
  // activation scale (a power of two: the fma then gives the scaled value
  // exactly)
  if (tid < 256) {
    const float *src = tid < 64 ? a.oscale : tid < 128 ? a.bias : tid < 192 ? a.oscale2 : a.bias2;
    lds_ep[tid] = gp(src)[tid & 63] * (tid < 128 ? a.out_inv_scale : a.out_inv_scale2);
  }
  // the intermediates' columns MW .. IW-1 are read only for the two padding
  // output columns and never written: zero both buffers once
  for (int i = tid; i < 2 * Lo::MID_BYTES / 16; i += 2 * Lo::NTG)
    reinterpret_cast<u32x4 *>(lds_mid)[i] = u32x4{0u, 0u, 0u, 0u};

  // Window loads by the layer-A waves (256 lanes): load i takes chunk q =
  // 256 i + t (t = tid mod 256) of the row-major window, pixel q / 4, chunk
  // q % 4; lanes past the window repeat chunk t (storing the bytes its owner
  // stores).  Positions beyond the one-pixel zero border read the border.
  const int tl = tid & 255;
  auto win_chunk = [&](int i) {
    int q = 256 * i + tl;
    asm volatile("" : "+v"(q));
    return q < Lo::NCHUNK ? q : tl;
  };
  auto load_chunk = [&](const MidTile &c, int i) -> u32x4 {
    const int q = win_chunk(i), p = q >> 2;
    const int r = p / IW, col = p % IW;
    const int Y = min(max(c.y0 - 2 + r, -1), c.ny) + 1, X = min(max(c.x0 - 2 + col, -1), c.nx) + 1;
    return *reinterpret_cast<const PNP_GLOBAL u32x4 *>(
        c.in + ((int64_t)Y * c.apitch + X) * Lo::PIXB + (q & 3) * 16);
  };
  auto put_chunk = [&](int i, const u32x4 &v) {
    const int q = win_chunk(i), p = q >> 2;
    *reinterpret_cast<u32x4 *>(lds_in + p8_off(p, p % IW, q & 3)) = v;
  };

  int tA = t_begin + slot;
  if (tA >= t_end) return;                       // uniform over the workgroup
  MidTile dA = mid_tile(a, tA), dB = dA;
  u32x4 pre[NLOAD];
  if (grp == 0) {
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) pre[i] = load_chunk(dA, i);
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) put_chunk(i, pre[i]);
  }
  // B fragment m = 3k + tau of a layer: lane group g < 2 reads unit 2m, g >= 2
  // unit 2m + 1, i.e. (window row, dx) = (2k, 0) | (2k, 1) for tau = 0,
  // (2k, 2) | (2k + 1, 0) for tau = 1, (2k + 1, 1) | (2k + 1, 2) for tau = 2;
  // the pixel is in column 16h + dx + l16, chunks 2(g & 1) (lo) and
  // 2(g & 1) + 1 (hi).  Column 16h + q swizzles as column q, so the address
  // is 64 (2k IW + 16h) (an immediate) plus bl[tau][lo/hi] (per lane).
  int bl[3][2];
#pragma unroll
  for (int tau = 0; tau < 3; ++tau)
#pragma unroll
    for (int hl = 0; hl < 2; ++hl) {
      const int u = 2 * tau + (g >> 1), drow = u / 3, q = u % 3 + l16;
      int v = drow * IW * Lo::PIXB + p8_off(q, q, 2 * (g & 1) + hl);
      asm volatile("" : "+v"(v));
      bl[tau][hl] = v;
    }
  __syncthreads();

  const int cpos = 16 * (g & 1) + l16;           // column of this lane's pixel after the swap
  const int cbyte = 16 * wq + 8 * (g >> 1);      // its 8 channels inside the pixel
  const int mid_w = p8_off(cpos, cpos, wq) + 8 * (g >> 1);
  bool haveB = false;
  int it = 0;
  while (true) {
    const bool haveA = tA < t_end;                // uniform
    const int tAn = tA + per_xcd;
    const MidTile dAn = mid_tile(a, tAn < t_end ? tAn : t_begin);
    f32x4 acc[NS][2];
    i32x8 Bb[PD + 1][2];

    auto layer = [&](const uint8_t *buf, const int (&base)[3][2], auto NRc, auto ep, auto pf) {
      constexpr int NR = decltype(NRc)::value, NO = NR - 2, NF = 3 * NR / 2;
      auto load_b = [&](auto mc) {
        constexpr int m = decltype(mc)::value, k = m / 3, tau = m % 3;
        static_for<0, 2>([&](auto hc) {
          constexpr int c = (2 * k * IW + 16 * decltype(hc)::value) * Lo::PIXB;
          const u32x4 lo = *reinterpret_cast<const u32x4 *>(buf + base[tau][0] + c);
          const u32x4 hi = *reinterpret_cast<const u32x4 *>(buf + base[tau][1] + c);
          Bb[m % (PD + 1)][decltype(hc)::value] =
              i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        });
      };
      static_for<0, PD>(load_b);
      static_for<0, NF>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        if constexpr (m + PD < NF) load_b(std::integral_constant<int, m + PD>{});
        pf(mc);
        static_for<0, NO>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
          if constexpr (p8s_first(o) == m) {
            acc[o % NS][0] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[o % NS][1] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
          if constexpr (p8s_first(o) <= m && m <= p8s_last(o)) {
            constexpr int j = 2 * m - 3 * o + 1;
#pragma unroll
            for (int h = 0; h < 2; ++h)
              acc[o % NS][h] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                  W[j], Bb[m % (PD + 1)][h], acc[o % NS][h], 0, 0, 0, 0, 0, 0);
          }
        });
        static_for<0, NO>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
          if constexpr (p8s_last(o) + E == m) ep(oc);
        });
        __builtin_amdgcn_sched_barrier(0);
      });
      static_for<0, NO>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        if constexpr (p8s_last(o) + E >= NF) ep(oc);
      });
    };

    // scale and bias (times the next layer's inverse activation scale),
    // ReLU, e4m3, then halves swapped between neighbouring 16-lane rows: each
    // lane holds 8 channels (8 bytes) of one pixel, block 0's for even rows,
    // block 1's for odd rows
    auto pack_row = [&](auto oc, int layer_i) -> u32x2 {
      constexpr int o = decltype(oc)::value;
      const float *ep = lds_ep + layer_i * 2 * Lo::F;
      const f32x4 osc = *reinterpret_cast<const f32x4 *>(ep + 16 * wq + 4 * g);
      const f32x4 bia = *reinterpret_cast<const f32x4 *>(ep + Lo::F + 16 * wq + 4 * g);
      uint32_t w[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 v = acc[o % NS][h];
        w[h] = pack_e4m3x4_relu(fmaf(v[0], osc[0], bia[0]), fmaf(v[1], osc[1], bia[1]),
                                fmaf(v[2], osc[2], bia[2]), fmaf(v[3], osc[3], bia[3]));
      }
      const auto sw = __builtin_amdgcn_permlane16_swap(w[0], w[1], false, false);
      return u32x2{sw[0], sw[1]};
    };

    if (grp == 0) {
      if (haveA) {
        // layer A of tile tA: intermediate rows into buffer it & 1, zero
        // outside the image; the next tile's window is loaded meanwhile
        uint8_t *mid = lds_mid + (it & 1) * Lo::MID_BYTES;
        const uint32_t in_x = (unsigned)(dA.x0 - 1 + cpos) < (unsigned)dA.nx ? ~0u : 0u;
        auto epA = [&](auto oc) {
          constexpr int o = decltype(oc)::value;
          const uint32_t in_y = (unsigned)(dA.y0 - 1 + o) < (unsigned)dA.ny ? ~0u : 0u;  // uniform
          const uint32_t keep = in_y & in_x;
          u32x2 q = pack_row(oc, 0);
          q &= u32x2{keep, keep};
          *reinterpret_cast<u32x2 *>(mid + o * IW * Lo::PIXB + mid_w) = q;
        };
        auto pfA = [&](auto mc) {
          constexpr int m = decltype(mc)::value;
          if constexpr (m >= 2 && m < 2 + NLOAD) pre[m - 2] = load_chunk(dAn, m - 2);
        };
        layer(lds_in, bl, std::integral_constant<int, Lo::IH>{}, epA, pfA);
      }
    } else {
      if (haveB) {
        // layer B of the previous tile from buffer (it - 1) & 1 to memory;
        // lanes outside the tile (and the padding columns) store to the trash
        const uint8_t *mid = lds_mid + ((it - 1) & 1) * Lo::MID_BYTES;
        const int64_t trash_b = dB.trash * Lo::PIXB + cbyte;
        const int64_t col_b = (int64_t)(dB.x0 + cpos + 1) * Lo::PIXB + cbyte;
        const int64_t ok_c = cpos < dB.w ? -1 : 0;
        auto epB = [&](auto oc) {
          constexpr int o = decltype(oc)::value;
          const int64_t ok = (o < dB.h ? -1 : 0) & ok_c;
          const int64_t roff = (int64_t)(dB.y0 + o + 1) * dB.apitch * Lo::PIXB;
          const int64_t bo = ((col_b + roff) & ok) | (trash_b & ~ok);
          *reinterpret_cast<PNP_GLOBAL u32x2 *>(dB.out + bo) = pack_row(oc, 1);
        };
        auto pfB = [&](auto) {};
        layer(mid, bl, std::integral_constant<int, Lo::MH>{}, epB, pfB);
      }
    }
    __syncthreads();                             // intermediate written / read, window read
    if (!haveA) break;                           // uniform: the last tile's layer B is done
    if (grp == 0) {
#pragma unroll
      for (int i = 0; i < NLOAD; ++i) put_chunk(i, pre[i]);
    }
    __syncthreads();                             // next window in place
    dB = dA;
    haveB = true;
    dA = dAn;
    tA = tAn;
    ++it;
  }
}

// G from the fused last layer's partials: G(p) = scale * sum over taps of the
// tap's partial at the neighbour the tap reads, + bias.  The records' zero
// border supplies the zero padding at the image edge.  A tile's records (its
// rows and columns plus one on each side) are contiguous per row, so they
// are staged in LDS with 16-byte loads, all issued before the first is
// stored, and the taps are summed from there.
__global__ __launch_bounds__(256) void g_from_s_kernel(ConvArgs a) {
  constexpr int RW = kConvTileW + 2, RREC = 12, NCH = RW * RREC / 4;   // 16-byte chunks per row
  constexpr int NQ = (18 * NCH + 255) / 256;
  __shared__ __attribute__((aligned(16))) float srec[18 * RW * RREC];
  const PNP_CONST TileRef &tl = cp(a.tiles)[xcd_tile(blockIdx.x, a.n_tiles)];
  const PNP_CONST JobDesc &j = cp(a.jobs)[tl.job];
  const PNP_GLOBAL float *S = gp(j.S);
  const int64_t spitch = j.nx + 2;
  const int rows = tl.h + 2, nch = (tl.w + 2) * RREC / 4;
  // record (y0 + r, x0 + c) of the bordered record grid holds pixel
  // (y0 + r - 1, x0 + c - 1); rows y0 .. y0+h+1, columns x0 .. x0+w+1.
  // Chunks past the tile read chunk 0 of its first row and drop it.
  f32x4 v[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q0 = threadIdx.x + 256 * i;
    const int r0 = q0 / NCH, k0 = q0 % NCH;
    const bool in = r0 < rows && k0 < nch;
    const int r = in ? r0 : 0, k = in ? k0 : 0;
    v[i] = *reinterpret_cast<const PNP_GLOBAL f32x4 *>(
        S + ((int64_t)(tl.y0 + r) * spitch + tl.x0) * RREC + 4 * k);
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + 256 * i;
    const int r = q / NCH, k = q % NCH;
    if (r < rows && k < nch) *reinterpret_cast<f32x4 *>(srec + r * RW * RREC + 4 * k) = v[i];
  }
  __syncthreads();
  const float sc = a.oscale[0], bi = a.bias[0];
  const int npix = tl.h * tl.w;
  for (int pix = threadIdx.x; pix < npix; pix += 256) {
    const int r = pix / tl.w, c = pix % tl.w;
    float acc = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      // output (Y, X) reads input (Y + dy - 1, X + dx - 1): record (r + dy, c + dx)
      const int dy = tap / 3, dx = tap % 3;
      acc += srec[((r + dy) * RW + (c + dx)) * RREC + tap];
    }
    gp(j.G)[(int64_t)(tl.y0 + r) * j.nx + tl.x0 + c] = acc * sc + bi;
  }
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
template <int IN_FMT, int OUT_FMT, int F, int NW>
static hipError_t launch_mid_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  const size_t lds = MidLayout<IN_FMT, OUT_FMT, F, NW>::LDS_BYTES;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&conv_mid_kernel<IN_FMT, OUT_FMT, F, NW>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((conv_mid_kernel<IN_FMT, OUT_FMT, F, NW>), dim3(n_wg), dim3(NW * 64), lds,
                     s, a);
  return hipGetLastError();
}

static_assert(2 * kNwLowp == RrLayout::TH, "bf16 tile rows");
template <int OUT_FMT>
static hipError_t launch_rr8_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  constexpr int lds = Rr8Layout<OUT_FMT>::LDS_BYTES;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&conv_mid_rr8_kernel<OUT_FMT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((conv_mid_rr8_kernel<OUT_FMT>), dim3(n_wg), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <bool FIRST, bool LAST>
static hipError_t launch_rr_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  constexpr int lds = RrLayout::lds_bytes(FIRST, LAST);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&conv_mid_rr_kernel<FIRST, LAST>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((conv_mid_rr_kernel<FIRST, LAST>), dim3(n_wg), dim3(256), lds, s, a);
  return hipGetLastError();
}
static hipError_t launch_rr(const ConvArgs &a, int n_wg, hipStream_t s) {
  return launch_rr_t<false, false>(a, n_wg, s);
}

bool mid_last_fusable(int in_fmt, int out_fmt, int F, int relu, int unit, int last_in_fmt,
                      int last_cin, int last_cout) {
  return in_fmt == FMT_BF16 && out_fmt == FMT_BF16 && F == 64 && relu && unit &&
         last_in_fmt == FMT_BF16 && last_cin == 64 && last_cout == 1;
}

hipError_t launch_conv_mid_last(const ConvArgs &a, int n_wg, bool first, hipStream_t s) {
  // first and last fused into one middle layer (K = 3) is not built: the
  // engine fuses the last layer only when K >= 4
  if (first || !a.last_w || a.tile_rows != RrLayout::TH) return hipErrorInvalidValue;
  return launch_rr_t<false, true>(a, n_wg, s);
}

hipError_t launch_g_from_s(const ConvArgs &a, int n_tiles, hipStream_t s) {
  if (a.tile_rows < 1 || a.tile_rows > 16) return hipErrorInvalidValue;   // LDS sized for 16
  hipLaunchKernelGGL(g_from_s_kernel, dim3(n_tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}


bool pair_fusable(int in_fmt, int out_fmt, int F, int relu, int unit, int in_fmt2, int out_fmt2,
                  int relu2, int unit2) {
  return in_fmt == FMT_BF16 && out_fmt == FMT_BF16 && F == 64 && relu && unit &&
         in_fmt2 == FMT_BF16 && out_fmt2 == FMT_BF16 && relu2 && unit2;
}

hipError_t launch_conv_pair_ws(const ConvArgs &a, int n_wg, hipStream_t s) {
  if (!a.wblob || !a.wblob2 || !a.bias || !a.bias2 || n_wg <= 0 || n_wg % 8 != 0)
    return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&conv_pair_ws_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       PairWsLayout::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(conv_pair_ws_kernel, dim3(n_wg), dim3(512), PairWsLayout::LDS_BYTES, s, a);
  return hipGetLastError();
}


bool pair8_fusable(int in_fmt, int out_fmt, int F, int relu, int in_fmt2, int out_fmt2,
                   int relu2) {
  return in_fmt == FMT_E4M3 && out_fmt == FMT_E4M3 && F == 64 && relu &&
         in_fmt2 == FMT_E4M3 && (out_fmt2 == FMT_E4M3 || out_fmt2 == FMT_BF16) && relu2;
}

int pair8_wg_per_cu() { return kPair8Wpe; }

template <int OUT2, bool FIRST, bool LAST>
static hipError_t launch_pair8_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  constexpr int lds = Pair8Layout::lds_bytes(FIRST);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&conv_pair8_kernel<OUT2, FIRST, LAST>),
        hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((conv_pair8_kernel<OUT2, FIRST, LAST>), dim3(n_wg), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_conv_pair8(const ConvArgs &a, int out_fmt2, bool first, bool last, int n_wg,
                             hipStream_t s) {
  if (!a.wblob_rr || !a.wblob2 || !a.bias || !a.bias2 || !a.oscale || !a.oscale2 || n_wg <= 0 ||
      n_wg % 8 != 0)
    return hipErrorInvalidValue;
  if (first && (!a.first_w || !a.first_bias || !a.first_oscale)) return hipErrorInvalidValue;
  if (last) {
    if (!a.last_w || out_fmt2 != FMT_BF16) return hipErrorInvalidValue;
    return first ? launch_pair8_t<FMT_BF16, true, true>(a, n_wg, s)
                 : launch_pair8_t<FMT_BF16, false, true>(a, n_wg, s);
  }
  if (first) return hipErrorInvalidValue;        // the first layer rides only with the last
  if (out_fmt2 == FMT_E4M3) return launch_pair8_t<FMT_E4M3, false, false>(a, n_wg, s);
  if (out_fmt2 == FMT_BF16) return launch_pair8_t<FMT_BF16, false, false>(a, n_wg, s);
  return hipErrorInvalidValue;
}

hipError_t launch_conv_pair8_ws(const ConvArgs &a, int n_wg, hipStream_t s) {
  if (!a.wblob_rr || !a.wblob2 || !a.bias || !a.bias2 || !a.oscale || !a.oscale2 || n_wg <= 0 ||
      n_wg % 8 != 0)
    return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&conv_pair8_ws_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       Pair8WsLayout::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(conv_pair8_ws_kernel, dim3(n_wg), dim3(512), Pair8WsLayout::LDS_BYTES, s, a);
  return hipGetLastError();
}

bool last_pair8_fusable(int out_fmt2, int last_in_fmt, int last_cin, int last_cout) {
  return out_fmt2 == FMT_BF16 && last_in_fmt == FMT_BF16 && last_cin == 64 &&
         last_cout == 1;
}

bool first_pair8_fusable(int in_fmt0, int out_fmt0, int cin0, int cout0, int relu0) {
  return in_fmt0 == FMT_BF16 && out_fmt0 == FMT_E4M3 && cin0 == 1 && cout0 == 64 &&
         relu0;
}

bool first_mid_fusable(int in_fmt0, int out_fmt0, int cout0, int relu0, int unit0, int in_fmt1,
                       int out_fmt1, int F, int relu1, int unit1) {
  return in_fmt0 == FMT_BF16 && out_fmt0 == FMT_BF16 && cout0 == 64 && relu0 &&
         unit0 && in_fmt1 == FMT_BF16 && out_fmt1 == FMT_BF16 && F == 64 && relu1 && unit1;
}

hipError_t launch_conv_first_mid(const ConvArgs &a, int n_wg, hipStream_t s) {
  if (!a.first_w || !a.first_bias || a.tile_rows != RrLayout::TH) return hipErrorInvalidValue;
  return launch_rr_t<true, false>(a, n_wg, s);
}

// tile rows of the middle-layer kernel for an input format
int mid_tile_rows(int in_fmt) {
  if (in_fmt == FMT_F32) return 8;
  return 2 * kNwLowp;
}

size_t mid_lds_bytes(int in_fmt, int F) {
  if (in_fmt == FMT_BF16 && F == 64) return RrLayout::LDS_BYTES;
  const int TH = mid_tile_rows(in_fmt);
  const int ib = in_fmt == FMT_F32 ? 4 : (in_fmt == FMT_BF16 ? 2 : 1);
  const int ob = in_fmt == FMT_E4M3 ? 2 : ib;          // widest output format
  const int pstr = F * ib + 16, ostr = F * ob + 16;
  int nstep = in_fmt == FMT_E4M3 ? 5 : 9 * (in_fmt == FMT_F32 ? F / 16 : F / 32);
  int nch = (in_fmt == FMT_F32 && F == 64) ? 3 : 1;
  int fragb = in_fmt == FMT_E4M3 ? 32 : 16;
  const size_t in_b = (size_t)(TH + 2) * (kConvTileW + 2) * pstr;
  const size_t out_b = (size_t)TH * kConvTileW * ostr;
  return std::max(in_b, out_b) + (size_t)(nstep / nch) * (F / 16) * 64 * fragb + 2 * F * 4;
}

hipError_t launch_conv_mid(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_wg,
                           hipStream_t s) {
  if (in_fmt == FMT_F32 && out_fmt == FMT_F32) {
    if (F == 16) return launch_mid_t<FMT_F32, FMT_F32, 16, 4>(a, n_wg, s);
    if (F == 32) return launch_mid_t<FMT_F32, FMT_F32, 32, 4>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_F32, FMT_F32, 64, 4>(a, n_wg, s);
  } else if (in_fmt == FMT_BF16 && out_fmt == FMT_BF16) {
    if (F == 64 && a.relu && a.unit_scale) return launch_rr(a, n_wg, s);
    if (F == 32) return launch_mid_t<FMT_BF16, FMT_BF16, 32, kNwLowp>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_BF16, FMT_BF16, 64, kNwLowp>(a, n_wg, s);
  } else if (in_fmt == FMT_E4M3 && F == 64) {
    if (a.relu && a.wblob_rr) {
      if (out_fmt == FMT_E4M3) return launch_rr8_t<FMT_E4M3>(a, n_wg, s);
      if (out_fmt == FMT_BF16) return launch_rr8_t<FMT_BF16>(a, n_wg, s);
    }
    if (out_fmt == FMT_E4M3) return launch_mid_t<FMT_E4M3, FMT_E4M3, 64, kNwLowp>(a, n_wg, s);
    if (out_fmt == FMT_BF16) return launch_mid_t<FMT_E4M3, FMT_BF16, 64, kNwLowp>(a, n_wg, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_conv_first(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_tiles,
                             hipStream_t s) {
#define FIRST(I, O, FF)                                                                    \
  if (in_fmt == I && out_fmt == O && F == FF) {                                            \
    hipLaunchKernelGGL((conv_first_kernel<I, O, FF>), dim3(n_tiles), dim3(256), 0, s, a); \
    return hipGetLastError();                                                              \
  }
  FIRST(FMT_F32, FMT_F32, 16) FIRST(FMT_F32, FMT_F32, 32) FIRST(FMT_F32, FMT_F32, 64)
  FIRST(FMT_BF16, FMT_BF16, 32) FIRST(FMT_BF16, FMT_BF16, 64)
  FIRST(FMT_BF16, FMT_E4M3, 64) FIRST(FMT_F32, FMT_BF16, 64) FIRST(FMT_F32, FMT_E4M3, 64)
#undef FIRST
  return hipErrorInvalidValue;
}

hipError_t launch_conv_last(int in_fmt, int F, const ConvArgs &a, int n_tiles, hipStream_t s) {
  // the LDS window holds at most 16-row tiles
  if (a.tile_rows < 1 || a.tile_rows > 16) return hipErrorInvalidValue;
#define LAST(I, FF)                                                                    \
  if (in_fmt == I && F == FF) {                                                        \
    hipLaunchKernelGGL((conv_last_kernel<I, FF>), dim3(n_tiles), dim3(256), 0, s, a); \
    return hipGetLastError();                                                          \
  }
  LAST(FMT_F32, 16) LAST(FMT_F32, 32) LAST(FMT_F32, 64)
#undef LAST
  if (in_fmt == FMT_BF16 && (F == 32 || F == 64)) {
    if (F == 32) hipLaunchKernelGGL(conv_last_mfma_kernel<32>, dim3(n_tiles), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(conv_last_mfma_kernel<64>, dim3(n_tiles), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_conv_single(const ConvArgs &a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL(conv_single_kernel, dim3(n_tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pnp
