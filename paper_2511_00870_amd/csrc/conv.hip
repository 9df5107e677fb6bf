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

// Implementation choices of the middle-layer kernel (all compute the same
// result): register pipeline across K steps, LDS-staged epilogue, and the
// register-resident-weight kernel for bf16 / e4m3.
#ifndef PNP_MID_PIPE
#define PNP_MID_PIPE 1
#endif
#ifndef PNP_MID_STAGE
#define PNP_MID_STAGE 1
#endif
#ifndef PNP_USE_RW
#define PNP_USE_RW 0
#endif
#ifndef PNP_NW_LOWP
#define PNP_NW_LOWP 8
#endif
#ifndef PNP_XCD_MAP
#define PNP_XCD_MAP 1
#endif

namespace pnp {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;
// native 16-byte vector: a first-class IR type, so arrays of it stay in
// registers (HIP's u32x4 struct is copied with memcpy and can be left in
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

// pack 4 consecutive output channels of one pixel and store them
template <int FMT> __device__ __forceinline__ void store4(void *p, f32x4 v, float inv_s);
template <> __device__ __forceinline__ void store4<FMT_F32>(void *p, f32x4 v, float) {
  *reinterpret_cast<f32x4 *>(p) = v;
}
template <> __device__ __forceinline__ void store4<FMT_BF16>(void *p, f32x4 v, float) {
  uint2 w;
  w.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
  w.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
  *reinterpret_cast<uint2 *>(p) = w;
}
template <> __device__ __forceinline__ void store4<FMT_E4M3>(void *p, f32x4 v, float inv_s) {
  uint32_t w = (uint32_t)f32_to_e4m3(v[0] * inv_s) | ((uint32_t)f32_to_e4m3(v[1] * inv_s) << 8) |
               ((uint32_t)f32_to_e4m3(v[2] * inv_s) << 16) |
               ((uint32_t)f32_to_e4m3(v[3] * inv_s) << 24);
  *reinterpret_cast<uint32_t *>(p) = w;
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
  __shared__ float sx[18 * WW];
  const TileRef tl = a.tiles[blockIdx.x];
  const JobDesc &j = a.jobs[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const float *xb = j.x[t & 1];
  const int WH = tl.h + 2, B = j.xborder;
  for (int q = threadIdx.x; q < WH * WW; q += 256) {
    const int i = q / WW, c = q % WW;
    sx[q] = quant_in<IN_FMT>(xb[(int64_t)(tl.y0 - 1 + i + B) * j.xpitch + (tl.x0 - 1 + c + B)],
                             a.in_inv_scale);
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
  uint8_t *out = reinterpret_cast<uint8_t *>(j.act[a.out_slot]);
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
    uint8_t *dst = out + ((int64_t)(tl.y0 + r + 1) * j.apitch + (tl.x0 + c + 1)) * (F * OB) +
                   grp * 16;
    u32x4 pk;
    if constexpr (OUT_FMT == FMT_F32) {
#pragma unroll
      for (int e = 0; e < 4; ++e) pk[e] = __float_as_uint(v[e]);
    } else if constexpr (OUT_FMT == FMT_BF16) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pk[e] = (uint32_t)f32_to_bf16(v[2 * e]) | ((uint32_t)f32_to_bf16(v[2 * e + 1]) << 16);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pk[e] = (uint32_t)f32_to_e4m3(v[4 * e] * a.out_inv_scale) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 1] * a.out_inv_scale) << 8) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 2] * a.out_inv_scale) << 16) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 3] * a.out_inv_scale) << 24);
    }
    *reinterpret_cast<u32x4 *>(dst) = pk;
  }
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
  const TileRef tl = a.tiles[blockIdx.x];
  const JobDesc &j = a.jobs[tl.job];
  const uint8_t *in = reinterpret_cast<const uint8_t *>(j.act[a.in_slot]);
  const int ch = threadIdx.x % NCH;
  float w[EPC][9];
#pragma unroll
  for (int e = 0; e < EPC; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) w[e][k] = a.wf32[(ch * EPC + e) * 9 + k];
  const int IH = tl.h + 2, WW = tl.w + 2, NQ = IH * WW * NCH;
  for (int q0 = 0; q0 < NQ; q0 += 256) {     // uniform trip count: all lanes exchange
    const int q = q0 + threadIdx.x;
    const bool ok = q < NQ;
    const int pix = q / NCH, row = pix / WW, col = pix % WW;
    float v[8], v8 = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = 0.0f;
    if (ok) {
      float xv[EPC];
      decode16<IN_FMT>(*reinterpret_cast<const u32x4 *>(
                           in + ((int64_t)(tl.y0 + row) * j.apitch + (tl.x0 + col)) * PIXB +
                           ch * 16), xv);
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
  __syncthreads();
  const float sc = a.oscale[0], bi = a.bias[0];
  const int npix = (int)tl.h * tl.w;
  for (int pix = threadIdx.x; pix < npix; pix += 256) {
    const int r = pix / tl.w, c = pix % tl.w;
    float acc = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc += sp[tap][(r + tap / 3) * IW + c + tap % 3];
    j.G[(int64_t)(tl.y0 + r) * j.nx + tl.x0 + c] = acc * sc + bi;
  }
}

// single 1 -> 1 layer (K = 1): reads x^(t) (FP32), writes G
__global__ __launch_bounds__(256) void conv_single_kernel(ConvArgs a) {
  const TileRef tl = a.tiles[blockIdx.x];
  const JobDesc &j = a.jobs[tl.job];
  const int64_t t = a.tick + j.t_offset;
  const float *xb = j.x[t & 1];
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
    j.G[(int64_t)Y * j.nx + X] = acc * a.oscale[0] + a.bias[0];
  }
}

// ---------------------------------------------------------------------
// Middle layers: F -> F on MFMA.
// ---------------------------------------------------------------------
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
  static constexpr int OUT_BYTES = PNP_MID_STAGE ? TH * TW * OSTR : 0;
  static constexpr int TILE_BYTES = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
  static constexpr int LDS_BYTES = TILE_BYTES + C::WBYTES;
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

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;

  // contiguous tile ranges per XCD (workgroups are dispatched round-robin
  // over the 8 XCDs): neighbouring tiles share their halo rows in one L2
  const int nwg = gridDim.x, b = blockIdx.x;
#if PNP_XCD_MAP
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);
#else
  const int slot = b, per_xcd = nwg, t_begin = 0, t_end = a.n_tiles;
#endif

  auto load_weights = [&](int chunk) {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(
        reinterpret_cast<const uint8_t *>(a.wblob) + (size_t)chunk * C::WBYTES);
    u32x4 *dst = reinterpret_cast<u32x4 *>(lds_w);
    for (int i = tid; i < C::WBYTES / 16; i += NT) dst[i] = src[i];
  };

  u32x4 pre[NLOAD];
  auto issue_loads = [&](int ti) {
    const TileRef tl = a.tiles[ti];
    const JobDesc &j = a.jobs[tl.job];
    const uint8_t *in = reinterpret_cast<const uint8_t *>(j.act[a.in_slot]);
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q = tid + i * NT;
      if (q < NCHUNK) {
        const int pix = q / C::CPP, c = q % C::CPP;
        const int row = pix / IW, col = pix % IW;
        pre[i] = *reinterpret_cast<const u32x4 *>(
            in + ((int64_t)(tl.y0 + row) * j.apitch + (tl.x0 + col)) * C::PIXB + c * 16);
      }
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
  int ti = t_begin + slot;
  if (ti < t_end) issue_loads(ti);

  while (ti < t_end) {
    __syncthreads();          // previous tile's output staging has been read
    store_lds();
    __syncthreads();
    const TileRef tl = a.tiles[ti];
    const int tn = ti + per_xcd;
    if (tn < t_end) issue_loads(tn);  // overlaps with the MFMA work below

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
#if PNP_MID_PIPE
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
#else
#pragma unroll 1
      for (int sl = 0; sl < C::STEPS_PER_CH; ++sl) {
        AT A0[MB], B0[4];
        load_step(ch * C::STEPS_PER_CH + sl, sl, A0, B0);
        mma_step(A0, B0, acc);
      }
#endif
    }

#if PNP_MID_STAGE
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
        const f32x4 osc = *reinterpret_cast<const f32x4 *>(a.oscale + mb * 16 + 4 * g);
        const f32x4 bia = *reinterpret_cast<const f32x4 *>(a.bias + mb * 16 + 4 * g);
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
      const JobDesc &j = a.jobs[tl.job];
      uint8_t *out = reinterpret_cast<uint8_t *>(j.act[a.out_slot]);
      constexpr int CPPO = Lo::OPIXB / 16;
      constexpr int NQ = TH * kConvTileW * CPPO;
#pragma unroll
      for (int q0 = 0; q0 < NQ; q0 += NT) {
        const int q = q0 + tid;
        const int pix = q / CPPO, c16 = q % CPPO;
        const int r = pix / kConvTileW, c = pix % kConvTileW;
        if (q < NQ && r < tl.h && c < tl.w)
          *reinterpret_cast<u32x4 *>(out + ((int64_t)(tl.y0 + r + 1) * j.apitch +
                                            (tl.x0 + c + 1)) * Lo::OPIXB + c16 * 16) =
              *reinterpret_cast<const u32x4 *>(lds_in + pix * Lo::OSTR + c16 * 16);
      }
    }
#else
    // epilogue: scale, bias, ReLU, round to the next layer's format, store
    // 4 consecutive channels of one pixel per lane
    {
      const JobDesc &j = a.jobs[tl.job];
      uint8_t *out = reinterpret_cast<uint8_t *>(j.act[a.out_slot]);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int r = 2 * wave + (nb >> 1), c = (nb & 1) * 16 + l16;
        if (r < tl.h && c < tl.w) {
          uint8_t *dst = out + ((int64_t)(tl.y0 + r + 1) * j.apitch + (tl.x0 + c + 1)) * Lo::OPIXB;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const f32x4 osc = *reinterpret_cast<const f32x4 *>(a.oscale + mb * 16 + 4 * g);
            const f32x4 bia = *reinterpret_cast<const f32x4 *>(a.bias + mb * 16 + 4 * g);
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
      }
    }
#endif
    ti = tn;
  }
}

// ---------------------------------------------------------------------
// Middle layers, register-resident weights (bf16 and e4m3, F = 64).
// Every wave keeps the whole layer's A fragments in registers (bf16: 288
// VGPRs, e4m3: 160), so LDS serves only the activations: half the LDS
// traffic of the LDS-resident-weight kernel.  One wave per SIMD; input
// tiles (8 x 32 output pixels) are double-buffered in LDS with one barrier
// per tile; each wave stages its own outputs in a private LDS region and
// stores whole pixels with 16-byte lanes.
// ---------------------------------------------------------------------
template <int IN_FMT, int OUT_FMT>
struct RwLayout {
  using C = MidCfg<IN_FMT, 64>;
  static constexpr int NW = 4, TH = 8, TW = kConvTileW;
  static constexpr int IH = TH + 2, IW = TW + 2;
  static constexpr int OB = FmtInfo<OUT_FMT>::bytes;
  static constexpr int OPIXB = 64 * OB;
  static constexpr int OSTR = OPIXB + 16;
  static constexpr int IN_BYTES = IH * IW * C::PSTR;
  static constexpr int STAGE_BYTES = 64 * OSTR;          // per wave
  static constexpr int LDS_BYTES = 2 * IN_BYTES + NW * STAGE_BYTES;
};

template <int IN_FMT, int OUT_FMT>
__global__ __launch_bounds__(256, 1) void conv_mid_rw_kernel(ConvArgs a) {
  using C = MidCfg<IN_FMT, 64>;
  using Lo = RwLayout<IN_FMT, OUT_FMT>;
  constexpr int IW = Lo::IW, NT = 256, MB = 4;
  constexpr int NCHUNK = Lo::IH * IW * C::CPP;
  constexpr int NLOAD = (NCHUNK + NT - 1) / NT;
  constexpr int NSTEP = C::NSTEP;
  constexpr int OB = Lo::OB;
  using AT = typename std::conditional<IN_FMT == FMT_BF16, bf16x8, i32x8>::type;

  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  uint8_t *stage = lds + 2 * Lo::IN_BYTES + wave * Lo::STAGE_BYTES;

  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  // the layer's weights, fragment order, into registers
  AT W[NSTEP][MB];
  {
    const uint8_t *wb = reinterpret_cast<const uint8_t *>(a.wblob) + lane * C::FRAGB;
#pragma unroll
    for (int st = 0; st < NSTEP; ++st)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        W[st][mb] = *reinterpret_cast<const AT *>(wb + (size_t)(st * MB + mb) * 64 * C::FRAGB);
  }

  u32x4 pre[NLOAD];
  auto issue_loads = [&](int ti) {
    const TileRef tl = a.tiles[ti];
    const JobDesc &j = a.jobs[tl.job];
    const uint8_t *in = reinterpret_cast<const uint8_t *>(j.act[a.in_slot]);
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q = tid + i * NT;
      if (q < NCHUNK) {
        const int pix = q / C::CPP, c = q % C::CPP;
        const int row = pix / IW, col = pix % IW;
        pre[i] = *reinterpret_cast<const u32x4 *>(
            in + ((int64_t)(tl.y0 + row) * j.apitch + (tl.x0 + col)) * C::PIXB + c * 16);
      }
    }
  };
  auto store_lds = [&](uint8_t *buf) {
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
      const int q = tid + i * NT;
      if (q < NCHUNK) {
        const int pix = q / C::CPP, c = q % C::CPP;
        *reinterpret_cast<u32x4 *>(buf + pix * C::PSTR + c * 16) = pre[i];
      }
    }
  };
  auto load_b = [&](const uint8_t *buf, int step, AT (&B)[4]) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      if constexpr (IN_FMT == FMT_BF16) {
        const int tap = step / 2, half = step % 2;
        const int pix = (2 * wave + (nb >> 1) + tap / 3) * IW + (nb & 1) * 16 + l16 + tap % 3;
        B[nb] = *reinterpret_cast<const bf16x8 *>(buf + pix * C::PSTR + (half * 4 + g) * 16);
      } else {
        const int tap_raw = 2 * step + (g >> 1);
        const int tap = tap_raw > 8 ? 8 : tap_raw;
        const int pix = (2 * wave + (nb >> 1) + tap / 3) * IW + (nb & 1) * 16 + l16 + tap % 3;
        const uint8_t *src = buf + pix * C::PSTR + (g & 1) * 32;
        const u32x4 lo = *reinterpret_cast<const u32x4 *>(src);
        const u32x4 hi = *reinterpret_cast<const u32x4 *>(src + 16);
        B[nb] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
    }
  };
  auto mma = [&](const AT (&A)[MB], const AT (&B)[4], f32x4 (&acc)[MB][4]) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        if constexpr (IN_FMT == FMT_BF16)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mb], B[nb], acc[mb][nb], 0, 0, 0);
        else
          acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              A[mb], B[nb], acc[mb][nb], 0, 0, 0, 0, 0, 0);
      }
  };

  int ti = t_begin + slot;
  int cur = 0;
  if (ti < t_end) {
    issue_loads(ti);
    store_lds(lds);
  }
  int tn = ti + per_xcd;
  if (tn < t_end) issue_loads(tn);

  while (ti < t_end) {
    __syncthreads();   // tile ti is in buffer cur; everyone is done with buffer cur^1
    uint8_t *buf = lds + cur * Lo::IN_BYTES;
    const int tnn = tn + per_xcd;
    if (tn < t_end) {
      store_lds(lds + (cur ^ 1) * Lo::IN_BYTES);
      if (tnn < t_end) issue_loads(tnn);
    }
    const TileRef tl = a.tiles[ti];

    f32x4 acc[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    AT B0[4], B1[4];
    load_b(buf, 0, B0);
#pragma unroll
    for (int st = 0; st < NSTEP; st += 2) {
      if (st + 1 < NSTEP) load_b(buf, st + 1, B1);
      mma(W[st], B0, acc);
      if (st + 1 < NSTEP) {
        if (st + 2 < NSTEP) load_b(buf, st + 2, B0);
        mma(W[st + 1], B1, acc);
      }
    }

    // epilogue: this wave's 64 pixels, staged privately, stored whole
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      uint8_t *dst = stage + (nb * 16 + l16) * Lo::OSTR;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const f32x4 osc = *reinterpret_cast<const f32x4 *>(a.oscale + mb * 16 + 4 * g);
        const f32x4 bia = *reinterpret_cast<const f32x4 *>(a.bias + mb * 16 + 4 * g);
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
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      const JobDesc &j = a.jobs[tl.job];
      uint8_t *out = reinterpret_cast<uint8_t *>(j.act[a.out_slot]);
      constexpr int CPPO = Lo::OPIXB / 16;
#pragma unroll
      for (int q0 = 0; q0 < 64 * CPPO; q0 += 64) {
        const int q = q0 + lane;
        const int p = q / CPPO, c16 = q % CPPO;           // p = nb * 16 + pixel in block
        const int r = 2 * wave + (p >> 5), c = p & 31;
        if (r < tl.h && c < tl.w)
          *reinterpret_cast<u32x4 *>(out + ((int64_t)(tl.y0 + r + 1) * j.apitch +
                                            (tl.x0 + c + 1)) * Lo::OPIXB + c16 * 16) =
              *reinterpret_cast<const u32x4 *>(stage + p * Lo::OSTR + c16 * 16);
      }
    }
    ti = tn;
    tn = tnn;
    cur ^= 1;
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

template <int IN_FMT, int OUT_FMT>
static hipError_t launch_rw_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  const size_t lds = RwLayout<IN_FMT, OUT_FMT>::LDS_BYTES;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&conv_mid_rw_kernel<IN_FMT, OUT_FMT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((conv_mid_rw_kernel<IN_FMT, OUT_FMT>), dim3(n_wg), dim3(256), lds, s, a);
  return hipGetLastError();
}

// bf16 / e4m3 with F = 64 use the register-resident-weight kernel
static bool use_rw(int in_fmt, int F) { return PNP_USE_RW && in_fmt != FMT_F32 && F == 64; }

// tile rows of the middle-layer kernel for an input format
int mid_tile_rows(int in_fmt) {
  if (in_fmt == FMT_F32 || PNP_USE_RW) return 8;
  return 2 * PNP_NW_LOWP;
}

size_t mid_lds_bytes(int in_fmt, int F) {
  if (use_rw(in_fmt, F))
    return in_fmt == FMT_BF16 ? RwLayout<FMT_BF16, FMT_BF16>::LDS_BYTES
                              : RwLayout<FMT_E4M3, FMT_BF16>::LDS_BYTES;
  const int TH = mid_tile_rows(in_fmt);
  const int ib = in_fmt == FMT_F32 ? 4 : (in_fmt == FMT_BF16 ? 2 : 1);
  const int ob = in_fmt == FMT_E4M3 ? 2 : ib;          // widest output format
  const int pstr = F * ib + 16, ostr = PNP_MID_STAGE ? F * ob + 16 : 0;
  int nstep = in_fmt == FMT_E4M3 ? 5 : 9 * (in_fmt == FMT_F32 ? F / 16 : F / 32);
  int nch = (in_fmt == FMT_F32 && F == 64) ? 3 : 1;
  int fragb = in_fmt == FMT_E4M3 ? 32 : 16;
  const size_t in_b = (size_t)(TH + 2) * (kConvTileW + 2) * pstr;
  const size_t out_b = (size_t)TH * kConvTileW * ostr;
  return std::max(in_b, out_b) + (size_t)(nstep / nch) * (F / 16) * 64 * fragb;
}

hipError_t launch_conv_mid(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_wg,
                           hipStream_t s) {
  if (use_rw(in_fmt, F)) {
    if (in_fmt == FMT_BF16 && out_fmt == FMT_BF16) return launch_rw_t<FMT_BF16, FMT_BF16>(a, n_wg, s);
    if (in_fmt == FMT_E4M3 && out_fmt == FMT_E4M3) return launch_rw_t<FMT_E4M3, FMT_E4M3>(a, n_wg, s);
    if (in_fmt == FMT_E4M3 && out_fmt == FMT_BF16) return launch_rw_t<FMT_E4M3, FMT_BF16>(a, n_wg, s);
  }
  if (in_fmt == FMT_F32 && out_fmt == FMT_F32) {
    if (F == 16) return launch_mid_t<FMT_F32, FMT_F32, 16, 4>(a, n_wg, s);
    if (F == 32) return launch_mid_t<FMT_F32, FMT_F32, 32, 4>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_F32, FMT_F32, 64, 4>(a, n_wg, s);
  } else if (in_fmt == FMT_BF16 && out_fmt == FMT_BF16) {
    if (F == 32) return launch_mid_t<FMT_BF16, FMT_BF16, 32, PNP_NW_LOWP>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_BF16, FMT_BF16, 64, PNP_NW_LOWP>(a, n_wg, s);
  } else if (in_fmt == FMT_E4M3 && F == 64) {
    if (out_fmt == FMT_E4M3) return launch_mid_t<FMT_E4M3, FMT_E4M3, 64, PNP_NW_LOWP>(a, n_wg, s);
    if (out_fmt == FMT_BF16) return launch_mid_t<FMT_E4M3, FMT_BF16, 64, PNP_NW_LOWP>(a, n_wg, s);
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
  LAST(FMT_F32, 16) LAST(FMT_F32, 32) LAST(FMT_F32, 64) LAST(FMT_BF16, 32) LAST(FMT_BF16, 64)
#undef LAST
  return hipErrorInvalidValue;
}

hipError_t launch_conv_single(const ConvArgs &a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL(conv_single_kernel, dim3(n_tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pnp
