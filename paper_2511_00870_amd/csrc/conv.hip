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
#include "device_common.h"
#include "kernels.h"

namespace pnp {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;

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
    uint4 pk;
    uint32_t *pw = reinterpret_cast<uint32_t *>(&pk);
    if constexpr (OUT_FMT == FMT_F32) {
#pragma unroll
      for (int e = 0; e < 4; ++e) pw[e] = __float_as_uint(v[e]);
    } else if constexpr (OUT_FMT == FMT_BF16) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pw[e] = (uint32_t)f32_to_bf16(v[2 * e]) | ((uint32_t)f32_to_bf16(v[2 * e + 1]) << 16);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        pw[e] = (uint32_t)f32_to_e4m3(v[4 * e] * a.out_inv_scale) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 1] * a.out_inv_scale) << 8) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 2] * a.out_inv_scale) << 16) |
                ((uint32_t)f32_to_e4m3(v[4 * e + 3] * a.out_inv_scale) << 24);
    }
    *reinterpret_cast<uint4 *>(dst) = pk;
  }
}

// ---------------------------------------------------------------------
// Last layer: F -> 1 (no activation); writes G (FP32, compact).  Each lane
// owns one 16-byte chunk of input channels of a pixel (its weights in
// registers); the lanes of a pixel are adjacent and their partial sums are
// combined with cross-lane shuffles.
// ---------------------------------------------------------------------
template <int FMT> __device__ __forceinline__ void decode16(uint4 raw, float *v);
template <> __device__ __forceinline__ void decode16<FMT_F32>(uint4 raw, float *v) {
  v[0] = __uint_as_float(raw.x); v[1] = __uint_as_float(raw.y);
  v[2] = __uint_as_float(raw.z); v[3] = __uint_as_float(raw.w);
}
template <> __device__ __forceinline__ void decode16<FMT_BF16>(uint4 raw, float *v) {
  const uint32_t u[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[2 * e] = __uint_as_float(u[e] << 16);
    v[2 * e + 1] = __uint_as_float(u[e] & 0xffff0000u);
  }
}
template <> __device__ __forceinline__ void decode16<FMT_E4M3>(uint4 raw, float *v) {
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
  constexpr int NCH = PIXB / 16;               // lanes per pixel
  constexpr int EPC = 16 / IB;                 // channels per lane
  constexpr int PPP = 256 / NCH;
  const TileRef tl = a.tiles[blockIdx.x];
  const JobDesc &j = a.jobs[tl.job];
  const uint8_t *in = reinterpret_cast<const uint8_t *>(j.act[a.in_slot]);
  const int ch = threadIdx.x % NCH, slot = threadIdx.x / NCH;
  float w[EPC][9];
#pragma unroll
  for (int e = 0; e < EPC; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) w[e][k] = a.wf32[(ch * EPC + e) * 9 + k];
  const float sc = a.oscale[0], bi = a.bias[0];
  const int npix = (int)tl.h * tl.w;
  for (int pix = slot; pix < npix; pix += PPP) {
    const int r = pix / tl.w, c = pix % tl.w;
    const int Y = tl.y0 + r, X = tl.x0 + c;
    float acc = 0.0f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const uint8_t *src =
          in + ((int64_t)(Y + tap / 3) * j.apitch + (X + tap % 3)) * PIXB + ch * 16;
      float v[EPC];
      decode16<IN_FMT>(*reinterpret_cast<const uint4 *>(src), v);
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc = fmaf(w[e][tap], v[e], acc);
    }
#pragma unroll
    for (int off = NCH / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (ch == 0) j.G[(int64_t)Y * j.nx + X] = acc * sc + bi;
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
__global__ __launch_bounds__(NW * 64) void conv_mid_kernel(ConvArgs a) {
  using C = MidCfg<IN_FMT, F>;
  constexpr int TH = 2 * NW, TW = kConvTileW;
  constexpr int IH = TH + 2, IW = TW + 2;
  constexpr int NT = NW * 64;
  constexpr int NCHUNK = IH * IW * C::CPP;
  constexpr int NLOAD = (NCHUNK + NT - 1) / NT;
  constexpr int OB = FmtInfo<OUT_FMT>::bytes;
  constexpr int MB = C::MB;

  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t *lds_in = lds;
  uint8_t *lds_w = lds + IH * IW * C::PSTR;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;

  // contiguous tile ranges per XCD (workgroups are dispatched round-robin
  // over the 8 XCDs): neighbouring tiles share their halo rows in one L2
  const int nwg = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per_xcd = (nwg - xcd + 7) >> 3;
  const int t_begin = (int)(((int64_t)a.n_tiles * xcd) >> 3);
  const int t_end = (int)(((int64_t)a.n_tiles * (xcd + 1)) >> 3);

  // per-lane epilogue constants: 4 consecutive output channels per M block
  f32x4 osc[MB], bia[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    osc[mb] = *reinterpret_cast<const f32x4 *>(a.oscale + mb * 16 + 4 * g);
    bia[mb] = *reinterpret_cast<const f32x4 *>(a.bias + mb * 16 + 4 * g);
  }

  auto load_weights = [&](int chunk) {
    const uint4 *src = reinterpret_cast<const uint4 *>(
        reinterpret_cast<const uint8_t *>(a.wblob) + (size_t)chunk * C::WBYTES);
    uint4 *dst = reinterpret_cast<uint4 *>(lds_w);
    for (int i = tid; i < C::WBYTES / 16; i += NT) dst[i] = src[i];
  };

  uint4 pre[NLOAD];
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
        pre[i] = *reinterpret_cast<const uint4 *>(
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
        *reinterpret_cast<uint4 *>(lds_in + pix * C::PSTR + c * 16) = pre[i];
      }
    }
  };

  if (C::NCH == 1) load_weights(0);
  int ti = t_begin + slot;
  if (ti < t_end) issue_loads(ti);

  while (ti < t_end) {
    __syncthreads();          // previous tile's LDS reads are done
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

    // pixel of N block nb for this lane, relative to the input tile origin
    auto in_pix = [&](int nb, int tap) {
      const int dy = tap / 3, dx = tap % 3;
      return (2 * wave + (nb >> 1) + dy) * IW + (nb & 1) * 16 + l16 + dx;
    };

#pragma unroll 1
    for (int ch = 0; ch < C::NCH; ++ch) {
      if (C::NCH > 1) {
        __syncthreads();
        load_weights(ch);
        __syncthreads();
      }
#pragma unroll 1
      for (int sl = 0; sl < C::STEPS_PER_CH; ++sl) {
        const int step = ch * C::STEPS_PER_CH + sl;
        const uint8_t *wf = lds_w + (size_t)sl * MB * 64 * C::FRAGB + lane * C::FRAGB;
        if constexpr (IN_FMT == FMT_BF16) {
          const int tap = step / (F / 32), half = step % (F / 32);
          bf16x8 A[MB], B[4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            A[mb] = *reinterpret_cast<const bf16x8 *>(wf + mb * 64 * 16);
#pragma unroll
          for (int nb = 0; nb < 4; ++nb)
            B[nb] = *reinterpret_cast<const bf16x8 *>(lds_in + in_pix(nb, tap) * C::PSTR +
                                                       (half * 4 + g) * 16);
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mb], B[nb], acc[mb][nb],
                                                                    0, 0, 0);
        } else if constexpr (IN_FMT == FMT_F32) {
          const int tap = step / (F / 16), ss = step % (F / 16);
          f32x4 A[MB], B[4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            A[mb] = *reinterpret_cast<const f32x4 *>(wf + mb * 64 * 16);
#pragma unroll
          for (int nb = 0; nb < 4; ++nb)
            B[nb] = *reinterpret_cast<const f32x4 *>(lds_in + in_pix(nb, tap) * C::PSTR +
                                                      (ss * 4 + g) * 16);
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
              for (int nb = 0; nb < 4; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mb][e], B[nb][e],
                                                                   acc[mb][nb], 0, 0, 0);
        } else {  // E4M3: step covers taps 2*step (lane groups 0,1) and 2*step+1 (2,3)
          const int tap_raw = 2 * step + (g >> 1);
          const int tap = tap_raw > 8 ? 8 : tap_raw;   // zero-weight slot reads tap 8
          i32x8 A[MB], B[4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            A[mb] = *reinterpret_cast<const i32x8 *>(wf + mb * 64 * 32);
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            const uint8_t *src = lds_in + in_pix(nb, tap) * C::PSTR + (g & 1) * 32;
            const uint4 lo = *reinterpret_cast<const uint4 *>(src);
            const uint4 hi = *reinterpret_cast<const uint4 *>(src + 16);
            B[nb] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                          (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
          }
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                  A[mb], B[nb], acc[mb][nb], 0, 0, 0, 0, 0, 0);
        }
      }
    }

    // epilogue: scale, bias, ReLU, round to the next layer's format, store
    const JobDesc &j = a.jobs[tl.job];
    uint8_t *out = reinterpret_cast<uint8_t *>(j.act[a.out_slot]);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int r = 2 * wave + (nb >> 1), c = (nb & 1) * 16 + l16;
      if (r < tl.h && c < tl.w) {
        uint8_t *dst = out + ((int64_t)(tl.y0 + r + 1) * j.apitch + (tl.x0 + c + 1)) * (F * OB);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          f32x4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float o = acc[mb][nb][e] * osc[mb][e] + bia[mb][e];
            if (a.relu) o = fmaxf(o, 0.0f);
            v[e] = o;
          }
          store4<OUT_FMT>(dst + (mb * 16 + 4 * g) * OB, v, a.out_inv_scale);
        }
      }
    }
    ti = tn;
  }
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
template <int IN_FMT, int OUT_FMT, int F, int NW>
static hipError_t launch_mid_t(const ConvArgs &a, int n_wg, hipStream_t s) {
  using C = MidCfg<IN_FMT, F>;
  constexpr int TH = 2 * NW;
  const size_t lds = (size_t)(TH + 2) * (kConvTileW + 2) * C::PSTR + C::WBYTES;
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

int mid_tile_rows(int in_fmt) { return in_fmt == FMT_F32 ? 8 : 16; }

size_t mid_lds_bytes(int in_fmt, int F) {
  const int TH = mid_tile_rows(in_fmt);
  const int ib = in_fmt == FMT_F32 ? 4 : (in_fmt == FMT_BF16 ? 2 : 1);
  const int pstr = F * ib + 16;
  int nstep = in_fmt == FMT_E4M3 ? 5 : 9 * (in_fmt == FMT_F32 ? F / 16 : F / 32);
  int nch = (in_fmt == FMT_F32 && F == 64) ? 3 : 1;
  int fragb = in_fmt == FMT_E4M3 ? 32 : 16;
  return (size_t)(TH + 2) * (kConvTileW + 2) * pstr + (size_t)(nstep / nch) * (F / 16) * 64 * fragb;
}

hipError_t launch_conv_mid(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_wg,
                           hipStream_t s) {
  if (in_fmt == FMT_F32 && out_fmt == FMT_F32) {
    if (F == 16) return launch_mid_t<FMT_F32, FMT_F32, 16, 4>(a, n_wg, s);
    if (F == 32) return launch_mid_t<FMT_F32, FMT_F32, 32, 4>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_F32, FMT_F32, 64, 4>(a, n_wg, s);
  } else if (in_fmt == FMT_BF16 && out_fmt == FMT_BF16) {
    if (F == 32) return launch_mid_t<FMT_BF16, FMT_BF16, 32, 8>(a, n_wg, s);
    if (F == 64) return launch_mid_t<FMT_BF16, FMT_BF16, 64, 8>(a, n_wg, s);
  } else if (in_fmt == FMT_E4M3 && F == 64) {
    if (out_fmt == FMT_E4M3) return launch_mid_t<FMT_E4M3, FMT_E4M3, 64, 8>(a, n_wg, s);
    if (out_fmt == FMT_BF16) return launch_mid_t<FMT_E4M3, FMT_BF16, 64, 8>(a, n_wg, s);
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
#define LAST(I, FF)                                                                     \
  if (in_fmt == I && F == FF) {                                                         \
    hipLaunchKernelGGL((conv_last_kernel<I, FF>), dim3(n_tiles), dim3(256), 0, s, a);  \
    return hipGetLastError();                                                           \
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
