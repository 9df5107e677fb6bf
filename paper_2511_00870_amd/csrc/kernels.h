// kernels.h -- launch interface of the gfx950 kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.h"

namespace pnp {

struct ConvArgs {
  const JobDesc *jobs;
  const TileRef *tiles;
  int32_t n_tiles;
  int32_t in_slot, out_slot;   // activation ping-pong slots read / written
  int32_t relu;
  int32_t tile_rows;           // rows of the conv tiles (<= 16)
  int32_t unit_scale;          // every output scale is 1
  int64_t tick;
  const void *wblob;           // middle layers: weights in MFMA fragment order
  const void *wblob_rr;        // e4m3 middle layers: row-reuse fragment order
  const float *wf32;           // first / last layer: quantised weights [c][9]
  const float *bias;           // [c_out]
  const float *oscale;         // [c_out]: weight scale x input scale
  float in_inv_scale;          // first layer: 1 / scale of its input format
  float out_inv_scale;         // 1 / scale of the next layer's input (e4m3), else 1
  // first layer fused into the first middle layer: its weights [c][9], bias,
  // output scales and 1 / next layer's input scale (the last two: e4m3 pairs)
  const float *first_w;
  const float *first_bias;
  const float *first_oscale;
  float first_out_inv_scale;
  // last layer fused into the last middle layer: its weights [c][9]
  const float *last_w;
  // second layer of a fused pair of middle layers: weights (fragment order;
  // e4m3: row-reuse order), bias, output scales, 1 / next layer's input scale
  const void *wblob2;
  const float *bias2;
  const float *oscale2;
  float out_inv_scale2;
};

// one stage of the DDFB denoiser (stage k = 1 .. K writes b_k, or G at K)
struct DdfbArgs {
  const JobDesc *jobs;
  const TileRef *tiles;        // kDdTile x kDdTile tiles over the whole image
  int32_t n_tiles;
  int32_t stage, K, F;
  int64_t tick;
  const float *w;              // K blocks of [F][3][3]: W_k maps 1 -> F channels
  float thresh;                // hard-tanh level
  float gamma[kMaxDdfbLayers]; // step sizes gamma_1 .. gamma_K
};

// large blur: one correlation of an image with an L x L kernel per output
// tile (the update tiles); epi selects input and epilogue
enum BlurEpi : int {
  EPI_RESIDUAL = 0,  // input x^(t), kernel flipped: residual m (K x - v) into JobDesc::res
  EPI_GRAD = 1,      // input JobDesc::res, kernel as is: K^T res / s2 into JobDesc::gdat
  EPI_KX = 2         // input x^(t), kernel flipped: K x into JobDesc::res (z-step)
};
struct BlurArgs {
  const JobDesc *jobs;
  const TileRef *tiles;
  int32_t n_tiles;
  int32_t epi;
  int64_t tick;
};

// data-fidelity gradient of a given image (compact ny x nx buffers)
struct GradArgs {
  const JobDesc *jobs;
  const TileRef *tiles;        // the job's update tiles
  int32_t n_tiles;
  int32_t epi;                 // 0: res = m (K x - y); 1: g = K^T res / sigma^2
  const float *x;
  float *res;
  float *g;
};

struct UpdateArgs {
  const JobDesc *jobs;
  const TileRef *tiles;
  int32_t n_tiles;
  int32_t pad;
  int64_t tick;
};

// convolution tile height of the middle-layer kernel for an input format
int mid_tile_rows(int in_fmt);
size_t mid_lds_bytes(int in_fmt, int F);
size_t update_lds_bytes(int r);

// first layer (1 -> 64, bf16) and first middle layer in one kernel; a holds the
// middle layer's arguments plus first_w / first_bias
hipError_t launch_conv_first_mid(const ConvArgs &a, int n_wg, hipStream_t s);
// middle layer whose output feeds the last layer directly: writes the last
// layer's per-tap partials (JobDesc::S) instead of its activations (first
// must be false: a middle layer with both fusions is not built)
hipError_t launch_conv_mid_last(const ConvArgs &a, int n_wg, bool first, hipStream_t s);
// G = sum over taps of the partials at the tap's neighbour, plus the bias
// two consecutive bf16 middle layers in one kernel, the two layers on
// separate waves (a: the first layer's arguments plus wblob2 / bias2; 8
// waves per workgroup; tiles of kPairWsTileH x kPairTileW); n_wg a positive
// multiple of 8
hipError_t launch_conv_pair_ws(const ConvArgs &a, int n_wg, hipStream_t s);
bool pair_fusable(int in_fmt, int out_fmt, int F, int relu, int unit, int in_fmt2, int out_fmt2,
                  int relu2, int unit2);
// two consecutive e4m3 middle layers in one kernel (a: the first layer's
// arguments with wblob_rr; wblob2 / bias2 / oscale2 / out_inv_scale2 the
// second's); out_fmt2: the second layer's output format (e4m3 or bf16);
// n_wg a positive multiple of 8, pair8_wg_per_cu() per CU
// first (only together with last): the network's first layer (bf16 -> e4m3)
// runs inside the kernel from x (first_w / first_bias / first_oscale /
// first_out_inv_scale)
// last: the second layer feeds the last layer, whose per-tap partials go to
// JobDesc::S (last_w; out_fmt2 must be bf16)
hipError_t launch_conv_pair8(const ConvArgs &a, int out_fmt2, bool first, bool last, int n_wg,
                             hipStream_t s);
// two consecutive e4m3 middle layers on separate waves with the taps packed
// without zero slots (a: as for launch_conv_pair8, with wblob_rr / wblob2 the
// layers' sliding-pair weights; e4m3 output; 8 waves per workgroup, one
// workgroup per CU; tiles of kPair8WsTileH x kPairTileW); n_wg a positive
// multiple of 8
hipError_t launch_conv_pair8_ws(const ConvArgs &a, int n_wg, hipStream_t s);
// the network's first layer (1 -> 64, bf16 weights, e4m3 output into
// j.act[out_slot]) on the matrix cores with the e4m3 first-layer pair's
// arithmetic (first_w / first_bias / first_oscale / first_out_inv_scale);
// over convolution tiles of at most 16 rows; n_wg workgroups, a positive
// multiple of 8, each walking tiles of its XCD's range
hipError_t launch_conv_first8(const ConvArgs &a, int n_wg, hipStream_t s);
bool last_pair8_fusable(int out_fmt2, int last_in_fmt, int last_cin, int last_cout);
bool first_pair8_fusable(int in_fmt0, int out_fmt0, int cin0, int cout0, int relu0);
bool pair8_fusable(int in_fmt, int out_fmt, int F, int relu, int in_fmt2, int out_fmt2,
                   int relu2);
int pair8_wg_per_cu();
hipError_t launch_g_from_s(const ConvArgs &a, int n_tiles, hipStream_t s);
bool mid_last_fusable(int in_fmt, int out_fmt, int F, int relu, int unit, int last_in_fmt,
                      int last_cin, int last_cout);
bool first_mid_fusable(int in_fmt0, int out_fmt0, int cout0, int relu0, int unit0, int in_fmt1,
                       int out_fmt1, int F, int relu1, int unit1);
hipError_t launch_conv_mid(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_wg,
                           hipStream_t s);
hipError_t launch_conv_first(int in_fmt, int out_fmt, int F, const ConvArgs &a, int n_tiles,
                             hipStream_t s);
hipError_t launch_conv_last(int in_fmt, int F, const ConvArgs &a, int n_tiles, hipStream_t s);
hipError_t launch_conv_single(const ConvArgs &a, int n_tiles, hipStream_t s);
// uniform_r: every resident job's blur half-width equals max_r
// mode: 0 (y or the exact z draw in the residual) or 1 (PSGLA: z1 and z2 held
// as state); every resident job must have that mode
hipError_t launch_fused_update(const UpdateArgs &a, int n_tiles, int max_r, bool uniform_r,
                               int mode, hipStream_t s);
// update with a precomputed data gradient (JobDesc::gdat)
hipError_t launch_update_pointwise(const UpdateArgs &a, int n_tiles, hipStream_t s);
// PSGLA z-step (after the x-update; tick such that t is the new iterate's)
hipError_t launch_zstep_psgla(const UpdateArgs &a, int n_tiles, int max_r, hipStream_t s);
// TV prior term G = (1/rho) D^T (D x - z) at x^(t), and the TV z-step
hipError_t launch_tv_prior(const UpdateArgs &a, int n_tiles, hipStream_t s);
hipError_t launch_zstep_tv(const UpdateArgs &a, int n_tiles, hipStream_t s);
hipError_t launch_ddfb_stage(const DdfbArgs &a, int n_tiles, hipStream_t s);
// large blur (half-width max_r > kMaxR)
hipError_t launch_blur_big(const BlurArgs &a, int n_tiles, int max_r, int kpitch, hipStream_t s);
size_t blur_big_lds_bytes(int r, int kpitch);
hipError_t launch_data_grad(const GradArgs &a, int n_tiles, int r, int kpitch, hipStream_t s);
// the static residual buffer of the allocation-free data gradient: look up
// its address on `device` (current) once; then noalloc_scratch(device)
constexpr int64_t kNoallocMaxPixels = (int64_t)1 << 23;
hipError_t noalloc_scratch_init(int device);
float *noalloc_scratch(int device);
hipError_t launch_amax(const float *p, size_t n, uint32_t *out, hipStream_t s);
hipError_t launch_stats_out(const JobDesc &j, int64_t n, float *mean, float *var, hipStream_t s);
hipError_t launch_welford_flush(const JobDesc &j, double n_a, double n_b, hipStream_t s);

}  // namespace pnp
