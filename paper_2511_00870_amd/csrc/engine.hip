// engine.hip -- host runtime: device memory, weight repacking, block and
// tile plans, and the launch sequence of one PnP-ULA iteration.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace pnp {

#define HIPOK(expr)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return Status::fail(PNPULA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------
// host rounding helpers (used only to repack weights on the host)
// ---------------------------------------------------------------------
float host_round_bf16(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return v;
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

uint8_t host_f32_to_e4m3(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  const float a = std::fabs(v);
  if (a != a) return (uint8_t)(sign | 0x7f);
  if (a >= 448.0f) return (uint8_t)(sign | 0x7e);
  if (a < 0.015625f) return (uint8_t)(sign | (uint8_t)std::nearbyint(a * 512.0f));
  uint32_t b;
  std::memcpy(&b, &a, 4);
  b += 0x7ffffu + ((b >> 20) & 1u);
  return (uint8_t)(sign | ((((b >> 23) - 120u) & 15u) << 3) | ((b >> 20) & 7u));
}

float host_e4m3_to_f32(uint8_t c) {
  const uint32_t e = (c >> 3) & 15u, m = c & 7u;
  float v = (e == 0) ? (float)m * 0.001953125f : std::ldexp(1.0f + (float)m / 8.0f, (int)e - 7);
  return (c & 0x80) ? -v : v;
}

float host_pow2_scale(float amax) {
  if (!(amax > 0.0f)) return 1.0f;
  int e;
  const double f = std::frexp((double)amax / 448.0, &e);
  return (float)((f == 0.5) ? std::ldexp(1.0, e - 1) : std::ldexp(1.0, e));
}

bool host_is_pow2(float v) {
  if (!(v > 0.0f) || !std::isfinite(v)) return false;
  int e;
  return std::frexp(v, &e) == 0.5f;
}

static float quant_host(float v, int fmt) {
  if (fmt == FMT_BF16) return host_round_bf16(v);
  if (fmt == FMT_E4M3) return host_e4m3_to_f32(host_f32_to_e4m3(v));
  return v;
}

static int fmt_bytes(int fmt) { return fmt == FMT_F32 ? 4 : (fmt == FMT_BF16 ? 2 : 1); }

// ---------------------------------------------------------------------
// engine lifetime
// ---------------------------------------------------------------------
Engine::~Engine() {
  if (stream) hipStreamSynchronize(stream);
  for (Job *j : resident) free_job(j);
  resident.clear();
  for (void *p : net.allocs) hipFree(p);
  hipFree(d_jobs);
  hipFree(d_conv);
  hipFree(d_upd);
  hipFree(d_pair);
  hipFree(d_pair_ws);
  hipFree(d_pair8ws);
  hipFree(d_ddfb);
  for (auto &r : prof_pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : prof_free) hipEventDestroy(e);
  if (own_stream && stream) hipStreamDestroy(stream);
}

Status Engine::init(void *user_stream) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1)
    return Status::fail(PNPULA_EDEVICE, "no HIP device");
  HIPOK(hipGetDevice(&device));
  hipDeviceProp_t prop;
  HIPOK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return Status::fail(PNPULA_EDEVICE,
                        std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
  n_cu = prop.multiProcessorCount;
  HIPOK(noalloc_scratch_init(device));
  if (user_stream) {
    stream = reinterpret_cast<hipStream_t>(user_stream);
    own_stream = false;
  } else {
    HIPOK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    own_stream = true;
  }
  return Status::ok();
}

// ---------------------------------------------------------------------
// denoiser: formats, scales and weight repacking
// ---------------------------------------------------------------------
Status Engine::set_net(int K, const int32_t *ch, const float *w, const float *b, int precision,
                       const float *act_scales) {
  if (K < 1 || !ch || !w || !b) return Status::fail(PNPULA_EINVAL, "denoiser missing");
  if (ch[0] != 1 || ch[K] != 1) return Status::fail(PNPULA_EINVAL, "channels must start and end at 1");
  if (precision < PNPULA_FP32 || precision > PNPULA_FP8_E4M3)
    return Status::fail(PNPULA_EINVAL, "unknown precision");
  int F = K > 1 ? ch[1] : 1;
  for (int k = 1; k < K; ++k)
    if (ch[k] != F) return Status::fail(PNPULA_EINVAL, "inner channel counts must be equal");
  if (K > 1) {
    bool ok = (precision == PNPULA_FP32 && (F == 16 || F == 32 || F == 64)) ||
              (precision == PNPULA_BF16 && (F == 32 || F == 64)) ||
              (precision == PNPULA_FP8_E4M3 && F == 64);
    if (!ok) return Status::fail(PNPULA_EINVAL, "unsupported feature count for this precision");
  }
  if (precision == PNPULA_FP8_E4M3 && K < 3)
    return Status::fail(PNPULA_EINVAL, "e4m3 needs at least 3 layers (first and last are bf16)");
  net = NetPlan();
  net.K = K;
  net.F = F;
  net.precision = precision;
  net.channels.assign(ch, ch + K + 1);
  size_t nw = 0, nb = 0;
  for (int k = 0; k < K; ++k) {
    nw += (size_t)ch[k] * ch[k + 1] * 9;
    nb += (size_t)ch[k + 1];
  }
  net.weights.assign(w, w + nw);
  net.biases.assign(b, b + nb);
  for (size_t i = 0; i < nw; ++i)
    if (!std::isfinite(w[i])) return Status::fail(PNPULA_EINVAL, "non-finite weight");
  // per-layer formats
  std::vector<int> fmt(K);
  for (int k = 0; k < K; ++k) {
    if (precision == PNPULA_FP32) fmt[k] = FMT_F32;
    else if (precision == PNPULA_BF16) fmt[k] = FMT_BF16;
    else fmt[k] = (k == 0 || k == K - 1) ? FMT_BF16 : FMT_E4M3;
  }
  net.act_scales.assign(K, 1.0f);
  if (precision == PNPULA_FP8_E4M3) {
    if (!act_scales) return Status::fail(PNPULA_EINVAL, "e4m3 needs act_scales");
    for (int k = 0; k < K; ++k) {
      if (fmt[k] == FMT_E4M3 && !host_is_pow2(act_scales[k]))
        return Status::fail(PNPULA_EINVAL, "activation scales must be powers of two");
      net.act_scales[k] = fmt[k] == FMT_E4M3 ? act_scales[k] : 1.0f;
    }
  }
  size_t woff = 0, boff = 0;
  net.layers.resize(K);
  for (int k = 0; k < K; ++k) {
    LayerPlan &L = net.layers[k];
    L.cin = ch[k];
    L.cout = ch[k + 1];
    L.in_fmt = fmt[k];
    L.out_fmt = (k < K - 1) ? fmt[k + 1] : FMT_F32;
    L.relu = k < K - 1;
    L.in_scale = net.act_scales[k];
    L.in_inv_scale = 1.0f / net.act_scales[k];
    L.out_inv_scale = (k < K - 1) ? 1.0f / net.act_scales[k + 1] : 1.0f;
    // weight scales (power of two per output channel for e4m3) and rounding
    std::vector<float> sw(L.cout, 1.0f);
    const float *wk = w + woff;
    if (L.in_fmt == FMT_E4M3)
      for (int co = 0; co < L.cout; ++co) {
        float amax = 0.f;
        for (int i = 0; i < L.cin * 9; ++i) amax = std::max(amax, std::fabs(wk[co * L.cin * 9 + i]));
        sw[co] = host_pow2_scale(amax);
      }
    std::vector<float> wq((size_t)L.cout * L.cin * 9);
    for (int co = 0; co < L.cout; ++co)
      for (int i = 0; i < L.cin * 9; ++i)
        wq[(size_t)co * L.cin * 9 + i] = quant_host(wk[(size_t)co * L.cin * 9 + i] / sw[co], L.in_fmt);
    std::vector<float> osc(L.cout);
    for (int co = 0; co < L.cout; ++co) osc[co] = sw[co] * L.in_scale;
    L.unit_scale = std::all_of(osc.begin(), osc.end(), [](float v) { return v == 1.0f; });
    // device copies: bias and oscale padded to 16 floats for vector loads
    const int cpad = std::max(L.cout, 16);
    std::vector<float> bias(cpad, 0.f), oscp(cpad, 0.f);
    for (int co = 0; co < L.cout; ++co) {
      bias[co] = b[boff + co];
      oscp[co] = osc[co];
    }
    HIPOK(hipMalloc(&L.bias, cpad * sizeof(float)));
    net.allocs.push_back(L.bias);
    HIPOK(hipMalloc(&L.oscale, cpad * sizeof(float)));
    net.allocs.push_back(L.oscale);
    HIPOK(hipMemcpy(L.bias, bias.data(), cpad * sizeof(float), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(L.oscale, oscp.data(), cpad * sizeof(float), hipMemcpyHostToDevice));
    const bool mid = (k > 0 && k < K - 1);
    if (!mid) {
      // [c][9]: first layer c = c_out (c_in = 1); last layer c = c_in (c_out = 1)
      std::vector<float> f((size_t)std::max(L.cin, L.cout) * 9);
      for (int co = 0; co < L.cout; ++co)
        for (int ci = 0; ci < L.cin; ++ci)
          for (int tap = 0; tap < 9; ++tap)
            f[(size_t)(L.cin == 1 ? co : ci) * 9 + tap] = wq[((size_t)co * L.cin + ci) * 9 + tap];
      HIPOK(hipMalloc(&L.wf32, f.size() * sizeof(float)));
      net.allocs.push_back(L.wf32);
      HIPOK(hipMemcpy(L.wf32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
      const int MB = F / 16;
      auto W = [&](int co, int ci, int tap) { return wq[((size_t)co * F + ci) * 9 + tap]; };
      std::vector<uint8_t> blob;
      if (L.in_fmt == FMT_BF16) {
        const int nstep = 9 * (F / 32);
        blob.resize((size_t)nstep * MB * 64 * 16);
        for (int s = 0; s < nstep; ++s)
          for (int mb = 0; mb < MB; ++mb)
            for (int l = 0; l < 64; ++l)
              for (int e = 0; e < 8; ++e) {
                const int tap = s / (F / 32), half = s % (F / 32);
                const int co = mb * 16 + (l & 15), ci = half * 32 + (l >> 4) * 8 + e;
                float v = W(co, ci, tap);
                uint32_t u;
                std::memcpy(&u, &v, 4);
                const uint16_t hb = (uint16_t)(u >> 16);   // already bf16-rounded
                std::memcpy(&blob[(((size_t)s * MB + mb) * 64 + l) * 16 + e * 2], &hb, 2);
              }
      } else if (L.in_fmt == FMT_F32) {
        const int nstep = 9 * (F / 16);
        blob.resize((size_t)nstep * MB * 64 * 16);
        for (int s = 0; s < nstep; ++s)
          for (int mb = 0; mb < MB; ++mb)
            for (int l = 0; l < 64; ++l)
              for (int e = 0; e < 4; ++e) {
                const int tap = s / (F / 16), ss = s % (F / 16);
                const int co = mb * 16 + (l & 15), ci = ss * 16 + (l >> 4) * 4 + e;
                const float v = W(co, ci, tap);
                std::memcpy(&blob[(((size_t)s * MB + mb) * 64 + l) * 16 + e * 4], &v, 4);
              }
      } else {  // e4m3, F == 64: 5 steps of two taps
        blob.assign((size_t)5 * MB * 64 * 32, 0);
        for (int s = 0; s < 5; ++s)
          for (int mb = 0; mb < MB; ++mb)
            for (int l = 0; l < 64; ++l)
              for (int e = 0; e < 32; ++e) {
                const int g = l >> 4, tap = 2 * s + (g >> 1);
                if (tap > 8) continue;
                const int co = mb * 16 + (l & 15), ci = 32 * (g & 1) + e;
                blob[(((size_t)s * MB + mb) * 64 + l) * 32 + e] = host_f32_to_e4m3(W(co, ci, tap));
              }
      }
      HIPOK(hipMalloc(&L.wblob, blob.size()));
      net.allocs.push_back(L.wblob);
      HIPOK(hipMemcpy(L.wblob, blob.data(), blob.size(), hipMemcpyHostToDevice));
      if (L.in_fmt == FMT_E4M3) {
        // row-reuse kernel: step (P, dy) pairs the horizontal taps (dx 0, 1)
        // for P = 0 and (dx 2, none) for P = 1; lane groups 0-1 hold the first
        // tap's 64 channels, groups 2-3 the second's (zero for none)
        std::vector<uint8_t> rr((size_t)6 * MB * 64 * 32, 0);
        for (int P = 0; P < 2; ++P)
          for (int dy = 0; dy < 3; ++dy)
            for (int mb = 0; mb < MB; ++mb)
              for (int l = 0; l < 64; ++l) {
                const int g = l >> 4;
                const int dx = (g < 2) ? (P == 0 ? 0 : 2) : (P == 0 ? 1 : -1);
                if (dx < 0) continue;
                const int co = mb * 16 + (l & 15), tap = 3 * dy + dx;
                for (int e = 0; e < 32; ++e)
                  rr[((((size_t)P * 3 + dy) * MB + mb) * 64 + l) * 32 + e] =
                      host_f32_to_e4m3(W(co, 32 * (g & 1) + e, tap));
              }
        HIPOK(hipMalloc(&L.wblob_rr, rr.size()));
        net.allocs.push_back(L.wblob_rr);
        HIPOK(hipMemcpy(L.wblob_rr, rr.data(), rr.size(), hipMemcpyHostToDevice));
        // split-layer pair kernel: fragment j holds taps j - 1 (lane groups
        // 0-1) and j (groups 2-3), taps numbered 3 dy + dx, zero outside 0..8
        std::vector<uint8_t> sl((size_t)10 * MB * 64 * 32, 0);
        for (int jf = 0; jf < 10; ++jf)
          for (int mb = 0; mb < MB; ++mb)
            for (int l = 0; l < 64; ++l) {
              const int g = l >> 4, tap = g < 2 ? jf - 1 : jf;
              if (tap < 0 || tap > 8) continue;
              const int co = mb * 16 + (l & 15);
              for (int e = 0; e < 32; ++e)
                sl[(((size_t)jf * MB + mb) * 64 + l) * 32 + e] =
                    host_f32_to_e4m3(W(co, 32 * (g & 1) + e, tap));
            }
        HIPOK(hipMalloc(&L.wblob_sl, sl.size()));
        net.allocs.push_back(L.wblob_sl);
        HIPOK(hipMemcpy(L.wblob_sl, sl.data(), sl.size(), hipMemcpyHostToDevice));
      }
    }
    woff += (size_t)L.cin * L.cout * 9;
    boff += (size_t)L.cout;
  }
  // activation buffers: every storage format gets its own pair (one buffer
  // when a single layer writes it), so a buffer's zero border is never
  // overwritten by pixels of a layout with a different pixel size
  {
    int base[3] = {-1, -1, -1}, count[3] = {0, 0, 0}, next = 0;
    for (int k = 0; k + 1 < K; ++k) count[net.layers[k].out_fmt] += 1;
    int parity[3] = {0, 0, 0};
    for (int k = 0; k + 1 < K; ++k) {
      const int f = net.layers[k].out_fmt;
      if (base[f] < 0) {
        base[f] = next;
        const int nb = count[f] > 1 ? 2 : 1;
        for (int i = 0; i < nb; ++i) net.buf_fmt[next + i] = f;
        next += nb;
      }
      net.layers[k].out_buf = base[f] + parity[f];
      if (count[f] > 1) parity[f] ^= 1;
      net.layers[k + 1].in_buf = net.layers[k].out_buf;
    }
  }
  conv_th = (K > 1) ? mid_tile_rows(net.layers[1].in_fmt) : 16;
  net.last_fused = false;
  if (K >= 4) {
    const LayerPlan &Lm = net.layers[K - 2], &Ll = net.layers[K - 1];
    net.last_fused = mid_last_fusable(Lm.in_fmt, Lm.out_fmt, net.F, Lm.relu, Lm.unit_scale,
                                      Ll.in_fmt, Ll.cin, Ll.cout) &&
                     conv_th == 16;
  }
  // e4m3 networks whose middle layers pair up exactly: the last pair's second
  // layer feeds the bf16 last layer, which then runs inside that kernel
  net.last_pair8 = false;
  if (K >= 4 && (K - 2) % 2 == 0 && !net.last_fused) {
    const LayerPlan &A = net.layers[K - 3], &B = net.layers[K - 2], &Ll = net.layers[K - 1];
    net.last_pair8 = pair8_fusable(A.in_fmt, A.out_fmt, net.F, A.relu, B.in_fmt, B.out_fmt,
                                   B.relu) &&
                     A.wblob_rr && B.wblob_rr &&
                     last_pair8_fusable(B.out_fmt, Ll.in_fmt, Ll.cin, Ll.cout);
  }
  plan_dirty = true;
  return Status::ok();
}

Status Engine::set_prior(const pnpula_config *c) {
  net = NetPlan();
  net.prior = c->prior;
  if (c->prior == PNPULA_PRIOR_DDFB) {
    const int K = c->ddfb_layers, F = c->ddfb_features;
    const size_t nw = (size_t)K * F * 9;
    for (size_t i = 0; i < nw; ++i)
      if (!std::isfinite(c->ddfb_weights[i])) return Status::fail(PNPULA_EINVAL, "non-finite weight");
    for (int k = 0; k < K; ++k)
      if (!std::isfinite(c->ddfb_gamma[k])) return Status::fail(PNPULA_EINVAL, "non-finite step size");
    net.ddfb_K = K;
    net.ddfb_F = F;
    net.ddfb_thresh = (float)c->ddfb_thresh;
    net.ddfb_gamma.assign(c->ddfb_gamma, c->ddfb_gamma + K);
    HIPOK(hipMalloc(&net.ddfb_w, nw * sizeof(float)));
    net.allocs.push_back(net.ddfb_w);
    HIPOK(hipMemcpy(net.ddfb_w, c->ddfb_weights, nw * sizeof(float), hipMemcpyHostToDevice));
  }
  plan_dirty = true;
  return Status::ok();
}

// ---------------------------------------------------------------------
// jobs
// ---------------------------------------------------------------------
int Engine::prior_radius(const pnpula_config *c) {
  if (c->prior == PNPULA_PRIOR_TV) return 1;
  if (c->prior == PNPULA_PRIOR_DDFB) return 2 * c->ddfb_layers;
  return c->n_layers;
}

Status Engine::validate_job(const pnpula_config *c, int, const std::vector<int> &) {
  if (!c) return Status::fail(PNPULA_EINVAL, "null config");
  if (c->ny < 1 || c->nx < 1) return Status::fail(PNPULA_EINVAL, "image size must be positive");
  if ((int64_t)c->ny * c->nx > (int64_t)1 << 40) return Status::fail(PNPULA_EINVAL, "image too large");
  if (!c->y) return Status::fail(PNPULA_EINVAL, "y is required");
  if (c->ksize < 1 || c->ksize % 2 == 0 || c->ksize > 2 * kMaxRBig + 1 || !c->kernel)
    return Status::fail(PNPULA_EINVAL, "blur size must be odd and at most 129");
  if (c->prior < PNPULA_PRIOR_CNN || c->prior > PNPULA_PRIOR_DDFB)
    return Status::fail(PNPULA_EINVAL, "unknown prior");
  if (c->likelihood < PNPULA_LIK_GAUSSIAN || c->likelihood > PNPULA_LIK_POISSON ||
      c->z_step < 0 || c->z_step > 1)
    return Status::fail(PNPULA_EINVAL, "unknown likelihood or z-step");
  if (c->likelihood == PNPULA_LIK_POISSON && c->z_step != 1)
    return Status::fail(PNPULA_EINVAL, "the Poisson likelihood needs the PSGLA z-step");
  if (!(c->eta >= 0) || !(c->rho2 >= 0) || !(c->beta >= 0) || !(c->kappa >= 0) ||
      !(c->kappa2 >= 0) || !std::isfinite(c->eta) || !std::isfinite(c->rho2) ||
      !std::isfinite(c->beta) || !std::isfinite(c->kappa) || !std::isfinite(c->kappa2))
    return Status::fail(PNPULA_EINVAL, "eta, kappa, rho2, kappa2, beta must be finite and >= 0");
  if ((c->z_step == 1 || c->prior == PNPULA_PRIOR_TV) && !(c->rho > 0 && c->kappa > 0))
    return Status::fail(PNPULA_EINVAL, "PSGLA needs rho > 0 and kappa > 0");
  if (c->rho2 > 0 && (c->z_step != 1 || !(c->kappa2 > 0)))
    return Status::fail(PNPULA_EINVAL, "the second z block needs the PSGLA z-step and kappa2 > 0");
  if (c->prior == PNPULA_PRIOR_TV && (c->z_step != 0 || c->likelihood != PNPULA_LIK_GAUSSIAN))
    return Status::fail(PNPULA_EINVAL, "the TV prior runs with the unsplit Gaussian likelihood");
  if (c->prior == PNPULA_PRIOR_DDFB &&
      (c->ddfb_layers < 1 || c->ddfb_layers > kMaxDdfbLayers || c->ddfb_features < 1 ||
       c->ddfb_features > 64 || !c->ddfb_weights || !c->ddfb_gamma || !(c->ddfb_thresh >= 0)))
    return Status::fail(PNPULA_EINVAL,
                        "DDFB needs 1..8 layers, 1..64 features, weights, step sizes, thresh >= 0");
  if (!(c->sigma > 0) || !(c->eps > 0) || !(c->delta > 0) || !(c->rho >= 0) ||
      !(c->alpha >= 0) || !(c->inv_lambda >= 0) || !std::isfinite(c->sigma) ||
      !std::isfinite(c->eps) || !std::isfinite(c->delta) || !std::isfinite(c->rho) ||
      !std::isfinite(c->alpha) || !std::isfinite(c->inv_lambda))
    return Status::fail(PNPULA_EINVAL, "sigma, eps, delta must be > 0; rho, alpha, inv_lambda >= 0");
  if (c->block_y < 1 || c->block_x < 1) return Status::fail(PNPULA_EINVAL, "block size must be >= 1");
  const int r = c->ksize / 2;
  const bool single = c->block_y >= c->ny && c->block_x >= c->nx;
  if (!single) {
    if (c->halo < std::max(2 * r, prior_radius(c)))
      return Status::fail(PNPULA_EINVAL, "halo must be >= max(2r, prior radius)");
    if (c->halo >= std::min(c->block_y, c->block_x))
      return Status::fail(PNPULA_EINVAL, "halo must be smaller than the blocks");
  }
  if (c->burn_in < 0) return Status::fail(PNPULA_EINVAL, "burn_in must be >= 0");
  if (c->welford_window < 0 || c->welford_window > 65536)
    return Status::fail(PNPULA_EINVAL, "welford_window out of range");
  return Status::ok();
}

struct Geometry {
  int B, rows, pitch;        // padded x / y / mask buffers
  int arows, apitch;         // activation buffers
};

static Geometry geometry(int ny, int nx, int r) {
  Geometry g;
  g.B = std::max(2 * r, 2);          // >= 2: the fused first layer reads x two pixels out
  g.rows = ny + 2 * g.B + kUpdTileH;
  g.pitch = ((nx + 2 * g.B + kUpdTileW) + 63) / 64 * 64;
  g.arows = ny + 2 + 16;
  g.apitch = nx + 2 + kConvTileW;
  return g;
}

// large blur: residual buffer with a zero border of r, and kernel rows
// padded to a multiple of 8 taps
static int64_t res_pitch(int nx, int r) { return ((int64_t)nx + 2 * r + kUpdTileW + 63) / 64 * 64; }
static int64_t res_rows(int ny, int r) { return (int64_t)ny + 2 * r + kUpdTileH; }
static int kbig_pitch(int L) { return (L + 7) / 8 * 8; }

size_t Engine::job_footprint(const pnpula_config *c, const NetPlan &n) {
  const int r = c->ksize / 2;
  const Geometry g = geometry(c->ny, c->nx, r);
  const size_t N = (size_t)c->ny * c->nx;
  const size_t xbytes = (size_t)g.rows * g.pitch * sizeof(float);
  size_t bytes = 3 * xbytes;                                            // x[2], y
  if (c->mask) bytes += (size_t)g.rows * g.pitch;
  if (c->z_step == 1) bytes += (c->rho2 > 0 ? 2 : 1) * xbytes;          // z1 (, z2)
  if (c->prior == PNPULA_PRIOR_TV) bytes += 2 * xbytes;                 // zh, zv
  if (c->prior == PNPULA_PRIOR_DDFB && c->ddfb_layers > 1)
    bytes += (size_t)(c->ddfb_layers - 1) * xbytes;                     // b_1 .. b_{K-1}
  if (r > kMaxR)
    bytes += (size_t)res_rows(c->ny, r) * res_pitch(c->nx, r) * sizeof(float) + N * sizeof(float) +
             2 * (size_t)c->ksize * kbig_pitch(c->ksize) * sizeof(float);
  for (int b = 0; b < 4; ++b)
    if (n.buf_fmt[b] >= 0) bytes += (size_t)g.arows * g.apitch * n.F * fmt_bytes(n.buf_fmt[b]);
  bytes += N * (sizeof(float) * 3 + sizeof(double) * 2);                // G, Welford
  if (n.last_fused || n.last_pair8)
    bytes += ((size_t)(c->ny + 2) * (c->nx + 2) + 1) * 12 * sizeof(float);
  bytes += 4096;
  return bytes;
}

template <class T>
static Status dalloc(Job *j, T **p, size_t bytes) {
  void *v = nullptr;
  hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return Status::fail(PNPULA_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  j->allocs.push_back(v);
  *p = reinterpret_cast<T *>(v);
  return Status::ok();
}

#define TRY(expr)                 \
  do {                            \
    Status s_ = (expr);           \
    if (!s_.good()) return s_;    \
  } while (0)

static void make_tiles(std::vector<TileRef> &out, int ny, int nx, int by, int bx, int TH, int TW) {
  out.clear();
  for (int y0 = 0; y0 < ny; y0 += by)
    for (int x0 = 0; x0 < nx; x0 += bx) {
      const int bh = std::min(by, ny - y0), bw = std::min(bx, nx - x0);
      for (int ty = 0; ty < bh; ty += TH)
        for (int tx = 0; tx < bw; tx += TW) {
          TileRef t{};
          t.job = 0;
          t.y0 = y0 + ty;
          t.x0 = x0 + tx;
          t.h = std::min(TH, bh - ty);
          t.w = std::min(TW, bw - tx);
          out.push_back(t);
        }
    }
}

Status Engine::make_job(const pnpula_config *c, Job **out) {
  TRY(validate_job(c, net.K, net.channels));
  Job *j = new Job();
  auto fail = [&](Status s) { free_job(j); return s; };
  const int ny = c->ny, nx = c->nx, r = c->ksize / 2, L = c->ksize;
  const Geometry g = geometry(ny, nx, r);
  const size_t N = (size_t)ny * nx;
  JobDesc &d = j->d;
  d.ny = ny;
  d.nx = nx;
  d.xpitch = g.pitch;
  d.xborder = g.B;
  d.apitch = g.apitch;
  d.arows = g.arows;
  d.r = r;
  d.has_mask = c->mask != nullptr;
  d.split = c->rho > 0;
  d.zmode = c->z_step == 1 ? 1 : (c->prior == PNPULA_PRIOR_TV ? 2 : 0);
  d.poisson = c->likelihood == PNPULA_LIK_POISSON;
  d.has_z2 = (d.zmode == 1 && c->rho2 > 0) || d.zmode == 2;
  d.xpos = c->prior == PNPULA_PRIOR_TV;
  d.big = r > kMaxR;
  if (d.zmode != 0) d.split = 0;          // z is chain state, not drawn in the update
  d.burn_in = c->burn_in;
  d.wwin = c->welford_window > 0 ? c->welford_window : 256;
  j->block_y = std::min(c->block_y, ny);
  j->block_x = std::min(c->block_x, nx);
  j->halo = c->halo;
  j->footprint = job_footprint(c, net);
  const size_t xbytes = (size_t)g.rows * g.pitch * sizeof(float);
  // inputs_on_device: y, kernel, mask and x0 are device pointers
  const hipMemcpyKind in_kind = c->inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  Status s;
  if (!(s = dalloc(j, &d.x[0], xbytes)).good()) return fail(s);
  if (!(s = dalloc(j, &d.x[1], xbytes)).good()) return fail(s);
  float *yb = nullptr;
  if (!(s = dalloc(j, &yb, xbytes)).good()) return fail(s);
  d.y = yb;
  hipError_t e = hipSuccess;
  e = hipMemsetAsync(d.x[0], 0, xbytes, stream);
  if (e == hipSuccess) e = hipMemsetAsync(d.x[1], 0, xbytes, stream);
  if (e == hipSuccess) e = hipMemsetAsync(yb, 0, xbytes, stream);
  const size_t hpitch = (size_t)nx * sizeof(float), dpitch = (size_t)g.pitch * sizeof(float);
  const size_t origin = (size_t)g.B * g.pitch + g.B;
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(yb + origin, dpitch, c->y, hpitch, hpitch, ny, in_kind, stream);
  if (e == hipSuccess && c->x0)
    e = hipMemcpy2DAsync(d.x[0] + origin, dpitch, c->x0, hpitch, hpitch, ny, in_kind, stream);
  if (e == hipSuccess && c->mask) {
    uint8_t *mb = nullptr;
    if (!(s = dalloc(j, &mb, (size_t)g.rows * g.pitch)).good()) return fail(s);
    e = hipMemsetAsync(mb, 0, (size_t)g.rows * g.pitch, stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(mb + origin, g.pitch, c->mask, nx, nx, ny, in_kind, stream);
    d.mask = mb;
  }
  // splitting variables held as state (z^(0) = 0) and the DDFB maps: padded
  // like x, zero border never written
  float **zb[2] = {&d.z1, &d.z2};
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    if (d.zmode == 0 || (i == 1 && !d.has_z2)) continue;
    if (!(s = dalloc(j, zb[i], xbytes)).good()) return fail(s);
    e = hipMemsetAsync(*zb[i], 0, xbytes, stream);
  }
  if (e == hipSuccess && c->prior == PNPULA_PRIOR_DDFB && c->ddfb_layers > 1) {
    const size_t mbytes = (size_t)(c->ddfb_layers - 1) * xbytes;
    if (!(s = dalloc(j, &d.dmaps, mbytes)).good()) return fail(s);
    e = hipMemsetAsync(d.dmaps, 0, mbytes, stream);
    d.dstride = (int64_t)g.rows * g.pitch;
  }
  if (e != hipSuccess) return fail(Status::fail(PNPULA_EDEVICE, hipGetErrorString(e)));
  for (int b = 0; b < 4; ++b) {
    if (net.buf_fmt[b] < 0) continue;
    const size_t abytes = (size_t)g.arows * g.apitch * net.F * fmt_bytes(net.buf_fmt[b]);
    uint8_t *ab = nullptr;
    if (!(s = dalloc(j, &ab, abytes)).good()) return fail(s);
    if (hipMemsetAsync(ab, 0, abytes, stream) != hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "memset"));
    d.act[b] = ab;
  }
  if (!(s = dalloc(j, &d.G, N * sizeof(float))).good()) return fail(s);
  d.S = nullptr;
  if (net.last_fused || net.last_pair8) {
    const size_t sbytes = ((size_t)(ny + 2) * (nx + 2) + 1) * 12 * sizeof(float);
    if (!(s = dalloc(j, &d.S, sbytes)).good()) return fail(s);
    if (hipMemsetAsync(d.S, 0, sbytes, stream) != hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "memset"));
  }
  if (!(s = dalloc(j, &d.wmean, N * sizeof(float))).good()) return fail(s);
  if (!(s = dalloc(j, &d.wm2, N * sizeof(float))).good()) return fail(s);
  if (!(s = dalloc(j, &d.mean, N * sizeof(double))).good()) return fail(s);
  if (!(s = dalloc(j, &d.m2, N * sizeof(double))).good()) return fail(s);
  if (!(s = dalloc(j, &d.flag, 64)).good()) return fail(s);
  if (hipMemsetAsync(d.flag, 0, 64, stream) != hipSuccess ||
      hipMemsetAsync(d.mean, 0, N * sizeof(double), stream) != hipSuccess ||
      hipMemsetAsync(d.m2, 0, N * sizeof(double), stream) != hipSuccess)
    return fail(Status::fail(PNPULA_EDEVICE, "memset"));
  // blur: full kernel, and its rank-1 factors when it is separable
  std::vector<float> kern(L * L);
  if (c->inputs_on_device) {
    if (hipMemcpy(kern.data(), c->kernel, (size_t)L * L * sizeof(float), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "kernel read from device failed"));
  } else {
    std::copy(c->kernel, c->kernel + L * L, kern.begin());
  }
  std::vector<float> ku(L, 0.f), kv(L, 0.f);
  {
    int pa = 0, pc = 0;
    double best = -1;
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b)
        if (std::fabs((double)kern[a * L + b]) > best) {
          best = std::fabs((double)kern[a * L + b]);
          pa = a;
          pc = b;
        }
    bool sep = best > 0;
    if (sep) {
      const double piv = kern[pa * L + pc];
      double scale = 0;
      for (int a = 0; a < L * L; ++a) scale = std::max(scale, std::fabs((double)kern[a]));
      for (int a = 0; a < L && sep; ++a)
        for (int b = 0; b < L; ++b) {
          const double pred = (double)kern[a * L + pc] * (double)kern[pa * L + b] / piv;
          if (std::fabs(pred - (double)kern[a * L + b]) > 1e-6 * scale) {
            sep = false;
            break;
          }
        }
      if (sep) {
        const double sq = std::sqrt(std::fabs(piv));
        for (int a = 0; a < L; ++a) ku[a] = (float)((double)kern[a * L + pc] / sq);
        for (int b = 0; b < L; ++b) kv[b] = (float)((double)kern[pa * L + b] / sq * (piv < 0 ? -1 : 1));
      }
    }
    d.separable = sep;
  }
  for (float v : kern)
    if (!std::isfinite(v)) return fail(Status::fail(PNPULA_EINVAL, "non-finite blur kernel"));
  float *kd = nullptr;
  if (!(s = dalloc(j, &kd, (size_t)3 * L * L * sizeof(float))).good()) return fail(s);
  std::vector<float> kall(3 * L * L, 0.f);
  std::copy(kern.begin(), kern.end(), kall.begin());
  std::copy(ku.begin(), ku.end(), kall.begin() + L * L);
  std::copy(kv.begin(), kv.end(), kall.begin() + 2 * L * L);
  if (hipMemcpyAsync(kd, kall.data(), kall.size() * sizeof(float), hipMemcpyHostToDevice, stream) !=
      hipSuccess)
    return fail(Status::fail(PNPULA_EDEVICE, "kernel upload"));
  d.kern = kd;
  d.ku = kd + L * L;
  d.kv = kd + 2 * L * L;
  {
    // correlation kernels of the whole-image passes (large blurs, the
    // data-gradient entry point): flip(k) for K x, k for K^T r
    const int Lp = kbig_pitch(L);
    std::vector<float> kb((size_t)2 * L * Lp, 0.f);
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b) {
        kb[(size_t)a * Lp + b] = kern[(size_t)(L - 1 - a) * L + (L - 1 - b)];
        kb[(size_t)L * Lp + (size_t)a * Lp + b] = kern[(size_t)a * L + b];
      }
    float *kbd = nullptr;
    if (!(s = dalloc(j, &kbd, kb.size() * sizeof(float))).good()) return fail(s);
    if (hipMemcpyAsync(kbd, kb.data(), kb.size() * sizeof(float), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "kernel upload"));
    d.kbig[0] = kbd;
    d.kbig[1] = kbd + (size_t)L * Lp;
    d.kpitch = Lp;
    // the host copy kb must outlive the asynchronous upload
    if (hipStreamSynchronize(stream) != hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "upload failed"));
  }
  if (d.big) {
    // residual buffer with a zero border of r, and the gradient
    d.rpitch = res_pitch(nx, r);
    const size_t rbytes = (size_t)res_rows(ny, r) * d.rpitch * sizeof(float);
    if (!(s = dalloc(j, &d.res, rbytes)).good()) return fail(s);
    if (hipMemsetAsync(d.res, 0, rbytes, stream) != hipSuccess)
      return fail(Status::fail(PNPULA_EDEVICE, "memset"));
    if (!(s = dalloc(j, &d.gdat, N * sizeof(float))).good()) return fail(s);
  }
  // coefficients (FP64, rounded once)
  const double sig2 = c->sigma * c->sigma;
  d.delta = (float)c->delta;
  d.cprior = (float)(c->alpha * c->delta / c->eps);
  d.cproj = (float)(c->delta * c->inv_lambda);
  d.sq2d = (float)std::sqrt(2.0 * c->delta);
  d.inv_s2 = (float)(c->rho > 0 ? 1.0 / c->rho : 1.0 / sig2);
  d.inv_sig2 = (float)(1.0 / sig2);
  d.zmix = (float)(c->rho > 0 ? c->rho / (c->rho + sig2) : 0.0);
  d.zsd = (float)(c->rho > 0 ? std::sqrt(c->rho * sig2 / (c->rho + sig2)) : 0.0);
  const double eta = c->eta > 0 ? c->eta : 1.0;
  if (d.zmode == 1) {                     // PSGLA: g = eta K^T m (eta m K x - z1)/rho + ...
    d.inv_s2 = (float)(eta / c->rho);
    d.eta = (float)eta;
    d.za1 = (float)(c->kappa / c->rho);
    d.zs1 = (float)std::sqrt(2.0 * c->kappa);
    d.zkappa = (float)c->kappa;
    d.zsig2 = (float)sig2;
    if (c->rho2 > 0) {
      d.za2 = (float)(c->kappa2 / c->rho2);
      d.zs2 = (float)std::sqrt(2.0 * c->kappa2);
      d.inv_rho2 = (float)(1.0 / c->rho2);
    }
  } else if (d.zmode == 2) {              // TV: unsplit data term, prior term delta G
    d.inv_s2 = (float)(1.0 / sig2);
    d.cprior = (float)c->delta;
    d.cproj = 0.0f;
    d.za1 = (float)(c->kappa / c->rho);
    d.zs1 = (float)std::sqrt(2.0 * c->kappa);
    d.zkappa = (float)(c->kappa * c->beta);
    d.inv_rho = (float)(1.0 / c->rho);
  }
  d.key0 = (uint32_t)c->seed;
  d.key1 = (uint32_t)(c->seed >> 32);
  d.chain = c->chain;
  d.wbase = 0;
  d.nbase = 0;
  j->t = 0;
  make_tiles(j->conv_tiles, ny, nx, j->block_y, j->block_x, conv_th, kConvTileW);
  make_tiles(j->upd_tiles, ny, nx, j->block_y, j->block_x, kUpdTileH, kUpdTileW);
  // the two-layer kernel tiles the whole image (every block of one job lives
  // in one set of activation buffers, so block edges need no tile edge), in
  // column bands 32 tiles wide, top to bottom: the 32 workgroups of an XCD
  // take one band row at a time, and the next band row's windows overlap the
  // previous one's while it is still in that XCD's L2
  make_tiles(j->pair_tiles, ny, nx, ny, 32 * kPairTileW, kPairTileH, kPairTileW);
  make_tiles(j->pair_ws_tiles, ny, nx, ny, 32 * kPairTileW, kPairWsTileH, kPairTileW);
  make_tiles(j->pair8ws_tiles, ny, nx, ny, 32 * kPairTileW, kPair8WsTileH, kPairTileW);
  if (c->prior == PNPULA_PRIOR_DDFB) make_tiles(j->ddfb_tiles, ny, nx, ny, nx, kDdTile, kDdTile);
  if (hipStreamSynchronize(stream) != hipSuccess)
    return fail(Status::fail(PNPULA_EDEVICE, "upload failed"));
  *out = j;
  return Status::ok();
}

void Engine::free_job(Job *j) {
  if (!j) return;
  for (void *p : j->allocs) hipFree(p);
  delete j;
}

// ---------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------
Status Engine::rebuild_plan() {
  std::vector<TileRef> conv, upd, pair, pair_ws, pair8ws, ddfb;
  max_r = 0;
  uniform_r = true;
  max_kpitch = 8;
  for (size_t ji = 0; ji < resident.size(); ++ji) {
    Job *j = resident[ji];
    if (ji == 0) {
      zmode = j->d.zmode;
      big = j->d.big;
    } else if (j->d.zmode != zmode || (bool)j->d.big != big) {
      return Status::fail(PNPULA_EINVAL, "resident jobs must share the z-step and blur path");
    }
    max_kpitch = std::max(max_kpitch, (int)j->d.kpitch);
    for (TileRef t : j->ddfb_tiles) {
      t.job = (int)ji;
      ddfb.push_back(t);
    }
    for (TileRef t : j->conv_tiles) {
      t.job = (int)ji;
      conv.push_back(t);
    }
    for (TileRef t : j->upd_tiles) {
      t.job = (int)ji;
      upd.push_back(t);
    }
    for (TileRef t : j->pair_tiles) {
      t.job = (int)ji;
      pair.push_back(t);
    }
    for (TileRef t : j->pair_ws_tiles) {
      t.job = (int)ji;
      pair_ws.push_back(t);
    }
    for (TileRef t : j->pair8ws_tiles) {
      t.job = (int)ji;
      pair8ws.push_back(t);
    }
    if (ji > 0 && j->d.r != max_r) uniform_r = false;
    max_r = std::max(max_r, j->d.r);
  }
  auto grow = [&](auto **p, size_t &cap, size_t need, size_t elem) -> Status {
    if (need > cap) {
      hipFree(*p);
      *p = nullptr;
      size_t n = std::max(need, cap * 2);
      void *v = nullptr;
      if (hipMalloc(&v, n * elem) != hipSuccess)
        return Status::fail(PNPULA_ENOMEM, "plan allocation failed");
      *p = reinterpret_cast<std::remove_reference_t<decltype(**p)> *>(v);
      cap = n;
    }
    return Status::ok();
  };
  HIPOK(hipStreamSynchronize(stream));
  TRY(grow(&d_conv, cap_conv, std::max<size_t>(conv.size(), 1), sizeof(TileRef)));
  TRY(grow(&d_upd, cap_upd, std::max<size_t>(upd.size(), 1), sizeof(TileRef)));
  TRY(grow(&d_pair, cap_pair, std::max<size_t>(pair.size(), 1), sizeof(TileRef)));
  TRY(grow(&d_pair_ws, cap_pair_ws, std::max<size_t>(pair_ws.size(), 1), sizeof(TileRef)));
  TRY(grow(&d_pair8ws, cap_pair8ws, std::max<size_t>(pair8ws.size(), 1), sizeof(TileRef)));
  TRY(grow(&d_jobs, cap_jobs, std::max<size_t>(resident.size(), 1), sizeof(JobDesc)));
  TRY(grow(&d_ddfb, cap_ddfb, std::max<size_t>(ddfb.size(), 1), sizeof(TileRef)));
  if (!ddfb.empty())
    HIPOK(hipMemcpyAsync(d_ddfb, ddfb.data(), ddfb.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  n_ddfb = (int)ddfb.size();
  if (!conv.empty())
    HIPOK(hipMemcpyAsync(d_conv, conv.data(), conv.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  if (!upd.empty())
    HIPOK(hipMemcpyAsync(d_upd, upd.data(), upd.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  if (!pair.empty())
    HIPOK(hipMemcpyAsync(d_pair, pair.data(), pair.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  if (!pair_ws.empty())
    HIPOK(hipMemcpyAsync(d_pair_ws, pair_ws.data(), pair_ws.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  if (!pair8ws.empty())
    HIPOK(hipMemcpyAsync(d_pair8ws, pair8ws.data(), pair8ws.size() * sizeof(TileRef), hipMemcpyHostToDevice, stream));
  n_conv = (int)conv.size();
  n_pair = (int)pair.size();
  n_pair_ws = (int)pair_ws.size();
  n_pair8ws = (int)pair8ws.size();
  n_upd = (int)upd.size();
  plan_dirty = false;
  return upload_descs();
}

Status Engine::upload_descs() {
  std::vector<JobDesc> ds(resident.size());
  for (size_t i = 0; i < resident.size(); ++i) {
    resident[i]->d.t_offset = resident[i]->t - ticks;
    ds[i] = resident[i]->d;
  }
  if (!ds.empty())
    HIPOK(hipMemcpyAsync(d_jobs, ds.data(), ds.size() * sizeof(JobDesc), hipMemcpyHostToDevice, stream));
  // the staging copy of pageable memory completes before return only for
  // small transfers; wait so that ds can be released safely
  HIPOK(hipStreamSynchronize(stream));
  return Status::ok();
}

// ---------------------------------------------------------------------
// profiling with events on the engine's stream
// ---------------------------------------------------------------------
void Engine::profile_enable(bool on) {
  hipStreamSynchronize(stream);
  for (auto &r : prof_pending) {
    prof_free.push_back(r.a);
    prof_free.push_back(r.b);
  }
  prof_pending.clear();
  for (int i = 0; i < kProfClasses; ++i) {
    prof_ms[i] = 0;
    prof_n[i] = 0;
  }
  profiling = on;
}

void Engine::prof_begin(int cls, ProfileRec *r) {
  r->cls = cls;
  r->a = r->b = nullptr;
  if (!profiling) return;
  for (hipEvent_t *e : {&r->a, &r->b}) {
    if (!prof_free.empty()) {
      *e = prof_free.back();
      prof_free.pop_back();
    } else {
      hipEventCreate(e);
    }
  }
  hipEventRecord(r->a, stream);
}

void Engine::prof_end(ProfileRec *r) {
  if (!profiling || !r->a) return;
  hipEventRecord(r->b, stream);
  prof_pending.push_back(*r);
}

Status Engine::profile_read(int cls, double *ms, int64_t *launches) {
  if (cls < 0 || cls >= kProfClasses) return Status::fail(PNPULA_EINVAL, "kernel class must be 0..9");
  HIPOK(hipStreamSynchronize(stream));
  for (auto &r : prof_pending) {
    float e = 0;
    if (hipEventElapsedTime(&e, r.a, r.b) == hipSuccess) {
      prof_ms[r.cls] += e;
      prof_n[r.cls] += 1;
    }
    prof_free.push_back(r.a);
    prof_free.push_back(r.b);
  }
  prof_pending.clear();
  if (ms) *ms = prof_ms[cls];
  if (launches) *launches = prof_n[cls];
  return Status::ok();
}

// ---------------------------------------------------------------------
// one iteration of every resident job
// ---------------------------------------------------------------------
// launch layer k of the denoiser over all resident jobs' tiles, reading and
// writing the activation buffers assigned to it when the network was set
Status Engine::launch_layer(int k, int64_t tick, bool prof, int in_slot, int out_slot) {
  const int K = net.K;
  const LayerPlan &L = net.layers[k];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_conv;
  a.n_tiles = n_conv;
  a.tile_rows = conv_th;
  a.tick = tick;
  a.relu = L.relu;
  a.unit_scale = L.unit_scale;
  a.bias = L.bias;
  a.oscale = L.oscale;
  a.in_inv_scale = L.in_inv_scale;
  a.out_inv_scale = L.out_inv_scale;
  a.in_slot = in_slot >= 0 ? in_slot : L.in_buf;
  a.out_slot = out_slot >= 0 ? out_slot : L.out_buf;
  ProfileRec pr;
  if (K == 1) {
    a.wf32 = L.wf32;
    if (prof) prof_begin(1, &pr);
    HIPOK(launch_conv_single(a, n_conv, stream));
  } else if (k == 0) {
    a.wf32 = L.wf32;
    if (prof) prof_begin(1, &pr);
    HIPOK(launch_conv_first(L.in_fmt, L.out_fmt, L.cout, a, n_conv, stream));
  } else if (k == K - 1) {
    a.wf32 = L.wf32;
    if (prof) prof_begin(2, &pr);
    HIPOK(launch_conv_last(L.in_fmt, L.cin, a, n_conv, stream));
  } else {
    a.wblob = L.wblob;
    a.wblob_rr = L.wblob_rr;
    const size_t lds = mid_lds_bytes(L.in_fmt, net.F);
    int occ = (int)std::max<size_t>(1, (160 * 1024) / lds);
    occ = std::min(occ, 4);
    const int need = ((n_conv + 7) / 8) * 8;
    const int n_wg = std::max(8, std::min(n_cu * occ, need) / 8 * 8);
    if (prof) prof_begin(0, &pr);
    HIPOK(launch_conv_mid(L.in_fmt, L.out_fmt, net.F, a, n_wg, stream));
  }
  if (prof) prof_end(&pr);
  return Status::ok();
}

// first layer and first middle layer in one kernel when the network allows it
// (bf16, 64 channels, ReLU, unit output scales)
bool Engine::first_mid_fused() const {
  if (net.K < 3) return false;
  const LayerPlan &L0 = net.layers[0], &L1 = net.layers[1];
  return first_mid_fusable(L0.in_fmt, L0.out_fmt, L0.cout, L0.relu, L0.unit_scale, L1.in_fmt,
                           L1.out_fmt, net.F, L1.relu, L1.unit_scale) &&
         conv_th == 16;
}

Status Engine::launch_first_mid(int64_t tick, bool prof) {
  const LayerPlan &L0 = net.layers[0], &L1 = net.layers[1];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_conv;
  a.n_tiles = n_conv;
  a.tile_rows = conv_th;
  a.tick = tick;
  a.relu = L1.relu;
  a.unit_scale = L1.unit_scale;
  a.bias = L1.bias;
  a.oscale = L1.oscale;
  a.in_inv_scale = L1.in_inv_scale;
  a.out_inv_scale = L1.out_inv_scale;
  a.in_slot = L1.in_buf;
  a.out_slot = L1.out_buf;
  a.wblob = L1.wblob;
  a.first_w = L0.wf32;
  a.first_bias = L0.bias;
  const int need = ((n_conv + 7) / 8) * 8;
  const int n_wg = std::max(8, std::min(n_cu, need) / 8 * 8);
  ProfileRec pr;
  if (prof) prof_begin(4, &pr);
  HIPOK(launch_conv_first_mid(a, n_wg, stream));
  if (prof) prof_end(&pr);
  return Status::ok();
}

// middle layer k writing the last layer's per-tap partials (JobDesc::S)
Status Engine::launch_mid_last(int k, int in_slot, int64_t tick, bool first, bool prof) {
  const LayerPlan &L = net.layers[k], &LL = net.layers[net.K - 1];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_conv;
  a.n_tiles = n_conv;
  a.tile_rows = conv_th;
  a.tick = tick;
  a.relu = L.relu;
  a.unit_scale = L.unit_scale;
  a.bias = L.bias;
  a.oscale = L.oscale;
  a.in_slot = in_slot >= 0 ? in_slot : L.in_buf;
  a.out_slot = L.out_buf;
  a.wblob = L.wblob;
  a.last_w = LL.wf32;
  if (first) {
    a.first_w = net.layers[0].wf32;
    a.first_bias = net.layers[0].bias;
  }
  const int need = ((n_conv + 7) / 8) * 8;
  const int n_wg = std::max(8, std::min(n_cu, need) / 8 * 8);
  ProfileRec pr;
  if (prof) prof_begin(5, &pr);
  HIPOK(launch_conv_mid_last(a, n_wg, first, stream));
  if (prof) prof_end(&pr);
  return Status::ok();
}

// middle layers k and k+1 in one kernel (64 channels, ReLU; bf16 with unit
// output scales, or e4m3), reading activation buffer in_slot and writing
// out_slot
bool Engine::pair_ok(int k) const {
  if (k < 1 || k + 1 > net.K - 2) return false;
  const LayerPlan &A = net.layers[k], &B = net.layers[k + 1];
  return pair_fusable(A.in_fmt, A.out_fmt, net.F, A.relu, A.unit_scale, B.in_fmt, B.out_fmt,
                      B.relu, B.unit_scale) ||
         (pair8_fusable(A.in_fmt, A.out_fmt, net.F, A.relu, B.in_fmt, B.out_fmt, B.relu) &&
          A.wblob_rr && B.wblob_rr);
}

// the first layer (bf16 -> e4m3) inside the kernel of the first e4m3 pair
bool Engine::first_pair8_ok() const {
  // only the pair that is both the first and the last (four layers)
  if (net.K != 4 || !net.last_pair8 || !pair_ok(1) || net.layers[1].in_fmt != FMT_E4M3)
    return false;
  if (net.last_fused && net.K - 2 == 2) return false;
  const LayerPlan &L0 = net.layers[0];
  if (!first_pair8_fusable(L0.in_fmt, L0.out_fmt, L0.cin, L0.cout, L0.relu)) return false;
  for (int i = 0; i < 4; ++i)
    if (i != net.layers[1].in_buf && net.buf_fmt[i] == net.buf_fmt[net.layers[1].in_buf])
      return true;
  return false;
}

// e4m3 networks whose first pair of middle layers goes to the split-layer
// kernel: the first layer runs as a kernel of its own, since the split-layer
// kernel has no place for it and carrying it in the one-group pair kernel
// costs more than writing and re-reading its e4m3 output
bool Engine::first8_ok() const {
  if (net.K < 5 || net.K - 2 <= 2 || !pair_ok(1)) return false;
  const LayerPlan &L0 = net.layers[0], &L1 = net.layers[1], &L2 = net.layers[2];
  if (L1.in_fmt != FMT_E4M3 || L2.out_fmt != FMT_E4M3 || !L1.wblob_sl || !L2.wblob_sl) return false;
  if (L0.out_buf != L1.in_buf) return false;
  return first_pair8_fusable(L0.in_fmt, L0.out_fmt, L0.cin, L0.cout, L0.relu) &&
         conv_th <= 16;
}

Status Engine::launch_first8(int64_t tick, bool prof) {
  const LayerPlan &L0 = net.layers[0];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_conv;
  a.n_tiles = n_conv;
  a.tile_rows = conv_th;
  a.tick = tick;
  a.first_w = L0.wf32;
  a.first_bias = L0.bias;
  a.first_oscale = L0.oscale;
  a.first_out_inv_scale = L0.out_inv_scale;
  a.out_slot = L0.out_buf;
  ProfileRec pr;
  if (prof) prof_begin(1, &pr);
  const int need = ((n_conv + 7) / 8) * 8;
  HIPOK(launch_conv_first8(a, std::max(8, std::min(6 * n_cu, need) / 8 * 8), stream));
  if (prof) prof_end(&pr);
  return Status::ok();
}

Status Engine::launch_pair(int k, int in_slot, int out_slot, int64_t tick, bool prof,
                           bool first, bool last) {
  const LayerPlan &A = net.layers[k], &B = net.layers[k + 1];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_pair;
  a.n_tiles = n_pair;
  a.tick = tick;
  a.relu = 1;
  a.unit_scale = 1;
  a.in_slot = in_slot;
  a.out_slot = out_slot;
  a.wblob = A.wblob;
  a.bias = A.bias;
  a.oscale = A.oscale;
  a.out_inv_scale = A.out_inv_scale;
  a.wblob2 = B.wblob;
  a.bias2 = B.bias;
  a.oscale2 = B.oscale;
  a.out_inv_scale2 = B.out_inv_scale;
  const bool e4m3 = A.in_fmt == FMT_E4M3;
  if (e4m3) {
    a.wblob_rr = A.wblob_rr;
    a.wblob2 = B.wblob_rr;
  }
  if (last) a.last_w = net.layers[net.K - 1].wf32;
  if (first) {
    const LayerPlan &L0 = net.layers[0];
    a.first_w = L0.wf32;
    a.first_bias = L0.bias;
    a.first_oscale = L0.oscale;
    a.first_out_inv_scale = L0.out_inv_scale;
  }
  const int per_cu = e4m3 ? pair8_wg_per_cu() : 1;
  const int need = ((n_pair + 7) / 8) * 8;
  const int n_wg = std::max(8, std::min(n_cu * per_cu, need) / 8 * 8);
  ProfileRec pr;
  if (prof) prof_begin(6, &pr);
  if (e4m3 && !first && !last && B.out_fmt == FMT_E4M3 && A.wblob_sl && B.wblob_sl) {
    // the split-layer form: one workgroup of 8 waves per CU
    a.wblob_rr = A.wblob_sl;
    a.wblob2 = B.wblob_sl;
    a.tiles = d_pair8ws;
    a.n_tiles = n_pair8ws;
    const int need8 = ((n_pair8ws + 7) / 8) * 8;
    HIPOK(launch_conv_pair8_ws(a, std::max(8, std::min(n_cu, need8) / 8 * 8), stream));
  } else if (e4m3) {
    HIPOK(launch_conv_pair8(a, B.out_fmt, first, last, n_wg, stream));
  } else {
    a.tiles = d_pair_ws;
    a.n_tiles = n_pair_ws;
    const int need_ws = ((n_pair_ws + 7) / 8) * 8;
    HIPOK(launch_conv_pair_ws(a, std::max(8, std::min(n_cu, need_ws) / 8 * 8), stream));
  }
  if (prof) prof_end(&pr);
  return Status::ok();
}

Status Engine::launch_g_from_s(int64_t tick, bool prof) {
  const LayerPlan &LL = net.layers[net.K - 1];
  ConvArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_conv;
  a.n_tiles = n_conv;
  a.tile_rows = conv_th;
  a.tick = tick;
  a.bias = LL.bias;
  a.oscale = LL.oscale;
  ProfileRec pr;
  if (prof) prof_begin(2, &pr);
  HIPOK(::pnp::launch_g_from_s(a, n_conv, stream));
  if (prof) prof_end(&pr);
  return Status::ok();
}

// the denoiser as the sampler runs it: first layer inside the first middle
// layer's kernel and last layer inside the last middle layer's (when the
// network allows), the rest layer by layer
Status Engine::run_fused_denoiser(int64_t tick, bool prof, const StageFn *on_stage) {
  const int K = net.K;
  const bool ff = first_mid_fused(), lf = net.last_fused;
  // cur: the activation buffer holding the latest layer's output once a
  // pair kernel has run (a pair writes the buffer its second layer would
  // have read, so later layers follow cur instead of the per-layer plan)
  int cur = -1;
  auto other = [&](int slot) {
    for (int i = 0; i < 4; ++i)
      if (i != slot && net.buf_fmt[i] == net.buf_fmt[slot]) return i;
    return -1;
  };
  int k = 0;
  auto stage = [&](int layer, int slot) -> Status {
    return on_stage ? (*on_stage)(layer, slot) : Status::ok();
  };
  if (ff) {
    TRY(launch_first_mid(tick, prof));
    TRY(stage(1, net.layers[1].out_buf));
    k = 2;
  } else if (first8_ok()) {
    TRY(launch_first8(tick, prof));
    TRY(stage(0, net.layers[0].out_buf));
    k = 1;
  } else if (first_pair8_ok()) {
    // four-layer e4m3 networks: the one pair feeds the last layer and also
    // carries the first layer
    const int in = net.layers[1].in_buf;
    const int out = net.layers[2].out_fmt == net.buf_fmt[in] ? other(in) : net.layers[2].out_buf;
    TRY(launch_pair(1, in, out, tick, prof, true, true));
    return launch_g_from_s(tick, prof);
  }
  for (; k < K; ++k) {
    const LayerPlan &L = net.layers[k];
    const int in = cur >= 0 ? cur : L.in_buf;
    if (lf && k == K - 2) {
      TRY(launch_mid_last(k, in, tick, false, prof));
      return launch_g_from_s(tick, prof);
    }
    // a pair writes the other buffer of its input's format, or the plan's
    // buffer when its second layer changes the format
    const int pair_out = net.layers[k + 1 < K ? k + 1 : k].out_fmt == net.buf_fmt[in]
                             ? other(in)
                             : net.layers[k + 1 < K ? k + 1 : k].out_buf;
    if (pair_ok(k) && !(lf && k + 1 == K - 2) && pair_out >= 0) {
      const int out = pair_out;
      const bool last = net.last_pair8 && k + 1 == K - 2;
      TRY(launch_pair(k, in, out, tick, prof, false, last));
      if (last) return launch_g_from_s(tick, prof);
      TRY(stage(k + 1, out));
      cur = out;
      ++k;
      continue;
    }
    if (cur < 0) {
      TRY(launch_layer(k, tick, prof));
      if (k + 1 < K) TRY(stage(k, L.out_buf));
      continue;
    }
    const int out = (k + 1 < K && L.out_fmt == net.buf_fmt[cur]) ? other(cur) : L.out_buf;
    TRY(launch_layer(k, tick, prof, in, out));
    if (k + 1 < K) TRY(stage(k, out));
    cur = k + 1 < K ? out : -1;
  }
  return Status::ok();
}

Status Engine::run_denoiser(int64_t tick) { return run_fused_denoiser(tick, true); }

// Prior term other than the residual CNN into JobDesc::G: the TV coupling
// term (1/rho) D^T (D x - z), or G = x - D(x) of the DDFB denoiser (one
// launch per stage).
Status Engine::run_prior_other(int64_t tick) {
  ProfileRec pr;
  if (net.prior == PNPULA_PRIOR_TV) {
    UpdateArgs u{};
    u.jobs = d_jobs;
    u.tiles = d_upd;
    u.n_tiles = n_upd;
    u.tick = tick;
    prof_begin(7, &pr);
    HIPOK(launch_tv_prior(u, n_upd, stream));
    prof_end(&pr);
    return Status::ok();
  }
  DdfbArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_ddfb;
  a.n_tiles = n_ddfb;
  a.K = net.ddfb_K;
  a.F = net.ddfb_F;
  a.tick = tick;
  a.w = net.ddfb_w;
  a.thresh = net.ddfb_thresh;
  for (int k = 0; k < net.ddfb_K; ++k) a.gamma[k] = net.ddfb_gamma[k];
  for (int k = 1; k <= net.ddfb_K; ++k) {
    a.stage = k;
    prof_begin(7, &pr);
    HIPOK(launch_ddfb_stage(a, n_ddfb, stream));
    prof_end(&pr);
  }
  return Status::ok();
}

Status Engine::tick() {
  if (plan_dirty) TRY(rebuild_plan());
  if (resident.empty()) return Status::ok();
  if (net.prior == PNPULA_PRIOR_CNN) TRY(run_denoiser(ticks));
  else TRY(run_prior_other(ticks));
  UpdateArgs u{};
  u.jobs = d_jobs;
  u.tiles = d_upd;
  u.n_tiles = n_upd;
  u.tick = ticks;
  ProfileRec pr;
  if (big) {
    // large blur: residual and adjoint as whole-image passes, then the update
    BlurArgs b{};
    b.jobs = d_jobs;
    b.tiles = d_upd;
    b.n_tiles = n_upd;
    b.tick = ticks;
    b.epi = EPI_RESIDUAL;
    prof_begin(9, &pr);
    HIPOK(launch_blur_big(b, n_upd, max_r, max_kpitch, stream));
    prof_end(&pr);
    b.epi = EPI_GRAD;
    prof_begin(9, &pr);
    HIPOK(launch_blur_big(b, n_upd, max_r, max_kpitch, stream));
    prof_end(&pr);
    prof_begin(3, &pr);
    HIPOK(launch_update_pointwise(u, n_upd, stream));
    prof_end(&pr);
  } else {
    prof_begin(3, &pr);
    HIPOK(launch_fused_update(u, n_upd, max_r, uniform_r, zmode == 1 ? 1 : 0, stream));
    prof_end(&pr);
  }
  if (zmode != 0) {
    // z-step from x^(t+1), noise at counter t+1
    UpdateArgs z = u;
    z.tick = ticks + 1;
    if (zmode == 1 && big) {
      BlurArgs b{};
      b.jobs = d_jobs;
      b.tiles = d_upd;
      b.n_tiles = n_upd;
      b.tick = ticks + 1;
      b.epi = EPI_KX;
      prof_begin(9, &pr);
      HIPOK(launch_blur_big(b, n_upd, max_r, max_kpitch, stream));
      prof_end(&pr);
    }
    prof_begin(8, &pr);
    if (zmode == 1) HIPOK(launch_zstep_psgla(z, n_upd, big ? 0 : max_r, stream));
    else HIPOK(launch_zstep_tv(z, n_upd, stream));
    prof_end(&pr);
  }
  ticks += 1;
  for (Job *j : resident) j->t += 1;
  return Status::ok();
}

Status Engine::sync_check(bool *diverged) {
  HIPOK(hipStreamSynchronize(stream));
  *diverged = false;
  for (Job *j : resident) {
    int32_t f = 0;
    HIPOK(hipMemcpy(&f, j->d.flag, sizeof f, hipMemcpyDeviceToHost));
    j->diverged = j->diverged || f != 0;
    *diverged = *diverged || j->diverged;
  }
  return Status::ok();
}

// ---------------------------------------------------------------------
// state and statistics of one job
// ---------------------------------------------------------------------
Status Engine::get_state(Job *j, float *x) {
  HIPOK(hipStreamSynchronize(stream));
  const JobDesc &d = j->d;
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  HIPOK(hipMemcpy2D(x, (size_t)d.nx * sizeof(float), d.x[j->t & 1] + origin,
                    (size_t)d.xpitch * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                    hipMemcpyDeviceToHost));
  return Status::ok();
}

static int64_t samples_at(const Job *j, int64_t t) {
  return std::max<int64_t>(0, t - j->d.burn_in);
}

Status Engine::flush_stats(Job *j, int64_t *n_total) {
  JobDesc &d = j->d;
  const int64_t s = samples_at(j, j->t);
  int64_t total = d.nbase;
  if (s > d.wbase) {
    const int64_t since = s - d.wbase;
    const int64_t pending = since % d.wwin;
    total = d.nbase + since;
    if (pending > 0) {
      const int64_t n_a = d.nbase + since - pending;
      HIPOK(launch_welford_flush(d, (double)n_a, (double)pending, stream));
    }
    d.wbase = s;
    d.nbase = total;
    TRY(upload_descs());
  }
  if (n_total) *n_total = total;
  return Status::ok();
}

Status Engine::read_stats(Job *j, double *mean, double *m2, int64_t *n) {
  int64_t total = 0;
  TRY(flush_stats(j, &total));
  HIPOK(hipStreamSynchronize(stream));
  const size_t N = (size_t)j->d.ny * j->d.nx;
  if (mean) HIPOK(hipMemcpy(mean, j->d.mean, N * sizeof(double), hipMemcpyDeviceToHost));
  if (m2) HIPOK(hipMemcpy(m2, j->d.m2, N * sizeof(double), hipMemcpyDeviceToHost));
  if (n) *n = total;
  return Status::ok();
}

Status Engine::set_state(Job *j, const float *x, int64_t t) {
  if (t < 0) return Status::fail(PNPULA_EINVAL, "t must be >= 0");
  TRY(flush_stats(j, nullptr));
  JobDesc &d = j->d;
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  HIPOK(hipMemcpy2DAsync(d.x[t & 1] + origin, (size_t)d.xpitch * sizeof(float), x,
                         (size_t)d.nx * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                         hipMemcpyHostToDevice, stream));
  j->t = t;
  d.wbase = samples_at(j, t);
  TRY(upload_descs());
  return Status::ok();
}

Status Engine::restore_stats(Job *j, const double *mean, const double *m2, int64_t n) {
  if (n < 0) return Status::fail(PNPULA_EINVAL, "n_samples must be >= 0");
  JobDesc &d = j->d;
  const size_t N = (size_t)d.ny * d.nx;
  HIPOK(hipMemcpyAsync(d.mean, mean, N * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPOK(hipMemcpyAsync(d.m2, m2, N * sizeof(double), hipMemcpyHostToDevice, stream));
  d.nbase = n;
  d.wbase = samples_at(j, j->t);
  TRY(upload_descs());
  return Status::ok();
}

// g = H^T (H x - y) / sigma^2 for device images x, g (ny*nx) through the
// device residual buffer res (ny*nx); queued on the stream, no allocation.
Status Engine::data_grad(Job *j, const float *x, float *g, float *res) {
  if (plan_dirty || resident.size() != 1 || resident[0] != j)
    return Status::fail(PNPULA_ESTATE, "the data gradient needs a single-job engine");
  if (j->d.poisson) return Status::fail(PNPULA_ESTATE, "the data term is not Gaussian");
  GradArgs a{};
  a.jobs = d_jobs;
  a.tiles = d_upd;
  a.n_tiles = n_upd;
  a.x = x;
  a.res = res;
  a.g = g;
  for (int epi = 0; epi < 2; ++epi) {
    a.epi = epi;
    HIPOK(launch_data_grad(a, n_upd, j->d.r, j->d.kpitch, stream));
  }
  return Status::ok();
}

// ---------------------------------------------------------------------
// checkpoint: header, x^(t), z1, z2 (when held), FP32 window mean / M2,
// FP64 mean / M2, each image compact
// ---------------------------------------------------------------------
namespace {
struct CkptHeader {
  uint64_t magic;
  int32_t ny, nx, zmode, has_z2;
  int64_t t, wbase, nbase;
};
constexpr uint64_t kCkptMagic = 0x31544b4350414c55ull;   // "ULAPCKT1"
}  // namespace

size_t Engine::checkpoint_bytes(const Job *j) const {
  const JobDesc &d = j->d;
  const size_t N = (size_t)d.ny * d.nx;
  const int nz = d.zmode == 0 ? 0 : (d.has_z2 ? 2 : 1);
  return sizeof(CkptHeader) + N * sizeof(float) * (1 + nz + 2) + N * sizeof(double) * 2;
}

Status Engine::checkpoint(Job *j, void *buf, size_t bytes) {
  if (bytes < checkpoint_bytes(j)) return Status::fail(PNPULA_EINVAL, "checkpoint buffer too small");
  HIPOK(hipStreamSynchronize(stream));
  const JobDesc &d = j->d;
  const size_t N = (size_t)d.ny * d.nx;
  CkptHeader h{kCkptMagic, d.ny, d.nx, d.zmode, d.has_z2, j->t, d.wbase, d.nbase};
  uint8_t *p = static_cast<uint8_t *>(buf);
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  float *f = reinterpret_cast<float *>(p);
  TRY(get_state(j, f));
  f += N;
  if (d.zmode != 0) {
    TRY(get_z(j, f, d.has_z2 ? f + N : nullptr));
    f += (d.has_z2 ? 2 : 1) * N;
  }
  HIPOK(hipMemcpy(f, d.wmean, N * sizeof(float), hipMemcpyDeviceToHost));
  HIPOK(hipMemcpy(f + N, d.wm2, N * sizeof(float), hipMemcpyDeviceToHost));
  double *g = reinterpret_cast<double *>(f + 2 * N);
  HIPOK(hipMemcpy(g, d.mean, N * sizeof(double), hipMemcpyDeviceToHost));
  HIPOK(hipMemcpy(g + N, d.m2, N * sizeof(double), hipMemcpyDeviceToHost));
  return Status::ok();
}

Status Engine::resume(Job *j, const void *buf, size_t bytes) {
  JobDesc &d = j->d;
  const size_t N = (size_t)d.ny * d.nx;
  CkptHeader h;
  if (bytes < sizeof h) return Status::fail(PNPULA_EINVAL, "checkpoint buffer too small");
  std::memcpy(&h, buf, sizeof h);
  if (h.magic != kCkptMagic || h.ny != d.ny || h.nx != d.nx || h.zmode != d.zmode ||
      h.has_z2 != d.has_z2 || h.t < 0 || bytes < checkpoint_bytes(j))
    return Status::fail(PNPULA_EINVAL, "checkpoint does not match this chain");
  const uint8_t *p = static_cast<const uint8_t *>(buf) + sizeof h;
  const float *f = reinterpret_cast<const float *>(p);
  HIPOK(hipStreamSynchronize(stream));
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  HIPOK(hipMemcpy2D(d.x[h.t & 1] + origin, (size_t)d.xpitch * sizeof(float), f,
                    (size_t)d.nx * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                    hipMemcpyHostToDevice));
  f += N;
  if (d.zmode != 0) {
    TRY(set_z(j, f, d.has_z2 ? f + N : nullptr));
    f += (d.has_z2 ? 2 : 1) * N;
  }
  HIPOK(hipMemcpy(d.wmean, f, N * sizeof(float), hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(d.wm2, f + N, N * sizeof(float), hipMemcpyHostToDevice));
  const double *g = reinterpret_cast<const double *>(f + 2 * N);
  HIPOK(hipMemcpy(d.mean, g, N * sizeof(double), hipMemcpyHostToDevice));
  HIPOK(hipMemcpy(d.m2, g + N, N * sizeof(double), hipMemcpyHostToDevice));
  j->t = h.t;
  d.wbase = h.wbase;
  d.nbase = h.nbase;
  TRY(upload_descs());
  return Status::ok();
}

Status Engine::get_z(Job *j, float *z1, float *z2) {
  const JobDesc &d = j->d;
  if (d.zmode == 0) return Status::fail(PNPULA_ESTATE, "the chain holds no z");
  HIPOK(hipStreamSynchronize(stream));
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  float *dst[2] = {z1, z2};
  const float *src[2] = {d.z1, d.z2};
  for (int i = 0; i < 2; ++i) {
    if (!dst[i]) continue;
    if (!src[i]) {
      std::fill(dst[i], dst[i] + (size_t)d.ny * d.nx, 0.0f);
      continue;
    }
    HIPOK(hipMemcpy2D(dst[i], (size_t)d.nx * sizeof(float), src[i] + origin,
                      (size_t)d.xpitch * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                      hipMemcpyDeviceToHost));
  }
  return Status::ok();
}

Status Engine::set_z(Job *j, const float *z1, const float *z2) {
  const JobDesc &d = j->d;
  if (d.zmode == 0) return Status::fail(PNPULA_ESTATE, "the chain holds no z");
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  const float *src[2] = {z1, z2};
  float *dst[2] = {d.z1, d.z2};
  for (int i = 0; i < 2; ++i) {
    if (!src[i] || !dst[i]) continue;
    HIPOK(hipMemcpy2DAsync(dst[i] + origin, (size_t)d.xpitch * sizeof(float), src[i],
                           (size_t)d.nx * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                           hipMemcpyHostToDevice, stream));
  }
  HIPOK(hipStreamSynchronize(stream));
  return Status::ok();
}

Status Engine::stats_device(Job *j, float *mean, float *var, int64_t *n) {
  int64_t total = 0;
  TRY(flush_stats(j, &total));
  HIPOK(launch_stats_out(j->d, total, mean, var, stream));
  HIPOK(hipStreamSynchronize(stream));
  if (n) *n = total;
  return Status::ok();
}

// Output of layer k (k < K - 1) held in activation buffer `slot`,
// dequantised to FP32 (value = code x the next layer's input scale), as
// channels planes of ny*nx (CHW).
Status Engine::read_act(Job *j, int k, int slot, float *dst) {
  const JobDesc &d = j->d;
  const LayerPlan &L = net.layers[k];
  const int ob = fmt_bytes(L.out_fmt), C = L.cout;
  const size_t pixb = (size_t)net.F * ob, N = (size_t)d.ny * d.nx;
  HIPOK(hipStreamSynchronize(stream));
  std::vector<uint8_t> buf((size_t)d.ny * d.nx * C * ob);
  const uint8_t *src = reinterpret_cast<const uint8_t *>(d.act[slot]);
  HIPOK(hipMemcpy2D(buf.data(), (size_t)d.nx * C * ob, src + ((size_t)d.apitch + 1) * pixb,
                    (size_t)d.apitch * pixb, (size_t)d.nx * C * ob, d.ny, hipMemcpyDeviceToHost));
  const float sc = net.act_scales[k + 1];
  for (size_t p = 0; p < N; ++p)
    for (int c = 0; c < C; ++c) {
      const uint8_t *e = &buf[(p * C + c) * ob];
      float v;
      if (L.out_fmt == FMT_F32) {
        std::memcpy(&v, e, 4);
      } else if (L.out_fmt == FMT_BF16) {
        uint32_t u = (uint32_t)(e[0] | (e[1] << 8)) << 16;
        std::memcpy(&v, &u, 4);
      } else {
        v = host_e4m3_to_f32(e[0]) * sc;
      }
      dst[(size_t)c * N + p] = v;
    }
  return Status::ok();
}

// The sampler's denoiser path on x, recording the activation each launch
// writes: stage i is the output of layer stage_layer[i], dequantised, as
// channels planes (CHW) at stage_acts + i * F * ny * nx.
Status Engine::denoise_stages(Job *j, const float *x, float *G, int32_t *n_stages,
                              int32_t *stage_layer, float *stage_acts) {
  if (plan_dirty) TRY(rebuild_plan());
  if (resident.size() != 1 || resident[0] != j)
    return Status::fail(PNPULA_ESTATE, "denoise needs a single-job engine");
  JobDesc &d = j->d;
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  const int64_t alt = j->t + 1;
  HIPOK(hipMemcpy2DAsync(d.x[alt & 1] + origin, (size_t)d.xpitch * sizeof(float), x,
                         (size_t)d.nx * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                         hipMemcpyHostToDevice, stream));
  const size_t plane = (size_t)net.F * d.ny * d.nx;
  int n = 0;
  StageFn fn = [&](int layer, int slot) -> Status {
    if (stage_layer) stage_layer[n] = layer;
    if (stage_acts) TRY(read_act(j, layer, slot, stage_acts + (size_t)n * plane));
    ++n;
    return Status::ok();
  };
  TRY(run_fused_denoiser(ticks + 1, false, &fn));
  HIPOK(hipStreamSynchronize(stream));
  if (G) HIPOK(hipMemcpy(G, d.G, (size_t)d.ny * d.nx * sizeof(float), hipMemcpyDeviceToHost));
  if (n_stages) *n_stages = n;
  return Status::ok();
}

// Run the denoiser of job j on a given image (placed in the ping-pong
// buffer that does not hold x^(t)); optionally read back every layer
// (dequantised) or the largest |input| of every layer.
Status Engine::denoise(Job *j, const float *x, float *G, float *layers, float *amax) {
  if (plan_dirty) TRY(rebuild_plan());
  if (resident.size() != 1 || resident[0] != j)
    return Status::fail(PNPULA_ESTATE, "denoise needs a single-job engine");
  JobDesc &d = j->d;
  const size_t origin = (size_t)d.xborder * d.xpitch + d.xborder;
  const int64_t alt = j->t + 1;       // parity of the spare buffer
  HIPOK(hipMemcpy2DAsync(d.x[alt & 1] + origin, (size_t)d.xpitch * sizeof(float), x,
                         (size_t)d.nx * sizeof(float), (size_t)d.nx * sizeof(float), d.ny,
                         hipMemcpyHostToDevice, stream));
  const int64_t tick_alt = ticks + 1;  // t = tick + t_offset = j->t + 1
  if (net.prior != PNPULA_PRIOR_CNN) {
    if (net.prior != PNPULA_PRIOR_DDFB || layers || amax)
      return Status::fail(PNPULA_ESTATE, "this prior has no denoiser to apply");
    TRY(run_prior_other(tick_alt));
    HIPOK(hipStreamSynchronize(stream));
    if (G) HIPOK(hipMemcpy(G, d.G, (size_t)d.ny * d.nx * sizeof(float), hipMemcpyDeviceToHost));
    return Status::ok();
  }
  const int K = net.K;
  const size_t N = (size_t)d.ny * d.nx;
  if (amax) {
    float m = 0.f;
    for (size_t p = 0; p < N; ++p) m = std::max(m, std::fabs(x[p]));
    amax[0] = m;
  }
  uint32_t *d_amax = nullptr;
  if (amax && K > 1) HIPOK(hipMalloc(&d_amax, sizeof(uint32_t) * K));
  struct Free {
    uint32_t *p;
    ~Free() { if (p) hipFree(p); }
  } guard{d_amax};
  if (d_amax) HIPOK(hipMemsetAsync(d_amax, 0, sizeof(uint32_t) * K, stream));
  float *lp = layers;
  int k0 = 0;
  if (!layers && !amax) {                         // the path the sampler runs
    TRY(run_fused_denoiser(tick_alt, false));
    k0 = K;
  }
  for (int k = k0; k < K; ++k) {
    const LayerPlan &L = net.layers[k];
    TRY(launch_layer(k, tick_alt, false));
    if (k == K - 1) break;
    const int C = L.cout;
    if (d_amax) {
      if (L.out_fmt != FMT_F32)
        return Status::fail(PNPULA_ESTATE, "calibration runs on an FP32 denoiser");
      HIPOK(launch_amax(reinterpret_cast<const float *>(d.act[L.out_buf]),
                        (size_t)(d.ny + 2 + 16) * d.apitch * net.F, d_amax + k + 1, stream));
    }
    if (lp) {
      TRY(read_act(j, k, L.out_buf, lp));
      lp += (size_t)C * N;
    }
  }
  HIPOK(hipStreamSynchronize(stream));
  if (lp) HIPOK(hipMemcpy(lp, d.G, N * sizeof(float), hipMemcpyDeviceToHost));
  if (G) HIPOK(hipMemcpy(G, d.G, N * sizeof(float), hipMemcpyDeviceToHost));
  if (d_amax) {
    std::vector<uint32_t> h(K);
    HIPOK(hipMemcpy(h.data(), d_amax, sizeof(uint32_t) * K, hipMemcpyDeviceToHost));
    for (int k = 1; k < K; ++k) std::memcpy(&amax[k], &h[k], 4);
  }
  return Status::ok();
}

}  // namespace pnp
