// api.hip -- C ABI of libpnpula.so (contexts).  Every entry point converts
// internal failures into status codes; nothing throws across the boundary.
#include <cstring>
#include <new>
#include <string>

#include "engine.h"

using pnp::Engine;
using pnp::Job;
using pnp::Status;

struct pnpula_ctx {
  Engine eng;
  Job *job = nullptr;
  std::string err;
};

static thread_local std::string g_create_error;

static pnpula_status report(pnpula_ctx *c, const Status &s) {
  if (!s.good() && c) c->err = s.msg;
  return s.code;
}

#define GUARD(ctx)                                                 \
  if (!(ctx)) return PNPULA_EINVAL;                                \
  if (!(ctx)->job) return report(ctx, Status::fail(PNPULA_ESTATE, "context has no chain"))

extern "C" {

pnpula_status pnpula_create(const pnpula_config *cfg, pnpula_ctx **out) {
  if (!out) return PNPULA_EINVAL;
  *out = nullptr;
  if (!cfg) {
    g_create_error = "null config";
    return PNPULA_EINVAL;
  }
  pnpula_ctx *c = new (std::nothrow) pnpula_ctx();
  if (!c) return PNPULA_ENOMEM;
  Status s = Engine::validate_job(cfg, cfg->n_layers, {});
  const bool cnn = cfg->prior == PNPULA_PRIOR_CNN;
  if (s.good() && cnn && (cfg->n_layers < 1 || !cfg->channels))
    s = Status::fail(PNPULA_EINVAL, "denoiser missing");
  if (s.good()) s = c->eng.init(cfg->stream);
  if (s.good())
    s = cnn ? c->eng.set_net(cfg->n_layers, cfg->channels, cfg->weights, cfg->biases,
                             cfg->precision, cfg->act_scales)
            : c->eng.set_prior(cfg);
  if (s.good()) s = c->eng.make_job(cfg, &c->job);
  if (s.good()) {
    c->eng.resident.push_back(c->job);
    s = c->eng.rebuild_plan();
  }
  if (!s.good()) {
    g_create_error = s.msg;
    delete c;
    return s.code;
  }
  *out = c;
  return PNPULA_OK;
}

pnpula_status pnpula_step(pnpula_ctx *c, int32_t n_iters) {
  GUARD(c);
  if (n_iters < 0) return report(c, Status::fail(PNPULA_EINVAL, "n_iters must be >= 0"));
  for (int32_t i = 0; i < n_iters; ++i) {
    Status s = c->eng.tick();
    if (!s.good()) return report(c, s);
  }
  return PNPULA_OK;
}

pnpula_status pnpula_sync(pnpula_ctx *c) {
  GUARD(c);
  bool div = false;
  Status s = c->eng.sync_check(&div);
  if (!s.good()) return report(c, s);
  if (div) return report(c, Status::fail(PNPULA_EDIVERGED, "a sample became non-finite"));
  return PNPULA_OK;
}

pnpula_status pnpula_stats_f64(pnpula_ctx *c, double *mean, double *m2, int64_t *n) {
  GUARD(c);
  return report(c, c->eng.read_stats(c->job, mean, m2, n));
}

pnpula_status pnpula_stats(pnpula_ctx *c, float *mean, float *var, int64_t *n_samples) {
  GUARD(c);
  const size_t N = (size_t)c->job->d.ny * c->job->d.nx;
  double *m = nullptr, *q = nullptr;
  try {
    m = new double[N];
    q = new double[N];
  } catch (...) {
    delete[] m;
    return report(c, Status::fail(PNPULA_ENOMEM, "host allocation failed"));
  }
  int64_t n = 0;
  Status s = c->eng.read_stats(c->job, m, q, &n);
  if (s.good()) {
    for (size_t p = 0; p < N; ++p) {
      if (mean) mean[p] = (float)m[p];
      if (var) var[p] = n >= 2 ? (float)(q[p] / (double)(n - 1)) : 0.0f;
    }
    if (n_samples) *n_samples = n;
  }
  delete[] m;
  delete[] q;
  return report(c, s);
}

pnpula_status pnpula_get_state(pnpula_ctx *c, float *x, int64_t *t) {
  GUARD(c);
  if (x) {
    Status s = c->eng.get_state(c->job, x);
    if (!s.good()) return report(c, s);
  }
  if (t) *t = c->job->t;
  return PNPULA_OK;
}

pnpula_status pnpula_set_state(pnpula_ctx *c, const float *x, int64_t t) {
  GUARD(c);
  if (!x) return report(c, Status::fail(PNPULA_EINVAL, "x is required"));
  return report(c, c->eng.set_state(c->job, x, t));
}

pnpula_status pnpula_restore(pnpula_ctx *c, const float *x, int64_t t, const double *mean,
                             const double *m2, int64_t n) {
  GUARD(c);
  if (!x || !mean || !m2) return report(c, Status::fail(PNPULA_EINVAL, "x, mean, m2 are required"));
  Status s = c->eng.set_state(c->job, x, t);
  if (s.good()) s = c->eng.restore_stats(c->job, mean, m2, n);
  return report(c, s);
}

pnpula_status pnpula_data_grad(pnpula_ctx *c, const float *x, float *g) {
  GUARD(c);
  if (!x || !g) return report(c, Status::fail(PNPULA_EINVAL, "x and g are required"));
  const size_t bytes = (size_t)c->job->d.ny * c->job->d.nx * sizeof(float);
  float *buf = nullptr;                       // x, residual, g
  if (hipMalloc(&buf, 3 * bytes) != hipSuccess) {
    (void)hipGetLastError();
    return report(c, Status::fail(PNPULA_ENOMEM, "device allocation failed"));
  }
  const size_t n = bytes / sizeof(float);
  hipStream_t st = c->eng.stream;
  Status s = Status::ok();
  if (hipMemcpyAsync(buf, x, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    s = Status::fail(PNPULA_EDEVICE, "copy of x failed");
  if (s.good()) s = c->eng.data_grad(c->job, buf, buf + 2 * n, buf + n);
  if (s.good() && (hipMemcpyAsync(g, buf + 2 * n, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess))
    s = Status::fail(PNPULA_EDEVICE, "data gradient failed");
  hipStreamSynchronize(st);
  hipFree(buf);
  return report(c, s);
}

pnpula_status pnpula_data_grad_noalloc(pnpula_ctx *c, const float *x, float *g) {
  GUARD(c);
  if (!x || !g) return report(c, Status::fail(PNPULA_EINVAL, "x and g are required"));
  if ((int64_t)c->job->d.ny * c->job->d.nx > pnp::kNoallocMaxPixels)
    return report(c, Status::fail(PNPULA_EINVAL, "image larger than the static buffer (" +
                                                     std::to_string(pnp::kNoallocMaxPixels) +
                                                     " pixels)"));
  float *res = pnp::noalloc_scratch(c->eng.device);
  if (!res) return report(c, Status::fail(PNPULA_EDEVICE, "static buffer not set up"));
  return report(c, c->eng.data_grad(c->job, x, g, res));
}

pnpula_status pnpula_checkpoint_size(pnpula_ctx *c, size_t *bytes) {
  GUARD(c);
  if (!bytes) return report(c, Status::fail(PNPULA_EINVAL, "bytes is required"));
  *bytes = c->eng.checkpoint_bytes(c->job);
  return PNPULA_OK;
}

pnpula_status pnpula_checkpoint(pnpula_ctx *c, void *buf, size_t bytes) {
  GUARD(c);
  if (!buf) return report(c, Status::fail(PNPULA_EINVAL, "buf is required"));
  return report(c, c->eng.checkpoint(c->job, buf, bytes));
}

pnpula_status pnpula_resume(pnpula_ctx *c, const void *buf, size_t bytes) {
  GUARD(c);
  if (!buf) return report(c, Status::fail(PNPULA_EINVAL, "buf is required"));
  return report(c, c->eng.resume(c->job, buf, bytes));
}

pnpula_status pnpula_get_z(pnpula_ctx *c, float *z1, float *z2) {
  GUARD(c);
  return report(c, c->eng.get_z(c->job, z1, z2));
}

pnpula_status pnpula_set_z(pnpula_ctx *c, const float *z1, const float *z2) {
  GUARD(c);
  return report(c, c->eng.set_z(c->job, z1, z2));
}

pnpula_status pnpula_stats_device(pnpula_ctx *c, float *mean, float *var, int64_t *n_samples) {
  GUARD(c);
  return report(c, c->eng.stats_device(c->job, mean, var, n_samples));
}

pnpula_status pnpula_denoise(pnpula_ctx *c, const float *x, float *G, float *layers) {
  GUARD(c);
  if (!x) return report(c, Status::fail(PNPULA_EINVAL, "x is required"));
  return report(c, c->eng.denoise(c->job, x, G, layers, nullptr));
}

pnpula_status pnpula_denoise_stages(pnpula_ctx *c, const float *x, float *G, int32_t *n_stages,
                                    int32_t *stage_layer, float *stage_acts) {
  GUARD(c);
  if (!x) return report(c, Status::fail(PNPULA_EINVAL, "x is required"));
  return report(c, c->eng.denoise_stages(c->job, x, G, n_stages, stage_layer, stage_acts));
}

pnpula_status pnpula_calibrate(pnpula_ctx *c, const float *x, float *amax) {
  GUARD(c);
  if (!x || !amax) return report(c, Status::fail(PNPULA_EINVAL, "x and amax are required"));
  // a temporary FP32 engine with the same denoiser and image size
  Engine tmp;
  const pnp::NetPlan &n = c->eng.net;
  Status s = tmp.init(c->eng.stream);
  if (s.good())
    s = tmp.set_net(n.K, n.channels.data(), n.weights.data(), n.biases.data(), PNPULA_FP32,
                    nullptr);
  pnpula_config cfg{};
  const float one = 1.0f;
  cfg.ny = c->job->d.ny;
  cfg.nx = c->job->d.nx;
  cfg.y = x;
  cfg.ksize = 1;
  cfg.kernel = &one;
  cfg.sigma = cfg.eps = cfg.delta = 1.0;
  cfg.block_y = cfg.ny;
  cfg.block_x = cfg.nx;
  cfg.n_layers = n.K;
  Job *j = nullptr;
  if (s.good()) s = tmp.make_job(&cfg, &j);
  if (s.good()) {
    tmp.resident.push_back(j);
    s = tmp.denoise(j, x, nullptr, nullptr, amax);
  }
  return report(c, s);
}

pnpula_status pnpula_profile(pnpula_ctx *c, int32_t enable) {
  GUARD(c);
  c->eng.profile_enable(enable != 0);
  return PNPULA_OK;
}

pnpula_status pnpula_profile_read(pnpula_ctx *c, int32_t cls, double *total_ms, int64_t *launches) {
  GUARD(c);
  return report(c, c->eng.profile_read(cls, total_ms, launches));
}

pnpula_status pnpula_state_device(pnpula_ctx *c, const float **base, int64_t *pitch,
                                  int64_t *offset) {
  GUARD(c);
  const pnp::JobDesc &d = c->job->d;
  if (base) *base = d.x[c->job->t & 1];
  if (pitch) *pitch = d.xpitch;
  if (offset) *offset = (int64_t)d.xborder * d.xpitch + d.xborder;
  return PNPULA_OK;
}

void pnpula_destroy(pnpula_ctx *c) { delete c; }

const char *pnpula_last_error(const pnpula_ctx *c) { return c ? c->err.c_str() : "null context"; }

const char *pnpula_create_error(void) { return g_create_error.c_str(); }

pnpula_status pnpula_footprint(const pnpula_config *cfg, size_t *bytes) {
  if (!cfg || !bytes) return PNPULA_EINVAL;
  Status s = Engine::validate_job(cfg, cfg->n_layers, {});
  if (!s.good()) {
    g_create_error = s.msg;
    return s.code;
  }
  pnp::NetPlan n;
  n.K = cfg->prior == PNPULA_PRIOR_CNN ? cfg->n_layers : 0;
  n.F = (n.K > 1 && cfg->channels) ? cfg->channels[1] : 1;
  // activation buffers as the engine assigns them (see Engine::set_net)
  if (n.K > 1) {
    if (cfg->precision == PNPULA_FP8_E4M3) {
      n.buf_fmt[0] = pnp::FMT_E4M3;
      if (n.K > 3) n.buf_fmt[1] = pnp::FMT_E4M3;
      n.buf_fmt[n.K > 3 ? 2 : 1] = pnp::FMT_BF16;
    } else {
      const int f = cfg->precision == PNPULA_BF16 ? pnp::FMT_BF16 : pnp::FMT_F32;
      n.buf_fmt[0] = f;
      if (n.K > 2) n.buf_fmt[1] = f;
    }
  }
  *bytes = Engine::job_footprint(cfg, n);
  return PNPULA_OK;
}

}  // extern "C"
