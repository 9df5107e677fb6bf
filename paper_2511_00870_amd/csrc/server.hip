// server.hip -- continuous batching of many sampling jobs on one GPU.
//
// Jobs (chains of different image sizes, operators and lengths) share the
// engine's denoiser.  Each tick: admit queued jobs first-in first-out while a
// slot is free and their footprint fits the memory budget; run one
// iteration of every resident job with one launch per kernel over the union
// of their tiles; retire jobs that reached their iteration count (FP64 merge
// of their statistics, results kept on the host, device memory released).
// Each tile is computed from its own job's data only and the generator is
// keyed per job and pixel, so a job's result does not depend on the jobs it
// shares the device with.
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "engine.h"

using pnp::Engine;
using pnp::Job;
using pnp::Status;

namespace {

struct Pending {
  int64_t id = 0;
  int32_t n_iters = 0;
  pnpula_config cfg{};
  std::vector<float> y, kernel, x0;
  std::vector<uint8_t> mask;
  size_t footprint = 0;
};

struct Result {
  int32_t ny = 0, nx = 0;
  std::vector<double> mean, m2;
  int64_t n = 0;
  pnpula_status status = PNPULA_OK;
  std::string msg;
};

}  // namespace

struct pnpula_server {
  Engine eng;
  std::deque<Pending> queue;
  std::map<int64_t, Result> done;
  size_t budget = 0, used = 0;
  int32_t max_slots = 1;
  int64_t next_id = 1;
  std::string err;
};

static pnpula_status sreport(pnpula_server *s, const Status &st) {
  if (!st.good() && s) s->err = st.msg;
  return st.code;
}

static Status admit(pnpula_server *s) {
  while (!s->queue.empty() && (int32_t)s->eng.resident.size() < s->max_slots) {
    Pending &p = s->queue.front();
    if (s->budget && p.footprint > s->budget) {
      Result r;
      r.status = PNPULA_ENOMEM;
      r.msg = "job footprint exceeds the memory budget";
      s->done[p.id] = std::move(r);
      s->queue.pop_front();
      continue;
    }
    if (s->budget && s->used + p.footprint > s->budget) break;   // wait for memory
    Job *j = nullptr;
    Status st = s->eng.make_job(&p.cfg, &j);
    if (!st.good()) {
      if (st.code == PNPULA_ENOMEM && !s->eng.resident.empty()) break;  // retry later
      Result r;
      r.status = st.code;
      r.msg = st.msg;
      s->done[p.id] = std::move(r);
      s->queue.pop_front();
      continue;
    }
    j->id = p.id;
    j->target = p.n_iters;
    s->used += j->footprint;
    s->eng.resident.push_back(j);
    s->eng.plan_dirty = true;
    s->queue.pop_front();
  }
  return Status::ok();
}

static Status retire(pnpula_server *s) {
  std::vector<Job *> keep;
  bool changed = false;
  for (Job *j : s->eng.resident) {
    if (j->t < j->target) {
      keep.push_back(j);
      continue;
    }
    Result r;
    r.ny = j->d.ny;
    r.nx = j->d.nx;
    const size_t N = (size_t)r.ny * r.nx;
    r.mean.resize(N);
    r.m2.resize(N);
    Status st = s->eng.read_stats(j, r.mean.data(), r.m2.data(), &r.n);
    int32_t flag = 0;
    if (st.good() && hipMemcpy(&flag, j->d.flag, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
      st = Status::fail(PNPULA_EDEVICE, "flag read failed");
    if (!st.good()) {
      r.status = st.code;
      r.msg = st.msg;
    } else if (flag) {
      r.status = PNPULA_EDIVERGED;
      r.msg = "a sample became non-finite";
    }
    s->done[j->id] = std::move(r);
    s->used -= j->footprint;
    s->eng.free_job(j);
    changed = true;
  }
  if (changed) {
    s->eng.resident = keep;
    s->eng.plan_dirty = true;
  }
  return Status::ok();
}

extern "C" {

pnpula_status pnpula_server_create(int32_t n_layers, const int32_t *channels, const float *weights,
                                   const float *biases, int32_t precision,
                                   const float *act_scales, size_t hbm_budget, int32_t max_slots,
                                   void *stream, pnpula_server **out) {
  if (!out) return PNPULA_EINVAL;
  *out = nullptr;
  if (max_slots < 1) return PNPULA_EINVAL;
  pnpula_server *s = new (std::nothrow) pnpula_server();
  if (!s) return PNPULA_ENOMEM;
  Status st = s->eng.init(stream);
  if (st.good()) st = s->eng.set_net(n_layers, channels, weights, biases, precision, act_scales);
  if (!st.good()) {
    pnpula_status c = st.code;
    delete s;
    return c;
  }
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  *out = s;
  return PNPULA_OK;
}

pnpula_status pnpula_server_submit(pnpula_server *s, const pnpula_config *cfg, int32_t n_iters,
                                   int64_t *job_id) {
  if (!s || !cfg || !job_id) return PNPULA_EINVAL;
  if (n_iters < 1) return sreport(s, Status::fail(PNPULA_EINVAL, "n_iters must be >= 1"));
  Status st = Engine::validate_job(cfg, s->eng.net.K, s->eng.net.channels);
  if (!st.good()) return sreport(s, st);
  // jobs share one launch per kernel: the server's CNN denoiser, the exact z
  // draw (or none) and the fused blur path; inputs are copied from the host
  if (cfg->prior != PNPULA_PRIOR_CNN || cfg->z_step != 0 || cfg->ksize > 2 * pnp::kMaxR + 1 ||
      cfg->inputs_on_device)
    return sreport(s, Status::fail(PNPULA_EINVAL,
                                   "served jobs use the CNN prior, no PSGLA z-step, blurs up to "
                                   "17 x 17 and host inputs"));
  Pending p;
  p.id = s->next_id++;
  p.n_iters = n_iters;
  p.cfg = *cfg;
  const size_t N = (size_t)cfg->ny * cfg->nx;
  p.y.assign(cfg->y, cfg->y + N);
  p.kernel.assign(cfg->kernel, cfg->kernel + (size_t)cfg->ksize * cfg->ksize);
  if (cfg->mask) p.mask.assign(cfg->mask, cfg->mask + N);
  if (cfg->x0) p.x0.assign(cfg->x0, cfg->x0 + N);
  p.cfg.y = p.y.data();
  p.cfg.kernel = p.kernel.data();
  p.cfg.mask = cfg->mask ? p.mask.data() : nullptr;
  p.cfg.x0 = cfg->x0 ? p.x0.data() : nullptr;
  p.cfg.stream = nullptr;
  p.footprint = Engine::job_footprint(cfg, s->eng.net);
  *job_id = p.id;
  s->queue.push_back(std::move(p));
  return PNPULA_OK;
}

pnpula_status pnpula_server_tick(pnpula_server *s, int32_t *active) {
  if (!s) return PNPULA_EINVAL;
  Status st = admit(s);
  if (st.good() && !s->eng.resident.empty()) st = s->eng.tick();
  if (st.good()) st = retire(s);
  if (active) *active = (int32_t)(s->eng.resident.size() + s->queue.size());
  return sreport(s, st);
}

pnpula_status pnpula_server_poll(pnpula_server *s, int64_t job_id, int32_t *done) {
  if (!s || !done) return PNPULA_EINVAL;
  *done = s->done.count(job_id) ? 1 : 0;
  return PNPULA_OK;
}

pnpula_status pnpula_server_result(pnpula_server *s, int64_t job_id, float *mean, float *var,
                                   int64_t *n_samples) {
  if (!s) return PNPULA_EINVAL;
  auto it = s->done.find(job_id);
  if (it == s->done.end()) return sreport(s, Status::fail(PNPULA_ESTATE, "job not finished"));
  Result &r = it->second;
  if (r.status != PNPULA_OK) {
    pnpula_status c = r.status;
    s->err = r.msg;
    s->done.erase(it);
    return c;
  }
  const size_t N = (size_t)r.ny * r.nx;
  for (size_t p = 0; p < N; ++p) {
    if (mean) mean[p] = (float)r.mean[p];
    if (var) var[p] = r.n >= 2 ? (float)(r.m2[p] / (double)(r.n - 1)) : 0.0f;
  }
  if (n_samples) *n_samples = r.n;
  s->done.erase(it);
  return PNPULA_OK;
}

pnpula_status pnpula_server_run_until_idle(pnpula_server *s) {
  if (!s) return PNPULA_EINVAL;
  int32_t active = 1;
  while (active > 0) {
    pnpula_status c = pnpula_server_tick(s, &active);
    if (c != PNPULA_OK) return c;
    if (s->eng.resident.empty() && !s->queue.empty()) {
      // nothing resident and the head job cannot be admitted
      return sreport(s, Status::fail(PNPULA_ENOMEM, "queued job can never be admitted"));
    }
  }
  return PNPULA_OK;
}

void pnpula_server_destroy(pnpula_server *s) { delete s; }

const char *pnpula_server_last_error(const pnpula_server *s) {
  return s ? s->err.c_str() : "null server";
}

}  // extern "C"
