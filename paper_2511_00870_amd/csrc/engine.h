// engine.h -- host runtime of the PnP-ULA sampler: the shared denoiser,
// resident chains (jobs), block/tile plans and the per-iteration launch
// sequence.  A context is an engine with one job; the server is an engine
// with a scheduler in front of it.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/pnpula.h"
#include "kernels.h"

namespace pnp {

struct Status {
  pnpula_status code = PNPULA_OK;
  std::string msg;
  static Status ok() { return {}; }
  static Status fail(pnpula_status c, std::string m) { return {c, std::move(m)}; }
  bool good() const { return code == PNPULA_OK; }
};

// One layer of the denoiser as the kernels consume it.
struct LayerPlan {
  int cin = 0, cout = 0;
  int in_fmt = FMT_F32;     // format of the layer's input and weights
  int out_fmt = FMT_F32;    // format the output is stored in (next layer's input)
  int relu = 0;
  int unit_scale = 0;        // every output scale is 1 (no e4m3 weight or input scale)
  float in_inv_scale = 1.f, out_inv_scale = 1.f;
  float in_scale = 1.f;     // scale of the stored input (e4m3), else 1
  int in_buf = 0, out_buf = 0;  // activation buffers read / written
  void *wblob = nullptr;    // middle layers: MFMA fragment order
  void *wblob_rr = nullptr; // e4m3 middle layers: row-reuse kernel's fragment order
  void *wblob_sl = nullptr; // e4m3 middle layers: sliding tap pairs (split-layer pair kernel)
  float *wf32 = nullptr;    // first / last layer: [c][9]
  float *bias = nullptr, *oscale = nullptr;
};

struct NetPlan {
  int K = 0, F = 0, precision = PNPULA_FP32;
  std::vector<int> channels;
  std::vector<float> weights, biases, act_scales;  // host copies
  std::vector<LayerPlan> layers;
  int buf_fmt[4] = {-1, -1, -1, -1};  // storage format of each activation buffer
  bool last_fused = false;   // the last layer runs inside the last middle layer's kernel
  bool last_pair8 = false;   // e4m3: the last layer runs inside the last pair's kernel
  std::vector<void *> allocs;
  // prior of the chain: PNPULA_PRIOR_CNN (the layers above), _TV or _DDFB
  int prior = PNPULA_PRIOR_CNN;
  int ddfb_K = 0, ddfb_F = 0;
  float ddfb_thresh = 0.f;
  std::vector<float> ddfb_gamma;
  float *ddfb_w = nullptr;   // device: K x F x 9
};

struct Job {
  JobDesc d{};              // host mirror of the device descriptor
  int64_t t = 0;            // current iteration
  int block_y = 0, block_x = 0, halo = 0;
  int64_t target = 0;       // serving: iterations to run
  int64_t id = 0;
  bool diverged = false;
  size_t footprint = 0;
  std::vector<void *> allocs;
  std::vector<TileRef> conv_tiles, upd_tiles;   // job field = 0 (set at planning)
  std::vector<TileRef> pair_tiles;              // e4m3 pair kernel: whole-image tiling
  std::vector<TileRef> pair_ws_tiles;           // split-layer pair kernel (bf16)
  std::vector<TileRef> pair8ws_tiles;           // split-layer pair kernel (e4m3)
  std::vector<TileRef> ddfb_tiles;              // DDFB stages: whole-image tiling
};

struct ProfileRec {
  int cls;
  hipEvent_t a, b;
};

class Engine {
 public:
  ~Engine();
  Status init(void *stream);
  Status set_net(int K, const int32_t *channels, const float *w, const float *b, int precision,
                 const float *act_scales);
  // TV or DDFB prior in place of the CNN (cfg's prior fields)
  Status set_prior(const pnpula_config *cfg);
  static Status validate_job(const pnpula_config *cfg, int K, const std::vector<int> &ch);
  // receptive-field radius of the prior term for cfg
  static int prior_radius(const pnpula_config *cfg);
  static size_t job_footprint(const pnpula_config *cfg, const NetPlan &net);
  Status make_job(const pnpula_config *cfg, Job **out);
  void free_job(Job *j);

  // run one iteration of every resident job
  Status tick();
  Status sync_check(bool *diverged);
  Status upload_descs();
  Status rebuild_plan();

  // single-job helpers
  Status get_state(Job *j, float *x);
  Status set_state(Job *j, const float *x, int64_t t);
  Status flush_stats(Job *j, int64_t *n_total);
  Status read_stats(Job *j, double *mean, double *m2, int64_t *n);
  Status restore_stats(Job *j, const double *mean, const double *m2, int64_t n);
  Status denoise(Job *j, const float *x, float *G, float *layers, float *amax);
  Status denoise_stages(Job *j, const float *x, float *G, int32_t *n_stages,
                        int32_t *stage_layer, float *stage_acts);
  Status read_act(Job *j, int k, int slot, float *dst);
  Status data_grad(Job *j, const float *x, float *g, float *res);
  size_t checkpoint_bytes(const Job *j) const;
  Status checkpoint(Job *j, void *buf, size_t bytes);
  Status resume(Job *j, const void *buf, size_t bytes);
  Status get_z(Job *j, float *z1, float *z2);
  Status set_z(Job *j, const float *z1, const float *z2);
  Status stats_device(Job *j, float *mean, float *var, int64_t *n);

  void profile_enable(bool on);
  Status profile_read(int cls, double *ms, int64_t *launches);

  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0, n_cu = 0;
  NetPlan net;
  std::vector<Job *> resident;
  int64_t ticks = 0;
  bool plan_dirty = true;
  std::string err;

 private:
  Status run_denoiser(int64_t tick);
  bool first_mid_fused() const;
  Status launch_first_mid(int64_t tick, bool prof);
  Status launch_mid_last(int k, int in_slot, int64_t tick, bool first, bool prof);
  Status launch_pair(int k, int in_slot, int out_slot, int64_t tick, bool prof,
                     bool first = false, bool last = false);
  bool pair_ok(int k) const;
  bool first_pair8_ok() const;
  bool first8_ok() const;
  Status launch_first8(int64_t tick, bool prof);
  Status launch_g_from_s(int64_t tick, bool prof);
  // called after each launch of the fused path that writes an activation
  // buffer: (index of the last layer it computed, buffer)
  using StageFn = std::function<Status(int, int)>;
  Status run_fused_denoiser(int64_t tick, bool prof, const StageFn *on_stage = nullptr);
  Status launch_layer(int k, int64_t tick, bool prof, int in_slot = -1, int out_slot = -1);
  Status run_prior_other(int64_t tick);
  JobDesc *d_jobs = nullptr;
  TileRef *d_conv = nullptr, *d_upd = nullptr, *d_pair = nullptr, *d_pair_ws = nullptr,
          *d_pair8ws = nullptr, *d_ddfb = nullptr;
  size_t cap_jobs = 0, cap_conv = 0, cap_upd = 0, cap_pair = 0, cap_pair_ws = 0, cap_pair8ws = 0,
         cap_ddfb = 0;
  int n_conv = 0, n_upd = 0, n_pair = 0, n_pair_ws = 0, n_pair8ws = 0, n_ddfb = 0, max_r = 0;
  bool uniform_r = true;      // every resident job has blur half-width max_r
  int zmode = 0;              // JobDesc::zmode of the resident jobs (all equal)
  bool big = false;           // the resident jobs take the large-blur path
  int max_kpitch = 8;
  int conv_th = 16;
  bool profiling = false;
  std::vector<ProfileRec> prof_pending;
  std::vector<hipEvent_t> prof_free;
  static constexpr int kProfClasses = 10;
  double prof_ms[kProfClasses] = {};
  int64_t prof_n[kProfClasses] = {};
  void prof_begin(int cls, ProfileRec *r);
  void prof_end(ProfileRec *r);
};

// host-side rounding used when repacking weights (round to nearest even)
float host_round_bf16(float v);
uint8_t host_f32_to_e4m3(float v);
float host_e4m3_to_f32(uint8_t c);
float host_pow2_scale(float amax);
bool host_is_pow2(float v);

}  // namespace pnp
