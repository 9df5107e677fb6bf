/*
 * pnpula.h -- C ABI of the MI355X plug-and-play ULA sampler (libpnpula.so).
 *
 * One context = one Markov chain of the split-Gibbs PnP-ULA sampler of
 * arXiv 2511.00870 (Sec. II-C, Eq. (sgs_pnp_ula_psgla:pnp_ula) and
 * Algorithm 1) for a grayscale image observed through y = m * (K x + noise):
 *
 *   z^(t) | x^(t)  ~ N((rho y + sigma^2 H x)/(rho + sigma^2),
 *                      rho sigma^2/(rho + sigma^2) I)         (rho > 0, t >= 1;
 *                                                               z^(0) = 0)
 *   x^(t+1) = x - delta H^T (H x - v)/s2 - (alpha delta/eps) G(x)
 *             + delta inv_lambda (clip_[0,1](x) - x) + sqrt(2 delta) xi
 *
 * with H = diag(m) K, (v, s2) = (y, sigma^2) when rho == 0 and (z, rho)
 * when rho > 0 (approximate data augmentation, Eq.
 * (general_posterior_l2_axda) with the Gaussian data term as f2), the
 * denoiser D_eps = Id - G (DnCNN form, Sec. II-B1 Example 2: a stack of
 * 3x3 convolutions with zero "half" padding, ReLU on all but the last
 * layer), and online Welford mean / variance of the samples after burn-in
 * (the MMSE estimate and the pixel-wise variance map, Sec. III-C).
 *
 * The image is split into blocks of block_y x block_x pixels with a halo
 * of `halo` pixels (Sec. II-A Defs. 1-2; Sec. II-B2): every block is
 * computed from its extended window of the previous iterate, which stays in
 * device memory, so the ghost-region exchange is an overlapping read.
 *
 * Noise: Philox4x32-10 (Salmon et al., SC'11), key = seed (low word, high
 * word), counter = (pixel mod 2^32, t, chain, pixel >> 32) with pixel = row
 * * nx + col; Box-Muller on u1 = ((w0 >> 8) + 1) 2^-24, u2 = (w1 >> 8) 2^-24:
 * xi = sqrt(-2 ln u1) cos(2 pi u2) and zeta = sqrt(-2 ln u1) sin(2 pi u2).
 *
 * Conventions for every call:
 *  - Host pointers unless stated otherwise.  Inputs are borrowed for the call
 *    and copied; outputs are caller-allocated.
 *  - Images are row-major ny x nx, float32 unless stated otherwise.
 *  - Status codes are returned; nothing throws or aborts across the ABI.
 *    pnpula_last_error() describes the last failure of a context, and
 *    pnpula_create_error() the last failed pnpula_create on this thread.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Work is queued on the context's HIP stream; calls that return data
 *    synchronise that stream first.
 */
#ifndef PNPULA_H
#define PNPULA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pnpula_ctx pnpula_ctx;

typedef enum {
  PNPULA_OK = 0,
  PNPULA_EINVAL = -1,     /* invalid argument or configuration */
  PNPULA_ENOMEM = -2,     /* device allocation failed / over the memory budget */
  PNPULA_EDEVICE = -3,    /* HIP runtime error or no usable gfx950 device */
  PNPULA_ESTATE = -4,     /* call not valid in the current state */
  PNPULA_EDIVERGED = -5   /* a sample became non-finite */
} pnpula_status;

/* arithmetic of the denoiser convolutions (chain state, likelihood
 * gradient and noise are always FP32; statistics are merged in FP64) */
typedef enum {
  PNPULA_FP32 = 0,        /* FP32 inputs and weights, FP32 accumulation */
  PNPULA_BF16 = 1,        /* bf16 (RNE) inputs and weights, FP32 accumulation */
  PNPULA_FP8_E4M3 = 2     /* OCP e4m3fn (RNE, saturating) inputs and weights with
                             per-output-channel power-of-two weight scales and
                             per-layer power-of-two activation scales; first and
                             last layer bf16; FP32 accumulation */
} pnpula_precision;

/* data terms (Sec. III-A) */
typedef enum { PNPULA_LIK_GAUSSIAN = 0, PNPULA_LIK_POISSON = 1 } pnpula_likelihood;

/* priors (Sec. II-B1, III-B): the residual CNN D = Id - G (Example 2); the
 * TV prior through AXDA with the x-chain kept in R+ (Sec. III-B2): the
 * x-step's prior term is (1/rho) D^T (D x - z), z = (zh, zv) held as state
 * and moved by the PSGLA step with the block soft threshold, and the
 * x-update ends with max(., 0) (the data term is not split; kappa, rho and
 * beta parameterise z); the DDFB denoiser (Example 3, Eqs. (ddfb_operator),
 * (dfb_operator:T)) with G = x - D(x). */
typedef enum { PNPULA_PRIOR_CNN = 0, PNPULA_PRIOR_TV = 1, PNPULA_PRIOR_DDFB = 2 } pnpula_prior;

typedef struct {
  int32_t ny, nx;                 /* image size (pixels) */
  const float *y;                 /* ny*nx observation, zero where mask == 0 */
  int32_t ksize;                  /* odd blur size L, 1 <= L <= 129 (above 17: the
                                     large-blur path, Sec. III-A2 motion blurs) */
  const float *kernel;            /* L*L blur, row-major; applied as a same-size
                                     linear convolution with zero boundary */
  const uint8_t *mask;            /* ny*nx of {0,1} applied after the blur; NULL:
                                     every pixel observed */
  double sigma;                   /* noise standard deviation (> 0) */
  double eps;                     /* denoiser level, variance convention (> 0):
                                     the prior term is (alpha delta/eps) G(x) */
  double alpha;                   /* prior weight (>= 0) */
  double delta;                   /* Langevin step (> 0) */
  double rho;                     /* splitting parameter (>= 0; 0: no z) */
  double inv_lambda;              /* 1/lambda of the [0,1] projection term (>= 0) */
  int32_t block_y, block_x;       /* block size (>= 1); blocks tile the image,
                                     the last row/column of blocks may be smaller */
  int32_t halo;                   /* ghost-region width, >= max(2 r, prior radius)
                                     with r = ksize/2 (prior radius: n_layers for the
                                     CNN, 1 for TV, 2 ddfb_layers for DDFB), and
                                     < min(block_y, block_x) unless a single block
                                     covers the image */
  int32_t n_layers;               /* denoiser depth K >= 1 (CNN prior only) */
  const int32_t *channels;        /* K+1 entries, channels[0] = channels[K] = 1,
                                     inner entries equal F in {16, 32, 64}
                                     (FP32) or {32, 64} (BF16) or 64 (FP8) */
  const float *weights;           /* per layer OIHW [c_out][c_in][3][3], layers
                                     concatenated (cross-correlation, as conv2d) */
  const float *biases;            /* per layer [c_out], concatenated */
  int32_t precision;              /* pnpula_precision */
  const float *act_scales;        /* K entries: power-of-two scale of each layer's
                                     input for e4m3 layers (others ignored);
                                     required for PNPULA_FP8_E4M3, else NULL */
  uint64_t seed;                  /* Philox key */
  uint32_t chain;                 /* Philox counter word 2 (independent chains) */
  int32_t burn_in;                /* samples x^(t) with t > burn_in enter the stats */
  int32_t welford_window;         /* FP32 Welford window before each FP64 merge
                                     (1..65536; 0: 256) */
  const float *x0;                /* ny*nx initial state; NULL: zeros */
  void *stream;                   /* hipStream_t to run on; NULL: a new stream */
  /* ---- the paper's other data terms and priors (all zero: the chain above).
   * PSGLA z-steps (Eq. (sgs_pnp_ula_psgla:psgla), Algorithm 1): z1 ~ eta m K x
   * carries the data term f, optionally z2 ~ x carries the indicator of R+;
   * both are chain state (z^(0) = 0) and move after each x-update by
   *   z <- prox_{kappa f}(z - (kappa/rho)(z - A x) + sqrt(2 kappa) zeta);
   * the x-step's data gradient is eta K^T m (eta m K x - z1)/rho
   * + (x - z2)/rho2. ---- */
  int32_t likelihood;             /* PNPULA_LIK_GAUSSIAN: f = (y - .)^2/(2 sigma^2);
                                     PNPULA_LIK_POISSON: y holds counts and
                                     f = KL(y || .) (Sec. III-A3); needs z_step 1 */
  int32_t z_step;                 /* 0: exact conditional draw of z (rho > 0) or no
                                     z (rho = 0); 1: PSGLA, z held as state */
  double eta;                     /* operator scale of z1 (Poisson: photon level;
                                     0 is taken as 1) */
  double kappa;                   /* PSGLA step of z1 (TV: of z), 0 < kappa <= rho */
  double rho2, kappa2;            /* second block (rho2 = 0: none) and its step */
  int32_t prior;                  /* pnpula_prior */
  double beta;                    /* TV weight: f = beta ||.||_{2,1} on z ~ D x */
  int32_t ddfb_layers;            /* DDFB iterations K (1..8) */
  int32_t ddfb_features;          /* DDFB feature maps F (1..64) */
  const float *ddfb_weights;      /* K blocks of [F][3][3]: W_k maps 1 -> F channels
                                     (cross-correlation, zero padding) */
  const float *ddfb_gamma;        /* K step sizes gamma_k */
  double ddfb_thresh;             /* hard-tanh level of the dual variables (>= 0) */
  int32_t inputs_on_device;       /* 1: y, kernel, mask and x0 are device pointers
                                     (read once at create); 0: host pointers */
} pnpula_config;

/* Validate cfg, allocate device memory, upload inputs and repack weights.
 * On success *out holds a context at t = 0 (the inputs of Algorithm 1: y,
 * the operator, the step sizes and splitting parameters, x^(0); z^(0) = 0
 * as in Sec. III-B). */
pnpula_status pnpula_create(const pnpula_config *cfg, pnpula_ctx **out);

/* Queue n_iters >= 0 iterations x^(t) -> x^(t+1) on the stream (asynchronous):
 * each is one pass of Algorithm 1 over every block (Eq.
 * (sgs_pnp_ula_psgla:pnp_ula) for x, Eq. (sgs:marginal_z) or Eq.
 * (sgs_pnp_ula_psgla:psgla) for z), followed by the statistics update. */
pnpula_status pnpula_step(pnpula_ctx *ctx, int32_t n_iters);

/* Wait for queued work; PNPULA_EDIVERGED if any sample so far was non-finite. */
pnpula_status pnpula_sync(pnpula_ctx *ctx);

/* MMSE estimate and pixel variance M2/(n-1) of the samples after burn-in
 * (the Monte Carlo estimates of Sec. III-C; FP64 merge of the FP32 windows,
 * rounded to FP32).  mean/var may be NULL.  n_samples receives n (var is 0
 * when n < 2). */
pnpula_status pnpula_stats(pnpula_ctx *ctx, float *mean, float *var, int64_t *n_samples);

/* Same statistics in FP64: mean and the sum of squared deviations M2. */
pnpula_status pnpula_stats_f64(pnpula_ctx *ctx, double *mean, double *m2, int64_t *n_samples);

/* State of the chain (not a passage of the paper: parity checks and
 * restarts).  The state is (x^(t), t) plus the statistics. */
pnpula_status pnpula_get_state(pnpula_ctx *ctx, float *x, int64_t *t);
/* Replace x and t (statistics are kept). */
pnpula_status pnpula_set_state(pnpula_ctx *ctx, const float *x, int64_t t);
/* Replace x, t and the FP64 statistics (mean, m2 of n samples). */
pnpula_status pnpula_restore(pnpula_ctx *ctx, const float *x, int64_t t, const double *mean,
                             const double *m2, int64_t n_samples);

/* Gradient of the Gaussian data-fidelity term at an arbitrary image x:
 *   g = H^T (H x - y) / sigma^2,   H = diag(m) K
 * (Eq. (potential_gaussian_likelihood); Sec. III-A1, III-A2) for the
 * context's observation y, blur K (any size up to 129 x 129) and mask m,
 * whatever the context's splitting.  x and g: host arrays of ny*nx floats.
 * Runs as two whole-image correlation passes (residual, then adjoint) on the
 * context's stream through device buffers allocated for the call; returns
 * after g is written.  PNPULA_ESTATE for a Poisson chain. */
pnpula_status pnpula_data_grad(pnpula_ctx *ctx, const float *x, float *g);

/* pnpula_data_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  x and g are DEVICE pointers of ny*nx floats.  The residual
 * lives in the library's static device buffer of PNPULA_NOALLOC_MAX_PIXELS
 * floats (32 MiB), one per GPU, held until the process ends; larger images
 * return PNPULA_EINVAL.  The call allocates nothing and queues its two
 * passes on the context's stream without synchronising (pnpula_sync waits).
 * Every call on one GPU shares that buffer: calls that overlap in time on
 * one GPU (e.g. on two streams) race; serialise them. */
#define PNPULA_NOALLOC_MAX_PIXELS (1 << 23)
pnpula_status pnpula_data_grad_noalloc(pnpula_ctx *ctx, const float *x, float *g);

/* Splitting variables held as chain state (PSGLA z-steps, Eq.
 * (sgs_pnp_ula_psgla:psgla); TV: z = (zh, zv) ~ D x, Sec. III-B2): z1 and z2
 * (ny*nx each; either may be NULL) of the current iterate.  PNPULA_ESTATE
 * when the chain holds no z (z_step 0 and prior not TV). */
pnpula_status pnpula_get_z(pnpula_ctx *ctx, float *z1, float *z2);
/* Replace z1 and z2 (either may be NULL: kept). */
pnpula_status pnpula_set_z(pnpula_ctx *ctx, const float *z1, const float *z2);

/* pnpula_stats with DEVICE outputs: mean and var (ny*nx floats each, either
 * may be NULL) are device pointers written on the context's stream, which
 * is synchronised before return. */
pnpula_status pnpula_stats_device(pnpula_ctx *ctx, float *mean, float *var, int64_t *n_samples);

/* Checkpoint of the whole chain state, for a resume that continues bit for
 * bit as if the chain had never stopped (the statistics' merge schedule
 * included): x^(t) and t, the splitting variables held as state, the FP32
 * Welford window as it stands and the FP64 statistics merged so far, in one
 * opaque host buffer of pnpula_checkpoint_size bytes.  Taking a checkpoint
 * does not change the chain. */
pnpula_status pnpula_checkpoint_size(pnpula_ctx *ctx, size_t *bytes);
pnpula_status pnpula_checkpoint(pnpula_ctx *ctx, void *buf, size_t bytes);
/* Load a checkpoint taken from a context of the same configuration (image
 * size, z-step and prior; PNPULA_EINVAL otherwise). */
pnpula_status pnpula_resume(pnpula_ctx *ctx, const void *buf, size_t bytes);

/* Apply the context's denoiser to an ny*nx image: G = x - D_eps(x) (FP32
 * output; Sec. II-B1, Eqs. (feedforward_cnn), (cnn:convolution), Example 2,
 * or the DDFB denoiser of Example 3).  layers (optional) receives every layer's output, dequantised
 * to FP32, as channels[k+1] planes of ny*nx per layer (CHW), concatenated. */
pnpula_status pnpula_denoise(pnpula_ctx *ctx, const float *x, float *G, float *layers);

/* The sampler's own (fused) denoiser path applied to an ny*nx image x, with
 * the activation written to memory by each of its launches returned for
 * inspection (Sec. II-B1, Eq. (cnn:convolution): each launch computes one
 * layer or two consecutive layers; the first and last layers may run inside
 * the launches next to them).  G receives x - D_eps(x) (FP32, may be NULL).
 * *n_stages receives the number of launches that wrote an activation;
 * stage_layer[i] the index (0-based) of the last layer launch i computed;
 * stage_acts + i * F * ny * nx its output dequantised to FP32 (value = code x
 * the next layer's activation scale), F planes of ny*nx (CHW).  stage_layer
 * needs n_layers entries and stage_acts (n_layers - 1) * F * ny * nx floats;
 * either may be NULL. */
pnpula_status pnpula_denoise_stages(pnpula_ctx *ctx, const float *x, float *G, int32_t *n_stages,
                                    int32_t *stage_layer, float *stage_acts);

/* Largest |input| of every layer when the denoiser (in FP32) is applied to
 * x: the data for choosing e4m3 activation scales (not in the paper: the
 * low-precision form). */
pnpula_status pnpula_calibrate(pnpula_ctx *ctx, const float *x, float *amax);

/* Per-kernel timing with HIP events on the context's stream (measurement,
 * not in the paper).  Classes:
 * 0 = middle convolution layers, 1 = first layer, 2 = last layer,
 * 3 = fused likelihood/update/statistics kernel, 4 = first layer fused with
 * the first middle layer, 5 = last middle layer writing the last layer's
 * per-tap partials (both bf16 networks; class 2 then times the kernel that
 * sums the partials into G), 6 = two consecutive middle layers in one
 * kernel (bf16 and e4m3 networks; for e4m3 the first pair also runs the first
 * layer and the last pair the last layer's partials, class 2 again timing the
 * sums), 7 = the prior term of the TV and DDFB chains (TV coupling term;
 * each DDFB stage), 8 = the z-steps held as state (PSGLA, TV), 9 = the
 * whole-image correlation passes of large blurs.  Enabling resets totals. */
pnpula_status pnpula_profile(pnpula_ctx *ctx, int32_t enable);
pnpula_status pnpula_profile_read(pnpula_ctx *ctx, int32_t kernel_class, double *total_ms,
                                  int64_t *launches);

/* Device pointer of the current x^(t) (padded layout: row pitch in floats
 * in *pitch, image origin at element *offset), for zero-copy consumers (not
 * in the paper). */
pnpula_status pnpula_state_device(pnpula_ctx *ctx, const float **base, int64_t *pitch,
                                  int64_t *offset);

void pnpula_destroy(pnpula_ctx *ctx);
const char *pnpula_last_error(const pnpula_ctx *ctx);
const char *pnpula_create_error(void);

/* Device memory one context of this configuration allocates (bytes); the
 * serving admission test (not in the paper). */
pnpula_status pnpula_footprint(const pnpula_config *cfg, size_t *bytes);

/* ------------------------------------------------------------------ *
 * Serving: many chains of different sizes share one denoiser and one
 * stream.  Each tick advances every resident job by one iteration with
 * one launch per kernel over all resident jobs' tiles.  Jobs are admitted
 * first-in first-out while their footprint fits the memory budget and a
 * slot is free, and retire when their iteration count is reached.  A job's
 * result does not depend on its co-residents.
 * ------------------------------------------------------------------ */
typedef struct pnpula_server pnpula_server;

/* weights/biases/channels/precision/act_scales as in pnpula_config;
 * hbm_budget bytes (0: no limit) for the jobs' footprints; max_slots >= 1;
 * stream as in pnpula_config. */
pnpula_status pnpula_server_create(int32_t n_layers, const int32_t *channels,
                                   const float *weights, const float *biases,
                                   int32_t precision, const float *act_scales,
                                   size_t hbm_budget, int32_t max_slots, void *stream,
                                   pnpula_server **out);
/* Queue a job (the network fields of cfg are ignored; cfg->stream too).
 * n_iters >= 1.  Inputs are copied.  *job_id identifies it. */
pnpula_status pnpula_server_submit(pnpula_server *s, const pnpula_config *cfg, int32_t n_iters,
                                   int64_t *job_id);
/* Admit, run one tick, retire.  *active receives the number of resident
 * plus queued jobs after the tick. */
pnpula_status pnpula_server_tick(pnpula_server *s, int32_t *active);
/* 1 when the job has finished (result available), 0 otherwise. */
pnpula_status pnpula_server_poll(pnpula_server *s, int64_t job_id, int32_t *done);
/* Statistics of a finished job (as pnpula_stats); releases the result. */
pnpula_status pnpula_server_result(pnpula_server *s, int64_t job_id, float *mean, float *var,
                                   int64_t *n_samples);
pnpula_status pnpula_server_run_until_idle(pnpula_server *s);
void pnpula_server_destroy(pnpula_server *s);
const char *pnpula_server_last_error(const pnpula_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PNPULA_H */
