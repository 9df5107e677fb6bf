/*
 * oracle.h -- plain FP64 CPU oracle of the plug-and-play Langevin sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product library
 * never calls it and shares no code with it.
 *
 * What it computes (paper: Sec. II-C, Eqs. (general_posterior_l2_axda),
 * (sgs:marginal_z), (sgs_pnp_ula_psgla:pnp_ula), Algorithm 1; denoiser: Sec.
 * II-B1, Eqs. (feedforward_cnn), (cnn:convolution), Example 2 (DnCNN);
 * blocks: Sec. II-A Defs. 1-2 and Sec. II-B2 overlap-save):
 *
 *   z^(t) | x^(t) ~ N((rho y + sigma^2 H x)/(rho + sigma^2),
 *                     rho sigma^2/(rho + sigma^2) I)      (t >= 1; z^(0) = 0)
 *   g      = H^T (H x - v) / s2,  (v, s2) = (y, sigma^2) if rho = 0
 *                                          (z, rho)     if rho > 0
 *   x^(t+1) = x - delta g - (alpha delta/eps) G(x)
 *             + delta inv_lambda (clip_[0,1](x) - x) + sqrt(2 delta) xi
 *
 * with H = diag(m) K (blur K: same-size linear convolution, zero boundary;
 * m: {0,1} mask), D_eps = Id - G, G a stack of 3x3 cross-correlation layers
 * with zero ("half") padding at every layer, ReLU on all but the last.
 * eps uses the variance convention (the prior term's coefficient is
 * alpha delta / eps).  Gaussian draws: Philox4x32-10 keyed by the seed, with
 * counter (pixel mod 2^32, t, chain, pixel >> 32), Box-Muller on two 24-bit
 * uniforms: xi from the cosine branch, zeta from the sine branch.
 *
 * Every floating-point quantity is FP64.  An optional quantisation mode
 * rounds each layer's input activations and weights to bf16 or OCP e4m3fn
 * (round-to-nearest-even, e4m3 saturating at +-448) with power-of-two
 * scales, so that low-precision layers can be checked one by one.
 */
#ifndef PNP_ORACLE_H
#define PNP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FMT_EXACT = 0, OR_FMT_BF16 = 1, OR_FMT_E4M3 = 2 };

typedef struct {
  int32_t n_layers;
  const int32_t *channels;   /* n_layers + 1 entries, first and last = 1 */
  const double *weights;     /* per layer OIHW [cout][cin][3][3], concatenated */
  const double *biases;      /* per layer [cout], concatenated */
  const int32_t *layer_fmt;  /* NULL: exact; else per-layer input/weight format */
  const double *act_scales;  /* per-layer input scale (power of two) for e4m3 */
} oracle_net;

typedef struct {
  int32_t ny, nx;
  const double *y;           /* ny*nx observation */
  int32_t ksize;             /* odd L */
  const double *kernel;      /* L*L, row-major */
  const uint8_t *mask;       /* NULL: every pixel observed */
  double sigma, eps, alpha, delta, rho, inv_lambda;
  int32_t block_y, block_x, halo;  /* blocks >= image: single block */
  oracle_net net;
  uint64_t seed;
  uint32_t chain;
  int32_t burn_in;
  const double *x0;          /* NULL: zeros */
  /* likelihood and splitting variable (Sec. III-A, Eq. (sgs_pnp_ula_psgla:psgla)) */
  int32_t likelihood;        /* 0 Gaussian, 1 Poisson: f = KL(y || .) */
  int32_t z_step;            /* 0 exact Gaussian conditional draw, 1 PSGLA */
  double eta;                /* operator eta diag(m) K (0 is taken as 1) */
  double kappa;              /* PSGLA step of the z block coupled to the operator */
  double rho2, kappa2;       /* second block z2 ~ x, f = indicator of R+ (rho2 = 0: none) */
  /* prior (Sec. II-B1 Examples 2-3, Sec. III-B2) */
  int32_t prior;             /* 0 residual CNN, 1 TV (PSGLA), 2 DDFB */
  double beta;               /* TV weight */
  int32_t ddfb_layers, ddfb_features;
  const double *ddfb_weights;  /* K blocks of [F][3][3]: W_k maps 1 -> F channels */
  const double *ddfb_gamma;    /* K step sizes gamma_k */
  double ddfb_thresh;          /* hard-tanh level */
} oracle_config;

typedef struct oracle_chain oracle_chain;

/* ---- chain (returns NULL and writes err on invalid input) ---- */
oracle_chain *oracle_create(const oracle_config *cfg, char *err, int errlen);
int  oracle_step(oracle_chain *c, int32_t n_iters);          /* 0 ok, -5 non-finite */
void oracle_get_state(const oracle_chain *c, double *x, int64_t *t);
void oracle_set_state(oracle_chain *c, const double *x, int64_t t);
void oracle_stats(const oracle_chain *c, double *mean, double *m2, int64_t *n);
void oracle_record_z(oracle_chain *c, int32_t on);           /* keep z of each step */
void oracle_last_z(const oracle_chain *c, double *z);        /* z used by last step */
/* state z^(t) of the PSGLA and TV chains (z1: the block coupled to the
 * operator, or the horizontal differences for TV; z2: the second block, or
 * the vertical differences); either may be NULL */
void oracle_get_z(const oracle_chain *c, double *z1, double *z2);
void oracle_set_z(oracle_chain *c, const double *z1, const double *z2);
void oracle_destroy(oracle_chain *c);
int  oracle_num_threads(void);

/* ---- primitives ---- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void oracle_gauss_pair(uint32_t w0, uint32_t w1, double *xi, double *zeta);
void oracle_noise(int32_t ny, int32_t nx, uint64_t seed, uint32_t t, uint32_t chain,
                  double *xi, double *zeta);
void oracle_blur(const double *x, int32_t ny, int32_t nx, const double *k, int32_t L,
                 double *out);
void oracle_blur_adjoint(const double *r, int32_t ny, int32_t nx, const double *k,
                         int32_t L, double *out);
void oracle_conv3x3(const double *in, int32_t cin, int32_t ny, int32_t nx,
                    const double *w, const double *b, int32_t cout, int32_t relu,
                    double *out);
double oracle_quantize(double v, int32_t fmt);
void oracle_quantize_n(const double *v, int64_t n, int32_t fmt, double scale, double *out);
void oracle_weight_scales(const oracle_net *net, int32_t layer, double *scales);
int  oracle_denoiser(const oracle_net *net, const double *x, int32_t ny, int32_t nx,
                     int32_t block_y, int32_t block_x, int32_t halo, double *G);
int  oracle_denoise_region(const oracle_net *net, const double *x, int32_t ny, int32_t nx,
                           int32_t y0, int32_t x0, int32_t h, int32_t w, double *G);
int  oracle_denoiser_layers(const oracle_net *net, const double *x, int32_t ny,
                            int32_t nx, double *acts, double *amax);
int  oracle_layers_from(const oracle_net *net, const double *in, int32_t ny, int32_t nx,
                        int32_t k0, int32_t k1, double *acts, double *amax);
int  oracle_data_grad(const oracle_config *cfg, const double *x, int64_t t, double *g);
int  oracle_step_region(const oracle_config *cfg, const double *x, int64_t t, int32_t y0,
                        int32_t x0, int32_t h, int32_t w, double *xnew);
int  oracle_step_region_z(const oracle_config *cfg, const double *x, const double *z1,
                          const double *z2, int64_t t, int32_t y0, int32_t x0, int32_t h,
                          int32_t w, double *xnew);
/* the DDFB denoiser D(v) of Eq. (ddfb_operator) on a whole image */
int  oracle_ddfb(const oracle_config *cfg, const double *v, int32_t ny, int32_t nx,
                 double *out);
/* the 2-D forward-difference operator D and its adjoint */
void oracle_grad2d(const double *x, int32_t ny, int32_t nx, double *dh, double *dv);
void oracle_grad2d_adjoint(const double *dh, const double *dv, int32_t ny, int32_t nx,
                           double *out);
/* proximity operators used by the z-steps (elementwise / per pixel) */
double oracle_prox_kl(double v, double y, double kappa);
double oracle_prox_gauss(double v, double y, double sigma, double kappa);
void oracle_prox_l21(double *vh, double *vv, double tau);

#ifdef __cplusplus
}
#endif
#endif
