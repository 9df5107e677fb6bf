/*
 * oracle.c -- plain FP64 CPU oracle of the plug-and-play Langevin sampler.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product library, and sharing
 * no code with it.  Readability over speed: every operator is a direct sum in
 * a fixed order (no FFT, no blocking beyond the paper's own blocks), and the
 * only parallelism is OpenMP over independent output rows/channels, which
 * does not change any result.
 *
 * Paper references (arXiv 2511.00870):
 *   - posterior and splitting: Sec. II-C, Eq. (general_posterior_l2_axda),
 *     conditionals (sgs:marginal_x), (sgs:marginal_z);
 *   - PnP-ULA x-transition: Eq. (sgs_pnp_ula_psgla:pnp_ula), Algorithm 1;
 *   - Gaussian likelihood, mask and blur operators: Sec. III-A1, III-A2,
 *     Eq. (likelihood:gaussian_inpainting), (potential_gaussian_likelihood);
 *   - CNN denoiser: Sec. II-B1 Eqs. (feedforward_cnn), (cnn:convolution),
 *     Example 2 (DnCNN: D = Id - G, ReLU except on the last layer);
 *   - blocks and halos: Sec. II-A Defs. 1-2 (local selection operators,
 *     localized operators), Sec. II-B2 (overlap-save: compute each block on
 *     its extended window and discard the entries with wrong boundary).
 *   - Philox4xW-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *     easy as 1, 2, 3", SC'11 (the paper does not name its generator).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ======================================================================
 * Philox4xW-10 (Salmon et al. SC'11, Sec. 4).  One round maps the counter
 * (X0, X1, X2, X3) with round key (K0, K1) to
 *   (hi(M1*X2) ^ X1 ^ K0, lo(M1*X2), hi(M0*X0) ^ X3 ^ K1, lo(M0*X0));
 * between rounds the key is bumped by the Weyl constants (W0, W1).
 * ==================================================================== */
#define PHILOX_ROUND_BODY(T, X, K, M0, M1, MULHI)            \
  do {                                                       \
    T hi0 = MULHI((M0), X[0]), lo0 = (T)((M0) * X[0]);       \
    T hi1 = MULHI((M1), X[2]), lo1 = (T)((M1) * X[2]);       \
    T n0 = hi1 ^ X[1] ^ K[0], n2 = hi0 ^ X[3] ^ K[1];        \
    X[0] = n0; X[1] = lo1; X[2] = n2; X[3] = lo0;            \
  } while (0)

static inline uint32_t mulhi32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}
static inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t X[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t K[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { K[0] += W0; K[1] += W1; }
    PHILOX_ROUND_BODY(uint32_t, X, K, M0, M1, mulhi32);
  }
  memcpy(out, X, sizeof X);
}

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t X[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint64_t K[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { K[0] += W0; K[1] += W1; }
    PHILOX_ROUND_BODY(uint64_t, X, K, M0, M1, mulhi64);
  }
  memcpy(out, X, sizeof X);
}

/* Box-Muller on two 24-bit uniforms u1 in (0,1], u2 in [0,1):
 * xi = sqrt(-2 ln u1) cos(2 pi u2), zeta = sqrt(-2 ln u1) sin(2 pi u2). */
void oracle_gauss_pair(uint32_t w0, uint32_t w1, double *xi, double *zeta) {
  const double two_m24 = 1.0 / 16777216.0;
  double u1 = (double)((w0 >> 8) + 1u) * two_m24;
  double u2 = (double)(w1 >> 8) * two_m24;
  double rad = sqrt(-2.0 * log(u1));
  double ang = 2.0 * M_PI * u2;
  *xi = rad * cos(ang);
  *zeta = rad * sin(ang);
}

/* The two Gaussian draws of pixel p at iteration t: xi^(t+1) (x-update,
 * Algorithm 1, "sample xi") and zeta^(t) (draw of z^(t)). */
static void draw_pixel(uint64_t seed, int64_t p, int64_t t, uint32_t chain,
                       double *xi, double *zeta) {
  uint32_t ctr[4] = {(uint32_t)p, (uint32_t)t, chain, (uint32_t)((uint64_t)p >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  oracle_philox4x32_10(ctr, key, w);
  oracle_gauss_pair(w[0], w[1], xi, zeta);
}

/* Three Gaussian draws of pixel p at counter t: the pair above from words
 * (w0, w1) and the cosine branch of a second Box-Muller pair from (w2, w3):
 * xi, the first z block's zeta and the second z block's zeta2. */
static void draw_pixel3(uint64_t seed, int64_t p, int64_t t, uint32_t chain, double *xi,
                        double *zeta, double *zeta2) {
  uint32_t ctr[4] = {(uint32_t)p, (uint32_t)t, chain, (uint32_t)((uint64_t)p >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  double unused;
  oracle_philox4x32_10(ctr, key, w);
  oracle_gauss_pair(w[0], w[1], xi, zeta);
  oracle_gauss_pair(w[2], w[3], zeta2, &unused);
}

void oracle_noise(int32_t ny, int32_t nx, uint64_t seed, uint32_t t, uint32_t chain,
                  double *xi, double *zeta) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < ny; ++i)
    for (int32_t j = 0; j < nx; ++j) {
      int64_t p = (int64_t)i * nx + j;
      draw_pixel(seed, p, t, chain, &xi[p], &zeta[p]);
    }
}

/* ======================================================================
 * Quantisation (round to nearest even).
 * bf16: 8 significant bits, exponent range of fp32 (subnormal step 2^-133).
 * e4m3fn (OCP): 4 significant bits, bias 7, min normal 2^-6, subnormal
 * step 2^-9, largest finite 448, no infinities: saturate to +-448.
 * ==================================================================== */
double oracle_quantize(double v, int32_t fmt) {
  if (fmt == OR_FMT_EXACT || v == 0.0 || isnan(v)) return v;
  if (fmt == OR_FMT_BF16) {
    if (isinf(v)) return v;
    int e;
    frexp(v, &e);
    int lead = e - 1;
    if (lead < -126) lead = -126;
    double ulp = ldexp(1.0, lead - 7);
    double q = nearbyint(v / ulp) * ulp;
    const double bmax = ldexp(255.0, 120); /* (2 - 2^-7) 2^127 */
    if (fabs(q) > bmax) q = copysign(INFINITY, v);
    return q;
  }
  /* e4m3fn */
  if (isinf(v)) return copysign(448.0, v);
  int e;
  frexp(v, &e);
  int lead = e - 1;
  if (lead < -6) lead = -6;
  double ulp = ldexp(1.0, lead - 3);
  double q = nearbyint(v / ulp) * ulp;
  if (q > 448.0) q = 448.0;
  if (q < -448.0) q = -448.0;
  return q;
}

/* out[i] = quantize(v[i] / scale) * scale for n values (the array form of
 * the rounding above, for checks over whole activation maps) */
void oracle_quantize_n(const double *v, int64_t n, int32_t fmt, double scale, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_quantize(v[i] / scale, fmt) * scale;
}

/* smallest power of two s with amax / s <= 448 (1 when amax == 0) */
static double pow2_scale(double amax) {
  if (!(amax > 0.0)) return 1.0;
  int e;
  double f = frexp(amax / 448.0, &e);
  return (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

static int layer_fmt(const oracle_net *n, int k) {
  return n->layer_fmt ? n->layer_fmt[k] : OR_FMT_EXACT;
}

static size_t weight_offset(const oracle_net *n, int k) {
  size_t off = 0;
  for (int i = 0; i < k; ++i) off += (size_t)n->channels[i] * n->channels[i + 1] * 9;
  return off;
}
static size_t bias_offset(const oracle_net *n, int k) {
  size_t off = 0;
  for (int i = 0; i < k; ++i) off += (size_t)n->channels[i + 1];
  return off;
}

/* per-output-channel weight scales of layer k (power of two for e4m3, else 1) */
void oracle_weight_scales(const oracle_net *n, int32_t k, double *scales) {
  int cin = n->channels[k], cout = n->channels[k + 1];
  const double *w = n->weights + weight_offset(n, k);
  for (int co = 0; co < cout; ++co) {
    if (layer_fmt(n, k) != OR_FMT_E4M3) { scales[co] = 1.0; continue; }
    double amax = 0.0;
    for (int i = 0; i < cin * 9; ++i) amax = fmax(amax, fabs(w[(size_t)co * cin * 9 + i]));
    scales[co] = pow2_scale(amax);
  }
}

/* ======================================================================
 * Valid-mode stencils on explicit arrays.  Zero boundaries are obtained by
 * padding the input with zeros before the call; a block's extended window
 * is obtained by copying the window (zeros outside the image).  Each output
 * is one sum in a fixed order, so results do not depend on which array the
 * stencil runs on.
 * ==================================================================== */

/* out[i][j] = sum_{a,c} k[a][c] in[i + L-1-a][j + L-1-c]: linear convolution
 * (flip) restricted to outputs whose support lies inside `in`. */
static void valid_conv(const double *in, int H, int W, const double *k, int L, double *out) {
  int Ho = H - L + 1, Wo = W - L + 1;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < Ho; ++i)
    for (int j = 0; j < Wo; ++j) {
      double acc = 0.0;
      for (int a = 0; a < L; ++a)
        for (int c = 0; c < L; ++c)
          acc += k[a * L + c] * in[(size_t)(i + L - 1 - a) * W + (j + L - 1 - c)];
      out[(size_t)i * Wo + j] = acc;
    }
}

/* out[i][j] = sum_{a,c} k[a][c] in[i + a][j + c]: the adjoint of valid_conv's
 * zero-boundary operator (correlation with the same kernel). */
static void valid_xcorr(const double *in, int H, int W, const double *k, int L, double *out) {
  int Ho = H - L + 1, Wo = W - L + 1;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < Ho; ++i)
    for (int j = 0; j < Wo; ++j) {
      double acc = 0.0;
      for (int a = 0; a < L; ++a)
        for (int c = 0; c < L; ++c)
          acc += k[a * L + c] * in[(size_t)(i + a) * W + (j + c)];
      out[(size_t)i * Wo + j] = acc;
    }
}

/* One CNN layer (Eq. (cnn:convolution)) on a valid region:
 *   out[co][i][j] = eta( oscale[co] * sum_ci sum_{a,c} w[co][ci][a][c]
 *                        in[ci][i+a][j+c]  +  b[co] )
 * in: [cin][H][W] -> out: [cout][H-2][W-2]; eta = ReLU if relu else Id.
 * Each output sums in the order (ci, a, c). */
static void valid_layer(const double *in, int cin, int H, int W, const double *w,
                        const double *b, const double *oscale, int cout, int relu,
                        double *out) {
  int Ho = H - 2, Wo = W - 2;
#pragma omp parallel for collapse(2) schedule(static)
  for (int co = 0; co < cout; ++co)
    for (int i = 0; i < Ho; ++i) {
      double *orow = out + ((size_t)co * Ho + i) * Wo;
      for (int j = 0; j < Wo; ++j) orow[j] = 0.0;
      for (int ci = 0; ci < cin; ++ci) {
        const double *wp = w + ((size_t)co * cin + ci) * 9;
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) {
            const double wv = wp[a * 3 + c];
            const double *irow = in + ((size_t)ci * H + i + a) * W + c;
            for (int j = 0; j < Wo; ++j) orow[j] += wv * irow[j];
          }
      }
      for (int j = 0; j < Wo; ++j) {
        double v = orow[j] * oscale[co] + b[co];
        if (relu && v < 0.0) v = 0.0;
        orow[j] = v;
      }
    }
}

/* copy a window [oy, oy+H) x [ox, ox+W) of C planes of an ny x nx image,
 * with zeros outside the image */
static void extract_window(const double *img, int C, int ny, int nx, int oy, int ox,
                           int H, int W, double *win) {
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < H; ++i)
      for (int j = 0; j < W; ++j) {
        int gi = oy + i, gj = ox + j;
        double v = 0.0;
        if (gi >= 0 && gi < ny && gj >= 0 && gj < nx)
          v = img[((size_t)c * ny + gi) * nx + gj];
        win[((size_t)c * H + i) * W + j] = v;
      }
}

/* zero the entries of a window that fall outside the image (half padding
 * at every layer, Eq. (cnn:convolution)) */
static void zero_outside(double *win, int C, int ny, int nx, int oy, int ox, int H, int W) {
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < H; ++i)
      for (int j = 0; j < W; ++j) {
        int gi = oy + i, gj = ox + j;
        if (gi < 0 || gi >= ny || gj < 0 || gj >= nx)
          win[((size_t)c * H + i) * W + j] = 0.0;
      }
}

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", n); abort(); }
  return p;
}

/* ======================================================================
 * Operators on whole images (zero boundary)
 * ==================================================================== */
void oracle_blur(const double *x, int32_t ny, int32_t nx, const double *k, int32_t L,
                 double *out) {
  int r = L / 2;
  int H = ny + 2 * r, W = nx + 2 * r;
  double *pad = xmalloc((size_t)H * W * sizeof(double));
  extract_window(x, 1, ny, nx, -r, -r, H, W, pad);
  valid_conv(pad, H, W, k, L, out);
  free(pad);
}

void oracle_blur_adjoint(const double *rr, int32_t ny, int32_t nx, const double *k,
                         int32_t L, double *out) {
  int r = L / 2;
  int H = ny + 2 * r, W = nx + 2 * r;
  double *pad = xmalloc((size_t)H * W * sizeof(double));
  extract_window(rr, 1, ny, nx, -r, -r, H, W, pad);
  valid_xcorr(pad, H, W, k, L, out);
  free(pad);
}

void oracle_conv3x3(const double *in, int32_t cin, int32_t ny, int32_t nx,
                    const double *w, const double *b, int32_t cout, int32_t relu,
                    double *out) {
  int H = ny + 2, W = nx + 2;
  double *pad = xmalloc((size_t)cin * H * W * sizeof(double));
  double *one = xmalloc((size_t)cout * sizeof(double));
  for (int c = 0; c < cout; ++c) one[c] = 1.0;
  extract_window(in, cin, ny, nx, -1, -1, H, W, pad);
  valid_layer(pad, cin, H, W, w, b, one, cout, relu, out);
  free(pad);
  free(one);
}

/* ======================================================================
 * Denoiser G = T_K o ... o T_1 on a window (Sec. II-B1, Example 2).
 * `win` holds channels[0] planes of size H x W whose global origin is
 * (oy, ox); each layer shrinks the valid region by one pixel per side and
 * re-zeroes what lies outside the image.  With quantisation, layer k rounds
 * its input (scaled by act_scales[k] for e4m3) and its weights (scaled per
 * output channel) to its format and rescales the exact sum.
 * Returns the final plane of size (H - 2K) x (W - 2K) in *res (caller frees).
 * ==================================================================== */
typedef struct {
  double *wq;      /* quantised weights, all layers */
  double *oscale;  /* per layer per output channel: s_w * s_a */
} prepared_net;

static void prepare_net(const oracle_net *n, prepared_net *p) {
  size_t nw = weight_offset(n, n->n_layers), nb = bias_offset(n, n->n_layers);
  p->wq = xmalloc(nw * sizeof(double));
  p->oscale = xmalloc(nb * sizeof(double));
  for (int k = 0; k < n->n_layers; ++k) {
    int cin = n->channels[k], cout = n->channels[k + 1], fmt = layer_fmt(n, k);
    const double *w = n->weights + weight_offset(n, k);
    double *wq = p->wq + weight_offset(n, k);
    double *os = p->oscale + bias_offset(n, k);
    oracle_weight_scales(n, k, os);
    double sa = (fmt == OR_FMT_E4M3 && n->act_scales) ? n->act_scales[k] : 1.0;
    for (int co = 0; co < cout; ++co) {
      for (int i = 0; i < cin * 9; ++i) {
        size_t idx = (size_t)co * cin * 9 + i;
        wq[idx] = oracle_quantize(w[idx] / os[co], fmt);
      }
      os[co] *= sa;
    }
  }
}

static void free_net(prepared_net *p) {
  free(p->wq);
  free(p->oscale);
}

static double *denoise_window(const oracle_net *n, const prepared_net *p, double *win,
                              int ny, int nx, int oy, int ox, int H, int W,
                              int keep_acts, double *acts_out, double *amax) {
  double *cur = win;
  int own = 0;
  for (int k = 0; k < n->n_layers; ++k) {
    int cin = n->channels[k], cout = n->channels[k + 1], fmt = layer_fmt(n, k);
    double sa = (fmt == OR_FMT_E4M3 && n->act_scales) ? n->act_scales[k] : 1.0;
    size_t nin = (size_t)cin * H * W;
    if (amax) {
      double m = 0.0;
      for (size_t i = 0; i < nin; ++i) m = fmax(m, fabs(cur[i]));
      amax[k] = m;
    }
    if (fmt != OR_FMT_EXACT) {
      if (!own) {  /* never modify the caller's window in place */
        double *cp = xmalloc(nin * sizeof(double));
        memcpy(cp, cur, nin * sizeof(double));
        cur = cp;
        own = 1;
      }
      for (size_t i = 0; i < nin; ++i) cur[i] = oracle_quantize(cur[i] / sa, fmt);
    }
    double *out = xmalloc((size_t)cout * (H - 2) * (W - 2) * sizeof(double));
    valid_layer(cur, cin, H, W, p->wq + weight_offset(n, k), n->biases + bias_offset(n, k),
                p->oscale + bias_offset(n, k), cout, k < n->n_layers - 1, out);
    if (own) free(cur);
    cur = out;
    own = 1;
    H -= 2; W -= 2; oy += 1; ox += 1;
    zero_outside(cur, cout, ny, nx, oy, ox, H, W);
    if (keep_acts) {  /* monolithic only: window == image after the layer */
      memcpy(acts_out, cur, (size_t)cout * H * W * sizeof(double));
      acts_out += (size_t)cout * H * W;
    }
  }
  return cur;
}

/* G(x) for the whole image.  block_y/block_x smaller than the image: each
 * block is computed from its own extended window of half-width `halo`
 * (one exchange of the whole receptive field, Sec. II-B2 last paragraph). */
int oracle_denoiser(const oracle_net *n, const double *x, int32_t ny, int32_t nx,
                    int32_t block_y, int32_t block_x, int32_t halo, double *G) {
  int K = n->n_layers;
  prepared_net p;
  prepare_net(n, &p);
  if (block_y <= 0 || block_x <= 0 || (block_y >= ny && block_x >= nx)) {
    int H = ny + 2 * K, W = nx + 2 * K;
    double *win = xmalloc((size_t)H * W * sizeof(double));
    extract_window(x, 1, ny, nx, -K, -K, H, W, win);
    double *res = denoise_window(n, &p, win, ny, nx, -K, -K, H, W, 0, NULL, NULL);
    memcpy(G, res, (size_t)ny * nx * sizeof(double));
    free(res);
    free(win);
  } else {
    if (halo < K) { free_net(&p); return -1; }
    for (int by = 0; by < ny; by += block_y)
      for (int bx = 0; bx < nx; bx += block_x) {
        int cy = (by + block_y <= ny) ? block_y : ny - by;
        int cx = (bx + block_x <= nx) ? block_x : nx - bx;
        int H = cy + 2 * halo, W = cx + 2 * halo;
        double *win = xmalloc((size_t)H * W * sizeof(double));
        extract_window(x, 1, ny, nx, by - halo, bx - halo, H, W, win);
        double *res = denoise_window(n, &p, win, ny, nx, by - halo, bx - halo, H, W, 0,
                                     NULL, NULL);
        int Hr = H - 2 * K, Wr = W - 2 * K, off = halo - K;
        for (int i = 0; i < cy; ++i)
          for (int j = 0; j < cx; ++j)
            G[(size_t)(by + i) * nx + bx + j] = res[(size_t)(i + off) * Wr + j + off];
        (void)Hr;
        free(res);
        free(win);
      }
  }
  free_net(&p);
  return 0;
}

/* G(x) on the region [y0, y0+h) x [x0, x0+w) of an ny x nx image, from the
 * region's extended window of half-width K (zeros outside the image): the
 * same window computation as a block, so sampled outputs of very large
 * images can be checked one region at a time. */
int oracle_denoise_region(const oracle_net *n, const double *x, int32_t ny, int32_t nx,
                          int32_t y0, int32_t x0, int32_t h, int32_t w, double *G) {
  if (y0 < 0 || x0 < 0 || h < 1 || w < 1 || y0 + h > ny || x0 + w > nx) return -1;
  int K = n->n_layers;
  prepared_net p;
  prepare_net(n, &p);
  int H = h + 2 * K, W = w + 2 * K;
  double *win = xmalloc((size_t)H * W * sizeof(double));
  extract_window(x, 1, ny, nx, y0 - K, x0 - K, H, W, win);
  double *res = denoise_window(n, &p, win, ny, nx, y0 - K, x0 - K, H, W, 0, NULL, NULL);
  memcpy(G, res, (size_t)h * w * sizeof(double));
  free(res);
  free(win);
  free_net(&p);
  return 0;
}

/* all layer outputs of the monolithic denoiser (layer k: channels[k+1]
 * planes), and the max |input| of every layer before its quantisation */
int oracle_denoiser_layers(const oracle_net *n, const double *x, int32_t ny, int32_t nx,
                           double *acts, double *amax) {
  return oracle_layers_from(n, x, ny, nx, 0, n->n_layers, acts, amax);
}

/* layers k0 .. k1-1 of the monolithic denoiser applied to `in` (the input of
 * layer k0: channels[k0] planes of ny x nx); acts receives their outputs as
 * in oracle_denoiser_layers, amax (optional) the max |input| of each */
int oracle_layers_from(const oracle_net *n, const double *in, int32_t ny, int32_t nx,
                       int32_t k0, int32_t k1, double *acts, double *amax) {
  int K = n->n_layers;
  if (k0 < 0 || k1 > K || k0 >= k1) return -1;
  prepared_net p;
  prepare_net(n, &p);
  const double *cur = in;
  for (int k = k0; k < k1; ++k) {
    int cin = n->channels[k], cout = n->channels[k + 1], fmt = layer_fmt(n, k);
    double sa = (fmt == OR_FMT_E4M3 && n->act_scales) ? n->act_scales[k] : 1.0;
    int H = ny + 2, W = nx + 2;
    size_t nin = (size_t)cin * H * W;
    double *pad = xmalloc(nin * sizeof(double));
    extract_window(cur, cin, ny, nx, -1, -1, H, W, pad);
    if (amax) {
      double m = 0.0;
      for (size_t i = 0; i < nin; ++i) m = fmax(m, fabs(pad[i]));
      amax[k - k0] = m;
    }
    if (fmt != OR_FMT_EXACT)
      for (size_t i = 0; i < nin; ++i) pad[i] = oracle_quantize(pad[i] / sa, fmt);
    valid_layer(pad, cin, H, W, p.wq + weight_offset(n, k), n->biases + bias_offset(n, k),
                p.oscale + bias_offset(n, k), cout, k < K - 1, acts);
    free(pad);
    cur = acts;
    acts += (size_t)cout * ny * nx;
  }
  free_net(&p);
  return 0;
}

/* ======================================================================
 * Likelihood gradient on a window (Eq. (sgs_pnp_ula_psgla:pnp_ula), the
 * data term; Algorithm 1 "u_1", "u_2"; closed-form z draw from
 * Eq. (sgs:marginal_z) with f2 the Gaussian data term, H2 = H):
 *   Kx on the window's valid region, then (t >= 1 and rho > 0)
 *   z = (rho y + sigma^2 m Kx)/(rho + sigma^2) + sqrt(rho sigma^2/(rho+sigma^2)) zeta,
 *   res = m (Kx - v) inside the image (0 outside), v = y or z,
 *   g = K^T res / s2 on the next valid region.
 * `win` = x on [oy, oy+H) x [ox, ox+W) (zeros outside the image); g is
 * written for the (H - 4r) x (W - 4r) region starting at (oy+2r, ox+2r).
 * z (optional) receives the drawn z on the (H-2r) x (W-2r) region.
 * ==================================================================== */
typedef struct {
  int32_t ny, nx, L;
  const double *y, *k;
  const uint8_t *m;
  double sigma, rho;
  uint64_t seed;
  uint32_t chain;
} grad_ctx;

static void grad_window(const grad_ctx *gc, const double *win, int oy, int ox, int H, int W,
                        int64_t t, double *g, double *zout) {
  int L = gc->L, r = L / 2;
  int H1 = H - 2 * r, W1 = W - 2 * r;   /* Kx region, origin (oy+r, ox+r) */
  double *kx = xmalloc((size_t)H1 * W1 * sizeof(double));
  valid_conv(win, H, W, gc->k, L, kx);
  const int split = gc->rho > 0.0;
  const double s2 = split ? gc->rho : gc->sigma * gc->sigma;
  const double sig2 = gc->sigma * gc->sigma;
  const double zsd = split ? sqrt(gc->rho * sig2 / (gc->rho + sig2)) : 0.0;
  for (int i = 0; i < H1; ++i)
    for (int j = 0; j < W1; ++j) {
      int gi = oy + r + i, gj = ox + r + j;
      size_t q = (size_t)i * W1 + j;
      double res = 0.0, z = 0.0;
      if (gi >= 0 && gi < gc->ny && gj >= 0 && gj < gc->nx) {
        int64_t p = (int64_t)gi * gc->nx + gj;
        double m = gc->m ? (double)gc->m[p] : 1.0;
        double v;
        if (split) {
          if (t >= 1) {
            double xi_unused, zeta;
            draw_pixel(gc->seed, p, t, gc->chain, &xi_unused, &zeta);
            z = (gc->rho * gc->y[p] + sig2 * (m * kx[q])) / (gc->rho + sig2) + zsd * zeta;
          } else {
            z = 0.0;  /* z^(0) = 0 (Sec. III-B) */
          }
          v = z;
        } else {
          v = gc->y[p];
        }
        res = m * (kx[q] - v);
      }
      if (zout) zout[q] = z;
      kx[q] = res;  /* reuse the buffer for the residual */
    }
  valid_xcorr(kx, H1, W1, gc->k, L, g);
  int n2 = (H1 - 2 * r) * (W1 - 2 * r);
  for (int i = 0; i < n2; ++i) g[i] /= s2;
  free(kx);
}

static grad_ctx make_grad_ctx(const oracle_config *c) {
  grad_ctx gc = {c->ny, c->nx, c->ksize, c->y, c->kernel, c->mask, c->sigma, c->rho,
                 c->seed, c->chain};
  return gc;
}

int oracle_data_grad(const oracle_config *c, const double *x, int64_t t, double *g) {
  int ny = c->ny, nx = c->nx, r = c->ksize / 2;
  grad_ctx gc = make_grad_ctx(c);
  if (c->block_y <= 0 || c->block_x <= 0 || (c->block_y >= ny && c->block_x >= nx)) {
    int H = ny + 4 * r, W = nx + 4 * r;
    double *win = xmalloc((size_t)H * W * sizeof(double));
    extract_window(x, 1, ny, nx, -2 * r, -2 * r, H, W, win);
    grad_window(&gc, win, -2 * r, -2 * r, H, W, t, g, NULL);
    free(win);
    return 0;
  }
  int h = c->halo;
  if (h < 2 * r) return -1;
  for (int by = 0; by < ny; by += c->block_y)
    for (int bx = 0; bx < nx; bx += c->block_x) {
      int cy = (by + c->block_y <= ny) ? c->block_y : ny - by;
      int cx = (bx + c->block_x <= nx) ? c->block_x : nx - bx;
      int H = cy + 2 * h, W = cx + 2 * h;
      double *win = xmalloc((size_t)H * W * sizeof(double));
      extract_window(x, 1, ny, nx, by - h, bx - h, H, W, win);
      int Hg = H - 4 * r, Wg = W - 4 * r, off = h - 2 * r;
      double *gw = xmalloc((size_t)Hg * Wg * sizeof(double));
      grad_window(&gc, win, by - h, bx - h, H, W, t, gw, NULL);
      for (int i = 0; i < cy; ++i)
        for (int j = 0; j < cx; ++j)
          g[(size_t)(by + i) * nx + bx + j] = gw[(size_t)(i + off) * Wg + j + off];
      free(gw);
      free(win);
    }
  return 0;
}

/* ======================================================================
 * Proximity operators of the z-steps (Eq. (sgs_pnp_ula_psgla:psgla)):
 *   prox_{kappa f}(v) = argmin_u kappa f(u) + |u - v|^2 / 2.
 * ==================================================================== */

/* f(u) = KL(y || u) = u - y log u (+ const), u >= 0 (Poisson data term,
 * Eq. (poisson:f2)): the stationarity condition u^2 - (v - kappa) u -
 * kappa y = 0 has one non-negative root. */
double oracle_prox_kl(double v, double y, double kappa) {
  double b = v - kappa;
  return 0.5 * (b + sqrt(b * b + 4.0 * kappa * y));
}

/* f(u) = (y - u)^2 / (2 sigma^2) (Gaussian data term as f2): the weighted
 * mean of v and y. */
double oracle_prox_gauss(double v, double y, double sigma, double kappa) {
  double s2 = sigma * sigma;
  return (s2 * v + kappa * y) / (s2 + kappa);
}

/* f(u) = ||u||_2 for one pixel's two differences (the l_{2,1} norm of the TV
 * prior, Sec. III-B2), scaled by tau: block soft thresholding. */
void oracle_prox_l21(double *vh, double *vv, double tau) {
  double nrm = sqrt(*vh * *vh + *vv * *vv);
  double f = nrm > tau ? 1.0 - tau / nrm : 0.0;
  *vh *= f;
  *vv *= f;
}

/* ======================================================================
 * 2-D discrete gradient D (Sec. III-B2): forward differences, zero in the
 * last column (horizontal) and last row (vertical); D^T its adjoint.
 * ==================================================================== */
void oracle_grad2d(const double *x, int32_t ny, int32_t nx, double *dh, double *dv) {
  for (int i = 0; i < ny; ++i)
    for (int j = 0; j < nx; ++j) {
      size_t p = (size_t)i * nx + j;
      dh[p] = j + 1 < nx ? x[p + 1] - x[p] : 0.0;
      dv[p] = i + 1 < ny ? x[p + nx] - x[p] : 0.0;
    }
}

void oracle_grad2d_adjoint(const double *dh, const double *dv, int32_t ny, int32_t nx,
                           double *out) {
  for (int i = 0; i < ny; ++i)
    for (int j = 0; j < nx; ++j) {
      size_t p = (size_t)i * nx + j;
      double v = 0.0;
      if (j >= 1) v += dh[p - 1];
      if (j + 1 < nx) v -= dh[p];
      if (i >= 1) v += dv[p - nx];
      if (i + 1 < ny) v -= dv[p];
      out[p] = v;
    }
}

/* ======================================================================
 * DDFB denoiser (Sec. II-B1 Example 3, Eqs. (ddfb_operator), (dfb_operator:T)):
 *   u_0 = W_K v,
 *   u_k = HT(u_{k-1} + gamma_k W_k P(v - W_k^* u_{k-1})),  k = 1 .. K-1,
 *   D(v) = P(v - gamma_K W_K^* u_{K-1}),
 * with W_k the 1 -> F zero-padded 3x3 cross-correlation, W_k^* its adjoint,
 * P the projection onto [0,1] and HT the clip to [-thresh, thresh].
 * On a window (origin (oy, ox), H x W) every map is zeroed outside the
 * image, the zero padding of each convolution of the whole-image operator;
 * each convolution shrinks the valid region by one pixel per side.
 * ==================================================================== */

/* out[c][i][j] = sum_{a,b} w[c][a][b] in[i+a][j+b]: in H x W -> F x (H-2) x (W-2) */
static void ddfb_fwd(const double *in, int H, int W, const double *w, int F, double *out) {
  int Ho = H - 2, Wo = W - 2;
  for (int c = 0; c < F; ++c)
    for (int i = 0; i < Ho; ++i)
      for (int j = 0; j < Wo; ++j) {
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) acc += w[c * 9 + a * 3 + b] * in[(size_t)(i + a) * W + j + b];
        out[((size_t)c * Ho + i) * Wo + j] = acc;
      }
}

/* adjoint: out[i][j] = sum_c sum_{a,b} w[c][a][b] u[c][i+2-a][j+2-b]:
 * F x H x W -> (H-2) x (W-2) */
static void ddfb_adj(const double *u, int H, int W, const double *w, int F, double *out) {
  int Ho = H - 2, Wo = W - 2;
  for (int i = 0; i < Ho; ++i)
    for (int j = 0; j < Wo; ++j) {
      double acc = 0.0;
      for (int c = 0; c < F; ++c)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            acc += w[c * 9 + a * 3 + b] * u[((size_t)c * H + i + 2 - a) * W + j + 2 - b];
      out[(size_t)i * Wo + j] = acc;
    }
}

static double clip01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* sub-window of C planes: rows/cols shrink by `d` on each side */
static double *crop(const double *in, int C, int H, int W, int d) {
  int Ho = H - 2 * d, Wo = W - 2 * d;
  double *out = xmalloc((size_t)C * Ho * Wo * sizeof(double));
  for (int c = 0; c < C; ++c)
    for (int i = 0; i < Ho; ++i)
      memcpy(out + ((size_t)c * Ho + i) * Wo, in + ((size_t)c * H + i + d) * W + d,
             (size_t)Wo * sizeof(double));
  return out;
}

/* D(v) on the window's region shrunk by 2K per side */
static double *ddfb_window(const oracle_config *cf, const double *win, int ny, int nx, int oy,
                           int ox, int H, int W) {
  const int K = cf->ddfb_layers, F = cf->ddfb_features;
  const double *WK = cf->ddfb_weights + (size_t)(K - 1) * F * 9;
  const double th = cf->ddfb_thresh;
  /* u_0 = W_K v on (H-2) x (W-2), origin (oy+1, ox+1) */
  int Hu = H - 2, Wu = W - 2, uy = oy + 1, ux = ox + 1;
  double *u = xmalloc((size_t)F * Hu * Wu * sizeof(double));
  ddfb_fwd(win, H, W, WK, F, u);
  zero_outside(u, F, ny, nx, uy, ux, Hu, Wu);
  for (int k = 1; k < K; ++k) {
    const double *Wk = cf->ddfb_weights + (size_t)(k - 1) * F * 9;
    const double gk = cf->ddfb_gamma[k - 1];
    /* b = P(v - W_k^* u) on (Hu-2) x (Wu-2), origin (uy+1, ux+1) */
    int Hb = Hu - 2, Wb = Wu - 2, by = uy + 1, bx = ux + 1;
    double *b = xmalloc((size_t)Hb * Wb * sizeof(double));
    ddfb_adj(u, Hu, Wu, Wk, F, b);
    for (int i = 0; i < Hb; ++i)
      for (int j = 0; j < Wb; ++j) {
        double v = win[(size_t)(by - oy + i) * W + (bx - ox + j)];
        b[(size_t)i * Wb + j] = clip01(v - b[(size_t)i * Wb + j]);
      }
    zero_outside(b, 1, ny, nx, by, bx, Hb, Wb);
    /* u <- HT(u + gamma_k W_k b) on (Hb-2) x (Wb-2), origin (by+1, bx+1) */
    int Hn = Hb - 2, Wn = Wb - 2, ny0 = by + 1, nx0 = bx + 1;
    double *wb = xmalloc((size_t)F * Hn * Wn * sizeof(double));
    ddfb_fwd(b, Hb, Wb, Wk, F, wb);
    double *un = crop(u, F, Hu, Wu, 2);
    for (size_t q = 0; q < (size_t)F * Hn * Wn; ++q) {
      double v = un[q] + gk * wb[q];
      un[q] = v < -th ? -th : (v > th ? th : v);
    }
    zero_outside(un, F, ny, nx, ny0, nx0, Hn, Wn);
    free(u);
    free(b);
    free(wb);
    u = un;
    Hu = Hn; Wu = Wn; uy = ny0; ux = nx0;
  }
  /* D(v) = P(v - gamma_K W_K^* u_{K-1}) on (Hu-2) x (Wu-2) */
  int Ho = Hu - 2, Wo = Wu - 2, oy2 = uy + 1, ox2 = ux + 1;
  double *out = xmalloc((size_t)Ho * Wo * sizeof(double));
  ddfb_adj(u, Hu, Wu, WK, F, out);
  const double gK = cf->ddfb_gamma[K - 1];
  for (int i = 0; i < Ho; ++i)
    for (int j = 0; j < Wo; ++j) {
      double v = win[(size_t)(oy2 - oy + i) * W + (ox2 - ox + j)];
      out[(size_t)i * Wo + j] = clip01(v - gK * out[(size_t)i * Wo + j]);
    }
  free(u);
  return out;
}

int oracle_ddfb(const oracle_config *cf, const double *v, int32_t ny, int32_t nx, double *out) {
  if (cf->ddfb_layers < 1 || cf->ddfb_features < 1 || !cf->ddfb_weights || !cf->ddfb_gamma)
    return -1;
  int R = 2 * cf->ddfb_layers;
  int H = ny + 2 * R, W = nx + 2 * R;
  double *win = xmalloc((size_t)H * W * sizeof(double));
  extract_window(v, 1, ny, nx, -R, -R, H, W, win);
  double *res = ddfb_window(cf, win, ny, nx, -R, -R, H, W);
  memcpy(out, res, (size_t)ny * nx * sizeof(double));
  free(res);
  free(win);
  return 0;
}

/* Data-term gradient with the splitting variable z1 held as chain state
 * (PSGLA z-steps): with A = eta diag(m) K,
 *   g = A^T (A x - z1) / rho = eta K^T (m (eta K x - z1)) / rho
 * on the window's region shrunk by 2r per side.  zwin holds z1 on the region
 * shrunk by r (origin (oy + r, ox + r)). */
static void grad_window_state(const oracle_config *c, const double *win, const double *zwin,
                              int oy, int ox, int H, int W, double *g) {
  int L = c->ksize, r = L / 2;
  int H1 = H - 2 * r, W1 = W - 2 * r;
  const double eta = c->eta > 0 ? c->eta : 1.0;
  double *kx = xmalloc((size_t)H1 * W1 * sizeof(double));
  valid_conv(win, H, W, c->kernel, L, kx);
  for (int i = 0; i < H1; ++i)
    for (int j = 0; j < W1; ++j) {
      int gi = oy + r + i, gj = ox + r + j;
      size_t q = (size_t)i * W1 + j;
      double res = 0.0;
      if (gi >= 0 && gi < c->ny && gj >= 0 && gj < c->nx) {
        int64_t p = (int64_t)gi * c->nx + gj;
        double m = c->mask ? (double)c->mask[p] : 1.0;
        res = m * (eta * (m * kx[q]) - zwin[q]);
      }
      kx[q] = res;
    }
  valid_xcorr(kx, H1, W1, c->kernel, L, g);
  int n2 = (H1 - 2 * r) * (W1 - 2 * r);
  for (int i = 0; i < n2; ++i) g[i] = eta * g[i] / c->rho;
  free(kx);
}

/* Prior radius of one iteration: the receptive field of the prior term. */
static int prior_radius(const oracle_config *c) {
  if (c->prior == 1) return 1;
  if (c->prior == 2) return 2 * c->ddfb_layers;
  return c->net.n_layers;
}

/* ======================================================================
 * The chain
 * ==================================================================== */
struct oracle_chain {
  oracle_config cfg;       /* pointers below are owned copies */
  double *y, *kernel, *w, *b, *act_scales, *dw, *dg;
  int32_t *channels, *fmt;
  uint8_t *mask;
  double *x, *z;
  double *z1, *z2;         /* PSGLA / TV state z^(t) (z^(0) = 0) */
  int64_t t;
  int64_t n;               /* Welford count */
  int record_z;
  double *mean, *m2;
};

static void *dup(const void *p, size_t n) {
  if (!p) return NULL;
  void *q = xmalloc(n);
  memcpy(q, p, n);
  return q;
}

oracle_chain *oracle_create(const oracle_config *cfg, char *err, int errlen) {
#define FAIL(msg)                                   \
  do {                                              \
    if (err && errlen > 0) snprintf(err, errlen, "%s", msg); \
    return NULL;                                    \
  } while (0)
  if (!cfg || cfg->ny <= 0 || cfg->nx <= 0) FAIL("image size must be positive");
  if (!cfg->y) FAIL("y is required");
  if (cfg->ksize < 1 || cfg->ksize % 2 == 0 || !cfg->kernel) FAIL("blur size must be odd");
  if (!(cfg->sigma > 0) || !(cfg->eps > 0) || !(cfg->delta > 0) || !(cfg->rho >= 0) ||
      !(cfg->alpha >= 0) || !(cfg->inv_lambda >= 0))
    FAIL("sigma, eps, delta must be > 0; rho, alpha, inv_lambda >= 0");
  const oracle_net *n = &cfg->net;
  if (cfg->prior < 0 || cfg->prior > 2) FAIL("unknown prior");
  if (cfg->prior == 0 &&
      (n->n_layers < 1 || !n->channels || n->channels[0] != 1 ||
       n->channels[n->n_layers] != 1 || !n->weights || !n->biases))
    FAIL("denoiser must map 1 channel to 1 channel");
  if (cfg->prior == 2 && (cfg->ddfb_layers < 1 || cfg->ddfb_features < 1 || !cfg->ddfb_weights ||
                          !cfg->ddfb_gamma || !(cfg->ddfb_thresh >= 0)))
    FAIL("DDFB needs layers, features, weights, step sizes and a threshold");
  if (cfg->likelihood < 0 || cfg->likelihood > 1 || cfg->z_step < 0 || cfg->z_step > 1)
    FAIL("unknown likelihood or z-step");
  if (cfg->likelihood == 1 && cfg->z_step != 1) FAIL("the Poisson likelihood needs the PSGLA z-step");
  if ((cfg->z_step == 1 || cfg->prior == 1) && !(cfg->rho > 0 && cfg->kappa > 0))
    FAIL("PSGLA needs rho > 0 and kappa > 0");
  if (cfg->prior == 1 && (cfg->z_step != 0 || cfg->likelihood != 0 || cfg->rho2 > 0))
    FAIL("the TV prior runs with the unsplit Gaussian likelihood");
  if (cfg->rho2 > 0 && !(cfg->kappa2 > 0)) FAIL("the second z block needs kappa2 > 0");
  if (!(cfg->rho2 >= 0) || !(cfg->beta >= 0) || !(cfg->eta >= 0)) FAIL("negative parameter");
  int r = cfg->ksize / 2;
  int blocked = cfg->block_y > 0 && cfg->block_x > 0 &&
                !(cfg->block_y >= cfg->ny && cfg->block_x >= cfg->nx);
  int pr = prior_radius(cfg);
  if (blocked && cfg->halo < (2 * r > pr ? 2 * r : pr))
    FAIL("halo must be >= max(2r, K)");
  oracle_chain *c = calloc(1, sizeof *c);
  if (!c) FAIL("out of memory");
  size_t N = (size_t)cfg->ny * cfg->nx;
  c->cfg = *cfg;
  c->y = dup(cfg->y, N * sizeof(double));
  c->kernel = dup(cfg->kernel, (size_t)cfg->ksize * cfg->ksize * sizeof(double));
  c->mask = dup(cfg->mask, N);
  if (cfg->prior == 0) {
    c->channels = dup(n->channels, (n->n_layers + 1) * sizeof(int32_t));
    c->w = dup(n->weights, weight_offset(n, n->n_layers) * sizeof(double));
    c->b = dup(n->biases, bias_offset(n, n->n_layers) * sizeof(double));
    c->fmt = dup(n->layer_fmt, n->n_layers * sizeof(int32_t));
    c->act_scales = dup(n->act_scales, n->n_layers * sizeof(double));
  }
  if (cfg->prior == 2) {
    c->dw = dup(cfg->ddfb_weights, (size_t)cfg->ddfb_layers * cfg->ddfb_features * 9 * sizeof(double));
    c->dg = dup(cfg->ddfb_gamma, (size_t)cfg->ddfb_layers * sizeof(double));
  }
  c->cfg.y = c->y;
  c->cfg.kernel = c->kernel;
  c->cfg.mask = c->mask;
  c->cfg.net.channels = c->channels;
  c->cfg.net.weights = c->w;
  c->cfg.net.biases = c->b;
  c->cfg.net.layer_fmt = c->fmt;
  c->cfg.net.act_scales = c->act_scales;
  c->cfg.ddfb_weights = c->dw;
  c->cfg.ddfb_gamma = c->dg;
  c->cfg.x0 = NULL;
  c->x = xmalloc(N * sizeof(double));
  c->z = calloc(N, sizeof(double));
  c->z1 = calloc(N, sizeof(double));
  c->z2 = calloc(N, sizeof(double));
  c->mean = calloc(N, sizeof(double));
  c->m2 = calloc(N, sizeof(double));
  if (cfg->x0) memcpy(c->x, cfg->x0, N * sizeof(double));
  else memset(c->x, 0, N * sizeof(double));
  c->t = 0;
  c->n = 0;
  return c;
#undef FAIL
}

/* Data-term gradient with z1 held as state, on the whole image (blocked
 * like oracle_data_grad when the configuration has several blocks), plus
 * the second block's (x - z2) / rho2. */
static int data_grad_state(const oracle_config *c, const double *x, const double *z1,
                           const double *z2, double *g) {
  int ny = c->ny, nx = c->nx, r = c->ksize / 2;
  int blocked = c->block_y > 0 && c->block_x > 0 && !(c->block_y >= ny && c->block_x >= nx);
  int by0 = blocked ? c->block_y : ny, bx0 = blocked ? c->block_x : nx;
  int h = blocked ? c->halo : 2 * r;
  if (h < 2 * r) return -1;
  for (int by = 0; by < ny; by += by0)
    for (int bx = 0; bx < nx; bx += bx0) {
      int cy = (by + by0 <= ny) ? by0 : ny - by;
      int cx = (bx + bx0 <= nx) ? bx0 : nx - bx;
      int H = cy + 2 * h, W = cx + 2 * h;
      double *win = xmalloc((size_t)H * W * sizeof(double));
      double *zw = xmalloc((size_t)(H - 2 * r) * (W - 2 * r) * sizeof(double));
      extract_window(x, 1, ny, nx, by - h, bx - h, H, W, win);
      extract_window(z1, 1, ny, nx, by - h + r, bx - h + r, H - 2 * r, W - 2 * r, zw);
      int Hg = H - 4 * r, Wg = W - 4 * r, off = h - 2 * r;
      double *gw = xmalloc((size_t)Hg * Wg * sizeof(double));
      grad_window_state(c, win, zw, by - h, bx - h, H, W, gw);
      for (int i = 0; i < cy; ++i)
        for (int j = 0; j < cx; ++j)
          g[(size_t)(by + i) * nx + bx + j] = gw[(size_t)(i + off) * Wg + j + off];
      free(gw);
      free(zw);
      free(win);
    }
  if (c->rho2 > 0)
    for (size_t p = 0; p < (size_t)ny * nx; ++p) g[p] += (x[p] - z2[p]) / c->rho2;
  return 0;
}

/* D(x) of the DDFB prior on the whole image, blocked like oracle_denoiser */
static int ddfb_blocked(const oracle_config *c, const double *x, double *D) {
  int ny = c->ny, nx = c->nx, R = 2 * c->ddfb_layers;
  int blocked = c->block_y > 0 && c->block_x > 0 && !(c->block_y >= ny && c->block_x >= nx);
  if (!blocked) return oracle_ddfb(c, x, ny, nx, D);
  int h = c->halo;
  if (h < R) return -1;
  for (int by = 0; by < ny; by += c->block_y)
    for (int bx = 0; bx < nx; bx += c->block_x) {
      int cy = (by + c->block_y <= ny) ? c->block_y : ny - by;
      int cx = (bx + c->block_x <= nx) ? c->block_x : nx - bx;
      int H = cy + 2 * h, W = cx + 2 * h;
      double *win = xmalloc((size_t)H * W * sizeof(double));
      extract_window(x, 1, ny, nx, by - h, bx - h, H, W, win);
      double *res = ddfb_window(c, win, ny, nx, by - h, bx - h, H, W);
      int Wr = W - 2 * R, off = h - R;
      for (int i = 0; i < cy; ++i)
        for (int j = 0; j < cx; ++j)
          D[(size_t)(by + i) * nx + bx + j] = res[(size_t)(i + off) * Wr + j + off];
      free(res);
      free(win);
    }
  return 0;
}

/* (1/rho) D^T (D x - z) of the TV prior's coupling term at pixel (i, j),
 * from x and the two difference planes of z (Sec. III-B2) */
static double tv_coupling(const oracle_config *c, const double *x, const double *zh,
                          const double *zv, int i, int j) {
  int ny = c->ny, nx = c->nx;
  size_t p = (size_t)i * nx + j;
  /* residual r = D x - z at pixel q, both components */
#define RH(q, jj) ((jj) + 1 < nx ? (x[(q) + 1] - x[q]) - zh[q] : -zh[q])
#define RV(q, ii) ((ii) + 1 < ny ? (x[(q) + nx] - x[q]) - zv[q] : -zv[q])
  double v = 0.0;
  if (j >= 1) v += RH(p - 1, j - 1);
  if (j + 1 < nx) v -= RH(p, j);
  if (i >= 1) v += RV(p - nx, i - 1);
  if (i + 1 < ny) v -= RV(p, i);
#undef RH
#undef RV
  return v / c->rho;
}

/* z^(t) -> z^(t+1) from x^(t+1) (Eq. (sgs_pnp_ula_psgla:psgla) and the
 * z-update of Algorithm 1; Sec. III-B2 for TV), noise from counter t+1 */
static void z_step(oracle_chain *c) {
  const oracle_config *cf = &c->cfg;
  int ny = cf->ny, nx = cf->nx;
  size_t N = (size_t)ny * nx;
  const int64_t tz = c->t;                 /* c->t already holds t+1 */
  if (cf->prior == 1) {                    /* TV: z ~ D x, f2 = beta ||.||_{2,1} */
    double *dh = xmalloc(N * sizeof(double)), *dv = xmalloc(N * sizeof(double));
    oracle_grad2d(c->x, ny, nx, dh, dv);
    const double a = cf->kappa / cf->rho, sq = sqrt(2.0 * cf->kappa), tau = cf->kappa * cf->beta;
    for (int i = 0; i < ny; ++i)
      for (int j = 0; j < nx; ++j) {
        int64_t p = (int64_t)i * nx + j;
        double xi_u, zh, zv;
        draw_pixel3(cf->seed, p, tz, cf->chain, &xi_u, &zh, &zv);
        double vh = c->z1[p] - a * (c->z1[p] - dh[p]) + sq * zh;
        double vv = c->z2[p] - a * (c->z2[p] - dv[p]) + sq * zv;
        oracle_prox_l21(&vh, &vv, tau);
        c->z1[p] = vh;
        c->z2[p] = vv;
      }
    free(dh);
    free(dv);
    return;
  }
  /* z1 ~ eta diag(m) K x with the likelihood as f; z2 ~ x with f = indicator of R+ */
  const double eta = cf->eta > 0 ? cf->eta : 1.0;
  double *kx = xmalloc(N * sizeof(double));
  oracle_blur(c->x, ny, nx, cf->kernel, cf->ksize, kx);
  const double a1 = cf->kappa / cf->rho, s1 = sqrt(2.0 * cf->kappa);
  const double a2 = cf->rho2 > 0 ? cf->kappa2 / cf->rho2 : 0.0, s2 = sqrt(2.0 * cf->kappa2);
  for (size_t p = 0; p < N; ++p) {
    double xi_u, ze1, ze2;
    draw_pixel3(cf->seed, (int64_t)p, tz, cf->chain, &xi_u, &ze1, &ze2);
    double m = cf->mask ? (double)cf->mask[p] : 1.0;
    double v = c->z1[p] - a1 * (c->z1[p] - eta * m * kx[p]) + s1 * ze1;
    if (m != 0.0)   /* unobserved entries carry no data term: prox = identity */
      v = cf->likelihood == 1 ? oracle_prox_kl(v, c->y[p], cf->kappa)
                              : oracle_prox_gauss(v, c->y[p], cf->sigma, cf->kappa);
    c->z1[p] = v;
    if (cf->rho2 > 0) {
      double w = c->z2[p] - a2 * (c->z2[p] - c->x[p]) + s2 * ze2;
      c->z2[p] = w > 0.0 ? w : 0.0;
    }
  }
  free(kx);
}

/* x^(t) -> x^(t+1) (Eq. (sgs_pnp_ula_psgla:pnp_ula), Algorithm 1; PSGLA
 * x-transition with the indicator of R+ for the TV prior, Sec. III-B2),
 * then z^(t+1) for the PSGLA and TV chains */
static int one_step(oracle_chain *c) {
  const oracle_config *cfg = &c->cfg;
  int ny = cfg->ny, nx = cfg->nx;
  size_t N = (size_t)ny * nx;
  double *g = xmalloc(N * sizeof(double));
  double *G = xmalloc(N * sizeof(double));
  /* data term (blocked when the configuration has several blocks) */
  if (cfg->prior == 1) {
    oracle_config cg = *cfg;
    cg.rho = 0.0;                          /* TV: the likelihood is not split */
    oracle_data_grad(&cg, c->x, c->t, g);
  } else if (cfg->z_step == 1) {
    data_grad_state(cfg, c->x, c->z1, c->z2, g);
  } else {
    oracle_data_grad(cfg, c->x, c->t, g);
  }
  /* record z for inspection (monolithic draw, identical values) */
  if (cfg->z_step == 0 && cfg->prior != 1 && cfg->rho > 0 && c->record_z) {
    int r = cfg->ksize / 2;
    int H = ny + 4 * r, W = nx + 4 * r;
    double *win = xmalloc((size_t)H * W * sizeof(double));
    double *gtmp = xmalloc(N * sizeof(double));
    double *zw = xmalloc((size_t)(ny + 2 * r) * (nx + 2 * r) * sizeof(double));
    grad_ctx gc = make_grad_ctx(cfg);
    extract_window(c->x, 1, ny, nx, -2 * r, -2 * r, H, W, win);
    grad_window(&gc, win, -2 * r, -2 * r, H, W, c->t, gtmp, zw);
    for (int i = 0; i < ny; ++i)
      for (int j = 0; j < nx; ++j)
        c->z[(size_t)i * nx + j] = zw[(size_t)(i + r) * (nx + 2 * r) + j + r];
    free(zw);
    free(gtmp);
    free(win);
  }
  /* prior term: G = Id - D_eps (residual CNN or DDFB) */
  if (cfg->prior == 0) {
    oracle_denoiser(&cfg->net, c->x, ny, nx, cfg->block_y, cfg->block_x, cfg->halo, G);
  } else if (cfg->prior == 2) {
    ddfb_blocked(cfg, c->x, G);
    for (size_t p = 0; p < N; ++p) G[p] = c->x[p] - G[p];
  }
  const double d = cfg->delta;
  const double cprior = cfg->alpha * d / cfg->eps;
  const double cproj = d * cfg->inv_lambda;
  const double sq = sqrt(2.0 * d);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int i = 0; i < ny; ++i)
    for (int j = 0; j < nx; ++j) {
      int64_t p = (int64_t)i * nx + j;
      double xi, zeta_unused;
      draw_pixel(cfg->seed, p, c->t, cfg->chain, &xi, &zeta_unused);
      double x = c->x[p];
      double xn;
      if (cfg->prior == 1) {
        double v = x - d * g[p] - d * tv_coupling(cfg, c->x, c->z1, c->z2, i, j) + sq * xi;
        xn = v > 0.0 ? v : 0.0;            /* prox of the indicator of R+ */
      } else {
        double proj = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
        xn = x - d * g[p] - cprior * G[p] + cproj * (proj - x) + sq * xi;
      }
      if (!isfinite(xn)) bad = 1;
      g[p] = xn;  /* x^(t+1) staged in g so every pixel reads x^(t) */
    }
  memcpy(c->x, g, N * sizeof(double));
  c->t += 1;
  if (cfg->z_step == 1 || cfg->prior == 1) z_step(c);
  /* online mean / variance of the samples after burn-in (Welford) */
  if (c->t > cfg->burn_in) {
    c->n += 1;
    const double inv = 1.0 / (double)c->n;
    for (size_t p = 0; p < N; ++p) {
      double dlt = c->x[p] - c->mean[p];
      c->mean[p] += dlt * inv;
      c->m2[p] += dlt * (c->x[p] - c->mean[p]);
    }
  }
  free(g);
  free(G);
  return bad ? -5 : 0;
}

/* x^(t+1) on the region [y0, y0+h) x [x0, x0+w) of the image described by
 * cfg, from the full x^(t) (and, for the PSGLA and TV chains, the full
 * z^(t) planes z1, z2): every operator is evaluated on the region's extended
 * window of half-width max(2r, prior radius) only (the same window
 * computation as a block), so sampled outputs of very large images can be
 * checked one region at a time. */
int oracle_step_region_z(const oracle_config *c, const double *x, const double *z1,
                         const double *z2, int64_t t, int32_t y0, int32_t x0, int32_t h,
                         int32_t w, double *xnew) {
  int ny = c->ny, nx = c->nx, r = c->ksize / 2, pr = prior_radius(c);
  if (y0 < 0 || x0 < 0 || h < 1 || w < 1 || y0 + h > ny || x0 + w > nx) return -1;
  if ((c->z_step == 1 || c->prior == 1) && (!z1 || (!z2 && (c->rho2 > 0 || c->prior == 1))))
    return -2;
  int hh = 2 * r > pr ? 2 * r : pr;
  int H = h + 2 * hh, W = w + 2 * hh;
  double *win = xmalloc((size_t)H * W * sizeof(double));
  extract_window(x, 1, ny, nx, y0 - hh, x0 - hh, H, W, win);
  int Hg = H - 4 * r, Wg = W - 4 * r, og = hh - 2 * r;
  double *g = xmalloc((size_t)Hg * Wg * sizeof(double));
  if (c->z_step == 1 && c->prior != 1) {
    double *zw = xmalloc((size_t)(H - 2 * r) * (W - 2 * r) * sizeof(double));
    extract_window(z1, 1, ny, nx, y0 - hh + r, x0 - hh + r, H - 2 * r, W - 2 * r, zw);
    grad_window_state(c, win, zw, y0 - hh, x0 - hh, H, W, g);
    free(zw);
  } else {
    grad_ctx gc = make_grad_ctx(c);
    if (c->prior == 1) gc.rho = 0.0;
    grad_window(&gc, win, y0 - hh, x0 - hh, H, W, t, g, NULL);
  }
  double *res = NULL;
  int Wd = 0, od = 0;
  if (c->prior == 0) {
    prepared_net pn;
    prepare_net(&c->net, &pn);
    res = denoise_window(&c->net, &pn, win, ny, nx, y0 - hh, x0 - hh, H, W, 0, NULL, NULL);
    free_net(&pn);
    Wd = W - 2 * pr;
    od = hh - pr;
  } else if (c->prior == 2) {
    res = ddfb_window(c, win, ny, nx, y0 - hh, x0 - hh, H, W);
    Wd = W - 2 * pr;
    od = hh - pr;
  }
  const double d = c->delta, cprior = c->alpha * d / c->eps, cproj = d * c->inv_lambda;
  const double sq = sqrt(2.0 * d);
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < w; ++j) {
      int64_t p = (int64_t)(y0 + i) * nx + (x0 + j);
      double xi, zeta_unused;
      draw_pixel(c->seed, p, t, c->chain, &xi, &zeta_unused);
      double xv = x[p];
      double gv = g[(size_t)(i + og) * Wg + j + og];
      if (c->z_step == 1 && c->prior != 1 && c->rho2 > 0) gv += (xv - z2[p]) / c->rho2;
      if (c->prior == 1) {
        double v = xv - d * gv - d * tv_coupling(c, x, z1, z2, y0 + i, x0 + j) + sq * xi;
        xnew[(size_t)i * w + j] = v > 0.0 ? v : 0.0;
        continue;
      }
      double proj = xv < 0.0 ? 0.0 : (xv > 1.0 ? 1.0 : xv);
      double Gv = res[(size_t)(i + od) * Wd + j + od];
      if (c->prior == 2) Gv = xv - Gv;
      xnew[(size_t)i * w + j] = xv - d * gv - cprior * Gv + cproj * (proj - xv) + sq * xi;
    }
  free(res);
  free(g);
  free(win);
  return 0;
}

int oracle_step_region(const oracle_config *c, const double *x, int64_t t, int32_t y0,
                       int32_t x0, int32_t h, int32_t w, double *xnew) {
  return oracle_step_region_z(c, x, NULL, NULL, t, y0, x0, h, w, xnew);
}

int oracle_step(oracle_chain *c, int32_t n_iters) {
  for (int32_t i = 0; i < n_iters; ++i) {
    int rc = one_step(c);
    if (rc) return rc;
  }
  return 0;
}

void oracle_get_state(const oracle_chain *c, double *x, int64_t *t) {
  if (x) memcpy(x, c->x, (size_t)c->cfg.ny * c->cfg.nx * sizeof(double));
  if (t) *t = c->t;
}

void oracle_set_state(oracle_chain *c, const double *x, int64_t t) {
  memcpy(c->x, x, (size_t)c->cfg.ny * c->cfg.nx * sizeof(double));
  c->t = t;
}

void oracle_stats(const oracle_chain *c, double *mean, double *m2, int64_t *n) {
  size_t N = (size_t)c->cfg.ny * c->cfg.nx;
  if (mean) memcpy(mean, c->mean, N * sizeof(double));
  if (m2) memcpy(m2, c->m2, N * sizeof(double));
  if (n) *n = c->n;
}

void oracle_last_z(const oracle_chain *c, double *z) {
  memcpy(z, c->z, (size_t)c->cfg.ny * c->cfg.nx * sizeof(double));
}

void oracle_record_z(oracle_chain *c, int32_t on) { c->record_z = on; }

void oracle_get_z(const oracle_chain *c, double *z1, double *z2) {
  size_t N = (size_t)c->cfg.ny * c->cfg.nx;
  if (z1) memcpy(z1, c->z1, N * sizeof(double));
  if (z2) memcpy(z2, c->z2, N * sizeof(double));
}

void oracle_set_z(oracle_chain *c, const double *z1, const double *z2) {
  size_t N = (size_t)c->cfg.ny * c->cfg.nx;
  if (z1) memcpy(c->z1, z1, N * sizeof(double));
  if (z2) memcpy(c->z2, z2, N * sizeof(double));
}

void oracle_destroy(oracle_chain *c) {
  if (!c) return;
  free(c->y); free(c->kernel); free(c->mask); free(c->channels); free(c->w); free(c->b);
  free(c->fmt); free(c->act_scales); free(c->dw); free(c->dg); free(c->x); free(c->z);
  free(c->z1); free(c->z2); free(c->mean); free(c->m2);
  free(c);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
