/*
 * nellox_oracle.c -- plain FP64 CPU oracle for parallel local autoregressive
 * lossless compression (Zhang, Townsend, Kang, Barber, "Parallel Neural Local
 * Lossless Compression", arXiv 2201.05213).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library shares no
 * code with it: this file includes nothing from the GPU sources, parses the
 * weight blob itself and implements its own coder.
 *
 * What it computes, in plain slow loops:
 *   - the local autoregressive model of Eq. (3): pixel (i,j) depends on rows
 *     i-h..i-1, columns j-h..j+h, and on row i, columns j-h..j-1, with zero
 *     padding outside the image (Sec. 2.1, Fig. 2b);
 *   - its realisation as a masked first convolution followed by 1x1 layers
 *     (Sec. 2.1): here a causal (2h+1)x(2h+1) kernel, then pre-activation
 *     residual blocks of two 1x1 layers with ELU, then a 1x1 head;
 *   - a 10-component discretised logistic mixture per pixel, channels coded
 *     R, G, B with each channel's mixture weights conditioned on the earlier
 *     channels (exact joint factorisation), means of G and B shifted linearly
 *     by the earlier channels;
 *   - 16-bit quantised CDFs: cdf_k = k + floor(clamp(F(B_k),0,1) * 65280);
 *   - a byte-renormalising rANS coder (stream coding, Sec. 2, Eq. (2) text),
 *     32-bit state, L = 2^23, precision 2^16, start state 1, states below
 *     a symbol's frequency coded through its bit-reversal-spread slots, the
 *     final state flushed as its significant bytes;
 *   - raster order (the sequential decoder of Sec. 2) and the topological
 *     (wavefront) order of Sec. 3 / Fig. 3: pixel (i,j) at step j + (h+1) i;
 *   - the patch scheme: an image is cut into patch_h x patch_w tiles anchored
 *     at (0,0), each coded as an independent image with its own stream;
 *   - the sheared model of Sec. 3.1 (ShearLoC, Algorithm 2): image and first
 *     kernel sheared with offset o = h + 1 (Fig. 4b, Fig. 5b/5d), so that one
 *     wavefront step is one column; decoding column by column, then unshear;
 *   - ancestral sampling from the same model in the same orders (the parallel
 *     generation Sec. 5 leaves to future work): each symbol is the inverse of
 *     its quantised CDF at a 16-bit uniform slot drawn from the Philox4x64-10
 *     counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
 * Every floating point quantity is double precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OX_NMIX 10
#define OX_NOUT 100
#define OX_TOTAL 65536u
#define OX_SPREAD 65280.0 /* 2^16 - 256: one count reserved per symbol */
#define OX_RANS_L (1u << 23)

/* error codes */
#define OX_OK 0
#define OX_E_ARG -1
#define OX_E_BLOB -2
#define OX_E_CAP -3
#define OX_E_CORRUPT -4
#define OX_E_NAN -5     /* an undecoded (poisoned) pixel reached the model */
#define OX_E_CDF -6     /* a CDF row broke its invariants */

typedef struct {
  int h, C, nb, K;
  double *params; /* owned, blob order */
  const double *conv_w, *conv_b;
  const double *w1[16], *b1[16], *w2[16], *b2[16];
  const double *head_w, *head_b;
} ox_model;

/* ---------------------------------------------------------------- model */

long ox_param_count(int h, int C, int nb) {
  long K = 2 * h + 1;
  return C * 3 * K * K + C + (long)nb * (2L * C * C + 2L * C) + (long)OX_NOUT * C + OX_NOUT;
}

void ox_model_free(ox_model *m) {
  if (!m) return;
  free(m->params);
  free(m);
}

ox_model *ox_model_new(int h, int C, int nb, const double *params) {
  if (h < 1 || h > 8 || C < 1 || C > 4096 || nb < 0 || nb > 16) return NULL;
  ox_model *m = (ox_model *)calloc(1, sizeof(ox_model));
  long n = ox_param_count(h, C, nb);
  m->params = (double *)malloc(sizeof(double) * n);
  memcpy(m->params, params, sizeof(double) * n);
  m->h = h; m->C = C; m->nb = nb; m->K = 2 * h + 1;
  const double *p = m->params;
  m->conv_w = p; p += (long)C * 3 * m->K * m->K;
  m->conv_b = p; p += C;
  for (int b = 0; b < nb; ++b) {
    m->w1[b] = p; p += (long)C * C;
    m->b1[b] = p; p += C;
    m->w2[b] = p; p += (long)C * C;
    m->b2[b] = p; p += C;
  }
  m->head_w = p; p += (long)OX_NOUT * C;
  m->head_b = p;
  return m;
}

static uint64_t ox_fnv1a64(const uint8_t *d, size_t n) {
  uint64_t x = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) { x ^= d[i]; x *= 0x100000001b3ull; }
  return x;
}

static uint32_t rd32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

/* Parse a weight blob. dims_out = {h, C, n_blocks}. Returns a new model or NULL. */
ox_model *ox_model_from_blob(const uint8_t *b, size_t n, int dims_out[3], uint64_t *hash_out) {
  if (n < 36 || memcmp(b, "NLXW", 4) != 0) return NULL;
  uint32_t ver = rd32(b + 4), h = rd32(b + 8), C = rd32(b + 12), nb = rd32(b + 16);
  uint32_t nmix = rd32(b + 20), flags = rd32(b + 24);
  if (ver != 1 || nmix != OX_NMIX || flags != 1 || h < 1 || h > 8 || C < 1 || C > 4096 || nb > 16)
    return NULL;
  long np = ox_param_count((int)h, (int)C, (int)nb);
  if (n != 28 + (size_t)np * 4 + 8) return NULL;
  uint64_t hh = 0;
  for (int k = 0; k < 8; ++k) hh |= (uint64_t)b[n - 8 + k] << (8 * k);
  if (hh != ox_fnv1a64(b, n - 8)) return NULL;
  double *tmp = (double *)malloc(sizeof(double) * np);
  for (long k = 0; k < np; ++k) {
    uint32_t u = rd32(b + 28 + 4 * k);
    float f;
    memcpy(&f, &u, 4);
    tmp[k] = (double)f;
  }
  ox_model *m = ox_model_new((int)h, (int)C, (int)nb, tmp);
  free(tmp);
  if (m && dims_out) { dims_out[0] = (int)h; dims_out[1] = (int)C; dims_out[2] = (int)nb; }
  if (hash_out) *hash_out = hh;
  return m;
}

/* Causal taps of the first kernel (Eq. 3, Fig. 2b, Fig. 5a/5c): kernel row dy
 * covers image row i-h+dy, column dx covers j-h+dx. Rows above the pixel are
 * fully visible; in the pixel's own row only the h columns to its left. */
int ox_tap_live(int h, int dy, int dx) { return dy < h || (dy == h && dx < h); }

static double ox_elu(double x) { return x > 0.0 ? x : expm1(x); }

/* Everything after the first layer (Sec. 2.1: 1x1 layers only): residual
 * blocks on the first layer's output a[C], then the head into theta[100]. */
static void ox_body(const ox_model *m, double *a, double *theta) {
  const int C = m->C;
  double u[C], z[C];
  for (int b = 0; b < m->nb; ++b) {
    for (int c = 0; c < C; ++c) u[c] = ox_elu(a[c]);
    for (int o = 0; o < C; ++o) {
      double s = m->b1[b][o];
      for (int c = 0; c < C; ++c) s += m->w1[b][(long)o * C + c] * u[c];
      z[o] = s;
    }
    for (int c = 0; c < C; ++c) u[c] = ox_elu(z[c]);
    for (int o = 0; o < C; ++o) {
      double s = m->b2[b][o];
      for (int c = 0; c < C; ++c) s += m->w2[b][(long)o * C + c] * u[c];
      a[o] += s;
    }
  }
  for (int c = 0; c < C; ++c) u[c] = ox_elu(a[c]);
  for (int o = 0; o < OX_NOUT; ++o) {
    double s = m->head_b[o];
    for (int c = 0; c < C; ++c) s += m->head_w[(long)o * C + c] * u[c];
    theta[o] = s;
  }
}

/* Pre-activation logits theta[100] of pixel (i,j) of a canvas of normalised
 * values (H x W x 3, NaN where not yet decoded). Positions outside the canvas
 * read as zero (the padding of Eq. 3). Returns OX_E_NAN if a NaN was read. */
static int ox_theta(const ox_model *m, const double *cv, int H, int W, int i, int j, double *theta) {
  const int h = m->h, K = m->K, C = m->C;
  double a[C];
  int nan_seen = 0;
  for (int c = 0; c < C; ++c) a[c] = m->conv_b[c];
  for (int dy = 0; dy < K; ++dy)
    for (int dx = 0; dx < K; ++dx) {
      if (!ox_tap_live(h, dy, dx)) continue;
      int y = i - h + dy, x = j - h + dx;
      if (y < 0 || y >= H || x < 0 || x >= W) continue; /* zero padding */
      for (int ch = 0; ch < 3; ++ch) {
        double v = cv[((long)y * W + x) * 3 + ch];
        if (isnan(v)) nan_seen = 1;
        for (int c = 0; c < C; ++c) a[c] += m->conv_w[(((long)c * 3 + ch) * K + dy) * K + dx] * v;
      }
    }
  ox_body(m, a, theta);
  return nan_seen ? OX_E_NAN : OX_OK;
}

/* ---------------------------------------------------------------- mixture */

/* Head layout: theta[0:10] mixture logits; theta[10+10c : 20+10c] means of
 * channel c; theta[40+10c : 50+10c] raw log-scales of channel c (floored at
 * -7); theta[70:80], [80:90], [90:100] the pre-tanh coefficients of
 * G|R, B|R and B|G. */
typedef struct {
  double logw[OX_NMIX];
  double mu[3][OX_NMIX], invs[3][OX_NMIX];
  double alpha[OX_NMIX], beta[OX_NMIX], gamma_[OX_NMIX];
} ox_mix;

static double ox_logsumexp(const double *v, int n) {
  double mx = -INFINITY;
  for (int k = 0; k < n; ++k) if (v[k] > mx) mx = v[k];
  if (mx == -INFINITY) return -INFINITY;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += exp(v[k] - mx);
  return mx + log(s);
}

static void ox_mix_from_theta(const double *th, ox_mix *mx) {
  double lse = ox_logsumexp(th, OX_NMIX);
  for (int m = 0; m < OX_NMIX; ++m) {
    mx->logw[m] = th[m] - lse;
    for (int c = 0; c < 3; ++c) {
      mx->mu[c][m] = th[10 + 10 * c + m];
      double ls = th[40 + 10 * c + m];
      if (ls < -7.0) ls = -7.0;
      mx->invs[c][m] = exp(-ls);
    }
    mx->alpha[m] = tanh(th[70 + m]);
    mx->beta[m] = tanh(th[80 + m]);
    mx->gamma_[m] = tanh(th[90 + m]);
  }
}

/* Bin edge B_k = (2k - 256)/255: symbol k covers [B_k, B_{k+1}), B_0 = -inf,
 * B_256 = +inf; its centre is the normalised value k/127.5 - 1. */
static double ox_edge(int k) { return (2.0 * k - 256.0) / 255.0; }

double ox_normalise(int v) { return v / 127.5 - 1.0; }

static double ox_logsigmoid(double z) {
  return z >= 0.0 ? -log1p(exp(-z)) : z - log1p(exp(z));
}

/* log of the probability that a logistic(mu, 1/invs) lands in bin k. */
double ox_log_bin(int k, double mu, double invs) {
  if (k <= 0) return ox_logsigmoid((ox_edge(1) - mu) * invs);
  if (k >= 255) return ox_logsigmoid(-(ox_edge(255) - mu) * invs);
  double zlo = (ox_edge(k) - mu) * invs, zhi = (ox_edge(k + 1) - mu) * invs;
  return ox_logsigmoid(zhi) + ox_logsigmoid(-zlo) + log(-expm1(zlo - zhi));
}

/* Mixture parameters of channel c given the already known earlier channels
 * (normalised values xr, xg). Weights are the posterior ones passed in. */
static void ox_channel_means(const ox_mix *mx, int c, double xr, double xg, double *mu) {
  for (int m = 0; m < OX_NMIX; ++m) {
    if (c == 0) mu[m] = mx->mu[0][m];
    else if (c == 1) mu[m] = mx->mu[1][m] + mx->alpha[m] * xr;
    else mu[m] = mx->mu[2][m] + mx->beta[m] * xr + mx->gamma_[m] * xg;
  }
}

static double ox_sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Quantised CDF row (257 entries) of a mixture with log-weights logw. */
static int ox_cdf_row(const double *logw, const double *mu, const double *invs, int32_t *cdf) {
  cdf[0] = 0;
  cdf[256] = (int32_t)OX_TOTAL;
  for (int k = 1; k < 256; ++k) {
    double b = ox_edge(k), F = 0.0;
    for (int m = 0; m < OX_NMIX; ++m) F += exp(logw[m]) * ox_sigmoid((b - mu[m]) * invs[m]);
    if (isnan(F)) return OX_E_NAN;
    if (F < 0.0) F = 0.0;
    if (F > 1.0) F = 1.0;
    cdf[k] = k + (int32_t)floor(F * OX_SPREAD);
  }
  for (int k = 0; k < 256; ++k)
    if (cdf[k + 1] - cdf[k] < 1) return OX_E_CDF;
  return OX_OK;
}

/* Posterior log-weights after observing symbol x of a channel, and that
 * channel's continuous log-probability (natural log). */
static double ox_posterior(double *logw, const double *mu, const double *invs, int x) {
  double t[OX_NMIX];
  for (int m = 0; m < OX_NMIX; ++m) t[m] = logw[m] + ox_log_bin(x, mu[m], invs[m]);
  double lp = ox_logsumexp(t, OX_NMIX);
  for (int m = 0; m < OX_NMIX; ++m) logw[m] = t[m] - lp;
  return lp;
}

/* ---------------------------------------------------------------- rANS */
/* Byte-wise rANS (Duda 2013) with precision M = 2^16, L = 2^23, a 32-bit
 * state, and no wasted start-up or flush bits:
 *   - the encoder starts at x = 1 and the decoder must end there: a damaged
 *     stream that runs out of bytes drains to 0, which a spread pop never
 *     leaves (the cost of this check is about one bit);
 *   - a push of symbol (s, f) from a state x >= f is the usual
 *     x <- floor(x / f) M + (x mod f) + s, after emitting low bytes while
 *     x >= 2^15 f;
 *   - a push from a state x < f (only ever at the start of a stream) uses
 *     the symbol's spread slots instead of its range [s, s + f): x <- the
 *     x-th (from 0) of the slots y in [0, M) whose 16-bit reversal lies in
 *     [s, s + f). Reversal deals f consecutive values out over [0, M) about
 *     M / f apart (every block of 2^(16-p) slots, 2^p <= f, holds one), so
 *     the state grows by about M / f, as it does once it is large; the usual
 *     rule would jump to s + x. Both rules are bijections, the first onto the
 *     states >= M, the second onto [0, M), so the decoder tells them apart by
 *     x < M;
 *   - the final state is flushed as its significant bytes only, most
 *     significant first; the decoder starts from x = 0 and reads bytes
 *     while x < L, as in any renormalisation.
 * A stream therefore costs its ideal length plus about the rounding of its
 * last byte. */

typedef struct {
  uint8_t *tmp; size_t n, cap; /* bytes in emission order */
} ox_bytes;

static int ox_push(ox_bytes *b, uint8_t v) {
  if (b->n == b->cap) {
    size_t nc = b->cap ? 2 * b->cap : 1024;
    uint8_t *t = (uint8_t *)realloc(b->tmp, nc);
    if (!t) return OX_E_CAP;
    b->tmp = t; b->cap = nc;
  }
  b->tmp[b->n++] = v;
  return OX_OK;
}

/* 16-bit bit reversal, from a table filled bit by bit on first use */
static uint16_t ox_rev_table[OX_TOTAL];
static int ox_rev_ready = 0;

static uint32_t ox_rev16(uint32_t v) {
  if (!ox_rev_ready) {
    for (uint32_t u = 0; u < OX_TOTAL; ++u) {
      uint32_t r = 0;
      for (int b = 0; b < 16; ++b)
        if (u & (1u << b)) r |= 1u << (15 - b);
      ox_rev_table[u] = (uint16_t)r;
    }
    ox_rev_ready = 1;
  }
  return ox_rev_table[v & 0xffffu];
}

static int ox_is_spread_slot(uint32_t y, uint32_t s, uint32_t f) {
  uint32_t v = ox_rev16(y);
  return v >= s && v < s + f;
}

/* The x-th spread slot of symbol (s, f), x < f: a plain scan. */
uint32_t ox_spread_select(uint32_t x, uint32_t s, uint32_t f) {
  uint32_t n = 0;
  for (uint32_t y = 0; y < OX_TOTAL; ++y)
    if (ox_is_spread_slot(y, s, f)) {
      if (n == x) return y;
      ++n;
    }
  return OX_TOTAL; /* x >= f */
}

/* Index of slot y among the spread slots of (s, f): slots below y. */
uint32_t ox_spread_rank(uint32_t y, uint32_t s, uint32_t f) {
  uint32_t n = 0;
  for (uint32_t u = 0; u < y; ++u) n += (uint32_t)ox_is_spread_slot(u, s, f);
  return n;
}

/* Encode symbols (start[n], freq[n]) given in decode order; writes the
 * stream (final state's significant bytes, most significant first, then the
 * renormalisation bytes in read order) into out. Returns the byte count or
 * a negative error. */
long ox_rans_encode(const uint32_t *start, const uint32_t *freq, long N, uint8_t *out, size_t cap) {
  ox_bytes b = {0, 0, 0};
  uint32_t x = 1;
  for (long n = N - 1; n >= 0; --n) {
    uint32_t f = freq[n], s = start[n];
    if (f == 0 || f > OX_TOTAL || s + f > OX_TOTAL) { free(b.tmp); return OX_E_ARG; }
    if (x < f) {
      x = ox_spread_select(x, s, f);
      continue;
    }
    uint64_t xmax = (uint64_t)(OX_RANS_L >> 16) * 256u * f;
    while ((uint64_t)x >= xmax) { ox_push(&b, (uint8_t)(x & 255u)); x >>= 8; }
    x = ((x / f) << 16) + (x % f) + s;
  }
  size_t nstate = 0;
  for (uint32_t v = x; v; v >>= 8) ++nstate;
  size_t total = nstate + b.n;
  if (total > cap) { free(b.tmp); return OX_E_CAP; }
  for (size_t k = 0; k < nstate; ++k) out[k] = (uint8_t)(x >> (8 * (nstate - 1 - k)));
  for (size_t k = 0; k < b.n; ++k) out[nstate + k] = b.tmp[b.n - 1 - k];
  free(b.tmp);
  return (long)total;
}

typedef struct {
  uint32_t x; const uint8_t *buf; size_t len, pos;
} ox_rdec;

static void ox_rdec_fill(ox_rdec *d) {
  while (d->x < OX_RANS_L && d->pos < d->len) d->x = (d->x << 8) | d->buf[d->pos++];
}

static void ox_rdec_init(ox_rdec *d, const uint8_t *buf, size_t len) {
  d->buf = buf; d->len = len; d->pos = 0; d->x = 0;
  ox_rdec_fill(d);
}

/* The value the symbol is searched with: the slot x mod M, or for a state
 * below M (a spread push) the reversal of the slot. */
static uint32_t ox_rdec_slot(const ox_rdec *d) {
  return d->x < OX_TOTAL ? ox_rev16(d->x) : (d->x & 0xffffu);
}

static void ox_rdec_advance(ox_rdec *d, uint32_t s, uint32_t f) {
  if (d->x < OX_TOTAL) d->x = ox_spread_rank(d->x, s, f);
  else d->x = f * (d->x >> 16) + (d->x & 0xffffu) - s;
  ox_rdec_fill(d);
}

/* a stream ends in the encoder's start state with every byte read */
static int ox_rdec_clean(const ox_rdec *d) { return d->x == 1u && d->pos == d->len; }

/* Decode N symbols, each with its own CDF row cdfs[n*257..]. */
long ox_rans_decode(const int32_t *cdfs, long N, const uint8_t *in, size_t len, int32_t *sym) {
  ox_rdec d;
  ox_rdec_init(&d, in, len);
  for (long n = 0; n < N; ++n) {
    const int32_t *c = cdfs + 257 * n;
    uint32_t slot = ox_rdec_slot(&d);
    int k = 0;
    while (k < 255 && (uint32_t)c[k + 1] <= slot) ++k;
    sym[n] = k;
    ox_rdec_advance(&d, (uint32_t)c[k], (uint32_t)(c[k + 1] - c[k]));
  }
  return ox_rdec_clean(&d) ? OX_OK : OX_E_CORRUPT;
}

/* ---------------------------------------------------------------- schedule */

/* Number of wavefront steps of an H x W lane (Sec. 3): T = W + (h+1)(H-1). */
long ox_steps(int H, int W, int h) { return (long)W + (long)(h + 1) * (H - 1); }

/* Symbol sequence of a lane in decode order: each entry is (i, j, c).
 * offset 0: raster order (i, j, c). offset o > 0: wavefront order, pixel
 * (i, j) at step t = j + o*i, symbols of a step ordered by channel, then by
 * increasing row. The paper's topological order (Fig. 3) is o = h + 1; any
 * o >= h + 1 is causal, o <= h is not. */
long ox_symbol_order(int H, int W, int offset, int *seq) {
  long n = 0;
  if (offset <= 0) {
    for (int i = 0; i < H; ++i)
      for (int j = 0; j < W; ++j)
        for (int c = 0; c < 3; ++c) { seq[3 * n] = i; seq[3 * n + 1] = j; seq[3 * n + 2] = c; ++n; }
  } else {
    long T = (long)W + (long)offset * (H - 1);
    for (long t = 0; t < T; ++t)
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < H; ++i) {
          long j = t - (long)offset * i;
          if (j < 0 || j >= W) continue;
          seq[3 * n] = i; seq[3 * n + 1] = (int)j; seq[3 * n + 2] = c; ++n;
        }
  }
  return n;
}

/* ---------------------------------------------------------------- lanes */

typedef struct { int y0, x0, h, w; } ox_rect;

static int ox_lanes(int H, int W, int ph, int pw, ox_rect *r) {
  if (ph <= 0 || ph > H) ph = H;
  if (pw <= 0 || pw > W) pw = W;
  int n = 0;
  for (int y = 0; y < H; y += ph)
    for (int x = 0; x < W; x += pw) {
      if (r) { r[n].y0 = y; r[n].x0 = x; r[n].h = (H - y < ph) ? H - y : ph; r[n].w = (W - x < pw) ? W - x : pw; }
      ++n;
    }
  return n;
}

int ox_lane_count(int H, int W, int ph, int pw) { return ox_lanes(H, W, ph, pw, NULL); }

/* Per-pixel work shared by encoder, decoder and statistics: the state of one
 * pixel between its channels. */
typedef struct {
  ox_mix mx;
  double logw[OX_NMIX];
  double xt[3];
} ox_px;

static int ox_px_begin(const ox_model *m, const double *cv, int H, int W, int i, int j, ox_px *p) {
  double th[OX_NOUT];
  int rc = ox_theta(m, cv, H, W, i, j, th);
  if (rc) return rc;
  ox_mix_from_theta(th, &p->mx);
  memcpy(p->logw, p->mx.logw, sizeof(p->logw));
  p->xt[0] = p->xt[1] = p->xt[2] = 0.0;
  return OX_OK;
}

/* CDF row of channel c of a pixel (earlier channels already set in p->xt). */
static int ox_px_cdf(const ox_px *p, int c, int32_t *cdf, double *mu) {
  ox_channel_means(&p->mx, c, p->xt[0], p->xt[1], mu);
  return ox_cdf_row(p->logw, mu, p->mx.invs[c], cdf);
}

/* Record the value x of channel c: posterior update; returns ln p(x | ...). */
static double ox_px_commit(ox_px *p, int c, const double *mu, int x) {
  double lp = ox_posterior(p->logw, mu, p->mx.invs[c], x);
  p->xt[c] = ox_normalise(x);
  return lp;
}

/* Statistics of one lane in raster order: quantised ideal bits, continuous
 * bits, optional CDF rows and per-pixel continuous bits (lane-local index). */
static int ox_lane_stats(const ox_model *m, const uint8_t *img, int W_img, ox_rect r, double *qbits,
                         double *cbits, int32_t *cdf_out, double *px_bits, int Wfull) {
  long n = (long)r.h * r.w;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  for (int y = 0; y < r.h; ++y)
    for (int x = 0; x < r.w; ++x)
      for (int c = 0; c < 3; ++c)
        cv[((long)y * r.w + x) * 3 + c] = ox_normalise(img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c]);
  int32_t cdf[257];
  double mu[OX_NMIX];
  int rc = OX_OK;
  for (int y = 0; y < r.h && !rc; ++y)
    for (int x = 0; x < r.w && !rc; ++x) {
      ox_px p;
      rc = ox_px_begin(m, cv, r.h, r.w, y, x, &p);
      if (rc) break;
      double pb = 0.0;
      for (int c = 0; c < 3; ++c) {
        rc = ox_px_cdf(&p, c, cdf, mu);
        if (rc) break;
        int v = img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c];
        if (cdf_out) memcpy(cdf_out + ((((long)(r.y0 + y)) * Wfull + r.x0 + x) * 3 + c) * 257, cdf, sizeof(cdf));
        *qbits += -log2((double)(cdf[v + 1] - cdf[v]) / OX_TOTAL);
        double lp = ox_px_commit(&p, c, mu, v);
        pb += -lp / log(2.0);
      }
      *cbits += pb;
      if (px_bits) px_bits[((long)(r.y0 + y)) * Wfull + r.x0 + x] = pb;
    }
  free(cv);
  return rc;
}

/* Whole-image statistics under a patch grid (ph, pw; 0 = whole image).
 * stats_out = {quantised ideal bits, continuous bits}. */
int ox_stats(const ox_model *m, const uint8_t *img, int H, int W, int ph, int pw, double *stats_out,
             int32_t *cdf_out, double *px_bits) {
  if (!m || !img || H < 1 || W < 1) return OX_E_ARG;
  int nl = ox_lane_count(H, W, ph, pw);
  ox_rect *r = (ox_rect *)malloc(sizeof(ox_rect) * nl);
  ox_lanes(H, W, ph, pw, r);
  double q = 0.0, cb = 0.0;
  int rc = OX_OK;
  for (int l = 0; l < nl && !rc; ++l) rc = ox_lane_stats(m, img, W, r[l], &q, &cb, cdf_out, px_bits, W);
  free(r);
  if (stats_out) { stats_out[0] = q; stats_out[1] = cb; }
  return rc;
}

/* theta[H*W][100] of every pixel (whole image as one lane) -- for cross
 * checks of the network against an independent implementation. */
int ox_theta_image(const ox_model *m, const uint8_t *img, int H, int W, double *theta) {
  long n = (long)H * W;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  for (long k = 0; k < 3 * n; ++k) cv[k] = ox_normalise(img[k]);
  int rc = OX_OK;
  for (int i = 0; i < H && !rc; ++i)
    for (int j = 0; j < W && !rc; ++j) rc = ox_theta(m, cv, H, W, i, j, theta + ((long)i * W + j) * OX_NOUT);
  free(cv);
  return rc;
}

/* ---------------------------------------------------------------- codec */
/* Oracle container: u32 n_lanes, u32 lane_bytes[n_lanes], payloads. */

static long ox_encode_lane(const ox_model *m, const uint8_t *img, int W_img, ox_rect r, int offset, uint8_t *out,
                           size_t cap) {
  long n = (long)r.h * r.w;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  for (int y = 0; y < r.h; ++y)
    for (int x = 0; x < r.w; ++x)
      for (int c = 0; c < 3; ++c)
        cv[((long)y * r.w + x) * 3 + c] = ox_normalise(img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c]);
  /* start/freq of every (pixel, channel), lane-local raster index */
  uint32_t *st = (uint32_t *)malloc(sizeof(uint32_t) * 3 * n), *fr = (uint32_t *)malloc(sizeof(uint32_t) * 3 * n);
  int32_t cdf[257];
  double mu[OX_NMIX];
  int rc = OX_OK;
  for (int y = 0; y < r.h && !rc; ++y)
    for (int x = 0; x < r.w && !rc; ++x) {
      ox_px p;
      rc = ox_px_begin(m, cv, r.h, r.w, y, x, &p);
      for (int c = 0; c < 3 && !rc; ++c) {
        rc = ox_px_cdf(&p, c, cdf, mu);
        if (rc) break;
        int v = img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c];
        long idx = ((long)y * r.w + x) * 3 + c;
        st[idx] = (uint32_t)cdf[v];
        fr[idx] = (uint32_t)(cdf[v + 1] - cdf[v]);
        ox_px_commit(&p, c, mu, v);
      }
    }
  long ret = rc;
  if (!rc) {
    int *seq = (int *)malloc(sizeof(int) * 9 * n);
    long N = ox_symbol_order(r.h, r.w, offset, seq);
    uint32_t *s2 = (uint32_t *)malloc(sizeof(uint32_t) * N), *f2 = (uint32_t *)malloc(sizeof(uint32_t) * N);
    for (long k = 0; k < N; ++k) {
      long idx = ((long)seq[3 * k] * r.w + seq[3 * k + 1]) * 3 + seq[3 * k + 2];
      s2[k] = st[idx]; f2[k] = fr[idx];
    }
    ret = ox_rans_encode(s2, f2, N, out, cap);
    free(s2); free(f2); free(seq);
  }
  free(st); free(fr); free(cv);
  return ret;
}

/* Encode an image; offset 0 = raster order, o > 0 = wavefront order with
 * step j + o*i. Returns container bytes written, or a negative error. */
long ox_encode_offset(const ox_model *m, const uint8_t *img, int H, int W, int offset, int ph, int pw, uint8_t *out,
                      size_t cap) {
  if (!m || !img || !out || H < 1 || W < 1 || offset < 0) return OX_E_ARG;
  int nl = ox_lane_count(H, W, ph, pw);
  ox_rect *r = (ox_rect *)malloc(sizeof(ox_rect) * nl);
  ox_lanes(H, W, ph, pw, r);
  size_t hdr = 4 + 4 * (size_t)nl;
  if (cap < hdr) { free(r); return OX_E_CAP; }
  size_t pos = hdr;
  long rc = OX_OK;
  for (int l = 0; l < nl; ++l) {
    long nbytes = ox_encode_lane(m, img, W, r[l], offset, out + pos, cap - pos);
    if (nbytes < 0) { rc = nbytes; break; }
    for (int k = 0; k < 4; ++k) out[4 + 4 * l + k] = (uint8_t)((uint32_t)nbytes >> (8 * k));
    pos += (size_t)nbytes;
  }
  for (int k = 0; k < 4; ++k) out[k] = (uint8_t)((uint32_t)nl >> (8 * k));
  free(r);
  return rc < 0 ? rc : (long)pos;
}

/* order 0 = raster, 1 = the paper's wavefront order (offset h + 1). */
long ox_encode(const ox_model *m, const uint8_t *img, int H, int W, int order, int ph, int pw, uint8_t *out,
               size_t cap) {
  if (!m || (order != 0 && order != 1)) return OX_E_ARG;
  return ox_encode_offset(m, img, H, W, order ? m->h + 1 : 0, ph, pw, out, cap);
}

/* Decode one lane; the canvas starts as NaN ("poisoned") so that a read of a
 * pixel the order has not produced yet turns into OX_E_NAN. */
static int ox_decode_lane(const ox_model *m, const uint8_t *in, size_t len, ox_rect r, int offset, uint8_t *img,
                          int W_img) {
  long n = (long)r.h * r.w;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  for (long k = 0; k < 3 * n; ++k) cv[k] = NAN;
  ox_px *pxs = (ox_px *)malloc(sizeof(ox_px) * n);
  int *seq = (int *)malloc(sizeof(int) * 3 * 3 * n);
  long N = ox_symbol_order(r.h, r.w, offset, seq);
  ox_rdec d;
  ox_rdec_init(&d, in, len);
  int rc = OX_OK;
  int32_t cdf[257];
  double mu[OX_NMIX];
  for (long k = 0; k < N && !rc; ++k) {
    int y = seq[3 * k], x = seq[3 * k + 1], c = seq[3 * k + 2];
    long pi = (long)y * r.w + x;
    if (c == 0) { rc = ox_px_begin(m, cv, r.h, r.w, y, x, &pxs[pi]); if (rc) break; }
    rc = ox_px_cdf(&pxs[pi], c, cdf, mu);
    if (rc) break;
    uint32_t slot = ox_rdec_slot(&d);
    int v = 0;
    while (v < 255 && (uint32_t)cdf[v + 1] <= slot) ++v;
    ox_rdec_advance(&d, (uint32_t)cdf[v], (uint32_t)(cdf[v + 1] - cdf[v]));
    ox_px_commit(&pxs[pi], c, mu, v);
    cv[pi * 3 + c] = ox_normalise(v);
    img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c] = (uint8_t)v;
  }
  if (!rc && !ox_rdec_clean(&d)) rc = OX_E_CORRUPT;
  free(cv); free(pxs); free(seq);
  return rc;
}

int ox_decode_offset(const ox_model *m, const uint8_t *in, size_t len, int H, int W, int offset, int ph, int pw,
                     uint8_t *img) {
  if (!m || !in || !img || H < 1 || W < 1 || offset < 0) return OX_E_ARG;
  int nl = ox_lane_count(H, W, ph, pw);
  if (len < 4 || (int)rd32(in) != nl || len < 4 + 4 * (size_t)nl) return OX_E_CORRUPT;
  ox_rect *r = (ox_rect *)malloc(sizeof(ox_rect) * nl);
  ox_lanes(H, W, ph, pw, r);
  size_t pos = 4 + 4 * (size_t)nl;
  int rc = OX_OK;
  for (int l = 0; l < nl && !rc; ++l) {
    size_t nb = rd32(in + 4 + 4 * l);
    if (pos + nb > len) { rc = OX_E_CORRUPT; break; }
    rc = ox_decode_lane(m, in + pos, nb, r[l], offset, img, W);
    pos += nb;
  }
  if (!rc && pos != len) rc = OX_E_CORRUPT;
  free(r);
  return rc;
}

int ox_decode(const ox_model *m, const uint8_t *in, size_t len, int H, int W, int order, int ph, int pw,
              uint8_t *img) {
  if (!m || (order != 0 && order != 1)) return OX_E_ARG;
  return ox_decode_offset(m, in, len, H, W, order ? m->h + 1 : 0, ph, pw, img);
}

/* ---------------------------------------------------------------- sampling */

/* Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
 * products; the key is bumped by the two Weyl constants between rounds. */
void ox_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x0, p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0, hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The uniform slot of channel c of pixel (y, x) of an H x W image (absolute
 * coordinates): the top 16 bits of word c of the Philox block with counter
 * (y W + x, 0, 0, 0) and key (seed, 0). */
uint32_t ox_sample_slot(uint64_t seed, int W, int y, int x, int c) {
  uint64_t ctr[4] = {(uint64_t)y * (uint64_t)W + (uint64_t)x, 0, 0, 0}, key[2] = {seed, 0}, o[4];
  ox_philox4x64(ctr, key, o);
  return (uint32_t)(o[c] >> 48);
}

/* Ancestral sampling of one lane in the decoding order of `offset`: per
 * symbol, the CDF row given what is already drawn, then the unique v with
 * cdf[v] <= slot < cdf[v + 1]; P(v) = freq_v / 2^16. */
static int ox_sample_lane(const ox_model *m, ox_rect r, int offset, uint64_t seed, uint8_t *img, int W_img) {
  long n = (long)r.h * r.w;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  for (long k = 0; k < 3 * n; ++k) cv[k] = NAN;
  ox_px *pxs = (ox_px *)malloc(sizeof(ox_px) * n);
  int *seq = (int *)malloc(sizeof(int) * 3 * 3 * n);
  long N = ox_symbol_order(r.h, r.w, offset, seq);
  int rc = OX_OK;
  int32_t cdf[257];
  double mu[OX_NMIX];
  for (long k = 0; k < N && !rc; ++k) {
    int y = seq[3 * k], x = seq[3 * k + 1], c = seq[3 * k + 2];
    long pi = (long)y * r.w + x;
    if (c == 0) { rc = ox_px_begin(m, cv, r.h, r.w, y, x, &pxs[pi]); if (rc) break; }
    rc = ox_px_cdf(&pxs[pi], c, cdf, mu);
    if (rc) break;
    uint32_t slot = ox_sample_slot(seed, W_img, r.y0 + y, r.x0 + x, c);
    int v = 0;
    while (v < 255 && (uint32_t)cdf[v + 1] <= slot) ++v;
    ox_px_commit(&pxs[pi], c, mu, v);
    cv[pi * 3 + c] = ox_normalise(v);
    img[(((long)(r.y0 + y)) * W_img + r.x0 + x) * 3 + c] = (uint8_t)v;
  }
  free(cv); free(pxs); free(seq);
  return rc;
}

/* Sample an H x W image (patches of ph x pw sampled independently, as they
 * are coded) in the order of `offset` (0 raster, h + 1 wavefront). */
int ox_sample(const ox_model *m, int H, int W, int offset, int ph, int pw, uint64_t seed, uint8_t *img) {
  if (!m || !img || H < 1 || W < 1 || offset < 0) return OX_E_ARG;
  int nl = ox_lane_count(H, W, ph, pw);
  ox_rect *r = (ox_rect *)malloc(sizeof(ox_rect) * nl);
  ox_lanes(H, W, ph, pw, r);
  int rc = OX_OK;
  for (int l = 0; l < nl && !rc; ++l) rc = ox_sample_lane(m, r[l], offset, seed, img, W);
  free(r);
  return rc;
}

/* ---------------------------------------------------------------- ShearLoC */

/* Shear (Sec. 3.1, Fig. 4b) an H x W x nc array with offset o into H x L x nc,
 * L = W + o (H - 1): element (i, j) goes to column j + o i; the rest is 0. */
void ox_shear(const double *x, int H, int W, int nc, int o, double *S) {
  long L = (long)W + (long)o * (H - 1);
  for (long k = 0; k < (long)H * L * nc; ++k) S[k] = 0.0;
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j)
      for (int c = 0; c < nc; ++c) S[((long)i * L + j + (long)o * i) * nc + c] = x[((long)i * W + j) * nc + c];
}

/* Undo the shear: x(i, j) = S(i, j + o i). */
void ox_unshear(const double *S, int H, int W, int nc, int o, double *x) {
  long L = (long)W + (long)o * (H - 1);
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j)
      for (int c = 0; c < nc; ++c) x[((long)i * W + j) * nc + c] = S[((long)i * L + j + (long)o * i) * nc + c];
}

/* The sheared first kernel (Sec. 3.1, Fig. 5b/5d): (h+1) rows by Q = h(h+2)
 * columns. Row a of the unsheared causal kernel moves right by o a
 * (o = h + 1); kernel column q then reads sheared column t - Q + q of the
 * pixel's own column t, so only earlier columns are read. */
int ox_shear_tap_live(int h, int a, int q) {
  int dx = q - (h + 1) * a;
  return a >= 0 && a <= h && dx >= 0 && dx <= 2 * h && ox_tap_live(h, a, dx);
}

/* Kp[c][ch][a][q] (C x 3 x (h+1) x h(h+2)) from the model's first kernel. */
void ox_shear_kernel(const ox_model *m, double *Kp) {
  const int h = m->h, K = m->K, C = m->C, Q = h * (h + 2);
  for (int c = 0; c < C; ++c)
    for (int ch = 0; ch < 3; ++ch)
      for (int a = 0; a <= h; ++a)
        for (int q = 0; q < Q; ++q) {
          double w = 0.0;
          if (ox_shear_tap_live(h, a, q)) w = m->conv_w[(((long)c * 3 + ch) * K + a) * K + (q - (h + 1) * a)];
          Kp[(((long)c * 3 + ch) * (h + 1) + a) * Q + q] = w;
        }
}

/* theta[100] of the pixel at row i, sheared column t, of a sheared canvas S
 * (H x L x 3, NaN where not decoded yet, 0 off the image): the sheared
 * kernel over columns t - Q .. t - 1 of rows i - h .. i (rows above the
 * image read 0), then the unchanged 1x1 layers. The live taps are visited
 * in the order of the unsheared kernel. */
static int ox_theta_sheared(const ox_model *m, const double *Kp, const double *S, int H, long L, int i, long t,
                            double *theta) {
  const int h = m->h, C = m->C, Q = h * (h + 2);
  double a[C];
  int nan_seen = 0;
  (void)H;
  for (int c = 0; c < C; ++c) a[c] = m->conv_b[c];
  for (int ka = 0; ka <= h; ++ka)
    for (int q = 0; q < Q; ++q) {
      if (!ox_shear_tap_live(h, ka, q)) continue;
      int r = i - h + ka;
      long tau = t - Q + q;
      if (r < 0 || tau < 0) continue; /* above the image / left of column 0 */
      for (int ch = 0; ch < 3; ++ch) {
        double v = S[((long)r * L + tau) * 3 + ch];
        if (isnan(v)) nan_seen = 1;
        for (int c = 0; c < C; ++c) a[c] += Kp[(((long)c * 3 + ch) * (h + 1) + ka) * Q + q] * v;
      }
    }
  ox_body(m, a, theta);
  return nan_seen ? OX_E_NAN : OX_OK;
}

/* theta of every pixel of a complete image, computed in the sheared model. */
int ox_theta_image_shear(const ox_model *m, const uint8_t *img, int H, int W, double *theta) {
  const int o = m->h + 1;
  long L = (long)W + (long)o * (H - 1), n = (long)H * W;
  double *cv = (double *)malloc(sizeof(double) * 3 * n);
  double *S = (double *)malloc(sizeof(double) * 3 * (size_t)H * L);
  double *Kp = (double *)malloc(sizeof(double) * (size_t)m->C * 3 * (m->h + 1) * m->h * (m->h + 2));
  for (long k = 0; k < 3 * n; ++k) cv[k] = ox_normalise(img[k]);
  ox_shear(cv, H, W, 3, o, S);
  ox_shear_kernel(m, Kp);
  int rc = OX_OK;
  for (int i = 0; i < H && !rc; ++i)
    for (int j = 0; j < W && !rc; ++j)
      rc = ox_theta_sheared(m, Kp, S, H, L, i, j + (long)o * i, theta + ((long)i * W + j) * OX_NOUT);
  free(cv); free(S); free(Kp);
  return rc;
}

/* Algorithm 2 on one lane: the canvas is kept sheared (NaN at every pixel not
 * decoded yet, 0 elsewhere); column t = 0 .. L-1 holds exactly the pixels of
 * wavefront step t, decoded in the coder's order from their predictive
 * distributions; the sheared byte canvas is unsheared at the end. */
static int ox_decode_lane_shear(const ox_model *m, const double *Kp, const uint8_t *in, size_t len, ox_rect r,
                                uint8_t *img, int W_img) {
  const int o = m->h + 1, H = r.h, W = r.w;
  long L = (long)W + (long)o * (H - 1), n = (long)H * W;
  double *nanimg = (double *)malloc(sizeof(double) * 3 * n);
  double *S = (double *)malloc(sizeof(double) * 3 * (size_t)H * L);
  double *Sb = (double *)malloc(sizeof(double) * 3 * (size_t)H * L);
  double *out = (double *)malloc(sizeof(double) * 3 * n);
  for (long k = 0; k < 3 * n; ++k) nanimg[k] = NAN;
  ox_shear(nanimg, H, W, 3, o, S); /* poisoned pixels, zero padding */
  for (long k = 0; k < 3 * (long)H * L; ++k) Sb[k] = 0.0;
  ox_px *pxs = (ox_px *)malloc(sizeof(ox_px) * n);
  int *seq = (int *)malloc(sizeof(int) * 3 * 3 * n);
  long N = ox_symbol_order(H, W, o, seq);
  ox_rdec d;
  ox_rdec_init(&d, in, len);
  int rc = OX_OK;
  int32_t cdf[257];
  double mu[OX_NMIX], th[OX_NOUT];
  for (long k = 0; k < N && !rc; ++k) {
    int i = seq[3 * k], j = seq[3 * k + 1], c = seq[3 * k + 2];
    long t = j + (long)o * i, pi = (long)i * W + j;
    if (c == 0) {
      rc = ox_theta_sheared(m, Kp, S, H, L, i, t, th);
      if (rc) break;
      ox_mix_from_theta(th, &pxs[pi].mx);
      memcpy(pxs[pi].logw, pxs[pi].mx.logw, sizeof(pxs[pi].logw));
      pxs[pi].xt[0] = pxs[pi].xt[1] = pxs[pi].xt[2] = 0.0;
    }
    rc = ox_px_cdf(&pxs[pi], c, cdf, mu);
    if (rc) break;
    uint32_t slot = ox_rdec_slot(&d);
    int v = 0;
    while (v < 255 && (uint32_t)cdf[v + 1] <= slot) ++v;
    ox_rdec_advance(&d, (uint32_t)cdf[v], (uint32_t)(cdf[v + 1] - cdf[v]));
    ox_px_commit(&pxs[pi], c, mu, v);
    S[((long)i * L + t) * 3 + c] = ox_normalise(v);
    Sb[((long)i * L + t) * 3 + c] = (double)v;
  }
  if (!rc && !ox_rdec_clean(&d)) rc = OX_E_CORRUPT;
  if (!rc) {
    ox_unshear(Sb, H, W, 3, o, out);
    for (int i = 0; i < H; ++i)
      for (int j = 0; j < W; ++j)
        for (int c = 0; c < 3; ++c)
          img[(((long)(r.y0 + i)) * W_img + r.x0 + j) * 3 + c] = (uint8_t)out[((long)i * W + j) * 3 + c];
  }
  free(nanimg); free(S); free(Sb); free(out); free(pxs); free(seq);
  return rc;
}

/* Decode a wavefront-order container with the sheared model (Algorithm 2). */
int ox_decode_shear(const ox_model *m, const uint8_t *in, size_t len, int H, int W, int ph, int pw, uint8_t *img) {
  if (!m || !in || !img || H < 1 || W < 1) return OX_E_ARG;
  int nl = ox_lane_count(H, W, ph, pw);
  if (len < 4 || (int)rd32(in) != nl || len < 4 + 4 * (size_t)nl) return OX_E_CORRUPT;
  ox_rect *r = (ox_rect *)malloc(sizeof(ox_rect) * nl);
  ox_lanes(H, W, ph, pw, r);
  double *Kp = (double *)malloc(sizeof(double) * (size_t)m->C * 3 * (m->h + 1) * m->h * (m->h + 2));
  ox_shear_kernel(m, Kp);
  size_t pos = 4 + 4 * (size_t)nl;
  int rc = OX_OK;
  for (int l = 0; l < nl && !rc; ++l) {
    size_t nb = rd32(in + 4 + 4 * l);
    if (pos + nb > len) { rc = OX_E_CORRUPT; break; }
    rc = ox_decode_lane_shear(m, Kp, in + pos, nb, r[l], img, W);
    pos += nb;
  }
  if (!rc && pos != len) rc = OX_E_CORRUPT;
  free(r); free(Kp);
  return rc;
}
