/*
 * EBCC oracle: a plain, slow, single-threaded CPU implementation of the EBCC
 * compression hot path (two-layer error-bounded compressor, arXiv 2510.22265).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the GPU library: every table below was typed in here from the published
 * standards the paper builds on.
 *
 * What it follows:
 *   - Method section, first paragraph: chunk -> 2-D field, min/max
 *     normalisation, JPEG2000 base layer, residual = input - base, wavelet
 *     transform of the residual, SPIHT bit-plane coding, embedded (prefix
 *     decodable) residual stream.
 *   - Method section, second paragraph, and Algorithm 1 (EBCC Compression
 *     Process): the base layer is run at a compression ratio r and decoded;
 *     the residual is DWT'd and SPIHT coded once; a binary search finds the
 *     lowest truncation point whose reconstruction meets max|A - A_rec| <= eps
 *     (a point with error > eps is a violation); output = Concat(base, residual).
 *   - Benchmarks section: eps is range-relative (max abs error over data range).
 *   - JPEG2000 Part 1 (ITU-T T.800), which the paper uses as its base codec:
 *     Annex F (9/7 irreversible lifting DWT), Annex D (EBCOT tier-1 coding
 *     passes and contexts), Annex C (MQ arithmetic coder), and PCRD-opt rate
 *     allocation (Taubman 2000).
 *   - Said & Pearlman 1996 (SPIHT), cited by the paper for the residual layer.
 *
 * Readings where the paper is silent (the full list is kept with the design
 * notes): a fixed base ratio r or Algorithm 1's q-feedback search, truncation
 * of the residual at bit-plane ends or (trunc = 1) at a byte position of the
 * tiles' codes read as one embedded sequence, power-of-two quantiser steps
 * tied to eps, midpoint reconstruction, FP32 lifting in a fixed operation
 * order with contraction off.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define EXPORT __attribute__((visibility("default")))

enum { REF_OK = 0, REF_EINVAL = -1, REF_ENOSPC = -2, REF_ECORRUPT = -3, REF_ENOMEM = -4 };
enum { MODE_CONST = 0, MODE_RAW = 1, MODE_CODED = 2 };
enum { ORI_LL = 0, ORI_HL = 1, ORI_LH = 2, ORI_HH = 3 };
#define HDR_BYTES 48
#define MAX_LEVELS 16
#define QMAX_BITS 23             /* quantised magnitudes are < 2^23 */
#define QMAX ((1u << QMAX_BITS) - 1u)
#define SEG_RMAX 65535           /* a code-block length must fit the u16 table field */

/* ======================================================================== */
/* 1. CDF 9/7 lifting DWT (T.800 Annex F, irreversible 9/7).                */
/* ======================================================================== */
/* Lifting factors of the CDF 9/7 wavelet (Daubechies-Sweldens factorisation). */
static const double A97 = -1.586134342059924;
static const double B97 = -0.052980118572961;
static const double G97 = 0.882911075530934;
static const double D97 = 0.443506852043971;
static const double K97 = 1.230174104914001;
/* Their nearest binary32 values, used by the FP32 transform. */
static const float A97F = -0x1.960ce6p+0f;
static const float B97F = -0x1.b2035cp-5f;
static const float G97F = 0x1.c40cecp-1f;
static const float D97F = 0x1.c626aap-2f;
static const float K97F = 0x1.3aecb0p+0f;
static const float IK97F = 0x1.a03386p-1f;   /* binary32 of 1/K */

/* One lifting step on the samples of parity `par` of v[0..n-1] (n >= 2),
 * whole-sample symmetric extension: v[-1] = v[1], v[n] = v[n-2].
 * Each update is exactly t = l + r; t = c * t; v = v (+|-) t in FP32. */
static void lift_f(float* v, long n, long par, float c, int sub) {
  for (long i = par; i < n; i += 2) {
    float l = (i - 1 >= 0) ? v[i - 1] : v[i + 1];
    float r = (i + 1 < n) ? v[i + 1] : v[i - 1];
    float t = l + r;
    t = c * t;
    v[i] = sub ? (v[i] - t) : (v[i] + t);
  }
}
static void lift_d(double* v, long n, long par, double c, int sub) {
  for (long i = par; i < n; i += 2) {
    double l = (i - 1 >= 0) ? v[i - 1] : v[i + 1];
    double r = (i + 1 < n) ? v[i + 1] : v[i - 1];
    double t = l + r;
    t = c * t;
    v[i] = sub ? (v[i] - t) : (v[i] + t);
  }
}

/* Forward 1-D transform of v (length n); result deinterleaved into v:
 * low-pass ceil(n/2) samples first, then high-pass floor(n/2). */
static void fwd1_f(float* v, long n, float* tmp) {
  if (n < 2) return;
  lift_f(v, n, 1, A97F, 0);
  lift_f(v, n, 0, B97F, 0);
  lift_f(v, n, 1, G97F, 0);
  lift_f(v, n, 0, D97F, 0);
  for (long i = 0; i < n; i++) v[i] = (i & 1) ? v[i] * K97F : v[i] * IK97F;
  long nl = (n + 1) / 2;
  for (long i = 0; i < n; i++) tmp[(i & 1) ? nl + i / 2 : i / 2] = v[i];
  memcpy(v, tmp, sizeof(float) * (size_t)n);
}
static void inv1_f(float* v, long n, float* tmp) {
  if (n < 2) return;
  long nl = (n + 1) / 2;
  for (long i = 0; i < n; i++) tmp[i] = v[(i & 1) ? nl + i / 2 : i / 2];
  memcpy(v, tmp, sizeof(float) * (size_t)n);
  for (long i = 0; i < n; i++) v[i] = (i & 1) ? v[i] * IK97F : v[i] * K97F;
  lift_f(v, n, 0, D97F, 1);
  lift_f(v, n, 1, G97F, 1);
  lift_f(v, n, 0, B97F, 1);
  lift_f(v, n, 1, A97F, 1);
}
static void fwd1_d(double* v, long n, double* tmp) {
  if (n < 2) return;
  lift_d(v, n, 1, A97, 0);
  lift_d(v, n, 0, B97, 0);
  lift_d(v, n, 1, G97, 0);
  lift_d(v, n, 0, D97, 0);
  for (long i = 0; i < n; i++) v[i] = (i & 1) ? v[i] * K97 : v[i] * (1.0 / K97);
  long nl = (n + 1) / 2;
  for (long i = 0; i < n; i++) tmp[(i & 1) ? nl + i / 2 : i / 2] = v[i];
  memcpy(v, tmp, sizeof(double) * (size_t)n);
}
static void inv1_d(double* v, long n, double* tmp) {
  if (n < 2) return;
  long nl = (n + 1) / 2;
  for (long i = 0; i < n; i++) tmp[i] = v[(i & 1) ? nl + i / 2 : i / 2];
  memcpy(v, tmp, sizeof(double) * (size_t)n);
  for (long i = 0; i < n; i++) v[i] = (i & 1) ? v[i] * (1.0 / K97) : v[i] * K97;
  lift_d(v, n, 0, D97, 1);
  lift_d(v, n, 1, G97, 1);
  lift_d(v, n, 0, B97, 1);
  lift_d(v, n, 1, A97, 1);
}

/* Number of levels actually applied: every level's input length must be >= 2. */
static int levels_eff(long ny, long nx, int L) {
  long m = ny < nx ? ny : nx;
  int f = 0;
  while ((2L << f) <= m) f++;        /* f = floor(log2 m) */
  if (L > f) L = f;
  if (L > MAX_LEVELS) L = MAX_LEVELS;
  return L < 0 ? 0 : L;
}
/* LL region sizes: h[0] = ny, h[l] = ceil(h[l-1] / 2). */
static void ll_sizes(long ny, long nx, int L, long* h, long* w) {
  h[0] = ny; w[0] = nx;
  for (int l = 1; l <= L; l++) { h[l] = (h[l - 1] + 1) / 2; w[l] = (w[l - 1] + 1) / 2; }
}

/* 2-D multi-level transform, Mallat layout in place (row-major, stride nx).
 * Each level: all columns of the current LL region (vertical), then all rows
 * (horizontal).  The inverse undoes the levels in reverse, rows then columns. */
static void dwt2_f(float* a, long ny, long nx, int L, int inverse) {
  long h[MAX_LEVELS + 1], w[MAX_LEVELS + 1];
  ll_sizes(ny, nx, L, h, w);
  long mx = ny > nx ? ny : nx;
  float* v = (float*)malloc(sizeof(float) * (size_t)mx);
  float* t = (float*)malloc(sizeof(float) * (size_t)mx);
  for (int s = 0; s < L; s++) {
    int l = inverse ? (L - 1 - s) : s;     /* transform region h[l] x w[l] */
    long H = h[l], W = w[l];
    if (!inverse) {
      for (long j = 0; j < W; j++) {
        for (long i = 0; i < H; i++) v[i] = a[i * nx + j];
        fwd1_f(v, H, t);
        for (long i = 0; i < H; i++) a[i * nx + j] = v[i];
      }
      for (long i = 0; i < H; i++) fwd1_f(a + i * nx, W, t);
    } else {
      for (long i = 0; i < H; i++) inv1_f(a + i * nx, W, t);
      for (long j = 0; j < W; j++) {
        for (long i = 0; i < H; i++) v[i] = a[i * nx + j];
        inv1_f(v, H, t);
        for (long i = 0; i < H; i++) a[i * nx + j] = v[i];
      }
    }
  }
  free(v); free(t);
}
static void dwt2_d(double* a, long ny, long nx, int L, int inverse) {
  long h[MAX_LEVELS + 1], w[MAX_LEVELS + 1];
  ll_sizes(ny, nx, L, h, w);
  long mx = ny > nx ? ny : nx;
  double* v = (double*)malloc(sizeof(double) * (size_t)mx);
  double* t = (double*)malloc(sizeof(double) * (size_t)mx);
  for (int s = 0; s < L; s++) {
    int l = inverse ? (L - 1 - s) : s;
    long H = h[l], W = w[l];
    if (!inverse) {
      for (long j = 0; j < W; j++) {
        for (long i = 0; i < H; i++) v[i] = a[i * nx + j];
        fwd1_d(v, H, t);
        for (long i = 0; i < H; i++) a[i * nx + j] = v[i];
      }
      for (long i = 0; i < H; i++) fwd1_d(a + i * nx, W, t);
    } else {
      for (long i = 0; i < H; i++) inv1_d(a + i * nx, W, t);
      for (long j = 0; j < W; j++) {
        for (long i = 0; i < H; i++) v[i] = a[i * nx + j];
        inv1_d(v, H, t);
        for (long i = 0; i < H; i++) a[i * nx + j] = v[i];
      }
    }
  }
  free(v); free(t);
}

/* ======================================================================== */
/* 2. Subbands, synthesis gains, code-blocks.                               */
/* ======================================================================== */
typedef struct { int level, orient; long y0, x0, h, w; } band_t;

/* Band order: LL_L, then HL_l, LH_l, HH_l for l = L .. 1.  HL = horizontal
 * high-pass (top-right), LH = vertical high-pass (bottom-left). */
static int make_bands(long ny, long nx, int L, band_t* b) {
  long h[MAX_LEVELS + 1], w[MAX_LEVELS + 1];
  ll_sizes(ny, nx, L, h, w);
  int n = 0;
  b[n++] = (band_t){L, ORI_LL, 0, 0, h[L], w[L]};
  for (int l = L; l >= 1; l--) {
    b[n++] = (band_t){l, ORI_HL, 0, w[l], h[l], w[l - 1] - w[l]};
    b[n++] = (band_t){l, ORI_LH, h[l], 0, h[l - 1] - h[l], w[l]};
    b[n++] = (band_t){l, ORI_HH, h[l], w[l], h[l - 1] - h[l], w[l - 1] - w[l]};
  }
  return n;
}

/* L2 norm of the 1-D synthesis basis function of a level-`level` coefficient
 * (low or high band), measured by running the FP64 inverse transform on a
 * unit impulse placed mid-band in a signal long enough to avoid the edges. */
static double synth_norm_1d(int level, int high) {
  if (level == 0) return 1.0;
  long n = 64L << level;
  long h[MAX_LEVELS + 1], w[MAX_LEVELS + 1];
  ll_sizes(n, n, level, h, w);
  double* v = (double*)calloc((size_t)n, sizeof(double));
  double* t = (double*)malloc(sizeof(double) * (size_t)n);
  long idx = high ? h[level] + (h[level - 1] - h[level]) / 2 : h[level] / 2;
  v[idx] = 1.0;
  for (int l = level - 1; l >= 0; l--) inv1_d(v, h[l], t);
  double s = 0;
  for (long i = 0; i < n; i++) s += v[i] * v[i];
  free(v); free(t);
  return sqrt(s);
}
/* Synthesis L2 norm w_b of a 2-D subband (separable: product of 1-D norms). */
EXPORT double ebcc_ref_band_norm(int level, int orient) {
  double lo = synth_norm_1d(level, 0), hi = synth_norm_1d(level, 1);
  switch (orient) {
    case ORI_LL: return lo * lo;
    case ORI_HL: return hi * lo;
    case ORI_LH: return lo * hi;
    default: return hi * hi;
  }
}
/* g_b = round(log2 w_b): the base quantiser step of band b is 2^(e0 - g_b),
 * i.e. steps are inversely proportional to the synthesis gain (rounded to a
 * power of two so that scaling is exact and distortions are integers). */
EXPORT int ebcc_ref_band_log2_gain(int level, int orient) {
  return (int)lround(log2(ebcc_ref_band_norm(level, orient)));
}

/* ======================================================================== */
/* 3. MQ arithmetic coder (T.800 Annex C).                                  */
/* ======================================================================== */
/* Probability estimation table: Qe, next index after MPS, after LPS, switch. */
static const struct { uint16_t qe; uint8_t nmps, nlps, sw; } MQT[47] = {
  {0x5601, 1, 1, 1},   {0x3401, 2, 6, 0},   {0x1801, 3, 9, 0},   {0x0AC1, 4, 12, 0},
  {0x0521, 5, 29, 0},  {0x0221, 38, 33, 0}, {0x5601, 7, 6, 1},   {0x5401, 8, 14, 0},
  {0x4801, 9, 14, 0},  {0x3801, 10, 14, 0}, {0x3001, 11, 17, 0}, {0x2401, 12, 18, 0},
  {0x1C01, 13, 20, 0}, {0x1601, 29, 21, 0}, {0x5601, 15, 14, 1}, {0x5401, 16, 14, 0},
  {0x5101, 17, 15, 0}, {0x4801, 18, 16, 0}, {0x3801, 19, 17, 0}, {0x3401, 20, 18, 0},
  {0x3001, 21, 19, 0}, {0x2801, 22, 19, 0}, {0x2401, 23, 20, 0}, {0x2201, 24, 21, 0},
  {0x1C01, 25, 22, 0}, {0x1801, 26, 23, 0}, {0x1601, 27, 24, 0}, {0x1401, 28, 25, 0},
  {0x1201, 29, 26, 0}, {0x1101, 30, 27, 0}, {0x0AC1, 31, 28, 0}, {0x09C1, 32, 29, 0},
  {0x08A1, 33, 30, 0}, {0x0521, 34, 31, 0}, {0x0441, 35, 32, 0}, {0x02A1, 36, 33, 0},
  {0x0221, 37, 34, 0}, {0x0141, 38, 35, 0}, {0x0111, 39, 36, 0}, {0x0085, 40, 37, 0},
  {0x0049, 41, 38, 0}, {0x0025, 42, 39, 0}, {0x0015, 43, 40, 0}, {0x0009, 44, 41, 0},
  {0x0005, 45, 42, 0}, {0x0001, 45, 43, 0}, {0x5601, 46, 46, 0}};

#define NCTX 19
enum { CX_SC0 = 9, CX_MR0 = 14, CX_RL = 17, CX_UNI = 18 };

/* Tier-1 initial states: all contexts at state 0 / MPS 0, except the
 * all-zero-neighbourhood ZC context (4), run-length (3) and uniform (46). */
static void ctx_init(uint8_t* I, uint8_t* M) {
  for (int i = 0; i < NCTX; i++) { I[i] = 0; M[i] = 0; }
  I[0] = 4; I[CX_RL] = 3; I[CX_UNI] = 46;
}

typedef struct {
  uint32_t C, A;
  int CT;
  long BP;          /* index of the current byte B; -1 = the dummy byte before the output */
  uint8_t* raw;     /* raw[0] is the dummy byte; output byte k lives at raw[k + 1] */
  long cap;         /* capacity of raw (bytes) */
  uint8_t I[NCTX], M[NCTX];
} mqe_t;

static void mqe_put(mqe_t* e, long pos, uint32_t v) {
  if (pos + 1 >= e->cap) {
    long nc = e->cap * 2 + 64;
    e->raw = (uint8_t*)realloc(e->raw, (size_t)nc);
    memset(e->raw + e->cap, 0, (size_t)(nc - e->cap));
    e->cap = nc;
  }
  e->raw[pos + 1] = (uint8_t)v;
}
static uint8_t mqe_get(const mqe_t* e, long pos) { return e->raw[pos + 1]; }

static void mqe_init(mqe_t* e) {
  e->cap = 256;
  e->raw = (uint8_t*)calloc((size_t)e->cap, 1);
  e->A = 0x8000; e->C = 0; e->BP = -1; e->CT = 12;
  ctx_init(e->I, e->M);
}
/* BYTEOUT with bit stuffing after 0xFF and carry propagation into B. */
static void mqe_byteout(mqe_t* e) {
  uint32_t B = mqe_get(e, e->BP);
  if (B == 0xFF) {
    e->BP++; mqe_put(e, e->BP, e->C >> 20); e->C &= 0xFFFFF; e->CT = 7;
  } else if (e->C < 0x8000000) {
    e->BP++; mqe_put(e, e->BP, e->C >> 19); e->C &= 0x7FFFF; e->CT = 8;
  } else {
    B += 1;
    mqe_put(e, e->BP, B);
    if (B == 0xFF) {
      e->C &= 0x7FFFFFF;
      e->BP++; mqe_put(e, e->BP, e->C >> 20); e->C &= 0xFFFFF; e->CT = 7;
    } else {
      e->BP++; mqe_put(e, e->BP, (e->C >> 19) & 0xFF); e->C &= 0x7FFFF; e->CT = 8;
    }
  }
}
static void mqe_renorm(mqe_t* e) {
  do {
    e->A <<= 1; e->C <<= 1; e->CT--;
    if (e->CT == 0) mqe_byteout(e);
  } while ((e->A & 0x8000) == 0);
}
/* Work counters (measurement only; they do not change any result): MQ
 * decisions coded and decoded on the calling thread since the last reset,
 * the code-blocks coded / decoded, and the most decisions in one block. */
static _Thread_local long g_mq_enc, g_mq_dec, g_mq_enc_blocks, g_mq_dec_blocks, g_mq_enc_max, g_mq_dec_max;
EXPORT void ebcc_ref_mq_counts(long* out, int reset) {
  if (out) {
    out[0] = g_mq_enc; out[1] = g_mq_enc_blocks; out[2] = g_mq_enc_max;
    out[3] = g_mq_dec; out[4] = g_mq_dec_blocks; out[5] = g_mq_dec_max;
  }
  if (reset) g_mq_enc = g_mq_dec = g_mq_enc_blocks = g_mq_dec_blocks = g_mq_enc_max = g_mq_dec_max = 0;
}

/* ENCODE: MPS takes the upper sub-interval, LPS the lower one of size Qe,
 * with conditional exchange when the MPS part would be the smaller. */
static void mqe_encode(mqe_t* e, int cx, int d) {
  g_mq_enc++;
  int s = e->I[cx];
  uint32_t qe = MQT[s].qe;
  e->A -= qe;
  if (d == e->M[cx]) {
    if ((e->A & 0x8000) == 0) {
      if (e->A < qe) e->A = qe; else e->C += qe;
      e->I[cx] = MQT[s].nmps;
      mqe_renorm(e);
    } else {
      e->C += qe;
    }
  } else {
    if (e->A < qe) e->C += qe; else e->A = qe;
    if (MQT[s].sw) e->M[cx] ^= 1;
    e->I[cx] = MQT[s].nlps;
    mqe_renorm(e);
  }
}
/* FLUSH on a copy of the coder state: returns the length of the codeword if
 * it were terminated now, and the (up to) 3 bytes at positions BP, BP+1, BP+2
 * that termination writes (position BP may gain a carry). */
static long mqe_flush_copy(const mqe_t* e, uint8_t tail[3], long* bp0) {
  uint8_t tb[4];
  tb[0] = mqe_get(e, e->BP);
  uint32_t C = e->C, A = e->A;
  int CT = e->CT;
  long bp = 0;                     /* index into tb, tb[0] is byte e->BP */
  uint32_t tempc = C + A;
  C |= 0xFFFF;
  if (C >= tempc) C -= 0x8000;
  for (int r = 0; r < 2; r++) {
    C <<= CT;
    uint32_t B = tb[bp];
    if (B == 0xFF) {
      bp++; tb[bp] = (uint8_t)(C >> 20); C &= 0xFFFFF; CT = 7;
    } else if (C < 0x8000000) {
      bp++; tb[bp] = (uint8_t)(C >> 19); C &= 0x7FFFF; CT = 8;
    } else {
      B += 1; tb[bp] = (uint8_t)B;
      if (B == 0xFF) {
        C &= 0x7FFFFFF; bp++; tb[bp] = (uint8_t)(C >> 20); C &= 0xFFFFF; CT = 7;
      } else {
        bp++; tb[bp] = (uint8_t)((C >> 19) & 0xFF); C &= 0x7FFFF; CT = 8;
      }
    }
  }
  tail[0] = tb[0]; tail[1] = tb[1]; tail[2] = tb[2];
  *bp0 = e->BP;
  long len = e->BP + 3;            /* bytes 0 .. BP+2 */
  if (tb[2] == 0xFF) len -= 1;     /* a trailing 0xFF is dropped */
  return len;
}

typedef struct {
  uint32_t C, A;
  int CT;
  long BP;
  const uint8_t* buf;
  long len;
  uint8_t I[NCTX], M[NCTX];
} mqd_t;
static uint32_t mqd_rd(const mqd_t* d, long i) { return (i >= 0 && i < d->len) ? d->buf[i] : 0xFF; }
/* BYTEIN: bytes past the end read as 0xFF; 0xFF followed by > 0x8F is a marker. */
static void mqd_bytein(mqd_t* d) {
  if (mqd_rd(d, d->BP) == 0xFF) {
    if (mqd_rd(d, d->BP + 1) > 0x8F) { d->C += 0xFF00; d->CT = 8; }
    else { d->BP++; d->C += mqd_rd(d, d->BP) << 9; d->CT = 7; }
  } else {
    d->BP++; d->C += mqd_rd(d, d->BP) << 8; d->CT = 8;
  }
}
static void mqd_init(mqd_t* d, const uint8_t* buf, long len) {
  d->buf = buf; d->len = len; d->BP = 0;
  d->C = mqd_rd(d, 0) << 16;
  mqd_bytein(d);
  d->C <<= 7; d->CT -= 7; d->A = 0x8000;
  ctx_init(d->I, d->M);
}
static void mqd_renorm(mqd_t* d) {
  do {
    if (d->CT == 0) mqd_bytein(d);
    d->A <<= 1; d->C <<= 1; d->CT--;
  } while ((d->A & 0x8000) == 0);
}
static int mqd_decode(mqd_t* d, int cx) {
  g_mq_dec++;
  int s = d->I[cx];
  uint32_t qe = MQT[s].qe;
  int D;
  d->A -= qe;
  if ((d->C >> 16) < qe) {                 /* lower sub-interval */
    if (d->A < qe) { D = d->M[cx]; d->I[cx] = MQT[s].nmps; }
    else { D = 1 - d->M[cx]; if (MQT[s].sw) d->M[cx] ^= 1; d->I[cx] = MQT[s].nlps; }
    d->A = qe;
    mqd_renorm(d);
  } else {                                 /* upper sub-interval */
    d->C -= qe << 16;
    if ((d->A & 0x8000) == 0) {
      if (d->A < qe) { D = 1 - d->M[cx]; if (MQT[s].sw) d->M[cx] ^= 1; d->I[cx] = MQT[s].nlps; }
      else { D = d->M[cx]; d->I[cx] = MQT[s].nmps; }
      mqd_renorm(d);
    } else {
      D = d->M[cx];
    }
  }
  return D;
}

/* Stand-alone MQ round trip for tests: symbols (cx[i], bit[i]) with the
 * tier-1 initial states; the codeword is terminated after the last symbol. */
EXPORT long ebcc_ref_mq_encode(const uint8_t* cx, const uint8_t* bits, long n, uint8_t* out, long cap) {
  mqe_t e; mqe_init(&e);
  for (long i = 0; i < n; i++) mqe_encode(&e, cx[i] % NCTX, bits[i] & 1);
  uint8_t tail[3]; long bp0;
  long len = mqe_flush_copy(&e, tail, &bp0);
  if (len > cap) { free(e.raw); return -1; }
  for (long k = 0; k < len; k++) out[k] = (k < bp0) ? mqe_get(&e, k) : tail[k - bp0];
  free(e.raw);
  return len;
}
EXPORT void ebcc_ref_mq_decode(const uint8_t* in, long len, const uint8_t* cx, long n, uint8_t* bits) {
  mqd_t d; mqd_init(&d, in, len);
  for (long i = 0; i < n; i++) bits[i] = (uint8_t)mqd_decode(&d, cx[i] % NCTX);
}

/* ======================================================================== */
/* 4. EBCOT tier-1 block coder (T.800 Annex D), default mode switches.      */
/* ======================================================================== */
/* Zero-coding context from the counts of significant horizontal (h),
 * vertical (v) and diagonal (d) neighbours (T.800 Table D.1). */
EXPORT int ebcc_ref_zc_ctx(int orient, int h, int v, int d) {
  if (orient == ORI_HH) {
    int hv = h + v;
    if (d >= 3) return 8;
    if (d == 2) return hv >= 1 ? 7 : 6;
    if (d == 1) return hv >= 2 ? 5 : (hv == 1 ? 4 : 3);
    return hv >= 2 ? 2 : (hv == 1 ? 1 : 0);
  }
  if (orient == ORI_HL) { int t = h; h = v; v = t; }
  if (h == 2) return 8;
  if (h == 1) return v >= 1 ? 7 : (d >= 1 ? 6 : 5);
  if (v == 2) return 4;
  if (v == 1) return 3;
  return d >= 2 ? 2 : (d == 1 ? 1 : 0);
}
/* Sign-coding context and XOR bit from the clamped horizontal and vertical
 * sign contributions hc, vc in {-1, 0, 1} (T.800 Tables D.2/D.3). */
EXPORT int ebcc_ref_sc_ctx(int hc, int vc, int* xorbit) {
  static const int ctx[3][3] = {{13, 12, 11}, {10, 9, 10}, {11, 12, 13}};   /* [hc+1][vc+1] */
  static const int xr[3][3] = {{1, 1, 1}, {1, 0, 0}, {0, 0, 0}};
  *xorbit = xr[hc + 1][vc + 1];
  return ctx[hc + 1][vc + 1];
}

/* Raw (uncoded) bits of the bypassed passes: written and read MSB-first;
 * reading past the end gives 0. */
typedef struct { uint8_t* buf; long nbits, cap; } rawbits_t;
static void raw_put(rawbits_t* r, int bit) {
  if ((r->nbits >> 3) >= r->cap) {
    long nc = r->cap * 2 + 256;
    r->buf = (uint8_t*)realloc(r->buf, (size_t)nc);
    memset(r->buf + r->cap, 0, (size_t)(nc - r->cap));
    r->cap = nc;
  }
  if (bit) r->buf[r->nbits >> 3] |= (uint8_t)(0x80 >> (r->nbits & 7));
  r->nbits++;
}
typedef struct { const uint8_t* buf; long nbytes, pos; } rawrd_t;
static int raw_get(rawrd_t* r) {
  long by = r->pos >> 3;
  int bit = by < r->nbytes ? (r->buf[by] >> (7 - (r->pos & 7))) & 1 : 0;
  r->pos++;
  return bit;
}

typedef struct {
  int w, h, orient, dec;
  const uint32_t* q;      /* encoder: magnitudes */
  uint8_t *sig, *vis, *ref, *neg;
  uint32_t* m;            /* known magnitude bits */
  int8_t* pk;             /* lowest known bit-plane of a significant sample */
  mqe_t* e;
  mqd_t* d;
  int64_t dd;             /* distortion reduction of the current pass */
  int rawpass;            /* the current pass is bypassed: its decisions are raw bits */
  rawbits_t* rw;          /* encoder: raw bits */
  rawrd_t* rr;            /* decoder: raw bits */
} t1_t;

static int t1_code(t1_t* t, int cx, int bit) {
  if (t->rawpass) {
    if (t->dec) return raw_get(t->rr);
    raw_put(t->rw, bit);
    return bit;
  }
  if (t->dec) return mqd_decode(t->d, cx);
  mqe_encode(t->e, cx, bit);
  return bit;
}
static int t1_sig(const t1_t* t, int y, int x) {
  return (y >= 0 && y < t->h && x >= 0 && x < t->w) ? t->sig[y * t->w + x] : 0;
}
static void t1_counts(const t1_t* t, int y, int x, int* H, int* V, int* D) {
  *H = t1_sig(t, y, x - 1) + t1_sig(t, y, x + 1);
  *V = t1_sig(t, y - 1, x) + t1_sig(t, y + 1, x);
  *D = t1_sig(t, y - 1, x - 1) + t1_sig(t, y - 1, x + 1) + t1_sig(t, y + 1, x - 1) + t1_sig(t, y + 1, x + 1);
}
static int t1_signc(const t1_t* t, int y, int x) {
  if (!t1_sig(t, y, x)) return 0;
  return t->neg[y * t->w + x] ? -1 : 1;
}
/* Squared reconstruction error in units of (step/2)^2 of a magnitude q whose
 * bits at and above plane p are known as m (midpoint reconstruction). */
static int64_t err2(uint32_t q, uint32_t m, int p) {
  int64_t e = 2 * (int64_t)q + 1;
  if (m) e -= 2 * (int64_t)m + ((int64_t)1 << p);
  return e * e;
}
static void t1_code_sign(t1_t* t, int y, int x) {
  int hc = t1_signc(t, y, x - 1) + t1_signc(t, y, x + 1);
  int vc = t1_signc(t, y - 1, x) + t1_signc(t, y + 1, x);
  hc = hc > 1 ? 1 : (hc < -1 ? -1 : hc);
  vc = vc > 1 ? 1 : (vc < -1 ? -1 : vc);
  int xr, cx = ebcc_ref_sc_ctx(hc, vc, &xr);
  if (t->rawpass) xr = 0;                      /* a bypassed pass sends the sign itself */
  int i = y * t->w + x;
  int b = t1_code(t, cx, t->dec ? 0 : (t->neg[i] ^ xr));
  if (t->dec) t->neg[i] = (uint8_t)(b ^ xr);
}
static void t1_become_sig(t1_t* t, int i, int p) {
  t->sig[i] = 1;
  t->pk[i] = (int8_t)p;
  if (t->dec) {
    t->m[i] = 1u << p;
  } else {
    t->m[i] = (t->q[i] >> p) << p;
    t->dd += err2(t->q[i], 0, 0) - err2(t->q[i], t->m[i], p);
  }
}
static int t1_bit(const t1_t* t, int i, int p) { return t->dec ? 0 : (int)((t->q[i] >> p) & 1u); }

/* Significance propagation: insignificant samples with a significant
 * neighbour (state as of the moment they are reached in the scan). */
static void t1_spp(t1_t* t, int p) {
  for (int y0 = 0; y0 < t->h; y0 += 4)
    for (int x = 0; x < t->w; x++)
      for (int y = y0; y < y0 + 4 && y < t->h; y++) {
        int i = y * t->w + x, H, V, D;
        if (t->sig[i]) continue;
        t1_counts(t, y, x, &H, &V, &D);
        if (H + V + D == 0) continue;
        int b = t1_code(t, ebcc_ref_zc_ctx(t->orient, H, V, D), t1_bit(t, i, p));
        t->vis[i] = 1;
        if (b) { t1_code_sign(t, y, x); t1_become_sig(t, i, p); }
      }
}
/* Magnitude refinement: samples significant before this bit-plane. */
static void t1_mrp(t1_t* t, int p) {
  for (int y0 = 0; y0 < t->h; y0 += 4)
    for (int x = 0; x < t->w; x++)
      for (int y = y0; y < y0 + 4 && y < t->h; y++) {
        int i = y * t->w + x, H, V, D;
        if (!t->sig[i] || t->vis[i]) continue;
        t1_counts(t, y, x, &H, &V, &D);
        int cx = t->ref[i] ? CX_MR0 + 2 : (H + V + D == 0 ? CX_MR0 : CX_MR0 + 1);
        int b = t1_code(t, cx, t1_bit(t, i, p));
        if (t->dec) {
          t->m[i] |= (uint32_t)b << p;
        } else {
          int64_t before = err2(t->q[i], t->m[i], t->pk[i]);
          t->m[i] = (t->q[i] >> p) << p;
          t->dd += before - err2(t->q[i], t->m[i], p);
        }
        t->pk[i] = (int8_t)p;
        t->ref[i] = 1;
      }
}
/* Cleanup: every sample not yet significant and not coded in this plane,
 * with run-length coding of full 4-sample stripe columns whose samples all
 * have an all-insignificant neighbourhood. */
static void t1_cp(t1_t* t, int p) {
  for (int y0 = 0; y0 < t->h; y0 += 4)
    for (int x = 0; x < t->w; x++) {
      int y = y0;
      if (y0 + 4 <= t->h) {
        int run = 1;
        for (int k = 0; k < 4 && run; k++) {
          int i = (y0 + k) * t->w + x, H, V, D;
          if (t->sig[i] || t->vis[i]) { run = 0; break; }
          t1_counts(t, y0 + k, x, &H, &V, &D);
          if (H + V + D) run = 0;
        }
        if (run) {
          int r = -1;
          if (!t->dec)
            for (int k = 0; k < 4; k++)
              if (t1_bit(t, (y0 + k) * t->w + x, p)) { r = k; break; }
          int any = t1_code(t, CX_RL, r >= 0);
          if (!any) continue;
          int b1 = t1_code(t, CX_UNI, r >= 0 ? (r >> 1) & 1 : 0);
          int b0 = t1_code(t, CX_UNI, r >= 0 ? r & 1 : 0);
          r = 2 * b1 + b0;
          int i = (y0 + r) * t->w + x;
          t1_code_sign(t, y0 + r, x);
          t1_become_sig(t, i, p);
          y = y0 + r + 1;
        }
      }
      for (; y < y0 + 4 && y < t->h; y++) {
        int i = y * t->w + x, H, V, D;
        if (t->sig[i] || t->vis[i]) continue;
        t1_counts(t, y, x, &H, &V, &D);
        int b = t1_code(t, ebcc_ref_zc_ctx(t->orient, H, V, D), t1_bit(t, i, p));
        if (b) { t1_code_sign(t, y, x); t1_become_sig(t, i, p); }
      }
    }
  memset(t->vis, 0, (size_t)(t->w * t->h));
}

static int bitlen32(uint32_t v) { int n = 0; while (v) { n++; v >>= 1; } return n; }

/* Selective arithmetic-coding bypass (T.800 D.6, the "lazy" mode; a
 * stream option): the significance propagation and magnitude refinement
 * passes after the first ten (bit-planes below the fourth from the top) send
 * their decisions as raw bits, sign bits included; cleanup passes stay
 * arithmetic coded.  One codeword per block still: after k > 10 passes it is
 * u16 (little-endian) the raw byte count, the MQ codeword terminated after
 * the last arithmetic-coded pass <= k, then the raw bits of the bypassed
 * passes <= k (MSB-first, zero padded).  The MQ coder's state runs on across
 * the bypassed passes.  In a stream with the bypass, a pass (any pass, the
 * first ten included) whose MQ part exceeds BYP_MQ_MAX bytes or whose raw
 * part exceeds BYP_RAW_MAX bytes is never kept. */
#define BYP_FIRST 11
#define BYP_MQ_MAX 49000
#define BYP_RAW_MAX 16000
static int t1_raw_pass(int bypass, int k, int ty) { return bypass && k >= BYP_FIRST && ty < 2; }

/* Result of encoding one code-block with all of its coding passes. */
typedef struct {
  int P, npass, bypass;
  int32_t R[3 * QMAX_BITS];        /* R[k]: codeword length terminated after k passes */
  int64_t D[3 * QMAX_BITS];        /* D[k]: cumulative distortion reduction */
  long bp[3 * QMAX_BITS];          /* MQ termination of the last arithmetic-coded pass <= k */
  uint8_t tail[3 * QMAX_BITS][3];
  int32_t Rmq[3 * QMAX_BITS];      /* its length */
  long rawb[3 * QMAX_BITS];        /* raw bits of the passes <= k */
  mqe_t e;
  rawbits_t raw;
} t1enc_t;

/* Pass k (0-based) of a block with P magnitude planes: pass 0 is the cleanup
 * pass of plane P-1; plane p < P-1 has SPP, MRP, CP as passes
 * 3(P-2-p)+1, +2, +3.  Total 3P-2 passes. */
static void t1_encode_block(const uint32_t* q, const uint8_t* neg, int w, int h, int orient, int bypass,
                            t1enc_t* out) {
  int n = w * h;
  uint32_t mx = 0;
  for (int i = 0; i < n; i++) if (q[i] > mx) mx = q[i];
  out->P = bitlen32(mx);
  out->npass = out->P ? 3 * out->P - 2 : 0;
  out->bypass = bypass;
  mqe_init(&out->e);
  out->R[0] = 0; out->D[0] = 0; out->Rmq[0] = 0; out->rawb[0] = 0; out->bp[0] = -1;
  out->raw.buf = NULL; out->raw.nbits = 0; out->raw.cap = 0;
  if (!out->P) return;
  t1_t t = {0};
  t.w = w; t.h = h; t.orient = orient; t.dec = 0; t.q = q;
  t.sig = (uint8_t*)calloc((size_t)n, 1); t.vis = (uint8_t*)calloc((size_t)n, 1);
  t.ref = (uint8_t*)calloc((size_t)n, 1); t.neg = (uint8_t*)malloc((size_t)n);
  memcpy(t.neg, neg, (size_t)n);
  t.m = (uint32_t*)calloc((size_t)n, 4); t.pk = (int8_t*)calloc((size_t)n, 1);
  t.e = &out->e;
  t.rw = &out->raw;
  int k = 0;
  const long dec0 = g_mq_enc;
  for (int p = out->P - 1; p >= 0; p--) {
    for (int ty = (p == out->P - 1) ? 2 : 0; ty < 3; ty++) {
      t.dd = 0;
      t.rawpass = t1_raw_pass(bypass, k + 1, ty);
      if (ty == 0) t1_spp(&t, p); else if (ty == 1) t1_mrp(&t, p); else t1_cp(&t, p);
      k++;
      out->D[k] = out->D[k - 1] + t.dd;
      if (t.rawpass) {           /* the MQ part is the last arithmetic-coded pass's */
        out->Rmq[k] = out->Rmq[k - 1]; out->bp[k] = out->bp[k - 1];
        memcpy(out->tail[k], out->tail[k - 1], 3);
      } else {
        out->Rmq[k] = (int32_t)mqe_flush_copy(&out->e, out->tail[k], &out->bp[k]);
      }
      out->rawb[k] = out->raw.nbits;
      const long rby = (out->rawb[k] + 7) >> 3;
      out->R[k] = (bypass && k >= BYP_FIRST) ? (int32_t)(2 + out->Rmq[k] + rby) : out->Rmq[k];
      /* with the bypass, every pass of the block: the MQ part and the raw
       * part share one fixed-size coder buffer */
      if (bypass && (out->Rmq[k] > BYP_MQ_MAX || rby > BYP_RAW_MAX)) out->R[k] = SEG_RMAX + 1;
    }
  }
  g_mq_enc_blocks++;
  if (g_mq_enc - dec0 > g_mq_enc_max) g_mq_enc_max = g_mq_enc - dec0;
  free(t.sig); free(t.vis); free(t.ref); free(t.neg); free(t.m); free(t.pk);
}
/* Codeword terminated after k passes: the bytes emitted before the byte the
 * termination touches, then the termination bytes of pass k. */
static void t1_codeword(const t1enc_t* te, int k, uint8_t* out) {
  if (k == 0) return;
  long R = te->Rmq[k], bp0 = te->bp[k];
  const int byp = te->bypass && k >= BYP_FIRST;
  const long rby = byp ? (te->rawb[k] + 7) >> 3 : 0;
  if (byp) { out[0] = (uint8_t)rby; out[1] = (uint8_t)(rby >> 8); out += 2; }
  for (long j = 0; j < R; j++) out[j] = (j < bp0) ? mqe_get(&te->e, j) : te->tail[k][j - bp0];
  if (byp) {
    for (long j = 0; j < rby; j++) out[R + j] = te->raw.buf[j];
    if (te->rawb[k] & 7) out[R + rby - 1] &= (uint8_t)(0xFF << (8 - (te->rawb[k] & 7)));
  }
}
/* Decode k passes of a codeword: magnitudes m, signs, lowest known plane. */
static int t1_decode_block(const uint8_t* cw, long len, int w, int h, int orient, int P, int k, int bypass,
                           uint32_t* m, uint8_t* neg, int8_t* pk) {
  int n = w * h;
  memset(m, 0, sizeof(uint32_t) * (size_t)n);
  memset(neg, 0, (size_t)n);
  memset(pk, 0, (size_t)n);
  if (P == 0 || k == 0) return REF_OK;
  rawrd_t rr = {NULL, 0, 0};
  if (bypass && k >= BYP_FIRST) {            /* u16 raw bytes, MQ codeword, raw bits */
    if (len < 2) return REF_ECORRUPT;
    long rby = cw[0] | ((long)cw[1] << 8);
    if (2 + rby > len) return REF_ECORRUPT;
    rr.buf = cw + len - rby; rr.nbytes = rby;
    cw += 2; len -= 2 + rby;
  }
  mqd_t d; mqd_init(&d, cw, len);
  t1_t t = {0};
  t.w = w; t.h = h; t.orient = orient; t.dec = 1; t.d = &d; t.rr = &rr;
  t.sig = (uint8_t*)calloc((size_t)n, 1); t.vis = (uint8_t*)calloc((size_t)n, 1);
  t.ref = (uint8_t*)calloc((size_t)n, 1); t.neg = neg; t.m = m; t.pk = pk;
  int done = 0;
  const long dec0 = g_mq_dec;
  for (int p = P - 1; p >= 0 && done < k; p--)
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3 && done < k; ty++) {
      t.rawpass = t1_raw_pass(bypass, done + 1, ty);
      if (ty == 0) t1_spp(&t, p); else if (ty == 1) t1_mrp(&t, p); else t1_cp(&t, p);
      done++;
    }
  g_mq_dec_blocks++;
  if (g_mq_dec - dec0 > g_mq_dec_max) g_mq_dec_max = g_mq_dec - dec0;
  free(t.sig); free(t.vis); free(t.ref);
  return REF_OK;
}

/* Test hooks for one block. */
EXPORT int ebcc_ref_t1_encode(const uint32_t* q, const uint8_t* neg, int w, int h, int orient, int bypass, int keep,
                              int32_t* R, int64_t* D, uint8_t* out, long cap, long* len) {
  t1enc_t* te = (t1enc_t*)calloc(1, sizeof(t1enc_t));
  t1_encode_block(q, neg, w, h, orient, bypass, te);
  for (int k = 0; k <= te->npass; k++) { if (R) R[k] = te->R[k]; if (D) D[k] = te->D[k]; }
  if (keep < 0 || keep > te->npass) keep = te->npass;
  int rc = te->npass;
  *len = te->R[keep];
  if (*len > cap) rc = REF_ENOSPC; else t1_codeword(te, keep, out);
  free(te->e.raw); free(te->raw.buf); free(te);
  return rc;
}
/* Raw bit counts rawb[0 .. npass] of a block encoded with the bypass
 * (test hook); returns npass. */
EXPORT int ebcc_ref_t1_rawbits(const uint32_t* q, const uint8_t* neg, int w, int h, int orient, long* rawb) {
  t1enc_t* te = (t1enc_t*)calloc(1, sizeof(t1enc_t));
  t1_encode_block(q, neg, w, h, orient, 1, te);
  for (int k = 0; k <= te->npass; k++) rawb[k] = te->rawb[k];
  int n = te->npass;
  free(te->e.raw); free(te->raw.buf); free(te);
  return n;
}
EXPORT int ebcc_ref_t1_decode(const uint8_t* cw, long len, int w, int h, int orient, int bypass, int P, int k,
                              uint32_t* m, uint8_t* neg, int8_t* pk) {
  return t1_decode_block(cw, len, w, h, orient, P, k, bypass, m, neg, pk);
}

/* ======================================================================== */
/* 5. PCRD rate allocation (convex hull + global slope order).              */
/* ======================================================================== */
typedef struct { double slope; int b, j; int32_t dR; int hk; } seg_t;
static double hull_slope(int64_t dD, int64_t dR) { return dR <= 0 ? INFINITY : (double)dD / (double)dR; }
/* Upper convex hull of (R_k, D_k), k = 0..n, with strictly decreasing slopes.
 * Points that do not increase D, or whose length exceeds SEG_RMAX, are never
 * hull points.  Returns hull size (hull[0] = 0). */
static int pcrd_hull(const int32_t* R, const int64_t* D, int n, int* hull) {
  int nh = 0;
  hull[nh++] = 0;
  for (int k = 1; k <= n; k++) {
    if (R[k] > SEG_RMAX) continue;
    if (D[k] <= D[hull[nh - 1]]) continue;
    while (nh >= 2) {
      int a = hull[nh - 2], b = hull[nh - 1];
      double sab = hull_slope(D[b] - D[a], (int64_t)R[b] - R[a]);
      double sbk = hull_slope(D[k] - D[b], (int64_t)R[k] - R[b]);
      if (sbk >= sab) nh--; else break;
    }
    hull[nh++] = k;
  }
  return nh;
}
static int seg_cmp(const void* pa, const void* pb) {
  const seg_t* a = (const seg_t*)pa; const seg_t* b = (const seg_t*)pb;
  if (a->slope > b->slope) return -1;
  if (a->slope < b->slope) return 1;
  if (a->b != b->b) return a->b < b->b ? -1 : 1;
  return a->j < b->j ? -1 : (a->j > b->j);
}
/* Segments in order of decreasing slope (ties: lower block, then lower
 * segment first) are accepted while the running length stays within the
 * budget; the first that does not fit ends the allocation.  kb[b] = passes
 * kept in block b.  R and D are [nblk][stride]. */
static long pcrd_af(int nblk, const int* npass, const int32_t* R, const int64_t* D, int stride, long budget,
                    uint8_t* kb, int* allfit) {
  seg_t* segs = (seg_t*)malloc(sizeof(seg_t) * (size_t)(nblk * stride + 1));
  int* hull = (int*)malloc(sizeof(int) * (size_t)(stride + 1));
  long ns = 0;
  for (int b = 0; b < nblk; b++) {
    kb[b] = 0;
    const int32_t* r = R + (long)b * stride; const int64_t* d = D + (long)b * stride;
    int nh = pcrd_hull(r, d, npass[b], hull);
    for (int j = 1; j < nh; j++) {
      seg_t s;
      s.slope = hull_slope(d[hull[j]] - d[hull[j - 1]], (int64_t)r[hull[j]] - r[hull[j - 1]]);
      s.b = b; s.j = j; s.dR = r[hull[j]] - r[hull[j - 1]]; s.hk = hull[j];
      segs[ns++] = s;
    }
  }
  qsort(segs, (size_t)ns, sizeof(seg_t), seg_cmp);
  long used = 0, i = 0;
  for (; i < ns; i++) {
    if (used + segs[i].dR > budget) break;
    used += segs[i].dR;
    kb[segs[i].b] = (uint8_t)segs[i].hk;
  }
  if (allfit) *allfit = (i == ns);
  free(segs); free(hull);
  return used;
}
static long pcrd(int nblk, const int* npass, const int32_t* R, const int64_t* D, int stride, long budget, uint8_t* kb) {
  return pcrd_af(nblk, npass, R, D, stride, budget, kb, NULL);
}
EXPORT long ebcc_ref_pcrd(int nblk, const int* npass, const int32_t* R, const int64_t* D, int stride, long budget, uint8_t* kb) {
  return pcrd(nblk, npass, R, D, stride, budget, kb);
}

/* ======================================================================== */
/* 6. SPIHT over spatial-orientation trees, coded per tile of LL roots.     */
/* ======================================================================== */
typedef struct { int band; long i, j; } node_t;
typedef struct {
  long ny, nx; int L, T;
  int nb; band_t b[3 * MAX_LEVELS + 1];
  long hL, wL, tiles_y, tiles_x;
} sgeom_t;

static void sgeom_init(sgeom_t* g, long ny, long nx, int L, int T) {
  g->ny = ny; g->nx = nx; g->L = L; g->T = T;
  g->nb = make_bands(ny, nx, L, g->b);
  g->hL = g->b[0].h; g->wL = g->b[0].w;
  g->tiles_y = (g->hL + T - 1) / T; g->tiles_x = (g->wL + T - 1) / T;
}
static long node_pos(const sgeom_t* g, node_t n) { return (g->b[n.band].y0 + n.i) * g->nx + g->b[n.band].x0 + n.j; }
/* Offspring of a node.  An LL root has the three co-located coefficients of
 * the coarsest HL, LH, HH bands.  A detail node (i, j) at level l >= 2 has the
 * 2x2 group (2i.., 2j..) of its orientation at level l-1; when the finer band
 * has one more row (column) than twice the coarser one, the last row (column)
 * of parents also takes it, so every coefficient has exactly one parent.
 * Level-1 nodes have none.  Order: rows, then columns, ascending. */
static int offspring(const sgeom_t* g, node_t n, node_t* o) {
  int k = 0;
  if (n.band == 0) {
    if (g->L == 0) return 0;
    for (int c = 1; c <= 3; c++)
      if (n.i < g->b[c].h && n.j < g->b[c].w) o[k++] = (node_t){c, n.i, n.j};
    return k;
  }
  const band_t* pb = &g->b[n.band];
  if (pb->level == 1) return 0;
  int cb = n.band + 3;
  const band_t* ch = &g->b[cb];
  long r1 = 2 * n.i + 2, c1 = 2 * n.j + 2;
  if (n.i == pb->h - 1) r1 = ch->h;
  if (n.j == pb->w - 1) c1 = ch->w;
  for (long r = 2 * n.i; r < r1 && r < ch->h; r++)
    for (long c = 2 * n.j; c < c1 && c < ch->w; c++) o[k++] = (node_t){cb, r, c};
  return k;
}

/* Per-position maxima over a node's descendants (maxD) and over its
 * grand-descendants and below (maxL), computed bottom-up. */
typedef struct { uint32_t *sub, *maxD, *maxL; } smax_t;
static void smax_build(const sgeom_t* g, const uint32_t* q, smax_t* s) {
  long N = g->ny * g->nx;
  s->sub = (uint32_t*)calloc((size_t)N, 4); s->maxD = (uint32_t*)calloc((size_t)N, 4);
  s->maxL = (uint32_t*)calloc((size_t)N, 4);
  node_t o[9];
  for (int bi = g->nb - 1; bi >= 0; bi--) {
    const band_t* b = &g->b[bi];
    for (long i = 0; i < b->h; i++)
      for (long j = 0; j < b->w; j++) {
        node_t n = {bi, i, j};
        long p = node_pos(g, n);
        int k = offspring(g, n, o);
        uint32_t md = 0, ml = 0;
        for (int c = 0; c < k; c++) {
          long pc = node_pos(g, o[c]);
          if (s->sub[pc] > md) md = s->sub[pc];
          if (s->maxD[pc] > ml) ml = s->maxD[pc];
        }
        s->maxD[p] = md; s->maxL[p] = ml;
        s->sub[p] = q[p] > md ? q[p] : md;
      }
  }
}
static void smax_free(smax_t* s) { free(s->sub); free(s->maxD); free(s->maxL); }

/* Number of coefficients in the tree rooted at n (n included). */
static long tree_size(const sgeom_t* g, node_t n) {
  node_t o[9];
  int k = offspring(g, n, o);
  long s = 1;
  for (int c = 0; c < k; c++) s += tree_size(g, o[c]);
  return s;
}

typedef struct { uint8_t* buf; long nbits, cap; } bitw_t;
static void bw_put(bitw_t* w, int bit) {
  if ((w->nbits >> 3) >= w->cap) {
    long nc = w->cap * 2 + 64;
    w->buf = (uint8_t*)realloc(w->buf, (size_t)nc);
    memset(w->buf + w->cap, 0, (size_t)(nc - w->cap));
    w->cap = nc;
  }
  if (bit) w->buf[w->nbits >> 3] |= (uint8_t)(0x80 >> (w->nbits & 7));
  w->nbits++;
}
/* Bit reader; bits at positions >= limit are not part of the stream (a
 * residual cut inside a tile's code), the decoder stops before the first. */
typedef struct { const uint8_t* buf; long nbytes, pos, limit; } bitr_t;
static int br_get(bitr_t* r) {
  long by = r->pos >> 3;
  int bit = (by < r->nbytes) ? (r->buf[by] >> (7 - (r->pos & 7))) & 1 : 0;
  r->pos++;
  return bit;
}

typedef struct { node_t n; uint8_t typeB, alive; } lis_t;
typedef struct { node_t n; uint8_t alive; } lip_t;

/* SPIHT on one tile (Said & Pearlman 1996 list algorithm).  Encoder when
 * dec == 0 (bits from q/neg), decoder otherwise (fills m/neg, and pk, the
 * lowest bit-plane known of each significant coefficient).  Codes the
 * planes n_top .. n_bot; plane_end_bits[n] (if given) receives the bit count
 * after plane n.  The decoder stops at the first bit its reader does not
 * hold (r->limit): a coefficient whose sign is not read stays
 * insignificant, a refinement bit not read leaves its plane unknown. */
static void spiht_tile(const sgeom_t* g, long ty, long tx, int n_top, int n_bot, int dec,
                       const uint32_t* q, const smax_t* sm, bitw_t* w, bitr_t* r,
                       uint32_t* m, uint8_t* neg, int8_t* pk, long* plane_end_bits, long* refine_start_bits,
                       int sort_only_last) {
  long i0 = ty * g->T, j0 = tx * g->T;
  long i1 = i0 + g->T < g->hL ? i0 + g->T : g->hL, j1 = j0 + g->T < g->wL ? j0 + g->T : g->wL;
  /* capacity: every coefficient of the tile's trees */
  long ncoef = 0;
  for (long i = i0; i < i1; i++)
    for (long j = j0; j < j1; j++) ncoef += tree_size(g, (node_t){0, i, j});
  lip_t* lip = (lip_t*)malloc(sizeof(lip_t) * (size_t)ncoef);
  lis_t* lis = (lis_t*)malloc(sizeof(lis_t) * (size_t)ncoef * 2);
  node_t* lsp = (node_t*)malloc(sizeof(node_t) * (size_t)ncoef);
  long nlip = 0, nlis = 0, nlsp = 0;
  node_t o[9], oo[9];
  for (long i = i0; i < i1; i++)
    for (long j = j0; j < j1; j++) {
      node_t n = {0, i, j};
      lip[nlip++] = (lip_t){n, 1};
      if (offspring(g, n, o) > 0) lis[nlis++] = (lis_t){n, 0, 1};
    }
#define EMIT(bitv) (dec ? br_get(r) : (bw_put(w, (bitv)), (bitv)))
#define CUT (dec && r->pos > r->limit)      /* the bit just read lies past the cut */
  for (int pl = n_top; pl >= n_bot; pl--) {
    uint64_t thr = (uint64_t)1 << pl;
    long lsp_prev = nlsp;
    for (long k = 0; k < nlip; k++) {
      if (!lip[k].alive) continue;
      long p = node_pos(g, lip[k].n);
      int s = EMIT(dec ? 0 : (q[p] >= thr));
      if (CUT) goto out;
      if (s) {
        int sg = EMIT(dec ? 0 : neg[p]);
        if (CUT) goto out;
        if (dec) { neg[p] = (uint8_t)sg; m[p] = (uint32_t)thr; pk[p] = (int8_t)pl; }
        lsp[nlsp++] = lip[k].n;
        lip[k].alive = 0;
      }
    }
    for (long k = 0; k < nlis; k++) {
      if (!lis[k].alive) continue;
      node_t n = lis[k].n;
      long p = node_pos(g, n);
      int no = offspring(g, n, o);
      if (!lis[k].typeB) {
        int s = EMIT(dec ? 0 : (sm->maxD[p] >= thr));
        if (CUT) goto out;
        if (!s) continue;
        int hasL = 0;
        for (int c = 0; c < no; c++) {
          long pc = node_pos(g, o[c]);
          int sc = EMIT(dec ? 0 : (q[pc] >= thr));
          if (CUT) goto out;
          if (sc) {
            int sg = EMIT(dec ? 0 : neg[pc]);
            if (CUT) goto out;
            if (dec) { neg[pc] = (uint8_t)sg; m[pc] = (uint32_t)thr; pk[pc] = (int8_t)pl; }
            lsp[nlsp++] = o[c];
          } else {
            lip[nlip++] = (lip_t){o[c], 1};
          }
          if (offspring(g, o[c], oo) > 0) hasL = 1;
        }
        lis[k].alive = 0;
        if (hasL) lis[nlis++] = (lis_t){n, 1, 1};
      } else {
        int s = EMIT(dec ? 0 : (sm->maxL[p] >= thr));
        if (CUT) goto out;
        if (!s) continue;
        for (int c = 0; c < no; c++)
          if (offspring(g, o[c], oo) > 0) lis[nlis++] = (lis_t){o[c], 0, 1};
        lis[k].alive = 0;
      }
    }
    if (refine_start_bits) refine_start_bits[pl] = dec ? r->pos : w->nbits;
    if (pl == n_bot && sort_only_last) break;
    for (long k = 0; k < lsp_prev; k++) {
      long p = node_pos(g, lsp[k]);
      int b = EMIT(dec ? 0 : (int)((q[p] >> pl) & 1u));
      if (CUT) goto out;
      if (dec) { if (b) m[p] |= (uint32_t)thr; pk[p] = (int8_t)pl; }
    }
    if (plane_end_bits) plane_end_bits[pl] = dec ? r->pos : w->nbits;
  }
out:
#undef CUT
#undef EMIT
  free(lip); free(lis); free(lsp);
}

/* Magnitude range of one tile's trees: the highest bit-plane, -1 if empty. */
static int tile_top_plane(const sgeom_t* g, const smax_t* sm, long ty, long tx) {
  long i0 = ty * g->T, j0 = tx * g->T;
  uint32_t mx = 0;
  for (long i = i0; i < i0 + g->T && i < g->hL; i++)
    for (long j = j0; j < j0 + g->T && j < g->wL; j++) {
      long p = node_pos(g, (node_t){0, i, j});
      if (sm->sub[p] > mx) mx = sm->sub[p];
    }
  return bitlen32(mx) - 1;
}

/* Full SPIHT code of every tile (planes n_t .. 0) with the bit position at
 * the end of each plane, so that any plane-end truncation can be cut out. */
typedef struct { long ntiles; int* ntop; bitw_t* w; long (*pend)[32]; long (*rs)[32]; } scode_t;
static void spiht_encode_all(const sgeom_t* g, const uint32_t* q, const uint8_t* neg, scode_t* sc) {
  smax_t sm; smax_build(g, q, &sm);
  sc->ntiles = g->tiles_y * g->tiles_x;
  sc->ntop = (int*)malloc(sizeof(int) * (size_t)sc->ntiles);
  sc->w = (bitw_t*)calloc((size_t)sc->ntiles, sizeof(bitw_t));
  sc->pend = (long(*)[32])calloc((size_t)sc->ntiles, sizeof(long[32]));
  sc->rs = (long(*)[32])calloc((size_t)sc->ntiles, sizeof(long[32]));
  for (long t = 0; t < sc->ntiles; t++) {
    long ty = t / g->tiles_x, tx = t % g->tiles_x;
    sc->ntop[t] = tile_top_plane(g, &sm, ty, tx);
    if (sc->ntop[t] >= 0)
      spiht_tile(g, ty, tx, sc->ntop[t], 0, 0, q, &sm, &sc->w[t], NULL, NULL, (uint8_t*)neg, NULL, sc->pend[t],
                 sc->rs[t], 0);
  }
  smax_free(&sm);
}
static void scode_free(scode_t* sc) {
  for (long t = 0; t < sc->ntiles; t++) free(sc->w[t].buf);
  free(sc->w); free(sc->ntop); free(sc->pend); free(sc->rs);
}
/* Residual section for truncation at the end of plane n_s: tile table
 * (u32: byte length | (n_t + 1) << 26, or 0 for a tile with no plane >= n_s),
 * then the tile payloads (MSB-first bits, zero padded to a byte). */
static long resid_section_size(const scode_t* sc, int n_s) {
  long sz = 4 * sc->ntiles;
  for (long t = 0; t < sc->ntiles; t++)
    if (sc->ntop[t] >= n_s) sz += (sc->pend[t][n_s] + 7) >> 3;
  return sz;
}
static void put_u32(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24); }
static void put_u16(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static uint32_t get_u32(const uint8_t* p) { return p[0] | (p[1] << 8) | (p[2] << 16) | ((uint32_t)p[3] << 24); }
static uint32_t get_u16(const uint8_t* p) { return p[0] | (p[1] << 8); }
static void resid_section_write(const scode_t* sc, int n_s, uint8_t* out) {
  uint8_t* pay = out + 4 * sc->ntiles;
  for (long t = 0; t < sc->ntiles; t++) {
    if (sc->ntop[t] < n_s) { put_u32(out + 4 * t, 0); continue; }
    long bits = sc->pend[t][n_s], by = (bits + 7) >> 3;
    put_u32(out + 4 * t, (uint32_t)by | ((uint32_t)(sc->ntop[t] + 1) << 26));
    memcpy(pay, sc->w[t].buf, (size_t)by);
    if (bits & 7) pay[by - 1] &= (uint8_t)(0xFF << (8 - (bits & 7)));
    pay += by;
  }
}
/* Byte-granular truncation (Algorithm 1's second binary search over a
 * byte position t of one embedded code).  The tiles' codes are read as one
 * embedded sequence ordered like a single SPIHT code: plane by plane, and
 * within a plane the sorting passes of every tile (in tile order), then
 * the refinement passes of every tile.  A prefix that ends inside plane n_s
 * keeps every plane above n_s, and of plane n_s either (kind 0) the sorting
 * passes of the tiles before the cut tile J and the first lJ bits of J's
 * code, or (kind 1) every sorting pass, the refinement passes of the tiles
 * before J and the first lJ bits of J's code.  Each tile's code is then
 * still a prefix of itself.  Section: the tile table and payloads as above,
 * then a trailer u32 J | kind << 31, u32 lJ.
 * Bits of tile t's code through plane n, and before plane n's refinement
 * pass (0 if the tile has no plane >= n). */
static long tile_bits(const scode_t* sc, long t, int n) { return sc->ntop[t] >= n ? sc->pend[t][n] : 0; }
static long tile_sort_bits(const scode_t* sc, long t, int n) { return sc->ntop[t] >= n ? sc->rs[t][n] : 0; }
/* Sequence position t (bits) with lo < t <= hi (lo, hi: bits through plane
 * n_s + 1, through n_s) -> the cut: kind, tile J and its code length lJ. */
static void byte_cut(const scode_t* sc, int n_s, long t, int* kind, long* J, long* lJ) {
  long u = t;
  for (long j = 0; j < sc->ntiles; j++) u -= tile_bits(sc, j, n_s + 1);
  for (int k = 0; k < 2; k++)
    for (long j = 0; j < sc->ntiles; j++) {
      long a = k ? tile_sort_bits(sc, j, n_s) : tile_bits(sc, j, n_s + 1);
      long len = (k ? tile_bits(sc, j, n_s) : tile_sort_bits(sc, j, n_s)) - a;
      if (len > 0 && u <= len) { *kind = k; *J = j; *lJ = a + u; return; }
      u -= len;
    }
  *kind = 1; *J = sc->ntiles - 1; *lJ = tile_bits(sc, sc->ntiles - 1, n_s);   /* not reached for t in range */
}
static long cut_tile_bits(const scode_t* sc, int n_s, int kind, long J, long lJ, long t) {
  if (t == J) return lJ;
  if (kind == 0) return t < J ? tile_sort_bits(sc, t, n_s) : tile_bits(sc, t, n_s + 1);
  return t < J ? tile_bits(sc, t, n_s) : tile_sort_bits(sc, t, n_s);
}
static long resid_section_size_bt(const scode_t* sc, int n_s, int kind, long J, long lJ) {
  long sz = 8 + 4 * sc->ntiles;
  for (long t = 0; t < sc->ntiles; t++) sz += (cut_tile_bits(sc, n_s, kind, J, lJ, t) + 7) >> 3;
  return sz;
}
static void resid_section_write_bt(const scode_t* sc, int n_s, int kind, long J, long lJ, uint8_t* out) {
  uint8_t* pay = out + 4 * sc->ntiles;
  for (long t = 0; t < sc->ntiles; t++) {
    long bits = cut_tile_bits(sc, n_s, kind, J, lJ, t), by = (bits + 7) >> 3;
    if (bits == 0) { put_u32(out + 4 * t, 0); continue; }
    put_u32(out + 4 * t, (uint32_t)by | ((uint32_t)(sc->ntop[t] + 1) << 26));
    memcpy(pay, sc->w[t].buf, (size_t)by);
    if (bits & 7) pay[by - 1] &= (uint8_t)(0xFF << (8 - (bits & 7)));
    pay += by;
  }
  put_u32(pay, (uint32_t)J | ((uint32_t)kind << 31)); put_u32(pay + 4, (uint32_t)lJ);
}
/* Decode a residual section: magnitudes m (known bits), signs, and the
 * lowest known plane of each significant coefficient.  bt: the section is
 * cut at a byte position (the two words above lead it). */
static int resid_section_decode(const sgeom_t* g, const uint8_t* in, long len, int n_s, int bt,
                                uint32_t* m, uint8_t* neg, int8_t* pk) {
  long nt = g->tiles_y * g->tiles_x;
  long J = nt, lJ = 0;
  int kind = 1;
  if (bt) {   /* the trailer */
    if (len < 8) return REF_ECORRUPT;
    len -= 8;
    J = get_u32(in + len) & 0x7FFFFFFF; kind = (int)(get_u32(in + len) >> 31); lJ = get_u32(in + len + 4);
    if (J >= nt) return REF_ECORRUPT;
  }
  if (len < 4 * nt) return REF_ECORRUPT;
  long off = 4 * nt;
  for (long t = 0; t < nt; t++) {
    uint32_t e = get_u32(in + 4 * t);
    long by = e & 0x3FFFFFF; int ntop = (int)(e >> 26) - 1;
    if (off + by > len) return REF_ECORRUPT;
    /* kind 0: tiles before J stop after plane n_s's sorting pass, tiles
     * after it at the end of plane n_s + 1; kind 1: tiles after J stop after
     * plane n_s's sorting pass */
    int nb = (kind == 0 && t > J) ? n_s + 1 : n_s;
    int sort_only = (kind == 0 && t < J) || (kind == 1 && t > J);
    if (t == J && (lJ > 8 * by || lJ <= 8 * (by - 1))) return REF_ECORRUPT;
    if (ntop >= nb) {
      bitr_t r = {in + off, by, 0, t == J ? lJ : 8 * by};
      spiht_tile(g, t / g->tiles_x, t % g->tiles_x, ntop, nb, 1, NULL, NULL, NULL, &r, m, neg, pk, NULL, NULL,
                 sort_only);
    }
    off += by;
  }
  return off == len ? REF_OK : REF_ECORRUPT;
}

EXPORT long ebcc_ref_spiht_encode(const uint32_t* q, const uint8_t* neg, long ny, long nx, int L, int T, int n_s,
                                  uint8_t* out, long cap) {
  sgeom_t g; sgeom_init(&g, ny, nx, L, T);
  scode_t sc; spiht_encode_all(&g, q, neg, &sc);
  long sz = resid_section_size(&sc, n_s);
  if (sz <= cap) resid_section_write(&sc, n_s, out);
  scode_free(&sc);
  return sz <= cap ? sz : -sz;
}
EXPORT int ebcc_ref_spiht_decode(const uint8_t* in, long len, long ny, long nx, int L, int T, int n_s,
                                 uint32_t* m, uint8_t* neg) {
  sgeom_t g; sgeom_init(&g, ny, nx, L, T);
  memset(m, 0, sizeof(uint32_t) * (size_t)(ny * nx));
  memset(neg, 0, (size_t)(ny * nx));
  int8_t* pk = (int8_t*)calloc((size_t)(ny * nx), 1);
  int rc = resid_section_decode(&g, in, len, n_s, 0, m, neg, pk);
  free(pk);
  return rc;
}
/* Test hooks of the byte-granular cut: the residual section of q/neg cut at
 * embedded position t (bits within plane n_s), and one tile's code decoded
 * from its first `limit` bits (magnitudes, signs, lowest known planes). */
EXPORT long ebcc_ref_spiht_encode_cut(const uint32_t* q, const uint8_t* neg, long ny, long nx, int L, int T, int n_s,
                                      long t, uint8_t* out, long cap, long* span) {
  sgeom_t g; sgeom_init(&g, ny, nx, L, T);
  scode_t sc; spiht_encode_all(&g, q, neg, &sc);
  long lo = 0, hi = 0;
  for (long j = 0; j < sc.ntiles; j++) { lo += tile_bits(&sc, j, n_s + 1); hi += tile_bits(&sc, j, n_s); }
  if (span) { span[0] = lo; span[1] = hi; }
  long sz = -1;
  if (t > lo && t <= hi) {
    int kind; long J, lJ; byte_cut(&sc, n_s, t, &kind, &J, &lJ);
    sz = resid_section_size_bt(&sc, n_s, kind, J, lJ);
    if (sz <= cap) resid_section_write_bt(&sc, n_s, kind, J, lJ, out); else sz = -sz;
  }
  scode_free(&sc);
  return sz;
}
EXPORT int ebcc_ref_spiht_decode_cut(const uint8_t* in, long len, long ny, long nx, int L, int T, int n_s,
                                     uint32_t* m, uint8_t* neg, int8_t* pk) {
  sgeom_t g; sgeom_init(&g, ny, nx, L, T);
  memset(m, 0, sizeof(uint32_t) * (size_t)(ny * nx));
  memset(neg, 0, (size_t)(ny * nx));
  memset(pk, 0, (size_t)(ny * nx));
  return resid_section_decode(&g, in, len, n_s, 1, m, neg, pk);
}

/* ======================================================================== */
/* 7. The two-layer compressor (Algorithm 1 with a fixed base ratio).       */
/* ======================================================================== */
static uint32_t stream_checksum(const uint8_t* p, long n) {
  uint32_t s = 0;
  for (long k = 0; 4 * k < n; k++) {
    uint32_t w = 0;
    for (int b = 0; b < 4; b++) if (4 * k + b < n) w |= (uint32_t)p[4 * k + b] << (8 * b);
    s += w * (uint32_t)(2 * k + 1);
  }
  return s;
}
static void write_header(uint8_t* o, int mode, int L, int cbl, long ny, long nx, float xmin, float range_f,
                         float inv_f, int e0, int er, int nmax, int ns, int T, uint32_t bb, uint32_t rb) {
  memset(o, 0, HDR_BYTES);
  o[0] = 'E'; o[1] = 'B'; o[2] = 'C'; o[3] = 'C';
  o[4] = 1; o[5] = (uint8_t)mode; o[6] = (uint8_t)L; o[7] = (uint8_t)cbl;
  put_u32(o + 8, (uint32_t)ny); put_u32(o + 12, (uint32_t)nx);
  memcpy(o + 16, &xmin, 4); memcpy(o + 20, &range_f, 4); memcpy(o + 24, &inv_f, 4);
  o[28] = (uint8_t)(int8_t)e0; o[29] = (uint8_t)(int8_t)er; o[30] = (uint8_t)(int8_t)nmax; o[31] = (uint8_t)(int8_t)ns;
  put_u16(o + 32, (uint32_t)T);
  put_u32(o + 36, bb); put_u32(o + 40, rb);
}

/* Quantised coefficient of a float y at scale 2^sh: floor(|y| * 2^sh) capped
 * to QMAX; the scaling by a power of two is exact in FP32. */
static uint32_t quant(float y, int sh, int qbits) {
  float v = ldexpf(fabsf(y), sh);
  float lim = ldexpf(1.0f, qbits);
  if (!(v < lim)) return (1u << qbits) - 1u;
  return (uint32_t)v;
}
/* Midpoint reconstruction: sign * (2m + 2^p) * 2^(e - 1), exact in FP32. */
static float dequant(uint32_t m, int p, int neg, int e) {
  if (!m) return 0.0f;
  float v = ldexpf((float)(2u * m + (1u << p)), e - 1);
  return neg ? -v : v;
}

/* Code-block list of the base layer. */
typedef struct { int band; long y0, x0; int w, h; } blk_t;
static long make_blocks(const band_t* bands, int nb, int cbw, int cbh, blk_t* out) {
  long n = 0;
  for (int bi = 0; bi < nb; bi++) {
    const band_t* b = &bands[bi];
    for (long by = 0; by < b->h; by += cbh)
      for (long bx = 0; bx < b->w; bx += cbw) {
        if (out) {
          out[n].band = bi; out[n].y0 = b->y0 + by; out[n].x0 = b->x0 + bx;
          out[n].h = (int)(b->h - by < cbh ? b->h - by : cbh);
          out[n].w = (int)(b->w - bx < cbw ? b->w - bx : cbw);
        }
        n++;
      }
  }
  return n;
}

/* Optional views of intermediate results (for stage-by-stage comparison). */
typedef struct {
  float* coef;        /* N: forward DWT of the normalised field */
  float* abase;       /* N: base-layer reconstruction (normalised domain) */
  float* cres;        /* N: forward DWT of the residual */
  uint8_t* kb;        /* nblocks: passes kept per block */
  uint8_t* pb;        /* nblocks: magnitude planes per block */
  int32_t* info;      /* [0]=mode [1]=L [2]=e0 [3]=e_r [4]=n_max [5]=n_s [6]=nblocks [7]=ntiles
                         [8]=base_bytes [9]=resid_bytes [10]=feasibility checks */
} ebcc_ref_trace;

typedef struct {
  long ny, nx; int L, cbw, cbh, T;
  band_t bands[3 * MAX_LEVELS + 1]; int nb;
  blk_t* blk; long nblk;
} layout_t;
static int band_gain(const band_t* b) { return ebcc_ref_band_log2_gain(b->level, b->orient); }

/* Base-layer reconstruction from the block table and codewords:
 * dec_base of Algorithm 1 (tier-1 decode, dequantise, inverse DWT). */
static int base_decode(const layout_t* ly, int e0, int bypass, const uint8_t* pbv, const uint8_t* kbv,
                       const uint8_t* const* cw, const long* cwlen, float* out) {
  int rc = REF_OK;
  long N = ly->ny * ly->nx;
  memset(out, 0, sizeof(float) * (size_t)N);
  uint32_t* m = (uint32_t*)malloc(4 * 4096); uint8_t* ng = (uint8_t*)malloc(4096); int8_t* pk = (int8_t*)malloc(4096);
  for (long b = 0; b < ly->nblk; b++) {
    const blk_t* k = &ly->blk[b];
    const band_t* bd = &ly->bands[k->band];
    if (t1_decode_block(cw[b], cwlen[b], k->w, k->h, bd->orient, pbv[b], kbv[b], bypass, m, ng, pk) != REF_OK)
      rc = REF_ECORRUPT;
    int e = e0 - band_gain(bd);
    for (int y = 0; y < k->h; y++)
      for (int x = 0; x < k->w; x++) {
        int i = y * k->w + x;
        out[(k->y0 + y) * ly->nx + k->x0 + x] = dequant(m[i], pk[i], ng[i], e);
      }
  }
  free(m); free(ng); free(pk);
  dwt2_f(out, ly->ny, ly->nx, ly->L, 1);
  return rc;
}

/* Residual reconstruction of a residual section at truncation plane n_s
 * (bt: cut at a byte position inside plane n_s): midpoint of each
 * coefficient's remaining interval, below its lowest known plane. */
static int resid_decode(const layout_t* ly, const uint8_t* sec, long len, int er, int ns, int bt, float* out) {
  long N = ly->ny * ly->nx;
  sgeom_t g; sgeom_init(&g, ly->ny, ly->nx, ly->L, ly->T);
  uint32_t* m = (uint32_t*)calloc((size_t)N, 4); uint8_t* ng = (uint8_t*)calloc((size_t)N, 1);
  int8_t* pk = (int8_t*)calloc((size_t)N, 1);
  int rc = resid_section_decode(&g, sec, len, ns, bt, m, ng, pk);
  for (long i = 0; i < N; i++) out[i] = dequant(m[i], pk[i], ng[i], er);
  free(m); free(ng); free(pk);
  dwt2_f(out, ly->ny, ly->nx, ly->L, 1);
  return rc;
}

/* x_hat = xmin + ((a_base + r + 0.5) * range), each an FP32 operation, and
 * the check |x - x_hat| <= eps in FP64 at every point. */
static float denorm(float abase, float r, float xmin, float range_f) {
  float a = abase + r;
  a = a + 0.5f;
  a = a * range_f;
  return xmin + a;
}
static int within_bound(const float* x, const float* abase, const float* r, long N, float xmin, float range_f, double eps) {
  for (long i = 0; i < N; i++) {
    float xh = denorm(abase[i], r ? r[i] : 0.0f, xmin, range_f);
    if (fabs((double)x[i] - (double)xh) > eps) return 0;
  }
  return 1;
}

static int layout_init(layout_t* ly, long ny, long nx, int L, int cbl2w, int cbl2h, int T) {
  ly->ny = ny; ly->nx = nx; ly->L = levels_eff(ny, nx, L);
  ly->cbw = 1 << cbl2w; ly->cbh = 1 << cbl2h; ly->T = T;
  ly->nb = make_bands(ny, nx, ly->L, ly->bands);
  ly->nblk = make_blocks(ly->bands, ly->nb, ly->cbw, ly->cbh, NULL);
  ly->blk = (blk_t*)malloc(sizeof(blk_t) * (size_t)ly->nblk);
  make_blocks(ly->bands, ly->nb, ly->cbw, ly->cbh, ly->blk);
  return REF_OK;
}

EXPORT size_t ebcc_ref_compress_bound(size_t ny, size_t nx) { return HDR_BYTES + 4 * ny * nx; }

/* ---------------------------------------------------------------------- */
/* enc_base at a ratio r, and Algorithm 1's feedback search over r.        */
/* ---------------------------------------------------------------------- */
typedef struct {
  const layout_t* ly;
  const int* np; const int32_t* R; const int64_t* D; int stride;
  t1enc_t* tes;                    /* every block's encoding with all of its passes */
  const uint8_t* pbv; int e0, bypass;
  const float* x; float xmin, range_f; double eps; long N;
  uint8_t* kb; uint8_t** cw; long* cwlen; float* abase;
  int evals;
} basectx_t;

/* Optional log of every enc_base evaluation (test hook): ratio, q_A (NaN
 * when not computed), whether every segment fitted, budget. */
static double* g_log_r; static double* g_log_q; static int* g_log_af; static long* g_log_bud;
static int g_log_cap, g_log_n;
EXPORT int ebcc_ref_alg1_log(double* r, double* q, int* af, long* bud, int cap) {
  int n = g_log_n;
  g_log_r = r; g_log_q = q; g_log_af = af; g_log_bud = bud; g_log_cap = r ? cap : 0; g_log_n = 0;
  return n;
}

/* Base payload budget for ratio r: header + block table + codewords fit
 * floor(4 N / r) bytes. */
static long base_budget(long N, long nblk, double r) {
  long t = (long)floor((double)(4 * N) / r) - HDR_BYTES - 4 * nblk;
  return t < 0 ? 0 : t;
}

/* enc_base(A, r) followed by dec_base: PCRD at r, the terminated codewords,
 * the decoded base (normalised domain) in c->abase.  Returns the payload. */
static long base_at(basectx_t* c, double r, int* allfit, long* budget) {
  long nblk = c->ly->nblk;
  long bud = base_budget(c->N, nblk, r);
  if (budget) *budget = bud;
  long used = pcrd_af((int)nblk, c->np, c->R, c->D, c->stride, bud, c->kb, allfit);
  for (long b = 0; b < nblk; b++) {
    free(c->cw[b]);
    c->cwlen[b] = c->kb[b] ? c->R[b * c->stride + c->kb[b]] : 0;
    c->cw[b] = (uint8_t*)malloc((size_t)c->cwlen[b] + 1);
    t1_codeword(&c->tes[b], c->kb[b], c->cw[b]);
  }
  base_decode(c->ly, c->e0, c->bypass, c->pbv, c->kb, (const uint8_t* const*)c->cw, c->cwlen, c->abase);
  c->evals++;
  if (g_log_n < g_log_cap) {
    int allfit_v = 0;
    if (allfit) allfit_v = *allfit;
    g_log_r[g_log_n] = r; g_log_q[g_log_n] = NAN; g_log_af[g_log_n] = allfit_v; g_log_bud[g_log_n] = bud;
  }
  g_log_n++;
  return used;
}

/* q_A: the proportion of samples whose base-layer error does not exceed
 * eps (Algorithm 1, enc_base). */
static double base_quality(const basectx_t* c) {
  long n = 0;
  for (long i = 0; i < c->N; i++) {
    float xh = denorm(c->abase[i], 0.0f, c->xmin, c->range_f);
    if (fabs((double)c->x[i] - (double)xh) <= c->eps) n++;
  }
  double qa = (double)n / (double)c->N;
  if (g_log_n >= 1 && g_log_n - 1 < g_log_cap) g_log_q[g_log_n - 1] = qa;
  return qa;
}

/* Algorithm 1's choice of the base ratio for proportion q, starting from r0:
 * halve r while q_A < q, else double it while q_A > q, then bisect until the
 * bracket is narrower than 1e-3 and keep the largest ratio seen with
 * q_A >= q.  Two guards the algorithm leaves open: halving stops once every
 * codable pass is kept (a smaller ratio cannot change the base), doubling
 * stops once the budget is zero.  Returns the ratio; *q_out = its q_A. */
static double alg1_ratio(basectx_t* c, double q, double r0, double* q_out) {
  int allfit; long bud;
  base_at(c, r0, &allfit, &bud);
  double qa0 = base_quality(c), qa = qa0, q_f = qa0;
  double r_low = r0, r_high = r0, r_f = r0;
  int guard = allfit;
  while (qa < q && !guard) {
    r_low = r_low / 2.0;
    base_at(c, r_low, &allfit, &bud);
    qa = base_quality(c);
    r_f = r_low; q_f = qa;
    guard = allfit;
  }
  qa = qa0;
  long bud0 = base_budget(c->N, c->ly->nblk, r0);
  int zero = bud0 == 0;
  while (qa > q && !zero) {
    r_high = r_high * 2.0;
    base_at(c, r_high, &allfit, &bud);
    qa = base_quality(c);
    zero = bud == 0;
  }
  while (r_high - r_low > 1e-3) {
    double r_mid = (r_low + r_high) / 2.0;
    base_at(c, r_mid, &allfit, &bud);
    qa = base_quality(c);
    if (qa < q) r_high = r_mid;
    else { r_low = r_mid; r_f = r_mid; q_f = qa; }
  }
  if (q_out) *q_out = q_f;
  return r_f;
}

EXPORT long ebcc_ref_base_budget(long N, long nblk, double r) { return base_budget(N, nblk, r); }

/* Compress a 2-D float32 field.
 *   bound_mode 0: err_bound is range-relative (eps = err_bound * (max - min));
 *   bound_mode 1: err_bound is absolute.
 *   base_ratio r >= 1: the base section (block table + codewords) plus the
 *   header fits floor(4 N / r) bytes.
 * Returns 0 and the stream length, or a negative status. */
EXPORT int ebcc_ref_compress_trace(const float* x, size_t ny_, size_t nx_, double err_bound, int bound_mode,
                                   double base_ratio, double q, int levels, int cbl2w, int cbl2h, int tile,
                                   int trunc, int bypass, uint8_t* out, size_t cap, size_t* out_len,
                                   ebcc_ref_trace* tr) {
  long ny = (long)ny_, nx = (long)nx_;
  if (out_len) *out_len = 0;
  if (ny < 1 || nx < 1 || ny > (1L << 24) || nx > (1L << 24) || ny * nx > (1L << 31) - 1) return REF_EINVAL;
  if (!(err_bound > 0) || !isfinite(err_bound) || !(base_ratio >= 1.0) || !isfinite(base_ratio)) return REF_EINVAL;
  if (!(q >= 0.0 && q <= 1.0)) return REF_EINVAL;
  if (levels < 0 || levels > MAX_LEVELS || cbl2w < 2 || cbl2h < 2 || cbl2w > 6 || cbl2h > 6 || tile < 1 || tile > 64 ||
      trunc < 0 || trunc > 1 || bypass < 0 || bypass > 1)
    return REF_EINVAL;
  long N = ny * nx;
  float xmin = x[0], xmax = x[0];
  for (long i = 0; i < N; i++) {
    if (!isfinite(x[i])) return REF_EINVAL;
    if (x[i] < xmin) xmin = x[i];
    if (x[i] > xmax) xmax = x[i];
  }
  if (xmin == 0.0f) xmin = 0.0f;                          /* +0 for a zero extreme */
  if (xmax == 0.0f) xmax = 0.0f;
  double range_d = (double)xmax - (double)xmin;
  double eps = bound_mode == 0 ? err_bound * range_d : err_bound;
  int cbl = cbl2w | (cbl2h << 4);
  if (tr && tr->info) memset(tr->info, 0, 11 * sizeof(int32_t));
  if (range_d == 0.0) {                                    /* constant field */
    if (cap < HDR_BYTES) { *out_len = HDR_BYTES; return REF_ENOSPC; }
    write_header(out, MODE_CONST, 0, cbl, ny, nx, xmin, 0.0f, 0.0f, 0, 0, -1, 0, tile, 0, 0);
    put_u32(out + 44, stream_checksum(out + HDR_BYTES, 0));
    *out_len = HDR_BYTES;
    if (tr && tr->info) tr->info[0] = MODE_CONST;
    return REF_OK;
  }
  double eps_norm = eps / range_d;
  int ex; frexp(eps_norm, &ex);
  int elog = ex - 1;                                       /* floor(log2 eps_norm) */
  float range_f = (float)range_d, inv_f = (float)(1.0 / range_d);
  layout_t ly; layout_init(&ly, ny, nx, levels, cbl2w, cbl2h, tile);
  int mode = MODE_CODED;
  if (elog < -40) mode = MODE_RAW;

  float* a = (float*)malloc(sizeof(float) * (size_t)N);
  float* coef = (float*)malloc(sizeof(float) * (size_t)N);
  float* abase = (float*)malloc(sizeof(float) * (size_t)N);
  float* cres = (float*)malloc(sizeof(float) * (size_t)N);
  float* rrec = (float*)malloc(sizeof(float) * (size_t)N);
  /* normalise: a = ((x - min) * (1/range)) - 0.5 */
  for (long i = 0; i < N; i++) { float t = x[i] - xmin; t = t * inv_f; a[i] = t - 0.5f; }
  int e0 = elog - 2; if (e0 < -20) e0 = -20; if (e0 > 0) e0 = 0;
  int er_final = 0, nmax_final = -1, ns_final = 0, checks = 0, bt_final = 0;
  uint8_t* pbv = (uint8_t*)calloc((size_t)ly.nblk, 1);
  uint8_t* kbv = (uint8_t*)calloc((size_t)ly.nblk, 1);
  uint8_t** cw = (uint8_t**)calloc((size_t)ly.nblk, sizeof(uint8_t*));
  long* cwlen = (long*)calloc((size_t)ly.nblk, sizeof(long));
  long base_payload = 0, resid_bytes = 0;
  uint8_t* resid = NULL;
  int rc = REF_OK;

  if (mode == MODE_CODED) {
    /* ---- base layer: DWT, quantise, tier-1, PCRD at ratio r ---- */
    memcpy(coef, a, sizeof(float) * (size_t)N);
    dwt2_f(coef, ny, nx, ly.L, 0);
    if (tr && tr->coef) memcpy(tr->coef, coef, sizeof(float) * (size_t)N);
    int stride = 3 * QMAX_BITS;
    int32_t* R = (int32_t*)calloc((size_t)(ly.nblk * stride), 4);
    int64_t* D = (int64_t*)calloc((size_t)(ly.nblk * stride), 8);
    int* np = (int*)calloc((size_t)ly.nblk, sizeof(int));
    t1enc_t* tes = (t1enc_t*)calloc((size_t)ly.nblk, sizeof(t1enc_t));
    uint32_t* qb = (uint32_t*)malloc(4 * 4096); uint8_t* nb = (uint8_t*)malloc(4096);
    for (long b = 0; b < ly.nblk; b++) {
      const blk_t* k = &ly.blk[b];
      const band_t* bd = &ly.bands[k->band];
      int sh = band_gain(bd) - e0;
      for (int y = 0; y < k->h; y++)
        for (int xx = 0; xx < k->w; xx++) {
          float c = coef[(k->y0 + y) * nx + k->x0 + xx];
          qb[y * k->w + xx] = quant(c, sh, QMAX_BITS);
          nb[y * k->w + xx] = (uint8_t)(c < 0.0f);
        }
      t1enc_t* te = &tes[b];
      t1_encode_block(qb, nb, k->w, k->h, bd->orient, bypass, te);
      pbv[b] = (uint8_t)te->P; np[b] = te->npass;
      for (int j = 0; j <= te->npass; j++) { R[b * stride + j] = te->R[j]; D[b * stride + j] = te->D[j]; }
    }
    basectx_t bc = {&ly, np, R, D, stride, tes, pbv, e0, bypass, x, xmin, range_f, eps, N,
                    kbv, cw, cwlen, abase, 0};
    /* base ratio: the given r (q = 0), or Algorithm 1's feedback search for
     * proportion q from r0 = r, plus the base-only search (q = 1) for the
     * final fallback */
    double r_use = base_ratio, r_only = -1.0;
    if (q > 0.0) {
      double qf;
      r_use = alg1_ratio(&bc, q, base_ratio, &qf);
      if (q < 1.0) {
        double q1;
        double r1 = alg1_ratio(&bc, 1.0, base_ratio, &q1);
        if (q1 >= 1.0) r_only = r1;            /* the base alone meets the bound */
      }
    }
    base_payload = base_at(&bc, r_use, NULL, NULL);
    if (tr && tr->kb) memcpy(tr->kb, kbv, (size_t)ly.nblk);
    if (tr && tr->pb) memcpy(tr->pb, pbv, (size_t)ly.nblk);

    /* ---- A_base = dec_base(e_base); residual = A - A_base; W = DWT ---- */
    if (tr && tr->abase) memcpy(tr->abase, abase, sizeof(float) * (size_t)N);
    for (long i = 0; i < N; i++) cres[i] = a[i] - abase[i];
    dwt2_f(cres, ny, nx, ly.L, 0);
    if (tr && tr->cres) memcpy(tr->cres, cres, sizeof(float) * (size_t)N);

    /* ---- truncation search over residual bit-planes ---- */
    checks++;
    if (!within_bound(x, abase, NULL, N, xmin, range_f, eps)) {
      sgeom_t g; sgeom_init(&g, ny, nx, ly.L, tile);
      uint32_t* qr = (uint32_t*)malloc(4 * (size_t)N); uint8_t* ngr = (uint8_t*)malloc((size_t)N);
      for (long i = 0; i < N; i++) ngr[i] = (uint8_t)(cres[i] < 0.0f);
      int found = 0;
      for (int att = 0; att < 5 && !found; att++) {
        int er = elog - 6 - att;
        uint32_t mx = 0;
        for (long i = 0; i < N; i++) { qr[i] = quant(cres[i], -er, QMAX_BITS); if (qr[i] > mx) mx = qr[i]; }
        int nmax = bitlen32(mx) - 1;
        if (nmax < 0) continue;
        scode_t sc; spiht_encode_all(&g, qr, ngr, &sc);
        /* feasible(k): residual truncated after the top k planes decodes to
         * a field within the bound everywhere. */
        int K = nmax + 1;
        #define FEASIBLE(kk, res) do { \
            int ns_ = nmax - (kk) + 1; long sz_ = resid_section_size(&sc, ns_); \
            uint8_t* sec_ = (uint8_t*)malloc((size_t)sz_ + 1); resid_section_write(&sc, ns_, sec_); \
            resid_decode(&ly, sec_, sz_, er, ns_, 0, rrec); free(sec_); checks++; \
            res = within_bound(x, abase, rrec, N, xmin, range_f, eps); } while (0)
        int okK; FEASIBLE(K, okK);
        if (okK) {
          int lo = 0, hi = K;
          while (hi - lo > 1) {
            int mid = (lo + hi) >> 1, okm;
            FEASIBLE(mid, okm);
            if (okm) hi = mid; else lo = mid;
          }
          #undef FEASIBLE
          found = 1;
          er_final = er; nmax_final = nmax; ns_final = nmax - hi + 1;
          if (!trunc) {
            resid_bytes = resid_section_size(&sc, ns_final);
            resid = (uint8_t*)malloc((size_t)resid_bytes + 1);
            resid_section_write(&sc, ns_final, resid);
          } else {
            /* Algorithm 1's second binary search at byte granularity, over
             * the embedded sequence from the end of plane n_s + 1 (known to
             * miss the bound) to the end of plane n_s (known to meet it):
             * t = 8 b bits, b integer; the end of plane n_s when 8 b passes it. */
            long vlo = 0, vhi = 0;
            for (long j = 0; j < sc.ntiles; j++) { vlo += tile_bits(&sc, j, ns_final + 1); vhi += tile_bits(&sc, j, ns_final); }
            long blo = vlo / 8, bhi = (vhi + 7) / 8;
            #define CUTAT(b) (8 * (b) < vhi ? 8 * (b) : vhi)
            while (bhi - blo > 1) {
              long bm = (blo + bhi) / 2, J, lJ;
              int kind;
              byte_cut(&sc, ns_final, CUTAT(bm), &kind, &J, &lJ);
              long sz = resid_section_size_bt(&sc, ns_final, kind, J, lJ);
              uint8_t* sec = (uint8_t*)malloc((size_t)sz + 1);
              resid_section_write_bt(&sc, ns_final, kind, J, lJ, sec);
              resid_decode(&ly, sec, sz, er, ns_final, 1, rrec);
              free(sec);
              checks++;
              if (within_bound(x, abase, rrec, N, xmin, range_f, eps)) bhi = bm; else blo = bm;
            }
            long J, lJ;
            int kind;
            byte_cut(&sc, ns_final, CUTAT(bhi), &kind, &J, &lJ);
            #undef CUTAT
            resid_bytes = resid_section_size_bt(&sc, ns_final, kind, J, lJ);
            resid = (uint8_t*)malloc((size_t)resid_bytes + 1);
            resid_section_write_bt(&sc, ns_final, kind, J, lJ, resid);
            bt_final = 1;
          }
        }
        scode_free(&sc);
      }
      free(qr); free(ngr);
      if (!found) mode = MODE_RAW;
    }
    /* fallback (end of Algorithm 1): the base alone at its own ratio when
     * that stream is smaller */
    if (r_only >= 0.0) {
      uint8_t* kb1 = (uint8_t*)calloc((size_t)ly.nblk, 1);
      long pay1 = pcrd((int)ly.nblk, np, R, D, stride, base_budget(N, ly.nblk, r_only), kb1);
      free(kb1);
      long ebcc_total = (mode == MODE_CODED) ? base_payload + resid_bytes : 4 * N;
      if (pay1 < ebcc_total) {
        base_payload = base_at(&bc, r_only, NULL, NULL);
        mode = MODE_CODED;
        er_final = 0; nmax_final = -1; ns_final = 0; resid_bytes = 0; bt_final = 0;
        free(resid); resid = NULL;
        if (tr && tr->kb) memcpy(tr->kb, kbv, (size_t)ly.nblk);
        if (tr && tr->abase) memcpy(tr->abase, abase, sizeof(float) * (size_t)N);
      }
    }
    for (long b = 0; b < ly.nblk; b++) { free(tes[b].e.raw); free(tes[b].raw.buf); }
    free(tes); free(qb); free(nb); free(R); free(D); free(np);
  }

  size_t total;
  /* a coded stream never exceeds the raw stream: fall back to raw */
  if (mode == MODE_CODED && 4 * (size_t)ly.nblk + (size_t)base_payload + (size_t)resid_bytes > 4 * (size_t)N)
    mode = MODE_RAW;
  if (mode == MODE_RAW) total = HDR_BYTES + 4 * (size_t)N;
  else total = HDR_BYTES + 4 * (size_t)ly.nblk + (size_t)base_payload + (size_t)resid_bytes;
  if (total > cap) { if (out_len) *out_len = total; rc = REF_ENOSPC; goto done; }
  if (mode == MODE_RAW) {
    write_header(out, MODE_RAW, 0, cbl, ny, nx, xmin, range_f, inv_f, 0, 0, -1, 0, tile, (uint32_t)(4 * N), 0);
    memcpy(out + HDR_BYTES, x, 4 * (size_t)N);
  } else {
    uint32_t bb = (uint32_t)(4 * ly.nblk + base_payload);
    write_header(out, MODE_CODED, ly.L, cbl, ny, nx, xmin, range_f, inv_f, e0, er_final, nmax_final, ns_final,
                 tile, bb, (uint32_t)resid_bytes);
    if (bt_final) out[34] |= 1;                            /* residual cut at a byte position */
    if (bypass) out[35] |= 1;                              /* tier-1 passes with the arithmetic-coding bypass */
    uint8_t* p = out + HDR_BYTES;
    for (long b = 0; b < ly.nblk; b++) {
      p[4 * b] = pbv[b]; p[4 * b + 1] = kbv[b]; put_u16(p + 4 * b + 2, (uint32_t)cwlen[b]);
    }
    p += 4 * ly.nblk;
    for (long b = 0; b < ly.nblk; b++) { memcpy(p, cw[b], (size_t)cwlen[b]); p += cwlen[b]; }
    if (resid_bytes) memcpy(p, resid, (size_t)resid_bytes);
  }
  put_u32(out + 44, stream_checksum(out + HDR_BYTES, (long)(total - HDR_BYTES)));
  *out_len = total;
  if (tr && tr->info) {
    int32_t* f = tr->info;
    f[0] = mode; f[1] = ly.L; f[2] = e0; f[3] = er_final; f[4] = nmax_final; f[5] = ns_final;
    sgeom_t g; sgeom_init(&g, ny, nx, ly.L, tile);
    f[6] = (int32_t)ly.nblk; f[7] = (int32_t)(g.tiles_y * g.tiles_x);
    f[8] = mode == MODE_CODED ? (int32_t)(4 * ly.nblk + base_payload) : 0;
    f[9] = (int32_t)resid_bytes; f[10] = checks;
  }
done:
  for (long b = 0; b < ly.nblk; b++) free(cw[b]);
  free(cw); free(cwlen); free(pbv); free(kbv); free(resid);
  free(a); free(coef); free(abase); free(cres); free(rrec); free(ly.blk);
  return rc;
}

EXPORT int ebcc_ref_compress(const float* x, size_t ny, size_t nx, double err_bound, int bound_mode,
                             double base_ratio, double q, int levels, int cbl2w, int cbl2h, int tile, int trunc,
                             int bypass, uint8_t* out, size_t cap, size_t* out_len) {
  return ebcc_ref_compress_trace(x, ny, nx, err_bound, bound_mode, base_ratio, q, levels, cbl2w, cbl2h, tile,
                                 trunc, bypass, out, cap, out_len, NULL);
}

/* Header fields of a stream (no payload validation). */
EXPORT int ebcc_ref_stream_info(const uint8_t* in, size_t len, size_t* ny, size_t* nx, int* mode) {
  if (len < HDR_BYTES || memcmp(in, "EBCC", 4) != 0 || in[4] != 1 || in[5] > MODE_CODED) return REF_ECORRUPT;
  *ny = get_u32(in + 8); *nx = get_u32(in + 12); *mode = in[5];
  return REF_OK;
}

/* Decompress: dec_base, then the residual layer decoded at its truncation
 * plane and inverse transformed, added, and mapped back to the data range. */
EXPORT int ebcc_ref_decompress(const uint8_t* in, size_t len, float* x, size_t ny_, size_t nx_) {
  long ny = (long)ny_, nx = (long)nx_;
  size_t hny, hnx; int mode;
  if (ebcc_ref_stream_info(in, len, &hny, &hnx, &mode) != REF_OK) return REF_ECORRUPT;
  if ((long)hny != ny || (long)hnx != nx || ny < 1 || nx < 1) return REF_EINVAL;
  uint32_t bb = get_u32(in + 36), rb = get_u32(in + 40);
  if ((size_t)HDR_BYTES + bb + rb != len) return REF_ECORRUPT;
  if (get_u32(in + 44) != stream_checksum(in + HDR_BYTES, (long)(len - HDR_BYTES))) return REF_ECORRUPT;
  long N = ny * nx;
  float xmin, range_f;
  memcpy(&xmin, in + 16, 4); memcpy(&range_f, in + 20, 4);
  if (mode == MODE_CONST) { for (long i = 0; i < N; i++) x[i] = xmin; return REF_OK; }
  if (mode == MODE_RAW) { if (bb != 4 * (uint32_t)N) return REF_ECORRUPT; memcpy(x, in + HDR_BYTES, 4 * (size_t)N); return REF_OK; }
  int L = in[6], cbl2w = in[7] & 15, cbl2h = in[7] >> 4, T = (int)get_u16(in + 32);
  int e0 = (int8_t)in[28], er = (int8_t)in[29], ns = (int8_t)in[31], bt = in[34] & 1, bypass = in[35] & 1;
  if (L != levels_eff(ny, nx, L) || cbl2w < 2 || cbl2h < 2 || cbl2w > 6 || cbl2h > 6 || T < 1) return REF_ECORRUPT;
  layout_t ly; layout_init(&ly, ny, nx, L, cbl2w, cbl2h, T);
  int rc = REF_OK;
  const uint8_t* p = in + HDR_BYTES;
  if ((long)bb < 4 * ly.nblk) { free(ly.blk); return REF_ECORRUPT; }
  uint8_t* pbv = (uint8_t*)malloc((size_t)ly.nblk); uint8_t* kbv = (uint8_t*)malloc((size_t)ly.nblk);
  const uint8_t** cw = (const uint8_t**)malloc(sizeof(uint8_t*) * (size_t)ly.nblk);
  long* cwlen = (long*)malloc(sizeof(long) * (size_t)ly.nblk);
  long off = 4 * ly.nblk;
  for (long b = 0; b < ly.nblk; b++) {
    pbv[b] = p[4 * b]; kbv[b] = p[4 * b + 1]; cwlen[b] = get_u16(p + 4 * b + 2);
    if (pbv[b] > QMAX_BITS || kbv[b] > (pbv[b] ? 3 * pbv[b] - 2 : 0)) rc = REF_ECORRUPT;
    cw[b] = p + off; off += cwlen[b];
  }
  if (off != (long)bb) rc = REF_ECORRUPT;
  float* abase = (float*)malloc(sizeof(float) * (size_t)N);
  float* r = (float*)calloc((size_t)N, sizeof(float));
  if (rc == REF_OK) {
    rc = base_decode(&ly, e0, bypass, pbv, kbv, cw, cwlen, abase);
    if (rc == REF_OK && rb) rc = resid_decode(&ly, in + HDR_BYTES + bb, rb, er, ns, bt, r);
  }
  if (rc == REF_OK)
    for (long i = 0; i < N; i++) x[i] = denorm(abase[i], r[i], xmin, range_f);
  free(pbv); free(kbv); free(cw); free(cwlen); free(abase); free(r); free(ly.blk);
  return rc;
}

/* FP32 and FP64 transforms for tests. */
EXPORT int ebcc_ref_levels(long ny, long nx, int L) { return levels_eff(ny, nx, L); }
EXPORT void ebcc_ref_dwt_f32(float* a, long ny, long nx, int L, int inverse) { dwt2_f(a, ny, nx, L, inverse); }
EXPORT void ebcc_ref_dwt_f64(double* a, long ny, long nx, int L, int inverse) { dwt2_d(a, ny, nx, L, inverse); }
EXPORT uint32_t ebcc_ref_checksum(const uint8_t* p, long n) { return stream_checksum(p, n); }
/* Entry i of the MQ probability-estimation table (for its pin against the
 * standard's Table C.2); returns -1 for i outside 0..46. */
EXPORT int ebcc_ref_mq_table(int i, int* qe, int* nmps, int* nlps, int* sw) {
  if (i < 0 || i >= 47) return -1;
  *qe = MQT[i].qe; *nmps = MQT[i].nmps; *nlps = MQT[i].nlps; *sw = MQT[i].sw;
  return 0;
}
/* The base-layer quantiser of one coefficient at scale 2^sh (23-bit cap). */
EXPORT uint32_t ebcc_ref_quant(float y, int sh) { return quant(y, sh, QMAX_BITS); }

