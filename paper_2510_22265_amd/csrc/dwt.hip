// Multi-level 2-D CDF 9/7 lifting DWT (JPEG2000 Part 1 Annex F, irreversible
// filter) in Mallat layout, with the field normalisation fused into the first
// forward pass and the reconstruction / bound check fused into the last
// inverse pass.
//
// Each level transforms the current LL region: all columns (vertical), then
// all rows (horizontal); the inverse undoes rows, then columns.  Every lifting
// update is the FP32 sequence t = l + r; t = c * t; v = v +/- t (compiled
// with contraction off), so any tiling reproduces the sequential transform bit
// for bit.  Tiles carry a 4-sample halo: the four lifting steps each widen
// the dependency cone by one sample.  Whole-sample symmetric extension is
// applied once to the loaded halo (mirrored indices); because each lifting
// step is symmetric under the reflection, this equals per-step mirroring
// exactly, also in FP32.
#include "common.h"

namespace ebcc {

// Nearest binary32 values of the 9/7 lifting factors and of K, 1/K.
#define L97_A (-0x1.960ce6p+0f)
#define L97_B (-0x1.b2035cp-5f)
#define L97_G (0x1.c40cecp-1f)
#define L97_D (0x1.c626aap-2f)
#define L97_K (0x1.3aecb0p+0f)
#define L97_IK (0x1.a03386p-1f)

constexpr int kHalo = 4;
constexpr int kColTileR = 64;   // output rows per column-pass tile
constexpr int kColTileC = 64;   // columns per column-pass tile (one per lane)
constexpr int kRowTileR = 16;   // rows per row-pass tile
constexpr int kRowTileC = 256;  // output columns per row-pass tile

// Whole-sample symmetric extension of index g into [0, n).
__device__ __forceinline__ int mirror(int g, int n) {
  if (n <= 1) return 0;
  int p = 2 * (n - 1);
  g %= p;
  if (g < 0) g += p;
  return g < n ? g : p - g;
}

struct Scal {   // per-field scalars held in registers
  float xmin, inv, range;
  double eps;
};
__device__ __forceinline__ Scal load_scal(const FieldParams* fp) {
  Scal s;
  s.xmin = fp->xmin; s.inv = fp->inv_f; s.range = fp->range_f; s.eps = fp->eps;
  return s;
}

// Prologue: the value of the level-1 input at flat index idx.
template <int PRO>
__device__ __forceinline__ float prologue(const float* __restrict__ src, int idx, const DwtIO& io, const Scal& sc) {
  if (PRO == PRO_COPY) return src[idx];
  float t = src[idx] - sc.xmin;
  t = t * sc.inv;
  t = t - 0.5f;
  if (PRO == PRO_NORM) return t;
  return t - io.abase[idx];
}

// Epilogue: reconstruction x_hat = xmin + ((abase + v + 0.5) * range).
template <int EPI>
__device__ __forceinline__ void epilogue(float* __restrict__ out, int idx, float v, const DwtIO& io, const Scal& sc) {
  if (EPI == EPI_STORE) { out[idx] = v; return; }
  float a = io.abase[idx] + v;
  a = a + 0.5f;
  a = a * sc.range;
  float xh = sc.xmin + a;
  if (EPI == EPI_FINAL) { io.xout[idx] = xh; return; }
  if (fabs((double)io.x[idx] - (double)xh) > sc.eps) atomicOr(io.flag, 1);
}

// One lifting step along the first LDS index (rows) of a column tile.
template <bool SUB>
__device__ __forceinline__ void lift_rows(float (*s)[kColTileC + 1], int nrows, int k, int par, float c, int tx, int ty) {
  int start = k + (((k & 1) != par) ? 1 : 0);
  for (int r = start + 2 * ty; r < nrows - k; r += 8) {
    float l = s[r - 1][tx], rr = s[r + 1][tx];
    float t = l + rr;
    t = c * t;
    s[r][tx] = SUB ? (s[r][tx] - t) : (s[r][tx] + t);
  }
  __syncthreads();
}

// Forward vertical pass on region H x W (stride nx): src -> dst deinterleaved.
template <int PRO>
__global__ __launch_bounds__(256) void k_fwd_cols(const float* __restrict__ src, float* __restrict__ dst,
                                                  int nx, int H, int W, DwtIO io) {
  __shared__ float s[kColTileR + 2 * kHalo][kColTileC + 1];
  const int NR = kColTileR + 2 * kHalo;
  int c0 = blockIdx.x * kColTileC, r0 = blockIdx.y * kColTileR;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int col = c0 + tx;
  Scal sc = {};
  if (PRO != PRO_COPY) sc = load_scal(io.fp);
  for (int r = ty; r < NR; r += 4) {
    int g = mirror(r0 - kHalo + r, H);
    s[r][tx] = (col < W) ? prologue<PRO>(src, g * nx + col, io, sc) : 0.0f;
  }
  __syncthreads();
  lift_rows<false>(s, NR, 1, 1, L97_A, tx, ty);
  lift_rows<false>(s, NR, 2, 0, L97_B, tx, ty);
  lift_rows<false>(s, NR, 3, 1, L97_G, tx, ty);
  lift_rows<false>(s, NR, 4, 0, L97_D, tx, ty);
  int nl = (H + 1) >> 1;
  for (int r = kHalo + ty; r < kColTileR + kHalo; r += 4) {
    int g = r0 - kHalo + r;
    if (g < H && col < W) {
      float v = s[r][tx];
      v = (g & 1) ? v * L97_K : v * L97_IK;
      int orow = (g & 1) ? nl + (g >> 1) : (g >> 1);
      dst[orow * nx + col] = v;
    }
  }
}

// Inverse vertical pass: deinterleaved src -> interleaved dst (via epilogue).
template <int EPI>
__global__ __launch_bounds__(256) void k_inv_cols(const float* __restrict__ src, float* __restrict__ dst,
                                                  int nx, int H, int W, DwtIO io) {
  __shared__ float s[kColTileR + 2 * kHalo][kColTileC + 1];
  const int NR = kColTileR + 2 * kHalo;
  int c0 = blockIdx.x * kColTileC, r0 = blockIdx.y * kColTileR;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int col = c0 + tx;
  int nl = (H + 1) >> 1;
  Scal sc = {};
  if (EPI != EPI_STORE) sc = load_scal(io.fp);
  for (int r = ty; r < NR; r += 4) {
    int g = mirror(r0 - kHalo + r, H);
    float v = 0.0f;
    if (col < W) {
      int srow = (g & 1) ? nl + (g >> 1) : (g >> 1);
      v = src[srow * nx + col];
      v = (g & 1) ? v * L97_IK : v * L97_K;
    }
    s[r][tx] = v;
  }
  __syncthreads();
  lift_rows<true>(s, NR, 1, 0, L97_D, tx, ty);
  lift_rows<true>(s, NR, 2, 1, L97_G, tx, ty);
  lift_rows<true>(s, NR, 3, 0, L97_B, tx, ty);
  lift_rows<true>(s, NR, 4, 1, L97_A, tx, ty);
  for (int r = kHalo + ty; r < kColTileR + kHalo; r += 4) {
    int g = r0 - kHalo + r;
    if (g < H && col < W) epilogue<EPI>(dst, g * nx + col, s[r][tx], io, sc);
  }
}

// One lifting step along the second LDS index (columns) of a row tile.
template <bool SUB>
__device__ __forceinline__ void lift_cols(float (*s)[kRowTileC + 2 * kHalo + 1], int ncols, int k, int par, float c,
                                          int tx, int ty) {
  int start = k + (((k & 1) != par) ? 1 : 0);
  for (int rr = ty; rr < kRowTileR; rr += 4)
    for (int cc = start + 2 * tx; cc < ncols - k; cc += 128) {
      float l = s[rr][cc - 1], r = s[rr][cc + 1];
      float t = l + r;
      t = c * t;
      s[rr][cc] = SUB ? (s[rr][cc] - t) : (s[rr][cc] + t);
    }
  __syncthreads();
}

// Forward horizontal pass on region H x W: src -> dst deinterleaved.
__global__ __launch_bounds__(256) void k_fwd_rows(const float* __restrict__ src, float* __restrict__ dst,
                                                  int nx, int H, int W) {
  __shared__ float s[kRowTileR][kRowTileC + 2 * kHalo + 1];
  const int NC = kRowTileC + 2 * kHalo;
  int c0 = blockIdx.x * kRowTileC, r0 = blockIdx.y * kRowTileR;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = 0; rr < kRowTileR; rr++) {
    int row = r0 + rr;
    for (int cc = threadIdx.x; cc < NC; cc += 256) {
      int g = mirror(c0 - kHalo + cc, W);
      s[rr][cc] = (row < H) ? src[row * nx + g] : 0.0f;
    }
  }
  __syncthreads();
  lift_cols<false>(s, NC, 1, 1, L97_A, tx, ty);
  lift_cols<false>(s, NC, 2, 0, L97_B, tx, ty);
  lift_cols<false>(s, NC, 3, 1, L97_G, tx, ty);
  lift_cols<false>(s, NC, 4, 0, L97_D, tx, ty);
  int nl = (W + 1) >> 1;
  for (int rr = 0; rr < kRowTileR; rr++) {
    int row = r0 + rr;
    if (row >= H) break;
    for (int cc = kHalo + threadIdx.x; cc < kRowTileC + kHalo; cc += 256) {
      int g = c0 - kHalo + cc;
      if (g < W) {
        float v = s[rr][cc];
        v = (g & 1) ? v * L97_K : v * L97_IK;
        int ocol = (g & 1) ? nl + (g >> 1) : (g >> 1);
        dst[row * nx + ocol] = v;
      }
    }
  }
}

// Inverse horizontal pass: deinterleaved src -> interleaved dst.
__global__ __launch_bounds__(256) void k_inv_rows(const float* __restrict__ src, float* __restrict__ dst,
                                                  int nx, int H, int W) {
  __shared__ float s[kRowTileR][kRowTileC + 2 * kHalo + 1];
  const int NC = kRowTileC + 2 * kHalo;
  int c0 = blockIdx.x * kRowTileC, r0 = blockIdx.y * kRowTileR;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int nl = (W + 1) >> 1;
  for (int rr = 0; rr < kRowTileR; rr++) {
    int row = r0 + rr;
    for (int cc = threadIdx.x; cc < NC; cc += 256) {
      int g = mirror(c0 - kHalo + cc, W);
      float v = 0.0f;
      if (row < H) {
        int scol = (g & 1) ? nl + (g >> 1) : (g >> 1);
        v = src[row * nx + scol];
        v = (g & 1) ? v * L97_IK : v * L97_K;
      }
      s[rr][cc] = v;
    }
  }
  __syncthreads();
  lift_cols<true>(s, NC, 1, 0, L97_D, tx, ty);
  lift_cols<true>(s, NC, 2, 1, L97_G, tx, ty);
  lift_cols<true>(s, NC, 3, 0, L97_B, tx, ty);
  lift_cols<true>(s, NC, 4, 1, L97_A, tx, ty);
  for (int rr = 0; rr < kRowTileR; rr++) {
    int row = r0 + rr;
    if (row >= H) break;
    for (int cc = kHalo + threadIdx.x; cc < kRowTileC + kHalo; cc += 256) {
      int g = c0 - kHalo + cc;
      if (g < W) dst[row * nx + g] = s[rr][cc];
    }
  }
}

// Elementwise prologue/epilogue (levels = 0, base-only check, plain copies).
// PRO value 3 means "the residual is zero".
template <int PRO, int EPI>
__global__ __launch_bounds__(256) void k_pointwise(const float* __restrict__ src, float* __restrict__ dst, int n, DwtIO io) {
  Scal sc = load_scal(io.fp);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = (PRO == 3) ? 0.0f : prologue<(PRO == 3 ? 0 : PRO)>(src, i, io, sc);
    epilogue<EPI>(dst, i, v, io, sc);
  }
}

static void sizes(int ny, int nx, int L, int* h, int* w) {
  h[0] = ny; w[0] = nx;
  for (int l = 1; l <= L; l++) { h[l] = (h[l - 1] + 1) / 2; w[l] = (w[l - 1] + 1) / 2; }
}

void dwt_forward(const float* src, float* a, float* tmp, int ny, int nx, int L, int prologue, const DwtIO& io,
                 hipStream_t st) {
  int h[kMaxLevels + 1], w[kMaxLevels + 1];
  sizes(ny, nx, L, h, w);
  if (L == 0) {
    pointwise(src, a, ny * nx, prologue, EPI_STORE, io, st);
    return;
  }
  for (int l = 1; l <= L; l++) {
    int H = h[l - 1], W = w[l - 1];
    dim3 gc((W + kColTileC - 1) / kColTileC, (H + kColTileR - 1) / kColTileR);
    const float* s = (l == 1) ? src : a;
    int pro = (l == 1) ? prologue : PRO_COPY;
    if (pro == PRO_NORM) k_fwd_cols<PRO_NORM><<<gc, 256, 0, st>>>(s, tmp, nx, H, W, io);
    else if (pro == PRO_NORM_MINUS) k_fwd_cols<PRO_NORM_MINUS><<<gc, 256, 0, st>>>(s, tmp, nx, H, W, io);
    else k_fwd_cols<PRO_COPY><<<gc, 256, 0, st>>>(s, tmp, nx, H, W, io);
    dim3 gr((W + kRowTileC - 1) / kRowTileC, (H + kRowTileR - 1) / kRowTileR);
    k_fwd_rows<<<gr, 256, 0, st>>>(tmp, a, nx, H, W);
  }
}

void dwt_inverse(float* a, float* tmp, float* out, int ny, int nx, int L, int epi, const DwtIO& io,
                 hipStream_t st) {
  int h[kMaxLevels + 1], w[kMaxLevels + 1];
  sizes(ny, nx, L, h, w);
  if (L == 0) {
    pointwise(a, out, ny * nx, PRO_COPY, epi, io, st);
    return;
  }
  for (int l = L; l >= 1; l--) {
    int H = h[l - 1], W = w[l - 1];
    dim3 gr((W + kRowTileC - 1) / kRowTileC, (H + kRowTileR - 1) / kRowTileR);
    k_inv_rows<<<gr, 256, 0, st>>>(a, tmp, nx, H, W);
    dim3 gc((W + kColTileC - 1) / kColTileC, (H + kColTileR - 1) / kColTileR);
    int e = (l == 1) ? epi : EPI_STORE;
    float* d = (l == 1) ? out : a;
    if (e == EPI_FINAL) k_inv_cols<EPI_FINAL><<<gc, 256, 0, st>>>(tmp, d, nx, H, W, io);
    else if (e == EPI_CHECK) k_inv_cols<EPI_CHECK><<<gc, 256, 0, st>>>(tmp, d, nx, H, W, io);
    else k_inv_cols<EPI_STORE><<<gc, 256, 0, st>>>(tmp, d, nx, H, W, io);
  }
}

void pointwise(const float* src, float* dst, int n, int pro, int epi, const DwtIO& io, hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
#define PW(P, E) k_pointwise<P, E><<<blocks, 256, 0, st>>>(src, dst, n, io)
  if (pro == 3) {
    if (epi == EPI_FINAL) PW(3, EPI_FINAL); else if (epi == EPI_CHECK) PW(3, EPI_CHECK); else PW(3, EPI_STORE);
  } else if (pro == PRO_NORM) {
    PW(PRO_NORM, EPI_STORE);
  } else if (pro == PRO_NORM_MINUS) {
    PW(PRO_NORM_MINUS, EPI_STORE);
  } else {
    if (epi == EPI_FINAL) PW(PRO_COPY, EPI_FINAL); else if (epi == EPI_CHECK) PW(PRO_COPY, EPI_CHECK); else PW(PRO_COPY, EPI_STORE);
  }
#undef PW
}

}  // namespace ebcc
