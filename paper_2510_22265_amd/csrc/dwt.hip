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

#include <algorithm>

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

// Size of the region level l (1-based) transforms: ceil(n / 2^(l-1)).
__device__ __forceinline__ int lvl_size(int n, int l) {
  for (int i = 1; i < l; i++) n = (n + 1) >> 1;
  return n;
}

// Prologue: the value of the level-1 input at flat index idx.
template <int PRO>
__device__ __forceinline__ float prologue(const float* __restrict__ src, int idx, const FieldDev& f, const Scal& sc) {
  if (PRO == PRO_COPY) return src[idx];
  float t = src[idx] - sc.xmin;
  t = t * sc.inv;
  t = t - 0.5f;
  if (PRO == PRO_NORM) return t;
  return t - f.buf[BUF_ABASE][idx];
}

// Epilogue: reconstruction x_hat = xmin + ((abase + v + 0.5) * range).
// Returns, for a bound check, whether this sample violates the bound; the
// caller gathers the answers of its workgroup (report_violation).
template <int EPI>
__device__ __forceinline__ bool epilogue(float* __restrict__ out, int idx, float v, const FieldDev& f, const Scal& sc) {
  if (EPI == EPI_STORE) { out[idx] = v; return false; }
  float a = f.buf[BUF_ABASE][idx] + v;
  a = a + 0.5f;
  a = a * sc.range;
  float xh = sc.xmin + a;
  if (EPI == EPI_FINAL) { f.buf[BUF_XOUT][idx] = xh; return false; }
  return fabs((double)f.buf[BUF_X][idx] - (double)xh) > sc.eps;
}

// The epilogue with its two loads (base reconstruction and, for a check,
// the original sample) already done by the caller: the same arithmetic.
template <int EPI>
__device__ __forceinline__ bool epilogue_loaded(int idx, float v, float abase, float x, const FieldDev& f,
                                                const Scal& sc) {
  float a = abase + v;
  a = a + 0.5f;
  a = a * sc.range;
  float xh = sc.xmin + a;
  if (EPI == EPI_FINAL) { f.buf[BUF_XOUT][idx] = xh; return false; }
  return fabs((double)x - (double)xh) > sc.eps;
}

// One atomic per workgroup that saw a violation.  Every thread of the
// workgroup calls it.  (Reading the flag first to skip the atomic costs
// more than it saves: thousands of wavefronts reading one word at system
// scope are served one after another.)
__device__ __forceinline__ void report_violation(bool bad, const FieldDev& f) {
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (__ballot(bad) != 0ull && __lane_id() == 0) s_bad = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_bad) atomicOr(&f.flags[0], 1);
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

// Forward vertical pass of level l on every active field (blockIdx.z):
// buf[src] (level 1: through the prologue) -> buf[BUF_TMP], deinterleaved.
template <int PRO>
__global__ __launch_bounds__(256) void k_fwd_cols(const FieldDev* __restrict__ F, int l, int src, int dst) {
  const FieldDev& f = F[blockIdx.z];
  if (!f.active || l > f.L) return;
  const int nx = f.nx, H = lvl_size(f.ny, l), W = lvl_size(f.nx, l);
  int c0 = blockIdx.x * kColTileC, r0 = blockIdx.y * kColTileR;
  if (c0 >= W || r0 >= H) return;
  const float* sp = f.buf[l == 1 ? src : dst];
  float* dp = f.buf[BUF_TMP];
  __shared__ float s[kColTileR + 2 * kHalo][kColTileC + 1];
  const int NR = kColTileR + 2 * kHalo;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int col = c0 + tx;
  Scal sc = {};
  if (PRO != PRO_COPY) sc = load_scal(f.fp);
  // every load of the thread first, then the LDS writes: the loads are
  // independent, and issuing them together hides the memory latency (a
  // generic pointer may alias LDS, so the compiler keeps the order written)
  constexpr int NPT = (kColTileR + 2 * kHalo) / 4;
  const int cl = col < W ? col : W - 1;   // in bounds; the value is dropped
  float v[NPT];
#pragma unroll
  for (int i = 0; i < NPT; i++) v[i] = prologue<PRO>(sp, mirror(r0 - kHalo + ty + 4 * i, H) * nx + cl, f, sc);
#pragma unroll
  for (int i = 0; i < NPT; i++) s[ty + 4 * i][tx] = (col < W) ? v[i] : 0.0f;
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
      dp[orow * nx + col] = v;
    }
  }
}

// Inverse vertical pass of level l: buf[BUF_TMP] (deinterleaved) -> level 1:
// the epilogue into buf[out]; other levels: buf[a].
template <int EPI>
__global__ __launch_bounds__(256) void k_inv_cols(const FieldDev* __restrict__ F, int l, int a, int out) {
  const FieldDev& f = F[blockIdx.z];
  if (!f.active || l > f.L) return;
  // a bound check only answers "is any sample violated": once the flag is
  // set the rest of the pass is moot (the flag only goes from 0 to 1).  One
  // thread reads it so that the whole workgroup takes the same branch.
  if (EPI == EPI_CHECK && l == 1) {
    __shared__ int s_done;
    if (threadIdx.x == 0) s_done = __hip_atomic_load(f.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_done) return;
  }
  const int nx = f.nx, H = lvl_size(f.ny, l), W = lvl_size(f.nx, l);
  int c0 = blockIdx.x * kColTileC, r0 = blockIdx.y * kColTileR;
  if (c0 >= W || r0 >= H) return;
  const float* sp = f.buf[BUF_TMP];
  float* dp = f.buf[l == 1 ? out : a];
  __shared__ float s[kColTileR + 2 * kHalo][kColTileC + 1];
  const int NR = kColTileR + 2 * kHalo;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int col = c0 + tx;
  int nl = (H + 1) >> 1;
  Scal sc = {};
  if (EPI != EPI_STORE) sc = load_scal(f.fp);
  constexpr int NPT = (kColTileR + 2 * kHalo) / 4;
  const int cl = col < W ? col : W - 1;
  float v[NPT];
#pragma unroll
  for (int i = 0; i < NPT; i++) {
    const int g = mirror(r0 - kHalo + ty + 4 * i, H);
    v[i] = sp[((g & 1) ? nl + (g >> 1) : (g >> 1)) * nx + cl];
  }
#pragma unroll
  for (int i = 0; i < NPT; i++) {
    const int g = mirror(r0 - kHalo + ty + 4 * i, H);
    s[ty + 4 * i][tx] = (col < W) ? ((g & 1) ? v[i] * L97_IK : v[i] * L97_K) : 0.0f;
  }
  __syncthreads();
  lift_rows<true>(s, NR, 1, 0, L97_D, tx, ty);
  lift_rows<true>(s, NR, 2, 1, L97_G, tx, ty);
  lift_rows<true>(s, NR, 3, 0, L97_B, tx, ty);
  lift_rows<true>(s, NR, 4, 1, L97_A, tx, ty);
  constexpr int NO = kColTileR / 4;
  if (EPI != EPI_STORE && l == 1) {
    // the epilogue's loads for all of the thread's rows first
    const float* ab = f.buf[BUF_ABASE];
    const float* xs = f.buf[BUF_X];
    float av[NO], xv[NO];
#pragma unroll
    for (int i = 0; i < NO; i++) {
      const int g = r0 + ty + 4 * i;
      const int idx = (g < H ? g : H - 1) * nx + cl;
      av[i] = ab[idx];
      xv[i] = EPI == EPI_CHECK ? xs[idx] : 0.0f;
    }
    bool bad = false;
#pragma unroll
    for (int i = 0; i < NO; i++) {
      const int g = r0 + ty + 4 * i;
      if (g < H && col < W) bad |= epilogue_loaded<EPI>(g * nx + col, s[kHalo + ty + 4 * i][tx], av[i], xv[i], f, sc);
    }
    if (EPI == EPI_CHECK) report_violation(bad, f);
  } else {
    for (int r = kHalo + ty; r < kColTileR + kHalo; r += 4) {
      int g = r0 - kHalo + r;
      if (g < H && col < W) dp[g * nx + col] = s[r][tx];
    }
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

// Forward horizontal pass of level l: buf[BUF_TMP] -> buf[dst] deinterleaved.
__global__ __launch_bounds__(256) void k_fwd_rows(const FieldDev* __restrict__ F, int l, int dst) {
  const FieldDev& f = F[blockIdx.z];
  if (!f.active || l > f.L) return;
  const int nx = f.nx, H = lvl_size(f.ny, l), W = lvl_size(f.nx, l);
  int c0 = blockIdx.x * kRowTileC, r0 = blockIdx.y * kRowTileR;
  if (c0 >= W || r0 >= H) return;
  const float* src = f.buf[BUF_TMP];
  float* dp = f.buf[dst];
  __shared__ float s[kRowTileR][kRowTileC + 2 * kHalo + 1];
  const int NC = kRowTileC + 2 * kHalo;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  {
    // loads first (see k_fwd_cols); each thread holds one column, and the
    // first NC - 256 threads a second one
    const int cc1 = threadIdx.x + 256;
    const int g0 = mirror(c0 - kHalo + (int)threadIdx.x, W);
    float v0[kRowTileR], v1[kRowTileR];
#pragma unroll
    for (int rr = 0; rr < kRowTileR; rr++) v0[rr] = src[(r0 + rr < H ? r0 + rr : H - 1) * nx + g0];
    if (cc1 < NC) {
      const int g1 = mirror(c0 - kHalo + cc1, W);
#pragma unroll
      for (int rr = 0; rr < kRowTileR; rr++) v1[rr] = src[(r0 + rr < H ? r0 + rr : H - 1) * nx + g1];
    }
#pragma unroll
    for (int rr = 0; rr < kRowTileR; rr++) {
      const bool in = r0 + rr < H;
      s[rr][threadIdx.x] = in ? v0[rr] : 0.0f;
      if (cc1 < NC) s[rr][cc1] = in ? v1[rr] : 0.0f;
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
        dp[row * nx + ocol] = v;
      }
    }
  }
}

// Inverse horizontal pass of level l: buf[a] (deinterleaved) -> buf[BUF_TMP].
__global__ __launch_bounds__(256) void k_inv_rows(const FieldDev* __restrict__ F, int l, int a) {
  const FieldDev& f = F[blockIdx.z];
  if (!f.active || l > f.L) return;
  const int nx = f.nx, H = lvl_size(f.ny, l), W = lvl_size(f.nx, l);
  int c0 = blockIdx.x * kRowTileC, r0 = blockIdx.y * kRowTileR;
  if (c0 >= W || r0 >= H) return;
  const float* src = f.buf[a];
  float* dp = f.buf[BUF_TMP];
  __shared__ float s[kRowTileR][kRowTileC + 2 * kHalo + 1];
  const int NC = kRowTileC + 2 * kHalo;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  int nl = (W + 1) >> 1;
  {
    // loads first (see k_fwd_cols)
    const int cc1 = threadIdx.x + 256;
    const int g0 = mirror(c0 - kHalo + (int)threadIdx.x, W);
    const int sc0 = (g0 & 1) ? nl + (g0 >> 1) : (g0 >> 1);
    float v0[kRowTileR], v1[kRowTileR];
#pragma unroll
    for (int rr = 0; rr < kRowTileR; rr++) v0[rr] = src[(r0 + rr < H ? r0 + rr : H - 1) * nx + sc0];
    int g1 = 0;
    if (cc1 < NC) {
      g1 = mirror(c0 - kHalo + cc1, W);
      const int sc1 = (g1 & 1) ? nl + (g1 >> 1) : (g1 >> 1);
#pragma unroll
      for (int rr = 0; rr < kRowTileR; rr++) v1[rr] = src[(r0 + rr < H ? r0 + rr : H - 1) * nx + sc1];
    }
#pragma unroll
    for (int rr = 0; rr < kRowTileR; rr++) {
      const bool in = r0 + rr < H;
      s[rr][threadIdx.x] = in ? ((g0 & 1) ? v0[rr] * L97_IK : v0[rr] * L97_K) : 0.0f;
      if (cc1 < NC) s[rr][cc1] = in ? ((g1 & 1) ? v1[rr] * L97_IK : v1[rr] * L97_K) : 0.0f;
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
      if (g < W) dp[row * nx + g] = s[rr][cc];
    }
  }
}

// Elementwise prologue/epilogue over whole fields (blockIdx.y = field).
// PRO value 3 means "the value is zero" (no residual).  lzero: only fields
// without transform levels take part.
template <int PRO, int EPI>
__global__ __launch_bounds__(256) void k_pointwise(const FieldDev* __restrict__ F, int src, int dst, int lzero) {
  const FieldDev& f = F[blockIdx.y];
  if (!f.active || (lzero && f.L != 0)) return;
  const int n = f.ny * f.nx;
  Scal sc = load_scal(f.fp);
  const float* sp = f.buf[src];
  float* dp = f.buf[dst];
  bool bad = false;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = (PRO == 3) ? 0.0f : prologue<(PRO == 3 ? 0 : PRO)>(sp, i, f, sc);
    bad |= epilogue<EPI>(dp, i, v, f, sc);
  }
  if (EPI == EPI_CHECK) report_violation(bad, f);
}

struct Grid2 { int gx, gy; };
static Grid2 level_grid(const FieldDev* Fh, int nf, int l, int tc, int tr) {
  Grid2 g{0, 0};
  for (int i = 0; i < nf; i++) {
    if (!Fh[i].active || l > Fh[i].L) continue;
    int H = Fh[i].ny, W = Fh[i].nx;
    for (int k = 1; k < l; k++) { H = (H + 1) / 2; W = (W + 1) / 2; }
    g.gx = std::max(g.gx, (W + tc - 1) / tc);
    g.gy = std::max(g.gy, (H + tr - 1) / tr);
  }
  return g;
}
static int max_L(const FieldDev* Fh, int nf) {
  int m = 0;
  for (int i = 0; i < nf; i++)
    if (Fh[i].active) m = std::max(m, Fh[i].L);
  return m;
}
static bool any_lzero(const FieldDev* Fh, int nf) {
  for (int i = 0; i < nf; i++)
    if (Fh[i].active && Fh[i].L == 0) return true;
  return false;
}
static int max_n(const FieldDev* Fh, int nf) {
  int m = 0;
  for (int i = 0; i < nf; i++)
    if (Fh[i].active) m = std::max(m, Fh[i].ny * Fh[i].nx);
  return m;
}

void dwt_forward(const FieldDev* F, const FieldDev* Fh, int nf, int src, int dst, int pro, hipStream_t st) {
  if (any_lzero(Fh, nf)) pointwise(F, Fh, nf, src, dst, pro, EPI_STORE, 1, st);
  int Lm = max_L(Fh, nf);
  for (int l = 1; l <= Lm; l++) {
    Grid2 c = level_grid(Fh, nf, l, kColTileC, kColTileR);
    if (c.gx == 0) continue;
    dim3 gc(c.gx, c.gy, nf);
    int p = (l == 1) ? pro : PRO_COPY;
    if (p == PRO_NORM) k_fwd_cols<PRO_NORM><<<gc, 256, 0, st>>>(F, l, src, dst);
    else if (p == PRO_NORM_MINUS) k_fwd_cols<PRO_NORM_MINUS><<<gc, 256, 0, st>>>(F, l, src, dst);
    else k_fwd_cols<PRO_COPY><<<gc, 256, 0, st>>>(F, l, src, dst);
    Grid2 r = level_grid(Fh, nf, l, kRowTileC, kRowTileR);
    k_fwd_rows<<<dim3(r.gx, r.gy, nf), 256, 0, st>>>(F, l, dst);
  }
}

// The passes of the inverse transform but the last (level 1's vertical pass,
// the one with the epilogue), and that last pass with the fields of one
// level (L = 0) done pointwise: split so that the first part can run on
// another stream before the epilogue's inputs are ready.
void dwt_inverse_head(const FieldDev* F, const FieldDev* Fh, int nf, int a, hipStream_t st) {
  int Lm = max_L(Fh, nf);
  for (int l = Lm; l >= 1; l--) {
    Grid2 r = level_grid(Fh, nf, l, kRowTileC, kRowTileR);
    if (r.gx == 0) continue;
    k_inv_rows<<<dim3(r.gx, r.gy, nf), 256, 0, st>>>(F, l, a);
    if (l == 1) break;
    Grid2 c = level_grid(Fh, nf, l, kColTileC, kColTileR);
    k_inv_cols<EPI_STORE><<<dim3(c.gx, c.gy, nf), 256, 0, st>>>(F, l, a, a);
  }
}

void dwt_inverse_tail(const FieldDev* F, const FieldDev* Fh, int nf, int a, int out, int epi, hipStream_t st) {
  if (any_lzero(Fh, nf)) pointwise(F, Fh, nf, a, out, PRO_COPY, epi, 1, st);
  Grid2 c = level_grid(Fh, nf, 1, kColTileC, kColTileR);
  if (c.gx == 0) return;
  dim3 gc(c.gx, c.gy, nf);
  if (epi == EPI_FINAL) k_inv_cols<EPI_FINAL><<<gc, 256, 0, st>>>(F, 1, a, out);
  else if (epi == EPI_CHECK) k_inv_cols<EPI_CHECK><<<gc, 256, 0, st>>>(F, 1, a, out);
  else k_inv_cols<EPI_STORE><<<gc, 256, 0, st>>>(F, 1, a, out);
}

void dwt_inverse(const FieldDev* F, const FieldDev* Fh, int nf, int a, int out, int epi, hipStream_t st) {
  dwt_inverse_head(F, Fh, nf, a, st);
  dwt_inverse_tail(F, Fh, nf, a, out, epi, st);
}

void pointwise(const FieldDev* F, const FieldDev* Fh, int nf, int src, int dst, int pro, int epi, int lzero,
               hipStream_t st) {
  int n = max_n(Fh, nf);
  int blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  dim3 g(blocks, nf);
#define PW(P, E) k_pointwise<P, E><<<g, 256, 0, st>>>(F, src, dst, lzero)
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
