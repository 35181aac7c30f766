// Host runtime and C ABI of libebcc.so: per-shape plans (subbands,
// code-blocks, SPIHT tiles), per-stream device workspaces, and the
// orchestration of the EBCC compression process (Algorithm 1 with a fixed
// base ratio and plane-granular truncation of the residual) and of
// decompression.  Also holds the small kernels of the path: min/max and
// field scalars, residual quantisation, reductions, scans, packing and the
// stream checksum.
#include "common.h"
#include "ebcc.h"

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace ebcc {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(EBCC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Stage profiling: HIP events recorded on the caller's stream at stage
// boundaries; the time since the previous boundary is added to the stage
// that just ended.  Off unless enabled (then every call synchronises once
// more at its end to read the events).
// ---------------------------------------------------------------------------
enum Stage {
  S_SCALARS, S_DWT, S_QUANT, S_T1ENC, S_PCRD, S_BASEREC, S_RESID, S_SEARCH, S_SPIHT, S_PACK,
  S_D_PARSE, S_D_T1, S_D_IDWT_BASE, S_D_SPIHT, S_D_FINAL, S_COUNT
};
static const char* kStageNames[S_COUNT] = {
    "scalars", "dwt_fwd", "quant_planes", "t1_encode", "pcrd", "base_recon", "resid_dwt_quant",
    "plane_search", "spiht_encode", "pack", "dec_parse", "t1_decode", "dec_idwt_base", "spiht_decode",
    "dec_final"};
static int g_prof = 0;
static double g_stage_ms[S_COUNT];
static long g_stage_calls[S_COUNT];
static std::mutex g_prof_mu;

struct Prof {
  hipStream_t st;
  bool on;
  hipEvent_t prev = nullptr;
  std::vector<std::pair<int, hipEvent_t>> marks;
  hipEvent_t first = nullptr;
  explicit Prof(hipStream_t s) : st(s), on(g_prof != 0) {
    if (!on) return;
    if (hipEventCreate(&first) != hipSuccess || hipEventRecord(first, st) != hipSuccess) on = false;
  }
  void mark(int stage) {
    if (!on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    marks.push_back(std::make_pair(stage, e));
  }
  ~Prof() {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t a = first;
    for (auto& m : marks) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, a, m.second) == hipSuccess) {
        g_stage_ms[m.first] += ms;
        g_stage_calls[m.first] += 1;
      }
      a = m.second;
    }
    for (auto& m : marks) (void)hipEventDestroy(m.second);
    (void)hipEventDestroy(first);
  }
};

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned f2o(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__global__ void k_init_fp(FieldParams* fp, int* flags, int nflags) {
  fp->xmin_bits = 0xFFFFFFFFu;
  fp->xmax_bits = 0u;
  fp->nonfinite = 0;
  for (int i = 0; i < nflags; i++) flags[i] = 0;
}

__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, int n, FieldParams* fp) {
  unsigned mn = 0xFFFFFFFFu, mx = 0u;
  int nf = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = x[i];
    if (!__builtin_isfinite(v)) { nf = 1; continue; }
    unsigned o = f2o(v);
    mn = o < mn ? o : mn;
    mx = o > mx ? o : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    unsigned a = __shfl_xor(mn, off), b = __shfl_xor(mx, off);
    int c = __shfl_xor(nf, off);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    nf |= c;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&fp->xmin_bits, mn);
    atomicMax(&fp->xmax_bits, mx);
    if (nf) atomicOr(&fp->nonfinite, 1);
  }
}

// Field scalars (range, bound, quantiser exponents) from min and max.
// eps is range-relative (Benchmarks section) or absolute.
__global__ void k_params(FieldParams* fp, double err, int bound_mode) {
  float xmin = o2f(fp->xmin_bits), xmax = o2f(fp->xmax_bits);
  if (xmin == 0.0f) xmin = 0.0f;   // +0 for a zero extreme
  if (xmax == 0.0f) xmax = 0.0f;
  fp->xmin = xmin;
  fp->xmax = xmax;
  double range_d = (double)xmax - (double)xmin;
  double eps = bound_mode == EBCC_BOUND_REL ? err * range_d : err;
  fp->range_d = range_d;
  fp->eps = eps;
  fp->range_f = 0.0f;
  fp->inv_f = 0.0f;
  fp->elog = 0;
  fp->e0 = 0;
  if (fp->nonfinite) { fp->mode = -1; return; }
  if (range_d == 0.0) { fp->mode = MODE_CONST; return; }
  double en = eps / range_d;
  int ex;
  frexp(en, &ex);
  int elog = ex - 1;                       // floor(log2(eps / range))
  fp->eps_norm = en;
  fp->elog = elog;
  fp->mode = elog < -40 ? MODE_RAW : MODE_CODED;
  int e0 = elog - 2;
  e0 = e0 < -20 ? -20 : (e0 > 0 ? 0 : e0);
  fp->e0 = e0;
  fp->range_f = (float)range_d;
  fp->inv_f = (float)(1.0 / range_d);
}

__global__ void k_set_decode_params(FieldParams* fp, float xmin, float range_f, int* flags, int nflags) {
  fp->xmin = xmin;
  fp->range_f = range_f;
  fp->inv_f = 0.0f;
  fp->eps = 0.0;
  for (int i = 0; i < nflags; i++) flags[i] = 0;
}

__global__ void k_zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int n, float v) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

// Residual quantisation q_r = floor(|c| * 2^-e_r) (capped), sign in bit 31.
__global__ __launch_bounds__(256) void k_quant_res(const float* __restrict__ c, int n, int er, uint32_t* __restrict__ qr,
                                                   unsigned* __restrict__ qmax) {
  unsigned mx = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = c[i];
    uint32_t q = quantq(v, -er);
    qr[i] = q | (v < 0.0f ? 0x80000000u : 0u);
    mx = q > mx ? q : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    unsigned a = __shfl_xor(mx, off);
    mx = a > mx ? a : mx;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(qmax, mx);
}

// Residual coefficients kept by truncation at the end of plane n_s, midpoint
// reconstructed: what the SPIHT decoder recovers from planes n_max .. n_s.
__global__ __launch_bounds__(256) void k_dequant_res(const uint32_t* __restrict__ qr, int n, int ns, int er,
                                                     float* __restrict__ out) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    uint32_t v = qr[i], q = v & 0x7FFFFFu;
    uint32_t m = (q >> ns) << ns;
    out[i] = dequant(m, ns, (int)(v >> 31), er);
  }
}

// Exclusive scan of n 32-bit lengths (len = (v >> shift) & mask) in one
// workgroup; off[i] = sum of the lengths before i; *total = sum of all.
__global__ __launch_bounds__(1024) void k_scan(const uint32_t* __restrict__ v, int n, int shift, uint32_t mask,
                                               int64_t* __restrict__ off, int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  int tid = threadIdx.x;
  int per = (n + 1023) / 1024;
  int b0 = tid * per, b1 = b0 + per < n ? b0 + per : n;
  int64_t s = 0;
  for (int i = b0; i < b1; i++) s += (int64_t)((v[i] >> shift) & mask);
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t t = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += t;
    __syncthreads();
  }
  int64_t run = part[tid] - s;
  for (int i = b0; i < b1; i++) {
    off[i] = run;
    run += (int64_t)((v[i] >> shift) & mask);
  }
  if (tid == 1023) *total = part[1023];
}

// Block table entries (P_b | k_b << 8 | len << 16) of the coded stream.
__global__ __launch_bounds__(256) void k_block_entries(const uint8_t* __restrict__ pb, const uint8_t* __restrict__ kb,
                                                       const int32_t* __restrict__ len, int nblk,
                                                       uint32_t* __restrict__ ent) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nblk; b += gridDim.x * 256)
    ent[b] = (uint32_t)pb[b] | ((uint32_t)kb[b] << 8) | ((uint32_t)len[b] << 16);
}

__global__ __launch_bounds__(256) void k_put_table(const uint32_t* __restrict__ ent, int n, uint8_t* __restrict__ out) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < n; b += gridDim.x * 256) {
    uint32_t v = ent[b];
    out[4 * b] = (uint8_t)v;
    out[4 * b + 1] = (uint8_t)(v >> 8);
    out[4 * b + 2] = (uint8_t)(v >> 16);
    out[4 * b + 3] = (uint8_t)(v >> 24);
  }
}

// Terminated codewords: bytes before the termination point from the
// encoder's buffer, then the bytes the termination of pass k_b writes.
__global__ __launch_bounds__(256) void k_gather_cw(const uint8_t* __restrict__ cw, const uint8_t* __restrict__ kb,
                                                   const int32_t* __restrict__ len, const int32_t* __restrict__ bpt,
                                                   const uint32_t* __restrict__ tailt, const int64_t* __restrict__ off,
                                                   int nblk, uint8_t* __restrict__ out) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int b = blockIdx.x * 4 + wave; b < nblk; b += gridDim.x * 4) {
    int k = kb[b], n = len[b];
    if (!k) continue;
    int bp = bpt[(size_t)b * kPassStride + k];
    uint32_t tl = tailt[(size_t)b * kPassStride + k];
    const uint8_t* src = cw + (size_t)b * kCwCap;
    uint8_t* dst = out + off[b];
    for (int j = lane; j < n; j += 64) dst[j] = j < bp ? src[j] : (uint8_t)(tl >> (8 * (j - bp)));
  }
}

__global__ __launch_bounds__(256) void k_gather_tiles(const uint8_t* __restrict__ slots, const int64_t* __restrict__ slot_off,
                                                      const uint32_t* __restrict__ tlen, const int64_t* __restrict__ off,
                                                      int nt, uint8_t* __restrict__ out) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = blockIdx.x * 4 + wave; t < nt; t += gridDim.x * 4) {
    int64_t cap = slot_off[t + 1] - slot_off[t];
    int n = (int)((int64_t)tlen[t] < cap ? (int64_t)tlen[t] : cap);
    const uint8_t* src = slots + slot_off[t];
    uint8_t* dst = out + off[t];
    for (int j = lane; j < n; j += 64) dst[j] = src[j];
  }
}

// Stream checksum: sum over the little-endian 32-bit words w_k of the bytes
// after the header (zero padded) of w_k * (2k + 1), modulo 2^32.
__global__ __launch_bounds__(256) void k_checksum(const uint8_t* __restrict__ p, const int64_t* __restrict__ total_dev,
                                                  int64_t total_host, unsigned* __restrict__ sum) {
  int64_t n = (total_dev ? *total_dev : total_host) - kHdr;
  const uint8_t* q = p + kHdr;
  int64_t nw = (n + 3) / 4;
  unsigned s = 0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nw; k += (int64_t)gridDim.x * 256) {
    uint32_t w = 0;
    for (int b = 0; b < 4; b++)
      if (4 * k + b < n) w |= (uint32_t)q[4 * k + b] << (8 * b);
    s += w * (uint32_t)(2 * k + 1);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(sum, s);
}

__device__ __forceinline__ void put32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
__global__ void k_header(uint8_t* o, const FieldParams* fp, int mode, int L, int cbl, int ny, int nx, int er, int nmax,
                         int ns, int T, uint32_t bb, uint32_t rb, const unsigned* csum) {
  for (int i = 0; i < kHdr; i++) o[i] = 0;
  o[0] = 'E'; o[1] = 'B'; o[2] = 'C'; o[3] = 'C';
  o[4] = 1; o[5] = (uint8_t)mode; o[6] = (uint8_t)L; o[7] = (uint8_t)cbl;
  put32(o + 8, (uint32_t)ny);
  put32(o + 12, (uint32_t)nx);
  put32(o + 16, __float_as_uint(fp->xmin));
  put32(o + 20, __float_as_uint(mode == MODE_CONST ? 0.0f : fp->range_f));
  put32(o + 24, __float_as_uint(mode == MODE_CONST ? 0.0f : fp->inv_f));
  o[28] = (uint8_t)(int8_t)(mode == MODE_CODED ? fp->e0 : 0);
  o[29] = (uint8_t)(int8_t)er;
  o[30] = (uint8_t)(int8_t)nmax;
  o[31] = (uint8_t)(int8_t)ns;
  o[32] = (uint8_t)T; o[33] = (uint8_t)(T >> 8);
  put32(o + 36, bb);
  put32(o + 40, rb);
  put32(o + 44, *csum);
}

// Decoder: offsets and validity of the base block table and the tile table.
__global__ __launch_bounds__(256) void k_check_tables(const uint8_t* __restrict__ in, int nblk, int64_t bb,
                                                      const int64_t* __restrict__ btot, int* __restrict__ flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    if (*btot != bb - 4 * (int64_t)nblk) atomicOr(flag, 1);
}
__global__ __launch_bounds__(256) void k_read_table(const uint8_t* __restrict__ tab, int n, uint32_t* __restrict__ ent) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < n; b += gridDim.x * 256)
    ent[b] = (uint32_t)tab[4 * b] | ((uint32_t)tab[4 * b + 1] << 8) | ((uint32_t)tab[4 * b + 2] << 16) |
             ((uint32_t)tab[4 * b + 3] << 24);
}

// ---------------------------------------------------------------------------
// Plans: per-shape geometry on the host and on the device.
// ---------------------------------------------------------------------------
struct Plan {
  int ny, nx, L, cbl2w, cbl2h, cbw, cbh, T;
  std::vector<Band> bands;
  std::vector<Blk> blks;
  std::vector<TileD> tiles;
  std::vector<int64_t> slot_off;   // ntiles + 1
  Band* d_bands = nullptr;
  Blk* d_blks = nullptr;
  TileD* d_tiles = nullptr;
  int64_t* d_slot_off = nullptr;
  int nblk = 0, ntiles = 0, nb = 0;
  int max_tile_coef = 0, max_tile_parents = 0;
  int spiht_cap = 0;   // LDS capacity class of the per-tile SPIHT kernels (0: global-memory kernels)
  ~Plan() {
    if (d_bands) (void)hipFree(d_bands);
    if (d_blks) (void)hipFree(d_blks);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_slot_off) (void)hipFree(d_slot_off);
  }
};

static int levels_eff(int ny, int nx, int L) {
  int m = ny < nx ? ny : nx, f = 0;
  while ((2L << f) <= m) f++;
  if (L > f) L = f;
  if (L > kMaxLevels) L = kMaxLevels;
  return L < 0 ? 0 : L;
}

static int build_plan(Plan& p) {
  int ny = p.ny, nx = p.nx, L = p.L;
  std::vector<int> h(L + 1), w(L + 1);
  h[0] = ny; w[0] = nx;
  for (int l = 1; l <= L; l++) { h[l] = (h[l - 1] + 1) / 2; w[l] = (w[l - 1] + 1) / 2; }
  // subbands: LL_L, then HL, LH, HH for l = L .. 1; gains g = l (LL),
  // l - 1 (HL, LH), l - 2 (HH): log2 of the 9/7 synthesis gains, rounded
  p.bands.push_back(Band{L, ORI_LL, 0, 0, h[L], w[L], L});
  for (int l = L; l >= 1; l--) {
    p.bands.push_back(Band{l, ORI_HL, 0, w[l], h[l], w[l - 1] - w[l], l - 1});
    p.bands.push_back(Band{l, ORI_LH, h[l], 0, h[l - 1] - h[l], w[l], l - 1});
    p.bands.push_back(Band{l, ORI_HH, h[l], w[l], h[l - 1] - h[l], w[l - 1] - w[l], l - 2});
  }
  p.nb = (int)p.bands.size();
  for (const Band& b : p.bands)
    for (int by = 0; by < b.h; by += p.cbh)
      for (int bx = 0; bx < b.w; bx += p.cbw)
        p.blks.push_back(Blk{b.y0 + by, b.x0 + bx, std::min(p.cbw, b.w - bx), std::min(p.cbh, b.h - by), b.orient, b.gain});
  p.nblk = (int)p.blks.size();
  // SPIHT tiles: T x T LL roots and the rectangles their trees cover per band
  int hL = h[L], wL = w[L], T = p.T;
  int ty = (hL + T - 1) / T, tx = (wL + T - 1) / T;
  int64_t off = 0, soff = 0;
  p.slot_off.push_back(0);
  for (int a = 0; a < ty; a++)
    for (int c = 0; c < tx; c++) {
      TileD t;
      t.i0 = a * T; t.i1 = std::min(hL, t.i0 + T);
      t.j0 = c * T; t.j1 = std::min(wL, t.j0 + T);
      int64_t n = (int64_t)(t.i1 - t.i0) * (t.j1 - t.j0), n1 = 0;
      for (int o = 0; o < 3 && L > 0; o++) {
        const Band& top = p.bands[1 + o];
        int r0 = t.i0, r1 = std::min(t.i1, top.h), c0 = t.j0, c1 = std::min(t.j1, top.w);
        for (int l = L;; l--) {
          if (r0 >= r1 || c0 >= c1) break;
          n += (int64_t)(r1 - r0) * (c1 - c0);
          if (l == 1) { n1 += (int64_t)(r1 - r0) * (c1 - c0); break; }
          const Band& pb = p.bands[1 + 3 * (L - l) + o];
          const Band& cb = p.bands[1 + 3 * (L - l + 1) + o];
          int nr0 = 2 * r0, nr1 = (r1 == pb.h) ? cb.h : std::min(2 * r1, cb.h);
          int nc0 = 2 * c0, nc1 = (c1 == pb.w) ? cb.w : std::min(2 * c1, cb.w);
          r0 = nr0; r1 = nr1; c0 = nc0; c1 = nc1;
        }
      }
      t.off = off;
      t.ncoef = (int)n;
      p.max_tile_coef = std::max(p.max_tile_coef, (int)n);
      p.max_tile_parents = std::max(p.max_tile_parents, (int)(L > 0 ? n - n1 : 0));
      t.pad = 0;
      off += n;
      soff += 12 * n + 16;
      p.tiles.push_back(t);
      p.slot_off.push_back(soff);
    }
  p.ntiles = (int)p.tiles.size();
  p.spiht_cap = spiht_lds_cap(std::max(p.max_tile_coef, 2 * p.max_tile_parents));
  if (off != (int64_t)ny * nx) return fail(EBCC_EINVAL, "internal: SPIHT trees do not cover the field");
  HIPCHK(hipMalloc(&p.d_bands, sizeof(Band) * p.bands.size()));
  HIPCHK(hipMemcpy(p.d_bands, p.bands.data(), sizeof(Band) * p.bands.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_blks, sizeof(Blk) * std::max<size_t>(1, p.blks.size())));
  if (p.nblk) HIPCHK(hipMemcpy(p.d_blks, p.blks.data(), sizeof(Blk) * p.blks.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_tiles, sizeof(TileD) * p.tiles.size()));
  HIPCHK(hipMemcpy(p.d_tiles, p.tiles.data(), sizeof(TileD) * p.tiles.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_slot_off, sizeof(int64_t) * p.slot_off.size()));
  HIPCHK(hipMemcpy(p.d_slot_off, p.slot_off.data(), sizeof(int64_t) * p.slot_off.size(), hipMemcpyHostToDevice));
  return EBCC_OK;
}

// SPIHT kernel family for a plan: LDS per tile when the tiles fit (the
// environment variable EBCC_SPIHT_KERNEL=global forces the global-memory
// kernels, for testing both families).
static int spiht_cap_for(const Plan* p) {
  const char* e = getenv("EBCC_SPIHT_KERNEL");
  return (e && e[0] == 'g') ? 0 : p->spiht_cap;
}

static std::mutex g_mu;
typedef std::tuple<int, int, int, int, int, int, int> PlanKey;   // device, ny, nx, L, cbl2w, cbl2h, T
static std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

static int get_plan(int ny, int nx, int L, int cbl2w, int cbl2h, int T, Plan** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  PlanKey key(dev, ny, nx, L, cbl2w, cbl2h, T);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) { *out = it->second.get(); return EBCC_OK; }
  std::unique_ptr<Plan> p(new Plan());
  p->ny = ny; p->nx = nx; p->L = L; p->cbl2w = cbl2w; p->cbl2h = cbl2h;
  p->cbw = 1 << cbl2w; p->cbh = 1 << cbl2h; p->T = T;
  int rc = build_plan(*p);
  if (rc) return rc;
  *out = p.get();
  g_plans[key] = std::move(p);
  return EBCC_OK;
}

// ---------------------------------------------------------------------------
// Workspaces: one device allocation per (device, stream), carved per call.
// ---------------------------------------------------------------------------
struct WS {
  void* base = nullptr;
  size_t cap = 0;
  ~WS() { if (base) (void)hipFree(base); }
};
typedef std::pair<int, hipStream_t> WSKey;
static std::map<WSKey, std::unique_ptr<WS>> g_ws;

struct Carve {
  char* p;
  size_t used;
  template <typename T> T* take(size_t n) {
    size_t a = (used + 255) & ~(size_t)255;
    T* r = (T*)(p ? p + a : nullptr);
    used = a + sizeof(T) * (n ? n : 1);
    return r;
  }
};

struct Bufs {
  FieldParams* fp;
  int* flags;            // [0] check violation, [1] decode corruption
  unsigned* u32s;        // [0] qmax, [1] checksum
  int64_t* totals;       // [0] base payload, [1] resid payload, [2] stream total
  float *coef, *tmp, *yhat, *abase, *cres, *chat;
  uint32_t *qr, *sub, *maxd, *maxl;
  void *planes, *signs, *sppf;
  uint8_t *pb, *kb, *hk, *nh, *cw, *slots;
  int32_t *R, *bpt, *dr, *len;
  int64_t *D, *boff, *toff;
  uint64_t *keys, *lists;
  uint32_t *tail, *tlen, *tent, *bent;
  int* misfit;
};

static size_t layout(const Plan& p, Bufs* b, char* base) {
  Carve c{base, 0};
  size_t N = (size_t)p.ny * p.nx;
  size_t ms = p.cbw <= 32 ? 4 : 8;
  size_t nb = p.nblk, nt = p.ntiles;
  b->fp = c.take<FieldParams>(1);
  b->flags = c.take<int>(8);
  b->u32s = c.take<unsigned>(8);
  b->totals = c.take<int64_t>(8);
  b->coef = c.take<float>(N); b->tmp = c.take<float>(N); b->yhat = c.take<float>(N);
  b->abase = c.take<float>(N); b->cres = c.take<float>(N); b->chat = c.take<float>(N);
  b->qr = c.take<uint32_t>(N); b->sub = c.take<uint32_t>(N); b->maxd = c.take<uint32_t>(N); b->maxl = c.take<uint32_t>(N);
  b->planes = c.take<char>(nb * kQBits * p.cbh * ms);
  b->signs = c.take<char>(nb * p.cbh * ms);
  b->sppf = c.take<char>(nb * p.cbh * ms);
  b->pb = c.take<uint8_t>(nb); b->kb = c.take<uint8_t>(nb); b->nh = c.take<uint8_t>(nb);
  b->hk = c.take<uint8_t>(nb * kPassStride);
  b->R = c.take<int32_t>(nb * kPassStride); b->bpt = c.take<int32_t>(nb * kPassStride);
  b->dr = c.take<int32_t>(nb * kPassStride); b->len = c.take<int32_t>(nb);
  b->D = c.take<int64_t>(nb * kPassStride); b->keys = c.take<uint64_t>(nb * kPassStride);
  b->tail = c.take<uint32_t>(nb * kPassStride);
  b->boff = c.take<int64_t>(nb); b->bent = c.take<uint32_t>(nb);
  b->cw = c.take<uint8_t>(nb * (size_t)kCwCap);
  b->tlen = c.take<uint32_t>(nt); b->tent = c.take<uint32_t>(nt); b->toff = c.take<int64_t>(nt);
  b->misfit = c.take<int>(nt);
  b->lists = c.take<uint64_t>(4 * N);
  b->slots = c.take<uint8_t>((size_t)p.slot_off.back());
  return c.used + 256;
}

static int get_ws(const Plan& p, hipStream_t st, Bufs* b) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  size_t need = layout(p, b, nullptr);
  std::lock_guard<std::mutex> lk(g_mu);
  std::unique_ptr<WS>& w = g_ws[WSKey(dev, st)];
  if (!w) w.reset(new WS());
  if (w->cap < need) {
    if (w->base) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(w->base));
      w->base = nullptr;
      w->cap = 0;
    }
    hipError_t e = hipMalloc(&w->base, need);
    if (e != hipSuccess) { w->base = nullptr; return fail(EBCC_ENOMEM, "workspace allocation failed"); }
    w->cap = need;
  }
  layout(p, b, (char*)w->base);
  return EBCC_OK;
}

static int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return g < 1 ? 1 : (int)g;
}

template <typename T>
static int d2h(T* h, const T* d, size_t n, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(h, d, sizeof(T) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return EBCC_OK;
}

static int check_params(size_t ny, size_t nx, const ebcc_params* p) {
  if (ny < 1 || nx < 1 || ny > (1u << 24) || nx > (1u << 24) || ny * nx > 0x7FFFFFFFull)
    return fail(EBCC_EINVAL, "field dimensions out of range");
  if (p->struct_size != sizeof(ebcc_params)) return fail(EBCC_EINVAL, "ebcc_params.struct_size mismatch");
  if (!(p->err_bound > 0) || !std::isfinite(p->err_bound)) return fail(EBCC_EINVAL, "err_bound must be > 0 and finite");
  if (p->bound_mode > 1) return fail(EBCC_EINVAL, "bad bound_mode");
  if (!(p->base_ratio >= 1.0) || !std::isfinite(p->base_ratio)) return fail(EBCC_EINVAL, "base_ratio must be >= 1");
  if (p->levels > (unsigned)kMaxLevels) return fail(EBCC_EINVAL, "levels out of range");
  if (p->cblk_log2w < 2 || p->cblk_log2w > 6 || p->cblk_log2h < 2 || p->cblk_log2h > 6)
    return fail(EBCC_EINVAL, "code-block size out of range");
  if (p->spiht_tile < 1 || p->spiht_tile > 64) return fail(EBCC_EINVAL, "spiht_tile out of range");
  if (p->q != 0.0) return fail(EBCC_ENOTIMPL, "the q-quantile base-ratio search is not implemented (q must be 0)");
  return EBCC_OK;
}

struct Trace {
  float *coef, *abase, *cres;
  uint8_t *kb, *pb;
  int32_t* info;
};

// RAW stream: header + the input bytes.
static int emit_raw(const float* x, size_t N, const Plan* pl, int cbl, int ny, int nx, int T, const Bufs& B, uint8_t* out,
                    size_t cap, size_t* out_len, hipStream_t st) {
  size_t total = kHdr + 4 * N;
  *out_len = total;
  if (total > cap) return fail(EBCC_ENOSPC, "output capacity too small");
  (void)pl;
  HIPCHK(hipMemcpyAsync(out + kHdr, x, 4 * N, hipMemcpyDeviceToDevice, st));
  k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 8);
  k_checksum<<<grid_for(N), 256, 0, st>>>(out, nullptr, (int64_t)total, &B.u32s[1]);
  k_header<<<1, 1, 0, st>>>(out, B.fp, MODE_RAW, 0, cbl, ny, nx, 0, -1, 0, T, (uint32_t)(4 * N), 0u, &B.u32s[1]);
  HIPCHK(hipGetLastError());
  return EBCC_OK;
}

static int compress_impl(const float* x, size_t ny_, size_t nx_, const ebcc_params* pp, uint8_t* out, size_t cap,
                         size_t* out_len, hipStream_t st, const Trace* tr) {
  ebcc_params dflt;
  if (!pp) { ebcc_params_default(&dflt); pp = &dflt; }
  if (!out_len) return fail(EBCC_EINVAL, "out_len is NULL");
  *out_len = 0;
  int rc = check_params(ny_, nx_, pp);
  if (rc) return rc;
  if (!x || !out) return fail(EBCC_EINVAL, "NULL buffer");
  int ny = (int)ny_, nx = (int)nx_;
  size_t N = (size_t)ny * nx;
  int L = levels_eff(ny, nx, (int)pp->levels);
  int cbl = (int)(pp->cblk_log2w | (pp->cblk_log2h << 4));
  int T = (int)pp->spiht_tile;
  Plan* pl;
  rc = get_plan(ny, nx, L, pp->cblk_log2w, pp->cblk_log2h, T, &pl);
  if (rc) return rc;
  Bufs B;
  rc = get_ws(*pl, st, &B);
  if (rc) return rc;
  int32_t info[11] = {0};
  Prof prof(st);

  // ---- scalars: min, max, range, eps, exponents ----
  k_init_fp<<<1, 1, 0, st>>>(B.fp, B.flags, 8);
  k_minmax<<<grid_for(N), 256, 0, st>>>(x, (int)N, B.fp);
  k_params<<<1, 1, 0, st>>>(B.fp, pp->err_bound, (int)pp->bound_mode);
  HIPCHK(hipGetLastError());
  prof.mark(S_SCALARS);
  FieldParams fp;
  if ((rc = d2h(&fp, B.fp, 1, st))) return rc;
  if (fp.mode < 0) return fail(EBCC_EINVAL, "input contains non-finite values");
  if (fp.mode == MODE_CONST) {
    *out_len = kHdr;
    if (cap < (size_t)kHdr) return fail(EBCC_ENOSPC, "output capacity too small");
    k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 8);
    k_header<<<1, 1, 0, st>>>(out, B.fp, MODE_CONST, 0, cbl, ny, nx, 0, -1, 0, T, 0u, 0u, &B.u32s[1]);
    HIPCHK(hipGetLastError());
    if (tr && tr->info) { info[0] = MODE_CONST; memcpy(tr->info, info, sizeof(info)); }
    return EBCC_OK;
  }
  if (fp.mode == MODE_RAW) {
    rc = emit_raw(x, N, pl, cbl, ny, nx, T, B, out, cap, out_len, st);
    if (tr && tr->info) { info[0] = MODE_RAW; memcpy(tr->info, info, sizeof(info)); }
    return rc;
  }
  const int e0 = fp.e0, elog = fp.elog;
  DwtIO io{x, B.abase, nullptr, &B.flags[0], B.fp};

  // ---- base layer: DWT of the normalised field, tier-1, PCRD at ratio r ----
  dwt_forward(x, B.coef, B.tmp, ny, nx, L, PRO_NORM, io, st);
  prof.mark(S_DWT);
  quant_planes(B.coef, nx, pl->d_blks, pl->nblk, e0, pl->cbw, pl->cbh, B.planes, B.signs, B.pb, st);
  prof.mark(S_QUANT);
  t1_encode(B.coef, nx, pl->d_blks, pl->nblk, e0, pl->cbw, pl->cbh, B.planes, B.signs, B.pb, B.cw, B.R, B.D, B.bpt,
            B.tail, B.sppf, st);
  prof.mark(S_T1ENC);
  int64_t total_budget = (int64_t)std::floor((double)(4.0 * (double)N) / pp->base_ratio);
  int64_t budget = total_budget - kHdr - 4 * (int64_t)pl->nblk;
  if (budget < 0) budget = 0;
  pcrd(B.pb, B.R, B.D, pl->nblk, budget, B.kb, B.hk, B.keys, B.dr, B.nh, B.len, st);
  prof.mark(S_PCRD);
  // ---- A_base = dec_base(e_base) (closed form), residual, its DWT ----
  virtual_decode(B.coef, nx, pl->d_blks, pl->nblk, e0, pl->cbw, pl->cbh, B.pb, B.kb, B.sppf, B.yhat, st);
  dwt_inverse(B.yhat, B.tmp, B.abase, ny, nx, L, EPI_STORE, io, st);
  pointwise(nullptr, nullptr, (int)N, 3, EPI_CHECK, io, st);   // does the base alone meet the bound?
  prof.mark(S_BASEREC);
  dwt_forward(x, B.cres, B.tmp, ny, nx, L, PRO_NORM_MINUS, io, st);
  int er = elog - 6;
  k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 8);
  k_quant_res<<<grid_for(N), 256, 0, st>>>(B.cres, (int)N, er, B.qr, &B.u32s[0]);
  HIPCHK(hipGetLastError());
  prof.mark(S_RESID);
  int hflag[2];
  unsigned qmax;
  if ((rc = d2h(hflag, B.flags, 1, st))) return rc;
  if ((rc = d2h(&qmax, B.u32s, 1, st))) return rc;
  int checks = 1;
  int mode = MODE_CODED, nmax = -1, ns = 0, er_out = 0;
  bool resid = hflag[0] != 0;
  auto feasible = [&](int k, int nm, int e_r, bool* ok) -> int {
    int s = nm - k + 1;
    k_zero_int<<<1, 64, 0, st>>>(B.flags, 1);
    k_dequant_res<<<grid_for(N), 256, 0, st>>>(B.qr, (int)N, s, e_r, B.chat);
    dwt_inverse(B.chat, B.tmp, nullptr, ny, nx, L, EPI_CHECK, io, st);
    HIPCHK(hipGetLastError());
    int f;
    int r = d2h(&f, B.flags, 1, st);
    if (r) return r;
    checks++;
    *ok = f == 0;
    return EBCC_OK;
  };
  if (resid) {
    bool found = false;
    for (int att = 0; att < 5 && !found; att++) {
      int e_r = elog - 6 - att;
      if (att > 0) {
        k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 1);
        k_quant_res<<<grid_for(N), 256, 0, st>>>(B.cres, (int)N, e_r, B.qr, &B.u32s[0]);
        if ((rc = d2h(&qmax, B.u32s, 1, st))) return rc;
      }
      int nm = qmax ? 31 - __builtin_clz(qmax) : -1;
      if (nm < 0) continue;
      int K = nm + 1;
      bool ok;
      if ((rc = feasible(K, nm, e_r, &ok))) return rc;
      if (!ok) continue;
      int lo = 0, hi = K;
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((rc = feasible(mid, nm, e_r, &ok))) return rc;
        if (ok) hi = mid; else lo = mid;
      }
      found = true;
      nmax = nm; ns = nm - hi + 1; er_out = e_r;
    }
    if (!found) mode = MODE_RAW;
  }
  prof.mark(S_SEARCH);
  if (mode == MODE_CODED && resid) {
    spiht_maxima(B.qr, nx, pl->d_bands, pl->bands.data(), pl->nb, L, B.sub, B.maxd, B.maxl, st);
    if (spiht_cap_for(pl))
      spiht_encode_lds(spiht_cap_for(pl), B.qr, B.sub, B.maxd, B.maxl, nx, pl->d_bands, pl->nb, L, pl->d_tiles,
                       pl->ntiles, ns, B.slots, pl->d_slot_off, B.tlen, B.tent, B.misfit, st);
    else
      spiht_encode(B.qr, B.sub, B.maxd, B.maxl, nx, pl->d_bands, pl->nb, L, pl->d_tiles, pl->ntiles, ns, B.lists,
                   B.slots, pl->d_slot_off, B.tlen, B.tent, st);
  }
  prof.mark(S_SPIHT);
  // ---- sizes ----
  k_block_entries<<<grid_for(pl->nblk), 256, 0, st>>>(B.pb, B.kb, B.len, pl->nblk, B.bent);
  k_scan<<<1, 1024, 0, st>>>(B.bent, pl->nblk, 16, 0xFFFFu, B.boff, &B.totals[0]);
  if (mode == MODE_CODED && resid) k_scan<<<1, 1024, 0, st>>>(B.tlen, pl->ntiles, 0, 0xFFFFFFFFu, B.toff, &B.totals[1]);
  HIPCHK(hipGetLastError());
  int64_t tot[2] = {0, 0};
  if ((rc = d2h(tot, B.totals, 2, st))) return rc;
  int64_t base_bytes = 4 * (int64_t)pl->nblk + tot[0];
  int64_t resid_bytes = (mode == MODE_CODED && resid) ? 4 * (int64_t)pl->ntiles + tot[1] : 0;
  if (mode == MODE_CODED && base_bytes + resid_bytes > 4 * (int64_t)N) mode = MODE_RAW;
  if (mode == MODE_RAW) {
    rc = emit_raw(x, N, pl, cbl, ny, nx, T, B, out, cap, out_len, st);
    if (tr && tr->info) { info[0] = MODE_RAW; info[10] = checks; memcpy(tr->info, info, sizeof(info)); }
    return rc;
  }
  size_t total = kHdr + (size_t)base_bytes + (size_t)resid_bytes;
  *out_len = total;
  if (total > cap) return fail(EBCC_ENOSPC, "output capacity too small");
  // ---- pack: header, block table, codewords, tile table, tile payloads ----
  uint8_t* bsec = out + kHdr;
  k_put_table<<<grid_for(pl->nblk), 256, 0, st>>>(B.bent, pl->nblk, bsec);
  k_gather_cw<<<grid_for(pl->nblk), 256, 0, st>>>(B.cw, B.kb, B.len, B.bpt, B.tail, B.boff, pl->nblk,
                                                  bsec + 4 * (size_t)pl->nblk);
  if (resid) {
    uint8_t* rsec = bsec + base_bytes;
    k_put_table<<<grid_for(pl->ntiles), 256, 0, st>>>(B.tent, pl->ntiles, rsec);
    k_gather_tiles<<<grid_for(pl->ntiles), 256, 0, st>>>(B.slots, pl->d_slot_off, B.tlen, B.toff, pl->ntiles,
                                                         rsec + 4 * (size_t)pl->ntiles);
  }
  k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 8);
  k_checksum<<<grid_for((total + 3) / 4), 256, 0, st>>>(out, nullptr, (int64_t)total, &B.u32s[1]);
  if (!resid) { nmax = -1; ns = 0; er_out = 0; }
  k_header<<<1, 1, 0, st>>>(out, B.fp, MODE_CODED, L, cbl, ny, nx, er_out, nmax, ns, T, (uint32_t)base_bytes,
                            (uint32_t)resid_bytes, &B.u32s[1]);
  HIPCHK(hipGetLastError());
  prof.mark(S_PACK);
  if (tr) {
    if (tr->coef) HIPCHK(hipMemcpyAsync(tr->coef, B.coef, 4 * N, hipMemcpyDeviceToDevice, st));
    if (tr->abase) HIPCHK(hipMemcpyAsync(tr->abase, B.abase, 4 * N, hipMemcpyDeviceToDevice, st));
    if (tr->cres) HIPCHK(hipMemcpyAsync(tr->cres, B.cres, 4 * N, hipMemcpyDeviceToDevice, st));
    if (tr->kb) HIPCHK(hipMemcpyAsync(tr->kb, B.kb, pl->nblk, hipMemcpyDeviceToDevice, st));
    if (tr->pb) HIPCHK(hipMemcpyAsync(tr->pb, B.pb, pl->nblk, hipMemcpyDeviceToDevice, st));
    if (tr->info) {
      info[0] = MODE_CODED; info[1] = L; info[2] = e0; info[3] = er_out; info[4] = nmax; info[5] = ns;
      info[6] = pl->nblk; info[7] = pl->ntiles; info[8] = (int32_t)base_bytes; info[9] = (int32_t)resid_bytes;
      info[10] = checks;
      memcpy(tr->info, info, sizeof(info));
    }
    HIPCHK(hipStreamSynchronize(st));
  }
  return EBCC_OK;
}

static uint32_t rd32(const uint8_t* p) { return p[0] | (p[1] << 8) | (p[2] << 16) | ((uint32_t)p[3] << 24); }

static int decompress_impl(const uint8_t* in, size_t in_len, float* x, size_t ny_, size_t nx_, hipStream_t st) {
  if (!in || !x) return fail(EBCC_EINVAL, "NULL buffer");
  if (in_len < (size_t)kHdr) return fail(EBCC_ECORRUPT, "stream shorter than its header");
  uint8_t h[kHdr];
  HIPCHK(hipMemcpyAsync(h, in, kHdr, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  size_t hny, hnx;
  int mode;
  if (ebcc_stream_info(h, kHdr, &hny, &hnx, &mode) != EBCC_OK) return fail(EBCC_ECORRUPT, "bad stream header");
  if (hny != ny_ || hnx != nx_ || ny_ < 1 || nx_ < 1) return fail(EBCC_EINVAL, "dimensions do not match the stream");
  int ny = (int)ny_, nx = (int)nx_;
  size_t N = (size_t)ny * nx;
  uint32_t bb = rd32(h + 36), rb = rd32(h + 40), csum = rd32(h + 44);
  if ((size_t)kHdr + bb + rb != in_len) return fail(EBCC_ECORRUPT, "stream length does not match its header");
  float xmin, range_f;
  memcpy(&xmin, h + 16, 4);
  memcpy(&range_f, h + 20, 4);
  int L = h[6], cbl2w = h[7] & 15, cbl2h = h[7] >> 4, T = h[32] | (h[33] << 8);
  int e0 = (int8_t)h[28], er = (int8_t)h[29], ns = (int8_t)h[31];
  if (mode == MODE_RAW && bb != 4 * N) return fail(EBCC_ECORRUPT, "raw stream of the wrong size");
  if (mode == MODE_CODED && (L != levels_eff(ny, nx, L) || cbl2w < 2 || cbl2w > 6 || cbl2h < 2 || cbl2h > 6 || T < 1 ||
                             T > 64 || ns < 0 || ns >= kQBits))
    return fail(EBCC_ECORRUPT, "bad coding parameters in the header");
  Plan* pl;
  int rc = get_plan(ny, nx, mode == MODE_CODED ? L : 0, mode == MODE_CODED ? cbl2w : 2, mode == MODE_CODED ? cbl2h : 2,
                    mode == MODE_CODED ? T : 1, &pl);
  if (rc) return rc;
  Bufs B;
  if ((rc = get_ws(*pl, st, &B))) return rc;
  Prof prof(st);
  k_set_decode_params<<<1, 1, 0, st>>>(B.fp, xmin, range_f, B.flags, 8);
  k_zero_int<<<1, 64, 0, st>>>((int*)B.u32s, 8);
  k_checksum<<<grid_for((in_len + 3) / 4), 256, 0, st>>>(in, nullptr, (int64_t)in_len, &B.u32s[1]);
  if (mode == MODE_CONST) {
    k_fill<<<grid_for(N), 256, 0, st>>>(x, (int)N, xmin);
  } else if (mode == MODE_RAW) {
    HIPCHK(hipMemcpyAsync(x, in + kHdr, 4 * N, hipMemcpyDeviceToDevice, st));
  } else {
    if ((int64_t)bb < 4 * (int64_t)pl->nblk) return fail(EBCC_ECORRUPT, "base section shorter than its table");
    const uint8_t* bsec = in + kHdr;
    DwtIO io{nullptr, B.abase, x, &B.flags[0], B.fp};
    k_read_table<<<grid_for(pl->nblk), 256, 0, st>>>(bsec, pl->nblk, B.bent);
    k_scan<<<1, 1024, 0, st>>>(B.bent, pl->nblk, 16, 0xFFFFu, B.boff, &B.totals[0]);
    k_check_tables<<<1, 64, 0, st>>>(bsec, pl->nblk, (int64_t)bb, &B.totals[0], &B.flags[1]);
    prof.mark(S_D_PARSE);
    t1_decode(bsec + 4 * (size_t)pl->nblk, (int64_t)bb - 4 * (int64_t)pl->nblk, B.bent, B.boff, nx, pl->d_blks,
              pl->nblk, e0, pl->cbw, pl->cbh, B.yhat, &B.flags[1], st);
    prof.mark(S_D_T1);
    if (rb) {
      dwt_inverse(B.yhat, B.tmp, B.abase, ny, nx, L, EPI_STORE, io, st);
      prof.mark(S_D_IDWT_BASE);
      if ((int64_t)rb < 4 * (int64_t)pl->ntiles) return fail(EBCC_ECORRUPT, "residual section shorter than its table");
      const uint8_t* rsec = bsec + bb;
      k_read_table<<<grid_for(pl->ntiles), 256, 0, st>>>(rsec, pl->ntiles, B.tent);
      k_scan<<<1, 1024, 0, st>>>(B.tent, pl->ntiles, 0, 0x3FFFFFFu, B.toff, &B.totals[1]);
      k_check_tables<<<1, 64, 0, st>>>(rsec, pl->ntiles, (int64_t)rb, &B.totals[1], &B.flags[1]);
      k_fill<<<grid_for(N), 256, 0, st>>>(B.chat, (int)N, 0.0f);
      // payload offsets relative to the residual section start
      if (spiht_cap_for(pl))
        spiht_decode_lds(spiht_cap_for(pl), rsec, (int64_t)rb, B.toff, nx, pl->d_bands, pl->nb, L, pl->d_tiles,
                         pl->ntiles, ns, er, B.chat, &B.flags[1], B.misfit, st);
      else
        spiht_decode(rsec, (int64_t)rb, B.toff, nx, pl->d_bands, pl->nb, L, pl->d_tiles, pl->ntiles, ns, er,
                     B.lists, B.qr, B.chat, &B.flags[1], st);
      prof.mark(S_D_SPIHT);
      dwt_inverse(B.chat, B.tmp, nullptr, ny, nx, L, EPI_FINAL, io, st);
      prof.mark(S_D_FINAL);
    } else {
      dwt_inverse(B.yhat, B.tmp, B.abase, ny, nx, L, EPI_STORE, io, st);
      prof.mark(S_D_IDWT_BASE);
      pointwise(nullptr, nullptr, (int)N, 3, EPI_FINAL, io, st);
      prof.mark(S_D_FINAL);
    }
  }
  HIPCHK(hipGetLastError());
  int fl[2];
  unsigned cs[2];
  if ((rc = d2h(fl, B.flags, 2, st))) return rc;
  if ((rc = d2h(cs, B.u32s, 2, st))) return rc;
  if (fl[1]) return fail(EBCC_ECORRUPT, "inconsistent block or tile tables");
  if (cs[1] != csum) return fail(EBCC_ECORRUPT, "checksum mismatch");
  return EBCC_OK;
}

}  // namespace ebcc

using namespace ebcc;

extern "C" {

void ebcc_params_default(ebcc_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(ebcc_params);
  p->bound_mode = EBCC_BOUND_REL;
  p->err_bound = 0.01;
  p->base_ratio = 30.0;
  p->q = 0.0;
  p->levels = 5;
  p->cblk_log2w = 5;
  p->cblk_log2h = 5;
  p->spiht_tile = 2;
}

size_t ebcc_compress_bound(size_t ny, size_t nx) { return (size_t)kHdr + 4 * ny * nx; }

int ebcc_compress(const float* d_x, size_t ny, size_t nx, const ebcc_params* p, uint8_t* d_out, size_t out_cap,
                  size_t* out_len, void* stream) {
  g_err.clear();
  return compress_impl(d_x, ny, nx, p, d_out, out_cap, out_len, (hipStream_t)stream, nullptr);
}

int ebcc_compress_trace(const float* d_x, size_t ny, size_t nx, const ebcc_params* p, uint8_t* d_out, size_t out_cap,
                        size_t* out_len, void* stream, float* d_coef, float* d_abase, float* d_cres, uint8_t* d_kb,
                        uint8_t* d_pb, int32_t* h_info) {
  g_err.clear();
  Trace tr{d_coef, d_abase, d_cres, d_kb, d_pb, h_info};
  return compress_impl(d_x, ny, nx, p, d_out, out_cap, out_len, (hipStream_t)stream, &tr);
}

int ebcc_decompress(const uint8_t* d_in, size_t in_len, float* d_x, size_t ny, size_t nx, void* stream) {
  g_err.clear();
  return decompress_impl(d_in, in_len, d_x, ny, nx, (hipStream_t)stream);
}

int ebcc_stream_info(const uint8_t* h, size_t len, size_t* ny, size_t* nx, int* mode) {
  if (!h || len < (size_t)kHdr || memcmp(h, "EBCC", 4) != 0 || h[4] != 1 || h[5] > MODE_CODED) return EBCC_ECORRUPT;
  if (ny) *ny = rd32(h + 8);
  if (nx) *nx = rd32(h + 12);
  if (mode) *mode = h[5];
  return EBCC_OK;
}

void ebcc_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  g_ws.clear();
  g_plans.clear();
}

const char* ebcc_status_str(int s) {
  switch (s) {
    case EBCC_OK: return "ok";
    case EBCC_EINVAL: return "invalid argument";
    case EBCC_ENOSPC: return "output buffer too small";
    case EBCC_ECORRUPT: return "corrupt stream";
    case EBCC_ENOMEM: return "out of device memory";
    case EBCC_EHIP: return "HIP runtime error";
    case EBCC_ENOTIMPL: return "not implemented";
    default: return "unknown status";
  }
}

const char* ebcc_last_error(void) { return g_err.c_str(); }

void ebcc_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof = on ? 1 : 0;
  for (int i = 0; i < S_COUNT; i++) { g_stage_ms[i] = 0.0; g_stage_calls[i] = 0; }
}

int ebcc_profile_read(double* ms, long* calls, int n) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < n && i < S_COUNT; i++) {
    if (ms) ms[i] = g_stage_ms[i];
    if (calls) calls[i] = g_stage_calls[i];
  }
  return S_COUNT;
}

const char* ebcc_profile_stage_name(int i) { return (i >= 0 && i < S_COUNT) ? kStageNames[i] : ""; }

}  // extern "C"
