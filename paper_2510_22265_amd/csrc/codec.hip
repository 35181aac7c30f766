// Host runtime and C ABI of libebcc.so: per-shape plans (subbands,
// code-blocks, SPIHT tiles), per-stream device workspaces, and the
// orchestration of the EBCC compression process (Algorithm 1 with a fixed
// base ratio and plane-granular truncation of the residual) and of
// decompression.  Also holds the small kernels of the path: min/max and
// field scalars, residual quantisation, reductions, scans, packing and the
// stream checksum.
#include "common.h"
#include "ebcc.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
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
// that just ended.  Off unless enabled.  A call only records its events
// (taken from a per-device pool) and queues them; they are read once the
// stream has passed them — at a later call, or in ebcc_profile_read, which
// waits for the outstanding ones — so profiling adds no synchronisation.
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
static std::mutex g_prof_mu;   // guards everything below and the accumulators

struct ProfRec {
  int dev;
  hipEvent_t first;
  std::vector<std::pair<int, hipEvent_t>> marks;
};
static std::vector<ProfRec> g_prof_pending;
static std::map<int, std::vector<hipEvent_t>> g_ev_pool;

static hipEvent_t pool_get(int dev) {
  std::vector<hipEvent_t>& p = g_ev_pool[dev];
  if (!p.empty()) {
    hipEvent_t e = p.back();
    p.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Adds the stage times of the queued calls the device has finished (all of
// them, waiting, when wait is set) and returns their events to the pool.
static void prof_resolve(bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < g_prof_pending.size(); i++) {
    ProfRec& r = g_prof_pending[i];
    hipEvent_t last = r.marks.empty() ? r.first : r.marks.back().second;
    if (wait) (void)hipEventSynchronize(last);
    else if (hipEventQuery(last) != hipSuccess) {
      if (keep != i) g_prof_pending[keep] = std::move(r);
      keep++;
      continue;
    }
    hipEvent_t a = r.first;
    for (auto& m : r.marks) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, a, m.second) == hipSuccess) {
        g_stage_ms[m.first] += ms;
        g_stage_calls[m.first] += 1;
      }
      a = m.second;
    }
    std::vector<hipEvent_t>& p = g_ev_pool[r.dev];
    p.push_back(r.first);
    for (auto& m : r.marks) p.push_back(m.second);
  }
  g_prof_pending.resize(keep);
}

struct Prof {
  hipStream_t st;
  bool on;
  ProfRec rec;
  explicit Prof(hipStream_t s, bool allowed = true) : st(s), on(allowed && g_prof != 0) {
    if (!on) return;
    rec.dev = 0;
    (void)hipGetDevice(&rec.dev);
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      rec.first = pool_get(rec.dev);
    }
    if (!rec.first || hipEventRecord(rec.first, st) != hipSuccess) on = false;
  }
  void mark(int stage) {
    if (!on) return;
    hipEvent_t e;
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      e = pool_get(rec.dev);
    }
    if (!e) return;
    if (hipEventRecord(e, st) != hipSuccess) {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_ev_pool[rec.dev].push_back(e);
      return;
    }
    rec.marks.push_back(std::make_pair(stage, e));
  }
  ~Prof() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(std::move(rec));
    prof_resolve(false);
  }
};


// ---------------------------------------------------------------------------
// Small kernels (every one takes the call's field table; field = blockIdx.y
// or one thread per field)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned f2o(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// Host-to-device copy through kernel arguments (the no-allocation entry
// point has no staging buffer): up to kArgChunk bytes per launch.
constexpr int kArgChunk = 2048;
struct ArgChunk {
  uint8_t b[kArgChunk];
};
__global__ __launch_bounds__(256) void k_put_bytes(uint8_t* __restrict__ dst, const ArgChunk c, int n) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = c.b[i];
}

// Stream headers of a decode batch gathered in one launch per kHdrArgs
// streams (their addresses travel as kernel arguments): workgroup i copies
// the 48 header bytes of stream i, or zeros for a stream shorter than a
// header, to out[48 i ..].
constexpr int kHdrArgs = 64;
struct HdrArgs {
  const uint8_t* p[kHdrArgs];
  int ok[kHdrArgs];
};
__global__ __launch_bounds__(64) void k_read_headers(const HdrArgs a, int n, uint8_t* __restrict__ out) {
  const int i = blockIdx.x, j = threadIdx.x;
  if (i < n && j < kHdr) out[kHdr * i + j] = a.ok[i] ? a.p[i][j] : (uint8_t)0;
}

__global__ void k_init_fields(const FieldDev* __restrict__ F, int nf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const FieldDev& f = F[i];
  f.fp->xmin_bits = 0xFFFFFFFFu;
  f.fp->xmax_bits = 0u;
  f.fp->nonfinite = 0;
  for (int k = 0; k < 8; k++) { f.flags[k] = 0; f.u32s[k] = 0; f.totals[k] = 0; }
}

// Block-wide reductions of 256 threads (the result is valid in thread 0);
// full-field sweeps make one atomic update per block.
__device__ __forceinline__ unsigned block_min(unsigned v, unsigned* sh) {
  for (int off = 32; off > 0; off >>= 1) { unsigned a = __shfl_xor(v, off); v = a < v ? a : v; }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < 4; k++) v = sh[k] < v ? sh[k] : v;
  return v;
}
__device__ __forceinline__ unsigned block_max(unsigned v, unsigned* sh) {
  for (int off = 32; off > 0; off >>= 1) { unsigned a = __shfl_xor(v, off); v = a > v ? a : v; }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < 4; k++) v = sh[k] > v ? sh[k] : v;
  return v;
}
__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) v = sh[0] + sh[1] + sh[2] + sh[3];
  return v;
}

__global__ __launch_bounds__(256) void k_minmax(const FieldDev* __restrict__ F) {
  __shared__ unsigned sh[4];
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx;
  const float* x = f.buf[BUF_X];
  unsigned mn = 0xFFFFFFFFu, mx = 0u, nf = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = x[i];
    if (!__builtin_isfinite(v)) { nf = 1; continue; }
    unsigned o = f2o(v);
    mn = o < mn ? o : mn;
    mx = o > mx ? o : mx;
  }
  mn = block_min(mn, sh);
  mx = block_max(mx, sh);
  nf = block_max(nf, sh);
  if (threadIdx.x == 0) {
    atomicMin(&f.fp->xmin_bits, mn);
    atomicMax(&f.fp->xmax_bits, mx);
    if (nf) atomicOr(&f.fp->nonfinite, 1);
  }
}

// Field scalars (range, bound, quantiser exponents) from min and max.
// eps is range-relative (Benchmarks section) or absolute.
__global__ void k_params(const FieldDev* __restrict__ F, int nfields) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields || !F[i].active) return;
  FieldParams* fp = F[i].fp;
  float xmin = o2f(fp->xmin_bits), xmax = o2f(fp->xmax_bits);
  if (xmin == 0.0f) xmin = 0.0f;   // +0 for a zero extreme
  if (xmax == 0.0f) xmax = 0.0f;
  fp->xmin = xmin;
  fp->xmax = xmax;
  double range_d = (double)xmax - (double)xmin;
  double eps = F[i].bound_mode == EBCC_BOUND_REL ? F[i].err * range_d : F[i].err;
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

// Decoder: header scalars into the field's parameters; flags cleared.
__global__ void k_set_decode(const FieldDev* __restrict__ F, int nfields, const float* __restrict__ xr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields) return;
  const FieldDev& f = F[i];
  f.fp->xmin = xr[2 * i];
  f.fp->range_f = xr[2 * i + 1];
  f.fp->inv_f = 0.0f;
  f.fp->eps = 0.0;
  for (int k = 0; k < 8; k++) { f.flags[k] = 0; f.u32s[k] = 0; f.totals[k] = 0; }
}

__global__ void k_zero_slot(const FieldDev* __restrict__ F, int nfields, int which) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields || !F[i].active) return;
  if (which == 0) F[i].flags[0] = 0;
  else if (which == 1) F[i].u32s[0] = 0;
  else F[i].u32s[2] = 0;
}

// Fill buf[which] with v (which = BUF_XOUT and v = NaN: fill with xmin).
__global__ __launch_bounds__(256) void k_fill(const FieldDev* __restrict__ F, int which, float v) {
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx;
  float val = (v != v) ? f.fp->xmin : v;
  float* p = f.buf[which];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = val;
}

// Residual quantisation q_r = floor(|c| * 2^-e_r) (capped), sign in bit 31.
__global__ __launch_bounds__(256) void k_quant_res(const FieldDev* __restrict__ F) {
  __shared__ unsigned sh[4];
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx, er = f.er;
  const float* c = f.buf[BUF_CRES];
  uint32_t* qr = f.qr;
  unsigned mx = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float v = c[i];
    uint32_t q = quantq(v, -er);
    qr[i] = q | (v < 0.0f ? 0x80000000u : 0u);
    mx = q > mx ? q : mx;
  }
  mx = block_max(mx, sh);
  if (threadIdx.x == 0 && mx) atomicMax(&f.u32s[0], mx);
}

// Residual coefficients kept by truncation at the end of plane n_s, midpoint
// reconstructed: what the SPIHT decoder recovers from planes n_max .. n_s.
__global__ __launch_bounds__(256) void k_dequant_res(const FieldDev* __restrict__ F) {
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx, ns = f.ns, er = f.er;
  const uint32_t* qr = f.qr;
  float* out = f.buf[BUF_CHAT];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    uint32_t v = qr[i], q = v & 0x7FFFFFu;
    uint32_t m = (q >> ns) << ns;
    out[i] = dequant(m, ns, (int)(v >> 31), er);
  }
}

// Small per-field results gathered for one device-to-host copy:
// violation flag, corruption flag, residual max, checksum, base and residual
// payload bytes, parameters mode.
__global__ void k_collect(const FieldDev* __restrict__ F, int nfields, int64_t* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields) return;
  const FieldDev& f = F[i];
  int64_t* o = out + 8 * i;
  o[0] = f.flags[0]; o[1] = f.flags[1]; o[2] = f.u32s[0]; o[3] = f.u32s[1];
  o[4] = f.totals[0]; o[5] = f.totals[1]; o[6] = f.u32s[2];
  o[7] = f.totals[2] | ((int64_t)(f.flags[2] & 1) << 48);   // PCRD payload, every segment fitted
}

// q_A of Algorithm 1's enc_base: samples whose base-layer reconstruction
// (zero residual, the decoder's arithmetic) is within eps, into u32s[2].
__global__ __launch_bounds__(256) void k_count_within(const FieldDev* __restrict__ F) {
  __shared__ unsigned sh[4];
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx;
  const float* x = f.buf[BUF_X];
  const float* ab = f.buf[BUF_ABASE];
  const float xmin = f.fp->xmin, range = f.fp->range_f;
  const double eps = f.fp->eps;
  unsigned cnt = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    float a = ab[i] + 0.0f;
    a = a + 0.5f;
    a = a * range;
    float xh = xmin + a;
    cnt += fabs((double)x[i] - (double)xh) <= eps ? 1u : 0u;
  }
  cnt = block_sum(cnt, sh);
  if (threadIdx.x == 0 && cnt) atomicAdd(&f.u32s[2], cnt);
}

// Exclusive scan of a field's 32-bit lengths (len = (v >> shift) & mask);
// which = 0: its code-blocks (total -> totals[0]), 1: its tiles (totals[1]).
__global__ __launch_bounds__(1024) void k_scan(const FieldDev* __restrict__ F, const uint32_t* __restrict__ v_g,
                                               int which, int shift, uint32_t mask, int64_t* __restrict__ off_g) {
  const FieldDev& f = F[blockIdx.x];
  if (!f.active) return;
  __shared__ int64_t part[1024];
  const int b0 = which ? f.tile0 : f.blk0;
  const int n = which ? f.ntiles : f.nblk;
  const uint32_t* v = v_g + b0;
  int64_t* off = off_g + b0;
  int tid = threadIdx.x;
  int per = (n + 1023) / 1024;
  int i0 = tid * per, i1 = i0 + per < n ? i0 + per : n;
  int64_t s = 0;
  for (int i = i0; i < i1; i++) s += (int64_t)((v[i] >> shift) & mask);
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t t = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += t;
    __syncthreads();
  }
  int64_t run = part[tid] - s;
  for (int i = i0; i < i1; i++) {
    off[i] = run;
    run += (int64_t)((v[i] >> shift) & mask);
  }
  if (tid == 1023) f.totals[which] = part[1023];
}

// Block table entries (P_b | k_b << 8 | len << 16) of the coded stream.
__global__ __launch_bounds__(256) void k_block_entries(const uint8_t* __restrict__ pb, const uint8_t* __restrict__ kb,
                                                       const int32_t* __restrict__ len, int nblk,
                                                       uint32_t* __restrict__ ent) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nblk; b += gridDim.x * 256)
    ent[b] = (uint32_t)pb[b] | ((uint32_t)kb[b] << 8) | ((uint32_t)len[b] << 16);
}

__device__ __forceinline__ void put32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
__device__ __forceinline__ uint32_t get32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// Block table of each field's stream.
__global__ __launch_bounds__(256) void k_put_blocks(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                    const uint32_t* __restrict__ ent, int nblk) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nblk; b += gridDim.x * 256) {
    const FieldDev& f = F[blk[b].field];
    if (!f.active) continue;
    put32(f.out + kHdr + 4 * (size_t)(b - f.blk0), ent[b]);
  }
}

// Terminated codewords: bytes before the termination point from the
// encoder's buffer, then the bytes the termination of pass k_b writes.  With
// the tier-1 bypass and k_b > 10: the raw byte count (u16), that MQ
// codeword (terminated after the last MQ-coded pass), then the raw bits of
// the bypassed passes from the buffer's raw area, the last byte's unused
// bits cleared.
__global__ __launch_bounds__(256) void k_gather_cw(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                   const uint8_t* __restrict__ cw, const uint8_t* __restrict__ kb,
                                                   const int32_t* __restrict__ len, const int32_t* __restrict__ bpt,
                                                   const uint32_t* __restrict__ tailt, const int32_t* __restrict__ rbt,
                                                   const int64_t* __restrict__ off, int nblk) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int b = blockIdx.x * 4 + wave; b < nblk; b += gridDim.x * 4) {
    const FieldDev& f = F[blk[b].field];
    int k = kb[b], n = len[b];
    if (!f.active || !k) continue;
    int bp = bpt[(size_t)b * kPassStride + k];
    uint32_t tl = tailt[(size_t)b * kPassStride + k];
    const uint8_t* src = cw + (size_t)b * kCwCap;
    uint8_t* dst = f.out + kHdr + 4 * (size_t)f.nblk + off[b];
    if (f.byp && k >= kBypFirst) {
      const int rbits = rbt[(size_t)b * kPassStride + k], rby = (rbits + 7) >> 3, nmq = n - 2 - rby;
      const uint8_t lastm = (uint8_t)(0xFF << ((8 - (rbits & 7)) & 7));
      for (int j = lane; j < n; j += 64) {
        uint8_t v;
        if (j < 2) v = (uint8_t)(rby >> (8 * j));
        else if (j < 2 + nmq) v = j - 2 < bp ? src[j - 2] : (uint8_t)(tl >> (8 * (j - 2 - bp)));
        else v = src[kRawOff + (j - 2 - nmq)] & (j == n - 1 ? lastm : (uint8_t)0xFF);
        dst[j] = v;
      }
      continue;
    }
    for (int j = lane; j < n; j += 64) dst[j] = j < bp ? src[j] : (uint8_t)(tl >> (8 * (j - bp)));
  }
}

// Tile table and tile payloads of each field with a residual section.
__global__ __launch_bounds__(256) void k_put_tiles(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                   const uint32_t* __restrict__ tent, int nt) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
    const FieldDev& f = F[tiles[t].field];
    if (!f.active || f.rb == 0) continue;
    put32(f.out + kHdr + f.bb + 4 * (size_t)(t - f.tile0), tent[t]);
    if (f.bt && t == f.tile0) {   // a byte-cut residual ends with its cut
      uint8_t* tr = f.out + kHdr + f.bb + f.rb - 8;
      put32(tr, (uint32_t)f.cut_tile | ((uint32_t)f.cut_kind << 31));
      put32(tr + 4, f.cut_bits);
    }
  }
}
__global__ __launch_bounds__(256) void k_gather_tiles(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                      const uint8_t* __restrict__ slots,
                                                      const int64_t* __restrict__ slot_off,
                                                      const uint32_t* __restrict__ tlen,
                                                      const uint32_t* __restrict__ tbits,
                                                      const int64_t* __restrict__ off, int nt) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = blockIdx.x * 4 + wave; t < nt; t += gridDim.x * 4) {
    const FieldDev& f = F[tiles[t].field];
    if (!f.active || f.rb == 0) continue;
    int64_t cap = slot_off[t + 1] - slot_off[t];
    int n = (int)((int64_t)tlen[t] < cap ? (int64_t)tlen[t] : cap);
    const uint8_t* src = slots + slot_off[t];
    uint8_t* dst = f.out + kHdr + f.bb + 4 * (size_t)f.ntiles + off[t];
    // a code cut inside a byte keeps that byte's leading bits only
    const int tail = f.bt ? (int)(tbits[t] & 7u) : 0;
    for (int j = lane; j < n; j += 64) {
      uint8_t v = src[j];
      if (tail && j == n - 1) v &= (uint8_t)(0xFFu << (8 - tail));
      dst[j] = v;
    }
  }
}

// Raw streams: the field's samples after the header.
__global__ __launch_bounds__(256) void k_copy_raw(const FieldDev* __restrict__ F, int to_stream) {
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int n = f.ny * f.nx;
  uint32_t* s = reinterpret_cast<uint32_t*>(f.out + kHdr);
  float* x = f.buf[to_stream ? BUF_X : BUF_XOUT];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    if (to_stream) put32(f.out + kHdr + 4 * (size_t)i, __float_as_uint(x[i]));
    else x[i] = __uint_as_float(get32(f.out + kHdr + 4 * (size_t)i));
  }
  (void)s;
}

// Stream checksum: sum over the little-endian 32-bit words w_k of the bytes
// after the header (zero padded) of w_k * (2k + 1), modulo 2^32.
__global__ __launch_bounds__(256) void k_checksum(const FieldDev* __restrict__ F) {
  __shared__ unsigned sh[4];
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  int64_t n = f.len - kHdr;
  const uint8_t* q = f.out + kHdr;
  int64_t nw = (n + 3) / 4;
  unsigned s = 0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nw; k += (int64_t)gridDim.x * 256) {
    uint32_t w = 0;
    for (int b = 0; b < 4; b++)
      if (4 * k + b < n) w |= (uint32_t)q[4 * k + b] << (8 * b);
    s += w * (uint32_t)(2 * k + 1);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) atomicAdd(&f.u32s[1], s);
}

__global__ void k_header(const FieldDev* __restrict__ F, int nfields) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields || !F[i].active) return;
  const FieldDev& f = F[i];
  uint8_t* o = f.out;
  const int mode = f.mode;
  for (int k = 0; k < kHdr; k++) o[k] = 0;
  o[0] = 'E'; o[1] = 'B'; o[2] = 'C'; o[3] = 'C';
  o[4] = 1; o[5] = (uint8_t)mode; o[6] = (uint8_t)(mode == MODE_CODED ? f.L : 0); o[7] = (uint8_t)f.cbl;
  put32(o + 8, (uint32_t)f.ny);
  put32(o + 12, (uint32_t)f.nx);
  put32(o + 16, __float_as_uint(f.fp->xmin));
  put32(o + 20, __float_as_uint(mode == MODE_CONST ? 0.0f : f.fp->range_f));
  put32(o + 24, __float_as_uint(mode == MODE_CONST ? 0.0f : f.fp->inv_f));
  o[28] = (uint8_t)(int8_t)(mode == MODE_CODED ? f.e0 : 0);
  o[29] = (uint8_t)(int8_t)(mode == MODE_CODED && f.rb ? f.er : 0);
  o[30] = (uint8_t)(int8_t)(mode == MODE_CODED && f.rb ? f.nmax : -1);
  o[31] = (uint8_t)(int8_t)(mode == MODE_CODED && f.rb ? f.ns : 0);
  o[32] = (uint8_t)f.T; o[33] = (uint8_t)(f.T >> 8);
  o[34] = (uint8_t)(mode == MODE_CODED && f.rb && f.bt ? 1 : 0);   // residual cut at a byte position
  o[35] = (uint8_t)(mode == MODE_CODED && f.byp ? 1 : 0);           // tier-1 arithmetic-coding bypass
  put32(o + 36, f.bb);
  put32(o + 40, f.rb);
  put32(o + 44, f.u32s[1]);
}

// Decoder: table entries and consistency of the block and tile tables.
__global__ __launch_bounds__(256) void k_read_blocks(const FieldDev* __restrict__ F, const Blk* __restrict__ blk, int nblk,
                                                     uint32_t* __restrict__ ent) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b < nblk; b += gridDim.x * 256) {
    const FieldDev& f = F[blk[b].field];
    ent[b] = f.active ? get32(f.out + kHdr + 4 * (size_t)(b - f.blk0)) : 0u;
  }
}
__global__ __launch_bounds__(256) void k_read_tiles(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                    int nt, uint32_t* __restrict__ ent) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
    const FieldDev& f = F[tiles[t].field];
    ent[t] = (f.active && f.rb) ? get32(f.out + kHdr + f.bb + 4 * (size_t)(t - f.tile0)) : 0u;
  }
}
__global__ void k_check_tables(const FieldDev* __restrict__ F, int nfields) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfields || !F[i].active) return;
  const FieldDev& f = F[i];
  if (f.totals[0] != (int64_t)f.bb - 4 * (int64_t)f.nblk) f.flags[1] = 1;
  if (f.rb && f.totals[1] != (int64_t)f.rb - 4 * (int64_t)f.ntiles - (f.bt ? 8 : 0)) f.flags[1] = 1;
}

// Asynchronous decoding: the host knows each stream's shape and the coding
// parameters of the call, not the stream's bytes.  One thread per stream
// checks the header (the host decoder's checks, plus agreement with the
// call's parameters), sets the field's scalars and its entries in the
// residual (Fr, scratch of the residual's inverse DWT in BUF_CRES) and
// no-residual (Fn) tables, and writes the stream's status.
struct AsyncCfg {
  int cbl, T, trunc, byp;
};

__device__ int levels_eff_dev(int ny, int nx, int L) {
  int m = ny < nx ? ny : nx, f = 0;
  while ((2L << f) <= m) f++;
  if (L > f) L = f;
  if (L > kMaxLevels) L = kMaxLevels;
  return L < 0 ? 0 : L;
}

__global__ void k_parse_async(FieldDev* __restrict__ F, FieldDev* __restrict__ Fr, FieldDev* __restrict__ Fn, int nf,
                              const uint8_t* __restrict__ in, const uint64_t* __restrict__ offs,
                              const uint64_t* __restrict__ lens, const AsyncCfg cfg, int32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  FieldDev f = F[i];
  const uint64_t len = lens[i];
  const uint8_t* h = in + offs[i];
  const int64_t N = (int64_t)f.ny * f.nx;
  int st = EBCC_OK, mode = MODE_CONST, bt = 0, byp = 0, e0 = 0, er = 0, ns = 0;
  uint32_t bb = 0, rb = 0;
  if (len < (uint64_t)kHdr) {
    st = EBCC_ECORRUPT;
  } else if (h[0] != 'E' || h[1] != 'B' || h[2] != 'C' || h[3] != 'C' || h[4] != 1 || h[5] > MODE_CODED) {
    st = EBCC_ECORRUPT;
  } else if (get32(h + 8) != (uint32_t)f.ny || get32(h + 12) != (uint32_t)f.nx) {
    st = EBCC_EINVAL;
  } else {
    mode = h[5];
    bb = get32(h + 36);
    rb = get32(h + 40);
    if ((uint64_t)kHdr + bb + rb != len) {
      st = EBCC_ECORRUPT;
    } else if (mode == MODE_RAW && (int64_t)bb != 4 * N) {
      st = EBCC_ECORRUPT;
    } else if (mode == MODE_CODED) {
      const int L = h[6], w2 = h[7] & 15, h2 = h[7] >> 4, T = h[32] | (h[33] << 8);
      e0 = (int8_t)h[28];
      er = (int8_t)h[29];
      ns = (int8_t)h[31];
      if (L != levels_eff_dev(f.ny, f.nx, L) || w2 < 2 || w2 > 6 || h2 < 2 || h2 > 6 || T < 1 || T > 64 || ns < 0 ||
          ns >= kQBits) {
        st = EBCC_ECORRUPT;
      } else {
        bt = rb ? (h[34] & 1) : 0;
        byp = h[35] & 1;
        if (L != f.L || h[7] != cfg.cbl || T != cfg.T || (bt && !cfg.trunc) || (byp && !cfg.byp))
          st = EBCC_EINVAL;   // coded with other parameters than the call's
        else if ((int64_t)bb < 4 * (int64_t)f.nblk)
          st = EBCC_ECORRUPT;
        else if (rb && (int64_t)rb < 4 * (int64_t)f.ntiles + (bt ? 8 : 0))
          st = EBCC_ECORRUPT;
      }
    }
  }
  const bool ok = st == EBCC_OK;
  f.out = const_cast<uint8_t*>(h);
  f.len = (int64_t)len;
  f.mode = mode;
  f.bb = bb; f.rb = rb;
  f.e0 = e0; f.er = er; f.ns = ns;
  f.bt = bt; f.byp = byp;
  f.active = ok ? 1 : 0;
  f.fp->xmin = ok ? __uint_as_float(get32(h + 16)) : 0.0f;
  f.fp->range_f = ok ? __uint_as_float(get32(h + 20)) : 0.0f;
  f.fp->inv_f = 0.0f;
  f.fp->eps = 0.0;
  for (int k = 0; k < 8; k++) { f.flags[k] = 0; f.u32s[k] = 0; f.totals[k] = 0; }
  F[i] = f;
  FieldDev r = f;
  r.active = ok && mode == MODE_CODED && rb != 0;
  r.buf[BUF_TMP] = r.buf[BUF_CRES];
  Fr[i] = r;
  FieldDev q = f;
  q.active = ok && mode == MODE_CODED && rb == 0;
  Fn[i] = q;
  status[i] = st;
}

// Asynchronous decoding: the fields of one role (a stream mode; mode < 0:
// every stream whose header passed) active, the others not.
__global__ void k_select_async(FieldDev* __restrict__ F, int nf, const int32_t* __restrict__ status, int mode) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  F[i].active = status[i] == EBCC_OK && (mode < 0 || F[i].mode == mode);
}

// Asynchronous decoding: a stream whose tables are inconsistent or whose
// checksum differs from its header's is corrupt.
__global__ void k_finish_async(const FieldDev* __restrict__ F, int nf, int32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf || status[i] != EBCC_OK) return;
  const FieldDev& f = F[i];
  if (f.flags[1]) status[i] = EBCC_ECORRUPT;
  else if (f.u32s[1] != get32(f.out + 44)) status[i] = EBCC_ECORRUPT;
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
  // tile indices grouped by SPIHT kernel class: LDS small, LDS big, global
  std::vector<int> tix;
  int ncls[4] = {0, 0, 0, 0};   // small, big, global lists, huge
  int* d_tix = nullptr;
  ~Plan() {
    if (d_bands) (void)hipFree(d_bands);
    if (d_blks) (void)hipFree(d_blks);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_slot_off) (void)hipFree(d_slot_off);
    if (d_tix) (void)hipFree(d_tix);
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
        p.blks.push_back(Blk{b.y0 + by, b.x0 + bx, std::min(p.cbw, b.w - bx), std::min(p.cbh, b.h - by), b.orient, b.gain, 0});
  p.nblk = (int)p.blks.size();
  // SPIHT tiles: T x T LL roots and the rectangles their trees cover per band
  int hL = h[L], wL = w[L], T = p.T;
  int ty = (hL + T - 1) / T, tx = (wL + T - 1) / T;
  std::vector<int> tcls;
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
      int64_t need = std::max<int64_t>(n, 4 * (L > 0 ? n - n1 : 0));
      tcls.push_back(need <= kSpihtSmall ? 0 : (need <= kSpihtBig ? 1 : (need <= kSpihtHuge ? 3 : 2)));
      t.field = 0;
      off += n;
      soff += 12 * n + 16;
      p.tiles.push_back(t);
      p.slot_off.push_back(soff);
    }
  p.ntiles = (int)p.tiles.size();
  for (int k = 0; k < 4; k++)
    for (int t = 0; t < p.ntiles; t++)
      if (tcls[t] == k) { p.tix.push_back(t); p.ncls[k]++; }
  if (off != (int64_t)ny * nx) return fail(EBCC_EINVAL, "internal: SPIHT trees do not cover the field");
  return EBCC_OK;
}

// Device bytes of a plan's tables.
static size_t plan_table_bytes(const Plan& p) {
  auto r = [](size_t n) { return (n + 255) & ~(size_t)255; };
  return r(sizeof(Band) * p.bands.size()) + r(sizeof(Blk) * std::max<size_t>(1, p.blks.size())) +
         r(sizeof(TileD) * p.tiles.size()) + r(sizeof(int) * p.tix.size()) + r(sizeof(int64_t) * p.slot_off.size());
}

static int upload_plan(Plan& p) {
  HIPCHK(hipMalloc(&p.d_bands, sizeof(Band) * p.bands.size()));
  HIPCHK(hipMemcpy(p.d_bands, p.bands.data(), sizeof(Band) * p.bands.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_blks, sizeof(Blk) * std::max<size_t>(1, p.blks.size())));
  if (p.nblk) HIPCHK(hipMemcpy(p.d_blks, p.blks.data(), sizeof(Blk) * p.blks.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_tiles, sizeof(TileD) * p.tiles.size()));
  HIPCHK(hipMemcpy(p.d_tiles, p.tiles.data(), sizeof(TileD) * p.tiles.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_tix, sizeof(int) * p.tix.size()));
  HIPCHK(hipMemcpy(p.d_tix, p.tix.data(), sizeof(int) * p.tix.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&p.d_slot_off, sizeof(int64_t) * p.slot_off.size()));
  HIPCHK(hipMemcpy(p.d_slot_off, p.slot_off.data(), sizeof(int64_t) * p.slot_off.size(), hipMemcpyHostToDevice));
  return EBCC_OK;
}

// SPIHT kernels: tiles that fit run with the tile in LDS, the others with
// global-memory lists; the environment variable EBCC_SPIHT_KERNEL=global
// sends every tile to the global-memory kernels (to test both families).
static std::mutex g_tune_mu;
static Tuning g_tuning = {0, 0, 32768, 0, 0, 10, 1};

Tuning tuning() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tuning;
}

static bool spiht_forced_global() {
  const char* e = getenv("EBCC_SPIHT_KERNEL");
  if (e && e[0]) return e[0] == 'g';
  return tuning().spiht == 1;
}

static std::mutex g_mu;
typedef std::tuple<int, int, int, int, int, int, int> PlanKey;   // device, ny, nx, L, cbl2w, cbl2h, T
static std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

// Host-only plans (geometry without device tables) for the size queries.
static std::map<PlanKey, std::unique_ptr<Plan>> g_hplans;
static int host_plan(int ny, int nx, int L, int cbl2w, int cbl2h, int T, Plan** out) {
  PlanKey key(-1, ny, nx, L, cbl2w, cbl2h, T);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_hplans.find(key);
  if (it != g_hplans.end()) { *out = it->second.get(); return EBCC_OK; }
  std::unique_ptr<Plan> p(new Plan());
  p->ny = ny; p->nx = nx; p->L = L; p->cbl2w = cbl2w; p->cbl2h = cbl2h;
  p->cbw = 1 << cbl2w; p->cbh = 1 << cbl2h; p->T = T;
  if (int rc = build_plan(*p)) return rc;
  *out = p.get();
  if (g_hplans.size() > 4096) g_hplans.clear();
  g_hplans[key] = std::move(p);
  return EBCC_OK;
}

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
  if (!rc) rc = upload_plan(*p);
  if (rc) return rc;
  *out = p.get();
  g_plans[key] = std::move(p);
  return EBCC_OK;
}


// ---------------------------------------------------------------------------
// Workspaces: one device allocation per (device, stream), carved per call.
// ---------------------------------------------------------------------------
// Host-to-device copies of a call go through the workspace's pinned staging
// buffer (the host source of an asynchronous copy must outlive it); the
// event recorded at the end of each call guards the buffer's reuse.
// Waits until everything queued on st has finished by polling an event.  A
// blocking synchronisation wakes the host thread tens of microseconds after
// the device is done, and a call makes several such round trips (header
// reads, search rounds, size tables).  One event per device and host thread.
static hipEvent_t sync_event() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  static thread_local std::map<int, hipEvent_t> evs;
  auto it = evs.find(dev);
  if (it != evs.end()) return it->second;
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  evs[dev] = e;
  return e;
}
static int wait_stream(hipStream_t st) {
  hipEvent_t ev = sync_event();
  if (!ev || hipEventRecord(ev, st) != hipSuccess) {
    HIPCHK(hipStreamSynchronize(st));
    return EBCC_OK;
  }
  // Poll for short waits (the common case: a few scalars after a short
  // launch sequence), then give the core away: yield for a few
  // milliseconds, sleep in 50 us steps beyond that.
  hipError_t e;
  const auto t0 = std::chrono::steady_clock::now();
  while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    const auto dt = std::chrono::steady_clock::now() - t0;
    if (dt < std::chrono::microseconds(200)) continue;
    if (dt < std::chrono::milliseconds(5)) std::this_thread::yield();
    else std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  if (e != hipSuccess) return fail(EBCC_EHIP, std::string("waiting for the stream: ") + hipGetErrorString(e));
  return EBCC_OK;
}

struct WS {
  void* base = nullptr;
  size_t cap = 0;
  // a workspace over the static scratch array: no pinned staging buffer, no
  // events, no extra streams; every wait is a stream synchronisation
  bool fixed = false;
  uint8_t* pin = nullptr;
  size_t pin_cap = 0;
  hipEvent_t ev = nullptr;
  bool ev_live = false;
  // second and third streams for independent launches of one call (SPIHT
  // tile classes), ordered against the caller's stream with events
  hipStream_t aux = nullptr, aux2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  // stream on which launch sequences are recorded into graphs (recording
  // runs nothing; the graph is then launched on the caller's stream)
  hipStream_t capst = nullptr;
  // pinned staging areas of the asynchronous decoder: an area is reused only
  // once the copies staged from it have run (its event), so a call returns
  // without waiting for the ones before it
  struct APin {
    uint8_t* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool live = false;
  };
  static constexpr int kAPins = 4;
  APin apin[kAPins];
  ~WS() {
    if (fixed) return;
    for (APin& a : apin) {
      if (a.live) (void)hipEventSynchronize(a.ev);
      if (a.p) (void)hipHostFree(a.p);
      if (a.ev) (void)hipEventDestroy(a.ev);
    }
    if (ev_live) (void)hipEventSynchronize(ev);
    if (base) (void)hipFree(base);
    if (pin) (void)hipHostFree(pin);
    if (ev) (void)hipEventDestroy(ev);
    if (aux) (void)hipStreamDestroy(aux);
    if (aux2) (void)hipStreamDestroy(aux2);
    if (capst) (void)hipStreamDestroy(capst);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_join2) (void)hipEventDestroy(ev_join2);
  }
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

static int get_ws(hipStream_t st, WS** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  std::unique_ptr<WS>& w = g_ws[WSKey(dev, st)];
  if (!w) {
    w.reset(new WS());
    HIPCHK(hipEventCreateWithFlags(&w->ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&w->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&w->ev_join, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&w->ev_join2, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&w->aux2, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&w->capst, hipStreamNonBlocking));
  }
  // the previous call's staged copies must have left the pinned buffer
  if (w->ev_live) HIPCHK(hipEventSynchronize(w->ev));
  w->ev_live = false;
  *out = w.get();
  return EBCC_OK;
}

// Device bytes grow_ws allocates for a workspace need (it keeps 1/8 slack).
static size_t ws_alloc(size_t need) { return need + need / 8; }

static int grow_ws(WS* w, size_t need, size_t pin_need, hipStream_t st, char** base) {
  if (w->pin_cap < pin_need) {
    if (w->pin) HIPCHK(hipHostFree(w->pin));
    w->pin = nullptr;
    w->pin_cap = 0;
    size_t alloc = std::max<size_t>(pin_need, 1 << 20);
    if (hipHostMalloc((void**)&w->pin, alloc, hipHostMallocDefault) != hipSuccess) {
      w->pin = nullptr;
      return fail(EBCC_ENOMEM, "pinned staging allocation failed");
    }
    w->pin_cap = alloc;
  }
  if (w->cap < need) {
    if (w->base) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(w->base));
      w->base = nullptr;
      w->cap = 0;
    }
    size_t alloc = ws_alloc(need);
    hipError_t e = hipMalloc(&w->base, alloc);
    if (e != hipSuccess) { w->base = nullptr; return fail(EBCC_ENOMEM, "workspace allocation failed"); }
    w->cap = alloc;
  }
  *base = (char*)w->base;
  return EBCC_OK;
}

// An asynchronous call's staging area of at least need bytes: one whose
// copies have run (waiting for the oldest when all are in flight), grown
// when too small.
static int async_pin(WS* w, size_t need, WS::APin** out) {
  for (int pass = 0; pass < 2; pass++) {
    for (WS::APin& a : w->apin) {
      if (a.live) {
        const hipError_t q = pass ? hipEventSynchronize(a.ev) : hipEventQuery(a.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(EBCC_EHIP, std::string("staging area event: ") + hipGetErrorString(q));
        a.live = false;
      }
      if (a.cap < need) {
        if (a.p) HIPCHK(hipHostFree(a.p));
        a.p = nullptr;
        a.cap = 0;
        const size_t alloc = std::max<size_t>(need, 1 << 20);
        if (hipHostMalloc((void**)&a.p, alloc, hipHostMallocDefault) != hipSuccess) {
          a.p = nullptr;
          return fail(EBCC_ENOMEM, "pinned staging allocation failed");
        }
        a.cap = alloc;
      }
      if (!a.ev) HIPCHK(hipEventCreateWithFlags(&a.ev, hipEventDisableTiming));
      *out = &a;
      return EBCC_OK;
    }
  }
  return fail(EBCC_EHIP, "internal: no staging area");
}

// Batches are processed in chunks of at most this many samples or fields.
constexpr size_t kChunkSamples = size_t(1) << 27;
constexpr int kChunkFields = 4096;

// Base payload budget for ratio r: header + block table + codewords fit
// floor(4 N / r) bytes (Algorithm 1's compression ratio r).
static int64_t base_budget(int64_t N, int64_t nblk, double r) {
  int64_t t = (int64_t)std::floor((double)(4 * N) / r) - kHdr - 4 * nblk;
  return t < 0 ? 0 : t;
}

// Full-field sweeps that reduce: about 16 elements per thread, at most 1024
// blocks per field.
static int grid_sweep(size_t n) {
  size_t g = (n + 4095) / 4096;
  if (g > 1024) g = 1024;
  return g < 1 ? 1 : (int)g;
}

static int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  return g < 1 ? 1 : (int)g;
}

static int check_params(size_t ny, size_t nx, const ebcc_params* p, double err) {
  if (ny < 1 || nx < 1 || ny > (1u << 24) || nx > (1u << 24) || ny * nx > 0x7FFFFFFFull)
    return fail(EBCC_EINVAL, "field dimensions out of range");
  if (p->struct_size != sizeof(ebcc_params)) return fail(EBCC_EINVAL, "ebcc_params.struct_size mismatch");
  if (!(err > 0) || !std::isfinite(err)) return fail(EBCC_EINVAL, "err_bound must be > 0 and finite");
  if (p->bound_mode > 1) return fail(EBCC_EINVAL, "bad bound_mode");
  if (!(p->base_ratio >= 1.0) || !std::isfinite(p->base_ratio)) return fail(EBCC_EINVAL, "base_ratio must be >= 1");
  if (p->levels > (unsigned)kMaxLevels) return fail(EBCC_EINVAL, "levels out of range");
  if (p->cblk_log2w < 2 || p->cblk_log2w > 6 || p->cblk_log2h < 2 || p->cblk_log2h > 6)
    return fail(EBCC_EINVAL, "code-block size out of range");
  if (p->spiht_tile < 1 || p->spiht_tile > 64) return fail(EBCC_EINVAL, "spiht_tile out of range");
  if (!(p->q >= 0.0 && p->q <= 1.0)) return fail(EBCC_EINVAL, "q must be 0 (fixed base ratio) or in (0, 1]");
  if (p->trunc > 1) return fail(EBCC_EINVAL, "trunc must be 0 (bit-plane ends) or 1 (byte positions)");
  if (p->bypass > 1) return fail(EBCC_EINVAL, "bypass must be 0 (every pass MQ coded) or 1 (raw passes after ten)");
  return EBCC_OK;
}

struct Trace {
  float *coef, *abase, *cres;
  uint8_t *kb, *pb;
  int32_t* info;
};

// One call over nf fields: the field table (host copy and device copy), the
// concatenated code-blocks and tiles of the coded fields, and the carved
// workspace.
struct Call {
  int nf = 0;
  hipStream_t st = nullptr;
  WS* ws = nullptr;
  size_t pin_used = 0;
  FieldParams* d_fp = nullptr;   // the fields' scalars, contiguous
  std::vector<FieldDev> Fh;
  std::vector<Plan*> plans;
  FieldDev* F = nullptr;
  // items of the coded fields
  int nblk = 0, ntiles = 0;
  const Blk* d_blk = nullptr;
  const TileD* d_tiles = nullptr;
  const int64_t* d_slot_off = nullptr;
  bool need_lists = false, forced_global = false;
  int cbw = 32, cbh = 32;
  const int* d_tix = nullptr;   // tile indices by class (see Plan::tix)
  int ncls[4] = {0, 0, 0, 0};
  // per-item arrays
  void *planes, *signs, *sppf;
  uint8_t *pb, *kb, *hk, *nh, *cw, *slots;
  int32_t *R, *bpt, *dr, *len;
  int64_t *D, *boff, *toff, *collect;
  uint64_t *keys, *lists;
  uint32_t *tail, *tlen, *tent, *bent;
  uint32_t *tcut, *tbits;   // byte-cut residuals: per tile bit counts around plane ns, final code bits
  int *border, *qctr;       // persistent tier-1 launches: block order and work counter
  int* tix_sorted;          // decoding: the LDS classes' tiles, longest payload first
  bool want_cpos = false;   // compression with byte-cut residuals: every coded field gets a cpos plane
  bool any_byp = false;     // some field's tier-1 passes use the arithmetic-coding bypass
  int32_t* rbt = nullptr;   // compression with the bypass: raw bits per block and pass
  int* misfit;
  Blk* d_blk_own;
  TileD* d_tiles_own;
  int64_t* d_slot_own;
  int* d_tix_own;
  // truncation-search candidates: a table of candidate entries (a field with
  // one truncation point each), their violation flags and, when the search
  // evaluates two bisection levels per round, three extra pairs of
  // residual/scratch planes per field
  int spec_depth = 1;
  FieldDev* Fc = nullptr;
  int* cand_flags = nullptr;
  std::vector<float*> cand_buf;   // per field: CHAT and TMP planes of the extra candidates, or none
  // plans without device tables (the no-allocation entry point): the
  // fields' subband tables are carved from the workspace and staged
  bool own_bands = false;
  Band* d_bands_own = nullptr;
  // asynchronous calls stage through an area of their own (WS::apin)
  WS::APin* apin = nullptr;
  size_t apin_used = 0;

  ~Call() {
    if (apin) {   // (normally marked right after the staging)
      if (!apin->live && hipEventRecord(apin->ev, st) == hipSuccess) apin->live = true;
      return;
    }
    if (ws && ws->ev && hipEventRecord(ws->ev, st) == hipSuccess) ws->ev_live = true;
  }
  int wait() {
    if (ws && ws->fixed) {
      HIPCHK(hipStreamSynchronize(st));
      return EBCC_OK;
    }
    return wait_stream(st);
  }
  // Asynchronous host-to-device copy through the pinned staging buffer.  A
  // fixed workspace has none: the bytes travel as kernel arguments, which
  // the launch copies, so the host source is free again when it returns.
  int stage(void* dst, const void* src, size_t n) {
    if (!n) return EBCC_OK;
    if (ws->fixed) {
      ArgChunk ch;
      for (size_t o = 0; o < n; o += kArgChunk) {
        const int m = (int)std::min<size_t>(kArgChunk, n - o);
        memcpy(ch.b, (const uint8_t*)src + o, m);
        k_put_bytes<<<1, 256, 0, st>>>((uint8_t*)dst + o, ch, m);
      }
      HIPCHK(hipGetLastError());
      return EBCC_OK;
    }
    if (apin) {
      const size_t a = (apin_used + 255) & ~(size_t)255;
      if (a + n > apin->cap) return fail(EBCC_ENOMEM, "internal: staging area smaller than the call's tables");
      memcpy(apin->p + a, src, n);
      HIPCHK(hipMemcpyAsync(dst, apin->p + a, n, hipMemcpyHostToDevice, st));
      apin_used = a + n;
      return EBCC_OK;
    }
    if (n > ws->pin_cap) return fail(EBCC_ENOMEM, "staging buffer smaller than a table");
    size_t a = (pin_used + 255) & ~(size_t)255;
    if (a + n > ws->pin_cap) {
      if (int rc = wait()) return rc;
      a = 0;
    }
    memcpy(ws->pin + a, src, n);
    HIPCHK(hipMemcpyAsync(dst, ws->pin + a, n, hipMemcpyHostToDevice, st));
    pin_used = a + n;
    return EBCC_OK;
  }
  // Device-to-host copy and synchronisation (the staging buffer is free again).
  template <typename T> int fetch(T* h, const T* d, size_t n) {
    HIPCHK(hipMemcpyAsync(h, d, sizeof(T) * n, hipMemcpyDeviceToHost, st));
    if (int rc = wait()) return rc;
    pin_used = 0;
    return EBCC_OK;
  }
  int upload() { return stage(F, Fh.data(), sizeof(FieldDev) * nf); }   // field table host -> device
  int max_nblk() const {   // code-blocks of the largest field of the call
    int m = 0;
    for (int i = 0; i < nf; i++) m = std::max(m, Fh[i].nblk);
    return m;
  }
  // Work launched on ws->aux and ws->aux2 between fork() and join() runs
  // concurrently with the caller's stream and is complete, for that stream,
  // after join().
  // Without extra streams (fixed workspace) everything runs on the caller's.
  hipStream_t aux_or(hipStream_t s) const { return ws->aux ? s : st; }
  int fork() { return fork_from(st); }
  int join() { return join_to(st); }
  // main: the stream the launches of the sequence go to (the caller's, or
  // the workspace's capture stream while a graph is recorded)
  int fork_from(hipStream_t main) {
    if (!ws->aux) return EBCC_OK;
    HIPCHK(hipEventRecord(ws->ev_fork, main));
    HIPCHK(hipStreamWaitEvent(ws->aux, ws->ev_fork, 0));
    HIPCHK(hipStreamWaitEvent(ws->aux2, ws->ev_fork, 0));
    return EBCC_OK;
  }
  int join_to(hipStream_t main) {
    if (!ws->aux) return EBCC_OK;
    HIPCHK(hipEventRecord(ws->ev_join, ws->aux));
    HIPCHK(hipEventRecord(ws->ev_join2, ws->aux2));
    HIPCHK(hipStreamWaitEvent(main, ws->ev_join, 0));
    HIPCHK(hipStreamWaitEvent(main, ws->ev_join2, 0));
    return EBCC_OK;
  }
  int set_active(const std::vector<int>& act) {
    for (int i = 0; i < nf; i++) Fh[i].active = act[i];
    return upload();
  }
  int collect_host(std::vector<int64_t>& v) {
    k_collect<<<(nf + 63) / 64, 64, 0, st>>>(F, nf, collect);
    HIPCHK(hipGetLastError());
    v.resize(8 * (size_t)nf);
    return fetch(v.data(), collect, v.size());
  }
};

// ---------------------------------------------------------------------------
// Launch sequences as HIP graphs.  A sequence of kernel launches (on the
// caller's stream and the workspace's two extra streams, joined by events)
// that depends on nothing the host decides while it runs is recorded once on
// the workspace's capture stream and kept under a key of everything its
// launches take (workspace and table addresses, the fields' geometry and
// roles, kernel choices); a later call with the same key launches the graph
// on its stream instead of issuing the launches one by one.  Not used with
// stage profiling (its events would be recorded), by the static-scratch
// entry point, or when EBCC_GRAPHS=0.  The sequences stage nothing and set
// no memory with hipMemset: every table is uploaded before them, and
// buffers are cleared by kernels.
// ---------------------------------------------------------------------------
struct GraphKey {
  std::string b;
  template <typename T> void add(const T& v) { b.append(reinterpret_cast<const char*>(&v), sizeof(T)); }
  GraphKey(const char* what, const Call& c) {
    b = what;
    b.push_back('\0');
    add(c.ws); add(c.ws->base); add(c.nf); add(c.nblk); add(c.ntiles); add(c.cbw); add(c.cbh);
    add(c.forced_global); add(c.d_blk); add(c.d_tiles); add(c.d_tix); add(c.d_slot_off); add(c.F); add(c.Fc);
    add(c.spec_depth); add(c.want_cpos); add(c.need_lists); add(c.any_byp);
    for (int k = 0; k < 4; k++) add(c.ncls[k]);
    const Tuning t = tuning();
    add(t);
    for (const char* v : {"EBCC_T1_KERNEL", "EBCC_T1_PIPE", "EBCC_T1_PERSIST", "EBCC_SPIHT_KERNEL"}) {
      const char* e = getenv(v);
      b += e ? e : "-";
      b.push_back('\0');
    }
    for (int i = 0; i < c.nf; i++) {
      const FieldDev& f = c.Fh[i];
      add(f.ny); add(f.nx); add(f.L); add(f.nb); add(f.blk0); add(f.nblk); add(f.tile0); add(f.ntiles);
      add(f.active); add(f.mode); add(f.bt); add(f.byp); add(c.plans[i]);
    }
  }
};

constexpr size_t kMaxGraphs = 512;
static std::mutex g_graph_mu;
static std::map<std::string, hipGraphExec_t> g_graphs;
// Keys met once: a sequence is recorded the second time its key comes up,
// so one-off shapes (a serving loop's ever-changing batches) pay no
// recording.  Forgotten when full.
constexpr size_t kMaxSeen = 4096;
static std::set<std::string> g_graph_seen;

static bool graphs_usable(const Call& c, const Prof& prof) {
  const char* e = getenv("EBCC_GRAPHS");
  if (e && e[0] == '0') return false;
  return !prof.on && c.ws && !c.ws->fixed && c.ws->capst && c.ws->aux;
}

// Runs seq(stream): from the graph cached under key; the first time a key
// comes up the launches are issued directly, the second time the sequence is
// recorded (when the cache is full the launches are always issued directly).
template <typename Seq>
static int run_graph(const GraphKey& key, Call& c, Seq& seq) {
  hipGraphExec_t ex = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key.b);
    if (it != g_graphs.end()) {
      ex = it->second;
    } else if (g_graphs.size() >= kMaxGraphs) {
      return seq(c.st);
    } else if (!g_graph_seen.count(key.b)) {
      if (g_graph_seen.size() >= kMaxSeen) g_graph_seen.clear();
      g_graph_seen.insert(key.b);
      return seq(c.st);
    } else {
      g_graph_seen.erase(key.b);
    }
  }
  if (!ex) {
    hipStream_t cs = c.ws->capst;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = seq(cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != EBCC_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess || !g) return fail(EBCC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(EBCC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graphs[key.b] = ex;
  }
  HIPCHK(hipGraphLaunch(ex, c.st));
  return EBCC_OK;
}

// Drops every cached graph (their tables and workspaces are being freed).
static void graphs_clear() {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
  g_graphs.clear();
  g_graph_seen.clear();
}

// Lay out (base == nullptr: measure) the workspace of a call; every coded
// field gets its buffers, items get their tables.
static size_t layout_call(Call& c, char* base, const std::vector<int>& coded) {
  Carve cv{base, 0};
  c.F = cv.take<FieldDev>(c.nf);
  c.d_fp = cv.take<FieldParams>(c.nf);
  int* flags = cv.take<int>(8 * (size_t)c.nf);
  unsigned* u32s = cv.take<unsigned>(8 * (size_t)c.nf);
  int64_t* totals = cv.take<int64_t>(8 * (size_t)c.nf);
  for (int i = 0; i < c.nf; i++) {
    FieldDev& f = c.Fh[i];
    size_t N = (size_t)f.ny * f.nx;
    f.fp = c.d_fp ? c.d_fp + i : nullptr;
    f.flags = flags ? flags + 8 * i : nullptr;
    f.u32s = u32s ? u32s + 8 * i : nullptr;
    f.totals = totals ? totals + 8 * i : nullptr;
    size_t nbuf = coded[i] ? N : 0;
    for (int b = BUF_COEF; b <= BUF_CHAT; b++) f.buf[b] = cv.take<float>(nbuf);
    f.qr = cv.take<uint32_t>(nbuf);
    f.cpos = (c.want_cpos && nbuf) ? cv.take<uint32_t>(nbuf) : nullptr;
    f.sub = cv.take<uint32_t>(nbuf);
    f.maxd = cv.take<uint32_t>(nbuf);
    f.maxl = cv.take<uint32_t>(nbuf);
  }
  size_t nb = c.nblk, nt = c.ntiles;
  size_t ms = c.cbw <= 32 ? 4 : 8;
  c.planes = cv.take<char>(nb * kQBits * c.cbh * ms);
  c.signs = cv.take<char>(nb * c.cbh * ms);
  c.sppf = cv.take<char>(nb * c.cbh * ms);
  c.pb = cv.take<uint8_t>(nb); c.kb = cv.take<uint8_t>(nb); c.nh = cv.take<uint8_t>(nb);
  c.hk = cv.take<uint8_t>(nb * kPassStride);
  c.R = cv.take<int32_t>(nb * kPassStride); c.bpt = cv.take<int32_t>(nb * kPassStride);
  c.dr = cv.take<int32_t>(nb * kPassStride); c.len = cv.take<int32_t>(nb);
  c.D = cv.take<int64_t>(nb * kPassStride); c.keys = cv.take<uint64_t>(nb * kPassStride);
  c.tail = cv.take<uint32_t>(nb * kPassStride);
  c.rbt = cv.take<int32_t>(c.any_byp ? nb * kPassStride : 0);
  c.boff = cv.take<int64_t>(nb); c.bent = cv.take<uint32_t>(nb);
  c.cw = cv.take<uint8_t>(nb * (size_t)kCwCap);
  c.tlen = cv.take<uint32_t>(nt); c.tent = cv.take<uint32_t>(nt); c.toff = cv.take<int64_t>(nt);
  c.misfit = cv.take<int>(nt);
  c.tcut = cv.take<uint32_t>(3 * nt);
  c.tbits = cv.take<uint32_t>(nt);
  c.border = cv.take<int>(nb);
  c.qctr = cv.take<int>(1);
  c.tix_sorted = cv.take<int>(nt);
  c.collect = cv.take<int64_t>(8 * (size_t)c.nf);
  // candidates per field and search round: "all planes" and the nodes of
  // spec_depth levels of the bisection tree
  const size_t ncand = std::max<size_t>(4, (size_t)1 << c.spec_depth);
  c.Fc = cv.take<FieldDev>(ncand * (size_t)c.nf);
  c.cand_flags = cv.take<int>(8 * ncand * (size_t)c.nf);
  c.cand_buf.assign(c.nf, nullptr);
  for (int i = 0; i < c.nf; i++)
    if (c.spec_depth > 1 && coded[i])
      c.cand_buf[i] = cv.take<float>(2 * (ncand - 1) * (size_t)c.Fh[i].ny * c.Fh[i].nx);
  if (c.own_bands) {
    size_t nbands = 0;
    for (int i = 0; i < c.nf; i++) nbands += c.plans[i]->bands.size();
    c.d_bands_own = cv.take<Band>(nbands);
    nbands = 0;
    for (int i = 0; i < c.nf; i++) {
      c.Fh[i].bands = c.d_bands_own ? c.d_bands_own + nbands : nullptr;
      nbands += c.plans[i]->bands.size();
    }
  }
  c.d_blk_own = cv.take<Blk>(nb);
  c.d_tiles_own = cv.take<TileD>(nt);
  c.d_slot_own = cv.take<int64_t>(nt + 1);
  c.d_tix_own = cv.take<int>(nt);
  int64_t lists = 0, slots = 0;
  for (int i = 0; i < c.nf; i++)
    if (coded[i]) { lists += (int64_t)c.Fh[i].ny * c.Fh[i].nx; slots += c.plans[i]->slot_off.back(); }
  c.lists = cv.take<uint64_t>(c.need_lists ? 4 * (size_t)lists : 0);
  c.slots = cv.take<uint8_t>((size_t)slots);
  return cv.used + 256;
}

// Largest single staged copy of a call, doubled (the staging buffer then
// holds at least two copies before it has to wait).
static size_t pin_need(const Call& c) {
  // the largest table staged at once: the search rounds' candidate fields
  // (up to 2^spec_depth per field), block and tile tables
  size_t m = sizeof(FieldDev) * (size_t)c.nf * std::max<size_t>(4, (size_t)1 << c.spec_depth);
  m = std::max(m, sizeof(Blk) * (size_t)c.nblk);
  m = std::max(m, sizeof(TileD) * (size_t)c.ntiles);
  m = std::max(m, sizeof(int64_t) * ((size_t)c.ntiles + 1));
  m = std::max(m, sizeof(int) * (size_t)c.ntiles);
  m = std::max(m, 2 * sizeof(float) * (size_t)c.nf);
  return 2 * m + 4096;
}

// Concatenate the coded fields' blocks and tiles (a single field reuses its
// plan's device tables).
static int build_items(Call& c, const std::vector<int>& coded) {
  int nb = 0, nt = 0;
  std::vector<int> ci;
  for (int i = 0; i < c.nf; i++)
    if (coded[i]) ci.push_back(i);
  for (int i : ci) {
    c.Fh[i].blk0 = nb; c.Fh[i].nblk = c.plans[i]->nblk; nb += c.plans[i]->nblk;
    c.Fh[i].tile0 = nt; c.Fh[i].ntiles = c.plans[i]->ntiles; nt += c.plans[i]->ntiles;
  }
  c.nblk = nb;
  c.ntiles = nt;
  return EBCC_OK;
}

static int upload_items(Call& c, const std::vector<int>& coded) {
  std::vector<int> ci;
  for (int i = 0; i < c.nf; i++)
    if (coded[i]) ci.push_back(i);
  if (c.own_bands) {   // plans without device tables: stage the subband tables
    for (int i = 0; i < c.nf; i++) {
      const Plan* p = c.plans[i];
      if (int rc = c.stage(const_cast<Band*>(c.Fh[i].bands), p->bands.data(), sizeof(Band) * p->bands.size()))
        return rc;
    }
  }
  if (ci.size() == 1 && ci[0] == 0 && c.plans[0]->d_blks) {
    c.d_blk = c.plans[0]->d_blks;
    c.d_tiles = c.plans[0]->d_tiles;
    c.d_slot_off = c.plans[0]->d_slot_off;
    c.d_tix = c.plans[0]->d_tix;
    for (int k = 0; k < 4; k++) c.ncls[k] = c.plans[0]->ncls[k];
    return EBCC_OK;
  }
  std::vector<Blk> blks;
  std::vector<TileD> tiles;
  std::vector<int64_t> soff;
  blks.reserve(c.nblk);
  tiles.reserve(c.ntiles);
  soff.reserve(c.ntiles + 1);
  int64_t lo = 0, so = 0;
  soff.push_back(0);
  for (int i : ci) {
    const Plan* p = c.plans[i];
    for (Blk b : p->blks) { b.field = i; blks.push_back(b); }
    for (size_t t = 0; t < p->tiles.size(); t++) {
      TileD d = p->tiles[t];
      d.field = i;
      d.off += lo;
      tiles.push_back(d);
      soff.push_back(so + p->slot_off[t + 1]);
    }
    lo += (int64_t)p->ny * p->nx;
    so += p->slot_off.back();
  }
  std::vector<int> tix;
  tix.reserve(c.ntiles);
  for (int k = 0; k < 4; k++) {
    c.ncls[k] = 0;
    for (int i : ci) {
      const Plan* p = c.plans[i];
      int base = c.Fh[i].tile0, o = 0;
      for (int q = 0; q < k; q++) o += p->ncls[q];
      for (int q = 0; q < p->ncls[k]; q++) tix.push_back(base + p->tix[o + q]);
      c.ncls[k] += p->ncls[k];
    }
  }
  int rc;
  if ((rc = c.stage(c.d_tix_own, tix.data(), sizeof(int) * tix.size()))) return rc;
  c.d_tix = c.d_tix_own;
  if ((rc = c.stage(c.d_blk_own, blks.data(), sizeof(Blk) * blks.size()))) return rc;
  if ((rc = c.stage(c.d_tiles_own, tiles.data(), sizeof(TileD) * tiles.size()))) return rc;
  if ((rc = c.stage(c.d_slot_own, soff.data(), sizeof(int64_t) * soff.size()))) return rc;
  c.d_blk = c.d_blk_own;
  c.d_tiles = c.d_tiles_own;
  c.d_slot_off = c.d_slot_own;
  return EBCC_OK;
}

struct FieldIn {
  const float* x;
  size_t ny, nx;
  double err;
};

// Geometry of a compress call whose fields' sizes and plans are set: every
// field is laid out as coded (the mode is known only on the device).
// Returns the workspace bytes the call needs.
static size_t compress_need(Call& c, const std::vector<int>& coded) {
  build_items(c, coded);
  // small calls evaluate four bisection levels per search round (one round
  // for up to 16 planes: one read-back), mid-sized ones two, large batches
  // one (the device is busy anyway)
  size_t tot = 0;
  for (auto& f : c.Fh) tot += (size_t)f.ny * f.nx;
  c.spec_depth = tot <= ((size_t)1 << 22) ? 4 : (tot <= ((size_t)1 << 24) ? 2 : 1);
  c.forced_global = spiht_forced_global();
  c.need_lists = c.forced_global;
  for (int i = 0; i < c.nf; i++) c.need_lists |= c.plans[i]->ncls[2] > 0;
  return layout_call(c, nullptr, coded);
}

// Algorithm 1's second binary search at byte granularity, for the fields
// sp marks (their residual planes n_max .. ns are SPIHT coded, with cpos and
// the tiles' bit counts tcut): the tiles' codes are read as one embedded
// sequence (plane by plane; sorting passes of every tile, then refinement
// passes), and the search bisects a position t = 8 b (bits, b integer; the
// end of plane ns when 8 b passes it) between the end of plane ns + 1,
// which misses the bound, and the end of plane ns, which meets it.  Every
// field advances in lockstep, spec_depth levels of its bisection per round
// (one launch sequence and one read-back); a candidate's coefficients come
// from spiht_cut_recon, its check from the inverse DWT's epilogue.  The
// chosen cut goes to each field's table entry and the tiles' final lengths
// to tlen/tent/tbits.
struct CutTables {
  std::vector<uint32_t> lo, rs, hi;        // per tile of the field: bits through ns + 1, before ns's refinement, through ns
  std::vector<int64_t> ps, pr;             // inclusive prefix sums of the sorting / refinement lengths of plane ns
  int64_t vlo = 0, vhi = 0;
  // position t (vlo < t <= vhi) of the embedded sequence -> the cut
  void cut(int64_t t, int* kind, int* J, uint32_t* lJ) const {
    int64_t u = t - vlo;
    const int64_t stot = ps.empty() ? 0 : ps.back();
    const std::vector<int64_t>& pre = u <= stot ? ps : pr;
    const std::vector<uint32_t>& base = u <= stot ? lo : rs;
    if (u > stot) u -= stot;
    const int j = (int)(std::lower_bound(pre.begin(), pre.end(), u) - pre.begin());
    const int jj = j < (int)pre.size() ? j : (int)pre.size() - 1;
    *kind = stot >= t - vlo ? 0 : 1;
    *J = jj;
    *lJ = (uint32_t)((int64_t)base[jj] + u - (jj ? pre[jj - 1] : 0));
  }
};

static int byte_search(Call& c, const std::vector<int>& sp, std::vector<int>& checks) {
  const int nf = c.nf;
  hipStream_t st = c.st;
  std::vector<uint32_t> tc(3 * (size_t)std::max(c.ntiles, 1));
  if (int rc = c.fetch(tc.data(), c.tcut, 3 * (size_t)c.ntiles)) return rc;
  std::vector<CutTables> ct(nf);
  std::vector<int64_t> blo(nf, 0), bhi(nf, 0);
  std::vector<int> on(nf, 0);
  int max_tiles = 0;
  for (int i = 0; i < nf; i++) {
    if (!sp[i] || !c.Fh[i].bt) continue;
    const FieldDev& f = c.Fh[i];
    CutTables& T = ct[i];
    int64_t s = 0, r = 0;
    for (int j = 0; j < f.ntiles; j++) {
      const uint32_t* e = &tc[3 * (size_t)(f.tile0 + j)];
      T.lo.push_back(e[0]); T.rs.push_back(e[1]); T.hi.push_back(e[2]);
      T.vlo += e[0]; T.vhi += e[2];
      s += (int64_t)e[1] - e[0]; r += (int64_t)e[2] - e[1];
      T.ps.push_back(s); T.pr.push_back(r);
    }
    blo[i] = T.vlo / 8; bhi[i] = (T.vhi + 7) / 8;
    on[i] = 1;
    max_tiles = std::max(max_tiles, f.ntiles);
  }
  auto at = [&](int i, int64_t b) { return std::min<int64_t>(8 * b, ct[i].vhi); };
  struct Cand { int field; int64_t b; int slot; };
  std::vector<FieldDev> Fch;
  for (int round = 0; round < 64; round++) {
    std::vector<Cand> cands;
    std::vector<int> nslot(nf, 0);
    std::function<void(int, int64_t, int64_t, int)> tree = [&](int i, int64_t l, int64_t h, int depth) {
      if (depth == 0 || h - l <= 1) return;
      const int64_t m = (l + h) >> 1;
      cands.push_back(Cand{i, m, nslot[i]++});
      tree(i, l, m, depth - 1);
      tree(i, m, h, depth - 1);
    };
    for (int i = 0; i < nf; i++)
      if (on[i]) tree(i, blo[i], bhi[i], c.spec_depth);
    if (cands.empty()) break;
    const int nc = (int)cands.size();
    Fch.resize(nc);
    size_t cmax = 0;
    for (int j = 0; j < nc; j++) {
      const Cand& q = cands[j];
      FieldDev f = c.Fh[q.field];
      f.active = 1;
      ct[q.field].cut(at(q.field, q.b), &f.cut_kind, &f.cut_tile, &f.cut_bits);
      f.flags = c.cand_flags + 8 * j;
      if (q.slot > 0) {
        size_t N = (size_t)f.ny * f.nx;
        f.buf[BUF_CHAT] = c.cand_buf[q.field] + (size_t)(2 * (q.slot - 1)) * N;
        f.buf[BUF_TMP] = c.cand_buf[q.field] + (size_t)(2 * (q.slot - 1) + 1) * N;
      }
      Fch[j] = f;
      cmax = std::max(cmax, (size_t)f.ny * f.nx);
    }
    if (int rc = c.stage(c.Fc, Fch.data(), sizeof(FieldDev) * nc)) return rc;
    k_zero_slot<<<(nc + 63) / 64, 64, 0, st>>>(c.Fc, nc, 0);
    spiht_cut_recon(c.Fc, nc, max_tiles, c.d_tiles, c.tcut, st);
    dwt_inverse(c.Fc, Fch.data(), nc, BUF_CHAT, BUF_CHAT, EPI_CHECK, st);
    HIPCHK(hipGetLastError());
    std::vector<int> cf(8 * (size_t)nc);
    if (int rc = c.fetch(cf.data(), c.cand_flags, 8 * (size_t)nc)) return rc;
    std::vector<std::map<int64_t, bool>> res(nf);
    for (int j = 0; j < nc; j++) {
      res[cands[j].field][cands[j].b] = cf[8 * j] == 0;
      checks[cands[j].field]++;
    }
    for (int i = 0; i < nf; i++) {
      if (!on[i]) continue;
      while (bhi[i] - blo[i] > 1) {
        const int64_t m = (blo[i] + bhi[i]) >> 1;
        auto it = res[i].find(m);
        if (it == res[i].end()) break;
        if (it->second) bhi[i] = m; else blo[i] = m;
      }
      if (bhi[i] - blo[i] <= 1) on[i] = 0;
    }
  }
  std::vector<int> btf(nf, 0);
  for (int i = 0; i < nf; i++) {
    if (!sp[i] || !c.Fh[i].bt) continue;
    FieldDev& f = c.Fh[i];
    ct[i].cut(at(i, bhi[i]), &f.cut_kind, &f.cut_tile, &f.cut_bits);
    btf[i] = 1;
  }
  if (int rc = c.set_active(btf)) return rc;
  spiht_cut_tiles(c.F, c.d_tiles, c.ntiles, c.tcut, c.tlen, c.tent, c.tbits, st);
  HIPCHK(hipGetLastError());
  return c.set_active(sp);
}

// Compress nf fields; stream i goes to out + off[i] (compacted in field
// order); lens[i] receives its length.  On ENOSPC *need holds the total.
// With fstat, a field whose input is not finite gets EBCC_EINVAL there and
// no stream (length 0), the others are still compressed and the call
// returns EBCC_EINVAL; without it such a field fails the call.
// With fixed_ws (the no-allocation entry point) the call runs in that
// workspace alone: plans are built for the call without device tables, the
// search depth is the largest that fits, and a call that does not fit fails
// before any launch.
static int compress_call(const std::vector<FieldIn>& in, const ebcc_params* pp, uint8_t* out, size_t cap,
                         std::vector<uint64_t>& offs, std::vector<uint64_t>& lens, size_t* need, hipStream_t st,
                         const Trace* tr, std::vector<int>* fstat = nullptr, WS* fixed_ws = nullptr) {
  ebcc_params dflt;
  if (!pp) { ebcc_params_default(&dflt); pp = &dflt; }
  const int nf = (int)in.size();
  *need = 0;
  offs.assign(nf, 0);
  lens.assign(nf, 0);
  if (nf == 0) return EBCC_OK;
  if (!out) return fail(EBCC_EINVAL, "NULL output buffer");
  int rc;
  for (int i = 0; i < nf; i++) {
    if ((rc = check_params(in[i].ny, in[i].nx, pp, in[i].err))) return rc;
    if (!in[i].x) return fail(EBCC_EINVAL, "NULL input buffer");
  }
  Call c;
  c.nf = nf;
  c.st = st;
  c.Fh.assign(nf, FieldDev());
  c.plans.assign(nf, nullptr);
  c.cbw = 1 << pp->cblk_log2w;
  c.cbh = 1 << pp->cblk_log2h;
  const int cbl = (int)(pp->cblk_log2w | (pp->cblk_log2h << 4)), T = (int)pp->spiht_tile;
  std::vector<std::unique_ptr<Plan>> own_plans;
  c.own_bands = fixed_ws != nullptr;
  for (int i = 0; i < nf; i++) {
    FieldDev& f = c.Fh[i];
    memset(&f, 0, sizeof(f));
    f.ny = (int)in[i].ny; f.nx = (int)in[i].nx;
    f.L = levels_eff(f.ny, f.nx, (int)pp->levels);
    f.buf[BUF_X] = const_cast<float*>(in[i].x);
    f.err = in[i].err; f.bound_mode = (int)pp->bound_mode;
    f.cbl = cbl; f.T = T; f.active = 1; f.byp = (int)pp->bypass;
    if (fixed_ws) {
      std::unique_ptr<Plan> p(new Plan());
      p->ny = f.ny; p->nx = f.nx; p->L = f.L; p->cbl2w = (int)pp->cblk_log2w; p->cbl2h = (int)pp->cblk_log2h;
      p->cbw = 1 << p->cbl2w; p->cbh = 1 << p->cbl2h; p->T = T;
      if ((rc = build_plan(*p))) return rc;
      c.plans[i] = p.get();
      own_plans.push_back(std::move(p));
    } else if ((rc = get_plan(f.ny, f.nx, f.L, pp->cblk_log2w, pp->cblk_log2h, T, &c.plans[i]))) {
      return rc;
    }
    f.bands = c.plans[i]->d_bands;
    f.nb = c.plans[i]->nb;
  }
  std::vector<int> coded(nf, 1);
  c.want_cpos = pp->trunc != 0;
  c.any_byp = pp->bypass != 0;
  size_t need_ws = compress_need(c, coded);
  char* base;
  if (fixed_ws) {
    // fewer bisection levels per search round take fewer candidate planes
    while (need_ws > fixed_ws->cap && c.spec_depth > 1) {
      c.spec_depth = c.spec_depth > 2 ? 2 : 1;
      need_ws = layout_call(c, nullptr, coded);
    }
    if (need_ws > fixed_ws->cap)
      return fail(EBCC_EINVAL, "the field needs " + std::to_string(need_ws) + " bytes of scratch; the static scratch "
                  "array holds " + std::to_string(fixed_ws->cap));
    c.ws = fixed_ws;
    base = (char*)fixed_ws->base;
  } else {
    if ((rc = get_ws(st, &c.ws))) return rc;
    if ((rc = grow_ws(c.ws, need_ws, pin_need(c), st, &base))) return rc;
  }
  layout_call(c, base, coded);
  Prof prof(st, fixed_ws == nullptr);

  // ---- scalars of every field: min, max, range, eps, exponents ----
  if ((rc = c.upload())) return rc;
  k_init_fields<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf);
  size_t maxN = 0;
  for (auto& f : c.Fh) maxN = std::max(maxN, (size_t)f.ny * f.nx);
  k_minmax<<<dim3(grid_sweep(maxN), nf), 256, 0, st>>>(c.F);
  k_params<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf);
  HIPCHK(hipGetLastError());
  prof.mark(S_SCALARS);
  std::vector<FieldParams> fps(nf);
  if ((rc = c.fetch(fps.data(), c.d_fp, nf))) return rc;
  std::vector<int> mode(nf), failed(nf, 0);
  int first_bad = EBCC_OK;
  std::string bad_msg;
  if (fstat) fstat->assign(nf, EBCC_OK);
  for (int i = 0; i < nf; i++) {
    if (fps[i].mode < 0) {
      std::string msg = "input field " + std::to_string(i) + " contains non-finite values";
      if (!fstat) return fail(EBCC_EINVAL, msg);
      (*fstat)[i] = EBCC_EINVAL;
      failed[i] = 1;
      if (first_bad == EBCC_OK) { first_bad = EBCC_EINVAL; bad_msg = msg; }
      mode[i] = MODE_CONST;   // no stream is written for it (below)
      c.Fh[i].e0 = 0;
      continue;
    }
    mode[i] = fps[i].mode;
    c.Fh[i].e0 = fps[i].e0;
  }
  // coded fields take part in the pipeline
  std::vector<int> act(nf), resid(nf, 0), nmax(nf, -1), checks(nf, 0);
  for (int i = 0; i < nf; i++) {
    act[i] = mode[i] == MODE_CODED && !failed[i];
    checks[i] = act[i];
    c.Fh[i].budget = base_budget((int64_t)in[i].ny * (int64_t)in[i].nx, c.plans[i]->nblk, pp->base_ratio);
    c.Fh[i].er = fps[i].elog - 6;
  }
  if ((rc = upload_items(c, coded))) return rc;
  std::vector<double> r_use(nf, pp->base_ratio), r_only(nf, -1.0);
  const std::vector<int> coded0(act);   // coded after the field scalars
  std::vector<int64_t> col;             // per-field results read back (k_collect)
  bool any = false;
  for (int v : act) any |= v != 0;
  // launch sequences without host decisions inside run from cached graphs
  const bool use_graphs = graphs_usable(c, prof);
  size_t maxN_all = 0;
  for (auto& f : c.Fh) maxN_all = std::max(maxN_all, (size_t)f.ny * f.nx);
  auto run_seq = [&](const char* name, auto& seq) -> int {
    if (!use_graphs) return seq(st);
    GraphKey key(name, c);
    key.add(maxN_all);
    return run_graph(key, c, seq);
  };
  if (any) {
    if ((rc = c.set_active(act))) return rc;
    // ---- base layer: DWT of the normalised field, tier-1, PCRD at ratio r ----
    auto seq_base = [&](hipStream_t s) -> int {
      dwt_forward(c.F, c.Fh.data(), nf, BUF_X, BUF_COEF, PRO_NORM, s);
      prof.mark(S_DWT);
      quant_planes(c.F, c.d_blk, c.nblk, c.cbw, c.cbh, c.planes, c.signs, c.pb, s);
      prof.mark(S_QUANT);
      const T1Split t1s{c.ws->aux, c.ws->ev_fork, c.ws->ev_join};
      t1_encode(c.F, c.d_blk, c.nblk, c.cbw, c.cbh, c.planes, c.signs, c.pb, c.cw, c.R, c.D, c.bpt, c.tail, c.sppf,
                s, &t1s, c.border, c.qctr, c.any_byp ? c.rbt : nullptr);
      prof.mark(S_T1ENC);
      HIPCHK(hipGetLastError());
      return EBCC_OK;
    };
    if ((rc = run_seq("enc_base", seq_base))) return rc;
    // ---- base ratio: the given r, or Algorithm 1's feedback search ----
    if (pp->q > 0.0) {
      auto fieldN = [&](int i) { return (int64_t)c.Fh[i].ny * c.Fh[i].nx; };
      auto search = [&](double q, std::vector<double>& rf, std::vector<double>& qf) -> int {
        // per field: phase 0 evaluates r0, 1 halves r_low, 2 doubles r_high,
        // 3 bisects; every round evaluates one ratio per field still
        // searching (PCRD, closed-form dec_base, inverse DWT, q_A count)
        struct S { int ph; double r_low, r_high, r_f, q_f, qa0, r_eval; bool zero0; };
        std::vector<S> sv(nf);
        std::vector<int> ev(nf, 0);
        const double r0 = pp->base_ratio;
        for (int i = 0; i < nf; i++)
          if (act[i]) {
            sv[i] = S{0, r0, r0, r0, 0.0, 0.0, r0, base_budget(fieldN(i), c.Fh[i].nblk, r0) == 0};
            ev[i] = 1;
          }
        auto bisect = [&](int i) {
          S& z = sv[i];
          if (z.r_high - z.r_low > 1e-3) { z.ph = 3; z.r_eval = (z.r_low + z.r_high) / 2.0; }
          else { z.ph = 4; ev[i] = 0; }
        };
        auto after_halving = [&](int i) {
          S& z = sv[i];
          if (z.qa0 > q && !z.zero0) { z.ph = 2; z.r_high = z.r_high * 2.0; z.r_eval = z.r_high; }
          else bisect(i);
        };
        for (int round = 0; round < 4096; round++) {
          bool anyev = false;
          for (int i = 0; i < nf; i++)
            if (ev[i]) { c.Fh[i].budget = base_budget(fieldN(i), c.Fh[i].nblk, sv[i].r_eval); anyev = true; }
          if (!anyev) break;
          int rc2;
          if ((rc2 = c.set_active(ev))) return rc2;
          k_zero_slot<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf, 2);
          pcrd(c.F, nf, c.max_nblk(), c.pb, c.R, c.D, c.kb, c.hk, c.keys, c.dr, c.nh, c.len, st);
          virtual_decode(c.F, c.d_blk, c.nblk, c.cbw, c.cbh, c.pb, c.kb, c.sppf, st);
          dwt_inverse(c.F, c.Fh.data(), nf, BUF_YHAT, BUF_ABASE, EPI_STORE, st);
          k_count_within<<<dim3(grid_sweep(maxN), nf), 256, 0, st>>>(c.F);
          HIPCHK(hipGetLastError());
          if ((rc2 = c.collect_host(col))) return rc2;
          for (int i = 0; i < nf; i++) {
            if (!ev[i]) continue;
            S& z = sv[i];
            const double qa = (double)col[8 * i + 6] / (double)fieldN(i);
            const bool allfit = ((col[8 * i + 7] >> 48) & 1) != 0;
            const int64_t bud = base_budget(fieldN(i), c.Fh[i].nblk, z.r_eval);
            if (z.ph == 0) {
              z.qa0 = qa; z.q_f = qa;
              if (qa < q && !allfit) { z.ph = 1; z.r_low = z.r_low / 2.0; z.r_eval = z.r_low; }
              else after_halving(i);
            } else if (z.ph == 1) {
              z.r_f = z.r_low; z.q_f = qa;
              if (qa < q && !allfit) { z.r_low = z.r_low / 2.0; z.r_eval = z.r_low; }
              else after_halving(i);
            } else if (z.ph == 2) {
              if (qa > q && bud != 0) { z.r_high = z.r_high * 2.0; z.r_eval = z.r_high; }
              else bisect(i);
            } else {
              if (qa < q) z.r_high = z.r_eval;
              else { z.r_low = z.r_eval; z.r_f = z.r_eval; z.q_f = qa; }
              bisect(i);
            }
          }
        }
        for (int i = 0; i < nf; i++) { rf[i] = sv[i].r_f; qf[i] = sv[i].q_f; }
        return EBCC_OK;
      };
      std::vector<double> qf(nf, 0.0);
      if ((rc = search(pp->q, r_use, qf))) return rc;
      if (pp->q < 1.0) {
        std::vector<double> r1(nf, 0.0), q1(nf, 0.0);
        if ((rc = search(1.0, r1, q1))) return rc;
        for (int i = 0; i < nf; i++)
          if (act[i] && q1[i] >= 1.0) r_only[i] = r1[i];   // the base alone meets the bound
      }
      for (int i = 0; i < nf; i++)
        if (act[i]) c.Fh[i].budget = base_budget(fieldN(i), c.Fh[i].nblk, r_use[i]);
      if ((rc = c.set_active(act))) return rc;
    }
    auto seq_resid = [&](hipStream_t s) -> int {
      pcrd(c.F, nf, c.max_nblk(), c.pb, c.R, c.D, c.kb, c.hk, c.keys, c.dr, c.nh, c.len, s);
      prof.mark(S_PCRD);
      // ---- A_base = dec_base(e_base) (closed form), residual, its DWT ----
      virtual_decode(c.F, c.d_blk, c.nblk, c.cbw, c.cbh, c.pb, c.kb, c.sppf, s);
      dwt_inverse(c.F, c.Fh.data(), nf, BUF_YHAT, BUF_ABASE, EPI_STORE, s);
      pointwise(c.F, c.Fh.data(), nf, BUF_CHAT, BUF_CHAT, 3, EPI_CHECK, 0, s);   // does the base alone meet the bound?
      prof.mark(S_BASEREC);
      dwt_forward(c.F, c.Fh.data(), nf, BUF_X, BUF_CRES, PRO_NORM_MINUS, s);
      k_quant_res<<<dim3(grid_sweep(maxN), nf), 256, 0, s>>>(c.F);
      HIPCHK(hipGetLastError());
      prof.mark(S_RESID);
      return EBCC_OK;
    };
    if ((rc = run_seq("enc_resid", seq_resid))) return rc;
    if ((rc = c.collect_host(col))) return rc;
    // ---- truncation search, all fields in lockstep: one launch + one sync per round ----
    enum { NONE = 0, CHECK_ALL, BISECT, REQUANT, FOUND, FAIL };
    std::vector<int> state(nf, NONE), att(nf, 0), lo(nf, 0), hi(nf, 0);
    auto start_attempt = [&](int i) {
      int q = (int)col[8 * i + 2];
      int nm = q ? 31 - __builtin_clz((unsigned)q) : -1;
      if (nm < 0) {
        if (++att[i] >= 5) { state[i] = FAIL; return; }
        state[i] = REQUANT;
        c.Fh[i].er = fps[i].elog - 6 - att[i];
        return;
      }
      nmax[i] = nm;
      state[i] = CHECK_ALL;
    };
    for (int i = 0; i < nf; i++)
      if (act[i] && col[8 * i + 0]) { resid[i] = 1; start_attempt(i); }
    // Candidates of a round: the bisection of Algorithm 1's residual loop,
    // spec_depth levels of its decision tree at once (all are evaluated;
    // the decisions then follow the tree, so the result is the sequential
    // bisection's); a field's first round also checks "all planes".
    struct Cand { int field, k, slot; };
    std::vector<FieldDev> Fch;
    for (int round = 0; round < 256; round++) {
      std::vector<int> rq(nf, 0);
      std::vector<Cand> cands;
      std::vector<int> nslot(nf, 0);
      bool anyrq = false;
      std::function<void(int, int, int, int)> tree = [&](int i, int l, int h, int depth) {
        if (depth == 0 || h - l <= 1) return;
        int m = (l + h) >> 1;
        cands.push_back(Cand{i, m, nslot[i]++});
        tree(i, l, m, depth - 1);
        tree(i, m, h, depth - 1);
      };
      for (int i = 0; i < nf; i++) {
        if (state[i] == REQUANT) { rq[i] = 1; anyrq = true; }
        if (state[i] == CHECK_ALL) {
          cands.push_back(Cand{i, nmax[i] + 1, nslot[i]++});
          if (c.spec_depth > 1) tree(i, 0, nmax[i] + 1, c.spec_depth);
        } else if (state[i] == BISECT) {
          tree(i, lo[i], hi[i], c.spec_depth);
        }
      }
      if (!anyrq && cands.empty()) break;
      if (anyrq) {
        if ((rc = c.set_active(rq))) return rc;
        k_zero_slot<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf, 1);
        k_quant_res<<<dim3(grid_sweep(maxN), nf), 256, 0, st>>>(c.F);
        k_collect<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf, c.collect);
      }
      const int nc = (int)cands.size();
      if (nc) {
        Fch.resize(nc);
        size_t cmax = 0;
        for (int j = 0; j < nc; j++) {
          const Cand& q = cands[j];
          FieldDev f = c.Fh[q.field];
          f.active = 1;
          f.ns = nmax[q.field] - q.k + 1;
          f.flags = c.cand_flags + 8 * j;
          if (q.slot > 0) {
            size_t N = (size_t)f.ny * f.nx;
            f.buf[BUF_CHAT] = c.cand_buf[q.field] + (size_t)(2 * (q.slot - 1)) * N;
            f.buf[BUF_TMP] = c.cand_buf[q.field] + (size_t)(2 * (q.slot - 1) + 1) * N;
          }
          Fch[j] = f;
          cmax = std::max(cmax, (size_t)f.ny * f.nx);
        }
        if ((rc = c.stage(c.Fc, Fch.data(), sizeof(FieldDev) * nc))) return rc;
        k_zero_slot<<<(nc + 63) / 64, 64, 0, st>>>(c.Fc, nc, 0);
        k_dequant_res<<<dim3(grid_for(cmax), nc), 256, 0, st>>>(c.Fc);
        dwt_inverse(c.Fc, Fch.data(), nc, BUF_CHAT, BUF_CHAT, EPI_CHECK, st);
      }
      HIPCHK(hipGetLastError());
      std::vector<int> cf(8 * (size_t)std::max(nc, 1));
      if (anyrq) {
        col.resize(8 * (size_t)nf);
        HIPCHK(hipMemcpyAsync(col.data(), c.collect, sizeof(int64_t) * col.size(), hipMemcpyDeviceToHost, st));
      }
      if ((rc = c.fetch(cf.data(), c.cand_flags, 8 * (size_t)std::max(nc, 1)))) return rc;
      // results per field: truncation point -> bound met
      std::vector<std::map<int, bool>> res(nf);
      for (int j = 0; j < nc; j++) {
        res[cands[j].field][cands[j].k] = cf[8 * j] == 0;
        checks[cands[j].field]++;
      }
      for (int i = 0; i < nf; i++) {
        if (rq[i]) { start_attempt(i); continue; }
        if (state[i] != CHECK_ALL && state[i] != BISECT) continue;
        if (state[i] == CHECK_ALL) {
          if (!res[i][nmax[i] + 1]) {
            if (++att[i] >= 5) { state[i] = FAIL; continue; }
            state[i] = REQUANT;
            c.Fh[i].er = fps[i].elog - 6 - att[i];
            continue;
          }
          lo[i] = 0; hi[i] = nmax[i] + 1;
          state[i] = BISECT;
        }
        while (hi[i] - lo[i] > 1) {
          int m = (lo[i] + hi[i]) >> 1;
          auto it = res[i].find(m);
          if (it == res[i].end()) break;
          if (it->second) hi[i] = m; else lo[i] = m;
        }
        if (hi[i] - lo[i] <= 1) { state[i] = FOUND; c.Fh[i].ns = nmax[i] - hi[i] + 1; }
      }
    }
    prof.mark(S_SEARCH);
    std::vector<int> sp(nf, 0);
    bool anysp = false;
    for (int i = 0; i < nf; i++) {
      if (state[i] == FAIL) { mode[i] = MODE_RAW; act[i] = 0; }
      if (state[i] == FOUND) { sp[i] = 1; anysp = true; }
      c.Fh[i].nmax = nmax[i];
      if (state[i] != FOUND) resid[i] = 0;
    }
    if (anysp) {
      for (int i = 0; i < nf; i++) c.Fh[i].bt = (pp->trunc && sp[i]) ? 1 : 0;
      if ((rc = c.set_active(sp))) return rc;
      auto seq_spiht = [&](hipStream_t s) -> int {
        spiht_maxima(c.F, c.Fh.data(), nf, s);
        if (c.forced_global) {
          spiht_encode(c.F, c.d_tiles, c.d_tix, c.ntiles, c.lists, c.slots, c.d_slot_off, c.tlen, c.tent, c.tcut, s);
        } else {
          // the classes run concurrently: global and huge tiles on the second
          // stream, big tiles on the third, small ones on the caller's
          const int *t0 = c.d_tix, *t1 = t0 + c.ncls[0], *t2 = t1 + c.ncls[1], *t3 = t2 + c.ncls[2];
          hipStream_t sa = c.ws->aux ? c.ws->aux : s, sb = c.ws->aux2 ? c.ws->aux2 : s;
          if (int rc2 = c.fork_from(s)) return rc2;
          spiht_encode(c.F, c.d_tiles, t2, c.ncls[2], c.lists, c.slots, c.d_slot_off, c.tlen, c.tent, c.tcut, sa);
          spiht_encode_lds(kSpihtHuge, c.F, c.d_tiles, t3, c.ncls[3], c.slots, c.d_slot_off, c.tlen, c.tent, c.tcut,
                           c.misfit, sa);
          spiht_encode_lds(kSpihtBig, c.F, c.d_tiles, t1, c.ncls[1], c.slots, c.d_slot_off, c.tlen, c.tent, c.tcut,
                           c.misfit, sb);
          spiht_encode_lds(kSpihtSmall, c.F, c.d_tiles, t0, c.ncls[0], c.slots, c.d_slot_off, c.tlen, c.tent, c.tcut,
                           c.misfit, s);
          if (int rc2 = c.join_to(s)) return rc2;
        }
        HIPCHK(hipGetLastError());
        return EBCC_OK;
      };
      if ((rc = run_seq("enc_spiht", seq_spiht))) return rc;
      if (pp->trunc && (rc = byte_search(c, sp, checks))) return rc;
      k_scan<<<nf, 1024, 0, st>>>(c.F, c.tlen, 1, 0, 0xFFFFFFFFu, c.toff);
    }
    prof.mark(S_SPIHT);
    // ---- sizes ----
    if ((rc = c.set_active(act))) return rc;
    k_block_entries<<<grid_for(c.nblk), 256, 0, st>>>(c.pb, c.kb, c.len, c.nblk, c.bent);
    k_scan<<<nf, 1024, 0, st>>>(c.F, c.bent, 0, 16, 0xFFFFu, c.boff);
    HIPCHK(hipGetLastError());
    if ((rc = c.collect_host(col))) return rc;
    for (int i = 0; i < nf; i++) {
      if (!act[i]) continue;
      FieldDev& f = c.Fh[i];
      f.bb = (uint32_t)(4 * (int64_t)f.nblk + col[8 * i + 4]);
      f.rb = resid[i] ? (uint32_t)(4 * (int64_t)f.ntiles + col[8 * i + 5] + (f.bt ? 8 : 0)) : 0u;
    }
    // ---- fallback (end of Algorithm 1): the base alone at its own ratio
    // when that stream is smaller ----
    std::vector<int> fbc(nf, 0);
    bool anyfb = false;
    for (int i = 0; i < nf; i++)
      if (coded0[i] && r_only[i] >= 0.0) {
        fbc[i] = 1; anyfb = true;
        c.Fh[i].budget = base_budget((int64_t)c.Fh[i].ny * c.Fh[i].nx, c.Fh[i].nblk, r_only[i]);
      }
    if (anyfb) {
      std::vector<int64_t> ebcc_total(nf, 0);
      for (int i = 0; i < nf; i++)
        if (fbc[i])
          ebcc_total[i] = mode[i] == MODE_CODED ? col[8 * i + 4] + (int64_t)c.Fh[i].rb
                                                : 4 * (int64_t)c.Fh[i].ny * c.Fh[i].nx;
      if ((rc = c.set_active(fbc))) return rc;
      pcrd(c.F, nf, c.max_nblk(), c.pb, c.R, c.D, c.kb, c.hk, c.keys, c.dr, c.nh, c.len, st);
      if ((rc = c.collect_host(col))) return rc;
      std::vector<int> sw(nf, 0), restore(nf, 0);
      bool anysw = false, anyrs = false;
      for (int i = 0; i < nf; i++) {
        if (!fbc[i]) continue;
        const int64_t pay1 = col[8 * i + 7] & (((int64_t)1 << 48) - 1);
        if (pay1 < ebcc_total[i]) {
          sw[i] = 1; anysw = true;
          mode[i] = MODE_CODED; act[i] = 1; resid[i] = 0;
          c.Fh[i].rb = 0;
        } else if (mode[i] == MODE_CODED) {
          restore[i] = 1; anyrs = true;
          c.Fh[i].budget = base_budget((int64_t)c.Fh[i].ny * c.Fh[i].nx, c.Fh[i].nblk, r_use[i]);
        }
      }
      if (anyrs) {   // PCRD at the search's ratio again for the fields that keep it
        if ((rc = c.set_active(restore))) return rc;
        pcrd(c.F, nf, c.max_nblk(), c.pb, c.R, c.D, c.kb, c.hk, c.keys, c.dr, c.nh, c.len, st);
      }
      if (anysw) {   // block table and base size of the base-only streams
        if ((rc = c.set_active(sw))) return rc;
        k_block_entries<<<grid_for(c.nblk), 256, 0, st>>>(c.pb, c.kb, c.len, c.nblk, c.bent);
        k_scan<<<nf, 1024, 0, st>>>(c.F, c.bent, 0, 16, 0xFFFFu, c.boff);
        HIPCHK(hipGetLastError());
        if ((rc = c.collect_host(col))) return rc;
        for (int i = 0; i < nf; i++)
          if (sw[i]) c.Fh[i].bb = (uint32_t)(4 * (int64_t)c.Fh[i].nblk + col[8 * i + 4]);
      }
    }
    for (int i = 0; i < nf; i++) {
      if (!act[i]) continue;
      FieldDev& f = c.Fh[i];
      if ((int64_t)f.bb + f.rb > 4 * (int64_t)f.ny * f.nx) { mode[i] = MODE_RAW; act[i] = 0; resid[i] = 0; }
    }
  }
  // ---- stream lengths and places ----
  uint64_t total = 0;
  for (int i = 0; i < nf; i++) {
    FieldDev& f = c.Fh[i];
    size_t N = (size_t)f.ny * f.nx;
    f.mode = mode[i];
    if (failed[i]) { f.len = 0; f.bb = 0; f.rb = 0; }
    else if (mode[i] == MODE_CONST) { f.len = kHdr; f.bb = 0; f.rb = 0; }
    else if (mode[i] == MODE_RAW) { f.len = kHdr + 4 * (int64_t)N; f.bb = (uint32_t)(4 * N); f.rb = 0; }
    else f.len = kHdr + (int64_t)f.bb + f.rb;
    offs[i] = total;
    lens[i] = (uint64_t)f.len;
    total += (uint64_t)f.len;
  }
  *need = total;
  if (total > cap) return fail(EBCC_ENOSPC, "output capacity too small");
  for (int i = 0; i < nf; i++) c.Fh[i].out = out + offs[i];
  // ---- pack: tables, codewords, tile tables and payloads, raw data, checksum, header ----
  // (the tables of the three roles are staged first: the coded fields in
  // c.F, the raw ones at c.Fc, every field with a stream at c.Fc + nf)
  if ((rc = c.set_active(act))) return rc;
  std::vector<int> rawm(nf, 0), all(nf, 1);
  bool anyraw = false;
  for (int i = 0; i < nf; i++) {
    if (mode[i] == MODE_RAW) { rawm[i] = 1; anyraw = true; }
    all[i] = !failed[i];
  }
  std::vector<FieldDev> Fraw(c.Fh), Fall(c.Fh);
  for (int i = 0; i < nf; i++) { Fraw[i].active = rawm[i]; Fall[i].active = all[i]; }
  FieldDev *const Frd = c.Fc, *const Fad = c.Fc + nf;
  if (anyraw && (rc = c.stage(Frd, Fraw.data(), sizeof(FieldDev) * nf))) return rc;
  if ((rc = c.stage(Fad, Fall.data(), sizeof(FieldDev) * nf))) return rc;
  auto seq_pack = [&](hipStream_t s) -> int {
    if (any) {
      k_put_blocks<<<grid_for(c.nblk), 256, 0, s>>>(c.F, c.d_blk, c.bent, c.nblk);
      k_gather_cw<<<std::max(1, (c.nblk + 3) / 4), 256, 0, s>>>(c.F, c.d_blk, c.cw, c.kb, c.len, c.bpt, c.tail,
                                                               c.rbt, c.boff, c.nblk);
      k_put_tiles<<<grid_for(c.ntiles), 256, 0, s>>>(c.F, c.d_tiles, c.tent, c.ntiles);
      k_gather_tiles<<<std::max(1, (c.ntiles + 3) / 4), 256, 0, s>>>(c.F, c.d_tiles, c.slots, c.d_slot_off, c.tlen,
                                                                      c.tbits, c.toff, c.ntiles);
    }
    if (anyraw) k_copy_raw<<<dim3(grid_for(maxN), nf), 256, 0, s>>>(Frd, 1);
    k_checksum<<<dim3(grid_sweep(maxN), nf), 256, 0, s>>>(Fad);
    k_header<<<(nf + 63) / 64, 64, 0, s>>>(Fad, nf);
    HIPCHK(hipGetLastError());
    return EBCC_OK;
  };
  {
    auto run_pack = [&]() -> int {
      if (!use_graphs) return seq_pack(st);
      GraphKey key("enc_pack", c);
      key.add(maxN_all); key.add(any); key.add(anyraw);
      for (int i = 0; i < nf; i++) { key.add(rawm[i]); key.add(all[i]); }
      return run_graph(key, c, seq_pack);
    };
    if ((rc = run_pack())) return rc;
  }
  prof.mark(S_PACK);
  if (tr && nf == 1) {
    const FieldDev& f = c.Fh[0];
    size_t N = (size_t)f.ny * f.nx;
    int32_t info[11] = {0};
    info[0] = mode[0];
    if (mode[0] == MODE_CODED) {
      if (tr->coef) HIPCHK(hipMemcpyAsync(tr->coef, f.buf[BUF_COEF], 4 * N, hipMemcpyDeviceToDevice, st));
      if (tr->abase) HIPCHK(hipMemcpyAsync(tr->abase, f.buf[BUF_ABASE], 4 * N, hipMemcpyDeviceToDevice, st));
      if (tr->cres) HIPCHK(hipMemcpyAsync(tr->cres, f.buf[BUF_CRES], 4 * N, hipMemcpyDeviceToDevice, st));
      if (tr->kb) HIPCHK(hipMemcpyAsync(tr->kb, c.kb, f.nblk, hipMemcpyDeviceToDevice, st));
      if (tr->pb) HIPCHK(hipMemcpyAsync(tr->pb, c.pb, f.nblk, hipMemcpyDeviceToDevice, st));
      info[1] = f.L; info[2] = f.e0;
      info[3] = resid[0] ? f.er : 0; info[4] = resid[0] ? nmax[0] : -1; info[5] = resid[0] ? f.ns : 0;
      info[6] = f.nblk; info[7] = f.ntiles; info[8] = (int32_t)f.bb; info[9] = (int32_t)f.rb;
    }
    info[10] = checks[0];
    if (tr->info) memcpy(tr->info, info, sizeof(info));
    if (int rc2 = c.wait()) return rc2;
  }
  if (first_bad != EBCC_OK) return fail(first_bad, bad_msg);
  return EBCC_OK;
}

static uint32_t rd32(const uint8_t* p) { return p[0] | (p[1] << 8) | (p[2] << 16) | ((uint32_t)p[3] << 24); }

struct StreamIn {
  const uint8_t* in;
  size_t len;
  float* x;
  size_t ny, nx;
};

// Decompress nf streams; status per stream in st_out (the first error is
// returned).  A stream whose header cannot be used is reported and skipped;
// the others are still decoded.
// Geometry of a decompress call whose coded streams' sizes and plans are
// set; returns the workspace bytes the call needs.
static size_t decompress_need(Call& c, const std::vector<int>& coded) {
  build_items(c, coded);
  c.forced_global = spiht_forced_global();
  c.need_lists = false;
  for (int i = 0; i < c.nf; i++)   // (the cut tile of a byte-cut residual decodes with global-memory lists)
    if (coded[i]) c.need_lists |= c.forced_global || c.plans[i]->ncls[2] > 0 || c.Fh[i].bt;
  return layout_call(c, nullptr, coded);
}

// Copies the first 48 bytes of each stream (device) to hdr (host); streams
// shorter than a header leave zeros.  The headers are gathered by kernels
// into the stream's pinned staging buffer (mapped host memory), then read
// after one wait: no copy per stream.
static int read_headers(const std::vector<const uint8_t*>& d_in, const std::vector<size_t>& len,
                        std::vector<uint8_t>& hdr, hipStream_t st) {
  const size_t n = d_in.size();
  hdr.assign(kHdr * n, 0);
  for (size_t i = 0; i < n; i++)
    if (!d_in[i]) return fail(EBCC_EINVAL, "NULL buffer");
  WS* ws = nullptr;
  if (int rc = get_ws(st, &ws)) return rc;
  char* base = nullptr;
  if (int rc = grow_ws(ws, 0, kHdr * n, st, &base)) return rc;
  uint8_t* d_pin = nullptr;
  HIPCHK(hipHostGetDevicePointer((void**)&d_pin, ws->pin, 0));
  for (size_t i0 = 0; i0 < n; i0 += kHdrArgs) {
    const int m = (int)std::min<size_t>(kHdrArgs, n - i0);
    HdrArgs a;
    for (int k = 0; k < kHdrArgs; k++) {
      const bool in = k < m && len[i0 + k] >= (size_t)kHdr;
      a.p[k] = in ? d_in[i0 + k] : nullptr;
      a.ok[k] = in ? 1 : 0;
    }
    k_read_headers<<<m, 64, 0, st>>>(a, m, d_pin + kHdr * i0);
  }
  HIPCHK(hipGetLastError());
  if (int rc = wait_stream(st)) return rc;
  memcpy(hdr.data(), ws->pin, kHdr * n);
  return EBCC_OK;
}

// The decode calls of a batch: one launch sequence decodes streams of one
// code-block size, so the coded streams are grouped by it (in order of first
// appearance; the others join the first group), and each group is cut into
// chunks of at most kChunkSamples samples or kChunkFields streams.
static std::vector<std::vector<int>> decode_calls(int n, const uint8_t* hdrs, const size_t* len, const size_t* ny,
                                                  const size_t* nx) {
  std::vector<int> key(n, -1);
  std::vector<int> order;
  for (int i = 0; i < n; i++) {
    const uint8_t* h = hdrs + kHdr * (size_t)i;
    if (len[i] >= (size_t)kHdr && memcmp(h, "EBCC", 4) == 0 && h[5] == MODE_CODED) key[i] = h[7];
    if (key[i] >= 0 && std::find(order.begin(), order.end(), key[i]) == order.end()) order.push_back(key[i]);
  }
  if (order.empty()) order.push_back(-1);
  std::vector<std::vector<int>> calls;
  for (size_t g = 0; g < order.size(); g++) {
    std::vector<int> idx;
    for (int i = 0; i < n; i++)
      if (key[i] == order[g] || (g == 0 && key[i] < 0)) idx.push_back(i);
    size_t k = 0;
    while (k < idx.size()) {
      std::vector<int> call;
      size_t samples = 0;
      while (k < idx.size() && (call.empty() || samples + ny[idx[k]] * nx[idx[k]] <= kChunkSamples) &&
             (int)call.size() < kChunkFields) {
        samples += ny[idx[k]] * nx[idx[k]];
        call.push_back(idx[k++]);
      }
      calls.push_back(call);
    }
  }
  return calls;
}

// The launch sequence that decodes the coded fields of a call (c.F's active
// entries), from the block and tile tables to the output: c.Fc holds the
// fields with a residual (scratch of the residual's inverse DWT in BUF_CRES),
// c.Fc + nf those without one; Frh and Fnh are their host copies (grid
// sizes).  anyres / anynores / anybt may be set when no field needs them:
// the kernels skip inactive fields, fields without a residual section and
// residuals not cut at a byte position.
static int decode_sequence(Call& c, Prof& prof, bool anyres, bool anynores, bool anybt, const FieldDev* Frh,
                           const FieldDev* Fnh, size_t maxN, hipStream_t s) {
  const int nf = c.nf;
  FieldDev* const Fnd = c.Fc + nf;
  k_read_blocks<<<grid_for(c.nblk), 256, 0, s>>>(c.F, c.d_blk, c.nblk, c.bent);
  k_scan<<<nf, 1024, 0, s>>>(c.F, c.bent, 0, 16, 0xFFFFu, c.boff);
  k_read_tiles<<<grid_for(c.ntiles), 256, 0, s>>>(c.F, c.d_tiles, c.ntiles, c.tent);
  k_scan<<<nf, 1024, 0, s>>>(c.F, c.tent, 1, 0, 0x3FFFFFFu, c.toff);
  k_check_tables<<<(nf + 63) / 64, 64, 0, s>>>(c.F, nf);
  prof.mark(S_D_PARSE);
  if (anyres) {
    // The residual layer decodes independently of the base layer: SPIHT
    // runs on the second and third streams while tier-1 decoding and the
    // base inverse DWT run on the caller's (the SPIHT kernels skip
    // fields without a residual section).
    k_fill<<<dim3(grid_for(maxN), nf), 256, 0, s>>>(c.F, BUF_CHAT, 0.0f);
    hipStream_t sa = c.ws->aux;
    if (int rc2 = c.fork_from(s)) return rc2;
    if (anybt) spiht_decode_cut(c.F, nf, c.d_tiles, c.toff, c.lists, sa);
    if (c.forced_global) {
      spiht_decode(c.F, c.d_tiles, c.d_tix, c.ntiles, c.toff, c.lists, sa);
    } else {
      // small tiles on one stream, the larger classes on another
      const int *t0 = c.d_tix, *t1 = t0 + c.ncls[0], *t2 = t1 + c.ncls[1], *t3 = t2 + c.ncls[2];
      hipStream_t sb = c.ws->aux2;
      // the LDS classes' tiles longest payload first (batches: the
      // longest decodes start first)
      int *o0 = c.tix_sorted, *o1 = o0 + c.ncls[0];
      spiht_tiles_longest_first(t0, c.ncls[0], c.tent, o0, sa);
      spiht_tiles_longest_first(t1, c.ncls[1], c.tent, o1, sb);
      spiht_decode(c.F, c.d_tiles, t2, c.ncls[2], c.toff, c.lists, sb);
      spiht_decode_lds(kSpihtHuge, c.F, c.d_tiles, t3, c.ncls[3], c.toff, c.misfit, sb);
      spiht_decode_lds(kSpihtBig, c.F, c.d_tiles, o1, c.ncls[1], c.toff, c.misfit, sb);
      spiht_decode_lds(kSpihtSmall, c.F, c.d_tiles, o0, c.ncls[0], c.toff, c.misfit, sa);
    }
    // all of the residual's inverse DWT but its last pass, in the shadow
    // of tier-1 decoding, once both SPIHT streams are done
    hipStream_t sb = c.ws->aux2;
    HIPCHK(hipEventRecord(c.ws->ev_join, sa));
    HIPCHK(hipStreamWaitEvent(sb, c.ws->ev_join, 0));
    dwt_inverse_head(c.Fc, Frh, nf, BUF_CHAT, sb);
  }
  // (no scalar/vector split here: the second stream is busy with SPIHT)
  t1_decode(c.F, c.d_blk, c.nblk, c.cbw, c.cbh, c.bent, c.boff, s, nullptr, c.border, c.qctr, c.any_byp);
  prof.mark(S_D_T1);
  dwt_inverse(c.F, c.Fh.data(), nf, BUF_YHAT, BUF_ABASE, EPI_STORE, s);
  prof.mark(S_D_IDWT_BASE);
  if (anyres) {
    if (int rc2 = c.join_to(s)) return rc2;
    prof.mark(S_D_SPIHT);
    dwt_inverse_tail(c.Fc, Frh, nf, BUF_CHAT, BUF_CHAT, EPI_FINAL, s);
  }
  if (anynores) pointwise(Fnd, Fnh, nf, BUF_CHAT, BUF_CHAT, 3, EPI_FINAL, 0, s);
  prof.mark(S_D_FINAL);
  HIPCHK(hipGetLastError());
  return EBCC_OK;
}

static int decompress_call(const std::vector<StreamIn>& in, const uint8_t* hdrs, std::vector<int>& st_out,
                           hipStream_t st) {
  const int nf = (int)in.size();
  st_out.assign(nf, EBCC_OK);
  if (nf == 0) return EBCC_OK;
  for (int i = 0; i < nf; i++)
    if (!in[i].in || !in[i].x) return fail(EBCC_EINVAL, "NULL buffer");
  std::vector<uint8_t> hdr(hdrs, hdrs + kHdr * (size_t)nf);
  Call c;
  c.nf = nf;
  c.st = st;
  c.Fh.assign(nf, FieldDev());
  c.plans.assign(nf, nullptr);
  std::vector<int> mode(nf, MODE_CONST), coded(nf, 0), good(nf, 0);
  std::vector<float> xr(2 * (size_t)nf, 0.0f);
  int rc, cbl2w = -1, cbl2h = -1;
  int first = EBCC_OK;
  auto bad = [&](int i, int code, const char* msg) {
    st_out[i] = code;
    if (first == EBCC_OK) first = fail(code, std::string(msg) + " (stream " + std::to_string(i) + ")");
  };
  for (int i = 0; i < nf; i++) {
    FieldDev& f = c.Fh[i];
    memset(&f, 0, sizeof(f));
    if (in[i].len < (size_t)kHdr) { bad(i, EBCC_ECORRUPT, "stream shorter than its header"); continue; }
    const uint8_t* h = hdr.data() + kHdr * (size_t)i;
    size_t hny, hnx;
    if (ebcc_stream_info(h, kHdr, &hny, &hnx, &mode[i]) != EBCC_OK) { bad(i, EBCC_ECORRUPT, "bad stream header"); continue; }
    if (hny != in[i].ny || hnx != in[i].nx || hny < 1 || hnx < 1 || hny * hnx > 0x7FFFFFFFull) {
      bad(i, EBCC_EINVAL, "dimensions do not match the stream");
      continue;
    }
    f.ny = (int)hny; f.nx = (int)hnx;
    size_t N = hny * hnx;
    f.bb = rd32(h + 36); f.rb = rd32(h + 40);
    f.len = (int64_t)in[i].len;
    if ((size_t)kHdr + f.bb + f.rb != in[i].len) { bad(i, EBCC_ECORRUPT, "stream length does not match its header"); continue; }
    if (mode[i] == MODE_RAW && f.bb != 4 * N) { bad(i, EBCC_ECORRUPT, "raw stream of the wrong size"); continue; }
    memcpy(&xr[2 * i], h + 16, 4);
    memcpy(&xr[2 * i + 1], h + 20, 4);
    f.out = const_cast<uint8_t*>(in[i].in);
    f.mode = mode[i];
    if (mode[i] == MODE_CODED) {
      int L = h[6], w2 = h[7] & 15, h2 = h[7] >> 4, T = h[32] | (h[33] << 8);
      f.e0 = (int8_t)h[28]; f.er = (int8_t)h[29]; f.ns = (int8_t)h[31];
      if (L != levels_eff(f.ny, f.nx, L) || w2 < 2 || w2 > 6 || h2 < 2 || h2 > 6 || T < 1 || T > 64 || f.ns < 0 ||
          f.ns >= kQBits) {
        bad(i, EBCC_ECORRUPT, "bad coding parameters in the header");
        continue;
      }
      if (cbl2w >= 0 && (w2 != cbl2w || h2 != cbl2h)) {
        bad(i, EBCC_EINVAL, "internal: streams decoded together must share the code-block size");
        continue;
      }
      f.L = L; f.T = T;
      f.bt = f.rb ? (h[34] & 1) : 0;
      f.byp = h[35] & 1;
      c.any_byp |= f.byp != 0;
      if ((rc = get_plan(f.ny, f.nx, L, w2, h2, T, &c.plans[i]))) return rc;
      if ((int64_t)f.bb < 4 * (int64_t)c.plans[i]->nblk) { bad(i, EBCC_ECORRUPT, "base section shorter than its table"); continue; }
      if (f.rb && (int64_t)f.rb < 4 * (int64_t)c.plans[i]->ntiles + (f.bt ? 8 : 0)) {
        bad(i, EBCC_ECORRUPT, "residual section shorter than its table");
        continue;
      }
      cbl2w = w2; cbl2h = h2;
      f.bands = c.plans[i]->d_bands;
      f.nb = c.plans[i]->nb;
      coded[i] = 1;
    }
    good[i] = 1;
  }
  if (cbl2w >= 0) { c.cbw = 1 << cbl2w; c.cbh = 1 << cbl2h; }
  bool anycoded = false;
  for (int i = 0; i < nf; i++) anycoded |= coded[i] != 0;
  size_t need_ws = decompress_need(c, coded);
  char* base;
  if ((rc = get_ws(st, &c.ws))) return rc;
  if ((rc = grow_ws(c.ws, need_ws, pin_need(c), st, &base))) return rc;
  layout_call(c, base, coded);
  for (int i = 0; i < nf; i++) {
    c.Fh[i].buf[BUF_XOUT] = in[i].x;
    c.Fh[i].active = good[i];
  }
  Prof prof(st);
  if ((rc = upload_items(c, coded))) return rc;
  float* d_xr = reinterpret_cast<float*>(c.collect);   // reuse: 2 floats per field fit 8 int64 per field
  if ((rc = c.stage(d_xr, xr.data(), sizeof(float) * xr.size()))) return rc;
  std::vector<int> all(good);
  if ((rc = c.set_active(all))) return rc;
  k_set_decode<<<(nf + 63) / 64, 64, 0, st>>>(c.F, nf, d_xr);
  size_t maxN = 0;
  for (auto& f : c.Fh) maxN = std::max(maxN, (size_t)f.ny * f.nx);
  k_checksum<<<dim3(grid_sweep(maxN), nf), 256, 0, st>>>(c.F);
  std::vector<int> cm(nf, 0), rm(nf, 0), cd(nf, 0), cr(nf, 0), cn(nf, 0);
  bool anyc = false, anyr = false, anyres = false, anynores = false;
  for (int i = 0; i < nf; i++) {
    if (!good[i]) continue;
    if (mode[i] == MODE_CONST) { cm[i] = 1; anyc = true; }
    if (mode[i] == MODE_RAW) { rm[i] = 1; anyr = true; }
    if (coded[i]) {
      cd[i] = 1;
      if (c.Fh[i].rb) { cr[i] = 1; anyres = true; } else { cn[i] = 1; anynores = true; }
    }
  }
  if (anyc) {
    if ((rc = c.set_active(cm))) return rc;
    k_fill<<<dim3(grid_for(maxN), nf), 256, 0, st>>>(c.F, BUF_XOUT, __builtin_nanf(""));
  }
  if (anyr) {
    if ((rc = c.set_active(rm))) return rc;
    k_copy_raw<<<dim3(grid_for(maxN), nf), 256, 0, st>>>(c.F, 0);
  }
  if (anycoded) {
    // Tables of the launch sequence, all staged before it: the coded fields
    // (c.F), the fields with a residual whose inverse DWT runs on the third
    // stream, scratch in BUF_CRES (unused when decoding) so that it does not
    // meet the base transform's BUF_TMP (c.Fc), the fields without one
    // (c.Fc + nf).  The sequence itself is only launches, so it runs from a
    // cached HIP graph when one matches the call.
    if ((rc = c.set_active(cd))) return rc;
    std::vector<FieldDev> Fr, Fn;
    if (anyres) {
      Fr = c.Fh;
      for (int i = 0; i < nf; i++) {
        Fr[i].active = cr[i];
        Fr[i].buf[BUF_TMP] = Fr[i].buf[BUF_CRES];
      }
      if ((rc = c.stage(c.Fc, Fr.data(), sizeof(FieldDev) * nf))) return rc;
    }
    FieldDev* const Fnd = c.Fc + nf;
    if (anynores) {
      Fn = c.Fh;
      for (int i = 0; i < nf; i++) Fn[i].active = cn[i];
      if ((rc = c.stage(Fnd, Fn.data(), sizeof(FieldDev) * nf))) return rc;
    }
    bool anybt = false;
    for (int i = 0; i < nf; i++) anybt |= cr[i] && c.Fh[i].bt;
    auto seq = [&](hipStream_t s) -> int {
      return decode_sequence(c, prof, anyres, anynores, anybt, Fr.data(), Fn.data(), maxN, s);
    };
    if (graphs_usable(c, prof)) {
      GraphKey key("decode", c);
      key.add(anyres); key.add(anynores); key.add(anybt); key.add(maxN);
      for (int i = 0; i < nf; i++) { key.add(cd[i]); key.add(cr[i]); key.add(cn[i]); }
      if ((rc = run_graph(key, c, seq))) return rc;
    } else if ((rc = seq(st))) {
      return rc;
    }
  }
  HIPCHK(hipGetLastError());
  if ((rc = c.set_active(all))) return rc;
  std::vector<int64_t> col;
  if ((rc = c.collect_host(col))) return rc;
  for (int i = 0; i < nf; i++) {
    if (!good[i]) continue;
    uint32_t csum = rd32(hdr.data() + kHdr * (size_t)i + 44);
    if (col[8 * i + 1]) bad(i, EBCC_ECORRUPT, "inconsistent block or tile tables");
    else if ((uint32_t)col[8 * i + 3] != csum) bad(i, EBCC_ECORRUPT, "checksum mismatch");
  }
  return first;
}

// Asynchronous batched decoding of streams [i0, i0 + m) of
// ebcc_decompress_batch_async: every field is laid out as coded with the
// call's parameters (geometry known on the host); the headers are checked
// and the fields' roles chosen on the device, every role's launches run and
// skip the fields that are not theirs, and the statuses stay on the device.
// Nothing waits for the device.
static int decompress_async_chunk(const uint8_t* d_in, const uint64_t* d_offs, const uint64_t* d_lens, int i0, int m,
                                  float* const* d_x, const size_t* ny, const size_t* nx, const ebcc_params* p,
                                  int32_t* d_status, hipStream_t st) {
  Call c;
  c.nf = m;
  c.st = st;
  c.Fh.assign(m, FieldDev());
  c.plans.assign(m, nullptr);
  const int w2 = (int)p->cblk_log2w, h2 = (int)p->cblk_log2h, T = (int)p->spiht_tile;
  std::vector<int> coded(m, 1);
  int rc;
  for (int k = 0; k < m; k++) {
    FieldDev& f = c.Fh[k];
    memset(&f, 0, sizeof(f));
    f.ny = (int)ny[i0 + k];
    f.nx = (int)nx[i0 + k];
    f.L = levels_eff(f.ny, f.nx, (int)p->levels);
    f.cbl = w2 | (h2 << 4);
    f.T = T;
    f.mode = MODE_CODED;
    f.active = 1;
    f.bt = (int)p->trunc;
    f.byp = (int)p->bypass;
    if ((rc = get_plan(f.ny, f.nx, f.L, w2, h2, T, &c.plans[k]))) return rc;
    f.bands = c.plans[k]->d_bands;
    f.nb = c.plans[k]->nb;
  }
  c.cbw = 1 << w2;
  c.cbh = 1 << h2;
  c.any_byp = p->bypass != 0;
  const size_t need_ws = decompress_need(c, coded);
  char* base;
  if ((rc = get_ws(st, &c.ws))) return rc;
  if ((rc = grow_ws(c.ws, need_ws, 0, st, &base))) return rc;
  layout_call(c, base, coded);
  for (int k = 0; k < m; k++) c.Fh[k].buf[BUF_XOUT] = d_x[i0 + k];
  // the field table and the item tables go through a staging area of the
  // call's own, free again once these copies have run
  const size_t stage_bytes = sizeof(FieldDev) * (size_t)m + sizeof(Blk) * (size_t)c.nblk +
                             (sizeof(TileD) + sizeof(int) + sizeof(int64_t)) * (size_t)c.ntiles + sizeof(int64_t) +
                             8 * 256;
  if ((rc = async_pin(c.ws, stage_bytes, &c.apin))) return rc;
  Prof prof(st);
  if ((rc = upload_items(c, coded))) return rc;
  if ((rc = c.upload())) return rc;
  HIPCHK(hipEventRecord(c.apin->ev, st));
  c.apin->live = true;
  size_t maxN = 0;
  for (auto& f : c.Fh) maxN = std::max(maxN, (size_t)f.ny * f.nx);
  const AsyncCfg cfg{w2 | (h2 << 4), T, (int)p->trunc, (int)p->bypass};
  int32_t* sts = d_status + i0;
  const int g = (m + 63) / 64;
  k_parse_async<<<g, 64, 0, st>>>(c.F, c.Fc, c.Fc + m, m, d_in, d_offs + i0, d_lens + i0, cfg, sts);
  k_checksum<<<dim3(grid_sweep(maxN), m), 256, 0, st>>>(c.F);
  k_select_async<<<g, 64, 0, st>>>(c.F, m, sts, MODE_CONST);
  k_fill<<<dim3(grid_for(maxN), m), 256, 0, st>>>(c.F, BUF_XOUT, __builtin_nanf(""));
  k_select_async<<<g, 64, 0, st>>>(c.F, m, sts, MODE_RAW);
  k_copy_raw<<<dim3(grid_for(maxN), m), 256, 0, st>>>(c.F, 0);
  k_select_async<<<g, 64, 0, st>>>(c.F, m, sts, MODE_CODED);
  const bool anybt = p->trunc != 0;
  auto seq = [&](hipStream_t s) -> int {
    return decode_sequence(c, prof, true, true, anybt, c.Fh.data(), c.Fh.data(), maxN, s);
  };
  if (graphs_usable(c, prof)) {
    GraphKey key("decode_async", c);
    key.add(anybt);
    key.add(maxN);
    if ((rc = run_graph(key, c, seq))) return rc;
  } else if ((rc = seq(st))) {
    return rc;
  }
  k_finish_async<<<g, 64, 0, st>>>(c.F, m, sts);
  HIPCHK(hipGetLastError());
  return EBCC_OK;
}

// ---------------------------------------------------------------------------
// Static scratch for callers that cannot allocate (ebcc_compress_noalloc).
// The array is a device symbol: host code reaches its memory only through
// the address hipGetSymbolAddress returns for the current device, taken once
// per device.  One host mutex per device serialises the calls that use it,
// and a call waits for its stream before releasing it, so the contents a
// call leaves are never read by the next one's kernels before they rewrite
// them.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

struct FixedScratch {
  std::mutex mu;
  WS ws;
};
static std::mutex g_fixed_mu;
static std::map<int, std::unique_ptr<FixedScratch>> g_fixed;

static int fixed_scratch(FixedScratch** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  auto it = g_fixed.find(dev);
  if (it != g_fixed.end()) { *out = it->second.get(); return EBCC_OK; }
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(EBCC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  std::unique_ptr<FixedScratch> f(new FixedScratch());
  f->ws.fixed = true;
  f->ws.base = ptr;
  f->ws.cap = kScratchBytes;
  *out = f.get();
  g_fixed[dev] = std::move(f);
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
  p->spiht_tile = 1;
  p->trunc = 0;
  p->bypass = 0;
}

size_t ebcc_compress_bound(size_t ny, size_t nx) { return (size_t)kHdr + 4 * ny * nx; }

int ebcc_compress(const float* d_x, size_t ny, size_t nx, const ebcc_params* p, uint8_t* d_out, size_t out_cap,
                  size_t* out_len, void* stream) {
  g_err.clear();
  if (!out_len) return fail(EBCC_EINVAL, "out_len is NULL");
  *out_len = 0;
  std::vector<FieldIn> in(1, FieldIn{d_x, ny, nx, p ? p->err_bound : 0.01});
  std::vector<uint64_t> offs, lens;
  size_t need = 0;
  int rc = compress_call(in, p, d_out, out_cap, offs, lens, &need, (hipStream_t)stream, nullptr);
  *out_len = rc == EBCC_ENOSPC ? need : (rc == EBCC_OK ? (size_t)lens[0] : 0);
  return rc;
}

int ebcc_compress_noalloc(const float* d_x, size_t ny, size_t nx, const ebcc_params* p, uint8_t* d_out,
                          size_t out_cap, size_t* out_len, void* stream) {
  g_err.clear();
  if (!out_len) return fail(EBCC_EINVAL, "out_len is NULL");
  *out_len = 0;
  FixedScratch* fs = nullptr;
  if (int rc = fixed_scratch(&fs)) return rc;
  std::lock_guard<std::mutex> lk(fs->mu);
  std::vector<FieldIn> in(1, FieldIn{d_x, ny, nx, p ? p->err_bound : 0.01});
  std::vector<uint64_t> offs, lens;
  size_t need = 0;
  hipStream_t st = (hipStream_t)stream;
  int rc = compress_call(in, p, d_out, out_cap, offs, lens, &need, st, nullptr, nullptr, &fs->ws);
  // the scratch is free for the next call only once this call's kernels are done
  hipError_t e = hipStreamSynchronize(st);
  if (rc == EBCC_OK && e != hipSuccess) rc = fail(EBCC_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  *out_len = rc == EBCC_ENOSPC ? need : (rc == EBCC_OK ? (size_t)lens[0] : 0);
  return rc;
}

int ebcc_compress_trace(const float* d_x, size_t ny, size_t nx, const ebcc_params* p, uint8_t* d_out, size_t out_cap,
                        size_t* out_len, void* stream, float* d_coef, float* d_abase, float* d_cres, uint8_t* d_kb,
                        uint8_t* d_pb, int32_t* h_info) {
  g_err.clear();
  if (!out_len) return fail(EBCC_EINVAL, "out_len is NULL");
  *out_len = 0;
  Trace tr{d_coef, d_abase, d_cres, d_kb, d_pb, h_info};
  std::vector<FieldIn> in(1, FieldIn{d_x, ny, nx, p ? p->err_bound : 0.01});
  std::vector<uint64_t> offs, lens;
  size_t need = 0;
  int rc = compress_call(in, p, d_out, out_cap, offs, lens, &need, (hipStream_t)stream, &tr);
  *out_len = rc == EBCC_ENOSPC ? need : (rc == EBCC_OK ? (size_t)lens[0] : 0);
  return rc;
}

int ebcc_compress_batch(int n, const float* const* d_x, const size_t* ny, const size_t* nx, const double* err_bounds,
                        const ebcc_params* p, uint8_t* d_out, size_t out_cap, uint64_t* h_offsets,
                        uint64_t* h_lengths, int* h_status, void* stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!d_x || !ny || !nx || !h_offsets || !h_lengths)))
    return fail(EBCC_EINVAL, "bad batch arguments");
  ebcc_params dflt;
  if (!p) { ebcc_params_default(&dflt); p = &dflt; }
  std::vector<int> stv(n, EBCC_OK);
  int first = EBCC_OK;
  std::string first_msg;
  auto note = [&](int rc) {
    if (rc != EBCC_OK && first == EBCC_OK) { first = rc; first_msg = g_err; }
  };
  // fields with bad arguments get their own status and no stream
  std::vector<int> ok;
  for (int i = 0; i < n; i++) {
    h_offsets[i] = 0; h_lengths[i] = 0;
    const double e = err_bounds ? err_bounds[i] : p->err_bound;
    int rc = check_params(ny[i], nx[i], p, e);
    if (rc == EBCC_OK && !d_x[i]) rc = fail(EBCC_EINVAL, "NULL input buffer");
    if (rc != EBCC_OK) { stv[i] = rc; note(rc); } else ok.push_back(i);
  }
  size_t done = 0;
  size_t k = 0;
  while (k < ok.size()) {
    // one chunk: consecutive fields up to kChunkSamples samples (at least one)
    std::vector<FieldIn> in;
    std::vector<int> idx;
    size_t samples = 0;
    while (k < ok.size() && (in.empty() || samples + ny[ok[k]] * nx[ok[k]] <= kChunkSamples) &&
           (int)in.size() < kChunkFields) {
      const int j = ok[k++];
      in.push_back(FieldIn{d_x[j], ny[j], nx[j], err_bounds ? err_bounds[j] : p->err_bound});
      idx.push_back(j);
      samples += ny[j] * nx[j];
    }
    std::vector<uint64_t> offs, lens;
    std::vector<int> fst;
    size_t need = 0;
    if (done > out_cap) {
      fail(EBCC_ENOSPC, "output capacity too small");
      for (int j : idx) stv[j] = EBCC_ENOSPC;
      note(EBCC_ENOSPC);
      continue;
    }
    int rc = compress_call(in, p, d_out + done, out_cap - done, offs, lens, &need, (hipStream_t)stream, nullptr, &fst);
    bool per_field = rc == EBCC_EINVAL && fst.size() == in.size();
    if (rc != EBCC_OK && !per_field) {
      for (int j : idx) stv[j] = rc;   // a failure of the whole chunk
      note(rc);
      if (rc != EBCC_ENOSPC) continue;
      done += need;                    // the space the chunk would have taken
      continue;
    }
    note(rc);
    for (size_t m = 0; m < idx.size(); m++) {
      stv[idx[m]] = per_field ? fst[m] : EBCC_OK;
      h_offsets[idx[m]] = done + offs[m];
      h_lengths[idx[m]] = lens[m];
    }
    done += need;
  }
  if (h_status)
    for (int i = 0; i < n; i++) h_status[i] = stv[i];
  if (first) g_err = first_msg;
  return first;
}

int ebcc_decompress(const uint8_t* d_in, size_t in_len, float* d_x, size_t ny, size_t nx, void* stream) {
  g_err.clear();
  if (!d_in || !d_x) return fail(EBCC_EINVAL, "NULL buffer");
  std::vector<StreamIn> in(1, StreamIn{d_in, in_len, d_x, ny, nx});
  std::vector<uint8_t> hdr;
  if (int rc = read_headers({d_in}, {in_len}, hdr, (hipStream_t)stream)) return rc;
  std::vector<int> st;
  return decompress_call(in, hdr.data(), st, (hipStream_t)stream);
}

int ebcc_decompress_batch(int n, const uint8_t* const* d_in, const size_t* in_len, float* const* d_x,
                          const size_t* ny, const size_t* nx, int* h_status, void* stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!d_in || !in_len || !d_x || !ny || !nx)))
    return fail(EBCC_EINVAL, "bad batch arguments");
  if (n == 0) return EBCC_OK;
  for (int i = 0; i < n; i++)
    if (!d_in[i] || !d_x[i]) return fail(EBCC_EINVAL, "NULL buffer in the batch");
  std::vector<uint8_t> hdr;
  if (int rc = read_headers(std::vector<const uint8_t*>(d_in, d_in + n), std::vector<size_t>(in_len, in_len + n), hdr,
                            (hipStream_t)stream))
    return rc;
  int first = EBCC_OK;
  std::string first_msg;
  for (const std::vector<int>& call : decode_calls(n, hdr.data(), in_len, ny, nx)) {
    std::vector<StreamIn> in;
    std::vector<uint8_t> h;
    for (int k : call) {
      in.push_back(StreamIn{d_in[k], in_len[k], d_x[k], ny[k], nx[k]});
      h.insert(h.end(), hdr.begin() + kHdr * (size_t)k, hdr.begin() + kHdr * (size_t)(k + 1));
    }
    std::vector<int> st;
    int rc = decompress_call(in, h.data(), st, (hipStream_t)stream);
    bool per_stream = false;
    for (int v : st) per_stream |= v != EBCC_OK;
    if (rc && !per_stream) st.assign(call.size(), rc);   // a failure of the whole call
    for (size_t k = 0; k < call.size(); k++)
      if (h_status) h_status[call[k]] = st.empty() ? rc : st[k];
    if (rc && first == EBCC_OK) { first = rc; first_msg = g_err; }
  }
  if (first) g_err = first_msg;
  return first;
}

int ebcc_decompress_batch_async(int n, const uint8_t* d_in, const uint64_t* d_offsets, const uint64_t* d_lengths,
                                float* const* d_x, const size_t* ny, const size_t* nx, const ebcc_params* p,
                                int32_t* d_status, void* stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!d_in || !d_offsets || !d_lengths || !d_x || !ny || !nx || !d_status)))
    return fail(EBCC_EINVAL, "bad batch arguments");
  ebcc_params dflt;
  if (!p) { ebcc_params_default(&dflt); p = &dflt; }
  for (int i = 0; i < n; i++) {
    if (int rc = check_params(ny[i], nx[i], p, 1.0)) return rc;
    if (!d_x[i]) return fail(EBCC_EINVAL, "NULL output buffer in the batch");
  }
  const hipStream_t st = (hipStream_t)stream;
  int i0 = 0;
  while (i0 < n) {
    // one chunk: consecutive streams up to kChunkSamples samples (at least one)
    int m = 0;
    size_t samples = 0;
    while (i0 + m < n && (m == 0 || samples + ny[i0 + m] * nx[i0 + m] <= kChunkSamples) && m < kChunkFields) {
      samples += ny[i0 + m] * nx[i0 + m];
      m++;
    }
    if (int rc = decompress_async_chunk(d_in, d_offsets, d_lengths, i0, m, d_x, ny, nx, p, d_status, st)) return rc;
    i0 += m;
  }
  return EBCC_OK;
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
  graphs_clear();
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
  prof_resolve(true);
  g_prof = on ? 1 : 0;
  for (int i = 0; i < S_COUNT; i++) { g_stage_ms[i] = 0.0; g_stage_calls[i] = 0; }
}

int ebcc_profile_read(double* ms, long* calls, int n) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_resolve(true);
  for (int i = 0; i < n && i < S_COUNT; i++) {
    if (ms) ms[i] = g_stage_ms[i];
    if (calls) calls[i] = g_stage_calls[i];
  }
  return S_COUNT;
}

int ebcc_tuning_get(ebcc_tuning* t) {
  if (!t) return fail(EBCC_EINVAL, "NULL tuning");
  Tuning v = tuning();
  t->struct_size = sizeof(ebcc_tuning);
  t->t1_encoder = v.t1_encoder;
  t->t1_decoder = v.t1_decoder;
  t->t1_wave_max = v.t1_wave_max;
  t->spiht = v.spiht;
  t->t1_lanes = v.t1_lanes;
  t->t1_split = v.t1_split;
  t->t1_persist = v.t1_persist;
  return EBCC_OK;
}

int ebcc_tuning_set(const ebcc_tuning* t) {
  if (!t || t->struct_size != sizeof(ebcc_tuning)) return fail(EBCC_EINVAL, "bad ebcc_tuning");
  if (t->t1_encoder < 0 || t->t1_encoder > 2 || t->t1_decoder < 0 || t->t1_decoder > 2 || t->t1_wave_max < 0 ||
      t->spiht < 0 || t->spiht > 1 ||
      !(t->t1_lanes == 0 || t->t1_lanes == 1 || t->t1_lanes == 4 || t->t1_lanes == 16 || t->t1_lanes == 64) ||
      t->t1_split < 0 || t->t1_split > 100 || t->t1_persist < 0 || t->t1_persist > 1)
    return fail(EBCC_EINVAL, "tuning value out of range");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuning = Tuning{t->t1_encoder, t->t1_decoder, t->t1_wave_max, t->spiht, t->t1_lanes, t->t1_split,
                    t->t1_persist};
  return EBCC_OK;
}

const char* ebcc_profile_stage_name(int i) { return (i >= 0 && i < S_COUNT) ? kStageNames[i] : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Workspace sizes: the same geometry and layout code as the calls, on
// host-only plans (no device memory is touched).
// ---------------------------------------------------------------------------
static size_t compress_ws(const std::vector<size_t>& ny, const std::vector<size_t>& nx, const ebcc_params* p) {
  Call c;
  c.nf = (int)ny.size();
  c.Fh.assign(c.nf, FieldDev());
  c.plans.assign(c.nf, nullptr);
  c.cbw = 1 << p->cblk_log2w;
  c.cbh = 1 << p->cblk_log2h;
  for (int i = 0; i < c.nf; i++) {
    FieldDev& f = c.Fh[i];
    memset(&f, 0, sizeof(f));
    f.ny = (int)ny[i]; f.nx = (int)nx[i];
    f.L = levels_eff(f.ny, f.nx, (int)p->levels);
    if (host_plan(f.ny, f.nx, f.L, p->cblk_log2w, p->cblk_log2h, (int)p->spiht_tile, &c.plans[i])) return 0;
  }
  std::vector<int> coded(c.nf, 1);
  c.want_cpos = p->trunc != 0;
  c.any_byp = p->bypass != 0;
  return ws_alloc(compress_need(c, coded));
}

static size_t decompress_ws(const std::vector<int>& call, const uint8_t* hdrs, const size_t* len, const size_t* ny,
                            const size_t* nx) {
  Call c;
  c.nf = (int)call.size();
  c.Fh.assign(c.nf, FieldDev());
  c.plans.assign(c.nf, nullptr);
  std::vector<int> coded(c.nf, 0);
  for (int m = 0; m < c.nf; m++) {
    const int i = call[m];
    const uint8_t* h = hdrs + kHdr * (size_t)i;
    FieldDev& f = c.Fh[m];
    memset(&f, 0, sizeof(f));
    f.ny = (int)ny[i]; f.nx = (int)nx[i];
    size_t hny, hnx;
    int mode;
    if (len[i] < (size_t)kHdr || ebcc_stream_info(h, kHdr, &hny, &hnx, &mode) != EBCC_OK || mode != MODE_CODED ||
        hny != ny[i] || hnx != nx[i] || hny * hnx > 0x7FFFFFFFull)
      continue;
    const int L = h[6], w2 = h[7] & 15, h2 = h[7] >> 4, T = h[32] | (h[33] << 8);
    if (L != levels_eff(f.ny, f.nx, L) || w2 < 2 || w2 > 6 || h2 < 2 || h2 > 6 || T < 1 || T > 64) continue;
    if (host_plan(f.ny, f.nx, L, w2, h2, T, &c.plans[m])) return 0;
    c.cbw = 1 << w2; c.cbh = 1 << h2;
    f.bt = h[34] & 1;
    coded[m] = 1;
  }
  return ws_alloc(decompress_need(c, coded));
}

extern "C" {

size_t ebcc_workspace_size(size_t ny, size_t nx, const ebcc_params* p) {
  g_err.clear();
  ebcc_params dflt;
  if (!p) { ebcc_params_default(&dflt); p = &dflt; }
  if (check_params(ny, nx, p, p->err_bound)) return 0;
  const int L = levels_eff((int)ny, (int)nx, (int)p->levels);
  Plan* pl = nullptr;
  if (host_plan((int)ny, (int)nx, L, p->cblk_log2w, p->cblk_log2h, (int)p->spiht_tile, &pl)) return 0;
  const size_t ws = compress_ws({ny}, {nx}, p);
  return ws ? ws + plan_table_bytes(*pl) : 0;
}

size_t ebcc_workspace_size_batch(int n, const size_t* ny, const size_t* nx, const ebcc_params* p,
                                 const uint8_t* h_hdrs, const size_t* in_len) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!ny || !nx)) || (h_hdrs && !in_len)) { fail(EBCC_EINVAL, "bad batch arguments"); return 0; }
  ebcc_params dflt;
  if (!p) { ebcc_params_default(&dflt); p = &dflt; }
  size_t best = 0;
  if (!h_hdrs) {
    std::vector<size_t> cy, cx;
    size_t samples = 0;
    auto flush = [&]() {
      if (cy.empty()) return true;
      size_t w = compress_ws(cy, cx, p);
      if (!w) return false;
      best = std::max(best, w);
      cy.clear(); cx.clear(); samples = 0;
      return true;
    };
    for (int i = 0; i < n; i++) {
      if (check_params(ny[i], nx[i], p, p->err_bound)) continue;   // such fields take no workspace
      if (!cy.empty() && (samples + ny[i] * nx[i] > kChunkSamples || (int)cy.size() >= kChunkFields))
        if (!flush()) return 0;
      cy.push_back(ny[i]); cx.push_back(nx[i]);
      samples += ny[i] * nx[i];
    }
    if (!flush()) return 0;
    return best;
  }
  for (const std::vector<int>& call : decode_calls(n, h_hdrs, in_len, ny, nx)) {
    size_t w = decompress_ws(call, h_hdrs, in_len, ny, nx);
    if (!w) return 0;
    best = std::max(best, w);
  }
  return best;
}

int ebcc_workspace_reserve(size_t bytes, void* stream) {
  g_err.clear();
  hipStream_t st = (hipStream_t)stream;
  WS* w = nullptr;
  if (int rc = get_ws(st, &w)) return rc;
  if (w->cap == bytes) return EBCC_OK;
  if (w->base) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(w->base));
    w->base = nullptr;
    w->cap = 0;
  }
  if (bytes && hipMalloc(&w->base, bytes) != hipSuccess) {
    w->base = nullptr;
    return fail(EBCC_ENOMEM, "workspace allocation failed");
  }
  w->cap = bytes;
  return EBCC_OK;
}

size_t ebcc_device_bytes(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  size_t t = 0;
  for (auto& kv : g_ws)
    if (kv.first.first == dev && kv.second) t += kv.second->cap;
  for (auto& kv : g_plans)
    if (std::get<0>(kv.first) == dev && kv.second) t += plan_table_bytes(*kv.second);
  return t;
}

}  // extern "C"
