// SPIHT (Said & Pearlman 1996) per tile with one wavefront per tile and the
// tile's coefficients and lists in LDS.
//
// Encoder: every list pass is processed 64 entries at a time.  Each lane takes
// one entry, computes the bits it emits and the entries it appends to each
// list; wavefront prefix sums place the bits in the output and the appended
// entries at the list tails, and removed entries are compacted in place.
// Entries appended to the LIS tail are reached by later chunks of the same
// pass, so the result is exactly the sequential algorithm's.
//
// Decoder: the bits decide what happens, so the LIS pass runs as
// wave-uniform code; the LIP pass skips runs of zero bits (insignificant
// entries) with one count-leading-zeros per run, and the refinement bits,
// whose positions are known, are read by all lanes at once.
//
// Tile-local coordinates: the tile's trees cover one rectangle per band;
// rectangles are numbered in band order, so a coefficient's local index is
// the rectangle's offset plus its raster index inside it.  LL roots come
// first, level-1 coefficients (which have no children) last.
#include "common.h"

namespace ebcc {


struct TileGeom {
  int r0[kMaxBands], c0[kMaxBands], hr[kMaxBands], wr[kMaxBands], off[kMaxBands + 1];
  uint64_t mg[kMaxBands];   // ceil(2^32 / wr): row of a rectangle index without a division
  int ncoef, nparents;
};

// Rectangles of the tile's trees (computed by lane 0).
__device__ void tile_geom(TileGeom& g, const Band* B, int nb, int L, const TileD& td) {
  g.r0[0] = td.i0; g.c0[0] = td.j0; g.hr[0] = td.i1 - td.i0; g.wr[0] = td.j1 - td.j0;
  for (int o = 1; o <= 3 && L > 0; o++) {
    int r1 = td.i1 < B[o].h ? td.i1 : B[o].h, c1 = td.j1 < B[o].w ? td.j1 : B[o].w;
    g.r0[o] = td.i0; g.c0[o] = td.j0;
    g.hr[o] = r1 > td.i0 ? r1 - td.i0 : 0;
    g.wr[o] = c1 > td.j0 ? c1 - td.j0 : 0;
  }
  for (int b = 4; b < nb; b++) {
    int pb = b - 3;
    if (g.hr[pb] == 0 || g.wr[pb] == 0) { g.r0[b] = g.c0[b] = 0; g.hr[b] = g.wr[b] = 0; continue; }
    int pr0 = g.r0[pb], pr1 = pr0 + g.hr[pb], pc0 = g.c0[pb], pc1 = pc0 + g.wr[pb];
    int r0 = 2 * pr0, r1 = (pr1 == B[pb].h) ? B[b].h : (2 * pr1 < B[b].h ? 2 * pr1 : B[b].h);
    int c0 = 2 * pc0, c1 = (pc1 == B[pb].w) ? B[b].w : (2 * pc1 < B[b].w ? 2 * pc1 : B[b].w);
    g.r0[b] = r0; g.c0[b] = c0;
    g.hr[b] = r1 > r0 ? r1 - r0 : 0;
    g.wr[b] = c1 > c0 ? c1 - c0 : 0;
  }
  int o = 0;
  for (int b = 0; b < nb; b++) {
    g.off[b] = o;
    o += g.hr[b] * g.wr[b];
    g.mg[b] = g.wr[b] > 0 ? ((1ull << 32) + (uint64_t)g.wr[b] - 1) / (uint64_t)g.wr[b] : 0;
  }
  g.off[nb] = o;
  g.ncoef = o;
  g.nparents = L >= 1 ? g.off[1 + 3 * (L - 1)] : 0;
}

__device__ __forceinline__ int band_of(const TileGeom& g, int nb, int local) {
  int b = nb - 1;
  while (b > 0 && local < g.off[b]) b--;
  return b;
}

// Position in the field (Mallat layout) of the tile coefficient `loc`.
__device__ __forceinline__ int loc_to_pos(const TileGeom& g, const Band* B, int nb, int nx, int loc) {
  const int b = band_of(g, nb, loc);
  const int rel = loc - g.off[b];
  const int li = (int)(((uint64_t)rel * g.mg[b]) >> 32), lj = rel - li * g.wr[b];
  return (B[b].y0 + g.r0[b] + li) * nx + B[b].x0 + g.c0[b] + lj;
}

// Offspring (local indices, row-major) of the node with local index `loc`.
__device__ __forceinline__ int offspring_local(const TileGeom& g, const Band* B, int nb, int L, int loc, int* ch,
                                               int* clevel) {
  int b = band_of(g, nb, loc);
  int rel = loc - g.off[b];
  // exact: rel * wr < 2^32 for tiles of up to 2^16 coefficients
  int li = (int)(((uint64_t)rel * g.mg[b]) >> 32), lj = rel - li * g.wr[b];
  int i = g.r0[b] + li, j = g.c0[b] + lj;
  int k = 0;
  if (b == 0) {
    *clevel = L;
    if (L == 0) return 0;
    for (int c = 1; c <= 3; c++)
      if (i < B[c].h && j < B[c].w) ch[k++] = g.off[c] + (i - g.r0[c]) * g.wr[c] + (j - g.c0[c]);
    return k;
  }
  *clevel = B[b].level - 1;
  if (B[b].level == 1) return 0;
  int cb = b + 3;
  int r1 = (i == B[b].h - 1) ? B[cb].h : 2 * i + 2;
  int c1 = (j == B[b].w - 1) ? B[cb].w : 2 * j + 2;
  if (r1 > B[cb].h) r1 = B[cb].h;
  if (c1 > B[cb].w) c1 = B[cb].w;
  for (int r = 2 * i; r < r1; r++)
    for (int c = 2 * j; c < c1; c++) ch[k++] = g.off[cb] + (r - g.r0[cb]) * g.wr[cb] + (c - g.c0[cb]);
  return k;
}

__device__ __forceinline__ int wscan_excl(int v, int lane, int* total) {
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  // the total is the same in every lane: readfirstlane tells the compiler,
  // which keeps the counters it feeds in scalar registers and the loops
  // they bound wave-uniform
  *total = __builtin_amdgcn_readfirstlane(__shfl(x, 63));
  return x - v;
}

// OR nb (<= 32) bits of v (MSB first) at bit offset rel of the window; the
// window's words hold stream bits big-endian (bit 31 first).
__device__ __forceinline__ void put_bits(uint32_t* bw, int rel, int nb, uint32_t v) {
  if (nb <= 0) return;
  int w = rel >> 5, b = rel & 31;
  if (b + nb <= 32) {
    atomicOr(&bw[w], v << (32 - b - nb));
  } else {
    int n1 = 32 - b, n2 = nb - n1;
    atomicOr(&bw[w], v >> n2);
    atomicOr(&bw[w + 1], v << (32 - n2));
  }
}
__device__ __forceinline__ uint32_t bswap32(uint32_t v) {
  return (v >> 24) | ((v >> 8) & 0xFF00u) | ((v << 8) & 0xFF0000u) | (v << 24);
}
__device__ __forceinline__ int blen(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

template <int CAP>
struct SpihtLds {
  Band B[kMaxBands];
  TileGeom g;
  uint32_t qv[CAP];          // magnitude | sign << 31 (decoder: decoded magnitude)
  uint8_t mdl[CAP / 4];      // bit length of the max over descendants (per parent)
  uint8_t mll[CAP / 4];      // bit length of the max over grand-descendants
  uint16_t lip[CAP], lsp[CAP];
  uint16_t lis[CAP / 2];     // local index | typeB << 15 (at most twice the parents)
  uint32_t bw[72];           // encoder output window (2048 bits + slack)
  int ntop, ok;
};

// Load the tile's geometry and coefficients; returns false when it does not fit.
template <int CAP>
__device__ bool spiht_setup(SpihtLds<CAP>& S, const Band* bands_g, int nb, int L, const TileD& td, int lane) {
  for (int i = lane; i < nb; i += 64) S.B[i] = bands_g[i];
  __syncthreads();
  if (lane == 0) {
    tile_geom(S.g, S.B, nb, L, td);
    S.ok = S.g.ncoef <= CAP && 4 * S.g.nparents <= CAP;
  }
  __syncthreads();
  return S.ok;
}

template <int CAP>
__global__ __launch_bounds__(64) void k_spiht_encode_lds(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                         const int* __restrict__ tix, uint8_t* __restrict__ slots,
                                                         const int64_t* __restrict__ slot_off,
                                                         uint32_t* __restrict__ tlen, uint32_t* __restrict__ tent,
                                                         uint32_t* __restrict__ tcut, int* __restrict__ misfit) {
  __shared__ SpihtLds<CAP> S;
  const int lane = threadIdx.x;
  const int t = tix[blockIdx.x];
  const TileD td = tiles[t];
  const FieldDev& f = F[td.field];
  if (!f.active) return;
  const uint32_t *qr = f.qr, *sub = f.sub, *maxd = f.maxd, *maxl = f.maxl;
  // byte-cut fields: the positions of the last plane's bits and the tile's
  // bit counts around that plane
  uint32_t* const cpos = f.cpos;
  const bool cut = cpos != nullptr;
  const Band* bands_g = f.bands;
  const int nx = f.nx, nb = f.nb, L = f.L, n_s = f.ns;
  if (!spiht_setup<CAP>(S, bands_g, nb, L, td, lane)) {
    if (lane == 0) misfit[t] = 1;
    return;
  }
  if (lane == 0) misfit[t] = 0;
  const TileGeom& g = S.g;
  // coefficients and descendant maxima into LDS; the tile's top plane
  // four samples per lane at a time, their global loads issued together
  // (a generic pointer may alias LDS, so loads written between LDS stores
  // would each wait for the one before)
  uint32_t mx = 0;
  for (int b = 0; b < nb; b++) {
    const int n = g.hr[b] * g.wr[b], wr = g.wr[b];
    const int y0 = S.B[b].y0 + g.r0[b], x0 = S.B[b].x0 + g.c0[b], off = g.off[b];
    for (int r0 = 0; r0 < n; r0 += 256) {
      int p[4];
      uint32_t qv[4], md[4], ml[4], sv[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int r = r0 + 64 * u + lane;
        const int rc = r < n ? r : n - 1;   // in bounds; the value is dropped
        const int li = rc / wr, lj = rc - li * wr;
        p[u] = (y0 + li) * nx + x0 + lj;
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const bool par = off + r0 + 64 * u + lane < g.nparents;
        qv[u] = qr[p[u]];
        md[u] = par ? maxd[p[u]] : 0u;
        ml[u] = par ? maxl[p[u]] : 0u;
        sv[u] = b == 0 ? sub[p[u]] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int r = r0 + 64 * u + lane;
        if (r >= n) continue;
        const int loc = off + r;
        S.qv[loc] = qv[u];
        if (loc < g.nparents) {
          S.mdl[loc] = (uint8_t)blen(md[u]);
          S.mll[loc] = (uint8_t)blen(ml[u]);
        }
        if (b == 0) mx = sv[u] > mx ? sv[u] : mx;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) { uint32_t v = __shfl_xor(mx, o); mx = v > mx ? v : mx; }
  mx = (uint32_t)__builtin_amdgcn_readfirstlane((int)mx);
  const int ntop = mx ? 31 - __builtin_clz(mx) : -1;
  if (ntop < n_s) {
    if (lane == 0) {
      tlen[t] = 0; tent[t] = 0;
      if (cut) { tcut[3 * t] = 0; tcut[3 * t + 1] = 0; tcut[3 * t + 2] = 0; }
    }
    return;
  }
  // initial lists: LIP = roots, LIS = roots with offspring (type A)
  const int nroots = g.hr[0] * g.wr[0];
  int nlis = 0;
  for (int r0 = 0; r0 < nroots; r0 += 64) {
    int r = r0 + lane;
    int ch[9], cl;
    int has = 0;
    if (r < nroots) {
      S.lip[r] = (uint16_t)r;
      has = offspring_local(g, S.B, nb, L, r, ch, &cl) > 0;
    }
    int tot;
    int pre = wscan_excl(has, lane, &tot);
    if (has) S.lis[nlis + pre] = (uint16_t)r;
    nlis += tot;
  }
  for (int i = lane; i < 72; i += 64) S.bw[i] = 0;
  __syncthreads();
  int nlip = nroots, nlsp = 0;
  int64_t bitpos = 0, wbase = 0;       // bits emitted; stream bit index of bw[0]
  uint8_t* out = slots + slot_off[t];
  const int64_t cap_bytes = slot_off[t + 1] - slot_off[t];
  auto flush = [&](bool final) {
    __syncthreads();
    int nfull = (int)((bitpos - wbase) >> 5);
    int nw = final ? (int)((bitpos - wbase + 31) >> 5) : nfull;
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out + (wbase >> 3));
    for (int i = lane; i < nw; i += 64)
      if ((wbase >> 3) + 4 * (int64_t)i + 4 <= cap_bytes) o32[i] = bswap32(S.bw[i]);
    if (!final && nfull > 0) {
      uint32_t part = S.bw[nfull];
      __syncthreads();
      for (int i = lane; i < 72; i += 64) S.bw[i] = (i == 0) ? part : 0u;
      wbase += 32 * (int64_t)nfull;
    }
    __syncthreads();
  };
  for (int pl = ntop; pl >= n_s; pl--) {
    const uint32_t thr = 1u << pl;
    const int lsp_prev = nlsp;
    const bool last = cut && pl == n_s;   // wave-uniform
    if (last && lane == 0) tcut[3 * t] = (uint32_t)bitpos;
    // sorting pass, LIP
    int surv = 0;
    for (int h0 = 0; h0 < nlip; h0 += 64) {
      int k = h0 + lane;
      bool act = k < nlip;
      int e = act ? S.lip[k] : 0;
      uint32_t q = act ? S.qv[e] : 0u;
      int s = act && (q & 0x7FFFFFu) >= thr;
      int nbits = act ? (s ? 2 : 1) : 0;
      uint32_t v = s ? (2u | (q >> 31)) : 0u;
      int tb, ts, tl;
      int pb = wscan_excl(nbits, lane, &tb);
      int ps = wscan_excl(s, lane, &ts);
      int pk = wscan_excl(act && !s, lane, &tl);
      __syncthreads();
      put_bits(S.bw, (int)(bitpos - wbase) + pb, nbits, v);
      if (s) S.lsp[nlsp + ps] = (uint16_t)e;
      if (act && !s) S.lip[surv + pk] = (uint16_t)e;
      if (last && s) cpos[loc_to_pos(g, S.B, nb, nx, e)] = (uint32_t)(bitpos + pb + 1);   // its sign bit
      bitpos += tb; nlsp += ts; surv += tl;
      flush(false);
    }
    nlip = surv;
    // sorting pass, LIS (grows while it is processed)
    int head = 0, kept = 0;
    while (head < nlis) {
      int k = head + lane;
      bool act = k < nlis;
      int e = act ? S.lis[k] : 0;
      int loc = e & 0x7FFF, typeB = e >> 15;
      int ch[9], cl = 0, no = 0;
      if (act) no = offspring_local(g, S.B, nb, L, loc, ch, &cl);
      int s = 0, nbits = 0, nlsp_a = 0, nlip_a = 0, nlis_a = 0;
      uint32_t v = 0;
      if (act) {
        if (!typeB) {
          s = S.mdl[loc] > pl;
          v = (uint32_t)s; nbits = 1;
          if (s) {
#pragma unroll
            for (int c = 0; c < 9; c++)
              if (c < no) {
                uint32_t q = S.qv[ch[c]];
                int sc = (q & 0x7FFFFFu) >= thr;
                v = (v << 1) | (uint32_t)sc; nbits++;
                if (sc) { v = (v << 1) | (q >> 31); nbits++; nlsp_a++; }
                else nlip_a++;
              }
            nlis_a = (no > 0 && cl >= 2) ? 1 : 0;
          }
        } else {
          s = S.mll[loc] > pl;
          v = (uint32_t)s; nbits = 1;
          if (s) nlis_a = no;
        }
      }
      int keep = act && !s;
      int tb, tk, tsp, tip, tis;
      int pb = wscan_excl(nbits, lane, &tb);
      int pk = wscan_excl(keep, lane, &tk);
      int psp = wscan_excl(nlsp_a, lane, &tsp);
      int pip = wscan_excl(nlip_a, lane, &tip);
      int pis = wscan_excl(nlis_a, lane, &tis);
      __syncthreads();
      put_bits(S.bw, (int)(bitpos - wbase) + pb, nbits, v);
      if (keep) S.lis[kept + pk] = (uint16_t)e;
      if (act && s) {
        if (!typeB) {
          int a = 0, b = 0;
          int64_t bp = bitpos + pb + 1;   // the first child's significance bit
#pragma unroll
          for (int c = 0; c < 9; c++)
            if (c < no) {
              int sc = (S.qv[ch[c]] & 0x7FFFFFu) >= thr;
              if (sc) {
                S.lsp[nlsp + psp + (a++)] = (uint16_t)ch[c];
                if (last) cpos[loc_to_pos(g, S.B, nb, nx, ch[c])] = (uint32_t)(bp + 1);
                bp += 2;
              } else {
                S.lip[nlip + pip + (b++)] = (uint16_t)ch[c];
                bp += 1;
              }
            }
          if (nlis_a) S.lis[nlis + pis] = (uint16_t)(loc | 0x8000);
        } else {
#pragma unroll
          for (int c = 0; c < 9; c++)
            if (c < no) S.lis[nlis + pis + c] = (uint16_t)ch[c];
        }
      }
      bitpos += tb; kept += tk; nlsp += tsp; nlip += tip;
      head += 64 < nlis - head ? 64 : nlis - head;
      nlis += tis;
      flush(false);
    }
    nlis = kept;
    // refinement pass
    if (last && lane == 0) tcut[3 * t + 1] = (uint32_t)bitpos;
    for (int h0 = 0; h0 < lsp_prev; h0 += 64) {
      int k = h0 + lane;
      bool act = k < lsp_prev;
      int n = lsp_prev - h0 < 64 ? lsp_prev - h0 : 64;
      uint32_t bit = act ? (S.qv[S.lsp[k]] >> pl) & 1u : 0u;
      if (last && act) cpos[loc_to_pos(g, S.B, nb, nx, S.lsp[k])] = (uint32_t)(bitpos + lane);
      __syncthreads();
      if (act) put_bits(S.bw, (int)(bitpos - wbase) + lane, 1, bit);
      bitpos += n;
      flush(false);
    }
  }
  flush(true);
  if (lane == 0) {
    uint32_t bytes = (uint32_t)((bitpos + 7) >> 3);
    tlen[t] = bytes;
    tent[t] = bytes | ((uint32_t)(ntop + 1) << 26);
    if (cut) tcut[3 * t + 2] = (uint32_t)bitpos;
  }
}

// Uniform reader of a tile payload (bytes past its end read as 0).  The
// window holds the next 32..63 bits MSB first and takes 32 more bits, one
// aligned word load, whenever fewer than 32 remain; the payload's byte
// offset within its first aligned word is fixed, so each refill is a funnel
// shift of two consecutive aligned words.
struct BitRU {
  const uint32_t* wp;      // aligned word holding the payload's first byte
  int len;                 // payload bytes
  int bytepos;             // payload bytes already in the window
  int sh;                  // 8 x (payload address mod 4)
  int nwords;              // aligned words that hold payload bytes
  int wi;                  // index of the next aligned word to load
  uint32_t prev;           // aligned word wi - 1
  uint64_t win;
  int wn;
  __device__ uint32_t word(int i) {
    // i < nwords: the word holds at least one payload byte, so it lies in
    // the payload's buffer; readfirstlane keeps the (uniform) value scalar
    return i < nwords ? (uint32_t)__builtin_amdgcn_readfirstlane((int)wp[i]) : 0u;
  }
  __device__ void init(const uint8_t* b, int64_t n) {
    const uint64_t a = (uint64_t)b;
    wp = reinterpret_cast<const uint32_t*>(a & ~(uint64_t)3);
    sh = 8 * (int)(a & 3);
    len = (int)n;
    nwords = (int)((a & 3) + (uint64_t)n + 3) >> 2;
    bytepos = 0;
    prev = word(0);
    wi = 1;
    win = 0;
    wn = 0;
    refill();
    refill();
  }
  __device__ void refill() {
    const uint32_t nxt = word(wi);
    uint32_t le = (uint32_t)(((((uint64_t)nxt) << 32) | prev) >> sh);   // next 4 bytes, first in the low byte
    prev = nxt;
    wi++;
    const int avail = len - bytepos;
    if (avail < 4) le &= avail <= 0 ? 0u : ((1u << (8 * avail)) - 1u);
    bytepos += 4;
    const uint32_t be = (le >> 24) | ((le >> 8) & 0xFF00u) | ((le << 8) & 0xFF0000u) | (le << 24);
    win |= (uint64_t)be << (32 - wn);
    wn += 32;
  }
  __device__ int get() {
    const int b = (int)(win >> 63);
    win <<= 1;
    if (--wn < 32) refill();
    return b;
  }
  // leading zeros among the valid bits
  __device__ int zeros() {
    const int z = win ? __builtin_clzll(win) : 64;
    return z < wn ? z : wn;
  }
  // n <= wn
  __device__ void skip(int n) {
    win = n < 64 ? win << n : 0;
    wn -= n;
    if (wn < 32) refill();
  }
};

// Tile geometry held in vector registers, lane b for band b, so that the
// wave-uniform decoder finds a node's band and offspring with a ballot and
// readlanes instead of LDS round trips.
struct GeomRegs {
  int off, wr, r0, c0, h, w, level, hr, y0, x0;
  uint32_t mlo, mhi;
  int nb;
  __device__ void load(const TileGeom& g, const Band* B, int nb_, int lane) {
    nb = nb_;
    const bool in = lane < nb;
    off = in ? g.off[lane] : 0x7FFFFFFF;
    wr = in ? g.wr[lane] : 0;
    r0 = in ? g.r0[lane] : 0;
    c0 = in ? g.c0[lane] : 0;
    h = in ? B[lane].h : 0;
    w = in ? B[lane].w : 0;
    level = in ? B[lane].level : 0;
    hr = in ? g.hr[lane] : 0;
    y0 = in ? B[lane].y0 : 0;
    x0 = in ? B[lane].x0 : 0;
    const uint64_t m = in ? g.mg[lane] : 0;
    mlo = (uint32_t)m;
    mhi = (uint32_t)(m >> 32);
  }
};
__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t rlu(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// Offspring of node loc (the same in every lane), described without an
// array: an LL root's (up to three) children k[0 .. n), or a detail node's
// children base + r * pitch + c for r in [r0, r1), c in [c0, c1), row-major.
// Same children, in the same order, as offspring_local.
struct Kids {
  int n, clevel;
  bool ll;
  int k0, k1, k2;
  int base, pitch, r0, r1, c0, c1;
};
__device__ __forceinline__ void kids_uniform(const GeomRegs& G, int L, int loc, Kids& K) {
  // bands are stored in order of offset: the node's band is the last one
  // starting at or before it
  const int b = __builtin_popcountll(__ballot(G.off <= loc)) - 1;
  const int rel = loc - rl(G.off, b);
  const uint64_t mg = (uint64_t)rlu(G.mlo, b) | ((uint64_t)rlu(G.mhi, b) << 32);
  const int wrb = rl(G.wr, b);
  const int li = (int)(((uint64_t)rel * mg) >> 32), lj = rel - li * wrb;
  const int i = rl(G.r0, b) + li, j = rl(G.c0, b) + lj;
  K.n = 0;
  K.k0 = K.k1 = K.k2 = 0;
  if (b == 0) {
    K.ll = true;
    K.clevel = L;
    if (L == 0) return;
#pragma unroll
    for (int c = 1; c <= 3; c++)
      if (i < rl(G.h, c) && j < rl(G.w, c)) {
        const int v = rl(G.off, c) + (i - rl(G.r0, c)) * rl(G.wr, c) + (j - rl(G.c0, c));
        if (K.n == 0) K.k0 = v;
        else if (K.n == 1) K.k1 = v;
        else K.k2 = v;
        K.n++;
      }
    return;
  }
  K.ll = false;
  const int lev = rl(G.level, b);
  K.clevel = lev - 1;
  if (lev == 1) return;
  const int cb = b + 3;
  const int hb = rl(G.h, b), wb = rl(G.w, b), hc = rl(G.h, cb), wc = rl(G.w, cb);
  int r1 = (i == hb - 1) ? hc : 2 * i + 2;
  int c1 = (j == wb - 1) ? wc : 2 * j + 2;
  if (r1 > hc) r1 = hc;
  if (c1 > wc) c1 = wc;
  K.pitch = rl(G.wr, cb);
  K.base = rl(G.off, cb) - rl(G.r0, cb) * K.pitch - rl(G.c0, cb);
  K.r0 = 2 * i; K.r1 = r1; K.c0 = 2 * j; K.c1 = c1;
  K.n = (r1 > 2 * i && c1 > 2 * j) ? (r1 - 2 * i) * (c1 - 2 * j) : 0;
}

// Children of a node loc of the detail band b > 0 (both the same in every
// lane), as kids_uniform finds them, with the arithmetic on the vector unit
// (the decoder's wave-uniform chain is bound by the compute unit's scalar
// issue): K.n, K.clevel and K.ll (false) are set, the other fields of K are
// not; child l < K.n is returned in lane l.
__device__ __forceinline__ int kids_lanes(const GeomRegs& G, int loc, int b, int lane, Kids& K) {
  K.ll = false;
  const int lev = rl(G.level, b);
  K.clevel = lev - 1;
  K.n = 0;
  if (lev == 1) return 0;
  // zero in every lane, but not known to be uniform: what depends on it is
  // computed by vector instructions
  const int vz = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u);
  const uint32_t rel = (uint32_t)(loc + vz - rl(G.off, b));
  const uint64_t mg = (uint64_t)rlu(G.mlo, b) | ((uint64_t)rlu(G.mhi, b) << 32);
  const int wrb = rl(G.wr, b);
  const int li = (int)(((uint64_t)rel * mg) >> 32), lj = (int)rel - li * wrb;
  const int i = rl(G.r0, b) + li, j = rl(G.c0, b) + lj;
  const int cb = b + 3;
  const int hb = rl(G.h, b), wb = rl(G.w, b), hc = rl(G.h, cb), wc = rl(G.w, cb);
  int r1 = (i == hb - 1) ? hc : 2 * i + 2;
  int c1 = (j == wb - 1) ? wc : 2 * j + 2;
  r1 = r1 < hc ? r1 : hc;
  c1 = c1 < wc ? c1 : wc;
  const int nr = r1 > 2 * i ? r1 - 2 * i : 0, ncv = c1 > 2 * j ? c1 - 2 * j : 0;
  K.n = __builtin_amdgcn_readfirstlane(nr * ncv);
  const int nc = __builtin_amdgcn_readfirstlane(ncv);
  const int pitch = rl(G.wr, cb);
  const int base = rl(G.off, cb) - rl(G.r0, cb) * pitch - rl(G.c0, cb);
  const int r = nc == 1 ? lane : (nc == 2 ? lane >> 1 : (lane * 11) >> 5);   // lane / nc, lane < 9
  return base + (2 * i + r) * pitch + 2 * j + (lane - r * nc);
}

// Significance and sign bits of up to four children of a significant set,
// read from the next eight bits of the code (first bit in bit 7 of the
// index): for n children, entry [n - 1][byte] holds the children found
// significant (bits 0-3), their signs (bits 4-7) and the bits the n
// children take (bits 8-11).  Each child takes its significance bit, and a
// sign bit after a 1.
struct KidsTab {
  uint32_t v[4][256];
};
constexpr KidsTab make_kids_tab() {
  KidsTab t{};
  for (int n = 1; n <= 4; n++)
    for (int b = 0; b < 256; b++) {
      int pos = 0;
      uint32_t sg = 0, sn = 0;
      for (int l = 0; l < n; l++) {
        const uint32_t bit = ((uint32_t)b >> (7 - pos)) & 1u;
        pos++;
        if (bit) {
          sn |= (((uint32_t)b >> (7 - pos)) & 1u) << l;
          pos++;
          sg |= 1u << l;
        }
      }
      t.v[n - 1][b] = sg | (sn << 4) | ((uint32_t)pos << 8);
    }
  return t;
}
__constant__ KidsTab c_kids_tab = make_kids_tab();

// LIP tokens in the next eight bits of the code (first bit in bit 7 of the
// index): each entry takes a 0 (it stays insignificant) or a 1 and its sign
// bit; entry [byte] holds the number of tokens that fit whole (bits 0-3,
// 1 to 8 when the byte holds a 1), which of them are 1 (bits 4-11) and
// their signs (bits 12-19).
struct LipTab {
  uint32_t v[256];
};
constexpr LipTab make_lip_tab() {
  LipTab t{};
  for (int b = 0; b < 256; b++) {
    int pos = 0, m = 0;
    uint32_t sg = 0, sn = 0;
    while (pos < 8) {
      if ((((uint32_t)b >> (7 - pos)) & 1u) == 0) {
        pos++;
        m++;
        continue;
      }
      if (pos + 1 >= 8) break;
      sn |= (((uint32_t)b >> (6 - pos)) & 1u) << m;
      sg |= 1u << m;
      pos += 2;
      m++;
    }
    t.v[b] = (uint32_t)m | (sg << 4) | (sn << 12);
  }
  return t;
}
__constant__ LipTab c_lip_tab = make_lip_tab();

// The decoder's LDS: the band table and the tile's geometry are needed only
// until the lists are set up and the geometry is in registers, so the
// decoded magnitudes reuse their space (more tiles resident per CU).
template <int CAP>
struct SpihtDecLds {
  union {
    struct {
      Band B[kMaxBands];
      TileGeom g;
    } s;
    uint32_t qv[CAP];        // decoded magnitude | sign << 31
  } u;
  uint16_t lip[CAP], lsp[CAP];
  uint16_t lis[CAP / 2];     // local index | typeB << 15 (at most twice the parents)
  int ok;
};

template <int CAP>
__global__ __launch_bounds__(64) void k_spiht_decode_lds(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                         const int* __restrict__ tix, const int64_t* __restrict__ toff,
                                                         int* __restrict__ misfit) {
  static_assert(sizeof(Band) * kMaxBands + sizeof(TileGeom) <= sizeof(uint32_t) * CAP, "decoder LDS union");
  __shared__ SpihtDecLds<CAP> S;
  const int lane = threadIdx.x;
  const int t = tix[blockIdx.x];
  const TileD td = tiles[t];
  const FieldDev& f = F[td.field];
  if (!f.active || f.rb == 0) return;
  const uint8_t* __restrict__ sec = f.out + kHdr + f.bb;
  const int64_t sec_len = f.rb;
  const Band* bands_g = f.bands;
  const int nx = f.nx, nb = f.nb, L = f.L, n_s = f.ns, e_r = f.er;
  float* chat = f.buf[BUF_CHAT];
  int* flag = &f.flags[1];
  const int tl = t - f.tile0;
  for (int i = lane; i < nb; i += 64) S.u.s.B[i] = bands_g[i];
  __syncthreads();
  if (lane == 0) {
    tile_geom(S.u.s.g, S.u.s.B, nb, L, td);
    S.ok = S.u.s.g.ncoef <= CAP && 4 * S.u.s.g.nparents <= CAP;
  }
  __syncthreads();
  if (!S.ok) {
    if (lane == 0) misfit[t] = 1;
    return;
  }
  if (lane == 0) misfit[t] = 0;
  const TileGeom& g = S.u.s.g;
  const uint32_t ent = (uint32_t)__builtin_amdgcn_readfirstlane(
      (int)((uint32_t)sec[4 * tl] | ((uint32_t)sec[4 * tl + 1] << 8) | ((uint32_t)sec[4 * tl + 2] << 16) |
            ((uint32_t)sec[4 * tl + 3] << 24)));
  const int64_t len = ent & 0x3FFFFFF;
  const int ntop = (int)(ent >> 26) - 1;
  const int64_t pbase = 4 * (int64_t)f.ntiles;
  const int64_t o0 = toff[t];
  // byte-cut fields: the trailer after the payloads names the cut; the cut
  // tile is decoded by its own launch, the others stop at a plane end or
  // before a refinement pass
  int n_bot = n_s, sort_only = 0;
  int64_t pay_end = sec_len;
  if (f.bt) {
    pay_end = sec_len - 8;
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)sec[pay_end] | ((uint32_t)sec[pay_end + 1] << 8) | ((uint32_t)sec[pay_end + 2] << 16) |
              ((uint32_t)sec[pay_end + 3] << 24)));
    const int J = (int)(w0 & 0x7FFFFFFFu), kind = (int)(w0 >> 31);
    if (tl == J) return;
    cut_tile_mode(kind, J, tl, n_s, &n_bot, &sort_only);
  }
  if (o0 < 0 || pbase + o0 + len > pay_end || ntop >= kQBits) {
    if (lane == 0) atomicOr(flag, 1);
    return;
  }
  if (ntop < n_bot) return;
  const uint8_t* pay = sec + pbase + o0;
  const int nroots = g.hr[0] * g.wr[0], ncoef = g.ncoef;
  int nlis = 0;
  for (int r0 = 0; r0 < nroots; r0 += 64) {
    int r = r0 + lane;
    int ch[9], cl;
    int has = 0;
    if (r < nroots) {
      S.lip[r] = (uint16_t)r;
      has = offspring_local(g, S.u.s.B, nb, L, r, ch, &cl) > 0;
    }
    int tot;
    int pre = wscan_excl(has, lane, &tot);
    if (has) S.lis[nlis + pre] = (uint16_t)r;
    nlis += tot;
  }
  GeomRegs G;
  G.load(g, S.u.s.B, nb, lane);
  // the band table and geometry are in registers now: their LDS becomes
  // the decoded magnitudes
  __syncthreads();
  for (int i = lane; i < ncoef; i += 64) S.u.qv[i] = 0;
  __syncthreads();
  int nlip = nroots, nlsp = 0;
  BitRU rd;
  rd.init(pay, len);
  for (int pl = ntop; pl >= n_bot; pl--) {
    const uint32_t thr = 1u << pl;
    const int lsp_prev = nlsp;
    // LIP: each entry's token is a 0 (it stays) or a 1 and its sign bit (it
    // becomes significant).  Runs of eight zeros or more (or up to the list's
    // end) are skipped with one count of leading zeros; otherwise the tokens
    // that fit in the next byte come from a table, the lanes (one per entry)
    // placing them.  Entries are read through a 64-entry register window;
    // survivors only move below the current position.
    int k = 0, surv = 0, pbase = 0, pcnt = 0;
    uint32_t pv = 0;
    while (k < nlip) {
      int z = rd.zeros();
      if (z > nlip - k) z = nlip - k;
      if (z > 0 && (z >= 8 || z == nlip - k)) {
        // survivors k .. k+z-1 move down to surv .. (ascending chunks are safe)
        if (surv != k)
          for (int c = 0; c < z; c += 64) {
            int i = c + lane;
            uint16_t v = i < z ? S.lip[k + i] : 0;
            __syncthreads();
            if (i < z) S.lip[surv + i] = v;
            __syncthreads();
          }
        rd.skip(z);
        k += z; surv += z;
        continue;
      }
      // entries k .. k + m - 1: the tokens that fit in the next byte
      const uint32_t te = c_lip_tab.v[(uint32_t)(rd.win >> 56)];
      int m = (int)(te & 15u);
      uint32_t sigm = (te >> 4) & 255u, sgnm = (te >> 12) & 255u;
      if (m > nlip - k) {
        m = nlip - k;
        sigm &= (1u << m) - 1u;
        sgnm &= (1u << m) - 1u;
      }
      const int nsig = __builtin_popcount(sigm);
      rd.skip(m + nsig);
      if (k < pbase || k + m > pbase + pcnt) {
        pbase = k;
        pcnt = nlip - k < 64 ? nlip - k : 64;
        pv = lane < pcnt ? (uint32_t)S.lip[k + lane] : 0u;
      }
      const int e = __shfl((int)pv, k - pbase + lane);   // lane < m: entry k + lane
      if (lane < m) {
        const int r1 = __builtin_popcount(sigm & ((1u << lane) - 1u));
        if ((sigm >> lane) & 1u) {
          S.u.qv[e] = thr | (((sgnm >> lane) & 1u) << 31);
          S.lsp[nlsp + r1] = (uint16_t)e;
        } else {
          S.lip[surv + lane - r1] = (uint16_t)e;
        }
      }
      nlsp += nsig;
      surv += m - nsig;
      k += m;
    }
    nlip = surv;
    // LIS: entries are read 64 at a time into a vector register (lane i:
    // entry base + i); a window never reaches past the list's end at the
    // time it is read, so entries appended later are read by a later window.
    // One wavefront runs the tile, so its LDS writes are seen by its later
    // reads in program order.
    int head = 0, kept = 0, wbase = 0, wcnt = 0;
    uint32_t wv = 0;
    while (head < nlis) {
      // a run of zero bits (sets that stay insignificant) leaves its entries
      // in the list: they move down to the kept ones 64 at a time (only
      // below the current position, which the window never reads again)
      int z = rd.zeros();
      if (z > nlis - head) z = nlis - head;
      if (z > 0) {
        if (kept != head)
          for (int c = 0; c < z; c += 64) {
            const int i = c + lane;
            const uint16_t v = i < z ? S.lis[head + i] : (uint16_t)0;
            __syncthreads();
            if (i < z) S.lis[kept + i] = v;
            __syncthreads();
          }
        rd.skip(z);
        head += z;
        kept += z;
        continue;
      }
      if (head - wbase >= wcnt) {
        wbase = head;
        wcnt = nlis - head < 64 ? nlis - head : 64;
        wv = lane < wcnt ? (uint32_t)S.lis[head + lane] : 0u;
      }
      const int e = (int)__builtin_amdgcn_readlane((int)wv, head - wbase);
      // no zero run starts here (the window always holds at least 32 valid
      // bits), so the set's significance bit is 1
      rd.skip(1);
      const int loc = e & 0x7FFF, typeB = e >> 15;
      const int bnd = __builtin_popcountll(__ballot(G.off <= loc)) - 1;
      Kids K;
      int cl = 0;   // a detail node's child K.n > lane in this lane
      if (bnd == 0) kids_uniform(G, L, loc, K);
      else cl = kids_lanes(G, loc, bnd, lane, K);
      if (!typeB && K.n <= 4) {
        // each child: its significance bit, and the sign when it is 1; up
        // to four children read at once (at most 8 bits) through a table of
        // the next byte, then placed by the lanes (one per child)
        const int n = K.n;
        const uint32_t te = n ? c_kids_tab.v[n - 1][(uint32_t)(rd.win >> 56)] : 0u;
        const uint32_t sigm = te & 15u, sgnm = (te >> 4) & 15u;
        if (n) rd.skip((int)(te >> 8));
        if (lane < n) {
          const int c = K.ll ? (lane == 0 ? K.k0 : (lane == 1 ? K.k1 : K.k2)) : cl;
          const uint32_t below = (1u << lane) - 1u;
          if ((sigm >> lane) & 1u) {
            S.u.qv[c] = thr | (((sgnm >> lane) & 1u) << 31);
            S.lsp[nlsp + __builtin_popcount(sigm & below)] = (uint16_t)c;
          } else {
            S.lip[nlip + lane - __builtin_popcount(sigm & below)] = (uint16_t)c;
          }
        }
        const int ns1 = __builtin_popcount(sigm);
        nlsp += ns1;
        nlip += n - ns1;
        if (n > 0 && K.clevel >= 2) {
          if (lane == 0) S.lis[nlis] = (uint16_t)(loc | 0x8000);
          nlis++;
        }
      } else if (!typeB) {
        // more than four children (the extra row or column of odd-sized
        // bands; never an LL root's): one at a time
        for (int l = 0; l < K.n; l++) {
          const int c = rl(cl, l);
          if (rd.get()) {
            const int sg = rd.get();
            if (lane == 0) { S.u.qv[c] = thr | ((uint32_t)sg << 31); S.lsp[nlsp] = (uint16_t)c; }
            nlsp++;
          } else {
            if (lane == 0) S.lip[nlip] = (uint16_t)c;
            nlip++;
          }
        }
        if (K.n > 0 && K.clevel >= 2) {
          if (lane == 0) S.lis[nlis] = (uint16_t)(loc | 0x8000);
          nlis++;
        }
      } else {
        // the children join the LIS as type-A entries, one per lane
        if (lane < K.n) {
          const int v = K.ll ? (lane == 0 ? K.k0 : (lane == 1 ? K.k1 : K.k2)) : cl;
          S.lis[nlis + lane] = (uint16_t)v;
        }
        nlis += K.n;
      }
      head++;
    }
    __syncthreads();
    nlis = kept;
    if (pl == n_bot && sort_only) break;   // a byte-cut field's tile that stops before this refinement pass
    // refinement: the next lsp_prev bits, 64 at a time from the uniform
    // reader, one per lane
    for (int h0 = 0; h0 < lsp_prev; h0 += 64) {
      const int n = lsp_prev - h0 < 64 ? lsp_prev - h0 : 64;
      const uint32_t w0 = (uint32_t)(rd.win >> 32);
      rd.skip(n < 32 ? n : 32);
      const uint32_t w1 = (uint32_t)(rd.win >> 32);
      if (n > 32) rd.skip(n - 32);
      const int kk = h0 + lane;
      if (lane < n) {
        const uint32_t b = lane < 32 ? (w0 >> (31 - lane)) & 1u : (w1 >> (63 - lane)) & 1u;
        if (b) S.u.qv[S.lsp[kk]] |= thr;
      }
    }
    __syncthreads();
  }
  // dequantised significant coefficients (band geometry from the lanes of
  // G, read in wave-uniform code)
  for (int b = 0; b < nb; b++) {
    const int wrb = rl(G.wr, b), n = rl(G.hr, b) * wrb, offb = rl(G.off, b);
    const int yb = rl(G.y0, b) + rl(G.r0, b), xb = rl(G.x0, b) + rl(G.c0, b);
    for (int r = lane; r < n; r += 64) {
      uint32_t v = S.u.qv[offb + r];
      if (!v) continue;
      int li = r / wrb, lj = r - li * wrb;
      int p = (yb + li) * nx + xb + lj;
      uint32_t m = v & 0x7FFFFFu;
      // lowest known plane: n_bot, or above it for coefficients significant
      // before a last plane whose refinement pass was not decoded
      const int pk = (sort_only && m >= (2u << n_s)) ? n_s + 1 : n_bot;
      float f = ldexpf((float)(2u * m + (1u << pk)), e_r - 1);
      chat[p] = (v >> 31) ? -f : f;
    }
  }
}

// Byte-cut candidates: the residual coefficients the decoder of each cut
// would reconstruct, one wavefront per tile of the candidate's field.  A
// coefficient known above plane ns + 1 is known there whatever the cut; of
// plane ns it needs one bit, at cpos in its tile's code: its sign bit (it
// becomes significant in plane ns) or its refinement bit.
struct CutGeomLds {
  Band B[kMaxBands];
  TileGeom g;
};
__global__ __launch_bounds__(64) void k_spiht_cut_recon(const FieldDev* __restrict__ Fc, const TileD* __restrict__ tiles,
                                                        const uint32_t* __restrict__ tcut) {
  __shared__ CutGeomLds S;
  const FieldDev& f = Fc[blockIdx.y];
  const int tl = (int)blockIdx.x;
  if (!f.active || tl >= f.ntiles) return;
  const int lane = threadIdx.x;
  const int t = f.tile0 + tl;
  const TileD td = tiles[t];
  const int nb = f.nb, nx = f.nx, ns = f.ns, er = f.er;
  for (int i = lane; i < nb; i += 64) S.B[i] = f.bands[i];
  __syncthreads();
  if (lane == 0) tile_geom(S.g, S.B, nb, f.L, td);
  __syncthreads();
  const TileGeom& g = S.g;
  const uint32_t ell = cut_tile_bits(f.cut_kind, f.cut_tile, f.cut_bits, tl, tcut[3 * t], tcut[3 * t + 1],
                                     tcut[3 * t + 2]);
  const uint32_t* __restrict__ qr = f.qr;
  const uint32_t* __restrict__ cpos = f.cpos;
  float* __restrict__ chat = f.buf[BUF_CHAT];
  const uint32_t lo = 1u << ns, hi = 2u << ns;
  for (int b = 0; b < nb; b++) {
    const int n = g.hr[b] * g.wr[b], wr = g.wr[b];
    if (n == 0) continue;
    const int y0 = S.B[b].y0 + g.r0[b], x0 = S.B[b].x0 + g.c0[b];
    for (int r = lane; r < n; r += 64) {
      const int li = r / wr, lj = r - li * wr;
      const int p = (y0 + li) * nx + x0 + lj;
      const uint32_t w = qr[p], m = w & 0x7FFFFFu;
      float v = 0.0f;
      if (m >= lo) {
        const bool known = cpos[p] < ell;
        if (m >= hi) {
          const int pk = known ? ns : ns + 1;
          v = dequant((m >> pk) << pk, pk, (int)(w >> 31), er);
        } else if (known) {
          v = dequant(lo, ns, (int)(w >> 31), er);
        }
      }
      chat[p] = v;
    }
  }
}

// Final tile lengths of the byte-cut fields.
__global__ __launch_bounds__(256) void k_spiht_cut_tiles(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                         int nt, const uint32_t* __restrict__ tcut,
                                                         uint32_t* __restrict__ tlen, uint32_t* __restrict__ tent,
                                                         uint32_t* __restrict__ tbits) {
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
    const FieldDev& f = F[tiles[t].field];
    if (!f.active) continue;
    const uint32_t ell = cut_tile_bits(f.cut_kind, f.cut_tile, f.cut_bits, t - f.tile0, tcut[3 * t],
                                       tcut[3 * t + 1], tcut[3 * t + 2]);
    const uint32_t by = (ell + 7) >> 3;
    tbits[t] = ell;
    tlen[t] = by;
    tent[t] = ell ? (by | (tent[t] & 0xFC000000u)) : 0u;
  }
}

// key: bit length of the payload's byte length, longest first
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const int* __restrict__ tix, int n, const uint32_t* __restrict__ tent,
                                                    int* __restrict__ out) {
  order_by_key(n, [&](int i) {
    const int bl = blen(tent[tix[i]] & 0x3FFFFFFu);
    return kQBits - (bl < kQBits ? bl : kQBits);
  }, tix, out, nullptr);
}

void spiht_tiles_longest_first(const int* tix, int n, const uint32_t* tent, int* out, hipStream_t st) {
  if (n <= 0) return;
  k_tile_order<<<1, kOrderThreads, 0, st>>>(tix, n, tent, out);
}

void spiht_cut_recon(const FieldDev* Fc, int ncand, int max_tiles, const TileD* tiles, const uint32_t* tcut,
                     hipStream_t st) {
  if (ncand <= 0 || max_tiles <= 0) return;
  k_spiht_cut_recon<<<dim3(max_tiles, ncand), 64, 0, st>>>(Fc, tiles, tcut);
}

void spiht_cut_tiles(const FieldDev* F, const TileD* tiles, int nt, const uint32_t* tcut, uint32_t* tlen,
                     uint32_t* tent, uint32_t* tbits, hipStream_t st) {
  if (nt <= 0) return;
  int g = (nt + 255) / 256;
  k_spiht_cut_tiles<<<g < 2048 ? g : 2048, 256, 0, st>>>(F, tiles, nt, tcut, tlen, tent, tbits);
}

void spiht_encode_lds(int cap, const FieldDev* F, const TileD* tiles, const int* tix, int ntix, uint8_t* slots,
                      const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, uint32_t* tcut, int* misfit,
                      hipStream_t st) {
  if (ntix <= 0) return;
  if (cap == kSpihtSmall)
    k_spiht_encode_lds<kSpihtSmall><<<ntix, 64, 0, st>>>(F, tiles, tix, slots, slot_off, tlen, tent, tcut, misfit);
  else if (cap == kSpihtBig)
    k_spiht_encode_lds<kSpihtBig><<<ntix, 64, 0, st>>>(F, tiles, tix, slots, slot_off, tlen, tent, tcut, misfit);
  else
    k_spiht_encode_lds<kSpihtHuge><<<ntix, 64, 0, st>>>(F, tiles, tix, slots, slot_off, tlen, tent, tcut, misfit);
}

void spiht_decode_lds(int cap, const FieldDev* F, const TileD* tiles, const int* tix, int ntix, const int64_t* toff,
                      int* misfit, hipStream_t st) {
  if (ntix <= 0) return;
  if (cap == kSpihtSmall)
    k_spiht_decode_lds<kSpihtSmall><<<ntix, 64, 0, st>>>(F, tiles, tix, toff, misfit);
  else if (cap == kSpihtBig)
    k_spiht_decode_lds<kSpihtBig><<<ntix, 64, 0, st>>>(F, tiles, tix, toff, misfit);
  else
    k_spiht_decode_lds<kSpihtHuge><<<ntix, 64, 0, st>>>(F, tiles, tix, toff, misfit);
}

}  // namespace ebcc
