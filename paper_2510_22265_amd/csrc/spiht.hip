// Residual layer of EBCC: SPIHT bit-plane coding (Said & Pearlman 1996, as
// cited in the paper's Method section) of the quantised wavelet coefficients
// of the residual, coded independently per tile of coarsest-LL roots.
//
// Spatial-orientation trees: an LL root has the three co-located
// coefficients of the coarsest HL, LH and HH bands as offspring; a detail
// coefficient (i, j) at level l >= 2 has the 2x2 group (2i.., 2j..) of its
// orientation one level finer, and when the finer band has one more row
// (column) than twice the coarser band, the parents of the last row (column)
// also take that row (column); level-1 coefficients are leaves.
//
//  * k_maxima: one launch per level, fine to coarse (level 2 first, the
//    three orientations side by side), one thread per node: the maximum
//    magnitude over the node's
//    descendants (maxD), over its grand-descendants and below (maxL), and
//    over its subtree including itself (sub).
//  * k_spiht_encode / k_spiht_decode: one lane per tile; the three lists
//    (LIP, LSP, LIS) are FIFO arrays in the tile's slice of a global scratch
//    (removal = clearing an "alive" bit), bits are packed MSB-first.
#include "common.h"

#include <algorithm>

namespace ebcc {

// List entry: j | i << 24 | band << 48 | typeB << 56 | alive << 57.
__device__ __forceinline__ uint64_t mk_node(int band, int i, int j) {
  return (uint64_t)(uint32_t)j | ((uint64_t)(uint32_t)i << 24) | ((uint64_t)band << 48);
}
__device__ __forceinline__ int nd_j(uint64_t n) { return (int)(n & 0xFFFFFF); }
__device__ __forceinline__ int nd_i(uint64_t n) { return (int)((n >> 24) & 0xFFFFFF); }
__device__ __forceinline__ int nd_band(uint64_t n) { return (int)((n >> 48) & 0xFF); }
constexpr uint64_t kTypeB = 1ull << 56, kAlive = 1ull << 57;

__device__ __forceinline__ int nd_pos(const Band* B, int nx, uint64_t n) {
  const Band& b = B[nd_band(n)];
  return (b.y0 + nd_i(n)) * nx + b.x0 + nd_j(n);
}

// Offspring of (band, i, j) in row-major order; returns the count (<= 9).
__device__ __forceinline__ int offspring(const Band* B, int L, int band, int i, int j, uint64_t* o) {
  int k = 0;
  if (band == 0) {
    if (L == 0) return 0;
    for (int c = 1; c <= 3; c++)
      if (i < B[c].h && j < B[c].w) o[k++] = mk_node(c, i, j);
    return k;
  }
  const Band& pb = B[band];
  if (pb.level == 1) return 0;
  int cb = band + 3;
  const Band& ch = B[cb];
  int r1 = (i == pb.h - 1) ? ch.h : 2 * i + 2;
  int c1 = (j == pb.w - 1) ? ch.w : 2 * j + 2;
  if (r1 > ch.h) r1 = ch.h;
  if (c1 > ch.w) c1 = ch.w;
  for (int r = 2 * i; r < r1; r++)
    for (int c = 2 * j; c < c1; c++) o[k++] = mk_node(cb, r, c);
  return k;
}
// Level of a node's offspring (roots: the coarsest detail level).
__device__ __forceinline__ int child_level(const Band* B, int L, int band) { return band == 0 ? L : B[band].level - 1; }

// Band index of (level, orientation 0..2) in a field with L levels; level 0
// denotes the LL roots.
__device__ __forceinline__ int band_index(int L, int lvl, int o) { return lvl == 0 ? 0 : 1 + 3 * (L - lvl) + o; }

__global__ __launch_bounds__(256) void k_maxima(const FieldDev* __restrict__ F, int lvl) {
  const FieldDev& f = F[blockIdx.y];
  const int o = (int)blockIdx.z;   // the three orientations of a level are independent
  if (!f.active || lvl > f.L || (lvl == 1)) return;
  const int L = f.L, nx = f.nx;
  const Band* bands = f.bands;
  const int band = band_index(L, lvl, o);
  const Band bd = bands[band];
  int n = bd.h * bd.w;
  int cl = child_level(bands, L, band);
  const uint32_t* qr = f.qr;
  uint32_t *sub = f.sub, *maxd = f.maxd, *maxl = f.maxl;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256) {
    int i = t / bd.w, j = t - i * bd.w;
    uint64_t oo[9];
    int no = offspring(bands, L, band, i, j, oo);
    uint32_t md = 0, ml = 0;
    for (int c = 0; c < no; c++) {
      int pc = nd_pos(bands, nx, oo[c]);
      uint32_t s, d;
      if (cl == 1) { s = qr[pc] & 0x7FFFFFu; d = 0; }
      else { s = sub[pc]; d = maxd[pc]; }
      md = s > md ? s : md;
      ml = d > ml ? d : ml;
    }
    int p = (bd.y0 + i) * nx + bd.x0 + j;
    uint32_t self = qr[p] & 0x7FFFFFu;
    sub[p] = self > md ? self : md;
    maxd[p] = md;
    maxl[p] = ml;
  }
}

// Largest band of (level, orientation) over the active fields (host side).
static int max_band_size(const FieldDev* Fh, int nf, int lvl, int o) {
  int m = 0;
  for (int i = 0; i < nf; i++) {
    const FieldDev& f = Fh[i];
    if (!f.active || lvl > f.L) continue;
    int h = f.ny, w = f.nx;
    int hp = h, wp = w;
    int lv = lvl == 0 ? f.L : lvl;
    for (int k = 1; k <= lv; k++) { hp = h; wp = w; h = (h + 1) / 2; w = (w + 1) / 2; }
    int bh, bw;
    if (lvl == 0) { bh = h; bw = w; }
    else if (o == 0) { bh = h; bw = wp - w; }
    else if (o == 1) { bh = hp - h; bw = w; }
    else { bh = hp - h; bw = wp - w; }
    m = std::max(m, bh * bw);
  }
  return m;
}

void spiht_maxima(const FieldDev* F, const FieldDev* Fh, int nf, hipStream_t st) {
  int Lm = 0;
  for (int i = 0; i < nf; i++)
    if (Fh[i].active) Lm = std::max(Lm, Fh[i].L);
  // finer parents first: levels 2 .. L (one launch per level, blockIdx.z
  // the orientation), then the LL roots
  for (int l = 2; l <= Lm; l++) {
    int n = 0;
    for (int o = 0; o < 3; o++) n = std::max(n, max_band_size(Fh, nf, l, o));
    int g = std::min(2048, std::max(1, (n + 255) / 256));
    if (n > 0) k_maxima<<<dim3(g, nf, 3), 256, 0, st>>>(F, l);
  }
  int n = max_band_size(Fh, nf, 0, 0);
  int g = std::min(2048, std::max(1, (n + 255) / 256));
  k_maxima<<<dim3(g, nf, 1), 256, 0, st>>>(F, 0);
}

// Tiles per wavefront: one per wavefront for a lone field (latency), up to
// 64 for large batches (throughput).
static int pick_tile_lanes(int items) {
  int l = 1;
  while (l < 64 && items / l > 8192) l *= 4;
  return l;
}

struct BitW {
  uint8_t* out;
  int64_t pos, cap;
  uint32_t acc;
  int n;
  __device__ void put(int b) {
    acc = (acc << 1) | (uint32_t)b;
    if (++n == 8) {
      if (pos < cap) out[pos] = (uint8_t)acc;
      pos++;
      acc = 0; n = 0;
    }
  }
  __device__ int64_t bits() const { return 8 * pos + n; }
  __device__ void flush() {
    if (n) {
      if (pos < cap) out[pos] = (uint8_t)(acc << (8 - n));
      pos++;
      acc = 0; n = 0;
    }
  }
};

template <int LANES>
__global__ __launch_bounds__(LANES) void k_spiht_encode(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                        const int* __restrict__ tix, int ntix,
                                                        uint64_t* __restrict__ lists,
                                                        uint8_t* __restrict__ slots,
                                                        const int64_t* __restrict__ slot_off,
                                                        uint32_t* __restrict__ tlen, uint32_t* __restrict__ tent,
                                                        uint32_t* __restrict__ tcut) {
  const int q = blockIdx.x * LANES + threadIdx.x;
  if (q >= ntix) return;
  const int t = tix[q];
  TileD td = tiles[t];
  const FieldDev& f = F[td.field];
  if (!f.active) return;
  const Band* B = f.bands;
  const int nx = f.nx, L = f.L, n_s = f.ns;
  const uint32_t *qr = f.qr, *sub = f.sub, *maxd = f.maxd, *maxl = f.maxl;
  // byte-cut fields: positions of the last plane's bits, bit counts around it
  uint32_t* const cpos = f.cpos;
  uint32_t mx = 0;
  for (int i = td.i0; i < td.i1; i++)
    for (int j = td.j0; j < td.j1; j++) {
      uint32_t s = sub[i * nx + j];
      mx = s > mx ? s : mx;
    }
  int ntop = mx ? 31 - __builtin_clz(mx) : -1;
  if (ntop < n_s) {
    tlen[t] = 0; tent[t] = 0;
    if (cpos) { tcut[3 * t] = 0; tcut[3 * t + 1] = 0; tcut[3 * t + 2] = 0; }
    return;
  }
  int nc = td.ncoef;
  uint64_t* lip = lists + 4 * td.off;
  uint64_t* lsp = lip + nc;
  uint64_t* lis = lsp + nc;
  int nlip = 0, nlsp = 0, nlis = 0;
  uint64_t o[9];
  for (int i = td.i0; i < td.i1; i++)
    for (int j = td.j0; j < td.j1; j++) {
      uint64_t n = mk_node(0, i, j);
      lip[nlip++] = n | kAlive;
      if (offspring(B, L, 0, i, j, o) > 0) lis[nlis++] = n | kAlive;
    }
  int64_t so = slot_off[t];
  BitW w{slots + so, 0, slot_off[t + 1] - so, 0u, 0};
  for (int pl = ntop; pl >= n_s; pl--) {
    uint32_t thr = 1u << pl;
    int lsp_prev = nlsp;
    const bool last = cpos && pl == n_s;
    if (last) tcut[3 * t] = (uint32_t)w.bits();
    for (int k = 0; k < nlip; k++) {
      uint64_t e = lip[k];
      if (!(e & kAlive)) continue;
      uint32_t v = qr[nd_pos(B, nx, e)];
      int s = (v & 0x7FFFFFu) >= thr;
      w.put(s);
      if (s) {
        if (last) cpos[nd_pos(B, nx, e)] = (uint32_t)w.bits();   // its sign bit
        w.put((int)(v >> 31));
        lsp[nlsp++] = e & ~kAlive;
        lip[k] = e & ~kAlive;
      }
    }
    for (int k = 0; k < nlis; k++) {
      uint64_t e = lis[k];
      if (!(e & kAlive)) continue;
      int band = nd_band(e), i = nd_i(e), j = nd_j(e);
      int p = nd_pos(B, nx, e);
      int no = offspring(B, L, band, i, j, o);
      if (!(e & kTypeB)) {
        int s = maxd[p] >= thr;
        w.put(s);
        if (!s) continue;
        for (int c = 0; c < no; c++) {
          uint32_t v = qr[nd_pos(B, nx, o[c])];
          int sc = (v & 0x7FFFFFu) >= thr;
          w.put(sc);
          if (sc) {
            if (last) cpos[nd_pos(B, nx, o[c])] = (uint32_t)w.bits();
            w.put((int)(v >> 31));
            lsp[nlsp++] = o[c];
          } else {
            lip[nlip++] = o[c] | kAlive;
          }
        }
        lis[k] = e & ~kAlive;
        if (no > 0 && child_level(B, L, band) >= 2) lis[nlis++] = (e & ~kAlive) | kTypeB | kAlive;
      } else {
        int s = maxl[p] >= thr;
        w.put(s);
        if (!s) continue;
        for (int c = 0; c < no; c++) lis[nlis++] = o[c] | kAlive;
        lis[k] = e & ~kAlive;
      }
    }
    if (last) tcut[3 * t + 1] = (uint32_t)w.bits();
    for (int k = 0; k < lsp_prev; k++) {
      uint32_t v = qr[nd_pos(B, nx, lsp[k])];
      if (last) cpos[nd_pos(B, nx, lsp[k])] = (uint32_t)w.bits();
      w.put((int)((v >> pl) & 1u));
    }
  }
  if (cpos) tcut[3 * t + 2] = (uint32_t)w.bits();
  w.flush();
  tlen[t] = (uint32_t)w.pos;
  tent[t] = (uint32_t)w.pos | ((uint32_t)(ntop + 1) << 26);
}

void spiht_encode(const FieldDev* F, const TileD* tiles, const int* tix, int ntix, uint64_t* lists, uint8_t* slots,
                  const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, uint32_t* tcut, hipStream_t st) {
  if (ntix <= 0) return;
  int ln = pick_tile_lanes(ntix);
#define ENC_L(LN) k_spiht_encode<LN><<<(ntix + LN - 1) / LN, LN, 0, st>>>(F, tiles, tix, ntix, lists, slots, slot_off, \
                                                                      tlen, tent, tcut)
  if (ln == 1) ENC_L(1); else if (ln == 4) ENC_L(4); else if (ln == 16) ENC_L(16); else ENC_L(64);
#undef ENC_L
}

// Bit reader; a read at or past `limit` (the cut of a byte-cut tile) returns
// -1 and decoding of the tile stops there.
struct BitR {
  const uint8_t* in;
  int64_t len, pos, limit;
  __device__ int get() {
    if (pos >= limit) return -1;
    int64_t by = pos >> 3;
    int b = (by < len) ? (in[by] >> (7 - (pos & 7))) & 1 : 0;
    pos++;
    return b;
  }
};

// sec: residual section (tile table then payloads); toff[t]: offset of tile
// t's payload after the table.  mags: N-sized scratch (magnitude | lowest
// known plane << 24 | sign << 31).  CUT: one lane per field, decoding the
// cut tile of a byte-cut field (tix unused); otherwise one lane per listed
// tile, the cut tiles skipped.
template <int LANES, bool CUT>
__global__ __launch_bounds__(LANES) void k_spiht_decode(const FieldDev* __restrict__ F, const TileD* __restrict__ tiles,
                                                        const int* __restrict__ tix, int ntix,
                                                        const int64_t* __restrict__ toff,
                                                        uint64_t* __restrict__ lists) {
  const int q = blockIdx.x * LANES + threadIdx.x;
  if (q >= ntix) return;
  int t;
  if (CUT) {
    const FieldDev& ff = F[q];
    if (!ff.active || ff.rb == 0 || !ff.bt) return;
    const uint8_t* tr = ff.out + kHdr + ff.bb + ff.rb - 8;
    const uint32_t w0 = (uint32_t)tr[0] | ((uint32_t)tr[1] << 8) | ((uint32_t)tr[2] << 16) | ((uint32_t)tr[3] << 24);
    const uint32_t J = w0 & 0x7FFFFFFFu;
    if (J >= (uint32_t)ff.ntiles) { atomicOr(&ff.flags[1], 1); return; }   // names no tile of the field
    t = ff.tile0 + (int)J;
  } else {
    t = tix[q];
  }
  TileD td = tiles[t];
  const FieldDev& f = F[td.field];
  if (!f.active || f.rb == 0) return;
  const Band* B = f.bands;
  const int nx = f.nx, L = f.L, n_s = f.ns, e_r = f.er;
  const uint8_t* sec = f.out + kHdr + f.bb;
  const int64_t sec_len = f.rb;
  uint32_t* mags = f.qr;
  float* chat = f.buf[BUF_CHAT];
  int* flag = &f.flags[1];
  const int tl = t - f.tile0;
  uint32_t ent = (uint32_t)sec[4 * tl] | ((uint32_t)sec[4 * tl + 1] << 8) | ((uint32_t)sec[4 * tl + 2] << 16) |
                 ((uint32_t)sec[4 * tl + 3] << 24);
  int64_t len = ent & 0x3FFFFFF;
  int ntop = (int)(ent >> 26) - 1;
  int64_t pbase = 4 * (int64_t)f.ntiles;      // payloads follow the tile table
  int64_t o0 = toff[t];
  // byte-cut fields: the trailer names the cut tile J (its code ends after
  // lJ bits) and where the other tiles stop
  int n_bot = n_s, sort_only = 0;
  int64_t pay_end = sec_len, limit = 8 * len;
  if (f.bt) {
    pay_end = sec_len - 8;
    const uint8_t* tr = sec + pay_end;
    const uint32_t w0 = (uint32_t)tr[0] | ((uint32_t)tr[1] << 8) | ((uint32_t)tr[2] << 16) | ((uint32_t)tr[3] << 24);
    const uint32_t lJ = (uint32_t)tr[4] | ((uint32_t)tr[5] << 8) | ((uint32_t)tr[6] << 16) | ((uint32_t)tr[7] << 24);
    const int J = (int)(w0 & 0x7FFFFFFFu), kind = (int)(w0 >> 31);
    if (!CUT && tl == J) return;
    cut_tile_mode(kind, J, tl, n_s, &n_bot, &sort_only);
    if (tl == J) {
      if ((int64_t)lJ > 8 * len || (int64_t)lJ <= 8 * (len - 1)) { atomicOr(flag, 1); return; }
      limit = lJ;
    }
  }
  if (o0 < 0 || pbase + o0 + len > pay_end || (ntop >= kQBits)) { atomicOr(flag, 1); return; }
  if (ntop < n_bot) return;
  int nc = td.ncoef;
  uint64_t* lip = lists + 4 * td.off;
  uint64_t* lsp = lip + nc;
  uint64_t* lis = lsp + nc;
  int nlip = 0, nlsp = 0, nlis = 0;
  uint64_t o[9];
  for (int i = td.i0; i < td.i1; i++)
    for (int j = td.j0; j < td.j1; j++) {
      uint64_t n = mk_node(0, i, j);
      lip[nlip++] = n | kAlive;
      if (offspring(B, L, 0, i, j, o) > 0) lis[nlis++] = n | kAlive;
    }
  BitR r{sec + pbase + o0, len, 0, limit};
  constexpr uint32_t kPkMask = 0x1Fu << 24;
  for (int pl = ntop; pl >= n_bot; pl--) {
    uint32_t thr = 1u << pl;
    int lsp_prev = nlsp;
    for (int k = 0; k < nlip; k++) {
      uint64_t e = lip[k];
      if (!(e & kAlive)) continue;
      const int s = r.get();
      if (s < 0) goto done;
      if (s) {
        const int sg = r.get();
        if (sg < 0) goto done;
        mags[nd_pos(B, nx, e)] = thr | ((uint32_t)pl << 24) | ((uint32_t)sg << 31);
        lsp[nlsp++] = e & ~kAlive;
        lip[k] = e & ~kAlive;
      }
    }
    for (int k = 0; k < nlis; k++) {
      uint64_t e = lis[k];
      if (!(e & kAlive)) continue;
      int band = nd_band(e), i = nd_i(e), j = nd_j(e);
      int no = offspring(B, L, band, i, j, o);
      const int s = r.get();
      if (s < 0) goto done;
      if (!(e & kTypeB)) {
        if (!s) continue;
        for (int c = 0; c < no; c++) {
          const int sc = r.get();
          if (sc < 0) goto done;
          if (sc) {
            const int sg = r.get();
            if (sg < 0) goto done;
            mags[nd_pos(B, nx, o[c])] = thr | ((uint32_t)pl << 24) | ((uint32_t)sg << 31);
            lsp[nlsp++] = o[c];
          } else {
            lip[nlip++] = o[c] | kAlive;
          }
        }
        lis[k] = e & ~kAlive;
        if (no > 0 && child_level(B, L, band) >= 2) lis[nlis++] = (e & ~kAlive) | kTypeB | kAlive;
      } else {
        if (!s) continue;
        for (int c = 0; c < no; c++) lis[nlis++] = o[c] | kAlive;
        lis[k] = e & ~kAlive;
      }
    }
    if (pl == n_bot && sort_only) break;
    for (int k = 0; k < lsp_prev; k++) {
      int p = nd_pos(B, nx, lsp[k]);
      const int b = r.get();
      if (b < 0) goto done;
      mags[p] = (mags[p] & ~kPkMask) | ((uint32_t)pl << 24) | (b ? thr : 0u);
    }
  }
done:
  for (int k = 0; k < nlsp; k++) {
    int p = nd_pos(B, nx, lsp[k]);
    uint32_t v = mags[p];
    uint32_t m = v & 0x7FFFFFu;
    const int pk = (int)((v >> 24) & 0x1Fu);
    float f = ldexpf((float)(2u * m + (1u << pk)), e_r - 1);
    chat[p] = (v >> 31) ? -f : f;
  }
}

void spiht_decode(const FieldDev* F, const TileD* tiles, const int* tix, int ntix, const int64_t* toff,
                  uint64_t* lists, hipStream_t st) {
  if (ntix <= 0) return;
  int ln = pick_tile_lanes(ntix);
#define DEC_L(LN) k_spiht_decode<LN, false><<<(ntix + LN - 1) / LN, LN, 0, st>>>(F, tiles, tix, ntix, toff, lists)
  if (ln == 1) DEC_L(1); else if (ln == 4) DEC_L(4); else if (ln == 16) DEC_L(16); else DEC_L(64);
#undef DEC_L
}

void spiht_decode_cut(const FieldDev* F, int nf, const TileD* tiles, const int64_t* toff, uint64_t* lists,
                      hipStream_t st) {
  if (nf <= 0) return;
  k_spiht_decode<64, true><<<(nf + 63) / 64, 64, 0, st>>>(F, tiles, nullptr, nf, toff, lists);
}

}  // namespace ebcc
