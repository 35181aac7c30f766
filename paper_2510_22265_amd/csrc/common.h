// Internal declarations shared by the HIP sources of libebcc.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace ebcc {

constexpr int kHdr = 48;             // stream header bytes
constexpr int kQBits = 23;           // quantised magnitudes are < 2^23
constexpr int kPassStride = 68;      // pass-table slots per block: index 0 (nothing) .. 3*23-2
constexpr int kSegRMax = 65535;      // a code-block codeword must fit the u16 table field
constexpr int kCwCap = 65536 + 64;   // codeword slot per block (longer passes are never kept)
constexpr int kMaxLevels = 16;
constexpr int kMaxBands = 3 * kMaxLevels + 1;
constexpr int kRInf = 0x7fffffff;    // length of a pass that can never be kept
// Tier-1 arithmetic-coding bypass (a stream option): passes kBypFirst and
// later (1-based) of the significance-propagation and refinement kinds are
// raw.  A block's coder buffer then holds the MQ bytes below kRawOff and the
// raw bits from kRawOff on; a pass whose MQ codeword exceeds kBypMqMax bytes
// or whose raw bits exceed kBypRawMax bytes is never kept.
constexpr int kBypFirst = 11;
constexpr int kBypMqMax = 49000;
constexpr int kBypRawMax = 16000;
constexpr int kRawOff = kCwCap - 16064;
constexpr int kRawCap = kCwCap - kRawOff;
static_assert(kRawOff % 4 == 0 && kRawCap >= kBypRawMax + 64 && kRawOff >= kBypMqMax + 512, "coder buffer layout");

enum { ORI_LL = 0, ORI_HL = 1, ORI_LH = 2, ORI_HH = 3 };
enum { MODE_CONST = 0, MODE_RAW = 1, MODE_CODED = 2 };

// A subband of the Mallat layout.
struct Band {
  int level, orient;
  int y0, x0, h, w;
  int gain;            // g_b: log2 of the subband's synthesis gain, rounded
};

// A code-block: position in the Mallat array, size, subband class, gain and
// the field (index into the call's field table) it belongs to.
struct Blk {
  int y0, x0;
  int w, h;
  int orient, gain;
  int field;
};

// A SPIHT tile: LL root rectangle, the offset of its list storage, its field.
struct TileD {
  int i0, j0, i1, j1;  // LL roots [i0, i1) x [j0, j1)
  int64_t off;         // start of this tile's slice in the per-coefficient scratch
  int ncoef;           // coefficients in the tile's trees
  int field;
};

// Scalars of one field, produced on the device from the input.
struct FieldParams {
  float xmin, xmax, range_f, inv_f;
  double range_d, eps, eps_norm;
  int nonfinite, mode, elog, e0;
  unsigned int xmin_bits, xmax_bits;   // order-preserving min/max accumulators
};

// Quantised magnitude floor(|y| * 2^sh), capped below 2^23 (power-of-two
// scaling is exact in FP32).
__device__ __forceinline__ uint32_t quantq(float y, int sh) {
  float v = ldexpf(fabsf(y), sh);
  if (!(v < 8388608.0f)) return (1u << kQBits) - 1u;
  return (uint32_t)v;
}
// Midpoint reconstruction sign * (2m + 2^p) * 2^(e-1), exact in FP32.
__device__ __forceinline__ float dequant(uint32_t m, int p, int neg, int e) {
  if (!m) return 0.0f;
  float v = ldexpf((float)(2u * m + (1u << p)), e - 1);
  return neg ? -v : v;
}

// Per-field table entry seen by every kernel: the field's device buffers,
// shape and coding state.  One call (a single field or a batch) passes an
// array of these; work items (code-blocks, tiles, DWT tiles) carry their
// field's index.
enum { BUF_X = 0, BUF_COEF, BUF_TMP, BUF_YHAT, BUF_ABASE, BUF_CRES, BUF_CHAT, BUF_XOUT, NBUF };
struct FieldDev {
  float* buf[NBUF];    // BUF_X is the caller's input (read only)
  FieldParams* fp;
  int* flags;          // [0] bound violated, [1] stream inconsistent
  unsigned* u32s;      // [0] residual magnitude max, [1] checksum
  int64_t* totals;     // [0] base payload bytes, [1] residual payload bytes
  uint32_t *qr, *sub, *maxd, *maxl;
  const Band* bands;   // the field's subband table
  uint8_t* out;        // compressed stream (output of compress, input of decompress)
  int ny, nx, L, nb;
  int blk0, nblk, tile0, ntiles;
  int active, ns, er, e0;
  int64_t budget;      // rate-allocation payload budget
  double err;          // requested bound (range-relative or absolute)
  int bound_mode, mode, nmax, cbl, T;
  uint32_t bb, rb;     // base and residual section bytes (header fields)
  int64_t len;         // stream length
  // Byte-granular truncation of the residual (Algorithm 1's second binary
  // search over one embedded code, the tiles' codes read plane by plane,
  // sorting passes of every tile before refinement passes): bt set; the cut
  // of plane ns is in the sorting (kind 0) or refinement (kind 1) passes, in
  // tile cut_tile (field-local index) after cut_bits bits of its code.
  // cpos[p] (compression): stream position, within its tile's code, of the
  // bit of plane ns that coefficient p needs (its sign bit when it becomes
  // significant in plane ns, its refinement bit when it was significant
  // before); null unless bt.
  uint32_t* cpos;
  int bt, cut_kind, cut_tile;
  uint32_t cut_bits;
  int byp;             // tier-1 passes with the arithmetic-coding bypass
};

// Byte-cut residual: code length (bits) of tile tl (field-local) of a cut
// field, from the tile's bit counts through plane ns + 1 (lo), before plane
// ns's refinement pass (rs) and through plane ns (hi).
__host__ __device__ __forceinline__ uint32_t cut_tile_bits(int kind, int J, uint32_t lJ, int tl, uint32_t lo,
                                                           uint32_t rs, uint32_t hi) {
  if (tl == J) return lJ;
  if (kind == 0) return tl < J ? rs : lo;
  return tl < J ? hi : rs;
}
// Decoding a tile of a cut field: the lowest plane it reaches and whether it
// stops before that plane's refinement pass (the cut tile itself stops at
// its bit count).
__host__ __device__ __forceinline__ void cut_tile_mode(int kind, int J, int tl, int ns, int* nbot, int* sort_only) {
  *nbot = (kind == 0 && tl > J) ? ns + 1 : ns;
  *sort_only = (kind == 0 && tl < J) || (kind == 1 && tl > J) || (kind == 0 && tl == J);
}

// Order of n work items by a key in [0, kQBits] (0 first), stable within a
// key, for the persistent and longest-first launches.  One workgroup of
// kOrderThreads threads: per-thread counts over a contiguous share of the
// items (keys read eight at a time, their loads issued together), a scan
// over (key, thread), a scatter.  order[i] receives map[item] (the item
// itself when map is null); *qctr, when given, is zeroed (a work counter).
constexpr int kOrderThreads = 1024;
template <typename KeyF>
__device__ __forceinline__ void order_by_key(int n, KeyF key, const int* __restrict__ map, int* __restrict__ order,
                                             int* __restrict__ qctr) {
  constexpr int T = kOrderThreads;
  __shared__ int cnt[kQBits + 1][T];
  __shared__ int base[kQBits + 1];
  const int t = threadIdx.x;
  const int per = (n + T - 1) / T;
  const int b0 = t * per < n ? t * per : n;
  const int b1 = b0 + per < n ? b0 + per : n;
  for (int k = 0; k <= kQBits; k++) cnt[k][t] = 0;
  for (int b = b0; b < b1; b += 8) {
    int kk[8];
#pragma unroll
    for (int u = 0; u < 8; u++) kk[u] = b + u < b1 ? key(b + u) : -1;
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (kk[u] >= 0) cnt[kk[u]][t]++;
  }
  __syncthreads();
  if (t <= kQBits) {   // exclusive scan of row t
    int sum = 0;
    for (int u = 0; u < T; u++) { const int v = cnt[t][u]; cnt[t][u] = sum; sum += v; }
    base[t] = sum;
  }
  __syncthreads();
  if (t == 0) {
    int sum = 0;
    for (int k = 0; k <= kQBits; k++) { const int v = base[k]; base[k] = sum; sum += v; }
    if (qctr) *qctr = 0;
  }
  __syncthreads();
  for (int b = b0; b < b1; b += 8) {
    int kk[8];
#pragma unroll
    for (int u = 0; u < 8; u++) kk[u] = b + u < b1 ? key(b + u) : -1;
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (kk[u] >= 0) {
        order[base[kk[u]] + cnt[kk[u]][t]] = map ? map[b + u] : b + u;
        cnt[kk[u]][t]++;
      }
  }
}

// Device kernels' launch wrappers (all asynchronous on `st`).
// dwt.hip
enum { PRO_COPY = 0, PRO_NORM = 1, PRO_NORM_MINUS = 2 };
enum { EPI_STORE = 0, EPI_FINAL = 1, EPI_CHECK = 2 };
// Forward multi-level DWT of every active field (F device table, Fh its host
// copy): level 1 reads buf[src] through the prologue, the Mallat result is
// left in buf[dst]; buf[BUF_TMP] is scratch.
void dwt_forward(const FieldDev* F, const FieldDev* Fh, int nf, int src, int dst, int prologue, hipStream_t st);
// Inverse multi-level DWT of buf[a] (destroyed); the last level goes through
// the epilogue into buf[out] (EPI_STORE), buf[BUF_XOUT] (EPI_FINAL), or only
// checks the bound (EPI_CHECK, flags[0]).
void dwt_inverse(const FieldDev* F, const FieldDev* Fh, int nf, int a, int out, int epilogue, hipStream_t st);
void dwt_inverse_head(const FieldDev* F, const FieldDev* Fh, int nf, int a, hipStream_t st);
void dwt_inverse_tail(const FieldDev* F, const FieldDev* Fh, int nf, int a, int out, int epilogue, hipStream_t st);
// Elementwise prologue (PRO_*, or 3 = zero) and epilogue over whole fields.
void pointwise(const FieldDev* F, const FieldDev* Fh, int nf, int src, int dst, int prologue, int epilogue,
               int lzero_only, hipStream_t st);

// t1.hip / t1wave.hip: code-blocks of every field in one launch; per-block
// tables are indexed by the block's position in the call's block array.
void quant_planes(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, void* planes, void* signs,
                  uint8_t* pb, hipStream_t st);
// Optional second stream (and the two events ordering it against the first)
// for the wave-per-block share of a lanes-per-block launch.
struct T1Split {
  hipStream_t aux;
  hipEvent_t ev_fork, ev_join;
};
// order (nblk ints) and qctr (one int): scratch of the persistent
// lanes-per-block launch, used when that launch is chosen (may be null).
// rbt (nblk * kPassStride): raw bits per block and pass when some field uses
// the bypass (the coders are then instantiated with the raw passes), else
// null.
void t1_encode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const void* planes,
               const void* signs, const uint8_t* pb, uint8_t* cw, int32_t* R, int64_t* D, int32_t* bp,
               uint32_t* tail, void* sppf, hipStream_t st, const T1Split* sp = nullptr, int* order = nullptr,
               int* qctr = nullptr, int32_t* rbt = nullptr);
void virtual_decode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint8_t* pb,
                    const uint8_t* kb, const void* sppf, hipStream_t st);
// table: per-block entries (P | k << 8 | len << 16); off: payload offsets
// within each field's base payload (which starts at out + 48 + 4 nblk).
// byp: some field uses the bypass (the decoders are then instantiated with
// the raw passes).
void t1_decode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint32_t* table,
               const int64_t* off, hipStream_t st, const T1Split* sp = nullptr, int* order = nullptr,
               int* qctr = nullptr, bool byp = false);
void t1_encode_wave(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const void* planes,
                    const void* signs, const uint8_t* pb, uint8_t* cw, int32_t* R, int32_t* bp,
                    uint32_t* tail, void* sppf, hipStream_t st, int32_t* rbt = nullptr);
// Running distortion reductions D[b][0 .. 3P_b - 2] of every block's coding
// passes (closed form from the magnitudes and the encoder's sppf masks);
// t1_encode runs it after the coders.
void t1_distortion(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint8_t* pb,
                   const void* sppf, int64_t* D, hipStream_t st);
void t1_decode_wave(const FieldDev* F, const Blk* blk, int nblk, int cbw, const uint32_t* table,
                    const int64_t* off, hipStream_t st, bool byp = false);
// Kernel choices (process-wide, set through the C ABI; the environment
// variables EBCC_T1_KERNEL=wave|lane and EBCC_SPIHT_KERNEL=global override;
// EBCC_T1_PIPE=0 replaces the pipelined wavefront encoder of 32x32 blocks
// by the single-wavefront one).
struct Tuning {
  int t1_encoder;    // 0 by work size, 1 wave per code-block, 2 lanes per code-block
  int t1_decoder;    // same
  int t1_wave_max;   // by work size: a wave per block up to this many blocks, lanes beyond
  int spiht;         // 0 LDS kernels by capacity class, 1 global-memory lists for every tile
  int t1_lanes;      // lanes-per-block kernels: blocks per wavefront (0 by work size, 1, 4, 16, 64)
  int t1_split;      // percent of a lanes-per-block launch's blocks run concurrently by the wave kernel
  int t1_persist;    // lanes-per-block encoding as one persistent launch over a work counter (0 off, 1 on)
};
Tuning tuning();

// pcrd.hip: one workgroup per field; kb/len per block.
void pcrd(const FieldDev* F, int nf, int max_nblk, const uint8_t* pb, const int32_t* R, const int64_t* D, uint8_t* kb,
          uint8_t* hk_scratch, uint64_t* key_scratch, int32_t* dr_scratch, uint8_t* nh_scratch, int32_t* len_out,
          hipStream_t st);

// spiht.hip: tiles of every field in one launch (global-memory lists).
// FieldDev.qr: residual magnitude (bits 0..22) and sign (bit 31).
void spiht_maxima(const FieldDev* F, const FieldDev* Fh, int nf, hipStream_t st);
// Encode every tile for planes n_t .. F.ns into its slot of `slots`
// (slot_off[t] ..); tlen[t] receives the byte length and tent[t] the tile
// table entry.
// tcut (byte-cut fields; may be null otherwise): per tile the bits through
// plane ns + 1, before plane ns's refinement pass and through plane ns.
void spiht_encode(const FieldDev* F, const TileD* tiles, const int* tix, int ntix, uint64_t* lists, uint8_t* slots,
                  const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, uint32_t* tcut, hipStream_t st);
// Decode residual sections (each field's starts at out + 48 + bb): writes the
// dequantised significant coefficients into buf[BUF_CHAT] (zero elsewhere);
// toff: payload offsets after each field's tile table.
void spiht_decode(const FieldDev* F, const TileD* tiles, const int* tix, int ntix, const int64_t* toff,
                  uint64_t* lists, hipStream_t st);
// The cut tile of every byte-cut field (one lane per field; the other
// decoders skip it): decoded to its bit count.
void spiht_decode_cut(const FieldDev* F, int nf, const TileD* tiles, const int64_t* toff, uint64_t* lists,
                      hipStream_t st);
// spihtwave.hip: one wavefront per tile with the tile in LDS, in three
// capacity classes (the coefficients of the tile's trees, and four times
// its parents, must fit: the decoder's set list holds up to twice the
// parents in half the capacity): small and big for the usual one-root tiles
// of 5 and 6 levels with the edge tiles that take the extra row or column
// of odd-sized bands, huge for larger edge tiles; larger tiles are coded
// with lists in global memory.  LDS per unit of capacity: 9 bytes in the
// decoder (15, 4 and 2 wavefronts per compute unit of 160 KB), 9.5 bytes
// plus the band table in the encoder (11, 3 and 2).
constexpr int kSpihtSmall = 1192;
constexpr int kSpihtBig = 4352;
constexpr int kSpihtHuge = 8192;
// Each SPIHT launch covers the tiles tix[0 .. ntix) of the call's tile array
// (tiles are launched in capacity classes).
void spiht_encode_lds(int cap, const FieldDev* F, const TileD* tiles, const int* tix, int ntix, uint8_t* slots,
                      const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, uint32_t* tcut, int* misfit,
                      hipStream_t st);
// Byte-cut candidates (Fc[0 .. ncand), each a field with its cut): the
// residual coefficients the decoder of that cut would reconstruct, into each
// candidate's buf[BUF_CHAT], from the field's magnitudes (qr), cpos and the
// tiles' tcut; max_tiles: the most tiles of a candidate's field.
void spiht_cut_recon(const FieldDev* Fc, int ncand, int max_tiles, const TileD* tiles, const uint32_t* tcut,
                     hipStream_t st);
// Final tile lengths of the byte-cut fields: tbits[t] = the tile's code bits,
// tlen[t] its bytes and tent[t] its table entry (tent holds the encoder's
// entry on input, for the tile's top plane).
void spiht_cut_tiles(const FieldDev* F, const TileD* tiles, int nt, const uint32_t* tcut, uint32_t* tlen,
                     uint32_t* tent, uint32_t* tbits, hipStream_t st);
void spiht_decode_lds(int cap, const FieldDev* F, const TileD* tiles, const int* tix, int ntix, const int64_t* toff,
                      int* misfit, hipStream_t st);
// The tiles tix[0 .. n) in order of their payload length (from their table
// entries tent), longest first, into out: a launch over them starts the
// longest decodes first.
void spiht_tiles_longest_first(const int* tix, int n, const uint32_t* tent, int* out, hipStream_t st);

}  // namespace ebcc
