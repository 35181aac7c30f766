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

enum { ORI_LL = 0, ORI_HL = 1, ORI_LH = 2, ORI_HH = 3 };
enum { MODE_CONST = 0, MODE_RAW = 1, MODE_CODED = 2 };

// A subband of the Mallat layout.
struct Band {
  int level, orient;
  int y0, x0, h, w;
  int gain;            // g_b: log2 of the subband's synthesis gain, rounded
};

// A code-block: position in the Mallat array, size, subband class and gain.
struct Blk {
  int y0, x0;
  int w, h;
  int orient, gain;
};

// A SPIHT tile: LL root rectangle and the offset of its list storage.
struct TileD {
  int i0, j0, i1, j1;  // LL roots [i0, i1) x [j0, j1)
  int64_t off;         // start of this tile's slice in the per-coefficient scratch
  int ncoef;           // coefficients in the tile's trees
  int pad;
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

// Device kernels' launch wrappers (all asynchronous on `st`).
// dwt.hip
enum { PRO_COPY = 0, PRO_NORM = 1, PRO_NORM_MINUS = 2 };
enum { EPI_STORE = 0, EPI_FINAL = 1, EPI_CHECK = 2 };
struct DwtIO {
  const float* x;            // original field (prologue/epilogue)
  const float* abase;        // base reconstruction (prologue NORM_MINUS, epilogues)
  float* xout;               // EPI_FINAL output
  int* flag;                 // EPI_CHECK violation flag
  const FieldParams* fp;     // xmin, inv_f, range_f, eps
};
// Forward multi-level DWT. Level 1 reads `src` through the prologue; the
// result (Mallat layout) is left in `a`.  `tmp` is an ny*nx scratch.
void dwt_forward(const float* src, float* a, float* tmp, int ny, int nx, int L, int prologue,
                 const DwtIO& io, hipStream_t st);
// Inverse multi-level DWT of `a` (destroyed).  The last level writes the
// result through the epilogue into `out` (EPI_STORE), io.xout (EPI_FINAL),
// or only checks it (EPI_CHECK).
void dwt_inverse(float* a, float* tmp, float* out, int ny, int nx, int L, int epilogue,
                 const DwtIO& io, hipStream_t st);
// Elementwise forms used when L = 0 and for the base-only check.
void pointwise(const float* src, float* dst, int n, int prologue, int epilogue, const DwtIO& io,
               hipStream_t st);

// t1.hip
void quant_planes(const float* coef, int nx, const Blk* blk, int nblk, int e0, int cbw, int cbh,
                  void* planes, void* signs, uint8_t* pb, hipStream_t st);
void t1_encode(const float* coef, int nx, const Blk* blk, int nblk, int e0, int cbw, int cbh,
               const void* planes, const void* signs, const uint8_t* pb, uint8_t* cw,
               int32_t* R, int64_t* D, int32_t* bp, uint32_t* tail, void* sppf, hipStream_t st);
void virtual_decode(const float* coef, int nx, const Blk* blk, int nblk, int e0, int cbw, int cbh,
                    const uint8_t* pb, const uint8_t* kb, const void* sppf, float* yhat, hipStream_t st);
void t1_decode(const uint8_t* sec, int64_t sec_len, const uint32_t* table, const int64_t* off,
               int nx, const Blk* blk, int nblk, int e0, int cbw, int cbh, float* yhat, int* flag,
               hipStream_t st);

// t1wave.hip: one wavefront per code-block (few blocks in flight)
void t1_encode_wave(const float* coef, int nx, const Blk* blk, int nblk, int e0, int cbw, int cbh,
                    const void* planes, const void* signs, const uint8_t* pb, uint8_t* cw,
                    int32_t* R, int64_t* D, int32_t* bp, uint32_t* tail, void* sppf, hipStream_t st);
void t1_decode_wave(const uint8_t* sec, int64_t sec_len, const uint32_t* table, const int64_t* off,
                    int nx, const Blk* blk, int nblk, int e0, int cbw, float* yhat, int* flag,
                    hipStream_t st);
// Tier-1 kernel choice: 0 = by work size, 1 = wave per block, 2 = lane per block.
int t1_variant();

// pcrd.hip
void pcrd(const uint8_t* pb, const int32_t* R, const int64_t* D, int nblk, int64_t budget,
          uint8_t* kb, uint8_t* hk_scratch, uint64_t* key_scratch, int32_t* dr_scratch,
          uint8_t* nh_scratch, int32_t* len_out, hipStream_t st);

// spiht.hip
// qr: per-coefficient residual magnitude (bits 0..22) and sign (bit 31).
void spiht_maxima(const uint32_t* qr, int nx, const Band* bands_dev, const Band* bands_host, int nb, int L,
                  uint32_t* sub, uint32_t* maxd, uint32_t* maxl, hipStream_t st);
// Encode every tile for planes n_t .. n_s into its slot of `slots`
// (slot_off[t] .. ); tlen[t] receives the byte length and tent[t] the tile
// table entry.
void spiht_encode(const uint32_t* qr, const uint32_t* sub, const uint32_t* maxd, const uint32_t* maxl, int nx,
                  const Band* bands, int nb, int L, const TileD* tiles, int ntiles, int n_s, uint64_t* lists,
                  uint8_t* slots, const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, hipStream_t st);
// spihtwave.hip: one wavefront per tile with the tile in LDS.  spiht_lds_cap
// gives the LDS capacity class for the largest tile (0 = does not fit).
int spiht_lds_cap(int max_tile_coef);
void spiht_encode_lds(int cap, const uint32_t* qr, const uint32_t* sub, const uint32_t* maxd, const uint32_t* maxl,
                      int nx, const Band* bands, int nb, int L, const TileD* tiles, int ntiles, int n_s,
                      uint8_t* slots, const int64_t* slot_off, uint32_t* tlen, uint32_t* tent, int* misfit,
                      hipStream_t st);
void spiht_decode_lds(int cap, const uint8_t* sec, int64_t sec_len, const int64_t* toff, int nx, const Band* bands,
                      int nb, int L, const TileD* tiles, int ntiles, int n_s, int e_r, float* chat, int* flag,
                      int* misfit, hipStream_t st);
// Decode the residual section: `sec` starts at the tile table.  Uses `mags`
// (ny*nx scratch) for the magnitude|sign of significant coefficients and
// writes their dequantised values into chat (which must be zero elsewhere).
void spiht_decode(const uint8_t* sec, int64_t sec_len, const int64_t* toff, int nx, const Band* bands, int nb,
                  int L, const TileD* tiles, int ntiles, int n_s, int e_r, uint64_t* lists, uint32_t* mags,
                  float* chat, int* flag, hipStream_t st);

}  // namespace ebcc
