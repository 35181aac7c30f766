// Tier-1 helpers shared by the lane-per-block and wave-per-block coders:
// the MQ probability table, context labels and distortion bookkeeping.
#pragma once
#include "common.h"

namespace ebcc {

// MQ probability-estimation table (T.800 Table C.2), packed as
// Qe | NMPS << 16 | NLPS << 22 | SWITCH << 28.
#define MQE(q, nm, nl, sw) ((uint32_t)(q) | ((uint32_t)(nm) << 16) | ((uint32_t)(nl) << 22) | ((uint32_t)(sw) << 28))
static __constant__ uint32_t c_mqt[47] = {
    MQE(0x5601, 1, 1, 1),   MQE(0x3401, 2, 6, 0),   MQE(0x1801, 3, 9, 0),   MQE(0x0AC1, 4, 12, 0),
    MQE(0x0521, 5, 29, 0),  MQE(0x0221, 38, 33, 0), MQE(0x5601, 7, 6, 1),   MQE(0x5401, 8, 14, 0),
    MQE(0x4801, 9, 14, 0),  MQE(0x3801, 10, 14, 0), MQE(0x3001, 11, 17, 0), MQE(0x2401, 12, 18, 0),
    MQE(0x1C01, 13, 20, 0), MQE(0x1601, 29, 21, 0), MQE(0x5601, 15, 14, 1), MQE(0x5401, 16, 14, 0),
    MQE(0x5101, 17, 15, 0), MQE(0x4801, 18, 16, 0), MQE(0x3801, 19, 17, 0), MQE(0x3401, 20, 18, 0),
    MQE(0x3001, 21, 19, 0), MQE(0x2801, 22, 19, 0), MQE(0x2401, 23, 20, 0), MQE(0x2201, 24, 21, 0),
    MQE(0x1C01, 25, 22, 0), MQE(0x1801, 26, 23, 0), MQE(0x1601, 27, 24, 0), MQE(0x1401, 28, 25, 0),
    MQE(0x1201, 29, 26, 0), MQE(0x1101, 30, 27, 0), MQE(0x0AC1, 31, 28, 0), MQE(0x09C1, 32, 29, 0),
    MQE(0x08A1, 33, 30, 0), MQE(0x0521, 34, 31, 0), MQE(0x0441, 35, 32, 0), MQE(0x02A1, 36, 33, 0),
    MQE(0x0221, 37, 34, 0), MQE(0x0141, 38, 35, 0), MQE(0x0111, 39, 36, 0), MQE(0x0085, 40, 37, 0),
    MQE(0x0049, 41, 38, 0), MQE(0x0025, 42, 39, 0), MQE(0x0015, 43, 40, 0), MQE(0x0009, 44, 41, 0),
    MQE(0x0005, 45, 42, 0), MQE(0x0001, 45, 43, 0), MQE(0x5601, 46, 46, 0)};
#undef MQE

constexpr int kNCtx = 19;
constexpr int CX_RL = 17, CX_UNI = 18, CX_MR = 14, CX_SC = 9;

// Zero-coding context label from neighbour significance counts (T.800 D.1).
__device__ __forceinline__ int zc_ctx(int o, int h, int v, int d) {
  if (o == ORI_HH) {
    int hv = h + v;
    if (d >= 3) return 8;
    if (d == 2) return hv ? 7 : 6;
    if (d == 1) return hv >= 2 ? 5 : (hv ? 4 : 3);
    return hv >= 2 ? 2 : hv;
  }
  if (o == ORI_HL) { int t = h; h = v; v = t; }
  if (h == 2) return 8;
  if (h == 1) return v ? 7 : (d ? 6 : 5);
  if (v) return 2 + v;                 // v = 2 -> 4, v = 1 -> 3
  return d >= 2 ? 2 : d;
}
// Sign-coding context (9..13) and XOR bit from clamped contributions.
__device__ __forceinline__ int sc_ctx(int hc, int vc, int* xr) {
  // hc = 0: 9 (vc = 0) or 10, XOR when vc < 0; hc = +-1: 12 + hc*vc, XOR when hc < 0
  int c, x;
  if (hc == 0) { c = vc ? 10 : 9; x = vc < 0; }
  else { c = 12 + hc * vc; x = hc < 0; }
  *xr = x;
  return c;
}

template <typename M> struct MaskBits { static constexpr int value = 8 * sizeof(M); };
template <typename M>
__device__ __forceinline__ int bt(M r, int x) {
  return (x >= 0 && x < MaskBits<M>::value) ? (int)((r >> x) & 1) : 0;
}
template <typename M> __device__ __forceinline__ int ctzm(M v);
template <> __device__ __forceinline__ int ctzm<uint32_t>(uint32_t v) { return __builtin_ctz(v); }
template <> __device__ __forceinline__ int ctzm<uint64_t>(uint64_t v) { return __builtin_ctzll(v); }
template <typename M>
__device__ __forceinline__ M nb3(int x) {   // bits x-1, x, x+1
  M m = (M)1 << x;
  if (x > 0) m |= (M)1 << (x - 1);
  if (x + 1 < MaskBits<M>::value) m |= (M)1 << (x + 1);
  return m;
}

// Bits x-1, x, x+1 of a row mask as bits 0, 1, 2 (0 outside the row), and
// the neighbourhood counts of T.800 Table D.1 from three such fields.
template <typename M>
__device__ __forceinline__ uint32_t f3(M m, int x) {
  return x > 0 ? (uint32_t)(m >> (x - 1)) & 7u : (uint32_t)(m << 1) & 7u;
}
template <>
__device__ __forceinline__ uint32_t f3<uint32_t>(uint32_t m, int x) {
  return (uint32_t)((((uint64_t)m) << 1) >> x) & 7u;
}
template <typename M>
__device__ __forceinline__ int btu(M m, int x) { return (int)((m >> x) & 1); }   // 0 <= x < bits
struct HVD { int h, v, d; bool any; };
__device__ __forceinline__ HVD hvd(uint32_t u3, uint32_t m3, uint32_t d3) {
  HVD r;
  r.h = __builtin_popcount(m3 & 5u);
  r.v = (int)((u3 >> 1) & 1u) + (int)((d3 >> 1) & 1u);
  r.d = __builtin_popcount(u3 & 5u) + __builtin_popcount(d3 & 5u);
  r.any = ((u3 | d3 | (m3 & 5u)) != 0u);
  return r;
}

// Neighbourhood pattern of a sample: u3 | m3 << 3 | d3 << 6 (the f3 fields
// of the rows above, at and below it); with the sample's own bit 0 it is
// nonzero iff a neighbour is significant.
__device__ __forceinline__ uint32_t zc_pat(uint32_t u3, uint32_t m3, uint32_t d3) { return u3 | (m3 << 3) | (d3 << 6); }
// Zero-coding label of a pattern (T.800 Table D.1).
__device__ __forceinline__ int zc_entry(int orient, uint32_t pat) {
  const HVD n = hvd(pat & 7u, (pat >> 3) & 7u, pat >> 6);
  return zc_ctx(orient, n.h, n.v, n.d);
}
// Sign-coding pattern: the four neighbours' (significant, negative) bits,
// left | right | above | below as sl | nl << 1 | sr << 2 | nr << 3 | su << 4 |
// nu << 5 | sd << 6 | nd << 7, from the f3 fields of the sample's own row
// (sm significance, nm sign) and the bits above and below.
__device__ __forceinline__ uint32_t sc_pat(uint32_t sm, uint32_t nm, uint32_t su, uint32_t nu, uint32_t sd,
                                           uint32_t nd) {
  return (sm & 5u) | ((nm & 5u) << 1) | (su << 4) | (nu << 5) | (sd << 6) | (nd << 7);
}
// (label - 9) | XOR bit << 3 of a sign-coding pattern (T.800 Table D.3).
__device__ __forceinline__ uint32_t sc_entry(uint32_t pat) {
  auto c = [&](int sh) { return (pat >> sh) & 1u ? (((pat >> (sh + 1)) & 1u) ? -1 : 1) : 0; };
  int hc = c(0) + c(2), vc = c(4) + c(6);
  hc = hc > 1 ? 1 : (hc < -1 ? -1 : hc);
  vc = vc > 1 ? 1 : (vc < -1 ? -1 : vc);
  int xr;
  const int cx = sc_ctx(hc, vc, &xr);
  return (uint32_t)((cx - CX_SC) | (xr << 3));
}

// Squared-error reductions (units of (step/2)^2) when a sample of magnitude q
// becomes significant at plane p, or is refined at plane p.
__device__ __forceinline__ int64_t sig_delta(uint32_t q, int p) {
  int64_t e0 = 2 * (int64_t)q + 1;
  int64_t m = (int64_t)((q >> p) << p);
  int64_t e1 = e0 - (2 * m + ((int64_t)1 << p));
  return e0 * e0 - e1 * e1;
}
__device__ __forceinline__ int64_t ref_delta(uint32_t q, int p) {
  int64_t e = 2 * (int64_t)q + 1;
  int64_t m0 = (int64_t)((q >> (p + 1)) << (p + 1));
  int64_t m1 = (int64_t)((q >> p) << p);
  int64_t a = e - (2 * m0 + ((int64_t)1 << (p + 1)));
  int64_t b = e - (2 * m1 + ((int64_t)1 << p));
  return a * a - b * b;
}


}  // namespace ebcc
