// Tier-1 coding (JPEG2000 Part 1 Annexes C and D) with one wavefront per
// code-block, for the latency-bound case of few blocks in flight (one field).
//
// The coding passes are inherently sequential per block, so the wavefront
// runs them as wave-uniform code: the scan position, the MQ registers and
// the current stripe's rows are uniform values (SGPRs, scalar ALU), while
// the vector registers act as a register file for the block: lane y holds
// row y's bit masks (significant, visited in this plane, refined, sign,
// magnitude bit of the current plane).  A stripe's six rows (the four rows
// plus one above and one below) are read into scalars with readlane when
// the stripe starts and written back when it ends.  The 19 context states
// live in one VGPR (lane = context) and the 47-entry probability table in
// another (lane = state), both read with readlane.  The per-pass distortion
// reductions are not computed here (k_t1_dist derives them from the
// magnitudes in closed form).
#include "common.h"
#include "t1_common.h"

#include <cstdlib>
#include <type_traits>

namespace ebcc {

template <typename M> __device__ __forceinline__ M rdl(M v, int l);
template <> __device__ __forceinline__ uint32_t rdl<uint32_t>(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
template <> __device__ __forceinline__ uint64_t rdl<uint64_t>(uint64_t v, int l) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint32_t rdl32(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

// Wave-uniform MQ encoder; lane 0 stores the finished bytes below cap (the
// block's coder buffer, or its MQ area when the buffer also holds raw bits).
struct MQW {
  uint32_t C, A, B;
  int CT, BP, cap;
};
__device__ __forceinline__ void mqw_emit(MQW& e, uint32_t nb, uint8_t* out, int lane) {
  if (lane == 0 && e.BP >= 0 && e.BP < e.cap) out[e.BP] = (uint8_t)e.B;
  e.BP++;
  e.B = nb;
}
__device__ __forceinline__ void mqw_byteout(MQW& e, uint8_t* out, int lane) {
  if (e.B == 0xFF) {
    mqw_emit(e, e.C >> 20, out, lane); e.C &= 0xFFFFF; e.CT = 7;
  } else if (e.C < 0x8000000u) {
    mqw_emit(e, e.C >> 19, out, lane); e.C &= 0x7FFFF; e.CT = 8;
  } else {
    e.B += 1;
    if (e.B == 0xFF) {
      e.C &= 0x7FFFFFF;
      mqw_emit(e, e.C >> 20, out, lane); e.C &= 0xFFFFF; e.CT = 7;
    } else {
      mqw_emit(e, (e.C >> 19) & 0xFF, out, lane); e.C &= 0x7FFFF; e.CT = 8;
    }
  }
}
__device__ __forceinline__ void mqw_renorm(MQW& e, uint8_t* out, int lane) {
  int n = __builtin_clz(e.A) - 16;
  while (n > 0) {
    int s = n < e.CT ? n : e.CT;
    e.A <<= s; e.C <<= s; e.CT -= s; n -= s;
    if (e.CT == 0) mqw_byteout(e, out, lane);
  }
}
// Context states live one per lane: lane c holds context c's whole table
// entry with its MPS in bit 31 and, in place of Qe, T = Qe + 0x8000 in the
// low half (NMPS << 16 | NLPS << 22 | SWITCH << 28 as in the table).  The
// common step (the MPS, A staying >= 0x8000, i.e. A >= T beforehand) is then
// one read and one compare.  tabv: lane i holds table entry i in the same
// form, read only when a state moves.  Everything is written with integer
// 0/1 values and masks: uniform booleans would otherwise become lane masks
// and pull the coder's arithmetic into dependent vector instructions.
__device__ __forceinline__ uint32_t mq_tab_init(int lane) { return lane < 47 ? c_mqt[lane] + 0x8000u : 0u; }
__device__ __forceinline__ uint32_t mq_ctx_init(int lane) {
  // T.800 Table D.7: all-zero neighbourhood context at index 4, run-length
  // at index 3, uniform at index 46, every other context at index 0
  const int idx = lane == 0 ? 4 : (lane == CX_RL ? 3 : (lane == CX_UNI ? 46 : 0));
  return lane < kNCtx ? c_mqt[idx] + 0x8000u : 0u;
}
// State after coding with state cs; x = 1 for the LPS, 0 for the MPS (the
// LPS moves to NLPS and flips the MPS when SWITCH is set).
__device__ __forceinline__ uint32_t mq_next(uint32_t cs, uint32_t x, uint32_t tabv) {
  const uint32_t m = (cs >> 31) ^ (x & (cs >> 28));
  return rdl32(tabv, (int)((cs >> (16 + 6 * x)) & 0x3f)) | (m << 31);
}
__device__ __forceinline__ void mqw_encode(MQW& e, uint32_t& ctxv, uint32_t tabv, int cx, int d, uint8_t* out, int lane) {
  const uint32_t cs = rdl32(ctxv, cx);
  const uint32_t key = (cs ^ ((uint32_t)d << 31)) & 0x8000FFFFu;   // T, plus bit 31 for the LPS
  if (__builtin_expect(key <= e.A, 1)) {
    const uint32_t q = key - 0x8000u;
    e.A -= q;
    e.C += q;
    return;
  }
  const uint32_t q = (cs & 0xFFFFu) - 0x8000u;
  const uint32_t Am = e.A - q;
  const uint32_t x = key >> 31;
  // the upper sub-interval (size A - Qe) goes to the MPS unless it is the
  // smaller one (conditional exchange)
  const uint32_t up = (x ^ 1u) ^ ((Am - q) >> 31);
  const uint32_t mu = 0u - up;
  e.A = q + ((Am - q) & mu);
  e.C += q & mu;
  const uint32_t ncs = mq_next(cs, x, tabv);
  if (lane == cx) ctxv = ncs;
  const int n = __builtin_clz(e.A) - 16;
  if (__builtin_expect(n < e.CT, 1)) {
    e.A <<= n;
    e.C <<= n;
    e.CT -= n;
  } else {
    mqw_renorm(e, out, lane);
  }
}
__device__ __forceinline__ int mqw_flush_copy(const MQW& e, uint32_t* tail) {
  uint32_t C = e.C, tempc = C + e.A;
  C |= 0xFFFF;
  if (C >= tempc) C -= 0x8000;
  uint32_t t0 = e.B, t1 = 0, t2 = 0;
  int CT = e.CT;
  // first BYTEOUT: byte 0 is the pending byte B
  C <<= CT;
  if (t0 == 0xFF) { t1 = (C >> 20) & 0xFF; C &= 0xFFFFF; CT = 7; }
  else if (C < 0x8000000u) { t1 = (C >> 19) & 0xFF; C &= 0x7FFFF; CT = 8; }
  else {
    t0 = (t0 + 1) & 0x1FF;
    if (t0 == 0xFF) { C &= 0x7FFFFFF; t1 = (C >> 20) & 0xFF; C &= 0xFFFFF; CT = 7; }
    else { t0 &= 0xFF; t1 = (C >> 19) & 0xFF; C &= 0x7FFFF; CT = 8; }
  }
  // second BYTEOUT: the pending byte is t1
  C <<= CT;
  if (t1 == 0xFF) { t2 = (C >> 20) & 0xFF; }
  else if (C < 0x8000000u) { t2 = (C >> 19) & 0xFF; }
  else {
    t1 += 1;
    if (t1 == 0xFF) { C &= 0x7FFFFFF; t2 = (C >> 20) & 0xFF; }
    else { t1 &= 0xFF; t2 = (C >> 19) & 0xFF; }
  }
  *tail = (t0 & 0xFF) | ((t1 & 0xFF) << 8) | ((t2 & 0xFF) << 16);
  return e.BP + 3 - (t2 == 0xFF ? 1 : 0);
}

// Raw bits of the bypassed passes (arithmetic-coding bypass), wave-uniform:
// n bits pending in acc (first bit in bit 31), W words stored.  Lane 0
// stores each full word MSB-first (big-endian bytes) into the raw area.
struct RawW {
  uint32_t acc;
  int n, W;
};
__device__ __forceinline__ void raww_put(RawW& r, int d, uint8_t* raw, int lane) {
  r.acc |= (uint32_t)d << (31 - r.n);
  if (++r.n == 32) {
    if (lane == 0 && r.W < kRawCap / 4) reinterpret_cast<uint32_t*>(raw)[r.W] = __builtin_bswap32(r.acc);
    r.W++;
    r.acc = 0;
    r.n = 0;
  }
}

template <typename M>
__device__ __forceinline__ M wmask_of(int w) {
  return (w >= MaskBits<M>::value) ? ~(M)0 : (((M)1 << w) - 1);
}

// Lane y: the columns of row y with at least one significant neighbour among
// the eight (rows y-1, y, y+1).  Significance does not change during a
// magnitude refinement pass, so its contexts are fixed at the pass start
// and computed here for all rows at once.
template <typename M> __device__ __forceinline__ M shfl_row(M v, int src);
template <> __device__ __forceinline__ uint32_t shfl_row<uint32_t>(uint32_t v, int src) {
  return (uint32_t)__shfl((int)v, src);
}
template <> __device__ __forceinline__ uint64_t shfl_row<uint64_t>(uint64_t v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src), hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
template <typename M>
__device__ __forceinline__ M neighbour_mask(M sig, int lane) {
  M up = shfl_row<M>(sig, lane > 0 ? lane - 1 : 0);
  M dn = shfl_row<M>(sig, lane < 63 ? lane + 1 : 63);
  if (lane == 0) up = 0;
  if (lane == 63) dn = 0;
  M v = up | dn;
  return (sig << 1) | (sig >> 1) | v | (v << 1) | (v >> 1);
}

__device__ __forceinline__ uint64_t lane_ptr(uint32_t pv, int i) {
  return (uint64_t)rdl32(pv, 2 * i) | ((uint64_t)rdl32(pv, 2 * i + 1) << 32);
}

// Zero-coding contexts as a table in one vector register: the neighbourhood
// pattern u3 | m3 << 3 | d3 << 6 (three f3 fields of the rows above, at and
// below the sample) indexes 512 four-bit labels, eight per lane.
__device__ __forceinline__ uint32_t zc_table(int orient, int lane) {
  uint32_t t = 0;
  for (int j = 0; j < 8; j++) t |= (uint32_t)zc_entry(orient, 8u * (uint32_t)lane + (uint32_t)j) << (4 * j);
  return t;
}
__device__ __forceinline__ int zc_look(uint32_t zct, uint32_t pat) {
  return (int)((rdl32(zct, (int)(pat >> 3)) >> (4u * (pat & 7u))) & 15u);
}

// Sign-coding contexts as a table: the pattern of the four neighbours'
// (significant, negative) bits, left | right | above | below with
// sl | nl << 1 | sr << 2 | nr << 3 | su << 4 | nu << 5 | sd << 6 | nd << 7,
// indexes 256 entries of (label - 9) | XOR bit << 3, eight per lane.
__device__ __forceinline__ uint32_t sc_table(int lane) {
  uint32_t t = 0;
  for (int j = 0; j < 8; j++) t |= sc_entry(8u * (uint32_t)lane + (uint32_t)j) << (4 * j);
  return lane < 32 ? t : 0u;
}
// sm, nm: f3 fields of the sample's own row (significance, sign); su, nu,
// sd, nd: the bits above and below.
__device__ __forceinline__ uint32_t sc_look(uint32_t sct, uint32_t sm, uint32_t nm, uint32_t su, uint32_t nu,
                                            uint32_t sd, uint32_t nd) {
  const uint32_t pat = sc_pat(sm, nm, su, nu, sd, nd);
  return (rdl32(sct, (int)(pat >> 3)) >> (4u * (pat & 7u))) & 15u;
}

// Row r' in [-1, 4] of the current stripe's significance / sign rows.
#define SR(rr) ((rr) < 0 ? sA : ((rr) > 3 ? sC : sB[(rr)]))
#define NR(rr) ((rr) < 0 ? nA : ((rr) > 3 ? nC : nB[(rr)]))

// BYP: the launch may hold fields with the arithmetic-coding bypass (their
// significance-propagation and refinement passes after the tenth write raw
// bits; rbt receives the raw bit count of every pass).
template <typename M, bool BYP>
__global__ __launch_bounds__(64) void k_t1_encode_wave(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                       int nblk, int cbh, const M* __restrict__ planes,
                                                       const M* __restrict__ signs, const uint8_t* __restrict__ pbv,
                                                       uint8_t* __restrict__ cw, int32_t* __restrict__ Rt,
                                                       int32_t* __restrict__ bpt,
                                                       uint32_t* __restrict__ tailt, M* __restrict__ sppf,
                                                       int32_t* __restrict__ rbt) {
  const int lane = threadIdx.x;
  const int b = blockIdx.x;
  const Blk k = blk[b];
  if (!F[k.field].active) return;
  const bool byp = BYP && F[k.field].byp;
  const int P = pbv[b];
  const int h = k.h, w = k.w;
  int32_t* R = Rt + (size_t)b * kPassStride;
  int32_t* BPk = bpt + (size_t)b * kPassStride;
  uint32_t* TL = tailt + (size_t)b * kPassStride;
  M* spo = sppf + (size_t)b * cbh;
  int32_t* RB = BYP ? rbt + (size_t)b * kPassStride : nullptr;
  // per-block table pointers used once per pass live in lanes of one vector
  // register (lane 2i / 2i+1: low / high half of pointer i).  They are read
  // back (readlane) only in wave-uniform control flow: inside a branch on the
  // lane index the compiler may fold the lane selects that built the
  // register by that branch's condition and read a lane before it was set.
  uint32_t pv = 0;
  {
    const uint64_t pp[5] = {(uint64_t)R, (uint64_t)BPk, (uint64_t)TL,
                            (uint64_t)(planes + (size_t)b * kQBits * cbh), (uint64_t)RB};
#pragma unroll
    for (int i = 0; i < 5; i++) {
      if (lane == 2 * i) pv = (uint32_t)pp[i];
      if (lane == 2 * i + 1) pv = (uint32_t)(pp[i] >> 32);
    }
  }
  if (lane == 0) {
    R[0] = 0; BPk[0] = -1; TL[0] = 0;
    if (byp) RB[0] = 0;
  }
  if (P == 0) {
    if (lane < h) spo[lane] = 0;
    return;
  }
  uint32_t tabv = mq_tab_init(lane);
  uint32_t ctxv = mq_ctx_init(lane);
  const uint32_t zct = zc_table(k.orient, lane), sct = sc_table(lane);
  M sig = 0, vis = 0, ref = 0, spp = 0, mag = 0;
  M neg = lane < h ? signs[(size_t)b * cbh + lane] : (M)0;
  const M wm = wmask_of<M>(w);
  uint8_t* out = cw + (size_t)b * kCwCap;
  uint8_t* const rawp = out + kRawOff;
  MQW e;
  e.C = 0; e.A = 0x8000; e.B = 0; e.CT = 12; e.BP = -1; e.cap = byp ? kRawOff : kCwCap;
  RawW rw;
  rw.acc = 0; rw.n = 0; rw.W = 0;
  // lengths past these are never kept: stop coding once one is reached
  const int mq_stop = byp ? kBypMqMax : 65536;
  int npass = 3 * P - 2, kk = 0;
  bool stop = false;
  int lrk = 0, lbp = -1;              // the last MQ-coded pass's termination
  uint32_t ltail = 0;
  auto rowv = [&](M v, int y) -> M { return (y >= 0 && y < h) ? rdl<M>(v, y) : (M)0; };

  for (int p = P - 1; p >= 0 && !stop; p--) {
    const M* const pl = (const M*)lane_ptr(pv, 3);
    mag = lane < h ? pl[(size_t)p * cbh + lane] : (M)0;
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3 && !stop; ty++) {
      // pass numbers 11 and later of planes p <= P - 5 (SPP, MRP) are raw
      const bool raw = byp && ty < 2 && p <= P - 5;
      const M nbm8 = (ty == 1) ? neighbour_mask<M>(sig, lane) : (M)0;
      // one instance of the stripe loop per pass type, so that each keeps
      // only the row masks its pass uses live
      auto stripes = [&](auto tyc) {
      constexpr int ty = decltype(tyc)::value;
      for (int y0 = 0; y0 < h && !stop; y0 += 4) {
        const int rn = h - y0 < 4 ? h - y0 : 4;
        M sA = rowv(sig, y0 - 1), sC = rowv(sig, y0 + 4);
        M sB[4], vB[4], fB[4], gB[4], nB[4];
        M nA = 0, nC = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int y = y0 + r;
          bool in = r < rn;
          sB[r] = in ? rdl<M>(sig, y) : (M)0;
          vB[r] = in ? rdl<M>(vis, y) : (M)0;
          fB[r] = (in && ty == 1) ? rdl<M>(ref, y) : (M)0;
          gB[r] = in ? rdl<M>(mag, y) : (M)0;
          // sign rows; in a refinement pass (no sign coding) the rows'
          // neighbour-significance masks instead
          nB[r] = in ? rdl<M>(ty == 1 ? nbm8 : neg, y) : (M)0;
        }
        if (ty != 1) { nA = rowv(neg, y0 - 1); nC = rowv(neg, y0 + 4); }
        // r is a compile-time constant in every caller (unrolled loops)
        auto code_sign = [&](int r, int x) {
          if (ty == 0 && raw) {                          // a raw pass sends the sign itself
            raww_put(rw, btu(nB[r], x), rawp, lane);
            return;
          }
          const uint32_t sc = sc_look(sct, f3(SR(r), x), f3(NR(r), x), btu(SR(r - 1), x), btu(NR(r - 1), x),
                                      btu(SR(r + 1), x), btu(NR(r + 1), x));
          mqw_encode(e, ctxv, tabv, CX_SC + (int)(sc & 7u), btu(nB[r], x) ^ (int)(sc >> 3), out, lane);
        };
        if (ty == 0) {                                   // significance propagation
          // candidate columns at the stripe start; a sample that becomes
          // significant in column x can only add column x + 1
          M c = 0;
#pragma unroll
          for (int r = 0; r < 4; r++)
            if (r < rn) {
              M nb = SR(r - 1) | SR(r) | SR(r + 1);
              nb = nb | (nb << 1) | (nb >> 1);
              c |= ~SR(r) & nb;
            }
          c &= wm;
          while (c) {
            const int x = ctzm(c);
            c &= c - 1;
            bool grew = false;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r >= rn) continue;
              M mid = sB[r];
              if (btu(mid, x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(mid, x), f3(SR(r + 1), x));
              if (!pat) continue;
              int bit = btu(gB[r], x);
              if (raw) raww_put(rw, bit, rawp, lane);
              else mqw_encode(e, ctxv, tabv, zc_look(zct, pat), bit, out, lane);
              vB[r] |= (M)1 << x;
              if (bit) {
                code_sign(r, x);
                sB[r] = mid | ((M)1 << x);
                grew = true;
              }
            }
            if (grew && x + 1 < w) c |= (M)1 << (x + 1);
          }
        } else if (ty == 1) {                            // magnitude refinement
          M mk = 0;
#pragma unroll
          for (int r = 0; r < 4; r++) mk |= sB[r] & ~vB[r];
          while (mk) {
            int x = ctzm(mk);
            mk &= mk - 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r >= rn || !btu(sB[r] & ~vB[r], x)) continue;
              if (raw) {
                raww_put(rw, btu(gB[r], x), rawp, lane);
              } else {
                const int cx = btu(fB[r], x) ? CX_MR + 2 : (btu(nB[r], x) ? CX_MR + 1 : CX_MR);
                mqw_encode(e, ctxv, tabv, cx, btu(gB[r], x), out, lane);
              }
              fB[r] |= (M)1 << x;
            }
          }
        } else {                                         // cleanup
          M u = 0;
#pragma unroll
          for (int r = 0; r < 4; r++)
            if (r < rn) u |= ~(sB[r] | vB[r]);
          u &= wm;
          while (u) {
            int x = ctzm(u);
            u &= u - 1;
            int rstart = 0;
            if (rn == 4) {
              bool run = true;
#pragma unroll
              for (int r = 0; r < 4; r++)
                if (btu(sB[r] | vB[r], x)) run = false;
              if (run) {
                M nbm = nb3<M>(x);
                if ((sA | sB[0] | sB[1] | sB[2] | sB[3] | sC) & nbm) run = false;
              }
              if (run) {
                int rr = -1;
#pragma unroll
                for (int r = 3; r >= 0; r--)
                  if (btu(gB[r], x)) rr = r;
                mqw_encode(e, ctxv, tabv, CX_RL, rr >= 0, out, lane);
                if (rr < 0) continue;
                mqw_encode(e, ctxv, tabv, CX_UNI, (rr >> 1) & 1, out, lane);
                mqw_encode(e, ctxv, tabv, CX_UNI, rr & 1, out, lane);
#pragma unroll
                for (int r = 0; r < 4; r++)
                  if (r == rr) {
                    code_sign(r, x);
                    sB[r] |= (M)1 << x;
                  }
                rstart = rr + 1;
              }
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r < rstart || r >= rn) continue;
              if (btu(sB[r] | vB[r], x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(sB[r], x), f3(SR(r + 1), x));
              int bit = btu(gB[r], x);
              mqw_encode(e, ctxv, tabv, zc_look(zct, pat), bit, out, lane);
              if (bit) {
                code_sign(r, x);
                sB[r] |= (M)1 << x;
              }
            }
          }
        }
        // write the stripe's rows back to the row registers (samples that
        // became significant: the bits new in the stripe's rows)
#pragma unroll
        for (int r = 0; r < 4; r++)
          if (r < rn && lane == y0 + r) {
            if (ty == 0) spp |= sB[r] & ~sig;
            sig = sB[r]; vis = vB[r];
            if (ty == 1) ref = fB[r];
          }
        // every later pass exceeds a length limit
        if (e.BP >= mq_stop || (byp && 32 * rw.W + rw.n > 8 * kBypRawMax)) stop = true;
      }
      };
      if (ty == 0) stripes(std::integral_constant<int, 0>{});
      else if (ty == 1) stripes(std::integral_constant<int, 1>{});
      else stripes(std::integral_constant<int, 2>{});
      if (stop) break;
      if (ty == 2) vis = 0;
      kk++;
      // a raw pass's MQ part is the last MQ-coded pass's codeword
      if (!raw) { lrk = mqw_flush_copy(e, &ltail); lbp = e.BP; }
      int rk = lrk, rbits = 0;
      if (byp) {
        rbits = 32 * rw.W + rw.n;
        const int rby = (rbits + 7) >> 3;
        if (kk >= kBypFirst) rk = 2 + lrk + rby;
        if (lrk > kBypMqMax || rby > kBypRawMax) rk = kRInf;
      }
      int32_t* const Rp = (int32_t*)lane_ptr(pv, 0);
      int32_t* const Bp = (int32_t*)lane_ptr(pv, 1);
      uint32_t* const Tp = (uint32_t*)lane_ptr(pv, 2);
      int32_t* const RBp = BYP ? (int32_t*)lane_ptr(pv, 4) : nullptr;
      if (lane == 0) {
        Rp[kk] = rk; Bp[kk] = lbp; Tp[kk] = ltail;
        if (byp) RBp[kk] = rbits;
      }
    }
  }
  if (lane == 0)
    for (int j = kk + 1; j <= npass; j++) { R[j] = kRInf; BPk[j] = 0; TL[j] = 0; }
  // the raw area's last, partial word
  if (byp && lane == 0 && rw.n && rw.W < kRawCap / 4) reinterpret_cast<uint32_t*>(rawp)[rw.W] = __builtin_bswap32(rw.acc);
  if (lane < h) spo[lane] = spp;
}

// ------------------------------------------------------------------------
// Tier-1 encoding with a pipeline of wavefronts per code-block (blocks of up
// to 32x32).  The significance state at the start of every bit-plane is a
// closed-form function of the magnitudes (significant before plane p iff
// q >> (p + 1) != 0, refined before iff q >> (p + 2) != 0), so the context
// modelling of different planes is independent: NM wavefronts each model
// one plane's three passes at a time, writing the (context, decision)
// pairs to LDS, while wavefront 0 runs the MQ coder over the previous
// round's planes.  Only the MQ coder is sequential; the stream is the one
// the single-wavefront coder writes.
// ------------------------------------------------------------------------
constexpr int kPipeSym = 2816 + 16;   // one 32x32 plane: 1024 decisions + 1024 signs + 256 RL + 512 UNI, padded

// With the arithmetic-coding bypass (BYP, a field's byp) the raw passes'
// records carry the plain decisions (signs uncoded), and wavefront 0 packs
// them into the raw area 256 at a time instead of MQ coding them.
template <int NM, bool BYP>
__global__ __launch_bounds__(64 * (NM + 1)) void k_t1_encode_pipe(
    const FieldDev* __restrict__ F, const Blk* __restrict__ blk, int nblk, int cbh, const uint32_t* __restrict__ planes,
    const uint32_t* __restrict__ signs, const uint8_t* __restrict__ pbv, uint8_t* __restrict__ cw,
    int32_t* __restrict__ Rt, int32_t* __restrict__ bpt, uint32_t* __restrict__ tailt,
    uint32_t* __restrict__ sppf, int32_t* __restrict__ rbt) {
  using M = uint32_t;
  __shared__ __align__(16) uint8_t sym[2][NM][kPipeSym];
  __shared__ int scnt[2][NM][3];
  __shared__ uint32_t sppm[32];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x;
  const Blk k = blk[b];
  if (!F[k.field].active) return;
  const bool byp = BYP && F[k.field].byp;
  const int P = pbv[b];
  const int h = k.h, w = k.w;
  int32_t* R = Rt + (size_t)b * kPassStride;
  int32_t* BPk = bpt + (size_t)b * kPassStride;
  uint32_t* TL = tailt + (size_t)b * kPassStride;
  int32_t* RB = BYP ? rbt + (size_t)b * kPassStride : nullptr;
  uint32_t* spo = sppf + (size_t)b * cbh;
  const uint32_t* const pl = planes + (size_t)b * kQBits * cbh;   // [plane][row] magnitude-bit masks
  if (wv == 0 && lane == 0) {
    R[0] = 0; BPk[0] = -1; TL[0] = 0;
    if (byp) RB[0] = 0;
  }
  if (P == 0) {
    if (wv == 0 && lane < h) spo[lane] = 0;
    return;
  }
  if (threadIdx.x < 32) sppm[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t tabv = mq_tab_init(lane);
  uint32_t ctxv = mq_ctx_init(lane);
  const uint32_t zct = zc_table(k.orient, lane), sct = sc_table(lane);
  const M wm = wmask_of<M>(w);
  auto rowv = [&](M v, int y) -> M { return (y >= 0 && y < h) ? rdl<M>(v, y) : (M)0; };

  // ---- one plane's context modelling (a modelling wavefront) ----
  auto model_plane = [&](const int p, uint8_t* buf, int* cnt) {
    // the row's state at the plane's start from the magnitude-bit masks:
    // significant iff a bit above p is set, refined iff one above p + 1 is
    M sig = 0, ref = 0, mag = 0, vis = 0, spp = 0;
    if (lane < h) {
      for (int pp = P - 1; pp >= p + 2; pp--) ref |= pl[(size_t)pp * cbh + lane];
      sig = ref | (p + 1 < P ? pl[(size_t)(p + 1) * cbh + lane] : (M)0);
      mag = pl[(size_t)p * cbh + lane];
    }
    const M neg = lane < h ? signs[(size_t)b * cbh + lane] : (M)0;
    int n = 0;
    auto emit = [&](int cx, int d) {
      if (lane == 0 && n < kPipeSym - 4) buf[n] = (uint8_t)(cx | (d << 7));   // (the bound always holds)
      n++;
    };
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3; ty++) {
      n = (n + 3) & ~3;                  // every pass starts on a 4-byte boundary
      const int n0 = n;
      const bool raw = byp && ty < 2 && p <= P - 5;   // passes 11 and later, SPP and MRP
      const M nbm8 = (ty == 1) ? neighbour_mask<M>(sig, lane) : (M)0;
        auto stripes = [&](auto tyc) {
        constexpr int ty = decltype(tyc)::value;
        for (int y0 = 0; y0 < h; y0 += 4) {
          const int rn = h - y0 < 4 ? h - y0 : 4;
          M sA = rowv(sig, y0 - 1), sC = rowv(sig, y0 + 4);
          M sB[4], vB[4], fB[4], gB[4], nB[4];
          M nA = 0, nC = 0;
  #pragma unroll
          for (int r = 0; r < 4; r++) {
            int y = y0 + r;
            bool in = r < rn;
            sB[r] = in ? rdl<M>(sig, y) : (M)0;
            vB[r] = in ? rdl<M>(vis, y) : (M)0;
            fB[r] = (in && ty == 1) ? rdl<M>(ref, y) : (M)0;
            gB[r] = in ? rdl<M>(mag, y) : (M)0;
            // sign rows; in a refinement pass (no sign coding) the rows'
            // neighbour-significance masks instead
            nB[r] = in ? rdl<M>(ty == 1 ? nbm8 : neg, y) : (M)0;
          }
          if (ty != 1) { nA = rowv(neg, y0 - 1); nC = rowv(neg, y0 + 4); }
          // r is a compile-time constant in every caller (unrolled loops)
          auto code_sign = [&](int r, int x) {
            if (ty == 0 && raw) {                        // a raw pass sends the sign itself
              emit(0, btu(nB[r], x));
              return;
            }
            const uint32_t sc = sc_look(sct, f3(SR(r), x), f3(NR(r), x), btu(SR(r - 1), x), btu(NR(r - 1), x),
                                        btu(SR(r + 1), x), btu(NR(r + 1), x));
            emit(CX_SC + (int)(sc & 7u), btu(nB[r], x) ^ (int)(sc >> 3));
          };
          if (ty == 0) {                                   // significance propagation
            // candidate columns at the stripe start; a sample that becomes
            // significant in column x can only add column x + 1
            M c = 0;
  #pragma unroll
            for (int r = 0; r < 4; r++)
              if (r < rn) {
                M nb = SR(r - 1) | SR(r) | SR(r + 1);
                nb = nb | (nb << 1) | (nb >> 1);
                c |= ~SR(r) & nb;
              }
            c &= wm;
            while (c) {
              const int x = ctzm(c);
              c &= c - 1;
              bool grew = false;
  #pragma unroll
              for (int r = 0; r < 4; r++) {
                if (r >= rn) continue;
                M mid = sB[r];
                if (btu(mid, x)) continue;
                const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(mid, x), f3(SR(r + 1), x));
                if (!pat) continue;
                int bit = btu(gB[r], x);
                emit(zc_look(zct, pat), bit);
                vB[r] |= (M)1 << x;
                if (bit) {
                  code_sign(r, x);
                  sB[r] = mid | ((M)1 << x);
                  grew = true;
                }
              }
              if (grew && x + 1 < w) c |= (M)1 << (x + 1);
            }
          } else if (ty == 1) {                            // magnitude refinement
            M mk = 0;
  #pragma unroll
            for (int r = 0; r < 4; r++) mk |= sB[r] & ~vB[r];
            while (mk) {
              int x = ctzm(mk);
              mk &= mk - 1;
  #pragma unroll
              for (int r = 0; r < 4; r++) {
                if (r >= rn || !btu(sB[r] & ~vB[r], x)) continue;
                const int cx = btu(fB[r], x) ? CX_MR + 2 : (btu(nB[r], x) ? CX_MR + 1 : CX_MR);
                emit(cx, btu(gB[r], x));
                fB[r] |= (M)1 << x;
              }
            }
          } else {                                         // cleanup
            M u = 0;
  #pragma unroll
            for (int r = 0; r < 4; r++)
              if (r < rn) u |= ~(sB[r] | vB[r]);
            u &= wm;
            while (u) {
              int x = ctzm(u);
              u &= u - 1;
              int rstart = 0;
              if (rn == 4) {
                bool run = true;
  #pragma unroll
                for (int r = 0; r < 4; r++)
                  if (btu(sB[r] | vB[r], x)) run = false;
                if (run) {
                  M nbm = nb3<M>(x);
                  if ((sA | sB[0] | sB[1] | sB[2] | sB[3] | sC) & nbm) run = false;
                }
                if (run) {
                  int rr = -1;
  #pragma unroll
                  for (int r = 3; r >= 0; r--)
                    if (btu(gB[r], x)) rr = r;
                  emit(CX_RL, rr >= 0);
                  if (rr < 0) continue;
                  emit(CX_UNI, (rr >> 1) & 1);
                  emit(CX_UNI, rr & 1);
  #pragma unroll
                  for (int r = 0; r < 4; r++)
                    if (r == rr) {
                      code_sign(r, x);
                      sB[r] |= (M)1 << x;
                    }
                  rstart = rr + 1;
                }
              }
  #pragma unroll
              for (int r = 0; r < 4; r++) {
                if (r < rstart || r >= rn) continue;
                if (btu(sB[r] | vB[r], x)) continue;
                const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(sB[r], x), f3(SR(r + 1), x));
                int bit = btu(gB[r], x);
                emit(zc_look(zct, pat), bit);
                if (bit) {
                  code_sign(r, x);
                  sB[r] |= (M)1 << x;
                }
              }
            }
          }
          // write the stripe's rows back to the row registers (samples that
          // became significant: the bits new in the stripe's rows)
  #pragma unroll
          for (int r = 0; r < 4; r++)
            if (r < rn && lane == y0 + r) {
              if (ty == 0) spp |= sB[r] & ~sig;
              sig = sB[r]; vis = vB[r];
              if (ty == 1) ref = fB[r];
            }
        }
        };
      if (ty == 0) stripes(std::integral_constant<int, 0>{});
      else if (ty == 1) stripes(std::integral_constant<int, 1>{});
      else stripes(std::integral_constant<int, 2>{});
      if (ty == 2) vis = 0;
      if (lane == 0) cnt[ty] = n - n0;
    }
    if (lane < h && spp) atomicOr(&sppm[lane], spp);
  };

  // ---- the MQ coder (wavefront 0) ----
  uint8_t* out = cw + (size_t)b * kCwCap;
  uint8_t* const rawp = out + kRawOff;
  MQW e;
  e.C = 0; e.A = 0x8000; e.B = 0; e.CT = 12; e.BP = -1; e.cap = byp ? kRawOff : kCwCap;
  const int mq_stop = byp ? kBypMqMax : 65536;   // lengths past these are never kept
  int kk = 0;
  bool stop = false;
  int lrk = 0, lbp = -1;             // the last MQ-coded pass's termination
  uint32_t ltail = 0;
  int rbits = 0;                     // raw bits so far; racc: the pending partial word
  uint32_t racc = 0;
  // m <= 256 raw decisions (bit 7 of each record), lane l holding records
  // 4l .. 4l + 3 in wv4, appended MSB-first at bit rbits of the raw area
  auto raw_append = [&](uint32_t wv4, int m) {
    uint32_t nib = 0;
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (4 * lane + j < m) nib |= ((wv4 >> (8 * j + 7)) & 1u) << (3 - j);
    // lane 8t: the chunk's word t (decisions 32t .. 32t + 31, first in bit 31)
    uint32_t part = nib << (28 - 4 * (lane & 7));
    part |= (uint32_t)__shfl_xor((int)part, 1);
    part |= (uint32_t)__shfl_xor((int)part, 2);
    part |= (uint32_t)__shfl_xor((int)part, 4);
    const int o = rbits & 31, W = rbits >> 5, T = (m + 31) >> 5;
    const uint32_t a = (uint32_t)__shfl((int)part, lane < 8 ? 8 * lane : 0);
    const uint32_t pa = (uint32_t)__shfl((int)part, (lane >= 1 && lane <= 8) ? 8 * (lane - 1) : 0);
    // lane t (t <= T): raw word W + t
    uint32_t dw = lane < T ? a >> o : 0u;
    if (lane == 0) dw |= racc;
    else if (o && lane <= T) dw |= pa << (32 - o);
    const int nfull = (o + m) >> 5;
    if (lane < nfull && W + lane < kRawCap / 4) reinterpret_cast<uint32_t*>(rawp)[W + lane] = __builtin_bswap32(dw);
    racc = rdl32(dw, nfull);
    rbits += m;
  };
  auto code_group = [&](const int s, const int g) {
    for (int j = 0; j < NM; j++) {
      const int p = P - 1 - g * NM - j;
      if (p < 0) break;
      const uint8_t* buf = sym[s][j];
      int off = 0;
      for (int ty = (p == P - 1) ? 2 : 0; ty < 3; ty++) {
        const int n = __builtin_amdgcn_readfirstlane(scnt[s][j][ty]);
        const bool raw = byp && ty < 2 && p <= P - 5;
        if (!stop && raw) {
          for (int i = 0; i < n; i += 256) {
            const int m = n - i < 256 ? n - i : 256;
            const bool in = 4 * lane < m && off + i + 4 * lane + 4 <= kPipeSym;
            raw_append(in ? *reinterpret_cast<const uint32_t*>(buf + off + i + 4 * lane) : 0u, m);
          }
        } else if (!stop) {
          for (int i = 0; i < n; i += 256) {
            // 256 decisions at a time: lane l holds bytes 4l .. 4l + 3
            const int m = n - i < 256 ? n - i : 256;
            const bool in = 4 * lane < m && off + i + 4 * lane + 4 <= kPipeSym;
            const uint32_t wv4 = in ? *reinterpret_cast<const uint32_t*>(buf + off + i + 4 * lane) : 0u;
            const int m4 = m & ~3;
            for (int t = 0; t < m4; t += 4) {
              const uint32_t w = rdl32(wv4, t >> 2);
              mqw_encode(e, ctxv, tabv, (int)(w & 0x1Fu), (int)((w >> 7) & 1u), out, lane);
              mqw_encode(e, ctxv, tabv, (int)((w >> 8) & 0x1Fu), (int)((w >> 15) & 1u), out, lane);
              mqw_encode(e, ctxv, tabv, (int)((w >> 16) & 0x1Fu), (int)((w >> 23) & 1u), out, lane);
              mqw_encode(e, ctxv, tabv, (int)((w >> 24) & 0x1Fu), (int)(w >> 31), out, lane);
            }
            if (m4 < m) {
              uint32_t w = rdl32(wv4, m4 >> 2);
              for (int t = m4; t < m; t++, w >>= 8)
                mqw_encode(e, ctxv, tabv, (int)(w & 0x1Fu), (int)((w >> 7) & 1u), out, lane);
            }
          }
        }
        if (!stop) {
          if (e.BP >= mq_stop || (byp && rbits > 8 * kBypRawMax)) {
            stop = true;                 // every later pass exceeds a length limit
          } else {
            kk++;
            // a raw pass's MQ part is the last MQ-coded pass's codeword
            if (!raw) { lrk = mqw_flush_copy(e, &ltail); lbp = e.BP; }
            int rk = lrk;
            if (byp) {
              const int rby = (rbits + 7) >> 3;
              if (kk >= kBypFirst) rk = 2 + lrk + rby;
              if (lrk > kBypMqMax || rby > kBypRawMax) rk = kRInf;
            }
            if (lane == 0) {
              R[kk] = rk; BPk[kk] = lbp; TL[kk] = ltail;
              if (byp) RB[kk] = rbits;
            }
          }
        }
        off += (n + 3) & ~3;
      }
    }
  };

  const int G = (P + NM - 1) / NM;       // rounds of NM planes
  for (int r = 0; r <= G; r++) {
    if (wv >= 1 && r < G) {
      const int j = wv - 1;
      const int p = P - 1 - r * NM - j;
      if (p >= 0) model_plane(p, sym[r & 1][j], scnt[r & 1][j]);
    }
    if (wv == 0 && r >= 1) code_group((r - 1) & 1, r - 1);
    __syncthreads();
  }
  if (wv == 0) {
    if (lane == 0)
      for (int jj = kk + 1; jj <= 3 * P - 2; jj++) { R[jj] = kRInf; BPk[jj] = 0; TL[jj] = 0; }
    // the raw area's last, partial word
    if (byp && lane == 0 && (rbits & 31) && (rbits >> 5) < kRawCap / 4)
      reinterpret_cast<uint32_t*>(rawp)[rbits >> 5] = __builtin_bswap32(racc);
    if (lane < h) spo[lane] = sppm[lane];
  }
}

// ------------------------------------------------------------------------
// Wave-uniform MQ decoder: bytes are read through a uniform 4-byte window;
// bytes past the codeword read as 0xFF.
// ------------------------------------------------------------------------
struct MQWD {
  uint32_t C, A, cur, nxt;
  int CT, BP, len;
  const uint8_t* buf;
  uint64_t wa;
  uint32_t word;
};
__device__ __forceinline__ uint32_t mqwd_rd(MQWD& d, int i) {
  if (i < 0 || i >= d.len) return 0xFFu;
  uint64_t a = (uint64_t)(d.buf + i);
  uint64_t wa = a & ~(uint64_t)3;
  if (wa != d.wa) {
    // the address is wave-uniform; a load through a generic pointer is not
    // known to be, so readfirstlane keeps the coder's state scalar
    d.word = (uint32_t)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const int*>(wa));
    d.wa = wa;
  }
  return (d.word >> (8 * (uint32_t)(a & 3))) & 0xFFu;
}
__device__ __forceinline__ void mqwd_adv(MQWD& d) {
  d.BP++;
  d.cur = d.nxt;
  d.nxt = mqwd_rd(d, d.BP + 1);
}
__device__ __forceinline__ void mqwd_bytein(MQWD& d) {
  if (d.cur == 0xFF) {
    if (d.nxt > 0x8F) { d.C += 0xFF00; d.CT = 8; }
    else { mqwd_adv(d); d.C += d.cur << 9; d.CT = 7; }
  } else {
    mqwd_adv(d); d.C += d.cur << 8; d.CT = 8;
  }
}
__device__ __forceinline__ void mqwd_init(MQWD& d, const uint8_t* buf, int len) {
  d.buf = buf; d.len = len; d.BP = 0; d.wa = ~(uint64_t)0; d.word = 0;
  d.cur = mqwd_rd(d, 0);
  d.nxt = mqwd_rd(d, 1);
  d.C = d.cur << 16;
  mqwd_bytein(d);
  d.C <<= 7; d.CT -= 7; d.A = 0x8000;
}
__device__ __forceinline__ void mqwd_renorm(MQWD& d) {
  do {
    if (d.CT == 0) mqwd_bytein(d);
    d.A <<= 1; d.C <<= 1; d.CT--;
  } while ((d.A & 0x8000) == 0);
}
__device__ __forceinline__ int mqwd_decode(MQWD& d, uint32_t& ctxv, uint32_t tabv, int cx, int lane) {
  const uint32_t cs = rdl32(ctxv, cx);
  const uint32_t T = cs & 0xFFFFu, mps = cs >> 31;
  // the MPS without renormalisation: C at or above Qe and A - Qe >= 0x8000
  const uint32_t ch = (d.C >> 16) + 0x8000u;
  if (__builtin_expect((d.A < ch ? d.A : ch) >= T, 1)) {
    const uint32_t q = T - 0x8000u;
    d.A -= q;
    d.C -= q << 16;
    return (int)mps;
  }
  const uint32_t q = T - 0x8000u;
  const uint32_t A = d.A - q;
  const uint32_t chigh = (ch - T) >> 31;         // C in the lower sub-interval of size Qe
  // the MPS was decoded iff exactly one of: C below Qe, A below Qe
  const uint32_t x = chigh ^ ((A - q) >> 31);    // 1: the LPS
  const uint32_t mc = 0u - chigh;
  d.A = (A & ~mc) | (q & mc);
  d.C -= (q << 16) & ~mc;
  const uint32_t ncs = mq_next(cs, x, tabv);
  if (lane == cx) ctxv = ncs;
  mqwd_renorm(d);
  return (int)(mps ^ x);
}

// Raw bits of the bypassed passes, read MSB-first through a wave-uniform
// 4-byte window like the MQ decoder's; bits past the end read as 0.
struct RawD {
  const uint8_t* buf;
  int nbytes, pos;
  uint64_t wa;
  uint32_t word;
};
__device__ __forceinline__ int rawd_get(RawD& r) {
  const int i = r.pos >> 3;
  uint32_t v = 0;
  if (i < r.nbytes) {
    const uint64_t a = (uint64_t)(r.buf + i), wa = a & ~(uint64_t)3;
    if (wa != r.wa) {
      r.word = (uint32_t)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const int*>(wa));
      r.wa = wa;
    }
    v = r.word >> (8 * (uint32_t)(a & 3));
  }
  const int bit = (int)((v >> (7 - (r.pos & 7))) & 1u);
  r.pos++;
  return bit;
}
// Lane j: raw bits pos + 32j .. pos + 32j + 31, the first in bit 0 (the
// layout of a refinement stripe's decoded bits).
__device__ __forceinline__ uint32_t rawd_words(const RawD& r, int lane) {
  const int s0 = r.pos + 32 * lane, i0 = s0 >> 3;
  uint64_t win = 0;
#pragma unroll
  for (int q = 0; q < 5; q++) win = (win << 8) | (i0 + q < r.nbytes ? r.buf[i0 + q] : 0u);
  return __builtin_bitreverse32((uint32_t)(win >> (8 - (s0 & 7))));
}

// Set bits of m in the columns (lanes) below this lane, and bit `lane` of m.
template <typename M> __device__ __forceinline__ int mbcnt_m(M m);
template <> __device__ __forceinline__ int mbcnt_m<uint32_t>(uint32_t m) {
  return (int)__builtin_amdgcn_mbcnt_lo(m, 0u);
}
template <> __device__ __forceinline__ int mbcnt_m<uint64_t>(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
template <typename M> __device__ __forceinline__ uint32_t col_bit(M m, int lane) {
  return lane < (int)(8 * sizeof(M)) ? (uint32_t)(m >> lane) & 1u : 0u;
}

// BYP: the launch may hold streams with the arithmetic-coding bypass.
template <typename M, bool BYP>
__global__ __launch_bounds__(64) void k_t1_decode_wave(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                       int nblk, const uint32_t* __restrict__ table,
                                                       const int64_t* __restrict__ off) {
  __shared__ uint32_t qm[64 * 64];   // decoded magnitudes [y][x], pitch 64
  __shared__ uint32_t rsym[64];      // a stripe's refinement contexts, one byte each
  const int lane = threadIdx.x;
  const int b = blockIdx.x;
  const Blk k = blk[b];
  const FieldDev& f = F[k.field];
  if (!f.active) return;
  const uint8_t* __restrict__ sec = f.out + kHdr + 4 * (size_t)f.nblk;
  const int64_t sec_len = (int64_t)f.bb - 4 * (int64_t)f.nblk;
  const int nx = f.nx, e0 = f.e0;
  float* yhat = f.buf[BUF_YHAT];
  int* flag = &f.flags[1];
  const int h = k.h, w = k.w;
  const uint32_t ent = table[b];
  const int P = ent & 0xFF, kb = (ent >> 8) & 0xFF, len = (int)(ent >> 16);
  const int64_t o = off[b];
  float* yb = yhat + (size_t)k.y0 * nx + k.x0;
  bool bad = P > kQBits || kb > (P ? 3 * P - 2 : 0) || o < 0 || o + len > sec_len;
  // bypass codeword after more than ten passes: u16 raw byte count, the MQ
  // codeword, the raw bytes
  const bool rawcw = BYP && f.byp && kb >= kBypFirst;
  int rby = 0;
  if (rawcw && !bad) {
    if (len < 2) {
      bad = true;
    } else {
      rby = __builtin_amdgcn_readfirstlane((int)sec[o] | ((int)sec[o + 1] << 8));
      if (2 + rby > len) bad = true;
    }
  }
  if (bad && lane == 0) atomicOr(flag, 1);
  if (bad || P == 0 || kb == 0) {
    for (int i = lane; i < w * h; i += 64) {
      int y = i / w, x = i - y * w;
      yb[(size_t)y * nx + x] = 0.0f;
    }
    return;
  }
  for (int i = lane; i < 64 * 64; i += 64) qm[i] = 0;
  __syncthreads();
  uint32_t tabv = mq_tab_init(lane);
  uint32_t ctxv = mq_ctx_init(lane);
  const uint32_t zct = zc_table(k.orient, lane), sct = sc_table(lane);
  M sig = 0, vis = 0, ref = 0, neg = 0, cur = 0, magp = 0;
  const M wm = wmask_of<M>(w);
  MQWD d;
  mqwd_init(d, sec + o + (rawcw ? 2 : 0), rawcw ? len - 2 - rby : len);
  RawD rr;
  rr.buf = sec + o + len - rby; rr.nbytes = rby; rr.pos = 0; rr.wa = ~(uint64_t)0; rr.word = 0;
  auto rowv = [&](M v, int y) -> M { return (y >= 0 && y < h) ? rdl<M>(v, y) : (M)0; };
  int done = 0, plast = P - 1;
  for (int p = P - 1; p >= 0 && done < kb; p--) {
    plast = p;
    cur = 0;
    magp = 0;
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3 && done < kb; ty++) {
      // pass numbers 11 and later of planes p <= P - 5 (SPP, MRP) are raw
      const bool raw = rawcw && ty < 2 && p <= P - 5;
      const M nbm8 = (ty == 1) ? neighbour_mask<M>(sig, lane) : (M)0;
      auto stripes = [&](auto tyc) {
      constexpr int ty = decltype(tyc)::value;
      for (int y0 = 0; y0 < h; y0 += 4) {
        const int rn = h - y0 < 4 ? h - y0 : 4;
        M sA = rowv(sig, y0 - 1), sC = rowv(sig, y0 + 4);
        M nA = rowv(neg, y0 - 1), nC = rowv(neg, y0 + 4);
        M sB[4], vB[4], fB[4], nB[4], mB[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int y = y0 + r;
          bool in = r < rn;
          sB[r] = in ? rdl<M>(sig, y) : (M)0;
          vB[r] = in ? rdl<M>(vis, y) : (M)0;
          fB[r] = (in && ty == 1) ? rdl<M>(ref, y) : (M)0;
          // decoded signs; in a refinement pass (no sign decoding) the
          // rows' neighbour-significance masks instead
          nB[r] = in ? rdl<M>(ty == 1 ? nbm8 : neg, y) : (M)0;
          mB[r] = 0;
        }
        auto dec_sign = [&](int r, int x) {
          int s;
          if (ty == 0 && raw) {
            s = rawd_get(rr);                            // a raw pass sends the sign itself
          } else {
            const uint32_t sc = sc_look(sct, f3(SR(r), x), f3(NR(r), x), btu(SR(r - 1), x), btu(NR(r - 1), x),
                                        btu(SR(r + 1), x), btu(NR(r + 1), x));
            s = mqwd_decode(d, ctxv, tabv, CX_SC + (int)(sc & 7u), lane) ^ (int)(sc >> 3);
          }
          if (s) nB[r] |= (M)1 << x;
        };
        if (ty == 0) {
          // candidate columns at the stripe start; a sample that becomes
          // significant in column x can only add column x + 1
          M c = 0;
#pragma unroll
          for (int r = 0; r < 4; r++)
            if (r < rn) {
              M nb = SR(r - 1) | SR(r) | SR(r + 1);
              nb = nb | (nb << 1) | (nb >> 1);
              c |= ~SR(r) & nb;
            }
          c &= wm;
          while (c) {
            const int x = ctzm(c);
            c &= c - 1;
            bool grew = false;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r >= rn) continue;
              M mid = sB[r];
              if (btu(mid, x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(mid, x), f3(SR(r + 1), x));
              if (!pat) continue;
              const int bit = raw ? rawd_get(rr) : mqwd_decode(d, ctxv, tabv, zc_look(zct, pat), lane);
              vB[r] |= (M)1 << x;
              if (bit) {
                dec_sign(r, x);
                sB[r] = mid | ((M)1 << x);
                grew = true;
              }
            }
            if (grew && x + 1 < w) c |= (M)1 << (x + 1);
          }
        } else if (ty == 1) {
          // Refinement: each context is fixed before the pass (refined in an
          // earlier plane, else the neighbourhood significance at the pass
          // start), so the lanes (one per column) list the stripe's contexts
          // in scan order, a tight loop decodes them, and the lanes take
          // their bits back.
          M Rr[4];
          int tot = 0;
#pragma unroll
          for (int r = 0; r < 4; r++) {
            Rr[r] = r < rn ? (sB[r] & ~vB[r]) : (M)0;
            tot += __builtin_popcountll((uint64_t)Rr[r]);
          }
          tot = __builtin_amdgcn_readfirstlane(tot);
          if (tot) {
            uint8_t* const sb8 = reinterpret_cast<uint8_t*>(rsym);
            int pos = 0;
#pragma unroll
            for (int r = 0; r < 4; r++) pos += mbcnt_m<M>(Rr[r]);
            uint32_t dv = 0;
            if (raw) {
              // a raw refinement pass: the stripe's bits are the next tot raw bits
              if (lane < ((tot + 31) >> 5)) dv = rawd_words(rr, lane);
              rr.pos += tot;
            } else {
              int pw = pos;
#pragma unroll
              for (int r = 0; r < 4; r++)
                if (col_bit<M>(Rr[r], lane)) {
                  const int c = col_bit<M>(fB[r], lane) ? 2 : (int)col_bit<M>(nB[r], lane);
                  sb8[pw++] = (uint8_t)(CX_MR + c);
                }
              const uint32_t wv4 = rsym[lane];
              uint32_t acc = 0;
              const int m4 = tot & ~3;
              for (int t = 0; t < m4; t += 4) {
                const uint32_t wd = rdl32(wv4, t >> 2);
                uint32_t b4 = (uint32_t)mqwd_decode(d, ctxv, tabv, (int)(wd & 0x1Fu), lane);
                b4 |= (uint32_t)mqwd_decode(d, ctxv, tabv, (int)((wd >> 8) & 0x1Fu), lane) << 1;
                b4 |= (uint32_t)mqwd_decode(d, ctxv, tabv, (int)((wd >> 16) & 0x1Fu), lane) << 2;
                b4 |= (uint32_t)mqwd_decode(d, ctxv, tabv, (int)((wd >> 24) & 0x1Fu), lane) << 3;
                acc |= b4 << (t & 31);
                if ((t & 31) == 28) {
                  if (lane == (t >> 5)) dv = acc;
                  acc = 0;
                }
              }
              if (m4 < tot) {
                uint32_t wd = rdl32(wv4, m4 >> 2);
                for (int t = m4; t < tot; t++, wd >>= 8)
                  acc |= (uint32_t)mqwd_decode(d, ctxv, tabv, (int)(wd & 0x1Fu), lane) << (t & 31);
              }
              if (tot & 31) {
                if (lane == (tot >> 5)) dv = acc;
              }
            }
            // bits pos, pos+1, ... belong to this column's rows in order
            const uint32_t lo = (uint32_t)__shfl((int)dv, pos >> 5), hi = (uint32_t)__shfl((int)dv, (pos >> 5) + 1);
            uint32_t win = (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (pos & 31));
#pragma unroll
            for (int r = 0; r < 4; r++) {
              const uint32_t has = col_bit<M>(Rr[r], lane);
              const bool one = has && (win & 1u);
              win >>= has;
              mB[r] = (M)__ballot(one);
              fB[r] |= Rr[r];
            }
          }
        } else {
          M u = 0;
#pragma unroll
          for (int r = 0; r < 4; r++)
            if (r < rn) u |= ~(sB[r] | vB[r]);
          u &= wm;
          while (u) {
            int x = ctzm(u);
            u &= u - 1;
            int rstart = 0;
            if (rn == 4) {
              bool run = true;
#pragma unroll
              for (int r = 0; r < 4; r++)
                if (btu(sB[r] | vB[r], x)) run = false;
              if (run) {
                M nbm = nb3<M>(x);
                if ((sA | sB[0] | sB[1] | sB[2] | sB[3] | sC) & nbm) run = false;
              }
              if (run) {
                if (!mqwd_decode(d, ctxv, tabv, CX_RL, lane)) continue;
                int b1 = mqwd_decode(d, ctxv, tabv, CX_UNI, lane);
                int b0 = mqwd_decode(d, ctxv, tabv, CX_UNI, lane);
                int rr = 2 * b1 + b0;
#pragma unroll
                for (int r = 0; r < 4; r++)
                  if (r == rr) {
                    dec_sign(r, x);
                    sB[r] |= (M)1 << x;
                  }
                rstart = rr + 1;
              }
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r < rstart || r >= rn) continue;
              if (btu(sB[r] | vB[r], x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(sB[r], x), f3(SR(r + 1), x));
              int bit = mqwd_decode(d, ctxv, tabv, zc_look(zct, pat), lane);
              if (bit) {
                dec_sign(r, x);
                sB[r] |= (M)1 << x;
              }
            }
          }
        }
        // write back; the samples coded in this plane: those that became
        // significant (their bit is 1) or were refined (bits in mB)
#pragma unroll
        for (int r = 0; r < 4; r++)
          if (r < rn && lane == y0 + r) {
            if (ty == 1) {
              cur |= sB[r] & ~vB[r];
              magp |= mB[r];
              ref = fB[r];
            } else {
              const M nw = sB[r] & ~sig;
              cur |= nw;
              magp |= nw;
              neg = nB[r];
            }
            sig = sB[r]; vis = vB[r];
          }
      }
      };
      if (ty == 0) stripes(std::integral_constant<int, 0>{});
      else if (ty == 1) stripes(std::integral_constant<int, 1>{});
      else stripes(std::integral_constant<int, 2>{});
      if (ty == 2) vis = 0;
      done++;
    }
    // this plane's decoded bits into the magnitudes of the row
    M mm = magp;
    while (mm) {
      int x = ctzm(mm);
      mm &= mm - 1;
      qm[lane * 64 + x] |= 1u << p;
    }
  }
  __syncthreads();
  const int e = e0 - k.gain;
  if (lane < h) {
    for (int x = 0; x < w; x++) {
      float v = 0.0f;
      if (bt(sig, x)) {
        int pk = bt(cur, x) ? plast : plast + 1;
        v = dequant(qm[lane * 64 + x], pk, bt(neg, x), e);
      }
      yb[(size_t)lane * nx + x] = v;
    }
  }
}

#undef SR
#undef NR

void t1_encode_wave(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const void* planes,
                    const void* signs, const uint8_t* pb, uint8_t* cw, int32_t* R, int32_t* bp,
                    uint32_t* tail, void* sppf, hipStream_t st, int32_t* rbt) {
  if (nblk <= 0) return;
  const char* pe = getenv("EBCC_T1_PIPE");
  const bool pipe = !(pe && pe[0] == '0');
  // three modelling wavefronts: with two the coder still waits for the
  // next planes now and then (1.51 against 1.46 ms per 721x1440 field),
  // with four or five they crowd the compute unit (1.59, 1.69 ms)
#define ENC_W(BYP)                                                                                                  \
  do {                                                                                                             \
    if (cbw <= 32 && cbh <= 32 && pipe)                                                                            \
      k_t1_encode_pipe<3, BYP><<<nblk, 256, 0, st>>>(F, blk, nblk, cbh, (const uint32_t*)planes,                    \
                                                    (const uint32_t*)signs, pb, cw, R, bp, tail,                    \
                                                    (uint32_t*)sppf, rbt);                                          \
    else if (cbw <= 32)                                                                                            \
      k_t1_encode_wave<uint32_t, BYP><<<nblk, 64, 0, st>>>(F, blk, nblk, cbh, (const uint32_t*)planes,              \
                                                          (const uint32_t*)signs, pb, cw, R, bp, tail,              \
                                                          (uint32_t*)sppf, rbt);                                    \
    else                                                                                                           \
      k_t1_encode_wave<uint64_t, BYP><<<nblk, 64, 0, st>>>(F, blk, nblk, cbh, (const uint64_t*)planes,              \
                                                          (const uint64_t*)signs, pb, cw, R, bp, tail,              \
                                                          (uint64_t*)sppf, rbt);                                    \
  } while (0)
  if (rbt) ENC_W(true);
  else ENC_W(false);
#undef ENC_W
}

void t1_decode_wave(const FieldDev* F, const Blk* blk, int nblk, int cbw, const uint32_t* table, const int64_t* off,
                    hipStream_t st, bool byp) {
  if (nblk <= 0) return;
  if (cbw <= 32) {
    if (byp) k_t1_decode_wave<uint32_t, true><<<nblk, 64, 0, st>>>(F, blk, nblk, table, off);
    else k_t1_decode_wave<uint32_t, false><<<nblk, 64, 0, st>>>(F, blk, nblk, table, off);
  } else {
    if (byp) k_t1_decode_wave<uint64_t, true><<<nblk, 64, 0, st>>>(F, blk, nblk, table, off);
    else k_t1_decode_wave<uint64_t, false><<<nblk, 64, 0, st>>>(F, blk, nblk, table, off);
  }
}

}  // namespace ebcc
