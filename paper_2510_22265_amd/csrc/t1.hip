// Base layer of EBCC: dead-zone quantisation, EBCOT tier-1 coding passes and
// the MQ arithmetic coder (JPEG2000 Part 1, Annexes C and D, default mode
// switches), as used by the paper's JPEG2000 base compression layer.
//
// Layout of the work:
//  * k_quant_planes: one wavefront per code-block.  Quantises the block and
//    builds, with ballots, one bit mask per (bit-plane, row) and per row of
//    signs, plus the block's number of magnitude planes P_b.
//  * k_t1_encode: one lane per code-block.  Coding-pass state (significance,
//    visited-in-this-plane, refined, sign, current plane's magnitudes) is kept
//    as one bit mask per block row in LDS, so the scan jumps from candidate
//    column to candidate column instead of visiting every sample.  The MQ
//    coder's registers live in VGPRs, its 19 context states in LDS.  At every
//    pass end the coder is flushed on a copy to obtain the exact terminated
//    length R_k and the bytes termination would write.
//  * k_virtual_decode: one wavefront per block, lanes over samples.  Gives the
//    base reconstruction for the kept passes in closed form (what the decoder
//    recovers), from q, P_b, k_b and a per-sample "became significant in a
//    significance-propagation pass" bit recorded by the encoder.
//  * k_t1_decode: one lane per block; the decoder for decompression.
#include "common.h"

#include <algorithm>
#include "t1_common.h"

#include <cstdlib>

namespace ebcc {

// ------------------------------------------------------------------------
// Quantisation and bit-plane masks (one wavefront per code-block).
// planes: [nblk][kQBits][cbh] masks; signs: [nblk][cbh]; pb: [nblk].
// ------------------------------------------------------------------------
template <typename M>
__global__ __launch_bounds__(256) void k_quant_planes(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                      int nblk, int cbw, int cbh, M* __restrict__ planes,
                                                      M* __restrict__ signs, uint8_t* __restrict__ pb) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int b = blockIdx.x * 4 + wave;
  if (b >= nblk) return;
  Blk k = blk[b];
  if (!F[k.field].active) return;
  const float* coef = F[k.field].buf[BUF_COEF];
  const int nx = F[k.field].nx, e0 = F[k.field].e0;
  int sh = k.gain - e0;
  uint32_t mx = 0;
  for (int i = lane; i < k.w * k.h; i += 64) {
    int y = i / k.w, x = i - y * k.w;
    uint32_t q = quantq(coef[(k.y0 + y) * nx + k.x0 + x], sh);
    mx = q > mx ? q : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t t = __shfl_xor(mx, o);
    mx = t > mx ? t : mx;
  }
  int P = mx ? 32 - __builtin_clz(mx) : 0;
  if (lane == 0) pb[b] = (uint8_t)P;
  // rows per ballot: 64 / cbw (cbw is a power of two <= 64)
  int rpb = 64 / cbw;
  int r = lane / cbw, x = lane - r * cbw;
  M* pl = planes + (size_t)b * kQBits * cbh;
  M* sg = signs + (size_t)b * cbh;
  uint64_t wm = (cbw == 64) ? ~0ull : ((1ull << cbw) - 1ull);
  for (int y0 = 0; y0 < k.h; y0 += rpb) {
    int y = y0 + r;
    bool valid = (x < k.w) && (y < k.h);
    float c = valid ? coef[(k.y0 + y) * nx + k.x0 + x] : 0.0f;
    uint32_t q = valid ? quantq(c, sh) : 0u;
    uint64_t bs = __ballot(valid && c < 0.0f);
    for (int p = 0; p < P; p++) {
      uint64_t bp = __ballot((q >> p) & 1u);
      // lane p keeps plane p's rows; the rows of this ballot go out one by one
      for (int rr = 0; rr < rpb; rr++) {
        if (y0 + rr >= k.h) break;
        M row = (M)((bp >> (rr * cbw)) & wm);
        if (lane == p) pl[(size_t)p * cbh + y0 + rr] = row;
      }
    }
    for (int rr = 0; rr < rpb; rr++) {
      if (y0 + rr >= k.h) break;
      if (lane == 63) sg[y0 + rr] = (M)((bs >> (rr * cbw)) & wm);
    }
  }
}

// ------------------------------------------------------------------------
// MQ encoder in registers.  B is the byte at index BP (not yet written: it
// may still receive a carry); BP = -1 is the dummy byte before the output.
// ------------------------------------------------------------------------
// Bytes are stored below cap: the block's coder buffer, or its MQ area when
// the buffer also holds raw bits (arithmetic-coding bypass).
struct MQEnc {
  uint32_t C, A, B;
  int CT, BP, cap;
  uint8_t* out;
};
__device__ __forceinline__ void mq_emit(MQEnc& e, uint32_t nb) {
  if (e.BP >= 0 && e.BP < e.cap) e.out[e.BP] = (uint8_t)e.B;
  e.BP++;
  e.B = nb;
}
__device__ __forceinline__ void mq_byteout(MQEnc& e) {
  if (e.B == 0xFF) {
    mq_emit(e, e.C >> 20); e.C &= 0xFFFFF; e.CT = 7;
  } else if (e.C < 0x8000000u) {
    mq_emit(e, e.C >> 19); e.C &= 0x7FFFF; e.CT = 8;
  } else {
    e.B += 1;
    if (e.B == 0xFF) {
      e.C &= 0x7FFFFFF;
      mq_emit(e, e.C >> 20); e.C &= 0xFFFFF; e.CT = 7;
    } else {
      mq_emit(e, (e.C >> 19) & 0xFF); e.C &= 0x7FFFF; e.CT = 8;
    }
  }
}
__device__ __forceinline__ void mq_renorm(MQEnc& e) {
  // shift until A >= 0x8000, emitting a byte whenever CT reaches 0
  int n = __builtin_clz(e.A) - 16;
  while (n > 0) {
    int s = n < e.CT ? n : e.CT;
    e.A <<= s; e.C <<= s; e.CT -= s; n -= s;
    if (e.CT == 0) mq_byteout(e);
  }
}
// cs: context state (index | MPS << 7)
__device__ __forceinline__ void mq_encode(MQEnc& e, uint8_t* cs_ptr, int d, const uint32_t* tab) {
  uint32_t cs = *cs_ptr;
  uint32_t ent = tab[cs & 0x7f];
  uint32_t qe = ent & 0xFFFF;
  uint32_t mps = cs >> 7;
  e.A -= qe;
  if ((uint32_t)d == mps) {
    if ((e.A & 0x8000) == 0) {
      if (e.A < qe) e.A = qe; else e.C += qe;
      *cs_ptr = (uint8_t)((cs & 0x80) | ((ent >> 16) & 0x3f));
      mq_renorm(e);
    } else {
      e.C += qe;
    }
  } else {
    if (e.A < qe) e.C += qe; else e.A = qe;
    uint32_t m = (ent >> 28) ? (mps ^ 1u) : mps;
    *cs_ptr = (uint8_t)((m << 7) | ((ent >> 22) & 0x3f));
    mq_renorm(e);
  }
}
// Terminate a copy of the coder: returns the codeword length and the bytes
// written at positions BP, BP+1, BP+2 (packed little-endian in *tail).
__device__ __forceinline__ int mq_flush_copy(const MQEnc& e, uint32_t* tail) {
  uint32_t C = e.C, tempc = C + e.A;
  C |= 0xFFFF;
  if (C >= tempc) C -= 0x8000;
  uint32_t tb[3] = {e.B, 0u, 0u};
  int bp = 0, CT = e.CT;
  for (int r = 0; r < 2; r++) {
    C <<= CT;
    uint32_t B = tb[bp];
    if (B == 0xFF) {
      bp++; tb[bp] = (C >> 20) & 0xFF; C &= 0xFFFFF; CT = 7;
    } else if (C < 0x8000000u) {
      bp++; tb[bp] = (C >> 19) & 0xFF; C &= 0x7FFFF; CT = 8;
    } else {
      B += 1; tb[bp] = B & 0xFF;
      if (B == 0xFF) {
        C &= 0x7FFFFFF; bp++; tb[bp] = (C >> 20) & 0xFF; C &= 0xFFFFF; CT = 7;
      } else {
        bp++; tb[bp] = (C >> 19) & 0xFF; C &= 0x7FFFF; CT = 8;
      }
    }
  }
  *tail = tb[0] | (tb[1] << 8) | (tb[2] << 16);
  return e.BP + 3 - (tb[2] == 0xFF ? 1 : 0);
}

// Coding-pass state of a workgroup's blocks, one bit mask per block row.
// The encoder reads its signs and magnitude bits from the bit-plane masks in
// global memory (read-only, cached), so it keeps four row arrays (more
// workgroups per compute unit); the decoder also keeps the decoded signs.
template <typename M, int ROWS, int LANES, bool ENC>
struct T1Shared {
  M sig[ROWS][LANES], vis[ROWS][LANES], ref[ROWS][LANES];
  M aux[ENC ? ROWS : 1][LANES];   // encoder: the significance-propagation masks
  M neg[ENC ? 1 : ROWS][LANES];
  uint8_t ctx[kNCtx][LANES];
  uint32_t mqt[47];
  // context labels by neighbourhood pattern: zero coding for LL/LH, HL and
  // HH blocks, and sign coding ((label - 9) | XOR bit << 3)
  uint8_t zct[3][512];
  uint8_t sct[256];
  __device__ void fill_tables(int t, int n) {
    for (int i = t; i < 47; i += n) mqt[i] = c_mqt[i];
    for (int i = t; i < 3 * 512; i += n) {
      const int c = i >> 9;
      zct[c][i & 511] = (uint8_t)zc_entry(c == 0 ? ORI_LL : (c == 1 ? ORI_HL : ORI_HH), (uint32_t)(i & 511));
    }
    for (int i = t; i < 256; i += n) sct[i] = (uint8_t)sc_entry((uint32_t)i);
  }
};

// Zero-coding label table of a block of orientation `orient`.
template <typename S_>
__device__ __forceinline__ const uint8_t* ztab_of(const S_& S, int orient) {
  return S.zct[orient == ORI_HH ? 2 : (orient == ORI_HL ? 1 : 0)];
}

// Row r' in [-1, 4] of the current stripe's significance / sign rows.
#define SR(rr) ((rr) < 0 ? sA : ((rr) > 3 ? sC : sB[(rr)]))
#define NR(rr) ((rr) < 0 ? nA : ((rr) > 3 ? nC : nB[(rr)]))

// ------------------------------------------------------------------------
// Tier-1 encoder: one lane per code-block.
// ------------------------------------------------------------------------
// BYP: the launch may hold fields with the arithmetic-coding bypass (their
// significance-propagation and refinement passes after the tenth write raw
// bits into the buffer's raw area; rbt receives each pass's raw bit count).
template <typename M, int ROWS, int LANES, bool BYP>
__device__ __forceinline__ void t1_enc_block(T1Shared<M, ROWS, LANES, true>& S, int lane, int b, const FieldDev* __restrict__ F,
                                             const Blk* __restrict__ blk, int nblk, int cbh,
                                             const M* __restrict__ planes, const M* __restrict__ signs,
                                             const uint8_t* __restrict__ pbv, uint8_t* __restrict__ cw,
                                             int32_t* __restrict__ Rt, int32_t* __restrict__ bpt, uint32_t* __restrict__ tailt,
                                             M* __restrict__ sppf, int32_t* __restrict__ rbt) {
  if (b >= nblk) return;
  Blk k = blk[b];
  if (!F[k.field].active) return;
  const bool byp = BYP && F[k.field].byp;
  int P = pbv[b];
  int32_t* R = Rt + (size_t)b * kPassStride;
  int32_t* BPk = bpt + (size_t)b * kPassStride;
  uint32_t* TL = tailt + (size_t)b * kPassStride;
  R[0] = 0; BPk[0] = -1; TL[0] = 0;
  int32_t* RB = BYP ? rbt + (size_t)b * kPassStride : nullptr;
  if (byp) RB[0] = 0;
  M* spo = sppf + (size_t)b * cbh;
  if (P == 0) {
    for (int y = 0; y < k.h; y++) spo[y] = 0;
    return;
  }
  const uint8_t* zt = ztab_of(S, k.orient);
  const M* sg = signs + (size_t)b * cbh;
  for (int y = 0; y < k.h; y++) {
    S.sig[y][lane] = 0; S.vis[y][lane] = 0; S.ref[y][lane] = 0; S.aux[y][lane] = 0;
  }
  for (int c = 0; c < kNCtx; c++) S.ctx[c][lane] = 0;
  S.ctx[0][lane] = 4; S.ctx[CX_RL][lane] = 3; S.ctx[CX_UNI][lane] = 46;
  MQEnc e;
  e.C = 0; e.A = 0x8000; e.B = 0; e.CT = 12; e.BP = -1; e.out = cw + (size_t)b * kCwCap;
  e.cap = byp ? kRawOff : kCwCap;
  // raw bits: racc holds rnb pending bits (first in bit 31), rwi words stored
  uint32_t racc = 0;
  int rnb = 0, rwi = 0;
  uint32_t* const rawp = reinterpret_cast<uint32_t*>(e.out + kRawOff);
  auto rawput = [&](int d) {
    racc |= (uint32_t)d << (31 - rnb);
    if (++rnb == 32) {
      if (rwi < kRawCap / 4) rawp[rwi] = __builtin_bswap32(racc);
      rwi++;
      racc = 0;
      rnb = 0;
    }
  };
  // lengths past these are never kept: stop coding once one is reached
  const int mq_stop = byp ? kBypMqMax : 65536;
  int lrk = 0, lbp = -1;              // the last MQ-coded pass's termination
  uint32_t ltail = 0;
  auto mq_enc = [&](uint8_t* cs, int bit) { mq_encode(e, cs, bit, S.mqt); };
  int npass = 3 * P - 2, kk = 0;
  bool stop = false;
  const int h = k.h, w = k.w;
  const M wm = (w >= MaskBits<M>::value) ? ~(M)0 : (((M)1 << w) - 1);
  auto rowm = [&](M (*a)[LANES], int y) -> M { return (y >= 0 && y < h) ? a[y][lane] : (M)0; };
  for (int p = P - 1; p >= 0 && !stop; p--) {
    const M* pl = planes + ((size_t)b * kQBits + p) * cbh;
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3 && !stop; ty++) {
      // pass numbers 11 and later of planes p <= P - 5 (SPP, MRP) are raw
      const bool raw = byp && ty < 2 && p <= P - 5;
      // the stripe's rows (and the rows above and below) are held in
      // registers while the stripe is coded, then written back; magnitude
      // bits and signs come from global memory (no sign coding in a
      // refinement pass)
      const bool sgn = ty != 1;
      for (int y0 = 0; y0 < h && !stop; y0 += 4) {
        const int rn = h - y0 < 4 ? h - y0 : 4;
        const M sA = rowm(S.sig, y0 - 1), sC = rowm(S.sig, y0 + 4);
        const M nA = (sgn && y0 > 0) ? sg[y0 - 1] : (M)0, nC = (sgn && y0 + 4 < h) ? sg[y0 + 4] : (M)0;
        M sB[4], vB[4], fB[4], gB[4], nB[4], aB[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const bool in = r < rn;
          sB[r] = in ? S.sig[y0 + r][lane] : (M)0;
          vB[r] = in ? S.vis[y0 + r][lane] : (M)0;
          fB[r] = (in && ty == 1) ? S.ref[y0 + r][lane] : (M)0;
          gB[r] = in ? pl[y0 + r] : (M)0;
          nB[r] = (in && sgn) ? sg[y0 + r] : (M)0;
          aB[r] = 0;
        }
        // r is a compile-time constant in every caller (unrolled loops)
        auto code_sign = [&](int r, int x) {
          if (raw) {                                     // a raw pass sends the sign itself
            rawput(btu(nB[r], x));
            return;
          }
          const uint32_t sc = S.sct[sc_pat(f3(SR(r), x), f3(NR(r), x), (uint32_t)btu(SR(r - 1), x),
                                           (uint32_t)btu(NR(r - 1), x), (uint32_t)btu(SR(r + 1), x),
                                           (uint32_t)btu(NR(r + 1), x))];
          mq_enc(&S.ctx[CX_SC + (int)(sc & 7u)][lane], btu(nB[r], x) ^ (int)(sc >> 3));
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
              const M mid = sB[r];
              if (btu(mid, x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(mid, x), f3(SR(r + 1), x));
              if (!pat) continue;
              const int bit = btu(gB[r], x);
              if (raw) rawput(bit);
              else mq_enc(&S.ctx[zt[pat]][lane], bit);
              vB[r] |= (M)1 << x;
              if (bit) {
                code_sign(r, x);
                sB[r] = mid | ((M)1 << x);
                aB[r] |= (M)1 << x;
                grew = true;
              }
            }
            if (grew && x + 1 < w) c |= (M)1 << (x + 1);
          }
        } else if (ty == 1) {                            // magnitude refinement
          M nbm[4];
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const M v = SR(r - 1) | SR(r + 1);
            nbm[r] = (SR(r) << 1) | (SR(r) >> 1) | v | (v << 1) | (v >> 1);
          }
          M mk = 0;
#pragma unroll
          for (int r = 0; r < 4; r++) mk |= sB[r] & ~vB[r];
          while (mk) {
            const int x = ctzm(mk);
            mk &= mk - 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r >= rn || !btu(sB[r] & ~vB[r], x)) continue;
              if (raw) {
                rawput(btu(gB[r], x));
              } else {
                const int cx = btu(fB[r], x) ? CX_MR + 2 : (btu(nbm[r], x) ? CX_MR + 1 : CX_MR);
                mq_enc(&S.ctx[cx][lane], btu(gB[r], x));
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
            const int x = ctzm(u);
            u &= u - 1;
            int rstart = 0;
            if (rn == 4) {
              bool run = true;
#pragma unroll
              for (int r = 0; r < 4; r++)
                if (btu(sB[r] | vB[r], x)) run = false;
              if (run && ((sA | sB[0] | sB[1] | sB[2] | sB[3] | sC) & nb3<M>(x))) run = false;
              if (run) {
                int rr = -1;
#pragma unroll
                for (int r = 3; r >= 0; r--)
                  if (btu(gB[r], x)) rr = r;
                mq_enc(&S.ctx[CX_RL][lane], rr >= 0);
                if (rr < 0) continue;
                mq_enc(&S.ctx[CX_UNI][lane], (rr >> 1) & 1);
                mq_enc(&S.ctx[CX_UNI][lane], rr & 1);
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
              const int bit = btu(gB[r], x);
              mq_enc(&S.ctx[zt[pat]][lane], bit);
              if (bit) {
                code_sign(r, x);
                sB[r] |= (M)1 << x;
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
          if (r < rn) {
            S.sig[y0 + r][lane] = sB[r];
            S.vis[y0 + r][lane] = vB[r];
            if (ty == 1) S.ref[y0 + r][lane] = fB[r];
            if (ty == 0) S.aux[y0 + r][lane] |= aB[r];
          }
        // every later pass exceeds a length limit
        if (e.BP >= mq_stop || (byp && 32 * rwi + rnb > 8 * kBypRawMax)) stop = true;
      }
      if (ty == 2)
        for (int y = 0; y < h; y++) S.vis[y][lane] = 0;
      if (stop) break;
      kk++;
      // a raw pass's MQ part is the last MQ-coded pass's codeword
      if (!raw) { lrk = mq_flush_copy(e, &ltail); lbp = e.BP; }
      int rk = lrk;
      if (byp) {
        const int rbits = 32 * rwi + rnb, rby = (rbits + 7) >> 3;
        if (kk >= kBypFirst) rk = 2 + lrk + rby;
        if (lrk > kBypMqMax || rby > kBypRawMax) rk = kRInf;
        RB[kk] = rbits;
      }
      R[kk] = rk;
      BPk[kk] = lbp;
      TL[kk] = ltail;
    }
  }
  for (int j = kk + 1; j <= npass; j++) { R[j] = kRInf; BPk[j] = 0; TL[j] = 0; }
  if (byp && rnb && rwi < kRawCap / 4) rawp[rwi] = __builtin_bswap32(racc);   // the last, partial word
  for (int y = 0; y < k.h; y++) spo[y] = S.aux[y][lane];
}

// One lane per code-block.  Without `order`, lane i of workgroup g codes
// block g * LANES + i.  With it (persistent launch: a grid the chip keeps
// resident), each workgroup takes the next group of LANES entries of
// `order` from the counter *qctr (zero at launch) until none is left; the
// order puts blocks with more bit-planes first, so the longest blocks start
// early and a workgroup's lanes hold blocks of similar length.
template <typename M, int ROWS, int LANES, bool BYP>
__global__ __launch_bounds__(LANES) void k_t1_encode(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                     int nblk, int cbh, const M* __restrict__ planes,
                                                     const M* __restrict__ signs, const uint8_t* __restrict__ pbv,
                                                     uint8_t* __restrict__ cw, int32_t* __restrict__ Rt,
                                                     int32_t* __restrict__ bpt,
                                                     uint32_t* __restrict__ tailt, M* __restrict__ sppf,
                                                     const int* __restrict__ order, int* __restrict__ qctr,
                                                     int32_t* __restrict__ rbt) {
  __shared__ T1Shared<M, ROWS, LANES, true> S;
  const int lane = threadIdx.x;
  S.fill_tables(lane, LANES);
  __syncthreads();
  if (!order) {
    t1_enc_block<M, ROWS, LANES, BYP>(S, lane, blockIdx.x * LANES + lane, F, blk, nblk, cbh, planes, signs, pbv, cw,
                                      Rt, bpt, tailt, sppf, rbt);
    return;
  }
  const int ngroups = (nblk + LANES - 1) / LANES;
  for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(qctr, 1);
    g = __shfl(g, 0);   // one wavefront per workgroup (LANES <= 64)
    if (g >= ngroups) break;
    const int i = g * LANES + lane;
    if (i < nblk)
      t1_enc_block<M, ROWS, LANES, BYP>(S, lane, order[i], F, blk, nblk, cbh, planes, signs, pbv, cw, Rt, bpt,
                                        tailt, sppf, rbt);
  }
}

// Block orders of the persistent launches (order_by_key, common.h).
__global__ __launch_bounds__(kOrderThreads) void k_t1_order(const uint8_t* __restrict__ pb, int nblk, int* __restrict__ order,
                                                  int* __restrict__ qctr) {
  order_by_key(nblk, [&](int b) { const int P = pb[b]; return kQBits - (P < kQBits ? P : kQBits); }, nullptr, order,
               qctr);
}
// decoding: by the planes its kept passes reach, k_b / 3 (k_b <= 3 * 23 - 2)
__global__ __launch_bounds__(kOrderThreads) void k_t1_order_dec(const uint32_t* __restrict__ table, int nblk,
                                                      int* __restrict__ order, int* __restrict__ qctr) {
  order_by_key(nblk, [&](int b) {
    const int kp = (int)((table[b] >> 8) & 0xFFu) / 3;
    return kQBits - (kp < kQBits ? kp : kQBits);
  }, nullptr, order, qctr);
}

// ------------------------------------------------------------------------
// Closed-form base reconstruction for the kept passes (one wave per block).
// ------------------------------------------------------------------------
template <typename M>
__global__ __launch_bounds__(256) void k_virtual_decode(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                        int nblk, int cbh, const uint8_t* __restrict__ pbv,
                                                        const uint8_t* __restrict__ kbv, const M* __restrict__ sppf) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int b = blockIdx.x * 4 + wave;
  if (b >= nblk) return;
  Blk k = blk[b];
  if (!F[k.field].active) return;
  const float* coef = F[k.field].buf[BUF_COEF];
  float* yhat = F[k.field].buf[BUF_YHAT];
  const int nx = F[k.field].nx, e0 = F[k.field].e0;
  int P = pbv[b], kb = kbv[b];
  int sh = k.gain - e0, e = e0 - k.gain;
  for (int i = lane; i < k.w * k.h; i += 64) {
    int y = i / k.w, x = i - y * k.w;
    int idx = (k.y0 + y) * nx + k.x0 + x;
    float c = coef[idx];
    uint32_t q = quantq(c, sh);
    float v = 0.0f;
    if (q && kb) {
      int ps = 31 - __builtin_clz(q);
      int sp;                                   // pass index that makes it significant
      if (ps == P - 1) sp = 0;
      else sp = 3 * (P - 2 - ps) + (bt(sppf[(size_t)b * cbh + y], x) ? 1 : 3);
      if (sp < kb) {
        int pk = ps;
        while (pk > 0 && 3 * (P - 2 - (pk - 1)) + 2 < kb) pk--;
        uint32_t m = (q >> pk) << pk;
        v = dequant(m, pk, c < 0.0f, e);
      }
    }
    yhat[idx] = v;
  }
}

// ------------------------------------------------------------------------
// Distortion reductions of every coding pass (the ΔD the rate allocation
// needs), from the magnitudes in closed form: a sample with top bit ps
// becomes significant at plane ps — in the cleanup pass of the block's top
// plane (ps = P-1), else in the significance-propagation pass of plane ps if
// the encoder recorded it there (sppf), in its cleanup pass otherwise — and
// is refined in the refinement pass of every plane below ps.  Pass numbers
// (1-based): 1 for the top plane's cleanup; 3(P-2-p)+2, +3, +4 for plane
// p < P-1's three passes.  One workgroup per block (one or four
// wavefronts); per plane, each wavefront sums its samples' reductions and
// adds them to the block's per-pass totals in LDS; the table holds running
// sums D[k] (D[0] = 0).  Integer sums: the same values in any order.
// ------------------------------------------------------------------------
template <typename M, int TH>
__global__ __launch_bounds__(TH) void k_t1_dist(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                int nblk, int cbh, const uint8_t* __restrict__ pbv,
                                                const M* __restrict__ sppf, int64_t* __restrict__ Dt) {
  // samples per thread of the largest block (64 rows of 32 or 64 columns)
  constexpr int kPer = 64 * 8 * (int)sizeof(M) / TH;
  __shared__ unsigned long long acc[kPassStride];
  const int b = blockIdx.x;
  const Blk k = blk[b];
  if (!F[k.field].active) return;
  const int P = pbv[b], npass = P ? 3 * P - 2 : 0;
  const int t = threadIdx.x, lane = t & 63;
  for (int i = t; i < kPassStride; i += TH) acc[i] = 0;
  __syncthreads();
  if (P > 0) {
    const float* coef = F[k.field].buf[BUF_COEF];
    const int nx = F[k.field].nx, sh = k.gain - F[k.field].e0;
    const int n = k.w * k.h;
    uint32_t qv[kPer];
    uint32_t spb = 0;
    static_assert(kPer <= 32, "one sppf bit per sample of the thread");
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const int i = t + TH * j;
      qv[j] = 0;
      if (i < n) {
        const int y = i / k.w, x = i - y * k.w;
        qv[j] = quantq(coef[(size_t)(k.y0 + y) * nx + k.x0 + x], sh);
        spb |= (uint32_t)bt(sppf[(size_t)b * cbh + y], x) << j;
      }
    }
    for (int p = P - 1; p >= 0; p--) {
      int64_t dspp = 0, dcp = 0, dref = 0;
#pragma unroll
      for (int j = 0; j < kPer; j++) {
        const uint32_t q = qv[j];
        if (!q) continue;
        const int ps = 31 - __builtin_clz(q);
        if (ps == p) {
          const int64_t d = sig_delta(q, p);
          if (p < P - 1 && ((spb >> j) & 1u)) dspp += d;
          else dcp += d;
        } else if (ps > p) {
          dref += ref_delta(q, p);
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        dspp += __shfl_xor(dspp, o);
        dcp += __shfl_xor(dcp, o);
        dref += __shfl_xor(dref, o);
      }
      if (lane == 0) {
        if (p == P - 1) {
          atomicAdd(&acc[1], (unsigned long long)dcp);
        } else {
          const int k0 = 3 * (P - 2 - p) + 2;
          atomicAdd(&acc[k0], (unsigned long long)dspp);
          atomicAdd(&acc[k0 + 1], (unsigned long long)dref);
          atomicAdd(&acc[k0 + 2], (unsigned long long)dcp);
        }
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    int64_t* Dd = Dt + (size_t)b * kPassStride;
    int64_t c = 0;
    Dd[0] = 0;
    for (int j = 1; j <= npass; j++) {
      c += (int64_t)acc[j];
      Dd[j] = c;
    }
  }
}

void t1_distortion(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint8_t* pb,
                   const void* sppf, int64_t* D, hipStream_t st) {
  if (nblk <= 0) return;
  // few blocks (one field): four wavefronts per block shorten the launch;
  // many: one wavefront per block does the least work
  if (cbw > 32)
    k_t1_dist<uint64_t, 256><<<nblk, 256, 0, st>>>(F, blk, nblk, cbh, pb, (const uint64_t*)sppf, D);
  else if (nblk <= 8192)
    k_t1_dist<uint32_t, 256><<<nblk, 256, 0, st>>>(F, blk, nblk, cbh, pb, (const uint32_t*)sppf, D);
  else
    k_t1_dist<uint32_t, 64><<<nblk, 64, 0, st>>>(F, blk, nblk, cbh, pb, (const uint32_t*)sppf, D);
}

// ------------------------------------------------------------------------
// MQ decoder (bytes past the codeword read as 0xFF).
// ------------------------------------------------------------------------
// The byte at BP (cur) and the one after it (nxt) are held in registers; the
// load of the following byte is issued as soon as BP advances.
struct MQDec {
  uint32_t C, A, cur, nxt;
  int CT, BP, len;
  const uint8_t* buf;
};
__device__ __forceinline__ uint32_t mq_rd(const MQDec& d, int i) { return (i >= 0 && i < d.len) ? d.buf[i] : 0xFFu; }
__device__ __forceinline__ void mq_adv(MQDec& d) {
  d.BP++;
  d.cur = d.nxt;
  d.nxt = mq_rd(d, d.BP + 1);
}
__device__ __forceinline__ void mq_bytein(MQDec& d) {
  if (d.cur == 0xFF) {
    if (d.nxt > 0x8F) { d.C += 0xFF00; d.CT = 8; }
    else { mq_adv(d); d.C += d.cur << 9; d.CT = 7; }
  } else {
    mq_adv(d); d.C += d.cur << 8; d.CT = 8;
  }
}
__device__ __forceinline__ void mq_dinit(MQDec& d, const uint8_t* buf, int len) {
  d.buf = buf; d.len = len; d.BP = 0;
  d.cur = mq_rd(d, 0);
  d.nxt = mq_rd(d, 1);
  d.C = d.cur << 16;
  mq_bytein(d);
  d.C <<= 7; d.CT -= 7; d.A = 0x8000;
}
__device__ __forceinline__ void mq_renormd(MQDec& d) {
  do {
    if (d.CT == 0) mq_bytein(d);
    d.A <<= 1; d.C <<= 1; d.CT--;
  } while ((d.A & 0x8000) == 0);
}
__device__ __forceinline__ int mq_decode(MQDec& d, uint8_t* cs_ptr, const uint32_t* tab) {
  uint32_t cs = *cs_ptr;
  uint32_t ent = tab[cs & 0x7f];
  uint32_t qe = ent & 0xFFFF, mps = cs >> 7;
  uint32_t nm = (ent >> 16) & 0x3f, nl = (ent >> 22) & 0x3f, sw = ent >> 28;
  int D;
  d.A -= qe;
  if ((d.C >> 16) < qe) {
    if (d.A < qe) { D = (int)mps; cs = (mps << 7) | nm; }
    else { D = (int)(mps ^ 1u); uint32_t m = sw ? (mps ^ 1u) : mps; cs = (m << 7) | nl; }
    d.A = qe;
    *cs_ptr = (uint8_t)cs;
    mq_renormd(d);
  } else {
    d.C -= qe << 16;
    if ((d.A & 0x8000) == 0) {
      if (d.A < qe) { D = (int)(mps ^ 1u); uint32_t m = sw ? (mps ^ 1u) : mps; cs = (m << 7) | nl; }
      else { D = (int)mps; cs = (mps << 7) | nm; }
      *cs_ptr = (uint8_t)cs;
      mq_renormd(d);
    } else {
      D = (int)mps;
    }
  }
  return D;
}

// ------------------------------------------------------------------------
// Tier-1 decoder: one lane per code-block.  `table` holds the 4-byte block
// entries (P_b | k_b << 8 | len << 16), `off` the payload offsets within
// `sec` (the whole base section).  Writes the dequantised coefficients of
// every sample of the block into yhat; the magnitudes being decoded are kept
// in yhat's storage as integers until the block is finished.
// ------------------------------------------------------------------------
// BYP: the launch may hold streams with the arithmetic-coding bypass.
template <typename M, int ROWS, int LANES, bool BYP>
__device__ __forceinline__ void t1_dec_block(T1Shared<M, ROWS, LANES, false>& S, int lane, int b,
                                             const FieldDev* __restrict__ F, const Blk* __restrict__ blk, int nblk,
                                             const uint32_t* __restrict__ table, const int64_t* __restrict__ off) {
  if (b >= nblk) return;
  Blk k = blk[b];
  const FieldDev& f = F[k.field];
  if (!f.active) return;
  const uint8_t* sec = f.out + kHdr + 4 * (size_t)f.nblk;
  const int64_t sec_len = (int64_t)f.bb - 4 * (int64_t)f.nblk;
  const int nx = f.nx, e0 = f.e0;
  float* yhat = f.buf[BUF_YHAT];
  int* flag = &f.flags[1];
  uint32_t ent = table[b];
  int P = ent & 0xFF, kb = (ent >> 8) & 0xFF, len = (int)(ent >> 16);
  int64_t o = off[b];
  float* yb = yhat + (size_t)k.y0 * nx + k.x0;
  uint32_t* mb = reinterpret_cast<uint32_t*>(yb);
  bool bad = P > kQBits || kb > (P ? 3 * P - 2 : 0) || o < 0 || o + len > sec_len;
  // bypass codeword after more than ten passes: u16 raw byte count, the MQ
  // codeword, the raw bytes
  const bool rawcw = BYP && f.byp && kb >= kBypFirst;
  int rby = 0;
  if (rawcw && !bad) {
    if (len < 2) {
      bad = true;
    } else {
      rby = (int)sec[o] | ((int)sec[o + 1] << 8);
      if (2 + rby > len) bad = true;
    }
  }
  if (bad) atomicOr(flag, 1);
  if (bad || P == 0 || kb == 0) {
    for (int y = 0; y < k.h; y++)
      for (int x = 0; x < k.w; x++) yb[y * nx + x] = 0.0f;
    return;
  }
  const uint8_t* zt = ztab_of(S, k.orient);
  for (int y = 0; y < k.h; y++) {
    S.sig[y][lane] = 0; S.vis[y][lane] = 0; S.ref[y][lane] = 0; S.neg[y][lane] = 0;
  }
  for (int c = 0; c < kNCtx; c++) S.ctx[c][lane] = 0;
  S.ctx[0][lane] = 4; S.ctx[CX_RL][lane] = 3; S.ctx[CX_UNI][lane] = 46;
  MQDec d;
  mq_dinit(d, sec + o + (rawcw ? 2 : 0), rawcw ? len - 2 - rby : len);
  auto mq_dec = [&](uint8_t* cs) { return mq_decode(d, cs, S.mqt); };
  // raw bits, MSB-first, bits past the end read as 0; the current byte and
  // the next one are held in registers (the next load is issued a byte early)
  const uint8_t* const rbuf = sec + o + len - rby;
  int rpos = 0;
  uint32_t rcur = (BYP && rby > 0) ? rbuf[0] : 0u, rnxt = (BYP && rby > 1) ? rbuf[1] : 0u;
  auto rawget = [&]() -> int {
    const int bit = (int)((rcur >> (7 - (rpos & 7))) & 1u);
    if ((++rpos & 7) == 0) {
      const int i = (rpos >> 3) + 1;
      rcur = rnxt;
      rnxt = i < rby ? rbuf[i] : 0u;
    }
    return bit;
  };
  const int h = k.h, w = k.w;
  const M wm = (w >= MaskBits<M>::value) ? ~(M)0 : (((M)1 << w) - 1);
  auto rowm = [&](M (*a)[LANES], int y) -> M { return (y >= 0 && y < h) ? a[y][lane] : (M)0; };
  // The magnitudes being decoded live in yhat's storage (as integers) until
  // the block is finished.  Their bits are set with atomic ORs, which need
  // no read back and so never wait.  Every access to that storage (the
  // zeroing, the ORs, the final reads) is atomic, so they are ordered per
  // location without fences.
  for (int y = 0; y < h; y++)
    for (int x = 0; x < w; x++) __hip_atomic_store(&mb[y * nx + x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  auto setbit = [&](int y, int x, int p) {
    (void)__hip_atomic_fetch_or(&mb[y * nx + x], 1u << p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // The samples whose bit of the last decoded plane is known: after its
  // significance-propagation pass, those that pass made significant (the
  // significant samples it visited); after its refinement or cleanup pass,
  // every significant sample (refinement codes the bit of each sample
  // significant before the plane).
  int done = 0, plast = P - 1, lastty = 2;
  for (int p = P - 1; p >= 0 && done < kb; p--) {
    plast = p;
    for (int ty = (p == P - 1) ? 2 : 0; ty < 3 && done < kb; ty++) {
      // pass numbers 11 and later of planes p <= P - 5 (SPP, MRP) are raw
      const bool raw = rawcw && ty < 2 && p <= P - 5;
      for (int y0 = 0; y0 < h; y0 += 4) {
        const int rn = h - y0 < 4 ? h - y0 : 4;
        const M sA = rowm(S.sig, y0 - 1), sC = rowm(S.sig, y0 + 4);
        const M nA = rowm(S.neg, y0 - 1), nC = rowm(S.neg, y0 + 4);
        M sB[4], vB[4], fB[4], nB[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const bool in = r < rn;
          sB[r] = in ? S.sig[y0 + r][lane] : (M)0;
          vB[r] = in ? S.vis[y0 + r][lane] : (M)0;
          fB[r] = (in && ty == 1) ? S.ref[y0 + r][lane] : (M)0;
          nB[r] = in ? S.neg[y0 + r][lane] : (M)0;
        }
        // r is a compile-time constant in every caller (unrolled loops)
        auto dec_sign = [&](int r, int x) {
          if (raw) {                                     // a raw pass sends the sign itself
            if (rawget()) nB[r] |= (M)1 << x;
            return;
          }
          const uint32_t sc = S.sct[sc_pat(f3(SR(r), x), f3(NR(r), x), (uint32_t)btu(SR(r - 1), x),
                                           (uint32_t)btu(NR(r - 1), x), (uint32_t)btu(SR(r + 1), x),
                                           (uint32_t)btu(NR(r + 1), x))];
          if (mq_dec(&S.ctx[CX_SC + (int)(sc & 7u)][lane]) ^ (int)(sc >> 3)) nB[r] |= (M)1 << x;
        };
        if (ty == 0) {                                   // significance propagation
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
              const M mid = sB[r];
              if (btu(mid, x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(mid, x), f3(SR(r + 1), x));
              if (!pat) continue;
              const int bit = raw ? rawget() : mq_dec(&S.ctx[zt[pat]][lane]);
              vB[r] |= (M)1 << x;
              if (bit) {
                dec_sign(r, x);
                sB[r] = mid | ((M)1 << x);
                setbit(y0 + r, x, p);
                grew = true;
              }
            }
            if (grew && x + 1 < w) c |= (M)1 << (x + 1);
          }
        } else if (ty == 1) {                            // magnitude refinement
          M nbm[4];
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const M v = SR(r - 1) | SR(r + 1);
            nbm[r] = (SR(r) << 1) | (SR(r) >> 1) | v | (v << 1) | (v >> 1);
          }
          M mk = 0;
#pragma unroll
          for (int r = 0; r < 4; r++) mk |= sB[r] & ~vB[r];
          while (mk) {
            const int x = ctzm(mk);
            mk &= mk - 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r >= rn || !btu(sB[r] & ~vB[r], x)) continue;
              const int cx = btu(fB[r], x) ? CX_MR + 2 : (btu(nbm[r], x) ? CX_MR + 1 : CX_MR);
              if (raw ? rawget() : mq_dec(&S.ctx[cx][lane])) setbit(y0 + r, x, p);
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
            const int x = ctzm(u);
            u &= u - 1;
            int rstart = 0;
            if (rn == 4) {
              bool run = true;
#pragma unroll
              for (int r = 0; r < 4; r++)
                if (btu(sB[r] | vB[r], x)) run = false;
              if (run && ((sA | sB[0] | sB[1] | sB[2] | sB[3] | sC) & nb3<M>(x))) run = false;
              if (run) {
                if (!mq_dec(&S.ctx[CX_RL][lane])) continue;
                const int b1 = mq_dec(&S.ctx[CX_UNI][lane]);
                const int b0 = mq_dec(&S.ctx[CX_UNI][lane]);
                const int rr = 2 * b1 + b0;
#pragma unroll
                for (int r = 0; r < 4; r++)
                  if (r == rr) {
                    dec_sign(r, x);
                    sB[r] |= (M)1 << x;
                    setbit(y0 + r, x, p);
                  }
                rstart = rr + 1;
              }
            }
#pragma unroll
            for (int r = 0; r < 4; r++) {
              if (r < rstart || r >= rn) continue;
              if (btu(sB[r] | vB[r], x)) continue;
              const uint32_t pat = zc_pat(f3(SR(r - 1), x), f3(sB[r], x), f3(SR(r + 1), x));
              if (mq_dec(&S.ctx[zt[pat]][lane])) {
                dec_sign(r, x);
                sB[r] |= (M)1 << x;
                setbit(y0 + r, x, p);
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
          if (r < rn) {
            S.sig[y0 + r][lane] = sB[r];
            S.vis[y0 + r][lane] = vB[r];
            if (ty == 1) S.ref[y0 + r][lane] = fB[r];
            else S.neg[y0 + r][lane] = nB[r];
          }
      }
      if (ty == 2)
        for (int y = 0; y < h; y++) S.vis[y][lane] = 0;
      done++;
      lastty = ty;
    }
  }
  const int e = e0 - k.gain;
  for (int y = 0; y < h; y++) {
    const M sg = S.sig[y][lane], ng = S.neg[y][lane];
    const M cur = lastty == 0 ? (sg & S.vis[y][lane]) : sg;
    for (int x = 0; x < w; x++) {
      float v = 0.0f;
      if (bt(sg, x)) {
        int pk = bt(cur, x) ? plast : plast + 1;
        v = dequant(__hip_atomic_load(&mb[y * nx + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), pk, bt(ng, x), e);
      }
      yb[y * nx + x] = v;
    }
  }
}

// One lane per code-block; with `order`, a persistent launch as for the
// encoder (blocks ordered by coding passes kept, most first).
template <typename M, int ROWS, int LANES, bool BYP>
__global__ __launch_bounds__(LANES) void k_t1_decode(const FieldDev* __restrict__ F, const Blk* __restrict__ blk,
                                                     int nblk, const uint32_t* __restrict__ table,
                                                     const int64_t* __restrict__ off, const int* __restrict__ order,
                                                     int* __restrict__ qctr) {
  __shared__ T1Shared<M, ROWS, LANES, false> S;
  const int lane = threadIdx.x;
  S.fill_tables(lane, LANES);
  __syncthreads();
  if (!order) {
    t1_dec_block<M, ROWS, LANES, BYP>(S, lane, blockIdx.x * LANES + lane, F, blk, nblk, table, off);
    return;
  }
  const int ngroups = (nblk + LANES - 1) / LANES;
  for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(qctr, 1);
    g = __shfl(g, 0);   // one wavefront per workgroup (LANES <= 64)
    if (g >= ngroups) break;
    const int i = g * LANES + lane;
    if (i < nblk) t1_dec_block<M, ROWS, LANES, BYP>(S, lane, order[i], F, blk, nblk, table, off);
  }
}

#undef SR
#undef NR

// ------------------------------------------------------------------------
// Launchers: mask width follows the code-block width, LDS rows its height,
// and the blocks per wavefront (lanes) the amount of work: a lone field's
// blocks are spread one per wavefront (no divergence, the whole chip busy),
// large batches pack up to 64 blocks per wavefront for throughput.
// ------------------------------------------------------------------------
static int pick_lanes(int items, int lanes_max) {
  const int forced = tuning().t1_lanes;
  if (forced > 0) return forced > lanes_max ? lanes_max : forced;
  const int resident = 8192;   // wavefronts the chip keeps in flight comfortably
  int l = 1;
  while (l < lanes_max && items / l > resident) l *= 4;
  return l > lanes_max ? lanes_max : l;
}
template <typename M, int ROWS>
constexpr int t1_lanes_max() {
  return (6 * ROWS * (int)sizeof(M) * 64 <= 49152) ? 64 : (6 * ROWS * (int)sizeof(M) * 16 <= 49152 ? 16 : 4);
}

#define T1_DISPATCH(CBW, CBH, MACRO)                               \
  do {                                                             \
    if ((CBW) <= 32) {                                             \
      if ((CBH) <= 16) MACRO(uint32_t, 16);                        \
      else if ((CBH) <= 32) MACRO(uint32_t, 32);                   \
      else MACRO(uint32_t, 64);                                    \
    } else {                                                       \
      if ((CBH) <= 16) MACRO(uint64_t, 16);                        \
      else if ((CBH) <= 32) MACRO(uint64_t, 32);                   \
      else MACRO(uint64_t, 64);                                    \
    }                                                              \
  } while (0)

// Workgroups of `threads` threads the device keeps resident at once.
template <typename K>
static int resident_groups(K kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
  return (cus > 0 ? cus : 1) * (per > 0 ? per : 1);
}

// order/qctr non-null: persistent launch (order filled by k_t1_order first).
template <typename M, int ROWS, bool BYP>
static void launch_encode(int nblk, const FieldDev* F, const Blk* blk, int cbh, const void* planes, const void* signs,
                          const uint8_t* pb, uint8_t* cw, int32_t* R, int32_t* bp, uint32_t* tail,
                          void* sppf, hipStream_t st, int* order, int* qctr, int32_t* rbt) {
  constexpr int LM = t1_lanes_max<M, ROWS>();
  int ln = pick_lanes(nblk, LM);
  if (order) k_t1_order<<<1, kOrderThreads, 0, st>>>(pb, nblk, order, qctr);
#define ENC_L(LN)                                                                                                  \
  do {                                                                                                             \
    const int groups = (nblk + LN - 1) / LN;                                                                       \
    const int grid = order ? std::min(groups, resident_groups(k_t1_encode<M, ROWS, LN, BYP>, LN)) : groups;        \
    k_t1_encode<M, ROWS, LN, BYP><<<grid, LN, 0, st>>>(F, blk, nblk, cbh, (const M*)planes, (const M*)signs, pb,    \
                                                       cw, R, bp, tail, (M*)sppf, order, qctr, rbt);                \
  } while (0)
  if (ln == 1) ENC_L(1);
  else if (ln == 4) ENC_L(4);
  else if (ln == 16 || LM == 16) ENC_L((LM >= 16 ? 16 : 4));
  else ENC_L((LM >= 64 ? 64 : 4));
#undef ENC_L
}

template <typename M, int ROWS, bool BYP>
static void launch_decode(int nblk, const FieldDev* F, const Blk* blk, const uint32_t* table, const int64_t* off,
                          hipStream_t st, int* order, int* qctr) {
  constexpr int LM = t1_lanes_max<M, ROWS>();
  int ln = pick_lanes(nblk, LM);
  if (order) k_t1_order_dec<<<1, kOrderThreads, 0, st>>>(table, nblk, order, qctr);
#define DEC_L(LN)                                                                                                  \
  do {                                                                                                             \
    const int groups = (nblk + LN - 1) / LN;                                                                       \
    const int grid = order ? std::min(groups, resident_groups(k_t1_decode<M, ROWS, LN, BYP>, LN)) : groups;        \
    k_t1_decode<M, ROWS, LN, BYP><<<grid, LN, 0, st>>>(F, blk, nblk, table, off, order, qctr);                     \
  } while (0)
  if (ln == 1) DEC_L(1);
  else if (ln == 4) DEC_L(4);
  else if (ln == 16 || LM == 16) DEC_L((LM >= 16 ? 16 : 4));
  else DEC_L((LM >= 64 ? 64 : 4));
#undef DEC_L
}

void quant_planes(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, void* planes, void* signs,
                  uint8_t* pb, hipStream_t st) {
  if (nblk <= 0) return;
  int g = (nblk + 3) / 4;
  if (cbw <= 32)
    k_quant_planes<uint32_t><<<g, 256, 0, st>>>(F, blk, nblk, cbw, cbh, (uint32_t*)planes, (uint32_t*)signs, pb);
  else
    k_quant_planes<uint64_t><<<g, 256, 0, st>>>(F, blk, nblk, cbw, cbh, (uint64_t*)planes, (uint64_t*)signs, pb);
}

// By work size: a wave per block up to Tuning::t1_wave_max blocks in the
// launch (latency: one field's blocks spread over the whole chip), lanes per
// block beyond (throughput: the 256-field batch encodes 1.5x and decodes
// 1.2x faster that way).
static bool use_wave(int nblk, bool decode) {
  const char* e = getenv("EBCC_T1_KERNEL");
  if (e && e[0] == 'w') return true;
  if (e && e[0] == 'l') return false;
  Tuning t = tuning();
  int v = decode ? t.t1_decoder : t.t1_encoder;
  return v == 1 || (v == 0 && nblk <= t.t1_wave_max);
}

// Lanes-per-block launches can hand the first t1_split percent of their
// blocks to the wave-per-block kernel on a second stream: that kernel runs on
// the scalar unit, the lanes kernel on the vector unit, so the two overlap.
static int split_count(int nblk, const T1Split* sp) {
  if (!sp || !sp->aux) return 0;
  const int pct = tuning().t1_split;
  return pct <= 0 ? 0 : (int)((int64_t)nblk * (pct > 100 ? 100 : pct) / 100);
}

// Persistent lanes-per-block launches (block order by bit-planes, work
// counter): tuning t1_persist, or EBCC_T1_PERSIST=0/1.
static bool use_persist() {
  const char* e = getenv("EBCC_T1_PERSIST");
  if (e && e[0]) return e[0] == '1';
  return tuning().t1_persist != 0;
}

void t1_encode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const void* planes, const void* signs,
               const uint8_t* pb, uint8_t* cw, int32_t* R, int64_t* D, int32_t* bp, uint32_t* tail, void* sppf,
               hipStream_t st, const T1Split* sp, int* order, int* qctr, int32_t* rbt) {
  if (nblk <= 0) return;
  if (use_wave(nblk, false)) {
    t1_encode_wave(F, blk, nblk, cbw, cbh, planes, signs, pb, cw, R, bp, tail, sppf, st, rbt);
    t1_distortion(F, blk, nblk, cbw, cbh, pb, sppf, D, st);
    return;
  }
  if (!(order && qctr && use_persist())) order = nullptr, qctr = nullptr;
  const Blk* const blk0 = blk;
  const uint8_t* const pb0 = pb;
  void* const sppf0 = sppf;
  const int nblk0 = nblk;
  const int s = order ? 0 : split_count(nblk, sp);
  if (s > 0) {
    (void)hipEventRecord(sp->ev_fork, st);
    (void)hipStreamWaitEvent(sp->aux, sp->ev_fork, 0);
    t1_encode_wave(F, blk, s, cbw, cbh, planes, signs, pb, cw, R, bp, tail, sppf, sp->aux, rbt);
    const size_t ms = cbw <= 32 ? 4 : 8;
    blk += s; pb += s; cw += (size_t)s * kCwCap;
    planes = (const char*)planes + (size_t)s * kQBits * cbh * ms;
    signs = (const char*)signs + (size_t)s * cbh * ms;
    sppf = (char*)sppf + (size_t)s * cbh * ms;
    R += (size_t)s * kPassStride;
    bp += (size_t)s * kPassStride; tail += (size_t)s * kPassStride;
    if (rbt) rbt += (size_t)s * kPassStride;
    nblk -= s;
  }
#define ENC(MT, RW)                                                                                        \
  do {                                                                                                     \
    if (rbt) launch_encode<MT, RW, true>(nblk, F, blk, cbh, planes, signs, pb, cw, R, bp, tail, sppf, st,    \
                                         order, qctr, rbt);                                                \
    else launch_encode<MT, RW, false>(nblk, F, blk, cbh, planes, signs, pb, cw, R, bp, tail, sppf, st,       \
                                      order, qctr, nullptr);                                               \
  } while (0)
  T1_DISPATCH(cbw, cbh, ENC);
#undef ENC
  if (s > 0) {
    (void)hipEventRecord(sp->ev_join, sp->aux);
    (void)hipStreamWaitEvent(st, sp->ev_join, 0);
  }
  t1_distortion(F, blk0, nblk0, cbw, cbh, pb0, sppf0, D, st);
}

void virtual_decode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint8_t* pb,
                    const uint8_t* kb, const void* sppf, hipStream_t st) {
  if (nblk <= 0) return;
  int g = (nblk + 3) / 4;
  if (cbw <= 32)
    k_virtual_decode<uint32_t><<<g, 256, 0, st>>>(F, blk, nblk, cbh, pb, kb, (const uint32_t*)sppf);
  else
    k_virtual_decode<uint64_t><<<g, 256, 0, st>>>(F, blk, nblk, cbh, pb, kb, (const uint64_t*)sppf);
}

void t1_decode(const FieldDev* F, const Blk* blk, int nblk, int cbw, int cbh, const uint32_t* table,
               const int64_t* off, hipStream_t st, const T1Split* sp, int* order, int* qctr, bool byp) {
  if (nblk <= 0) return;
  if (use_wave(nblk, true)) {
    t1_decode_wave(F, blk, nblk, cbw, table, off, st, byp);
    return;
  }
  if (!(order && qctr && use_persist())) order = nullptr, qctr = nullptr;
  const int s = order ? 0 : split_count(nblk, sp);
  if (s > 0) {
    (void)hipEventRecord(sp->ev_fork, st);
    (void)hipStreamWaitEvent(sp->aux, sp->ev_fork, 0);
    t1_decode_wave(F, blk, s, cbw, table, off, sp->aux, byp);
    blk += s; table += s; off += s; nblk -= s;
  }
#define DEC(MT, RW)                                                               \
  do {                                                                            \
    if (byp) launch_decode<MT, RW, true>(nblk, F, blk, table, off, st, order, qctr);  \
    else launch_decode<MT, RW, false>(nblk, F, blk, table, off, st, order, qctr);     \
  } while (0)
  T1_DISPATCH(cbw, cbh, DEC);
#undef DEC
  if (s > 0) {
    (void)hipEventRecord(sp->ev_join, sp->aux);
    (void)hipStreamWaitEvent(st, sp->ev_join, 0);
  }
}

}  // namespace ebcc
