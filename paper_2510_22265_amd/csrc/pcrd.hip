// Rate allocation of the base layer: post-compression rate-distortion
// optimisation (PCRD, Taubman 2000) meeting the base compression ratio r of
// the paper's enc_base(A, r, eps) (Algorithm 1).
//
//  1. one thread per code-block (64-thread workgroups over all the fields'
//     blocks) builds the upper convex hull of its (R_k, D_k) pass points
//     (strictly decreasing slopes; passes that do not add distortion
//     reduction or whose length exceeds 65535 are skipped); the block's pass
//     table is first copied to LDS with its loads issued together, so the
//     hull walk reads LDS, not a chain of dependent global loads;
// then one workgroup per field:
//  2. the segments are ordered by the composite key (slope descending,
//     block ascending, segment ascending); segments are accepted in that
//     order until the first one that would overflow the byte budget.  The
//     first non-fitting segment is found by a radix select over the 104-bit
//     key (8-bit digits, LDS histograms of segment lengths), so no sort is
//     materialised; after two digits the few segments still in play move
//     to LDS;
//  3. one thread per block keeps the segments whose key is above the
//     threshold and writes k_b and the codeword length R_{k_b}.
#include "common.h"

namespace ebcc {

constexpr int kPcrdThreads = 1024;
constexpr int kPcrdCand = 2048;    // LDS candidates after the first two digits

__device__ __forceinline__ double seg_slope(int64_t dD, int64_t dR) {
  return dR <= 0 ? __longlong_as_double(0x7ff0000000000000ll) : (double)dD / (double)dR;
}

typedef unsigned __int128 u128;

__device__ __forceinline__ u128 seg_key(uint64_t slope_bits, int b, int j) {
  return ((u128)slope_bits << 40) | ((u128)(0xFFFFFFFFu - (uint32_t)b) << 8) | (u128)(0xFFu - (uint32_t)j);
}

constexpr int kHullThreads = 64;

__global__ __launch_bounds__(kHullThreads) void k_pcrd_hull(const FieldDev* __restrict__ F,
                                                            const uint8_t* __restrict__ pb_g,
                                                            const int32_t* __restrict__ R_g,
                                                            const int64_t* __restrict__ D_g, uint8_t* __restrict__ hk_g,
                                                            uint64_t* __restrict__ keys_g, int32_t* __restrict__ dr_g,
                                                            uint8_t* __restrict__ nhv_g) {
  __shared__ int64_t sd[kHullThreads][kPassStride];
  __shared__ int32_t sr[kHullThreads][kPassStride];
  __shared__ uint8_t sh[kHullThreads][kPassStride];
  const FieldDev& f = F[blockIdx.y];
  if (!f.active) return;
  const int b = blockIdx.x * kHullThreads + (int)threadIdx.x;
  if (b >= f.nblk) return;   // no barrier below
  const size_t gb = (size_t)f.blk0 + (size_t)b;
  const int P = pb_g[gb];
  const int n = P ? 3 * P - 2 : 0;
  const int32_t* r = R_g + gb * kPassStride;
  const int64_t* d = D_g + gb * kPassStride;
  int32_t* lr = sr[threadIdx.x];
  int64_t* ld = sd[threadIdx.x];
  uint8_t* h = sh[threadIdx.x];
  for (int k0 = 0; k0 <= n; k0 += 8) {
    int32_t rv[8];
    int64_t dv[8];
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (k0 + u <= n) { rv[u] = r[k0 + u]; dv[u] = d[k0 + u]; }
#pragma unroll
    for (int u = 0; u < 8; u++)
      if (k0 + u <= n) { lr[k0 + u] = rv[u]; ld[k0 + u] = dv[u]; }
  }
  int nh = 0;
  h[nh++] = 0;
  for (int k = 1; k <= n; k++) {
    const int32_t rk = lr[k];
    if (rk > kSegRMax) continue;
    const int64_t dk = ld[k];
    if (dk <= ld[h[nh - 1]]) continue;
    while (nh >= 2) {
      const int a = h[nh - 2], c = h[nh - 1];
      const double sac = seg_slope(ld[c] - ld[a], (int64_t)lr[c] - lr[a]);
      const double sck = seg_slope(dk - ld[c], (int64_t)rk - lr[c]);
      if (sck >= sac) nh--; else break;
    }
    h[nh++] = (uint8_t)k;
  }
  nhv_g[gb] = (uint8_t)nh;
  uint8_t* hk = hk_g + gb * kPassStride;
  uint64_t* keys = keys_g + gb * kPassStride;
  int32_t* dr = dr_g + gb * kPassStride;
  hk[0] = 0;
  for (int j = 1; j < nh; j++) {
    const int a = h[j - 1], c = h[j];
    hk[j] = (uint8_t)c;
    keys[j] = (uint64_t)__double_as_longlong(seg_slope(ld[c] - ld[a], (int64_t)lr[c] - lr[a]));
    dr[j] = lr[c] - lr[a];
  }
}

__global__ __launch_bounds__(kPcrdThreads) void k_pcrd(const FieldDev* __restrict__ F,
                                                       const int32_t* __restrict__ R_g, uint8_t* __restrict__ kb_g, uint8_t* __restrict__ hk_g,
                                                       uint64_t* __restrict__ keys_g, int32_t* __restrict__ dr_g,
                                                       uint8_t* __restrict__ nhv_g, int32_t* __restrict__ len_g) {
  __shared__ unsigned long long hist[256];
  __shared__ uint64_t c_hi[kPcrdCand], c_lo[kPcrdCand];
  __shared__ uint32_t c_dr[kPcrdCand];
  __shared__ int s_cnt;
  __shared__ int s_choice;
  __shared__ int s_allfit;
  __shared__ unsigned long long s_acc;
  const FieldDev& f = F[blockIdx.x];
  if (!f.active) return;
  // this field's blocks: [blk0, blk0 + nblk) of the call's block arrays
  const size_t b0 = (size_t)f.blk0;
  const int nblk = f.nblk;
  const int64_t budget = f.budget < 0 ? 0 : f.budget;
  const int32_t* R = R_g + b0 * kPassStride;
  uint8_t* kb = kb_g + b0;
  uint8_t* hk = hk_g + b0 * kPassStride;
  uint64_t* keys = keys_g + b0 * kPassStride;
  int32_t* dr = dr_g + b0 * kPassStride;
  uint8_t* nhv = nhv_g + b0;
  int32_t* len_out = len_g + b0;
  int tid = threadIdx.x;
  // 2. radix select of the first segment that does not fit.  The first two
  // digits scan every segment in global memory; the segments that still
  // match the selected prefix are then copied to LDS (when they fit) and the
  // remaining digits scan only those.
  u128 prefix = 0;
  unsigned long long acc = 0;
  bool allfit = false;
  int ncand = -1;   // LDS candidate count (-1: not compacted)
  for (int dgt = 0; dgt < 13; dgt++) {
    for (int i = tid; i < 256; i += kPcrdThreads) hist[i] = 0;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    int sh = 104 - 8 * (dgt + 1);
    if (ncand < 0) {
      for (int b = tid; b < nblk; b += kPcrdThreads) {
        const int nh = nhv[b];
        const uint64_t* kp = keys + (size_t)b * kPassStride;
        const int32_t* dp = dr + (size_t)b * kPassStride;
        for (int j0 = 1; j0 < nh; j0 += 4) {
          uint64_t kk[4];
          int32_t dd[4];
#pragma unroll
          for (int u = 0; u < 4; u++)   // independent loads first
            if (j0 + u < nh) { kk[u] = kp[j0 + u]; dd[u] = dp[j0 + u]; }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int j = j0 + u;
            if (j >= nh) break;
            u128 key = seg_key(kk[u], b, j);
            if (dgt > 0 && (key >> (sh + 8)) != prefix) continue;
            int dg = (int)((key >> sh) & 0xFF);
            atomicAdd(&hist[dg], (unsigned long long)dd[u]);
          }
        }
      }
    } else {
      for (int q = tid; q < ncand; q += kPcrdThreads) {
        u128 key = ((u128)c_hi[q] << 40) | (u128)c_lo[q];
        if (dgt > 0 && (key >> (sh + 8)) != prefix) continue;
        int dg = (int)((key >> sh) & 0xFF);
        atomicAdd(&hist[dg], (unsigned long long)c_dr[q]);
      }
    }
    __syncthreads();
    if (tid < 64) {
      // digits from 255 down: the first whose segments would overflow the
      // budget after all higher digits are accepted.  Lane q holds digits
      // 255 - 4q .. 252 - 4q; a wave prefix sum gives each lane the total
      // of the digits above its own.
      unsigned long long v[4], sum = 0;
#pragma unroll
      for (int i = 0; i < 4; i++) { v[i] = hist[255 - 4 * tid - i]; sum += v[i]; }
      unsigned long long inc = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(inc, o);
        if (tid >= o) inc += t;
      }
      unsigned long long a = acc + (inc - sum);   // accepted before this lane's digits
      int hit = -1;
      unsigned long long ahit = 0;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        if (hit < 0 && a + v[i] > (unsigned long long)budget) { hit = i; ahit = a; }
        a += v[i];
      }
      const unsigned long long m = __ballot(hit >= 0);
      const int first = m ? __builtin_ctzll(m) : -1;
      if (first < 0) {
        if (tid == 63) { s_choice = -1; s_acc = a; s_allfit = 1; }
      } else if (tid == first) {
        s_choice = 255 - 4 * tid - hit;
        s_acc = ahit;
        s_allfit = 0;
      }
    }
    __syncthreads();
    if (s_allfit) { allfit = true; break; }
    prefix = (prefix << 8) | (u128)s_choice;
    acc = s_acc;
    if (dgt == 1 && ncand < 0) {
      // compact the segments that match the 16-bit prefix into LDS
      for (int b = tid; b < nblk; b += kPcrdThreads) {
        const int nh = nhv[b];
        const uint64_t* kp = keys + (size_t)b * kPassStride;
        const int32_t* dp = dr + (size_t)b * kPassStride;
        for (int j0 = 1; j0 < nh; j0 += 4) {
          uint64_t kk[4];
          int32_t dd[4];
#pragma unroll
          for (int u = 0; u < 4; u++)
            if (j0 + u < nh) { kk[u] = kp[j0 + u]; dd[u] = dp[j0 + u]; }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int j = j0 + u;
            if (j >= nh) break;
            u128 key = seg_key(kk[u], b, j);
            if ((key >> sh) != prefix) continue;
            int q = atomicAdd(&s_cnt, 1);
            if (q < kPcrdCand) {
              c_hi[q] = (uint64_t)(key >> 40);
              c_lo[q] = (uint64_t)(key & (((u128)1 << 40) - 1));
              c_dr[q] = (uint32_t)dd[u];
            }
          }
        }
      }
      __syncthreads();
      if (s_cnt <= kPcrdCand) ncand = s_cnt;
    }
    __syncthreads();
  }
  // 3. kept passes per block: every segment with key above the threshold;
  // the accepted payload and whether every segment fitted go to the field
  unsigned long long used = 0;
  for (int b = tid; b < nblk; b += kPcrdThreads) {
    int nh = nhv[b];
    int k = 0;
    for (int j = 1; j < nh; j++) {
      u128 key = seg_key(keys[(size_t)b * kPassStride + j], b, j);
      if (allfit || key > prefix) k = hk[(size_t)b * kPassStride + j];
      else break;
    }
    kb[b] = (uint8_t)k;
    len_out[b] = k ? R[(size_t)b * kPassStride + k] : 0;
    used += (unsigned long long)len_out[b];
  }
  for (int o = 32; o > 0; o >>= 1) used += __shfl_xor(used, o);
  if ((tid & 63) == 0) hist[tid >> 6] = used;      // the histogram is free again
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kPcrdThreads / 64; w++) t += hist[w];
    f.totals[2] = (int64_t)t;
    f.flags[2] = allfit ? 1 : 0;
  }
}

void pcrd(const FieldDev* F, int nf, int max_nblk, const uint8_t* pb, const int32_t* R, const int64_t* D, uint8_t* kb,
          uint8_t* hk_scratch, uint64_t* key_scratch, int32_t* dr_scratch, uint8_t* nh_scratch, int32_t* len_out,
          hipStream_t st) {
  if (nf <= 0) return;
  if (max_nblk > 0)
    k_pcrd_hull<<<dim3((unsigned)((max_nblk + kHullThreads - 1) / kHullThreads), (unsigned)nf), kHullThreads, 0, st>>>(
        F, pb, R, D, hk_scratch, key_scratch, dr_scratch, nh_scratch);
  k_pcrd<<<nf, kPcrdThreads, 0, st>>>(F, R, kb, hk_scratch, key_scratch, dr_scratch, nh_scratch, len_out);
}

}  // namespace ebcc
