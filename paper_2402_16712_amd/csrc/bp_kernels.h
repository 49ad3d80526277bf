// bp_kernels.h -- Algorithm 2 (Sec. 2): the breakpoints of every segment's
// solution path v_k(lambda) and the lambda_max beyond which v_k = 0.
//
// For the segment (j, k) with the points sorted by (ratio, row), exact prefix
// weights S_p, W = S_n', A the weight of the negative ratios and B = A + the
// weight of the zero ratios:
//   * 0 minimises at lambda = 0 (2A <= W <= 2B): one entry (0, 0, row -1);
//   * negative side (2A > W): from the lambda = 0 minimiser p0 up to the last
//     negative point, the entry of point p is (max(0, 2 S_{p-1} - W), r_p, i_p),
//     then the terminal entry (2A - W, 0, -1);
//   * positive side (W > 2B): from p0 down to the first positive point, the
//     entry of p is (max(0, W - 2 S_p), r_p, i_p), then (W - 2B, 0, -1).
// This is the paper's loop (lambda_p = sgn(r_p)(weight after p - weight
// before p) - w_p, kept where lambda_p + 2 w_p > 0) with the zero ratios left
// out, listed in increasing lambda.  Each lambda is exact in 128-bit fixed
// point and rounded once to the nearest double.  The lambda = 0 minimiser
// (v, row) comes from the segment kernel run at lambda = 0.
//
// Two kernels, one wave per segment: k_bp_count (entries per segment and
// lambda_max), then, after the host scans the counts into offsets,
// k_bp_emit (the entries).  Column j is read from global memory (it stays in
// L2 across the segments of one j); the entries of a window of keys are
// sorted in the wave's LDS list, windows too large for it are halved in key
// space, and a single key with more tied rows than the list holds is
// streamed in row order (its rows are already in sorted order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fit_kernels.h"

// The double nearest to x * 2^e0 (ties to even); x < 2^127, e0 >= -1074.
__device__ __forceinline__ double fixed_to_double(u128 x, int e0) {
  if (x == 0) return 0.0;
  const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  const int h = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);   // top bit
  // bits kept: 53 in the normal range, fewer where the result is subnormal
  int keep = 53;
  if (e0 + h < -1022) keep = 53 - (-1022 - (e0 + h));
  const int shift = h + 1 - keep;                  // bits rounded away
  if (shift <= 0) return ldexp((double)lo, e0);    // exact (x < 2^53)
  // e0 >= -1074 keeps keep >= 1: the result is at least the smallest subnormal
  u128 q = x >> shift;
  const u128 rem = x & (((u128)1 << shift) - 1), half = (u128)1 << (shift - 1);
  if (rem > half || (rem == half && (q & 1))) q += 1;
  return ldexp((double)(uint64_t)q, e0 + shift);
}

// Segments (j, k) in tiles of ts x ts dealt to the 8 XCDs round robin (the
// dispatcher places workgroups on XCDs round robin by blockIdx), so the 2 ts
// columns a tile reads stay in one XCD's L2 while its waves work through the
// tile.  Slot f of an XCD's sequence is tile x + 8 (f / ts^2), segment
// f mod ts^2 of it.  Every tile belongs to the workgroups with blockIdx = its
// index mod 8, so the grid must have at least 8 workgroups.
struct XcdTiles {
  int m, ts, nt, x;
  long long ntiles, wx, nwx;
  __device__ __forceinline__ XcdTiles(int m_, int ts_, int waves_per_block) : m(m_), ts(ts_) {
    nt = (m + ts - 1) / ts;
    ntiles = (long long)nt * nt;
    x = blockIdx.x & 7;
    const long long bx = blockIdx.x >> 3, nbx = (gridDim.x - x + 7) >> 3;
    wx = bx * waves_per_block + (threadIdx.x >> 6);
    nwx = nbx * waves_per_block;
  }
  // false past the end; g = -1 for a slot of a partial tile outside the matrix
  __device__ __forceinline__ bool at(long long f, long long &g) const {
    const long long per = (long long)ts * ts, r = f / per, t = x + 8 * r;
    if (t >= ntiles) return false;
    const int sl = (int)(f - r * per);
    const int j = (int)(t / nt) * ts + sl / ts, k = (int)(t % nt) * ts + sl % ts;
    g = (j < m && k < m) ? (long long)j * m + k : -1;
    return true;
  }
};

// tile edge for columns of n rows: 2 ts columns in about 2 MB
__host__ __device__ constexpr int xcd_tile(int n) {
  return (1 << 20) / (8 * n) > 64 ? 64 : ((1 << 20) / (8 * n) < 4 ? 4 : (1 << 20) / (8 * n));
}

// Is element (key, row) at or above the pair (lk, lr) in sorted order?
__device__ __forceinline__ bool pair_ge(uint64_t key, int row, uint64_t lk, int lr) {
  return key > lk || (key == lk && row >= lr);
}
__device__ __forceinline__ bool pair_le(uint64_t key, int row, uint64_t hk, int hr) {
  return key < hk || (key == hk && row <= hr);
}

// ------------------------------------------------------------------ counts
// counts[g] (int64, written to offsets + 1 + g) and lambda_max[g] of segment
// g = j m + k; V0, R0: v_k and its row at lambda = 0 (m x m, row -1 for 0).
// kList: also list each segment's entries (key, row), when there are at most
// wcap (<= BP_LIST_MAX) of them, in row order at wkeys/wrows[g wcap ..]
// (staged in LDS, stored once per segment), and in wsb[g] the exact weight
// of the negative ratios (negative minimiser) or of the negative and zero
// ones (positive): the emit pass then takes its first window from there
// instead of scanning the rows again.
constexpr int BP_LIST_MAX = 128;
template <bool kList>
__global__ void __launch_bounds__(256)
k_bp_count(const double *__restrict__ X, int n, int m, long long ld, const ColInfo *__restrict__ ci,
           const double *__restrict__ V0, const int *__restrict__ R0, long long *__restrict__ counts,
           double *__restrict__ lmax, uint64_t *__restrict__ wkeys, unsigned short *__restrict__ wrows,
           u128 *__restrict__ wsb, int wcap) {
  const int lane = threadIdx.x & 63;
  __shared__ uint64_t skeys[4][BP_LIST_MAX];
  __shared__ unsigned short srows[4][BP_LIST_MAX];
  uint64_t *lk = skeys[(threadIdx.x >> 6) & 3];
  unsigned short *lr = srows[(threadIdx.x >> 6) & 3];
  const int ts = xcd_tile(n);
  const int T = (n + 63) >> 6;
  int Tp = 1;
  while (Tp < T) Tp <<= 1;
  const XcdTiles tl(m, ts, blockDim.x >> 6);
  for (long long f = tl.wx;; f += tl.nwx) {
    long long g;
    if (!tl.at(f, g)) break;
    if (g < 0) continue;
    // the segment is the same for the whole wave (scalar registers)
    const int j = __builtin_amdgcn_readfirstlane((int)(g / m)), k = __builtin_amdgcn_readfirstlane((int)(g % m));
    g = (long long)j * m + k;
    const ColInfo cj = ci[j];
    if (j == k || cj.flags) {
      if (lane == 0) {
        counts[g] = 0;
        lmax[g] = 0.0;
      }
      continue;
    }
    const SegIO s{X + (long long)k * ld, X + (long long)j * ld, n, T, Tp, cj.e0, lane, false};
    const int r0 = R0[g];
    const double v0 = V0[g];
    const uint64_t mkey = key_of(v0 + 0.0);
    const bool neg = v0 < 0.0;
    // weights as FP64 sums of 37-bit chunks (exact, see weight_chunks);
    // the columns are read one slot ahead
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, z0 = 0.0, z1 = 0.0, z2 = 0.0;
    int cnt = 0, nin = 0;
    const __amdgpu_buffer_rsrc_t rj = col_rsrc(s.sxj, n), rk = col_rsrc(s.xk, n);
    int off = lane * 8;
    double an = col_ld(rj, off), bn = col_ld(rk, off);
    for (int t = 0; t < T; ++t) {
      const int i = lane + 64 * t;
      const double a = an, b = bn;
      off += 512;
      an = col_ld(rj, off);
      bn = col_ld(rk, off);
      const uint64_t key = key_of_pair(i < n, a, b);
      const bool valid = key != KEY_NONE;
      const bool ng = key < KEY_ZERO, zr = key == KEY_ZERO;
      double c0, c1, c2;
      weight_chunks(a, s.e0, c0, c1, c2);
      // masked adds as fma with a 0/1 factor: the same exact sums (whole
      // numbers below 2^53; c 0 adds +0) in one op instead of select + add
      const double fn = ng ? 1.0 : 0.0, fz = zr ? 1.0 : 0.0;
      a0 = fma(c0, fn, a0);
      a1 = fma(c1, fn, a1);
      a2 = fma(c2, fn, a2);
      z0 = fma(c0, fz, z0);
      z1 = fma(c1, fz, z1);
      z2 = fma(c2, fz, z2);
      if (r0 >= 0 && valid) {
        const bool in = neg ? (key < KEY_ZERO && pair_ge(key, i, mkey, r0))
                            : (key > KEY_ZERO && pair_le(key, i, mkey, r0));
        cnt += in ? 1 : 0;
      }
      if constexpr (kList) {
        // the emit pass's first window: the same elements, in row order
        const bool inl = r0 >= 0 && valid &&
                         (neg ? (key < KEY_ZERO && pair_ge(key, i, mkey, r0))
                              : (key > KEY_ZERO && pair_le(key, i, mkey, r0)));
        const uint64_t im = __ballot(inl);
        const int pos = nin + lanes_below(im);
        nin += __builtin_popcountll(im);
        if (inl && pos < wcap) {
          lk[pos] = key;
          lr[pos] = (unsigned short)i;
        }
      }
    }
    const u128 A = chunks_to_u128(wave_sum_dbl(a0), wave_sum_dbl(a1), wave_sum_dbl(a2)),
               B = A + chunks_to_u128(wave_sum_dbl(z0), wave_sum_dbl(z1), wave_sum_dbl(z2)), W = cj.wfix;
    cnt = wave_sum_int(cnt);
    if constexpr (kList) {
      if (nin <= wcap) {
        wave_lds_sync();
        for (int e = lane; e < nin; e += 64) {
          wkeys[g * wcap + e] = lk[e];
          wrows[g * wcap + e] = lr[e];
        }
        wave_lds_sync();
      }
      if (lane == 0) wsb[g] = neg ? A : B;
    }
    u128 lm = 0;
    if ((A << 1) > W) lm = (A << 1) - W;
    else if (W > (B << 1)) lm = W - (B << 1);
    if (lane == 0) {
      counts[g] = (long long)((r0 >= 0 ? cnt : 0) + 1);
      lmax[g] = fixed_to_double(lm, cj.e0);
    }
  }
}

constexpr int BP_SCAN_BLOCKS = 1024;

// Inclusive block scan of one value per thread (1024 threads); returns the
// thread's inclusive prefix and leaves the block total in *tot.
__device__ __forceinline__ long long block_scan_ll(long long x, long long *sh, long long *tot) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  long long v = x;
  for (int d = 1; d < 64; d <<= 1) {
    const long long o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  if (lane == 63) sh[w] = v;
  __syncthreads();
  long long before = 0, all = 0;
  for (int q = 0; q < 16; ++q) {
    if (q < w) before += sh[q];
    all += sh[q];
  }
  __syncthreads();
  *tot = all;
  return before + v;
}

// Offsets: counts sit in offsets[1..count]; afterwards offsets[q] = the sum
// of counts 1..q and offsets[0] = 0.  Three passes: chunk sums, their scan,
// the chunks' scans.
__global__ void __launch_bounds__(1024)
k_bp_scan_sums(const long long *__restrict__ offsets, long long count, long long *__restrict__ part) {
  __shared__ long long sh[16];
  const long long chunk = (count + gridDim.x - 1) / gridDim.x;
  const long long b0 = (long long)blockIdx.x * chunk, e = min(count, b0 + chunk);
  long long sum = 0;
  for (long long q = b0 + threadIdx.x; q < e; q += 1024) sum += offsets[1 + q];
  long long tot;
  (void)block_scan_ll(sum, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_bp_scan_top(long long *__restrict__ part, int nb) {
  __shared__ long long sh[16];
  const long long x = threadIdx.x < nb ? part[threadIdx.x] : 0;
  long long tot;
  const long long incl = block_scan_ll(x, sh, &tot);
  if (threadIdx.x < nb) part[threadIdx.x] = incl - x;   // exclusive
}

__global__ void __launch_bounds__(1024)
k_bp_scan_fin(long long *__restrict__ offsets, long long count, const long long *__restrict__ part) {
  __shared__ long long sh[16];
  const long long chunk = (count + gridDim.x - 1) / gridDim.x;
  const long long b0 = (long long)blockIdx.x * chunk, e = min(count, b0 + chunk);
  long long carry = part[blockIdx.x];
  for (long long t0 = b0; t0 < e; t0 += 1024) {
    const long long q = t0 + threadIdx.x;
    const long long x = q < e ? offsets[1 + q] : 0;
    long long tot;
    const long long incl = block_scan_ll(x, sh, &tot);
    if (q < e) offsets[1 + q] = carry + incl;
    carry += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

// ------------------------------------------------------------------ entries
constexpr int BP_CAP = 512;                     // window list entries per wave
constexpr int BP_WAVES = 4;
constexpr int BP_MAX_ROUNDS = 4096;             // windows and halvings per segment

// writes one entry if `at` lies inside the segment's range [lo, hi); returns
// false (nothing written) otherwise
__device__ __forceinline__ bool bp_write(double *lam, double *v, int *row, long long at, long long lo,
                                         long long hi, double l, double vv, int r) {
  if (at < lo || at >= hi) return false;
  lam[at] = l;
  v[at] = vv;
  row[at] = r;
  return true;
}

__global__ void __launch_bounds__(256)
k_bp_emit(const double *__restrict__ X, int n, int m, long long ld, const ColInfo *__restrict__ ci,
          const double *__restrict__ V0, const int *__restrict__ R0, const long long *__restrict__ offsets,
          const double *__restrict__ lmax, long long capacity, double *__restrict__ lam, double *__restrict__ v,
          int *__restrict__ row, int *__restrict__ status, int *__restrict__ sticky,
          const uint64_t *__restrict__ wkeys, const unsigned short *__restrict__ wrows,
          const u128 *__restrict__ wsb, int wcap) {
  __shared__ uint64_t skeys[BP_WAVES][BP_CAP];
  __shared__ unsigned short srows[BP_WAVES][BP_CAP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t *lk = skeys[wave];
  unsigned short *lr = srows[wave];
  const long long nseg = (long long)m * m;
  if (offsets[nseg] > capacity) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
      if (status) atomicCAS(status, 0, L1LINE_ESIZE);
      if (sticky) atomicCAS(sticky, 0, L1LINE_ESIZE);
    }
    return;
  }
  const int ts = xcd_tile(n);
  const int T = (n + 63) >> 6;
  int Tp = 1;
  while (Tp < T) Tp <<= 1;
  const XcdTiles tl(m, ts, BP_WAVES);
  for (long long f = tl.wx;; f += tl.nwx) {
    long long g;
    if (!tl.at(f, g)) break;
    if (g < 0) continue;
    // the segment is the same for the whole wave (scalar registers)
    const int j = __builtin_amdgcn_readfirstlane((int)(g / m)), k = __builtin_amdgcn_readfirstlane((int)(g % m));
    g = (long long)j * m + k;
    const long long base = offsets[g], cnt = offsets[g + 1] - base;
    if (cnt == 0) continue;
    const ColInfo cj = ci[j];
    const int r0 = R0[g];
    if (r0 >= 0) {
      const SegIO s{X + (long long)k * ld, X + (long long)j * ld, n, T, Tp, cj.e0, lane, false};
      const u128 W = cj.wfix;
      const bool neg = V0[g] < 0.0;
      long long emitted = 0;
      // the window is [lo, hi] in (key, row) order, sweeping away from the
      // lambda = 0 minimiser towards 0
      uint64_t lo_k = key_of(V0[g] + 0.0), hi_k = KEY_ZERO - 1;
      int lo_r = r0, hi_r = 0xFFFF;
      if (!neg) {
        hi_k = lo_k;
        hi_r = r0;
        lo_k = KEY_ZERO + 1;
        lo_r = 0;
      }
      const uint64_t end_k = neg ? KEY_ZERO - 1 : KEY_ZERO + 1;   // the window edge nearest 0
      uint64_t w_lo = lo_k, w_hi = hi_k;          // current window keys (halved on overflow)
      int rounds = 0;
      bool bad = false;
      while (emitted < cnt - 1) {
        if (++rounds > BP_MAX_ROUNDS) {
          bad = true;
          break;
        }
        // one exact pass: weight of everything below the window, the
        // window's elements to the list
        const uint64_t wk_lo = neg ? lo_k : w_lo, wk_hi = neg ? w_hi : hi_k;
        const int wr_lo = neg ? lo_r : (w_lo == lo_k ? lo_r : 0);
        const int wr_hi = neg ? (w_hi == hi_k ? hi_r : 0xFFFF) : hi_r;
        // (weights as FP64 sums of 37-bit chunks, see weight_chunks; the
        // columns read one slot ahead)
        u128 Sb;
        int nwin = 0;
        bool listed = false;
        if (rounds == 1 && cnt - 1 <= wcap) {
          // the count pass listed this first window (every entry of the
          // segment); the weight below it is the count pass's weight of
          // the negative and zero ratios (positive minimiser), or of the
          // negative ones less the list's own (negative: the list is the
          // negative ratios from the minimiser on), taken after the sort
          listed = true;
          nwin = (int)(cnt - 1);
          const uint64_t *__restrict__ gk = wkeys + g * wcap;
          const unsigned short *__restrict__ gr = wrows + g * wcap;
          for (int e = lane; e < nwin; e += 64) {
            lk[e] = gk[e];
            lr[e] = gr[e];
          }
          Sb = wsb[g];
        } else {
        double b0 = 0.0, b1 = 0.0, b2 = 0.0;
        const __amdgpu_buffer_rsrc_t rj = col_rsrc(s.sxj, n), rk = col_rsrc(s.xk, n);
        int off = lane * 8;
        double an = col_ld(rj, off), bn = col_ld(rk, off);
        for (int t = 0; t < T; ++t) {
          const int i = lane + 64 * t;
          const double a = an, b = bn;
          off += 512;
          an = col_ld(rj, off);
          bn = col_ld(rk, off);
          const uint64_t key = key_of_pair(i < n, a, b);
          const bool valid = key != KEY_NONE;
          const bool lt = valid && !pair_ge(key, i, wk_lo, wr_lo);
          const bool in = valid && !lt && pair_le(key, i, wk_hi, wr_hi);
          double c0, c1, c2;
          weight_chunks(a, s.e0, c0, c1, c2);
          const double fl = lt ? 1.0 : 0.0;   // masked adds as fma (exact, as above)
          b0 = fma(c0, fl, b0);
          b1 = fma(c1, fl, b1);
          b2 = fma(c2, fl, b2);
          const uint64_t wm = __ballot(in);
          const int pos = nwin + lanes_below(wm);
          nwin += __builtin_popcountll(wm);
          if (in && pos < BP_CAP) {
            lk[pos] = key;
            lr[pos] = (unsigned short)i;
          }
        }
        Sb = chunks_to_u128(wave_sum_dbl(b0), wave_sum_dbl(b1), wave_sum_dbl(b2));
        nwin = uni_int(nwin);
        }
        wave_lds_sync();
        if (nwin > BP_CAP) {
          if (wk_lo == wk_hi) {
            // one key with more tied rows than the list: rows are in sorted
            // order already; stream them tile by tile
            u128 run = Sb;
            int done = 0;
            for (int t = 0; t < T; ++t) {
              const int i = lane + 64 * t;
              const uint64_t key = seg_key(s, i);
              const bool valid = key != KEY_NONE;
              const bool in = valid && pair_ge(key, i, wk_lo, wr_lo) && pair_le(key, i, wk_hi, wr_hi);
              const u128 w = seg_weight(s, i, in);
              const u128 incl = wave_incl_scan_u128(w, lane);
              const uint64_t wm = __ballot(in);
              const int rank = done + __builtin_popcountll(wm & ((1ull << lane) - 1ull));
              if (in) {
                const u128 Sprev = run + incl - w, Sp = run + incl;
                u128 lb = 0;
                long long at;
                if (neg) {
                  lb = (Sprev << 1) > W ? (Sprev << 1) - W : (u128)0;
                  at = base + emitted + rank;
                } else {
                  lb = W > (Sp << 1) ? W - (Sp << 1) : (u128)0;
                  at = base + emitted + (nwin - 1 - rank);
                }
                if (!bp_write(lam, v, row, at, base, base + cnt - 1, fixed_to_double(lb, cj.e0), ratio_of_key(key), i))
                  bad = true;
              }
              run += shfl_u128(incl, 63);
              done += __builtin_popcountll(wm);
            }
            emitted += nwin;
          } else {
            // halve the window in key space, keeping the edge nearest the
            // lambda = 0 minimiser
            if (neg) w_hi = wk_lo + (wk_hi - wk_lo) / 2;
            else w_lo = wk_hi - (wk_hi - wk_lo) / 2;
            continue;
          }
        } else {
          const int N = wave_sort_list(lk, lr, nwin, lane);
          const int E = N >> 6;
          u128 tot, incl;
          wave_list_sums(s, lk, lr, E, tot, incl);
          if (listed && neg) Sb -= shfl_u128(incl, 63);
          u128 run = Sb + incl - tot;                 // weight before this lane's entries
          for (int q = 0; q < E; ++q) {
            const int e = E * lane + q;
            const uint64_t key = lk[e];
            if (key == KEY_NONE) break;
            const int rr = (int)lr[e];
            const u128 w = seg_weight(s, rr, true);
            const u128 Sprev = run, Sp = run + w;
            run = Sp;
            u128 lb = 0;
            long long at;
            if (neg) {
              lb = (Sprev << 1) > W ? (Sprev << 1) - W : (u128)0;
              at = base + emitted + e;
            } else {
              lb = W > (Sp << 1) ? W - (Sp << 1) : (u128)0;
              at = base + emitted + (nwin - 1 - e);
            }
            if (!bp_write(lam, v, row, at, base, base + cnt - 1, fixed_to_double(lb, cj.e0), ratio_of_key(key), rr))
              bad = true;
          }
          wave_lds_sync();
          emitted += nwin;
        }
        // next window: the keys between this one and 0
        if (neg) {
          if (wk_hi >= end_k) break;
          lo_k = wk_hi + 1;
          lo_r = 0;
          w_hi = end_k;
        } else {
          if (wk_lo <= end_k) break;
          hi_k = wk_lo - 1;
          hi_r = 0xFFFF;
          w_lo = end_k;
        }
      }
      bad = __ballot(bad) != 0;
      if (bad || emitted != cnt - 1) {
        if (lane == 0) {
          if (status) atomicCAS(status, 0, L1LINE_EINTERNAL);
          if (sticky) atomicCAS(sticky, 0, L1LINE_EINTERNAL);
        }
      }
    }
    if (lane == 0) bp_write(lam, v, row, base + cnt - 1, base, base + cnt, lmax[g], 0.0, -1);
  }
}
