// fit_kernels.h -- kernels of the fixed-lambda fit and the lambda path
// (Sec. 2: Lemma 1 per (j, k) segment, Algorithm 1 objective and argmin).
#pragma once

#include "device_common.h"

#include <l1line.h>

enum : int {
  COL_NONFINITE = 1,   // a NaN or an infinity in the column
  COL_WIDE = 2,        // nonzero magnitudes too spread for 128-bit sums
};

enum : int {
  SEG_INTERNAL = 1,    // a selection exceeded its round bound
};

struct ColInfo {
  u128 wfix;    // exact sum of |x_ij| / 2^e0 over the column
  double W;     // R64 sum of |x_ij| (column mass)
  int e0;       // exponent of the lowest set bit over nonzero |x_ij|
  int nnz;      // nonzeros
  int zeros;    // exact zeros
  int flags;    // COL_*
  int bemin;    // smallest biased exponent field over nonzero entries
  int bemax;    // largest biased exponent field over nonzero entries
};

// One problem of a batch, as the kernels see it.  Workspace offsets are in
// elements of the batch-wide arrays.
struct ProbDesc {
  const double *X;      // n x m, column-major
  long long ld;
  int n, m, L;
  int lam_off;          // first penalty in the flat penalty array
  int col_off;          // first column in ColInfo / segflags
  int out_off;          // first (problem, lambda) slot: sum of L over earlier problems
  long long ws_off;     // first element of this problem's L*m*m block in V / E / R
  long long z_off;      // first element of this problem's L*m block in Z / zflag
  long long pair_off;   // first element of this problem's m*m block of sign sums
  long long mask_off;   // first word of this problem's zero-segment mask (mj ceil(m / 64) words)
  double *Vout;         // L*m
  long long *Jout;      // L
  double *OBJout;       // L
  int *ROWout;          // L*m or null
  double *ZALLout;      // L*m or null
  int *status;          // 1 or null
};

// A workgroup's unit of work: problem b, preserved column j, k in [kbeg, kend).
struct WorkItem {
  int b, j, kbeg, kend;
};

// first index i in [0, count) with prefix[i + 1] > g (prefix has count + 1 entries)
__device__ __forceinline__ int find_owner(const int *__restrict__ prefix, int count, long long g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ columns
// One wave per column: finiteness, counts, the fixed-point exponent e0, the
// range check, the exact fixed-point mass and the R64 column mass.
__device__ __forceinline__ void colprep_wave(const double *__restrict__ x, int n, ColInfo *__restrict__ out,
                                             int lane) {
  int bad = 0, nnz = 0, zeros = 0, lsb = 1 << 20, hb = -(1 << 20), bemin = 4096, bemax = -1;
  double part = 0.0;
  for (int i = lane; i < n; i += 64) {
    double v = x[i];
    double a = fabs(v);
    part = part + a;
    if (!isfinite(v)) {
      bad = 1;
    } else if (v == 0.0) {
      ++zeros;
    } else {
      ++nnz;
      lsb = min(lsb, lowest_bit_exp(a));
      hb = max(hb, highest_bit_exp(a));
      const int be = (int)((__double_as_longlong(a) >> 52) & 0x7ff);
      bemin = min(bemin, be);
      bemax = max(bemax, be);
    }
  }
  double W = wave_r64_tree(part);
  bad = wave_max_int(bad);
  nnz = wave_sum_int(nnz);
  zeros = wave_sum_int(zeros);
  lsb = wave_min_int(lsb);
  hb = wave_max_int(hb);
  bemin = wave_min_int(bemin);
  bemax = wave_max_int(bemax);
  int flags = bad ? COL_NONFINITE : 0;
  int e0 = nnz ? lsb : 0;
  if (!bad && nnz) {
    int bl = 32 - __builtin_clz((unsigned)nnz);
    if ((hb - e0 + 1) + bl > 124) flags |= COL_WIDE;
  }
  u128 s = 0;
  if (!flags) {
    for (int i = lane; i < n; i += 64) {
      double v = x[i];
      if (v != 0.0) s += fixed_of(fabs(v), e0);
    }
    s = wave_sum_u128(s);
  }
  if (lane == 0) {
    ColInfo c;
    c.wfix = s;
    c.W = W;
    c.e0 = e0;
    c.nnz = nnz;
    c.zeros = zeros;
    c.flags = flags;
    c.bemin = bemin;
    c.bemax = bemax;
    *out = c;
  }
}

__global__ void __launch_bounds__(256)
k_colprep(const double *__restrict__ X, int n, int m, long long ld, ColInfo *__restrict__ ci) {
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= m) return;
  colprep_wave(X + (long long)col * ld, n, ci + col, threadIdx.x & 63);
}

// every column of every problem: colstart[b] = first column of problem b
__global__ void __launch_bounds__(256)
k_colprep_batch(const ProbDesc *__restrict__ P, const int *__restrict__ colstart, int B, int total_cols,
                ColInfo *__restrict__ ci, int *__restrict__ segflags, const int *__restrict__ gate, int gate_on) {
  const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g >= total_cols) return;
  if (gate && *gate != gate_on) return;
  const int b = find_owner(colstart, B, g);
  const ProbDesc d = P[b];
  const int col = g - colstart[b];
  colprep_wave(d.X + (long long)col * d.ld, d.n, ci + g, threadIdx.x & 63);
  if ((threadIdx.x & 63) == 0) segflags[g] = 0;
}

// ----------------------------------------------------------- segment access
// One wave streams over the rows of segment (j, k); row i = lane + 64 t for
// slot t < T.  Column j sits in LDS, column k is read from global memory
// (it stays in L2/MALL across the concurrent workgroups).  Nothing per row
// is kept in registers: every pass recomputes the ratio it needs, which keeps
// the register count low and the occupancy high.
struct SegIO {
  const double *__restrict__ xk;   // column k (device memory)
  const double *__restrict__ sxj;  // column j (LDS when lds, else device memory)
  int n, T, Tp, e0, lane;          // rows, slots, pow2 >= T, fixed-point exponent
  bool lds;                        // a compile-time constant at every construction
};

// x_ij of row i, through the address space column j lives in
__device__ __forceinline__ double sxj_at(const SegIO &s, int i) {
  return s.lds ? s.sxj[i] : gld(s.sxj + i);
}

// x_ij of row i < 64 T, 0 past row n: the zero-padded LDS copy, or the
// column in device memory through its range-checked descriptor rj
__device__ __forceinline__ double sxj_pad(const SegIO &s, __amdgpu_buffer_rsrc_t rj, int i) {
  return s.lds ? s.sxj[i] : col_ld(rj, i * 8);
}

// key of fl(x_ik / x_ij) + 0.0; KEY_NONE outside the matrix or where x_ij = 0
__device__ __forceinline__ uint64_t seg_key(const SegIO &s, int i) {
  const bool in = i < s.n;
  const int ic = in ? i : 0;
  const double a = sxj_at(s, ic), b = gld(s.xk + ic);
  double r = b / a;
  r = r + 0.0;
  return (in && a != 0.0) ? key_of(r) : KEY_NONE;
}

// the same key from x_ij = a and x_ik = b already loaded (in: the row is
// inside the matrix); branch-free, so that loads of the next slot issued
// before it stay in flight across the divide
__device__ __forceinline__ uint64_t key_of_pair(bool in, double a, double b) {
  const bool ok = in && a != 0.0;
  double r = b / (ok ? a : 1.0);
  r = r + 0.0;
  return ok ? key_of(r) : KEY_NONE;
}

// The top 32 bits of the key of row i's ratio, estimated by the hardware
// reciprocal (x_ij != 0 at sample rows).  Sample keys only place window
// bounds and pivots, and any keys are valid there (every element is decided
// exactly against them), so neither the IEEE divide nor the low 32 bits of
// the key are needed: a bound derived from a prefix p is p 2^32 (lower) or
// p 2^32 + 2^32 - 1 (upper), at most 2^-20 relative off the sample's ratio.
__device__ __forceinline__ uint32_t sample_key32(const SegIO &s, int i) {
  const double a = sxj_at(s, i), b = gld(s.xk + i);
  double r = b * __builtin_amdgcn_rcp(a);
  r = r + 0.0;
  return (uint32_t)(key_of(r) >> 32);
}

// exact weight |x_ij| / 2^e0 of row i, 0 where !valid
__device__ __forceinline__ u128 seg_weight(const SegIO &s, int i, bool valid) {
  const double a = sxj_at(s, valid ? i : 0);
  return valid ? fixed_of_col(a, s.e0) : (u128)0;
}

__device__ __forceinline__ void take_sample(bool c, int pri, uint64_t key, int t, int &bp, uint64_t &bk,
                                            int &bt) {
  const bool better = c && pri < bp;
  bp = better ? pri : bp;
  bk = better ? key : bk;
  bt = better ? t : bt;
}

// Per-wave LDS area: the elements (key, row) that fall in the key window of
// the exact pass, and a 64-entry compaction buffer.
// Per-wave LDS: the <= 64 final candidates of the selection rounds, and the
// window list (keys and rows, capacity chosen per launch: WIN_CAP for single
// penalties, PATH_CAP for paths when the LDS allows).
constexpr int WIN_CAP = 512;
constexpr int PATH_CAP = 1024;
// (the LDS sort pads a list to the next power of two, which must stay
// inside the wave's area)
static_assert((WIN_CAP & (WIN_CAP - 1)) == 0 && (PATH_CAP & (PATH_CAP - 1)) == 0,
              "window list capacities must be powers of two");
struct WaveScratch {
  uint64_t ckey[64];
  int crow[64];
  // bisection of a window too full for the list: lower end and element
  // count of the part that holds the target, probe passes so far (kept here,
  // off the registers of the window pass)
  uint64_t blo;
  int bcnt, steps;
};

// Element sources of the exact selection: every row of the column (ratio
// recomputed), or the window list in LDS.  Slot t of lane l is element
// l + 64 t; both enumerate their elements in increasing row order.
// sbase / cbase: weight and count of the elements below every listed one
// (the selection's sums and counts are over all elements of the segment).
struct ColSrc {
  const SegIO &s;
  u128 sbase;
  int cbase;
  __device__ __forceinline__ int slots() const { return s.T; }
  __device__ __forceinline__ void at(int t, uint64_t &key, int &row) const {
    row = s.lane + 64 * t;
    key = seg_key(s, row);
  }
};

struct ListSrc {
  const SegIO &s;
  u128 sbase;
  int cbase;
  const uint64_t *keys;
  const unsigned short *rows;
  int nlist;
  __device__ __forceinline__ int slots() const { return (nlist + 63) >> 6; }
  __device__ __forceinline__ void at(int t, uint64_t &key, int &row) const {
    const int e = s.lane + 64 * t;
    const bool in = e < nlist;
    key = in ? keys[e] : KEY_NONE;
    row = in ? (int)rows[e] : 0;
  }
};

// ------------------------------------------------- finishing <= 64 candidates
// Candidates are the elements with klo < key <= khi (count <= 64); Slo is the
// exact weight of all elements with key <= klo.  Compact them to LDS, sort by
// (key, row) across the lanes, scan their exact weights from Slo and take the
// first whose prefix reaches tau.
template <class Src>
__device__ __forceinline__ void wave_finish(const SegIO &s, const Src &src, uint64_t klo, uint64_t khi, int count,
                                            u128 Slo, u128 tau, WaveScratch *ws, uint64_t &okey, int &orow,
                                            int &err) {
  const int lane = s.lane;
  int base = 0;
  const int ns = src.slots();
#pragma unroll 2
  for (int t = 0; t < ns; ++t) {
    uint64_t key;
    int row;
    src.at(t, key, row);
    const bool c = key > klo && key <= khi;
    const uint64_t mask = __ballot(c);
    const int pos = base + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
    if (c && pos < 64) {
      ws->ckey[pos] = key;
      ws->crow[pos] = row;
    }
    base += __builtin_popcountll(mask);
  }
  wave_lds_sync();
  uint64_t ck = lane < count ? ws->ckey[lane] : KEY_NONE;
  int cr = lane < count ? ws->crow[lane] : 0x7fffffff;
  wave_lds_sync();
  wave_sort_key_row(ck, cr, lane);
  const u128 w = seg_weight(s, lane < count ? cr : 0, lane < count);
  const u128 S = wave_incl_scan_u128(w, lane) + Slo;
  const uint64_t hit = __ballot(lane < count && S >= tau);
  if (!hit || base != count) {
    err |= SEG_INTERNAL;
    okey = KEY_NONE;
    orow = -1;
    return;
  }
  const int srcl = __builtin_ctzll(hit);
  okey = uni_u64(shfl_u64(ck, srcl));
  orow = uni_int(__shfl(cr, srcl));
}

// ----------------------------------------------------------- selection rounds
// Exact selection: find the first element, in (ratio, row) order, whose
// inclusive prefix weight reaches tau.  Candidates are the elements with
// klo < key <= khi; Slo/Clo (Shi/Chi) are the exact weight and count of ALL
// elements with key <= klo (<= khi).  Rounds take two pivots from a weighted
// sample of the candidates and count exactly; a round without progress
// switches to key-space bisection; a single repeated key falls back to row
// order.
template <class Src>
__device__ __forceinline__ void wave_select_rounds(const SegIO &s, const Src &src, uint64_t klo, uint64_t khi,
                                                   u128 Slo, u128 Shi, int Clo, int Chi, u128 tau,
                                                   WaveScratch *ws, uint64_t &okey, int &orow, int &err) {
  constexpr double DELTA = 0.15;
  const int lane = s.lane;
  const int ns = src.slots();
  int nsp = 1;
  while (nsp < ns) nsp <<= 1;
  int count = Chi - Clo;
  bool bisect = false, single_key = false;
  int rounds = 0;
  uint64_t sk = KEY_NONE;
  int sr = 0;
  okey = KEY_NONE;
  orow = -1;
  while (count > 64) {
    if (++rounds > 160) {
      err |= SEG_INTERNAL;
      return;
    }
    uint64_t plo, phi;
    if (!bisect) {
      double sw = (sk != KEY_NONE) ? fabs(sxj_at(s, sr)) : 0.0;
      wave_sort_key_dbl(sk, sw, lane);
      const double cw = wave_incl_scan_dbl(sw, lane);
      const double tot = __shfl(cw, 63);
      const double f = u128_to_double_approx(tau - Slo) / u128_to_double_approx(Shi - Slo);
      const double flo = (f - DELTA) * tot, fhi = (f + DELTA) * tot;
      const uint64_t mlo = __ballot(sk != KEY_NONE && cw <= flo);
      const uint64_t mhi = __ballot(sk != KEY_NONE && cw >= fhi);
      plo = mlo ? uni_u64(shfl_u64(sk, 63 - __builtin_clzll(mlo))) : klo;
      phi = mhi ? uni_u64(shfl_u64(sk, __builtin_ctzll(mhi))) : khi;
      if (phi < plo) phi = plo;
    } else {
      uint64_t cmin = KEY_NONE, cmax = 0;
#pragma unroll 2
      for (int t = 0; t < ns; ++t) {
        uint64_t key;
        int row;
        src.at(t, key, row);
        const bool c = key > klo && key <= khi;
        cmin = (c && key < cmin) ? key : cmin;
        cmax = (c && key > cmax) ? key : cmax;
      }
      cmin = wave_min_u64(cmin);
      cmax = wave_max_u64(cmax);
      if (cmin == cmax) {
        single_key = true;
        khi = cmax;
        break;
      }
      plo = phi = cmin + ((cmax - cmin) >> 1);
    }
    // exact weights and counts at or below each pivot, and one sample per
    // lane from each of the three sub-intervals
    u128 s1 = 0, s2 = 0;
    int c1 = 0, c2 = 0;
    uint64_t ka = KEY_NONE, kb = KEY_NONE, kc = KEY_NONE;
    int pa = nsp, pb = nsp, pc = nsp, ra = 0, rb = 0, rc = 0;
    const int start = (lane * 11 + rounds * 5) & (nsp - 1);
#pragma unroll 2
    for (int t = 0; t < ns; ++t) {
      uint64_t key;
      int row;
      src.at(t, key, row);
      const bool valid = key != KEY_NONE;
      const u128 w = seg_weight(s, row, valid);
      const bool le1 = valid && key <= plo, le2 = valid && key <= phi;
      s1 += le1 ? w : (u128)0;
      s2 += le2 ? w : (u128)0;
      c1 += le1 ? 1 : 0;
      c2 += le2 ? 1 : 0;
      const int pri = (t - start) & (nsp - 1);
      take_sample(key > klo && le1, pri, key, row, pa, ka, ra);
      take_sample(key > plo && le2, pri, key, row, pb, kb, rb);
      take_sample(key > phi && key <= khi, pri, key, row, pc, kc, rc);
    }
    s1 = wave_sum_u128(s1) + src.sbase;
    s2 = wave_sum_u128(s2) + src.sbase;
    c1 = wave_sum_int(c1) + src.cbase;
    c2 = wave_sum_int(c2) + src.cbase;
    if (s1 >= tau) {
      khi = plo; Shi = s1; Chi = c1;
      sk = ka; sr = ra;
    } else if (s2 >= tau) {
      klo = plo; Slo = s1; Clo = c1;
      khi = phi; Shi = s2; Chi = c2;
      sk = kb; sr = rb;
    } else {
      klo = phi; Slo = s2; Clo = c2;
      sk = kc; sr = rc;
    }
    const int ncount = Chi - Clo;
    bisect = (ncount == count);
    count = ncount;
  }
  if (!single_key) {
    wave_finish(s, src, klo, khi, count, Slo, tau, ws, okey, orow, err);
    return;
  }
  // every candidate has the same key K: (key, row) order is enumeration order
  const uint64_t K = khi;
  u128 S = Slo;
  for (int t = 0; t < ns; ++t) {
    uint64_t key;
    int row;
    src.at(t, key, row);
    const bool c = key == K;
    const u128 w = seg_weight(s, row, c);
    const u128 sc = wave_incl_scan_u128(w, lane) + S;
    const uint64_t hit = __ballot(c && sc >= tau);
    if (hit) {
      const int sl = __builtin_ctzll(hit);
      okey = K;
      orow = uni_int(__shfl(row, sl));
      return;
    }
    S = uni_u128(shfl_u128(sc, 63));
  }
  err |= SEG_INTERNAL;
}

// --------------------------------------------------- sorting the window list
// The window list (nlist entries, row order) is padded to a power of two
// N >= 64 with KEY_NONE and sorted by (key, row) with a bitonic network in
// LDS (each lane handles N/128 compare-exchanges per stage).  Returns N.
__device__ __forceinline__ int wave_sort_lds(uint64_t *lk, unsigned short *lr, int nlist, int lane) {
  int N = 64;
  while (N < nlist) N <<= 1;
  for (int e = nlist + lane; e < N; e += 64) {
    lk[e] = KEY_NONE;
    lr[e] = 0xFFFF;
  }
  wave_lds_sync();
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int pidx = lane; pidx < (N >> 1); pidx += 64) {
        const int e = ((pidx & ~(stride - 1)) << 1) | (pidx & (stride - 1));
        const int f = e + stride;
        const uint64_t ke = lk[e], kf = lk[f];
        const unsigned re = lr[e], rf = lr[f];
        const bool up = (e & size) == 0;
        const bool gt = ke > kf || (ke == kf && re > rf);
        const bool lt = ke < kf || (ke == kf && re < rf);
        if (up ? gt : lt) {
          lk[e] = kf;
          lk[f] = ke;
          lr[e] = (unsigned short)rf;
          lr[f] = (unsigned short)re;
        }
      }
      wave_lds_sync();
    }
  }
  return N;
}

// Exact weights of the sorted list: lane l owns the E = N/64 consecutive
// entries [E l, E l + E); tot = their exact weight, incl = inclusive scan of
// tot over the lanes.
__device__ __forceinline__ void wave_list_sums(const SegIO &s, const uint64_t *lk, const unsigned short *lr, int E,
                                               u128 &tot, u128 &incl) {
  tot = 0;
  for (int q = 0; q < E; ++q) {
    const int e = E * s.lane + q;
    const bool valid = lk[e] != KEY_NONE;
    tot += seg_weight(s, valid ? (int)lr[e] : 0, valid);
  }
  incl = wave_incl_scan_u128_x(tot, s.lane);
}

// Lane-parallel resolution: every lane with a target (active) finds the first
// list entry whose exact prefix weight, counted from Slo (the weight of every
// element below the list), reaches its tau.  A binary search over the lanes'
// inclusive sums finds the owning lane, a walk over its entries the element.
// hit = false when tau lies outside (Slo, Slo + weight of the list].
// The weight below the list is known to lie in [SloA, SloB]; the search runs
// at SloA, and amb is set where the answer at SloB could differ: the hit
// status, or an earlier entry reaching tau (the entries before the found one
// weigh run_prev - SloA; at SloB the found entry is still the first iff
// run_prev + (SloB - SloA) < tau; it still reaches tau since SloB >= SloA).
__device__ __forceinline__ void wave_resolve(const SegIO &s, const uint64_t *lk, const unsigned short *lr, int E,
                                             u128 SloA, u128 SloB, u128 tot, u128 incl, bool active, u128 tau,
                                             uint64_t &okey, int &orow, bool &hit, bool &amb) {
  const u128 wall = readlane_u128(incl, 63);
  const bool inwin = active && tau > SloA && tau <= SloA + wall;
  const bool inwinB = active && tau > SloB && tau <= SloB + wall;
  int lo = 0, hi = 63;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int mid = (lo + hi) >> 1;
    const u128 im = shfl_u128(incl, mid);
    if (SloA + im >= tau) hi = mid;
    else lo = mid + 1;
  }
  const u128 totc = shfl_u128(tot, lo), inclc = shfl_u128(incl, lo);
  hit = false;
  amb = inwin != inwinB;
  if (inwin) {
    u128 run = SloA + inclc - totc;
    for (int q = 0; q < E; ++q) {
      const int e = E * lo + q;
      const uint64_t key = lk[e];
      const bool valid = key != KEY_NONE;
      const u128 before = run;
      run += seg_weight(s, valid ? (int)lr[e] : 0, valid);
      if (valid && run >= tau) {
        okey = key;
        orow = (int)lr[e];
        hit = true;
        amb = amb || !(before + (SloB - SloA) < tau);
        break;
      }
    }
  }
}

// Resolution of one target tau, the same on every lane: the entry's owner is
// the first lane whose inclusive sum, counted from Slo, reaches tau (one
// ballot), and a walk over that lane's E entries finds the entry.  The exact
// weight below the list is known to lie in [SloA, SloB]; amb = the answer is
// not the same at both ends (then nothing is reported).
__device__ __forceinline__ void wave_resolve_one(const SegIO &s, const uint64_t *lk, const unsigned short *lr,
                                                 int E, u128 SloA, u128 SloB, u128 tot, u128 incl, u128 tau,
                                                 uint64_t &okey, int &orow, bool &hit, bool &amb) {
  auto find = [&](u128 Slo, uint64_t &k, int &r) -> bool {
    const uint64_t owner = __ballot(Slo + incl >= tau);
    if (!(tau > Slo) || owner == 0) return false;
    const int lo = __builtin_ctzll(owner);
    u128 run = Slo + readlane_u128(incl, lo) - readlane_u128(tot, lo);
    for (int q = 0; q < E; ++q) {
      const int e = E * lo + q;
      const uint64_t key = lk[e];
      const bool valid = key != KEY_NONE;
      run += seg_weight(s, valid ? (int)lr[e] : 0, valid);
      if (valid && run >= tau) {
        k = key;
        r = (int)lr[e];
        return true;
      }
    }
    return false;
  };
  uint64_t k2 = KEY_NONE;
  int r2 = -1;
  hit = find(SloA, k2, r2);
  amb = false;
  if (SloB != SloA) {
    uint64_t k3 = KEY_NONE;
    int r3 = -1;
    const bool h3 = find(SloB, k3, r3);
    amb = h3 != hit || k3 != k2 || r3 != r2;
  }
  okey = k2;
  orow = r2;
}

// e_jk = R64 over i of |x_ik - fl(v x_ij)| (result in lane 0).  kPad: rows
// past n are read as 0 instead of masked (the single-penalty kernels; the
// several-penalty ones keep the masked loop, which spills less there)
template <bool kPad>
__device__ __forceinline__ double wave_residual(const SegIO &s, double v) {
  // column k in batches of RB loads issued back to back (the sum is still
  // taken slot by slot in increasing order)
  constexpr int RB = 8;
  double p = 0.0;
  if (kPad && __builtin_isfinite(v)) {
    // rows past n read 0 from both columns and add |0 - v 0| = +0, which
    // leaves the lane's partial as it is: no per-row masks or clamps
    const __amdgpu_buffer_rsrc_t rk = col_rsrc(s.xk, s.n), rj = col_rsrc(s.lds ? s.xk : s.sxj, s.n);
    int t0 = 0;
    for (; t0 + RB <= s.T; t0 += RB) {
      double xk[RB], xj[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        xk[r] = col_ld(rk, (s.lane + 64 * (t0 + r)) * 8);
        xj[r] = sxj_pad(s, rj, s.lane + 64 * (t0 + r));
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const double prod = v * xj[r];
        const double d = xk[r] - prod;
        p = p + fabs(d);
      }
    }
    for (; t0 < s.T; ++t0) {
      const int i = s.lane + 64 * t0;
      const double prod = v * sxj_pad(s, rj, i);
      const double d = col_ld(rk, i * 8) - prod;
      p = p + fabs(d);
    }
    return wave_r64_tree_x(p);
  }
  // (an infinite ratio: v 0 is NaN, so the rows past n are masked)
  for (int t0 = 0; t0 < s.T; t0 += RB) {
    double xk[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = s.lane + 64 * (t0 + r);
      xk[r] = gld(s.xk + (i < s.n ? i : 0));
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = s.lane + 64 * (t0 + r);
      const bool in = i < s.n;
      const double prod = v * sxj_at(s, in ? i : 0);
      const double d = xk[r] - prod;
      p = p + (in ? fabs(d) : 0.0);
    }
  }
  return wave_r64_tree_x(p);
}

// G residuals in one pass over the rows (the same sums as wave_residual,
// G at a time); e[r] is the wave's R64 sum for v[r].
template <int G>
__device__ __forceinline__ void wave_residual_multi(const SegIO &s, const double *v, double *e) {
  double p[G];
#pragma unroll
  for (int r = 0; r < G; ++r) p[r] = 0.0;
  bool fin = true;
#pragma unroll
  for (int r = 0; r < G; ++r) fin = fin && __builtin_isfinite(v[r]);
  if (fin) {
    // rows past n read 0 from both columns and add |0 - v 0| = +0; the
    // rows in batches of RB slots, every load of a batch issued before the
    // first is used (the sums still run slot by slot in increasing order)
    const __amdgpu_buffer_rsrc_t rk = col_rsrc(s.xk, s.n), rj = col_rsrc(s.lds ? s.xk : s.sxj, s.n);
    constexpr int RB = 4;
    // batch t0's loads are issued while batch t0 - RB is scored
    auto load_batch = [&](int t0, double *av, double *bv) {
      if (t0 + RB <= s.T) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int i = s.lane + 64 * (t0 + q);
          av[q] = sxj_pad(s, rj, i);
          bv[q] = col_ld(rk, i * 8);
        }
      } else {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          // (slots past T, of the last batch: 0 from both columns)
          const bool in = t0 + q < s.T;
          const int i = s.lane + 64 * (t0 + q);
          av[q] = in ? sxj_pad(s, rj, i) : 0.0;
          bv[q] = in ? col_ld(rk, i * 8) : 0.0;
        }
      }
    };
    double an[RB], bn[RB];
    load_batch(0, an, bn);
    for (int t0 = 0; t0 < s.T; t0 += RB) {
      double av[RB], bv[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        av[q] = an[q];
        bv[q] = bn[q];
      }
      if (t0 + RB < s.T) load_batch(t0 + RB, an, bn);
#pragma unroll
      for (int q = 0; q < RB; ++q) {
#pragma unroll
        for (int r = 0; r < G; ++r) {
          const double prod = v[r] * av[q];
          const double d = bv[q] - prod;
          p[r] = p[r] + fabs(d);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r) e[r] = readlane_dbl(wave_r64_tree_x(p[r]), 0);
    return;
  }
  const int l0 = s.lane < s.n ? s.lane : 0;
  double an = sxj_at(s, l0), bn = gld(s.xk + l0);
  for (int t = 0; t < s.T; ++t) {
    const int i = s.lane + 64 * t;
    const bool in = i < s.n;
    const double a = an, b = bn;
    if (t + 1 < s.T) {
      const int i2 = i + 64 < s.n ? i + 64 : 0;
      an = sxj_at(s, i2);
      bn = gld(s.xk + i2);
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const double prod = v[r] * a;
      const double d = b - prod;
      p[r] = p[r] + (in ? fabs(d) : 0.0);
    }
  }
#pragma unroll
  for (int r = 0; r < G; ++r) e[r] = readlane_dbl(wave_r64_tree_x(p[r]), 0);
}

// The next RJ residual jobs of mask jm (lanes whose target needs its own
// e_jk; v_l: the lane's ratio): one pass over the rows scores them all, and
// each job's lane receives its e in e_l.  Clears the jobs taken from jm.
template <int RJ>
__device__ __forceinline__ void run_jobs(const SegIO &s, uint64_t &jm, double v_l, int lane, double &e_l) {
  int jl[RJ];
  double jv[RJ], je[RJ];
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    jl[r] = jm ? __builtin_ctzll(jm) : -1;
    jm &= jm ? jm - 1 : 0;
    jv[r] = jl[r] >= 0 ? readlane_dbl(v_l, jl[r]) : 0.0;
  }
  wave_residual_multi<RJ>(s, jv, je);
#pragma unroll
  for (int r = 0; r < RJ; ++r)
    if (lane == jl[r]) e_l = je[r];
}

// Bitonic sort of 128 keys held two per lane (element 2*lane + r), ascending.
__device__ __forceinline__ void wave_sort2(uint64_t &a, uint64_t &b, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool up = ((2 * lane) & size) == 0;
      if (stride == 1) {
        const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        a = up ? lo : hi;
        b = up ? hi : lo;
      } else {
        const int ls = stride >> 1;
        const uint64_t oa = shfl_xor_u64(a, ls), ob = shfl_xor_u64(b, ls);
        const bool keep_min = (((2 * lane) & stride) == 0) == up;
        a = keep_min ? (oa < a ? oa : a) : (oa > a ? oa : a);
        b = keep_min ? (ob < b ? ob : b) : (ob > b ? ob : b);
      }
    }
  }
}

// Bitonic sort of 128 (key, row) pairs held two per lane (element
// 2 lane + r), ascending in (key, row).
__device__ __forceinline__ void wave_sort2_kr(uint64_t &ka, int &ra, uint64_t &kb, int &rb, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool up = ((2 * lane) & size) == 0;
      if (stride == 1) {
        const bool sw = (kb < ka || (kb == ka && rb < ra)) == up;
        const uint64_t tk = ka;
        const int tr = ra;
        ka = sw ? kb : ka;
        ra = sw ? rb : ra;
        kb = sw ? tk : kb;
        rb = sw ? tr : rb;
      } else {
        const int ls = stride >> 1;
        const bool keep_min = (((2 * lane) & stride) == 0) == up;
        const uint64_t oka = shfl_xor_u64(ka, ls), okb = shfl_xor_u64(kb, ls);
        const int ora = __shfl_xor(ra, ls), orb = __shfl_xor(rb, ls);
        const bool la = oka < ka || (oka == ka && ora < ra), lb = okb < kb || (okb == kb && orb < rb);
        if (la == keep_min) {
          ka = oka;
          ra = ora;
        }
        if (lb == keep_min) {
          kb = okb;
          rb = orb;
        }
      }
    }
  }
}

// Bitonic sort of 128 32-bit keys held two per lane (element 2 lane + r),
// ascending, through VALU lane exchanges.
__device__ __forceinline__ void wave_sort2_u32_x(uint32_t &a, uint32_t &b, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool up = ((2 * lane) & size) == 0;
      if (stride == 1) {
        const uint32_t lo = min(a, b), hi = max(a, b);
        a = up ? lo : hi;
        b = up ? hi : lo;
      } else {
        const int ls = stride >> 1;
        const uint32_t oa = xswap32(a, ls), ob = xswap32(b, ls);
        const bool keep_min = (((2 * lane) & stride) == 0) == up;
        a = keep_min ? min(oa, a) : max(oa, a);
        b = keep_min ? min(ob, b) : max(ob, b);
      }
    }
  }
}

// wave_sort2 and wave_sort2_kr through VALU lane exchanges (same networks)
__device__ __forceinline__ void wave_sort2_x(uint64_t &a, uint64_t &b, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool up = ((2 * lane) & size) == 0;
      if (stride == 1) {
        const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        a = up ? lo : hi;
        b = up ? hi : lo;
      } else {
        const int ls = stride >> 1;
        const uint64_t oa = xswap64(a, ls), ob = xswap64(b, ls);
        const bool keep_min = (((2 * lane) & stride) == 0) == up;
        a = keep_min ? (oa < a ? oa : a) : (oa > a ? oa : a);
        b = keep_min ? (ob < b ? ob : b) : (ob > b ? ob : b);
      }
    }
  }
}

__device__ __forceinline__ void wave_sort2_kr_x(uint64_t &ka, int &ra, uint64_t &kb, int &rb, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const bool up = ((2 * lane) & size) == 0;
      if (stride == 1) {
        const bool sw = (kb < ka || (kb == ka && rb < ra)) == up;
        const uint64_t tk = ka;
        const int tr = ra;
        ka = sw ? kb : ka;
        ra = sw ? rb : ra;
        kb = sw ? tk : kb;
        rb = sw ? tr : rb;
      } else {
        const int ls = stride >> 1;
        const bool keep_min = (((2 * lane) & stride) == 0) == up;
        const uint64_t oka = xswap64(ka, ls), okb = xswap64(kb, ls);
        const int ora = (int)xswap32((uint32_t)ra, ls), orb = (int)xswap32((uint32_t)rb, ls);
        const bool la = oka < ka || (oka == ka && ora < ra), lb = okb < kb || (okb == kb && orb < rb);
        ka = la == keep_min ? oka : ka;
        ra = la == keep_min ? ora : ra;
        kb = lb == keep_min ? okb : kb;
        rb = lb == keep_min ? orb : rb;
      }
    }
  }
}

// The same network over 256 entries, four per lane (entry 4 lane + q in
// slot q): strides 1 and 2 pair slots of one lane, longer strides pair slot q
// with slot q of lane (lane ^ stride / 4).
__device__ __forceinline__ void wave_sort4_kr_x(uint64_t (&k)[4], int (&r)[4], int lane) {
#pragma unroll
  for (int size = 2; size <= 256; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride < 4) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q & stride) continue;
          const int p = q | stride;
          const bool up = ((4 * lane + q) & size) == 0;
          const bool sw = (k[p] < k[q] || (k[p] == k[q] && r[p] < r[q])) == up;
          const uint64_t tk = k[q];
          const int tr = r[q];
          k[q] = sw ? k[p] : k[q];
          r[q] = sw ? r[p] : r[q];
          k[p] = sw ? tk : k[p];
          r[p] = sw ? tr : r[p];
        }
      } else {
        const int ls = stride >> 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool up = ((4 * lane + q) & size) == 0;
          const bool keep_min = ((lane & ls) == 0) == up;
          const uint64_t ok = xswap64(k[q], ls);
          const int orow = (int)xswap32((uint32_t)r[q], ls);
          const bool lt = ok < k[q] || (ok == k[q] && orow < r[q]);
          k[q] = lt == keep_min ? ok : k[q];
          r[q] = lt == keep_min ? orow : r[q];
        }
      }
    }
  }
}

// Sorts the window list lk/lr[0, nlist) ascending in (key, row) and pads it
// with (KEY_NONE, 0xFFFF) to N = the returned power of two (>= 64).  Lists of
// up to 256 are sorted in registers (VALU lane exchanges, no LDS round trips
// per stage) and written back; longer ones by the LDS network.
__device__ __forceinline__ int wave_sort_list(uint64_t *lk, unsigned short *lr, int nlist, int lane) {
  if (nlist > 256) return wave_sort_lds(lk, lr, nlist, lane);
  if (nlist > 128) {
    uint64_t k[4];
    int r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 4 * lane + q;
      k[q] = e < nlist ? lk[e] : KEY_NONE;
      r[q] = e < nlist ? (int)lr[e] : 0xFFFF;
    }
    wave_sort4_kr_x(k, r, lane);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lk[4 * lane + q] = k[q];
      lr[4 * lane + q] = (unsigned short)r[q];
    }
    wave_lds_sync();
    return 256;
  }
  if (nlist <= 64) {
    uint64_t k = lane < nlist ? lk[lane] : KEY_NONE;
    int r = lane < nlist ? (int)lr[lane] : 0xFFFF;
    wave_sort_key_row_x(k, r, lane);
    wave_lds_sync();
    lk[lane] = k;
    lr[lane] = (unsigned short)r;
    wave_lds_sync();
    return 64;
  }
  const int e = 2 * lane;
  uint64_t ka = e < nlist ? lk[e] : KEY_NONE, kb = e + 1 < nlist ? lk[e + 1] : KEY_NONE;
  int ra = e < nlist ? (int)lr[e] : 0xFFFF, rb = e + 1 < nlist ? (int)lr[e + 1] : 0xFFFF;
  wave_sort2_kr_x(ka, ra, kb, rb, lane);
  wave_lds_sync();
  lk[e] = ka;
  lr[e] = (unsigned short)ra;
  lk[e + 1] = kb;
  lr[e + 1] = (unsigned short)rb;
  wave_lds_sync();
  return 128;
}

// --------------------------------------------------------------- sign sums
// For the pair (j, k) the ratio of row i, x_ik / x_ij, is positive, negative
// or zero with the signs of x_ik and x_ij (barring underflow, checked per
// segment).  Its weight is |x_ij|, so
//   D_jk  = sum_i x_ij sgn(x_ik)        = (weight of positive ratios) - (negative)
//   Zr_jk = sum_i |x_ij| [x_ik == 0]    = weight of the zero ratios
// and 0 minimises g_jk exactly when |D_jk| <= lambda + Zr_jk (Lemma 1 at the
// point 0).  Both are dense contractions over the rows: X^T sgn(X) and
// |X|^T [X == 0], computed here for all pairs with FP64 MFMA (16x16x4).
// Their rounding error (at most about n 2^-52 of the column mass) is far
// below the decision margin the segment kernel applies.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int SS_TILE = 64;     // 64 (j) x 64 (k) outputs per workgroup, 4 waves of 16 x 64
constexpr int SS_ROWS = 16;     // rows i per LDS stage
constexpr int SS_LD = SS_TILE + 2;

// Fragment layout of v_mfma_f64_16x16x4f64 (wave64, measured on gfx950):
// lane l holds A[l & 15][l >> 4], B[l >> 4][l & 15] and D[(l >> 4) + 4 q][l & 15],
// q = 0..3 (unlike the FP32-output forms, the row index steps by 4 per
// register).
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One 64 x 64 output tile of the sign sums of a column-major matrix; rows j of
// the tile are j0.. j0 + 63 of the candidate list (cand) or of 0..m-1.
// out[j m + k] = (D_jk, Zr_jk).  Every thread of the 256-wide block calls it.
__device__ __forceinline__ void signsum_tile(const double *__restrict__ X, int ilo, int ihi, int m, long long ld,
                                             const int *__restrict__ cand, int mj, int j0, int k0,
                                             double2 *__restrict__ out, bool by_index) {
  __shared__ double sA[SS_ROWS * SS_LD];
  __shared__ double sB[SS_ROWS * SS_LD];
  __shared__ int sj[SS_TILE];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < SS_TILE) {
    const int jj = j0 + tid;
    sj[tid] = jj < mj ? (cand ? cand[jj] : jj) : -1;
  }
  __syncthreads();
  f64x4 accD[4], accZ[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accD[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    accZ[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
  }
  // rows in stages of SS_ROWS: each thread loads its PER + PER elements of
  // the next stage into registers while the current one is multiplied, and
  // stores column k's elements as their signs (computed once per element,
  // not once per wave that reads them)
  constexpr int PER = SS_ROWS * SS_TILE / 256;
  double pa[PER], pb[PER];
  auto load = [&](int i0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int c = e / SS_ROWS, r = e % SS_ROWS, i = i0 + r;
      const int jc = sj[c], kc = k0 + c;
      pa[q] = (i < ihi && jc >= 0) ? X[(long long)jc * ld + i] : 0.0;
      pb[q] = (i < ihi && kc < m) ? X[(long long)kc * ld + i] : 0.0;
    }
  };
  load(ilo);
  for (int i0 = ilo; i0 < ihi; i0 += SS_ROWS) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int c = e / SS_ROWS, r = e % SS_ROWS;
      const double x = pb[q];
      sA[r * SS_LD + c] = pa[q];
      sB[r * SS_LD + c] = x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0);
    }
    __syncthreads();
    if (i0 + SS_ROWS < ihi) load(i0 + SS_ROWS);
#pragma unroll 2
    for (int kk = 0; kk < SS_ROWS / 4; ++kk) {
      const int r = 4 * kk + (lane >> 4);
      const double a = sA[r * SS_LD + 16 * wave + (lane & 15)];
      const double aa = fabs(a);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double sg = sB[r * SS_LD + 16 * t + (lane & 15)];
        accD[t] = mfma_f64(a, sg, accD[t]);
        // exact zeros are rare: skip the product when this 4 x 16 block has none
        if (__ballot(sg == 0.0)) accZ[t] = mfma_f64(aa, sg == 0.0 ? 1.0 : 0.0, accZ[t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = k0 + 16 * t + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jl = 16 * wave + (lane >> 4) + 4 * q, j = sj[jl];
      if (j >= 0 && k < m) out[(long long)(by_index ? j0 + jl : j) * m + k] = make_double2(accD[t][q], accZ[t][q]);
    }
  }
}

// tstart[b] = first tile of problem b; problem b has ceil(mj / 64) x
// ceil(m / 64) tiles with mj = ncand when cand is given (problem 0 only),
// else m.  DZ[pair_off + j m + k] = (D_jk, Zr_jk).
// split > 1 (one problem, a candidate list): block g sums tile g / split over
// the rows of part g % split into part[(g % split) ncand m + jj m + k] (jj
// the candidate's index); k_signsum_parts adds the parts.
__global__ void __launch_bounds__(256)
k_signsum_batch(const ProbDesc *__restrict__ P, const int *__restrict__ tstart, int B,
                const int *__restrict__ cand, int ncand, double2 *__restrict__ DZ,
                const int *__restrict__ gate, int gate_on, int split, double2 *__restrict__ part) {
  if (gate && *gate != gate_on) return;
  if (split > 1) {
    const ProbDesc d = P[0];
    const int tile = blockIdx.x / split, sp = blockIdx.x % split;
    const int tk_count = (d.m + SS_TILE - 1) / SS_TILE;
    const int rows = (d.n + split - 1) / split;
    const int ilo = min(d.n, sp * rows), ihi = min(d.n, ilo + rows);
    signsum_tile(d.X, ilo, ihi, d.m, d.ld, cand, ncand, (tile / tk_count) * SS_TILE, (tile % tk_count) * SS_TILE,
                 part + (long long)sp * ncand * d.m, true);
    return;
  }
  const int g = blockIdx.x;
  const int b = find_owner(tstart, B, g);
  const ProbDesc d = P[b];
  const int mj = cand ? ncand : d.m;
  const int tk_count = (d.m + SS_TILE - 1) / SS_TILE;
  const int tloc = g - tstart[b];
  signsum_tile(d.X, 0, d.n, d.m, d.ld, cand, mj, (tloc / tk_count) * SS_TILE, (tloc % tk_count) * SS_TILE,
               DZ + d.pair_off, false);
}

// DZ[cand[jj] m + k] = the parts' sums added in part order (one problem)
__global__ void __launch_bounds__(256)
k_signsum_parts(const double2 *__restrict__ part, int split, const int *__restrict__ cand, int ncand, int m,
                double2 *__restrict__ DZ, const int *__restrict__ gate, int gate_on) {
  if (gate && *gate != gate_on) return;
  const long long per = (long long)ncand * m;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (long long)gridDim.x * blockDim.x) {
    double2 acc = part[e];
    for (int sp = 1; sp < split; ++sp) {
      const double2 x = part[(long long)sp * per + e];
      acc.x = acc.x + x.x;
      acc.y = acc.y + x.y;
    }
    DZ[(long long)cand[e / m] * m + e % m] = acc;
  }
}

// ---------------------------------------------------------------- segments
// Workgroup = (preserved column j, one part of the k range); its waves take
// the next k from an LDS counter.  For every (j, k) and lambda_t it writes
//   V[(t m + j) m + k] = v_k,  E[...] = e_jk,  R[...] = median row (-1 for 0).
//
// Per segment:
//  1. the sign sums D_jk, Zr_jk (k_signsum_batch) decide, with a rigorous
//     error margin, whether 0 minimises g_jk -- then v_k = 0 and e_jk is the
//     R64 column mass of k (|x_ik - fl(0 x_ij)| = |x_ik|) -- or on which side
//     of 0 the minimiser lies.  Otherwise an exact pass (128-bit sums)
//     decides.
//  2. The ratios of 128 rows drawn once per j with probability proportional
//     to |x_ij| estimate where the weighted median lies: a key window.
//  3. One exact pass sums the weight below the window and appends the
//     window's elements (key, row) to an LDS list, which is sorted and
//     scanned exactly.
//  Whatever the window does not settle goes to the general rounds.
constexpr int SEG_WAVES = 4;
constexpr int SAMPLE_ROWS = 128;
constexpr int SXJ_LDS_MAX = 4096;   // longest column j copied to LDS (32 KB)
constexpr int SEG_MASK_WORDS = 64;  // zero-segment mask words an item holds (one per lane: 4096 k)

__host__ __device__ constexpr size_t seg_sxj_bytes(int n) {
  return ((size_t)((n + 63) / 64) * 64 * 8 + 15) / 16 * 16;
}
__host__ __device__ constexpr size_t seg_lds_bytes(int n, int L, int lcap) {
  return seg_sxj_bytes(n) + SAMPLE_ROWS * 4 + (size_t)L * 16 +
         SEG_WAVES * (sizeof(WaveScratch) + (size_t)lcap * (sizeof(uint64_t) + sizeof(unsigned short))) + 16;
}


// ------------------------------------------------ division-free window pass
// Fast form of the exact pass.  For a row with a = x_ij != 0 and b = x_ik the
// ratio is q = b / a = u / |a| with u = b sgn(a) (exact), so q <= bound
// exactly when u <= bound |a|.  Comparing u with fl(bound' |a|), bound' the
// window bound moved outwards by 2^-49 of its magnitude, decides without a
// division, and rigorously, whether fl(q) lies at or below the window (its
// weight |a| joins an FP64 sum) or above it (dropped); rows inside the guard
// band or the window are listed by row and get their exact key (one IEEE
// divide each) in a second pass over the list, which keeps the window's
// elements (key, row) in row order -- the list the exact pass builds.  Zero
// bounds are sign tests: u < 0 is u <= -2^-1074 (the smallest subnormal).
// Valid when every nonzero magnitude of columns j and k lies in
// [2^-300, 2^300]: then q and the products stay normal.
constexpr int FAST_BEXP_LO = 1023 - 300, FAST_BEXP_HI = 1023 + 300;

__device__ __forceinline__ bool fast_columns(const ColInfo &c) {
  return c.nnz == 0 || (c.bemin >= FAST_BEXP_LO && c.bemax <= FAST_BEXP_HI);
}

// thresholds: "at or below the window" = u <= fma(lo_g, |a|, c_lo), "above
// the window" = u > fma(hi_g, |a|, c_hi)
struct FastBounds {
  double lo_g, c_lo, hi_g, c_hi;
};
__device__ __forceinline__ FastBounds fast_bounds(uint64_t plo, uint64_t phi) {
  constexpr double TINY = 0x1p-1074;
  FastBounds f{0.0, 0.0, 0.0, 0.0};
  if (plo == 0) {
    f.c_lo = -__builtin_inf();                      // nothing at or below
  } else if (plo == KEY_ZERO - 1) {
    f.c_lo = -TINY;                                  // every negative ratio
  } else {
    const double lo = ratio_of_key(plo);
    f.lo_g = lo - fabs(lo) * 0x1p-49;
  }
  if (phi == KEY_NONE - 1) {
    f.c_hi = __builtin_inf();                        // nothing above
  } else if (phi == KEY_ZERO - 1) {
    f.c_hi = -TINY;                                  // every ratio >= 0
  } else {
    const double hi = ratio_of_key(phi);
    f.hi_g = hi + fabs(hi) * 0x1p-49;
  }
  return f;
}

// floor(x / 2^e0) for a finite x >= 0 below 2^(e0 + 127)
__device__ __forceinline__ u128 fixed_floor(double x, int e0) {
  return x > 0.0 ? fixed_of(x, e0) : (u128)0;
}

// The fast pass over the rows of segment (j, k) for the window (plo, phi]:
// lk / lr receive the window's elements in row order (count nwin; nwin >
// lcap reports an overflow, the list then unusable), and [SA, SB] brackets
// the exact weight of the elements at or below the window (units 2^e0).
template <class LdJ, class LdK>
__device__ __forceinline__ void fast_window_pass(const SegIO &s, LdJ ldj, LdK ldk, uint64_t plo, uint64_t phi,
                                                 uint64_t *lk, unsigned short *lr, int lcap, int &nwin, u128 &SA,
                                                 u128 &SB) {
  const FastBounds f = fast_bounds(plo, phi);
  const int lane = s.lane, T = s.T;
  double S = 0.0;
  int nc = 0;
  // rows in batches of FB slots, every load of a batch issued before the
  // first is used (one slot at a time left the wave waiting on L2 latency)
  constexpr int FB = 4;
  // batch t0's loads are issued while batch t0 - FB is classified
  auto load_batch = [&](int t0, double *av, double *bv) {
    if (t0 + FB <= T) {
      // a whole batch (every one at 2000 rows): no per-slot guard
#pragma unroll
      for (int r = 0; r < FB; ++r) {
        const int i = lane + 64 * (t0 + r);
        av[r] = ldj(i);
        bv[r] = ldk(i);
      }
    } else {
#pragma unroll
      for (int r = 0; r < FB; ++r) {
        const int i = lane + 64 * (t0 + r);
        const bool in = t0 + r < T;
        av[r] = in ? ldj(i) : 0.0;
        bv[r] = in ? ldk(i) : 0.0;
      }
    }
  };
  double an[FB], bn[FB];
  load_batch(0, an, bn);
  for (int t0 = 0; t0 < T; t0 += FB) {
    double av[FB], bv[FB];
#pragma unroll
    for (int r = 0; r < FB; ++r) {
      av[r] = an[r];
      bv[r] = bn[r];
    }
    if (t0 + FB < T) load_batch(t0 + FB, an, bn);
#pragma unroll
    for (int r = 0; r < FB; ++r) {
      const int i = lane + 64 * (t0 + r);
      const double a = av[r], b = bv[r];
      const double aa = fabs(a);
      const double u =
          __longlong_as_double(__double_as_longlong(b) ^ (__double_as_longlong(a) & (long long)KEY_ZERO));
      const bool valid = a != 0.0;
      const bool below = valid && u <= fma(f.lo_g, aa, f.c_lo);
      const bool above = u > fma(f.hi_g, aa, f.c_hi);
      S = fma(aa, below ? 1.0 : 0.0, S);
      const bool cand = valid && !below && !above;
      const uint64_t cm = __ballot(cand);
      const int pos = nc + lanes_below(cm);
      nc += __builtin_popcountll(cm);
      if (cand && pos < lcap) lr[pos] = (unsigned short)i;
    }
  }
  nc = uni_int(nc);
  wave_lds_sync();
  int nw = 0;
  if (nc <= lcap) {
    // exact keys of the listed rows, GB slots of gathers in flight; the
    // window's elements are compacted to the front (an entry never moves
    // above its own slot, and a batch is read before it is written)
    constexpr int GB = 4;
    for (int e0 = 0; e0 < nc; e0 += 64 * GB) {
      int rows[GB];
      double av[GB], bv[GB];
#pragma unroll
      for (int r = 0; r < GB; ++r) {
        const int e = e0 + 64 * r + lane;
        rows[r] = e < nc ? (int)lr[e] : -1;
      }
#pragma unroll
      for (int r = 0; r < GB; ++r) {
        const int row = rows[r] < 0 ? 0 : rows[r];
        av[r] = sxj_at(s, row);
        bv[r] = gld(s.xk + row);
      }
#pragma unroll
      for (int r = 0; r < GB; ++r) {
        const bool in = rows[r] >= 0;
        const uint64_t key = key_of_pair(in, av[r], bv[r]);
        const bool le = in && key <= plo;
        const bool inw = in && key > plo && key <= phi;
        S = fma(fabs(av[r]), le ? 1.0 : 0.0, S);
        const uint64_t wm = __ballot(inw);
        const int pos = nw + lanes_below(wm);
        nw += __builtin_popcountll(wm);
        if (inw) {
          lk[pos] = key;
          lr[pos] = (unsigned short)rows[r];
        }
      }
    }
    nw = uni_int(nw);
  } else {
    nw = nc;                                         // overflow
  }
  wave_lds_sync();
  nwin = nw;
  // FP64 sum of nonnegative terms: each lane adds at most T + ceil(nc / 64)
  // terms in sequence, then six tree levels; the error is below
  // (terms + 8) 2^-52 of the sum
  const double St = wave_sum_dbl_x(S);
  const double dlt = (double)(T + ((min(nc, lcap) + 63) >> 6) + 8) * 0x1p-52 * St;
  SA = fixed_floor(St - dlt, s.e0);
  SB = fixed_floor(St + dlt, s.e0) + 1;
}

// Probe point of a window (plo, phi] that holds more elements than the
// list: the middle one of the sample keys inside it, or with none inside the
// key halfway between its ends (when both are keys of finite ratios).  Any
// key inside the window serves: it only steers where the next exact listing
// pass looks.
// The sorted sample (128 top-32-bit keys, packed in pairs) is read from smp
// in LDS.
// false: no key strictly inside the window was found.
// sample key ix (top 32 bits, times 2^32) of a sorted sample stored as
// packed pairs: entry l holds keys 2 l (low half) and 2 l + 1 (high half)
__device__ __forceinline__ uint64_t sample_key(const uint64_t *smp, int ix) {
  const uint64_t w = smp[ix >> 1];
  return (ix & 1) ? (w & 0xFFFFFFFF00000000ull) : (w << 32);
}

__device__ __forceinline__ int sample_count(const uint64_t *smp, uint64_t bound, bool strict) {
  // sample keys at or below bound (strict: below); the keys ascend
  int lo = 0;
#pragma unroll
  for (int step = 64; step >= 1; step >>= 1) {
    const uint64_t k = sample_key(smp, lo + step - 1);
    if (strict ? k < bound : k <= bound) lo += step;
  }
  return lo;
}

__device__ __forceinline__ bool window_midpoint(const uint64_t *smp, uint64_t plo, uint64_t phi, uint64_t &mid) {
  const int i0 = sample_count(smp, plo, false), i1 = sample_count(smp, phi, true);
  if (i1 > i0) {
    mid = sample_key(smp, (i0 + i1) >> 1);
    return true;
  }
  // the keys of the finite doubles form one interval, [key(-inf), key(+inf)]
  constexpr uint64_t KEY_NEG_INF = 0x000FFFFFFFFFFFFFull, KEY_POS_INF = 0xFFF0000000000000ull;
  if (plo < KEY_NEG_INF || phi > KEY_POS_INF) return false;
  mid = plo + ((phi - plo) >> 1);
  return mid > plo;
}

// The side of the minimiser of segment (j, k) at penalty lam from the sign
// sums dz = (D_jk, Zr_jk): 0 when 0 minimises g_jk, 1 negative, 2 positive,
// 3 undecided (the exact pass decides).  Decision margin 2^-32 (W_j + lam):
// far above the rounding error of the sign sums (at most ~n 2^-52 of W_j,
// plus n 2^-1022 should the matrix unit flush subnormal terms: hence the
// floor on the margin).  unc: the sums cannot be trusted for this segment.
__device__ __forceinline__ int sign_sum_side(double2 dz, double lam, double Wj, bool unc) {
  const double M = 0x1p-32 * (Wj + lam);
  const double d1 = lam + dz.y + dz.x;               // >= 0  <=>  2A <= W + lambda
  const double d2 = lam + dz.y - dz.x;               // >= 0  <=>  W <= 2B + lambda
  if (unc || !(M >= 0x1p-1000)) return 3;
  if (d1 > M && d2 > M) return 0;
  if (d1 < -M) return 1;
  if (d2 < -M) return 2;
  return 3;
}

// The sign sums cannot decide segment (j, k) when a ratio could underflow to
// 0 (exponent fields more than 1000 apart) or a sum is not finite.
__device__ __forceinline__ bool sign_sums_unsure(const ColInfo &cj, const ColInfo &ck, double2 dz) {
  const bool maybe_tiny = ck.nnz > 0 && cj.nnz > 0 && ck.bemin - cj.bemax < -1000;
  return maybe_tiny || !isfinite(dz.x) || !isfinite(dz.y);
}

// Segments settled by the sign sums alone.  One thread per pair (j, k), one
// wave per 64 consecutive k of a preserved column: where every penalty of the
// problem has 0 as a minimiser (sign_sum_side, the segment kernel's own test),
// writes v_k = 0, e_jk = the R64 mass of column k, row -1 for every penalty
// and sets bit k & 63 of mask word (jj, k >> 6); the segment kernel skips such
// segments.  wstart[b] = first mask word of problem b (mj ceil(m / 64) words,
// mj = ncand with a candidate list, problem 0 only, else m).
__global__ void __launch_bounds__(256)
k_zero_segments(const ProbDesc *__restrict__ P, const int *__restrict__ wstart, int B, int total_words,
                const double *__restrict__ lam_all, const ColInfo *__restrict__ ci,
                const double2 *__restrict__ DZ, double *__restrict__ V, double *__restrict__ E,
                int *__restrict__ R, unsigned long long *__restrict__ mask, const int *__restrict__ cand,
                const int *__restrict__ gate, int gate_on) {
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w >= total_words) return;
  if (gate && *gate != gate_on) return;
  const int b = find_owner(wstart, B, w);
  const ProbDesc d = P[b];
  const int wpr = (d.m + 63) >> 6;
  const int wl = w - wstart[b];
  const int jj = wl / wpr, k = (wl - jj * wpr) * 64 + lane;
  const int j = cand ? cand[jj] : jj;
  bool skip = false;
  if (k < d.m && k != j) {
    const ColInfo cj = ci[d.col_off + j], ck = ci[d.col_off + k];
    if (!cj.flags && !ck.flags) {
      const double2 dz = DZ[d.pair_off + (long long)j * d.m + k];
      const bool unc = sign_sums_unsure(cj, ck, dz);
      const double *lam = lam_all + d.lam_off;
      skip = true;
      for (int t = 0; t < d.L && skip; ++t) skip = sign_sum_side(dz, lam[t], cj.W, unc) == 0;
      if (skip) {
        const long long mm = (long long)d.m * d.m, base = d.ws_off + (long long)j * d.m + k;
        for (int t = 0; t < d.L; ++t) {
          V[base + t * mm] = 0.0;
          E[base + t * mm] = ck.W;
          R[base + t * mm] = -1;
        }
      }
    }
  }
  const unsigned long long bits = __ballot(skip);
  if (lane == 0) mask[d.mask_off + wl] = bits;
}

// exact A (negative ratios), B (non-positive), counts, one sample per side
struct ExactSides {
  u128 A, B;
  int N, Z, NV;
};

__device__ __forceinline__ ExactSides exact_sides(const SegIO &s) {
  u128 a128 = 0, z128 = 0;
  int cN = 0, cZ = 0, cV = 0;
#pragma unroll 2
  for (int tt = 0; tt < s.T; ++tt) {
    const int i = s.lane + 64 * tt;
    const uint64_t key = seg_key(s, i);
    const bool valid = key != KEY_NONE;
    const u128 w = seg_weight(s, i, valid);
    const bool neg = key < KEY_ZERO, zer = key == KEY_ZERO;
    a128 += neg ? w : (u128)0;
    z128 += zer ? w : (u128)0;
    cN += neg ? 1 : 0;
    cZ += zer ? 1 : 0;
    cV += valid ? 1 : 0;
  }
  ExactSides e;
  e.A = wave_sum_u128(a128);
  e.B = e.A + wave_sum_u128(z128);
  e.N = wave_sum_int(cN);
  e.Z = wave_sum_int(cZ);
  e.NV = wave_sum_int(cV);
  return e;
}

// Selection of one target from the division-free pass's window list in
// FP64.  The list holds the window's elements (row order, count nwin); the
// exact weight below the window lies in [SA, SB] (units 2^e0); tau is the
// target's threshold (same units): the answer is the first element, in
// (key, row) order, at which the weight below the window plus the list's
// prefix reaches tau -- what the exact selection finds.  Here the weights
// |x_ij| are summed in FP64.  Every value compared is a sum of nonnegative
// weights of column j or a difference of such sums, at most W_j, reached
// through at most 40 roundings (list sums: 8 per lane and 6 tree levels;
// 128-bit values converted with 3; the walk's running sum), so it lies
// within 40 u W_j of its exact value (u = 2^-53).  A comparison whose
// operands differ by more than tol = 2^-38 W_j (2^15 u W_j) therefore has
// the exact comparison's outcome; a closer one sets amb, and the caller
// redoes the segment with the exact pass.  Live segments have lambda < W_j,
// so tau is at most W_j.  Lists over 128 elements are first cut at three
// sample keys (piv, ascending) to the part that holds the target, as the
// exact path does.
__device__ __forceinline__ void select_one_fp64(const SegIO &s, uint64_t *lk, unsigned short *lr, int &nwin,
                                                int lane, u128 SA, u128 SB, u128 tau, double Wd,
                                                const uint64_t *piv, uint64_t &okey, int &orow, bool &hit,
                                                bool &amb) {
  const double tol = 0x1p-38 * Wd;
  // tau - (weight below the list) at both ends of the interval, in the
  // column's own units; 0 when tau is at or below it (exactly known)
  auto real_of = [&](u128 x) { return ldexp(u128_to_double_approx(x), s.e0); };
  double DA = tau > SA ? real_of(tau - SA) : 0.0, DB = tau > SB ? real_of(tau - SB) : 0.0;
  bool und = false;
  if (nwin > 128) {
    const uint64_t p0 = piv[0], p1 = piv[1] < p0 ? p0 : piv[1], p2 = piv[2] < p1 ? p1 : piv[2];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int e = lane; e < nwin; e += 64) {
      const uint64_t key = lk[e];
      const double w = fabs(sxj_at(s, lr[e]));
      a0 = a0 + (key < p0 ? w : 0.0);
      a1 = a1 + (key < p1 ? w : 0.0);
      a2 = a2 + (key < p2 ? w : 0.0);
    }
    a0 = wave_sum_dbl_x(a0);
    a1 = wave_sum_dbl_x(a1);
    a2 = wave_sum_dbl_x(a2);
    // parts below the target: pivots p with (weight below p) < D
    auto below = [&](double D) {
      const double d0 = a0 - D, d1 = a1 - D, d2 = a2 - D;
      und = und || fabs(d0) <= tol || fabs(d1) <= tol || fabs(d2) <= tol;
      return (d0 < 0.0 ? 1 : 0) + (d1 < 0.0 ? 1 : 0) + (d2 < 0.0 ? 1 : 0);
    };
    const int c = below(DA), cB = below(DB);
    if (und || c != cB) {
      amb = true;
      return;
    }
    const uint64_t plo2 = c == 0 ? 0 : (c == 1 ? p0 : (c == 2 ? p1 : p2)), phi2 = c == 0 ? p0 : (c == 1 ? p1 : p2);
    const double base = c == 0 ? 0.0 : (c == 1 ? a0 : (c == 2 ? a1 : a2));
    // (c > 0: base < D by more than tol at both ends, so both stay positive)
    DA = DA - base;
    DB = DB - base;
    // stable in-place compaction: an element never moves above its own
    // slot, so slots not yet read are never overwritten
    int kept = 0;
    for (int e0 = 0; e0 < nwin; e0 += 64) {
      const int e = e0 + lane;
      const bool in = e < nwin;
      const uint64_t key = in ? lk[e] : 0;
      const unsigned short row = in ? lr[e] : 0;
      const bool keep = in && (c == 0 || key >= plo2) && (c == 3 || key < phi2);
      const uint64_t km = __ballot(keep);
      const int d = kept + lanes_below(km);
      kept += __builtin_popcountll(km);
      if (keep) {
        lk[d] = key;
        lr[d] = row;
      }
    }
    nwin = uni_int(kept);
    wave_lds_sync();
  }
  const int N = wave_sort_list(lk, lr, nwin, lane);
  const int E = N >> 6;
  // lane l owns the sorted entries [E l, E l + E)
  double tot = 0.0;
  for (int q = 0; q < E; ++q) {
    const int e = E * lane + q;
    const bool valid = lk[e] != KEY_NONE;
    tot = tot + (valid ? fabs(sxj_at(s, lr[e])) : 0.0);
  }
  const double incl = wave_incl_scan_dbl_x(tot, lane);
  // the search at the lower end of [SA, SB] (D = DA); the upper end (DB <=
  // DA) is then checked by one comparison: the found entry stays the first
  // to reach DB iff the weight before it is below DB, and a miss above the
  // list stays one iff the list's total is below DB
  auto find = [&](double D, uint64_t &k, int &r, double &prev) -> bool {
    if (!(D > 0.0)) return false;                  // tau at or below the list
    const double df = incl - D;
    und = und || __ballot(fabs(df) <= tol) != 0;
    const uint64_t owner = __ballot(df >= 0.0);
    if (owner == 0) return false;                  // above the list
    const int lo = __builtin_ctzll(owner);
    double run = readlane_dbl(incl, lo) - readlane_dbl(tot, lo);
    for (int q = 0; q < E; ++q) {
      const int e = E * lo + q;
      const uint64_t key = lk[e];
      if (key == KEY_NONE) break;
      prev = run;
      run = run + fabs(sxj_at(s, lr[e]));
      const double d = run - D;
      und = und || fabs(d) <= tol;
      if (d >= 0.0) {
        k = key;
        r = (int)lr[e];
        return true;
      }
    }
    und = true;                                    // (the owner's entries must reach D)
    return false;
  };
  uint64_t kA = KEY_NONE;
  int rA = -1;
  double prevA = 0.0;
  const bool hA = find(DA, kA, rA, prevA);
  if (DB != DA) {
    if (hA) {
      // (DB > 0 is exactly known: DB = 0 means tau is at or below SB)
      und = und || (DB > 0.0 && fabs(prevA - DB) <= tol);
      amb = amb || !(DB > 0.0 && prevA - DB < 0.0);
    } else if (DA > 0.0) {
      const double d = readlane_dbl(incl, 63) - DB;
      und = und || fabs(d) <= tol;
      amb = amb || d >= 0.0;
    }
  }
  amb = amb || und;
  okey = kA;
  orow = rA;
  hit = hA;
}

// One work item, by the whole workgroup (every thread calls it).  ci, V, E,
// R and segflags are this problem's slices.  kLdsJ: column j is copied to LDS
// (the pointer's address space is then known to the compiler: LDS loads).
template <bool kLdsJ, bool kMulti>
__device__ __forceinline__ void seg_item(const double *__restrict__ X, int n, int m, long long ld,
                                         const ColInfo *__restrict__ ci, const double *__restrict__ lam, int L,
                                         const double2 *__restrict__ DZ, int j, int kbeg, int kend,
                                         double *__restrict__ V,
                                         double *__restrict__ E, int *__restrict__ R, int *__restrict__ segflags,
                                         const unsigned long long *__restrict__ maskrow, int lcap, int sxj_rows,
                                         unsigned char *smem) {
  const int T = (n + 63) >> 6;
  // penalties: the single-penalty instantiation has exactly one (one group,
  // one pass, trip counts the compiler sees)
  const int Lg = kMulti ? L : 1;
  // column j in LDS when the launch reserved room for it (n <= sxj_rows),
  // else read from global memory (it stays in L2 across the item's k)
  constexpr bool lds_j = kLdsJ;
  (void)sxj_rows;
  double *sxj_lds = (double *)smem;                 // T*64 entries, zero padded
  int *srow = (int *)(smem + (lds_j ? seg_sxj_bytes(n) : 0));
  u128 *slam = (u128 *)(srow + SAMPLE_ROWS);
  WaveScratch *wsc = (WaveScratch *)(slam + L);
  uint64_t *lkeys = (uint64_t *)(wsc + SEG_WAVES);
  unsigned short *lrows = (unsigned short *)(lkeys + (size_t)SEG_WAVES * lcap);
  int *knext = (int *)(lrows + (size_t)SEG_WAVES * lcap);

  const ColInfo cj = ci[j];
  const double *xjg = X + (long long)j * ld;
  if constexpr (kLdsJ)
    for (int i = threadIdx.x; i < T * 64; i += blockDim.x) sxj_lds[i] = i < n ? xjg[i] : 0.0;
  const double *__restrict__ sxj = kLdsJ ? (const double *)sxj_lds : xjg;
  for (int t = threadIdx.x; t < L; t += blockDim.x) slam[t] = lambda_fixed(lam[t], cj.e0);
  if (threadIdx.x == 0) *knext = 0;
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the item's live segments: k in [kbeg, kend) not settled by
  // k_zero_segments.  Lane l holds word l of the item's mask inverted (bit b:
  // segment 64 (w0 + l) + b is live) and the live count of the words below
  // it; the waves claim live segments by their rank, so settled ones cost no
  // claim.  Without the mask every segment of the range is live.
  const int w0 = kbeg >> 6, nwords = kend > kbeg ? ((kend - 1) >> 6) - w0 + 1 : 0;
  const bool use_mask = maskrow != nullptr && nwords <= SEG_MASK_WORDS;
  uint64_t live = 0;
  int kpre = 0, nlive = kend - kbeg;
  if (use_mask) {
    if (lane < nwords) {
      const int lo = max(kbeg - 64 * (w0 + lane), 0), hi = min(kend - 64 * (w0 + lane), 64);
      const uint64_t range = (hi == 64 ? ~0ull : (1ull << hi) - 1ull) & ~((1ull << lo) - 1ull);
      live = ~maskrow[w0 + lane] & range;
    }
    const int cnt = __builtin_popcountll(live);
    kpre = wave_excl_scan_int(cnt, lane);
    nlive = uni_int(__shfl(kpre + cnt, 63));
  }
  if (wave == 0) {
    // systematic sample of SAMPLE_ROWS rows with probability ~ |x_ij|: the
    // cumulative weight runs over the rows in order, 64 rows (one per lane)
    // at a time; sample r is the row whose weight interval holds (r + 1/2)
    // step.  Consecutive lanes read consecutive rows (no LDS bank conflicts).
    auto wt = [&](int i) {
      const double a = sxj[i < n ? i : 0];
      return i < n ? fabs(a) : 0.0;
    };
    double part = 0.0;
    for (int t = 0; t < T; ++t) part = part + wt(lane + 64 * t);
    const double all = wave_sum_dbl_x(part);
    for (int r = lane; r < SAMPLE_ROWS; r += 64) srow[r] = -1;
    wave_lds_sync();
    if (all > 0.0) {
      const double step = all / SAMPLE_ROWS;
      double base = 0.0;
      for (int t = 0; t < T; ++t) {
        const int i = lane + 64 * t;
        const double w = wt(i);
        const double incl = base + wave_incl_scan_dbl_x(w, lane);
        const double cum = incl - w;
        int r = (int)ceil(cum / step - 0.5);
        r = r < 0 ? 0 : r;
        for (; w > 0.0 && r < SAMPLE_ROWS && (r + 0.5) * step < incl; ++r) srow[r] = i;
        base = readlane_dbl(incl, 63);
      }
    }
    wave_lds_sync();
    // samples no row took (rounding at the end) repeat the nearest earlier
    // sample, or the column's first nonzero row; sampled rows increase with
    // r (an inclusive max-scan over the entries, two per lane, finds that
    // row), and any row with x_ij != 0 would do
    int first = 0;
    for (int t = 0; t < T; ++t) {
      const uint64_t nzm = __ballot(wt(lane + 64 * t) != 0.0);
      if (nzm) {
        first = 64 * t + __builtin_ctzll(nzm);
        break;
      }
    }
    const int s0 = srow[2 * lane], s1 = srow[2 * lane + 1];
    const int c1 = max(s0, s1);
    int tot = c1, x = c1;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int o = (int)xswap32((uint32_t)tot, d);
      x = (lane & d) ? max(x, o) : x;
      tot = max(tot, o);
    }
    // (x: the largest row over entries [0, 2 lane + 2); prev: over [0, 2 lane))
    const int up1 = __shfl_up(x, 1);
    const int prev = lane > 0 ? up1 : -1;
    const int e0 = max(prev, s0), e1 = max(e0, s1);
    wave_lds_sync();
    srow[2 * lane] = e0 >= 0 ? e0 : first;
    srow[2 * lane + 1] = e1 >= 0 ? e1 : first;
  }
  __syncthreads();

  WaveScratch *ws = wsc + wave;
  uint64_t *lk = lkeys + (size_t)wave * lcap;
  unsigned short *lr = lrows + (size_t)wave * lcap;
  const long long mm = (long long)m * m;
  const double Wd = cj.W;
  int Tp = 1;
  while (Tp < T) Tp <<= 1;
  int err = 0;

  // claims are taken one segment ahead, so the counter's round trip overlaps
  // the current segment (claims only grow: once one is past the live count,
  // so is every later one)
  int claim = 0;
  if (lane == 0) claim = atomicAdd(knext, 1);
  while (true) {
    const int c = __builtin_amdgcn_readlane(claim, 0);
    if (c >= nlive) break;
    if (lane == 0) claim = atomicAdd(knext, 1);
    int k = kbeg + c;
    if (use_mask) {
      // the c-th live segment: the last word whose live prefix is <= c, then
      // the (c - prefix)-th set bit of that word
      const int w = __builtin_popcountll(__ballot(lane < nwords && kpre <= c)) - 1;
      const uint64_t lw = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(live >> 32), w) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)live, w);
      const int r = c - __builtin_amdgcn_readlane(kpre, w);
      k = 64 * (w0 + w) + __builtin_ctzll(__ballot(((lw >> lane) & 1ull) && lanes_below(lw) == r));
    }
    const long long base = (long long)j * m + k;
    if (k == j || cj.flags) {
      if (lane == 0) {
        for (int t = 0; t < Lg; ++t) {
          V[t * mm + base] = (k == j) ? 1.0 : __longlong_as_double(0x7ff8000000000000ll);
          E[t * mm + base] = 0.0;
          R[t * mm + base] = -1;
        }
      }
      continue;
    }
    const ColInfo ck = ci[k];
    const SegIO s{X + (long long)k * ld, sxj, n, T, Tp, cj.e0, lane, kLdsJ};
    const double Wk = ck.W;
    const bool fast_seg = fast_columns(cj) && fast_columns(ck);

    // 1. sign sums.  |x_ik / x_ij| can underflow to 0 only if the exponent
    // fields differ by more than 1000: the column ranges rule that out for the
    // whole segment in the usual case, else the exact pass decides.
    const double2 dz = DZ[(long long)j * m + k];
    const bool unc = sign_sums_unsure(cj, ck, dz);

    bool have_exact = false;
    ExactSides ex;
    const u128 W = cj.wfix;
    // (a) the side of every penalty: v_k = 0, or the minimiser is negative
    // (1) or positive (2).  A <= B makes the nonzero side the same for every
    // penalty of the segment.
    uint64_t nz0 = 0, nz1 = 0;                     // bit t: v_k != 0 at penalty t
    int sd = 0;
    if constexpr (kMulti) {
      // one penalty per lane, in groups of 64
      for (int g0 = 0; g0 < L; g0 += 64) {
        const int t = g0 + lane;
        const bool in = t < L;
        int side = 0;
        if (in) side = sign_sum_side(dz, lam[t], Wd, unc);
        if (__ballot(side == 3)) {
          if (!have_exact) {
            ex = exact_sides(s);
            have_exact = true;
          }
          if (side == 3) {
            const u128 lamf = slam[t], WpL = W + lamf;
            side = ((ex.A << 1) <= WpL && W <= (ex.B << 1) + lamf) ? 0 : ((ex.A << 1) > WpL ? 1 : 2);
          }
        }
        const uint64_t nzm = __ballot(side != 0);
        if (g0 == 0) nz0 = nzm;
        else nz1 = nzm;
        // every nonzero penalty has the same side (A <= B)
        if (nzm) sd = __builtin_amdgcn_readlane(side, __builtin_ctzll(nzm));
      }
    } else {
      for (int t = 0; t < Lg; ++t) {
        int side = sign_sum_side(dz, lam[t], Wd, unc);
        if (side == 3) {
          if (!have_exact) {
            ex = exact_sides(s);
            have_exact = true;
          }
          const u128 lamf = slam[t], WpL = W + lamf;
          side = ((ex.A << 1) <= WpL && W <= (ex.B << 1) + lamf) ? 0 : ((ex.A << 1) > WpL ? 1 : 2);
        }
        if (side) {
          sd = side;
          if (t < 64) nz0 |= 1ull << t;
          else nz1 |= 1ull << (t - 64);
        }
      }
    }
    if ((nz0 | nz1) == 0) {
      // v_k = 0 at every penalty: e_jk = R64 sum of |x_ik|
      for (int t = lane; t < Lg; t += 64) {
        V[t * mm + base] = 0.0;
        E[t * mm + base] = Wk;
        R[t * mm + base] = -1;
      }
      continue;
    }
    const bool neg = sd == 1;
    const uint64_t klo0 = neg ? 0ull : KEY_ZERO, khi0 = neg ? KEY_ZERO - 1 : KEY_NONE - 1;
    // the sample's keys (top 32 bits), sorted across the wave
    uint32_t sa = sample_key32(s, srow[lane]), sb = sample_key32(s, srow[lane + 64]);
    wave_sort2_u32_x(sa, sb, lane);
    // one penalty: the sorted sample (index 2 l + c in lane l) goes to the
    // wave's LDS scratch, free until the rounds after the window (several:
    // the rounds between groups reuse that area, so it stays in registers)
    if constexpr (!kMulti) {
      ws->ckey[lane] = ((uint64_t)sb << 32) | sa;
      wave_lds_sync();
    }
    // sample position ix as a lower or upper key bound
    auto sample_lo = [&](int ix) {
      if constexpr (!kMulti) return sample_key(ws->ckey, ix);
      return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)((ix & 1) ? sb : sa), ix >> 1)) << 32;
    };
    auto sample_hi = [&](int ix) { return sample_lo(ix) | 0xFFFFFFFFull; };
    int prev_row = -2;
    double prev_e = 0.0;
    // penalties in groups of 64, lane l holding the target of penalty 64 g + l
    for (int g = 0; 64 * g < Lg; ++g) {
      const uint64_t nzg = g ? nz1 : nz0;
      const int tl = 64 * g + lane;
      const bool act = ((nzg >> lane) & 1ull) != 0;
      // negative side: first S_p > (W + lambda)/2; positive: first S_p >= (W - lambda)/2
      double q = 2.0;
      if (act) {
        const double lamt = lam[tl];
        q = (neg ? 0.5 * (Wd + lamt) : 0.5 * (Wd - lamt)) / Wd;
      }
      // window bounds on the targets' weight fractions (positive doubles
      // order as their bit patterns)
      double qmin, qmax;
      if constexpr (!kMulti) {
        // one penalty: lane 0's target (no cross-lane reduction)
        qmin = qmax = __longlong_as_double((long long)uni_u64((uint64_t)__double_as_longlong(fmax(q, 0.0))));
      } else {
        qmin = __longlong_as_double((long long)wave_min_u64_x((uint64_t)__double_as_longlong(fmax(q, 0.0))));
        qmax = __longlong_as_double((long long)wave_max_u64_x((uint64_t)__double_as_longlong(act ? fmax(q, 0.0) : 0.0)));
      }
      uint64_t okey = KEY_NONE;
      int orow = -1;
      bool hit = false;
      // the ratios of the weighted row sample bracket the targets: a key
      // window; one exact pass lists the window's elements, one sort serves
      // every penalty.  A window too wide for the list is retried per penalty.
      for (int pass = 0; nzg && pass <= (kMulti ? 64 : 0); ++pass) {
        double wlo = qmin, whi = qmax;
        bool mine = act;
        if (pass > 0) {
          const int t = pass - 1;
          if (!((nzg >> t) & 1ull) || __builtin_amdgcn_readlane((int)hit, t)) continue;
          wlo = whi = readlane_dbl(q, t);
          mine = lane == t;
        }
        constexpr double WDELTA = 0.08;
        const int ilo = (int)floor((wlo - WDELTA) * SAMPLE_ROWS) - 1;
        const int ihi = (int)ceil((whi + WDELTA) * SAMPLE_ROWS);
        uint64_t plo = klo0, phi = khi0;
        if (ilo >= 0 && ilo < SAMPLE_ROWS) {
          const uint64_t v = sample_lo(ilo);
          plo = v > plo ? v : plo;
        }
        if (ihi >= 0 && ihi < SAMPLE_ROWS) {
          const uint64_t v = sample_hi(ihi);
          phi = v < phi ? v : phi;
        }
        if (plo > khi0) plo = khi0;
        if (phi < plo) phi = plo;

        const __amdgpu_buffer_rsrc_t rk = col_rsrc(s.xk, n), rj = col_rsrc(s.lds ? s.xk : s.sxj, n);
        // columns read through the range-checked descriptor (0 past row n)
        // or the zero-padded LDS copy: no clamps
        auto ldjp = [&](int i) { return sxj_pad(s, rj, i); };
        auto ldkp = [&](int i) { return col_ld(rk, i * 8); };
        // the division-free pass first; the exact pass when the columns'
        // ranges rule the fast one out, or when the weight below the window,
        // known from it only within an interval, leaves the selection open
        bool use_fast = fast_seg;
        bool ovf = false;
        bool probe = false;
        ws->steps = 0;
        while (true) {
          int nwin = 0;
          u128 SlwA, SlwB;
          if (use_fast) {
            fast_window_pass(s, ldjp, ldkp, plo, phi, lk, lr, lcap, nwin, SlwA, SlwB);
          } else {
            // exact pass: weight at or below the window; the window's
            // elements go to the LDS list (in row order).  The weight below
            // the window in three FP64 sums of 37-bit chunks (whole numbers
            // below 2^53: every add is exact)
            double c0s = 0.0, c1s = 0.0, c2s = 0.0;
            // columns j and k are read one slot ahead so the loads overlap
            // the divide; the weight reuses x_ij (one penalty: rows past n
            // read 0, key NONE and no weight; several: clamped to row 0,
            // which spills less there)
            auto ldj = [&](int i) { return kMulti ? sxj_at(s, i < n ? i : 0) : ldjp(i); };
            auto ldk = [&](int i) { return kMulti ? gld(s.xk + (i < n ? i : 0)) : ldkp(i); };
            double anext = ldj(lane), bnext = ldk(lane);
            for (int tt = 0; tt < T; ++tt) {
              const int i = lane + 64 * tt;
              const double a = anext, b = bnext;
              if (tt + 1 < T) {
                anext = ldj(i + 64);
                bnext = ldk(i + 64);
              }
              const uint64_t key = key_of_pair(i < n, a, b);
              const bool valid = key != KEY_NONE;
              const bool le_lo = valid && key <= plo;
              const bool inwin = valid && key > plo && key <= phi;
              {
                double c0, c1, c2;
                weight_chunks(a, s.e0, c0, c1, c2);
                // masked adds as fma with a 0/1 factor: the same exact sums
                // (whole numbers below 2^53; c 0 adds +0), one op each
                const double fl = le_lo ? 1.0 : 0.0;
                c0s = fma(c0, fl, c0s);
                c1s = fma(c1, fl, c1s);
                c2s = fma(c2, fl, c2s);
              }
              const uint64_t wm = __ballot(inwin);
              const int pos = nwin + lanes_below(wm);
              nwin += __builtin_popcountll(wm);
              if (inwin && pos < lcap) {
                lk[pos] = key;
                lr[pos] = (unsigned short)i;
              }
            }
            SlwA = SlwB = chunks_to_u128(wave_sum_dbl_x(c0s), wave_sum_dbl_x(c1s), wave_sum_dbl_x(c2s));
            nwin = uni_int(nwin);
            wave_lds_sync();
          }
          const u128 lamf = act ? slam[tl] : (u128)0;
          const u128 tau = neg ? ((W + lamf) >> 1) + 1 : (W - lamf + 1) >> 1;
          if (!kMulti && use_fast && (probe || nwin > lcap)) {
            // one target and division-free classes: a window too full for
            // the list is bisected.  (blo, phi] holds the target and about
            // bcnt elements; a probe pass over (plo, phi], plo inside it,
            // gives the weight at or below plo, which names the half.
            const uint64_t tm = __ballot(mine && !hit);
            if (__builtin_popcountll(tm) == 1 && ws->steps < 12) {
              const bool at_or_below = readlane_u128(tau, __builtin_ctzll(tm)) <= SlwA;
              bool more = true;
              if (!probe) {
                // the window itself: the target at or below it is a miss
                if (at_or_below) {
                  ovf = true;
                  break;
                }
                ws->blo = plo;
                ws->bcnt = nwin;
              } else if (at_or_below) {
                // at or below the probe point: (blo, plo], not listed yet
                ws->bcnt -= nwin;
                phi = plo;
                plo = ws->blo;
              } else {
                ws->blo = plo;
                ws->bcnt = nwin;
                more = nwin > lcap;
              }
              probe = false;
              if (more) {
                ws->steps += 1;
                if (ws->bcnt <= lcap) continue;      // list (blo, phi] in one pass
                uint64_t mid;
                if (!window_midpoint(ws->ckey, plo, phi, mid)) {
                  ovf = true;
                  break;
                }
                plo = mid;
                probe = true;
                continue;
              }
            }
            probe = false;
          }
          if (nwin > lcap) {
            ovf = true;
            break;
          }
          const bool want = mine && !hit;
          const uint64_t wantm = __ballot(want);
          u128 SloA = SlwA, SloB = SlwB;
          bool amb = false;
          if constexpr (!kMulti) {
            if (use_fast) {
              // one target after the division-free pass: the rest in FP64
              // with rigorous margins (a close call is redone exactly)
              uint64_t piv[3];
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                int ix = (int)floor((wlo + 0.04 * (c - 1)) * SAMPLE_ROWS);
                ix = ix < 0 ? 0 : (ix >= SAMPLE_ROWS ? SAMPLE_ROWS - 1 : ix);
                piv[c] = sample_lo(ix);
              }
              uint64_t k2 = KEY_NONE;
              int r2 = -1;
              bool h2 = false;
              if (wantm & 1ull)
                select_one_fp64(s, lk, lr, nwin, lane, SlwA, SlwB, uni_u128(tau), Wd, piv, k2, r2, h2, amb);
              if (!amb && h2 && lane == 0) {
                okey = k2;
                orow = r2;
                hit = true;
              }
              wave_lds_sync();
              if (!amb) break;
              use_fast = false;
              continue;
            }
          }
          if (__builtin_popcountll(wantm) == 1 && nwin > 128) {
            // one target: only the quarter of the window that holds it is
            // sorted.  Three sample keys around the target split the list;
            // the exact weights below them pick the part (a contiguous range
            // of the sorted order), which is compacted to the list's front.
            const u128 tau1 = uni_u128(shfl_u128(tau, __builtin_ctzll(wantm)));
            uint64_t piv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              int ix = (int)floor((wlo + 0.04 * (c - 1)) * SAMPLE_ROWS);
              ix = ix < 0 ? 0 : (ix >= SAMPLE_ROWS ? SAMPLE_ROWS - 1 : ix);
              piv[c] = sample_lo(ix);
            }
            piv[1] = piv[1] < piv[0] ? piv[0] : piv[1];
            piv[2] = piv[2] < piv[1] ? piv[1] : piv[2];
            u128 a0 = 0, a1 = 0, a2 = 0;
            for (int e = lane; e < nwin; e += 64) {
              const uint64_t key = lk[e];
              const u128 w = fixed_of_col(sxj_at(s, lr[e]), s.e0);
              a0 += key < piv[0] ? w : (u128)0;
              a1 += key < piv[1] ? w : (u128)0;
              a2 += key < piv[2] ? w : (u128)0;
            }
            a0 = wave_sum_u128_x(a0);
            a1 = wave_sum_u128_x(a1);
            a2 = wave_sum_u128_x(a2);
            const int c = (SlwA + a0 < tau1 ? 1 : 0) + (SlwA + a1 < tau1 ? 1 : 0) + (SlwA + a2 < tau1 ? 1 : 0);
            const int cB = (SlwB + a0 < tau1 ? 1 : 0) + (SlwB + a1 < tau1 ? 1 : 0) + (SlwB + a2 < tau1 ? 1 : 0);
            if (c != cB) {
              amb = true;
            } else {
              const uint64_t plo2 = c == 0 ? 0 : piv[c - 1], phi2 = c == 3 ? KEY_NONE : piv[c];
              const u128 ac = c == 0 ? (u128)0 : (c == 1 ? a0 : (c == 2 ? a1 : a2));
              SloA = SlwA + ac;
              SloB = SlwB + ac;
              // stable in-place compaction: an element never moves above its
              // own slot, so slots not yet read are never overwritten
              int kept = 0;
              for (int e0 = 0; e0 < nwin; e0 += 64) {
                const int e = e0 + lane;
                const bool in = e < nwin;
                const uint64_t key = in ? lk[e] : 0;
                const unsigned short row = in ? lr[e] : 0;
                const bool keep = in && (c == 0 || key >= plo2) && (c == 3 || key < phi2);
                const uint64_t km = __ballot(keep);
                const int d = kept + lanes_below(km);
                kept += __builtin_popcountll(km);
                if (keep) {
                  lk[d] = key;
                  lr[d] = row;
                }
              }
              nwin = uni_int(kept);
              wave_lds_sync();
            }
          }
          if (!amb) {
            const int N = wave_sort_list(lk, lr, nwin, lane);
            u128 tot, incl;
            wave_list_sums(s, lk, lr, N >> 6, tot, incl);
            uint64_t k2 = KEY_NONE;
            int r2 = -1;
            bool h2 = false;
            if constexpr (!kMulti) {
              // one penalty: its target sits in lane 0
              if (wantm & 1ull) wave_resolve_one(s, lk, lr, N >> 6, SloA, SloB, tot, incl, uni_u128(tau), k2, r2, h2, amb);
              h2 = h2 && lane == 0;
            } else {
              // the answer must not depend on where in [SloA, SloB] the
              // exact weight below the list lies
              bool amb_l = false;
              wave_resolve(s, lk, lr, N >> 6, SloA, SloB, tot, incl, want, tau, k2, r2, h2, amb_l);
              amb = __ballot(want && amb_l) != 0;
            }
            if (!amb && h2) {
              okey = k2;
              orow = r2;
              hit = true;
            }
          }
          wave_lds_sync();
          if (!amb) break;
          use_fast = false;                          // redo the pass exactly
        }
        if (ovf) {
          // the list cannot hold the window: after the shared window, retry
          // each penalty with its own; a single penalty goes to the rounds
          if (pass == 0 && __builtin_popcountll(nzg) == 1) break;
          continue;
        }
        // the shared window held: the targets it missed go to the rounds
        if (pass == 0) break;
      }

      // targets the windows missed: rounds over the whole side
      uint64_t left = __ballot(act && !hit);
      while (left) {
        const int t = __builtin_ctzll(left);
        left &= left - 1;
        if (!have_exact) {
          ex = exact_sides(s);
          have_exact = true;
        }
        const u128 lamf = slam[64 * g + t];
        const u128 tau = neg ? ((W + lamf) >> 1) + 1 : (W - lamf + 1) >> 1;
        uint64_t k2 = KEY_NONE;
        int r2 = -1;
        const ColSrc cs{s, (u128)0, 0};
        wave_select_rounds(s, cs, klo0, khi0, neg ? (u128)0 : ex.B, neg ? ex.A : W, neg ? 0 : ex.N + ex.Z,
                           neg ? ex.N : ex.NV, tau, ws, k2, r2, err);
        if (lane == t) {
          okey = k2;
          orow = r2;
        }
      }

      if constexpr (!kMulti) {
        // one penalty (lane 0): the residual of its row, or the column mass
        // of k where v_k = 0; values taken from lane 0 without shuffles
        const int orw0 = __builtin_amdgcn_readfirstlane((nzg & 1ull) ? orow : -1);
        const double v0 = orw0 >= 0 ? ratio_of_key(uni_u64(okey)) : 0.0;
        const double e0 = orw0 >= 0 ? wave_residual<true>(s, v0) : Wk;   // (the sum in lane 0)
        if (lane == 0) {
          V[base] = v0;
          E[base] = e0;
          R[base] = orw0;
        }
        continue;
      }
      // residuals, reused while the selected row repeats: the group's targets
      // whose row differs from the previous target's are the jobs, scored up
      // to RJ at a time in one pass over the rows
      const int tend = min(Lg, 64 * g + 64);
      const int cnt = tend - 64 * g;
      int orw_l = -1;
      double v_l = 0.0;
      if (lane < cnt && ((nzg >> lane) & 1ull)) {
        orw_l = orow;
        v_l = ratio_of_key(okey);
      }
      int prv = __shfl_up(orw_l, 1);
      if (lane == 0) prv = prev_row;
      const bool need = lane < cnt && orw_l >= 0 && orw_l != prv;
      const uint64_t needm = __ballot(need);
      double e_l = 0.0;
      if (__builtin_popcountll(needm) == 1) {
        const int jl = __builtin_ctzll(needm);
        const double e1 = readlane_dbl(wave_residual<!kMulti>(s, readlane_dbl(v_l, jl)), 0);
        if (lane == jl) e_l = e1;
      } else if constexpr (kMulti) {
        // (one penalty: at most one job)
        uint64_t jm = needm;
        while (jm) {
          if (__builtin_popcountll(jm) > 4) run_jobs<8>(s, jm, v_l, lane, e_l);
          else run_jobs<4>(s, jm, v_l, lane, e_l);
        }
      }
      // each target takes the e of the last job at or before it (or the
      // previous group's last e when its row continues from there)
      double e_t;
      if (orw_l < 0) {
        e_t = Wk;                                    // R64 sum of |x_ik|
      } else {
        const uint64_t upto = needm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
        const double ej = __shfl(e_l, upto ? 63 - __builtin_clzll(upto) : 0);
        e_t = upto ? ej : prev_e;
      }
      if (lane < cnt) {
        const int t = 64 * g + lane;
        V[t * mm + base] = orw_l >= 0 ? v_l : 0.0;
        E[t * mm + base] = e_t;
        R[t * mm + base] = orw_l;
      }
      prev_row = __builtin_amdgcn_readlane(orw_l, cnt - 1);
      prev_e = readlane_dbl(e_t, cnt - 1);
    }
  }
  if (err && lane == 0) atomicOr(segflags + j, err);
  __syncthreads();   // the LDS is reused by the next item
}

// Persistent segment kernel: every workgroup pulls work items from the
// counter of its XCD until none is left.  Explicit items (a batch) come in
// one list per XCD, [xstart[x], xstart[x + 1]).  With items == nullptr the
// items of problem 0 are
// implicit and routed by XCD: its k range is cut into SEG_XCDS * chunks
// equal parts, XCD x owns parts [x chunks, (x + 1) chunks) and enumerates
// them part by part, every preserved column j (or cand[jj]) within a part, so
// the columns k that the workgroups of one XCD stream stay in its L2.
// Workgroups are dispatched to the XCDs round-robin (blockIdx mod 8); one
// whose XCD has no item left takes items of the next XCDs (the routing only
// affects where data is cached, never the results).  kLdsJ: every problem's
// column j fits the launch's LDS copy (n <= sxj_rows), else all are read from
// global memory.  nitems = items per XCD
// (implicit) or in total (explicit).  gate (optional): the kernel does
// nothing unless *gate == gate_on.
constexpr int SEG_XCDS = 8;

template <bool kLdsJ, bool kMulti>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_seg_batch(const ProbDesc *__restrict__ P, const WorkItem *__restrict__ items, int nitems, int chunks,
            int *__restrict__ counter, const int *__restrict__ xstart, const double *__restrict__ lam_all,
            const ColInfo *__restrict__ ci,
            const double2 *__restrict__ DZ, double *__restrict__ V, double *__restrict__ E,
            int *__restrict__ R, int *__restrict__ segflags, const int *__restrict__ cand, int ncand,
            const int *__restrict__ gate, int gate_on, const unsigned long long *__restrict__ segmask, int lcap,
            int sxj_rows) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_item, s_tried;                  // s_tried: XCD partitions found empty
  if (gate && *gate != gate_on) return;
  if (threadIdx.x == 0) s_tried = 0;
  while (true) {
    if (threadIdx.x == 0) {
      int q = -1;
      const int home = blockIdx.x % SEG_XCDS;
      for (int tried = s_tried; tried < SEG_XCDS; ++tried) {
        const int x = (home + tried) % SEG_XCDS;
        const int c = atomicAdd(counter + x, 1);
        const int have = items ? xstart[x + 1] - xstart[x] : nitems;
        if (c < have) {
          q = items ? xstart[x] + c : x * nitems + c;
          break;
        }
        s_tried = tried + 1;
      }
      s_item = q;
    }
    __syncthreads();
    const int q = uni_int(s_item);
    __syncthreads();
    if (q < 0) break;
    WorkItem it;
    int jj;                                        // row of the item's column in the mask
    if (items) {
      it = items[q];
      jj = it.j;
    } else {
      const int m0 = P[0].m;
      const int mj = cand ? ncand : m0;
      const int x = q / nitems, c = q % nitems;
      const int part = x * chunks + c / mj;
      jj = c % mj;
      const int kchunk = (m0 + SEG_XCDS * chunks - 1) / (SEG_XCDS * chunks);
      it.b = 0;
      it.j = cand ? cand[jj] : jj;
      it.kbeg = min(m0, part * kchunk);
      it.kend = min(m0, it.kbeg + kchunk);
      if (it.kbeg >= it.kend) continue;            // an empty part of a narrow matrix
    }
    const ProbDesc d = P[it.b];
    const unsigned long long *maskrow =
        segmask ? segmask + d.mask_off + (long long)jj * ((d.m + 63) >> 6) : nullptr;
    seg_item<kLdsJ, kMulti>(d.X, d.n, d.m, d.ld, ci + d.col_off, lam_all + d.lam_off, d.L, DZ + d.pair_off, it.j,
                    it.kbeg, it.kend, V + d.ws_off, E + d.ws_off, R + d.ws_off, segflags + d.col_off, maskrow,
                    lcap, sxj_rows, smem);
  }
}

// ------------------------------------------------------------ per-j objective
// One wave per (problem, lambda_t, j): E_j = R64_k e_jk, P_j = R64_k |v_k|,
// z_j = E_j + fl(lambda P_j).  zflag marks an infinite or NaN v_k.
// zstart[b] = first (t, j) slot of problem b (sum of L m over earlier ones).
__global__ void __launch_bounds__(64)
k_reduce_batch(const ProbDesc *__restrict__ P, const int *__restrict__ zstart, int B,
               const double *__restrict__ lam_all, const double *__restrict__ V, const double *__restrict__ E,
               double *__restrict__ Z, int *__restrict__ zflag, const int *__restrict__ jmask,
               const int *__restrict__ gate, int gate_on) {
  if (gate && *gate != gate_on) return;
  const long long g = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = find_owner(zstart, B, g);
  const ProbDesc d = P[b];
  const int local = (int)(g - zstart[b]);
  const int t = local / d.m, j = local % d.m;
  if (jmask && !jmask[j]) {
    // not a candidate (problem 0 only): never the argmin
    if (lane == 0) {
      Z[d.z_off + (long long)t * d.m + j] = __longlong_as_double(0x7ff0000000000000ll);
      zflag[d.z_off + (long long)t * d.m + j] = 0;
    }
    return;
  }
  const long long off = d.ws_off + ((long long)t * d.m + j) * d.m;
  double pe = 0.0, pv = 0.0;
  int bad = 0;
  for (int k = lane; k < d.m; k += 64) {
    pe = pe + E[off + k];
    const double a = fabs(V[off + k]);
    pv = pv + a;
    bad |= !isfinite(a);
  }
  pe = wave_r64_tree(pe);
  pv = wave_r64_tree(pv);
  bad = wave_max_int(bad);
  if (lane == 0) {
    const double pen = lam_all[d.lam_off + t] * pv;
    const double z = pe + pen;
    Z[d.z_off + (long long)t * d.m + j] = z;
    zflag[d.z_off + (long long)t * d.m + j] = bad;
  }
}

// -------------------------------------------------------------- argmin/gather
// One workgroup per (problem, lambda_t): j* = lexicographic argmin of
// (z_j, j); gathers v*, rows, z_all.  The workgroup of t = 0 also folds the
// problem's flags into its status word.  ostart[b] = sum of L over earlier
// problems.
__global__ void __launch_bounds__(256)
k_argmin_batch(const ProbDesc *__restrict__ P, const int *__restrict__ ostart, int B,
               const double *__restrict__ V, const int *__restrict__ R, const double *__restrict__ Z,
               const int *__restrict__ zflag, const ColInfo *__restrict__ ci, const int *__restrict__ segflags,
               const int *__restrict__ jmask, const int *__restrict__ gate, int gate_on, int *__restrict__ sticky) {
  __shared__ double sz[256];
  __shared__ int sj[256];
  __shared__ int sflag[256];
  if (gate && *gate != gate_on) return;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int b = find_owner(ostart, B, g);
  const ProbDesc d = P[b];
  const int t = g - ostart[b];
  const int m = d.m;
  const double *z = Z + d.z_off + (long long)t * m;
  double bz = 0.0;
  int bj = -1;
  for (int j = tid; j < m; j += blockDim.x) {
    double v = z[j];
    if (isnan(v)) v = __longlong_as_double(0x7ff0000000000000ll);
    if (bj < 0 || v < bz) { bz = v; bj = j; }
  }
  sz[tid] = bz;
  sj[tid] = bj;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (tid < s) {
      const int oj = sj[tid + s];
      const double oz = sz[tid + s];
      if (oj >= 0 && (sj[tid] < 0 || oz < sz[tid] || (oz == sz[tid] && oj < sj[tid]))) {
        sz[tid] = oz;
        sj[tid] = oj;
      }
    }
    __syncthreads();
  }
  const int js = sj[0];
  const long long src = d.ws_off + ((long long)t * m + js) * m;
  for (int k = tid; k < m; k += blockDim.x) {
    d.Vout[(long long)t * m + k] = V[src + k];
    if (d.ROWout) d.ROWout[(long long)t * m + k] = R[src + k];
    if (d.ZALLout) d.ZALLout[(long long)t * m + k] = z[k];
  }
  if (tid == 0) {
    d.Jout[t] = js;
    d.OBJout[t] = z[js];
  }
  if (t == 0 && (d.status || sticky)) {
    // condition bits; the status is the first that applies of: non-finite
    // input, too-wide column, selection bound, overflowed ratio
    int f = 0;
    for (int j = tid; j < m; j += blockDim.x) {
      const int cf = ci[d.col_off + j].flags;
      if (cf & COL_NONFINITE) f |= 1;
      if (cf & COL_WIDE) f |= 2;
      if (segflags[d.col_off + j] && (!jmask || jmask[j])) f |= 4;
    }
    for (long long q = tid; q < (long long)d.L * m; q += blockDim.x)
      if (zflag[d.z_off + q]) f |= 8;
    sflag[tid] = f;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
      if (tid < s) sflag[tid] |= sflag[tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      const int bb = sflag[0];
      const int st = (bb & 1) ? L1LINE_ENONFINITE : (bb & 2) ? L1LINE_EWIDE : (bb & 4) ? L1LINE_EINTERNAL
                   : (bb & 8) ? L1LINE_ERANGE : L1LINE_OK;
      if (d.status) *d.status = st;
      // the context's sticky error keeps the first data-dependent error
      if (sticky && st != L1LINE_OK) atomicCAS(sticky, 0, st);
    }
  }
}

// Column statistics to user buffers.
__global__ void k_colstats_out(const ColInfo *__restrict__ ci, int m, double *__restrict__ W,
                               int *__restrict__ zeros, int *__restrict__ status) {
  __shared__ int sflag[256];
  int f = 0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    ColInfo c = ci[j];
    if (W) W[j] = c.W;
    if (zeros) zeros[j] = c.zeros;
    if (c.flags & COL_NONFINITE) f = L1LINE_ENONFINITE;
  }
  sflag[threadIdx.x] = f;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (threadIdx.x < s) sflag[threadIdx.x] = min(sflag[threadIdx.x], sflag[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && status) *status = sflag[0];
}
