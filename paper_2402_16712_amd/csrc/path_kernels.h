// path_kernels.h -- Algorithm 3 (Sec. 2): the exact solution path z*(lambda),
// v*(lambda) over every lambda >= 0, merged from the per-coordinate paths of
// Algorithm 2.
//
// For a preserved coordinate j, Algorithm 2's entries fix every v_k on each
// interval of lambda, and with them a line z_j = E_j + lambda P_j:
//   E_j = sum_k e_jk(v_k)   (e_jk scored as Algorithm 1 scores it, e_jj = 0)
//   P_j = 1 + sum_{k != j} |v_k|.
// Entry t of segment (j, k) holds for lambda >= its (rounded) breakpoint.
// E_j and P_j are exact: every e and |v| is an integer multiple of a global
// power of two (2^sE, 2^sP), and the lines are 128-bit integers in those
// units.  The merge over j (the paper's beta_L / beta_U comparisons) is a sweep
// in lambda that follows the lowest line through its crossings, with every
// comparison exact and every reported crossing rounded once.
//
// Pipeline (one GPU, everything on the device):
//   1. Algorithm 2's entries (bp_kernels.h).
//   2. k_sp_resid: e for every entry, up to 16 entries per pass over the rows
//      (columns through buffer loads, the 16 R64 trees folded together); the
//      global maxima that fix the scales.
//   3. k_sp_delta: each entry's change of (E, P) in fixed point.
//   4. k_sp_sort: one workgroup per j sorts j's entries by breakpoint (stable
//      LSD radix over the key bytes, tiles ranked and laid out by digit in
//      LDS before coalesced stores) and scans the changes into the exact
//      line after every entry.
//   5. k_sp_tiles: lambda tiles at quantiles of a sample of the breakpoints.
//   6. k_sp_slack, k_sp_bounds, k_sp_surv: per (tile, j) a lower bound of
//      z_j and per tile an upper bound of z*; a j whose lower bound exceeds
//      the upper bound cannot be on the path in that tile.  The bounds come
//      from the line just right of the tile's left end plus a proven slack:
//      each z_j differs from a concave, increasing function (the same
//      objective with the residuals summed exactly in real arithmetic) by at
//      most Delta_j, which covers the rounding of every residual and of every
//      breakpoint.
//   7. k_sp_sweep (count, then emit after k_sp_toff places each tile's
//      records): one wave per tile follows the lowest surviving line.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bp_kernels.h"

constexpr int SP_TMAX = 4096;      // lambda tiles
constexpr int SP_SAMPLES = 4096;   // breakpoints sampled to place them
constexpr int SP_RG = 16;          // entries scored per pass over the rows

struct PathScale {
  int sE, sP;        // units of E and P: 2^sE, 2^sP
  double lam_top;    // the largest breakpoint (every v_k is 0 beyond it)
  int bad;           // 1: a value has bits below its unit, or |v| >= 2^110;
                     // 2: a tile kept no line (non-finite bounds)
  int pad;
};

// ------------------------------------------------------------- exact helpers
struct U256 {
  uint64_t w[4];
};

__device__ __forceinline__ U256 u256_of(u128 a) {
  U256 r;
  r.w[0] = (uint64_t)a;
  r.w[1] = (uint64_t)(a >> 64);
  r.w[2] = r.w[3] = 0;
  return r;
}

__device__ __forceinline__ int u256_bitlen(const U256 &a) {
  for (int t = 3; t >= 0; --t)
    if (a.w[t]) return 64 * t + 64 - __builtin_clzll(a.w[t]);
  return 0;
}

__device__ __forceinline__ int u128_bitlen(u128 a) {
  const uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
  return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}

__device__ __forceinline__ int u256_cmp(const U256 &a, const U256 &b) {
  for (int t = 3; t >= 0; --t)
    if (a.w[t] != b.w[t]) return a.w[t] < b.w[t] ? -1 : 1;
  return 0;
}

// a << s for 0 <= s < 256 (bits above 2^256 are dropped; callers keep the
// result below 2^256)
__device__ __forceinline__ U256 u256_shl(const U256 &a, int s) {
  U256 r;
  const int q = s >> 6, b = s & 63;
  for (int t = 3; t >= 0; --t) {
    const int src = t - q;
    uint64_t v = src >= 0 ? a.w[src] << b : 0;
    if (b && src - 1 >= 0) v |= a.w[src - 1] >> (64 - b);
    r.w[t] = v;
  }
  return r;
}

__device__ __forceinline__ U256 u256_sub(const U256 &a, const U256 &b) {
  U256 r;
  uint64_t borrow = 0;
  for (int t = 0; t < 4; ++t) {
    const uint64_t x = a.w[t], y = b.w[t];
    const uint64_t d = x - y - borrow;
    borrow = (x < y) || (x == y && borrow) ? 1 : 0;
    r.w[t] = d;
  }
  return r;
}

// 128 x 128 -> 256-bit product
__device__ __forceinline__ U256 u256_mul(u128 a, u128 b) {
  const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  U256 r;
  r.w[0] = (uint64_t)p00;
  u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  r.w[1] = (uint64_t)mid;
  u128 up = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
  r.w[2] = (uint64_t)up;
  r.w[3] = (uint64_t)((up >> 64) + (p11 >> 64));
  return r;
}

// sign of A 2^a - B 2^b for nonzero A, B
__device__ __forceinline__ int cmp_scaled(const U256 &A, int a, const U256 &B, int b) {
  const int la = u256_bitlen(A), lb = u256_bitlen(B);
  if (la + a != lb + b) return la + a > lb + b ? 1 : -1;
  // equal top positions: |a - b| = |lb - la| < 256, and the shifted value keeps
  // the other's bit length
  if (a >= b) return u256_cmp(u256_shl(A, a - b), B);
  return u256_cmp(A, u256_shl(B, b - a));
}

// Order of the lines a and b just right of lambda = p (p >= 0): -1 when a is
// lower there, +1 when b is.  Values E + p P first (exact), then the slope.
__device__ __forceinline__ int line_cmp_at(u128 Ea, u128 Pa, u128 Eb, u128 Pb, double p, int sE, int sP) {
  const bool negE = Ea < Eb, negP = Pa < Pb;
  const u128 dE = negE ? Eb - Ea : Ea - Eb, dP = negP ? Pb - Pa : Pa - Pb;
  int val;
  if (dP == 0 || !(p > 0.0)) {
    val = dE == 0 ? 0 : (negE ? -1 : 1);
  } else if (dE == 0) {
    val = negP ? -1 : 1;
  } else if (negE == negP) {
    val = negE ? -1 : 1;
  } else {
    uint64_t M;
    int Ep;
    dbl_parts(p, M, Ep);
    const int c = cmp_scaled(u256_of(dE), sE, u256_mul(dP, (u128)M), Ep + sP);
    val = c == 0 ? 0 : (c > 0 ? (negE ? -1 : 1) : (negP ? -1 : 1));
  }
  if (val) return val;
  return Pa == Pb ? 0 : (Pa < Pb ? -1 : 1);
}

// The double nearest to q 2^e, plus a sticky bit below q (ties to even);
// q >= 2^55.
__device__ __forceinline__ double round_u256(const U256 &q, int e, bool sticky) {
  const int top = u256_bitlen(q) - 1;
  int keep = 53;
  if (top + e < -1022) keep = 53 - (-1022 - (top + e));
  const int shift = top + 1 - keep;
  if (shift > 250) return 0.0;
  U256 r = q;
  // r >>= shift
  {
    const int qq = shift >> 6, b = shift & 63;
    U256 t;
    for (int i = 0; i < 4; ++i) {
      const int src = i + qq;
      uint64_t v = src < 4 ? q.w[src] >> b : 0;
      if (b && src + 1 < 4) v |= q.w[src + 1] << (64 - b);
      t.w[i] = v;
    }
    r = t;
  }
  // remainder against half an ulp
  const U256 back = u256_shl(r, shift);
  const U256 rem = u256_sub(q, back);
  U256 half = u256_of(0);
  half = u256_shl(u256_of(1), shift - 1);
  const int c = u256_cmp(rem, half);
  uint64_t m = r.w[0];   // at most 2^53
  if (c > 0 || (c == 0 && (sticky || (m & 1)))) m += 1;
  return ldexp((double)m, e + shift);
}

// The double nearest to (N / D) 2^e0 for N, D > 0.
__device__ __forceinline__ double ratio_to_double(u128 N, u128 D, int e0) {
  const int ln = u128_bitlen(N), ld = u128_bitlen(D);
  const int sh = ld + 56 > ln ? ld + 56 - ln : 0;
  U256 R = u256_shl(u256_of(N), sh);
  const U256 Dw = u256_of(D);
  U256 q = u256_of(0);
  for (int pos = u256_bitlen(R) - ld; pos >= 0; --pos) {
    const U256 t = u256_shl(Dw, pos);
    if (u256_cmp(R, t) >= 0) {
      R = u256_sub(R, t);
      q.w[pos >> 6] |= 1ull << (pos & 63);
    }
  }
  const bool sticky = (R.w[0] | R.w[1] | R.w[2] | R.w[3]) != 0;
  return round_u256(q, e0 - sh, sticky);
}

// first position in [0, len) whose key is >= kb (len if none)
__device__ __forceinline__ long long lower_bound_u64(const uint64_t *__restrict__ a, long long len, uint64_t kb) {
  long long lo = 0, hi = len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (a[mid] < kb) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// first position in [0, len) whose key is > kb (len if none)
__device__ __forceinline__ long long upper_bound_u64(const uint64_t *__restrict__ a, long long len, uint64_t kb) {
  long long lo = 0, hi = len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (a[mid] <= kb) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double dofbits(uint64_t b) { return __longlong_as_double((long long)b); }

// ------------------------------------------------------------------ residuals
// G entries of one segment scored in one pass over the rows: lane l sums
// rows l, l + 64, ... in increasing order (the R64 partials), the rows of the
// next slot loaded while this slot is scored; then the R64 tree per entry.
// One level of the R64 tree for K entries at once: the lanes below stride d
// keep the first half of the entries, the others the second half, and each
// adds its partner's value for the kept entry (lane l with lane l + d, the
// pair the tree adds).  Half the shuffles of K separate trees.
template <int K>
__device__ __forceinline__ void sp_fold(double *v, int lane, int d) {
  const bool up = (lane & d) != 0;
#pragma unroll
  for (int i = 0; i < K / 2; ++i) {
    const double lo = v[i], hi = v[K / 2 + i];
    const double keep = up ? hi : lo, send = up ? lo : hi;
    const double recv = __shfl_xor(send, d);
    v[i] = up ? recv + keep : keep + recv;
  }
}

// R64 sums of G lane-partials at once: returns entry (lane >> (6 - log2 G))
// mod G's sum in the lanes whose low 6 - log2 G bits are zero.
template <int G>
__device__ __forceinline__ double sp_tree(double (&p)[G], int lane) {
  static_assert(G == 4 || G == 8 || G == 16, "group size");
  constexpr int LG = G == 16 ? 4 : G == 8 ? 3 : 2;
  sp_fold<G>(p, lane, 32);
  sp_fold<G / 2>(p, lane, 16);
  if constexpr (LG >= 3) sp_fold<G / 4>(p, lane, 8);
  if constexpr (LG >= 4) sp_fold<G / 8>(p, lane, 4);
  double x = p[0];
#pragma unroll
  for (int d = 32 >> LG; d >= 1; d >>= 1) {
    const double o = __shfl_xor(x, d);
    x = (lane & d) ? o + x : x + o;
  }
  return x;
}

// Rows lane + 64 s for s < steps; a row past n reads 0 and adds
// |0 - v 0| = +0, which leaves the lane's partial as it is.  The next row
// step is loaded before the current one is used.
template <int G>
__device__ __forceinline__ void sp_score(__amdgpu_buffer_rsrc_t rj, __amdgpu_buffer_rsrc_t rk, int steps, int lane,
                                         const double *__restrict__ ev, long long t0, long long b,
                                         double *__restrict__ ee, double &emax, double &vmax) {
  double v[G], p[G];
#pragma unroll
  for (int r = 0; r < G; ++r) {
    v[r] = t0 + r < b ? ev[t0 + r] : 0.0;
    p[r] = 0.0;
  }
  int off = lane * 8;
  double xa = col_ld(rj, off), ya = col_ld(rk, off);
  int s = 0;
  for (; s + 2 <= steps; s += 2) {
    const double xb = col_ld(rj, off + 512), yb = col_ld(rk, off + 512);
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const double prod = v[r] * xa;
      const double d = ya - prod;
      p[r] = p[r] + fabs(d);
    }
    off += 1024;
    xa = col_ld(rj, off);
    ya = col_ld(rk, off);
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const double prod = v[r] * xb;
      const double d = yb - prod;
      p[r] = p[r] + fabs(d);
    }
  }
  if (s < steps) {
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const double prod = v[r] * xa;
      const double d = ya - prod;
      p[r] = p[r] + fabs(d);
    }
  }
#pragma unroll
  for (int r = 0; r < G; ++r)
    if (t0 + r < b) vmax = fmax(vmax, fabs(v[r]));
  constexpr int SH = G == 16 ? 2 : G == 8 ? 3 : 4;
  const double e = sp_tree<G>(p, lane);
  const int r = (lane >> SH) & (G - 1);
  if ((lane & ((1 << SH) - 1)) == 0 && t0 + r < b) {
    ee[t0 + r] = e;
    emax = fmax(emax, e);
  }
}

// One wave per segment g = j m + k: e_t = R64 over the rows of
// |x_ik - fl(v_t x_ij)| for each entry (the order Algorithm 1 uses), the
// largest |v| of the segment, and the global maxima of e, |v| and the
// breakpoints (nonnegative doubles order as their bit patterns).  Entries in
// groups of 16, the last group of 8 or 4 when that covers the rest; segments
// in XCD tiles (at least 8 workgroups).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_sp_resid(const double *__restrict__ X, int n, int m, long long ld, const long long *__restrict__ offsets,
           const double *__restrict__ elam, const double *__restrict__ ev, double *__restrict__ ee,
           double *__restrict__ segv, unsigned long long *__restrict__ gmax, int *__restrict__ next) {
  const int lane = threadIdx.x & 63;
  const XcdTiles tl(m, xcd_tile(n), blockDim.x >> 6);
  double we = 0.0, wv = 0.0, wl = 0.0;   // the wave's maxima, one atomic each at the end
  for (;;) {
    // the XCD's next tile slot from its own counter (next[x], zero at
    // launch): the waves of an XCD stay on neighbouring slots, whose
    // columns share its L2, however long their segments
    int fi = 0;
    if (lane == 0) fi = atomicAdd(next + tl.x, 1);
    const long long f = __builtin_amdgcn_readfirstlane(__shfl(fi, 0));
    long long g;
    if (!tl.at(f, g)) break;
    if (g < 0) continue;
    // the segment is the same for the whole wave: its values go to scalar
    // registers
    const int j = __builtin_amdgcn_readfirstlane((int)(g / m)), k = __builtin_amdgcn_readfirstlane((int)(g % m));
    g = (long long)j * m + k;
    const long long a = offsets[g], b = offsets[g + 1];
    if (j == k || a == b) {
      if (lane == 0) segv[g] = 0.0;
      continue;
    }
    const __amdgpu_buffer_rsrc_t rj = col_rsrc(X + (long long)j * ld, n), rk = col_rsrc(X + (long long)k * ld, n);
    const int steps = (n + 63) >> 6;
    double emax = 0.0, vmax = 0.0;
    long long t0 = a;
    for (; b - t0 > 8; t0 += SP_RG) sp_score<SP_RG>(rj, rk, steps, lane, ev, t0, b, ee, emax, vmax);
    if (b - t0 > 4) sp_score<8>(rj, rk, steps, lane, ev, t0, b, ee, emax, vmax);
    else if (b - t0 > 0) sp_score<4>(rj, rk, steps, lane, ev, t0, b, ee, emax, vmax);
    if (lane == 0) segv[g] = vmax;
    we = fmax(we, emax);
    wv = fmax(wv, vmax);
    wl = fmax(wl, elam[b - 1]);
  }
  // e's maximum sits in the lanes that held the sums
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) we = fmax(we, __shfl_xor(we, d));
  if (lane == 0) {
    atomicMax(gmax + 0, (unsigned long long)dbits(we));
    atomicMax(gmax + 1, (unsigned long long)dbits(wv));
    atomicMax(gmax + 2, (unsigned long long)dbits(wl));
  }
}

// Units: E_j < m 2^(top(e) + 1) < 2^124 units of 2^sE with sE = top(e) - 110
// (m <= 8192), likewise P_j with the largest of |v| and 1.
__global__ void k_sp_scale(const unsigned long long *__restrict__ gmax, PathScale *__restrict__ sc) {
  if (threadIdx.x || blockIdx.x) return;
  const double emax = dofbits(gmax[0]), vmax = fmax(dofbits(gmax[1]), 1.0);
  PathScale s;
  s.sE = emax > 0.0 ? max(highest_bit_exp(emax) - 110, -1074) : -1074;
  s.sP = max(highest_bit_exp(vmax) - 110, -1074);
  s.lam_top = dofbits(gmax[2]);
  s.bad = s.sP > 0 ? 1 : 0;   // the preserved coordinate's 1 must be a whole number of units
  s.pad = 0;
  *sc = s;
}

// --------------------------------------------------------------------- deltas
// The change of (E, P) at each entry: entry t replaces entry t - 1 of its
// segment (entry 0 replaces nothing).  Two's complement in 128 bits.
// An entry's change of the line: value E and slope P, one 32-byte record so
// that the sort's gather of both touches one cache line.
struct alignas(32) SpDelta {
  u128 E, P;
};

__global__ void __launch_bounds__(256)
k_sp_delta(int m, const long long *__restrict__ offsets, const double *__restrict__ ev,
           const double *__restrict__ ee, PathScale *__restrict__ sc, SpDelta *__restrict__ dz) {
  const int lane = threadIdx.x & 63;
  const long long nseg = (long long)m * m;
  const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
  const int sE = sc->sE, sP = sc->sP;
  int bad = 0;
  for (long long g = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g < nseg; g += waves) {
    const long long a = offsets[g], b = offsets[g + 1];
    for (long long t = a + lane; t < b; t += 64) {
      const double e = ee[t], v = fabs(ev[t]);
      const double pe = t > a ? ee[t - 1] : 0.0, pv = t > a ? fabs(ev[t - 1]) : 0.0;
      if ((e != 0.0 && lowest_bit_exp(e) < sE) || (v != 0.0 && lowest_bit_exp(v) < sP)) bad = 1;
      SpDelta dl;
      dl.E = fixed_of(e, sE) - fixed_of(pe, sE);
      dl.P = fixed_of(v, sP) - fixed_of(pv, sP);
      dz[t] = dl;
    }
  }
  if (bad) atomicOr(&sc->bad, 1);
}

// ------------------------------------------------------------ sort and lines
// One workgroup of 1024 per preserved coordinate j: its entries
// [offsets[j m], offsets[j m + m]) sorted by breakpoint, stably (ties keep
// the (k, t) order), then the exact line after every entry:
// stE/stP[s] = (0, 1) + the changes of sorted entries 0..s.
//
// The sort is a least-significant-digit radix over the 8 bytes of the key
// (the bits of a nonnegative double order like the double). One read of the
// breakpoints counts all 8 digits; a pass whose digit is the same for every
// entry is skipped. A pass takes tiles of SP_SORT_TILE entries: each wave
// ranks its 256 entries by digit (64 at a time, in index order), the tile is
// laid out digit by digit in LDS, and then written out in runs, so
// consecutive lanes store to consecutive addresses of a digit's range.
constexpr int SP_SORT_TILE = 4096;
struct SpSortLds {
  uint64_t key[SP_SORT_TILE];
  uint32_t id[SP_SORT_TILE];
  unsigned wcnt[16][256];   // per wave: running count, then start within its digit
  unsigned gb[8][256];      // per pass: count, then next output index of each digit
  unsigned tb[256];         // tile: first LDS index of each digit
  unsigned tc[256];         // tile: entries of each digit
  int nrun;                 // passes that move entries
  int run[8];
  u128 wt[16], wtp[16];    // wave totals of a tile's changes of E and P
  u128 wp[16], wpp[16];    // their exclusive prefix
  u128 tt, ttp;            // tile totals
};
constexpr size_t SP_SORT_LDS = sizeof(SpSortLds);

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_sp_sort(int m, const long long *__restrict__ offsets, const double *__restrict__ elam, uint64_t *__restrict__ keyA,
          uint32_t *__restrict__ idA, uint64_t *__restrict__ keyB, uint32_t *__restrict__ idB,
          const SpDelta *__restrict__ dz, const PathScale *__restrict__ sc,
          u128 *__restrict__ stE, u128 *__restrict__ stP) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sp_smem[];
  SpSortLds &L = *reinterpret_cast<SpSortLds *>(sp_smem);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int j = blockIdx.x;
  const long long a = offsets[(long long)j * m], N = offsets[(long long)j * m + m] - a;
  for (int q = tid; q < 8 * 256; q += 1024) L.gb[q >> 8][q & 255] = 0;
  __syncthreads();
  for (long long s = tid; s < N; s += 1024) {
    const uint64_t key = dbits(elam[a + s]);
#pragma unroll
    for (int p = 0; p < 8; ++p) atomicAdd(&L.gb[p][(key >> (8 * p)) & 255], 1u);
  }
  __syncthreads();
  if (tid < 512) {
    // wave p turns pass p's counts into first output indices
    const int p = w;
    unsigned c[4], t = 0;
    bool one = false;
    for (int r = 0; r < 4; ++r) {
      c[r] = L.gb[p][4 * lane + r];
      t += c[r];
      one |= (long long)c[r] == N;
    }
    unsigned run = (unsigned)wave_excl_scan_int((int)t, lane);
    for (int r = 0; r < 4; ++r) {
      L.gb[p][4 * lane + r] = run;
      run += c[r];
    }
    const bool skip = __ballot(one) != 0ull;
    if (lane == 0) L.run[p] = skip ? 0 : 1;
  }
  __syncthreads();
  if (tid == 0) {
    int c = 0;
    for (int p = 0; p < 8; ++p)
      if (L.run[p]) L.run[c++] = p;
    L.nrun = c;
  }
  __syncthreads();
  const int nrun = L.nrun;
  if (nrun == 0) {
    // every key the same: the index order is the sorted order
    for (long long s = tid; s < N; s += 1024) {
      keyA[a + s] = dbits(elam[a + s]);
      idA[a + s] = (uint32_t)(a + s);
    }
  }
  // the last moving pass writes keyA/idA
  uint64_t *kout = (nrun & 1) ? keyA : keyB;
  uint32_t *iout = (nrun & 1) ? idA : idB;
  const uint64_t *kin = nullptr;
  const uint32_t *iin = nullptr;
  for (int ip = 0; ip < nrun; ++ip) {
    const int p = L.run[ip], sh = 8 * p;
    for (long long t0 = 0; t0 < N; t0 += SP_SORT_TILE) {
      for (int r = 0; r < 4; ++r) L.wcnt[w][4 * lane + r] = 0;
      const int tn = (int)min((long long)SP_SORT_TILE, N - t0);
      uint64_t key[4];
      uint32_t id[4];
      if (ip == 0) {
        const double *__restrict__ lb = elam + a + t0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = w * 256 + r * 64 + lane;
          key[r] = e < tn ? dbits(lb[e]) : 0ull;
          id[r] = (uint32_t)(a + t0) + (uint32_t)e;
        }
      } else {
        const uint64_t *__restrict__ kb = kin + a + t0;
        const uint32_t *__restrict__ ib = iin + a + t0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = w * 256 + r * 64 + lane;
          key[r] = e < tn ? kb[e] : 0ull;
          id[r] = e < tn ? ib[e] : 0u;
        }
      }
      // (digit << 16) | rank within the wave's digit, all ones past the end
      unsigned pk[4];
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool valid = w * 256 + r * 64 + lane < tn;
        const int d = (int)((key[r] >> sh) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
          const uint64_t bb = __ballot((d >> bit) & 1);
          peers &= ((d >> bit) & 1) ? bb : ~bb;
        }
        const int rank = lanes_below(peers);
        const unsigned off = L.wcnt[w][d];
        pk[r] = valid ? ((unsigned)d << 16) | (off + (unsigned)rank) : ~0u;
        wave_lds_sync();
        if (valid && rank == 0) L.wcnt[w][d] = off + (unsigned)__builtin_popcountll(peers);
        wave_lds_sync();
      }
      __syncthreads();
      if (tid < 256) {
        unsigned run = 0;
        for (int q = 0; q < 16; ++q) {
          const unsigned c = L.wcnt[q][tid];
          L.wcnt[q][tid] = run;
          run += c;
        }
        L.tc[tid] = run;
      }
      __syncthreads();
      if (tid < 64) {
        unsigned c[4], t = 0;
        for (int r = 0; r < 4; ++r) {
          c[r] = L.tc[4 * lane + r];
          t += c[r];
        }
        unsigned run = (unsigned)wave_excl_scan_int((int)t, lane);
        for (int r = 0; r < 4; ++r) {
          L.tb[4 * lane + r] = run;
          run += c[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (pk[r] != ~0u) {
          const int d = (int)(pk[r] >> 16);
          const unsigned pos = L.tb[d] + L.wcnt[w][d] + (pk[r] & 0xffffu);
          L.key[pos] = key[r];
          L.id[pos] = id[r];
        }
      }
      __syncthreads();
      uint64_t *__restrict__ ko = kout + a;
      uint32_t *__restrict__ io = iout + a;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = r * 1024 + tid;
        if (q < tn) {
          const uint64_t k = L.key[q];
          const int d = (int)((k >> sh) & 255);
          const unsigned dst = L.gb[p][d] + (unsigned)q - L.tb[d];
          ko[dst] = k;
          io[dst] = L.id[q];
        }
      }
      __syncthreads();
      if (tid < 256) L.gb[p][tid] += L.tc[tid];
    }
    // this pass's output is the next one's input; the buffers alternate
    // so that the last pass ends in keyA/idA
    __syncthreads();
    kin = kout;
    iin = iout;
    kout = (kout == keyA) ? keyB : keyA;
    iout = (iout == idA) ? idB : idA;
  }
  __syncthreads();
  // exact lines in sorted order: one entry per lane (its value and slope
  // change read together), then the lanes, then the 16 waves
  u128 cE = 0, cP = fixed_of(1.0, sc->sP);
  for (long long t0 = 0; t0 < N; t0 += 1024) {
    const long long s0 = t0 + tid;
    u128 x = 0, y = 0;
    if (s0 < N) {
      const SpDelta d0 = dz[idA[a + s0]];
      x = d0.E;
      y = d0.P;
    }
    const u128 ix = wave_incl_scan_u128(x, lane), iy = wave_incl_scan_u128(y, lane);
    if (lane == 63) {
      L.wt[w] = ix;
      L.wtp[w] = iy;
    }
    __syncthreads();
    if (tid < 64) {
      const u128 ox = lane < 16 ? L.wt[lane] : (u128)0, oy = lane < 16 ? L.wtp[lane] : (u128)0;
      const u128 sx = wave_incl_scan_u128(ox, lane), sy = wave_incl_scan_u128(oy, lane);
      if (lane < 16) {
        L.wp[lane] = sx - ox;
        L.wpp[lane] = sy - oy;
      }
      if (lane == 15) {
        L.tt = sx;
        L.ttp = sy;
      }
    }
    __syncthreads();
    if (s0 < N) {
      stE[a + s0] = cE + L.wp[w] + ix;
      stP[a + s0] = cP + L.wpp[w] + iy;
    }
    cE += L.tt;
    cP += L.ttp;
  }
}

// ---------------------------------------------------------------------- tiles
// Tile boundaries b_0 = 0 < b_1 < ... < b_{T-1} = lambda_top at quantiles of
// a strided sample of the breakpoints and on a uniform grid; tile i is
// [b_i, b_{i+1}), the last [lambda_top, inf).  T = 1 when lambda_top is 0.
__global__ void __launch_bounds__(1024)
k_sp_tiles(long long NE, const double *__restrict__ elam, const PathScale *__restrict__ sc, double *__restrict__ bnd,
           int *__restrict__ T) {
  __shared__ uint64_t smp[SP_SAMPLES];
  const int tid = threadIdx.x;
  for (int s = tid; s < SP_SAMPLES; s += 1024) {
    const long long idx = NE > 0 ? ((long long)s * NE + NE / 2) / SP_SAMPLES : 0;
    smp[s] = NE > 0 ? dbits(elam[idx]) : 0;
  }
  __syncthreads();
  for (int size = 2; size <= SP_SAMPLES; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < SP_SAMPLES / 2; t += 1024) {
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = smp[lo], y = smp[hi];
        if ((x > y) == up) {
          smp[lo] = y;
          smp[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    // half the boundaries at quantiles of the sample, half on a uniform grid
    // over (0, lambda_top) (wide stretches with few breakpoints still get
    // narrow tiles), merged in order without repeats
    const double top = sc->lam_top;
    constexpr int H = SP_TMAX / 2;
    int c = 1;
    bnd[0] = 0.0;
    if (top > 0.0) {
      int qa = 1, ua = 1;
      while (qa < H || ua < H) {
        const double xq = qa < H ? dofbits(smp[((long long)qa * SP_SAMPLES) / H]) : INFINITY;
        const double xu = ua < H ? top * ((double)ua / (double)H) : INFINITY;
        double x;
        if (xq <= xu) {
          x = xq;
          ++qa;
        } else {
          x = xu;
          ++ua;
        }
        if (x > bnd[c - 1] && x < top) bnd[c++] = x;
      }
      bnd[c++] = top;
    }
    *T = c;
  }
}

// Delta_j: the distance between z_j and the concave increasing objective with
// exact residuals.  Per segment: (n + 4) u (W_k + V W_j) for the rounding of the
// residual terms, their R64 sum and of the ratios, plus ulp(lambda_top) V for
// breakpoints rounded to doubles (V the largest |v| of the segment); 1.5 covers
// the rounding of this sum.
__global__ void k_sp_slack(int n, int m, const ColInfo *__restrict__ ci, const double *__restrict__ segv,
                           const PathScale *__restrict__ sc, double *__restrict__ D) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const double top = sc->lam_top;
  const double ulp = top > 0.0 ? ldexp(1.0, highest_bit_exp(top) - 52) : 0.0;
  const double u = ldexp(1.0, -53) * (double)(n + 4);
  const double Wj = ci[j].W;
  double s = 0.0;
  for (int k = 0; k < m; ++k) {
    if (k == j) continue;
    const double V = segv[(long long)j * m + k];
    s += u * (ci[k].W + V * Wj) + ulp * V;
  }
  D[j] = 1.5 * s;
}

// Per tile i < T - 1 (one block): LB[i m + j] = lower bound of z_j on the tile,
// U[i] = the smallest upper bound of any z_j over the tile.  With c_j the
// concave increasing function within Delta_j of z_j and (E, P) the line of z_j
// just right of b_i: z_j >= c_j(b_i) - Delta_j >= E + b_i P - 2 Delta_j on the
// tile, and z_j(lambda) <= (the objective with v held at that line's v) +
// Delta_j <= E + lambda P + 2 Delta_j.
__global__ void __launch_bounds__(256)
k_sp_bounds(int m, const long long *__restrict__ offsets, const uint64_t *__restrict__ key,
            const u128 *__restrict__ stE, const u128 *__restrict__ stP, const PathScale *__restrict__ sc,
            const double *__restrict__ bnd, const int *__restrict__ Tp, const double *__restrict__ D,
            double *__restrict__ LB, double *__restrict__ U) {
  __shared__ double red[4];
  const int T = *Tp, i = blockIdx.x;
  if (i >= T - 1) return;
  const int sE = sc->sE, sP = sc->sP;
  const double bl = bnd[i], br = bnd[i + 1];
  const uint64_t kb = dbits(bl);
  const u128 one = fixed_of(1.0, sP);
  const double lo_f = 1.0 - ldexp(1.0, -44), hi_f = 1.0 + ldexp(1.0, -44);
  double umin = INFINITY;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const long long a = offsets[(long long)j * m], N = offsets[(long long)j * m + m] - a;
    const long long pos = upper_bound_u64(key + a, N, kb);   // the line right of b_i
    const u128 E = pos > 0 ? stE[a + pos - 1] : (u128)0, P = pos > 0 ? stP[a + pos - 1] : one;
    const double Ed = fixed_to_double(E, sE), Pd = fixed_to_double(P, sP);
    const double zl = Ed + bl * Pd, zu = Ed + br * Pd;
    LB[(long long)i * m + j] = zl * lo_f - 2.001 * D[j];
    umin = fmin(umin, zu * hi_f + 2.001 * D[j]);
  }
  for (int d = 32; d >= 1; d >>= 1) umin = fmin(umin, __shfl_xor(umin, d));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = umin;
  __syncthreads();
  if (threadIdx.x == 0) U[i] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Survivors of tile i in ascending j: list[i m + c], cnt[i].  The last tile
// [lambda_top, inf) has every v_k = 0, so all lines have slope 1 and the
// smallest E (then j) is the only survivor.
__global__ void __launch_bounds__(256)
k_sp_surv(int m, const long long *__restrict__ offsets, const u128 *__restrict__ stE, const double *__restrict__ LB,
          const double *__restrict__ U, const int *__restrict__ Tp, int *__restrict__ list, int *__restrict__ cnt) {
  __shared__ int wsum[4];
  __shared__ int run;
  __shared__ u128 bestE[4];
  __shared__ int bestJ[4];
  const int T = *Tp, i = blockIdx.x;
  if (i >= T) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int *L = list + (long long)i * m;
  if (i < T - 1) {
    const double u = U[i];
    if (tid == 0) run = 0;
    __syncthreads();
    for (int j0 = 0; j0 < m; j0 += 256) {
      const int j = j0 + tid;
      const bool keep = j < m && LB[(long long)i * m + j] <= u;
      const uint64_t bl = __ballot(keep);
      const int r = __builtin_popcountll(bl & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[w] = __builtin_popcountll(bl);
      __syncthreads();
      int off = run;
      for (int q = 0; q < w; ++q) off += wsum[q];
      if (keep) L[off + r] = j;
      __syncthreads();
      if (tid == 0) run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
      __syncthreads();
    }
    if (tid == 0) cnt[i] = run;
  } else {
    u128 be = ~(u128)0;
    int bj = m;
    for (int j = tid; j < m; j += 256) {
      const long long a = offsets[(long long)j * m], N = offsets[(long long)j * m + m] - a;
      const u128 E = N > 0 ? stE[a + N - 1] : (u128)0;
      if (E < be || (E == be && j < bj)) {
        be = E;
        bj = j;
      }
    }
    for (int d = 32; d >= 1; d >>= 1) {
      const uint64_t lo = shfl_xor_u64((uint64_t)be, d), hi = shfl_xor_u64((uint64_t)(be >> 64), d);
      const u128 oe = (((u128)hi) << 64) | lo;
      const int oj = __shfl_xor(bj, d);
      if (oe < be || (oe == be && oj < bj)) {
        be = oe;
        bj = oj;
      }
    }
    if (lane == 0) {
      bestE[w] = be;
      bestJ[w] = bj;
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 1; q < 4; ++q)
        if (bestE[q] < be || (bestE[q] == be && bestJ[q] < bj)) {
          be = bestE[q];
          bj = bestJ[q];
        }
      L[0] = bj;
      cnt[i] = 1;
    }
  }
}

// ---------------------------------------------------------------------- sweep
struct PathOut {
  double *lam;
  long long *j;
  int *k;
  double *v;
  int *row;
  double *E;
  double *P;
};

// Per tile: j at the start (after the entries at b_i), j at the end, the
// records after the start point, and the entries of the start's j at b_i.
struct TileInfo {
  int jstart, jend, nstart, npoints;   // npoints: breakpoint values the sweep visited
  long long ninner;
};

// the line of survivor position pos of coordinate j (pos = first entry not applied)
__device__ __forceinline__ void sp_line(const u128 *__restrict__ stE, const u128 *__restrict__ stP, long long a,
                                        long long pos, u128 one, u128 &E, u128 &P) {
  if (pos > a) {
    E = stE[pos - 1];
    P = stP[pos - 1];
  } else {
    E = 0;
    P = one;
  }
}

// m records at lambda: coordinate j's v (each segment's last entry with
// breakpoint <= p) and its line
__device__ void sp_batch(int m, int j, double lam, double p, const long long *__restrict__ offsets,
                         const double *__restrict__ elam, const double *__restrict__ ev, const int *__restrict__ erow,
                         double Ed, double Pd, const PathOut &o, long long at, long long cap, int lane) {
  for (int k = lane; k < m; k += 64) {
    double v = 1.0;
    int r = -1;
    if (k != j) {
      const long long g = (long long)j * m + k, a = offsets[g], b = offsets[g + 1];
      long long lo = a, hi = b;   // first entry with breakpoint > p
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (elam[mid] <= p) lo = mid + 1; else hi = mid;
      }
      if (lo > a) {
        v = ev[lo - 1];
        r = erow[lo - 1];
      } else {
        v = 0.0;
      }
    }
    const long long q = at + k;
    if (q < cap) {
      o.lam[q] = lam;
      o.j[q] = j;
      o.k[q] = k;
      o.v[q] = v;
      o.row[q] = r;
      o.E[q] = Ed;
      o.P[q] = Pd;
    }
  }
}

// records of coordinate j's sorted entries [s0, s1) (all at lambda p)
__device__ void sp_events(int m, int j, double p, long long s0, long long s1, const long long *__restrict__ offsets,
                          const uint32_t *__restrict__ id, const double *__restrict__ ev, const int *__restrict__ erow,
                          const u128 *__restrict__ stE, const u128 *__restrict__ stP, int sE, int sP,
                          const PathOut &o, long long at, long long cap, int lane) {
  const long long *segs = offsets + (long long)j * m;
  for (long long s = s0 + lane; s < s1; s += 64) {
    const uint32_t e = id[s];
    int lo = 0, hi = m - 1;   // the segment holding entry e: last g with offsets[g] <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid] <= (long long)e) lo = mid; else hi = mid - 1;
    }
    const long long q = at + (s - s0);
    if (q < cap) {
      o.lam[q] = p;
      o.j[q] = j;
      o.k[q] = lo;
      o.v[q] = ev[e];
      o.row[q] = erow[e];
      o.E[q] = fixed_to_double(stE[s], sE);
      o.P[q] = fixed_to_double(stP[s], sP);
    }
  }
}

// One wave per tile.  emit = 0: fill info[i]; emit = 1: write the tile's
// records from toff[i] (start-of-tile batch when swflag[i]).
__global__ void __launch_bounds__(64)
k_sp_sweep(int m, const long long *__restrict__ offsets, const double *__restrict__ elam,
           const double *__restrict__ ev, const int *__restrict__ erow, const uint64_t *__restrict__ key,
           const uint32_t *__restrict__ id, const u128 *__restrict__ stE, const u128 *__restrict__ stP,
           PathScale *__restrict__ sc, const double *__restrict__ bnd, const int *__restrict__ Tp,
           const int *__restrict__ list, const int *__restrict__ cnt, long long *__restrict__ spos,
           long long *__restrict__ spb, TileInfo *__restrict__ info, const long long *__restrict__ toff,
           const int *__restrict__ swflag, int emit, PathOut o, long long cap) {
  const int T = *Tp, i = blockIdx.x, lane = threadIdx.x;
  if (i >= T) return;
  const int c = cnt[i];
  if (c < 1) {   // no line survived: only non-finite bounds can do this
    if (!emit && lane == 0) atomicOr(&sc->bad, 2);
    return;
  }
  const int *L = list + (long long)i * m;
  long long *POS = spos + (long long)i * m, *PB = spb + (long long)i * m;
  const int sE = sc->sE, sP = sc->sP;
  const u128 one = fixed_of(1.0, sP);
  const double bl = bnd[i], br = i + 1 < T ? bnd[i + 1] : INFINITY;
  for (int s = lane; s < c; s += 64) {
    const int j = L[s];
    const long long a = offsets[(long long)j * m], N = offsets[(long long)j * m + m] - a;
    POS[s] = a + lower_bound_u64(key + a, N, dbits(bl));
  }
  __syncthreads();
  long long at = emit ? toff[i] : 0, ninner = 0;
  int jstart = -1, nstart = 0, cur = -1, npoints = 0;   // cur: survivor index of the lowest line
  double p = bl;
  while (true) {
    ++npoints;
    // apply the entries at p; the next breakpoint of any survivor
    const uint64_t kp = dbits(p);
    uint64_t qk = ~0ull;
    for (int s = lane; s < c; s += 64) {
      const int j = L[s];
      const long long b = offsets[(long long)j * m + m];
      long long pos = POS[s];
      PB[s] = pos;
      while (pos < b && key[pos] == kp) ++pos;
      POS[s] = pos;
      if (pos < b && key[pos] < qk) qk = key[pos];
    }
    __syncthreads();
    qk = wave_min_u64(qk);
    const double q = qk == ~0ull ? br : fmin(dofbits(qk), br);
    // the lowest line just right of p (value, slope, then j)
    int bs = -1;
    u128 bE = 0, bP = 0;
    for (int s = lane; s < c; s += 64) {
      const int j = L[s];
      u128 E, P;
      sp_line(stE, stP, offsets[(long long)j * m], POS[s], one, E, P);
      if (bs < 0 || line_cmp_at(E, P, bE, bP, p, sE, sP) < 0) {   // ascending s: ties keep the lower j
        bs = s;
        bE = E;
        bP = P;
      }
    }
    for (int d = 1; d < 64; d <<= 1) {
      const int os = __shfl_xor(bs, d);
      const u128 oE = shfl_u128(bE, lane ^ d), oP = shfl_u128(bP, lane ^ d);
      bool take = false;
      if (os >= 0) {
        if (bs < 0) take = true;
        else {
          const int cc = line_cmp_at(oE, oP, bE, bP, p, sE, sP);
          take = cc < 0 || (cc == 0 && os < bs);
        }
      }
      if (take) {
        bs = os;
        bE = oE;
        bP = oP;
      }
    }
    bs = uni_int(bs);
    bE = uni_u128(bE);
    bP = uni_u128(bP);
    const int jn = L[bs];
    const long long nev = POS[bs] - PB[bs];
    if (p == bl) {
      jstart = jn;
      nstart = (int)nev;
      if (emit) {
        if (swflag[i]) {
          sp_batch(m, jn, p, p, offsets, elam, ev, erow, fixed_to_double(bE, sE), fixed_to_double(bP, sP), o, at,
                   cap, lane);
          at += m;
        } else {
          sp_events(m, jn, p, PB[bs], POS[bs], offsets, id, ev, erow, stE, stP, sE, sP, o, at, cap, lane);
          at += nev;
        }
      }
    } else if (bs != cur) {
      ninner += m;
      if (emit) {
        sp_batch(m, jn, p, p, offsets, elam, ev, erow, fixed_to_double(bE, sE), fixed_to_double(bP, sP), o, at, cap,
                 lane);
        at += m;
      }
    } else {
      ninner += nev;
      if (emit) {
        sp_events(m, jn, p, PB[bs], POS[bs], offsets, id, ev, erow, stE, stP, sE, sP, o, at, cap, lane);
        at += nev;
      }
    }
    cur = bs;
    // crossings inside (p, q): the first line of smaller slope to meet the
    // current one; among lines meeting it there, the smallest slope, then j
    while (true) {
      u128 cE, cP;
      sp_line(stE, stP, offsets[(long long)L[cur] * m], POS[cur], one, cE, cP);
      int xs = -1;
      u128 xN = 0, xD = 0, xP = 0;
      for (int s = lane; s < c; s += 64) {
        const int j = L[s];
        u128 E, P;
        sp_line(stE, stP, offsets[(long long)j * m], POS[s], one, E, P);
        if (!(P < cP) || !(E > cE)) continue;
        const u128 N = E - cE, D = cP - P;
        bool take = xs < 0;
        if (!take) {
          const int cc = u256_cmp(u256_mul(N, xD), u256_mul(xN, D));
          take = cc < 0 || (cc == 0 && P < xP);   // ascending s keeps the lower j on full ties
        }
        if (take) {
          xs = s;
          xN = N;
          xD = D;
          xP = P;
        }
      }
      for (int d = 1; d < 64; d <<= 1) {
        const int os = __shfl_xor(xs, d);
        const u128 oN = shfl_u128(xN, lane ^ d), oD = shfl_u128(xD, lane ^ d), oP = shfl_u128(xP, lane ^ d);
        bool take = false;
        if (os >= 0) {
          if (xs < 0) take = true;
          else {
            const int cc = u256_cmp(u256_mul(oN, xD), u256_mul(xN, oD));
            take = cc < 0 || (cc == 0 && (oP < xP || (oP == xP && os < xs)));
          }
        }
        if (take) {
          xs = os;
          xN = oN;
          xD = oD;
          xP = oP;
        }
      }
      xs = uni_int(xs);
      if (xs < 0) break;
      xN = uni_u128(xN);
      xD = uni_u128(xD);
      if (q < INFINITY) {
        uint64_t Mq;
        int Eq;
        dbl_parts(q, Mq, Eq);
        // crossing N/D 2^(sE - sP) at or beyond q: the entries at q decide
        if (cmp_scaled(u256_of(xN), sE - sP, u256_mul(xD, (u128)Mq), Eq) >= 0) break;
      }
      cur = xs;
      ninner += m;
      if (emit) {
        u128 nE, nP;
        const int jx = L[xs];
        sp_line(stE, stP, offsets[(long long)jx * m], POS[xs], one, nE, nP);
        sp_batch(m, jx, ratio_to_double(xN, xD, sE - sP), p, offsets, elam, ev, erow, fixed_to_double(nE, sE),
                 fixed_to_double(nP, sP), o, at, cap, lane);
        at += m;
      }
    }
    if (!(q < br)) break;
    p = q;
  }
  if (!emit && lane == 0) {
    TileInfo t;
    t.jstart = jstart;
    t.jend = L[cur];
    t.nstart = nstart;
    t.npoints = npoints;
    t.ninner = ninner;
    info[i] = t;
  }
}

// Record counts per tile: a batch of m at the start of tile 0 and wherever the
// coordinate at a tile's start differs from the one at the previous tile's
// end, else the start's own entries; exclusive offsets toff[0..T], total in
// toff[T].
__global__ void __launch_bounds__(1024)
k_sp_toff(int m, const int *__restrict__ Tp, const TileInfo *__restrict__ info, int *__restrict__ swflag,
          long long *__restrict__ toff, long long *__restrict__ total) {
  __shared__ long long part[1024];
  const int T = *Tp, tid = threadIdx.x;
  const int chunk = (T + 1023) / 1024;
  const int b = tid * chunk, e = min(T, b + chunk);
  long long sum = 0;
  for (int i = b; i < e; ++i) {
    const bool sw = i == 0 || info[i].jstart != info[i - 1].jend;
    swflag[i] = sw ? 1 : 0;
    sum += (sw ? m : info[i].nstart) + info[i].ninner;
  }
  part[tid] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const long long add = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  long long run = part[tid] - sum;
  for (int i = b; i < e; ++i) {
    toff[i] = run;
    run += (swflag[i] ? m : info[i].nstart) + info[i].ninner;
  }
  if (tid == 1023) {
    toff[T] = part[1023];
    *total = part[1023];
  }
}
