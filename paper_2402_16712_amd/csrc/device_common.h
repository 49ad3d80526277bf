// device_common.h -- wave64 primitives, order-preserving keys and exact
// 128-bit fixed-point weights shared by the l1line kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;

#define L1_WAVE 64

// Order-preserving map from a non-NaN double to uint64: a < b  <=>  key(a) < key(b).
// Callers pass canonical zeros (+0.0), so every zero ratio has the same key.
constexpr uint64_t KEY_ZERO = 0x8000000000000000ull;   // key(+0.0)
constexpr uint64_t KEY_NONE = ~0ull;                   // "no element" (above +inf)

__device__ __forceinline__ uint64_t key_of(double r) {
  uint64_t b = (uint64_t)__double_as_longlong(r);
  return (b >> 63) ? ~b : (b | KEY_ZERO);
}

__device__ __forceinline__ double ratio_of_key(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & ~KEY_ZERO) : ~k;
  return __longlong_as_double((long long)b);
}

// A load through the global address space: for pointers into device memory
// whose address space the compiler cannot see (struct fields), so that it
// emits a global load and waits for the memory counter only.
__device__ __forceinline__ double gld(const double *p) {
  return *(const __attribute__((address_space(1))) double *)p;
}

// number of set bits of the wave mask m in lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---------------------------------------------------------------- fixed point
// A finite nonzero |x| is M * 2^E with M < 2^53 (E = -1074 for subnormals).
__device__ __forceinline__ void dbl_parts(double a, uint64_t &M, int &E) {
  uint64_t b = (uint64_t)__double_as_longlong(a) & ~KEY_ZERO;
  int be = (int)(b >> 52);
  M = b & 0xFFFFFFFFFFFFFull;
  if (be) {
    M |= 1ull << 52;
    E = be - 1075;
  } else {
    E = -1074;
  }
}

__device__ __forceinline__ int lowest_bit_exp(double a) {
  uint64_t M; int E;
  dbl_parts(a, M, E);
  return E + __builtin_ctzll(M);
}

__device__ __forceinline__ int highest_bit_exp(double a) {
  uint64_t M; int E;
  dbl_parts(a, M, E);
  return E + 63 - __builtin_clzll(M);
}

// |x| / 2^e0 as an exact integer; e0 <= lowest_bit_exp(|x|) and the column
// range check keep the result below 2^124.
__device__ __forceinline__ u128 fixed_of(double a, int e0) {
  uint64_t M; int E;
  dbl_parts(a, M, E);
  const int sh = E - e0;
  const u128 up = ((u128)M) << (sh & 127);
  const u128 dn = (u128)(M >> ((-sh) & 63));   // only trailing zero bits are shifted out
  return (sh >= 0) ? (sh < 128 ? up : (u128)0) : (-sh < 64 ? dn : (u128)0);
}

// fixed_of for a weight of a column that passed the range check
// (lowest_bit_exp(a) >= e0, highest_bit_exp(a) - e0 < 124; 0 gives 0).  When
// E < e0 the bits shifted out of M are zeros.  Branch-free (64-bit shifts and
// selects).
__device__ __forceinline__ u128 fixed_of_col(double a, int e0) {
  uint64_t M; int E;
  dbl_parts(a, M, E);
  const int d = E - e0;
  M = d < 0 ? M >> ((-d) & 63) : M;
  const int sh = d < 0 ? 0 : d;
  const bool low = sh < 64;
  const uint64_t lo = low ? M << (sh & 63) : 0;
  const uint64_t hi = low ? ((M >> 1) >> (63 - (sh & 63))) : M << ((sh - 64) & 63);
  return (((u128)hi) << 64) | lo;
}

// The same weight |a| / 2^e0 (a whole number) as three 37-bit chunks held
// in doubles: |a| / 2^e0 = c2 2^74 + c1 2^37 + c0.  Scaling by powers of two,
// floor and the fused remainders are exact.  With the column range check
// (|a| / 2^e0 < 2^(124 - b), b the bit length of the column's nonzero count,
// at most 16 for fewer than 65536 rows) every chunk sum over a column stays
// below 2^53 (c0, c1 < 2^37 summed fewer than 2^16 times; c2 < 2^(50 - b)),
// so FP64 adds of chunks are exact in any order.
__device__ __forceinline__ void weight_chunks(double a, int e0, double &c0, double &c1, double &c2) {
  const double ws = ldexp(fabs(a), -e0);
  c2 = floor(ws * 0x1p-74);
  const double r = fma(-c2, 0x1p74, ws);
  c1 = floor(r * 0x1p-37);
  c0 = fma(-c1, 0x1p37, r);
}

// A column through a raw buffer descriptor (word 3: 32-bit data format, no
// swizzle); n < 65536 rows, so n 8 bytes fits the size field.  Loads past
// the column's end return 0, so a wave can run a uniform loop over row
// steps with no bounds branch.
constexpr int COL_RSRC_WORD3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_rsrc(const double *p, int n) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, n * 8, COL_RSRC_WORD3);
}
__device__ __forceinline__ double col_ld(__amdgpu_buffer_rsrc_t r, int off) {
  const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  double d;
  __builtin_memcpy(&d, &u, sizeof d);
  return d;
}

// an exact whole double below 2^64 as an integer
__device__ __forceinline__ uint64_t u64_of_whole(double v) {
  const double hi = floor(v * 0x1p-32);
  const double lo = fma(-hi, 0x1p32, v);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// c2 2^74 + c1 2^37 + c0 for whole chunk sums below 2^53
__device__ __forceinline__ u128 chunks_to_u128(double c0, double c1, double c2) {
  return ((u128)u64_of_whole(c2) << 74) + ((u128)u64_of_whole(c1) << 37) + (u128)u64_of_whole(c0);
}

// floor(lambda / 2^e0), saturated at 2^126 (beyond every weight sum of a
// column that passed the range check, so it acts as +infinity).
__device__ __forceinline__ u128 lambda_fixed(double lam, int e0) {
  if (!(lam > 0.0)) return 0;
  uint64_t M; int E;
  dbl_parts(lam, M, E);
  int hb = E + 63 - __builtin_clzll(M);
  if (hb - e0 >= 126) return ((u128)1) << 126;
  int sh = E - e0;
  if (sh >= 0) return ((u128)M) << sh;
  if (-sh >= 64) return 0;
  return (u128)(M >> (-sh));
}

__device__ __forceinline__ double u128_to_double_approx(u128 x) {
  return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}

// ------------------------------------------------------------ wave primitives
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  return (uint64_t)__shfl_xor((unsigned long long)x, m);
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
  return (uint64_t)__shfl((unsigned long long)x, src);
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t x, int d) {
  return (uint64_t)__shfl_up((unsigned long long)x, d);
}

__device__ __forceinline__ u128 shfl_u128(u128 x, int src) {
  uint64_t lo = shfl_u64((uint64_t)x, src), hi = shfl_u64((uint64_t)(x >> 64), src);
  return (((u128)hi) << 64) | lo;
}

// Values equal on every lane, moved to scalar registers.
__device__ __forceinline__ int uni_int(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni_u64(uint64_t x) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ u128 uni_u128(u128 x) {
  return (((u128)uni_u64((uint64_t)(x >> 64))) << 64) | uni_u64((uint64_t)x);
}

// Exact sum over the wave (integer adds: any order gives the same result).
__device__ __forceinline__ u128 wave_sum_u128(u128 x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t lo = shfl_xor_u64((uint64_t)x, d), hi = shfl_xor_u64((uint64_t)(x >> 64), d);
    x += (((u128)hi) << 64) | lo;
  }
  return uni_u128(x);
}

__device__ __forceinline__ int wave_sum_int(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return uni_int(x);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t o = shfl_xor_u64(x, d);
    x = o < x ? o : x;
  }
  return uni_u64(x);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint64_t o = shfl_xor_u64(x, d);
    x = o > x ? o : x;
  }
  return uni_u64(x);
}

// Sum over the wave in an unspecified order (for approximate sums only).
__device__ __forceinline__ double wave_sum_dbl(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = x + __shfl_xor(x, d);
  return __shfl(x, 0);
}

__device__ __forceinline__ int wave_min_int(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d));
  return uni_int(x);
}

__device__ __forceinline__ int wave_max_int(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, __shfl_xor(x, d));
  return uni_int(x);
}

// Inclusive scans across the 64 lanes.
__device__ __forceinline__ u128 wave_incl_scan_u128(u128 x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t lo = shfl_up_u64((uint64_t)x, d), hi = shfl_up_u64((uint64_t)(x >> 64), d);
    if (lane >= d) x += (((u128)hi) << 64) | lo;
  }
  return x;
}

__device__ __forceinline__ int wave_excl_scan_int(int x, int lane) {
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int o = __shfl_up(incl, d);
    if (lane >= d) incl += o;
  }
  return incl - x;
}

__device__ __forceinline__ double wave_incl_scan_dbl(double x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double o = __shfl_up(x, d);
    if (lane >= d) x = x + o;
  }
  return x;
}

// R64 tree: p[l] = p[l] + p[l+d] for d = 32..1; the result is in lane 0.
__device__ __forceinline__ double wave_r64_tree(double p) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    double o = __shfl_down(p, d);
    p = p + o;
  }
  return p;
}

// Bitonic sort of one (key, payload) pair per lane, ascending by key then row.
__device__ __forceinline__ void wave_sort_key_row(uint64_t &key, int &row, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t ok = shfl_xor_u64(key, stride);
      int orow = __shfl_xor(row, stride);
      bool up = (lane & size) == 0;
      bool lower = (lane & stride) == 0;
      bool other_less = ok < key || (ok == key && orow < row);
      bool other_greater = ok > key || (ok == key && orow > row);
      bool take = (lower == up) ? other_less : other_greater;
      if (take) { key = ok; row = orow; }
    }
  }
}

// Bitonic sort of (key, weight) by key only (order among equal keys is fixed
// by the network; used for pivot sampling only).
__device__ __forceinline__ void wave_sort_key_dbl(uint64_t &key, double &w, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t ok = shfl_xor_u64(key, stride);
      double ow = __shfl_xor(w, stride);
      bool up = (lane & size) == 0;
      bool lower = (lane & stride) == 0;
      bool take = (lower == up) ? (ok < key) : (ok > key);
      if (take) { key = ok; w = ow; }
    }
  }
}

// Keep the scheduler from hoisting every load of an unrolled slot loop (each
// weight is 4 VGPRs): fence after every 4 slots.
#define L1_SLOT_FENCE(t) \
  do {                    \
    if (((t) & 3) == 3) __builtin_amdgcn_sched_barrier(0); \
  } while (0)

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------ VALU lane exchanges
// x of lane (lane ^ m), m in {1, 2, 4, 8, 16, 32} (a constant once the
// caller's loop is unrolled), without an LDS round trip: DPP quad permutes
// for 1 and 2, two row shifts merged through bank masks for 4, the row
// rotation by 8, and gfx950's row swaps (v_permlane16_swap,
// v_permlane32_swap) for 16 and 32.  Lane layouts checked on the hardware.
// Every lane of the wave must be active.
__device__ __forceinline__ uint32_t xswap32(uint32_t x, int m) {
  const int v = (int)x;
  switch (m) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    case 4: {
      const int t = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xF, 0x5, false);    // row_shl:4, banks 0 and 2
      return (uint32_t)__builtin_amdgcn_update_dpp(t, v, 0x114, 0xF, 0xA, false); // row_shr:4, banks 1 and 3
    }
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // row_ror:8
    case 16: {
      const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
      return (threadIdx.x & 16) ? p[0] : p[1];
    }
    default: {
      const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
      return (threadIdx.x & 32) ? p[0] : p[1];
    }
  }
}
__device__ __forceinline__ uint64_t xswap64(uint64_t x, int m) {
  return ((uint64_t)xswap32((uint32_t)(x >> 32), m) << 32) | xswap32((uint32_t)x, m);
}
__device__ __forceinline__ double xswapd(double x, int m) {
  return __longlong_as_double((long long)xswap64((uint64_t)__double_as_longlong(x), m));
}
__device__ __forceinline__ u128 xswap128(u128 x, int m) {
  return (((u128)xswap64((uint64_t)(x >> 64), m)) << 64) | xswap64((uint64_t)x, m);
}
__device__ __forceinline__ u128 readlane_u128(u128 x, int l) {
  const uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  const uint32_t w0 = __builtin_amdgcn_readlane((int)(uint32_t)lo, l), w1 = __builtin_amdgcn_readlane((int)(uint32_t)(lo >> 32), l),
                 w2 = __builtin_amdgcn_readlane((int)(uint32_t)hi, l), w3 = __builtin_amdgcn_readlane((int)(uint32_t)(hi >> 32), l);
  return (((u128)(((uint64_t)w3 << 32) | w2)) << 64) | (((uint64_t)w1 << 32) | w0);
}

// The same reductions, scans and sorts as above through VALU exchanges
// (the segment kernel's wave-convergent hot paths).
__device__ __forceinline__ u128 wave_sum_u128_x(u128 x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += xswap128(x, d);
  return uni_u128(x);
}

__device__ __forceinline__ double wave_sum_dbl_x(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = x + xswapd(x, d);
  return __longlong_as_double((long long)uni_u64((uint64_t)__double_as_longlong(x)));
}

// R64 tree (p[l] = p[l] + p[l + d] for d = 32..1, the result in lane 0): for
// l < d the partner l ^ d is l + d, so lane 0 adds the same values in the
// same order as wave_r64_tree.
__device__ __forceinline__ double wave_r64_tree_x(double p) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) p = p + xswapd(p, d);
  return p;
}

// inclusive scan: at level d a lane adds the total of the partner half-block
// when its own bit d is set (exact integer adds)
__device__ __forceinline__ u128 wave_incl_scan_u128_x(u128 x, int lane) {
  u128 tot = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const u128 o = xswap128(tot, d);
    x += (lane & d) ? o : (u128)0;
    tot += o;
  }
  return x;
}

// Minimum / maximum over the wave through VALU exchanges (uniform result)
__device__ __forceinline__ uint64_t wave_min_u64_x(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = xswap64(x, d);
    x = o < x ? o : x;
  }
  return uni_u64(x);
}
__device__ __forceinline__ uint64_t wave_max_u64_x(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = xswap64(x, d);
    x = o > x ? o : x;
  }
  return uni_u64(x);
}

// x of lane l (l uniform), without an LDS round trip
__device__ __forceinline__ double readlane_dbl(double x, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// FP64 inclusive scan by the same butterfly (each result takes at most six
// rounded adds of partial sums)
__device__ __forceinline__ double wave_incl_scan_dbl_x(double x, int lane) {
  double tot = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double o = xswapd(tot, d);
    x = (lane & d) ? x + o : x;
    tot = tot + o;
  }
  return x;
}

// (A lane keeping the minimum takes its partner's pair when that is less,
// one keeping the maximum when it is not less: the same result, since two
// equal pairs are interchangeable, with one comparison instead of two.)
__device__ __forceinline__ void wave_sort_key_row_x(uint64_t &key, int &row, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t ok = xswap64(key, stride);
      const int orow = (int)xswap32((uint32_t)row, stride);
      const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
      const bool other_less = ok < key || (ok == key && orow < row);
      const bool take = other_less == keep_min;
      key = take ? ok : key;
      row = take ? orow : row;
    }
  }
}
