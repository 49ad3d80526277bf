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
};

struct LamArgs {
  int L;
  double lam[L1LINE_MAX_LAMBDAS];
};

// ------------------------------------------------------------------ columns
// One wave per column: finiteness, counts, the fixed-point exponent e0, the
// range check, the exact fixed-point mass and the R64 column mass.
__global__ void __launch_bounds__(256)
k_colprep(const double *__restrict__ X, int n, int m, long long ld, ColInfo *__restrict__ ci) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= m) return;
  const double *x = X + (long long)col * ld;
  int bad = 0, nnz = 0, zeros = 0, lsb = 1 << 20, hb = -(1 << 20);
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
    }
  }
  double W = wave_r64_tree(part);
  bad = wave_max_int(bad);
  nnz = wave_sum_int(nnz);
  zeros = wave_sum_int(zeros);
  lsb = wave_min_int(lsb);
  hb = wave_max_int(hb);
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
    ci[col] = c;
  }
}

// ---------------------------------------------------------- exact selection
// Find the first element, in (ratio, row) order, whose inclusive prefix
// weight reaches tau.  Candidates are the elements with klo < key <= khi;
// Slo/Clo (Shi/Chi) are the exact weight and count of ALL elements with
// key <= klo (<= khi).  Element (lane, t) is row lane + 64 t.
template <int T>
__device__ __forceinline__ void wave_select(const uint64_t (&keys)[T], const u128 *__restrict__ swf,
                                            const double *__restrict__ sxj, const double *__restrict__ xk,
                                            int n, int tmax, uint64_t klo, uint64_t khi,
                                            u128 Slo, u128 Shi, int Clo, int Chi, u128 tau, int lane,
                                            uint64_t *__restrict__ wkey, int *__restrict__ wrow,
                                            uint64_t &okey, int &orow, int &err) {
  constexpr double DELTA = 0.15;
  int count = Chi - Clo;
  bool bisect = false;
  int rounds = 0;
  okey = KEY_NONE;
  orow = -1;
  bool single_key = false;
  while (count > 64) {
    if (++rounds > 160) {
      err |= SEG_INTERNAL;
      return;
    }
    uint64_t plo, phi;
    if (!bisect) {
      // one candidate per lane, from a lane/round dependent slot
      const int start = (lane * 11 + rounds * 5) & (T - 1);
      uint64_t sk = KEY_NONE;
      int spri = T, st = 0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        bool c = keys[t] > klo && keys[t] <= khi;
        int pri = (t - start) & (T - 1);
        if (c && pri < spri) {
          spri = pri;
          sk = keys[t];
          st = t;
        }
      }
      double sw = (sk != KEY_NONE) ? fabs(sxj[lane + 64 * st]) : 0.0;
      wave_sort_key_dbl(sk, sw, lane);
      double cw = wave_incl_scan_dbl(sw, lane);
      double tot = __shfl(cw, 63);
      double f = u128_to_double_approx(tau - Slo) / u128_to_double_approx(Shi - Slo);
      double flo = (f - DELTA) * tot, fhi = (f + DELTA) * tot;
      uint64_t mlo = __ballot(sk != KEY_NONE && cw <= flo);
      uint64_t mhi = __ballot(sk != KEY_NONE && cw >= fhi);
      plo = mlo ? uni_u64(shfl_u64(sk, 63 - __builtin_clzll(mlo))) : klo;
      phi = mhi ? uni_u64(shfl_u64(sk, __builtin_ctzll(mhi))) : khi;
      if (phi < plo) phi = plo;
    } else {
      // key-space bisection between the extreme candidates: always progresses
      uint64_t cmin = KEY_NONE, cmax = 0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        bool c = keys[t] > klo && keys[t] <= khi;
        if (c) {
          cmin = keys[t] < cmin ? keys[t] : cmin;
          cmax = keys[t] > cmax ? keys[t] : cmax;
        }
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
    // exact weights and counts of all elements at or below each pivot
    u128 s1 = 0, s2 = 0;
    int c1 = 0, c2 = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      uint64_t kk = keys[t];
      if (kk != KEY_NONE) {
        u128 w = swf[lane + 64 * t];
        if (kk <= plo) { s1 += w; ++c1; }
        if (kk <= phi) { s2 += w; ++c2; }
      }
      L1_SLOT_FENCE(t);
    }
    s1 = wave_sum_u128(s1);
    s2 = wave_sum_u128(s2);
    c1 = wave_sum_int(c1);
    c2 = wave_sum_int(c2);
    if (s1 >= tau) {
      khi = plo; Shi = s1; Chi = c1;
    } else if (s2 >= tau) {
      klo = plo; Slo = s1; Clo = c1;
      khi = phi; Shi = s2; Chi = c2;
    } else {
      klo = phi; Slo = s2; Clo = c2;
    }
    int ncount = Chi - Clo;
    bisect = (ncount == count);
    count = ncount;
  }

  if (!single_key) {
    // <= 64 candidates: one per lane, bitonic sort by (key, row), exact scan
    int mine = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) mine += (keys[t] > klo && keys[t] <= khi) ? 1 : 0;
    int off = wave_excl_scan_int(mine, lane);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (keys[t] > klo && keys[t] <= khi && off < 64) {
        wkey[off] = keys[t];
        wrow[off] = lane + 64 * t;
        ++off;
      }
    }
    wave_lds_sync();
    uint64_t ck = lane < count ? wkey[lane] : KEY_NONE;
    int cr = lane < count ? wrow[lane] : 0x7fffffff;
    wave_lds_sync();
    wave_sort_key_row(ck, cr, lane);
    u128 w = lane < count ? swf[cr] : (u128)0;
    u128 S = wave_incl_scan_u128(w, lane) + Slo;
    uint64_t hit = __ballot(lane < count && S >= tau);
    if (!hit) {
      err |= SEG_INTERNAL;
      return;
    }
    int src = __builtin_ctzll(hit);
    okey = uni_u64(shfl_u64(ck, src));
    orow = uni_int(__shfl(cr, src));
    return;
  }

  // every candidate has the same key K: (key, row) order is row order, and
  // rows ascend with (t, lane).  Rare: walk the rows again from memory.
  const uint64_t K = khi;
  u128 S = Slo;
  for (int t = 0; t < tmax; ++t) {
    int i = lane + 64 * t;
    bool c = false;
    if (i < n && sxj[i] != 0.0) {
      double r = xk[i] / sxj[i];
      r = r + 0.0;
      c = key_of(r) == K;
    }
    u128 w = c ? swf[i] : (u128)0;
    u128 sc = wave_incl_scan_u128(w, lane) + S;
    uint64_t hit = __ballot(c && sc >= tau);
    if (hit) {
      int src = __builtin_ctzll(hit);
      okey = K;
      orow = src + 64 * t;
      return;
    }
    S = uni_u128(shfl_u128(sc, 63));
  }
  err |= SEG_INTERNAL;
}

// e_jk = R64 over i of |x_ik - fl(v x_ij)| (result in lane 0)
template <int T>
__device__ __forceinline__ double wave_residual(const double *__restrict__ xk, int n,
                                                const double *__restrict__ sxj, double v, int lane) {
  double p = 0.0;
#pragma unroll 4
  for (int t = 0; t < T; ++t) {
    int i = lane + 64 * t;
    if (i < n) {
      double prod = v * sxj[i];
      double d = xk[i] - prod;
      p = p + fabs(d);
    }
  }
  return wave_r64_tree(p);
}

// ---------------------------------------------------------------- segments
// One workgroup per preserved column j; each wave walks k = wave, wave+4, ...
// For every (j, k) and every lambda_t it writes
//   V[(t m + j) m + k] = v_k,  E[...] = e_jk,  R[...] = median row (-1 for 0).
// LDS: column j (x and exact fixed-point weight), lambda in fixed point for
// column j, and a 64-entry compaction area per wave.
constexpr int SEG_WAVES = 4;

__host__ __device__ constexpr size_t seg_lds_bytes(int n, int L) {
  return ((size_t)n * 8 + 15) / 16 * 16 + (size_t)n * 16 + (size_t)L * 16 + SEG_WAVES * 64 * 16;
}

template <int T>
__global__ void __launch_bounds__(256)
k_fit_seg(const double *__restrict__ X, int n, int m, long long ld, const ColInfo *__restrict__ ci,
          LamArgs la, double *__restrict__ V, double *__restrict__ E, int *__restrict__ R,
          int *__restrict__ segflags) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int j = blockIdx.x;
  const int L = la.L;
  double *sxj = (double *)smem;
  u128 *swf = (u128 *)(smem + ((size_t)n * 8 + 15) / 16 * 16);
  u128 *slam = swf + n;
  unsigned char *wscr = (unsigned char *)(slam + L);

  const ColInfo cj = ci[j];
  const double *xj = X + (long long)j * ld;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double x = xj[i];
    sxj[i] = x;
    swf[i] = (x != 0.0 && !cj.flags) ? fixed_of(fabs(x), cj.e0) : (u128)0;
  }
  for (int t = threadIdx.x; t < L; t += blockDim.x) slam[t] = lambda_fixed(la.lam[t], cj.e0);
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t *wkey = (uint64_t *)(wscr + wave * 64 * 16);
  int *wrow = (int *)(wkey + 64);
  const long long mm = (long long)m * m;
  int err = 0;

  for (int k = wave; k < m; k += SEG_WAVES) {
    const long long base = (long long)j * m + k;
    if (k == j || cj.flags) {
      if (lane == 0) {
        for (int t = 0; t < L; ++t) {
          V[t * mm + base] = (k == j) ? 1.0 : __longlong_as_double(0x7ff8000000000000ll);
          E[t * mm + base] = 0.0;
          R[t * mm + base] = -1;
        }
      }
      continue;
    }
    const double *xk = X + (long long)k * ld;
    // ratios -> keys; exact mass of the negative and zero blocks
    uint64_t keys[T];
    u128 accA = 0, accZ = 0;
    int cN = 0, cZ = 0, cV = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int i = lane + 64 * t;
      uint64_t key = KEY_NONE;
      if (i < n) {
        double a = sxj[i];
        double b = xk[i];
        if (a != 0.0) {
          double r = b / a;
          r = r + 0.0;
          key = key_of(r);
        }
      }
      keys[t] = key;
      if (key != KEY_NONE) {
        ++cV;
        u128 w = swf[i];
        if (key < KEY_ZERO) { accA += w; ++cN; }
        else if (key == KEY_ZERO) { accZ += w; ++cZ; }
      }
      L1_SLOT_FENCE(t);
    }
    const u128 A = wave_sum_u128(accA);
    const u128 B = A + wave_sum_u128(accZ);
    const int N = wave_sum_int(cN), Z = wave_sum_int(cZ), NV = wave_sum_int(cV);
    const u128 W = cj.wfix;

    int prev_row = -2;
    double prev_e = 0.0;
    for (int t = 0; t < L; ++t) {
      const u128 lamf = slam[t];
      const u128 WpL = W + lamf;
      const u128 twoA = A << 1, twoB = B << 1;
      uint64_t okey = KEY_NONE;
      int orow = -1;
      if (!(twoA <= WpL && W <= twoB + lamf)) {      // else 0 minimises g_jk
        const bool neg = twoA > WpL;
        // negative side: first S_p > (W + lambda)/2; positive: first S_p >= (W - lambda)/2
        const u128 tau = neg ? (WpL >> 1) + 1 : (W - lamf + 1) >> 1;
        wave_select<T>(keys, swf, sxj, xk, n, T, neg ? 0ull : KEY_ZERO, neg ? KEY_ZERO - 1 : KEY_NONE - 1,
                       neg ? (u128)0 : B, neg ? A : W, neg ? 0 : N + Z, neg ? N : NV, tau, lane, wkey,
                       wrow, okey, orow, err);
      }
      const double v = (orow >= 0) ? ratio_of_key(okey) : 0.0;
      double e;
      if (orow == prev_row) {
        e = prev_e;
      } else {
        e = wave_residual<T>(xk, n, sxj, v, lane);
        e = __shfl(e, 0);
      }
      prev_row = orow;
      prev_e = e;
      if (lane == 0) {
        V[t * mm + base] = v;
        E[t * mm + base] = e;
        R[t * mm + base] = orow;
      }
    }
  }
  if (err && lane == 0) atomicOr(segflags + j, err);
}

// ------------------------------------------------------------ per-j objective
// One wave per (j, lambda_t): E_j = R64_k e_jk, P_j = R64_k |v_k|,
// z_j = E_j + fl(lambda P_j).  zflag marks an infinite or NaN v_k.
__global__ void __launch_bounds__(64)
k_reduce(const double *__restrict__ V, const double *__restrict__ E, int m, LamArgs la,
         double *__restrict__ Z, int *__restrict__ zflag) {
  const int j = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  const long long off = ((long long)t * m + j) * m;
  double pe = 0.0, pv = 0.0;
  int bad = 0;
  for (int k = lane; k < m; k += 64) {
    pe = pe + E[off + k];
    double a = fabs(V[off + k]);
    pv = pv + a;
    bad |= !isfinite(a);
  }
  pe = wave_r64_tree(pe);
  pv = wave_r64_tree(pv);
  bad = wave_max_int(bad);
  if (lane == 0) {
    double pen = la.lam[t] * pv;
    double z = pe + pen;
    Z[(long long)t * m + j] = z;
    zflag[(long long)t * m + j] = bad;
  }
}

// -------------------------------------------------------------- argmin/gather
// One workgroup per lambda_t: j* = lexicographic argmin of (z_j, j); gathers
// v*, rows, z_all.  Workgroup 0 also folds every flag into the status word.
__global__ void __launch_bounds__(256)
k_argmin(const double *__restrict__ V, const int *__restrict__ R, const double *__restrict__ Z,
         const int *__restrict__ zflag, const ColInfo *__restrict__ ci, const int *__restrict__ segflags,
         int m, int L, double *__restrict__ vout, int64_t *__restrict__ jout, double *__restrict__ objout,
         int *__restrict__ rowout, double *__restrict__ zall, int *__restrict__ status) {
  __shared__ double sz[256];
  __shared__ int sj[256];
  __shared__ int sflag[256];
  const int t = blockIdx.x, tid = threadIdx.x;
  const double *z = Z + (long long)t * m;
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
      int oj = sj[tid + s];
      double oz = sz[tid + s];
      if (oj >= 0 && (sj[tid] < 0 || oz < sz[tid] || (oz == sz[tid] && oj < sj[tid]))) {
        sz[tid] = oz;
        sj[tid] = oj;
      }
    }
    __syncthreads();
  }
  const int js = sj[0];
  const long long mm = (long long)m * m;
  const long long src = t * mm + (long long)js * m;
  for (int k = tid; k < m; k += blockDim.x) {
    vout[(long long)t * m + k] = V[src + k];
    if (rowout) rowout[(long long)t * m + k] = R[src + k];
    if (zall) zall[(long long)t * m + k] = z[k];
  }
  if (tid == 0) {
    jout[t] = js;
    objout[t] = z[js];
  }
  if (t == 0 && status) {
    // condition bits; the status is the first that applies of: non-finite
    // input, too-wide column, selection bound, overflowed ratio
    int f = 0;
    for (int j = tid; j < m; j += blockDim.x) {
      int cf = ci[j].flags;
      if (cf & COL_NONFINITE) f |= 1;
      if (cf & COL_WIDE) f |= 2;
      if (segflags[j]) f |= 4;
    }
    for (long long q = tid; q < (long long)L * m; q += blockDim.x)
      if (zflag[q]) f |= 8;
    sflag[tid] = f;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
      if (tid < s) sflag[tid] |= sflag[tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      int b = sflag[0];
      *status = (b & 1) ? L1LINE_ENONFINITE : (b & 2) ? L1LINE_EWIDE : (b & 4) ? L1LINE_EINTERNAL
              : (b & 8) ? L1LINE_ERANGE : L1LINE_OK;
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
