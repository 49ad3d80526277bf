// l1line.hip -- C ABI (include/l1line.h) and host runtime of the gfx950
// library: argument checks, the context workspace, kernel dispatch.
#include <hip/hip_runtime.h>

#include <l1line.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "fit_kernels.h"

struct ProfRec {
  const char *name;
  hipEvent_t start, stop;
};

struct l1line_ctx_s {
  int device;
  void *ws;          // device workspace, grown on demand
  size_t ws_bytes;
  bool profiling;
  std::vector<ProfRec> prof;
};

// Brackets one kernel launch with events when the context is profiling.
struct ProfScope {
  l1line_ctx ctx;
  hipStream_t s;
  ProfRec rec;
  bool on;
  ProfScope(l1line_ctx c, hipStream_t st, const char *name) : ctx(c), s(st), on(c && c->profiling) {
    if (!on) return;
    rec.name = name;
    if (hipEventCreate(&rec.start) != hipSuccess || hipEventCreate(&rec.stop) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(rec.start, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.stop, s);
    ctx->prof.push_back(rec);
  }
};

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return L1LINE_EHIP;           \
  } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int ensure_ws(l1line_ctx ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->ws_bytes) return L1LINE_OK;
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->ws_bytes = want;
  return L1LINE_OK;
}

static int check_matrix(const double *X, int64_t n, int64_t m, int64_t ld) {
  if (!X || n < 1 || m < 1 || ld < n) return L1LINE_EINVAL;
  if (m > (1ll << 24) || ld > (1ll << 40)) return L1LINE_EINVAL;
  if (n > L1LINE_MAX_N) return L1LINE_ESIZE;
  return L1LINE_OK;
}

static int check_lambdas(const double *lam, int64_t L) {
  if (!lam || L < 1 || L > L1LINE_MAX_LAMBDAS) return L1LINE_EINVAL;
  for (int64_t t = 0; t < L; ++t)
    if (!(lam[t] >= 0.0) || isinf(lam[t])) return L1LINE_EINVAL;
  return L1LINE_OK;
}

// Workspace layout of one fit / path call.
struct FitWs {
  ColInfo *ci;
  double *V, *E, *Z;
  int *R, *segflags, *zflag;
  size_t bytes;
};

static FitWs layout_fit(void *base, int64_t m, int64_t L) {
  FitWs w;
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b, 256); return o; };
  size_t o_ci = take(sizeof(ColInfo) * m);
  size_t o_v = take(sizeof(double) * L * m * m);
  size_t o_e = take(sizeof(double) * L * m * m);
  size_t o_r = take(sizeof(int) * L * m * m);
  size_t o_z = take(sizeof(double) * L * m);
  size_t o_sf = take(sizeof(int) * m);
  size_t o_zf = take(sizeof(int) * L * m);
  char *b = (char *)base;
  w.ci = (ColInfo *)(b + o_ci);
  w.V = (double *)(b + o_v);
  w.E = (double *)(b + o_e);
  w.R = (int *)(b + o_r);
  w.Z = (double *)(b + o_z);
  w.segflags = (int *)(b + o_sf);
  w.zflag = (int *)(b + o_zf);
  w.bytes = off;
  return w;
}

__global__ void k_fill_int(int *p, long long count, int value) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

static int launch_seg(l1line_ctx ctx, const double *X, int n, int m, long long ld, const FitWs &w,
                      const LamArgs &la, hipStream_t s) {
  const size_t lds = seg_lds_bytes(n, la.L);
  static bool attr_set = false;
  if (!attr_set) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_fit_seg, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)seg_lds_bytes(L1LINE_MAX_N, L1LINE_MAX_LAMBDAS)));
    attr_set = true;
  }
  // enough workgroups to fill the chip several times over (and to even out
  // the uneven cost of the segments), at least 8 k per workgroup
  int ksplit = (6144 + m - 1) / m;
  ksplit = ksplit < 1 ? 1 : ksplit;
  const int kmax = m / 8 > 1 ? m / 8 : 1;
  ksplit = ksplit > kmax ? kmax : ksplit;
  {
    ProfScope ps(ctx, s, "fit_seg");
    hipLaunchKernelGGL(k_fit_seg, dim3((unsigned)(m * ksplit)), dim3(64 * SEG_WAVES), lds, s, X, n, m, ld,
                       w.ci, la, ksplit, w.V, w.E, w.R, w.segflags);
  }
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

static int run_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, const LamArgs &la,
                    double *V, int64_t *J, double *OBJ, int32_t *ROW, double *ZALL, int32_t *status,
                    hipStream_t s) {
  const int64_t L = la.L;
  FitWs probe = layout_fit(nullptr, m, L);
  int st = ensure_ws(ctx, probe.bytes, s);
  if (st) return st;
  FitWs w = layout_fit(ctx->ws, m, L);
  {
    ProfScope ps(ctx, s, "colprep");
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, w.segflags,
                       (long long)m, 0);
    hipLaunchKernelGGL(k_colprep, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, X, (int)n, (int)m,
                       (long long)ld, w.ci);
  }
  HIP_TRY(hipGetLastError());
  st = launch_seg(ctx, X, (int)n, (int)m, (long long)ld, w, la, s);
  if (st) return st;
  {
    ProfScope ps(ctx, s, "reduce");
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)m, (unsigned)L), dim3(64), 0, s, w.V, w.E, (int)m, la, w.Z,
                       w.zflag);
  }
  {
    ProfScope ps(ctx, s, "argmin");
    hipLaunchKernelGGL(k_argmin, dim3((unsigned)L), dim3(256), 0, s, w.V, w.R, w.Z, w.zflag, w.ci,
                       w.segflags, (int)m, (int)L, V, J, OBJ, ROW, ZALL, status);
  }
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

extern "C" {

int l1line_create(l1line_ctx *ctx, int device) {
  if (!ctx) return L1LINE_EINVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return L1LINE_EHIP;
  if (device < 0 || device >= count) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(device));
  l1line_ctx c = new (std::nothrow) l1line_ctx_s();
  if (!c) return L1LINE_ENOMEM;
  c->device = device;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->profiling = false;
  *ctx = c;
  return L1LINE_OK;
}

static void prof_clear(l1line_ctx ctx) {
  for (auto &r : ctx->prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  ctx->prof.clear();
}

int l1line_destroy(l1line_ctx ctx) {
  if (!ctx) return L1LINE_EINVAL;
  int st = L1LINE_OK;
  if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) st = L1LINE_EHIP;
  prof_clear(ctx);
  if (ctx->ws && hipFree(ctx->ws) != hipSuccess) st = L1LINE_EHIP;
  delete ctx;
  return st;
}

int l1line_profile(l1line_ctx ctx, int enable) {
  if (!ctx) return L1LINE_EINVAL;
  ctx->profiling = enable != 0;
  return L1LINE_OK;
}

int l1line_profile_read(l1line_ctx ctx, const char *kernel, double *total_ms, int64_t *launches, int reset) {
  if (!ctx) return L1LINE_EINVAL;
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto &r : ctx->prof) {
    if (kernel && strcmp(kernel, r.name) != 0) continue;
    HIP_TRY(hipEventSynchronize(r.stop));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.start, r.stop));
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  if (reset) prof_clear(ctx);
  return L1LINE_OK;
}

const char *l1line_strerror(int code) {
  switch (code) {
    case L1LINE_OK: return "ok";
    case L1LINE_EINVAL: return "invalid argument";
    case L1LINE_EHIP: return "HIP runtime error";
    case L1LINE_ENONFINITE: return "X holds a NaN or an infinity";
    case L1LINE_ERANGE: return "a selected ratio overflowed";
    case L1LINE_ENOMEM: return "workspace allocation failed";
    case L1LINE_EWIDE: return "column magnitudes too spread for exact 128-bit weight sums";
    case L1LINE_ESIZE: return "n exceeds L1LINE_MAX_N";
    case L1LINE_EINTERNAL: return "selection round bound exceeded";
    default: return "unknown status";
  }
}

int l1line_column_stats(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double *W,
                        int32_t *zeros, int32_t *status, void *stream) {
  if (!ctx) return L1LINE_EINVAL;
  if (!X || n < 1 || m < 1 || ld < n || m > (1ll << 24) || n > (1ll << 30)) return L1LINE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  int st = ensure_ws(ctx, align_up(sizeof(ColInfo) * m, 256), s);
  if (st) return st;
  ColInfo *ci = (ColInfo *)ctx->ws;
  hipLaunchKernelGGL(k_colprep, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                     ci);
  hipLaunchKernelGGL(k_colstats_out, dim3(1), dim3(256), 0, s, ci, (int)m, W, zeros, status);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_fit(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, double *v,
               int64_t *j, double *obj, int32_t *median_row, double *z_all, int32_t *status, void *stream) {
  if (!ctx || !v || !j || !obj) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  LamArgs la;
  memset(&la, 0, sizeof la);
  la.L = 1;
  la.lam[0] = lambda;
  return run_path(ctx, X, n, m, ld, la, v, j, obj, median_row, z_all, status, (hipStream_t)stream);
}

int l1line_fit_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, const double *lambdas,
                    int64_t L, double *V, int64_t *J, double *OBJ, int32_t *ROW, double *ZALL, int32_t *status,
                    void *stream) {
  if (!ctx || !V || !J || !OBJ) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(lambdas, L);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  LamArgs la;
  memset(&la, 0, sizeof la);
  la.L = (int)L;
  for (int64_t t = 0; t < L; ++t) la.lam[t] = lambdas[t];
  return run_path(ctx, X, n, m, ld, la, V, J, OBJ, ROW, ZALL, status, (hipStream_t)stream);
}

}  // extern "C"
