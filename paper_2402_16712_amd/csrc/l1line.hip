// l1line.hip -- C ABI (include/l1line.h) and host runtime of the gfx950
// library: argument checks, the context workspace, batch layout (problem
// descriptors and work items), kernel dispatch, captured launch graphs, the
// autotuner and kernel timing.
#include <hip/hip_runtime.h>

#include <l1line.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fit_kernels.h"
#include "ranker_kernels.h"
#include "bp_kernels.h"
#include "comp_kernels.h"
#include "path_kernels.h"
#include "peak_kernels.h"

// ------------------------------------------------------------------- context
struct ProfRec {
  const char *name;
  hipEvent_t start, stop;
};

struct TuneParams {
  int blocks_per_cu;   // persistent workgroups per compute unit
  int kchunk_min;      // fewest k per work item
  int items_per_cu;    // target number of work items per compute unit
};

// Size class of a launch, the key of autotuned launch parameters: one
// problem or a batch, one penalty or several, and the bit lengths of the
// largest n, the largest m and (halved) of the total work sum n m^2 L.
struct TuneKey {
  int batch, multi, nb, mb, wb;
  bool operator==(const TuneKey &o) const {
    return batch == o.batch && multi == o.multi && nb == o.nb && mb == o.mb && wb == o.wb;
  }
};

struct l1line_ctx_s {
  int device;
  int num_cu;
  void *ws;                 // device workspace, grown on demand
  size_t ws_bytes;
  void *stage;              // pinned host staging of the batch layout
  size_t stage_bytes;
  hipEvent_t stage_done;    // the last copy out of `stage` has finished
  bool stage_pending;
  hipStream_t cap_stream;   // stream used to capture launch graphs
  hipGraphExec_t graph;     // cached graph of the last captured batch layout
  uint64_t graph_key;
  TuneParams tune;          // default launch parameters (size classes without a tuned entry)
  std::vector<std::pair<TuneKey, TuneParams>> tuned;   // autotuned entries per size class
  std::vector<std::string> tune_foreign;               // cache lines of other architectures, kept
  std::string arch;         // gcnArchName of the device (cache key)
  bool profiling;
  std::vector<ProfRec> prof;
  void *rk;                 // ranker scratch (features, sign sums, MLP buffers)
  size_t rk_bytes;
  void *sp;                 // solution-path scratch (per breakpoint entry, per tile and column)
  size_t sp_bytes;
  void *bl;                 // Algorithm 2: each segment's entries listed by the count pass
  size_t bl_bytes;
  int *sticky;              // device: first data-dependent error of any call on the context
  int host_err;             // first argument / runtime error an entry point returned
  std::string tune_path;    // launch-parameter cache file ("" = none)
  float *rk_w;              // ranker: FP32 weights, Adam moments m1, m2 (device, 3 x L1LINE_MLP_PARAMS)
  bool rk_have_w, rk_have_state;
  int64_t rk_step;          // Adam steps taken (checkpoint state)
  // the dynamic-LDS limits raised on this context's device for the kernels
  // that take more than 64 KB (segment kernels, path sort, MLP backward)
  bool attr_seg, attr_sort, attr_bwd;
  uint64_t rk_seed, rk_cursor;  // training-set seed and next example (checkpoint state)
  void *scratch;            // this device's address of the no-alloc workspace (null if unavailable)
};

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return L1LINE_EHIP;           \
  } while (0)

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

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------- no-alloc workspace
// Workspace of l1line_fit_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  In host code the name is
// only a host-side stand-in: kernels and copies take the device address that
// hipGetSymbolAddress returns, fetched once per device (with that device
// current) when the first context on it is created.
constexpr size_t NOALLOC_BYTES = (size_t)L1LINE_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// The calling thread's current device must be `device`.
static void *scratch_address(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

static void drop_graph(l1line_ctx ctx) {
  if (ctx->graph) {
    (void)hipGraphExecDestroy(ctx->graph);
    ctx->graph = nullptr;
  }
  ctx->graph_key = 0;
}

static int ensure_ws(l1line_ctx ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->ws_bytes) return L1LINE_OK;
  drop_graph(ctx);
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->ws_bytes = want;
  return L1LINE_OK;
}

static int ensure_rk(l1line_ctx ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->rk_bytes) return L1LINE_OK;
  if (ctx->rk) {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->rk));
    ctx->rk = nullptr;
    ctx->rk_bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&ctx->rk, want) != hipSuccess) {
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->rk_bytes = want;
  return L1LINE_OK;
}

static int ensure_bl(l1line_ctx ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->bl_bytes) return L1LINE_OK;
  if (ctx->bl) {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->bl));
    ctx->bl = nullptr;
    ctx->bl_bytes = 0;
  }
  const size_t want = align_up(bytes, 1 << 20);
  if (hipMalloc(&ctx->bl, want) != hipSuccess) {
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->bl_bytes = want;
  return L1LINE_OK;
}

// Algorithm 2's entry lists: the count pass keeps the entries (key, row) of
// each segment that has at most BP_LIST of them, and the weight below them,
// so that the entry pass skips its scan of the rows for those segments.  Within a budget of
// BP_LIST_BUDGET bytes, else not used (capacity 0).
constexpr int BP_LIST = BP_LIST_MAX;
constexpr size_t BP_LIST_BUDGET = (size_t)6 << 30;
struct BpList {
  uint64_t *keys = nullptr;
  unsigned short *rows = nullptr;
  u128 *sb = nullptr;
  int cap = 0;
};
static int bp_list(l1line_ctx ctx, long long nseg, hipStream_t s, BpList *L) {
  const size_t kb = align_up(sizeof(uint64_t) * BP_LIST * (size_t)nseg, 256),
               rb = align_up(sizeof(unsigned short) * BP_LIST * (size_t)nseg, 256),
               sb = align_up(sizeof(u128) * (size_t)nseg, 256);
  *L = BpList();
  if (kb + rb + sb > BP_LIST_BUDGET) return L1LINE_OK;
  const int st = ensure_bl(ctx, kb + rb + sb, s);
  if (st == L1LINE_ENOMEM) return L1LINE_OK;   // run without the lists
  if (st) return st;
  char *b = (char *)ctx->bl;
  L->keys = (uint64_t *)b;
  L->rows = (unsigned short *)(b + kb);
  L->sb = (u128 *)(b + kb + rb);
  L->cap = BP_LIST;
  return L1LINE_OK;
}

static int ensure_sp(l1line_ctx ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->sp_bytes) return L1LINE_OK;
  if (ctx->sp) {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->sp));
    ctx->sp = nullptr;
    ctx->sp_bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  if (hipMalloc(&ctx->sp, want) != hipSuccess) {
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->sp_bytes = want;
  return L1LINE_OK;
}

static int ensure_stage(l1line_ctx ctx, size_t bytes) {
  if (ctx->stage_pending) {
    HIP_TRY(hipEventSynchronize(ctx->stage_done));
    ctx->stage_pending = false;
  }
  if (bytes <= ctx->stage_bytes) return L1LINE_OK;
  if (ctx->stage) HIP_TRY(hipHostFree(ctx->stage));
  ctx->stage = nullptr;
  ctx->stage_bytes = 0;
  const size_t want = align_up(bytes + bytes / 4, 1 << 16);
  if (hipHostMalloc(&ctx->stage, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return L1LINE_ENOMEM;
  }
  ctx->stage_bytes = want;
  return L1LINE_OK;
}

// ---------------------------------------------------------------- validation
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

static int check_problem(const l1line_problem &p) {
  int st = check_matrix(p.X, p.n, p.m, p.ld);
  if (st) return st;
  st = check_lambdas(p.lambdas, p.L);
  if (st) return st;
  if (!p.V || !p.J || !p.OBJ) return L1LINE_EINVAL;
  return L1LINE_OK;
}

// -------------------------------------------------------------- batch layout
// Device workspace of one batch call:
//   meta  (copied from the pinned staging buffer): ProbDesc[B], colstart,
//         zstart, ostart (B+1 ints each), penalties, work items, counter
//   data: ColInfo, segflags, V, E, R, Z, zflag
struct BatchLayout {
  int B, nitems, ksplit, nmax, Lmax;
  int ss_split, ss_ncand, ss_m;   // sign sums of a candidate list: row parts, candidates, m
  int xstart[SEG_XCDS + 1];   // explicit items: XCD x owns [xstart[x], xstart[x + 1])
  long long total_cols, total_z, total_out, total_ws, total_lam, total_pairs, total_tiles, total_words;
  size_t o_desc, o_colstart, o_zstart, o_ostart, o_tstart, o_wstart, o_lam, o_items, o_counter, o_xstart,
      meta_bytes;
  size_t o_ci, o_segflags, o_DZ, o_DZp, o_mask, o_V, o_E, o_R, o_Z, o_zflag, bytes;
};

static void layout_sizes(BatchLayout &Ly) {
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b, 256); return o; };
  Ly.o_desc = take(sizeof(ProbDesc) * Ly.B);
  Ly.o_colstart = take(sizeof(int) * (Ly.B + 1));
  Ly.o_zstart = take(sizeof(int) * (Ly.B + 1));
  Ly.o_ostart = take(sizeof(int) * (Ly.B + 1));
  Ly.o_tstart = take(sizeof(int) * (Ly.B + 1));
  Ly.o_wstart = take(sizeof(int) * (Ly.B + 1));
  Ly.o_lam = take(sizeof(double) * Ly.total_lam);
  Ly.o_items = take(sizeof(WorkItem) * (Ly.ksplit ? 0 : Ly.nitems));
  Ly.o_counter = take(sizeof(int) * 16);
  Ly.o_xstart = take(sizeof(int) * (SEG_XCDS + 1));
  Ly.meta_bytes = off;
  Ly.o_ci = take(sizeof(ColInfo) * Ly.total_cols);
  Ly.o_segflags = take(sizeof(int) * Ly.total_cols);
  Ly.o_DZ = take(2 * sizeof(double) * Ly.total_pairs);
  Ly.o_DZp = take(Ly.ss_split > 1 ? 2 * sizeof(double) * Ly.ss_split * (size_t)Ly.ss_ncand * Ly.ss_m : 0);
  Ly.o_mask = take(sizeof(unsigned long long) * Ly.total_words);
  Ly.o_V = take(sizeof(double) * Ly.total_ws);
  Ly.o_E = take(sizeof(double) * Ly.total_ws);
  Ly.o_R = take(sizeof(int) * Ly.total_ws);
  Ly.o_Z = take(sizeof(double) * Ly.total_z);
  Ly.o_zflag = take(sizeof(int) * Ly.total_z);
  Ly.bytes = off;
}

__global__ void k_fill_int(int *p, long long count, int value) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

static uint64_t fnv1a(const void *data, size_t n, uint64_t h) {
  const unsigned char *p = (const unsigned char *)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}


// Optional restrictions of a one-problem run (device pointers): cand / ncand
// restrict the preserved columns to a list, jmask marks them for the
// reduction, gate / gate_on make every kernel a no-op unless *gate == gate_on,
// ci (ungated runs) is the problem's column info computed by an earlier
// kernel on the same stream.
struct RunOpts {
  const int *cand;
  int ncand;
  const int *jmask;
  const int *gate;
  int gate_on;
  const ColInfo *ci;
};
static const RunOpts kNoOpts = {nullptr, 0, nullptr, nullptr, 0, nullptr};

// Build the layout, stage the metadata, launch (or replay) the sequence.
// `only_seg_ms` (autotuner): time the segment kernel alone.
// Workspace arrays of the last run, for follow-up kernels on the same stream
// (valid until the context's next run): per-(j, k) v and median row of
// lambda index 0 of problem 0, and the column info.
struct BatchPtrs {
  double *V;
  int *R;
  ColInfo *ci;
};

// Sizes, work items and workspace layout of a batch call (no allocation for
// B == 1: its items are implicit).
static int plan_batch(l1line_ctx ctx, const l1line_problem *probs, int64_t B, const TuneParams &tp,
                      const RunOpts &ro, BatchLayout &Ly, std::vector<WorkItem> &items) {
  memset(&Ly, 0, sizeof Ly);
  Ly.B = (int)B;
  Ly.nmax = 1;
  Ly.Lmax = 1;
  double total_cost = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    const l1line_problem &p = probs[b];
    Ly.total_cols += p.m;
    Ly.total_z += p.L * p.m;
    Ly.total_out += p.L;
    Ly.total_ws += p.L * p.m * p.m;
    Ly.total_lam += p.L;
    Ly.total_pairs += p.m * p.m;
    const int64_t mj = (ro.cand && B == 1) ? ro.ncand : p.m;
    Ly.total_tiles += ((mj + SS_TILE - 1) / SS_TILE) * ((p.m + SS_TILE - 1) / SS_TILE);
    Ly.total_words += mj * ((p.m + 63) / 64);
    Ly.nmax = std::max<int>(Ly.nmax, (int)p.n);
    Ly.Lmax = std::max<int>(Ly.Lmax, (int)p.L);
    total_cost += (double)p.n * (double)p.m * (double)p.m;
  }
  if (Ly.total_cols > (1ll << 30) || Ly.total_z > (1ll << 30) || Ly.total_out > (1ll << 30) ||
      Ly.total_tiles > (1ll << 30) || Ly.total_words > (1ll << 30))
    return L1LINE_EINVAL;

  // work items: split every problem's k range so the whole batch offers
  // about items_per_cu items per compute unit, each with >= kchunk_min k
  const double target = (double)tp.items_per_cu * ctx->num_cu;
  if (B == 1) {
    const int m = (int)probs[0].m;
    // implicit items routed by XCD: each XCD's part of the k range is cut
    // into chunks of at most ~2 MB of columns k (half an XCD's L2), but an
    // item keeps at least kImplicitKmin columns k: short items cost a column
    // j load, a row sample and a workgroup barrier each, which at large n
    // (one workgroup per CU) outweighs the L2 reuse
    constexpr int kImplicitKmin = 256;
    const double part_bytes = 8.0 * (double)probs[0].n * (double)m / SEG_XCDS;
    int chunks = (int)ceil(part_bytes / (2.0 * 1024 * 1024));
    const int kmin = std::max(kImplicitKmin, tp.kchunk_min);
    chunks = std::max(1, std::min(chunks, std::max(1, m / (SEG_XCDS * kmin))));
    // few preserved columns (a candidate list): cut finer so that every
    // persistent workgroup gets items, down to 16 columns k per item
    const int mj = ro.cand ? ro.ncand : m;
    const long long want = 2ll * tp.blocks_per_cu * ctx->num_cu;
    if ((long long)mj * chunks * SEG_XCDS < want) {
      const int need = (int)((want + (long long)mj * SEG_XCDS - 1) / ((long long)mj * SEG_XCDS));
      chunks = std::max(chunks, std::min(need, std::max(1, m / (SEG_XCDS * 16))));
    }
    Ly.ksplit = chunks;
    Ly.nitems = (ro.cand ? ro.ncand : m) * chunks;     // per XCD
    (void)target;
  } else {
    // problems to XCDs, largest first onto the least loaded one; an XCD
    // works through its problems largest first, so its workgroups share one
    // matrix at a time in their L2 (stealing from the next XCDs evens out
    // the end)
    std::vector<int> order((size_t)B);
    for (int64_t b = 0; b < B; ++b) order[(size_t)b] = (int)b;
    auto cost = [&](int b) { return (double)probs[b].n * (double)probs[b].m * (double)probs[b].m; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    double load[SEG_XCDS] = {0};
    std::vector<int> owned[SEG_XCDS];
    for (int b : order) {
      int x = 0;
      for (int y = 1; y < SEG_XCDS; ++y)
        if (load[y] < load[x]) x = y;
      load[x] += cost(b);
      owned[x].push_back(b);
    }
    for (int x = 0; x < SEG_XCDS; ++x) {
      Ly.xstart[x] = (int)items.size();
      for (int b : owned[x]) {
        const int m = (int)probs[b].m;
        const double share = target * cost(b) / total_cost;
        int ksplit = (int)ceil(share / m);
        const int kmax = std::max(1, m / tp.kchunk_min);
        ksplit = std::max(1, std::min(ksplit, kmax));
        const int kchunk = (m + ksplit - 1) / ksplit;
        for (int j = 0; j < m; ++j)
          for (int k0 = 0; k0 < m; k0 += kchunk) items.push_back(WorkItem{b, j, k0, std::min(m, k0 + kchunk)});
      }
    }
    Ly.xstart[SEG_XCDS] = (int)items.size();
    Ly.ksplit = 0;
    Ly.nitems = (int)items.size();
  }
  // a candidate list leaves few sign-sum tiles (32 columns j: one row of
  // tiles): their rows are cut into parts, summed apart and then added, so
  // that every compute unit gets work (parts of at least 512 rows)
  if (B == 1 && ro.cand) {
    const long long want = 2ll * ctx->num_cu;
    long long sp = std::min<long long>(16, (want + Ly.total_tiles - 1) / std::max(1ll, Ly.total_tiles));
    sp = std::min<long long>(sp, std::max<long long>(1, probs[0].n / 512));
    Ly.ss_split = (int)std::max<long long>(1, sp);
    Ly.ss_ncand = ro.ncand;
    Ly.ss_m = (int)probs[0].m;
  }
  layout_sizes(Ly);
  return L1LINE_OK;
}

// The problem descriptor of problem b with the batch's workspace offsets.
struct MetaCursor {
  long long col, z, out, wsoff, lamoff, pairoff, tiles, words;
};
static ProbDesc prob_desc(const l1line_problem &p, const MetaCursor &c) {
  ProbDesc q;
  q.X = p.X;
  q.ld = p.ld;
  q.n = (int)p.n;
  q.m = (int)p.m;
  q.L = (int)p.L;
  q.lam_off = (int)c.lamoff;
  q.col_off = (int)c.col;
  q.out_off = (int)c.out;
  q.ws_off = c.wsoff;
  q.z_off = c.z;
  q.pair_off = c.pairoff;
  q.mask_off = c.words;
  q.Vout = p.V;
  q.Jout = (long long *)p.J;
  q.OBJout = p.OBJ;
  q.ROWout = p.ROW;
  q.ZALLout = p.ZALL;
  q.status = p.status;
  return q;
}
static void advance(MetaCursor &c, const l1line_problem &p, const RunOpts &ro, int64_t B) {
  c.col += p.m;
  c.z += p.L * p.m;
  c.out += p.L;
  c.wsoff += p.L * p.m * p.m;
  c.lamoff += p.L;
  c.pairoff += p.m * p.m;
  const int64_t mj = (ro.cand && B == 1) ? ro.ncand : p.m;
  c.tiles += ((mj + SS_TILE - 1) / SS_TILE) * ((p.m + SS_TILE - 1) / SS_TILE);
  c.words += mj * ((p.m + 63) / 64);
}

// The metadata block (the first Ly.meta_bytes of the workspace) in host memory h.
static void fill_meta(char *h, const BatchLayout &Ly, const l1line_problem *probs, int64_t B,
                      const std::vector<WorkItem> &items, const RunOpts &ro) {
  memset(h, 0, Ly.meta_bytes);
  ProbDesc *hd = (ProbDesc *)(h + Ly.o_desc);
  int *hcol = (int *)(h + Ly.o_colstart), *hz = (int *)(h + Ly.o_zstart), *ho = (int *)(h + Ly.o_ostart);
  int *ht = (int *)(h + Ly.o_tstart), *hw = (int *)(h + Ly.o_wstart);
  double *hlam = (double *)(h + Ly.o_lam);
  MetaCursor c = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = 0; b < B; ++b) {
    const l1line_problem &p = probs[b];
    hd[b] = prob_desc(p, c);
    hcol[b] = (int)c.col;
    hz[b] = (int)c.z;
    ho[b] = (int)c.out;
    ht[b] = (int)c.tiles;
    hw[b] = (int)c.words;
    for (int64_t t = 0; t < p.L; ++t) hlam[c.lamoff + t] = p.lambdas[t];
    advance(c, p, ro, B);
  }
  hcol[B] = (int)c.col;
  ht[B] = (int)c.tiles;
  hw[B] = (int)c.words;
  hz[B] = (int)c.z;
  ho[B] = (int)c.out;
  if (!items.empty()) memcpy(h + Ly.o_items, items.data(), sizeof(WorkItem) * items.size());
  memcpy(h + Ly.o_xstart, Ly.xstart, sizeof Ly.xstart);
}

// The launch sequence of one batch call on stream ls, the workspace at d
// (its metadata block already in place or written by an earlier kernel on
// ls).  `prof`: bracket the kernels with the context's timing events;
// t0 / t1 (optional): events recorded around the segment kernel.
static int launch_seq(l1line_ctx ctx, hipStream_t ls, const BatchLayout &Ly, char *d, int64_t B,
                      const TuneParams &tp, const RunOpts &ro, bool prof, hipEvent_t t0, hipEvent_t t1,
                      BatchPtrs *outp) {
  const ProbDesc *dP = (const ProbDesc *)(d + Ly.o_desc);
  const int *dcol = (const int *)(d + Ly.o_colstart), *dz = (const int *)(d + Ly.o_zstart),
            *dout = (const int *)(d + Ly.o_ostart), *dtile = (const int *)(d + Ly.o_tstart),
            *dwst = (const int *)(d + Ly.o_wstart);
  const double *dlam = (const double *)(d + Ly.o_lam);
  const WorkItem *ditems = Ly.ksplit ? nullptr : (const WorkItem *)(d + Ly.o_items);
  int *dcounter = (int *)(d + Ly.o_counter);
  const int *dxstart = (const int *)(d + Ly.o_xstart);
  ColInfo *dci = (ColInfo *)(d + Ly.o_ci);
  int *dsegflags = (int *)(d + Ly.o_segflags);
  double *dV = (double *)(d + Ly.o_V), *dE = (double *)(d + Ly.o_E), *dZ = (double *)(d + Ly.o_Z);
  int *dR = (int *)(d + Ly.o_R), *dzflag = (int *)(d + Ly.o_zflag);
  double2 *dDZ = (double2 *)(d + Ly.o_DZ);
  unsigned long long *dmask = (unsigned long long *)(d + Ly.o_mask);
  if (outp) *outp = BatchPtrs{dV, dR, dci};
  l1line_ctx pc = prof ? ctx : nullptr;

  // window list capacity: the larger path list where the LDS allows it
  // the dynamic LDS the segment kernels may request (about 154 KB of the
  // CU's 160 KB): the path list's larger capacity is taken when it fits
  const size_t lds_max = seg_lds_bytes(4 * SXJ_LDS_MAX, L1LINE_MAX_LAMBDAS, WIN_CAP);
  // column j goes to LDS up to SXJ_LDS_MAX rows; longer ones are read from
  // global memory, which keeps room for more workgroups per CU.  The copy is
  // also left out where that lets more workgroups share a CU (column j then
  // comes from L2, where it stays across the item's k): the several-penalty
  // kernel's 1024-entry lists leave room for two 2000-row workgroups per CU
  // with the copy and three without (path L = 64 at 2000x2000: 66.8 -> 61.7
  // ms).  At most four: the waves per SIMD the kernel's registers allow.
  auto wg_per_cu = [](size_t bytes) {
    const size_t b = (bytes + 16 + 511) / 512 * 512;   // + static LDS, 512-byte granules
    return std::min<size_t>(4, (size_t)160 * 1024 / b);
  };
  int sxj_rows = Ly.nmax <= SXJ_LDS_MAX ? Ly.nmax : 0;
  const int lcap = (Ly.Lmax > 1 && seg_lds_bytes(sxj_rows, Ly.Lmax, PATH_CAP) <= lds_max) ? PATH_CAP : WIN_CAP;
  if (sxj_rows > 0 &&
      wg_per_cu(seg_lds_bytes(0, Ly.Lmax, lcap)) > wg_per_cu(seg_lds_bytes(sxj_rows, Ly.Lmax, lcap)))
    sxj_rows = 0;
  const size_t lds = seg_lds_bytes(sxj_rows, Ly.Lmax, lcap);
  if (!ctx->attr_seg) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_seg_batch<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_max));
    HIP_TRY(hipFuncSetAttribute((const void *)k_seg_batch<false, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
    HIP_TRY(hipFuncSetAttribute((const void *)k_seg_batch<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_max));
    HIP_TRY(hipFuncSetAttribute((const void *)k_seg_batch<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_max));
    ctx->attr_seg = true;
  }
  const long long all_items = Ly.ksplit ? (long long)Ly.nitems * SEG_XCDS : (long long)Ly.nitems;
  const int grid_seg = (int)std::max(1ll, std::min(all_items, (long long)tp.blocks_per_cu * ctx->num_cu));
  {
    ProfScope ps(pc, ls, "colprep");
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ls, dcounter, 16ll, 0);
    if (ro.ci && B == 1 && !ro.gate) {
      HIP_TRY(hipMemcpyAsync(dci, ro.ci, sizeof(ColInfo) * Ly.total_cols, hipMemcpyDeviceToDevice, ls));
      hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((Ly.total_cols + 255) / 256)), dim3(256), 0, ls, dsegflags,
                         (long long)Ly.total_cols, 0);
    } else {
      hipLaunchKernelGGL(k_colprep_batch, dim3((unsigned)((Ly.total_cols + 3) / 4)), dim3(256), 0, ls, dP, dcol,
                         (int)B, (int)Ly.total_cols, dci, dsegflags, ro.gate, ro.gate_on);
    }
  }
  {
    ProfScope ps(pc, ls, "signsum");
    const int split = Ly.ss_split > 1 ? Ly.ss_split : 1;
    double2 *dDZp = (double2 *)(d + Ly.o_DZp);
    hipLaunchKernelGGL(k_signsum_batch, dim3((unsigned)(Ly.total_tiles * split)), dim3(256), 0, ls, dP, dtile,
                       (int)B, (B == 1) ? ro.cand : nullptr, ro.ncand, dDZ, ro.gate, ro.gate_on, split, dDZp);
    if (split > 1)
      hipLaunchKernelGGL(k_signsum_parts,
                         dim3((unsigned)std::min<long long>(1024, ((long long)Ly.ss_ncand * Ly.ss_m + 255) / 256)),
                         dim3(256), 0, ls, (const double2 *)dDZp, split, ro.cand, Ly.ss_ncand, Ly.ss_m, dDZ, ro.gate,
                         ro.gate_on);
  }
  {
    ProfScope ps(pc, ls, "zero_seg");
    hipLaunchKernelGGL(k_zero_segments, dim3((unsigned)((Ly.total_words + 3) / 4)), dim3(256), 0, ls, dP, dwst,
                       (int)B, (int)Ly.total_words, dlam, dci, dDZ, dV, dE, dR, dmask,
                       (B == 1) ? ro.cand : nullptr, ro.gate, ro.gate_on);
  }
  if (t0) HIP_TRY(hipEventRecord(t0, ls));
  {
    ProfScope ps(pc, ls, "fit_seg");
    // single-penalty problems take the instantiation tuned for one target
    const bool multi = Ly.Lmax > 1;
    auto kseg = sxj_rows > 0 ? (multi ? k_seg_batch<true, true> : k_seg_batch<true, false>)
                             : (multi ? k_seg_batch<false, true> : k_seg_batch<false, false>);
    hipLaunchKernelGGL(kseg, dim3((unsigned)grid_seg), dim3(64 * SEG_WAVES), lds, ls, dP, ditems,
                       Ly.nitems, Ly.ksplit, dcounter, dxstart, dlam, dci, dDZ, dV, dE, dR, dsegflags, ro.cand,
                       ro.ncand,
                       ro.gate, ro.gate_on, dmask, lcap, sxj_rows);
  }
  if (t1) HIP_TRY(hipEventRecord(t1, ls));
  {
    ProfScope ps(pc, ls, "reduce");
    hipLaunchKernelGGL(k_reduce_batch, dim3((unsigned)Ly.total_z), dim3(64), 0, ls, dP, dz, (int)B, dlam, dV, dE,
                       dZ, dzflag, ro.jmask, ro.gate, ro.gate_on);
  }
  {
    ProfScope ps(pc, ls, "argmin");
    hipLaunchKernelGGL(k_argmin_batch, dim3((unsigned)Ly.total_out), dim3(256), 0, ls, dP, dout, (int)B, dV, dR,
                       dZ, dzflag, dci, dsegflags, ro.jmask, ro.gate, ro.gate_on, ctx->sticky);
  }
  return L1LINE_OK;
}

static int run_batch(l1line_ctx ctx, const l1line_problem *probs, int64_t B, int flags, hipStream_t s,
                     const TuneParams &tp, float *only_seg_ms, const RunOpts &ro = kNoOpts,
                     BatchPtrs *outp = nullptr) {
  BatchLayout Ly;
  std::vector<WorkItem> items;
  int st = plan_batch(ctx, probs, B, tp, ro, Ly, items);
  if (st) return st;
  st = ensure_ws(ctx, Ly.bytes, s);
  if (st) return st;
  st = ensure_stage(ctx, Ly.meta_bytes);
  if (st) return st;

  // metadata into the pinned staging buffer
  char *h = (char *)ctx->stage;
  char *d = (char *)ctx->ws;
  fill_meta(h, Ly, probs, B, items, ro);

  uint64_t key = fnv1a(h, Ly.meta_bytes, 1469598103934665603ull);
  key = fnv1a(&tp, sizeof tp, key);
  key = fnv1a(&ctx->ws, sizeof ctx->ws, key);
  key = fnv1a(&ro, sizeof ro, key);
  const bool use_graph = (flags & L1LINE_BATCH_GRAPH) && !ctx->profiling && !only_seg_ms;
  if (use_graph && ctx->graph && ctx->graph_key == key) {
    // the device metadata of this layout is still in place: replay
    if (outp) {
      BatchPtrs bp{(double *)(d + Ly.o_V), (int *)(d + Ly.o_R), (ColInfo *)(d + Ly.o_ci)};
      *outp = bp;
    }
    HIP_TRY(hipGraphLaunch(ctx->graph, s));
    return L1LINE_OK;
  }
  drop_graph(ctx);
  HIP_TRY(hipMemcpyAsync(d, h, Ly.meta_bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(ctx->stage_done, s));
  ctx->stage_pending = true;

  hipStream_t ls = s;
  if (use_graph) {
    // the metadata copy above must land before the captured kernels run on
    // the capture stream's replay (replays go to `s`, after the copy)
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ls = ctx->cap_stream;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (only_seg_ms) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
  }
  st = launch_seq(ctx, ls, Ly, d, B, tp, ro, true, t0, t1, outp);
  const hipError_t le = hipGetLastError();
  if (use_graph) {
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
    if (st || le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st ? st : L1LINE_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return L1LINE_EHIP;
    ctx->graph = ex;
    ctx->graph_key = key;
    HIP_TRY(hipGraphLaunch(ctx->graph, s));
    return L1LINE_OK;
  }
  if (st) return st;
  if (le != hipSuccess) return L1LINE_EHIP;
  if (only_seg_ms) {
    HIP_TRY(hipEventSynchronize(t1));
    HIP_TRY(hipEventElapsedTime(only_seg_ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
  }
  return L1LINE_OK;
}

static l1line_problem single(const double *X, int64_t n, int64_t m, int64_t ld, const double *lambdas, int64_t L,
                             double *V, int64_t *J, double *OBJ, int32_t *ROW, double *ZALL, int32_t *status) {
  l1line_problem p;
  p.X = X;
  p.n = n;
  p.m = m;
  p.ld = ld;
  p.lambdas = lambdas;
  p.L = L;
  p.V = V;
  p.J = J;
  p.OBJ = OBJ;
  p.ROW = ROW;
  p.ZALL = ZALL;
  p.status = status;
  return p;
}

static const TuneParams kDefaultTune = {4, 8, 24};

static int bitlen(double x) {
  int b = 0;
  while (x >= 1.0 && b < 200) {
    x *= 0.5;
    ++b;
  }
  return b;
}

static TuneKey tune_key(const l1line_problem *probs, int64_t B) {
  int64_t nmax = 1, mmax = 1, lmax = 1;
  double work = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    nmax = std::max<int64_t>(nmax, probs[b].n);
    mmax = std::max<int64_t>(mmax, probs[b].m);
    lmax = std::max<int64_t>(lmax, probs[b].L);
    work += (double)probs[b].n * (double)probs[b].m * (double)probs[b].m * (double)probs[b].L;
  }
  return TuneKey{B > 1 ? 1 : 0, lmax > 1 ? 1 : 0, bitlen((double)nmax), bitlen((double)mmax), bitlen(work) / 2};
}

// The launch parameters of a call: its size class's tuned entry, else the default.
static TuneParams tune_for(l1line_ctx ctx, const l1line_problem *probs, int64_t B, bool *tuned = nullptr) {
  const TuneKey key = tune_key(probs, B);
  for (const auto &e : ctx->tuned)
    if (e.first == key) {
      if (tuned) *tuned = true;
      return e.second;
    }
  if (tuned) *tuned = false;
  return ctx->tune;
}

extern "C" {

// Launch-parameter cache, text lines:
//   l1line-tune <workgroups per CU> <fewest k per item> <items per CU>      (default)
//   l1line-tune-class <arch> <batch> <multi> <nb> <mb> <wb> <wg/CU> <k> <items/CU>
// Entries of other architectures are kept when the file is rewritten;
// malformed lines are ignored.
static bool tune_ok(int a, int k, int i) {
  return a >= 1 && a <= 16 && k >= 1 && k <= (1 << 20) && i >= 1 && i <= 4096;
}

static void tune_load(l1line_ctx c) {
  if (c->tune_path.empty()) return;
  FILE *f = fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    int a = 0, k = 0, i = 0;
    char arch[160];
    TuneKey key;
    if (sscanf(line, "l1line-tune %d %d %d", &a, &k, &i) == 3) {
      if (tune_ok(a, k, i)) c->tune = TuneParams{a, k, i};
    } else if (sscanf(line, "l1line-tune-class %159s %d %d %d %d %d %d %d %d", arch, &key.batch, &key.multi, &key.nb,
                      &key.mb, &key.wb, &a, &k, &i) == 9) {
      if (!tune_ok(a, k, i)) continue;
      if (c->arch == arch) {
        c->tuned.push_back({key, TuneParams{a, k, i}});
      } else {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        c->tune_foreign.push_back(l);
      }
    }
  }
  fclose(f);
}

static int tune_save(l1line_ctx c) {
  if (c->tune_path.empty()) return L1LINE_OK;
  const std::string tmp = c->tune_path + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return L1LINE_EIO;
  bool ok = fprintf(f, "l1line-tune %d %d %d\n", c->tune.blocks_per_cu, c->tune.kchunk_min, c->tune.items_per_cu) > 0;
  for (const auto &e : c->tuned)
    ok = ok && fprintf(f, "l1line-tune-class %s %d %d %d %d %d %d %d %d\n", c->arch.c_str(), e.first.batch,
                       e.first.multi, e.first.nb, e.first.mb, e.first.wb, e.second.blocks_per_cu,
                       e.second.kchunk_min, e.second.items_per_cu) > 0;
  for (const auto &l : c->tune_foreign) ok = ok && fprintf(f, "%s\n", l.c_str()) > 0;
  if (fclose(f) != 0 || !ok) return L1LINE_EIO;
  return rename(tmp.c_str(), c->tune_path.c_str()) == 0 ? L1LINE_OK : L1LINE_EIO;
}

int l1line_create(l1line_ctx *ctx, int device, const char *tune_cache_path) {
  if (!ctx) return L1LINE_EINVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return L1LINE_EHIP;
  if (device < 0 || device >= count) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  l1line_ctx c = new (std::nothrow) l1line_ctx_s();
  if (!c) return L1LINE_ENOMEM;
  c->device = device;
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->stage = nullptr;
  c->stage_bytes = 0;
  c->stage_pending = false;
  c->graph = nullptr;
  c->graph_key = 0;
  c->tune = kDefaultTune;
  c->profiling = false;
  c->rk = nullptr;
  c->rk_bytes = 0;
  c->sp = nullptr;
  c->bl = nullptr;
  c->bl_bytes = 0;
  c->sp_bytes = 0;
  c->sticky = nullptr;
  c->host_err = L1LINE_OK;
  c->rk_w = nullptr;
  c->rk_have_w = c->rk_have_state = false;
  c->rk_step = 0;
  c->rk_seed = c->rk_cursor = 0;
  c->scratch = scratch_address(device);   // device is current (hipSetDevice above)
  c->arch = prop.gcnArchName[0] ? std::string(prop.gcnArchName) : std::string("unknown");
  for (auto &ch : c->arch)
    if (ch == ' ') ch = '_';
  if (tune_cache_path) c->tune_path = tune_cache_path;
  tune_load(c);
  if (hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void **)&c->sticky, sizeof(int)) != hipSuccess || hipMemset(c->sticky, 0, sizeof(int)) != hipSuccess) {
    if (c->sticky) (void)hipFree(c->sticky);
    delete c;
    return L1LINE_EHIP;
  }
  *ctx = c;
  return L1LINE_OK;
}

// Records the first nonzero status an entry point returns on the context.
static int note(l1line_ctx ctx, int st) {
  if (ctx && st != L1LINE_OK && ctx->host_err == L1LINE_OK) ctx->host_err = st;
  return st;
}

int l1line_last_error(l1line_ctx ctx) {
  if (!ctx) return L1LINE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return L1LINE_EHIP;
  int dev = 0;
  if (hipMemcpy(&dev, ctx->sticky, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return L1LINE_EHIP;
  const int st = ctx->host_err != L1LINE_OK ? ctx->host_err : dev;
  ctx->host_err = L1LINE_OK;
  if (dev != 0 && hipMemset(ctx->sticky, 0, sizeof(int)) != hipSuccess) return L1LINE_EHIP;
  return st;
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
  drop_graph(ctx);
  if (ctx->ws && hipFree(ctx->ws) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->stage && hipHostFree(ctx->stage) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->rk && hipFree(ctx->rk) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->sp && hipFree(ctx->sp) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->bl && hipFree(ctx->bl) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->sticky && hipFree(ctx->sticky) != hipSuccess) st = L1LINE_EHIP;
  if (ctx->rk_w && hipFree(ctx->rk_w) != hipSuccess) st = L1LINE_EHIP;
  (void)hipEventDestroy(ctx->stage_done);
  (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return st;
}

// Measured ceilings (microbenchmarks of peak_kernels.h), best of 3 timed
// runs after one warm-up each.
static int measure_peaks_impl(l1line_ctx ctx, double *out) {
  if (!ctx || !out) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  const long long n16 = (1ll << 30) / 16;             // 1 GiB per copy buffer
  const int grid = ctx->num_cu * 8;
  void *a = nullptr, *b = nullptr, *sink = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = L1LINE_OK;
  if (hipMalloc(&a, n16 * 16) != hipSuccess || hipMalloc(&b, n16 * 16) != hipSuccess ||
      hipMalloc(&sink, (size_t)grid * 256 * 8) != hipSuccess) {
    (void)hipGetLastError();
    st = L1LINE_ENOMEM;
  }
  if (!st && (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = L1LINE_EHIP;
  if (!st && hipMemsetAsync(a, 0, n16 * 16, s) != hipSuccess) st = L1LINE_EHIP;
  auto best_ms = [&](auto launch) -> float {
    float best = 1e30f;
    for (int rep = 0; rep < 4 && !st; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) { st = L1LINE_EHIP; break; }
      launch();
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = L1LINE_EHIP;
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = L1LINE_EHIP; break; }
      if (rep > 0 && ms < best) best = ms;                 // rep 0 warms up
    }
    return best;
  };
  if (!st) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(k_peak_copy, dim3(ctx->num_cu * 16), dim3(256), 0, s, (const double2 *)a, (double2 *)b, n16);
    });
    out[0] = 2.0 * n16 * 16 / (ms * 1e-3) / 1e9;
  }
  if (!st) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(k_peak_lds, dim3(grid), dim3(256), 0, s, (unsigned *)sink);
    });
    out[1] = (double)grid * 256 * PEAK_LDS_ITER * 4 * 16 / (ms * 1e-3) / 1e9;
  }
  if (!st) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(k_peak_fma, dim3(grid), dim3(256), 0, s, (double *)sink, 0.999999, 1e-7);
    });
    out[2] = (double)grid * 256 * PEAK_FMA_ITER * 8 * 2 / (ms * 1e-3) / 1e12;
  }
  if (!st) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(k_peak_mfma_f64, dim3(grid), dim3(256), 0, s, (double *)sink, 1e-3);
    });
    out[3] = (double)grid * 4 * PEAK_MFMA_ITER * 4 * 2048 / (ms * 1e-3) / 1e12;
  }
  if (!st) {
    const float ms = best_ms([&] {
      hipLaunchKernelGGL(k_peak_mfma_bf16, dim3(grid), dim3(256), 0, s, (float *)sink, 1e-3f);
    });
    out[4] = (double)grid * 4 * PEAK_MFMA_ITER * 4 * 16384 / (ms * 1e-3) / 1e12;
  }
  if (!st && hipGetLastError() != hipSuccess) st = L1LINE_EHIP;
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (sink) (void)hipFree(sink);
  return st;
}

int l1line_measure_peaks(l1line_ctx ctx, double *out) { return note(ctx, measure_peaks_impl(ctx, out)); }

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
    case L1LINE_ESIZE: return "a size exceeds a library limit (L1LINE_MAX_N rows, L1LINE_RANKER_MAX_M ranked columns, L1LINE_BP_MAX_M columns for breakpoints, or the breakpoint capacity)";
    case L1LINE_EINTERNAL: return "selection round bound exceeded";
    case L1LINE_EIO: return "file missing, unreadable or malformed";
    case L1LINE_ENOMODEL: return "the context holds no ranker weights";
    default: return "unknown status";
  }
}

static int column_stats_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double *W,
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

int l1line_column_stats(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double *W,
                        int32_t *zeros, int32_t *status, void *stream) {
  return note(ctx, column_stats_impl(ctx, X, n, m, ld, W, zeros, status, stream));
}

static int fit_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, double *v,
               int64_t *j, double *obj, int32_t *median_row, double *z_all, int32_t *status, void *stream) {
  if (!ctx || !v || !j || !obj) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const l1line_problem p = single(X, n, m, ld, &lambda, 1, v, j, obj, median_row, z_all, status);
  return run_batch(ctx, &p, 1, 0, (hipStream_t)stream, tune_for(ctx, &p, 1), nullptr);
}

int l1line_fit(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, double *v,
               int64_t *j, double *obj, int32_t *median_row, double *z_all, int32_t *status, void *stream) {
  return note(ctx, fit_impl(ctx, X, n, m, ld, lambda, v, j, obj, median_row, z_all, status, stream));
}

// Metadata of a one-problem call written by a kernel from its arguments, so
// that the no-alloc call needs no host staging buffer.  One thread.
__global__ void k_meta_single(ProbDesc pd, double lam, long long tiles, BatchLayout Ly, char *d) {
  if (threadIdx.x != 0) return;
  *(ProbDesc *)(d + Ly.o_desc) = pd;
  int *col = (int *)(d + Ly.o_colstart), *z = (int *)(d + Ly.o_zstart), *o = (int *)(d + Ly.o_ostart),
      *t = (int *)(d + Ly.o_tstart);
  col[0] = 0;
  col[1] = pd.m;
  z[0] = 0;
  z[1] = pd.m;
  o[0] = 0;
  o[1] = 1;
  t[0] = 0;
  t[1] = (int)tiles;
  int *ws = (int *)(d + Ly.o_wstart);
  ws[0] = 0;
  ws[1] = (int)Ly.total_words;
  *(double *)(d + Ly.o_lam) = lam;
  int *xs = (int *)(d + Ly.o_xstart);
  for (int x = 0; x <= SEG_XCDS; ++x) xs[x] = Ly.xstart[x];
}

static int fit_noalloc_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                            double *v, int64_t *j, double *obj, int32_t *median_row, double *z_all,
                            int32_t *status, void *stream) {
  if (!ctx || !v || !j || !obj) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  if (m > L1LINE_NOALLOC_MAX_M) return L1LINE_ESIZE;
  if (!ctx->scratch) return L1LINE_EHIP;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const l1line_problem p = single(X, n, m, ld, &lambda, 1, v, j, obj, median_row, z_all, status);
  BatchLayout Ly;
  std::vector<WorkItem> items;        // stays empty: one problem's items are implicit
  const TuneParams tp = tune_for(ctx, &p, 1);
  st = plan_batch(ctx, &p, 1, tp, kNoOpts, Ly, items);
  if (st) return st;
  if (Ly.bytes > NOALLOC_BYTES || !items.empty()) return L1LINE_ESIZE;
  const MetaCursor c0 = {0, 0, 0, 0, 0, 0, 0, 0};
  MetaCursor c1 = c0;
  advance(c1, p, kNoOpts, 1);
  char *d = (char *)ctx->scratch;
  hipLaunchKernelGGL(k_meta_single, dim3(1), dim3(64), 0, s, prob_desc(p, c0), lambda, c1.tiles, Ly, d);
  st = launch_seq(ctx, s, Ly, d, 1, tp, kNoOpts, false, nullptr, nullptr, nullptr);
  if (st) return st;
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_fit_noalloc(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, double *v,
                       int64_t *j, double *obj, int32_t *median_row, double *z_all, int32_t *status,
                       void *stream) {
  return note(ctx, fit_noalloc_impl(ctx, X, n, m, ld, lambda, v, j, obj, median_row, z_all, status, stream));
}

static int fit_path_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, const double *lambdas,
                    int64_t L, double *V, int64_t *J, double *OBJ, int32_t *ROW, double *ZALL, int32_t *status,
                    void *stream) {
  if (!ctx || !V || !J || !OBJ) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(lambdas, L);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const l1line_problem p = single(X, n, m, ld, lambdas, L, V, J, OBJ, ROW, ZALL, status);
  return run_batch(ctx, &p, 1, 0, (hipStream_t)stream, tune_for(ctx, &p, 1), nullptr);
}

int l1line_fit_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, const double *lambdas,
                    int64_t L, double *V, int64_t *J, double *OBJ, int32_t *ROW, double *ZALL, int32_t *status,
                    void *stream) {
  return note(ctx, fit_path_impl(ctx, X, n, m, ld, lambdas, L, V, J, OBJ, ROW, ZALL, status, stream));
}

static int fit_batch_impl(l1line_ctx ctx, const l1line_problem *probs, int64_t B, int flags, void *stream) {
  if (!ctx || !probs || B < 1 || B > (1 << 20)) return L1LINE_EINVAL;
  if (flags & ~L1LINE_BATCH_GRAPH) return L1LINE_EINVAL;
  for (int64_t b = 0; b < B; ++b) {
    const int st = check_problem(probs[b]);
    if (st) return st;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  return run_batch(ctx, probs, B, flags, (hipStream_t)stream, tune_for(ctx, probs, B), nullptr);
}

int l1line_fit_batch(l1line_ctx ctx, const l1line_problem *probs, int64_t B, int flags, void *stream) {
  return note(ctx, fit_batch_impl(ctx, probs, B, flags, stream));
}

static int autotune_impl(l1line_ctx ctx, const l1line_problem *probs, int64_t B, void *stream, int32_t *params_out) {
  if (!ctx || !probs || B < 1 || B > (1 << 20)) return L1LINE_EINVAL;
  for (int64_t b = 0; b < B; ++b) {
    const int st = check_problem(probs[b]);
    if (st) return st;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const bool was_profiling = ctx->profiling;
  ctx->profiling = false;
  TuneParams best = tune_for(ctx, probs, B);
  float best_ms = 1e30f;
  // the grid: persistent workgroups per CU x fewest k per item x items per
  // CU; one problem's items are implicit (items per CU unused, at least 256
  // k per item unless more is asked), so its grid varies the first two
  const int bpc[] = {2, 3, 4};
  const int kmin_batch[] = {8, 32, 128}, kmin_one[] = {64, 256, 512};
  const int ipc_batch[] = {12, 24, 48}, ipc_one[] = {24};
  const int *kmin = B > 1 ? kmin_batch : kmin_one;
  const int *ipc = B > 1 ? ipc_batch : ipc_one;
  const int nipc = B > 1 ? 3 : 1;
  for (int a : bpc)
    for (int kq = 0; kq < 3; ++kq)
      for (int iq = 0; iq < nipc; ++iq) {
        const TuneParams tp{a, kmin[kq], ipc[iq]};
        float ms = 0.f;
        const int st = run_batch(ctx, probs, B, 0, s, tp, &ms);
        if (st) {
          ctx->profiling = was_profiling;
          return st;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = tp;
        }
      }
  const TuneKey key = tune_key(probs, B);
  bool found = false;
  for (auto &e : ctx->tuned)
    if (e.first == key) {
      e.second = best;
      found = true;
    }
  if (!found) ctx->tuned.push_back({key, best});
  ctx->profiling = was_profiling;
  drop_graph(ctx);
  if (params_out) {
    params_out[0] = best.blocks_per_cu;
    params_out[1] = best.kchunk_min;
    params_out[2] = best.items_per_cu;
  }
  return tune_save(ctx);
}

int l1line_autotune(l1line_ctx ctx, const l1line_problem *probs, int64_t B, void *stream, int32_t *params_out) {
  return note(ctx, autotune_impl(ctx, probs, B, stream, params_out));
}

int l1line_tune_set(l1line_ctx ctx, const int32_t *params) {
  if (!ctx || !params) return L1LINE_EINVAL;
  if (params[0] < 1 || params[0] > 16 || params[1] < 1 || params[1] > (1 << 20) || params[2] < 1 ||
      params[2] > 4096)
    return L1LINE_EINVAL;
  ctx->tune = TuneParams{params[0], params[1], params[2]};
  drop_graph(ctx);
  return L1LINE_OK;
}

int l1line_tune_lookup(l1line_ctx ctx, const l1line_problem *probs, int64_t B, int32_t *params, int32_t *tuned) {
  if (!ctx || !probs || !params || B < 1 || B > (1 << 20)) return note(ctx, L1LINE_EINVAL);
  for (int64_t b = 0; b < B; ++b) {
    const int st = check_problem(probs[b]);
    if (st) return note(ctx, st);
  }
  bool t = false;
  const TuneParams tp = tune_for(ctx, probs, B, &t);
  params[0] = tp.blocks_per_cu;
  params[1] = tp.kchunk_min;
  params[2] = tp.items_per_cu;
  if (tuned) *tuned = t ? 1 : 0;
  return L1LINE_OK;
}

int l1line_tune_get(l1line_ctx ctx, int32_t *params) {
  if (!ctx || !params) return L1LINE_EINVAL;
  params[0] = ctx->tune.blocks_per_cu;
  params[1] = ctx->tune.kchunk_min;
  params[2] = ctx->tune.items_per_cu;
  return L1LINE_OK;
}

// ------------------------------------------------------------------ ranker

static int mlp_forward(l1line_ctx ctx, const float *P, const float *F, int64_t N, float *out, float *H1, float *H2,
                       hipStream_t s) {
  ProfScope ps(ctx, s, "mlp_fwd");
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((N + FWD_ROWS - 1) / FWD_ROWS)), dim3(64), 0, s, P, F, (int)N, out,
                     H1, H2);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

static int mlp_forward_impl(l1line_ctx ctx, const float *params, const float *F, int64_t N, float *out, void *stream) {
  if (!ctx || !params || !F || !out || N < 1 || N > (1ll << 24)) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  return mlp_forward(ctx, params, F, N, out, nullptr, nullptr, (hipStream_t)stream);
}

int l1line_mlp_forward(l1line_ctx ctx, const float *params, const float *F, int64_t N, float *out, void *stream) {
  return note(ctx, mlp_forward_impl(ctx, params, F, N, out, stream));
}

static int mlp_grad_impl(l1line_ctx ctx, const float *params, const float *F, const float *y, int64_t N, float *grad,
                    float *loss, void *stream) {
  if (!ctx || !params || !F || !y || !grad || N < 1 || N > (1ll << 22)) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int ntiles = (int)((N + BWD_ROWS - 1) / BWD_ROWS);
  const size_t fb = sizeof(float);
  const size_t o_out = 0, o_h1 = align_up(fb * N, 256), o_h2 = o_h1 + align_up(fb * N * MLP_H, 256),
               o_g = o_h2 + align_up(fb * N * MLP_H, 256), o_l = o_g + align_up(fb * ntiles * MLP_NPARAM, 256),
               total = o_l + align_up(fb * ntiles, 256);
  int st = ensure_rk(ctx, total, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  float *out = (float *)(b + o_out), *H1 = (float *)(b + o_h1), *H2 = (float *)(b + o_h2);
  float *gpart = (float *)(b + o_g), *lpart = (float *)(b + o_l);
  st = mlp_forward(ctx, params, F, N, out, H1, H2, s);
  if (st) return st;
  if (!ctx->attr_bwd) {
    HIP_TRY(hipFuncSetAttribute((const void *)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BWD_LDS));
    ctx->attr_bwd = true;
  }
  {
    ProfScope ps(ctx, s, "mlp_bwd");
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)ntiles), dim3(64), BWD_LDS, s, params, F, y, (int)N, out, H1, H2,
                       gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, gpart, lpart, ntiles, grad,
                       loss);
  }
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_mlp_grad(l1line_ctx ctx, const float *params, const float *F, const float *y, int64_t N, float *grad,
                    float *loss, void *stream) {
  return note(ctx, mlp_grad_impl(ctx, params, F, y, N, grad, loss, stream));
}

static int mlp_adam_impl(l1line_ctx ctx, float *params, float *m1, float *m2, const float *grad, int64_t step, float lr,
                    void *stream) {
  if (!ctx || !params || !m1 || !m2 || !grad || step < 1 || !(lr > 0.0f)) return L1LINE_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, m1, m2,
                     grad, (long long)step, lr, 0.9f, 0.999f, 1e-8f);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_mlp_adam(l1line_ctx ctx, float *params, float *m1, float *m2, const float *grad, int64_t step, float lr,
                    void *stream) {
  return note(ctx, mlp_adam_impl(ctx, params, m1, m2, grad, step, lr, stream));
}

// ranker scratch layout for a matrix of n x m: sign sums, slope aggregates,
// column info, statistics, features, scores, candidates, mask, flags
struct RkLayout {
  size_t o_DZ, o_agg, o_ci, o_stats, o_F, o_score, o_cand, o_mask, o_flag, o_margin, o_H, o_L, o_S, bytes;
};

static RkLayout rk_layout(int64_t n, int64_t m) {
  RkLayout R;
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = align_up(off + b, 256); return o; };
  R.o_DZ = take(2 * sizeof(double) * m * m);
  // BF16 planes of the feature sign sums (high and low parts, signs)
  const size_t plane = sizeof(__bf16) * (size_t)fss_rows(n) * (size_t)m;
  R.o_H = take(plane);
  R.o_L = take(plane);
  R.o_S = take(plane);
  R.o_agg = take(sizeof(double) * 4 * m);
  R.o_ci = take(sizeof(ColInfo) * m);
  R.o_stats = take(sizeof(double) * 3 * FEAT_Q);
  R.o_F = take(sizeof(float) * MLP_IN * m);
  R.o_score = take(sizeof(float) * m);
  R.o_cand = take(sizeof(int) * m);
  R.o_mask = take(sizeof(int) * m);
  R.o_flag = take(sizeof(int) * 4);
  R.o_margin = take(sizeof(float) * 4);
  R.bytes = off;
  return R;
}

// the feature sign sums into DZ (the ranker scratch's, or the caller's);
// column info of X into the scratch
static int feature_signsums(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double2 *DZ,
                            hipStream_t s) {
  const RkLayout R = rk_layout(n, m);
  int st = ensure_rk(ctx, R.bytes, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  ColInfo *ci = (ColInfo *)(b + R.o_ci);
  __bf16 *Hp = (__bf16 *)(b + R.o_H), *Lp = (__bf16 *)(b + R.o_L), *Sp = (__bf16 *)(b + R.o_S);
  const int np = (int)fss_rows(n);
  const long long tb = (m + FSS_T - 1) / FSS_T;
  hipLaunchKernelGGL(k_colprep, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld, ci);
  hipLaunchKernelGGL(k_feat_planes, dim3((unsigned)(m * ((np + 255) / 256))), dim3(256), 0, s, X, (int)n, (int)m,
                     (long long)ld, np, (const ColInfo *)ci, Hp, Lp, Sp);
  {
    ProfScope ps(ctx, s, "feat_signsum");
    hipLaunchKernelGGL(k_feat_signsum, dim3((unsigned)((tb * tb + 3) / 4)), dim3(256), 0, s, (const __bf16 *)Hp,
                       (const __bf16 *)Lp, (const __bf16 *)Sp, (int)m, np, (const ColInfo *)ci, DZ);
  }
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

static int ranker_features(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                           float *F, hipStream_t s) {
  const RkLayout R = rk_layout(n, m);
  int st = ensure_rk(ctx, R.bytes, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  ColInfo *ci = (ColInfo *)(b + R.o_ci);
  double2 *DZ = (double2 *)(b + R.o_DZ);
  double *agg = (double *)(b + R.o_agg), *stats = (double *)(b + R.o_stats);
  st = feature_signsums(ctx, X, n, m, ld, DZ, s);
  if (st) return st;
  hipLaunchKernelGGL(k_slope_aggr, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, (const double2 *)DZ, ci, (int)m,
                     lambda, agg);
  hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(256), 0, s, (const double *)agg, (int)m, ci, stats);
  hipLaunchKernelGGL(k_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, (const double *)agg, (int)m,
                     (int)n, lambda, ci, stats, F);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

static int ranker_features_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                           float *F, void *stream) {
  if (!ctx || !F) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  if (m > L1LINE_RANKER_MAX_M) return L1LINE_ESIZE;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  return ranker_features(ctx, X, n, m, ld, lambda, F, (hipStream_t)stream);
}

int l1line_ranker_features(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                           float *F, void *stream) {
  return note(ctx, ranker_features_impl(ctx, X, n, m, ld, lambda, F, stream));
}

static int ranker_signsums_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double *DZ,
                                void *stream) {
  if (!ctx || !DZ) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  if (m > L1LINE_RANKER_MAX_M) return L1LINE_ESIZE;
  HIP_TRY(hipSetDevice(ctx->device));
  return feature_signsums(ctx, X, n, m, ld, (double2 *)DZ, (hipStream_t)stream);
}

int l1line_ranker_signsums(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double *DZ,
                           void *stream) {
  return note(ctx, ranker_signsums_impl(ctx, X, n, m, ld, DZ, stream));
}

__global__ void k_copy_flag(const int *src, int *dst) {
  if (threadIdx.x == 0) *dst = *src;
}

static int fit_ranked_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                           int32_t K, double margin_threshold, double *v, int64_t *j, double *obj,
                           int32_t *median_row, int32_t *used_fallback, float *scores, int32_t *status,
                           void *stream) {
  if (!ctx || !v || !j || !obj) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  if (K < 1 || K > m || !(margin_threshold >= 0.0) || isinf(margin_threshold)) return L1LINE_EINVAL;
  if (m > L1LINE_RANKER_MAX_M) return L1LINE_ESIZE;
  if (!ctx->rk_have_w) return L1LINE_ENOMODEL;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const RkLayout R = rk_layout(n, m);
  st = ensure_rk(ctx, R.bytes, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  float *F = (float *)(b + R.o_F);
  float *sc = scores ? scores : (float *)(b + R.o_score);
  int *cand = (int *)(b + R.o_cand), *mask = (int *)(b + R.o_mask), *flag = (int *)(b + R.o_flag);
  float *margin = (float *)(b + R.o_margin);
  {
    ProfScope ps(ctx, s, "features");
    st = ranker_features(ctx, X, n, m, ld, lambda, F, s);
    if (st) return st;
  }
  st = mlp_forward(ctx, ctx->rk_w, F, m, sc, nullptr, nullptr, s);
  if (st) return st;
  if (m <= TOPK_LDS_MAX)
    hipLaunchKernelGGL(k_topk_lds, dim3(1), dim3(1024), 0, s, sc, (int)m, (int)K, margin_threshold, cand, mask, flag,
                       margin);
  else
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(256), 0, s, sc, (int)m, (int)K, margin_threshold, cand, mask, flag,
                       margin);
  HIP_TRY(hipGetLastError());
  const l1line_problem p = single(X, n, m, ld, &lambda, 1, v, j, obj, median_row, nullptr, status);
  // exact solve of the K candidates
  // (the column info the features computed)
  const RunOpts rc{cand, (int)K, mask, nullptr, 0, (const ColInfo *)(b + R.o_ci)};
  st = run_batch(ctx, &p, 1, 0, s, tune_for(ctx, &p, 1), nullptr, rc);
  if (st) return st;
  // exhaustive solve, which does nothing unless the margin test failed
  const RunOpts rf{nullptr, 0, nullptr, flag, 1, nullptr};
  st = run_batch(ctx, &p, 1, 0, s, tune_for(ctx, &p, 1), nullptr, rf);
  if (st) return st;
  if (used_fallback) hipLaunchKernelGGL(k_copy_flag, dim3(1), dim3(64), 0, s, flag, used_fallback);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_fit_ranked(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, int32_t K,
                      double margin_threshold, double *v, int64_t *j, double *obj, int32_t *median_row,
                      int32_t *used_fallback, float *scores, int32_t *status, void *stream) {
  return note(ctx, fit_ranked_impl(ctx, X, n, m, ld, lambda, K, margin_threshold, v, j, obj, median_row,
                                   used_fallback, scores, status, stream));
}

// ------------------------------------------------------- ranker weights
static int ensure_rk_w(l1line_ctx ctx) {
  if (ctx->rk_w) return L1LINE_OK;
  if (hipMalloc((void **)&ctx->rk_w, 3 * sizeof(float) * MLP_NPARAM) != hipSuccess) {
    ctx->rk_w = nullptr;
    return L1LINE_ENOMEM;
  }
  HIP_TRY(hipMemset(ctx->rk_w, 0, 3 * sizeof(float) * MLP_NPARAM));
  return L1LINE_OK;
}

// Weight file (little endian): "L1RK", u32 version 1, u32 parameter count,
// u32 flags (bit 0: Adam state follows), i64 step, u64 seed, u64 next
// example; f32 weights[count]; with bit 0, f32 m1[count], f32 m2[count].
struct RkHeader {
  char magic[4];
  uint32_t version, nparam, flags;
  int64_t step;
  uint64_t seed, cursor;
};

static int rk_write(l1line_ctx ctx, const char *path, bool with_state) {
  std::vector<float> h((with_state ? 3 : 1) * (size_t)MLP_NPARAM);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(h.data(), ctx->rk_w, sizeof(float) * h.size(), hipMemcpyDeviceToHost));
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "wb");
  if (!f) return L1LINE_EIO;
  RkHeader hd;
  memcpy(hd.magic, "L1RK", 4);
  hd.version = 1;
  hd.nparam = MLP_NPARAM;
  hd.flags = with_state ? 1u : 0u;
  hd.step = ctx->rk_step;
  hd.seed = ctx->rk_seed;
  hd.cursor = ctx->rk_cursor;
  bool ok = fwrite(&hd, sizeof hd, 1, f) == 1 && fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return L1LINE_EIO;
  }
  return L1LINE_OK;
}

static int rk_read(l1line_ctx ctx, const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return L1LINE_EIO;
  RkHeader hd;
  std::vector<float> h;
  bool ok = fread(&hd, sizeof hd, 1, f) == 1 && memcmp(hd.magic, "L1RK", 4) == 0 && hd.version == 1 &&
            hd.nparam == (uint32_t)MLP_NPARAM && (hd.flags & ~1u) == 0;
  if (ok) {
    h.resize(((hd.flags & 1u) ? 3 : 1) * (size_t)MLP_NPARAM);
    ok = fread(h.data(), sizeof(float), h.size(), f) == h.size();
  }
  fclose(f);
  if (!ok) return L1LINE_EIO;
  for (float x : h)
    if (!std::isfinite(x)) return L1LINE_EIO;
  int st = ensure_rk_w(ctx);
  if (st) return st;
  HIP_TRY(hipMemcpy(ctx->rk_w, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
  if (!(hd.flags & 1u)) HIP_TRY(hipMemset(ctx->rk_w + MLP_NPARAM, 0, 2 * sizeof(float) * MLP_NPARAM));
  ctx->rk_have_w = true;
  ctx->rk_have_state = (hd.flags & 1u) != 0;
  ctx->rk_step = hd.step;
  ctx->rk_seed = hd.seed;
  ctx->rk_cursor = hd.cursor;
  return L1LINE_OK;
}

int l1line_ranker_load(l1line_ctx ctx, const char *path) {
  if (!ctx || !path) return L1LINE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return note(ctx, L1LINE_EHIP);
  return note(ctx, rk_read(ctx, path));
}

int l1line_ranker_save(l1line_ctx ctx, const char *path) {
  if (!ctx || !path) return L1LINE_EINVAL;
  if (!ctx->rk_have_w) return note(ctx, L1LINE_ENOMODEL);
  if (hipSetDevice(ctx->device) != hipSuccess) return note(ctx, L1LINE_EHIP);
  return note(ctx, rk_write(ctx, path, ctx->rk_have_state));
}

int l1line_ranker_set_params(l1line_ctx ctx, const float *params, void *stream) {
  if (!ctx || !params) return L1LINE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return note(ctx, L1LINE_EHIP);
  int st = ensure_rk_w(ctx);
  if (st) return note(ctx, st);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(ctx->rk_w, params, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemsetAsync(ctx->rk_w + MLP_NPARAM, 0, 2 * sizeof(float) * MLP_NPARAM, s) != hipSuccess)
    return note(ctx, L1LINE_EHIP);
  ctx->rk_have_w = true;
  ctx->rk_have_state = false;
  ctx->rk_step = 0;
  return L1LINE_OK;
}

int l1line_ranker_get_params(l1line_ctx ctx, float *params, void *stream) {
  if (!ctx || !params) return L1LINE_EINVAL;
  if (!ctx->rk_have_w) return note(ctx, L1LINE_ENOMODEL);
  if (hipSetDevice(ctx->device) != hipSuccess) return note(ctx, L1LINE_EHIP);
  if (hipMemcpyAsync(params, ctx->rk_w, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess)
    return note(ctx, L1LINE_EHIP);
  return L1LINE_OK;
}

// splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the host-side stream for the initial weights and
// the sizes of the training matrices
static uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// He-normal weights (variance 2 / fan-in; 1 / fan-in for the output layer),
// zero biases, from the seed
static void rk_init_host(uint64_t seed, std::vector<float> &w) {
  w.assign(MLP_NPARAM, 0.f);
  uint64_t x = seed ^ 0x5EEDC0DE12345678ull;
  auto normal = [&]() {
    const double u1 = ((double)(splitmix64(x) >> 11) + 0.5) * 0x1p-53, u2 = (double)(splitmix64(x) >> 11) * 0x1p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  };
  for (int q = 0; q < MLP_IN * MLP_H; ++q) w[OFF_W1 + q] = (float)(normal() * sqrt(2.0 / MLP_IN));
  for (int q = 0; q < MLP_H * MLP_H; ++q) w[OFF_W2 + q] = (float)(normal() * sqrt(2.0 / MLP_H));
  for (int q = 0; q < MLP_H; ++q) w[OFF_W3 + q] = (float)(normal() * sqrt(1.0 / MLP_H));
}

int l1line_ranker_train(l1line_ctx ctx, const char *ckpt_path, int64_t steps, uint64_t seed) {
  if (!ctx || steps < 0) return L1LINE_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return note(ctx, L1LINE_EHIP);
  int st = ensure_rk_w(ctx);
  if (st) return note(ctx, st);
  // resume from the checkpoint when there is one, else start from the seed
  FILE *probe = ckpt_path ? fopen(ckpt_path, "rb") : nullptr;
  if (probe) {
    fclose(probe);
    st = rk_read(ctx, ckpt_path);
    if (st) return note(ctx, st);
    if (!ctx->rk_have_state) return note(ctx, L1LINE_EIO);
  } else {
    std::vector<float> w;
    rk_init_host(seed, w);
    if (hipMemcpy(ctx->rk_w, w.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->rk_w + MLP_NPARAM, 0, 2 * sizeof(float) * MLP_NPARAM) != hipSuccess)
      return note(ctx, L1LINE_EHIP);
    ctx->rk_step = 0;
    ctx->rk_seed = seed;
    ctx->rk_cursor = 0;
  }
  ctx->rk_have_w = ctx->rk_have_state = true;
  constexpr int kNmax = 4000, kMmax = 500, kSaveEvery = 1000;
  constexpr float kLr = 1e-3f;
  // training buffers: matrix, column info, fit outputs, features, targets, gradient
  const size_t fb = sizeof(float), db = sizeof(double);
  const size_t o_X = 0, o_ci = align_up(db * kNmax * kMmax, 256), o_v = o_ci + align_up(sizeof(ColInfo) * kMmax, 256),
               o_j = o_v + align_up(db * kMmax, 256), o_obj = o_j + 256, o_z = o_obj + 256,
               o_mass = o_z + align_up(db * kMmax, 256), o_F = o_mass + 256,
               o_y = o_F + align_up(fb * MLP_IN * kMmax, 256), o_g = o_y + align_up(fb * kMmax, 256),
               o_loss = o_g + align_up(fb * MLP_NPARAM, 256), total = o_loss + 256;
  char *buf = nullptr;
  if (hipMalloc((void **)&buf, total) != hipSuccess) return note(ctx, L1LINE_ENOMEM);
  double *X = (double *)(buf + o_X), *V = (double *)(buf + o_v), *OBJ = (double *)(buf + o_obj);
  double *Z = (double *)(buf + o_z), *mass = (double *)(buf + o_mass);
  int64_t *J = (int64_t *)(buf + o_j);
  ColInfo *ci = (ColInfo *)(buf + o_ci);
  float *F = (float *)(buf + o_F), *y = (float *)(buf + o_y), *g = (float *)(buf + o_g), *loss = (float *)(buf + o_loss);
  hipStream_t s = nullptr;
  while (st == L1LINE_OK && ctx->rk_step < steps) {
    // example `cursor` of the seed: its sizes, then its entries on the device
    uint64_t hx = ctx->rk_seed * 0x9E3779B97F4A7C15ull + ctx->rk_cursor;
    const uint64_t h = splitmix64(hx);
    const int n = 500 + (int)(h % 3501), m = 50 + (int)((h >> 32) % 451);
    const PhiloxKey key{(uint32_t)(h ^ (h >> 32)), (uint32_t)(ctx->rk_seed ^ (ctx->rk_cursor << 20))};
    hipLaunchKernelGGL(k_gen_training, dim3((unsigned)(((long long)n * m + 255) / 256)), dim3(256), 0, s, X, n, m, key);
    hipLaunchKernelGGL(k_colprep, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, X, n, m, (long long)n, ci);
    hipLaunchKernelGGL(k_max_mass, dim3(1), dim3(256), 0, s, (const ColInfo *)ci, m, mass);
    double big = 0.0;
    if (hipGetLastError() != hipSuccess || hipMemcpy(&big, mass, db, hipMemcpyDeviceToHost) != hipSuccess) {
      st = L1LINE_EHIP;
      break;
    }
    const double lam = 0.05 * big;
    // labels: the exact z_j of every column
    const l1line_problem p = single(X, n, m, n, &lam, 1, V, J, OBJ, nullptr, Z, nullptr);
    st = run_batch(ctx, &p, 1, 0, s, tune_for(ctx, &p, 1), nullptr);
    if (st) break;
    st = ranker_features(ctx, X, n, m, n, lam, F, s);
    if (st) break;
    hipLaunchKernelGGL(k_targets, dim3(1), dim3(256), 0, s, (const double *)Z, m, y);
    st = mlp_grad_impl(ctx, ctx->rk_w, F, y, m, g, loss, s);
    if (st) break;
    ++ctx->rk_step;
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, ctx->rk_w,
                       ctx->rk_w + MLP_NPARAM, ctx->rk_w + 2 * MLP_NPARAM, (const float *)g,
                       (long long)ctx->rk_step, kLr, 0.9f, 0.999f, 1e-8f);
    if (hipGetLastError() != hipSuccess) {
      st = L1LINE_EHIP;
      break;
    }
    ++ctx->rk_cursor;
    if (ckpt_path && (ctx->rk_step % kSaveEvery == 0 || ctx->rk_step == steps)) st = rk_write(ctx, ckpt_path, true);
  }
  if (hipDeviceSynchronize() != hipSuccess && st == L1LINE_OK) st = L1LINE_EHIP;
  (void)hipFree(buf);
  return note(ctx, st);
}

// ------------------------------------------------------------ Algorithm 2
// offsets[1..count] (per-segment counts) into offsets (offsets[0] = 0);
// part: BP_SCAN_BLOCKS scratch values
static void scan_offsets(hipStream_t s, long long *offsets, long long count, long long *part) {
  const int nb = (int)std::max(1ll, std::min((long long)BP_SCAN_BLOCKS, (count + 4095) / 4096));
  hipLaunchKernelGGL(k_bp_scan_sums, dim3(nb), dim3(1024), 0, s, (const long long *)offsets, count, part);
  hipLaunchKernelGGL(k_bp_scan_top, dim3(1), dim3(1024), 0, s, part, nb);
  hipLaunchKernelGGL(k_bp_scan_fin, dim3(nb), dim3(1024), 0, s, offsets, count, (const long long *)part);
}

static int breakpoints_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, int64_t *offsets,
                            double *lambda_max, double *lam, double *v, int32_t *row, int64_t capacity,
                            int32_t *status, void *stream) {
  if (!ctx || !offsets || capacity < 0 || (capacity > 0 && (!lam || !v || !row))) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  if (n > L1LINE_BP_MAX_N) return L1LINE_ESIZE;
  if (m > L1LINE_BP_MAX_M) return L1LINE_ESIZE;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // scratch: the lambda = 0 fit's outputs and lambda_max when not requested
  const size_t o_v = 0, o_j = align_up(sizeof(double) * m, 256), o_obj = o_j + 256,
               o_part = o_obj + 256, o_lm = o_part + align_up(sizeof(long long) * BP_SCAN_BLOCKS, 256),
               total = o_lm + (lambda_max ? 0 : align_up(sizeof(double) * m * m, 256));
  st = ensure_rk(ctx, total, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  double *lm = lambda_max ? lambda_max : (double *)(b + o_lm);
  const double zero = 0.0;
  const l1line_problem p = single(X, n, m, ld, &zero, 1, (double *)(b + o_v), (int64_t *)(b + o_j),
                                  (double *)(b + o_obj), nullptr, nullptr, status);
  BatchPtrs bp;
  st = run_batch(ctx, &p, 1, 0, s, tune_for(ctx, &p, 1), nullptr, kNoOpts, &bp);
  if (st) return st;
  const long long nseg = (long long)m * m;
  const unsigned grid = (unsigned)std::max(8ll, std::min((nseg + 3) / 4, (long long)ctx->num_cu * 8));
  BpList bl;
  if (capacity > 0) {
    st = bp_list(ctx, nseg, s, &bl);
    if (st) return st;
  }
  {
    ProfScope ps(ctx, s, "bp_count");
    if (bl.cap > 0)
      hipLaunchKernelGGL(k_bp_count<true>, dim3(grid), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                         (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, (long long *)offsets + 1,
                         lm, bl.keys, bl.rows, bl.sb, bl.cap);
    else
      hipLaunchKernelGGL(k_bp_count<false>, dim3(grid), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                         (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, (long long *)offsets + 1,
                         lm, (uint64_t *)nullptr, (unsigned short *)nullptr, (u128 *)nullptr, 0);
    scan_offsets(s, (long long *)offsets, nseg, (long long *)(b + o_part));
  }
  if (capacity > 0) {
    ProfScope ps(ctx, s, "bp_emit");
    hipLaunchKernelGGL(k_bp_emit, dim3(grid), dim3(64 * BP_WAVES), 0, s, X, (int)n, (int)m, (long long)ld,
                       (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, (const long long *)offsets,
                       (const double *)lm, (long long)capacity, lam, v, (int *)row, (int *)status, ctx->sticky,
                       (const uint64_t *)bl.keys, (const unsigned short *)bl.rows, (const u128 *)bl.sb, bl.cap);
  }
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_breakpoints(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, int64_t *offsets,
                       double *lambda_max, double *lam, double *v, int32_t *row, int64_t capacity, int32_t *status,
                       void *stream) {
  return note(ctx, breakpoints_impl(ctx, X, n, m, ld, offsets, lambda_max, lam, v, row, capacity, status, stream));
}

// ------------------------------------------------------------ components
static int components_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda,
                           int64_t p, double *work, double *V, int64_t *J, double *OBJ, int32_t *status,
                           void *stream) {
  if (!ctx || !work || !V || !J || !OBJ || p < 1 || p > m || p > L1LINE_MAX_COMPONENTS) return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  st = check_lambdas(&lambda, 1);
  if (st) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const size_t o_W = 0, o_cw = align_up(sizeof(double) * p * m, 256), o_U = o_cw + align_up(sizeof(double) * p, 256),
               o_s = o_U + align_up(sizeof(double) * m, 256), o_cst = o_s + align_up(sizeof(double) * n, 256),
               o_flag = o_cst + align_up(sizeof(int) * p, 256), total = o_flag + align_up(sizeof(int) * p, 256);
  st = ensure_rk(ctx, total, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  double *Wb = (double *)(b + o_W), *cw = (double *)(b + o_cw), *U = (double *)(b + o_U), *sv = (double *)(b + o_s);
  int *cst = (int *)(b + o_cst), *flag = (int *)(b + o_flag);
  const long long nm = (long long)n * m;
  hipLaunchKernelGGL(k_copy_matrix, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, X, (long long)ld, (int)n,
                     (int)m, work);
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((2 * p + 63) / 64)), dim3(64), 0, s, cst, 2ll * p, 0);
  for (int64_t c = 0; c < p; ++c) {
    const l1line_problem pr = single(work, n, m, n, &lambda, 1, V + c * m, J + c, OBJ + c, nullptr, nullptr,
                                     cst + c);
    st = run_batch(ctx, &pr, 1, 0, s, tune_for(ctx, &pr, 1), nullptr);
    if (st) return st;
    if (c == p - 1) break;
    hipLaunchKernelGGL(k_gs, dim3(1), dim3(64), 0, s, (const double *)(V + c * m), Wb, cw, (int)c, (int)m, U,
                       flag + c);
    hipLaunchKernelGGL(k_rowdot, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, (const double *)work, (int)n,
                       (int)m, (const double *)(Wb + c * m), sv);
    hipLaunchKernelGGL(k_deflate, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, work, (int)n, (int)m,
                       (const double *)sv, (const double *)U);
  }
  hipLaunchKernelGGL(k_comp_status, dim3(1), dim3(64), 0, s, (const int *)cst, (const int *)flag, (int)p, status,
                     ctx->sticky);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_components(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, double lambda, int64_t p,
                      double *work, double *V, int64_t *J, double *OBJ, int32_t *status, void *stream) {
  return note(ctx, components_impl(ctx, X, n, m, ld, lambda, p, work, V, J, OBJ, status, stream));
}

// ------------------------------------------------------------ solution path
static int solution_path_impl(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, int64_t capacity,
                              int64_t *count, double *lam, int64_t *jo, int32_t *ko, double *vo, int32_t *ro,
                              double *Eo, double *Po, int32_t *status, void *stream) {
  if (!ctx || !count || capacity < 0 ||
      (capacity > 0 && (!lam || !jo || !ko || !vo || !ro || !Eo || !Po)))
    return L1LINE_EINVAL;
  int st = check_matrix(X, n, m, ld);
  if (st) return st;
  if (n > L1LINE_BP_MAX_N) return L1LINE_ESIZE;
  if (m > L1LINE_BP_MAX_M) return L1LINE_ESIZE;
  *count = 0;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const long long mm = (long long)m * m;
  // small scratch: the lambda = 0 fit, Algorithm 2's offsets, per-segment and
  // per-tile values
  const size_t o_v = 0, o_j = align_up(sizeof(double) * m, 256), o_obj = o_j + 256, o_fst = o_obj + 256,
               o_off = o_fst + 256, o_lm = o_off + align_up(sizeof(long long) * (mm + 1), 256),
               o_segv = o_lm + align_up(sizeof(double) * mm, 256), o_gmax = o_segv + align_up(sizeof(double) * mm, 256),
               o_sc = o_gmax + 256, o_T = o_sc + 256, o_tot = o_T + 256, o_D = o_tot + 256,
               o_bnd = o_D + align_up(sizeof(double) * m, 256), o_U = o_bnd + align_up(sizeof(double) * SP_TMAX, 256),
               o_cnt = o_U + align_up(sizeof(double) * SP_TMAX, 256),
               o_info = o_cnt + align_up(sizeof(int) * SP_TMAX, 256),
               o_sw = o_info + align_up(sizeof(TileInfo) * SP_TMAX, 256),
               o_toff = o_sw + align_up(sizeof(int) * SP_TMAX, 256),
               o_part = o_toff + align_up(sizeof(long long) * (SP_TMAX + 1), 256),
               small = o_part + align_up(sizeof(long long) * BP_SCAN_BLOCKS, 256);
  st = ensure_rk(ctx, small, s);
  if (st) return st;
  char *b = (char *)ctx->rk;
  int *fst = (int *)(b + o_fst);
  long long *offsets = (long long *)(b + o_off);
  double *lm = (double *)(b + o_lm), *segv = (double *)(b + o_segv), *D = (double *)(b + o_D);
  unsigned long long *gmax = (unsigned long long *)(b + o_gmax);
  PathScale *sc = (PathScale *)(b + o_sc);
  int *Tp = (int *)(b + o_T), *cnt = (int *)(b + o_cnt), *sw = (int *)(b + o_sw);
  long long *tot = (long long *)(b + o_tot), *toff = (long long *)(b + o_toff);
  double *bnd = (double *)(b + o_bnd), *U = (double *)(b + o_U);
  TileInfo *info = (TileInfo *)(b + o_info);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, fst, 1ll, 0);
  const double zero = 0.0;
  const l1line_problem p0 = single(X, n, m, ld, &zero, 1, (double *)(b + o_v), (int64_t *)(b + o_j),
                                   (double *)(b + o_obj), nullptr, nullptr, fst);
  BatchPtrs bp;
  st = run_batch(ctx, &p0, 1, 0, s, tune_for(ctx, &p0, 1), nullptr, kNoOpts, &bp);
  if (st) return st;
  const unsigned grid = (unsigned)std::max(8ll, std::min((mm + 3) / 4, (long long)ctx->num_cu * 8));
  BpList bl;
  st = bp_list(ctx, mm, s, &bl);
  if (st) return st;
  {
    ProfScope ps(ctx, s, "bp_count");
    if (bl.cap > 0)
      hipLaunchKernelGGL(k_bp_count<true>, dim3(grid), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                         (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, offsets + 1, lm, bl.keys,
                         bl.rows, bl.sb, bl.cap);
    else
      hipLaunchKernelGGL(k_bp_count<false>, dim3(grid), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                         (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, offsets + 1, lm,
                         (uint64_t *)nullptr, (unsigned short *)nullptr, (u128 *)nullptr, 0);
    scan_offsets(s, offsets, mm, (long long *)(b + o_part));
  }
  long long NE = 0;
  int h_fst = 0;
  HIP_TRY(hipMemcpyAsync(&NE, offsets + mm, sizeof NE, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&h_fst, fst, sizeof h_fst, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h_fst) return h_fst;
  if (NE < 0 || NE > (long long)UINT32_MAX) return L1LINE_ESIZE;
  // per-entry arrays, then per (tile, column) arrays
  const size_t e8 = align_up(sizeof(double) * NE, 256), e4 = align_up(sizeof(int) * NE, 256),
               e16 = align_up(sizeof(u128) * NE, 256), tm = (size_t)SP_TMAX * m;
  const size_t q_lam = 0, q_v = q_lam + e8, q_row = q_v + e8, q_e = q_row + e4, q_dz = q_e + e8,
               q_kA = q_dz + 2 * e16, q_kB = q_kA + e8, q_iA = q_kB + e8, q_iB = q_iA + e4, q_sE = q_iB + e4,
               q_sP = q_sE + e16, q_LB = q_sP + e16, q_list = q_LB + align_up(sizeof(double) * tm, 256),
               q_pos = q_list + align_up(sizeof(int) * tm, 256), q_pb = q_pos + align_up(sizeof(long long) * tm, 256),
               big = q_pb + align_up(sizeof(long long) * tm, 256);
  st = ensure_sp(ctx, big, s);
  if (st) return st;
  char *c = (char *)ctx->sp;
  double *elam = (double *)(c + q_lam), *ev = (double *)(c + q_v), *ee = (double *)(c + q_e),
         *LB = (double *)(c + q_LB);
  int *erow = (int *)(c + q_row), *list = (int *)(c + q_list);
  SpDelta *dz = (SpDelta *)(c + q_dz);
  u128 *stE = (u128 *)(c + q_sE), *stP = (u128 *)(c + q_sP);
  uint64_t *keyA = (uint64_t *)(c + q_kA), *keyB = (uint64_t *)(c + q_kB);
  uint32_t *idA = (uint32_t *)(c + q_iA), *idB = (uint32_t *)(c + q_iB);
  long long *spos = (long long *)(c + q_pos), *spb = (long long *)(c + q_pb);
  {
    ProfScope ps(ctx, s, "bp_emit");
    hipLaunchKernelGGL(k_bp_emit, dim3(grid), dim3(64 * BP_WAVES), 0, s, X, (int)n, (int)m, (long long)ld,
                       (const ColInfo *)bp.ci, (const double *)bp.V, (const int *)bp.R, (const long long *)offsets,
                       (const double *)lm, (long long)NE, elam, ev, erow, fst, ctx->sticky,
                       (const uint64_t *)bl.keys, (const unsigned short *)bl.rows, (const u128 *)bl.sb, bl.cap);
  }
  // the maxima (4 x 8 bytes) and the residual kernel's slot counters (8 ints)
  HIP_TRY(hipMemsetAsync(gmax, 0, 4 * sizeof(unsigned long long) + 8 * sizeof(int), s));
  {
    ProfScope ps(ctx, s, "sp_resid");
    hipLaunchKernelGGL(k_sp_resid, dim3(grid), dim3(256), 0, s, X, (int)n, (int)m, (long long)ld,
                       (const long long *)offsets, (const double *)elam, (const double *)ev, ee, segv, gmax,
                       (int *)(gmax + 4));
  }
  hipLaunchKernelGGL(k_sp_scale, dim3(1), dim3(1), 0, s, (const unsigned long long *)gmax, sc);
  {
    ProfScope ps(ctx, s, "sp_delta");
    hipLaunchKernelGGL(k_sp_delta, dim3(grid), dim3(256), 0, s, (int)m, (const long long *)offsets,
                       (const double *)ev, (const double *)ee, sc, dz);
  }
  {
    ProfScope ps(ctx, s, "sp_sort");
    if (!ctx->attr_sort) {
      HIP_TRY(hipFuncSetAttribute((const void *)k_sp_sort, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)SP_SORT_LDS));
      ctx->attr_sort = true;
    }
    hipLaunchKernelGGL(k_sp_sort, dim3((unsigned)m), dim3(1024), SP_SORT_LDS, s, (int)m, (const long long *)offsets,
                       (const double *)elam, keyA, idA, keyB, idB, (const SpDelta *)dz,
                       (const PathScale *)sc, stE, stP);
  }
  {
    ProfScope ps(ctx, s, "sp_bounds");
    hipLaunchKernelGGL(k_sp_tiles, dim3(1), dim3(1024), 0, s, NE, (const double *)elam, (const PathScale *)sc, bnd,
                       Tp);
    hipLaunchKernelGGL(k_sp_slack, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, (int)n, (int)m,
                       (const ColInfo *)bp.ci, (const double *)segv, (const PathScale *)sc, D);
    hipLaunchKernelGGL(k_sp_bounds, dim3(SP_TMAX), dim3(256), 0, s, (int)m, (const long long *)offsets,
                       (const uint64_t *)keyA, (const u128 *)stE, (const u128 *)stP, (const PathScale *)sc,
                       (const double *)bnd, (const int *)Tp, (const double *)D, LB, U);
    hipLaunchKernelGGL(k_sp_surv, dim3(SP_TMAX), dim3(256), 0, s, (int)m, (const long long *)offsets,
                       (const u128 *)stE, (const double *)LB, (const double *)U, (const int *)Tp, list, cnt);
  }
  PathOut out{lam, (long long *)jo, (int *)ko, vo, (int *)ro, Eo, Po};
  {
    ProfScope ps(ctx, s, "sp_sweep");
    hipLaunchKernelGGL(k_sp_sweep, dim3(SP_TMAX), dim3(64), 0, s, (int)m, (const long long *)offsets,
                       (const double *)elam, (const double *)ev, (const int *)erow, (const uint64_t *)keyA,
                       (const uint32_t *)idA, (const u128 *)stE, (const u128 *)stP, sc,
                       (const double *)bnd, (const int *)Tp, (const int *)list, (const int *)cnt, spos, spb, info,
                       (const long long *)toff, (const int *)sw, 0, out, 0ll);
    hipLaunchKernelGGL(k_sp_toff, dim3(1), dim3(1024), 0, s, (int)m, (const int *)Tp, (const TileInfo *)info, sw,
                       toff, tot);
  }
  PathScale hsc;
  long long total = 0;
  HIP_TRY(hipMemcpyAsync(&total, tot, sizeof total, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&hsc, sc, sizeof hsc, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&h_fst, fst, sizeof h_fst, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  if (h_fst) return h_fst;
  if (hsc.bad) {
    const int code = (hsc.bad & 1) ? L1LINE_EWIDE : L1LINE_EINTERNAL;
    if (status) hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, (int *)status, 1ll, code);
    return code;
  }
  *count = total;
  if (capacity == 0) return L1LINE_OK;
  if (total > capacity) return L1LINE_ESIZE;
  {
    ProfScope ps(ctx, s, "sp_sweep");
    hipLaunchKernelGGL(k_sp_sweep, dim3(SP_TMAX), dim3(64), 0, s, (int)m, (const long long *)offsets,
                       (const double *)elam, (const double *)ev, (const int *)erow, (const uint64_t *)keyA,
                       (const uint32_t *)idA, (const u128 *)stE, (const u128 *)stP, sc,
                       (const double *)bnd, (const int *)Tp, (const int *)list, (const int *)cnt, spos, spb, info,
                       (const long long *)toff, (const int *)sw, 1, out, (long long)capacity);
  }
  if (status) hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, (int *)status, 1ll, 0);
  HIP_TRY(hipGetLastError());
  return L1LINE_OK;
}

int l1line_solution_path(l1line_ctx ctx, const double *X, int64_t n, int64_t m, int64_t ld, int64_t capacity,
                         int64_t *count, double *lam, int64_t *j, int32_t *k, double *v, int32_t *row, double *E,
                         double *P, int32_t *status, void *stream) {
  return note(ctx, solution_path_impl(ctx, X, n, m, ld, capacity, count, lam, j, k, v, row, E, P, status, stream));
}

}  // extern "C"
