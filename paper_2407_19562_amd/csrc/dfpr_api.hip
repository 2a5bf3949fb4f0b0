// C entry points of libdfpr: argument checks, graph lifetime, host/device
// marshalling and error reporting.  All computation runs in the kernels of
// dfpr_build.hip, dfpr_apply.hip and dfpr_rank.hip.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dfpr_common.h"

namespace dfpr {

int apply_batch(dfpr_graph *g, int64_t nd, const int32_t *ds,
                const int32_t *dd, int64_t ni, const int32_t *is,
                const int32_t *id, int64_t *applied_del, int64_t *applied_ins);
int run_rank(dfpr_graph *g, int kind, dfpr_stats *st);
int set_ranks_device(dfpr_graph *g, const double *r);
int read_ranks_device(const dfpr_graph *g, double *out);
int stream_copy(void *dst, const void *src, int64_t bytes, hipStream_t s,
                float *ms);
int update_many(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats);
int update_many_noalloc(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats);

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int scratch_get(dfpr_graph *g, int i, size_t bytes, void **out) {
  Scratch &s = g->scratch[i];
  if (bytes == 0) bytes = 1;
  if (s.bytes < bytes) {
    if (s.p) {
      DFPR_HIP(hipStreamSynchronize(g->stream));
      DFPR_HIP(hipFree(s.p));
      s.p = nullptr;
      s.bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    DFPR_HIP(hipMalloc(&s.p, want));
    s.bytes = want;
  }
  *out = s.p;
  return DFPR_OK;
}

int check_params(const dfpr_params *p) {
  if (!p) return fail(DFPR_EINVAL, "params is NULL");
  if (!(p->alpha > 0.0 && p->alpha < 1.0)) return fail(DFPR_EINVAL, "alpha must be in (0,1)");
  if (!(p->tol > 0.0)) return fail(DFPR_EINVAL, "tol must be > 0");
  if (!(p->frontier_tol >= 0.0)) return fail(DFPR_EINVAL, "frontier_tol must be >= 0");
  if (p->max_iters < 1 || p->max_iters > kMaxIters)
    return fail(DFPR_EINVAL, "max_iters must be in [1, 8000]");
  if (p->precision != 32 && p->precision != 64)
    return fail(DFPR_EINVAL, "precision must be 32 or 64");
  if (p->mode != DFPR_ASYNC && p->mode != DFPR_SYNC) return fail(DFPR_EINVAL, "bad mode");
  if (p->split_min_degree < 0) return fail(DFPR_EINVAL, "split_min_degree must be >= 0");
  if (p->kahan_min_degree < 0) return fail(DFPR_EINVAL, "kahan_min_degree must be >= 0");
  if (p->chunk != 0 && (p->chunk < 64 || p->chunk % 64 || p->chunk > 4096))
    return fail(DFPR_EINVAL, "chunk must be 0 or a multiple of 64 in [64, 4096]");
  if (p->block_size != 0 && (p->block_size < 64 || p->block_size > 256 || p->block_size % 64))
    return fail(DFPR_EINVAL, "block_size must be 0, 64, 128, 192 or 256");
  if (p->timeout_ms < 0) return fail(DFPR_EINVAL, "timeout_ms must be >= 0");
  if (p->reorder < 0 || p->reorder > 2) return fail(DFPR_EINVAL, "reorder must be 0, 1 or 2");
  // block_size 0: the library's choice, at most 256 threads
  const int64_t waves = (p->block_size > 0 ? p->block_size : 256) / 64;
  if (p->grid_blocks < 0 || (int64_t)p->grid_blocks * waves > 32768)
    return fail(DFPR_EINVAL, "grid_blocks * waves per block must be <= 32768");
  if (p->graph_replay < 0 || p->graph_replay > 2)
    return fail(DFPR_EINVAL, "graph_replay must be 0, 1 or 2");
  if (p->lf_stop != DFPR_STOP_TOL && p->lf_stop != DFPR_STOP_FRONTIER)
    return fail(DFPR_EINVAL, "lf_stop must be DFPR_STOP_TOL or DFPR_STOP_FRONTIER");
  return DFPR_OK;
}

static void release(dfpr_graph *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  void *ptrs[] = {g->out.off, g->out.deg, g->out.cap, g->out.adj,
                  g->in.off,  g->in.deg,  g->in.cap,  g->in.adj,
                  g->R[0],    g->R[1],    g->C[0],    g->C[1],
                  g->flags,   g->wl,      g->ctl,     g->sync_max,
                  g->sync_grab, g->sync_len, g->gflags, g->gwl,
                  g->ext2int, g->int2ext, g->steps,
                  g->split.lrow, g->split.lpre, g->split.lcnt, g->split.prow,
                  g->split.ppart, g->split.ptag, g->split.xrow, g->tiles, g->faults};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &s : g->scratch)
    if (s.p) (void)hipFree(s.p);
  if (g->h_ctl) (void)hipHostFree(g->h_ctl);
  for (auto &e : g->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : g->iter_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &row : g->replay)
    for (auto &x : row)
      if (x) (void)hipGraphExecDestroy(x);
  if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
  delete g;
}

static int alloc_graph(dfpr_graph *g) {
  const size_t n = (size_t)g->n;
  DFPR_HIP(hipMalloc(&g->out.off, n * 8));
  DFPR_HIP(hipMalloc(&g->out.deg, n * 4));
  DFPR_HIP(hipMalloc(&g->out.cap, n * 4));
  DFPR_HIP(hipMalloc(&g->in.off, n * 8));
  DFPR_HIP(hipMalloc(&g->in.deg, n * 4));
  DFPR_HIP(hipMalloc(&g->in.cap, n * 4));
  for (int i = 0; i < 2; ++i) {
    DFPR_HIP(hipMalloc(&g->R[i], n * g->elem));
    DFPR_HIP(hipMalloc(&g->C[i], n * g->elem));
  }
  const size_t fbytes = (n + 3) / 4 * 4;
  DFPR_HIP(hipMalloc(&g->flags, fbytes));
  DFPR_HIP(hipMemsetAsync(g->flags, 0, fbytes, g->stream));
  DFPR_HIP(hipMalloc(&g->steps, (n + 1) * 4));
  DFPR_HIP(hipMalloc(&g->tiles, 2 * (n / 256 + 2) * 16));
  DFPR_HIP(hipMemsetAsync(g->tiles, 0, 2 * (n / 256 + 2) * 16, g->stream));
  DFPR_HIP(hipMalloc(&g->wl, n * 4));
  DFPR_HIP(hipMemsetAsync(g->wl, 0xFF, n * 4, g->stream));
  g->ngroups = (int32_t)((n + kGroup - 1) / kGroup);
  const size_t gbytes = ((size_t)g->ngroups + 3) / 4 * 4;
  DFPR_HIP(hipMalloc(&g->gflags, gbytes));
  DFPR_HIP(hipMemsetAsync(g->gflags, 0, gbytes, g->stream));
  DFPR_HIP(hipMalloc(&g->gwl, (size_t)g->ngroups * 4));
  DFPR_HIP(hipMemsetAsync(g->gwl, 0xFF, (size_t)g->ngroups * 4, g->stream));
  g->gwl_cap = g->ngroups;  // ensure_split adds room for the pieces
  DFPR_HIP(hipMalloc(&g->ctl, sizeof(Ctl)));
  DFPR_HIP(hipMemsetAsync(g->ctl, 0, sizeof(Ctl), g->stream));
  DFPR_HIP(hipHostMalloc(&g->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  DFPR_HIP(hipMalloc(&g->sync_max, kMaxIters * 8));
  DFPR_HIP(hipMalloc(&g->sync_grab, kClaimers * kClaimStride * 8));
  DFPR_HIP(hipMalloc(&g->sync_len, kMaxIters * 8));
  for (auto &e : g->ev) DFPR_HIP(hipEventCreate(&e));
  return DFPR_OK;
}

// Copies a host array to a device scratch slot (or passes device pointers).
static int stage(dfpr_graph *g, int slot, const int32_t *p, int64_t count,
                 int mem, const int32_t **out) {
  if (count == 0 || mem == DFPR_MEM_DEVICE) {
    *out = p;
    return DFPR_OK;
  }
  void *d = nullptr;
  int rc = scratch_get(g, slot, (size_t)count * 4, &d);
  if (rc) return rc;
  DFPR_HIP(hipMemcpyAsync(d, p, (size_t)count * 4, hipMemcpyHostToDevice, g->stream));
  *out = (const int32_t *)d;
  return DFPR_OK;
}

static int check_mem(int mem) {
  return (mem == DFPR_MEM_HOST || mem == DFPR_MEM_DEVICE)
             ? DFPR_OK
             : fail(DFPR_EINVAL, "mem must be DFPR_MEM_HOST or DFPR_MEM_DEVICE");
}

}  // namespace dfpr

using namespace dfpr;

extern "C" {

int dfpr_params_default(dfpr_params *p) {
  if (!p) return fail(DFPR_EINVAL, "params is NULL");
  memset(p, 0, sizeof(*p));
  p->alpha = 0.85;
  p->tol = 1e-10;
  p->frontier_tol = 1e-13;
  p->max_iters = 500;
  p->precision = 64;
  p->mode = DFPR_ASYNC;
  p->kahan_min_degree = 0;
  p->split_min_degree = 0;
  p->chunk = 0;
  p->block_size = 0;
  p->reorder = 2;
  p->renormalize = 0;
  p->timeout_ms = 60000;
  p->grid_blocks = 0;
  p->graph_replay = 2;
  p->lf_stop = DFPR_STOP_TOL;
  return DFPR_OK;
}

int dfpr_graph_create(int32_t n, int64_t m, const int32_t *src,
                      const int32_t *dst, int mem, const dfpr_params *params,
                      void *hip_stream, dfpr_graph **out) {
  if (!out) return fail(DFPR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0) return fail(DFPR_EINVAL, "n must be > 0");
  if (m < 0 || (m > 0 && (!src || !dst))) return fail(DFPR_EINVAL, "bad edge arrays");
  if (m > ((int64_t)1 << 31)) return fail(DFPR_EINVAL, "m above 2^31 is not supported");
  int rc = check_mem(mem);
  if (rc) return rc;
  dfpr_params p;
  if (params)
    p = *params;
  else
    dfpr_params_default(&p);
  if ((rc = check_params(&p))) return rc;
  if (mem == DFPR_MEM_HOST)
    for (int64_t i = 0; i < m; ++i)
      if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n)
        return fail(DFPR_EINVAL, "edge id outside [0, n)");
  dfpr_graph *g = new dfpr_graph();
  g->n = n;
  g->p = p;
  g->elem = p.precision == 64 ? 8 : 4;
  g->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&g->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&g->cu_count, hipDeviceAttributeMultiprocessorCount, g->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&g->wallclock_khz, hipDeviceAttributeWallClockRate, g->device);
  if (e != hipSuccess) {
    release(g);
    return fail(DFPR_EHIP, std::string("device query: ") + hipGetErrorString(e));
  }
  if ((rc = alloc_graph(g))) {
    release(g);
    return rc;
  }
  const int32_t *ds = src, *dd = dst;
  if ((rc = stage(g, 14, src, m, mem, &ds)) || (rc = stage(g, 15, dst, m, mem, &dd))) {
    release(g);
    return rc;
  }
  if ((rc = build_graph(g, m, ds, dd))) {
    release(g);
    return rc;
  }
  if ((rc = init_uniform_ranks(g)) || (rc = ensure_split(g))) {
    release(g);
    return rc;
  }
  e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) {
    release(g);
    return fail(DFPR_EHIP, hipGetErrorString(e));
  }
  for (int i = 14; i < 16; ++i) {
    if (g->scratch[i].p) (void)hipFree(g->scratch[i].p);
    g->scratch[i] = Scratch{};
  }
  *out = g;
  return DFPR_OK;
}

int dfpr_graph_destroy(dfpr_graph *g) {
  release(g);
  return DFPR_OK;
}

int dfpr_set_params(dfpr_graph *g, const dfpr_params *p) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (p->precision != g->p.precision)
    return fail(DFPR_EINVAL, "precision is fixed at graph creation");
  g->p = *p;
  // piece arrays sized for the (possibly lower) split threshold now, not in
  // the next update
  return ensure_split(g);
}

int dfpr_get_params(const dfpr_graph *g, dfpr_params *p) {
  if (!g || !p) return fail(DFPR_EINVAL, "NULL argument");
  *p = g->p;
  return DFPR_OK;
}

int dfpr_graph_size(const dfpr_graph *g, int32_t *n, int64_t *m) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  return DFPR_OK;
}

int dfpr_static(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 0, stats);
}

int dfpr_naive_dynamic(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 1, stats);
}

int dfpr_static_lock_free(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 3, stats);
}

int dfpr_naive_dynamic_lock_free(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 4, stats);
}

int dfpr_set_faults(dfpr_graph *g, const int32_t *table, int32_t count) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (count < 0 || (count > 0 && !table)) return fail(DFPR_EINVAL, "bad fault table");
  for (int32_t i = 0; i < count; ++i)
    if (table[i] < -1 || table[i] > 1000000)
      return fail(DFPR_EINVAL, "fault entries must be -1, 0 or a delay in (0, 1e6] us");
  DFPR_HIP(hipStreamSynchronize(g->stream));
  if (g->faults) {
    DFPR_HIP(hipFree(g->faults));
    g->faults = nullptr;
  }
  g->nfaults = 0;
  g->fault_stops = 0;
  if (count == 0) return DFPR_OK;
  DFPR_HIP(hipMalloc(&g->faults, (size_t)count * 4));
  DFPR_HIP(hipMemcpy(g->faults, table, (size_t)count * 4, hipMemcpyHostToDevice));
  g->nfaults = count;
  for (int32_t i = 0; i < count; ++i)
    if (table[i] < 0) g->fault_stops = 1;
  return DFPR_OK;
}

int dfpr_update(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 2, stats);
}

int dfpr_add_vertices(dfpr_graph *g, int32_t count, int32_t *first_id) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  return add_vertices(g, count, first_id);
}

int dfpr_remove_vertices(dfpr_graph *g, int32_t count) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  return remove_vertices(g, count);
}

int dfpr_mark_reachable(dfpr_graph *g, int64_t *marked) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  return mark_reachable(g, marked);
}

int dfpr_update_traversal(dfpr_graph *g, dfpr_stats *stats) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (stats) *stats = dfpr_stats{};
  return run_rank(g, 5, stats);
}

int dfpr_update_many(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats) {
  if (count < 0 || (count > 0 && !gs)) return fail(DFPR_EINVAL, "bad graph list");
  for (int32_t i = 0; i < count; ++i)
    if (!gs[i]) return fail(DFPR_EINVAL, "NULL graph in list");
  return update_many(gs, count, stats);
}

int dfpr_update_many_noalloc(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats) {
  if (count < 0 || (count > 0 && !gs)) return fail(DFPR_EINVAL, "bad graph list");
  for (int32_t i = 0; i < count; ++i)
    if (!gs[i]) return fail(DFPR_EINVAL, "NULL graph in list");
  return update_many_noalloc(gs, count, stats);
}

int dfpr_set_ranks(dfpr_graph *g, const double *r, int mem) {
  if (!g || !r) return fail(DFPR_EINVAL, "NULL argument");
  int rc = check_mem(mem);
  if (rc) return rc;
  const double *d = r;
  if (mem == DFPR_MEM_HOST) {
    void *tmp = nullptr;
    if ((rc = scratch_get(g, 13, (size_t)g->n * 8, &tmp))) return rc;
    DFPR_HIP(hipMemcpyAsync(tmp, r, (size_t)g->n * 8, hipMemcpyHostToDevice, g->stream));
    d = (const double *)tmp;
  }
  if ((rc = set_ranks_device(g, d))) return rc;
  DFPR_HIP(hipStreamSynchronize(g->stream));
  return DFPR_OK;
}

int dfpr_read_ranks(const dfpr_graph *g, double *out, int mem) {
  if (!g || !out) return fail(DFPR_EINVAL, "NULL argument");
  int rc = check_mem(mem);
  if (rc) return rc;
  dfpr_graph *gm = const_cast<dfpr_graph *>(g);
  if (mem == DFPR_MEM_DEVICE) {
    if ((rc = read_ranks_device(g, out))) return rc;
  } else {
    void *tmp = nullptr;
    if ((rc = scratch_get(gm, 13, (size_t)g->n * 8, &tmp))) return rc;
    if ((rc = read_ranks_device(g, (double *)tmp))) return rc;
    DFPR_HIP(hipMemcpyAsync(out, tmp, (size_t)g->n * 8, hipMemcpyDeviceToHost, g->stream));
  }
  DFPR_HIP(hipStreamSynchronize(g->stream));
  return DFPR_OK;
}

int dfpr_apply_batch(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
                     const int32_t *del_dst, int64_t n_ins,
                     const int32_t *ins_src, const int32_t *ins_dst, int mem,
                     int64_t *applied_del, int64_t *applied_ins) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (n_del < 0 || n_ins < 0) return fail(DFPR_EINVAL, "negative batch size");
  if ((n_del > 0 && (!del_src || !del_dst)) || (n_ins > 0 && (!ins_src || !ins_dst)))
    return fail(DFPR_EINVAL, "NULL batch array");
  if (n_del + n_ins > ((int64_t)1 << 31)) return fail(DFPR_EINVAL, "batch too large");
  int rc = check_mem(mem);
  if (rc) return rc;
  if (mem == DFPR_MEM_HOST) {
    const int32_t n = g->n;
    for (int64_t i = 0; i < n_del; ++i)
      if (del_src[i] < 0 || del_src[i] >= n || del_dst[i] < 0 || del_dst[i] >= n)
        return fail(DFPR_EINVAL, "batch id outside [0, n)");
    for (int64_t i = 0; i < n_ins; ++i)
      if (ins_src[i] < 0 || ins_src[i] >= n || ins_dst[i] < 0 || ins_dst[i] >= n)
        return fail(DFPR_EINVAL, "batch id outside [0, n)");
  }
  const int32_t *a, *b, *c, *d;
  if ((rc = stage(g, 4, del_src, n_del, mem, &a)) || (rc = stage(g, 5, del_dst, n_del, mem, &b)) ||
      (rc = stage(g, 6, ins_src, n_ins, mem, &c)) || (rc = stage(g, 15, ins_dst, n_ins, mem, &d)))
    return rc;
  return apply_batch(g, n_del, a, b, n_ins, c, d, applied_del, applied_ins);
}

int dfpr_read_edges(const dfpr_graph *g, int dir, int32_t *src, int32_t *dst,
                    int64_t cap, int64_t *count) {
  if (!g || !count) return fail(DFPR_EINVAL, "NULL argument");
  if (dir != DFPR_OUT && dir != DFPR_IN) return fail(DFPR_EINVAL, "bad direction");
  const Adj &A = dir == DFPR_OUT ? g->out : g->in;
  const size_t n = (size_t)g->n;
  std::vector<int64_t> off(n);
  std::vector<int32_t> deg(n);
  std::vector<int32_t> adj((size_t)A.adj_cap);
  DFPR_HIP(hipMemcpyAsync(off.data(), A.off, n * 8, hipMemcpyDeviceToHost, g->stream));
  DFPR_HIP(hipMemcpyAsync(deg.data(), A.deg, n * 4, hipMemcpyDeviceToHost, g->stream));
  DFPR_HIP(hipMemcpyAsync(adj.data(), A.adj, (size_t)A.adj_cap * 4, hipMemcpyDeviceToHost,
                          g->stream));
  std::vector<int32_t> ext(g->int2ext ? n : 0);
  if (g->int2ext)
    DFPR_HIP(hipMemcpyAsync(ext.data(), g->int2ext, n * 4, hipMemcpyDeviceToHost, g->stream));
  DFPR_HIP(hipStreamSynchronize(g->stream));
  auto X = [&](int64_t v) { return g->int2ext ? ext[(size_t)v] : (int32_t)v; };
  int64_t total = 0;
  for (size_t v = 0; v < n; ++v) total += deg[v];
  *count = total;
  if (!src || !dst) return DFPR_OK;
  if (cap < total) return fail(DFPR_EINVAL, "cap smaller than the edge count");
  int64_t k = 0;
  for (size_t v = 0; v < n; ++v) {
    for (int32_t j = 0; j < deg[v]; ++j) {
      const int32_t w = X(adj[(size_t)off[v] + j]);
      if (dir == DFPR_OUT) {
        src[k] = X((int64_t)v);
        dst[k] = w;
      } else {
        src[k] = w;
        dst[k] = X((int64_t)v);
      }
      ++k;
    }
  }
  return DFPR_OK;
}

int dfpr_read_marks(const dfpr_graph *g, uint8_t *affected, int64_t *count) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (affected) {
    std::vector<uint8_t> f(((size_t)g->n + 3) / 4 * 4);
    std::vector<int32_t> ext(g->int2ext ? (size_t)g->n : 0);
    DFPR_HIP(hipMemcpyAsync(f.data(), g->flags, f.size(), hipMemcpyDeviceToHost, g->stream));
    if (g->int2ext)
      DFPR_HIP(hipMemcpyAsync(ext.data(), g->int2ext, (size_t)g->n * 4, hipMemcpyDeviceToHost,
                              g->stream));
    DFPR_HIP(hipStreamSynchronize(g->stream));
    for (int32_t v = 0; v < g->n; ++v)
      affected[g->int2ext ? ext[(size_t)v] : v] = (f[v] & kVA) ? 1 : 0;
  }
  if (count) {
    unsigned long long t = 0;
    DFPR_HIP(hipMemcpyAsync(&t, &g->ctl->marked, 8, hipMemcpyDeviceToHost, g->stream));
    DFPR_HIP(hipStreamSynchronize(g->stream));
    *count = (int64_t)t;
  }
  return DFPR_OK;
}

int dfpr_graph_bytes(const dfpr_graph *g, int64_t *bytes) {
  if (!g || !bytes) return fail(DFPR_EINVAL, "NULL argument");
  const int64_t n = g->n;
  int64_t b = 2 * (n * 16 + 0) + 4 * (g->out.adj_cap + g->in.adj_cap) + 4 * n * g->elem +
              (n + 3) / 4 * 4 + n * 4 + (int64_t)sizeof(Ctl) + 3 * 8 * kMaxIters;
  for (const auto &s : g->scratch) b += (int64_t)s.bytes;
  *bytes = b;
  return DFPR_OK;
}

int dfpr_stream_copy(void *dst, const void *src, int64_t bytes, void *hip_stream,
                     float *ms) {
  if (!dst || !src || bytes < 0) return fail(DFPR_EINVAL, "bad copy arguments");
  return stream_copy(dst, src, bytes, (hipStream_t)hip_stream, ms);
}

int dfpr_last_kernel_bytes(const dfpr_graph *g, double *bytes, int32_t *launches) {
  if (!g) return fail(DFPR_EINVAL, "graph is NULL");
  if (bytes) *bytes = g->last_bytes;
  if (launches) *launches = g->last_launches;
  return DFPR_OK;
}

const char *dfpr_strerror(int status) {
  switch (status) {
    case DFPR_OK: return "ok";
    case DFPR_NOTCONVERGED: return "iteration cap reached before convergence";
    case DFPR_EINVAL: return "invalid argument";
    case DFPR_ENOMEM: return "out of device memory";
    case DFPR_EHIP: return "HIP runtime error";
    case DFPR_EABORT: return "watchdog abort";
    case DFPR_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

const char *dfpr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
