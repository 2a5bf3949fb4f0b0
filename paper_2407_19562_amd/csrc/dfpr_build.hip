// Graph construction: an edge list (device memory) becomes the slack CSR of
// both directions.  Edges form a set (Section 3.4): duplicates and self pairs
// are dropped; the self-loop of every vertex (Section 5.1.3) is implicit and
// never stored.
//
// Per direction: 64-bit keys (row << 32 | other) are radix-sorted, the first
// key of every run of equal keys survives, row degrees are counted, row
// capacities get slack for in-place insertion, and the surviving keys are
// scattered into their rows (rows end up sorted by the other endpoint).
#include <cstring>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "dfpr_common.h"

namespace dfpr {

namespace {

constexpr unsigned long long kNoKey = ~0ull;

__global__ void k_validate(int64_t m, const int32_t *a, const int32_t *b,
                           int32_t n, Ctl *ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = a[i], y = b[i];
    if (x < 0 || x >= n || y < 0 || y >= n) atomicOr(&ctl->invalid, 1);
  }
}

__global__ void k_make_keys(int64_t m, const int32_t *row,
                            const int32_t *other, unsigned long long *keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t r = (uint32_t)row[i], o = (uint32_t)other[i];
    keys[i] = r == o ? kNoKey : ((unsigned long long)r << 32 | o);
  }
}

__global__ void k_heads(int64_t m, const unsigned long long *keys,
                        int64_t *head) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[i];
    head[i] = (k != kNoKey && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
  }
}

__global__ void k_degrees(int64_t m, const unsigned long long *keys,
                          const int64_t *head, int32_t *deg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    if (head[i]) atomicAdd(deg + (keys[i] >> 32), 1);
}

__global__ void k_capacity(int32_t n, const int32_t *deg, int32_t *cap,
                           int64_t *cap64) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = deg[v];
    const int32_t extra = d >> 3 > 4 ? d >> 3 : 4;
    const int32_t c = (d + extra + 3) & ~3;
    cap[v] = c;
    cap64[v] = c;
  }
}

__global__ void k_widen(int32_t n, const int32_t *a, int64_t *b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    b[v] = a[v];
}

// head[] was turned into the exclusive rank of each surviving key by the
// scan; `alive` re-derives survival from the keys themselves.
__global__ void k_fill(int64_t m, const unsigned long long *keys,
                       const int64_t *rank, const int64_t *dstart,
                       const int64_t *off, int32_t *adj) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[i];
    const bool alive = k != kNoKey && (i == 0 || keys[i - 1] != k);
    if (!alive) continue;
    const uint32_t r = (uint32_t)(k >> 32);
    adj[off[r] + (rank[i] - dstart[r])] = (int32_t)(uint32_t)k;
  }
}

__global__ void k_count_src(int64_t m, const int32_t *src, int32_t *cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(cnt + src[i], 1);
}

// Sort key of vertex v: decreasing out-degree, then increasing id.
__global__ void k_order_keys(int32_t n, const int32_t *cnt, int32_t maxdeg,
                             unsigned long long *keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = (unsigned long long)(uint32_t)(maxdeg - cnt[v]) << 32 | (uint32_t)v;
}

__global__ void k_perm_from_keys(int32_t n, const unsigned long long *keys,
                                 int32_t *int2ext, int32_t *ext2int) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)(uint32_t)keys[i];
    int2ext[i] = v;
    ext2int[v] = (int32_t)i;
  }
}

__global__ void k_map_ids(int64_t m, const int32_t *map, const int32_t *a,
                          const int32_t *b, int32_t *a2, int32_t *b2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    a2[i] = map[a[i]];
    b2[i] = map[b[i]];
  }
}

inline int grid_for(int64_t work, int cu) {
  int64_t b = (work + 255) / 256;
  const int64_t lim = (int64_t)cu * 16;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

int build_graph(dfpr_graph *g, int64_t m, const int32_t *src,
                const int32_t *dst) {
  hipStream_t s = g->stream;
  const int32_t n = g->n;
  const int cu = g->cu_count;
  // range check of every id (all or nothing)
  DFPR_HIP(hipMemsetAsync(g->ctl, 0, sizeof(Ctl), s));
  if (m > 0) {
    k_validate<<<grid_for(m, cu), 256, 0, s>>>(m, src, dst, n, g->ctl);
    DFPR_HIP(hipGetLastError());
  }
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  if (g->h_ctl->invalid) return fail(DFPR_EINVAL, "edge id outside [0, n)");

  const size_t mk = (size_t)(m > 0 ? m : 1);
  void *keys_a, *keys_b, *rank, *tmp;
  int rc;

  // Internal order: decreasing out-degree (an ordering heuristic, so the
  // raw input counts, duplicates included, are good enough).  The hot
  // contributions of a power-law graph then sit in few cache lines.
  if (g->p.reorder != 0 && m > 0) {
    int32_t *cnt;
    if ((rc = scratch_get(g, 2, (size_t)n * 4, (void **)&cnt))) return rc;
    DFPR_HIP(hipMemsetAsync(cnt, 0, (size_t)n * 4, s));
    k_count_src<<<grid_for(m, cu), 256, 0, s>>>(m, src, cnt);
    std::vector<int32_t> hc((size_t)n);
    DFPR_HIP(hipMemcpyAsync(hc.data(), cnt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    int32_t maxdeg = 0;
    for (int32_t x : hc) maxdeg = x > maxdeg ? x : maxdeg;
    const double mean = (double)m / (double)n;
    // automatic: large, skewed graphs, in either scheme (the lock-free
    // scheme lists the groups of a sorted graph interleaved, with pieces
    // from a lower in-degree and smaller claims, so that its claims stay
    // even although the first groups hold the heaviest rows)
    const bool autosort = (double)maxdeg >= 8.0 * mean && n >= (1 << 20);
    if (g->p.reorder == 1 || (g->p.reorder == 2 && autosort)) {
      if ((rc = scratch_get(g, 0, (size_t)n * 8, &keys_a))) return rc;
      if ((rc = scratch_get(g, 1, (size_t)n * 8, &keys_b))) return rc;
      k_order_keys<<<grid_for(n, cu), 256, 0, s>>>(n, cnt, maxdeg,
                                                   (unsigned long long *)keys_a);
      size_t tb = 0;
      DFPR_HIP(rocprim::radix_sort_keys(nullptr, tb, (unsigned long long *)keys_a,
                                        (unsigned long long *)keys_b, (size_t)n, 0, 64, s));
      if ((rc = scratch_get(g, 5, tb, &tmp))) return rc;
      DFPR_HIP(rocprim::radix_sort_keys(tmp, tb, (unsigned long long *)keys_a,
                                        (unsigned long long *)keys_b, (size_t)n, 0, 64, s));
      DFPR_HIP(hipMalloc(&g->ext2int, (size_t)n * 4));
      DFPR_HIP(hipMalloc(&g->int2ext, (size_t)n * 4));
      k_perm_from_keys<<<grid_for(n, cu), 256, 0, s>>>(n, (unsigned long long *)keys_b,
                                                       g->int2ext, g->ext2int);
      int32_t *ms, *md;
      if ((rc = scratch_get(g, 6, mk * 4, (void **)&ms))) return rc;
      if ((rc = scratch_get(g, 7, mk * 4, (void **)&md))) return rc;
      k_map_ids<<<grid_for(m, cu), 256, 0, s>>>(m, g->ext2int, src, dst, ms, md);
      DFPR_HIP(hipGetLastError());
      src = ms;
      dst = md;
    }
  }
  if ((rc = scratch_get(g, 0, mk * 8, &keys_a))) return rc;
  if ((rc = scratch_get(g, 1, mk * 8, &keys_b))) return rc;
  if ((rc = scratch_get(g, 2, mk * 8, &rank))) return rc;
  int64_t *cap64, *dstart;
  if ((rc = scratch_get(g, 3, (size_t)n * 8, (void **)&cap64))) return rc;
  if ((rc = scratch_get(g, 4, (size_t)n * 8, (void **)&dstart))) return rc;

  int64_t stored = -1;
  for (int dir = 0; dir < 2; ++dir) {
    Adj &A = dir == 0 ? g->out : g->in;
    const int32_t *row = dir == 0 ? src : dst;
    const int32_t *oth = dir == 0 ? dst : src;
    unsigned long long *ka = (unsigned long long *)keys_a;
    unsigned long long *kb = (unsigned long long *)keys_b;
    int64_t *rk = (int64_t *)rank;
    int64_t uniq = 0;
    if (m > 0) {
      k_make_keys<<<grid_for(m, cu), 256, 0, s>>>(m, row, oth, ka);
      size_t tb = 0;
      DFPR_HIP(rocprim::radix_sort_keys(nullptr, tb, ka, kb, (size_t)m, 0, 64, s));
      if ((rc = scratch_get(g, 5, tb, &tmp))) return rc;
      DFPR_HIP(rocprim::radix_sort_keys(tmp, tb, ka, kb, (size_t)m, 0, 64, s));
      k_heads<<<grid_for(m, cu), 256, 0, s>>>(m, kb, rk);
      DFPR_HIP(hipMemsetAsync(A.deg, 0, sizeof(int32_t) * n, s));
      k_degrees<<<grid_for(m, cu), 256, 0, s>>>(m, kb, rk, A.deg);
      // exclusive rank of the surviving keys
      tb = 0;
      DFPR_HIP(rocprim::exclusive_scan(nullptr, tb, rk, rk, (int64_t)0, (size_t)m,
                                       rocprim::plus<int64_t>(), s));
      if ((rc = scratch_get(g, 5, tb, &tmp))) return rc;
      DFPR_HIP(rocprim::exclusive_scan(tmp, tb, rk, rk, (int64_t)0, (size_t)m,
                                       rocprim::plus<int64_t>(), s));
      int64_t last_rank = 0;
      unsigned long long last_keys[2] = {0, 0};
      DFPR_HIP(hipMemcpyAsync(&last_rank, rk + (m - 1), 8, hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipMemcpyAsync(last_keys, kb + (m > 1 ? m - 2 : 0), m > 1 ? 16 : 8,
                              hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipStreamSynchronize(s));
      const unsigned long long kl = m > 1 ? last_keys[1] : last_keys[0];
      const bool last_alive = kl != kNoKey && (m == 1 || last_keys[0] != kl);
      uniq = last_rank + (last_alive ? 1 : 0);
    } else {
      DFPR_HIP(hipMemsetAsync(A.deg, 0, sizeof(int32_t) * n, s));
    }
    if (stored >= 0 && stored != uniq)
      return fail(DFPR_EHIP, "in/out edge counts disagree");
    stored = uniq;

    k_capacity<<<grid_for(n, cu), 256, 0, s>>>(n, A.deg, A.cap, cap64);
    size_t tb = 0;
    DFPR_HIP(rocprim::exclusive_scan(nullptr, tb, cap64, A.off, (int64_t)0, (size_t)n,
                                     rocprim::plus<int64_t>(), s));
    if ((rc = scratch_get(g, 5, tb, &tmp))) return rc;
    DFPR_HIP(rocprim::exclusive_scan(tmp, tb, cap64, A.off, (int64_t)0, (size_t)n,
                                     rocprim::plus<int64_t>(), s));
    k_widen<<<grid_for(n, cu), 256, 0, s>>>(n, A.deg, cap64);
    tb = 0;
    DFPR_HIP(rocprim::exclusive_scan(nullptr, tb, cap64, dstart, (int64_t)0, (size_t)n,
                                     rocprim::plus<int64_t>(), s));
    if ((rc = scratch_get(g, 5, tb, &tmp))) return rc;
    DFPR_HIP(rocprim::exclusive_scan(tmp, tb, cap64, dstart, (int64_t)0, (size_t)n,
                                     rocprim::plus<int64_t>(), s));
    int64_t last_off = 0;
    int32_t last_cap = 0;
    DFPR_HIP(hipMemcpyAsync(&last_off, A.off + (n - 1), 8, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(&last_cap, A.cap + (n - 1), 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    const int64_t total = last_off + last_cap;
    int64_t spare = total / 4;
    if (spare < (1 << 16)) spare = 1 << 16;
    A.adj_cap = (total + spare + 3) & ~3ll;
    DFPR_HIP(hipMalloc(&A.adj, sizeof(int32_t) * A.adj_cap));
    if (m > 0)
      k_fill<<<grid_for(m, cu), 256, 0, s>>>(m, kb, rk, dstart, A.off, A.adj);
    DFPR_HIP(hipGetLastError());
    unsigned long long used = (unsigned long long)total;
    DFPR_HIP(hipMemcpyAsync(&g->ctl->adj_used[dir], &used, 8, hipMemcpyHostToDevice, s));
    DFPR_HIP(hipStreamSynchronize(s));
  }
  g->m = stored;
  // the build scratch is large; give it back
  for (int i = 0; i < 8; ++i) {
    if (g->scratch[i].p) (void)hipFree(g->scratch[i].p);
    g->scratch[i].p = nullptr;
    g->scratch[i].bytes = 0;
  }
  return DFPR_OK;
}

}  // namespace dfpr
