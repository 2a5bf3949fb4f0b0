// Vertex insertion and removal with rescaled ranks.  The paper keeps the
// vertex set fixed (Section 3.4) and names vertex additions and deletions,
// with the existing ranks scaled before the computation, as future work
// (Section 6).  Reading taken here: the teleport term of Eq. 1 is
// (1 - alpha)/n, so ranks that satisfy Eq. 1 for n vertices, multiplied by
// n_old / n_new, satisfy it for n_new vertices wherever the edges did not
// change; a vertex with no edges but its self-loop has rank 1 / n_new.  So
//   adding k vertices: ids n .. n+k-1, no edges, rank 1 / (n+k); every
//     other rank times n / (n+k); nothing is marked (the rescaled ranks are
//     already the new fixed point); edges to and from the new vertices come
//     as ordinary batches;
//   removing the k highest ids: every incident edge is deleted as a batch
//     (marking as any batch does), the marks on removed ids are dropped,
//     every remaining rank is multiplied by n / (n-k), and the next update
//     recomputes the marked vertices.
// Per-vertex arrays grow by reallocation (contents copied, new entries
// zero or -1 as at creation) and are left as they are when vertices go.
// New rows start with no slots; their first insertion moves them to the
// spare tail of the adjacency array like any row that outgrows its slots.
#include <vector>

#include "dfpr_common.h"

namespace dfpr {

namespace {

constexpr int kVBlock = 256;

inline int vgrid(int64_t work, int cu) {
  int64_t b = (work + kVBlock - 1) / kVBlock;
  const int64_t lim = (int64_t)(cu > 0 ? cu : 1) * 16;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

// R[i] *= f for i < n_keep; R[i] = 1 / n_new for n_keep <= i < n_new.
template <typename T>
__global__ void k_rescale(T *R, int32_t n_keep, int32_t n_new, double f) {
  const double fresh = 1.0 / (double)n_new;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_new;
       i += (int64_t)gridDim.x * blockDim.x)
    R[i] = i < n_keep ? (T)((double)R[i] * f) : (T)fresh;
}

__global__ void k_iota(int32_t *a, int32_t from, int32_t to) {
  for (int64_t i = from + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < to;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}

__global__ void k_count_flags(const uint32_t *flags, int64_t words, Ctl *ctl) {
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    c += __popc(flags[i] & (kVA * 0x01010101u));
  c = wave_sum(c);
  if (lane_id() == 0 && c) atomicAdd((unsigned long long *)&ctl->marked, c);
}

// Copies rows first .. first+count-1 of one adjacency direction to
// out[pos[i] ..] (one wavefront per row).
__global__ void k_gather_rows(const int64_t *off, const int32_t *deg, const int32_t *adj,
                              int32_t first, int32_t count, const int64_t *pos,
                              int32_t *out) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t i = wave; i < count; i += waves) {
    const int64_t o = off[first + i];
    const int32_t d = deg[first + i];
    for (int32_t j = lane; j < d; j += kWave) out[pos[i] + j] = adj[o + j];
  }
}

// Reallocates *p from old_bytes to new_bytes, keeping the contents; the new
// tail is set to `fill` (a byte value) unless fill < 0.
int grow(dfpr_graph *g, void **p, size_t old_bytes, size_t new_bytes, int fill) {
  hipStream_t s = g->stream;
  void *q = nullptr;
  DFPR_HIP(hipMalloc(&q, new_bytes));
  hipError_t e = hipSuccess;
  if (old_bytes > 0 && *p)
    e = hipMemcpyAsync(q, *p, old_bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && fill >= 0 && new_bytes > old_bytes)
    e = hipMemsetAsync(static_cast<char *>(q) + old_bytes, fill, new_bytes - old_bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    // the old array stays in place; the new one is given back
    (void)hipFree(q);
    return fail(DFPR_EHIP, std::string("growing a per-vertex array: ") + hipGetErrorString(e));
  }
  if (*p) DFPR_HIP(hipFree(*p));
  *p = q;
  return DFPR_OK;
}

template <typename P>
int grow_t(dfpr_graph *g, P **p, size_t old_bytes, size_t new_bytes, int fill) {
  void *v = *p;
  int rc = grow(g, &v, old_bytes, new_bytes, fill);
  *p = static_cast<P *>(v);
  return rc;
}

int rescale_ranks(dfpr_graph *g, int32_t n_keep, double f) {
  hipStream_t s = g->stream;
  const int b = vgrid(g->n, g->cu_count);
  if (g->elem == 8)
    k_rescale<double><<<b, kVBlock, 0, s>>>((double *)g->R[g->cur], n_keep, g->n, f);
  else
    k_rescale<float><<<b, kVBlock, 0, s>>>((float *)g->R[g->cur], n_keep, g->n, f);
  DFPR_HIP(hipGetLastError());
  return refresh_contributions(g);
}

inline size_t flag_bytes(int64_t n) { return (size_t)((n + 3) / 4 * 4); }

}  // namespace

int add_vertices(dfpr_graph *g, int32_t count, int32_t *first_id) {
  if (count <= 0) return fail(DFPR_EINVAL, "count must be > 0");
  if ((int64_t)g->n + count > (int64_t)INT32_MAX - 1)
    return fail(DFPR_EINVAL, "vertex count would exceed 2^31 - 2");
  hipStream_t s = g->stream;
  DFPR_HIP(hipStreamSynchronize(s));
  const int64_t n0 = g->n, n1 = n0 + count;
  const int64_t ng0 = g->ngroups, ng1 = (n1 + kGroup - 1) / kGroup;
  int rc;
  // every array is grown before n changes, so a failure leaves a graph
  // that still works with the old vertex count
  for (Adj *A : {&g->out, &g->in}) {
    if ((rc = grow_t(g, &A->off, n0 * 8, n1 * 8, 0))) return rc;
    if ((rc = grow_t(g, &A->deg, n0 * 4, n1 * 4, 0))) return rc;
    if ((rc = grow_t(g, &A->cap, n0 * 4, n1 * 4, 0))) return rc;
  }
  for (int i = 0; i < 2; ++i) {
    if ((rc = grow(g, &g->R[i], n0 * g->elem, n1 * g->elem, -1))) return rc;
    if ((rc = grow(g, &g->C[i], n0 * g->elem, n1 * g->elem, -1))) return rc;
  }
  // flag bytes past the last vertex may hold bits (a static pass marks
  // whole words): cleared before they become vertices
  const size_t fb0 = flag_bytes(n0);
  DFPR_HIP(hipMemsetAsync(reinterpret_cast<uint8_t *>(g->flags) + n0, 0, fb0 - n0, s));
  if ((rc = grow_t(g, &g->flags, fb0, flag_bytes(n1), 0))) return rc;
  const size_t gb0 = flag_bytes(ng0);
  DFPR_HIP(hipMemsetAsync(reinterpret_cast<uint8_t *>(g->gflags) + ng0, 0, gb0 - ng0, s));
  if ((rc = grow_t(g, &g->gflags, gb0, flag_bytes(ng1), 0))) return rc;
  // the worklist is sized again for the new group count by ensure_split
  // below; until then it keeps its entries (all -1 between updates)
  if ((rc = grow_t(g, &g->wl, n0 * 4, n1 * 4, 0xFF))) return rc;
  if ((rc = grow_t(g, &g->steps, (n0 + 1) * 4, (n1 + 1) * 4, -1))) return rc;
  // tile sums are rebuilt by every update
  if ((rc = grow(g, &g->tiles, 0, 2 * (n1 / 256 + 2) * 16, 0))) return rc;
  if (g->ext2int) {
    if ((rc = grow_t(g, &g->ext2int, n0 * 4, n1 * 4, -1))) return rc;
    if ((rc = grow_t(g, &g->int2ext, n0 * 4, n1 * 4, -1))) return rc;
    // added vertices keep their ids inside
    k_iota<<<vgrid(count, g->cu_count), kVBlock, 0, s>>>(g->ext2int, (int32_t)n0, (int32_t)n1);
    k_iota<<<vgrid(count, g->cu_count), kVBlock, 0, s>>>(g->int2ext, (int32_t)n0, (int32_t)n1);
    DFPR_HIP(hipGetLastError());
  }
  g->n = (int32_t)n1;
  g->ngroups = (int32_t)ng1;
  if ((rc = rescale_ranks(g, (int32_t)n0, (double)n0 / (double)n1))) return rc;
  if ((rc = ensure_split(g))) return rc;
  DFPR_HIP(hipStreamSynchronize(s));
  if (first_id) *first_id = (int32_t)n0;
  return DFPR_OK;
}

int remove_vertices(dfpr_graph *g, int32_t count) {
  if (count <= 0 || count >= g->n)
    return fail(DFPR_EINVAL, "count must be in [1, n)");
  hipStream_t s = g->stream;
  DFPR_HIP(hipStreamSynchronize(s));
  const int32_t n0 = g->n, n1 = n0 - count;
  // the removed caller ids must be the same ids inside (always so for the
  // caller's order and for vertices added by dfpr_add_vertices)
  std::vector<int32_t> i2e;
  if (g->ext2int) {
    std::vector<int32_t> top((size_t)count);
    DFPR_HIP(hipMemcpy(top.data(), g->ext2int + n1, (size_t)count * 4, hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < count; ++i)
      if (top[(size_t)i] != n1 + i)
        return fail(DFPR_EINVAL,
                    "the highest ids are reordered inside this graph: create it with "
                    "reorder 0 to remove vertices");
    i2e.resize((size_t)n0);
    DFPR_HIP(hipMemcpy(i2e.data(), g->int2ext, (size_t)n0 * 4, hipMemcpyDeviceToHost));
  }
  // every edge incident to a removed vertex, in caller ids: the removed
  // rows of both directions are gathered on the device and copied once
  std::vector<int32_t> ds, dd;
  for (int dir = 0; dir < 2; ++dir) {
    const Adj &A = dir == 0 ? g->out : g->in;
    std::vector<int32_t> deg((size_t)count);
    DFPR_HIP(hipMemcpy(deg.data(), A.deg + n1, (size_t)count * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> pos((size_t)count);
    int64_t total = 0;
    for (int32_t i = 0; i < count; ++i) {
      pos[(size_t)i] = total;
      total += deg[(size_t)i];
    }
    if (total == 0) continue;
    void *dpos = nullptr, *drows = nullptr;
    int rc;
    if ((rc = scratch_get(g, 8, (size_t)count * 8, &dpos))) return rc;
    if ((rc = scratch_get(g, 9, (size_t)total * 4, &drows))) return rc;
    DFPR_HIP(hipMemcpyAsync(dpos, pos.data(), (size_t)count * 8, hipMemcpyHostToDevice, s));
    k_gather_rows<<<vgrid((int64_t)count * kWave, g->cu_count), kVBlock, 0, s>>>(
        A.off, A.deg, A.adj, n1, count, static_cast<const int64_t *>(dpos),
        static_cast<int32_t *>(drows));
    DFPR_HIP(hipGetLastError());
    std::vector<int32_t> rows((size_t)total);
    DFPR_HIP(hipMemcpyAsync(rows.data(), drows, (size_t)total * 4, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    for (int32_t i = 0; i < count; ++i) {
      const int32_t r = n1 + i;
      for (int64_t j = pos[(size_t)i]; j < pos[(size_t)i] + deg[(size_t)i]; ++j) {
        const int32_t x = rows[(size_t)j];
        const int32_t xe = i2e.empty() ? x : i2e[(size_t)x];
        ds.push_back(dir == 0 ? r : xe);
        dd.push_back(dir == 0 ? xe : r);
      }
    }
  }
  if (!ds.empty()) {
    int rc = dfpr_apply_batch(g, (int64_t)ds.size(), ds.data(), dd.data(), 0, nullptr,
                              nullptr, DFPR_MEM_HOST, nullptr, nullptr);
    if (rc) return rc;
  }
  // the removed ids leave the vertex set with their marks
  const int64_t ng1 = ((int64_t)n1 + kGroup - 1) / kGroup;
  DFPR_HIP(hipMemsetAsync(reinterpret_cast<uint8_t *>(g->flags) + n1, 0,
                          flag_bytes(n0) - (size_t)n1, s));
  DFPR_HIP(hipMemsetAsync(reinterpret_cast<uint8_t *>(g->gflags) + ng1, 0,
                          flag_bytes(g->ngroups) - (size_t)ng1, s));
  g->n = n1;
  g->ngroups = (int32_t)ng1;
  const int64_t words = ((int64_t)n1 + 3) / 4;
  DFPR_HIP(hipMemsetAsync(&g->ctl->marked, 0, sizeof(long long), s));
  k_count_flags<<<vgrid(words, g->cu_count), kVBlock, 0, s>>>(g->flags, words, g->ctl);
  DFPR_HIP(hipGetLastError());
  int rc = rescale_ranks(g, n1, (double)n0 / (double)n1);
  if (rc) return rc;
  long long marked = 0;
  DFPR_HIP(hipMemcpyAsync(&marked, &g->ctl->marked, 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  g->pending_marks = marked;
  return DFPR_OK;
}

}  // namespace dfpr
