// Marking of the Dynamic Traversal approach (Section 3.5.2; Algorithms 7
// and 8, before the iterations): every vertex reachable in the current
// graph from the previous or current out-neighbours of a batch source is
// affected.  The batch application has already marked those out-neighbours
// (and, through the self-loops, the sources); this pass extends the marks
// to their closure under the stored out-edges.
//
// Breadth first, one launch per level.  Level L expands the vertices listed
// in list[L & 1] (one wavefront per vertex, lanes striding over its
// out-row) and appends every vertex it marks first (the affected bit set by
// a fetch-or on the flag word, so each vertex is listed once) to
// list[(L + 1) & 1].  An expanded vertex gets kEX, so the update that
// follows never scans its out-row again: a Dynamic Frontier update over
// these marks recomputes the closed set without growing it, which is the
// Dynamic Traversal update.  The three level counters rotate so that no
// launch both reads and clears the same one:
//   cnt[L % 3]        vertices listed for level L (read)
//   cnt[(L + 1) % 3]  vertices listed for level L + 1 (appended to)
//   cnt[(L + 2) % 3]  cleared by level L for level L + 1 to append to
// The host launches levels in groups (8 levels, doubling up to 64) and
// stops at the first empty level it reads.
// Every vertex is listed at most once over the whole traversal, so each
// list holds at most n entries and the traversal takes at most n levels.
#include "dfpr_common.h"

namespace dfpr {

namespace {

constexpr int kTravBlock = 256;
constexpr int kTravLevelsPerPoll = 8;
constexpr int kTravMaxLevelsPerPoll = 64;

inline int grid_for(int64_t work, int cu) {
  int64_t b = (work + kTravBlock - 1) / kTravBlock;
  const int64_t lim = (int64_t)cu * 16;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

__global__ void k_trav_init(unsigned long long *cnt) {
  if (blockIdx.x == 0 && threadIdx.x < 3) cnt[threadIdx.x] = 0;
}

// Level 0: every affected vertex whose out-row has not been walked.
__global__ void __launch_bounds__(kTravBlock) k_trav_seed(const uint32_t *flags, int32_t n,
                                                           int32_t *list,
                                                           unsigned long long *cnt) {
  // the loop bound is uniform over the workgroup: wave_append needs every
  // lane of the wavefront
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = base + threadIdx.x;
    bool want = false;
    if (v < n) {
      const uint32_t f = flag_byte(flags, (int32_t)v, false);
      want = (f & kVA) && !(f & kEX);
    }
    wave_append(want, (int32_t)v, list, cnt, false);
  }
}

__global__ void __launch_bounds__(kTravBlock) k_trav_level(
    const int64_t *out_off, const int32_t *out_deg, const int32_t *out_adj, uint32_t *flags,
    uint32_t *gflags, const int32_t *in, int32_t *next, unsigned long long *cnt, int level,
    Ctl *ctl) {
  const unsigned long long len = cnt[level % 3];
  unsigned long long *ocnt = cnt + (level + 1) % 3;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(level + 2) % 3] = 0;
  const int lane = lane_id();
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const long long waves = (long long)gridDim.x * blockDim.x / kWave;
  unsigned long long found = 0;
  for (long long i = wave; i < (long long)len; i += waves) {
    const int32_t x = in[i];
    if (lane == 0) flag_set(flags, x, kEX);
    const int64_t off = out_off[x];
    const int32_t d = out_deg[x];
    for (int32_t b = 0; b < d; b += kWave) {
      const int32_t j = b + lane;
      bool fresh = false;
      int32_t y = -1;
      if (j < d) {
        y = out_adj[off + j];
        if (!(flag_byte(flags, y, false) & kVA)) fresh = !(flag_set(flags, y, kVA) & kVA);
        // group bytes only go from 0 to listed during the marking
        if (fresh) reinterpret_cast<uint8_t *>(gflags)[y >> kGroupShift] = (uint8_t)kGA;
      }
      found += (unsigned long long)wave_append(fresh, y, next, ocnt, false);
    }
  }
  if (lane == 0 && found) atomicAdd((unsigned long long *)&ctl->marked, found);
}

}  // namespace

int mark_reachable(dfpr_graph *g, int64_t *marked) {
  hipStream_t s = g->stream;
  if (g->pending_marks == 0 || g->n == 0) {
    if (marked) *marked = 0;
    return DFPR_OK;
  }
  const int cu = g->cu_count > 0 ? g->cu_count : 1;
  void *la = nullptr, *lb = nullptr, *c = nullptr;
  int rc;
  if ((rc = scratch_get(g, 8, (size_t)g->n * 4, &la))) return rc;
  if ((rc = scratch_get(g, 9, (size_t)g->n * 4, &lb))) return rc;
  if ((rc = scratch_get(g, 10, 3 * sizeof(unsigned long long), &c))) return rc;
  auto *cnt = static_cast<unsigned long long *>(c);
  int32_t *lists[2] = {static_cast<int32_t *>(la), static_cast<int32_t *>(lb)};
  k_trav_init<<<1, 64, 0, s>>>(cnt);
  k_trav_seed<<<grid_for(g->n, cu), kTravBlock, 0, s>>>(g->flags, g->n, lists[0], cnt);
  DFPR_HIP(hipGetLastError());
  // a fixed grid of 32 wavefronts per CU strides over each level's list
  // (8 per CU measured the same on the grid and 1% slower on R-MAT)
  const int blocks = 8 * cu;
  unsigned long long h[3] = {0, 0, 0};
  // the poll interval doubles up to kTravMaxLevelsPerPoll, so a deep
  // traversal (a road-like grid needs thousands of levels) pays few host
  // round trips; levels past the last one return at once
  int64_t poll = kTravLevelsPerPoll, next_poll = kTravLevelsPerPoll;
  for (int64_t level = 0;; ++level) {
    if (level > (int64_t)g->n + kTravMaxLevelsPerPoll)
      return fail(DFPR_EHIP, "traversal did not end within n levels");
    const int L = (int)level;
    k_trav_level<<<blocks, kTravBlock, 0, s>>>(g->out.off, g->out.deg, g->out.adj, g->flags,
                                               g->gflags, lists[L & 1], lists[(L + 1) & 1],
                                               cnt, L, g->ctl);
    DFPR_HIP(hipGetLastError());
    if (level + 1 == next_poll) {
      DFPR_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipStreamSynchronize(s));
      if (h[(level + 1) % 3] == 0) break;
      if (poll < kTravMaxLevelsPerPoll) poll *= 2;
      next_poll += poll;
    }
  }
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  g->pending_marks = (int64_t)g->h_ctl->marked;
  if (marked) *marked = g->pending_marks;
  return DFPR_OK;
}

}  // namespace dfpr
