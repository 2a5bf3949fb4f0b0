// In-place batch update of the slack CSR (Section 3.4) and the initial
// marking of the Dynamic Frontier approach (Section 4.1.1; Algorithms 1
// and 2, before the iterations).
//
// Per direction the batch becomes 64-bit keys row << 32 | other << 1 | ins
// (ins = 0 deletion, 1 insertion), radix-sorted and de-duplicated, so each
// touched row owns one contiguous segment, sorted by the other endpoint with
// a deletion ahead of an insertion of the same pair.  One wavefront edits one
// row:
//   deletions: every row entry is looked up (binary search) among the
//     segment's deletions and the survivors are compacted in place
//     (ballot + popcount prefix), O(deg log k) per row whatever k is;
//   insertions: row entries are looked up among the segment's insertions to
//     drop those already present, then the new ones are appended; a row that
//     would outgrow its slots first moves to the spare tail of the adjacency
//     array (atomic bump pointer).  When the spare tail runs out the host
//     grows the array and re-runs the rows left pending.
// Marking: for every source u with a real change, u itself (self-loop), its
// current out-neighbours and the targets of its deleted edges -- together
// (G^{t-1} union G^t).out(u) -- get the affected flag and their 256-vertex
// group the listed flag, by plain byte stores (between updates a flag byte
// only ever goes from 0 to set, so the stores need no atomics); the set
// flags are counted afterwards.  The update builds its work lists from
// these flags.
// Rows of at least kLongApply entries are not left to one wavefront:
// their deletions run in a second launch with a 1024-thread workgroup per
// row (segment keys staged in LDS, block-wide compaction), and their
// out-rows are marked by every wavefront of a second launch together.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "dfpr_common.h"

namespace dfpr {

namespace {

constexpr unsigned long long kNoKey = ~0ull;
constexpr uint8_t kApplied = 1, kExists = 2;
constexpr int32_t kLongApply = 4096;  // row entries from which rows are
                                      // edited by more than one wavefront
constexpr int kLongBlock = 1024;      // threads of a long-row deletion block
constexpr int kKeyLds = 2048;         // segment keys staged in LDS
constexpr int kDelPer = 8;            // row entries per thread and round of it

inline int grid_for(int64_t work, int cu) {
  int64_t b = (work + 255) / 256;
  const int64_t lim = (int64_t)cu * 16;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

__global__ void k_validate2(int64_t m1, const int32_t *a1, const int32_t *b1,
                            int64_t m2, const int32_t *a2, const int32_t *b2,
                            int32_t n, Ctl *ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m1 + m2;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = i < m1 ? a1[i] : a2[i - m1];
    const int32_t y = i < m1 ? b1[i] : b2[i - m1];
    if (x < 0 || x >= n || y < 0 || y >= n) atomicOr(&ctl->invalid, 1);
  }
}

// dir 0: rows are sources (out), dir 1: rows are targets (in)
// ids are mapped to the internal order when `map` is set
__global__ void k_batch_keys(int dir, int64_t nd, const int32_t *ds,
                             const int32_t *dd, int64_t ni, const int32_t *is,
                             const int32_t *id, const int32_t *map,
                             unsigned long long *keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nd + ni;
       i += (int64_t)gridDim.x * blockDim.x) {
    const bool ins = i >= nd;
    int32_t a = ins ? is[i - nd] : ds[i];
    int32_t b = ins ? id[i - nd] : dd[i];
    if (map) {
      a = map[a];
      b = map[b];
    }
    const uint32_t u = (uint32_t)a;
    const uint32_t v = (uint32_t)b;
    const uint32_t row = dir == 0 ? u : v, oth = dir == 0 ? v : u;
    keys[i] = u == v ? kNoKey
                     : ((unsigned long long)row << 32 |
                        (unsigned long long)oth << 1 | (ins ? 1u : 0u));
  }
}

// head: first copy of a key; seg: first key of a row
__global__ void k_batch_heads(int64_t m, const unsigned long long *k,
                              int64_t *head, int64_t *seg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long x = k[i];
    const bool h = x != kNoKey && (i == 0 || k[i - 1] != x);
    const bool s = x != kNoKey && (i == 0 || (k[i - 1] >> 32) != (x >> 32));
    head[i] = h;
    seg[i] = s;
  }
}

__global__ void k_batch_compact(int64_t m, const unsigned long long *k,
                                const int64_t *hrank, const int64_t *srank,
                                unsigned long long *uk, int64_t *segstart) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long x = k[i];
    const bool h = x != kNoKey && (i == 0 || k[i - 1] != x);
    const bool s = x != kNoKey && (i == 0 || (k[i - 1] >> 32) != (x >> 32));
    if (h) uk[hrank[i]] = x;
    if (s) segstart[srank[i]] = hrank[i];
  }
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__device__ __forceinline__ int64_t find_key(const unsigned long long *uk,
                                            int64_t a, int64_t b,
                                            unsigned long long key) {
  int64_t lo = a, hi = b;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (uk[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < b && uk[lo] == key) ? lo : -1;
}

struct AdjView {
  int64_t *off;
  int32_t *deg;
  int32_t *cap;
  int32_t *adj;
  int64_t adj_cap;
};

__global__ void k_apply_delete(int64_t S, const int64_t *segstart,
                               const unsigned long long *uk, uint8_t *status,
                               AdjView A, int32_t *long_list,
                               unsigned long long *long_cnt) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t s = wave; s < S; s += nwaves) {
    const int64_t a = segstart[s], b = segstart[s + 1];
    bool has_del = false;
    for (int64_t i = a; i < b && !has_del; i += kWave) {
      const bool d = i + lane < b && (uk[i + lane] & 1ull) == 0;
      has_del = __ballot(d) != 0;
    }
    if (!has_del) continue;
    const uint32_t row = (uint32_t)(uk[a] >> 32);
    const int64_t off = A.off[row];
    const int32_t deg = A.deg[row];
    if (deg >= kLongApply) {  // k_apply_delete_long
      if (lane == 0) long_list[atomicAdd(long_cnt, 1ull)] = (int32_t)s;
      continue;
    }
    int32_t w = 0;
    for (int32_t t = 0; t < deg; t += kWave) {
      const int32_t idx = t + lane;
      int32_t x = -1;
      bool keep = false;
      if (idx < deg) {
        x = A.adj[off + idx];
        const int64_t j = find_key(uk, a, b,
                                   (unsigned long long)row << 32 |
                                       (unsigned long long)(uint32_t)x << 1);
        if (j >= 0) status[j] |= kApplied;
        keep = j < 0;
      }
      const uint64_t mask = __ballot(keep);
      if (keep) A.adj[off + w + __popcll(mask & lanemask_lt())] = x;
      w += __popcll(mask);
    }
    if (lane == 0) A.deg[row] = w;
  }
}

// Lookup of `key` among n sorted keys in LDS; index or -1.
__device__ __forceinline__ int32_t find_key_lds(const unsigned long long *keys,
                                                int32_t n, unsigned long long key) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (keys[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && keys[lo] == key) ? lo : -1;
}

// Exclusive prefix of x over the workgroup (at most 1024 threads, whole
// wavefronts); *total = sum.  Starts with a barrier, so the LDS it uses can
// be reused by the next call.
__device__ __forceinline__ int32_t block_scan_excl(int32_t x, int32_t *lds,
                                                   int32_t *total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int32_t incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  __syncthreads();
  if (lane == kWave - 1) lds[w] = incl;
  __syncthreads();
  int32_t before = 0, sum = 0;
  for (int i = 0; i < nw; ++i) {
    const int32_t t = lds[i];
    before += i < w ? t : 0;
    sum += t;
  }
  *total = sum;
  return before + incl - x;
}

// Deletions on the rows k_apply_delete deferred: one workgroup per row,
// row entries looked up among the segment's keys (staged in LDS when they
// fit) and the survivors compacted in place in order.
__global__ void __launch_bounds__(kLongBlock) k_apply_delete_long(
    const int32_t *long_list, const unsigned long long *long_cnt,
    const int64_t *segstart, const unsigned long long *uk, uint8_t *status,
    AdjView A) {
  __shared__ unsigned long long keys[kKeyLds];
  __shared__ int32_t part[kLongBlock / kWave];
  const unsigned long long cnt = *long_cnt;
  for (unsigned long long j = blockIdx.x; j < cnt; j += gridDim.x) {
    const int64_t sg = long_list[j];
    const int64_t a = segstart[sg], b = segstart[sg + 1];
    const int64_t nk = b - a;
    const bool staged = nk <= kKeyLds;
    __syncthreads();  // the previous row's readers of `keys` are done
    if (staged)
      for (int64_t i = threadIdx.x; i < nk; i += blockDim.x) keys[i] = uk[a + i];
    __syncthreads();
    const uint32_t row = (uint32_t)(uk[a] >> 32);
    const int64_t off = A.off[row];
    const int32_t deg = A.deg[row];
    // each thread takes kDelPer consecutive entries per round, so a row of
    // 100,000 entries takes 13 rounds (each a memory round trip and a
    // block scan) instead of 100
    int32_t w = 0;
    const int32_t step = (int32_t)blockDim.x * kDelPer;
    for (int32_t t = 0; t < deg; t += step) {
      const int32_t first = t + (int32_t)threadIdx.x * kDelPer;
      int32_t xs[kDelPer];
#pragma unroll
      for (int i = 0; i < kDelPer; ++i) xs[i] = first + i < deg ? A.adj[off + first + i] : -1;
      uint32_t keepm = 0;
      int32_t cnt = 0;
#pragma unroll
      for (int i = 0; i < kDelPer; ++i) {
        if (first + i >= deg) break;
        const unsigned long long key =
            (unsigned long long)row << 32 | (unsigned long long)(uint32_t)xs[i] << 1;
        int64_t k = -1;
        if (staged) {
          const int32_t q = find_key_lds(keys, (int32_t)nk, key);
          k = q >= 0 ? a + q : -1;
        } else {
          k = find_key(uk, a, b, key);
        }
        if (k >= 0) {
          status[k] |= kApplied;
        } else {
          keepm |= 1u << i;
          ++cnt;
        }
      }
      int32_t total = 0;
      // every entry of this round is read before the scan's barriers; the
      // survivors land, in order, at or below their own positions
      int32_t pos = w + block_scan_excl(cnt, part, &total);
#pragma unroll
      for (int i = 0; i < kDelPer; ++i)
        if (keepm & (1u << i)) A.adj[off + pos++] = xs[i];
      w += total;
    }
    if (threadIdx.x == 0) A.deg[row] = w;
  }
}

__global__ void k_apply_insert(int64_t S, const int64_t *segstart,
                               const unsigned long long *uk, uint8_t *status,
                               uint8_t *done, AdjView A,
                               unsigned long long *used, int *overflow) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t s = wave; s < S; s += nwaves) {
    if (done[s]) continue;
    const int64_t a = segstart[s], b = segstart[s + 1];
    const uint32_t row = (uint32_t)(uk[a] >> 32);
    int64_t off = A.off[row];
    const int32_t deg = A.deg[row];
    // drop insertions of edges already present
    int n_ins = 0;
    for (int64_t i = a; i < b; i += kWave)
      n_ins += __popcll(__ballot(i + lane < b && (uk[i + lane] & 1ull)));
    if (n_ins == 0) {
      if (lane == 0) done[s] = 1;
      continue;
    }
    // kDelPer row entries per lane in flight at once: the longest row
    // (a hub's in-row of ~10^5 entries) bounds the kernel
    for (int32_t t = 0; t < deg; t += kWave * kDelPer) {
      int32_t xs[kDelPer];
#pragma unroll
      for (int i = 0; i < kDelPer; ++i) {
        const int32_t idx = t + i * kWave + lane;
        xs[i] = idx < deg ? A.adj[off + idx] : -1;
      }
#pragma unroll
      for (int i = 0; i < kDelPer; ++i) {
        if (t + i * kWave + lane >= deg) continue;
        const int64_t j = find_key(uk, a, b,
                                   (unsigned long long)row << 32 |
                                       (unsigned long long)(uint32_t)xs[i] << 1 | 1ull);
        if (j >= 0) status[j] |= kExists;
      }
    }
    int k_new = 0;
    for (int64_t i = a; i < b; i += kWave) {
      const int64_t e = i + lane;
      const bool c = e < b && (uk[e] & 1ull) && !(status[e] & kExists);
      k_new += __popcll(__ballot(c));
    }
    if (k_new == 0) {
      if (lane == 0) done[s] = 1;
      continue;
    }
    const int32_t cap = A.cap[row];
    if (deg + k_new > cap) {
      int64_t need = 2 * ((int64_t)deg + k_new);
      if (need < 8) need = 8;
      need = (need + 3) & ~3ll;
      unsigned long long p = 0;
      if (lane == 0)
        p = __hip_atomic_fetch_add(used, (unsigned long long)need,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      p = __shfl(p, 0);
      if ((int64_t)p + need > A.adj_cap) {
        if (lane == 0) atomicOr(overflow, 1);
        continue;  // left pending; the host grows the array and re-runs
      }
      // the row moves to its new slot with kDelPer loads in flight per lane
      for (int32_t t = lane; t < deg; t += kWave * kDelPer) {
        int32_t x[kDelPer];
#pragma unroll
        for (int i = 0; i < kDelPer; ++i)
          x[i] = t + i * kWave < deg ? A.adj[off + t + i * kWave] : 0;
#pragma unroll
        for (int i = 0; i < kDelPer; ++i)
          if (t + i * kWave < deg) A.adj[p + t + i * kWave] = x[i];
      }
      off = (int64_t)p;
      if (lane == 0) {
        A.off[row] = off;
        A.cap[row] = (int32_t)need;
      }
    }
    int32_t w = deg;
    for (int64_t i = a; i < b; i += kWave) {
      const int64_t e = i + lane;
      const bool c = e < b && (uk[e] & 1ull) && !(status[e] & kExists);
      const uint64_t mask = __ballot(c);
      if (c) {
        A.adj[off + w + __popcll(mask & lanemask_lt())] =
            (int32_t)((uk[e] >> 1) & 0x7FFFFFFFull);
        status[e] |= kApplied;
      }
      w += __popcll(mask);
    }
    if (lane == 0) {
      A.deg[row] = w;
      done[s] = 1;
    }
  }
}

__global__ void k_count_applied(int64_t U, const unsigned long long *uk,
                                const uint8_t *status,
                                unsigned long long *del_cnt,
                                unsigned long long *ins_cnt) {
  unsigned long long d = 0, in = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < U;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (status[i] & kApplied) {
      if (uk[i] & 1ull)
        ++in;
      else
        ++d;
    }
  }
  d = wave_sum(d);
  in = wave_sum(in);
  if (lane_id() == 0) {
    if (d) atomicAdd(del_cnt, d);
    if (in) atomicAdd(ins_cnt, in);
  }
}

// Marks (G^{t-1} U G^t).out(u) for every source u with a real change.
template <typename T>
__global__ void k_mark_sources(int64_t S, const int64_t *segstart,
                               const unsigned long long *uk,
                               const uint8_t *status, AdjView out,
                               const T *R, T *C, uint32_t *flags,
                               uint32_t *gflags, Ctl *ctl, int32_t *long_list) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  auto mark = [&](bool act, int32_t v) {
    if (act) mark_plain(flags, gflags, v);
  };
  for (int64_t s = wave; s < S; s += nwaves) {
    const int64_t a = segstart[s], b = segstart[s + 1];
    bool any = false;
    for (int64_t i = a; i < b && !any; i += kWave)
      any = __ballot(i + lane < b && (status[i + lane] & kApplied)) != 0;
    if (!any) continue;
    const int32_t u = (int32_t)(uk[a] >> 32);
    const int64_t off = out.off[u];
    const int32_t deg = out.deg[u];
    if (lane == 0) C[u] = (T)((double)R[u] / (double)(deg + 1));
    // u itself (implicit self-loop), then its current out-row (long rows:
    // k_mark_long)
    const bool defer = deg >= kLongApply;
    if (defer && lane == 0) long_list[atomicAdd(&ctl->nlong_mark, 1ull)] = u;
    const int32_t rdeg = defer ? 0 : deg;
    for (int32_t t = -1; t < rdeg; t += kWave) {
      const int32_t idx = t + lane;
      const bool act = idx < rdeg;
      mark(act, act ? (idx < 0 ? u : out.adj[off + idx]) : -1);
    }
    // targets of the deleted edges of u (they were out-neighbours in G^{t-1})
    for (int64_t i = a; i < b; i += kWave) {
      const int64_t e = i + lane;
      const bool act = e < b && !(uk[e] & 1ull) && (status[e] & kApplied);
      mark(act, act ? (int32_t)((uk[e] >> 1) & 0x7FFFFFFFull) : -1);
    }
  }
}

// Out-rows deferred by k_mark_sources: one workgroup per row (rows strided
// over the workgroups), its threads striding over the row.  Having every
// thread of the grid walk every row in turn left most threads idle and made
// the launch a chain of per-row load latencies (1.1 ms per 1e-3 batch on
// the 2^22 R-MAT).
__global__ void k_mark_long(const int32_t *long_list, AdjView out, uint32_t *flags,
                            uint32_t *gflags, const Ctl *ctl) {
  const unsigned long long cnt = ctl->nlong_mark;
  for (unsigned long long j = blockIdx.x; j < cnt; j += gridDim.x) {
    const int32_t u = long_list[j];
    const int64_t off = out.off[u];
    const int32_t deg = out.deg[u];
    // kDelPer entries per thread in flight at once: a row of 100,000
    // entries is a few rounds of loads, not one per 1024 entries
    for (int32_t t = threadIdx.x; t < deg; t += (int32_t)blockDim.x * kDelPer) {
      int32_t v[kDelPer];
#pragma unroll
      for (int i = 0; i < kDelPer; ++i) {
        const int32_t idx = t + i * (int32_t)blockDim.x;
        v[i] = idx < deg ? out.adj[off + idx] : -1;
      }
#pragma unroll
      for (int i = 0; i < kDelPer; ++i)
        if (v[i] >= 0) mark_plain(flags, gflags, v[i]);
    }
  }
}

// Marked vertices (affected flag set) into ctl->marked: one atomic per
// workgroup.
__global__ void __launch_bounds__(256) k_count_marked(const uint32_t *flags, int64_t words,
                                                      Ctl *ctl) {
  __shared__ unsigned long long part[256 / kWave];
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    c += __popc(flags[i] & 0x01010101u);
  c = wave_sum(c);
  if (lane_id() == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += part[w];
    if (t) atomicAdd((unsigned long long *)&ctl->marked, t);
  }
}

}  // namespace

// Sorts and de-duplicates the batch for one direction.  Outputs (in scratch
// slots base..base+2): uk[U] keys, segstart[S+1], status[U] zeroed.
static int prepare_direction(dfpr_graph *g, int dir, int64_t nd,
                             const int32_t *ds, const int32_t *dd, int64_t ni,
                             const int32_t *is, const int32_t *id, int base,
                             unsigned long long **uk_out, int64_t **seg_out,
                             uint8_t **status_out, int64_t *U_out,
                             int64_t *S_out) {
  hipStream_t s = g->stream;
  const int cu = g->cu_count;
  const int64_t m = nd + ni;
  int rc;
  void *ka, *kb, *hr, *sr, *tmp, *uk, *seg, *st;
  if ((rc = scratch_get(g, 0, m * 8, &ka))) return rc;
  if ((rc = scratch_get(g, 1, m * 8, &kb))) return rc;
  if ((rc = scratch_get(g, 2, m * 8, &hr))) return rc;
  if ((rc = scratch_get(g, 3, m * 8, &sr))) return rc;
  k_batch_keys<<<grid_for(m, cu), 256, 0, s>>>(dir, nd, ds, dd, ni, is, id, g->ext2int,
                                               (unsigned long long *)ka);
  size_t tb = 0;
  DFPR_HIP(rocprim::radix_sort_keys(nullptr, tb, (unsigned long long *)ka,
                                    (unsigned long long *)kb, (size_t)m, 0, 64, s));
  if ((rc = scratch_get(g, 7, tb, &tmp))) return rc;
  DFPR_HIP(rocprim::radix_sort_keys(tmp, tb, (unsigned long long *)ka,
                                    (unsigned long long *)kb, (size_t)m, 0, 64, s));
  k_batch_heads<<<grid_for(m, cu), 256, 0, s>>>(m, (unsigned long long *)kb,
                                                (int64_t *)hr, (int64_t *)sr);
  // counts: last head/seg flag + exclusive scans
  int64_t lastf[2] = {0, 0};
  DFPR_HIP(hipMemcpyAsync(&lastf[0], (int64_t *)hr + (m - 1), 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipMemcpyAsync(&lastf[1], (int64_t *)sr + (m - 1), 8, hipMemcpyDeviceToHost, s));
  for (int q = 0; q < 2; ++q) {
    int64_t *arr = q == 0 ? (int64_t *)hr : (int64_t *)sr;
    tb = 0;
    DFPR_HIP(rocprim::exclusive_scan(nullptr, tb, arr, arr, (int64_t)0, (size_t)m,
                                     rocprim::plus<int64_t>(), s));
    if ((rc = scratch_get(g, 7, tb, &tmp))) return rc;
    DFPR_HIP(rocprim::exclusive_scan(tmp, tb, arr, arr, (int64_t)0, (size_t)m,
                                     rocprim::plus<int64_t>(), s));
  }
  int64_t lastr[2] = {0, 0};
  DFPR_HIP(hipMemcpyAsync(&lastr[0], (int64_t *)hr + (m - 1), 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipMemcpyAsync(&lastr[1], (int64_t *)sr + (m - 1), 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const int64_t U = lastr[0] + lastf[0];
  const int64_t S = lastr[1] + lastf[1];
  if ((rc = scratch_get(g, base, (U > 0 ? U : 1) * 8, &uk))) return rc;
  if ((rc = scratch_get(g, base + 1, (S + 1) * 8, &seg))) return rc;
  if ((rc = scratch_get(g, base + 2, (U > 0 ? U : 1) + (S + 1), &st))) return rc;
  k_batch_compact<<<grid_for(m, cu), 256, 0, s>>>(m, (unsigned long long *)kb,
                                                  (int64_t *)hr, (int64_t *)sr,
                                                  (unsigned long long *)uk,
                                                  (int64_t *)seg);
  k_set_i64<<<1, 64, 0, s>>>((int64_t *)seg + S, U);
  DFPR_HIP(hipMemsetAsync(st, 0, (U > 0 ? U : 1) + (S + 1), s));
  DFPR_HIP(hipGetLastError());
  *uk_out = (unsigned long long *)uk;
  *seg_out = (int64_t *)seg;
  *status_out = (uint8_t *)st;
  *U_out = U;
  *S_out = S;
  return DFPR_OK;
}

static int grow_adj(dfpr_graph *g, int dir) {
  Adj &A = dir == 0 ? g->out : g->in;
  hipStream_t s = g->stream;
  unsigned long long used = 0;
  DFPR_HIP(hipMemcpyAsync(&used, &g->ctl->adj_used[dir], 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  int64_t want = A.adj_cap * 2;
  if ((int64_t)used + A.adj_cap / 2 > want) want = (int64_t)used + A.adj_cap / 2;
  want = (want + 3) & ~3ll;
  int32_t *na = nullptr;
  DFPR_HIP(hipMalloc(&na, sizeof(int32_t) * want));
  DFPR_HIP(hipMemcpyAsync(na, A.adj, sizeof(int32_t) * A.adj_cap,
                          hipMemcpyDeviceToDevice, s));
  DFPR_HIP(hipStreamSynchronize(s));
  DFPR_HIP(hipFree(A.adj));
  A.adj = na;
  A.adj_cap = want;
  return DFPR_OK;
}

int apply_batch(dfpr_graph *g, int64_t nd, const int32_t *ds,
                const int32_t *dd, int64_t ni, const int32_t *is,
                const int32_t *id, int64_t *applied_del,
                int64_t *applied_ins) {
  hipStream_t s = g->stream;
  const int cu = g->cu_count;
  const int64_t m = nd + ni;
  DFPR_HIP(hipMemsetAsync(&g->ctl->invalid, 0, sizeof(int) * 2, s));
  DFPR_HIP(hipMemsetAsync(&g->ctl->ins_applied, 0, sizeof(unsigned long long) * 4, s));
  if (m == 0) {
    if (applied_del) *applied_del = 0;
    if (applied_ins) *applied_ins = 0;
    return DFPR_OK;
  }
  k_validate2<<<grid_for(m, cu), 256, 0, s>>>(nd, ds, dd, ni, is, id, g->n, g->ctl);
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  if (g->h_ctl->invalid) return fail(DFPR_EINVAL, "batch id outside [0, n)");

  unsigned long long *uk[2];
  int64_t *seg[2];
  uint8_t *st[2];
  int64_t U[2], S[2];
  // in direction first; slot 14 holds each direction's list of long rows
  // with deletions in turn, slot 0 (free once both directions are
  // prepared) the marking's list of long out-rows
  for (int dir = 1; dir >= 0; --dir) {
    const int base = 8 + 3 * dir;
    int rc = prepare_direction(g, dir, nd, ds, dd, ni, is, id, base, &uk[dir],
                               &seg[dir], &st[dir], &U[dir], &S[dir]);
    if (rc) return rc;
    Adj &A = dir == 0 ? g->out : g->in;
    if (S[dir] == 0) continue;
    uint8_t *done = st[dir] + (U[dir] > 0 ? U[dir] : 1);
    const int blocks = grid_for(S[dir] * 64, cu);
    AdjView v{A.off, A.deg, A.cap, A.adj, A.adj_cap};
    void *ll = nullptr;
    int rc1 = scratch_get(g, 14, (size_t)S[dir] * 4, &ll);
    if (rc1) return rc1;
    DFPR_HIP(hipMemsetAsync(&g->ctl->nlong_del, 0, sizeof(unsigned long long), s));
    k_apply_delete<<<blocks, 256, 0, s>>>(S[dir], seg[dir], uk[dir], st[dir], v,
                                          (int32_t *)ll, &g->ctl->nlong_del);
    DFPR_HIP(hipGetLastError());
    k_apply_delete_long<<<cu > 0 ? cu : 1, kLongBlock, 0, s>>>(
        (const int32_t *)ll, &g->ctl->nlong_del, seg[dir], uk[dir], st[dir], v);
    DFPR_HIP(hipGetLastError());
    for (int attempt = 0; attempt < 16; ++attempt) {
      AdjView w{A.off, A.deg, A.cap, A.adj, A.adj_cap};
      k_apply_insert<<<blocks, 256, 0, s>>>(S[dir], seg[dir], uk[dir], st[dir],
                                            done, w, &g->ctl->adj_used[dir],
                                            &g->ctl->overflow);
      DFPR_HIP(hipGetLastError());
      int ovf = 0;
      DFPR_HIP(hipMemcpyAsync(&ovf, &g->ctl->overflow, sizeof(int), hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipStreamSynchronize(s));
      if (!ovf) break;
      DFPR_HIP(hipMemsetAsync(&g->ctl->overflow, 0, sizeof(int), s));
      int rc2 = grow_adj(g, dir);
      if (rc2) return rc2;
      if (attempt == 15) return fail(DFPR_ENOMEM, "adjacency growth did not converge");
    }
    k_count_applied<<<grid_for(U[dir], cu) < 64 ? grid_for(U[dir], cu) : 64, 256, 0, s>>>(
        U[dir], uk[dir], st[dir],
        dir == 0 ? &g->ctl->del_applied : &g->ctl->del_applied_in,
        dir == 0 ? &g->ctl->ins_applied : &g->ctl->ins_applied_in);
    DFPR_HIP(hipGetLastError());
  }
  // marking over the out-direction segments
  if (S[0] > 0) {
    const int blocks = grid_for(S[0] * 64, cu);
    AdjView o{g->out.off, g->out.deg, g->out.cap, g->out.adj, g->out.adj_cap};
    void *ml = nullptr;
    int rc1 = scratch_get(g, 0, (size_t)S[0] * 4, &ml);
    if (rc1) return rc1;
    DFPR_HIP(hipMemsetAsync(&g->ctl->nlong_mark, 0, sizeof(unsigned long long), s));
    if (g->elem == 8)
      k_mark_sources<double><<<blocks, 256, 0, s>>>(
          S[0], seg[0], uk[0], st[0], o, (const double *)g->R[g->cur],
          (double *)g->C[g->cur], g->flags, g->gflags, g->ctl, (int32_t *)ml);
    else
      k_mark_sources<float><<<blocks, 256, 0, s>>>(
          S[0], seg[0], uk[0], st[0], o, (const float *)g->R[g->cur],
          (float *)g->C[g->cur], g->flags, g->gflags, g->ctl, (int32_t *)ml);
    DFPR_HIP(hipGetLastError());
    k_mark_long<<<cu > 0 ? 4 * cu : 1, 256, 0, s>>>((const int32_t *)ml, o, g->flags,
                                                   g->gflags, g->ctl);
    DFPR_HIP(hipGetLastError());
    // the count covers every batch applied since the last update
    const int64_t words = ((int64_t)g->n + 3) / 4;
    DFPR_HIP(hipMemsetAsync(&g->ctl->marked, 0, sizeof(long long), s));
    // one workgroup per CU: each adds its count with one atomic on one word
    k_count_marked<<<cu > 0 ? cu : 1, 256, 0, s>>>(g->flags, words, g->ctl);
    DFPR_HIP(hipGetLastError());
  }
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const Ctl &h = *g->h_ctl;
  if (h.del_applied != h.del_applied_in || h.ins_applied != h.ins_applied_in)
    return fail(DFPR_EHIP, "in/out adjacency disagree after the batch");
  g->m += (int64_t)h.ins_applied - (int64_t)h.del_applied;
  g->pending_marks = (int64_t)h.marked;
  // piece arrays follow adjacency growth here, so updates allocate nothing
  if (int rc = ensure_split(g)) return rc;
  if (applied_del) *applied_del = (int64_t)h.del_applied;
  if (applied_ins) *applied_ins = (int64_t)h.ins_applied;
  return DFPR_OK;
}

}  // namespace dfpr
