// Rank iteration kernels: the gather of Eq. 1, frontier expansion and
// convergence (Section 4; Algorithms 1 and 2), plus static / naive-dynamic
// PageRank (Algorithm 3; Section 3.5.1) and small helpers.
//
// Work units:
//   step   up to 256 vertices, four per lane.  Their in-rows are flattened
//          into one edge range (prefix of the row lengths in LDS); every
//          round each lane loads kUnroll row entries and then as many
//          contributions C[u] = R[u] / (out-degree(u) + 1), all independent,
//          and adds them to the owning row's LDS accumulator.  The implicit
//          self-loop adds C[v].
//   piece  up to kPiece consecutive in-edges of one long row (in-degree at
//          or above split_min_degree), summed by a whole wavefront in
//          registers; the wavefront completing the row's last piece adds
//          the partial sums in piece order and finishes the vertex.
//   finish r = (1 - alpha)/n + alpha * sum, dr = |r - R[v]|; when dr exceeds
//          the frontier tolerance every out-neighbour is marked affected
//          (once per vertex and update: flag bit kEX).
//
// Scheduling:
//   k_df_async   one persistent launch (lock-free scheme, Algorithm 2).  A
//                64-bit word holds the sweep index, a cursor into the group
//                worklist and the number of claims in flight; wavefronts
//                claim worklist entries with fetch_add (256-vertex groups,
//                whose affected vertices they recompute in place, and the
//                pieces of affected long rows).  A sweep ends the update
//                when no claim is held and no claim completed during that
//                sweep saw a rank change above the iteration tolerance or
//                affected a new vertex (change_sweep watermark).  No grid
//                barrier anywhere: sweeps overlap.
//   k_sync_iter  one launch per iteration reading R/C and writing the other
//                buffer (Algorithm 1): wavefronts claim the iteration's
//                pieces, then its edge-balanced steps; k_sync_finish ends
//                the loop on the device so the host polls every few
//                iterations.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "dfpr_common.h"

namespace dfpr {

enum Mode { kAsync = 0, kSyncDF = 1, kAll = 2 };

template <typename T>
struct RankArgs {
  int32_t n;
  const int64_t *in_off;
  const int32_t *in_deg;
  const int32_t *in_adj;
  const int64_t *out_off;
  const int32_t *out_deg;
  const int32_t *out_adj;
  const T *Rr;
  const T *Cr;
  T *Rw;
  T *Cw;
  uint32_t *flags;
  int32_t *wl;
  uint32_t *gflags;
  int32_t *gwl;
  Ctl *ctl;
  double alpha, base, tol, ftol;
  double wtol;  // lock-free scheme: a claim with a rank change above wtol
                // (or a newly affected vertex) forces another sweep
  int32_t split_min, kahan_min, chunk, max_iters;
  unsigned long long timeout_ticks;
  unsigned long long *sync_max;
  unsigned long long *sync_grab;
  unsigned long long *sync_len;  // per iteration: steps | pieces << 32
  int32_t *lrow;                 // rows gathered in pieces (Split)
  int32_t *lpre;
  int32_t *prow;
  double *ppart;
  int32_t *lcnt;
  int32_t *ptag;                 // lock-free: launch that wrote ppart[p]
  int32_t epoch;                 // lock-free: this launch
  int32_t *xrow;                 // deferred long out-rows (Split)
  const int32_t *faults;         // injected faults per workgroup (or null)
  int32_t nfaults;
  int32_t fault_stops;           // some entry of faults stops its workgroups
  uint32_t ticks_per_us;         // wall-clock ticks per microsecond
  int32_t group_stripes;         // lock-free: interleaved runs of the group
                                 // worklist (list_groups)
};

// Injected fault of the calling workgroup, taken after each completed claim
// (fault simulation: a delay, or a crash-stop at a claim boundary).
// faults[blockIdx.x % nfaults]: 0 none, > 0 sleep that many microseconds,
// < 0 stop claiming.  Returns true when the workgroup stops.
template <typename T>
__device__ __forceinline__ bool injected_fault(const RankArgs<T> &A) {
  if (A.nfaults <= 0) return false;
  const int32_t f = A.faults[blockIdx.x % (unsigned)A.nfaults];
  if (f < 0) return true;
  if (f > 0) {
    const unsigned long long t0 = wall_clock64();
    const unsigned long long d = (unsigned long long)f * A.ticks_per_us;
    while (wall_clock64() - t0 < d) __builtin_amdgcn_s_sleep(64);
  }
  return false;
}

struct Counters {
  unsigned long long vertices = 0, edges = 0, out_scanned = 0;
};

template <typename T, bool COH>
__device__ __forceinline__ T ldc(const T *C, int32_t u) {
  if constexpr (COH)
    return load_agent(C + u);
  else
    return C[u];
}

// One step of a wavefront covers kRows = 256 vertices, four per lane
// (row r = k * 64 + lane holds the lane's k-th vertex).
constexpr int kQ = 4;
constexpr int kRows = kQ * kWave;
// independent row entries (and then contributions) each lane loads per
// round; with the rounds pipelined, 6 measured best on the 2^22 R-MAT (4, 5
// and 8 were 1-3% slower)
constexpr int kUnroll = 6;

// Edge positions of a step covered by the owner bitmap (steps of the
// barrier-based scheme stay below 16384 plus one row under the piece
// threshold; longer ones fall back to a binary search).
constexpr int32_t kBitCap = 20480;
constexpr int32_t kBitWords = kBitCap / 32;

struct BitWord {
  uint32_t bits;  // bit b: a non-empty row starts at edge position 32 w + b
  uint32_t cnt;   // rows starting before word w
};

// Per-wavefront LDS: the flattened edge list of the current step (prefix of
// the row lengths and the row starts), the owner bitmap, and per-row
// accumulators.

template <typename T>
struct WaveLds {
  int32_t pre[kRows + 1];
  int32_t vbuf[kRows];  // lock-free scheme: affected vertices gathered from
                        // the claimed group parts, processed 256 at a time
  BitWord bm[kBitWords];  // owner bitmap of the step's edge positions
  int64_t off[kRows];
  double acc[kRows];  // fp64 sums (fp64 ranks; fp32 rows at/above the
                      // compensation threshold)
  float accf[sizeof(T) == 4 ? kRows : 1];  // fp32 sums (fp32 rows below it)
};

// The calling wavefront's WaveLds, from the launch's dynamic LDS (one per
// wavefront of the workgroup: launch with lds_bytes<T>(block_size)).
template <typename T>
__device__ __forceinline__ WaveLds<T> &wave_lds() {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  return reinterpret_cast<WaveLds<T> *>(dyn_lds)[threadIdx.x / kWave];
}

template <typename T>
constexpr size_t lds_bytes(int block_size) {
  return sizeof(WaveLds<T>) * (size_t)(block_size / kWave);
}

// s_waitcnt vmcnt(0) in the gfx9 encoding (expcnt and lgkmcnt at their
// maxima): waits until the wavefront's global loads and stores complete.
constexpr int kWaitVmcnt0 = 0x0F70;

// Orders the calling wavefront's earlier global stores before its later
// global accesses as every other wavefront of the device sees them, by
// waiting until the stores have completed.  This suffices wherever the
// values exchanged between wavefronts inside a launch are written and read
// with device-scope atomic accesses (store_agent, load_agent, atomic RMWs):
// those go to the device's coherence point past the XCD's L2, so a
// completed store is visible to any later such load.  An agent-scope
// release fence would also write back the XCD's L2 (buffer_wbl2) and an
// acquire invalidate it (buffer_inv), which stalls every wavefront of the
// XCD: per piece of a long row that had cost the barrier-based update on
// the 2^22 R-MAT 31.3 against 21.9 ms, and per lock-free claim the grid
// update 4.2 against 3.1 ms.
__device__ __forceinline__ void stores_complete() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no compiler reordering across
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Orders LDS traffic of the lanes of one wavefront (no cross-wave sync).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// Largest row r with pre[r] <= e (pre non-decreasing, pre[kRows] > e).
__device__ __forceinline__ int find_owner(const int32_t *pre, int32_t e) {
  int lo = 0, hi = kRows;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Publishes the 256 rows (off, len) of the step as one flattened range in
// LDS; returns its total length.  Clears the accumulators.
template <typename T>
__device__ __forceinline__ int32_t flatten_rows(WaveLds<T> &L, const int64_t *off,
                                               const int32_t *len) {
  const int lane = lane_id();
  wave_lds_fence();
  int32_t base = 0;
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int32_t incl = wave_incl_scan(len[k]);
    const int r = k * kWave + lane;
    L.pre[r] = base + incl - len[k];
    L.off[r] = off[k];
    L.acc[r] = 0.0;
    if constexpr (sizeof(T) == 4) L.accf[r] = 0.f;
    base += __shfl(incl, kWave - 1);
  }
  if (lane == 0) L.pre[kRows] = base;
  wave_lds_fence();
  return base;
}

// Publishes the non-empty rows among the step's 256 (off, len), in order,
// as one flattened range in LDS: pre[k] and off[k] for the k-th non-empty
// row, pre[k] = total beyond them; rank[q] (per lane) is the position of the
// lane's q-th row among them, or -1.  Clears the accumulators.  When the
// range fits kBitCap it also builds the owner bitmap: the row owning edge e
// is then cnt[e / 32] + (set bits of bits[e / 32] at or below e % 32) - 1,
// two LDS reads where a binary search over 256 rows took eight dependent
// ones (about a fifth of a barrier-based iteration on the 2^22 R-MAT).
template <typename T>
__device__ __forceinline__ int32_t flatten_nonempty(WaveLds<T> &L, const int64_t *off,
                                                   const int32_t *len, int32_t *rank) {
  const int lane = lane_id();
  wave_lds_fence();
  int32_t base = 0, nbase = 0;
  int32_t start[kQ];
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int32_t incl = wave_incl_scan(len[k]);
    const bool ne = len[k] > 0;
    const int32_t nincl = wave_incl_scan(ne ? 1 : 0);
    start[k] = base + incl - len[k];
    rank[k] = ne ? nbase + nincl - 1 : -1;
    if (ne) {
      L.pre[rank[k]] = start[k];
      L.off[rank[k]] = off[k];
    }
    base += __shfl(incl, kWave - 1);
    nbase += __shfl(nincl, kWave - 1);
  }
  const int32_t total = base, nnz = nbase;
  for (int32_t r = nnz + lane; r <= kRows; r += kWave) L.pre[r] = total;
  for (int32_t r = lane; r < nnz; r += kWave) {
    L.acc[r] = 0.0;
    if constexpr (sizeof(T) == 4) L.accf[r] = 0.f;
  }
  if (total <= kBitCap) {
    const int32_t words = (total + 31) >> 5;
    for (int32_t w = lane; w < words; w += kWave) L.bm[w].bits = 0u;
    wave_lds_fence();
#pragma unroll
    for (int k = 0; k < kQ; ++k)
      if (rank[k] >= 0) atomicOr(&L.bm[start[k] >> 5].bits, 1u << (start[k] & 31));
    wave_lds_fence();
    // counts before each word: each lane a run of consecutive words
    const int32_t per = (words + kWave - 1) / kWave;
    const int32_t w0 = lane * per;
    const int32_t w1 = w0 + per < words ? w0 + per : words;
    int32_t mine = 0;
    for (int32_t w = w0; w < w1; ++w) mine += __popc(L.bm[w].bits);
    int32_t run = wave_incl_scan(mine) - mine;
    for (int32_t w = w0; w < w1; ++w) {
      L.bm[w].cnt = (uint32_t)run;
      run += __popc(L.bm[w].bits);
    }
  }
  wave_lds_fence();
  return total;
}

// Sums over the in-rows of the step's 256 vertices, edge-parallel: every
// round loads kUnroll x 64 row entries, then as many contributions, all
// independent, and adds them to the owners' LDS accumulators.  The rounds
// are software-pipelined: the owners and row entries of round k + 1 are
// found and loaded while the contributions of round k are in flight, so a
// round waits for one memory latency instead of two in a row.
template <typename T, bool COH>
__device__ __forceinline__ void gather_flat(const RankArgs<T> &A, WaveLds<T> &L,
                                            const int64_t *off,
                                            const int32_t *deg, double *sum) {
  const int lane = lane_id();
  // barrier-based scheme, fp32 ranks: rows of at least kahan_min in-edges
  // sum in fp64, shorter ones in fp32; the choice rides in bit 62 of the
  // row's offset in LDS (read there anyway) and in bit 8 of the owner, so
  // no edge reads the row's length again
  constexpr bool kMixed = sizeof(T) == 4 && !COH;
  constexpr int64_t kWideBit = 1ll << 62;
  int32_t rank[kQ];
  int32_t total;
  if constexpr (kMixed) {
    int64_t offw[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) offw[k] = off[k] | (deg[k] >= A.kahan_min ? kWideBit : 0);
    total = flatten_nonempty(L, offw, deg, rank);
  } else {
    total = flatten_nonempty(L, off, deg, rank);
  }
  const bool bitmap = total <= kBitCap;
  int own[kUnroll];
  int32_t idx[kUnroll];
  // Owners and row entries of the round starting at edge `base` (called
  // with total > 0).  Lanes past the end load the last edge again and get
  // owner -1: every load is unconditional, so no load sits in a branch that
  // the compiler's wait-count tracking must treat as possibly skipped
  // (which made it wait for all loads in flight before each contribution
  // load).
  auto fetch = [&](int32_t base) {
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int32_t e = base + j * kWave + lane;
      const int32_t ec = e < total ? e : total - 1;
      int o;
      if (bitmap) {
        const BitWord bw = L.bm[ec >> 5];
        o = (int)bw.cnt + __popc(bw.bits & ((2u << (ec & 31)) - 1u)) - 1;
      } else {
        o = find_owner(L.pre, ec);
      }
      const int64_t ro = L.off[o];
      if constexpr (kMixed) {
        idx[j] = A.in_adj[(ro & (kWideBit - 1)) + (ec - L.pre[o])];
        own[j] = e < total ? (o | (ro & kWideBit ? 0x100 : 0)) : -1;
      } else {
        idx[j] = A.in_adj[ro + (ec - L.pre[o])];
        own[j] = e < total ? o : -1;
      }
    }
  };
  if (total > 0) fetch(0);
  for (int32_t base = 0; base < total; base += kUnroll * kWave) {
    int cur[kUnroll];
    T c[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      cur[j] = own[j];
      c[j] = ldc<T, COH>(A.Cr, idx[j]);
    }
    const int32_t next = base + kUnroll * kWave;
    if (next < total) fetch(next);
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      if (cur[j] < 0) continue;
      if constexpr (!kMixed) {
        // lock-free scheme, fp32 ranks: every row in fp64 as well.  fp32
        // atomics add in arrival order, so a row's rounded sum can differ
        // by ulps from one sweep to the next, and a rank that keeps moving
        // by two ulps never meets the stopping rule
        atomicAdd(&L.acc[cur[j]], (double)c[j]);
      } else {
        const int r = cur[j] & 0xFF;
        if (cur[j] & 0x100)
          atomicAdd(&L.acc[r], (double)c[j]);
        else
          atomicAdd(&L.accf[r], (float)c[j]);
      }
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int r = rank[k];
    sum[k] = r >= 0 ? L.acc[r] : 0.0;
    if constexpr (sizeof(T) == 4) sum[k] += r >= 0 ? (double)L.accf[r] : 0.0;
  }
}

// Lock-free scheme: lists long row v (in-degree d >= split_min, just
// affected) with its pieces, and appends the pieces to the group worklist
// as entries -(p + 2).  One lane; rare (a row is listed once per update).
__device__ __forceinline__ void list_long_row(Ctl *ctl, int32_t *lrow, int32_t *lpre,
                                              int32_t *lcnt, int32_t *prow, int32_t *gwl,
                                              int32_t v, int32_t d) {
  const int32_t np = (d + kPiece - 1) / kPiece;
  const unsigned long long j = __hip_atomic_fetch_add(&ctl->nlong, 1ull, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long p0 = __hip_atomic_fetch_add(
      &ctl->npieces, (unsigned long long)np, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  store_agent(lrow + j, v);
  store_agent(lpre + j, (int32_t)p0);
  store_agent(lcnt + j, 0);
  for (int32_t k = 0; k < np; ++k) store_agent(prow + p0 + k, (int32_t)j);
  // the row's table is in place before a claim can read one of its pieces
  stores_complete();
  const unsigned long long pos = __hip_atomic_fetch_add(
      &ctl->gtail, (unsigned long long)np, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int32_t k = 0; k < np; ++k) store_agent(gwl + pos + k, -(int32_t)(p0 + k) - 2);
}

// Lock-free scheme: appends the parts of newly listed groups (lanes with
// `want`) to the worklist, with one atomic per wavefront.  All 64 lanes call
// it.  The group byte carries log2(parts) (k_group_parts).
__device__ __forceinline__ void append_group_parts(bool want, int32_t g,
                                                   const uint32_t *gflags, int32_t *gwl,
                                                   unsigned long long *gtail) {
  if (__ballot(want) == 0) return;
  uint32_t l = 0;
  if (want) l = (flag_byte(gflags, g, true) >> kGPartShift) & 7u;
  const int32_t cnt = want ? (1 << l) : 0;
  const int32_t incl = wave_incl_scan(cnt);
  const int32_t total = __shfl(incl, kWave - 1);
  unsigned long long base = 0;
  if (lane_id() == 0)
    base = __hip_atomic_fetch_add(gtail, (unsigned long long)total, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, 0);
  for (int32_t p = 0; p < cnt; ++p)
    store_agent(gwl + base + (incl - cnt) + p,
                g | (p << kEntryPartShift) | ((int32_t)l << kEntryLogShift));
}

// Synchronous scheme: marks w affected; true when w is newly affected.
__device__ __forceinline__ bool mark_vertex_sync(uint32_t *flags, int32_t w) {
  if (flag_byte(flags, w, false) & kVA) return false;
  return !(flag_set(flags, w, kVA) & kVA);
}

// Frontier expansion over the out-rows of the step's expanding vertices,
// flattened like the gather.  Synchronous scheme: out-neighbours get the
// affected flag (the worklist is rebuilt from the flags after the
// iteration).  Lock-free scheme: newly affected out-neighbours also get
// their group listed.
template <typename T, int MODE>
__device__ __forceinline__ void expand_flat(const RankArgs<T> &A, WaveLds<T> &L,
                                            const int64_t *oo,
                                            const int32_t *od,
                                            long long &newly) {
  const int lane = lane_id();
  const int32_t total = flatten_rows(L, oo, od);
  for (int32_t base = 0; base < total; base += kUnroll * kWave) {
    int32_t w[kUnroll];
    // unconditional loads (lanes past the end repeat the last entry and
    // are dropped), as in gather_flat
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int32_t e = base + j * kWave + lane;
      const int32_t ec = e < total ? e : total - 1;
      const int o = find_owner(L.pre, ec);
      const int32_t x = A.out_adj[L.off[o] + (ec - L.pre[o])];
      w[j] = e < total ? x : -1;
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      if constexpr (MODE == kAsync) {
        MarkOut o{false, false, -1};
        if (w[j] >= 0) o = mark_affected(A.flags, A.gflags, w[j]);
        newly += o.vnew ? 1 : 0;
        append_group_parts(o.gnew, o.g, A.gflags, A.gwl, &A.ctl->gtail);
        if (o.vnew) {
          // a long row joins the worklist as pieces (its group skips it)
          const int32_t dw = A.in_deg[w[j]];
          if (dw >= A.split_min)
            list_long_row(A.ctl, A.lrow, A.lpre, A.lcnt, A.prow, A.gwl, w[j], dw);
        }
      } else {
        if (w[j] >= 0 && mark_vertex_sync(A.flags, w[j])) ++newly;
      }
    }
  }
}

// Completes the step's vertices from their in-row sums (Eq. 1 with the
// implicit self-loop): new rank and contribution, the change test against
// the frontier tolerance, and the frontier expansion of vertices that moved
// (v[k] < 0: empty slot; deg[k]: in-edges the caller's gather summed).  All
// 64 lanes call it.
template <typename T, int MODE>
__device__ __forceinline__ void finish_rows(const RankArgs<T> &A, WaveLds<T> &L,
                                            const int32_t *v, const int32_t *deg,
                                            const double *sum, Counters &cnt,
                                            double &maxdr, long long &newly,
                                            bool &moved) {
  constexpr bool COH = MODE == kAsync;
  bool expand[kQ];
  int32_t od[kQ];
  int64_t oo[kQ];
  bool any_expand = false;
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    expand[k] = false;
    od[k] = 0;
    oo[k] = 0;
    if (v[k] < 0) continue;
    const int32_t x = v[k];
    // every per-vertex value in one round trip: the flag byte and the
    // out-row offset are needed only if the vertex moved
    const double selfc = (double)ldc<T, COH>(A.Cr, x);
    const T old = COH ? load_agent(A.Rr + x) : A.Rr[x];
    const int32_t d = A.out_deg[x];
    const uint32_t fb = MODE != kAll ? flag_byte(A.flags, x, COH) : 0u;
    const int64_t xo = MODE != kAll ? A.out_off[x] : 0;
    const double r = A.base + A.alpha * (sum[k] + selfc);
    const T rT = (T)r;
    const double dr = fabs((double)rT - (double)old);
    const T cT = (T)(r / (double)(d + 1));
    if constexpr (COH) {
      store_agent(A.Rw + x, rT);
      store_agent(A.Cw + x, cT);
    } else {
      A.Rw[x] = rT;
      A.Cw[x] = cT;
    }
    cnt.vertices += 1;
    cnt.edges += (unsigned long long)deg[k] + 1;
    maxdr = dr > maxdr ? dr : maxdr;
    // fp32 ranks: a change of one unit in the last place is rounding noise
    // of the unordered sums, never a reason for another sweep (a rank of
    // 1e-2 has ulp 9e-10, above the iteration tolerance)
    double wt = A.wtol;
    if constexpr (sizeof(T) == 4) {
      const float ar = fabsf((float)rT);
      const double ulp = (double)__uint_as_float(__float_as_uint(ar) + 1u) - (double)ar;
      wt = ulp > wt ? ulp : wt;
    }
    if (dr > wt) moved = true;
    if constexpr (MODE != kAll) {
      if (dr > A.ftol) {
        // a vertex that already marked all its out-neighbours has nothing
        // left to mark: affected flags are never cleared within an update
        if (!(fb & kEX)) {
          expand[k] = true;
          cnt.out_scanned += (unsigned long long)d;
          if (MODE == kSyncDF && d >= A.split_min) {
            // marked after the iteration by whole workgroups (the marks
            // take effect in the next iteration either way)
            const unsigned long long j = atomicAdd(&A.ctl->nexp, 1ull);
            A.xrow[j] = x;
          } else {
            od[k] = d;
            oo[k] = xo;
            any_expand = any_expand || d > 0;
          }
        }
      }
    }
  }
  if constexpr (MODE == kAll) return;
  if (__ballot(any_expand) != 0) expand_flat<T, MODE>(A, L, oo, od, newly);
#pragma unroll
  for (int k = 0; k < kQ; ++k)
    if (expand[k]) flag_set(A.flags, v[k], kEX);
}

// Processes one step: four vertices per lane (vin[k] < 0: empty slot).  All
// 64 lanes call it.  `moved` is set when a rank changed by more than the
// watermark tolerance (lock-free scheme); `maxdr` tracks the largest
// change.  Rows with at least split_min in-edges are left to the piece
// path.
template <typename T, int MODE>
__device__ __forceinline__ void process_step(const RankArgs<T> &A, WaveLds<T> &L,
                                             const int32_t *vin, Counters &cnt,
                                             double &maxdr, long long &newly,
                                             bool &moved) {
  constexpr bool COH = MODE == kAsync;
  int32_t v[kQ];
  int64_t off[kQ];
  int32_t deg[kQ];
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    v[k] = vin[k];
    off[k] = 0;
    deg[k] = 0;
    if (v[k] >= 0) {
      // degree and offset in one round trip (the offset of a long row is
      // read for nothing)
      const int32_t d = A.in_deg[v[k]];
      const int64_t o = A.in_off[v[k]];
      if (d >= A.split_min) {
        v[k] = -1;
      } else {
        off[k] = o;
        deg[k] = d;
      }
    }
  }
  double sum[kQ];
  gather_flat<T, COH>(A, L, off, deg, sum);
  finish_rows<T, MODE>(A, L, v, deg, sum, cnt, maxdr, newly, moved);
}

// One piece of a long row: the wavefront sums up to kPiece consecutive
// in-edges of the row in registers (fp64 for both rank types) and publishes
// the partial sum; the wavefront that completes the row's last piece adds
// the row's partial sums in piece order (so the result does not depend on
// which piece finished when) and finishes the vertex.
//   barrier-based scheme, static PageRank: every piece of the row is summed
//     once per iteration, and the finishing wavefront resets the counter;
//   lock-free scheme: sweeps overlap, so a piece can be summed again before
//     a slow piece of the previous sweep is in.  The counter runs on, and
//     every np-th completion finishes the vertex from the latest partial
//     sums, provided each piece was summed during this launch (tagged with
//     the launch); otherwise `moved` forces another sweep.
template <typename T, int MODE>
__device__ void process_piece(const RankArgs<T> &A, WaveLds<T> &L, int32_t p,
                              Counters &cnt, double &maxdr, long long &newly,
                              bool &moved) {
  constexpr bool COH = MODE == kAsync;
  const int lane = lane_id();
  const int32_t j = __builtin_amdgcn_readfirstlane(COH ? load_agent(A.prow + p) : A.prow[p]);
  const int32_t v = __builtin_amdgcn_readfirstlane(COH ? load_agent(A.lrow + j) : A.lrow[j]);
  const int32_t first =
      __builtin_amdgcn_readfirstlane(COH ? load_agent(A.lpre + j) : A.lpre[j]);
  const int32_t d = __builtin_amdgcn_readfirstlane(A.in_deg[v]);
  const int32_t np = (d + kPiece - 1) / kPiece;
  const int32_t *row = A.in_adj + A.in_off[v];
  const int32_t a = (p - first) * kPiece;
  const int32_t b = a + kPiece < d ? a + kPiece : d;
  double part = 0.0;
  // pipelined like gather_flat: the next round's row entries load while
  // this round's contributions are in flight; lanes past the end load the
  // last entry again and add nothing (a < b for every piece)
  int32_t idx[kUnroll];
  auto fetch = [&](int32_t e0) {
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int32_t e = e0 + q * kWave + lane;
      idx[q] = row[e < b ? e : b - 1];
    }
  };
  fetch(a);
  for (int32_t e0 = a; e0 < b; e0 += kUnroll * kWave) {
    T c[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) c[q] = ldc<T, COH>(A.Cr, idx[q]);
    const int32_t next = e0 + kUnroll * kWave;
    if (next < b) fetch(next);
#pragma unroll
    for (int q = 0; q < kUnroll; ++q)
      part += e0 + q * kWave + lane < b ? (double)c[q] : 0.0;
  }
  part = wave_sum(part);
  if (lane == 0) cnt.edges += (unsigned long long)(b - a);
  double total = part;
  if (np > 1) {
    int last = 0;
    if (lane == 0) {
      store_agent(A.ppart + p, part);
      if (COH) store_agent(A.ptag + p, A.epoch);
      // the partial sum (and tag) complete before the count that publishes
      // them; the finishing wavefront reads them with device-scope loads
      stores_complete();
      const int32_t before = __hip_atomic_fetch_add(A.lcnt + j, 1, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      last = COH ? (before + 1) % np == 0 : before == np - 1;
    }
    if (!__builtin_amdgcn_readfirstlane(last)) return;
    if constexpr (COH) {
      bool have = true;
      for (int32_t k = lane; k < np; k += kWave)
        have = have && load_agent(A.ptag + first + k) == A.epoch;
      if (__ballot(!have) != 0) {
        moved = true;  // a piece not yet summed in this launch: next sweep
        return;
      }
    }
    // fixed order: lane k adds pieces k, k + 64, ..., then the wave sum
    double t = 0.0;
    for (int32_t k = lane; k < np; k += kWave) t += load_agent(A.ppart + first + k);
    total = wave_sum(t);
    // barrier-based: every piece of the row has arrived, ready for the next
    // iteration
    if (!COH && lane == 0) store_agent(A.lcnt + j, 0);
  }
  int32_t vv[kQ];
  int32_t dd[kQ];
  double ss[kQ];
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    vv[k] = (k == 0 && lane == 0) ? v : -1;
    dd[k] = 0;
    ss[k] = total;
  }
  finish_rows<T, MODE>(A, L, vv, dd, ss, cnt, maxdr, newly, moved);
}

template <typename T>
__device__ __forceinline__ void flush_counters(Ctl *ctl, Counters &c) {
  const unsigned long long v = wave_sum(c.vertices);
  const unsigned long long e = wave_sum(c.edges);
  const unsigned long long o = wave_sum(c.out_scanned);
  if (lane_id() == 0) {
    if (v) atomicAdd(&ctl->vertices, v);
    if (e) atomicAdd(&ctl->edges, e);
    if (o) atomicAdd(&ctl->out_scanned, o);
  }
}

// Sweep-end decision, lane 0 only, on a state word W read with a relaxed
// load whose cursor reached the end of the group worklist.
//
// Convergence (Algorithm 2's R_C flags, kept per claim): a claim that saw
// a rank change above the watermark tolerance wtol (the iteration
// tolerance for DF updates, or the frontier tolerance) or met an entry it
// could not finish raises change_sweep to the sweep index current when it
// is published (after the claim's stores completed, and before its
// in-flight mark drops).  Sweep S may end the launch only when no claim is held and
// change_sweep < S: then every worklist entry was processed during S and
// no rank moved by more than wtol, so every R_C is 0.  Otherwise the next
// sweep starts as soon as a claim completed during S has seen a change,
// without waiting for the other claims still held (no barrier).  (Starting
// it before any such change was tried: no faster, and one clean sweep more
// at the end.)
template <typename T>
__device__ void sweep_end(const RankArgs<T> &A, unsigned long long W,
                          int *done_count) {
  unsigned long long *st = &A.ctl->state;
  const unsigned long long bound = load_agent(&A.ctl->gtail);
  const unsigned long long cur = (W >> kCursorShift) & kCursorMask;
  if (cur < bound) return;
  const unsigned long long sweep = (W >> kSweepShift) & kSweepMask;
  const unsigned long long inflight = W & kInflightMask;
  const long long cs = load_agent(&A.ctl->change_sweep);
  unsigned long long nw;
  if (cs >= (long long)sweep) {
    // a claim completed during this sweep saw a change: the next sweep
    // starts at once, while this sweep's other claims finish
    const unsigned long long ns = sweep + 1;
    if ((long long)ns >= A.max_iters)
      nw = kDone | kCapped | (ns << kSweepShift);
    else
      nw = (ns << kSweepShift) | inflight;
  } else if (inflight == 0) {
    // confirm once with acquire ordering before ending the graph's update
    if (__hip_atomic_load(st, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != W) return;
    if (load_agent(&A.ctl->change_sweep) >= (long long)sweep) return;
    nw = kDone | ((sweep + 1) << kSweepShift);
  } else {
    return;  // claims in flight, no change seen in this sweep yet: wait
  }
  unsigned long long expect = W;
  const bool won = __hip_atomic_compare_exchange_strong(
      st, &expect, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (won && (nw & kDone) && done_count) atomicAdd(done_count, 1);
}

enum StepResult { kWorked = 0, kNoWork = 1, kGraphDone = 2, kStop = 3 };

// Scheduling state of one workgroup of the lock-free scheme on one graph
// (the same copy in every thread; `seen` is kept by thread 0).
//
// Claims are made per workgroup, and the workgroup's wavefronts share the
// claimed entries: the scheduling word is one per graph, and every
// operation on it is a round trip to the device's coherence point, so
// wavefronts claiming one by one either waited on the word (many small
// claims) or were too few to keep the memory system busy (few large ones).
// A workgroup keeps its in-flight mark after a claim and trades it for the
// next claim in the same fetch_add (the cursor advances, the count stays).
// The change of the finished claim is published after that atomic, while
// the new mark still keeps the sweep from ending, and only when the
// watermark the workgroup last saw is below the current sweep.
struct WaveSched {
  bool held = false;       // holds an in-flight mark
  bool moved = false;      // its finished claim saw a change to publish
  long long seen = -1;     // change_sweep as last returned (thread 0)
  unsigned idle = 0;       // consecutive steps without work (backoff)
  unsigned polls = 0;      // steps made (abort polling)
};

// Thread 0's decision of a step, broadcast to the workgroup.
struct ClaimShare {
  unsigned long long p, end;
  int code;
  int held;
};

// Thread 0: publishes a finished claim's change at sweep `now`.
template <typename T>
__device__ __forceinline__ void publish(const RankArgs<T> &A, WaveSched &ws, long long now) {
  if (ws.seen < now) {
    const long long before = __hip_atomic_fetch_max(&A.ctl->change_sweep, now, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    ws.seen = before > now ? before : now;
  }
}

// Thread 0: drops the workgroup's in-flight mark, publishing its last
// change first (the workgroup's stores are already performed).
template <typename T>
__device__ __forceinline__ void release_mark(const RankArgs<T> &A, WaveSched &ws) {
  if (!ws.held) return;
  if (ws.moved)
    publish(A, ws, (long long)((load_agent(&A.ctl->state) >> kSweepShift) & kSweepMask));
  // the watermark update is performed before the in-flight mark drops
  stores_complete();
  __hip_atomic_fetch_sub(&A.ctl->state, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  ws.held = false;
  ws.moved = false;
}

constexpr int kScan = 16;  // worklist entries read at once (a claim holds at most 16)

// Processes the worklist entries [b, e) of a claim in place, one wavefront.
// Pieces of long rows are summed one by one.  The affected vertices of the
// group parts are gathered into steps of up to 256 vertices: the
// parts of a frontier are sparse (on the road-like grid a quarter of a
// part's ids are affected), and each step costs a chain of dependent memory
// round trips however few vertices it holds.
template <typename T>
__device__ __forceinline__ void process_claim(const RankArgs<T> &A, WaveLds<T> &L,
                                              unsigned long long b, unsigned long long e,
                                              Counters &cnt, long long &newly, bool &moved) {
  const int lane = lane_id();
  const uint64_t below = lanemask_lt();
  double unused = 0.0;
  int32_t nbuf = 0;  // vertices gathered (the same in every lane)
  auto flush = [&]() {
    if (nbuf == 0) return;
    wave_lds_fence();
    int32_t vv[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
      const int32_t pos = k * kWave + lane;
      vv[k] = pos < nbuf ? L.vbuf[pos] : -1;
    }
    wave_lds_fence();
    process_step<T, kAsync>(A, L, vv, cnt, unused, newly, moved);
    nbuf = 0;
  };
  // entries are read kScan at a time, and the flag words of all their
  // group parts are loaded before any is used: two memory round trips per
  // kScan entries instead of two per entry
  for (unsigned long long g0 = b; g0 < e; g0 += kScan) {
    const int32_t ne = (int32_t)(e - g0 < (unsigned long long)kScan ? e - g0 : kScan);
    const int32_t xl = lane < ne ? load_agent(A.gwl + g0 + lane) : -1;
    // one 32-bit flag word per lane: the flags of the part's vertices
    // v0 + 4 lane .. v0 + 4 lane + 3 (a part spans 16 to 256 ids)
    auto flag_word = [&](int32_t x) -> uint32_t {
      if (x < 0) return 0u;
      const int32_t l = (x >> kEntryLogShift) & 7;
      const int32_t span = kGroup >> l;
      const int32_t v0 = ((x & kEntryGroupMask) << kGroupShift) +
                         ((x >> kEntryPartShift) & 15) * span;
      const int32_t v = v0 + 4 * lane;
      return 4 * lane < span && v < A.n ? load_agent(A.flags + (v >> 2)) : 0u;
    };
    uint32_t fw[kScan];
#pragma unroll
    for (int j = 0; j < kScan; ++j)
      fw[j] = j < ne ? flag_word(__builtin_amdgcn_readlane(xl, j)) : 0u;
#pragma unroll
    for (int j = 0; j < kScan; ++j) {
      if (j >= ne) break;
      int32_t x = __builtin_amdgcn_readlane(xl, j);
      uint32_t f = fw[j];
      if (x == -1) {
        // slot reserved, entry not yet stored when the batch was read
        // (appends at the tail race with claims there): read it again
        x = lane == 0 ? load_agent(A.gwl + g0 + j) : -1;
        x = __builtin_amdgcn_readfirstlane(x);
        if (x == -1) {
          // still not stored: its appender holds a mark; count it as work
          // left all the same
          moved = true;
          continue;
        }
        f = flag_word(x);
      }
      if (x <= -2) {  // a piece of an affected long row
        process_piece<T, kAsync>(A, L, -x - 2, cnt, unused, newly, moved);
        continue;
      }
      const int32_t l = (x >> kEntryLogShift) & 7;
      const int32_t span = kGroup >> l;
      const int32_t v0 = ((x & kEntryGroupMask) << kGroupShift) +
                         ((x >> kEntryPartShift) & 15) * span;
      const int32_t v = v0 + 4 * lane;
      // affected vertices in id order (consecutive rows keep their edges
      // contiguous for the gather): a lane's count (0..4) is summed over
      // the lanes below it bit by bit, one ballot per bit
      bool aff[4];
      uint32_t c = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        aff[i] = v + i < A.n && ((f >> (8 * i)) & kVA);
        c += aff[i] ? 1u : 0u;
      }
      const uint64_t m0 = __ballot(c & 1u), m1 = __ballot(c & 2u), m2 = __ballot(c & 4u);
      const int32_t total = __popcll(m0) + 2 * __popcll(m1) + 4 * __popcll(m2);
      if (nbuf + total > kRows) flush();
      int32_t pos = nbuf + __popcll(m0 & below) + 2 * __popcll(m1 & below) +
                    4 * __popcll(m2 & below);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (aff[i]) L.vbuf[pos++] = v + i;
      nbuf += total;
    }
  }
  flush();
}

// Idle backoff: 64 * 2^min(idle, 4) sleep units, so workgroups without work
// poll the scheduling word less often the longer they find nothing.
__device__ __forceinline__ void idle_sleep(unsigned idle) {
  const unsigned k = idle < 4 ? idle : 4;
  for (unsigned i = 0; i < (1u << k); ++i) __builtin_amdgcn_s_sleep(64);
}

// One scheduling step of the lock-free scheme on one graph, made by the
// whole workgroup: thread 0 claims `per` positions of the worklist (a
// workgroup without a mark first reads the word, so that idle workgroups
// neither claim past the end nor hold more marks than the graph has
// entries), and the wavefronts process the claimed entries in turn.  Thread
// 0 also polls the abort flag and the watchdog; kStop ends the kernel.
template <typename T>
__device__ int df_async_step(const RankArgs<T> &A, WaveLds<T> &L, Counters &cnt,
                             long long &newly, unsigned long long per, int *done_count,
                             int *abort_flag, unsigned long long t_start,
                             unsigned long long timeout_ticks, WaveSched &ws,
                             ClaimShare &sh) {
  if (threadIdx.x == 0) {
    int code = kWorked;
    unsigned long long p = 0, end = 0;
    ++ws.polls;
    if ((ws.polls & 15u) == 0 && load_agent(abort_flag)) {
      code = kStop;
    } else if (ws.idle > 0 && timeout_ticks && (ws.polls & 63u) == 0 &&
               wall_clock64() - t_start > timeout_ticks) {
      store_agent(abort_flag, 1);
      code = kStop;
    } else if (!ws.held) {
      const unsigned long long W = load_agent(&A.ctl->state);
      const unsigned long long gt = load_agent(&A.ctl->gtail);
      if (W & kDone) {
        code = kGraphDone;
      } else if (((W >> kCursorShift) & kCursorMask) >= gt) {
        sweep_end(A, W, done_count);
        code = kNoWork;
      } else if ((W & kInflightMask) >= gt) {
        code = kNoWork;
      }
    }
    if (code == kWorked) {
      // claim: cursor += per for each wavefront, and one more mark unless
      // the workgroup holds one
      const unsigned long long take = per * (blockDim.x / kWave);
      const unsigned long long grab = (take << kCursorShift) | (ws.held ? 0ull : 1ull);
      const unsigned long long W2 = __hip_atomic_fetch_add(&A.ctl->state, grab, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long gt = load_agent(&A.ctl->gtail);
      // the previous claim's change, at the sweep current now: changes made
      // late in an old sweep still force a fresh full sweep
      if (ws.moved) publish(A, ws, (long long)((W2 >> kSweepShift) & kSweepMask));
      ws.moved = false;
      ws.held = true;
      if (W2 & kDone) {
        // the sweep cap ended the update: nothing more to give back
        ws.held = false;
        code = kGraphDone;
      } else {
        p = (W2 >> kCursorShift) & kCursorMask;
        if (p >= gt) {
          release_mark(A, ws);
          // the cursor has passed the end: try to close the sweep
          sweep_end(A, load_agent(&A.ctl->state), done_count);
          code = kNoWork;
        } else {
          end = p + take < gt ? p + take : gt;
        }
      }
    }
    sh.p = p;
    sh.end = end;
    sh.code = code;
    sh.held = ws.held ? 1 : 0;
  }
  __syncthreads();
  const int code = sh.code;
  const unsigned long long p = sh.p, end = sh.end;
  ws.held = sh.held != 0;
  if (code != kWorked) {
    ws.moved = false;
    ++ws.idle;
    __syncthreads();  // sh is read before thread 0 writes it again
    return code;
  }
  ws.idle = 0;
  // wavefront w takes the w-th run of `per` entries (neighbouring groups)
  const unsigned long long w = threadIdx.x / kWave;
  const unsigned long long b = p + w * per < end ? p + w * per : end;
  const unsigned long long e = b + per < end ? b + per : end;
  bool moved = false;
  process_claim<T>(A, L, b, e, cnt, newly, moved);
  // every store of this claim (ranks, contributions, flags, worklist
  // entries), by every wavefront, is performed before the workgroup's next
  // operation on the scheduling word, which gives its mark back
  stores_complete();
  ws.moved = __syncthreads_or(moved ? 1 : 0) != 0;
  return kWorked;
}

template <typename T>
__device__ __forceinline__ void flush_graph(Ctl *ctl, Counters &cnt,
                                            long long &newly) {
  flush_counters<T>(ctl, cnt);
  newly = wave_sum(newly);
  if (lane_id() == 0 && newly)
    atomicAdd((unsigned long long *)&ctl->newly, (unsigned long long)newly);
  cnt = Counters();
  newly = 0;
}

__device__ __forceinline__ unsigned long long groups_per_claim(int chunk) {
  // at least one so the cursor always advances
  return chunk >= kGroup ? (unsigned long long)(chunk / kGroup) : 1ull;
}

// The lock-free persistent kernel for one graph.
template <typename T>
__global__ void __launch_bounds__(256) k_df_async(RankArgs<T> A) {
  __shared__ ClaimShare sh;
  WaveLds<T> &L = wave_lds<T>();
  Counters cnt;
  long long newly = 0;
  const unsigned long long t_start = wall_clock64();
  const unsigned long long per = groups_per_claim(A.chunk);
  WaveSched ws;
  while (true) {
    const int r = df_async_step<T>(A, L, cnt, newly, per, nullptr, &A.ctl->abort, t_start,
                                   A.timeout_ticks, ws, sh);
    if (r == kGraphDone || r == kStop) break;
    if (r == kWorked) {
      if (injected_fault(A)) {
        // a stop at a claim boundary: the mark goes back first, so the
        // others can finish the update
        if (threadIdx.x == 0) release_mark(A, ws);
        break;
      }
      continue;
    }
    idle_sleep(ws.idle - 1);
  }
  flush_graph<T>(A.ctl, cnt, newly);
}

constexpr int kManyBits = 4096;

// The lock-free persistent kernel for many graphs at once: each workgroup
// works on one graph until it finds nothing to claim there, then moves to
// the next; the launch ends when every graph's update has ended.
template <typename T>
__global__ void __launch_bounds__(256) k_df_async_many(const RankArgs<T> *descs,
                                                       int count, int *done_count,
                                                       int *abort_flag,
                                                       unsigned long long timeout_ticks) {
  __shared__ ClaimShare sh;
  __shared__ int all_done;
  // graphs this workgroup has seen finished (the first kManyBits of them):
  // skipped without touching their scheduling words
  __shared__ uint32_t seen_done[kManyBits / 32];
  for (int i = threadIdx.x; i < kManyBits / 32; i += blockDim.x) seen_done[i] = 0u;
  WaveLds<T> &L = wave_lds<T>();
  int gi = (int)(blockIdx.x % (unsigned)count);
  RankArgs<T> A = descs[gi];
  unsigned long long per = groups_per_claim(A.chunk);
  Counters cnt;
  long long newly = 0;
  const unsigned long long t_start = wall_clock64();
  int idle = 0;
  unsigned laps = 0;
  WaveSched ws;
  while (true) {
    if (threadIdx.x == 0) all_done = load_agent(done_count) >= count;
    __syncthreads();
    const bool stop_all = all_done != 0;
    __syncthreads();
    if (stop_all) break;
    const int r = df_async_step<T>(A, L, cnt, newly, per, done_count, abort_flag, t_start,
                                   timeout_ticks, ws, sh);
    if (r == kStop) break;
    if (r == kWorked) {
      idle = 0;
      laps = 0;
      continue;
    }
    // nothing to claim here (no mark held): move on to the next graph not
    // seen finished
    flush_graph<T>(A.ctl, cnt, newly);
    if (r == kGraphDone && gi < kManyBits && threadIdx.x == 0)
      seen_done[gi >> 5] |= 1u << (gi & 31);
    __syncthreads();
    int next = gi;
    for (int k = 1; k <= count; ++k) {
      const int c = gi + k < count ? gi + k : gi + k - count;
      if (c >= kManyBits || !(seen_done[c >> 5] & (1u << (c & 31)))) {
        next = c;
        break;
      }
    }
    __syncthreads();
    gi = next;
    A = descs[gi];
    per = groups_per_claim(A.chunk);
    const unsigned polls = ws.polls;
    ws = WaveSched();  // the watermark seen belongs to the previous graph
    ws.polls = polls;
    // eight visits without work (or a lap over fewer graphs) back off
    if (++idle >= (count < 8 ? count : 8)) {
      idle = 0;
      idle_sleep(laps++);
    }
  }
  flush_graph<T>(A.ctl, cnt, newly);
}

// One iteration of the barrier-based scheme (or of static PageRank): the
// worklist (all vertices for static) is cut into steps of at most 256
// entries and about kStepEdges in-edges, and wavefronts claim steps.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_sync_iter(RankArgs<T> A, const int32_t *steps) {
  if (A.ctl->sync_done) return;
  const int iter = A.ctl->iter;  // device-side, so a captured launch replays
  WaveLds<T> &L = wave_lds<T>();
  const int lane = lane_id();
  Counters cnt;
  double maxdr = 0.0;
  long long newly = 0;  // vertices this wavefront marked for the first time
  unsigned long long done_items = 0;
  // pieces of long rows first (their finishing wavefronts may still have
  // an out-row to mark), then the steps
  const unsigned long long packed = A.sync_len[iter];
  const unsigned long long npieces = packed >> 32;
  const unsigned long long nitems = npieces + (packed & 0xFFFFFFFFull);
  // claims are spread over nctr counters, at most kClaimers and no more
  // than the grid has wavefronts (item c + nctr * k from counter c): one
  // hot counter serialised ~20K claims per iteration on the 2^22 R-MAT.
  // (Blocks of consecutive items per counter, the counters of one XCD
  // taking neighbouring blocks so that neighbouring steps share an L2,
  // made the update slower on both the R-MAT and the road-like grid, and
  // 1.3x slower on the 2^14 R-MAT.)  Every wavefront drains its own
  // counter, so all items
  // are claimed unless wavefronts stop early (an injected stop fault); then
  // a wavefront that drained its own counter takes over the others in
  // turn, so the items behind a counter whose wavefronts stopped are still
  // claimed.  Counters only grow, so a plain read that shows one drained
  // skips it.  Without stop faults the scan is skipped: each probe of a
  // counter is a device-coherent access, and with the scan always on the
  // launches on the 2^22 R-MAT took 0.79 ms instead of 0.69 ms.
  const unsigned wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * (blockDim.x / kWave);
  const unsigned nctr = nwaves < (unsigned)kClaimers ? nwaves : (unsigned)kClaimers;
  const unsigned c = wave % nctr;
  const unsigned scan = A.fault_stops ? nctr : 1u;
  bool stopped = false;
  for (unsigned k = 0; k < scan && !stopped; ++k) {
    const unsigned cc = (c + k) % nctr;
    unsigned long long *ctr = A.sync_grab + cc * kClaimStride;
    if (k > 0) {
      unsigned long long seen = 0;
      if (lane == 0) seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cc + nctr * bcast0(seen) >= nitems) continue;
    }
    while (true) {
      unsigned long long u = 0;
      if (lane == 0) u = cc + nctr * atomicAdd(ctr, 1ull);
      u = bcast0(u);
      if (u >= nitems) break;
      if (u < npieces) {
        bool unused_moved = false;
        process_piece<T, MODE>(A, L, (int32_t)u, cnt, maxdr, newly, unused_moved);
      } else {
        u -= npieces;
        const int32_t start = steps[u], end = steps[u + 1];
        int32_t vv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const int32_t pos = start + q * kWave + lane;
          vv[q] = pos < end ? (MODE == kAll ? pos : A.wl[pos]) : -1;
        }
        bool unused_moved = false;
        process_step<T, MODE>(A, L, vv, cnt, maxdr, newly, unused_moved);
      }
      ++done_items;
      if (injected_fault(A)) {
        stopped = true;
        break;
      }
    }
  }
  maxdr = wave_max(maxdr);
  const unsigned long long v = wave_sum(cnt.vertices);
  const unsigned long long e = wave_sum(cnt.edges);
  const unsigned long long o = wave_sum(cnt.out_scanned);
  newly = wave_sum(newly);
  if (lane == 0) {
    unsigned long long *slot = A.sync_grab + c * kClaimStride;
    if (maxdr > 0.0)
      atomicMax(slot + kSlotMaxDr, (unsigned long long)__double_as_longlong(maxdr));
    if (v) atomicAdd(slot + kSlotVertices, v);
    if (e) atomicAdd(slot + kSlotEdges, e);
    if (o) atomicAdd(slot + kSlotOut, o);
    if (newly) atomicAdd(slot + kSlotNewly, (unsigned long long)newly);
    if (done_items) atomicAdd(slot + kSlotItems, done_items);
  }
}

// Sum of the slots' newly-affected counts.
__device__ __forceinline__ unsigned long long slots_newly(const unsigned long long *slots) {
  unsigned long long t = 0;
#pragma unroll
  for (int c = 0; c < kClaimers; ++c) t += slots[c * kClaimStride + kSlotNewly];
  return t;
}

// Call totals of the slots into the control block (after the loop).
__global__ void k_slot_totals(const unsigned long long *slots, Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long v = 0, e = 0, o = 0;
  for (int c = 0; c < kClaimers; ++c) {
    v += slots[c * kClaimStride + kSlotVertices];
    e += slots[c * kClaimStride + kSlotEdges];
    o += slots[c * kClaimStride + kSlotOut];
  }
  ctl->vertices = v;
  ctl->edges = e;
  ctl->out_scanned = o;
}

// Marks the out-neighbours of the long out-rows deferred by the iteration
// (one workgroup per row, threads striding it) and counts the newly
// affected vertices.
__global__ void __launch_bounds__(256) k_expand_long(const int32_t *xrow,
                                                     const int64_t *out_off,
                                                     const int32_t *out_deg,
                                                     const int32_t *out_adj,
                                                     uint32_t *flags, Ctl *ctl,
                                                     unsigned long long *slots) {
  const unsigned long long nx = ctl->nexp;
  long long newly = 0;
  for (unsigned long long j = blockIdx.x; j < nx; j += gridDim.x) {
    const int32_t v = xrow[j];
    const int32_t *row = out_adj + out_off[v];
    const int32_t d = out_deg[v];
    for (int32_t e = threadIdx.x; e < d; e += blockDim.x)
      if (mark_vertex_sync(flags, row[e])) ++newly;
  }
  newly = wave_sum(newly);
  if (lane_id() == 0 && newly)
    atomicAdd(slots + (blockIdx.x % kClaimers) * kClaimStride + kSlotNewly,
              (unsigned long long)newly);
}

// One wavefront: the iteration's largest change from the slots, the
// convergence decision, and the slot words reset for the next iteration.
__global__ void k_sync_finish(Ctl *ctl, unsigned long long *sync_max,
                              unsigned long long *sync_len,
                              unsigned long long *slots,
                              double tol, int max_iters, int df) {
  const int t = threadIdx.x;
  unsigned long long bits = 0, items = 0;
  if (t < kClaimers) {
    unsigned long long *slot = slots + t * kClaimStride;
    bits = slot[kSlotMaxDr];
    items = slot[kSlotItems];
    slot[kSlotClaim] = 0;
    slot[kSlotNewly] = 0;
    slot[kSlotMaxDr] = 0;
    slot[kSlotItems] = 0;
  }
  // non-negative doubles order like their bit patterns
  bits = wave_max(bits);
  items = wave_sum(items);
  if (t != 0) return;
  ctl->nexp = 0;
  if (ctl->sync_done) return;
  const int iter = ctl->iter;
  const unsigned long long packed = sync_len[iter];
  if (items != (packed >> 32) + (packed & 0xFFFFFFFFull)) {
    // work items left unprocessed (every workgroup stopped by an injected
    // fault): the iteration is incomplete
    ctl->abort = 1;
    ctl->sync_done = 1;
    ctl->sync_final = iter + 1;
    ctl->sync_conv = 0;
    return;
  }
  sync_max[iter] = bits;
  const double md = __longlong_as_double((long long)bits);
  if (md <= tol || iter + 1 >= max_iters) {
    ctl->sync_done = 1;
    ctl->sync_final = iter + 1;
    ctl->sync_conv = md <= tol ? 1 : 0;
  } else {
    sync_len[iter + 1] = ctl->nsteps | (ctl->npieces << 32);
    ctl->iter = iter + 1;
  }
}

__global__ void k_sync_begin(Ctl *ctl, unsigned long long *sync_max,
                             unsigned long long *sync_grab,
                             unsigned long long *sync_len, int iters) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < iters;
       i += gridDim.x * blockDim.x) {
    sync_max[i] = 0;
    sync_len[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < kClaimers * kClaimStride) sync_grab[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sync_len[0] = ctl->nsteps | (ctl->npieces << 32);
    ctl->sync_done = 0;
    ctl->sync_final = 0;
    ctl->sync_conv = 0;
    ctl->iter = 0;
    ctl->vertices = ctl->edges = ctl->out_scanned = 0;
    ctl->abort = 0;
    ctl->newly = 0;
    ctl->nexp = 0;
  }
}

__global__ void k_async_begin(Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl->state = 0ull;
  ctl->newly = 0;
  ctl->change_sweep = -1;
  ctl->gtail = 0;
  ctl->nlong = 0;
  ctl->npieces = 0;
  ctl->vertices = ctl->edges = ctl->out_scanned = 0;
  ctl->abort = 0;
}

// Clears the flags of every worklist vertex and the worklist itself.
__global__ void k_cleanup(uint32_t *flags, int32_t *wl,
                          unsigned long long len) {
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
       i < len; i += (unsigned long long)gridDim.x * blockDim.x) {
    const int32_t v = wl[i];
    if (v >= 0) reinterpret_cast<uint8_t *>(flags)[v] = 0;
    wl[i] = -1;
  }
}

// Clears the group flags, the vertex flags of every listed group and the
// group worklist (one thread per worklist entry; the parts of a group clear
// the same flags, pieces nothing).
__global__ void k_cleanup_groups(uint32_t *gflags, uint32_t *flags, int32_t *gwl,
                                 unsigned long long glen, int32_t n) {
  const int64_t words_per_group = kGroup / 4;
  const int64_t wmax = ((int64_t)n + 3) / 4;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
       i < glen; i += (unsigned long long)gridDim.x * blockDim.x) {
    const int32_t x = gwl[i];
    gwl[i] = -1;
    if (x < 0) continue;
    const int32_t grp = x & kEntryGroupMask;
    const int64_t w0 = (int64_t)grp * words_per_group;
    for (int64_t k = 0; k < words_per_group && w0 + k < wmax; ++k) flags[w0 + k] = 0u;
    reinterpret_cast<uint8_t *>(gflags)[grp] = 0;
  }
}

// Per-graph summary of the control block, gathered for many graphs at once.
struct Summary {
  unsigned long long state, tail, gtail, vertices, edges, out_scanned;
  long long marked, newly;
  int abort, pad;
};

template <typename T>
__global__ void k_gather_summary(const RankArgs<T> *descs, int count, Summary *out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const Ctl *c = descs[i].ctl;
    Summary s;
    s.state = c->state;
    s.tail = c->tail;
    s.gtail = c->gtail;
    s.vertices = c->vertices;
    s.edges = c->edges;
    s.out_scanned = c->out_scanned;
    s.marked = c->marked;
    s.newly = c->newly;
    s.abort = c->abort;
    s.pad = 0;
    out[i] = s;
  }
}

template <typename T>
__global__ void k_begin_many(const RankArgs<T> *descs, int count, int *done_count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    Ctl *c = descs[i].ctl;
    c->state = 0ull;
    c->newly = 0;
    c->change_sweep = -1;
    c->gtail = 0;
    c->nlong = 0;
    c->npieces = 0;
    c->abort = 0;
    c->vertices = c->edges = c->out_scanned = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *done_count = 0;
}

// One workgroup per graph: clears the flags and worklists the update used.
template <typename T>
__global__ void k_cleanup_many(const RankArgs<T> *descs, int count) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const RankArgs<T> &A = descs[i];
    Ctl *c = A.ctl;
    const unsigned long long len = c->tail, glen = c->gtail, nl = c->nlong;
    for (unsigned long long k = threadIdx.x; k < nl; k += blockDim.x) A.lcnt[k] = 0;
    for (unsigned long long k = threadIdx.x; k < len; k += blockDim.x) {
      const int32_t v = A.wl[k];
      if (v >= 0) reinterpret_cast<uint8_t *>(A.flags)[v] = 0;
      A.wl[k] = -1;
    }
    const int64_t wmax = ((int64_t)A.n + 3) / 4;
    for (unsigned long long k = threadIdx.x; k < glen; k += blockDim.x) {
      const int32_t x = A.gwl[k];
      A.gwl[k] = -1;
      if (x < 0) continue;
      const int32_t grp = x & kEntryGroupMask;
      const int64_t w0 = (int64_t)grp * (kGroup / 4);
      for (int64_t q = 0; q < kGroup / 4 && w0 + q < wmax; ++q) A.flags[w0 + q] = 0u;
      reinterpret_cast<uint8_t *>(A.gflags)[grp] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      c->tail = 0;
      c->gtail = 0;
      c->change_sweep = -1;
      c->marked = 0;
      c->newly = 0;
    }
    __syncthreads();
  }
}

__global__ void k_reset_marks(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->tail = 0;
    ctl->gtail = 0;
    ctl->change_sweep = -1;
    ctl->marked = 0;
    ctl->newly = 0;
  }
}

template <typename T>
__global__ void k_uniform(int32_t n, const int32_t *out_deg, T *R, T *C) {
  const double r = 1.0 / (double)n;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    R[v] = (T)r;
    C[v] = (T)(r / (double)(out_deg[v] + 1));
  }
}

template <typename T>
__global__ void k_contrib(int32_t n, const int32_t *out_deg, const T *R,
                          T *C) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    C[v] = (T)((double)R[v] / (double)(out_deg[v] + 1));
}

template <typename T>
__global__ void k_sum(int32_t n, const T *R, double *out) {
  double s = 0.0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    s += (double)R[v];
  s = wave_sum(s);
  if (lane_id() == 0) atomicAdd(out, s);
}

// Renormalisation of fp32 ranks: scales the ranks by 1 / sum and recomputes
// the contributions, but only when |1 - sum| exceeds `guard` (n * tau).  A
// converged update misses up to about n * tau of mass by its own
// truncation (every affected vertex within tau of the fixed point, errors
// of one sign); rescaling that would move the largest ranks by
// R_v * (sum - 1) (2^22 R-MAT, lock-free fp32: the top rank by 1.8e-9, 3e-6
// of its value), and shifting every rank by (1 - sum) / n made small graphs,
// whose error lies along the ranks themselves, worse.  Drift beyond it
// (fp32 rounding accumulated over many updates) is rescaled.
template <typename T>
__global__ void k_scale(int32_t n, const int32_t *out_deg, const double *sum,
                        double guard, T *R, T *C) {
  const double sm = *sum;
  if (fabs(1.0 - sm) <= guard) return;
  const double f = 1.0 / sm;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const double r = (double)R[v] * f;
    R[v] = (T)r;
    C[v] = (T)(r / (double)(out_deg[v] + 1));
  }
}

// Ranks in the caller's id order <-> the internal order (int2ext may be
// null: identity).
template <typename T>
__global__ void k_ranks_in(int32_t n, const int32_t *int2ext, const double *ext,
                           T *R) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    R[i] = (T)ext[int2ext ? int2ext[i] : i];
}

template <typename T>
__global__ void k_ranks_out(int32_t n, const int32_t *int2ext, const T *R,
                            double *ext) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    ext[int2ext ? int2ext[i] : i] = (double)R[i];
}

__global__ void k_f32_to_f64(int32_t n, const float *a, double *b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    b[v] = (double)a[v];
}

__global__ void k_f64_to_f32(int32_t n, const double *a, float *b) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    b[v] = (float)a[v];
}

// Streaming copy for the bandwidth reference: each workgroup copies one
// contiguous range, four 16-byte loads in flight per thread before their
// stores (on MI355X 5.3 TB/s for 1 GiB, against 4.8 TB/s for a grid-stride
// loop of single loads and 5.2 TB/s for hipMemcpyAsync).
constexpr int kCopyUnroll = 4;
__global__ void __launch_bounds__(256) k_copy16(const int4 *src, int4 *dst, int64_t n16) {
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t b = blockIdx.x * per;
  const int64_t e = b + per < n16 ? b + per : n16;
  for (int64_t i = b + threadIdx.x; i < e; i += kCopyUnroll * 256) {
    int4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t j = i + u * 256;
      v[u] = j < e ? src[j] : int4{};
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t j = i + u * 256;
      if (j < e) dst[j] = v[u];
    }
  }
}

__global__ void k_copy1(const uint8_t *src, uint8_t *dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// --- host side ---------------------------------------------------------------

namespace {

inline int grid_for(int64_t work, int cu) {
  int64_t b = (work + 255) / 256;
  const int64_t lim = (int64_t)cu * 16;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

// Which launch a default launch parameter is chosen for.
enum LaunchKind { kLaunchSync = 0, kLaunchAsync = 1, kLaunchMany = 2 };

// The graph's internal order is by decreasing out-degree (reorder at
// creation): its heaviest rows sit together in the first groups.
inline bool degree_sorted(const dfpr_graph *g) { return g->int2ext != nullptr; }

// Interleaved runs of the lock-free group worklist on a degree-sorted graph
// (list_groups).  In id order its heaviest groups come first, and the
// cursor ran through the light tail while claims on the heavy head were
// still running: the 2^22 R-MAT update took 95 sweeps instead of 41.
constexpr int32_t kGroupStripes = 64;

// Vertices per wavefront of a lock-free claim.  Default, one graph: one
// 256-vertex group per 1024 groups of the graph, 1..16 (claims are costly
// next to the work of a small graph's sweep, and too few per sweep leave
// the device idle on a small one: the 2^14 R-MAT ran 10x slower with 16
// groups per wavefront than with one, the 2^22 R-MAT and the 4096 x 4096
// grid fastest with 16, which 32 made slower again).  Batched launch: 4
// groups, as the many graphs keep the device busy (over 1024 graphs of
// 1e3..1e6 edges, 1.8x faster than one group per wavefront, and 9-13%
// faster than 16).
inline int effective_chunk(const dfpr_graph *g, int kind = kLaunchAsync) {
  if (g->p.chunk > 0) return g->p.chunk;
  if (kind == kLaunchMany) return 4 * kGroup;
  // a degree-sorted graph's heavy groups would make 16-group claims longer
  // than a sweep: at most 4 there (2^22 R-MAT, sorted: 30.1 ms per update
  // with 4-group claims against 48.7 ms with 16, pieces from 2048 in-edges)
  const int most = degree_sorted(g) ? 4 : 16;
  int per = g->ngroups / 1024;
  per = per < 1 ? 1 : (per > most ? most : per);
  return per * kGroup;
}

// Threads per workgroup of the rank kernel: the block_size parameter, or
// by default 128 for the barrier-based scheme (256 was as fast on the large
// graphs and 9% slower on the 2^14 R-MAT), 256 for the lock-free scheme on
// one graph (a claim serves four wavefronts: the grid update took 4.4 ms
// against 5.0 ms with 128), 128 for the batched launch (its autotuned
// choice with 4-group claims in both precisions).
inline int block_for(const dfpr_graph *g, int kind) {
  if (g->p.block_size > 0) return g->p.block_size;
  return kind == kLaunchSync ? 128 : (kind == kLaunchAsync ? 256 : 128);
}

// Lock-free grid: enough workgroups that each takes about kChunksPerWave
// claims per sweep (a claim is one workgroup's, shared by its wavefronts).
// With more claim holders than a sweep has chunks, new sweeps start over
// entries still being processed and every workgroup contends for the one
// scheduling word (the 2^22 R-MAT ran 8x slower with every co-resident
// wavefront claiming than with a quarter of them).
constexpr int kChunksPerWave = 4;

inline long long claim_chunks(const dfpr_graph *g, unsigned long long gtail,
                              int kind = kLaunchAsync) {
  const long long per = effective_chunk(g, kind) / kGroup;
  return ((long long)gtail + per - 1) / per;
}

// Workgroups for `chunks` wavefront chunks per sweep (a workgroup claims
// one per wavefront): one claim per workgroup up to four wavefronts per CU
// in all (small graphs: the 2^14 R-MAT's 64 groups ran 3.7x faster with 64
// wavefronts than with 16), beyond that one per kChunksPerWave claims.
inline long long async_blocks(long long chunks, int cu_count, int waves_per_block) {
  const long long claims = (chunks + waves_per_block - 1) / waves_per_block;
  const long long floor_b =
      (4ll * (cu_count > 0 ? cu_count : 1) + waves_per_block - 1) / waves_per_block;
  long long b = (claims + kChunksPerWave - 1) / kChunksPerWave;
  if (b < floor_b) b = floor_b;
  if (b > claims) b = claims;
  return b > 0 ? b : 1;
}

// The lock-free scheme sums rows of kAsyncSplitMax in-edges or more in
// pieces whatever split_min_degree says: a claim must stay short next to a
// sweep, since a claim that outlives the sweep it began in computes from
// values a sweep old (with pieces disabled, one wavefront summing a
// 25,000-edge row ended the update 1.1e-9 from the fixed point).
constexpr int32_t kAsyncSplitMax = 8192;
// Default piece thresholds (split_min_degree 0), measured on the 2^22
// R-MAT.  Barrier-based: update 22.5 ms with pieces from 2048 or 4096
// in-edges, 22.7 ms from 8192, 26.3 ms from 16384.  Lock-free: 35.2 ms from
// 2048 or 4096, 32.5 ms from 8192, the most it allows.  (While finishing a
// row took acquire-release ordering, whose cache maintenance stalls a
// whole XCD, each piece cost so much that 6144..12288 was the barrier-based
// optimum at 24.7 ms, and 2048 gave 31.3 ms.)
constexpr int32_t kSyncSplitDefault = 2048;
// Lock-free default on a degree-sorted graph, where the rows just below the
// threshold sit together in the first groups: 2^22 R-MAT update 23.7 ms
// with pieces from 512 in-edges, 24.5 ms from 1024, 30.1 ms from 2048 (all
// with 4-group claims); 2^20 R-MAT of average degree 4: 5.2 ms from 512,
// 4.7 ms from 1024.
constexpr int32_t kAsyncSplitSorted = 512;

inline int32_t sync_split(const dfpr_graph *g) {
  return g->p.split_min_degree > 0 ? g->p.split_min_degree : kSyncSplitDefault;
}

inline int32_t async_split(const dfpr_graph *g) {
  if (g->p.split_min_degree <= 0) return degree_sorted(g) ? kAsyncSplitSorted : kAsyncSplitMax;
  return g->p.split_min_degree < kAsyncSplitMax ? g->p.split_min_degree : kAsyncSplitMax;
}

template <typename T>
RankArgs<T> make_args(dfpr_graph *g, int rd, int wr) {
  RankArgs<T> A;
  std::memset(&A, 0, sizeof(A));  // padding included: the args are hashed
  A.n = g->n;
  A.in_off = g->in.off;
  A.in_deg = g->in.deg;
  A.in_adj = g->in.adj;
  A.out_off = g->out.off;
  A.out_deg = g->out.deg;
  A.out_adj = g->out.adj;
  A.Rr = (const T *)g->R[rd];
  A.Cr = (const T *)g->C[rd];
  A.Rw = (T *)g->R[wr];
  A.Cw = (T *)g->C[wr];
  A.flags = g->flags;
  A.wl = g->wl;
  A.gflags = g->gflags;
  A.gwl = g->gwl;
  A.ctl = g->ctl;
  A.alpha = g->p.alpha;
  A.base = (1.0 - g->p.alpha) / (double)g->n;
  A.tol = g->p.tol;
  A.ftol = g->p.frontier_tol;
  A.wtol = g->p.lf_stop == DFPR_STOP_FRONTIER ? g->p.frontier_tol : g->p.tol;
  A.split_min = sync_split(g);
  A.kahan_min = g->p.kahan_min_degree;
  A.chunk = effective_chunk(g);
  A.max_iters = g->p.max_iters;
  A.timeout_ticks = g->p.timeout_ms > 0
                        ? (unsigned long long)g->p.timeout_ms * (unsigned long long)g->wallclock_khz
                        : 0ull;
  A.sync_max = g->sync_max;
  A.sync_grab = g->sync_grab;
  A.sync_len = g->sync_len;
  A.lrow = g->split.lrow;
  A.lpre = g->split.lpre;
  A.prow = g->split.prow;
  A.ppart = g->split.ppart;
  A.lcnt = g->split.lcnt;
  A.ptag = g->split.ptag;
  A.epoch = g->async_epoch;
  A.xrow = g->split.xrow;
  A.faults = g->faults;
  A.nfaults = g->nfaults;
  A.fault_stops = g->nfaults > 0 ? g->fault_stops : 0;
  A.ticks_per_us = (uint32_t)(g->wallclock_khz / 1000 > 0 ? g->wallclock_khz / 1000 : 1);
  A.group_stripes = degree_sorted(g) ? kGroupStripes : 1;
  return A;
}

// Co-resident workgroups (or the grid_blocks override).  The in-flight
// field of the scheduling word holds 16 bits, so the grid stays below 32768
// wavefronts; chunk <= 4096 keeps cursor overshoot far below 2^32.
template <typename K>
int persistent_blocks(dfpr_graph *g, K kernel, size_t lds, int block) {
  int blocks = g->p.grid_blocks;
  if (blocks <= 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * g->cu_count;
  }
  const int max_blocks = 32768 / (block / kWave);
  return blocks > max_blocks ? max_blocks : blocks;
}

// bytes the rank iteration must move, from the device counters
double algorithmic_bytes(const dfpr_graph *g, const Ctl &h) {
  const double e = (double)h.edges - (double)h.vertices;  // stored in-edges
  if (g->elem == 8)
    return 12.0 * e + 52.0 * (double)h.vertices + 5.0 * (double)h.out_scanned;
  return 8.0 * e + 36.0 * (double)h.vertices + 5.0 * (double)h.out_scanned;
}

// Work items of one barrier-based iteration, built from the affected flags
// (or from every vertex, for static PageRank) in three launches: per-tile
// counts, a scan over tiles, and an emit pass.  A tile is 256 or 1024
// consecutive vertex ids (see tile_per); its selected vertices keep id
// order.
//   worklist  wl[0 .. tail) (affected vertices; not written for static)
//   steps     worklist positions where a step starts, plus a sentinel: a
//             step never crosses a tile, starts at every kRows-th selected
//             vertex of the tile (the first included) and at every vertex
//             whose in-edges reach past a multiple of kStepEdges of the
//             tile's running count
//   pieces    rows with at least split_min in-edges count as one entry in
//             the steps and are summed in pieces of kPiece in-edges:
//             split.lrow (their ids), split.lpre (first piece of each),
//             split.prow (long row of each piece)
// Totals land in ctl->tail / nsteps / nlong / npieces.  Rows of fewer
// in-edges are never split, so a step can exceed kStepEdges by one row.
constexpr int32_t kStepEdges = 16384;
constexpr int kSyncWavesPerCU = 12;

struct TileSum {
  int32_t sel, steps, nlong, pieces;
};

struct TileSumPlus {
  __device__ __host__ TileSum operator()(const TileSum &a, const TileSum &b) const {
    return TileSum{a.sel + b.sel, a.steps + b.steps, a.nlong + b.nlong, a.pieces + b.pieces};
  }
};

// Exclusive block-wide prefix of x over the 256 threads; *total = sum.
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t *lds4,
                                                   int32_t *total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int32_t incl = wave_incl_scan(x);
  __syncthreads();
  if (lane == kWave - 1) lds4[w] = incl;
  __syncthreads();
  int32_t before = 0, sum = 0;
#pragma unroll
  for (int i = 0; i < 256 / kWave; ++i) {
    const int32_t t = lds4[i];
    before += i < w ? t : 0;
    sum += t;
  }
  *total = sum;
  return before + incl - x;
}

// Exclusive prefixes of K values over the 256-thread workgroup with one
// pair of barriers; tot[f] = the workgroup's sum of value f.
template <int K>
__device__ __forceinline__ void block_excl_scan_k(const int32_t *x, int32_t *ex,
                                                  int32_t *tot, int32_t (*lds)[256 / kWave]) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  int32_t incl[K];
#pragma unroll
  for (int f = 0; f < K; ++f) incl[f] = wave_incl_scan(x[f]);
  __syncthreads();  // earlier readers of lds are done
  if (lane == kWave - 1)
#pragma unroll
    for (int f = 0; f < K; ++f) lds[f][w] = incl[f];
  __syncthreads();
#pragma unroll
  for (int f = 0; f < K; ++f) {
    int32_t before = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < 256 / kWave; ++i) {
      const int32_t t = lds[f][i];
      before += i < w ? t : 0;
      sum += t;
    }
    ex[f] = before + incl[f] - x[f];
    tot[f] = sum;
  }
}

// A tile is 256 * PER consecutive ids, one 256-thread workgroup, PER ids
// per thread: PER = 4 for large graphs (a quarter of the workgroups and
// barriers: the 2^24-vertex grid's item building 8.3 -> 3.8 ms per update),
// PER = 1 for small ones, where the latency of one pass matters more.
constexpr int kTileLarge = 4;
inline int tile_per(int32_t n) { return n >= (1 << 20) ? kTileLarge : 1; }

template <int PER>
struct TileScan {
  int32_t v0;           // first id of the thread
  bool sel[PER], start[PER], is_long[PER];
  int32_t rank[PER];    // position among the tile's selected vertices
  int32_t srank[PER];   // position among the tile's step starts
  int32_t lrank[PER];   // position among the tile's long rows
  int32_t ppre[PER];    // first piece among the tile's pieces
  int32_t npieces[PER]; // pieces of the row
  TileSum tot;
};

template <bool ALL, int PER>
__device__ __forceinline__ TileScan<PER> tile_scan(const uint32_t *flags,
                                                   const int32_t *deg, int32_t n,
                                                   int32_t split) {
  constexpr int kPerThread = PER;
  __shared__ int32_t lds[3][256 / kWave];
  TileScan<PER> r;
  r.v0 = (int32_t)blockIdx.x * 256 * PER + (int32_t)threadIdx.x * kPerThread;
  const uint32_t fw = r.v0 < n ? flags[r.v0 >> 2] : 0u;
  int32_t len[kPerThread];
  int32_t c_sel = 0, c_len = 0;
  int32_t loc_rank[kPerThread], loc_y[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int32_t v = r.v0 + q;
    r.sel[q] = v < n && (ALL || ((fw >> (8 * (v & 3))) & 0xFFu) != 0);
    const int32_t d = r.sel[q] ? deg[v] : 0;
    r.is_long[q] = r.sel[q] && d >= split;
    len[q] = r.sel[q] ? (r.is_long[q] ? 1 : d + 1) : 0;
    r.npieces[q] = r.is_long[q] ? (d + kPiece - 1) / kPiece : 0;
    loc_rank[q] = c_sel;
    loc_y[q] = c_len;
    c_sel += r.sel[q] ? 1 : 0;
    c_len += len[q];
  }
  int32_t x2[2] = {c_sel, c_len}, b2[2], t2[2];
  block_excl_scan_k<2>(x2, b2, t2, lds);
  // a step starts every kRows selected vertices of the tile and at every
  // vertex whose in-edges reach past a multiple of kStepEdges of the
  // tile's running count
  int32_t c_start = 0, c_long = 0, c_pieces = 0;
  int32_t loc_s[kPerThread], loc_l[kPerThread], loc_p[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    r.rank[q] = b2[0] + loc_rank[q];
    const int32_t y = b2[1] + loc_y[q];
    r.start[q] = r.sel[q] && (r.rank[q] % kRows == 0 ||
                              (y + len[q] - 1) / kStepEdges != (y - 1) / kStepEdges);
    loc_s[q] = c_start;
    loc_l[q] = c_long;
    loc_p[q] = c_pieces;
    c_start += r.start[q] ? 1 : 0;
    c_long += r.is_long[q] ? 1 : 0;
    c_pieces += r.npieces[q];
  }
  int32_t x3[3] = {c_start, c_long, c_pieces}, b3[3], t3[3];
  block_excl_scan_k<3>(x3, b3, t3, lds);
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    r.srank[q] = b3[0] + loc_s[q];
    r.lrank[q] = b3[1] + loc_l[q];
    r.ppre[q] = b3[2] + loc_p[q];
  }
  r.tot = TileSum{t2[0], t3[0], t3[1], t3[2]};
  return r;
}

template <bool ALL, int PER>
__global__ void __launch_bounds__(256) k_tile_count(const uint32_t *flags,
                                                    const int32_t *deg, int32_t n,
                                                    int32_t split, TileSum *sums,
                                                    const unsigned long long *slots,
                                                    int reuse) {
  if (reuse && slots_newly(slots) == 0) return;  // nothing newly affected: keep
  const TileScan<PER> r = tile_scan<ALL, PER>(flags, deg, n, split);
  if (threadIdx.x == 0) {
    sums[blockIdx.x] = r.tot;
    if (blockIdx.x == gridDim.x - 1) sums[gridDim.x] = TileSum{0, 0, 0, 0};
  }
}

template <bool ALL, int PER>
__global__ void __launch_bounds__(256) k_tile_emit(const uint32_t *flags,
                                                   const int32_t *deg, int32_t n,
                                                   int32_t split, const TileSum *pre,
                                                   int32_t *wl, int32_t *steps,
                                                   Split S, Ctl *ctl,
                                                   const unsigned long long *slots,
                                                   int reuse) {
  if (reuse && slots_newly(slots) == 0) return;
  const TileScan<PER> r = tile_scan<ALL, PER>(flags, deg, n, split);
  const TileSum b = pre[blockIdx.x];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (!r.sel[q]) continue;
    const int32_t v = r.v0 + q;
    const int32_t pos = b.sel + r.rank[q];
    if (!ALL) wl[pos] = v;
    if (r.start[q]) steps[b.steps + r.srank[q]] = pos;
    if (r.is_long[q]) {
      const int32_t j = b.nlong + r.lrank[q];
      const int32_t p0 = b.pieces + r.ppre[q];
      S.lrow[j] = v;
      S.lpre[j] = p0;
      for (int32_t k = 0; k < r.npieces[q]; ++k) S.prow[p0 + k] = j;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const TileSum t = pre[gridDim.x];
    if (!ALL) ctl->tail = (unsigned long long)t.sel;
    ctl->nsteps = (unsigned long long)t.steps;
    ctl->nlong = (unsigned long long)t.nlong;
    ctl->npieces = (unsigned long long)t.pieces;
    steps[t.steps] = t.sel;
    S.lpre[t.nlong] = t.pieces;
  }
}

// Group worklist of the lock-free scheme from the listed flags: one
// 256-thread workgroup per graph compacts the graph's group flags into gwl,
// each listed group as its parts (log2 in the group byte), after the
// entries already there (the pieces of the long rows, k_list_long), and
// sets gtail.  The groups go in id order (stripes 1), or interleaved from
// `stripes` equal runs of ids: position i takes group (i mod stripes) *
// rows + i / stripes, so neighbouring entries come from far-apart runs.
__device__ __forceinline__ void list_groups(const uint8_t *gflags, int32_t ngroups,
                                            int32_t *gwl, unsigned long long *gtail,
                                            int32_t stripes) {
  __shared__ int32_t lds4[4];
  int32_t base = (int32_t)*gtail;
  const int32_t rows = (ngroups + stripes - 1) / stripes;
  const int32_t padded = rows * stripes;
  for (int32_t g0 = 0; g0 < padded; g0 += kRows) {
    const int32_t i = g0 + (int32_t)threadIdx.x;
    const int32_t gi = (i % stripes) * rows + i / stripes;
    const uint32_t b = i < padded && gi < ngroups ? gflags[gi] : 0u;
    const bool sel = (b & kGA) != 0;
    const int32_t l = (int32_t)((b >> kGPartShift) & 7u);
    const int32_t cnt = sel ? (1 << l) : 0;
    int32_t total = 0;
    const int32_t pos = block_excl_scan(cnt, lds4, &total);
    for (int32_t p = 0; p < cnt; ++p)
      gwl[base + pos + p] = gi | (p << kEntryPartShift) | (l << kEntryLogShift);
    base += total;
  }
  __syncthreads();  // every thread has read *gtail
  if (threadIdx.x == 0) *gtail = (unsigned long long)base;
}

// Lock-free scheme, at launch: the parts of every group (listed or not:
// groups listed later read them too), from the in-edges of its rows below
// the piece threshold.  One wavefront per group; the group byte keeps its
// other bits.
__device__ __forceinline__ void group_parts(uint32_t *gflags, const int32_t *deg, int32_t n,
                                            int32_t split, int32_t g) {
  const int lane = lane_id();
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int32_t v = (g << kGroupShift) + k * kWave + lane;
    const int32_t d = v < n ? deg[v] : 0;
    sum += d < split ? d : 0;
  }
  sum = wave_sum(sum);
  if (lane == 0) {
    int32_t l = 0;
    while (l < kMaxPartLog && (kPartEdges << l) < sum) ++l;
    uint8_t *b = reinterpret_cast<uint8_t *>(gflags) + g;
    *b = (uint8_t)((*b & ~(7u << kGPartShift)) | ((uint32_t)l << kGPartShift));
  }
}

__global__ void __launch_bounds__(256) k_group_parts(uint32_t *gflags, const int32_t *deg,
                                                     int32_t n, int32_t ngroups,
                                                     int32_t split) {
  const int32_t w = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int32_t nw = (int32_t)(gridDim.x * blockDim.x / kWave);
  for (int32_t g = w; g < ngroups; g += nw) group_parts(gflags, deg, n, split, g);
}

template <typename T>
__global__ void __launch_bounds__(256) k_group_parts_many(const RankArgs<T> *descs, int count) {
  const int32_t w = (int32_t)(threadIdx.x / kWave);
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const RankArgs<T> &A = descs[i];
    const int32_t ng = (A.n + kGroup - 1) / kGroup;
    for (int32_t g = w; g < ng; g += (int32_t)(blockDim.x / kWave))
      group_parts(A.gflags, A.in_deg, A.n, A.split_min, g);
  }
}

// Lock-free scheme, at launch: every affected long row is listed with its
// pieces at the head of the group worklist, so the long chains start
// first.  Rows that become affected during the update are listed by the
// frontier expansion.
__device__ __forceinline__ void list_long_rows(const uint32_t *flags, const int32_t *deg,
                                               int32_t n, int32_t split, int64_t v0,
                                               int64_t stride, Ctl *ctl, int32_t *lrow,
                                               int32_t *lpre, int32_t *lcnt,
                                               int32_t *prow, int32_t *gwl) {
  for (int64_t v = v0; v < n; v += stride) {
    if (!(reinterpret_cast<const uint8_t *>(flags)[v] & kVA)) continue;
    const int32_t d = deg[v];
    if (d >= split) list_long_row(ctl, lrow, lpre, lcnt, prow, gwl, (int32_t)v, d);
  }
}

__global__ void __launch_bounds__(256) k_list_long(const uint32_t *flags, const int32_t *deg,
                                                   int32_t n, int32_t split, Ctl *ctl,
                                                   Split S, int32_t *gwl) {
  list_long_rows(flags, deg, n, split, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                 (int64_t)gridDim.x * blockDim.x, ctl, S.lrow, S.lpre, S.lcnt, S.prow, gwl);
}

template <typename T>
__global__ void __launch_bounds__(256) k_list_long_many(const RankArgs<T> *descs, int count) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const RankArgs<T> &A = descs[i];
    list_long_rows(A.flags, A.in_deg, A.n, A.split_min, threadIdx.x, blockDim.x, A.ctl, A.lrow,
                   A.lpre, A.lcnt, A.prow, A.gwl);
  }
}

// After a lock-free launch: the piece counters of its long rows back to 0
// (the barrier-based scheme counts each iteration from 0).
__global__ void k_zero_lcnt(int32_t *lcnt, const Ctl *ctl) {
  const unsigned long long nl = ctl->nlong;
  for (unsigned long long j = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; j < nl;
       j += (unsigned long long)gridDim.x * blockDim.x)
    lcnt[j] = 0;
}

__global__ void __launch_bounds__(256) k_list_groups(const uint32_t *gflags, int32_t ngroups,
                                                     int32_t *gwl, Ctl *ctl, int32_t stripes) {
  list_groups(reinterpret_cast<const uint8_t *>(gflags), ngroups, gwl, &ctl->gtail, stripes);
}

template <typename T>
__global__ void __launch_bounds__(256) k_list_groups_many(const RankArgs<T> *descs, int count) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const RankArgs<T> &A = descs[i];
    list_groups(reinterpret_cast<const uint8_t *>(A.gflags), (A.n + kGroup - 1) / kGroup,
                A.gwl, &A.ctl->gtail, A.group_stripes);
    __syncthreads();
  }
}

__global__ void k_zero_bytes(uint32_t *p, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Exclusive scan of nt1 tile sums by one workgroup (whole wavefronts, at
// most 16): each thread sums a contiguous run, the run totals are scanned
// across the workgroup, and each thread writes its run's prefixes.
__global__ void __launch_bounds__(1024) k_tile_scan(const TileSum *sums, TileSum *pre,
                                                    int32_t nt1,
                                                    const unsigned long long *slots,
                                                    int reuse) {
  if (reuse && slots_newly(slots) == 0) return;
  __shared__ int32_t wtot[4][1024 / kWave];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int32_t per = (nt1 + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
  const int32_t b = (int32_t)threadIdx.x * per;
  const int32_t e = b + per < nt1 ? b + per : nt1;
  TileSum t{0, 0, 0, 0};
#pragma unroll 8
  for (int32_t i = b; i < e; ++i) t = TileSumPlus()(t, sums[i]);
  int32_t v[4] = {t.sel, t.steps, t.nlong, t.pieces};
  int32_t ex[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int32_t incl = wave_incl_scan(v[f]);
    if (lane == kWave - 1) wtot[f][w] = incl;
    ex[f] = incl - v[f];
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 4; ++f)
    for (int i = 0; i < w; ++i) ex[f] += wtot[f][i];
  TileSum run{ex[0], ex[1], ex[2], ex[3]};
  for (int32_t i = b; i < e; ++i) {
    pre[i] = run;
    run = TileSumPlus()(run, sums[i]);
  }
}

// Launches the three steps that build the work items of the next
// barrier-based iteration (all = true: every vertex, static PageRank) on
// stream s; no host synchronisation, so the launches can be captured.
// reuse: the previous items stay when the last iteration affected no new
// vertex (decided on the device).
void launch_items(dfpr_graph *g, bool all, bool reuse, hipStream_t s) {
  const int per = tile_per(g->n);
  const int32_t nt = (g->n + 256 * per - 1) / (256 * per);
  TileSum *sums = (TileSum *)g->tiles;
  TileSum *pre = sums + (nt + 1);
  const uint32_t *fl = g->flags;
  const int32_t split = sync_split(g);
  const int ru = all ? 0 : (reuse ? 1 : 0);
  const unsigned long long *sl = g->sync_grab;
  if (per == kTileLarge) {
    if (all)
      k_tile_count<true, kTileLarge><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, sums, sl, 0);
    else
      k_tile_count<false, kTileLarge><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, sums, sl, ru);
  } else {
    if (all)
      k_tile_count<true, 1><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, sums, sl, 0);
    else
      k_tile_count<false, 1><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, sums, sl, ru);
  }
  k_tile_scan<<<1, 1024, 0, s>>>(sums, pre, nt + 1, sl, ru);
  if (per == kTileLarge) {
    if (all)
      k_tile_emit<true, kTileLarge><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, pre, g->wl,
                                                       g->steps, g->split, g->ctl, sl, 0);
    else
      k_tile_emit<false, kTileLarge><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, pre, g->wl,
                                                        g->steps, g->split, g->ctl, sl, ru);
  } else {
    if (all)
      k_tile_emit<true, 1><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, pre, g->wl, g->steps,
                                              g->split, g->ctl, sl, 0);
    else
      k_tile_emit<false, 1><<<nt, 256, 0, s>>>(fl, g->in.deg, g->n, split, pre, g->wl, g->steps,
                                               g->split, g->ctl, sl, ru);
  }
}

// Builds the work items of the next barrier-based iteration on the graph's
// stream (see launch_items).
int build_items(dfpr_graph *g, bool all, bool reuse) {
  launch_items(g, all, reuse, g->stream);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

inline uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// The instantiated two-iteration graph for the scheme and the current rank
// parity, captured again whenever an argument of its launches changed
// (buffers regrown, parameters set).  Capture runs on a private stream; the
// graph is launched on the graph's own stream.
template <typename T, typename F>
int replay_graph(dfpr_graph *g, int mode, int blocks, size_t lds, F &launch_iteration,
                 hipGraphExec_t *out) {
  const int m = mode == kAll ? 1 : 0;
  const int par = g->cur & 1;
  uint64_t key = 1469598103934665603ull;
  for (int k = 0; k < 2; ++k) {
    RankArgs<T> A = make_args<T>(g, par ^ k, par ^ k ^ 1);
    key = fnv1a(key, &A, sizeof(A));
  }
  const void *ptrs[] = {g->steps, g->tiles, g->wl, g->flags, g->ctl, g->sync_grab,
                        g->sync_max, g->sync_len, g->split.xrow, g->out.off,
                        g->out.deg, g->out.adj, g->in.deg};
  key = fnv1a(key, ptrs, sizeof(ptrs));
  const int64_t vals[] = {blocks, (int64_t)lds, block_for(g, kLaunchSync),
                          sync_split(g), g->p.max_iters, g->n, g->cu_count,
                          (int64_t)sizeof(T)};
  key = fnv1a(key, vals, sizeof(vals));
  double tol = g->p.tol;
  key = fnv1a(key, &tol, sizeof(tol));
  if (g->replay[m][par] && g->replay_key[m][par] == key) {
    *out = g->replay[m][par];
    return DFPR_OK;
  }
  if (g->replay[m][par]) {
    DFPR_HIP(hipGraphExecDestroy(g->replay[m][par]));
    g->replay[m][par] = nullptr;
  }
  if (!g->capture_stream)
    DFPR_HIP(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
  hipStream_t cs = g->capture_stream;
  DFPR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  launch_iteration(par, cs, nullptr, nullptr);
  launch_iteration(par ^ 1, cs, nullptr, nullptr);
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(cs, &graph);
  const hipError_t e0 = hipGetLastError();
  if (e1 != hipSuccess || e0 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(DFPR_EHIP, std::string("graph capture: ") +
                               hipGetErrorString(e1 != hipSuccess ? e1 : e0));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(DFPR_EHIP, std::string("graph instantiate: ") +
                                                   hipGetErrorString(e2));
  g->replay[m][par] = exec;
  g->replay_key[m][par] = key;
  *out = exec;
  return DFPR_OK;
}

template <typename T>
int run_sync(dfpr_graph *g, int mode, dfpr_stats *st) {
  hipStream_t s = g->stream;
  const int iters = g->p.max_iters;
  if (mode != kAll) {
    // the Jacobi target starts equal to the current vectors
    DFPR_HIP(hipMemcpyAsync(g->R[1 - g->cur], g->R[g->cur], (size_t)g->n * g->elem,
                            hipMemcpyDeviceToDevice, s));
    DFPR_HIP(hipMemcpyAsync(g->C[1 - g->cur], g->C[g->cur], (size_t)g->n * g->elem,
                            hipMemcpyDeviceToDevice, s));
  }
  {
    int rc = ensure_split(g);
    if (rc) return rc;
    if ((rc = build_items(g, mode == kAll, false))) return rc;
  }
  k_sync_begin<<<4, 256, 0, s>>>(g->ctl, g->sync_max, g->sync_grab, g->sync_len, iters);
  DFPR_HIP(hipGetLastError());
  auto kern = mode == kAll ? k_sync_iter<T, kAll> : k_sync_iter<T, kSyncDF>;
  const int block = block_for(g, kLaunchSync);
  const size_t lds = lds_bytes<T>(block);
  int blocks = persistent_blocks(g, kern, lds, block);
  if (g->p.grid_blocks <= 0) {
    // no more wavefronts than an iteration can have items (tiles, edge
    // steps, pieces), and at most kSyncWavesPerCU per CU: measured on the
    // 2^22 R-MAT with the pipelined gather, 12 per CU beat 8, 10, 14 and 16
    const int wpb = block / kWave;
    const int64_t items = 2 * (((int64_t)g->n + kRows - 1) / kRows) +
                          g->in.adj_cap / kStepEdges + 1 + g->split.pcap;
    int64_t want = (items + wpb - 1) / wpb;
    const int64_t cap = (int64_t)kSyncWavesPerCU * (g->cu_count > 0 ? g->cu_count : 1) / wpb;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    if (want < blocks) blocks = (int)want;
  }
  const int xgrid = g->cu_count > 0 ? g->cu_count : 1;
  const int poll = 8;
  // one iteration's launches on stream q: rank kernel, deferred out-rows,
  // next items, convergence decision (iteration index on the device)
  auto launch_iteration = [&](int parity, hipStream_t q, hipEvent_t e0, hipEvent_t e1) {
    RankArgs<T> A = make_args<T>(g, parity, parity ^ 1);
    if (e0) (void)hipEventRecord(e0, q);
    kern<<<blocks, block, lds, q>>>(A, g->steps);
    if (e1) (void)hipEventRecord(e1, q);
    if (mode != kAll) {
      k_expand_long<<<xgrid, 256, 0, q>>>(g->split.xrow, g->out.off, g->out.deg,
                                          g->out.adj, g->flags, g->ctl, g->sync_grab);
      launch_items(g, false, true, q);
    }
    k_sync_finish<<<1, 64, 0, q>>>(g->ctl, g->sync_max, g->sync_len, g->sync_grab,
                                   g->p.tol, iters, mode == kSyncDF);
  };
  const bool replay = g->p.graph_replay == 1 ||
                      (g->p.graph_replay == 2 && g->in.adj_cap <= (int64_t(1) << 22));
  hipGraphExec_t exec = nullptr;
  if (replay && replay_graph<T>(g, mode, blocks, lds, launch_iteration, &exec) != DFPR_OK) {
    // a capture can fail when other threads drive the device meanwhile;
    // replay only saves launch overhead, so the iterations run launched
    // one by one instead (nothing captured has run)
    (void)hipGetLastError();
    exec = nullptr;
  }
  if (!exec) {
    while ((int)g->iter_ev.size() < 2 * iters) {
      hipEvent_t e = nullptr;
      DFPR_HIP(hipEventCreate(&e));
      g->iter_ev.push_back(e);
    }
  }
  DFPR_HIP(hipEventRecord(g->ev[1], s));
  int it = 0;
  if (exec) {
    // two iterations per replay, the host polls every `poll` iterations
    for (; it < iters; it += 2) {
      DFPR_HIP(hipGraphLaunch(exec, s));
      if ((it + 2) % poll == 0 || it + 2 >= iters) {
        DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        DFPR_HIP(hipStreamSynchronize(s));
        if (g->h_ctl->sync_done) break;
      }
    }
  } else {
    for (; it < iters; ++it) {
      launch_iteration((g->cur + it) & 1, s, g->iter_ev[2 * it], g->iter_ev[2 * it + 1]);
      if ((it + 1) % poll == 0 || it + 1 == iters) {
        DFPR_HIP(hipGetLastError());
        DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        DFPR_HIP(hipStreamSynchronize(s));
        if (g->h_ctl->sync_done) break;
      }
    }
  }
  DFPR_HIP(hipEventRecord(g->ev[2], s));
  k_slot_totals<<<1, 64, 0, s>>>(g->sync_grab, g->ctl);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const Ctl h = *g->h_ctl;
  const int final_it = h.sync_final;
  double md = 0.0;
  if (final_it > 0) {
    unsigned long long bits = 0;
    DFPR_HIP(hipMemcpy(&bits, g->sync_max + (final_it - 1), 8, hipMemcpyDeviceToHost));
    std::memcpy(&md, &bits, 8);
  }
  g->cur = (g->cur + final_it) & 1;
  g->last_bytes = algorithmic_bytes(g, h);
  g->last_launches = final_it;
  if (st) {
    st->sweeps = final_it;
    st->converged = h.sync_conv;
    st->vertices_processed = (int64_t)h.vertices;
    st->edges_gathered = (int64_t)h.edges;
    st->out_edges_scanned = (int64_t)h.out_scanned;
    st->max_delta = md;
    // the iteration kernels alone (the item building between them is not
    // included); iterations after the last one exit at once.  Replayed
    // loops: the whole loop.
    float ms = 0.f;
    if (exec) {
      (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[2]);
    } else {
      for (int i = 0; i < final_it; ++i) {
        float x = 0.f;
        (void)hipEventElapsedTime(&x, g->iter_ev[2 * i], g->iter_ev[2 * i + 1]);
        ms += x;
      }
    }
    st->ms_kernel = ms;
  }
  if (h.abort) return fail(DFPR_EABORT, "an iteration left work items unprocessed "
                                       "(every workgroup stopped by an injected fault)");
  return h.sync_conv ? DFPR_OK : DFPR_NOTCONVERGED;
}

}  // namespace


// Entries the lock-free worklist can hold at once: every piece, and every
// group in its parts.  A group with s in-edges below the piece threshold
// takes 2^l parts, 2^l < 2 * ceil(s / kPartEdges), so all groups together
// take fewer than 2 * (ngroups + in-edge slots / kPartEdges).
int64_t worklist_cap(const dfpr_graph *g) {
  return 2 * ((int64_t)g->ngroups + g->in.adj_cap / kPartEdges) + g->split.pcap + 16;
}

// Sizes the piece arrays for the current adjacency capacities and
// threshold: a row with at least split_min entries holds that many slots,
// so at most adj_cap / split_min in-rows are long (with at most
// adj_cap / kPiece + (long rows) pieces), and at most out adj_cap /
// split_min out-rows can be deferred in one iteration.  The lock-free
// scheme's worklist holds every group and every piece.
int ensure_split(dfpr_graph *g) {
  Split &S = g->split;
  const int32_t lmin = async_split(g) < sync_split(g) ? async_split(g) : sync_split(g);
  int64_t lcap = g->in.adj_cap / lmin + 1;
  if (lcap > (int64_t)g->n + 1) lcap = (int64_t)g->n + 1;
  const int64_t pcap = g->in.adj_cap / kPiece + lcap + 1;
  int64_t xcap = g->out.adj_cap / sync_split(g) + 1;
  if (xcap > (int64_t)g->n + 1) xcap = (int64_t)g->n + 1;
  if (lcap > S.lcap || pcap > S.pcap || xcap > S.xcap) {
    DFPR_HIP(hipStreamSynchronize(g->stream));
    void *old[] = {S.lrow, S.lpre, S.lcnt, S.prow, S.ppart, S.ptag, S.xrow};
    for (void *p : old)
      if (p) DFPR_HIP(hipFree(p));
    S = Split();
    DFPR_HIP(hipMalloc(&S.lrow, (size_t)lcap * 4));
    DFPR_HIP(hipMalloc(&S.lpre, (size_t)(lcap + 1) * 4));
    DFPR_HIP(hipMalloc(&S.lcnt, (size_t)lcap * 4));
    DFPR_HIP(hipMalloc(&S.prow, (size_t)pcap * 4));
    DFPR_HIP(hipMalloc(&S.ppart, (size_t)pcap * 8));
    DFPR_HIP(hipMalloc(&S.ptag, (size_t)pcap * 4));
    DFPR_HIP(hipMalloc(&S.xrow, (size_t)xcap * 4));
    DFPR_HIP(hipMemsetAsync(S.lcnt, 0, (size_t)lcap * 4, g->stream));
    DFPR_HIP(hipMemsetAsync(S.ptag, 0, (size_t)pcap * 4, g->stream));
    S.lcap = lcap;
    S.pcap = pcap;
    S.xcap = xcap;
  }
  const int64_t gneed = worklist_cap(g);
  if (gneed > g->gwl_cap) {
    DFPR_HIP(hipStreamSynchronize(g->stream));
    if (g->gwl) DFPR_HIP(hipFree(g->gwl));
    g->gwl = nullptr;
    g->gwl_cap = 0;
    DFPR_HIP(hipMalloc(&g->gwl, (size_t)gneed * 4));
    DFPR_HIP(hipMemsetAsync(g->gwl, 0xFF, (size_t)gneed * 4, g->stream));
    g->gwl_cap = gneed;
  }
  return DFPR_OK;
}

// True when ensure_split would allocate nothing.
bool split_ready(const dfpr_graph *g) {
  const Split &S = g->split;
  const int32_t lmin = async_split(g) < sync_split(g) ? async_split(g) : sync_split(g);
  int64_t lcap = g->in.adj_cap / lmin + 1;
  if (lcap > (int64_t)g->n + 1) lcap = (int64_t)g->n + 1;
  const int64_t pcap = g->in.adj_cap / kPiece + lcap + 1;
  int64_t xcap = g->out.adj_cap / sync_split(g) + 1;
  if (xcap > (int64_t)g->n + 1) xcap = (int64_t)g->n + 1;
  return lcap <= S.lcap && pcap <= S.pcap && xcap <= S.xcap && worklist_cap(g) <= g->gwl_cap;
}

namespace {

// Every vertex affected, with its out-row counted as marked (nothing to
// expand) and every group listed: the lock-free static and naive-dynamic
// runs.
__global__ void k_mark_all(uint32_t *flags, int64_t fwords, uint32_t *gflags,
                           int64_t gwords) {
  const uint32_t fv = (kVA | kEX) * 0x01010101u;
  const uint32_t gv = kGA * 0x01010101u;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < fwords;
       i += (int64_t)gridDim.x * blockDim.x) {
    flags[i] = fv;
    if (i < gwords) gflags[i] = gv;
  }
}

// all: every vertex is affected (lock-free static / naive-dynamic,
// Algorithms 4 and 6).  Otherwise the DF update of the pending marks
// (Algorithm 2).  Either way the launch ends after a full sweep in which
// no vertex moved by more than the frontier tolerance.
template <typename T>
int run_async(dfpr_graph *g, dfpr_stats *st, bool all = false) {
  hipStream_t s = g->stream;
  {
    int rc = ensure_split(g);
    if (rc) return rc;
  }
  ++g->async_epoch;
  k_async_begin<<<1, 64, 0, s>>>(g->ctl);
  if (all) {
    // flag bytes past n in the last word and group bytes past the last
    // group stay harmless: no kernel reads a flag of an id >= n, and the
    // group list is built from the first ngroups bytes only
    const int64_t fwords = ((int64_t)g->n + 3) / 4;
    const int64_t gwords = ((int64_t)g->ngroups + 3) / 4;
    k_mark_all<<<grid_for(fwords, g->cu_count), 256, 0, s>>>(g->flags, fwords, g->gflags,
                                                             gwords);
  }
  k_group_parts<<<grid_for((int64_t)g->ngroups * kWave, g->cu_count), 256, 0, s>>>(
      g->gflags, g->in.deg, g->n, g->ngroups, async_split(g));
  k_list_long<<<grid_for(g->n, g->cu_count), 256, 0, s>>>(
      g->flags, g->in.deg, g->n, async_split(g), g->ctl, g->split, g->gwl);
  k_list_groups<<<1, 256, 0, s>>>(g->gflags, g->ngroups, g->gwl, g->ctl,
                                  degree_sorted(g) ? kGroupStripes : 1);
  DFPR_HIP(hipGetLastError());
  RankArgs<T> A = make_args<T>(g, g->cur, g->cur);
  A.split_min = async_split(g);
  // DF and DT updates stop by the lf_stop rule (make_args); the whole-set
  // runs (lock-free static and naive-dynamic) always at the frontier
  // tolerance
  if (all) A.wtol = A.ftol;
  // grid from the groups listed by the marking (kChunksPerWave)
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const int block = block_for(g, kLaunchAsync);
  const int waves_per_block = block / kWave;
  const size_t lds = lds_bytes<T>(block);
  int blocks = persistent_blocks(g, k_df_async<T>, lds, block);
  if (g->p.grid_blocks <= 0) {
    const long long want =
        async_blocks(claim_chunks(g, g->h_ctl->gtail), g->cu_count, waves_per_block);
    if (want < blocks) blocks = (int)want;
  }
  DFPR_HIP(hipEventRecord(g->ev[1], s));
  k_df_async<T><<<blocks, block, lds, s>>>(A);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipEventRecord(g->ev[2], s));
  k_zero_lcnt<<<grid_for(g->split.lcap, g->cu_count), 256, 0, s>>>(g->split.lcnt, g->ctl);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const Ctl h = *g->h_ctl;
  const int sweeps = (int)((h.state >> kSweepShift) & kSweepMask);
  const bool capped = (h.state & kCapped) != 0;
  g->last_bytes = algorithmic_bytes(g, h);
  g->last_launches = 1;
  if (st) {
    st->sweeps = sweeps;
    st->converged = (h.state & kDone) && !capped && !h.abort;
    st->vertices_processed = (int64_t)h.vertices;
    st->edges_gathered = (int64_t)h.edges;
    st->out_edges_scanned = (int64_t)h.out_scanned;
    st->max_delta = -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[2]);
    st->ms_kernel = ms;
  }
  if (h.abort) return fail(DFPR_EABORT, "persistent kernel watchdog fired");
  if (!(h.state & kDone))
    return fail(DFPR_EABORT, "every workgroup stopped before the update converged");
  return capped ? DFPR_NOTCONVERGED : DFPR_OK;
}

template <typename T>
int renormalize(dfpr_graph *g) {
  hipStream_t s = g->stream;
  DFPR_HIP(hipMemsetAsync(&g->ctl->sum, 0, sizeof(double), s));
  k_sum<T><<<grid_for(g->n, g->cu_count), 256, 0, s>>>(g->n, (const T *)g->R[g->cur],
                                                       &g->ctl->sum);
  k_scale<T><<<grid_for(g->n, g->cu_count), 256, 0, s>>>(
      g->n, g->out.deg, &g->ctl->sum, (double)g->n * g->p.tol, (T *)g->R[g->cur],
      (T *)g->C[g->cur]);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

int finish_update(dfpr_graph *g) {
  hipStream_t s = g->stream;
  unsigned long long len = g->h_ctl->tail;
  if (len > 0)
    k_cleanup<<<grid_for((int64_t)len, g->cu_count), 256, 0, s>>>(g->flags, g->wl, len);
  const unsigned long long glen = g->h_ctl->gtail;
  if (glen > 0) {
    k_cleanup_groups<<<grid_for((int64_t)glen, g->cu_count), 256, 0, s>>>(
        g->gflags, g->flags, g->gwl, glen, g->n);
  }
  // the marking lists groups in both schemes; only the lock-free one
  // builds and clears the group worklist
  const int64_t gwords = ((int64_t)g->ngroups + 3) / 4;
  k_zero_bytes<<<grid_for(gwords, g->cu_count), 256, 0, s>>>(g->gflags, gwords);
  k_reset_marks<<<1, 64, 0, s>>>(g->ctl);
  DFPR_HIP(hipGetLastError());
  g->pending_marks = 0;
  return DFPR_OK;
}

}  // namespace

int init_uniform_ranks(dfpr_graph *g) {
  hipStream_t s = g->stream;
  const int b = grid_for(g->n, g->cu_count);
  if (g->elem == 8)
    k_uniform<double><<<b, 256, 0, s>>>(g->n, g->out.deg, (double *)g->R[g->cur],
                                        (double *)g->C[g->cur]);
  else
    k_uniform<float><<<b, 256, 0, s>>>(g->n, g->out.deg, (float *)g->R[g->cur],
                                       (float *)g->C[g->cur]);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

int refresh_contributions(dfpr_graph *g) {
  hipStream_t s = g->stream;
  const int b = grid_for(g->n, g->cu_count);
  if (g->elem == 8)
    k_contrib<double><<<b, 256, 0, s>>>(g->n, g->out.deg, (const double *)g->R[g->cur],
                                        (double *)g->C[g->cur]);
  else
    k_contrib<float><<<b, 256, 0, s>>>(g->n, g->out.deg, (const float *)g->R[g->cur],
                                       (float *)g->C[g->cur]);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

int set_ranks_device(dfpr_graph *g, const double *r) {
  hipStream_t s = g->stream;
  const int b = grid_for(g->n, g->cu_count);
  if (g->elem == 8)
    k_ranks_in<double><<<b, 256, 0, s>>>(g->n, g->int2ext, r, (double *)g->R[g->cur]);
  else
    k_ranks_in<float><<<b, 256, 0, s>>>(g->n, g->int2ext, r, (float *)g->R[g->cur]);
  DFPR_HIP(hipGetLastError());
  return refresh_contributions(g);
}

int read_ranks_device(const dfpr_graph *g, double *out) {
  hipStream_t s = g->stream;
  const int b = grid_for(g->n, g->cu_count);
  if (g->elem == 8)
    k_ranks_out<double><<<b, 256, 0, s>>>(g->n, g->int2ext, (const double *)g->R[g->cur], out);
  else
    k_ranks_out<float><<<b, 256, 0, s>>>(g->n, g->int2ext, (const float *)g->R[g->cur], out);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

// mode: kAll for static / naive-dynamic, otherwise the graph's own mode.
int run_rank(dfpr_graph *g, int kind, dfpr_stats *st) {
  hipStream_t s = g->stream;
  DFPR_HIP(hipEventRecord(g->ev[0], s));
  int rc;
  if (kind == 0 || kind == 1) {  // static (restart) / naive-dynamic
    if (kind == 0) {
      rc = init_uniform_ranks(g);
      if (rc) return rc;
    }
    rc = g->elem == 8 ? run_sync<double>(g, kAll, st) : run_sync<float>(g, kAll, st);
  } else if (kind == 3 || kind == 4) {  // the same, lock-free
    if (kind == 3) {
      rc = init_uniform_ranks(g);
      if (rc) return rc;
    }
    rc = g->elem == 8 ? run_async<double>(g, st, true) : run_async<float>(g, st, true);
    if (st) {
      st->initial_marked = g->n;
      st->affected = g->n;
    }
    // every vertex was recomputed: batches applied before are served too
    int rc2 = finish_update(g);
    if (rc2) return rc2;
  } else {
    if (kind == 5) {
      // Dynamic Traversal: the closure of the marks, then the update over
      // it (every marked vertex has its out-row walked, so nothing grows)
      rc = mark_reachable(g, nullptr);
      if (rc) return rc;
    }
    if (g->pending_marks == 0) {
      // nothing affected: ranks stay bit-identical
      g->last_bytes = 0;
      g->last_launches = 0;
      if (st) {
        *st = dfpr_stats{};
        st->converged = 1;
        st->max_delta = 0.0;
      }
      return DFPR_OK;
    }
    if (g->p.mode == DFPR_SYNC)
      rc = g->elem == 8 ? run_sync<double>(g, kSyncDF, st) : run_sync<float>(g, kSyncDF, st);
    else
      rc = g->elem == 8 ? run_async<double>(g, st) : run_async<float>(g, st);
    if (rc < 0) {
      (void)finish_update(g);
      return rc;
    }
    if (st) {
      st->initial_marked = (int64_t)g->h_ctl->marked;
      st->affected = g->p.mode == DFPR_SYNC
                         ? (int64_t)g->h_ctl->tail
                         : (int64_t)g->h_ctl->marked + (int64_t)g->h_ctl->newly;
    }
    int rc2 = finish_update(g);
    if (rc2) return rc2;
  }
  if (rc < 0) return rc;
  if (g->elem == 4 && g->p.renormalize) {
    int rc3 = renormalize<float>(g);
    if (rc3) return rc3;
  }
  DFPR_HIP(hipEventRecord(g->ev[3], s));
  DFPR_HIP(hipEventSynchronize(g->ev[3]));
  if (st) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[3]);
    st->ms = ms;
  }
  return rc;
}

namespace {

// Buffers of one batched launch: device memory for the descriptors, the
// summaries and the done counter, and host staging for the same.  The
// regular entry point grows them on demand; the allocation-free one passes
// fixed arrays.
template <typename T>
struct ManyWork {
  void *dev = nullptr;  // device bytes >= count * (descriptor + summary) + 256
  RankArgs<T> *hdesc = nullptr;
  Summary *hsum = nullptr;
  dfpr_graph **act = nullptr;
};

template <typename T>
int update_many_t(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats,
                  const ManyWork<T> &W) {
  dfpr_graph **act = W.act;
  int na = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (stats) {
      stats[i] = dfpr_stats{};
      stats[i].converged = 1;
    }
    if (gs[i]->pending_marks > 0) act[na++] = gs[i];
  }
  if (na == 0) return DFPR_OK;
  dfpr_graph *g0 = act[0];
  hipStream_t s = g0->stream;
  for (int i = 0; i < na; ++i)
    if (act[i]->stream != s) DFPR_HIP(hipStreamSynchronize(act[i]->stream));
  for (int i = 0; i < na; ++i) ++act[i]->async_epoch;
  RankArgs<T> *h = W.hdesc;
  for (int i = 0; i < na; ++i) {
    h[i] = make_args<T>(act[i], act[i]->cur, act[i]->cur);
    h[i].split_min = async_split(act[i]);
    h[i].chunk = effective_chunk(act[i], kLaunchMany);
  }
  // device copies: descriptors, summaries, the done counter (set to 0 by
  // k_begin_many, so nothing needs clearing beforehand)
  const size_t dbytes = sizeof(RankArgs<T>) * na;
  const size_t sbytes = sizeof(Summary) * na;
  void *buf = W.dev;
  RankArgs<T> *d_desc = (RankArgs<T> *)buf;
  Summary *d_sum = (Summary *)((char *)buf + dbytes);
  int *d_done = (int *)((char *)buf + dbytes + sbytes + 128);
  DFPR_HIP(hipMemcpyAsync(d_desc, h, dbytes, hipMemcpyHostToDevice, s));
  const int gb = grid_for(na, g0->cu_count);
  k_begin_many<T><<<gb, 256, 0, s>>>(d_desc, na, d_done);
  k_group_parts_many<T><<<na < g0->cu_count * 8 ? na : g0->cu_count * 8, 256, 0, s>>>(d_desc,
                                                                                        na);
  k_list_long_many<T><<<na < g0->cu_count * 8 ? na : g0->cu_count * 8, 256, 0, s>>>(d_desc,
                                                                                      na);
  k_list_groups_many<T><<<na < g0->cu_count * 8 ? na : g0->cu_count * 8, 256, 0, s>>>(d_desc,
                                                                                        na);
  k_gather_summary<T><<<gb, 256, 0, s>>>(d_desc, na, d_sum);
  Summary *hs = W.hsum;
  DFPR_HIP(hipMemcpyAsync(hs, d_sum, sbytes, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  long long chunks = 0;
  for (int i = 0; i < na; ++i) chunks += claim_chunks(act[i], hs[i].gtail, kLaunchMany);
  const int block = block_for(g0, kLaunchMany);
  const int wpb = block / kWave;
  const size_t lds = lds_bytes<T>(block);
  int blocks = persistent_blocks(g0, k_df_async_many<T>, lds, block);
  if (g0->p.grid_blocks <= 0) {
    const long long want = async_blocks(chunks, g0->cu_count, wpb);
    if (want < blocks) blocks = (int)want;
  }
  const unsigned long long ticks =
      g0->p.timeout_ms > 0 ? (unsigned long long)g0->p.timeout_ms * (unsigned long long)g0->wallclock_khz
                           : 0ull;
  DFPR_HIP(hipEventRecord(g0->ev[0], s));
  k_df_async_many<T><<<blocks, block, lds, s>>>(d_desc, na, d_done, &g0->ctl->abort,
                                                         ticks);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipEventRecord(g0->ev[1], s));
  k_gather_summary<T><<<gb, 256, 0, s>>>(d_desc, na, d_sum);
  DFPR_HIP(hipMemcpyAsync(hs, d_sum, sbytes, hipMemcpyDeviceToHost, s));
  k_cleanup_many<T><<<na < g0->cu_count * 8 ? na : g0->cu_count * 8, 256, 0, s>>>(d_desc, na);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipStreamSynchronize(s));
  float kms = 0.f;
  (void)hipEventElapsedTime(&kms, g0->ev[0], g0->ev[1]);
  int worst = DFPR_OK;
  bool aborted = false;
  for (int i = 0, j = 0; i < count; ++i) {
    if (gs[i]->pending_marks <= 0) continue;
    dfpr_graph *g = gs[i];
    const Summary &x = hs[j++];
    Ctl c{};
    c.vertices = x.vertices;
    c.edges = x.edges;
    c.out_scanned = x.out_scanned;
    g->last_bytes = algorithmic_bytes(g, c);
    g->last_launches = 1;
    g->pending_marks = 0;
    const bool capped = (x.state & kCapped) != 0;
    aborted = aborted || x.abort;
    if (capped && worst == DFPR_OK) worst = DFPR_NOTCONVERGED;
    if (stats) {
      dfpr_stats &st = stats[i];
      st.sweeps = (int)((x.state >> kSweepShift) & kSweepMask);
      st.converged = !capped && !x.abort;
      st.initial_marked = x.marked;
      st.affected = x.marked + x.newly;
      st.vertices_processed = (long long)x.vertices;
      st.edges_gathered = (long long)x.edges;
      st.out_edges_scanned = (long long)x.out_scanned;
      st.max_delta = -1.0;
      st.ms_kernel = kms;
      st.ms = kms;
    }
    if (g->elem == 4 && g->p.renormalize) {
      int r2 = renormalize<float>(g);
      if (r2) return r2;
    }
  }
  if (aborted) return fail(DFPR_EABORT, "batched persistent kernel watchdog fired");
  return worst;
}

}  // namespace

namespace {

int check_many(dfpr_graph *const *gs, int32_t count) {
  const int elem = gs[0]->elem;
  const int dev = gs[0]->device;
  for (int32_t i = 0; i < count; ++i) {
    if (gs[i]->elem != elem) return fail(DFPR_EINVAL, "graphs mix fp32 and fp64 ranks");
    if (gs[i]->device != dev) return fail(DFPR_EINVAL, "graphs live on different devices");
    for (int32_t j = 0; j < i; ++j)
      if (gs[j] == gs[i]) return fail(DFPR_EINVAL, "a graph appears twice");
  }
  return DFPR_OK;
}

int sync_fp32(dfpr_graph *const *gs, int32_t count, int rc) {
  if (rc >= 0 && gs[0]->elem == 4) {
    for (int32_t i = 0; i < count; ++i) DFPR_HIP(hipStreamSynchronize(gs[i]->stream));
  }
  return rc;
}

}  // namespace

int update_many(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats) {
  if (count == 0) return DFPR_OK;
  int rc = check_many(gs, count);
  if (rc) return rc;
  for (int32_t i = 0; i < count; ++i)
    if (gs[i]->pending_marks > 0 && (rc = ensure_split(gs[i]))) return rc;
  std::vector<dfpr_graph *> act((size_t)count);
  std::vector<Summary> hsum((size_t)count);
  const size_t bytes = (sizeof(RankArgs<double>) + sizeof(Summary)) * (size_t)count + 256;
  void *dev = nullptr;
  if ((rc = scratch_get(gs[0], 12, bytes, &dev))) return rc;
  if (gs[0]->elem == 8) {
    std::vector<RankArgs<double>> hd((size_t)count);
    rc = update_many_t<double>(gs, count, stats,
                               ManyWork<double>{dev, hd.data(), hsum.data(), act.data()});
  } else {
    std::vector<RankArgs<float>> hd((size_t)count);
    rc = update_many_t<float>(gs, count, stats,
                              ManyWork<float>{dev, hd.data(), hsum.data(), act.data()});
  }
  return sync_fp32(gs, count, rc);
}

}  // namespace dfpr

// --- the batched launch without allocation --------------------------------------
//
// Device workspace of dfpr_update_many_noalloc: a fixed array in the code
// object, one copy per device, held until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in).
namespace {
constexpr int32_t kNoAllocMaxGraphs = DFPR_NOALLOC_MAX_GRAPHS;
constexpr size_t kNoAllocBytes =
    (sizeof(dfpr::RankArgs<double>) + sizeof(dfpr::Summary)) * kNoAllocMaxGraphs + 256;
static_assert(sizeof(dfpr::RankArgs<double>) == sizeof(dfpr::RankArgs<float>),
              "descriptors of both precisions share the workspace layout");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace dfpr {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;       // one allocation-free call at a time
void *g_noalloc_dev[kMaxDevices];  // scratch's address per device
// host staging, fixed size
alignas(64) unsigned char g_noalloc_hdesc[sizeof(RankArgs<double>) * kNoAllocMaxGraphs];
Summary g_noalloc_hsum[kNoAllocMaxGraphs];
dfpr_graph *g_noalloc_act[kNoAllocMaxGraphs];

// scratch's device address on `dev` (current), looked up once per device
int noalloc_workspace(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DFPR_EINVAL, "device index out of range");
  if (!g_noalloc_dev[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DFPR_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e));
    g_noalloc_dev[dev] = ptr;
  }
  *out = g_noalloc_dev[dev];
  return DFPR_OK;
}

}  // namespace

int update_many_noalloc(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats) {
  if (count > kNoAllocMaxGraphs)
    return fail(DFPR_EINVAL, "dfpr_update_many_noalloc takes at most " +
                                 std::to_string(kNoAllocMaxGraphs) + " graphs");
  if (count == 0) return DFPR_OK;
  int rc = check_many(gs, count);
  if (rc) return rc;
  for (int32_t i = 0; i < count; ++i)
    if (gs[i]->pending_marks > 0 && !split_ready(gs[i]))
      return fail(DFPR_ESTATE, "piece arrays of a graph are not sized for its adjacency");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  const int dev = gs[0]->device;
  int cur = -1;
  DFPR_HIP(hipGetDevice(&cur));
  if (cur != dev) DFPR_HIP(hipSetDevice(dev));
  void *ws = nullptr;
  rc = noalloc_workspace(dev, &ws);
  if (rc == DFPR_OK) {
    if (gs[0]->elem == 8)
      rc = update_many_t<double>(
          gs, count, stats,
          ManyWork<double>{ws, reinterpret_cast<RankArgs<double> *>(g_noalloc_hdesc),
                           g_noalloc_hsum, g_noalloc_act});
    else
      rc = update_many_t<float>(
          gs, count, stats,
          ManyWork<float>{ws, reinterpret_cast<RankArgs<float> *>(g_noalloc_hdesc),
                          g_noalloc_hsum, g_noalloc_act});
    rc = sync_fp32(gs, count, rc);
  }
  if (cur != dev) {
    const hipError_t e = hipSetDevice(cur);
    if (e != hipSuccess && rc >= 0) return fail(DFPR_EHIP, hipGetErrorString(e));
  }
  return rc;
}

int stream_copy(void *dst, const void *src, int64_t bytes, hipStream_t s,
                float *ms) {
  int dev = 0, cu = 0;
  DFPR_HIP(hipGetDevice(&dev));
  DFPR_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t a, b;
  DFPR_HIP(hipEventCreate(&a));
  DFPR_HIP(hipEventCreate(&b));
  DFPR_HIP(hipEventRecord(a, s));
  const int64_t n16 = bytes / 16;
  if (n16 > 0)
    k_copy16<<<cu * 8, 256, 0, s>>>((const int4 *)src, (int4 *)dst, n16);
  const int64_t rem = bytes - n16 * 16;
  if (rem > 0)
    k_copy1<<<1, 256, 0, s>>>((const uint8_t *)src + n16 * 16, (uint8_t *)dst + n16 * 16, rem);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipEventRecord(b, s));
  DFPR_HIP(hipEventSynchronize(b));
  float t = 0.f;
  (void)hipEventElapsedTime(&t, a, b);
  if (ms) *ms = t;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return DFPR_OK;
}

}  // namespace dfpr
