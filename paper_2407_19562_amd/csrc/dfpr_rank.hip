// Rank iteration kernels: the gather of Eq. 1, frontier expansion and
// convergence (Section 4; Algorithms 1 and 2), plus static / naive-dynamic
// PageRank (Algorithm 3; Section 3.5.1) and small helpers.
//
// Work unit: one wavefront takes a group of 64 worklist positions (or 64
// consecutive vertex ids in a dense sweep), one vertex per lane.
//   gather: a lane sums its own in-row when the in-degree is below
//     wave_min_degree (16-byte index loads, two accumulators); rows at or
//     above it are gathered by the whole wavefront, one row at a time,
//     64 lanes striding the row and a shuffle reduction.  The sum reads the
//     contributions C[u] = R[u] / (out-degree(u) + 1), so one random 4- or
//     8-byte load per in-edge; the implicit self-loop adds C[v].
//   update: r = (1 - alpha)/n + alpha * sum, dr = |r - R[v]|.
//   frontier (dr > frontier_tol): every out-neighbour gets the affected
//     flag (and, in the lock-free scheme, the not-converged flag); newly
//     affected vertices are appended with one atomic per wavefront.
//   convergence: lock-free scheme -- R_C[v] = (dr > tol) and a global count
//     of set R_C flags; barrier-based scheme -- max dr per iteration.
//
// Scheduling:
//   k_df_async   one persistent launch.  A single 64-bit word holds the
//                sweep index, a cursor into the current sweep's index space
//                and the number of wavefronts holding a chunk.  Wavefronts
//                grab chunks with fetch_add; the first to find the cursor at
//                the end either starts the next sweep (some R_C still set)
//                or, when no R_C is set and no chunk is held, ends the
//                launch.  No grid barrier exists anywhere: sweeps overlap
//                and ranks are updated in place (Algorithm 2's scheme).
//   k_sync_iter  one launch per iteration reading R/C and writing the other
//                buffer (Algorithm 1); k_sync_finish ends the loop on the
//                device so the host only polls every few iterations.
#include <cmath>
#include <cstring>

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
  Ctl *ctl;
  double alpha, base, tol, ftol;
  int32_t wave_min, kahan_min, chunk, dense_div, max_iters;
  unsigned long long timeout_ticks;
  unsigned long long *sync_max;
  unsigned long long *sync_grab;
  unsigned long long *sync_len;
};

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

// --- per-lane gather over a light in-row -------------------------------------

template <bool COH>
__device__ __forceinline__ double gather_lane(const double *C,
                                              const int32_t *row, int32_t deg,
                                              bool) {
  double s0 = 0.0, s1 = 0.0;
  int32_t k = 0;
  for (; k + 4 <= deg; k += 4) {
    const int4 q = *reinterpret_cast<const int4 *>(row + k);
    const double a = ldc<double, COH>(C, q.x), b = ldc<double, COH>(C, q.y);
    const double c = ldc<double, COH>(C, q.z), d = ldc<double, COH>(C, q.w);
    s0 += a + b;
    s1 += c + d;
  }
  for (; k < deg; ++k) s0 += ldc<double, COH>(C, row[k]);
  return s0 + s1;
}

// fp32: plain or compensated (Kahan) single-precision sums; returns the
// compensated value widened to fp64.
template <bool COH>
__device__ __forceinline__ double gather_lane(const float *C,
                                              const int32_t *row, int32_t deg,
                                              bool kahan) {
  if (!kahan) {
    float s0 = 0.f, s1 = 0.f;
    int32_t k = 0;
    for (; k + 4 <= deg; k += 4) {
      const int4 q = *reinterpret_cast<const int4 *>(row + k);
      const float a = ldc<float, COH>(C, q.x), b = ldc<float, COH>(C, q.y);
      const float c = ldc<float, COH>(C, q.z), d = ldc<float, COH>(C, q.w);
      s0 += a + b;
      s1 += c + d;
    }
    for (; k < deg; ++k) s0 += ldc<float, COH>(C, row[k]);
    return (double)s0 + (double)s1;
  }
  float s = 0.f, comp = 0.f;
  int32_t k = 0;
  for (; k + 4 <= deg; k += 4) {
    const int4 q = *reinterpret_cast<const int4 *>(row + k);
    const float x[4] = {ldc<float, COH>(C, q.x), ldc<float, COH>(C, q.y),
                        ldc<float, COH>(C, q.z), ldc<float, COH>(C, q.w)};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float y = x[j] - comp;
      const float t = s + y;
      comp = (t - s) - y;
      s = t;
    }
  }
  for (; k < deg; ++k) {
    const float y = ldc<float, COH>(C, row[k]) - comp;
    const float t = s + y;
    comp = (t - s) - y;
    s = t;
  }
  return (double)s - (double)comp;
}

// --- whole-wavefront gather over a heavy in-row --------------------------------

template <typename T, bool COH>
__device__ __forceinline__ double gather_wave(const T *C, const int32_t *row,
                                              int32_t deg, bool kahan) {
  const int lane = lane_id();
  if constexpr (sizeof(T) == 8) {
    double s0 = 0.0, s1 = 0.0;
    int32_t k = lane;
    for (; k + 3 * kWave < deg; k += 4 * kWave) {
      const int32_t i0 = row[k], i1 = row[k + kWave];
      const int32_t i2 = row[k + 2 * kWave], i3 = row[k + 3 * kWave];
      const double a = ldc<T, COH>(C, i0), b = ldc<T, COH>(C, i1);
      const double c = ldc<T, COH>(C, i2), d = ldc<T, COH>(C, i3);
      s0 += a + b;
      s1 += c + d;
    }
    for (; k < deg; k += kWave) s0 += ldc<T, COH>(C, row[k]);
    return wave_sum(s0 + s1);
  } else {
    float s = 0.f, comp = 0.f;
    int32_t k = lane;
    for (; k + 3 * kWave < deg; k += 4 * kWave) {
      const int32_t i0 = row[k], i1 = row[k + kWave];
      const int32_t i2 = row[k + 2 * kWave], i3 = row[k + 3 * kWave];
      const float x[4] = {ldc<T, COH>(C, i0), ldc<T, COH>(C, i1),
                          ldc<T, COH>(C, i2), ldc<T, COH>(C, i3)};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (kahan) {
          const float y = x[j] - comp;
          const float t = s + y;
          comp = (t - s) - y;
          s = t;
        } else {
          s += x[j];
        }
      }
    }
    for (; k < deg; k += kWave) {
      const float xv = ldc<T, COH>(C, row[k]);
      if (kahan) {
        const float y = xv - comp;
        const float t = s + y;
        comp = (t - s) - y;
        s = t;
      } else {
        s += xv;
      }
    }
    return wave_sum((double)s - (double)comp);
  }
}

// Marks w affected (and not converged in the lock-free scheme); returns true
// when w was not affected before (the caller appends it).
template <int MODE>
__device__ __forceinline__ bool mark_vertex(uint32_t *flags, int32_t w,
                                            long long &nc) {
  if constexpr (MODE == kAsync) {
    const uint32_t b = flag_byte(flags, w, true);
    if ((b & (kVA | kRC)) == (kVA | kRC)) return false;
    const uint32_t old = flag_set(flags, w, kVA | kRC);
    nc += (old & kRC) ? 0 : 1;
    return !(old & kVA);
  } else {
    const uint32_t b = flag_byte(flags, w, false);
    if (b & kVA) return false;
    const uint32_t old = flag_set(flags, w, kVA);
    return !(old & kVA);
  }
}

// Processes one vertex per lane (v < 0: idle lane).  All 64 lanes call it.
template <typename T, int MODE>
__device__ __forceinline__ void process_group(const RankArgs<T> &A, int32_t v,
                                              Counters &cnt, double &maxdr,
                                              long long &nc) {
  constexpr bool COH = MODE == kAsync;
  const int lane = lane_id();
  const bool valid = v >= 0;
  int64_t off = 0;
  int32_t deg = 0;
  if (valid) {
    off = A.in_off[v];
    deg = A.in_deg[v];
  }
  const bool heavy = valid && deg >= A.wave_min;
  double sum = 0.0;
  if (valid && !heavy)
    sum = gather_lane<COH>(A.Cr, A.in_adj + off, deg, deg >= A.kahan_min);
  uint64_t hm = __ballot(heavy);
  while (hm) {
    const int l = __ffsll((long long)hm) - 1;
    hm &= hm - 1;
    const int64_t o = __shfl(off, l);
    const int32_t d = __shfl(deg, l);
    const double part = gather_wave<T, COH>(A.Cr, A.in_adj + o, d, d >= A.kahan_min);
    if (lane == l) sum = part;
  }

  bool expand = false;
  int32_t od = 0;
  if (valid) {
    const double selfc = (double)ldc<T, COH>(A.Cr, v);
    const double r = A.base + A.alpha * (sum + selfc);
    const T rT = (T)r;
    const T old = COH ? load_agent(A.Rr + v) : A.Rr[v];
    const double dr = fabs((double)rT - (double)old);
    od = A.out_deg[v];
    const T cT = (T)(r / (double)(od + 1));
    if constexpr (COH) {
      store_agent(A.Rw + v, rT);
      store_agent(A.Cw + v, cT);
    } else {
      A.Rw[v] = rT;
      A.Cw[v] = cT;
    }
    cnt.vertices += 1;
    cnt.edges += (unsigned long long)deg + 1;
    if constexpr (MODE != kAll) expand = dr > A.ftol;
    if constexpr (MODE == kAsync) {
      // own R_C: set while dr > tol (the self-loop re-marks it when the
      // change exceeds the frontier tolerance; the tol test clears it)
      const uint32_t b = flag_byte(A.flags, v, true);
      if (dr > A.tol) {
        if (!(b & kRC)) {
          const uint32_t o2 = flag_set(A.flags, v, kRC);
          nc += (o2 & kRC) ? 0 : 1;
        }
      } else if (b & kRC) {
        const uint32_t o2 = flag_clear(A.flags, v, kRC);
        nc -= (o2 & kRC) ? 1 : 0;
      }
    } else {
      maxdr = dr > maxdr ? dr : maxdr;
    }
  }
  if constexpr (MODE == kAll) return;

  // frontier expansion over out-rows (the self-loop is handled above)
  int64_t oo = 0;
  if (expand) oo = A.out_off[v];
  const bool oheavy = expand && od >= A.wave_min;
  const int32_t my = (expand && !oheavy) ? od : 0;
  if (expand) cnt.out_scanned += (unsigned long long)od;
  const int32_t trips = wave_max(my);
  for (int32_t k = 0; k < trips; ++k) {
    bool want = false;
    int32_t w = -1;
    if (k < my) {
      w = A.out_adj[oo + k];
      want = mark_vertex<MODE>(A.flags, w, nc);
    }
    wave_append(want, w, A.wl, &A.ctl->tail, COH);
  }
  uint64_t om = __ballot(oheavy);
  while (om) {
    const int l = __ffsll((long long)om) - 1;
    om &= om - 1;
    const int64_t o = __shfl(oo, l);
    const int32_t d = __shfl(od, l);
    for (int32_t t = 0; t < d; t += kWave) {
      bool want = false;
      int32_t w = -1;
      if (t + lane < d) {
        w = A.out_adj[o + t + lane];
        want = mark_vertex<MODE>(A.flags, w, nc);
      }
      wave_append(want, w, A.wl, &A.ctl->tail, COH);
    }
  }
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

// Sweep-end decision, lane 0 only.
template <typename T>
__device__ void sweep_end(const RankArgs<T> &A) {
  unsigned long long *st = &A.ctl->state;
  const unsigned long long W =
      __hip_atomic_load(st, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (W & kDone) return;
  const bool dense = W & kDense;
  const unsigned long long tail = load_agent(&A.ctl->tail);
  const unsigned long long bound = dense ? (unsigned long long)A.n : tail;
  const unsigned long long cur = (W >> kCursorShift) & kCursorMask;
  if (cur < bound) return;
  const unsigned long long sweep = (W >> kSweepShift) & kSweepMask;
  const unsigned long long inflight = W & kInflightMask;
  const long long nc = load_agent(&A.ctl->nc);
  unsigned long long nw;
  if (nc > 0) {
    const unsigned long long ns = sweep + 1;
    if ((long long)ns >= A.max_iters) {
      nw = kDone | kCapped | (ns << kSweepShift);
    } else {
      const bool d = dense || (A.dense_div > 0 &&
                               tail * (unsigned long long)A.dense_div >
                                   (unsigned long long)A.n);
      nw = (d ? kDense : 0ull) | (ns << kSweepShift) | inflight;
    }
  } else if (inflight == 0) {
    nw = kDone | ((sweep + 1) << kSweepShift);
  } else {
    return;
  }
  unsigned long long expect = W;
  __hip_atomic_compare_exchange_strong(st, &expect, nw, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__global__ void __launch_bounds__(256) k_df_async(RankArgs<T> A) {
  const int lane = lane_id();
  Counters cnt;
  const unsigned long long t_start = wall_clock64();
  const unsigned long long chunk = (unsigned long long)A.chunk;
  const unsigned long long grab = (chunk << kCursorShift) | 1ull;
  unsigned polls = 0;
  double unused = 0.0;
  while (true) {
    unsigned long long W = 0, tl = 0;
    int ab = 0;
    if (lane == 0) {
      W = load_agent(&A.ctl->state);
      tl = load_agent(&A.ctl->tail);
      ab = load_agent(&A.ctl->abort);
    }
    W = bcast0(W);
    tl = bcast0(tl);
    ab = __builtin_amdgcn_readfirstlane(ab);
    if ((W & kDone) || ab) break;
    const unsigned long long bound = (W & kDense) ? (unsigned long long)A.n : tl;
    if (((W >> kCursorShift) & kCursorMask) >= bound) {
      if (lane == 0) sweep_end(A);
      __builtin_amdgcn_s_sleep(2);
      if (A.timeout_ticks && ((++polls & 63u) == 0)) {
        const bool late = wall_clock64() - t_start > A.timeout_ticks;
        if (late) {
          if (lane == 0) store_agent(&A.ctl->abort, 1);
          break;
        }
      }
      continue;
    }
    unsigned long long W2 = 0;
    if (lane == 0) {
      W2 = __hip_atomic_fetch_add(&A.ctl->state, grab, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
      tl = load_agent(&A.ctl->tail);
    }
    W2 = bcast0(W2);
    tl = bcast0(tl);
    if (W2 & kDone) break;
    const bool dn = W2 & kDense;
    const unsigned long long p = (W2 >> kCursorShift) & kCursorMask;
    const unsigned long long bnd = dn ? (unsigned long long)A.n : tl;
    if (p >= bnd) {
      if (lane == 0)
        __hip_atomic_fetch_sub(&A.ctl->state, 1ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    const unsigned long long end = p + chunk < bnd ? p + chunk : bnd;
    long long nc = 0;
    for (unsigned long long g0 = p; g0 < end; g0 += kWave) {
      const unsigned long long pos = g0 + lane;
      int32_t v = -1;
      if (pos < end) {
        if (dn) {
          v = (int32_t)pos;
          if (!(flag_byte(A.flags, v, true) & kVA)) v = -1;
        } else {
          v = load_agent(A.wl + pos);
        }
      }
      process_group<T, kAsync>(A, v, cnt, unused, nc);
    }
    nc = wave_sum(nc);
    if (lane == 0) {
      if (nc)
        __hip_atomic_fetch_add(&A.ctl->nc, nc, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_sub(&A.ctl->state, 1ull, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  flush_counters<T>(A.ctl, cnt);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_sync_iter(RankArgs<T> A, int iter) {
  if (A.ctl->sync_done) return;
  const int lane = lane_id();
  Counters cnt;
  double maxdr = 0.0;
  long long nc = 0;
  const unsigned long long len =
      MODE == kAll ? (unsigned long long)A.n : A.sync_len[iter];
  const unsigned long long chunk = (unsigned long long)A.chunk;
  while (true) {
    unsigned long long p = 0;
    if (lane == 0) p = atomicAdd(&A.sync_grab[iter], chunk);
    p = bcast0(p);
    if (p >= len) break;
    const unsigned long long end = p + chunk < len ? p + chunk : len;
    for (unsigned long long g0 = p; g0 < end; g0 += kWave) {
      const unsigned long long pos = g0 + lane;
      int32_t v = -1;
      if (pos < end) v = MODE == kAll ? (int32_t)pos : A.wl[pos];
      process_group<T, MODE>(A, v, cnt, maxdr, nc);
    }
  }
  maxdr = wave_max(maxdr);
  if (lane == 0 && maxdr > 0.0)
    atomicMax(&A.sync_max[iter], (unsigned long long)__double_as_longlong(maxdr));
  flush_counters<T>(A.ctl, cnt);
}

__global__ void k_sync_finish(Ctl *ctl, const unsigned long long *sync_max,
                              unsigned long long *sync_len, int iter,
                              double tol, int max_iters, int df) {
  if (threadIdx.x != 0 || ctl->sync_done) return;
  const double md = __longlong_as_double((long long)sync_max[iter]);
  if (md <= tol || iter + 1 >= max_iters) {
    ctl->sync_done = 1;
    ctl->sync_final = iter + 1;
    ctl->pad = md <= tol ? 1 : 0;
  } else if (df) {
    sync_len[iter + 1] = ctl->tail;
  }
}

__global__ void k_sync_begin(Ctl *ctl, unsigned long long *sync_max,
                             unsigned long long *sync_grab,
                             unsigned long long *sync_len, int iters) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < iters;
       i += gridDim.x * blockDim.x) {
    sync_max[i] = 0;
    sync_grab[i] = 0;
    sync_len[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sync_len[0] = ctl->tail;
    ctl->sync_done = 0;
    ctl->sync_final = 0;
    ctl->pad = 0;
    ctl->vertices = ctl->edges = ctl->out_scanned = 0;
    ctl->abort = 0;
  }
}

__global__ void k_async_begin(Ctl *ctl, int dense) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl->state = dense ? kDense : 0ull;
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

__global__ void k_reset_marks(Ctl *ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->tail = 0;
    ctl->nc = 0;
    ctl->marked = 0;
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

template <typename T>
__global__ void k_scale(int32_t n, const int32_t *out_deg, const double *sum,
                        T *R, T *C) {
  const double f = 1.0 / *sum;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const double r = (double)R[v] * f;
    R[v] = (T)r;
    C[v] = (T)(r / (double)(out_deg[v] + 1));
  }
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

__global__ void k_copy16(const int4 *src, int4 *dst, int64_t n16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
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

template <typename T>
RankArgs<T> make_args(dfpr_graph *g, int rd, int wr) {
  RankArgs<T> A;
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
  A.ctl = g->ctl;
  A.alpha = g->p.alpha;
  A.base = (1.0 - g->p.alpha) / (double)g->n;
  A.tol = g->p.tol;
  A.ftol = g->p.frontier_tol;
  A.wave_min = g->p.wave_min_degree;
  A.kahan_min = g->p.kahan_min_degree;
  A.chunk = g->p.chunk;
  A.dense_div = g->p.dense_div;
  A.max_iters = g->p.max_iters;
  A.timeout_ticks = g->p.timeout_ms > 0
                        ? (unsigned long long)g->p.timeout_ms * (unsigned long long)g->wallclock_khz
                        : 0ull;
  A.sync_max = g->sync_max;
  A.sync_grab = g->sync_grab;
  A.sync_len = g->sync_len;
  return A;
}

// Co-resident workgroups (or the grid_blocks override).  The in-flight
// field of the scheduling word holds 16 bits, so the grid stays below 32768
// wavefronts; chunk <= 4096 keeps cursor overshoot far below 2^32.
template <typename K>
int persistent_blocks(dfpr_graph *g, K kernel) {
  int blocks = g->p.grid_blocks;
  if (blocks <= 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel,
                                                     g->p.block_size, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * g->cu_count;
  }
  const int max_blocks = 32768 / (g->p.block_size / kWave);
  return blocks > max_blocks ? max_blocks : blocks;
}

// bytes the rank iteration must move, from the device counters
double algorithmic_bytes(const dfpr_graph *g, const Ctl &h) {
  const double e = (double)h.edges - (double)h.vertices;  // stored in-edges
  if (g->elem == 8)
    return 12.0 * e + 52.0 * (double)h.vertices + 5.0 * (double)h.out_scanned;
  return 8.0 * e + 36.0 * (double)h.vertices + 5.0 * (double)h.out_scanned;
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
  k_sync_begin<<<4, 256, 0, s>>>(g->ctl, g->sync_max, g->sync_grab, g->sync_len, iters);
  DFPR_HIP(hipGetLastError());
  auto kern = mode == kAll ? k_sync_iter<T, kAll> : k_sync_iter<T, kSyncDF>;
  const int blocks = persistent_blocks(g, kern);
  DFPR_HIP(hipEventRecord(g->ev[1], s));
  const int poll = 8;
  int it = 0;
  for (; it < iters; ++it) {
    RankArgs<T> A = make_args<T>(g, (g->cur + it) & 1, (g->cur + it + 1) & 1);
    kern<<<blocks, g->p.block_size, 0, s>>>(A, it);
    k_sync_finish<<<1, 64, 0, s>>>(g->ctl, g->sync_max, g->sync_len, it, g->p.tol,
                                   iters, mode == kSyncDF);
    if ((it + 1) % poll == 0 || it + 1 == iters) {
      DFPR_HIP(hipGetLastError());
      DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipStreamSynchronize(s));
      if (g->h_ctl->sync_done) break;
    }
  }
  DFPR_HIP(hipEventRecord(g->ev[2], s));
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
    st->converged = h.pad;
    st->vertices_processed = (int64_t)h.vertices;
    st->edges_gathered = (int64_t)h.edges;
    st->out_edges_scanned = (int64_t)h.out_scanned;
    st->max_delta = md;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[2]);
    st->ms_kernel = ms;
  }
  return h.pad ? DFPR_OK : DFPR_NOTCONVERGED;
}

template <typename T>
int run_async(dfpr_graph *g, dfpr_stats *st) {
  hipStream_t s = g->stream;
  const bool dense = g->p.dense_div > 0 &&
                     (int64_t)g->pending_marks * g->p.dense_div > (int64_t)g->n;
  k_async_begin<<<1, 64, 0, s>>>(g->ctl, dense ? 1 : 0);
  DFPR_HIP(hipGetLastError());
  RankArgs<T> A = make_args<T>(g, g->cur, g->cur);
  const int blocks = persistent_blocks(g, k_df_async<T>);
  DFPR_HIP(hipEventRecord(g->ev[1], s));
  k_df_async<T><<<blocks, g->p.block_size, 0, s>>>(A);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipEventRecord(g->ev[2], s));
  DFPR_HIP(hipMemcpyAsync(g->h_ctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  const Ctl h = *g->h_ctl;
  const int sweeps = (int)((h.state >> kSweepShift) & kSweepMask);
  const bool capped = (h.state & kCapped) != 0;
  g->last_bytes = algorithmic_bytes(g, h);
  g->last_launches = 1;
  if (st) {
    st->sweeps = sweeps;
    st->converged = !capped && !h.abort;
    st->vertices_processed = (int64_t)h.vertices;
    st->edges_gathered = (int64_t)h.edges;
    st->out_edges_scanned = (int64_t)h.out_scanned;
    st->max_delta = -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, g->ev[1], g->ev[2]);
    st->ms_kernel = ms;
  }
  if (h.abort) return fail(DFPR_EABORT, "persistent kernel watchdog fired");
  return capped ? DFPR_NOTCONVERGED : DFPR_OK;
}

template <typename T>
int renormalize(dfpr_graph *g) {
  hipStream_t s = g->stream;
  DFPR_HIP(hipMemsetAsync(&g->ctl->sum, 0, sizeof(double), s));
  k_sum<T><<<grid_for(g->n, g->cu_count), 256, 0, s>>>(g->n, (const T *)g->R[g->cur],
                                                       &g->ctl->sum);
  k_scale<T><<<grid_for(g->n, g->cu_count), 256, 0, s>>>(
      g->n, g->out.deg, &g->ctl->sum, (T *)g->R[g->cur], (T *)g->C[g->cur]);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

int finish_update(dfpr_graph *g) {
  hipStream_t s = g->stream;
  unsigned long long len = g->h_ctl->tail;
  if (len > 0)
    k_cleanup<<<grid_for((int64_t)len, g->cu_count), 256, 0, s>>>(g->flags, g->wl, len);
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
  if (g->elem == 8) {
    DFPR_HIP(hipMemcpyAsync(g->R[g->cur], r, (size_t)g->n * 8, hipMemcpyDeviceToDevice, s));
  } else {
    k_f64_to_f32<<<grid_for(g->n, g->cu_count), 256, 0, s>>>(g->n, r, (float *)g->R[g->cur]);
    DFPR_HIP(hipGetLastError());
  }
  return refresh_contributions(g);
}

int read_ranks_device(const dfpr_graph *g, double *out) {
  hipStream_t s = g->stream;
  if (g->elem == 8) {
    DFPR_HIP(hipMemcpyAsync(out, g->R[g->cur], (size_t)g->n * 8, hipMemcpyDeviceToDevice, s));
  } else {
    k_f32_to_f64<<<grid_for(g->n, g->cu_count), 256, 0, s>>>(g->n, (const float *)g->R[g->cur],
                                                             out);
    DFPR_HIP(hipGetLastError());
  }
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
  } else {
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
      st->affected = (int64_t)g->h_ctl->tail;
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
    k_copy16<<<cu * 8, 512, 0, s>>>((const int4 *)src, (int4 *)dst, n16);
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
