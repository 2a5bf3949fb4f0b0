// Internal definitions shared by the HIP translation units of libdfpr.
//
// Device layout of one graph (every array in HBM, owned by the library):
//   slack CSR per direction (out: rows are sources, in: rows are targets)
//     off[n]  int64  first slot of the row in adj (always a multiple of 4,
//                    so a row starts on a 16-byte boundary)
//     deg[n]  int32  stored entries (the implicit self-loop is not stored)
//     cap[n]  int32  slots reserved for the row (multiple of 4)
//     adj[*]  int32  row entries; rows that outgrow their slots move to the
//                    spare tail of the same array (bump allocation)
//   ranks R[2][n] and contributions C[2][n] = R / (out-degree + 1), fp64 or
//   fp32; only R[cur], C[cur] are meaningful between calls (the second
//   buffer is the Jacobi target of synchronous iterations)
//   flags[n] bytes: bit 0 affected (V_A), bit 2 out-neighbours marked
//   worklist wl[n] int32 (unused slots hold -1), appended through ctl->tail
//   per 256-vertex group: gflags bytes (bit 0: listed) and the group
//   worklist gwl that the lock-free scheme sweeps
//   Ctl: counters and the scheduling word of the persistent kernel
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dfpr.h"

namespace dfpr {

constexpr int kWave = 64;
constexpr int kMaxIters = 8000;  // sweep index field holds 13 bits

// Flag bits in the per-vertex byte.
constexpr uint32_t kVA = 1u;  // affected
constexpr uint32_t kEX = 4u;  // all out-neighbours marked (synchronous DF)

// Vertices are also grouped by id into aligned groups of kGroup; the
// lock-free scheme schedules whole groups.  Flag bit in the per-group byte:
constexpr int kGroup = 256;
constexpr int kGroupShift = 8;
constexpr uint32_t kGA = 1u;  // group holds an affected vertex (listed)
// Bits 4..6 of the group byte (set at the start of a lock-free launch):
// log2 of the parts the group is claimed in.  A group whose rows below the
// piece threshold hold many in-edges is split into up to 16 parts of equal
// vertex ranges, so no claim holds a group far longer than the others
// (with degree-sorted ids the first groups hold the heaviest rows).
constexpr uint32_t kGPartShift = 4;
constexpr int kMaxPartLog = 4;
constexpr int32_t kPartEdges = 16384;  // target in-edges per part
// Worklist entry of a group part: group | part << 23 | log2(parts) << 27
// (non-negative); a piece of a long row is -(p + 2); -1 is an empty slot.
constexpr int kEntryPartShift = 23;
constexpr int32_t kEntryGroupMask = (1 << kEntryPartShift) - 1;
constexpr int kEntryLogShift = 27;

// Scheduling word of the persistent kernel (one 64-bit atomic):
//   bit 63 done, bit 61 stopped at the sweep cap,
//   bits 48..60 sweep index, bits 16..47 cursor, bits 0..15 workers that
//   hold a chunk.
constexpr uint64_t kDone = 1ull << 63;
constexpr uint64_t kCapped = 1ull << 61;
constexpr int kSweepShift = 48;
constexpr uint64_t kSweepMask = 0x1FFFull;
constexpr int kCursorShift = 16;
constexpr uint64_t kCursorMask = 0xFFFFFFFFull;
constexpr uint64_t kInflightMask = 0xFFFFull;

// Per-slot words of the barrier-based iteration (unsigned long long, one
// 128-byte line per slot).  Wavefront w uses slot c = w % nctr (nctr: at
// most kClaimers, at most the grid's wavefronts): it claims the items
// c + nctr * k from the slot's counter and adds its statistics there, so
// no word is updated by every wavefront.
constexpr int kClaimers = 16;
constexpr int kClaimStride = 16;
enum SlotWord {
  kSlotClaim = 0,     // claim counter (reset after each iteration)
  kSlotVertices = 1,  // rank recomputations of the call
  kSlotEdges = 2,     // in-edges gathered (self-loops included)
  kSlotOut = 3,       // out-edges scanned by frontier expansion
  kSlotNewly = 4,     // vertices newly affected in this iteration
  kSlotMaxDr = 5,     // largest rank change of this iteration (fp64 bits)
  kSlotItems = 6      // work items completed in this iteration
};

// Device control block of one graph.  The words every wavefront of the
// persistent kernel touches sit on cache lines of their own.
struct Ctl {
  alignas(128) unsigned long long state;  // async scheduling word
  alignas(128) unsigned long long tail;   // vertex worklist length
  unsigned long long nsteps;              // steps of the current worklist
  unsigned long long nlong;               // rows gathered in pieces
  unsigned long long npieces;             // their pieces
  unsigned long long nexp;                // long out-rows left to mark
  unsigned long long nlong_del;           // apply: long rows with deletions
  unsigned long long nlong_mark;          // apply: long out-rows to mark
  alignas(128) unsigned long long gtail;  // group worklist length
  alignas(128) long long change_sweep;    // last sweep in which a claim saw
                                          // a change above the watermark
                                          // tolerance or affected a vertex
  alignas(128) int abort;                 // watchdog fired
  alignas(128) long long marked;          // vertices affected by the marking
  long long newly;                        // vertices affected during the update
  unsigned long long vertices;            // stats of the running update
  unsigned long long edges;
  unsigned long long out_scanned;
  unsigned long long ins_applied;  // apply_batch results (out direction)
  unsigned long long del_applied;
  unsigned long long ins_applied_in;  // the same seen from the in direction
  unsigned long long del_applied_in;
  unsigned long long adj_used[2];  // bump pointers: out, in
  int invalid;                     // an input id was out of range
  int overflow;                    // an adjacency array ran out of slots
  int sync_done;                   // synchronous iteration finished
  int sync_final;                  // iterations made by the synchronous loop
  int sync_conv;                   // synchronous loop met the tolerance
  int iter;                        // barrier-based iteration in progress
  double sum;                      // fp64 rank sum (renormalisation)
};

// One direction of the slack CSR.
struct Adj {
  int64_t *off = nullptr;
  int32_t *deg = nullptr;
  int32_t *cap = nullptr;
  int32_t *adj = nullptr;
  int64_t adj_cap = 0;  // slots allocated in adj
};

// Rows gathered in pieces (both schemes and static PageRank): a row whose
// in-degree reaches split_min_degree is cut into pieces of kPiece
// in-edges.  Whole wavefronts sum one piece each; the wavefront that
// finishes a row's last piece adds the partial sums in piece order and
// completes the vertex.  Barrier-based scheme: the rows are rebuilt from
// the affected flags every iteration.  Lock-free scheme: a row is listed
// when it becomes affected, and its pieces join the group worklist as
// entries -(p + 2).
constexpr int kPiece = 4096;
struct Split {
  int32_t *lrow = nullptr;  // [lcap] vertex of long row j
  int32_t *lpre = nullptr;  // [lcap + 1] first piece of long row j
  int32_t *lcnt = nullptr;  // [lcap] pieces of row j finished (barrier-based:
                            // the last resets it; lock-free: counts on)
  int32_t *prow = nullptr;  // [pcap] long row of piece p
  double *ppart = nullptr;  // [pcap] partial sum of piece p
  int32_t *ptag = nullptr;  // [pcap] lock-free scheme: launch that last wrote
                            // ppart[p]
  int32_t *xrow = nullptr;  // [xcap] vertices whose long out-rows are marked
                            // after the iteration (Ctl::nexp entries)
  int64_t lcap = 0, pcap = 0, xcap = 0;
};

// Reusable device scratch (grown on demand), in 16 slots:
//   graph build   0-7 temporaries; 14, 15 staged host edge arrays
//   apply_batch   4, 5, 6, 15 staged host batch arrays; per direction 0-3
//                 and 7 temporaries, 8-10 (out) / 11-13 (in) sorted keys,
//                 segments and status; 14 long rows with deletions; 0 long
//                 out-rows to mark (after both directions are prepared)
//   update        14 scan temporaries, 15 tile sums; update_many 12
//                 descriptors; 13 rank staging of set/read calls
//   traversal     8, 9 level lists, 10 level counters (marking, before an
//                 update)
struct Scratch {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace dfpr

struct dfpr_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t n = 0;
  int64_t m = 0;  // stored edges (host mirror)
  dfpr_params p{};
  dfpr::Adj out, in;
  void *R[2] = {nullptr, nullptr};
  void *C[2] = {nullptr, nullptr};
  int cur = 0;
  int elem = 8;  // bytes per rank (8 fp64, 4 fp32)
  uint32_t *flags = nullptr;
  int32_t *wl = nullptr;
  int32_t ngroups = 0;
  uint32_t *gflags = nullptr;  // [ngroups] bytes
  int32_t *gwl = nullptr;      // worklist of the lock-free scheme: group
                               // parts and the pieces of long rows
                               // [gwl_cap], unused slots -1
  int64_t gwl_cap = 0;
  int32_t async_epoch = 0;     // lock-free launches so far (piece tags)
  int32_t *steps = nullptr;    // step starts over the worklist [n + 1]
  void *tiles = nullptr;       // per-tile sums and their prefixes
                               // [2 * (n / 256 + 2)] x 16 bytes
  // barrier-based loop replayed from HIP graphs: per (scheme, parity of
  // the current rank buffer) an instantiated two-iteration graph and the
  // hash of the arguments it was captured with
  hipGraphExec_t replay[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  uint64_t replay_key[2][2] = {{0, 0}, {0, 0}};
  hipStream_t capture_stream = nullptr;
  int32_t *faults = nullptr;   // injected faults per workgroup (dfpr_set_faults)
  int32_t nfaults = 0;
  int32_t fault_stops = 0;     // some entry stops its workgroups
  dfpr::Split split;           // rows gathered in pieces
  int32_t *ext2int = nullptr;  // caller id -> internal id (null: identity)
  int32_t *int2ext = nullptr;  // internal id -> caller id
  dfpr::Ctl *ctl = nullptr;
  dfpr::Ctl *h_ctl = nullptr;           // pinned host mirror
  unsigned long long *sync_max = nullptr;   // [kMaxIters] bit patterns
  unsigned long long *sync_grab = nullptr;  // claim counters of the
                                            // barrier-based iteration
  unsigned long long *sync_len = nullptr;   // [kMaxIters] worklist snapshot
  int64_t pending_marks = 0;  // host view of marks not yet consumed
  dfpr::Scratch scratch[16];
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> iter_ev;  // around each barrier-based iteration
                                    // kernel: [2 * i] before, [2 * i + 1] after
  double last_bytes = 0.0;
  int32_t last_launches = 0;
  int cu_count = 0;
  int wallclock_khz = 0;
};

namespace dfpr {

// Error plumbing: every entry point returns a status and records a message.
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define DFPR_HIP(expr)                                                    \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return ::dfpr::fail(e_ == hipErrorOutOfMemory ? DFPR_ENOMEM : DFPR_EHIP, \
                          std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Grows scratch slot `i` of g to at least `bytes`.
int scratch_get(dfpr_graph *g, int i, size_t bytes, void **out);

// Validates params.
int check_params(const dfpr_params *p);

// Builders (dfpr_build.hip).
int build_graph(dfpr_graph *g, int64_t m, const int32_t *src,
                const int32_t *dst);

// Dynamic Traversal marking (dfpr_traverse.hip): extends the pending marks
// to everything reachable from them; *marked (may be null) gets the total.
int mark_reachable(dfpr_graph *g, int64_t *marked);

// Vertex insertion and removal with rescaled ranks (dfpr_vertices.hip).
int add_vertices(dfpr_graph *g, int32_t count, int32_t *first_id);
int remove_vertices(dfpr_graph *g, int32_t count);

// Ranks (dfpr_rank.hip).
// Sizes the piece arrays and the group worklist for the current adjacency
// capacities and split threshold (allocates only when they grew).
int ensure_split(dfpr_graph *g);
int init_uniform_ranks(dfpr_graph *g);
int refresh_contributions(dfpr_graph *g);

// Device helpers ------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t flag_byte(const uint32_t *flags, int32_t v,
                                              bool coherent) {
  uint32_t w = coherent ? load_agent(flags + (v >> 2)) : flags[v >> 2];
  return (w >> ((v & 3) * 8)) & 0xFFu;
}

// Sets `bits` in the flag byte of v and returns the byte's previous bits.
__device__ __forceinline__ uint32_t flag_set(uint32_t *flags, int32_t v,
                                             uint32_t bits) {
  const int sh = (v & 3) * 8;
  uint32_t old = __hip_atomic_fetch_or(flags + (v >> 2), bits << sh,
                                       __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return (old >> sh) & 0xFFu;
}

__device__ __forceinline__ uint32_t flag_clear(uint32_t *flags, int32_t v,
                                               uint32_t bits) {
  const int sh = (v & 3) * 8;
  uint32_t old = __hip_atomic_fetch_and(flags + (v >> 2), ~(bits << sh),
                                        __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
  return (old >> sh) & 0xFFu;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o);
    x = y > x ? y : x;
  }
  return x;
}

// Broadcast lane 0's 64-bit value to the wave (all lanes active).
__device__ __forceinline__ unsigned long long bcast0(unsigned long long x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Appends v (on lanes where `want` holds) to the worklist with one atomic
// per wave.  All lanes of the wave must call it together.
__device__ __forceinline__ int wave_append(bool want, int32_t v,
                                           int32_t *wl,
                                           unsigned long long *tail,
                                           bool coherent) {
  const uint64_t mask = __ballot(want);
  if (mask == 0) return 0;
  const int cnt = __popcll(mask);
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader)
    base = __hip_atomic_fetch_add(tail, (unsigned long long)cnt,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader);
  if (want) {
    const unsigned long long pos = base + __popcll(mask & lanemask_lt());
    if (coherent)
      store_agent(wl + pos, v);
    else
      wl[pos] = v;
  }
  return cnt;
}

// Marks v affected and lists its group with plain byte stores: valid while
// no other bit of these bytes changes concurrently (the marking phase
// between updates, where a byte only goes from 0 to the flag).
__device__ __forceinline__ void mark_plain(uint32_t *flags, uint32_t *gflags, int32_t v) {
  reinterpret_cast<uint8_t *>(flags)[v] = (uint8_t)kVA;
  reinterpret_cast<uint8_t *>(gflags)[v >> kGroupShift] = (uint8_t)kGA;
}

struct MarkOut {
  bool vnew;
  bool gnew;
  int32_t g;
};

// Marks v affected and lists its group.  vnew / gnew report whether v / its
// group were new (decided by the atomics).  The pre-checks skip the atomics
// when the bits are already set: coherent (agent-scope) ones inside the
// lock-free kernel, plain ones elsewhere, where a stale read only costs an
// extra atomic (bits only go from 0 to 1 within an update, so no read shows
// a bit that is not set).  A vertex found affected needs nothing more: the
// caller that set its bit lists its group.
__device__ __forceinline__ MarkOut mark_affected(uint32_t *flags,
                                                 uint32_t *gflags, int32_t v,
                                                 bool coherent = true) {
  MarkOut o{false, false, v >> kGroupShift};
  if (flag_byte(flags, v, coherent) & kVA) return o;
  o.vnew = !(flag_set(flags, v, kVA) & kVA);
  if (!(flag_byte(gflags, o.g, coherent) & kGA))
    o.gnew = !(flag_set(gflags, o.g, kGA) & kGA);
  return o;
}

}  // namespace dfpr
