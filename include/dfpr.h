/*
 * dfpr.h -- Dynamic Frontier PageRank on MI355X (gfx950), C ABI.
 *
 * Method: "Lock-Free Computation of PageRank in Dynamic Graphs"
 * (arXiv 2407.19562).  After a batch of edge deletions and insertions
 * (Section 3.4), the ranks of the previous graph are updated by the Dynamic
 * Frontier approach (Section 4.1): the out-neighbours of every batch source
 * in the previous and current graph are marked affected, affected vertices
 * are recomputed with Eq. 1 (Section 3.1) pulling over their in-edges, a
 * vertex whose rank moves by more than the frontier tolerance marks its
 * out-neighbours (Section 4.1.1), and the loop ends when the L-infinity
 * change is within the iteration tolerance (Algorithms 1 and 2).
 *
 * Conventions shared by every entry point:
 *  - Status: 0 is success; negative values are errors (DFPR_E*), and
 *    DFPR_NOTCONVERGED (> 0) is a warning: ranks are valid but the sweep cap
 *    was reached.  Nothing crosses the ABI as an exception.
 *    dfpr_last_error() returns a message for the last failure on the
 *    calling thread.
 *  - Memory: every array argument is a plain pointer with an explicit
 *    element count; `mem` says whether it is host memory (DFPR_MEM_HOST) or
 *    device memory on the graph's device (DFPR_MEM_DEVICE).  Inputs are only
 *    read, and are no longer needed once the call returns.  Outputs are
 *    written by the call and complete when it returns.
 *  - Ownership: the library owns every buffer of a graph (adjacency, ranks,
 *    flags, worklist, counters).  The caller owns its own arrays.
 *  - Streams: every device operation of a graph is ordered on the stream
 *    given at creation (a hipStream_t passed as void*; NULL is the null
 *    stream).  A call returns after its work on that stream has finished.
 *    One graph must not be used from two threads at once; distinct graphs
 *    are independent.
 *  - Vertex ids are int32 in [0, n).  Batches keep n fixed (Section 3.4);
 *    only dfpr_add_vertices and dfpr_remove_vertices change it.
 *  - Every vertex carries an implicit self-loop (dead-end removal,
 *    Section 5.1.3): |out(u)| counts it, and a batch edge (v, v) is ignored.
 */
#ifndef DFPR_H
#define DFPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DFPR_OK 0
#define DFPR_NOTCONVERGED 1 /* sweep cap reached; ranks valid              */
#define DFPR_EINVAL (-1)    /* bad argument: null pointer, id outside [0,n),
                               n <= 0, alpha outside (0,1), tol <= 0, ...  */
#define DFPR_ENOMEM (-2)    /* device allocation failed; graph unchanged   */
#define DFPR_EHIP (-3)      /* HIP runtime error; destroy the graph        */
#define DFPR_EABORT (-4)    /* a kernel gave up (watchdog, or injected
                               faults stopped every workgroup); marks are
                               cleared and the ranks are unspecified       */
#define DFPR_ESTATE (-5)    /* call not valid in the graph's current state */

/* where an array argument lives */
#define DFPR_MEM_HOST 0
#define DFPR_MEM_DEVICE 1

/* scheduling of the rank iteration */
#define DFPR_ASYNC 0 /* one persistent launch; in-place (Gauss-Seidel-like)
                        ranks, dynamic claims of 256-vertex groups and of
                        4096-edge pieces of long rows, no grid barrier;
                        ends after a full sweep that meets the lf_stop rule
                        (the lock-free variant, Algorithm 2)             */
#define DFPR_SYNC 1  /* one launch per iteration; two rank vectors and an
                        L-infinity norm per iteration (the barrier-based
                        variant, Algorithm 1)                             */

/* stopping rule of the lock-free DF and DT updates (dfpr_params.lf_stop) */
#define DFPR_STOP_TOL 0      /* a full sweep in which no rank moves by more
                                than tol: Algorithm 1's test (delta R <= tau)
                                over the sweeps of the in-place iteration    */
#define DFPR_STOP_FRONTIER 1 /* a full sweep in which no rank moves by more
                                than frontier_tol: Algorithm 2's R_C flags
                                read strictly (every change above tau_f
                                re-opens its out-neighbours)                 */

/* adjacency directions for dfpr_read_edges */
#define DFPR_OUT 0
#define DFPR_IN 1

typedef struct dfpr_graph dfpr_graph; /* opaque */

typedef struct {
  double alpha;          /* damping factor (Section 5.1.2: 0.85)            */
  double tol;            /* iteration tolerance tau, L-infinity (1e-10)     */
  double frontier_tol;   /* frontier tolerance tau_f (Section 4.4: tau/1000)*/
  int32_t max_iters;     /* cap on sweeps / iterations (500)                */
  int32_t precision;     /* 64: fp64 ranks; 32: fp32 ranks and sums with fp64
                            change tests and norms                          */
  int32_t mode;          /* DFPR_ASYNC (default, the paper's lock-free
                            method) or DFPR_SYNC (faster on one MI355X for
                            large graphs)                                   */
  int32_t kahan_min_degree; /* fp32 ranks, barrier-based scheme: rows with
                               at least this in-degree accumulate in fp64,
                               shorter rows in fp32 (default 0: every row
                               in fp64, which measured faster, as fp32 LDS
                               atomic adds to one row stall the wavefront);
                               the lock-free scheme accumulates every row
                               in fp64                                      */
  int32_t split_min_degree; /* rows with at least this in-degree are
                               summed in pieces of 4096 in-edges by whole
                               wavefronts (partial sums added in piece
                               order), the rest in edge-balanced steps of
                               up to 256 rows; 0 (default): 2048 for the
                               barrier-based scheme, 8192 for the lock-free
                               one (512 on a graph in degree-sorted order,
                               see reorder).  In the lock-free scheme a
                               row's pieces are claimed like groups, and
                               rows of 8192 or more in-edges always go in
                               pieces (a claim must stay short next to a
                               sweep)                                       */
  int32_t chunk;         /* lock-free scheme: vertices per wavefront of a
                            claim, whole 256-vertex groups (chunk / 256, at
                            least one); a multiple of 64 in [64, 4096], or
                            0 (default): one group per 1024 groups of the
                            graph, 1..16 (1..4 on a graph in degree-sorted
                            order), and 4 groups in the batched launch.  A
                            claim is made by a whole workgroup, for all its
                            wavefronts                                     */
  int32_t block_size;    /* threads per workgroup of the rank kernel: 64,
                            128, 192 or 256, or 0 (default): 128 for the
                            barrier-based scheme, 256 for the lock-free
                            scheme on one graph, 128 for the batched
                            launch (dfpr_update_many takes the first
                            graph's)                                        */
  int32_t reorder;       /* internal vertex order, fixed at creation:
                            0 keep the caller's ids; 1 sort by decreasing
                            out-degree, so the contributions read most often
                            share cache lines; 2 (default) sort when the
                            graph is large (n >= 2^20) and its out-degree
                            skewed (max >= 8 x mean).  On a sorted graph
                            the lock-free scheme lists its groups
                            interleaved, so that its claims stay even.
                            Ids at the ABI are always the caller's.        */
  int32_t renormalize;   /* fp32: after each update rescale the ranks to
                            sum 1 (fp64 sum) when they miss it by more than
                            n * tol, the update's own truncation          */
  int32_t timeout_ms;    /* watchdog for the persistent kernel (0: none)    */
  int32_t grid_blocks;   /* workgroups of the rank kernels; 0 = automatic:
                            barrier-based, at most 12 wavefronts per CU and
                            no more than an iteration's work items;
                            lock-free, about four claims per workgroup per
                            sweep and at least four wavefronts per CU      */
  int32_t graph_replay;  /* barrier-based loop: 0 one launch sequence per
                            iteration from the host; 1 two iterations
                            captured once in a HIP graph and replayed (kernel
                            time is then reported for the whole loop);
                            2 (default) replay when the graph has at most
                            2^22 in-edge slots, where launches dominate.
                            A capture that fails (other threads' device
                            calls can invalidate it) falls back to
                            launching the iterations one by one; callers
                            that drive graphs from several threads at once
                            are better off with 0                          */
  int32_t lf_stop;       /* lock-free DF / DT updates: DFPR_STOP_TOL
                            (default) or DFPR_STOP_FRONTIER.  The lock-free
                            static and naive-dynamic calls always use the
                            frontier rule                                   */
} dfpr_params;

typedef struct {
  int32_t sweeps;        /* iterations (sync) or sweeps (async) performed   */
  int32_t converged;     /* 1 if the tolerance was met before the cap       */
  int64_t initial_marked;     /* vertices affected by the initial marking   */
  int64_t affected;           /* vertices affected at the end               */
  int64_t vertices_processed; /* rank recomputations, summed over sweeps    */
  int64_t edges_gathered;     /* in-edges read by the gathers, the implicit
                                 self-loop included                         */
  int64_t out_edges_scanned;  /* out-edges read by frontier expansion       */
  double max_delta;      /* sync: L-infinity change of the last iteration;
                            async: -1 (not tracked)                         */
  float ms;              /* device time of the call (HIP events)            */
  float ms_kernel;       /* device time of the rank kernel launches alone
                            (barrier-based: sum over the iteration kernels,
                            without the item building between them)        */
} dfpr_stats;

/* Fills `p` with the paper's defaults (alpha 0.85, tol 1e-10,
 * frontier_tol tol/1000, 500 iterations, fp64, async) and this library's
 * launch defaults.  Returns DFPR_EINVAL if p is NULL. */
int dfpr_params_default(dfpr_params *p);

/* Builds a graph on the current HIP device from n vertices and m edges
 * (src[i] -> dst[i]).  Duplicate edges and self pairs in the input are
 * dropped (edges form a set).  Ranks start at 1/n.  `params` may be NULL
 * (defaults).  On success *out receives the handle.  Errors: DFPR_EINVAL
 * (n <= 0, m < 0, null pointers with m > 0, an id outside [0, n), bad
 * params), DFPR_ENOMEM, DFPR_EHIP. */
int dfpr_graph_create(int32_t n, int64_t m, const int32_t *src,
                      const int32_t *dst, int mem, const dfpr_params *params,
                      void *hip_stream, dfpr_graph **out);

/* Frees every device buffer of the graph.  NULL is accepted. */
int dfpr_graph_destroy(dfpr_graph *g);

/* Replaces / reads the graph's parameters.  Validated like create. */
int dfpr_set_params(dfpr_graph *g, const dfpr_params *p);
int dfpr_get_params(const dfpr_graph *g, dfpr_params *p);

/* Number of vertices and of stored edges (self-loops not counted). */
int dfpr_graph_size(const dfpr_graph *g, int32_t *n, int64_t *m);

/* Static PageRank (Eq. 1; Algorithm 3): ranks restart at 1/n and Jacobi
 * iterations over every vertex run until the L-infinity change is <= tol or
 * max_iters.  Pending marks are kept.  Returns DFPR_NOTCONVERGED at the
 * cap.  `stats` may be NULL. */
int dfpr_static(dfpr_graph *g, dfpr_stats *stats);

/* Naive-dynamic PageRank (Section 3.5.1): the same iteration over every
 * vertex, started from the current ranks. */
int dfpr_naive_dynamic(dfpr_graph *g, dfpr_stats *stats);

/* Lock-free static and naive-dynamic PageRank (Algorithms 4 and 6,
 * Section 3.5.1): every vertex is recomputed in place by the persistent
 * kernel of the lock-free scheme, from 1/n (static) or from the current
 * ranks (naive-dynamic), until a full sweep moves no vertex by more than
 * frontier_tol (stricter than the tol at which those algorithms clear R_C:
 * with tol alone a hub with 25000 in-edges ended 1.04e-9 from the fixed
 * point), or max_iters sweeps.
 * Batches applied before the call count as served (their marks are
 * cleared).  Returns DFPR_NOTCONVERGED at the cap, DFPR_EABORT if the
 * watchdog fired. */
int dfpr_static_lock_free(dfpr_graph *g, dfpr_stats *stats);
int dfpr_naive_dynamic_lock_free(dfpr_graph *g, dfpr_stats *stats);

/* Fault simulation (Sections 4.3 and 5.1, fault simulation): table[count]
 * (host memory, copied) gives each workgroup w of the rank kernels the
 * fault table[w % count], taken after every claim it completes: 0 none;
 * d in (0, 1e6] sleep d microseconds (a random thread delay); -1 stop
 * claiming (a crash-stop at a claim boundary: the workgroup holds no
 * work when it stops, and the others finish its share).  A crash while
 * holding a claim is not simulated; it would keep the lock-free scheme's
 * in-flight count above zero until the watchdog (timeout_ms) aborts.
 * count 0 clears the table.  Applies to dfpr_update, dfpr_static,
 * dfpr_naive_dynamic and their lock-free forms, not to dfpr_update_many.
 * DFPR_EINVAL for entries outside those values. */
int dfpr_set_faults(dfpr_graph *g, const int32_t *table, int32_t count);

/* Overwrites the ranks with r[n] (fp64; rounded for fp32 graphs). */
int dfpr_set_ranks(dfpr_graph *g, const double *r, int mem);

/* Copies the ranks to out[n] as fp64. */
int dfpr_read_ranks(const dfpr_graph *g, double *out, int mem);

/* Applies one batch (Section 3.4) in place to both the out- and the
 * in-adjacency: first every deletion (del_src[i] -> del_dst[i]), then every
 * insertion, with set semantics (deleting an absent edge or inserting a
 * present one changes nothing; self pairs are ignored; duplicates count
 * once).  The whole batch is validated before anything changes (all or
 * nothing on DFPR_EINVAL).  The sources of the edges that really changed
 * are marked for the next dfpr_update (Algorithm 1/2 initial marking: the
 * out-neighbours of u in the previous and the current graph, u itself
 * through its self-loop); several batches may be applied before one
 * update.  applied_del / applied_ins (may be NULL) receive the number of
 * edges actually deleted / inserted.  Errors: DFPR_EINVAL, DFPR_ENOMEM
 * (graph unchanged), DFPR_EHIP. */
int dfpr_apply_batch(dfpr_graph *g, int64_t n_del, const int32_t *del_src,
                     const int32_t *del_dst, int64_t n_ins,
                     const int32_t *ins_src, const int32_t *ins_dst, int mem,
                     int64_t *applied_del, int64_t *applied_ins);

/* Dynamic Frontier update (Section 4; Algorithm 1 in DFPR_SYNC mode,
 * Algorithm 2's lock-free scheme in DFPR_ASYNC mode) from the current ranks
 * over the vertices marked since the last update; consumes the marks.
 * Returns DFPR_OK, DFPR_NOTCONVERGED, DFPR_EABORT (watchdog), DFPR_EHIP.
 * `stats` may be NULL. */
int dfpr_update(dfpr_graph *g, dfpr_stats *stats);

/* Vertex insertion (an extension: the paper keeps the vertex set fixed,
 * Section 3.4, and names vertex additions with ranks scaled before the
 * computation as future work, Section 6).  Appends `count` vertices with
 * caller ids n .. n+count-1 (*first_id, may be NULL, receives n) and no
 * edges but their self-loops.  Every existing rank is multiplied by
 * n / (n+count) and the new ranks are 1 / (n+count): with Eq. 1's teleport
 * term (1-alpha)/n this maps a fixed point of the old graph to one of the
 * new graph exactly, so nothing is marked.  Edges to and from the new
 * vertices are ordinary batches (dfpr_apply_batch, then dfpr_update).
 * Pending marks are kept.  Per-vertex device arrays are reallocated (the
 * call synchronizes the graph's stream); on DFPR_ENOMEM the graph is
 * unchanged.  Errors: DFPR_EINVAL (count <= 0, or n + count above
 * 2^31 - 2), DFPR_ENOMEM, DFPR_EHIP. */
int dfpr_add_vertices(dfpr_graph *g, int32_t count, int32_t *first_id);

/* Vertex removal (the same extension): removes the `count` highest caller
 * ids n-count .. n-1 with every edge incident to them.  Those edges are
 * deleted as one batch (marking the remaining out-neighbours of their
 * sources, and the sources, as dfpr_apply_batch does), the removed ids'
 * marks are dropped, and every remaining rank is multiplied by
 * n / (n-count); the next dfpr_update recomputes the marked vertices.
 * To remove other vertices, give them the highest ids first.  A graph
 * whose internal order was changed at creation (reorder) accepts removal
 * only of vertices it keeps in the caller's order there (those added by
 * dfpr_add_vertices).  Synchronizes the graph's stream.  Errors:
 * DFPR_EINVAL (count outside [1, n), or reordered ids), DFPR_ENOMEM,
 * DFPR_EHIP. */
int dfpr_remove_vertices(dfpr_graph *g, int32_t count);

/* Dynamic Traversal marking (Section 3.5.2; Algorithms 7 and 8, before the
 * iterations): extends the marks of the batches applied since the last
 * update to every vertex reachable from them along the current graph's
 * out-edges, breadth first on the device.  Since dfpr_apply_batch marked
 * (G^{t-1} U G^t).out(u) of every changed source u, the result is the
 * affected set of Algorithm 7.  Every vertex it marks has had its out-row
 * walked, so a following dfpr_update recomputes exactly this set and never
 * grows it: the pair is the Dynamic Traversal update.  Marks added by a
 * later dfpr_apply_batch before the update grow as Dynamic Frontier marks.
 * *marked (may be NULL) receives the number of marked vertices.  Idempotent;
 * with nothing marked it does nothing.  Errors: DFPR_EINVAL, DFPR_ENOMEM,
 * DFPR_EHIP. */
int dfpr_mark_reachable(dfpr_graph *g, int64_t *marked);

/* Dynamic Traversal update (Algorithm 7 in DFPR_SYNC mode, Algorithm 8's
 * lock-free scheme in DFPR_ASYNC mode): dfpr_mark_reachable followed by
 * dfpr_update, timed together in stats->ms; stats->initial_marked is the
 * size of the reachable set.  The lock-free scheme ends by the lf_stop
 * rule, as the lock-free DF update does.  Same returns as dfpr_update. */
int dfpr_update_traversal(dfpr_graph *g, dfpr_stats *stats);

/* Dynamic Frontier updates of `count` graphs in one persistent launch
 * (async scheduling only; all graphs on the same device, the first graph's
 * stream is used).  stats[count] may be NULL.  Returns the worst status. */
int dfpr_update_many(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats);

/* dfpr_update_many for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and returns as dfpr_update_many, but the launch's
 * descriptors, summaries and done counter live in a fixed workspace that
 * the library holds in each device's code object (about 1.5 MB per device,
 * kept until the process ends), so the call makes no hipMalloc, hipFree or
 * other allocating call on the host or the device.  At most
 * DFPR_NOALLOC_MAX_GRAPHS graphs (DFPR_EINVAL above that).  Every graph's
 * piece arrays must already fit its adjacency, which graph creation,
 * dfpr_apply_batch, dfpr_set_params and dfpr_add_vertices guarantee
 * (DFPR_ESTATE otherwise).  The workspace is shared by every call on a
 * device and keeps the last call's contents; calls are serialised inside
 * the library, and a caller that overlaps this call with dfpr_update_many
 * on the same graphs races. */
#define DFPR_NOALLOC_MAX_GRAPHS 4096
int dfpr_update_many_noalloc(dfpr_graph *const *gs, int32_t count,
                             dfpr_stats *stats);

/* Copies the stored edges (self-loops excluded) of one direction to host
 * arrays src[cap], dst[cap] (row order unspecified); *count receives the
 * edge count.  DFPR_EINVAL if cap is too small. */
int dfpr_read_edges(const dfpr_graph *g, int dir, int32_t *src, int32_t *dst,
                    int64_t cap, int64_t *count);

/* Affected flags after the marking (1 byte per vertex; all zero once an
 * update has consumed them) and the number of vertices the pending
 * batches marked; for tests. */
int dfpr_read_marks(const dfpr_graph *g, uint8_t *affected, int64_t *count);

/* Device bytes held by the graph. */
int dfpr_graph_bytes(const dfpr_graph *g, int64_t *bytes);

/* Copies `bytes` bytes from src to dst (device pointers) with a streaming
 * kernel on `hip_stream`; *ms receives its device time.  Used to measure
 * the achievable HBM bandwidth next to the rank kernels. */
int dfpr_stream_copy(void *dst, const void *src, int64_t bytes,
                     void *hip_stream, float *ms);

/* Algorithmic bytes of the rank kernel launches of the last dfpr_update /
 * dfpr_static / dfpr_naive_dynamic call and the number of those launches.
 * Per gathered in-edge 12 bytes (fp64) or 8 (fp32): the 4-byte index and
 * the contribution; per recomputed vertex 52 or 36: in-row offset 8,
 * in-degree 4, out-degree 4, worklist entry 4, rank read and write,
 * contribution write and the vertex's own contribution; per scanned
 * out-edge 5 (index and flag byte). */
int dfpr_last_kernel_bytes(const dfpr_graph *g, double *bytes,
                           int32_t *launches);

const char *dfpr_strerror(int status);
const char *dfpr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFPR_H */
