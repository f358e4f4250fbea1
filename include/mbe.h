/*
 * mbe.h -- C interface of the MI355X maximal biclique enumeration library (libmbe.so).
 *
 * The library enumerates the maximal bicliques of a bipartite graph G = (U u V, E): the
 * pairs (A, B) with A a non-empty subset of U, B a non-empty subset of V, every a in A
 * adjacent to every b in B, and neither side extendable (B = N(A) and A = N(B), with N(X)
 * the common neighbours of X).  This is the set defined in section II-A of "Accelerating
 * Maximal Biclique Enumeration on GPUs" (Hsieh, Chang, Cheng, Kuo, arXiv 2401.05039), and
 * the search that produces it is the MBEA branch-and-bound of Algorithm 1 (section II-B),
 * run as a depth-first search on an explicit per-wave stack inside HIP kernels for gfx950.
 *
 * Conventions shared by every entry point:
 *   - Vertex ids are int32, 0-based.  |E| fits in int32.
 *   - Results are exact integers; there is no floating point anywhere in the search.
 *   - Every call is synchronous on the stream given in mbe_options (NULL: the null stream)
 *     and returns 0 (MBE_OK) or a negative MBE_ERR_* code; mbe_strerror names the code.
 *   - Input arrays are owned by the caller and never written or freed by the library.
 *   - The library allocates device memory for its own working state and keeps it cached per
 *     device between calls.  Calls on one device are serialised by an internal lock.
 *   - A search runs one persistent kernel per mask-width class of top-level candidates,
 *     concurrently, on streams the library creates per device (five).  HIP maps a process's
 *     streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default), and kernels of streams
 *     that share a queue run one after another: for the concurrent form, set
 *     GPU_MAX_HW_QUEUES to 8 or more before the process first uses the GPU.  Results never
 *     depend on it.
 */
#ifndef MBE_H
#define MBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------- error codes */
#define MBE_OK                    0
#define MBE_ERR_INVALID_ARG      -1  /* null pointer where one is required, negative size */
#define MBE_ERR_INVALID_GRAPH    -2  /* bad offsets, unsorted/duplicate row, id out of range,
                                        or the two CSR arrays are not transposes */
#define MBE_ERR_BUFFER_TOO_SMALL -3  /* records did not fit; the mbe_result is still complete */
#define MBE_ERR_OUT_OF_MEMORY    -4  /* device allocation failed, or the caller's workspace is too small */
#define MBE_ERR_DEVICE           -5  /* a HIP runtime call failed */
#define MBE_ERR_UNSUPPORTED      -6  /* (kept for binary compatibility; no longer returned) */
#define MBE_ERR_SCRATCH_LIMIT    -7  /* mbe_count_noalloc: the call does not fit the fixed scratch */
#define MBE_ERR_TIMEOUT          -8  /* server: the request passed its deadline (result unspecified) */
#define MBE_ERR_CANCELLED        -9  /* server: the request was cancelled (result unspecified) */

/* Widest fixed mask class: top-level candidates of degree up to this many are searched with
 * neighbour sets held in registers as bit masks of 64 * 2^c bits (c = 0..4); candidates of any
 * larger degree go to the wide search, whose masks have any width (see mbe_count). */
#define MBE_MAX_DEGREE 1024

/* ------------------------------------------------------------------------- graph */
/*
 * The bipartite graph as two compressed-sparse-row arrays that must be exact transposes.
 *   u_off[n_u + 1]: u_off[0] = 0, non-decreasing, u_off[n_u] = n_edges.
 *   u_adj[n_edges]: row u = u_adj[u_off[u] .. u_off[u+1]) lists N(u) (ids in V), strictly
 *                   ascending.
 *   v_off[n_v + 1], v_adj[n_edges]: the same for V, listing ids in U.
 * on_device = 0: the four arrays are host memory (copied to the device by the call);
 * on_device = 1: they are device memory of the current HIP device (e.g. torch data_ptr()).
 */
typedef struct mbe_graph {
    int32_t n_u, n_v;
    int32_t n_edges;
    const int32_t *u_off, *u_adj;
    const int32_t *v_off, *v_adj;
    int32_t on_device;
} mbe_graph;

/* ------------------------------------------------------------------------- result */
/*
 * count      number of maximal bicliques found
 * hash       sum over them of h(A, B), mod 2^64, with
 *              mix(z) = SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014),
 *              K = 0x9E3779B97F4A7C15, hu(a) = mix(K (2a+1)), hv(b) = mix(K (2b+2)),
 *              h(A, B) = mix(sum_{a in A} hu(a) + mix(sum_{b in B} hv(b) + K)).
 *            It does not depend on the order of bicliques or of vertices inside them.
 * out_ints   sum over bicliques of 2 + |A| + |B| (the ints mbe_enumerate needs)
 * nodes, nonmaximal, max_depth, bytes_alg
 *            search-tree diagnostics, filled when mbe_options.diagnostics = 1, else 0:
 *            candidates taken, candidates whose maximality check failed, deepest level
 *            (top level = 1), and the algorithmic bytes of the tree (4 bytes per id read or
 *            written by the reverse-scanning method of section III-E, see the design notes).
 * side       candidate side used: 1 = U, 2 = V
 * kernel_ms  device time of the search kernel(s) of this call, from HIP events
 * phase_cycles  with diagnostics: shader-clock cycles summed over waves, per phase of the
 *            search (the breakdown of the paper's evaluation, section IV): [0] top-level
 *            candidate set-up, [1] settling single-vertex nodes, [2] maximality tests of the
 *            other nodes, [3] scans of maximal nodes, [4] building child lists, [5] waiting,
 *            stealing and claiming
 * shared_chunks  64-candidate chunks of third-level lists searched by a wave other than the
 *            list's owner (steal_k = 3; for a batch, the whole call's); counted in every mode
 * attempts   search launches the call needed: a launch whose wave stacks or frame-header
 *            arrays run out is repeated with twice the room (a device remembers the largest
 *            room an earlier call needed and starts there)
 * status     batched and served results: the graph's own status (0 for every graph the call
 *            searched; a call that fails reports its error as the return code instead)
 * bytes_design  with diagnostics = 2: the bytes of device memory that the search's own loads,
 *            stores and atomics request (the design's traffic model, before any cache): the
 *            top-level candidates' reverse scans and local universes, every frame's lists,
 *            per-bit tables and position rows written and read, per node the rows, masks and
 *            tables it reads; the rebuilds of shared lists by helping workgroups are left out,
 *            so the tally depends on the graph alone, not on the launch shape or timing
 */
typedef struct mbe_result {
    uint64_t count;
    uint64_t hash;
    uint64_t out_ints;
    uint64_t nodes;
    uint64_t nonmaximal;
    uint64_t bytes_alg;
    uint32_t max_depth;
    uint32_t side;
    double kernel_ms;
    uint64_t phase_cycles[6];
    uint64_t shared_chunks;
    uint32_t attempts;
    int32_t status;
    uint64_t bytes_design;
} mbe_result;

/* ------------------------------------------------------------------------- options */
/*
 * Zero-initialised fields mean "default"; a NULL mbe_options pointer means all defaults.
 *   side         0: the smaller side holds the candidates (U on a tie); 1: U; 2: V.
 *                The answer does not depend on it; records are always reported as (A in U,
 *                B in V).
 *   wg_waves     64-lane waves per workgroup (1..8; default 8).
 *   grid         workgroups of the persistent search kernel (default: 2 per compute unit).
 *   diagnostics  1: also compute nodes / nonmaximal / max_depth / bytes_alg (the search then
 *                keeps the method's full Q lists, so that the tallies are the method's);
 *                2: the production search (pruned Q lists, as with 0) that also tallies
 *                bytes_design.  Other values are invalid.
 *   no_validate  1: skip the O(|E|) check of the CSR pair (the caller vouches for it).
 *   steal_k      work sharing below a top-level candidate (the k of section III-D): 2
 *                (default): the candidates of its child list that need a full node are
 *                claimed one at a time by the owning workgroup's waves and, once a workgroup
 *                of the launch is idle (the rest of the list then moves to a global slot), by
 *                idle workgroups, which rebuild the same list; 1: by the owning workgroup
 *                only; 3: as 2, and in the classes of degree above 64 the child lists of
 *                second-level nodes are shared too: a wave publishes the rest of such a list
 *                (in 64-candidate chunks) once a wave or workgroup is idle, and idle waves of
 *                its workgroup and idle workgroups (after every launch's top-level
 *                candidates are handed out) claim chunks and rebuild the list themselves.
 *                Results never depend on it.
 *   root_lo, root_hi
 *                restrict the search to the top-level candidates whose rank lies in
 *                [root_lo, root_hi) (rank = position in ascending (degree, id) order among
 *                candidates of degree > 0); root_hi <= 0 means "to the end".  Results over
 *                disjoint rank ranges add up to the whole result.
 *   stream       hipStream_t to run on, or NULL.
 *   prune        the embedded pruning of section II-C; the answer is the same, the tree and
 *                its tallies are the pruned ones:
 *                1: iMBEA's candidate pruning: when a node's candidate x is maximal, every
 *                   other candidate that joins L' and has no neighbour in R outside R' leaves
 *                   P and joins Q with x (a preparation pass finds the candidates with equal
 *                   rows);
 *                2: the pivot rule: in every candidate list below the top level, the first
 *                   candidate p of the largest count |N(p) n R| is taken first, and the
 *                   candidates whose neighbours within R are all neighbours of p (every
 *                   maximal biclique holding one of them holds p) are never taken: they are
 *                   candidates for p's node and Q entries for the nodes after them.
 *                Either way every top-level candidate is searched by the wide search, Q
 *                lists are kept whole, and the fixed mask classes are not used.  Other
 *                values, and pruning with diagnostics = 2, mbe_count_loads or the batched
 *                and served forms: MBE_ERR_INVALID_ARG.
 *   workspace, workspace_bytes
 *                (mbe_count only) device memory owned by the caller, on the current device,
 *                from which every device buffer of the call is carved instead of the
 *                library's per-device buffers: nothing is allocated, the class launches run
 *                one after another on the call's stream, and the search grid shrinks to the
 *                arena slots that fit.  The caller keeps the memory valid until the call
 *                returns and must not share it with a concurrent call; its contents are
 *                unspecified afterwards.  A call that needs more returns
 *                MBE_ERR_OUT_OF_MEMORY.  NULL: the library's buffers.  A non-NULL workspace
 *                with workspace_bytes 0, a NULL one with workspace_bytes > 0, or a workspace
 *                with mbe_enumerate, mbe_count_noalloc, mbe_count_loads,
 *                mbe_workspace_size, the batched or the served form: MBE_ERR_INVALID_ARG.
 */
typedef struct mbe_options {
    int32_t side;
    int32_t wg_waves;
    int32_t grid;
    int32_t diagnostics;
    int32_t no_validate;
    int32_t steal_k;
    int64_t root_lo;
    int64_t root_hi;
    void *stream;
    int32_t prune;
    void *workspace;
    uint64_t workspace_bytes;
} mbe_options;

/*
 * Count the maximal bicliques of g and hash them (algorithm: MBEA, Algorithm 1, with the
 * reverse-scanning count of section III-E).  out receives the mbe_result described above.
 * Any degree is taken: top-level candidates of degree at most MBE_MAX_DEGREE run in one
 * persistent kernel per mask-width class, the rest (degree above 1024) in the wide search
 * after them, with the same candidate order, tree and tallies.
 * Errors: MBE_ERR_INVALID_ARG (g or out NULL, negative sizes, missing arrays),
 * MBE_ERR_INVALID_GRAPH, MBE_ERR_OUT_OF_MEMORY, MBE_ERR_DEVICE.
 * An empty side or zero edges gives count = hash = 0.
 */
int mbe_count(const mbe_graph *g, const mbe_options *opt, mbe_result *out);

/*
 * Device memory a mbe_count of g with these options holds: *bytes receives the sum of the
 * graph upload (host graphs), the preparation arrays (ranking keys, order, rank, sort
 * temporaries) and the search arena (per-workgroup universe, top-level list and per-wave
 * stacks, sized from the largest 2-hop neighbourhood of a candidate) with its work-sharing
 * slots.  It runs the preparation (validation and ranking, which give the neighbourhood
 * bound) on the device but no search.  Later calls on a device start from the largest stack
 * room earlier ones needed, which is included.  mbe_enumerate adds its record staging:
 * about 12 bytes per int of buf_cap_ints plus the sort temporaries.  The memory stays with
 * the library (per device) for later calls.  Errors as mbe_count; MBE_ERR_INVALID_ARG if
 * bytes is NULL.  An empty side or zero edges gives 0.
 */
int mbe_workspace_size(const mbe_graph *g, const mbe_options *opt, size_t *bytes);

/*
 * The load study of section IV (the per-block time distribution of its evaluation): mbe_count
 * with diagnostics = 2, also returning one record per workgroup of every search launch of the
 * call: rec[4i .. 4i+3] = (mask words of the launch's class, 0 for the wide search; start and
 * end of the workgroup in nanoseconds from the earliest start of the call; nanoseconds it
 * spent finding work: claiming top-level candidates, scanning for lists to share, waiting
 * while others were busy).  Times come from the device wall clock.  A workgroup is busy for
 * (end - start - wait) of the launch.  *n_records receives the number of records; when it
 * exceeds cap_records the call returns MBE_ERR_BUFFER_TOO_SMALL with out complete and rec
 * unspecified.  Errors as mbe_count, plus MBE_ERR_INVALID_ARG (out or n_records NULL,
 * cap_records < 0, rec NULL with cap_records > 0).
 */
int mbe_count_loads(const mbe_graph *g, const mbe_options *opt, mbe_result *out, uint64_t *rec,
                    int64_t cap_records, int64_t *n_records);

/*
 * For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: mbe_count without any allocation.  The
 * result is the one mbe_count returns.  Every device buffer of the call (graph copy for host
 * graphs, ranking arrays and sort temporaries, search arena, sharing slots, accumulators) is
 * carved from a fixed scratch array of MBE_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends; the call makes no hipMalloc or hipFree and
 * no allocating library call.  Set-up, once per device at the first such call there (that
 * device current): the address of the device's scratch copy is looked up, and the library's
 * per-device timing events are created.
 *   - The caller passes the graph (host or device arrays, as for mbe_count) and out.
 *   - The mask-width class launches run one after another on opt->stream, and the search grid
 *     is cut down to the arena slots that fit in the scratch (results do not depend on it).
 *   - A call that would need more than the scratch holds (even one arena slot, or the
 *     ranking arrays) returns MBE_ERR_SCRATCH_LIMIT.  Roughly: the ranking needs
 *     ~40 bytes per candidate-side vertex, and one arena slot ~ (8 W + 40) bytes per vertex of
 *     the largest 2-hop neighbourhood plus ~ 8 waves x (16 bytes per such vertex + 64 KiB).
 *   - The scratch keeps the last call's contents; each call clears what must start at zero.
 *     Calls on one device are serialised by the library's per-device lock, so two calls never
 *     use the scratch at once; work the caller enqueues on the stream meanwhile must not
 *     touch it either.
 *   - mbe_enumerate, the batched form and the server have no such variant.
 * Errors as mbe_count, plus MBE_ERR_SCRATCH_LIMIT.
 */
#define MBE_NOALLOC_SCRATCH_BYTES (256u << 20)
int mbe_count_noalloc(const mbe_graph *g, const mbe_options *opt, mbe_result *out);

/*
 * As mbe_count, and also write the bicliques to buf as records
 *     [|A|, |B|, a_1 < ... < a_|A|, b_1 < ... < b_|B|]     (A in U, B in V)
 * sorted by A lexicographically (a total order: A determines B).  buf holds buf_cap_ints
 * int32 values; buf_on_device = 1 if it is device memory, 0 if host memory.  When the
 * records need more than buf_cap_ints ints the call returns MBE_ERR_BUFFER_TOO_SMALL with
 * out fully filled (out->out_ints is the size needed) and buf's contents unspecified.
 */
int mbe_enumerate(const mbe_graph *g, const mbe_options *opt, mbe_result *out,
                  int32_t *buf, uint64_t buf_cap_ints, int32_t buf_on_device);

/*
 * Count and hash the maximal bicliques of each of n independent graphs in one pass (the
 * batched form of mbe_count).  The graphs are packed as a disjoint union, each keeping its
 * own candidate side (mbe_options.side applies to all of them), ranked per graph on the
 * device, and searched by one persistent kernel per mask-width class over a shared work
 * list ordered by mask class and then by decreasing candidate degree.  outs[i] receives
 * graph i's mbe_result, equal to what mbe_count would return for it; kernel_ms is the device
 * time of the whole batch.  Host graphs only (on_device = 0); root_lo / root_hi are ignored.
 * Errors as mbe_count; on MBE_ERR_INVALID_GRAPH no graph is searched.  Packed totals (candidate-side and other-side
 * vertices, edges, summed in 64 bits over the graphs with edges) must each stay below 2^31 - 1,
 * else MBE_ERR_INVALID_ARG before any device work.
 */
int mbe_count_batch(const mbe_graph *gs, int32_t n, const mbe_options *opt, mbe_result *outs);

/*
 * Autotuner of the batched form: runs mbe_count_batch on the given graphs (a representative
 * sample of the batches to come) under each candidate launch setting -- waves per workgroup
 * in {8, 4, 2} times steal_k in {2, 3} -- starting from base (NULL: defaults), checks that
 * every setting gives the same per-graph count and hash, and writes the fastest setting
 * (wall time of the whole call) to *best and its time in milliseconds to *best_ms (may be
 * NULL).  Errors as mbe_count_batch; MBE_ERR_DEVICE if two settings disagree.
 */
int mbe_tune_batch(const mbe_graph *gs, int32_t n, const mbe_options *base, mbe_options *best, double *best_ms);

/* ------------------------------------------------------------------------- serving */
/*
 * A server runs enumeration requests with continuous batching.  Each of its slots (a host
 * thread with its own HIP stream and a device workspace that stays allocated between
 * batches) takes the queued requests in arrival order while their estimated device
 * footprint (CSR, preparation arrays, and the search arena of the largest local universe)
 * fits the slot's share of hbm_budget_bytes, and runs them as one mbe_count_batch pass.
 * With slots >= 2 a new batch starts while another is still on the device.  A request's
 * result is the one mbe_count returns for its graph alone.
 *   hbm_budget_bytes  device memory the slots may plan for (0: half of the free memory)
 *   slots             concurrent batches (1..8; default 2)
 *   max_batch         most requests per batch (default 4096)
 *   small_edges       with slots >= 2, slot 0 is reserved for requests with at most this many
 *                     edges, so that small requests do not queue behind large ones
 *                     (default 65536; negative: no reserved slot)
 *   search            per-search options (side, wg_waves, grid, diagnostics, no_validate)
 *   request_timeout_ms  deadline of every request submitted with mbe_server_submit, counted
 *                     from its submission (0: none); see mbe_server_submit_timeout
 *
 * Deadlines and cancellation: a request that passes its deadline, or is cancelled, before a
 * slot took it leaves the queue at once.  One that is already on the device stops being
 * worked on: its top-level candidates that no workgroup has claimed are skipped (each graph
 * of a batch has a word in pinned host memory that the search reads before it claims a
 * candidate of that graph), while those in flight run to their end, so the batch it shares
 * finishes early by what the skipped candidates would have cost.  Either way its wait
 * returns MBE_ERR_TIMEOUT or MBE_ERR_CANCELLED with an unspecified result; the other
 * requests of the batch are not affected.
 */
typedef struct mbe_server mbe_server;
typedef struct mbe_server_options {
    size_t hbm_budget_bytes;
    int32_t slots;
    int32_t max_batch;
    int64_t small_edges;
    mbe_options search;
    double request_timeout_ms;
} mbe_server_options;

/* Start a server on the current device (opt may be NULL).  *out receives the handle. */
int mbe_server_create(const mbe_server_options *opt, mbe_server **out);

/* Queue a host graph (copied before the call returns); *ticket identifies the request.  Its
 * deadline is the server's request_timeout_ms. */
int mbe_server_submit(mbe_server *s, const mbe_graph *g, uint64_t *ticket);

/* mbe_server_submit with a deadline of timeout_ms after submission for this request
 * (0: none; negative or NaN: MBE_ERR_INVALID_ARG). */
int mbe_server_submit_timeout(mbe_server *s, const mbe_graph *g, double timeout_ms, uint64_t *ticket);

/* Cancel a request that has not been waited for: its wait returns MBE_ERR_CANCELLED unless
 * it was already done (then the cancellation has no effect).  MBE_ERR_INVALID_ARG for an
 * unknown ticket. */
int mbe_server_cancel(mbe_server *s, uint64_t ticket);

/* Block until the request is done; out receives its result and latency_ms (may be NULL)
 * the time from submission to completion.  Returns the request's status.  A ticket can be
 * waited for once. */
int mbe_server_wait(mbe_server *s, uint64_t ticket, mbe_result *out, double *latency_ms);

/* Finish the queued requests, stop the slots and free their device memory. */
int mbe_server_destroy(mbe_server *s);

/* Human-readable name of a return code (static storage; never NULL). */
const char *mbe_strerror(int code);

/* Library version as "major.minor.patch" (static storage). */
const char *mbe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MBE_H */
