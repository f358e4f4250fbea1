// Internal declarations shared by the C-ABI layer (mbe_api.hip) and the kernels
// (mbe_search.hip, mbe_prep.hip, mbe_records.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mbe {

// Accumulator slots (unsigned long long each) written by the search kernels.
enum AccSlot : int {
    ACC_COUNT = 0,
    ACC_HASH = 1,
    ACC_OUT_INTS = 2,
    ACC_NODES = 3,
    ACC_NONMAX = 4,
    ACC_BYTES = 5,
    ACC_MAX_DEPTH = 6,
    ACC_RECORDS = 7,    // records reserved in the record arena
    ACC_REC_INTS = 8,   // ints reserved in the record arena
    ACC_NEED_UCAP = 9,  // largest universe met (max), for resizing after an overflow
    ACC_SHARED = 10,    // third-level chunks searched by a wave other than the list's owner
    ACC_PHASE = 11,     // 6 slots: shader-clock cycles per search phase (diagnostics only)
    ACC_DBYTES = 17,    // design-byte tally of the production search (tally instances only)
    ACC_SLOTS = 24,
};

// Search phases timed in diagnostics mode (cycles summed over waves).
enum Phase : int {
    PH_ROOT = 0,    // top-level candidate: reverse scans, universe, child list and its tables
    PH_LIGHT = 1,   // 64-candidate chunks: settling the |R'| = 1 candidates
    PH_CHECK = 2,   // |R'| >= 2 candidates: maximality test
    PH_EXPAND = 3,  // maximal candidates: scan of the list, expansion, report
    PH_CHILD = 4,   // building child lists and their tables
    PH_WAIT = 5,    // waiting for the workgroup, stealing, claiming
    PH_COUNT = 6,
};

// Status bits raised by kernels.
enum FlagBits : unsigned int {
    FLAG_STACK_OVERFLOW = 1u << 0,     // a wave's explicit stack was too small: rerun larger
    FLAG_DEPTH_OVERFLOW = 1u << 1,     // frame-header array too small: rerun larger
    FLAG_RECORD_OVERFLOW = 1u << 2,    // record arena too small (count/hash still exact)
    FLAG_BAD_GRAPH = 1u << 3,          // validation failure
    FLAG_DEGREE = 1u << 4,             // candidate degree above the supported mask width
    FLAG_UNIVERSE_OVERFLOW = 1u << 5,  // a local universe or its posting lists did not fit
    FLAG_NO_SLOT = 1u << 6,            // a workgroup found no free arena slot: rerun one class at a time
    FLAG_SHARE_MISMATCH = 1u << 7,     // a rebuilt third-level list was not its owner's (internal error)
};
constexpr unsigned int FLAG_RERUN = FLAG_STACK_OVERFLOW | FLAG_DEPTH_OVERFLOW | FLAG_UNIVERSE_OVERFLOW | FLAG_NO_SLOT;

// Capacities of the search arena.
struct SearchDims {
    int32_t ucap;      // local-universe capacity (entries)
    int32_t nwords;    // words of the rank bitmap
    int32_t Wmax;      // widest mask class in use (words)
    int32_t waves;     // waves per workgroup
    int64_t scap;      // per-wave stack capacity (32-bit words)
    int32_t maxdepth;  // per-wave frame headers
    int32_t pad;
};

// Byte offsets of the per-workgroup and per-wave regions of the search arena.
struct ArenaLayout {
    size_t wg_bytes;    // stride between workgroups
    size_t off_bitmap;  // u64[nwords]          membership bitmap over candidate ranks
    size_t off_bpre;    // u32[nwords+1]        popcount prefix of the bitmap words
    size_t off_M;       // u64[ucap*Wmax]       neighbour masks of the local universe
    size_t off_gid;     // i32[ucap]            global id of each universe entry
    size_t off_cnt;     // u32[ucap]            top-level counts |N(v) n N(x)|
    size_t off_hv;      // u64[64*Wmax]         R-side hash term of each position of N(x)
    size_t off_deg;     // u32[64*Wmax]         degree of each position of N(x)
    size_t off_t1v;     // u32[ucap]            sort staging (ids)
    size_t off_t1c;     // u32[ucap]            sort staging (keys)
    size_t off_S1;      // u32[s1_words]        the top-level node's child list as a frame
    size_t off_hb;      // u64[ucap/64+1]       top-level candidates with |R'| >= 2, per chunk
    size_t off_hpre;    // u32[ucap/64+2]       popcount prefix of those words
    size_t off_hpos;    // u32[ucap]            their positions, in list order
    size_t s1_words;
    size_t off_waves;   // start of the per-wave regions
    size_t wave_bytes;  // stride between waves
    size_t off_w_stack; // u32[scap]            frames (lists, masks, per-bit tables)
    size_t off_w_u;     // u32[ucap]            a maximal node's entries, in list order
    size_t off_w_hdr;   // frame headers[maxdepth]
};

// Arena of the wide search (top-level candidates of degree above 64 * 16, any width): per
// workgroup slot, then per wave.  Masks of a universe entry take Wx words.
struct WideLayout {
    int32_t Wx;          // words of a universe mask: ceil(largest top-level degree / 64)
    int32_t reps;        // workgroups that rebuild one top-level candidate and share its chunks
    int64_t scap;        // per-wave stack capacity (32-bit words)
    int32_t maxdepth;    // per-wave frame headers
    int32_t pad;
    size_t wg_bytes;     // stride between workgroup slots
    size_t off_bitmap;   // u64[nwords]            membership bitmap over candidate ranks
    size_t off_bpre;     // u32[nwords+1]          its popcount prefix
    size_t off_M;        // u64[ucap*Wx]           neighbour masks of the local universe
    size_t off_gid;      // i32[ucap]              global id of each universe entry
    size_t off_cnt;      // u32[ucap]              top-level counts
    size_t off_hv;       // u64[64*Wx]             R-side hash term per position of N(x)
    size_t off_deg;      // u32[64*Wx]             degree per position of N(x)
    size_t off_t1v;      // u32[ucap]              sort staging (ids)
    size_t off_t1c;      // u32[ucap]              sort staging (keys)
    size_t off_whist;    // u32[64*Wx+1]           top-level sort histogram
    size_t off_S1;       // the top-level list as a frame
    size_t off_waves;    // start of the per-wave regions
    size_t wave_bytes;   // stride between waves
    size_t off_w_stack;  // u32[scap]              frames
    size_t off_w_u;      // u32[ucap]              a maximal node's entries, in list order
    size_t off_w_u2;     // u32[ucap]              (candidate pruning) the same, regrouped
    size_t off_w_bl;     // u32[64*Wx]             the bits of a node's R'
    size_t off_w_hist;   // u32[64*Wx+2]           counting-sort histogram of a child list
    size_t off_w_mr;     // u64[Wx]                a node's R' words
    size_t off_w_rr;     // u64[Wx]                R' as positions of N(x) (records)
    size_t off_w_hdr;    // frame headers[maxdepth]
};

// One graph of the packed candidate-orientation arrays.  A single call has one; a batch
// packs its graphs as a disjoint union, each graph in its own orientation.
struct GraphDesc {
    const int32_t *order;       // order[r]: packed candidate id of local rank r
    unsigned long long *acc;    // this graph's ACC_SLOTS accumulators
    unsigned long long total_fw;// sum over its candidates of (2 + deg v), for the byte tally
    int32_t ncand;              // candidates of degree > 0
    int32_t nwords;             // words of its rank bitmap
    int32_t c_is_v;             // its candidate side is V
    int32_t cbase, obase;       // first packed id of its candidate / other side
    int32_t pad;
};

// Work-stealing slot of one workgroup: while it searches a top-level candidate whose child
// list has more than one 64-candidate chunk left, word = (epoch << 32) | chunks claimed so
// far (in candidates) and the other fields name the task; word = 0 otherwise.
struct StealSlot {
    unsigned long long word;
    int32_t g, k, limit, pad;
    unsigned long long pad2;
};

// Third-level sharing slot of one wave (steal_k >= 3): while the wave searches the child list
// of a second-level node and others are idle, word = (epoch << 32) | 64-candidate chunks of
// that list claimed so far, and the other fields name the list: graph g, top-level rank k,
// limit = number of chunks, position i1 of the second-level node in the top-level list, first
// = list position of chunk 0.  word = 0 otherwise.  Epochs come from a per-launch counter, so
// a claim against a withdrawn list always fails.  word, g, k and limit sit where they sit in a
// StealSlot, and the two have the same size: idle workgroups scan both kinds with one loop.
struct PubSlot {
    unsigned long long word;
    int32_t g, k, limit, i1, first, pad;
};
static_assert(sizeof(PubSlot) == sizeof(StealSlot), "slot kinds share a stride");
static_assert(offsetof(PubSlot, limit) == offsetof(StealSlot, limit), "slot kinds share a head");

struct SearchArgs {
    // packed graph(s) in candidate orientation: rows of c_off / c_adj are candidates, ids in
    // c_adj are other-side ids and vice versa
    const int32_t *c_off, *c_adj, *o_off, *o_adj;
    const int32_t *rank;   // rank[v]: local rank of candidate v within its graph, -1 if deg v = 0
    const GraphDesc *graphs;
    // work list: tasks[t] = (graph << 32) | local rank; NULL means graph 0, ranks [lo, hi)
    const unsigned long long *tasks;
    // arena
    char *arena;
    SearchDims dims;
    ArenaLayout lay;
    StealSlot *steal;           // one per arena slot for this launch's mask class, zeroed first
    int32_t steal_on;           // 0: no stealing (each top-level candidate stays in one workgroup)
    unsigned int *steal_live;   // number of this launch's slots currently published (zeroed first)
    int32_t nslots;             // arena slots shared by the concurrent launches
    int32_t k3;                 // 1: third-level lists are shared too (steal_k >= 3)
    PubSlot *pub;               // nslots * pubw third-level slots of this launch (zeroed first)
    int32_t pubw;               // slots per arena slot (waves per workgroup)
    unsigned int *pub_live;     // third-level slots currently published (zeroed first)
    unsigned int *busy;         // workgroups holding a task (zeroed first)
    unsigned int *hungry;       // workgroups waiting for work while others are busy (zeroed first)
    unsigned int *epoch_ctr;    // source of third-level epochs (zeroed first)
    int32_t cls;                // mask class of this launch
    const unsigned int *cls_ctr;  // top-level candidate counters of the five class launches
    int64_t cls_n[5];           // top-level candidates of each class launch
    unsigned int *slot_busy;    // nslots flags: a slot is held by a running workgroup
    // outputs
    unsigned long long *acc;    // run-wide slots (overflow sizes, record cursors)
    unsigned int *flags;
    // wide search (wide_kernel only): its own arena of workgroup slots, one chunk counter per
    // top-level candidate of the launch (zeroed first)
    char *warena;
    WideLayout wl;
    unsigned int *wide_items;
    // candidate pruning (wide search only, when not NULL): twin[v] = the lowest rank of a
    // candidate whose row equals v's
    const int32_t *twin;
    // pivot rule (wide search only, when nonzero): child lists are regrouped around a pivot
    int32_t pivot;
    // load records (tally instances only, when not NULL): per workgroup of the launch, its
    // start and end on the wall clock and the time it spent finding work (3 u64 each)
    unsigned long long *wg_load;
    // cancellation (batched work lists only, when not NULL): one word per graph in host
    // memory that the device reads at system scope; a graph whose word is nonzero has its
    // top-level candidates that no workgroup has claimed yet skipped (those in flight finish)
    const unsigned int *cancel;
    // record arena (mbe_enumerate only)
    int32_t *rec;
    unsigned long long rec_cap;
    unsigned long long *rec_offs;
    unsigned long long rec_offs_cap;
};

// Arena layout for the given capacities (host side).
ArenaLayout search_layout(const SearchDims &d);

// Workgroups of one search launch that fit on a compute unit at once (nwords: words of the
// launch's rank bitmap, which small graphs keep in LDS).
int search_occupancy(int W, bool diag, bool enumerate, int waves, int nwords);

// Launch the search over tasks [lo, hi) of the work list (or ranks [lo, hi) of graph 0 when
// it is NULL), all of whose top-level candidates have degree at most 64*W.  counter must be
// zero.  tb (diag and enumerate off): the production search that also tallies its design
// bytes into ACC_DBYTES.
hipError_t launch_search(const SearchArgs &a, int W, bool diag, bool enumerate, bool tb, int64_t lo,
                         int64_t hi, unsigned int *counter, int grid, int waves, hipStream_t s);

// Wide search: layout for the given capacities (Wx words per universe mask), and the launch
// over tasks [lo, hi) of the work list (or ranks [lo, hi) of graph 0), each of whose
// top-level candidates is shared by wl.reps workgroups; counter must be zero.
WideLayout wide_layout(const SearchDims &d, int Wx, int64_t scap, int32_t maxdepth, int waves);
// prune: 0 the plain search, 1 iMBEA's candidate pruning (a.twin set), 2 the pivot rule.
hipError_t launch_wide(const SearchArgs &a, bool diag, bool enumerate, bool tb, int64_t lo, int64_t hi,
                       unsigned int *counter, int grid, int waves, hipStream_t s, int prune = 0);

// Graph preparation and validation (mbe_prep.hip).
hipError_t launch_validate(int32_t n_u, int32_t n_v, int32_t n_edges, const int32_t *u_off, const int32_t *u_adj,
                           const int32_t *v_off, const int32_t *v_adj, unsigned int *flags, hipStream_t s);
// keys[v] = (deg v << 32) | v for every candidate; also counts candidates per mask class and
// bounds the local universes (see mbe_prep.hip).
hipError_t launch_rank_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                            unsigned long long *keys, unsigned long long *stats, hipStream_t s);
hipError_t launch_rank_scatter(int32_t nc, int32_t nzero, const unsigned long long *sorted,
                               int32_t *order, int32_t *rank, hipStream_t s);
hipError_t radix_sort_u64(void *temp, size_t *temp_bytes, const unsigned long long *in,
                          unsigned long long *out, int32_t n, int end_bit, hipStream_t s);

// Zero fills by kernel (mbe_prep.hip): bytes and width_bytes are multiples of 4, pointers
// 4-byte aligned; the 2-D form clears rows runs of width_bytes spaced pitch bytes apart.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_zero_2d(void *base, size_t pitch, size_t width_bytes, size_t rows, hipStream_t s);

// Twins for the candidate pruning (mbe_prep.hip): row keys, their sort, and twin[v] = the
// lowest rank with v's exact row.
hipError_t launch_row_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, unsigned long long *key,
                           unsigned int *val, hipStream_t s);
hipError_t sort_pairs_u64_u32(void *temp, size_t *temp_bytes, const unsigned long long *kin, unsigned long long *kout,
                              const unsigned int *vin, unsigned int *vout, int32_t n, hipStream_t s);
hipError_t launch_twins(int32_t nc, const unsigned long long *key, const unsigned int *val, const int32_t *c_off,
                        const int32_t *c_adj, const int32_t *rank, int32_t *twin, hipStream_t s);

// Batched preparation (mbe_prep.hip).
hipError_t launch_batch_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                             const int32_t *graph_of, const int32_t *cbase, unsigned long long *keys,
                             unsigned long long *gstats, unsigned long long *stats, hipStream_t s);
hipError_t launch_batch_scatter(int32_t nc, const unsigned long long *sorted, const int32_t *graph_of,
                                const int32_t *cbase, const unsigned long long *gstats, int32_t *order, int32_t *rank,
                                unsigned int *task_key, unsigned long long *task, const int32_t *tbase,
                                hipStream_t s);
hipError_t segmented_sort_u64(void *temp, size_t *temp_bytes, const unsigned long long *in, unsigned long long *out,
                              int32_t n, int32_t nseg, const int32_t *seg_begin, const int32_t *seg_end, int end_bit,
                              hipStream_t s);
hipError_t sort_pairs_u32_u64(void *temp, size_t *temp_bytes, const unsigned int *kin, unsigned int *kout,
                              const unsigned long long *vin, unsigned long long *vout, int32_t n, int end_bit,
                              hipStream_t s);

// Record canonicalisation (mbe_records.hip).
hipError_t canonical_records(const int32_t *rec, unsigned long long *offs, unsigned long long n_rec,
                             unsigned long long *offs_tmp, unsigned long long *lens,
                             int32_t *out, void *temp, size_t *temp_bytes, hipStream_t s);

}  // namespace mbe
