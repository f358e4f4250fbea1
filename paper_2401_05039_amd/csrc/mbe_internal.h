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
    ACC_RECORDS = 7,   // records reserved in the record arena
    ACC_REC_INTS = 8,  // ints reserved in the record arena
    ACC_SLOTS = 16,
};

// Status bits raised by kernels.
enum FlagBits : unsigned int {
    FLAG_STACK_OVERFLOW = 1u << 0,   // a wave's explicit stack was too small: rerun larger
    FLAG_DEPTH_OVERFLOW = 1u << 1,   // frame-header array too small: rerun larger
    FLAG_RECORD_OVERFLOW = 1u << 2,  // record arena too small (count/hash still exact)
    FLAG_BAD_GRAPH = 1u << 3,        // validation failure
    FLAG_DEGREE = 1u << 4,           // candidate degree above the supported mask width
};

// Byte offsets of the per-workgroup and per-wave regions of the search arena.
struct ArenaLayout {
    size_t wg_bytes;      // stride between workgroups
    size_t off_bitmap;    // u64[nwords]     membership bitmap over candidate ranks
    size_t off_bpre;      // u32[nwords+1]   popcount prefix of the bitmap words
    size_t off_M;         // u64[ucap*W]     neighbour masks of the local universe
    size_t off_gid;       // i32[ucap]       global id of each universe entry
    size_t off_cnt;       // u32[ucap]       top-level counts |N(v) n N(x)|
    size_t off_hv;        // u64[64*Wmax]    hash term of each local other-side vertex
    size_t off_deg;       // u32[64*Wmax]    degree of each local other-side vertex
    size_t off_S1;        // u32[ucap]       the top-level node's child candidate list
    size_t off_t1v;       // u32[ucap]       sort staging (ids)
    size_t off_t1c;       // u32[ucap]       sort staging (keys)
    size_t off_waves;     // start of the per-wave regions
    size_t wave_bytes;    // stride between waves
    size_t off_w_stack;   // u32[scap]       explicit DFS stack of candidate lists
    size_t off_w_tv;      // u32[ucap]       child staging (ids)
    size_t off_w_tc;      // u32[ucap]       child staging (keys)
    size_t off_w_hdr;     // frame headers[maxdepth]
};

struct SearchArgs {
    // graph in candidate orientation
    int32_t nc, no, ncand, c_is_v;
    const int32_t *c_off, *c_adj, *o_off, *o_adj;
    const int32_t *order;  // order[r]: candidate of rank r (ascending (deg, id), deg > 0)
    const int32_t *rank;   // rank[v]: rank of candidate v, -1 if deg v = 0
    uint64_t total_fw;     // sum over candidates of (2 + deg v), for the byte tally
    // arena
    char *arena;
    ArenaLayout lay;
    int32_t ucap, scap, maxdepth, nwords;
    // outputs
    unsigned long long *acc;
    unsigned int *flags;
    // record arena (mbe_enumerate only)
    int32_t *rec;
    unsigned long long rec_cap;
    unsigned long long *rec_offs;
    unsigned long long rec_offs_cap;
};

// Launch the search over the candidates of rank [lo, hi), all of whose degrees are at most
// 64*W for the given mask width class.  counter must be zero.
hipError_t launch_search(const SearchArgs &a, int W, bool diag, bool enumerate, int64_t lo,
                         int64_t hi, unsigned int *counter, int grid, int waves, size_t lds_bytes,
                         hipStream_t s);

size_t frame_header_bytes(int W);
size_t search_lds_bytes(int W, int waves);

// Graph preparation and validation (mbe_prep.hip).
hipError_t launch_validate(int32_t n_rows, int32_t n_cols, int32_t n_edges, const int32_t *off,
                           const int32_t *adj, const int32_t *t_off, const int32_t *t_adj,
                           unsigned int *flags, hipStream_t s);
// keys[v] = (deg v << 32) | v for every candidate; also counts candidates per mask class.
hipError_t launch_rank_keys(int32_t nc, const int32_t *c_off, unsigned long long *keys,
                            unsigned long long *stats, hipStream_t s);
hipError_t launch_rank_scatter(int32_t nc, int32_t nzero, const unsigned long long *sorted,
                               int32_t *order, int32_t *rank, hipStream_t s);
hipError_t radix_sort_u64(void *temp, size_t *temp_bytes, const unsigned long long *in,
                          unsigned long long *out, int32_t n, int end_bit, hipStream_t s);

// Record canonicalisation (mbe_records.hip).
hipError_t canonical_records(const int32_t *rec, unsigned long long *offs, unsigned long long n_rec,
                             unsigned long long *offs_tmp, unsigned long long *lens,
                             int32_t *out, void *temp, size_t *temp_bytes, hipStream_t s);

}  // namespace mbe
