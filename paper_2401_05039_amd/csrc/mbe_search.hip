// Depth-first MBEA search on gfx950 (wave64).
//
// What is computed: the maximal bicliques of Algorithm 1 (MBEA, section II-B), in the
// library's letters: the candidate x joins the growing set L (candidate side C), the
// shrinking set R (other side O) becomes R' = R n N(x), the maximality check fails when a
// vertex of Q is adjacent to all of R', the expansion moves every candidate of P adjacent
// to all of R' into L', and P' / Q' keep the vertices with 0 < |N(v) n R'| < |R'|.  The
// counts come from reverse scanning (section III-E): walk the vertices of R' and their
// neighbours rather than every candidate's list.  Candidates are taken in ascending count
// (sections II-C and III-E), ties in the order of the parent's list.
//
// How it maps to the hardware (the build's own design, not the paper's CUDA one):
//
//  * Coarse grain (section III-C's first-level subtrees): one workgroup owns one top-level
//    candidate x at a time, claimed from a global atomic counter, largest degree first.
//
//  * Local universe.  Every vertex below x is a 2-hop neighbour of x and every R below x is
//    a subset of N(x).  The workgroup runs the reverse scan over N(x) once and gives each
//    2-hop neighbour v the mask M[v] = N(v) n N(x) over the positions of N(x) (W 64-bit
//    words).  Universe entries are numbered in top-level rank order, so the top-level Q is
//    a prefix.  Below the top level the CSR is never read again.
//
//  * Frames.  A frame is the candidate list of one search node: entry k carries its mask
//    restricted to the frame's R, so a child's R' is simply the candidate's own mask.  When
//    |R| <= 64 the masks are compressed to |R| bits (one word).  Each frame also holds
//    inverted per-bit tables -- the paper's reverse scan turned into an index: for every bit
//    b of R, the first list position with b, the number of entries with b, the sum of their
//    L-side hash terms and the posting list of positions with b.
//
//  * Nodes.  A candidate at position i with |R'| = 1 (almost every node on power-law
//    graphs) is settled by one lookup: it is maximal exactly when the first entry with its
//    bit is itself, and then L' is every entry with that bit.  The 64 lanes of a wave settle
//    64 such candidates at once.  Candidates with |R'| >= 2 are handled by the whole wave:
//    a maximality test on the rarest bit's posting list, and for maximal nodes one scan of
//    the list that counts, compacts (ballot + prefix sum) and stably counting-sorts P'.
//
//  * Second level (the paper's k = 2 subtrees): the waves of the workgroup claim 64-wide
//    chunks of the top-level node's child list from an LDS counter; each wave then runs its
//    own depth-first search on an explicit stack of frames (section III-B's goal: no
//    recursion and no allocation; frames are laid back to back in one preallocated array).
//
// Counts and hashes are commutative u64 sums, so results do not depend on which lane, wave
// or workgroup settled which node.

#include "mbe_internal.h"

namespace mbe {

namespace {

constexpr uint64_t kHashK = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kShared = 0xFFFFFFFFu;
constexpr uint32_t kMovedMark = 1u << 30;  // added to the LDS item counter when the list moves  // frame offset meaning "the workgroup's top-level list"
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kQKeep = 256;      // most incomparable Q' masks a compressed child keeps
// classes that reduce Q' through the presence word when |R'| <= 6 (the widest class runs out
// of scalar registers with it)
template <int W>
constexpr bool kSmallRPrune = W <= 4;
// A maximal node's listed entries (stu) stay in the wave's LDS for lists of at most this many
// entries, in global scratch for longer ones.
constexpr int kStuLds = 256;
constexpr int kWaveLds = 1024 + 8 * kQKeep + 4 * kStuLds;  // LDS bytes per wave besides the histogram
// The fixed-width classes keep a graph's rank bitmap and its popcount prefix in LDS, after the
// waves' regions, when the bitmap has at most this many words (131,072 candidates); larger
// graphs keep them in the workgroup's arena slot.
constexpr int kRankLdsWords = 2048;
__host__ __device__ constexpr size_t rank_lds_bytes(int nwords) {
    return nwords <= kRankLdsWords ? ((size_t)nwords * 12 + 4 + 15) / 16 * 16 : 0;
}

// LDS after the workgroup header: the waves' histograms (4 bytes per bit each), which the
// top-level list build reuses for its tables (16 bytes per bit), hence at least that much.
__host__ __device__ constexpr size_t hist_region_bytes(int bits, int waves) {
    return (size_t)bits * (waves >= 4 ? 4 * (size_t)waves : 16);
}

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
__device__ __forceinline__ uint64_t hash_u(int32_t a) { return mix64(kHashK * (2ull * (uint64_t)(uint32_t)a + 1ull)); }
__device__ __forceinline__ uint64_t hash_v(int32_t b) { return mix64(kHashK * (2ull * (uint64_t)(uint32_t)b + 2ull)); }
__device__ __forceinline__ uint64_t pair_hash(int c_is_v, uint64_t sL, uint64_t sR) {
    // h(A, B) = mix(sum hu(A) + mix(sum hv(B) + K)); A is the U side.
    return c_is_v ? mix64(sR + mix64(sL + kHashK)) : mix64(sL + mix64(sR + kHashK));
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Wave-uniform values moved to scalar registers (the value of the first active lane; only
// for values every lane holds alike).
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t uni(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | (uint64_t)uni((uint32_t)x);
}
// lane 63's value (a wave-wide scan total) in a scalar register
__device__ __forceinline__ int last_lane(int x) { return __builtin_amdgcn_readlane(x, 63); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return uni(v);
}
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return uni(v);
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return uni(v);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return uni(v);
}
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int ln = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (ln >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t align2(uint32_t x) { return (x + 1u) & ~1u; }

// Global atomics are performed in L2, so a plain load issued after them may still be served
// from a stale line in this compute unit's vector L1, or overtake them.  After a phase that
// builds data with global atomics (and its barrier, if other waves read it), every reading
// wave waits for its memory operations and invalidates the L1.  The data involved is private
// to one workgroup, hence on one compute unit and one L2: the L2 stays valid.
// Wait until this wave's memory operations are done, so that plain stores made by some
// lanes are in place before other lanes load them.
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void see_atomics() {
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("buffer_inv sc0" ::: "memory");
}

// Whether the graph of work-list entry ti has been cancelled by the host (batched calls of a
// server only): the word lives in host memory, so it is read at system scope.
__device__ __forceinline__ bool root_cancelled(const SearchArgs &a, int64_t ti) {
    if (!a.cancel || !a.tasks) return false;
    const int g = (int)(a.tasks[ti] >> 32);
    return __hip_atomic_load(a.cancel + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u;
}

// Workgroup memory (LDS) pointers carry their address space, so that accesses and atomics
// through them are LDS instructions even where the compiler cannot trace them to the shared
// array (through a generic pointer they would be flat instructions).
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
template <typename T>
__device__ __forceinline__ T *lds_at(unsigned char *base, size_t off) {
    return (T *)(base + off);
}
__device__ __forceinline__ uint32_t lds_add32(lds_u32 *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_min32(lds_u32 *p, uint32_t v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add64(lds_u64 *p, uint64_t v) {
    __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(void *p, uint64_t v) {
    __hip_atomic_fetch_add((lds_u64 *)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_max(void *p, uint64_t v) {
    __hip_atomic_fetch_max((lds_u64 *)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_or(void *p, uint64_t v) {
    __hip_atomic_fetch_or((lds_u64 *)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Set bits of a rank-bitmap word, in the workgroup's arena slot or in LDS.
__device__ __forceinline__ void bm_or(uint64_t *p, uint64_t v) {
    atomicOr(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
__device__ __forceinline__ void bm_or(lds_u64 *p, uint64_t v) {
    __hip_atomic_fetch_or(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------------------------------ frames

// Registers of the frame a wave is working on; saved whole in the header array on descent.
struct FrameState {
    uint32_t off;    // 32-bit-word offset of the frame's data in the wave stack, or kShared
    uint32_t top;    // first free stack word above this frame
    int32_t n;       // list length
    int32_t nq;      // positions [0, nq) are the node's Q; candidates are [nq, n)
    int32_t level;   // search depth of the candidates taken from this list (top level = 1)
    int32_t nL;      // |L| of the nodes below
    int32_t wf;      // mask words per entry
    int32_t narrow;  // 1: bits are compressed positions of R, mapped by orig[] to N(x) positions
    int32_t chunk;   // base position of the current 64-candidate chunk
    int32_t rbits;   // rows held by the frame: mask bits [0, rbits) can be set
    uint64_t heavy;  // lanes of the current chunk still to be handled one by one
    uint64_t sL;     // sum of the L-side hash terms of L
    uint64_t fw;     // sum over the list of (2 + deg v), byte tally only
};

__device__ __forceinline__ FrameState uni_frame(const FrameState &f) {
    FrameState u;
    u.off = uni(f.off);
    u.top = uni(f.top);
    u.n = uni(f.n);
    u.nq = uni(f.nq);
    u.level = uni(f.level);
    u.nL = uni(f.nL);
    u.wf = uni(f.wf);
    u.narrow = uni(f.narrow);
    u.chunk = uni(f.chunk);
    u.rbits = uni(f.rbits);
    u.heavy = uni(f.heavy);
    u.sL = uni(f.sL);
    u.fw = uni(f.fw);
    return u;
}

// Word layout of a frame's data starting at a 2-aligned offset o:
//   ids[n] | hs[n] (u64) | masks[n][wf] (u64) | first[64wf] | cnt[64wf] | H[64wf] (u64) |
//   orig[64] | rows[rbits][nw] (u64), nw = ceil(n / 64)
// ids are universe indices (kept for diagnostics), hs the L-side hash term of each entry.
// Row b is the position bitmap of mask bit b: bit k % 64 of its word k / 64 is set when entry
// k holds bit b; only bits [0, rbits) can be set (rbits = |R| for a compressed frame).
// first / cnt / H: per bit, the first position holding it, how many entries hold it, and the
// sum of their hash terms (valid for bits below rbits).
struct FrameView {
    const uint32_t *ids;
    const uint64_t *hs;
    const uint64_t *masks;
    uint32_t *first;
    uint32_t *cnt;
    uint64_t *H;
    uint32_t *orig;
    uint64_t *hR;  // (narrow frames) the R-side hash term of each bit: hvl[orig[b]]
    uint64_t *rows;
    int nw;
};

__device__ __forceinline__ uint32_t frame_words_fixed(int n, int wf, int rbits) {
    const uint32_t bits = 64u * (uint32_t)wf, nw = ((uint32_t)n + 63u) >> 6;
    uint32_t o = align2((uint32_t)n);
    o += 2u * (uint32_t)n;                 // hs
    o += 2u * (uint32_t)n * (uint32_t)wf;  // masks
    o += 2u * bits;                        // first, cnt
    o += 2u * bits;                        // H
    o += 64u;                              // orig
    o += 128u;                             // hR
    o += 2u * (uint32_t)rbits * nw;        // rows
    return o;
}

__device__ __forceinline__ FrameView frame_view(uint32_t *base, int n, int wf, int rbits) {
    const uint32_t bits = 64u * (uint32_t)wf;
    FrameView v;
    v.nw = (n + 63) >> 6;
    v.ids = base;
    uint32_t o = align2((uint32_t)n);
    v.hs = reinterpret_cast<const uint64_t *>(base + o);
    o += 2u * (uint32_t)n;
    v.masks = reinterpret_cast<const uint64_t *>(base + o);
    o += 2u * (uint32_t)n * (uint32_t)wf;
    v.first = base + o;
    o += bits;
    v.cnt = base + o;
    o += bits;
    v.H = reinterpret_cast<uint64_t *>(base + o);
    o += 2u * bits;
    v.orig = base + o;
    o += 64u;
    v.hR = reinterpret_cast<uint64_t *>(base + o);
    o += 128u;
    v.rows = reinterpret_cast<uint64_t *>(base + o);
    return v;
}

// 64 x 64 bit-matrix transpose across the wave: on entry lane i holds row i (bit j is element
// (i, j)), on return lane j holds column j (bit i is element (i, j)).  Recursive block swap:
// at block size s, the upper-right and lower-left s x s blocks trade places.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x) {
    const int ln = lane_id();
    const uint64_t keep[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                              0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int sft = 32 >> l;
        const uint64_t lo = keep[l];  // bits whose index has bit sft clear
        const uint64_t y = __shfl_xor(x, sft);
        x = (ln & sft) ? ((x & ~lo) | ((y & ~lo) >> sft)) : ((x & lo) | ((y & lo) << sft));
    }
    return x;
}

// Rows [64q, 64q + 64) at word w of a frame, from mask word q of entries 64w .. 64w + 63
// (x: this lane's entry's word, 0 past the end).  One wave.
__device__ __forceinline__ void store_rows(const FrameView &v, int q, int w, uint64_t x) {
    v.rows[(size_t)(64 * q + lane_id()) * v.nw + w] = wave_transpose64(x);
}

struct Ctx {
    const int32_t *gid;    // universe global ids
    const uint64_t *M;     // universe masks (records only)
    const uint64_t *hvl;   // R-side hash term per position of N(x_root)
    const uint32_t *degl;  // degree per position of N(x_root)
    const int32_t *row;    // N(x_root)
    const int32_t *c_off;
    uint32_t *s1;                     // the workgroup's top-level list frame
    uint32_t *stk;                    // this wave's stack
    uint32_t *stu;                    // a maximal node's Q' and P' positions in list order
    uint32_t *stu_l;                  // the same in this wave's LDS (lists of at most kStuLds entries)
    lds_u32 *tl_first, *tl_cnt;       // this wave's LDS tables for narrow children
    lds_u64 *tl_H;
    lds_u64 *qk;                      // this wave's LDS list of kept Q' masks (kQKeep)
    lds_u32 *hist;                    // this wave's LDS histogram
    int64_t scap;
    int32_t x_root, s0, c_is_v, Wroot;
    int32_t cbase, obase;  // first packed id of the current graph's candidate / other side
    // records
    int32_t *rec;
    unsigned long long rec_cap, rec_offs_cap;
    unsigned long long *rec_offs;
    unsigned long long *acc;
    unsigned int *flags;
};

struct WaveAcc {  // per-lane partial tallies, summed over the wave at the end
    uint64_t count, hash, out_ints, nodes, nonmax, bytes;
    uint64_t dbytes;  // design-byte tally (TB instances): global bytes this search's loads and stores request
    uint32_t max_depth;
    uint64_t ph[PH_COUNT];  // cycles per phase (wave-uniform; diagnostics only)
};

// Hash terms use the graph's own ids (packed id minus the graph's base).
__device__ __forceinline__ uint64_t hl(const Ctx &c, int32_t v) {
    return c.c_is_v ? hash_v(v - c.cbase) : hash_u(v - c.cbase);
}
__device__ __forceinline__ uint64_t hr(const Ctx &c, int32_t w) {
    return c.c_is_v ? hash_u(w - c.obase) : hash_v(w - c.obase);
}

__device__ __forceinline__ uint32_t *frame_base(const Ctx &c, uint32_t off) { return off == kShared ? c.s1 : c.stk + off; }

__device__ __forceinline__ uint32_t root_pos(const FrameState &F, const FrameView &v, uint32_t b) {
    return F.narrow ? v.orig[b] : b;
}

// The R-side hash term of frame bit b: narrow frames keep it per bit (hR), other frames'
// bits are positions of N(x) already.
__device__ __forceinline__ uint64_t root_hash(const Ctx &c, const FrameState &F, const FrameView &v, uint32_t b) {
    return F.narrow ? v.hR[b] : c.hvl[b];
}
__device__ __forceinline__ uint64_t deg_of(const Ctx &c, uint32_t li) {
    const int32_t g = c.gid[li];
    return (uint64_t)(c.c_off[g + 1] - c.c_off[g]);
}

// Stable counting sort of n staged (parent position, key) pairs by key (keys in [1, nbins));
// sorted slot s receives parent position p through put(s, p).  One wave.
template <typename Put>
__device__ __forceinline__ void wave_sort_by_key(const uint32_t *src, const uint32_t *key_of, int n, int nbins, lds_u32 *hist,
                                 Put put) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    for (int b = ln; b < nbins; b += 64) hist[b] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        if (j < n) lds_add32(&hist[key_of[j]], 1u);
    }
    __builtin_amdgcn_wave_barrier();
    int carry = 0;
    for (int base = 0; base < nbins; base += 64) {
        const int b = base + ln;
        const int h = b < nbins ? (int)hist[b] : 0;
        const int incl = wave_incl_scan(h);
        if (b < nbins) hist[b] = (uint32_t)(carry + incl - h);
        carry += last_lane(incl);
    }
    __builtin_amdgcn_wave_barrier();
    const int nbits = nbins <= 1 ? 1 : 32 - __clz(nbins - 1);
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        const bool act = j < n;
        const uint32_t key = act ? key_of[j] : 0u;
        const uint32_t p = act ? src[j] : 0u;
        uint64_t same = __ballot(act);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (key >> bit) & 1u;
            const uint64_t bb = __ballot(act && on);
            same &= on ? bb : ~bb;
        }
        uint32_t start = 0;
        if (act) start = hist[key];
        __builtin_amdgcn_wave_barrier();
        if (act) {
            put(start + (uint32_t)__popcll(same & below), p);
            if ((same >> ln) == 1ull) hist[key] = start + (uint32_t)__popcll(same);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-bit tables and rows of a wide frame whose entries are in place; its masks lie within
// the words of R (m): rows of the other words are never read and are not written.  One wave.
template <int WF>
__device__ __forceinline__ void build_tables_wide(const FrameView &v, int n, int nq, const uint64_t (&m)[WF]) {
    constexpr int bits = 64 * WF;
    const int ln = lane_id();
    for (int b = ln; b < bits; b += 64) {
        v.first[b] = kNone;
        v.cnt[b] = 0u;
        v.H[b] = 0ull;
    }
    wait_mem();
    for (int base = 0; base < n; base += 64) {
        const int k = base + ln;
        const bool act = k < n;
        const uint64_t h = act && k >= nq ? v.hs[k] : 0ull;  // Q entries carry no hash term
#pragma unroll
        for (int w = 0; w < WF; ++w) {
            if (!m[w]) continue;  // uniform
            const uint64_t x = act ? v.masks[(size_t)k * WF + w] : 0ull;
            uint64_t y = x;
            while (y) {
                const int b = 64 * w + __ffsll((unsigned long long)y) - 1;
                y &= y - 1ull;
                atomicMin(&v.first[b], (uint32_t)k);
                atomicAdd(&v.cnt[b], 1u);
                atomicAdd(reinterpret_cast<unsigned long long *>(&v.H[b]), (unsigned long long)h);
            }
            store_rows(v, w, base >> 6, x);
        }
    }
    see_atomics();
}

// Narrow frames (one mask word per entry) accumulate first / cnt / H in the wave's LDS
// scratch while their entries are written (narrow_table_add); narrow_table_finish writes the
// tables out and builds the rows.  One wave.
__device__ __forceinline__ void narrow_table_clear(const Ctx &c) {
    const int ln = lane_id();
    c.tl_first[ln] = kNone;
    c.tl_cnt[ln] = 0u;
    c.tl_H[ln] = 0ull;
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ void narrow_table_add(const Ctx &c, uint32_t slot, uint64_t m, uint64_t h) {
    while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1ull;
        lds_min32(&c.tl_first[b], slot);
        lds_add32(&c.tl_cnt[b], 1u);
        lds_add64(&c.tl_H[b], h);
    }
}
__device__ __forceinline__ void narrow_table_finish(const Ctx &c, const FrameView &v, int n, int r) {
    const int ln = lane_id();
    __builtin_amdgcn_wave_barrier();
    if (ln < r) {
        v.first[ln] = c.tl_first[ln];
        v.cnt[ln] = c.tl_cnt[ln];
        v.H[ln] = c.tl_H[ln];
    }
    for (int base = 0; base < n; base += 64) {
        const int k = base + ln;
        const uint64_t t = wave_transpose64(k < n ? v.masks[k] : 0ull);
        if (ln < r) v.rows[(size_t)ln * v.nw + (base >> 6)] = t;
    }
    wait_mem();
}

// Write the record of the maximal biclique (L', R') of a node.  R' is given as positions of
// N(x_root) (Rr, Wroot words).  L' = {x_root} u {universe v : M[v] contains R'}: every vertex
// adjacent to all of R'.  Sides are sorted later by the canonicaliser.
__device__ __forceinline__ void write_record(const Ctx &c, const uint64_t *Rr, int nL, int r) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    const unsigned long long len = 2ull + (unsigned long long)nL + (unsigned long long)r;
    unsigned long long off = 0, idx = 0;
    if (ln == 0) {
        off = atomicAdd(&c.acc[ACC_REC_INTS], len);
        idx = atomicAdd(&c.acc[ACC_RECORDS], 1ull);
    }
    off = __shfl(off, 0);
    idx = __shfl(idx, 0);
    if (off + len > c.rec_cap || idx >= c.rec_offs_cap) {
        if (ln == 0) atomicOr(c.flags, (unsigned int)FLAG_RECORD_OVERFLOW);
        return;
    }
    int32_t *o = c.rec + off;
    int32_t *pl = o + 2 + (c.c_is_v ? r : 0);   // where L' goes
    int32_t *pr = o + 2 + (c.c_is_v ? 0 : nL);  // where R' goes
    if (ln == 0) {
        o[0] = c.c_is_v ? r : nL;
        o[1] = c.c_is_v ? nL : r;
        c.rec_offs[idx] = off;
        pl[0] = c.x_root - c.cbase;
    }
    int k = 1;
    for (int base = 0; base < c.s0; base += 64) {
        const int li = base + ln;
        bool in = li < c.s0;
        if (in) {
            const uint64_t *m = c.M + (size_t)li * c.Wroot;
            for (int w = 0; w < c.Wroot; ++w) in = in && ((m[w] & Rr[w]) == Rr[w]);
        }
        const uint64_t b = __ballot(in);
        const int at = k + __popcll(b & below);
        if (in && at < nL) pl[at] = c.gid[li] - c.cbase;  // never past the reserved record
        k += __popcll(b);
    }
    int q = 0;
    for (int w = 0; w < c.Wroot; ++w) {
        const bool in = (Rr[w] >> ln) & 1ull;
        const uint64_t b = __ballot(in);
        const int at = q + __popcll(b & below);
        if (in && at < r) pr[at] = c.row[w * 64 + ln] - c.obase;
        q += __popcll(b);
    }
}

// Candidates [base, base+64) of frame F: lanes with |R'| = 1 are settled here; the rest are
// returned as a lane mask.
template <int WF, bool DIAG, bool ENUM, bool TB = false>
__device__ __forceinline__ uint64_t light_chunk(const Ctx &c, const FrameState &F, const FrameView &v, int base, WaveAcc &acc,
                                bool settle = true) {
    const int ln = lane_id();
    const int i = base + ln;
    const bool act = i < F.n;
    uint64_t m[WF];
    int r = 0;
#pragma unroll
    for (int w = 0; w < WF; ++w) {
        m[w] = act ? v.masks[(size_t)i * WF + w] : 0ull;
        r += __popcll(m[w]);
    }
    if (ENUM) return __ballot(act);
    const bool light = settle && act && r == 1;
    if (light) {
        int b = 0;
#pragma unroll
        for (int w = 0; w < WF; ++w)
            if (m[w]) b = 64 * w + __ffsll((unsigned long long)m[w]) - 1;
        const bool maximal = v.first[b] == (uint32_t)i;  // no earlier entry holds bit b
        const uint32_t rp = root_pos(F, v, (uint32_t)b);
        if (maximal) {
            // L' = L u {every entry with bit b}: all of them sit at positions >= i
            const uint64_t sL = F.sL + v.H[b];
            acc.count += 1;
            acc.hash += pair_hash(c.c_is_v, sL, root_hash(c, F, v, (uint32_t)b));
            acc.out_ints += 2ull + (uint64_t)F.nL + (uint64_t)v.cnt[b] + 1ull;
        }
        if (DIAG) {
            acc.nodes += 1;
            if (!maximal) acc.nonmax += 1;
            if ((uint32_t)F.level > acc.max_depth) acc.max_depth = (uint32_t)F.level;
            const uint64_t dx = deg_of(c, v.ids[i]);
            const uint64_t rs = 2ull + (uint64_t)c.degl[rp];
            const uint64_t fw = F.fw - (2ull + dx);
            acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + 1ull);
        }
        // first[b]; for a maximal node H[b], cnt[b], the R-side hash term (and orig[b])
        if (TB) acc.dbytes += 4ull + (maximal ? 20ull : 0ull);
    }
    if (TB && act && settle) acc.dbytes += 8ull * WF;  // the entry's mask
    return __ballot(act && r >= 2);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// The compression of entry k's mask to the |R'| bits of R' (bit t = the t-th bit of R').
template <int WF>
__device__ __forceinline__ uint64_t compress_mask(const FrameView &v, const uint64_t (&m)[WF], int k) {
    uint64_t out = 0;
    int t = 0;
#pragma unroll
    for (int w = 0; w < WF; ++w) {
        if (!m[w]) continue;  // uniform
        uint64_t mm = m[w];
        const uint64_t xx = v.masks[(size_t)k * WF + w];
        while (mm) {  // the same trip count on every lane: m is uniform
            const int p = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1ull;
            out |= ((xx >> p) & 1ull) << t;
            ++t;
        }
    }
    return out;
}

// Q' of a compressed child, reduced to its inclusion-maximal masks.  A Q entry only ever
// serves as a witness that some later R'' (a subset of R') is not maximal, and an entry
// whose mask over R' lies inside another's witnesses nothing the other does not, so only
// one entry per maximal mask needs to stay.  The Q' entries are stu[0, qn); the kept
// compressed masks go to c.qk.  Returns their number, or -1 when more than kQKeep are
// incomparable (then nothing is dropped).  Cost per chunk of 64 entries: one pass over the
// kept masks, and one over the chunk's candidates.
template <int WF, bool SMALL_R>
__device__ __forceinline__ int prune_q(const Ctx &c, const FrameView &v, const uint64_t (&m)[WF], int qn, int r,
                                       const uint32_t *stu) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    if (SMALL_R && r <= 6) {
        // every compressed mask is a value below 64: the set of values present is one word,
        // its superset closure takes six shift-and-mask rounds, and the maximal values are
        // the present ones no strictly larger present value contains
        uint64_t pres = 0;
        for (int base = 0; base < qn; base += 64) {
            const int j = base + ln;
            if (j < qn) pres |= 1ull << compress_mask<WF>(v, m, (int)stu[j]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pres |= __shfl_xor(pres, o);
        pres = uni(pres);
        // value T: some present S contains T (round t adds the sets that differ in bit t)
        uint64_t sup = pres;
        sup |= (sup >> 1) & 0x5555555555555555ull;
        sup |= (sup >> 2) & 0x3333333333333333ull;
        sup |= (sup >> 4) & 0x0F0F0F0F0F0F0F0Full;
        sup |= (sup >> 8) & 0x00FF00FF00FF00FFull;
        sup |= (sup >> 16) & 0x0000FFFF0000FFFFull;
        sup |= (sup >> 32) & 0x00000000FFFFFFFFull;
        // value T: some present S strictly contains T (T plus one more bit, then any superset)
        const uint64_t above = ((sup >> 1) & 0x5555555555555555ull) | ((sup >> 2) & 0x3333333333333333ull) |
                               ((sup >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((sup >> 8) & 0x00FF00FF00FF00FFull) |
                               ((sup >> 16) & 0x0000FFFF0000FFFFull) | ((sup >> 32) & 0x00000000FFFFFFFFull);
        const uint64_t mx = pres & ~above;
        if ((mx >> ln) & 1ull) c.qk[__popcll(mx & below)] = (uint64_t)ln;
        __builtin_amdgcn_wave_barrier();
        return __popcll(mx);
    }
    int nk = 0;
    for (int base = 0; base < qn; base += 64) {
        const int j = base + ln;
        const bool act = j < qn;
        const uint64_t x = act ? compress_mask<WF>(v, m, (int)stu[j]) : 0ull;
        bool cand = act;
        for (int t = 0; t < nk; ++t) {
            const uint64_t y = c.qk[t];  // same address on every lane
            if ((x & ~y) == 0ull) cand = false;
        }
        // among this chunk: drop x when another candidate holds more, or the same in a lower lane
        bool keep = cand;
        for (uint64_t q = __ballot(cand); q; q &= q - 1ull) {
            const int l = __ffsll((unsigned long long)q) - 1;
            const uint64_t y = readlane64(x, l);
            if (l != ln && (x & ~y) == 0ull && (x != y || l < ln)) keep = false;
        }
        const uint64_t sb = __ballot(keep);
        if (!sb) continue;
        // kept masks inside a new survivor go (compacted in place, 64 at a time: an entry
        // only moves down, past entries already read); the survivors join
        int ns = 0;
        for (int blk = 0; blk < nk; blk += 64) {
            const int t = blk + ln;
            const uint64_t y = t < nk ? c.qk[t] : 0ull;
            bool stay = t < nk;
            for (uint64_t q = sb; q; q &= q - 1ull) {
                const uint64_t xs = readlane64(x, __ffsll((unsigned long long)q) - 1);
                if ((y & ~xs) == 0ull) stay = false;
            }
            const uint64_t stb = __ballot(stay);
            __builtin_amdgcn_wave_barrier();
            if (stay) c.qk[ns + __popcll(stb & below)] = y;
            __builtin_amdgcn_wave_barrier();
            ns += __popcll(stb);
        }
        const int nn = ns + __popcll(sb);
        if (nn > kQKeep) return -1;
        if (keep) c.qk[ns + __popcll(sb & below)] = x;
        __builtin_amdgcn_wave_barrier();
        nk = nn;
    }
    return nk;
}

// Write the child frame of the maximal node at position i at the top of the wave's stack.
// Its entries are the positions stu[0, nu) of the node's list, in list order: the first qn
// (before i) form Q' and keep their order, the other pn (after i, 0 < |mask n R'| < |R'|)
// form P', stably sorted by that count.  Each entry is written straight to its slot: c.hist
// holds, per count, the number of P' entries (filled by the caller).  Masks are restricted
// to R' and, when NARROW, compressed to |R'| bits; the tables and rows follow.  Sets the
// layout fields of C; false when the stack is full.
template <int WF, int W, bool NARROW, bool DIAG, bool TB = false>
__device__ __forceinline__ bool build_child(const Ctx &c, const FrameState &F, const FrameView &v, const uint64_t (&m)[WF], int nu,
                            int r, int qn, int pn, FrameState &C, int preq, WaveAcc &acc, bool tally,
                            const uint32_t *stu) {
    const bool stu_g = stu == c.stu;  // (design bytes: the listed entries are global only then)
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    int nzw = 0;  // words of R' (the mask words an entry's gathers read)
#pragma unroll
    for (int w = 0; w < WF; ++w) nzw += m[w] ? 1 : 0;
    // Q': with diagnostics off, a compressed child keeps only its inclusion-maximal masks
    // (the tallies of diagnostics mode count the full Q' of the method).  preq >= 0: the
    // caller already left them in c.qk, and stu[0, pn) packs each P' entry's position (low
    // 26 bits) with its compressed mask
    int nq2 = qn;
    bool pruned = false;
    if (preq >= 0) {
        nq2 = preq;
        pruned = true;
    } else if constexpr (NARROW && !DIAG) {
        if (qn > 1) {
            const int nk = prune_q<WF, kSmallRPrune<W>>(c, v, m, qn, r, stu);
            if (TB && tally && ln == 0) acc.dbytes += (uint64_t)qn * ((stu_g ? 4ull : 0ull) + 8ull * (uint64_t)nzw);  // stu, masks
            if (nk >= 0) {
                nq2 = nk;
                pruned = true;
            }
        }
    }
    const int n2 = nq2 + pn;
    constexpr int wf2 = NARROW ? 1 : W;
    const uint32_t off2 = F.top;
    const int rbits2 = NARROW ? r : 64 * W;
    const uint32_t top2 = align2(off2 + frame_words_fixed(n2, wf2, rbits2));
    if ((int64_t)top2 > c.scap) {
        if (ln == 0) atomicOr(c.flags, (unsigned int)FLAG_STACK_OVERFLOW);
        return false;
    }
    uint32_t *cb = c.stk + off2;
    FrameView v2 = frame_view(cb, n2, wf2, rbits2);
    uint32_t *ids2 = cb;
    uint64_t *hs2 = const_cast<uint64_t *>(v2.hs);
    uint64_t *masks2 = const_cast<uint64_t *>(v2.masks);
    if (NARROW) {
        // orig2[t] = N(x_root) position of the t-th bit of R'
        int t0 = 0;
#pragma unroll
        for (int w = 0; w < WF; ++w) {
            const bool on = (m[w] >> ln) & 1ull;
            const uint64_t bb = __ballot(on);
            if (on) {
                const int at = t0 + __popcll(bb & below);
                v2.orig[at] = root_pos(F, v, (uint32_t)(64 * w + ln));
                v2.hR[at] = root_hash(c, F, v, (uint32_t)(64 * w + ln));
            }
            t0 += __popcll(bb);
        }
        narrow_table_clear(c);
        if (pruned) {
            for (int t = ln; t < nq2; t += 64) {
                const uint64_t x = c.qk[t];
                masks2[t] = x;
                narrow_table_add(c, (uint32_t)t, x, 0ull);
            }
        }
    }
    // first slot of each count among the P' entries
    int carry = nq2;
    for (int base = 0; base < r; base += 64) {
        const int b = base + ln;
        const int h = b < r ? (int)c.hist[b] : 0;
        const int incl = wave_incl_scan(h);
        if (b < r) c.hist[b] = (uint32_t)(carry + incl - h);
        carry += last_lane(incl);
    }
    __builtin_amdgcn_wave_barrier();
    const int nbits = r <= 1 ? 1 : 32 - __clz(r - 1);
    for (int base = pruned ? qn : 0; base < nu; base += 64) {
        const int j = base + ln;
        const bool act = j < nu;
        const uint32_t e = act ? stu[j] : 0u;
        const int k = preq >= 0 ? (int)(e & 0x3FFFFFFu) : (int)e;
        uint64_t x[WF];
        int cnt = 0;
        if (preq >= 0) {
#pragma unroll
            for (int w = 0; w < WF; ++w) x[w] = 0ull;
            cnt = __popc(e >> 26);
        } else {
#pragma unroll
            for (int w = 0; w < WF; ++w) {
                x[w] = act && m[w] ? v.masks[(size_t)k * WF + w] & m[w] : 0ull;  // words of R' only
                cnt += __popcll(x[w]);
            }
        }
        const bool inp = act && j >= qn;
        uint32_t slot = (uint32_t)j;  // Q' entries keep their list order
        if (__ballot(inp)) {
            // stable placement among equal counts: lanes with the same count, in lane order
            uint64_t same = __ballot(inp);
            for (int bit = 0; bit < nbits; ++bit) {
                const bool on = (cnt >> bit) & 1;
                const uint64_t bb = __ballot(inp && on);
                same &= on ? bb : ~bb;
            }
            uint32_t start = 0;
            if (inp) start = c.hist[cnt];
            __builtin_amdgcn_wave_barrier();
            if (inp) {
                slot = start + (uint32_t)__popcll(same & below);
                if ((same >> ln) == 1ull) c.hist[cnt] = start + (uint32_t)__popcll(same);
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (act) {
            if (DIAG) ids2[slot] = v.ids[k];
            // Q entries' hash terms are never read (a node whose bit some Q entry holds is
            // not maximal), so they are not copied
            const uint64_t h = inp ? v.hs[k] : 0ull;
            if (inp) hs2[slot] = h;
            if (NARROW) {
                uint64_t out = 0;
                if (preq >= 0) {
                    out = (uint64_t)(e >> 26);
                } else {
                    int t = 0;
#pragma unroll
                    for (int w = 0; w < WF; ++w) {
                        uint64_t mm = m[w];
                        while (mm) {  // the same trip count on every lane: m is uniform
                            const int p = __ffsll((unsigned long long)mm) - 1;
                            mm &= mm - 1ull;
                            out |= ((x[w] >> p) & 1ull) << t;
                            ++t;
                        }
                    }
                }
                masks2[slot] = out;
                narrow_table_add(c, slot, out, h);
            } else {
#pragma unroll
                for (int w = 0; w < WF; ++w) masks2[(size_t)slot * W + w] = x[w];
            }
        }
    }
    wait_mem();
    if (TB && tally && ln == 0) {
        const uint64_t nloop = (uint64_t)(nu - (pruned ? qn : 0));
        uint64_t b = nloop * ((stu_g ? 4ull : 0ull) + 8ull * (uint64_t)wf2) + 16ull * (uint64_t)pn;  // stu; child masks; hs in and out
        if (preq < 0) b += nloop * 8ull * (uint64_t)nzw;                           // the entries' masks over R'
        if (NARROW) {
            b += 8ull * (uint64_t)(pruned ? nq2 : 0) + 4ull * (uint64_t)r * (F.narrow ? 2ull : 1ull) +  // kept Q'; orig
                 16ull * (uint64_t)r;                                                                    // hR
            b += 16ull * (uint64_t)r + 8ull * (uint64_t)n2 + 8ull * (uint64_t)r * (uint64_t)v2.nw;   // tables; rows
        } else {
            // tables cleared, each entry's hash term and mask words read, its bits' table atomics
            // (tallied per lane below), rows of the words of R'
            b += 16ull * 64ull * W + (uint64_t)n2 * (8ull + 8ull * (uint64_t)nzw) +
                 8ull * 64ull * (uint64_t)nzw * (uint64_t)v2.nw;
        }
        acc.dbytes += b;
    }
    if constexpr (NARROW) {
        narrow_table_finish(c, v2, n2, r);
    } else {
        static_assert(WF == W, "wide children come from wide lists");
        build_tables_wide<W>(v2, n2, nq2, m);
        if (TB && tally)
            for (int k = ln; k < n2; k += 64) {
                uint64_t bits = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) bits += (uint64_t)__popcll(masks2[(size_t)k * W + w]);
                acc.dbytes += 16ull * bits;
            }
    }
    C.off = off2;
    C.top = top2;
    C.n = n2;
    C.nq = nq2;
    C.wf = wf2;
    C.narrow = NARROW ? 1 : 0;
    C.chunk = nq2 - 64;
    C.rbits = rbits2;
    C.heavy = 0ull;
    return true;
}

// OR (u) and AND (a), over the bits b of R' listed in c.hist[0, r), of word wd of row b; a
// is 0 when !in.  Rows are read four at a time.
__device__ __forceinline__ void fold_rows(const Ctx &c, const FrameView &v, int r, int wd, bool in, uint64_t &u,
                                          uint64_t &a) {
    u = 0ull;
    a = ~0ull;
    for (int t = 0; t < r; t += 4) {
        const uint32_t b0 = uni(c.hist[t]);
        const uint32_t b1 = uni(c.hist[t + 1 < r ? t + 1 : t]);
        const uint32_t b2 = uni(c.hist[t + 2 < r ? t + 2 : t]);
        const uint32_t b3 = uni(c.hist[t + 3 < r ? t + 3 : t]);
        if (in) {
            const uint64_t x0 = v.rows[(size_t)b0 * v.nw + wd], x1 = v.rows[(size_t)b1 * v.nw + wd];
            const uint64_t x2 = v.rows[(size_t)b2 * v.nw + wd], x3 = v.rows[(size_t)b3 * v.nw + wd];
            u |= (x0 | x1) | (x2 | x3);
            a &= (x0 & x1) & (x2 & x3);
        }
    }
    if (!in) a = 0ull;
}

// The candidate at position i of frame F, |R'| = r >= 1, handled by the whole wave.
// Returns true when a child frame was written (its state in C).  report = false rebuilds the
// child frame of a node another wave owns: nothing is counted or recorded.
template <int WF, int W, bool DIAG, bool ENUM, bool TB = false>
__device__ __forceinline__ bool heavy_node(const Ctx &c, const FrameState &F, const FrameView &v, int i, FrameState &C,
                           WaveAcc &acc, bool report) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    uint64_t m[WF];
    int r = 0;
#pragma unroll
    for (int w = 0; w < WF; ++w) {
        m[w] = uni(v.masks[(size_t)i * WF + w]);  // R' (uniform)
        r += __popcll(m[w]);
    }

    // the bits of R', ascending, in c.hist[0, r)
    {
        int t0 = 0;
#pragma unroll
        for (int w = 0; w < WF; ++w) {
            const bool on = (m[w] >> ln) & 1ull;
            const uint64_t bb = __ballot(on);
            if (on) c.hist[t0 + __popcll(bb & below)] = (uint32_t)(64 * w + ln);
            t0 += __popcll(bb);
        }
        __builtin_amdgcn_wave_barrier();
    }

    // maximality: an earlier entry holding every bit of R' ends the node -- a position below
    // i in the AND of R''s rows.  If some bit of R' first appears at i itself, nothing
    // earlier can hold R'.
    bool first_here = false;
#pragma unroll
    for (int w = 0; w < WF; ++w)
        if (((m[w] >> ln) & 1ull) && v.first[64 * w + ln] == (uint32_t)i) first_here = true;
    bool nonmax = false;
    uint64_t tp = DIAG ? clock64() : 0ull;
    if (TB && report && ln == 0) acc.dbytes += 8ull * WF + 4ull * (uint64_t)r;  // R'; first[] of its bits
    if (!__ballot(first_here)) {
        const int wl = i >> 6;  // the word holding position i
        for (int base = 0; base <= wl; base += 64) {
            const int wd = base + ln;
            uint64_t u, a;
            fold_rows(c, v, r, wd, wd <= wl, u, a);
            if (TB && report && ln == 0) acc.dbytes += 8ull * (uint64_t)r * (uint64_t)min(64, wl + 1 - base);
            if (wd == wl) a &= (1ull << (i & 63)) - 1ull;
            if (__ballot(a != 0ull)) {
                nonmax = true;
                break;
            }
        }
    }

    uint64_t dx = 0, rs = 0;
    if (DIAG) {
        const uint64_t now = clock64();
        acc.ph[PH_CHECK] += now - tp;
        tp = now;
        dx = deg_of(c, v.ids[i]);
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < WF; ++w)
            if ((m[w] >> ln) & 1ull) t += 2ull + (uint64_t)c.degl[root_pos(F, v, (uint32_t)(64 * w + ln))];
        rs = wave_sum_u64(t);
        if (ln == 0 && report) {
            acc.nodes += 1;
            if ((uint32_t)F.level > acc.max_depth) acc.max_depth = (uint32_t)F.level;
        }
    }
    if (nonmax) {
        if (DIAG && ln == 0 && report) {
            acc.nonmax += 1;
            const uint64_t fw = F.fw - (2ull + dx);
            acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r);
        }
        return false;
    }

    // maximal.  Per word of positions: the OR of R''s rows gives the entries sharing a bit
    // with R', the AND those holding all of it (after i only, the node being maximal; they
    // join L').  The rest -- Q' before i, P' after -- are listed in stu in list order, and
    // the P' counts |mask n R'| are tallied per value in c.hist for the child's stable sort.
    //
    // When |R'| <= 6 (and diagnostics are off) the rows give each entry's compressed mask
    // directly (its bit in each of R''s rows), so no entry is read: Q' is reduced to its
    // maximal masks through the presence word (as in prune_q) and only P' is listed, each
    // stu word packing the position (low 26 bits) with the compressed mask.
    int qn = 0, nu = 0;
    // the listed entries (at most F.n - 1): in the wave's LDS when they fit
    uint32_t *const stu = F.n <= kStuLds ? c.stu_l : c.stu;
    int ne_l = 0, qn_l = 0;
    uint64_t exps = 0, fwc = 0;
    // (the two-word class takes it on its own two-word lists only: register budget)
    const bool fastq = !DIAG && kSmallRPrune<W> && (W != 2 || WF == W) && r <= 6 && F.n < (1 << 26);
    int preq = -1;  // with fastq: the number of maximal Q' masks left in c.qk
    if (fastq) {
        int bl[6];  // the bits of R'
#pragma unroll
        for (int t = 0; t < 6; ++t) bl[t] = t < r ? (int)uni(c.hist[t]) : 0;
        __builtin_amdgcn_wave_barrier();
        for (int b = ln; b < r; b += 64) c.hist[b] = 0u;
        __builtin_amdgcn_wave_barrier();
        const int wi = i >> 6;
        const uint64_t bi = 1ull << (i & 63);
        uint64_t pres = 0;
        for (int base = 0; base < v.nw; base += 64) {
            const int wd = base + ln;
            const bool in = wd < v.nw;
            uint64_t x[6];
            uint64_t u = 0ull, a = in ? ~0ull : 0ull;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                x[t] = (t < r && in) ? v.rows[(size_t)bl[t] * v.nw + wd] : 0ull;
                if (t < r) {
                    u |= x[t];
                    a &= x[t];
                }
            }
            if (wd == wi) {
                u &= ~bi;
                a &= ~bi;
            }
            ne_l += __popcll(a);
            for (uint64_t f = a; f;) {
                const int b = __ffsll((unsigned long long)f) - 1;
                f &= f - 1ull;
                exps += v.hs[64 * wd + b];
            }
            const uint64_t qp = u & ~a;
            const uint64_t before = wd < wi ? ~0ull : (wd == wi ? bi - 1ull : 0ull);
            auto cmask = [&](int p) {
                uint32_t cm = 0;
#pragma unroll
                for (int t = 0; t < 6; ++t)
                    if (t < r) cm |= (uint32_t)((x[t] >> p) & 1ull) << t;
                return cm;
            };
            for (uint64_t q = qp & before; q; q &= q - 1ull) pres |= 1ull << cmask(__ffsll((unsigned long long)q) - 1);
            uint64_t pm = qp & ~before;
            const int pc = __popcll(pm);
            const int incl = wave_incl_scan(pc);
            int at = nu + incl - pc;
            while (pm) {
                const int b = __ffsll((unsigned long long)pm) - 1;
                pm &= pm - 1ull;
                const uint32_t cm = cmask(b);
                stu[at++] = (uint32_t)(64 * wd + b) | (cm << 26);
                lds_add32(&c.hist[__popc(cm)], 1u);
            }
            nu += last_lane(incl);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pres |= __shfl_xor(pres, o);
        pres = uni(pres);
        uint64_t sup = pres;
        sup |= (sup >> 1) & 0x5555555555555555ull;
        sup |= (sup >> 2) & 0x3333333333333333ull;
        sup |= (sup >> 4) & 0x0F0F0F0F0F0F0F0Full;
        sup |= (sup >> 8) & 0x00FF00FF00FF00FFull;
        sup |= (sup >> 16) & 0x0000FFFF0000FFFFull;
        sup |= (sup >> 32) & 0x00000000FFFFFFFFull;
        const uint64_t above = ((sup >> 1) & 0x5555555555555555ull) | ((sup >> 2) & 0x3333333333333333ull) |
                               ((sup >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((sup >> 8) & 0x00FF00FF00FF00FFull) |
                               ((sup >> 16) & 0x0000FFFF0000FFFFull) | ((sup >> 32) & 0x00000000FFFFFFFFull);
        const uint64_t mx = pres & ~above;
        if ((mx >> ln) & 1ull) c.qk[__popcll(mx & below)] = (uint64_t)ln;
        preq = __popcll(mx);
        qn = 0;
        wait_mem();  // stu is read by other lanes below
        __builtin_amdgcn_wave_barrier();
    } else {
        const int wi = i >> 6;
        const uint64_t bi = 1ull << (i & 63);
        for (int base = 0; base < v.nw; base += 64) {
            const int wd = base + ln;
            uint64_t u, a;
            fold_rows(c, v, r, wd, wd < v.nw, u, a);
            if (wd == wi) {
                u &= ~bi;
                a &= ~bi;
            }
            ne_l += __popcll(a);
            for (uint64_t f = a; f;) {
                const int b = __ffsll((unsigned long long)f) - 1;
                f &= f - 1ull;
                exps += v.hs[64 * wd + b];
            }
            uint64_t qp = u & ~a;
            qn_l += __popcll(qp & (wd < wi ? ~0ull : (wd == wi ? bi - 1ull : 0ull)));
            const int pc = __popcll(qp);
            const int incl = wave_incl_scan(pc);
            int at = nu + incl - pc;
            while (qp) {
                const int b = __ffsll((unsigned long long)qp) - 1;
                qp &= qp - 1ull;
                stu[at++] = (uint32_t)(64 * wd + b);
            }
            nu += last_lane(incl);
        }
        qn = wave_sum_i32(qn_l);
        wait_mem();  // stu is read by other lanes below
        for (int b = ln; b < r; b += 64) c.hist[b] = 0u;
        __builtin_amdgcn_wave_barrier();
        for (int base = DIAG ? 0 : qn; base < nu; base += 64) {
            const int j = base + ln;
            if (j < nu) {
                const int k = (int)stu[j];
                if (j >= qn) {
                    int cnt = 0;
#pragma unroll
                    for (int w = 0; w < WF; ++w)
                        if (m[w]) cnt += __popcll(v.masks[(size_t)k * WF + w] & m[w]);  // words of R' only
                    lds_add32(&c.hist[cnt], 1u);
                }
                if (DIAG) fwc += 2ull + deg_of(c, v.ids[k]);
            }
        }
    }
    const int ne = wave_sum_i32(ne_l);
    const int pn = nu - qn;
    if (TB && report && ln == 0) {
        // R''s rows over every word of positions, the joiners' hash terms, the listed entries
        // (written, and for the counts of P' read back with their mask words over R'),
        // the R-side hash terms (and orig) of R'
        int nzw = 0;
#pragma unroll
        for (int w = 0; w < WF; ++w) nzw += m[w] ? 1 : 0;
        const uint64_t sb = stu == c.stu ? 4ull : 0ull;  // (listed entries in global scratch)
        uint64_t b = 8ull * (uint64_t)r * (uint64_t)v.nw + 8ull * (uint64_t)ne + sb * (uint64_t)nu;
        if (!fastq) b += (uint64_t)pn * (sb + 8ull * (uint64_t)nzw);
        b += (uint64_t)r * 8ull;
        acc.dbytes += b;
    }

    // report (L', R')
    const uint64_t sL = F.sL + v.hs[i] + wave_sum_u64(exps);
    uint64_t sr = 0;
#pragma unroll
    for (int w = 0; w < WF; ++w)
        if ((m[w] >> ln) & 1ull) sr += root_hash(c, F, v, (uint32_t)(64 * w + ln));
    sr = wave_sum_u64(sr);
    const int nL = F.nL + 1 + ne;
    if (ln == 0 && report) {
        acc.count += 1;
        acc.hash += pair_hash(c.c_is_v, sL, sr);
        acc.out_ints += 2ull + (uint64_t)nL + (uint64_t)r;
    }
    if (ENUM && report) {
        uint64_t Rr[16];
        for (int w = 0; w < 16; ++w) Rr[w] = 0ull;
#pragma unroll
        for (int w = 0; w < WF; ++w) {
            uint64_t mm = m[w];
            while (mm) {
                const int b = 64 * w + __ffsll((unsigned long long)mm) - 1;
                mm &= mm - 1ull;
                const uint32_t rp = root_pos(F, v, (uint32_t)b);
                Rr[rp >> 6] |= 1ull << (rp & 63);
            }
        }
        write_record(c, Rr, nL, r);
    }
    if (DIAG && ln == 0 && report) {
        const uint64_t fw = F.fw - (2ull + dx);
        acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r + (uint64_t)pn +
                             (uint64_t)qn);
    }
    if (DIAG) {
        const uint64_t now = clock64();
        acc.ph[PH_EXPAND] += now - tp;
        tp = now;
    }
    if (pn == 0) return false;

    // child frame: Q' then P' stably sorted by count; masks restricted to R' and, when
    // |R'| <= 64, compressed to |R'| bits
    bool ok;
    if constexpr (WF == 1) {
        ok = build_child<1, W, true, DIAG, TB>(c, F, v, m, nu, r, qn, pn, C, preq, acc, report, stu);
    } else {
        ok = r <= 64 ? build_child<WF, W, true, DIAG, TB>(c, F, v, m, nu, r, qn, pn, C, preq, acc, report, stu)
                     : build_child<WF, W, false, DIAG, TB>(c, F, v, m, nu, r, qn, pn, C, preq, acc, report, stu);
    }
    if (!ok) return false;
    C.level = F.level + 1;
    C.nL = nL;
    C.sL = sL;
    C.fw = DIAG ? wave_sum_u64(fwc) : 0ull;
    if (DIAG) acc.ph[PH_CHILD] += clock64() - tp;
    return true;
}

// A wave's third-level sharing state (kept in LDS: it is needed only between chunks).
struct WaveShare {
    int cdepth;   // depth whose chunks are claimed through slot cidx (-1: none)
    int cidx;     // that slot (index into the launch's third-level slots)
    unsigned int cepoch;
    int cfirst;   // list position of chunk 0, and the number of chunks
    int climit;
    int pend;     // a chunk claimed before the list was rebuilt (-1: none)
    int hitem;    // top-level position of the node whose list is rebuilt
    int item1;    // top-level position of the node whose list is at depth 1
    int cown;     // 1: this wave published slot cidx
    int pad[3];
};
typedef __attribute__((address_space(3))) WaveShare lds_ws;

struct WGShared {
    unsigned long long task;
    int s0;
    uint32_t claim;     // next top-level item (owner, before the list moves to the steal slot)
    uint32_t moved;     // 0: items claimed in LDS; 2: moving to the steal slot; 1: moved
    int published;      // the steal slot holds this task's list
    int nonmax;
    int pcount;
    unsigned long long exps;
    unsigned long long fw1;
    unsigned long long hvsum;
    unsigned long long rs1;
    int nexp;
    int graph;  // graph whose tallies the workgroup is holding
    int mode;   // 0 done, 1 own task, 2 stolen top-level list, 3 stolen third-level list
    int victim; // workgroup whose child list a stolen task shares
    unsigned int epoch;
    int gclaim; // chunks are claimed through the global steal slot
    int sg, sk; // graph and rank of a stolen task
    int slot;   // arena slot held by this workgroup
    int scan[16];
    unsigned long long red[16];  // per-graph tally reduction
    unsigned long long cov[16];  // bits of N(x) held by a multi-bit top-level Q mask
    int held;            // the workgroup counts in a.busy
    int roots_done;      // this launch's top-level candidates are all handed out
    uint32_t busyw;      // waves holding work in the current task
    uint32_t idlew;      // waves looking for a third-level list to help with
    uint32_t npub;       // third-level lists published by the workgroup's waves
    int others_done;     // (wave 0) the other launches' top-level candidates are all handed out
    int vpub;            // mode 3: the third-level slot taken, and its epoch
    unsigned int vepoch;
    int tg, tk;          // graph and top-level rank of the current task
    FrameState topf;     // the top-level frame of the current task
    WaveShare ws[16];
};

// Add the workgroup's tallies to a graph's accumulators and clear them.  All threads call.
template <bool DIAG, bool TB = false>
__device__ __forceinline__ void flush_acc(WaveAcc &acc, unsigned long long *gacc, WGShared *sh) {
    const int ln = lane_id();
    uint64_t v[8];
    v[0] = wave_sum_u64(acc.count);
    v[1] = wave_sum_u64(acc.hash);
    v[2] = wave_sum_u64(acc.out_ints);
    v[3] = DIAG ? wave_sum_u64(acc.nodes) : 0ull;
    v[4] = DIAG ? wave_sum_u64(acc.nonmax) : 0ull;
    v[5] = DIAG ? wave_sum_u64(acc.bytes) : 0ull;
    v[6] = DIAG ? (uint64_t)wave_max_u32(acc.max_depth) : 0ull;
    v[7] = TB ? wave_sum_u64(acc.dbytes) : 0ull;
    if (ln == 0) {
        for (int q = 0; q < 6; ++q)
            if (v[q]) lds_add(&sh->red[q], v[q]);
        if (v[6]) lds_max(&sh->red[6], v[6]);
        if (v[7]) lds_add(&sh->red[7], v[7]);
        if (DIAG)
            for (int q = 0; q < PH_COUNT; ++q)
                if (acc.ph[q]) lds_add(&sh->red[8 + q], acc.ph[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int slot[6] = {ACC_COUNT, ACC_HASH, ACC_OUT_INTS, ACC_NODES, ACC_NONMAX, ACC_BYTES};
        for (int q = 0; q < 6; ++q) {
            if (sh->red[q]) atomicAdd(&gacc[slot[q]], sh->red[q]);
            sh->red[q] = 0ull;
        }
        if (sh->red[6]) atomicMax(&gacc[ACC_MAX_DEPTH], sh->red[6]);
        sh->red[6] = 0ull;
        if (sh->red[7]) atomicAdd(&gacc[ACC_DBYTES], sh->red[7]);
        sh->red[7] = 0ull;
        for (int q = 0; q < PH_COUNT; ++q) {
            if (sh->red[8 + q]) atomicAdd(&gacc[ACC_PHASE + q], sh->red[8 + q]);
            sh->red[8 + q] = 0ull;
        }
    }
    __syncthreads();
    acc = WaveAcc{};
}

// Claim the next step items of a published list: returns the first one's index, or -1 once
// the list is used up or its owner has moved on (epoch changed).
__device__ __forceinline__ int claim_chunk(unsigned long long *word, unsigned int epoch, int limit, unsigned int step) {
    unsigned long long old = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if ((unsigned int)(old >> 32) != epoch) return -1;
        const unsigned int got = (unsigned int)old;
        if ((int)got >= limit) return -1;
        const unsigned long long prev = atomicCAS(word, old, old + (unsigned long long)step);
        if (prev == old) return (int)got;
        old = prev;
    }
}

// Block-wide exclusive prefix of popcounts over nwords bitmap words into bpre; total in
// sh->s0.  All threads call it; on return every thread sees all of bpre (a thread writes a
// run of ceil(nwords / threads) entries, so callers read entries other threads wrote).
template <typename BM, typename BP>  // global or LDS words
__device__ __forceinline__ void block_popcount_prefix(const BM *bitmap, BP *bpre, int nwords, WGShared *sh) {
    const int tid = threadIdx.x, nt = blockDim.x, wid = tid >> 6, nw = nt >> 6;
    const int per = (nwords + nt - 1) / nt;
    const int b0 = tid * per;
    int local = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nwords) local += __popcll(bitmap[b0 + q]);
    const int incl = wave_incl_scan(local);
    if (lane_id() == 63) sh->scan[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = sh->scan[w];
            sh->scan[w] = run;
            run += t;
        }
        sh->s0 = run;
    }
    __syncthreads();
    int run = sh->scan[wid] + incl - local;
    for (int q = 0; q < per; ++q) {
        if (b0 + q < nwords) {
            bpre[b0 + q] = (uint32_t)run;
            run += __popcll(bitmap[b0 + q]);
        }
    }
    wait_mem();
    __syncthreads();
}

// Moves the unclaimed rest [r, H) of the workgroup's top-level item list to its steal slot
// and marks the LDS item counter, so later claims go to the slot.  Lane 0 of the one wave that
// set the move flag from 0 to 2 calls it; the flag becomes 1 once the slot is out.
__device__ __forceinline__ void move_top_list(const SearchArgs &a, WGShared *sh, StealSlot *slot, lds_u32 *claim_l,
                                              lds_u32 *moved_l, int g, int k, int H, unsigned int epoch) {
    const uint32_t rest = lds_add32(claim_l, kMovedMark) & (kMovedMark - 1u);
    if ((int)rest < H) {
        slot->g = g;
        slot->k = k;
        slot->limit = H;
        __threadfence();
        __hip_atomic_store(&slot->word, ((unsigned long long)epoch << 32) | rest, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(a.steal_live, 1u);
        sh->published = 1;
    }
    __hip_atomic_store(moved_l, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A wave without work looks for a published third-level list with a chunk left -- the one its
// workgroup took (thief3), else one published by a wave of its workgroup -- and claims a
// chunk.  On success the claim and the list are left in the wave's share record (the list
// sits at depth 1 once rebuilt).  Returns false once no wave of the workgroup holds work, or
// a capacity ran out.  Every exit of its loop is wave-uniform.
__device__ __forceinline__ bool find_shared_list(const SearchArgs &a, WGShared *sh, lds_ws *me, lds_u32 *busyw,
                                              lds_u32 *idlew, lds_u32 *npub, int my_slot, int nw, bool thief3) {
    const int ln = lane_id();
    if (ln == 0) lds_add32(idlew, 1u);
    bool got_one = false;
    for (bool first = true;; first = false) {
        if (uni(__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & FLAG_RERUN) break;
        // the slots are read only while the workgroup has lists out (the list it took is
        // looked at once: its owner is in another workgroup)
        if (!(thief3 && first) && uni(__hip_atomic_load(npub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) == 0u) {
            if (uni(__hip_atomic_load(busyw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) == 0u) break;
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        // lane 0: the list this workgroup took; lanes 1..nw: its waves' slots
        int idx = -1;
        if (ln == 0) idx = thief3 && first ? sh->vpub : -1;
        else if (ln <= nw) idx = my_slot * a.pubw + (ln - 1);
        bool ok = false;
        unsigned int e = 0;
        int lim = 0, fi = 0, it = 0;
        if (idx >= 0) {
            PubSlot *ps = &a.pub[idx];
            const unsigned long long w1 = __hip_atomic_load(&ps->word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            e = (unsigned int)(w1 >> 32);
            if (e != 0u && (ln != 0 || e == sh->vepoch)) {
                lim = __hip_atomic_load(&ps->limit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fi = __hip_atomic_load(&ps->first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                it = __hip_atomic_load(&ps->i1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const unsigned long long w2 = __hip_atomic_load(&ps->word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                ok = (unsigned int)(w2 >> 32) == e && (int)(unsigned int)w2 < lim;
            }
        }
        const uint64_t okb = __ballot(ok);
        if (okb) {
            const int src = __ffsll((unsigned long long)okb) - 1;
            idx = __builtin_amdgcn_readlane(idx, src);
            e = (unsigned int)__builtin_amdgcn_readlane((int)e, src);
            lim = __builtin_amdgcn_readlane(lim, src);
            if (ln == 0) lds_add32(busyw, 1u);  // before the claim: waiting waves see work
            int got = 0;
            if (ln == 0) got = claim_chunk(&a.pub[idx].word, e, lim, 1u);
            got = __builtin_amdgcn_readlane(got, 0);
            if (got >= 0) {
                if (ln == 0) atomicAdd(&a.acc[ACC_SHARED], 1ull);
                me->cidx = idx;
                me->cepoch = e;
                me->cfirst = __builtin_amdgcn_readlane(fi, src);
                me->climit = lim;
                me->hitem = __builtin_amdgcn_readlane(it, src);
                me->pend = got;
                me->cdepth = 1;
                got_one = true;
                break;
            }
            if (ln == 0) lds_add32(busyw, ~0u);
            continue;
        }
        // nothing to take: done once no wave of the workgroup holds work
        if (uni(__hip_atomic_load(busyw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) == 0u) break;
        __builtin_amdgcn_s_sleep(8);
    }
    if (ln == 0) lds_add32(idlew, ~0u);
    return got_one;
}

// The classes of up to eight mask words keep four waves per SIMD resident (two 8-wave
// workgroups per compute unit): their register budget is capped at 128.  That spills some
// state to scratch (up to about 90 bytes per lane in the production instances, several
// hundred in the diagnostics instances), and still measured faster than 203-234 registers at
// two waves per SIMD: power-law step 47.8 -> 39.1 ms,
// skewed sample 1.76 -> 1.27 s.  The search waits on memory latency, and more resident waves
// hide it.
// TB (with DIAG and ENUM off): the production search, also tallying its design bytes.
template <int W, bool DIAG, bool ENUM, bool TB = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(W <= 8 ? 4 : 2))) void search_kernel(SearchArgs a, int64_t lo, int64_t hi, unsigned int *counter) {
    extern __shared__ unsigned char lds_raw[];
    WGShared *sh = reinterpret_cast<WGShared *>(lds_raw);
    const int tid = threadIdx.x, nt = blockDim.x, wid = uni(tid >> 6), nw = nt >> 6, ln = lane_id();
    constexpr int BITS = 64 * W;
    // third-level sharing is built into the multi-word classes only: the single-word class
    // (small top-level lists, register budget capped for residency) never publishes or helps
    constexpr bool kShare3 = W >= 2;
    const bool k3 = kShare3 && a.k3;

    // take a free arena slot (the launches of all mask classes share the slots; there are as
    // many as workgroups that can be resident at once, so one is always free)
    if (threadIdx.x == 0) {
        int got = -1;
        for (int round = 0; round < 64 && got < 0; ++round)
            for (int j = 0; j < a.nslots && got < 0; ++j) {
                const int sidx = (int)((blockIdx.x + (unsigned)j) % (unsigned)a.nslots);
                if (atomicCAS(&a.slot_busy[sidx], 0u, 1u) == 0u) got = sidx;
            }
        reinterpret_cast<WGShared *>(lds_raw)->slot = got;
        if (got < 0) atomicOr(a.flags, (unsigned int)FLAG_NO_SLOT);
    }
    __syncthreads();
    const int my_slot = reinterpret_cast<WGShared *>(lds_raw)->slot;
    if (my_slot < 0) return;
    char *wg = a.arena + (size_t)my_slot * a.lay.wg_bytes;
    uint64_t *bitmap = reinterpret_cast<uint64_t *>(wg + a.lay.off_bitmap);
    uint32_t *bpre = reinterpret_cast<uint32_t *>(wg + a.lay.off_bpre);
    uint64_t *M = reinterpret_cast<uint64_t *>(wg + a.lay.off_M);
    int32_t *gid = reinterpret_cast<int32_t *>(wg + a.lay.off_gid);
    uint32_t *cnt1 = reinterpret_cast<uint32_t *>(wg + a.lay.off_cnt);
    uint64_t *hvl = reinterpret_cast<uint64_t *>(wg + a.lay.off_hv);
    uint32_t *degl = reinterpret_cast<uint32_t *>(wg + a.lay.off_deg);
    uint32_t *t1v = reinterpret_cast<uint32_t *>(wg + a.lay.off_t1v);
    uint32_t *t1c = reinterpret_cast<uint32_t *>(wg + a.lay.off_t1c);
    uint32_t *s1 = reinterpret_cast<uint32_t *>(wg + a.lay.off_S1);
    uint64_t *hb = reinterpret_cast<uint64_t *>(wg + a.lay.off_hb);
    uint32_t *hpre = reinterpret_cast<uint32_t *>(wg + a.lay.off_hpre);
    uint32_t *hpos = reinterpret_cast<uint32_t *>(wg + a.lay.off_hpos);
    char *wv = wg + a.lay.off_waves + (size_t)wid * a.lay.wave_bytes;
    FrameState *hdr = reinterpret_cast<FrameState *>(wv + a.lay.off_w_hdr);

    Ctx c;
    c.gid = gid;
    c.M = M;
    c.hvl = hvl;
    c.degl = degl;
    c.c_off = a.c_off;
    c.s1 = s1;
    c.stk = reinterpret_cast<uint32_t *>(wv + a.lay.off_w_stack);
    c.stu = reinterpret_cast<uint32_t *>(wv + a.lay.off_w_u);
    c.hist = lds_at<lds_u32>(lds_raw, sizeof(WGShared) + (size_t)wid * BITS * 4);
    {
        // per wave: narrow-child tables first[64] cnt[64] (u32), H[64] (u64); kept Q' masks
        const size_t tb = sizeof(WGShared) + hist_region_bytes(BITS, nw) + (size_t)wid * kWaveLds;
        c.tl_first = lds_at<lds_u32>(lds_raw, tb);
        c.tl_cnt = c.tl_first + 64;
        c.tl_H = lds_at<lds_u64>(lds_raw, tb + 512);
        c.qk = lds_at<lds_u64>(lds_raw, tb + 1024);
        c.stu_l = reinterpret_cast<uint32_t *>(lds_raw + tb + 1024 + 8 * kQKeep);
    }
    // the rank bitmap and its prefix: in LDS when the launch's graphs are small enough
    const bool rl = a.dims.nwords <= kRankLdsWords;
    lds_u64 *const lbm = lds_at<lds_u64>(lds_raw, sizeof(WGShared) + hist_region_bytes(BITS, nw) + (size_t)nw * kWaveLds);
    lds_u32 *const lbp = reinterpret_cast<lds_u32 *>(lbm + (rl ? a.dims.nwords : 0));
    auto with_rank = [&](auto &&f) {
        if (rl) f(lbm, lbp);
        else f(bitmap, bpre);
    };
    if (rl)
        for (int wd = tid; wd < a.dims.nwords; wd += nt) lbm[wd] = 0ull;
    c.scap = a.dims.scap;
    c.c_is_v = 0;
    c.cbase = 0;
    c.obase = 0;
    c.Wroot = W;
    c.rec = a.rec;
    c.rec_cap = a.rec_cap;
    c.rec_offs = a.rec_offs;
    c.rec_offs_cap = a.rec_offs_cap;
    c.acc = a.acc;
    c.flags = a.flags;

    WaveAcc acc{};
    bool aborted = false;
    const int ucap = a.dims.ucap;
    if (tid < 16) sh->red[tid] = 0ull;
    uint64_t t_mark = DIAG ? clock64() : 0ull;  // start of the phase being timed
    // (tally instances) this workgroup's start on the wall clock and its time finding work
    const uint64_t ld_start = TB ? wall_clock64() : 0ull;
    uint64_t ld_wait = 0;
    if (tid == 0) {
        sh->graph = -1;
        sh->held = 0;
        sh->roots_done = 0;
        sh->others_done = 0;
        sh->npub = 0u;
    }
    __syncthreads();

    for (;;) {
        if (wid == 0) {
            // a fresh top-level candidate, else a share of another workgroup's top-level list,
            // else (third-level sharing) a third-level list; with third-level sharing on, a
            // workgroup that finds none waits while others of its launch are busy, once no
            // launch has top-level candidates left (before that, leaving frees the CU for
            // the other launches).  Stop once a capacity ran out (the host reruns).
            if (ln == 0) {
                if (sh->held) atomicSub(a.busy, 1u);
                sh->held = 0;
            }
            bool waited = false;
            const uint64_t ld_w0 = TB ? wall_clock64() : 0ull;
            for (;;) {
                int mode = 0;
                unsigned int t = 0;
                if (ln == 0) {
                    const unsigned int f = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (f & FLAG_RERUN) {
                        mode = -1;
                    } else if (!sh->roots_done) {
                        for (;;) {
                            t = atomicAdd(counter, 1u);
                            if (lo + (int64_t)t >= hi) {
                                sh->roots_done = 1;
                                break;
                            }
                            if (!root_cancelled(a, lo + (int64_t)t)) {
                                mode = 1;
                                break;
                            }
                        }
                    }
                }
                mode = __builtin_amdgcn_readlane(mode, 0);
                if (mode == 1) {
                    if (ln == 0) {
                        sh->mode = 1;
                        sh->task = t;
                        sh->epoch = t + 1u;
                    }
                    break;
                }
                if (mode < 0) {
                    if (ln == 0) sh->mode = 0;
                    break;
                }
                // a published top-level list with at least two unclaimed items, else (third-level
                // sharing) a published third-level list with at least two unclaimed chunks; 64
                // slots at a time (the two slot kinds share their head fields and stride)
                bool found = false;
#pragma unroll 1
                for (int kind = 0; kind < 2 && !found; ++kind) {
                    const bool on = kind == 0 ? a.steal_on != 0 : k3;
                    if (!on || __hip_atomic_load(kind == 0 ? a.steal_live : a.pub_live, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT) == 0u)
                        continue;
                    char *arr = kind == 0 ? reinterpret_cast<char *>(a.steal) : reinterpret_cast<char *>(a.pub);
                    const int total = kind == 0 ? a.nslots : a.nslots * a.pubw;
                    const int start = kind == 0 ? my_slot : my_slot * a.pubw;
                    for (int base = 1 - kind; base < total && !found; base += 64) {  // (not its own slot)
                        const int j = base + ln;
                        bool ok = false;
                        int idx = 0, sg = 0, sk = 0;
                        unsigned int e = 0;
                        if (j < total) {
                            idx = (start + j) % total;
                            StealSlot *sl = reinterpret_cast<StealSlot *>(arr + (size_t)idx * sizeof(StealSlot));
                            const unsigned long long w1 =
                                __hip_atomic_load(&sl->word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                            e = (unsigned int)(w1 >> 32);
                            if (e != 0u) {
                                sg = __hip_atomic_load(&sl->g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                sk = __hip_atomic_load(&sl->k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                const int lim = __hip_atomic_load(&sl->limit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                                const unsigned long long w2 =
                                    __hip_atomic_load(&sl->word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                                // the owner has not moved on, and two or more are left
                                ok = (unsigned int)(w2 >> 32) == e && (int)(unsigned int)w2 + 2 <= lim;
                            }
                        }
                        const uint64_t okb = __ballot(ok);
                        if (okb) {
                            const int src = __ffsll((unsigned long long)okb) - 1;
                            idx = __builtin_amdgcn_readlane(idx, src);
                            sg = __builtin_amdgcn_readlane(sg, src);
                            sk = __builtin_amdgcn_readlane(sk, src);
                            e = (unsigned int)__builtin_amdgcn_readlane((int)e, src);
                            if (ln == 0) {
                                sh->mode = 2 + kind;
                                sh->victim = idx;
                                sh->vpub = idx;
                                sh->epoch = e;
                                sh->vepoch = e;
                                sh->sg = sg;
                                sh->sk = sk;
                            }
                            found = true;
                        }
                    }
                }
                if (found) break;
                int wait = 0;
                if (ln == 0 && (k3 || a.steal_on) &&
                    __hip_atomic_load(a.busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0u) {
                    wait = 1;
                    if (!sh->others_done) {
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            if (q != a.cls && (int64_t)__hip_atomic_load(&a.cls_ctr[q], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT) < a.cls_n[q])
                                wait = 0;
                        if (wait) sh->others_done = 1;  // (they stay handed out)
                    }
                }
                if (!__builtin_amdgcn_readlane(wait, 0)) {
                    if (ln == 0) sh->mode = 0;
                    break;
                }
                if (ln == 0 && !waited) atomicAdd(a.hungry, 1u);
                waited = true;
                __builtin_amdgcn_s_sleep(64);
            }
            if (ln == 0) {
                if (waited) atomicSub(a.hungry, 1u);
                if (sh->mode != 0) {
                    atomicAdd(a.busy, 1u);
                    sh->held = 1;
                }
            }
            if (TB) ld_wait += wall_clock64() - ld_w0;
        }
        __syncthreads();
        if (DIAG) {
            const uint64_t now = clock64();
            acc.ph[PH_WAIT] += now - t_mark;
            t_mark = now;
        }
        const int mode = uni(sh->mode);
        if (mode == 0) break;
        const bool thief = mode >= 2;  // the top-level node belongs to another workgroup
        const bool thief3 = kShare3 && mode == 3;
        int g = 0;
        int64_t k;
        if (thief) {
            g = uni(sh->sg);
            k = uni(sh->sk);
        } else if (a.tasks) {
            const unsigned long long tk = a.tasks[lo + (int64_t)sh->task];
            g = (int)(tk >> 32);
            k = (int64_t)(tk & 0xFFFFFFFFull);
        } else {
            k = hi - 1 - (int64_t)sh->task;  // ranks are claimed from the top (largest degree) down
        }
        if (g != sh->graph) {
            // tallies belong to the graph they were found in
            if (sh->graph >= 0) flush_acc<DIAG, TB>(acc, a.graphs[sh->graph].acc, sh);
            __syncthreads();
            if (tid == 0) sh->graph = g;
            __syncthreads();
        }
        const GraphDesc gd = a.graphs[g];
        c.c_is_v = gd.c_is_v;
        c.cbase = gd.cbase;
        c.obase = gd.obase;
        const int nwords = gd.nwords;
        const int32_t x = gd.order[k];
        const int32_t rb = a.c_off[x];
        const int32_t d = a.c_off[x + 1] - rb;
        const int32_t *row = a.c_adj + rb;
        c.row = row;
        c.x_root = x;

        // -- the 2-hop walk of x, spread over the whole workgroup: walk index t belongs to the
        //    neighbour w_j with woff[j] <= t < woff[j+1] and reads entry wbase[j] + t - woff[j]
        //    of the other side's CSR (a hub neighbour no longer holds up one wave alone)
        // (wide classes keep one neighbour per wave: their registers are spent elsewhere)
        constexpr bool kFlatWalk = W <= 2;
        lds_u32 *woff = lds_at<lds_u32>(lds_raw, sizeof(WGShared));
        lds_u32 *wbase = woff + (BITS + 1);
        if (kFlatWalk && wid == 0) {
            int carry = 0;
            for (int base = 0; base < d; base += 64) {
                const int j = base + ln;
                int dw = 0;
                if (j < d) {
                    const int32_t w = row[j];
                    const int32_t e0 = a.o_off[w];
                    dw = a.o_off[w + 1] - e0;
                    wbase[j] = (uint32_t)e0;
                }
                const int incl = wave_incl_scan(dw);
                if (j < d) woff[j] = (uint32_t)(carry + incl - dw);
                carry += last_lane(incl);
            }
            if (ln == 0) woff[d] = (uint32_t)carry;
        }
        if (kFlatWalk) __syncthreads();
        const int walk = kFlatWalk ? (int)uni(woff[d]) : 0;
        auto walk_at = [&](int t, int &j) {
            int lo = 0, hi = d - 1;  // the last neighbour whose walk starts at or before t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int)woff[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            j = lo;
            return a.o_adj[wbase[lo] + (uint32_t)(t - (int)woff[lo])];
        };

        // -- reverse scan 1: mark the ranks of all 2-hop neighbours of x
        with_rank([&](auto *bm, auto *) {
            if constexpr (kFlatWalk) {
                for (int t = tid; t < walk; t += nt) {
                    int j;
                    const int32_t v = walk_at(t, j);
                    if (v != x) {
                        const int32_t rk = a.rank[v];
                        bm_or(&bm[rk >> 6], 1ull << (rk & 63));
                    }
                }
            } else {
                for (int j = wid; j < d; j += nw) {
                    const int32_t w = row[j];
                    const int32_t e0 = a.o_off[w], e1 = a.o_off[w + 1];
                    for (int p = e0 + ln; p < e1; p += 64) {
                        const int32_t v = a.o_adj[p];
                        if (v != x) {
                            const int32_t rk = a.rank[v];
                            bm_or(&bm[rk >> 6], 1ull << (rk & 63));
                        }
                    }
                }
            }
        });
        uint64_t hv_local = 0, rs_local = 0;
        for (int j = tid; j < BITS; j += nt) {
            if (j < d) {
                const int32_t w = row[j];
                const uint64_t h = hr(c, w);
                hvl[j] = h;
                hv_local += h;
                const uint32_t dw = (uint32_t)(a.o_off[w + 1] - a.o_off[w]);
                degl[j] = dw;
                rs_local += 2ull + dw;
            } else {
                hvl[j] = 0ull;
                degl[j] = 0u;
            }
        }
        if (tid == 0) {
            sh->nonmax = 0;
            sh->pcount = 0;
            sh->exps = 0;
            sh->fw1 = 0;
            sh->hvsum = 0;
            sh->rs1 = 0;
            sh->nexp = 0;
            sh->claim = 0u;
            sh->moved = 0u;
            sh->published = 0;
            sh->gclaim = 0;
        }
        __syncthreads();
        see_atomics();  // the rank bitmap was built with atomics
        hv_local = wave_sum_u64(hv_local);
        rs_local = wave_sum_u64(rs_local);
        if (ln == 0) {
            lds_add(&sh->hvsum, hv_local);
            lds_add(&sh->rs1, rs_local);
        }

        // -- universe numbering: prefix of bitmap popcounts (rank order)
        with_rank([&](auto *bm, auto *bp) { block_popcount_prefix(bm, bp, nwords, sh); });
        wait_mem();
        __syncthreads();
        const int s0 = uni(sh->s0);
        if (s0 > ucap) {
            // the universe does not fit: clear the bitmap, note the size, skip (rerun later)
            with_rank([&](auto *bm, auto *) {
                for (int wd = tid; wd < nwords; wd += nt) bm[wd] = 0ull;
            });
            if (tid == 0) {
                atomicOr(a.flags, (unsigned int)FLAG_UNIVERSE_OVERFLOW);
                atomicMax(&a.acc[ACC_NEED_UCAP], (unsigned long long)s0);
            }
            __syncthreads();
            if (DIAG) {
                const uint64_t now = clock64();
                acc.ph[PH_ROOT] += now - t_mark;
                t_mark = now;
            }
            continue;
        }
        int nq0 = 0;
        with_rank([&](auto *bm, auto *bp) {
            nq0 = (int)bp[k >> 6] + __popcll(bm[k >> 6] & ((1ull << (k & 63)) - 1ull));
            for (int wd = tid; wd < nwords; wd += nt) {
                uint64_t bits = bm[wd];
                uint32_t pos = bp[wd];
                while (bits) {
                    const int b = __ffsll((unsigned long long)bits) - 1;
                    bits &= bits - 1ull;
                    gid[pos++] = gd.order[wd * 64 + b];
                }
            }
        });
        nq0 = uni(nq0);
        c.s0 = s0;
        for (size_t q = tid; q < (size_t)s0 * W; q += nt) M[q] = 0ull;
        wait_mem();
        __syncthreads();

        // -- reverse scan 2: M[v] gets bit j for every w_j in N(x) adjacent to v
        with_rank([&](auto *bm, auto *bp) {
            if constexpr (kFlatWalk) {
                for (int t = tid; t < walk; t += nt) {
                    int j;
                    const int32_t v = walk_at(t, j);
                    if (v != x) {
                        const int32_t rk = a.rank[v];
                        const uint32_t li =
                            bp[rk >> 6] + (uint32_t)__popcll(bm[rk >> 6] & ((1ull << (rk & 63)) - 1ull));
                        atomicOr(reinterpret_cast<unsigned long long *>(&M[(size_t)li * W + (j >> 6)]), 1ull << (j & 63));
                    }
                }
            } else {
                for (int j = wid; j < d; j += nw) {
                    const int32_t w = row[j];
                    const int32_t e0 = a.o_off[w], e1 = a.o_off[w + 1];
                    for (int p = e0 + ln; p < e1; p += 64) {
                        const int32_t v = a.o_adj[p];
                        if (v != x) {
                            const int32_t rk = a.rank[v];
                            const uint32_t li =
                                bp[rk >> 6] + (uint32_t)__popcll(bm[rk >> 6] & ((1ull << (rk & 63)) - 1ull));
                            atomicOr(reinterpret_cast<unsigned long long *>(&M[(size_t)li * W + (j >> 6)]), 1ull << (j & 63));
                        }
                    }
                }
            }
        });
        __syncthreads();
        see_atomics();  // M was built with atomics

        // -- the top-level node for x: counts, maximality against earlier ranks, expansion
        with_rank([&](auto *bm, auto *) {
            for (int wd = tid; wd < nwords; wd += nt) bm[wd] = 0ull;
        });
        {
            bool nm = false;
            int pc = 0, nexp = 0;
            uint64_t ex = 0, fw = 0;
            for (int li = tid; li < s0; li += nt) {
                int cc = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) cc += __popcll(M[(size_t)li * W + w]);
                cnt1[li] = (uint32_t)cc;
                const int32_t g = gid[li];
                const uint64_t dg = DIAG ? 2ull + (uint64_t)(a.c_off[g + 1] - a.c_off[g]) : 0ull;
                if (li < nq0) {
                    if (cc == d) {
                        nm = true;
                    } else {
                        fw += dg;
                    }
                } else if (cc == d) {
                    ex += hl(c, g);
                    ++nexp;
                } else {
                    ++pc;
                    fw += dg;
                }
            }
            if (__ballot(nm) && ln == 0) atomicOr(&sh->nonmax, 1);
            ex = wave_sum_u64(ex);
            fw = wave_sum_u64(fw);
            pc = wave_sum_i32(pc);
            nexp = wave_sum_i32(nexp);
            if (ln == 0) {
                atomicAdd(&sh->pcount, pc);
                atomicAdd(&sh->nexp, nexp);
                lds_add(&sh->exps, ex);
                lds_add(&sh->fw1, fw);
            }
        }
        wait_mem();
        __syncthreads();
        const bool root_nonmax = uni(sh->nonmax) != 0;
        const int P1 = uni(sh->pcount);
        if (TB && tid == 0 && !thief) {
            // x's row; its neighbours' offsets (walk set-up, hash and degree terms); both reverse
            // scans (rows, ranks and mask atomics; bitmap atomics and the universe index lookups
            // unless the bitmap is in LDS); the terms per position of N(x); bitmap prefix,
            // universe ids and bitmap clear (the bitmap's part unless in LDS); universe masks
            // cleared, then read with the counts and ids
            const uint64_t dd = (uint64_t)d, wk = (uint64_t)sh->rs1 - 2ull * dd, su = (uint64_t)s0;
            acc.dbytes += 4ull * (dd + 2ull) + 16ull * dd + (rl ? 24ull : 44ull) * wk + 12ull * BITS +
                          (rl ? 0ull : 32ull * (uint64_t)nwords) + 8ull * su + 16ull * W * su + 8ull * su;
        }
        if (tid == 0 && !thief) {  // a stolen task's top-level node belongs to its owner
            const uint64_t dx = (uint64_t)d;
            if (DIAG) {
                acc.nodes += 1;
                if (acc.max_depth < 1) acc.max_depth = 1;
                const uint64_t fwtop = gd.total_fw - (2ull + dx);
                const uint64_t rs = sh->rs1;
                uint64_t b = (2ull + dx) + (rs < fwtop ? rs : fwtop) + (uint64_t)(gd.ncand - 1) + dx;
                if (root_nonmax) acc.nonmax += 1;
                else b += (uint64_t)P1 + (uint64_t)nq0;
                acc.bytes += 4ull * b;
            }
            if (!root_nonmax) {
                const uint64_t sL = hl(c, x) + sh->exps;
                const int nL = 1 + sh->nexp;
                acc.count += 1;
                acc.hash += pair_hash(c.c_is_v, sL, sh->hvsum);
                acc.out_ints += 2ull + (uint64_t)nL + (uint64_t)d;
            }
        }
        if (ENUM && !root_nonmax && !thief && wid == 0) {
            uint64_t R1[16];
            for (int w = 0; w < 16; ++w) {
                const int bits = d - 64 * w;
                R1[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : ((1ull << bits) - 1ull));
            }
            write_record(c, R1, 1 + sh->nexp, d);
        }
        if (root_nonmax || P1 == 0) {
            __syncthreads();
            if (DIAG) {
                const uint64_t now = clock64();
                acc.ph[PH_ROOT] += now - t_mark;
                t_mark = now;
            }
            continue;
        }
        // -- Q1 of the list: the universe entries ranked before x (all of them meet N(x)).
        //    With diagnostics off, a single-bit mask is dropped when a Q1 mask of two or more
        //    bits holds its bit, and of the other single-bit masks only the first per bit is
        //    kept: a Q entry only witnesses that some R (a subset of N(x)) is not maximal, and
        //    the dropped ones witness nothing the kept ones do not.  The count stays nq0 in
        //    the tallies of diagnostics mode, which keep the method's full Q1.  Lists of up
        //    to 256 are kept whole: there the pass's workgroup barriers cost more than the
        //    shorter child lists save (measured).
        uint32_t *ids1 = s1;
        if (!DIAG && nq0 > 256) {
            lds_u32 *first1 = lds_at<lds_u32>(lds_raw, sizeof(WGShared));  // BITS words
            for (int b = tid; b < BITS; b += nt) first1[b] = kNone;
            if (tid < W) sh->cov[tid] = 0ull;
            __syncthreads();
            for (int li = tid; li < nq0; li += nt)
                if (cnt1[li] >= 2u) {
#pragma unroll 1
                    for (int w = 0; w < W; ++w) {
                        const uint64_t y = M[(size_t)li * W + w];
                        if (y) lds_or(&sh->cov[w], y);
                    }
                }
            __syncthreads();
            auto single_bit = [&](int li) {
                int b = 0;
#pragma unroll 1
                for (int w = 0; w < W; ++w) {
                    const uint64_t y = M[(size_t)li * W + w];
                    if (y) b = 64 * w + __ffsll((unsigned long long)y) - 1;
                }
                return b;
            };
            for (int li = tid; li < nq0; li += nt)
                if (cnt1[li] == 1u) {
                    const int b = single_bit(li);
                    if (!((sh->cov[b >> 6] >> (b & 63)) & 1ull)) lds_min32(&first1[b], (uint32_t)li);
                }
            __syncthreads();
            const int nwq = (nq0 + 63) >> 6;
            for (int q = wid; q < nwq; q += nw) {
                const int li = 64 * q + ln;
                bool keep = false;
                if (li < nq0) keep = cnt1[li] >= 2u || first1[single_bit(li)] == (uint32_t)li;
                const uint64_t kb = __ballot(keep);
                if (ln == 0) hb[q] = kb;
            }
            wait_mem();
            __syncthreads();
            block_popcount_prefix(hb, hpre, nwq, sh);
            for (int q = tid; q < nwq; q += nt) {
                uint64_t bits = hb[q];
                uint32_t at = hpre[q];
                while (bits) {
                    const int bb = __ffsll((unsigned long long)bits) - 1;
                    bits &= bits - 1ull;
                    ids1[at++] = (uint32_t)(64 * q + bb);
                }
            }
        } else {
            for (int li = tid; li < nq0; li += nt) ids1[li] = (uint32_t)li;
            if (tid == 0) sh->s0 = nq0;
        }
        __syncthreads();
        const int nqk = uni(sh->s0);  // Q1 entries kept in the list
        const int n1 = nqk + P1;

        // -- the top-level child list as a frame: ids Q1 (earlier ranks) ++ P1 sorted by
        //    count, masks over the positions of N(x), per-bit tables
        FrameView v1 = frame_view(s1, n1, W, d);
        if (wid == 0) {
            int pn = 0;
            for (int base = nq0; base < s0; base += 64) {
                const int li = base + ln;
                const bool act = li < s0;
                const uint32_t cc = act ? cnt1[li] : 0u;
                const bool pk = act && (int)cc < d;
                const uint64_t pb = __ballot(pk);
                if (pk) {
                    const int p = pn + __popcll(pb & lanes_below());
                    t1v[p] = (uint32_t)li;
                    t1c[p] = cc;
                }
                pn += __popcll(pb);
            }
            wait_mem();
            wave_sort_by_key(t1v, t1c, pn, d, c.hist, [&](uint32_t slot, uint32_t li) { ids1[nqk + slot] = li; });
        }
        // per-bit tables accumulated in LDS (the histograms' space, idle here, 16 bytes per
        // bit), then written out
        lds_u64 *lH = lds_at<lds_u64>(lds_raw, sizeof(WGShared));
        lds_u32 *lfirst = lds_at<lds_u32>(lds_raw, sizeof(WGShared) + (size_t)BITS * 8);
        lds_u32 *lcnt = lfirst + BITS;
        __syncthreads();  // wave 0's sort is done with its histogram
        for (int b = tid; b < BITS; b += nt) {
            lfirst[b] = kNone;
            lcnt[b] = 0u;
            lH[b] = 0ull;
        }
        wait_mem();
        __syncthreads();
        uint64_t *masks1 = const_cast<uint64_t *>(v1.masks);
        uint64_t *hs1 = const_cast<uint64_t *>(v1.hs);
        for (int j = tid; j < n1; j += nt) {
            const uint32_t li = ids1[j];
            const uint64_t h = hl(c, gid[li]);
            hs1[j] = h;
            const uint64_t ht = j < nqk ? 0ull : h;  // Q entries carry no hash term
#pragma unroll 1
            for (int w = 0; w < W; ++w) {
                uint64_t mm = M[(size_t)li * W + w];
                masks1[(size_t)j * W + w] = mm;
                while (mm) {
                    const int b = 64 * w + __ffsll((unsigned long long)mm) - 1;
                    mm &= mm - 1ull;
                    lds_min32(&lfirst[b], (uint32_t)j);
                    lds_add32(&lcnt[b], 1u);
                    lds_add64(&lH[b], ht);
                }
            }
        }
        __syncthreads();
        for (int b = tid; b < BITS; b += nt) {
            v1.first[b] = lfirst[b];
            v1.cnt[b] = lcnt[b];
            v1.H[b] = lH[b];
        }
        // position rows of the top-level list, one (64-entry chunk, mask word) block per wave
        const int qd = (d + 63) >> 6;  // mask words holding bits of N(x)
        for (int job = wid; job < v1.nw * qd; job += nw) {
            const int w = job / qd, q = job - w * qd;
            const int j = 64 * w + ln;
            const uint64_t t = wave_transpose64(j < n1 ? masks1[(size_t)j * W + q] : 0ull);
            if (64 * q + ln < d) v1.rows[(size_t)(64 * q + ln) * v1.nw + w] = t;
        }
        wait_mem();
        __syncthreads();

        // -- top-level light pass: chunks of P1 are split over the waves; candidates with
        //    |R'| = 1 are settled here (by the owner only), and those with |R'| >= 2 are
        //    flagged per chunk.  Their ordered list hpos depends on the list alone, so a
        //    thief that rebuilt the list finds the same items at the same indices.
        FrameState top;
        top.off = kShared;
        top.top = 0;
        top.n = n1;
        top.nq = nqk;
        top.level = 2;
        top.nL = 1 + sh->nexp;
        top.wf = W;
        top.narrow = 0;
        top.chunk = 0;
        top.rbits = d;
        top.heavy = 0ull;
        top.sL = hl(c, x) + sh->exps;
        top.fw = uni((uint64_t)sh->fw1);
        const int nch = thief3 ? 0 : (P1 + 63) >> 6;  // a third-level thief takes no top-level item
        for (int q = wid; q < nch; q += nw) {
            const uint64_t tl = DIAG ? clock64() : 0ull;
            const uint64_t hm = light_chunk<W, DIAG, ENUM, TB>(c, top, v1, nqk + 64 * q, acc, !thief);
            if (DIAG) acc.ph[PH_LIGHT] += clock64() - tl;
            if (ln == 0) hb[q] = hm;
        }
        wait_mem();
        __syncthreads();
        block_popcount_prefix(hb, hpre, nch, sh);
        for (int q = tid; q < nch; q += nt) {
            uint64_t bits = hb[q];
            uint32_t at = hpre[q];
            while (bits) {
                const int bb = __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1ull;
                hpos[at++] = (uint32_t)(nqk + 64 * q + bb);
            }
        }
        wait_mem();
        __syncthreads();
        const int H = uni(sh->s0);
        if (TB && tid == 0 && !thief) {
            // the top-level list: Q1 (pruned, or copied), P1 staged and sorted, ids / hash terms /
            // masks (universe masks read), tables, rows (list masks read, rows written), chunk
            // flags, their prefix and the item list (written, read at the claims), the header
            const uint64_t n1u = (uint64_t)n1, q0 = (uint64_t)nq0;
            uint64_t b = (!DIAG && nq0 > 256)
                             ? q0 * (12ull + 16ull * W) + 12ull * (uint64_t)((nq0 + 63) >> 6) + 4ull * (uint64_t)nqk
                             : 4ull * q0;
            b += 4ull * (uint64_t)(s0 - nq0) + 20ull * (uint64_t)P1;
            b += n1u * (24ull + 16ull * W) + 16ull * BITS;
            b += 8ull * n1u * (uint64_t)qd + 8ull * (uint64_t)d * (uint64_t)v1.nw;
            b += 24ull * (uint64_t)nch + 8ull * (uint64_t)H + sizeof(FrameState);
            acc.dbytes += b;
        }

        // -- share the items.  The owner's waves claim them from an LDS counter; once a
        //    workgroup of the launch is idle, the wave whose claim notices it moves the rest of
        //    the list to the global steal slot, and from then on everyone (idle workgroups
        //    rebuild the same list) claims there.  A thief claims there from the start.
        StealSlot *slot = mode == 2 ? &a.steal[sh->victim] : &a.steal[my_slot];
        if (tid == 0) {
            sh->topf = top;
            sh->tg = g;
            sh->tk = (int)k;
            sh->busyw = thief3 ? 0u : (uint32_t)nw;
            sh->idlew = 0u;
            if (mode == 2) sh->gclaim = 1;
        }
        __syncthreads();
        bool gclaim = uni(sh->gclaim) != 0;
        lds_u32 *claim_l = lds_at<lds_u32>(lds_raw, offsetof(WGShared, claim));
        lds_u32 *moved_l = lds_at<lds_u32>(lds_raw, offsetof(WGShared, moved));
        const unsigned int epoch = uni(sh->epoch);
        if (DIAG) {
            const uint64_t now = clock64();
            acc.ph[PH_ROOT] += now - t_mark;
            t_mark = now;
        }

        // -- second level and below.  Each wave claims one top-level item at a time, expands
        //    it and searches depth-first below it.  With third-level sharing, a wave whose
        //    second-level list (depth 1) still has two or more chunks to go publishes it in
        //    its slot once some wave or workgroup is idle, and from then on takes that list's
        //    chunks through the slot like anyone else.  A wave left without work helps: it
        //    claims a chunk of a list published by a wave of its workgroup (or of the
        //    third-level list this workgroup took), rebuilds the list from the top-level frame
        //    (the owner's own node call, reporting nothing; lists are built deterministically)
        //    and searches the chunks it claims.  Nobody waits for a helper: every chunk is
        //    searched by the wave that claimed it, and an owner claims until none is left.
        lds_u32 *busyw = lds_at<lds_u32>(lds_raw, offsetof(WGShared, busyw));
        lds_u32 *idlew = lds_at<lds_u32>(lds_raw, offsetof(WGShared, idlew));
        lds_u32 *npub = lds_at<lds_u32>(lds_raw, offsetof(WGShared, npub));
        lds_ws *me = lds_at<lds_ws>(lds_raw, offsetof(WGShared, ws) + (size_t)wid * sizeof(WaveShare));
        me->cdepth = -1;
        me->cown = 0;
        me->hitem = -1;
        me->pend = -1;
        hdr[0] = top;  // every lane stores the same header
        wait_mem();
        bool src_top = !thief3;  // the current source: top-level items (else one published list)
        // idle workgroups of this launch, as read at the previous check (the load is issued
        // one check ahead, so its latency hides under the chunk in between)
        uint32_t hungry_seen = 0u;
        for (;;) {
            if (!src_top && !find_shared_list(a, sh, me, busyw, idlew, npub, my_slot, nw, thief3)) break;
            FrameState cur = uni_frame(sh->topf);
            int depth = 0;
            while (!aborted) {
                const FrameView v = frame_view(frame_base(c, cur.off), cur.n, cur.wf, cur.rbits);
                int i;
                if (depth == 0) {
                    if (src_top) {
                        int got = 0, mv = 0;
                        if (ln == 0) {
                            if (gclaim) {
                                got = claim_chunk(&slot->word, epoch, H, 1u);
                            } else {
                                const uint32_t t = lds_add32(claim_l, 1u);
                                got = (int)(t & (kMovedMark - 1u));
                                if (t >= kMovedMark) {
                                    // the rest of the list went to the steal slot: wait until it
                                    // is out (the moving wave is a few stores from done), claim there
                                    while (__hip_atomic_load(moved_l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 1u)
                                        __builtin_amdgcn_s_sleep(1);
                                    got = claim_chunk(&slot->word, epoch, H, 1u);
                                    mv = 1;
                                } else if (uint32_t none = 0u;
                                           a.steal_on && got + 2 < H && (got & 7) == 0 &&
                                           __hip_atomic_load(a.hungry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0u &&
                                           __hip_atomic_compare_exchange_strong(moved_l, &none, 2u, __ATOMIC_RELAXED,
                                                                               __ATOMIC_RELAXED,
                                                                               __HIP_MEMORY_SCOPE_WORKGROUP)) {
                                    // a workgroup is idle: move the rest of the list to the steal
                                    // slot (this claim keeps item got)
                                    move_top_list(a, sh, slot, claim_l, moved_l, g, (int)k, H, epoch);
                                    mv = 1;
                                }
                            }
                        }
                        got = __builtin_amdgcn_readlane(got, 0);
                        if (__builtin_amdgcn_readlane(mv, 0)) gclaim = true;
                        if (got < 0 || got >= H) break;
                        i = (int)uni(hpos[got]);
                        if (k3) me->item1 = i;
                    } else {
                        // a helped list: rebuild it once (the node call below reports nothing)
                        i = uni(me->hitem);
                        if (i < 0) break;
                        me->hitem = -1;
                    }
                } else {
                    if (cur.heavy == 0ull) {
                        int base = cur.chunk + 64;
                        if (kShare3 && a.steal_on && depth == 1) {
                            if (k3 && uni(me->cdepth) == 1) {
                                int got = uni(me->pend);
                                me->pend = -1;
                                if (got < 0) {
                                    if (ln == 0) {
                                        got = claim_chunk(&a.pub[me->cidx].word, me->cepoch, me->climit, 1u);
                                        if (got >= 0 && !me->cown) atomicAdd(&a.acc[ACC_SHARED], 1ull);
                                    }
                                    got = __builtin_amdgcn_readlane(got, 0);
                                }
                                if (got >= 0) {
                                    base = uni(me->cfirst) + 64 * got;
                                } else {
                                    // every chunk is claimed: the owner withdraws the list
                                    base = cur.n;
                                    if (ln == 0 && me->cown) {
                                        __hip_atomic_store(&a.pub[me->cidx].word, 0ull, __ATOMIC_RELEASE,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                                        atomicSub(a.pub_live, 1u);
                                        lds_add32(npub, ~0u);
                                    }
                                    me->cown = 0;
                                    me->cdepth = -1;
                                }
                            } else if (src_top) {
                                // idle workgroups of this launch, as read at the previous check
                                // (the load is issued one check ahead: its latency hides under
                                // the chunk in between)
                                const bool want = uni(hungry_seen) > 0u;
                                hungry_seen = __hip_atomic_load(a.hungry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                if (want) {
                                    // the top-level list goes out first (its items are the coarser
                                    // work): the owner's next top-level claim may be far off when
                                    // second-level subtrees are large
                                    // (the owning workgroup's list only: a thief's slot is its victim's)
                                    if (ln == 0 && mode == 1 &&
                                        __hip_atomic_load(moved_l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u &&
                                        (int)(__hip_atomic_load(claim_l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) &
                                              (kMovedMark - 1u)) + 1 < H) {
                                        uint32_t none = 0u;
                                        if (__hip_atomic_compare_exchange_strong(moved_l, &none, 2u, __ATOMIC_RELAXED,
                                                                                 __ATOMIC_RELAXED,
                                                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
                                            move_top_list(a, sh, slot, claim_l, moved_l, g, (int)k, H, epoch);
                                    }
                                    if (k3 && cur.n - base > 64) {
                                        // publish the rest of this list, then claim its chunks like a helper
                                        const int idx = my_slot * a.pubw + wid;
                                        const int lim = (cur.n - base + 63) >> 6;
                                        if (ln == 0) {
                                            PubSlot *mp = &a.pub[idx];
                                            const unsigned int e = atomicAdd(a.epoch_ctr, 1u) + 1u;
                                            mp->g = sh->tg;
                                            mp->k = sh->tk;
                                            mp->i1 = me->item1;
                                            mp->first = base;
                                            mp->limit = lim;
                                            __threadfence();
                                            __hip_atomic_store(&mp->word, (unsigned long long)e << 32, __ATOMIC_RELEASE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                                            atomicAdd(a.pub_live, 1u);
                                            lds_add32(npub, 1u);
                                            me->cepoch = e;
                                        }
                                        me->cidx = idx;
                                        me->cfirst = base;
                                        me->climit = lim;
                                        me->cdepth = 1;
                                        me->cown = 1;
                                        continue;
                                    }
                                }
                            }
                        }
                        if (base >= cur.n) {
                            --depth;
                            cur = uni_frame(hdr[depth]);  // hdr[0] holds the top-level list
                            continue;
                        }
                        cur.chunk = base;
                        const uint64_t tl = DIAG ? clock64() : 0ull;
                        cur.heavy = (cur.wf == 1) ? light_chunk<1, DIAG, ENUM, TB>(c, cur, v, base, acc)
                                                  : light_chunk<W, DIAG, ENUM, TB>(c, cur, v, base, acc);
                        if (DIAG) acc.ph[PH_LIGHT] += clock64() - tl;
                        continue;
                    }
                    const int lane = __ffsll((unsigned long long)cur.heavy) - 1;
                    cur.heavy &= cur.heavy - 1ull;
                    i = cur.chunk + lane;
                }
                FrameState ch;
                const bool report = src_top || depth > 0;
                const bool pushed = (cur.wf == 1) ? heavy_node<1, W, DIAG, ENUM, TB>(c, cur, v, i, ch, acc, report)
                                                  : heavy_node<W, W, DIAG, ENUM, TB>(c, cur, v, i, ch, acc, report);
                if (pushed) {
                    if (depth >= a.dims.maxdepth) {
                        if (ln == 0) atomicOr(a.flags, (unsigned int)FLAG_DEPTH_OVERFLOW);
                        aborted = true;
                        break;
                    }
                    if (depth > 0) {
                        hdr[depth] = cur;  // every lane stores the same header
                        wait_mem();
                        if (TB && ln == 0) acc.dbytes += 2ull * sizeof(FrameState);  // saved, read back on return
                    }
                    ++depth;
                    cur = ch;
                } else if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_STACK_OVERFLOW) {
                    aborted = true;
                }
            }
            if (!k3) break;
            // a helped list whose rebuild pushed no frame (the owner's call did; never reached)
            if (!src_top && !aborted && uni(me->pend) >= 0 && ln == 0)
                atomicOr(a.flags, (unsigned int)FLAG_SHARE_MISMATCH);
            // (after an abort) a list still published is withdrawn
            if (ln == 0 && me->cown) {
                __hip_atomic_store(&a.pub[me->cidx].word, 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                atomicSub(a.pub_live, 1u);
                lds_add32(npub, ~0u);
            }
            me->cown = 0;
            me->cdepth = -1;
            me->pend = -1;
            me->hitem = -1;
            if (ln == 0) lds_add32(busyw, ~0u);  // this wave's work in the source is done
            if (aborted) break;
            src_top = false;
        }
        if (DIAG) t_mark = clock64();  // from here to the next task: waiting
        __syncthreads();
        // every chunk is claimed: withdraw the list (thieves still finish the chunks they hold)
        if (tid == 0 && sh->published) {
            __hip_atomic_store(&slot->word, 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            atomicSub(a.steal_live, 1u);
        }
    }

    // tallies of the last graph
    if (sh->graph >= 0) flush_acc<DIAG, TB>(acc, a.graphs[sh->graph].acc, sh);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (TB && a.wg_load) {
            a.wg_load[3 * (size_t)blockIdx.x] = ld_start;
            a.wg_load[3 * (size_t)blockIdx.x + 1] = wall_clock64();
            a.wg_load[3 * (size_t)blockIdx.x + 2] = ld_wait;
        }
        __threadfence();
        atomicExch(&a.slot_busy[my_slot], 0u);
    }
}

// ============================================================================ wide roots
//
// Top-level candidates of degree above the widest mask class (64 * 16 bits) are searched by
// wide_kernel: the same method, candidate order, tree and tallies as search_kernel, in a
// simpler form whose sets may be of any width.
//  * Every frame, the top-level list included, maps its mask bits to positions of N(x)
//    through orig[], and masks below the top level are compressed to |R| bits (ceil(|R|/64)
//    words per entry), so the width shrinks with depth.
//  * A node's R' words, the list of its bits and a child's counting-sort histogram live in
//    per-wave global scratch; Q lists are kept whole.
//  * Several workgroups (replicas) rebuild the same top-level list (deterministically) and
//    claim its 64-candidate chunks from a per-candidate counter; replica 0 reports the
//    top-level node itself.

// ids[n] | hs[n] (u64) | masks[n][wf] (u64) | first[rb] | cnt[rb] | H[rb] (u64) | orig[rb] |
// rows[rb][nw] (u64) | skip[2], with wf = ceil(rb / 64), nw = ceil(n / 64); 32-bit words.
// skip[0] (pivot rule only): the number of covered candidates right after the pivot.
__device__ __forceinline__ uint64_t wframe_words(int n, int rb) {
    const uint64_t wf = ((uint64_t)rb + 63u) >> 6, nw = ((uint64_t)n + 63u) >> 6;
    uint64_t o = align2((uint32_t)n);
    o += 2ull * (uint64_t)n;
    o += 2ull * (uint64_t)n * wf;
    o += 4ull * (uint64_t)rb;  // first, cnt, H
    o += (uint64_t)rb;         // orig
    o = (o + 1ull) & ~1ull;
    o += 2ull * (uint64_t)rb * nw;
    o += 2ull;                 // skip
    return o;
}

struct WFrameView {
    const uint32_t *ids;
    const uint64_t *hs;
    const uint64_t *masks;
    uint32_t *first;
    uint32_t *cnt;
    uint64_t *H;
    uint32_t *orig;
    uint64_t *rows;
    uint32_t *skip;
    int nw, wf;
};

__device__ __forceinline__ WFrameView wframe_view(uint32_t *base, int n, int rb) {
    WFrameView v;
    v.wf = (rb + 63) >> 6;
    v.nw = (n + 63) >> 6;
    uint64_t o = align2((uint32_t)n);
    v.ids = base;
    v.hs = reinterpret_cast<const uint64_t *>(base + o);
    o += 2ull * (uint64_t)n;
    v.masks = reinterpret_cast<const uint64_t *>(base + o);
    o += 2ull * (uint64_t)n * (uint64_t)v.wf;
    v.first = base + o;
    o += (uint64_t)rb;
    v.cnt = base + o;
    o += (uint64_t)rb;
    v.H = reinterpret_cast<uint64_t *>(base + o);
    o += 2ull * (uint64_t)rb;
    v.orig = base + o;
    o += (uint64_t)rb;
    o = (o + 1ull) & ~1ull;
    v.rows = reinterpret_cast<uint64_t *>(base + o);
    o += 2ull * (uint64_t)rb * (uint64_t)v.nw;
    v.skip = base + o;
    return v;
}

// The wave's scratch of the wide search.
struct WCtx {
    Ctx c;
    uint32_t *stu2;  // (candidate pruning) a child list's entries while they are regrouped
    uint32_t *bl;    // the bits of R' (frame bit indices), ascending
    uint32_t *hist;  // counting-sort histogram of a child list
    uint64_t *mR;    // R' words (frame bits)
    uint64_t *Rr;    // R' as positions of N(x) (records)
};

// Candidates [base, base + 64) of frame F: lanes with |R'| = 1 are settled (when settle), the
// lanes with |R'| >= 2 are returned.
// IMB: the candidate pruning of section II-C (see heavy_wide); a single-bit candidate whose
// bit is first held by an earlier candidate of the list (a twin, maximal as the first holder)
// left the list with it and is not a node.
// PIV: the pivot rule (see heavy_wide); the candidates the pivot covers, right after it, are
// not taken.
template <bool DIAG, bool ENUM, bool TB, bool IMB = false, bool PIV = false>
__device__ __forceinline__ uint64_t light_wide(const WCtx &w, const FrameState &F, const WFrameView &v, int base,
                                               WaveAcc &acc) {
    const Ctx &c = w.c;
    const int ln = lane_id();
    const int i = base + ln;
    const int nskip = PIV ? (int)uni(*v.skip) : 0;
    const bool act = i < F.n && !(PIV && i > F.nq && i <= F.nq + nskip);
    int r = 0, b = 0;
    if (act)
        for (int q = 0; q < v.wf; ++q) {
            const uint64_t x = v.masks[(size_t)i * v.wf + q];
            if (x) {
                r += __popcll(x);
                b = 64 * q + __ffsll((unsigned long long)x) - 1;
            }
        }
    if (TB && act) acc.dbytes += 8ull * (uint64_t)v.wf;
    if (ENUM) return __ballot(act);
    if (act && r == 1) {
        const bool maximal = v.first[b] == (uint32_t)i;  // no earlier entry holds bit b
        const bool gone = IMB && v.first[b] >= (uint32_t)F.nq && v.first[b] < (uint32_t)i;
        const uint32_t rp = v.orig[b];
        if (maximal) {
            acc.count += 1;
            acc.hash += pair_hash(c.c_is_v, F.sL + v.H[b], c.hvl[rp]);
            acc.out_ints += 2ull + (uint64_t)F.nL + (uint64_t)v.cnt[b] + 1ull;
        }
        if (DIAG && !gone) {
            acc.nodes += 1;
            if (!maximal) acc.nonmax += 1;
            if ((uint32_t)F.level > acc.max_depth) acc.max_depth = (uint32_t)F.level;
            const uint64_t dx = deg_of(c, v.ids[i]);
            const uint64_t rs = 2ull + (uint64_t)c.degl[rp];
            const uint64_t fw = F.fw - (2ull + dx);
            acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + 1ull);
        }
        if (TB) acc.dbytes += 8ull + (maximal ? 24ull : 0ull);
    }
    return __ballot(act && r >= 2);
}

// Add a child entry's compressed mask word q (bits 64q ..) to the child's per-bit tables.
__device__ __forceinline__ void wide_table_add(const WFrameView &v2, int q, uint64_t x, uint32_t slot, uint64_t h) {
    while (x) {
        const int t = 64 * q + __ffsll((unsigned long long)x) - 1;
        x &= x - 1ull;
        atomicMin(&v2.first[t], slot);
        atomicAdd(&v2.cnt[t], 1u);
        atomicAdd(reinterpret_cast<unsigned long long *>(&v2.H[t]), (unsigned long long)h);
    }
}

// The candidate at position i of frame F, |R'| >= 2, handled by the whole wave (maximality
// check, expansion, report, child list).  Returns true when a child frame was written (its
// state in C).
// IMB: the candidate pruning of section II-C.  Candidates of a list are sorted by count, so an
// earlier candidate holding all of a candidate's mask has the same mask (a twin).  When x is
// maximal, its later twins leave the list and join Q with x: a twin whose first twin (the
// earliest) is maximal is never a node, and for the nodes between the two it is a Q entry --
// their child lists take it into Q' instead of P'.  The first twin is maximal exactly when no
// Q entry of the list holds the mask.
// PIV: the pivot pruning of section II-C.  A child list's candidates, sorted by count, are
// regrouped as the pivot p (the first of the largest count), then the candidates whose masks
// lie inside p's (covered: every maximal biclique with one of them holds p), then the rest,
// each group in sorted order; skip[0] of the child frame holds the number covered.  The
// covered ones are never taken: they are candidates for p's node and Q entries (positions
// before) for the nodes after them.
template <bool DIAG, bool ENUM, bool TB, bool IMB = false, bool PIV = false>
__device__ __forceinline__ bool heavy_wide(const WCtx &w, const FrameState &F, const WFrameView &v, int i, FrameState &C,
                                           WaveAcc &acc) {
    const Ctx &c = w.c;
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    const int wf = v.wf;
    // R' (entry i's mask) into the scratch, and its bits in ascending order
    int r = 0;
    for (int q = ln; q < wf; q += 64) {
        const uint64_t x = v.masks[(size_t)i * wf + q];
        w.mR[q] = x;
        r += __popcll(x);
    }
    r = wave_sum_i32(r);
    wait_mem();
    {
        int t0 = 0;
        for (int q = 0; q < wf; ++q) {
            const uint64_t x = uni(w.mR[q]);
            if (!x) continue;
            const bool on = (x >> ln) & 1ull;
            const uint64_t bb = __ballot(on);
            if (on) w.bl[t0 + __popcll(bb & below)] = (uint32_t)(64 * q + ln);
            t0 += __popcll(bb);
        }
        wait_mem();
    }
    if (TB && ln == 0) acc.dbytes += 16ull * (uint64_t)wf + 8ull * (uint64_t)r;

    // maximality: an earlier entry holding all of R' -- a position below i in the AND of R''s
    // rows; a bit of R' first held at i rules that out at once
    bool fh = false;
    for (int t = ln; t < r; t += 64)
        if (v.first[w.bl[t]] == (uint32_t)i) fh = true;
    bool nonmax = false, gone = false;
    if (!__ballot(fh)) {
        const int wl = i >> 6;
        bool inq = false, inp = false;  // (IMB) holders of R' among the Q entries, among earlier candidates
        for (int base = 0; base <= wl && (IMB || !nonmax); base += 64) {
            const int wd = base + ln;
            const bool in = wd <= wl;
            uint64_t a = in ? ~0ull : 0ull;
            int t = 0;
            for (; t < r; ++t) {
                const uint32_t bt = uni(w.bl[t]);
                if (in) a &= v.rows[(size_t)bt * v.nw + wd];
                if ((t & 7) == 7 && !__ballot(a != 0ull)) break;
            }
            if (wd == wl) a &= (1ull << (i & 63)) - 1ull;
            if (__ballot(a != 0ull)) nonmax = true;
            if (IMB) {
                const int q0 = F.nq - 64 * wd;  // positions of word wd below nq
                const uint64_t qm = q0 >= 64 ? ~0ull : (q0 <= 0 ? 0ull : ((1ull << q0) - 1ull));
                inq = inq || (a & qm) != 0ull;
                inp = inp || (a & ~qm) != 0ull;
            }
            if (TB && ln == 0) acc.dbytes += 8ull * (uint64_t)(t < r ? t + 1 : r) * (uint64_t)min(64, wl + 1 - base);
        }
        if (IMB) gone = !__ballot(inq) && __ballot(inp);
    }
    if (gone) return false;  // left the list with its first twin: not a node
    uint64_t dx = 0, rs = 0;
    if (DIAG) {
        dx = deg_of(c, v.ids[i]);
        uint64_t t2 = 0;
        for (int t = ln; t < r; t += 64) t2 += 2ull + (uint64_t)c.degl[v.orig[w.bl[t]]];
        rs = wave_sum_u64(t2);
        if (ln == 0) {
            acc.nodes += 1;
            if ((uint32_t)F.level > acc.max_depth) acc.max_depth = (uint32_t)F.level;
        }
    }
    if (nonmax) {
        if (DIAG && ln == 0) {
            acc.nonmax += 1;
            const uint64_t fw = F.fw - (2ull + dx);
            acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r);
        }
        return false;
    }

    // maximal: per word of positions the OR of R''s rows lists the entries meeting R', the AND
    // those holding all of it (after i; they join L'); the others, Q' before i and P' after,
    // go to stu in list order
    int nu = 0, ne_l = 0, qn_l = 0;
    uint64_t exps = 0;
    {
        const int wi = i >> 6;
        const uint64_t bi = 1ull << (i & 63);
        for (int base = 0; base < v.nw; base += 64) {
            const int wd = base + ln;
            const bool in = wd < v.nw;
            uint64_t u = 0ull, a = in ? ~0ull : 0ull;
            for (int t = 0; t < r; ++t) {
                const uint32_t bt = uni(w.bl[t]);
                if (in) {
                    const uint64_t x = v.rows[(size_t)bt * v.nw + wd];
                    u |= x;
                    a &= x;
                }
            }
            if (wd == wi) {
                u &= ~bi;
                a &= ~bi;
            }
            ne_l += __popcll(a);
            for (uint64_t f = a; f;) {
                const int b = __ffsll((unsigned long long)f) - 1;
                f &= f - 1ull;
                exps += v.hs[64 * wd + b];
            }
            uint64_t qp = u & ~a;
            qn_l += __popcll(qp & (wd < wi ? ~0ull : (wd == wi ? bi - 1ull : 0ull)));
            const int pc = __popcll(qp);
            const int incl = wave_incl_scan(pc);
            int at = nu + incl - pc;
            while (qp) {
                const int b = __ffsll((unsigned long long)qp) - 1;
                qp &= qp - 1ull;
                c.stu[at++] = (uint32_t)(64 * wd + b);
            }
            nu += last_lane(incl);
        }
    }
    int qn = wave_sum_i32(qn_l);
    const int ne = wave_sum_i32(ne_l);
    wait_mem();  // stu is read by other lanes below
    if (IMB) {
        // entries after i that left the list with an earlier twin (of the same count as i, a
        // twin before i, none of the Q entries holding their mask) are Q entries for i: they go
        // to Q' (stu becomes Q' | the moved ones | the rest of P', each in list order)
        const int wl = i >> 6;
        int nmv = 0;
        for (int base = qn; base < nu; base += 64) {
            const int j = base + ln;
            bool mv = false;
            uint32_t k = 0;
            if (j < nu) {
                k = c.stu[j];
                int cnt = 0;
                for (int q = 0; q < wf; ++q) cnt += __popcll(v.masks[(size_t)k * wf + q]);
                if (cnt == r) {
                    bool inq = false, inp = false;
                    for (int wd = 0; wd <= wl; ++wd) {
                        uint64_t a = ~0ull;
                        for (int q = 0; q < wf && a; ++q) {
                            uint64_t x = v.masks[(size_t)k * wf + q];
                            while (x && a) {
                                const int bt = 64 * q + __ffsll((unsigned long long)x) - 1;
                                x &= x - 1ull;
                                a &= v.rows[(size_t)bt * v.nw + wd];
                            }
                        }
                        if (wd == wl) a &= (1ull << (i & 63)) - 1ull;
                        const int q0 = F.nq - 64 * wd;
                        const uint64_t qm = q0 >= 64 ? ~0ull : (q0 <= 0 ? 0ull : ((1ull << q0) - 1ull));
                        inq = inq || (a & qm) != 0ull;
                        inp = inp || (a & ~qm) != 0ull;
                    }
                    mv = inp && !inq;
                }
                c.stu[j] = k | (mv ? 0x80000000u : 0u);  // (positions are below 2^31)
            }
            nmv += __popcll(__ballot(mv));
        }
        if (nmv > 0) {
            wait_mem();
            // stable partition of stu[qn, nu) into the moved entries, then the others
            int am = qn, ak = qn + nmv;
            for (int base = qn; base < nu; base += 64) {
                const int j = base + ln;
                const uint32_t e = j < nu ? c.stu[j] : 0u;
                const bool act = j < nu;
                const bool mv = act && (e & 0x80000000u);
                const uint64_t bm = __ballot(mv), bk = __ballot(act && !mv);
                if (mv) w.stu2[am - qn + __popcll(bm & below)] = e & 0x7FFFFFFFu;
                if (act && !mv) w.stu2[ak - qn + __popcll(bk & below)] = e;
                am += __popcll(bm);
                ak += __popcll(bk);
            }
            wait_mem();
            for (int j = qn + ln; j < nu; j += 64) c.stu[j] = w.stu2[j - qn];
            wait_mem();
            qn += nmv;
        } else {
            for (int j = qn + ln; j < nu; j += 64) c.stu[j] &= 0x7FFFFFFFu;
            wait_mem();
        }
    }
    const int pn = nu - qn;
    // histogram of the P' counts |mask n R'|
    for (int b = ln; b <= r; b += 64) w.hist[b] = 0u;
    wait_mem();
    uint64_t fwc = 0;
    int cmax = 0;  // (PIV) the largest count
    for (int base = 0; base < nu; base += 64) {
        const int j = base + ln;
        if (j < nu) {
            const int k = (int)c.stu[j];
            if (j >= qn) {
                int cnt = 0;
                for (int q = 0; q < wf; ++q) {
                    const uint64_t mq = w.mR[q];
                    if (mq) cnt += __popcll(v.masks[(size_t)k * wf + q] & mq);
                }
                atomicAdd(&w.hist[cnt], 1u);
                if (PIV) cmax = cnt > cmax ? cnt : cmax;
            }
            if (DIAG) fwc += 2ull + deg_of(c, v.ids[k]);
        }
    }
    see_atomics();  // the histogram was built with atomics
    if (TB && ln == 0)
        acc.dbytes += 8ull * (uint64_t)r * (uint64_t)v.nw + 8ull * (uint64_t)ne + 8ull * (uint64_t)nu +
                      (uint64_t)pn * 8ull * (uint64_t)wf + 16ull * (uint64_t)r;

    // report (L', R')
    const uint64_t sL = F.sL + v.hs[i] + wave_sum_u64(exps);
    uint64_t sr = 0;
    for (int t = ln; t < r; t += 64) sr += c.hvl[v.orig[w.bl[t]]];
    sr = wave_sum_u64(sr);
    const int nL = F.nL + 1 + ne;
    if (ln == 0) {
        acc.count += 1;
        acc.hash += pair_hash(c.c_is_v, sL, sr);
        acc.out_ints += 2ull + (uint64_t)nL + (uint64_t)r;
    }
    if (ENUM) {
        for (int q = ln; q < c.Wroot; q += 64) w.Rr[q] = 0ull;
        wait_mem();
        for (int t = ln; t < r; t += 64) {
            const uint32_t rp = v.orig[w.bl[t]];
            atomicOr(reinterpret_cast<unsigned long long *>(&w.Rr[rp >> 6]), 1ull << (rp & 63));
        }
        see_atomics();
        write_record(c, w.Rr, nL, r);
    }
    if (DIAG && ln == 0) {
        const uint64_t fw = F.fw - (2ull + dx);
        acc.bytes += 4ull * ((2ull + dx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r + (uint64_t)pn +
                             (uint64_t)qn);
    }
    if (pn == 0) return false;

    // child list: Q' in list order, then P' stably sorted by count; masks compressed to the r
    // bits of R' (child bit t = frame bit bl[t]), mapped to N(x) through orig
    const int n2 = nu, wf2 = (r + 63) >> 6;
    const uint32_t off2 = F.top;
    const uint64_t top2 = ((uint64_t)off2 + wframe_words(n2, r) + 1ull) & ~1ull;
    if ((int64_t)top2 > c.scap) {
        if (ln == 0) atomicOr(c.flags, (unsigned int)FLAG_STACK_OVERFLOW);
        return false;
    }
    uint32_t *cb = c.stk + off2;
    const WFrameView v2 = wframe_view(cb, n2, r);
    uint32_t *ids2 = cb;
    uint64_t *hs2 = const_cast<uint64_t *>(v2.hs);
    uint64_t *masks2 = const_cast<uint64_t *>(v2.masks);
    int carry = qn;
    for (int base = 0; base <= r; base += 64) {
        const int b = base + ln;
        const int h = b <= r ? (int)w.hist[b] : 0;
        const int incl = wave_incl_scan(h);
        if (b <= r) w.hist[b] = (uint32_t)(carry + incl - h);
        carry += last_lane(incl);
    }
    for (int t = ln; t < r; t += 64) {
        v2.orig[t] = v.orig[w.bl[t]];
        v2.first[t] = kNone;
        v2.cnt[t] = 0u;
        v2.H[t] = 0ull;
    }
    wait_mem();
    const int nbits = r <= 1 ? 1 : 32 - __clz(r - 1);
    if (PIV) {
        // the P' entries in sorted order into stu2 (the placement the plain build makes), then
        // regrouped into stu[qn, nu): the pivot, the entries it covers, the others
        const int cm = __builtin_amdgcn_readfirstlane(wave_max_u32((uint32_t)cmax));
        const int pslot = (int)uni(w.hist[cm]) - qn;  // the first slot of the largest count
        wait_mem();
        for (int base = qn; base < nu; base += 64) {
            const int j = base + ln;
            const bool inp = j < nu;
            const int k = inp ? (int)c.stu[j] : 0;
            int cnt = 0;
            if (inp)
                for (int q = 0; q < wf; ++q) {
                    const uint64_t mq = w.mR[q];
                    if (mq) cnt += __popcll(v.masks[(size_t)k * wf + q] & mq);
                }
            uint64_t same = __ballot(inp);
            for (int bit = 0; bit < nbits; ++bit) {
                const bool on = (cnt >> bit) & 1;
                const uint64_t bb = __ballot(inp && on);
                same &= on ? bb : ~bb;
            }
            uint32_t start = 0;
            if (inp) start = w.hist[cnt];
            if (inp) {
                w.stu2[start + (uint32_t)__popcll(same & below) - (uint32_t)qn] = (uint32_t)k;
                if ((same >> ln) == 1ull) w.hist[cnt] = start + (uint32_t)__popcll(same);
            }
            see_atomics();  // (the next round reads the updated histogram entries; stu2 after)
        }
        const int kp = (int)uni(w.stu2[pslot]);
        int ncov = 0;
        for (int base = 0; base < pn; base += 64) {
            const int t = base + ln;
            bool cov = false;
            if (t < pn && t != pslot) {
                const int k = (int)w.stu2[t];
                cov = true;
                for (int q = 0; q < wf && cov; ++q) {
                    const uint64_t mq = w.mR[q];
                    if (mq) cov = ((v.masks[(size_t)k * wf + q] & mq) & ~v.masks[(size_t)kp * wf + q]) == 0ull;
                }
            }
            if (t < pn) w.stu2[t] |= cov ? 0x80000000u : 0u;  // (positions are below 2^31)
            ncov += __popcll(__ballot(cov));
        }
        wait_mem();
        int ac = qn + 1, ao = qn + 1 + ncov;
        if (ln == 0) c.stu[qn] = (uint32_t)kp;
        for (int base = 0; base < pn; base += 64) {
            const int t = base + ln;
            const bool act = t < pn && t != pslot;
            const uint32_t e = t < pn ? w.stu2[t] : 0u;
            const bool cov = act && (e & 0x80000000u);
            const uint64_t bc = __ballot(cov), bo = __ballot(act && !cov);
            if (cov) c.stu[ac + __popcll(bc & below)] = e & 0x7FFFFFFFu;
            if (act && !cov) c.stu[ao + __popcll(bo & below)] = e;
            ac += __popcll(bc);
            ao += __popcll(bo);
        }
        if (ln == 0) *v2.skip = (uint32_t)ncov;
        wait_mem();
    }
    for (int base = 0; base < nu; base += 64) {
        const int j = base + ln;
        const bool act = j < nu;
        const int k = act ? (int)c.stu[j] : 0;
        const bool inp = !PIV && act && j >= qn;  // (PIV: stu is in its final order)
        int cnt = 0;
        if (inp)
            for (int q = 0; q < wf; ++q) {
                const uint64_t mq = w.mR[q];
                if (mq) cnt += __popcll(v.masks[(size_t)k * wf + q] & mq);
            }
        uint32_t slot = (uint32_t)j;  // Q' entries keep their list order
        if (__ballot(inp)) {
            // stable placement among equal counts: lanes with the same count, in lane order
            uint64_t same = __ballot(inp);
            for (int bit = 0; bit < nbits; ++bit) {
                const bool on = (cnt >> bit) & 1;
                const uint64_t bb = __ballot(inp && on);
                same &= on ? bb : ~bb;
            }
            uint32_t start = 0;
            if (inp) start = w.hist[cnt];
            if (inp) {
                slot = start + (uint32_t)__popcll(same & below);
                if ((same >> ln) == 1ull) w.hist[cnt] = start + (uint32_t)__popcll(same);
            }
            see_atomics();  // (the next round reads the updated histogram entries)
        }
        if (act) {
            ids2[slot] = v.ids[k];
            const uint64_t h = v.hs[k];
            hs2[slot] = h;
            uint64_t ow = 0;
            int t = 0;
            for (int q = 0; q < wf; ++q) {
                uint64_t mq = w.mR[q];
                if (!mq) continue;
                const uint64_t x = v.masks[(size_t)k * wf + q];
                while (mq) {
                    const int p = __ffsll((unsigned long long)mq) - 1;
                    mq &= mq - 1ull;
                    ow |= ((x >> p) & 1ull) << (t & 63);
                    ++t;
                    if ((t & 63) == 0) {
                        masks2[(size_t)slot * wf2 + ((t >> 6) - 1)] = ow;
                        wide_table_add(v2, (t >> 6) - 1, ow, slot, h);
                        ow = 0ull;
                    }
                }
            }
            if (t & 63) {
                masks2[(size_t)slot * wf2 + (t >> 6)] = ow;
                wide_table_add(v2, t >> 6, ow, slot, h);
            }
        }
    }
    see_atomics();
    // position rows: one 64-entry block of one mask word per transpose
    for (int q = 0; q < wf2; ++q)
        for (int blk = 0; blk < v2.nw; ++blk) {
            const int e = 64 * blk + ln;
            const uint64_t t = wave_transpose64(e < n2 ? masks2[(size_t)e * wf2 + q] : 0ull);
            if (64 * q + ln < r) v2.rows[(size_t)(64 * q + ln) * v2.nw + blk] = t;
        }
    wait_mem();
    if (TB && ln == 0)
        acc.dbytes += (uint64_t)n2 * (4ull + 16ull + 8ull * (uint64_t)wf2 + 8ull * (uint64_t)wf) + 32ull * (uint64_t)r +
                      16ull * (uint64_t)r * (uint64_t)n2 / 64ull + 8ull * (uint64_t)r * (uint64_t)v2.nw;
    C.off = off2;
    C.top = (uint32_t)top2;
    C.n = n2;
    C.nq = qn;
    C.level = F.level + 1;
    C.nL = nL;
    C.wf = wf2;
    C.narrow = 1;
    C.chunk = qn - 64;
    C.rbits = r;
    C.heavy = 0ull;
    C.sL = sL;
    C.fw = DIAG ? wave_sum_u64(fwc) : 0ull;
    return true;
}

// Stable counting sort by key, as wave_sort_by_key, with the histogram in global memory.
template <typename Put>
__device__ __forceinline__ void wave_sort_by_key_g(const uint32_t *src, const uint32_t *key_of, int n, int nbins,
                                                   uint32_t *hist, Put put) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    for (int b = ln; b < nbins; b += 64) hist[b] = 0u;
    wait_mem();
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        if (j < n) atomicAdd(&hist[key_of[j]], 1u);
    }
    see_atomics();
    int carry = 0;
    for (int base = 0; base < nbins; base += 64) {
        const int b = base + ln;
        const int h = b < nbins ? (int)hist[b] : 0;
        const int incl = wave_incl_scan(h);
        if (b < nbins) hist[b] = (uint32_t)(carry + incl - h);
        carry += last_lane(incl);
    }
    wait_mem();
    const int nbits = nbins <= 1 ? 1 : 32 - __clz(nbins - 1);
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        const bool act = j < n;
        const uint32_t key = act ? key_of[j] : 0u;
        const uint32_t p = act ? src[j] : 0u;
        uint64_t same = __ballot(act);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (key >> bit) & 1u;
            const uint64_t bb = __ballot(act && on);
            same &= on ? bb : ~bb;
        }
        uint32_t start = 0;
        if (act) start = hist[key];
        if (act) {
            put(start + (uint32_t)__popcll(same & below), p);
            if ((same >> ln) == 1ull) hist[key] = start + (uint32_t)__popcll(same);
        }
        see_atomics();  // (the next round reads the updated histogram entries)
    }
}

// IMB: with the candidate pruning of section II-C (every top-level candidate is searched here
// then): see heavy_wide; at the top level a candidate's twins are the candidates with its exact
// row (a.twin), every first twin is maximal (no earlier candidate can hold its row), and the
// later twins are never nodes.
template <bool DIAG, bool ENUM, bool TB, bool IMB = false, bool PIV = false>
__global__ __launch_bounds__(512) void wide_kernel(SearchArgs a, int64_t lo, int64_t hi, unsigned int *counter) {
    extern __shared__ unsigned char lds_raw[];
    WGShared *sh = reinterpret_cast<WGShared *>(lds_raw);
    const int tid = threadIdx.x, nt = blockDim.x, wid = uni(tid >> 6), nw = nt >> 6, ln = lane_id();
    const WideLayout &L = a.wl;
    const int Wx = L.Wx;
    char *wg = a.warena + (size_t)blockIdx.x * L.wg_bytes;
    uint64_t *bitmap = reinterpret_cast<uint64_t *>(wg + L.off_bitmap);
    uint32_t *bpre = reinterpret_cast<uint32_t *>(wg + L.off_bpre);
    uint64_t *M = reinterpret_cast<uint64_t *>(wg + L.off_M);
    int32_t *gid = reinterpret_cast<int32_t *>(wg + L.off_gid);
    uint32_t *cnt1 = reinterpret_cast<uint32_t *>(wg + L.off_cnt);
    uint64_t *hvl = reinterpret_cast<uint64_t *>(wg + L.off_hv);
    uint32_t *degl = reinterpret_cast<uint32_t *>(wg + L.off_deg);
    uint32_t *t1v = reinterpret_cast<uint32_t *>(wg + L.off_t1v);
    uint32_t *t1c = reinterpret_cast<uint32_t *>(wg + L.off_t1c);
    uint32_t *whist = reinterpret_cast<uint32_t *>(wg + L.off_whist);
    uint32_t *s1 = reinterpret_cast<uint32_t *>(wg + L.off_S1);
    char *wv = wg + L.off_waves + (size_t)wid * L.wave_bytes;
    FrameState *hdr = reinterpret_cast<FrameState *>(wv + L.off_w_hdr);

    WCtx w;
    Ctx &c = w.c;
    c.gid = gid;
    c.M = M;
    c.hvl = hvl;
    c.degl = degl;
    c.c_off = a.c_off;
    c.s1 = s1;
    c.stk = reinterpret_cast<uint32_t *>(wv + L.off_w_stack);
    c.stu = reinterpret_cast<uint32_t *>(wv + L.off_w_u);
    c.scap = L.scap;
    c.c_is_v = 0;
    c.cbase = 0;
    c.obase = 0;
    c.Wroot = Wx;
    c.rec = a.rec;
    c.rec_cap = a.rec_cap;
    c.rec_offs = a.rec_offs;
    c.rec_offs_cap = a.rec_offs_cap;
    c.acc = a.acc;
    c.flags = a.flags;
    w.stu2 = reinterpret_cast<uint32_t *>(wv + L.off_w_u2);
    w.bl = reinterpret_cast<uint32_t *>(wv + L.off_w_bl);
    w.hist = reinterpret_cast<uint32_t *>(wv + L.off_w_hist);
    w.mR = reinterpret_cast<uint64_t *>(wv + L.off_w_mr);
    w.Rr = reinterpret_cast<uint64_t *>(wv + L.off_w_rr);

    WaveAcc acc{};
    const uint64_t ld_start = TB ? wall_clock64() : 0ull;
    const int ucap = a.dims.ucap;
    const int64_t nroots = hi - lo;
    const int64_t ntasks = nroots * (int64_t)L.reps;
    if (tid < 16) sh->red[tid] = 0ull;
    if (tid == 0) sh->graph = -1;
    __syncthreads();

    for (;;) {
        if (tid == 0) {
            const unsigned int f = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long t = (f & FLAG_RERUN) ? ~0ull : (unsigned long long)atomicAdd(counter, 1u);
            while (t != ~0ull && (int64_t)t < ntasks && root_cancelled(a, lo + (int64_t)t % nroots))
                t = (unsigned long long)atomicAdd(counter, 1u);
            sh->task = t;
        }
        __syncthreads();
        const unsigned long long tt = sh->task;
        if (tt == ~0ull || (int64_t)tt >= ntasks) break;
        const int64_t ri = (int64_t)tt % nroots;   // top-level candidates of largest degree first
        const bool owner = (int64_t)tt < nroots;   // replica 0 reports the top-level node
        int g = 0;
        int64_t k;
        if (a.tasks) {
            const unsigned long long tk = a.tasks[lo + ri];
            g = (int)(tk >> 32);
            k = (int64_t)(tk & 0xFFFFFFFFull);
        } else {
            k = hi - 1 - ri;
        }
        if (g != sh->graph) {
            if (sh->graph >= 0) flush_acc<DIAG, TB>(acc, a.graphs[sh->graph].acc, sh);
            __syncthreads();
            if (tid == 0) sh->graph = g;
            __syncthreads();
        }
        const GraphDesc gd = a.graphs[g];
        c.c_is_v = gd.c_is_v;
        c.cbase = gd.cbase;
        c.obase = gd.obase;
        const int nwords = gd.nwords;
        const int32_t x = gd.order[k];
        const int32_t rbx = a.c_off[x];
        const int32_t d = a.c_off[x + 1] - rbx;
        const int32_t *row = a.c_adj + rbx;
        c.row = row;
        c.x_root = x;
        const int wd = (d + 63) >> 6;

        // -- reverse scan 1: mark the ranks of all 2-hop neighbours of x
        for (int j = wid; j < d; j += nw) {
            const int32_t wv2 = row[j];
            const int32_t e0 = a.o_off[wv2], e1 = a.o_off[wv2 + 1];
            for (int p = e0 + ln; p < e1; p += 64) {
                const int32_t v = a.o_adj[p];
                if (v != x) {
                    const int32_t rk = a.rank[v];
                    atomicOr(reinterpret_cast<unsigned long long *>(&bitmap[rk >> 6]), 1ull << (rk & 63));
                }
            }
        }
        uint64_t hv_local = 0, rs_local = 0;
        for (int j = tid; j < d; j += nt) {
            const int32_t wv2 = row[j];
            const uint64_t h = hr(c, wv2);
            hvl[j] = h;
            hv_local += h;
            const uint32_t dw = (uint32_t)(a.o_off[wv2 + 1] - a.o_off[wv2]);
            degl[j] = dw;
            rs_local += 2ull + dw;
        }
        if (tid == 0) {
            sh->nonmax = 0;
            sh->pcount = 0;
            sh->exps = 0;
            sh->fw1 = 0;
            sh->hvsum = 0;
            sh->rs1 = 0;
            sh->nexp = 0;
        }
        __syncthreads();
        see_atomics();
        hv_local = wave_sum_u64(hv_local);
        rs_local = wave_sum_u64(rs_local);
        if (ln == 0) {
            lds_add(&sh->hvsum, hv_local);
            lds_add(&sh->rs1, rs_local);
        }
        block_popcount_prefix(bitmap, bpre, nwords, sh);
        const int s0 = uni(sh->s0);
        if (s0 > ucap) {
            for (int q = tid; q < nwords; q += nt) bitmap[q] = 0ull;
            if (tid == 0) {
                atomicOr(a.flags, (unsigned int)FLAG_UNIVERSE_OVERFLOW);
                atomicMax(&a.acc[ACC_NEED_UCAP], (unsigned long long)s0);
            }
            __syncthreads();
            continue;
        }
        const int nq0 = (int)bpre[k >> 6] + __popcll(bitmap[k >> 6] & ((1ull << (k & 63)) - 1ull));
        c.s0 = s0;
        for (int q = tid; q < nwords; q += nt) {
            uint64_t bits = bitmap[q];
            uint32_t pos = bpre[q];
            while (bits) {
                const int b = __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1ull;
                gid[pos++] = gd.order[q * 64 + b];
            }
        }
        for (size_t q = tid; q < (size_t)s0 * Wx; q += nt) M[q] = 0ull;
        wait_mem();
        __syncthreads();
        // -- reverse scan 2: M[v] gets bit j for every w_j in N(x) adjacent to v
        for (int j = wid; j < d; j += nw) {
            const int32_t wv2 = row[j];
            const int32_t e0 = a.o_off[wv2], e1 = a.o_off[wv2 + 1];
            for (int p = e0 + ln; p < e1; p += 64) {
                const int32_t v = a.o_adj[p];
                if (v != x) {
                    const int32_t rk = a.rank[v];
                    const uint32_t li =
                        bpre[rk >> 6] + (uint32_t)__popcll(bitmap[rk >> 6] & ((1ull << (rk & 63)) - 1ull));
                    atomicOr(reinterpret_cast<unsigned long long *>(&M[(size_t)li * Wx + (j >> 6)]), 1ull << (j & 63));
                }
            }
        }
        __syncthreads();
        see_atomics();
        for (int q = tid; q < nwords; q += nt) bitmap[q] = 0ull;
        // -- the top-level node for x: counts, maximality against earlier ranks, expansion
        {
            bool nm = false;
            int pc = 0, nexp = 0;
            uint64_t ex = 0, fw = 0;
            for (int li = tid; li < s0; li += nt) {
                int cc = 0;
                for (int q = 0; q < wd; ++q) cc += __popcll(M[(size_t)li * Wx + q]);
                cnt1[li] = (uint32_t)cc;
                const int32_t gv = gid[li];
                const uint64_t dg = DIAG ? 2ull + (uint64_t)(a.c_off[gv + 1] - a.c_off[gv]) : 0ull;
                if (li < nq0) {
                    if (cc == d) nm = true;
                    else fw += dg;
                } else if (cc == d) {
                    ex += hl(c, gv);
                    ++nexp;
                } else {
                    ++pc;
                    fw += dg;
                }
            }
            if (__ballot(nm) && ln == 0) atomicOr(&sh->nonmax, 1);
            ex = wave_sum_u64(ex);
            fw = wave_sum_u64(fw);
            pc = wave_sum_i32(pc);
            nexp = wave_sum_i32(nexp);
            if (ln == 0) {
                atomicAdd(&sh->pcount, pc);
                atomicAdd(&sh->nexp, nexp);
                lds_add(&sh->exps, ex);
                lds_add(&sh->fw1, fw);
            }
        }
        wait_mem();
        __syncthreads();
        const bool root_nonmax = uni(sh->nonmax) != 0;
        const int P1 = uni(sh->pcount);
        if (tid == 0 && owner) {
            const uint64_t dx = (uint64_t)d;
            // (IMB: a top-level candidate with an earlier twin is exactly a non-maximal one,
            // and it left the list with its first twin: not a node)
            if (DIAG && !(IMB && root_nonmax)) {
                acc.nodes += 1;
                if (acc.max_depth < 1) acc.max_depth = 1;
                const uint64_t fwtop = gd.total_fw - (2ull + dx);
                const uint64_t rs = sh->rs1;
                uint64_t b = (2ull + dx) + (rs < fwtop ? rs : fwtop) + (uint64_t)(gd.ncand - 1) + dx;
                if (root_nonmax) acc.nonmax += 1;
                else b += (uint64_t)P1 + (uint64_t)nq0;
                acc.bytes += 4ull * b;
            }
            if (TB) {
                const uint64_t wk = (uint64_t)sh->rs1 - 2ull * dx, su = (uint64_t)s0;
                acc.dbytes += 4ull * (dx + 2ull) + 16ull * dx + 44ull * wk + 12ull * dx + 32ull * (uint64_t)nwords +
                              8ull * su + 16ull * (uint64_t)wd * su + 8ull * su;
            }
            if (!root_nonmax) {
                acc.count += 1;
                acc.hash += pair_hash(c.c_is_v, hl(c, x) + sh->exps, sh->hvsum);
                acc.out_ints += 2ull + (uint64_t)(1 + sh->nexp) + (uint64_t)d;
            }
        }
        if (ENUM && !root_nonmax && owner && wid == 0) {
            for (int q = ln; q < Wx; q += 64) {
                const int bits = d - 64 * q;
                w.Rr[q] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : ((1ull << bits) - 1ull));
            }
            wait_mem();
            write_record(c, w.Rr, 1 + sh->nexp, d);
        }
        if (root_nonmax || P1 == 0) {
            __syncthreads();
            continue;
        }
        // -- the top-level list as a frame: Q1 (earlier ranks) ++ P1 stably sorted by count,
        //    masks over the positions of N(x), per-bit tables, rows
        const int n1 = nq0 + P1;
        const WFrameView v1 = wframe_view(s1, n1, d);
        uint32_t *ids1 = s1;
        for (int li = tid; li < nq0; li += nt) ids1[li] = (uint32_t)li;
        if (wid == 0) {
            // (IMB) candidates ranked after x with a twin ranked before x left the list with it:
            // they join Q1, after the earlier ranks, in rank order
            int pn = 0, nmv = 0;
            for (int base = nq0; base < s0; base += 64) {
                const int li = base + ln;
                const bool act2 = li < s0;
                const uint32_t cc = act2 ? cnt1[li] : 0u;
                const bool cand = act2 && (int)cc < d;
                const bool mv = IMB && cand && a.twin[gid[li]] < (int32_t)k;
                const bool pk = cand && !mv;
                const uint64_t pb = __ballot(pk), mb = __ballot(mv);
                if (pk) {
                    const int p = pn + __popcll(pb & lanes_below());
                    t1v[p] = (uint32_t)li;
                    t1c[p] = cc;
                }
                if (mv) ids1[nq0 + nmv + __popcll(mb & lanes_below())] = (uint32_t)li;
                pn += __popcll(pb);
                nmv += __popcll(mb);
            }
            if (ln == 0) sh->pcount = pn;  // the candidates left in the list
            wait_mem();
            const int q1 = nq0 + nmv;
            wave_sort_by_key_g(t1v, t1c, pn, d, whist, [&](uint32_t slot, uint32_t li) { ids1[q1 + slot] = li; });
            if (PIV) {
                // (PIV) regrouped: the pivot (the first of the largest count), the candidates
                // whose masks lie inside its mask, the others; t1v is free after the sort
                wait_mem();
                const uint32_t cm = cnt1[uni(ids1[q1 + pn - 1])];
                int nmax = 0;
                for (int base = 0; base < pn; base += 64) {
                    const int t = base + ln;
                    nmax += __popcll(__ballot(t < pn && cnt1[ids1[q1 + t]] == cm));
                }
                const int pslot = pn - nmax;
                const uint32_t lp = uni(ids1[q1 + pslot]);
                int ncov = 0;
                for (int base = 0; base < pn; base += 64) {
                    const int t = base + ln;
                    bool cov = false;
                    uint32_t li = 0;
                    if (t < pn) li = ids1[q1 + t];
                    if (t < pn && t != pslot) {
                        cov = true;
                        for (int q = 0; q < wd && cov; ++q)
                            cov = (M[(size_t)li * Wx + q] & ~M[(size_t)lp * Wx + q]) == 0ull;
                    }
                    if (t < pn) t1v[t] = li | (cov ? 0x80000000u : 0u);  // (indices are below 2^31)
                    ncov += __popcll(__ballot(cov));
                }
                wait_mem();
                int ac = 1, ao = 1 + ncov;
                if (ln == 0) ids1[q1] = lp;
                for (int base = 0; base < pn; base += 64) {
                    const int t = base + ln;
                    const bool act = t < pn && t != pslot;
                    const uint32_t e = t < pn ? t1v[t] : 0u;
                    const bool cov = act && (e & 0x80000000u);
                    const uint64_t bc = __ballot(cov), bo = __ballot(act && !cov);
                    if (cov) ids1[q1 + ac + __popcll(bc & lanes_below())] = e & 0x7FFFFFFFu;
                    if (act && !cov) ids1[q1 + ao + __popcll(bo & lanes_below())] = e;
                    ac += __popcll(bc);
                    ao += __popcll(bo);
                }
                if (ln == 0) *v1.skip = (uint32_t)ncov;
                wait_mem();
            }
        }
        for (int b = tid; b < d; b += nt) {
            v1.first[b] = kNone;
            v1.cnt[b] = 0u;
            v1.H[b] = 0ull;
            v1.orig[b] = (uint32_t)b;
        }
        wait_mem();
        __syncthreads();
        uint64_t *masks1 = const_cast<uint64_t *>(v1.masks);
        uint64_t *hs1 = const_cast<uint64_t *>(v1.hs);
        for (int j = tid; j < n1; j += nt) {
            const uint32_t li = ids1[j];
            const uint64_t h = hl(c, gid[li]);
            hs1[j] = h;
            for (int q = 0; q < wd; ++q) {
                uint64_t mm = M[(size_t)li * Wx + q];
                masks1[(size_t)j * wd + q] = mm;
                while (mm) {
                    const int b = 64 * q + __ffsll((unsigned long long)mm) - 1;
                    mm &= mm - 1ull;
                    atomicMin(&v1.first[b], (uint32_t)j);
                    atomicAdd(&v1.cnt[b], 1u);
                    atomicAdd(reinterpret_cast<unsigned long long *>(&v1.H[b]), (unsigned long long)h);
                }
            }
        }
        __syncthreads();
        see_atomics();
        for (int job = wid; job < v1.nw * wd; job += nw) {
            const int blk = job / wd, q = job - blk * wd;
            const int e = 64 * blk + ln;
            const uint64_t t = wave_transpose64(e < n1 ? masks1[(size_t)e * wd + q] : 0ull);
            if (64 * q + ln < d) v1.rows[(size_t)(64 * q + ln) * v1.nw + blk] = t;
        }
        wait_mem();
        __syncthreads();
        if (TB && tid == 0 && owner)
            acc.dbytes += 4ull * (uint64_t)nq0 + 4ull * (uint64_t)(s0 - nq0) + 20ull * (uint64_t)P1 +
                          (uint64_t)n1 * (24ull + 16ull * (uint64_t)wd) + 32ull * (uint64_t)d +
                          8ull * (uint64_t)n1 * (uint64_t)wd + 8ull * (uint64_t)d * (uint64_t)v1.nw;

        const int P1c = IMB ? uni(sh->pcount) : P1;  // candidates of the list
        FrameState top;
        top.off = kShared;
        top.top = 0;
        top.n = n1;
        top.nq = n1 - P1c;
        top.level = 2;
        top.nL = 1 + uni(sh->nexp);
        top.wf = wd;
        top.narrow = 1;
        top.chunk = 0;
        top.rbits = d;
        top.heavy = 0ull;
        top.sL = hl(c, x) + uni((uint64_t)sh->exps);
        top.fw = uni((uint64_t)sh->fw1);
        const int nch = (P1c + 63) >> 6;

        // -- chunks of the top-level list, claimed by every wave of every replica; each wave
        //    searches depth-first below the candidates of its chunk
        bool aborted = false;
        for (;;) {
            int q = 0;
            if (ln == 0) q = (int)atomicAdd(&a.wide_items[ri], 1u);
            q = __builtin_amdgcn_readlane(q, 0);
            if (q >= nch) break;
            if (uni(__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & FLAG_RERUN) break;
            FrameState cur = top;
            cur.chunk = top.nq + 64 * q;
            cur.heavy = light_wide<DIAG, ENUM, TB, IMB, PIV>(w, cur, v1, cur.chunk, acc);
            int depth = 0;
            while (!aborted) {
                const WFrameView v = wframe_view(frame_base(c, cur.off), cur.n, cur.rbits);
                if (cur.heavy == 0ull) {
                    if (depth == 0) break;  // the chunk is done
                    const int base = cur.chunk + 64;
                    if (base >= cur.n) {
                        --depth;
                        cur = uni_frame(hdr[depth]);
                        continue;
                    }
                    cur.chunk = base;
                    cur.heavy = light_wide<DIAG, ENUM, TB, IMB, PIV>(w, cur, v, base, acc);
                    continue;
                }
                const int lane = __ffsll((unsigned long long)cur.heavy) - 1;
                cur.heavy &= cur.heavy - 1ull;
                FrameState ch;
                if (heavy_wide<DIAG, ENUM, TB, IMB, PIV>(w, cur, v, cur.chunk + lane, ch, acc)) {
                    if (depth + 1 >= L.maxdepth) {
                        if (ln == 0) atomicOr(a.flags, (unsigned int)FLAG_DEPTH_OVERFLOW);
                        aborted = true;
                        break;
                    }
                    hdr[depth] = cur;  // every lane stores the same header
                    wait_mem();
                    if (TB && ln == 0) acc.dbytes += 2ull * sizeof(FrameState);
                    ++depth;
                    cur = ch;
                } else if (__hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_STACK_OVERFLOW) {
                    aborted = true;
                }
            }
            if (aborted) break;
        }
        __syncthreads();
    }
    if (sh->graph >= 0) flush_acc<DIAG, TB>(acc, a.graphs[sh->graph].acc, sh);
    if (TB && a.wg_load && tid == 0) {
        a.wg_load[3 * (size_t)blockIdx.x] = ld_start;
        a.wg_load[3 * (size_t)blockIdx.x + 1] = wall_clock64();
        a.wg_load[3 * (size_t)blockIdx.x + 2] = 0ull;  // replicas take chunks without waiting
    }
}

size_t lds_bytes(int W, int waves, int nwords) {
    return sizeof(WGShared) + hist_region_bytes(64 * W, waves) + (size_t)waves * kWaveLds + rank_lds_bytes(nwords);
}

template <int W>
hipError_t launch_w(const SearchArgs &a, bool diag, bool enumerate, bool tb, int64_t lo, int64_t hi, unsigned int *counter,
                    int grid, int waves, hipStream_t s) {
    dim3 g(grid), b(64 * waves);
    const size_t lds = lds_bytes(W, waves, a.dims.nwords);
    if (tb && !diag && !enumerate)
        hipLaunchKernelGGL((search_kernel<W, false, false, true>), g, b, lds, s, a, lo, hi, counter);
    else if (diag && enumerate)
        hipLaunchKernelGGL((search_kernel<W, true, true>), g, b, lds, s, a, lo, hi, counter);
    else if (diag)
        hipLaunchKernelGGL((search_kernel<W, true, false>), g, b, lds, s, a, lo, hi, counter);
    else if (enumerate)
        hipLaunchKernelGGL((search_kernel<W, false, true>), g, b, lds, s, a, lo, hi, counter);
    else
        hipLaunchKernelGGL((search_kernel<W, false, false>), g, b, lds, s, a, lo, hi, counter);
    return hipGetLastError();
}

size_t align_up(size_t x, size_t al) { return (x + al - 1) / al * al; }

template <int W, bool DIAG, bool ENUM>
int occ(int waves, int nwords) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search_kernel<W, DIAG, ENUM>, 64 * waves,
                                                      lds_bytes(W, waves, nwords)) != hipSuccess)
        return 2;
    return nb > 0 ? nb : 1;
}

template <int W>
int occ_w(bool diag, bool enumerate, int waves, int nwords) {
    if (diag && enumerate) return occ<W, true, true>(waves, nwords);
    if (diag) return occ<W, true, false>(waves, nwords);
    if (enumerate) return occ<W, false, true>(waves, nwords);
    return occ<W, false, false>(waves, nwords);
}

}  // namespace

int search_occupancy(int W, bool diag, bool enumerate, int waves, int nwords) {
    switch (W) {
        case 1: return occ_w<1>(diag, enumerate, waves, nwords);
        case 2: return occ_w<2>(diag, enumerate, waves, nwords);
        case 4: return occ_w<4>(diag, enumerate, waves, nwords);
        case 8: return occ_w<8>(diag, enumerate, waves, nwords);
        default: return occ_w<16>(diag, enumerate, waves, nwords);
    }
}

WideLayout wide_layout(const SearchDims &d, int Wx, int64_t scap, int32_t maxdepth, int waves) {
    WideLayout L{};
    L.Wx = Wx;
    L.scap = scap;
    L.maxdepth = maxdepth;
    const size_t ucap = (size_t)d.ucap, W = (size_t)Wx, bits = 64 * W;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.off_bitmap = take((size_t)d.nwords * 8);
    L.off_bpre = take(((size_t)d.nwords + 1) * 4);
    L.off_M = take(ucap * W * 8);
    L.off_gid = take(ucap * 4);
    L.off_cnt = take(ucap * 4);
    L.off_hv = take(bits * 8);
    L.off_deg = take(bits * 4);
    L.off_t1v = take(ucap * 4);
    L.off_t1c = take(ucap * 4);
    L.off_whist = take((bits + 1) * 4);
    // the top-level list: ids | hs | masks | first, cnt | H | orig | rows (see wframe_view)
    const size_t s1_words = align_up(ucap, 2) + 2 * ucap + 2 * ucap * W + 4 * bits + bits + 2 + 2 * bits * ((ucap + 63) / 64) + 2;
    L.off_S1 = take(s1_words * 4);
    L.off_waves = o;
    size_t w = 0;
    auto wtake = [&](size_t bytes) {
        const size_t at = w;
        w = align_up(w + bytes, 256);
        return at;
    };
    L.off_w_stack = wtake((size_t)scap * 4);
    L.off_w_u = wtake(ucap * 4);
    L.off_w_u2 = wtake(ucap * 4);
    L.off_w_bl = wtake(bits * 4);
    L.off_w_hist = wtake((bits + 2) * 4);
    L.off_w_mr = wtake(W * 8);
    L.off_w_rr = wtake(W * 8);
    L.off_w_hdr = wtake((size_t)maxdepth * sizeof(FrameState));
    L.wave_bytes = w;
    L.wg_bytes = align_up(o + (size_t)waves * w, 4096);
    return L;
}

hipError_t launch_wide(const SearchArgs &a, bool diag, bool enumerate, bool tb, int64_t lo, int64_t hi,
                       unsigned int *counter, int grid, int waves, hipStream_t s, int prune) {
    dim3 g(grid), b(64 * waves);
    const size_t lds = sizeof(WGShared);
    if (prune == 2) {
        if (enumerate)
            hipLaunchKernelGGL((wide_kernel<false, true, false, false, true>), g, b, lds, s, a, lo, hi, counter);
        else if (diag)
            hipLaunchKernelGGL((wide_kernel<true, false, false, false, true>), g, b, lds, s, a, lo, hi, counter);
        else
            hipLaunchKernelGGL((wide_kernel<false, false, false, false, true>), g, b, lds, s, a, lo, hi, counter);
        return hipGetLastError();
    }
    if (prune == 1) {
        if (enumerate)
            hipLaunchKernelGGL((wide_kernel<false, true, false, true>), g, b, lds, s, a, lo, hi, counter);
        else if (diag)
            hipLaunchKernelGGL((wide_kernel<true, false, false, true>), g, b, lds, s, a, lo, hi, counter);
        else
            hipLaunchKernelGGL((wide_kernel<false, false, false, true>), g, b, lds, s, a, lo, hi, counter);
        return hipGetLastError();
    }
    if (tb && !diag && !enumerate)
        hipLaunchKernelGGL((wide_kernel<false, false, true>), g, b, lds, s, a, lo, hi, counter);
    else if (diag && enumerate)
        hipLaunchKernelGGL((wide_kernel<true, true, false>), g, b, lds, s, a, lo, hi, counter);
    else if (diag)
        hipLaunchKernelGGL((wide_kernel<true, false, false>), g, b, lds, s, a, lo, hi, counter);
    else if (enumerate)
        hipLaunchKernelGGL((wide_kernel<false, true, false>), g, b, lds, s, a, lo, hi, counter);
    else
        hipLaunchKernelGGL((wide_kernel<false, false, false>), g, b, lds, s, a, lo, hi, counter);
    return hipGetLastError();
}

ArenaLayout search_layout(const SearchDims &d) {
    ArenaLayout L{};
    const size_t ucap = (size_t)d.ucap, W = (size_t)d.Wmax, bits = 64 * W;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.off_bitmap = take((size_t)d.nwords * 8);
    L.off_bpre = take(((size_t)d.nwords + 1) * 4);
    L.off_M = take(ucap * W * 8);
    L.off_gid = take(ucap * 4);
    L.off_cnt = take(ucap * 4);
    L.off_hv = take(bits * 8);
    L.off_deg = take(bits * 4);
    L.off_t1v = take(ucap * 4);
    L.off_t1c = take(ucap * 4);
    // ids | hs | masks | first, cnt | H | orig | rows (see frame_view)
    L.s1_words = align_up(ucap, 2) + 2 * ucap + 2 * ucap * W + 2 * bits + 2 * bits + 64 + 128 + 2 * bits * ((ucap + 63) / 64) + 2;
    L.off_S1 = take(L.s1_words * 4);
    L.off_hb = take((ucap / 64 + 1) * 8);
    L.off_hpre = take((ucap / 64 + 2) * 4);
    L.off_hpos = take(ucap * 4);
    L.off_waves = o;
    size_t w = 0;
    auto wtake = [&](size_t bytes) {
        const size_t at = w;
        w = align_up(w + bytes, 256);
        return at;
    };
    L.off_w_stack = wtake((size_t)d.scap * 4);
    L.off_w_u = wtake(ucap * 4);
    L.off_w_hdr = wtake((size_t)d.maxdepth * sizeof(FrameState));
    L.wave_bytes = w;
    L.wg_bytes = align_up(o + (size_t)d.waves * w, 4096);
    return L;
}

hipError_t launch_search(const SearchArgs &a, int W, bool diag, bool enumerate, bool tb, int64_t lo, int64_t hi,
                         unsigned int *counter, int grid, int waves, hipStream_t s) {
    switch (W) {
        case 1: return launch_w<1>(a, diag, enumerate, tb, lo, hi, counter, grid, waves, s);
        case 2: return launch_w<2>(a, diag, enumerate, tb, lo, hi, counter, grid, waves, s);
        case 4: return launch_w<4>(a, diag, enumerate, tb, lo, hi, counter, grid, waves, s);
        case 8: return launch_w<8>(a, diag, enumerate, tb, lo, hi, counter, grid, waves, s);
        case 16: return launch_w<16>(a, diag, enumerate, tb, lo, hi, counter, grid, waves, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mbe
