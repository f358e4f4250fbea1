// Depth-first MBEA search on gfx950 (wave64).
//
// What is computed: the maximal bicliques of Algorithm 1 (MBEA, section II-B), in the
// library's letters: the candidate x joins the growing set L (candidate side C), the
// shrinking set R (other side O) becomes R' = R n N(x), the maximality check fails when a
// vertex of Q is adjacent to all of R', the expansion moves every candidate of P adjacent
// to all of R' into L', and P' / Q' keep the vertices with 0 < |N(v) n R'| < |R'|.  The
// counts |N(v) n R'| come from the reverse scan of section III-E: walk R' and its
// neighbours instead of every candidate's list.  Candidates are taken in ascending count
// (sections II-C and III-E), ties in the order of the parent's list.
//
// How it maps to the hardware (this is the build's own design, not the paper's CUDA one):
//
//  * Coarse grain (section III-C's first-level subtrees): one workgroup owns one top-level
//    candidate x at a time, claimed from a global atomic counter, heaviest ranks first.
//
//  * Local universe.  Every vertex that can appear below x is a 2-hop neighbour of x and
//    every R below x is a subset of N(x).  The workgroup runs the reverse scan over N(x)
//    once and builds, for each 2-hop neighbour v, the mask M[v] = N(v) n N(x) as W 64-bit
//    words over the positions of N(x) (W = ceil(deg x / 64)).  Universe entries are indexed
//    in top-level rank order, so the top-level Q (earlier ranks) is a prefix.  After that a
//    count |N(v) n R'| is popcount(M[v] & R') and never touches the CSR again.
//
//  * Fine grain.  The top-level node's children are independent subtrees (the paper's k = 2
//    level): the waves of the workgroup claim them from an LDS counter and each runs its
//    own depth-first search.  A node is one pass of the wave over the parent's candidate
//    list: 64 lanes read 64 entries, AND them with R', popcount, and ballot/prefix-sum
//    compact the survivors; P' is stably counting-sorted by its counts.
//
//  * Compact stack (section III-B's goal: no recursion, no allocation).  A wave's frames
//    are candidate lists laid back to back in one preallocated array; a child's list is
//    strictly shorter than its parent's and is written right after it.  Frame headers
//    (list position, R as W words, the running hash of L) sit in a small array.
//
// Counts and hashes are commutative u64 sums, so results do not depend on which wave or
// workgroup handled which subtree.

#include "mbe_internal.h"

namespace mbe {

namespace {

constexpr uint64_t kHashK = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
__device__ __forceinline__ uint64_t hash_u(int32_t a) {
    return mix64(kHashK * (2ull * (uint64_t)(uint32_t)a + 1ull));
}
__device__ __forceinline__ uint64_t hash_v(int32_t b) {
    return mix64(kHashK * (2ull * (uint64_t)(uint32_t)b + 2ull));
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int ln = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (ln >= o) v += t;
    }
    return v;
}

template <int W>
struct Frame {
    const uint32_t *S;  // candidate list: [0, nq) Q part, [nq, n) P part in processing order
    int32_t n, nq, pos, level;
    int32_t end;        // candidates [pos, end) of the list are still to be taken here
    int32_t top;        // first free stack entry above this frame's list
    int32_t nL;         // |L| of the nodes below this frame
    uint64_t sL;        // sum of the L-side hash terms of L
    uint64_t fw;        // sum over S of (2 + deg v), byte tally only
    uint64_t R[W];      // R as a mask over the positions of N(x_root)
};

template <int W>
struct Ctx {
    const uint64_t *M;    // universe masks
    const int32_t *gid;   // universe global ids
    const uint64_t *hvl;  // R-side hash term per local other-side vertex
    const uint32_t *degl; // degree per local other-side vertex
    const int32_t *row;   // N(x_root) global ids
    const int32_t *c_off;
    int32_t x_root, s0, c_is_v;
    uint32_t *tv, *tc;    // per-wave staging for P'
    uint32_t *hist;       // per-wave LDS histogram (64*W bins)
    // records
    int32_t *rec;
    unsigned long long rec_cap, rec_offs_cap;
    unsigned long long *rec_offs;
    unsigned long long *acc;
    unsigned int *flags;
};

struct WaveAcc {
    uint64_t count, hash, out_ints, nodes, nonmax, bytes;
    uint32_t max_depth;
};

__device__ __forceinline__ uint64_t hash_L(int c_is_v, int32_t v) { return c_is_v ? hash_v(v) : hash_u(v); }
__device__ __forceinline__ uint64_t pair_hash(int c_is_v, uint64_t sL, uint64_t sR) {
    // h(A, B) = mix(sum hu(A) + mix(sum hv(B) + K)); A is the U side.
    return c_is_v ? mix64(sR + mix64(sL + kHashK)) : mix64(sL + mix64(sR + kHashK));
}

template <int W>
__device__ __forceinline__ int masked_count(const uint64_t *m, const uint64_t (&R)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += __popcll(m[w] & R[w]);
    return c;
}

// Stable counting sort by key of n staged (id, key) pairs into out[0, n); keys in [1, nbins).
// One wave; hist is this wave's LDS histogram.
__device__ void wave_sort_by_key(const uint32_t *tv, const uint32_t *tc, int n, int nbins,
                                 uint32_t *hist, uint32_t *out) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    for (int b = ln; b < nbins; b += 64) hist[b] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        if (j < n) atomicAdd(&hist[tc[j]], 1u);
    }
    __builtin_amdgcn_wave_barrier();
    int carry = 0;
    for (int base = 0; base < nbins; base += 64) {
        const int b = base + ln;
        const int h = b < nbins ? (int)hist[b] : 0;
        const int incl = wave_incl_scan(h);
        if (b < nbins) hist[b] = (uint32_t)(carry + incl - h);
        carry += __shfl(incl, 63);
    }
    __builtin_amdgcn_wave_barrier();
    const int nbits = nbins <= 1 ? 1 : 32 - __clz(nbins - 1);
    for (int base = 0; base < n; base += 64) {
        const int j = base + ln;
        const bool act = j < n;
        const uint32_t key = act ? tc[j] : 0u;
        const uint32_t v = act ? tv[j] : 0u;
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
            out[start + __popcll(same & below)] = v;
            // the highest lane of each equal-key group advances the bin
            if ((same >> ln) == 1ull) hist[key] = start + (uint32_t)__popcll(same);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Write one record [|A|, |B|, A..., B...] for the maximal biclique (L', R') of the current
// node: L' = {x_root} u {universe v : M[v] contains R'} (every vertex adjacent to all of
// R'), R' = the positions set in R.  Sides are sorted later by the canonicaliser.
template <int W>
__device__ void write_record(const Ctx<W> &c, const uint64_t (&R)[W], int nL, int r) {
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
    const int la = c.c_is_v ? r : nL;  // |A|
    int32_t *pl = o + 2 + (c.c_is_v ? r : 0);   // where L' goes
    int32_t *pr = o + 2 + (c.c_is_v ? 0 : nL);  // where R' goes
    if (ln == 0) {
        o[0] = la;
        o[1] = c.c_is_v ? nL : r;
        c.rec_offs[idx] = off;
        pl[0] = c.x_root;
    }
    int k = 1;
    for (int base = 0; base < c.s0; base += 64) {
        const int li = base + ln;
        bool in = li < c.s0;
        if (in) {
            const uint64_t *m = c.M + (size_t)li * W;
#pragma unroll
            for (int w = 0; w < W; ++w) in = in && ((m[w] & R[w]) == R[w]);
        }
        const uint64_t b = __ballot(in);
        const int at = k + __popcll(b & below);
        if (in && at < nL) pl[at] = c.gid[li];  // never past the reserved record
        k += __popcll(b);
    }
    int q = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const bool in = (R[w] >> ln) & 1ull;
        const uint64_t b = __ballot(in);
        const int at = q + __popcll(b & below);
        if (in && at < r) pr[at] = c.row[w * 64 + ln];
        q += __popcll(b);
    }
}

// One node: candidate S[i] of frame F.  Returns true when a child frame was written to C
// (C.S must point at free stack space of at least F.n - 1 entries).
template <int W, bool DIAG, bool ENUM>
__device__ bool process_node(const Ctx<W> &c, const Frame<W> &F, int i, Frame<W> &C, WaveAcc &acc) {
    const int ln = lane_id();
    const uint64_t below = lanes_below();
    const uint32_t x = F.S[i];
    const uint64_t *mx = c.M + (size_t)x * W;
    uint64_t R[W];
    int r = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        R[w] = F.R[w] & mx[w];  // R' = R n N(x)
        r += __popcll(R[w]);
    }
    uint32_t *cs = const_cast<uint32_t *>(C.S);

    // maximality check against Q = S[0, i): a vertex adjacent to all of R' ends the node
    int qn = 0;
    bool nonmax = false;
    uint64_t fwq = 0;
    for (int base = 0; base < i; base += 64) {
        const int j = base + ln;
        const bool act = j < i;
        uint32_t v = 0;
        int cnt = 0;
        if (act) {
            v = F.S[j];
            cnt = masked_count<W>(c.M + (size_t)v * W, R);
        }
        if (__ballot(act && cnt == r)) {
            nonmax = true;
            break;
        }
        const bool keep = act && cnt > 0;
        const uint64_t kb = __ballot(keep);
        if (keep) {
            cs[qn + __popcll(kb & below)] = v;
            if (DIAG) fwq += 2ull + (uint64_t)(c.c_off[c.gid[v] + 1] - c.c_off[c.gid[v]]);
        }
        qn += __popcll(kb);
    }

    uint64_t degx = 0, rs = 0;
    if (DIAG) {
        acc.nodes += 1;
        if ((uint32_t)F.level > acc.max_depth) acc.max_depth = (uint32_t)F.level;
        degx = (uint64_t)(c.c_off[c.gid[x] + 1] - c.c_off[c.gid[x]]);
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
            if ((R[w] >> ln) & 1ull) t += 2ull + (uint64_t)c.degl[w * 64 + ln];
        rs = wave_sum_u64(t);
    }
    if (nonmax) {
        if (DIAG) {
            acc.nonmax += 1;
            const uint64_t fw = F.fw - (2ull + degx);
            acc.bytes += 4ull * ((2ull + degx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r);
        }
        return false;
    }

    // expansion over P = S(i, n): adjacent to all of R' joins L', partially adjacent joins P'
    int pn = 0, ne = 0;
    uint64_t exps = 0, fwp = 0;
    for (int base = i + 1; base < F.n; base += 64) {
        const int j = base + ln;
        const bool act = j < F.n;
        uint32_t v = 0;
        int cnt = 0;
        if (act) {
            v = F.S[j];
            cnt = masked_count<W>(c.M + (size_t)v * W, R);
        }
        const bool full = act && cnt == r;
        if (full) exps += hash_L(c.c_is_v, c.gid[v]);
        ne += __popcll(__ballot(full));
        const bool pk = act && cnt > 0 && cnt < r;
        const uint64_t pb = __ballot(pk);
        if (pk) {
            const int p = pn + __popcll(pb & below);
            c.tv[p] = v;
            c.tc[p] = (uint32_t)cnt;
            if (DIAG) fwp += 2ull + (uint64_t)(c.c_off[c.gid[v] + 1] - c.c_off[c.gid[v]]);
        }
        pn += __popcll(pb);
    }

    // report (L', R')
    const uint64_t sL = F.sL + hash_L(c.c_is_v, c.gid[x]) + wave_sum_u64(exps);
    uint64_t sr = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if ((R[w] >> ln) & 1ull) sr += c.hvl[w * 64 + ln];
    sr = wave_sum_u64(sr);
    const int nL = F.nL + 1 + ne;
    acc.count += 1;
    acc.hash += pair_hash(c.c_is_v, sL, sr);
    acc.out_ints += 2ull + (uint64_t)nL + (uint64_t)r;
    if (ENUM) write_record<W>(c, R, nL, r);
    if (DIAG) {
        const uint64_t fw = F.fw - (2ull + degx);
        acc.bytes += 4ull * ((2ull + degx) + (rs < fw ? rs : fw) + (uint64_t)(F.n - 1) + (uint64_t)r +
                             (uint64_t)pn + (uint64_t)qn);
    }
    if (pn == 0) return false;

    wave_sort_by_key(c.tv, c.tc, pn, r, c.hist, cs + qn);
    __threadfence_block();
    C.n = qn + pn;
    C.nq = qn;
    C.pos = qn;
    C.end = qn + pn;
    C.level = F.level + 1;
    C.nL = nL;
    C.sL = sL;
    C.fw = DIAG ? wave_sum_u64(fwq + fwp) : 0ull;
#pragma unroll
    for (int w = 0; w < W; ++w) C.R[w] = R[w];
    return true;
}

struct WGShared {
    unsigned long long task;
    int s0;
    int claim;
    int nonmax;
    int pcount;
    unsigned long long exps;
    unsigned long long fw1;
    unsigned long long hvsum;
    unsigned long long rs1;
    int nexp;
    int pad;
    int scan[16];  // per-wave partial sums for the block scan
};

// Block-wide exclusive prefix of popcounts over nwords bitmap words into bpre; returns total
// through sh->s0.  All threads must call it.
__device__ void block_popcount_prefix(const uint64_t *bitmap, uint32_t *bpre, int nwords, WGShared *sh) {
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
}

template <int W, bool DIAG, bool ENUM>
__global__ __launch_bounds__(512) void search_kernel(SearchArgs a, int64_t lo, int64_t hi,
                                                      unsigned int *counter) {
    extern __shared__ unsigned char lds_raw[];
    WGShared *sh = reinterpret_cast<WGShared *>(lds_raw);
    const int tid = threadIdx.x, nt = blockDim.x, wid = tid >> 6, nw = nt >> 6, ln = lane_id();
    uint32_t *hist = reinterpret_cast<uint32_t *>(lds_raw + sizeof(WGShared)) + (size_t)wid * (64 * W);

    char *wg = a.arena + (size_t)blockIdx.x * a.lay.wg_bytes;
    uint64_t *bitmap = reinterpret_cast<uint64_t *>(wg + a.lay.off_bitmap);
    uint32_t *bpre = reinterpret_cast<uint32_t *>(wg + a.lay.off_bpre);
    uint64_t *M = reinterpret_cast<uint64_t *>(wg + a.lay.off_M);
    int32_t *gid = reinterpret_cast<int32_t *>(wg + a.lay.off_gid);
    uint32_t *cnt1 = reinterpret_cast<uint32_t *>(wg + a.lay.off_cnt);
    uint64_t *hvl = reinterpret_cast<uint64_t *>(wg + a.lay.off_hv);
    uint32_t *degl = reinterpret_cast<uint32_t *>(wg + a.lay.off_deg);
    uint32_t *S1 = reinterpret_cast<uint32_t *>(wg + a.lay.off_S1);
    uint32_t *t1v = reinterpret_cast<uint32_t *>(wg + a.lay.off_t1v);
    uint32_t *t1c = reinterpret_cast<uint32_t *>(wg + a.lay.off_t1c);
    char *wv = wg + a.lay.off_waves + (size_t)wid * a.lay.wave_bytes;
    uint32_t *stk = reinterpret_cast<uint32_t *>(wv + a.lay.off_w_stack);
    Frame<W> *hdr = reinterpret_cast<Frame<W> *>(wv + a.lay.off_w_hdr);

    Ctx<W> c;
    c.M = M;
    c.gid = gid;
    c.hvl = hvl;
    c.degl = degl;
    c.c_off = a.c_off;
    c.c_is_v = a.c_is_v;
    c.tv = reinterpret_cast<uint32_t *>(wv + a.lay.off_w_tv);
    c.tc = reinterpret_cast<uint32_t *>(wv + a.lay.off_w_tc);
    c.hist = hist;
    c.rec = a.rec;
    c.rec_cap = a.rec_cap;
    c.rec_offs = a.rec_offs;
    c.rec_offs_cap = a.rec_offs_cap;
    c.acc = a.acc;
    c.flags = a.flags;

    WaveAcc acc = {0, 0, 0, 0, 0, 0, 0};
    bool aborted = false;

    for (;;) {
        if (tid == 0) {
            // stop claiming once any wave has run out of stack: the host reruns with more
            const unsigned int f = __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh->task = (f & (FLAG_STACK_OVERFLOW | FLAG_DEPTH_OVERFLOW)) ? (1ull << 62)
                                                                          : (unsigned long long)atomicAdd(counter, 1u);
        }
        __syncthreads();
        const int64_t t = (int64_t)sh->task;
        if (lo + t >= hi) break;
        const int64_t k = hi - 1 - t;  // ranks are claimed from the top (largest degree) down
        const int32_t x = a.order[k];
        const int32_t rb = a.c_off[x];
        const int32_t d = a.c_off[x + 1] - rb;
        const int32_t *row = a.c_adj + rb;
        c.row = row;
        c.x_root = x;

        // -- reverse scan 1: mark the ranks of all 2-hop neighbours of x
        for (int j = wid; j < d; j += nw) {
            const int32_t w = row[j];
            const int32_t e0 = a.o_off[w], e1 = a.o_off[w + 1];
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
            const int32_t w = row[j];
            const uint64_t h = a.c_is_v ? hash_u(w) : hash_v(w);
            hvl[j] = h;
            hv_local += h;
            const uint32_t dw = (uint32_t)(a.o_off[w + 1] - a.o_off[w]);
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
            sh->claim = 0;
        }
        __threadfence_block();
        __syncthreads();
        hv_local = wave_sum_u64(hv_local);
        rs_local = wave_sum_u64(rs_local);
        if (ln == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&sh->hvsum), (unsigned long long)hv_local);
            atomicAdd(reinterpret_cast<unsigned long long *>(&sh->rs1), (unsigned long long)rs_local);
        }

        // -- universe numbering: prefix of bitmap popcounts (rank order)
        block_popcount_prefix(bitmap, bpre, a.nwords, sh);
        __threadfence_block();
        __syncthreads();
        const int s0 = sh->s0;
        const int nq0 = (int)bpre[k >> 6] + __popcll(bitmap[k >> 6] & ((1ull << (k & 63)) - 1ull));
        c.s0 = s0;
        for (int wd = tid; wd < a.nwords; wd += nt) {
            uint64_t bits = bitmap[wd];
            uint32_t pos = bpre[wd];
            while (bits) {
                const int b = __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1ull;
                gid[pos++] = a.order[wd * 64 + b];
            }
        }
        for (size_t q = tid; q < (size_t)s0 * W; q += nt) M[q] = 0ull;
        __threadfence_block();
        __syncthreads();

        // -- reverse scan 2: M[v] gets bit j for every w_j in N(x) adjacent to v
        for (int j = wid; j < d; j += nw) {
            const int32_t w = row[j];
            const int32_t e0 = a.o_off[w], e1 = a.o_off[w + 1];
            for (int p = e0 + ln; p < e1; p += 64) {
                const int32_t v = a.o_adj[p];
                if (v != x) {
                    const int32_t rk = a.rank[v];
                    const uint32_t li = bpre[rk >> 6] + (uint32_t)__popcll(bitmap[rk >> 6] & ((1ull << (rk & 63)) - 1ull));
                    atomicOr(reinterpret_cast<unsigned long long *>(&M[(size_t)li * W + (j >> 6)]), 1ull << (j & 63));
                }
            }
        }
        __threadfence_block();
        __syncthreads();

        // -- the top-level node for x: counts, maximality against earlier ranks, expansion
        for (int wd = tid; wd < a.nwords; wd += nt) bitmap[wd] = 0ull;
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
                    if (cc == d) nm = true;
                    else fw += dg;
                } else if (cc == d) {
                    ex += hash_L(a.c_is_v, g);
                    ++nexp;
                } else {
                    ++pc;
                    fw += dg;
                }
            }
            if (__ballot(nm) && ln == 0) atomicOr(&sh->nonmax, 1);
            ex = wave_sum_u64(ex);
            fw = wave_sum_u64(fw);
            for (int o = 32; o > 0; o >>= 1) {
                pc += __shfl_xor(pc, o);
                nexp += __shfl_xor(nexp, o);
            }
            if (ln == 0) {
                atomicAdd(&sh->pcount, pc);
                atomicAdd(&sh->nexp, nexp);
                atomicAdd(reinterpret_cast<unsigned long long *>(&sh->exps), (unsigned long long)ex);
                atomicAdd(reinterpret_cast<unsigned long long *>(&sh->fw1), (unsigned long long)fw);
            }
        }
        __threadfence_block();
        __syncthreads();
        const bool root_nonmax = sh->nonmax != 0;
        const int P1 = sh->pcount;
        if (tid == 0 && !aborted) {
            const uint64_t dx = (uint64_t)d;
            if (DIAG) {
                acc.nodes += 1;
                if (acc.max_depth < 1) acc.max_depth = 1;
                const uint64_t fwtop = a.total_fw - (2ull + dx);
                const uint64_t rs = sh->rs1;
                uint64_t b = (2ull + dx) + (rs < fwtop ? rs : fwtop) + (uint64_t)(a.ncand - 1) + dx;
                if (root_nonmax) acc.nonmax += 1;
                else b += (uint64_t)P1 + (uint64_t)nq0;
                acc.bytes += 4ull * b;
            }
            if (!root_nonmax) {
                const uint64_t sL = hash_L(a.c_is_v, x) + sh->exps;
                const int nL = 1 + sh->nexp;
                acc.count += 1;
                acc.hash += pair_hash(a.c_is_v, sL, sh->hvsum);
                acc.out_ints += 2ull + (uint64_t)nL + (uint64_t)d;
            }
        }
        if (ENUM && !root_nonmax && wid == 0) {
            uint64_t R1[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int bits = d - 64 * w;
                R1[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : ((1ull << bits) - 1ull));
            }
            write_record<W>(c, R1, 1 + sh->nexp, d);
        }
        if (root_nonmax || P1 == 0) {
            __syncthreads();
            continue;
        }

        // -- the top-level child list S1 = Q1 (earlier ranks) ++ P1 sorted by count
        for (int li = tid; li < nq0; li += nt) S1[li] = (uint32_t)li;
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
            __threadfence_block();
            wave_sort_by_key(t1v, t1c, pn, d, hist, S1 + nq0);
        }
        __threadfence_block();
        __syncthreads();

        // -- second level: waves claim the top-level children, each a depth-first search
        Frame<W> F1;
        F1.S = S1;
        F1.n = nq0 + P1;
        F1.nq = nq0;
        F1.pos = nq0;
        F1.level = 2;
        F1.nL = 1 + sh->nexp;
        F1.sL = hash_L(a.c_is_v, x) + sh->exps;
        F1.fw = sh->fw1;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int bits = d - 64 * w;
            F1.R[w] = bits >= 64 ? ~0ull : (bits <= 0 ? 0ull : ((1ull << bits) - 1ull));
        }
        F1.end = F1.n;
        F1.top = 0;
        while (!aborted) {
            int i = 0;
            if (ln == 0) i = atomicAdd(&sh->claim, 1);
            i = __shfl(i, 0) + nq0;
            if (i >= F1.n) break;
            // the claimed child is a one-candidate range of the shared top-level list
            Frame<W> cur = F1;
            cur.pos = i;
            cur.end = i + 1;
            int depth = 0;
            for (;;) {
                if (cur.pos >= cur.end) {
                    if (depth == 0) break;
                    --depth;
                    cur = hdr[depth];
                    continue;
                }
                const int ii = cur.pos++;
                if ((size_t)cur.top + (size_t)cur.n > (size_t)a.scap) {
                    if (ln == 0) atomicOr(a.flags, (unsigned int)FLAG_STACK_OVERFLOW);
                    aborted = true;
                    break;
                }
                Frame<W> ch;
                ch.S = stk + cur.top;
                if (process_node<W, DIAG, ENUM>(c, cur, ii, ch, acc)) {
                    if (depth >= a.maxdepth) {
                        if (ln == 0) atomicOr(a.flags, (unsigned int)FLAG_DEPTH_OVERFLOW);
                        aborted = true;
                        break;
                    }
                    ch.top = cur.top + ch.n;
                    hdr[depth] = cur;  // every lane stores the same header
                    __threadfence_block();
                    ++depth;
                    cur = ch;
                }
            }
        }
        __syncthreads();
    }

    // flush this wave's tallies (values are wave-uniform except thread 0's top-level ones)
    if (ln == 0) {
        if (acc.count) atomicAdd(&a.acc[ACC_COUNT], (unsigned long long)acc.count);
        if (acc.hash) atomicAdd(&a.acc[ACC_HASH], (unsigned long long)acc.hash);
        if (acc.out_ints) atomicAdd(&a.acc[ACC_OUT_INTS], (unsigned long long)acc.out_ints);
        if (DIAG) {
            atomicAdd(&a.acc[ACC_NODES], (unsigned long long)acc.nodes);
            atomicAdd(&a.acc[ACC_NONMAX], (unsigned long long)acc.nonmax);
            atomicAdd(&a.acc[ACC_BYTES], (unsigned long long)acc.bytes);
            atomicMax(&a.acc[ACC_MAX_DEPTH], (unsigned long long)acc.max_depth);
        }
    }
}

template <int W>
hipError_t launch_w(const SearchArgs &a, bool diag, bool enumerate, int64_t lo, int64_t hi,
                    unsigned int *counter, int grid, int waves, size_t lds, hipStream_t s) {
    dim3 g(grid), b(64 * waves);
    if (diag && enumerate)
        hipLaunchKernelGGL((search_kernel<W, true, true>), g, b, lds, s, a, lo, hi, counter);
    else if (diag)
        hipLaunchKernelGGL((search_kernel<W, true, false>), g, b, lds, s, a, lo, hi, counter);
    else if (enumerate)
        hipLaunchKernelGGL((search_kernel<W, false, true>), g, b, lds, s, a, lo, hi, counter);
    else
        hipLaunchKernelGGL((search_kernel<W, false, false>), g, b, lds, s, a, lo, hi, counter);
    return hipGetLastError();
}

}  // namespace

size_t frame_header_bytes(int W) {
    switch (W) {
        case 1: return sizeof(Frame<1>);
        case 2: return sizeof(Frame<2>);
        case 4: return sizeof(Frame<4>);
        case 8: return sizeof(Frame<8>);
        default: return sizeof(Frame<16>);
    }
}

size_t search_lds_bytes(int W, int waves) {
    return sizeof(WGShared) + (size_t)waves * 64 * W * sizeof(uint32_t);
}

hipError_t launch_search(const SearchArgs &a, int W, bool diag, bool enumerate, int64_t lo, int64_t hi,
                         unsigned int *counter, int grid, int waves, size_t lds, hipStream_t s) {
    switch (W) {
        case 1: return launch_w<1>(a, diag, enumerate, lo, hi, counter, grid, waves, lds, s);
        case 2: return launch_w<2>(a, diag, enumerate, lo, hi, counter, grid, waves, lds, s);
        case 4: return launch_w<4>(a, diag, enumerate, lo, hi, counter, grid, waves, lds, s);
        case 8: return launch_w<8>(a, diag, enumerate, lo, hi, counter, grid, waves, lds, s);
        case 16: return launch_w<16>(a, diag, enumerate, lo, hi, counter, grid, waves, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mbe
