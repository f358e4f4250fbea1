// C-ABI entry points of libmbe.so (declared in include/mbe.h).
//
// One call = validate the CSR pair, rank the candidates, run the persistent search kernel
// once per mask-width class (widest first), read back the 16 accumulators, and for
// mbe_enumerate put the records into canonical order.  Device working memory is cached per
// device and grows on demand; calls on one device are serialised by a mutex.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mbe.h"
#include "mbe_internal.h"

namespace {

using namespace mbe;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool fresh = false;  // set when ensure() allocated new memory (contents undefined)
    hipError_t ensure(size_t n) {
        fresh = false;
        if (n <= bytes && p) return hipSuccess;
        fresh = true;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t want = n < 256 ? 256 : n;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = want;
        return hipSuccess;
    }
    template <typename T>
    T *as(size_t byte_off = 0) const {
        return reinterpret_cast<T *>(static_cast<char *>(p) + byte_off);
    }
};

struct DeviceState {
    std::mutex mu;
    DevBuf graph, prep, sort_tmp, arena, small, steal, slots, warena, witems, loads, twin;
    DevBuf rec, rec_offs, rec_tmp, rec_lens, canon_tmp, out_tmp;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cus = 0;
    // one stream per mask class, so the class launches overlap (created on first use)
    hipStream_t cls_stream[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // the largest wave-stack and frame-header capacities an earlier call had to grow to:
    // later calls start there instead of repeating a launch that runs out
    int64_t scap_floor = 0;
    int32_t depth_floor = 0;
    int64_t wscap_floor = 0;   // the same for the wide search
    int32_t wdepth_floor = 0;
    // device address of this device's copy of the no-allocation scratch (set up on the first
    // mbe_count_noalloc call on the device)
    char *scratch = nullptr;
};

hipError_t ensure_class_streams(DeviceState *st) {
    if (st->fork) return hipSuccess;
    for (int c = 0; c < 5; ++c) {
        hipError_t e = hipStreamCreateWithFlags(&st->cls_stream[c], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&st->join[c], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    return hipEventCreateWithFlags(&st->fork, hipEventDisableTiming);
}

std::mutex g_states_mu;
DeviceState *g_states[64] = {nullptr};

DeviceState *state_for(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_states_mu);
    if (!g_states[dev]) {
        DeviceState *s = new DeviceState();
        if (hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
            delete s;
            return nullptr;
        }
        if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || s->cus <= 0)
            s->cus = 256;
        g_states[dev] = s;
    }
    return g_states[dev];
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Fixed device scratch of mbe_count_noalloc, for callers that cannot allocate.  Each device
// that runs the library holds its own copy until the process ends.  In host code the name
// `scratch` is not a device address: the address of a device's copy comes from
// hipGetSymbolAddress, taken once per device (DeviceState::scratch), and only that address is
// handed to kernels and copies.
constexpr size_t kScratchBytes = (size_t)MBE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device memory of one call handed out in order from a fixed region (the scratch).
struct FixedRegion {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void *take(size_t bytes, size_t align = 256) {
        const size_t at = align_up(used, align);
        if (at > cap || bytes > cap - at) return nullptr;
        used = at + bytes;
        return base + at;
    }
};

int map_err(hipError_t e) {
    if (e == hipSuccess) return MBE_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MBE_ERR_OUT_OF_MEMORY;
    return MBE_ERR_DEVICE;
}

#define MBE_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return map_err(_e);      \
    } while (0)

#define MBE_CALL(expr)                                 \
    do {                                               \
        const int _r = (expr);                         \
        if (_r != MBE_OK) return _r;                   \
    } while (0)

// Host-side check of a CSR pair (the same rules as the device validator): both offset arrays
// start at 0, never decrease and end at n_edges; the U rows strictly ascend with V ids in
// range; and the V side is exactly their transpose.  One pass in U-row order keeps a cursor
// per V row: the entry (r, c) must be the next entry of V row c, so each V row is consumed in
// ascending r (which also makes the V rows sorted, duplicate-free and in range), and every
// V row must be consumed to its end.  O(|E|).
bool host_valid_pair(int32_t n_u, int32_t n_v, int32_t n_edges, const int32_t *u_off, const int32_t *u_adj,
                     const int32_t *v_off, const int32_t *v_adj) {
    auto offsets_ok = [&](int32_t n, const int32_t *off) {
        if (off[0] != 0 || off[n] != n_edges) return false;
        for (int32_t r = 0; r < n; ++r)
            if (off[r] > off[r + 1]) return false;
        return true;
    };
    if (!offsets_ok(n_u, u_off) || !offsets_ok(n_v, v_off)) return false;
    std::vector<int32_t> cur(v_off, v_off + n_v);
    for (int32_t r = 0; r < n_u; ++r) {
        int32_t prev = -1;
        for (int32_t p = u_off[r]; p < u_off[r + 1]; ++p) {
            const int32_t c = u_adj[p];
            if (c <= prev || c >= n_v) return false;
            prev = c;
            const int32_t q = cur[c];
            if (q >= v_off[c + 1] || v_adj[q] != r) return false;
            cur[c] = q + 1;
        }
    }
    for (int32_t c = 0; c < n_v; ++c)
        if (cur[c] != v_off[c + 1]) return false;
    return true;
}

// Top-level candidates above the widest mask class: rank (or task) range [lo, hi), searched by
// the wide kernel with Wx words per universe mask.
struct WideRange {
    int64_t lo = 0, hi = 0;
    int Wx = 0;
};

// Device memory the wide search's workgroup slots may take (their count shrinks to fit).
constexpr size_t kWideArenaBytes = (size_t)4 << 30;

struct Opts {
    int side, waves, grid, diag, no_validate, steal_k;
    int tb;     // diagnostics = 2: the production search with its design-byte tally
    int prune;  // section II-C: 1 iMBEA's candidate pruning, 2 the pivot rule
    int64_t root_lo, root_hi;
    hipStream_t stream;
    char *ws;         // the caller's workspace (mbe_count), or NULL
    size_t ws_bytes;
};

Opts read_opts(const mbe_options *o) {
    Opts r{0, 8, 0, 0, 0, 2, 0, 0, 0, -1, nullptr, nullptr, 0};
    if (!o) return r;
    r.side = o->side;
    r.waves = o->wg_waves > 0 ? o->wg_waves : 8;
    r.grid = o->grid > 0 ? o->grid : 0;
    r.diag = o->diagnostics == 1;
    r.tb = o->diagnostics == 2;
    r.prune = o->prune;
    if (r.prune < 0 || r.prune > 2) r.side = -1;  // (rejected as an invalid argument)
    if (r.prune && r.tb) r.side = -1;             // (no tally instance with pruning: rejected)
    if (o->diagnostics < 0 || o->diagnostics > 2) r.side = -1;  // (rejected as an invalid argument)
    r.no_validate = o->no_validate != 0;
    r.steal_k = o->steal_k == 0 ? 2 : o->steal_k;
    r.root_lo = o->root_lo > 0 ? o->root_lo : 0;
    r.root_hi = o->root_hi > 0 ? o->root_hi : -1;
    r.stream = static_cast<hipStream_t>(o->stream);
    r.ws = static_cast<char *>(o->workspace);
    r.ws_bytes = (size_t)o->workspace_bytes;
    if ((r.ws != nullptr) != (r.ws_bytes > 0)) r.side = -1;  // (rejected as an invalid argument)
    return r;
}

int run_search(DeviceState *st, SearchArgs &a, SearchDims dims, const int64_t *cls_lo, const int64_t *cls_hi,
               bool diag, bool enumerate, bool tb, int grid, int waves, unsigned long long *run_acc, size_t run_acc_bytes,
               unsigned long long *hacc, unsigned int *hflags_out, float *ms, hipStream_t s,
               unsigned long long *graph_acc, size_t graph_acc_bytes, int *attempts, char *small, FixedRegion *fx,
               const WideRange &wr, std::vector<unsigned long long> *loads = nullptr);

size_t search_footprint(DeviceState *st, SearchDims dims, const int64_t *cls_lo, const int64_t *cls_hi, bool diag,
                        bool enumerate, int grid, int waves, const WideRange &wr);

// mbe_count / mbe_enumerate; with ws_out, only the preparation runs and *ws_out receives the
// device bytes the search of this call would hold; with fixed (mbe_count_noalloc), every
// device buffer of the call is carved from the device's scratch and nothing is allocated
int run(const mbe_graph *g, const mbe_options *opt_in, mbe_result *out, int32_t *ubuf, uint64_t ucap_ints,
        int ubuf_on_device, bool enumerate, size_t *ws_out = nullptr, bool fixed = false,
        std::vector<unsigned long long> *loads = nullptr) {
    if (!g || !out) return MBE_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    if (g->n_u < 0 || g->n_v < 0 || g->n_edges < 0) return MBE_ERR_INVALID_ARG;
    Opts opt = read_opts(opt_in);
    if (opt.side < 0 || opt.side > 2 || opt.waves < 1 || opt.waves > 8 ||
        opt.steal_k < 1 || opt.steal_k > 3)
        return MBE_ERR_INVALID_ARG;
    if (enumerate && !ubuf && ucap_ints > 0) return MBE_ERR_INVALID_ARG;
    if (opt.ws && (fixed || enumerate || ws_out || loads)) return MBE_ERR_INVALID_ARG;  // (mbe_count only)
    const int side = opt.side ? opt.side : (g->n_v < g->n_u ? 2 : 1);
    out->side = (uint32_t)side;
    if (g->n_edges > 0 && (g->n_u == 0 || g->n_v == 0)) return MBE_ERR_INVALID_GRAPH;
    if (g->n_edges > 0 && (!g->u_off || !g->u_adj || !g->v_off || !g->v_adj)) return MBE_ERR_INVALID_ARG;
    if (!g->on_device && !opt.no_validate) {
        // host arrays: check before any device work
        if ((g->n_u > 0 && !g->u_off) || (g->n_v > 0 && !g->v_off)) return MBE_ERR_INVALID_ARG;
        if (g->n_edges > 0 || (g->u_off && g->v_off)) {
            if (!host_valid_pair(g->n_u, g->n_v, g->n_edges, g->u_off, g->u_adj, g->v_off, g->v_adj))
                return MBE_ERR_INVALID_GRAPH;
        }
    }
    if (g->n_u == 0 || g->n_v == 0 || g->n_edges == 0) return MBE_OK;

    int dev = 0;
    MBE_TRY(hipGetDevice(&dev));
    DeviceState *st = state_for(dev);
    if (!st) return MBE_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(st->mu);
    hipStream_t s = opt.stream;

    FixedRegion fxr, *fx = nullptr;
    if (opt.ws) {
        // the caller's workspace: every buffer of the call is carved from it
        const size_t skip = align_up((size_t)(uintptr_t)opt.ws, 256) - (size_t)(uintptr_t)opt.ws;
        if (skip >= opt.ws_bytes) return MBE_ERR_SCRATCH_LIMIT;
        fxr.base = opt.ws + skip;
        fxr.cap = opt.ws_bytes - skip;
        fx = &fxr;
    } else if (fixed) {
        if (enumerate || ws_out) return MBE_ERR_INVALID_ARG;
        if (!st->scratch) {
            // set-up, once per device (this device is current): the address of its copy
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return map_err(e);
            if (!p) return MBE_ERR_DEVICE;
            st->scratch = static_cast<char *>(p);
        }
        fxr.base = st->scratch;
        fxr.cap = kScratchBytes;
        fx = &fxr;
    }
    // a buffer of the call: the device's cached buffer b (grown when needed), or a piece of
    // the scratch
    auto mem = [&](DevBuf &b, size_t bytes, char **p) -> int {
        if (fx) {
            *p = static_cast<char *>(fx->take(bytes));
            return *p ? MBE_OK : MBE_ERR_SCRATCH_LIMIT;
        }
        const hipError_t e = b.ensure(bytes);
        if (e != hipSuccess) return map_err(e);
        *p = b.as<char>();
        return MBE_OK;
    };

    const int32_t nu = g->n_u, nv = g->n_v, ne = g->n_edges;
    const int32_t *u_off = g->u_off, *u_adj = g->u_adj, *v_off = g->v_off, *v_adj = g->v_adj;
    if (!g->on_device) {
        const size_t b_uoff = align_up(((size_t)nu + 1) * 4, 256), b_voff = align_up(((size_t)nv + 1) * 4, 256);
        const size_t b_adj = align_up((size_t)ne * 4, 256);
        char *gb = nullptr;
        MBE_CALL(mem(st->graph, b_uoff + b_voff + 2 * b_adj, &gb));
        int32_t *d_uoff = reinterpret_cast<int32_t *>(gb), *d_voff = reinterpret_cast<int32_t *>(gb + b_uoff);
        int32_t *d_uadj = reinterpret_cast<int32_t *>(gb + b_uoff + b_voff);
        int32_t *d_vadj = reinterpret_cast<int32_t *>(gb + b_uoff + b_voff + b_adj);
        MBE_TRY(hipMemcpyAsync(d_uoff, u_off, ((size_t)nu + 1) * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_voff, v_off, ((size_t)nv + 1) * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_uadj, u_adj, (size_t)ne * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_vadj, v_adj, (size_t)ne * 4, hipMemcpyHostToDevice, s));
        u_off = d_uoff;
        v_off = d_voff;
        u_adj = d_uadj;
        v_adj = d_vadj;
    }

    // small device block: acc[16] | flags | counters[8] + live steal slots[8] + third-level
    // sharing counters[48] | stats[16]
    char *small = nullptr;
    MBE_CALL(mem(st->small, 4096, &small));
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(small);
    unsigned int *flags = reinterpret_cast<unsigned int *>(small + 256);
    unsigned long long *stats = reinterpret_cast<unsigned long long *>(small + 1024);

    if (!opt.no_validate && g->on_device) {
        MBE_TRY(launch_zero(flags, 4, s));
        MBE_TRY(launch_validate(nu, nv, ne, u_off, u_adj, v_off, v_adj, flags, s));
        unsigned int hf = 0;
        MBE_TRY(hipMemcpyAsync(&hf, flags, 4, hipMemcpyDeviceToHost, s));
        MBE_TRY(hipStreamSynchronize(s));
        if (hf & FLAG_BAD_GRAPH) return MBE_ERR_INVALID_GRAPH;
    }

    const bool c_is_v = side == 2;
    const int32_t nc = c_is_v ? nv : nu, no = c_is_v ? nu : nv;
    const int32_t *c_off = c_is_v ? v_off : u_off, *c_adj = c_is_v ? v_adj : u_adj;
    const int32_t *o_off = c_is_v ? u_off : v_off, *o_adj = c_is_v ? u_adj : v_adj;

    // rank the candidates by (degree, id)
    const size_t b_keys = align_up((size_t)nc * 8, 256), b_i32 = align_up((size_t)nc * 4, 256);
    char *pb = nullptr;
    MBE_CALL(mem(st->prep, 2 * b_keys + 2 * b_i32, &pb));
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(pb);
    unsigned long long *sorted = reinterpret_cast<unsigned long long *>(pb + b_keys);
    int32_t *order = reinterpret_cast<int32_t *>(pb + 2 * b_keys);
    int32_t *rank = reinterpret_cast<int32_t *>(pb + 2 * b_keys + b_i32);
    MBE_TRY(launch_zero(stats, 16 * 8, s));
    MBE_TRY(launch_rank_keys(nc, c_off, c_adj, o_off, keys, stats, s));
    int end_bit = 32;
    while (end_bit < 64 && ((unsigned long long)no >> (end_bit - 32)) != 0ull) ++end_bit;
    size_t tmp_bytes = 0;
    MBE_TRY(radix_sort_u64(nullptr, &tmp_bytes, keys, sorted, nc, end_bit, s));
    char *tb = nullptr;
    MBE_CALL(mem(st->sort_tmp, tmp_bytes, &tb));
    if (!fx) tmp_bytes = st->sort_tmp.bytes;
    MBE_TRY(radix_sort_u64(tb, &tmp_bytes, keys, sorted, nc, end_bit, s));
    unsigned long long hstats[16];
    MBE_TRY(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
    MBE_TRY(hipStreamSynchronize(s));
    const int32_t nzero = (int32_t)hstats[0];
    const int32_t ncand = nc - nzero;
    if (ncand <= 0) return MBE_OK;
    MBE_TRY(launch_rank_scatter(nc, nzero, sorted, order, rank, s));

    // rank ranges of the mask-width classes (ranks ascend with degree)
    int64_t cls_lo[5], cls_hi[5];
    int64_t run_r = 0;
    int Wmax = 1;
    for (int c = 0; c < 5; ++c) {
        cls_lo[c] = run_r;
        run_r += (int64_t)hstats[1 + c];
        cls_hi[c] = run_r;
        if (hstats[1 + c]) Wmax = 1 << c;
    }
    const int64_t lo = std::min<int64_t>(opt.root_lo, ncand);
    const int64_t hi = opt.root_hi < 0 ? ncand : std::min<int64_t>(opt.root_hi, ncand);
    // candidates of degree above 64 * 16 rank after every class: the wide search takes them
    // (with the candidate pruning, it takes every top-level candidate)
    WideRange wr;
    wr.lo = std::max<int64_t>(run_r, lo);
    wr.hi = std::min<int64_t>(run_r + (int64_t)hstats[6] + (int64_t)hstats[7], hi);
    wr.Wx = (int)((hstats[8] + 63) / 64);
    int32_t *twin = nullptr;
    if (opt.prune) {
        wr.lo = lo;
        wr.hi = hi;
        for (int c = 0; c < 5; ++c) cls_lo[c] = cls_hi[c] = 0;
    }
    if (opt.prune == 1) {
        // twins: candidates with equal rows, found by a sort of row keys; twin[v] = the lowest
        // rank with v's row
        const size_t b_k = align_up((size_t)nc * 8, 256), b_v = align_up((size_t)nc * 4, 256);
        char *tw = nullptr;
        MBE_CALL(mem(st->twin, 2 * b_k + 3 * b_v, &tw));
        unsigned long long *tkey = reinterpret_cast<unsigned long long *>(tw);
        unsigned long long *tkey2 = reinterpret_cast<unsigned long long *>(tw + b_k);
        unsigned int *tval = reinterpret_cast<unsigned int *>(tw + 2 * b_k);
        unsigned int *tval2 = reinterpret_cast<unsigned int *>(tw + 2 * b_k + b_v);
        twin = reinterpret_cast<int32_t *>(tw + 2 * b_k + 2 * b_v);
        MBE_TRY(launch_row_keys(nc, c_off, c_adj, tkey, tval, s));
        size_t tb_bytes = 0;
        MBE_TRY(sort_pairs_u64_u32(nullptr, &tb_bytes, tkey, tkey2, tval, tval2, nc, s));
        char *ttmp = nullptr;
        if (fx) {
            MBE_CALL(mem(st->sort_tmp, tb_bytes, &ttmp));
        } else {
            // (the ranking's sort temporaries are done with)
            MBE_TRY(st->sort_tmp.ensure(tb_bytes));
            ttmp = st->sort_tmp.as<char>();
            tb_bytes = st->sort_tmp.bytes;
        }
        MBE_TRY(sort_pairs_u64_u32(ttmp, &tb_bytes, tkey, tkey2, tval, tval2, nc, s));
        MBE_TRY(launch_twins(nc, tkey2, tval2, c_off, c_adj, rank, twin, s));
    }

    const int waves = opt.waves;
    const int grid = opt.grid > 0 ? opt.grid : 0;  // 0: occupancy-sized per class
    SearchDims dims{};
    dims.nwords = (ncand + 63) / 64;
    dims.Wmax = Wmax;
    dims.waves = waves;
    dims.ucap = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ncand, (int64_t)hstats[9]));
    dims.scap = 4 * (int64_t)dims.ucap + 16384;
    dims.maxdepth = 64 * Wmax + 2;

    if (ws_out) {
        int64_t cls_a[5], cls_b[5];
        for (int c = 0; c < 5; ++c) {
            cls_a[c] = std::max(cls_lo[c], lo);
            cls_b[c] = std::min(cls_hi[c], hi);
        }
        size_t bytes = 4096 + 2 * b_keys + 2 * b_i32 + tmp_bytes;
        if (!g->on_device)
            bytes += align_up(((size_t)nu + 1) * 4, 256) + align_up(((size_t)nv + 1) * 4, 256) +
                     2 * align_up((size_t)ne * 4, 256);
        *ws_out = bytes + search_footprint(st, dims, cls_a, cls_b, opt.diag, enumerate, grid, waves, wr);
        return MBE_OK;
    }

    // record arena for mbe_enumerate
    unsigned long long rec_cap = 0, offs_cap = 0;
    if (enumerate) {
        rec_cap = ucap_ints;
        offs_cap = ucap_ints / 4 + 1;
        MBE_TRY(st->rec.ensure((size_t)rec_cap * 4 + 256));
        MBE_TRY(st->rec_offs.ensure((size_t)offs_cap * 8));
    }

    // one graph descriptor, in the small device block
    GraphDesc gd{};
    gd.order = order;
    gd.acc = acc;
    gd.total_fw = 2ull * (unsigned long long)ncand + (unsigned long long)ne;
    gd.ncand = ncand;
    gd.nwords = dims.nwords;
    gd.c_is_v = c_is_v ? 1 : 0;
    gd.cbase = 0;
    gd.obase = 0;
    GraphDesc *d_gd = reinterpret_cast<GraphDesc *>(small + 2048);
    MBE_TRY(hipMemcpyAsync(d_gd, &gd, sizeof(gd), hipMemcpyHostToDevice, s));

    SearchArgs a{};
    a.twin = twin;
    a.pivot = opt.prune == 2 ? 1 : 0;
    a.steal_on = opt.steal_k >= 2 ? 1 : 0;
    a.k3 = opt.steal_k >= 3 ? 1 : 0;
    a.c_off = c_off;
    a.c_adj = c_adj;
    a.o_off = o_off;
    a.o_adj = o_adj;
    a.rank = rank;
    a.graphs = d_gd;
    a.tasks = nullptr;
    a.acc = acc;
    a.flags = flags;
    a.rec = enumerate ? st->rec.as<int32_t>() : nullptr;
    a.rec_cap = rec_cap;
    a.rec_offs = enumerate ? st->rec_offs.as<unsigned long long>() : nullptr;
    a.rec_offs_cap = offs_cap;

    unsigned long long hacc[ACC_SLOTS];
    unsigned int hflags = 0;
    float ms = 0.f;
    int64_t cls_a[5], cls_b[5];
    for (int c = 0; c < 5; ++c) {
        cls_a[c] = std::max(cls_lo[c], lo);
        cls_b[c] = std::min(cls_hi[c], hi);
    }
    {
        int attempts = 0;
        const int rc = run_search(st, a, dims, cls_a, cls_b, opt.diag, enumerate, opt.tb, grid, waves, acc, ACC_SLOTS * 8, hacc,
                                  &hflags, &ms, s, nullptr, 0, &attempts, small, fx, wr, loads);
        out->attempts = (uint32_t)attempts;
        if (rc != MBE_OK) return rc;
    }

    out->count = hacc[ACC_COUNT];
    out->hash = hacc[ACC_HASH];
    out->out_ints = hacc[ACC_OUT_INTS];
    out->nodes = hacc[ACC_NODES];
    out->nonmaximal = hacc[ACC_NONMAX];
    out->bytes_alg = hacc[ACC_BYTES];
    out->max_depth = (uint32_t)hacc[ACC_MAX_DEPTH];
    out->kernel_ms = ms;
    for (int q = 0; q < PH_COUNT; ++q) out->phase_cycles[q] = hacc[ACC_PHASE + q];
    out->shared_chunks = hacc[ACC_SHARED];
    out->bytes_design = hacc[ACC_DBYTES];

    if (!enumerate) return MBE_OK;
    if ((hflags & FLAG_RECORD_OVERFLOW) || out->out_ints > ucap_ints) return MBE_ERR_BUFFER_TOO_SMALL;
    const unsigned long long n_rec = hacc[ACC_RECORDS];
    if (n_rec == 0) return MBE_OK;
    MBE_TRY(st->rec_tmp.ensure((size_t)n_rec * 8));
    MBE_TRY(st->rec_lens.ensure((size_t)n_rec * 8));
    size_t canon_bytes = 0;
    MBE_TRY(canonical_records(st->rec.as<int32_t>(), st->rec_offs.as<unsigned long long>(), n_rec,
                              st->rec_tmp.as<unsigned long long>(), st->rec_lens.as<unsigned long long>(), nullptr,
                              nullptr, &canon_bytes, s));
    MBE_TRY(st->canon_tmp.ensure(canon_bytes));
    canon_bytes = st->canon_tmp.bytes;
    int32_t *dst = ubuf;
    if (!ubuf_on_device) {
        MBE_TRY(st->out_tmp.ensure((size_t)out->out_ints * 4));
        dst = st->out_tmp.as<int32_t>();
    }
    MBE_TRY(canonical_records(st->rec.as<int32_t>(), st->rec_offs.as<unsigned long long>(), n_rec,
                              st->rec_tmp.as<unsigned long long>(), st->rec_lens.as<unsigned long long>(), dst,
                              st->canon_tmp.p, &canon_bytes, s));
    if (!ubuf_on_device) MBE_TRY(hipMemcpyAsync(ubuf, dst, (size_t)out->out_ints * 4, hipMemcpyDeviceToHost, s));
    MBE_TRY(hipStreamSynchronize(s));
    return MBE_OK;
}

// Arena slots of a search: concurrent class launches need no more than fit on the device at
// once or than the launches have workgroups; one class at a time, the largest of each class's
// grid and residency.  cls_grid / cls_res receive each class's grid and residency.
//
// Grids: each class gets as many workgroups as fit on the device, except that when several
// classes run side by side and the widest (launched first, so its workgroups would take every
// compute unit) has fewer than two top-level candidates per workgroup, it gets half: the
// narrower classes then start at once beside it.  On the power-law graph (578 eight-word
// candidates) that took the step from 34.1 to 32.4 ms; a quarter measured the same there, but
// halving the widest class whatever its size slowed the batched form (20.9 -> 22.5 s), whose
// widest class holds many candidates.
int search_slots(DeviceState *st, const int64_t *cls_lo, const int64_t *cls_hi, bool diag, bool enumerate, int grid,
                 int waves, int nwords, bool sequential, int *cls_grid, int *cls_res) {
    int64_t cap = 1, sum_grid = 0;
    for (int c = 0; c < 5; ++c) {
        cls_grid[c] = cls_res[c] = 0;
        if (cls_lo[c] >= cls_hi[c]) continue;
        cls_res[c] = st->cus * search_occupancy(1 << c, diag, enumerate, waves, nwords);
        cls_grid[c] = grid > 0 ? grid : cls_res[c];
        cap = std::max<int64_t>(cap, cls_res[c]);
        sum_grid += cls_grid[c];
    }
    int ncls = 0, widest = -1;
    for (int c = 0; c < 5; ++c)
        if (cls_lo[c] < cls_hi[c]) {
            ++ncls;
            widest = c;
        }
    if (grid <= 0 && !sequential && ncls >= 2 && cls_hi[widest] - cls_lo[widest] < 2 * (int64_t)cls_res[widest]) {
        sum_grid -= cls_grid[widest];
        cls_grid[widest] = std::max(1, cls_res[widest] / 2);
        sum_grid += cls_grid[widest];
    }
    int nslots = (int)std::max<int64_t>(1, std::min(cap, sum_grid));
    if (sequential) {
        nslots = 1;
        for (int c = 0; c < 5; ++c) nslots = std::max(nslots, std::min(cls_grid[c], cls_res[c]));
    }
    return nslots;
}

// Device bytes the search of a call holds: the arena slots, the slot flags and the sharing
// slots (with the capacities the device has already grown to).
// The wide search's arena layout and grid for a call: workgroups up to twice the compute units
// (or the caller's grid), at most 16 per top-level candidate, and no more than kWideArenaBytes
// (or cap, when positive) of slots.
WideLayout wide_plan(DeviceState *st, const SearchDims &dims, const WideRange &wr, int64_t wscap, int32_t wdepth,
                     int grid, int waves, size_t cap, int *wgrid) {
    WideLayout wl = wide_layout(dims, wr.Wx, wscap, wdepth, waves);
    const int64_t nroots = wr.hi - wr.lo;
    const int64_t budget = (int64_t)((cap ? cap : kWideArenaBytes) / wl.wg_bytes);
    int64_t g = std::min<int64_t>(grid > 0 ? grid : 2 * (int64_t)st->cus, nroots * 16);
    g = std::min<int64_t>(g, budget);
    *wgrid = (int)g;
    wl.reps = g > 0 ? (int)((g + nroots - 1) / nroots) : 1;
    return wl;
}

size_t search_footprint(DeviceState *st, SearchDims dims, const int64_t *cls_lo, const int64_t *cls_hi, bool diag,
                        bool enumerate, int grid, int waves, const WideRange &wr) {
    dims.scap = std::max<int64_t>(dims.scap, st->scap_floor);
    dims.maxdepth = std::max<int32_t>(dims.maxdepth, st->depth_floor);
    int cls_grid[5], cls_res[5];
    const size_t nslots = (size_t)search_slots(st, cls_lo, cls_hi, diag, enumerate, grid, waves, dims.nwords, false, cls_grid, cls_res);
    size_t bytes = search_layout(dims).wg_bytes * nslots + sizeof(unsigned int) * nslots + sizeof(StealSlot) * nslots * 5 +
                   sizeof(PubSlot) * nslots * (size_t)waves * 5;
    if (wr.lo < wr.hi) {
        int wgrid = 0;
        const WideLayout wl = wide_plan(st, dims, wr, std::max<int64_t>(st->wscap_floor, 8 * (int64_t)dims.ucap + 65536),
                                        std::max<int32_t>(st->wdepth_floor, 256), grid, waves, 0, &wgrid);
        bytes += wl.wg_bytes * (size_t)std::max(wgrid, 1) + 4 * (size_t)(wr.hi - wr.lo);
    }
    return bytes;
}

// Search run shared by the single-graph and batched calls: sizes the arena, launches one
// persistent kernel per mask-width class (widest first) and reruns with larger capacities
// when a kernel reports an overflow.  hacc / hflags receive the run-wide slots and flags.
int run_search(DeviceState *st, SearchArgs &a, SearchDims dims, const int64_t *cls_lo, const int64_t *cls_hi,
               bool diag, bool enumerate, bool tb, int grid, int waves, unsigned long long *run_acc, size_t run_acc_bytes,
               unsigned long long *hacc, unsigned int *hflags_out, float *ms, hipStream_t s,
               unsigned long long *graph_acc, size_t graph_acc_bytes, int *attempts, char *small, FixedRegion *fx,
               const WideRange &wr, std::vector<unsigned long long> *loads) {
    dims.scap = std::max<int64_t>(dims.scap, st->scap_floor);
    dims.maxdepth = std::max<int32_t>(dims.maxdepth, st->depth_floor);
    const bool wide = wr.lo < wr.hi;
    int64_t wscap = std::max<int64_t>(st->wscap_floor, 8 * (int64_t)dims.ucap + 65536);
    int32_t wdepth = std::max<int32_t>(st->wdepth_floor, 256);
    unsigned int *flags = a.flags;
    unsigned int *counters = reinterpret_cast<unsigned int *>(small + 512);
    unsigned int hflags = 0;
    // the fixed-memory form runs the classes one after another on the caller's stream (it
    // creates no streams of its own)
    if (!fx) MBE_TRY(ensure_class_streams(st));
    // persistent grids: as many workgroups per class as fit on the device at once (unless the
    // caller fixed the grid); the arena has one slot per workgroup that can be resident
    int cls_grid[5], cls_res[5];
    bool sequential = fx != nullptr;
    const size_t mark = fx ? fx->used : 0;
    for (int attempt = 0;; ++attempt) {
        int nslots = search_slots(st, cls_lo, cls_hi, diag, enumerate, grid, waves, dims.nwords, sequential, cls_grid, cls_res);
        a.dims = dims;
        a.lay = search_layout(dims);
        // per arena slot: its busy flag, and per class one top-level and `waves` third-level
        // sharing slots
        const size_t share_per_slot = sizeof(StealSlot) * 5 + sizeof(PubSlot) * (size_t)waves * 5;
        char *share = nullptr;
        // the wide search's own arena (its slots first: with fixed memory it takes up to half of
        // what is left, the classes the rest)
        SearchArgs aw{};
        int wgrid = 0;
        if (wide) {
            if (fx) fx->used = mark;
            const size_t wcap = fx ? (fx->cap - std::min(fx->cap, align_up(mark, 4096) + 4096)) / 2 : 0;
            aw.wl = wide_plan(st, dims, wr, wscap, wdepth, grid, waves, wcap, &wgrid);
            const int64_t nroots = wr.hi - wr.lo;
            if (wgrid < 1) return fx ? MBE_ERR_SCRATCH_LIMIT : MBE_ERR_OUT_OF_MEMORY;
            if (fx) {
                aw.warena = static_cast<char *>(fx->take(aw.wl.wg_bytes * (size_t)wgrid, 4096));
                aw.wide_items = static_cast<unsigned int *>(fx->take(4 * (size_t)nroots));
                if (!aw.warena || !aw.wide_items) return MBE_ERR_SCRATCH_LIMIT;
                MBE_TRY(launch_zero(aw.warena, aw.wl.wg_bytes * (size_t)wgrid, s));
            } else {
                MBE_TRY(st->warena.ensure(aw.wl.wg_bytes * (size_t)wgrid));
                MBE_TRY(st->witems.ensure(4 * (size_t)nroots));
                aw.warena = st->warena.as<char>();
                aw.wide_items = st->witems.as<unsigned int>();
            }
            MBE_TRY(launch_zero_2d(aw.warena + aw.wl.off_bitmap, aw.wl.wg_bytes, (size_t)dims.nwords * 8, (size_t)wgrid, s));
            MBE_TRY(launch_zero(aw.wide_items, 4 * (size_t)nroots, s));
        }
        if (fx) {
            // as many arena slots as fit in what the call has left of the scratch
            const size_t wmark = fx->used;
            fx->used = wide ? wmark : mark;
            const size_t start = align_up(fx->used, 4096), slack = 2 * 4096;
            const size_t left = fx->cap > start + slack ? fx->cap - start - slack : 0;
            const size_t per_slot = a.lay.wg_bytes + sizeof(unsigned int) + share_per_slot;
            const int64_t fit = (int64_t)(left / per_slot);
            if (fit < 1) return MBE_ERR_SCRATCH_LIMIT;
            nslots = (int)std::min<int64_t>(nslots, fit);
            a.arena = static_cast<char *>(fx->take(a.lay.wg_bytes * (size_t)nslots, 4096));
            a.slot_busy = static_cast<unsigned int *>(fx->take(sizeof(unsigned int) * (size_t)nslots));
            share = static_cast<char *>(fx->take(share_per_slot * (size_t)nslots));
            if (!a.arena || !a.slot_busy || !share) return MBE_ERR_SCRATCH_LIMIT;
            // the scratch holds whatever the last call left there
            MBE_TRY(launch_zero(a.arena, a.lay.wg_bytes * (size_t)nslots, s));
        } else {
            MBE_TRY(st->arena.ensure(a.lay.wg_bytes * (size_t)nslots));
            a.arena = st->arena.as<char>();
            // kernels keep their scratch bitmaps zero between uses; new memory starts zero too
            if (st->arena.fresh) MBE_TRY(launch_zero(st->arena.p, st->arena.bytes, s));
            MBE_TRY(st->slots.ensure(sizeof(unsigned int) * (size_t)nslots));
            a.slot_busy = st->slots.as<unsigned int>();
            MBE_TRY(st->steal.ensure(share_per_slot * (size_t)nslots));
            share = st->steal.as<char>();
        }
        a.nslots = nslots;
        // per class: nslots top-level slots, then nslots * waves third-level slots
        const size_t steal_bytes = sizeof(StealSlot) * (size_t)nslots * 5;
        const size_t pub_bytes = sizeof(PubSlot) * (size_t)nslots * (size_t)waves * 5;
        MBE_TRY(launch_zero_2d(a.arena + a.lay.off_bitmap, a.lay.wg_bytes, (size_t)dims.nwords * 8, (size_t)nslots, s));
        MBE_TRY(launch_zero(a.slot_busy, sizeof(unsigned int) * (size_t)nslots, s));
        MBE_TRY(launch_zero(share, steal_bytes + (a.k3 ? pub_bytes : 0), s));
        MBE_TRY(launch_zero(run_acc, run_acc_bytes, s));
        if (graph_acc && graph_acc != run_acc) MBE_TRY(launch_zero(graph_acc, graph_acc_bytes, s));
        MBE_TRY(launch_zero(flags, 4, s));
        MBE_TRY(launch_zero(counters, 64 * 4, s));
        // load records (tally runs that ask for them): 3 u64 per workgroup of every launch
        std::vector<std::pair<int, int64_t>> load_launch;  // (mask words, 0 = wide; workgroups)
        unsigned long long *load_buf = nullptr;
        int64_t load_n = 0;
        if (loads && tb && !fx) {
            for (int c = 4; c >= 0; --c)
                if (cls_lo[c] < cls_hi[c]) load_n += cls_grid[c];
            if (wide) load_n += wgrid;
            MBE_TRY(st->loads.ensure(24 * (size_t)std::max<int64_t>(load_n, 1)));
            load_buf = st->loads.as<unsigned long long>();
            MBE_TRY(launch_zero(load_buf, 24 * (size_t)std::max<int64_t>(load_n, 1), s));
        }
        int64_t load_off = 0;
        MBE_TRY(hipEventRecord(st->ev0, s));
        if (!sequential) MBE_TRY(hipEventRecord(st->fork, s));
        for (int c = 4; c >= 0; --c) {
            if (cls_lo[c] >= cls_hi[c]) continue;
            SearchArgs ac = a;
            ac.steal = reinterpret_cast<StealSlot *>(share) + (size_t)c * nslots;
            ac.steal_live = counters + 8 + c;
            ac.pub = reinterpret_cast<PubSlot *>(share + steal_bytes) + (size_t)c * nslots * (size_t)waves;
            ac.pubw = waves;
            ac.pub_live = counters + 16 + c;
            ac.busy = counters + 24 + c;
            ac.hungry = counters + 32 + c;
            ac.epoch_ctr = counters + 40 + c;
            ac.cls = c;
            ac.cls_ctr = counters;
            for (int q = 0; q < 5; ++q) ac.cls_n[q] = std::max<int64_t>(0, cls_hi[q] - cls_lo[q]);
            hipStream_t cs = s;
            if (!sequential) {
                cs = st->cls_stream[c];
                MBE_TRY(hipStreamWaitEvent(cs, st->fork, 0));
            }
            // (with fixed memory the grid is at most the slots that fit)
            const int gsz = fx ? std::min(cls_grid[c], nslots) : cls_grid[c];
            if (load_buf) {
                ac.wg_load = load_buf + 3 * load_off;
                load_launch.push_back({1 << c, gsz});
                load_off += gsz;
            }
            MBE_TRY(launch_search(ac, 1 << c, diag, enumerate, tb, cls_lo[c], cls_hi[c], counters + c, gsz, waves, cs));
            if (!sequential) {
                MBE_TRY(hipEventRecord(st->join[c], cs));
                MBE_TRY(hipStreamWaitEvent(s, st->join[c], 0));
            }
        }
        if (wide) {
            // the wide top-level candidates, after the classes, on the call's stream
            SearchArgs ac = a;
            ac.warena = aw.warena;
            ac.wl = aw.wl;
            ac.wide_items = aw.wide_items;
            if (load_buf) {
                ac.wg_load = load_buf + 3 * load_off;
                load_launch.push_back({0, wgrid});
                load_off += wgrid;
            }
            MBE_TRY(launch_wide(ac, diag, enumerate, tb, wr.lo, wr.hi, counters + 5, wgrid, waves, s,
                                a.twin != nullptr ? 1 : (a.pivot ? 2 : 0)));
        }
        MBE_TRY(hipEventRecord(st->ev1, s));
        MBE_TRY(hipMemcpyAsync(hacc, run_acc, ACC_SLOTS * 8, hipMemcpyDeviceToHost, s));
        MBE_TRY(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, s));
        MBE_TRY(hipStreamSynchronize(s));
        MBE_TRY(hipEventElapsedTime(ms, st->ev0, st->ev1));
        if (hflags & FLAG_SHARE_MISMATCH) return MBE_ERR_DEVICE;
        if (attempts) *attempts = attempt + 1;
        if (!(hflags & FLAG_RERUN)) {
            if (load_buf) {
                std::vector<unsigned long long> raw(3 * (size_t)load_off);
                MBE_TRY(hipMemcpy(raw.data(), load_buf, raw.size() * 8, hipMemcpyDeviceToHost));
                loads->clear();
                int64_t at = 0;
                for (const auto &l : load_launch)
                    for (int64_t b = 0; b < l.second; ++b, ++at) {
                        if (raw[3 * at] == 0) continue;  // a workgroup that found no arena slot
                        loads->push_back((unsigned long long)l.first);
                        loads->push_back(raw[3 * at]);
                        loads->push_back(raw[3 * at + 1]);
                        loads->push_back(raw[3 * at + 2]);
                    }
            }
            break;
        }
        if (attempt >= 8) return MBE_ERR_OUT_OF_MEMORY;
        if (hflags & FLAG_NO_SLOT) sequential = true;
        if (hflags & FLAG_STACK_OVERFLOW) {
            dims.scap = std::min<int64_t>(dims.scap * 2, (int64_t)1 << 31);
            wscap = std::min<int64_t>(wscap * 2, (int64_t)1 << 31);
        }
        if (hflags & FLAG_DEPTH_OVERFLOW) {
            dims.maxdepth *= 2;
            wdepth *= 2;
        }
        if (hflags & FLAG_UNIVERSE_OVERFLOW) {
            dims.ucap = (int32_t)std::max<int64_t>(dims.ucap, (int64_t)hacc[ACC_NEED_UCAP]);
            dims.scap = std::max<int64_t>(dims.scap, 4 * (int64_t)dims.ucap + 16384);
        }
    }
    st->scap_floor = std::max<int64_t>(st->scap_floor, dims.scap);
    st->depth_floor = std::max<int32_t>(st->depth_floor, dims.maxdepth);
    if (wide) {
        st->wscap_floor = std::max<int64_t>(st->wscap_floor, wscap);
        st->wdepth_floor = std::max<int32_t>(st->wdepth_floor, wdepth);
    }
    *hflags_out = hflags;
    return MBE_OK;
}

int degree_class(int64_t d) {
    int c = 0;
    while (c < 6 && d > (64ll << c)) ++c;
    return c;
}

// Host checks of batch input (before any device work): sizes, pointers and, unless the
// caller vouches for them, the CSR pairs.
int check_graphs(const mbe_graph *gs, int32_t n, bool validate) {
    for (int32_t i = 0; i < n; ++i) {
        const mbe_graph &g = gs[i];
        if (g.n_u < 0 || g.n_v < 0 || g.n_edges < 0 || g.on_device) return MBE_ERR_INVALID_ARG;
        if (g.n_edges > 0 && (g.n_u == 0 || g.n_v == 0)) return MBE_ERR_INVALID_GRAPH;
        if ((g.n_u > 0 && !g.u_off) || (g.n_v > 0 && !g.v_off) || (g.n_edges > 0 && (!g.u_adj || !g.v_adj)))
            return MBE_ERR_INVALID_ARG;
        if (validate && g.u_off && g.v_off &&
            !host_valid_pair(g.n_u, g.n_v, g.n_edges, g.u_off, g.u_adj, g.v_off, g.v_adj))
            return MBE_ERR_INVALID_GRAPH;
    }
    return MBE_OK;
}

// Packed sizes of a batch, summed in 64 bits before anything is packed: the packed candidate
// and other-side ids and the edge offsets are int32, so a batch whose totals do not fit is
// refused (MBE_ERR_INVALID_ARG) before any allocation or device work.
int batch_totals(const mbe_graph *gs, int32_t n, int side_opt, int64_t *nc_tot, int64_t *no_tot, int64_t *e_tot) {
    int64_t NC = 0, NO = 0, E = 0;
    for (int32_t i = 0; i < n; ++i) {
        const mbe_graph &g = gs[i];
        if (g.n_edges == 0) continue;
        const int sd = side_opt ? side_opt : (g.n_v < g.n_u ? 2 : 1);
        NC += sd == 2 ? g.n_v : g.n_u;
        NO += sd == 2 ? g.n_u : g.n_v;
        E += g.n_edges;
        if (NC >= INT32_MAX || NO >= INT32_MAX || E > INT32_MAX) return MBE_ERR_INVALID_ARG;
    }
    if (nc_tot) *nc_tot = NC;
    if (no_tot) *no_tot = NO;
    if (e_tot) *e_tot = E;
    return MBE_OK;
}

// The batched pass on a given workspace and stream (the caller holds the workspace and has
// run check_graphs).
int run_batch_on(DeviceState *st, hipStream_t s, const mbe_graph *gs, int32_t n, const mbe_options *opt_in,
                 mbe_result *outs, const unsigned int *cancel = nullptr);

int run_batch(const mbe_graph *gs, int32_t n, const mbe_options *opt_in, mbe_result *outs) {
    if (n < 0 || (n > 0 && (!gs || !outs))) return MBE_ERR_INVALID_ARG;
    const Opts opt = read_opts(opt_in);
    if (opt.prune || opt.ws) return MBE_ERR_INVALID_ARG;
    if (opt.side < 0 || opt.side > 2 || opt.waves < 1 || opt.waves > 8 ||
        opt.steal_k < 1 || opt.steal_k > 3)
        return MBE_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i) std::memset(&outs[i], 0, sizeof(outs[i]));
    const int rc = check_graphs(gs, n, !opt.no_validate);
    if (rc != MBE_OK) return rc;
    MBE_CALL(batch_totals(gs, n, opt.side, nullptr, nullptr, nullptr));
    bool any = false;
    for (int32_t i = 0; i < n; ++i) any = any || (gs[i].n_edges > 0);
    if (!any) {
        for (int32_t i = 0; i < n; ++i) outs[i].side = (uint32_t)(opt.side ? opt.side : (gs[i].n_v < gs[i].n_u ? 2 : 1));
        return MBE_OK;
    }
    int dev = 0;
    MBE_TRY(hipGetDevice(&dev));
    DeviceState *st = state_for(dev);
    if (!st) return MBE_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(st->mu);
    return run_batch_on(st, opt.stream, gs, n, opt_in, outs);
}

int run_batch_on(DeviceState *st, hipStream_t s, const mbe_graph *gs, int32_t n, const mbe_options *opt_in,
                 mbe_result *outs, const unsigned int *cancel) {
    if (n < 0 || (n > 0 && (!gs || !outs))) return MBE_ERR_INVALID_ARG;
    Opts opt = read_opts(opt_in);
    if (opt.side < 0 || opt.side > 2 || opt.waves < 1 || opt.waves > 8 ||
        opt.steal_k < 1 || opt.steal_k > 3)
        return MBE_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i) std::memset(&outs[i], 0, sizeof(outs[i]));
    // host checks and packing (each graph keeps its own candidate side); totals are checked in
    // 64 bits before anything is packed
    MBE_CALL(batch_totals(gs, n, opt.side, nullptr, nullptr, nullptr));
    std::vector<int32_t> side(n), nc(n), no(n);
    std::vector<int64_t> cb(n + 1, 0), ob(n + 1, 0), eb(n + 1, 0);
    int64_t NC = 0, NO = 0, E = 0;
    int max_no = 1;
    for (int32_t i = 0; i < n; ++i) {
        const mbe_graph &g = gs[i];
        side[i] = opt.side ? opt.side : (g.n_v < g.n_u ? 2 : 1);
        outs[i].side = (uint32_t)side[i];
        nc[i] = side[i] == 2 ? g.n_v : g.n_u;
        no[i] = side[i] == 2 ? g.n_u : g.n_v;
        if (g.n_edges == 0) nc[i] = no[i] = 0;  // nothing to search: keep it out of the pack
    }
    for (int32_t i = 0; i < n; ++i) {
        cb[i + 1] = cb[i] + nc[i];
        ob[i + 1] = ob[i] + no[i];
        eb[i + 1] = eb[i] + (nc[i] ? gs[i].n_edges : 0);
        max_no = std::max(max_no, no[i]);
    }
    NC = cb[n];
    NO = ob[n];
    E = eb[n];
    if (NC == 0) return MBE_OK;
    std::vector<int32_t> c_off(NC + 1), o_off(NO + 1), c_adj(E), o_adj(E), graph_of(NC);
    int64_t cls_cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<int64_t> ncand_h(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (!nc[i]) continue;
        const mbe_graph &g = gs[i];
        const bool cv = side[i] == 2;
        const int32_t *go = cv ? g.v_off : g.u_off, *ga = cv ? g.v_adj : g.u_adj;
        const int32_t *ho = cv ? g.u_off : g.v_off, *ha = cv ? g.u_adj : g.v_adj;
        for (int32_t v = 0; v < nc[i]; ++v) {
            c_off[cb[i] + v] = (int32_t)(eb[i] + go[v]);
            graph_of[cb[i] + v] = i;
            const int64_t d = go[v + 1] - go[v];
            if (d > 0) {
                ++ncand_h[i];
                ++cls_cnt[degree_class(d)];
            }
        }
        for (int32_t w = 0; w < no[i]; ++w) o_off[ob[i] + w] = (int32_t)(eb[i] + ho[w]);
        for (int32_t e = 0; e < g.n_edges; ++e) {
            c_adj[eb[i] + e] = ga[e] + (int32_t)ob[i];
            o_adj[eb[i] + e] = ha[e] + (int32_t)cb[i];
        }
    }
    c_off[NC] = (int32_t)E;
    o_off[NO] = (int32_t)E;

    // device copies: graph | prep | per-graph accumulators
    auto al = [](size_t b) { return align_up(b, 256); };
    const size_t b_coff = al((NC + 1) * 4), b_ooff = al((NO + 1) * 4), b_adj = al(E * 4), b_nc = al(NC * 4);
    const size_t b_cb = al((n + 1) * 4);
    MBE_TRY(st->graph.ensure(b_coff + b_ooff + 2 * b_adj + b_nc + b_cb));
    int32_t *d_coff = st->graph.as<int32_t>(0);
    int32_t *d_ooff = st->graph.as<int32_t>(b_coff);
    int32_t *d_cadj = st->graph.as<int32_t>(b_coff + b_ooff);
    int32_t *d_oadj = st->graph.as<int32_t>(b_coff + b_ooff + b_adj);
    int32_t *d_gof = st->graph.as<int32_t>(b_coff + b_ooff + 2 * b_adj);
    int32_t *d_cb = st->graph.as<int32_t>(b_coff + b_ooff + 2 * b_adj + b_nc);
    MBE_TRY(hipMemcpyAsync(d_coff, c_off.data(), (NC + 1) * 4, hipMemcpyHostToDevice, s));
    MBE_TRY(hipMemcpyAsync(d_ooff, o_off.data(), (NO + 1) * 4, hipMemcpyHostToDevice, s));
    if (E) MBE_TRY(hipMemcpyAsync(d_cadj, c_adj.data(), E * 4, hipMemcpyHostToDevice, s));
    if (E) MBE_TRY(hipMemcpyAsync(d_oadj, o_adj.data(), E * 4, hipMemcpyHostToDevice, s));
    MBE_TRY(hipMemcpyAsync(d_gof, graph_of.data(), NC * 4, hipMemcpyHostToDevice, s));
    std::vector<int32_t> cb32(cb.begin(), cb.end());  // (the totals fit int32: checked above)
    MBE_TRY(hipMemcpyAsync(d_cb, cb32.data(), (n + 1) * 4, hipMemcpyHostToDevice, s));

    int64_t NT = 0;
    std::vector<int32_t> tb(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) tb[i + 1] = tb[i] + (int32_t)ncand_h[i];
    NT = tb[n];
    const size_t b_keys = al(NC * 8), b_i32 = al(NC * 4), b_t = al(std::max<int64_t>(NT, 1) * 8),
                 b_tk = al(std::max<int64_t>(NT, 1) * 4), b_gs = al((size_t)n * 16), b_gd = al((size_t)n * sizeof(GraphDesc)),
                 b_ga = al((size_t)n * ACC_SLOTS * 8), b_tb = al((n + 1) * 4);
    MBE_TRY(st->prep.ensure(2 * b_keys + 2 * b_i32 + 2 * b_t + 2 * b_tk + b_gs + b_gd + b_ga + b_tb));
    size_t po = 0;
    auto take = [&](size_t b) { const size_t at = po; po += b; return at; };
    unsigned long long *keys = st->prep.as<unsigned long long>(take(b_keys));
    unsigned long long *sorted = st->prep.as<unsigned long long>(take(b_keys));
    int32_t *order = st->prep.as<int32_t>(take(b_i32));
    int32_t *rank = st->prep.as<int32_t>(take(b_i32));
    unsigned long long *task = st->prep.as<unsigned long long>(take(b_t));
    unsigned long long *task_sorted = st->prep.as<unsigned long long>(take(b_t));
    unsigned int *tkey = st->prep.as<unsigned int>(take(b_tk));
    unsigned int *tkey_sorted = st->prep.as<unsigned int>(take(b_tk));
    unsigned long long *gstats = st->prep.as<unsigned long long>(take(b_gs));
    GraphDesc *d_gd = st->prep.as<GraphDesc>(take(b_gd));
    unsigned long long *gacc = st->prep.as<unsigned long long>(take(b_ga));
    int32_t *d_tb = st->prep.as<int32_t>(take(b_tb));
    MBE_TRY(st->small.ensure(4096));
    unsigned long long *acc = st->small.as<unsigned long long>(0);
    unsigned int *flags = st->small.as<unsigned int>(256);
    unsigned long long *stats = st->small.as<unsigned long long>(1024);
    MBE_TRY(hipMemcpyAsync(d_tb, tb.data(), (n + 1) * 4, hipMemcpyHostToDevice, s));
    MBE_TRY(launch_zero(gstats, (size_t)n * 16, s));
    MBE_TRY(launch_zero(stats, 16 * 8, s));
    MBE_TRY(launch_batch_keys((int32_t)NC, d_coff, d_cadj, d_ooff, d_gof, d_cb, keys, gstats, stats, s));
    int end_bit = 32;
    while (end_bit < 64 && ((unsigned long long)max_no >> (end_bit - 32)) != 0ull) ++end_bit;
    size_t tmp = 0;
    MBE_TRY(segmented_sort_u64(nullptr, &tmp, keys, sorted, (int32_t)NC, n, d_cb, d_cb + 1, end_bit, s));
    size_t tmp2 = 0;
    MBE_TRY(sort_pairs_u32_u64(nullptr, &tmp2, tkey, tkey_sorted, task, task_sorted, (int32_t)NT, 14, s));
    MBE_TRY(st->sort_tmp.ensure(std::max(tmp, tmp2)));
    tmp = st->sort_tmp.bytes;
    MBE_TRY(segmented_sort_u64(st->sort_tmp.p, &tmp, keys, sorted, (int32_t)NC, n, d_cb, d_cb + 1, end_bit, s));
    std::vector<unsigned long long> hg((size_t)n * 2);
    unsigned long long hstats[16];
    MBE_TRY(hipMemcpyAsync(hg.data(), gstats, (size_t)n * 16, hipMemcpyDeviceToHost, s));
    MBE_TRY(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
    MBE_TRY(launch_batch_scatter((int32_t)NC, sorted, d_gof, d_cb, gstats, order, rank, tkey, task, d_tb, s));
    tmp = st->sort_tmp.bytes;
    MBE_TRY(sort_pairs_u32_u64(st->sort_tmp.p, &tmp, tkey, tkey_sorted, task, task_sorted, (int32_t)NT, 14, s));
    MBE_TRY(hipStreamSynchronize(s));

    // descriptors and capacities
    std::vector<GraphDesc> gd(n);
    int64_t ucap = 1, maxc = 1;
    for (int32_t i = 0; i < n; ++i) {
        GraphDesc &d = gd[i];
        std::memset(&d, 0, sizeof(d));
        d.order = order + cb[i];
        d.acc = gacc + (size_t)i * ACC_SLOTS;
        d.ncand = (int32_t)ncand_h[i];
        d.total_fw = 2ull * (unsigned long long)ncand_h[i] + (unsigned long long)(eb[i + 1] - eb[i]);
        d.nwords = (int32_t)((ncand_h[i] + 63) / 64);
        d.c_is_v = side[i] == 2 ? 1 : 0;
        d.cbase = (int32_t)cb[i];
        d.obase = (int32_t)ob[i];
        ucap = std::max<int64_t>(ucap, std::min<int64_t>(ncand_h[i], (int64_t)hg[2 * i + 1]));
        maxc = std::max<int64_t>(maxc, ncand_h[i]);
    }
    MBE_TRY(hipMemcpyAsync(d_gd, gd.data(), (size_t)n * sizeof(GraphDesc), hipMemcpyHostToDevice, s));
    int Wmax = 1;
    int64_t cls_lo[5], cls_hi[5], run_t = 0;
    for (int c = 0; c < 5; ++c) {
        cls_lo[c] = run_t;
        run_t += cls_cnt[c];
        cls_hi[c] = run_t;
        if (cls_cnt[c]) Wmax = 1 << c;
    }
    SearchDims dims{};
    dims.nwords = (int32_t)((maxc + 63) / 64);
    dims.Wmax = Wmax;
    dims.waves = opt.waves;
    dims.ucap = (int32_t)ucap;
    dims.scap = 4 * ucap + 16384;
    dims.maxdepth = 64 * Wmax + 2;
    const int grid = opt.grid > 0 ? opt.grid : 0;  // 0: occupancy-sized per class

    SearchArgs a{};
    a.steal_on = opt.steal_k >= 2 ? 1 : 0;
    a.k3 = opt.steal_k >= 3 ? 1 : 0;
    a.c_off = d_coff;
    a.c_adj = d_cadj;
    a.o_off = d_ooff;
    a.o_adj = d_oadj;
    a.rank = rank;
    a.graphs = d_gd;
    a.tasks = task_sorted;
    a.acc = acc;
    a.flags = flags;
    a.cancel = cancel;
    unsigned long long hacc[ACC_SLOTS];
    unsigned int hflags = 0;
    float ms = 0.f;
    int attempts = 0;
    WideRange wr;
    wr.lo = run_t;
    wr.hi = run_t + cls_cnt[5] + cls_cnt[6];
    wr.Wx = (int)((hstats[8] + 63) / 64);
    int rc = run_search(st, a, dims, cls_lo, cls_hi, opt.diag, false, opt.tb, grid, opt.waves, acc, ACC_SLOTS * 8, hacc, &hflags,
                        &ms, s, gacc, (size_t)n * ACC_SLOTS * 8, &attempts, st->small.as<char>(), nullptr, wr);
    if (rc != MBE_OK) return rc;
    std::vector<unsigned long long> hga((size_t)n * ACC_SLOTS);
    MBE_TRY(hipMemcpyAsync(hga.data(), gacc, hga.size() * 8, hipMemcpyDeviceToHost, s));
    MBE_TRY(hipStreamSynchronize(s));
    for (int32_t i = 0; i < n; ++i) {
        const unsigned long long *q = &hga[(size_t)i * ACC_SLOTS];
        outs[i].count = q[ACC_COUNT];
        outs[i].hash = q[ACC_HASH];
        outs[i].out_ints = q[ACC_OUT_INTS];
        outs[i].nodes = q[ACC_NODES];
        outs[i].nonmaximal = q[ACC_NONMAX];
        outs[i].bytes_alg = q[ACC_BYTES];
        outs[i].max_depth = (uint32_t)q[ACC_MAX_DEPTH];
        outs[i].kernel_ms = ms;
        for (int ph = 0; ph < PH_COUNT; ++ph) outs[i].phase_cycles[ph] = q[ACC_PHASE + ph];
        outs[i].shared_chunks = hacc[ACC_SHARED];  // (the whole call's)
        outs[i].attempts = (uint32_t)attempts;
        outs[i].bytes_design = q[ACC_DBYTES];
    }
    return MBE_OK;
}

// ------------------------------------------------------------------------------ serving
//
// Continuous batching: requests are queued as they arrive; each of the server's slots (a
// worker thread with its own stream and device workspace, kept between batches) takes the
// queued requests in arrival order while their estimated device footprint fits the slot's
// share of the memory budget, runs them as one batched pass, and posts the results.  With
// two or more slots a batch starts while the previous one is still on the device, so
// requests that arrive during a run are admitted as soon as a slot and memory free up.

using Clock = std::chrono::steady_clock;

struct ServerRequest {
    uint64_t ticket = 0;
    std::vector<int32_t> u_off, u_adj, v_off, v_adj;
    mbe_graph g{};
    size_t csr_bytes = 0, arena_bytes = 0;
    Clock::time_point arrival, finish, deadline;
    bool has_deadline = false;
    mbe_result result{};
    int rc = 0;
    bool done = false;
    // on the device: the slot and position in its batch (their cancel word); stop: the
    // return code (timeout or cancelled) it ends with, 0 while it is wanted
    int slot = -1, pos = -1;
    int stop = 0;
};

void free_state(DeviceState *st) {
    DevBuf *bufs[] = {&st->graph, &st->prep, &st->sort_tmp, &st->arena, &st->small, &st->steal, &st->slots, &st->warena,
                      &st->witems, &st->loads, &st->twin, &st->rec,
                      &st->rec_offs, &st->rec_tmp, &st->rec_lens, &st->canon_tmp, &st->out_tmp};
    for (DevBuf *b : bufs)
        if (b->p) {
            (void)hipFree(b->p);
            b->p = nullptr;
            b->bytes = 0;
        }
    if (st->ev0) (void)hipEventDestroy(st->ev0);
    if (st->ev1) (void)hipEventDestroy(st->ev1);
    if (st->fork) {
        (void)hipEventDestroy(st->fork);
        for (int c = 0; c < 5; ++c) {
            (void)hipEventDestroy(st->join[c]);
            (void)hipStreamDestroy(st->cls_stream[c]);
        }
    }
}

}  // namespace

struct mbe_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<ServerRequest>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<ServerRequest>> live;
    uint64_t next_ticket = 1;
    bool stopping = false;
    size_t slot_budget = 0;
    int max_batch = 4096;
    int64_t small_edges = 1 << 16;  // slot 0 takes only requests this small (when slots >= 2)
    int nslots = 1;
    int device = 0;
    int cus = 256;
    mbe_options search{};
    double timeout_ms = 0.0;  // default deadline of a request (0: none)
    std::vector<std::thread> workers;
    std::thread watchdog;
    std::condition_variable cv_deadline;
    std::vector<DeviceState *> states;
    std::vector<hipStream_t> streams;
    std::vector<unsigned int *> cancel;      // per slot, max_batch words of pinned host memory
    std::vector<unsigned int *> cancel_dev;  // the same words' device addresses
    uint64_t batches = 0, served = 0;

    // End a request that will not be run or whose run no longer counts (mu held): one still
    // queued leaves the queue and is done at once; one on the device has its cancel word set
    // and ends when its batch does.
    void stop_request(const std::shared_ptr<ServerRequest> &r, int why) {
        if (r->done || r->stop) return;
        r->stop = why;
        if (r->slot < 0) {
            for (auto it = pending.begin(); it != pending.end(); ++it)
                if (it->get() == r.get()) {
                    pending.erase(it);
                    break;
                }
            r->rc = why;
            r->result.status = why;
            r->finish = Clock::now();
            r->done = true;
            std::vector<int32_t>().swap(r->u_adj);
            std::vector<int32_t>().swap(r->v_adj);
            cv_done.notify_all();
        } else {
            __atomic_store_n(&cancel[r->slot][r->pos], 1u, __ATOMIC_RELEASE);
        }
    }

    // Ends the requests that passed their deadline, sleeping until the next one.
    void watch() {
        std::unique_lock<std::mutex> lk(mu);
        while (!stopping) {
            const Clock::time_point now = Clock::now();
            Clock::time_point next = Clock::time_point::max();
            for (auto &kv : live) {
                const std::shared_ptr<ServerRequest> &r = kv.second;
                if (!r->has_deadline || r->done || r->stop) continue;
                if (r->deadline <= now) stop_request(r, MBE_ERR_TIMEOUT);
                else next = std::min(next, r->deadline);
            }
            if (next == Clock::time_point::max()) cv_deadline.wait(lk);
            else cv_deadline.wait_until(lk, next);
        }
    }

    // device bytes a request adds: its CSR and preparation arrays, and the search arena its
    // largest local universe needs (the arena is shared by a batch, so only its maximum counts)
    void estimate(ServerRequest &r) const {
        const mbe_graph &g = r.g;
        // the candidate side the search takes (search.side, else the smaller side)
        const bool c_is_v = search.side == 2 || (search.side == 0 && g.n_v < g.n_u);
        const int64_t nc = c_is_v ? g.n_v : g.n_u, no = c_is_v ? g.n_u : g.n_v;
        r.csr_bytes = (size_t)4 * ((size_t)g.n_u + g.n_v + 2 + 2 * (size_t)g.n_edges) + (size_t)48 * nc + 4096;
        int64_t dmax = 0;
        const int32_t *off = c_is_v ? g.v_off : g.u_off;
        for (int64_t v = 0; v < nc && off; ++v) dmax = std::max<int64_t>(dmax, off[v + 1] - off[v]);
        int64_t W = 1;
        while (64 * W < dmax && W < 16) W *= 2;
        const int waves = search.wg_waves > 0 ? search.wg_waves : 8;
        const int grid = search.grid > 0 ? search.grid : 2 * cus;
        // universe, top-level list and item tables per workgroup; stack and staging per wave
        const size_t per_wg = (size_t)nc * (size_t)(24 * W + 60) + (size_t)waves * ((size_t)nc * 24 + 65536) +
                              (size_t)no / 8 + 65536;
        r.arena_bytes = per_wg * (size_t)grid;
    }

    void worker(int slot) {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<std::shared_ptr<ServerRequest>> batch;
            {
                // slot 0 is the small-request lane when there are other slots: requests queued
                // behind a large one still start at once
                const bool small_lane = slot == 0 && nslots >= 2 && small_edges >= 0;
                auto eligible = [&](const ServerRequest &r) { return !small_lane || r.g.n_edges <= small_edges; };
                auto any_eligible = [&] {
                    for (const auto &r : pending)
                        if (eligible(*r)) return true;
                    return false;
                };
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || any_eligible(); });
                if (!any_eligible()) return;  // stopping; other slots finish the rest
                size_t csr = 0, arena = 0;
                // the packed batch indexes vertices and edges with int32
                int64_t ids = 0, edges = 0;
                for (auto it = pending.begin(); it != pending.end() && (int)batch.size() < max_batch;) {
                    const ServerRequest &r = **it;
                    if (!eligible(r)) {
                        ++it;
                        continue;
                    }
                    const size_t need = csr + r.csr_bytes + std::max(arena, r.arena_bytes);
                    if (!batch.empty() && need > slot_budget) break;
                    const int64_t ids2 = ids + (int64_t)r.g.n_u + r.g.n_v, edges2 = edges + r.g.n_edges;
                    if (!batch.empty() && (ids2 >= INT32_MAX || edges2 > INT32_MAX)) break;
                    ids = ids2;
                    edges = edges2;
                    csr += r.csr_bytes;
                    arena = std::max(arena, r.arena_bytes);
                    // its cancel word is cleared before it is marked as on the device (the
                    // previous batch of this slot has finished reading the words)
                    (*it)->slot = slot;
                    (*it)->pos = (int)batch.size();
                    cancel[slot][batch.size()] = 0u;
                    batch.push_back(*it);
                    it = pending.erase(it);
                }
            }
            std::vector<mbe_graph> gs(batch.size());
            std::vector<mbe_result> rs(batch.size());
            for (size_t i = 0; i < batch.size(); ++i) gs[i] = batch[i]->g;
            mbe_options o = search;
            o.stream = streams[slot];
            o.no_validate = 1;  // checked at submission
            const int rc = run_batch_on(states[slot], streams[slot], gs.data(), (int32_t)gs.size(), &o, rs.data(),
                                        cancel_dev[slot]);
            const Clock::time_point now = Clock::now();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (size_t i = 0; i < batch.size(); ++i) {
                    batch[i]->result = rs[i];
                    batch[i]->rc = batch[i]->stop ? batch[i]->stop : rc != MBE_OK ? rc : rs[i].status;
                    if (batch[i]->stop) batch[i]->result.status = batch[i]->stop;
                    batch[i]->finish = now;
                    batch[i]->done = true;
                    // the graph copy is no longer needed
                    std::vector<int32_t>().swap(batch[i]->u_adj);
                    std::vector<int32_t>().swap(batch[i]->v_adj);
                }
                ++batches;
                served += batch.size();
            }
            cv_done.notify_all();
        }
    }
};

namespace {

// Free the slots' device state, streams and cancel words (no worker is running).
void release_slots(mbe_server *sv) {
    for (DeviceState *st : sv->states) {
        free_state(st);
        delete st;
    }
    for (hipStream_t strm : sv->streams) (void)hipStreamDestroy(strm);
    for (unsigned int *cw : sv->cancel) (void)hipHostFree(cw);
    sv->states.clear();
    sv->streams.clear();
    sv->cancel.clear();
    sv->cancel_dev.clear();
}

int server_create(const mbe_server_options *opt, mbe_server **out) {
    if (!out) return MBE_ERR_INVALID_ARG;
    *out = nullptr;
    int slots = opt && opt->slots > 0 ? opt->slots : 2;
    if (slots > 8) return MBE_ERR_INVALID_ARG;
    std::unique_ptr<mbe_server> sv(new mbe_server());
    if (opt) {
        sv->search = opt->search;
        if (opt->max_batch > 0) sv->max_batch = opt->max_batch;
        if (opt->small_edges != 0) sv->small_edges = opt->small_edges;
        if (!(opt->request_timeout_ms >= 0.0)) return MBE_ERR_INVALID_ARG;  // (NaN too)
        sv->timeout_ms = opt->request_timeout_ms;
    }
    sv->search.root_lo = sv->search.root_hi = 0;
    if (sv->search.workspace || sv->search.workspace_bytes) return MBE_ERR_INVALID_ARG;
    if (sv->search.wg_waves < 0 || sv->search.wg_waves > 8 || sv->search.side < 0 || sv->search.side > 2 ||
        sv->search.steal_k < 0 || sv->search.steal_k > 3)
        return MBE_ERR_INVALID_ARG;
    MBE_TRY(hipGetDevice(&sv->device));
    if (hipDeviceGetAttribute(&sv->cus, hipDeviceAttributeMultiprocessorCount, sv->device) != hipSuccess || sv->cus <= 0)
        sv->cus = 256;
    size_t budget = opt ? opt->hbm_budget_bytes : 0;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        MBE_TRY(hipMemGetInfo(&free_b, &total_b));
        budget = free_b / 2;
    }
    sv->slot_budget = budget / (size_t)slots;
    sv->nslots = slots;
    for (int k = 0; k < slots; ++k) {
        // (on a failure, what the slots made so far is released)
        DeviceState *st = new DeviceState();
        st->cus = sv->cus;
        sv->states.push_back(st);
        if (hipEventCreate(&st->ev0) != hipSuccess || hipEventCreate(&st->ev1) != hipSuccess) {
            release_slots(sv.get());
            return MBE_ERR_DEVICE;
        }
        hipStream_t strm = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&strm, hipStreamNonBlocking);
        if (e != hipSuccess) {
            release_slots(sv.get());
            return map_err(e);
        }
        sv->streams.push_back(strm);
        // cancel words: fine-grained pinned host memory, which a running kernel reads
        void *cw = nullptr;
        e = hipHostMalloc(&cw, (size_t)sv->max_batch * sizeof(unsigned int), hipHostMallocCoherent | hipHostMallocMapped);
        if (e != hipSuccess) {
            release_slots(sv.get());
            return MBE_ERR_OUT_OF_MEMORY;
        }
        std::memset(cw, 0, (size_t)sv->max_batch * sizeof(unsigned int));
        sv->cancel.push_back(static_cast<unsigned int *>(cw));
        void *cwd = nullptr;
        e = hipHostGetDevicePointer(&cwd, cw, 0);
        if (e != hipSuccess) {
            release_slots(sv.get());
            return map_err(e);
        }
        sv->cancel_dev.push_back(static_cast<unsigned int *>(cwd));
    }
    mbe_server *raw = sv.get();
    for (int k = 0; k < slots; ++k) sv->workers.emplace_back([raw, k] { raw->worker(k); });
    sv->watchdog = std::thread([raw] { raw->watch(); });
    *out = sv.release();
    return MBE_OK;
}

}  // namespace

extern "C" {

int mbe_server_create(const mbe_server_options *opt, mbe_server **out) { return server_create(opt, out); }

int mbe_server_submit(mbe_server *sv, const mbe_graph *g, uint64_t *ticket) {
    if (!sv) return MBE_ERR_INVALID_ARG;
    return mbe_server_submit_timeout(sv, g, sv->timeout_ms, ticket);
}

int mbe_server_submit_timeout(mbe_server *sv, const mbe_graph *g, double timeout_ms, uint64_t *ticket) {
    if (!sv || !g || !ticket || !(timeout_ms >= 0.0)) return MBE_ERR_INVALID_ARG;
    if (g->on_device || g->n_u < 0 || g->n_v < 0 || g->n_edges < 0) return MBE_ERR_INVALID_ARG;
    if ((g->n_u > 0 && !g->u_off) || (g->n_v > 0 && !g->v_off) || (g->n_edges > 0 && (!g->u_adj || !g->v_adj)))
        return MBE_ERR_INVALID_ARG;
    {
        // a malformed graph is refused here, so it can never fail the batch it would join
        const int rc = check_graphs(g, 1, sv->search.no_validate == 0);
        if (rc != MBE_OK) return rc;
    }
    auto r = std::make_shared<ServerRequest>();
    r->arrival = Clock::now();
    if (timeout_ms > 0.0) {
        r->has_deadline = true;
        const double capped = std::min(timeout_ms, 1e12);  // (about 30 years)
        r->deadline = r->arrival + std::chrono::duration_cast<Clock::duration>(
                                       std::chrono::duration<double, std::milli>(capped));
    }
    r->u_off.assign(g->u_off ? g->u_off : nullptr, g->u_off ? g->u_off + g->n_u + 1 : nullptr);
    r->v_off.assign(g->v_off ? g->v_off : nullptr, g->v_off ? g->v_off + g->n_v + 1 : nullptr);
    r->u_adj.assign(g->u_adj ? g->u_adj : nullptr, g->u_adj ? g->u_adj + g->n_edges : nullptr);
    r->v_adj.assign(g->v_adj ? g->v_adj : nullptr, g->v_adj ? g->v_adj + g->n_edges : nullptr);
    r->g = *g;
    r->g.u_off = r->u_off.empty() ? nullptr : r->u_off.data();
    r->g.v_off = r->v_off.empty() ? nullptr : r->v_off.data();
    r->g.u_adj = r->u_adj.empty() ? nullptr : r->u_adj.data();
    r->g.v_adj = r->v_adj.empty() ? nullptr : r->v_adj.data();
    sv->estimate(*r);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) return MBE_ERR_INVALID_ARG;
        r->ticket = sv->next_ticket++;
        sv->live[r->ticket] = r;
        sv->pending.push_back(r);
    }
    sv->cv_work.notify_all();  // the small-request lane may be the one that can take it
    if (r->has_deadline) sv->cv_deadline.notify_all();
    *ticket = r->ticket;
    return MBE_OK;
}

int mbe_server_cancel(mbe_server *sv, uint64_t ticket) {
    if (!sv) return MBE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return MBE_ERR_INVALID_ARG;
    sv->stop_request(it->second, MBE_ERR_CANCELLED);
    return MBE_OK;
}

int mbe_server_wait(mbe_server *sv, uint64_t ticket, mbe_result *out, double *latency_ms) {
    if (!sv || !out) return MBE_ERR_INVALID_ARG;
    std::shared_ptr<ServerRequest> r;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->live.find(ticket);
        if (it == sv->live.end()) return MBE_ERR_INVALID_ARG;
        r = it->second;
        sv->cv_done.wait(lk, [&] { return r->done; });
        sv->live.erase(it);
    }
    *out = r->result;
    if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(r->finish - r->arrival).count();
    return r->rc;
}

int mbe_server_destroy(mbe_server *sv) {
    if (!sv) return MBE_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    sv->cv_deadline.notify_all();
    for (auto &t : sv->workers) t.join();
    if (sv->watchdog.joinable()) sv->watchdog.join();
    for (hipStream_t strm : sv->streams) (void)hipStreamSynchronize(strm);
    release_slots(sv);
    delete sv;
    return MBE_OK;
}


int mbe_count_batch(const mbe_graph *gs, int32_t n, const mbe_options *opt, mbe_result *outs) {
    return run_batch(gs, n, opt, outs);
}

int mbe_tune_batch(const mbe_graph *gs, int32_t n, const mbe_options *base, mbe_options *best, double *best_ms) {
    if (!gs || n <= 0 || !best) return MBE_ERR_INVALID_ARG;
    const mbe_options b = base ? *base : mbe_options{};
    std::vector<mbe_result> ref((size_t)n), outs((size_t)n);
    // candidates: waves per workgroup x work sharing; the first run also warms the workspace
    static const int kWaves[] = {8, 4, 2};
    static const int kSteal[] = {2, 3};
    double bt = 0.0;
    bool have = false;
    for (int wi = 0; wi < 3; ++wi) {
        for (int si = 0; si < 2; ++si) {
            mbe_options o = b;
            o.wg_waves = kWaves[wi];
            o.steal_k = kSteal[si];
            o.diagnostics = 0;
            if (!have) {
                const int rc = run_batch(gs, n, &o, ref.data());
                if (rc != MBE_OK) return rc;
            }
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = run_batch(gs, n, &o, outs.data());
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rc != MBE_OK) return rc;
            for (int32_t i = 0; i < n; ++i)  // every setting must give the same answers
                if (outs[i].count != ref[i].count || outs[i].hash != ref[i].hash) return MBE_ERR_DEVICE;
            if (!have || ms < bt) {
                bt = ms;
                *best = o;
                have = true;
            }
        }
    }
    if (best_ms) *best_ms = bt;
    return MBE_OK;
}


int mbe_count(const mbe_graph *g, const mbe_options *opt, mbe_result *out) {
    const int rc = run(g, opt, out, nullptr, 0, 0, false);
    // a caller's workspace that is too small reads as out of memory
    return rc == MBE_ERR_SCRATCH_LIMIT && opt && opt->workspace ? MBE_ERR_OUT_OF_MEMORY : rc;
}

int mbe_count_loads(const mbe_graph *g, const mbe_options *opt, mbe_result *out, uint64_t *rec, int64_t cap_records,
                    int64_t *n_records) {
    if (!out || !n_records || cap_records < 0 || (cap_records > 0 && !rec)) return MBE_ERR_INVALID_ARG;
    *n_records = 0;
    mbe_options o = opt ? *opt : mbe_options{};
    if (o.prune) return MBE_ERR_INVALID_ARG;
    o.diagnostics = 2;
    std::vector<unsigned long long> raw;
    const int rc = run(g, &o, out, nullptr, 0, 0, false, nullptr, false, &raw);
    if (rc != MBE_OK) return rc;
    const int64_t n = (int64_t)(raw.size() / 4);
    *n_records = n;
    if (n == 0) return MBE_OK;
    int dev = 0, khz = 0;
    MBE_TRY(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    unsigned long long t0 = ~0ull;
    for (int64_t i = 0; i < n; ++i) t0 = std::min(t0, raw[4 * i + 1]);
    if (n > cap_records) return MBE_ERR_BUFFER_TOO_SMALL;
    const double ns_per_tick = 1.0e6 / (double)khz;
    for (int64_t i = 0; i < n; ++i) {
        rec[4 * i] = raw[4 * i];
        rec[4 * i + 1] = (uint64_t)((double)(raw[4 * i + 1] - t0) * ns_per_tick);
        rec[4 * i + 2] = (uint64_t)((double)(raw[4 * i + 2] - t0) * ns_per_tick);
        rec[4 * i + 3] = (uint64_t)((double)raw[4 * i + 3] * ns_per_tick);
    }
    return MBE_OK;
}

int mbe_count_noalloc(const mbe_graph *g, const mbe_options *opt, mbe_result *out) {
    return run(g, opt, out, nullptr, 0, 0, false, nullptr, true);
}

int mbe_workspace_size(const mbe_graph *g, const mbe_options *opt, size_t *bytes) {
    if (!bytes) return MBE_ERR_INVALID_ARG;
    *bytes = 0;
    mbe_result r;
    return run(g, opt, &r, nullptr, 0, 0, false, bytes);
}

int mbe_enumerate(const mbe_graph *g, const mbe_options *opt, mbe_result *out, int32_t *buf,
                  uint64_t buf_cap_ints, int32_t buf_on_device) {
    return run(g, opt, out, buf, buf_cap_ints, buf_on_device, true);
}

const char *mbe_strerror(int code) {
    switch (code) {
        case MBE_OK: return "ok";
        case MBE_ERR_INVALID_ARG: return "invalid argument";
        case MBE_ERR_INVALID_GRAPH: return "invalid graph (offsets, row order, id range or transpose mismatch)";
        case MBE_ERR_BUFFER_TOO_SMALL: return "record buffer too small";
        case MBE_ERR_OUT_OF_MEMORY: return "out of device memory (or the caller's workspace is too small)";
        case MBE_ERR_DEVICE: return "HIP runtime error";
        case MBE_ERR_UNSUPPORTED: return "unsupported input";
        case MBE_ERR_SCRATCH_LIMIT: return "the call needs more device memory than the fixed scratch of mbe_count_noalloc";
        case MBE_ERR_TIMEOUT: return "the request passed its deadline";
        case MBE_ERR_CANCELLED: return "the request was cancelled";
        default: return "unknown error";
    }
}

const char *mbe_version(void) { return "0.1.0"; }

}  // extern "C"
