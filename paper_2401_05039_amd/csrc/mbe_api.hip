// C-ABI entry points of libmbe.so (declared in include/mbe.h).
//
// One call = validate the CSR pair, rank the candidates, run the persistent search kernel
// once per mask-width class (widest first), read back the 16 accumulators, and for
// mbe_enumerate put the records into canonical order.  Device working memory is cached per
// device and grows on demand; calls on one device are serialised by a mutex.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mbe.h"
#include "mbe_internal.h"

namespace {

using namespace mbe;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
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
    DevBuf graph, prep, sort_tmp, arena, small;
    DevBuf rec, rec_offs, rec_tmp, rec_lens, canon_tmp, out_tmp;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cus = 0;
};

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

ArenaLayout make_layout(int32_t ucap, int32_t nwords, int Wmax, int waves, int32_t scap, int32_t maxdepth) {
    ArenaLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.off_bitmap = take((size_t)nwords * 8);
    L.off_bpre = take(((size_t)nwords + 1) * 4);
    L.off_M = take((size_t)ucap * Wmax * 8);
    L.off_gid = take((size_t)ucap * 4);
    L.off_cnt = take((size_t)ucap * 4);
    L.off_hv = take((size_t)64 * Wmax * 8);
    L.off_deg = take((size_t)64 * Wmax * 4);
    L.off_S1 = take((size_t)ucap * 4);
    L.off_t1v = take((size_t)ucap * 4);
    L.off_t1c = take((size_t)ucap * 4);
    L.off_waves = o;
    size_t w = 0;
    auto wtake = [&](size_t bytes) {
        size_t at = w;
        w = align_up(w + bytes, 256);
        return at;
    };
    L.off_w_stack = wtake((size_t)scap * 4);
    L.off_w_tv = wtake((size_t)ucap * 4);
    L.off_w_tc = wtake((size_t)ucap * 4);
    L.off_w_hdr = wtake((size_t)maxdepth * frame_header_bytes(Wmax));
    L.wave_bytes = w;
    L.wg_bytes = align_up(o + (size_t)waves * w, 4096);
    return L;
}

// Host-side check of one CSR direction against its transpose (same rules as the device
// validator): offsets start at 0, never decrease and end at n_edges; rows strictly ascend
// with ids in range; every (r, c) appears as (c, r) in the other direction.
bool host_valid(int32_t n_rows, int32_t n_cols, int32_t n_edges, const int32_t *off, const int32_t *adj,
                const int32_t *t_off, const int32_t *t_adj) {
    if (off[0] != 0 || off[n_rows] != n_edges) return false;
    for (int32_t r = 0; r < n_rows; ++r) {
        const int32_t b = off[r], e = off[r + 1];
        if (b > e || b < 0 || e > n_edges) return false;
        int32_t prev = -1;
        for (int32_t p = b; p < e; ++p) {
            const int32_t c = adj[p];
            if (c <= prev || c >= n_cols) return false;
            prev = c;
            const int32_t *lo = t_adj + t_off[c], *hi = t_adj + t_off[c + 1];
            if (t_off[c] < 0 || t_off[c + 1] > n_edges || t_off[c] > t_off[c + 1]) return false;
            const int32_t *it = std::lower_bound(lo, hi, r);
            if (it == hi || *it != r) return false;
        }
    }
    return true;
}

struct Opts {
    int side, waves, grid, diag, no_validate;
    int64_t root_lo, root_hi;
    hipStream_t stream;
};

Opts read_opts(const mbe_options *o) {
    Opts r{0, 8, 0, 0, 0, 0, -1, nullptr};
    if (!o) return r;
    r.side = o->side;
    r.waves = o->wg_waves > 0 ? o->wg_waves : 8;
    r.grid = o->grid > 0 ? o->grid : 0;
    r.diag = o->diagnostics != 0;
    r.no_validate = o->no_validate != 0;
    r.root_lo = o->root_lo > 0 ? o->root_lo : 0;
    r.root_hi = o->root_hi > 0 ? o->root_hi : -1;
    r.stream = static_cast<hipStream_t>(o->stream);
    return r;
}

int run(const mbe_graph *g, const mbe_options *opt_in, mbe_result *out, int32_t *ubuf, uint64_t ucap_ints,
        int ubuf_on_device, bool enumerate) {
    if (!g || !out) return MBE_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    if (g->n_u < 0 || g->n_v < 0 || g->n_edges < 0) return MBE_ERR_INVALID_ARG;
    Opts opt = read_opts(opt_in);
    if (opt.side < 0 || opt.side > 2 || opt.waves < 1 || opt.waves > 8) return MBE_ERR_INVALID_ARG;
    if (enumerate && !ubuf && ucap_ints > 0) return MBE_ERR_INVALID_ARG;
    const int side = opt.side ? opt.side : (g->n_v < g->n_u ? 2 : 1);
    out->side = (uint32_t)side;
    if (g->n_edges > 0 && (g->n_u == 0 || g->n_v == 0)) return MBE_ERR_INVALID_GRAPH;
    if (g->n_edges > 0 && (!g->u_off || !g->u_adj || !g->v_off || !g->v_adj)) return MBE_ERR_INVALID_ARG;
    if (!g->on_device && !opt.no_validate) {
        // host arrays: check before any device work
        if ((g->n_u > 0 && !g->u_off) || (g->n_v > 0 && !g->v_off)) return MBE_ERR_INVALID_ARG;
        if (g->n_edges > 0 || (g->u_off && g->v_off)) {
            if (!host_valid(g->n_u, g->n_v, g->n_edges, g->u_off, g->u_adj, g->v_off, g->v_adj) ||
                !host_valid(g->n_v, g->n_u, g->n_edges, g->v_off, g->v_adj, g->u_off, g->u_adj))
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

    const int32_t nu = g->n_u, nv = g->n_v, ne = g->n_edges;
    const int32_t *u_off = g->u_off, *u_adj = g->u_adj, *v_off = g->v_off, *v_adj = g->v_adj;
    if (!g->on_device) {
        const size_t b_uoff = align_up(((size_t)nu + 1) * 4, 256), b_voff = align_up(((size_t)nv + 1) * 4, 256);
        const size_t b_adj = align_up((size_t)ne * 4, 256);
        MBE_TRY(st->graph.ensure(b_uoff + b_voff + 2 * b_adj));
        int32_t *d_uoff = st->graph.as<int32_t>(0), *d_voff = st->graph.as<int32_t>(b_uoff);
        int32_t *d_uadj = st->graph.as<int32_t>(b_uoff + b_voff), *d_vadj = st->graph.as<int32_t>(b_uoff + b_voff + b_adj);
        MBE_TRY(hipMemcpyAsync(d_uoff, u_off, ((size_t)nu + 1) * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_voff, v_off, ((size_t)nv + 1) * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_uadj, u_adj, (size_t)ne * 4, hipMemcpyHostToDevice, s));
        MBE_TRY(hipMemcpyAsync(d_vadj, v_adj, (size_t)ne * 4, hipMemcpyHostToDevice, s));
        u_off = d_uoff;
        v_off = d_voff;
        u_adj = d_uadj;
        v_adj = d_vadj;
    }

    // small device block: acc[16] | flags | counters[8] | stats[16]
    MBE_TRY(st->small.ensure(4096));
    unsigned long long *acc = st->small.as<unsigned long long>(0);
    unsigned int *flags = st->small.as<unsigned int>(256);
    unsigned int *counters = st->small.as<unsigned int>(512);
    unsigned long long *stats = st->small.as<unsigned long long>(1024);

    if (!opt.no_validate && g->on_device) {
        MBE_TRY(hipMemsetAsync(flags, 0, 4, s));
        MBE_TRY(launch_validate(nu, nv, ne, u_off, u_adj, v_off, v_adj, flags, s));
        MBE_TRY(launch_validate(nv, nu, ne, v_off, v_adj, u_off, u_adj, flags, s));
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
    MBE_TRY(st->prep.ensure(2 * b_keys + 2 * b_i32));
    unsigned long long *keys = st->prep.as<unsigned long long>(0);
    unsigned long long *sorted = st->prep.as<unsigned long long>(b_keys);
    int32_t *order = st->prep.as<int32_t>(2 * b_keys);
    int32_t *rank = st->prep.as<int32_t>(2 * b_keys + b_i32);
    MBE_TRY(hipMemsetAsync(stats, 0, 16 * 8, s));
    MBE_TRY(launch_rank_keys(nc, c_off, keys, stats, s));
    int end_bit = 32;
    while (end_bit < 64 && ((unsigned long long)no >> (end_bit - 32)) != 0ull) ++end_bit;
    size_t tmp_bytes = 0;
    MBE_TRY(radix_sort_u64(nullptr, &tmp_bytes, keys, sorted, nc, end_bit, s));
    MBE_TRY(st->sort_tmp.ensure(tmp_bytes));
    tmp_bytes = st->sort_tmp.bytes;
    MBE_TRY(radix_sort_u64(st->sort_tmp.p, &tmp_bytes, keys, sorted, nc, end_bit, s));
    unsigned long long hstats[16];
    MBE_TRY(hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
    MBE_TRY(hipStreamSynchronize(s));
    const int32_t nzero = (int32_t)hstats[0];
    const int32_t ncand = nc - nzero;
    if (ncand <= 0) return MBE_OK;
    if (hstats[8] > (unsigned long long)MBE_MAX_DEGREE) return MBE_ERR_UNSUPPORTED;
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

    const int waves = opt.waves;
    const int grid = opt.grid > 0 ? opt.grid : 2 * st->cus;
    const int32_t nwords = (ncand + 63) / 64;
    int32_t scap = 2 * ncand + 1024;
    int32_t maxdepth = 64 * Wmax + 2;

    // record arena for mbe_enumerate
    unsigned long long rec_cap = 0, offs_cap = 0;
    if (enumerate) {
        rec_cap = ucap_ints;
        offs_cap = ucap_ints / 4 + 1;
        MBE_TRY(st->rec.ensure((size_t)rec_cap * 4 + 256));
        MBE_TRY(st->rec_offs.ensure((size_t)offs_cap * 8));
    }

    SearchArgs a{};
    a.nc = nc;
    a.no = no;
    a.ncand = ncand;
    a.c_is_v = c_is_v ? 1 : 0;
    a.c_off = c_off;
    a.c_adj = c_adj;
    a.o_off = o_off;
    a.o_adj = o_adj;
    a.order = order;
    a.rank = rank;
    a.total_fw = 2ull * (unsigned long long)ncand + (unsigned long long)ne;
    a.ucap = ncand;
    a.nwords = nwords;
    a.acc = acc;
    a.flags = flags;
    a.rec = enumerate ? st->rec.as<int32_t>() : nullptr;
    a.rec_cap = rec_cap;
    a.rec_offs = enumerate ? st->rec_offs.as<unsigned long long>() : nullptr;
    a.rec_offs_cap = offs_cap;

    unsigned long long hacc[ACC_SLOTS];
    unsigned int hflags = 0;
    float ms = 0.f;
    for (int attempt = 0; attempt < 8; ++attempt) {
        a.scap = scap;
        a.maxdepth = maxdepth;
        a.lay = make_layout(ncand, nwords, Wmax, waves, scap, maxdepth);
        MBE_TRY(st->arena.ensure(a.lay.wg_bytes * (size_t)grid));
        a.arena = st->arena.as<char>();
        MBE_TRY(hipMemset2DAsync(a.arena + a.lay.off_bitmap, a.lay.wg_bytes, 0, (size_t)nwords * 8, (size_t)grid, s));
        MBE_TRY(hipMemsetAsync(acc, 0, ACC_SLOTS * 8, s));
        MBE_TRY(hipMemsetAsync(flags, 0, 4, s));
        MBE_TRY(hipMemsetAsync(counters, 0, 8 * 4, s));
        MBE_TRY(hipEventRecord(st->ev0, s));
        for (int c = 4; c >= 0; --c) {
            const int64_t clo = std::max(cls_lo[c], lo), chi = std::min(cls_hi[c], hi);
            if (clo >= chi) continue;
            const int W = 1 << c;
            MBE_TRY(launch_search(a, W, opt.diag, enumerate, clo, chi, counters + c, grid, waves,
                                  search_lds_bytes(W, waves), s));
        }
        MBE_TRY(hipEventRecord(st->ev1, s));
        MBE_TRY(hipMemcpyAsync(hacc, acc, sizeof(hacc), hipMemcpyDeviceToHost, s));
        MBE_TRY(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, s));
        MBE_TRY(hipStreamSynchronize(s));
        MBE_TRY(hipEventElapsedTime(&ms, st->ev0, st->ev1));
        if (!(hflags & (FLAG_STACK_OVERFLOW | FLAG_DEPTH_OVERFLOW))) break;
        if (hflags & FLAG_STACK_OVERFLOW) scap = (int32_t)std::min<int64_t>((int64_t)scap * 2, (int64_t)1 << 30);
        if (hflags & FLAG_DEPTH_OVERFLOW) maxdepth *= 2;
        if (attempt == 7) return MBE_ERR_OUT_OF_MEMORY;
    }

    out->count = hacc[ACC_COUNT];
    out->hash = hacc[ACC_HASH];
    out->out_ints = hacc[ACC_OUT_INTS];
    out->nodes = hacc[ACC_NODES];
    out->nonmaximal = hacc[ACC_NONMAX];
    out->bytes_alg = hacc[ACC_BYTES];
    out->max_depth = (uint32_t)hacc[ACC_MAX_DEPTH];
    out->kernel_ms = ms;

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

}  // namespace

extern "C" {

int mbe_count(const mbe_graph *g, const mbe_options *opt, mbe_result *out) {
    return run(g, opt, out, nullptr, 0, 0, false);
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
        case MBE_ERR_OUT_OF_MEMORY: return "out of device memory";
        case MBE_ERR_DEVICE: return "HIP runtime error";
        case MBE_ERR_UNSUPPORTED: return "candidate degree above MBE_MAX_DEGREE";
        default: return "unknown error";
    }
}

const char *mbe_version(void) { return "0.1.0"; }

}  // extern "C"
