// C ABI of libpetar: context, argument checks, workspace, and the ordered
// launches of the tree build and the long-range force (see include/petar.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/petar.h"
#include "launch.h"
#include "validate.h"
#include "walk.h"

using namespace petar;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

thread_local std::string g_last_error;

}  // namespace

// host_scalar: pinned words for the single values read back by the filter,
// cluster and artificial-particle calls.
constexpr int kHostScalarWords = 8;

struct petar_ctx {
    int device = PETAR_NO_DEVICE;
    hipStream_t stream = nullptr;
    petar_params params{};
    std::string err;
    int64_t ws_bytes = 0;

    // tree build
    DevBuf key0, key1, val0, val1, sort_ws, scan_ws, bbox_part, rootbox, status, emit, base;
    DevBuf ps, orig, rank, rr, rsk;
    DevBuf nd_lo, nd_hi, nd_com, nd_S, nd_q, nd_info, nd_parent, level_off;
    DevBuf pre_info, pre_parent, pre_nchild, new_of_old, lkey0, lkey1, lval0, lval1;
    // force
    DevBuf gflag, gpos, groups, spill, queue, counts, nbcnt, radii_ws, nbhead, nbleaf, sys_off;
    DevBuf nbrowoff, nbrows;  // neighbour rows: offsets (input order) and scratch
    DevBuf tflag, tpos, tidx;  // target compaction (petar_set_targets)
    // second-stage filter and clusters
    DevBuf cl_keep, cl_row, cl_counts, cl_parent, cl_root, cl_rootpos, cl_status, cl_flags,
        cl_key0, cl_key1, cl_val0, cl_val1;
    // artificial particles
    DevBuf art_single, art_spos, art_status, art_pairof, tt_ginv, grp_off, grp_idx;
    bool tt_ginv_ready = false;
    uint32_t nbhead_cap = 0, nbleaf_cap = 0;
    int64_t nbrows_cap = 0;  // entries of nbrows; grown when a call's rows needed more

    Status *host_status = nullptr;  // pinned
    int64_t *host_scalar = nullptr; // pinned

    bool have_tree = false;
    bool have_counts = false;
    const uint8_t *target = nullptr;  // caller's target flags (input order), none: all
    int64_t n = 0;
    double theta = 0.0;
    int leaf_size = 0;
    int64_t n_nodes = 0;
    int levels = kMaxLevel;
    int deep = kMaxLevel;  // deepest cell level: the per-level passes start above it
    bool build_stats_pending = false;  // eager build not yet read back (see settle_build_stats)
    int n_sys = 1;

    int force_waves[2][5] = {{0}};
    int nb_waves = 0;

    // captured step (petar_step_graph)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_stale = true;
    std::vector<int64_t> graph_key;  // arguments the graph was captured with
    int64_t node_cap = 0;            // cell capacity of the captured graph

    hipEvent_t ev[8] = {};
    petar_stats stats{};
};

namespace {

petar_status fail(petar_ctx *ctx, petar_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_last_error = buf;
    return st;
}

#define HIP_TRY(ctx, expr)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), PETAR_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

#define TRY(expr)                          \
    do {                                   \
        petar_status s_ = (expr);          \
        if (s_ != PETAR_OK) return s_;     \
    } while (0)

// Grows a device buffer to at least `bytes` (contents are not kept).
petar_status ensure(petar_ctx *ctx, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.cap >= bytes) return PETAR_OK;
    size_t want = bytes + bytes / 8;  // headroom against small growth
    int64_t after = ctx->ws_bytes - (int64_t)b.cap + (int64_t)want;
    if (ctx->params.workspace_cap > 0 && after > ctx->params.workspace_cap) {
        want = bytes;
        after = ctx->ws_bytes - (int64_t)b.cap + (int64_t)want;
        if (after > ctx->params.workspace_cap)
            return fail(ctx, PETAR_E_NOMEM, "workspace cap of %lld bytes exceeded (need %lld)",
                        (long long)ctx->params.workspace_cap, (long long)after);
    }
    if (b.p) {
        // work queued by an earlier call (the second half of a tree build)
        // may still use the buffer
        (void)hipStreamSynchronize(ctx->stream);
        hipFree(b.p);
        ctx->ws_bytes -= (int64_t)b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    ctx->graph_stale = true;  // a captured step graph may hold the old address
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(ctx, PETAR_E_NOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    b.cap = want;
    ctx->ws_bytes += (int64_t)want;
    return PETAR_OK;
}

template <typename T>
T *ptr(DevBuf &b) {
    return static_cast<T *>(b.p);
}

PreOrder pre_view(petar_ctx *c) {
    PreOrder p;
    p.info = ptr<uint4>(c->pre_info);
    p.parent = ptr<uint32_t>(c->pre_parent);
    p.nchild = ptr<uint32_t>(c->pre_nchild);
    p.new_of_old = ptr<uint32_t>(c->new_of_old);
    return p;
}

TreeDev tree_view(petar_ctx *c) {
    TreeDev t;
    t.n_nodes_dev = &ptr<Status>(c->status)->n_nodes;  // set by the build (0 on overflow)
    t.ps = ptr<double4>(c->ps);
    t.rr = ptr<double2>(c->rr);
    t.rsk = ptr<double>(c->rsk);
    t.orig = ptr<uint32_t>(c->orig);
    t.rank = ptr<uint32_t>(c->rank);
    t.nd_lo = ptr<double4>(c->nd_lo);
    t.nd_hi = ptr<double4>(c->nd_hi);
    t.nd_com = ptr<double4>(c->nd_com);
    t.nd_S = ptr<double>(c->nd_S);
    t.nd_q = ptr<float4>(c->nd_q);
    t.nd_info = ptr<uint4>(c->nd_info);
    t.nd_parent = ptr<uint32_t>(c->nd_parent);
    t.level_off = ptr<uint32_t>(c->level_off);
    t.n = c->n;
    t.n_nodes = c->n_nodes;
    return t;
}

void zero_status(petar_ctx *c, hipStream_t s) {
    fill_i64(ptr<int64_t>(c->status), 0, (int64_t)(sizeof(Status) / sizeof(int64_t)), s);
}

void zero_force_status(petar_ctx *c, hipStream_t s) {
    fill_i64(ptr<int64_t>(c->status), 0, kStatusForceWords, s);
}

petar_status read_status(petar_ctx *c, hipStream_t s) {
    HIP_TRY(c, hipMemcpyAsync(c->host_status, c->status.p, sizeof(Status), hipMemcpyDeviceToHost,
                              s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return PETAR_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();  // a missing timing is not an error of the call
        return 0.f;
    }
    return ms;
}

// Fills the counters of the last eager build once its status words have
// been read (host_status current: `fresh`; else they are read here). The
// build fields of Status are not touched by the force calls.
petar_status settle_build_stats(petar_ctx *c, bool fresh) {
    if (!c->build_stats_pending) return PETAR_OK;
    if (!fresh) TRY(read_status(c, c->stream));
    c->stats.n_leaves = c->host_status->n_leaves;
    c->stats.max_level = c->host_status->max_level;
    c->stats.ms_build = elapsed(c->ev[0], c->ev[1]);
    c->build_stats_pending = false;
    return PETAR_OK;
}

void drop_graph(petar_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_stale = true;
}

void free_all(petar_ctx *c) {
    DevBuf *bufs[] = {&c->key0,     &c->key1,        &c->val0,       &c->val1,       &c->sort_ws,
                      &c->scan_ws,  &c->bbox_part,   &c->rootbox,    &c->status,     &c->emit,
                      &c->base,     &c->ps,          &c->orig,       &c->rank,       &c->rr,         &c->rsk,
                      &c->nd_lo,    &c->nd_hi,       &c->nd_com,     &c->nd_S,       &c->nd_q,       &c->nd_info,    &c->nd_parent,
                      &c->level_off, &c->pre_info,   &c->pre_parent, &c->pre_nchild, &c->new_of_old,
                      &c->lkey0,    &c->lkey1,       &c->lval0,      &c->lval1,
                      &c->gflag,    &c->gpos,        &c->groups,     &c->spill,
                      &c->queue,    &c->counts,      &c->nbcnt,      &c->radii_ws,   &c->nbhead, &c->nbleaf,
                      &c->nbrowoff, &c->nbrows,
                      &c->cl_keep,  &c->cl_row,      &c->cl_counts,   &c->cl_parent,  &c->cl_root,    &c->cl_rootpos,
                      &c->cl_status,   &c->cl_flags,   &c->cl_key0,    &c->cl_key1,
                      &c->cl_val0,  &c->cl_val1,
                      &c->art_single, &c->art_spos, &c->art_status, &c->art_pairof, &c->tt_ginv,
                      &c->grp_off,  &c->grp_idx,  &c->tflag,      &c->tpos,       &c->tidx,
                      &c->sys_off};
    for (DevBuf *b : bufs) {
        if (b->p) hipFree(b->p);
        b->p = nullptr;
        b->cap = 0;
    }
    c->ws_bytes = 0;
    c->tt_ginv_ready = false;
}

}  // namespace

extern "C" {

const char *petar_status_string(petar_status s) {
    switch (s) {
        case PETAR_OK: return "ok";
        case PETAR_E_INVALID: return "invalid argument";
        case PETAR_E_NOMEM: return "out of device memory / workspace cap";
        case PETAR_E_HIP: return "HIP runtime error";
        case PETAR_E_NB_OVERFLOW: return "neighbour list capacity too small";
        case PETAR_E_STATE: return "call order violated";
        case PETAR_E_NODEVICE: return "context has no device";
        case PETAR_E_INTERNAL: return "internal limit exceeded";
    }
    return "unknown status";
}

const char *petar_last_error(petar_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

petar_status petar_create(petar_ctx **out, int device, void *hip_stream) {
    if (!out) return fail(nullptr, PETAR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (device < PETAR_NO_DEVICE) return fail(nullptr, PETAR_E_INVALID, "bad device %d", device);
    petar_ctx *c = new (std::nothrow) petar_ctx();
    if (!c) return fail(nullptr, PETAR_E_NOMEM, "host allocation failed");
    c->params.G = 1.0;
    c->params.precision = PETAR_MIXED;
    c->params.i_per_lane = 1;
    c->params.record_counts = 0;
    c->params.workspace_cap = 0;
    c->device = device;
    if (device != PETAR_NO_DEVICE) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
            delete c;
            return fail(nullptr, PETAR_E_INVALID, "device %d not present (%d devices)", device, ndev);
        }
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_status, sizeof(Status));
        if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_scalar, kHostScalarWords * sizeof(int64_t));
        for (int k = 0; k < 8 && e == hipSuccess; k++) e = hipEventCreate(&c->ev[k]);
        // set-up of this device's fixed scratch (petar_clusters_noalloc)
        void *scratch_ptr = nullptr;
        size_t scratch_bytes = 0;
        if (e == hipSuccess) e = noalloc_scratch(device, &scratch_ptr, &scratch_bytes);
        if (e != hipSuccess) {
            petar_destroy(c);
            return fail(nullptr, PETAR_E_HIP, "context setup failed: %s", hipGetErrorString(e));
        }
        c->stream = (hipStream_t)hip_stream;
    }
    *out = c;
    return PETAR_OK;
}

petar_status petar_destroy(petar_ctx *ctx) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (ctx->device != PETAR_NO_DEVICE) {
        hipSetDevice(ctx->device);
        if (ctx->stream) hipStreamSynchronize(ctx->stream);
        drop_graph(ctx);
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
        free_all(ctx);
        if (ctx->host_status) hipHostFree(ctx->host_status);
        if (ctx->host_scalar) hipHostFree(ctx->host_scalar);
        for (int k = 0; k < 8; k++)
            if (ctx->ev[k]) hipEventDestroy(ctx->ev[k]);
    }
    delete ctx;
    return PETAR_OK;
}

petar_status petar_set_params(petar_ctx *ctx, const petar_params *p) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_params(p)) return fail(ctx, PETAR_E_INVALID, "%s", m);
    ctx->params = *p;
    return PETAR_OK;
}

petar_status petar_get_params(petar_ctx *ctx, petar_params *p) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (!p) return fail(ctx, PETAR_E_INVALID, "params is NULL");
    *p = ctx->params;
    return PETAR_OK;
}

petar_status petar_changeover_radii(petar_ctx *ctx, const double *mass, const double *vel,
                                    int64_t n, double r_in_ref, double r_out_ref,
                                    double search_factor, double cr_dt, double *r_in,
                                    double *r_out, double *r_search) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_radii_args(mass, n, r_in_ref, r_out_ref, search_factor, cr_dt, r_in,
                                         r_out, r_search))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    TRY(ensure(ctx, ctx->radii_ws, 1025 * sizeof(double)));
    launch_changeover_radii(mass, vel, n, r_in_ref, r_out_ref, search_factor, cr_dt, r_in, r_out,
                            r_search, ptr<double>(ctx->radii_ws), ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PETAR_OK;
}

}  // extern "C"

namespace {

// Filter of a candidate CSR (mode 0: pericentre, mode 1: group relation) into
// out_offsets[n + 1] / out_idx[capacity]; *required = kept entries.
petar_status filter_impl(petar_ctx *ctx, FilterArgs a, int64_t *out_offsets, int32_t *out_idx,
                         int64_t capacity, int64_t *required) {
    const int64_t n = a.n;
    hipStream_t s = ctx->stream;
    // candidate count and CSR sanity (one host read)
    TRY(ensure(ctx, ctx->cl_status, 8));
    int32_t *bad = ptr<int32_t>(ctx->cl_status);
    fill_i64(ptr<int64_t>(ctx->cl_status), 0, 1, s);
    launch_check_csr(a.offsets, n, bad, s);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, a.offsets + n, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar + 1, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const int64_t n_cand = ctx->host_scalar[0];
    int32_t b0 = 0;
    memcpy(&b0, ctx->host_scalar + 1, 4);
    if (b0) return fail(ctx, PETAR_E_INVALID, "candidate offsets must start at 0 and not decrease");
    if (out_idx == nullptr) {  // internal output sized to the candidates
        TRY(ensure(ctx, ctx->grp_idx, (size_t)(n_cand > 0 ? n_cand : 1) * 4));
        out_idx = ptr<int32_t>(ctx->grp_idx);
        capacity = n_cand;
    }
    TRY(ensure(ctx, ctx->cl_keep, (size_t)(n_cand > 0 ? n_cand : 1)));
    TRY(ensure(ctx, ctx->cl_row, (size_t)(n_cand > 0 ? n_cand : 1) * 4));
    TRY(ensure(ctx, ctx->cl_counts, (size_t)(n + 1) * 4));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(n + 1) * 8));
    launch_filter(a, n_cand, ptr<int32_t>(ctx->cl_row), ptr<uint8_t>(ctx->cl_keep),
                  ptr<uint32_t>(ctx->cl_counts), bad, s);
    scan_u32_to_i64(ptr<uint32_t>(ctx->cl_counts), out_offsets, n, ptr<int64_t>(ctx->scan_ws), s);
    launch_filter_write(a, ptr<uint8_t>(ctx->cl_keep), out_offsets, out_idx, capacity, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, out_offsets + n, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar + 1, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int32_t b = 0;
    memcpy(&b, ctx->host_scalar + 1, 4);
    if (b) return fail(ctx, PETAR_E_INVALID, "candidate index outside [0, N)");
    *required = ctx->host_scalar[0];
    if (*required > capacity)
        return fail(ctx, PETAR_E_NB_OVERFLOW, "neighbour capacity %lld < required %lld",
                    (long long)capacity, (long long)*required);
    return PETAR_OK;
}

// Scratch of the clusters pass for n particles.
struct ClusterWs {
    int32_t *parent;             // [n] union-find parents
    uint32_t *root, *rootpos;    // [n + 1] root flags, their exclusive scan
    int32_t *flags;              // [2] bad offsets, bad index
    uint64_t *key0, *key1;       // [n] sort keys (double-buffered)
    uint32_t *val0, *val1;       // [n] sort values
    void *sort_ws;               // sort_ws_bytes(n)
    int64_t *scan_ws;            // scan_ws_elems(n + 1)
};

// Lays ClusterWs out from `base` in 256-byte aligned pieces and returns the
// bytes it spans; with base == nullptr only the size is computed.
size_t cluster_ws_carve(char *base, int64_t n, ClusterWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t un = (size_t)n;
    ClusterWs c;
    c.parent = (int32_t *)take(un * 4);
    c.root = (uint32_t *)take((un + 1) * 4);
    c.rootpos = (uint32_t *)take((un + 1) * 4);
    c.flags = (int32_t *)take(8);
    c.key0 = (uint64_t *)take(un * 8);
    c.key1 = (uint64_t *)take(un * 8);
    c.val0 = (uint32_t *)take(un * 4);
    c.val1 = (uint32_t *)take(un * 4);
    c.sort_ws = take((size_t)sort_ws_bytes(n));
    c.scan_ws = (int64_t *)take((size_t)scan_ws_elems(n + 1) * 8);
    if (w) *w = c;
    return off;
}

// Components of a CSR (label, offsets, members as petar_clusters) with the
// scratch in w.
petar_status clusters_core(petar_ctx *ctx, int64_t n, const int64_t *nb_offsets,
                           const int32_t *nb_idx, int32_t *label, int64_t *cl_offsets,
                           int32_t *members, int64_t *n_clusters, const ClusterWs &w) {
    hipStream_t s = ctx->stream;
    // flags = {bad offsets, bad index}
    int32_t *csr_bad = w.flags, *bad = csr_bad + 1;
    fill_i64((int64_t *)w.flags, 0, 1, s);
    launch_check_csr(nb_offsets, n, csr_bad, s);
    launch_components(nb_offsets, nb_idx, n, w.parent, label, w.root, bad, csr_bad, s);
    scan_u32_to_u32(w.root, w.rootpos, n, w.scan_ws, s);
    // members: stable radix sort of the particle indices by cluster index
    uint64_t *k = w.key0, *ka = w.key1;
    uint32_t *v = w.val0, *va = w.val1;
    launch_cluster_keys(label, n, w.rootpos, k, v, s);
    int passes = 1;
    while (passes < 4 && (n - 1) >> (8 * passes)) passes++;
    radix_sort(&k, &v, &ka, &va, n, passes, w.sort_ws, s);
    HIP_TRY(ctx, hipMemcpyAsync(members, v, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    launch_cluster_offsets(k, n, cl_offsets, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, w.rootpos + n, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar + 1, csr_bad, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int32_t fl[2] = {0, 0};
    memcpy(fl, ctx->host_scalar + 1, 8);
    if (fl[0]) return fail(ctx, PETAR_E_INVALID, "neighbour offsets must start at 0 and not decrease");
    if (fl[1]) return fail(ctx, PETAR_E_INVALID, "neighbour index outside [0, N)");
    uint32_t nc = 0;
    memcpy(&nc, ctx->host_scalar, 4);
    *n_clusters = nc;
    return PETAR_OK;
}

// petar_clusters with the scratch in the context's workspace.
petar_status clusters_impl(petar_ctx *ctx, int64_t n, const int64_t *nb_offsets,
                           const int32_t *nb_idx, int32_t *label, int64_t *cl_offsets,
                           int32_t *members, int64_t *n_clusters) {
    TRY(ensure(ctx, ctx->cl_parent, (size_t)n * 4));
    TRY(ensure(ctx, ctx->cl_root, (size_t)(n + 1) * 4));
    TRY(ensure(ctx, ctx->cl_rootpos, (size_t)(n + 1) * 4));
    TRY(ensure(ctx, ctx->cl_flags, 8));
    TRY(ensure(ctx, ctx->cl_key0, (size_t)n * 8));
    TRY(ensure(ctx, ctx->cl_key1, (size_t)n * 8));
    TRY(ensure(ctx, ctx->cl_val0, (size_t)n * 4));
    TRY(ensure(ctx, ctx->cl_val1, (size_t)n * 4));
    TRY(ensure(ctx, ctx->sort_ws, (size_t)sort_ws_bytes(n)));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(n + 1) * 8));
    ClusterWs w;
    w.parent = ptr<int32_t>(ctx->cl_parent);
    w.root = ptr<uint32_t>(ctx->cl_root);
    w.rootpos = ptr<uint32_t>(ctx->cl_rootpos);
    w.flags = ptr<int32_t>(ctx->cl_flags);
    w.key0 = ptr<uint64_t>(ctx->cl_key0);
    w.key1 = ptr<uint64_t>(ctx->cl_key1);
    w.val0 = ptr<uint32_t>(ctx->cl_val0);
    w.val1 = ptr<uint32_t>(ctx->cl_val1);
    w.sort_ws = ctx->sort_ws.p;
    w.scan_ws = ptr<int64_t>(ctx->scan_ws);
    return clusters_core(ctx, n, nb_offsets, nb_idx, label, cl_offsets, members, n_clusters, w);
}

}  // namespace

extern "C" {

petar_status petar_clusters(petar_ctx *ctx, int64_t n, const int64_t *nb_offsets,
                            const int32_t *nb_idx, int32_t *label, int64_t *cl_offsets,
                            int32_t *members, int64_t *n_clusters) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_cluster_args(n, nb_offsets, nb_idx, label, cl_offsets, members,
                                           n_clusters))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return clusters_impl(ctx, n, nb_offsets, nb_idx, label, cl_offsets, members, n_clusters);
}

petar_status petar_clusters_noalloc(petar_ctx *ctx, int64_t n, const int64_t *nb_offsets,
                                    const int32_t *nb_idx, int32_t *label, int64_t *cl_offsets,
                                    int32_t *members, int64_t *n_clusters) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_cluster_args(n, nb_offsets, nb_idx, label, cl_offsets, members,
                                           n_clusters))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (n > kNoAllocMaxN)
        return fail(ctx, PETAR_E_INVALID,
                    "N = %lld exceeds the fixed scratch of petar_clusters_noalloc "
                    "(at most %lld particles); use petar_clusters",
                    (long long)n, (long long)kNoAllocMaxN);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *base = nullptr;
    size_t bytes = 0;
    HIP_TRY(ctx, noalloc_scratch(ctx->device, &base, &bytes));
    ClusterWs w;
    if (cluster_ws_carve((char *)base, n, &w) > bytes)
        return fail(ctx, PETAR_E_INTERNAL, "fixed scratch of %zu bytes too small for N = %lld",
                    bytes, (long long)n);
    return clusters_core(ctx, n, nb_offsets, nb_idx, label, cl_offsets, members, n_clusters, w);
}

petar_status petar_nb_filter(petar_ctx *ctx, int64_t n, const double *pos, const double *vel,
                             const double *mass, const double *r_nb, double c_v,
                             const int64_t *cand_offsets, const int32_t *cand_idx,
                             petar_nblist *out) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_filter_args(n, pos, vel, mass, r_nb, c_v, cand_offsets, cand_idx,
                                          out))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    FilterArgs a{pos, vel, mass, r_nb, cand_offsets, cand_idx, n, c_v, ctx->params.G, 0};
    return filter_impl(ctx, a, out->offsets_dev, out->idx_dev, out->capacity, &out->required);
}

petar_status petar_groups(petar_ctx *ctx, int64_t n, const double *pos, const double *vel,
                          const double *mass, const double *r_in, double theta,
                          const int64_t *cand_offsets, const int32_t *cand_idx, int32_t *label,
                          int64_t *grp_offsets, int32_t *members, int64_t *n_groups,
                          int32_t *pairs, int64_t pair_cap, int64_t *n_pairs) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_groups_args(n, pos, vel, mass, r_in, theta, cand_offsets, cand_idx,
                                          label, grp_offsets, members, n_groups, pairs, pair_cap,
                                          n_pairs))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    TRY(ensure(ctx, ctx->grp_off, (size_t)(n + 1) * 8));
    FilterArgs a{pos, vel, mass, r_in, cand_offsets, cand_idx, n, theta, ctx->params.G, 1};
    int64_t kept = 0;
    TRY(filter_impl(ctx, a, ptr<int64_t>(ctx->grp_off), nullptr, 0, &kept));
    TRY(clusters_impl(ctx, n, ptr<int64_t>(ctx->grp_off), ptr<int32_t>(ctx->grp_idx), label,
                      grp_offsets, members, n_groups));
    const int64_t ng = *n_groups;
    TRY(ensure(ctx, ctx->art_single, (size_t)(ng + 1) * 4));
    TRY(ensure(ctx, ctx->art_spos, (size_t)(ng + 1) * 4));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(ng + 1) * 8));
    uint32_t *flag = ptr<uint32_t>(ctx->art_single), *where = ptr<uint32_t>(ctx->art_spos);
    launch_group_pairs(grp_offsets, members, ng, pos, vel, mass, n, ctx->params.G, flag, s);
    scan_u32_to_u32(flag, where, ng, ptr<int64_t>(ctx->scan_ws), s);
    launch_group_pairs_write(grp_offsets, members, ng, flag, where, pairs, pair_cap, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, where + ng, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    uint32_t np = 0;
    memcpy(&np, ctx->host_scalar, 4);
    *n_pairs = np;
    return PETAR_OK;
}

petar_status petar_kick(petar_ctx *ctx, int64_t n, double *vel, const double *acc, double dt) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (n < 1 || n > kMaxParticles) return fail(ctx, PETAR_E_INVALID, "N must be in [1, 2^31)");
    if (!vel || !acc) return fail(ctx, PETAR_E_INVALID, "vel and acc must not be NULL");
    if (!std::isfinite(dt)) return fail(ctx, PETAR_E_INVALID, "dt must be finite");
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    launch_kick(vel, acc, n, dt, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return PETAR_OK;
}

petar_status petar_artificial_make(petar_ctx *ctx, int64_t n, const double *pos, const double *vel,
                                   const double *mass, const double *r_in, const double *r_out,
                                   const double *r_search, int64_t n_pair, const int32_t *pairs,
                                   int order, double c_d, petar_art_set *set, double *frame,
                                   int32_t *pair_of) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_art_make_args(n, pos, vel, mass, r_in, r_out, r_search, n_pair,
                                            pairs, order, c_d, set, frame))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    TRY(ensure(ctx, ctx->art_single, (size_t)n * 4));
    TRY(ensure(ctx, ctx->art_spos, (size_t)(n + 1) * 4));
    TRY(ensure(ctx, ctx->art_status, 16));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(n + 1) * 8));
    if (!pair_of) {
        TRY(ensure(ctx, ctx->art_pairof, (size_t)n * 4));
        pair_of = ptr<int32_t>(ctx->art_pairof);
    }
    int32_t *bad = ptr<int32_t>(ctx->art_status);
    fill_i64(ptr<int64_t>(ctx->art_status), 0, 2, s);
    ArtArgs a{pos, vel, mass, r_in, r_out, r_search, n, pairs, n_pair, order, c_d,
              ctx->params.G, n - 2 * n_pair, set->n_out, set->pos_dev, set->mass_dev,
              set->r_in_dev, set->r_out_dev, set->r_search_dev, set->src_dev, frame, pair_of,
              set->target_dev};
    launch_art_make(a, ptr<uint32_t>(ctx->art_single), ptr<uint32_t>(ctx->art_spos),
                    ptr<int64_t>(ctx->scan_ws), bad, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, bad, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int32_t b[4] = {0, 0, 0, 0};
    memcpy(b, ctx->host_scalar, 16);
    if (b[0]) return fail(ctx, PETAR_E_INVALID, "%d pairs with an index outside [0, N) or i == j", b[0]);
    if (b[1]) return fail(ctx, PETAR_E_INVALID, "a particle appears in more than one pair");
    if (b[2]) return fail(ctx, PETAR_E_INVALID, "%d pairs are not bound", b[2]);
    return PETAR_OK;
}

petar_status petar_tidal_fit(petar_ctx *ctx, int order, int64_t n, const double *pos,
                             int64_t n_pair, const int32_t *pairs, const double *frame,
                             int64_t n_out, const int32_t *src, const double *acc_set,
                             const double *pot_set, double *tensor, double *acc, double *pot) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_tidal_fit_args(order, n, pos, n_pair, pairs, frame, n_out, src,
                                             acc_set, pot_set, tensor, acc, pot))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int P = order == 2 ? 4 : 8;
    if (!ctx->tt_ginv_ready) {
        // both orders, order 2 first (6 x 12), then order 3 (16 x 24)
        TRY(ensure(ctx, ctx->tt_ginv, (72 + 384) * 8));
        HIP_TRY(ctx, hipMemcpy(ctx->tt_ginv.p, tidal_ginv_host(2), 72 * 8, hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipMemcpy(ptr<double>(ctx->tt_ginv) + 72, tidal_ginv_host(3), 384 * 8,
                               hipMemcpyHostToDevice));
        ctx->tt_ginv_ready = true;
    }
    FitArgs f{order, n_pair, n_out - n_pair * (P + 4), n_out, acc_set, pot_set, frame,
              ptr<double>(ctx->tt_ginv) + (order == 2 ? 0 : 72), tensor, pos, n, pairs, src,
              acc, pot};
    launch_tidal_fit(f, s);
    HIP_TRY(ctx, hipGetLastError());
    return PETAR_OK;
}

petar_status petar_tidal_eval(petar_ctx *ctx, int order, int64_t n_pair, const double *tensor,
                              const double *frame, int64_t n_pt, const int32_t *pair_of,
                              const double *pos, double *acc, double *pot) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_tidal_eval_args(order, n_pair, tensor, frame, n_pt, pair_of, pos,
                                              acc))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    if (n_pt == 0) return PETAR_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    TRY(ensure(ctx, ctx->art_status, 16));
    int32_t *bad = ptr<int32_t>(ctx->art_status);
    fill_i64(ptr<int64_t>(ctx->art_status), 0, 1, s);
    EvalArgs e{order, n_pair, tensor, frame, n_pt, pair_of, pos, acc, pot, bad};
    launch_tidal_eval(e, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int32_t b = 0;
    memcpy(&b, ctx->host_scalar, 4);
    if (b) return fail(ctx, PETAR_E_INVALID, "%d points with pair_of >= n_pair", b);
    return PETAR_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------- build
// The tree build runs in two phases around the only host read it needs in
// eager mode (the cell count, to size the cell arrays):
//   A: root cube(s), keys, sort, particle gather, cell counting and scan;
//   B: cells in pre-order, level sort, level-order layout, multipoles.
// One system (n_sys == 0): one root cube, 21 levels. Batches: one root cube
// per system, kBatchLevels levels, system id above the Morton digits.

struct BuildArgs {
    const double *pos;
    const double *mass;
    int64_t n;
    double theta;
    int leaf_size;
    int n_sys;                  // 0: one system
    const int64_t *sys_off;     // host offsets [n_sys + 1] (batched)
};

petar_status alloc_build_a(petar_ctx *ctx, const BuildArgs &a) {
    const size_t N = (size_t)a.n;
    const int n_boxes = a.n_sys > 0 ? a.n_sys : 1;
    const int64_t scan_need = scan_ws_elems(a.n + 1);  // the cell-count scan
    TRY(ensure(ctx, ctx->key0, N * 8));
    TRY(ensure(ctx, ctx->key1, N * 8));
    TRY(ensure(ctx, ctx->val0, N * 4));
    TRY(ensure(ctx, ctx->val1, N * 4));
    TRY(ensure(ctx, ctx->sort_ws, (size_t)sort_ws_bytes(a.n)));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_need * 8));
    TRY(ensure(ctx, ctx->bbox_part, (size_t)bbox_partial_blocks(a.n) * 6 * 8));
    TRY(ensure(ctx, ctx->rootbox, sizeof(RootBox) * (size_t)n_boxes));
    TRY(ensure(ctx, ctx->status, sizeof(Status)));
    TRY(ensure(ctx, ctx->emit, (N + kDeepWords) * 4));  // + the deepest-level words
    TRY(ensure(ctx, ctx->base, (N + 1) * 8));
    TRY(ensure(ctx, ctx->ps, N * sizeof(double4)));
    TRY(ensure(ctx, ctx->orig, N * 4));
    TRY(ensure(ctx, ctx->rank, N * 4));
    TRY(ensure(ctx, ctx->level_off, 32 * 4));
    if (a.n_sys > 0) TRY(ensure(ctx, ctx->sys_off, (size_t)(a.n_sys + 1) * 8));
    return PETAR_OK;
}

petar_status alloc_build_b(petar_ctx *ctx, int64_t node_cap) {
    const size_t M = (size_t)node_cap;
    const int64_t n = ctx->n;
    TRY(ensure(ctx, ctx->nd_lo, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_hi, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_com, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_S, M * 6 * 8));
    TRY(ensure(ctx, ctx->nd_q, M * 2 * sizeof(float4)));
    TRY(ensure(ctx, ctx->nd_info, M * sizeof(uint4)));
    TRY(ensure(ctx, ctx->nd_parent, M * 4));
    TRY(ensure(ctx, ctx->pre_info, M * sizeof(uint4)));
    TRY(ensure(ctx, ctx->pre_parent, M * 4));
    TRY(ensure(ctx, ctx->pre_nchild, M * 4));
    TRY(ensure(ctx, ctx->new_of_old, M * 4));
    TRY(ensure(ctx, ctx->lkey0, M * 8));
    TRY(ensure(ctx, ctx->lkey1, M * 8));
    TRY(ensure(ctx, ctx->lval0, M * 4));
    TRY(ensure(ctx, ctx->lval1, M * 4));
    TRY(ensure(ctx, ctx->sort_ws, (size_t)sort_ws_bytes(node_cap > n ? node_cap : n)));
    return PETAR_OK;
}

// Phase A. The sorted keys end in key0 (8 passes).
void enqueue_build_a(petar_ctx *ctx, const BuildArgs &a, hipStream_t s) {
    zero_status(ctx, s);
    const int n_boxes = a.n_sys > 0 ? a.n_sys : 1;
    const int levels = a.n_sys > 0 ? kBatchLevels : kMaxLevel;
    RootBox *rb = ptr<RootBox>(ctx->rootbox);
    fill_i64(ptr<int64_t>(ctx->rootbox), 0, (int64_t)(sizeof(RootBox) / 8) * n_boxes, s);
    uint64_t *k = ptr<uint64_t>(ctx->key0), *ka = ptr<uint64_t>(ctx->key1);
    uint32_t *v = ptr<uint32_t>(ctx->val0), *va = ptr<uint32_t>(ctx->val1);
    if (a.n_sys > 0) {
        const int64_t *off = ptr<int64_t>(ctx->sys_off);
        launch_bbox_systems(a.pos, a.mass, a.n, off, a.n_sys, rb, s);
        launch_keys_systems(a.pos, a.n, off, a.n_sys, rb, k, v, s);
    } else {
        launch_bbox(a.pos, a.mass, a.n, ptr<double>(ctx->bbox_part), rb, s);
        launch_keys(a.pos, a.n, rb, k, v, s);
    }
    radix_sort(&k, &v, &ka, &va, a.n, 8, ctx->sort_ws.p, s);
    launch_gather_particles(a.pos, a.mass, v, a.n, ptr<double4>(ctx->ps), ptr<uint32_t>(ctx->orig),
                            ptr<uint32_t>(ctx->rank), s);
    uint32_t *deep_slots = ptr<uint32_t>(ctx->emit) + a.n;
    fill_u32(deep_slots, 0, kDeepWords, s);
    launch_octree_count(k, a.n, a.leaf_size, levels, ptr<uint32_t>(ctx->emit), deep_slots, s);
    scan_u32_to_i64(ptr<uint32_t>(ctx->emit), ptr<int64_t>(ctx->base), a.n,
                    ptr<int64_t>(ctx->scan_ws), s);
    launch_build_head(ptr<int64_t>(ctx->base), a.n, rb, deep_slots, ptr<Status>(ctx->status), s);
}

// Phase B with cell arrays of node_cap entries (the cell count is read on the
// device; more cells than node_cap raise Status::cell_overflow). The
// bottom-up passes launch levels deep-1 .. 0 (no cell deeper than deep has
// children).
void enqueue_build_b(petar_ctx *ctx, const BuildArgs &a, int64_t node_cap, int deep,
                     hipStream_t s) {
    const int levels = a.n_sys > 0 ? kBatchLevels : kMaxLevel;
    TreeDev t = tree_view(ctx);
    t.n_nodes = node_cap;
    PreOrder pre = pre_view(ctx);
    Status *st = ptr<Status>(ctx->status);
    fill_u32(pre.nchild, 0, node_cap, s);
    uint64_t *lk = ptr<uint64_t>(ctx->lkey0), *lka = ptr<uint64_t>(ctx->lkey1);
    uint32_t *lv = ptr<uint32_t>(ctx->lval0), *lva = ptr<uint32_t>(ctx->lval1);
    const uint64_t *k = ptr<uint64_t>(ctx->key0);
    launch_octree_write(k, a.n, a.leaf_size, levels, ptr<int64_t>(ctx->base), pre, lk, lv,
                        node_cap, st, s);
    radix_sort(&lk, &lv, &lka, &lva, node_cap, 1, ctx->sort_ws.p, s,
               t.n_nodes_dev);
    launch_relayout(lv, pre, ptr<RootBox>(ctx->rootbox), k, levels, t,
                    ptr<uint32_t>(ctx->level_off), s);
    launch_moments(t, deep, s);
    launch_tree_summary(t, st, s);
}

void set_tree_state(petar_ctx *ctx, const BuildArgs &a, int64_t node_cap, int deep) {
    ctx->n = a.n;
    ctx->n_nodes = node_cap;
    ctx->levels = a.n_sys > 0 ? kBatchLevels : kMaxLevel;
    ctx->deep = deep;
    ctx->theta = a.theta;
    ctx->leaf_size = a.leaf_size;
    ctx->n_sys = a.n_sys > 0 ? a.n_sys : 1;
}

petar_status copy_offsets(petar_ctx *ctx, const BuildArgs &a, hipStream_t s) {
    if (a.n_sys > 0)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->sys_off.p, a.sys_off, (size_t)(a.n_sys + 1) * 8,
                                    hipMemcpyHostToDevice, s));
    return PETAR_OK;
}

petar_status build_eager(petar_ctx *ctx, const BuildArgs &a) {
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    ctx->have_tree = false;
    ctx->have_counts = false;
    ctx->target = nullptr;
    ctx->n = a.n;
    TRY(alloc_build_a(ctx, a));
    TRY(copy_offsets(ctx, a, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
    enqueue_build_a(ctx, a, s);
    HIP_TRY(ctx, hipGetLastError());
    TRY(read_status(ctx, s));  // cell count, input check, deepest level
    if (ctx->host_status->bad_input)
        return fail(ctx, PETAR_E_INVALID, "non-finite position or mass, or negative mass");
    const int64_t n_nodes = ctx->host_status->cells;
    if (n_nodes < 1 || n_nodes >= (int64_t)kNone)
        return fail(ctx, PETAR_E_INTERNAL, "cell count %lld out of range", (long long)n_nodes);
    const int levels = a.n_sys > 0 ? kBatchLevels : kMaxLevel;
    const uint32_t deep = ctx->host_status->deep;
    if (deep > (uint32_t)levels)
        return fail(ctx, PETAR_E_INTERNAL, "deepest cell level %lld out of range", (long long)deep);
    TRY(alloc_build_b(ctx, n_nodes));
    enqueue_build_b(ctx, a, n_nodes, (int)deep, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    // No wait for the second half: it reads only the context's sorted copies
    // and cannot fail (the cell arrays hold exactly n_nodes cells), so the
    // next call's launches queue behind it. Its counters are read with the
    // next status read (settle_build_stats).
    set_tree_state(ctx, a, n_nodes, (int)deep);
    ctx->have_tree = true;
    ctx->stats = petar_stats{};
    ctx->stats.n = a.n;
    ctx->stats.n_nodes = n_nodes;
    ctx->stats.workspace_bytes = ctx->ws_bytes;
    ctx->build_stats_pending = true;
    return PETAR_OK;
}

// ---------------------------------------------------------------- force
struct ForceArgs {
    int group_size;
    const double *r_in, *r_out, *r_search;
    double *acc, *pot;
    petar_nblist *nb;
    double *kick_vel = nullptr;  // fused kick (petar_force_long_kick)
    double kick_dt = 0.0;
};

petar_status alloc_force(petar_ctx *ctx, const ForceArgs &a) {
    const int64_t n = ctx->n, n_nodes = ctx->n_nodes;
    const int prec = ctx->params.precision, ipl = ctx->params.i_per_lane;
    int &fw = ctx->force_waves[prec][ipl];
    if (fw == 0) fw = force_resident_waves(prec, ipl, ctx->device);
    if (a.nb && ctx->nb_waves == 0) ctx->nb_waves = nb_resident_waves(ctx->device);
    int spill_waves = fw > ctx->nb_waves ? fw : ctx->nb_waves;
    TRY(ensure(ctx, ctx->rr, (size_t)n * sizeof(double2)));
    TRY(ensure(ctx, ctx->rsk, (size_t)n * 8));
    TRY(ensure(ctx, ctx->gflag, (size_t)(n_nodes + 1) * 4));
    TRY(ensure(ctx, ctx->gpos, (size_t)(n_nodes + 1) * 4));
    TRY(ensure(ctx, ctx->groups, (size_t)n_nodes * 4));
    TRY(ensure(ctx, ctx->queue, 64 * 4));
    TRY(ensure(ctx, ctx->spill, (size_t)spill_waves * (size_t)kSpillCap * 4));
    if (ctx->params.record_counts) TRY(ensure(ctx, ctx->counts, (size_t)n * 4 * 4));
    if (a.nb) {
        TRY(ensure(ctx, ctx->nbcnt, (size_t)(n + 1) * 4));
        // near-leaf hand-over of the force walk; grown after a call overflowed
        auto cap = [](uint64_t want, uint32_t have) {
            if (want < have) want = have;
            return (uint32_t)(want > 0xffffffffull ? 0xffffffffull : want);
        };
        ctx->nbhead_cap = cap((uint64_t)n_nodes + 4096, ctx->nbhead_cap);
        ctx->nbleaf_cap = cap((uint64_t)n * 2 + 4096, ctx->nbleaf_cap);
        TRY(ensure(ctx, ctx->nbhead, (size_t)ctx->nbhead_cap * sizeof(uint4)));
        TRY(ensure(ctx, ctx->nbleaf, (size_t)ctx->nbleaf_cap * sizeof(uint2)));
        // rows: a first guess of 32 entries a particle (no more than the
        // caller's list capacity, which is all the exact fallback needs), then
        // what the previous call needed (finish_force grows it and redoes the
        // passes)
        const int64_t first = std::min<int64_t>(32 * n, a.nb->capacity) + 4096;
        if (ctx->nbrows_cap < first) ctx->nbrows_cap = first;
        TRY(ensure(ctx, ctx->nbrowoff, (size_t)(n + 1) * 8));
        TRY(ensure(ctx, ctx->nbrows, (size_t)ctx->nbrows_cap * 4));
    }
    if (ctx->target) {
        TRY(ensure(ctx, ctx->tflag, (size_t)n * 4));
        TRY(ensure(ctx, ctx->tpos, (size_t)(n + 1) * 4));
        TRY(ensure(ctx, ctx->tidx, (size_t)n * 4));
    }
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(n_nodes + n + 1) * 8));
    return PETAR_OK;
}

// The neighbour passes over the near leaves handed over by the force walk
// (the walk-based pass takes over on the device if the records overflowed).
// Rows: kBounds, the force kernel has stored each target's list bound in
// nbcnt (input order) and their prefix sum places the rows; kRedo, the
// rows of the previous passes again (they outgrew the scratch, which has
// been enlarged); kExact, a counting pass first gives exact bounds (when the
// walk's bounds ask for more rows than the scratch may hold). kRedo and
// kExact run on the kept records and clear the pass queues and the
// long-list count again.
enum NbRows { kBounds, kRedo, kExact };

void enqueue_nb(petar_ctx *ctx, petar_nblist *nb, hipStream_t s, bool timed, NbRows mode) {
    const int64_t n = ctx->n;
    TreeDev t = tree_view(ctx);
    Status *st = ptr<Status>(ctx->status);
    uint32_t *queue = ptr<uint32_t>(ctx->queue);
    NbRecords rec;
    rec.head = ptr<uint4>(ctx->nbhead);
    rec.leaf = ptr<uint2>(ctx->nbleaf);
    rec.count = queue + 16;  // [16] headers, [17] leaf entries (zeroed with the queue)
    rec.head_cap = ctx->nbhead_cap;
    rec.leaf_cap = ctx->nbleaf_cap;
    const uint32_t *groups = ptr<uint32_t>(ctx->groups);
    uint32_t *spill = ptr<uint32_t>(ctx->spill);
    uint32_t *cnt = ptr<uint32_t>(ctx->nbcnt);
    int64_t *row_off = ptr<int64_t>(ctx->nbrowoff);
    int32_t *rows = ptr<int32_t>(ctx->nbrows);
    int64_t *ws = ptr<int64_t>(ctx->scan_ws);
    if (timed) (void)hipEventRecord(ctx->ev[6], s);
    if (mode != kBounds) fill_u32(queue + 8, 0, 8, s);
    if (mode == kExact) {
        fill_u32(cnt, 0, n + 1, s);
        launch_nb_count_rec(t, rec, st, cnt, s);
        launch_nb_write(t, groups, st, cnt, nullptr, nullptr, 0, spill, queue + 11, rec,
                        ctx->nb_waves, s);
    }
    if (mode != kRedo) scan_u32_to_i64(cnt, row_off, n, ws, s);  // bounds -> rows
    fill_u32(cnt, 0, n + 1, s);  // the counts of the testing pass
    launch_nb_write_rec(t, rec, st, row_off, cnt, rows, ctx->nbrows_cap, s);
    launch_nb_write(t, groups, st, cnt, row_off, rows, ctx->nbrows_cap, spill, queue + 9, rec,
                    ctx->nb_waves, s);
    scan_u32_to_i64(cnt, nb->offsets_dev, n, ws, s);
    launch_nb_sort(row_off, rows, nb->offsets_dev, nb->idx_dev, n, nb->capacity, st, cnt,
                   queue + 10, s);
    launch_nb_summary(nb->offsets_dev, row_off, n, queue + 16, st, s);
    if (timed) (void)hipEventRecord(ctx->ev[7], s);
}

// Every launch of the force call; no host synchronisation (capturable).
// `timed` records the stage events (not inside a captured graph).
void enqueue_force(petar_ctx *ctx, const ForceArgs &a, hipStream_t s, bool timed) {
    const int64_t n = ctx->n, n_nodes = ctx->n_nodes;
    const int prec = ctx->params.precision, ipl = ctx->params.i_per_lane;
    const int fw = ctx->force_waves[prec][ipl];
    TreeDev t = tree_view(ctx);
    PreOrder pre = pre_view(ctx);
    Status *st = ptr<Status>(ctx->status);
    uint32_t *queue = ptr<uint32_t>(ctx->queue);
    if (timed) (void)hipEventRecord(ctx->ev[2], s);
    zero_force_status(ctx, s);
    fill_u32(queue, 0, 64, s);
    launch_gather_radii(a.r_in, a.r_out, a.r_search, t, st, s);
    launch_rsmax(t, s);
    launch_group_flags(pre, t, a.group_size, ptr<uint32_t>(ctx->gflag), s);
    scan_u32_to_u32(ptr<uint32_t>(ctx->gflag), ptr<uint32_t>(ctx->gpos), n_nodes,
                    ptr<int64_t>(ctx->scan_ws), s);
    launch_group_compact(pre, t, ptr<uint32_t>(ctx->gflag), ptr<uint32_t>(ctx->gpos),
                         ptr<uint32_t>(ctx->groups), st, s);
    const uint32_t *tpos = nullptr, *tidx = nullptr;
    if (ctx->target) {  // targets of each group: a compacted list in Morton order
        launch_target_flags(ctx->target, t, ptr<uint32_t>(ctx->tflag), a.acc, a.pot, s);
        scan_u32_to_u32(ptr<uint32_t>(ctx->tflag), ptr<uint32_t>(ctx->tpos), n,
                        ptr<int64_t>(ctx->scan_ws), s);
        launch_target_compact(ptr<uint32_t>(ctx->tflag), ptr<uint32_t>(ctx->tpos), n,
                              ptr<uint32_t>(ctx->tidx), s);
        tpos = ptr<uint32_t>(ctx->tpos);
        tidx = ptr<uint32_t>(ctx->tidx);
    }

    ForceLaunch f;
    f.t = t;
    f.groups = ptr<uint32_t>(ctx->groups);
    f.st_in = st;
    f.st = st;
    f.th2 = ctx->theta * ctx->theta;
    f.G = ctx->params.G;
    f.acc = a.acc;
    f.pot = a.pot;
    f.spill = ptr<uint32_t>(ctx->spill);
    f.queue = queue;
    f.counts = ctx->params.record_counts ? ptr<int32_t>(ctx->counts) : nullptr;
    f.nb.head = a.nb ? ptr<uint4>(ctx->nbhead) : nullptr;
    f.nb.leaf = a.nb ? ptr<uint2>(ctx->nbleaf) : nullptr;
    f.nb.count = queue + 16;  // [16] headers, [17] leaf entries (zeroed with the queue)
    f.nb.head_cap = a.nb ? ctx->nbhead_cap : 0;
    f.nb.leaf_cap = a.nb ? ctx->nbleaf_cap : 0;
    f.nb_bound = a.nb ? ptr<uint32_t>(ctx->nbcnt) : nullptr;
    f.kick_vel = a.kick_vel;
    f.kick_dt = a.kick_dt;
    f.tpos = tpos;
    f.tidx = tidx;
    f.precision = prec;
    f.ipl = ipl;
    if (timed) (void)hipEventRecord(ctx->ev[4], s);
    launch_force(f, fw, s);
    if (timed) (void)hipEventRecord(ctx->ev[5], s);
    if (a.nb) enqueue_nb(ctx, a.nb, s, timed, kBounds);
    if (timed) (void)hipEventRecord(ctx->ev[3], s);
}

// Reads the status words after a force call and fills the statistics.
petar_status finish_force(petar_ctx *ctx, const ForceArgs &a, hipStream_t s, bool timed) {
    HIP_TRY(ctx, hipGetLastError());
    TRY(read_status(ctx, s));
    TRY(settle_build_stats(ctx, true));
    const Status &h = *ctx->host_status;
    bool exact = false;
    if (a.nb && !h.invalid_radii && !h.stack_overflow && !h.cell_overflow &&
        h.nb_rows > ctx->nbrows_cap) {
        // The rows outgrew the scratch (nothing was written): enlarge it and
        // run the neighbour passes again on the kept records (a captured
        // graph holds the old scratch and is captured again). Rows beyond
        // 256 entries a particle (degenerate leaves, huge search radii) or
        // the workspace cap are not taken: exact counts bound the rows
        // instead, which then need no more than the caller's capacity.
        const int64_t want = h.nb_rows + h.nb_rows / 16 + 4096;
        const int64_t limit = std::max<int64_t>(256 * ctx->n, int64_t(1) << 24);
        const int64_t cap_bytes = ctx->params.workspace_cap;
        const int64_t after = ctx->ws_bytes - (int64_t)ctx->nbrows.cap + want * 4;
        exact = want > limit || (cap_bytes > 0 && after > cap_bytes);
        if (!exact) {
            ctx->nbrows_cap = want;
        } else if (a.nb->capacity + 4096 > ctx->nbrows_cap) {
            ctx->nbrows_cap = a.nb->capacity + 4096;
        }
        if ((size_t)ctx->nbrows_cap * 4 > ctx->nbrows.cap) {
            TRY(ensure(ctx, ctx->nbrows, (size_t)ctx->nbrows_cap * 4));
            ctx->graph_stale = true;
        }
        enqueue_nb(ctx, a.nb, s, timed, exact ? kExact : kRedo);
        HIP_TRY(ctx, hipGetLastError());
        TRY(read_status(ctx, s));
    }
    if (h.invalid_radii)
        return fail(ctx, PETAR_E_INVALID,
                    "radii must be finite with 0 <= r_in < r_out <= r_search for every particle");
    if (h.stack_overflow)
        return fail(ctx, PETAR_E_INTERNAL, "tree-walk stack exceeded %d entries", kSpillCap);
    ctx->have_counts = ctx->params.record_counts != 0;
    ctx->stats.n_groups = h.n_groups;
    ctx->stats.inter_pc = (int64_t)h.inter[0];
    ctx->stats.inter_far = (int64_t)h.inter[1];
    ctx->stats.inter_near = (int64_t)h.inter[2];
    if (timed) {
        ctx->stats.ms_force = elapsed(ctx->ev[2], ctx->ev[3]);
        ctx->stats.ms_force_kernel = elapsed(ctx->ev[4], ctx->ev[5]);
        ctx->stats.ms_nb = a.nb ? elapsed(ctx->ev[6], ctx->ev[7]) : 0.0;
    }
    ctx->stats.workspace_bytes = ctx->ws_bytes;
    if (a.nb) {
        const uint32_t used[2] = {h.rec_used[0], h.rec_used[1]};  // hand-over claimed
        auto grow = [](uint32_t need) {
            uint64_t want = (uint64_t)need + need / 4;
            return (uint32_t)(want > 0xffffffffull ? 0xffffffffull : want);
        };
        if (used[0] > ctx->nbhead_cap || used[1] > ctx->nbleaf_cap) {  // grow for the next call
            if (used[0] > ctx->nbhead_cap) ctx->nbhead_cap = grow(used[0]);
            if (used[1] > ctx->nbleaf_cap) ctx->nbleaf_cap = grow(used[1]);
            ctx->graph_stale = true;
        }
        // exact rows that do not fit hold more entries than the capacity
        a.nb->required = exact && h.nb_rows > ctx->nbrows_cap ? h.nb_rows : h.nb_total;
        ctx->stats.nb_total = a.nb->required;
        if (a.nb->required > a.nb->capacity)
            return fail(ctx, PETAR_E_NB_OVERFLOW, "neighbour capacity %lld < required %lld",
                        (long long)a.nb->capacity, (long long)a.nb->required);
    }
    return PETAR_OK;
}

}  // namespace

extern "C" {

petar_status petar_tree_build(petar_ctx *ctx, const double *pos, const double *mass, int64_t n,
                              double theta, int leaf_size) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_build_args(pos, mass, n, theta, leaf_size))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    BuildArgs a{pos, mass, n, theta, leaf_size, 0, nullptr};
    return build_eager(ctx, a);
}

petar_status petar_batch_build(petar_ctx *ctx, int n_sys, const int64_t *sys_offsets,
                               const double *pos, const double *mass, double theta,
                               int leaf_size) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_batch_args(n_sys, sys_offsets))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    const int64_t n = sys_offsets[n_sys];
    if (const char *m = check_build_args(pos, mass, n, theta, leaf_size))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    BuildArgs a{pos, mass, n, theta, leaf_size, n_sys, sys_offsets};
    return build_eager(ctx, a);
}

petar_status petar_set_targets(petar_ctx *ctx, const uint8_t *target) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    if (!ctx->have_tree) return fail(ctx, PETAR_E_STATE, "petar_tree_build has not succeeded");
    ctx->target = target;
    return PETAR_OK;
}

petar_status petar_force_long(petar_ctx *ctx, int group_size, const double *r_in,
                              const double *r_out, const double *r_search, double *acc,
                              double *pot, petar_nblist *nb) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_force_args(group_size, r_in, r_out, r_search, acc, pot, nb))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    if (!ctx->have_tree) return fail(ctx, PETAR_E_STATE, "petar_tree_build has not succeeded");
    if (nb && ctx->target)
        return fail(ctx, PETAR_E_INVALID, "neighbour lists need every particle as a target "
                                          "(petar_set_targets(ctx, NULL) first)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ForceArgs a{group_size, r_in, r_out, r_search, acc, pot, nb};
    TRY(alloc_force(ctx, a));
    enqueue_force(ctx, a, ctx->stream, true);
    return finish_force(ctx, a, ctx->stream, true);
}

petar_status petar_force_long_kick(petar_ctx *ctx, int group_size, const double *r_in,
                                   const double *r_out, const double *r_search, double *acc,
                                   double *pot, petar_nblist *nb, double *vel, double dt) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_force_args(group_size, r_in, r_out, r_search, acc, pot, nb))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (!vel) return fail(ctx, PETAR_E_INVALID, "vel must not be NULL");
    if (!std::isfinite(dt)) return fail(ctx, PETAR_E_INVALID, "dt must be finite");
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    if (!ctx->have_tree) return fail(ctx, PETAR_E_STATE, "petar_tree_build has not succeeded");
    if (nb && ctx->target)
        return fail(ctx, PETAR_E_INVALID, "neighbour lists need every particle as a target "
                                          "(petar_set_targets(ctx, NULL) first)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ForceArgs a{group_size, r_in, r_out, r_search, acc, pot, nb, vel, dt};
    TRY(alloc_force(ctx, a));
    enqueue_force(ctx, a, ctx->stream, true);
    return finish_force(ctx, a, ctx->stream, true);
}

petar_status petar_step_graph(petar_ctx *ctx, int n_sys, const int64_t *sys_offsets,
                              const double *pos, const double *mass, int64_t N, double theta,
                              int leaf_size, int group_size, const double *r_in,
                              const double *r_out, const double *r_search, double *acc,
                              double *pot, petar_nblist *nb) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (n_sys < 0) return fail(ctx, PETAR_E_INVALID, "n_sys must be >= 0");
    if (n_sys > 0) {
        if (const char *m = check_batch_args(n_sys, sys_offsets))
            return fail(ctx, PETAR_E_INVALID, "%s", m);
        N = sys_offsets[n_sys];
    }
    if (const char *m = check_build_args(pos, mass, N, theta, leaf_size))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (const char *m = check_force_args(group_size, r_in, r_out, r_search, acc, pot, nb))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    BuildArgs ba{pos, mass, N, theta, leaf_size, n_sys, sys_offsets};
    ForceArgs fa{group_size, r_in, r_out, r_search, acc, pot, nb};
    ctx->target = nullptr;  // the step builds a new tree: every particle is a target

    // everything the captured launches depend on
    std::vector<int64_t> key = {(int64_t)(intptr_t)pos, (int64_t)(intptr_t)mass, N, n_sys,
                                leaf_size, group_size, (int64_t)(intptr_t)r_in,
                                (int64_t)(intptr_t)r_out, (int64_t)(intptr_t)r_search,
                                (int64_t)(intptr_t)acc, (int64_t)(intptr_t)pot,
                                nb ? (int64_t)(intptr_t)nb->offsets_dev : 0,
                                nb ? (int64_t)(intptr_t)nb->idx_dev : 0, nb ? nb->capacity : -1,
                                ctx->params.precision, ctx->params.i_per_lane,
                                ctx->params.record_counts};
    double th = theta, g = ctx->params.G;
    int64_t bits;
    memcpy(&bits, &th, 8);
    key.push_back(bits);
    memcpy(&bits, &g, 8);
    key.push_back(bits);
    for (int sIdx = 0; sIdx <= n_sys && n_sys > 0; sIdx++) key.push_back(sys_offsets[sIdx]);

    if (ctx->graph_stale || !ctx->gexec || key != ctx->graph_key) {
        // eager step (its results are this call's), then capture with room for
        // twice as many cells as this tree has
        drop_graph(ctx);
        TRY(build_eager(ctx, ba));
        TRY(alloc_force(ctx, fa));
        enqueue_force(ctx, fa, ctx->stream, true);
        petar_status st = finish_force(ctx, fa, ctx->stream, true);
        if (st != PETAR_OK && st != PETAR_E_NB_OVERFLOW) return st;
        const int64_t node_cap = 2 * ctx->n_nodes + 1024;
        ctx->have_tree = false;  // the arrays may move; the next replay rebuilds them
        TRY(alloc_build_b(ctx, node_cap));
        const int64_t n_nodes_now = ctx->n_nodes;
        ctx->n_nodes = node_cap;
        TRY(alloc_force(ctx, fa));
        ctx->n_nodes = n_nodes_now;
        if (!ctx->cap_stream)
            HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->cap_stream;
        // (no stage events inside the graph: replays do not update events
        // recorded by captured nodes, so a replay is timed as a whole)
        HIP_TRY(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        enqueue_build_a(ctx, ba, cs);
        // a replay's tree may be deeper than this one: every level is launched
        const int all_levels = ba.n_sys > 0 ? kBatchLevels : kMaxLevel;
        enqueue_build_b(ctx, ba, node_cap, all_levels, cs);
        set_tree_state(ctx, ba, node_cap, all_levels);
        enqueue_force(ctx, fa, cs, false);
        hipError_t e = hipStreamEndCapture(cs, &ctx->graph);
        if (e == hipSuccess) e = hipGetLastError();  // launches inside the capture
        if (e == hipSuccess) e = hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(ctx);
            return fail(ctx, PETAR_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        }
        ctx->graph_key = key;
        ctx->node_cap = node_cap;
        ctx->graph_stale = false;
        ctx->n_nodes = n_nodes_now;
        ctx->stats.ms_graph = 0.0;
        return st;
    }
    // replay
    hipStream_t s = ctx->stream;
    set_tree_state(ctx, ba, ctx->node_cap, ba.n_sys > 0 ? kBatchLevels : kMaxLevel);
    ctx->have_tree = false;
    HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
    HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    petar_status st = finish_force(ctx, fa, s, false);
    const Status &h = *ctx->host_status;
    if (h.cell_overflow) {  // tree outgrew the captured capacity: redo eagerly, recapture next
        ctx->graph_stale = true;
        TRY(build_eager(ctx, ba));
        TRY(alloc_force(ctx, fa));
        enqueue_force(ctx, fa, ctx->stream, true);
        return finish_force(ctx, fa, ctx->stream, true);
    }
    ctx->have_tree = true;
    ctx->stats.n = N;
    ctx->stats.n_nodes = h.n_nodes;
    ctx->stats.n_leaves = h.n_leaves;
    ctx->stats.max_level = h.max_level;
    ctx->stats.ms_build = 0.0;
    ctx->build_stats_pending = false;
    ctx->stats.ms_force = 0.0;
    ctx->stats.ms_force_kernel = 0.0;
    ctx->stats.ms_nb = 0.0;
    ctx->stats.ms_graph = elapsed(ctx->ev[0], ctx->ev[1]);
    return st;
}

petar_status petar_copy_counts(petar_ctx *ctx, int32_t *counts) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (!counts) return fail(ctx, PETAR_E_INVALID, "counts is NULL");
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    if (!ctx->have_counts)
        return fail(ctx, PETAR_E_STATE, "no counts recorded (set params.record_counts first)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpyAsync(counts, ctx->counts.p, (size_t)ctx->n * 16,
                                hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PETAR_OK;
}

petar_status petar_get_stats(petar_ctx *ctx, petar_stats *out) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (!out) return fail(ctx, PETAR_E_INVALID, "stats is NULL");
    if (ctx->device != PETAR_NO_DEVICE) {
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        TRY(settle_build_stats(ctx, false));
    }
    ctx->stats.workspace_bytes = ctx->ws_bytes;
    *out = ctx->stats;
    return PETAR_OK;
}

}  // extern "C"
