// C ABI of libpetar: context, argument checks, workspace, and the ordered
// launches of the tree build and the long-range force (see include/petar.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

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

struct petar_ctx {
    int device = PETAR_NO_DEVICE;
    hipStream_t stream = nullptr;
    petar_params params{};
    std::string err;
    int64_t ws_bytes = 0;

    // tree build
    DevBuf key0, key1, val0, val1, sort_ws, scan_ws, bbox_part, rootbox, status, emit, base;
    DevBuf ps, orig, rr, rsk;
    DevBuf nd_lo, nd_hi, nd_com, nd_S, nd_info, nd_child, nd_parent;
    DevBuf level_count, level_off, level_ws, level_nodes;
    // force
    DevBuf gflag, gpos, groups, spill, queue, counts, nbcnt, radii_ws;

    Status *host_status = nullptr;  // pinned
    int64_t *host_scalar = nullptr; // pinned

    bool have_tree = false;
    bool have_counts = false;
    int64_t n = 0;
    double theta = 0.0;
    int leaf_size = 0;
    int64_t n_nodes = 0;
    uint64_t *sorted_key = nullptr;

    int force_waves[2][5] = {{0}};
    int nb_waves = 0;

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
        hipFree(b.p);
        ctx->ws_bytes -= (int64_t)b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
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

TreeDev tree_view(petar_ctx *c) {
    TreeDev t;
    t.ps = ptr<double4>(c->ps);
    t.rr = ptr<double2>(c->rr);
    t.rsk = ptr<double>(c->rsk);
    t.orig = ptr<uint32_t>(c->orig);
    t.nd_lo = ptr<double4>(c->nd_lo);
    t.nd_hi = ptr<double4>(c->nd_hi);
    t.nd_com = ptr<double4>(c->nd_com);
    t.nd_S = ptr<double>(c->nd_S);
    t.nd_info = ptr<uint4>(c->nd_info);
    t.nd_child = ptr<uint32_t>(c->nd_child);
    t.nd_parent = ptr<uint32_t>(c->nd_parent);
    t.n = c->n;
    t.n_nodes = c->n_nodes;
    return t;
}

petar_status zero_status(petar_ctx *c) {
    fill_i64(ptr<int64_t>(c->status), 0, (int64_t)(sizeof(Status) / sizeof(int64_t)), c->stream);
    return PETAR_OK;
}

petar_status read_status(petar_ctx *c) {
    HIP_TRY(c, hipMemcpyAsync(c->host_status, c->status.p, sizeof(Status), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PETAR_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

void free_all(petar_ctx *c) {
    DevBuf *bufs[] = {&c->key0,     &c->key1,        &c->val0,       &c->val1,       &c->sort_ws,
                      &c->scan_ws,  &c->bbox_part,   &c->rootbox,    &c->status,     &c->emit,
                      &c->base,     &c->ps,          &c->orig,       &c->rr,         &c->rsk,
                      &c->nd_lo,    &c->nd_hi,       &c->nd_com,     &c->nd_S,       &c->nd_info,
                      &c->nd_child, &c->nd_parent,   &c->level_count, &c->level_off, &c->level_ws,
                      &c->level_nodes, &c->gflag,    &c->gpos,       &c->groups,     &c->spill,
                      &c->queue,    &c->counts,      &c->nbcnt,      &c->radii_ws};
    for (DevBuf *b : bufs) {
        if (b->p) hipFree(b->p);
        b->p = nullptr;
        b->cap = 0;
    }
    c->ws_bytes = 0;
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
        if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_scalar, 4 * sizeof(int64_t));
        for (int k = 0; k < 8 && e == hipSuccess; k++) e = hipEventCreate(&c->ev[k]);
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

petar_status petar_tree_build(petar_ctx *ctx, const double *pos, const double *mass, int64_t n,
                              double theta, int leaf_size) {
    if (!ctx) return fail(nullptr, PETAR_E_INVALID, "ctx is NULL");
    if (const char *m = check_build_args(pos, mass, n, theta, leaf_size))
        return fail(ctx, PETAR_E_INVALID, "%s", m);
    if (ctx->device == PETAR_NO_DEVICE) return fail(ctx, PETAR_E_NODEVICE, "no device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    ctx->have_tree = false;
    ctx->have_counts = false;

    const size_t N = (size_t)n;
    int64_t sort_scan = 256 * ((n + 2047) / 2048);
    int64_t scan_need = scan_ws_elems(sort_scan > n + 1 ? sort_scan : n + 1);
    TRY(ensure(ctx, ctx->key0, N * 8));
    TRY(ensure(ctx, ctx->key1, N * 8));
    TRY(ensure(ctx, ctx->val0, N * 4));
    TRY(ensure(ctx, ctx->val1, N * 4));
    TRY(ensure(ctx, ctx->sort_ws, (size_t)sort_ws_bytes(n)));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_need * 8));
    TRY(ensure(ctx, ctx->bbox_part, (size_t)bbox_partial_blocks(n) * 6 * 8));
    TRY(ensure(ctx, ctx->rootbox, sizeof(RootBox)));
    TRY(ensure(ctx, ctx->status, sizeof(Status)));
    TRY(ensure(ctx, ctx->emit, N * 4));
    TRY(ensure(ctx, ctx->base, (N + 1) * 8));
    TRY(ensure(ctx, ctx->ps, N * sizeof(double4)));
    TRY(ensure(ctx, ctx->orig, N * 4));
    TRY(ensure(ctx, ctx->level_count, 32 * 4));
    TRY(ensure(ctx, ctx->level_off, 32 * 4));

    HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
    zero_status(ctx);
    fill_i64(ptr<int64_t>(ctx->rootbox), 0, (int64_t)(sizeof(RootBox) / 8), s);
    RootBox *rb = ptr<RootBox>(ctx->rootbox);
    launch_bbox(pos, mass, n, ptr<double>(ctx->bbox_part), rb, s);
    uint64_t *k = ptr<uint64_t>(ctx->key0), *ka = ptr<uint64_t>(ctx->key1);
    uint32_t *v = ptr<uint32_t>(ctx->val0), *va = ptr<uint32_t>(ctx->val1);
    launch_keys(pos, n, rb, k, v, s);
    radix_sort(&k, &v, &ka, &va, n, ctx->sort_ws.p, ptr<int64_t>(ctx->scan_ws), s);
    launch_gather_particles(pos, mass, v, n, ptr<double4>(ctx->ps), ptr<uint32_t>(ctx->orig), s);
    launch_octree_count(k, n, leaf_size, ptr<uint32_t>(ctx->emit), s);
    scan_u32_to_i64(ptr<uint32_t>(ctx->emit), ptr<int64_t>(ctx->base), n,
                    ptr<int64_t>(ctx->scan_ws), s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, ptr<int64_t>(ctx->base) + n, 8,
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar + 1, &rb->bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int32_t bad = 0;
    memcpy(&bad, ctx->host_scalar + 1, 4);
    if (bad) return fail(ctx, PETAR_E_INVALID, "non-finite position or mass, or negative mass");
    int64_t n_nodes = ctx->host_scalar[0];
    if (n_nodes < 1 || n_nodes >= (int64_t)kNone)
        return fail(ctx, PETAR_E_INTERNAL, "cell count %lld out of range", (long long)n_nodes);

    const size_t M = (size_t)n_nodes;
    TRY(ensure(ctx, ctx->nd_lo, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_hi, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_com, M * sizeof(double4)));
    TRY(ensure(ctx, ctx->nd_S, M * 6 * 8));
    TRY(ensure(ctx, ctx->nd_info, M * sizeof(uint4)));
    TRY(ensure(ctx, ctx->nd_child, M * 8 * 4));
    TRY(ensure(ctx, ctx->nd_parent, M * 4));
    TRY(ensure(ctx, ctx->level_nodes, M * 4));
    TRY(ensure(ctx, ctx->level_ws, (size_t)level_ws_elems(n_nodes) * 4));
    ctx->n = n;
    ctx->n_nodes = n_nodes;
    ctx->sorted_key = k;
    TreeDev t = tree_view(ctx);
    fill_u32(t.nd_child, kNone, n_nodes * 8, s);
    launch_octree_write(k, n, leaf_size, ptr<int64_t>(ctx->base), rb, t, s);
    launch_level_buckets(t, ptr<uint32_t>(ctx->level_count), ptr<uint32_t>(ctx->level_off),
                         ptr<uint32_t>(ctx->level_ws), ptr<uint32_t>(ctx->level_nodes), s);
    for (int L = kMaxLevel; L >= 0; L--)
        launch_moments_level(t, L, ptr<uint32_t>(ctx->level_off), ptr<uint32_t>(ctx->level_nodes),
                             s);
    launch_tree_summary(t, ptr<uint32_t>(ctx->level_count), ptr<Status>(ctx->status), s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    TRY(read_status(ctx));
    ctx->have_tree = true;
    ctx->theta = theta;
    ctx->leaf_size = leaf_size;
    ctx->stats = petar_stats{};
    ctx->stats.n = n;
    ctx->stats.n_nodes = n_nodes;
    ctx->stats.n_leaves = ctx->host_status->n_leaves;
    ctx->stats.max_level = ctx->host_status->max_level;
    ctx->stats.ms_build = elapsed(ctx->ev[0], ctx->ev[1]);
    ctx->stats.workspace_bytes = ctx->ws_bytes;
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
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t n = ctx->n, n_nodes = ctx->n_nodes;
    const int prec = ctx->params.precision, ipl = ctx->params.i_per_lane;
    int &fw = ctx->force_waves[prec][ipl];
    if (fw == 0) fw = force_resident_waves(prec, ipl, ctx->device);
    if (nb && ctx->nb_waves == 0) ctx->nb_waves = nb_resident_waves(ctx->device);
    int spill_waves = fw > ctx->nb_waves ? fw : ctx->nb_waves;

    TRY(ensure(ctx, ctx->rr, (size_t)n * sizeof(double2)));
    TRY(ensure(ctx, ctx->rsk, (size_t)n * 8));
    TRY(ensure(ctx, ctx->gflag, (size_t)(n_nodes + 1) * 4));
    TRY(ensure(ctx, ctx->gpos, (size_t)(n_nodes + 1) * 4));
    TRY(ensure(ctx, ctx->groups, (size_t)n_nodes * 4));
    TRY(ensure(ctx, ctx->queue, 64 * 4));
    TRY(ensure(ctx, ctx->spill, (size_t)spill_waves * (size_t)kSpillCap * 4));
    if (ctx->params.record_counts) TRY(ensure(ctx, ctx->counts, (size_t)n * 4 * 4));
    if (nb) TRY(ensure(ctx, ctx->nbcnt, (size_t)(n + 1) * 4));
    TRY(ensure(ctx, ctx->scan_ws, (size_t)scan_ws_elems(n_nodes + n + 1) * 8));

    TreeDev t = tree_view(ctx);
    Status *st = ptr<Status>(ctx->status);
    uint32_t *queue = ptr<uint32_t>(ctx->queue);
    HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
    zero_status(ctx);
    fill_u32(queue, 0, 64, s);
    launch_gather_radii(r_in, r_out, r_search, t, st, s);
    for (int L = kMaxLevel; L >= 0; L--)
        launch_rsmax_level(t, L, ptr<uint32_t>(ctx->level_off), ptr<uint32_t>(ctx->level_nodes), s);
    launch_group_flags(t, group_size, ptr<uint32_t>(ctx->gflag), s);
    scan_u32_to_u32(ptr<uint32_t>(ctx->gflag), ptr<uint32_t>(ctx->gpos), n_nodes,
                    ptr<int64_t>(ctx->scan_ws), s);
    launch_group_compact(t, ptr<uint32_t>(ctx->gflag), ptr<uint32_t>(ctx->gpos),
                         ptr<uint32_t>(ctx->groups), st, s);

    ForceLaunch f;
    f.t = t;
    f.groups = ptr<uint32_t>(ctx->groups);
    f.st_in = st;
    f.st = st;
    f.th2 = ctx->theta * ctx->theta;
    f.G = ctx->params.G;
    f.acc = acc;
    f.pot = pot;
    f.spill = ptr<uint32_t>(ctx->spill);
    f.queue = queue;
    f.counts = ctx->params.record_counts ? ptr<int32_t>(ctx->counts) : nullptr;
    f.precision = prec;
    f.ipl = ipl;
    HIP_TRY(ctx, hipEventRecord(ctx->ev[4], s));
    launch_force(f, fw, s);
    HIP_TRY(ctx, hipEventRecord(ctx->ev[5], s));
    if (nb) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev[6], s));
        fill_u32(ptr<uint32_t>(ctx->nbcnt), 0, n + 1, s);
        launch_nb_count(t, f.groups, st, ptr<uint32_t>(ctx->nbcnt), f.spill, queue + 8,
                        ctx->nb_waves, s);
        scan_u32_to_i64(ptr<uint32_t>(ctx->nbcnt), nb->offsets_dev, n, ptr<int64_t>(ctx->scan_ws),
                        s);
        launch_nb_write(t, f.groups, st, nb->offsets_dev, nb->idx_dev, nb->capacity, f.spill,
                        queue + 9, ctx->nb_waves, s);
        launch_nb_sort(nb->offsets_dev, nb->idx_dev, n, nb->capacity, st,
                       ptr<uint32_t>(ctx->nbcnt), queue + 10, s);
        HIP_TRY(ctx, hipMemcpyAsync(ctx->host_scalar, nb->offsets_dev + n, 8,
                                    hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipEventRecord(ctx->ev[7], s));
    }
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
    TRY(read_status(ctx));
    const Status &h = *ctx->host_status;
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
    ctx->stats.ms_force = elapsed(ctx->ev[2], ctx->ev[3]);
    ctx->stats.ms_force_kernel = elapsed(ctx->ev[4], ctx->ev[5]);
    ctx->stats.ms_nb = nb ? elapsed(ctx->ev[6], ctx->ev[7]) : 0.0;
    ctx->stats.workspace_bytes = ctx->ws_bytes;
    if (nb) {
        nb->required = ctx->host_scalar[0];
        ctx->stats.nb_total = nb->required;
        if (nb->required > nb->capacity)
            return fail(ctx, PETAR_E_NB_OVERFLOW, "neighbour capacity %lld < required %lld",
                        (long long)nb->capacity, (long long)nb->required);
    }
    return PETAR_OK;
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
    *out = ctx->stats;
    return PETAR_OK;
}

}  // extern "C"
