// Second-stage neighbour filter and clusters (Sec. "Orbit-dependent
// neighbour criterion" and Sec. "Clustering").
//
// Filter: a first-stage candidate j of i is kept iff the pericentre
// separation of the pair's two-body Kepler orbit is below c_v * r_nb,i.
// With r = x_j - x_i, v = v_j - v_i, mu = G (m_i + m_j): specific energy
// eps = v^2/2 - mu/|r|, angular momentum h = |r x v|, eccentricity
// e = sqrt(1 + 2 eps h^2/mu^2) and r_p = h^2 / (mu (1 + e)), over the whole
// orbit; r_p = 0 for coincident particles and |r x v|/|v| for two massless
// ones. FP64 without contraction, in this exact order, so that every
// decision is reproducible by any implementation of the same formula.
//
// Clusters: connected components of the kept pairs. A lock-free union-find
// hooks the larger root under the smaller one (so every component ends with
// its smallest index as root, whatever the order of the unions); reads of
// the parent array are device-coherent atomics, finds halve the paths.
#include "launch.h"

namespace petar {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int threads, int64_t cap) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ double pericentre(double xi, double yi, double zi, double vxi, double vyi, double vzi,
                             double mi, double xj, double yj, double zj, double vxj, double vyj,
                             double vzj, double mj, double G) {
#pragma clang fp contract(off)
    double dx = xj - xi;
    double dy = yj - yi;
    double dz = zj - zi;
    double dvx = vxj - vxi;
    double dvy = vyj - vyi;
    double dvz = vzj - vzi;
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    double hx = dy * dvz - dz * dvy;
    double hy = dz * dvx - dx * dvz;
    double hz = dx * dvy - dy * dvx;
    double h2 = (hx * hx + hy * hy) + hz * hz;
    double mu = G * (mi + mj);
    if (d2 == 0.0) return 0.0;
    if (mu > 0.0) {
        double d = sqrt(d2);
        double eps = 0.5 * v2 - mu / d;
        double e2 = 1.0 + ((2.0 * eps) * h2) / (mu * mu);
        double e = e2 > 0.0 ? sqrt(e2) : 0.0;
        return h2 / (mu * (1.0 + e));
    }
    return v2 > 0.0 ? sqrt(h2 / v2) : sqrt(d2);
}

// keep[e] for every candidate entry, kept count per row; bad indices flag.
__global__ __launch_bounds__(kThreads) void k_filter_mark(FilterArgs a, uint8_t *keep,
                                                          uint32_t *counts, int32_t *bad) {
    const int64_t n = a.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double xi = a.pos[i], yi = a.pos[n + i], zi = a.pos[2 * n + i];
        const double vxi = a.vel[i], vyi = a.vel[n + i], vzi = a.vel[2 * n + i];
        const double mi = a.mass[i];
        const double lim = a.c_v * a.r_nb[i];
        uint32_t c = 0;
        for (int64_t e = a.offsets[i]; e < a.offsets[i + 1]; e++) {
            const int64_t j = a.idx[e];
            if (j < 0 || j >= n) {
                atomicOr(bad, 1);
                keep[e] = 0;
                continue;
            }
            const double rp = pericentre(xi, yi, zi, vxi, vyi, vzi, mi, a.pos[j], a.pos[n + j],
                                         a.pos[2 * n + j], a.vel[j], a.vel[n + j], a.vel[2 * n + j],
                                         a.mass[j], a.G);
            const bool k = rp < lim;
            keep[e] = k ? 1 : 0;
            c += k ? 1u : 0u;
        }
        counts[i] = c;
    }
}

__global__ __launch_bounds__(kThreads) void k_filter_write(FilterArgs a, const uint8_t *keep,
                                                           const int64_t *out_offsets,
                                                           int32_t *out_idx, int64_t capacity) {
    const int64_t n = a.n;
    if (out_offsets[n] > capacity) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t w = out_offsets[i];
        for (int64_t e = a.offsets[i]; e < a.offsets[i + 1]; e++)
            if (keep[e]) out_idx[w++] = a.idx[e];
    }
}

// ------------------------------------------------------------ union-find
__device__ __forceinline__ int32_t load_parent(int32_t *parent, int32_t x) {
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x; every node visited on the way is pointed at its grandparent
// (an ancestor, so concurrent finds and hooks stay consistent: only roots
// are ever hooked, and a node that is not a root never becomes one).
__device__ int32_t uf_find(int32_t *parent, int32_t x) {
    int32_t cur = x, next = load_parent(parent, cur);
    while (cur != next) {
        const int32_t nn = load_parent(parent, next);
        if (next != nn)
            __hip_atomic_store(parent + cur, nn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cur = next;
        next = nn;
    }
    return cur;
}

__global__ __launch_bounds__(kThreads) void k_uf_init(int32_t *parent, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        parent[i] = (int32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_uf_union(const int64_t *offsets, const int32_t *idx,
                                                       int64_t n, int32_t *parent, int32_t *bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = offsets[i]; e < offsets[i + 1]; e++) {
            const int32_t j = idx[e];
            if (j < 0 || j >= n) {
                atomicOr(bad, 1);
                continue;
            }
            while (true) {
                const int32_t ra = uf_find(parent, (int32_t)i), rb = uf_find(parent, j);
                if (ra == rb) break;
                const int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
                if (atomicCAS(parent + hi, hi, lo) == hi) break;  // else hi was hooked: retry
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_uf_label(int32_t *parent, int64_t n, int32_t *label,
                                                       uint32_t *is_root) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = uf_find(parent, (int32_t)i);
        label[i] = r;
        is_root[i] = r == (int32_t)i ? 1u : 0u;
    }
}

// Cluster index of every root (exclusive scan of is_root) -> member counts.
__global__ __launch_bounds__(kThreads) void k_cl_count(const int32_t *label, int64_t n,
                                                       const uint32_t *root_pos, uint32_t *count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(count + root_pos[label[i]], 1u);
}

__global__ __launch_bounds__(kThreads) void k_cl_scatter(const int32_t *label, int64_t n,
                                                         const uint32_t *root_pos,
                                                         const int64_t *cl_offsets,
                                                         uint32_t *cursor, int32_t *members) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = root_pos[label[i]];
        const uint32_t s = atomicAdd(cursor + c, 1u);
        members[cl_offsets[c] + s] = (int32_t)i;
    }
}

}  // namespace

void launch_filter(const FilterArgs &a, uint8_t *keep, uint32_t *counts, int32_t *bad,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_filter_mark, dim3(grid_for(a.n, kThreads, 8192)), dim3(kThreads), 0, s, a,
                       keep, counts, bad);
}

void launch_filter_write(const FilterArgs &a, const uint8_t *keep, const int64_t *out_offsets,
                         int32_t *out_idx, int64_t capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_filter_write, dim3(grid_for(a.n, kThreads, 8192)), dim3(kThreads), 0, s,
                       a, keep, out_offsets, out_idx, capacity);
}

void launch_union_find(const int64_t *offsets, const int32_t *idx, int64_t n, int32_t *parent,
                       int32_t *label, uint32_t *is_root, int32_t *bad, hipStream_t s) {
    const dim3 g(grid_for(n, kThreads, 8192)), b(kThreads);
    hipLaunchKernelGGL(k_uf_init, g, b, 0, s, parent, n);
    hipLaunchKernelGGL(k_uf_union, g, b, 0, s, offsets, idx, n, parent, bad);
    hipLaunchKernelGGL(k_uf_label, g, b, 0, s, parent, n, label, is_root);
}

void launch_cluster_lists(const int32_t *label, int64_t n, const uint32_t *root_pos,
                          uint32_t *count, const int64_t *cl_offsets, uint32_t *cursor,
                          int32_t *members, int phase, hipStream_t s) {
    const dim3 g(grid_for(n, kThreads, 8192)), b(kThreads);
    if (phase == 0)
        hipLaunchKernelGGL(k_cl_count, g, b, 0, s, label, n, root_pos, count);
    else
        hipLaunchKernelGGL(k_cl_scatter, g, b, 0, s, label, n, root_pos, cl_offsets, cursor,
                           members);
}

}  // namespace petar
