// Second-stage neighbour filter, clusters and SDAR groups (Sec. "Orbit-
// dependent neighbour criterion", Sec. "Clustering" and eq. rbin).
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
// Clusters: connected components of the kept pairs by a one-pass union-find
// whose roots are the smallest index of each component (so the result does
// not depend on the order of the unions).
#include <mutex>

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

// SDAR group relation (eq. rbin): r_ij < theta max(r_in,i, r_in,j), as
// d^2 < (theta R)^2 in FP64 without contraction, in this order.
__device__ bool group_pair(double xi, double yi, double zi, double ri, double xj, double yj,
                           double zj, double rj, double theta) {
#pragma clang fp contract(off)
    double dx = xj - xi;
    double dy = yj - yi;
    double dz = zj - zi;
    double d2 = sum_sq3(dx, dy, dz);
    double R = fmax(ri, rj);
    double g = theta * R;
    double g2 = g * g;
    return d2 < g2;
}

// CSR sanity: offsets start at 0 and never decrease (so every row range
// lies inside [0, offsets[n])); raises *bad otherwise.
__global__ __launch_bounds__(kThreads) void k_check_csr(const int64_t *offsets, int64_t n,
                                                        int32_t *bad) {
    int b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (offsets[i + 1] < offsets[i]) b = 1;
        if (i == 0 && offsets[0] != 0) b = 1;
    }
    if (__ballot(b) && lane_id() == 0) atomicOr(bad, 1);
}

// Row of every candidate entry (one thread per row; rows are short).
__global__ __launch_bounds__(kThreads) void k_filter_rows(FilterArgs a, int32_t *row) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = a.offsets[i]; e < a.offsets[i + 1]; e++) row[e] = (int32_t)i;
}

// keep[e] for every candidate entry (one thread per entry, so the gathers
// of the partners' data overlap); an index outside [0, n) raises *bad.
__global__ __launch_bounds__(kThreads) void k_filter_test(FilterArgs a, const int32_t *row,
                                                          int64_t n_cand, uint8_t *keep,
                                                          int32_t *bad) {
    const int64_t n = a.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_cand;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = row[e], j = a.idx[e];
        if (j < 0 || j >= n) {
            atomicOr(bad, 1);
            keep[e] = 0;
            continue;
        }
        if (a.mode == 1) {
            keep[e] = group_pair(a.pos[i], a.pos[n + i], a.pos[2 * n + i], a.r_nb[i], a.pos[j],
                                 a.pos[n + j], a.pos[2 * n + j], a.r_nb[j], a.c_v)
                          ? 1
                          : 0;
            continue;
        }
        const double rp = pericentre(a.pos[i], a.pos[n + i], a.pos[2 * n + i], a.vel[i],
                                     a.vel[n + i], a.vel[2 * n + i], a.mass[i], a.pos[j],
                                     a.pos[n + j], a.pos[2 * n + j], a.vel[j], a.vel[n + j],
                                     a.vel[2 * n + j], a.mass[j], a.G);
        keep[e] = rp < a.c_v * a.r_nb[i] ? 1 : 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_filter_count(FilterArgs a, const uint8_t *keep,
                                                           uint32_t *counts) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c = 0;
        for (int64_t e = a.offsets[i]; e < a.offsets[i + 1]; e++) c += keep[e];
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

// ------------------------------------------------------------ components
// Union-find over the pairs in one pass. Every parent pointer goes to a
// smaller index (parent[v] <= v), so a root is the smallest index of its
// tree. rep() follows the pointers and halves the path behind it with plain
// stores, which only ever replace a non-root's parent by one of its
// ancestors; a union links the larger of two roots under the smaller with a
// compare-and-swap, and a failed swap continues from the value it returns
// (a smaller ancestor), so the loop ends. Plain loads may return older,
// larger ancestors (caches of other XCDs are not coherent inside a
// launch): the chain still leads into the same tree, and every link is
// checked by the swap at the coherence point. After all unions each
// component is one tree whose root is its smallest index.
__device__ __forceinline__ int32_t uf_rep(int32_t *parent, int32_t v) {
    int32_t cur = parent[v];
    if (cur == v) return v;
    int32_t prev = v, next;
    while (cur > (next = parent[cur])) {
        parent[prev] = next;
        prev = cur;
        cur = next;
    }
    return cur;
}

// parent[v] = min(v, smallest in-range neighbour of v). Skipped when the
// CSR check failed (offsets could then reach outside the index array).
__global__ __launch_bounds__(kThreads) void k_uf_init(const int64_t *offsets, const int32_t *idx,
                                                      int64_t n, int32_t *parent,
                                                      const int32_t *csr_bad) {
    if (*csr_bad) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t m = (int32_t)v;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; e++) {
            const int32_t u = idx[e];
            if (u >= 0 && u < m) m = u;
        }
        parent[v] = m;
    }
}

// Every particle straight to the end of its chain after the init, so that
// the finds of the union pass start from flat trees.
__global__ __launch_bounds__(kThreads) void k_uf_flatten(int32_t *parent, int64_t n,
                                                         const int32_t *csr_bad) {
    if (*csr_bad) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = uf_rep(parent, (int32_t)v);
}

__global__ __launch_bounds__(kThreads) void k_uf_union(const int64_t *offsets, const int32_t *idx,
                                                       int64_t n, int32_t *parent, int32_t *bad,
                                                       const int32_t *csr_bad) {
    if (*csr_bad) return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = offsets[v]; e < offsets[v + 1]; e++) {
            const int32_t u = idx[e];
            if (u < 0 || u >= n) {
                atomicOr(bad, 1);
                continue;
            }
            int32_t vr = uf_rep(parent, (int32_t)v), ur = uf_rep(parent, u);
            while (vr != ur) {
                if (vr < ur) {
                    const int32_t old = atomicCAS(parent + ur, ur, vr);
                    if (old == ur) break;
                    ur = old;
                } else {
                    const int32_t old = atomicCAS(parent + vr, vr, ur);
                    if (old == vr) break;
                    vr = old;
                }
            }
        }
    }
}

// Labels from the final trees (every particle alone when the CSR check
// failed, so that the later passes stay in bounds before the error returns).
__global__ __launch_bounds__(kThreads) void k_uf_label(int32_t *parent, int64_t n, int32_t *label,
                                                       uint32_t *is_root, const int32_t *csr_bad) {
    const bool skip = *csr_bad != 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = skip ? (int32_t)v : uf_rep(parent, (int32_t)v);
        label[v] = r;
        is_root[v] = r == (int32_t)v ? 1u : 0u;
    }
}

// Sort keys for the member lists: cluster index per particle (a stable
// radix sort by it keeps the members of each cluster ascending).
__global__ __launch_bounds__(kThreads) void k_cl_keys(const int32_t *label, int64_t n,
                                                      const uint32_t *root_pos, uint64_t *key,
                                                      uint32_t *val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        key[i] = root_pos[label[i]];
        val[i] = (uint32_t)i;
    }
}

// Cluster offsets from the sorted cluster indices: a cluster starts where
// its index first appears (entries past the last cluster stay n).
__global__ __launch_bounds__(kThreads) void k_cl_offsets(const uint64_t *key, int64_t n,
                                                         int64_t *cl_offsets) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || key[i] != key[i - 1]) cl_offsets[key[i]] = i;
}

__global__ __launch_bounds__(kThreads) void k_group_pairs(const int64_t *off, const int32_t *mem,
                                                          int64_t n_groups, const double *pos,
                                                          const double *vel, const double *mass,
                                                          int64_t n, double G, uint32_t *is_pair) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += (int64_t)gridDim.x * blockDim.x) {
        uint32_t f = 0;
        if (off[g + 1] - off[g] == 2) {
            const int64_t i = mem[off[g]], j = mem[off[g] + 1];
            const double r[3] = {pos[j] - pos[i], pos[n + j] - pos[n + i],
                                 pos[2 * n + j] - pos[2 * n + i]};
            const double v[3] = {vel[j] - vel[i], vel[n + j] - vel[n + i],
                                 vel[2 * n + j] - vel[2 * n + i]};
            const double mu = G * (mass[i] + mass[j]);
            double rr;
            const double E = kepler_energy(r, v, mu, &rr);
            f = (rr > 0.0 && E < 0.0) ? 1u : 0u;
        }
        is_pair[g] = f;
    }
}

__global__ __launch_bounds__(kThreads) void k_group_pairs_write(const int64_t *off,
                                                                const int32_t *mem,
                                                                int64_t n_groups,
                                                                const uint32_t *is_pair,
                                                                const uint32_t *pos,
                                                                int32_t *pairs, int64_t cap) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (!is_pair[g]) continue;
        const int64_t k = pos[g];
        pairs[k] = mem[off[g]];
        pairs[cap + k] = mem[off[g] + 1];
    }
}

}  // namespace

void launch_group_pairs(const int64_t *grp_offsets, const int32_t *members, int64_t n_groups,
                        const double *pos, const double *vel, const double *mass, int64_t n,
                        double G, uint32_t *is_pair, hipStream_t s) {
    hipLaunchKernelGGL(k_group_pairs, dim3(grid_for(n_groups, kThreads, 8192)), dim3(kThreads), 0,
                       s, grp_offsets, members, n_groups, pos, vel, mass, n, G, is_pair);
}

void launch_group_pairs_write(const int64_t *grp_offsets, const int32_t *members, int64_t n_groups,
                              const uint32_t *is_pair, const uint32_t *pos, int32_t *pairs,
                              int64_t pair_cap, hipStream_t s) {
    hipLaunchKernelGGL(k_group_pairs_write, dim3(grid_for(n_groups, kThreads, 8192)),
                       dim3(kThreads), 0, s, grp_offsets, members, n_groups, is_pair, pos, pairs,
                       pair_cap);
}

void launch_check_csr(const int64_t *offsets, int64_t n, int32_t *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_csr, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s,
                       offsets, n, bad);
}

void launch_filter(const FilterArgs &a, int64_t n_cand, int32_t *row, uint8_t *keep,
                   uint32_t *counts, int32_t *bad, hipStream_t s) {
    const dim3 g(grid_for(a.n, kThreads, 8192)), b(kThreads);
    hipLaunchKernelGGL(k_filter_rows, g, b, 0, s, a, row);
    hipLaunchKernelGGL(k_filter_test, dim3(grid_for(n_cand, kThreads, 16384)), b, 0, s, a,
                       (const int32_t *)row, n_cand, keep, bad);
    hipLaunchKernelGGL(k_filter_count, g, b, 0, s, a, (const uint8_t *)keep, counts);
}

void launch_filter_write(const FilterArgs &a, const uint8_t *keep, const int64_t *out_offsets,
                         int32_t *out_idx, int64_t capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_filter_write, dim3(grid_for(a.n, kThreads, 8192)), dim3(kThreads), 0, s,
                       a, keep, out_offsets, out_idx, capacity);
}

void launch_components(const int64_t *offsets, const int32_t *idx, int64_t n, int32_t *parent,
                       int32_t *label, uint32_t *is_root, int32_t *bad, const int32_t *csr_bad,
                       hipStream_t s) {
    const dim3 g(grid_for(n, kThreads, 8192)), b(kThreads);
    hipLaunchKernelGGL(k_uf_init, g, b, 0, s, offsets, idx, n, parent, csr_bad);
    hipLaunchKernelGGL(k_uf_flatten, g, b, 0, s, parent, n, csr_bad);
    hipLaunchKernelGGL(k_uf_union, g, b, 0, s, offsets, idx, n, parent, bad, csr_bad);
    hipLaunchKernelGGL(k_uf_label, g, b, 0, s, parent, n, label, is_root, csr_bad);
}

void launch_cluster_keys(const int32_t *label, int64_t n, const uint32_t *root_pos, uint64_t *key,
                         uint32_t *val, hipStream_t s) {
    hipLaunchKernelGGL(k_cl_keys, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, label,
                       n, root_pos, key, val);
}

void launch_cluster_offsets(const uint64_t *sorted_key, int64_t n, int64_t *cl_offsets,
                            hipStream_t s) {
    fill_i64(cl_offsets, n, n + 1, s);
    hipLaunchKernelGGL(k_cl_offsets, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s,
                       sorted_key, n, cl_offsets);
}

namespace {

// The scratch of petar_clusters_noalloc. Its name is a host-side stand-in
// in host code: kernels get the per-device address kept below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

}  // namespace

hipError_t noalloc_scratch(int device, void **out, size_t *bytes) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

}  // namespace petar
