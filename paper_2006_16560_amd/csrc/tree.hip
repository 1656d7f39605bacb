// Octree construction: root cube, Morton keys, radix sort, cells from the
// sorted keys, bottom-up multipoles; and the per-call preparation of the
// force (radii in Morton order, per-cell max search radius, i-groups).
//
// Tree definition (Barnes-Hut octree of the P3T long-range part, Sec.
// "Particle-tree with individual time steps" and the P3T figure caption):
// root cube [lo, lo + ext) with ext the largest extent of the particles;
// integer coordinates q = floor((x - lo) 2^21 / ext) (clamped to 2^21 - 1);
// a cell of level l holds the particles sharing the top l bits of q on
// every axis. A cell with <= leaf_size particles, or at level 21, is a
// leaf; otherwise its non-empty octants are its children. Cells carry mass,
// centre of mass, second moment about it (giving the traceless quadrupole of
// eq. quadtr), particle bounding box and max search radius.
#include "launch.h"

namespace petar {

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int threads = kThreads, int64_t cap = 65535) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// ------------------------------------------------------------------ bbox
constexpr int kBBoxBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_bbox_partial(const double *pos, const double *mass,
                                                           int64_t n, double *part, RootBox *rb) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; d++) {
            double x = pos[(int64_t)d * n + i];
            if (!isfinite(x)) bad = 1;
            lo[d] = fmin(lo[d], x);
            hi[d] = fmax(hi[d], x);
        }
        double m = mass[i];
        if (!isfinite(m) || m < 0.0) bad = 1;
    }
    __shared__ double sh[kThreads / kWave][6];
    int w = threadIdx.x / kWave;
    for (int d = 0; d < 3; d++) {
        double a = wave_min(lo[d]), b = wave_max(hi[d]);
        if (lane_id() == 0) {
            sh[w][d] = a;
            sh[w][3 + d] = b;
        }
    }
    if (__ballot(bad)) {
        if (lane_id() == 0) atomicAdd(&rb->bad, 1);
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = sh[0][threadIdx.x];
        for (int k = 1; k < kThreads / kWave; k++)
            v = threadIdx.x < 3 ? fmin(v, sh[k][threadIdx.x]) : fmax(v, sh[k][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_bbox_final(const double *part, int nblk, RootBox *rb) {
#pragma clang fp contract(off)
    __shared__ double sh[kThreads / kWave][6];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], part[b * 6 + d]);
            hi[d] = fmax(hi[d], part[b * 6 + 3 + d]);
        }
    int w = threadIdx.x / kWave;
    for (int d = 0; d < 3; d++) {
        double a = wave_min(lo[d]), b = wave_max(hi[d]);
        if (lane_id() == 0) {
            sh[w][d] = a;
            sh[w][3 + d] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double l[3], h[3];
        for (int d = 0; d < 3; d++) {
            l[d] = sh[0][d];
            h[d] = sh[0][3 + d];
            for (int k = 1; k < kThreads / kWave; k++) {
                l[d] = fmin(l[d], sh[k][d]);
                h[d] = fmax(h[d], sh[k][3 + d]);
            }
        }
        double ext = 0.0;
        for (int d = 0; d < 3; d++) {
            double e = h[d] - l[d];
            if (e > ext) ext = e;
        }
        if (!(ext > 0.0)) ext = 1.0;
        for (int d = 0; d < 3; d++) rb->lo[d] = l[d];
        rb->ext = ext;
        rb->scale = 2097152.0 / ext;
    }
}

// ------------------------------------------------------------------ keys
__global__ __launch_bounds__(kThreads) void k_keys(const double *pos, int64_t n, const RootBox *rb,
                                                   uint64_t *key, uint32_t *idx) {
#pragma clang fp contract(off)
    double scale = rb->scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t q[3];
        for (int d = 0; d < 3; d++) {
            double t = (pos[(int64_t)d * n + i] - rb->lo[d]) * scale;
            uint64_t v = (uint64_t)t;
            q[d] = v > 2097151ull ? 2097151ull : v;
        }
        key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        idx[i] = (uint32_t)i;
    }
}

// Batched mode: each system gets its own root cube (one block per system)
// and keys with the system id above kBatchLevels octal digits.
__global__ __launch_bounds__(kThreads) void k_bbox_systems(const double *pos, const double *mass,
                                                           int64_t n, const int64_t *off,
                                                           RootBox *rb) {
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const int64_t beg = off[s], end = off[s + 1];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        for (int d = 0; d < 3; d++) {
            double x = pos[(int64_t)d * n + i];
            if (!isfinite(x)) bad = 1;
            lo[d] = fmin(lo[d], x);
            hi[d] = fmax(hi[d], x);
        }
        double m = mass[i];
        if (!isfinite(m) || m < 0.0) bad = 1;
    }
    __shared__ double sh[kThreads / kWave][6];
    const int w = threadIdx.x / kWave;
    for (int d = 0; d < 3; d++) {
        double a = wave_min(lo[d]), b = wave_max(hi[d]);
        if (lane_id() == 0) {
            sh[w][d] = a;
            sh[w][3 + d] = b;
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicAdd(&rb[0].bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        double l[3], h[3];
        for (int d = 0; d < 3; d++) {
            l[d] = sh[0][d];
            h[d] = sh[0][3 + d];
            for (int k = 1; k < kThreads / kWave; k++) {
                l[d] = fmin(l[d], sh[k][d]);
                h[d] = fmax(h[d], sh[k][3 + d]);
            }
        }
        double ext = 0.0;
        for (int d = 0; d < 3; d++) {
            double e = h[d] - l[d];
            if (e > ext) ext = e;
        }
        if (!(ext > 0.0)) ext = 1.0;
        for (int d = 0; d < 3; d++) rb[s].lo[d] = end > beg ? l[d] : 0.0;
        rb[s].ext = ext;
        rb[s].scale = ldexp(1.0, kBatchLevels) / ext;
    }
}

__global__ __launch_bounds__(kThreads) void k_keys_systems(const double *pos, int64_t n,
                                                           const int64_t *off, int n_sys,
                                                           const RootBox *rb, uint64_t *key,
                                                           uint32_t *idx) {
#pragma clang fp contract(off)
    const uint64_t qmax = (1ull << kBatchLevels) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_sys;  // system s with off[s] <= i < off[s+1]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (off[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        const RootBox &b = rb[lo];
        uint64_t q[3];
        for (int d = 0; d < 3; d++) {
            double t = (pos[(int64_t)d * n + i] - b.lo[d]) * b.scale;
            uint64_t v = (uint64_t)t;
            q[d] = v > qmax ? qmax : v;
        }
        key[i] = ((uint64_t)lo << (3 * kBatchLevels)) |
                 (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        idx[i] = (uint32_t)i;
    }
}

// ------------------------------------------------------------- radix sort
// LSD, 8-bit digits, 8 passes. Per pass: tile histograms, one exclusive scan
// per digit over the tiles (a block per digit, which also gives the digit's
// total), and a stable scatter that scans the 256 digit totals itself, ranks
// equal digits inside a tile with wave ballots and reorders the tile through
// LDS so that the global writes are contiguous runs per digit.
constexpr int kSortRounds = 8;
constexpr int kSortTile = kThreads * kSortRounds;  // 2048 keys
constexpr int kRadix = 256;

__global__ __launch_bounds__(kThreads) void k_sort_hist(const uint64_t *key, int64_t n, int shift,
                                                        uint32_t *hist, int64_t ntiles,
                                                        const int64_t *n_dev) {
    if (n_dev) n = *n_dev;
    __shared__ uint32_t cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; r++) {
        int64_t k = base + r * kThreads + threadIdx.x;
        if (k < n) atomicAdd(&cnt[(key[k] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Block d: exclusive prefix of digit d's tile counts over the tiles, and the
// digit's total.
constexpr int kRowPer = 4;  // counts per thread and chunk
__global__ __launch_bounds__(kThreads) void k_sort_rowscan(const uint32_t *hist, int64_t ntiles,
                                                           uint32_t *offs, uint32_t *dtot) {
    __shared__ uint32_t wsum[kThreads / kWave];
    const int t = threadIdx.x, w = t / kWave;
    const uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t *orow = offs + (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < ntiles; c0 += (int64_t)kThreads * kRowPer) {
        uint32_t v[kRowPer], sum = 0;
#pragma unroll
        for (int q = 0; q < kRowPer; q++) {
            const int64_t i = c0 + (int64_t)t * kRowPer + q;
            v[q] = i < ntiles ? row[i] : 0u;
            sum += v[q];
        }
        const uint32_t incl = wave_incl_scan(sum);
        if (lane_id() == kWave - 1) wsum[w] = incl;
        __syncthreads();
        uint32_t off = carry, tot = 0;
        for (int k = 0; k < kThreads / kWave; k++) {
            if (k < w) off += wsum[k];
            tot += wsum[k];
        }
        off += incl - sum;
#pragma unroll
        for (int q = 0; q < kRowPer; q++) {
            const int64_t i = c0 + (int64_t)t * kRowPer + q;
            if (i < ntiles) orow[i] = off;
            off += v[q];
        }
        carry += tot;
        __syncthreads();
    }
    if (t == 0) dtot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint64_t *key_in,
                                                           const uint32_t *val_in,
                                                           uint64_t *key_out, uint32_t *val_out,
                                                           int64_t n, int shift,
                                                           const uint32_t *hist,
                                                           const uint32_t *offs,
                                                           const uint32_t *dtot, int64_t ntiles,
                                                           const int64_t *n_dev) {
    if (n_dev) n = *n_dev;
    __shared__ uint64_t sk[kSortTile];
    __shared__ uint32_t sv[kSortTile];
    __shared__ uint32_t tile_start[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t wave_cnt[kThreads / kWave][kRadix];  // running, then wave offsets
    __shared__ uint32_t wsum[kThreads / kWave], wsum_d[kThreads / kWave];
    const int t = threadIdx.x;
    const int w = t / kWave;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kSortTile;
    // exclusive scans over the digits of this tile's counts and of the
    // digit totals; a key at tile position p with digit d goes to
    // gbase[d] + p (modulo 2^32; the true position is below n)
    const uint32_t c = hist[(int64_t)t * ntiles + tile], dt = dtot[t];
    const uint32_t incl = wave_incl_scan(c), incl_d = wave_incl_scan(dt);
    if (lane_id() == kWave - 1) {
        wsum[w] = incl;
        wsum_d[w] = incl_d;
    }
    for (int k = 0; k < kThreads / kWave; k++) wave_cnt[k][t] = 0;
    __syncthreads();
    uint32_t off = 0, off_d = 0;
    for (int k = 0; k < w; k++) {
        off += wsum[k];
        off_d += wsum_d[k];
    }
    tile_start[t] = off + incl - c;
    gbase[t] = (off_d + incl_d - dt) + offs[(int64_t)t * ntiles + tile] - (off + incl - c);
    // Each wave ranks its own quarter of the tile, kSortRounds keys per lane
    // in order: a key's rank among the wave's earlier keys of its digit is
    // the wave's running count plus the matching lanes below it (8 ballots).
    constexpr int kSub = kSortTile / (kThreads / kWave);  // keys of a wave
    uint64_t kk[kSortRounds];
    uint32_t vv[kSortRounds], rk[kSortRounds];
    uint32_t *cnt = wave_cnt[w];
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t k = base + (int64_t)w * kSub + r * kWave + lane_id();
        const bool valid = k < n;
        kk[r] = valid ? key_in[k] : 0;
        vv[r] = valid ? val_in[k] : 0;
        const int d = (int)((kk[r] >> shift) & 255);
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const unsigned long long bb = __ballot((d >> b) & 1);
            m &= ((d >> b) & 1) ? bb : ~bb;
        }
        const int wrank = lanes_below(m);
        const uint32_t before = valid ? cnt[d] : 0u;
        wave_sync();  // every lane has read its digit's count
        rk[r] = before + (uint32_t)wrank;
        if (valid && wrank == 0) cnt[d] = before + (uint32_t)__popcll(m);
        wave_sync();
    }
    __syncthreads();
    // wave offsets of digit t: the counts of the earlier waves
    {
        uint32_t acc = 0;
        for (int q = 0; q < kThreads / kWave; q++) {
            const uint32_t v = wave_cnt[q][t];
            wave_cnt[q][t] = acc;
            acc += v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t k = base + (int64_t)w * kSub + r * kWave + lane_id();
        if (k < n) {
            const int d = (int)((kk[r] >> shift) & 255);
            const uint32_t p = tile_start[d] + cnt[d] + rk[r];
            sk[p] = kk[r];
            sv[p] = vv[r];
        }
    }
    __syncthreads();
    int64_t tile_n = n - base < kSortTile ? n - base : kSortTile;
    for (int p = t; p < tile_n; p += kThreads) {
        const uint64_t k2 = sk[p];
        const int d = (int)((k2 >> shift) & 255);
        const uint32_t g = gbase[d] + (uint32_t)p;
        key_out[g] = k2;
        val_out[g] = sv[p];
    }
}

// ------------------------------------------------------------ gathers
// orig[k] = input index of the k-th particle in Morton order; rank is its
// inverse. The particle data are then moved with coalesced reads in input
// order and scattered writes (which the caches merge), rather than with
// scattered reads of four separate arrays.
__global__ __launch_bounds__(kThreads) void k_rank(const uint32_t *idx, int64_t n, uint32_t *orig,
                                                   uint32_t *rank) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = idx[k];
        orig[k] = o;
        rank[o] = (uint32_t)k;
    }
}

__global__ __launch_bounds__(kThreads) void k_scatter_particles(const double *pos,
                                                                const double *mass,
                                                                const uint32_t *rank, int64_t n,
                                                                double4 *ps) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        ps[rank[i]] = make_double4(pos[i], pos[n + i], pos[2 * n + i], mass[i]);
}

// ------------------------------------------------------------ octree
// Run searches over the sorted keys. The keys sharing key[k]'s level-`level`
// prefix form one contiguous run. A search brackets the run's boundary by
// galloping (steps growing 16-fold) and then narrows the bracket 8-fold per
// round with 7 independent probes, so a run of length d costs about
// 2 log16(d) + 1 rounds of dependent loads rather than 2 log2(d).
constexpr int kProbes = 7;

// First index after k whose level-`level` prefix differs from key[k]'s.
__device__ int64_t run_end(const uint64_t *key, int64_t n, int64_t k, int level, int levels) {
    const uint64_t p = key_prefix(key[k], level, levels);
    int64_t lo = k, hi = k + 1, step = 1;  // key[lo] in the run; hi == n or key[hi] out of it
    while (hi < n && key_prefix(key[hi], level, levels) == p) {
        lo = hi;
        step <<= 4;
        hi = k + step;
    }
    if (hi > n) hi = n;
    while (hi - lo > 1) {
        const int64_t m = hi - lo;
        int64_t q[kProbes];
        bool in[kProbes];
#pragma unroll
        for (int j = 0; j < kProbes; j++) {
            q[j] = lo + m * (j + 1) / (kProbes + 1);
            in[j] = key_prefix(key[q[j]], level, levels) == p;
        }
        int64_t nlo = lo, nhi = hi;
#pragma unroll
        for (int j = 0; j < kProbes; j++) {
            if (in[j])
                nlo = q[j] > nlo ? q[j] : nlo;
            else
                nhi = q[j] < nhi ? q[j] : nhi;
        }
        lo = nlo;
        hi = nhi;
    }
    return hi;
}

// First index whose level-`level` prefix equals key[k]'s.
__device__ int64_t run_start(const uint64_t *key, int64_t k, int level, int levels) {
    const uint64_t p = key_prefix(key[k], level, levels);
    int64_t lo = k, hi = k - 1, step = 1;  // key[lo] in the run; hi == -1 or key[hi] out of it
    while (hi >= 0 && key_prefix(key[hi], level, levels) == p) {
        lo = hi;
        step <<= 4;
        hi = k - step;
    }
    if (hi < -1) hi = -1;
    while (lo - hi > 1) {
        const int64_t m = lo - hi;
        int64_t q[kProbes];
        bool in[kProbes];
#pragma unroll
        for (int j = 0; j < kProbes; j++) {
            q[j] = lo - m * (j + 1) / (kProbes + 1);
            in[j] = key_prefix(key[q[j]], level, levels) == p;
        }
        int64_t nlo = lo, nhi = hi;
#pragma unroll
        for (int j = 0; j < kProbes; j++) {
            if (in[j])
                nlo = q[j] < nlo ? q[j] : nlo;
            else
                nhi = q[j] > nhi ? q[j] : nhi;
        }
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Shallowest level at which particle k starts a cell (0 where a system starts).
__device__ __forceinline__ int first_level(const uint64_t *key, int64_t k, int levels) {
    return k == 0 ? 0 : common_digits(key[k - 1], key[k], levels) + 1;
}

// Cells are identified by (level, first particle). Particle k starts the
// cells of levels first_level(k)..21 that contain it; such a cell exists iff
// its parent holds more than leaf_size particles. Each particle emits the
// chain of existing cells it starts, from the shallowest; ordering the
// emitted cells by (first particle, level) is a depth-first pre-order.
//
// Both tests only compare a cell size with leaf_size, so they need no search
// over the sorted keys:
//  * the level-L cell holding k-1 and k has more than leaf_size particles iff
//    some window [j, j + leaf_size] with k - leaf_size <= j < k lies in one
//    level-L cell;
//  * the level-l cell starting at k holds at most leaf_size particles iff
//    key[k + leaf_size] (if any) is outside it, i.e. the chain ends at
//    level max(first_level, common_digits(k, k + leaf_size) + 1), capped
//    at the deepest level.
__device__ __forceinline__ bool parent_big(const uint64_t *key, int64_t n, int64_t k, int L,
                                           int leaf_size, int levels) {
    const int64_t j0 = k - leaf_size > 0 ? k - leaf_size : 0;
    for (int64_t j = j0; j < k; j++) {
        if (j + leaf_size >= n) break;
        if (common_digits(key[j], key[j + leaf_size], levels) >= L) return true;
    }
    return false;
}

__device__ __forceinline__ int chain_last(const uint64_t *key, int64_t n, int64_t k, int l0,
                                          int leaf_size, int levels) {
    const int cd = k + leaf_size < n ? common_digits(key[k], key[k + leaf_size], levels) : -1;
    int last = cd + 1 > l0 ? cd + 1 : l0;
    return last < levels ? last : levels;
}

// Also the deepest cell level: each block's maximum goes into one of
// kDeepSlots words kDeepStride apart (atomicMax; spreading the blocks over
// words in different cache lines keeps them from queueing on one line); the
// host takes the maximum of the words with the cell count and launches the
// per-level passes only down to that level.
__global__ __launch_bounds__(kThreads) void k_octree_count(const uint64_t *key, int64_t n,
                                                           int leaf_size, int levels,
                                                           uint32_t *emit, uint32_t *deep_slots) {
    __shared__ int wmax[kThreads / kWave];
    int deepest = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int l0 = first_level(key, k, levels);
        uint32_t cnt = 0;
        if (l0 <= levels && (l0 == 0 || parent_big(key, n, k, l0 - 1, leaf_size, levels))) {
            const int last = chain_last(key, n, k, l0, leaf_size, levels);
            cnt = (uint32_t)(last - l0 + 1);
            deepest = last > deepest ? last : deepest;
        }
        emit[k] = cnt;
    }
    deepest = (int)wave_max((double)deepest);
    if (lane_id() == 0) wmax[threadIdx.x / kWave] = deepest;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int w = 0; w < kThreads / kWave; w++) m = wmax[w] > m ? wmax[w] : m;
        if (m > 0) atomicMax(&deep_slots[(blockIdx.x % kDeepSlots) * kDeepStride], (uint32_t)m);
    }
}

// Two passes over the emitted cells: a thread per particle writes the
// (particle, level) of each cell its chain starts, then a thread per cell
// finds the cell's particle count and parent (galloping searches over the
// keys), so that no thread walks a whole root-to-leaf chain of searches.
__global__ __launch_bounds__(kThreads) void k_octree_emit(const uint64_t *key, int64_t n,
                                                          int levels, const int64_t *base,
                                                          PreOrder pre, const Status *st) {
    if (st->cell_overflow) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = base[k];
        const int64_t nemit = base[k + 1] - b;
        if (nemit == 0) continue;
        const int l0 = first_level(key, k, levels);
        for (int u = 0; u < nemit; u++)
            pre.info[b + u] = make_uint4((uint32_t)k, 0u, (uint32_t)(l0 + u) << 1, 0u);
    }
}

__global__ __launch_bounds__(kThreads) void k_octree_write(const uint64_t *key, int64_t n,
                                                           int leaf_size, int levels,
                                                           const int64_t *base, PreOrder pre,
                                                           uint64_t *lkey, uint32_t *lval,
                                                           const Status *st) {
    const int64_t n_cells = st->n_nodes;  // 0 after an overflow
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint4 e = pre.info[c];
        const int64_t k = e.x;
        const int l = (int)(e.z >> 1);
        const int64_t b = base[k];
        const int64_t nemit = base[k + 1] - b;
        const int64_t u = c - b;
        const uint32_t idx = (uint32_t)c;
        // the last cell of the chain holds <= leaf_size particles unless it
        // sits at the deepest level; the others hold more
        const bool small = u == nemit - 1 && (k + leaf_size >= n ||
                           common_digits(key[k], key[k + leaf_size], levels) < l);
        uint32_t cnt = 1;
        if (small) {
            while (cnt < (uint32_t)leaf_size && k + cnt < n &&
                   common_digits(key[k], key[k + cnt], levels) >= l)
                cnt++;
        } else {
            cnt = (uint32_t)(run_end(key, n, k, l, levels) - k);
        }
        const bool leaf = (cnt <= (uint32_t)leaf_size) || l == levels;
        pre.info[idx] = make_uint4((uint32_t)k, cnt, (leaf ? kLeafFlag : 0u) | ((uint32_t)l << 1),
                                   0u);
        uint32_t parent;
        if (u > 0) {
            parent = idx - 1;
        } else if (l == 0) {
            parent = kNone;  // root of a system
        } else {
            const int L = l - 1;
            const int64_t s = run_start(key, k, L, levels);
            parent = (uint32_t)(base[s] + (L - first_level(key, s, levels)));
        }
        pre.parent[idx] = parent;
        if (parent != kNone) atomicAdd(&pre.nchild[parent], 1u);
        lkey[idx] = (uint64_t)l;
        lval[idx] = idx;
    }
}

// Device cell count for the build's second half: the scanned count, or 0
// (with Status::cell_overflow raised) when it exceeds the arrays' capacity,
// so that every later kernel does nothing.
// What the host needs after the first half of an eager build, gathered into
// the status words so that one copy reads it: the cell count, the input
// check of the root box and the deepest cell level.
__global__ void k_build_head(const int64_t *base, int64_t n, const RootBox *rb,
                             const uint32_t *deep_slots, Status *st) {
    if (blockIdx.x != 0) return;
    uint32_t d = 0;
    for (int w = threadIdx.x; w < kDeepSlots; w += blockDim.x) {
        const uint32_t v = deep_slots[w * kDeepStride];
        d = v > d ? v : d;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t u = (uint32_t)__shfl_down((int)d, o, kWave);
        d = u > d ? u : d;
    }
    if (threadIdx.x == 0) {
        st->cells = base[n];
        st->bad_input = rb->bad;
        st->deep = d;
    }
}

__global__ void k_cell_count(const int64_t *base, int64_t n, int64_t node_cap, Status *st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t c = base[n];
        if (c > node_cap) {
            st->cell_overflow = 1;
            c = 0;
        }
        st->n_nodes = c;
    }
}

// perm[new] = old after the stable sort by level; its inverse.
__global__ __launch_bounds__(kThreads) void k_invert(const uint32_t *perm, const int64_t *n_dev,
                                                     uint32_t *new_of_old) {
    const int64_t n_nodes = *n_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes;
         i += (int64_t)gridDim.x * blockDim.x)
        new_of_old[perm[i]] = (uint32_t)i;
}

// Level-order cell records. Sorting the pre-order cells stably by level keeps
// each level in Morton order, so siblings are contiguous and the first child
// of a cell is the cell that follows it in pre-order.
__global__ __launch_bounds__(kThreads) void k_relayout(const uint32_t *perm, PreOrder pre,
                                                       const RootBox *rb, const uint64_t *key,
                                                       int levels, TreeDev t) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t old = perm[i];
        uint4 in = pre.info[old];
        uint32_t nc = pre.nchild[old];
        uint32_t first = nc ? pre.new_of_old[old + 1] : 0u;
        t.nd_info[i] = make_uint4(in.x, in.y, in.z | (nc << 8), first);
        const uint32_t par = pre.parent[old];
        t.nd_parent[i] = par == kNone ? kNone : pre.new_of_old[par];
        const uint64_t sys = key[in.x] >> (3 * levels);
        t.nd_hi[i].w = ldexp(rb[sys].ext, -info_level(in.z));
    }
}

// level_off[l] = first cell of level >= l (cells are sorted by level).
__global__ void k_level_offsets(TreeDev t, uint32_t *level_off) {
    int l = threadIdx.x;
    if (l > kMaxLevel + 1) return;  // levels above the deepest one get n_nodes
    int64_t lo = 0, hi = *t.n_nodes_dev;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (info_level(t.nd_info[mid].z) < l)
            lo = mid + 1;
        else
            hi = mid;
    }
    level_off[l] = (uint32_t)lo;
}

// Cell data of cell c. Leaves sum their particles (two passes: centre of
// mass, then the second moment about it); other cells combine their children
// with the parallel-axis shift. Items (particles or children) are summed in
// their order. Up to 8 items are loaded before any is used, so that their
// loads overlap instead of costing one memory latency each (the slots past
// the last item repeat it and are not summed; box minima and maxima do not
// depend on order or repeats); longer leaves (at the deepest level) loop.
template <bool leaf>
__device__ void cell_moments(const TreeDev &t, uint32_t c, const uint4 info) {
    const uint32_t first = leaf ? info.x : info.w;
    const uint32_t cnt = leaf ? info.y : (uint32_t)info_nchild(info.z);
    double M = 0, sx = 0, sy = 0, sz = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double S[6] = {0, 0, 0, 0, 0, 0};
    double cx = 0, cy = 0, cz = 0;
    auto centre = [&]() {
        if (M > 0.0) {
            cx = sx / M;
            cy = sy / M;
            cz = sz / M;
        } else {
            cx = 0.5 * (lo[0] + hi[0]);
            cy = 0.5 * (lo[1] + hi[1]);
            cz = 0.5 * (lo[2] + hi[2]);
        }
    };
    // (x, y, z, mass) of an item: a particle, or a child's centre and mass
    auto mass_point = [&](const double4 &p) {
        M += p.w;
        sx += p.w * p.x;
        sy += p.w * p.y;
        sz += p.w * p.z;
    };
    auto grow_box = [&](double x0, double y0, double z0, double x1, double y1, double z1) {
        lo[0] = fmin(lo[0], x0);
        lo[1] = fmin(lo[1], y0);
        lo[2] = fmin(lo[2], z0);
        hi[0] = fmax(hi[0], x1);
        hi[1] = fmax(hi[1], y1);
        hi[2] = fmax(hi[2], z1);
    };
    auto second_particle = [&](const double4 &p) {
        double qx = p.x - cx, qy = p.y - cy, qz = p.z - cz;
        S[0] += p.w * qx * qx;
        S[1] += p.w * qy * qy;
        S[2] += p.w * qz * qz;
        S[3] += p.w * qx * qy;
        S[4] += p.w * qx * qz;
        S[5] += p.w * qy * qz;
    };
    auto second_child = [&](const double4 &cm, const double *Sc) {
        double dx = cm.x - cx, dy = cm.y - cy, dz = cm.z - cz;
        S[0] += Sc[0] + cm.w * dx * dx;
        S[1] += Sc[1] + cm.w * dy * dy;
        S[2] += Sc[2] + cm.w * dz * dz;
        S[3] += Sc[3] + cm.w * dx * dy;
        S[4] += Sc[4] + cm.w * dx * dz;
        S[5] += Sc[5] + cm.w * dy * dz;
    };
    if (cnt >= 1 && cnt <= 8) {
        double4 p[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t o = first + (k < cnt ? k : cnt - 1);
            p[k] = leaf ? t.ps[o] : t.nd_com[o];
        }
        if constexpr (leaf) {
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) grow_box(p[k].x, p[k].y, p[k].z, p[k].x, p[k].y, p[k].z);
        } else {
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) {
                const uint32_t o = first + (k < cnt ? k : cnt - 1);
                const double4 l4 = t.nd_lo[o], h4 = t.nd_hi[o];
                grow_box(l4.x, l4.y, l4.z, h4.x, h4.y, h4.z);
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++)
            if (k < cnt) mass_point(p[k]);
        centre();
        if constexpr (leaf) {
#pragma unroll
            for (uint32_t k = 0; k < 8; k++)
                if (k < cnt) second_particle(p[k]);
        } else {
            double Sk[8][6];
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) {
                const uint32_t o = first + (k < cnt ? k : cnt - 1);
#pragma unroll
                for (int j = 0; j < 6; j++) Sk[k][j] = t.nd_S[(int64_t)o * 6 + j];
            }
#pragma unroll
            for (uint32_t k = 0; k < 8; k++)
                if (k < cnt) second_child(p[k], Sk[k]);
        }
    } else if constexpr (leaf) {
        for (uint32_t k = first; k < first + cnt; k++) {
            const double4 p = t.ps[k];
            mass_point(p);
            grow_box(p.x, p.y, p.z, p.x, p.y, p.z);
        }
        centre();
        for (uint32_t k = first; k < first + cnt; k++) second_particle(t.ps[k]);
    }
    t.nd_com[c] = make_double4(cx, cy, cz, M);
    double4 l4 = t.nd_lo[c];
    l4.x = lo[0];
    l4.y = lo[1];
    l4.z = lo[2];
    t.nd_lo[c] = l4;
    double side = t.nd_hi[c].w;
    t.nd_hi[c] = make_double4(hi[0], hi[1], hi[2], side);
    for (int k = 0; k < 6; k++) t.nd_S[(int64_t)c * 6 + k] = S[k];
    float4 q0, q1;
    quad_f32(S, M, &q0, &q1);
    t.nd_q[2 * (int64_t)c] = q0;
    t.nd_q[2 * (int64_t)c + 1] = q1;
}

// Bottom-up cell data: every leaf in one launch (leaves of all levels are
// independent), then one launch per level, deepest first, for the other
// cells (each combines its children, which are complete by then).
__global__ __launch_bounds__(kThreads) void k_moments_leaves(TreeDev t) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_nodes;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint4 info = t.nd_info[c];
        if (info.z & kLeafFlag) cell_moments<true>(t, (uint32_t)c, info);
    }
}

__global__ __launch_bounds__(kThreads) void k_moments_level(TreeDev t, int level) {
    const uint32_t beg = t.level_off[level], end = t.level_off[level + 1];
    for (int64_t c = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < end;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint4 info = t.nd_info[c];
        if (!(info.z & kLeafFlag)) cell_moments<false>(t, (uint32_t)c, info);
    }
}

__global__ __launch_bounds__(kThreads) void k_tree_summary(TreeDev t, Status *st) {
    __shared__ uint32_t sh[kThreads / kWave];
    const int64_t n_nodes = *t.n_nodes_dev;
    uint32_t leaves = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_nodes;
         c += (int64_t)gridDim.x * blockDim.x)
        leaves += t.nd_info[c].z & kLeafFlag;
    leaves = wave_sum(leaves);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = leaves;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int w = 0; w < kThreads / kWave; w++) b += sh[w];
        if (b) atomicAdd((unsigned long long *)&st->n_leaves, (unsigned long long)b);
        if (blockIdx.x == 0 && n_nodes > 0) st->max_level = info_level(t.nd_info[n_nodes - 1].z);
    }
}

// ------------------------------------------------------- force preparation
// Radii into Morton order (coalesced reads, scattered writes), with the
// validity check 0 <= r_in < r_out <= r_search (all finite).
__global__ __launch_bounds__(kThreads) void k_gather_radii(const double *r_in, const double *r_out,
                                                           const double *r_search, TreeDev t,
                                                           Status *st) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < t.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = t.rank[i];
        double a = r_in[i], b = r_out[i], c = r_search[i];
        if (!(isfinite(a) && isfinite(b) && isfinite(c) && a >= 0.0 && a < b && b <= c)) bad = 1;
        t.rr[k] = make_double2(a, b);
        t.rsk[k] = c;
    }
    if (__ballot(bad) && lane_id() == 0) atomicAdd(&st->invalid_radii, 1);
}

// Largest search radius per cell. Leaves take the maximum over their
// particles and other cells start at 0; then every leaf raises its ancestors
// with a 64-bit atomicMax on the bits of the value (the order of
// non-negative doubles is that of their bits), climbing only while it raised
// the cell above, since otherwise the value there came from another leaf
// that climbs on. The result does not depend on the order of the atomics.
__global__ __launch_bounds__(kThreads) void k_rsmax_leaves(TreeDev t) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_nodes;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint4 info = t.nd_info[c];
        double r = 0.0;
        if (info.z & kLeafFlag)
            for (uint32_t k = info.x; k < info.x + info.y; k++) r = fmax(r, t.rsk[k]);
        t.nd_lo[c].w = r;
    }
}

__global__ __launch_bounds__(kThreads) void k_rsmax_up(TreeDev t) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_nodes;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (!(t.nd_info[c].z & kLeafFlag)) continue;
        const unsigned long long v = (unsigned long long)__double_as_longlong(t.nd_lo[c].w);
        for (uint32_t p = t.nd_parent[c]; p != kNone; p = t.nd_parent[p]) {
            const unsigned long long old =
                atomicMax((unsigned long long *)&t.nd_lo[p].w, v);
            if (old >= v) break;
        }
    }
}

// i-groups: the first cells on each root-to-leaf path holding <= group_size
// particles, or leaves.
__global__ __launch_bounds__(kThreads) void k_group_flags(PreOrder pre, TreeDev t,
                                                          int group_size, uint32_t *flag) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < t.n_nodes;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (c >= n_nodes) {
            flag[c] = 0u;
            continue;
        }
        uint4 info = pre.info[c];
        bool small = info.y <= (uint32_t)group_size || (info.z & kLeafFlag);
        uint32_t p = pre.parent[c];
        bool parent_big = p == kNone || pre.info[p].y > (uint32_t)group_size;
        flag[c] = (small && parent_big) ? 1u : 0u;
    }
}

// Groups listed in pre-order (= Morton order of their particles), as
// level-order cell indices.
__global__ __launch_bounds__(kThreads) void k_group_compact(PreOrder pre, TreeDev t,
                                                            const uint32_t *flag,
                                                            const uint32_t *pos, uint32_t *groups,
                                                            Status *st) {
    const int64_t n_nodes = *t.n_nodes_dev;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_nodes;
         c += (int64_t)gridDim.x * blockDim.x)
        if (flag[c]) groups[pos[c]] = pre.new_of_old[c];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->n_groups = pos[n_nodes];
}

// ------------------------------------------------------- changeover radii
__global__ __launch_bounds__(kThreads) void k_mass_partial(const double *mass, int64_t n,
                                                           double *part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += mass[i];
    __shared__ double sh[kThreads / kWave];
    s = wave_sum(s);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int k = 0; k < kThreads / kWave; k++) v += sh[k];
        part[blockIdx.x] = v;
    }
}

// Mean mass <m> = (sum m)/N, summed in a fixed order (deterministic).
// Mean mass from the block partials: one wave, strided partial sums, then a
// butterfly (a fixed order, so the result is reproducible).
__global__ void k_mass_final(double *part, int nblk, int64_t n) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kWave) v += part[b];
    v = wave_sum(v);
    if (threadIdx.x == 0) part[nblk] = v / (double)n;
}

__global__ __launch_bounds__(kThreads) void k_radii(const double *mass, const double *vel,
                                                    int64_t n, const double *mave_p,
                                                    double rin_ref, double rout_ref,
                                                    double search_factor, double cr_dt,
                                                    double *r_in, double *r_out, double *r_s) {
    const double mave = *mave_p;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ratio = mave > 0.0 ? mass[i] / mave : 1.0;
        double s = cbrt(ratio > 1.0 ? ratio : 1.0);
        double ro = s * rout_ref;
        r_in[i] = s * rin_ref;
        r_out[i] = ro;
        if (vel) {
            double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
            r_s[i] = ro + cr_dt * sqrt(vx * vx + vy * vy + vz * vz);
        } else {
            r_s[i] = search_factor * ro;
        }
    }
}

}  // namespace

// ------------------------------------------------------------ launchers
int bbox_partial_blocks(int64_t n) { return (int)grid_for(n, kThreads, kBBoxBlocks); }

void launch_bbox(const double *pos, const double *mass, int64_t n, double *part, RootBox *rb,
                 hipStream_t s) {
    int nb = bbox_partial_blocks(n);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kThreads), 0, s, pos, mass, n, part, rb);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kThreads), 0, s, (const double *)part, nb, rb);
}

void launch_bbox_systems(const double *pos, const double *mass, int64_t n, const int64_t *off,
                         int n_sys, RootBox *rb, hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_systems, dim3(n_sys), dim3(kThreads), 0, s, pos, mass, n, off, rb);
}

void launch_keys_systems(const double *pos, int64_t n, const int64_t *off, int n_sys,
                         const RootBox *rb, uint64_t *key, uint32_t *idx, hipStream_t s) {
    hipLaunchKernelGGL(k_keys_systems, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, pos,
                       n, off, n_sys, rb, key, idx);
}

void launch_keys(const double *pos, int64_t n, const RootBox *rb, uint64_t *key, uint32_t *idx,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, pos, n, rb,
                       key, idx);
}

int64_t sort_ws_bytes(int64_t n) {
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    if (ntiles < 1) ntiles = 1;
    return (int64_t)sizeof(uint32_t) * (2 * kRadix * ntiles + kRadix + 4);
}

void radix_sort(uint64_t **key, uint32_t **val, uint64_t **key_alt, uint32_t **val_alt, int64_t n,
                int passes, void *ws, hipStream_t s, const int64_t *n_dev) {
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    if (ntiles < 1) ntiles = 1;
    uint32_t *hist = (uint32_t *)ws;
    uint32_t *offs = hist + kRadix * ntiles;
    uint32_t *dtot = offs + kRadix * ntiles;
    for (int pass = 0; pass < passes; pass++) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)ntiles), dim3(kThreads), 0, s,
                           (const uint64_t *)*key, n, shift, hist, ntiles, n_dev);
        hipLaunchKernelGGL(k_sort_rowscan, dim3(kRadix), dim3(kThreads), 0, s,
                           (const uint32_t *)hist, ntiles, offs, dtot);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)ntiles), dim3(kThreads), 0, s,
                           (const uint64_t *)*key, (const uint32_t *)*val, *key_alt, *val_alt, n,
                           shift, (const uint32_t *)hist, (const uint32_t *)offs,
                           (const uint32_t *)dtot, ntiles, n_dev);
        uint64_t *tk = *key;
        *key = *key_alt;
        *key_alt = tk;
        uint32_t *tv = *val;
        *val = *val_alt;
        *val_alt = tv;
    }
}

void launch_gather_particles(const double *pos, const double *mass, const uint32_t *idx,
                             int64_t n, double4 *ps, uint32_t *orig, uint32_t *rank,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, idx, n,
                       orig, rank);
    hipLaunchKernelGGL(k_scatter_particles, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0,
                       s, pos, mass, (const uint32_t *)rank, n, ps);
}

void launch_octree_count(const uint64_t *key, int64_t n, int leaf_size, int levels,
                         uint32_t *emit, uint32_t *deep_slots, hipStream_t s) {
    hipLaunchKernelGGL(k_octree_count, dim3(grid_for(n)), dim3(kThreads), 0, s, key, n, leaf_size,
                       levels, emit, deep_slots);
}

void launch_build_head(const int64_t *base, int64_t n, const RootBox *rb,
                       const uint32_t *deep_slots, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_build_head, dim3(1), dim3(kWave), 0, s, base, n, rb, deep_slots, st);
}

void launch_octree_write(const uint64_t *key, int64_t n, int leaf_size, int levels,
                         const int64_t *base, PreOrder pre, uint64_t *lkey, uint32_t *lval,
                         int64_t node_cap, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_count, dim3(1), dim3(64), 0, s, base, n, node_cap, st);
    hipLaunchKernelGGL(k_octree_emit, dim3(grid_for(n)), dim3(kThreads), 0, s, key, n, levels,
                       base, pre, (const Status *)st);
    hipLaunchKernelGGL(k_octree_write, dim3(grid_for(node_cap)), dim3(kThreads), 0, s, key, n,
                       leaf_size, levels, base, pre, lkey, lval, (const Status *)st);
}

void launch_relayout(const uint32_t *perm, PreOrder pre, const RootBox *rb, const uint64_t *key,
                     int levels, TreeDev t, uint32_t *level_off, hipStream_t s) {
    hipLaunchKernelGGL(k_invert, dim3(grid_for(t.n_nodes)), dim3(kThreads), 0, s, perm,
                       t.n_nodes_dev, pre.new_of_old);
    hipLaunchKernelGGL(k_relayout, dim3(grid_for(t.n_nodes)), dim3(kThreads), 0, s, perm, pre, rb,
                       key, levels, t);
    hipLaunchKernelGGL(k_level_offsets, dim3(1), dim3(32), 0, s, t, level_off);
}

void launch_moments(const TreeDev &t, int levels, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_leaves, dim3(grid_for(t.n_nodes, kThreads, 8192)), dim3(kThreads),
                       0, s, t);
    for (int l = levels - 1; l >= 0; l--)
        hipLaunchKernelGGL(k_moments_level, dim3(grid_for(t.n_nodes, kThreads, 1024)),
                           dim3(kThreads), 0, s, t, l);
}

void launch_tree_summary(const TreeDev &t, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_summary, dim3(grid_for(t.n_nodes, kThreads, 256)), dim3(kThreads), 0,
                       s, t, st);
}

void launch_gather_radii(const double *r_in, const double *r_out, const double *r_search,
                         TreeDev t, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_radii, dim3(grid_for(t.n, kThreads, 8192)), dim3(kThreads), 0, s,
                       r_in, r_out, r_search, t, st);
}

void launch_rsmax(const TreeDev &t, hipStream_t s) {
    hipLaunchKernelGGL(k_rsmax_leaves, dim3(grid_for(t.n_nodes, kThreads, 8192)), dim3(kThreads), 0,
                       s, t);
    hipLaunchKernelGGL(k_rsmax_up, dim3(grid_for(t.n_nodes, kThreads, 8192)), dim3(kThreads), 0, s,
                       t);
}

void launch_group_flags(const PreOrder &pre, const TreeDev &t, int group_size, uint32_t *flag,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(t.n_nodes)), dim3(kThreads), 0, s, pre, t,
                       group_size, flag);
}

void launch_group_compact(const PreOrder &pre, const TreeDev &t, const uint32_t *flag,
                          const uint32_t *pos, uint32_t *groups, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_group_compact, dim3(grid_for(t.n_nodes)), dim3(kThreads), 0, s, pre, t,
                       flag, pos, groups, st);
}

void launch_changeover_radii(const double *mass, const double *vel, int64_t n, double rin_ref,
                             double rout_ref, double search_factor, double cr_dt, double *r_in,
                             double *r_out, double *r_search, double *ws, hipStream_t s) {
    int nb = (int)grid_for(n, kThreads, 1024);
    hipLaunchKernelGGL(k_mass_partial, dim3(nb), dim3(kThreads), 0, s, mass, n, ws);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(64), 0, s, ws, nb, n);
    hipLaunchKernelGGL(k_radii, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, mass, vel,
                       n, (const double *)(ws + nb), rin_ref, rout_ref, search_factor, cr_dt, r_in,
                       r_out, r_search);
}

}  // namespace petar
