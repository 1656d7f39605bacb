// Neighbour candidates (first stage of the neighbour search: all j != i
// with |r_j - r_i| < max(r_search,i, r_search,j)), as CSR lists in input
// order, each sorted by original index.
//
// Per i-group a wavefront walks only the near region: a cell is opened iff
// its box is closer to the group's box than max(rs_group, rs_cell); the
// leaves reached are tested pair by pair with the FP64 relation of common.h.
// The box test is conservative for the pair test (same rounding, monotone),
// so every candidate is found. Two passes (count, write) around one prefix
// sum, then a per-list sort.
#include "launch.h"
#include "walk.h"

namespace petar {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

struct NbLds {
    uint32_t stack[kStackLds];
    uint32_t leaf_start[kWave], leaf_cnt[kWave], leaf_pre[kWave];
    double4 jp[kWave];
    double jr[kWave];
    uint32_t jk[kWave];
};

__device__ __forceinline__ int find_leaf(const uint32_t *pre, int nleaf, uint32_t s) {
    int lo = 0, hi = nleaf;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= s)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// kWrite == false: count per target; true: write orig indices at wpos.
template <bool kWrite>
__device__ void nb_flush(NbLds &L, int nleaf, const TreeDev &t, const double4 &pi, double rsi,
                         uint32_t ki, bool valid, uint32_t &count, int32_t *out, int64_t wpos) {
    wave_sync();
    const int lane = lane_id();
    uint32_t c = lane < nleaf ? L.leaf_cnt[lane] : 0u;
    uint32_t incl = wave_incl_scan(c);
    uint32_t total = (uint32_t)uniform((int)__shfl(incl, kWave - 1, kWave));
    if (lane < nleaf) L.leaf_pre[lane] = incl - c;
    wave_sync();
    for (uint32_t base = 0; base < total; base += kWave) {
        uint32_t s = base + lane;
        if (s < total) {
            int l = find_leaf(L.leaf_pre, nleaf, s);
            uint32_t k = L.leaf_start[l] + (s - L.leaf_pre[l]);
            L.jp[lane] = t.ps[k];
            L.jr[lane] = t.rsk[k];
            L.jk[lane] = k;
        }
        wave_sync();
        int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
        for (int j = 0; j < m; j++) {
            double4 pj = L.jp[j];
            uint32_t kj = L.jk[j];
            bool hit = valid && kj != ki && nb_pair(pi.x, pi.y, pi.z, rsi, pj.x, pj.y, pj.z, L.jr[j]);
            if (hit) {
                if (kWrite) out[wpos + count] = (int32_t)t.orig[kj];
                count++;
            }
        }
        wave_sync();
    }
}

template <bool kWrite>
__global__ __launch_bounds__(kThreads) void k_nb(TreeDev t, const uint32_t *groups, Status *st,
                                                 uint32_t *cnt_orig, const int64_t *offsets,
                                                 int32_t *idx, int64_t capacity, uint32_t *spill,
                                                 uint32_t *queue, const uint32_t *rec_count,
                                                 uint32_t rec_cap) {
    __shared__ NbLds lds_all[kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    NbLds &L = lds_all[w];
    const int lane = lane_id();
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow) return;
    if (rec_count && *rec_count <= rec_cap) return;  // the record passes run instead
    if (kWrite && offsets[t.n] > capacity) return;
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + w;
    const int64_t n_groups = st->n_groups;
    WaveStack stk;
    stk.lds = L.stack;
    stk.spill = spill + gwave * kSpillCap;
    while (true) {
        uint32_t v = 0;
        if (lane == 0) v = atomicAdd(queue, 1u);
        int64_t g = (int64_t)(uint32_t)uniform((int)v);
        if (g >= n_groups) break;
        const uint32_t gnode = groups[g];
        const uint4 ginfo = t.nd_info[gnode];
        const GroupGeom G = load_group(t.nd_lo, t.nd_hi, gnode);
        for (uint32_t chunk = 0; chunk < ginfo.y; chunk += kWave) {
            uint32_t off = chunk + lane;
            bool valid = off < ginfo.y;
            uint32_t ki = ginfo.x + (valid ? off : 0u);
            double4 pi = t.ps[ki];
            double rsi = t.rsk[ki];
            uint32_t count = 0;
            int64_t wpos = 0;
            if (kWrite && valid) wpos = offsets[t.orig[ki]];
            int nleaf = 0;
            stk.init((uint32_t)uniform((int)root_of(t.nd_info, t.level_off, ginfo.x)));
            bool ok = true;
            while (!stk.empty()) {
                uint32_t node = stk.pop();
                bool leaf_hit = false, open = false;
                uint4 info = make_uint4(0, 0, 0, 0);
                if (node != kNone) {
                    double4 lo = t.nd_lo[node], hi = t.nd_hi[node];
                    info = t.nd_info[node];
                    double D2, R2;
                    box_terms(G, lo, hi, &D2, &R2);
                    if (D2 < R2) {
                        if (info.z & kLeafFlag)
                            leaf_hit = true;
                        else
                            open = true;
                    }
                }
                int nc = open ? info_nchild(info.z) : 0;
                if (!stk.push(info.w, nc)) {
                    ok = false;
                    break;
                }
                unsigned long long m = __ballot(leaf_hit);
                int cnt = __popcll(m);
                if (cnt) {
                    if (nleaf + cnt > kWave) {
                        nb_flush<kWrite>(L, nleaf, t, pi, rsi, ki, valid, count, idx, wpos);
                        nleaf = 0;
                    }
                    if (leaf_hit) {
                        int p = nleaf + lanes_below(m);
                        L.leaf_start[p] = info.x;
                        L.leaf_cnt[p] = info.y;
                    }
                    nleaf += cnt;
                }
            }
            if (!ok) {
                if (lane == 0) atomicAdd(&st->stack_overflow, 1);
                break;
            }
            if (nleaf) nb_flush<kWrite>(L, nleaf, t, pi, rsi, ki, valid, count, idx, wpos);
            if (!kWrite && valid) cnt_orig[t.orig[ki]] = count;
        }
    }
}

// Neighbour passes over the near-leaf records written by the force walk:
// one wave per record (group particles x leaf particles), FP64 pair test.
// Counting adds 1 per hit; writing takes a slot per hit from a per-target
// cursor (the lists are sorted afterwards, so the slot order is irrelevant).
template <bool kWrite>
__global__ __launch_bounds__(kThreads) void k_nb_rec(TreeDev t, const uint4 *rec,
                                                     const uint32_t *rec_count, const Status *st,
                                                     uint32_t *cnt_orig, const int64_t *offsets,
                                                     uint32_t *cursor, int32_t *idx,
                                                     int64_t capacity, uint32_t rec_cap) {
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow) return;
    if (kWrite && offsets[t.n] > capacity) return;
    const uint32_t nrec = *rec_count;
    if (nrec > rec_cap) return;  // overflowed: the walk-based passes run instead
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = wave0; r < nrec; r += nwaves) {
        const uint4 q = rec[r];  // group first, group count, leaf first, leaf count
        const uint32_t pairs = q.y * q.w;
        for (uint32_t p = lane; p < pairs; p += kWave) {
            const uint32_t a = p / q.w, b = p - a * q.w;
            const uint32_t ki = q.x + a, kj = q.z + b;
            if (ki == kj) continue;
            const double4 pi = t.ps[ki], pj = t.ps[kj];
            if (!nb_pair(pi.x, pi.y, pi.z, t.rsk[ki], pj.x, pj.y, pj.z, t.rsk[kj])) continue;
            const uint32_t oi = t.orig[ki];
            if (kWrite) {
                const uint32_t slot = atomicAdd(&cursor[oi], 1u);
                idx[offsets[oi] + slot] = (int32_t)t.orig[kj];
            } else {
                atomicAdd(&cnt_orig[oi], 1u);
            }
        }
    }
}

// Sorts each list ascending. Short lists (<= 32 entries, almost all) are
// insertion-sorted by one thread; longer ones are queued and sorted by a
// whole block with a bitonic network in LDS (heap sort by one thread above
// kLongMax entries).
constexpr int kShortMax = 32;
constexpr int kLongMax = 4096;

__global__ __launch_bounds__(kThreads) void k_nb_sort_short(const int64_t *offsets, int32_t *idx,
                                                            int64_t n, int64_t capacity,
                                                            const Status *st, uint32_t *long_list,
                                                            uint32_t *long_count) {
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow || offsets[n] > capacity)
        return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = offsets[i], e = offsets[i + 1];
        int64_t len = e - b;
        if (len > kShortMax) {
            long_list[atomicAdd(long_count, 1u)] = (uint32_t)i;
            continue;
        }
        int32_t *a = idx + b;
        for (int64_t p = 1; p < len; p++) {
            int32_t v = a[p];
            int64_t q = p - 1;
            while (q >= 0 && a[q] > v) {
                a[q + 1] = a[q];
                q--;
            }
            a[q + 1] = v;
        }
    }
}

__device__ void heap_sort(int32_t *a, int64_t len) {
    for (int64_t s = len / 2 - 1; s >= 0; s--) {
        int64_t r = s;
        while (true) {
            int64_t c = 2 * r + 1;
            if (c >= len) break;
            if (c + 1 < len && a[c + 1] > a[c]) c++;
            if (a[r] >= a[c]) break;
            int32_t tmp = a[r];
            a[r] = a[c];
            a[c] = tmp;
            r = c;
        }
    }
    for (int64_t end = len - 1; end > 0; end--) {
        int32_t tmp = a[0];
        a[0] = a[end];
        a[end] = tmp;
        int64_t r = 0;
        while (true) {
            int64_t c = 2 * r + 1;
            if (c >= end) break;
            if (c + 1 < end && a[c + 1] > a[c]) c++;
            if (a[r] >= a[c]) break;
            int32_t t2 = a[r];
            a[r] = a[c];
            a[c] = t2;
            r = c;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_nb_sort_long(const int64_t *offsets, int32_t *idx,
                                                           int64_t n, int64_t capacity,
                                                           const Status *st,
                                                           const uint32_t *long_list,
                                                           const uint32_t *long_count) {
    __shared__ int32_t sh[kLongMax];
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow || offsets[n] > capacity)
        return;
    const uint32_t nl = *long_count;
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint32_t i = long_list[q];
        const int64_t b = offsets[i];
        const int64_t len = offsets[i + 1] - b;
        int32_t *a = idx + b;
        if (len > kLongMax) {
            if (threadIdx.x == 0) heap_sort(a, len);
            __syncthreads();
            continue;
        }
        int P = 1;
        while (P < len) P <<= 1;
        for (int t = threadIdx.x; t < P; t += blockDim.x) sh[t] = t < len ? a[t] : 0x7fffffff;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = threadIdx.x; t < P; t += blockDim.x) {
                    int u = t ^ j;
                    if (u > t) {
                        int32_t x = sh[t], y = sh[u];
                        bool up = (t & k) == 0;
                        if ((x > y) == up) {
                            sh[t] = y;
                            sh[u] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int t = threadIdx.x; t < len; t += blockDim.x) a[t] = sh[t];
        __syncthreads();
    }
}

}  // namespace

int nb_resident_waves(int device) {
    int a = 0, b = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_nb<false>, kThreads, 0);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_nb<true>, kThreads, 0);
    int per_cu = a < b ? a : b;
    if (per_cu < 1) per_cu = 1;
    hipDeviceProp_t p;
    hipGetDeviceProperties(&p, device);
    return per_cu * p.multiProcessorCount * kWavesPerBlock;
}

void launch_nb_count_rec(const TreeDev &t, const uint4 *rec, const uint32_t *rec_count,
                         uint32_t rec_cap, const Status *st, uint32_t *cnt_orig, hipStream_t s) {
    hipLaunchKernelGGL(k_nb_rec<false>, dim3(4096), dim3(kThreads), 0, s, t, rec, rec_count, st,
                       cnt_orig, (const int64_t *)nullptr, (uint32_t *)nullptr,
                       (int32_t *)nullptr, (int64_t)0, rec_cap);
}

void launch_nb_write_rec(const TreeDev &t, const uint4 *rec, const uint32_t *rec_count,
                         uint32_t rec_cap, const Status *st, const int64_t *offsets,
                         uint32_t *cursor, int32_t *idx, int64_t capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_nb_rec<true>, dim3(4096), dim3(kThreads), 0, s, t, rec, rec_count, st,
                       (uint32_t *)nullptr, offsets, cursor, idx, capacity, rec_cap);
}

void launch_nb_count(const TreeDev &t, const uint32_t *groups, Status *st, uint32_t *cnt_orig,
                     uint32_t *spill, uint32_t *queue, const uint32_t *rec_count, uint32_t rec_cap,
                     int resident_waves, hipStream_t s) {
    hipLaunchKernelGGL(k_nb<false>, dim3(resident_waves / kWavesPerBlock), dim3(kThreads), 0, s, t,
                       groups, st, cnt_orig, (const int64_t *)nullptr, (int32_t *)nullptr,
                       (int64_t)0, spill, queue, rec_count, rec_cap);
}

void launch_nb_write(const TreeDev &t, const uint32_t *groups, Status *st,
                     const int64_t *offsets, int32_t *idx, int64_t capacity, uint32_t *spill,
                     uint32_t *queue, const uint32_t *rec_count, uint32_t rec_cap,
                     int resident_waves, hipStream_t s) {
    hipLaunchKernelGGL(k_nb<true>, dim3(resident_waves / kWavesPerBlock), dim3(kThreads), 0, s, t,
                       groups, st, (uint32_t *)nullptr, offsets, idx, capacity, spill, queue,
                       rec_count, rec_cap);
}

void launch_nb_sort(const int64_t *offsets, int32_t *idx, int64_t n, int64_t capacity,
                    const Status *st, uint32_t *long_list, uint32_t *long_count, hipStream_t s) {
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_nb_sort_short, dim3((unsigned)blocks), dim3(kThreads), 0, s, offsets, idx,
                       n, capacity, st, long_list, long_count);
    hipLaunchKernelGGL(k_nb_sort_long, dim3(1024), dim3(kThreads), 0, s, offsets, idx, n, capacity,
                       st, (const uint32_t *)long_list, (const uint32_t *)long_count);
}

}  // namespace petar
