// Neighbour candidates (first stage of the neighbour search: all j != i
// with |r_j - r_i| < max(r_search,i, r_search,j)), as CSR lists in input
// order, each sorted by original index.
//
// The force walk hands over, per i-group, every leaf whose box is closer to
// the group's box than max(rs_group, rs_leaf); the pairs of the group with
// those leaves are tested with the FP64 relation of common.h. The box test
// is conservative for the pair test (same rounding, monotone), so every
// candidate is found. A target's candidates lie among the particles of its
// group's near leaves, whose number the force walk stores as the bound of
// its list: a prefix sum of the bounds gives every target a row of scratch
// (input order), one testing pass writes the hits into the rows and counts
// them, a prefix sum of the counts gives the CSR offsets, and a per-list
// sort moves the rows into the CSR. If the hand-over buffers
// overflowed, a walk of the near region per group (same opening rule)
// replaces the hand-over; if the bounds ask for more scratch than the
// caller allows, a counting pass gives exact bounds first.
#include "launch.h"
#include "walk.h"

namespace petar {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

struct NbLds {
    uint32_t stack[kStackLds + kStackSlack];
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

// Tests the buffered leaves' particles against each lane's target and
// writes the hits (input-order indices) at out[wpos + count] (out null:
// counts only).
__device__ void nb_flush(NbLds &L, int nleaf, const TreeDev &t, const double4 &pi, double rsi,
                         uint32_t ki, bool valid, uint32_t &count, int32_t *out, int64_t wpos) {
    wave_sync();
    const int lane = lane_id();
    uint32_t c = lane < nleaf ? L.leaf_cnt[lane] : 0u;
    uint32_t incl = wave_incl_scan(c);
    uint32_t total = last_lane(incl);
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
                if (out) out[wpos + count] = (int32_t)t.orig[kj];
                count++;
            }
        }
        wave_sync();
    }
}

__global__ __launch_bounds__(kThreads) void k_nb(TreeDev t, const uint32_t *groups, Status *st,
                                                 uint32_t *cursor, const int64_t *row_off,
                                                 int32_t *rows, int64_t row_cap, uint32_t *spill,
                                                 uint32_t *queue, NbRecords rec) {
    __shared__ NbLds lds_all[kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    NbLds &L = lds_all[w];
    const int lane = lane_id();
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow) return;
    if (rec.count && rec.count[0] <= rec.head_cap && rec.count[1] <= rec.leaf_cap)
        return;  // the record passes run instead
    if (rows && row_off[t.n] > row_cap) return;
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
            if (rows && valid) wpos = row_off[t.orig[ki]];
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
                        nb_flush(L, nleaf, t, pi, rsi, ki, valid, count, rows, wpos);
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
            if (nleaf) nb_flush(L, nleaf, t, pi, rsi, ki, valid, count, rows, wpos);
            if (valid) cursor[t.orig[ki]] = count;
        }
    }
}

// Neighbour passes over the near leaves handed over by the force walk. A
// header lists one flush of a group's near leaves; a group may have several.
//
// Testing pass. A wave takes one header at a time: the group's targets sit
// in the lanes (FP64 position and squared search radius in registers; a
// group of g < 64 targets puts each target on 64/g lanes that split the
// source loop), the leaves' particles are staged in LDS 64 at a time with
// one load per lane (the next batch is loaded into registers while the
// current one is tested), and every lane tests its target against its share
// of the staged particles (LDS broadcasts). A lane collects its hits in LDS
// and takes kHitBuf slots at a time of its target's row (row_off, input
// order) from a per-target cursor, which ends as the target's count (the
// lists are sorted afterwards, so the slot order is irrelevant). Nothing is
// written when the rows exceed the scratch (row_off[n] > row_cap): the
// caller enlarges it and runs the passes again.
constexpr int kHitBuf = 8;

struct NbRecLds {
    uint32_t start[kWave], pre[kWave];
    double4 jp[kWave];  // x, y, z, r_search^2 of the staged batch
    uint32_t jk[kWave];
    uint32_t hit[kHitBuf][kWave];  // a lane's hits not yet written
};

// The pair relation of common.h with the squares of the search radii:
// for non-negative radii, rounding is monotone, so the rounded square of
// max(rs_i, rs_j) is the larger of the two rounded squares and
// d2 < fl(max^2) holds iff d2 < fl(rs_i^2) or d2 < fl(rs_j^2).
// (Two compares: d2 passes through an empty asm between them, which keeps
// the compiler from folding them into a max that would need a
// canonicalisation of pj.w.)
__device__ __forceinline__ bool nb_pair_sq(const double4 &pi, double rsi2, const double4 &pj) {
#pragma clang fp contract(off)
    double rj2 = pj.w;
    double d2 = sum_sq3(pj.x - pi.x, pj.y - pi.y, pj.z - pi.z);
    const bool near_i = d2 < rsi2;
    asm volatile("" : "+v"(d2), "+v"(rj2));
    return near_i | (d2 < rj2);
}

// kCount: only count each target's hits into cursor (the exact bounds of
// the fallback for rows too large for the scratch; row_off, rows unused).
template <bool kCount>
__global__ __launch_bounds__(kThreads) void k_nb_rec(TreeDev t, NbRecords rec, const Status *st,
                                                     const int64_t *row_off, uint32_t *cursor,
                                                     int32_t *rows, int64_t row_cap) {
    __shared__ NbRecLds lds_all[kWavesPerBlock];
    NbRecLds &L = lds_all[uniform((int)(threadIdx.x / kWave))];
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow) return;
    if (!kCount && row_off[t.n] > row_cap) return;
    const uint32_t nrec = rec.count[0];
    if (nrec > rec.head_cap || rec.count[1] > rec.leaf_cap) return;  // walk-based passes run
    const int lane = lane_id();
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = wave0; r < nrec; r += nwaves) {
        const uint4 q = rec.head[r];
        const uint32_t gfirst = (uint32_t)uniform((int)q.x), gn = (uint32_t)uniform((int)q.y);
        const uint32_t loff = (uint32_t)uniform((int)q.z);
        const int nleaf = uniform((int)q.w);
        uint2 lf = make_uint2(0u, 0u);
        if (lane < nleaf) lf = rec.leaf[loff + lane];
        const uint32_t incl = wave_incl_scan(lf.y);
        const uint32_t total = last_lane(incl);
        wave_sync();
        if (lane < nleaf) {
            L.start[lane] = lf.x;
            L.pre[lane] = incl - lf.y;
        }
        wave_sync();
        for (uint32_t a0 = 0; a0 < gn; a0 += kWave) {
            const int g = (int)(gn - a0 < (uint32_t)kWave ? gn - a0 : (uint32_t)kWave);
            const int S = kWave / g;  // lanes per target
            const int a = lane % g, sl = lane / g;
            const bool act = sl < S;
            const uint32_t ki = gfirst + a0 + (uint32_t)a;
            const double4 pi = t.ps[ki];
            const double rsi = t.rsk[ki];
            const double rsi2 = rsi * rsi;
            const uint32_t oi = t.orig[ki];
            uint32_t c = 0;
            // one batch of 64 sources into registers (lane = source)
            double4 pn = make_double4(0.0, 0.0, 0.0, 0.0);
            uint32_t kn = 0;
            auto gather = [&](uint32_t base) {
                const uint32_t sidx = base + lane;
                if (sidx < total) {
                    const int l = find_leaf(L.pre, nleaf, sidx);
                    kn = L.start[l] + (sidx - L.pre[l]);
                    const double4 p = t.ps[kn];
                    const double rs = t.rsk[kn];
                    pn = make_double4(p.x, p.y, p.z, rs * rs);
                }
            };
            // this lane's buffered hits into its target's row
            auto flush = [&]() {
                const int64_t w0 = row_off[oi] + (int64_t)atomicAdd(&cursor[oi], c);
                for (uint32_t h = 0; h < c; h++) rows[w0 + h] = (int32_t)t.orig[L.hit[h][lane]];
                c = 0;
            };
            // the staged source at byte p of L.jp
            const char *jbase = (const char *)L.jp;
            auto test = [&](const char *p) {
                if (nb_pair_sq(pi, rsi2, *(const double4 *)p)) {
                    const uint32_t kj = L.jk[(uint32_t)(p - jbase) >> 5];
                    if (kj != ki) {
                        if constexpr (!kCount) {
                            if (c == (uint32_t)kHitBuf) flush();
                            L.hit[c][lane] = kj;
                        }
                        c++;
                    }
                }
            };
            gather(0);
            for (uint32_t base = 0; base < total; base += kWave) {
                wave_sync();  // the previous batch has been read
                if (base + lane < total) {
                    L.jp[lane] = pn;
                    L.jk[lane] = kn;
                }
                wave_sync();
                if (base + kWave < total) gather(base + kWave);
                const int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
                if (act) {
                    const int step = S * 32;
                    const char *p = jbase + sl * 32, *pend = jbase + m * 32;
                    for (; p + step < pend; p += 2 * step) {
                        test(p);
                        test(p + step);
                    }
                    if (p < pend) test(p);
                }
            }
            if (c) {
                if constexpr (kCount)
                    atomicAdd(&cursor[oi], c);
                else
                    flush();
            }
            wave_sync();
        }
    }
}

// Sorts each list ascending and moves it from its scratch row into the CSR.
// A block takes 256 consecutive targets (input order); their lists are
// contiguous in the CSR, so the block gathers them from the rows into LDS
// (when they fit; else straight into the CSR), each thread sorts its own
// short list (<= 32 entries, almost all) in registers, and the block writes
// them out with coalesced stores. Longer lists are queued and sorted in the
// CSR: up to kWaveMax entries a wave each (bitonic network over the wave's
// registers, 1 to 32 entries a lane: no barriers, so a list of a few hundred
// entries does not hold a block through hundreds of them), above that a
// block each (bitonic network in LDS), and above kLongMax entries a heap
// sort by one thread.
constexpr int kShortMax = 32;
constexpr int kWaveMax = 32 * kWave;
constexpr int kLongMax = 4096;
constexpr int kStage = 4096;

// A list of at most N entries sorted in registers by a bitonic network of
// N (a power of two) inputs, the tail padded with INT32_MAX. Every lane of
// a wave runs the same network, sized by the longest short list in the wave.
template <int N>
__device__ __forceinline__ void sort_in_registers(int32_t *a, int len) {
    int32_t v[N];
#pragma unroll
    for (int q = 0; q < N; q++) v[q] = q < len ? a[q] : INT32_MAX;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t x = v[i], y = v[l];
                    const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
                    v[i] = (i & k) == 0 ? lo : hi;
                    v[l] = (i & k) == 0 ? hi : lo;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < N; q++)
        if (q < len) a[q] = v[q];
}

__global__ __launch_bounds__(kThreads) void k_nb_sort_short(const int64_t *row_off,
                                                            const int32_t *rows,
                                                            const int64_t *offsets, int32_t *idx,
                                                            int64_t n, int64_t capacity,
                                                            const Status *st, uint32_t *long_list,
                                                            uint32_t *long_count) {
    __shared__ int32_t sh[kStage];
    __shared__ int64_t row0[kThreads];       // row of each target of the block
    __shared__ int64_t dst0[kThreads + 1];   // its list's start in the block's CSR range
    if (st->invalid_radii || st->stack_overflow || st->cell_overflow || offsets[n] > capacity)
        return;
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < n;
         base += (int64_t)gridDim.x * kThreads) {
        const int64_t i = base + threadIdx.x;
        const int64_t iend = base + kThreads < n ? base + kThreads : n;
        const int nt = (int)(iend - base);
        const int64_t r0 = offsets[base], r1 = offsets[iend];
        const bool staged = r1 - r0 <= kStage;  // same for the whole block
        int64_t b = 0, len = 0;
        if (i < n) {
            b = offsets[i];
            len = offsets[i + 1] - b;
        }
        __syncthreads();  // the previous targets are done with the LDS
        if ((int)threadIdx.x < nt) {
            row0[threadIdx.x] = row_off[i];
            dst0[threadIdx.x] = b - r0;
        }
        if (threadIdx.x == 0) dst0[nt] = r1 - r0;
        __syncthreads();
        // entry e of the block's CSR range belongs to the target j with
        // dst0[j] <= e < dst0[j + 1]
        int32_t *dst = staged ? sh : idx + r0;
        for (int64_t e = threadIdx.x; e < r1 - r0; e += kThreads) {
            int lo = 0, hi = nt;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (dst0[mid] <= e)
                    lo = mid;
                else
                    hi = mid;
            }
            dst[e] = rows[row0[lo] + (e - dst0[lo])];
        }
        __syncthreads();
        // longer lists go to the wave or block sorts (one queue slot claim per wave)
        const bool is_long = len > kShortMax;
        const unsigned long long lm = __ballot(is_long);
        if (lm) {
            uint32_t first = 0;
            if (lane_id() == __ffsll((long long)lm) - 1) first = atomicAdd(long_count, (uint32_t)__popcll(lm));
            first = (uint32_t)__shfl((int)first, __ffsll((long long)lm) - 1, kWave);
            if (is_long) long_list[first + (uint32_t)lanes_below(lm)] = (uint32_t)i;
        }
        const int ls = (len > 1 && !is_long) ? (int)len : 0;
        int32_t *a = dst + (b - r0);
        const int m = (int)wave_max((double)ls);
        if (m > 16)
            sort_in_registers<32>(a, ls);
        else if (m > 8)
            sort_in_registers<16>(a, ls);
        else if (m > 4)
            sort_in_registers<8>(a, ls);
        else if (m > 2)
            sort_in_registers<4>(a, ls);
        else if (m > 1)
            sort_in_registers<2>(a, ls);
        if (staged) {
            __syncthreads();
            for (int64_t e = threadIdx.x; e < r1 - r0; e += kThreads) idx[r0 + e] = sh[e];
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

// A list of at most 64 E entries sorted by one wave: entry g = E lane + e in
// register e of its lane, a bitonic network whose exchanges within a lane
// stay in registers and across lanes use a shuffle, the tail padded with
// INT32_MAX.
template <int E>
__device__ __forceinline__ void sort_in_wave(int32_t *a, int len) {
    const int lane = lane_id();
    int32_t v[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int g = lane * E + e;
        v[e] = g < len ? a[g] : INT32_MAX;
    }
#pragma unroll
    for (int k = 2; k <= kWave * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= E) {
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const int g = lane * E + e;
                    const int32_t y = __shfl_xor(v[e], j / E, kWave);
                    const bool keep_min = ((g & k) == 0) == ((g & j) == 0);
                    v[e] = keep_min ? (v[e] < y ? v[e] : y) : (v[e] < y ? y : v[e]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const int l = e ^ j;
                    if (l > e) {
                        const bool up = ((lane * E + e) & k) == 0;
                        const int32_t x = v[e], y = v[l];
                        const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
                        v[e] = up ? lo : hi;
                        v[l] = up ? hi : lo;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int g = lane * E + e;
        if (g < len) a[g] = v[e];
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
    // lists of up to kWaveMax entries: a wave each
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * blockDim.x / kWave;
    for (uint32_t q = wave0; q < nl; q += nwaves) {
        const uint32_t i = long_list[q];
        const int64_t b = offsets[i];
        const int len = (int)uniform((int)(offsets[i + 1] - b > kLongMax ? kLongMax + 1
                                                                           : offsets[i + 1] - b));
        if (len <= kWave)
            sort_in_wave<1>(idx + b, len);
        else if (len <= 2 * kWave)
            sort_in_wave<2>(idx + b, len);
        else if (len <= 4 * kWave)
            sort_in_wave<4>(idx + b, len);
        else if (len <= 8 * kWave)
            sort_in_wave<8>(idx + b, len);
        else if (len <= 16 * kWave)
            sort_in_wave<16>(idx + b, len);
        else if (len <= kWaveMax)
            sort_in_wave<32>(idx + b, len);
    }
    // longer lists: a block each
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint32_t i = long_list[q];
        const int64_t b = offsets[i];
        const int64_t len = offsets[i + 1] - b;
        if (len <= kWaveMax) continue;
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
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_nb, kThreads, 0) != hipSuccess)
        per_cu = 1;
    if (per_cu < 1) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 256;  // MI355X
    return per_cu * cus * kWavesPerBlock;
}

void launch_nb_write_rec(const TreeDev &t, const NbRecords &rec, const Status *st,
                         const int64_t *row_off, uint32_t *cursor, int32_t *rows, int64_t row_cap,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_nb_rec<false>, dim3(2048), dim3(kThreads), 0, s, t, rec, st, row_off,
                       cursor, rows, row_cap);
}

void launch_nb_count_rec(const TreeDev &t, const NbRecords &rec, const Status *st,
                         uint32_t *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_nb_rec<true>, dim3(2048), dim3(kThreads), 0, s, t, rec, st,
                       (const int64_t *)nullptr, cnt, (int32_t *)nullptr, (int64_t)0);
}

void launch_nb_write(const TreeDev &t, const uint32_t *groups, Status *st, uint32_t *cursor,
                     const int64_t *row_off, int32_t *rows, int64_t row_cap, uint32_t *spill,
                     uint32_t *queue, const NbRecords &rec, int resident_waves, hipStream_t s) {
    hipLaunchKernelGGL(k_nb, dim3(resident_waves / kWavesPerBlock), dim3(kThreads), 0, s, t,
                       groups, st, cursor, row_off, rows, row_cap, spill, queue, rec);
}

__global__ void k_nb_summary(const int64_t *offsets, const int64_t *row_off, int64_t n,
                             const uint32_t *rec_count, Status *st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->nb_total = offsets[n];
        st->nb_rows = row_off[n];
        st->rec_used[0] = rec_count[0];
        st->rec_used[1] = rec_count[1];
    }
}

void launch_nb_summary(const int64_t *offsets, const int64_t *row_off, int64_t n,
                       const uint32_t *rec_count, Status *st, hipStream_t s) {
    hipLaunchKernelGGL(k_nb_summary, dim3(1), dim3(kWave), 0, s, offsets, row_off, n, rec_count,
                       st);
}

void launch_nb_sort(const int64_t *row_off, const int32_t *rows, const int64_t *offsets,
                    int32_t *idx, int64_t n, int64_t capacity, const Status *st,
                    uint32_t *long_list, uint32_t *long_count, hipStream_t s) {
    int64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_nb_sort_short, dim3((unsigned)blocks), dim3(kThreads), 0, s, row_off,
                       rows, offsets, idx, n, capacity, st, long_list, long_count);
    hipLaunchKernelGGL(k_nb_sort_long, dim3(1024), dim3(kThreads), 0, s, offsets, idx, n, capacity,
                       st, (const uint32_t *)long_list, (const uint32_t *)long_count);
}

}  // namespace petar
