// Long-range force kernel: group-wise tree walk fused with the interaction
// passes, one wavefront per i-group, persistent over per-XCD work queues.
//
// Per group the walk sorts every cell it reaches into
//   multipole (PC): the cell is inside the opening angle and no pair can be
//                   within search range -> monopole + quadrupole field;
//   far leaf:       opened leaf out of search range -> Newtonian pairs;
//   near leaf:      opened leaf within search range -> pairs weighted by
//                   the changeover functions (1 - K) and (1 - W)/r.
// Cells are buffered in LDS; a full buffer is staged as records relative to
// the group centre (FP32 in mixed mode, FP64 otherwise) and broadcast from
// LDS to all lanes. A lane holds up to IPL targets; small groups spread one
// target over S lanes that split the j loop. In mixed precision the FP32
// per-tile partial sums are folded into Neumaier-compensated FP32
// accumulators and converted to FP64 at the end.
#include "launch.h"
#include "walk.h"

namespace petar {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr float kFarAway = 1e18f;  // position of padding records (zero mass)

template <typename R>
struct Vec;
template <>
struct Vec<float> {
    using v4 = float4;
    using v2 = float2;
};
template <>
struct Vec<double> {
    using v4 = double4;
    using v2 = double2;
};

// One tile of up to 64 sources, structure of arrays so that every read is an
// aligned 16/8/4-byte broadcast:
//   PC:   a = (x, y, z, M), b = (A'xx, A'yy, A'zz, A'xy), c = (A'xz, A'yz)
//   far:  a = (x, y, z, m)
//   near: a = (x, y, z, m), c = (r_in, r_out), k = index in Morton order
template <typename R>
struct Tile {
    typename Vec<R>::v4 a[kWave];
    typename Vec<R>::v4 b[kWave];
    typename Vec<R>::v2 c[kWave];
    uint32_t k[kWave];
};

template <typename R>
struct WaveLds {
    uint32_t stack[kStackLds];
    uint32_t pc_buf[kWave];
    uint32_t far_start[kWave], far_pre[kWave];
    uint32_t near_start[kWave], near_pre[kWave];
    GroupGeom g;
    Tile<R> tile;
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Accumulators: tile partials folded into compensated sums (FP32) or plain
// FP64 sums.
template <typename R>
struct Acc;
template <>
struct Acc<float> {
    float s[4], c[4];
    __device__ void zero() {
        for (int k = 0; k < 4; k++) s[k] = c[k] = 0.f;
    }
    __device__ void add(int k, float v) {
        float t = s[k] + v;
        c[k] += (fabsf(s[k]) >= fabsf(v)) ? ((s[k] - t) + v) : ((v - t) + s[k]);
        s[k] = t;
    }
    __device__ double get(int k) const { return (double)s[k] + (double)c[k]; }
};
template <>
struct Acc<double> {
    double s[4];
    __device__ void zero() {
        for (int k = 0; k < 4; k++) s[k] = 0.0;
    }
    __device__ void add(int k, double v) { s[k] += v; }
    __device__ double get(int k) const { return s[k]; }
};

// Folds the partial sums of the lanes lane ^ d (d = W, 2W, .., 32) that
// handled other j subsets of the same target.
__device__ __forceinline__ void combine_split(Acc<float> &a, int W) {
    for (int d = W; d < kWave; d <<= 1) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            float s2 = __shfl_xor(a.s[k], d, kWave);
            float c2 = __shfl_xor(a.c[k], d, kWave);
            a.add(k, s2);
            a.c[k] += c2;
        }
    }
}
__device__ __forceinline__ void combine_split(Acc<double> &a, int W) {
    for (int d = W; d < kWave; d <<= 1) {
#pragma unroll
        for (int k = 0; k < 4; k++) a.s[k] += __shfl_xor(a.s[k], d, kWave);
    }
}

template <typename R, int IPL>
struct Targets {
    R x[IPL], y[IPL], z[IPL], rin[IPL], rout[IPL];
    uint32_t k[IPL];  // index in Morton order, kNone for an empty slot
    Acc<R> acc[IPL];
};

// Work layout of the current chunk of targets (wave-uniform except sl).
struct Layout {
    int nu;  // target slots in use per lane (1..IPL)
    int S;   // lanes sharing a target (j loop split), 1 when nu > 1
    int sl;  // this lane's j subset
};

// ---------------------------------------------------------------- loops
// Each loop runs uniformly over a tile padded to a multiple of pad_of(S):
// S lanes share a target and take every S-th source; F sources per lane
// are unrolled per iteration.

__host__ __device__ constexpr int pad_of(int S) { return S >= 4 ? S : 4; }

template <typename R, int U>
struct Partial {
    R ax[U], ay[U], az[U], ph[U];
    __device__ void zero() {
#pragma unroll
        for (int u = 0; u < U; u++) ax[u] = ay[u] = az[u] = ph[u] = (R)0;
    }
};

template <typename R, int IPL, int U>
__device__ __forceinline__ void pc_one(const typename Vec<R>::v4 &a, const typename Vec<R>::v4 &b,
                                       const typename Vec<R>::v2 &c, const Targets<R, IPL> &T,
                                       Partial<R, U> &P) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        R Rx = T.x[u] - a.x, Ry = T.y[u] - a.y, Rz = T.z[u] - a.z;
        R r2 = Rx * Rx + Ry * Ry + Rz * Rz;
        R ri = rsq(r2);
        R ri2 = ri * ri;
        R qx = b.x * Rx + b.w * Ry + c.x * Rz;
        R qy = b.w * Rx + b.y * Ry + c.y * Rz;
        R qz = c.x * Rx + c.y * Ry + b.z * Rz;
        R rqr = Rx * qx + Ry * qy + Rz * qz;
        R ri3 = ri * ri2;
        R ri5 = ri3 * ri2;
        R mri = a.w * ri;
        R t = rqr * ri5;                  // R.A'R / r^5
        R t7 = t * ri2;                   // R.A'R / r^7
        R coef = (R)5 * t7 + mri * ri2;   // M/r^3 + 5 R.A'R/r^7
        R two5 = ri5 + ri5;
        // a += (2/r^5) A'R - coef R ;  phi -= M/r + R.A'R/r^5
        P.ax[u] += two5 * qx;
        P.ay[u] += two5 * qy;
        P.az[u] += two5 * qz;
        P.ax[u] -= coef * Rx;
        P.ay[u] -= coef * Ry;
        P.az[u] -= coef * Rz;
        P.ph[u] -= mri;
        P.ph[u] -= t;
    }
}

template <typename R, int IPL, int U>
__device__ __forceinline__ void far_one(const typename Vec<R>::v4 &p, const Targets<R, IPL> &T,
                                        Partial<R, U> &P) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        R dx = p.x - T.x[u], dy = p.y - T.y[u], dz = p.z - T.z[u];
        R r2 = dx * dx + dy * dy + dz * dz;
        R ri = rsq(r2);
        R mri = p.w * ri;
        R mri3 = mri * ri * ri;
        P.ax[u] += mri3 * dx;
        P.ay[u] += mri3 * dy;
        P.az[u] += mri3 * dz;
        P.ph[u] -= mri;
    }
}

template <typename R, int IPL, int U>
__device__ __forceinline__ void near_one(const typename Vec<R>::v4 &p,
                                         const typename Vec<R>::v2 &rr, uint32_t kj,
                                         const Targets<R, IPL> &T, Partial<R, U> &P) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        R dx = p.x - T.x[u], dy = p.y - T.y[u], dz = p.z - T.z[u];
        R r2 = dx * dx + dy * dy + dz * dz;
        R rin = T.rin[u] > rr.x ? T.rin[u] : rr.x;
        R rout = T.rout[u] > rr.y ? T.rout[u] : rr.y;
        R ri = r2 > (R)0 ? rsq(r2) : (R)0;
        R r = r2 * ri;
        R dr = rout - rin;
        R sum = rout + rin;
        R x = (r - rin) * rcp(dr);
        R lam = dr * rcp(sum);
        R xc = x < (R)0 ? (R)0 : (x > (R)1 ? (R)1 : x);
        R x2 = xc * xc, x4 = x2 * x2;
        R xm = xc - (R)1, xm2 = xm * xm;
        // 1 - K(x) = x^4 [(35 - 84x + 70x^2 - 20x^3) - 35 Lambda (x-1)^4]
        R fw = x4 * (((R)35 + xc * ((R)-84 + xc * ((R)70 - (R)20 * xc))) -
                     (R)35 * lam * xm2 * xm2);
        // (1 - W)/r = 2/(r_in + r_out) - Lambda x^5 (14 - 28x + 20x^2 - 5x^3)/r
        R pw_in = (R)2 * rcp(sum) -
                  lam * x4 * xc * ((R)14 + xc * ((R)-28 + xc * ((R)20 - (R)5 * xc))) * ri;
        R pw = x >= (R)1 ? ri : pw_in;
        bool self = kj == T.k[u];
        fw = self ? (R)0 : fw;
        pw = self ? (R)0 : pw;
        R mf = p.w * fw * ri * ri * ri;
        P.ax[u] += mf * dx;
        P.ay[u] += mf * dy;
        P.az[u] += mf * dz;
        P.ph[u] -= p.w * pw;
    }
}

enum { kTilePc = 0, kTileFar = 1, kTileNear = 2 };

// mpad is a multiple of pad_of(S); F sources per lane per iteration.
template <int KIND, int U, int S, typename R, int IPL>
__device__ void loop_kind(const Tile<R> &tile, int mpad, int sl, Targets<R, IPL> &T) {
    constexpr int F = KIND == kTileFar ? pad_of(S) / S : (KIND == kTilePc && S <= 2 ? 2 : 1);
    Partial<R, U> P;
    P.zero();
    for (int jj = 0; jj < mpad; jj += F * S) {
#pragma unroll
        for (int f = 0; f < F; f++) {
            const int j = jj + f * S + sl;
            if (KIND == kTilePc) pc_one<R, IPL, U>(tile.a[j], tile.b[j], tile.c[j], T, P);
            if (KIND == kTileFar) far_one<R, IPL, U>(tile.a[j], T, P);
            if (KIND == kTileNear) near_one<R, IPL, U>(tile.a[j], tile.c[j], tile.k[j], T, P);
        }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        T.acc[u].add(0, P.ax[u]);
        T.acc[u].add(1, P.ay[u]);
        T.acc[u].add(2, P.az[u]);
        T.acc[u].add(3, P.ph[u]);
    }
}

// Runs the loop of a staged tile with the number of target slots in use and
// the split factor (both wave-uniform).
template <int KIND, typename R, int IPL>
__device__ __forceinline__ void run_tile(const Tile<R> &tile, int mpad, const Layout &ly,
                                         Targets<R, IPL> &T) {
    constexpr int U2 = IPL >= 2 ? 2 : 1;
    if (IPL > 2 && ly.nu > 2)
        loop_kind<KIND, IPL, 1>(tile, mpad, ly.sl, T);
    else if (IPL >= 2 && ly.nu == 2)
        loop_kind<KIND, U2, 1>(tile, mpad, ly.sl, T);
    else if (ly.S == 1)
        loop_kind<KIND, 1, 1>(tile, mpad, ly.sl, T);
    else if (ly.S == 2)
        loop_kind<KIND, 1, 2>(tile, mpad, ly.sl, T);
    else if (ly.S == 4)
        loop_kind<KIND, 1, 4>(tile, mpad, ly.sl, T);
    else
        loop_kind<KIND, 1, 8>(tile, mpad, ly.sl, T);
}

__device__ __forceinline__ int pad_to(int m, int S) {
    const int q = pad_of(S);
    return (m + q - 1) / q * q;
}

// ---- multipole tile
template <typename R, int IPL>
__device__ void flush_pc(WaveLds<R> &L, int npc, const ForceLaunch &f, const Layout &ly,
                         Targets<R, IPL> &T) {
    wave_sync();
    const int lane = lane_id();
    const int mpad = pad_to(npc, ly.S);
    if (lane < npc) {
        uint32_t c = L.pc_buf[lane];
        double4 cm = f.t.nd_com[c];
        const double *S = f.t.nd_S + (int64_t)c * 6;
        double tr = S[0] + S[1] + S[2];
        L.tile.a[lane] = {(R)(cm.x - L.g.c[0]), (R)(cm.y - L.g.c[1]), (R)(cm.z - L.g.c[2]),
                          (R)cm.w};
        L.tile.b[lane] = {(R)(1.5 * S[0] - 0.5 * tr), (R)(1.5 * S[1] - 0.5 * tr),
                          (R)(1.5 * S[2] - 0.5 * tr), (R)(1.5 * S[3])};
        L.tile.c[lane] = {(R)(1.5 * S[4]), (R)(1.5 * S[5])};
    } else if (lane < mpad) {
        L.tile.a[lane] = {(R)kFarAway, (R)kFarAway, (R)kFarAway, (R)0};
        L.tile.b[lane] = {(R)0, (R)0, (R)0, (R)0};
        L.tile.c[lane] = {(R)0, (R)0};
    }
    wave_sync();
    run_tile<kTilePc>(L.tile, mpad, ly, T);
    wave_sync();
}

// Binary search of the buffered leaf that holds expanded slot s.
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

// ---- leaves (far: Newtonian pairs; near: changeover pairs). On entry
// pre[] holds each buffered leaf's particle count; it is turned into an
// exclusive prefix and the particles are expanded in tiles of 64.
template <int KIND, typename R, int IPL>
__device__ uint32_t flush_leaves(WaveLds<R> &L, const uint32_t *start, uint32_t *pre, int nleaf,
                                 const ForceLaunch &f, const Layout &ly, Targets<R, IPL> &T,
                                 bool record, uint32_t gstart, uint32_t gn) {
    wave_sync();
    const int lane = lane_id();
    uint32_t c = lane < nleaf ? pre[lane] : 0u;
    if (KIND == kTileNear && record) {
        // hand the near leaves of this group to the neighbour-list passes:
        // one header per flush and the flushed leaves
        uint32_t hb = 0, lb = 0;
        if (lane == 0) {
            hb = atomicAdd(&f.nb.count[0], 1u);
            lb = atomicAdd(&f.nb.count[1], (uint32_t)nleaf);
        }
        hb = (uint32_t)uniform((int)hb);
        lb = (uint32_t)uniform((int)lb);
        if (hb < f.nb.head_cap && (uint64_t)lb + (uint64_t)nleaf <= f.nb.leaf_cap) {
            if (lane < nleaf) f.nb.leaf[lb + lane] = make_uint2(start[lane], c);
            if (lane == 0) f.nb.head[hb] = make_uint4(gstart, gn, lb, (uint32_t)nleaf);
        }
    }
    uint32_t incl = wave_incl_scan(c);
    uint32_t total = (uint32_t)uniform((int)__shfl(incl, kWave - 1, kWave));
    if (lane < nleaf) pre[lane] = incl - c;
    wave_sync();
    for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t s = base + lane;
        const int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
        const int mpad = pad_to(m, ly.S);
        if (s < total) {
            int l = find_leaf(pre, nleaf, s);
            uint32_t k = start[l] + (s - pre[l]);
            double4 p = f.t.ps[k];
            L.tile.a[lane] = {(R)(p.x - L.g.c[0]), (R)(p.y - L.g.c[1]), (R)(p.z - L.g.c[2]),
                              (R)p.w};
            if (KIND == kTileNear) {
                double2 rr = f.t.rr[k];
                L.tile.c[lane] = {(R)rr.x, (R)rr.y};
                L.tile.k[lane] = k;
            }
        } else if (lane < mpad) {
            L.tile.a[lane] = {(R)kFarAway, (R)kFarAway, (R)kFarAway, (R)0};
            if (KIND == kTileNear) {
                L.tile.c[lane] = {(R)0, (R)1};
                L.tile.k[lane] = kNone - 1;
            }
        }
        wave_sync();
        run_tile<KIND>(L.tile, mpad, ly, T);
        wave_sync();
    }
    return total;
}

enum { kKindNone = 0, kKindPc = 1, kKindFar = 2, kKindNear = 3, kKindOpen = 4 };

template <typename R, int IPL>
__global__ __launch_bounds__(kThreads) void k_force(ForceLaunch f) {
    __shared__ WaveLds<R> lds_all[kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    WaveLds<R> &L = lds_all[w];
    const int lane = lane_id();
    const int64_t gwave = (int64_t)blockIdx.x * kWavesPerBlock + w;
    if (f.st_in->invalid_radii || f.st_in->cell_overflow) return;
    const int64_t n_groups = f.st_in->n_groups;
    const int64_t n = f.t.n;
    WaveStack stk;
    stk.lds = L.stack;
    stk.spill = f.spill + gwave * kSpillCap;
    unsigned long long cnt_pc = 0, cnt_far = 0, cnt_near = 0;
    int q = blockIdx.x & 7;  // work queue of this XCD
    int moves = 0;
    const int CH = kWave * IPL;
    while (true) {
        int64_t qlo = n_groups * q / 8, qhi = n_groups * (q + 1) / 8;
        uint32_t v = 0;
        if (lane == 0) v = atomicAdd(&f.queue[q], 1u);
        v = (uint32_t)uniform((int)v);
        int64_t g = qlo + (int64_t)v;
        if (g >= qhi) {
            if (++moves >= 8) break;
            q = (q + 1) & 7;
            continue;
        }
        const uint32_t gnode = (uint32_t)uniform((int)f.groups[g]);
        const uint4 ginfo = f.t.nd_info[gnode];
        wave_sync();
        if (lane == 0) L.g = load_group(f.t.nd_lo, f.t.nd_hi, gnode);
        wave_sync();
        const uint32_t gstart = (uint32_t)uniform((int)ginfo.x);
        const uint32_t gn = (uint32_t)uniform((int)ginfo.y);
        for (uint32_t chunk = 0; chunk < gn; chunk += CH) {
            const uint32_t active = gn - chunk < (uint32_t)CH ? gn - chunk : (uint32_t)CH;
            Layout ly;
            ly.nu = (int)((active + kWave - 1) / kWave);
            // One slot in use: S lanes share a target and split the j loop
            // (lane = sl * W + il).
            ly.S = ly.nu > 1 ? 1 : (active <= 8 ? 8 : (active <= 16 ? 4 : (active <= 32 ? 2 : 1)));
            const int W = kWave / ly.S;
            const int il = lane & (W - 1);
            ly.sl = lane / W;
            Targets<R, IPL> T;
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                uint32_t off = chunk + u * kWave + il;
                bool valid = off < gn;
                uint32_t k = gstart + (valid ? off : 0u);
                double4 p = f.t.ps[k];
                double2 rr = f.t.rr[k];
                T.x[u] = (R)(p.x - L.g.c[0]);
                T.y[u] = (R)(p.y - L.g.c[1]);
                T.z[u] = (R)(p.z - L.g.c[2]);
                T.rin[u] = (R)rr.x;
                T.rout[u] = (R)rr.y;
                T.k[u] = valid ? k : kNone;
                T.acc[u].zero();
            }
            uint64_t n_pc = 0, n_far = 0, n_near = 0;
            int npc = 0, nfar = 0, nnear = 0;
            const bool record = f.nb.head != nullptr && chunk == 0;
            stk.init((uint32_t)uniform((int)root_of(f.t.nd_info, f.t.level_off, gstart)));
            bool ok = true;
            while (!stk.empty()) {
                uint32_t node = stk.pop();
                int kind = kKindNone;
                uint4 info = make_uint4(0, 0, 0, 0);
                if (node != kNone) {
                    double4 lo = f.t.nd_lo[node], hi = f.t.nd_hi[node], cm = f.t.nd_com[node];
                    info = f.t.nd_info[node];
                    double D2, R2;
                    box_terms(L.g, lo, hi, &D2, &R2);
                    bool near = D2 < R2;
                    if (!near && mac_accept(L.g, cm, hi.w, f.th2))
                        kind = kKindPc;
                    else if (info.z & kLeafFlag)
                        kind = near ? kKindNear : kKindFar;
                    else
                        kind = kKindOpen;
                }
                int nc = kind == kKindOpen ? info_nchild(info.z) : 0;
                if (!stk.push(info.w, nc)) {
                    ok = false;
                    break;
                }
                unsigned long long m;
                int cnt;
                m = __ballot(kind == kKindPc);
                cnt = __popcll(m);
                if (cnt) {
                    if (npc + cnt > kWave) {
                        flush_pc(L, npc, f, ly, T);
                        n_pc += npc;
                        npc = 0;
                    }
                    if (kind == kKindPc) L.pc_buf[npc + lanes_below(m)] = node;
                    npc += cnt;
                }
                m = __ballot(kind == kKindFar);
                cnt = __popcll(m);
                if (cnt) {
                    if (nfar + cnt > kWave) {
                        n_far += flush_leaves<kTileFar>(L, L.far_start, L.far_pre, nfar, f, ly, T,
                                                        false, gstart, gn);
                        nfar = 0;
                    }
                    if (kind == kKindFar) {
                        int p = nfar + lanes_below(m);
                        L.far_start[p] = info.x;
                        L.far_pre[p] = info.y;
                    }
                    nfar += cnt;
                }
                m = __ballot(kind == kKindNear);
                cnt = __popcll(m);
                if (cnt) {
                    if (nnear + cnt > kWave) {
                        n_near += flush_leaves<kTileNear>(L, L.near_start, L.near_pre, nnear, f,
                                                          ly, T, record, gstart, gn);
                        nnear = 0;
                    }
                    if (kind == kKindNear) {
                        int p = nnear + lanes_below(m);
                        L.near_start[p] = info.x;
                        L.near_pre[p] = info.y;
                    }
                    nnear += cnt;
                }
            }
            if (!ok) {
                if (lane == 0) atomicAdd(&f.st->stack_overflow, 1);
                break;
            }
            if (npc) {
                flush_pc(L, npc, f, ly, T);
                n_pc += npc;
            }
            if (nfar) n_far += flush_leaves<kTileFar>(L, L.far_start, L.far_pre, nfar, f, ly, T,
                                                        false, gstart, gn);
            if (nnear)
                n_near += flush_leaves<kTileNear>(L, L.near_start, L.near_pre, nnear, f, ly, T,
                                                  record, gstart, gn);
            cnt_pc += n_pc * active;
            cnt_far += n_far * active;
            cnt_near += n_near * active - active;  // minus the self pairs
            if (ly.S > 1) combine_split(T.acc[0], W);
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                if (T.k[u] == kNone || ly.sl != 0) continue;
                uint32_t o = f.t.orig[T.k[u]];
                f.acc[o] = f.G * T.acc[u].get(0);
                f.acc[n + o] = f.G * T.acc[u].get(1);
                f.acc[2 * n + o] = f.G * T.acc[u].get(2);
                f.pot[o] = f.G * T.acc[u].get(3);
                if (f.counts) {
                    f.counts[o] = (int32_t)n_pc;
                    f.counts[n + o] = (int32_t)n_far;
                    f.counts[2 * n + o] = (int32_t)n_near;
                    f.counts[3 * n + o] = (int32_t)gn;
                }
            }
        }
    }
    if (lane == 0) {
        if (cnt_pc) atomicAdd(&f.st->inter[0], cnt_pc);
        if (cnt_far) atomicAdd(&f.st->inter[1], cnt_far);
        if (cnt_near) atomicAdd(&f.st->inter[2], cnt_near);
    }
}

template <typename R, int IPL>
int resident_for(int device) {
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force<R, IPL>, kThreads, 0);
    hipDeviceProp_t p;
    (void)hipGetDeviceProperties(&p, device);
    if (per_cu < 1) per_cu = 1;
    return per_cu * p.multiProcessorCount * kWavesPerBlock;
}

template <typename R, int IPL>
void launch_t(const ForceLaunch &f, int resident_waves, hipStream_t s) {
    int blocks = resident_waves / kWavesPerBlock;
    hipLaunchKernelGGL((k_force<R, IPL>), dim3(blocks), dim3(kThreads), 0, s, f);
}

}  // namespace

int64_t force_spill_elems_per_wave() { return kSpillCap; }

int force_resident_waves(int precision, int ipl, int device) {
    if (precision == 1) {
        if (ipl == 4) return resident_for<double, 4>(device);
        if (ipl == 2) return resident_for<double, 2>(device);
        return resident_for<double, 1>(device);
    }
    if (ipl == 4) return resident_for<float, 4>(device);
    if (ipl == 2) return resident_for<float, 2>(device);
    return resident_for<float, 1>(device);
}

void launch_force(const ForceLaunch &f, int resident_waves, hipStream_t s) {
    if (f.precision == 1) {
        if (f.ipl == 4)
            launch_t<double, 4>(f, resident_waves, s);
        else if (f.ipl == 2)
            launch_t<double, 2>(f, resident_waves, s);
        else
            launch_t<double, 1>(f, resident_waves, s);
    } else {
        if (f.ipl == 4)
            launch_t<float, 4>(f, resident_waves, s);
        else if (f.ipl == 2)
            launch_t<float, 2>(f, resident_waves, s);
        else
            launch_t<float, 1>(f, resident_waves, s);
    }
}

}  // namespace petar
