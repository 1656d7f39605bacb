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
// target over S lanes that split the j loop. In mixed precision each tile of
// at most 64 sources is summed in FP32 and the tile partials are accumulated
// in FP64 (two instructions per component and tile; a Neumaier-compensated
// FP32 sum takes seven).
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

// Tiles of up to 64 sources (plus padding); every read is an aligned
// 16/8/4-byte broadcast:
//   multipoles: a = (x, y, z, M), b = 2 (A'xx, A'yy, A'zz, A'xy), c = 2 (A'xz, A'yz)
//   particles:  a = (x, y, z, m), c = (r_in, r_out), k = index in Morton order
//               (far leaves use a only)
// Multipole entries are written by the walk as soon as a cell is accepted
// (its data are already in registers); particle entries are expanded from
// the buffered leaves when those are flushed.
constexpr int kTileCap = 72;  // 64 entries + padding up to a multiple of the loop step

template <typename R>
struct PcEntry {
    typename Vec<R>::v4 a, b;
    typename Vec<R>::v2 c, pad;
};
template <typename R>
struct PartEntry {
    typename Vec<R>::v4 a;
    typename Vec<R>::v2 c;
    uint32_t k, pad[sizeof(R) == 4 ? 1 : 3];
};
// Array of entries: one LDS base per tile, immediate offsets per field.
template <typename R>
struct PcTile {
    PcEntry<R> e[kTileCap];
};
template <typename R>
struct PartTile {
    PartEntry<R> e[kTileCap];
};

template <typename R>
struct WaveLds {
    uint32_t stack[kStackLds + kStackSlack];
    uint32_t far_start[kWave], far_pre[kWave];
    uint32_t near_start[kWave], near_pre[kWave];
    GroupGeom g;
    PcTile<R> pc;
    PartTile<R> part;
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Accumulators: FP64 sums of the tile partials (FP32 partials in mixed
// precision, FP64 ones otherwise).
template <typename R>
struct Acc;
template <>
struct Acc<float> {
    double s[4];  // FP64 sums of the FP32 tile partials
    __device__ void zero() {
        for (int k = 0; k < 4; k++) s[k] = 0.0;
    }
    __device__ void add(int k, float v) { s[k] += (double)v; }
    __device__ double get(int k) const { return s[k]; }
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

template <typename R, int IPL>
struct Targets {
    R x[IPL], y[IPL], z[IPL], rin[IPL], rout[IPL];
    uint32_t k[IPL];  // index in Morton order, kNone for an empty slot
    Acc<R> acc[IPL];
};

// Work layout of a chunk of targets. nu target slots per lane are in use;
// W lanes hold one slot each of distinct targets, and S = 64 / W such lane
// sets split the source loop (lane = sl * W + il). Lanes past S * W idle:
// they mirror split 0 and their sums are dropped. Everything but sl, il and
// act is wave-uniform.
struct Layout {
    int nu, W, S;
    int sl, il;
    bool act;
};

// Chooses (nu, S) to keep as many lanes busy as possible: nu = 1 with
// S = 64 / active lanes per target, or, when the kernel holds two targets
// per lane and it is better, nu = 2 with S = 64 / ceil(active/2); chunks
// above 64 targets use nu = ceil(active / 64), S = 1. Splits up to
// kSplitFixed have loops of their own (fixed stride, unrolled, tiles padded
// to the step); wider ones (groups of at most 7 targets) share a loop with
// the stride in a register and no padding.
template <int IPL>
__device__ __forceinline__ Layout choose_layout(uint32_t active) {
    Layout ly;
    if (active > (uint32_t)kWave) {
        ly.nu = (int)((active + kWave - 1) / kWave);
        ly.W = kWave;
        ly.S = 1;
    } else {
        const int a = (int)active;
        const int S1 = kWave / a;
        ly.nu = 1;
        ly.W = a;
        ly.S = S1;
        if (IPL >= 2 && a >= 2) {
            const int W2 = (a + 1) / 2;
            const int S2 = kWave / W2;
            if (S2 > 2 * S1) {  // utilisation a * S / (64 * nu) is higher
                ly.nu = 2;
                ly.W = W2;
                ly.S = S2;
            }
        }
    }
    const int lane = lane_id();
    ly.sl = lane / ly.W;
    ly.il = lane - ly.sl * ly.W;
    ly.act = ly.sl < ly.S;
    if (!ly.act) ly.sl = 0;
    return ly;
}

// ---------------------------------------------------------------- loops
// Each loop runs uniformly over a tile padded to a multiple of its step
// F * S: S lanes share a target and take every S-th source, F sources per
// lane are unrolled per iteration.
enum { kTilePc = 0, kTileFar = 1, kTileNear = 2 };
constexpr int kSplitFixed = 8;  // widest split with a fixed-stride loop

__host__ __device__ constexpr int unroll_of(int kind, int S) {
    return kind == kTileFar ? (S >= 4 ? 1 : 4 / S) : (kind == kTilePc && S <= 4 ? 2 : 1);
}
__device__ __forceinline__ int pad_to(int m, int kind, int S) {
    if (S > kSplitFixed) return m;  // runtime stride: lanes past the end are masked
    const int q = unroll_of(kind, S) * S;
    return (m + q - 1) / q * q;
}

template <typename R, int U>
struct Partial {
    R ax[U], ay[U], az[U], ph[U];
    __device__ void zero() {
#pragma unroll
        for (int u = 0; u < U; u++) ax[u] = ay[u] = az[u] = ph[u] = (R)0;
    }
};

// Multipole term of one cell: with R the target minus the centre of mass,
// q = A'R and the tile holding 2A' (so q2 = 2q):
//   a   += (2/r^5) A'R - (M/r^3 + 5 R.A'R/r^7) R
//   phi -= M/r + R.A'R/r^5
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
        R qx = b.x * Rx + b.w * Ry + c.x * Rz;  // 2 A'R
        R qy = b.w * Rx + b.y * Ry + c.y * Rz;
        R qz = c.x * Rx + c.y * Ry + b.z * Rz;
        R rqr = Rx * qx + Ry * qy + Rz * qz;    // 2 R.A'R
        R ri5 = ri * (ri2 * ri2);
        R mri = a.w * ri;                       // M/r
        R t2 = rqr * ri5;                       // 2 R.A'R / r^5
        R coef = ((R)2.5 * t2 + mri) * ri2;     // M/r^3 + 5 R.A'R/r^7
        P.ax[u] += ri5 * qx;
        P.ay[u] += ri5 * qy;
        P.az[u] += ri5 * qz;
        P.ax[u] -= coef * Rx;
        P.ay[u] -= coef * Ry;
        P.az[u] -= coef * Rz;
        P.ph[u] -= mri;
        P.ph[u] -= (R)0.5 * t2;
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

// mpad is a multiple of the step F * S.
template <int KIND, int U, int S, typename R, int IPL, typename TileT>
__device__ void loop_kind(const TileT &tile, int mpad, int sl, Targets<R, IPL> &T) {
    constexpr int F = unroll_of(KIND, S);
    Partial<R, U> P;
    P.zero();
    for (int jj = 0; jj < mpad; jj += F * S) {
#pragma unroll
        for (int f = 0; f < F; f++) {
            const int j = jj + f * S + sl;
            if constexpr (KIND == kTilePc)
                pc_one<R, IPL, U>(tile.e[j].a, tile.e[j].b, tile.e[j].c, T, P);
            else if constexpr (KIND == kTileFar)
                far_one<R, IPL, U>(tile.e[j].a, T, P);
            else
                near_one<R, IPL, U>(tile.e[j].a, tile.e[j].c, tile.e[j].k, T, P);
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

// Splits wider than kSplitFixed: the stride S is a register, each lane
// takes entries sl, sl + S, ... below m (no padding).
template <int KIND, int U, typename R, int IPL, typename TileT>
__device__ void loop_kind_wide(const TileT &tile, int m, int sl, int S, Targets<R, IPL> &T) {
    Partial<R, U> P;
    P.zero();
    for (int j = sl; j < m; j += S) {
        if constexpr (KIND == kTilePc)
            pc_one<R, IPL, U>(tile.e[j].a, tile.e[j].b, tile.e[j].c, T, P);
        else if constexpr (KIND == kTileFar)
            far_one<R, IPL, U>(tile.e[j].a, T, P);
        else
            near_one<R, IPL, U>(tile.e[j].a, tile.e[j].c, tile.e[j].k, T, P);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        T.acc[u].add(0, P.ax[u]);
        T.acc[u].add(1, P.ay[u]);
        T.acc[u].add(2, P.az[u]);
        T.acc[u].add(3, P.ph[u]);
    }
}

// Runs the loop of a staged tile for the chunk's layout (nu, S).
template <int KIND, typename R, int IPL, typename TileT>
__device__ __forceinline__ void run_tile(const TileT &tile, int mpad, const Layout &ly,
                                         Targets<R, IPL> &T) {
    if constexpr (IPL > 2) {
        if (ly.nu > 2) {
            loop_kind<KIND, IPL, 1>(tile, mpad, ly.sl, T);
            return;
        }
    }
    if (ly.S > kSplitFixed) {
        if constexpr (IPL >= 2) {
            if (ly.nu == 2) {
                loop_kind_wide<KIND, 2>(tile, mpad, ly.sl, ly.S, T);
                return;
            }
        }
        loop_kind_wide<KIND, 1>(tile, mpad, ly.sl, ly.S, T);
        return;
    }
    if constexpr (IPL >= 2) {
        if (ly.nu == 2) {
            switch (ly.S) {
                case 1: loop_kind<KIND, 2, 1>(tile, mpad, ly.sl, T); break;
                case 2: loop_kind<KIND, 2, 2>(tile, mpad, ly.sl, T); break;
                case 3: loop_kind<KIND, 2, 3>(tile, mpad, ly.sl, T); break;
                case 4: loop_kind<KIND, 2, 4>(tile, mpad, ly.sl, T); break;
                case 5: loop_kind<KIND, 2, 5>(tile, mpad, ly.sl, T); break;
                case 6: loop_kind<KIND, 2, 6>(tile, mpad, ly.sl, T); break;
                case 7: loop_kind<KIND, 2, 7>(tile, mpad, ly.sl, T); break;
                default: loop_kind<KIND, 2, 8>(tile, mpad, ly.sl, T); break;
            }
            return;
        }
    }
    switch (ly.S) {
        case 1: loop_kind<KIND, 1, 1>(tile, mpad, ly.sl, T); break;
        case 2: loop_kind<KIND, 1, 2>(tile, mpad, ly.sl, T); break;
        case 3: loop_kind<KIND, 1, 3>(tile, mpad, ly.sl, T); break;
        case 4: loop_kind<KIND, 1, 4>(tile, mpad, ly.sl, T); break;
        case 5: loop_kind<KIND, 1, 5>(tile, mpad, ly.sl, T); break;
        case 6: loop_kind<KIND, 1, 6>(tile, mpad, ly.sl, T); break;
        case 7: loop_kind<KIND, 1, 7>(tile, mpad, ly.sl, T); break;
        default: loop_kind<KIND, 1, 8>(tile, mpad, ly.sl, T); break;
    }
}

// ---- multipole tile: entries [0, npc) were written by the walk; pads the
// tile to the loop's multiple and runs it.
template <typename R, int IPL>
__device__ void flush_pc(WaveLds<R> &L, int npc, const Layout &ly, Targets<R, IPL> &T) {
    const int mpad = pad_to(npc, kTilePc, ly.S);
    for (int t = npc + lane_id(); t < mpad; t += kWave) {
        L.pc.e[t].a = {(R)kFarAway, (R)kFarAway, (R)kFarAway, (R)0};
        L.pc.e[t].b = {(R)0, (R)0, (R)0, (R)0};
        L.pc.e[t].c = {(R)0, (R)0};
    }
    wave_sync();
    run_tile<kTilePc>(L.pc, mpad, ly, T);
    wave_sync();
}

// Multipole entry of cell data held in registers (relative to the group
// centre; traceless quadrupole A' = 3/2 S - 1/2 tr(S) I of the second
// moment S about the centre of mass). FP32: the doubled A' and M come
// rounded from the build (nd_q); FP64: from the second moments.
template <typename R>
struct CellQuad;
template <>
struct CellQuad<float> {
    float4 q0, q1;
    __device__ void load(const TreeDev &t, uint32_t nd) {
        q0 = t.nd_q[2 * (int64_t)nd];
        q1 = t.nd_q[2 * (int64_t)nd + 1];
    }
};
template <>
struct CellQuad<double> {
    double2 s01, s23, s45;
    __device__ void load(const TreeDev &t, uint32_t nd) {
        const double2 *Sp = reinterpret_cast<const double2 *>(t.nd_S) + (int64_t)nd * 3;
        s01 = Sp[0];
        s23 = Sp[1];
        s45 = Sp[2];
    }
};

__device__ __forceinline__ void stage_pc(WaveLds<float> &L, int p, const double4 &cm,
                                         const CellQuad<float> &q) {
    L.pc.e[p].a = {(float)(cm.x - L.g.c[0]), (float)(cm.y - L.g.c[1]),
                   (float)(cm.z - L.g.c[2]), q.q1.z};
    L.pc.e[p].b = q.q0;
    L.pc.e[p].c = {q.q1.x, q.q1.y};
}
__device__ __forceinline__ void stage_pc(WaveLds<double> &L, int p, const double4 &cm,
                                         const CellQuad<double> &q) {
    const double2 s01 = q.s01, s23 = q.s23, s45 = q.s45;
    const double tr = s01.x + s01.y + s23.x;
    L.pc.e[p].a = {cm.x - L.g.c[0], cm.y - L.g.c[1], cm.z - L.g.c[2], cm.w};
    L.pc.e[p].b = {2.0 * (1.5 * s01.x - 0.5 * tr), 2.0 * (1.5 * s01.y - 0.5 * tr),
                   2.0 * (1.5 * s23.x - 0.5 * tr), 2.0 * (1.5 * s23.y)};
    L.pc.e[p].c = {2.0 * (1.5 * s45.x), 2.0 * (1.5 * s45.y)};
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

// Source particle k (position p) into entry e of the particle tile.
template <int KIND, typename R>
__device__ __forceinline__ void stage_part(WaveLds<R> &L, int e, const double4 &p, uint32_t k,
                                           const ForceLaunch &f) {
    L.part.e[e].a = {(R)(p.x - L.g.c[0]), (R)(p.y - L.g.c[1]), (R)(p.z - L.g.c[2]), (R)p.w};
    if (KIND == kTileNear) {
        const double2 rr = f.t.rr[k];
        L.part.e[e].c = {(R)rr.x, (R)rr.y};
        L.part.e[e].k = k;
    }
}

// ---- leaves (far: Newtonian pairs; near: changeover pairs). On entry
// pre[] holds each buffered leaf's particle count; it is turned into an
// exclusive prefix and the particles are expanded in tiles of 64. Returns
// the number of source particles run. kSub: a force on a subset of targets
// (no neighbour lists), where particles of zero mass are dropped as sources
// (their terms are zero) and the rest packed to the front of the tile.
template <int KIND, bool kSub, typename R, int IPL>
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
    uint32_t total = last_lane(incl);
    if (lane < nleaf) pre[lane] = incl - c;
    wave_sync();
    uint32_t kept = 0;
    for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t s = base + lane;
        int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
        bool have = false;
        if (s < total) {
            const int l = find_leaf(pre, nleaf, s);
            const uint32_t k = start[l] + (s - pre[l]);
            const double4 p = f.t.ps[k];
            have = p.w != 0.0;
            stage_part<KIND>(L, lane, p, k, f);
        }
        if constexpr (kSub) {
            // move the entries with mass to the front of the tile
            const unsigned long long km = __ballot(have);
            if (km != (m == kWave ? ~0ull : (1ull << m) - 1ull)) {
                wave_sync();
                const typename Vec<R>::v4 a = L.part.e[lane].a;
                typename Vec<R>::v2 c = {(R)0, (R)0};
                uint32_t k = 0;
                if (KIND == kTileNear) {
                    c = L.part.e[lane].c;
                    k = L.part.e[lane].k;
                }
                wave_sync();
                if (have) {
                    const int e = lanes_below(km);
                    L.part.e[e].a = a;
                    if (KIND == kTileNear) {
                        L.part.e[e].c = c;
                        L.part.e[e].k = k;
                    }
                }
                m = __popcll(km);
            }
        }
        const int mpad = pad_to(m, KIND, ly.S);
        for (int t = m + lane; t < mpad; t += kWave) {
            L.part.e[t].a = {(R)kFarAway, (R)kFarAway, (R)kFarAway, (R)0};
            if (KIND == kTileNear) {
                L.part.e[t].c = {(R)0, (R)1};
                L.part.e[t].k = kNone - 1;
            }
        }
        wave_sync();
        run_tile<KIND>(L.part, mpad, ly, T);
        wave_sync();
        kept += (uint32_t)m;
    }
    return kept;
}

// Folds the partial sums of the S lanes that split one target's sources
// into the lane of split 0, in the fixed order of the splits (staged in the
// multipole tile, which is free once the walk of the chunk is done).
template <typename R>
__device__ __forceinline__ void fold_in(Acc<R> &a, const double *src, int k, int lane2) {
    a.s[k] += src[k * kWave + lane2];
}
template <typename R>
__device__ __forceinline__ void park(const Acc<R> &a, double *dst, int lane) {
    for (int k = 0; k < 4; k++) dst[k * kWave + lane] = a.s[k];
}

template <typename R, int IPL>
__device__ void combine_split(WaveLds<R> &L, Targets<R, IPL> &T, const Layout &ly) {
    static_assert(sizeof(PcTile<R>) >= 4 * kWave * sizeof(double), "fold buffer");
    double *buf = reinterpret_cast<double *>(&L.pc);
    const int lane = lane_id();
#pragma unroll
    for (int u = 0; u < IPL; u++) {
        if (u >= ly.nu) break;
        wave_sync();
        park(T.acc[u], buf, lane);
        wave_sync();
        if (ly.act && ly.sl == 0) {
            for (int s2 = 1; s2 < ly.S; s2++) {
                const int lane2 = s2 * ly.W + ly.il;
#pragma unroll
                for (int k = 0; k < 4; k++) fold_in(T.acc[u], buf, k, lane2);
            }
        }
    }
    wave_sync();
}

enum { kKindNone = 0, kKindPc = 1, kKindFar = 2, kKindNear = 3, kKindOpen = 4 };

// Long-range kick fused into the output write (eq. lfmap: v += a_L dt with
// dt the half step), v + a dt rounded twice as written.
__device__ __forceinline__ void kick_write(double *vel, int64_t n, uint32_t o, double ax,
                                           double ay, double az, double dt) {
#pragma clang fp contract(off)
    vel[o] = vel[o] + ax * dt;
    vel[n + o] = vel[n + o] + ay * dt;
    vel[2 * n + o] = vel[2 * n + o] + az * dt;
}

// kSub: the targets are the listed subset (tpos, tidx) and cells and
// particles of zero mass are no sources; otherwise every particle is a
// target.
template <typename R, int IPL, bool kSub>
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
    // theta^2 held in a vector register: as a scalar it shares a register
    // tuple with other kernel arguments, which the compiler spills and then
    // reloads whole at every walk step
    double th2 = f.th2;
    asm volatile("" : "+v"(th2));
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
        const uint32_t gstart = (uint32_t)uniform((int)ginfo.x);
        const uint32_t gn = (uint32_t)uniform((int)ginfo.y);
        // the group's targets: all its particles, or the listed subset
        uint32_t t0 = gstart, tn = gn;
        if constexpr (kSub) {
            t0 = (uint32_t)uniform((int)f.tpos[gstart]);
            tn = (uint32_t)uniform((int)f.tpos[gstart + gn]) - t0;
            if (tn == 0) continue;  // sources only: no walk
        }
        wave_sync();
        if (lane == 0) L.g = load_group(f.t.nd_lo, f.t.nd_hi, gnode);
        wave_sync();
        for (uint32_t chunk = 0; chunk < tn; chunk += CH) {
            const uint32_t active = tn - chunk < (uint32_t)CH ? tn - chunk : (uint32_t)CH;
            const Layout ly = choose_layout<IPL>(active);
            Targets<R, IPL> T;
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                uint32_t off = chunk + u * ly.W + ly.il;
                bool valid = ly.act && u < ly.nu && off < tn;
                uint32_t k = kSub ? f.tidx[t0 + (valid ? off : 0u)] : gstart + (valid ? off : 0u);
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
                const uint32_t node = stk.pop();
                // Lanes without a cell classify cell 0 (always present) and
                // are then marked idle: the wave issues these instructions
                // for all lanes anyway, and no default values are needed.
                const bool live = node != kNone;
                const uint32_t nd = live ? node : 0u;
                const double4 lo = f.t.nd_lo[nd], hi = f.t.nd_hi[nd];
                const double4 cm = f.t.nd_com[nd];
                CellQuad<R> quad;
                quad.load(f.t, nd);
                const uint4 info = f.t.nd_info[nd];
                double D2, R2;
                box_terms(L.g, lo, hi, &D2, &R2);
                const bool near = D2 < R2;
                const bool accept = mac_accept(L.g, cm, hi.w, th2) & !near;
                int kind = !live ? kKindNone
                                 : (accept ? kKindPc
                                           : ((info.z & kLeafFlag)
                                                  ? (near ? kKindNear : kKindFar)
                                                  : kKindOpen));
                // on a subset of targets (no neighbour lists), a cell of zero
                // mass is dropped with its subtree: it exerts no force
                if constexpr (kSub) {
                    if (cm.w == 0.0) kind = kKindNone;
                }
                int nc = kind == kKindOpen ? info_nchild(info.z) : 0;
                if (!stk.push(info.w, nc)) {
                    ok = false;
                    break;
                }
                unsigned long long m;
                int cnt;
                // Each buffer is filled to 64 entries before it is run: a
                // batch that does not fit completes it, the buffer is run,
                // and the rest of the batch (still in the lanes' registers)
                // starts the next one.
                m = __ballot(kind == kKindPc);
                cnt = __popcll(m);
                if (cnt) {
                    const int p = npc + lanes_below(m);
                    if (kind == kKindPc && p < kWave) stage_pc(L, p, cm, quad);
                    if (npc + cnt >= kWave) {
                        flush_pc(L, kWave, ly, T);
                        n_pc += kWave;
                        if (kind == kKindPc && p >= kWave) stage_pc(L, p - kWave, cm, quad);
                        npc += cnt - kWave;
                    } else {
                        npc += cnt;
                    }
                }
                m = __ballot(kind == kKindFar);
                cnt = __popcll(m);
                if (cnt) {
                    const int p = nfar + lanes_below(m);
                    if (kind == kKindFar && p < kWave) {
                        L.far_start[p] = info.x;
                        L.far_pre[p] = info.y;
                    }
                    if (nfar + cnt >= kWave) {
                        n_far += flush_leaves<kTileFar, kSub>(L, L.far_start, L.far_pre, kWave,
                                                              f, ly, T, false, gstart, gn);
                        if (kind == kKindFar && p >= kWave) {
                            L.far_start[p - kWave] = info.x;
                            L.far_pre[p - kWave] = info.y;
                        }
                        nfar += cnt - kWave;
                    } else {
                        nfar += cnt;
                    }
                }
                m = __ballot(kind == kKindNear);
                cnt = __popcll(m);
                if (cnt) {
                    const int p = nnear + lanes_below(m);
                    if (kind == kKindNear && p < kWave) {
                        L.near_start[p] = info.x;
                        L.near_pre[p] = info.y;
                    }
                    if (nnear + cnt >= kWave) {
                        n_near += flush_leaves<kTileNear, kSub>(L, L.near_start, L.near_pre,
                                                                kWave, f, ly, T, record, gstart,
                                                                gn);
                        if (kind == kKindNear && p >= kWave) {
                            L.near_start[p - kWave] = info.x;
                            L.near_pre[p - kWave] = info.y;
                        }
                        nnear += cnt - kWave;
                    } else {
                        nnear += cnt;
                    }
                }
            }
            if (!ok) {
                if (lane == 0) atomicAdd(&f.st->stack_overflow, 1);
                break;
            }
            if (npc) {
                wave_sync();
                flush_pc(L, npc, ly, T);
                n_pc += npc;
            }
            if (nfar)
                n_far += flush_leaves<kTileFar, kSub>(L, L.far_start, L.far_pre, nfar, f, ly, T,
                                                      false, gstart, gn);
            if (nnear)
                n_near += flush_leaves<kTileNear, kSub>(L, L.near_start, L.near_pre, nnear, f, ly,
                                                        T, record, gstart, gn);
            cnt_pc += n_pc * active;
            cnt_far += n_far * active;
            // minus the self pairs: every target's, or on a subset (massless
            // sources dropped) those of the targets with mass
            uint32_t n_self = active;
            if constexpr (kSub) {
                n_self = 0;
#pragma unroll
                for (int u = 0; u < IPL; u++) {
                    const bool own = T.k[u] != kNone && ly.sl == 0;
                    n_self += (uint32_t)__popcll(
                        __ballot(own && f.t.ps[own ? T.k[u] : 0u].w != 0.0));
                }
            }
            cnt_near += n_near * active - n_self;
            if (ly.S > 1) combine_split(L, T, ly);
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                if (T.k[u] == kNone || ly.sl != 0) continue;
                uint32_t o = f.t.orig[T.k[u]];
                const double ax = f.G * T.acc[u].get(0), ay = f.G * T.acc[u].get(1),
                             az = f.G * T.acc[u].get(2);
                f.acc[o] = ax;
                f.acc[n + o] = ay;
                f.acc[2 * n + o] = az;
                f.pot[o] = f.G * T.acc[u].get(3);
                if (f.kick_vel) kick_write(f.kick_vel, n, o, ax, ay, az, f.kick_dt);
                if (f.nb_bound) f.nb_bound[o] = (uint32_t)n_near;
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

__global__ __launch_bounds__(kThreads) void k_target_flags(const uint8_t *target,
                                                            const uint32_t *orig, int64_t n,
                                                            uint32_t *flag, double *acc,
                                                            double *pot) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t o = orig[k];
        const bool t = target[o] != 0;
        flag[k] = t ? 1u : 0u;
        if (!t) {
            acc[o] = 0.0;
            acc[n + o] = 0.0;
            acc[2 * n + o] = 0.0;
            pot[o] = 0.0;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_target_compact(const uint32_t *flag,
                                                              const uint32_t *tpos, int64_t n,
                                                              uint32_t *tidx) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        if (flag[k]) tidx[tpos[k]] = (uint32_t)k;
}

inline unsigned blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <typename R, int IPL>
int resident_for(int device) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force<R, IPL, false>, kThreads,
                                                     0) !=
        hipSuccess)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 256;  // MI355X
    if (per_cu < 1) per_cu = 1;
    return per_cu * cus * kWavesPerBlock;
}

template <typename R, int IPL>
void launch_t(const ForceLaunch &f, int resident_waves, hipStream_t s) {
    int blocks = resident_waves / kWavesPerBlock;
    if (f.tidx)
        hipLaunchKernelGGL((k_force<R, IPL, true>), dim3(blocks), dim3(kThreads), 0, s, f);
    else
        hipLaunchKernelGGL((k_force<R, IPL, false>), dim3(blocks), dim3(kThreads), 0, s, f);
}

}  // namespace

int64_t force_spill_elems_per_wave() { return kSpillCap; }

void launch_target_flags(const uint8_t *target, const TreeDev &t, uint32_t *flag, double *acc,
                         double *pot, hipStream_t s) {
    hipLaunchKernelGGL(k_target_flags, dim3(blocks_for(t.n)), dim3(kThreads), 0, s, target,
                       (const uint32_t *)t.orig, t.n, flag, acc, pot);
}

void launch_target_compact(const uint32_t *flag, const uint32_t *tpos, int64_t n, uint32_t *tidx,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_target_compact, dim3(blocks_for(n)), dim3(kThreads), 0, s, flag, tpos,
                       n, tidx);
}

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
