// Long-range force kernel: group-wise tree walk fused with the interaction
// passes, one wavefront per i-group, persistent over a device work queue.
//
// Per group the walk sorts every cell it reaches into
//   multipole (PC): the cell is inside the opening angle and no pair can be
//                   within search range -> monopole + quadrupole field;
//   far leaf:       opened leaf out of search range -> Newtonian pairs;
//   near leaf:      opened leaf within search range -> pairs weighted by
//                   the changeover functions (1 - K) and (1 - W)/r.
// Cells are buffered in LDS and, when a buffer holds a tile, staged as
// FP32 (or FP64) records relative to the group centre and broadcast to all
// lanes; each lane holds 1, 2 or 4 target particles. In mixed precision the
// per-tile FP32 partial sums are folded into Neumaier-compensated FP32
// accumulators and converted to FP64 at the end.
#include "launch.h"
#include "walk.h"

namespace petar {

namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

template <typename R>
struct PcRec {  // centre of mass (group-relative), mass, traceless quadrupole
    R x, y, z, m;
    R qxx, qyy, qzz, qxy;
    R qxz, qyz, pad0, pad1;
};
template <typename R>
struct JRec {
    R x, y, z, m;
};
template <typename R>
struct NRec {
    R x, y, z, m;
    R rin, rout;
    uint32_t k, pad;
};

template <typename R>
union Tile {
    PcRec<R> pc[kWave];
    JRec<R> j[kWave];
    NRec<R> nr[kWave];
};

template <typename R>
struct WaveLds {
    uint32_t stack[kStackLds];
    uint32_t pc_buf[kWave];
    uint32_t far_start[kWave], far_cnt[kWave], far_pre[kWave];
    uint32_t near_start[kWave], near_cnt[kWave], near_pre[kWave];
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
    uint32_t k[IPL];
    bool valid[IPL];
    Acc<R> acc[IPL];
};

template <typename R, int IPL>
__device__ __forceinline__ void fold(Targets<R, IPL> &T, const R (&ax)[IPL], const R (&ay)[IPL],
                                     const R (&az)[IPL], const R (&ph)[IPL]) {
#pragma unroll
    for (int u = 0; u < IPL; u++) {
        T.acc[u].add(0, ax[u]);
        T.acc[u].add(1, ay[u]);
        T.acc[u].add(2, az[u]);
        T.acc[u].add(3, ph[u]);
    }
}

// ---- multipole tile
template <typename R, int IPL>
__device__ void flush_pc(WaveLds<R> &L, int npc, const ForceLaunch &f, const GroupGeom &G,
                         Targets<R, IPL> &T, int S, int sl) {
    wave_sync();
    const int lane = lane_id();
    if (lane < npc) {
        uint32_t c = L.pc_buf[lane];
        double4 cm = f.t.nd_com[c];
        const double *S = f.t.nd_S + (int64_t)c * 6;
        double tr = S[0] + S[1] + S[2];
        PcRec<R> r;
        r.x = (R)(cm.x - G.c[0]);
        r.y = (R)(cm.y - G.c[1]);
        r.z = (R)(cm.z - G.c[2]);
        r.m = (R)cm.w;
        r.qxx = (R)(1.5 * S[0] - 0.5 * tr);
        r.qyy = (R)(1.5 * S[1] - 0.5 * tr);
        r.qzz = (R)(1.5 * S[2] - 0.5 * tr);
        r.qxy = (R)(1.5 * S[3]);
        r.qxz = (R)(1.5 * S[4]);
        r.qyz = (R)(1.5 * S[5]);
        r.pad0 = r.pad1 = (R)0;
        L.tile.pc[lane] = r;
    }
    wave_sync();
    R ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
    for (int u = 0; u < IPL; u++) ax[u] = ay[u] = az[u] = ph[u] = (R)0;
    for (int j = sl; j < npc; j += S) {
        const PcRec<R> c = L.tile.pc[j];
#pragma unroll
        for (int u = 0; u < IPL; u++) {
            R Rx = T.x[u] - c.x, Ry = T.y[u] - c.y, Rz = T.z[u] - c.z;
            R r2 = Rx * Rx + Ry * Ry + Rz * Rz;
            R ri = rsq(r2);
            R ri2 = ri * ri;
            R qx = c.qxx * Rx + c.qxy * Ry + c.qxz * Rz;
            R qy = c.qxy * Rx + c.qyy * Ry + c.qyz * Rz;
            R qz = c.qxz * Rx + c.qyz * Ry + c.qzz * Rz;
            R rqr = Rx * qx + Ry * qy + Rz * qz;
            R ri3 = ri * ri2;
            R ri5 = ri3 * ri2;
            R mri = c.m * ri;
            R coef = -(mri * ri2 + (R)5 * rqr * ri5 * ri2);
            R two5 = (R)2 * ri5;
            ax[u] += coef * Rx + two5 * qx;
            ay[u] += coef * Ry + two5 * qy;
            az[u] += coef * Rz + two5 * qz;
            ph[u] -= mri + rqr * ri5;
        }
    }
    fold(T, ax, ay, az, ph);
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

// ---- far leaves: Newtonian pairs
template <typename R, int IPL>
__device__ uint32_t flush_far(WaveLds<R> &L, int nleaf, const ForceLaunch &f, const GroupGeom &G,
                              Targets<R, IPL> &T, int S, int sl) {
    wave_sync();
    const int lane = lane_id();
    uint32_t c = lane < nleaf ? L.far_cnt[lane] : 0u;
    uint32_t incl = wave_incl_scan(c);
    uint32_t total = __shfl(incl, kWave - 1, kWave);
    if (lane < nleaf) L.far_pre[lane] = incl - c;
    wave_sync();
    for (uint32_t base = 0; base < total; base += kWave) {
        uint32_t s = base + lane;
        if (s < total) {
            int l = find_leaf(L.far_pre, nleaf, s);
            uint32_t k = L.far_start[l] + (s - L.far_pre[l]);
            double4 p = f.t.ps[k];
            JRec<R> r;
            r.x = (R)(p.x - G.c[0]);
            r.y = (R)(p.y - G.c[1]);
            r.z = (R)(p.z - G.c[2]);
            r.m = (R)p.w;
            L.tile.j[lane] = r;
        }
        wave_sync();
        int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
        R ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
        for (int u = 0; u < IPL; u++) ax[u] = ay[u] = az[u] = ph[u] = (R)0;
        for (int j = sl; j < m; j += S) {
            const JRec<R> p = L.tile.j[j];
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                R dx = p.x - T.x[u], dy = p.y - T.y[u], dz = p.z - T.z[u];
                R r2 = dx * dx + dy * dy + dz * dz;
                R ri = rsq(r2);
                R mri = p.m * ri;
                R mri3 = mri * ri * ri;
                ax[u] += mri3 * dx;
                ay[u] += mri3 * dy;
                az[u] += mri3 * dz;
                ph[u] -= mri;
            }
        }
        fold(T, ax, ay, az, ph);
        wave_sync();
    }
    return total;
}

// ---- near leaves: changeover-weighted pairs
template <typename R, int IPL>
__device__ uint32_t flush_near(WaveLds<R> &L, int nleaf, const ForceLaunch &f, const GroupGeom &G,
                               Targets<R, IPL> &T, int S, int sl) {
    wave_sync();
    const int lane = lane_id();
    uint32_t c = lane < nleaf ? L.near_cnt[lane] : 0u;
    uint32_t incl = wave_incl_scan(c);
    uint32_t total = __shfl(incl, kWave - 1, kWave);
    if (lane < nleaf) L.near_pre[lane] = incl - c;
    wave_sync();
    for (uint32_t base = 0; base < total; base += kWave) {
        uint32_t s = base + lane;
        if (s < total) {
            int l = find_leaf(L.near_pre, nleaf, s);
            uint32_t k = L.near_start[l] + (s - L.near_pre[l]);
            double4 p = f.t.ps[k];
            double2 rr = f.t.rr[k];
            NRec<R> r;
            r.x = (R)(p.x - G.c[0]);
            r.y = (R)(p.y - G.c[1]);
            r.z = (R)(p.z - G.c[2]);
            r.m = (R)p.w;
            r.rin = (R)rr.x;
            r.rout = (R)rr.y;
            r.k = k;
            r.pad = 0;
            L.tile.nr[lane] = r;
        }
        wave_sync();
        int m = (int)(total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave);
        R ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
        for (int u = 0; u < IPL; u++) ax[u] = ay[u] = az[u] = ph[u] = (R)0;
        for (int j = sl; j < m; j += S) {
            const NRec<R> p = L.tile.nr[j];
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                R dx = p.x - T.x[u], dy = p.y - T.y[u], dz = p.z - T.z[u];
                R r2 = dx * dx + dy * dy + dz * dz;
                R rin = T.rin[u] > p.rin ? T.rin[u] : p.rin;
                R rout = T.rout[u] > p.rout ? T.rout[u] : p.rout;
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
                bool self = p.k == T.k[u];
                fw = self ? (R)0 : fw;
                pw = self ? (R)0 : pw;
                R mf = p.m * fw * ri * ri * ri;
                ax[u] += mf * dx;
                ay[u] += mf * dy;
                az[u] += mf * dz;
                ph[u] -= p.m * pw;
            }
        }
        fold(T, ax, ay, az, ph);
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
    if (f.st_in->invalid_radii) return;
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
        const uint32_t gnode = f.groups[g];
        const uint4 ginfo = f.t.nd_info[gnode];
        const GroupGeom G = load_group(f.t.nd_lo, f.t.nd_hi, gnode);
        const uint32_t gstart = ginfo.x, gn = ginfo.y;
        for (uint32_t chunk = 0; chunk < gn; chunk += CH) {
            const uint32_t active = gn - chunk < (uint32_t)CH ? gn - chunk : (uint32_t)CH;
            // Small groups with one target per lane: S lanes share a target and
            // split the j loop (lane = sl * W + il).
            int S = 1;
            if (IPL == 1) S = active <= 8 ? 8 : (active <= 16 ? 4 : (active <= 32 ? 2 : 1));
            const int W = kWave / S;
            const int il = lane & (W - 1), sl = lane / W;
            Targets<R, IPL> T;
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                uint32_t off = chunk + u * kWave + il;
                T.valid[u] = off < gn;
                uint32_t k = gstart + (T.valid[u] ? off : 0u);
                double4 p = f.t.ps[k];
                double2 rr = f.t.rr[k];
                T.x[u] = (R)(p.x - G.c[0]);
                T.y[u] = (R)(p.y - G.c[1]);
                T.z[u] = (R)(p.z - G.c[2]);
                T.rin[u] = (R)rr.x;
                T.rout[u] = (R)rr.y;
                T.k[u] = T.valid[u] ? k : kNone;
                T.acc[u].zero();
            }
            uint64_t n_pc = 0, n_far = 0, n_near = 0;
            int npc = 0, nfar = 0, nnear = 0;
            stk.init(0u);
            bool ok = true;
            while (!stk.empty()) {
                uint32_t node = stk.pop();
                int kind = kKindNone;
                uint4 info = make_uint4(0, 0, 0, 0);
                if (node != kNone) {
                    double4 lo = f.t.nd_lo[node], hi = f.t.nd_hi[node], cm = f.t.nd_com[node];
                    info = f.t.nd_info[node];
                    double D2, R2;
                    box_terms(G, lo, hi, &D2, &R2);
                    bool near = D2 < R2;
                    if (!near && mac_accept(G, cm, hi.w, f.th2))
                        kind = kKindPc;
                    else if (info.z & kLeafFlag)
                        kind = near ? kKindNear : kKindFar;
                    else
                        kind = kKindOpen;
                }
                uint32_t ch[8];
                int nc = 0;
                if (kind == kKindOpen)
                    nc = load_children(f.t.nd_child, node, ch);
                else
                    no_children(ch);
                if (!stk.push(ch, nc)) {
                    ok = false;
                    break;
                }
                unsigned long long m;
                int cnt;
                m = __ballot(kind == kKindPc);
                cnt = __popcll(m);
                if (cnt) {
                    if (npc + cnt > kWave) {
                        flush_pc(L, npc, f, G, T, S, sl);
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
                        n_far += flush_far(L, nfar, f, G, T, S, sl);
                        nfar = 0;
                    }
                    if (kind == kKindFar) {
                        int p = nfar + lanes_below(m);
                        L.far_start[p] = info.x;
                        L.far_cnt[p] = info.y;
                    }
                    nfar += cnt;
                }
                m = __ballot(kind == kKindNear);
                cnt = __popcll(m);
                if (cnt) {
                    if (nnear + cnt > kWave) {
                        n_near += flush_near(L, nnear, f, G, T, S, sl);
                        nnear = 0;
                    }
                    if (kind == kKindNear) {
                        int p = nnear + lanes_below(m);
                        L.near_start[p] = info.x;
                        L.near_cnt[p] = info.y;
                    }
                    nnear += cnt;
                }
            }
            if (!ok) {
                if (lane == 0) atomicAdd(&f.st->stack_overflow, 1);
                break;
            }
            if (npc) {
                flush_pc(L, npc, f, G, T, S, sl);
                n_pc += npc;
            }
            if (nfar) n_far += flush_far(L, nfar, f, G, T, S, sl);
            if (nnear) n_near += flush_near(L, nnear, f, G, T, S, sl);
            cnt_pc += n_pc * active;
            cnt_far += n_far * active;
            cnt_near += n_near * active - active;  // minus the self pairs
            if (S > 1) combine_split(T.acc[0], W);
#pragma unroll
            for (int u = 0; u < IPL; u++) {
                if (!T.valid[u] || sl != 0) continue;
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
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_force<R, IPL>, kThreads, 0);
    hipDeviceProp_t p;
    hipGetDeviceProperties(&p, device);
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
