// Artificial particles of the long-range step (Sec. "Artificial particle
// algorithm for weak perturbation"): for every bound pair (a binary treated
// as a group by the short-range integrator) the set of the long-range force
// replaces the two members by
//   * the centre of mass and P tidal-tensor measure points, zero mass, at
//     r_cm + d_c u_p with the unit offsets of Table A (P = 4, a regular
//     tetrahedron, for the second-order tensor; P = 8 for the third order);
//   * three pseudoparticles of mass (m1 + m2)/3 at the positions of eq. psep,
//     which carry the pair's mass, centre of mass and orbit-averaged
//     quadrupole (eq. avebinquad) to every other particle.
// After the long-range force on that set, the post-fit turns the field at
// the centre and at the measure points into the tensor coefficients of
// eq. tt through the generalized inverse of the linear map eq. map, and
// evaluates the fitted field (and its potential) at the members.
//
// Every stage is an FP64 kernel with one thread per pair or particle: the
// work is a few hundred flops per pair and bound by memory, far below the
// cost of the force on the set that sits between make and fit. The pair
// blocks are written, and the measure-point accelerations read, through
// LDS so that consecutive lanes touch consecutive addresses.
#include <cmath>
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

// Unit offsets of the measure points (Table A, coordinates relative to the
// centre of mass in units of d_c, the half edge of the tetrahedron or cube).
__host__ __device__ inline void tt_unit(int order, int p, double u[3]) {
    const double h = 0.70710678118654752440;  // sqrt(2)/2
    if (order == 2) {
        u[0] = p == 0 ? 1.0 : (p == 1 ? -1.0 : 0.0);
        u[1] = p == 2 ? 1.0 : (p == 3 ? -1.0 : 0.0);
        u[2] = p < 2 ? -h : h;
    } else {
        // four points at z = -1, then the same four at z = +1, going round
        // +x, +y, -x, -y
        const int q = p & 3;
        u[0] = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
        u[1] = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
        u[2] = p < 4 ? -1.0 : 1.0;
    }
}

// Field of the tensor part of the model at offset (x, y, z), split into its
// first-order part a1 (T = [xx xy xz yy yz zz]) and, for order 3, its
// second-order part a2 (T[6..15] = [xxx xxy xxz xyy xyz xzz yyy yyz yzz
// zzz]); these are the evaluation rows of Table A without A(r_cm).
__host__ __device__ inline void tt_field(int order, const double *T, double x, double y, double z,
                                         double a1[3], double a2[3]) {
    a1[0] = T[0] * x + T[1] * y + T[2] * z;
    a1[1] = T[1] * x + T[3] * y + T[4] * z;
    a1[2] = T[2] * x + T[4] * y + T[5] * z;
    a2[0] = a2[1] = a2[2] = 0.0;
    if (order == 3) {
        const double xx = x * x, yy = y * y, zz = z * z;
        const double xy2 = 2.0 * x * y, xz2 = 2.0 * x * z, yz2 = 2.0 * y * z;
        const double *U = T + 6;
        a2[0] = U[0] * xx + U[1] * xy2 + U[2] * xz2 + U[3] * yy + U[4] * yz2 + U[5] * zz;
        a2[1] = U[1] * xx + U[3] * xy2 + U[4] * xz2 + U[6] * yy + U[7] * yz2 + U[8] * zz;
        a2[2] = U[2] * xx + U[4] * xy2 + U[5] * xz2 + U[7] * yy + U[8] * yz2 + U[9] * zz;
    }
}

inline int tt_points(int order) { return order == 2 ? 4 : 8; }
inline int tt_unknowns(int order) { return order == 2 ? 6 : 16; }

// Least-squares inverse of the map from the tensor coefficients to the
// field at the measure points (d_c = 1): Householder QR of the 3P x K
// design matrix, G = R^-1 Q^T. Row-major K x 3P.
void ginv_by_qr(int order, double *g) {
    const int P = tt_points(order), K = tt_unknowns(order), m = 3 * P;
    double A[24][16], Qt[24][24];
    for (int k = 0; k < K; k++) {
        double T[16] = {0};
        T[k] = 1.0;
        for (int p = 0; p < P; p++) {
            double u[3], a1[3], a2[3];
            tt_unit(order, p, u);
            tt_field(order, T, u[0], u[1], u[2], a1, a2);
            for (int d = 0; d < 3; d++) A[3 * p + d][k] = a1[d] + a2[d];
        }
    }
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) Qt[r][c] = r == c ? 1.0 : 0.0;
    for (int j = 0; j < K; j++) {
        double v[24], nrm = 0.0;
        for (int r = j; r < m; r++) {
            v[r] = A[r][j];
            nrm += v[r] * v[r];
        }
        nrm = std::sqrt(nrm);
        const double alpha = v[j] > 0.0 ? -nrm : nrm;
        v[j] -= alpha;
        double vv = 0.0;
        for (int r = j; r < m; r++) vv += v[r] * v[r];
        if (vv == 0.0) continue;
        for (int c = j; c < K; c++) {
            double s = 0.0;
            for (int r = j; r < m; r++) s += v[r] * A[r][c];
            s = 2.0 * s / vv;
            for (int r = j; r < m; r++) A[r][c] -= s * v[r];
        }
        for (int c = 0; c < m; c++) {
            double s = 0.0;
            for (int r = j; r < m; r++) s += v[r] * Qt[r][c];
            s = 2.0 * s / vv;
            for (int r = j; r < m; r++) Qt[r][c] -= s * v[r];
        }
    }
    // back substitution R G = (Q^T)[0:K, :]
    for (int c = 0; c < m; c++)
        for (int k = K - 1; k >= 0; k--) {
            double s = Qt[k][c];
            for (int l = k + 1; l < K; l++) s -= A[k][l] * g[l * m + c];
            g[k * m + c] = s / A[k][k];
        }
}

struct Kepler {
    double a, e;        // semi-major axis, eccentricity (length of the eccentricity vector)
    double s;           // a sqrt(m1 m2) / (m1 + m2), the scale of eq. psep
    double ex[3], ey[3];  // orbital frame: pericentre direction, in-plane normal
    double px[3], py[3];  // eq. psep offsets in that frame
    bool ok;
};

// Orbit of a pair from its relative state (eq. dr, eq. r1r2): bound iff the
// specific energy is negative; e is the length of the eccentricity vector
// v x h / mu - r/|r| (well conditioned for nearly circular orbits). The
// frame's x axis points to the pericentre (the eccentricity vector; the
// separation for a circular orbit, e below 1e-12), z along the angular
// momentum; a radial orbit is the limit e = 1 along the separation.
__device__ Kepler kepler(double m1, double m2, const double r[3], const double v[3], double G) {
    Kepler k;
    const double M = m1 + m2, mu = G * M;
    double rr;
    const double E = kepler_energy(r, v, mu, &rr);
    k.ok = rr > 0.0 && E < 0.0;
    if (!k.ok) return k;
    k.a = -mu / (2.0 * E);
    const double h[3] = {r[1] * v[2] - r[2] * v[1], r[2] * v[0] - r[0] * v[2],
                         r[0] * v[1] - r[1] * v[0]};
    const double h2 = h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
    k.s = k.a * sqrt(m1 * m2) / M;
    const double hn = sqrt(h2);
    double ep;  // eccentricity used for the point offsets
    if (hn > 0.0) {
        const double z[3] = {h[0] / hn, h[1] / hn, h[2] / hn};
        const double ev[3] = {(v[1] * h[2] - v[2] * h[1]) / mu - r[0] / rr,
                              (v[2] * h[0] - v[0] * h[2]) / mu - r[1] / rr,
                              (v[0] * h[1] - v[1] * h[0]) / mu - r[2] / rr};
        ep = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        k.e = ep;
        if (ep > 1e-12) {
            for (int d = 0; d < 3; d++) k.ex[d] = ev[d] / ep;
        } else {
            for (int d = 0; d < 3; d++) k.ex[d] = r[d] / rr;
            ep = 0.0;
        }
        k.ey[0] = z[1] * k.ex[2] - z[2] * k.ex[1];
        k.ey[1] = z[2] * k.ex[0] - z[0] * k.ex[2];
        k.ey[2] = z[0] * k.ex[1] - z[1] * k.ex[0];
    } else {
        ep = k.e = 1.0;
        for (int d = 0; d < 3; d++) {
            k.ex[d] = r[d] / rr;
            k.ey[d] = 0.0;
        }
    }
    const double b = sqrt(3.0 * ep * ep + 0.75), c = sqrt(1.0 - ep * ep);
    k.px[0] = 0.0;
    k.py[0] = c;
    k.px[1] = b;
    k.py[1] = -0.5 * c;
    k.px[2] = -b;
    k.py[2] = -0.5 * c;
    return k;
}

__global__ __launch_bounds__(kThreads) void k_art_mark(ArtArgs a, int32_t *bad) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < a.n_pair;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = a.pairs[b], j = a.pairs[a.n_pair + b];
        if (i < 0 || j < 0 || i >= a.n || j >= a.n || i == j) {
            atomicAdd(&bad[0], 1);
            continue;
        }
        if (atomicCAS(&a.pair_of[i], -1, (int32_t)b) != -1) atomicAdd(&bad[1], 1);
        if (atomicCAS(&a.pair_of[j], -1, (int32_t)b) != -1) atomicAdd(&bad[1], 1);
    }
}

__global__ __launch_bounds__(kThreads) void k_art_flags(ArtArgs a, uint32_t *single) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x)
        single[i] = a.pair_of[i] < 0 ? 1u : 0u;
}

// Singles keep their input order at the front of the set. spos is the
// exclusive scan of the single flags (< n <= n_out whatever the pairs).
__global__ __launch_bounds__(kThreads) void k_art_singles(ArtArgs a, const uint32_t *spos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (a.pair_of[i] >= 0) continue;
        const int64_t k = spos[i];
        for (int d = 0; d < 3; d++) a.o_pos[d * a.n_out + k] = a.pos[d * a.n + i];
        a.o_mass[k] = a.mass[i];
        a.o_rin[k] = a.r_in[i];
        a.o_rout[k] = a.r_out[i];
        a.o_rs[k] = a.r_search[i];
        a.src[k] = (int32_t)i;
        if (a.o_target) a.o_target[k] = 1;
    }
}

// One block of P + 4 particles per pair: centre, measure points,
// pseudoparticles. A workgroup takes 256 consecutive pairs: each thread
// computes its pair's orbit and offsets into LDS, then the workgroup writes
// the 256 (P + 4) consecutive entries of every output array with
// consecutive threads on consecutive addresses. Indices were checked by
// k_art_mark; they are checked again so that no access leaves the arrays.
constexpr int kPairsPerBlock = 256;

struct PairLds {
    double cm[3][kPairsPerBlock];
    double dc[kPairsPerBlock];
    double off[3][3][kPairsPerBlock];  // pseudoparticle t, axis d
    double m3[kPairsPerBlock];
    double rin[kPairsPerBlock], rout[kPairsPerBlock], rs[kPairsPerBlock];
    uint8_t ok[kPairsPerBlock];
};

__global__ __launch_bounds__(kPairsPerBlock) void k_art_pairs(ArtArgs a, int32_t *bad) {
    __shared__ PairLds L;
    const int P = a.order == 2 ? 4 : 8, B = P + 4;
    const int64_t b0 = (int64_t)blockIdx.x * kPairsPerBlock;
    const int t = threadIdx.x;
    const int cnt = (int)(a.n_pair - b0 < kPairsPerBlock ? a.n_pair - b0 : kPairsPerBlock);
    if (t < cnt) {
        const int64_t b = b0 + t;
        const int32_t i = a.pairs[b], j = a.pairs[a.n_pair + b];
        uint8_t ok = 0;
        if (i >= 0 && j >= 0 && i < a.n && j < a.n && i != j) {
            const double m1 = a.mass[i], m2 = a.mass[j], M = m1 + m2;
            double x1[3], x2[3], r[3], v[3], cm[3];
            for (int d = 0; d < 3; d++) {
                x1[d] = a.pos[d * a.n + i];
                x2[d] = a.pos[d * a.n + j];
                r[d] = x2[d] - x1[d];
                v[d] = a.vel[d * a.n + j] - a.vel[d * a.n + i];
                cm[d] = (m1 * x1[d] + m2 * x2[d]) / M;
            }
            const Kepler k = kepler(m1, m2, r, v, a.G);
            if (!k.ok || !(M > 0.0)) {
                atomicAdd(&bad[2], 1);
            } else {
                ok = 1;
                const double d_c = a.c_d * k.a * (1.0 + k.e);
                for (int d = 0; d < 3; d++) {
                    L.cm[d][t] = cm[d];
                    for (int q = 0; q < 3; q++)
                        L.off[q][d][t] = k.s * (k.px[q] * k.ex[d] + k.py[q] * k.ey[d]);
                    a.frame[d * a.n_pair + b] = cm[d];
                }
                L.dc[t] = d_c;
                L.m3[t] = M / 3.0;
                L.rin[t] = fmax(a.r_in[i], a.r_in[j]);
                L.rout[t] = fmax(a.r_out[i], a.r_out[j]);
                L.rs[t] = fmax(a.r_search[i], a.r_search[j]);
                a.frame[3 * a.n_pair + b] = d_c;
            }
        }
        L.ok[t] = ok;
    }
    __syncthreads();
    const int64_t base0 = a.n_single + b0 * B;
    for (int e = t; e < cnt * B; e += kPairsPerBlock) {
        const int pr = e / B, q = e - pr * B;
        if (!L.ok[pr]) continue;
        double p[3], m = 0.0;
        if (q == 0) {
            for (int d = 0; d < 3; d++) p[d] = L.cm[d][pr];
        } else if (q <= P) {
            double u[3];
            tt_unit(a.order, q - 1, u);
            for (int d = 0; d < 3; d++) p[d] = L.cm[d][pr] + L.dc[pr] * u[d];
        } else {
            for (int d = 0; d < 3; d++) p[d] = L.cm[d][pr] + L.off[q - 1 - P][d][pr];
            m = L.m3[pr];
        }
        const int64_t o = base0 + e;
        for (int d = 0; d < 3; d++) a.o_pos[d * a.n_out + o] = p[d];
        a.o_mass[o] = m;
        a.o_rin[o] = L.rin[pr];
        a.o_rout[o] = L.rout[pr];
        a.o_rs[o] = L.rs[pr];
        a.src[o] = -1;
        if (a.o_target) a.o_target[o] = q <= P ? 1 : 0;  // pseudoparticles are sources only
    }
}

// Potential of the model: phi_cm - r'.(A(r_cm) + a1/2 + a2/3), whose minus
// gradient is A(r_cm) + a1 + a2 (T_ij and T_ijk symmetric).
__device__ inline void tt_eval(int order, const double *rec, double x, double y, double z,
                               double acc[3], double *pot) {
    double a1[3], a2[3];
    tt_field(order, rec + 4, x, y, z, a1, a2);
    const double r[3] = {x, y, z};
    double ph = rec[0];
    for (int d = 0; d < 3; d++) {
        acc[d] = rec[1 + d] + a1[d] + a2[d];
        ph -= r[d] * (rec[1 + d] + 0.5 * a1[d] + a2[d] / 3.0);
    }
    *pot = ph;
}

// A workgroup takes 128 consecutive pairs and first copies the
// accelerations of their centres and measure points (the first P + 1 entries
// of each block) into LDS, consecutive threads on consecutive addresses;
// each thread then fits its own pair from LDS.
constexpr int kFitPairs = 128;

template <int ORDER>
__global__ __launch_bounds__(kFitPairs) void k_tidal_fit(FitArgs f) {
    constexpr int P = ORDER == 2 ? 4 : 8, K = ORDER == 2 ? 6 : 16, R = 4 + K, B = P + 4;
    __shared__ double sa[3][kFitPairs * (P + 1)];
    const int64_t b0 = (int64_t)blockIdx.x * kFitPairs;
    const int t = threadIdx.x;
    const int cnt = (int)(f.n_pair - b0 < kFitPairs ? f.n_pair - b0 : kFitPairs);
    const int64_t base0 = f.n_single + b0 * B;
    for (int e = t; e < cnt * (P + 1); e += kFitPairs) {
        const int pr = e / (P + 1), q = e - pr * (P + 1);
        for (int d = 0; d < 3; d++) sa[d][e] = f.acc_set[d * f.n_out + base0 + pr * B + q];
    }
    __syncthreads();
    if (t >= cnt) return;
    const int64_t b = b0 + t;
    const int64_t base = base0 + (int64_t)t * B;
    double A0[3], Ap[3 * P];
    for (int d = 0; d < 3; d++) A0[d] = sa[d][t * (P + 1)];
#pragma unroll
    for (int p = 0; p < P; p++)
        for (int d = 0; d < 3; d++) Ap[3 * p + d] = sa[d][t * (P + 1) + 1 + p] - A0[d];
    const double d_c = f.frame[3 * f.n_pair + b];
    double rec[R];
    rec[0] = f.pot_set ? f.pot_set[base] : 0.0;
    for (int d = 0; d < 3; d++) rec[1 + d] = A0[d];
#pragma unroll
    for (int k = 0; k < K; k++) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 3 * P; r++) s += f.ginv[k * 3 * P + r] * Ap[r];
        rec[4 + k] = k < 6 ? s / d_c : s / (d_c * d_c);
    }
#pragma unroll
    for (int k = 0; k < R; k++) f.tensor[k * f.n_pair + b] = rec[k];
    if (!f.acc) return;
    const int32_t mem[2] = {f.pairs[b], f.pairs[f.n_pair + b]};
    for (int q = 0; q < 2; q++) {
        const int64_t i = mem[q];
        if (i < 0 || i >= f.n) continue;
        double acc[3], pot;
        tt_eval(ORDER, rec, f.pos[i] - f.frame[b], f.pos[f.n + i] - f.frame[f.n_pair + b],
                f.pos[2 * f.n + i] - f.frame[2 * f.n_pair + b], acc, &pot);
        for (int d = 0; d < 3; d++) f.acc[d * f.n + i] = acc[d];
        if (f.pot) f.pot[i] = pot;
    }
}

__global__ __launch_bounds__(kThreads) void k_art_scatter(FitArgs f) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < f.n_single;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = f.src[k];
        if (i < 0 || i >= f.n) continue;
        for (int d = 0; d < 3; d++) f.acc[d * f.n + i] = f.acc_set[d * f.n_out + k];
        if (f.pot) f.pot[i] = f.pot_set[k];
    }
}

template <int ORDER>
__global__ __launch_bounds__(kThreads) void k_tidal_eval(EvalArgs e) {
    constexpr int R = ORDER == 2 ? 10 : 20;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e.n_pt;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e.pair_of[i];
        if (b < 0) continue;
        if (b >= e.n_pair) {
            atomicAdd(e.bad, 1);
            continue;
        }
        double rec[R];
#pragma unroll
        for (int k = 0; k < R; k++) rec[k] = e.tensor[k * e.n_pair + b];
        double acc[3], pot;
        tt_eval(ORDER, rec, e.pos[i] - e.frame[b], e.pos[e.n_pt + i] - e.frame[e.n_pair + b],
                e.pos[2 * e.n_pt + i] - e.frame[2 * e.n_pair + b], acc, &pot);
        for (int d = 0; d < 3; d++) e.acc[d * e.n_pt + i] = acc[d];
        if (e.pot) e.pot[i] = pot;
    }
}

__global__ __launch_bounds__(kThreads) void k_kick(double *vel, const double *acc, int64_t n3,
                                                   double dt) {
#pragma clang fp contract(off)
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n3;
         k += (int64_t)gridDim.x * blockDim.x)
        vel[k] = vel[k] + acc[k] * dt;
}

}  // namespace

void launch_kick(double *vel, const double *acc, int64_t n, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_kick, dim3(grid_for(3 * n, kThreads, 16384)), dim3(kThreads), 0, s, vel,
                       acc, 3 * n, dt);
}

const double *tidal_ginv_host(int order) {
    static double g2[6 * 12], g3[16 * 24];
    static std::once_flag once;
    std::call_once(once, [] {
        ginv_by_qr(2, g2);
        ginv_by_qr(3, g3);
    });
    return order == 2 ? g2 : g3;
}

void launch_art_make(const ArtArgs &a, uint32_t *single, uint32_t *spos, int64_t *scan_ws,
                     int32_t *bad, hipStream_t s) {
    const dim3 b(kThreads);
    const dim3 gp(grid_for(a.n_pair, kThreads, 8192)), gn(grid_for(a.n, kThreads, 8192));
    fill_u32(reinterpret_cast<uint32_t *>(a.pair_of), 0xffffffffu, a.n, s);
    if (a.n_pair > 0) hipLaunchKernelGGL(k_art_mark, gp, b, 0, s, a, bad);
    hipLaunchKernelGGL(k_art_flags, gn, b, 0, s, a, single);
    scan_u32_to_u32(single, spos, a.n, scan_ws, s);
    hipLaunchKernelGGL(k_art_singles, gn, b, 0, s, a, (const uint32_t *)spos);
    if (a.n_pair > 0)
        hipLaunchKernelGGL(k_art_pairs, dim3((unsigned)((a.n_pair + kPairsPerBlock - 1) /
                                                        kPairsPerBlock)),
                           dim3(kPairsPerBlock), 0, s, a, bad);
}

void launch_tidal_fit(const FitArgs &f, hipStream_t s) {
    const dim3 b(kThreads);
    if (f.n_pair > 0) {
        const dim3 g((unsigned)((f.n_pair + kFitPairs - 1) / kFitPairs)), bf(kFitPairs);
        if (f.order == 2)
            hipLaunchKernelGGL(k_tidal_fit<2>, g, bf, 0, s, f);
        else
            hipLaunchKernelGGL(k_tidal_fit<3>, g, bf, 0, s, f);
    }
    if (f.acc && f.n_single > 0)
        hipLaunchKernelGGL(k_art_scatter, dim3(grid_for(f.n_single, kThreads, 8192)), b, 0, s, f);
}

void launch_tidal_eval(const EvalArgs &e, hipStream_t s) {
    if (e.n_pt <= 0) return;
    const dim3 g(grid_for(e.n_pt, kThreads, 8192)), b(kThreads);
    if (e.order == 2)
        hipLaunchKernelGGL(k_tidal_eval<2>, g, b, 0, s, e);
    else
        hipLaunchKernelGGL(k_tidal_eval<3>, g, b, 0, s, e);
}

}  // namespace petar
