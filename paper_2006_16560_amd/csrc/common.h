// Internal definitions shared by the HIP translation units of libpetar.
// Device data layout (all in HBM, library-owned unless noted):
//   particles in Morton order:  ps[k]   = (x, y, z, m)      double4
//                               rr[k]   = (r_in, r_out)     double2
//                               rsk[k]  = r_search          double
//                               orig[k] = input index       uint32
//   octree cells in level order (root first; inside a level in Morton
//   order, so the children of a cell are contiguous):
//                               nd_lo[c]  = (lo.x, lo.y, lo.z, max r_search)
//                               nd_hi[c]  = (hi.x, hi.y, hi.z, side)
//                               nd_com[c] = (com.x, com.y, com.z, M)
//                               nd_S[c*6 + 0..5] = second moment about com
//                                        (xx, yy, zz, xy, xz, yz)
//                               nd_q[2c], nd_q[2c+1] = FP32 multipole record:
//                                        (2A'xx, 2A'yy, 2A'zz, 2A'xy),
//                                        (2A'xz, 2A'yz, M, 0)
//                               nd_info[c] = (first particle, count, flags, first child)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace petar {

constexpr int kMaxLevel = 21;           // 21 bits per axis, 63-bit keys (one system)
constexpr int kBatchLevels = 18;        // per-system depth in batched mode
constexpr int kMaxSystems = 512;        // batched mode: system id above 54 key bits
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kWave = 64;
// nd_info.z: bit 0 leaf, bits 1..5 level, bits 8..11 number of children.
constexpr uint32_t kLeafFlag = 1u;
__host__ __device__ __forceinline__ int info_level(uint32_t z) { return (int)((z >> 1) & 31u); }
__host__ __device__ __forceinline__ int info_nchild(uint32_t z) { return (int)((z >> 8) & 15u); }

// Root cube of the particle set (device-resident, written by the bbox pass).
struct RootBox {
    double lo[3];
    double ext;      // side of the root cube
    double scale;    // 2^21 / ext
    int32_t bad;     // count of non-finite coordinates / masses or negative masses
    int32_t pad;
};

// Status words read back once per call. The force fields come first so a
// force call can clear them without touching the build fields.
struct Status {
    // force
    int32_t invalid_radii;   // non-finite or out-of-order radii
    int32_t stack_overflow;  // walk stack exceeded its capacity
    unsigned long long inter[3];  // pc, far, near interactions
    int64_t n_groups;
    int64_t nb_total;        // neighbour-list entries
    uint32_t rec_used[2];    // near-leaf hand-over claimed: headers, leaf entries
    int64_t nb_rows;         // scratch entries the neighbour rows need
    // build
    int32_t cell_overflow;   // more cells than the preallocated capacity (captured graphs)
    int32_t pad;
    int64_t n_nodes;
    int64_t n_leaves;
    int64_t max_level;
    int64_t cells;           // cells counted by the first half of an eager build
    int32_t bad_input;       // non-finite or negative input (the root box's count)
    uint32_t deep;           // deepest cell level
};
constexpr int kStatusForceWords = 8;  // int64 words of the force fields

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int lanes_below(unsigned long long mask) {
    return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

// Inclusive prefix sum across the 64 lanes of a wave (all lanes active).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (lane_id() >= d) v += u;
    }
    return v;
}

// 32-bit version on DPP lane moves (no LDS round trips): shifts by 1, 2, 4
// and 8 lanes within each row of 16 give the row prefixes; the last lane of
// row 0 (and of row 2) is then broadcast into row 1 (row 3), and the last
// lane of row 1 into rows 2 and 3. Lanes without a source add 0.
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}
template <>
__device__ __forceinline__ int wave_incl_scan<int>(int v) {
    return wave_incl_scan_dpp(v);
}
template <>
__device__ __forceinline__ uint32_t wave_incl_scan<uint32_t>(uint32_t v) {
    return (uint32_t)wave_incl_scan_dpp((int)v);
}

// Value of the last lane (e.g. the total of an inclusive scan), wave-uniform.
__device__ __forceinline__ uint32_t last_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
__device__ __forceinline__ int last_lane(int v) { return __builtin_amdgcn_readlane(v, kWave - 1); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, kWave));
    return v;
}

// Orders LDS (and global) accesses of one wave: the data written by some
// lanes is visible to the others after this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---- Morton keys. With L levels the octal digit of level l (1..L) is bits
// 3(L-l)..3(L-l)+2, ordered (x, y, z) from most to least significant; bits
// from 3L upwards hold the system id (batched mode; 0 for one system).
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Prefix identifying the level-`level` cell of a key (level 0: the system).
__device__ __forceinline__ uint64_t key_prefix(uint64_t key, int level, int levels) {
    return key >> (3 * (levels - level));
}

// Number of leading octal digits two keys share (0..levels), or -1 when they
// belong to different systems.
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b, int levels) {
    uint64_t x = a ^ b;
    if (x == 0) return levels;
    if (x >> (3 * levels)) return -1;
    return (__clzll((long long)x) - (64 - 3 * levels)) / 3;
}

// ---- FP64 geometry of the walk, rounded exactly as written (no contraction).
// The maxima are fmax: on finite inputs they can differ from a comparison-
// based maximum only in the sign of a zero, which squaring removes.
__device__ __forceinline__ double gap_box(double alo, double ahi, double blo, double bhi) {
#pragma clang fp contract(off)
    double t1 = blo - ahi;
    double t2 = alo - bhi;
    return fmax(fmax(t1, t2), 0.0);
}

__device__ __forceinline__ double gap_point(double alo, double ahi, double p) {
#pragma clang fp contract(off)
    double t1 = p - ahi;
    double t2 = alo - p;
    return fmax(fmax(t1, t2), 0.0);
}

__device__ __forceinline__ double sum_sq3(double gx, double gy, double gz) {
#pragma clang fp contract(off)
    double xx = gx * gx;
    double yy = gy * gy;
    double zz = gz * gz;
    double s = xx + yy;
    return s + zz;
}

// Traceless quadrupole A' = 3/2 S - 1/2 tr(S) I (eq. quadtr) of the second
// moment S about the centre of mass, doubled and rounded to FP32, with the
// mass: the two records the mixed-precision force kernel stages per
// accepted cell. Doubling is exact after rounding.
__device__ __forceinline__ void quad_f32(const double S[6], double M, float4 *q0, float4 *q1) {
#pragma clang fp contract(off)
    const double tr = (S[0] + S[1]) + S[2];
    const double h = 0.5 * tr;
    *q0 = make_float4(2.0f * (float)(1.5 * S[0] - h), 2.0f * (float)(1.5 * S[1] - h),
                      2.0f * (float)(1.5 * S[2] - h), 2.0f * (float)(1.5 * S[3]));
    *q1 = make_float4(2.0f * (float)(1.5 * S[4]), 2.0f * (float)(1.5 * S[5]), (float)M, 0.0f);
}

// Specific Kepler energy v^2/2 - mu/|r| of a pair (eq. dr) from its relative
// position r and velocity v, with |r| in *rr. Its sign decides integer
// outputs (which pairs are bound binaries), so every operation is rounded
// as written: squares summed x, y, then z, no contraction.
__device__ __forceinline__ double kepler_energy(const double r[3], const double v[3], double mu,
                                                double *rr) {
#pragma clang fp contract(off)
    const double r2 = sum_sq3(r[0], r[1], r[2]);
    const double v2 = sum_sq3(v[0], v[1], v[2]);
    *rr = sqrt(r2);
    const double kin = 0.5 * v2;
    const double pot = mu / *rr;
    return kin - pot;
}

// Neighbour relation of the first search stage: d^2 < max(rs_i, rs_j)^2.
__device__ __forceinline__ bool nb_pair(double xi, double yi, double zi, double rsi, double xj,
                                        double yj, double zj, double rsj) {
#pragma clang fp contract(off)
    double dx = xj - xi;
    double dy = yj - yi;
    double dz = zj - zi;
    double d2 = sum_sq3(dx, dy, dz);
    double R = fmax(rsi, rsj);
    double R2 = R * R;
    return d2 < R2;
}

}  // namespace petar
