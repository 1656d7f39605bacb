// Wave-wide depth-first traversal of the octree for one i-group.
//
// One wavefront walks the tree for its group: each step pops up to 64 cells
// (one per lane), classifies them in parallel and pushes the children of the
// opened cells. The stack lives in LDS (kStackLds entries per wave); when a
// push would not fit, its oldest entries move to a per-wave global area, and
// pops refill from there when the LDS part is empty. Cells are classified with the
// FP64 geometry of common.h, rounded as written, so the decisions are
// reproducible bit for bit by any implementation of the same formulas.
#pragma once

#include "common.h"

namespace petar {

constexpr int kStackLds = 512;       // >= 64 lanes x 8 children
constexpr int kStackSlack = 8;       // room for the overhang of the last push (see push)
constexpr int kSpillCap = 16384;     // per resident wave

struct GroupGeom {
    double lo[3], hi[3];
    double rs;       // max r_search of the group's particles
    double c[3];     // centre of the bounding box (origin of FP32 coordinates)
};

__device__ __forceinline__ GroupGeom load_group(const double4 *nd_lo, const double4 *nd_hi,
                                                uint32_t g) {
    GroupGeom G;
    double4 lo = nd_lo[g], hi = nd_hi[g];
    G.lo[0] = lo.x;
    G.lo[1] = lo.y;
    G.lo[2] = lo.z;
    G.hi[0] = hi.x;
    G.hi[1] = hi.y;
    G.hi[2] = hi.z;
    G.rs = lo.w;
    for (int d = 0; d < 3; d++) G.c[d] = 0.5 * (G.lo[d] + G.hi[d]);
    return G;
}

// Squared distance between the group's box and a cell's box, and the
// squared pair-search radius max(rs_group, rs_cell)^2.
__device__ __forceinline__ void box_terms(const GroupGeom &G, const double4 &lo,
                                          const double4 &hi, double *D2, double *R2) {
#pragma clang fp contract(off)
    *D2 = sum_sq3(gap_box(G.lo[0], G.hi[0], lo.x, hi.x), gap_box(G.lo[1], G.hi[1], lo.y, hi.y),
                  gap_box(G.lo[2], G.hi[2], lo.z, hi.z));
    double R = fmax(G.rs, lo.w);
    *R2 = R * R;
}

// Multipole acceptance: side^2 < theta^2 * dmin^2 with dmin the distance
// from the group's box to the cell's centre of mass.
__device__ __forceinline__ bool mac_accept(const GroupGeom &G, const double4 &com, double side,
                                           double th2) {
#pragma clang fp contract(off)
    double dm2 = sum_sq3(gap_point(G.lo[0], G.hi[0], com.x), gap_point(G.lo[1], G.hi[1], com.y),
                         gap_point(G.lo[2], G.hi[2], com.z));
    double side2 = side * side;
    double rhs = th2 * dm2;
    return side2 < rhs;
}

// Root of the tree (system) that holds particle `first`: level 0 lists the
// roots, one per system, in particle order.
__device__ __forceinline__ uint32_t root_of(const uint4 *nd_info, const uint32_t *level_off,
                                            uint32_t first) {
    uint32_t lo = 0, hi = level_off[1];
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (nd_info[mid].x <= first)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

struct WaveStack {
    uint32_t *lds;     // kStackLds + kStackSlack entries
    uint32_t *spill;   // kSpillCap entries
    int sp_l;          // entries in LDS (wave-uniform)
    int sp_g;          // entries in the spill (wave-uniform)

    __device__ void init(uint32_t root) {
        if (lane_id() == 0) lds[0] = root;
        sp_l = 1;
        sp_g = 0;
        wave_sync();
    }
    __device__ bool empty() const { return sp_l == 0 && sp_g == 0; }

    // Pops up to 64 cells; lane l gets one or kNone.
    __device__ uint32_t pop() {
        if (sp_l == 0) {
            int m = sp_g < kStackLds / 2 ? sp_g : kStackLds / 2;
            wave_sync();
            for (int t = lane_id(); t < m; t += kWave) lds[t] = spill[sp_g - m + t];
            sp_g -= m;
            sp_l = m;
            wave_sync();
        }
        int take = sp_l < kWave ? sp_l : kWave;
        uint32_t v = lane_id() < take ? lds[sp_l - take + lane_id()] : kNone;
        sp_l -= take;
        wave_sync();
        return v;
    }

    // Pushes each lane's children: the nc cells first .. first + nc - 1
    // (children are contiguous in level order). Returns false on spill
    // overflow.
    __device__ bool push(uint32_t first, int nc) {
        int incl = wave_incl_scan(nc);
        int tot = last_lane(incl);
        if (tot == 0) return true;
        if (sp_l + tot > kStackLds) {
            // move the oldest entries, as many as the push needs rounded up
            // to whole waves, to the spill and shift the rest down (the
            // order of the whole stack is unchanged)
            int h = (sp_l + tot - kStackLds + kWave - 1) / kWave * kWave;
            h = h < sp_l ? h : sp_l;
            if (sp_g + h > kSpillCap) return false;
            for (int t = lane_id(); t < h; t += kWave) spill[sp_g + t] = lds[t];
            wave_sync();
            for (int t0 = 0; t0 < sp_l - h; t0 += kWave) {
                const int t = t0 + lane_id();
                const uint32_t v = t < sp_l - h ? lds[h + t] : 0u;
                wave_sync();
                if (t < sp_l - h) lds[t] = v;
                wave_sync();
            }
            sp_g += h;
            sp_l -= h;
        }
        int p = sp_l + incl - nc;
        if (nc > 0) {
            // Each pushing lane writes 8 slots, the highest first, without a
            // test per slot (an octree cell has at most 8 children). A slot
            // past its own nc children lies in the range of a later pushing
            // lane, which writes that slot at a smaller offset, i.e. in a
            // later store of this sequence, or past the new top of the stack
            // (kStackSlack spare entries). The stores of a wave reach LDS in
            // program order; the empty asm statements keep the compiler from
            // reordering or merging them.
#pragma unroll
            for (int c = 7; c >= 0; c--) {
                lds[p + c] = first + (uint32_t)c;
                asm volatile("" ::: "memory");
            }
        }
        sp_l += tot;
        wave_sync();
        return true;
    }
};

}  // namespace petar
