// Host-side launchers of the HIP kernels (one definition per .hip file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace petar {

// ---------------------------------------------------------------- scan.hip
// Exclusive prefix sum of n counts into out[0..n] (out[n] = total).
// ws must hold scan_ws_elems(n) int64 values.
int64_t scan_ws_elems(int64_t n);
void scan_u32_to_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s);
void scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n, int64_t *ws, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- tree.hip
struct TreeDev {
    // particles (Morton order)
    double4 *ps;
    double2 *rr;
    double *rsk;
    uint32_t *orig;             // input index of each particle
    uint32_t *rank;             // Morton position of each input index
    // cells
    double4 *nd_lo, *nd_hi, *nd_com;
    double *nd_S;
    float4 *nd_q;               // [2 n_nodes]: 2A' and M in FP32 (quad_f32)
    uint4 *nd_info;
    uint32_t *nd_parent;        // kNone for a root
    const uint32_t *level_off;  // [23]: cells of level l are [level_off[l], level_off[l+1])
    const int64_t *n_nodes_dev; // number of cells (device); n_nodes below bounds it
    int64_t n;
    int64_t n_nodes;            // capacity of the cell arrays (grid sizes)
};

// Cells as emitted in depth-first pre-order, kept for the group selection
// (groups listed in Morton order) and the renumbering into level order.
struct PreOrder {
    uint4 *info;        // (first particle, count, leaf | level << 1, -)
    uint32_t *parent;   // kNone for the root
    uint32_t *nchild;
    uint32_t *new_of_old;
};

int bbox_partial_blocks(int64_t n);
void launch_bbox(const double *pos, const double *mass, int64_t n, double *part, RootBox *rb,
                 hipStream_t s);
void launch_keys(const double *pos, int64_t n, const RootBox *rb, uint64_t *key, uint32_t *idx,
                 hipStream_t s);
// batched mode: rb[n_sys], off = system offsets on the device [n_sys + 1]
void launch_bbox_systems(const double *pos, const double *mass, int64_t n, const int64_t *off,
                         int n_sys, RootBox *rb, hipStream_t s);
void launch_keys_systems(const double *pos, int64_t n, const int64_t *off, int n_sys,
                         const RootBox *rb, uint64_t *key, uint32_t *idx, hipStream_t s);

// LSD radix sort of (key, value) pairs on the low 8*passes key bits, stable.
// Buffers are swapped in place: the sorted result ends in (*key, *val).
int64_t sort_ws_bytes(int64_t n);
// n bounds the element count; with n_dev the actual count is read on the device.
void radix_sort(uint64_t **key, uint32_t **val, uint64_t **key_alt, uint32_t **val_alt, int64_t n,
                int passes, void *ws, hipStream_t s,
                const int64_t *n_dev = nullptr);

void launch_gather_particles(const double *pos, const double *mass, const uint32_t *idx,
                             int64_t n, double4 *ps, uint32_t *orig, uint32_t *rank,
                             hipStream_t s);
// Also the deepest cell level: the maximum of deep_slots[w * kDeepStride],
// w < kDeepSlots (kDeepWords words, zeroed by the caller), after the kernel.
constexpr int kDeepSlots = 32;
constexpr int kDeepStride = 32;  // 128 B
constexpr int kDeepWords = kDeepSlots * kDeepStride;
void launch_octree_count(const uint64_t *key, int64_t n, int leaf_size, int levels,
                         uint32_t *emit, uint32_t *deep_slots, hipStream_t s);
// st->cells = base[n], st->bad_input = rb->bad, st->deep = the deepest level
// among deep_slots (kDeepWords words).
void launch_build_head(const int64_t *base, int64_t n, const RootBox *rb,
                       const uint32_t *deep_slots, Status *st, hipStream_t s);
// Pre-order cells; also the level keys (lkey, lval) sorted next.
// Cells beyond node_cap are not written; st->cell_overflow is raised instead.
void launch_octree_write(const uint64_t *key, int64_t n, int leaf_size, int levels,
                         const int64_t *base, PreOrder pre, uint64_t *lkey, uint32_t *lval,
                         int64_t node_cap, Status *st, hipStream_t s);
// Level-order arrays from the level-sorted permutation perm (new -> old).
// rb holds one root box per system (one in single-system mode).
void launch_relayout(const uint32_t *perm, PreOrder pre, const RootBox *rb, const uint64_t *key,
                     int levels, TreeDev t, uint32_t *level_off, hipStream_t s);
void launch_moments(const TreeDev &t, int levels, hipStream_t s);
void launch_tree_summary(const TreeDev &t, Status *st, hipStream_t s);

// force_long preparation
void launch_gather_radii(const double *r_in, const double *r_out, const double *r_search,
                         TreeDev t, Status *st, hipStream_t s);
void launch_rsmax(const TreeDev &t, hipStream_t s);
// flag[] is written for every slot up to t.n_nodes (the capacity), 0 past the cells.
void launch_group_flags(const PreOrder &pre, const TreeDev &t, int group_size, uint32_t *flag,
                        hipStream_t s);
void launch_group_compact(const PreOrder &pre, const TreeDev &t, const uint32_t *flag,
                          const uint32_t *pos, uint32_t *groups, Status *st, hipStream_t s);

// changeover radii (eq. rcut / eq. rnb)
void launch_changeover_radii(const double *mass, const double *vel, int64_t n, double rin_ref,
                             double rout_ref, double search_factor, double cr_dt, double *r_in,
                             double *r_out, double *r_search, double *ws, hipStream_t s);

// --------------------------------------------------------------- force.hip
// Near leaves handed from the force walk to the neighbour passes: one header
// per near flush of a group (group's first particle, group size, first leaf
// entry, number of leaf entries) and the flushed leaves (first particle,
// particle count), all in Morton order. count[0] and count[1] are the
// headers and leaf entries claimed; either above its capacity means the
// lists are incomplete and the walk-based passes run instead.
struct NbRecords {
    uint4 *head;
    uint2 *leaf;
    uint32_t *count;
    uint32_t head_cap, leaf_cap;
};

struct ForceLaunch {
    TreeDev t;
    const uint32_t *groups;
    const Status *st_in;       // n_groups and validity flags
    Status *st;                // counters out
    double th2;                // theta^2
    double G;
    double *acc, *pot;         // caller's outputs, input order
    uint32_t *spill;           // walk stack spill, per resident wave
    uint32_t *queue;           // 8 work-queue heads
    int32_t *counts;           // optional per-particle counts [4][n]
    NbRecords nb;              // near-leaf lists for the neighbour passes (head null: none)
    uint32_t *nb_bound;        // optional [n], input order: particles of the group's near
                               // leaves, a bound of each target's neighbour list
    double *kick_vel;          // optional [3][n]: vel += kick_dt * acc with the output write
    double kick_dt;
    int precision;             // 0 mixed, 1 fp64
    int ipl;                   // 1, 2, 4
    // optional target subset: tpos[k] = targets before Morton position k
    // ([n + 1]), tidx = their Morton positions; null: every particle
    const uint32_t *tpos, *tidx;
};
// flag[k] = target[orig[k]] != 0 (Morton order); acc and pot of the
// particles that are not targets are set to 0 (input order).
void launch_target_flags(const uint8_t *target, const TreeDev &t, uint32_t *flag, double *acc,
                         double *pot, hipStream_t s);
// tidx[tpos[k]] = k for every flagged k.
void launch_target_compact(const uint32_t *flag, const uint32_t *tpos, int64_t n, uint32_t *tidx,
                           hipStream_t s);
int force_resident_waves(int precision, int ipl, int device);
int64_t force_spill_elems_per_wave();
void launch_force(const ForceLaunch &f, int resident_waves, hipStream_t s);

// -------------------------------------------------------------- nblist.hip
// Neighbour lists around two prefix sums, all per target in input order. The
// force walk bounds each target's list by the particles of its group's near
// leaves (nb_bound); the prefix sum of the bounds gives every target a row
// of scratch (row_off); a testing pass writes each target's hits into its
// row and counts them (cursor); the prefix sum of the counts gives the CSR
// offsets; a per-list sort moves the rows into the CSR.
// Testing pass over the near-leaf records of the force walk; it does nothing
// when the records overflowed (*rec_count > rec_cap) or the rows exceed the
// scratch (row_off[n] > row_cap).
void launch_nb_write_rec(const TreeDev &t, const NbRecords &rec, const Status *st,
                         const int64_t *row_off, uint32_t *cursor, int32_t *rows, int64_t row_cap,
                         hipStream_t s);
// The same counting only (cnt += hits): exact bounds for the
// fallback when the walk's bounds ask for more rows than the scratch may
// hold.
void launch_nb_count_rec(const TreeDev &t, const NbRecords &rec, const Status *st,
                         uint32_t *cnt, hipStream_t s);
// Walk-based testing pass: runs only when the near-leaf records overflowed
// (or were not written: rec.count == nullptr); stores the counts in cursor
// (rows null: counts only).
void launch_nb_write(const TreeDev &t, const uint32_t *groups, Status *st, uint32_t *cursor,
                     const int64_t *row_off, int32_t *rows, int64_t row_cap, uint32_t *spill,
                     uint32_t *queue, const NbRecords &rec, int resident_waves, hipStream_t s);
// st->nb_total = offsets[n], st->nb_rows = row_off[n], st->rec_used =
// rec_count[0..1] (one status copy then tells the host the list size, the
// scratch the rows need and the hand-over use).
void launch_nb_summary(const int64_t *offsets, const int64_t *row_off, int64_t n,
                       const uint32_t *rec_count, Status *st, hipStream_t s);
void launch_nb_sort(const int64_t *row_off, const int32_t *rows, const int64_t *offsets,
                    int32_t *idx, int64_t n, int64_t capacity, const Status *st,
                    uint32_t *long_list, uint32_t *long_count, hipStream_t s);
int nb_resident_waves(int device);

// ------------------------------------------------------------ cluster.hip
// Second-stage neighbour filter over a candidate CSR (input order).
// mode 0: pericentre < c_v r_nb[i] (second neighbour stage);
// mode 1: separation < c_v max(r_nb[i], r_nb[j]) (SDAR groups, r_nb = r_in,
// c_v = theta).
struct FilterArgs {
    const double *pos, *vel, *mass, *r_nb;  // [3][n], [3][n], [n], [n]
    const int64_t *offsets;                 // [n + 1]
    const int32_t *idx;
    int64_t n;
    double c_v, G;
    int mode;
};
// *bad |= (offsets[0] != 0 or offsets decrease somewhere)
void launch_check_csr(const int64_t *offsets, int64_t n, int32_t *bad, hipStream_t s);
void launch_filter(const FilterArgs &a, int64_t n_cand, int32_t *row, uint8_t *keep,
                   uint32_t *counts, int32_t *bad, hipStream_t s);
void launch_filter_write(const FilterArgs &a, const uint8_t *keep, const int64_t *out_offsets,
                         int32_t *out_idx, int64_t capacity, hipStream_t s);
// Components of a neighbour CSR (pairs taken both ways): label[i] =
// smallest index of i's component, is_root[i] = (label[i] == i); parent is
// scratch [n]; *bad |= an index outside [0, n). Nothing runs when *csr_bad.
void launch_components(const int64_t *offsets, const int32_t *idx, int64_t n, int32_t *parent,
                       int32_t *label, uint32_t *is_root, int32_t *bad, const int32_t *csr_bad,
                       hipStream_t s);
// Keys (cluster index, root_pos = cluster index of each root) and values
// (particle index) whose stable sort lists the members of every cluster in
// ascending order; cluster offsets from the sorted keys.
void launch_cluster_keys(const int32_t *label, int64_t n, const uint32_t *root_pos, uint64_t *key,
                         uint32_t *val, hipStream_t s);
void launch_cluster_offsets(const uint64_t *sorted_key, int64_t n, int64_t *cl_offsets,
                            hipStream_t s);
// Fixed device scratch of petar_clusters_noalloc: one array of
// kNoAllocScratchBytes per device, in the code object's static data, so the
// call needs no allocation. noalloc_scratch() must be called with `device`
// current; the first call on a device looks the array up
// (hipGetSymbolAddress) and keeps its address, later calls return it.
constexpr int64_t kNoAllocMaxN = int64_t(1) << 20;
constexpr size_t kNoAllocScratchBytes = size_t(40) << 20;
hipError_t noalloc_scratch(int device, void **ptr, size_t *bytes);
// Binaries among the groups: is_pair[g] = 1 for a group of exactly two
// members with negative Kepler energy (G (m1 + m2) / r > v^2 / 2).
void launch_group_pairs(const int64_t *grp_offsets, const int32_t *members, int64_t n_groups,
                        const double *pos, const double *vel, const double *mass, int64_t n,
                        double G, uint32_t *is_pair, hipStream_t s);
// pairs[pos[g]] and pairs[pair_cap + pos[g]] for every flagged group.
void launch_group_pairs_write(const int64_t *grp_offsets, const int32_t *members, int64_t n_groups,
                              const uint32_t *is_pair, const uint32_t *pos, int32_t *pairs,
                              int64_t pair_cap, hipStream_t s);

// --------------------------------------------------------- artificial.hip
// Set of the long-range force with artificial particles: singles first (input
// order), then one block of P + 4 per pair (centre, P measure points, three
// pseudoparticles); P = 4 (order 2) or 8 (order 3).
struct ArtArgs {
    const double *pos, *vel, *mass, *r_in, *r_out, *r_search;  // [3][n], [3][n], [n] x4
    int64_t n;
    const int32_t *pairs;  // [2][n_pair]
    int64_t n_pair;
    int order;
    double c_d, G;
    int64_t n_single, n_out;  // n - 2 n_pair, n_single + n_pair (P + 4)
    double *o_pos, *o_mass, *o_rin, *o_rout, *o_rs;  // [3][n_out], [n_out] x4
    int32_t *src;      // [n_out]: input index of a single, -1 for artificial
    double *frame;     // [4][n_pair]: centre of mass, d_c
    int32_t *pair_of;  // [n]: pair of a member, -1 for a single
    uint8_t *o_target; // optional [n_out]: 1 for singles, centres and measure points
};
// bad[0]: index outside [0, n) or i == j; bad[1]: particle in two pairs;
// bad[2]: pair not bound. single/spos hold n and n + 1 entries.
void launch_art_make(const ArtArgs &a, uint32_t *single, uint32_t *spos, int64_t *scan_ws,
                     int32_t *bad, hipStream_t s);

// Post-fit: per pair the record [phi(r_cm), A(r_cm), T] ([4 + K][n_pair]);
// with acc set, the members' field and the singles' copies ([3][n]).
struct FitArgs {
    int order;
    int64_t n_pair, n_single, n_out;
    const double *acc_set, *pot_set;  // [3][n_out], [n_out] (pot_set may be null)
    const double *frame;              // [4][n_pair]
    const double *ginv;               // K x 3P, row-major, device
    double *tensor;                   // [4 + K][n_pair]
    const double *pos;                // [3][n] (when acc is set)
    int64_t n;
    const int32_t *pairs, *src;       // [2][n_pair], [n_out]
    double *acc, *pot;                // [3][n], [n] (may be null)
};
void launch_tidal_fit(const FitArgs &f, hipStream_t s);

struct EvalArgs {
    int order;
    int64_t n_pair;
    const double *tensor, *frame;  // [4 + K][n_pair], [4][n_pair]
    int64_t n_pt;
    const int32_t *pair_of;        // [n_pt], < 0: point skipped
    const double *pos;             // [3][n_pt]
    double *acc, *pot;             // [3][n_pt], [n_pt] (pot may be null)
    int32_t *bad;                  // count of pair_of >= n_pair
};
void launch_tidal_eval(const EvalArgs &e, hipStream_t s);
// v += a dt over [3][n] (long-range kick).
void launch_kick(double *vel, const double *acc, int64_t n, double dt, hipStream_t s);
// Generalized inverse of the measure-point map at d_c = 1 (host memory,
// K x 3P row-major), computed once.
const double *tidal_ginv_host(int order);

}  // namespace petar
