// Host-side argument checks of the C ABI (no device access). Each returns
// nullptr when the arguments are acceptable, else a message.
#include "validate.h"

#include <cmath>

namespace petar {

const char *check_params(const petar_params *p) {
    if (!p) return "params is NULL";
    if (!std::isfinite(p->G) || !(p->G > 0.0)) return "params.G must be finite and > 0";
    if (p->precision != PETAR_MIXED && p->precision != PETAR_FP64)
        return "params.precision must be PETAR_MIXED or PETAR_FP64";
    if (p->i_per_lane != 1 && p->i_per_lane != 2 && p->i_per_lane != 4)
        return "params.i_per_lane must be 1, 2 or 4";
    if (p->record_counts != 0 && p->record_counts != 1) return "params.record_counts must be 0 or 1";
    if (p->workspace_cap < 0) return "params.workspace_cap must be >= 0";
    return nullptr;
}

const char *check_build_args(const double *pos, const double *mass, int64_t n, double theta,
                             int leaf_size) {
    if (!pos) return "pos is NULL";
    if (!mass) return "mass is NULL";
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (!std::isfinite(theta) || theta < 0.0) return "theta must be finite and >= 0";
    if (leaf_size < 1 || leaf_size > kMaxLeafSize) return "leaf_size must be in [1, 2^20]";
    return nullptr;
}

const char *check_batch_args(int n_sys, const int64_t *off) {
    if (!off) return "sys_offsets is NULL";
    if (n_sys < 1 || n_sys > kMaxSystemsHost) return "n_sys must be in [1, 512]";
    if (off[0] != 0) return "sys_offsets[0] must be 0";
    for (int s = 0; s < n_sys; s++)
        if (off[s + 1] <= off[s]) return "every system needs at least one particle";
    return nullptr;
}

const char *check_force_args(int group_size, const double *r_in, const double *r_out,
                             const double *r_search, const double *acc, const double *pot,
                             const petar_nblist *nb) {
    if (group_size < 1 || group_size > kMaxGroupSize) return "group_size must be in [1, 2^20]";
    if (!r_in || !r_out || !r_search) return "radius array is NULL";
    if (!acc) return "acc is NULL";
    if (!pot) return "pot is NULL";
    if (nb) {
        if (!nb->offsets_dev) return "nb->offsets_dev is NULL";
        if (nb->capacity < 0) return "nb->capacity must be >= 0";
        if (nb->capacity > 0 && !nb->idx_dev) return "nb->idx_dev is NULL";
    }
    return nullptr;
}

const char *check_radii_args(const double *mass, int64_t n, double r_in_ref, double r_out_ref,
                             double search_factor, double cr_dt, const double *r_in,
                             const double *r_out, const double *r_search) {
    if (!mass) return "mass is NULL";
    if (!r_in || !r_out || !r_search) return "output radius array is NULL";
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (!std::isfinite(r_in_ref) || !std::isfinite(r_out_ref) || r_in_ref < 0.0 ||
        !(r_out_ref > r_in_ref))
        return "need 0 <= r_in_ref < r_out_ref (finite)";
    if (!std::isfinite(search_factor) || search_factor < 1.0)
        return "search_factor must be finite and >= 1";
    if (!std::isfinite(cr_dt) || cr_dt < 0.0) return "cr_dt must be finite and >= 0";
    return nullptr;
}

const char *check_filter_args(int64_t n, const double *pos, const double *vel, const double *mass,
                              const double *r_nb, double c_v, const int64_t *cand_offsets,
                              const int32_t *cand_idx, const petar_nblist *out) {
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (!pos || !vel || !mass || !r_nb) return "pos, vel, mass and r_nb must not be NULL";
    if (!std::isfinite(c_v) || !(c_v > 0.0)) return "c_v must be finite and > 0";
    if (!cand_offsets || !cand_idx) return "candidate offsets and idx must not be NULL";
    if (!out) return "out is NULL";
    if (!out->offsets_dev) return "out->offsets_dev is NULL";
    if (out->capacity < 0) return "out->capacity must be >= 0";
    if (out->capacity > 0 && !out->idx_dev) return "out->idx_dev is NULL";
    return nullptr;
}

const char *check_cluster_args(int64_t n, const int64_t *nb_offsets, const int32_t *nb_idx,
                               const int32_t *label, const int64_t *cl_offsets,
                               const int32_t *members, const int64_t *n_clusters) {
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (!nb_offsets || !nb_idx) return "neighbour offsets and idx must not be NULL";
    if (!label || !cl_offsets || !members) return "label, cl_offsets and members must not be NULL";
    if (!n_clusters) return "n_clusters is NULL";
    return nullptr;
}

const char *check_groups_args(int64_t n, const double *pos, const double *vel, const double *mass,
                              const double *r_in, double theta, const int64_t *cand_offsets,
                              const int32_t *cand_idx, const int32_t *label,
                              const int64_t *grp_offsets, const int32_t *members,
                              const int64_t *n_groups, const int32_t *pairs, int64_t pair_cap,
                              const int64_t *n_pairs) {
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (!pos || !vel || !mass || !r_in) return "pos, vel, mass and r_in must not be NULL";
    if (!std::isfinite(theta) || !(theta > 0.0)) return "theta must be finite and > 0";
    if (!cand_offsets || !cand_idx) return "candidate offsets and idx must not be NULL";
    if (!label || !grp_offsets || !members) return "label, grp_offsets and members must not be NULL";
    if (!n_groups || !n_pairs) return "n_groups and n_pairs must not be NULL";
    if (pair_cap < n / 2) return "pair_cap must be >= N/2";
    if (pair_cap > 0 && !pairs) return "pairs must not be NULL";
    return nullptr;
}

namespace {
int art_points(int order) { return order == 2 ? 4 : 8; }
}  // namespace

const char *check_art_make_args(int64_t n, const double *pos, const double *vel,
                                const double *mass, const double *r_in, const double *r_out,
                                const double *r_search, int64_t n_pair, const int32_t *pairs,
                                int order, double c_d, const petar_art_set *set,
                                const double *frame) {
    if (n < 1) return "N must be >= 1";
    if (n > kMaxParticles) return "N must be < 2^31";
    if (order != 2 && order != 3) return "order must be 2 or 3";
    if (!std::isfinite(c_d) || !(c_d > 0.0)) return "c_d must be finite and > 0";
    if (n_pair < 0 || 2 * n_pair > n) return "n_pair must be in [0, N/2]";
    if (!pos || !vel || !mass) return "pos, vel and mass must not be NULL";
    if (!r_in || !r_out || !r_search) return "r_in, r_out and r_search must not be NULL";
    if (n_pair > 0 && (!pairs || !frame)) return "pairs and frame must not be NULL";
    if (!set) return "set is NULL";
    const int64_t want = n + n_pair * (art_points(order) + 2);
    if (set->n_out != want) return "set->n_out must be N + n_pair (P + 2), P = 4 or 8";
    if (want > kMaxParticles) return "the set must hold < 2^31 particles";
    if (!set->pos_dev || !set->mass_dev || !set->r_in_dev || !set->r_out_dev ||
        !set->r_search_dev || !set->src_dev)
        return "set buffers must not be NULL";
    return nullptr;
}

const char *check_tidal_fit_args(int order, int64_t n, const double *pos, int64_t n_pair,
                                 const int32_t *pairs, const double *frame, int64_t n_out,
                                 const int32_t *src, const double *acc_set, const double *pot_set,
                                 const double *tensor, const double *acc, const double *pot) {
    if (order != 2 && order != 3) return "order must be 2 or 3";
    if (n_pair < 0) return "n_pair must be >= 0";
    if (n_out < n_pair * (art_points(order) + 4) || n_out > kMaxParticles)
        return "n_out must be >= n_pair (P + 4) and < 2^31";
    if (!acc_set) return "acc_set must not be NULL";
    if (n_pair > 0 && (!frame || !tensor)) return "frame and tensor must not be NULL";
    if (pot && !acc) return "pot requires acc";
    if (acc) {
        if (n < 1 || n > kMaxParticles) return "N must be in [1, 2^31)";
        if (!pos || !src) return "pos and src must not be NULL";
        if (n_pair > 0 && !pairs) return "pairs must not be NULL";
        if (pot && !pot_set) return "pot requires pot_set";
    }
    return nullptr;
}

const char *check_tidal_eval_args(int order, int64_t n_pair, const double *tensor,
                                  const double *frame, int64_t n_pt, const int32_t *pair_of,
                                  const double *pos, const double *acc) {
    if (order != 2 && order != 3) return "order must be 2 or 3";
    if (n_pair < 0 || n_pair > kMaxParticles) return "n_pair must be in [0, 2^31)";
    if (n_pt < 0 || n_pt > kMaxParticles) return "n_pt must be in [0, 2^31)";
    if (n_pt > 0 && (!pair_of || !pos || !acc)) return "pair_of, pos and acc must not be NULL";
    if (n_pt > 0 && n_pair > 0 && (!tensor || !frame)) return "tensor and frame must not be NULL";
    return nullptr;
}

}  // namespace petar
