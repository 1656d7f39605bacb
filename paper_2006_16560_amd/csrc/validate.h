// Host-side argument checks of the C ABI (pure C++, no HIP calls).
#pragma once

#include <stdint.h>

#include "../../include/petar.h"

namespace petar {

constexpr int64_t kMaxParticles = 2147483647LL;  // indices are 32-bit
constexpr int kMaxLeafSize = 1 << 20;
constexpr int kMaxGroupSize = 1 << 20;
constexpr int kMaxSystemsHost = 512;  // batched mode

const char *check_params(const petar_params *p);
const char *check_build_args(const double *pos, const double *mass, int64_t n, double theta,
                             int leaf_size);
const char *check_batch_args(int n_sys, const int64_t *sys_offsets);
const char *check_force_args(int group_size, const double *r_in, const double *r_out,
                             const double *r_search, const double *acc, const double *pot,
                             const petar_nblist *nb);
const char *check_radii_args(const double *mass, int64_t n, double r_in_ref, double r_out_ref,
                             double search_factor, double cr_dt, const double *r_in,
                             const double *r_out, const double *r_search);

const char *check_filter_args(int64_t n, const double *pos, const double *vel, const double *mass,
                              const double *r_nb, double c_v, const int64_t *cand_offsets,
                              const int32_t *cand_idx, const petar_nblist *out);
const char *check_cluster_args(int64_t n, const int64_t *nb_offsets, const int32_t *nb_idx,
                               const int32_t *label, const int64_t *cl_offsets,
                               const int32_t *members, const int64_t *n_clusters);

const char *check_groups_args(int64_t n, const double *pos, const double *vel, const double *mass,
                              const double *r_in, double theta, const int64_t *cand_offsets,
                              const int32_t *cand_idx, const int32_t *label,
                              const int64_t *grp_offsets, const int32_t *members,
                              const int64_t *n_groups, const int32_t *pairs, int64_t pair_cap,
                              const int64_t *n_pairs);
const char *check_art_make_args(int64_t n, const double *pos, const double *vel,
                                const double *mass, const double *r_in, const double *r_out,
                                const double *r_search, int64_t n_pair, const int32_t *pairs,
                                int order, double c_d, const petar_art_set *set,
                                const double *frame);
const char *check_tidal_fit_args(int order, int64_t n, const double *pos, int64_t n_pair,
                                 const int32_t *pairs, const double *frame, int64_t n_out,
                                 const int32_t *src, const double *acc_set, const double *pot_set,
                                 const double *tensor, const double *acc, const double *pot);
const char *check_tidal_eval_args(int order, int64_t n_pair, const double *tensor,
                                  const double *frame, int64_t n_pt, const int32_t *pair_of,
                                  const double *pos, const double *acc);

}  // namespace petar
