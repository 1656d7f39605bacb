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

}  // namespace petar
