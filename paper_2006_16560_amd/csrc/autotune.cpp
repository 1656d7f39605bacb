// Autotuner of the tree/walk parameters: leaf size, i-group size and targets
// per lane. It times a step (tree build + long-range force + neighbour
// lists) for each candidate on the caller's particles -- one system, or a
// batch of independent systems built as one forest -- and keeps the
// fastest; results are cached as JSON lines keyed by (floor(log2 N),
// floor(log2 n_sys), theta, precision), and the lookups read them back for
// an N hint (a single system is the batch of one, bucket 0).
//
// The paper tunes its integrator parameters (dt_L, r_out) by scanning
// wall-clock time over a range of values (Sec. "Performance on GPU-based
// Desktop", the dt_L scan); this applies the same practice to the
// GPU-specific parameters of the long-range force.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/petar.h"

namespace {

struct Entry {
    int nbucket = -1;
    int sbucket = 0;  // floor(log2 n_sys); absent in entries of single systems
    double theta = 0.0;
    int precision = 0;
    petar_tuned t{};
};

int n_bucket(int64_t n) {
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n) b++;
    return b;
}

bool same_key(const Entry &e, int nb, int sb, double theta, int prec) {
    return e.nbucket == nb && e.sbucket == sb && std::fabs(e.theta - theta) < 1e-12 &&
           e.precision == prec;
}

// Reads "key": number pairs from one line of the cache.
bool parse_line(const char *line, Entry *e) {
    auto num = [&](const char *key, double *v) {
        const char *p = std::strstr(line, key);
        if (!p) return false;
        p = std::strchr(p, ':');
        if (!p) return false;
        return std::sscanf(p + 1, "%lf", v) == 1;
    };
    double nb, th, pr, lf, gs, ipl, ms;
    if (!num("\"n_bucket\"", &nb) || !num("\"theta\"", &th) || !num("\"precision\"", &pr) ||
        !num("\"leaf_size\"", &lf) || !num("\"group_size\"", &gs) || !num("\"i_per_lane\"", &ipl) ||
        !num("\"ms\"", &ms))
        return false;
    double sb = 0.0;
    if (!num("\"sys_bucket\"", &sb)) sb = 0.0;
    e->nbucket = (int)nb;
    e->sbucket = (int)sb;
    e->theta = th;
    e->precision = (int)pr;
    e->t.leaf_size = (int)lf;
    e->t.group_size = (int)gs;
    e->t.i_per_lane = (int)ipl;
    e->t.ms = ms;
    return true;
}

std::vector<Entry> read_cache(const char *path) {
    std::vector<Entry> out;
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return out;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        Entry e;
        if (parse_line(line, &e)) out.push_back(e);
    }
    std::fclose(f);
    return out;
}

void write_cache(const char *path, const std::vector<Entry> &entries) {
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const Entry &e : entries)
        std::fprintf(f,
                     "{\"n_bucket\": %d, \"sys_bucket\": %d, \"theta\": %.17g, "
                     "\"precision\": %d, \"leaf_size\": %d, \"group_size\": %d, "
                     "\"i_per_lane\": %d, \"ms\": %.17g}\n",
                     e.nbucket, e.sbucket, e.theta, e.precision, e.t.leaf_size,
                     e.t.group_size, e.t.i_per_lane, e.t.ms);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

petar_status lookup(petar_ctx *ctx, int64_t N_hint, int n_sys, double theta,
                    const char *cache_path, petar_tuned *out) {
    if (!ctx || !out || !cache_path || N_hint < 1 || n_sys < 1 || !(theta >= 0.0))
        return PETAR_E_INVALID;
    petar_params p;
    petar_status st = petar_get_params(ctx, &p);
    if (st != PETAR_OK) return st;
    const int nb = n_bucket(N_hint), sb = n_bucket(n_sys);
    for (const Entry &e : read_cache(cache_path)) {
        if (same_key(e, nb, sb, theta, p.precision)) {
            *out = e.t;
            return PETAR_OK;
        }
    }
    return PETAR_E_STATE;
}

// The candidate sweep. build(leaf) builds the tree (or forest) of the
// caller's particles; N is their total number.
template <typename Build>
petar_status tune(petar_ctx *ctx, const Build &build, int64_t N, int n_sys, double theta,
                  const double *r_in, const double *r_out, const double *r_search,
                  const char *cache_path, petar_tuned *out) {
    petar_params p;
    petar_status st = petar_get_params(ctx, &p);
    if (st != PETAR_OK) return st;
    const int nb = n_bucket(N < 1 ? 1 : N), sb = n_bucket(n_sys < 1 ? 1 : n_sys);
    std::vector<Entry> cache = read_cache(cache_path);
    for (const Entry &e : cache) {
        if (same_key(e, nb, sb, theta, p.precision)) {
            *out = e.t;
            p.i_per_lane = e.t.i_per_lane;
            return petar_set_params(ctx, &p);
        }
    }
    // argument check of the build entry point (it reports the exact problem)
    if ((st = build(8)) != PETAR_OK) return st;
    if (!r_in || !r_out || !r_search) return PETAR_E_INVALID;
    // Scratch outputs of the timing runs, neighbour lists included (a step
    // of the hot path returns them): the capacity is what the first
    // candidate needs plus a quarter, grown when a later one needs more.
    double *acc = nullptr, *pot = nullptr;
    int64_t *offs = nullptr;
    int32_t *idx = nullptr;
    int64_t cap = 0;
    auto release = [&]() {
        if (acc) (void)hipFree(acc);
        if (pot) (void)hipFree(pot);
        if (offs) (void)hipFree(offs);
        if (idx) (void)hipFree(idx);
        acc = pot = nullptr;
        offs = nullptr;
        idx = nullptr;
    };
    if (hipMalloc((void **)&acc, (size_t)N * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&pot, (size_t)N * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&offs, (size_t)(N + 1) * sizeof(int64_t)) != hipSuccess) {
        release();
        return PETAR_E_NOMEM;
    }
    const int leaves[] = {4, 8, 16};
    const int groups[] = {32, 48, 64, 96, 128, 192, 256};
    const int ipls[] = {1, 2};
    petar_tuned best{};
    best.ms = -1.0;
    for (int leaf : leaves) {
        for (int group : groups) {
            for (int ipl : ipls) {
                p.i_per_lane = ipl;
                if ((st = petar_set_params(ctx, &p)) != PETAR_OK) {
                    release();
                    return st;
                }
                constexpr int kReps = 6;  // a warm-up call, then the median of five
                double ms[kReps];
                for (int rep = 0; rep < kReps; rep++) {
                    st = build(leaf);
                    petar_nblist nbl{offs, idx, cap, 0};
                    if (st == PETAR_OK)
                        st = petar_force_long(ctx, group, r_in, r_out, r_search, acc, pot, &nbl);
                    if (st == PETAR_E_NB_OVERFLOW) {
                        if (idx) (void)hipFree(idx);
                        idx = nullptr;
                        cap = nbl.required + nbl.required / 4 + 1;
                        if (hipMalloc((void **)&idx, (size_t)cap * sizeof(int32_t)) != hipSuccess) {
                            release();
                            return PETAR_E_NOMEM;
                        }
                        rep--;  // not timed: repeat with room for the lists
                        continue;
                    }
                    if (st != PETAR_OK) {
                        release();
                        return st;
                    }
                    petar_stats s;
                    petar_get_stats(ctx, &s);
                    ms[rep] = s.ms_build + s.ms_force;
                }
                std::sort(ms + 1, ms + kReps);
                const double t = ms[1 + (kReps - 1) / 2];
                if (best.ms < 0.0 || t < best.ms) {
                    best.leaf_size = leaf;
                    best.group_size = group;
                    best.i_per_lane = ipl;
                    best.ms = t;
                }
            }
        }
    }
    release();
    p.i_per_lane = best.i_per_lane;
    if ((st = petar_set_params(ctx, &p)) != PETAR_OK) return st;
    *out = best;
    if (cache_path) {
        Entry e;
        e.nbucket = nb;
        e.sbucket = sb;
        e.theta = theta;
        e.precision = p.precision;
        e.t = best;
        cache.push_back(e);
        write_cache(cache_path, cache);
    }
    return PETAR_OK;
}

}  // namespace

extern "C" petar_status petar_autotune_lookup(petar_ctx *ctx, int64_t N_hint, double theta,
                                              const char *cache_path, petar_tuned *out) {
    return lookup(ctx, N_hint, 1, theta, cache_path, out);
}

extern "C" petar_status petar_autotune_lookup_batch(petar_ctx *ctx, int64_t N_hint, int n_sys,
                                                    double theta, const char *cache_path,
                                                    petar_tuned *out) {
    return lookup(ctx, N_hint, n_sys, theta, cache_path, out);
}

extern "C" petar_status petar_autotune(petar_ctx *ctx, const double *pos, const double *mass,
                                       int64_t N, double theta, const double *r_in,
                                       const double *r_out, const double *r_search,
                                       const char *cache_path, petar_tuned *out) {
    if (!ctx || !out) return PETAR_E_INVALID;
    auto build = [&](int leaf) { return petar_tree_build(ctx, pos, mass, N, theta, leaf); };
    return tune(ctx, build, N, 1, theta, r_in, r_out, r_search, cache_path, out);
}

extern "C" petar_status petar_autotune_batch(petar_ctx *ctx, int n_sys, const int64_t *sys_offsets,
                                             const double *pos, const double *mass, double theta,
                                             const double *r_in, const double *r_out,
                                             const double *r_search, const char *cache_path,
                                             petar_tuned *out) {
    if (!ctx || !out || !sys_offsets || n_sys < 1) return PETAR_E_INVALID;
    const int64_t N = sys_offsets[n_sys];
    auto build = [&](int leaf) {
        return petar_batch_build(ctx, n_sys, sys_offsets, pos, mass, theta, leaf);
    };
    return tune(ctx, build, N, n_sys, theta, r_in, r_out, r_search, cache_path, out);
}
