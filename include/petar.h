/*
 * petar.h -- C ABI of the MI355X (gfx950) long-range P3T tree-force library.
 *
 * The library computes the long-range half of the particle-particle
 * particle-tree (P3T) Hamiltonian split used by PeTar (Wang, Iwasawa,
 * Nitadori & Makino 2020, Sec. "Hybrid methods with Hamiltonian splitting"
 * and eq. cf): for every particle i
 *
 *   a_L,i   = sum_j G m_j (1 - K(x_ij)) (r_j - r_i) / |r_j - r_i|^3
 *   phi_L,i = -sum_j G m_j (1 - W(x_ij)) / |r_j - r_i|
 *
 * with the changeover weights W (potential) and K (force, eq. Wij) of the
 * section "Mass-dependent changeover function", pair radii
 * r_in,ij = max(r_in,i, r_in,j), r_out,ij = max(r_out,i, r_out,j),
 * x = (r - r_in,ij)/(r_out,ij - r_in,ij). Distant particles are grouped in
 * a Barnes-Hut octree whose cells, when they lie inside the opening angle
 * theta as seen from a group of target particles, act through their centre
 * of mass and traceless quadrupole (eq. quad, eq. quadtr; Sec. "Particle-
 * tree with individual time steps"). Alongside the force it returns the
 * neighbour candidates of the first stage of the neighbour search (Sec.
 * "Orbit-dependent neighbour criterion"): all j != i with
 * |r_j - r_i| < max(r_search,i, r_search,j).
 *
 * Conventions shared by every call
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors) on the context's device; everything else is host memory.
 *  - Arrays of vectors are structure-of-arrays: pos[3][N] means x[0..N),
 *    then y, then z, contiguous FP64.
 *  - The caller owns every input and output buffer. The library owns the
 *    tree and all scratch memory held by the context (freed by
 *    petar_destroy).
 *  - All work is enqueued on the context's HIP stream. A call returns after
 *    it has read back the small status words it needs (the inputs may be
 *    reused as soon as it returns; outputs are complete when the stream is).
 *  - Every call validates its arguments before any launch and returns a
 *    petar_status; petar_last_error() gives a message for the last failure.
 *  - One context per host thread / stream; contexts are independent.
 */
#ifndef PETAR_H
#define PETAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PETAR_API __attribute__((visibility("default")))
#else
#define PETAR_API
#endif

typedef struct petar_ctx petar_ctx;

typedef enum {
    PETAR_OK = 0,
    PETAR_E_INVALID = -1,     /* bad argument (pointer, size, value range, non-finite input) */
    PETAR_E_NOMEM = -2,       /* device allocation failed or exceeds the workspace cap       */
    PETAR_E_HIP = -3,         /* a HIP runtime call failed                                   */
    PETAR_E_NB_OVERFLOW = -4, /* neighbour capacity too small; nb->required holds the need   */
    PETAR_E_STATE = -5,       /* call order violated (e.g. force before tree build)          */
    PETAR_E_NODEVICE = -6,    /* context created without a device (validation only)          */
    PETAR_E_INTERNAL = -7     /* a kernel reported an internal limit (message says which)    */
} petar_status;

typedef enum {
    PETAR_MIXED = 0, /* FP32 pair arithmetic on group-relative coordinates, compensated sums */
    PETAR_FP64 = 1   /* the same walk and kernels with FP64 pair arithmetic                  */
} petar_precision;

/* Pass as `device` to petar_create for a context that validates arguments
 * but owns no GPU (every call that would launch returns PETAR_E_NODEVICE). */
#define PETAR_NO_DEVICE (-1)

typedef struct {
    double G;              /* gravitational constant (default 1, Henon units)            */
    int precision;         /* petar_precision (default PETAR_MIXED)                      */
    int i_per_lane;        /* target particles per lane in the force kernel: 1, 2 or 4   */
    int record_counts;     /* 1: keep per-particle interaction counts (petar_copy_counts) */
    int64_t workspace_cap; /* max bytes of library-owned device memory (0: no cap)        */
} petar_params;

/* Neighbour lists in CSR form, input order. offsets_dev[N+1] (int64) and
 * idx_dev[capacity] (int32) are caller-owned device buffers. On return
 * `required` is the total number of entries. Each list is sorted by
 * ascending original index and excludes i itself. */
typedef struct {
    int64_t *offsets_dev;
    int32_t *idx_dev;
    int64_t capacity;
    int64_t required;
} petar_nblist;

/* Counters of the last petar_force_long / petar_tree_build. */
typedef struct {
    int64_t n;                 /* particles                                     */
    int64_t n_nodes;           /* octree cells                                  */
    int64_t n_leaves;
    int64_t n_groups;          /* i-groups of the last force call               */
    int64_t max_level;
    int64_t inter_pc;          /* particle-cell (multipole) interactions        */
    int64_t inter_far;         /* particle-particle, Newtonian (far leaves)     */
    int64_t inter_near;        /* particle-particle, changeover (near leaves)   */
    int64_t nb_total;          /* neighbour-list entries                        */
    /* device times (HIP events) of the last eager calls; a graph replay     */
    /* sets ms_graph and zeroes the stage times                              */
    double ms_build;           /* device time of the last tree build            */
    double ms_force;           /* device time of the last force call (total)   */
    double ms_force_kernel;    /* device time of the walk + interaction kernel  */
    double ms_nb;              /* device time of the neighbour-list stage       */
    double ms_graph;           /* device time of the last replayed step graph   */
    int64_t workspace_bytes;   /* library-owned device memory                   */
} petar_stats;

/* Create a context on `device` (HIP ordinal, or PETAR_NO_DEVICE) whose work
 * goes to `hip_stream` (a hipStream_t; NULL for the default stream). */
PETAR_API petar_status petar_create(petar_ctx **out, int device, void *hip_stream);
PETAR_API petar_status petar_destroy(petar_ctx *ctx);

/* Defaults: G = 1, PETAR_MIXED, i_per_lane = 1, no counts, no cap. */
PETAR_API petar_status petar_set_params(petar_ctx *ctx, const petar_params *params);
PETAR_API petar_status petar_get_params(petar_ctx *ctx, petar_params *params);

/* Per-particle changeover radii, eq. rcut: with s_i = max(1, m_i/<m>)^(1/3)
 * and <m> = sum(m)/N, r_in,i = s_i r_in_ref and r_out,i = s_i r_out_ref.
 * The search radius is search_factor * r_out,i when vel_dev is NULL, else
 * eq. rnb: r_out,i + cr_dt |v_i| with cr_dt = C_r * dt_L.
 * Requires 0 <= r_in_ref < r_out_ref, search_factor >= 1, cr_dt >= 0.
 * mass_dev[N], vel_dev[3][N] (or NULL); outputs [N] each. */
PETAR_API petar_status petar_changeover_radii(petar_ctx *ctx, const double *mass_dev, const double *vel_dev,
                                    int64_t N, double r_in_ref, double r_out_ref,
                                    double search_factor, double cr_dt, double *r_in_dev,
                                    double *r_out_dev, double *r_search_dev);

/* Build the Barnes-Hut octree of N particles (Sec. "Particle-tree with
 * individual time steps": the particle-tree half of P3T; its cells carry
 * the mass, centre of mass and traceless quadrupole of eq. quad and
 * eq. quadtr): pos_dev[3][N], mass_dev[N] (m >= 0, finite). theta >= 0 is
 * the opening angle used by the following force calls; leaf_size >= 1
 * bounds the particles of a leaf cell (cells at the deepest level, 21, may
 * hold more). 1 <= N < 2^31.
 * The positions are copied into the context (sorted); the caller may change
 * its buffers afterwards. The call returns once the cell count has been read
 * back; the rest of the build (cell data from the sorted copies) is still
 * queued on the stream, and the counters it sets (n_leaves, max_level,
 * ms_build) are read with the next force call or petar_get_stats. */
PETAR_API petar_status petar_tree_build(petar_ctx *ctx, const double *pos_dev, const double *mass_dev,
                              int64_t N, double theta, int leaf_size);

/* Batched mode: n_sys independent particle systems (star clusters) stored
 * back to back, each with the octree of petar_tree_build (Sec. "Particle-
 * tree with individual time steps"; each system is one star cluster like
 * the models of Sec. "Benchmark", Table inpar). System s holds particles
 * sys_offsets[s] .. sys_offsets[s+1]-1 (sys_offsets is a host array of
 * n_sys + 1 entries, sys_offsets[0] = 0, strictly increasing;
 * 1 <= n_sys <= 512). Builds one octree per system (own root cube, 18
 * levels) in a single pass; the next petar_force_long computes every
 * system's long-range force and neighbour lists in one launch, with no
 * interaction between systems. Output indices are global (input order). */
PETAR_API petar_status petar_batch_build(petar_ctx *ctx, int n_sys, const int64_t *sys_offsets,
                                         const double *pos_dev, const double *mass_dev,
                                         double theta, int leaf_size);

/* Long-range acceleration and potential of the P3T split (eq. cf; pair
 * weights 1 - K and (1 - W)/r of eq. Wij; cells accepted inside the
 * opening angle act through their monopole and quadrupole, eq. quadtr) on
 * every particle of the last tree build (input order), and the first-stage
 * neighbour candidates (Sec. "Orbit-dependent neighbour criterion"):
 * acc_dev[3][N], pot_dev[N]. group_size >= 1 is the i-group size of the
 * walk. r_in_dev, r_out_dev, r_search_dev [N] are the changeover and search
 * radii; 0 <= r_in < r_out <= r_search and finite for every particle. nb
 * may be NULL (no neighbour lists). On PETAR_E_NB_OVERFLOW acc and pot are
 * complete and nb->required is set: the caller retries with a larger
 * buffer. With lists, the library also holds scratch rows of 4 bytes per
 * pair its near test examines (bounded by 256 entries a particle and by
 * params.workspace_cap; beyond that it counts exactly first and needs no
 * more rows than nb->capacity). */
PETAR_API petar_status petar_force_long(petar_ctx *ctx, int group_size, const double *r_in_dev,
                              const double *r_out_dev, const double *r_search_dev,
                              double *acc_dev, double *pot_dev, petar_nblist *nb);

/* Restricts the following petar_force_long / petar_force_long_kick calls on
 * the current tree to a subset of target particles: target_dev[N] (uint8,
 * input order, caller-owned and kept alive until those calls return),
 * nonzero for a particle whose force is wanted. Every particle still acts as
 * a source. The force, potential (and kick) of the others are not computed:
 * their acc and pot entries are set to 0 and their velocities are left
 * alone. This gives the particles of the artificial set their roles (Sec.
 * "Artificial particle algorithm for weak perturbation"): the measure points
 * only receive the long-range force, the pseudoparticles (eq. psep) only
 * exert it (petar_art_set.target_dev). Cells of zero mass (the massless
 * measure points and centres of the set) are skipped with their subtrees,
 * and particles of zero mass in the leaves reached are no sources: they
 * exert no force, so only the interaction counts change. The targets'
 * forces are those of an unrestricted call up to the rounding order of
 * their sums (a group's targets may be spread differently over the lanes,
 * and the skipped zero terms shift the others). NULL restores every
 * particle as a target; a new tree build does too. Neighbour lists cannot be asked for
 * while a subset is set (PETAR_E_INVALID). Errors: PETAR_E_STATE without a
 * tree. */
PETAR_API petar_status petar_set_targets(petar_ctx *ctx, const uint8_t *target_dev);

/* petar_force_long with the long-range kick of the KDK cycle fused into its
 * output write (eq. lfmap): additionally vel_dev[3][N] (input order) +=
 * dt * acc, rounded as v + (a dt) in FP64; dt (the half step) finite.
 * On PETAR_E_NB_OVERFLOW the kick has been applied with the complete acc:
 * retry the neighbour lists with petar_force_long, not with this call. */
PETAR_API petar_status petar_force_long_kick(petar_ctx *ctx, int group_size,
                                             const double *r_in_dev, const double *r_out_dev,
                                             const double *r_search_dev, double *acc_dev,
                                             double *pot_dev, petar_nblist *nb, double *vel_dev,
                                             double dt);

/* One evaluation of the long-range force of the P3T kick (eq. cf,
 * eq. Wij; step iv of the integration cycle of Sec. "Hybrid N-body code":
 * the tree is built anew for every long-range force) -- tree build (petar_tree_build when
 * n_sys == 0, else petar_batch_build with sys_offsets[n_sys + 1] and
 * N = sys_offsets[n_sys]) followed by petar_force_long -- executed as a
 * captured hipGraph. The first call (and any call whose pointers, sizes,
 * offsets or parameters differ from the captured ones) runs eagerly and
 * captures the launches on a private stream; later calls replay the graph
 * on the context's stream with one status read at the end. Buffer contents
 * may change between calls. The graph holds cells for twice the tree of the
 * capturing call; a tree that outgrows it is redone eagerly and recaptured
 * on the next call. Results and errors are those of the two eager calls. */
PETAR_API petar_status petar_step_graph(petar_ctx *ctx, int n_sys, const int64_t *sys_offsets,
                                        const double *pos_dev, const double *mass_dev, int64_t N,
                                        double theta, int leaf_size, int group_size,
                                        const double *r_in_dev, const double *r_out_dev,
                                        const double *r_search_dev, double *acc_dev,
                                        double *pot_dev, petar_nblist *nb);

/* Per-particle interaction counts of the last force call (input order),
 * counts_dev[4][N] int32: multipole cells, far-leaf particles, near-leaf
 * particles (including the particle itself) and the size of its i-group.
 * Requires params.record_counts = 1 before the force call. */
PETAR_API petar_status petar_copy_counts(petar_ctx *ctx, int32_t *counts_dev);

PETAR_API petar_status petar_get_stats(petar_ctx *ctx, petar_stats *stats);

/* Tree/walk parameters picked by petar_autotune. */
typedef struct {
    int leaf_size;   /* for petar_tree_build                     */
    int group_size;  /* for petar_force_long                     */
    int i_per_lane;  /* also stored into the context's params    */
    double ms;       /* measured build + force time (device ms)  */
} petar_tuned;

/* Times one step -- tree build, long-range force and neighbour lists -- on
 * the given particles (same argument rules as petar_tree_build /
 * petar_force_long) for leaf sizes {4, 8, 16}, group sizes {32, 48, 64, 96,
 * 128, 192, 256} and 1 or 2 targets per lane (a warm-up step, then the
 * median device time of five), keeps the fastest, sets
 * params.i_per_lane to it and returns it in *out. With cache_path (host
 * string, may be NULL) results are read from / appended to a JSON-lines
 * file keyed by (floor(log2 N), theta, precision); a cache hit returns
 * without launching anything. The practice follows the paper's wall-clock
 * scans of its integrator parameters (Sec. "Performance on GPU-based
 * Desktop", the scan of the long step). Allocates its own scratch outputs.
 * Leaves the context holding a tree of some candidate: rebuild with the
 * returned leaf size. */
PETAR_API petar_status petar_autotune(petar_ctx *ctx, const double *pos_dev,
                                      const double *mass_dev, int64_t N, double theta,
                                      const double *r_in_dev, const double *r_out_dev,
                                      const double *r_search_dev, const char *cache_path,
                                      petar_tuned *out);

/* petar_autotune for a batch of independent systems, the forest of
 * petar_batch_build (n_sys >= 1 systems; sys_offsets[n_sys + 1] host array,
 * same rules; N = sys_offsets[n_sys] particles in pos_dev[3][N],
 * mass_dev[N] and the radii [N]): times the batched step (petar_batch_build
 * + petar_force_long with neighbour lists) for the same candidates and
 * keeps the fastest, as petar_autotune does. Cache entries of batches also
 * carry floor(log2 n_sys) (a single system is the batch of one, bucket 0),
 * so batched and single-system choices for one N do not mix. The batching
 * of uneven systems into one launch is this library's (the paper integrates
 * one system per run); the practice of scanning wall-clock time over
 * parameters is the paper's (Sec. "Performance on GPU-based Desktop"). */
PETAR_API petar_status petar_autotune_batch(petar_ctx *ctx, int n_sys,
                                            const int64_t *sys_offsets, const double *pos_dev,
                                            const double *mass_dev, double theta,
                                            const double *r_in_dev, const double *r_out_dev,
                                            const double *r_search_dev, const char *cache_path,
                                            petar_tuned *out);

/* The parameters petar_autotune stored in cache_path (host string) for
 * (floor(log2 N_hint), theta, params.precision of ctx), without particles
 * and without launching anything (also on a PETAR_NO_DEVICE context).
 * Returns PETAR_E_STATE when the cache holds no such entry (or cannot be
 * read), PETAR_E_INVALID for N_hint < 1, theta < 0 or a NULL pointer. */
PETAR_API petar_status petar_autotune_lookup(petar_ctx *ctx, int64_t N_hint, double theta,
                                             const char *cache_path, petar_tuned *out);

/* The same for a batch: the parameters petar_autotune_batch stored for
 * (floor(log2 N_hint), floor(log2 n_sys), theta, params.precision);
 * n_sys = 1 reads the single-system entries. Errors as for
 * petar_autotune_lookup, PETAR_E_INVALID also for n_sys < 1. */
PETAR_API petar_status petar_autotune_lookup_batch(petar_ctx *ctx, int64_t N_hint, int n_sys,
                                                   double theta, const char *cache_path,
                                                   petar_tuned *out);

/* Second stage of the neighbour search (Sec. "Orbit-dependent neighbour
 * criterion"): keeps a first-stage candidate j of particle i iff the
 * pericentre separation of the pair's two-body Kepler orbit,
 * r_p = h^2 / (mu (1 + e)) with mu = G (m_i + m_j), specific energy
 * v^2/2 - mu/r, angular momentum h = |r x v| and e = sqrt(1 + 2 E h^2/mu^2),
 * is below c_v * r_nb_dev[i] (FP64; the whole orbit, whatever its phase;
 * 0 for coincident particles, |r x v|/|v| for two massless ones). G is the
 * context's params.G.
 * Inputs (device, input order): pos_dev[3][N], vel_dev[3][N], mass_dev[N],
 * r_nb_dev[N] (the first-stage search radii, eq. rnb), and the candidate
 * CSR cand_offsets_dev[N + 1] / cand_idx_dev (e.g. the lists of
 * petar_force_long); c_v > 0 (the paper uses 1.5). Output: out->offsets_dev
 * [N + 1] and out->idx_dev (capacity out->capacity) with the kept entries in
 * list order (sorted lists stay sorted); out->required = total kept. Errors:
 * PETAR_E_INVALID for bad arguments, candidate offsets that do not start at
 * 0 or decrease, or a candidate index outside [0, N),
 * PETAR_E_NB_OVERFLOW (offsets complete, idx not written) when the capacity
 * is too small. The context's tree is not used or changed. */
PETAR_API petar_status petar_nb_filter(petar_ctx *ctx, int64_t N, const double *pos_dev,
                                       const double *vel_dev, const double *mass_dev,
                                       const double *r_nb_dev, double c_v,
                                       const int64_t *cand_offsets_dev,
                                       const int32_t *cand_idx_dev, petar_nblist *out);

/* Clusters (Sec. "Clustering"): connected components of the neighbour
 * graph given as a CSR (nb_offsets_dev[N + 1], nb_idx_dev, each pair taken
 * in both directions), so that every member of a cluster has all its
 * neighbours in the same cluster. Outputs (device, caller-owned):
 * label_dev[N] = smallest particle index of the particle's cluster;
 * cl_offsets_dev[N + 1] and members_dev[N] list the clusters by label with
 * members ascending (entries past n_clusters of cl_offsets_dev equal N);
 * *n_clusters (host) = number of clusters. Deterministic. Errors:
 * PETAR_E_INVALID for bad arguments, offsets that do not start at 0 or
 * decrease, or an index outside [0, N). */
PETAR_API petar_status petar_clusters(petar_ctx *ctx, int64_t N, const int64_t *nb_offsets_dev,
                                      const int32_t *nb_idx_dev, int32_t *label_dev,
                                      int64_t *cl_offsets_dev, int32_t *members_dev,
                                      int64_t *n_clusters);

/* petar_clusters for callers that cannot allocate device memory (code under
 * stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, with the scratch
 * taken from a fixed array of 40 MiB that every device the library runs on
 * holds from its first petar_create on that device until the process ends.
 * No hipMalloc, hipFree or other allocation is made by the call.
 * N <= 1048576 (2^20); a larger N returns PETAR_E_INVALID (use
 * petar_clusters). All calls on one device share its array, which keeps the
 * last call's contents: calls that overlap on one device (other streams,
 * other contexts, other host threads) race and must be serialised by the
 * caller. Returns after the same status read as petar_clusters. */
PETAR_API petar_status petar_clusters_noalloc(petar_ctx *ctx, int64_t N,
                                              const int64_t *nb_offsets_dev,
                                              const int32_t *nb_idx_dev, int32_t *label_dev,
                                              int64_t *cl_offsets_dev, int32_t *members_dev,
                                              int64_t *n_clusters);

/* SDAR groups (Sec. "SDAR", eq. rbin): connected components of the pairs
 * with r_ij < theta r_in,ij, r_in,ij = max(r_in,i, r_in,j) (FP64, tested
 * as d^2 < (theta r_in,ij)^2), among the candidate CSR cand_offsets_dev
 * [N + 1] / cand_idx_dev (the lists of petar_force_long hold every pair
 * closer than max(r_search) >= r_out > r_in, so none is missed for
 * theta <= 1). Outputs as petar_clusters: label_dev[N] (smallest member
 * index), grp_offsets_dev[N + 1], members_dev[N], *n_groups; and the
 * binaries: the groups of exactly two members with negative Kepler energy
 * v^2/2 - G (m_i + m_j)/r (G = params.G), smaller index first, in group
 * order, written to pairs_dev[0 .. n_pairs) and pairs_dev[pair_cap ..
 * pair_cap + n_pairs) (pair_cap >= N/2), *n_pairs. Inputs pos_dev,
 * vel_dev [3][N], mass_dev, r_in_dev [N]; theta > 0. Groups of three or
 * more members get no binary entry. Errors as petar_clusters. */
PETAR_API petar_status petar_groups(petar_ctx *ctx, int64_t N, const double *pos_dev,
                                    const double *vel_dev, const double *mass_dev,
                                    const double *r_in_dev, double theta,
                                    const int64_t *cand_offsets_dev, const int32_t *cand_idx_dev,
                                    int32_t *label_dev, int64_t *grp_offsets_dev,
                                    int32_t *members_dev, int64_t *n_groups, int32_t *pairs_dev,
                                    int64_t pair_cap, int64_t *n_pairs);

/* Long-range kick of the KDK cycle (eq. lfmap): vel_dev[3][N] += dt *
 * acc_dev[3][N] (dt the half step), FP64 without contraction. */
PETAR_API petar_status petar_kick(petar_ctx *ctx, int64_t N, double *vel_dev,
                                  const double *acc_dev, double dt);

/* ---- Artificial particles (Sec. "Artificial particle algorithm for weak
 * perturbation"). A bound pair that the short-range integrator treats as a
 * group leaves the long-range set; in its place come its centre of mass
 * and the P measure points of the tidal tensor (zero mass; P = 4 at the
 * corners of a regular tetrahedron for order 2, 8 for order 3, the offsets
 * d_c u_p of Table A) and the three pseudoparticles of eq. psep (mass
 * (m1 + m2)/3 each, carrying the pair's orbit-averaged quadrupole, eq.
 * avebinquad). The set goes through petar_tree_build / petar_force_long
 * like any other particles; petar_tidal_fit then turns the field at the
 * centre and at the measure points into the tensor of eq. tt (the
 * generalized inverse of eq. map) and evaluates it at the members. */

/* Output set of petar_artificial_make (caller-owned device buffers). */
typedef struct {
    double *pos_dev;      /* [3][n_out]                                          */
    double *mass_dev;     /* [n_out]                                             */
    double *r_in_dev;     /* [n_out]                                             */
    double *r_out_dev;    /* [n_out]                                             */
    double *r_search_dev; /* [n_out]                                             */
    int32_t *src_dev;     /* [n_out]: input index of a single, -1 if artificial  */
    int64_t n_out;        /* must equal N + n_pair (P + 2)                       */
    uint8_t *target_dev;  /* [n_out] or NULL: 1 for the particles whose long-range */
                          /* force is used (singles, centres, measure points), 0 */
                          /* for pseudoparticles (sources only); for             */
                          /* petar_set_targets                                   */
} petar_art_set;

/* Builds the set: the N - 2 n_pair singles first, in input order, then for
 * pair b (pairs_dev[2][n_pair], int32 input indices i = pairs[b], j =
 * pairs[n_pair + b]) the block at n_single + b (P + 4): centre of mass,
 * the P measure points at r_cm + d_c u_p, the three pseudoparticles
 * (eq. psep rotated into the orbit's frame: x to the pericentre, z along
 * the angular momentum; x along the separation for a circular orbit; a
 * radial orbit as e = 1). Every artificial particle takes the larger of
 * the members' r_in, r_out and r_search. d_c = c_d a (1 + e) from the
 * pair's Kepler orbit with G = params.G. Inputs: pos_dev, vel_dev [3][N],
 * mass_dev and radii [N] (input order); order 2 or 3; c_d > 0. Outputs:
 * *set, frame_dev[4][n_pair] = (r_cm, d_c), and pair_of_dev[N] (may be
 * NULL) = the pair of a member, -1 for a single. Errors: PETAR_E_INVALID
 * for bad arguments, an index outside [0, N), i == j, a particle in two
 * pairs, or a pair that is not bound (specific energy >= 0); the outputs
 * are then undefined. */
PETAR_API petar_status petar_artificial_make(petar_ctx *ctx, int64_t N, const double *pos_dev,
                                             const double *vel_dev, const double *mass_dev,
                                             const double *r_in_dev, const double *r_out_dev,
                                             const double *r_search_dev, int64_t n_pair,
                                             const int32_t *pairs_dev, int order, double c_d,
                                             petar_art_set *set, double *frame_dev,
                                             int32_t *pair_of_dev);

/* Post-fit after the long-range force on the set: acc_set_dev[3][n_out]
 * and pot_set_dev[n_out] (may be NULL) are the outputs of petar_force_long
 * for the set of petar_artificial_make (its blocks at n_out - n_pair (P + 4)
 * onwards). Writes per pair the record tensor_dev[4 + K][n_pair] = phi(r_cm),
 * A(r_cm) (3), then the K = 6 (order 2: xx xy xz yy yz zz) or 16 (order 3:
 * also xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz) coefficients of Table A, the
 * least-squares solution of eq. map for the field differences at the
 * measure points (the third-order coefficients include the 1/2 of eq. tt).
 * With acc_dev[3][N] (may be NULL) also the long-range field of every input
 * particle: singles copy theirs from the set (through set->src_dev), the
 * members of pair b take the fitted field at their position pos_dev[3][N];
 * pot_dev[N] (needs pot_set_dev) likewise, members from the model potential
 * phi(r_cm) - r'.(A(r_cm) + a1/2 + a2/3), a1 and a2 the first- and second-
 * order parts of the fitted field at r' = r - r_cm. */
PETAR_API petar_status petar_tidal_fit(petar_ctx *ctx, int order, int64_t N, const double *pos_dev,
                                       int64_t n_pair, const int32_t *pairs_dev,
                                       const double *frame_dev, int64_t n_out,
                                       const int32_t *src_dev, const double *acc_set_dev,
                                       const double *pot_set_dev, double *tensor_dev,
                                       double *acc_dev, double *pot_dev);

/* Fitted field (and potential, pot_dev may be NULL) at n_pt points
 * pos_dev[3][n_pt], point k taking the tensor of pair pair_of_dev[k]
 * (points with pair_of < 0 are left untouched), e.g. the members along
 * their orbits between two long-range steps. Errors: PETAR_E_INVALID for
 * bad arguments or a pair_of >= n_pair. */
PETAR_API petar_status petar_tidal_eval(petar_ctx *ctx, int order, int64_t n_pair,
                                        const double *tensor_dev, const double *frame_dev,
                                        int64_t n_pt, const int32_t *pair_of_dev,
                                        const double *pos_dev, double *acc_dev, double *pot_dev);

/* Message of the last failure on ctx (thread-local message if ctx is NULL). */
PETAR_API const char *petar_last_error(petar_ctx *ctx);
PETAR_API const char *petar_status_string(petar_status status);

#ifdef __cplusplus
}
#endif

#endif /* PETAR_H */
