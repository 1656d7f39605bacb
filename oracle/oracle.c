/*
 * FP64 CPU oracle for the long-range (tree) part of the P3T force split of
 * PeTar (Wang, Iwasawa, Nitadori & Makino 2020).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code, header, table or
 * helper with the GPU library.
 *
 * Everything is plain, slow and written to be checked against the paper by
 * eye: FP64 throughout, no blocking, no fusion, OpenMP only over the
 * independent target particles. Build with -ffp-contract=off so the
 * neighbour distance test rounds exactly as written.
 *
 * Contents
 *   1. Changeover functions f, W, K  (Sec. "Mass-dependent changeover
 *      function": definitions of f, W and the force weight, eq. Wij).
 *   2. Changeover radii (eq. rcut) and neighbour search radius (eq. rnb).
 *   3. Direct sums: long-range (H_L of eq. cf), short-range (H_S), Newton.
 *   4. Neighbour candidates (Sec. "Orbit-dependent neighbour criterion",
 *      stage 1: spherical search), pair radius max(r_s,i, r_s,j).
 *   5. Multipole of a particle set: monopole + traceless quadrupole
 *      (eq. quad, eq. quadtr) and its field.
 *   6. Barnes-Hut tree force (Sec. "Particle-tree with individual time
 *      steps" and the P3T figure caption: cells inside the opening angle are
 *      replaced by centre-of-mass + quadrupole super-particles), group-wise
 *      walk with the search-radius opening rule.
 *   7. Second-stage neighbour filter (Kepler pericentre, Sec. "Orbit-
 *      dependent neighbour criterion") and clusters (Sec. "Clustering").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------
 * 1. Changeover functions (literal forms of the paper).
 *    x = (r - r_in,ij)/(r_out,ij - r_in,ij),
 *    Lambda = (r_out,ij - r_in,ij)/(r_out,ij + r_in,ij).
 * ---------------------------------------------------------------------- */

/* f(x) = 1 + Lambda x^5 (14 - 28x + 20x^2 - 5x^3) */
OR_EXPORT double oracle_f(double x, double lam)
{
    double x2 = x * x;
    double x5 = x2 * x2 * x;
    return 1.0 + lam * x5 * (14.0 - 28.0 * x + 20.0 * x2 - 5.0 * x2 * x);
}

/* Potential weight W(x): Lambda(1-2x) for x <= 0, Lambda(1-2x) - 1 + f(x)
 * inside, 0 for x >= 1. */
OR_EXPORT double oracle_W(double x, double lam)
{
    if (x <= 0.0) return lam * (1.0 - 2.0 * x);
    if (x >= 1.0) return 0.0;
    return lam * (1.0 - 2.0 * x) - 1.0 + oracle_f(x, lam);
}

/* Force weight K(x) (eq. Wij): 1 for x <= 0,
 * (x-1)^4 (1 + 4x + 10x^2 + 20x^3 + 35 Lambda x^4) inside, 0 for x >= 1. */
OR_EXPORT double oracle_K(double x, double lam)
{
    if (x <= 0.0) return 1.0;
    if (x >= 1.0) return 0.0;
    double xm = x - 1.0;
    double xm4 = xm * xm * xm * xm;
    double x2 = x * x;
    return xm4 * (1.0 + 4.0 * x + 10.0 * x2 + 20.0 * x2 * x + 35.0 * lam * x2 * x2);
}

/* Pair changeover radii: r_in,ij = max(r_in,i, r_in,j), same for r_out. */
static void pair_radii(double rin_i, double rout_i, double rin_j, double rout_j,
                       double *rin, double *rout)
{
    *rin = rin_i > rin_j ? rin_i : rin_j;
    *rout = rout_i > rout_j ? rout_i : rout_j;
}

/* Long-range weights of one pair at distance r (> 0 or == 0):
 *   fw = 1 - K(x)            (force:  a += G m fw (r_j - r_i)/r^3)
 *   pw = (1 - W(x)) / r      (potential: phi -= G m pw)
 * At r == 0 the x <= 0 branch holds and (1 - W)/r is its limit
 * 2/(r_in + r_out) (the literal form is 0/0 there). */
static void long_weights(double r, double rin, double rout, double *fw, double *pw)
{
    double lam = (rout - rin) / (rout + rin);
    double x = (r - rin) / (rout - rin);
    *fw = 1.0 - oracle_K(x, lam);
    if (r > 0.0)
        *pw = (1.0 - oracle_W(x, lam)) / r;
    else
        *pw = 2.0 / (rin + rout);
}

/* ------------------------------------------------------------------------
 * 2. Radii. eq. rcut: r_in,i = max(1, m_i/<m>)^(1/3) r_in,ref, same for
 *    r_out; <m> = (sum m)/N. Search radius: search_factor * r_out,i, or
 *    eq. rnb r_out,i + C_r |v_i| dt_L when velocities are given
 *    (cr_dt = C_r * dt_L). Returns 0, or -1 on invalid arguments.
 * ---------------------------------------------------------------------- */
OR_EXPORT int oracle_radii(const double *mass, const double *vel, int64_t n,
                           double rin_ref, double rout_ref, double search_factor,
                           double cr_dt, double *r_in, double *r_out, double *r_search)
{
    if (n < 1 || !(rin_ref >= 0.0) || !(rout_ref > rin_ref)) return -1;
    double msum = 0.0;
    for (int64_t i = 0; i < n; i++) msum += mass[i];
    double mave = msum / (double)n;
    for (int64_t i = 0; i < n; i++) {
        double ratio = mave > 0.0 ? mass[i] / mave : 1.0;
        double s = cbrt(ratio > 1.0 ? ratio : 1.0);
        r_in[i] = s * rin_ref;
        r_out[i] = s * rout_ref;
        if (vel) {
            double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
            r_search[i] = r_out[i] + cr_dt * sqrt(vx * vx + vy * vy + vz * vz);
        } else {
            r_search[i] = search_factor * r_out[i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * 3. Direct sums over all j != i, for the target indices idx[0..n_idx).
 *    pos is SoA [3][n]; acc is SoA [3][n_idx]; pot is [n_idx].
 * ---------------------------------------------------------------------- */
OR_EXPORT void oracle_force_long(const double *pos, const double *mass, const double *r_in,
                                 const double *r_out, int64_t n, double G, const int64_t *idx,
                                 int64_t n_idx, double *acc, double *pot)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_idx; k++) {
        int64_t i = idx ? idx[k] : k;
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double rin, rout, fw, pw;
            pair_radii(r_in[i], r_out[i], r_in[j], r_out[j], &rin, &rout);
            long_weights(r, rin, rout, &fw, &pw);
            if (fw != 0.0) {
                double s = G * mass[j] * fw / (r * r * r);
                ax += s * dx;
                ay += s * dy;
                az += s * dz;
            }
            ph -= G * mass[j] * pw;
        }
        acc[k] = ax;
        acc[n_idx + k] = ay;
        acc[2 * n_idx + k] = az;
        pot[k] = ph;
    }
}

/* Short-range companion (H_S of eq. cf): weights K(x) for the force and
 * W(x)/r for the potential. Singular at r == 0 (callers avoid it). */
OR_EXPORT void oracle_force_short(const double *pos, const double *mass, const double *r_in,
                                  const double *r_out, int64_t n, double G, const int64_t *idx,
                                  int64_t n_idx, double *acc, double *pot)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_idx; k++) {
        int64_t i = idx ? idx[k] : k;
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double rin, rout;
            pair_radii(r_in[i], r_out[i], r_in[j], r_out[j], &rin, &rout);
            double lam = (rout - rin) / (rout + rin);
            double x = (r - rin) / (rout - rin);
            double s = G * mass[j] * oracle_K(x, lam) / (r * r * r);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
            ph -= G * mass[j] * oracle_W(x, lam) / r;
        }
        acc[k] = ax;
        acc[n_idx + k] = ay;
        acc[2 * n_idx + k] = az;
        pot[k] = ph;
    }
}

/* Plain Newtonian direct sum (no changeover). */
OR_EXPORT void oracle_force_newton(const double *pos, const double *mass, int64_t n, double G,
                                   const int64_t *idx, int64_t n_idx, double *acc, double *pot)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_idx; k++) {
        int64_t i = idx ? idx[k] : k;
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double s = G * mass[j] / (r * r * r);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
            ph -= G * mass[j] / r;
        }
        acc[k] = ax;
        acc[n_idx + k] = ay;
        acc[2 * n_idx + k] = az;
        pot[k] = ph;
    }
}

/* ------------------------------------------------------------------------
 * 4. Neighbour candidates: j != i with d^2 < R^2, R = max(r_s,i, r_s,j),
 *    d^2 = ((dx*dx) + (dy*dy)) + (dz*dz), dx = x_j - x_i, each operation
 *    rounded (no contraction). Lists come out in ascending j.
 *    counts[k] receives the count of target k. If out != NULL, the lists
 *    are written back to back (capacity entries at most). Returns the total.
 * ---------------------------------------------------------------------- */
static int is_neighbour(const double *X, const double *Y, const double *Z, const double *rs,
                        int64_t i, int64_t j)
{
    double dx = X[j] - X[i];
    double dy = Y[j] - Y[i];
    double dz = Z[j] - Z[i];
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double d2 = xx + yy;
    d2 = d2 + zz;
    double R = rs[i] > rs[j] ? rs[i] : rs[j];
    double R2 = R * R;
    return d2 < R2;
}

OR_EXPORT int64_t oracle_neighbours(const double *pos, const double *r_search, int64_t n,
                                    const int64_t *idx, int64_t n_idx, int64_t *counts,
                                    int32_t *out, int64_t capacity)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_idx; k++) {
        int64_t i = idx ? idx[k] : k;
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++)
            if (j != i && is_neighbour(X, Y, Z, r_search, i, j)) c++;
        counts[k] = c;
    }
    int64_t total = 0;
    for (int64_t k = 0; k < n_idx; k++) total += counts[k];
    if (out && total <= capacity) {
        int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_idx + 1));
        start[0] = 0;
        for (int64_t k = 0; k < n_idx; k++) start[k + 1] = start[k] + counts[k];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < n_idx; k++) {
            int64_t i = idx ? idx[k] : k;
            int64_t w = start[k];
            for (int64_t j = 0; j < n; j++)
                if (j != i && is_neighbour(X, Y, Z, r_search, i, j)) out[w++] = (int32_t)j;
        }
        free(start);
    }
    return total;
}

/* ------------------------------------------------------------------------
 * 5. Multipole of a particle set about its centre of mass c:
 *    M = sum m, A' = (3/2) sum m q q^T - (1/2) (sum m |q|^2) I, q = x - c
 *    (eq. quad, eq. quadtr; the trace term multiplies the identity).
 *    quad6 = (A'xx, A'yy, A'zz, A'xy, A'xz, A'yz).
 *    Field at R = p - c (attracting):
 *      phi = -G (M/|R| + R.A'R/|R|^5)
 *      a   = G (-M R/|R|^3 + 2 A'R/|R|^5 - 5 (R.A'R) R/|R|^7)   (a = -grad phi)
 * ---------------------------------------------------------------------- */
static void moments(const double *X, const double *Y, const double *Z, const double *mass,
                    const int64_t *members, int64_t cnt, double *M, double com[3], double A[6])
{
    double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = 0; k < cnt; k++) {
        int64_t j = members[k];
        m += mass[j];
        sx += mass[j] * X[j];
        sy += mass[j] * Y[j];
        sz += mass[j] * Z[j];
        double p[3] = {X[j], Y[j], Z[j]};
        for (int d = 0; d < 3; d++) {
            if (p[d] < lo[d]) lo[d] = p[d];
            if (p[d] > hi[d]) hi[d] = p[d];
        }
    }
    *M = m;
    if (m > 0.0) {
        com[0] = sx / m;
        com[1] = sy / m;
        com[2] = sz / m;
    } else { /* massless set: use the centre of its bounding box */
        for (int d = 0; d < 3; d++) com[d] = 0.5 * (lo[d] + hi[d]);
    }
    double axx = 0, ayy = 0, azz = 0, axy = 0, axz = 0, ayz = 0, q2 = 0;
    for (int64_t k = 0; k < cnt; k++) {
        int64_t j = members[k];
        double qx = X[j] - com[0], qy = Y[j] - com[1], qz = Z[j] - com[2];
        axx += mass[j] * qx * qx;
        ayy += mass[j] * qy * qy;
        azz += mass[j] * qz * qz;
        axy += mass[j] * qx * qy;
        axz += mass[j] * qx * qz;
        ayz += mass[j] * qy * qz;
        q2 += mass[j] * (qx * qx + qy * qy + qz * qz);
    }
    A[0] = 1.5 * axx - 0.5 * q2;
    A[1] = 1.5 * ayy - 0.5 * q2;
    A[2] = 1.5 * azz - 0.5 * q2;
    A[3] = 1.5 * axy;
    A[4] = 1.5 * axz;
    A[5] = 1.5 * ayz;
}

static void multipole_field(double M, const double c[3], const double A[6], double G,
                            double px, double py, double pz, double *a, double *phi)
{
    double Rx = px - c[0], Ry = py - c[1], Rz = pz - c[2];
    double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    double r = sqrt(r2);
    double ARx = A[0] * Rx + A[3] * Ry + A[4] * Rz;
    double ARy = A[3] * Rx + A[1] * Ry + A[5] * Rz;
    double ARz = A[4] * Rx + A[5] * Ry + A[2] * Rz;
    double RAR = Rx * ARx + Ry * ARy + Rz * ARz;
    double r3 = r2 * r, r5 = r3 * r2, r7 = r5 * r2;
    a[0] += G * (-M * Rx / r3 + 2.0 * ARx / r5 - 5.0 * RAR * Rx / r7);
    a[1] += G * (-M * Ry / r3 + 2.0 * ARy / r5 - 5.0 * RAR * Ry / r7);
    a[2] += G * (-M * Rz / r3 + 2.0 * ARz / r5 - 5.0 * RAR * Rz / r7);
    *phi -= G * (M / r + RAR / r5);
}

OR_EXPORT void oracle_multipole(const double *pos, const double *mass, int64_t n, double *M,
                                double *com, double *quad6)
{
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < n; k++) all[k] = k;
    moments(pos, pos + n, pos + 2 * n, mass, all, n, M, com, quad6);
    free(all);
}

/* Field of (M, com, quad6) at npts points (SoA [3][npts]). */
OR_EXPORT void oracle_multipole_eval(double M, const double *com, const double *quad6, double G,
                                     const double *pts, int64_t npts, double *acc, double *pot)
{
    for (int64_t k = 0; k < npts; k++) {
        double a[3] = {0, 0, 0}, ph = 0.0;
        multipole_field(M, com, quad6, G, pts[k], pts[npts + k], pts[2 * npts + k], a, &ph);
        acc[k] = a[0];
        acc[npts + k] = a[1];
        acc[2 * npts + k] = a[2];
        pot[k] = ph;
    }
}

/* ------------------------------------------------------------------------
 * 6. Barnes-Hut tree force with group-wise walk.
 *
 *  Root cube: lo_d = min x_d, ext = max_d (max x_d - min x_d) (1 if 0).
 *  Integer coordinate per axis: q = floor((x - lo) * (2^L/ext)), clamped
 *  to 2^L - 1, with L = max_level (21 by default). A cell at level l holds
 *  the particles sharing the top l bits of all three q; its side is
 *  ext / 2^l. A cell with <= leaf_size particles, or at level L, is a leaf;
 *  otherwise its non-empty octants are children.
 *  Cell data: mass, centre of mass, A' (section 5), particle bounding box,
 *  max r_search of its members.
 *  i-groups: the first cells on each root-to-leaf path that hold
 *  <= group_size particles or are leaves.
 *  Walk of group g (members' bounding box B_g, max r_search S_g), per cell:
 *    D2   = squared distance between B_g and the cell's bounding box
 *    dmin2= squared distance from B_g to the cell's centre of mass
 *    R    = max(S_g, cell max r_search)
 *    multipole  iff side^2 < theta^2 * dmin2  and not (D2 < R^2)
 *    otherwise a leaf is "near" (pairs with changeover weights) if
 *    D2 < R^2, "far" (plain Newtonian pairs) if not; an internal cell opens.
 *  Since r_search >= r_out, every pair reached through a multipole or a far
 *  leaf has x >= 1, where K = W = 0: the long-range force there is plain
 *  Newtonian and the expansion is exact in form.
 *  With skip_massless (a force on a subset of targets), a cell of zero mass
 *  is dropped with its subtree before the tests, and a particle of zero mass
 *  in a far or near leaf is not a source: its multipole and every pair term
 *  with such a particle are zero, so no value changes, only the interaction
 *  counts.
 * ---------------------------------------------------------------------- */

#define OR_MAXLEVEL 21 /* default depth: 21 bits per axis */

typedef struct {
    int64_t begin, count; /* range in the member permutation */
    int level;
    int leaf;
    int64_t child[8];
    int nchild;
    double M, com[3], A[6], lo[3], hi[3], rsmax;
} ocell;

typedef struct {
    ocell *c;
    int64_t n, cap;
} ocells;

static int64_t push_cell(ocells *cs)
{
    if (cs->n == cs->cap) {
        cs->cap = cs->cap ? 2 * cs->cap : 1024;
        cs->c = (ocell *)realloc(cs->c, sizeof(ocell) * (size_t)cs->cap);
    }
    memset(&cs->c[cs->n], 0, sizeof(ocell));
    return cs->n++;
}

typedef struct {
    const double *X, *Y, *Z, *mass, *rs;
    const uint32_t *q; /* [3][n] integer coordinates */
    int64_t n;
    int leaf_size;
    int max_level; /* levels below the root (bits per axis) */
    int64_t *perm, *tmp;
    ocells cells;
} obuild;

static int octant(const obuild *b, int64_t j, int level)
{
    int shift = b->max_level - 1 - level; /* bit of the child level */
    int bx = (b->q[j] >> shift) & 1;
    int by = (b->q[b->n + j] >> shift) & 1;
    int bz = (b->q[2 * b->n + j] >> shift) & 1;
    return (bx << 2) | (by << 1) | bz;
}

static int64_t build_cell(obuild *b, int64_t begin, int64_t count, int level)
{
    int64_t id = push_cell(&b->cells);
    ocell *c = &b->cells.c[id];
    c->begin = begin;
    c->count = count;
    c->level = level;
    c->leaf = (count <= b->leaf_size || level == b->max_level);
    if (c->leaf) return id;
    /* stable partition of the range by child octant */
    int64_t cnt[8] = {0}, off[8];
    for (int64_t k = begin; k < begin + count; k++) cnt[octant(b, b->perm[k], level)]++;
    off[0] = begin;
    for (int o = 1; o < 8; o++) off[o] = off[o - 1] + cnt[o - 1];
    int64_t w[8];
    memcpy(w, off, sizeof(w));
    for (int64_t k = begin; k < begin + count; k++) {
        int64_t j = b->perm[k];
        b->tmp[w[octant(b, j, level)]++] = j;
    }
    memcpy(b->perm + begin, b->tmp + begin, sizeof(int64_t) * (size_t)count);
    int64_t kids[8];
    int nk = 0;
    for (int o = 0; o < 8; o++)
        if (cnt[o]) kids[nk++] = build_cell(b, off[o], cnt[o], level + 1);
    c = &b->cells.c[id]; /* the array may have moved */
    c->nchild = nk;
    for (int o = 0; o < nk; o++) c->child[o] = kids[o];
    return id;
}

static double box_dist2(const double alo[3], const double ahi[3], const double blo[3],
                        const double bhi[3])
{
    double g[3];
    for (int d = 0; d < 3; d++) {
        double t1 = blo[d] - ahi[d];
        double t2 = alo[d] - bhi[d];
        double t = t1 > t2 ? t1 : t2;
        g[d] = t > 0.0 ? t : 0.0;
    }
    double gx = g[0] * g[0];
    double gy = g[1] * g[1];
    double gz = g[2] * g[2];
    double s = gx + gy;
    return s + gz;
}

static double point_box_dist2(const double alo[3], const double ahi[3], const double p[3])
{
    double g[3];
    for (int d = 0; d < 3; d++) {
        double t1 = p[d] - ahi[d];
        double t2 = alo[d] - p[d];
        double t = t1 > t2 ? t1 : t2;
        g[d] = t > 0.0 ? t : 0.0;
    }
    double gx = g[0] * g[0];
    double gy = g[1] * g[1];
    double gz = g[2] * g[2];
    double s = gx + gy;
    return s + gz;
}

typedef struct {
    int64_t *pc, *far, *near; /* cell ids */
    int64_t npc, nfar, nnear, cap;
} olists;

/* Each cell enters a group's lists at most once, so lists sized to the
 * number of cells never overflow. */
static void lists_push(int64_t **a, int64_t *na, int64_t v) { (*a)[(*na)++] = v; }

static void walk(const ocells *cs, int64_t cid, const ocell *g, double th2, double ext,
                 int skip_massless, olists *L)
{
    const ocell *c = &cs->c[cid];
    if (skip_massless && c->M == 0.0) return;
    double D2 = box_dist2(g->lo, g->hi, c->lo, c->hi);
    double dmin2 = point_box_dist2(g->lo, g->hi, c->com);
    double R = g->rsmax > c->rsmax ? g->rsmax : c->rsmax;
    double R2 = R * R;
    double side = ldexp(ext, -c->level);
    double side2 = side * side;
    double rhs = th2 * dmin2;
    if (side2 < rhs && !(D2 < R2)) {
        lists_push(&L->pc, &L->npc, cid);
        return;
    }
    if (c->leaf) {
        if (D2 < R2)
            lists_push(&L->near, &L->nnear, cid);
        else
            lists_push(&L->far, &L->nfar, cid);
        return;
    }
    for (int k = 0; k < c->nchild; k++) walk(cs, c->child[k], g, th2, ext, skip_massless, L);
}

static void find_groups(const ocells *cs, int64_t cid, int group_size, int64_t *groups,
                        int64_t *ng)
{
    const ocell *c = &cs->c[cid];
    if (c->count <= group_size || c->leaf) {
        groups[(*ng)++] = cid;
        return;
    }
    for (int k = 0; k < c->nchild; k++) find_groups(cs, c->child[k], group_size, groups, ng);
}

/* Tree structure summary: info[0..5] = n_cells, n_leaves, n_groups,
 * max_level, max leaf count, sum over leaves of count (== n). */
static int build_tree(const double *pos, const double *mass, const double *r_search, int64_t n,
                      int leaf_size, int max_level, obuild *b, double *ext_out)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
    double lo[3] = {X[0], Y[0], Z[0]}, hi[3] = {X[0], Y[0], Z[0]};
    for (int64_t i = 1; i < n; i++) {
        double p[3] = {X[i], Y[i], Z[i]};
        for (int d = 0; d < 3; d++) {
            if (p[d] < lo[d]) lo[d] = p[d];
            if (p[d] > hi[d]) hi[d] = p[d];
        }
    }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    if (!(ext > 0.0)) ext = 1.0;
    const double cells_per_axis = ldexp(1.0, max_level); /* 2^max_level */
    const uint64_t qmax = ((uint64_t)1 << max_level) - 1;
    double scale = cells_per_axis / ext;
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    const double *P[3] = {X, Y, Z};
    for (int d = 0; d < 3; d++)
        for (int64_t i = 0; i < n; i++) {
            double t = (P[d][i] - lo[d]) * scale;
            uint64_t v = (uint64_t)t;
            if (v > qmax) v = qmax;
            q[(size_t)d * n + i] = (uint32_t)v;
        }
    memset(b, 0, sizeof(*b));
    b->X = X;
    b->Y = Y;
    b->Z = Z;
    b->mass = mass;
    b->rs = r_search;
    b->q = q;
    b->n = n;
    b->leaf_size = leaf_size;
    b->max_level = max_level;
    b->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    b->tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) b->perm[i] = i;
    build_cell(b, 0, n, 0);
    /* cell data straight from each cell's members */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < b->cells.n; k++) {
        ocell *c = &b->cells.c[k];
        const int64_t *mem = b->perm + c->begin;
        moments(X, Y, Z, mass, mem, c->count, &c->M, c->com, c->A);
        for (int d = 0; d < 3; d++) {
            c->lo[d] = INFINITY;
            c->hi[d] = -INFINITY;
        }
        c->rsmax = 0.0;
        for (int64_t t = 0; t < c->count; t++) {
            int64_t j = mem[t];
            double p[3] = {X[j], Y[j], Z[j]};
            for (int d = 0; d < 3; d++) {
                if (p[d] < c->lo[d]) c->lo[d] = p[d];
                if (p[d] > c->hi[d]) c->hi[d] = p[d];
            }
            if (r_search && r_search[j] > c->rsmax) c->rsmax = r_search[j];
        }
    }
    free(q);
    b->q = NULL;
    *ext_out = ext;
    return 0;
}

static void free_tree(obuild *b)
{
    free(b->perm);
    free(b->tmp);
    free(b->cells.c);
}

OR_EXPORT int oracle_tree_info(const double *pos, const double *mass, int64_t n, int leaf_size,
                               int group_size, int max_level, int64_t *info)
{
    if (n < 1 || leaf_size < 1 || group_size < 1 || max_level < 1 || max_level > 21) return -1;
    obuild b;
    double ext;
    build_tree(pos, mass, NULL, n, leaf_size, max_level, &b, &ext);
    int64_t nleaf = 0, maxlev = 0, maxleaf = 0, sumleaf = 0;
    for (int64_t k = 0; k < b.cells.n; k++) {
        ocell *c = &b.cells.c[k];
        if (c->level > maxlev) maxlev = c->level;
        if (c->leaf) {
            nleaf++;
            sumleaf += c->count;
            if (c->count > maxleaf) maxleaf = c->count;
        }
    }
    int64_t *groups = (int64_t *)malloc(sizeof(int64_t) * (size_t)b.cells.n);
    int64_t ng = 0;
    find_groups(&b.cells, 0, group_size, groups, &ng);
    info[0] = b.cells.n;
    info[1] = nleaf;
    info[2] = ng;
    info[3] = maxlev;
    info[4] = maxleaf;
    info[5] = sumleaf;
    free(groups);
    free_tree(&b);
    return 0;
}

/* Number of particles of leaf c that act as sources: all of them, or with
 * skip_massless those of non-zero mass. */
static int64_t source_count(const obuild *b, const ocell *c, const double *mass,
                            int skip_massless)
{
    if (!skip_massless) return c->count;
    int64_t k = 0;
    for (int64_t u = 0; u < c->count; u++) k += mass[b->perm[c->begin + u]] != 0.0;
    return k;
}

/* Tree force for the targets idx[0..n_idx) (all particles if idx == NULL).
 * acc SoA [3][n_idx], pot [n_idx]. counts (optional) SoA [4][n_idx]:
 * number of multipole cells, far-leaf particles and near-leaf particles in
 * the target's group lists, and the size of its group. skip_massless: drop
 * cells of zero mass from the walk and particles of zero mass from the leaf
 * lists (same values, fewer counted interactions). Returns 0 or -1. */
OR_EXPORT int oracle_tree_force(const double *pos, const double *mass, const double *r_in,
                                const double *r_out, const double *r_search, int64_t n,
                                double theta, int leaf_size, int group_size, int max_level,
                                double G, const int64_t *idx, int64_t n_idx, int skip_massless,
                                double *acc, double *pot, int64_t *counts)
{
    if (n < 1 || leaf_size < 1 || group_size < 1 || !(theta >= 0.0) || max_level < 1 ||
        max_level > 21)
        return -1;
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
    obuild b;
    double ext;
    build_tree(pos, mass, r_search, n, leaf_size, max_level, &b, &ext);
    int64_t *groups = (int64_t *)malloc(sizeof(int64_t) * (size_t)b.cells.n);
    int64_t ng = 0;
    find_groups(&b.cells, 0, group_size, groups, &ng);
    /* particle -> group, and target -> slot */
    int64_t *gof = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t g = 0; g < ng; g++) {
        ocell *c = &b.cells.c[groups[g]];
        for (int64_t t = 0; t < c->count; t++) gof[b.perm[c->begin + t]] = g;
    }
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) slot[i] = -1;
    char *gwant = (char *)calloc((size_t)ng, 1);
    for (int64_t k = 0; k < n_idx; k++) {
        int64_t i = idx ? idx[k] : k;
        slot[i] = k;
        gwant[gof[i]] = 1;
    }
    double th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ng; g++) {
        if (!gwant[g]) continue;
        const ocell *gc = &b.cells.c[groups[g]];
        olists L;
        L.cap = b.cells.n;
        L.pc = (int64_t *)malloc(sizeof(int64_t) * (size_t)L.cap);
        L.far = (int64_t *)malloc(sizeof(int64_t) * (size_t)L.cap);
        L.near = (int64_t *)malloc(sizeof(int64_t) * (size_t)L.cap);
        L.npc = L.nfar = L.nnear = 0;
        walk(&b.cells, 0, gc, th2, ext, skip_massless, &L);
        /* particles of the far and near leaves (with skip_massless, those
         * with mass) */
        int64_t nfarp = 0, nnearp = 0;
        for (int64_t t = 0; t < L.nfar; t++)
            nfarp += source_count(&b, &b.cells.c[L.far[t]], mass, skip_massless);
        for (int64_t t = 0; t < L.nnear; t++)
            nnearp += source_count(&b, &b.cells.c[L.near[t]], mass, skip_massless);
        for (int64_t m = 0; m < gc->count; m++) {
            int64_t i = b.perm[gc->begin + m];
            int64_t k = slot[i];
            if (k < 0) continue;
            double a[3] = {0, 0, 0}, ph = 0.0;
            /* multipole cells */
            for (int64_t t = 0; t < L.npc; t++) {
                const ocell *c = &b.cells.c[L.pc[t]];
                multipole_field(c->M, c->com, c->A, G, X[i], Y[i], Z[i], a, &ph);
            }
            /* far leaves: Newtonian pairs */
            for (int64_t t = 0; t < L.nfar; t++) {
                const ocell *c = &b.cells.c[L.far[t]];
                for (int64_t u = 0; u < c->count; u++) {
                    int64_t j = b.perm[c->begin + u];
                    if (skip_massless && mass[j] == 0.0) continue;
                    double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    double s = G * mass[j] / (r * r * r);
                    a[0] += s * dx;
                    a[1] += s * dy;
                    a[2] += s * dz;
                    ph -= G * mass[j] / r;
                }
            }
            /* near leaves: pairs with changeover weights */
            for (int64_t t = 0; t < L.nnear; t++) {
                const ocell *c = &b.cells.c[L.near[t]];
                for (int64_t u = 0; u < c->count; u++) {
                    int64_t j = b.perm[c->begin + u];
                    if (j == i || (skip_massless && mass[j] == 0.0)) continue;
                    double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    double rin, rout, fw, pw;
                    pair_radii(r_in[i], r_out[i], r_in[j], r_out[j], &rin, &rout);
                    long_weights(r, rin, rout, &fw, &pw);
                    if (fw != 0.0) {
                        double s = G * mass[j] * fw / (r * r * r);
                        a[0] += s * dx;
                        a[1] += s * dy;
                        a[2] += s * dz;
                    }
                    ph -= G * mass[j] * pw;
                }
            }
            acc[k] = a[0];
            acc[n_idx + k] = a[1];
            acc[2 * n_idx + k] = a[2];
            pot[k] = ph;
            if (counts) {
                counts[k] = L.npc;
                counts[n_idx + k] = nfarp;
                counts[2 * n_idx + k] = nnearp;
                counts[3 * n_idx + k] = gc->count;
            }
        }
        free(L.pc);
        free(L.far);
        free(L.near);
    }
    free(gwant);
    free(slot);
    free(gof);
    free(groups);
    free_tree(&b);
    return 0;
}

/* ------------------------------------------------------------------------
 * 7. Neighbours, second stage, and clusters (Sec. "Clustering" and
 *    "Orbit-dependent neighbour criterion").
 *
 *  Second stage: a first-stage candidate j of particle i is a true
 *  neighbour iff the pericentre separation of the two-body Kepler orbit of
 *  the pair is below C_v * r_nb,i, where r_nb,i is the first-stage search
 *  radius of i (eq. rnb). With r = x_j - x_i, v = v_j - v_i and
 *  mu = G (m_i + m_j):
 *    specific energy  eps = v^2/2 - mu/|r|
 *    angular momentum h   = |r x v|
 *    eccentricity     e   = sqrt(1 + 2 eps h^2 / mu^2)
 *    pericentre       r_p = h^2 / (mu (1 + e))     (any conic; e clamped at 0)
 *  taken over the whole orbit, whatever the current phase. Coincident
 *  particles have r_p = 0. Two massless particles move on straight lines:
 *  r_p = |r x v| / |v| (or |r| when v = 0).
 *
 *  Clusters: connected components of the graph whose edges are the true
 *  neighbour pairs (in either direction), so that every member has all its
 *  neighbours in its own cluster. A cluster is labelled by its smallest
 *  particle index; clusters are listed by label, members ascending.
 * ---------------------------------------------------------------------- */

OR_EXPORT double oracle_pericentre(const double xi[3], const double vi[3], double mi,
                                   const double xj[3], const double vj[3], double mj, double G)
{
    double dx = xj[0] - xi[0];
    double dy = xj[1] - xi[1];
    double dz = xj[2] - xi[2];
    double dvx = vj[0] - vi[0];
    double dvy = vj[1] - vi[1];
    double dvz = vj[2] - vi[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double v2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
    double hx = dy * dvz - dz * dvy;
    double hy = dz * dvx - dx * dvz;
    double hz = dx * dvy - dy * dvx;
    double h2 = (hx * hx + hy * hy) + hz * hz;
    double mu = G * (mi + mj);
    if (d2 == 0.0) return 0.0;
    if (mu > 0.0) {
        double d = sqrt(d2);
        double eps = 0.5 * v2 - mu / d;
        double e2 = 1.0 + ((2.0 * eps) * h2) / (mu * mu);
        double e = e2 > 0.0 ? sqrt(e2) : 0.0;
        return h2 / (mu * (1.0 + e));
    }
    return v2 > 0.0 ? sqrt(h2 / v2) : sqrt(d2);
}

/* Filters the CSR candidate lists (offsets [n+1], idx) into true
 * neighbours. counts[i] receives the kept count; out (capacity cap, may be
 * NULL) the kept indices in list order. Returns the total kept. pos, vel
 * are SoA [3][n]. */
OR_EXPORT int64_t oracle_nb_filter(const double *pos, const double *vel, const double *mass,
                                   const double *r_nb, int64_t n, double c_v, double G,
                                   const int64_t *offsets, const int32_t *idx, int64_t *counts,
                                   int32_t *out, int64_t cap)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++) {
        double xi[3] = {pos[i], pos[n + i], pos[2 * n + i]};
        double vi[3] = {vel[i], vel[n + i], vel[2 * n + i]};
        double lim = c_v * r_nb[i];
        int64_t c = 0;
        for (int64_t e = offsets[i]; e < offsets[i + 1]; e++) {
            int64_t j = idx[e];
            double xj[3] = {pos[j], pos[n + j], pos[2 * n + j]};
            double vj[3] = {vel[j], vel[n + j], vel[2 * n + j]};
            double rp = oracle_pericentre(xi, vi, mass[i], xj, vj, mass[j], G);
            if (rp < lim) {
                if (out && total < cap) out[total] = (int32_t)j;
                total++;
                c++;
            }
        }
        counts[i] = c;
    }
    return total;
}

static int64_t uf_find(int64_t *parent, int64_t x)
{
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) { /* path compression (does not change the roots) */
        int64_t next = parent[x];
        parent[x] = r;
        x = next;
    }
    return r;
}

/* Connected components of the neighbour graph (offsets [n+1], idx).
 * label[i] = smallest index of i's cluster. cl_offsets [n+1] (first
 * n_clusters + 1 entries used) and members [n] list the clusters by label,
 * members ascending. Returns the number of clusters. */
OR_EXPORT int64_t oracle_clusters(int64_t n, const int64_t *offsets, const int32_t *idx,
                                  int32_t *label, int64_t *cl_offsets, int32_t *members)
{
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = offsets[i]; e < offsets[i + 1]; e++) {
            int64_t a = uf_find(parent, i), b = uf_find(parent, idx[e]);
            if (a == b) continue;
            if (a < b)
                parent[b] = a; /* the smaller index stays the root */
            else
                parent[a] = b;
        }
    int64_t *count = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        label[i] = (int32_t)uf_find(parent, i);
        count[label[i]]++;
    }
    /* clusters in label order; members ascending by construction */
    int64_t nc = 0, off = 0;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t r = 0; r < n; r++) {
        if (count[r] == 0) continue;
        cl_offsets[nc++] = off;
        start[r] = off;
        off += count[r];
    }
    cl_offsets[nc] = off;
    for (int64_t i = 0; i < n; i++) members[start[label[i]]++] = (int32_t)i;
    free(start);
    free(count);
    free(parent);
    return nc;
}

/* ------------------------------------------------------------------------
 * 8. Artificial particles (Sec. "Artificial particle algorithm for weak
 *    perturbation"): tidal-tensor measure points and fit (eq. tt, eq. map,
 *    Table A), pseudoparticle multipole of a binary (eq. quad, eq. quadtr,
 *    eq. dr, eq. r1r2, eq. avebinquad, eq. psep).
 *
 *  Measure points: r_cm + d_c u_p with the unit offsets u_p of Table A
 *  (order 2: 4 tetrahedron corners; order 3: 8 points).
 *  Field model (the evaluation rows of Table A): with r' = r - r_cm,
 *    A_i(r) = A_i(r_cm) + sum_j T_ij r'_j              (order 2)
 *             + sum_jk T_ijk r'_j r'_k                 (order 3)
 *  T_ij and T_ijk fully symmetric: 6 and 10 unknowns, collected as
 *    [xx xy xz yy yz zz] and [xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz].
 *  Fit: least squares over the 3 P equations A'(r_p) = A(r_p) - A(r_cm),
 *  i.e. the generalized inverse of the linear map (normal equations,
 *  solved by Gaussian elimination with partial pivoting).
 * ---------------------------------------------------------------------- */

static const double OR_S2 = 0.70710678118654752440; /* sqrt(2)/2 */

static int tidal_npts(int order) { return order == 2 ? 4 : 8; }
static int tidal_nunk(int order) { return order == 2 ? 6 : 16; }

static void tidal_unit(int order, int p, double u[3])
{
    static const double t2[4][3] = {{1, 0, -OR_S2}, {-1, 0, -OR_S2}, {0, 1, OR_S2}, {0, -1, OR_S2}};
    static const double t3[8][3] = {{1, 0, -1}, {0, 1, -1}, {-1, 0, -1}, {0, -1, -1},
                                    {1, 0, 1},  {0, 1, 1},  {-1, 0, 1},  {0, -1, 1}};
    for (int d = 0; d < 3; d++) u[d] = order == 2 ? t2[p][d] : t3[p][d];
}

/* Row of the design matrix: coefficient of unknown k in component i of the
 * model at offset r. */
static double tidal_coef(int order, int i, int k, const double r[3])
{
    static const int pair[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    static const int trip[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                    {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    if (k < 6) { /* T_ab contributes to A_a via r_b and (if a != b) to A_b via r_a */
        int a = pair[k][0], b = pair[k][1];
        double c = 0.0;
        if (i == a) c += r[b];
        if (i == b && a != b) c += r[a];
        return c;
    }
    (void)order;
    /* T_abc (a <= b <= c) enters A_i = sum_jk T_ijk r_j r_k through every
     * ordered (j, k) with {i, j, k} = {a, b, c}: take one i out of the
     * multiset; the remaining pair {p, q} gives r_p^2, or 2 r_p r_q if
     * p != q. */
    int t[3] = {trip[k - 6][0], trip[k - 6][1], trip[k - 6][2]};
    int at = -1;
    for (int q = 0; q < 3; q++)
        if (t[q] == i) at = q;
    if (at < 0) return 0.0;
    int rest[2], nr = 0;
    for (int q = 0; q < 3; q++)
        if (q != at) rest[nr++] = t[q];
    return rest[0] == rest[1] ? r[rest[0]] * r[rest[0]] : 2.0 * r[rest[0]] * r[rest[1]];
}

OR_EXPORT int oracle_tidal_points(int order, const double cm[3], double d_c, double *out)
{
    if (order != 2 && order != 3) return -1;
    int P = tidal_npts(order);
    for (int p = 0; p < P; p++) {
        double u[3];
        tidal_unit(order, p, u);
        for (int d = 0; d < 3; d++) out[3 * p + d] = cm[d] + d_c * u[d];
    }
    return P;
}

/* Generalized inverse of the design matrix for d_c = 1: ginv [K][3P]. */
OR_EXPORT int oracle_tidal_ginv(int order, double *ginv)
{
    if (order != 2 && order != 3) return -1;
    int P = tidal_npts(order), K = tidal_nunk(order), R = 3 * P;
    double *M = (double *)malloc(sizeof(double) * (size_t)R * K);
    for (int p = 0; p < P; p++) {
        double u[3];
        tidal_unit(order, p, u);
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < K; k++) M[(3 * p + i) * K + k] = tidal_coef(order, i, k, u);
    }
    /* normal matrix N = M^T M and its inverse by Gauss-Jordan */
    double N[16][32];
    for (int a = 0; a < K; a++) {
        for (int b = 0; b < K; b++) {
            double s = 0.0;
            for (int r = 0; r < R; r++) s += M[r * K + a] * M[r * K + b];
            N[a][b] = s;
            N[a][K + b] = a == b ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < K; c++) {
        int piv = c;
        for (int r = c + 1; r < K; r++)
            if (fabs(N[r][c]) > fabs(N[piv][c])) piv = r;
        if (fabs(N[piv][c]) < 1e-300) {
            free(M);
            return -2; /* rank deficient */
        }
        if (piv != c)
            for (int b = 0; b < 2 * K; b++) {
                double t = N[c][b];
                N[c][b] = N[piv][b];
                N[piv][b] = t;
            }
        double d = N[c][c];
        for (int b = 0; b < 2 * K; b++) N[c][b] /= d;
        for (int r = 0; r < K; r++) {
            if (r == c) continue;
            double f = N[r][c];
            if (f == 0.0) continue;
            for (int b = 0; b < 2 * K; b++) N[r][b] -= f * N[c][b];
        }
    }
    for (int a = 0; a < K; a++)
        for (int r = 0; r < R; r++) {
            double s = 0.0;
            for (int b = 0; b < K; b++) s += N[a][K + b] * M[r * K + b];
            ginv[a * R + r] = s;
        }
    free(M);
    return K;
}

/* T from measured accelerations: acc_cm[3], acc_pts[3P] (point-major,
 * x y z); out[3 + K] = A(r_cm), then the K unknowns. */
OR_EXPORT int oracle_tidal_fit(int order, double d_c, const double acc_cm[3],
                               const double *acc_pts, double *out)
{
    if (order != 2 && order != 3) return -1;
    int P = tidal_npts(order), K = tidal_nunk(order), R = 3 * P;
    double ginv[16 * 24];
    if (oracle_tidal_ginv(order, ginv) != K) return -2;
    for (int d = 0; d < 3; d++) out[d] = acc_cm[d];
    for (int k = 0; k < K; k++) {
        double s = 0.0;
        for (int r = 0; r < R; r++) s += ginv[k * R + r] * (acc_pts[r] - acc_cm[r % 3]);
        /* unknowns of order 1 scale with 1/d_c, of order 2 with 1/d_c^2 */
        out[3 + k] = k < 6 ? s / d_c : s / (d_c * d_c);
    }
    return 3 + K;
}

/* Field of the fitted model at offset r' from the centre, t = [A(r_cm),
 * T]. With out_pot non-NULL also the potential of the model, whose
 * gradient is minus the field (A = -grad phi): phi(r) = phi_cm -
 * sum_i r'_i (A_i(r_cm) + (1/2) sum_j T_ij r'_j + (1/3) sum_jk T_ijk r'_j
 * r'_k), i.e. the first-order part of A_i weighted 1/2 and the second-
 * order part 1/3. */
OR_EXPORT void oracle_tidal_eval(int order, const double *t, const double rp[3], double phi_cm,
                                 double out[3], double *out_pot)
{
    int K = tidal_nunk(order);
    double pot = phi_cm;
    for (int i = 0; i < 3; i++) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < K; k++) {
            double c = t[3 + k] * tidal_coef(order, i, k, rp);
            if (k < 6)
                s1 += c;
            else
                s2 += c;
        }
        out[i] = t[i] + s1 + s2;
        pot -= rp[i] * (t[i] + 0.5 * s1 + s2 / 3.0);
    }
    if (out_pot) *out_pot = pot;
}

/* Semi-major axis and eccentricity of a two-body orbit (eq. dr): out[0] = a,
 * out[1] = e. Returns -1 (and leaves out alone) for an unbound pair
 * (specific energy >= 0) or coincident particles. */
OR_EXPORT int oracle_binary_elements(double m1, double m2, const double x1[3], const double x2[3],
                                     const double v1[3], const double v2[3], double G,
                                     double out[2])
{
    double mu = G * (m1 + m2), r[3], v[3];
    for (int d = 0; d < 3; d++) {
        r[d] = x2[d] - x1[d];
        v[d] = v2[d] - v1[d];
    }
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double E = 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - mu / rr;
    if (!(rr > 0.0) || !(E < 0.0)) return -1;
    double h[3] = {r[1] * v[2] - r[2] * v[1], r[2] * v[0] - r[0] * v[2], r[0] * v[1] - r[1] * v[0]};
    /* e as the length of the eccentricity vector v x h / mu - r/|r| (well
     * conditioned also for nearly circular orbits, unlike 1 - h^2/(mu a)) */
    double ev[3] = {(v[1] * h[2] - v[2] * h[1]) / mu - r[0] / rr,
                    (v[2] * h[0] - v[0] * h[2]) / mu - r[1] / rr,
                    (v[0] * h[1] - v[1] * h[0]) / mu - r[2] / rr};
    out[0] = -mu / (2.0 * E);
    out[1] = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
    return 0;
}

/* Three pseudoparticles of a bound binary (masses (m1 + m2)/3 each) at the
 * positions of eq. psep in the orbital frame (x towards the pericentre,
 * z along the angular momentum; for e = 0 x along the current separation),
 * placed around the centre of mass. out_pos[3][3] (point-major). A radial
 * orbit (zero angular momentum) is the limit e = 1 along the separation.
 * Returns 0, or -1 for an unbound pair or coincident particles. */
OR_EXPORT int oracle_pseudo_particles(double m1, double m2, const double x1[3], const double x2[3],
                                      const double v1[3], const double v2[3], double G,
                                      double *out_pos, double *out_mass)
{
    double M = m1 + m2, mu = G * M;
    double r[3], v[3], cm[3];
    for (int d = 0; d < 3; d++) {
        r[d] = x2[d] - x1[d];
        v[d] = v2[d] - v1[d];
        cm[d] = (m1 * x1[d] + m2 * x2[d]) / M;
    }
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double v2s = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double E = 0.5 * v2s - mu / rr;
    if (!(E < 0.0) || !(rr > 0.0)) return -1;
    double a = -mu / (2.0 * E);
    double h[3] = {r[1] * v[2] - r[2] * v[1], r[2] * v[0] - r[0] * v[2], r[0] * v[1] - r[1] * v[0]};
    double hn = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    if (!(hn > 0.0)) {
        /* radial orbit (e = 1): the three points lie on the line of the
         * separation, the in-plane y offsets vanish */
        double s = a * sqrt(m1 * m2 / M / M), q = sqrt(3.75);
        for (int d = 0; d < 3; d++) {
            out_pos[d] = cm[d];
            out_pos[3 + d] = cm[d] + s * q * r[d] / rr;
            out_pos[6 + d] = cm[d] - s * q * r[d] / rr;
        }
        *out_mass = M / 3.0;
        return 0;
    }
    /* eccentricity vector e = v x h / mu - r/|r| */
    double ev[3] = {(v[1] * h[2] - v[2] * h[1]) / mu - r[0] / rr,
                    (v[2] * h[0] - v[0] * h[2]) / mu - r[1] / rr,
                    (v[0] * h[1] - v[1] * h[0]) / mu - r[2] / rr};
    double e = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
    double z[3] = {h[0] / hn, h[1] / hn, h[2] / hn}, x[3];
    if (e > 1e-12) {
        for (int d = 0; d < 3; d++) x[d] = ev[d] / e;
    } else {
        for (int d = 0; d < 3; d++) x[d] = r[d] / rr;
        e = 0.0;
    }
    double y[3] = {z[1] * x[2] - z[2] * x[1], z[2] * x[0] - z[0] * x[2], z[0] * x[1] - z[1] * x[0]};
    double redm = m1 * m2 / M;
    double s = a * sqrt(redm / M);
    double px[3] = {0.0, sqrt(3.0 * e * e + 0.75), -sqrt(3.0 * e * e + 0.75)};
    double py[3] = {sqrt(1.0 - e * e), -sqrt((1.0 - e * e) / 4.0), -sqrt((1.0 - e * e) / 4.0)};
    for (int k = 0; k < 3; k++)
        for (int d = 0; d < 3; d++) out_pos[3 * k + d] = cm[d] + s * (px[k] * x[d] + py[k] * y[d]);
    *out_mass = M / 3.0;
    return 0;
}

/* ------------------------------------------------------------------------
 * 9. SDAR groups (Sec. "SDAR", eq. rbin): pairs closer than
 *    r_g,ij = theta r_in,ij with r_in,ij = max(r_in,i, r_in,j), tested as
 *    d^2 < (theta r_in,ij)^2 in this order of operations; the groups are the
 *    connected components of this relation (computed with section 7's
 *    components from the CSR written here, all j != i, ascending).
 * ---------------------------------------------------------------------- */
static int is_group_pair(const double *X, const double *Y, const double *Z, const double *r_in,
                         double theta, int64_t i, int64_t j)
{
    double dx = X[j] - X[i];
    double dy = Y[j] - Y[i];
    double dz = Z[j] - Z[i];
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double d2 = xx + yy;
    d2 = d2 + zz;
    double R = r_in[i] > r_in[j] ? r_in[i] : r_in[j];
    double g = theta * R;
    double g2 = g * g;
    return d2 < g2;
}

OR_EXPORT int64_t oracle_group_relation(const double *pos, const double *r_in, int64_t n,
                                        double theta, int64_t *counts, int32_t *out,
                                        int64_t capacity)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++)
            if (j != i && is_group_pair(X, Y, Z, r_in, theta, i, j)) c++;
        counts[i] = c;
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++) total += counts[i];
    if (out && total <= capacity) {
        int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        start[0] = 0;
        for (int64_t i = 0; i < n; i++) start[i + 1] = start[i] + counts[i];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; i++) {
            int64_t w = start[i];
            for (int64_t j = 0; j < n; j++)
                if (j != i && is_group_pair(X, Y, Z, r_in, theta, i, j)) out[w++] = (int32_t)j;
        }
        free(start);
    }
    return total;
}
