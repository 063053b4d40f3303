/*
 * FP64 CPU oracle of the CRK-HACC short-range step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its binding may link,
 * load or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Plain, slow and obviously correct: one target particle at a time, its
 * neighbours found either by brute force over all particles or with a
 * periodic k-d tree, every sum accumulated in double precision in
 * ascending neighbour index.  Inputs are the float32 values the GPU path consumes,
 * widened to double.
 *
 * What each function computes (the paper names the method, CRKSPH, and the
 * long/short gravity split, but prints none of the formulas, so each is the
 * standard definition of the named method, with the readings listed in the
 * design notes):
 *   - cubic-spline (M4) kernel W(r,h) with support 2h;
 *   - orc_density: V_i = 1/sum_j W(r_ij,h_i), rho~_i = sum_j m_j W(r_ij,h_i),
 *     gathered over gas j including j = i (pairwise sums of the form of
 *     Eq. (1), Sec. IV-B.2);
 *   - orc_coefficients: reproducing-kernel moments and the correction
 *     coefficients A, B, grad A, grad B that make the corrected kernel
 *     A(1 + B.x)W reproduce constant and linear fields exactly (CRKSPH,
 *     Sec. IV-A), then rho = A (rho~ + B.M1), ideal-gas P and c;
 *   - orc_velocity_gradient: the corrected-kernel gradient of the velocity
 *     field (exact for linear fields);
 *   - orc_hydro: the antisymmetric CRKSPH pair force F_ij = -F_ji (Eq. (2)
 *     and its (anti)symmetry, Sec. IV-B.2) and the work-split du/dt, which
 *     conserve momentum and energy (Sec. IV-A); optionally with the
 *     viscosity acting on a limited linear reconstruction of both velocities
 *     at the pair midpoint (CRKSPH's viscosity, named in Sec. IV-A), and
 *     optionally with the pair work taken at the time-centred velocities of
 *     a kick (the compatible energy update, which makes one kick conserve
 *     the total energy exactly);
 *   - orc_gravity: the short-range remainder of Newtonian gravity inside the
 *     handover scale r_c (Sec. IV-A): Plummer-softened 1/r^2 minus the force
 *     between two S2 clouds of diameter r_c (Hockney & Eastwood), zero
 *     beyond r_c.
 * Parity-pinned by the tests under tests/ (normalisation, reproducing
 * conditions, lattice symmetry, conservation, closed forms, quadrature,
 * brute force versus the tree, exact gradients of linear fields).  The
 * viscosity form and constants are a reading: pinned only by conservation,
 * Galilean invariance and the cases where the reconstruction removes the
 * viscosity of a linear flow or reduces to the plain form.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* periodic geometry                                                          */
/* ------------------------------------------------------------------------ */

/* minimum-image separation along one axis in the unit periodic box */
static double min_image(double d)
{
    if (d > 0.5) d -= 1.0;
    else if (d < -0.5) d += 1.0;
    return d;
}

/* ------------------------------------------------------------------------ */
/* cubic-spline kernel                                                        */
/* ------------------------------------------------------------------------ */

/* W(r, h) and dW/dr of the M4 cubic spline with support 2h, normalised to 1
 * in three dimensions. */
void orc_kernel(double r, double h, double *W, double *dWdr)
{
    double q = r / h;
    double s = 1.0 / (M_PI * h * h * h);
    if (q < 1.0) {
        *W = s * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
        *dWdr = s / h * (-3.0 * q + 2.25 * q * q);
    } else if (q < 2.0) {
        double t = 2.0 - q;
        *W = s * 0.25 * t * t * t;
        *dWdr = -s / h * 0.75 * t * t;
    } else {
        *W = 0.0;
        *dWdr = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* short-range gravity                                                        */
/* ------------------------------------------------------------------------ */

/* Force between two unit-mass S2 clouds of diameter a at separation r
 * (Hockney & Eastwood's S2 shape: density falling linearly to zero at
 * radius a/2).  Equals 1/r^2 for r >= a. */
double orc_s2_force(double r, double a)
{
    double xi = 2.0 * r / a;
    double c = 1.0 / (35.0 * a * a);
    if (xi < 1.0) {
        double x2 = xi * xi, x3 = x2 * xi, x4 = x3 * xi, x5 = x4 * xi,
               x6 = x5 * xi;
        return c * (224.0 * xi - 224.0 * x3 + 70.0 * x4 + 48.0 * x5 - 21.0 * x6);
    }
    if (xi < 2.0) {
        double t = 2.0 - xi;
        double t5 = t * t * t * t * t;
        return 1.0 / (r * r)
               - c * t5 * (7.0 * xi * xi * xi + 22.0 * xi * xi + 10.0 * xi + 4.0)
                     / (xi * xi);
    }
    return 1.0 / (r * r);
}

/* Short-range force magnitude g(r) per unit mass pair: Plummer-softened
 * Newtonian force minus the S2 long-range part, cut at r_c. */
double orc_grav_g(double r, double r_c, double eps)
{
    if (r >= r_c) return 0.0;
    double s = r * r + eps * eps;
    return r / (s * sqrt(s)) - orc_s2_force(r, r_c);
}

/* ------------------------------------------------------------------------ */
/* neighbour search                                                           */
/* ------------------------------------------------------------------------ */

/* A k-d tree over n points of the periodic unit box (coordinates in [1, 2)):
 * nodes split at the median of their widest extent down to leaves of at
 * most KD_LEAF points, each node with its bounding box and, when smoothing
 * lengths are given, the largest h of its points.  brute = 1 skips the tree
 * and tests every point.  Any search structure gives the same neighbours:
 * every list is sorted by index, so the sums run in ascending neighbour
 * index whatever the structure (and equal the brute-force sums exactly). */
#define KD_LEAF 32
typedef struct {
    int64_t n;
    int brute;
    int64_t *idx;          /* point indices, grouped by node */
    int64_t nn;            /* nodes in use */
    int64_t *start, *count;
    int64_t *left;         /* first child (the second is left + 1), -1: leaf */
    double *lo, *hi;       /* 3 per node */
    double *hmax;          /* per node, NULL without smoothing lengths */
} search_t;

static double coord(const double *x, const double *y, const double *z, int a,
                    int64_t i)
{
    return a == 0 ? x[i] : (a == 1 ? y[i] : z[i]);
}

/* Reorders idx[0..n) so that idx[k] holds the point of rank k along axis a
 * (ties in any order), smaller keys before it and larger after it:
 * quickselect with a three-way partition around a median-of-three pivot. */
static void select_kth(int64_t *idx, int64_t n, int64_t k, const double *x,
                       const double *y, const double *z, int a)
{
    int64_t lo = 0, hi = n;  /* the rank-k element lies in [lo, hi) */
    while (hi - lo > 1) {
        double p0 = coord(x, y, z, a, idx[lo]);
        double p1 = coord(x, y, z, a, idx[lo + (hi - lo) / 2]);
        double p2 = coord(x, y, z, a, idx[hi - 1]);
        double piv = p0 < p1 ? (p1 < p2 ? p1 : (p0 < p2 ? p2 : p0))
                             : (p0 < p2 ? p0 : (p1 < p2 ? p2 : p1));
        /* [lo, lt) < piv, [lt, i) == piv, (gt, hi) > piv */
        int64_t lt = lo, i = lo, gt = hi - 1;
        while (i <= gt) {
            double v = coord(x, y, z, a, idx[i]);
            if (v < piv) {
                int64_t t = idx[lt]; idx[lt] = idx[i]; idx[i] = t;
                ++lt; ++i;
            } else if (v > piv) {
                int64_t t = idx[gt]; idx[gt] = idx[i]; idx[i] = t;
                --gt;
            } else {
                ++i;
            }
        }
        if (k < lt) hi = lt;
        else if (k > gt) lo = gt + 1;
        else return;
    }
}

/* Fills node nd (bounding box, h_max) and splits it at the median of its
 * widest extent; large subtrees are built as parallel tasks (the node
 * numbering then depends on scheduling, the neighbour lists do not). */
static void build_node(search_t *s, int64_t nd, const double *x,
                       const double *y, const double *z, const double *h)
{
    int64_t st = s->start[nd], c = s->count[nd];
    int64_t *I = s->idx + st;
    double lo[3] = {4.0, 4.0, 4.0}, hi[3] = {-4.0, -4.0, -4.0}, hm = 0.0;
    for (int64_t q = 0; q < c; ++q) {
        int64_t i = I[q];
        double p[3] = {x[i], y[i], z[i]};
        for (int a = 0; a < 3; ++a) {
            if (p[a] < lo[a]) lo[a] = p[a];
            if (p[a] > hi[a]) hi[a] = p[a];
        }
        if (h && h[i] > hm) hm = h[i];
    }
    for (int a = 0; a < 3; ++a) {
        s->lo[3 * nd + a] = lo[a];
        s->hi[3 * nd + a] = hi[a];
    }
    if (h) s->hmax[nd] = hm;
    s->left[nd] = -1;
    if (c <= KD_LEAF) return;
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    int64_t half = c / 2;
    select_kth(I, c, half, x, y, z, ax);
    int64_t l;
#pragma omp atomic capture
    { l = s->nn; s->nn += 2; }
    s->start[l] = st;
    s->count[l] = half;
    s->start[l + 1] = st + half;
    s->count[l + 1] = c - half;
    s->left[nd] = l;
    if (c > 200000) {
#pragma omp task
        build_node(s, l, x, y, z, h);
#pragma omp task
        build_node(s, l + 1, x, y, z, h);
#pragma omp taskwait
    } else {
        build_node(s, l, x, y, z, h);
        build_node(s, l + 1, x, y, z, h);
    }
}

static int search_build(search_t *s, int64_t n, const double *x,
                        const double *y, const double *z, const double *h,
                        int brute)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->brute = brute;
    if (brute || n == 0) {
        s->brute = 1;
        return 0;
    }
    int64_t cap = 2 * (n / (KD_LEAF / 2) + 2);
    s->idx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    s->start = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    s->count = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    s->left = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    s->lo = (double *)malloc((size_t)cap * 3 * sizeof(double));
    s->hi = (double *)malloc((size_t)cap * 3 * sizeof(double));
    if (h) s->hmax = (double *)malloc((size_t)cap * sizeof(double));
    if (!s->idx || !s->start || !s->count || !s->left || !s->lo || !s->hi ||
        (h && !s->hmax))
        return -1;
    for (int64_t i = 0; i < n; ++i) s->idx[i] = i;
    s->nn = 1;
    s->start[0] = 0;
    s->count[0] = n;
#pragma omp parallel
#pragma omp single
    build_node(s, 0, x, y, z, h);
    return 0;
}

static void search_free(search_t *s)
{
    free(s->idx);
    free(s->start);
    free(s->count);
    free(s->left);
    free(s->lo);
    free(s->hi);
    free(s->hmax);
}

/* Neighbours of one target: indices j, sorted ascending, whose
 * minimum-image separation x_i - x_j has r^2 < R^2 (hi <= 0), or
 * r < 2 max(hi, h_j) (hi > 0, smoothing lengths h given). */
typedef struct {
    int64_t j;
    double dx, dy, dz, r2;
} nbr_rec;
typedef struct {
    int64_t n, cap;
    nbr_rec *r;
    int64_t *stack;
    int64_t scap;
} nbr_t;

static void nbr_push(nbr_t *nb, int64_t j, double dx, double dy, double dz,
                     double r2)
{
    if (nb->n == nb->cap) {
        nb->cap = nb->cap ? 2 * nb->cap : 256;
        nb->r = (nbr_rec *)realloc(nb->r, (size_t)nb->cap * sizeof(nbr_rec));
        if (!nb->r) abort();
    }
    nbr_rec *e = &nb->r[nb->n++];
    e->j = j;
    e->dx = dx;
    e->dy = dy;
    e->dz = dz;
    e->r2 = r2;
}

static void nbr_free(nbr_t *nb)
{
    free(nb->r);
    free(nb->stack);
}

static int nbr_cmp(const void *a, const void *b)
{
    int64_t ja = ((const nbr_rec *)a)->j, jb = ((const nbr_rec *)b)->j;
    return (ja > jb) - (ja < jb);
}

static void test_point(nbr_t *nb, int64_t j, const double *X, const double *Y,
                       const double *Z, const double *H, double px, double py,
                       double pz, double R, double hi)
{
    double dx = min_image(px - X[j]);
    double dy = min_image(py - Y[j]);
    double dz = min_image(pz - Z[j]);
    double r2 = dx * dx + dy * dy + dz * dz;
    double lim = hi > 0.0 ? 2.0 * (hi > H[j] ? hi : H[j]) : R;
    if (r2 < lim * lim) nbr_push(nb, j, dx, dy, dz, r2);
}

/* distance from p to the interval [lo, hi] over the periodic images of p */
static double box_gap(double p, double lo, double hi)
{
    double best = 1.0;
    for (int s = -1; s <= 1; ++s) {
        double q = p + (double)s;
        double d = q < lo ? lo - q : (q > hi ? q - hi : 0.0);
        if (d < best) best = d;
    }
    return best;
}

static void find_neighbours(const search_t *s, const double *X,
                            const double *Y, const double *Z, const double *H,
                            double px, double py, double pz, double R,
                            double hi, nbr_t *nb)
{
    nb->n = 0;
    if (s->brute) {
        for (int64_t j = 0; j < s->n; ++j)
            test_point(nb, j, X, Y, Z, H, px, py, pz, R, hi);
        return;
    }
    if (nb->scap < 256) {
        nb->scap = 256;
        nb->stack = (int64_t *)realloc(nb->stack, 256 * sizeof(int64_t));
        if (!nb->stack) abort();
    }
    int64_t sp = 0;
    nb->stack[sp++] = 0;
    while (sp > 0) {
        int64_t nd = nb->stack[--sp];
        double gx = box_gap(px, s->lo[3 * nd], s->hi[3 * nd]);
        double gy = box_gap(py, s->lo[3 * nd + 1], s->hi[3 * nd + 1]);
        double gz = box_gap(pz, s->lo[3 * nd + 2], s->hi[3 * nd + 2]);
        double rad = hi > 0.0 ? 2.0 * (hi > s->hmax[nd] ? hi : s->hmax[nd]) : R;
        if (gx * gx + gy * gy + gz * gz >= rad * rad) continue;
        if (s->left[nd] < 0) {
            const int64_t *I = s->idx + s->start[nd];
            for (int64_t q = 0; q < s->count[nd]; ++q)
                test_point(nb, I[q], X, Y, Z, H, px, py, pz, R, hi);
        } else {
            if (sp + 2 > nb->scap) {
                nb->scap *= 2;
                nb->stack = (int64_t *)realloc(nb->stack,
                                               (size_t)nb->scap * sizeof(int64_t));
                if (!nb->stack) abort();
            }
            nb->stack[sp++] = s->left[nd] + 1;
            nb->stack[sp++] = s->left[nd];
        }
    }
    qsort(nb->r, (size_t)nb->n, sizeof(nbr_rec), nbr_cmp);
}

static int64_t target_index(const int64_t *targets, int64_t k)
{
    return targets ? targets[k] : k;
}

/* ------------------------------------------------------------------------ */
/* neighbour lists (used by the tests to expand sampled targets)              */
/* ------------------------------------------------------------------------ */

/* For each target i: the gas j with r_ij < 2 h_i (mode 0, the gather range
 * of the density and coefficient sums) or r_ij < 2 max(h_i, h_j) (mode 1,
 * the range of the force sums), j = i included.  With idx == NULL only the
 * counts are written; otherwise idx receives the concatenated lists
 * (offsets = running sum of counts). */
int orc_neighbours(int64_t n, const double *x, const double *y,
                   const double *z, const double *h, int mode, int64_t nt,
                   const int64_t *targets, int brute, int64_t *counts,
                   const int64_t *offsets, int64_t *idx)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, h, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double hi = h[i];
        int64_t c = 0;
        find_neighbours(&cl, x, y, z, h, x[i], y[i], z[i], 2.0 * hi,
                        mode ? hi : 0.0, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double r2 = nb.r[q].r2;
            double lim = mode ? 2.0 * (hi > h[j] ? hi : h[j]) : 2.0 * hi;
            if (r2 < lim * lim) {
                if (idx) idx[offsets[k] + c] = j;
                c++;
            }
        }
        counts[k] = c;
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* density / volume                                                           */
/* ------------------------------------------------------------------------ */

int orc_density(int64_t n, const double *x, const double *y, const double *z,
                const double *h, const double *m, int64_t nt,
                const int64_t *targets, int brute, double *V,
                double *rho_tilde)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, h, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double hi = h[i];
        double sw = 0.0, smw = 0.0;
        find_neighbours(&cl, x, y, z, h, x[i], y[i], z[i], 2.0 * hi, 0.0, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double r2 = nb.r[q].r2;
            double W, dW;
            orc_kernel(sqrt(r2), hi, &W, &dW);
            sw += W;
            smw += m[j] * W;
        }
        V[k] = 1.0 / sw;
        rho_tilde[k] = smw;
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* reproducing-kernel correction coefficients                                 */
/* ------------------------------------------------------------------------ */

/* m2 counts as singular when det(m2) <= DEGENERATE (tr(m2)/3)^3, i.e. its
 * eigenvalues multiply to less than 1e-5 of the cube of their mean: such a
 * neighbourhood (a single particle, a pair, three points, a sheet) cannot fix
 * the linear correction.  The bound lies far above the rounding noise of
 * float32 moment sums (about 1e-7 relative), so float32 and float64
 * evaluations take the same branch except in a narrow band, a few 1e-7
 * relative wide, around the bound itself. */
#define DEGENERATE 1e-5

/* Solve the reproducing conditions at one particle from its moments.
 * m2 is symmetric; inverted through its adjugate.  Returns 1 when m2 is
 * singular (then B = grad B = 0, A = 1/m0, grad A = -grad m0 / m0^2). */
static int solve_coefficients(double m0, const double m1[3],
                              const double m2[3][3], const double dm0[3],
                              const double dm1[3][3] /* [g][a] */,
                              const double dm2[3][3][3] /* [g][a][b] */,
                              double *A, double B[3], double dA[3],
                              double dB[3][3] /* [g][a] */)
{
    double c00 = m2[1][1] * m2[2][2] - m2[1][2] * m2[2][1];
    double c01 = m2[1][2] * m2[2][0] - m2[1][0] * m2[2][2];
    double c02 = m2[1][0] * m2[2][1] - m2[1][1] * m2[2][0];
    double det = m2[0][0] * c00 + m2[0][1] * c01 + m2[0][2] * c02;
    double tr = m2[0][0] + m2[1][1] + m2[2][2];
    if (!(fabs(det) > DEGENERATE * tr * tr * tr / 27.0) || !(tr > 0.0)) {
        *A = 1.0 / m0;
        for (int g = 0; g < 3; ++g) {
            B[g] = 0.0;
            dA[g] = -dm0[g] / (m0 * m0);
            for (int a = 0; a < 3; ++a) dB[g][a] = 0.0;
        }
        return 1;
    }
    double inv[3][3];
    inv[0][0] = c00 / det;
    inv[0][1] = (m2[0][2] * m2[2][1] - m2[0][1] * m2[2][2]) / det;
    inv[0][2] = (m2[0][1] * m2[1][2] - m2[0][2] * m2[1][1]) / det;
    inv[1][0] = c01 / det;
    inv[1][1] = (m2[0][0] * m2[2][2] - m2[0][2] * m2[2][0]) / det;
    inv[1][2] = (m2[0][2] * m2[1][0] - m2[0][0] * m2[1][2]) / det;
    inv[2][0] = c02 / det;
    inv[2][1] = (m2[0][1] * m2[2][0] - m2[0][0] * m2[2][1]) / det;
    inv[2][2] = (m2[0][0] * m2[1][1] - m2[0][1] * m2[1][0]) / det;

    /* B = -m2^{-1} m1 */
    for (int a = 0; a < 3; ++a) {
        B[a] = 0.0;
        for (int b = 0; b < 3; ++b) B[a] -= inv[a][b] * m1[b];
    }
    /* A = 1 / (m0 + B.m1) */
    double Bm1 = B[0] * m1[0] + B[1] * m1[1] + B[2] * m1[2];
    *A = 1.0 / (m0 + Bm1);
    for (int g = 0; g < 3; ++g) {
        /* d_g B = -m2^{-1} (d_g m1 + d_g m2 . B) */
        double rhs[3];
        for (int a = 0; a < 3; ++a) {
            rhs[a] = dm1[g][a];
            for (int b = 0; b < 3; ++b) rhs[a] += dm2[g][a][b] * B[b];
        }
        for (int a = 0; a < 3; ++a) {
            dB[g][a] = 0.0;
            for (int b = 0; b < 3; ++b) dB[g][a] -= inv[a][b] * rhs[b];
        }
        /* d_g A = -A^2 (d_g m0 + d_g B . m1 + B . d_g m1) */
        double s = dm0[g];
        for (int a = 0; a < 3; ++a) s += dB[g][a] * m1[a] + B[a] * dm1[g][a];
        dA[g] = -(*A) * (*A) * s;
    }
    return 0;
}

/* For each target: A, B[3], gradA[3], gradB[9] (gradB[3g+a] = d_g B^a),
 * corrected density rho, pressure P and sound speed cs; degenerate[k] = 1
 * when the moment matrix was singular. */
int orc_coefficients(int64_t n, const double *x, const double *y,
                     const double *z, const double *h, const double *m,
                     const double *V, const double *u, double gamma,
                     int64_t nt, const int64_t *targets, int brute, double *A,
                     double *B, double *gradA, double *gradB, double *rho,
                     double *P, double *cs, int *degenerate)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, h, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double hi = h[i];
        double m0 = 0.0, m1[3] = {0, 0, 0}, m2[3][3] = {{0}}, dm0[3] = {0, 0, 0};
        double sxdw[3][3] = {{0}};        /* sum V x^a d_g W   [g][a]    */
        double sxxdw[3][3][3] = {{{0}}};  /* sum V x^a x^b d_g W [g][a][b] */
        double M1[3] = {0, 0, 0}, rt = 0.0;
        find_neighbours(&cl, x, y, z, h, x[i], y[i], z[i], 2.0 * hi, 0.0, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double dx = nb.r[q].dx, dy = nb.r[q].dy;
            double dz = nb.r[q].dz, r2 = nb.r[q].r2;
            double r = sqrt(r2);
            double W, dW;
            orc_kernel(r, hi, &W, &dW);
            double xv[3] = {dx, dy, dz};
            double gW[3];
            for (int g = 0; g < 3; ++g) gW[g] = (r > 0.0) ? dW * xv[g] / r : 0.0;
            double Vj = V[j];
            m0 += Vj * W;
            rt += m[j] * W;
            for (int a = 0; a < 3; ++a) {
                m1[a] += Vj * xv[a] * W;
                M1[a] += m[j] * xv[a] * W;
                dm0[a] += Vj * gW[a];
                for (int b = 0; b < 3; ++b) m2[a][b] += Vj * xv[a] * xv[b] * W;
            }
            for (int g = 0; g < 3; ++g)
                for (int a = 0; a < 3; ++a) {
                    sxdw[g][a] += Vj * xv[a] * gW[g];
                    for (int b = 0; b < 3; ++b)
                        sxxdw[g][a][b] += Vj * xv[a] * xv[b] * gW[g];
                }
        }
        double dm1[3][3], dm2[3][3][3];
        for (int g = 0; g < 3; ++g)
            for (int a = 0; a < 3; ++a) {
                dm1[g][a] = (a == g ? m0 : 0.0) + sxdw[g][a];
                for (int b = 0; b < 3; ++b)
                    dm2[g][a][b] = (a == g ? m1[b] : 0.0) + (b == g ? m1[a] : 0.0)
                                   + sxxdw[g][a][b];
            }
        double a_, b_[3], da_[3], db_[3][3];
        int deg = solve_coefficients(m0, m1, m2, dm0, dm1, dm2, &a_, b_, da_, db_);
        A[k] = a_;
        for (int g = 0; g < 3; ++g) {
            B[3 * k + g] = b_[g];
            gradA[3 * k + g] = da_[g];
            for (int a = 0; a < 3; ++a) gradB[9 * k + 3 * g + a] = db_[g][a];
        }
        double r_ = a_ * (rt + b_[0] * M1[0] + b_[1] * M1[1] + b_[2] * M1[2]);
        rho[k] = r_;
        P[k] = (gamma - 1.0) * r_ * u[i];
        cs[k] = sqrt(gamma * (gamma - 1.0) * u[i]);
        if (degenerate) degenerate[k] = deg;
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* CRKSPH pair forces                                                         */
/* ------------------------------------------------------------------------ */

/* Gradient of particle k's corrected kernel at separation y (= x_k - x_other),
 * with the kernel at k's own smoothing length. */
static void grad_rk(const double y[3], double hk, double Ak, const double *Bk,
                    const double *dAk, const double *dBk, double out[3])
{
    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double W, dW;
    orc_kernel(r, hk, &W, &dW);
    double By = Bk[0] * y[0] + Bk[1] * y[1] + Bk[2] * y[2];
    for (int g = 0; g < 3; ++g) {
        double gW = (r > 0.0) ? dW * y[g] / r : 0.0;
        double dBy = dBk[3 * g + 0] * y[0] + dBk[3 * g + 1] * y[1]
                     + dBk[3 * g + 2] * y[2];
        out[g] = dAk[g] * (1.0 + By) * W + Ak * (dBy + Bk[g]) * W
                 + Ak * (1.0 + By) * gW;
    }
}

/* Velocity gradient with the corrected kernel (the CRKSPH gradient of a
 * field, Sec. IV-A):
 *   dv[a][b]_i = sum_j V_j (v_j^a - v_i^a) g_i^b(x_ij)
 * over gas j with r_ij < 2 h_i (j = i adds zero).  The corrected kernel
 * reproduces constants, so sum_j V_j g_i(x_ij) = 0 and this is the gradient
 * of the reproduced field; a linear field comes back exactly. */
int orc_velocity_gradient(int64_t n, const double *x, const double *y,
                          const double *z, const double *vx, const double *vy,
                          const double *vz, const double *h, const double *V,
                          const double *A, const double *B,
                          const double *gradA, const double *gradB,
                          int64_t nt, const int64_t *targets, int brute,
                          double *dv)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, h, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double hi = h[i];
        double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        find_neighbours(&cl, x, y, z, h, x[i], y[i], z[i], 2.0 * hi, 0.0, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double xij[3] = {nb.r[q].dx, nb.r[q].dy, nb.r[q].dz};
            double gi[3];
            grad_rk(xij, hi, A[i], &B[3 * i], &gradA[3 * i], &gradB[9 * i], gi);
            double dvj[3] = {vx[j] - vx[i], vy[j] - vy[i], vz[j] - vz[i]};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) D[3 * a + b] += V[j] * dvj[a] * gi[b];
        }
        for (int e = 0; e < 9; ++e) dv[9 * k + e] = D[e];
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* Limiter of the linear velocity reconstruction for the pair (i, j), with
 * s_k = x_ij . (dv_k x_ij) the velocity gradient of each side projected on
 * the pair axis: van Leer's limiter of their ratio, 4 s_i s_j / (s_i + s_j)^2
 * when they agree in sign, else 0 (symmetric in i and j); a close pair,
 * eta = r / max(h_i, h_j) below eta_crit, is damped further by
 * exp(-((eta - eta_crit) / eta_fold)^2). */
static double recon_limiter(double si, double sj, double r, double hmax,
                            double eta_crit, double eta_fold)
{
    double phi = 0.0;
    if (si * sj > 0.0) phi = 4.0 * si * sj / ((si + sj) * (si + sj));
    double eta = r / hmax;
    if (eta < eta_crit) {
        double t = (eta - eta_crit) / eta_fold;
        phi *= exp(-t * t);
    }
    return phi;
}

int orc_hydro(int64_t n, const double *x, const double *y, const double *z,
              const double *vx, const double *vy, const double *vz,
              const double *h, const double *m, const double *V,
              const double *rho, const double *P, const double *cs,
              const double *A, const double *B, const double *gradA,
              const double *gradB, double Cl, double Cq, double epsQ,
              const double *dv, double eta_crit, double eta_fold,
              const double *v1x, const double *v1y, const double *v1z,
              int64_t nt, const int64_t *targets, int brute, double *ax,
              double *ay, double *az, double *dudt)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, h, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double hi = h[i];
        double f[3] = {0, 0, 0}, work = 0.0;
        find_neighbours(&cl, x, y, z, h, x[i], y[i], z[i], 0.0, hi, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double dx = nb.r[q].dx, dy = nb.r[q].dy;
            double dz = nb.r[q].dz, r2 = nb.r[q].r2;
            double lim = 2.0 * (hi > h[j] ? hi : h[j]);
            if (j != i && r2 < lim * lim) {
                double xij[3] = {dx, dy, dz};
                double xji[3] = {-dx, -dy, -dz};
                double gi[3], gj[3];
                grad_rk(xij, hi, A[i], &B[3 * i], &gradA[3 * i], &gradB[9 * i], gi);
                grad_rk(xji, h[j], A[j], &B[3 * j], &gradA[3 * j], &gradB[9 * j], gj);
                double vij[3] = {vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j]};
                /* velocity difference seen by the viscosity: the actual one,
                 * or (dv given) both sides' velocities extrapolated linearly
                 * to the pair midpoint, limited */
                double vt[3] = {vij[0], vij[1], vij[2]};
                if (dv) {
                    const double *Di = &dv[9 * i], *Dj = &dv[9 * j];
                    double ei[3], ej[3];
                    for (int a = 0; a < 3; ++a) {
                        ei[a] = Di[3 * a] * dx + Di[3 * a + 1] * dy + Di[3 * a + 2] * dz;
                        ej[a] = Dj[3 * a] * dx + Dj[3 * a + 1] * dy + Dj[3 * a + 2] * dz;
                    }
                    double si = ei[0] * dx + ei[1] * dy + ei[2] * dz;
                    double sj = ej[0] * dx + ej[1] * dy + ej[2] * dz;
                    double phi = recon_limiter(si, sj, sqrt(r2),
                                               hi > h[j] ? hi : h[j],
                                               eta_crit, eta_fold);
                    for (int a = 0; a < 3; ++a)
                        vt[a] = vij[a] - 0.5 * phi * (ei[a] + ej[a]);
                }
                double vdx = vt[0] * dx + vt[1] * dy + vt[2] * dz;
                double mui = hi * vdx / (r2 + epsQ * hi * hi);
                double muj = h[j] * vdx / (r2 + epsQ * h[j] * h[j]);
                if (mui > 0.0) mui = 0.0;
                if (muj > 0.0) muj = 0.0;
                double Qi = rho[i] * (-Cl * cs[i] * mui + Cq * mui * mui);
                double Qj = rho[j] * (-Cl * cs[j] * muj + Cq * muj * muj);
                double pp = P[i] + P[j];
                double Fij[3];
                for (int g = 0; g < 3; ++g)
                    Fij[g] = -0.5 * V[i] * V[j]
                             * (pp * (gi[g] - gj[g]) + Qi * gi[g] - Qj * gj[g]);
                for (int g = 0; g < 3; ++g) f[g] += Fij[g];
                /* the pair's work: with the velocities after the kick (v1)
                 * given, at the time-centred velocities (v + v1)/2 */
                double wv[3] = {vij[0], vij[1], vij[2]};
                if (v1x) {
                    wv[0] = 0.5 * (vij[0] + (v1x[i] - v1x[j]));
                    wv[1] = 0.5 * (vij[1] + (v1y[i] - v1y[j]));
                    wv[2] = 0.5 * (vij[2] + (v1z[i] - v1z[j]));
                }
                work += wv[0] * Fij[0] + wv[1] * Fij[1] + wv[2] * Fij[2];
            }
        }
        ax[k] = f[0] / m[i];
        ay[k] = f[1] / m[i];
        az[k] = f[2] / m[i];
        dudt[k] = -0.5 * work / m[i];
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* short-range gravity                                                        */
/* ------------------------------------------------------------------------ */

/* a_i = -G sum_{j != i, r < r_c} m_j g(r) x_ij / r over all particles of the
 * box (both species, concatenated by the caller). */
int orc_gravity(int64_t n, const double *x, const double *y, const double *z,
                const double *m, double r_c, double eps, double G, int64_t nt,
                const int64_t *targets, int brute, double *ax, double *ay,
                double *az)
{
    search_t cl;
    if (search_build(&cl, n, x, y, z, NULL, brute)) return -1;
#pragma omp parallel
    {
    nbr_t nb = {0, 0, NULL, NULL, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = target_index(targets, k);
        double a[3] = {0, 0, 0};
        find_neighbours(&cl, x, y, z, NULL, x[i], y[i], z[i], r_c, 0.0, &nb);
        for (int64_t q = 0; q < nb.n; ++q) {
            int64_t j = nb.r[q].j;
            double dx = nb.r[q].dx, dy = nb.r[q].dy;
            double dz = nb.r[q].dz, r2 = nb.r[q].r2;
            if (j != i && r2 > 0.0) {
                double r = sqrt(r2);
                double s = -G * m[j] * orc_grav_g(r, r_c, eps) / r;
                a[0] += s * dx;
                a[1] += s * dy;
                a[2] += s * dz;
            }
        }
        ax[k] = a[0];
        ay[k] = a[1];
        az[k] = a[2];
    }
    nbr_free(&nb);
    }
    search_free(&cl);
    return 0;
}

/* Number of threads the parallel loops above use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
