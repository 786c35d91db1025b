/*
 * Plain FP64 CPU oracle for the short-range P3M pair force.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or constant with the
 * GPU library.
 *
 * What it computes (paper section 2.1.3, lower "short-range" half of
 * eq. p3m_gravity):
 *
 *   a_i = - sum_{j != i, |r_ij| < r_cut} mu_j * phi(|r_ij|) * r_ij
 *   phi(r) = g(r / (2 x_s)) / r^3  +  [r < eps_b] (|r|_B^-3 - r^-3)
 *   g(u) = erfc(u) + (2/sqrt(pi)) u exp(-u^2)
 *
 * The second term is the softening bracket of eq. p3m_gravity with the
 * B-spline shape (section 2.1.1, eq. bspline_force; eps_b = 2.8 eps, zero
 * for point particles, where the bracket vanishes).  For r < eps_b the
 * difference g/r^3 - r^-3 cancels to O(u^3), so it is evaluated as
 * (g - 1)/r^3 with g - 1 = (2/sqrt(pi)) u exp(-u^2) - erf(u), from its
 * Maclaurin series for u < 1/2 and in long double above (the same quantity,
 * written without the cancelling r^-3 terms).
 *
 * where mu_j = G m_j and r_ij = x_i - x_j is taken to the nearest periodic
 * image (the single image n' of eq. p3m_gravity; minimum image per
 * component).  The sum is strict, |r| < r_cut, and a candidate is rejected
 * when r^2 >= r_cut^2 (section 2.1.3, "Other optimisations"), with r^2 =
 * fma(dz, dz, fma(dy, dy, dx * dx)).  The bracket of
 * eq. p3m_gravity, r^-3 erfc(u) + r^-2 exp(-u^2) / (sqrt(pi) x_s), equals
 * g(u) / r^3 because r / (sqrt(pi) x_s) = 2u / sqrt(pi).
 *
 * Receivers are the active particles only, suppliers are all particles
 * (section 2.2.2, "Individual time steps").  A pair at exactly zero
 * separation contributes nothing (the j = i divergence is removed in
 * eq. force; coincident distinct particles are treated the same way).
 *
 * Accumulation is Neumaier-compensated FP64.  Compile with
 * -ffp-contract=off and without fast-math.
 *
 * Parity of the values themselves is pinned in the test suite against
 * closed forms and invariants (the paper prints no force values).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_2_SQRTPI 1.12837916709551257390 /* 2/sqrt(pi) */
#define ORACLE_SQRTPI   1.77245385090551602730 /* sqrt(pi) */

typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nsum_val(const nsum *a) { return a->s + a->c; }

/* Short-range force shape g(u) of the bracket of eq. p3m_gravity. */
static inline double g_sr(double u) {
    return erfc(u) + ORACLE_2_SQRTPI * u * exp(-u * u);
}

/* |r|_B^-3 of eq. bspline_force, x = r / eps_b < 1. */
static double bspline_rm3(double x, double eps_b) {
    const double k = 32.0 / (eps_b * eps_b * eps_b);
    if (x < 0.5) return k * (x * x * x - 6.0 / 5.0 * x * x + 1.0 / 3.0);
    return k * (-x * x * x / 3.0 + 6.0 / 5.0 * x * x - 1.5 * x + 2.0 / 3.0
                - 1.0 / (480.0 * x * x * x));
}

/* d|r|_B^-3 / dr, x = r / eps_b < 1 (derivative of the expression above). */
static double bspline_rm3_dr(double x, double eps_b) {
    const double k = 32.0 / (eps_b * eps_b * eps_b * eps_b);
    if (x < 0.5) return k * (3.0 * x * x - 12.0 / 5.0 * x);
    return k * (-x * x + 12.0 / 5.0 * x - 1.5 + 3.0 / (480.0 * x * x * x * x));
}

/* (g(u) - 1) / r^3 for the softened range, without the cancelling terms.
 * g - 1 = (2/sqrt(pi)) u exp(-u^2) - erf(u); subtracting the Maclaurin
 * series of erf(u) = (2/sqrt(pi)) sum_n (-1)^n u^(2n+1) / (n! (2n+1)) from
 * that of (2/sqrt(pi)) u exp(-u^2) = (2/sqrt(pi)) sum_n (-1)^n u^(2n+1) / n!
 * term by term gives
 *   (g - 1) / u^3 = (2/sqrt(pi)) sum_{n>=1} (-1)^n 2n u^(2n-2) / (n! (2n+1)),
 * used for u < 1/2 (where the direct difference loses the u^3 term to
 * rounding); above that the direct difference in long double is accurate. */
static double gm1_over_r3(double r, double x_s) {
    long double u = (long double)r / (2.0L * (long double)x_s);
    long double rl = r;
    if (u < 0.5L) {
        long double u2 = u * u, term = 1.0L, sum = 0.0L;   /* term = u^(2n-2) / n! */
        for (int n = 1; n <= 30; ++n) {
            term = (n == 1) ? 1.0L : term * u2 / n;
            long double t = (long double)(2 * n) * term / (long double)(2 * n + 1);
            sum += (n & 1) ? -t : t;
        }
        long double h = 1.12837916709551257389615890312154517L * sum;   /* (g-1)/u^3 */
        return (double)(h / (8.0L * (long double)x_s * x_s * x_s));
    }
    long double gm1 = 1.12837916709551257389615890312154517L * u * expl(-u * u) - erfl(u);
    return (double)(gm1 / (rl * rl * rl));
}

/* phi(r) of the header: the pair factor of a_i = -sum mu_j phi r_ij. */
static double pair_phi(double r, double r2, double x_s, double eps_b) {
    if (eps_b > 0.0 && r < eps_b) return gm1_over_r3(r, x_s) + bspline_rm3(r / eps_b, eps_b);
    return g_sr(r / (2.0 * x_s)) / (r2 * r);
}

/* Nearest periodic image of a coordinate difference. */
/* r^2 = fma(dz, dz, fma(dy, dy, dx * dx)): the squared distance of the
 * cut-off test, r^2 < r_cut^2 (section 2.1.3, "Other optimisations"), with
 * its rounding fixed (the paper leaves it open) so that every implementation
 * takes the same accept / reject decision near r_cut. */
static inline double sq_dist(double dx, double dy, double dz) {
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* The same squared distance for n rows (dx, dy, dz) of d, for the numpy
 * oracles that take a cut-off decision. */
void p3o_sq_dist(int64_t n, const double *d, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = sq_dist(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
}

static inline double min_image(double d, double box) {
    return d - box * rint(d / box);
}

int p3o_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Brute force over all suppliers for each listed receiver.
 *   pos    n x 3 row-major, mass n (NULL -> 1), recv list of n_recv indices.
 *   acc    n_recv x 3 out, cnt n_recv accepted pairs out (may be NULL),
 *   absum  n_recv out: sum_j |pair force| (may be NULL).
 */
void p3o_force(int64_t n, const double *pos, const double *mass, double box, double x_s,
               double r_cut, double eps_b, int64_t n_recv, const int64_t *recv, double *acc,
               int64_t *cnt, double *absum) {
    const double rc2 = r_cut * r_cut;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_recv; ++q) {
        const int64_t i = recv[q];
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ab = {0, 0};
        int64_t c = 0;
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image(xi - pos[3 * j], box);
            double dy = min_image(yi - pos[3 * j + 1], box);
            double dz = min_image(zi - pos[3 * j + 2], box);
            double r2 = sq_dist(dx, dy, dz);
            if (r2 >= rc2 || r2 == 0.0) continue;
            double r = sqrt(r2);
            double mu = mass ? mass[j] : 1.0;
            double s = mu * pair_phi(r, r2, x_s, eps_b);
            nsum_add(&ax, -s * dx);
            nsum_add(&ay, -s * dy);
            nsum_add(&az, -s * dz);
            nsum_add(&ab, fabs(s) * r);
            ++c;
        }
        acc[3 * q] = nsum_val(&ax);
        acc[3 * q + 1] = nsum_val(&ay);
        acc[3 * q + 2] = nsum_val(&az);
        if (cnt) cnt[q] = c;
        if (absum) absum[q] = nsum_val(&ab);
    }
}

/* ---------------------------------------------------------------------- */
/* Independent cell-list version (section 2.1.3, "Tiles"): cubic cells of
 * side >= r_cut, so every partner of a particle lies in the surrounding
 * 3 x 3 x 3 block of cells.  Needs at least 3 cells per dimension so that
 * no neighbour cell is visited twice; the caller falls back to p3o_force
 * otherwise.  Used for full-size checks that brute force cannot afford. */

typedef struct {
    int nc;            /* cells per dimension */
    double cell;       /* cell side */
    int64_t *start;    /* nc^3 + 1 */
    int64_t *order;    /* particle indices grouped by cell */
} cell_list;

static int cell_coord(double x, double box, int nc) {
    double w = x - box * floor(x / box);
    int c = (int)floor(w * nc / box);
    if (c >= nc) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

static int build_cells(cell_list *cl, int64_t n, const double *pos, double box, double r_cut) {
    int nc = (int)floor(box / r_cut);
    if (nc < 3) return -1;
    cl->nc = nc;
    cl->cell = box / nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    cl->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    cl->order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *key = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_coord(pos[3 * i], box, nc), cy = cell_coord(pos[3 * i + 1], box, nc),
            cz = cell_coord(pos[3 * i + 2], box, nc);
        key[i] = ((int64_t)cx * nc + cy) * nc + cz;
        cl->start[key[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cl->start[c + 1] += cl->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, cl->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) cl->order[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void free_cells(cell_list *cl) {
    free(cl->start);
    free(cl->order);
}

int p3o_force_tiled(int64_t n, const double *pos, const double *mass, double box, double x_s,
                    double r_cut, double eps_b, int64_t n_recv, const int64_t *recv, double *acc,
                    int64_t *cnt, double *absum) {
    cell_list cl;
    if (build_cells(&cl, n, pos, box, r_cut) != 0) return -1;
    const int nc = cl.nc;
    const double rc2 = r_cut * r_cut;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_recv; ++q) {
        const int64_t i = recv[q];
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        int cx = cell_coord(xi, box, nc), cy = cell_coord(yi, box, nc), cz = cell_coord(zi, box, nc);
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ab = {0, 0};
        int64_t c = 0;
        for (int ox = -1; ox <= 1; ++ox)
        for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -1; oz <= 1; ++oz) {
            int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc, nz = (cz + oz + nc) % nc;
            int64_t cell = ((int64_t)nx * nc + ny) * nc + nz;
            for (int64_t p = cl.start[cell]; p < cl.start[cell + 1]; ++p) {
                int64_t j = cl.order[p];
                if (j == i) continue;
                double dx = min_image(xi - pos[3 * j], box);
                double dy = min_image(yi - pos[3 * j + 1], box);
                double dz = min_image(zi - pos[3 * j + 2], box);
                double r2 = sq_dist(dx, dy, dz);
                if (r2 >= rc2 || r2 == 0.0) continue;
                double r = sqrt(r2);
                double mu = mass ? mass[j] : 1.0;
                double s = mu * pair_phi(r, r2, x_s, eps_b);
                nsum_add(&ax, -s * dx);
                nsum_add(&ay, -s * dy);
                nsum_add(&az, -s * dz);
                nsum_add(&ab, fabs(s) * r);
                ++c;
            }
        }
        acc[3 * q] = nsum_val(&ax);
        acc[3 * q + 1] = nsum_val(&ay);
        acc[3 * q + 2] = nsum_val(&az);
        if (cnt) cnt[q] = c;
        if (absum) absum[q] = nsum_val(&ab);
    }
    free_cells(&cl);
    return 0;
}

/*
 * Candidate / accepted pair census of the cell list by neighbour kind
 * (0 same cell, 1 shares a face, 2 shares only an edge, 3 only a corner).
 * With cells of side exactly r_cut this is the experiment behind the
 * rejection percentages quoted in section 2.1.3 ("Subtiles").
 */
int p3o_cell_census(int64_t n, const double *pos, double box, double r_cut,
                    int64_t *candidates4, int64_t *accepted4) {
    cell_list cl;
    if (build_cells(&cl, n, pos, box, r_cut) != 0) return -1;
    const int nc = cl.nc;
    const double rc2 = r_cut * r_cut;
    int64_t cand[4] = {0, 0, 0, 0}, acc[4] = {0, 0, 0, 0};
    #pragma omp parallel
    {
        int64_t lc[4] = {0, 0, 0, 0}, la[4] = {0, 0, 0, 0};
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
            int cx = cell_coord(xi, box, nc), cy = cell_coord(yi, box, nc), cz = cell_coord(zi, box, nc);
            for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
            for (int oz = -1; oz <= 1; ++oz) {
                int kind = (ox != 0) + (oy != 0) + (oz != 0);
                int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc, nz = (cz + oz + nc) % nc;
                int64_t cell = ((int64_t)nx * nc + ny) * nc + nz;
                for (int64_t p = cl.start[cell]; p < cl.start[cell + 1]; ++p) {
                    int64_t j = cl.order[p];
                    if (j == i) continue;
                    double dx = min_image(xi - pos[3 * j], box);
                    double dy = min_image(yi - pos[3 * j + 1], box);
                    double dz = min_image(zi - pos[3 * j + 2], box);
                    double r2 = sq_dist(dx, dy, dz);
                    lc[kind]++;
                    if (r2 < rc2 && r2 > 0.0) la[kind]++;
                }
            }
        }
        #pragma omp critical
        for (int k = 0; k < 4; ++k) { cand[k] += lc[k]; acc[k] += la[k]; }
    }
    for (int k = 0; k < 4; ++k) { candidates4[k] = cand[k]; accepted4[k] = acc[k]; }
    free_cells(&cl);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Vector-Jacobian product of the force above with respect to positions.
 *
 * Loss L = sum_{i active} w_i . a_i.  Writing a_i = -sum_j mu_j F(r_ij) with
 * F(r) = phi(|r|) r, the Jacobian J(r) = dF/dr = phi I + (phi'(r)/r) r r^T is
 * symmetric and even in r, and
 *   dL/dx_k = - sum_{j != k, |r_kj| < r_cut} J(r_kj) (mu_j w_k [k act] - mu_k w_j [j act]).
 * With g'(u) = -(4/sqrt(pi)) u^2 exp(-u^2) and phi = g/r^3:
 *   phi'(r)/r = -3 g / r^5 - exp(-u^2) / (2 sqrt(pi) x_s^3 r^2);
 * inside the softening length phi = (g - 1)/r^3 + |r|_B^-3, whose derivative
 * adds d|r|_B^-3/dr / r + 3 / r^5 (the -3 g / r^5 and +3 / r^5 terms are
 * combined as -3 (g - 1) / r^5).
 * The pair set is the one of the forward sum (fixed at these positions). */
static inline void pair_jvp(double dx, double dy, double dz, double r2, double x_s,
                            double eps_b, double vx, double vy, double vz, double *ox,
                            double *oy, double *oz) {
    double r = sqrt(r2);
    double u = r / (2.0 * x_s);
    double e = exp(-u * u);
    double gauss = e / (2.0 * ORACLE_SQRTPI * x_s * x_s * x_s * r2);
    double phi, c;   /* c = -phi'(r) / r */
    if (eps_b > 0.0 && r < eps_b) {
        double gm1r3 = gm1_over_r3(r, x_s);
        phi = gm1r3 + bspline_rm3(r / eps_b, eps_b);
        c = 3.0 * gm1r3 / r2 + gauss - bspline_rm3_dr(r / eps_b, eps_b) / r;
    } else {
        double g = erfc(u) + ORACLE_2_SQRTPI * u * e;
        phi = g / (r2 * r);
        c = 3.0 * g / (r2 * r2 * r) + gauss;
    }
    double rv = dx * vx + dy * vy + dz * vz;
    *ox = phi * vx - c * rv * dx;
    *oy = phi * vy - c * rv * dy;
    *oz = phi * vz - c * rv * dz;
}

void p3o_vjp(int64_t n, const double *pos, const double *mass, const uint8_t *active,
             const double *w, double box, double x_s, double r_cut, double eps_b, int64_t n_k,
             const int64_t *kidx, double *grad) {
    const double rc2 = r_cut * r_cut;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_k; ++q) {
        const int64_t k = kidx[q];
        const int ak = active ? (active[k] != 0) : 1;
        const double muk = mass ? mass[k] : 1.0;
        nsum gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            int aj = active ? (active[j] != 0) : 1;
            if (!ak && !aj) continue;
            double dx = min_image(pos[3 * k] - pos[3 * j], box);
            double dy = min_image(pos[3 * k + 1] - pos[3 * j + 1], box);
            double dz = min_image(pos[3 * k + 2] - pos[3 * j + 2], box);
            double r2 = sq_dist(dx, dy, dz);
            if (r2 >= rc2 || r2 == 0.0) continue;
            double muj = mass ? mass[j] : 1.0;
            double vx = 0, vy = 0, vz = 0;
            if (ak) { vx += muj * w[3 * k]; vy += muj * w[3 * k + 1]; vz += muj * w[3 * k + 2]; }
            if (aj) { vx -= muk * w[3 * j]; vy -= muk * w[3 * j + 1]; vz -= muk * w[3 * j + 2]; }
            double ox, oy, oz;
            pair_jvp(dx, dy, dz, r2, x_s, eps_b, vx, vy, vz, &ox, &oy, &oz);
            nsum_add(&gx, -ox);
            nsum_add(&gy, -oy);
            nsum_add(&gz, -oz);
        }
        grad[3 * q] = nsum_val(&gx);
        grad[3 * q + 1] = nsum_val(&gy);
        grad[3 * q + 2] = nsum_val(&gz);
    }
}

int p3o_vjp_tiled(int64_t n, const double *pos, const double *mass, const uint8_t *active,
                  const double *w, double box, double x_s, double r_cut, double eps_b,
                  int64_t n_k, const int64_t *kidx, double *grad) {
    cell_list cl;
    if (build_cells(&cl, n, pos, box, r_cut) != 0) return -1;
    const int nc = cl.nc;
    const double rc2 = r_cut * r_cut;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n_k; ++q) {
        const int64_t k = kidx[q];
        const int ak = active ? (active[k] != 0) : 1;
        const double muk = mass ? mass[k] : 1.0;
        const double xk = pos[3 * k], yk = pos[3 * k + 1], zk = pos[3 * k + 2];
        int cx = cell_coord(xk, box, nc), cy = cell_coord(yk, box, nc), cz = cell_coord(zk, box, nc);
        nsum gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
        for (int ox_ = -1; ox_ <= 1; ++ox_)
        for (int oy_ = -1; oy_ <= 1; ++oy_)
        for (int oz_ = -1; oz_ <= 1; ++oz_) {
            int nx = (cx + ox_ + nc) % nc, ny = (cy + oy_ + nc) % nc, nz = (cz + oz_ + nc) % nc;
            int64_t cell = ((int64_t)nx * nc + ny) * nc + nz;
            for (int64_t p = cl.start[cell]; p < cl.start[cell + 1]; ++p) {
                int64_t j = cl.order[p];
                if (j == k) continue;
                int aj = active ? (active[j] != 0) : 1;
                if (!ak && !aj) continue;
                double dx = min_image(xk - pos[3 * j], box);
                double dy = min_image(yk - pos[3 * j + 1], box);
                double dz = min_image(zk - pos[3 * j + 2], box);
                double r2 = sq_dist(dx, dy, dz);
                if (r2 >= rc2 || r2 == 0.0) continue;
                double muj = mass ? mass[j] : 1.0;
                double vx = 0, vy = 0, vz = 0;
                if (ak) { vx += muj * w[3 * k]; vy += muj * w[3 * k + 1]; vz += muj * w[3 * k + 2]; }
                if (aj) { vx -= muk * w[3 * j]; vy -= muk * w[3 * j + 1]; vz -= muk * w[3 * j + 2]; }
                double ox, oy, oz;
                pair_jvp(dx, dy, dz, r2, x_s, eps_b, vx, vy, vz, &ox, &oy, &oz);
                nsum_add(&gx, -ox);
                nsum_add(&gy, -oy);
                nsum_add(&gz, -oz);
            }
        }
        grad[3 * q] = nsum_val(&gx);
        grad[3 * q + 1] = nsum_val(&gy);
        grad[3 * q + 2] = nsum_val(&gz);
    }
    free_cells(&cl);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Central finite differences of L = sum_{i active} w_i . a_i with respect
 * to x_k, for listed particles k.  Only pair terms that involve k change
 * when x_k moves:
 *   L_k(y) = [k act] w_k . a_k(y) - sum_{i act, i != k} mu_k w_i . F(x_i - y),
 * so the difference quotient of L_k equals that of L.
 *   mode 0 (fixed): the pair set is frozen at the unperturbed positions
 *                   (the derivative the adjoint defines);
 *   mode 1 (plain): the pair set is re-evaluated at each perturbed position;
 *                   straddle[q] = 1 when any pair of k changes membership
 *                   between the -h, 0 and +h positions. */
static double local_loss(int64_t n, const double *pos, const double *mass, const uint8_t *active,
                         const double *w, double box, double x_s, double r_cut, double eps_b,
                         int64_t k, const double *y, int mode, int *flip) {
    const double rc2 = r_cut * r_cut;
    const int ak = active ? (active[k] != 0) : 1;
    const double muk = mass ? mass[k] : 1.0;
    nsum L = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        int aj = active ? (active[j] != 0) : 1;
        if (!ak && !aj) continue;
        double dx0 = min_image(pos[3 * k] - pos[3 * j], box);
        double dy0 = min_image(pos[3 * k + 1] - pos[3 * j + 1], box);
        double dz0 = min_image(pos[3 * k + 2] - pos[3 * j + 2], box);
        double r20 = sq_dist(dx0, dy0, dz0);
        int in0 = (r20 < rc2 && r20 > 0.0);
        double dx = min_image(y[0] - pos[3 * j], box);
        double dy = min_image(y[1] - pos[3 * j + 1], box);
        double dz = min_image(y[2] - pos[3 * j + 2], box);
        double r2 = sq_dist(dx, dy, dz);
        int in1 = (r2 < rc2 && r2 > 0.0);
        if (in0 != in1 && flip) *flip = 1;
        int use = mode == 0 ? in0 : in1;
        if (!use || r2 == 0.0) continue;
        double r = sqrt(r2);
        double phi = pair_phi(r, r2, x_s, eps_b);
        double muj = mass ? mass[j] : 1.0;
        /* F(x_k - x_j) = phi * d, contributes -mu_j F to a_k and +mu_k F to a_j */
        if (ak) nsum_add(&L, -muj * phi * (w[3 * k] * dx + w[3 * k + 1] * dy + w[3 * k + 2] * dz));
        if (aj) nsum_add(&L, muk * phi * (w[3 * j] * dx + w[3 * j + 1] * dy + w[3 * j + 2] * dz));
    }
    return nsum_val(&L);
}

void p3o_fd_grad(int64_t n, const double *pos, const double *mass, const uint8_t *active,
                 const double *w, double box, double x_s, double r_cut, double eps_b, double h,
                 int mode, int64_t n_k, const int64_t *kidx, double *grad, uint8_t *straddle) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_k; ++q) {
        const int64_t k = kidx[q];
        int flip = 0;
        for (int d = 0; d < 3; ++d) {
            double yp[3] = {pos[3 * k], pos[3 * k + 1], pos[3 * k + 2]};
            double ym[3] = {yp[0], yp[1], yp[2]};
            yp[d] += h;
            ym[d] -= h;
            double lp = local_loss(n, pos, mass, active, w, box, x_s, r_cut, eps_b, k, yp, mode,
                                   &flip);
            double lm = local_loss(n, pos, mass, active, w, box, x_s, r_cut, eps_b, k, ym, mode,
                                   &flip);
            grad[3 * q + d] = (lp - lm) / (2.0 * h);
        }
        if (straddle) straddle[q] = (uint8_t)flip;
    }
}
