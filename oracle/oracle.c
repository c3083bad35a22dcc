/*
 * CPU oracle for the many-body MD force path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  The HIP product path never calls it, and it
 * shares no source with that path.
 *
 * Plain, slow, obviously correct double-precision code, written from
 * Hou et al., "Molecular dynamics simulations with many-body potentials on
 * multiple GPUs":
 *   - per-atom energy, total energy and force: Section 2, eqs. (1)-(3);
 *   - linked-cell neighbour search over the 26 surrounding cells of a periodic
 *     box: Section 3.2 (the "normative" linked-list algorithm);
 *   - the density pass and the force pass over a neighbour list with the
 *     cutoff re-checked inside the loop: Section 3.3, Figs. 5 and 6;
 *   - the SETB embedding F = -sqrt(rho): Section 4.
 *   - the pair virial and pressure of eq. (6) and the Berendsen barostat of
 *     eq. (5);
 *   - the electron-gas friction of eq. (4);
 *   - several atom species (the superscripts a, b of eqs. (1)-(3)) and frozen
 *     atoms (the atom states of Section 3.1).
 * Velocity-Verlet replaces the paper's predictor-corrector (Section 3.3).
 * The adjoint with respect to B-spline potential coefficients is derived from
 * eqs. (2)-(3) by differentiating the force and energy with respect to the
 * three potential functions (the derivation is written next to orc_adjoint).
 * Where the paper leaves a choice open (how the friction enters the
 * integrator, which function gives the derivative of rho_j with several
 * species, what a frozen atom does), the reading taken is stated next to the
 * function that implements it.
 *
 * Build with -ffp-contract=off: the squared distance of the neighbour test is
 * (dx*dx + dy*dy) + dz*dz with every product and sum rounded separately.
 *
 * Units: Angstrom, eV, fs, amu.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FS 1
#define ORC_SMTB 2
#define ORC_SPLINE 3
#define ORC_BSPLINE 4

/* (eV/Angstrom)/amu in Angstrom/fs^2: (e / u) * 1e10 * 1e-20 */
static const double ORC_KAPPA = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;

typedef struct {
    int kind;
    double rc;
    const double *par;    /* FS: c d c0 c1 c2 A; SMTB: A xi p q r0 */
    const double *tab[3]; /* phi(r), f(r), F(rho) */
    int ntab[3];          /* SPLINE: intervals; BSPLINE: coefficients */
    double lo[3], hi[3];
} orc_pot;

/* ------------------------------------------------------------------ tables */

/* Per-interval cubic S = a + b t + c t^2 + d t^3 on a uniform grid. */
static void spline_eval(const double *tab, int nint, double lo, double hi, double x,
                        double *s, double *ds, double *dds)
{
    double h = (hi - lo) / nint;
    double u = (x - lo) / h;
    int m = (int)floor(u);
    if (m < 0) m = 0;
    if (m > nint - 1) m = nint - 1;
    double t = u - m;
    const double *c = tab + 4 * m;
    *s = c[0] + c[1] * t + c[2] * t * t + c[3] * t * t * t;
    *ds = (c[1] + 2.0 * c[2] * t + 3.0 * c[3] * t * t) / h;
    *dds = (2.0 * c[2] + 6.0 * c[3] * t) / (h * h);
}

/* Uniform cubic B-spline pieces on one interval, t in [0, 1]. */
static void bspline_basis(double t, double b[4], double db[4], double ddb[4])
{
    double s = 1.0 - t;
    b[0] = s * s * s / 6.0;
    b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    b[3] = t * t * t / 6.0;
    db[0] = -s * s / 2.0;
    db[1] = (9.0 * t * t - 12.0 * t) / 6.0;
    db[2] = (-9.0 * t * t + 6.0 * t + 3.0) / 6.0;
    db[3] = t * t / 2.0;
    ddb[0] = s;
    ddb[1] = 3.0 * t - 2.0;
    ddb[2] = -3.0 * t + 1.0;
    ddb[3] = t;
}

/* Interval index m and local coordinate t of x on the B-spline grid. */
static void bspline_locate(int ncoef, double lo, double hi, double x, int *m, double *t, double *h)
{
    int nint = ncoef - 3;
    *h = (hi - lo) / nint;
    double u = (x - lo) / *h;
    int k = (int)floor(u);
    if (k < 0) k = 0;
    if (k > nint - 1) k = nint - 1;
    *m = k;
    *t = u - k;
}

static void bspline_eval(const double *th, int ncoef, double lo, double hi, double x,
                         double *s, double *ds, double *dds)
{
    int m;
    double t, h, b[4], db[4], ddb[4];
    bspline_locate(ncoef, lo, hi, x, &m, &t, &h);
    bspline_basis(t, b, db, ddb);
    *s = *ds = *dds = 0.0;
    for (int l = 0; l < 4; ++l) {
        *s += th[m + l] * b[l];
        *ds += th[m + l] * db[l] / h;
        *dds += th[m + l] * ddb[l] / (h * h);
    }
}

/* -------------------------------------------------------------- potential */

/* Pair potential V(r) (phi) and dV/dr: eq. (1). */
static void pot_pair(const orc_pot *p, double r, double *v, double *dv)
{
    double dd;
    switch (p->kind) {
    case ORC_FS: {
        double c = p->par[0], c0 = p->par[2], c1 = p->par[3], c2 = p->par[4];
        if (r >= c) { *v = 0.0; *dv = 0.0; return; }
        double poly = c0 + c1 * r + c2 * r * r;
        *v = (r - c) * (r - c) * poly;
        *dv = 2.0 * (r - c) * poly + (r - c) * (r - c) * (c1 + 2.0 * c2 * r);
        return;
    }
    case ORC_SMTB: {
        double A = p->par[0], pp = p->par[2], r0 = p->par[4];
        double e = exp(-pp * (r / r0 - 1.0));
        *v = 2.0 * A * e;
        *dv = -pp / r0 * 2.0 * A * e;
        return;
    }
    case ORC_SPLINE:
        spline_eval(p->tab[0], p->ntab[0], p->lo[0], p->hi[0], r, v, dv, &dd);
        return;
    case ORC_BSPLINE:
        bspline_eval(p->tab[0], p->ntab[0], p->lo[0], p->hi[0], r, v, dv, &dd);
        return;
    }
    *v = *dv = 0.0;
}

/* Density contribution rho(r) (f) and its derivative: eq. (1). */
static void pot_dens(const orc_pot *p, double r, double *f, double *df)
{
    double dd;
    switch (p->kind) {
    case ORC_FS: {
        double d = p->par[1];
        if (r >= d) { *f = 0.0; *df = 0.0; return; }
        *f = (r - d) * (r - d);
        *df = 2.0 * (r - d);
        return;
    }
    case ORC_SMTB: {
        double xi = p->par[1], q = p->par[3], r0 = p->par[4];
        double e = exp(-2.0 * q * (r / r0 - 1.0));
        *f = xi * xi * e;
        *df = -2.0 * q / r0 * xi * xi * e;
        return;
    }
    case ORC_SPLINE:
        spline_eval(p->tab[1], p->ntab[1], p->lo[1], p->hi[1], r, f, df, &dd);
        return;
    case ORC_BSPLINE:
        bspline_eval(p->tab[1], p->ntab[1], p->lo[1], p->hi[1], r, f, df, &dd);
        return;
    }
    *f = *df = 0.0;
}

/* Embedding F(rho), F', F''.  FS: F = -A sqrt(rho); SMTB: F = -sqrt(rho)
 * (Section 4); rho = 0 gives zero for all three. */
static void pot_embed(const orc_pot *p, double rho, double *F, double *dF, double *ddF)
{
    switch (p->kind) {
    case ORC_FS:
    case ORC_SMTB: {
        double A = (p->kind == ORC_FS) ? p->par[5] : 1.0;
        if (rho <= 0.0) { *F = *dF = *ddF = 0.0; return; }
        double s = sqrt(rho);
        *F = -A * s;
        *dF = -A / (2.0 * s);
        *ddF = A / (4.0 * rho * s);
        return;
    }
    case ORC_SPLINE:
        spline_eval(p->tab[2], p->ntab[2], p->lo[2], p->hi[2], rho, F, dF, ddF);
        return;
    case ORC_BSPLINE:
        bspline_eval(p->tab[2], p->ntab[2], p->lo[2], p->hi[2], rho, F, dF, ddF);
        return;
    }
    *F = *dF = *ddF = 0.0;
}

/* Exported for tests: evaluate one of the three functions (0 phi, 1 f, 2 F). */
void orc_pot_eval(const orc_pot *p, int which, double x, double *v, double *d1, double *d2)
{
    *d2 = 0.0;
    if (which == 0) pot_pair(p, x, v, d1);
    else if (which == 1) pot_dens(p, x, v, d1);
    else pot_embed(p, x, v, d1, d2);
}

/* --------------------------------------------------------------- geometry */

/* Wrap a coordinate into [0, L) by adding or subtracting L. */
static double wrap1(double x, double L)
{
    while (x < 0.0) x += L;
    while (x >= L) x -= L;
    return x;
}

void orc_wrap(int64_t n, double *x, double *y, double *z, double L)
{
    for (int64_t i = 0; i < n; ++i) {
        x[i] = wrap1(x[i], L);
        y[i] = wrap1(y[i], L);
        z[i] = wrap1(z[i], L);
    }
}

/* Minimum-image component of x_j - x_i. */
static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/* Minimum-image separation x_j - x_i and its square, (dx dx + dy dy) + dz dz. */
static double sep2(const double *x, const double *y, const double *z, int64_t i, int64_t j,
                   double L, double *dx, double *dy, double *dz)
{
    *dx = min_image(x[j] - x[i], L);
    *dy = min_image(y[j] - y[i], L);
    *dz = min_image(z[j] - z[i], L);
    double a = *dx * *dx;
    double b = *dy * *dy;
    double c = *dz * *dz;
    return (a + b) + c;
}

/* ---------------------------------------------------------- neighbour list */

static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Cells per dimension: the largest count whose cell edge is not below rlist. */
static int cells_per_dim(double L, double rlist)
{
    int nc = (int)floor(L / rlist);
    while (nc > 1 && L / nc < rlist) --nc;
    return nc < 1 ? 1 : nc;
}

/* Linked-cell structure: head[cell] and next[atom] chains (Section 3.2). */
typedef struct {
    int nc;
    int64_t *head, *next;
} orc_cells;

static int cell_coord(double x, double L, int nc)
{
    int c = (int)floor(x / L * nc);
    if (c < 0) c = 0;
    if (c > nc - 1) c = nc - 1;
    return c;
}

static void cells_build(orc_cells *cl, int64_t n, const double *x, const double *y,
                        const double *z, double L, double rcell)
{
    int nc = cells_per_dim(L, rcell);
    cl->nc = nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    cl->head = (int64_t *)malloc(sizeof(int64_t) * ncell);
    cl->next = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t c = 0; c < ncell; ++c) cl->head[c] = -1;
    /* push in descending order so that each chain lists ascending ids */
    for (int64_t i = n - 1; i >= 0; --i) {
        int cx = cell_coord(wrap1(x[i], L), L, nc);
        int cy = cell_coord(wrap1(y[i], L), L, nc);
        int cz = cell_coord(wrap1(z[i], L), L, nc);
        int64_t c = ((int64_t)cz * nc + cy) * nc + cx;
        cl->next[i] = cl->head[c];
        cl->head[c] = i;
    }
}

static void cells_free(orc_cells *cl)
{
    free(cl->head);
    free(cl->next);
}

/* Distinct neighbour-cell offsets along one dimension ({-1,0,1} mod nc). */
static int stencil_1d(int c, int nc, int out[3])
{
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
        int v = ((c + d) % nc + nc) % nc;
        int dup = 0;
        for (int q = 0; q < k; ++q) dup |= (out[q] == v);
        if (!dup) out[k++] = v;
    }
    return k;
}

/* Neighbours of atom i within r2max (j != i), written ascending into out. */
static int cells_query(const orc_cells *cl, const double *x, const double *y, const double *z,
                       double L, int64_t i, double r2max, int32_t *out, int cap, int *total)
{
    int nc = cl->nc;
    int cx = cell_coord(wrap1(x[i], L), L, nc);
    int cy = cell_coord(wrap1(y[i], L), L, nc);
    int cz = cell_coord(wrap1(z[i], L), L, nc);
    int sx[3], sy[3], sz[3];
    int kx = stencil_1d(cx, nc, sx), ky = stencil_1d(cy, nc, sy), kz = stencil_1d(cz, nc, sz);
    int n = 0;
    for (int a = 0; a < kz; ++a)
        for (int b = 0; b < ky; ++b)
            for (int c = 0; c < kx; ++c) {
                int64_t cell = ((int64_t)sz[a] * nc + sy[b]) * nc + sx[c];
                for (int64_t j = cl->head[cell]; j >= 0; j = cl->next[j]) {
                    if (j == i) continue;
                    double dx, dy, dz;
                    if (sep2(x, y, z, i, j, L, &dx, &dy, &dz) < r2max) {
                        if (n < cap) out[n] = (int32_t)j;
                        ++n;
                    }
                }
            }
    *total = n;
    int m = n < cap ? n : cap;
    qsort(out, (size_t)m, sizeof(int32_t), cmp_i32);
    return m;
}

/* Full Verlet list by linked cells.  count[i] = true neighbour count; ids is
 * row-major [n][maxn] in ascending order.  Returns the largest count (a value
 * above maxn means the rows were truncated). */
int orc_list_cells(int64_t n, const double *x, const double *y, const double *z, double L,
                   double rlist, int maxn, int32_t *count, int32_t *ids)
{
    orc_cells cl;
    cells_build(&cl, n, x, y, z, L, rlist);
    double r2 = rlist * rlist;
    int worst = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : worst)
    for (int64_t i = 0; i < n; ++i) {
        int tot;
        cells_query(&cl, x, y, z, L, i, r2, ids + i * maxn, maxn, &tot);
        count[i] = tot;
        if (tot > worst) worst = tot;
    }
    cells_free(&cl);
    return worst;
}

/* Same list by brute force over all pairs. */
int orc_list_brute(int64_t n, const double *x, const double *y, const double *z, double L,
                   double rlist, int maxn, int32_t *count, int32_t *ids)
{
    double r2 = rlist * rlist;
    int worst = 0;
#pragma omp parallel for schedule(static) reduction(max : worst)
    for (int64_t i = 0; i < n; ++i) {
        int k = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            if (sep2(x, y, z, i, j, L, &dx, &dy, &dz) < r2) {
                if (k < maxn) ids[i * maxn + k] = (int32_t)j;
                ++k;
            }
        }
        count[i] = k;
        if (k > worst) worst = k;
    }
    return worst;
}

/* ---------------------------------------------------------------- passes */

/* Density pass: rho_i = sum over listed j with r < rc of rho(r_ij) (eq. 3
 * definition of rho_i; Fig. 5). */
void orc_density(int64_t n, const double *x, const double *y, const double *z, double L,
                 const orc_pot *p, const int32_t *count, const int32_t *ids, int maxn,
                 double *rho)
{
    double rc2 = p->rc * p->rc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < count[i]; ++k) {
            int64_t j = ids[i * maxn + k];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double f, df;
                pot_dens(p, sqrt(r2), &f, &df);
                s += f;
            }
        }
        rho[i] = s;
    }
}

/* Embedding pass: F(rho_i), F'(rho_i), F''(rho_i). */
void orc_embed(int64_t n, const orc_pot *p, const double *rho, double *F, double *Fp,
               double *Fpp)
{
    for (int64_t i = 0; i < n; ++i) {
        double a, b, c;
        pot_embed(p, rho[i], &a, &b, &c);
        if (F) F[i] = a;
        if (Fp) Fp[i] = b;
        if (Fpp) Fpp[i] = c;
    }
}

/* Force pass, eq. (3) with r_ij = x_i - x_j:
 *   f_i = -sum_j [(F'(rho_i) + F'(rho_j)) rho'(r) + V'(r)] (x_i - x_j)/r
 * and per-atom energy e_i = F(rho_i) + 1/2 sum_j V(r) (eq. 1). */
void orc_forces(int64_t n, const double *x, const double *y, const double *z, double L,
                const orc_pot *p, const int32_t *count, const int32_t *ids, int maxn,
                const double *Femb, const double *Fp, double *fx, double *fy, double *fz,
                double *e_atom)
{
    double rc2 = p->rc * p->rc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0;
        for (int k = 0; k < count[i]; ++k) {
            int64_t j = ids[i * maxn + k];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double r = sqrt(r2);
                double v, dv, f, df;
                pot_pair(p, r, &v, &dv);
                pot_dens(p, r, &f, &df);
                double coef = ((Fp[i] + Fp[j]) * df + dv) / r;
                /* (x_i - x_j) = -(dx, dy, dz) */
                ax += coef * dx;
                ay += coef * dy;
                az += coef * dz;
                ep += 0.5 * v;
            }
        }
        fx[i] = ax;
        fy[i] = ay;
        fz[i] = az;
        if (e_atom) e_atom[i] = Femb[i] + ep;
    }
}

/* ---------------------------------------------------- direct (list-free) */

/* Total energy, eq. (2), by a direct sum over all pairs (minimum image). */
double orc_energy_direct(int64_t n, const double *x, const double *y, const double *z, double L,
                         const orc_pot *p)
{
    double rc2 = p->rc * p->rc;
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rho = 0.0, pair = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double r = sqrt(r2), v, dv, f, df;
                pot_pair(p, r, &v, &dv);
                pot_dens(p, r, &f, &df);
                rho += f;
                pair += v;
            }
        }
        double F, dF, ddF;
        pot_embed(p, rho, &F, &dF, &ddF);
        e += F + 0.5 * pair;
    }
    return e;
}

/* Forces, eq. (3), by direct sums over all pairs; also rho and e_i. */
void orc_forces_direct(int64_t n, const double *x, const double *y, const double *z, double L,
                       const orc_pot *p, double *rho, double *fx, double *fy, double *fz,
                       double *e_atom)
{
    double rc2 = p->rc * p->rc;
    double *Fp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double f, df;
                pot_dens(p, sqrt(r2), &f, &df);
                s += f;
            }
        }
        rho[i] = s;
        double F, ddF;
        pot_embed(p, s, &F, &Fp[i], &ddF);
        e_atom[i] = F;
    }
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double r = sqrt(r2), v, dv, f, df;
                pot_pair(p, r, &v, &dv);
                pot_dens(p, r, &f, &df);
                double coef = ((Fp[i] + Fp[j]) * df + dv) / r;
                ax += coef * dx;
                ay += coef * dy;
                az += coef * dz;
                ep += 0.5 * v;
            }
        }
        fx[i] = ax;
        fy[i] = ay;
        fz[i] = az;
        e_atom[i] += ep;
    }
    free(Fp);
}

/* Sampled evaluation for large systems: for each listed atom idx[s], its
 * density, per-atom energy and force, from linked cells of edge >= rc.
 * The densities of the neighbours of each sampled atom are evaluated the
 * same way, so no full pass over the system is needed. */
void orc_sample_forces(int64_t n, const double *x, const double *y, const double *z, double L,
                       const orc_pot *p, int64_t nsample, const int64_t *idx, double *rho_out,
                       double *fx, double *fy, double *fz, double *e_atom)
{
    orc_cells cl;
    cells_build(&cl, n, x, y, z, L, p->rc);
    double rc2 = p->rc * p->rc;
    const int cap = 4096;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsample; ++s) {
        int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * cap);
        int32_t *nb2 = (int32_t *)malloc(sizeof(int32_t) * cap);
        int64_t i = idx[s];
        int tot;
        int m = cells_query(&cl, x, y, z, L, i, rc2, nb, cap, &tot);
        double rho_i = 0.0;
        for (int k = 0; k < m; ++k) {
            double dx, dy, dz, f, df;
            pot_dens(p, sqrt(sep2(x, y, z, i, nb[k], L, &dx, &dy, &dz)), &f, &df);
            rho_i += f;
        }
        double Fi, Fpi, Fppi;
        pot_embed(p, rho_i, &Fi, &Fpi, &Fppi);
        double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0;
        for (int k = 0; k < m; ++k) {
            int64_t j = nb[k];
            int tot2;
            int m2 = cells_query(&cl, x, y, z, L, j, rc2, nb2, cap, &tot2);
            double rho_j = 0.0;
            for (int q = 0; q < m2; ++q) {
                double dx, dy, dz, f, df;
                pot_dens(p, sqrt(sep2(x, y, z, j, nb2[q], L, &dx, &dy, &dz)), &f, &df);
                rho_j += f;
            }
            double Fj, Fpj, Fppj;
            pot_embed(p, rho_j, &Fj, &Fpj, &Fppj);
            double dx, dy, dz;
            double r = sqrt(sep2(x, y, z, i, j, L, &dx, &dy, &dz));
            double v, dv, f, df;
            pot_pair(p, r, &v, &dv);
            pot_dens(p, r, &f, &df);
            double coef = ((Fpi + Fpj) * df + dv) / r;
            ax += coef * dx;
            ay += coef * dy;
            az += coef * dz;
            ep += 0.5 * v;
        }
        rho_out[s] = rho_i;
        fx[s] = ax;
        fy[s] = ay;
        fz[s] = az;
        e_atom[s] = Fi + ep;
        free(nb);
        free(nb2);
    }
    cells_free(&cl);
}

/* Sampled neighbour rows: ascending ids within rlist for each idx[s]. */
void orc_sample_list(int64_t n, const double *x, const double *y, const double *z, double L,
                     double rlist, int64_t nsample, const int64_t *idx, int maxn, int32_t *count,
                     int32_t *ids)
{
    orc_cells cl;
    cells_build(&cl, n, x, y, z, L, rlist);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < nsample; ++s) {
        int tot;
        cells_query(&cl, x, y, z, L, idx[s], rlist * rlist, ids + s * maxn, maxn, &tot);
        count[s] = tot;
    }
    cells_free(&cl);
}

/* --------------------------------------------------------- velocity Verlet */

/* List radius of a box: rc + skin, kept below half the box length so that
 * the minimum image is unique. */
double orc_rlist(double rc, double skin, double L)
{
    double r = rc + skin;
    double half = 0.5 * L - 1e-9;
    return r < half ? r : half;
}

typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz;
    double L, mass, dt, skin;
    const orc_pot *p;
    int maxn;
} orc_md;

static int md_rebuild(orc_md *s, double rlist, int32_t *count, int32_t *ids, double *xr,
                      double *yr, double *zr)
{
    orc_wrap(s->n, s->x, s->y, s->z, s->L);
    int worst = orc_list_cells(s->n, s->x, s->y, s->z, s->L, rlist, s->maxn, count, ids);
    memcpy(xr, s->x, sizeof(double) * s->n);
    memcpy(yr, s->y, sizeof(double) * s->n);
    memcpy(zr, s->z, sizeof(double) * s->n);
    return worst > s->maxn ? -1 : 0;
}

static double md_forces(orc_md *s, const int32_t *count, const int32_t *ids, double *rho,
                        double *F, double *Fp, double *fx, double *fy, double *fz, double *e)
{
    orc_density(s->n, s->x, s->y, s->z, s->L, s->p, count, ids, s->maxn, rho);
    orc_embed(s->n, s->p, rho, F, Fp, NULL);
    orc_forces(s->n, s->x, s->y, s->z, s->L, s->p, count, ids, s->maxn, F, Fp, fx, fy, fz, e);
    double E = 0.0;
    for (int64_t i = 0; i < s->n; ++i) E += e[i];
    return E;
}

static double md_kinetic(const orc_md *s)
{
    double k = 0.0;
    for (int64_t i = 0; i < s->n; ++i)
        k += s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i] + s->vz[i] * s->vz[i];
    return 0.5 * s->mass * k / ORC_KAPPA;
}

/* nsteps of velocity Verlet (kick, drift, conditional rebuild, force, kick).
 * The list is rebuilt when some atom moved more than half the skin since the
 * last build.  epot/ekin (length nsteps+1, may be NULL) receive the energies
 * after each step (index 0: initial state).  Returns the number of rebuilds,
 * or -1 if a neighbour row overflowed maxn. */
int orc_vv(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
           double L, const orc_pot *p, double mass, double dt, double skin, int nsteps, int maxn,
           double *epot, double *ekin)
{
    orc_md s = {n, x, y, z, vx, vy, vz, L, mass, dt, skin, p, maxn};
    double rlist = orc_rlist(p->rc, skin, L);
    double half_skin = 0.5 * (rlist - p->rc);
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1) * maxn);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb);
    double *rho = malloc(nb), *F = malloc(nb), *Fp = malloc(nb);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb), *e = malloc(nb);
    int rebuilds = 0, bad = 0;
    bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
    double E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
    if (epot) epot[0] = E;
    if (ekin) ekin[0] = md_kinetic(&s);
    double c = 0.5 * dt * ORC_KAPPA / mass;
    for (int step = 1; step <= nsteps; ++step) {
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            double ddx = x[i] - xr[i], ddy = y[i] - yr[i], ddz = z[i] - zr[i];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 > worst) worst = d2;
        }
        if (worst > half_skin * half_skin) {
            bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
            ++rebuilds;
        }
        E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
        }
        if (epot) epot[step] = E;
        if (ekin) ekin[step] = md_kinetic(&s);
    }
    free(count); free(ids); free(xr); free(yr); free(zr);
    free(rho); free(F); free(Fp); free(fx); free(fy); free(fz); free(e);
    return bad ? -1 : rebuilds;
}

/* ------------------------------------------------------------- atom states */

/*
 * Atom states (Section 3.1): an atom marked frozen is not allowed to move.
 * It keeps zero velocity (its velocity is zeroed at the start and after
 * every kick), so the drift leaves it in place; it still exerts and feels
 * forces, which act on the free atoms.  Otherwise as orc_vv.
 */
int orc_vv_frozen(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                  double L, const orc_pot *p, double mass, double dt, double skin, int nsteps,
                  int maxn, const uint8_t *frozen, double *epot, double *ekin)
{
    orc_md s = {n, x, y, z, vx, vy, vz, L, mass, dt, skin, p, maxn};
    double rlist = orc_rlist(p->rc, skin, L);
    double half_skin = 0.5 * (rlist - p->rc);
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1) * maxn);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb);
    double *rho = malloc(nb), *F = malloc(nb), *Fp = malloc(nb);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb), *e = malloc(nb);
    for (int64_t i = 0; i < n; ++i)
        if (frozen[i]) vx[i] = vy[i] = vz[i] = 0.0;
    int rebuilds = 0, bad = 0;
    bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
    double E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
    if (epot) epot[0] = E;
    if (ekin) ekin[0] = md_kinetic(&s);
    double c = 0.5 * dt * ORC_KAPPA / mass;
    for (int step = 1; step <= nsteps; ++step) {
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (frozen[i]) continue;
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            double ddx = x[i] - xr[i], ddy = y[i] - yr[i], ddz = z[i] - zr[i];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 > worst) worst = d2;
        }
        if (worst > half_skin * half_skin) {
            bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
            ++rebuilds;
        }
        E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
        for (int64_t i = 0; i < n; ++i) {
            if (frozen[i]) continue;
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
        }
        if (epot) epot[step] = E;
        if (ekin) ekin[step] = md_kinetic(&s);
    }
    free(count); free(ids); free(xr); free(yr); free(zr);
    free(rho); free(F); free(Fp); free(fx); free(fy); free(fz); free(e);
    return bad ? -1 : rebuilds;
}

/* ---------------------------------------------------------------- thermostat */

/*
 * Eq. (4): each atom exchanges energy with an electron gas held at T_e through
 * the friction -(m / tau) ((T_i - T_e) / T_i) v_i (the printed equation leaves
 * out the mass that makes the term a force), T_i = m v_i^2 / (3 k_B) being
 * the instantaneous temperature of atom i.  On its own the friction keeps the
 * direction of v_i and gives d(v^2)/dt = -(2 / tau) (v^2 - v_e^2) with
 * v_e^2 = 3 k_B T_e / m, so over a time t
 *     v^2(t) = v_e^2 + (v^2(0) - v_e^2) exp(-2 t / tau).
 * Velocity Verlet takes this flow exactly over each half step, outside the
 * force half kicks (friction, kick, drift, force, kick, friction), which is
 * stable for any tau and any T_i.  An atom at rest has no direction and is
 * left at rest.
 */
static const double ORC_KB = 8.617333262e-5; /* eV/K */

typedef struct {
    int on;
    double e;  /* exp(-dt / tau): the flow over half a step */
    double ve2; /* v_e^2 in the velocity units (Angstrom/fs)^2 */
} orc_thermo;

static orc_thermo thermo_of(double te, double tau, double dt, double mass)
{
    orc_thermo t = {0, 1.0, 0.0};
    if (tau > 0.0) {
        t.on = 1;
        t.e = exp(-dt / tau);
        t.ve2 = 3.0 * ORC_KB * te * ORC_KAPPA / mass;
    }
    return t;
}

static void friction_flow(orc_md *s, const orc_thermo *t)
{
    if (!t->on) return;
    for (int64_t i = 0; i < s->n; ++i) {
        double v2 = s->vx[i] * s->vx[i] + s->vy[i] * s->vy[i] + s->vz[i] * s->vz[i];
        if (v2 > 0.0) {
            double g = sqrt(t->e * v2 + (1.0 - t->e) * t->ve2) / sqrt(v2);
            s->vx[i] *= g;
            s->vy[i] *= g;
            s->vz[i] *= g;
        }
    }
}

/* Velocity Verlet with the electron-gas friction of eq. (4) (tau <= 0: none,
 * which is orc_vv).  Arguments and results as orc_vv. */
int orc_vv_thermo(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                  double L, const orc_pot *p, double mass, double dt, double skin, int nsteps,
                  int maxn, double te, double tau, double *epot, double *ekin)
{
    orc_md s = {n, x, y, z, vx, vy, vz, L, mass, dt, skin, p, maxn};
    orc_thermo th = thermo_of(te, tau, dt, mass);
    double rlist = orc_rlist(p->rc, skin, L);
    double half_skin = 0.5 * (rlist - p->rc);
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1) * maxn);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb);
    double *rho = malloc(nb), *F = malloc(nb), *Fp = malloc(nb);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb), *e = malloc(nb);
    int rebuilds = 0, bad = 0;
    bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
    double E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
    if (epot) epot[0] = E;
    if (ekin) ekin[0] = md_kinetic(&s);
    double c = 0.5 * dt * ORC_KAPPA / mass;
    for (int step = 1; step <= nsteps; ++step) {
        friction_flow(&s, &th);
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            double ddx = x[i] - xr[i], ddy = y[i] - yr[i], ddz = z[i] - zr[i];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 > worst) worst = d2;
        }
        if (worst > half_skin * half_skin) {
            bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
            ++rebuilds;
        }
        E = md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
        }
        friction_flow(&s, &th);
        if (epot) epot[step] = E;
        if (ekin) ekin[step] = md_kinetic(&s);
    }
    free(count); free(ids); free(xr); free(yr); free(zr);
    free(rho); free(F); free(Fp); free(fx); free(fy); free(fz); free(e);
    return bad ? -1 : rebuilds;
}

/* ------------------------------------------------------------------ pressure */

/*
 * Virial of eq. (6) for a periodic box.  Summing f_i . r_i over atoms is not
 * invariant under the periodic images, so the sum is taken in its pair form:
 * with the pair decomposition of eq. (3), f_i = sum_j f_ij and f_ji = -f_ij,
 * sum_i f_i . r_i = sum_{i<j} f_ij . r_ij with r_ij = r_i - r_j the minimum
 * image separation.  f_ij = -[(F'_i + F'_j) f'(r) + phi'(r)] r_ij / r, so
 *   W = -1/2 sum_i sum_{j in L_i, r < rc} [(F'_i + F'_j) f'(r_ij) + phi'(r_ij)] r_ij.
 * The pressure is then P = (N k_B T + W/3)/V with N k_B T = (2/3) E_kin,
 * i.e. P = (2 E_kin + W) / (3 V).
 */
double orc_virial(int64_t n, const double *x, const double *y, const double *z, double L,
                  const orc_pot *p, const int32_t *count, const int32_t *ids, int maxn,
                  const double *Fp)
{
    double rc2 = p->rc * p->rc;
    double w = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < count[i]; ++k) {
            int64_t j = ids[i * maxn + k];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double r = sqrt(r2), v, dv, f, df;
                pot_pair(p, r, &v, &dv);
                pot_dens(p, r, &f, &df);
                w += ((Fp[i] + Fp[j]) * df + dv) * r;
            }
        }
    }
    return -0.5 * w;
}

/* The same virial by a direct sum over all pairs (densities included). */
double orc_virial_direct(int64_t n, const double *x, const double *y, const double *z, double L,
                         const orc_pot *p)
{
    double rc2 = p->rc * p->rc;
    double *Fp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double f, df;
                pot_dens(p, sqrt(r2), &f, &df);
                s += f;
            }
        }
        double F, ddF;
        pot_embed(p, s, &F, &Fp[i], &ddF);
    }
    double w = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 < rc2) {
                double r = sqrt(r2), v, dv, f, df;
                pot_pair(p, r, &v, &dv);
                pot_dens(p, r, &f, &df);
                w -= ((Fp[i] + Fp[j]) * df + dv) * r;
            }
        }
    free(Fp);
    return w;
}

/*
 * Velocity Verlet with the Berendsen barostat of eq. (5).  Every step: half
 * kick, drift, then every coordinate and the box edge are multiplied by
 * mu = [1 - beta (dt / tau) (P0 - P)]^(1/3), with P the pressure of eq. (6)
 * at the end of the previous step (for the first step, of the initial state);
 * conditional rebuild, forces, half kick, new pressure.  The paper writes
 * eq. (5) without the compressibility beta (beta = 1 in its units).
 * The list radius is fixed from the initial box; the reference positions of
 * the rebuild test are scaled with the coordinates, and the list is rebuilt
 * when 2 max|x - x_ref| + |1 - s| r_list reaches r_list - rc, with s the
 * product of the scale factors since the last build (pair separations that
 * were >= r_list at the build are then still >= rc).
 * With tau_t > 0 the friction of eq. (4) is applied as in orc_vv_thermo (its
 * flow before the first half kick and after the second, the pressure taken
 * after it).
 * L (in/out) is the box edge; press (length nsteps+1, may be NULL) receives
 * the pressures.  Returns the number of rebuilds, or -1 on row overflow.
 */
int orc_vv_baro(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                double *Lio, const orc_pot *p, double mass, double dt, double skin, int nsteps,
                int maxn, double p0, double tau, double beta, double te, double tau_t,
                double *press)
{
    double L = *Lio;
    orc_md s = {n, x, y, z, vx, vy, vz, L, mass, dt, skin, p, maxn};
    orc_thermo th = thermo_of(te, tau_t, dt, mass);
    double rlist = orc_rlist(p->rc, skin, L);
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1) * maxn);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb);
    double *rho = malloc(nb), *F = malloc(nb), *Fp = malloc(nb);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb), *e = malloc(nb);
    int rebuilds = 0, bad = 0;
    bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
    md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
    double W = orc_virial(n, x, y, z, s.L, p, count, ids, maxn, Fp);
    double P = (2.0 * md_kinetic(&s) + W) / (3.0 * s.L * s.L * s.L);
    if (press) press[0] = P;
    double c = 0.5 * dt * ORC_KAPPA / mass, strain = 1.0;
    for (int step = 1; step <= nsteps; ++step) {
        double mu = cbrt(1.0 - beta * (dt / tau) * (p0 - P));
        friction_flow(&s, &th);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            x[i] *= mu;
            y[i] *= mu;
            z[i] *= mu;
            xr[i] *= mu;
            yr[i] *= mu;
            zr[i] *= mu;
        }
        s.L *= mu;
        strain *= mu;
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double ddx = x[i] - xr[i], ddy = y[i] - yr[i], ddz = z[i] - zr[i];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 > worst) worst = d2;
        }
        double half = 0.5 * ((rlist - p->rc) - fabs(1.0 - strain) * rlist);
        if (half < 0.0 || worst > half * half) {
            bad |= md_rebuild(&s, rlist, count, ids, xr, yr, zr);
            strain = 1.0;
            ++rebuilds;
        }
        md_forces(&s, count, ids, rho, F, Fp, fx, fy, fz, e);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c * fx[i];
            vy[i] += c * fy[i];
            vz[i] += c * fz[i];
        }
        friction_flow(&s, &th);
        W = orc_virial(n, x, y, z, s.L, p, count, ids, maxn, Fp);
        P = (2.0 * md_kinetic(&s) + W) / (3.0 * s.L * s.L * s.L);
        if (press) press[step] = P;
    }
    *Lio = s.L;
    free(count); free(ids); free(xr); free(yr); free(zr);
    free(rho); free(F); free(Fp); free(fx); free(fy); free(fz); free(e);
    return bad ? -1 : rebuilds;
}

/* ----------------------------------------------------------- several species */

/*
 * Eqs. (1)-(3) with atom types, a the type of atom i and b that of atom j:
 *   rho_i = sum_j rho^(ab)(r_ij)    (density at an a atom contributed by a b atom)
 *   E_i   = F^(a)(rho_i) + 1/2 sum_j V^(ab)(r_ij)
 *   f_i   = -sum_j [F^(a)'(rho_i) rho^(ab)'(r) + F^(b)'(rho_j) rho^(ba)'(r)
 *                   + V^(ab)'(r)] (x_i - x_j) / r
 * The derivative of rho_j with respect to r_ij comes from the function that
 * builds rho_j, rho^(ba); eq. (3) as printed writes rho^(ab) in both places,
 * which is the same function when there is one species.  The embedding
 * function is taken per type of the embedded atom.  V^(ab) = V^(ba).
 * Tables are per-interval cubics on grids shared by all tables of one kind.
 *
 * Cutoffs per pair of types (Sections 3.2 and 3.3: RCUT(ity, jty)): a pair
 * of types a, b interacts while r < RCUT(a, b) (symmetric, at most rc), and
 * the neighbour list of an atom of type a holds the atoms j of type b with
 * r < RCUT(a, b) + skin (the list radius of the box, min(. + skin, L/2 -
 * 1e-9), taken per pair).  Without per-pair cutoffs every pair uses rc.
 */
typedef struct {
    int ntypes;
    double rc;
    const double *V;   /* [T*T][nint[0]][4], index a*T + b */
    const double *rho; /* [T*T][nint[1]][4], index a*T + b */
    const double *F;   /* [T][nint[2]][4] */
    int nint[3];
    double lo[3], hi[3];
    const double *rcp; /* [T*T] RCUT(a, b), index a*T + b, or NULL: rc for every pair */
} orc_alloy;

static double alloy_rc(const orc_alloy *p, int a, int b)
{
    return p->rcp ? p->rcp[a * p->ntypes + b] : p->rc;
}

static void alloy_fn(const orc_alloy *p, int which, int idx, double x, double *s, double *ds,
                     double *dds)
{
    const double *base = which == 0 ? p->V : (which == 1 ? p->rho : p->F);
    spline_eval(base + (size_t)idx * p->nint[which] * 4, p->nint[which], p->lo[which],
                p->hi[which], x, s, ds, dds);
}

/* Neighbour j of atom i: the k-th list entry, or (ids == NULL) the k-th atom
 * other than i in index order. */
static int64_t alloy_nb(const int32_t *ids, int maxn, int64_t i, int k)
{
    if (ids) return ids[i * maxn + k];
    return k < i ? k : k + 1;
}

/* rho, F, F' (any may be NULL except Fp), forces, per-atom energies and the
 * pair virial W = -1/2 sum_i sum_j [...] r of eq. (6), for one box.  With
 * ids == NULL every pair is visited (minimum image); else the list. */
double orc_alloy_eval(int64_t n, const double *x, const double *y, const double *z, double L,
                      const orc_alloy *p, const int32_t *type, const int32_t *count,
                      const int32_t *ids, int maxn, double *rho_out, double *F_out, double *Fp,
                      double *fx, double *fy, double *fz, double *e_atom)
{
    const int T = p->ntypes;
    double *rho = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *Fe = malloc(sizeof(double) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int cnt = ids ? count[i] : (int)(n - 1);
        double s = 0.0;
        for (int k = 0; k < cnt; ++k) {
            int64_t j = alloy_nb(ids, maxn, i, k);
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            double rc = alloy_rc(p, type[i], type[j]);
            if (r2 < rc * rc) {
                double f, df, dd;
                alloy_fn(p, 1, type[i] * T + type[j], sqrt(r2), &f, &df, &dd);
                s += f;
            }
        }
        rho[i] = s;
        double dd;
        alloy_fn(p, 2, type[i], s, &Fe[i], &Fp[i], &dd);
    }
    double W = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : W)
    for (int64_t i = 0; i < n; ++i) {
        int cnt = ids ? count[i] : (int)(n - 1);
        int a = type[i];
        double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0, w = 0.0;
        for (int k = 0; k < cnt; ++k) {
            int64_t j = alloy_nb(ids, maxn, i, k);
            int b = type[j];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            double rc = alloy_rc(p, a, b);
            if (r2 < rc * rc) {
                double r = sqrt(r2), dd;
                double v, dv, fab, dfab, fba, dfba;
                alloy_fn(p, 0, a * T + b, r, &v, &dv, &dd);
                alloy_fn(p, 1, a * T + b, r, &fab, &dfab, &dd);
                alloy_fn(p, 1, b * T + a, r, &fba, &dfba, &dd);
                double g = Fp[i] * dfab + Fp[j] * dfba + dv;
                double coef = g / r;
                /* (x_i - x_j) = -(dx, dy, dz) */
                ax += coef * dx;
                ay += coef * dy;
                az += coef * dz;
                ep += 0.5 * v;
                w += g * r;
            }
        }
        if (fx) { fx[i] = ax; fy[i] = ay; fz[i] = az; }
        if (e_atom) e_atom[i] = Fe[i] + ep;
        W += w;
    }
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * n);
    if (F_out) memcpy(F_out, Fe, sizeof(double) * n);
    free(rho);
    free(Fe);
    return -0.5 * W;
}

/* Neighbour list of one box with the list radius taken per pair of types:
 * the cell list at the largest radius (that of rc), then each row keeps, in
 * ascending order, the j with r^2 < rl(a, b)^2, rl(a, b) = min(RCUT(a, b) +
 * skin, L/2 - 1e-9).  Returns the longest row before the filter (> maxn:
 * overflow). */
int orc_alloy_list(int64_t n, const double *x, const double *y, const double *z, double L,
                   const orc_alloy *p, const int32_t *type, double skin, int maxn, int32_t *count,
                   int32_t *ids)
{
    int worst = orc_list_cells(n, x, y, z, L, orc_rlist(p->rc, skin, L), maxn, count, ids);
    if (worst > maxn || !p->rcp) return worst;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t *row = ids + i * maxn;
        int k = 0;
        for (int m = 0; m < count[i]; ++m) {
            int64_t j = row[m];
            double rl = orc_rlist(alloy_rc(p, type[i], type[j]), skin, L);
            double dx, dy, dz;
            if (sep2(x, y, z, i, j, L, &dx, &dy, &dz) < rl * rl) row[k++] = (int32_t)j;
        }
        count[i] = k;
    }
    return worst;
}

static int alloy_rebuild(orc_md *s, const orc_alloy *p, const int32_t *type, int32_t *count,
                         int32_t *ids, double *xr, double *yr, double *zr)
{
    orc_wrap(s->n, s->x, s->y, s->z, s->L);
    int worst = orc_alloy_list(s->n, s->x, s->y, s->z, s->L, p, type, s->skin, s->maxn, count,
                               ids);
    memcpy(xr, s->x, sizeof(double) * s->n);
    memcpy(yr, s->y, sizeof(double) * s->n);
    memcpy(zr, s->z, sizeof(double) * s->n);
    return worst > s->maxn ? -1 : 0;
}

static double alloy_kinetic(int64_t n, const double *vx, const double *vy, const double *vz,
                            const int32_t *type, const double *mass_t)
{
    double K = 0.0;
    for (int64_t i = 0; i < n; ++i)
        K += 0.5 * mass_t[type[i]] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) / ORC_KAPPA;
    return K;
}

/* The friction flow of eq. (4) over half a step (see orc_vv_thermo), with the
 * per-atom factors e = exp(-dt / tau) and v_e^2 of the atom's type. */
static void alloy_friction(int64_t n, double *vx, double *vy, double *vz, const double *ge,
                           const double *gv2)
{
    for (int64_t i = 0; i < n; ++i) {
        double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        if (v2 > 0.0) {
            double g = sqrt(ge[i] * v2 + (1.0 - ge[i]) * gv2[i]) / sqrt(v2);
            vx[i] *= g;
            vy[i] *= g;
            vz[i] *= g;
        }
    }
}

/* Velocity Verlet for several species: atom i has mass mass_t[type[i]]; with
 * tau > 0 the electron-gas friction of eq. (4) as in orc_vv_thermo, with
 * v_e^2 = 3 k_B T_e / m of the atom's type.  Otherwise as orc_vv. */
int orc_alloy_vv(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                 double L, const orc_alloy *p, const int32_t *type, const double *mass_t,
                 double dt, double skin, int nsteps, int maxn, double te, double tau,
                 double *epot, double *ekin)
{
    double rlist = orc_rlist(p->rc, skin, L);
    double half_skin = 0.5 * (rlist - p->rc);
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1) * maxn);
    double *xr = malloc(nb), *yr = malloc(nb), *zr = malloc(nb), *c = malloc(nb);
    double *Fp = malloc(nb), *e = malloc(nb);
    double *fx = malloc(nb), *fy = malloc(nb), *fz = malloc(nb);
    double *ge = malloc(nb), *gv2 = malloc(nb);
    orc_md s = {n, x, y, z, vx, vy, vz, L, 0.0, dt, skin, NULL, maxn};
    for (int64_t i = 0; i < n; ++i) {
        double m = mass_t[type[i]];
        c[i] = 0.5 * dt * ORC_KAPPA / m;
        orc_thermo th = thermo_of(te, tau, dt, m);
        ge[i] = th.e;
        gv2[i] = th.ve2;
    }
    int on = tau > 0.0;
    int rebuilds = 0, bad = 0;
    bad |= alloy_rebuild(&s, p, type, count, ids, xr, yr, zr);
    orc_alloy_eval(n, x, y, z, L, p, type, count, ids, maxn, NULL, NULL, Fp, fx, fy, fz, e);
    if (epot) {
        epot[0] = 0.0;
        for (int64_t i = 0; i < n; ++i) epot[0] += e[i];
    }
    if (ekin) ekin[0] = alloy_kinetic(n, vx, vy, vz, type, mass_t);
    for (int step = 1; step <= nsteps; ++step) {
        if (on) alloy_friction(n, vx, vy, vz, ge, gv2);
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c[i] * fx[i];
            vy[i] += c[i] * fy[i];
            vz[i] += c[i] * fz[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            double ddx = x[i] - xr[i], ddy = y[i] - yr[i], ddz = z[i] - zr[i];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (d2 > worst) worst = d2;
        }
        if (worst > half_skin * half_skin) {
            bad |= alloy_rebuild(&s, p, type, count, ids, xr, yr, zr);
            ++rebuilds;
        }
        orc_alloy_eval(n, x, y, z, L, p, type, count, ids, maxn, NULL, NULL, Fp, fx, fy, fz, e);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += c[i] * fx[i];
            vy[i] += c[i] * fy[i];
            vz[i] += c[i] * fz[i];
        }
        if (on) alloy_friction(n, vx, vy, vz, ge, gv2);
        if (epot) {
            epot[step] = 0.0;
            for (int64_t i = 0; i < n; ++i) epot[step] += e[i];
        }
        if (ekin) ekin[step] = alloy_kinetic(n, vx, vy, vz, type, mass_t);
    }
    free(count); free(ids); free(xr); free(yr); free(zr); free(c);
    free(Fp); free(e); free(fx); free(fy); free(fz); free(ge); free(gv2);
    return bad ? -1 : rebuilds;
}

/* ------------------------------------------------------------------ adjoint */

/*
 * Vector-Jacobian product of (forces, box energy) with respect to the
 * B-spline coefficients of phi, f and F, for one box.
 *
 * Given g_i = dL/df_i and e = dL/dE, vary the three functions at fixed
 * positions in eqs. (2)-(3).  With u_ij = (x_i - x_j)/r_ij, c_ij = g_i . u_ij
 * and full (symmetric) neighbour sets:
 *   s_i      = sum_j f'(r_ij) (g_i - g_j) . u_ij
 *   lambda_i = e F'(rho_i) - F''(rho_i) s_i
 *   dL/dphi_k = sum_{i->j} [ e/2 B_k(r_ij) - B'_k(r_ij) c_ij ]
 *   dL/df_k   = sum_{i->j} [ lambda_i B_k(r_ij) - (F'_i + F'_j) B'_k(r_ij) c_ij ]
 *   dL/dF_k   = sum_i [ e C_k(rho_i) - C'_k(rho_i) s_i ]
 * where B_k, C_k are the B-spline basis functions of the r and rho grids.
 * The terms with F'(rho_j) come from swapping i and j in the sum of eq. (3).
 * gtheta[0:K] (phi), [K:2K] (f), [2K:3K] (F) are accumulated (+=).
 */
void orc_adjoint(int64_t n, const double *x, const double *y, const double *z, double L,
                 const orc_pot *p, const int32_t *count, const int32_t *ids, int maxn,
                 const double *gx, const double *gy, const double *gz, double e, double *gtheta)
{
    int K = p->ntab[0]; /* coefficients per function (equal for the three) */
    double rc2 = p->rc * p->rc;
    size_t nb = sizeof(double) * (n > 0 ? n : 1);
    double *rho = malloc(nb), *F = malloc(nb), *Fp = malloc(nb), *Fpp = malloc(nb);
    double *sv = malloc(nb);
    orc_density(n, x, y, z, L, p, count, ids, maxn, rho);
    orc_embed(n, p, rho, F, Fp, Fpp);
    /* s_i */
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < count[i]; ++k) {
            int64_t j = ids[i * maxn + k];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 >= rc2) continue;
            double r = sqrt(r2), f, df;
            pot_dens(p, r, &f, &df);
            double ux = -dx / r, uy = -dy / r, uz = -dz / r;
            s += df * ((gx[i] - gx[j]) * ux + (gy[i] - gy[j]) * uy + (gz[i] - gz[j]) * uz);
        }
        sv[i] = s;
    }
    double *gphi = gtheta, *gf = gtheta + K, *gF = gtheta + 2 * K;
    for (int64_t i = 0; i < n; ++i) {
        double lam = e * Fp[i] - Fpp[i] * sv[i];
        for (int k = 0; k < count[i]; ++k) {
            int64_t j = ids[i * maxn + k];
            double dx, dy, dz;
            double r2 = sep2(x, y, z, i, j, L, &dx, &dy, &dz);
            if (r2 >= rc2) continue;
            double r = sqrt(r2);
            double cij = -(gx[i] * dx + gy[i] * dy + gz[i] * dz) / r;
            int m;
            double t, h, b[4], db[4], ddb[4];
            bspline_locate(K, p->lo[0], p->hi[0], r, &m, &t, &h);
            bspline_basis(t, b, db, ddb);
            for (int l = 0; l < 4; ++l) gphi[m + l] += 0.5 * e * b[l] - db[l] / h * cij;
            bspline_locate(p->ntab[1], p->lo[1], p->hi[1], r, &m, &t, &h);
            bspline_basis(t, b, db, ddb);
            for (int l = 0; l < 4; ++l)
                gf[m + l] += lam * b[l] - (Fp[i] + Fp[j]) * db[l] / h * cij;
        }
        int m;
        double t, h, b[4], db[4], ddb[4];
        bspline_locate(p->ntab[2], p->lo[2], p->hi[2], rho[i], &m, &t, &h);
        bspline_basis(t, b, db, ddb);
        for (int l = 0; l < 4; ++l) gF[m + l] += e * b[l] - db[l] / h * sv[i];
    }
    free(rho); free(F); free(Fp); free(Fpp); free(sv);
}

/* Number of OpenMP threads the oracle's parallel loops use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
