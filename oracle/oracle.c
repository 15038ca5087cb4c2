/*
 * oracle.c -- plain, slow FP64 CPU reference for the short-range non-bonded
 * path.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark, never by the product
 * library, and it shares no code, header or constant table with it.
 *
 * What it computes (the plain definitions the cluster-pair method reaches):
 *  - the pair set P(r_list): every unordered atom pair {i,j}, i != j, whose
 *    minimum-image distance is inside the buffered list radius.  The paper
 *    defines the cluster-pair list as holding all cluster pairs with atoms that
 *    may be close enough to interact, constructed with a buffer (Section "SIMD
 *    parallelism"); the set of atom pairs it covers within r_list is this set.
 *  - forces, energies and virial of all pairs inside the spherical cut-off
 *    (Section "Introduction": non-bonded van der Waals and Coulomb interactions
 *    within a given spherical boundary), with Lennard-Jones 12-6 plus
 *    reaction-field or Ewald real-space Coulomb.  The paper writes no formula;
 *    the textbook forms used are listed in the project's design notes.
 *  - a velocity-Verlet trajectory (Section "Introduction": positions and
 *    velocities updated from the forces via Newton's second law with a finite
 *    time step).
 *
 * Every loop is an O(N^2) loop over all pairs, in FP64, with the minimum image
 * of a rectangular or triclinic box (min_image_r2).  Build with -ffp-contract=off so that the pair-set
 * criterion is evaluated with separately rounded IEEE-754 operations.
 * OpenMP parallelises over i only (each thread writes only its own rows), so
 * results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 1/(4 pi eps0) in kJ mol^-1 nm e^-2 (conventional MD value). */
#define ORACLE_ONE_4PI_EPS0 138.935458
#define ORACLE_SQRT_PI 1.7724538509055160273

/* ---------------------------------------------------------------------- */
/* Periodic box: lattice vectors a = (box[0], 0, 0), b = (box[3], box[1], 0), */
/* c = (box[4], box[5], box[2]) -- rectangular when box[3..5] are 0, a       */
/* rhombic dodecahedron or another triclinic cell otherwise (the paper runs  */
/* rectangular and rhombic-dodecahedron boxes, Fig. 6).  invbox[k] = 1 /     */
/* box[k] for k < 3.                                                         */
/* Minimum image: d = x_j - x_i, then the multiples of c, b and a nearest to */
/* d's z, y and x components are removed, in that order:                     */
/*   k = rint(d_z / c_z), d -= k c;  k = rint(d_y / b_y), d -= k b;          */
/*   k = rint(d_x / a_x), d -= k a.                                          */
/* Each step leaves the earlier components alone, so the result has          */
/* |d_x| <= a_x/2, |d_y| <= b_y/2, |d_z| <= c_z/2, which makes it the        */
/* shortest image of every pair closer than half the smallest of a_x, b_y,   */
/* c_z.  In a rectangular box this is the per-dimension minimum image.       */
/* r^2 = (dx*dx + dy*dy) + dz*dz.                                            */
/* ---------------------------------------------------------------------- */
static double min_image_r2(const double *xi, const double *xj, const double *box,
                           const double *invbox, double d[3])
{
    for (int k = 0; k < 3; ++k) d[k] = xj[k] - xi[k];
    double kc = nearbyint(d[2] * invbox[2]);
    d[0] = d[0] - kc * box[4];
    d[1] = d[1] - kc * box[5];
    d[2] = d[2] - kc * box[2];
    double kb = nearbyint(d[1] * invbox[1]);
    d[0] = d[0] - kb * box[3];
    d[1] = d[1] - kb * box[1];
    double ka = nearbyint(d[0] * invbox[0]);
    d[0] = d[0] - ka * box[0];
    double dxx = d[0] * d[0];
    double dyy = d[1] * d[1];
    double dzz = d[2] * d[2];
    double t = dxx + dyy;
    return t + dzz;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/*
 * oracle_pairs: the exact pair set.  {i,j} is in P iff r^2 < r_list^2 (strict,
 * r_list^2 computed as one FP64 product).  Pairs are written as (i, j) with
 * i < j, sorted lexicographically, at most `cap` of them; the return value is
 * the total count (also when it exceeds cap).  Returns -1 on bad arguments.
 */
int64_t oracle_pairs(int32_t n, const double *x, const double *box, const double *invbox,
                     double r_list, int32_t *pairs, int64_t cap, int32_t nthreads)
{
    if (n < 0 || !x || !box || !invbox) return -1;
    set_threads(nthreads);
    const double rl2 = r_list * r_list;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n; ++i) {
        int64_t c = 0;
        double d[3];
        for (int32_t j = i + 1; j < n; ++j)
            if (min_image_r2(x + 3 * i, x + 3 * j, box, invbox, d) < rl2) ++c;
        cnt[i + 1] = c;
    }
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    if (pairs && cap > 0) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int32_t i = 0; i < n; ++i) {
            int64_t p = cnt[i];
            double d[3];
            for (int32_t j = i + 1; j < n && p < cap; ++j)
                if (min_image_r2(x + 3 * i, x + 3 * j, box, invbox, d) < rl2) {
                    pairs[2 * p] = i;
                    pairs[2 * p + 1] = j;
                    ++p;
                }
        }
    }
    free(cnt);
    return total;
}

/* ---------------------------------------------------------------------- */
/* Interaction model                                                       */
/* ---------------------------------------------------------------------- */
typedef struct {
    double rc, rc2;
    int coulomb;   /* 0 none, 1 reaction field, 2 Ewald real space */
    double fel;    /* 1/(4 pi eps0 eps_r) */
    double krf, crf;
    double beta;
    double ew_shift; /* erfc(beta rc)/rc, 0 without potential shift */
    int lj;        /* 0 single C6/C12, 1 Lorentz-Berthelot from sigma/epsilon */
    double c6, c12;
    int pot_shift;
} model_t;

static void model_init(model_t *m, double rc, int coulomb, double eps_r, double eps_rf,
                       double beta, int lj, double c6, double c12, int pot_shift)
{
    m->rc = rc;
    m->rc2 = rc * rc;
    m->coulomb = coulomb;
    m->fel = ORACLE_ONE_4PI_EPS0 / eps_r;
    /* Reaction field: k_rf = (eps_rf - eps_r) / ((2 eps_rf + eps_r) rc^3), which is
     * 1/(2 rc^3) for eps_rf -> infinity; c_rf = 1/rc + k_rf rc^2 so that V(rc) = 0. */
    if (eps_rf <= 0.0)
        m->krf = 1.0 / (2.0 * rc * rc * rc);
    else
        m->krf = (eps_rf - eps_r) / ((2.0 * eps_rf + eps_r) * rc * rc * rc);
    m->crf = 1.0 / rc + m->krf * rc * rc;
    m->beta = beta;
    m->ew_shift = pot_shift ? erfc(beta * rc) / rc : 0.0;
    m->lj = lj;
    m->c6 = c6;
    m->c12 = c12;
    m->pot_shift = pot_shift;
}

/* One pair at squared distance r2 (< rc^2).  Returns the scalar s with
 * F_i = s * r_ij (r_ij = x_i - x_j), and the LJ and Coulomb energies. */
static double pair_interaction(const model_t *m, double r2, double qq, double c6, double c12,
                               double *vlj, double *vc)
{
    double r = sqrt(r2);
    double rinv = 1.0 / r;
    double rinv2 = rinv * rinv;
    double rinv6 = rinv2 * rinv2 * rinv2;
    /* LJ 12-6: V = C12/r^12 - C6/r^6; -dV/dr / r = (12 C12/r^12 - 6 C6/r^6)/r^2 */
    double v = c12 * rinv6 * rinv6 - c6 * rinv6;
    double s = (12.0 * c12 * rinv6 * rinv6 - 6.0 * c6 * rinv6) * rinv2;
    if (m->pot_shift) {
        double rc6 = 1.0 / (m->rc2 * m->rc2 * m->rc2);
        v -= c12 * rc6 * rc6 - c6 * rc6;
    }
    *vlj = v;
    double ec = 0.0;
    if (m->coulomb == 1) {
        /* V = f qq (1/r + k_rf r^2 - c_rf); -dV/dr / r = f qq (1/r^3 - 2 k_rf) */
        ec = m->fel * qq * (rinv + m->krf * r2 - m->crf);
        s += m->fel * qq * (rinv * rinv2 - 2.0 * m->krf);
    } else if (m->coulomb == 2) {
        /* V = f qq erfc(beta r)/r; -dV/dr / r = f qq (erfc(beta r)/r + 2 beta/sqrt(pi) exp(-beta^2 r^2)) / r^2 */
        double br = m->beta * r;
        double erfc_r = erfc(br) * rinv;
        ec = m->fel * qq * (erfc_r - m->ew_shift);
        s += m->fel * qq * (erfc_r + 2.0 * m->beta / ORACLE_SQRT_PI * exp(-br * br)) * rinv2;
    }
    *vc = ec;
    return s;
}

static void pair_lj_params(const model_t *m, const double *lja, const double *ljb, int32_t i,
                           int32_t j, double *c6, double *c12)
{
    if (m->lj == 1) {
        /* Lorentz-Berthelot: sigma_ij = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j) */
        double sig = 0.5 * (lja[i] + lja[j]);
        double eps = sqrt(ljb[i] * ljb[j]);
        double s6 = sig * sig * sig * sig * sig * sig;
        *c6 = 4.0 * eps * s6;
        *c12 = 4.0 * eps * s6 * s6;
    } else {
        *c6 = m->c6;
        *c12 = m->c12;
    }
}

/* Force, half the pair energies and a quarter of -r_ij (x) F_ij from every
 * partner j != i of atom i (full loop over j: each unordered pair is seen from
 * both ends, which adds up to the pair energy once and the virial
 * Xi = -1/2 sum_{i<j} r_ij (x) F_ij). */
static void atom_row(const model_t *m, int32_t n, const double *x, const double *q,
                     const double *lja, const double *ljb, const double *box,
                     const double *invbox, int32_t i, double f[3], double e[2], double vir[9])
{
    double fi[3] = {0, 0, 0}, elj = 0, ec = 0;
    double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3];
        double r2 = min_image_r2(x + 3 * i, x + 3 * j, box, invbox, d);
        if (!(r2 < m->rc2)) continue;
        double c6, c12, vlj, vc;
        pair_lj_params(m, lja, ljb, i, j, &c6, &c12);
        double s = pair_interaction(m, r2, q[i] * q[j], c6, c12, &vlj, &vc);
        /* d = x_j - x_i (min image), so r_ij = -d */
        double rij[3] = {-d[0], -d[1], -d[2]};
        for (int a = 0; a < 3; ++a) fi[a] += s * rij[a];
        elj += 0.5 * vlj;
        ec += 0.5 * vc;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) w[3 * a + b] += -0.25 * rij[a] * (s * rij[b]);
    }
    for (int a = 0; a < 3; ++a) f[a] = fi[a];
    e[0] = elj;
    e[1] = ec;
    for (int a = 0; a < 9; ++a) vir[a] = w[a];
}

/*
 * oracle_forces: f[N,3] (kJ/mol/nm), ener[2] = {E_LJ, E_coul} (kJ/mol),
 * vir[9] = Xi (row-major), all FP64.  lja/ljb are per-atom sigma/epsilon for
 * lj = 1 and ignored for lj = 0 (c6/c12 used).  Any output may be NULL.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_forces(int32_t n, const double *x, const double *q, const double *lja,
                  const double *ljb, const double *box, const double *invbox, double rc,
                  int32_t coulomb, double eps_r, double eps_rf, double beta, int32_t lj,
                  double c6, double c12, int32_t pot_shift, int32_t nthreads, double *f,
                  double *ener, double *vir)
{
    if (n < 0 || !x || !q || !box || !invbox) return -1;
    if (lj == 1 && (!lja || !ljb)) return -1;
    model_t m;
    model_init(&m, rc, coulomb, eps_r, eps_rf, beta, lj, c6, c12, pot_shift);
    set_threads(nthreads);
    double *rows = (double *)malloc(sizeof(double) * 14 * (size_t)(n > 0 ? n : 1));
    if (!rows) return -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int32_t i = 0; i < n; ++i) {
        double *r = rows + 14 * (size_t)i;
        atom_row(&m, n, x, q, lja, ljb, box, invbox, i, r, r + 3, r + 5);
    }
    double e[2] = {0, 0}, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t i = 0; i < n; ++i) {
        const double *r = rows + 14 * (size_t)i;
        if (f) for (int a = 0; a < 3; ++a) f[3 * i + a] = r[a];
        e[0] += r[3];
        e[1] += r[4];
        for (int a = 0; a < 9; ++a) w[a] += r[5 + a];
    }
    if (ener) { ener[0] = e[0]; ener[1] = e[1]; }
    if (vir) for (int a = 0; a < 9; ++a) vir[a] = w[a];
    free(rows);
    return 0;
}

/*
 * oracle_forces_subset: forces on the atoms listed in idx[0..nidx) only
 * (f_sub[nidx,3]), and each listed atom's half pair energies (e_sub[nidx,2],
 * may be NULL).  Same O(N) loop per listed atom as oracle_forces.
 */
int oracle_forces_subset(int32_t n, const double *x, const double *q, const double *lja,
                         const double *ljb, const double *box, const double *invbox, double rc,
                         int32_t coulomb, double eps_r, double eps_rf, double beta, int32_t lj,
                         double c6, double c12, int32_t pot_shift, int32_t nthreads,
                         const int32_t *idx, int32_t nidx, double *f_sub, double *e_sub)
{
    if (n < 0 || nidx < 0 || !x || !q || !box || !invbox || !idx || !f_sub) return -1;
    if (lj == 1 && (!lja || !ljb)) return -1;
    for (int32_t k = 0; k < nidx; ++k)
        if (idx[k] < 0 || idx[k] >= n) return -1;
    model_t m;
    model_init(&m, rc, coulomb, eps_r, eps_rf, beta, lj, c6, c12, pot_shift);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t k = 0; k < nidx; ++k) {
        double e[2], w[9];
        atom_row(&m, n, x, q, lja, ljb, box, invbox, idx[k], f_sub + 3 * (size_t)k, e, w);
        if (e_sub) { e_sub[2 * k] = e[0]; e_sub[2 * k + 1] = e[1]; }
    }
    return 0;
}

/*
 * oracle_md: velocity Verlet in FP64 with all-pairs forces recomputed every
 * step (no list).  Per step: v += dt/2 F/m; x += dt v; F = F(x); v += dt/2 F/m.
 * x[N,3] and v[N,3] are updated in place.  trace[nsteps,4] (may be NULL)
 * receives E_LJ, E_coul, E_kin, E_total after each step.
 */
int oracle_md(int32_t n, double *x, double *v, const double *mass, const double *q,
              const double *lja, const double *ljb, const double *box, const double *invbox,
              double rc, int32_t coulomb, double eps_r, double eps_rf, double beta, int32_t lj,
              double c6, double c12, int32_t pot_shift, int32_t nthreads, double dt,
              int32_t nsteps, double *trace)
{
    if (n < 0 || nsteps < 0 || !x || !v || !mass) return -1;
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!f) return -1;
    double e[2];
    if (oracle_forces(n, x, q, lja, ljb, box, invbox, rc, coulomb, eps_r, eps_rf, beta, lj, c6,
                      c12, pot_shift, nthreads, f, e, NULL) != 0) {
        free(f);
        return -1;
    }
    for (int32_t s = 0; s < nsteps; ++s) {
        for (int32_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                v[3 * i + a] += 0.5 * dt * f[3 * i + a] / mass[i];
                x[3 * i + a] += dt * v[3 * i + a];
            }
        oracle_forces(n, x, q, lja, ljb, box, invbox, rc, coulomb, eps_r, eps_rf, beta, lj, c6,
                      c12, pot_shift, nthreads, f, e, NULL);
        double ke = 0.0;
        for (int32_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                v[3 * i + a] += 0.5 * dt * f[3 * i + a] / mass[i];
                ke += 0.5 * mass[i] * v[3 * i + a] * v[3 * i + a];
            }
        if (trace) {
            trace[4 * s] = e[0];
            trace[4 * s + 1] = e[1];
            trace[4 * s + 2] = ke;
            trace[4 * s + 3] = e[0] + e[1] + ke;
        }
    }
    free(f);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
