/*
 * FP64 CPU oracle for the short-range coarse-grained MD step of ESPResSo++
 * (arXiv 2608.14911).  TEST INFRASTRUCTURE ONLY: nothing on the product path
 * may link, load or call this file.  It shares no code with the HIP library.
 *
 * What the paper fixes and what this file restates in plain code:
 *   - Verlet neighbour lists with a skin over linked cells
 *     (section "Software design", paragraphs on VerletList / CellGrid, and the
 *     "Example usage" script: VerletList(cutoff=rc), system.skin);
 *   - the truncated, energy-shifted Lennard-Jones potential with shift='auto'
 *     and its capped variant LennardJonesCapped(caprad) used for push-off
 *     ("Example usage");
 *   - bonded interactions ("Functionality": bonded interactions), here the
 *     FENE bond and the cosine bending angle of the Kremer-Grest melt;
 *   - VelocityVerlet with the LangevinThermostat extension ("Example usage",
 *     "Software design": integrator extensions).
 * The paper prints no formulas; the closed forms below are the textbook ones
 * that those class names denote.  Readings where the paper is silent:
 *   - minimum image by compare-and-shift (no rint, no division);
 *   - r^2 = (dx*dx + dy*dy) + dz*dz with no fused multiply-add (built with
 *     -ffp-contract=off) so neighbour sets are exactly reproducible;
 *   - cutoffs strict: interacting iff r^2 < rc^2, listed iff r^2 < rv^2;
 *   - Langevin force inside velocity Verlet:
 *       F_tot = F(x_n) - gamma m v' + sqrt(2 gamma m kT / dt) xi_n,
 *     v' the half-step velocity (the on-step velocity before the first step);
 *   - noise xi from Philox4x64-10 (Salmon et al. 2011), key (seed, stream),
 *     counter (step, tag, 0, 0), Box-Muller in FP64.
 * Plain loops, FP64 throughout.  The linked-cell force path is the paper's own
 * cell decomposition; the brute-force path is its O(N^2) definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_BOND_BROKEN -5
#define ORC_ERR_NONFINITE -6
#define ORC_ERR_NL_OVERFLOW -4

/* ------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).              */
/* ------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        __uint128_t p0 = (__uint128_t)PHILOX_M0 * x0;
        __uint128_t p1 = (__uint128_t)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Philox4x32-10 (the same paper): four 32-bit words, 10 rounds of two
 * 32x32->64 multiplies by the published multipliers, the key bumped by the
 * published Weyl constants between rounds. */
static const uint32_t PHILOX32_M0 = 0xD2511F53u;
static const uint32_t PHILOX32_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX32_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX32_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX32_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX32_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0; x1 = lo1; x2 = n2; x3 = lo0;
        k0 += PHILOX32_W0;
        k1 += PHILOX32_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in the open interval (0,1) from the top 53 bits */
static double u01_open(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

/* Three standard normals for (seed, stream, step, tag): Box-Muller on the
 * four uniforms of one Philox block; the fourth normal is discarded. */
void orc_gauss3(uint64_t seed, uint64_t stream, uint64_t step, uint64_t tag, double out[3]) {
    uint64_t ctr[4] = {step, tag, 0, 0};
    uint64_t key[2] = {seed, stream};
    uint64_t r[4];
    orc_philox4x64_10(ctr, key, r);
    double u0 = u01_open(r[0]), u1 = u01_open(r[1]);
    double u2 = u01_open(r[2]), u3 = u01_open(r[3]);
    const double two_pi = 6.283185307179586;
    double rad0 = sqrt(-2.0 * log(u0));
    double rad1 = sqrt(-2.0 * log(u2));
    out[0] = rad0 * cos(two_pi * u1);
    out[1] = rad0 * sin(two_pi * u1);
    out[2] = rad1 * cos(two_pi * u3);
}

/* ------------------------------------------------------------------ */
/* Pair potential: truncated LJ, energy shift (auto = u(rc)), optional */
/* capping radius below which u and |f| are frozen at their cap values. */
/* pp layout per type pair: eps, sigma, rc, shift (NaN = auto), caprad */
/* ------------------------------------------------------------------ */
typedef struct { double eps, sigma, rc, shift, caprad; } orc_pair;

static double lj_shift(const orc_pair* p) {
    if (!isnan(p->shift)) return p->shift;
    double s2 = (p->sigma * p->sigma) / (p->rc * p->rc);
    double s6 = s2 * s2 * s2;
    return 4.0 * p->eps * (s6 * s6 - s6);
}

/* For r2 < rc^2: energy u and f_over_r with force on i = f_over_r * (r_i - r_j). */
static void lj_eval(const orc_pair* p, double r2, double* u, double* f_over_r) {
    double re2 = r2;
    int capped = (p->caprad > 0.0) && (r2 < p->caprad * p->caprad);
    if (capped) re2 = p->caprad * p->caprad;
    double s2 = (p->sigma * p->sigma) / re2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    *u = 4.0 * p->eps * (s12 - s6) - lj_shift(p);
    double f_over_re = 24.0 * p->eps * (2.0 * s12 - s6) / re2; /* |f(re)| / re */
    if (capped)
        *f_over_r = f_over_re * sqrt(re2) / sqrt(r2); /* |f(caprad)| / r */
    else
        *f_over_r = f_over_re;
}

/* Exported scalar evaluation (for closed-form pins). Returns 1 if inside rc. */
int orc_pair_eval(const double* pp, double r, double* u, double* f) {
    orc_pair p = {pp[0], pp[1], pp[2], pp[3], pp[4]};
    double r2 = r * r;
    if (!(r2 < p.rc * p.rc)) { *u = 0.0; *f = 0.0; return 0; }
    double fr;
    lj_eval(&p, r2, u, &fr);
    *f = fr * r; /* radial force magnitude, positive = repulsive */
    return 1;
}

/* FENE: u = -1/2 K R0^2 ln(1 - r^2/R0^2); force on i = -K/(1 - r^2/R0^2) (r_i - r_j) */
static int fene_eval(double K, double R0, double r2, double* u, double* f_over_r) {
    double q = r2 / (R0 * R0);
    if (!(q < 1.0)) return ORC_ERR_BOND_BROKEN;
    *u = -0.5 * K * R0 * R0 * log(1.0 - q);
    *f_over_r = -K / (1.0 - q);
    return ORC_OK;
}

int orc_fene_eval(double K, double R0, double r, double* u, double* f) {
    double fr = 0.0;
    *u = 0.0;
    int st = fene_eval(K, R0, r * r, u, &fr);
    *f = fr * r;
    return st;
}

/* ------------------------------------------------------------------ */
/* Periodic orthorhombic box: compare-based minimum image              */
/* ------------------------------------------------------------------ */
static double min_image(double d, double L, double halfL) {
    if (d > halfL) d -= L;
    else if (d < -halfL) d += L;
    return d;
}

/* Cosine bending for particles (a, b, c), b the centre.  b1 = r_b - r_a,
 * b2 = r_c - r_b (both minimum-imaged), u = k (1 - cos theta) with
 * cos theta = b1.b2/(|b1||b2|); theta = 0 on a straight chain.
 * Forces: F_a = -k d cos/d b1, F_c = k d cos/d b2, F_b = -(F_a + F_c). */
static void bend_eval(double k, const double b1[3], const double b2[3], double* u,
                      double Fa[3], double Fb[3], double Fc[3]) {
    double l1sq = b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2];
    double l2sq = b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2];
    double l1 = sqrt(l1sq), l2 = sqrt(l2sq);
    double dot = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
    double c = dot / (l1 * l2);
    *u = k * (1.0 - c);
    for (int d = 0; d < 3; ++d) {
        double dc_db1 = b2[d] / (l1 * l2) - c * b1[d] / l1sq;
        double dc_db2 = b1[d] / (l1 * l2) - c * b2[d] / l2sq;
        Fa[d] = -k * dc_db1;
        Fc[d] = k * dc_db2;
        Fb[d] = -(Fa[d] + Fc[d]);
    }
}

int orc_bend_eval(double k, const double* ra, const double* rb, const double* rc, double* u,
                  double* Fa, double* Fb, double* Fc) {
    double b1[3], b2[3];
    for (int d = 0; d < 3; ++d) { b1[d] = rb[d] - ra[d]; b2[d] = rc[d] - rb[d]; }
    bend_eval(k, b1, b2, u, Fa, Fb, Fc);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* System description shared by the force / step routines              */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int32_t* type; /* may be NULL: all type 0 */
    int32_t ntypes;
    const double* pp;    /* ntypes*ntypes*5 */
    double box[3];
    int64_t nbonds;
    const int32_t* bonds; /* [nbonds][2] */
    double fene_K, fene_R0;
    int64_t nangles;
    const int32_t* angles; /* [nangles][3], centre in the middle */
    double k_bend;
} orc_sys;

/* obs layout (doubles): 0 e_pair, 1 e_bond, 2 e_angle, 3 virial W,
 * 4..9 virial tensor xx yy zz xy xz yz, 10 the sum of the magnitudes of the
 * virial's terms, sum |r_ij . f_ij| over pairs and bonds plus
 * |r_ab . F_a| + |r_cb . F_c| per angle: the scale against which W, a sum of
 * terms of both signs, can be compared */
#define ORC_NOBS 11

static int type_of(const orc_sys* s, int64_t i) { return s->type ? s->type[i] : 0; }
static orc_pair pair_of(const orc_sys* s, int ti, int tj) {
    const double* q = s->pp + 5 * (ti * s->ntypes + tj);
    orc_pair p = {q[0], q[1], q[2], q[3], q[4]};
    return p;
}

static void add_tensor(double* obs, double s, const double r[3], const double f[3]) {
    /* s * r (x) f, symmetric part stored as xx yy zz xy xz yz */
    obs[4] += s * r[0] * f[0];
    obs[5] += s * r[1] * f[1];
    obs[6] += s * r[2] * f[2];
    obs[7] += s * 0.5 * (r[0] * f[1] + r[1] * f[0]);
    obs[8] += s * 0.5 * (r[0] * f[2] + r[2] * f[0]);
    obs[9] += s * 0.5 * (r[1] * f[2] + r[2] * f[1]);
}

/* Bonded forces (FENE + bending), serial.  fscale[i] += sum of |f| of each
 * term acting on i (for condition-aware tolerances). */
static int bonded_forces(const orc_sys* s, const double* pos, double* F, double* obs,
                         double* fscale) {
    const double L[3] = {s->box[0], s->box[1], s->box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    int status = ORC_OK;
    for (int64_t b = 0; b < s->nbonds; ++b) {
        int64_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double rij[3];
        for (int d = 0; d < 3; ++d) rij[d] = -min_image(pos[3 * j + d] - pos[3 * i + d], L[d], H[d]);
        double r2 = (rij[0] * rij[0] + rij[1] * rij[1]) + rij[2] * rij[2];
        double u, fr;
        if (fene_eval(s->fene_K, s->fene_R0, r2, &u, &fr) != ORC_OK) { status = ORC_ERR_BOND_BROKEN; continue; }
        double f[3] = {fr * rij[0], fr * rij[1], fr * rij[2]};
        for (int d = 0; d < 3; ++d) { F[3 * i + d] += f[d]; F[3 * j + d] -= f[d]; }
        obs[1] += u;
        obs[3] += fr * r2;
        obs[10] += fabs(fr * r2);
        add_tensor(obs, 1.0, rij, f);
        if (fscale) {
            double fm = fabs(fr) * sqrt(r2);
            fscale[i] += fm; fscale[j] += fm;
        }
    }
    for (int64_t a = 0; a < s->nangles; ++a) {
        int64_t ia = s->angles[3 * a], ib = s->angles[3 * a + 1], ic = s->angles[3 * a + 2];
        double b1[3], b2[3];
        for (int d = 0; d < 3; ++d) {
            b1[d] = min_image(pos[3 * ib + d] - pos[3 * ia + d], L[d], H[d]);
            b2[d] = min_image(pos[3 * ic + d] - pos[3 * ib + d], L[d], H[d]);
        }
        double u, Fa[3], Fb[3], Fc[3];
        bend_eval(s->k_bend, b1, b2, &u, Fa, Fb, Fc);
        for (int d = 0; d < 3; ++d) {
            F[3 * ia + d] += Fa[d]; F[3 * ib + d] += Fb[d]; F[3 * ic + d] += Fc[d];
        }
        obs[2] += u;
        /* virial: (r_a - r_b).F_a + (r_c - r_b).F_c */
        double rab[3] = {-b1[0], -b1[1], -b1[2]};
        const double wa = rab[0] * Fa[0] + rab[1] * Fa[1] + rab[2] * Fa[2];
        const double wc = b2[0] * Fc[0] + b2[1] * Fc[1] + b2[2] * Fc[2];
        obs[3] += wa;
        obs[3] += wc;
        obs[10] += fabs(wa) + fabs(wc);
        add_tensor(obs, 1.0, rab, Fa);
        add_tensor(obs, 1.0, b2, Fc);
        if (fscale) {
            double na = sqrt(Fa[0] * Fa[0] + Fa[1] * Fa[1] + Fa[2] * Fa[2]);
            double nb = sqrt(Fb[0] * Fb[0] + Fb[1] * Fb[1] + Fb[2] * Fb[2]);
            double nc = sqrt(Fc[0] * Fc[0] + Fc[1] * Fc[1] + Fc[2] * Fc[2]);
            fscale[ia] += na; fscale[ib] += nb; fscale[ic] += nc;
        }
    }
    return status;
}

/* Pair forces by the O(N^2) definition: every unordered pair once. */
static void pair_forces_brute(const orc_sys* s, const double* pos, double* F, double* obs,
                              double* fscale) {
    const double L[3] = {s->box[0], s->box[1], s->box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    for (int64_t i = 0; i < s->n; ++i) {
        for (int64_t j = i + 1; j < s->n; ++j) {
            orc_pair p = pair_of(s, type_of(s, i), type_of(s, j));
            double dx = min_image(pos[3 * j] - pos[3 * i], L[0], H[0]);
            double dy = min_image(pos[3 * j + 1] - pos[3 * i + 1], L[1], H[1]);
            double dz = min_image(pos[3 * j + 2] - pos[3 * i + 2], L[2], H[2]);
            double r2 = (dx * dx + dy * dy) + dz * dz;
            if (!(r2 < p.rc * p.rc)) continue;
            double u, fr;
            lj_eval(&p, r2, &u, &fr);
            double rij[3] = {-dx, -dy, -dz};
            double f[3] = {fr * rij[0], fr * rij[1], fr * rij[2]};
            for (int d = 0; d < 3; ++d) { F[3 * i + d] += f[d]; F[3 * j + d] -= f[d]; }
            obs[0] += u;
            obs[3] += fr * r2;
            obs[10] += fabs(fr * r2);
            add_tensor(obs, 1.0, rij, f);
            if (fscale) {
                double fm = fabs(fr) * sqrt(r2);
                fscale[i] += fm; fscale[j] += fm;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Linked cells (the paper's CellGrid): cell side >= cutoff, >= 3 per  */
/* side.  Used for the force loop at large N and for neighbour sets.   */
/* ------------------------------------------------------------------ */
typedef struct {
    int nc[3];
    int64_t ncell;
    int64_t* head;  /* first particle in cell, -1 if empty */
    int64_t* next;  /* next particle in the same cell */
} orc_cells;

static int cells_build(orc_cells* c, int64_t n, const double* pos, const double box[3], double cut) {
    for (int d = 0; d < 3; ++d) {
        c->nc[d] = (int)floor(box[d] / (cut * (1.0 + 1e-12)));
        if (c->nc[d] < 3) return ORC_ERR_ARG;
    }
    c->ncell = (int64_t)c->nc[0] * c->nc[1] * c->nc[2];
    c->head = (int64_t*)malloc(sizeof(int64_t) * c->ncell);
    c->next = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t k = 0; k < c->ncell; ++k) c->head[k] = -1;
    /* insert in reverse so that each cell's chain is in ascending index order */
    for (int64_t i = n - 1; i >= 0; --i) {
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            int k = (int)floor(pos[3 * i + d] / box[d] * c->nc[d]);
            if (k < 0) k = 0;
            if (k >= c->nc[d]) k = c->nc[d] - 1;
            ci[d] = k;
        }
        int64_t cell = ((int64_t)ci[2] * c->nc[1] + ci[1]) * c->nc[0] + ci[0];
        c->next[i] = c->head[cell];
        c->head[cell] = i;
    }
    return ORC_OK;
}

static void cells_free(orc_cells* c) { free(c->head); free(c->next); }

static int64_t cell_of(const orc_cells* c, const double* p, const double box[3]) {
    int ci[3];
    for (int d = 0; d < 3; ++d) {
        int k = (int)floor(p[d] / box[d] * c->nc[d]);
        if (k < 0) k = 0;
        if (k >= c->nc[d]) k = c->nc[d] - 1;
        ci[d] = k;
    }
    return ((int64_t)ci[2] * c->nc[1] + ci[1]) * c->nc[0] + ci[0];
}

static double rc_max_of(const orc_sys* s) {
    double m = 0.0;
    for (int a = 0; a < s->ntypes * s->ntypes; ++a)
        if (s->pp[5 * a + 2] > m) m = s->pp[5 * a + 2];
    return m;
}

/* Pair forces via linked cells: for each i, all j in the 27 surrounding
 * cells.  Each pair is seen from both sides; energy and virial take half. */
static int pair_forces_cells(const orc_sys* s, const double* pos, double* F, double* obs,
                             double* fscale, int nthreads) {
    orc_cells c;
    if (cells_build(&c, s->n, pos, s->box, rc_max_of(s)) != ORC_OK) {
        pair_forces_brute(s, pos, F, obs, fscale);
        return ORC_OK;
    }
    const double L[3] = {s->box[0], s->box[1], s->box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    double e_pair = 0, w = 0, wabs = 0, t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0, t5 = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads) \
    reduction(+ : e_pair, w, wabs, t0, t1, t2, t3, t4, t5)
#endif
    for (int64_t i = 0; i < s->n; ++i) {
        int ti = type_of(s, i);
        int64_t ci = cell_of(&c, pos + 3 * i, s->box);
        int cx = (int)(ci % c.nc[0]), cy = (int)((ci / c.nc[0]) % c.nc[1]), cz = (int)(ci / ((int64_t)c.nc[0] * c.nc[1]));
        double fi[3] = {0, 0, 0}, fs = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int nx = (cx + ox + c.nc[0]) % c.nc[0];
                    int ny = (cy + oy + c.nc[1]) % c.nc[1];
                    int nz = (cz + oz + c.nc[2]) % c.nc[2];
                    int64_t cell = ((int64_t)nz * c.nc[1] + ny) * c.nc[0] + nx;
                    for (int64_t j = c.head[cell]; j >= 0; j = c.next[j]) {
                        if (j == i) continue;
                        orc_pair p = pair_of(s, ti, type_of(s, j));
                        double dx = min_image(pos[3 * j] - pos[3 * i], L[0], H[0]);
                        double dy = min_image(pos[3 * j + 1] - pos[3 * i + 1], L[1], H[1]);
                        double dz = min_image(pos[3 * j + 2] - pos[3 * i + 2], L[2], H[2]);
                        double r2 = (dx * dx + dy * dy) + dz * dz;
                        if (!(r2 < p.rc * p.rc)) continue;
                        double u, fr;
                        lj_eval(&p, r2, &u, &fr);
                        fi[0] -= fr * dx; fi[1] -= fr * dy; fi[2] -= fr * dz;
                        e_pair += 0.5 * u;
                        w += 0.5 * fr * r2;
                        wabs += 0.5 * fabs(fr * r2);
                        t0 += 0.5 * fr * dx * dx; t1 += 0.5 * fr * dy * dy; t2 += 0.5 * fr * dz * dz;
                        t3 += 0.5 * fr * dx * dy; t4 += 0.5 * fr * dx * dz; t5 += 0.5 * fr * dy * dz;
                        fs += fabs(fr) * sqrt(r2);
                    }
                }
        for (int d = 0; d < 3; ++d) F[3 * i + d] += fi[d];
        if (fscale) fscale[i] += fs;
    }
    obs[0] += e_pair; obs[3] += w; obs[10] += wabs;
    obs[4] += t0; obs[5] += t1; obs[6] += t2; obs[7] += t3; obs[8] += t4; obs[9] += t5;
    cells_free(&c);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Exported force routine                                              */
/* ------------------------------------------------------------------ */
int orc_forces(int64_t n, const double* pos, const int32_t* type, int32_t ntypes, const double* pp,
               const double* box, int64_t nbonds, const int32_t* bonds, double fene_K, double fene_R0,
               int64_t nangles, const int32_t* angles, double k_bend, int32_t use_cells, int32_t nthreads,
               double* F, double* obs, double* fscale) {
    if (n < 0 || ntypes < 1 || !pos || !pp || !box || !F || !obs) return ORC_ERR_ARG;
    orc_sys s = {n, type, ntypes, pp, {box[0], box[1], box[2]}, nbonds, bonds, fene_K, fene_R0,
                 nangles, angles, k_bend};
    memset(F, 0, sizeof(double) * 3 * n);
    memset(obs, 0, sizeof(double) * ORC_NOBS);
    if (fscale) memset(fscale, 0, sizeof(double) * n);
    if (use_cells) pair_forces_cells(&s, pos, F, obs, fscale, nthreads);
    else pair_forces_brute(&s, pos, F, obs, fscale);
    int st = bonded_forces(&s, pos, F, obs, fscale);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(F[i])) return ORC_ERR_NONFINITE;
    return st;
}

/* ------------------------------------------------------------------ */
/* Neighbour sets: full Verlet list NL(i) = { j != i : r_ij^2 < rv^2 }  */
/* by brute force over all j, for the requested particles.             */
/* Output rows are in ascending j.                                     */
/* ------------------------------------------------------------------ */
int orc_neighbors(int64_t n, const double* pos, const double* box, double rv, int64_t nquery,
                  const int64_t* query, int32_t cap, int32_t* count, int32_t* idx, int32_t nthreads) {
    const double L[3] = {box[0], box[1], box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    const double rv2 = rv * rv;
    int overflow = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(| : overflow)
#endif
    for (int64_t q = 0; q < nquery; ++q) {
        int64_t i = query ? query[q] : q;
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image(pos[3 * j] - pos[3 * i], L[0], H[0]);
            double dy = min_image(pos[3 * j + 1] - pos[3 * i + 1], L[1], H[1]);
            double dz = min_image(pos[3 * j + 2] - pos[3 * i + 2], L[2], H[2]);
            double r2 = (dx * dx + dy * dy) + dz * dz;
            if (r2 < rv2) {
                if (c < cap) idx[q * (int64_t)cap + c] = (int32_t)j;
                else overflow = 1;
                ++c;
            }
        }
        count[q] = c;
    }
    return overflow ? ORC_ERR_NL_OVERFLOW : ORC_OK;
}

/* Same sets through the oracle's own linked cells, for all particles. */
int orc_neighbors_cells(int64_t n, const double* pos, const double* box, double rv, int32_t cap,
                        int32_t* count, int32_t* idx, int32_t nthreads) {
    orc_cells c;
    if (cells_build(&c, n, pos, box, rv) != ORC_OK)
        return orc_neighbors(n, pos, box, rv, n, NULL, cap, count, idx, nthreads);
    const double L[3] = {box[0], box[1], box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    const double rv2 = rv * rv;
    int overflow = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads) reduction(| : overflow)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int64_t ci = cell_of(&c, pos + 3 * i, box);
        int cx = (int)(ci % c.nc[0]), cy = (int)((ci / c.nc[0]) % c.nc[1]), cz = (int)(ci / ((int64_t)c.nc[0] * c.nc[1]));
        int32_t cnt = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int nx = (cx + ox + c.nc[0]) % c.nc[0];
                    int ny = (cy + oy + c.nc[1]) % c.nc[1];
                    int nz = (cz + oz + c.nc[2]) % c.nc[2];
                    int64_t cell = ((int64_t)nz * c.nc[1] + ny) * c.nc[0] + nx;
                    for (int64_t j = c.head[cell]; j >= 0; j = c.next[j]) {
                        if (j == i) continue;
                        double dx = min_image(pos[3 * j] - pos[3 * i], L[0], H[0]);
                        double dy = min_image(pos[3 * j + 1] - pos[3 * i + 1], L[1], H[1]);
                        double dz = min_image(pos[3 * j + 2] - pos[3 * i + 2], L[2], H[2]);
                        double r2 = (dx * dx + dy * dy) + dz * dz;
                        if (r2 < rv2) {
                            if (cnt < cap) idx[i * (int64_t)cap + cnt] = (int32_t)j;
                            else overflow = 1;
                            ++cnt;
                        }
                    }
                }
        count[i] = cnt;
    }
    cells_free(&c);
    return overflow ? ORC_ERR_NL_OVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Velocity Verlet with optional Langevin force (integrator 0 = NVE,   */
/* 1 = Langevin).  State: positions in [0,L), velocities, image        */
/* counters, step counter, and vel_half (1 = vel holds the half-step   */
/* velocity v_{n-1/2}; 0 = vel holds the on-step velocity v_n).        */
/* Each step n:                                                        */
/*   F_tot = F(x_n) [- gamma m v' + sqrt(2 gamma m kT/dt) xi_n]        */
/*   v_n     = v' + dt/(2m) F_tot    (v_n = v' when vel_half == 0)     */
/*   v_{n+h} = v_n + dt/(2m) F_tot                                      */
/*   x_{n+1} = x_n + dt v_{n+h}, wrapped into [0,L)                     */
/* obs_hist[k*ORC_NHIST + ...] records step n's energies at x_n and    */
/* the on-step kinetic energy of v_n:                                  */
/*   0 e_pair 1 e_bond 2 e_angle 3 e_kin 4 W 5..10 tensor (pot+kin-free)*/
/* ------------------------------------------------------------------ */
#define ORC_NHIST 11

int orc_run(int64_t n, double* pos, double* vel, int32_t* image, const int32_t* type,
            const double* mass_by_type, int32_t ntypes, const double* pp, const double* box,
            int64_t nbonds, const int32_t* bonds, double fene_K, double fene_R0, int64_t nangles,
            const int32_t* angles, double k_bend, double dt, int32_t integrator, double temperature,
            double gamma, uint64_t seed, int64_t* step, int32_t* vel_half, int64_t nsteps,
            int32_t use_cells, int32_t nthreads, double* obs_hist) {
    if (n <= 0 || !pos || !vel || !box || !mass_by_type || dt <= 0.0) return ORC_ERR_ARG;
    double* F = (double*)malloc(sizeof(double) * 3 * n);
    double obs[ORC_NOBS];
    const double L[3] = {box[0], box[1], box[2]};
    int status = ORC_OK;
    for (int64_t s = 0; s < nsteps; ++s) {
        int st = orc_forces(n, pos, type, ntypes, pp, box, nbonds, bonds, fene_K, fene_R0, nangles,
                            angles, k_bend, use_cells, nthreads, F, obs, NULL);
        if (st != ORC_OK) { status = st; break; }
        double ekin = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double m = mass_by_type[type ? type[i] : 0];
            double xi[3] = {0, 0, 0};
            double amp = 0.0;
            if (integrator == 1) {
                orc_gauss3(seed, 0, (uint64_t)*step, (uint64_t)i, xi);
                amp = sqrt(2.0 * gamma * m * temperature / dt);
            }
            double hdt_m = 0.5 * dt / m;
            double vv2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                double vp = vel[3 * i + d];
                double ft = F[3 * i + d];
                if (integrator == 1) ft = (ft - gamma * m * vp) + amp * xi[d];
                double von = *vel_half ? vp + hdt_m * ft : vp;
                double vh = von + hdt_m * ft;
                vv2 += von * von;
                double x = pos[3 * i + d] + dt * vh;
                int img = image ? image[3 * i + d] : 0;
                if (x < 0.0) { x += L[d]; img -= 1; }
                if (x >= L[d]) { x -= L[d]; img += 1; }
                pos[3 * i + d] = x;
                if (image) image[3 * i + d] = img;
                vel[3 * i + d] = vh;
            }
            ekin += 0.5 * m * vv2;
        }
        if (obs_hist) {
            double* h = obs_hist + s * ORC_NHIST;
            h[0] = obs[0]; h[1] = obs[1]; h[2] = obs[2]; h[3] = ekin; h[4] = obs[3];
            for (int k = 0; k < 6; ++k) h[5 + k] = obs[4 + k];
        }
        *step += 1;
        *vel_half = 1;
    }
    free(F);
    return status;
}

/* ------------------------------------------------------------------ */
/* Lees-Edwards sheared boundaries and the DPD thermostat               */
/* (section "New Features": Lees-Edwards boundary conditions; section   */
/* "Functionality": dissipative particle dynamics).  The paper gives no */
/* formulas; these are the textbook definitions (Lees & Edwards 1972;   */
/* Espanol & Warren 1995; Groot & Warren 1997).                          */
/*                                                                      */
/* Shear: flow along x, gradient along y.  The periodic image one box   */
/* above (y + Ly) is displaced by +delta(t) in x and moves with          */
/* +gammadot Ly in x, delta(t) = gammadot Ly t mod Lx, t = step dt.      */
/* Minimum image of d = r_j - r_i (fixed operation order, shared with   */
/* the GPU): dy by compare-and-shift with s = +1 when dy > Ly/2 (j's     */
/* nearest image lies one box below), -1 when dy < -Ly/2; dx = the x    */
/* minimum image of x_j - x_i, then if s != 0 the x minimum image of     */
/* dx - s delta_w, delta_w = delta folded into (-Lx/2, Lx/2]; dz as      */
/* usual.  The image's velocity is v_j - s gammadot Ly e_x.             */
/*                                                                      */
/* DPD, per pair with r = |r_i - r_j| < rc_d, e = (r_i - r_j)/r,        */
/* v_ij = v_i - v_j (image velocity), w = 1 - r/rc_d:                    */
/*   F_i^D = -gamma w^2 (e . v_ij) e,  F_i^R = sigma w theta_ij e/sqrt(dt),*/
/*   sigma^2 = 2 gamma kT, theta_ij = theta_ji ~ N(0,1): Philox4x64-10  */
/*   keyed (seed, 6), counter (step, min tag, max tag, 0), Box-Muller on */
/*   the first two uniforms.                                             */
/* The dissipative force takes the half-step velocity v' (the velocity  */
/* the Langevin friction also takes): Groot-Warren's modified velocity  */
/* Verlet with lambda = 1/2.                                             */
/* ------------------------------------------------------------------ */
typedef struct { int on; double delta, delta_w, vjump; } orc_le;

static orc_le le_at(const double box[3], double shear_rate, int64_t step, double dt) {
    orc_le le = {shear_rate != 0.0, 0.0, 0.0, shear_rate * box[1]};
    if (le.on) {
        double d = fmod(shear_rate * box[1] * ((double)step * dt), box[0]);
        if (d < 0.0) d += box[0];
        le.delta = d;
        le.delta_w = d > 0.5 * box[0] ? d - box[0] : d;
    }
    return le;
}

static void le_diff(const orc_le* le, const double L[3], const double H[3], const double* ri, const double* rj,
                    double d[3], int* s) {
    double dy = rj[1] - ri[1];
    int sy = 0;
    if (dy > H[1]) { dy -= L[1]; sy = 1; }
    else if (dy < -H[1]) { dy += L[1]; sy = -1; }
    double dx = min_image(rj[0] - ri[0], L[0], H[0]);
    if (le->on && sy != 0) dx = min_image(dx - sy * le->delta_w, L[0], H[0]);
    d[0] = dx;
    d[1] = dy;
    d[2] = min_image(rj[2] - ri[2], L[2], H[2]);
    *s = le->on ? sy : 0;
}

/* theta_ij for the unordered pair {ti, tj} at this step: Philox4x32-10 at
 * counter (step low word, step high word, min tag, max tag) with key (seed
 * low word, seed high word ^ 6), Box-Muller on the first two words as
 * uniforms (w + 1/2) 2^-32 */
double orc_dpd_theta(uint64_t seed, uint64_t step, uint64_t ti, uint64_t tj) {
    const uint64_t a = ti < tj ? ti : tj, b = ti < tj ? tj : ti;
    uint32_t ctr[4] = {(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)a, (uint32_t)b};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 6u};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    const double two_pi = 6.283185307179586;
    const double u0 = ((double)r[0] + 0.5) * 0x1.0p-32, u1 = ((double)r[1] + 0.5) * 0x1.0p-32;
    return sqrt(-2.0 * log(u0)) * cos(two_pi * u1);
}

/* Tabulated interactions (section "Functionality": tabulated potentials;
 * section "New Features": AngularCosineSquared, TabulatedSubEnsAngular).
 * Pair table of type pair p (when pair_rmin[p] is not NaN): npair points of
 * u and of the radial force f = -du/dr on the uniform grid
 * r_k = rmin + k (rc - rmin)/(npair - 1), rc the pair's cutoff; u and f are
 * interpolated linearly in r (below rmin: the rmin values), zero from rc on.
 * Angles, with phi the bond angle at the centre (pi for a straight chain):
 * kind 0 the cosine bending k (1 - cos theta), theta = pi - phi; kind 1
 * AngularCosineSquared u = K (cos phi - cos phi0)^2; kind 2 a table of u and
 * du/dphi on the uniform grid phi_k = k pi/(nang - 1), interpolated linearly
 * in phi, dU/dcos(phi) = -(du/dphi)/max(sin phi, 1e-8).  A weighted sum of
 * several angle tables on one grid (TabulatedSubEnsAngular) is the table of
 * the weighted sums (orc_angle_tables_combine). */
typedef struct {
    int32_t npair;
    const double* pair_rmin;   /* [ntypes^2], NaN = Lennard-Jones */
    const double* pair_u;      /* [ntypes^2][npair] */
    const double* pair_f;
    int32_t angle_kind;
    double angle_K, angle_phi0;
    int32_t nang;
    const double* angle_u;     /* [nang] */
    const double* angle_g;     /* [nang] du/dphi */
    /* AdResS (section "Statement of need", section "Functionality"): force
     * interpolation between an atomistic pair force (the pair table above)
     * and a coarse-grained one (these tables, npair points on
     * r_k = cg_rmin + k (cg_rc - cg_rmin)/(npair - 1)), on single-site
     * molecules: F_ij = w_i w_j F^AT_ij + (1 - w_i w_j) F^CG_ij with the
     * weight of the position along x, d = |x - x0| (minimum image):
     * w = 1 for d < d_at, 0 for d > d_at + d_hy, cos^2(pi (d - d_at)/(2 d_hy))
     * between.  The reported energy is the same interpolation of u. */
    int32_t adress;
    double ad_x0, ad_dat, ad_dhy;
    const double* cg_rmin;     /* [ntypes^2], NaN = no coarse-grained force */
    const double* cg_rc;       /* [ntypes^2] */
    const double* cg_u;        /* [ntypes^2][npair] */
    const double* cg_f;
} orc_tabs;

typedef struct {
    double shear_rate, dpd_rc, dpd_gamma, kT, dt;
    uint64_t seed;
    int64_t step;
    const orc_tabs* tabs;
} orc_ext;

static double lerp_table(const double* t, int32_t n, double x, double x0, double dx) {
    double q = (x - x0) / dx;
    if (q < 0.0) return t[0];
    int64_t k = (int64_t)floor(q);
    if (k > n - 2) k = n - 2;
    const double a = q - (double)k;
    return (1.0 - a) * t[k] + a * t[k + 1];
}

/* pair energy and f/r for r2 < rc^2 (tables or Lennard-Jones) */
static void pair_eval_ext(const orc_sys* s, const orc_tabs* tb, int ti, int tj, double r2, double* u, double* fr) {
    const int tp = ti * s->ntypes + tj;
    orc_pair p = pair_of(s, ti, tj);
    if (tb && tb->npair > 1 && !isnan(tb->pair_rmin[tp])) {
        const double r = sqrt(r2);
        const double rmin = tb->pair_rmin[tp];
        const double dr = (p.rc - rmin) / (double)(tb->npair - 1);
        *u = lerp_table(tb->pair_u + (int64_t)tp * tb->npair, tb->npair, r, rmin, dr);
        *fr = lerp_table(tb->pair_f + (int64_t)tp * tb->npair, tb->npair, r, rmin, dr) / r;
        return;
    }
    lj_eval(&p, r2, u, fr);
}

/* AdResS weight of a position x along the slab axis. */
double orc_adress_weight(double x, double Lx, double x0, double dat, double dhy) {
    const double d = fabs(min_image(x - x0, Lx, 0.5 * Lx));
    if (d < dat) return 1.0;
    if (d >= dat + dhy) return 0.0;
    const double c = cos(1.5707963267948966 * (d - dat) / dhy);
    return c * c;
}

/* coarse-grained pair energy and f/r, zero from cg_rc on */
static int cg_eval(const orc_sys* s, const orc_tabs* tb, int ti, int tj, double r2, double* u, double* fr) {
    const int tp = ti * s->ntypes + tj;
    *u = 0.0;
    *fr = 0.0;
    if (isnan(tb->cg_rmin[tp]) || !(r2 < tb->cg_rc[tp] * tb->cg_rc[tp])) return 0;
    const double r = sqrt(r2);
    const double rmin = tb->cg_rmin[tp];
    const double dr = (tb->cg_rc[tp] - rmin) / (double)(tb->npair - 1);
    *u = lerp_table(tb->cg_u + (int64_t)tp * tb->npair, tb->npair, r, rmin, dr);
    *fr = lerp_table(tb->cg_f + (int64_t)tp * tb->npair, tb->npair, r, rmin, dr) / r;
    return 1;
}

/* Angle energy and forces for the angle kinds above; b1 = r_b - r_a,
 * b2 = r_c - r_b (b the centre). */
static void angle_eval_ext(const orc_sys* s, const orc_tabs* tb, const double b1[3], const double b2[3], double* u,
                           double Fa[3], double Fb[3], double Fc[3]) {
    const int kind = tb ? tb->angle_kind : 0;
    if (kind == 0) {
        bend_eval(s->k_bend, b1, b2, u, Fa, Fb, Fc);
        return;
    }
    double l1sq = b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2];
    double l2sq = b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2];
    double l1 = sqrt(l1sq), l2 = sqrt(l2sq);
    double c = (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / (l1 * l2);   /* cos theta = -cos phi */
    const double cphi = -c;
    double dUdc;   /* dU / d(cos theta) */
    if (kind == 1) {
        const double d = cphi - cos(tb->angle_phi0);
        *u = tb->angle_K * d * d;
        dUdc = -2.0 * tb->angle_K * d;
    } else {
        const double cl = cphi > 1.0 ? 1.0 : (cphi < -1.0 ? -1.0 : cphi);
        const double phi = acos(cl);
        const double dphi = 3.141592653589793 / (double)(tb->nang - 1);
        *u = lerp_table(tb->angle_u, tb->nang, phi, 0.0, dphi);
        const double g = lerp_table(tb->angle_g, tb->nang, phi, 0.0, dphi);
        const double sn = sin(phi);
        dUdc = g / (sn > 1e-8 ? sn : 1e-8);   /* dU/dcos(phi) = -g/sin(phi), dcos(phi)/dcos(theta) = -1 */
    }
    for (int d = 0; d < 3; ++d) {
        const double dc_db1 = b2[d] / (l1 * l2) - c * b1[d] / l1sq;
        const double dc_db2 = b1[d] / (l1 * l2) - c * b2[d] / l2sq;
        Fa[d] = dUdc * dc_db1;        /* b1 = r_b - r_a: dc/dr_a = -dc/db1 */
        Fc[d] = -dUdc * dc_db2;
        Fb[d] = -(Fa[d] + Fc[d]);
    }
}

/* TabulatedSubEnsAngular: the table of sum_m w_m (u_m, g_m) over ntab tables
 * of n points each (rows of u and g). */
void orc_angle_tables_combine(int32_t ntab, int32_t n, const double* u, const double* g, const double* w,
                              double* u_out, double* g_out) {
    for (int32_t k = 0; k < n; ++k) {
        double su = 0.0, sg = 0.0;
        for (int32_t m = 0; m < ntab; ++m) {
            su += w[m] * u[(int64_t)m * n + k];
            sg += w[m] * g[(int64_t)m * n + k];
        }
        u_out[k] = su;
        g_out[k] = sg;
    }
}

/* Conservative pair forces (the LJ table) under the sheared minimum image,
 * by brute force over all pairs, and (dpd_rc > 0) the DPD pair forces at
 * velocities vel into Fd.  Each unordered pair once. */
static void pair_forces_ext(const orc_sys* s, const orc_ext* x, const double* pos, const double* vel, double* F,
                            double* Fd, double* obs, double* fscale) {
    const double L[3] = {s->box[0], s->box[1], s->box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    const orc_le le = le_at(s->box, x->shear_rate, x->step, x->dt);
    const double sigma = sqrt(2.0 * x->dpd_gamma * x->kT), isdt = 1.0 / sqrt(x->dt);
    const double rcd2 = x->dpd_rc * x->dpd_rc;
    for (int64_t i = 0; i < s->n; ++i) {
        for (int64_t j = i + 1; j < s->n; ++j) {
            double d[3];
            int sy;
            le_diff(&le, L, H, pos + 3 * i, pos + 3 * j, d, &sy);
            const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            orc_pair p = pair_of(s, type_of(s, i), type_of(s, j));
            const orc_tabs* tb = x->tabs;
            const int ad = tb && tb->adress;
            double ucg = 0.0, frcg = 0.0;
            const int cg_in = ad ? cg_eval(s, tb, type_of(s, i), type_of(s, j), r2, &ucg, &frcg) : 0;
            const int at_in = r2 < p.rc * p.rc;
            if (at_in || cg_in) {
                double u = 0.0, fr = 0.0;
                if (at_in) pair_eval_ext(s, tb, type_of(s, i), type_of(s, j), r2, &u, &fr);
                if (ad) {
                    const double lam = orc_adress_weight(pos[3 * i], L[0], tb->ad_x0, tb->ad_dat, tb->ad_dhy) *
                                       orc_adress_weight(pos[3 * j], L[0], tb->ad_x0, tb->ad_dat, tb->ad_dhy);
                    u = lam * u + (1.0 - lam) * ucg;
                    fr = lam * fr + (1.0 - lam) * frcg;
                }
                double rij[3] = {-d[0], -d[1], -d[2]};
                double f[3] = {fr * rij[0], fr * rij[1], fr * rij[2]};
                for (int k = 0; k < 3; ++k) { F[3 * i + k] += f[k]; F[3 * j + k] -= f[k]; }
                obs[0] += u;
                obs[3] += fr * r2;
                obs[10] += fabs(fr * r2);
                add_tensor(obs, 1.0, rij, f);
                if (fscale) {
                    double fm = fabs(fr) * sqrt(r2);
                    fscale[i] += fm; fscale[j] += fm;
                }
            }
            if (Fd && r2 < rcd2) {
                const double r = sqrt(r2);
                const double w = 1.0 - r / x->dpd_rc;
                const double e[3] = {-d[0] / r, -d[1] / r, -d[2] / r};          /* (r_i - r_j) / r */
                double vij[3];
                for (int k = 0; k < 3; ++k) vij[k] = vel[3 * i + k] - vel[3 * j + k];
                vij[0] += sy * le.vjump;                                          /* v_i - (v_j - s vjump e_x) */
                const double ev = (e[0] * vij[0] + e[1] * vij[1]) + e[2] * vij[2];
                const double th = orc_dpd_theta(x->seed, (uint64_t)x->step, (uint64_t)i, (uint64_t)j);
                const double a = -x->dpd_gamma * w * w * ev + sigma * w * th * isdt;
                for (int k = 0; k < 3; ++k) { Fd[3 * i + k] += a * e[k]; Fd[3 * j + k] -= a * e[k]; }
                if (fscale) { fscale[i] += fabs(a); fscale[j] += fabs(a); }
            }
        }
    }
}

/* Bonded forces under the sheared minimum image (the same terms as
 * bonded_forces). */
static int bonded_forces_ext(const orc_sys* s, const orc_ext* x, const double* pos, double* F, double* obs,
                             double* fscale) {
    const double L[3] = {s->box[0], s->box[1], s->box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    const orc_le le = le_at(s->box, x->shear_rate, x->step, x->dt);
    int status = ORC_OK;
    for (int64_t b = 0; b < s->nbonds; ++b) {
        int64_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double d[3];
        int sy;
        le_diff(&le, L, H, pos + 3 * i, pos + 3 * j, d, &sy);
        double rij[3] = {-d[0], -d[1], -d[2]};
        double r2 = (rij[0] * rij[0] + rij[1] * rij[1]) + rij[2] * rij[2];
        double u, fr;
        if (fene_eval(s->fene_K, s->fene_R0, r2, &u, &fr) != ORC_OK) { status = ORC_ERR_BOND_BROKEN; continue; }
        double f[3] = {fr * rij[0], fr * rij[1], fr * rij[2]};
        for (int k = 0; k < 3; ++k) { F[3 * i + k] += f[k]; F[3 * j + k] -= f[k]; }
        obs[1] += u;
        obs[3] += fr * r2;
        obs[10] += fabs(fr * r2);
        add_tensor(obs, 1.0, rij, f);
        if (fscale) {
            double fm = fabs(fr) * sqrt(r2);
            fscale[i] += fm; fscale[j] += fm;
        }
    }
    for (int64_t a = 0; a < s->nangles; ++a) {
        int64_t ia = s->angles[3 * a], ib = s->angles[3 * a + 1], ic = s->angles[3 * a + 2];
        double b1[3], b2[3];
        int sy;
        le_diff(&le, L, H, pos + 3 * ia, pos + 3 * ib, b1, &sy);
        le_diff(&le, L, H, pos + 3 * ib, pos + 3 * ic, b2, &sy);
        double u, Fa[3], Fb[3], Fc[3];
        angle_eval_ext(s, x->tabs, b1, b2, &u, Fa, Fb, Fc);
        for (int k = 0; k < 3; ++k) { F[3 * ia + k] += Fa[k]; F[3 * ib + k] += Fb[k]; F[3 * ic + k] += Fc[k]; }
        obs[2] += u;
        double rab[3] = {-b1[0], -b1[1], -b1[2]};
        const double wa = rab[0] * Fa[0] + rab[1] * Fa[1] + rab[2] * Fa[2];
        const double wc = b2[0] * Fc[0] + b2[1] * Fc[1] + b2[2] * Fc[2];
        obs[3] += wa;
        obs[3] += wc;
        obs[10] += fabs(wa) + fabs(wc);
        add_tensor(obs, 1.0, rab, Fa);
        add_tensor(obs, 1.0, b2, Fc);
        if (fscale) {
            fscale[ia] += sqrt(Fa[0] * Fa[0] + Fa[1] * Fa[1] + Fa[2] * Fa[2]);
            fscale[ib] += sqrt(Fb[0] * Fb[0] + Fb[1] * Fb[1] + Fb[2] * Fb[2]);
            fscale[ic] += sqrt(Fc[0] * Fc[0] + Fc[1] * Fc[1] + Fc[2] * Fc[2]);
        }
    }
    return status;
}

/* Conservative forces F (and, with dpd_rc > 0 and Fd non-NULL, the DPD
 * thermostat forces Fd at velocities vel) under the sheared boundaries at
 * time step * dt.  Brute force over pairs.  fscale[i]: the sum of the
 * magnitudes of every pair and bonded force term on i, DPD pair forces
 * included when computed. */
int orc_forces_ext(int64_t n, const double* pos, const double* vel, const int32_t* type, int32_t ntypes,
                   const double* pp, const double* box, int64_t nbonds, const int32_t* bonds, double fene_K,
                   double fene_R0, int64_t nangles, const int32_t* angles, double k_bend, double shear_rate,
                   double dpd_rc, double dpd_gamma, double kT, double dt, uint64_t seed, int64_t step,
                   const orc_tabs* tabs, double* F, double* Fd, double* obs, double* fscale) {
    if (n < 0 || ntypes < 1 || !pos || !pp || !box || !F || !obs || dt <= 0.0) return ORC_ERR_ARG;
    if (Fd && dpd_rc > 0.0 && !vel) return ORC_ERR_ARG;
    orc_sys s = {n, type, ntypes, pp, {box[0], box[1], box[2]}, nbonds, bonds, fene_K, fene_R0,
                 nangles, angles, k_bend};
    orc_ext x = {shear_rate, dpd_rc, dpd_gamma, kT, dt, seed, step, tabs};
    memset(F, 0, sizeof(double) * 3 * n);
    if (Fd) memset(Fd, 0, sizeof(double) * 3 * n);
    memset(obs, 0, sizeof(double) * ORC_NOBS);
    if (fscale) memset(fscale, 0, sizeof(double) * n);
    pair_forces_ext(&s, &x, pos, vel, F, (dpd_rc > 0.0) ? Fd : NULL, obs, fscale);
    int st = bonded_forces_ext(&s, &x, pos, F, obs, fscale);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(F[i])) return ORC_ERR_NONFINITE;
    return st;
}

/* Verlet-list sets under the sheared minimum image at time step * dt, by
 * brute force (rows ascending). */
int orc_neighbors_le(int64_t n, const double* pos, const double* box, double rv, double shear_rate, double dt,
                     int64_t step, int32_t cap, int32_t* count, int32_t* idx) {
    const double L[3] = {box[0], box[1], box[2]};
    const double H[3] = {0.5 * L[0], 0.5 * L[1], 0.5 * L[2]};
    const orc_le le = le_at(box, shear_rate, step, dt);
    const double rv2 = rv * rv;
    int overflow = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            int sy;
            le_diff(&le, L, H, pos + 3 * i, pos + 3 * j, d, &sy);
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            if (r2 < rv2) {
                if (c < cap) idx[i * (int64_t)cap + c] = (int32_t)j;
                else overflow = 1;
                ++c;
            }
        }
        count[i] = c;
    }
    return overflow ? ORC_ERR_NL_OVERFLOW : ORC_OK;
}

/* Velocity Verlet as orc_run, extended: integrator 2 = DPD (the pair
 * thermostat above instead of the Langevin friction and noise), and
 * shear_rate != 0 = Lees-Edwards boundaries.  A particle leaving through
 * y = Ly re-enters at y - Ly with x - delta(t_{n+1}) and v_x - gammadot Ly
 * (through y = 0: the opposite shifts), before the x fold into [0, Lx).
 * History columns as orc_run. */
int orc_run_ext(int64_t n, double* pos, double* vel, int32_t* image, const int32_t* type,
                const double* mass_by_type, int32_t ntypes, const double* pp, const double* box,
                int64_t nbonds, const int32_t* bonds, double fene_K, double fene_R0, int64_t nangles,
                const int32_t* angles, double k_bend, double dt, int32_t integrator, double temperature,
                double gamma, uint64_t seed, double shear_rate, double dpd_rc, const orc_tabs* tabs, int64_t* step,
                int32_t* vel_half, int64_t nsteps, double* obs_hist) {
    if (n <= 0 || !pos || !vel || !box || !mass_by_type || dt <= 0.0) return ORC_ERR_ARG;
    if (integrator < 0 || integrator > 2) return ORC_ERR_ARG;
    double* F = (double*)malloc(sizeof(double) * 3 * n);
    double* Fd = (double*)malloc(sizeof(double) * 3 * n);
    double obs[ORC_NOBS];
    const double L[3] = {box[0], box[1], box[2]};
    int status = ORC_OK;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int dpd = integrator == 2;
        int st = orc_forces_ext(n, pos, vel, type, ntypes, pp, box, nbonds, bonds, fene_K, fene_R0, nangles, angles,
                                k_bend, shear_rate, dpd ? dpd_rc : 0.0, gamma, temperature, dt, seed, *step, tabs, F,
                                dpd ? Fd : NULL, obs, NULL);
        if (st != ORC_OK) { status = st; break; }
        const orc_le le_next = le_at(box, shear_rate, *step + 1, dt);
        double ekin = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double m = mass_by_type[type ? type[i] : 0];
            double xi[3] = {0, 0, 0};
            double amp = 0.0;
            if (integrator == 1) {
                orc_gauss3(seed, 0, (uint64_t)*step, (uint64_t)i, xi);
                amp = sqrt(2.0 * gamma * m * temperature / dt);
            }
            double hdt_m = 0.5 * dt / m;
            double vv2 = 0.0, xn[3], vh[3];
            for (int d = 0; d < 3; ++d) {
                double vp = vel[3 * i + d];
                double ft = F[3 * i + d];
                if (integrator == 1) ft = (ft - gamma * m * vp) + amp * xi[d];
                if (dpd) ft = ft + Fd[3 * i + d];
                double von = *vel_half ? vp + hdt_m * ft : vp;
                vh[d] = von + hdt_m * ft;
                vv2 += von * von;
                xn[d] = pos[3 * i + d] + dt * vh[d];
            }
            int img[3] = {0, 0, 0};
            if (image) for (int d = 0; d < 3; ++d) img[d] = image[3 * i + d];
            if (le_next.on) {
                if (xn[1] >= L[1]) { xn[1] -= L[1]; xn[0] -= le_next.delta; vh[0] -= le_next.vjump; img[1] += 1; }
                else if (xn[1] < 0.0) { xn[1] += L[1]; xn[0] += le_next.delta; vh[0] += le_next.vjump; img[1] -= 1; }
            }
            for (int d = 0; d < 3; ++d) {
                if (xn[d] < 0.0) { xn[d] += L[d]; img[d] -= 1; }
                if (xn[d] >= L[d]) { xn[d] -= L[d]; img[d] += 1; }
                pos[3 * i + d] = xn[d];
                vel[3 * i + d] = vh[d];
                if (image) image[3 * i + d] = img[d];
            }
            ekin += 0.5 * m * vv2;
        }
        if (obs_hist) {
            double* h = obs_hist + s * ORC_NHIST;
            h[0] = obs[0]; h[1] = obs[1]; h[2] = obs[2]; h[3] = ekin; h[4] = obs[3];
            for (int k = 0; k < 6; ++k) h[5 + k] = obs[4 + k];
        }
        *step += 1;
        *vel_half = 1;
    }
    free(F);
    free(Fd);
    return status;
}

int orc_nthreads_default(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
