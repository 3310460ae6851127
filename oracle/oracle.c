/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the coupled double-distribution
 * thermal lattice Boltzmann method of Xu, Shi & Xi, "Lattice Boltzmann
 * simulations of three-dimensional thermal convective flows at high Rayleigh
 * number", Int. J. Heat Mass Transfer (2019), arXiv:1903.08882.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * HIP path is compared against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library: every constant below is written out
 * (or derived) here from the paper's definitions.
 *
 * What it computes (section / equation of the paper):
 *   - D3Q19 velocity set and the 19x19 moment matrix M built from its
 *     polynomial definition (Sec. 2.2, definition of M);
 *   - D3Q7 velocity set and the 7x7 matrix N built from its polynomial
 *     definition (Sec. 2.3, definition of N; the printed row for <e_z| has a
 *     sign typo, the polynomial row e_z is used);
 *   - the MRT collision of f with Guo forcing written in moment space
 *     (Sec. 2.2, Eq. MRT, m^eq, S, F' = M^-1 (I - S/2) M F~), and the MRT
 *     collision of g (Sec. 2.3, Eq. MRT_T, n^eq, Q);
 *   - half-way bounce-back for f, half-way anti-bounce-back (fixed T) and
 *     bounce-back (adiabatic) for g (Sec. 2.2 and 2.3 boundary schemes),
 *     applied while push-streaming into a second array;
 *   - observables: link heat flux through the isothermal walls, volume means
 *     of |u|^2, w^2, wT, uT, and central-difference dissipation rates
 *     (Sec. 3 and Sec. 4 definitions of Nu, Re, eps_u, eps_T);
 *   - the steady-state residual (Sec. 3 criterion).
 *
 * Layout: population q (0..18 = f_0..f_18, 19..25 = g_0..g_6) of node
 * (x, y, z) lives at pop[q*V + x + N*(y + N*z)], V = N^3.  Node (i, j, k)
 * sits at ((i+1/2), (j+1/2), (k+1/2)) lattice units; the walls are the planes
 * 0 and N of each axis, so the cell height H equals N.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q19 19
#define Q7 7
#define NPOP 26

/* Number of OpenMP threads the whole-lattice loops use. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Lattices                                                                 */
/* ------------------------------------------------------------------------ */

/* D3Q19 velocities in the order of the printed 3x19 array (Sec. 2.2). */
static const int E19[Q19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, 1, 0},  {1, -1, 0},
    {-1, -1, 0}, {1, 0, 1}, {-1, 0, 1}, {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},  {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

/* D3Q7 velocities in the order of the printed 3x7 array (Sec. 2.3). */
static const int E7[Q7][3] = {{0, 0, 0}, {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},
                              {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Index of the velocity opposite to e_i, found by search. */
static int opposite19(int i) {
    for (int j = 0; j < Q19; ++j)
        if (E19[j][0] == -E19[i][0] && E19[j][1] == -E19[i][1] &&
            E19[j][2] == -E19[i][2])
            return j;
    return -1;
}
static int opposite7(int i) {
    for (int j = 0; j < Q7; ++j)
        if (E7[j][0] == -E7[i][0] && E7[j][1] == -E7[i][1] && E7[j][2] == -E7[i][2])
            return j;
    return -1;
}

/* Weights of f^eq (Sec. 2.2): 1/3 at rest, 1/18 on axes, 1/36 on diagonals. */
static double w19(int i) {
    int e2 = E19[i][0] * E19[i][0] + E19[i][1] * E19[i][1] + E19[i][2] * E19[i][2];
    return e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* ------------------------------------------------------------------------ */
/* Moment matrices from their polynomial definitions                        */
/* ------------------------------------------------------------------------ */

/* Row r of M evaluated at velocity e (Sec. 2.2, the bracket list defining M). */
static double m_row_poly(int r, const int e[3]) {
    double ex = e[0], ey = e[1], ez = e[2];
    double e2 = ex * ex + ey * ey + ez * ez;
    switch (r) {
    case 0: return 1.0;
    case 1: return 19.0 * e2 - 30.0;
    case 2: return 21.0 / 2.0 * e2 * e2 - 53.0 / 2.0 * e2 + 12.0;
    case 3: return ex;
    case 4: return (5.0 * e2 - 9.0) * ex;
    case 5: return ey;
    case 6: return (5.0 * e2 - 9.0) * ey;
    case 7: return ez;
    case 8: return (5.0 * e2 - 9.0) * ez;
    case 9: return 3.0 * ex * ex - e2;
    case 10: return (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2);
    case 11: return ey * ey - ez * ez;
    case 12: return (3.0 * e2 - 5.0) * (ey * ey - ez * ez);
    case 13: return ex * ey;
    case 14: return ey * ez;
    case 15: return ex * ez;
    case 16: return (ey * ey - ez * ez) * ex;
    case 17: return (ez * ez - ex * ex) * ey;
    case 18: return (ex * ex - ey * ey) * ez;
    }
    return 0.0;
}

/* Row r of N evaluated at velocity e (Sec. 2.3, the bracket list defining N). */
static double n_row_poly(int r, const int e[3]) {
    double ex = e[0], ey = e[1], ez = e[2];
    double e2 = ex * ex + ey * ey + ez * ez;
    switch (r) {
    case 0: return 1.0;
    case 1: return ex;
    case 2: return ey;
    case 3: return ez;
    case 4: return -6.0 + 7.0 * e2;
    case 5: return 3.0 * ex * ex - e2;
    case 6: return ey * ey - ez * ez;
    }
    return 0.0;
}

void orc_matrix_M(double *M /* 19*19, row-major */) {
    for (int r = 0; r < Q19; ++r)
        for (int i = 0; i < Q19; ++i) M[r * Q19 + i] = m_row_poly(r, E19[i]);
}

void orc_matrix_N(double *Nm /* 7*7, row-major */) {
    for (int r = 0; r < Q7; ++r)
        for (int i = 0; i < Q7; ++i) Nm[r * Q7 + i] = n_row_poly(r, E7[i]);
}

/* Plain Gauss-Jordan inverse with partial pivoting; returns 0 if singular. */
static int invert(int n, const double *A, double *Ainv) {
    double *a = (double *)malloc(sizeof(double) * n * 2 * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + c]) > fabs(a[piv * 2 * n + c])) piv = r;
        if (fabs(a[piv * 2 * n + c]) < 1e-12) { free(a); return 0; }
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) {
                double t = a[c * 2 * n + k];
                a[c * 2 * n + k] = a[piv * 2 * n + k];
                a[piv * 2 * n + k] = t;
            }
        double d = a[c * 2 * n + c];
        for (int k = 0; k < 2 * n; ++k) a[c * 2 * n + k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double fct = a[r * 2 * n + c];
            if (fct != 0.0)
                for (int k = 0; k < 2 * n; ++k) a[r * 2 * n + k] -= fct * a[c * 2 * n + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r * 2 * n + n + c];
    free(a);
    return 1;
}

int orc_invert(int n, const double *A, double *Ainv) { return invert(n, A, Ainv); }

void orc_velocities19(int *e /* 19*3 */, int *opp /* 19 */, double *w /* 19 */) {
    for (int i = 0; i < Q19; ++i) {
        for (int a = 0; a < 3; ++a) e[i * 3 + a] = E19[i][a];
        opp[i] = opposite19(i);
        w[i] = w19(i);
    }
}

void orc_velocities7(int *e /* 7*3 */, int *opp /* 7 */) {
    for (int i = 0; i < Q7; ++i) {
        for (int a = 0; a < 3; ++a) e[i * 3 + a] = E7[i][a];
        opp[i] = opposite7(i);
    }
}

/* ------------------------------------------------------------------------ */
/* Parameters                                                               */
/* ------------------------------------------------------------------------ */

/* Field order must match the ctypes mirror in oracle/__init__.py. */
typedef struct {
    int N;          /* nodes per side; H = N lattice units                  */
    int cell;       /* 0 = side-heated (hot x=0, cold x=N), 1 = Rayleigh-Benard
                       (hot z=0, cold z=N); gravity along -z, buoyancy +z     */
    double Ra, Pr;
    double U;       /* free-fall velocity sqrt(g beta dT H), lattice units  */
    double T0;      /* reference temperature of the buoyancy term           */
    double T_hot, T_cold;
    double H, dT;
    double nu, kappa, gbeta;
    double tau_f, s_e, s_q; /* s_e = s_eps = s_nu = s_pi = 1/tau_f; s_q = s_m */
    double q_k, q_e, q_nu, a_T;
    double wT0, wT1;        /* D3Q7 weights: rest, axis                       */
} orc_params;

/*
 * Derive the lattice parameters from (N, Ra, Pr, U).
 *   Sec. 2.1: Ra = g beta dT H^3/(nu kappa), Pr = nu/kappa, free-fall scaling
 *             => nu = U H sqrt(Pr/Ra), kappa = U H / sqrt(Ra Pr),
 *                g beta = U^2 / (H dT).
 *   Sec. 2.2: nu = c_s^2 (tau_f - 1/2); s_q = s_m = 8(2 tau_f - 1)/(8 tau_f - 1).
 *   Sec. 2.3: kappa = (6 + a_T)/21 (1/q_k - 1/2), q_k = 3 - sqrt 3,
 *             q_e = q_nu = 4 sqrt 3 - 6, weights (1-a_T)/7 and (6+a_T)/42.
 * Returns 0 on success, -1 for an invalid argument, -2 when a_T leaves the
 * range where every D3Q7 weight is non-negative.
 */
int orc_derive(int N, double Ra, double Pr, int cell, double U, double T0,
               orc_params *p) {
    memset(p, 0, sizeof(*p));
    if (N < 3 || !(Ra > 0) || !(Pr > 0) || !(U > 0) || (cell != 0 && cell != 1))
        return -1;
    p->N = N;
    p->cell = cell;
    p->Ra = Ra;
    p->Pr = Pr;
    p->U = U;
    p->T0 = T0;
    p->T_hot = 0.5;
    p->T_cold = -0.5;
    p->H = (double)N;
    p->dT = p->T_hot - p->T_cold;
    p->nu = U * p->H * sqrt(Pr / Ra);
    p->kappa = U * p->H / sqrt(Ra * Pr);
    p->gbeta = U * U / (p->H * p->dT);
    p->tau_f = 3.0 * p->nu + 0.5;
    p->s_e = 1.0 / p->tau_f;
    p->s_q = 8.0 * (2.0 * p->tau_f - 1.0) / (8.0 * p->tau_f - 1.0);
    p->q_k = 3.0 - sqrt(3.0);
    p->q_e = 4.0 * sqrt(3.0) - 6.0;
    p->q_nu = 4.0 * sqrt(3.0) - 6.0;
    /* kappa = (6 + a_T)/21 * (1/q_k - 1/2) solved for a_T */
    p->a_T = 21.0 * p->kappa / (1.0 / p->q_k - 0.5) - 6.0;
    p->wT0 = (1.0 - p->a_T) / 7.0;
    p->wT1 = (6.0 + p->a_T) / 42.0;
    if (!(p->a_T > -6.0 && p->a_T <= 1.0)) return -2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibria and moment-space closed forms                                 */
/* ------------------------------------------------------------------------ */

/* f^eq (Sec. 2.2) with c_s^2 = 1/3. */
void orc_feq(double rho, const double u[3], double *feq) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q19; ++i) {
        double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
        feq[i] = w19(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* g^eq (Sec. 2.3): w_i T [1 + 7/(6+a_T) (e.u)/c_s^2]. */
void orc_geq(const orc_params *p, double T, const double u[3], double *geq) {
    for (int i = 0; i < Q7; ++i) {
        double eu = E7[i][0] * u[0] + E7[i][1] * u[1] + E7[i][2] * u[2];
        double w = i == 0 ? p->wT0 : p->wT1;
        geq[i] = w * T * (1.0 + 7.0 / (6.0 + p->a_T) * eu * 3.0);
    }
}

/* m^eq, the printed closed form (Sec. 2.2). */
void orc_meq(double rho, const double u[3], double *m) {
    double ux = u[0], uy = u[1], uz = u[2];
    double uu = ux * ux + uy * uy + uz * uz;
    double v[Q19] = {1.0,
                     -11.0 + 19.0 * uu,
                     3.0 - 11.0 / 2.0 * uu,
                     ux,
                     -2.0 / 3.0 * ux,
                     uy,
                     -2.0 / 3.0 * uy,
                     uz,
                     -2.0 / 3.0 * uz,
                     2.0 * ux * ux - uy * uy - uz * uz,
                     -0.5 * (2.0 * ux * ux - uy * uy - uz * uz),
                     uy * uy - uz * uz,
                     -0.5 * (uy * uy - uz * uz),
                     ux * uy,
                     uy * uz,
                     ux * uz,
                     0.0,
                     0.0,
                     0.0};
    for (int k = 0; k < Q19; ++k) m[k] = rho * v[k];
}

/* M F~, the printed closed form of the forcing moments (Sec. 2.2). */
void orc_force_moments(const double u[3], const double F[3], double *mf) {
    double ux = u[0], uy = u[1], uz = u[2];
    double Fx = F[0], Fy = F[1], Fz = F[2];
    double uF = ux * Fx + uy * Fy + uz * Fz;
    double v[Q19] = {0.0,
                     38.0 * uF,
                     -11.0 * uF,
                     Fx,
                     -2.0 / 3.0 * Fx,
                     Fy,
                     -2.0 / 3.0 * Fy,
                     Fz,
                     -2.0 / 3.0 * Fz,
                     4.0 * ux * Fx - 2.0 * uy * Fy - 2.0 * uz * Fz,
                     -2.0 * ux * Fx + uy * Fy + uz * Fz,
                     2.0 * uy * Fy - 2.0 * uz * Fz,
                     -uy * Fy + uz * Fz,
                     ux * Fy + uy * Fx,
                     uy * Fz + uz * Fy,
                     ux * Fz + uz * Fx,
                     0.0,
                     0.0,
                     0.0};
    for (int k = 0; k < Q19; ++k) mf[k] = v[k];
}

/* n^eq (Sec. 2.3). */
void orc_neq(const orc_params *p, double T, const double u[3], double *n) {
    n[0] = T;
    n[1] = u[0] * T;
    n[2] = u[1] * T;
    n[3] = u[2] * T;
    n[4] = p->a_T * T;
    n[5] = 0.0;
    n[6] = 0.0;
}

/* Relaxation diagonals S (Sec. 2.2) and Q (Sec. 2.3). */
void orc_relaxation(const orc_params *p, double *S /* 19 */, double *Qd /* 7 */) {
    double sr = 0.0, sj = 0.0;
    double se = p->s_e, seps = p->s_e, snu = p->s_e, spi = p->s_e;
    double sq = p->s_q, sm = p->s_q;
    double s[Q19] = {sr, se, seps, sj, sq, sj, sq, sj, sq, snu,
                     spi, snu, spi, snu, snu, snu, sm, sm, sm};
    for (int k = 0; k < Q19; ++k) S[k] = s[k];
    double q[Q7] = {0.0, p->q_k, p->q_k, p->q_k, p->q_e, p->q_nu, p->q_nu};
    for (int k = 0; k < Q7; ++k) Qd[k] = q[k];
}

/* ------------------------------------------------------------------------ */
/* One-node collision                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double M[Q19 * Q19], Minv[Q19 * Q19];
    double Nm[Q7 * Q7], Ninv[Q7 * Q7];
    double S[Q19], Qd[Q7];
} orc_mats;

static void build_mats(const orc_params *p, orc_mats *mt) {
    orc_matrix_M(mt->M);
    invert(Q19, mt->M, mt->Minv);
    orc_matrix_N(mt->Nm);
    invert(Q7, mt->Nm, mt->Ninv);
    orc_relaxation(p, mt->S, mt->Qd);
}

/*
 * Macroscopic variables of one node (Sec. 2.2 and 2.3):
 *   rho = sum f, T = sum g, F = rho g beta (T - T0) z^, u = (sum e f + F/2)/rho.
 * macro = {rho, ux, uy, uz, T}; F receives the force.
 */
void orc_macros(const orc_params *p, const double *f, const double *g,
                double *macro, double *F) {
    double rho = 0.0, T = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q19; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += E19[i][a] * f[i];
    }
    for (int i = 0; i < Q7; ++i) T += g[i];
    F[0] = 0.0;
    F[1] = 0.0;
    F[2] = rho * p->gbeta * (T - p->T0);
    macro[0] = rho;
    for (int a = 0; a < 3; ++a) macro[1 + a] = (j[a] + 0.5 * F[a]) / rho;
    macro[4] = T;
}

/*
 * Post-collision populations of one node.
 *   f+ = f - M^-1 S (m - m^eq) + M^-1 (I - S/2) M F~        (Eq. MRT)
 *   g+ = g - N^-1 Q (n - n^eq)                               (Eq. MRT_T)
 */
static void collide_node(const orc_params *p, const orc_mats *mt, const double *f,
                         const double *g, double *fp, double *gp, double *macro) {
    double F[3], m[Q19], meq[Q19], mf[Q19], dm[Q19];
    orc_macros(p, f, g, macro, F);
    double rho = macro[0], T = macro[4];
    double u[3] = {macro[1], macro[2], macro[3]};

    for (int k = 0; k < Q19; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < Q19; ++i) m[k] += mt->M[k * Q19 + i] * f[i];
    }
    orc_meq(rho, u, meq);
    orc_force_moments(u, F, mf);
    for (int k = 0; k < Q19; ++k)
        dm[k] = -mt->S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * mt->S[k]) * mf[k];
    for (int i = 0; i < Q19; ++i) {
        double d = 0.0;
        for (int k = 0; k < Q19; ++k) d += mt->Minv[i * Q19 + k] * dm[k];
        fp[i] = f[i] + d;
    }

    double n[Q7], neq[Q7], dn[Q7];
    for (int k = 0; k < Q7; ++k) {
        n[k] = 0.0;
        for (int i = 0; i < Q7; ++i) n[k] += mt->Nm[k * Q7 + i] * g[i];
    }
    orc_neq(p, T, u, neq);
    for (int k = 0; k < Q7; ++k) dn[k] = -mt->Qd[k] * (n[k] - neq[k]);
    for (int i = 0; i < Q7; ++i) {
        double d = 0.0;
        for (int k = 0; k < Q7; ++k) d += mt->Ninv[i * Q7 + k] * dn[k];
        gp[i] = g[i] + d;
    }
}

void orc_collide(const orc_params *p, const double *f, const double *g, double *fp,
                 double *gp, double *macro) {
    orc_mats mt;
    build_mats(p, &mt);
    collide_node(p, &mt, f, g, fp, gp, macro);
}

/* ------------------------------------------------------------------------ */
/* Whole-lattice operations                                                 */
/* ------------------------------------------------------------------------ */

static inline size_t nid(int N, int x, int y, int z) {
    return (size_t)x + (size_t)N * ((size_t)y + (size_t)N * (size_t)z);
}

/* Wall temperature of the face crossed when leaving through axis a toward
 * side s (-1 = plane 0, +1 = plane N); returns 0 for an adiabatic face. */
static int wall_is_isothermal(const orc_params *p, int a, int s, double *Tw) {
    int axis = p->cell == 0 ? 0 : 2;
    if (a != axis) return 0;
    *Tw = s < 0 ? p->T_hot : p->T_cold;
    return 1;
}

/*
 * Initialise from fields: f = f^eq(rho, u), g = g^eq(T, u) (Sec. 2.2 and 2.3
 * equilibria).  fields = [u, v, w, T] planes of V nodes; rho = NULL means 1.
 */
void orc_init_fields(const orc_params *p, const double *fields, const double *rho,
                     double *pop) {
    int N = p->N;
    size_t V = (size_t)N * N * N;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < (long long)V; ++n) {
        double u[3] = {fields[n], fields[V + n], fields[2 * V + n]};
        double T = fields[3 * V + n];
        double fe[Q19], ge[Q7];
        orc_feq(rho ? rho[n] : 1.0, u, fe);
        orc_geq(p, T, u, ge);
        for (int i = 0; i < Q19; ++i) pop[i * V + n] = fe[i];
        for (int i = 0; i < Q7; ++i) pop[(Q19 + i) * V + n] = ge[i];
    }
}

/*
 * One time step: collide every node, then push-stream into pop_out.
 * A link whose target lies outside the box is reflected into the opposite
 * slot of the same node (half-way schemes, Sec. 2.2 and 2.3):
 *   f_opp(x, t+1) = f_i+(x, t)                                   no-slip
 *   g_opp(x, t+1) = -g_i+(x, t) + (6 + a_T)/21 T_w               fixed T
 *   g_opp(x, t+1) =  g_i+(x, t)                                  adiabatic
 * flux[0..3] receive the heat entering the fluid through the hot wall, the
 * cold wall, and the two walls' mid-lines (sum over the links, not averaged):
 * each anti-bounce-back link carries (6 + a_T)/21 T_w - 2 g_i+.
 */
void orc_step(const orc_params *p, const double *pop_in, double *pop_out,
              double *flux /* 4 */) {
    int N = p->N;
    size_t V = (size_t)N * N * N;
    orc_mats mt;
    build_mats(p, &mt);
    int opp19[Q19], opp7[Q7];
    for (int i = 0; i < Q19; ++i) opp19[i] = opposite19(i);
    for (int i = 0; i < Q7; ++i) opp7[i] = opposite7(i);
    double *zflux = (double *)calloc((size_t)N * 4, sizeof(double));
    int mid_lo = (N - 1) / 2, mid_hi = N / 2; /* central index / indices */

#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        double *zf = zflux + 4 * (size_t)z;
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                size_t n = nid(N, x, y, z);
                double f[Q19], g[Q7], fp[Q19], gp[Q7], macro[5];
                for (int i = 0; i < Q19; ++i) f[i] = pop_in[i * V + n];
                for (int i = 0; i < Q7; ++i) g[i] = pop_in[(Q19 + i) * V + n];
                collide_node(p, &mt, f, g, fp, gp, macro);
                int c[3] = {x, y, z};
                for (int i = 0; i < Q19; ++i) {
                    int t[3], inside = 1;
                    for (int a = 0; a < 3; ++a) {
                        t[a] = c[a] + E19[i][a];
                        if (t[a] < 0 || t[a] >= N) inside = 0;
                    }
                    if (inside)
                        pop_out[i * V + nid(N, t[0], t[1], t[2])] = fp[i];
                    else
                        pop_out[opp19[i] * V + n] = fp[i];
                }
                for (int i = 0; i < Q7; ++i) {
                    int t[3], inside = 1, a_out = -1, s_out = 0;
                    for (int a = 0; a < 3; ++a) {
                        t[a] = c[a] + E7[i][a];
                        if (t[a] < 0 || t[a] >= N) {
                            inside = 0;
                            a_out = a;
                            s_out = t[a] < 0 ? -1 : 1;
                        }
                    }
                    if (inside) {
                        pop_out[(Q19 + i) * V + nid(N, t[0], t[1], t[2])] = gp[i];
                        continue;
                    }
                    double Tw;
                    if (wall_is_isothermal(p, a_out, s_out, &Tw)) {
                        double two_w = (6.0 + p->a_T) / 21.0;
                        pop_out[(Q19 + opp7[i]) * V + n] = -gp[i] + two_w * Tw;
                        double q = two_w * Tw - 2.0 * gp[i];
                        int hot = s_out < 0;
                        /* mid-line: central index of y, along z (side-heated)
                         * or along x (Rayleigh-Benard) */
                        int on_mid = (y == mid_lo || y == mid_hi);
                        double wmid = (mid_lo == mid_hi) ? 1.0 : 0.5;
                        zf[hot ? 0 : 1] += q;
                        if (on_mid) zf[hot ? 2 : 3] += wmid * q;
                    } else {
                        pop_out[(Q19 + opp7[i]) * V + n] = gp[i];
                    }
                }
            }
    }
    for (int k = 0; k < 4; ++k) flux[k] = 0.0;
    for (int z = 0; z < N; ++z)
        for (int k = 0; k < 4; ++k) flux[k] += zflux[4 * (size_t)z + k];
    free(zflux);
}

/* Macroscopic planes [rho, u, v, w, T] of every node. */
void orc_macro_fields(const orc_params *p, const double *pop, double *macro) {
    int N = p->N;
    size_t V = (size_t)N * N * N;
#pragma omp parallel for schedule(static)
    for (long long n = 0; n < (long long)V; ++n) {
        double f[Q19], g[Q7], mc[5], F[3];
        for (int i = 0; i < Q19; ++i) f[i] = pop[i * V + n];
        for (int i = 0; i < Q7; ++i) g[i] = pop[(Q19 + i) * V + n];
        orc_macros(p, f, g, mc, F);
        for (int k = 0; k < 5; ++k) macro[k * V + n] = mc[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Observables                                                              */
/* ------------------------------------------------------------------------ */

/*
 * Derivative of a plane phi along axis a at node c, second order:
 *   interior            (phi[k+1] - phi[k-1]) / 2
 *   first node (k = 0)  -4/3 phi_w + phi_0 + 1/3 phi_1   (quadratic through the
 *                        wall point half a cell away and the next two nodes)
 *   last node           mirror image of the above
 * At an adiabatic face of T a mirror ghost node is used instead (dT/dn = 0),
 * giving (phi_1 - phi_0)/2.  wall_lo/wall_hi are the wall values; adiab_lo /
 * adiab_hi select the mirror rule.
 */
double orc_fd_derivative(int N, const double *phi, int a, const int c[3],
                         double wall_lo, double wall_hi, int adiab_lo,
                         int adiab_hi) {
    int k = c[a];
    int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]};
    cm[a] = k - 1;
    cp[a] = k + 1;
    double here = phi[nid(N, c[0], c[1], c[2])];
    if (k > 0 && k < N - 1)
        return 0.5 * (phi[nid(N, cp[0], cp[1], cp[2])] - phi[nid(N, cm[0], cm[1], cm[2])]);
    if (k == 0) {
        double nxt = phi[nid(N, cp[0], cp[1], cp[2])];
        if (adiab_lo) return 0.5 * (nxt - here);
        return -4.0 / 3.0 * wall_lo + here + 1.0 / 3.0 * nxt;
    }
    double prv = phi[nid(N, cm[0], cm[1], cm[2])];
    if (adiab_hi) return 0.5 * (here - prv);
    return 4.0 / 3.0 * wall_hi - here - 1.0 / 3.0 * prv;
}

/*
 * Raw observables of a state, in lattice units (sums in FP64):
 *   r[0], r[1]  mean link heat flux into the fluid through the hot / cold
 *               wall (from flux[0..1] of the last step, divided by N^2)
 *   r[2], r[3]  the same on the wall mid-line (divided by N)
 *   r[4], r[5]  mean of -dT/dn_in at the hot / cold wall, one-sided
 *               (-8 T_w + 9 T_0 - T_1)/3 along the inward normal
 *   r[6], r[7]  the same on the mid-line
 *   r[8]        <u^2 + v^2 + w^2>            r[9]   <w^2>
 *   r[10]       <w T>                        r[11]  <u T>
 *   r[12]       <eps_u> = <nu/2 sum_ij (d_i u_j + d_j u_i)^2>   (Sec. 4)
 *   r[13]       <eps_T> = <kappa sum_i (d_i T)^2>               (Sec. 4)
 *   r[14]       <(rho - 1)^2>                r[15]  <T>
 *   r[16]       <rho - 1>                    r[17]  <(div u)^2>
 * macro = [rho, u, v, w, T] planes; flux as produced by orc_step.
 */
#define NRAW 18
void orc_observables(const orc_params *p, const double *macro, const double *flux,
                     double *r) {
    int N = p->N;
    size_t V = (size_t)N * N * N;
    const double *rho = macro, *U3[3] = {macro + V, macro + 2 * V, macro + 3 * V};
    const double *T = macro + 4 * V;
    int axis = p->cell == 0 ? 0 : 2;
    double *zs = (double *)calloc((size_t)N * NRAW, sizeof(double));
    int mid_lo = (N - 1) / 2, mid_hi = N / 2;
    double wmid = (mid_lo == mid_hi) ? 1.0 : 0.5;

#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        double *acc = zs + (size_t)z * NRAW;
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                int c[3] = {x, y, z};
                size_t n = nid(N, x, y, z);
                double u[3] = {U3[0][n], U3[1][n], U3[2][n]};
                double du[3][3]; /* du[i][j] = d_i u_j */
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        du[i][j] = orc_fd_derivative(N, U3[j], i, c, 0.0, 0.0, 0, 0);
                double dT[3];
                for (int i = 0; i < 3; ++i) {
                    int iso = (i == axis);
                    dT[i] = orc_fd_derivative(N, T, i, c, p->T_hot, p->T_cold, !iso, !iso);
                }
                double eu = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double sij = du[i][j] + du[j][i];
                        eu += sij * sij;
                    }
                eu *= 0.5 * p->nu;
                double eT = p->kappa * (dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]);
                double div = du[0][0] + du[1][1] + du[2][2];
                double drho = rho[n] - 1.0;
                acc[8] += u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                acc[9] += u[2] * u[2];
                acc[10] += u[2] * T[n];
                acc[11] += u[0] * T[n];
                acc[12] += eu;
                acc[13] += eT;
                acc[14] += drho * drho;
                acc[15] += T[n];
                acc[16] += drho;
                acc[17] += div * div;
                /* one-sided wall gradients at the two isothermal walls */
                int k = c[axis];
                int on_mid = (y == mid_lo || y == mid_hi);
                if (k == 0) {
                    int c1[3] = {x, y, z};
                    c1[axis] = 1;
                    double g = -(-8.0 * p->T_hot + 9.0 * T[n] - T[nid(N, c1[0], c1[1], c1[2])]) / 3.0;
                    acc[4] += g;
                    if (on_mid) acc[6] += wmid * g;
                }
                if (k == N - 1) {
                    int c1[3] = {x, y, z};
                    c1[axis] = N - 2;
                    /* inward normal is -axis: -dT/dn_in = +dT/daxis at the wall */
                    double g = (8.0 * p->T_cold - 9.0 * T[n] + T[nid(N, c1[0], c1[1], c1[2])]) / 3.0;
                    acc[5] += g;
                    if (on_mid) acc[7] += wmid * g;
                }
            }
    }
    for (int k = 0; k < NRAW; ++k) r[k] = 0.0;
    for (int z = 0; z < N; ++z)
        for (int k = 0; k < NRAW; ++k) r[k] += zs[(size_t)z * NRAW + k];
    free(zs);
    double A = (double)N * N, L = (double)N;
    r[0] = flux[0] / A;
    r[1] = flux[1] / A;
    r[2] = flux[2] / L;
    r[3] = flux[3] / L;
    r[4] /= A;
    r[5] /= A;
    r[6] /= L;
    r[7] /= L;
    for (int k = 8; k < NRAW; ++k) r[k] /= (double)V;
}

/*
 * Plane-averaged Nusselt number across the cell (Sec. 3, the Nu(y) of its
 * Fig. 4, which runs from the hot to the cold wall; here along x for the
 * side-heated cell and along z for Rayleigh-Benard): on node plane k of that
 * axis a,
 *   out[k] = H/(kappa dT) * ( <u_a T>_k - kappa <d_a T>_k ),
 * the convective plus the conductive heat flux through the plane in units of
 * the conduction flux kappa dT/H, means over the plane's N^2 nodes, d_a T
 * from orc_fd_derivative (central inside; at the first node next to a wall
 * the quadratic through the wall temperature).
 */
void orc_nusselt_profile(const orc_params *p, const double *macro, double *out) {
    int N = p->N;
    size_t V = (size_t)N * N * N;
    int axis = p->cell == 0 ? 0 : 2;
    const double *ua = macro + (size_t)(1 + axis) * V, *T = macro + 4 * V;
    double *conv = (double *)calloc((size_t)N, sizeof(double));
    double *cond = (double *)calloc((size_t)N, sizeof(double));
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                int c[3] = {x, y, z};
                size_t n = nid(N, x, y, z);
                conv[c[axis]] += ua[n] * T[n];
                cond[c[axis]] += orc_fd_derivative(N, T, axis, c, p->T_hot, p->T_cold, 0, 0);
            }
    double A = (double)N * N;
    for (int k = 0; k < N; ++k)
        out[k] = p->H / (p->kappa * p->dT) * (conv[k] / A - p->kappa * cond[k] / A);
    free(conv);
    free(cond);
}

/*
 * Steady-state residual between two macro states (Sec. 3 criterion):
 *   res[0] = max |T - T_old|
 *   res[1] = sum |T - T_old| / sum |T_old|            (relative L1 of T)
 *   res[2] = sum ||u - u_old||_2 / sum ||u_old||_2    (relative L2 of u)
 */
void orc_residual(const orc_params *p, const double *macro, const double *macro_old,
                  double *res) {
    size_t V = (size_t)p->N * p->N * p->N;
    double mx = 0.0, l1 = 0.0, l1o = 0.0, l2 = 0.0, l2o = 0.0;
    for (size_t n = 0; n < V; ++n) {
        double d = fabs(macro[4 * V + n] - macro_old[4 * V + n]);
        if (d > mx) mx = d;
        l1 += d;
        l1o += fabs(macro_old[4 * V + n]);
        double s = 0.0, so = 0.0;
        for (int a = 1; a <= 3; ++a) {
            double du = macro[a * V + n] - macro_old[a * V + n];
            s += du * du;
            so += macro_old[a * V + n] * macro_old[a * V + n];
        }
        l2 += sqrt(s);
        l2o += sqrt(so);
    }
    res[0] = mx;
    res[1] = l1 / l1o;
    res[2] = l2 / l2o;
}
