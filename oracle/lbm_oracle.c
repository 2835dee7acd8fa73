/*
 * FP64 CPU oracle for the D2Q37 (and, built with -DORC_Q=17 or -DORC_Q=9, D2Q17 or D2Q9) lattice Boltzmann
 * scheme with a perfectly matched layer (PML) and open outer boundaries, following
 * arXiv 2504.20169.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant with the HIP library: the lattice
 * weights are re-derived here from the quadrature conditions, the equilibrium is the printed
 * polynomial (Sec. 2, eqs. feq-2, feq-3 and feq-4), and the characteristic boundary solves S x = L with a generic
 * elimination instead of a closed-form inverse.
 *
 * Units: thermal units (c_s = 1, xi_i = r e_i) for rho, u, T in the equilibrium and moments;
 * lattice units (dx = dt = 1, integer e_i) for streaming, the PML gradient term and the
 * characteristic derivatives.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 *
 * Pins (tests/test_oracle_*.py), for every stencil: quadrature moments vs the Gaussian up to the
 * rule's degree (9, 7 and 5) and the published D2Q37 / closed-form D2Q17 and D2Q9 weights;
 * equilibrium moments vs Maxwellian moments (to order 4, 3 and 2); exact conservation on a
 * periodic box; rest and uniform states stationary under every boundary and PML; sigma_max = 0
 * PML identical to no PML; linear growth of Q under a constant deviation; mirror symmetry;
 * linear acoustics vs the linearised Navier-Stokes-Fourier solution; ZG+PML reflecting less
 * than ZG; one step of the PML collision and of the appendix terms in closed form.  The
 * characteristic boundary is pinned in closed form by plane simple waves
 * (tests/test_oracle_lodi_pins.py): an outgoing acoustic wave, an entropy and a shear wave
 * translated by their characteristic speeds over one step and an incoming acoustic wave frozen,
 * on x and y sides, and its corner rule by two such waves leaving through the two sides of a
 * corner.  CBC (A) is pinned by an entropy wave carried along the edge at u_t / r cells per step,
 * a quadratic shear profile along the edge (its viscous part, nu = (tau - 1/2) / r^2), and an
 * acoustic wave running along the edge (its acoustic edge characteristics, with the incoming
 * normal acoustic wave taking Ma times its transverse part, the reading of eq. CBC-Relax),
 * besides uniform-flow invariance, symmetry, its exact reduction to the LODI boundary for plane
 * waves and the trend that it beats the LODI boundary on a vortex outflow.
 */
#include <tgmath.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Arithmetic type: double, the oracle's precision.  A build with -DORC_REAL="long double" takes the
 * same steps in x87 extended precision (64-bit significand); the tests use that build only to
 * measure the double build's own accumulated rounding error (a conditioning floor for the
 * comparison with the library), never as a reference of its own.  The entry points take and
 * return double in both builds. */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

/* Velocity stencil of this compilation: ORC_Q = 37 (default), 17 or 9, one shared library each. */
#ifndef ORC_Q
#define ORC_Q 37
#endif
#define NQ ORC_Q

/* ------------------------------------------------------------------------------------------ */
/* Lattice: Sec. 2 "Velocity stencils".  D2Q37, D2Q17 and D2Q9 are the minimal ninth-, seventh- */
/* and fifth-order rules with integer velocities of maximum displacement 3 and non-negative      */
/* weights.                                                                                      */
/* ------------------------------------------------------------------------------------------ */

static int    LE[NQ][2];   /* integer velocities e_i (lattice units) */
static real LW[NQ];      /* weights w_i */
static real LR;          /* scale r: thermal velocity xi_i = r e_i */
static int    lattice_ok = 0;

/* The shells by |e|^2; the grid search below over |ex|,|ey| <= 3 picks exactly these velocities
 * (for D2Q17: the rest velocity, the 4 axis and 4 diagonal unit velocities, (+-2,+-2) and the 4
 * axis velocities of length 3; for D2Q9: the rest velocity and the axis and diagonal unit
 * velocities). */
#if ORC_Q == 9
#define NS 3
static const int SHELL_E2[NS] = {0, 1, 2};
#elif ORC_Q == 17
#define NS 5
static const int SHELL_E2[NS] = {0, 1, 2, 8, 9};
#else
#define NS 8
static const int SHELL_E2[NS] = {0, 1, 2, 4, 5, 8, 9, 10};
#endif

static int shell_of(int ex, int ey) {
    int s = ex * ex + ey * ey;
    for (int k = 0; k < NS; ++k)
        if (SHELL_E2[k] == s) return k;
    return -1;
}

static long double gauss_moment(int a) { /* E[X^a], X ~ N(0,1) */
    if (a % 2) return 0.0L;
    long double m = 1.0L;
    for (int k = a - 1; k > 0; k -= 2) m *= k;
    return m;
}

static long double ipow_ld(long double x, int n) {
    long double p = 1.0L;
    for (int k = 0; k < n; ++k) p *= x;
    return p;
}

/* Dense solve A x = b (n <= 8) by Gaussian elimination with partial pivoting; b <- x. */
static int solve_ld(int n, long double *A, long double *b) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r * n + c]) > fabsl(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0L) return -1;
        if (p != c) {
            for (int k = 0; k < n; ++k) {
                long double t = A[c * n + k]; A[c * n + k] = A[p * n + k]; A[p * n + k] = t;
            }
            long double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            long double m = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= m * A[c * n + k];
            b[r] -= m * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        long double s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
    return 0;
}

/* The D4-invariant even moment conditions X^a Y^b of the rule (degree 9 for D2Q37, 7 for
 * D2Q17, 5 for D2Q9).  The first NS are solved for the shell weights at a trial q = r^2; the
 * residual of the last fixes q.  For D2Q37 the mixed conditions are dependent among themselves,
 * so X^8 is kept for the residual; for D2Q9, e_x^4 = e_x^2 on unit velocities, so X^2 and X^4
 * differ only by the power of q and X^4 is the residual. */
#if ORC_Q == 9
static const int MOM[NS + 1][2] = {{0, 0}, {2, 0}, {2, 2}, {4, 0}};
#elif ORC_Q == 17
static const int MOM[NS + 1][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0}, {4, 2}};
#else
static const int MOM[NS + 1][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0},
                                   {4, 2}, {6, 2}, {4, 4}, {8, 0}};
#endif

/* Shell sum of e_x^a e_y^b over the integer velocities of shell s. */
static long double shell_sum(int s, int a, int b) {
    long double acc = 0.0L;
    for (int ey = -3; ey <= 3; ++ey)
        for (int ex = -3; ex <= 3; ++ex)
            if (shell_of(ex, ey) == s) acc += ipow_ld(ex, a) * ipow_ld(ey, b);
    return acc;
}

/* For a trial q = r^2, solve the first NS conditions for the shell weights and return the
 * residual of the last. */
static int weights_for(long double q, long double w[NS], long double *resid) {
    long double A[NS * NS], rhs[NS];
    for (int k = 0; k < NS; ++k) {
        int a = MOM[k][0], b = MOM[k][1];
        for (int s = 0; s < NS; ++s) A[k * NS + s] = shell_sum(s, a, b) * ipow_ld(q, (a + b) / 2);
        rhs[k] = gauss_moment(a) * gauss_moment(b);
    }
    if (solve_ld(NS, A, rhs)) return -1;
    for (int s = 0; s < NS; ++s) w[s] = rhs[s];
    int a = MOM[NS][0], b = MOM[NS][1];
    long double m = 0.0L;
    for (int s = 0; s < NS; ++s) m += w[s] * shell_sum(s, a, b) * ipow_ld(q, (a + b) / 2);
    *resid = m - gauss_moment(a) * gauss_moment(b);
    return 0;
}

static int build_lattice(void) {
    if (lattice_ok) return 0;
    int n = 0;
    for (int ey = -3; ey <= 3; ++ey)
        for (int ex = -3; ex <= 3; ++ex)
            if (shell_of(ex, ey) >= 0) { LE[n][0] = ex; LE[n][1] = ey; ++n; }
    if (n != NQ) return -1;
    /* Scan q for sign changes of the ninth residual; keep the root with all weights positive. */
    long double best_q = -1.0L, best_w[NS];
    long double qa = 0.5L, wa[NS], ra;
    if (weights_for(qa, wa, &ra)) return -1;
    for (int step = 1; step <= 5000; ++step) {
        long double qb = 0.5L + step * 0.001L, wb[NS], rb;
        if (weights_for(qb, wb, &rb)) return -1;
        if ((ra < 0) != (rb < 0)) {
            long double lo = qa, hi = qb, rlo = ra;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi), wm[NS], rm;
                weights_for(mid, wm, &rm);
                if ((rm < 0) == (rlo < 0)) { lo = mid; rlo = rm; } else hi = mid;
            }
            long double wq[NS], rq;
            weights_for(0.5L * (lo + hi), wq, &rq);
            int pos = 1;
            for (int s = 0; s < NS; ++s) pos &= (wq[s] > 0.0L);
            if (pos) { best_q = 0.5L * (lo + hi); memcpy(best_w, wq, sizeof wq); break; }
        }
        qa = qb; ra = rb;
    }
    if (best_q < 0) return -1;
    LR = (real)sqrtl(best_q);
    for (int i = 0; i < NQ; ++i) LW[i] = (real)best_w[shell_of(LE[i][0], LE[i][1])];
    lattice_ok = 1;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Equilibrium (c_s = 1, theta = T - 1): eq. feq-4 (fourth-order Hermite expansion) for D2Q37, */
/* eq. feq-3 (third order) for D2Q17, eq. feq-2 (second order) for D2Q9, each the one before    */
/* plus its next Hermite term.  Reading for feq-4: the factor printed as (c_i^2 - 4) in        */
/* the theta (u.c)^2 term is (c_i^2 - 6), the value the fourth-order Hermite contraction gives  */
/* in two dimensions; only with it are mass, momentum and energy moments exact.                 */
/* ------------------------------------------------------------------------------------------ */
static void feq_q(real rho, real ux, real uy, real T, real out[NQ]) {
    real th = T - 1.0;
    real b = ux * ux + uy * uy;
    for (int i = 0; i < NQ; ++i) {
        real cx = LR * LE[i][0], cy = LR * LE[i][1];
        real a = ux * cx + uy * cy;
        real s = cx * cx + cy * cy;
        real t1 = a;
        real t2 = 0.5 * (a * a - b + th * (s - 2.0));
        real t3 = (a / 6.0) * (a * a - 3.0 * b + 3.0 * th * (s - 4.0));
#if ORC_Q == 9
        (void)t3;
        out[i] = LW[i] * rho * (1.0 + t1 + t2);
#elif ORC_Q == 17
        out[i] = LW[i] * rho * (1.0 + t1 + t2 + t3);
#else
        real t4 = ((real)1 / 24) * (a * a * a * a - 6.0 * a * a * b + 3.0 * b * b
                                    + 6.0 * th * (a * a * (s - 6.0) + b * (4.0 - s))
                                    + 3.0 * th * th * (s * s - 8.0 * s + 8.0));
        out[i] = LW[i] * rho * (1.0 + t1 + t2 + t3 + t4);
#endif
    }
}

/* Macroscopic moments, eq. macro with the ideal-gas relation e = (d/2) T, d = 2:
 * rho = sum f, rho u = sum f xi, d rho e = 2 rho T = sum f |xi - u|^2. */
static void moments_q(const real f[NQ], real U[4]) {
    real rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < NQ; ++i) {
        rho += f[i];
        jx += f[i] * (LR * LE[i][0]);
        jy += f[i] * (LR * LE[i][1]);
    }
    real ux = jx / rho, uy = jy / rho;
    real e2 = 0.0;
    for (int i = 0; i < NQ; ++i) {
        real dx = LR * LE[i][0] - ux, dy = LR * LE[i][1] - uy;
        e2 += f[i] * (dx * dx + dy * dy);
    }
    U[0] = rho; U[1] = ux; U[2] = uy; U[3] = e2 / (2.0 * rho);
}

/* ------------------------------------------------------------------------------------------ */
/* Run state                                                                                    */
/* ------------------------------------------------------------------------------------------ */
enum { SIDE_XMIN = 0, SIDE_XMAX = 1, SIDE_YMIN = 2, SIDE_YMAX = 3 };
enum { BC_PERIODIC = 0, BC_ZG = 1, BC_NRBC = 2, BC_NRBC_A = 3 };

typedef struct orc_run {
    int Lx, Ly, Nx, Ny;
    int pml[4];
    int W;
    real sigma_max;
    int bc[4];
    real tau, rho0, ux0, uy0, T0;
    int ready;
    long step;
    real *f;   /* post-collision populations f*[node][i] */
    real *g;   /* post-stream, post-boundary populations */
    real *Qa;  /* PML auxiliary Q[node][i], full grid (zero outside the Q region) */
    real *U;   /* U^n = (rho, ux, uy, T) of the post-stream, post-boundary state, [node][4] */
    real *Un;  /* U^{n+1} */
    real fbar[NQ];
    unsigned pml_terms;   /* appendix: PML moments in the characteristic target (bits I, II, III) */
} orc_run;

static char orc_err[256];
const char *orc_last_error(void) { return orc_err; }
static int fail(const char *m) { snprintf(orc_err, sizeof orc_err, "%s", m); return -1; }

int orc_lattice(int *e, double *w, double *r) {
    if (build_lattice()) return fail("quadrature solve failed");
    for (int i = 0; i < NQ; ++i) { e[2 * i] = LE[i][0]; e[2 * i + 1] = LE[i][1]; w[i] = (double)LW[i]; }
    *r = (double)LR;
    return 0;
}

int orc_feq(double rho, double ux, double uy, double T, double *out) {
    if (build_lattice()) return fail("quadrature solve failed");
    real f[NQ];
    feq_q(rho, ux, uy, T, f);
    for (int i = 0; i < NQ; ++i) out[i] = (double)f[i];
    return 0;
}

int orc_moments_of(const double *f, double *U) {
    if (build_lattice()) return fail("quadrature solve failed");
    real g[NQ], V[4];
    for (int i = 0; i < NQ; ++i) g[i] = f[i];
    moments_q(g, V);
    for (int k = 0; k < 4; ++k) U[k] = (double)V[k];
    return 0;
}

orc_run *orc_create(int Lx, int Ly, double tau, double rho0, double ux0, double uy0, double T0) {
    if (build_lattice()) { fail("quadrature solve failed"); return NULL; }
    if (Lx < 1 || Ly < 1 || !(tau > 0.5)) { fail("bad size or tau"); return NULL; }
    orc_run *r = calloc(1, sizeof *r);
    r->Lx = Lx; r->Ly = Ly; r->tau = tau;
    r->rho0 = rho0; r->ux0 = ux0; r->uy0 = uy0; r->T0 = T0;
    for (int s = 0; s < 4; ++s) r->bc[s] = BC_PERIODIC;
    return r;
}

void orc_destroy(orc_run *r) {
    if (!r) return;
    free(r->f); free(r->g); free(r->Qa); free(r->U); free(r->Un);
    free(r);
}

static int open_x(const orc_run *r) { return r->bc[SIDE_XMIN] != BC_PERIODIC; }
static int open_y(const orc_run *r) { return r->bc[SIDE_YMIN] != BC_PERIODIC; }

int orc_set_pml(orc_run *r, unsigned mask, int W, double sigma_max) {
    if (r->ready) return fail("configure before init");
    if (W < 0 || sigma_max < 0) return fail("bad PML");
    r->W = W; r->sigma_max = sigma_max;
    for (int s = 0; s < 4; ++s) r->pml[s] = (W > 0) && ((mask >> s) & 1u);
    return 0;
}

/* Appendix (eq. NSF-CHAR-PML): which moments of the PML collision term enter the target
 * update of characteristic boundary nodes: bit 0 term I, bit 1 term II, bit 2 term III. */
int orc_set_nrbc_pml_terms(orc_run *r, unsigned flags) {
    if (r->ready) return fail("configure before init");
    if (flags > 7u) return fail("bad PML term flags");
    r->pml_terms = flags;
    return 0;
}

int orc_set_bc(orc_run *r, unsigned mask, int kind) {
    if (r->ready) return fail("configure before init");
    if (kind < 0 || kind > 3) return fail("bad bc");
    for (int s = 0; s < 4; ++s)
        if ((mask >> s) & 1u) r->bc[s] = kind;
    return 0;
}

static void geometry(orc_run *r) {
    r->Nx = r->Lx + (r->pml[0] + r->pml[1]) * r->W;
    r->Ny = r->Ly + (r->pml[2] + r->pml[3]) * r->W;
}

int orc_grid(orc_run *r, int *Nx, int *Ny) {
    geometry(r);
    *Nx = r->Nx; *Ny = r->Ny;
    return 0;
}

/* PML ring level of an axis coordinate: W at the outer layer, 1 next to the bulk, 0 in the bulk
 * (Sec. 3, eq. PML_ramp "i-th level of nodes").  At corners the Chebyshev level is used. */
static int level_axis(int c, int n, int wlo, int whi) {
    if (c < wlo) return wlo - c;
    if (c >= n - whi) return c - (n - whi) + 1;
    return 0;
}

static real sigma_at(const orc_run *r, int x, int y) {
    if (r->W == 0) return 0.0;
    int lx = level_axis(x, r->Nx, r->pml[0] ? r->W : 0, r->pml[1] ? r->W : 0);
    int ly = level_axis(y, r->Ny, r->pml[2] ? r->W : 0, r->pml[3] ? r->W : 0);
    int l = lx > ly ? lx : ly;
    if (l == 0) return 0.0;
    real t = (real)l / (real)r->W;
    return r->sigma_max * t * t;
}

/* Nodes carrying Q: the PML plus the first bulk ring (central differences at level 1 need Q
 * next to it), at least three layers deep so the one-sided difference at the outer layer
 * finds tracked values. */
static int in_qregion(const orc_run *r, int x, int y) {
    if (r->W == 0) return 0;
    int d = r->W + 1 < 3 ? 3 : r->W + 1;
    return (r->pml[0] && x < d) || (r->pml[1] && x >= r->Nx - d) ||
           (r->pml[2] && y < d) || (r->pml[3] && y >= r->Ny - d);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

int orc_init(orc_run *r, const double *rho, const double *ux, const double *uy, const double *T) {
    if (r->ready) return fail("already initialised");
    if ((r->bc[0] == BC_PERIODIC) != (r->bc[1] == BC_PERIODIC) ||
        (r->bc[2] == BC_PERIODIC) != (r->bc[3] == BC_PERIODIC))
        return fail("periodic must be set on both sides of an axis");
    for (int s = 0; s < 4; ++s)
        if (r->pml[s] && r->bc[s] == BC_PERIODIC) return fail("PML on a periodic side");
    geometry(r);
    if ((open_x(r) && r->Nx < 7) || (open_y(r) && r->Ny < 7)) return fail("open axis needs N >= 7");
    size_t nn = (size_t)r->Nx * r->Ny;
    r->f = malloc(nn * NQ * sizeof(real));
    r->g = malloc(nn * NQ * sizeof(real));
    r->Qa = calloc(nn * NQ, sizeof(real));
    r->U = malloc(nn * 4 * sizeof(real));
    r->Un = malloc(nn * 4 * sizeof(real));
    if (!r->f || !r->g || !r->Qa || !r->U || !r->Un) return fail("out of memory");
    /* Sec. 2 (algorithm outline): initialise to the equilibrium of the given fields; the
     * stored state is post-collision, and U^0 is the initial field. */
    for (size_t n = 0; n < nn; ++n) {
        feq_q(rho[n], ux[n], uy[n], T[n], r->f + n * NQ);
        r->U[4 * n] = rho[n]; r->U[4 * n + 1] = ux[n]; r->U[4 * n + 2] = uy[n]; r->U[4 * n + 3] = T[n];
    }
    /* Mean equilibrium of eq. decomp-NJ from the run's mean state. */
    feq_q(r->rho0, r->ux0, r->uy0, r->T0, r->fbar);
    r->step = 0;
    r->ready = 1;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Characteristic boundary (Sec. 4): LODI analysis of the Euler part along the outward normal,   */
/* eq. PNR (incoming amplitudes zero) and eq. thermal_LODI_macro_evo advanced by one explicit     */
/* step.  Primitive variables in the normal frame V = (rho, u_n, u_t, T), p = rho T, gamma = 2:  */
/* A = S^{-1} Lambda S with Lambda = diag(u_n - c, u_n, u_n, u_n + c), c = sqrt(2T).             */
/* Reading (the paper defers the solver to a companion paper): the amplitude of an outgoing wave */
/* k, L_k = lambda_k (S dV/dn)_k, takes the upwind difference over the cell interval that the    */
/* characteristic crosses in one step, nu_k = lambda_k / r cells (linear interpolation at the    */
/* foot point x_b - nu_k n); for nu_k <= 1 this is the first-order explicit upwind update, and    */
/* it stays stable at sound speeds sqrt(2)/r above 1 cell/step (1.18 for D2Q37; 0.86 for D2Q17). */
/* S is frozen at x_b.  The foot point is limited to two cells (the U^n strips are five layers   */
/* deep).                                                                                        */
/* ------------------------------------------------------------------------------------------ */
static void lodi_increment(const orc_run *r, int side, int x, int y, real dU[4]) {
    int nx = side == SIDE_XMIN ? -1 : side == SIDE_XMAX ? 1 : 0;
    int ny = side == SIDE_YMIN ? -1 : side == SIDE_YMAX ? 1 : 0;
    real V[3][4];
    for (int k = 0; k < 3; ++k) {
        const real *u = r->U + 4 * ((size_t)(y - k * ny) * r->Nx + (x - k * nx));
        real un = nx ? nx * u[1] : ny * u[2];
        real ut = nx ? u[2] : u[1];
        V[k][0] = u[0]; V[k][1] = un; V[k][2] = ut; V[k][3] = u[3];
    }
    real rho = V[0][0], un = V[0][1], T = V[0][3];
    real c = sqrt(2.0 * T);
    real lam[4] = {un - c, un, un, un + c};
    real S[16] = {T, -rho * c, 0, rho,
                    T, 0, 0, -rho,
                    0, 0, 1, 0,
                    T, rho * c, 0, rho};
    long double Lb[4];
    for (int k = 0; k < 4; ++k) {
        real w[3];
        for (int j = 0; j < 3; ++j) {
            w[j] = 0.0;
            for (int m = 0; m < 4; ++m) w[j] += S[4 * k + m] * V[j][m];
        }
        if (lam[k] > 0.0) {                    /* outgoing: keep its amplitude */
            real nu = lam[k] / LR;
            if (nu > 2.0) nu = 2.0;
            int j = (int)floor(nu);
            if (j > 1) j = 1;
            real phi = nu - j;
            real wfoot = (1.0 - phi) * w[j] + phi * w[j + 1];
            Lb[k] = LR * (w[0] - wfoot);       /* = lambda_k (S dV/dn)_k over the crossed interval */
        } else {
            Lb[k] = 0.0;                       /* incoming: eq. PNR */
        }
    }
    /* dV/dt = -S^{-1} Lbar (thermal units); one lattice step is 1/r thermal time units per cell. */
    long double A[16];
    for (int k = 0; k < 16; ++k) A[k] = S[k];
    solve_ld(4, A, Lb);
    real d[4];
    for (int k = 0; k < 4; ++k) d[k] = -(real)Lb[k] / LR;
    dU[0] = d[0];
    dU[3] = d[3];
    if (nx) { dU[1] = nx * d[1]; dU[2] = d[2]; }
    else    { dU[2] = ny * d[1]; dU[1] = d[2]; }
}

/* Primitive state (rho, u_a, u_b, T) of node (x, y) with u_a along the unit lattice vector
 * (ax, ay) and u_b along (bx, by). */
static void prim_frame(const orc_run *r, int x, int y, int ax, int ay, int bx, int by, real V[4]) {
    const real *u = r->U + 4 * ((size_t)y * r->Nx + x);
    V[0] = u[0];
    V[1] = ax * u[1] + ay * u[2];
    V[2] = bx * u[1] + by * u[2];
    V[3] = u[3];
}

/* Left eigenvectors of the 2-D Euler flux Jacobian along a direction, for primitive variables
 * (rho, u_along, u_across, T), p = rho T, gamma = 2, c = sqrt(2T): rows for the eigenvalues
 * u - c, u (entropy), u (shear), u + c. */
static void left_eig(real rho, real T, real S[16]) {
    const real c = sqrt(2.0 * T);
    const real v[16] = {T, -rho * c, 0, rho,
                          T, 0, 0, -rho,
                          0, 0, 1, 0,
                          T, rho * c, 0, rho};
    memcpy(S, v, sizeof v);
}

/* x = S^{-1} b for a 4x4 S (generic elimination). */
static void solve4(const real S[16], const real b[4], real x[4]) {
    long double A[16], y[4];
    for (int k = 0; k < 16; ++k) A[k] = S[k];
    for (int k = 0; k < 4; ++k) y[k] = b[k];
    solve_ld(4, A, y);
    for (int k = 0; k < 4; ++k) x[k] = (real)y[k];
}

/* Increment over one step of the edge characteristics of the states Vn[j - 2 .. j + 2] (normal
 * frame (rho, u_n, u_t, T)) at Vn[j]: each characteristic variable of the Euler flux along the
 * edge, with the eigenvectors frozen at Vn[j], moves over the interval its characteristic
 * crosses in one step (linear interpolation at the foot point, at most 2 cells). */
static void edge_advect(const real Vn[7][4], int j, real dV[4]) {
    const real *v = Vn[j];
    const real rho = v[0], ut = v[2], T = v[3], c = sqrt(2.0 * T);
    real St[16];
    left_eig(rho, T, St);
    const real lam[4] = {ut - c, ut, ut, ut + c};
    real dW[4];
    for (int k = 0; k < 4; ++k) {
        real w[5];
        for (int m = 0; m < 5; ++m) {
            const real *u = Vn[j - 2 + m];
            const real vt[4] = {u[0], u[2], u[1], u[3]};   /* (rho, u_t, u_n, T) */
            w[m] = 0.0;
            for (int l = 0; l < 4; ++l) w[m] += St[4 * k + l] * vt[l];
        }
        real nu = lam[k] / LR;                             /* cells per step along +t */
        if (!(nu == nu)) nu = 0.0;
        if (nu > 2.0) nu = 2.0;
        if (nu < -2.0) nu = -2.0;
        const real a = fabs(nu);
        int i = (int)floor(a);
        if (i > 1) i = 1;
        const real phi = a - i;
        const int sgn = nu > 0.0 ? -1 : 1;                   /* foot point at -nu */
        /* in differences, so that a state constant along the edge gives exactly zero */
        dW[k] = -((1.0 - phi) * (w[2] - w[2 + sgn * i]) + phi * (w[2] - w[2 + sgn * (i + 1)]));
    }
    real dt[4];
    solve4(St, dW, dt);
    dV[0] = dt[0]; dV[1] = dt[2]; dV[2] = dt[1]; dV[3] = dt[3];
}

/* Characteristic boundary "CBC (A)" (Sec. 4, eq. thermal_CBC_macro_evo; Sec. 5.2, eq. CBC-Relax):
 * the one-step target of a boundary node on one open side keeps, besides the LODI amplitudes of
 * its outgoing waves, the transverse (Euler flux along the edge) and viscous parts of the
 * characteristic system, dU/dt = -S^{-1} (Lbar + T + V), with the incoming amplitudes relaxed.
 * Readings (the paper defers the solver to a companion paper):
 *  - transverse part T: the Euler flux along the edge in the edge's own characteristic
 *    variables, each advected over the interval its characteristic crosses in one step (as the
 *    normal LODI amplitudes), on the boundary node's own layer (edge_advect);
 *  - viscous part V: the tangential second derivatives only (the normal viscous fluxes of an
 *    outflow vanish): nu d2u/dt2 for both velocity components and 2 nu d2T/dt2 (Pr = 1,
 *    c_p/c_v = 2), nu = (tau - 1/2)/r^2 in lattice units, central differences along the edge,
 *    taken of the transverse-advected states (advection, then diffusion: an unsplit sum of the
 *    two explicit parts is unstable once the edge CFL number plus twice the diffusion number
 *    exceeds one, which the D2Q17 sound speed alone nearly reaches);
 *  - eq. CBC-Relax with T and V taken as right-hand-side terms: an incoming amplitude is
 *    (1 - Ma) T_inc + V_inc of them, which leaves it Ma T_inc per step (Ma = |u0|, c_s = 1).
 * Edge neighbours beyond an open edge's ends repeat the end node.  Returns the increment in the
 * global frame. */
static void cbc_a_increment(const orc_run *r, int side, int x, int y, real dU[4]) {
    const int Nx = r->Nx, Ny = r->Ny;
    const int nx = side == SIDE_XMIN ? -1 : side == SIDE_XMAX ? 1 : 0;
    const int ny = side == SIDE_YMIN ? -1 : side == SIDE_YMAX ? 1 : 0;
    const int tx = nx ? 0 : 1, ty = nx ? 1 : 0;        /* tangent: +y on x sides, +x on y sides */
    const int nt = nx ? Ny : Nx, ct = nx ? y : x;
    const int topen = nx ? open_y(r) : open_x(r);
    /* states along the edge, ct - 3 .. ct + 3, in the normal frame (rho, u_n, u_t, T) */
    real Vn[7][4];
    for (int j = -3; j <= 3; ++j) {
        int c = ct + j;
        if (topen) c = clampi(c, 0, nt - 1);
        else c = ((c % nt) + nt) % nt;
        prim_frame(r, nx ? x : c, nx ? c : y, nx, ny, tx, ty, Vn[j + 3]);
    }
    const real rho = Vn[3][0], un = Vn[3][1], T = Vn[3][3];
    const real c = sqrt(2.0 * T);
    real S[16];
    left_eig(rho, T, S);
    const real lam[4] = {un - c, un, un, un + c};
    /* 1. LODI amplitudes of the outgoing normal characteristics (as lodi_increment) */
    real D[4];
    {
        real V[3][4];
        for (int k = 0; k < 3; ++k) prim_frame(r, x - k * nx, y - k * ny, nx, ny, tx, ty, V[k]);
        for (int k = 0; k < 4; ++k) {
            real w[3];
            for (int j = 0; j < 3; ++j) {
                w[j] = 0.0;
                for (int m = 0; m < 4; ++m) w[j] += S[4 * k + m] * V[j][m];
            }
            D[k] = 0.0;
            if (lam[k] > 0.0) {
                real nu = lam[k] / LR;
                if (nu > 2.0) nu = 2.0;
                int j = (int)floor(nu);
                if (j > 1) j = 1;
                real phi = nu - j;
                D[k] = (1.0 - phi) * (w[0] - w[j]) + phi * (w[0] - w[j + 1]);
            }
        }
    }
    /* 2. transverse part at the node and its two edge neighbours, then 3. the viscous part of
     * the advected states */
    real Va[3][4], dVT[4];
    for (int j = -1; j <= 1; ++j) {
        real d[4];
        edge_advect(Vn, j + 3, d);
        for (int m = 0; m < 4; ++m) Va[j + 1][m] = Vn[j + 3][m] + d[m];
        if (j == 0) memcpy(dVT, d, sizeof d);
    }
    real dVV[4] = {0.0, 0.0, 0.0, 0.0};
    if (!(topen && (ct == 0 || ct == nt - 1))) {
        const real nuv = (r->tau - 0.5) / (LR * LR);
        dVV[1] = nuv * (Va[2][1] - 2.0 * Va[1][1] + Va[0][1]);
        dVV[2] = nuv * (Va[2][2] - 2.0 * Va[1][2] + Va[0][2]);
        dVV[3] = 2.0 * nuv * (Va[2][3] - 2.0 * Va[1][3] + Va[0][3]);
    }
    /* 4. characteristic combination: outgoing waves take LODI + T + V, incoming Ma T */
    const real ma = sqrt(r->ux0 * r->ux0 + r->uy0 * r->uy0);
    real dw[4];
    for (int k = 0; k < 4; ++k) {
        real a = 0.0, b = 0.0;
        for (int m = 0; m < 4; ++m) { a += S[4 * k + m] * dVT[m]; b += S[4 * k + m] * dVV[m]; }
        dw[k] = lam[k] > 0.0 ? -D[k] + a + b : ma * a;
    }
    real d[4];
    solve4(S, dw, d);
    dU[0] = d[0];
    dU[3] = d[3];
    if (nx) { dU[1] = nx * d[1]; dU[2] = d[2]; }
    else    { dU[2] = ny * d[1]; dU[1] = d[2]; }
}

/* d Q_i / d alpha at (x, y), alpha = 0 (x) or 1 (y): central differences, one-sided second
 * order at the outermost layer of an open axis (eqs. FD-dx-center, FD-dx-bw). */
static real grad_q(const orc_run *r, int x, int y, int i, int al) {
    const int Nx = r->Nx, Ny = r->Ny;
    int c = al ? y : x, nmax = al ? Ny : Nx, op = al ? open_y(r) : open_x(r);
#define QAT(cc) (al ? r->Qa[((size_t)(cc) * Nx + x) * NQ + i] : r->Qa[((size_t)y * Nx + (cc)) * NQ + i])
    real d;
    if (op && c == 0)
        d = -0.5 * (3.0 * QAT(0) - 4.0 * QAT(1) + QAT(2));
    else if (op && c == nmax - 1)
        d = 0.5 * (3.0 * QAT(nmax - 1) - 4.0 * QAT(nmax - 2) + QAT(nmax - 3));
    else {
        int cp = c + 1, cm = c - 1;
        if (!op) { cp = (cp + nmax) % nmax; cm = (cm + nmax) % nmax; }
        d = 0.5 * (QAT(cp) - QAT(cm));
    }
#undef QAT
    return d;
}

/* Appendix, eq. NSF-CHAR-PML: with a PML the macroscopic equations carry extra source terms
 * built from the auxiliary moments, phi = (1, xi_x, xi_y, |xi|^2/2):
 *   I = sum_i phi_i e_i . grad Q_i,  II = 2 sum_i phi_i fhat_i,  III = sigma sum_i phi_i Q_i,
 * in conserved variables (rho, rho u, rho (|u|^2/2 + T)).  Over one step the selected terms move
 * the characteristic target by s = +sigma (I + II + III), the signs printed in the appendix,
 * converted to the primitive (rho, ux, uy, T) at U^n by the chain rule.  Q and U are those of
 * level n. */
static void pml_source(const orc_run *r, int x, int y, real dU[4]) {
    dU[0] = dU[1] = dU[2] = dU[3] = 0.0;
    const real sg = sigma_at(r, x, y);
    if (!(sg > 0.0) || !r->pml_terms) return;
    const size_t n = (size_t)y * r->Nx + x;
    const real *u = r->U + 4 * n;
    real fe[NQ];
    feq_q(u[0], u[1], u[2], u[3], fe);
    real s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < NQ; ++i) {
        real xi_x = LR * LE[i][0], xi_y = LR * LE[i][1];
        real phi[4] = {1.0, xi_x, xi_y, 0.5 * (xi_x * xi_x + xi_y * xi_y)};
        real a = 0.0;
        if (r->pml_terms & 1u) a += LE[i][0] * grad_q(r, x, y, i, 0) + LE[i][1] * grad_q(r, x, y, i, 1);
        if (r->pml_terms & 2u) a += 2.0 * (fe[i] - r->fbar[i]);
        if (r->pml_terms & 4u) a += sg * r->Qa[n * NQ + i];
        for (int k = 0; k < 4; ++k) s[k] += phi[k] * a;
    }
    for (int k = 0; k < 4; ++k) s[k] *= sg;
    const real rho = u[0], ux = u[1], uy = u[2], T = u[3];
    dU[0] = s[0];
    dU[1] = (s[1] - ux * s[0]) / rho;
    dU[2] = (s[2] - uy * s[0]) / rho;
    dU[3] = (s[3] - ux * s[1] - uy * s[2] + (0.5 * (ux * ux + uy * uy) - T) * s[0]) / rho;
}

static int is_boundary_side(const orc_run *r, int side, int x, int y) {
    if (r->bc[side] == BC_PERIODIC) return 0;
    switch (side) {
    case SIDE_XMIN: return x < 3;
    case SIDE_XMAX: return x >= r->Nx - 3;
    case SIDE_YMIN: return y < 3;
    default:        return y >= r->Ny - 3;
    }
}

/* One time step: stream (eq. lbe), boundary (eq. zg-bc or the characteristic Dirichlet fill),
 * moments (eq. macro), Q update (eq. PMLQ, trapezoid), collision (BGK + eq. PMLCOLL). */
static void one_step(orc_run *r) {
    const int Nx = r->Nx, Ny = r->Ny;
    const int ox = open_x(r), oy = open_y(r);

    /* 1. pull streaming; populations whose source lies outside an open edge are unknown. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            real *gn = r->g + ((size_t)y * Nx + x) * NQ;
            for (int i = 0; i < NQ; ++i) {
                int sx = x - LE[i][0], sy = y - LE[i][1];
                int known = 1;
                if (ox) known &= (sx >= 0 && sx < Nx); else sx = ((sx % Nx) + Nx) % Nx;
                if (oy) known &= (sy >= 0 && sy < Ny); else sy = ((sy % Ny) + Ny) % Ny;
                gn[i] = known ? r->f[((size_t)sy * Nx + sx) * NQ + i] : NAN;
            }
        }

    /* 2. boundary nodes: the outer three layers of every open side.  ZG copies all q
     * populations of the adjacent fluid node x_f; the characteristic boundary adds
     * feq(U_tgt) - feq(U(x_f)) to them (non-equilibrium extrapolation). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            int bnd = 0, nrbc = 0;
            for (int s = 0; s < 4; ++s)
                if (is_boundary_side(r, s, x, y)) {
                    bnd += 1;
                    nrbc |= (r->bc[s] == BC_NRBC || r->bc[s] == BC_NRBC_A);
                }
            if (!bnd) continue;
            int xf = ox ? clampi(x, 3, Nx - 4) : x;
            int yf = oy ? clampi(y, 3, Ny - 4) : y;
            const real *gf = r->g + ((size_t)yf * Nx + xf) * NQ;
            real *gb = r->g + ((size_t)y * Nx + x) * NQ;
            if (!nrbc) {
                for (int i = 0; i < NQ; ++i) gb[i] = gf[i];
                continue;
            }
            const real *Ub = r->U + 4 * ((size_t)y * Nx + x);
            real Ut[4] = {Ub[0], Ub[1], Ub[2], Ub[3]};
            for (int s = 0; s < 4; ++s) {
                if (!is_boundary_side(r, s, x, y)) continue;
                real d[4];
                if (r->bc[s] == BC_NRBC_A && bnd == 1) cbc_a_increment(r, s, x, y, d);
                else if (r->bc[s] == BC_NRBC || r->bc[s] == BC_NRBC_A) lodi_increment(r, s, x, y, d);
                else continue;
                for (int k = 0; k < 4; ++k) Ut[k] += d[k];
            }
            {
                real d[4];
                pml_source(r, x, y, d);
                for (int k = 0; k < 4; ++k) Ut[k] += d[k];
            }
            real Uf[4], ft[NQ], ff[NQ];
            moments_q(gf, Uf);
            feq_q(Ut[0], Ut[1], Ut[2], Ut[3], ft);
            feq_q(Uf[0], Uf[1], Uf[2], Uf[3], ff);
            for (int i = 0; i < NQ; ++i) gb[i] = ft[i] + (gf[i] - ff[i]);
        }

    /* 3. moments of the post-stream, post-boundary state. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            size_t n = (size_t)y * Nx + x;
            moments_q(r->g + n * NQ, r->Un + 4 * n);
        }

    /* 4. Q^{n+1} = Q^n + (1/2)(fhat^n + fhat^{n+1}), fhat = feq - fbar (eq. PMLQ, trapezoid). */
    if (r->W > 0) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < Ny; ++y)
            for (int x = 0; x < Nx; ++x) {
                if (!in_qregion(r, x, y)) continue;
                size_t n = (size_t)y * Nx + x;
                real e0[NQ], e1[NQ];
                const real *u0 = r->U + 4 * n, *u1 = r->Un + 4 * n;
                feq_q(u0[0], u0[1], u0[2], u0[3], e0);
                feq_q(u1[0], u1[1], u1[2], u1[3], e1);
                real *q = r->Qa + n * NQ;
                for (int i = 0; i < NQ; ++i)
                    q[i] = q[i] + 0.5 * ((e0[i] - r->fbar[i]) + (e1[i] - r->fbar[i]));
            }
    }

    /* 5. collision: BGK, then on PML nodes (sigma > 0) add
     *    Omega^PML = -sigma (e_i . grad Q_i + 2 fhat_i + sigma Q_i)   (eq. PMLCOLL)
     * with grad Q central, one-sided at the outermost layer of an open axis (eqs. FD-dx-*). */
    const real inv_tau = 1.0 / r->tau;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            size_t n = (size_t)y * Nx + x;
            const real *gn = r->g + n * NQ;
            const real *u = r->Un + 4 * n;
            real fe[NQ];
            feq_q(u[0], u[1], u[2], u[3], fe);
            real *fo = r->f + n * NQ;
            real sg = sigma_at(r, x, y);
            for (int i = 0; i < NQ; ++i) fo[i] = gn[i] - inv_tau * (gn[i] - fe[i]);
            if (sg > 0.0) {
                for (int i = 0; i < NQ; ++i) {
                    real d[2];
                    for (int al = 0; al < 2; ++al) {
                        int c = al ? y : x, nmax = al ? Ny : Nx, op = al ? oy : ox;
#define QAT(cc) (al ? r->Qa[((size_t)(cc) * Nx + x) * NQ + i] : r->Qa[((size_t)y * Nx + (cc)) * NQ + i])
                        if (op && c == 0)
                            d[al] = -0.5 * (3.0 * QAT(0) - 4.0 * QAT(1) + QAT(2));
                        else if (op && c == nmax - 1)
                            d[al] = 0.5 * (3.0 * QAT(nmax - 1) - 4.0 * QAT(nmax - 2) + QAT(nmax - 3));
                        else {
                            int cp = c + 1, cm = c - 1;
                            if (!op) { cp = (cp + nmax) % nmax; cm = (cm + nmax) % nmax; }
                            d[al] = 0.5 * (QAT(cp) - QAT(cm));
                        }
#undef QAT
                    }
                    real q = r->Qa[n * NQ + i];
                    real fhat = fe[i] - r->fbar[i];
                    real om = -sg * (LE[i][0] * d[0] + LE[i][1] * d[1] + 2.0 * fhat + sg * q);
                    fo[i] = fo[i] + om;
                }
            }
        }

    real *t = r->U; r->U = r->Un; r->Un = t;
    r->step += 1;
}

int orc_step(orc_run *r, long nsteps, int nthreads) {
    if (!r->ready) return fail("not initialised");
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (long k = 0; k < nsteps; ++k) one_step(r);
    return 0;
}

long orc_step_count(const orc_run *r) { return r->step; }

int orc_threads(void) { return omp_get_max_threads(); }

/* Moments of the current state (Sec. 2, last step of the algorithm outline): those of the
 * post-stream, post-boundary populations of the last step; at step 0 those of f*(0). */
static int moments_real(const orc_run *r, real *rho, real *ux, real *uy, real *T) {
    if (!r->ready) return fail("not initialised");
    size_t nn = (size_t)r->Nx * r->Ny;
    for (size_t n = 0; n < nn; ++n) {
        real U[4];
        if (r->step == 0) moments_q(r->f + n * NQ, U);
        else memcpy(U, r->U + 4 * n, sizeof U);
        if (rho) rho[n] = U[0];
        if (ux) ux[n] = U[1];
        if (uy) uy[n] = U[2];
        if (T) T[n] = U[3];
    }
    return 0;
}

/* moments_real for the caller, in double. */
int orc_moments(const orc_run *r, double *rho, double *ux, double *uy, double *T) {
    if (!r->ready) return fail("not initialised");
    size_t nn = (size_t)r->Nx * r->Ny;
    for (size_t n = 0; n < nn; ++n) {
        real U[4];
        if (r->step == 0) moments_q(r->f + n * NQ, U);
        else memcpy(U, r->U + 4 * n, sizeof U);
        if (rho) rho[n] = (double)U[0];
        if (ux) ux[n] = (double)U[1];
        if (uy) uy[n] = (double)U[2];
        if (T) T[n] = (double)U[3];
    }
    return 0;
}

/* Post-collision populations, layout [i][y][x] in this file's velocity order. */
int orc_populations(const orc_run *r, double *out) {
    if (!r->ready) return fail("not initialised");
    size_t nn = (size_t)r->Nx * r->Ny;
    for (int i = 0; i < NQ; ++i)
        for (size_t n = 0; n < nn; ++n) out[(size_t)i * nn + n] = (double)r->f[n * NQ + i];
    return 0;
}

int orc_pml_q(const orc_run *r, double *out) {
    if (!r->ready) return fail("not initialised");
    size_t nn = (size_t)r->Nx * r->Ny;
    for (int i = 0; i < NQ; ++i)
        for (size_t n = 0; n < nn; ++n) out[(size_t)i * nn + n] = (double)r->Qa[n * NQ + i];
    return 0;
}

int orc_sigma(orc_run *r, double *out) {
    geometry(r);
    for (int y = 0; y < r->Ny; ++y)
        for (int x = 0; x < r->Nx; ++x) out[(size_t)y * r->Nx + x] = (double)sigma_at(r, x, y);
    return 0;
}

/* Global relative L2 errors over the bulk (Sec. 5 "Reference Simulation"):
 * e_Z = sqrt( sum_bulk ((Z - Zref)/Zref)^2 ), Z in {rho, ux, T}; references are bulk-sized
 * Ly x Lx arrays; the sum runs in row-major order. */
int orc_error_norms(const orc_run *r, const double *ref_rho, const double *ref_ux,
                    const double *ref_T, double out[3]) {
    if (!r->ready) return fail("not initialised");
    int x0 = r->pml[0] ? r->W : 0, y0 = r->pml[2] ? r->W : 0;
    size_t nn = (size_t)r->Nx * r->Ny;
    real *rho = malloc(nn * sizeof(real)), *ux = malloc(nn * sizeof(real)),
           *T = malloc(nn * sizeof(real));
    moments_real(r, rho, ux, NULL, T);
    real s[3] = {0, 0, 0};
    for (int y = 0; y < r->Ly; ++y)
        for (int x = 0; x < r->Lx; ++x) {
            size_t n = (size_t)(y + y0) * r->Nx + (x + x0), m = (size_t)y * r->Lx + x;
            real a = (rho[n] - ref_rho[m]) / ref_rho[m];
            real b = (ux[n] - ref_ux[m]) / ref_ux[m];
            real c = (T[n] - ref_T[m]) / ref_T[m];
            s[0] += a * a; s[1] += b * b; s[2] += c * c;
        }
    free(rho); free(ux); free(T);
    for (int k = 0; k < 3; ++k) out[k] = (double)sqrt(s[k]);
    return 0;
}
