/* Sanitizer driver for the CPU oracle (oracle/lbm_oracle.c): built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py), it walks every entry point over small
 * grids in every boundary configuration -- each boundary kind with and without a PML, a PML on
 * some sides only, the appendix's PML-moment terms, one and two threads -- and the documented
 * error paths, so an out-of-bounds access, a use after free, a leak or undefined arithmetic in
 * the oracle ends the run with a report.  Exit status 0 when every call behaved as documented.
 * Compiled once per stencil with -DORC_Q. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_run orc_run;
const char *orc_last_error(void);
int orc_lattice(int *e, double *w, double *r);
int orc_feq(double rho, double ux, double uy, double T, double *out);
int orc_moments_of(const double *f, double *U);
orc_run *orc_create(int Lx, int Ly, double tau, double rho0, double ux0, double uy0, double T0);
void orc_destroy(orc_run *r);
int orc_set_pml(orc_run *r, unsigned mask, int W, double sigma_max);
int orc_set_nrbc_pml_terms(orc_run *r, unsigned flags);
int orc_set_bc(orc_run *r, unsigned mask, int kind);
int orc_grid(orc_run *r, int *Nx, int *Ny);
int orc_init(orc_run *r, const double *rho, const double *ux, const double *uy, const double *T);
int orc_step(orc_run *r, long nsteps, int nthreads);
long orc_step_count(const orc_run *r);
int orc_moments(const orc_run *r, double *rho, double *ux, double *uy, double *T);
int orc_populations(const orc_run *r, double *out);
int orc_pml_q(const orc_run *r, double *out);
int orc_sigma(orc_run *r, double *out);
int orc_error_norms(const orc_run *r, const double *ref_rho, const double *ref_ux,
                    const double *ref_T, double out[3]);

#ifndef ORC_Q
#define ORC_Q 37
#endif

static int failures = 0;

#define EXPECT(cond, what)                                                        \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "FAIL q=%d: %s (%s)\n", ORC_Q, what, orc_last_error()); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

/* fields of a small vortex-free perturbed state: smooth, positive, deterministic */
static void fields(int Nx, int Ny, double *rho, double *ux, double *uy, double *T) {
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            size_t n = (size_t)y * Nx + x;
            double a = sin(0.7 * x + 0.3 * y), b = cos(0.4 * x - 0.9 * y);
            rho[n] = 1.0 + 1e-3 * a;
            ux[n] = 0.05 + 1e-3 * b;
            uy[n] = -1e-3 * a * b;
            T[n] = 1.0 + 5e-4 * b;
        }
}

static void run_case(int Lx, int Ly, int bcx, int bcy, unsigned pml_mask, int W, unsigned terms,
                     int threads) {
    orc_run *r = orc_create(Lx, Ly, 0.8, 1.0, 0.05, 0.0, 1.0);
    EXPECT(r != NULL, "create");
    if (!r) return;
    EXPECT(orc_set_bc(r, 1 | 2, bcx) == 0, "set_bc x");
    EXPECT(orc_set_bc(r, 4 | 8, bcy) == 0, "set_bc y");
    EXPECT(orc_set_pml(r, pml_mask, W, 0.05) == 0, "set_pml");
    EXPECT(orc_set_nrbc_pml_terms(r, terms) == 0, "set terms");
    int Nx = 0, Ny = 0;
    orc_grid(r, &Nx, &Ny);
    size_t nn = (size_t)Nx * Ny;
    double *F = malloc(4 * nn * sizeof(double));
    double *P = malloc((size_t)ORC_Q * nn * sizeof(double));
    double *Q = malloc((size_t)ORC_Q * nn * sizeof(double));
    double *S = malloc(nn * sizeof(double));
    double *ref = malloc(3 * (size_t)Lx * Ly * sizeof(double));
    fields(Nx, Ny, F, F + nn, F + 2 * nn, F + 3 * nn);
    EXPECT(orc_sigma(r, S) == 0, "sigma");
    EXPECT(orc_init(r, F, F + nn, F + 2 * nn, F + 3 * nn) == 0, "init");
    EXPECT(orc_set_bc(r, 1, bcx) != 0, "setter after init must fail");
    EXPECT(orc_init(r, F, F + nn, F + 2 * nn, F + 3 * nn) != 0, "second init must fail");
    EXPECT(orc_moments(r, F, F + nn, F + 2 * nn, F + 3 * nn) == 0, "moments at step 0");
    EXPECT(orc_step(r, 4, threads) == 0, "step");
    EXPECT(orc_step_count(r) == 4, "step count");
    EXPECT(orc_moments(r, F, F + nn, F + 2 * nn, F + 3 * nn) == 0, "moments");
    EXPECT(orc_populations(r, P) == 0, "populations");
    EXPECT(orc_pml_q(r, Q) == 0, "pml_q");
    for (size_t n = 0; n < 4 * nn; ++n) EXPECT(isfinite(F[n]), "finite moments");
    for (size_t n = 0; n < (size_t)ORC_Q * nn; ++n) EXPECT(isfinite(P[n]) && isfinite(Q[n]), "finite state");
    for (size_t m = 0; m < 3 * (size_t)Lx * Ly; ++m) ref[m] = 1.0 + 1e-3 * (double)(m % 7);
    double e[3];
    EXPECT(orc_error_norms(r, ref, ref + (size_t)Lx * Ly, ref + 2 * (size_t)Lx * Ly, e) == 0, "error norms");
    EXPECT(isfinite(e[0]) && isfinite(e[1]) && isfinite(e[2]), "finite norms");
    free(F); free(P); free(Q); free(S); free(ref);
    orc_destroy(r);
}

int main(void) {
    int e[2 * ORC_Q];
    double w[ORC_Q], rr, f[ORC_Q], U[4];
    EXPECT(orc_lattice(e, w, &rr) == 0, "lattice");
    EXPECT(orc_feq(1.01, 0.02, -0.01, 0.99, f) == 0, "feq");
    EXPECT(orc_moments_of(f, U) == 0, "moments_of");
    EXPECT(fabs(U[0] - 1.01) < 1e-12 && fabs(U[3] - 0.99) < 1e-12, "moments of feq");

    /* boundary kinds: 0 periodic, 1 ZG, 2 characteristic (LODI), 3 CBC (A) */
    int cases = 0;
    for (int bcx = 0; bcx < 4; ++bcx)
        for (int bcy = 0; bcy < 4; ++bcy)
            for (int W = 0; W <= 4; W += 4) {
                unsigned mask = 0;
                if (bcx) mask |= 1 | 2;
                if (bcy) mask |= 4 | 8;
                if (W && !mask) continue;
                run_case(9, 8, bcx, bcy, W ? mask : 0, W, 0, 1);
                ++cases;
            }
    /* a PML on some open sides only; the appendix terms; two threads; a 1 x 1 periodic grid */
    run_case(10, 9, 2, 1, 1 | 8, 3, 0, 2);
    run_case(8, 8, 2, 2, 15, 5, 7, 2);
    run_case(8, 7, 3, 2, 2, 4, 5, 1);
    run_case(1, 1, 0, 0, 0, 0, 0, 1);
    cases += 4;

    /* documented error paths */
    EXPECT(orc_create(0, 5, 0.8, 1, 0, 0, 1) == NULL, "zero size must fail");
    EXPECT(orc_create(5, 5, 0.5, 1, 0, 0, 1) == NULL, "tau 0.5 must fail");
    orc_run *r = orc_create(5, 5, 0.8, 1, 0, 0, 1);
    double F[4 * 25];
    fields(5, 5, F, F + 25, F + 50, F + 75);
    EXPECT(orc_set_bc(r, 1, 7) != 0, "unknown bc must fail");
    EXPECT(orc_set_pml(r, 15, -1, 0.1) != 0, "negative W must fail");
    EXPECT(orc_set_nrbc_pml_terms(r, 8) != 0, "unknown term flag must fail");
    EXPECT(orc_set_bc(r, 1, 1) == 0, "set one side");
    EXPECT(orc_init(r, F, F + 25, F + 50, F + 75) != 0, "periodic on one side only must fail");
    EXPECT(orc_set_bc(r, 2, 1) == 0, "set the other side");
    EXPECT(orc_init(r, F, F + 25, F + 50, F + 75) != 0, "open axis below 7 nodes must fail");
    EXPECT(orc_step(r, 1, 1) != 0, "step before init must fail");
    orc_destroy(r);
    orc_destroy(NULL);

    printf("oracle q=%d: %d configurations, %d failures\n", ORC_Q, cases, failures);
    return failures ? 1 : 0;
}
