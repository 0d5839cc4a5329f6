/* Driver for the sanitizer build of the oracle (test infrastructure, CPU only).
 *
 * Linked with oracle/oracle.c under -fsanitize=address,undefined; calls every entry point of the
 * oracle on a small lattice with ragged extents and on a lattice of extent 2 (the smallest the
 * layouts allow), so that any out-of-bounds access, use after free or undefined arithmetic in the
 * oracle aborts the run.  Prints "sanitize ok" and returns 0 when everything ran. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

long orc_site_index(const int L[4], const int c[4]);
void orc_site_coords(const int L[4], long i, int c[4]);
void orc_gamma(int mu, double *out);
void orc_hop_w(const int L[4], int t_bc, const double *U, const double *psi, double *out, int out_parity,
               const double *w);
void orc_hop(const int L[4], int t_bc, const double *U, const double *psi, double *out, int out_parity);
double orc_clover_build(const int L[4], const double *U, double *clover);
double orc_clover_build_w(const int L[4], const double *U, double *clover, double wt, double ws);
void orc_packed_apply(const int L[4], const double *packed, const double *psi, double *out);
void orc_clover_apply(const int L[4], const double *clover, const double *psi, double *out, double kappa,
                      double csw);
long orc_clover_invert(const int L[4], const double *clover, double kappa, double csw, double *clover_inv);
void orc_dirac_w(const int L[4], int t_bc, const double *U, const double *clover, const double *psi, double *out,
                 double kappa, double csw, const double *w);
void orc_dirac(const int L[4], int t_bc, const double *U, const double *clover, const double *psi, double *out,
               double kappa, double csw);
int orc_bicgstab(const int L[4], int t_bc, const double *U, const double *clover, double kappa, double csw,
                 const double *b, double *x, double tol, int maxiter, double *res_hist, double *out);

static unsigned long long rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}

/* links close to the identity: 1 + small noise, then rows 0 and 1 orthonormalised and row 2 their
   conjugate cross product, so every link is in SU(3) */
static void make_links(long nlinks, double complex *U)
{
    for (long l = 0; l < nlinks; l++) {
        double complex *u = U + 9 * l;
        for (int e = 0; e < 9; e++) u[e] = (e % 4 == 0 ? 1.0 : 0.0) + 0.2 * (urand() + I * urand());
        double n0 = 0;
        for (int c = 0; c < 3; c++) n0 += creal(u[c] * conj(u[c]));
        for (int c = 0; c < 3; c++) u[c] /= sqrt(n0);
        double complex d = 0;
        for (int c = 0; c < 3; c++) d += conj(u[c]) * u[3 + c];
        for (int c = 0; c < 3; c++) u[3 + c] -= d * u[c];
        double n1 = 0;
        for (int c = 0; c < 3; c++) n1 += creal(u[3 + c] * conj(u[3 + c]));
        for (int c = 0; c < 3; c++) u[3 + c] /= sqrt(n1);
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

static int run(const int L[4])
{
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    double complex *U = malloc(sizeof(double complex) * 36 * V);
    double complex *psi = malloc(sizeof(double complex) * 12 * V), *out = malloc(sizeof(double complex) * 12 * V);
    double complex *x = calloc(12 * V, sizeof(double complex));
    double *clov = malloc(sizeof(double) * 72 * V), *inv = malloc(sizeof(double) * 72 * V);
    double *hist = malloc(sizeof(double) * 201), res[3], g[32];
    const double w[4] = {0.9, 0.9, 0.9, 1.0};
    make_links(4 * V, U);
    for (long k = 0; k < 12 * V; k++) psi[k] = urand() + I * urand();
    int c[4];
    for (long i = 0; i < V; i++) {
        orc_site_coords(L, i, c);
        if (orc_site_index(L, c) != i) return 1;
    }
    for (int mu = 0; mu < 4; mu++) orc_gamma(mu, g);
    for (int par = -1; par < 2; par++) {
        orc_hop(L, 1, (double *)U, (double *)psi, (double *)out, par);
        orc_hop_w(L, -1, (double *)U, (double *)psi, (double *)out, par, w);
    }
    orc_clover_build(L, (double *)U, clov);
    orc_clover_build_w(L, (double *)U, clov, 0.9, 1.1);
    orc_clover_build(L, (double *)U, clov);
    orc_packed_apply(L, clov, (double *)psi, (double *)out);
    orc_clover_apply(L, clov, (double *)psi, (double *)out, 0.12, 1.0);
    if (orc_clover_invert(L, clov, 0.12, 1.0, inv) != 0) return 2;
    orc_dirac(L, 1, (double *)U, clov, (double *)psi, (double *)out, 0.12, 1.0);
    orc_dirac_w(L, -1, (double *)U, clov, (double *)psi, (double *)out, 0.12, 1.0, w);
    int st = orc_bicgstab(L, 1, (double *)U, clov, 0.11, 1.0, (double *)psi, (double *)x, 1e-10, 200, hist, res);
    if (st != 0 || !(res[1] <= 1e-10)) return 3;
    /* iteration cap reached: the status path that returns the best iterate */
    for (long k = 0; k < 12 * V; k++) x[k] = 0;
    orc_bicgstab(L, 1, (double *)U, clov, 0.11, 1.0, (double *)psi, (double *)x, 1e-14, 2, hist, res);
    free(U), free(psi), free(out), free(x), free(clov), free(inv), free(hist);
    return 0;
}

int main(void)
{
    const int a[4] = {6, 4, 2, 6}, b[4] = {2, 2, 2, 2}, d[4] = {4, 6, 4, 2};
    int e = run(a);
    if (!e) e = run(b);
    if (!e) e = run(d);
    if (e) {
        fprintf(stderr, "sanitize run failed: %d\n", e);
        return e;
    }
    printf("sanitize ok\n");
    return 0;
}
