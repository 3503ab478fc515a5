/* Memory-safety driver for the oracle (test infrastructure): builds small
 * hierarchies of every kind the oracle supports and runs each entry point
 * once, so that a build with -fsanitize=address,undefined reports any
 * out-of-bounds access, leak or undefined behaviour.  Exit status 0 = clean. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int or_create3(int n, int levels, int degree, double lo, double hi, int rule, int coarse_solver,
               double coarse_rtol, int coarse_max_it, int galerkin, const double *kx, const double *ky,
               const double *kz, void **out);
void or_destroy(void *hp);
int or_pcg2(void *hp, const double *f, double *x, double rtol, int max_it, int flexible, int *its,
            double *relres, double *relres_true, long *coarse_its);
int or_adjoint_gradient(void *hp, const double *phi, const double *dl_dphi, double *gx, double *gy,
                        double *gz, double *lambda, double rtol, int max_it, int *its);
int or_vcycle(void *hp, const double *r, double *z);
int or_smooth(void *hp, int l, const double *b, double *x, int x0_zero);
int or_level_n(void *hp, int l);
int or_get_a27(void *hp, int l, double *out);
int or_level_interval(void *hp, int l, double *lo, double *hi);
int or_set_mixed(void *hp);
int or_last_restarts(void *hp);
void or_round_bf16_raw(size_t count, const double *in, double *out);

static double urand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static int run(int n, int levels, int rule, int coarse_solver, int galerkin, int flexible, int mixed)
{
    size_t nv = (size_t)n * n * n, nx = (size_t)n * n * (n - 1);
    double *kx = malloc(nx * sizeof(double)), *ky = malloc(nx * sizeof(double)),
           *kz = malloc(nx * sizeof(double));
    double *f = calloc(nv, sizeof(double)), *x = calloc(nv, sizeof(double)), *z = calloc(nv, sizeof(double));
    double *gx = calloc(nx, sizeof(double)), *gy = calloc(nx, sizeof(double)), *gz = calloc(nx, sizeof(double));
    double *lam = calloc(nv, sizeof(double));
    unsigned s = 12345u + (unsigned)n;
    for (size_t i = 0; i < nx; i++) {
        kx[i] = exp(2.0 * urand(&s) - 1.0);
        ky[i] = exp(2.0 * urand(&s) - 1.0);
        kz[i] = exp(2.0 * urand(&s) - 1.0);
    }
    for (int k = 1; k < n - 1; k++)
        for (int j = 1; j < n - 1; j++)
            for (int i = 1; i < n - 1; i++)
                f[((size_t)k * n + j) * n + i] = 2.0 * urand(&s) - 1.0;
    void *H = NULL;
    int st = or_create3(n, levels, 2, 0.25, 2.0, rule, coarse_solver, 1e-4, 500, galerkin, kx, ky, kz, &H);
    if (st != 0) {
        fprintf(stderr, "create failed %d (n=%d levels=%d)\n", st, n, levels);
        return 1;
    }
    if (mixed && or_set_mixed(H) != 0) {
        fprintf(stderr, "mixed mode refused (n=%d levels=%d)\n", n, levels);
        or_destroy(H);
        return 1;
    }
    int its = 0;
    double rr, rt, lo, hi;
    long cits = 0;
    st = or_pcg2(H, f, x, 1e-8, 300, flexible, &its, &rr, &rt, &cits);
    or_vcycle(H, f, z);
    for (int l = 0; l < levels; l++) {
        or_level_interval(H, l, &lo, &hi);
        if (l + 1 < levels) {
            int nl = or_level_n(H, l);
            double *b = calloc((size_t)nl * nl * nl, sizeof(double)), *y = calloc((size_t)nl * nl * nl, sizeof(double));
            or_smooth(H, l, b, y, 1);
            if (galerkin && l >= galerkin) {
                double *a = malloc((size_t)nl * nl * nl * 27 * sizeof(double));
                or_get_a27(H, l, a);
                free(a);
            }
            free(b);
            free(y);
        }
    }
    int its2 = 0;
    if (!coarse_solver)
        or_adjoint_gradient(H, x, x, gx, gy, gz, lam, 1e-8, 300, &its2);
    printf("n=%d levels=%d rule=%d coarse=%d galerkin=%d mixed=%d: status %d, %d its, %d restarts, true %.2e\n",
           n, levels, rule, coarse_solver, galerkin, mixed, st, its, or_last_restarts(H), rt);
    or_round_bf16_raw(nx, kx, gx);
    or_destroy(H);
    free(kx);
    free(ky);
    free(kz);
    free(f);
    free(x);
    free(z);
    free(gx);
    free(gy);
    free(gz);
    free(lam);
    return st != 0 || !(rt <= 1e-8);
}

int main(void)
{
    int bad = 0;
    for (int mixed = 0; mixed <= 1; mixed++) {
        bad |= run(3, 1, 0, 0, 0, 0, mixed);
        bad |= run(9, 3, 1, 0, 0, 0, mixed);
        bad |= run(17, 4, 0, 0, 1, 0, mixed);
        bad |= run(17, 4, 0, 0, 2, 0, mixed);
        bad |= run(17, 2, 0, 1, 0, 1, mixed);
        bad |= run(33, 5, 0, 0, 0, 0, mixed);
    }
    return bad;
}
