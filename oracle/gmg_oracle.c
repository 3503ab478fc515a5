/*
 * gmg_oracle.c -- plain FP64 CPU oracle for the multigrid-preconditioned
 * conjugate-gradient solve of the variable-coefficient diffusion problem
 *
 *        -div(k grad phi) = f                       (Eq. 2 of the paper)
 *
 * on a structured 3D vertex grid with zero Dirichlet boundary values.
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only so that the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark can check the GPU
 * library against something obviously correct.  The GPU library never links,
 * loads or calls it, and the two share no code, headers or constants.
 *
 * Everything here is written for readability, not speed: one loop nest per
 * mathematical operation, no blocking, no fusion, no reordering beyond what
 * the definition states.  Loops over z-planes carry an OpenMP "parallel for"
 * only so that large grids finish in reasonable time; every reduction is
 * summed per plane and then plane by plane in order, so results do not depend
 * on the thread count.
 *
 * Storage (all arrays C order, x fastest):
 *   vertex vectors   u[k][j][i],        shape (N, N, N),   h = 1/(N-1)
 *   x-faces          kx[k][j][i],       shape (N, N, N-1), link (i,j,k)-(i+1,j,k)
 *   y-faces          ky[k][j][i],       shape (N, N-1, N), link (i,j,k)-(i,j+1,k)
 *   z-faces          kz[k][j][i],       shape (N-1, N, N), link (i,j,k)-(i,j,k+1)
 * Interior vertices have all three indices in 1..N-2; every vector value at a
 * boundary vertex is treated as zero.
 *
 * Parity status: every routine below is pinned by the CPU test suite against
 * closed forms, invariants or brute force (sine-mode eigenvalues, an exact
 * quadratic solution, dense assembly, the Chebyshev polynomial, the adjoint
 * of restriction/prolongation, dense two-grid composition, finite
 * differences; for the reduced-precision mode: exact rational bfloat16
 * rounding, a dense composition from the rounded level matrices, and the
 * FP32 search direction read back through or_last_direction).  No routine is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LEVELS 16
#define OR_MAX_COARSE 4096 /* largest dense coarsest system the oracle factors */

/* ------------------------------------------------------------------------ */
/* index helpers                                                            */
/* ------------------------------------------------------------------------ */
static size_t vid(int n, int i, int j, int k) { return ((size_t)k * n + j) * n + i; }
static size_t xid(int n, int i, int j, int k) { return ((size_t)k * n + j) * (n - 1) + i; }
static size_t yid(int n, int i, int j, int k) { return ((size_t)k * (n - 1) + j) * n + i; }
static size_t zid(int n, int i, int j, int k) { return ((size_t)k * n + j) * n + i; }
static int interior(int n, int i, int j, int k)
{
    return i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2 && k >= 1 && k <= n - 2;
}
/* value of a vertex vector, zero on (and outside) the boundary */
static double val(int n, const double *u, int i, int j, int k)
{
    return interior(n, i, j, k) ? u[vid(n, i, j, k)] : 0.0;
}
static size_t nvert(int n) { return (size_t)n * n * n; }

/* ------------------------------------------------------------------------ */
/* Rounding to the storage formats of the reduced-precision mode (an        */
/* addition to the paper's method).  Both round to nearest, ties to even,   */
/* straight from the FP64 value:                                            */
/*   FP32      24 significant bits (the C conversion double -> float);      */
/*   bfloat16   8 significant bits, the exponent range of FP32.             */
/* or_round_bf16 covers finite values whose magnitude lies in the normal    */
/* range of bfloat16, [2^-126, 2^128) after rounding; or_bf16_ok tells      */
/* whether a value does.                                                    */
/* ------------------------------------------------------------------------ */
double or_round_f32(double v) { return (double)(float)v; }

double or_round_bf16(double v)
{
    if (v == 0.0 || !isfinite(v))
        return v;
    int e;
    double m = frexp(v, &e); /* v = m 2^e with 1/2 <= |m| < 1 */
    /* m 2^8 has 8 bits before the binary point; nearbyint rounds the rest
     * away in the default mode, to nearest with ties to even */
    return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

int or_bf16_ok(double v)
{
    double r = or_round_bf16(fabs(v));
    return isfinite(v) && r >= ldexp(1.0, -126) && r < ldexp(1.0, 128);
}

void or_round_bf16_raw(size_t count, const double *in, double *out)
{
    for (size_t i = 0; i < count; i++)
        out[i] = or_round_bf16(in[i]);
}

/* ------------------------------------------------------------------------ */
/* Operator (Eq. 2, 7-point finite differences as in Sec. 4.1, Disc. A):    */
/*   (A u)_p = h^-2 sum_{faces f of p} k_f (u_p - u_q(f))                   */
/* ------------------------------------------------------------------------ */
void or_apply_raw(int n, const double *kx, const double *ky, const double *kz,
                  const double *u, double *out)
{
    double s = (double)(n - 1) * (double)(n - 1); /* h^-2 */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (!interior(n, i, j, k)) {
                    out[vid(n, i, j, k)] = 0.0;
                    continue;
                }
                double up = u[vid(n, i, j, k)];
                double acc = 0.0;
                acc += kx[xid(n, i - 1, j, k)] * (up - val(n, u, i - 1, j, k));
                acc += kx[xid(n, i, j, k)] * (up - val(n, u, i + 1, j, k));
                acc += ky[yid(n, i, j - 1, k)] * (up - val(n, u, i, j - 1, k));
                acc += ky[yid(n, i, j, k)] * (up - val(n, u, i, j + 1, k));
                acc += kz[zid(n, i, j, k - 1)] * (up - val(n, u, i, j, k - 1));
                acc += kz[zid(n, i, j, k)] * (up - val(n, u, i, j, k + 1));
                out[vid(n, i, j, k)] = s * acc;
            }
}

/* Diagonal of A: d_p = h^-2 * (sum of the six face coefficients of p). */
void or_diag_raw(int n, const double *kx, const double *ky, const double *kz, double *d)
{
    double s = (double)(n - 1) * (double)(n - 1);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (!interior(n, i, j, k)) {
                    d[vid(n, i, j, k)] = 0.0;
                    continue;
                }
                double acc = kx[xid(n, i - 1, j, k)] + kx[xid(n, i, j, k)] + ky[yid(n, i, j - 1, k)] +
                             ky[yid(n, i, j, k)] + kz[zid(n, i, j, k - 1)] + kz[zid(n, i, j, k)];
                d[vid(n, i, j, k)] = s * acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Coarse face coefficients for the re-discretized coarse operators         */
/* (Sec. 2.1.1 and Sec. 4.3 use re-discretized coarse operators; the paper  */
/* gives no averaging rule).  A coarse x-link spans two fine x-links in     */
/* series along the line y=2J, z=2K, and the lines beside it at y=2J+a,     */
/* z=2K+b (a,b in -1..1) are averaged with weights w_a w_b,                 */
/* w = (1/4, 1/2, 1/4).  Along the link the two fine values p, q combine by */
/*   rule 0 (arithmetic): (p + q)/2                                          */
/*   rule 1 (harmonic):   2pq/(p + q)                                        */
/* Only coarse links with at least one interior end point are set; the      */
/* others are 0.                                                            */
/* ------------------------------------------------------------------------ */
static double along(int rule, double p, double q)
{
    if (rule == 1)
        return (p + q) > 0.0 ? 2.0 * p * q / (p + q) : 0.0;
    return 0.5 * (p + q);
}
static const double W3[3] = {0.25, 0.5, 0.25};

void or_coarsen_k_raw(int n, const double *kx, const double *ky, const double *kz,
                      int nc, double *kxc, double *kyc, double *kzc, int rule)
{
    memset(kxc, 0, sizeof(double) * (size_t)nc * nc * (nc - 1));
    memset(kyc, 0, sizeof(double) * (size_t)nc * (nc - 1) * nc);
    memset(kzc, 0, sizeof(double) * (size_t)(nc - 1) * nc * nc);
    /* x-links: I in 0..nc-2, J and K interior */
    for (int K = 1; K <= nc - 2; K++)
        for (int J = 1; J <= nc - 2; J++)
            for (int I = 0; I <= nc - 2; I++) {
                double acc = 0.0;
                for (int b = -1; b <= 1; b++)
                    for (int a = -1; a <= 1; a++) {
                        double p = kx[xid(n, 2 * I, 2 * J + a, 2 * K + b)];
                        double q = kx[xid(n, 2 * I + 1, 2 * J + a, 2 * K + b)];
                        acc += W3[a + 1] * W3[b + 1] * along(rule, p, q);
                    }
                kxc[xid(nc, I, J, K)] = acc;
            }
    /* y-links: J in 0..nc-2, I and K interior */
    for (int K = 1; K <= nc - 2; K++)
        for (int J = 0; J <= nc - 2; J++)
            for (int I = 1; I <= nc - 2; I++) {
                double acc = 0.0;
                for (int b = -1; b <= 1; b++)
                    for (int a = -1; a <= 1; a++) {
                        double p = ky[yid(n, 2 * I + a, 2 * J, 2 * K + b)];
                        double q = ky[yid(n, 2 * I + a, 2 * J + 1, 2 * K + b)];
                        acc += W3[a + 1] * W3[b + 1] * along(rule, p, q);
                    }
                kyc[yid(nc, I, J, K)] = acc;
            }
    /* z-links: K in 0..nc-2, I and J interior */
    for (int K = 0; K <= nc - 2; K++)
        for (int J = 1; J <= nc - 2; J++)
            for (int I = 1; I <= nc - 2; I++) {
                double acc = 0.0;
                for (int b = -1; b <= 1; b++)
                    for (int a = -1; a <= 1; a++) {
                        double p = kz[zid(n, 2 * I + a, 2 * J + b, 2 * K)];
                        double q = kz[zid(n, 2 * I + a, 2 * J + b, 2 * K + 1)];
                        acc += W3[a + 1] * W3[b + 1] * along(rule, p, q);
                    }
                kzc[zid(nc, I, J, K)] = acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Restriction (Alg. 1, "restrict residual"): full weighting, the tensor    */
/* product of (1/4, 1/2, 1/4) around fine vertex 2I.  Coarse boundary = 0.  */
/* ------------------------------------------------------------------------ */
void or_restrict_raw(int n, const double *r, int nc, double *rc)
{
#pragma omp parallel for schedule(static)
    for (int K = 0; K < nc; K++)
        for (int J = 0; J < nc; J++)
            for (int I = 0; I < nc; I++) {
                if (!interior(nc, I, J, K)) {
                    rc[vid(nc, I, J, K)] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int c = -1; c <= 1; c++)
                    for (int b = -1; b <= 1; b++)
                        for (int a = -1; a <= 1; a++)
                            acc += W3[a + 1] * W3[b + 1] * W3[c + 1] *
                                   val(n, r, 2 * I + a, 2 * J + b, 2 * K + c);
                rc[vid(nc, I, J, K)] = acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Prolongation and correction (Alg. 1, "prolongate error"): trilinear      */
/* interpolation, x_fine += P e.  In 1D an even fine index 2I takes e_I; an */
/* odd one 2I+1 takes (e_I + e_{I+1})/2; 3D is the tensor product.          */
/* ------------------------------------------------------------------------ */
static int interp_1d(int i, int *idx, double *w)
{
    if ((i & 1) == 0) {
        idx[0] = i / 2;
        w[0] = 1.0;
        return 1;
    }
    idx[0] = (i - 1) / 2;
    w[0] = 0.5;
    idx[1] = (i + 1) / 2;
    w[1] = 0.5;
    return 2;
}

void or_prolong_add_raw(int nc, const double *e, int n, double *x)
{
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++) {
                int ii[2], jj[2], kk[2];
                double wi[2], wj[2], wk[2];
                int ni = interp_1d(i, ii, wi), nj = interp_1d(j, jj, wj), nk = interp_1d(k, kk, wk);
                double acc = 0.0;
                for (int c = 0; c < nk; c++)
                    for (int b = 0; b < nj; b++)
                        for (int a = 0; a < ni; a++)
                            acc += wi[a] * wj[b] * wk[c] * val(nc, e, ii[a], jj[b], kk[c]);
                x[vid(n, i, j, k)] += acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Galerkin coarse operators (the other coarse-operator construction of     */
/* Sec. 3.3.2 and Sec. 4.2): A_c = R A P with trilinear P and R = P^T / 8.  */
/* With a 7-point (or 27-point) fine operator A_c couples each coarse       */
/* vertex to its 3x3x3 neighbourhood, so it is stored as 27 coefficients    */
/* per vertex: a27[p*27 + (dz+1)*9 + (dy+1)*3 + (dx+1)] multiplies          */
/* u[p + (dx,dy,dz)].  Rows and columns of boundary vertices are absent.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    const double *kx, *ky, *kz; /* 7-point link form (a27 == NULL) */
    const double *a27;          /* or a 27-point stencil per vertex */
} or_op;

static int d27(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }

void or_apply27_raw(int n, const double *a27, const double *u, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (!interior(n, i, j, k)) {
                    out[vid(n, i, j, k)] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++)
                            acc += a27[vid(n, i, j, k) * 27 + d27(dx, dy, dz)] *
                                   val(n, u, i + dx, j + dy, k + dz);
                out[vid(n, i, j, k)] = acc;
            }
}

static void op_apply(const or_op *A, const double *u, double *out)
{
    if (A->a27)
        or_apply27_raw(A->n, A->a27, u, out);
    else
        or_apply_raw(A->n, A->kx, A->ky, A->kz, u, out);
}

static void op_diag(const or_op *A, double *d)
{
    if (!A->a27) {
        or_diag_raw(A->n, A->kx, A->ky, A->kz, d);
        return;
    }
    int n = A->n;
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++)
                d[vid(n, i, j, k)] = interior(n, i, j, k) ? A->a27[vid(n, i, j, k) * 27 + d27(0, 0, 0)] : 0.0;
}

/* entry A[p][q] of a fine operator for interior p and any q (0 unless q is an
 * interior stencil neighbour of p) */
static double op_entry(const or_op *A, int pi, int pj, int pk, int qi, int qj, int qk)
{
    int n = A->n;
    int dx = qi - pi, dy = qj - pj, dz = qk - pk;
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1 || !interior(n, qi, qj, qk))
        return 0.0;
    if (A->a27)
        return A->a27[vid(n, pi, pj, pk) * 27 + d27(dx, dy, dz)];
    double s = (double)(n - 1) * (double)(n - 1);
    int nz = (dx != 0) + (dy != 0) + (dz != 0);
    if (nz == 0)
        return s * (A->kx[xid(n, pi - 1, pj, pk)] + A->kx[xid(n, pi, pj, pk)] + A->ky[yid(n, pi, pj - 1, pk)] +
                    A->ky[yid(n, pi, pj, pk)] + A->kz[zid(n, pi, pj, pk - 1)] + A->kz[zid(n, pi, pj, pk)]);
    if (nz > 1)
        return 0.0;
    if (dx)
        return -s * A->kx[xid(n, dx < 0 ? pi - 1 : pi, pj, pk)];
    if (dy)
        return -s * A->ky[yid(n, pi, dy < 0 ? pj - 1 : pj, pk)];
    return -s * A->kz[zid(n, pi, pj, dz < 0 ? pk - 1 : pk)];
}

/* 1D trilinear weight of coarse index J at fine index q */
static double pw(int q, int J)
{
    int d = q - 2 * J;
    return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0;
}

/* a27c = R A P on the coarse grid of A's grid, from the definitions of R, A, P:
 * (R A P)[I][J] = sum_p sum_q R[I][p] A[p][q] P[q][J] with R[I][p] = P[p][I]/8. */
void or_galerkin_op(const or_op *A, int nc, double *a27c)
{
    memset(a27c, 0, sizeof(double) * nvert(nc) * 27);
#pragma omp parallel for schedule(dynamic)
    for (int K = 1; K <= nc - 2; K++)
        for (int J = 1; J <= nc - 2; J++)
            for (int I = 1; I <= nc - 2; I++)
                for (int pk = 2 * K - 1; pk <= 2 * K + 1; pk++)
                    for (int pj = 2 * J - 1; pj <= 2 * J + 1; pj++)
                        for (int pi = 2 * I - 1; pi <= 2 * I + 1; pi++) {
                            double r = pw(pi, I) * pw(pj, J) * pw(pk, K) / 8.0;
                            for (int qk = pk - 1; qk <= pk + 1; qk++)
                                for (int qj = pj - 1; qj <= pj + 1; qj++)
                                    for (int qi = pi - 1; qi <= pi + 1; qi++) {
                                        double a = op_entry(A, pi, pj, pk, qi, qj, qk);
                                        if (a == 0.0)
                                            continue;
                                        for (int Ck = qk / 2 - 1; Ck <= qk / 2 + 1; Ck++)
                                            for (int Cj = qj / 2 - 1; Cj <= qj / 2 + 1; Cj++)
                                                for (int Ci = qi / 2 - 1; Ci <= qi / 2 + 1; Ci++) {
                                                    if (!interior(nc, Ci, Cj, Ck))
                                                        continue;
                                                    double w = pw(qi, Ci) * pw(qj, Cj) * pw(qk, Ck);
                                                    if (w == 0.0)
                                                        continue;
                                                    a27c[vid(nc, I, J, K) * 27 + d27(Ci - I, Cj - J, Ck - K)] +=
                                                        r * a * w;
                                                }
                                    }
                        }
}

void or_galerkin_raw(int n, const double *kx, const double *ky, const double *kz, const double *a27, int nc,
                     double *a27c)
{
    or_op A = {n, kx, ky, kz, a27};
    or_galerkin_op(&A, nc, a27c);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev smoother preconditioned by Jacobi (the smoother of Sec. 4.3 and */
/* of the PETSc option examples in Sec. 3.3).  Chebyshev acceleration on    */
/* D^-1 A over the interval [lo, hi], following the published three-term    */
/* recurrence (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,  */
/* Alg. 12.1):                                                              */
/*   theta=(hi+lo)/2, delta=(hi-lo)/2, sigma=theta/delta                     */
/*   r0 = b - A x0, d0 = D^-1 r0 / theta, rho0 = 1/sigma                     */
/*   x_{j+1} = x_j + d_j;  r_{j+1} = r_j - A d_j;                            */
/*   rho_{j+1} = 1/(2 sigma - rho_j);                                        */
/*   d_{j+1} = rho_{j+1} rho_j d_j + (2 rho_{j+1}/delta) D^-1 r_{j+1}        */
/* degree steps in total; x0 = 0 when x0_zero is set (r0 = b, no matvec).   */
/* work must hold 4 vertex vectors.                                         */
/* ------------------------------------------------------------------------ */
static void cheb_op(const or_op *A, int degree, double lo, double hi, const double *b, double *x, int x0_zero,
                    double *work)
{
    int n = A->n;
    size_t nv = nvert(n);
    double *r = work, *d = work + nv, *t = work + 2 * nv, *dg = work + 3 * nv;
    double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    op_diag(A, dg);
    if (x0_zero) {
        memset(x, 0, sizeof(double) * nv);
        for (size_t p = 0; p < nv; p++)
            r[p] = b[p];
    } else {
        op_apply(A, x, t);
        for (size_t p = 0; p < nv; p++)
            r[p] = b[p] - t[p];
    }
    for (size_t p = 0; p < nv; p++)
        d[p] = dg[p] > 0.0 ? r[p] / dg[p] / theta : 0.0;
    double rho = 1.0 / sigma;
    for (int j = 0; j < degree; j++) {
        for (size_t p = 0; p < nv; p++)
            x[p] += d[p];
        if (j + 1 < degree) {
            op_apply(A, d, t);
            for (size_t p = 0; p < nv; p++)
                r[p] -= t[p];
            double rho_new = 1.0 / (2.0 * sigma - rho);
            for (size_t p = 0; p < nv; p++)
                d[p] = rho_new * rho * d[p] + (2.0 * rho_new / delta) * (dg[p] > 0.0 ? r[p] / dg[p] : 0.0);
            rho = rho_new;
        }
    }
    /* boundary entries stay zero */
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++)
                if (!interior(n, i, j, k))
                    x[vid(n, i, j, k)] = 0.0;
}

void or_cheb_raw(int n, const double *kx, const double *ky, const double *kz, int degree, double lo, double hi,
                 const double *b, double *x, int x0_zero, double *work)
{
    or_op A = {n, kx, ky, kz, NULL};
    cheb_op(&A, degree, lo, hi, b, x, x0_zero, work);
}

/* ------------------------------------------------------------------------ */
/* Dense assembly and Cholesky factorization of the coarsest operator.      */
/* The coarsest level is solved exactly (Sec. 1 and Sec. 3.3.1 use LU; A   */
/* is symmetric positive definite here, so Cholesky L L^T).                 */
/* Unknown numbering: interior vertices in C order, x fastest.              */
/* ------------------------------------------------------------------------ */
static int unk(int n, int i, int j, int k) { return ((k - 1) * (n - 2) + (j - 1)) * (n - 2) + (i - 1); }

void or_assemble_dense_raw(int n, const double *kx, const double *ky, const double *kz, double *A)
{
    int m = (n - 2) * (n - 2) * (n - 2);
    double s = (double)(n - 1) * (double)(n - 1);
    memset(A, 0, sizeof(double) * (size_t)m * m);
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++) {
                int p = unk(n, i, j, k);
                /* the six links of p: coefficient and neighbour */
                double kf[6] = {kx[xid(n, i - 1, j, k)], kx[xid(n, i, j, k)], ky[yid(n, i, j - 1, k)],
                                ky[yid(n, i, j, k)],     kz[zid(n, i, j, k - 1)], kz[zid(n, i, j, k)]};
                int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                                {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                for (int f = 0; f < 6; f++) {
                    A[(size_t)p * m + p] += s * kf[f];
                    if (interior(n, nb[f][0], nb[f][1], nb[f][2]))
                        A[(size_t)p * m + unk(n, nb[f][0], nb[f][1], nb[f][2])] -= s * kf[f];
                }
            }
}

static void assemble_dense_op(const or_op *A, double *M)
{
    if (!A->a27) {
        or_assemble_dense_raw(A->n, A->kx, A->ky, A->kz, M);
        return;
    }
    int n = A->n;
    int m = (n - 2) * (n - 2) * (n - 2);
    memset(M, 0, sizeof(double) * (size_t)m * m);
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++)
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++)
                            if (interior(n, i + dx, j + dy, k + dz))
                                M[(size_t)unk(n, i, j, k) * m + unk(n, i + dx, j + dy, k + dz)] +=
                                    A->a27[vid(n, i, j, k) * 27 + d27(dx, dy, dz)];
}

/* In-place Cholesky: on return the lower triangle of A holds L.  Returns 0, */
/* or -1 when a pivot is not positive (A not SPD).                          */
int or_cholesky_raw(int m, double *A)
{
    for (int j = 0; j < m; j++) {
        double dsum = A[(size_t)j * m + j];
        for (int c = 0; c < j; c++)
            dsum -= A[(size_t)j * m + c] * A[(size_t)j * m + c];
        if (!(dsum > 0.0))
            return -1;
        double ljj = sqrt(dsum);
        A[(size_t)j * m + j] = ljj;
        for (int r = j + 1; r < m; r++) {
            double s = A[(size_t)r * m + j];
            for (int c = 0; c < j; c++)
                s -= A[(size_t)r * m + c] * A[(size_t)j * m + c];
            A[(size_t)r * m + j] = s / ljj;
        }
    }
    return 0;
}

/* Solve L L^T y = rhs with the factor from or_cholesky_raw (in place on y). */
void or_chol_solve_raw(int m, const double *L, double *y)
{
    for (int r = 0; r < m; r++) { /* forward: L w = rhs */
        double s = y[r];
        for (int c = 0; c < r; c++)
            s -= L[(size_t)r * m + c] * y[c];
        y[r] = s / L[(size_t)r * m + r];
    }
    for (int r = m - 1; r >= 0; r--) { /* backward: L^T y = w */
        double s = y[r];
        for (int c = r + 1; c < m; c++)
            s -= L[(size_t)c * m + r] * y[c];
        y[r] = s / L[(size_t)r * m + r];
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev interval of a Galerkin level.  The fixed bound 2 on the        */
/* spectrum of D^-1 A holds for the 7-point M-matrix, not for R A P, whose  */
/* rows mix signs.  On a Galerkin level the interval's upper end is 1.1     */
/* times an estimate of lambda_max(D^-1 A): the largest eigenvalue of the   */
/* tridiagonal matrix of OR_LANCZOS_STEPS Lanczos steps in the D inner      */
/* product (D^-1 A is self-adjoint there), from the fixed start vector      */
/* u0 = 1 + ((7i + 11j + 13k) mod 5) / 4 at interior vertices.  The lower   */
/* end keeps the ratio lo/hi of the default interval.                      */
/* ------------------------------------------------------------------------ */
#define OR_LANCZOS_STEPS 20
#define OR_LANCZOS_SAFETY 1.1

/* largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..m-1]
 * and off-diagonal b[0..m-2], by bisection on the Sturm count */
static double tridiag_max_eig(int m, const double *a, const double *b)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; i++) {
        double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        if (a[i] - r < lo)
            lo = a[i] - r;
        if (a[i] + r > hi)
            hi = a[i] + r;
    }
    for (int it = 0; it < 2000; it++) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi))
            break;
        int below = 0; /* eigenvalues below mid = negative pivots of T - mid I */
        double q = 1.0;
        for (int i = 0; i < m; i++) {
            q = a[i] - mid - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
            if (q == 0.0)
                q = -1e-300;
            if (q < 0.0)
                below++;
        }
        if (below == m)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

static double lanczos_max(const or_op *A, int steps, double *work)
{
    int n = A->n;
    size_t nv = nvert(n);
    double *v = work, *vp = work + nv, *w = work + 2 * nv, *dg = work + 3 * nv;
    double al[64] = {0}, be[64] = {0};
    if (steps > 64)
        steps = 64;
    op_diag(A, dg);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++)
                v[vid(n, i, j, k)] = interior(n, i, j, k) ? 1.0 + 0.25 * ((7 * i + 11 * j + 13 * k) % 5) : 0.0;
    double s = 0.0;
    for (size_t p = 0; p < nv; p++)
        s += v[p] * dg[p] * v[p];
    s = sqrt(s);
    for (size_t p = 0; p < nv; p++) {
        v[p] /= s;
        vp[p] = 0.0;
    }
    double beta = 0.0;
    int m = 0;
    for (int j = 0; j < steps; j++) {
        op_apply(A, v, w);
        double alpha = 0.0;
        for (size_t p = 0; p < nv; p++)
            alpha += v[p] * w[p];
        for (size_t p = 0; p < nv; p++)
            w[p] = dg[p] > 0.0 ? w[p] / dg[p] - alpha * v[p] - beta * vp[p] : 0.0;
        double bn = 0.0;
        for (size_t p = 0; p < nv; p++)
            bn += w[p] * dg[p] * w[p];
        bn = sqrt(bn);
        al[m] = alpha;
        be[m] = bn;
        m++;
        if (!(bn > 1e-14 * fabs(alpha)))
            break; /* invariant subspace: T holds the exact eigenvalues */
        for (size_t p = 0; p < nv; p++) {
            vp[p] = v[p];
            v[p] = w[p] / bn;
        }
        beta = bn;
    }
    return tridiag_max_eig(m, al, be);
}

double or_lanczos_max_raw(int n, const double *kx, const double *ky, const double *kz, const double *a27,
                          int steps, double *work)
{
    or_op A = {n, kx, ky, kz, a27};
    return lanczos_max(&A, steps, work);
}

/* ------------------------------------------------------------------------ */
/* Hierarchy (Sec. 2.1.1: per level an operator, a smoother, R and P; an    */
/* exact solver on the coarsest level).  Coarsening factor 2 (Sec. 1):      */
/* N_{l+1} = (N_l - 1)/2 + 1, coarse vertex I sits on fine vertex 2I.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double *kx, *ky, *kz;
    double *a27;              /* Galerkin coarse operator (NULL: the 7-point link form) */
    double *vkx, *vky, *vkz;  /* reduced-precision mode: the links rounded to bfloat16 */
    double *va27;             /* reduced-precision mode: a27 rounded to FP32 */
    double lo, hi;            /* Chebyshev interval of D^-1 A on this level */
    double *x, *b, *r, *work; /* work: 4 vectors for the smoother */
} or_level;

/* the level's operator in FP64: used to build the hierarchy (Galerkin
 * products, Lanczos intervals, the coarsest factor) */
static or_op level_op(const or_level *L)
{
    or_op A = {L->n, L->kx, L->ky, L->kz, L->a27};
    return A;
}

/* the level's operator as the V-cycle applies it: the FP64 one, or its
 * rounded copy in the reduced-precision mode */
static or_op vcycle_op(const or_level *L)
{
    if (L->vkx) {
        or_op A = {L->n, L->vkx, L->vky, L->vkz, L->va27};
        return A;
    }
    return level_op(L);
}

typedef struct {
    int levels, degree, rule;
    double lo, hi;
    or_level lv[OR_MAX_LEVELS];
    int m;       /* unknowns on the coarsest level */
    double *chol; /* m x m, lower triangle = L (exact coarse solve only) */
    int coarse_solver;     /* 0: exact Cholesky; 1: truncated hierarchy, inexact coarse CG */
    int galerkin;          /* g > 0: levels l >= g take R A P, levels below g are re-discretized
                              (g = 1: Galerkin throughout, Sec. 3.3.2; g > 1: the hybrid
                              construction of Sec. 3.3.3); 0: re-discretized throughout */
    double coarse_rtol;    /* coarse CG relative residual target */
    int coarse_max_it;
    long coarse_its;       /* coarse CG iterations since the last reset */
    int mixed;             /* 1: reduced-precision preconditioner (or_set_mixed) */
    int restarts;          /* true-residual restarts of the last CG solve */
    double *last_p;        /* the search direction as the last CG solve left it (N^3), an
                              observable for the tests; NULL before the first solve */
} or_hier;

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_DIMS = 2, OR_ERR_COEFF = 3, OR_ERR_NOMEM = 4,
       OR_ERR_NOT_CONVERGED = 6, OR_ERR_BREAKDOWN = 7 };

void or_destroy(void *hp)
{
    or_hier *H = (or_hier *)hp;
    if (!H)
        return;
    for (int l = 0; l < H->levels; l++) {
        free(H->lv[l].kx);
        free(H->lv[l].ky);
        free(H->lv[l].kz);
        free(H->lv[l].a27);
        free(H->lv[l].vkx);
        free(H->lv[l].vky);
        free(H->lv[l].vkz);
        free(H->lv[l].va27);
        free(H->lv[l].x);
        free(H->lv[l].b);
        free(H->lv[l].r);
        free(H->lv[l].work);
    }
    free(H->chol);
    free(H->last_p);
    free(H);
}

int or_create3(int n, int levels, int degree, double lo, double hi, int rule, int coarse_solver,
               double coarse_rtol, int coarse_max_it, int galerkin, const double *kx, const double *ky,
               const double *kz, void **out);

int or_create2(int n, int levels, int degree, double lo, double hi, int rule, int coarse_solver,
               double coarse_rtol, int coarse_max_it, const double *kx, const double *ky, const double *kz,
               void **out)
{
    return or_create3(n, levels, degree, lo, hi, rule, coarse_solver, coarse_rtol, coarse_max_it, 0, kx, ky, kz,
                      out);
}

int or_create3(int n, int levels, int degree, double lo, double hi, int rule, int coarse_solver,
               double coarse_rtol, int coarse_max_it, int galerkin, const double *kx, const double *ky,
               const double *kz, void **out)
{
    *out = NULL;
    if (n < 3 || levels < 1 || levels > OR_MAX_LEVELS || degree < 1 || !(lo > 0.0) || !(hi > lo) ||
        rule < 0 || rule > 1 || coarse_solver < 0 || coarse_solver > 1 || galerkin < 0 ||
        (coarse_solver == 1 && (!(coarse_rtol > 0.0) || coarse_max_it < 1)))
        return OR_ERR_ARG;
    if ((n - 1) % (1 << (levels - 1)) != 0)
        return OR_ERR_DIMS;
    int ncoarse = (n - 1) / (1 << (levels - 1)) + 1;
    if (ncoarse < 3)
        return OR_ERR_DIMS;
    int m = (ncoarse - 2) * (ncoarse - 2) * (ncoarse - 2);
    if (coarse_solver == 0 && m > OR_MAX_COARSE)
        return OR_ERR_DIMS;
    /* coefficients must be positive and finite on every active link (a link
     * is active when one of its end points is interior; the values on links
     * between two boundary vertices are never read) */
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 0; i <= n - 2; i++) {
                double a = kx[xid(n, i, j, k)], b = ky[yid(n, j, i, k)], c = kz[zid(n, j, k, i)];
                if (!(a > 0.0) || !isfinite(a) || !(b > 0.0) || !isfinite(b) || !(c > 0.0) ||
                    !isfinite(c))
                    return OR_ERR_COEFF;
            }
    or_hier *H = (or_hier *)calloc(1, sizeof(or_hier));
    if (!H)
        return OR_ERR_NOMEM;
    H->levels = levels;
    H->degree = degree;
    H->rule = rule;
    H->coarse_solver = coarse_solver;
    H->galerkin = galerkin;
    H->coarse_rtol = coarse_rtol;
    H->coarse_max_it = coarse_max_it;
    H->lo = lo;
    H->hi = hi;
    int nl = n;
    for (int l = 0; l < levels; l++) {
        or_level *L = &H->lv[l];
        L->n = nl;
        size_t nv = nvert(nl), nfl = (size_t)nl * nl * (nl - 1);
        L->kx = (double *)malloc(sizeof(double) * nfl);
        L->ky = (double *)malloc(sizeof(double) * nfl);
        L->kz = (double *)malloc(sizeof(double) * nfl);
        L->x = (double *)calloc(nv, sizeof(double));
        L->b = (double *)calloc(nv, sizeof(double));
        L->r = (double *)calloc(nv, sizeof(double));
        L->work = (double *)calloc(4 * nv, sizeof(double));
        if (!L->kx || !L->ky || !L->kz || !L->x || !L->b || !L->r || !L->work) {
            H->levels = l + 1;
            or_destroy(H);
            return OR_ERR_NOMEM;
        }
        if (l == 0) {
            memcpy(L->kx, kx, sizeof(double) * nfl);
            memcpy(L->ky, ky, sizeof(double) * nfl);
            memcpy(L->kz, kz, sizeof(double) * nfl);
        } else {
            or_level *F = &H->lv[l - 1];
            or_coarsen_k_raw(F->n, F->kx, F->ky, F->kz, nl, L->kx, L->ky, L->kz, rule);
            if (H->galerkin && l >= H->galerkin) {
                L->a27 = (double *)calloc(nv * 27, sizeof(double));
                if (!L->a27) {
                    H->levels = l + 1;
                    or_destroy(H);
                    return OR_ERR_NOMEM;
                }
                or_op Fo = level_op(F);
                or_galerkin_op(&Fo, nl, L->a27);
            }
        }
        L->lo = lo;
        L->hi = hi;
        nl = (nl - 1) / 2 + 1;
    }
    /* Chebyshev intervals of the smoothed Galerkin levels (the coarsest level is
     * solved, not smoothed) */
    for (int l = 1; l + 1 < levels; l++) {
        or_level *L = &H->lv[l];
        if (!L->a27)
            continue;
        or_op Ao = level_op(L);
        L->hi = OR_LANCZOS_SAFETY * lanczos_max(&Ao, OR_LANCZOS_STEPS, L->work);
        L->lo = L->hi * (lo / hi);
    }
    or_level *C = &H->lv[levels - 1];
    H->m = m;
    if (coarse_solver == 1) { /* truncated hierarchy: no factorization */
        *out = H;
        return OR_OK;
    }
    H->chol = (double *)malloc(sizeof(double) * (size_t)m * m);
    if (!H->chol) {
        or_destroy(H);
        return OR_ERR_NOMEM;
    }
    {
        or_op Co = level_op(C);
        assemble_dense_op(&Co, H->chol);
    }
    if (or_cholesky_raw(m, H->chol) != 0) {
        or_destroy(H);
        return OR_ERR_COEFF;
    }
    *out = H;
    return OR_OK;
}

int or_create(int n, int levels, int degree, double lo, double hi, int rule, const double *kx,
              const double *ky, const double *kz, void **out)
{
    return or_create2(n, levels, degree, lo, hi, rule, 0, 0.0, 0, kx, ky, kz, out);
}

int or_level_n(void *hp, int l)
{
    or_hier *H = (or_hier *)hp;
    return (l >= 0 && l < H->levels) ? H->lv[l].n : -1;
}

int or_get_k(void *hp, int l, double *kx, double *ky, double *kz)
{
    or_hier *H = (or_hier *)hp;
    if (l < 0 || l >= H->levels)
        return OR_ERR_ARG;
    int n = H->lv[l].n;
    size_t nf = (size_t)n * n * (n - 1);
    memcpy(kx, H->lv[l].kx, sizeof(double) * nf);
    memcpy(ky, H->lv[l].ky, sizeof(double) * nf);
    memcpy(kz, H->lv[l].kz, sizeof(double) * nf);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision preconditioner (the MIXED mode; not in the paper).      */
/* After this call the hierarchy applies the exact-arithmetic value of the   */
/* preconditioner that the mixed mode uses:                                  */
/*  - every level's link coefficients, built in FP64 as above, rounded once  */
/*    to bfloat16; 27-point Galerkin coefficients rounded once to FP32; the  */
/*    Jacobi diagonal follows from the rounded coefficients;                */
/*  - Chebyshev intervals and the coarsest Cholesky factor stay those of     */
/*    the FP64 operators (the inexact coarse CG of a truncated hierarchy     */
/*    uses the rounded coefficients);                                        */
/*  - the V-cycle's input and output are rounded to FP32 (or_vcycle);       */
/*  - the outer CG stays FP64 (operator with the FP64 links, x, r, q, dot    */
/*    products), except that each new search direction p = z + beta p is    */
/*    rounded once to FP32, and that when the recursive residual passes but  */
/*    the FP64 true residual does not, CG restarts from r = b - A x (at most */
/*    20 times).                                                             */
/* The V-cycle arithmetic stays FP64 here: a GPU V-cycle computing in FP32   */
/* agrees with it to FP32 roundoff, not bit for bit.                         */
/* Returns OR_ERR_COEFF if a link of a smoothed or CG-solved level rounds    */
/* outside the normal bfloat16 range.                                        */
/* ------------------------------------------------------------------------ */
static void free_vcycle_copies(or_hier *H)
{
    for (int l = 0; l < H->levels; l++) {
        or_level *L = &H->lv[l];
        free(L->vkx);
        free(L->vky);
        free(L->vkz);
        free(L->va27);
        L->vkx = L->vky = L->vkz = L->va27 = NULL;
    }
}

static int make_vcycle_copies(or_hier *H);

int or_set_mixed(void *hp)
{
    or_hier *H = (or_hier *)hp;
    if (H->mixed)
        return OR_OK;
    int st = make_vcycle_copies(H);
    if (st != OR_OK) {
        free_vcycle_copies(H);
        return st;
    }
    H->mixed = 1;
    return OR_OK;
}

static int make_vcycle_copies(or_hier *H)
{
    for (int l = 0; l < H->levels; l++) {
        or_level *L = &H->lv[l];
        int n = L->n;
        size_t nfl = (size_t)n * n * (n - 1);
        L->vkx = (double *)calloc(nfl, sizeof(double));
        L->vky = (double *)calloc(nfl, sizeof(double));
        L->vkz = (double *)calloc(nfl, sizeof(double));
        if (!L->vkx || !L->vky || !L->vkz)
            return OR_ERR_NOMEM;
        for (size_t f = 0; f < nfl; f++) {
            L->vkx[f] = or_round_bf16(L->kx[f]);
            L->vky[f] = or_round_bf16(L->ky[f]);
            L->vkz[f] = or_round_bf16(L->kz[f]);
        }
        /* active links (one end point interior) must stay normal bfloat16
         * values; the coarsest level of an exact solve keeps FP64 */
        int used = l + 1 < H->levels || H->coarse_solver == 1;
        for (int k = 1; used && !L->a27 && k <= n - 2; k++)
            for (int j = 1; j <= n - 2; j++)
                for (int i = 0; i <= n - 2; i++)
                    if (!or_bf16_ok(L->kx[xid(n, i, j, k)]) || !or_bf16_ok(L->ky[yid(n, j, i, k)]) ||
                        !or_bf16_ok(L->kz[zid(n, j, k, i)]))
                        return OR_ERR_COEFF;
        if (L->a27) {
            size_t m = nvert(n) * 27;
            L->va27 = (double *)malloc(sizeof(double) * m);
            if (!L->va27)
                return OR_ERR_NOMEM;
            for (size_t q = 0; q < m; q++)
                L->va27[q] = or_round_f32(L->a27[q]);
        }
    }
    return OR_OK;
}

static double dot_int(int n, const double *a, const double *b);

/* Inexact coarsest solve of a truncated hierarchy (the truncation strategy of
 * Sec. 1 and Sec. 3.3.1: fewer levels, an iterative coarse solver to a
 * relative tolerance): CG preconditioned by Jacobi from x = 0, stopped when
 * ||r|| <= coarse_rtol ||b|| or after coarse_max_it iterations. */
static int coarse_cg(or_hier *H, const double *b, double *x)
{
    or_level *C = &H->lv[H->levels - 1];
    int n = C->n;
    size_t nv = nvert(n);
    double *r = C->work, *p = C->work + nv, *q = C->work + 2 * nv, *dg = C->work + 3 * nv;
    double *z = (double *)calloc(nv, sizeof(double));
    if (!z)
        return OR_ERR_NOMEM;
    or_op Ao = vcycle_op(C);
    op_diag(&Ao, dg);
    for (size_t i = 0; i < nv; i++) {
        x[i] = 0.0;
        r[i] = b[i];
        z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
        p[i] = z[i];
    }
    double bb = dot_int(n, b, b);
    double rho = dot_int(n, r, z);
    if (bb == 0.0) {
        free(z);
        return OR_OK;
    }
    for (int it = 0; it < H->coarse_max_it; it++) {
        op_apply(&Ao, p, q);
        double pq = dot_int(n, p, q);
        if (!(pq > 0.0))
            break;
        double alpha = rho / pq;
        for (size_t i = 0; i < nv; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        H->coarse_its++;
        if (dot_int(n, r, r) <= H->coarse_rtol * H->coarse_rtol * bb)
            break;
        for (size_t i = 0; i < nv; i++)
            z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
        double rho_new = dot_int(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (size_t i = 0; i < nv; i++)
            p[i] = z[i] + beta * p[i];
    }
    free(z);
    return OR_OK;
}

/* coarsest solve: x = A_c^-1 b (exact), or the inexact CG of a truncated hierarchy */
int or_coarse_solve(void *hp, const double *b, double *x)
{
    or_hier *H = (or_hier *)hp;
    if (H->coarse_solver == 1)
        return coarse_cg(H, b, x);
    int n = H->lv[H->levels - 1].n;
    double *y = (double *)malloc(sizeof(double) * (size_t)H->m);
    if (!y)
        return OR_ERR_NOMEM;
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++)
                y[unk(n, i, j, k)] = b[vid(n, i, j, k)];
    or_chol_solve_raw(H->m, H->chol, y);
    memset(x, 0, sizeof(double) * nvert(n));
    for (int k = 1; k <= n - 2; k++)
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++)
                x[vid(n, i, j, k)] = y[unk(n, i, j, k)];
    free(y);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* V-cycle: Alg. 1 (two-level multigrid) applied recursively, one cycle,   */
/* zero initial guess, pre- and post-smoothing by one Chebyshev-Jacobi      */
/* polynomial each, exact solve on the coarsest level.                      */
/*   V(l, b): l = last -> A_l^-1 b.  Otherwise                               */
/*     x = Cheb(b, x0 = 0); r = b - A_l x; e = V(l+1, R r);                  */
/*     x += P e; x = Cheb(b, x0 = x).                                        */
/* The result is written to H->lv[l].x; b is H->lv[l].b.                    */
/* ------------------------------------------------------------------------ */
static int vcycle_level(or_hier *H, int l)
{
    or_level *L = &H->lv[l];
    if (l == H->levels - 1)
        return or_coarse_solve(H, L->b, L->x);
    or_level *C = &H->lv[l + 1];
    or_op A = vcycle_op(L);
    cheb_op(&A, H->degree, L->lo, L->hi, L->b, L->x, 1, L->work);
    op_apply(&A, L->x, L->r);
    size_t nv = nvert(L->n);
    for (size_t p = 0; p < nv; p++)
        L->r[p] = L->b[p] - L->r[p];
    or_restrict_raw(L->n, L->r, C->n, C->b);
    int st = vcycle_level(H, l + 1);
    if (st != OR_OK)
        return st;
    or_prolong_add_raw(C->n, C->x, L->n, L->x);
    cheb_op(&A, H->degree, L->lo, L->hi, L->b, L->x, 0, L->work);
    return OR_OK;
}

/* z = B r, with B the V-cycle preconditioner on the finest level. */
int or_vcycle(void *hp, const double *r, double *z)
{
    or_hier *H = (or_hier *)hp;
    or_level *L = &H->lv[0];
    size_t nv = nvert(L->n);
    for (int k = 0; k < L->n; k++)
        for (int j = 0; j < L->n; j++)
            for (int i = 0; i < L->n; i++)
                L->b[vid(L->n, i, j, k)] = H->mixed ? or_round_f32(val(L->n, r, i, j, k)) : val(L->n, r, i, j, k);
    int st = vcycle_level(H, 0);
    for (size_t p = 0; p < nv; p++)
        z[p] = H->mixed ? or_round_f32(L->x[p]) : L->x[p];
    return st;
}

/* Smoother on an arbitrary level (exposed for the kernel-level checks). */
int or_smooth(void *hp, int l, const double *b, double *x, int x0_zero)
{
    or_hier *H = (or_hier *)hp;
    if (l < 0 || l >= H->levels)
        return OR_ERR_ARG;
    or_level *L = &H->lv[l];
    or_op A = vcycle_op(L);
    cheb_op(&A, H->degree, L->lo, L->hi, b, x, x0_zero, L->work);
    return OR_OK;
}

int or_apply(void *hp, int l, const double *u, double *out)
{
    or_hier *H = (or_hier *)hp;
    if (l < 0 || l >= H->levels)
        return OR_ERR_ARG;
    or_level *L = &H->lv[l];
    or_op A = vcycle_op(L);
    op_apply(&A, u, out);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Dot products over the interior, summed per z-plane and then in order.    */
/* ------------------------------------------------------------------------ */
static double dot_int(int n, const double *a, const double *b)
{
    double *plane = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 1; k <= n - 2; k++) {
        double s = 0.0;
        for (int j = 1; j <= n - 2; j++)
            for (int i = 1; i <= n - 2; i++)
                s += a[vid(n, i, j, k)] * b[vid(n, i, j, k)];
        plane[k] = s;
    }
    double s = 0.0;
    for (int k = 1; k <= n - 2; k++)
        s += plane[k];
    free(plane);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Preconditioned conjugate gradients (Sec. 2.1: CG as the Krylov method,   */
/* the V-cycle as preconditioner).  Stop when ||r||_2 <= rtol ||b||_2 (the  */
/* relative reduction of the initial residual used in Sec. 4.2 and 4.3,     */
/* with x0 = 0).  its counts the updates of x.  On exit relres is the       */
/* recursive residual ratio and relres_true = ||b - A x|| / ||b||.          */
/* ------------------------------------------------------------------------ */
static int pcg_impl(void *hp, const double *f, double *x, double rtol, int max_it, int flexible, int *its,
                    double *relres, double *relres_true);

int or_pcg(void *hp, const double *f, double *x, double rtol, int max_it, int *its,
           double *relres, double *relres_true)
{
    return pcg_impl(hp, f, x, rtol, max_it, 0, its, relres, relres_true);
}

/* flexible = 1: Polak-Ribiere beta = z_{k+1}.(r_{k+1} - r_k) / (r_k.z_k), which
 * with r_{k+1} - r_k = -alpha q_k is -alpha (q_k.z_{k+1}) / rho_k; it keeps CG
 * convergent when the preconditioner varies between iterations (an inexact
 * coarse solve). */
int or_pcg2(void *hp, const double *f, double *x, double rtol, int max_it, int flexible, int *its,
            double *relres, double *relres_true, long *coarse_its)
{
    or_hier *H = (or_hier *)hp;
    H->coarse_its = 0;
    int st = pcg_impl(hp, f, x, rtol, max_it, flexible, its, relres, relres_true);
    if (coarse_its)
        *coarse_its = H->coarse_its;
    return st;
}

static int pcg_impl(void *hp, const double *f, double *x, double rtol, int max_it, int flexible, int *its,
                    double *relres, double *relres_true)
{
    or_hier *H = (or_hier *)hp;
    or_level *L = &H->lv[0];
    int n = L->n;
    size_t nv = nvert(n);
    double *b = (double *)calloc(nv, sizeof(double));
    double *r = (double *)calloc(nv, sizeof(double));
    double *z = (double *)calloc(nv, sizeof(double));
    double *p = (double *)calloc(nv, sizeof(double));
    double *q = (double *)calloc(nv, sizeof(double));
    if (!b || !r || !z || !p || !q) {
        free(b); free(r); free(z); free(p); free(q);
        return OR_ERR_NOMEM;
    }
    int st = OR_OK;
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++)
                b[vid(n, i, j, k)] = val(n, f, i, j, k);
    memset(x, 0, sizeof(double) * nv);
    memcpy(r, b, sizeof(double) * nv);
    double bnorm = sqrt(dot_int(n, b, b));
    *its = 0;
    *relres = 0.0;
    *relres_true = 0.0;
    H->restarts = 0;
    if (bnorm == 0.0)
        goto done;
    if (!isfinite(bnorm)) {
        st = OR_ERR_ARG;
        goto done;
    }
    *relres = 1.0;
    for (;;) {
        /* start (or restart) of the recurrence from the current r */
        or_vcycle(H, r, z);
        memcpy(p, z, sizeof(double) * nv);
        double rho = dot_int(n, r, z);
        st = OR_ERR_NOT_CONVERGED;
        while (*its < max_it) {
            or_apply_raw(n, L->kx, L->ky, L->kz, p, q);
            double pq = dot_int(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) {
                st = OR_ERR_BREAKDOWN;
                break;
            }
            double alpha = rho / pq;
            for (size_t i = 0; i < nv; i++) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            *its += 1;
            double rnorm = sqrt(dot_int(n, r, r));
            *relres = rnorm / bnorm;
            if (!isfinite(rnorm)) {
                st = OR_ERR_BREAKDOWN;
                break;
            }
            if (rnorm <= rtol * bnorm) {
                st = OR_OK;
                break;
            }
            or_vcycle(H, r, z);
            double rho_new = dot_int(n, r, z);
            double beta = flexible ? -alpha * dot_int(n, q, z) / rho : rho_new / rho;
            rho = rho_new;
            for (size_t i = 0; i < nv; i++)
                p[i] = H->mixed ? or_round_f32(z[i] + beta * p[i]) : z[i] + beta * p[i];
        }
        /* true residual q = b - A x */
        or_apply_raw(n, L->kx, L->ky, L->kz, x, q);
        for (size_t i = 0; i < nv; i++)
            q[i] = b[i] - q[i];
        double tnorm = sqrt(dot_int(n, q, q));
        *relres_true = tnorm / bnorm;
        if (st != OR_OK || !H->mixed || tnorm <= rtol * bnorm || H->restarts >= 20 || *its >= max_it)
            break;
        /* reduced precision: the recursive residual passed, the true one did
         * not; continue from the true residual with a fresh search direction */
        H->restarts++;
        memcpy(r, q, sizeof(double) * nv);
    }
    if (st == OR_OK && H->mixed && !(*relres_true <= rtol))
        st = OR_ERR_NOT_CONVERGED;
done:
    if (!H->last_p)
        H->last_p = (double *)malloc(sizeof(double) * nv);
    if (H->last_p)
        memcpy(H->last_p, p, sizeof(double) * nv);
    free(b); free(r); free(z); free(p); free(q);
    return st;
}

int or_last_restarts(void *hp) { return ((or_hier *)hp)->restarts; }

/* The search direction p as the last CG solve left it: the direction the
 * next x update would use (after a solve stopped by max_it), N^3 values. */
int or_last_direction(void *hp, double *out)
{
    or_hier *H = (or_hier *)hp;
    if (!H || !out || !H->last_p)
        return OR_ERR_ARG;
    memcpy(out, H->last_p, sizeof(double) * nvert(H->lv[0].n));
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint gradient.  With A(k) phi = f and a loss L(phi):                  */
/*   A lambda = dL/dphi          (A is symmetric, so A^T = A)               */
/*   dL/dk_f  = -h^-2 (lambda_p - lambda_q)(phi_p - phi_q)                   */
/*   dL/dtheta_f = k_f dL/dk_f   with theta = ln k                          */
/* for every link f = (p,q) with at least one interior end point; a         */
/* boundary end point contributes zero values.  Links between two boundary  */
/* vertices get 0.  lambda (may be NULL) receives the adjoint solution.     */
/* The coarse hierarchy only preconditions the solve and is not             */
/* differentiated.                                                          */
/* ------------------------------------------------------------------------ */
int or_adjoint_gradient(void *hp, const double *phi, const double *dl_dphi, double *gx, double *gy,
                        double *gz, double *lambda, double rtol, int max_it, int *its)
{
    or_hier *H = (or_hier *)hp;
    or_level *L = &H->lv[0];
    int n = L->n;
    double s = (double)(n - 1) * (double)(n - 1);
    double *lam = (double *)calloc(nvert(n), sizeof(double));
    if (!lam)
        return OR_ERR_NOMEM;
    double rr, rt;
    int st = or_pcg(H, dl_dphi, lam, rtol, max_it, its, &rr, &rt);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n - 1; i++) {
                double g = 0.0;
                if (interior(n, i, j, k) || interior(n, i + 1, j, k))
                    g = -s * (val(n, lam, i, j, k) - val(n, lam, i + 1, j, k)) *
                        (val(n, phi, i, j, k) - val(n, phi, i + 1, j, k));
                gx[xid(n, i, j, k)] = g != 0.0 ? L->kx[xid(n, i, j, k)] * g : 0.0;
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n - 1; j++)
            for (int i = 0; i < n; i++) {
                double g = 0.0;
                if (interior(n, i, j, k) || interior(n, i, j + 1, k))
                    g = -s * (val(n, lam, i, j, k) - val(n, lam, i, j + 1, k)) *
                        (val(n, phi, i, j, k) - val(n, phi, i, j + 1, k));
                gy[yid(n, i, j, k)] = g != 0.0 ? L->ky[yid(n, i, j, k)] * g : 0.0;
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n - 1; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double g = 0.0;
                if (interior(n, i, j, k) || interior(n, i, j, k + 1))
                    g = -s * (val(n, lam, i, j, k) - val(n, lam, i, j, k + 1)) *
                        (val(n, phi, i, j, k) - val(n, phi, i, j, k + 1));
                gz[zid(n, i, j, k)] = g != 0.0 ? L->kz[zid(n, i, j, k)] * g : 0.0;
            }
    if (lambda)
        memcpy(lambda, lam, sizeof(double) * nvert(n));
    free(lam);
    return st;
}

/* Copy the 27-point coarse operator of level l (Galerkin hierarchies). */
int or_level_interval(void *hp, int l, double *lo, double *hi)
{
    or_hier *H = (or_hier *)hp;
    if (l < 0 || l >= H->levels)
        return OR_ERR_ARG;
    *lo = H->lv[l].lo;
    *hi = H->lv[l].hi;
    return OR_OK;
}

int or_get_a27(void *hp, int l, double *out)
{
    or_hier *H = (or_hier *)hp;
    if (l < 0 || l >= H->levels || !H->lv[l].a27)
        return OR_ERR_ARG;
    memcpy(out, H->lv[l].a27, sizeof(double) * nvert(H->lv[l].n) * 27);
    return OR_OK;
}
