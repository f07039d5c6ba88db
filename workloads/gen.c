/*
 * Seeded synthetic test matrices for eigenvector refinement.
 *
 * Input generation only: this file holds none of the refinement method's
 * arithmetic. It builds A = Q diag(lambda) Q^T with Q a product of Householder
 * reflectors H_k = I - 2 v_k v_k^T / (v_k^T v_k), as a stand-in for the
 * geometric-spectrum random symmetric matrices of the paper's experiments
 * (Sec. 4, randsvd with geometric spectrum).
 *
 * Every loop runs in a fixed order and the file is built with
 * -ffp-contract=off, so a given (v, lambda) always yields the same bits on any
 * x86-64 host. The generated A is exactly symmetric: only the upper triangle
 * is updated and it is mirrored at the end.
 *
 * Storage: column-major n x n, element (i, j) at i + j*n.
 */
#include <stdlib.h>
#include <string.h>

/* M <- H M H for symmetric M (upper triangle authoritative), H = I - tau v v^T,
 * tau = 2 / (v^T v). Uses p = tau M v, K = tau/2 v^T p, q = p - K v,
 * M <- M - v q^T - q v^T. */
static void reflect_two_sided(int n, double *M, const double *v, double *p)
{
    double vv = 0.0;
    for (int i = 0; i < n; ++i) vv += v[i] * v[i];
    const double tau = 2.0 / vv;
    /* p = M v using the upper triangle only: M(i,j) for i<=j is M[i + j*n] */
    for (int i = 0; i < n; ++i) p[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        const double *col = M + (size_t)j * n;
        double acc = 0.0;
        for (int i = 0; i <= j; ++i) acc += col[i] * v[i];          /* row j, cols i<=j */
        for (int i = j + 1; i < n; ++i) acc += M[j + (size_t)i * n] * v[i]; /* M(j,i), i>j */
        p[j] = acc;
    }
    double vp = 0.0;
    for (int i = 0; i < n; ++i) { p[i] *= tau; vp += v[i] * p[i]; }
    const double K = 0.5 * tau * vp;
    for (int i = 0; i < n; ++i) p[i] = p[i] - K * v[i];   /* p now holds q */
    for (int j = 0; j < n; ++j) {
        double *col = M + (size_t)j * n;
        const double vj = v[j], qj = p[j];
        for (int i = 0; i <= j; ++i) col[i] = (col[i] - v[i] * qj) - p[i] * vj;
    }
}

/* A = H_1 ... H_m diag(lam) H_m ... H_1. V holds the m reflector vectors,
 * column-major n x m. Output A column-major, exactly symmetric. */
int wl_householder_sym(int n, int m, const double *V, const double *lam, double *A)
{
    if (n <= 0 || m < 0 || !V || !lam || !A) return -1;
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p) return -2;
    memset(A, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) A[i + (size_t)i * n] = lam[i];
    for (int k = m - 1; k >= 0; --k) reflect_two_sided(n, A, V + (size_t)k * n, p);
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) A[i + (size_t)j * n] = A[j + (size_t)i * n];
    free(p);
    return 0;
}

/* Q = H_1 H_2 ... H_m, column-major. Q's column j is the eigenvector of the
 * unrounded Q diag(lam) Q^T for lam_j. */
int wl_householder_q(int n, int m, const double *V, double *Q)
{
    if (n <= 0 || m < 0 || !V || !Q) return -1;
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p) return -2;
    memset(Q, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
    /* Q <- H_k Q for k = m..1, i.e. Q = H_1 (H_2 (... (H_m I))) */
    for (int k = m - 1; k >= 0; --k) {
        const double *v = V + (size_t)k * n;
        double vv = 0.0;
        for (int i = 0; i < n; ++i) vv += v[i] * v[i];
        const double tau = 2.0 / vv;
        for (int j = 0; j < n; ++j) {
            double *col = Q + (size_t)j * n;
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += v[i] * col[i];
            s *= tau;
            for (int i = 0; i < n; ++i) col[i] = col[i] - s * v[i];
        }
    }
    free(p);
    return 0;
}

/* Diagonal-plus-rank-one matrix A = diag(dg) + rho u u^T assembled in FP64:
 * off-diagonal entries rho*u_i*u_j, diagonal fl(dg_i + rho*u_i^2). The caller
 * chooses u and rho with few significant bits so every off-diagonal product is
 * exact; the diagonal rounding is recorded by the caller from A itself. */
int wl_diag_rank1(int n, const double *dg, double rho, const double *u, double *A)
{
    if (n <= 0 || !dg || !u || !A) return -1;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            A[i + (size_t)j * n] = (i == j) ? dg[i] + (rho * u[i]) * u[i] : (rho * u[i]) * u[j];
    return 0;
}

/* Complex Hermitian counterpart: M <- H M H with H = I - tau v v^H, tau = 2 / (v^H v),
 * M Hermitian stored as real and imaginary parts (upper triangle authoritative).
 * With p = tau M v, K = (tau/2) Re(v^H p) and q = p - K v: H M H = M - v q^H - q v^H. */
static void reflect_two_sided_c(int n, double *Mr, double *Mi, const double *vr,
                                const double *vi, double *pr, double *pi)
{
    double vv = 0.0;
    for (int i = 0; i < n; ++i) vv += vr[i] * vr[i] + vi[i] * vi[i];
    const double tau = 2.0 / vv;
    /* p_j = sum_i M(j, i) v_i; M(j, i) = conj(M(i, j)) for i < j */
    for (int j = 0; j < n; ++j) {
        double ar = 0.0, ai = 0.0;
        for (int i = 0; i < n; ++i) {
            double mr, mi;
            if (i >= j) { mr = Mr[j + (size_t)i * n]; mi = Mi[j + (size_t)i * n]; }
            else        { mr = Mr[i + (size_t)j * n]; mi = -Mi[i + (size_t)j * n]; }
            ar += mr * vr[i] - mi * vi[i];
            ai += mr * vi[i] + mi * vr[i];
        }
        pr[j] = tau * ar;
        pi[j] = tau * ai;
    }
    double vp = 0.0;   /* Re(v^H p) */
    for (int i = 0; i < n; ++i) vp += vr[i] * pr[i] + vi[i] * pi[i];
    const double K = 0.5 * tau * vp;
    for (int i = 0; i < n; ++i) { pr[i] -= K * vr[i]; pi[i] -= K * vi[i]; }   /* q */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) {
            /* v_i conj(q_j) + q_i conj(v_j) */
            const double tr = (vr[i] * pr[j] + vi[i] * pi[j]) + (pr[i] * vr[j] + pi[i] * vi[j]);
            const double ti = (vi[i] * pr[j] - vr[i] * pi[j]) + (pi[i] * vr[j] - pr[i] * vi[j]);
            Mr[i + (size_t)j * n] -= tr;
            Mi[i + (size_t)j * n] -= ti;
        }
}

/* A = H_1 ... H_m diag(lam) H_m ... H_1 with complex reflectors (Vr + i Vi, column-major
 * n x m). Output: real and imaginary parts, column-major, exactly Hermitian (the lower
 * triangle mirrors the upper one, the diagonal is real). */
int wl_householder_herm(int n, int m, const double *Vr, const double *Vi, const double *lam,
                        double *Ar, double *Ai)
{
    if (n <= 0 || m < 0 || !Vr || !Vi || !lam || !Ar || !Ai) return -1;
    double *pr = (double *)malloc(sizeof(double) * (size_t)n);
    double *pi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!pr || !pi) { free(pr); free(pi); return -2; }
    memset(Ar, 0, sizeof(double) * (size_t)n * n);
    memset(Ai, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) Ar[i + (size_t)i * n] = lam[i];
    for (int k = m - 1; k >= 0; --k)
        reflect_two_sided_c(n, Ar, Ai, Vr + (size_t)k * n, Vi + (size_t)k * n, pr, pi);
    for (int j = 0; j < n; ++j) {
        Ai[j + (size_t)j * n] = 0.0;
        for (int i = j + 1; i < n; ++i) {
            Ar[i + (size_t)j * n] = Ar[j + (size_t)i * n];
            Ai[i + (size_t)j * n] = -Ai[j + (size_t)i * n];
        }
    }
    free(pr); free(pi);
    return 0;
}
