/*
 * Plain FP64 CPU oracle for the linear-quadratic tracker (LQT).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Source: Sarkka & Garcia-Fernandez, "Temporal Parallelisation of Dynamic
 * Programming and Linear Quadratic Control" (arXiv 2104.03186).
 *
 *  - oracle_solve: the sequential LQT solution of Section II-B: the backward
 *    recursion for S_k, v_k and the gain K_k, the control law
 *    u_k = -K_k x_k + K^v_k v_{k+1} - K^c_k c_k, and the forward pass of the
 *    dynamics from x_0 under that law.  d_k denotes K^v_k v_{k+1} - K^c_k c_k.
 *  - oracle_element: the one-step conditional value function elements
 *    (A, b, C, eta, J) of Section IV-B (lemma on the LQT scan elements),
 *    including the terminal element.  The terminal eta is H_T^T X_T r_T: the
 *    printed form lacks X_T, which contradicts the terminal cost of the
 *    problem statement (Section II-B) and the start of the backward recursion.
 *  - oracle_combine: the LQT associative operator of Section IV-A (lemma on
 *    the LQT combination rule), evaluated literally with two LU solves.
 *  - oracle_cost: the total cost of the problem statement, Section II-B.
 *  - oracle_solve_gen: the sequential solution for the generalised stage
 *    cost with a state-control cross term and a control reference (the
 *    extension to more general cost functions, Section IV-D), by dynamic
 *    programming written out from that cost.
 *
 * Every routine is a direct transcription of a definition: no blocking, no
 * fusion, no reordering.  All arithmetic is IEEE double precision.
 *
 * Array conventions (row-major, contiguous):
 *   F [n][n] (or [T][n][n] when per-step), c [n] (or [T][n], NULL means 0),
 *   L [n][m], H [p][n], X [p][p], U [m][m], r [T][p],
 *   HT [pT][n], XT [pT][pT], rT [pT], x0 [n].
 *   Outputs: S [T+1][n][n], v [T+1][n], K [T][m][n], d [T][m],
 *            x [T+1][n], u [T][m].
 *
 * Return codes: 0 success, 1 invalid argument, 3 a matrix that must be
 * positive definite is not, 4 a non-finite value was produced.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOTPD = 3, OR_ENONFINITE = 4 };
enum { PS_F = 1, PS_c = 2, PS_L = 4, PS_H = 8, PS_X = 16, PS_U = 32 };

/* ---- plain dense helpers (row-major) ---------------------------------- */

/* C[r][c] = sum_k A[r][k] * B[k][c] ; A is r x k, B is k x c */
static void mm(int nr, int nk, int nc, const double *A, const double *B, double *C) {
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
            double s = 0.0;
            for (int k = 0; k < nk; ++k) s += A[i * nk + k] * B[k * nc + j];
            C[i * nc + j] = s;
        }
}

/* C = A^T B ; A is nk x nr, B is nk x nc */
static void mtm(int nr, int nk, int nc, const double *A, const double *B, double *C) {
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
            double s = 0.0;
            for (int k = 0; k < nk; ++k) s += A[k * nr + i] * B[k * nc + j];
            C[i * nc + j] = s;
        }
}

/* y = A x ; A is nr x nc */
static void mv(int nr, int nc, const double *A, const double *x, double *y) {
    for (int i = 0; i < nr; ++i) {
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += A[i * nc + j] * x[j];
        y[i] = s;
    }
}

/* y = A^T x ; A is nr x nc, y has nc entries */
static void mtv(int nr, int nc, const double *A, const double *x, double *y) {
    for (int j = 0; j < nc; ++j) {
        double s = 0.0;
        for (int i = 0; i < nr; ++i) s += A[i * nc + j] * x[i];
        y[j] = s;
    }
}

/* In-place Cholesky A = R R^T (R lower) of an m x m symmetric matrix.
 * Returns 0, or OR_ENOTPD when a pivot is not strictly positive. */
static int cholesky(int m, double *A) {
    for (int j = 0; j < m; ++j) {
        double s = A[j * m + j];
        for (int k = 0; k < j; ++k) s -= A[j * m + k] * A[j * m + k];
        if (!(s > 0.0)) return OR_ENOTPD;
        double rjj = sqrt(s);
        A[j * m + j] = rjj;
        for (int i = j + 1; i < m; ++i) {
            double t = A[i * m + j];
            for (int k = 0; k < j; ++k) t -= A[i * m + k] * A[j * m + k];
            A[i * m + j] = t / rjj;
        }
        for (int i = 0; i < j; ++i) A[i * m + j] = 0.0;
    }
    return OR_OK;
}

/* Solve (R R^T) Y = B in place for an m x nc right-hand side, R from cholesky. */
static void chol_solve(int m, int nc, const double *R, double *B) {
    for (int c = 0; c < nc; ++c) {
        for (int i = 0; i < m; ++i) { /* forward: R z = b */
            double s = B[i * nc + c];
            for (int k = 0; k < i; ++k) s -= R[i * m + k] * B[k * nc + c];
            B[i * nc + c] = s / R[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) { /* backward: R^T y = z */
            double s = B[i * nc + c];
            for (int k = i + 1; k < m; ++k) s -= R[k * m + i] * B[k * nc + c];
            B[i * nc + c] = s / R[i * m + i];
        }
    }
}

/* Solve M Y = B (M n x n, B n x nc) by LU with partial pivoting.  M and B are
 * overwritten (B with the solution).  Returns 0, or OR_EINVAL when singular. */
static int lu_solve(int n, int nc, double *M, double *B) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > fabs(M[p * n + k])) p = i;
        if (M[p * n + k] == 0.0) return OR_EINVAL;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
            for (int j = 0; j < nc; ++j) { double t = B[k * nc + j]; B[k * nc + j] = B[p * nc + j]; B[p * nc + j] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            double f = M[i * n + k] / M[k * n + k];
            M[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            for (int j = 0; j < nc; ++j) B[i * nc + j] -= f * B[k * nc + j];
        }
    }
    for (int i = n - 1; i >= 0; --i)
        for (int j = 0; j < nc; ++j) {
            double s = B[i * nc + j];
            for (int k = i + 1; k < n; ++k) s -= M[i * n + k] * B[k * nc + j];
            B[i * nc + j] = s / M[i * n + i];
        }
    return OR_OK;
}

/* S <- (S + S^T) / 2 */
static void symmetrize(int n, double *S) {
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double s = 0.5 * (S[i * n + j] + S[j * n + i]);
            S[i * n + j] = s;
            S[j * n + i] = s;
        }
}

static int all_finite(size_t cnt, const double *a) {
    for (size_t i = 0; i < cnt; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* Pointer to the step-k copy of a matrix that is per-step when `bit` is set. */
static const double *at(const double *base, uint32_t per_step, uint32_t bit, int64_t k, size_t sz) {
    return (per_step & bit) ? base + (size_t)k * sz : base;
}

/* ---- the sequential solution, Section II-B ----------------------------- */

int oracle_solve(int n, int m, int p, int pT, int64_t T, uint32_t per_step,
                 const double *F, const double *c, const double *L, const double *H,
                 const double *X, const double *U, const double *r,
                 const double *HT, const double *XT, const double *rT, const double *x0,
                 double *S, double *v, double *K, double *d, double *x, double *u) {
    if (n < 1 || m < 1 || p < 1 || pT < 1 || T < 1) return OR_EINVAL;
    if (!F || !L || !H || !X || !U || !r || !HT || !XT || !rT || !x0) return OR_EINVAL;
    if (!S || !v || !K || !d || !x || !u) return OR_EINVAL;

    const size_t nn = (size_t)n * n, nm = (size_t)n * m, pn = (size_t)p * n;
    const size_t pp = (size_t)p * p, mm_ = (size_t)m * m;
    int rc = OR_OK;
    double *XH = malloc(sizeof(double) * (size_t)(p > pT ? p : pT) * n);
    double *Xr = malloc(sizeof(double) * (size_t)(p > pT ? p : pT));
    double *SL = malloc(sizeof(double) * nm);
    double *Mk = malloc(sizeof(double) * mm_);
    double *SF = malloc(sizeof(double) * nn);
    double *Ft = malloc(sizeof(double) * nn);
    double *Sc = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * n);
    double *Lw = malloc(sizeof(double) * m);
    double *Q = malloc(sizeof(double) * nn);
    double *hq = malloc(sizeof(double) * n);
    double *t1 = malloc(sizeof(double) * n);
    double *t2 = malloc(sizeof(double) * n);
    if (!XH || !Xr || !SL || !Mk || !SF || !Ft || !Sc || !w || !Lw || !Q || !hq || !t1 || !t2) {
        rc = OR_EINVAL;
        goto done;
    }

    /* Terminal value function: S_T = H_T^T X_T H_T (made exactly symmetric),
     * v_T = H_T^T X_T r_T. */
    double *ST = S + (size_t)T * nn, *vT = v + (size_t)T * n;
    mm(pT, pT, n, XT, HT, XH);
    mtm(n, pT, n, HT, XH, ST);
    mv(pT, pT, XT, rT, Xr);
    mtv(pT, n, HT, Xr, vT);
    symmetrize(n, ST);

    for (int64_t k = T - 1; k >= 0; --k) {
        const double *Fk = at(F, per_step, PS_F, k, nn);
        const double *ck = c ? at(c, per_step, PS_c, k, n) : NULL;
        const double *Lk = at(L, per_step, PS_L, k, nm);
        const double *Hk = at(H, per_step, PS_H, k, pn);
        const double *Xk = at(X, per_step, PS_X, k, pp);
        const double *Uk = at(U, per_step, PS_U, k, mm_);
        const double *S1 = S + (size_t)(k + 1) * nn, *v1 = v + (size_t)(k + 1) * n;
        double *Sk = S + (size_t)k * nn, *vk = v + (size_t)k * n;
        double *Kk = K + (size_t)k * m * n, *dk = d + (size_t)k * m;

        /* M_k = L^T S_{k+1} L + U, factorised by Cholesky. */
        mm(n, n, m, S1, Lk, SL);
        mtm(m, n, m, Lk, SL, Mk);
        for (size_t i = 0; i < mm_; ++i) Mk[i] += Uk[i];
        rc = cholesky(m, Mk);
        if (rc) goto done;

        /* K_k = M_k^{-1} L^T S_{k+1} F. */
        mm(n, n, n, S1, Fk, SF);
        mtm(m, n, n, Lk, SF, Kk);
        chol_solve(m, n, Mk, Kk);

        /* d_k = M_k^{-1} L^T (v_{k+1} - S_{k+1} c_k) = K^v_k v_{k+1} - K^c_k c_k. */
        if (ck) mv(n, n, S1, ck, Sc); else memset(Sc, 0, sizeof(double) * n);
        for (int i = 0; i < n; ++i) w[i] = v1[i] - Sc[i];
        mtv(n, m, Lk, w, Lw);
        memcpy(dk, Lw, sizeof(double) * m);
        chol_solve(m, 1, Mk, dk);

        /* Closed-loop matrix F - L K. */
        mm(n, m, n, Lk, Kk, Ft);
        for (size_t i = 0; i < nn; ++i) Ft[i] = Fk[i] - Ft[i];

        /* S_k = F^T S_{k+1} (F - L K) + H^T X H, then made exactly symmetric. */
        mm(n, n, n, S1, Ft, Q);
        mtm(n, n, n, Fk, Q, Sk);
        mm(p, p, n, Xk, Hk, XH);
        mtm(n, p, n, Hk, XH, Q);
        for (size_t i = 0; i < nn; ++i) Sk[i] += Q[i];
        symmetrize(n, Sk);

        /* v_k = (F - L K)^T (v_{k+1} - S_{k+1} c_k) + H^T X r_k. */
        mtv(n, n, Ft, w, vk);
        mv(p, p, Xk, r + (size_t)k * p, Xr);
        mtv(p, n, Hk, Xr, hq);
        for (int i = 0; i < n; ++i) vk[i] += hq[i];
    }

    /* Forward pass: u_k = -K_k x_k + d_k, x_{k+1} = F x_k + c + L u_k. */
    memcpy(x, x0, sizeof(double) * n);
    for (int64_t k = 0; k < T; ++k) {
        const double *Fk = at(F, per_step, PS_F, k, nn);
        const double *ck = c ? at(c, per_step, PS_c, k, n) : NULL;
        const double *Lk = at(L, per_step, PS_L, k, nm);
        const double *xk = x + (size_t)k * n;
        double *uk = u + (size_t)k * m, *xn = x + (size_t)(k + 1) * n;
        mv(m, n, K + (size_t)k * m * n, xk, uk);
        for (int i = 0; i < m; ++i) uk[i] = -uk[i] + d[(size_t)k * m + i];
        mv(n, n, Fk, xk, t1);
        mv(n, m, Lk, uk, t2);
        for (int i = 0; i < n; ++i) xn[i] = t1[i] + t2[i] + (ck ? ck[i] : 0.0);
    }

    if (!all_finite((size_t)(T + 1) * nn, S) || !all_finite((size_t)(T + 1) * n, x))
        rc = OR_ENONFINITE;

done:
    free(XH); free(Xr); free(SL); free(Mk); free(SF); free(Ft); free(Sc);
    free(w); free(Lw); free(Q); free(hq); free(t1); free(t2);
    return rc;
}

/* ---- generalised stage cost, Section IV-D ------------------------------- */

/*
 * The sequential solution for the stage cost with a state-control cross term
 * and a control reference (the extension to more general cost functions):
 *   l_k = 1/2 (H x - r)^T X (H x - r) + (H x - r)^T M (u - s)
 *         + 1/2 (u - s)^T U (u - s),
 * M [p][m] (or [T][p][m] with per-step bit 64), s [T][m] (NULL means 0).
 * Dynamic programming written out from that cost (not through the paper's
 * transformation to the standard form, which the tests check against it):
 * with V_{k+1}(x) = 1/2 x^T S x - v^T x, the step cost plus V_{k+1}(F x + c +
 * L u) is 1/2 x^T Aq x + x^T Bq u + 1/2 u^T W u - a^T x - b^T u + const,
 *   Aq = H^T X H + F^T S F,   Bq = H^T M + F^T S L,   W = U + L^T S L,
 *   a = H^T X r + H^T M s + F^T (v - S c),   b = M^T r + U s + L^T (v - S c),
 * minimised by u = -K x + d, K = W^{-1} Bq^T, d = W^{-1} b, giving
 *   S_k = Aq - Bq K (made exactly symmetric),  v_k = a - Bq d.
 * The forward pass is the same as for the standard cost.
 */
enum { PS_M = 64 };

int oracle_solve_gen(int n, int m, int p, int pT, int64_t T, uint32_t per_step,
                     const double *F, const double *c, const double *L, const double *H,
                     const double *X, const double *U, const double *r,
                     const double *HT, const double *XT, const double *rT, const double *x0,
                     const double *M, const double *s,
                     double *S, double *v, double *K, double *d, double *x, double *u) {
    if (n < 1 || m < 1 || p < 1 || pT < 1 || T < 1) return OR_EINVAL;
    if (!F || !L || !H || !X || !U || !r || !HT || !XT || !rT || !x0 || !M) return OR_EINVAL;
    if (!S || !v || !K || !d || !x || !u) return OR_EINVAL;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, pn = (size_t)p * n;
    const size_t pp = (size_t)p * p, mm_ = (size_t)m * m, pm = (size_t)p * m;
    int rc = OR_OK;
    const int pq = p > pT ? p : pT;
    double *XH = malloc(sizeof(double) * (size_t)pq * n), *Xr = malloc(sizeof(double) * (size_t)pq);
    double *SF = malloc(sizeof(double) * nn), *SL = malloc(sizeof(double) * nm);
    double *Aq = malloc(sizeof(double) * nn), *Bq = malloc(sizeof(double) * nm);
    double *W = malloc(sizeof(double) * mm_), *HM = malloc(sizeof(double) * nm);
    double *Sc = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    double *av = malloc(sizeof(double) * n), *bv = malloc(sizeof(double) * m);
    double *tm = malloc(sizeof(double) * m), *tn = malloc(sizeof(double) * n);
    double *BK = malloc(sizeof(double) * nn), *t1 = malloc(sizeof(double) * n), *t2 = malloc(sizeof(double) * n);
    if (!XH || !Xr || !SF || !SL || !Aq || !Bq || !W || !HM || !Sc || !w || !av || !bv || !tm || !tn || !BK ||
        !t1 || !t2) {
        rc = OR_EINVAL;
        goto done;
    }
    double *ST = S + (size_t)T * nn, *vT = v + (size_t)T * n;
    mm(pT, pT, n, XT, HT, XH);
    mtm(n, pT, n, HT, XH, ST);
    mv(pT, pT, XT, rT, Xr);
    mtv(pT, n, HT, Xr, vT);
    symmetrize(n, ST);
    for (int64_t k = T - 1; k >= 0; --k) {
        const double *Fk = at(F, per_step, PS_F, k, nn);
        const double *ck = c ? at(c, per_step, PS_c, k, n) : NULL;
        const double *Lk = at(L, per_step, PS_L, k, nm);
        const double *Hk = at(H, per_step, PS_H, k, pn);
        const double *Xk = at(X, per_step, PS_X, k, pp);
        const double *Uk = at(U, per_step, PS_U, k, mm_);
        const double *Mk = at(M, per_step, PS_M, k, pm);
        const double *rk = r + (size_t)k * p;
        const double *S1 = S + (size_t)(k + 1) * nn, *v1 = v + (size_t)(k + 1) * n;
        double *Sk = S + (size_t)k * nn, *vk = v + (size_t)k * n;
        double *Kk = K + (size_t)k * m * n, *dk = d + (size_t)k * m;
        /* Aq = H^T X H + F^T S F */
        mm(p, p, n, Xk, Hk, XH);
        mtm(n, p, n, Hk, XH, Aq);
        mm(n, n, n, S1, Fk, SF);
        mtm(n, n, n, Fk, SF, BK);
        for (size_t i = 0; i < nn; ++i) Aq[i] += BK[i];
        /* Bq = H^T M + F^T S L */
        mtm(n, p, m, Hk, Mk, HM);
        mm(n, n, m, S1, Lk, SL);
        mtm(n, n, m, Fk, SL, Bq);
        for (size_t i = 0; i < nm; ++i) Bq[i] += HM[i];
        /* W = U + L^T S L */
        mtm(m, n, m, Lk, SL, W);
        for (size_t i = 0; i < mm_; ++i) W[i] += Uk[i];
        /* w = v - S c */
        if (ck) mv(n, n, S1, ck, Sc); else memset(Sc, 0, sizeof(double) * n);
        for (int i = 0; i < n; ++i) w[i] = v1[i] - Sc[i];
        /* a = H^T X r + H^T M s + F^T w ;  b = M^T r + U s + L^T w */
        mv(p, p, Xk, rk, Xr);
        mtv(p, n, Hk, Xr, av);
        mtv(n, n, Fk, w, tn);
        for (int i = 0; i < n; ++i) av[i] += tn[i];
        mtv(p, m, Mk, rk, bv);
        mtv(n, m, Lk, w, tm);
        for (int i = 0; i < m; ++i) bv[i] += tm[i];
        if (s) {
            const double *sk = s + (size_t)k * m;
            mv(n, m, HM, sk, tn);
            for (int i = 0; i < n; ++i) av[i] += tn[i];
            mv(m, m, Uk, sk, tm);
            for (int i = 0; i < m; ++i) bv[i] += tm[i];
        }
        /* K = W^{-1} Bq^T ; d = W^{-1} b */
        rc = cholesky(m, W);
        if (rc) goto done;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) Kk[i * n + j] = Bq[j * m + i];
        chol_solve(m, n, W, Kk);
        memcpy(dk, bv, sizeof(double) * m);
        chol_solve(m, 1, W, dk);
        /* S_k = Aq - Bq K ; v_k = a - Bq d */
        mm(n, m, n, Bq, Kk, BK);
        for (size_t i = 0; i < nn; ++i) Sk[i] = Aq[i] - BK[i];
        symmetrize(n, Sk);
        mv(n, m, Bq, dk, tn);
        for (int i = 0; i < n; ++i) vk[i] = av[i] - tn[i];
    }
    memcpy(x, x0, sizeof(double) * n);
    for (int64_t k = 0; k < T; ++k) {
        const double *Fk = at(F, per_step, PS_F, k, nn);
        const double *ck = c ? at(c, per_step, PS_c, k, n) : NULL;
        const double *Lk = at(L, per_step, PS_L, k, nm);
        const double *xk = x + (size_t)k * n;
        double *uk = u + (size_t)k * m, *xn = x + (size_t)(k + 1) * n;
        mv(m, n, K + (size_t)k * m * n, xk, uk);
        for (int i = 0; i < m; ++i) uk[i] = -uk[i] + d[(size_t)k * m + i];
        mv(n, n, Fk, xk, t1);
        mv(n, m, Lk, uk, t2);
        for (int i = 0; i < n; ++i) xn[i] = t1[i] + t2[i] + (ck ? ck[i] : 0.0);
    }
    if (!all_finite((size_t)(T + 1) * nn, S) || !all_finite((size_t)(T + 1) * n, x)) rc = OR_ENONFINITE;
done:
    free(XH); free(Xr); free(SF); free(SL); free(Aq); free(Bq); free(W); free(HM); free(Sc); free(w);
    free(av); free(bv); free(tm); free(tn); free(BK); free(t1); free(t2);
    return rc;
}

/* ---- scan elements and the associative operator, Section IV ------------ */

/*
 * One element (A, b, C, eta, J), each n-dimensional, packed as
 *   A[n*n] | b[n] | C[n*n] | eta[n] | J[n*n]     (3n^2 + 2n doubles).
 * It parameterises the dual function of the conditional value function
 * V_{k->i}(x_k, x_i), Section IV-A.
 */

/* Element a_k = V_{k->k+1} for k < T; the terminal element for k == T. */
int oracle_element(int n, int m, int p, int pT, int64_t T, uint32_t per_step, int64_t k,
                   const double *F, const double *c, const double *L, const double *H,
                   const double *X, const double *U, const double *r,
                   const double *HT, const double *XT, const double *rT, double *e) {
    const size_t nn = (size_t)n * n;
    double *A = e, *b = e + nn, *C = e + nn + n, *eta = e + 2 * nn + n, *J = e + 2 * nn + 2 * n;
    if (k < 0 || k > T) return OR_EINVAL;
    int q = (k == T) ? pT : p;
    double *XH = malloc(sizeof(double) * (size_t)q * n);
    double *Xr = malloc(sizeof(double) * (size_t)q);
    double *Ui = malloc(sizeof(double) * (size_t)m * m);
    double *UiLt = malloc(sizeof(double) * (size_t)m * n);
    int rc = OR_OK;
    if (k == T) {
        /* A = 0, b = 0, C = 0, eta = H_T^T X_T r_T, J = H_T^T X_T H_T. */
        memset(A, 0, sizeof(double) * nn);
        memset(b, 0, sizeof(double) * n);
        memset(C, 0, sizeof(double) * nn);
        mm(pT, pT, n, XT, HT, XH);
        mtm(n, pT, n, HT, XH, J);
        mv(pT, pT, XT, rT, Xr);
        mtv(pT, n, HT, Xr, eta);
    } else {
        const double *Fk = at(F, per_step, PS_F, k, nn);
        const double *ck = c ? at(c, per_step, PS_c, k, n) : NULL;
        const double *Lk = at(L, per_step, PS_L, k, (size_t)n * m);
        const double *Hk = at(H, per_step, PS_H, k, (size_t)p * n);
        const double *Xk = at(X, per_step, PS_X, k, (size_t)p * p);
        const double *Uk = at(U, per_step, PS_U, k, (size_t)m * m);
        /* A = F_k, b = c_k */
        memcpy(A, Fk, sizeof(double) * nn);
        if (ck) memcpy(b, ck, sizeof(double) * n); else memset(b, 0, sizeof(double) * n);
        /* C = L U^{-1} L^T */
        memcpy(Ui, Uk, sizeof(double) * m * m);
        rc = cholesky(m, Ui);
        if (rc) goto done;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) UiLt[i * n + j] = Lk[j * m + i];
        chol_solve(m, n, Ui, UiLt);
        mm(n, m, n, Lk, UiLt, C);
        /* eta = H^T X r_k, J = H^T X H */
        mv(p, p, Xk, r + (size_t)k * p, Xr);
        mtv(p, n, Hk, Xr, eta);
        mm(p, p, n, Xk, Hk, XH);
        mtm(n, p, n, Hk, XH, J);
    }
done:
    free(XH); free(Xr); free(Ui); free(UiLt);
    return rc;
}

/*
 * out = e1 (x) e2, with e1 = V_{k->j} (earlier) and e2 = V_{j->i} (later):
 *   A   = A2 (I + C1 J2)^{-1} A1
 *   b   = A2 (I + C1 J2)^{-1} (b1 + C1 eta2) + b2
 *   C   = A2 (I + C1 J2)^{-1} C1 A2^T + C2
 *   eta = A1^T (I + J2 C1)^{-1} (eta2 - J2 b1) + eta1
 *   J   = A1^T (I + J2 C1)^{-1} J2 A1 + J1
 * The two inverses are applied by two separate LU solves with partial
 * pivoting.  `out` may not alias the inputs.
 */
int oracle_combine(int n, const double *e1, const double *e2, double *out) {
    const size_t nn = (size_t)n * n;
    const double *A1 = e1, *b1 = e1 + nn, *C1 = e1 + nn + n, *eta1 = e1 + 2 * nn + n, *J1 = e1 + 2 * nn + 2 * n;
    const double *A2 = e2, *b2 = e2 + nn, *C2 = e2 + nn + n, *eta2 = e2 + 2 * nn + n, *J2 = e2 + 2 * nn + 2 * n;
    double *A = out, *b = out + nn, *C = out + nn + n, *eta = out + 2 * nn + n, *J = out + 2 * nn + 2 * n;
    int nrhs = 2 * n + 1;
    double *M = malloc(sizeof(double) * nn);
    double *R = malloc(sizeof(double) * nn * 4 + sizeof(double) * 2 * n);
    double *Y = malloc(sizeof(double) * nn);
    double *t = malloc(sizeof(double) * n);
    double *CA = malloc(sizeof(double) * nn);
    int rc = OR_OK;

    /* Solve (I + C1 J2) [Ya | Yc | yb] = [A1 | C1 A2^T | b1 + C1 eta2]. */
    mm(n, n, n, C1, J2, M);
    for (int i = 0; i < n; ++i) M[i * n + i] += 1.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += C1[i * n + q] * A2[j * n + q];
            CA[i * n + j] = s;
        }
    mv(n, n, C1, eta2, t);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            R[i * nrhs + j] = A1[i * n + j];
            R[i * nrhs + n + j] = CA[i * n + j];
        }
        R[i * nrhs + 2 * n] = b1[i] + t[i];
    }
    rc = lu_solve(n, nrhs, M, R);
    if (rc) goto done;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Y[i * n + j] = R[i * nrhs + j];
    mm(n, n, n, A2, Y, A);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Y[i * n + j] = R[i * nrhs + n + j];
    mm(n, n, n, A2, Y, C);
    for (size_t i = 0; i < nn; ++i) C[i] += C2[i];
    for (int i = 0; i < n; ++i) t[i] = R[i * nrhs + 2 * n];
    mv(n, n, A2, t, b);
    for (int i = 0; i < n; ++i) b[i] += b2[i];

    /* Solve (I + J2 C1) [Zj | ze] = [J2 A1 | eta2 - J2 b1]. */
    int nr2 = n + 1;
    mm(n, n, n, J2, C1, M);
    for (int i = 0; i < n; ++i) M[i * n + i] += 1.0;
    mm(n, n, n, J2, A1, CA);
    mv(n, n, J2, b1, t);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) R[i * nr2 + j] = CA[i * n + j];
        R[i * nr2 + n] = eta2[i] - t[i];
    }
    rc = lu_solve(n, nr2, M, R);
    if (rc) goto done;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Y[i * n + j] = R[i * nr2 + j];
    mtm(n, n, n, A1, Y, J);
    for (size_t i = 0; i < nn; ++i) J[i] += J1[i];
    for (int i = 0; i < n; ++i) t[i] = R[i * nr2 + n];
    mtv(n, n, A1, t, eta);
    for (int i = 0; i < n; ++i) eta[i] += eta1[i];
done:
    free(CA); free(M); free(R); free(Y); free(t);
    return rc;
}

/* ---- total cost of a trajectory, Section II-B --------------------------- */

double oracle_cost(int n, int m, int p, int pT, int64_t T, uint32_t per_step,
                   const double *H, const double *X, const double *U, const double *r,
                   const double *HT, const double *XT, const double *rT,
                   const double *x, const double *u) {
    int q = p > pT ? p : pT;
    double *e = malloc(sizeof(double) * q), *Xe = malloc(sizeof(double) * q);
    double *Uu = malloc(sizeof(double) * m);
    double J = 0.0;
    for (int64_t k = 0; k < T; ++k) {
        const double *Hk = at(H, per_step, PS_H, k, (size_t)p * n);
        const double *Xk = at(X, per_step, PS_X, k, (size_t)p * p);
        const double *Uk = at(U, per_step, PS_U, k, (size_t)m * m);
        mv(p, n, Hk, x + (size_t)k * n, e);
        for (int i = 0; i < p; ++i) e[i] -= r[(size_t)k * p + i];
        mv(p, p, Xk, e, Xe);
        for (int i = 0; i < p; ++i) J += 0.5 * e[i] * Xe[i];
        mv(m, m, Uk, u + (size_t)k * m, Uu);
        for (int i = 0; i < m; ++i) J += 0.5 * u[(size_t)k * m + i] * Uu[i];
    }
    mv(pT, n, HT, x + (size_t)T * n, e);
    for (int i = 0; i < pT; ++i) e[i] -= rT[i];
    mv(pT, pT, XT, e, Xe);
    for (int i = 0; i < pT; ++i) J += 0.5 * e[i] * Xe[i];
    free(e); free(Xe); free(Uu);
    return J;
}
