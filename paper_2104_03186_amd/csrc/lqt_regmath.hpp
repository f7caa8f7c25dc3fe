// Register-resident small dense linear algebra for the LQT scan (gfx950).
//
// Every routine is a fully unrolled template over compile-time sizes, so all
// matrix entries live in VGPRs and every index is a constant: no scratch, no
// dynamic register indexing.  Matrices are row-major; symmetric matrices are
// stored as the packed upper triangle (row i holds columns i..N-1).
#pragma once

#include <hip/hip_runtime.h>

#define LQT_DI __device__ __forceinline__
#define LQT_UNROLL _Pragma("unroll")

namespace lqt {

template <int N>
struct Sym {
    static constexpr int size = N * (N + 1) / 2;
    // Offset of entry (i, j) in the packed upper triangle.
    static constexpr int at(int i, int j) {
        return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
    }
};

// out[R][C] = A[R][K] * B[K][C]
template <int R, int K, int C>
LQT_DI void mm(const double* A, const double* B, double* out) {
    LQT_UNROLL for (int i = 0; i < R; ++i)
    LQT_UNROLL for (int j = 0; j < C; ++j) {
        double s = A[i * K] * B[j];
        LQT_UNROLL for (int k = 1; k < K; ++k) s = fma(A[i * K + k], B[k * C + j], s);
        out[i * C + j] = s;
    }
}

// out[R][C] = A^T B with A stored [K][R], B [K][C]
template <int R, int K, int C>
LQT_DI void mtm(const double* A, const double* B, double* out) {
    LQT_UNROLL for (int i = 0; i < R; ++i)
    LQT_UNROLL for (int j = 0; j < C; ++j) {
        double s = A[i] * B[j];
        LQT_UNROLL for (int k = 1; k < K; ++k) s = fma(A[k * R + i], B[k * C + j], s);
        out[i * C + j] = s;
    }
}

// out[N][C] = S B with S symmetric packed N x N, B [N][C]
template <int N, int C>
LQT_DI void sm(const double* S, const double* B, double* out) {
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < C; ++j) {
        double s = S[Sym<N>::at(i, 0)] * B[j];
        LQT_UNROLL for (int k = 1; k < N; ++k) s = fma(S[Sym<N>::at(i, k)], B[k * C + j], s);
        out[i * C + j] = s;
    }
}

// y[R] = A[R][C] x
template <int R, int C>
LQT_DI void mv(const double* A, const double* x, double* y) {
    LQT_UNROLL for (int i = 0; i < R; ++i) {
        double s = A[i * C] * x[0];
        LQT_UNROLL for (int j = 1; j < C; ++j) s = fma(A[i * C + j], x[j], s);
        y[i] = s;
    }
}

// y[C] = A^T x with A [R][C]
template <int R, int C>
LQT_DI void mtv(const double* A, const double* x, double* y) {
    LQT_UNROLL for (int j = 0; j < C; ++j) {
        double s = A[j] * x[0];
        LQT_UNROLL for (int i = 1; i < R; ++i) s = fma(A[i * C + j], x[i], s);
        y[j] = s;
    }
}

// y[N] = S x, S symmetric packed
template <int N>
LQT_DI void smv(const double* S, const double* x, double* y) {
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = S[Sym<N>::at(i, 0)] * x[0];
        LQT_UNROLL for (int j = 1; j < N; ++j) s = fma(S[Sym<N>::at(i, j)], x[j], s);
        y[i] = s;
    }
}

LQT_DI void cswap(bool c, double& a, double& b) {
    double ta = c ? b : a;
    double tb = c ? a : b;
    a = ta;
    b = tb;
}

// Mi = M^{-1} by Gauss-Jordan elimination with partial pivoting.  The row
// exchanges are conditional swaps with static indices (pivot search by a
// sequence of compare-and-swap), so the matrices stay in registers.  M is
// destroyed.  A singular M yields non-finite entries (caught by the caller's
// finiteness check).
template <int N>
LQT_DI void inv_pivot(double* M, double* Mi) {
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) Mi[i * N + j] = (i == j) ? 1.0 : 0.0;
    LQT_UNROLL for (int k = 0; k < N; ++k) {
        LQT_UNROLL for (int i = k + 1; i < N; ++i) {
            const bool sw = fabs(M[i * N + k]) > fabs(M[k * N + k]);
            LQT_UNROLL for (int j = k; j < N; ++j) cswap(sw, M[k * N + j], M[i * N + j]);
            LQT_UNROLL for (int j = 0; j < N; ++j) cswap(sw, Mi[k * N + j], Mi[i * N + j]);
        }
        const double p = 1.0 / M[k * N + k];
        LQT_UNROLL for (int j = k + 1; j < N; ++j) M[k * N + j] *= p;
        LQT_UNROLL for (int j = 0; j < N; ++j) Mi[k * N + j] *= p;
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            if (i == k) continue;
            const double f = M[i * N + k];
            LQT_UNROLL for (int j = k + 1; j < N; ++j) M[i * N + j] = fma(-f, M[k * N + j], M[i * N + j]);
            LQT_UNROLL for (int j = 0; j < N; ++j) Mi[i * N + j] = fma(-f, Mi[k * N + j], Mi[i * N + j]);
        }
    }
}

// In-place lower Cholesky factor of an M x M SPD matrix given as packed
// upper triangle W; R (full [M][M], lower) receives the factor and rinv the
// reciprocals of its diagonal.  Returns false when a pivot is not > 0
// (including NaN).
template <int M>
LQT_DI bool chol(const double* W, double* R, double* rinv) {
    bool ok = true;
    LQT_UNROLL for (int j = 0; j < M; ++j) {
        double s = W[Sym<M>::at(j, j)];
        LQT_UNROLL for (int k = 0; k < j; ++k) s = fma(-R[j * M + k], R[j * M + k], s);
        ok = ok && (s > 0.0);
        const double rjj = sqrt(s);
        const double ri = 1.0 / rjj;
        R[j * M + j] = rjj;
        rinv[j] = ri;
        LQT_UNROLL for (int i = j + 1; i < M; ++i) {
            double t = W[Sym<M>::at(j, i)];
            LQT_UNROLL for (int k = 0; k < j; ++k) t = fma(-R[i * M + k], R[j * M + k], t);
            R[i * M + j] = t * ri;
        }
        LQT_UNROLL for (int i = 0; i < j; ++i) R[i * M + j] = 0.0;
    }
    return ok;
}

// B[M][C] <- R^{-1} B  (R lower, forward substitution)
template <int M, int C>
LQT_DI void lsolve(const double* R, const double* rinv, double* B) {
    LQT_UNROLL for (int i = 0; i < M; ++i)
    LQT_UNROLL for (int c = 0; c < C; ++c) {
        double s = B[i * C + c];
        LQT_UNROLL for (int k = 0; k < i; ++k) s = fma(-R[i * M + k], B[k * C + c], s);
        B[i * C + c] = s * rinv[i];
    }
}

// B[M][C] <- R^{-T} B  (back substitution with the transpose of lower R)
template <int M, int C>
LQT_DI void ltsolve(const double* R, const double* rinv, double* B) {
    LQT_UNROLL for (int i = M - 1; i >= 0; --i)
    LQT_UNROLL for (int c = 0; c < C; ++c) {
        double s = B[i * C + c];
        LQT_UNROLL for (int k = i + 1; k < M; ++k) s = fma(-R[k * M + i], B[k * C + c], s);
        B[i * C + c] = s * rinv[i];
    }
}

}  // namespace lqt
