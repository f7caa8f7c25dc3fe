// LQT scan elements and operators in registers (lane-per-element form).
//
// Element (A, b, C, eta, J): parameters of the dual form of the conditional
// value function V_{k->i}(x_k, x_i), Section IV-A of Sarkka & Garcia-Fernandez
// (arXiv 2104.03186).  C and J are symmetric and kept as packed upper
// triangles, so every combined C and J is exactly symmetric.
#pragma once

#include "lqt_regmath.hpp"

namespace lqt {

template <int N>
struct Elem {
    static constexpr int NS = Sym<N>::size;
    static constexpr int size = N * N + N + NS + N + NS;  // doubles in memory
    double A[N * N];
    double b[N];
    double C[NS];
    double e[N];  // eta
    double J[NS];
};

template <int N>
LQT_DI void set_identity(Elem<N>& x) {
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        LQT_UNROLL for (int j = 0; j < N; ++j) x.A[i * N + j] = (i == j) ? 1.0 : 0.0;
        x.b[i] = 0.0;
        x.e[i] = 0.0;
    }
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) {
        x.C[i] = 0.0;
        x.J[i] = 0.0;
    }
}

template <int N>
LQT_DI void store_elem(double* p, const Elem<N>& x) {
    int o = 0;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) p[o++] = x.A[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) p[o++] = x.b[i];
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) p[o++] = x.C[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) p[o++] = x.e[i];
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) p[o++] = x.J[i];
}

template <int N>
LQT_DI void load_elem(const double* p, Elem<N>& x) {
    int o = 0;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) x.A[i] = p[o++];
    LQT_UNROLL for (int i = 0; i < N; ++i) x.b[i] = p[o++];
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) x.C[i] = p[o++];
    LQT_UNROLL for (int i = 0; i < N; ++i) x.e[i] = p[o++];
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) x.J[i] = p[o++];
}

template <int N>
LQT_DI Elem<N> shfl_up_elem(const Elem<N>& x, int d) {
    Elem<N> y;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.A[i] = __shfl_up(x.A[i], d, 64);
    LQT_UNROLL for (int i = 0; i < N; ++i) y.b[i] = __shfl_up(x.b[i], d, 64);
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) y.C[i] = __shfl_up(x.C[i], d, 64);
    LQT_UNROLL for (int i = 0; i < N; ++i) y.e[i] = __shfl_up(x.e[i], d, 64);
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) y.J[i] = __shfl_up(x.J[i], d, 64);
    return y;
}

template <int N>
LQT_DI Elem<N> shfl_down_elem(const Elem<N>& x, int d) {
    Elem<N> y;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.A[i] = __shfl_down(x.A[i], d, 64);
    LQT_UNROLL for (int i = 0; i < N; ++i) y.b[i] = __shfl_down(x.b[i], d, 64);
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) y.C[i] = __shfl_down(x.C[i], d, 64);
    LQT_UNROLL for (int i = 0; i < N; ++i) y.e[i] = __shfl_down(x.e[i], d, 64);
    LQT_UNROLL for (int i = 0; i < Elem<N>::NS; ++i) y.J[i] = __shfl_down(x.J[i], d, 64);
    return y;
}

// y <- x (x) y, with x the earlier element (k->j) and y the later (j->i).
// Combination rule of Section IV-A:
//   A = A_y M^{-1} A_x,  b = A_y M^{-1}(b_x + C_x eta_y) + b_y,
//   C = A_y M^{-1} C_x A_y^T + C_y,
//   eta = A_x^T M^{-T}(eta_y - J_y b_x) + eta_x,  J = A_x^T M^{-T} J_y A_x + J_x,
// with M = I + C_x J_y.  Since C_x and J_y are symmetric,
// (I + J_y C_x)^{-1} = M^{-T}, so A_x^T M^{-T} = (M^{-1} A_x)^T and one
// pivoted inverse serves all five updates.
template <int N>
LQT_DI void combine(const Elem<N>& x, Elem<N>& y) {
    using S = Sym<N>;
    double Mm[N * N], Mi[N * N];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = (i == j) ? 1.0 : 0.0;
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(x.C[S::at(i, k)], y.J[S::at(k, j)], s);
        Mm[i * N + j] = s;
    }
    inv_pivot<N>(Mm, Mi);

    double T1[N * N];  // M^{-1} A_x
    mm<N, N, N>(Mi, x.A, T1);

    double t[N], t2[N], nb[N];
    smv<N>(x.C, y.e, t);
    LQT_UNROLL for (int i = 0; i < N; ++i) t[i] += x.b[i];
    mv<N, N>(Mi, t, t2);
    mv<N, N>(y.A, t2, nb);
    LQT_UNROLL for (int i = 0; i < N; ++i) nb[i] += y.b[i];

    double Q[N * N], R[N * N], nC[S::size];
    LQT_UNROLL for (int i = 0; i < N; ++i)  // Q = M^{-1} C_x
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = Mi[i * N] * x.C[S::at(0, j)];
        LQT_UNROLL for (int k = 1; k < N; ++k) s = fma(Mi[i * N + k], x.C[S::at(k, j)], s);
        Q[i * N + j] = s;
    }
    mm<N, N, N>(y.A, Q, R);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = y.C[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(R[i * N + k], y.A[j * N + k], s);
        nC[S::at(i, j)] = s;
    }

    double nA[N * N];
    mm<N, N, N>(y.A, T1, nA);

    double ne[N];
    smv<N>(y.J, x.b, t);
    LQT_UNROLL for (int i = 0; i < N; ++i) t[i] = y.e[i] - t[i];
    mtv<N, N>(T1, t, ne);
    LQT_UNROLL for (int i = 0; i < N; ++i) ne[i] += x.e[i];

    double P[N * N], nJ[S::size];
    sm<N, N>(y.J, x.A, P);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = x.J[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(T1[k * N + i], P[k * N + j], s);
        nJ[S::at(i, j)] = s;
    }

    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.A[i] = nA[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        y.b[i] = nb[i];
        y.e[i] = ne[i];
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) {
        y.C[i] = nC[i];
        y.J[i] = nJ[i];
    }
}

// Constant per-step data of a one-step element a_k (Section IV-B):
// A = F_k, b = c_k, C = L_k U_k^{-1} L_k^T = G G^T with G = L_k R_U^{-T}
// (U_k = R_U R_U^T), eta = H_k^T X_k r_k, J = H_k^T X_k H_k.
template <int N, int M>
struct Step {
    double F[N * N];
    double c[N];
    double G[N * M];
    double e[N];
    double J[Sym<N>::size];
};

// y <- a_k (x) y for a one-step element a_k.  The same combination rule as
// `combine`, with (I + C_k J_y)^{-1} expanded by the matrix inversion lemma
// through the factor C_k = G G^T (the identity used in the paper's appendix
// proof that the element fold reproduces the Riccati recursion):
//   W = I + G^T J_y G = R R^T,  Y = R^{-1} G^T J_y,  Gt = G R^{-T},
//   M^{-1} = I - Gt Y,  M^{-1} C_k = Gt Gt^T,  M^{-T} J_y = J_y - Y^T Y.
// Only an m x m Cholesky is needed; W >= I, so it cannot fail for finite y.
template <int N, int M>
LQT_DI void step_combine(const Step<N, M>& a, Elem<N>& y) {
    using S = Sym<N>;
    using SM = Sym<M>;
    double Z[M * N];  // G^T J_y
    LQT_UNROLL for (int p = 0; p < M; ++p)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = a.G[p] * y.J[S::at(0, j)];
        LQT_UNROLL for (int i = 1; i < N; ++i) s = fma(a.G[i * M + p], y.J[S::at(i, j)], s);
        Z[p * N + j] = s;
    }
    double W[SM::size], R[M * M], rinv[M];
    LQT_UNROLL for (int p = 0; p < M; ++p)
    LQT_UNROLL for (int q = p; q < M; ++q) {
        double s = (p == q) ? 1.0 : 0.0;
        LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(Z[p * N + j], a.G[j * M + q], s);
        W[SM::at(p, q)] = s;
    }
    chol<M>(W, R, rinv);
    double Y[M * N], GtT[M * N];
    LQT_UNROLL for (int i = 0; i < M * N; ++i) Y[i] = Z[i];
    lsolve<M, N>(R, rinv, Y);
    LQT_UNROLL for (int p = 0; p < M; ++p)
    LQT_UNROLL for (int i = 0; i < N; ++i) GtT[p * N + i] = a.G[i * M + p];
    lsolve<M, N>(R, rinv, GtT);

    double V[N * M];  // A_y Gt
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int p = 0; p < M; ++p) {
        double s = y.A[i * N] * GtT[p * N];
        LQT_UNROLL for (int k = 1; k < N; ++k) s = fma(y.A[i * N + k], GtT[p * N + k], s);
        V[i * M + p] = s;
    }
    double nC[S::size];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = y.C[S::at(i, j)];
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(V[i * M + p], V[j * M + p], s);
        nC[S::at(i, j)] = s;
    }
    double YF[M * N], nA[N * N], AF[N * N];
    mm<M, N, N>(Y, a.F, YF);
    mm<N, N, N>(y.A, a.F, AF);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = AF[i * N + j];
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-V[i * M + p], YF[p * N + j], s);
        nA[i * N + j] = s;
    }
    double q[M], Yc[M], g2[N], nb[N];
    mv<M, N>(GtT, y.e, q);
    mv<M, N>(Y, a.c, Yc);
    LQT_UNROLL for (int p = 0; p < M; ++p) q[p] -= Yc[p];
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = a.c[i];
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(GtT[p * N + i], q[p], s);
        g2[i] = s;
    }
    mv<N, N>(y.A, g2, nb);
    LQT_UNROLL for (int i = 0; i < N; ++i) nb[i] += y.b[i];

    double w[N], Jc[N], ne[N];
    smv<N>(y.J, a.c, Jc);
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = y.e[i] - Jc[i];
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-Y[p * N + i], q[p], s);
        w[i] = s;
    }
    mtv<N, N>(a.F, w, ne);
    LQT_UNROLL for (int i = 0; i < N; ++i) ne[i] += a.e[i];

    double Qm[S::size], QF[N * N], nJ[S::size];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = y.J[S::at(i, j)];
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-Y[p * N + i], Y[p * N + j], s);
        Qm[S::at(i, j)] = s;
    }
    sm<N, N>(Qm, a.F, QF);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = a.J[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(a.F[k * N + i], QF[k * N + j], s);
        nJ[S::at(i, j)] = s;
    }

    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.A[i] = nA[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        y.b[i] = nb[i];
        y.e[i] = ne[i];
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) {
        y.C[i] = nC[i];
        y.J[i] = nJ[i];
    }
}

// The one-step element itself (used to seed a fold).
template <int N, int M>
LQT_DI void step_elem(const Step<N, M>& a, Elem<N>& y) {
    using S = Sym<N>;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.A[i] = a.F[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        y.b[i] = a.c[i];
        y.e[i] = a.e[i];
    }
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = a.G[i * M] * a.G[j * M];
        LQT_UNROLL for (int p = 1; p < M; ++p) s = fma(a.G[i * M + p], a.G[j * M + p], s);
        y.C[S::at(i, j)] = s;
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) y.J[i] = a.J[i];
}

// Value function (S, v) <- x (x) (0, 0, 0, v, S): the combination rule with a
// right operand whose A, b, C vanish (a suffix that contains the terminal
// element, Section IV-B), which keeps A = b = C = 0 and gives
//   S' = A_x^T M^{-T} S A_x + J_x,  v' = A_x^T M^{-T}(v - S b_x) + eta_x,
// M = I + C_x S.
template <int N>
LQT_DI void anchor(const Elem<N>& x, double* Sv, double* v) {
    using S = Sym<N>;
    double Mm[N * N], Mi[N * N];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = (i == j) ? 1.0 : 0.0;
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(x.C[S::at(i, k)], Sv[S::at(k, j)], s);
        Mm[i * N + j] = s;
    }
    inv_pivot<N>(Mm, Mi);
    double T1[N * N];
    mm<N, N, N>(Mi, x.A, T1);
    double t[N], nv[N];
    smv<N>(Sv, x.b, t);
    LQT_UNROLL for (int i = 0; i < N; ++i) t[i] = v[i] - t[i];
    mtv<N, N>(T1, t, nv);
    double P[N * N], nS[S::size];
    sm<N, N>(Sv, x.A, P);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = x.J[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(T1[k * N + i], P[k * N + j], s);
        nS[S::at(i, j)] = s;
    }
    LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = nv[i] + x.e[i];
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = nS[i];
}

// Forward prefix from a fixed initial state (Method 2 of Section IV-C): the
// conditional value function V_{0->k} initialised with the element
// (0, x_0, 0, 0, 0) keeps A = eta = J = 0 under every later combination, so
// it is carried as (b, C).  (b, C) <- (0, b, C, 0, 0) (x) e is the
// combination rule with that left operand:
//   M = I + C J_e,  b' = A_e M^{-1}(b + C eta_e) + b_e,
//   C' = A_e M^{-1} C A_e^T + C_e.
template <int N>
LQT_DI void fanchor(const Elem<N>& e, double* b, double* Cs) {
    using S = Sym<N>;
    double Mm[N * N], Mi[N * N];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = (i == j) ? 1.0 : 0.0;
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(Cs[S::at(i, k)], e.J[S::at(k, j)], s);
        Mm[i * N + j] = s;
    }
    inv_pivot<N>(Mm, Mi);
    double t[N], t2[N], nb[N];
    smv<N>(Cs, e.e, t);
    LQT_UNROLL for (int i = 0; i < N; ++i) t[i] += b[i];
    mv<N, N>(Mi, t, t2);
    mv<N, N>(e.A, t2, nb);
    double Q[N * N], R[N * N];
    LQT_UNROLL for (int i = 0; i < N; ++i)  // Q = M^{-1} C
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = Mi[i * N] * Cs[S::at(0, j)];
        LQT_UNROLL for (int k = 1; k < N; ++k) s = fma(Mi[i * N + k], Cs[S::at(k, j)], s);
        Q[i * N + j] = s;
    }
    mm<N, N, N>(e.A, Q, R);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = e.C[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(R[i * N + k], e.A[j * N + k], s);
        Cs[S::at(i, j)] = s;
    }
    LQT_UNROLL for (int i = 0; i < N; ++i) b[i] = nb[i] + e.b[i];
}

// Optimal state from the forward prefix (b, C) and the value function
// (S_k full, v_k) at the same step (lemma on Method 2 of Section IV-C):
// x_k = (I + C S_k)^{-1}(b + C v_k).
template <int N>
LQT_DI void prefix_state(const double* b, const double* Cs, const double* Sk, const double* vk, double* x) {
    using S = Sym<N>;
    double Mm[N * N], Mi[N * N], t[N];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) {
        double s = (i == j) ? 1.0 : 0.0;
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(Cs[S::at(i, k)], Sk[k * N + j], s);
        Mm[i * N + j] = s;
    }
    inv_pivot<N>(Mm, Mi);
    smv<N>(Cs, vk, t);
    LQT_UNROLL for (int i = 0; i < N; ++i) t[i] += b[i];
    mv<N, N>(Mi, t, x);
}

// One down-sweep application a_k (x) (0, 0, 0, v_{k+1}, S_{k+1}) written in
// the matrix-inversion-lemma form that the paper's appendix proves equal to
// the Riccati recursion, fused with the control-law extraction of
// Section II-B (the same m x m factorisation serves both):
//   M_k = L^T S L + U = R R^T,  K = M_k^{-1} L^T S F,
//   d = M_k^{-1} L^T (v - S c),
//   S' = F^T S F - (R^{-1} L^T S F)^T (R^{-1} L^T S F) + H^T X H,
//   v' = F^T (v - S c) - K^T L^T (v - S c) + H^T X r.
// Also returns the closed-loop map Ft = F - L K, ct = c + L d (Section IV-C).
// Returns false when M_k is not positive definite.  HASC = false: c = 0
// (c is not read).
template <int N, int M, bool HASC = true>
LQT_DI bool riccati_step(const double* F, const double* c, const double* L, const double* Uu,
                         const double* Js, const double* ek, double* Sv, double* v,
                         double* K, double* d, double* Ft, double* ct) {
    using S = Sym<N>;
    using SM = Sym<M>;
    double SL[N * M];
    sm<N, M>(Sv, L, SL);
    double W[SM::size], R[M * M], rinv[M];
    LQT_UNROLL for (int p = 0; p < M; ++p)
    LQT_UNROLL for (int q = p; q < M; ++q) {
        double s = Uu[p * M + q];
        LQT_UNROLL for (int i = 0; i < N; ++i) s = fma(L[i * M + p], SL[i * M + q], s);
        W[SM::at(p, q)] = s;
    }
    const bool ok = chol<M>(W, R, rinv);
    double SF[N * N], Y[M * N];
    sm<N, N>(Sv, F, SF);
    mtm<M, N, N>(L, SF, Y);
    lsolve<M, N>(R, rinv, Y);
    LQT_UNROLL for (int i = 0; i < M * N; ++i) K[i] = Y[i];
    ltsolve<M, N>(R, rinv, K);
    double w[N], z[M];
    if constexpr (HASC) {
        double Sc[N];
        smv<N>(Sv, c, Sc);
        LQT_UNROLL for (int i = 0; i < N; ++i) w[i] = v[i] - Sc[i];
    } else {
        LQT_UNROLL for (int i = 0; i < N; ++i) w[i] = v[i];
    }
    mtv<N, M>(L, w, z);
    LQT_UNROLL for (int p = 0; p < M; ++p) d[p] = z[p];
    lsolve<M, 1>(R, rinv, d);
    ltsolve<M, 1>(R, rinv, d);
    double nS[S::size], nv[N];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = Js[S::at(i, j)];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(F[k * N + i], SF[k * N + j], s);
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-Y[p * N + i], Y[p * N + j], s);
        nS[S::at(i, j)] = s;
    }
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = ek[i];
        LQT_UNROLL for (int k = 0; k < N; ++k) s = fma(F[k * N + i], w[k], s);
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-K[p * N + i], z[p], s);
        nv[i] = s;
    }
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        LQT_UNROLL for (int j = 0; j < N; ++j) {
            double s = F[i * N + j];
            LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(-L[i * M + p], K[p * N + j], s);
            Ft[i * N + j] = s;
        }
        double s = HASC ? c[i] : 0.0;
        LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(L[i * M + p], d[p], s);
        ct[i] = s;
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = nS[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = nv[i];
    return ok;
}

// Affine map x -> F x + c (element of the forward scan, Section IV-C).
template <int N>
struct Aff {
    static constexpr int size = N * N + N;
    double F[N * N];
    double c[N];
};

template <int N>
LQT_DI void aff_identity(Aff<N>& a) {
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        LQT_UNROLL for (int j = 0; j < N; ++j) a.F[i * N + j] = (i == j) ? 1.0 : 0.0;
        a.c[i] = 0.0;
    }
}

// late <- late o early: F = F_l F_e, c = F_l c_e + c_l (trajectory combination
// rule of Section IV-C; the earlier map is applied first).
template <int N>
LQT_DI void aff_after(const Aff<N>& early, Aff<N>& late) {
    double nF[N * N], nc[N];
    mm<N, N, N>(late.F, early.F, nF);
    mv<N, N>(late.F, early.c, nc);
    LQT_UNROLL for (int i = 0; i < N * N; ++i) late.F[i] = nF[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) late.c[i] += nc[i];
}

template <int N>
LQT_DI void store_aff(double* p, const Aff<N>& a) {
    LQT_UNROLL for (int i = 0; i < N * N; ++i) p[i] = a.F[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) p[N * N + i] = a.c[i];
}

template <int N>
LQT_DI void load_aff(const double* p, Aff<N>& a) {
    LQT_UNROLL for (int i = 0; i < N * N; ++i) a.F[i] = p[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) a.c[i] = p[N * N + i];
}

template <int N>
LQT_DI Aff<N> shfl_up_aff(const Aff<N>& a, int d) {
    Aff<N> y;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) y.F[i] = __shfl_up(a.F[i], d, 64);
    LQT_UNROLL for (int i = 0; i < N; ++i) y.c[i] = __shfl_up(a.c[i], d, 64);
    return y;
}

}  // namespace lqt
