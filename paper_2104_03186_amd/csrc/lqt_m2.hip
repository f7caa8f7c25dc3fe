// Trajectory by forward prefixes (Method 2 of Section IV-C) on the chunked
// engines (wavefront engine, classes 8/16/32; workgroup engines, classes
// 16/32/64).  The backward pass of the engine has left, for every chunk
// c >= 1, its element E_c = a_k0 (x) ... (x) a_k1-1 (the same product the
// forward scan needs) and the values S_k, v_k and gains K_k, d_k of every step.
//
// The forward prefix from the known start is V_{0->k} = i (x) a_0 (x) ... (x)
// a_{k-1} with the initial-state element i = (0, x_0, 0, 0, 0) (the remark on
// a known start in Section IV-B).  Under the combination rule of Section IV-A
// a left operand of the form (0, b, C, 0, 0) stays of that form:
//   (0, b, C, 0, 0) (x) (A, b_E, C_E, eta_E, J_E) = (0, b', C', 0, 0),
//   b' = A M^{-1} (b + C eta_E) + b_E,   C' = A M^{-1} C A^T + C_E,
//   M = I + C J_E,
// so a prefix is carried as (b, C).  Then (lemma on Method 2, Section IV-C)
//   x_k = (I + C_{0,k} S_k)^{-1} (b_{0,k} + C_{0,k} v_k),  u_k = -K_k x_k + d_k.
//
// m2c_chain (one workgroup per instance): the prefix at every chunk start --
// chunk 0 walked step by step from i, then one combination with each chunk
// element; stored over the chunk-map records of the workspace.  m2c_walk
// (one workgroup per chunk): from the chunk's start prefix, per step x_k, u_k
// and the prefix advanced by the step's element.  Every linear system is
// solved by Gaussian elimination with partial pivoting (M and I + C S_k have
// eigenvalues >= 1 for C, J_E, S_k positive semi-definite).  Inputs and
// outputs are double (a plan with float results solves these instances with
// double results in scratch and rounds them afterwards).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_ws.hpp"

namespace lqt {

namespace {

constexpr int kM2T = 256;  // threads per workgroup

#define MDI __device__ __forceinline__

MDI void msync() { __syncthreads(); }

// Sources of one element in global or LDS memory (row-major with the given
// leading dimensions).  One-step elements give C_E through its factor G
// (C_E = G G^T, n x mg); chunk elements give C_E itself.
struct ElemView {
    const double* A;
    int lda;
    const double* b;  // may be null (zero)
    const double* C;  // C_E, or its factor G
    int ldc;
    int mg;           // > 0: C holds the n x mg factor G
    const double* eta;
    const double* J;
    int ldj;
};

// Gaussian elimination with partial pivoting of the n x n matrix Mm (LDS,
// leading dimension ld; destroyed), applied to the ny columns of Y (LDS,
// leading dimension ld) and, when given, the vector rhs: on return Y holds
// M^{-1} Y and rhs holds M^{-1} rhs.
MDI void lu_solve(int n, double* Mm, int ld, double* Y, int ny, double* rhs, int* piv) {
    const int t = threadIdx.x;
#pragma unroll 1
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            int p = j;
            double best = fabs(Mm[j * ld + j]);
            for (int i = j + 1; i < n; ++i) {
                const double a = fabs(Mm[i * ld + j]);
                if (a > best) {
                    best = a;
                    p = i;
                }
            }
            *piv = p;
        }
        msync();
        const int p = *piv;
        if (p != j) {
            for (int q = t; q < n + ny + 1; q += kM2T) {
                if (q < n) {
                    const double x = Mm[j * ld + q];
                    Mm[j * ld + q] = Mm[p * ld + q];
                    Mm[p * ld + q] = x;
                } else if (q < n + ny) {
                    const double x = Y[j * ld + q - n];
                    Y[j * ld + q - n] = Y[p * ld + q - n];
                    Y[p * ld + q - n] = x;
                } else if (rhs) {
                    const double x = rhs[j];
                    rhs[j] = rhs[p];
                    rhs[p] = x;
                }
            }
            msync();
        }
        const double inv = 1.0 / Mm[j * ld + j];
        for (int i = j + 1 + t; i < n; i += kM2T) Mm[i * ld + j] *= inv;
        msync();
        const int rows = n - j - 1, tail = n - j - 1, cols = tail + ny + 1;
        for (int idx = t; idx < rows * cols; idx += kM2T) {
            const int i = j + 1 + idx / cols, q = idx - (idx / cols) * cols;
            const double l = Mm[i * ld + j];
            if (q < tail) Mm[i * ld + j + 1 + q] = fma(-l, Mm[j * ld + j + 1 + q], Mm[i * ld + j + 1 + q]);
            else if (q < tail + ny) Y[i * ld + q - tail] = fma(-l, Y[j * ld + q - tail], Y[i * ld + q - tail]);
            else if (rhs) rhs[i] = fma(-l, rhs[j], rhs[i]);
        }
        msync();
    }
    // back substitution, one thread per column
    for (int c = t; c < ny + 1; c += kM2T) {
        if (c == ny && !rhs) continue;
        double* col = c < ny ? Y + c : rhs;
        const int cs = c < ny ? ld : 1;
#pragma unroll 1
        for (int j = n - 1; j >= 0; --j) {
            double s = col[j * cs];
            for (int q = j + 1; q < n; ++q) s = fma(-Mm[j * ld + q], col[q * cs], s);
            col[j * cs] = s / Mm[j * ld + j];
        }
    }
    msync();
}

// (b, C) <- (0, b, C, 0, 0) (x) E.  Cm, b: the prefix (LDS, leading
// dimension ld); Mm, Y: n x n LDS work matrices; tv: n-vector; piv: LDS int.
MDI void fwd_combine(int n, double* Cm, double* b, const ElemView& E, double* Mm, double* Y, double* tv, int ld,
                     int* piv) {
    const int t = threadIdx.x;
    // M = I + C J_E ; Y = C ; tv = b + C eta_E
    for (int idx = t; idx < n * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double s = (i == j) ? 1.0 : 0.0;
        for (int q = 0; q < n; ++q) s = fma(Cm[i * ld + q], E.J[q * E.ldj + j], s);
        Mm[i * ld + j] = s;
        Y[i * ld + j] = Cm[i * ld + j];
    }
    for (int i = t; i < n; i += kM2T) {
        double s = b[i];
        for (int q = 0; q < n; ++q) s = fma(Cm[i * ld + q], E.eta[q], s);
        tv[i] = s;
    }
    msync();
    lu_solve(n, Mm, ld, Y, n, tv, piv);  // Y = M^{-1} C, tv = M^{-1} (b + C eta_E)
    // Mm := A Y ; b' = A tv + b_E
    for (int idx = t; idx < n * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double s = 0.0;
        for (int q = 0; q < n; ++q) s = fma(E.A[i * E.lda + q], Y[q * ld + j], s);
        Mm[i * ld + j] = s;
    }
    for (int i = t; i < n; i += kM2T) {
        double s = E.b ? E.b[i] : 0.0;
        for (int q = 0; q < n; ++q) s = fma(E.A[i * E.lda + q], tv[q], s);
        b[i] = s;
    }
    msync();
    // C' = (A Y) A^T + C_E, symmetrised
    for (int idx = t; idx < n * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        if (j < i) continue;
        double sij = 0.0, sji = 0.0;
        for (int q = 0; q < n; ++q) {
            sij = fma(Mm[i * ld + q], E.A[j * E.lda + q], sij);
            sji = fma(Mm[j * ld + q], E.A[i * E.lda + q], sji);
        }
        double ce = 0.0;
        if (E.mg > 0) {
            for (int a = 0; a < E.mg; ++a) ce = fma(E.C[i * E.ldc + a], E.C[j * E.ldc + a], ce);
        } else {
            ce = 0.5 * (E.C[i * E.ldc + j] + E.C[j * E.ldc + i]);
        }
        const double v = 0.5 * (sij + sji) + ce;
        Cm[i * ld + j] = v;
        Cm[j * ld + i] = v;
    }
    msync();
}

// Constants of an instance and, for a time-varying one, the LDS buffers that
// receive G_k, J_k of a step.
struct StepCtx {
    const GInst* I;
    int n, m, p;
    int D;            // record dimension of the workspace (n, or the padded engine dimension)
    const double* G;  // invariant factor G (n x m), leading dimension ldg
    int ldg;
    const double* J;  // invariant J (n x n), leading dimension ldj
    int ldj;
    const double* W;  // invariant W = H^T X (n x p), leading dimension ldw
    int ldw;
    const double* F;  // invariant F (workgroup engines: the padded copy in the constants)
    int ldf;
    bool var;         // L, U, H or X per step (wavefront engine only)
    double *Gs, *Js;  // LDS (var)
    int ld;
};

MDI StepCtx step_ctx(const GInst& I, double* Gs, double* Js, int ld) {
    StepCtx s;
    s.I = &I;
    s.n = I.n;
    s.m = I.m;
    s.p = I.p;
    s.D = ws_dim(I.n, I.eng);
    s.var = (I.per_step & (kPS_L | kPS_U | kPS_H | kPS_X)) != 0;
    s.Gs = Gs;
    s.Js = Js;
    s.ld = ld;
    const InstWs ws = inst_ws(I);
    if (I.eng == 0) {
        const CstW cl = cst_layout(I.n, I.m, I.p);
        s.G = ws.cst + cl.G;
        s.ldg = I.m;
        s.J = ws.cst + cl.J;
        s.ldj = I.n;
        s.W = ws.cst + cl.W;
        s.ldw = I.p;
        s.F = I.F;
        s.ldf = I.n;
    } else {
        const int D = eng_dim(I.eng), Mc = I.eng == 64 ? 32 : (I.eng == kEng32m16 ? 16 : D);
        const int64_t oL = (int64_t)D * D, oG = oL + (int64_t)D * Mc, oU = oG + (int64_t)D * Mc;
        const int64_t oJ = oU + (int64_t)Mc * Mc, oW = oJ + (int64_t)D * D;
        s.G = ws.cst + oG;
        s.ldg = Mc;
        s.J = ws.cst + oJ;
        s.ldj = D;
        s.W = ws.cst + oW;
        s.ldw = D;
        s.F = ws.cst;  // time-invariant F (only c varies on these engines)
        s.ldf = D;
    }
    return s;
}

// The one-step element a_k = (F_k, c_k, G_k G_k^T, eta_k = H_k^T X_k r_k,
// J_k = H_k^T X_k H_k).  eta (LDS n-vector) receives eta_k; for a
// time-varying step G_k, J_k are formed in the context's LDS buffers (tmp:
// an LDS work matrix, piv: LDS int).
MDI ElemView step_elem(const StepCtx& s, int64_t k, double* eta, double* tmp, int* piv) {
    const GInst& I = *s.I;
    const int n = s.n, m = s.m, p = s.p, ld = s.ld, t = threadIdx.x;
    ElemView E;
    const uint32_t ps = I.per_step;
    E.A = (I.eng == 0) ? step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n) : s.F;
    E.lda = s.ldf;
    E.b = I.c ? step_ptr(I.c, ps, kPS_c, k, n) : nullptr;
    const double* rk = I.r + k * p;
    if (!s.var) {
        for (int i = t; i < n; i += kM2T) {
            double a = 0.0;
            for (int j = 0; j < p; ++j) a = fma(s.W[i * s.ldw + j], rk[j], a);
            eta[i] = a;
        }
        E.C = s.G;
        E.ldc = s.ldg;
        E.mg = m;
        E.J = s.J;
        E.ldj = s.ldj;
        E.eta = eta;
        msync();
        return E;
    }
    // time-varying step (wavefront engine, n, m, p <= 32)
    const double* L = step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m);
    const double* U = step_ptr(I.U, ps, kPS_U, k, (int64_t)m * m);
    const double* H = step_ptr(I.H, ps, kPS_H, k, (int64_t)p * n);
    const double* X = step_ptr(I.X, ps, kPS_X, k, (int64_t)p * p);
    // C_E = L_k U_k^{-1} L_k^T formed directly (mg = 0): Gs := U_k^{-1} L_k^T
    // by one solve, then C_E = L_k Gs
    for (int idx = t; idx < m * m; idx += kM2T) {
        const int i = idx / m, j = idx - (idx / m) * m;
        tmp[i * ld + j] = 0.5 * (U[i * m + j] + U[j * m + i]);
    }
    for (int idx = t; idx < m * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        s.Gs[i * ld + j] = L[j * m + i];  // L^T
    }
    msync();
    lu_solve(m, tmp, ld, s.Gs, n, nullptr, piv);  // Gs = U^{-1} L^T (m x n)
    // J_k = H^T X H and eta_k = H^T X r_k: tmp := X H (p x n) first
    for (int idx = t; idx < p * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double a = 0.0;
        for (int q = 0; q < p; ++q) a = fma(X[i * p + q], H[q * n + j], a);
        tmp[i * ld + j] = a;
    }
    msync();
    for (int idx = t; idx < n * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double a = 0.0;
        for (int q = 0; q < p; ++q) a = fma(H[q * n + i], tmp[q * ld + j], a);
        s.Js[i * ld + j] = a;
    }
    for (int i = t; i < n; i += kM2T) {  // eta = (X H)^T r: X symmetric
        double a = 0.0;
        for (int q = 0; q < p; ++q) a = fma(tmp[q * ld + i], rk[q], a);
        eta[i] = a;
    }
    msync();
    // C_E = L (U^{-1} L^T) into tmp (n x n)
    for (int idx = t; idx < n * n; idx += kM2T) {
        const int i = idx / n, j = idx - (idx / n) * n;
        double a = 0.0;
        for (int q = 0; q < m; ++q) a = fma(L[i * m + q], s.Gs[q * ld + j], a);
        tmp[i * ld + j] = a;
    }
    msync();
    E.C = tmp;
    E.ldc = ld;
    E.mg = 0;
    E.J = s.Js;
    E.ldj = ld;
    E.eta = eta;
    return E;
}

// First and one-past-last step of chunk c (the workgroup engines align their
// chunks to the end of the horizon).
MDI void m2_span(const GInst& I, int64_t c, int64_t& k0, int64_t& k1) {
    if (I.eng == 0) {
        k0 = c * I.B;
        k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    } else {
        k1 = I.T - (I.NC - 1 - c) * (int64_t)I.B;
        k0 = k1 - I.B > 0 ? k1 - I.B : 0;
    }
}

template <int N>
struct M2L {
    static constexpr int ld = N + 1;
    static constexpr int mat = N * ld;
    // Cm, Mm, Y [, Gs, Js, tmp: time-varying steps, N <= 32] + 4 vectors
    static constexpr int mats = N <= 32 ? 6 : 3;
    static constexpr size_t bytes = sizeof(double) * (mats * mat + 4 * (N + 2)) + 64;
};

template <int N>
__global__ __launch_bounds__(kM2T) void m2c_chain(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    __shared__ int piv;
    constexpr int ld = M2L<N>::ld;
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    if (!I.traj) return;
    const int t = threadIdx.x, n = I.n;
    double* Cm = dyn;
    double* Mm = Cm + M2L<N>::mat;
    double* Y = Mm + M2L<N>::mat;
    double* Gs = Y + M2L<N>::mat;
    double* Js = Gs + (N <= 32 ? M2L<N>::mat : 0);
    double* Tw = Js + (N <= 32 ? M2L<N>::mat : 0);
    double* b = dyn + M2L<N>::mats * M2L<N>::mat;
    double* eta = b + (N + 2);
    double* tv = eta + (N + 2);
    const StepCtx sc = step_ctx(I, Gs, Js, ld);
    if (N > 32 && sc.var) return;  // not routed here: above 32 states only c varies per step
    const InstWs ws = inst_ws(I);
    const int D = sc.D;
    const int64_t VD = val_doubles(D);
    for (int idx = t; idx < n * n; idx += kM2T) Cm[(idx / n) * ld + idx % n] = 0.0;
    for (int i = t; i < n; i += kM2T) b[i] = I.x0[i];
    msync();
    auto store = [&](int64_t c) {  // (C, b) over the chunk-map record of chunk c
        double* o = ws.map + c * VD;
        for (int idx = t; idx < n * n; idx += kM2T) o[(idx / n) * D + idx % n] = Cm[(idx / n) * ld + idx % n];
        for (int i = t; i < n; i += kM2T) o[D * D + i] = b[i];
    };
    store(0);
    int64_t k0, k1;
    m2_span(I, 0, k0, k1);
#pragma unroll 1
    for (int64_t k = k0; k < k1 && I.NC > 1; ++k) {
        const ElemView E = step_elem(sc, k, eta, Tw, &piv);
        fwd_combine(n, Cm, b, E, Mm, Y, tv, ld, &piv);
    }
    const int64_t ED = elem_doubles(D);
    const bool opf = I.eng != 0 && I.c == nullptr;  // operator form: matrix part in agg[0]
#pragma unroll 1
    for (int64_t c = 1; c < I.NC; ++c) {
        msync();
        store(c);
        if (c == I.NC - 1) break;
        const double* e = ws.agg + c * ED;
        const double* em = opf ? ws.agg : e;
        ElemView E;
        E.A = em;
        E.lda = D;
        E.b = e + (int64_t)D * D;
        E.C = em + (int64_t)D * D + D;
        E.ldc = D;
        E.mg = 0;
        E.eta = e + 2 * (int64_t)D * D + D;
        E.J = em + 2 * (int64_t)D * D + 2 * D;
        E.ldj = D;
        fwd_combine(n, Cm, b, E, Mm, Y, tv, ld, &piv);
    }
}

template <int N>
__global__ __launch_bounds__(kM2T) void m2c_walk(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    __shared__ int piv;
    __shared__ int bad;
    constexpr int ld = M2L<N>::ld;
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    if (!I.traj) return;
    const int64_t c = gc - I.chunk0;
    const int t = threadIdx.x, n = I.n, m = I.m;
    double* Cm = dyn;
    double* Mm = Cm + M2L<N>::mat;
    double* Y = Mm + M2L<N>::mat;
    double* Gs = Y + M2L<N>::mat;
    double* Js = Gs + (N <= 32 ? M2L<N>::mat : 0);
    double* Tw = Js + (N <= 32 ? M2L<N>::mat : 0);
    double* b = dyn + M2L<N>::mats * M2L<N>::mat;
    double* eta = b + (N + 2);
    double* tv = eta + (N + 2);
    double* xv = tv + (N + 2);
    const StepCtx sc = step_ctx(I, Gs, Js, ld);
    if (N > 32 && sc.var) return;  // not routed here: above 32 states only c varies per step
    const InstWs ws = inst_ws(I);
    const int D = sc.D;
    const double* rec = ws.map + c * val_doubles(D);
    for (int idx = t; idx < n * n; idx += kM2T) Cm[(idx / n) * ld + idx % n] = rec[(idx / n) * D + idx % n];
    for (int i = t; i < n; i += kM2T) b[i] = rec[D * D + i];
    if (t == 0) bad = 0;
    msync();
    const double* Sg = (const double*)I.S;
    const double* vg = (const double*)I.v;
    const double* Kg = (const double*)I.K;
    const double* dg = (const double*)I.d;
    double* xo = (double*)I.m2x;
    double* uo = (double*)I.m2u;
    int64_t k0, k1;
    m2_span(I, c, k0, k1);
    const int64_t kend = (c == I.NC - 1) ? I.T : k1 - 1;  // the last chunk also gives x_T
#pragma unroll 1
    for (int64_t k = k0; k <= kend; ++k) {
        // x_k = (I + C S_k)^{-1} (b + C v_k)
        const double* Sk = Sg + k * n * n;
        const double* vk = vg + k * n;
        for (int idx = t; idx < n * n; idx += kM2T) {
            const int i = idx / n, j = idx - (idx / n) * n;
            double s = (i == j) ? 1.0 : 0.0;
            for (int q = 0; q < n; ++q) s = fma(Cm[i * ld + q], Sk[q * n + j], s);
            Mm[i * ld + j] = s;
        }
        for (int i = t; i < n; i += kM2T) {
            double s = b[i];
            for (int q = 0; q < n; ++q) s = fma(Cm[i * ld + q], vk[q], s);
            xv[i] = s;
        }
        msync();
        lu_solve(n, Mm, ld, Y, 0, xv, &piv);
        if (t < n) {
            if (xo) xo[k * n + t] = xv[t];
            if (!isfinite(xv[t])) bad = 1;
        }
        if (k < I.T && uo && t < m) {
            double s = dg[k * m + t];
            for (int j = 0; j < n; ++j) s = fma(-Kg[(k * m + t) * n + j], xv[j], s);
            uo[k * m + t] = s;
            if (!isfinite(s)) bad = 1;
        }
        if (k < kend) {
            const ElemView E = step_elem(sc, k, eta, Tw, &piv);
            fwd_combine(n, Cm, b, E, Mm, Y, tv, ld, &piv);
        } else {
            msync();
        }
    }
    if (t == 0 && bad) raise_status(I.status, 4);
}

template <int N>
hipError_t m2c_run(const GInst* d_inst, int ninst, int64_t nchunks, hipStream_t s, const StageHook* h) {
    constexpr size_t lds = M2L<N>::bytes;
    static bool attr = false;
    if (!attr && lds > 64 * 1024) {  // above the default dynamic LDS limit
        const void* ks[] = {(const void*)m2c_chain<N>, (const void*)m2c_walk<N>};
        for (const void* k : ks)
            if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                return hipGetLastError();
    }
    attr = true;
    if (h) h->begin(h->ctx, "m2c_chain", s);
    m2c_chain<N><<<(unsigned)ninst, kM2T, lds, s>>>(d_inst, ninst);
    if (h) h->end(h->ctx, s);
    if (h) h->begin(h->ctx, "m2c_walk", s);
    m2c_walk<N><<<(unsigned)nchunks, kM2T, lds, s>>>(d_inst, ninst, nchunks);
    if (h) h->end(h->ctx, s);
    return hipGetLastError();
}

}  // namespace

hipError_t m2_chunked(int N, const GInst* d_inst, int ninst, int64_t nchunks, hipStream_t s, const StageHook* h) {
    if (N <= 8) return m2c_run<8>(d_inst, ninst, nchunks, s, h);
    if (N <= 16) return m2c_run<16>(d_inst, ninst, nchunks, s, h);
    if (N <= 32) return m2c_run<32>(d_inst, ninst, nchunks, s, h);
    return m2c_run<64>(d_inst, ninst, nchunks, s, h);
}

}  // namespace lqt
