// Wavefront-per-chunk LQT pipeline for general state dimension (gfx950).
//
// One wavefront owns one chunk of B consecutive steps of one instance.  The
// element being folded and every temporary live in the wavefront's slice of
// LDS (row-major, leading dimension n + 1 so column walks spread over the
// banks); the 64 lanes cooperate on every matrix product, factorisation and
// solve.  All instances of a solve share each launch: the flat chunk index is
// mapped to its instance by a binary search over the instances' first chunk.
//
// Phases (the reduce-then-scan organisation of the block processing of
// Section V-C, with the per-instance top level done sequentially -- a batch
// has far more instances than the GPU has SIMDs):
//   g_prep    per instance: G (G G^T = L U^{-1} L^T), J = H^T X H, W = H^T X
//             and the terminal value S_T = H_T^T X_T H_T, v_T = H_T^T X_T r_T;
//   g_fold    per chunk: fold the one-step elements a_k (Section IV-B) with
//             the combination rule (Section IV-A) into the chunk element;
//   g_chain   per instance: value function at every chunk start, walking the
//             chunks from the terminal value with the anchored combination;
//   g_final   per chunk: down-sweep in Riccati form fused with the gain
//             extraction (writes S, v, K, d) and the chunk's closed-loop map;
//   g_fchain  per instance: state at every chunk start from x_0 (Method 1
//             affine maps, Section IV-C);
//   g_roll    per chunk: u_k = -K_k x_k + d_k, x_{k+1} = F x_k + c + L u_k.
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"

namespace lqt {

namespace {

constexpr int kW = 64;
#define WDI __device__ __forceinline__

WDI void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

WDI void raise(int32_t* st, int32_t code) {
    if (st) atomicCAS(st, 0, code);
}

// ---- wavefront-cooperative dense kernels on LDS -------------------------------
// Matrices are row-major with an explicit leading dimension.  Every routine
// ends with wsync(); outputs never alias inputs unless stated.

// C = alpha op(A) op(B) + beta C; op(A) is R x K, op(B) is K x Q.
// sym: only the upper triangle is computed and mirrored (C square, symmetric).
template <bool TA, bool TB>
WDI void wgemm(int R, int K, int Q, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
               double alpha, double beta, int lane, bool sym = false) {
    const int tot = R * Q;
    for (int idx = lane; idx < tot; idx += kW) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        if (sym && q < r) continue;
        double s = 0.0;
        for (int k = 0; k < K; ++k) {
            const double a = TA ? A[k * lda + r] : A[r * lda + k];
            const double b = TB ? B[q * ldb + k] : B[k * ldb + q];
            s = fma(a, b, s);
        }
        const double v = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * C[r * ldc + q]);
        C[r * ldc + q] = v;
        if (sym && q != r) C[q * ldc + r] = v;
    }
    wsync();
}

// y = alpha op(A) x + beta y (A is R x K when not transposed).
template <bool TA>
WDI void wgemv(int R, int K, const double* A, int lda, const double* x, double* y, double alpha, double beta,
               int lane) {
    for (int r = lane; r < R; r += kW) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s = fma(TA ? A[k * lda + r] : A[r * lda + k], x[k], s);
        y[r] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[r]);
    }
    wsync();
}

WDI void wcopy(int R, int Q, const double* A, int lda, double* B, int ldb, int lane) {
    for (int idx = lane; idx < R * Q; idx += kW) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        B[r * ldb + q] = A[r * lda + q];
    }
    wsync();
}

// Lower Cholesky factor of the symmetric m x m matrix A, in place (upper
// triangle zeroed).  Returns false if a pivot is not > 0 (also for NaN).
WDI bool wchol(int m, double* A, int lda, int lane) {
    bool ok = true;
    for (int j = 0; j < m; ++j) {
        double s = A[j * lda + j];
        for (int k = 0; k < j; ++k) s = fma(-A[j * lda + k], A[j * lda + k], s);
        ok = ok && (s > 0.0);
        const double rjj = sqrt(s);
        wsync();  // every lane has read the diagonal before it changes
        if (lane == 0) A[j * lda + j] = rjj;
        for (int i = j + 1 + lane; i < m; i += kW) {
            double t = A[i * lda + j];
            for (int k = 0; k < j; ++k) t = fma(-A[i * lda + k], A[j * lda + k], t);
            A[i * lda + j] = t / rjj;
        }
        for (int i = lane; i < j; i += kW) A[i * lda + j] = 0.0;
        wsync();
    }
    return ok;
}

// B (m x q) <- R^{-1} B  (R lower), one column per lane.
WDI void wtrsm_l(int m, int q, const double* R, int ldr, double* B, int ldb, int lane) {
    for (int c = lane; c < q; c += kW)
        for (int i = 0; i < m; ++i) {
            double s = B[i * ldb + c];
            for (int k = 0; k < i; ++k) s = fma(-R[i * ldr + k], B[k * ldb + c], s);
            B[i * ldb + c] = s / R[i * ldr + i];
        }
    wsync();
}

// B (m x q) <- R^{-T} B  (R lower), one column per lane.
WDI void wtrsm_lt(int m, int q, const double* R, int ldr, double* B, int ldb, int lane) {
    for (int c = lane; c < q; c += kW)
        for (int i = m - 1; i >= 0; --i) {
            double s = B[i * ldb + c];
            for (int k = i + 1; k < m; ++k) s = fma(-R[k * ldr + i], B[k * ldb + c], s);
            B[i * ldb + c] = s / R[i * ldr + i];
        }
    wsync();
}

// Mi = M^{-1} by Gauss-Jordan elimination with partial pivoting; M destroyed.
// A singular M gives non-finite entries (caught by the finiteness checks).
WDI void winv(int n, double* Mm, int ldm, double* Mi, int ldi, int lane) {
    for (int idx = lane; idx < n * n; idx += kW) {
        const int r = idx / n, q = idx - (idx / n) * n;
        Mi[r * ldi + q] = (r == q) ? 1.0 : 0.0;
    }
    wsync();
    for (int k = 0; k < n; ++k) {
        // pivot row: largest |M[i][k]|, i >= k (lowest index on ties)
        double best = -1.0;
        int bi = k;
        for (int i = k + lane; i < n; i += kW) {
            const double v = fabs(Mm[i * ldm + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        for (int off = kW / 2; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, kW);
            const int oi = __shfl_xor(bi, off, kW);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int p = bi;  // uniform after the butterfly
        if (p != k) {
            for (int q = lane; q < n; q += kW) {
                double t = Mm[k * ldm + q];
                Mm[k * ldm + q] = Mm[p * ldm + q];
                Mm[p * ldm + q] = t;
                t = Mi[k * ldi + q];
                Mi[k * ldi + q] = Mi[p * ldi + q];
                Mi[p * ldi + q] = t;
            }
            wsync();
        }
        const double inv = 1.0 / Mm[k * ldm + k];
        wsync();  // every lane has read the pivot before row k is scaled
        for (int q = lane; q < n; q += kW) {
            Mm[k * ldm + q] *= inv;
            Mi[k * ldi + q] *= inv;
        }
        wsync();
        // eliminate column k from every other row: one (row, column) pair per
        // iteration; the multiplier column k of M is updated last, after all
        // lanes have used it (second pass).
        for (int idx = lane; idx < n * n; idx += kW) {
            const int r = idx / n, q = idx - (idx / n) * n;
            if (r == k) continue;
            const double fr = Mm[r * ldm + k];
            Mi[r * ldi + q] = fma(-fr, Mi[k * ldi + q], Mi[r * ldi + q]);
            if (q != k) Mm[r * ldm + q] = fma(-fr, Mm[k * ldm + q], Mm[r * ldm + q]);
        }
        wsync();
        for (int r = lane; r < n; r += kW)
            if (r != k) Mm[r * ldm + k] = 0.0;
        wsync();
    }
}

// ---- per-instance descriptor helpers -------------------------------------------

WDI const double* step_ptr(const double* base, uint32_t ps, uint32_t bit, int64_t k, int64_t sz) {
    return (ps & bit) ? base + k * sz : base;
}

// Layout of the wavefront's LDS slice for maximum dimension N (doubles).
struct WaveLds {
    int ld;      // leading dimension N + 1
    int mat;     // doubles per matrix slot (N * ld)
    int slots;   // matrix slots
    int vecs;    // vector slots of N doubles
    __host__ __device__ int doubles() const { return slots * mat + vecs * (ld + 1); }
};

__host__ __device__ inline WaveLds wave_lds(int N) {
    WaveLds w;
    w.ld = N + 1;
    w.mat = N * (N + 1);
    w.slots = 13;
    w.vecs = 10;
    return w;
}

struct Slots {
    double* m[13];
    double* v[10];
};

WDI Slots slots_of(double* base, const WaveLds& w) {
    Slots s;
    for (int i = 0; i < 13; ++i) s.m[i] = base + i * w.mat;
    for (int i = 0; i < 10; ++i) s.v[i] = base + 13 * w.mat + i * (w.ld + 1);
    return s;
}

WDI int find_instance(const GInst* inst, int ninst, int64_t chunk) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].chunk0 <= chunk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Load a matrix from global (R x Q, row stride gq) into LDS (leading dim ld).
WDI void gload(int R, int Q, const double* g, int gq, double* l, int ld, int lane) {
    for (int idx = lane; idx < R * Q; idx += kW) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        l[r * ld + q] = g[r * gq + q];
    }
    wsync();
}

WDI void gstore(int R, int Q, const double* l, int ld, double* g, int gq, int lane) {
    for (int idx = lane; idx < R * Q; idx += kW) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        g[r * gq + q] = l[r * ld + q];
    }
}

// Instance constants in the workspace.
struct CstW {
    int64_t G, J, W, ST, VT, end;
};

__host__ __device__ inline CstW cst_layout(int n, int m, int p) {
    CstW c;
    c.G = 0;
    c.J = c.G + (int64_t)n * m;
    c.W = c.J + (int64_t)n * n;
    c.ST = c.W + (int64_t)n * p;
    c.VT = c.ST + (int64_t)n * n;
    c.end = c.VT + n;
    return c;
}

__host__ __device__ inline int64_t elem_doubles(int n) { return 3 * (int64_t)n * n + 2 * n; }
__host__ __device__ inline int64_t val_doubles(int n) { return (int64_t)n * n + n; }

struct InstWs {
    double *cst, *agg, *val, *map, *xs;
};

WDI InstWs inst_ws(const GInst& I) {
    InstWs w;
    const int n = I.n;
    const CstW c = cst_layout(n, I.m, I.p > 0 ? I.p : 1);
    w.cst = I.ws;
    w.agg = w.cst + ((c.end + 31) & ~int64_t(31));
    w.val = w.agg + I.NC * elem_doubles(n);
    w.map = w.val + (I.NC + 1) * val_doubles(n);
    w.xs = w.map + I.NC * val_doubles(n);
    return w;
}

}  // namespace

int64_t wave_inst_ws_doubles(int n, int m, int p, int64_t NC) {
    const CstW c = cst_layout(n, m, p > 0 ? p : 1);
    return ((c.end + 31) & ~int64_t(31)) + NC * elem_doubles(n) + (NC + 1) * val_doubles(n) +
           NC * val_doubles(n) + NC * n + 32;
}

namespace {

// ---- g_prep: per-instance constants -----------------------------------------------

__global__ __launch_bounds__(kW) void g_prep(const GInst* inst, int ninst, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int i = blockIdx.x;
    if (i >= ninst) return;
    const GInst& I = inst[i];
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m, p = I.p, pT = I.pT;
    const WaveLds wl = wave_lds(N);
    const int ld = wl.ld;
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, p);
    double* cst = ws.cst;
    if (lane == 0 && I.status) *I.status = 0;
    bool ok = true;
    if (!(I.per_step & (kPS_L | kPS_U | kPS_H | kPS_X))) {
        // G: G^T = R_U^{-1} L^T with U = R_U R_U^T
        gload(m, m, I.U, m, s.m[0], ld, lane);
        ok = wchol(m, s.m[0], ld, lane);
        for (int idx = lane; idx < m * n; idx += kW) {
            const int a = idx / n, j = idx - (idx / n) * n;
            s.m[1][a * ld + j] = I.L[j * m + a];
        }
        wsync();
        wtrsm_l(m, n, s.m[0], ld, s.m[1], ld, lane);
        for (int idx = lane; idx < n * m; idx += kW) {
            const int j = idx / m, a = idx - (idx / m) * m;
            cst[cl.G + j * m + a] = s.m[1][a * ld + j];
        }
        // W = H^T X (n x p), J = W H (n x n)
        gload(p, n, I.H, n, s.m[2], ld, lane);
        gload(p, p, I.X, p, s.m[3], ld, lane);
        wgemm<true, false>(n, p, p, s.m[2], ld, s.m[3], ld, s.m[4], ld, 1.0, 0.0, lane);
        wgemm<false, false>(n, p, n, s.m[4], ld, s.m[2], ld, s.m[5], ld, 1.0, 0.0, lane, true);
        gstore(n, p, s.m[4], ld, cst + cl.W, p, lane);
        gstore(n, n, s.m[5], ld, cst + cl.J, n, lane);
    }
    // terminal value
    gload(pT, n, I.HT, n, s.m[2], ld, lane);
    gload(pT, pT, I.XT, pT, s.m[3], ld, lane);
    for (int q = lane; q < pT; q += kW) s.v[0][q] = I.rT[q];
    wsync();
    wgemm<true, false>(n, pT, pT, s.m[2], ld, s.m[3], ld, s.m[4], ld, 1.0, 0.0, lane);
    wgemm<false, false>(n, pT, n, s.m[4], ld, s.m[2], ld, s.m[5], ld, 1.0, 0.0, lane, true);
    wgemv<false>(n, pT, s.m[4], ld, s.v[0], s.v[1], 1.0, 0.0, lane);
    gstore(n, n, s.m[5], ld, cst + cl.ST, n, lane);
    for (int q = lane; q < n; q += kW) cst[cl.VT + q] = s.v[1][q];
    if (!ok && lane == 0) raise(I.status, 3);
}

// Step data of a_k into LDS: F (n x n), c (n), G (n x m), eta (n), J (n x n).
// Time-varying L, U, H, X are factorised here, per step.
WDI bool load_step(const GInst& I, int64_t k, const double* cst, const CstW& cl, double* Us, double* Ht,
                   double* Xt, int ld, double* F, double* c, double* G, double* e, double* J, int lane,
                   bool need_G, bool need_J) {
    const int n = I.n, m = I.m, p = I.p;
    const uint32_t ps = I.per_step;
    bool ok = true;
    gload(n, n, step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n), n, F, ld, lane);
    for (int q = lane; q < n; q += kW) c[q] = I.c ? step_ptr(I.c, ps, kPS_c, k, n)[q] : 0.0;
    const double* r = I.r + k * p;
    if (!(ps & (kPS_L | kPS_U | kPS_H | kPS_X))) {
        if (need_G) gload(n, m, cst + cl.G, m, G, ld, lane);
        if (need_J) gload(n, n, cst + cl.J, n, J, ld, lane);
        for (int q = lane; q < n; q += kW) {
            double t = 0.0;
            for (int j = 0; j < p; ++j) t = fma(cst[cl.W + q * p + j], r[j], t);
            e[q] = t;
        }
        wsync();
    } else {
        // Us, Ht, Xt: scratch for the per-step factorisations
        gload(m, m, step_ptr(I.U, ps, kPS_U, k, (int64_t)m * m), m, Us, ld, lane);
        ok = wchol(m, Us, ld, lane);
        if (need_G) {
            const double* L = step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m);
            for (int idx = lane; idx < m * n; idx += kW) {
                const int a = idx / n, j = idx - (idx / n) * n;
                Ht[a * ld + j] = L[j * m + a];
            }
            wsync();
            wtrsm_l(m, n, Us, ld, Ht, ld, lane);
            for (int idx = lane; idx < n * m; idx += kW) {
                const int j = idx / m, a = idx - (idx / m) * m;
                G[j * ld + a] = Ht[a * ld + j];
            }
            wsync();
        }
        gload(p, n, step_ptr(I.H, ps, kPS_H, k, (int64_t)p * n), n, Ht, ld, lane);
        gload(p, p, step_ptr(I.X, ps, kPS_X, k, (int64_t)p * p), p, Xt, ld, lane);
        // W = H^T X into Us (no longer needed)
        wgemm<true, false>(n, p, p, Ht, ld, Xt, ld, Us, ld, 1.0, 0.0, lane);
        if (need_J) wgemm<false, false>(n, p, n, Us, ld, Ht, ld, J, ld, 1.0, 0.0, lane, true);
        for (int q = lane; q < n; q += kW) {
            double t = 0.0;
            for (int j = 0; j < p; ++j) t = fma(Us[q * ld + j], r[j], t);
            e[q] = t;
        }
        wsync();
    }
    return ok;
}

// P <- a_k (x) P with C_k = G G^T (matrix inversion lemma form of the
// combination rule; see the lane-per-element pipeline for the identities).
// P = (PA, Pb, PC, Pe, PJ) in LDS.  Uses slots 5..9 and vectors 5..9.
WDI void w_step_combine(int n, int m, const double* F, const double* c, const double* G, const double* ek,
                        const double* Js, double* PA, double* Pb, double* PC, double* Pe, double* PJ,
                        Slots& s, int ld, int lane) {
    double* Z = s.m[5];    // m x n: G^T J_P, then Y = R^{-1} Z
    double* Wm = s.m[6];   // m x m: I + Z G, then R
    double* GtT = s.m[7];  // m x n: R^{-1} G^T
    double* V = s.m[8];    // n x m: A_P Gt
    double* T9 = s.m[9];   // n x n scratch
    double* q = s.v[5];
    double* g2 = s.v[6];
    double* w = s.v[7];
    double* nb = s.v[8];
    double* ne = s.v[9];
    wgemm<true, false>(m, n, n, G, ld, PJ, ld, Z, ld, 1.0, 0.0, lane);
    wgemm<false, false>(m, n, m, Z, ld, G, ld, Wm, ld, 1.0, 0.0, lane, true);
    for (int a = lane; a < m; a += kW) Wm[a * ld + a] += 1.0;
    wsync();
    wchol(m, Wm, ld, lane);  // W >= I: cannot fail for finite inputs
    wtrsm_l(m, n, Wm, ld, Z, ld, lane);  // Z := Y
    for (int idx = lane; idx < m * n; idx += kW) {
        const int a = idx / n, j = idx - (idx / n) * n;
        GtT[a * ld + j] = G[j * ld + a];
    }
    wsync();
    wtrsm_l(m, n, Wm, ld, GtT, ld, lane);
    wgemm<false, true>(n, n, m, PA, ld, GtT, ld, V, ld, 1.0, 0.0, lane);  // V = A_P Gt
    // q = Gt^T eta_P - Y c
    wgemv<false>(m, n, GtT, ld, Pe, q, 1.0, 0.0, lane);
    wgemv<false>(m, n, Z, ld, c, q, -1.0, 1.0, lane);
    // b_new = A_P (c + Gt q) + b_P
    for (int j = lane; j < n; j += kW) {
        double t = c[j];
        for (int a = 0; a < m; ++a) t = fma(GtT[a * ld + j], q[a], t);
        g2[j] = t;
    }
    wsync();
    wgemv<false>(n, n, PA, ld, g2, nb, 1.0, 0.0, lane);
    // eta_new = F^T (eta_P - J_P c - Y^T q) + e_k
    wgemv<false>(n, n, PJ, ld, c, w, -1.0, 0.0, lane);
    for (int j = lane; j < n; j += kW) {
        double t = w[j] + Pe[j];
        for (int a = 0; a < m; ++a) t = fma(-Z[a * ld + j], q[a], t);
        w[j] = t;
    }
    wsync();
    wgemv<true>(n, n, F, ld, w, ne, 1.0, 0.0, lane);
    for (int j = lane; j < n; j += kW) {
        Pb[j] = nb[j] + Pb[j];
        Pe[j] = ne[j] + ek[j];
    }
    // C_new = C_P + V V^T
    wgemm<false, true>(n, m, n, V, ld, V, ld, PC, ld, 1.0, 1.0, lane, true);
    // A_new = A_P F - V (Y F)
    wgemm<false, false>(m, n, n, Z, ld, F, ld, Wm, ld, 1.0, 0.0, lane);   // YF in Wm (R no longer needed)
    wgemm<false, false>(n, n, n, PA, ld, F, ld, T9, ld, 1.0, 0.0, lane);  // A_P F
    wgemm<false, false>(n, m, n, V, ld, Wm, ld, T9, ld, -1.0, 1.0, lane);
    wcopy(n, n, T9, ld, PA, ld, lane);
    // J_new = F^T (J_P - Y^T Y) F + J_k
    wgemm<true, false>(n, m, n, Z, ld, Z, ld, PJ, ld, -1.0, 1.0, lane, true);
    wgemm<false, false>(n, n, n, PJ, ld, F, ld, T9, ld, 1.0, 0.0, lane);
    wgemm<true, false>(n, n, n, F, ld, T9, ld, PJ, ld, 1.0, 0.0, lane, true);
    for (int idx = lane; idx < n * n; idx += kW) {
        const int r = idx / n, q2 = idx - (idx / n) * n;
        PJ[r * ld + q2] += Js[r * ld + q2];
    }
    wsync();
}

// (S, v) <- E (x) (0, 0, 0, v, S): anchored combination rule.  Uses slots 5..8.
WDI void w_anchor(int n, const double* EA, const double* Eb, const double* EC, const double* Ee,
                  const double* EJ, double* Sm, double* v, Slots& s, int ld, int lane) {
    double* Mm = s.m[5];
    double* Mi = s.m[6];
    double* T1 = s.m[7];
    double* P = s.m[8];
    double* t = s.v[5];
    double* nv = s.v[6];
    wgemm<false, false>(n, n, n, EC, ld, Sm, ld, Mm, ld, 1.0, 0.0, lane);
    for (int a = lane; a < n; a += kW) Mm[a * ld + a] += 1.0;
    wsync();
    winv(n, Mm, ld, Mi, ld, lane);
    wgemm<false, false>(n, n, n, Mi, ld, EA, ld, T1, ld, 1.0, 0.0, lane);
    wgemv<false>(n, n, Sm, ld, Eb, t, -1.0, 0.0, lane);
    for (int j = lane; j < n; j += kW) t[j] += v[j];
    wsync();
    wgemv<true>(n, n, T1, ld, t, nv, 1.0, 0.0, lane);
    wgemm<false, false>(n, n, n, Sm, ld, EA, ld, P, ld, 1.0, 0.0, lane);
    wgemm<true, false>(n, n, n, T1, ld, P, ld, Sm, ld, 1.0, 0.0, lane, true);
    for (int idx = lane; idx < n * n; idx += kW) {
        const int r = idx / n, q = idx - (idx / n) * n;
        Sm[r * ld + q] += EJ[r * ld + q];
    }
    for (int j = lane; j < n; j += kW) v[j] = nv[j] + Ee[j];
    wsync();
}

// ---- g_fold ---------------------------------------------------------------------

__global__ __launch_bounds__(kW) void g_fold(const GInst* inst, int ninst, int64_t nchunks, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const int ii = find_instance(inst, ninst, gc);
    const GInst& I = inst[ii];
    const int64_t c = gc - I.chunk0;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m;
    const WaveLds wl = wave_lds(N);
    const int ld = wl.ld;
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, I.p);
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double *PA = s.m[0], *PC = s.m[1], *PJ = s.m[2], *F = s.m[3], *G = s.m[4];
    double* Js = s.m[10];  // J of the step (constant when time-invariant)
    double *Pb = s.v[0], *Pe = s.v[1], *cc = s.v[2], *ek = s.v[3];
    bool ok = true;
    const bool var = (I.per_step & (kPS_L | kPS_U | kPS_H | kPS_X)) != 0;
    // slots 5..7 are free while the step data is loaded (step_combine's scratch)
    ok = load_step(I, k1 - 1, ws.cst, cl, s.m[5], s.m[6], s.m[7], ld, F, cc, G, ek, Js, lane, true, true) && ok;
    wcopy(n, n, F, ld, PA, ld, lane);
    wgemm<false, true>(n, m, n, G, ld, G, ld, PC, ld, 1.0, 0.0, lane, true);
    wcopy(n, n, Js, ld, PJ, ld, lane);
    for (int j = lane; j < n; j += kW) {
        Pb[j] = cc[j];
        Pe[j] = ek[j];
    }
    wsync();
    for (int64_t k = k1 - 2; k >= k0; --k) {
        ok = load_step(I, k, ws.cst, cl, s.m[5], s.m[6], s.m[7], ld, F, cc, G, ek, Js, lane, var, var) && ok;
        w_step_combine(n, m, F, cc, G, ek, Js, PA, Pb, PC, Pe, PJ, s, ld, lane);
    }
    double* out = ws.agg + c * elem_doubles(n);
    const int64_t nn = (int64_t)n * n;
    gstore(n, n, PA, ld, out, n, lane);
    for (int j = lane; j < n; j += kW) out[nn + j] = Pb[j];
    gstore(n, n, PC, ld, out + nn + n, n, lane);
    for (int j = lane; j < n; j += kW) out[2 * nn + n + j] = Pe[j];
    gstore(n, n, PJ, ld, out + 2 * nn + 2 * n, n, lane);
    if (!ok && lane == 0) raise(I.status, 3);
}

// ---- g_chain: value at every chunk start, one wavefront per instance ------------

__global__ __launch_bounds__(kW) void g_chain(const GInst* inst, int ninst, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    const int lane = threadIdx.x;
    const int n = I.n;
    const WaveLds wl = wave_lds(N);
    const int ld = wl.ld;
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, I.m, I.p);
    const int64_t nn = (int64_t)n * n;
    double *EA = s.m[0], *EC = s.m[1], *EJ = s.m[2], *Sm = s.m[3];
    double *Eb = s.v[0], *Ee = s.v[1], *v = s.v[2];
    gload(n, n, ws.cst + cl.ST, n, Sm, ld, lane);
    for (int j = lane; j < n; j += kW) v[j] = ws.cst[cl.VT + j];
    wsync();
    double* vo = ws.val + I.NC * val_doubles(n);
    gstore(n, n, Sm, ld, vo, n, lane);
    for (int j = lane; j < n; j += kW) vo[nn + j] = v[j];
    for (int64_t c = I.NC - 1; c >= 0; --c) {
        const double* e = ws.agg + c * elem_doubles(n);
        gload(n, n, e, n, EA, ld, lane);
        gload(n, n, e + nn + n, n, EC, ld, lane);
        gload(n, n, e + 2 * nn + 2 * n, n, EJ, ld, lane);
        for (int j = lane; j < n; j += kW) {
            Eb[j] = e[nn + j];
            Ee[j] = e[2 * nn + n + j];
        }
        wsync();
        w_anchor(n, EA, Eb, EC, Ee, EJ, Sm, v, s, ld, lane);
        vo = ws.val + c * val_doubles(n);
        gstore(n, n, Sm, ld, vo, n, lane);
        for (int j = lane; j < n; j += kW) vo[nn + j] = v[j];
    }
}

// ---- g_final: down-sweep with gain extraction, chunk closed-loop map -----------

__global__ __launch_bounds__(kW) void g_final(const GInst* inst, int ninst, int64_t nchunks, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const int ii = find_instance(inst, ninst, gc);
    const GInst& I = inst[ii];
    const int64_t c = gc - I.chunk0;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m;
    const WaveLds wl = wave_lds(N);
    const int ld = wl.ld;
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, I.p);
    const int64_t nn = (int64_t)n * n;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    const uint32_t ps = I.per_step;
    const bool var = (ps & (kPS_L | kPS_U | kPS_H | kPS_X)) != 0;
    double *Sm = s.m[0], *F = s.m[1], *L = s.m[2], *Um = s.m[3], *Js = s.m[4];
    double *SL = s.m[5], *R = s.m[6], *SF = s.m[7], *Y = s.m[8], *K = s.m[9];
    double *Phi = s.m[10], *Ft = s.m[11], *T12 = s.m[12];
    double *v = s.v[0], *cc = s.v[1], *ek = s.v[2], *w = s.v[3], *z = s.v[4], *d = s.v[5];
    double *phi = s.v[6], *ct = s.v[7], *nv = s.v[8], *t9 = s.v[9];
    // value at the chunk end (= start of chunk c + 1)
    const double* vin = ws.val + (c + 1) * val_doubles(n);
    gload(n, n, vin, n, Sm, ld, lane);
    for (int j = lane; j < n; j += kW) v[j] = vin[nn + j];
    for (int idx = lane; idx < n * n; idx += kW) {
        const int r = idx / n, q = idx - (idx / n) * n;
        Phi[r * ld + q] = (r == q) ? 1.0 : 0.0;
    }
    for (int j = lane; j < n; j += kW) phi[j] = 0.0;
    wsync();
    if (k1 == I.T) {
        if (I.S) gstore(n, n, Sm, ld, I.S + I.T * nn, n, lane);
        if (I.v)
            for (int j = lane; j < n; j += kW) I.v[I.T * n + j] = v[j];
    }
    double fin = 0.0;
    bool ok = true;
    for (int64_t k = k1 - 1; k >= k0; --k) {
        // step data: F, c, L, U, J_k, eta_k
        // slots 5..7 (SL, R, SF) are free here and serve as scratch
        ok = load_step(I, k, ws.cst, cl, SL, R, SF, ld, F, cc, T12, ek, Js, lane, false, var || k == k1 - 1) && ok;
        gload(n, m, step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m), m, L, ld, lane);
        gload(m, m, step_ptr(I.U, ps, kPS_U, k, (int64_t)m * m), m, Um, ld, lane);
        // M_k = L^T S L + U = R R^T
        wgemm<false, false>(n, n, m, Sm, ld, L, ld, SL, ld, 1.0, 0.0, lane);
        wgemm<true, false>(m, n, m, L, ld, SL, ld, R, ld, 1.0, 0.0, lane, true);
        for (int idx = lane; idx < m * m; idx += kW) {
            const int a = idx / m, b = idx - (idx / m) * m;
            if (b >= a) {
                const double u = 0.5 * (Um[a * ld + b] + Um[b * ld + a]);
                R[a * ld + b] += u;
                if (b != a) R[b * ld + a] += u;
            }
        }
        wsync();
        ok = wchol(m, R, ld, lane) && ok;
        // Y = R^{-1} L^T S F ; K = R^{-T} Y
        wgemm<false, false>(n, n, n, Sm, ld, F, ld, SF, ld, 1.0, 0.0, lane);
        wgemm<true, false>(m, n, n, L, ld, SF, ld, Y, ld, 1.0, 0.0, lane);
        wtrsm_l(m, n, R, ld, Y, ld, lane);
        wcopy(m, n, Y, ld, K, ld, lane);
        wtrsm_lt(m, n, R, ld, K, ld, lane);
        // w = v - S c ; z = L^T w ; d = M^{-1} z
        wgemv<false>(n, n, Sm, ld, cc, w, -1.0, 0.0, lane);
        for (int j = lane; j < n; j += kW) w[j] += v[j];
        wsync();
        wgemv<true>(m, n, L, ld, w, z, 1.0, 0.0, lane);
        for (int a = lane; a < m; a += kW) d[a] = z[a];
        wsync();
        wtrsm_l(m, 1, R, ld, d, 1, lane);
        wtrsm_lt(m, 1, R, ld, d, 1, lane);
        // S' = F^T S F - Y^T Y + J ; v' = F^T w - K^T z + eta
        wgemm<true, false>(n, n, n, F, ld, SF, ld, T12, ld, 1.0, 0.0, lane, true);
        wgemm<true, false>(n, m, n, Y, ld, Y, ld, T12, ld, -1.0, 1.0, lane, true);
        wgemv<true>(n, n, F, ld, w, nv, 1.0, 0.0, lane);
        wgemv<true>(n, m, K, ld, z, nv, -1.0, 1.0, lane);
        for (int idx = lane; idx < n * n; idx += kW) {
            const int r = idx / n, q = idx - (idx / n) * n;
            Sm[r * ld + q] = T12[r * ld + q] + Js[r * ld + q];
        }
        for (int j = lane; j < n; j += kW) v[j] = nv[j] + ek[j];
        wsync();
        // Ft = F - L K ; ct = c + L d
        wcopy(n, n, F, ld, Ft, ld, lane);
        wgemm<false, false>(n, m, n, L, ld, K, ld, Ft, ld, -1.0, 1.0, lane);
        wgemv<false>(n, m, L, ld, d, ct, 1.0, 0.0, lane);
        for (int j = lane; j < n; j += kW) ct[j] += cc[j];
        wsync();
        // outputs (contiguous rows, coalesced across the wavefront)
        if (I.S) gstore(n, n, Sm, ld, I.S + k * nn, n, lane);
        if (I.v)
            for (int j = lane; j < n; j += kW) I.v[k * n + j] = v[j];
        gstore(m, n, K, ld, I.K + k * m * n, n, lane);
        for (int a = lane; a < m; a += kW) I.d[k * m + a] = d[a];
        for (int idx = lane; idx < n * n; idx += kW) fin += Sm[(idx / n) * ld + (idx % n)];
        for (int j = lane; j < n; j += kW) fin += v[j];
        // chunk map: Phi <- Phi Ft, phi <- Phi ct + phi
        wgemv<false>(n, n, Phi, ld, ct, t9, 1.0, 0.0, lane);
        for (int j = lane; j < n; j += kW) phi[j] += t9[j];
        wgemm<false, false>(n, n, n, Phi, ld, Ft, ld, T12, ld, 1.0, 0.0, lane);
        wcopy(n, n, T12, ld, Phi, ld, lane);
    }
    double* mo = ws.map + c * val_doubles(n);
    gstore(n, n, Phi, ld, mo, n, lane);
    for (int j = lane; j < n; j += kW) mo[nn + j] = phi[j];
    // any lane's non-finite partial sum marks the instance
    const bool bad = !isfinite(fin);
    if (__any(bad) && lane == 0) raise(I.status, 4);
    if (!ok && lane == 0) raise(I.status, 3);
}

// ---- forward pass ------------------------------------------------------------------

__global__ __launch_bounds__(kW) void g_fchain(const GInst* inst, int ninst, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    const int lane = threadIdx.x;
    const int n = I.n;
    const WaveLds wl = wave_lds(N);
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const int64_t nn = (int64_t)n * n;
    double* x = s.v[0];
    double* t = s.v[1];
    for (int j = lane; j < n; j += kW) x[j] = I.x0[j];
    wsync();
    for (int64_t c = 0; c < I.NC; ++c) {
        for (int j = lane; j < n; j += kW) ws.xs[c * n + j] = x[j];
        const double* mp = ws.map + c * val_doubles(n);
        for (int r = lane; r < n; r += kW) {
            double a = mp[nn + r];
            for (int q = 0; q < n; ++q) a = fma(mp[r * n + q], x[q], a);
            t[r] = a;
        }
        wsync();
        for (int j = lane; j < n; j += kW) x[j] = t[j];
        wsync();
    }
}

__global__ __launch_bounds__(kW) void g_roll(const GInst* inst, int ninst, int64_t nchunks, int N) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const int ii = find_instance(inst, ninst, gc);
    const GInst& I = inst[ii];
    const int64_t c = gc - I.chunk0;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m;
    const WaveLds wl = wave_lds(N);
    const int ld = wl.ld;
    Slots s = slots_of(dyn, wl);
    const InstWs ws = inst_ws(I);
    const uint32_t ps = I.per_step;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double *F = s.m[0], *L = s.m[1];
    double *x = s.v[0], *u = s.v[1], *t = s.v[2];
    for (int j = lane; j < n; j += kW) x[j] = ws.xs[c * n + j];
    wsync();
    double fin = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        if (k == k0 || (ps & kPS_F)) gload(n, n, step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n), n, F, ld, lane);
        if (k == k0 || (ps & kPS_L)) gload(n, m, step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m), m, L, ld, lane);
        const double* Kk = I.K + k * m * n;
        for (int a = lane; a < m; a += kW) {
            double sacc = I.d[k * m + a];
            for (int j = 0; j < n; ++j) sacc = fma(-Kk[a * n + j], x[j], sacc);
            u[a] = sacc;
        }
        wsync();
        if (I.x)
            for (int j = lane; j < n; j += kW) I.x[k * n + j] = x[j];
        if (I.u)
            for (int a = lane; a < m; a += kW) I.u[k * m + a] = u[a];
        const double* cp = I.c ? step_ptr(I.c, ps, kPS_c, k, n) : nullptr;
        for (int r = lane; r < n; r += kW) {
            double a = cp ? cp[r] : 0.0;
            for (int q = 0; q < n; ++q) a = fma(F[r * ld + q], x[q], a);
            for (int q = 0; q < m; ++q) a = fma(L[r * ld + q], u[q], a);
            t[r] = a;
        }
        wsync();
        for (int j = lane; j < n; j += kW) {
            x[j] = t[j];
            fin += t[j];
        }
        wsync();
    }
    if (k1 == I.T && I.x)
        for (int j = lane; j < n; j += kW) I.x[I.T * n + j] = x[j];
    if (__any(!isfinite(fin)) && lane == 0) raise(I.status, 4);
}

struct WStage {
    const StageHook* h;
    hipStream_t s;
    WStage(const StageHook* hook, const char* name, hipStream_t st) : h(hook), s(st) {
        if (h) h->begin(h->ctx, name, s);
    }
    ~WStage() {
        if (h) h->end(h->ctx, s);
    }
};

}  // namespace

size_t wave_lds_bytes(int nmax) { return (size_t)wave_lds(nmax).doubles() * sizeof(double); }

hipError_t wave_solve(const GInst* d_inst, int ninst, int64_t nchunks, int nmax, bool want_fwd, hipStream_t s,
                      const StageHook* h) {
    const size_t lds = wave_lds_bytes(nmax);
    static bool attr = false;
    if (!attr) {
        const void* ks[] = {(const void*)g_prep, (const void*)g_fold, (const void*)g_chain,
                            (const void*)g_final, (const void*)g_fchain, (const void*)g_roll};
        for (const void* k : ks) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    {
        WStage st(h, "g_prep", s);
        g_prep<<<ninst, kW, lds, s>>>(d_inst, ninst, nmax);
    }
    {
        WStage st(h, "g_fold", s);
        g_fold<<<(unsigned)nchunks, kW, lds, s>>>(d_inst, ninst, nchunks, nmax);
    }
    {
        WStage st(h, "g_chain", s);
        g_chain<<<ninst, kW, lds, s>>>(d_inst, ninst, nmax);
    }
    {
        WStage st(h, "g_final", s);
        g_final<<<(unsigned)nchunks, kW, lds, s>>>(d_inst, ninst, nchunks, nmax);
    }
    if (want_fwd) {
        {
            WStage st(h, "g_fchain", s);
            g_fchain<<<ninst, kW, lds, s>>>(d_inst, ninst, nmax);
        }
        WStage st(h, "g_roll", s);
        g_roll<<<(unsigned)nchunks, kW, lds, s>>>(d_inst, ninst, nchunks, nmax);
    }
    return hipGetLastError();
}

}  // namespace lqt
