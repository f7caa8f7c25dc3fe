// Workgroup-per-chunk LQT pipeline for the dense class 32 < max(n, m, p, pT)
// <= 64, m <= 32 (gfx950).
//
// One workgroup of four wavefronts owns one chunk of B consecutive steps.
// The chunk's state matrices (64 x 64, zero-padded) and every temporary live
// in the workgroup's LDS (about 155 KB of the 160 KB); the products run on the
// matrix cores (16x16x4 FP64 MFMA, four 16 x 16 output tiles per wavefront).
// Instance constants (F, L, G, U, J, W, padded) are read from the workspace,
// where they stay cache-resident for all chunks of the instance.
//
// The one-step combination a_k (x) P is taken in Cholesky form: with
// C_k = G G^T and W = I + G^T J_P G = R R^T (m x m), V = R^{-1} G^T J_P and
// Q = A_P G R^{-T}, the combination rule of Section IV-A becomes
//   A' = A_P F - Q (V F),     C' = C_P + Q Q^T,   J' = F^T (J_P - V^T V) F + J_k,
//   b' = A_P (c + G W^{-1} h) + b_P,   eta' = F^T (eta_P - J_P c - V^T R^{-1} h) + eta_k,
// with h = G^T eta_P - G^T J_P c.  Every update is a product of an operand
// with itself or of small factors, so all of them fit the LDS budget and the
// symmetric ones are exactly symmetric.  The down-sweep step (value function
// and gains) uses the same factorisation of M_k = L^T S L + U = R R^T:
// K = R^{-T} V with V = R^{-1} L^T S F, and S' = F^T S F - V^T V + J.
//
// Phases (as in the wavefront classes): b_prep (constants, terminal value),
// b_fold (chunk elements), b_chain (value at chunk starts, per instance),
// b_final (values, gains, chunk maps), b_fchain (state at chunk starts),
// b_roll (trajectory).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_ws.hpp"

namespace lqt {

namespace {

constexpr int kT = 256;  // threads per workgroup
constexpr int N = kBlockN, M = kBlockM;
constexpr int LN = N + 2, LM = M + 2;  // LDS leading dimensions
#define BDI __device__ __forceinline__

typedef double dvec4 __attribute__((ext_vector_type(4)));

BDI void bsync() { __syncthreads(); }

// C (R x Q) = alpha op(A) op(B) + alpha2 op(A2) op(B2) + beta C + E on the
// matrix cores.  op(A) is R x K, op(A2) is R x K2 (K2 = 0: no second term).
// Operand layout of the 16x16x4 FP64 MFMA (measured on gfx950): lane l
// supplies A[l % 16][4s + l / 16] and B[4s + l / 16][l % 16]; accumulator
// element v of lane l is C[l / 16 + 4 v][l % 16].  Every tile is computed into
// registers before a workgroup barrier and written after it, so C may alias
// any operand.  SYM: C is symmetric; only tiles on or above the diagonal are
// computed and each value is written to both mirrored positions.  E (may be
// null, row stride lde) is added to the result.
template <int R, int Q, int K, bool TA, bool TB, bool SYM, int K2 = 0, bool TA2 = false, bool TB2 = false>
BDI void bgemm(const double* A, int lda, const double* B, int ldb, double* C, int ldc, double alpha, double beta,
               const double* E = nullptr, int lde = 0, const double* A2 = nullptr, int lda2 = 0,
               const double* B2 = nullptr, int ldb2 = 0, double alpha2 = 0.0) {
    constexpr int TR = R / 16, TQ = Q / 16;
    static_assert(R % 16 == 0 && Q % 16 == 0 && K % 4 == 0 && K2 % 4 == 0, "tile shape");
    static_assert(!SYM || R == Q, "symmetric result must be square");
    constexpr int NT = SYM ? TR * (TR + 1) / 2 : TR * TQ;
    constexpr int PER = (NT + 3) / 4;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i0 = lane & 15, kk = lane >> 4;
    double out[PER][4];
    int tbi[PER], tbj[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int t = wave + 4 * q;
        tbi[q] = -1;
        tbj[q] = 0;
        if (t < NT) {  // uniform over the wavefront
            int bi, bj;
            if constexpr (SYM) {
                int tt = t;
                bi = 0;
                while (tt >= TR - bi) {
                    tt -= TR - bi;
                    ++bi;
                }
                bj = bi + tt;
            } else {
                bi = t / TQ;
                bj = t - bi * TQ;
            }
            tbi[q] = bi;
            tbj[q] = bj;
            const int ar = 16 * bi + i0, bc = 16 * bj + i0;
            dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int s = 0; s < K / 4; ++s) {
                const int kx = 4 * s + kk;
                const double a = TA ? A[kx * lda + ar] : A[ar * lda + kx];
                const double b = TB ? B[bc * ldb + kx] : B[kx * ldb + bc];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            dvec4 acc2 = {0.0, 0.0, 0.0, 0.0};
            if constexpr (K2 > 0) {
#pragma unroll 4
                for (int s = 0; s < K2 / 4; ++s) {
                    const int kx = 4 * s + kk;
                    const double a = TA2 ? A2[kx * lda2 + ar] : A2[ar * lda2 + kx];
                    const double b = TB2 ? B2[bc * ldb2 + kx] : B2[kx * ldb2 + bc];
                    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc2, 0, 0, 0);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bi + kk + 4 * v, c = 16 * bj + i0;
                double o = alpha * acc[v];
                if constexpr (K2 > 0) o = fma(alpha2, acc2[v], o);
                if (beta != 0.0) o = fma(beta, C[r * ldc + c], o);
                if (E) o += E[r * lde + c];
                out[q][v] = o;
            }
        }
    }
    bsync();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (tbi[q] < 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * tbi[q] + kk + 4 * v, c = 16 * tbj[q] + i0;
            if (SYM && tbi[q] == tbj[q] && r > c) continue;  // written as the mirror of (c, r)
            C[r * ldc + c] = out[q][v];
            if (SYM) C[c * ldc + r] = out[q][v];
        }
    }
    bsync();
}

// y = alpha op(A) x + beta y; op(A) is R x K (R <= kT).  Reads finish before a
// barrier, so y may alias x.
template <int R, int K, bool TA>
BDI void bgemv(const double* A, int lda, const double* x, double* y, double alpha, double beta) {
    const int t = threadIdx.x;
    double s = 0.0;
    if (t < R) {
#pragma unroll 8
        for (int k = 0; k < K; ++k) s = fma(TA ? A[k * lda + t] : A[t * lda + k], x[k], s);
        s = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[t]);
    }
    bsync();
    if (t < R) y[t] = s;
    bsync();
}

// Lower Cholesky factor of the symmetric matrix A (its first m rows and
// columns; the padding is the identity), in place, upper triangle zeroed.
// Returns false if a pivot is not > 0 (NaN included).
BDI bool bchol(double* A, int ld, int m) {
    const int t = threadIdx.x;
    bool ok = true;
    for (int j = 0; j < m; ++j) {
        double s = A[j * ld + j];
        for (int k = 0; k < j; ++k) s = fma(-A[j * ld + k], A[j * ld + k], s);
        ok = ok && (s > 0.0);
        const double rjj = sqrt(s);
        const double inv = 1.0 / rjj;
        const int i = j + 1 + t;
        double val = 0.0;
        if (i < m) {
            val = A[i * ld + j];
            for (int k = 0; k < j; ++k) val = fma(-A[i * ld + k], A[j * ld + k], val);
            val *= inv;
        }
        bsync();  // every thread has read A[j][j]
        if (t == 0) A[j * ld + j] = rjj;
        if (i < m) A[i * ld + j] = val;
        if (t < j) A[t * ld + j] = 0.0;
        bsync();
    }
    return ok;
}

// X = R^{-1} for the lower triangular M x M matrix R whose first m rows and
// columns are factorised (identity beyond); X is lower triangular.  Row i of
// X depends only on rows < i.
BDI void btrinv(const double* R, int ldr, double* X, int ldx, int m) {
    const int t = threadIdx.x;
    for (int idx = t; idx < M * M; idx += kT) {
        const int r = idx / M, q = idx - (idx / M) * M;
        X[r * ldx + q] = (r == q && r >= m) ? 1.0 : 0.0;
    }
    bsync();
    for (int i = 0; i < m; ++i) {
        if (t <= i) {
            const int j = t;
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = j; k < i; ++k) s = fma(-R[i * ldr + k], X[k * ldx + j], s);
            X[i * ldx + j] = s / R[i * ldr + i];
        }
        bsync();
    }
}

// Mi = Mm^{-1} (N x N, Gauss-Jordan with partial pivoting; Mm destroyed).
BDI void binv(double* Mm, int ld, double* Mi, int ldi, int* piv_sh) {
    const int t = threadIdx.x;
    for (int idx = t; idx < N * N; idx += kT) {
        const int r = idx / N, q = idx - (idx / N) * N;
        Mi[r * ldi + q] = (r == q) ? 1.0 : 0.0;
    }
    bsync();
    for (int k = 0; k < N; ++k) {
        if (t < 64) {  // wavefront 0 finds the pivot row
            double best = -1.0;
            int bi = k;
            if (t >= k) {
                best = fabs(Mm[t * ld + k]);
                bi = t;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if (t == 0) *piv_sh = bi;
        }
        bsync();
        const int p = *piv_sh;
        if (p != k) {
            if (t < N) {
                const double a = Mm[k * ld + t];
                Mm[k * ld + t] = Mm[p * ld + t];
                Mm[p * ld + t] = a;
            } else if (t < 2 * N) {
                const int q = t - N;
                const double a = Mi[k * ldi + q];
                Mi[k * ldi + q] = Mi[p * ldi + q];
                Mi[p * ldi + q] = a;
            }
            bsync();
        }
        const double inv = 1.0 / Mm[k * ld + k];
        bsync();
        if (t < N) Mm[k * ld + t] *= inv;
        else if (t < 2 * N) Mi[k * ldi + t - N] *= inv;
        bsync();
        for (int idx = t; idx < N * 2 * N; idx += kT) {
            const int r = idx / (2 * N), q = idx - r * (2 * N);
            if (r == k) continue;
            const double f = Mm[r * ld + k];
            if (q < N) {
                if (q != k) Mm[r * ld + q] = fma(-f, Mm[k * ld + q], Mm[r * ld + q]);
            } else {
                Mi[r * ldi + q - N] = fma(-f, Mi[k * ldi + q - N], Mi[r * ldi + q - N]);
            }
        }
        bsync();
        if (t < N && t != k) Mm[t * ld + k] = 0.0;
        bsync();
    }
}

// LDS R x Q block (leading dimension ld) <- global rows R0 x cols Q0 (row
// stride gq), zero padded, `diag` on the padded diagonal.
template <int R, int Q>
BDI void bload(double* l, int ld, const double* g, int gq, int R0, int Q0, double diag = 0.0) {
    for (int idx = threadIdx.x; idx < R * Q; idx += kT) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        l[r * ld + q] = (r < R0 && q < Q0) ? g[r * gq + q] : ((r == q && r >= R0) ? diag : 0.0);
    }
    bsync();
}

// global (row stride gq) <- the leading R0 x Q0 block of an LDS matrix
template <typename OT>
BDI void bstore(OT* g, int gq, const double* l, int ld, int R0, int Q0) {
    for (int idx = threadIdx.x; idx < R0 * Q0; idx += kT) {
        const int r = idx / Q0, q = idx - (idx / Q0) * Q0;
        g[r * gq + q] = (OT)l[r * ld + q];
    }
}

// ---- b_prep: padded constants and terminal value ---------------------------------

__global__ __launch_bounds__(kT) void b_prep(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    const int i = blockIdx.x;
    if (i >= ninst) return;
    const GInst& I = inst[i];
    const int t = threadIdx.x;
    const int n = I.n, m = I.m, p = I.p, pT = I.pT;
    const InstWs ws = inst_ws(I);
    double* cst = ws.cst;
    if (t == 0 && I.status) *I.status = 0;
    double* H = dyn;            // N x LN
    double* X = H + N * LN;     // N x LN
    double* Wm = X + N * LN;    // N x LN
    double* Um = Wm + N * LN;   // M x LM
    double* Ri = Um + M * LM;   // M x LM
    double* Lm = Ri + M * LM;   // N x LM
    double* vec = Lm + N * LM;  // 2 N
    for (int idx = t; idx < N * N; idx += kT) {
        const int r = idx / N, q = idx - (idx / N) * N;
        cst[CstB::F + idx] = (r < n && q < n) ? I.F[r * n + q] : 0.0;
    }
    for (int idx = t; idx < N * M; idx += kT) {
        const int r = idx / M, q = idx - (idx / M) * M;
        cst[CstB::L + idx] = (r < n && q < m) ? I.L[r * m + q] : 0.0;
    }
    // U symmetrised, identity on the padding
    for (int idx = t; idx < M * M; idx += kT) {
        const int a = idx / M, b = idx - (idx / M) * M;
        const double u = (a < m && b < m) ? 0.5 * (I.U[a * m + b] + I.U[b * m + a]) : (a == b ? 1.0 : 0.0);
        Um[a * LM + b] = u;
        cst[CstB::U + idx] = u;
    }
    bload<N, M>(Lm, LM, I.L, m, n, m);  // (barrier)
    const bool ok = bchol(Um, LM, m);
    btrinv(Um, LM, Ri, LM, m);
    // G = L R_U^{-T}: G G^T = L U^{-1} L^T
    bgemm<N, M, M, false, true, false>(Lm, LM, Ri, LM, cst + CstB::G, M, 1.0, 0.0);
    // W = H^T X (n x p), J = W H
    bload<N, N>(H, LN, I.H, n, p, n);
    bload<N, N>(X, LN, I.X, p, p, p);
    bgemm<N, N, N, true, false, false>(H, LN, X, LN, Wm, LN, 1.0, 0.0);
    for (int idx = t; idx < N * N; idx += kT) cst[CstB::W + idx] = Wm[(idx / N) * LN + idx % N];
    bgemm<N, N, N, false, false, true>(Wm, LN, H, LN, cst + CstB::J, N, 1.0, 0.0);
    // terminal value S_T = H_T^T X_T H_T, v_T = H_T^T X_T r_T (Section IV-B,
    // terminal element with the terminal weight)
    bload<N, N>(H, LN, I.HT, n, pT, n);
    bload<N, N>(X, LN, I.XT, pT, pT, pT);
    if (t < N) vec[t] = (t < pT) ? I.rT[t] : 0.0;
    bgemm<N, N, N, true, false, false>(H, LN, X, LN, Wm, LN, 1.0, 0.0);
    bgemm<N, N, N, false, false, true>(Wm, LN, H, LN, cst + CstB::ST, N, 1.0, 0.0);
    bgemv<N, N, false>(Wm, LN, vec, vec + N, 1.0, 0.0);
    if (t < N) cst[CstB::VT + t] = vec[N + t];
    if (!ok && t == 0) raise_status(I.status, 3);
}

// Per-step vectors of step k: c_k (zero padded) and eta_k = W r_k.
BDI void step_vectors(const GInst& I, const double* Wg, int64_t k, double* cc, double* ek) {
    const int t = threadIdx.x;
    const int n = I.n, p = I.p;
    if (t < N) {
        cc[t] = (I.c && t < n) ? step_ptr(I.c, I.per_step, kPS_c, k, n)[t] : 0.0;
        const double* r = I.r + k * p;
        double s = 0.0;
        for (int j = 0; j < p; ++j) s = fma(Wg[t * N + j], r[j], s);
        ek[t] = s;
    }
    bsync();
}

// ---- b_fold: chunk element ---------------------------------------------------------

constexpr size_t kFoldLds = sizeof(double) * (3 * N * LN + M * LN + 2 * M * LM + N * LM + 10 * N);

__global__ __launch_bounds__(kT) void b_fold(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    const int t = threadIdx.x;
    const int m = I.m;
    const InstWs ws = inst_ws(I);
    const double* Fg = ws.cst + CstB::F;
    const double* Gg = ws.cst + CstB::G;
    const double* Jg = ws.cst + CstB::J;
    const double* Wg = ws.cst + CstB::W;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double* PA = dyn;
    double* PC = PA + N * LN;
    double* PJ = PC + N * LN;
    double* V = PJ + N * LN;   // M x LN
    double* Rm = V + M * LN;   // M x LM
    double* Ri = Rm + M * LM;  // M x LM
    double* Q = Ri + M * LM;   // N x LM
    double* vb = Q + N * LM;
    double *Pb = vb, *Pe = vb + N, *cc = vb + 2 * N, *ek = vb + 3 * N, *h = vb + 4 * N, *g = vb + 5 * N;
    double *hw = vb + 6 * N, *w1 = vb + 7 * N, *w2 = vb + 8 * N, *jc = vb + 9 * N;
    bool ok = true;
    // the chunk's last step: P = a_{k1-1}
    step_vectors(I, Wg, k1 - 1, cc, ek);
    bload<N, N>(PA, LN, Fg, N, N, N);
    bload<N, N>(PJ, LN, Jg, N, N, N);
    bgemm<N, N, M, false, true, true>(Gg, M, Gg, M, PC, LN, 1.0, 0.0);
    if (t < N) {
        Pb[t] = cc[t];
        Pe[t] = ek[t];
    }
    bsync();
#pragma unroll 1
    for (int64_t k = k1 - 2; k >= k0; --k) {
        step_vectors(I, Wg, k, cc, ek);
        // Z = G^T J_P (into V); W = I + Z G
        bgemm<M, N, N, true, false, false>(Gg, M, PJ, LN, V, LN, 1.0, 0.0);
        bgemm<M, M, N, false, false, true>(V, LN, Gg, M, Rm, LM, 1.0, 0.0);
        if (t < M) Rm[t * LM + t] += 1.0;
        // h = G^T eta_P - Z c ; jc = J_P c
        if (t < M) {
            double s = 0.0;
            for (int j = 0; j < N; ++j) s = fma(Gg[j * M + t], Pe[j], s);
            for (int j = 0; j < N; ++j) s = fma(-V[t * LN + j], cc[j], s);
            h[t] = s;
        } else if (t >= 64 && t < 64 + N) {
            const int r = t - 64;
            double s = 0.0;
            for (int j = 0; j < N; ++j) s = fma(PJ[r * LN + j], cc[j], s);
            jc[r] = s;
        }
        bsync();
        ok = bchol(Rm, LM, m) && ok;  // W >= I: fails only on non-finite data
        btrinv(Rm, LM, Ri, LM, m);
        // V = R^{-1} Z ; g = R^{-1} h ; hw = W^{-1} h = R^{-T} g
        bgemm<M, N, M, false, false, false>(Ri, LM, V, LN, V, LN, 1.0, 0.0);
        bgemv<M, M, false>(Ri, LM, h, g, 1.0, 0.0);
        bgemv<M, M, true>(Ri, LM, g, hw, 1.0, 0.0);
        // w1 = eta_P - J_P c - V^T g ; w2 = c + G hw
        if (t < N) {
            double s = Pe[t] - jc[t];
            for (int i = 0; i < M; ++i) s = fma(-V[i * LN + t], g[i], s);
            w1[t] = s;
        } else if (t >= 64 && t < 64 + N) {
            const int r = t - 64;
            double s = cc[r];
            for (int q = 0; q < M; ++q) s = fma(Gg[r * M + q], hw[q], s);
            w2[r] = s;
        }
        bsync();
        // eta' = F^T w1 + eta_k ; b' = A_P w2 + b_P
        if (t < N) {
            double s = ek[t];
            for (int j = 0; j < N; ++j) s = fma(Fg[j * N + t], w1[j], s);
            Pe[t] = s;
        } else if (t >= 64 && t < 64 + N) {
            const int r = t - 64;
            double s = Pb[r];
            for (int j = 0; j < N; ++j) s = fma(PA[r * LN + j], w2[j], s);
            Pb[r] = s;
        }
        bsync();
        // Q = A_P G R^{-T}
        bgemm<N, M, N, false, false, false>(PA, LN, Gg, M, Q, LM, 1.0, 0.0);
        bgemm<N, M, M, false, true, false>(Q, LM, Ri, LM, Q, LM, 1.0, 0.0);
        // C' = C_P + Q Q^T ; J_P - V^T V
        bgemm<N, N, M, false, true, true>(Q, LM, Q, LM, PC, LN, 1.0, 1.0);
        bgemm<N, N, M, true, false, true>(V, LN, V, LN, PJ, LN, -1.0, 1.0);
        // A' = A_P F - Q (V F)
        bgemm<M, N, N, false, false, false>(V, LN, Fg, N, V, LN, 1.0, 0.0);
        bgemm<N, N, N, false, false, false, M, false, false>(PA, LN, Fg, N, PA, LN, 1.0, 0.0, nullptr, 0, Q, LM, V,
                                                             LN, -1.0);
        // J' = F^T (J_P - V^T V) F + J_k
        bgemm<N, N, N, false, false, false>(PJ, LN, Fg, N, PJ, LN, 1.0, 0.0);
        bgemm<N, N, N, true, false, true>(Fg, N, PJ, LN, PJ, LN, 1.0, 0.0, Jg, N);
    }
    double* out = ws.agg + c * elem_doubles(N);
    for (int idx = t; idx < N * N; idx += kT) {
        const int r = idx / N, q = idx - (idx / N) * N;
        out[idx] = PA[r * LN + q];
        out[N * N + N + idx] = PC[r * LN + q];
        out[2 * N * N + 2 * N + idx] = PJ[r * LN + q];
    }
    if (t < N) {
        out[N * N + t] = Pb[t];
        out[2 * N * N + N + t] = Pe[t];
    }
    if (!ok && t == 0) raise_status(I.status, 3);
}

// ---- b_chain: value function at every chunk start -------------------------------------

constexpr size_t kChainLds = sizeof(double) * (3 * N * LN + 4 * N) + 64;

__global__ __launch_bounds__(kT) void b_chain(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    const int t = threadIdx.x;
    const InstWs ws = inst_ws(I);
    double* S = dyn;
    double* Mm = S + N * LN;
    double* Mi = Mm + N * LN;
    double* v = Mi + N * LN;
    double* tv = v + N;
    double* nv = tv + N;
    int* piv = (int*)(nv + 2 * N);
    bload<N, N>(S, LN, ws.cst + CstB::ST, N, N, N);
    if (t < N) v[t] = ws.cst[CstB::VT + t];
    bsync();
    const int64_t VD = val_doubles(N);
    double* vo = ws.val + I.NC * VD;
    for (int idx = t; idx < N * N; idx += kT) vo[idx] = S[(idx / N) * LN + idx % N];
    if (t < N) vo[N * N + t] = v[t];
#pragma unroll 1
    for (int64_t c = I.NC - 1; c >= 0; --c) {
        const double* e = ws.agg + c * elem_doubles(N);
        const double *EA = e, *Eb = e + N * N, *EC = e + N * N + N, *Ee = e + 2 * N * N + N;
        const double* EJ = e + 2 * N * N + 2 * N;
        // (S, v) <- E (x) (0, 0, 0, v, S):  M = I + C_E S
        bgemm<N, N, N, false, false, false>(EC, N, S, LN, Mm, LN, 1.0, 0.0);
        if (t < N) Mm[t * LN + t] += 1.0;
        bsync();
        binv(Mm, LN, Mi, LN, piv);
        // T1 = M^{-1} A_E (into Mm)
        bgemm<N, N, N, false, false, false>(Mi, LN, EA, N, Mm, LN, 1.0, 0.0);
        // v' = T1^T (v - S b_E) + eta_E
        if (t < N) {
            double s = v[t];
            for (int j = 0; j < N; ++j) s = fma(-S[t * LN + j], Eb[j], s);
            tv[t] = s;
        }
        bsync();
        if (t < N) {
            double s = Ee[t];
            for (int j = 0; j < N; ++j) s = fma(Mm[j * LN + t], tv[j], s);
            nv[t] = s;
        }
        // P = S A_E (into Mi) ; S' = T1^T P + J_E
        bgemm<N, N, N, false, false, false>(S, LN, EA, N, Mi, LN, 1.0, 0.0);
        bgemm<N, N, N, true, false, true>(Mm, LN, Mi, LN, S, LN, 1.0, 0.0, EJ, N);
        if (t < N) v[t] = nv[t];
        bsync();
        vo = ws.val + c * VD;
        for (int idx = t; idx < N * N; idx += kT) vo[idx] = S[(idx / N) * LN + idx % N];
        if (t < N) vo[N * N + t] = v[t];
    }
}

// ---- b_final: values, gains and the chunk's closed-loop map ---------------------------------

constexpr size_t kFinalLds = sizeof(double) * (3 * N * LN + N * LM + 2 * M * LM + M * LN + 12 * N);

template <typename OT>
__global__ __launch_bounds__(kT) void b_final(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    const int t = threadIdx.x;
    const int n = I.n, m = I.m;
    const InstWs ws = inst_ws(I);
    const double* Fg = ws.cst + CstB::F;
    const double* Lg = ws.cst + CstB::L;
    const double* Ug = ws.cst + CstB::U;
    const double* Jg = ws.cst + CstB::J;
    const double* Wg = ws.cst + CstB::W;
    OT* const oS = (OT*)I.S;
    OT* const oV = (OT*)I.v;
    OT* const oK = (OT*)I.K;
    OT* const oD = (OT*)I.d;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double* S = dyn;
    double* SF = S + N * LN;
    double* Phi = SF + N * LN;
    double* B1 = Phi + N * LN;  // N x LM: S L, then Phi L
    double* Rm = B1 + N * LM;   // M x LM
    double* Ri = Rm + M * LM;   // M x LM
    double* V = Ri + M * LM;    // M x LN: R^{-1} L^T S F, then K
    double* vb = V + M * LN;
    double *v = vb, *cc = vb + N, *ek = vb + 2 * N, *w = vb + 3 * N, *z = vb + 4 * N, *zz = vb + 5 * N;
    double *d = vb + 6 * N, *nv = vb + 7 * N, *ct = vb + 8 * N, *phi = vb + 9 * N, *t9 = vb + 10 * N;
    const int64_t VD = val_doubles(N);
    const double* vin = ws.val + (c + 1) * VD;
    bload<N, N>(S, LN, vin, N, N, N);
    for (int idx = t; idx < N * N; idx += kT) {
        const int r = idx / N, q = idx - (idx / N) * N;
        Phi[r * LN + q] = (r == q) ? 1.0 : 0.0;
    }
    if (t < N) {
        v[t] = vin[N * N + t];
        phi[t] = 0.0;
    }
    bsync();
    if (k1 == I.T) {
        if (oS) bstore(oS + I.T * n * n, n, S, LN, n, n);
        if (oV && t < n) oV[I.T * n + t] = (OT)v[t];
    }
    double fin = 0.0;
    bool ok = true;
#pragma unroll 1
    for (int64_t k = k1 - 1; k >= k0; --k) {
        step_vectors(I, Wg, k, cc, ek);
        // M_k = L^T S L + U = R R^T
        bgemm<N, M, N, false, false, false>(S, LN, Lg, M, B1, LM, 1.0, 0.0);
        bgemm<M, M, N, true, false, true>(Lg, M, B1, LM, Rm, LM, 1.0, 0.0, Ug, M);
        ok = bchol(Rm, LM, m) && ok;
        btrinv(Rm, LM, Ri, LM, m);
        // SF = S F ; V = R^{-1} L^T S F
        bgemm<N, N, N, false, false, false>(S, LN, Fg, N, SF, LN, 1.0, 0.0);
        bgemm<M, N, N, true, false, false>(Lg, M, SF, LN, V, LN, 1.0, 0.0);
        bgemm<M, N, M, false, false, false>(Ri, LM, V, LN, V, LN, 1.0, 0.0);
        // w = v - S c ; z = L^T w ; zz = R^{-1} z ; d = R^{-T} zz
        if (t < N) {
            double s = v[t];
            for (int j = 0; j < N; ++j) s = fma(-S[t * LN + j], cc[j], s);
            w[t] = s;
        }
        bsync();
        bgemv<M, N, true>(Lg, M, w, z, 1.0, 0.0);
        bgemv<M, M, false>(Ri, LM, z, zz, 1.0, 0.0);
        bgemv<M, M, true>(Ri, LM, zz, d, 1.0, 0.0);
        // v' = F^T w - V^T zz + eta_k (= F^T w - K^T z + eta_k)
        if (t < N) {
            double s = ek[t];
            for (int j = 0; j < N; ++j) s = fma(Fg[j * N + t], w[j], s);
            for (int i = 0; i < M; ++i) s = fma(-V[i * LN + t], zz[i], s);
            nv[t] = s;
        }
        // S' = F^T S F - V^T V + J (= F^T S F - P^T M^{-1} P + J)
        bgemm<N, N, N, true, false, true, M, true, false>(Fg, N, SF, LN, S, LN, 1.0, 0.0, Jg, N, V, LN, V, LN,
                                                          -1.0);
        if (t < N) v[t] = nv[t];
        // K = R^{-T} V
        bgemm<M, N, M, true, false, false>(Ri, LM, V, LN, V, LN, 1.0, 0.0);
        // c~ = c + L d
        if (t < N) {
            double s = cc[t];
            for (int q = 0; q < M; ++q) s = fma(Lg[t * M + q], d[q], s);
            ct[t] = s;
        }
        bsync();
        if (oS) bstore(oS + k * n * n, n, S, LN, n, n);
        if (oV && t < n) oV[k * n + t] = (OT)v[t];
        bstore(oK + k * m * n, n, V, LN, m, n);
        if (t < m) oD[k * m + t] = (OT)d[t];
        for (int idx = t; idx < n * n; idx += kT) fin += S[(idx / n) * LN + idx % n];
        if (t < n) fin += v[t];
        // chunk map: phi <- Phi c~ + phi ; Phi <- Phi (F - L K)
        bgemv<N, N, false>(Phi, LN, ct, t9, 1.0, 0.0);
        if (t < N) phi[t] += t9[t];
        bgemm<N, M, N, false, false, false>(Phi, LN, Lg, M, B1, LM, 1.0, 0.0);
        bgemm<N, N, N, false, false, false, M, false, false>(Phi, LN, Fg, N, Phi, LN, 1.0, 0.0, nullptr, 0, B1, LM,
                                                             V, LN, -1.0);
    }
    double* mo = ws.map + c * VD;
    for (int idx = t; idx < N * N; idx += kT) mo[idx] = Phi[(idx / N) * LN + idx % N];
    if (t < N) mo[N * N + t] = phi[t];
    if (!isfinite(fin)) raise_status(I.status, 4);
    if (!ok && t == 0) raise_status(I.status, 3);
}

// ---- forward pass ------------------------------------------------------------------------

constexpr size_t kSmallLds = sizeof(double) * 4 * N;

__global__ __launch_bounds__(kT) void b_fchain(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    const int t = threadIdx.x;
    const InstWs ws = inst_ws(I);
    double* x = dyn;
    double* y = x + N;
    if (t < N) x[t] = (t < I.n) ? I.x0[t] : 0.0;
    bsync();
    const int64_t VD = val_doubles(N);
#pragma unroll 1
    for (int64_t c = 0; c < I.NC; ++c) {
        if (t < N) ws.xs[c * N + t] = x[t];
        const double* mp = ws.map + c * VD;
        if (t < N) {
            double s = mp[N * N + t];
            for (int q = 0; q < N; ++q) s = fma(mp[t * N + q], x[q], s);
            y[t] = s;
        }
        bsync();
        if (t < N) x[t] = y[t];
        bsync();
    }
}

template <typename OT>
__global__ __launch_bounds__(kT) void b_roll(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    const int t = threadIdx.x;
    const int n = I.n, m = I.m;
    const InstWs ws = inst_ws(I);
    const double* Fg = ws.cst + CstB::F;
    const double* Lg = ws.cst + CstB::L;
    const OT* const iK = (const OT*)I.K;
    const OT* const iD = (const OT*)I.d;
    OT* const oX = (OT*)I.x;
    OT* const oU = (OT*)I.u;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double* x = dyn;
    double* u = x + N;
    double* y = u + N;
    if (t < N) {
        x[t] = ws.xs[c * N + t];
        u[t] = 0.0;
    }
    bsync();
    double fin = 0.0;
#pragma unroll 1
    for (int64_t k = k0; k < k1; ++k) {
        if (t < m) {
            const OT* Kk = iK + k * m * n;
            double s = (double)iD[k * m + t];
            for (int j = 0; j < n; ++j) s = fma(-(double)Kk[t * n + j], x[j], s);
            u[t] = s;
        }
        bsync();
        if (oX && t < n) oX[k * n + t] = (OT)x[t];
        if (oU && t < m) oU[k * m + t] = (OT)u[t];
        if (t < N) {
            double s = (I.c && t < n) ? step_ptr(I.c, I.per_step, kPS_c, k, n)[t] : 0.0;
            for (int q = 0; q < N; ++q) s = fma(Fg[t * N + q], x[q], s);
            for (int q = 0; q < M; ++q) s = fma(Lg[t * M + q], u[q], s);
            y[t] = s;
            fin += s;
        }
        bsync();
        if (t < N) x[t] = y[t];
        bsync();
    }
    if (k1 == I.T && oX && t < n) oX[I.T * n + t] = (OT)x[t];
    if (!isfinite(fin)) raise_status(I.status, 4);
}

constexpr size_t kPrepLds = sizeof(double) * (3 * N * LN + 2 * M * LM + N * LM + 2 * N);

struct BStage {
    const StageHook* h;
    hipStream_t s;
    BStage(const StageHook* hook, const char* name, hipStream_t st) : h(hook), s(st) {
        if (h) h->begin(h->ctx, name, s);
    }
    ~BStage() {
        if (h) h->end(h->ctx, s);
    }
};

template <typename OT>
void run_block(const GInst* d_inst, int ninst, int64_t nchunks, bool want_fwd, hipStream_t s, const StageHook* h) {
    static bool attr = false;
    if (!attr) {
        const void* ks[] = {(const void*)b_prep, (const void*)b_fold, (const void*)b_chain,
                            (const void*)b_final<OT>};
        for (const void* k : ks) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    {
        BStage st(h, "t64_prep", s);
        b_prep<<<ninst, kT, kPrepLds, s>>>(d_inst, ninst);
    }
    {
        BStage st(h, "t64_fold", s);
        b_fold<<<(unsigned)nchunks, kT, kFoldLds, s>>>(d_inst, ninst, nchunks);
    }
    {
        BStage st(h, "t64_chain", s);
        b_chain<<<ninst, kT, kChainLds, s>>>(d_inst, ninst);
    }
    {
        BStage st(h, "t64_final", s);
        b_final<OT><<<(unsigned)nchunks, kT, kFinalLds, s>>>(d_inst, ninst, nchunks);
    }
    if (want_fwd) {
        {
            BStage st(h, "t64_fchain", s);
            b_fchain<<<ninst, kT, kSmallLds, s>>>(d_inst, ninst);
        }
        BStage st(h, "t64_roll", s);
        b_roll<OT><<<(unsigned)nchunks, kT, kSmallLds, s>>>(d_inst, ninst, nchunks);
    }
}

static_assert(kFoldLds <= 160 * 1024 && kFinalLds <= 160 * 1024 && kChainLds <= 160 * 1024 &&
                  kPrepLds <= 160 * 1024,
              "LDS budget of the workgroup class");

}  // namespace

hipError_t block_solve(const GInst* d_inst, int ninst, int64_t nchunks, bool want_fwd, bool f32, hipStream_t s,
                       const StageHook* h) {
    if (f32) run_block<float>(d_inst, ninst, nchunks, want_fwd, s, h);
    else run_block<double>(d_inst, ninst, nchunks, want_fwd, s, h);
    return hipGetLastError();
}

}  // namespace lqt
