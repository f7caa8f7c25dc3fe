// Wavefront-per-chunk LQT pipeline for general state dimension (gfx950).
//
// One wavefront owns one chunk of B consecutive steps of one instance.  The
// element being folded and every temporary live in the wavefront's slice of
// LDS; the 64 lanes cooperate on every matrix product, factorisation and
// solve.  Matrices are zero-padded to a size class N x N (N = 8, 16, 32) so
// that every loop is unrolled at compile time.  All instances of a size class
// share each launch: the flat chunk index is mapped to its instance by a
// binary search over the instances' first chunk.
//
// Phases (the reduce-then-scan organisation of the block processing of
// Section V-C, with the per-instance top level done sequentially -- a batch
// has far more instances than the GPU has SIMDs):
//   g_prep    per instance: G (G G^T = L U^{-1} L^T), J = H^T X H, W = H^T X
//             and the terminal value S_T = H_T^T X_T H_T, v_T = H_T^T X_T r_T;
//   t_fold    per chunk: fold the one-step elements a_k (Section IV-B) with
//             the combination rule (Section IV-A) into the chunk element;
//   t_chain   per instance: value function at every chunk start, walking the
//             chunks from the terminal value with the anchored combination
//             (instances with many chunks: t_tlevel + t_tanchor, the scan
//             over the chunk elements as a tree);
//   t_final   per chunk: down-sweep in Riccati form fused with the gain
//             extraction (writes S, v, K, d) and the chunk's closed-loop map;
//   t_fchain  per instance: state at every chunk start from x_0 (Method 1
//             affine maps, Section IV-C);
//   t_roll    per chunk: u_k = -K_k x_k + d_k, x_{k+1} = F x_k + c + L u_k.
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_ws.hpp"

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

// ---- per-instance descriptor helpers -------------------------------------------

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

}  // namespace

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

// ---- forward pass ------------------------------------------------------------------

// ============================================================================
// Size-class kernels: every matrix is zero-padded to a compile-time N x N
// (N = 8, 16, 32), so all loops unroll and each lane owns a fixed output tile
// of every product (an 8 x 8 grid of tiles covers the N x N result).  The
// padding is exact: F, G, L, J, S, C, x are zero outside the n / m block, and
// every matrix that is factorised or inverted (U, I + G^T J G, I + C S,
// L^T S L + U) is the identity there.
// ============================================================================

template <int N>
struct TL {
    // 16-byte aligned rows, rows spread over the banks; class 8 unpadded (a
    // smaller LDS footprint keeps more wavefronts resident)
    static constexpr int ld = N == 8 ? 8 : N + 2;
    static constexpr int mat = N * ld;
    static constexpr int T = N / 8;    // per-lane output tile is T x T
};

typedef double dvec4 __attribute__((ext_vector_type(4)));
constexpr bool kT8Mfma = true;  // class-8 products on the matrix cores

// C = alpha op(A) op(B) + beta C on the matrix cores (N = 16, 32): 16 x 16
// output tiles, 16 x 16 x 4 FP64 MFMA per k-slice.  Operand layout (measured
// on gfx950): lane l supplies A[l % 16][4s + l / 16] and B[4s + l / 16][l % 16];
// accumulator element v of lane l is C[l / 16 + 4 v][l % 16].
template <int N, bool TA, bool TB, bool SYM>
WDI void tgemm_mfma(const double* A, const double* B, double* C, double alpha, double beta, int lane) {
    constexpr int ld = TL<N>::ld, NT = N / 16;
    const int i0 = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < NT; ++bi)
#pragma unroll
        for (int bj = 0; bj < NT; ++bj) {
            if (SYM && bi > bj) continue;
            dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < N / 4; ++s4) {
                const int kx = 4 * s4 + kk;
                const int ar = 16 * bi + i0, bc = 16 * bj + i0;
                const double a = TA ? A[kx * ld + ar] : A[ar * ld + kx];
                const double b = TB ? B[bc * ld + kx] : B[kx * ld + bc];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            double out[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bi + kk + 4 * v, c = 16 * bj + i0;
                out[v] = (beta == 0.0) ? alpha * acc[v] : fma(alpha, acc[v], beta * C[r * ld + c]);
            }
            // every lane has read its C inputs before any tile entry is written
            if (SYM) wsync();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bi + kk + 4 * v, c = 16 * bj + i0;
                if (SYM && r > c) continue;  // written as the mirror of (c, r)
                C[r * ld + c] = out[v];
                if (SYM) C[c * ld + r] = out[v];
            }
        }
    wsync();
}

// The same for N = 8 on the matrix cores: one 16 x 16 output tile whose rows
// and columns beyond 8 are never read (their lanes supply zeros) and a
// reduction of two 4-deep steps; per lane four LDS reads and two writes
// instead of the sixteen reads of the per-lane VALU tile.
template <bool TA, bool TB, bool SYM>
WDI void tgemm8_mfma(const double* A, const double* B, double* C, double alpha, double beta, int lane) {
    constexpr int ld = TL<8>::ld;
    const int i0 = lane & 15, kk = lane >> 4;
    const bool in = i0 < 8;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
        const int kx = 4 * s4 + kk;
        const double a = in ? (TA ? A[kx * ld + i0] : A[i0 * ld + kx]) : 0.0;
        const double b = in ? (TB ? B[i0 * ld + kx] : B[kx * ld + i0]) : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double out[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {  // rows kk + 4 v < 8 of column i0
        const int r = kk + 4 * v;
        out[v] = (beta == 0.0 || !in) ? alpha * acc[v] : fma(alpha, acc[v], beta * C[r * ld + i0]);
    }
    if (SYM) wsync();
    if (in) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int r = kk + 4 * v;
            if (SYM && r > i0) continue;  // written as the mirror of (i0, r)
            C[r * ld + i0] = out[v];
            if (SYM) C[i0 * ld + r] = out[v];
        }
    }
    wsync();
}

// C = alpha op(A) op(B) + beta C, all N x N.  sym: the result is symmetric;
// only tiles on or above the diagonal are computed and each value is written
// to both mirrored positions (exactly symmetric).
template <int N, bool TA, bool TB, bool SYM = false>
WDI void tgemm(const double* A, const double* B, double* C, double alpha, double beta, int lane) {
    if constexpr (N >= 16) {
        tgemm_mfma<N, TA, TB, SYM>(A, B, C, alpha, beta, lane);
        return;
    }
    if constexpr (N == 8 && kT8Mfma) {
        tgemm8_mfma<TA, TB, SYM>(A, B, C, alpha, beta, lane);
        return;
    }
    constexpr int ld = TL<N>::ld, T = TL<N>::T;
    const int tr = lane >> 3, tc = lane & 7;
    const int r0 = tr * T, c0 = tc * T;
    if (!(SYM && tr > tc)) {
        double acc[T][T];
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j) acc[i][j] = 0.0;
#pragma unroll 8
        for (int k = 0; k < N; ++k) {
            double a[T], b[T];
#pragma unroll
            for (int i = 0; i < T; ++i) a[i] = TA ? A[k * ld + r0 + i] : A[(r0 + i) * ld + k];
#pragma unroll
            for (int j = 0; j < T; ++j) b[j] = TB ? B[(c0 + j) * ld + k] : B[k * ld + c0 + j];
#pragma unroll
            for (int i = 0; i < T; ++i)
#pragma unroll
                for (int j = 0; j < T; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        double out[T][T];
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j)
                out[i][j] = (beta == 0.0) ? alpha * acc[i][j] : fma(alpha, acc[i][j], beta * C[(r0 + i) * ld + c0 + j]);
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j) {
                if (SYM && tr == tc && j < i) continue;  // lower part of a diagonal tile: mirror of (j, i)
                C[(r0 + i) * ld + c0 + j] = out[i][j];
                if (SYM) C[(c0 + j) * ld + r0 + i] = out[i][j];
            }
    }
    wsync();
}

// y = alpha op(A) x + beta y (N x N, vectors of N)
template <int N, bool TA>
WDI void tgemv(const double* A, const double* x, double* y, double alpha, double beta, int lane) {
    constexpr int ld = TL<N>::ld;
    if (lane < N) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) s = fma(TA ? A[k * ld + lane] : A[lane * ld + k], x[k], s);
        y[lane] = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * y[lane]);
    }
    wsync();
}

template <int N>
WDI void tcopy(const double* A, double* B, int lane) {
    constexpr int ld = TL<N>::ld;
    for (int idx = lane; idx < N * N; idx += kW) B[(idx / N) * ld + (idx % N)] = A[(idx / N) * ld + (idx % N)];
    wsync();
}

template <int N>
WDI void tzero(double* A, int lane) {
    constexpr int ld = TL<N>::ld;
    for (int idx = lane; idx < N * N; idx += kW) A[(idx / N) * ld + (idx % N)] = 0.0;
    wsync();
}

// Lower Cholesky factor in place; upper triangle zeroed.
template <int N>
WDI bool tchol(double* A, int lane) {
    constexpr int ld = TL<N>::ld;
    bool ok = true;
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
        double s = A[j * ld + j];
        for (int k = 0; k < j; ++k) s = fma(-A[j * ld + k], A[j * ld + k], s);
        ok = ok && (s > 0.0);
        const double rjj = sqrt(s);
        const double rinv = 1.0 / rjj;
        wsync();
        if (lane == j) A[j * ld + j] = rjj;
        if (lane > j && lane < N) {
            double t = A[lane * ld + j];
            for (int k = 0; k < j; ++k) t = fma(-A[lane * ld + k], A[j * ld + k], t);
            A[lane * ld + j] = t * rinv;
        }
        if (lane < j) A[lane * ld + j] = 0.0;
        wsync();
    }
    return ok;
}

// B <- R^{-1} B (R lower, N x N); lane c updates column c in place.
template <int N>
WDI void ttrsm_l(const double* R, double* B, int lane) {
    constexpr int ld = TL<N>::ld;
    if (lane < N) {
#pragma unroll 1
        for (int i = 0; i < N; ++i) {
            double s = B[i * ld + lane];
#pragma unroll 4
            for (int k = 0; k < i; ++k) s = fma(-R[i * ld + k], B[k * ld + lane], s);
            B[i * ld + lane] = s / R[i * ld + i];
        }
    }
    wsync();
}

// Lower Cholesky factor of the leading m x m block in place (upper triangle
// zeroed); the padded block is the identity and stays so.  Returns false if a
// pivot is not > 0 (including NaN).
template <int N>
WDI bool tchol_m(double* A, int m, int lane) {
    constexpr int ld = TL<N>::ld;
    bool ok = true;
#pragma unroll 1
    for (int j = 0; j < m; ++j) {
        double s = A[j * ld + j];
        for (int k = 0; k < j; ++k) s = fma(-A[j * ld + k], A[j * ld + k], s);
        ok = ok && (s > 0.0);
        const double rjj = sqrt(s);
        const double rinv = 1.0 / rjj;
        wsync();
        if (lane == j) A[j * ld + j] = rjj;
        if (lane > j && lane < m) {
            double t = A[lane * ld + j];
            for (int k = 0; k < j; ++k) t = fma(-A[lane * ld + k], A[j * ld + k], t);
            A[lane * ld + j] = t * rinv;
        }
        if (lane < j) A[lane * ld + j] = 0.0;
        wsync();
    }
    return ok;
}

// Triangular solves with the factor R of tchol_m (rows and columns >= m are
// the identity): B <- R^{-1} B (forward) or B <- R^{-T} B (backward) for the
// N columns of B, lane c solving column c, and, when x is given, the vector x
// solved the same way by lane N (a wavefront has 64 lanes, N <= 32).
template <int N, bool TRANS>
WDI void ttrsm_m(const double* R, double* B, double* x, int m, int lane) {
    constexpr int ld = TL<N>::ld;
    if (lane < N || (x && lane == N)) {
        double* col = lane < N ? B + lane : x;
        const int cs = lane < N ? ld : 1;
        if (!TRANS) {
#pragma unroll 1
            for (int i = 0; i < m; ++i) {
                double s = col[i * cs];
#pragma unroll 4
                for (int k = 0; k < i; ++k) s = fma(-R[i * ld + k], col[k * cs], s);
                col[i * cs] = s / R[i * ld + i];
            }
        } else {
#pragma unroll 1
            for (int i = m - 1; i >= 0; --i) {
                double s = col[i * cs];
#pragma unroll 4
                for (int k = i + 1; k < m; ++k) s = fma(-R[k * ld + i], col[k * cs], s);
                col[i * cs] = s / R[i * ld + i];
            }
        }
    }
    wsync();
}

WDI double rlane64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __hiloint2double(hi, lo);
}

// Mi = M^{-1} for N <= 16, Gauss-Jordan with partial pivoting in registers:
// lane r < N keeps row r of [M | I]; a column's pivot is the largest
// magnitude among the rows not yet pivots (wavefront reduction), the pivot
// row is read lane to lane by the whole wavefront and every other row is
// eliminated in place.  Rows are not exchanged: row c of the inverse is the
// identity part of the c-th pivot row.  No LDS traffic and no wavefront
// ordering inside the elimination.
template <int N>
WDI void tinv_reg(const double* Mm, double* Mi, int lane) {
    constexpr int ld = TL<N>::ld;
    const int r = lane;
    const bool act = r < N;
    double a[2 * N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        a[j] = act ? Mm[r * ld + j] : 0.0;
        a[N + j] = (act && r == j) ? 1.0 : 0.0;
    }
    bool used = !act;
    int ci = 0;  // this row's place in the pivot order
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double best = used ? -1.0 : fabs(a[k]);
        int bi = r;
#pragma unroll
        for (int off = kW / 2; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, kW);
            const int oi = __shfl_xor(bi, off, kW);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int p = __builtin_amdgcn_readfirstlane(bi);
        const double inv = 1.0 / rlane64(a[k], p);
        const bool me = r == p;
        const double f = me ? 0.0 : a[k] * inv;
        // columns before k are unit vectors already (zero in the pivot row)
#pragma unroll
        for (int j = k + 1; j < 2 * N; ++j) {
            const double pj = rlane64(a[j], p);
            a[j] = me ? pj * inv : fma(-f, pj, a[j]);
        }
        a[k] = me ? 1.0 : 0.0;
        if (me) ci = k;
        used = used || me;
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < N; ++j) Mi[ci * ld + j] = a[N + j];
    }
    wsync();
}

// Mi = M^{-1}, Gauss-Jordan with partial pivoting (M destroyed): the register
// form up to N = 16, else in LDS with explicit row exchanges.
template <int N>
WDI void tinv(double* Mm, double* Mi, int lane) {
    if constexpr (N <= 16) {
        tinv_reg<N>(Mm, Mi, lane);
        return;
    }
    constexpr int ld = TL<N>::ld;
    for (int idx = lane; idx < N * N; idx += kW) {
        const int r = idx / N, q = idx % N;
        Mi[r * ld + q] = (r == q) ? 1.0 : 0.0;
    }
    wsync();
#pragma unroll 1
    for (int k = 0; k < N; ++k) {
        double best = -1.0;
        int bi = k;
        if (lane >= k && lane < N) {
            best = fabs(Mm[lane * ld + k]);
            bi = lane;
        }
        for (int off = kW / 2; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, kW);
            const int oi = __shfl_xor(bi, off, kW);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int p = bi;
        if (p != k) {
            if (lane < N) {
                double t = Mm[k * ld + lane];
                Mm[k * ld + lane] = Mm[p * ld + lane];
                Mm[p * ld + lane] = t;
                t = Mi[k * ld + lane];
                Mi[k * ld + lane] = Mi[p * ld + lane];
                Mi[p * ld + lane] = t;
            }
            wsync();
        }
        const double inv = 1.0 / Mm[k * ld + k];
        wsync();
        if (lane < N) {
            Mm[k * ld + lane] *= inv;
            Mi[k * ld + lane] *= inv;
        }
        wsync();
        for (int idx = lane; idx < N * N; idx += kW) {
            const int r = idx / N, q = idx % N;
            if (r == k) continue;
            const double fr = Mm[r * ld + k];
            Mi[r * ld + q] = fma(-fr, Mi[k * ld + q], Mi[r * ld + q]);
            if (q != k) Mm[r * ld + q] = fma(-fr, Mm[k * ld + q], Mm[r * ld + q]);
        }
        wsync();
        if (lane < N && lane != k) Mm[lane * ld + k] = 0.0;
        wsync();
    }
}

// global (R x Q, row stride gq) -> LDS N x N, zero padded; `diag` on the
// padded diagonal (1 for matrices that are factorised).
template <int N>
WDI void tload(int R, int Q, const double* g, int gq, double* l, int lane, double diag = 0.0) {
    constexpr int ld = TL<N>::ld;
    for (int idx = lane; idx < N * N; idx += kW) {
        const int r = idx / N, q = idx % N;
        l[r * ld + q] = (r < R && q < Q) ? g[r * gq + q] : ((r == q && r >= R) ? diag : 0.0);
    }
    wsync();
}

template <int N, typename OT>
WDI void tstore(int R, int Q, const double* l, OT* g, int gq, int lane) {
    constexpr int ld = TL<N>::ld;
    for (int idx = lane; idx < R * Q; idx += kW) {
        const int r = idx / Q, q = idx - (idx / Q) * Q;
        g[r * gq + q] = (OT)l[r * ld + q];
    }
}

// LDS of a class-N kernel: NM matrix slots, then NV vector slots.  Each
// kernel takes only the slots it uses (and is launched with that much LDS),
// so the kernels with few slots keep more wavefronts resident.
template <int N, int NM = 14, int NV = 12>
struct TSlots {
    double* m[NM];
    double* v[NV];
    static constexpr int NMv = NM, NVv = NV;
    static constexpr int doubles() { return NM * TL<N>::mat + NV * (N + 2); }
    static constexpr size_t bytes() { return sizeof(double) * doubles(); }
};

template <int N, int NM = 14, int NV = 12>
WDI TSlots<N, NM, NV> tslots(double* base) {
    TSlots<N, NM, NV> s;
#pragma unroll
    for (int i = 0; i < NM; ++i) s.m[i] = base + i * TL<N>::mat;
#pragma unroll
    for (int i = 0; i < NV; ++i) s.v[i] = base + NM * TL<N>::mat + i * (N + 2);
    return s;
}

// Slots of each kernel: fold, chain and anchor, tree level, down-sweep,
// forward tree level, roll-out.
template <int N> using FoldSlots = TSlots<N, 12, 10>;
template <int N> using ChainSlots = TSlots<N, 8, 5>;
template <int N> using LevelSlots = TSlots<N, 12, 9>;
template <int N> using FinalSlots = TSlots<N, 14, 11>;
template <int N> using FLevelSlots = TSlots<N, 3, 2>;
template <int N> using RollSlots = TSlots<N, 2, 4>;
template <int N> using FmatSlots = TSlots<N, 15, 10>;  // operator-form matrix fold

// eta_k = W r_k (W = H^T X in LDS, n x p zero padded, p <= N).
template <int N>
WDI void teta(const double* W, const double* rk, int p, double* e, int lane) {
    constexpr int ld = TL<N>::ld;
    if (lane < N) {
        double s = 0.0;
        for (int j = 0; j < p; ++j) s = fma(W[lane * ld + j], rk[j], s);
        e[lane] = s;
    }
    wsync();
}

// Step data for a time-varying step k (any of L, U, H, X per step): G_k,
// J_k and eta_k computed from the step's matrices (p <= N).
template <int N>
WDI bool tstep_var(const GInst& I, int64_t k, double* Us, double* Ht, double* Xt, double* G, double* J, double* e,
                   bool need_G, int lane) {
    constexpr int ld = TL<N>::ld;
    const int n = I.n, m = I.m, p = I.p;
    const uint32_t ps = I.per_step;
    tload<N>(m, m, step_ptr(I.U, ps, kPS_U, k, (int64_t)m * m), m, Us, lane, 1.0);
    const bool ok = tchol<N>(Us, lane);
    if (need_G) {
        const double* L = step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m);
        for (int idx = lane; idx < N * N; idx += kW) {  // Ht := L^T (zero padded)
            const int a = idx / N, j = idx % N;
            Ht[a * ld + j] = (a < m && j < n) ? L[j * m + a] : 0.0;
        }
        wsync();
        ttrsm_l<N>(Us, Ht, lane);
        for (int idx = lane; idx < N * N; idx += kW) {
            const int j = idx / N, a = idx % N;
            G[j * ld + a] = Ht[a * ld + j];
        }
        wsync();
    }
    tload<N>(p, n, step_ptr(I.H, ps, kPS_H, k, (int64_t)p * n), n, Ht, lane);
    tload<N>(p, p, step_ptr(I.X, ps, kPS_X, k, (int64_t)p * p), p, Xt, lane);
    tgemm<N, true, false>(Ht, Xt, Us, 1.0, 0.0, lane);  // W = H^T X
    tgemm<N, false, false, true>(Us, Ht, J, 1.0, 0.0, lane);
    if (lane < N) {
        double s = 0.0;
        const double* r = I.r + k * p;
        for (int j = 0; j < p; ++j) s = fma(Us[lane * ld + j], r[j], s);
        e[lane] = s;
    }
    wsync();
    return ok;
}

template <int N>
WDI void tvec_load(int n, const double* g, double* l, int lane) {
    if (lane < N) l[lane] = (lane < n) ? g[lane] : 0.0;
    wsync();
}

// P <- a_k (x) P, matrix inversion lemma form of the combination rule with
// C_k = G G^T: W = I + G^T J_P G = R R^T (m x m, W >= I), Z = G^T J_P,
// V = R^{-1} Z, Q = (A_P G) R^{-T}, y = R^{-1} (G^T eta_P - Z c); then
//   (I + C_k J_P)^{-1} = I - G W^{-1} Z,
//   A' = A_P F - Q (V F),        C' = C_P + Q Q^T,
//   b' = A_P c + Q y + b_P,      eta' = F^T (eta_P - J_P c - V^T y) + eta_k,
//   J' = F^T (J_P - V^T V) F + J_k.
// Every inverse is applied as triangular solves with the Cholesky factor, and
// the symmetric updates are products of a factor with itself.
// With opE (slots with at least 15 matrices), also stores the operators of
// the vector part for c = 0: eta' = E eta_P + eta_k and b' = b_P + B^ eta_P,
// E = F^T (I - V^T R^{-1} G^T) at opE and B^ = Q R^{-1} G^T after it (n x n
// each, row-major).
template <int N, typename SL>
WDI void t_step_combine(int m, const double* F, const double* c, const double* G, const double* ek,
                        const double* Js, double* PA, double* Pb, double* PC, double* Pe, double* PJ, SL& s,
                        int lane, int n = 0, double* opE = nullptr) {
    double* Z = s.m[7];
    double* Rf = s.m[8];
    double* VF = s.m[9];
    double* Qt = s.m[10];
    double* T9 = s.m[11];
    double *y = s.v[5], *w = s.v[7], *nb = s.v[8], *ne = s.v[9];
    constexpr int ld = TL<N>::ld;
    tgemm<N, true, false>(G, PJ, Z, 1.0, 0.0, lane);               // Z = G^T J_P
    tgemm<N, false, false, true>(Z, G, Rf, 1.0, 0.0, lane);        // Z G
    if (lane < N) Rf[lane * ld + lane] += 1.0;
    wsync();
    tchol_m<N>(Rf, m, lane);                                       // W >= I: always SPD
    // y0 = G^T eta_P - Z c, then V = R^{-1} Z (in Z) and y = R^{-1} y0
    tgemv<N, true>(G, Pe, y, 1.0, 0.0, lane);
    tgemv<N, false>(Z, c, y, -1.0, 1.0, lane);
    ttrsm_m<N, false>(Rf, Z, y, m, lane);
    tgemm<N, true, true>(G, PA, Qt, 1.0, 0.0, lane);               // (A_P G)^T
    ttrsm_m<N, false>(Rf, Qt, nullptr, m, lane);                   // Q^T = R^{-1} (A_P G)^T
    if constexpr (SL::NMv >= 15) {
        if (opE) {
            double *Gt = s.m[12], *Tm = s.m[13], *Em = s.m[14];
            for (int idx = lane; idx < N * N; idx += kW) {  // G^T
                const int a = idx / N, j = idx % N;
                Gt[a * ld + j] = G[j * ld + a];
            }
            wsync();
            ttrsm_m<N, false>(Rf, Gt, nullptr, m, lane);          // R^{-1} G^T
            tgemm<N, true, false>(Z, Gt, Tm, -1.0, 0.0, lane);    // -V^T R^{-1} G^T
            if (lane < N) Tm[lane * ld + lane] += 1.0;
            wsync();
            tgemm<N, true, false>(F, Tm, Em, 1.0, 0.0, lane);     // E
            tstore<N>(n, n, Em, opE, n, lane);
            wsync();
            tgemm<N, true, false>(Qt, Gt, Em, 1.0, 0.0, lane);    // B^
            tstore<N>(n, n, Em, opE + (int64_t)n * n, n, lane);
            wsync();
        }
    }
    // b' = A_P c + Q y + b_P
    tgemv<N, false>(PA, c, nb, 1.0, 0.0, lane);
    tgemv<N, true>(Qt, y, nb, 1.0, 1.0, lane);
    // eta' = F^T (eta_P - J_P c - V^T y) + eta_k
    tgemv<N, false>(PJ, c, w, -1.0, 0.0, lane);
    tgemv<N, true>(Z, y, w, -1.0, 1.0, lane);
    if (lane < N) w[lane] += Pe[lane];
    wsync();
    tgemv<N, true>(F, w, ne, 1.0, 0.0, lane);
    if (lane < N) {
        Pb[lane] += nb[lane];
        Pe[lane] = ne[lane] + ek[lane];
    }
    wsync();
    // C' = C_P + Q Q^T
    tgemm<N, true, false, true>(Qt, Qt, PC, 1.0, 1.0, lane);
    // A' = A_P F - Q (V F)
    tgemm<N, false, false>(Z, F, VF, 1.0, 0.0, lane);
    tgemm<N, false, false>(PA, F, T9, 1.0, 0.0, lane);
    tgemm<N, true, false>(Qt, VF, T9, -1.0, 1.0, lane);
    tcopy<N>(T9, PA, lane);
    // J' = F^T (J_P - V^T V) F + J_k
    tgemm<N, true, false, true>(Z, Z, PJ, -1.0, 1.0, lane);
    tgemm<N, false, false>(PJ, F, T9, 1.0, 0.0, lane);
    tgemm<N, true, false, true>(F, T9, PJ, 1.0, 0.0, lane);
    for (int idx = lane; idx < N * N; idx += kW) PJ[(idx / N) * ld + idx % N] += Js[(idx / N) * ld + idx % N];
    wsync();
}

// Operator form of the fold for instances with opf set (class 8,
// time-invariant, no offsets c, trajectory by maps): every chunk but the last
// has the full length B and the same matrix part (A, C, J), so one wavefront
// per instance folds one full chunk's B steps once, storing for each relative
// step j (counted from the chunk's end) the operators of the vector part
// (t_step_combine with opE), and writes the matrix part to chunk 0's element
// slot (chunk 0's element is never needed).  t_fold then runs only the vector
// recursion per chunk.
template <int N>
__global__ __launch_bounds__(kW) void t_fmat(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    if (!I.opf) return;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m, p = I.p;
    FmatSlots<N> s = tslots<N, FmatSlots<N>::NMv, FmatSlots<N>::NVv>(dyn);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, p);
    double *PA = s.m[0], *PC = s.m[1], *PJ = s.m[2], *F = s.m[3], *G = s.m[4], *Js = s.m[5];
    double *Pb = s.v[0], *Pe = s.v[1], *cc = s.v[2], *ek = s.v[3];
    tload<N>(n, m, ws.cst + cl.G, m, G, lane);
    tload<N>(n, n, ws.cst + cl.J, n, Js, lane);
    tload<N>(n, n, I.F, n, F, lane);
    if (lane < N) {
        cc[lane] = 0.0;
        ek[lane] = 0.0;
        Pb[lane] = 0.0;
        Pe[lane] = 0.0;
    }
    wsync();
    tcopy<N>(F, PA, lane);
    tgemm<N, false, true, true>(G, G, PC, 1.0, 0.0, lane);
    tcopy<N>(Js, PJ, lane);
    const int64_t nn = (int64_t)n * n;
#pragma unroll 1
    for (int j = 1; j < I.B; ++j)
        t_step_combine<N>(m, F, cc, G, ek, Js, PA, Pb, PC, Pe, PJ, s, lane, n, ws.ops + (int64_t)(j - 1) * 2 * nn);
    double* out = ws.agg;
    tstore<N>(n, n, PA, out, n, lane);
    tstore<N>(n, n, PC, out + nn + n, n, lane);
    tstore<N>(n, n, PJ, out + 2 * nn + 2 * n, n, lane);
}

// Vector part of a full chunk's element for an instance with opf set: the
// matrix part is the common one (t_fmat); eta and b by the stored operators,
// eta' = E_j eta + W r_k, b' = b + B^_j eta, with the operator rows and the
// reference of the next step loaded one step ahead.
template <int N>
WDI void t_fold_vec(const GInst& I, const InstWs& ws, int64_t c, int64_t k1, const double* W, double* Pb, double* Pe,
                    double* rk, int lane) {
    constexpr int ld = TL<N>::ld;
    const int n = I.n, p = I.p;
    const int64_t nn = (int64_t)n * n, ED = elem_doubles(n);
    const double* src = ws.agg;
    double* out = ws.agg + c * ED;
    for (int64_t idx = lane; idx < nn; idx += kW) {
        out[idx] = src[idx];
        out[nn + n + idx] = src[nn + n + idx];
        out[2 * nn + 2 * n + idx] = src[2 * nn + 2 * n + idx];
    }
    // eta = W r_{k1-1}, b = 0
    if (lane < N) rk[lane] = lane < p ? I.r[(k1 - 1) * p + lane] : 0.0;
    wsync();
    if (lane < N) {
        double e = 0.0;
        for (int q = 0; q < p; ++q) e = fma(W[lane * ld + q], rk[q], e);
        Pe[lane] = lane < n ? e : 0.0;
        Pb[lane] = 0.0;
    }
    wsync();
    double Er[N], Br[N], rr = 0.0;
    auto fetch = [&](int j) {
        if (j < I.B) {
            const double* E = ws.ops + (int64_t)(j - 1) * 2 * nn + (int64_t)lane * n;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                Er[l] = (lane < n && l < n) ? E[l] : 0.0;
                Br[l] = (lane < n && l < n) ? E[nn + l] : 0.0;
            }
            rr = lane < p ? I.r[(k1 - 1 - j) * p + lane] : 0.0;
        }
    };
    fetch(1);
#pragma unroll 1
    for (int j = 1; j < I.B; ++j) {
        double Ej[N], Bj[N];
#pragma unroll
        for (int l = 0; l < N; ++l) {
            Ej[l] = Er[l];
            Bj[l] = Br[l];
        }
        if (lane < N) rk[lane] = rr;
        fetch(j + 1);
        wsync();
        double nb = 0.0, ne = 0.0;
        if (lane < N) {
            nb = Pb[lane];
#pragma unroll
            for (int l = 0; l < N; ++l) {
                nb = fma(Bj[l], Pe[l], nb);
                ne = fma(Ej[l], Pe[l], ne);
            }
            for (int q = 0; q < p; ++q) ne = fma(W[lane * ld + q], rk[q], ne);
        }
        wsync();
        if (lane < N) {
            Pb[lane] = nb;
            Pe[lane] = ne;
        }
        wsync();
    }
    if (lane < n) {
        out[nn + lane] = Pb[lane];
        out[2 * nn + n + lane] = Pe[lane];
    }
}

template <int N>
__global__ __launch_bounds__(kW) void t_fold(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    // the first chunk's element is never used: the chain needs the elements
    // of chunks 1..NC-1 only (the value at the start of chunk 0 is not an input)
    if (c == 0) return;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m, p = I.p;
    FoldSlots<N> s = tslots<N, FoldSlots<N>::NMv, FoldSlots<N>::NVv>(dyn);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, p);
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    const uint32_t ps = I.per_step;
    const bool var = (ps & (kPS_L | kPS_U | kPS_H | kPS_X)) != 0;
    double *PA = s.m[0], *PC = s.m[1], *PJ = s.m[2], *F = s.m[3], *G = s.m[4], *Js = s.m[5], *W = s.m[6];
    double *Pb = s.v[0], *Pe = s.v[1], *cc = s.v[2], *ek = s.v[3], *rk = s.v[4];
    bool ok = true;
    if (!var) {
        tload<N>(n, m, ws.cst + cl.G, m, G, lane);
        tload<N>(n, n, ws.cst + cl.J, n, Js, lane);
        tload<N>(n, p, ws.cst + cl.W, p, W, lane);
    }
    if constexpr (N == 8) {
        if (I.opf && k1 - k0 == I.B) {
            t_fold_vec<N>(I, ws, c, k1, W, Pb, Pe, rk, lane);
            return;
        }
    }
    auto step_data = [&](int64_t k, bool first) {
        if (first || (ps & kPS_F)) tload<N>(n, n, step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n), n, F, lane);
        if (first || (ps & kPS_c)) {
            if (lane < N) cc[lane] = (I.c && lane < n) ? step_ptr(I.c, ps, kPS_c, k, n)[lane] : 0.0;
            wsync();
        }
        if (var) {
            // scratch: T9 (11), V (10), GtT (9) are free between combines
            ok = tstep_var<N>(I, k, s.m[9], s.m[10], s.m[11], G, Js, ek, true, lane) && ok;
        } else {
            if (lane < p) rk[lane] = I.r[k * p + lane];
            wsync();
            teta<N>(W, rk, p, ek, lane);
        }
    };
    step_data(k1 - 1, true);
    tcopy<N>(F, PA, lane);
    tgemm<N, false, true, true>(G, G, PC, 1.0, 0.0, lane);
    tcopy<N>(Js, PJ, lane);
    if (lane < N) {
        Pb[lane] = cc[lane];
        Pe[lane] = ek[lane];
    }
    wsync();
#pragma unroll 1
    for (int64_t k = k1 - 2; k >= k0; --k) {
        step_data(k, false);
        t_step_combine<N>(m, F, cc, G, ek, Js, PA, Pb, PC, Pe, PJ, s, lane);
    }
    double* out = ws.agg + c * elem_doubles(n);
    const int64_t nn = (int64_t)n * n;
    tstore<N>(n, n, PA, out, n, lane);
    if (lane < n) out[nn + lane] = Pb[lane];
    tstore<N>(n, n, PC, out + nn + n, n, lane);
    if (lane < n) out[2 * nn + n + lane] = Pe[lane];
    tstore<N>(n, n, PJ, out + 2 * nn + 2 * n, n, lane);
    if (!ok && lane == 0) raise(I.status, 3);
}

// Value functions at every chunk start, one wavefront per instance.
template <int N>
__global__ __launch_bounds__(kW) void t_chain(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    if (I.tree) return;  // t_tlevel + t_tanchor
    const int lane = threadIdx.x;
    const int n = I.n;
    ChainSlots<N> s = tslots<N, ChainSlots<N>::NMv, ChainSlots<N>::NVv>(dyn);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, I.m, I.p);
    const int64_t nn = (int64_t)n * n;
    double *EA = s.m[0], *EC = s.m[1], *EJ = s.m[2], *Sm = s.m[3];
    double *Mm = s.m[4], *Mi = s.m[5], *T1 = s.m[6], *P = s.m[7];
    double *Eb = s.v[0], *Ee = s.v[1], *v = s.v[2], *t = s.v[3], *nv = s.v[4];
    tload<N>(n, n, ws.cst + cl.ST, n, Sm, lane);
    tvec_load<N>(n, ws.cst + cl.VT, v, lane);
    double* vo = ws.val + I.NC * val_doubles(n);
    tstore<N>(n, n, Sm, vo, n, lane);
    if (lane < n) vo[nn + lane] = v[lane];
#pragma unroll 1
    for (int64_t c = I.NC - 1; c >= 1; --c) {  // val[0] is never read
        const double* e = ws.agg + c * elem_doubles(n);
        tload<N>(n, n, e, n, EA, lane);
        tload<N>(n, n, e + nn + n, n, EC, lane);
        tload<N>(n, n, e + 2 * nn + 2 * n, n, EJ, lane);
        tvec_load<N>(n, e + nn, Eb, lane);
        tvec_load<N>(n, e + 2 * nn + n, Ee, lane);
        // (S, v) <- E (x) (0, 0, 0, v, S)
        tgemm<N, false, false>(EC, Sm, Mm, 1.0, 0.0, lane);
        if (lane < N) Mm[lane * TL<N>::ld + lane] += 1.0;
        wsync();
        tinv<N>(Mm, Mi, lane);
        tgemm<N, false, false>(Mi, EA, T1, 1.0, 0.0, lane);
        tgemv<N, false>(Sm, Eb, t, -1.0, 0.0, lane);
        if (lane < N) t[lane] += v[lane];
        wsync();
        tgemv<N, true>(T1, t, nv, 1.0, 0.0, lane);
        tgemm<N, false, false>(Sm, EA, P, 1.0, 0.0, lane);
        tgemm<N, true, false, true>(T1, P, Sm, 1.0, 0.0, lane);
        for (int idx = lane; idx < N * N; idx += kW)
            Sm[(idx / N) * TL<N>::ld + idx % N] += EJ[(idx / N) * TL<N>::ld + idx % N];
        if (lane < N) v[lane] = nv[lane] + Ee[lane];
        wsync();
        vo = ws.val + c * val_doubles(n);
        tstore<N>(n, n, Sm, vo, n, lane);
        if (lane < n) vo[nn + lane] = v[lane];
    }
}

// Chunk scan as a tree for instances with tree set (as on the workgroup
// engines): level l replaces element c by E_c (x) E_{c+2^l}
// with the general combination rule of Section IV-A; t_tanchor anchors the
// suffixes on the terminal value (Section IV-B).  Records are n-dimensional.
template <int N>
__global__ __launch_bounds__(kW) void t_tlevel(const GInst* inst, int ninst, int64_t nchunks, int level) {
    extern __shared__ __align__(16) double dyn[];
    constexpr int ld = TL<N>::ld;
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    if (!I.tree || c == 0) return;  // the first chunk's element is never needed
    const int lane = threadIdx.x;
    const int n = I.n;
    const int64_t nn = (int64_t)n * n, ED = elem_doubles(n);
    const InstWs ws = inst_ws(I);
    const int64_t dist = int64_t(1) << level;
    const double* src = level == 0 ? ws.agg : ws.tree + ((level - 1) & 1) * I.NC * ED;
    double* dst = ws.tree + (level & 1) * I.NC * ED + c * ED;
    const double* ex = src + c * ED;
    if (c + dist >= I.NC) {  // nothing later at this distance: carried over
        for (int64_t idx = lane; idx < ED; idx += kW) dst[idx] = ex[idx];
        return;
    }
    const double* ey = src + (c + dist) * ED;
    LevelSlots<N> s = tslots<N, LevelSlots<N>::NMv, LevelSlots<N>::NVv>(dyn);
    double *XA = s.m[0], *XC = s.m[1], *XJ = s.m[2], *YA = s.m[3], *YC = s.m[4], *YJ = s.m[5];
    double *Mm = s.m[6], *Mi = s.m[7], *T1 = s.m[8], *U1 = s.m[9], *W1 = s.m[10], *R1 = s.m[11];
    double *xb = s.v[0], *xe = s.v[1], *yb = s.v[2], *ye = s.v[3], *y0 = s.v[4], *z = s.v[5], *w = s.v[6];
    double *o1 = s.v[7], *o2 = s.v[8];
    tload<N>(n, n, ex, n, XA, lane);
    tload<N>(n, n, ex + nn + n, n, XC, lane);
    tload<N>(n, n, ex + 2 * nn + 2 * n, n, XJ, lane);
    tload<N>(n, n, ey, n, YA, lane);
    tload<N>(n, n, ey + nn + n, n, YC, lane);
    tload<N>(n, n, ey + 2 * nn + 2 * n, n, YJ, lane);
    tvec_load<N>(n, ex + nn, xb, lane);
    tvec_load<N>(n, ex + 2 * nn + n, xe, lane);
    tvec_load<N>(n, ey + nn, yb, lane);
    tvec_load<N>(n, ey + 2 * nn + n, ye, lane);
    // M = I + C_x J_y (the identity on the padding)
    tgemm<N, false, false>(XC, YJ, Mm, 1.0, 0.0, lane);
    if (lane < N) Mm[lane * ld + lane] += 1.0;
    wsync();
    tinv<N>(Mm, Mi, lane);
    // y0 = b_x + C_x eta_y ; z = M^{-1} y0 ; w = eta_y - J_y b_x
    tgemv<N, false>(XC, ye, y0, 1.0, 0.0, lane);
    if (lane < N) y0[lane] += xb[lane];
    wsync();
    tgemv<N, false>(Mi, y0, z, 1.0, 0.0, lane);
    tgemv<N, false>(YJ, xb, w, -1.0, 0.0, lane);
    if (lane < N) w[lane] += ye[lane];
    wsync();
    tgemm<N, false, false>(Mi, XA, T1, 1.0, 0.0, lane);        // T = M^{-1} A_x
    tgemm<N, false, false>(Mi, XC, U1, 1.0, 0.0, lane);        // M^{-1} C_x (symmetric)
    tgemm<N, false, false>(YA, U1, W1, 1.0, 0.0, lane);        // A_y M^{-1} C_x
    tgemm<N, false, true, true>(W1, YA, R1, 1.0, 0.0, lane);   // A_y M^{-1} C_x A_y^T
    for (int idx = lane; idx < N * N; idx += kW) R1[(idx / N) * ld + idx % N] += YC[(idx / N) * ld + idx % N];
    wsync();
    tstore<N>(n, n, R1, dst + nn + n, n, lane);                // C
    tgemm<N, false, false>(YA, T1, W1, 1.0, 0.0, lane);        // A = A_y T
    tstore<N>(n, n, W1, dst, n, lane);
    tgemm<N, false, false>(YJ, XA, U1, 1.0, 0.0, lane);        // J_y A_x
    tgemm<N, true, false, true>(T1, U1, R1, 1.0, 0.0, lane);   // T^T J_y A_x
    for (int idx = lane; idx < N * N; idx += kW) R1[(idx / N) * ld + idx % N] += XJ[(idx / N) * ld + idx % N];
    wsync();
    tstore<N>(n, n, R1, dst + 2 * nn + 2 * n, n, lane);        // J
    tgemv<N, false>(YA, z, o1, 1.0, 0.0, lane);                // A_y z
    tgemv<N, true>(T1, w, o2, 1.0, 0.0, lane);                 // T^T w
    if (lane < n) {
        dst[nn + lane] = o1[lane] + yb[lane];                   // b
        dst[2 * nn + n + lane] = o2[lane] + xe[lane];           // eta
    }
}

template <int N>
__global__ __launch_bounds__(kW) void t_tanchor(const GInst* inst, int ninst, int64_t nchunks, int levels) {
    extern __shared__ __align__(16) double dyn[];
    constexpr int ld = TL<N>::ld;
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    if (!I.tree) return;
    const int lane = threadIdx.x;
    const int n = I.n;
    const int64_t nn = (int64_t)n * n, ED = elem_doubles(n);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, I.m, I.p);
    if (c == 0) {  // the terminal value (the value at chunk 0's start is never read)
        double* vo = ws.val + I.NC * val_doubles(n);
        for (int64_t idx = lane; idx < nn; idx += kW) vo[idx] = ws.cst[cl.ST + idx];
        if (lane < n) vo[nn + lane] = ws.cst[cl.VT + lane];
        return;
    }
    const double* e = (levels > 0 ? ws.tree + ((levels - 1) & 1) * I.NC * ED : ws.agg) + c * ED;
    ChainSlots<N> s = tslots<N, ChainSlots<N>::NMv, ChainSlots<N>::NVv>(dyn);
    double *EA = s.m[0], *EC = s.m[1], *EJ = s.m[2], *Sm = s.m[3];
    double *Mm = s.m[4], *Mi = s.m[5], *T1 = s.m[6], *P = s.m[7];
    double *Eb = s.v[0], *Ee = s.v[1], *v = s.v[2], *t = s.v[3], *nv = s.v[4];
    tload<N>(n, n, ws.cst + cl.ST, n, Sm, lane);
    tvec_load<N>(n, ws.cst + cl.VT, v, lane);
    tload<N>(n, n, e, n, EA, lane);
    tload<N>(n, n, e + nn + n, n, EC, lane);
    tload<N>(n, n, e + 2 * nn + 2 * n, n, EJ, lane);
    tvec_load<N>(n, e + nn, Eb, lane);
    tvec_load<N>(n, e + 2 * nn + n, Ee, lane);
    // (S, v) <- E (x) (0, 0, 0, v_T, S_T)
    tgemm<N, false, false>(EC, Sm, Mm, 1.0, 0.0, lane);
    if (lane < N) Mm[lane * ld + lane] += 1.0;
    wsync();
    tinv<N>(Mm, Mi, lane);
    tgemm<N, false, false>(Mi, EA, T1, 1.0, 0.0, lane);
    tgemv<N, false>(Sm, Eb, t, -1.0, 0.0, lane);
    if (lane < N) t[lane] += v[lane];
    wsync();
    tgemv<N, true>(T1, t, nv, 1.0, 0.0, lane);
    tgemm<N, false, false>(Sm, EA, P, 1.0, 0.0, lane);
    tgemm<N, true, false, true>(T1, P, Sm, 1.0, 0.0, lane);
    for (int idx = lane; idx < N * N; idx += kW) Sm[(idx / N) * ld + idx % N] += EJ[(idx / N) * ld + idx % N];
    if (lane < N) v[lane] = nv[lane] + Ee[lane];
    wsync();
    double* vo = ws.val + c * val_doubles(n);
    tstore<N>(n, n, Sm, vo, n, lane);
    if (lane < n) vo[nn + lane] = v[lane];
}

// State at every chunk start from x_0 (x_{c+1} = Phi_c x_c + phi_c), one
// wavefront per instance: lane l holds row l % N of the maps' column group
// l / N (N^2 / 64 columns) and the maps of the next kTPre chunks are loaded
// into registers ahead of their use.
constexpr int kTPre = 4;

template <int N>
__global__ __launch_bounds__(kW) void t_fchain(const GInst* inst, int ninst) {
    extern __shared__ __align__(16) double dyn[];
    constexpr int G = kW / N;    // column groups
    constexpr int QW = N / G;    // columns per lane
    const int ii = blockIdx.x;
    if (ii >= ninst) return;
    const GInst& I = inst[ii];
    if (I.tree) return;  // t_ftlevel
    const int lane = threadIdx.x;
    const int n = I.n;
    const int r = lane % N, g = lane / N;
    const bool act = r < n;
    const InstWs ws = inst_ws(I);
    const int64_t VD = val_doubles(n);
    double* x = dyn;             // N (zero beyond n)
    double* part = x + N;        // G x N partial products
    if (lane < N) x[lane] = (lane < n) ? I.x0[lane] : 0.0;
    double buf[kTPre][QW + 1];
    auto load = [&](int64_t c, double* d) {
        if (c < I.NC) {
            const double* mp = ws.map + c * VD;
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const int col = g * QW + q;
                d[q] = (act && col < n) ? mp[(int64_t)r * n + col] : 0.0;
            }
            d[QW] = (act && g == 0) ? mp[(int64_t)n * n + r] : 0.0;
        }
    };
#pragma unroll
    for (int j = 0; j < kTPre; ++j) load(j, buf[j]);
    wsync();
#pragma unroll 1
    for (int64_t c0 = 0; c0 < I.NC; c0 += kTPre) {
#pragma unroll
        for (int j = 0; j < kTPre; ++j) {
            const int64_t c = c0 + j;
            if (c < I.NC) {
                if (lane < n) ws.xs[c * n + lane] = x[lane];
                double a = buf[j][QW];
#pragma unroll
                for (int q = 0; q < QW; ++q) a = fma(buf[j][q], x[g * QW + q], a);
                part[g * N + r] = a;
                load(c + kTPre, buf[j]);
                wsync();
                if (lane < N) {
                    double y = part[lane];
#pragma unroll
                    for (int v = 1; v < G; ++v) y += part[v * N + lane];
                    x[lane] = y;
                }
                wsync();
            }
        }
    }
}

// State at every chunk start of an instance with tree set: the forward scan
// over the chunk maps (Method 1 of Section IV-C) by recursive doubling.
// Level l (d = 2^l) replaces map c by map_c o map_{c-d} where c >= d, so map
// c becomes the composition of maps 0 .. c.  x_0 is folded into map 0 at
// level 0; a map whose prefix reaches map 0 is then a constant (its value is
// x_{c+1}) and only its vector is kept: after level l the maps c < 2^(l+1)
// are constants.  Maps 0 .. NC-2 are scanned; the last level writes the
// states at the chunk starts.  Records are n-dimensional, NC - 1 <= 2^levels.
template <int N>
__global__ __launch_bounds__(kW) void t_ftlevel(const GInst* inst, int ninst, int64_t nchunks, int level, int last) {
    extern __shared__ __align__(16) double dyn[];
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    if (!I.tree || c > I.NC - 2) return;
    const int lane = threadIdx.x;
    const int n = I.n;
    const int64_t nn = (int64_t)n * n, VD = val_doubles(n), ED = elem_doubles(n);
    const InstWs ws = inst_ws(I);
    const int64_t dist = int64_t(1) << level;
    const double* src = level == 0 ? ws.map : ws.tree + ((level - 1) & 1) * I.NC * ED;
    const double* mc = src + c * VD;
    FLevelSlots<N> s = tslots<N, FLevelSlots<N>::NMv, FLevelSlots<N>::NVv>(dyn);
    double *P = s.m[0], *Q = s.m[1], *R = s.m[2];
    double *xz = s.v[0], *yv = s.v[1];
    // lane < n: row `lane` of (Phi v + phi) for the record rec (n x n, then n)
    auto apply = [&](const double* rec, const double* v) {
        double a = rec[nn + lane];
        for (int j = 0; j < n; ++j) a = fma(rec[(int64_t)lane * n + j], v[j], a);
        return a;
    };
    double o = 0.0;
    if (level == 0 && c <= 1) {  // x_1 = Phi_0 x_0 + phi_0
        if (lane < n) xz[lane] = I.x0[lane];
        wsync();
        if (lane < n) yv[lane] = apply(src, xz);
        wsync();
    } else if (c >= dist) {
        if (lane < n) yv[lane] = src[(c - dist) * VD + nn + lane];
        wsync();
    }
    if (c < dist) {  // carried over (a constant already)
        if (lane < n) o = level == 0 ? yv[lane] : mc[nn + lane];
    } else {
        if (lane < n) o = apply(mc, yv);
        if (c >= 2 * dist) {  // map_c o map_{c-d}: the matrix part
            tload<N>(n, n, mc, n, P, lane);
            tload<N>(n, n, src + (c - dist) * VD, n, Q, lane);
            tgemm<N, false, false>(P, Q, R, 1.0, 0.0, lane);
            tstore<N>(n, n, R, ws.tree + (level & 1) * I.NC * ED + c * VD, n, lane);
        }
    }
    if (last) {
        if (lane < n) {
            ws.xs[(c + 1) * n + lane] = o;
            if (c == 0) ws.xs[lane] = I.x0[lane];
        }
    } else if (lane < n) {
        ws.tree[(level & 1) * I.NC * ED + c * VD + nn + lane] = o;
    }
}

template <int N, typename OT>
__global__ __launch_bounds__(kW) void t_final(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    constexpr int ld = TL<N>::ld;
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m, p = I.p;
    FinalSlots<N> s = tslots<N, FinalSlots<N>::NMv, FinalSlots<N>::NVv>(dyn);
    const InstWs ws = inst_ws(I);
    const CstW cl = cst_layout(n, m, p);
    const int64_t nn = (int64_t)n * n;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    const uint32_t ps = I.per_step;
    const bool var = (ps & (kPS_L | kPS_U | kPS_H | kPS_X)) != 0;
    double *Sm = s.m[0], *F = s.m[1], *L = s.m[2], *Um = s.m[3], *Js = s.m[4], *W = s.m[5];
    double *SL = s.m[6], *R = s.m[7], *SF = s.m[8], *K = s.m[10];
    double *Phi = s.m[11], *Ft = s.m[12], *T13 = s.m[13];
    double *v = s.v[0], *cc = s.v[1], *ek = s.v[2], *w = s.v[3], *z = s.v[4], *d = s.v[5];
    double *phi = s.v[6], *ct = s.v[7], *nv = s.v[8], *t9 = s.v[9], *rk = s.v[10];
    OT* const oS = (OT*)I.S;
    OT* const oV = (OT*)I.v;
    OT* const oK = (OT*)I.K;
    OT* const oD = (OT*)I.d;
    const double* vin = ws.val + (c + 1) * val_doubles(n);
    tload<N>(n, n, vin, n, Sm, lane);
    tvec_load<N>(n, vin + nn, v, lane);
    for (int idx = lane; idx < N * N; idx += kW) Phi[(idx / N) * ld + idx % N] = ((idx / N) == (idx % N)) ? 1.0 : 0.0;
    if (lane < N) phi[lane] = 0.0;
    wsync();
    if (!var) {
        tload<N>(n, n, ws.cst + cl.J, n, Js, lane);
        tload<N>(n, p, ws.cst + cl.W, p, W, lane);
    }
    if (k1 == I.T) {
        if (oS) tstore<N>(n, n, Sm, oS + I.T * nn, n, lane);
        if (oV && lane < n) oV[I.T * n + lane] = (OT)v[lane];
    }
    double fin = 0.0;
    bool ok = true;
#pragma unroll 1
    for (int64_t k = k1 - 1; k >= k0; --k) {
        const bool first = (k == k1 - 1);
        if (first || (ps & kPS_F)) tload<N>(n, n, step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n), n, F, lane);
        if (first || (ps & kPS_L)) tload<N>(n, m, step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m), m, L, lane);
        if (first || (ps & kPS_U)) tload<N>(m, m, step_ptr(I.U, ps, kPS_U, k, (int64_t)m * m), m, Um, lane, 1.0);
        if (first || (ps & kPS_c)) {
            if (lane < N) cc[lane] = (I.c && lane < n) ? step_ptr(I.c, ps, kPS_c, k, n)[lane] : 0.0;
            wsync();
        }
        if (var) {
            ok = tstep_var<N>(I, k, SL, R, SF, T13, Js, ek, false, lane) && ok;
        } else {
            if (lane < p) rk[lane] = I.r[k * p + lane];
            wsync();
            teta<N>(W, rk, p, ek, lane);
        }
        // M_k = L^T S L + U = R R^T (Cholesky; SPD)
        tgemm<N, false, false>(Sm, L, SL, 1.0, 0.0, lane);
        for (int idx = lane; idx < N * N; idx += kW) {  // symmetrised U (identity on the padding)
            const int a = idx / N, b = idx % N;
            R[a * ld + b] = 0.5 * (Um[a * ld + b] + Um[b * ld + a]);
        }
        wsync();
        tgemm<N, true, false, true>(L, SL, R, 1.0, 1.0, lane);
        ok = tchol_m<N>(R, m, lane) && ok;
        // P = L^T S F, then V = R^{-1} P (in SL) and K = R^{-T} V
        tgemm<N, false, false>(Sm, F, SF, 1.0, 0.0, lane);
        tgemm<N, true, false>(L, SF, SL, 1.0, 0.0, lane);
        // w = v - S c ; z = L^T w ; zr = R^{-1} z (in z) ; d = R^{-T} zr
        tgemv<N, false>(Sm, cc, w, -1.0, 0.0, lane);
        if (lane < N) w[lane] += v[lane];
        wsync();
        tgemv<N, true>(L, w, z, 1.0, 0.0, lane);
        ttrsm_m<N, false>(R, SL, z, m, lane);
        tcopy<N>(SL, K, lane);
        if (lane < N) d[lane] = z[lane];
        wsync();
        ttrsm_m<N, true>(R, K, d, m, lane);
        // S' = F^T S F - V^T V + J ; v' = F^T w - V^T zr + eta
        tgemm<N, true, false, true>(F, SF, T13, 1.0, 0.0, lane);
        tgemm<N, true, false, true>(SL, SL, T13, -1.0, 1.0, lane);
        tgemv<N, true>(F, w, nv, 1.0, 0.0, lane);
        tgemv<N, true>(SL, z, nv, -1.0, 1.0, lane);
        for (int idx = lane; idx < N * N; idx += kW)
            Sm[(idx / N) * ld + idx % N] = T13[(idx / N) * ld + idx % N] + Js[(idx / N) * ld + idx % N];
        if (lane < N) v[lane] = nv[lane] + ek[lane];
        wsync();
        tcopy<N>(F, Ft, lane);
        tgemm<N, false, false>(L, K, Ft, -1.0, 1.0, lane);
        tgemv<N, false>(L, d, ct, 1.0, 0.0, lane);
        if (lane < N) ct[lane] += cc[lane];
        wsync();
        if (oS) tstore<N>(n, n, Sm, oS + k * nn, n, lane);
        if (oV && lane < n) oV[k * n + lane] = (OT)v[lane];
        tstore<N>(m, n, K, oK + k * m * n, n, lane);
        if (lane < m) oD[k * m + lane] = (OT)d[lane];
        for (int idx = lane; idx < n * n; idx += kW) fin += Sm[(idx / n) * ld + idx % n];
        if (lane < n) fin += v[lane];
        tgemv<N, false>(Phi, ct, t9, 1.0, 0.0, lane);
        if (lane < N) phi[lane] += t9[lane];
        wsync();
        tgemm<N, false, false>(Phi, Ft, T13, 1.0, 0.0, lane);
        tcopy<N>(T13, Phi, lane);
    }
    double* mo = ws.map + c * val_doubles(n);
    tstore<N>(n, n, Phi, mo, n, lane);
    if (lane < n) mo[nn + lane] = phi[lane];
    if (__any(!isfinite(fin)) && lane == 0) raise(I.status, 4);
    if (!ok && lane == 0) raise(I.status, 3);
}

template <int N, typename OT>
__global__ __launch_bounds__(kW) void t_roll(const GInst* inst, int ninst, int64_t nchunks) {
    extern __shared__ __align__(16) double dyn[];
    constexpr int ld = TL<N>::ld;
    const int64_t gc = blockIdx.x;
    if (gc >= nchunks) return;
    const GInst& I = inst[find_instance(inst, ninst, gc)];
    const int64_t c = gc - I.chunk0;
    const int lane = threadIdx.x;
    const int n = I.n, m = I.m;
    RollSlots<N> s = tslots<N, RollSlots<N>::NMv, RollSlots<N>::NVv>(dyn);
    const InstWs ws = inst_ws(I);
    const uint32_t ps = I.per_step;
    const int64_t k0 = c * I.B;
    const int64_t k1 = (k0 + I.B < I.T) ? k0 + I.B : I.T;
    double *F = s.m[0], *L = s.m[1];
    double *x = s.v[0], *u = s.v[1], *t = s.v[2], *cc = s.v[3];
    const OT* const iK = (const OT*)I.K;
    const OT* const iD = (const OT*)I.d;
    OT* const oX = (OT*)I.x;
    OT* const oU = (OT*)I.u;
    // every lane takes part: G consecutive lanes share a row of K (u = d - K x)
    // and of [F L] (x' = F x + L u + c), each summing every G-th term, then a
    // butterfly over the group
    constexpr int G = kW / N;
    static_assert((G & (G - 1)) == 0, "row groups of a power of two lanes");
    const int r = lane / G, g = lane % G;
    tvec_load<N>(n, ws.xs + c * n, x, lane);
    double fin = 0.0;
#pragma unroll 1
    for (int64_t k = k0; k < k1; ++k) {
        const bool first = (k == k0);
        if (first || (ps & kPS_F)) tload<N>(n, n, step_ptr(I.F, ps, kPS_F, k, (int64_t)n * n), n, F, lane);
        if (first || (ps & kPS_L)) tload<N>(n, m, step_ptr(I.L, ps, kPS_L, k, (int64_t)n * m), m, L, lane);
        if (first || (ps & kPS_c)) {
            if (lane < N) cc[lane] = (I.c && lane < n) ? step_ptr(I.c, ps, kPS_c, k, n)[lane] : 0.0;
            wsync();
        }
        {
            double a = 0.0;
            if (r < m) {
                const OT* Kr = iK + k * m * n + (int64_t)r * n;
                for (int j = g; j < n; j += G) a = fma(-(double)Kr[j], x[j], a);
            }
#pragma unroll
            for (int o = G / 2; o >= 1; o >>= 1) a += __shfl_xor(a, o, G);
            if (g == 0) u[r] = r < m ? (double)iD[k * m + r] + a : 0.0;
        }
        wsync();
        if (oX && lane < n) oX[k * n + lane] = (OT)x[lane];
        if (oU && lane < m) oU[k * m + lane] = (OT)u[lane];
        {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < N / G; ++i) a = fma(F[r * ld + g + i * G], x[g + i * G], a);
#pragma unroll
            for (int i = 0; i < N / G; ++i) a = fma(L[r * ld + g + i * G], u[g + i * G], a);
#pragma unroll
            for (int o = G / 2; o >= 1; o >>= 1) a += __shfl_xor(a, o, G);
            if (g == 0) t[r] = cc[r] + a;
        }
        wsync();
        if (lane < N) {
            x[lane] = t[lane];
            fin += t[lane];
        }
        wsync();
    }
    if (k1 == I.T && oX && lane < n) oX[I.T * n + lane] = (OT)x[lane];
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

int tile_class(int need) {
    if (need <= 8) return 8;
    if (need <= 16) return 16;
    if (need <= 32) return 32;
    if (need <= 64) return 64;
    return 0;
}


template <int N>
struct TileNames;
template <>
struct TileNames<8> {
    static constexpr const char* n[10] = {"t8_prep", "t8_fold", "t8_chain", "t8_final", "t8_fchain", "t8_roll",
                                          "t8_tree", "t8_tanchor", "t8_ftree", "t8_fmat"};
};
template <>
struct TileNames<16> {
    static constexpr const char* n[10] = {"t16_prep", "t16_fold", "t16_chain", "t16_final", "t16_fchain", "t16_roll",
                                          "t16_tree", "t16_tanchor", "t16_ftree", "t16_fmat"};
};
template <>
struct TileNames<32> {
    static constexpr const char* n[10] = {"t32_prep", "t32_fold", "t32_chain", "t32_final", "t32_fchain", "t32_roll",
                                          "t32_tree", "t32_tanchor", "t32_ftree", "t32_fmat"};
};

template <int N, typename OT>
static void run_tile(const GInst* d_inst, int ninst, int64_t nchunks, int64_t tree_nc, bool want_fwd, hipStream_t s,
                     const StageHook* h, bool opf_any) {
    const char* const* nm = TileNames<N>::n;
    const size_t glds = wave_lds_bytes(N);
    static bool attr = false;
    if (!attr) {
        const void* ks[] = {(const void*)t_fold<N>, (const void*)t_chain<N>, (const void*)t_final<N, OT>,
                            (const void*)t_roll<N, OT>, (const void*)g_prep, (const void*)t_tlevel<N>,
                            (const void*)t_tanchor<N>, (const void*)t_ftlevel<N>, (const void*)t_fmat<N>};
        for (const void* k : ks) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    {
        WStage st(h, nm[0], s);
        g_prep<<<ninst, kW, glds, s>>>(d_inst, ninst, N);
    }
    if (N == 8 && opf_any) {
        WStage st(h, nm[9], s);
        t_fmat<N><<<ninst, kW, FmatSlots<N>::bytes(), s>>>(d_inst, ninst);
    }
    {
        WStage st(h, nm[1], s);
        t_fold<N><<<(unsigned)nchunks, kW, FoldSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks);
    }
    int levels = 0;  // tree levels: 2^levels >= NC - 1 for every tree instance
    while ((int64_t(1) << levels) < tree_nc - 1) ++levels;
    if (tree_nc >= 2) {
        if (levels > 0) {
            WStage st(h, nm[6], s);
            for (int l = 0; l < levels; ++l)
                t_tlevel<N><<<(unsigned)nchunks, kW, LevelSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks, l);
        }
        WStage st(h, nm[7], s);
        t_tanchor<N><<<(unsigned)nchunks, kW, ChainSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks, levels);
    }
    {
        WStage st(h, nm[2], s);
        t_chain<N><<<ninst, kW, ChainSlots<N>::bytes(), s>>>(d_inst, ninst);
    }
    {
        WStage st(h, nm[3], s);
        t_final<N, OT><<<(unsigned)nchunks, kW, FinalSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks);
    }
    if (want_fwd) {
        if (tree_nc >= 2) {
            const int fl = levels > 0 ? levels : 1;
            WStage st(h, nm[8], s);
            for (int l = 0; l < fl; ++l)
                t_ftlevel<N><<<(unsigned)nchunks, kW, FLevelSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks, l, l == fl - 1);
        }
        {
            WStage st(h, nm[4], s);
            t_fchain<N><<<ninst, kW, sizeof(double) * (1 + kW / N) * N, s>>>(d_inst, ninst);
        }
        WStage st(h, nm[5], s);
        t_roll<N, OT><<<(unsigned)nchunks, kW, RollSlots<N>::bytes(), s>>>(d_inst, ninst, nchunks);
    }
}

template <typename OT>
static hipError_t tile_typed(int N, const GInst* d_inst, int ninst, int64_t nchunks, int64_t tree_nc, bool want_fwd,
                             hipStream_t s, const StageHook* h, bool opf_any) {
    switch (N) {
        case 8: run_tile<8, OT>(d_inst, ninst, nchunks, tree_nc, want_fwd, s, h, opf_any); break;
        case 16: run_tile<16, OT>(d_inst, ninst, nchunks, tree_nc, want_fwd, s, h, opf_any); break;
        case 32: run_tile<32, OT>(d_inst, ninst, nchunks, tree_nc, want_fwd, s, h, opf_any); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t tile_solve(int N, const GInst* d_inst, int ninst, int64_t nchunks, int64_t tree_nc, bool want_fwd, bool f32,
                      hipStream_t s, const StageHook* h, bool opf_any) {
    return f32 ? tile_typed<float>(N, d_inst, ninst, nchunks, tree_nc, want_fwd, s, h, opf_any)
               : tile_typed<double>(N, d_inst, ninst, nchunks, tree_nc, want_fwd, s, h, opf_any);
}

}  // namespace lqt
