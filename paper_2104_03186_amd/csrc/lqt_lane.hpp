// Lane-per-element machinery shared by the lane pipeline (one long instance
// per launch sequence) and the batched lane kernel (one workgroup per
// instance): constants layout, step data modes and loads, coalesced row
// transfers, and the cross-wavefront suffix scan.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lqt_internal.hpp"
#include "lqt_ops.hpp"

namespace lqt {

constexpr int kWave = 64;
constexpr int kBlock = 256;
static_assert(kBlock == kSmallTopBlock, "blocks of wavefront units in the backward top levels");

// Orders this wavefront's LDS accesses around a cooperative transfer.  Each
// staging area belongs to one wavefront, whose LDS operations execute in
// order, so only the compiler must be kept from moving accesses across; a
// workgroup barrier would also drain every outstanding global store.
LQT_DI void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wait until every outstanding vector-memory request of the wavefront has
// completed (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).
LQT_DI void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

LQT_DI void raise_status(int32_t* st, int32_t code) {
    if (st) atomicCAS(st, 0, code);  // first failure wins
}


// ---- per-step data ---------------------------------------------------------

template <int N, int M>
struct CstLayout {
    static constexpr int NS = Sym<N>::size;
    static constexpr int G = 0;
    static constexpr int J = G + N * M;
    static constexpr int ST = J + NS;
    static constexpr int VT = ST + NS;
    static constexpr int W = VT + N;  // followed by N * p doubles
    static constexpr int der = N * M + NS + N;  // per-step derived record (varying mode)
};

// Terminal value function S_T = H_T^T X_T H_T, v_T = H_T^T X_T r_T
// (terminal element of Section IV-B, with the terminal weight X_T).
template <int N>
LQT_DI void terminal_value(const SmallArgs& a, double* ST, double* vT) {
    using S = Sym<N>;
    const int pT = a.pT;
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double acc_v = 0.0;
        LQT_UNROLL for (int j = i; j < N; ++j) ST[S::at(i, j)] = 0.0;
        for (int q = 0; q < pT; ++q) {
            double wiq = 0.0;  // (H_T^T X_T)[i][q]
            for (int s = 0; s < pT; ++s) wiq = fma(a.HT[s * N + i], a.XT[s * pT + q], wiq);
            acc_v = fma(wiq, a.rT[q], acc_v);
            LQT_UNROLL for (int j = i; j < N; ++j) ST[S::at(i, j)] = fma(wiq, a.HT[q * N + j], ST[S::at(i, j)]);
        }
        vT[i] = acc_v;
    }
}

// One-step constants from (L, U, H, X) of one step: G with G G^T = L U^{-1} L^T,
// J = H^T X H, and (when W != nullptr) W = H^T X.  Returns false if U is not PD.
template <int N, int M>
LQT_DI bool step_constants(const double* L, const double* U, const double* H, const double* X, int p,
                           double* G, double* J, double* W) {
    using S = Sym<N>;
    using SM = Sym<M>;
    double Us[SM::size], R[M * M], rinv[M];
    LQT_UNROLL for (int i = 0; i < M; ++i)
    LQT_UNROLL for (int j = i; j < M; ++j) Us[SM::at(i, j)] = 0.5 * (U[i * M + j] + U[j * M + i]);
    const bool ok = chol<M>(Us, R, rinv);
    double Gt[M * N];
    LQT_UNROLL for (int q = 0; q < M; ++q)
    LQT_UNROLL for (int i = 0; i < N; ++i) Gt[q * N + i] = L[i * M + q];
    lsolve<M, N>(R, rinv, Gt);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int q = 0; q < M; ++q) G[i * M + q] = Gt[q * N + i];
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        LQT_UNROLL for (int j = i; j < N; ++j) J[S::at(i, j)] = 0.0;
        for (int q = 0; q < p; ++q) {
            double wiq = 0.0;
            for (int s = 0; s < p; ++s) wiq = fma(H[s * N + i], X[s * p + q], wiq);
            if (W) W[i * p + q] = wiq;
            LQT_UNROLL for (int j = i; j < N; ++j) J[S::at(i, j)] = fma(wiq, H[q * N + j], J[S::at(i, j)]);
        }
    }
    return ok;
}

// Same constants when H and X are square (p = n): every input is loaded into
// registers up front, so the one lane does not wait on a chain of loads.
template <int N, int M>
LQT_DI bool step_constants_sq(const double* Lp, const double* Up, const double* Hp, const double* Xp, double* G,
                              double* J, double* W) {
    using S = Sym<N>;
    using SM = Sym<M>;
    double L[N * M], U[M * M], H[N * N], X[N * N];
    LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = Lp[i];
    LQT_UNROLL for (int i = 0; i < M * M; ++i) U[i] = Up[i];
    LQT_UNROLL for (int i = 0; i < N * N; ++i) H[i] = Hp[i];
    LQT_UNROLL for (int i = 0; i < N * N; ++i) X[i] = Xp[i];
    double Us[SM::size], R[M * M], rinv[M];
    LQT_UNROLL for (int i = 0; i < M; ++i)
    LQT_UNROLL for (int j = i; j < M; ++j) Us[SM::at(i, j)] = 0.5 * (U[i * M + j] + U[j * M + i]);
    const bool ok = chol<M>(Us, R, rinv);
    double Gt[M * N];
    LQT_UNROLL for (int q = 0; q < M; ++q)
    LQT_UNROLL for (int i = 0; i < N; ++i) Gt[q * N + i] = L[i * M + q];
    lsolve<M, N>(R, rinv, Gt);
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int q = 0; q < M; ++q) G[i * M + q] = Gt[q * N + i];
    double Wl[N * N];
    mtm<N, N, N>(H, X, Wl);  // H^T X
    LQT_UNROLL for (int i = 0; i < N * N; ++i) W[i] = Wl[i];
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = i; j < N; ++j) {
        double s = Wl[i * N] * H[j];
        LQT_UNROLL for (int q = 1; q < N; ++q) s = fma(Wl[i * N + q], H[q * N + j], s);
        J[S::at(i, j)] = s;
    }
    return ok;
}

// Time-invariant problems: constants once.  One lane; it also initialises the
// status word (no other kernel of the solve has run yet).
template <int N, int M>
__global__ void k_prep_invariant(SmallArgs a) {
    using CL = CstLayout<N, M>;
    using S = Sym<N>;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* cst = a.cst;
    bool ok;
    double ST[S::size], vT[N];
    if (a.p == N && a.pT == N) {
        ok = step_constants_sq<N, M>(a.L, a.U, a.H, a.X, cst + CL::G, cst + CL::J, cst + CL::W);
        double HT[N * N], XT[N * N], rT[N], Wt[N * N], Xr[N];
        LQT_UNROLL for (int i = 0; i < N * N; ++i) HT[i] = a.HT[i];
        LQT_UNROLL for (int i = 0; i < N * N; ++i) XT[i] = a.XT[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) rT[i] = a.rT[i];
        mtm<N, N, N>(HT, XT, Wt);  // H_T^T X_T
        mv<N, N>(Wt, rT, Xr);
        LQT_UNROLL for (int i = 0; i < N; ++i) vT[i] = Xr[i];
        LQT_UNROLL for (int i = 0; i < N; ++i)
        LQT_UNROLL for (int j = i; j < N; ++j) {
            double s = Wt[i * N] * HT[j];
            LQT_UNROLL for (int q = 1; q < N; ++q) s = fma(Wt[i * N + q], HT[q * N + j], s);
            ST[S::at(i, j)] = s;
        }
    } else {
        ok = step_constants<N, M>(a.L, a.U, a.H, a.X, a.p, cst + CL::G, cst + CL::J, cst + CL::W);
        terminal_value<N>(a, ST, vT);
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) cst[CL::ST + i] = ST[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) cst[CL::VT + i] = vT[i];
    if (a.status) *a.status = ok ? 0 : 3;
}

// Time-varying problems: one record (G_k, J_k, eta_k) per step; thread T
// computes the terminal value.
template <int N, int M>
__global__ void k_prep_varying(SmallArgs a) {
    using CL = CstLayout<N, M>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > a.T) return;
    if (k == a.T) {
        double ST[Sym<N>::size], vT[N];
        terminal_value<N>(a, ST, vT);
        LQT_UNROLL for (int i = 0; i < Sym<N>::size; ++i) a.cst[CL::ST + i] = ST[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) a.cst[CL::VT + i] = vT[i];
        return;
    }
    const uint32_t ps = a.per_step;
    const int p = a.p;
    const double* L = a.L + ((ps & kPS_L) ? k * N * M : 0);
    const double* U = a.U + ((ps & kPS_U) ? k * M * M : 0);
    const double* H = a.H + ((ps & kPS_H) ? k * p * N : 0);
    const double* X = a.X + ((ps & kPS_X) ? k * p * p : 0);
    double* rec = a.der + k * CL::der;
    if (!step_constants<N, M>(L, U, H, X, p, rec, rec + N * M, nullptr)) raise_status(a.status, 3);
    // eta_k = H^T X r_k
    const double* r = a.r + k * p;
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int q = 0; q < p; ++q) {
            double wiq = 0.0;
            for (int t = 0; t < p; ++t) wiq = fma(H[t * N + i], X[t * p + q], wiq);
            s = fma(wiq, r[q], s);
        }
        rec[N * M + Sym<N>::size + i] = s;
    }
}

// Step data of element a_k into st.  In time-invariant mode only eta varies
// (st.F, st.c, st.G, st.J are loaded once by load_invariant).
template <int N, int M>
LQT_DI void load_invariant(const SmallArgs& a, Step<N, M>& st) {
    using CL = CstLayout<N, M>;
    LQT_UNROLL for (int i = 0; i < N * N; ++i) st.F[i] = a.F[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) st.c[i] = a.c ? a.c[i] : 0.0;
    LQT_UNROLL for (int i = 0; i < N * M; ++i) st.G[i] = a.cst[CL::G + i];
    LQT_UNROLL for (int i = 0; i < Sym<N>::size; ++i) st.J[i] = a.cst[CL::J + i];
}

// Step data modes: time-invariant with square H, X (the reference row feeds
// eta directly), time-invariant general, per-step (time-varying), and
// time-invariant except the offsets c_k (constants of the invariant mode,
// c_k read per step; e.g. the standard form of the generalised cost).
enum Mode { kFast = 0, kInv = 1, kVar = 2, kInvC = 3 };

template <int N, int M, int MODE>
LQT_DI void load_step(const SmallArgs& a, int64_t k, Step<N, M>& st) {
    using CL = CstLayout<N, M>;
    if constexpr (MODE == kVar) {
        const uint32_t ps = a.per_step;
        const double* F = a.F + ((ps & kPS_F) ? k * N * N : 0);
        LQT_UNROLL for (int i = 0; i < N * N; ++i) st.F[i] = F[i];
        const double* c = a.c ? a.c + ((ps & kPS_c) ? k * N : 0) : nullptr;
        LQT_UNROLL for (int i = 0; i < N; ++i) st.c[i] = c ? c[i] : 0.0;
        const double* rec = a.der + k * CL::der;
        LQT_UNROLL for (int i = 0; i < N * M; ++i) st.G[i] = rec[i];
        LQT_UNROLL for (int i = 0; i < Sym<N>::size; ++i) st.J[i] = rec[N * M + i];
        LQT_UNROLL for (int i = 0; i < N; ++i) st.e[i] = rec[N * M + Sym<N>::size + i];
    } else {
        // eta_k = W r_k with W = H^T X
        const int p = a.p;
        const double* W = a.cst + CL::W;
        const double* r = a.r + k * p;
        LQT_UNROLL for (int i = 0; i < N; ++i) st.e[i] = 0.0;
        for (int q = 0; q < p; ++q) {
            const double rq = r[q];
            LQT_UNROLL for (int i = 0; i < N; ++i) st.e[i] = fma(W[i * p + q], rq, st.e[i]);
        }
        if constexpr (MODE == kInvC) LQT_UNROLL for (int i = 0; i < N; ++i) st.c[i] = a.c[k * N + i];
    }
}

// ---- coalesced transfers -----------------------------------------------------
//
// Output rows of one time step k are R contiguous elements (S_k, K_k, ...) of
// the result type OT (double, or float for FP32 results).  In the chunked
// layout lane l of a wavefront handles row (cw0 + l) * B + j at step j, so
// lanes are B rows apart.  Per-lane stores would issue one small request per
// lane and per element; instead each lane deposits its row in LDS (row stride
// R | 1 elements, conflict-free) and the wavefront writes the 64 rows in
// vector pieces, consecutive lanes on consecutive pieces.

// Elements per vector piece for rows of R elements of type OT: 16 bytes where
// R allows it, else 8, else one element (rows start 16-byte aligned when the
// array does and R * sizeof(OT) is a multiple of 16).
template <typename OT, int R>
struct PieceW {
    static constexpr int v16 = 16 / (int)sizeof(OT);
    static constexpr int W = (R % v16 == 0) ? v16 : ((sizeof(OT) == 4 && R % 2 == 0) ? 2 : 1);
};

template <typename OT, int W>
struct VecOf {
    typedef OT T __attribute__((ext_vector_type(W)));
};

// W elements from src (any type) to g, converted to OT, as one access
template <int W, typename OT, typename ST>
LQT_DI void put_piece(OT* g, const ST* src) {
    if constexpr (W == 1) {
        g[0] = (OT)src[0];
    } else {
        typename VecOf<OT, W>::T t;
        LQT_UNROLL for (int i = 0; i < W; ++i) t[i] = (OT)src[i];
        *reinterpret_cast<typename VecOf<OT, W>::T*>(g) = t;
    }
}

template <int W, typename OT, typename DT>
LQT_DI void get_piece(const OT* g, DT* dst) {
    if constexpr (W == 1) {
        dst[0] = (DT)g[0];
    } else {
        const typename VecOf<OT, W>::T t = *reinterpret_cast<const typename VecOf<OT, W>::T*>(g);
        LQT_UNROLL for (int i = 0; i < W; ++i) dst[i] = (DT)t[i];
    }
}

template <int R>
struct Staged {
    static constexpr int stride = R | 1;
    static constexpr int elems = kWave * stride;
};

template <int R, typename OT>
LQT_DI void lds_put_row(OT* lds, int lane, const double* v) {
    LQT_UNROLL for (int i = 0; i < R; ++i) lds[lane * Staged<R>::stride + i] = (OT)v[i];
}

// rows (cw0 + rec) * B + j, valid when cw0 + rec < NC and the row < T
// (CHECK = false: the caller knows every row of the wavefront is valid)
template <int R, bool CHECK = true, typename OT>
LQT_DI void wave_store_rows(const OT* lds, OT* g, int64_t cw0, int64_t NC, int B, int j, int64_t T, int lane) {
    constexpr int st = Staged<R>::stride;
    constexpr int W = PieceW<OT, R>::W;
    constexpr int P = R / W;  // pieces per row
    if constexpr (!CHECK && kWave % P == 0) {
        // piece it of lane l belongs to record it * (64 / P) + l / P: one
        // per-lane base address and a uniform stride per piece
        constexpr int RPI = kWave / P;  // records per piece index
        const int rec0 = lane / P;
        const int off = (lane - rec0 * P) * W;
        OT* gb = g + ((cw0 + rec0) * B + j) * R + off;
        const int64_t stride = (int64_t)RPI * B * R;
        LQT_UNROLL for (int it = 0; it < P; ++it)
            put_piece<W>(gb + it * stride, lds + (it * RPI + rec0) * st + off);
    } else {
        LQT_UNROLL for (int it = 0; it < P; ++it) {
            const int piece = it * kWave + lane;
            const int rec = piece / P;
            const int off = (piece - rec * P) * W;
            const int64_t c = cw0 + rec;
            const int64_t row = c * B + j;
            if (!CHECK || (c < NC && row < T)) put_piece<W>(g + row * R + off, lds + rec * st + off);
        }
    }
}

// Direct per-lane row store/load (vector pieces where the row length allows).
template <int R, typename OT>
LQT_DI void store_row(OT* g, const double* v) {
    constexpr int W = PieceW<OT, R>::W;
    LQT_UNROLL for (int i = 0; i < R; i += W) put_piece<W>(g + i, v + i);
}

template <int R, typename OT>
LQT_DI void load_row(const OT* g, double* v) {
    constexpr int W = PieceW<OT, R>::W;
    LQT_UNROLL for (int i = 0; i < R; i += W) get_piece<W>(g + i, v + i);
}

template <int N>
LQT_DI void full_from_packed(const double* Sv, double* full) {
    LQT_UNROLL for (int i = 0; i < N; ++i)
    LQT_UNROLL for (int j = 0; j < N; ++j) full[i * N + j] = Sv[Sym<N>::at(i, j)];
}

// e = W r for W = H^T X square (p = n)
template <int N>
LQT_DI void eta_sq(const double* W, const double* rr, double* e) {
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double t = W[i * N] * rr[0];
        LQT_UNROLL for (int q = 1; q < N; ++q) t = fma(W[i * N + q], rr[q], t);
        e[i] = t;
    }
}

// ---- backward pass ---------------------------------------------------------

// Row index clamped into the lane's chunk [k0, k1) (any valid row for idle
// lanes), so prefetch loads are unconditional: loads under branches make the
// compiler drain every outstanding memory operation at the loop head.
LQT_DI int64_t clamp_row(int64_t k, int64_t k0, int64_t k1, bool active) {
    if (!active) return 0;
    return k < k0 ? k0 : (k >= k1 ? k1 - 1 : k);
}

// Suffix scan across the wavefronts of a workgroup.  On entry lane 0 of
// wavefront wv holds that wavefront's total in `agg`; nw wavefronts hold
// elements.
// On return R holds the suffix of the totals of wavefronts wv+1 .. nw-1
// (has_R false: there is none).  Hillis-Steele over the nw totals, ping-pong
// buffers in LDS, one workgroup barrier per round (nw is uniform).
template <int N>
LQT_DI bool wave_suffix(double (*sh)[kBlock / kWave][Elem<N>::size], const Elem<N>& agg, int nw, Elem<N>& R) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    if (lane == 0) store_elem<N>(sh[0][wv], agg);
    __syncthreads();
    int src = 0;
    if (nw > 2) {
        Elem<N> X;
        load_elem<N>(sh[0][wv], X);
        for (int d = 1; d < nw; d <<= 1) {
            if (wv + d < nw) {
                Elem<N> Y;
                load_elem<N>(sh[src][wv + d], Y);
                combine<N>(X, Y);
                X = Y;
            }
            if (lane == 0) store_elem<N>(sh[src ^ 1][wv], X);
            __syncthreads();
            src ^= 1;
        }
    }
    const bool has_R = wv + 1 < nw;
    if (has_R) load_elem<N>(sh[src][wv + 1], R);
    return has_R;
}


}  // namespace lqt
