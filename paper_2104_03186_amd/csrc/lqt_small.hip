// Lane-per-element LQT pipeline for small state dimension (gfx950).
//
// Each lane owns one chunk of B consecutive time steps and keeps a whole
// scan element in registers.  The reverse scan of Section IV-B is organised
// as reduce-then-scan (the block processing of Section V-C applied at three
// levels):
//
//   k_bwd_reduce  lane folds its chunk's one-step elements into the chunk
//                 element (step_combine), then a Hillis-Steele suffix scan
//                 across the 64 lanes of the wavefront (combine);
//   k_bwd_top     one workgroup scans the per-wavefront totals and anchors
//                 them on the terminal element: value function (S, v) at the
//                 first step of every wavefront unit;
//   k_bwd_final   lane anchors its in-wave suffix on that value, then walks
//                 its chunk backwards applying the down-sweep step in
//                 Riccati form fused with the gain extraction (writes S, v,
//                 K, d) and composes the chunk's closed-loop affine map;
//                 Hillis-Steele prefix scan of the maps across the wavefront;
//   k_fwd_top     one workgroup scans the per-wavefront affine totals from
//                 x_0: the state at the first step of every wavefront unit;
//   k_fwd_final   lane applies its in-wave prefix to get the state at its
//                 chunk start and rolls x_{k+1} = F x_k + c + L u_k forward
//                 with u_k = -K_k x_k + d_k (writes x, u).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_ops.hpp"

namespace lqt {

constexpr int kWave = 64;
constexpr int kBlock = 256;

LQT_DI void raise_status(int32_t* st, int32_t code) {
    if (st) atomicCAS(st, 0, code);  // first failure wins
}

__global__ void k_init_status(int32_t* st) {
    if (threadIdx.x == 0 && st) *st = 0;
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

// Time-invariant problems: constants once.  One lane.
template <int N, int M>
__global__ void k_prep_invariant(SmallArgs a) {
    using CL = CstLayout<N, M>;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* cst = a.cst;
    if (!step_constants<N, M>(a.L, a.U, a.H, a.X, a.p, cst + CL::G, cst + CL::J, cst + CL::W))
        raise_status(a.status, 3);
    double ST[Sym<N>::size], vT[N];
    terminal_value<N>(a, ST, vT);
    LQT_UNROLL for (int i = 0; i < Sym<N>::size; ++i) cst[CL::ST + i] = ST[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) cst[CL::VT + i] = vT[i];
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

template <int N, int M, bool VAR>
LQT_DI void load_step(const SmallArgs& a, int64_t k, Step<N, M>& st) {
    using CL = CstLayout<N, M>;
    if constexpr (VAR) {
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
    }
}

// ---- backward pass ---------------------------------------------------------

template <int N, int M, bool VAR>
__global__ __launch_bounds__(kBlock) void k_bwd_reduce(SmallArgs a) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool active = c < a.NC;
    Elem<N> P;
    if (active) {
        Step<N, M> st;
        if constexpr (!VAR) load_invariant<N, M>(a, st);
        const int64_t k0 = c * a.B;
        const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
        load_step<N, M, VAR>(a, k1 - 1, st);
        step_elem<N, M>(st, P);
        for (int64_t k = k1 - 2; k >= k0; --k) {
            load_step<N, M, VAR>(a, k, st);
            step_combine<N, M>(st, P);
        }
    } else {
        set_identity<N>(P);
    }
    // Suffix scan across the wavefront: lane l ends with E_l (x) ... (x) E_63.
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_down_elem<N>(P, d);
        if (lane + d < kWave && c + d < a.NC) {
            combine<N>(P, Q);
            P = Q;
        }
    }
    if (active) store_elem<N>(a.lane_el + c * Elem<N>::size, P);
}

// One workgroup: the value function at the first step of every wavefront
// unit g (stored in wave_val[g]), from the unit totals (= the in-wave suffix
// of each unit's first lane) and the terminal value.
template <int N>
__global__ __launch_bounds__(kBlock) void k_bwd_top(SmallArgs a, int64_t ld_cst_st) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    __shared__ double sh[kBlock / kWave][Elem<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int NG = a.NG;
    const int q = (NG + kBlock - 1) / kBlock;
    const int lo = tid * q < NG ? tid * q : NG;
    const int hi = lo + q < NG ? lo + q : NG;
    Elem<N> agg, tot;
    set_identity<N>(agg);
    for (int g = hi - 1; g >= lo; --g) {
        load_elem<N>(a.lane_el + (int64_t)g * kWave * Elem<N>::size, tot);
        combine<N>(tot, agg);
    }
    // reverse inclusive scan of agg across the block
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_down_elem<N>(agg, d);
        if (lane + d < kWave) {
            combine<N>(agg, Q);
            agg = Q;
        }
    }
    if (lane == 0) store_elem<N>(sh[wv], agg);
    __syncthreads();
    Elem<N> R;
    set_identity<N>(R);
    for (int w = kBlock / kWave - 1; w > wv; --w) {
        load_elem<N>(sh[w], tot);
        combine<N>(tot, R);
    }
    // suffix strictly after this lane, then anchored on the terminal value
    Elem<N> nxt = shfl_down_elem<N>(agg, 1);
    if (lane == kWave - 1) set_identity<N>(nxt);
    combine<N>(nxt, R);
    double Sv[S::size], v[N];
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = a.cst[ld_cst_st + i];
    LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = a.cst[ld_cst_st + S::size + i];
    anchor<N>(R, Sv, v);
    for (int g = hi - 1; g >= lo; --g) {
        load_elem<N>(a.lane_el + (int64_t)g * kWave * Elem<N>::size, tot);
        anchor<N>(tot, Sv, v);
        double* o = a.wave_val + (int64_t)g * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = Sv[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = v[i];
    }
    if (tid == 0) {
        double* o = a.wave_val + (int64_t)NG * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = a.cst[ld_cst_st + i];
        LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = a.cst[ld_cst_st + S::size + i];
    }
}

template <int N>
LQT_DI void write_value(const SmallArgs& a, int64_t k, const double* Sv, const double* v, double& fin) {
    using S = Sym<N>;
    if (a.S) {
        double* o = a.S + k * N * N;
        LQT_UNROLL for (int i = 0; i < N; ++i)
        LQT_UNROLL for (int j = 0; j < N; ++j) o[i * N + j] = Sv[S::at(i, j)];
    }
    if (a.v) {
        double* o = a.v + k * N;
        LQT_UNROLL for (int i = 0; i < N; ++i) o[i] = v[i];
    }
    LQT_UNROLL for (int i = 0; i < S::size; ++i) fin += Sv[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) fin += v[i];
}

template <int N, int M, bool VAR>
__global__ __launch_bounds__(kBlock) void k_bwd_final(SmallArgs a) {
    using S = Sym<N>;
    using CL = CstLayout<N, M>;
    constexpr int VS = S::size + N;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t g = c / kWave;
    const bool active = c < a.NC;
    Aff<N> phi;
    aff_identity<N>(phi);
    if (active) {
        double Sv[S::size], v[N];
        const double* wv = a.wave_val + (g + 1 < a.NG ? g + 1 : a.NG) * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = wv[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = wv[S::size + i];
        if (lane < kWave - 1 && c + 1 < a.NC) {
            Elem<N> nx;
            load_elem<N>(a.lane_el + (c + 1) * Elem<N>::size, nx);
            anchor<N>(nx, Sv, v);
        }
        const int64_t k0 = c * a.B;
        const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
        double fin = 0.0;
        if (k1 == a.T) write_value<N>(a, a.T, Sv, v, fin);
        // invariant step data
        double F[N * N], cc[N], L[N * M], U[M * M], Js[S::size], e[N];
        const uint32_t ps = a.per_step;
        bool ok = true;
        for (int64_t k = k1 - 1; k >= k0; --k) {
            const double* Fp = a.F + ((VAR && (ps & kPS_F)) ? k * N * N : 0);
            const double* Lp = a.L + ((VAR && (ps & kPS_L)) ? k * N * M : 0);
            const double* Up = a.U + ((VAR && (ps & kPS_U)) ? k * M * M : 0);
            const double* cp = a.c ? a.c + ((VAR && (ps & kPS_c)) ? k * N : 0) : nullptr;
            LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = Fp[i];
            LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = Lp[i];
            LQT_UNROLL for (int i = 0; i < M * M; ++i) U[i] = Up[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = cp ? cp[i] : 0.0;
            if constexpr (VAR) {
                const double* rec = a.der + k * CL::der;
                LQT_UNROLL for (int i = 0; i < S::size; ++i) Js[i] = rec[N * M + i];
                LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = rec[N * M + S::size + i];
            } else {
                LQT_UNROLL for (int i = 0; i < S::size; ++i) Js[i] = a.cst[CL::J + i];
                const int p = a.p;
                const double* W = a.cst + CL::W;
                const double* r = a.r + k * p;
                LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = 0.0;
                for (int q = 0; q < p; ++q) {
                    const double rq = r[q];
                    LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = fma(W[i * p + q], rq, e[i]);
                }
            }
            double K[M * N], d[M], Ft[N * N], ct[N];
            ok = riccati_step<N, M>(F, cc, L, U, Js, e, Sv, v, K, d, Ft, ct) && ok;
            write_value<N>(a, k, Sv, v, fin);
            double* Ko = a.K + k * M * N;
            LQT_UNROLL for (int i = 0; i < M * N; ++i) Ko[i] = K[i];
            double* dO = a.d + k * M;
            LQT_UNROLL for (int i = 0; i < M; ++i) dO[i] = d[i];
            // compose the chunk map: phi <- phi o (Ft, ct)
            Aff<N> step;
            LQT_UNROLL for (int i = 0; i < N * N; ++i) step.F[i] = Ft[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) step.c[i] = ct[i];
            aff_after<N>(step, phi);
        }
        if (!ok) raise_status(a.status, 3);
        if (!isfinite(fin)) raise_status(a.status, 4);
    }
    if (!a.want_fwd) return;
    // inclusive prefix across the wavefront: lane l ends with f_l o ... o f_0
    for (int d = 1; d < kWave; d <<= 1) {
        Aff<N> Q = shfl_up_aff<N>(phi, d);
        if (lane >= d) aff_after<N>(Q, phi);
    }
    if (active) store_aff<N>(a.lane_aff + c * Aff<N>::size, phi);
}

// ---- forward pass ----------------------------------------------------------

// One workgroup: the state at the first step of every wavefront unit.
template <int N>
__global__ __launch_bounds__(kBlock) void k_fwd_top(SmallArgs a) {
    __shared__ double sh[kBlock / kWave][Aff<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int NG = a.NG;
    const int q = (NG + kBlock - 1) / kBlock;
    const int lo = tid * q < NG ? tid * q : NG;
    const int hi = lo + q < NG ? lo + q : NG;
    auto unit_total = [&](int g, Aff<N>& t) {
        const int64_t first = (int64_t)g * kWave;
        const int64_t last = (first + kWave < a.NC ? first + kWave : a.NC) - 1;
        load_aff<N>(a.lane_aff + last * Aff<N>::size, t);
    };
    Aff<N> agg, t;
    aff_identity<N>(agg);
    for (int g = lo; g < hi; ++g) {
        unit_total(g, t);
        aff_after<N>(agg, t);
        agg = t;
    }
    for (int d = 1; d < kWave; d <<= 1) {
        Aff<N> Q = shfl_up_aff<N>(agg, d);
        if (lane >= d) aff_after<N>(Q, agg);
    }
    if (lane == kWave - 1) store_aff<N>(sh[wv], agg);
    __syncthreads();
    Aff<N> R;
    aff_identity<N>(R);
    for (int w = 0; w < wv; ++w) {
        load_aff<N>(sh[w], t);
        aff_after<N>(R, t);
        R = t;
    }
    Aff<N> prev = shfl_up_aff<N>(agg, 1);
    if (lane == 0) aff_identity<N>(prev);
    aff_after<N>(R, prev);
    double x[N], nx[N];
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.x0[i];
    mv<N, N>(prev.F, x, nx);
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + prev.c[i];
    for (int g = lo; g < hi; ++g) {
        LQT_UNROLL for (int i = 0; i < N; ++i) a.wave_x[(int64_t)g * N + i] = x[i];
        unit_total(g, t);
        mv<N, N>(t.F, x, nx);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + t.c[i];
    }
}

template <int N, int M, bool VAR>
__global__ __launch_bounds__(kBlock) void k_fwd_final(SmallArgs a) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.NC) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t g = c / kWave;
    double x[N], t[N];
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.wave_x[g * N + i];
    if (lane > 0) {
        Aff<N> pre;
        load_aff<N>(a.lane_aff + (c - 1) * Aff<N>::size, pre);
        mv<N, N>(pre.F, x, t);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = t[i] + pre.c[i];
    }
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    const uint32_t ps = a.per_step;
    double fin = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        const double* Fp = a.F + ((VAR && (ps & kPS_F)) ? k * N * N : 0);
        const double* Lp = a.L + ((VAR && (ps & kPS_L)) ? k * N * M : 0);
        const double* cp = a.c ? a.c + ((VAR && (ps & kPS_c)) ? k * N : 0) : nullptr;
        const double* Kp = a.K + k * M * N;
        const double* dp = a.d + k * M;
        double u[M];
        LQT_UNROLL for (int p = 0; p < M; ++p) {
            double s = dp[p];
            LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(-Kp[p * N + j], x[j], s);
            u[p] = s;
        }
        if (a.x) {
            LQT_UNROLL for (int i = 0; i < N; ++i) a.x[k * N + i] = x[i];
        }
        if (a.u) {
            LQT_UNROLL for (int p = 0; p < M; ++p) a.u[k * M + p] = u[p];
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            double s = cp ? cp[i] : 0.0;
            LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(Fp[i * N + j], x[j], s);
            LQT_UNROLL for (int p = 0; p < M; ++p) s = fma(Lp[i * M + p], u[p], s);
            t[i] = s;
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            x[i] = t[i];
            fin += t[i];
        }
    }
    if (k1 == a.T && a.x) {
        LQT_UNROLL for (int i = 0; i < N; ++i) a.x[a.T * N + i] = x[i];
    }
    if (!isfinite(fin)) raise_status(a.status, 4);
}

// ---- launcher ----------------------------------------------------------------

struct Stage {
    const StageHook* h;
    hipStream_t s;
    Stage(const StageHook* hook, const char* name, hipStream_t st) : h(hook), s(st) {
        if (h) h->begin(h->ctx, name, s);
    }
    ~Stage() {
        if (h) h->end(h->ctx, s);
    }
};

template <int N, int M>
static hipError_t run_small(const SmallArgs& a, hipStream_t s, const StageHook* h) {
    using CL = CstLayout<N, M>;
    const bool var = (a.per_step & (kPS_F | kPS_c | kPS_L | kPS_H | kPS_X | kPS_U)) != 0;
    const unsigned grid = (unsigned)((a.NC + kBlock - 1) / kBlock);
    {
        Stage st(h, "init_status", s);
        k_init_status<<<1, 64, 0, s>>>(a.status);
    }
    if (var) {
        const unsigned pg = (unsigned)((a.T + 1 + kBlock - 1) / kBlock);
        {
            Stage st(h, "prep_varying", s);
            k_prep_varying<N, M><<<pg, kBlock, 0, s>>>(a);
        }
        Stage st(h, "bwd_reduce", s);
        k_bwd_reduce<N, M, true><<<grid, kBlock, 0, s>>>(a);
    } else {
        {
            Stage st(h, "prep_invariant", s);
            k_prep_invariant<N, M><<<1, 64, 0, s>>>(a);
        }
        Stage st(h, "bwd_reduce", s);
        k_bwd_reduce<N, M, false><<<grid, kBlock, 0, s>>>(a);
    }
    {
        Stage st(h, "bwd_top", s);
        k_bwd_top<N><<<1, kBlock, 0, s>>>(a, CL::ST);
    }
    {
        Stage st(h, "bwd_final", s);
        if (var) k_bwd_final<N, M, true><<<grid, kBlock, 0, s>>>(a);
        else k_bwd_final<N, M, false><<<grid, kBlock, 0, s>>>(a);
    }
    if (a.want_fwd) {
        {
            Stage st(h, "fwd_top", s);
            k_fwd_top<N><<<1, kBlock, 0, s>>>(a);
        }
        Stage st(h, "fwd_final", s);
        if (var) k_fwd_final<N, M, true><<<grid, kBlock, 0, s>>>(a);
        else k_fwd_final<N, M, false><<<grid, kBlock, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <int N, int M>
static size_t cst_doubles(int p) {
    return (size_t)CstLayout<N, M>::W + (size_t)N * p;
}

#define LQT_SMALL_CASES(X) \
    X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(3, 3) X(4, 1) X(4, 2) X(4, 3) X(4, 4)

bool small_supported(int n, int m) {
#define X(N, M) if (n == N && m == M) return true;
    LQT_SMALL_CASES(X)
#undef X
    return false;
}

size_t small_cst_doubles(int n, int m, int p) {
#define X(N, M) if (n == N && m == M) return cst_doubles<N, M>(p);
    LQT_SMALL_CASES(X)
#undef X
    return 0;
}

size_t small_der_doubles(int n, int m) { return (size_t)n * m + (size_t)n * (n + 1) / 2 + n; }
size_t small_elem_doubles(int n) { return (size_t)n * n + 2 * n + (size_t)n * (n + 1); }
size_t small_aff_doubles(int n) { return (size_t)n * n + n; }
size_t small_val_doubles(int n) { return (size_t)n * (n + 1) / 2 + n; }

hipError_t small_solve(const SmallArgs& a, hipStream_t s, const StageHook* hook) {
#define X(N, M) if (a.n == N && a.m == M) return run_small<N, M>(a, s, hook);
    LQT_SMALL_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace lqt
