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

#include <type_traits>

#include "lqt_internal.hpp"
#include "lqt_lane.hpp"
#include "lqt_ops.hpp"

namespace lqt {
__global__ void k_init_status(int32_t* st) {
    if (threadIdx.x == 0 && st) *st = 0;
}

template <int N, int M, int MODE>
__global__ __launch_bounds__(kBlock) void k_bwd_reduce(SmallArgs a) {
    using CL = CstLayout<N, M>;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool active = c < a.NC;
    Elem<N> P;
    if (active) {
        Step<N, M> st;
        if constexpr (MODE != kVar) load_invariant<N, M>(a, st);
        const int64_t k0 = c * a.B;
        const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
        if constexpr (MODE == kFast) {
            // Rows are consumed k1-1, k1-2, ..., k0.  Two row buffers are
            // reloaded right after use, two steps ahead of their next use.
            const double* W = a.cst + CL::W;
            const double* r = a.r;
            double rA[N], rB[N];
            load_row<N>(r + clamp_row(k1 - 1, k0, k1, true) * N, rA);
            load_row<N>(r + clamp_row(k1 - 2, k0, k1, true) * N, rB);
            eta_sq<N>(W, rA, st.e);
            step_elem<N, M>(st, P);
            load_row<N>(r + clamp_row(k1 - 3, k0, k1, true) * N, rA);
            for (int64_t k = k1 - 2; k >= k0; k -= 2) {
                eta_sq<N>(W, rB, st.e);
                step_combine<N, M>(st, P);
                load_row<N>(r + clamp_row(k - 2, k0, k1, true) * N, rB);
                if (k - 1 >= k0) {
                    eta_sq<N>(W, rA, st.e);
                    step_combine<N, M>(st, P);
                }
                load_row<N>(r + clamp_row(k - 3, k0, k1, true) * N, rA);
            }
        } else {
            load_step<N, M, MODE>(a, k1 - 1, st);
            step_elem<N, M>(st, P);
            for (int64_t k = k1 - 2; k >= k0; --k) {
                load_step<N, M, MODE>(a, k, st);
                step_combine<N, M>(st, P);
            }
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

// One workgroup: reverse scan of cnt elements el[g * stride], g = 0..cnt-1
// (each covering a run of consecutive steps, in time order), anchored on the
// value term (packed S, then v): out[g] = value function at the first step
// covered by element g, out[cnt] = term.
template <int N>
__global__ __launch_bounds__(kBlock) void k_bwd_top(const double* el, int64_t stride, int cnt, const double* term,
                                                    double* out) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    __shared__ double sh[2][kBlock / kWave][Elem<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int q = (cnt + kBlock - 1) / kBlock;
    const int lo = tid * q < cnt ? tid * q : cnt;
    const int hi = lo + q < cnt ? lo + q : cnt;
    const int nt = (cnt + q - 1) / q;                         // threads holding elements
    const int nw = (nt + kWave - 1) / kWave;                  // wavefronts holding elements
    Elem<N> agg, tot;
    if (hi > lo) {
        load_elem<N>(el + (int64_t)(hi - 1) * stride, agg);
        for (int g = hi - 2; g >= lo; --g) {
            load_elem<N>(el + (int64_t)g * stride, tot);
            combine<N>(tot, agg);
        }
    } else {
        set_identity<N>(agg);
    }
    // suffix across the wavefront (rounds beyond the populated lanes skipped)
    for (int d = 1; d < kWave && d < nt; d <<= 1) {
        Elem<N> Q = shfl_down_elem<N>(agg, d);
        if (lane + d < kWave && tid + d < nt) {
            combine<N>(agg, Q);
            agg = Q;
        }
    }
    Elem<N> R;
    const bool has_R = wave_suffix<N>(sh, agg, nw, R);
    // suffix strictly after this thread's range, then anchored on the terminal value
    Elem<N> nxt = shfl_down_elem<N>(agg, 1);
    const bool has_nxt = lane + 1 < kWave && tid + 1 < nt;
    if (has_R) {
        if (has_nxt) combine<N>(nxt, R);
        nxt = R;
    }
    double Sv[S::size], v[N];
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = term[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = term[S::size + i];
    if (has_R || has_nxt) anchor<N>(nxt, Sv, v);
    for (int g = hi - 1; g >= lo; --g) {
        load_elem<N>(el + (int64_t)g * stride, tot);
        anchor<N>(tot, Sv, v);
        double* o = out + (int64_t)g * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = Sv[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = v[i];
    }
    if (tid == 0) {
        double* o = out + (int64_t)cnt * VS;
        LQT_UNROLL for (int i = 0; i < VS; ++i) o[i] = term[i];
    }
}

// Long instances (more than kBlock wavefront units): the units are grouped
// in blocks of kBlock, one workgroup each.  mid_el[g] = E_g (x) ... (x) E_l,
// E_g the total of unit g (the in-wave suffix of its first lane) and l the
// last unit of g's block; the first unit's entry is the block total.
template <int N>
__global__ __launch_bounds__(kBlock) void k_bwd_mid(SmallArgs a) {
    __shared__ double sh[2][kBlock / kWave][Elem<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int64_t g0 = (int64_t)blockIdx.x * kBlock;
    const int64_t g = g0 + tid;
    const int nb = (int)(a.NG - g0 < kBlock ? a.NG - g0 : kBlock);  // units in this block
    const int nw = (nb + kWave - 1) / kWave;
    Elem<N> agg;
    if (tid < nb) load_elem<N>(a.lane_el + g * kWave * Elem<N>::size, agg);
    else set_identity<N>(agg);
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_down_elem<N>(agg, d);
        if (lane + d < kWave && tid + d < nb) {
            combine<N>(agg, Q);
            agg = Q;
        }
    }
    Elem<N> R;
    if (wave_suffix<N>(sh, agg, nw, R)) {
        combine<N>(agg, R);
        agg = R;
    }
    if (tid < nb) store_elem<N>(a.mid_el + g * Elem<N>::size, agg);
}

// wave_val[g] = mid_el[g] anchored on the value at the start of the next
// block; wave_val[NG] = the terminal value.  That block value comes from
// blk_val (k_bwd_top over the block totals), or, when chain is set (few
// blocks), is formed here by anchoring the totals of the later blocks on the
// terminal value one after another, which saves the top-level launch.
constexpr int kDownChain = 8;  // most blocks for the chained form

template <int N>
__global__ __launch_bounds__(kBlock) void k_bwd_down(SmallArgs a, int64_t ld_cst_st, int chain) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g > a.NG) return;
    double* o = a.wave_val + g * VS;
    if (g == a.NG) {
        LQT_UNROLL for (int i = 0; i < VS; ++i) o[i] = a.cst[ld_cst_st + i];
        return;
    }
    const int64_t b = g / kBlock;
    double Sv[S::size], v[N];
    if (chain) {
        LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = a.cst[ld_cst_st + i];
        LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = a.cst[ld_cst_st + S::size + i];
        for (int64_t bb = a.NB - 1; bb > b; --bb) {  // uniform over a wavefront
            Elem<N> tb;
            load_elem<N>(a.mid_el + bb * kBlock * Elem<N>::size, tb);
            anchor<N>(tb, Sv, v);
        }
    } else {
        const double* bv = a.blk_val + (b + 1) * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = bv[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = bv[S::size + i];
    }
    Elem<N> e;
    load_elem<N>(a.mid_el + g * Elem<N>::size, e);
    anchor<N>(e, Sv, v);
    LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = Sv[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = v[i];
}

// Per-block copy of the time-invariant step data (read from LDS inside the
// step loops: after the first output store the compiler could no longer keep
// such loads on the scalar path).
template <int N, int M>
struct InvShared {
    double F[N * N], L[N * M], U[M * M], J[Sym<N>::size], c[N], W[N * N];
};

template <int N, int M>
LQT_DI void load_inv_shared(const SmallArgs& a, InvShared<N, M>& sh) {
    using CL = CstLayout<N, M>;
    const int t = threadIdx.x;
    if (t < N * N) sh.F[t] = a.F[t];
    if (t < N * M) sh.L[t] = a.L[t];
    if (t < M * M) sh.U[t] = a.U[t];
    if (t < Sym<N>::size) sh.J[t] = a.cst[CL::J + t];
    if (t < N) sh.c[t] = a.c ? a.c[t] : 0.0;
    if (t < N * N) sh.W[t] = (a.p == N) ? a.cst[CL::W + t] : 0.0;
}

template <int N, int M, int MODE, bool ALL, typename OT, bool HASC>
__global__ __launch_bounds__(kBlock) void k_bwd_final(SmallArgs a) {
    using S = Sym<N>;
    using CL = CstLayout<N, M>;
    constexpr int VS = S::size + N;
    __shared__ __align__(16) OT shS[kBlock / kWave][Staged<N * N>::elems];
    // Per-wavefront staging of K rows, one step at a time; full wavefronts
    // instead stage K and v of two consecutive steps and d of four, written
    // as one contiguous piece each (rows of one step are only 16 to 64 bytes).
    constexpr int kGroup = Staged<2 * M * N>::elems + Staged<2 * N>::elems + Staged<4 * M>::elems;
    constexpr int kStage = kGroup > Staged<M * N>::elems ? kGroup : Staged<M * N>::elems;
    __shared__ __align__(16) OT stage[kBlock / kWave][kStage];
    OT(*const shK)[kStage] = stage;
    OT* const shK2w = stage[threadIdx.x / kWave];
    OT* const shV2w = shK2w + Staged<2 * M * N>::elems;
    OT* const shD4w = shV2w + Staged<2 * N>::elems;
    OT* const oS = (OT*)a.S;
    OT* const oV = (OT*)a.v;
    OT* const oK = (OT*)a.K;
    OT* const oD = (OT*)a.d;
    __shared__ InvShared<N, M> inv;
    if constexpr (MODE != kVar) {
        load_inv_shared<N, M>(a, inv);
        __syncthreads();
    }
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int64_t g = c / kWave;
    const int64_t cw0 = c - lane;
    const bool active = c < a.NC;
    const int B = a.B;
    const int64_t T = a.T;
    const bool wantS = ALL || oS, wantV = ALL || oV;
    Aff<N> phi;
    aff_identity<N>(phi);
    double Sv[S::size], v[N];
    const int64_t k0 = c * B;
    const int64_t k1 = (k0 + B < T) ? k0 + B : T;
    double fin = 0.0;
    bool ok = true;
    if (active) {
        const double* wvp = a.wave_val + (g + 1) * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = wvp[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = wvp[S::size + i];
        if (lane < kWave - 1 && c + 1 < a.NC) {
            Elem<N> nx;
            load_elem<N>(a.lane_el + (c + 1) * Elem<N>::size, nx);
            anchor<N>(nx, Sv, v);
        }
        if (k1 == T) {  // terminal value S_T, v_T
            double full[N * N];
            full_from_packed<N>(Sv, full);
            if (wantS) store_row<N * N>(oS + T * N * N, full);
            if (wantV) store_row<N>(oV + T * N, v);
        }
    }
    const uint32_t ps = a.per_step;
    const int p = a.p;
    // A wavefront whose 64 chunks are all complete runs without per-step
    // bounds tests (FULL); the last wavefront of the instance keeps them.
    const bool full_wave = (cw0 + kWave <= a.NC) && ((cw0 + kWave) * B <= T) && (B % 4 == 0);
    auto body = [&](bool FULL, int j, const double* rr) {
        const int64_t k = k0 + j;
        if (FULL || (active && k < k1)) {
            double F[N * N], cc[N], L[N * M], U[M * M], Js[S::size], e[N];
            if constexpr (MODE == kVar) {
                const double* Fp = a.F + ((ps & kPS_F) ? k * N * N : 0);
                const double* Lp = a.L + ((ps & kPS_L) ? k * N * M : 0);
                const double* Up = a.U + ((ps & kPS_U) ? k * M * M : 0);
                const double* cp = a.c ? a.c + ((ps & kPS_c) ? k * N : 0) : nullptr;
                LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = Fp[i];
                LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = Lp[i];
                LQT_UNROLL for (int i = 0; i < M * M; ++i) U[i] = Up[i];
                LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = cp ? cp[i] : 0.0;
                const double* rec = a.der + k * CL::der;
                LQT_UNROLL for (int i = 0; i < S::size; ++i) Js[i] = rec[N * M + i];
                LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = rec[N * M + S::size + i];
            } else {
                LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = inv.F[i];
                LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = inv.L[i];
                LQT_UNROLL for (int i = 0; i < M * M; ++i) U[i] = inv.U[i];
                if constexpr (MODE == kInvC) LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = a.c[k * N + i];
                else LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = inv.c[i];
                LQT_UNROLL for (int i = 0; i < S::size; ++i) Js[i] = inv.J[i];
                if constexpr (MODE == kFast) {
                    eta_sq<N>(inv.W, rr, e);
                } else {
                    const double* W = a.cst + CL::W;
                    const double* r = a.r + k * p;
                    LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = 0.0;
                    for (int q = 0; q < p; ++q) {
                        const double rq = r[q];
                        LQT_UNROLL for (int i = 0; i < N; ++i) e[i] = fma(W[i * p + q], rq, e[i]);
                    }
                }
            }
            double K[M * N], d[M], Ft[N * N], ct[N];
            ok = riccati_step<N, M, HASC>(F, cc, L, U, Js, e, Sv, v, K, d, Ft, ct) && ok;
            LQT_UNROLL for (int i = 0; i < S::size; ++i) fin += Sv[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) fin += v[i];
            if (wantS) {
                double full[N * N];
                full_from_packed<N>(Sv, full);
                lds_put_row<N * N>(shS[wv], lane, full);
            }
            if (FULL) {
                // slots: K and v by step parity, d by step modulo 4
                LQT_UNROLL for (int i = 0; i < M * N; ++i)
                    shK2w[lane * Staged<2 * M * N>::stride + (j & 1) * M * N + i] = (OT)K[i];
                if (wantV) LQT_UNROLL for (int i = 0; i < N; ++i)
                    shV2w[lane * Staged<2 * N>::stride + (j & 1) * N + i] = (OT)v[i];
                LQT_UNROLL for (int i = 0; i < M; ++i)
                    shD4w[lane * Staged<4 * M>::stride + (j & 3) * M + i] = (OT)d[i];
            } else {
                lds_put_row<M * N>(shK[wv], lane, K);
                if (wantV) store_row<N>(oV + k * N, v);
                store_row<M>(oD + k * M, d);
            }
            // compose the chunk map: phi <- phi o (Ft, ct)
            Aff<N> step;
            LQT_UNROLL for (int i = 0; i < N * N; ++i) step.F[i] = Ft[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) step.c[i] = ct[i];
            aff_after<N>(step, phi);
        }
        wave_sync();
        if (FULL) {
            if (wantS) wave_store_rows<N * N, false>(shS[wv], oS, cw0, a.NC, B, j, T, lane);
            if ((j & 1) == 0) {  // steps j, j + 1 staged: rows 2 (k / 2), 2 (k / 2) + 1
                wave_store_rows<2 * M * N, false>(shK2w, oK, cw0, a.NC, B / 2, j / 2, T / 2, lane);
                if (wantV) wave_store_rows<2 * N, false>(shV2w, oV, cw0, a.NC, B / 2, j / 2, T / 2, lane);
            }
            if ((j & 3) == 0) wave_store_rows<4 * M, false>(shD4w, oD, cw0, a.NC, B / 4, j / 4, T / 4, lane);
        } else {
            if (wantS) wave_store_rows<N * N, true>(shS[wv], oS, cw0, a.NC, B, j, T, lane);
            wave_store_rows<M * N, true>(shK[wv], oK, cw0, a.NC, B, j, T, lane);
        }
        wave_sync();
    };
    // Reference rows (fast mode): step j uses rA when B-1-j is even, rB
    // otherwise; each buffer is reloaded right after use.
    double rA[N], rB[N];
    auto fetch = [&](bool FULL, int j, double* buf) {
        if constexpr (MODE == kFast) {
            const int64_t row = FULL ? k0 + (j < 0 ? 0 : j) : clamp_row(k0 + j, k0, k1, active);
            load_row<N>(a.r + row * N, buf);
        }
    };
    // whole-chunk row preload: the shapes whose down-sweep keeps the rows
    // without spilling (n m <= 8, every output written)
    constexpr bool kPreRows = ALL && MODE == kFast && N * M <= 8;
    if (kPreRows && full_wave && B == 16) {
        // Every reference row of the chunk is loaded before the first output
        // store: one counter tracks loads and stores alike, so a wait for a
        // row loaded behind earlier stores would also wait for those stores,
        // every step.  Rows are consumed from rr[0], rr[1], two steps per
        // iteration, then shifted down.
        double rr[16][N];
        LQT_UNROLL for (int i = 0; i < 16; ++i) load_row<N>(a.r + (k0 + 15 - i) * N, rr[i]);
#pragma unroll 1
        for (int it = 0; it < 8; ++it) {
            body(true, 15 - 2 * it, rr[0]);
            body(true, 14 - 2 * it, rr[1]);
            LQT_UNROLL for (int i = 0; i < 14; ++i)
                LQT_UNROLL for (int q = 0; q < N; ++q) rr[i][q] = rr[i + 2][q];
        }
    } else if (full_wave) {
        fetch(true, B - 1, rA);
        fetch(true, B - 2, rB);
        for (int j = B - 1; j >= 0; j -= 2) {
            body(true, j, rA);
            fetch(true, j - 2, rA);
            if (j - 1 >= 0) {
                body(true, j - 1, rB);
                fetch(true, j - 3, rB);
            }
        }
    } else {
        fetch(false, B - 1, rA);
        fetch(false, B - 2, rB);
        for (int j = B - 1; j >= 0; j -= 2) {
            body(false, j, rA);
            fetch(false, j - 2, rA);
            if (j - 1 >= 0) {
                body(false, j - 1, rB);
                fetch(false, j - 3, rB);
            }
        }
    }
    if (active) {
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

// Forward roll-out with a compile-time chunk length: every gain row of the
// chunk is loaded into registers before the first store.
template <int N, int M, int BC, typename OT>
__global__ __launch_bounds__(kBlock) void k_fwd_final_regs(SmallArgs a) {
    // full wavefronts stage x and u of four consecutive steps and write each
    // group as one contiguous piece per chunk
    __shared__ __align__(16) OT shX[kBlock / kWave][Staged<4 * N>::elems];
    __shared__ __align__(16) OT shU[kBlock / kWave][Staged<4 * M>::elems];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t cw0 = c - (threadIdx.x & (kWave - 1));
    const bool full = (cw0 + kWave <= a.NC) && ((cw0 + kWave) * BC <= a.T) && (BC % 4 == 0);
    const int wv = threadIdx.x / kWave;
    if (c >= a.NC) return;  // never taken in a full wavefront
    const OT* const iK = (const OT*)a.K;
    const OT* const iD = (const OT*)a.d;
    OT* const oX = (OT*)a.x;
    OT* const oU = (OT*)a.u;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t T = a.T;
    const int64_t k0 = c * BC;
    const int64_t k1 = (k0 + BC < T) ? k0 + BC : T;
    constexpr int KD = M * N + M;
    double gk[BC][KD];
    LQT_UNROLL for (int j = 0; j < BC; ++j) {
        const int64_t kk = clamp_row(k0 + j, k0, k1, true);
        load_row<M * N>(iK + kk * M * N, gk[j]);
        load_row<M>(iD + kk * M, gk[j] + M * N);
    }
    double F[N * N], L[N * M], cc[N];
    LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = a.F[i];
    LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = a.L[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = a.c ? a.c[i] : 0.0;
    double x[N], t[N];
    const int64_t g = c / kWave;
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.wave_x[g * N + i];
    if (lane > 0) {
        Aff<N> pre;
        load_aff<N>(a.lane_aff + (c - 1) * Aff<N>::size, pre);
        mv<N, N>(pre.F, x, t);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = t[i] + pre.c[i];
    }
    double fin = 0.0;
    LQT_UNROLL for (int j = 0; j < BC; ++j) {
        const int64_t k = k0 + j;
        double u[M];
        LQT_UNROLL for (int q = 0; q < M; ++q) {
            double s = gk[j][M * N + q];
            LQT_UNROLL for (int i = 0; i < N; ++i) s = fma(-gk[j][q * N + i], x[i], s);
            u[q] = s;
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            double s = cc[i];
            LQT_UNROLL for (int q = 0; q < N; ++q) s = fma(F[i * N + q], x[q], s);
            LQT_UNROLL for (int q = 0; q < M; ++q) s = fma(L[i * M + q], u[q], s);
            t[i] = s;
        }
        if (full) {
            LQT_UNROLL for (int i = 0; i < N; ++i) shX[wv][lane * Staged<4 * N>::stride + (j & 3) * N + i] = (OT)x[i];
            LQT_UNROLL for (int q = 0; q < M; ++q) shU[wv][lane * Staged<4 * M>::stride + (j & 3) * M + q] = (OT)u[q];
            if ((j & 3) == 3) {
                wave_sync();
                wave_store_rows<4 * N, false>(shX[wv], oX, cw0, a.NC, BC / 4, j / 4, T / 4, lane);
                wave_store_rows<4 * M, false>(shU[wv], oU, cw0, a.NC, BC / 4, j / 4, T / 4, lane);
                wave_sync();
            }
            LQT_UNROLL for (int i = 0; i < N; ++i) {
                x[i] = t[i];
                fin += t[i];
            }
        } else if (k < k1) {
            store_row<N>(oX + k * N, x);
            store_row<M>(oU + k * M, u);
            LQT_UNROLL for (int i = 0; i < N; ++i) {
                x[i] = t[i];
                fin += t[i];
            }
        }
    }
    if (k1 == T) store_row<N>(oX + T * N, x);
    if (!isfinite(fin)) raise_status(a.status, 4);
}

// ---- forward pass ----------------------------------------------------------

// One workgroup: the state at the first step of every wavefront unit.  Up
// to kFwdRegs unit totals per thread are loaded once, all at the start, and
// kept in registers for the roll-out at the end.
constexpr int kFwdRegs = 4;

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
    const bool regs = q <= kFwdRegs;
    Aff<N> u[kFwdRegs];
    if (regs) {
        LQT_UNROLL for (int i = 0; i < kFwdRegs; ++i) {
            if (lo + i < hi) unit_total(lo + i, u[i]);
        }
    }
    Aff<N> agg, t;
    aff_identity<N>(agg);
    if (regs) {
        LQT_UNROLL for (int i = 0; i < kFwdRegs; ++i) {
            if (lo + i < hi) {
                t = u[i];
                aff_after<N>(agg, t);
                agg = t;
            }
        }
    } else {
        for (int g = lo; g < hi; ++g) {
            unit_total(g, t);
            aff_after<N>(agg, t);
            agg = t;
        }
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
    if (regs) {
        LQT_UNROLL for (int k = 0; k < kFwdRegs; ++k) {
            if (lo + k < hi) {
                LQT_UNROLL for (int i = 0; i < N; ++i) a.wave_x[(int64_t)(lo + k) * N + i] = x[i];
                mv<N, N>(u[k].F, x, nx);
                LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + u[k].c[i];
            }
        }
    } else {
        for (int g = lo; g < hi; ++g) {
            LQT_UNROLL for (int i = 0; i < N; ++i) a.wave_x[(int64_t)g * N + i] = x[i];
            unit_total(g, t);
            mv<N, N>(t.F, x, nx);
            LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + t.c[i];
        }
    }
}

// Long instances with few blocks of kBlock units: k_fwd_mid composes the
// unit totals within each block (inclusive prefix, one workgroup per block,
// stored over the backward pass's mid_el, which is no longer needed);
// k_fwd_down applies the totals of the earlier blocks to x_0 in turn, then
// the unit's in-block prefix.
template <int N>
__global__ __launch_bounds__(kBlock) void k_fwd_mid(SmallArgs a) {
    static_assert(Aff<N>::size <= Elem<N>::size, "the unit prefixes reuse mid_el");
    __shared__ double sh[kBlock / kWave][Aff<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int64_t g0 = (int64_t)blockIdx.x * kBlock;
    const int64_t g = g0 + tid;
    const int nb = (int)(a.NG - g0 < kBlock ? a.NG - g0 : kBlock);
    Aff<N> agg, t;
    if (tid < nb) {
        const int64_t last = ((g + 1) * kWave < a.NC ? (g + 1) * kWave : a.NC) - 1;
        load_aff<N>(a.lane_aff + last * Aff<N>::size, agg);
    } else {
        aff_identity<N>(agg);
    }
    for (int d = 1; d < kWave; d <<= 1) {
        Aff<N> Q = shfl_up_aff<N>(agg, d);
        if (lane >= d) aff_after<N>(Q, agg);
    }
    if (lane == kWave - 1) store_aff<N>(sh[wv], agg);
    __syncthreads();
    if (wv > 0) {
        Aff<N> R;
        load_aff<N>(sh[0], R);
        for (int w = 1; w < wv; ++w) {
            load_aff<N>(sh[w], t);
            aff_after<N>(R, t);
            R = t;
        }
        aff_after<N>(R, agg);
    }
    if (tid < nb) store_aff<N>(a.mid_el + g * Aff<N>::size, agg);
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_fwd_down(SmallArgs a) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.NG) return;
    const int64_t b = g / kBlock;
    double x[N], nx[N];
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.x0[i];
    Aff<N> t;
    for (int64_t bb = 0; bb < b; ++bb) {  // earlier blocks are full; uniform over a wavefront
        load_aff<N>(a.mid_el + ((bb + 1) * kBlock - 1) * Aff<N>::size, t);
        mv<N, N>(t.F, x, nx);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + t.c[i];
    }
    if (g > b * kBlock) {
        load_aff<N>(a.mid_el + (g - 1) * Aff<N>::size, t);
        mv<N, N>(t.F, x, nx);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = nx[i] + t.c[i];
    }
    LQT_UNROLL for (int i = 0; i < N; ++i) a.wave_x[g * N + i] = x[i];
}

template <int N, int M, int MODE, bool ALL, typename OT>
__global__ __launch_bounds__(kBlock) void k_fwd_final(SmallArgs a) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.NC) return;
    const OT* const iK = (const OT*)a.K;
    const OT* const iD = (const OT*)a.d;
    OT* const oX = (OT*)a.x;
    OT* const oU = (OT*)a.u;
    const int lane = threadIdx.x & (kWave - 1);
    const int B = a.B;
    const int64_t T = a.T;
    const int64_t k0 = c * B;
    const int64_t k1 = (k0 + B < T) ? k0 + B : T;
    const bool wantX = ALL || oX, wantU = ALL || oU;
    constexpr int KD = M * N + M;  // one gain row: K_k then d_k
    auto load_gain = [&](int64_t k, double* gk) {
        const int64_t kk = clamp_row(k, k0, k1, true);
        load_row<M * N>(iK + kk * M * N, gk);
        load_row<M>(iD + kk * M, gk + M * N);
    };
    const uint32_t ps = a.per_step;
    // time-invariant F, L, c stay in registers for the whole chunk
    double F0[N * N], L0[N * M], c0[N];
    if constexpr (MODE != kVar) {
        LQT_UNROLL for (int i = 0; i < N * N; ++i) F0[i] = a.F[i];
        LQT_UNROLL for (int i = 0; i < N * M; ++i) L0[i] = a.L[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) c0[i] = a.c ? a.c[i] : 0.0;
    }
    double gA[KD], gB[KD];
    load_gain(k0, gA);
    load_gain(k0 + 1, gB);
    double x[N], t[N];
    const int64_t g = c / kWave;
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.wave_x[g * N + i];
    if (lane > 0) {
        Aff<N> pre;
        load_aff<N>(a.lane_aff + (c - 1) * Aff<N>::size, pre);
        mv<N, N>(pre.F, x, t);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = t[i] + pre.c[i];
    }
    double fin = 0.0;
    auto step = [&](int64_t k, const double* gk) {
        double F[N * N], L[N * M], cc[N];
        if constexpr (MODE == kVar) {
            const double* Fp = a.F + ((ps & kPS_F) ? k * N * N : 0);
            const double* Lp = a.L + ((ps & kPS_L) ? k * N * M : 0);
            const double* cp = a.c ? a.c + ((ps & kPS_c) ? k * N : 0) : nullptr;
            LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = Fp[i];
            LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = Lp[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = cp ? cp[i] : 0.0;
        } else {
            LQT_UNROLL for (int i = 0; i < N * N; ++i) F[i] = F0[i];
            LQT_UNROLL for (int i = 0; i < N * M; ++i) L[i] = L0[i];
            if constexpr (MODE == kInvC) LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = a.c[k * N + i];
            else LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = c0[i];
        }
        double u[M];
        LQT_UNROLL for (int q = 0; q < M; ++q) {
            double s = gk[M * N + q];
            LQT_UNROLL for (int i = 0; i < N; ++i) s = fma(-gk[q * N + i], x[i], s);
            u[q] = s;
        }
        if (wantX) store_row<N>(oX + k * N, x);
        if (wantU) store_row<M>(oU + k * M, u);
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            double s = cc[i];
            LQT_UNROLL for (int q = 0; q < N; ++q) s = fma(F[i * N + q], x[q], s);
            LQT_UNROLL for (int q = 0; q < M; ++q) s = fma(L[i * M + q], u[q], s);
            t[i] = s;
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            x[i] = t[i];
            fin += t[i];
        }
    };
    for (int64_t k = k0; k < k1; k += 2) {
        step(k, gA);
        load_gain(k + 2, gA);
        if (k + 1 < k1) step(k + 1, gB);
        load_gain(k + 3, gB);
    }
    if (k1 == T && wantX) store_row<N>(oX + T * N, x);
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

// ---- trajectory by forward prefixes (Method 2 of Section IV-C) --------------
//
// The forward pass reuses the scan elements: V_{0->k} = i (x) a_0 (x) ... (x)
// a_{k-1} with the initial-state element i = (0, x_0, 0, 0, 0), carried as
// (b, C) (fanchor), and x_k = (I + C S_k)^{-1}(b + C v_k) with the value
// function of the backward pass.  Structure as in the backward pass, in the
// other direction: k_m2_reduce folds each chunk left to right and scans the
// wavefront (inclusive prefixes), k_m2_top forms (b, C) at every wavefront
// unit's first step, k_m2_final walks each chunk forward.  The element scan
// does not depend on the backward pass.

template <int N, int M, int MODE>
__global__ __launch_bounds__(kBlock) void k_m2_reduce(SmallArgs a) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool active = c < a.NC;
    Elem<N> P;
    if (active) {
        Step<N, M> st;
        if constexpr (MODE != kVar) load_invariant<N, M>(a, st);
        const int64_t k0 = c * a.B;
        const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
        load_step<N, M, MODE>(a, k0, st);
        step_elem<N, M>(st, P);
        for (int64_t k = k0 + 1; k < k1; ++k) {
            load_step<N, M, MODE>(a, k, st);
            Elem<N> E;
            step_elem<N, M>(st, E);
            combine<N>(P, E);  // E <- P (x) E
            P = E;
        }
    } else {
        set_identity<N>(P);
    }
    // prefix across the wavefront: lane l ends with E_0 (x) ... (x) E_l
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_up_elem<N>(P, d);
        if (lane >= d) combine<N>(Q, P);  // P <- Q (x) P
    }
    if (active) store_elem<N>(a.m2_el + c * Elem<N>::size, P);
}

// One workgroup: (C, b) of V_{0->k} at the start of every one of `cnt`
// consecutive segments (out[g]), from the segment totals and x_0.  The total
// of segment g is the prefix element el[last], last = min((g + 1) span, n_el)
// - 1: wavefront units over the in-wave prefixes (span 64), or blocks of
// kBlock units over the in-block prefixes of the unit totals.
template <int N>
__global__ __launch_bounds__(kBlock) void k_m2_top(SmallArgs a, const double* el, int span, int64_t n_el, int cnt,
                                                   double* out) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    __shared__ double sh[kBlock / kWave][Elem<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int NG = cnt;
    const int q = (NG + kBlock - 1) / kBlock;
    const int lo = tid * q < NG ? tid * q : NG;
    const int hi = lo + q < NG ? lo + q : NG;
    auto unit_total = [&](int g, Elem<N>& t) {
        const int64_t last = ((int64_t)(g + 1) * span < n_el ? (int64_t)(g + 1) * span : n_el) - 1;
        load_elem<N>(el + last * Elem<N>::size, t);
    };
    Elem<N> agg, t;
    set_identity<N>(agg);
    for (int g = lo; g < hi; ++g) {
        unit_total(g, t);
        combine<N>(agg, t);  // t <- agg (x) t
        agg = t;
    }
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_up_elem<N>(agg, d);
        if (lane >= d) combine<N>(Q, agg);
    }
    if (lane == kWave - 1) store_elem<N>(sh[wv], agg);
    __syncthreads();
    // prefix of everything before this thread's range, anchored on x_0
    Elem<N> R;
    set_identity<N>(R);
    for (int w = 0; w < wv; ++w) {
        load_elem<N>(sh[w], t);
        combine<N>(R, t);
        R = t;
    }
    Elem<N> prev = shfl_up_elem<N>(agg, 1);
    if (lane == 0) set_identity<N>(prev);
    combine<N>(R, prev);  // prev <- R (x) prev
    double b[N], Cs[S::size];
    LQT_UNROLL for (int i = 0; i < N; ++i) b[i] = a.x0[i];
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Cs[i] = 0.0;
    fanchor<N>(prev, b, Cs);
    for (int g = lo; g < hi; ++g) {
        double* o = out + (int64_t)g * VS;
        LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = Cs[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = b[i];
        unit_total(g, t);
        fanchor<N>(t, b, Cs);
    }
}

// Long instances (more than kBlock wavefront units): k_m2_mid forms the
// inclusive prefixes of the unit totals within each block of kBlock units
// (one workgroup per block), k_m2_top the value at every block start, and
// k_m2_down the value at every unit start: the block's start value advanced
// by the in-block prefix of the units before it.
template <int N>
__global__ __launch_bounds__(kBlock) void k_m2_mid(SmallArgs a) {
    __shared__ double sh[kBlock / kWave][Elem<N>::size];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int64_t g0 = (int64_t)blockIdx.x * kBlock;
    const int64_t g = g0 + tid;
    const int nb = (int)(a.NG - g0 < kBlock ? a.NG - g0 : kBlock);
    Elem<N> agg, t;
    if (tid < nb) {
        const int64_t last = ((g + 1) * kWave < a.NC ? (g + 1) * kWave : a.NC) - 1;
        load_elem<N>(a.m2_el + last * Elem<N>::size, agg);
    } else {
        set_identity<N>(agg);
    }
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_up_elem<N>(agg, d);
        if (lane >= d) combine<N>(Q, agg);  // agg <- Q (x) agg
    }
    if (lane == kWave - 1) store_elem<N>(sh[wv], agg);
    __syncthreads();
    if (wv > 0) {
        Elem<N> R;
        load_elem<N>(sh[0], R);
        for (int w = 1; w < wv; ++w) {
            load_elem<N>(sh[w], t);
            combine<N>(R, t);  // t <- R (x) t
            R = t;
        }
        combine<N>(R, agg);
    }
    if (tid < nb) store_elem<N>(a.m2_mid + g * Elem<N>::size, agg);
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_m2_down(SmallArgs a) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.NG) return;
    const int64_t b = g / kBlock;
    double bb[N], Cs[S::size];
    const double* bv = a.m2_blk + b * VS;
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Cs[i] = bv[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) bb[i] = bv[S::size + i];
    if (g > b * kBlock) {
        Elem<N> e;
        load_elem<N>(a.m2_mid + (g - 1) * Elem<N>::size, e);
        fanchor<N>(e, bb, Cs);
    }
    double* o = a.m2_val + g * VS;
    LQT_UNROLL for (int i = 0; i < S::size; ++i) o[i] = Cs[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) o[S::size + i] = bb[i];
}

// Lane c: (b, C) at its chunk's first step (its unit's value advanced by the
// in-wave prefix of the lanes before it), then per step x_k from S_k, v_k,
// u_k = -K_k x_k + d_k, and (b, C) advanced by the step's element.
template <int N, int M, int MODE, typename OT>
__global__ __launch_bounds__(kBlock) void k_m2_final(SmallArgs a) {
    using S = Sym<N>;
    constexpr int VS = S::size + N;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.NC) return;
    const int lane = threadIdx.x & (kWave - 1);
    const OT* const iS = (const OT*)a.S;
    const OT* const iV = (const OT*)a.v;
    const OT* const iK = (const OT*)a.K;
    const OT* const iD = (const OT*)a.d;
    OT* const oX = (OT*)a.x;
    OT* const oU = (OT*)a.u;
    double b[N], Cs[S::size];
    const double* gv = a.m2_val + (c / kWave) * VS;
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Cs[i] = gv[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) b[i] = gv[S::size + i];
    if (lane > 0) {
        Elem<N> e;
        load_elem<N>(a.m2_el + (c - 1) * Elem<N>::size, e);
        fanchor<N>(e, b, Cs);
    }
    Step<N, M> st;
    if constexpr (MODE != kVar) load_invariant<N, M>(a, st);
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    const int64_t kend = (k1 == a.T) ? k1 : k1 - 1;  // the last chunk also gives x_T
    // Software pipeline: at the top of step k one explicit wait covers the
    // rows of step k (and every earlier request); then step k-1's x, u are
    // stored and step k+1's rows requested, and step k's arithmetic runs with
    // no further wait.  A wait thus never drains a request younger than one
    // step (one counter tracks loads and stores alike, so the wait the
    // compiler would place before the first use of a row would also drain
    // the stores and loads issued just before it).
    struct Rows {
        double S[N * N], v[N], K[M * N], d[M], r[N];
    };
    auto fetch = [&](int64_t k, Rows& R) {
        load_row<N * N>(iS + k * N * N, R.S);
        load_row<N>(iV + k * N, R.v);
        if (k < a.T) {
            load_row<M * N>(iK + k * M * N, R.K);
            load_row<M>(iD + k * M, R.d);
            if constexpr (MODE == kFast) load_row<N>(a.r + k * N, R.r);
        }
    };
    double px[N], pu[M];
    bool pend_x = false, pend_u = false;
    int64_t pk = 0;
    auto flush = [&]() {
        if (pend_x) store_row<N>(oX + pk * N, px);
        if (pend_u) store_row<M>(oU + pk * M, pu);
        pend_x = pend_u = false;
    };
    double Wl[N * N];  // W = H^T X (square H, X)
    if constexpr (MODE == kFast) {
        LQT_UNROLL for (int i = 0; i < N * N; ++i) Wl[i] = a.cst[CstLayout<N, M>::W + i];
    }
    auto step = [&](int64_t k, const Rows& R) {
        double x[N];
        prefix_state<N>(b, Cs, R.S, R.v, x);
        LQT_UNROLL for (int i = 0; i < N; ++i) px[i] = x[i];
        pk = k;
        pend_x = oX != nullptr;
        if (k == a.T) return;
        LQT_UNROLL for (int i = 0; i < M; ++i) {
            double sacc = R.d[i];
            LQT_UNROLL for (int j = 0; j < N; ++j) sacc = fma(-R.K[i * N + j], x[j], sacc);
            pu[i] = sacc;
        }
        pend_u = oU != nullptr;
        if constexpr (MODE == kFast) {
            eta_sq<N>(Wl, R.r, st.e);
        } else {
            load_step<N, M, MODE>(a, k, st);
        }
        Elem<N> E;
        step_elem<N, M>(st, E);
        fanchor<N>(E, b, Cs);
    };
    Rows RA, RB;
    fetch(k0, RA);
    for (int64_t k = k0; k <= kend; k += 2) {
        vm_wait_all();
        flush();
        if (k + 1 <= kend) fetch(k + 1, RB);
        step(k, RA);
        if (k + 1 > kend) break;
        vm_wait_all();
        flush();
        if (k + 2 <= kend) fetch(k + 2, RA);
        step(k + 1, RB);
    }
    vm_wait_all();
    flush();

}

template <int N, int M, int MODE, typename OT>
static void run_mode(const SmallArgs& a, hipStream_t s, const StageHook* h, const SideStream* side) {
    using CL = CstLayout<N, M>;
    const unsigned grid = (unsigned)((a.NC + kBlock - 1) / kBlock);
    const bool all = a.S && a.v && a.x && a.u;
    const bool even = (N % 2 == 0) && (M % 2 == 0);
    if (MODE == kVar) {
        {
            Stage st(h, "init_status", s);
            k_init_status<<<1, 64, 0, s>>>(a.status);
        }
        const unsigned pg = (unsigned)((a.T + 1 + kBlock - 1) / kBlock);
        Stage st(h, "prep_varying", s);
        k_prep_varying<N, M><<<pg, kBlock, 0, s>>>(a);
    } else {
        Stage st(h, "prep_invariant", s);
        k_prep_invariant<N, M><<<1, 64, 0, s>>>(a);
    }
    // forward element scan of the prefix trajectory: independent of the
    // backward pass, on the side stream when the plan provides one
    const bool m2 = a.want_fwd && a.traj == 1;
    hipStream_t s2 = s;
    if (m2 && side && hipEventRecord(side->fork, s) == hipSuccess &&
        hipStreamWaitEvent(side->side, side->fork, 0) == hipSuccess)
        s2 = side->side;
    if (m2) {
        {
            Stage st(h, "m2_reduce", s2);
            k_m2_reduce<N, M, MODE><<<grid, kBlock, 0, s2>>>(a);
        }
        if (a.NG > kBlock) {
            {
                Stage st(h, "m2_mid", s2);
                k_m2_mid<N><<<(unsigned)a.NB, kBlock, 0, s2>>>(a);
            }
            {
                Stage st(h, "m2_top", s2);
                k_m2_top<N><<<1, kBlock, 0, s2>>>(a, a.m2_mid, kBlock, a.NG, a.NB, a.m2_blk);
            }
            Stage st(h, "m2_down", s2);
            k_m2_down<N><<<(unsigned)a.NB, kBlock, 0, s2>>>(a);
        } else {
            Stage st(h, "m2_top", s2);
            k_m2_top<N><<<1, kBlock, 0, s2>>>(a, a.m2_el, kWave, a.NC, a.NG, a.m2_val);
        }
    }
    {
        Stage st(h, "bwd_reduce", s);
        k_bwd_reduce<N, M, MODE><<<grid, kBlock, 0, s>>>(a);
    }
    if (a.NG > kBlock) {
        {
            Stage st(h, "bwd_mid", s);
            k_bwd_mid<N><<<(unsigned)a.NB, kBlock, 0, s>>>(a);
        }
        const int chain = a.NB <= kDownChain ? 1 : 0;
        if (!chain) {
            Stage st(h, "bwd_top", s);
            k_bwd_top<N><<<1, kBlock, 0, s>>>(a.mid_el, (int64_t)kBlock * Elem<N>::size, a.NB, a.cst + CL::ST,
                                               a.blk_val);
        }
        Stage st(h, "bwd_down", s);
        k_bwd_down<N><<<(unsigned)((a.NG + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(a, CL::ST, chain);
    } else {
        Stage st(h, "bwd_top", s);
        k_bwd_top<N><<<1, kBlock, 0, s>>>(a.lane_el, (int64_t)kWave * Elem<N>::size, a.NG, a.cst + CL::ST,
                                           a.wave_val);
    }
    {
        Stage st(h, "bwd_final", s);
        const bool hasc = a.c != nullptr;
        if (all && hasc) k_bwd_final<N, M, MODE, true, OT, true><<<grid, kBlock, 0, s>>>(a);
        else if (all) k_bwd_final<N, M, MODE, true, OT, false><<<grid, kBlock, 0, s>>>(a);
        else if (hasc) k_bwd_final<N, M, MODE, false, OT, true><<<grid, kBlock, 0, s>>>(a);
        else k_bwd_final<N, M, MODE, false, OT, false><<<grid, kBlock, 0, s>>>(a);
    }
    if (m2) {
        if (s2 != s) {  // join: the walk needs the element scan
            (void)hipEventRecord(side->join, s2);
            (void)hipStreamWaitEvent(s, side->join, 0);
        }
        Stage st(h, "m2_final", s);
        k_m2_final<N, M, MODE, OT><<<grid, kBlock, 0, s>>>(a);
    } else if (a.want_fwd) {
        if (a.NG > kBlock && a.NB <= kDownChain) {
            {
                Stage st(h, "fwd_mid", s);
                k_fwd_mid<N><<<(unsigned)a.NB, kBlock, 0, s>>>(a);
            }
            Stage st(h, "fwd_down", s);
            k_fwd_down<N><<<(unsigned)((a.NG + kBlock - 1) / kBlock), kBlock, 0, s>>>(a);
        } else {
            Stage st(h, "fwd_top", s);
            k_fwd_top<N><<<1, kBlock, 0, s>>>(a);
        }
        Stage st(h, "fwd_final", s);
        const bool regs = (MODE == kFast || MODE == kInv) && all && even;
        bool fdone = false;
        if constexpr (N % 2 == 0 && M % 2 == 0) {
            // gain rows of the whole chunk in registers: up to 128 values
            fdone = true;
            if (regs && a.B == 4) k_fwd_final_regs<N, M, 4, OT><<<grid, kBlock, 0, s>>>(a);
            else if (regs && a.B == 8) k_fwd_final_regs<N, M, 8, OT><<<grid, kBlock, 0, s>>>(a);
            else if constexpr (M * N <= 8) {
                if (regs && a.B == 16) k_fwd_final_regs<N, M, 16, OT><<<grid, kBlock, 0, s>>>(a);
                else fdone = false;
            } else {
                fdone = false;
            }
        }
        if (fdone) {
        } else if (all) k_fwd_final<N, M, MODE, true, OT><<<grid, kBlock, 0, s>>>(a);
        else k_fwd_final<N, M, MODE, false, OT><<<grid, kBlock, 0, s>>>(a);
    }
}

template <int N, int M, typename OT>
static void run_typed(const SmallArgs& a, hipStream_t s, const StageHook* h, const SideStream* side) {
    const uint32_t ps = a.per_step & (kPS_F | kPS_c | kPS_L | kPS_H | kPS_X | kPS_U);
    if (ps == kPS_c) run_mode<N, M, kInvC, OT>(a, s, h, side);
    else if (ps) run_mode<N, M, kVar, OT>(a, s, h, side);
    else if (a.p == N) run_mode<N, M, kFast, OT>(a, s, h, side);
    else run_mode<N, M, kInv, OT>(a, s, h, side);
}

template <int N, int M>
static hipError_t run_small(const SmallArgs& a, hipStream_t s, const StageHook* h, const SideStream* side) {
    if (a.f32) run_typed<N, M, float>(a, s, h, side);
    else run_typed<N, M, double>(a, s, h, side);
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

hipError_t small_solve(const SmallArgs& a, hipStream_t s, const StageHook* hook, const SideStream* side) {
#define X(N, M) if (a.n == N && a.m == M) return run_small<N, M>(a, s, hook, side);
    LQT_SMALL_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace lqt
