// Batched lane kernel: many n <= 4 instances of moderate horizon solved in
// one launch, one workgroup of 256 lanes per instance, the whole scan of one
// instance inside its workgroup.
//
// Lane c owns chunk c of B = ceil(T / 256) consecutive steps (NC <= 256
// chunks) and keeps a scan element in registers.  The reverse scan is the
// block processing of Section V-C with the parallel scan of Section II-C over
// the chunk elements, entirely on chip:
//   1. fold: the lane's one-step elements into its chunk element (combination
//      rule of Section IV-A in the step form);
//   2. suffix scan across the wavefront (shuffles), then across the four
//      wavefronts of the workgroup (LDS);
//   3. the value function at the lane's chunk end: the suffix after it
//      anchored on the terminal value (Section IV-B);
//   4. down-sweep of the chunk in Riccati form fused with the gain
//      extraction (writes S, v, K, d) composing the chunk's closed-loop
//      affine map (Method 1 of Section IV-C);
//   5. prefix of the maps across the wavefront and the workgroup from x_0:
//      the state at the lane's chunk start;
//   6. roll-out of the chunk: u_k = -K_k x_k + d_k, x_{k+1} = F x_k + c_k +
//      L u_k (writes x, u).
// The instance constants come from a preceding one-workgroup-per-instance
// kernel (k_lb_prep).  Time-invariant instances (c may vary per step).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_lane.hpp"
#include "lqt_ops.hpp"

namespace lqt {

namespace {

template <int N, int M>
__global__ __launch_bounds__(64) void k_lb_prep(const SmallArgs* tab, int ninst) {
    using CL = CstLayout<N, M>;
    using S = Sym<N>;
    if (threadIdx.x != 0 || (int)blockIdx.x >= ninst) return;
    const SmallArgs& a = tab[blockIdx.x];
    double* cst = a.cst;
    bool ok;
    double ST[S::size], vT[N];
    if (a.p == N) {
        ok = step_constants_sq<N, M>(a.L, a.U, a.H, a.X, cst + CL::G, cst + CL::J, cst + CL::W);
    } else {
        ok = step_constants<N, M>(a.L, a.U, a.H, a.X, a.p, cst + CL::G, cst + CL::J, cst + CL::W);
    }
    terminal_value<N>(a, ST, vT);
    LQT_UNROLL for (int i = 0; i < S::size; ++i) cst[CL::ST + i] = ST[i];
    LQT_UNROLL for (int i = 0; i < N; ++i) cst[CL::VT + i] = vT[i];
    if (a.status) *a.status = ok ? 0 : 3;
}

template <int N>
LQT_DI void aff_apply(const Aff<N>& f, const double* x, double* y) {
    LQT_UNROLL for (int i = 0; i < N; ++i) {
        double s = f.c[i];
        LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(f.F[i * N + j], x[j], s);
        y[i] = s;
    }
}

template <int N, int M, int MODE, typename OT>
__global__ __launch_bounds__(kBlock) void k_lb_solve(const SmallArgs* tab, int ninst) {
    using S = Sym<N>;
    using CL = CstLayout<N, M>;
    __shared__ double sh[2][kBlock / kWave][Elem<N>::size];
    __shared__ double shA[kBlock / kWave][Aff<N>::size];
    if ((int)blockIdx.x >= ninst) return;
    const SmallArgs& a = tab[blockIdx.x];
    const int c = threadIdx.x;  // chunk of this lane
    const int lane = c & (kWave - 1);
    const int wv = c / kWave;
    const int NC = (int)a.NC;
    const int B = a.B;
    const int64_t T = a.T;
    const bool active = c < NC;
    const int64_t k0 = (int64_t)c * B;
    const int64_t k1 = (k0 + B < T) ? k0 + B : T;
    const int nw = (NC + kWave - 1) / kWave;  // wavefronts holding chunks
    Step<N, M> st;
    load_invariant<N, M>(a, st);
    // 1. fold the chunk: P = a_k0 (x) ... (x) a_k1-1
    Elem<N> P;
    if (active) {
        load_step<N, M, MODE>(a, k1 - 1, st);
        step_elem<N, M>(st, P);
        for (int64_t k = k1 - 2; k >= k0; --k) {
            load_step<N, M, MODE>(a, k, st);
            step_combine<N, M>(st, P);
        }
    } else {
        set_identity<N>(P);
    }
    // 2. suffix across the wavefront, then across the workgroup's wavefronts
    for (int d = 1; d < kWave; d <<= 1) {
        Elem<N> Q = shfl_down_elem<N>(P, d);
        if (lane + d < kWave && c + d < NC) {
            combine<N>(P, Q);
            P = Q;
        }
    }
    Elem<N> R;
    const bool has_R = wave_suffix<N>(sh, P, nw, R);
    // 3. value at the chunk end: (suffix after this chunk) anchored on the terminal value
    Elem<N> nxt = shfl_down_elem<N>(P, 1);
    const bool has_nxt = lane + 1 < kWave && c + 1 < NC;
    if (has_R) {
        if (has_nxt) combine<N>(nxt, R);
        nxt = R;
    }
    double Sv[S::size], v[N];
    LQT_UNROLL for (int i = 0; i < S::size; ++i) Sv[i] = a.cst[CL::ST + i];
    LQT_UNROLL for (int i = 0; i < N; ++i) v[i] = a.cst[CL::VT + i];
    if (has_R || has_nxt) anchor<N>(nxt, Sv, v);
    // 4. down-sweep with gains; chunk map
    OT* const oS = (OT*)a.S;
    OT* const oV = (OT*)a.v;
    OT* const oK = (OT*)a.K;
    OT* const oD = (OT*)a.d;
    Aff<N> phi;
    aff_identity<N>(phi);
    double fin = 0.0;
    bool ok = true;
    if (active) {
        if (k1 == T) {
            double full[N * N];
            full_from_packed<N>(Sv, full);
            if (oS) store_row<N * N>(oS + T * N * N, full);
            if (oV) store_row<N>(oV + T * N, v);
        }
        for (int64_t k = k1 - 1; k >= k0; --k) {
            double cc[N], K[M * N], d[M], Ft[N * N], ct[N];
            if constexpr (MODE == kInvC) {
                LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = a.c[k * N + i];
            } else {
                LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = st.c[i];
            }
            load_step<N, M, MODE>(a, k, st);  // eta_k
            ok = riccati_step<N, M, true>(st.F, cc, a.L, a.U, st.J, st.e, Sv, v, K, d, Ft, ct) && ok;
            LQT_UNROLL for (int i = 0; i < S::size; ++i) fin += Sv[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) fin += v[i];
            if (oS) {
                double full[N * N];
                full_from_packed<N>(Sv, full);
                store_row<N * N>(oS + k * N * N, full);
            }
            if (oV) store_row<N>(oV + k * N, v);
            store_row<M * N>(oK + k * M * N, K);
            store_row<M>(oD + k * M, d);
            Aff<N> f;
            LQT_UNROLL for (int i = 0; i < N * N; ++i) f.F[i] = Ft[i];
            LQT_UNROLL for (int i = 0; i < N; ++i) f.c[i] = ct[i];
            aff_after<N>(f, phi);
        }
        if (!ok) raise_status(a.status, 3);
        if (!isfinite(fin)) raise_status(a.status, 4);
    }
    if (!a.want_fwd) return;  // uniform over the workgroup
    // 5. inclusive prefix of the maps across the wavefront (lane l: f_l o ... o f_0)
    for (int d = 1; d < kWave; d <<= 1) {
        Aff<N> Q = shfl_up_aff<N>(phi, d);
        if (lane >= d) aff_after<N>(Q, phi);
    }
    if (lane == kWave - 1) {
        LQT_UNROLL for (int i = 0; i < N * N; ++i) shA[wv][i] = phi.F[i];
        LQT_UNROLL for (int i = 0; i < N; ++i) shA[wv][N * N + i] = phi.c[i];
    }
    __syncthreads();
    double x[N];
    LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = a.x0[i];
    for (int w = 0; w < wv; ++w) {  // totals of the earlier wavefronts, in time order
        Aff<N> tw;
        LQT_UNROLL for (int i = 0; i < N * N; ++i) tw.F[i] = shA[w][i];
        LQT_UNROLL for (int i = 0; i < N; ++i) tw.c[i] = shA[w][N * N + i];
        double y[N];
        aff_apply<N>(tw, x, y);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = y[i];
    }
    Aff<N> before = shfl_up_aff<N>(phi, 1);  // maps of the earlier lanes of the wavefront
    if (lane > 0) {
        double y[N];
        aff_apply<N>(before, x, y);
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = y[i];
    }
    if (!active) return;
    // 6. roll-out of the chunk
    OT* const oX = (OT*)a.x;
    OT* const oU = (OT*)a.u;
    for (int64_t k = k0; k < k1; ++k) {
        double K[M * N], d[M], u[M], cc[N], y[N];
        load_row<M * N>(oK + k * M * N, K);
        load_row<M>(oD + k * M, d);
        if (oX) store_row<N>(oX + k * N, x);
        LQT_UNROLL for (int i = 0; i < M; ++i) {
            double s = d[i];
            LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(-K[i * N + j], x[j], s);
            u[i] = s;
        }
        if (oU) store_row<M>(oU + k * M, u);
        if constexpr (MODE == kInvC) {
            LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = a.c[k * N + i];
        } else {
            LQT_UNROLL for (int i = 0; i < N; ++i) cc[i] = st.c[i];
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) {
            double s = cc[i];
            LQT_UNROLL for (int j = 0; j < N; ++j) s = fma(st.F[i * N + j], x[j], s);
            LQT_UNROLL for (int j = 0; j < M; ++j) s = fma(a.L[i * M + j], u[j], s);
            y[i] = s;
        }
        LQT_UNROLL for (int i = 0; i < N; ++i) x[i] = y[i];
    }
    if (k1 == T && oX) store_row<N>(oX + T * N, x);
}

template <int N, int M, int MODE, typename OT>
void lb_run(const SmallArgs* d_tab, int ninst, hipStream_t s, const StageHook* h) {
    if (h) h->begin(h->ctx, "lb_prep", s);
    k_lb_prep<N, M><<<(unsigned)ninst, 64, 0, s>>>(d_tab, ninst);
    if (h) h->end(h->ctx, s);
    if (h) h->begin(h->ctx, "lb_solve", s);
    k_lb_solve<N, M, MODE, OT><<<(unsigned)ninst, kBlock, 0, s>>>(d_tab, ninst);
    if (h) h->end(h->ctx, s);
}

template <int N, int M>
hipError_t lb_dispatch(int mode, bool f32, const SmallArgs* d_tab, int ninst, hipStream_t s, const StageHook* h) {
    if (mode == kFast) {
        if (f32) lb_run<N, M, kFast, float>(d_tab, ninst, s, h);
        else lb_run<N, M, kFast, double>(d_tab, ninst, s, h);
    } else if (mode == kInvC) {
        if (f32) lb_run<N, M, kInvC, float>(d_tab, ninst, s, h);
        else lb_run<N, M, kInvC, double>(d_tab, ninst, s, h);
    } else {
        if (f32) lb_run<N, M, kInv, float>(d_tab, ninst, s, h);
        else lb_run<N, M, kInv, double>(d_tab, ninst, s, h);
    }
    return hipGetLastError();
}

}  // namespace

int lane_batch_mode(int n, int p, uint32_t per_step, bool has_c) {
    const uint32_t ps = per_step & (kPS_F | kPS_c | kPS_L | kPS_H | kPS_X | kPS_U);
    if (ps & ~(uint32_t)kPS_c) return -1;  // time-varying matrices: not on this kernel
    if (ps & kPS_c) return has_c ? (int)kInvC : -1;
    return p == n ? (int)kFast : (int)kInv;
}

int lane_batch_chunk(int64_t T) { return (int)((T + kBlock - 1) / kBlock); }

hipError_t lane_batch_solve(int n, int m, int mode, bool f32, const SmallArgs* d_tab, int ninst, hipStream_t s,
                            const StageHook* h) {
    if (ninst <= 0) return hipSuccess;
#define X(NN, MM) \
    if (n == NN && m == MM) return lb_dispatch<NN, MM>(mode, f32, d_tab, ninst, s, h);
    X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(3, 3) X(4, 1) X(4, 2) X(4, 3) X(4, 4)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace lqt
