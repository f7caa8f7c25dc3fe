// Finite state and control spaces (Section III-D): value functions by a
// reverse scan of one-step conditional value functions under the min-plus
// product (the associative operator of Section III-B), the control law, and
// the trajectory by composing the closed-loop maps (Method 1 of Section
// III-C).
//
// Structure: the horizon is cut into NC <= 256 chunks of B steps and the
// chunks into groups of kGroup.
//   k_fs_reduce  one workgroup per chunk: P_c = E_{k0} (x) ... (x) E_{k1-1}
//                (D x D, folded right to left; E_k never formed:
//                (E_k (x) P)(x, y) = min_u l_k(x, u) + P(f_k(x, u), y));
//   k_fs_group   one workgroup per group: Q_g = P_{c0} (x) ... (x) P_{c1-1};
//   k_fs_top     one wavefront: V at every group start from V_T (min-plus
//                matrix-vector products, lanes = states);
//   k_fs_gdown   one wavefront per group: V at every chunk start;
//   k_fs_final   one wavefront per chunk: V_k, u_k and the closed-loop next
//                state of every step (lanes = states, V_{k+1} shuffled across
//                the lanes), and the chunk's composed map phi_c;
//   k_fs_fwd_top one workgroup: the state at every chunk start (phi_c in LDS);
//   k_fs_fwd_final one wavefront per chunk: x_k and the applied control,
//                64 steps of closed-loop maps staged in LDS at a time.
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"

namespace lqt {

namespace {

constexpr int kFsBlock = 256;
constexpr int kWaveFs = 64;
constexpr int kFsMaxD = 32;
constexpr int kFsStage = 64;  // steps staged per round of the forward walk

__device__ __forceinline__ int fs_next(const FsArgs& a, int64_t k, int i, int u) {
    const int32_t* t = a.next + ((a.per_step & 1) ? k * a.D * a.Du : 0);
    const int nx = t[i * a.Du + u];
    return (nx >= 0 && nx < a.D) ? nx : -1;
}

__device__ __forceinline__ double fs_cost(const FsArgs& a, int64_t k, int i, int u) {
    const double* t = a.cost + ((a.per_step & 2) ? k * a.D * a.Du : 0);
    return t[i * a.Du + u];
}

__global__ __launch_bounds__(kFsBlock) void k_fs_reduce(FsArgs a) {
    __shared__ double P[2][kFsMaxD * kFsMaxD];
    const int D = a.D, DD = D * D;
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    for (int e = t; e < DD; e += kFsBlock) P[0][e] = (e / D == e % D) ? 0.0 : __builtin_inf();
    __syncthreads();
    int cur = 0;
    for (int64_t k = k1 - 1; k >= k0; --k) {
        for (int e = t; e < DD; e += kFsBlock) {
            const int i = e / D, j = e - (e / D) * D;
            double acc = __builtin_inf();
            for (int u = 0; u < a.Du; ++u) {
                const int nx = fs_next(a, k, i, u);
                if (nx >= 0) acc = fmin(acc, fs_cost(a, k, i, u) + P[cur][nx * D + j]);
            }
            P[cur ^ 1][e] = acc;
        }
        __syncthreads();
        cur ^= 1;
    }
    double* out = a.P + c * DD;
    for (int e = t; e < DD; e += kFsBlock) out[e] = P[cur][e];
}

__global__ __launch_bounds__(kFsBlock) void k_fs_group(FsArgs a) {
    __shared__ double Q[2][kFsMaxD * kFsMaxD];
    __shared__ double Pc[kFsMaxD * kFsMaxD];
    const int D = a.D, DD = D * D;
    const int t = threadIdx.x;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    for (int e = t; e < DD; e += kFsBlock) Q[0][e] = (e / D == e % D) ? 0.0 : __builtin_inf();
    int cur = 0;
    for (int c = c1 - 1; c >= c0; --c) {
        __syncthreads();
        for (int e = t; e < DD; e += kFsBlock) Pc[e] = a.P[(int64_t)c * DD + e];
        __syncthreads();
        for (int e = t; e < DD; e += kFsBlock) {
            const int i = e / D, j = e - (e / D) * D;
            double acc = __builtin_inf();
            for (int m = 0; m < D; ++m) acc = fmin(acc, Pc[i * D + m] + Q[cur][m * D + j]);
            Q[cur ^ 1][e] = acc;
        }
        cur ^= 1;
    }
    __syncthreads();
    for (int e = t; e < DD; e += kFsBlock) a.Q[(int64_t)g * DD + e] = Q[cur][e];
}

// V(i) <- min_j M(i, j) + V(j); lanes are states (V of lane j by shuffle).
__device__ __forceinline__ double fs_matvec(const double* M, int D, int lane, double V) {
    double acc = __builtin_inf();
    for (int j = 0; j < D; ++j) {
        const double vj = __shfl(V, j, kWaveFs);
        if (lane < D) acc = fmin(acc, M[lane * D + j] + vj);
    }
    return acc;
}

__global__ __launch_bounds__(kWaveFs) void k_fs_top(FsArgs a) {
    const int lane = threadIdx.x;
    const int D = a.D;
    double V = lane < D ? a.cost_T[lane] : __builtin_inf();
    if (lane < D) {
        a.gval[(int64_t)a.NG * D + lane] = V;
        a.cval[(int64_t)a.NC * D + lane] = V;
    }
    for (int g = a.NG - 1; g >= 0; --g) {
        V = fs_matvec(a.Q + (int64_t)g * D * D, D, lane, V);
        if (lane < D) a.gval[(int64_t)g * D + lane] = V;
    }
}

__global__ __launch_bounds__(kWaveFs) void k_fs_gdown(FsArgs a) {
    const int lane = threadIdx.x;
    const int D = a.D;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    double V = lane < D ? a.gval[(int64_t)(g + 1) * D + lane] : __builtin_inf();
    for (int c = c1 - 1; c > c0; --c) {
        V = fs_matvec(a.P + (int64_t)c * D * D, D, lane, V);
        if (lane < D) a.cval[(int64_t)c * D + lane] = V;
    }
    if (lane < D) a.cval[(int64_t)c0 * D + lane] = a.gval[(int64_t)g * D + lane];
}

__global__ __launch_bounds__(kWaveFs) void k_fs_final(FsArgs a) {
    const int lane = threadIdx.x;
    const int D = a.D;
    const int64_t c = blockIdx.x;
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    const bool st = lane < D;
    double V = st ? a.cval[(c + 1) * D + lane] : __builtin_inf();
    int phi = lane;
    if (c == a.NC - 1 && st && a.V) a.V[a.T * D + lane] = V;
    for (int64_t k = k1 - 1; k >= k0; --k) {
        double best = __builtin_inf();
        int arg = -1, to = -1;
        for (int u = 0; u < a.Du; ++u) {
            const int nx = st ? fs_next(a, k, lane, u) : -1;
            const double vn = __shfl(V, nx >= 0 ? nx : 0, kWaveFs);
            if (nx >= 0) {
                const double val = fs_cost(a, k, lane, u) + vn;
                if (val < best) {  // strict: the smallest index among equal minima
                    best = val;
                    arg = u;
                    to = nx;
                }
            }
        }
        const int pn = __shfl(phi, to >= 0 ? to : 0, kWaveFs);
        phi = to >= 0 ? pn : -1;
        if (st) {
            if (a.V) a.V[k * D + lane] = best;
            a.ulaw[k * D + lane] = arg;
            a.nxt[k * D + lane] = to;
        }
        V = best;
    }
    if (st) a.phi[c * D + lane] = phi;
}

__global__ __launch_bounds__(kFsBlock) void k_fs_fwd_top(FsArgs a) {
    __shared__ int32_t ph[kFsMaxNC * kFsMaxD];
    const int D = a.D;
    for (int e = threadIdx.x; e < a.NC * D; e += kFsBlock) ph[e] = a.phi[e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    int x = a.x0;
    a.xs[0] = x;
    for (int c = 0; c < a.NC; ++c) {
        x = x >= 0 ? ph[c * D + x] : -1;
        a.xs[c + 1] = x;
    }
    if (a.status) {
        const double v0 = a.cval[a.x0];
        *a.status = (v0 < __builtin_inf()) ? 0 : 4;  // LQT_ENONFINITE: no admissible path
    }
}

__global__ __launch_bounds__(kWaveFs) void k_fs_fwd_final(FsArgs a) {
    __shared__ int32_t nb[kFsStage * kFsMaxD], ub[kFsStage * kFsMaxD];
    __shared__ int32_t xk[kFsStage], uk[kFsStage];
    const int lane = threadIdx.x;
    const int D = a.D;
    const int64_t c = blockIdx.x;
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    int x = a.xs[c];
    for (int64_t kb = k0; kb < k1; kb += kFsStage) {
        const int S = (int)((k1 - kb < kFsStage) ? k1 - kb : kFsStage);
        for (int e = lane; e < S * D; e += kWaveFs) {
            nb[e] = a.nxt[kb * D + e];
            ub[e] = a.ulaw[kb * D + e];
        }
        __syncthreads();
        if (lane == 0) {
            for (int j = 0; j < S; ++j) {
                xk[j] = x;
                uk[j] = x >= 0 ? ub[j * D + x] : -1;
                x = x >= 0 ? nb[j * D + x] : -1;
            }
        }
        __syncthreads();
        if (lane < S) {
            if (a.x) a.x[kb + lane] = xk[lane];
            if (a.ux) a.ux[kb + lane] = uk[lane];
        }
        __syncthreads();
    }
    if (c == a.NC - 1 && lane == 0 && a.x) a.x[a.T] = x;
}

}  // namespace

void fs_shape(int64_t T, int32_t& B, int32_t& NC, int32_t& NG) {
    const int64_t b = (T + kFsMaxNC - 1) / kFsMaxNC;
    B = (int32_t)(b < 16 ? 16 : b);
    NC = (int32_t)((T + B - 1) / B);
    NG = (NC + kFsGroup - 1) / kFsGroup;
}

hipError_t fs_solve(const FsArgs& a, hipStream_t s, const StageHook* h) {
    auto run = [&](const char* name, auto launch) {
        if (h) h->begin(h->ctx, name, s);
        launch();
        if (h) h->end(h->ctx, s);
    };
    run("fs_reduce", [&] { k_fs_reduce<<<a.NC, kFsBlock, 0, s>>>(a); });
    run("fs_group", [&] { k_fs_group<<<a.NG, kFsBlock, 0, s>>>(a); });
    run("fs_top", [&] { k_fs_top<<<1, kWaveFs, 0, s>>>(a); });
    run("fs_gdown", [&] { k_fs_gdown<<<a.NG, kWaveFs, 0, s>>>(a); });
    run("fs_final", [&] { k_fs_final<<<a.NC, kWaveFs, 0, s>>>(a); });
    if (a.x || a.ux || a.status) {
        run("fs_fwd_top", [&] { k_fs_fwd_top<<<1, kFsBlock, 0, s>>>(a); });
        if (a.x || a.ux) run("fs_fwd_final", [&] { k_fs_fwd_final<<<a.NC, kWaveFs, 0, s>>>(a); });
    }
    return hipGetLastError();
}

}  // namespace lqt
