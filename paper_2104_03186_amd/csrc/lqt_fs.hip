// Finite state and control spaces (Section III-D): value functions by a
// reverse scan of one-step conditional value functions under the min-plus
// product (the associative operator of Section III-B), the control law, and
// the trajectory by composing the closed-loop maps (Method 1 of Section
// III-C).
//
// Structure: the horizon is cut into NC <= kFsMaxNC chunks of B steps and the
// chunks into groups of kFsGroup.
//   k_fs_reduce  one workgroup per chunk: P_c = E_{k0} (x) ... (x) E_{k1-1}
//                (D x D, folded right to left; E_k never formed:
//                (E_k (x) P)(x, y) = min_u l_k(x, u) + P(f_k(x, u), y));
//   k_fs_group   one workgroup per group: Q_g = P_{c0} (x) ... (x) P_{c1-1};
//   k_fs_top     one workgroup: V at every group start from V_T (min-plus
//                matrix-vector products, lanes = states);
//   k_fs_gdown   one workgroup per group: V at every chunk start;
//   k_fs_final   one wavefront per chunk: V_k, u_k and the closed-loop next
//                state of every step (lanes = states, V_{k+1} shuffled across
//                the lanes), and the chunk's composed map phi_c;
//   k_fs_fwd_group one wavefront per group: the composition of its chunk maps;
//   k_fs_fwd_top one wavefront: the state at every group start (group maps in
//                LDS); k_fs_fwd_gdown: the state at every chunk start;
//   k_fs_fwd_final one wavefront per chunk: x_k and the applied control,
//                64 steps of closed-loop maps staged in LDS at a time.
// The step tables are staged in LDS a slab of steps at a time, so the
// sequential walks wait on memory once per slab, not once per step.
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"

namespace lqt {

namespace {

constexpr int kFsBlock = 256;
constexpr int kWaveFs = 64;
constexpr int kFsMaxD = 32;
constexpr int kFsStage = 64;          // steps staged per round of the forward walk
constexpr int kSlabBytes = 32 * 1024;  // LDS for the step tables of a slab of steps
constexpr int kGroupLds = 40 * 1024;   // LDS for a batch of chunk products in the group fold

// Copy n elements from global memory into LDS (thread tid of nt), eight
// loads in flight per thread before their stores: a load followed at once by
// its LDS store would wait for that load, one global-memory latency per
// element.  op is applied to every value on the way.
template <typename T, typename Op>
__device__ __forceinline__ void stage_copy(T* dst, const T* src, int64_t n, int tid, int nt, Op op) {
    int64_t e = tid;
    for (; e + 7 * (int64_t)nt < n; e += 8 * (int64_t)nt) {
        T r[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = src[e + q * nt];
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[e + q * nt] = op(r[q]);
    }
    for (; e < n; e += nt) dst[e] = op(src[e]);
}

struct Same {
    template <typename T>
    __device__ T operator()(T v) const { return v; }
};

// Steps per slab of staged tables (at least one).
__device__ __forceinline__ int fs_slab_steps(const FsArgs& a) {
    const int per = a.D * a.Du * (int)(sizeof(double) + sizeof(int32_t));
    const int s = kSlabBytes / per;
    return s > 0 ? s : 1;
}

// Stage the tables of steps [ks, ke) (per-step tables) or the shared tables
// (once, ks = ke = -1 ignored) into LDS: nx[j][x][u], cs[j][x][u], j = k - ks.
// Next states outside 0..D-1 become -1.
__device__ __forceinline__ void fs_stage(const FsArgs& a, int64_t ks, int64_t ke, int32_t* nx, double* cs,
                                         int tid, int nthreads) {
    const int row = a.D * a.Du;
    const int64_t n_steps = ke - ks;
    const int64_t nn = (a.per_step & 1) ? n_steps * row : row;
    const int64_t nc = (a.per_step & 2) ? n_steps * row : row;
    const int32_t* gn = a.next + ((a.per_step & 1) ? ks * row : 0);
    const double* gc = a.cost + ((a.per_step & 2) ? ks * row : 0);
    const int D = a.D;
    stage_copy(nx, gn, nn, tid, nthreads, [D](int32_t v) { return (v >= 0 && v < D) ? v : -1; });
    stage_copy(cs, gc, nc, tid, nthreads, Same{});
}

// Offsets of step j of a slab in the staged tables.
__device__ __forceinline__ int fs_nrow(const FsArgs& a, int j) { return (a.per_step & 1) ? j * a.D * a.Du : 0; }
__device__ __forceinline__ int fs_crow(const FsArgs& a, int j) { return (a.per_step & 2) ? j * a.D * a.Du : 0; }

__global__ __launch_bounds__(kFsBlock) void k_fs_reduce(FsArgs a) {
    __shared__ double P[2][kFsMaxD * kFsMaxD];
    __shared__ double cs[kSlabBytes / 12];
    __shared__ int32_t nx[kSlabBytes / 12];
    const int D = a.D, DD = D * D, Du = a.Du;
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    const int S = fs_slab_steps(a);
    // the entries of this thread (e = t + q kFsBlock): row offset i Du in the
    // step tables and column j, fixed for the whole fold
    constexpr int kEntries = kFsMaxD * kFsMaxD / kFsBlock;
    int erow[kEntries], ecol[kEntries];
    const int ne = t < DD ? (DD - t + kFsBlock - 1) / kFsBlock : 0;
#pragma unroll
    for (int q = 0; q < kEntries; ++q) {
        const int e = t + q * kFsBlock;
        erow[q] = (e / D) * Du;
        ecol[q] = e % D;
    }
    for (int e = t; e < DD; e += kFsBlock) P[0][e] = (e / D == e % D) ? 0.0 : __builtin_inf();
    int cur = 0;
    for (int64_t ke = k1; ke > k0; ke -= S) {
        const int64_t ks = (ke - S > k0) ? ke - S : k0;
        __syncthreads();
        fs_stage(a, ks, ke, nx, cs, t, kFsBlock);
        __syncthreads();
        for (int64_t k = ke - 1; k >= ks; --k) {
            const int jn = fs_nrow(a, (int)(k - ks)), jc = fs_crow(a, (int)(k - ks));
#pragma unroll
            for (int q = 0; q < kEntries; ++q) {
                if (q < ne) {
                    double acc = __builtin_inf();
                    for (int u = 0; u < Du; ++u) {
                        const int to = nx[jn + erow[q] + u];
                        if (to >= 0) acc = fmin(acc, cs[jc + erow[q] + u] + P[cur][to * D + ecol[q]]);
                    }
                    P[cur ^ 1][t + q * kFsBlock] = acc;
                }
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    double* out = a.P + c * DD;
    for (int e = t; e < DD; e += kFsBlock) out[e] = P[cur][e];
}

__global__ __launch_bounds__(kFsBlock) void k_fs_group(FsArgs a) {
    __shared__ double Q[2][kFsMaxD * kFsMaxD];
    __shared__ double Pb[kGroupLds / sizeof(double)];
    const int D = a.D, DD = D * D;
    const int t = threadIdx.x;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    int nb = (int)(kGroupLds / sizeof(double)) / DD;
    nb = nb < 1 ? 1 : nb;
    for (int e = t; e < DD; e += kFsBlock) Q[0][e] = (e / D == e % D) ? 0.0 : __builtin_inf();
    int cur = 0;
    // chunk products staged a batch at a time (every load in flight together)
    for (int ce = c1; ce > c0; ce -= nb) {
        const int cs = (ce - nb > c0) ? ce - nb : c0;
        __syncthreads();
        stage_copy(Pb, a.P + (int64_t)cs * DD, (int64_t)(ce - cs) * DD, t, kFsBlock, Same{});
        __syncthreads();
        for (int c = ce - 1; c >= cs; --c) {
            const double* Pc = Pb + (c - cs) * DD;
            for (int e = t; e < DD; e += kFsBlock) {
                const int i = e / D, j = e - (e / D) * D;
                double acc = __builtin_inf();
                for (int m = 0; m < D; ++m) acc = fmin(acc, Pc[i * D + m] + Q[cur][m * D + j]);
                Q[cur ^ 1][e] = acc;
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    __syncthreads();
    for (int e = t; e < DD; e += kFsBlock) a.Q[(int64_t)g * DD + e] = Q[cur][e];
}

constexpr int kChainLds = 48 * 1024;  // LDS for a batch of matrices of a chain

// Chain of min-plus matrix-vector products from V_end over the matrices
// M_{hi-1}, ..., M_{lo} (consecutive, D*D each); lanes are states.  The
// matrices are staged into LDS a batch at a time (every load of a batch in
// flight together, so the chain waits on memory once per batch), and each
// product reads its row and the current V (broadcast) from LDS with every
// read independent of the others.  out[c] receives the value before matrix c
// for c in (lo, hi) and, with out_lo, for c = lo.
__device__ __forceinline__ double fs_chain(const double* M, int lo, int hi, int D, int lane, double V,
                                           double* out, bool out_lo, double* lds) {
    __shared__ double vsh[kFsMaxD];
    __shared__ double ob[32 * kFsMaxD];  // values of the batch, stored after it (no global store
                                         // may be outstanding at the barriers between products)
    const int DD = D * D;
    int nb = kChainLds / (int)sizeof(double) / DD;
    nb = nb < 1 ? 1 : (nb > 32 ? 32 : nb);
    for (int ce = hi; ce > lo; ce -= nb) {
        const int cs = (ce - nb > lo) ? ce - nb : lo;
        __syncthreads();
        const double* src = M + (int64_t)cs * DD;
        stage_copy(lds, src, (int64_t)(ce - cs) * DD, lane, (int)blockDim.x, Same{});
        __syncthreads();
        for (int c = ce - 1; c >= cs; --c) {
            const double* row = lds + (c - cs) * DD + (lane < D ? lane : 0) * D;
            if (lane < D) vsh[lane] = V;
            __syncthreads();
            double acc = __builtin_inf();
#pragma unroll
            for (int j = 0; j < kFsMaxD; ++j)
                if (j < D) acc = fmin(acc, row[j] + vsh[j]);
            __syncthreads();
            V = lane < D ? acc : __builtin_inf();
            if (lane < D) ob[(c - cs) * kFsMaxD + lane] = V;
        }
        for (int c = cs; c < ce; ++c)
            if (lane < D && (c > lo || out_lo)) out[(int64_t)c * D + lane] = ob[(c - cs) * kFsMaxD + lane];
    }
    return V;
}

__global__ __launch_bounds__(kFsBlock) void k_fs_top(FsArgs a) {
    __shared__ double lds[kChainLds / sizeof(double)];
    const int lane = threadIdx.x;
    const int D = a.D;
    const double V = lane < D ? a.cost_T[lane] : __builtin_inf();
    if (lane < D) {
        a.gval[(int64_t)a.NG * D + lane] = V;
        a.cval[(int64_t)a.NC * D + lane] = V;
    }
    (void)fs_chain(a.Q, 0, a.NG, D, lane, V, a.gval, true, lds);
}

__global__ __launch_bounds__(kFsBlock) void k_fs_gdown(FsArgs a) {
    __shared__ double lds[kChainLds / sizeof(double)];
    const int lane = threadIdx.x;
    const int D = a.D;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    const double V = lane < D ? a.gval[(int64_t)(g + 1) * D + lane] : __builtin_inf();
    (void)fs_chain(a.P, c0, c1, D, lane, V, a.cval, false, lds);
    if (lane < D) a.cval[(int64_t)c0 * D + lane] = a.gval[(int64_t)g * D + lane];
}

__global__ __launch_bounds__(kWaveFs) void k_fs_final(FsArgs a) {
    __shared__ double cs[kSlabBytes / 12];
    __shared__ int32_t nx[kSlabBytes / 12];
    const int lane = threadIdx.x;
    const int D = a.D, Du = a.Du;
    const int64_t c = blockIdx.x;
    const int64_t k0 = c * a.B;
    const int64_t k1 = (k0 + a.B < a.T) ? k0 + a.B : a.T;
    const bool st = lane < D;
    const int S = fs_slab_steps(a);
    double V = st ? a.cval[(c + 1) * D + lane] : __builtin_inf();
    int phi = lane;
    if (c == a.NC - 1 && st && a.V) a.V[a.T * D + lane] = V;
    for (int64_t ke = k1; ke > k0; ke -= S) {
        const int64_t ks = (ke - S > k0) ? ke - S : k0;
        __syncthreads();
        fs_stage(a, ks, ke, nx, cs, lane, kWaveFs);
        __syncthreads();
        for (int64_t k = ke - 1; k >= ks; --k) {
            const int jn = fs_nrow(a, (int)(k - ks)), jc = fs_crow(a, (int)(k - ks));
            double best = __builtin_inf();
            int arg = -1, to = -1;
            for (int u = 0; u < Du; ++u) {
                const int nxt = st ? nx[jn + lane * Du + u] : -1;
                const double vn = __shfl(V, nxt >= 0 ? nxt : 0, kWaveFs);
                if (nxt >= 0) {
                    const double val = cs[jc + lane * Du + u] + vn;
                    if (val < best) {  // strict: the smallest index among equal minima
                        best = val;
                        arg = u;
                        to = nxt;
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
    }
    if (st) a.phi[c * D + lane] = phi;
}

// Group map: the composition of the group's chunk maps, in time order.
__global__ __launch_bounds__(kWaveFs) void k_fs_fwd_group(FsArgs a) {
    const int lane = threadIdx.x;
    const int D = a.D;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    int rows[kFsGroup];
#pragma unroll
    for (int i = 0; i < kFsGroup; ++i) rows[i] = (c0 + i < c1 && lane < D) ? a.phi[(int64_t)(c0 + i) * D + lane] : -1;
    int y = lane;
#pragma unroll
    for (int i = 0; i < kFsGroup; ++i) {
        if (c0 + i < c1) {
            const int v = __shfl(rows[i], y >= 0 ? y : 0, kWaveFs);
            y = y >= 0 ? v : -1;
        }
    }
    if (lane < D) a.gphi[(int64_t)g * D + lane] = y;
}

__global__ __launch_bounds__(kWaveFs) void k_fs_fwd_top(FsArgs a) {
    __shared__ int32_t ph[(kFsMaxNC / kFsGroup) * kFsMaxD];
    const int D = a.D;
    for (int e = threadIdx.x; e < a.NG * D; e += kWaveFs) ph[e] = a.gphi[e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    int x = a.x0;
    a.gxs[0] = x;
    for (int g = 0; g < a.NG; ++g) {
        x = x >= 0 ? ph[g * D + x] : -1;
        a.gxs[g + 1] = x;
    }
    if (a.status) {
        const double v0 = a.cval[a.x0];
        *a.status = (v0 < __builtin_inf()) ? 0 : 4;  // LQT_ENONFINITE: no admissible path
    }
}

__global__ __launch_bounds__(kWaveFs) void k_fs_fwd_gdown(FsArgs a) {
    __shared__ int32_t ph[kFsGroup * kFsMaxD];
    const int D = a.D;
    const int g = blockIdx.x;
    const int c0 = g * kFsGroup;
    const int c1 = (c0 + kFsGroup < a.NC) ? c0 + kFsGroup : a.NC;
    for (int e = threadIdx.x; e < (c1 - c0) * D; e += kWaveFs) ph[e] = a.phi[(int64_t)c0 * D + e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    int x = a.gxs[g];
    for (int c = c0; c < c1; ++c) {
        a.xs[c] = x;
        x = x >= 0 ? ph[(c - c0) * D + x] : -1;
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
        stage_copy(nb, a.nxt + kb * D, S * D, lane, kWaveFs, Same{});
        stage_copy(ub, a.ulaw + kb * D, S * D, lane, kWaveFs, Same{});
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
    run("fs_top", [&] { k_fs_top<<<1, kFsBlock, 0, s>>>(a); });
    run("fs_gdown", [&] { k_fs_gdown<<<a.NG, kFsBlock, 0, s>>>(a); });
    run("fs_final", [&] { k_fs_final<<<a.NC, kWaveFs, 0, s>>>(a); });
    if (a.x || a.ux || a.status) {
        run("fs_fwd_group", [&] { k_fs_fwd_group<<<a.NG, kWaveFs, 0, s>>>(a); });
        run("fs_fwd_top", [&] { k_fs_fwd_top<<<1, kWaveFs, 0, s>>>(a); });
        if (a.x || a.ux) {
            run("fs_fwd_gdown", [&] { k_fs_fwd_gdown<<<a.NG, kWaveFs, 0, s>>>(a); });
            run("fs_fwd_final", [&] { k_fs_fwd_final<<<a.NC, kWaveFs, 0, s>>>(a); });
        }
    }
    return hipGetLastError();
}

}  // namespace lqt
