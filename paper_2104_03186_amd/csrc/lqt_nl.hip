// Iterated linearisation for nonlinear dynamics (the nonlinear extension of Section IV-D): the device
// side of one round -- the first-order Taylor expansion of the dynamics about
// the nominal trajectory, and the round's convergence measure.  Model: the
// unicycle of the nonlinear experiment (Section VI-E).  The nominal is held
// in double on every plan (a MIXED plan converts at entry and exit).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"

namespace lqt {

namespace {

constexpr int kNlBlock = 256;

// Block maximum of v (all threads of the block call it) into *out, ordered
// as the bit patterns of non-negative doubles (a NaN is reported as +inf).
__device__ __forceinline__ void block_max_into(double v, unsigned long long* out) {
    __shared__ double sh[kNlBlock];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kNlBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = (sh[0] == sh[0]) ? sh[0] : __builtin_inf();
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
    }
}

// One thread per step k: F_k = df/dx, L_k = df/du at (xbar_k, ubar_k),
// c_k = f(xbar_k, ubar_k) - F_k xbar_k - L_k ubar_k, and a double copy of
// ubar_k for the change measure.  Unicycle, x = (p_x, p_y, theta, s),
// u = (a, w): f = (p_x + s cos(theta) dt, p_y + s sin(theta) dt, theta + w dt,
// s + a dt).  With prev (the previous round's change word), the previous
// round's change max |ubar_k - copy_k| is folded in before the copy is
// overwritten: the nominal of this round is the previous round's result.
__global__ __launch_bounds__(kNlBlock) void k_nl_linearise_unicycle(NlArgs g, unsigned long long* prev) {
    const int64_t k = (int64_t)blockIdx.x * kNlBlock + threadIdx.x;
    double diff = 0.0;
    if (k < g.T) {
        const double* xb = g.x + k * 4;
        const double* ub = g.u + k * 2;
        const double px = xb[0], py = xb[1], th = xb[2], sp = xb[3];
        const double a = ub[0], w = ub[1];
        const double dt = g.dt[k];
        double sn, cs;
        sincos(th, &sn, &cs);
        double F[16] = {1.0, 0.0, -sp * sn * dt, cs * dt,
                        0.0, 1.0, sp * cs * dt, sn * dt,
                        0.0, 0.0, 1.0, 0.0,
                        0.0, 0.0, 0.0, 1.0};
        double L[8] = {0.0, 0.0,
                       0.0, 0.0,
                       0.0, dt,
                       dt, 0.0};
        const double fx[4] = {px + sp * cs * dt, py + sp * sn * dt, th + w * dt, sp + a * dt};
        const double xv[4] = {px, py, th, sp};
        const double uv[2] = {a, w};
        double* Fo = g.F + k * 16;
        double* Lo = g.L + k * 8;
        double* co = g.c + k * 4;
        for (int i = 0; i < 4; ++i) {
            double acc = fx[i];
            for (int j = 0; j < 4; ++j) acc -= F[i * 4 + j] * xv[j];
            for (int j = 0; j < 2; ++j) acc -= L[i * 2 + j] * uv[j];
            co[i] = acc;
        }
        for (int i = 0; i < 16; ++i) Fo[i] = F[i];
        for (int i = 0; i < 8; ++i) Lo[i] = L[i];
        if (prev) diff = fmax(fabs(a - g.ubar[k * 2]), fabs(w - g.ubar[k * 2 + 1]));
        g.ubar[k * 2] = a;
        g.ubar[k * 2 + 1] = w;
    }
    if (prev) block_max_into(diff, prev);
}

// max |u_new - ubar| over the horizon into *out (ordered as the bit patterns
// of non-negative doubles; *out starts at zero).
__global__ __launch_bounds__(kNlBlock) void k_nl_change(NlArgs g, unsigned long long* out) {
    const double* u = g.u;
    const int64_t n = g.T * 2;
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kNlBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNlBlock)
        mx = fmax(mx, fabs(u[i] - g.ubar[i]));
    block_max_into(mx, out);
}

// Zero `count` doubles (the change words and the round status words).
__global__ void k_nl_zero(double* p, int count, int32_t* st, int nst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (p && i < count) p[i] = 0.0;
    if (st && i < nst) st[i] = 0;
}

// The first non-zero round status into *out.
__global__ void k_nl_status(const int32_t* st, int n, int32_t* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t v = 0;
    for (int i = 0; i < n && v == 0; ++i) v = st[i];
    *out = v;
}

template <typename S, typename D>
__global__ __launch_bounds__(kNlBlock) void k_nl_convert(const S* src, D* dst, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * kNlBlock + threadIdx.x;
    if (i < count) dst[i] = (D)src[i];
}

unsigned grid_for(int64_t count) { return (unsigned)((count + kNlBlock - 1) / kNlBlock); }

}  // namespace

hipError_t nl_start(double* change, int iterations, int32_t* round_status, hipStream_t s) {
    const int n = iterations > 0 ? iterations : 1;
    k_nl_zero<<<(n + 255) / 256, 256, 0, s>>>(change, iterations, round_status, iterations);
    return hipGetLastError();
}

hipError_t nl_linearise(const NlArgs& g, double* prev_change, hipStream_t s) {
    unsigned long long* prev = (unsigned long long*)prev_change;
    k_nl_linearise_unicycle<<<grid_for(g.T), kNlBlock, 0, s>>>(g, prev);
    return hipGetLastError();
}

hipError_t nl_change(const NlArgs& g, double* out, hipStream_t s) {
    if (!out) return hipSuccess;
    const unsigned grid = grid_for(g.T * 2) < 1024u ? grid_for(g.T * 2) : 1024u;
    k_nl_change<<<grid, kNlBlock, 0, s>>>(g, (unsigned long long*)out);
    return hipGetLastError();
}

hipError_t convert_array(const void* src, bool src_f32, void* dst, bool dst_f32, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned grid = grid_for(count);
    if (src_f32 && !dst_f32)
        k_nl_convert<float, double><<<grid, kNlBlock, 0, s>>>((const float*)src, (double*)dst, count);
    else if (!src_f32 && dst_f32)
        k_nl_convert<double, float><<<grid, kNlBlock, 0, s>>>((const double*)src, (float*)dst, count);
    else if (src_f32)
        k_nl_convert<float, float><<<grid, kNlBlock, 0, s>>>((const float*)src, (float*)dst, count);
    else
        k_nl_convert<double, double><<<grid, kNlBlock, 0, s>>>((const double*)src, (double*)dst, count);
    return hipGetLastError();
}

hipError_t nl_finish(const int32_t* round_status, int iterations, int32_t* status, hipStream_t s) {
    if (!status) return hipSuccess;
    k_nl_status<<<1, 64, 0, s>>>(round_status, iterations, status);
    return hipGetLastError();
}

}  // namespace lqt
