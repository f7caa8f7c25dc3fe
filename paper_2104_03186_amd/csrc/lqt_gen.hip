// Generalised stage cost (the extension to more general cost functions,
// Section IV-D of Sarkka & Garcia-Fernandez, arXiv 2104.03186):
//   l_k = 1/2 (H x - r)^T X (H x - r) + (H x - r)^T M (u - s) + 1/2 (u - s)^T U (u - s).
// The instance is transformed on the device to the standard form, solved by
// the ordinary pipelines, and its gains and controls mapped back.  With
// Z = U^{-1} M^T (m x p):
//   F~ = F - L Z H,   c~_k = c_k + L Z r_k + L s_k,   X~ = X - M Z,   U~ = U,
//   K_k = K~_k + Z H,   d_k = d~_k + Z r_k + s_k,
//   u_k = u~_k - Z (H x_k - r_k) + s_k        (S, v and x are unchanged).
// L, H, X, U and M are time-invariant here; F, c, r and s may vary per step.
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"

namespace lqt {

namespace {

constexpr int kGenBlock = 256;

// One workgroup: Z (Cholesky of U, then one column of Z per thread), X~, Z H,
// L Z and, when F is shared by every step, F~.
__global__ __launch_bounds__(kGenBlock) void k_gen_const(GenArgs g) {
    extern __shared__ double Uc[];  // m x m
    const int t = threadIdx.x;
    const int n = g.n, m = g.m, p = g.p;
    for (int i = t; i < m * m; i += kGenBlock) {
        const int r = i / m, c = i - r * m;
        Uc[i] = 0.5 * (g.U[r * m + c] + g.U[c * m + r]);
    }
    __syncthreads();
    // right-looking Cholesky U = R R^T (R lower, in place).  U is not checked
    // here: U~ = U, and the solve of the transformed instance reports a U
    // that is not positive definite through the instance's status word.
    for (int j = 0; j < m; ++j) {
        __syncthreads();
        if (t == 0) Uc[j * m + j] = sqrt(Uc[j * m + j]);
        __syncthreads();
        const double rjj = Uc[j * m + j];
        for (int i = j + 1 + t; i < m; i += kGenBlock) Uc[i * m + j] /= rjj;
        __syncthreads();
        for (int idx = t; idx < (m - j - 1) * (m - j - 1); idx += kGenBlock) {
            const int i = j + 1 + idx / (m - j - 1), c = j + 1 + idx % (m - j - 1);
            if (c <= i) Uc[i * m + c] -= Uc[i * m + j] * Uc[c * m + j];
        }
    }
    __syncthreads();
    // Z = U^{-1} M^T: thread q solves R R^T z = (column q of M^T = row q of M)
    for (int q = t; q < p; q += kGenBlock) {
        double* z = g.Z;  // m x p, column q written in place
        for (int i = 0; i < m; ++i) {
            double sacc = g.M ? g.M[q * m + i] : 0.0;
            for (int k = 0; k < i; ++k) sacc -= Uc[i * m + k] * z[k * p + q];
            z[i * p + q] = sacc / Uc[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double sacc = z[i * p + q];
            for (int k = i + 1; k < m; ++k) sacc -= Uc[k * m + i] * z[k * p + q];
            z[i * p + q] = sacc / Uc[i * m + i];
        }
    }
    __threadfence_block();
    __syncthreads();
    // X~ = X - M Z (p x p), made exactly symmetric
    for (int idx = t; idx < p * p; idx += kGenBlock) {
        const int i = idx / p, j = idx - i * p;
        if (j < i) continue;
        double a = 0.0, b = 0.0;
        for (int k = 0; k < m; ++k) {
            const double mi = g.M ? g.M[i * m + k] : 0.0, mj = g.M ? g.M[j * m + k] : 0.0;
            a += mi * g.Z[k * p + j];
            b += mj * g.Z[k * p + i];
        }
        const double xij = 0.5 * (g.X[i * p + j] + g.X[j * p + i]) - 0.5 * (a + b);
        g.Xt[i * p + j] = xij;
        g.Xt[j * p + i] = xij;
    }
    // Z H (m x n) and L Z (n x p)
    for (int idx = t; idx < m * n; idx += kGenBlock) {
        const int i = idx / n, j = idx - i * n;
        double sacc = 0.0;
        for (int q = 0; q < p; ++q) sacc += g.Z[i * p + q] * g.H[q * n + j];
        g.ZH[idx] = sacc;
    }
    for (int idx = t; idx < n * p; idx += kGenBlock) {
        const int i = idx / p, j = idx - i * p;
        double sacc = 0.0;
        for (int k = 0; k < m; ++k) sacc += g.L[i * m + k] * g.Z[k * p + j];
        g.LZ[idx] = sacc;
    }
    __threadfence_block();
    __syncthreads();
    // F~ = F - L (Z H) when F is shared by every step
    if (!(g.per_step & kPS_F)) {
        for (int idx = t; idx < n * n; idx += kGenBlock) {
            const int i = idx / n, j = idx - i * n;
            double sacc = g.F[idx];
            for (int k = 0; k < m; ++k) sacc -= g.L[i * m + k] * g.ZH[k * n + j];
            g.Ft[idx] = sacc;
        }
    }
}

// One thread per entry of c~ ([T][n]): c~_k = c_k + (L Z) r_k + L s_k.
__global__ __launch_bounds__(kGenBlock) void k_gen_c(GenArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x;
    const int n = g.n, m = g.m, p = g.p;
    if (idx >= g.T * n) return;
    const int64_t k = idx / n;
    const int i = (int)(idx - k * n);
    double acc = g.c ? g.c[(g.per_step & kPS_c) ? idx : i] : 0.0;
    const double* rk = g.r + k * p;
    for (int q = 0; q < p; ++q) acc += g.LZ[i * p + q] * rk[q];
    if (g.s) {
        const double* sk = g.s + k * m;
        for (int j = 0; j < m; ++j) acc += g.L[i * m + j] * sk[j];
    }
    g.ct[idx] = acc;
}

// One thread per entry of a per-step F~ ([T][n][n]): F~_k = F_k - L (Z H).
__global__ __launch_bounds__(kGenBlock) void k_gen_F(GenArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x;
    const int n = g.n, m = g.m;
    if (idx >= g.T * n * n) return;
    const int e = (int)(idx % (n * n));
    const int i = e / n, j = e - i * n;
    double acc = g.F[idx];
    for (int q = 0; q < m; ++q) acc -= g.L[i * m + q] * g.ZH[q * n + j];
    g.Ft[idx] = acc;
}

// One thread per gain entry ([T][m][n]): K_k = K~_k + Z H.
template <typename OT>
__global__ __launch_bounds__(kGenBlock) void k_gen_K(GenArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x;
    const int mn = g.m * g.n;
    if (idx >= g.T * mn) return;
    OT* K = (OT*)g.K;
    K[idx] = (OT)((double)K[idx] + g.ZH[idx % mn]);
}

// One thread per control entry ([T][m]): with w = Z r_k + s_k,
// d_k = d~_k + w and u_k = u~_k - (Z H) x_k + w.
template <typename OT>
__global__ __launch_bounds__(kGenBlock) void k_gen_du(GenArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * kGenBlock + threadIdx.x;
    const int n = g.n, m = g.m, p = g.p;
    if (idx >= g.T * m) return;
    const int64_t k = idx / m;
    const int i = (int)(idx - k * m);
    double w = g.s ? g.s[idx] : 0.0;
    const double* rk = g.r + k * p;
    for (int q = 0; q < p; ++q) w += g.Z[i * p + q] * rk[q];
    if (g.d) {
        OT* d = (OT*)g.d;
        d[idx] = (OT)((double)d[idx] + w);
    }
    if (g.u) {
        OT* u = (OT*)g.u;
        const OT* xk = (const OT*)g.x + k * n;
        double a = (double)u[idx] + w;
        for (int j = 0; j < n; ++j) a -= g.ZH[i * n + j] * (double)xk[j];
        u[idx] = (OT)a;
    }
}

unsigned grid_of(int64_t count) { return (unsigned)((count + kGenBlock - 1) / kGenBlock); }

}  // namespace

size_t gen_ws_doubles(int n, int m, int p, int64_t T, bool f_per_step) {
    return (size_t)m * p + (size_t)m * n + (size_t)n * p + (size_t)p * p +
           (f_per_step ? (size_t)T * n * n : (size_t)n * n) + (size_t)T * n + 64;
}

void gen_layout(GenArgs& g, double* ws) {
    g.Z = ws;
    g.ZH = g.Z + (size_t)g.m * g.p;
    g.LZ = g.ZH + (size_t)g.m * g.n;
    g.Xt = g.LZ + (size_t)g.n * g.p;
    g.Ft = g.Xt + (size_t)g.p * g.p;
    g.ct = g.Ft + ((g.per_step & kPS_F) ? (size_t)g.T * g.n * g.n : (size_t)g.n * g.n);
}

hipError_t gen_transform(const GenArgs& g, hipStream_t s) {
    k_gen_const<<<1, kGenBlock, sizeof(double) * (size_t)g.m * g.m, s>>>(g);
    k_gen_c<<<grid_of(g.T * g.n), kGenBlock, 0, s>>>(g);
    if (g.per_step & kPS_F) k_gen_F<<<grid_of(g.T * g.n * g.n), kGenBlock, 0, s>>>(g);
    return hipGetLastError();
}

hipError_t gen_post(const GenArgs& g, hipStream_t s) {
    if (g.K) {
        if (g.f32) k_gen_K<float><<<grid_of(g.T * g.m * g.n), kGenBlock, 0, s>>>(g);
        else k_gen_K<double><<<grid_of(g.T * g.m * g.n), kGenBlock, 0, s>>>(g);
    }
    if (g.d || g.u) {
        if (g.f32) k_gen_du<float><<<grid_of(g.T * g.m), kGenBlock, 0, s>>>(g);
        else k_gen_du<double><<<grid_of(g.T * g.m), kGenBlock, 0, s>>>(g);
    }
    return hipGetLastError();
}

}  // namespace lqt
