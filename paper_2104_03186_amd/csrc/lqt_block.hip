// Workgroup-per-chunk LQT pipeline (gfx950) for time-invariant instances of
// the classes 16 and 32 (class 32 in two variants: 32- or 16-wide control
// blocks) and for the dense class 32 < max(n, m, p, pT) <= 64, m <= 32.
//
// One workgroup owns one chunk of B consecutive steps (class 64: four
// wavefronts, 64 x 64 zero-padded state, about 155 KB of the 160 KB of LDS;
// class 32: two wavefronts, 32 x 32; class 16: one wavefront, 16 x 16).  The
// chunk's state matrices and every temporary live in the workgroup's LDS; the
// products run on the matrix cores (16x16x4 FP64 MFMA, 16 x 16 output tiles
// spread over the wavefronts).
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
// b_fold (chunk elements), b_chain (value at chunk starts, per instance; for
// instances with tree set b_tlevel + b_tanchor, the scan over the chunk
// elements as a tree), b_final (values, gains, chunk maps), b_fchain (state
// at chunk starts; b_ftlevel, a tree over the chunk maps, for instances with
// tree set), b_roll (trajectory).
#include <hip/hip_runtime.h>

#include "lqt_internal.hpp"
#include "lqt_ws.hpp"

namespace lqt {

#define BDI __device__ __forceinline__
typedef double dvec4 __attribute__((ext_vector_type(4)));

namespace blk64 {
constexpr int N = 64, M = 32, NW = 4;
using CB = CstBT<N, M>;
constexpr const char* kNames[11] = {"t64_prep", "t64_fold", "t64_chain", "t64_final", "t64_fchain", "t64_roll",
                                    "t64_fmat", "t64_fvec", "t64_tree", "t64_tanchor", "t64_ftree"};
#include "lqt_block.inc"
}  // namespace blk64

namespace blk32 {
constexpr int N = 32, M = 32, NW = 2;
using CB = CstBT<N, M>;
constexpr const char* kNames[11] = {"b32_prep", "b32_fold", "b32_chain", "b32_final", "b32_fchain", "b32_roll",
                                    "b32_fmat", "b32_fvec", "b32_tree", "b32_tanchor", "b32_ftree"};
#include "lqt_block.inc"
}  // namespace blk32

namespace blk32h {
constexpr int N = 32, M = 16, NW = 2;
using CB = CstBT<N, M>;
constexpr const char* kNames[11] = {"b32h_prep", "b32h_fold", "b32h_chain", "b32h_final", "b32h_fchain", "b32h_roll",
                                   "b32h_fmat", "b32h_fvec", "b32h_tree", "b32h_tanchor", "b32h_ftree"};
#include "lqt_block.inc"
}  // namespace blk32h

namespace blk16 {
constexpr int N = 16, M = 16, NW = 1;
using CB = CstBT<N, M>;
constexpr const char* kNames[11] = {"b16_prep", "b16_fold", "b16_chain", "b16_final", "b16_fchain", "b16_roll",
                                    "b16_fmat", "b16_fvec", "b16_tree", "b16_tanchor", "b16_ftree"};
#include "lqt_block.inc"
}  // namespace blk16

hipError_t block_solve(int N, const GInst* d_inst, int ninst, int64_t nchunks, int64_t max_nc, int64_t tree_nc,
                       bool want_fwd, bool f32, hipStream_t s, const StageHook* h) {
    switch (N) {
        case 64:
            if (f32) blk64::run_block<float>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            else blk64::run_block<double>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            break;
        case 32:
            if (f32) blk32::run_block<float>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            else blk32::run_block<double>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            break;
        case kEng32m16:
            if (f32) blk32h::run_block<float>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            else blk32h::run_block<double>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            break;
        case 16:
            if (f32) blk16::run_block<float>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            else blk16::run_block<double>(d_inst, ninst, nchunks, max_nc, tree_nc, want_fwd, s, h);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lqt
