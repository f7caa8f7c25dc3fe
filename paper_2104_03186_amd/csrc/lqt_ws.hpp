// Per-instance workspace layout of the chunked pipelines (wavefront size
// classes 8/16/32 and the workgroup class 64), shared by host and device code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lqt_internal.hpp"

namespace lqt {

// Dense workgroup class: instances with max(n, m, p, pT) above 32 use
// zero-padded 64 x 64 state matrices and 32-wide control blocks.
constexpr int kBlockN = 64;
constexpr int kBlockM = 32;

__host__ __device__ inline int imax4(int a, int b, int c, int d) {
    const int x = a > b ? a : b, y = c > d ? c : d;
    return x > y ? x : y;
}

__host__ __device__ inline bool block_class(int n, int m, int p, int pT) { return imax4(n, m, p, pT) > 32; }

// Instance constants of the wavefront classes (unpadded, row-major).
struct CstW {
    int64_t G, J, W, ST, VT, end;
};

__host__ __device__ inline CstW cst_layout(int n, int m, int p) {
    CstW c;
    c.G = 0;
    c.J = c.G + (int64_t)n * m;
    c.W = c.J + (int64_t)n * n;
    c.ST = c.W + (int64_t)n * p;
    c.VT = c.ST + (int64_t)n * n;
    c.end = c.VT + n;
    return c;
}

// Instance constants of a workgroup engine with padded dimensions N (state)
// and M (control), zero-padded (row stride N for n-wide and M for m-wide
// matrices; U is the identity on its padding): F, L, G (G G^T = L U^{-1} L^T),
// U (symmetrised), J = H^T X H, W = H^T X (n x p), S_T, v_T.
template <int N, int M>
struct CstBT {
    static constexpr int64_t F = 0;
    static constexpr int64_t L = F + N * N;
    static constexpr int64_t G = L + N * M;
    static constexpr int64_t U = G + N * M;
    static constexpr int64_t J = U + M * M;
    static constexpr int64_t W = J + N * N;
    static constexpr int64_t ST = W + N * N;
    static constexpr int64_t VT = ST + N * N;
    static constexpr int64_t WT = VT + N;  // W transposed (coalesced reads of W r by lanes over W's rows)
    static constexpr int64_t end = WT + N * N;
};

// Engine of an instance: 0 = wavefront engine (records of dimension n), or
// a workgroup engine: 16, 32, 64 (padded state dimension N, control blocks
// M = min(N, 32)) or kEng32m16 (N = 32 with M = 16, for m <= 16).
constexpr int kEng32m16 = 33;

__host__ __device__ inline int eng_dim(int eng) { return eng == kEng32m16 ? 32 : eng; }

__host__ __device__ inline int64_t eng_cst_end(int eng) {
    switch (eng) {
        case 16: return CstBT<16, 16>::end;
        case 32: return CstBT<32, 32>::end;
        case kEng32m16: return CstBT<32, 16>::end;
        case 64: return CstBT<64, 32>::end;
    }
    return 0;
}

// Element, value and map records: dimension n (wavefront classes) or the
// padded 64 (workgroup class).
__host__ __device__ inline int64_t elem_doubles(int n) { return 3 * (int64_t)n * n + 2 * n; }
__host__ __device__ inline int64_t val_doubles(int n) { return (int64_t)n * n + n; }

// Record dimension and constants size of an instance on engine `eng`.
__host__ __device__ inline int ws_dim(int n, int eng) { return eng ? eng_dim(eng) : n; }
__host__ __device__ inline int64_t ws_cst_doubles(int n, int m, int p, int eng) {
    const int64_t e = eng ? eng_cst_end(eng) : cst_layout(n, m, p > 0 ? p : 1).end;
    return (e + 31) & ~int64_t(31);
}

// Operator form of the chunk fold (workgroup engines, instances without
// offsets c): every chunk after the first has the full length B and, the
// instance being time-invariant, the same matrix part (A, C, J); its vector
// part (b, eta) is linear in the chunk's references.  ops holds, for the
// relative steps j = 1 .. B-1 of the fold, the two d x d operators that carry
// eta_P into the new (eta, b); opr the 2d x (B p) matrix that maps the chunk's
// references (time order, p per step) to its (b, eta).
__host__ __device__ inline bool ws_op_form(int eng, bool has_c) { return eng != 0 && !has_c; }
__host__ __device__ inline int64_t ws_ops_doubles(int d, int64_t B) { return (B > 1 ? B - 1 : 0) * 2 * (int64_t)d * d; }
__host__ __device__ inline int64_t ws_opr_doubles(int d, int64_t B, int p) { return 2 * (int64_t)d * B * p; }
// Doubles of ops (and opr) of an instance: the workgroup engines' operator
// form, or the wavefront engine's (opf: ops only, the vector recursion runs
// per chunk with them).
__host__ __device__ inline int64_t ws_op_doubles(int eng, bool has_c, bool opf, int d, int64_t B, int p) {
    if (eng != 0) return ws_op_form(eng, has_c) ? ws_ops_doubles(d, B) + ws_opr_doubles(d, B, p) : 0;
    return opf ? ws_ops_doubles(d, B) : 0;
}

// Chunk scans of an instance as trees (either chunked engine; GInst::tree):
// the value at the chunk starts by recursive doubling over the chunk elements
// and the state at the chunk starts by recursive doubling over the chunk maps
// (about log2 NC levels, every chunk in parallel) instead of one walk over the
// chunks.  The levels alternate between two element buffers.  By default an
// instance takes the trees from kTreeMinNC chunks on.
constexpr int64_t kTreeMinNC = 128;

// cst | agg[NC] (chunk elements; in the operator form agg[0] holds the common
//     matrix part) | val[NC + 1] (value at chunk starts and T) | map[NC] (chunk
//     affine maps) | xs[NC] (state at chunk starts) | ops | opr (operator form)
//     | tree[2][NC] (chunk elements or chunk maps of the tree levels)
__host__ __device__ inline int64_t ws_doubles(int n, int m, int p, int eng, int64_t NC, int64_t B = 0,
                                              bool has_c = true, bool tree_scan = false, bool opf = false) {
    const int d = ws_dim(n, eng);
    const int64_t ops = ws_op_doubles(eng, has_c, opf, d, B, p);
    const int64_t tree = tree_scan ? 2 * NC * elem_doubles(d) : 0;
    return ws_cst_doubles(n, m, p, eng) + NC * elem_doubles(d) + (NC + 1) * val_doubles(d) + NC * val_doubles(d) +
           NC * d + ops + tree + 32;
}

struct InstWs {
    double *cst, *agg, *val, *map, *xs, *ops, *opr, *tree;
    int d;  // record dimension
};

__device__ inline InstWs inst_ws(const GInst& I) {
    InstWs w;
    const int d = ws_dim(I.n, I.eng);
    w.d = d;
    w.cst = I.ws;
    w.agg = w.cst + ws_cst_doubles(I.n, I.m, I.p, I.eng);
    w.val = w.agg + I.NC * elem_doubles(d);
    w.map = w.val + (I.NC + 1) * val_doubles(d);
    w.xs = w.map + I.NC * val_doubles(d);
    w.ops = w.xs + I.NC * d;
    w.opr = w.ops + ws_ops_doubles(d, I.B);
    w.tree = w.ops + ws_op_doubles(I.eng, I.c != nullptr, I.opf != 0, d, I.B, I.p);
    return w;
}

__device__ inline const double* step_ptr(const double* base, uint32_t ps, uint32_t bit, int64_t k, int64_t sz) {
    return (ps & bit) ? base + k * sz : base;
}

// Instance owning flat chunk index `chunk` (instances sorted by chunk0).
__device__ inline int find_instance(const GInst* inst, int ninst, int64_t chunk) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].chunk0 <= chunk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// First failure wins.
__device__ inline void raise_status(int32_t* st, int32_t code) {
    if (st) atomicCAS(st, 0, code);
}

}  // namespace lqt
