// Internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqt {

enum : uint32_t { kPS_F = 1, kPS_c = 2, kPS_L = 4, kPS_H = 8, kPS_X = 16, kPS_U = 32 };

// Kernel arguments of the lane-per-element pipeline for one instance.
// Wavefront units per block in the backward top levels of the lane pipeline.
constexpr int kSmallTopBlock = 256;

struct SmallArgs {
    // problem (device pointers)
    const double *F, *c, *L, *U, *H, *X, *r, *HT, *XT, *rT, *x0;
    int64_t T;
    int32_t n, m, p, pT;
    uint32_t per_step;
    // outputs (device pointers; S, v, x, u may be null); element type is
    // double, or float when f32 is set
    void *S, *v, *K, *d, *x, *u;
    int32_t* status;
    int32_t f32;
    // workspace
    double* cst;       // per-instance constants
    double* der;       // per-step derived data (time-varying problems)
    double* lane_el;   // [NC] in-wave suffix elements
    double* wave_val;  // [NG + 1] value function at wavefront-unit starts
    double* lane_aff;  // [NC] in-wave prefix affine maps
    double* wave_x;    // [NG] state at wavefront-unit starts
    double* mid_el;    // [NG] in-block suffixes of the unit totals (NG > kSmallTopBlock)
    double* blk_val;   // [NB + 1] value function at block starts (NG > kSmallTopBlock, many blocks)
    int64_t NC;        // number of chunks
    int32_t B;         // steps per chunk
    int32_t NG;        // number of wavefront units (64 chunks each)
    int32_t NB;        // blocks of kSmallTopBlock units
    int32_t want_fwd;  // run the forward pass
    int32_t traj;      // forward pass: 0 = scan of the closed-loop maps, 1 = forward prefixes
    double* m2_el;     // [NC] in-wave prefixes of the chunk elements (traj 1)
    double* m2_val;    // [NG] (C, b) of the forward prefix at wavefront-unit starts (traj 1)
    double* m2_mid;    // [NG] in-block prefixes of the unit totals (traj 1, NG > kSmallTopBlock)
    double* m2_blk;    // [NB] (C, b) at block starts (traj 1, NG > kSmallTopBlock)
};

// Optional per-kernel timing hook: begin/end are called on the host around
// every kernel launch of a solve (they record HIP events on the stream).
struct StageHook {
    void (*begin)(void* ctx, const char* name, hipStream_t s);
    void (*end)(void* ctx, hipStream_t s);
    void* ctx;
};

// One instance of the wavefront-per-chunk pipeline (device-resident array).
struct GInst {
    const double *F, *c, *L, *U, *H, *X, *r, *HT, *XT, *rT, *x0;
    void *S, *v, *K, *d, *x, *u;  // element type: double, or float for FP32 results
    int32_t* status;
    int64_t T;
    int32_t n, m, p, pT;
    uint32_t per_step;
    int32_t B;        // steps per chunk
    int64_t NC;       // chunks
    int64_t chunk0;   // flat index of the first chunk over the launch
    double* ws;       // instance workspace (ws_doubles)
    int32_t eng;      // 0: wavefront engine; else padded dimension of the workgroup engine
    int32_t traj;     // 1: trajectory by forward prefixes (Method 2) into m2x, m2u (x, u are then null)
    void *m2x, *m2u;  // Method 2 states and controls (double)
    int32_t tree;     // 1: chunk scans as trees (NC >= 2; workspace sized with the tree buffers)
    int32_t opf;      // 1: wavefront-engine fold in operator form (class 8, time-invariant, no c, maps)
};

size_t wave_lds_bytes(int nmax);

// Size-class variant of the wavefront pipeline: matrices zero-padded to N x N
// with N = tile_class(max(n, m, p)) in {8, 16, 32} (0: no class).
int tile_class(int need);
// tree_nc: the most chunks of an instance of the launch with tree set (0: none).
// opf_any: some instance of the launch has opf set.
hipError_t tile_solve(int N, const GInst* d_inst, int ninst, int64_t nchunks, int64_t tree_nc, bool want_fwd, bool f32,
                      hipStream_t s, const StageHook* h, bool opf_any = false);
// Workgroup engines (N = 16, 32, 64; time-invariant except c; class 64:
// n, p, pT <= 64 and m <= 32).
hipError_t block_solve(int N, const GInst* d_inst, int ninst, int64_t nchunks, int64_t max_nc, int64_t tree_nc,
                       bool want_fwd, bool f32, hipStream_t s, const StageHook* h);
// Trajectory by forward prefixes (Method 2) for the instances of a launch
// group with traj set, after the group's backward pass (double S, v, K, d;
// writes m2x, m2u); N = the group's size class (8, 16, 32, 64).
hipError_t m2_chunked(int N, const GInst* d_inst, int ninst, int64_t nchunks, hipStream_t s, const StageHook* h);

// Batched lane kernel (n <= 4, time-invariant except c): one workgroup of
// 256 lanes per instance, chunks of lane_batch_chunk(T) steps.  mode: the
// step-data mode of an instance, or -1 when the kernel does not take it.
int lane_batch_mode(int n, int p, uint32_t per_step, bool has_c);
int lane_batch_chunk(int64_t T);
// Instances of one (n, m, mode) group; d_tab: device table of their
// arguments (cst, K, d workspace filled in; NC, B from lane_batch_chunk).
hipError_t lane_batch_solve(int n, int m, int mode, bool f32, const SmallArgs* d_tab, int ninst, hipStream_t s,
                            const StageHook* h);

bool small_supported(int n, int m);
size_t small_cst_doubles(int n, int m, int p);
size_t small_der_doubles(int n, int m);
size_t small_elem_doubles(int n);
size_t small_aff_doubles(int n);
size_t small_val_doubles(int n);
// A second stream and two events owned by the plan: the forward element scan
// of the prefix trajectory runs on `side`, concurrently with the backward
// pass on the solve's stream (fork after the constants, join before the
// forward walk).
struct SideStream {
    hipStream_t side;
    hipEvent_t fork, join;
};
hipError_t small_solve(const SmallArgs& a, hipStream_t s, const StageHook* hook, const SideStream* side = nullptr);

// Generalised stage cost (Section IV-D): one instance's transform to the
// standard form and the map of its gains and controls back.  Inputs are the
// instance's device arrays (L, H, X, U, M time-invariant; F and c as in the
// problem); Z .. ct are workspace (gen_layout); K, d, u, x are the solve's
// outputs (double, or float when f32 is set; any of K, d, u may be null).
struct GenArgs {
    const double *F, *c, *L, *H, *X, *U, *M, *r, *s;
    int64_t T;
    int32_t n, m, p;
    uint32_t per_step;
    double *Z, *ZH, *LZ, *Xt, *Ft, *ct;
    void *K, *d, *u;
    const void* x;
    int32_t f32;
};
size_t gen_ws_doubles(int n, int m, int p, int64_t T, bool f_per_step);
void gen_layout(GenArgs& g, double* ws);
hipError_t gen_transform(const GenArgs& g, hipStream_t s);
hipError_t gen_post(const GenArgs& g, hipStream_t s);

// Iterated linearisation (the nonlinear extension of Section IV-D), unicycle model: one round's
// expansion of the dynamics about the nominal (x, u, double) into per-step
// F, L, c, plus a copy of the nominal controls for the change measure.
struct NlArgs {
    const double* dt;
    int64_t T;
    const double *x, *u;       // nominal trajectory [T+1][4], [T][2]
    double *F, *L, *c, *ubar;  // [T][4][4], [T][4][2], [T][4], [T][2]
};
hipError_t nl_start(double* change, int iterations, int32_t* round_status, hipStream_t s);
// prev_change (nullable): the previous round's change word, completed here.
hipError_t nl_linearise(const NlArgs& g, double* prev_change, hipStream_t s);
hipError_t nl_change(const NlArgs& g, double* out, hipStream_t s);
hipError_t nl_finish(const int32_t* round_status, int iterations, int32_t* status, hipStream_t s);
// dst[i] = src[i] for i < count, each side float (f32 set) or double.
hipError_t convert_array(const void* src, bool src_f32, void* dst, bool dst_f32, int64_t count, hipStream_t s);

// Finite state and control spaces (Section III-D).  The horizon is cut into
// NC <= kFsMaxNC chunks of B steps, the chunks into groups of kFsGroup.
constexpr int kFsMaxNC = 2048;
constexpr int kFsGroup = 32;
struct FsArgs {
    const int32_t* next;   // [D][Du] or [T][D][Du]
    const double* cost;    // [D][Du] or [T][D][Du]
    const double* cost_T;  // [D]
    int64_t T;
    int32_t D, Du;
    uint32_t per_step;     // bit 0: next per step; bit 1: cost per step
    int32_t x0;
    int32_t B, NC, NG;
    // outputs (V, x, ux, status may be null; ulaw is the caller's u or workspace)
    double* V;
    int32_t *ulaw, *x, *ux, *status;
    // workspace
    double *P, *Q, *gval, *cval;  // [NC][D][D], [NG][D][D], [NG + 1][D], [NC + 1][D]
    int32_t *nxt, *phi, *xs;      // [T][D], [NC][D], [NC + 1]
    int32_t *gphi, *gxs;          // [NG][D] group maps, [NG + 1] states at group starts
};
void fs_shape(int64_t T, int32_t& B, int32_t& NC, int32_t& NG);
hipError_t fs_solve(const FsArgs& a, hipStream_t s, const StageHook* h);

}  // namespace lqt
