// Host runtime of the LQT solver: plans, validation, workspace, launches,
// status and the continuous-batching serving interface (submit/poll).
// Implements include/lqt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lqt.h"
#include "lqt_internal.hpp"
#include "lqt_serve.hpp"
#include "lqt_ws.hpp"

namespace {

constexpr int kMaxNx = 64;         // largest state dimension of the kernels
constexpr int kWaveMaxN = 64;      // chunked paths: n, p, pT up to this (m up to 32 above 32)
constexpr int64_t kSmallMinT = 8192;  // lane-per-element path for long n <= 4 instances

// Serving defaults: device pool for in-flight requests (when the plan sets no
// budget), concurrent batches (one stream each), requests per batch, queue.
constexpr size_t kDefaultServePool = size_t(8) << 30;
constexpr int kServeSlots = 4;
constexpr int kServeBatchMax = 512;
constexpr int kDefaultQueue = 4096;

// Path of an instance: a function of the instance and the plan (routing
// overrides, trajectory method), never of the batch, so a result is the same
// alone and in any mix.  n <= 4 instances of horizon up to kBatchMaxT that
// are time-invariant except c take the batched lane kernel (one workgroup
// per instance) unless the plan recovers the trajectory by forward prefixes;
// longer n <= 4 instances the lane pipeline; the rest the chunked engines.
// Routing override 1 takes the lane pipeline wherever it applies, 2 the
// chunked engines, 3 the batched lane kernel wherever it applies.
enum class Path { Small, Wave, Batch };
constexpr int64_t kBatchMaxT = 16384;

Path path_of(const lqt_routing& R, bool prefix, const lqt_problem& p) {
    const bool small_ok = lqt::small_supported(p.nx, p.nu);
    const bool batch_ok = small_ok && lqt::lane_batch_mode(p.nx, p.ny, p.per_step, p.c != nullptr) >= 0;
    if (R.path == 1 && small_ok) return Path::Small;
    if (R.path == 2) return Path::Wave;
    if (R.path == 3 && batch_ok) return Path::Batch;
    if (batch_ok && p.T <= kBatchMaxT && !prefix) return Path::Batch;
    return (small_ok && p.T >= kSmallMinT) ? Path::Small : Path::Wave;
}

// Engine of a chunked-path instance: the workgroup engine (padded dimension
// 16, 32 or 64) for time-invariant instances (only c and r may vary per step)
// of the classes 16 and 32 and for every class-64 instance, else the
// wavefront engine (0).  Routing override block = 1 keeps the classes 16 and
// 32 on the wavefront engine.
int tile_class_of(const lqt_problem& p) {
    return lqt::tile_class(std::max(std::max(p.nx, p.nu), std::max(p.ny, p.nyT)));
}

int eng_of(const lqt_routing& R, const lqt_problem& p) {
    const int cls = tile_class_of(p);
    if (cls == 64) return 64;
    if (R.block != 1 && (cls == 16 || cls == 32) && !(p.per_step & ~(uint32_t)LQT_PS_c))
        return (cls == 32 && p.nu <= 16) ? lqt::kEng32m16 : cls;
    return 0;
}

// Chunk length of a chunked-path instance.  Default: about 64 chunks per
// instance, between 16 and 256 steps; an instance longer than kTreeT takes
// 64-step chunks instead (at least 257 of them, scanned as a tree, so that
// the per-chunk fold and down-sweep stay short).  A plan tuned by lqt_tune uses about `div` chunks per instance for
// the launch group, at least 16 steps each (div = 1: one chunk, no element
// fold at all -- the instance is then solved by the sequential down-sweep
// alone, which pays when a batch has enough instances to fill the GPU).  The
// routing override wave_chunk fixes the length.  Plans that recover the
// trajectory by forward prefixes keep the longer chunks: their forward walk
// over the chunk elements is sequential in the number of chunks.
constexpr int kTuneDivs[] = {1, 4, 16, 64, 256};
constexpr int64_t kTreeT = 16384;

int wave_chunk(const lqt_routing& R, int64_t T, int div = 0, bool prefix = false) {
    if (R.wave_chunk >= 1 && R.wave_chunk <= 4096) return R.wave_chunk;
    if (div <= 0) {
        if (T > kTreeT && !prefix) return 64;
        const int64_t b = (T + 63) / 64;
        return (int)std::max<int64_t>(16, std::min<int64_t>(256, b));
    }
    const int64_t b = (T + div - 1) / div;
    return (int)std::max<int64_t>(16, std::min<int64_t>(int64_t(1) << 30, b));
}

// Chunk scans of a chunked-path instance with NC chunks as trees (GInst::tree):
// the routing override tree (1: from two chunks on, 2: never), else from
// kTreeMinNC chunks on.
bool tree_for(const lqt_routing& R, int64_t NC) {
    if (NC < 2 || R.tree == 2) return false;
    return R.tree == 1 || NC >= lqt::kTreeMinNC;
}

// Chunk length of an instance whose chunks are scanned as trees on request
// (routing tree = 1, for latency): about as many chunks as the size class's
// tree kernels keep resident on the GPU at once, 8 to 64 steps each.  Short
// chunks shorten the sequential fold and down-sweep inside every chunk; the
// trees add only about log2 of the chunk count in dependent steps.
int tree_chunk(int64_t T, int cls) {
    const int64_t width = cls <= 8 ? 4096 : (cls <= 16 ? 2048 : (cls <= 32 ? 1024 : 256));
    return (int)std::max<int64_t>(8, std::min<int64_t>(64, (T + width - 1) / width));
}

// Launch group of a chunked-path instance: size class (8, 16, 32, 64) and
// engine (wavefront / workgroup), as an index 0..7.
int group_key(const lqt_routing& R, const lqt_problem& p) {
    const int cls = tile_class_of(p);
    const int ci = cls <= 8 ? 0 : (cls <= 16 ? 1 : (cls <= 32 ? 2 : 3));
    return 2 * ci + (eng_of(R, p) ? 1 : 0);
}

thread_local std::string g_create_error;

}  // namespace

struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    bool on = false;
    std::string only;  // record only this stage ("" = every stage)
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    hipEvent_t cur_a = nullptr;
    const char* cur_name = nullptr;
    std::vector<std::string> names;  // first-launch order
    std::unordered_map<std::string, std::pair<int64_t, double>> acc;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    static void begin(void* ctx, const char* name, hipStream_t s) {
        Profiler* p = (Profiler*)ctx;
        p->cur_name = nullptr;
        if (!p->only.empty() && p->only != name) return;
        p->cur_a = p->get();
        p->cur_name = name;
        (void)hipEventRecord(p->cur_a, s);
    }
    static void end(void* ctx, hipStream_t s) {
        Profiler* p = (Profiler*)ctx;
        if (!p->cur_name) return;
        hipEvent_t b = p->get();
        (void)hipEventRecord(b, s);
        p->pending.push_back({p->cur_name, p->cur_a, b});
    }
};

// Device workspace of one stream of launches, plus the pinned host copy of
// the wavefront-path instance table and the event of its last upload (the
// host table is rewritten only after that copy has finished).
struct Arena {
    char* ws = nullptr;
    size_t cap = 0;
    bool owned = true;  // false: ws points into the serving pool
    lqt::GInst* ginst_host = nullptr;
    size_t ginst_cap = 0;
    lqt::SmallArgs* sargs_host = nullptr;  // batched-lane instance table (pinned)
    size_t sargs_cap = 0;
    hipEvent_t ginst_done = nullptr;       // both tables uploaded
    bool capture = false;  // work is being recorded into a graph: no host waits on events, none recorded
};

// A recorded launch sequence of the plan (lqt_set_graphs): the graph and the
// arenas it runs in, which no other work of the plan uses.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    Arena main, nl;
};

// Device side of one serving slot: its stream, its batch's arena (a range of
// the serving pool), status words and completion event.
struct Slot {
    hipStream_t stream = nullptr;
    Arena arena;
    int32_t* status_dev = nullptr;   // [kServeBatchMax] per-request status words
    int32_t* status_host = nullptr;  // pinned copy, valid once `done` has fired
    hipEvent_t done = nullptr;
};

struct PendingReq {
    lqt_problem p;
    lqt_outputs o;
};

// The device operations of the serving core (lqt_serve.hpp).
struct ServeOps {
    lqt_plan_t plan = nullptr;
    struct Acc;
    Acc acc();
    int launch(int slot, const size_t* req, size_t count, size_t off, size_t len);
    int query(int slot);
    int status(int slot, size_t i);
    void drain(int slot);
};

struct lqt_plan_s {
    lqt_plan_desc desc{};
    Profiler prof;
    Arena main;
    std::string err;
    std::recursive_mutex mu;
    // serving state: device pool and slots, the host admission core, the
    // payloads of queued requests (by ticket), and the progress thread
    char* pool = nullptr;
    std::vector<Slot> slots;
    lqt::ServeCore<ServeOps> core;
    ServeOps ops;
    std::unordered_map<uint64_t, PendingReq> payload;
    uint64_t next_ticket = 1;
    std::thread progress;
    std::condition_variable_any wake;
    bool stop = false;
    // graph replay (lqt_set_graphs): recorded launch sequences by call signature
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    std::map<std::string, GraphEntry*> gcache;
    int tune_div[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // chunks per instance per launch group (0: default)
    lqt_routing route{};                          // routing and chunking overrides (lqt_set_routing)
    lqt::SideStream side{};  // prefix trajectory: element scan beside the backward pass
    bool has_side = false;
    Arena nl;                // iterated linearisation: linearised model, nominal controls, round status
    Arena fs;                // finite-state solves: chunk and group products, values, closed-loop maps
};

namespace {

lqt_status fail(lqt_plan_t p, lqt_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

Path path_of(lqt_plan_t plan, const lqt_problem& p) {
    return path_of(plan->route, plan->desc.trajectory == LQT_TRAJ_PREFIX, p);
}

lqt_status fail(lqt_plan_t p, lqt_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (p) p->err = buf;
    else g_create_error = buf;
    return code;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int chunk_length(const lqt_routing& R, int64_t T) {
    if (R.lane_chunk >= 1 && R.lane_chunk <= 1024) return R.lane_chunk;
    // About 64K lanes (one wavefront per SIMD on 256 CUs), at most 16 steps
    // per lane; measured best for the n = 4 pipeline at T = 1e6.
    int64_t b = (T + 65535) / 65536;
    return (int)std::max<int64_t>(1, std::min<int64_t>(16, b));
}

struct Layout {
    size_t cst, der, lane_el, wave_val, lane_aff, wave_x, mid_el, blk_val, K, d, m2_el, m2_val, m2_mid, m2_blk, S, v,
        x, u, total;
    int64_t NC;
    int B, NG, NB;
};

// m2: forward pass by prefixes (Method 2), which reads S and v (scratch when
// the caller does not take them).  wide: Method 2 with float results -- the
// solve runs with double results in scratch (S, v, K, d, x, u) and they are
// rounded to the caller's float arrays afterwards, since the states of
// Method 2 are solved from S_k and v_k (I + C S_k is ill-conditioned enough
// that float-rounded S_k, v_k would cost the 1e-5 accuracy of the controls).
Layout layout_for(const lqt_routing& R, const lqt_problem& p, bool need_K, bool need_d, bool m2 = false,
                  bool need_S = false, bool need_v = false, bool wide = false) {
    using namespace lqt;
    Layout L{};
    if (wide) need_K = need_d = need_S = need_v = true;
    const int n = p.nx, m = p.nu;
    L.B = chunk_length(R, p.T);
    L.NC = (p.T + L.B - 1) / L.B;
    L.NG = (int)((L.NC + 63) / 64);
    L.NB = (L.NG + lqt::kSmallTopBlock - 1) / lqt::kSmallTopBlock;
    const bool blocks = L.NG > lqt::kSmallTopBlock;
    const bool var = p.per_step != 0;
    size_t off = 0;
    auto take = [&](size_t doubles) {
        size_t o = off;
        off = align_up(off + doubles * sizeof(double));
        return o;
    };
    L.cst = take(small_cst_doubles(n, m, std::max(p.ny, 1)));
    L.der = take(var ? (size_t)p.T * small_der_doubles(n, m) : 0);
    L.lane_el = take((size_t)L.NC * small_elem_doubles(n));
    L.wave_val = take((size_t)(L.NG + 1) * small_val_doubles(n));
    L.lane_aff = take((size_t)L.NC * small_aff_doubles(n));
    L.wave_x = take((size_t)L.NG * n);
    L.mid_el = take(blocks ? (size_t)L.NG * small_elem_doubles(n) : 0);
    L.blk_val = take(blocks ? (size_t)(L.NB + 1) * small_val_doubles(n) : 0);
    L.K = take(need_K ? (size_t)p.T * m * n : 0);
    L.d = take(need_d ? (size_t)p.T * m : 0);
    L.m2_el = take(m2 ? (size_t)L.NC * small_elem_doubles(n) : 0);
    L.m2_val = take(m2 ? (size_t)L.NG * small_val_doubles(n) : 0);
    L.m2_mid = take(m2 && blocks ? (size_t)L.NG * small_elem_doubles(n) : 0);
    L.m2_blk = take(m2 && blocks ? (size_t)L.NB * small_val_doubles(n) : 0);
    L.S = take(m2 && need_S ? (size_t)(p.T + 1) * n * n : 0);
    L.v = take(m2 && need_v ? (size_t)(p.T + 1) * n : 0);
    L.x = take(m2 && wide ? (size_t)(p.T + 1) * n : 0);
    L.u = take(m2 && wide ? (size_t)p.T * m : 0);
    L.total = off;
    return L;
}

// Wavefront-engine fold in operator form (GInst::opf): class 8 on the
// wavefront engine, time-invariant (only r per step), no offsets c,
// trajectory by maps, at least two chunks of at least two steps.
bool opf_for(lqt_plan_t plan, const lqt_problem& p, int64_t B, int64_t NC) {
    return eng_of(plan->route, p) == 0 && tile_class_of(p) == 8 && p.c == nullptr &&
           (p.per_step & (LQT_PS_F | LQT_PS_L | LQT_PS_U | LQT_PS_H | LQT_PS_X)) == 0 &&
           plan->desc.trajectory != LQT_TRAJ_PREFIX && NC >= 2 && B >= 2;
}

int chunk_for(lqt_plan_t plan, const lqt_problem& p) {
    const int div = plan->tune_div[group_key(plan->route, p)];
    const bool prefix = plan->desc.trajectory == LQT_TRAJ_PREFIX;
    if (plan->route.tree == 1 && plan->route.wave_chunk == 0 && div <= 0 && !prefix)
        return tree_chunk(p.T, tile_class_of(p));
    return wave_chunk(plan->route, p.T, div, prefix);
}

// Workspace of one wavefront-path instance, and of its K, d scratch when the
// caller does not take K and d.
size_t wave_bytes(lqt_plan_t plan, const lqt_problem& p) {
    const int B = chunk_for(plan, p);
    const int64_t NC = (p.T + B - 1) / B;
    const int64_t wd = lqt::ws_doubles(p.nx, p.nu, p.ny, eng_of(plan->route, p), NC, B, p.c != nullptr,
                                       tree_for(plan->route, NC), opf_for(plan, p, B, NC));
    return align_up((size_t)wd * sizeof(double));
}
// Scratch of one chunked-path instance beside its engine workspace: the
// double gains when the caller does not take K and d, and for the forward-
// prefix trajectory (Method 2) the double S, v it reads.  A plan with float
// results and forward prefixes solves its chunked instances with double
// results ("wide"): every requested family goes to double scratch first and
// is rounded into the caller's arrays afterwards.
struct WaveScratch {
    bool m2 = false, wide = false;
    size_t kd = 0, S = 0, v = 0, x = 0, u = 0;
    size_t total() const { return kd + S + v + x + u; }
};

WaveScratch wave_scratch(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o, bool f32) {
    WaveScratch w;
    const bool prefix = plan->desc.trajectory == LQT_TRAJ_PREFIX;
    w.m2 = prefix && (o.x || o.u);
    w.wide = prefix && f32;
    const size_t T = (size_t)p.T, n = (size_t)p.nx, m = (size_t)p.nu;
    if (!o.K || !o.d || w.wide) w.kd = align_up(T * (m * n + m) * sizeof(double));
    if ((w.m2 && !o.S) || (w.wide && o.S) || (w.m2 && w.wide)) w.S = align_up((T + 1) * n * n * sizeof(double));
    if ((w.m2 && !o.v) || (w.wide && o.v) || (w.m2 && w.wide)) w.v = align_up((T + 1) * n * sizeof(double));
    if (w.m2 && w.wide && o.x) w.x = align_up((T + 1) * n * sizeof(double));
    if (w.m2 && w.wide && o.u) w.u = align_up(T * m * sizeof(double));
    return w;
}

// Generalised stage cost (Section IV-D): an instance with M or s is solved as
// its standard-form transform, whose c~ varies per step.
bool is_gen(const lqt_problem& p) { return p.M || p.s; }

// Shape of the standard-form instance a generalised one is solved as (the
// sizes depend on the presence of c, not on its values).
lqt_problem std_shape(const lqt_problem& p) {
    if (!is_gen(p)) return p;
    lqt_problem q = p;
    q.per_step |= LQT_PS_c;
    if (!q.c) q.c = p.r;
    q.M = nullptr;
    q.s = nullptr;
    return q;
}

// Transform workspace of a generalised instance, and the state scratch of
// the control map when the caller takes u without x.
size_t gen_bytes(const lqt_problem& p, const lqt_outputs& o) {
    if (!is_gen(p)) return 0;
    size_t b = align_up(lqt::gen_ws_doubles(p.nx, p.nu, p.ny, p.T, p.per_step & LQT_PS_F) * sizeof(double));
    if (o.u && !o.x) b += align_up((size_t)(p.T + 1) * p.nx * sizeof(double));
    return b;
}

// Workspace of one batched-lane instance: its constants, and the double gains
// when the caller does not take K and d (the kernel always writes them).
size_t batch_bytes(const lqt_problem& p, const lqt_outputs& o) {
    size_t b = align_up(lqt::small_cst_doubles(p.nx, p.nu, std::max(p.ny, 1)) * sizeof(double));
    if (!o.K || !o.d) b += align_up((size_t)p.T * (p.nu * p.nx + p.nu) * sizeof(double));
    return b;
}

// Device bytes of one launch group: the transform regions of generalised
// instances, then the small-path instances, which run one after another in
// one region (the largest), each wavefront-path instance's own region, then
// the instance table, then the batched-lane instances and their table.
struct BatchSize {
    lqt_plan_t plan = nullptr;
    size_t gen = 0, small = 0, wave = 0, batch = 0;
    size_t nwave = 0, nbatch = 0;
    bool f32 = false;  // float results
    BatchSize(lqt_plan_t pl, bool f) : plan(pl), f32(f) {}
    explicit BatchSize(lqt_plan_t pl) : plan(pl), f32(pl->desc.prec == LQT_PREC_MIXED) {}
    void add(const lqt_problem& p0, const lqt_outputs& o) {
        gen += gen_bytes(p0, o);
        const lqt_problem p = std_shape(p0);
        const Path path = path_of(plan, p);
        if (path == Path::Small) {
            const bool m2 = plan->desc.trajectory == LQT_TRAJ_PREFIX && (o.x || o.u);
            small = std::max(small,
                             align_up(layout_for(plan->route, p, !o.K, !o.d, m2, !o.S, !o.v, m2 && f32).total));
        } else if (path == Path::Batch) {
            batch += batch_bytes(p, o);
            ++nbatch;
        } else {
            wave += wave_bytes(plan, p) + wave_scratch(plan, p0, o, f32).total();
            ++nwave;
        }
    }
    size_t wave_end() const { return gen + small + (nwave ? wave + align_up(nwave * sizeof(lqt::GInst)) : 0); }
    size_t total() const { return wave_end() + (nbatch ? batch + align_up(nbatch * sizeof(lqt::SmallArgs)) : 0); }
};

lqt_status validate(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o, int idx) {
    if (p.nx < 1 || p.nu < 1 || p.ny < 1 || p.nyT < 1)
        return fail(plan, LQT_EINVAL, "instance %d: dimensions must be >= 1 (nx=%d nu=%d ny=%d nyT=%d)", idx,
                    p.nx, p.nu, p.ny, p.nyT);
    if (p.T < 1) return fail(plan, LQT_EINVAL, "instance %d: T must be >= 1 (got %lld)", idx, (long long)p.T);
    if (p.nx > plan->desc.max_nx || p.nu > plan->desc.max_nu)
        return fail(plan, LQT_EINVAL, "instance %d: nx=%d nu=%d exceed the plan's max_nx=%d max_nu=%d", idx, p.nx,
                    p.nu, plan->desc.max_nx, plan->desc.max_nu);
    if (path_of(plan, p) == Path::Wave) {
        if (std::max(std::max(p.nx, p.nu), std::max(p.ny, p.nyT)) > kWaveMaxN)
            return fail(plan, LQT_ENOTSUP, "instance %d: dimensions nx=%d nu=%d ny=%d nyT=%d exceed %d", idx, p.nx,
                        p.nu, p.ny, p.nyT, kWaveMaxN);
        if (lqt::block_class(p.nx, p.nu, p.ny, p.nyT)) {
            if (p.nu > lqt::kBlockM)
                return fail(plan, LQT_ENOTSUP, "instance %d: nu=%d above %d needs all dimensions <= 32", idx, p.nu,
                            lqt::kBlockM);
            if (p.per_step & ~(uint32_t)LQT_PS_c)
                return fail(plan, LQT_ENOTSUP,
                            "instance %d: above 32 states only c may vary per step (per_step=0x%x)", idx,
                            p.per_step);
        }
    }
    if (p.per_step & ~63u) return fail(plan, LQT_EINVAL, "instance %d: unknown per_step bits 0x%x", idx, p.per_step);
    if (is_gen(p) && (p.per_step & (LQT_PS_L | LQT_PS_H | LQT_PS_X | LQT_PS_U)))
        return fail(plan, LQT_ENOTSUP,
                    "instance %d: with M or s (generalised cost) only F and c may vary per step (per_step=0x%x)", idx,
                    p.per_step);
    if (!p.F || !p.L || !p.H || !p.X || !p.U || !p.r || !p.HT || !p.XT || !p.rT || !p.x0)
        return fail(plan, LQT_EINVAL, "instance %d: a required input pointer is NULL", idx);
    if ((p.per_step & LQT_PS_c) && !p.c)
        return fail(plan, LQT_EINVAL, "instance %d: per_step has LQT_PS_c but c is NULL", idx);
    const void* aligned[] = {p.r, o.S, o.v, o.K, o.d, o.x, o.u};
    for (const void* q : aligned)
        if (q && ((uintptr_t)q & 15u))
            return fail(plan, LQT_EINVAL, "instance %d: r and output arrays must be 16-byte aligned", idx);
    const bool fwd = o.x || o.u;
    if (fwd && (!o.K) != (!o.d))
        return fail(plan, LQT_EINVAL, "instance %d: K and d must both be given or both be NULL", idx);
    return LQT_OK;
}

// Grow an owned arena to `bytes` (synchronous: the old buffer may be in use).
lqt_status ensure_ws(lqt_plan_t plan, Arena& A, size_t bytes) {
    if (bytes <= A.cap) return LQT_OK;
    if (!A.owned) return fail(plan, LQT_ENOMEM, "batch needs %zu bytes, its pool range holds %zu", bytes, A.cap);
    if (plan->desc.hbm_budget_bytes && bytes > plan->desc.hbm_budget_bytes)
        return fail(plan, LQT_ENOMEM, "workspace of %zu bytes exceeds the plan budget of %zu bytes", bytes,
                    plan->desc.hbm_budget_bytes);
    if (A.ws) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(A.ws) != hipSuccess)
            return fail(plan, LQT_EHIP, "hipFree of the old workspace failed");
        A.ws = nullptr;
        A.cap = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(plan, LQT_ENOMEM, "hipMalloc of %zu workspace bytes failed", bytes);
    }
    A.ws = (char*)p;
    A.cap = bytes;
    return LQT_OK;
}

lqt_status launch_one(lqt_plan_t plan, char* base, const lqt_problem& p, const lqt_outputs& o, hipStream_t s,
                      int32_t* status_override, bool f32, bool hooks = true) {
    const bool fwd = o.x || o.u;
    const bool need_K = !o.K, need_d = !o.d;
    const bool m2 = plan->desc.trajectory == LQT_TRAJ_PREFIX && fwd;
    const bool wide = m2 && f32;
    Layout L = layout_for(plan->route, p, need_K, need_d, m2, !o.S, !o.v, wide);
    lqt::SmallArgs a{};
    a.F = p.F; a.c = p.c; a.L = p.L; a.U = p.U; a.H = p.H; a.X = p.X; a.r = p.r;
    a.HT = p.HT; a.XT = p.XT; a.rT = p.rT; a.x0 = p.x0;
    a.T = p.T; a.n = p.nx; a.m = p.nu; a.p = p.ny; a.pT = p.nyT;
    a.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
    a.S = (o.S && !wide) ? o.S : (m2 ? (void*)(base + L.S) : nullptr);
    a.v = (o.v && !wide) ? o.v : (m2 ? (void*)(base + L.v) : nullptr);
    a.K = (o.K && !wide) ? o.K : (void*)(base + L.K);
    a.d = (o.d && !wide) ? o.d : (void*)(base + L.d);
    a.x = wide ? (o.x ? (void*)(base + L.x) : nullptr) : o.x;
    a.u = wide ? (o.u ? (void*)(base + L.u) : nullptr) : o.u;
    a.f32 = (f32 && !wide) ? 1 : 0;
    a.status = status_override ? status_override : o.status;
    a.cst = (double*)(base + L.cst);
    a.der = (double*)(base + L.der);
    a.lane_el = (double*)(base + L.lane_el);
    a.wave_val = (double*)(base + L.wave_val);
    a.lane_aff = (double*)(base + L.lane_aff);
    a.wave_x = (double*)(base + L.wave_x);
    a.mid_el = (double*)(base + L.mid_el);
    a.blk_val = (double*)(base + L.blk_val);
    a.NC = L.NC; a.B = L.B; a.NG = L.NG; a.NB = L.NB;
    a.want_fwd = fwd ? 1 : 0;
    a.traj = m2 ? 1 : 0;
    a.m2_el = (double*)(base + L.m2_el);
    a.m2_val = (double*)(base + L.m2_val);
    a.m2_mid = (double*)(base + L.m2_mid);
    a.m2_blk = (double*)(base + L.m2_blk);
    const bool prof = hooks && plan->prof.on;
    lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
    hipError_t e = lqt::small_solve(a, s, prof ? &hook : nullptr, plan->has_side ? &plan->side : nullptr);
    if (e == hipSuccess && wide) {
        // the double results rounded into the caller's float arrays
        if (prof) Profiler::begin(&plan->prof, "narrow", s);
        const int64_t T = p.T, n = p.nx, m = p.nu;
        const void* src[6] = {a.S, a.v, a.K, a.d, a.x, a.u};
        void* dst[6] = {o.S, o.v, o.K, o.d, o.x, o.u};
        const int64_t cnt[6] = {(T + 1) * n * n, (T + 1) * n, T * m * n, T * m, (T + 1) * n, T * m};
        for (int i = 0; i < 6 && e == hipSuccess; ++i)
            if (dst[i]) e = lqt::convert_array(src[i], false, dst[i], true, cnt[i], s);
        if (prof) Profiler::end(&plan->prof, s);
    }
    if (e != hipSuccess) return fail(plan, LQT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return LQT_OK;
}

// Generalised instance (Section IV-D): lay out its transform at `ws` (taking
// `off` bytes forward), enqueue the transform to the standard form and turn
// (tp, to) -- copies of the instance and its outputs -- into the standard-form
// instance the solve takes.  g keeps what the map-back needs.
lqt_status gen_prepare(lqt_plan_t plan, char* ws, size_t& off, const lqt_problem& p, const lqt_outputs& o,
                       lqt_problem& tp, lqt_outputs& to, bool f32, hipStream_t s, lqt::GenArgs& g) {
    g = lqt::GenArgs{};
    g.F = p.F; g.c = p.c; g.L = p.L; g.H = p.H; g.X = p.X; g.U = p.U; g.M = p.M; g.r = p.r; g.s = p.s;
    g.T = p.T; g.n = p.nx; g.m = p.nu; g.p = p.ny;
    g.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
    lqt::gen_layout(g, (double*)(ws + off));
    off += align_up(lqt::gen_ws_doubles(p.nx, p.nu, p.ny, p.T, p.per_step & LQT_PS_F) * sizeof(double));
    tp = p;
    to = o;
    if (o.u && !o.x) {
        to.x = ws + off;
        off += align_up((size_t)(p.T + 1) * p.nx * sizeof(double));
    }
    g.K = to.K; g.d = to.d; g.u = to.u; g.x = to.x;
    g.f32 = f32 ? 1 : 0;
    tp.F = g.Ft; tp.c = g.ct; tp.X = g.Xt;
    tp.per_step |= LQT_PS_c;
    tp.M = nullptr;
    tp.s = nullptr;
    hipError_t e = lqt::gen_transform(g, s);
    if (e != hipSuccess) return fail(plan, LQT_EHIP, "transform launch failed: %s", hipGetErrorString(e));
    return LQT_OK;
}

// Instance-table entry of a chunked-path instance whose workspace starts at
// ws and whose K, d scratch (used when the caller does not take K and d)
// starts at kd.
lqt::GInst make_ginst(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o, char* ws, char* kd,
                      int64_t chunk0, int32_t* status, const WaveScratch& w) {
    lqt::GInst g{};
    g.F = p.F; g.c = p.c; g.L = p.L; g.U = p.U; g.H = p.H; g.X = p.X; g.r = p.r;
    g.HT = p.HT; g.XT = p.XT; g.rT = p.rT; g.x0 = p.x0;
    g.S = o.S; g.v = o.v; g.x = o.x; g.u = o.u;
    double* kdd = (double*)kd;  // sized for double gains; float ones use part of it
    g.K = (o.K && !w.wide) ? o.K : (void*)kdd;
    g.d = (o.d && !w.wide) ? o.d : (void*)(kdd + (size_t)p.T * p.nu * p.nx);
    char* sc = kd + w.kd;  // Method 2 / wide scratch: S | v | x | u
    if (w.S) g.S = sc;
    if (w.v) g.v = sc + w.S;
    if (w.wide && !w.S) g.S = nullptr;
    if (w.wide && !w.v) g.v = nullptr;
    if (w.m2) {
        g.traj = 1;
        g.x = g.u = nullptr;
        g.m2x = w.wide ? (o.x ? (void*)(sc + w.S + w.v) : nullptr) : o.x;
        g.m2u = w.wide ? (o.u ? (void*)(sc + w.S + w.v + w.x) : nullptr) : o.u;
    }
    g.status = status;
    g.T = p.T; g.n = p.nx; g.m = p.nu; g.p = p.ny; g.pT = p.nyT;
    g.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
    g.B = chunk_for(plan, p);
    g.NC = (p.T + g.B - 1) / g.B;
    g.chunk0 = chunk0;
    g.ws = (double*)ws;
    g.eng = eng_of(plan->route, p);
    g.tree = tree_for(plan->route, g.NC) ? 1 : 0;
    g.opf = opf_for(plan, p, g.B, g.NC) ? 1 : 0;
    return g;
}

// Arguments of one batched-lane instance whose workspace (batch_bytes)
// starts at ws.
lqt::SmallArgs make_batch_args(const lqt_problem& p, const lqt_outputs& o, char* ws, int32_t* status, bool f32) {
    lqt::SmallArgs a{};
    a.F = p.F; a.c = p.c; a.L = p.L; a.U = p.U; a.H = p.H; a.X = p.X; a.r = p.r;
    a.HT = p.HT; a.XT = p.XT; a.rT = p.rT; a.x0 = p.x0;
    a.T = p.T; a.n = p.nx; a.m = p.nu; a.p = p.ny; a.pT = p.nyT;
    a.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
    a.cst = (double*)ws;
    double* kd = (double*)(ws + align_up(lqt::small_cst_doubles(p.nx, p.nu, std::max(p.ny, 1)) * sizeof(double)));
    a.S = o.S; a.v = o.v; a.x = o.x; a.u = o.u;
    a.K = o.K ? o.K : (void*)kd;  // sized for double gains; float ones use part of it
    a.d = o.d ? o.d : (void*)(kd + (size_t)p.T * p.nu * p.nx);
    a.status = status;
    a.f32 = f32 ? 1 : 0;
    a.B = lqt::lane_batch_chunk(p.T);
    a.NC = (p.T + a.B - 1) / a.B;
    a.want_fwd = (o.x || o.u) ? 1 : 0;
    return a;
}

// Solve a set of instances on stream s in arena A.  status_override (if not
// null) gives per-instance device status words used instead of outs[i].status.
// Results are float when f32 is set (the plan's precision unless the caller
// says otherwise), else double.
lqt_status solve_all(lqt_plan_t plan, Arena& A, const lqt_problem* probs, const lqt_outputs* outs, int32_t count,
                     hipStream_t s, int32_t* const* status_override, int f32_override = -1) {
    const bool f32 = f32_override < 0 ? plan->desc.prec == LQT_PREC_MIXED : f32_override != 0;
    // partition by path; wavefront instances ordered by size class
    std::vector<int> small, wave, batch;
    for (int i = 0; i < count; ++i) {
        const Path path = path_of(plan, probs[i]);
        (path == Path::Small ? small : (path == Path::Batch ? batch : wave)).push_back(i);
    }
    // launch groups: (size class, engine)
    auto cls = [&](int i) {
        const int e = eng_of(plan->route, probs[i]);
        return 4 * tile_class_of(probs[i]) + (e == 0 ? 0 : (e == lqt::kEng32m16 ? 2 : 1));
    };
    std::stable_sort(wave.begin(), wave.end(), [&](int a, int b) { return cls(a) < cls(b); });
    // workspace: [generalised-cost transforms] [small-path region (largest small instance)] [wave region]
    // [instance table]
    BatchSize bs(plan, f32);
    for (int i = 0; i < count; ++i) bs.add(probs[i], outs[i]);
    std::vector<int64_t> ws_off(wave.size()), kd_off(wave.size());
    std::vector<WaveScratch> wsc(wave.size());
    size_t wave_need = 0;
    for (size_t j = 0; j < wave.size(); ++j) {
        ws_off[j] = (int64_t)wave_need;
        wave_need += wave_bytes(plan, std_shape(probs[wave[j]]));
        kd_off[j] = (int64_t)wave_need;
        wsc[j] = wave_scratch(plan, probs[wave[j]], outs[wave[j]], f32);
        wave_need += wsc[j].total();
    }
    lqt_status st = ensure_ws(plan, A, bs.total());
    if (st != LQT_OK) return st;
    // generalised instances: transform to the standard form (Section IV-D) at
    // the start of the arena, solve the transforms, map the results back
    std::vector<lqt_problem> tp;
    std::vector<lqt_outputs> to;
    std::vector<lqt::GenArgs> gens;
    if (bs.gen) {
        tp.assign(probs, probs + count);
        to.assign(outs, outs + count);
        size_t off = 0;
        if (plan->prof.on) Profiler::begin(&plan->prof, "gen_transform", s);
        for (int i = 0; i < count; ++i) {
            if (!is_gen(probs[i])) continue;
            lqt::GenArgs g;
            st = gen_prepare(plan, A.ws, off, probs[i], outs[i], tp[i], to[i], f32, s, g);
            if (st != LQT_OK) return st;
            gens.push_back(g);
        }
        if (plan->prof.on) Profiler::end(&plan->prof, s);
        probs = tp.data();
        outs = to.data();
    }
    auto post = [&]() -> lqt_status {
        if (gens.empty()) return LQT_OK;
        if (plan->prof.on) Profiler::begin(&plan->prof, "gen_post", s);
        for (const lqt::GenArgs& g : gens) {
            hipError_t e = lqt::gen_post(g, s);
            if (e != hipSuccess) return fail(plan, LQT_EHIP, "map-back launch failed: %s", hipGetErrorString(e));
        }
        if (plan->prof.on) Profiler::end(&plan->prof, s);
        return LQT_OK;
    };
    char* const base = A.ws + bs.gen;
    for (int i : small) {
        st = launch_one(plan, base, probs[i], outs[i], s, status_override ? status_override[i] : nullptr, f32);
        if (st != LQT_OK) return st;
    }
    if ((!batch.empty() || !wave.empty()) && A.ginst_done && !A.capture)
        (void)hipEventSynchronize(A.ginst_done);  // the previous upload has left the host tables
    if (!batch.empty()) {
        // one launch pair per (n, m, step-data mode) group
        auto bkey = [&](int i) {
            const lqt_problem& p = probs[i];
            return (p.nx * 8 + p.nu) * 4 + lqt::lane_batch_mode(p.nx, p.ny, p.per_step, p.c != nullptr);
        };
        std::stable_sort(batch.begin(), batch.end(), [&](int a, int b) { return bkey(a) < bkey(b); });
        if (A.sargs_cap < batch.size()) {
            if (A.sargs_host) (void)hipHostFree(A.sargs_host);
            A.sargs_host = nullptr;
            A.sargs_cap = 0;
            const size_t cap = std::max<size_t>(batch.size(), 256);
            if (hipHostMalloc((void**)&A.sargs_host, cap * sizeof(lqt::SmallArgs), 0) != hipSuccess)
                return fail(plan, LQT_ENOMEM, "pinned instance table allocation failed");
            A.sargs_cap = cap;
        }
        char* const bbase = A.ws + bs.wave_end();
        size_t off = 0;
        for (size_t j = 0; j < batch.size(); ++j) {
            A.sargs_host[j] = make_batch_args(probs[batch[j]], outs[batch[j]], bbase + off,
                                              status_override ? status_override[batch[j]] : outs[batch[j]].status,
                                              f32);
            off += batch_bytes(probs[batch[j]], outs[batch[j]]);
        }
        lqt::SmallArgs* d_tab = (lqt::SmallArgs*)(bbase + bs.batch);
        if (hipMemcpyAsync(d_tab, A.sargs_host, batch.size() * sizeof(lqt::SmallArgs), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(plan, LQT_EHIP, "instance table upload failed");
        lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
        for (size_t j0 = 0; j0 < batch.size();) {
            size_t j1 = j0;
            while (j1 < batch.size() && bkey(batch[j1]) == bkey(batch[j0])) ++j1;
            const lqt_problem& p0 = probs[batch[j0]];
            hipError_t e = lqt::lane_batch_solve(p0.nx, p0.nu, lqt::lane_batch_mode(p0.nx, p0.ny, p0.per_step,
                                                                                   p0.c != nullptr),
                                                 f32, d_tab + j0, (int)(j1 - j0), s, plan->prof.on ? &hook : nullptr);
            if (e != hipSuccess) return fail(plan, LQT_EHIP, "batched lane launch failed: %s", hipGetErrorString(e));
            j0 = j1;
        }
        if (wave.empty() && !A.capture) {
            if (!A.ginst_done && hipEventCreateWithFlags(&A.ginst_done, hipEventDisableTiming) != hipSuccess)
                return fail(plan, LQT_EHIP, "event creation failed");
            (void)hipEventRecord(A.ginst_done, s);
        }
    }
    if (wave.empty()) return post();
    if (A.ginst_cap < wave.size()) {
        if (A.ginst_host) (void)hipHostFree(A.ginst_host);
        A.ginst_host = nullptr;
        A.ginst_cap = 0;
        const size_t cap = std::max<size_t>(wave.size(), 64);
        if (hipHostMalloc((void**)&A.ginst_host, cap * sizeof(lqt::GInst), 0) != hipSuccess)
            return fail(plan, LQT_ENOMEM, "pinned instance table allocation failed");
        A.ginst_cap = cap;
    }
    char* wbase = base + bs.small;
    std::vector<char> want_fwd_c(wave.size(), 0);
    int64_t chunk0 = 0;
    for (size_t j = 0; j < wave.size(); ++j) {
        if (j > 0 && cls(wave[j]) != cls(wave[j - 1])) chunk0 = 0;  // each class numbers its own chunks
        const lqt_problem& p = probs[wave[j]];
        const lqt_outputs& o = outs[wave[j]];
        lqt::GInst& g = A.ginst_host[j];
        g = make_ginst(plan, p, o, wbase + ws_off[j], wbase + kd_off[j], chunk0,
                       status_override ? status_override[wave[j]] : o.status, wsc[j]);
        chunk0 += g.NC;
        want_fwd_c[j] = (g.x || g.u) ? 1 : (g.traj ? 2 : 0);
    }
    lqt::GInst* d_inst = (lqt::GInst*)(wbase + bs.wave);
    if (hipMemcpyAsync(d_inst, A.ginst_host, wave.size() * sizeof(lqt::GInst), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return fail(plan, LQT_EHIP, "instance table upload failed");
    if (!A.capture) {
        if (!A.ginst_done && hipEventCreateWithFlags(&A.ginst_done, hipEventDisableTiming) != hipSuccess)
            return fail(plan, LQT_EHIP, "event creation failed");
        (void)hipEventRecord(A.ginst_done, s);
    }
    lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
    // chunked groups of a plan with forward prefixes and float results run
    // with double results (wide) and are rounded afterwards
    const bool gf32 = f32 && plan->desc.trajectory != LQT_TRAJ_PREFIX;
    for (size_t j0 = 0; j0 < wave.size();) {
        size_t j1 = j0;
        int64_t nch = 0, max_nc = 0, tree_nc = 0;
        bool fwd = false, m2 = false, opf_any = false;
        while (j1 < wave.size() && cls(wave[j1]) == cls(wave[j0])) {
            nch += A.ginst_host[j1].NC;
            max_nc = std::max(max_nc, A.ginst_host[j1].NC);
            if (A.ginst_host[j1].tree) tree_nc = std::max(tree_nc, A.ginst_host[j1].NC);
            opf_any = opf_any || A.ginst_host[j1].opf;
            fwd = fwd || want_fwd_c[j1] == 1;
            m2 = m2 || want_fwd_c[j1] == 2;
            ++j1;
        }
        const lqt_problem& p0 = probs[wave[j0]];
        const int eng = eng_of(plan->route, p0);
        const lqt::StageHook* hk = plan->prof.on ? &hook : nullptr;
        hipError_t e = eng ? lqt::block_solve(eng, d_inst + j0, (int)(j1 - j0), nch, max_nc, tree_nc, fwd, gf32, s, hk)
                           : lqt::tile_solve(tile_class_of(p0), d_inst + j0, (int)(j1 - j0), nch, tree_nc, fwd, gf32, s,
                                             hk, opf_any);
        if (e == hipSuccess && m2)
            e = lqt::m2_chunked(eng ? lqt::eng_dim(eng) : tile_class_of(p0), d_inst + j0, (int)(j1 - j0), nch, s,
                                hk);
        if (e != hipSuccess) return fail(plan, LQT_EHIP, "wavefront-path launch failed: %s", hipGetErrorString(e));
        j0 = j1;
    }
    // wide instances: double results rounded into the caller's float arrays
    bool any_wide = false;
    for (const WaveScratch& w : wsc) any_wide = any_wide || w.wide;
    if (any_wide) {
        if (plan->prof.on) Profiler::begin(&plan->prof, "narrow", s);
        for (size_t j = 0; j < wave.size(); ++j) {
            if (!wsc[j].wide) continue;
            const lqt_problem& p = probs[wave[j]];
            const lqt_outputs& o = outs[wave[j]];
            const lqt::GInst& g = A.ginst_host[j];
            const int64_t T = p.T, n = p.nx, m = p.nu;
            const void* src[6] = {g.S, g.v, g.K, g.d, g.traj ? g.m2x : nullptr, g.traj ? g.m2u : nullptr};
            void* dst[6] = {o.S, o.v, o.K, o.d, o.x, o.u};
            const int64_t cnt[6] = {(T + 1) * n * n, (T + 1) * n, T * m * n, T * m, (T + 1) * n, T * m};
            for (int i = 0; i < 6; ++i) {
                if (!dst[i] || !src[i]) continue;
                hipError_t e = lqt::convert_array(src[i], false, dst[i], true, cnt[i], s);
                if (e != hipSuccess) return fail(plan, LQT_EHIP, "narrowing launch failed: %s", hipGetErrorString(e));
            }
        }
        if (plan->prof.on) Profiler::end(&plan->prof, s);
    }
    return post();
}

// ---- allocation-free solve ---------------------------------------------------
//
// lqt_solve_noalloc keeps its workspace in `scratch`, a fixed device array of
// the library (one per device, held until the process ends), instead of
// memory the plan allocates.  Host code reaches it only through the device
// address read once per device at plan creation (noalloc_base).

}  // namespace

constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};

// Reads this device's address of `scratch` (the device must be current).
// Once per device; a failure leaves the pointer null and lqt_solve_noalloc
// then reports LQT_EHIP.
void noalloc_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[dev]) return;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    g_noalloc_ptr[dev] = (char*)ptr;
}

char* noalloc_base(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc_ptr[dev];
}

// Stores one instance-table entry into device memory from the kernel's
// arguments (no host staging buffer).
__global__ void k_put_inst(lqt::GInst g, lqt::GInst* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = g;
}

__global__ void k_put_sargs(lqt::SmallArgs a, lqt::SmallArgs* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}

// One instance solved with its whole workspace in [base, base + cap): the
// regions of solve_all for a batch of one, the instance table included.
// Enqueues kernels only: no device or host allocation, no events.
lqt_status solve_static(lqt_plan_t plan, char* base, size_t cap, const lqt_problem& p0, const lqt_outputs& o0,
                        hipStream_t s) {
    const bool f32 = plan->desc.prec == LQT_PREC_MIXED;
    BatchSize bs(plan, f32);
    bs.add(p0, o0);
    if (bs.total() > cap)
        return fail(plan, LQT_ENOMEM,
                    "lqt_solve_noalloc: the instance needs %zu bytes of workspace, the static workspace holds %zu "
                    "(nx=%d nu=%d T=%lld)", bs.total(), cap, p0.nx, p0.nu, (long long)p0.T);
    lqt_problem p = p0;
    lqt_outputs o = o0;
    lqt::GenArgs g{};
    const bool gen = is_gen(p0);
    lqt_status st = LQT_OK;
    if (gen) {
        size_t off = 0;
        if ((st = gen_prepare(plan, base, off, p0, o0, p, o, f32, s, g)) != LQT_OK) return st;
    }
    char* const b = base + bs.gen;
    const Path path = path_of(plan, p);
    if (path == Path::Small) {
        if ((st = launch_one(plan, b, p, o, s, nullptr, f32, false)) != LQT_OK) return st;
    } else if (path == Path::Batch) {
        char* const bb = base + bs.wave_end();
        const lqt::SmallArgs a = make_batch_args(p, o, bb, o.status, f32);
        lqt::SmallArgs* d_tab = (lqt::SmallArgs*)(bb + bs.batch);
        k_put_sargs<<<1, 64, 0, s>>>(a, d_tab);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = lqt::lane_batch_solve(p.nx, p.nu, lqt::lane_batch_mode(p.nx, p.ny, p.per_step, p.c != nullptr), f32,
                                      d_tab, 1, s, nullptr);
        if (e != hipSuccess) return fail(plan, LQT_EHIP, "batched lane launch failed: %s", hipGetErrorString(e));
    } else {
        char* const ws = b + bs.small;
        char* const kd = ws + wave_bytes(plan, std_shape(p0));
        const WaveScratch w = wave_scratch(plan, p0, o0, f32);
        if (w.wide)
            return fail(plan, LQT_ENOTSUP,
                        "lqt_solve_noalloc: forward prefixes with float results on the chunked engines are "
                        "provided by lqt_solve only");
        const lqt::GInst gi = make_ginst(plan, p, o, ws, kd, 0, o.status, w);
        lqt::GInst* d_inst = (lqt::GInst*)(ws + bs.wave);
        k_put_inst<<<1, 64, 0, s>>>(gi, d_inst);
        hipError_t e = hipGetLastError();
        const bool fwd = gi.x || gi.u;
        const int eng = eng_of(plan->route, p);
        if (e == hipSuccess)
            e = eng ? lqt::block_solve(eng, d_inst, 1, gi.NC, gi.NC, gi.tree ? gi.NC : 0, fwd, f32, s, nullptr)
                    : lqt::tile_solve(tile_class_of(p), d_inst, 1, gi.NC, gi.tree ? gi.NC : 0, fwd, f32, s, nullptr,
                                      gi.opf != 0);
        if (e == hipSuccess && gi.traj)
            e = lqt::m2_chunked(eng ? lqt::eng_dim(eng) : tile_class_of(p), d_inst, 1, gi.NC, s, nullptr);
        if (e != hipSuccess) return fail(plan, LQT_EHIP, "wavefront-path launch failed: %s", hipGetErrorString(e));
    }
    if (gen) {
        hipError_t e = lqt::gen_post(g, s);
        if (e != hipSuccess) return fail(plan, LQT_EHIP, "map-back launch failed: %s", hipGetErrorString(e));
    }
    return LQT_OK;
}

void arena_release(Arena& A) {
    if (A.ginst_done) (void)hipEventDestroy(A.ginst_done);
    if (A.ginst_host) (void)hipHostFree(A.ginst_host);
    if (A.sargs_host) (void)hipHostFree(A.sargs_host);
    if (A.owned && A.ws) (void)hipFree(A.ws);
    A = Arena{};
}

// ---- serving: continuous batching -----------------------------------------
//
// The admission logic (per-lane FIFOs, batches as long FIFO prefixes that fit
// one free range of the pool, slots owned by lanes) is the host-only core of
// lqt_serve.hpp; the operations below are its device side.  Progress is made
// inside lqt_submit and lqt_poll and by a progress thread of the plan, so
// queued requests are launched and finished batches retired also while the
// caller does neither.

size_t serve_bytes(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o) {
    BatchSize b(plan);
    b.add(p, o);
    return b.total();
}

// Lane of a request: 1 (long) when its critical path is long -- the chunked
// engines walk about 3 B + NC steps in sequence (fold, chain, down-sweep,
// roll-out) at a cost that grows with the size class -- else 0.
int serve_lane(lqt_plan_t plan, const lqt_problem& p0) {
    const lqt_problem p = std_shape(p0);
    if (path_of(plan, p) != Path::Wave) return 0;  // one launch sequence of short walks
    const int64_t B = chunk_for(plan, p), NC = (p.T + B - 1) / B;
    return (3 * B + NC) * (int64_t)tile_class_of(p) > 4096 ? 1 : 0;
}

}  // namespace

struct ServeOps::Acc {
    BatchSize bs;
    lqt_plan_t plan;
    explicit Acc(lqt_plan_t pl) : bs(pl), plan(pl) {}
    void add(size_t h) {
        const PendingReq& r = plan->payload.at(h);
        bs.add(r.p, r.o);
    }
    size_t total() const { return bs.total(); }
};

ServeOps::Acc ServeOps::acc() { return Acc(plan); }

int ServeOps::launch(int si, const size_t* req, size_t count, size_t off, size_t len) {
    Slot& s = plan->slots[si];
    std::vector<lqt_problem> ps(count);
    std::vector<lqt_outputs> os(count);
    std::vector<int32_t*> ovr(count);
    for (size_t i = 0; i < count; ++i) {
        auto it = plan->payload.find(req[i]);
        ps[i] = it->second.p;
        os[i] = it->second.o;
        ovr[i] = s.status_dev + i;
        plan->payload.erase(it);  // the batch's launch takes what it needs
    }
    s.arena.ws = plan->pool + off;
    s.arena.cap = len;
    lqt_status st = solve_all(plan, s.arena, ps.data(), os.data(), (int32_t)count, s.stream, ovr.data());
    if (st == LQT_OK &&
        hipMemcpyAsync(s.status_host, s.status_dev, count * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream) !=
            hipSuccess)
        st = fail(plan, LQT_EHIP, "status copy failed");
    for (size_t i = 0; st == LQT_OK && i < count; ++i)
        if (os[i].status &&
            hipMemcpyAsync(os[i].status, s.status_dev + i, sizeof(int32_t), hipMemcpyDefault, s.stream) != hipSuccess)
            st = fail(plan, LQT_EHIP, "status copy failed");
    if (st == LQT_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = fail(plan, LQT_EHIP, "event record failed");
    return st;
}

int ServeOps::query(int si) {
    const hipError_t q = hipEventQuery(plan->slots[si].done);
    if (q == hipSuccess) return 1;
    (void)hipGetLastError();
    return q == hipErrorNotReady ? 0 : -1;
}

int ServeOps::status(int si, size_t i) { return plan->slots[si].status_host[i]; }

void ServeOps::drain(int si) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(plan->slots[si].stream);
    (void)hipGetLastError();
}

namespace {

void slot_release(Slot& s) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.status_dev) (void)hipFree(s.status_dev);
    if (s.status_host) (void)hipHostFree(s.status_host);
    arena_release(s.arena);
    s = Slot{};
}

// Progress thread: retires finished batches and launches queued requests
// every ~50 us while work is in flight; sleeps until a submit otherwise.
void serve_progress(lqt_plan_t plan) {
    (void)hipSetDevice(plan->desc.device);
    std::unique_lock<std::recursive_mutex> lk(plan->mu);
    while (!plan->stop) {
        (void)plan->core.pump(plan->ops);
        if (plan->core.idle()) {
            plan->wake.wait_for(lk, std::chrono::milliseconds(20));
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        }
    }
}

// All or nothing: the pool and every slot exist afterwards, or none of them
// (plan->pool is set last, so a failed set-up is retried by the next submit).
lqt_status serve_init(lqt_plan_t plan) {
    if (plan->pool) return LQT_OK;
    const size_t want = plan->desc.hbm_budget_bytes ? plan->desc.hbm_budget_bytes : kDefaultServePool;
    std::vector<Slot> slots(kServeSlots);
    bool ok = true;
    for (Slot& s : slots) {
        s.arena.owned = false;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&s.status_dev, kServeBatchMax * sizeof(int32_t)) != hipSuccess ||
            hipHostMalloc((void**)&s.status_host, kServeBatchMax * sizeof(int32_t), 0) != hipSuccess) {
            ok = false;
            break;
        }
    }
    void* p = nullptr;
    if (ok && hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        for (Slot& s : slots) slot_release(s);
        return fail(plan, LQT_ENOMEM, "hipMalloc of the %zu-byte serving pool failed", want);
    }
    if (!ok) {
        (void)hipGetLastError();
        for (Slot& s : slots) slot_release(s);
        return fail(plan, LQT_EHIP, "serving slot set-up failed");
    }
    plan->slots = std::move(slots);
    std::vector<int> lanes(kServeSlots);
    for (int i = 0; i < kServeSlots; ++i) lanes[i] = i < kServeSlots / 2 ? 0 : 1;  // half short, half long
    plan->core.init(want, lanes, kServeBatchMax, plan->desc.max_inflight);
    plan->ops.plan = plan;
    plan->pool = (char*)p;
    plan->stop = false;
    plan->progress = std::thread(serve_progress, plan);
    return LQT_OK;
}

// The rounds of lqt_nl_iterate enqueued on stream s, with the linearised
// model in arena NA and the solves in arena MA (p, o: the validated instance
// of a round, model pointers filled in here).
lqt_status nl_enqueue(lqt_plan_t plan, Arena& NA, Arena& MA, const lqt_nl_problem& pr, lqt_problem p, lqt_outputs o,
                      int32_t iterations, void* x, void* u, double* change, int32_t* status, hipStream_t s) {
    const lqt_nl_problem* prob = &pr;
    const int n = 4, m = 2;
    const int64_t T = prob->T;
    lqt_status st = LQT_OK;
    // A MIXED plan iterates in double: the nominal trajectory of every round
    // is kept in double workspace (xd, ud), each round is solved with double
    // results, and only the last round's x and u are rounded to float.
    const bool f32 = plan->desc.prec == LQT_PREC_MIXED;
    const size_t model = align_up((size_t)T * (n * n + n * m + n + m) * sizeof(double));
    const size_t nominal = f32 ? align_up((size_t)((T + 1) * n + T * m) * sizeof(double)) : 0;
    st = ensure_ws(plan, NA, model + nominal + align_up((size_t)iterations * sizeof(int32_t)));
    if (st != LQT_OK) return st;
    lqt::NlArgs g{};
    g.dt = prob->dt;
    g.T = T;
    g.F = (double*)NA.ws;
    g.L = g.F + (size_t)T * n * n;
    g.c = g.L + (size_t)T * n * m;
    g.ubar = g.c + (size_t)T * n;
    double* xd = f32 ? (double*)(NA.ws + model) : nullptr;
    double* ud = f32 ? xd + (size_t)(T + 1) * n : nullptr;
    g.x = f32 ? xd : (const double*)x;
    g.u = f32 ? ud : (const double*)u;
    int32_t* round_status = (int32_t*)(NA.ws + model + nominal);
    p.F = g.F; p.L = g.L; p.c = g.c;
    o.x = f32 ? (void*)xd : x;
    o.u = f32 ? (void*)ud : u;
    auto launched = [&](hipError_t e) -> lqt_status {
        return e == hipSuccess ? LQT_OK : fail(plan, LQT_EHIP, "launch failed: %s", hipGetErrorString(e));
    };
    if ((st = launched(lqt::nl_start(change, iterations, round_status, s))) != LQT_OK) return st;
    if (f32) {
        if ((st = launched(lqt::convert_array(x, true, xd, false, (T + 1) * n, s))) != LQT_OK) return st;
        if ((st = launched(lqt::convert_array(u, true, ud, false, T * m, s))) != LQT_OK) return st;
    }
    for (int it = 0; it < iterations; ++it) {
        // the change of round it - 1 is completed by this round's linearisation
        if (plan->prof.on) Profiler::begin(&plan->prof, "nl_linearise", s);
        st = launched(lqt::nl_linearise(g, (change && it > 0) ? change + it - 1 : nullptr, s));
        if (plan->prof.on) Profiler::end(&plan->prof, s);
        if (st != LQT_OK) return st;
        o.status = round_status + it;
        if ((st = solve_all(plan, MA, &p, &o, 1, s, nullptr, 0)) != LQT_OK) return st;
    }
    if (change) {
        if (plan->prof.on) Profiler::begin(&plan->prof, "nl_change", s);
        st = launched(lqt::nl_change(g, change + iterations - 1, s));
        if (plan->prof.on) Profiler::end(&plan->prof, s);
        if (st != LQT_OK) return st;
    }
    if (f32) {
        if ((st = launched(lqt::convert_array(xd, false, x, true, (T + 1) * n, s))) != LQT_OK) return st;
        if ((st = launched(lqt::convert_array(ud, false, u, true, T * m, s))) != LQT_OK) return st;
    }
    return launched(lqt::nl_finish(round_status, iterations, status, s));
}


// ---- graph replay (lqt_set_graphs) ------------------------------------------
//
// A call whose signature (every argument's bytes: dimensions, per-step bits
// and device pointers) has been seen before replays the HIP graph recorded
// for it.  The first call runs directly in the entry's own arenas (sizing
// them, producing its results), then the same enqueue is recorded by stream
// capture on the plan's capture stream and instantiated.  Every host-side
// decision of an enqueue depends on the signature alone, and the instance
// tables of a graph live in its own pinned buffers, so a replay performs the
// recorded work on the current contents of the same buffers.

void sig_add(std::string& k, const void* p, size_t n) { k.append((const char*)p, n); }

template <class T>
void sig_val(std::string& k, const T& v) {
    sig_add(k, &v, sizeof v);
}

// field by field (struct padding is not part of a signature)
void sig_problem(std::string& k, const lqt_problem& p) {
    sig_val(k, p.nx); sig_val(k, p.nu); sig_val(k, p.ny); sig_val(k, p.nyT); sig_val(k, p.T);
    sig_val(k, p.per_step);
    const double* ptr[] = {p.F, p.c, p.L, p.H, p.X, p.U, p.r, p.HT, p.XT, p.rT, p.x0, p.M, p.s};
    sig_add(k, ptr, sizeof ptr);
}

void sig_outputs(std::string& k, const lqt_outputs& o) {
    const void* ptr[] = {o.S, o.v, o.K, o.d, o.x, o.u, o.status};
    sig_add(k, ptr, sizeof ptr);
}

void sig_nl(std::string& k, const lqt_nl_problem& p) {
    sig_val(k, (int32_t)p.model); sig_val(k, p.ny); sig_val(k, p.nyT); sig_val(k, p.T); sig_val(k, p.per_step);
    const double* ptr[] = {p.dt, p.H, p.X, p.U, p.r, p.HT, p.XT, p.rT, p.x0};
    sig_add(k, ptr, sizeof ptr);
}

constexpr size_t kGraphCacheMax = 64;  // recorded signatures kept per plan

void graph_free(GraphEntry* e) {
    if (!e) return;
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    arena_release(e->main);
    arena_release(e->nl);
    delete e;
}

void graph_clear(lqt_plan_t plan) {
    if (plan->gcache.empty()) return;
    (void)hipDeviceSynchronize();  // a replay in flight may still use an entry's arenas
    for (auto& kv : plan->gcache) graph_free(kv.second);
    plan->gcache.clear();
}

template <class Enqueue>
lqt_status graph_run(lqt_plan_t plan, const std::string& key, hipStream_t s, Enqueue enqueue) {
    auto it = plan->gcache.find(key);
    if (it != plan->gcache.end()) {
        if (hipGraphLaunch(it->second->exec, s) != hipSuccess)
            return fail(plan, LQT_EHIP, "graph launch failed: %s", hipGetErrorString(hipGetLastError()));
        return LQT_OK;
    }
    if (plan->gcache.size() >= kGraphCacheMax) graph_clear(plan);
    GraphEntry* e = new (std::nothrow) GraphEntry();
    if (!e) return fail(plan, LQT_ENOMEM, "graph entry: out of host memory");
    lqt_status st = enqueue(*e, s);  // direct run: sizes the arenas, produces this call's results
    if (st != LQT_OK) {
        (void)hipStreamSynchronize(s);
        graph_free(e);
        return st;
    }
    for (Arena* A : {&e->main, &e->nl})
        if (A->ginst_done) (void)hipEventSynchronize(A->ginst_done);  // host tables free to be rewritten
    e->main.capture = e->nl.capture = true;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
        const lqt_status cst = enqueue(*e, plan->cap_stream);
        ok = hipStreamEndCapture(plan->cap_stream, &g) == hipSuccess && cst == LQT_OK && g;
    }
    e->main.capture = e->nl.capture = false;
    if (ok) ok = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok) {  // not recorded: this call's results stand, later calls record again
        (void)hipStreamSynchronize(s);
        graph_free(e);
        return LQT_OK;
    }
    plan->gcache[key] = e;
    return LQT_OK;
}

}  // namespace

extern "C" {

lqt_status lqt_plan(const lqt_plan_desc* desc, lqt_plan_t* out) {
    if (!desc || !out) return fail(nullptr, LQT_EINVAL, "lqt_plan: NULL argument");
    *out = nullptr;
    if (desc->max_nx < 1 || desc->max_nu < 1)
        return fail(nullptr, LQT_EINVAL, "lqt_plan: max_nx and max_nu must be >= 1");
    if (desc->max_nx > kMaxNx)
        return fail(nullptr, LQT_ENOTSUP, "lqt_plan: max_nx=%d exceeds the library's limit %d", desc->max_nx, kMaxNx);
    if (desc->prec != LQT_PREC_FP64 && desc->prec != LQT_PREC_MIXED)
        return fail(nullptr, LQT_EINVAL, "lqt_plan: unknown precision %d", (int)desc->prec);
    if (desc->trajectory != LQT_TRAJ_MAPS && desc->trajectory != LQT_TRAJ_PREFIX)
        return fail(nullptr, LQT_EINVAL, "lqt_plan: unknown trajectory method %d", (int)desc->trajectory);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(nullptr, LQT_EHIP, "lqt_plan: no HIP device");
    }
    if (desc->device < 0 || desc->device >= ndev)
        return fail(nullptr, LQT_EINVAL, "lqt_plan: device %d out of range [0, %d)", desc->device, ndev);
    if (hipSetDevice(desc->device) != hipSuccess) return fail(nullptr, LQT_EHIP, "lqt_plan: hipSetDevice failed");
    lqt_plan_s* p = new (std::nothrow) lqt_plan_s();
    if (!p) return fail(nullptr, LQT_ENOMEM, "lqt_plan: out of host memory");
    p->desc = *desc;
    p->err.reserve(600);  // error texts (<= 512 bytes) are then formatted without allocating
    if (p->desc.max_inflight <= 0) p->desc.max_inflight = kDefaultQueue;
    noalloc_init(desc->device);
    if (desc->trajectory == LQT_TRAJ_PREFIX) {
        // a failure leaves the element scan on the solve's own stream
        lqt::SideStream& sd = p->side;
        if (hipStreamCreateWithFlags(&sd.side, hipStreamNonBlocking) == hipSuccess) {
            if (hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) == hipSuccess) {
                if (hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) == hipSuccess) {
                    p->has_side = true;
                } else {
                    (void)hipEventDestroy(sd.fork);
                    (void)hipStreamDestroy(sd.side);
                }
            } else {
                (void)hipStreamDestroy(sd.side);
            }
        }
        (void)hipGetLastError();
    }
    if (desc->max_steps > 0) {
        lqt_problem probe{};
        probe.nx = desc->max_nx; probe.nu = desc->max_nu; probe.ny = desc->max_nx; probe.nyT = desc->max_nx;
        probe.T = desc->max_steps;
        size_t need = 0;
        // size for the worst case among the supported (n, m) up to the maxima
        for (int n = 1; n <= desc->max_nx; ++n)
            for (int m = 1; m <= desc->max_nu; ++m)
                if (lqt::small_supported(n, m)) {
                    probe.nx = n; probe.nu = m; probe.ny = n;
                    need = std::max(need, layout_for(p->route, probe, true, true,
                                                     desc->trajectory == LQT_TRAJ_PREFIX, true, true).total);
                }
        // and for one wavefront-path instance of the largest dimensions
        {
            const int64_t B = wave_chunk(p->route, desc->max_steps, 0, desc->trajectory == LQT_TRAJ_PREFIX);
            const int64_t NC = (desc->max_steps + B - 1) / B;
            const int cls = lqt::tile_class(std::max(desc->max_nx, desc->max_nu));
            const int64_t wd = std::max(lqt::ws_doubles(desc->max_nx, desc->max_nu, desc->max_nx, 0, NC, B, false, true,
                                                        true),
                                        lqt::ws_doubles(desc->max_nx, desc->max_nu, desc->max_nx, cls, NC, B, false,
                                                        true));
            const size_t w = (size_t)wd * 8 +
                             (size_t)desc->max_steps * (desc->max_nu * desc->max_nx + desc->max_nu) * 8 + 4096;
            need = std::max(need, w);
        }
        lqt_status st = ensure_ws(p, p->main, need);
        if (st != LQT_OK) {
            g_create_error = p->err;
            if (p->has_side) {
                (void)hipStreamDestroy(p->side.side);
                (void)hipEventDestroy(p->side.fork);
                (void)hipEventDestroy(p->side.join);
            }
            delete p;
            return st;
        }
    }
    *out = p;
    return LQT_OK;
}

lqt_status lqt_solve(lqt_plan_t plan, const lqt_problem* probs, const lqt_outputs* outs, int32_t count,
                     void* stream) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_solve: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (count < 0 || (count > 0 && (!probs || !outs))) return fail(plan, LQT_EINVAL, "lqt_solve: bad count/arrays");
    for (int i = 0; i < count; ++i) {
        lqt_status st = validate(plan, probs[i], outs[i], i);
        if (st != LQT_OK) return st;
    }
    if (count == 0) return LQT_OK;
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    if (!plan->graphs || plan->prof.on) return solve_all(plan, plan->main, probs, outs, count, s, nullptr);
    std::string key("solve");
    sig_val(key, count);
    for (int32_t i = 0; i < count; ++i) {
        sig_problem(key, probs[i]);
        sig_outputs(key, outs[i]);
    }
    return graph_run(plan, key, s, [&](GraphEntry& e, hipStream_t gs) {
        return solve_all(plan, e.main, probs, outs, count, gs, nullptr);
    });
}

lqt_status lqt_solve_noalloc(lqt_plan_t plan, const lqt_problem* prob, const lqt_outputs* out, void* stream) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_solve_noalloc: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (!prob || !out) return fail(plan, LQT_EINVAL, "lqt_solve_noalloc: NULL problem or outputs");
    lqt_status st = validate(plan, *prob, *out, 0);
    if (st != LQT_OK) return st;
    char* const base = noalloc_base(plan->desc.device);
    if (!base)
        return fail(plan, LQT_EHIP, "lqt_solve_noalloc: the static workspace of device %d is not available",
                    plan->desc.device);
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    return solve_static(plan, base, kNoAllocBytes, *prob, *out, (hipStream_t)stream);
}

lqt_status lqt_tune(lqt_plan_t plan, const lqt_problem* probs, const lqt_outputs* outs, int32_t count, void* stream,
                    int32_t* chosen) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_tune: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (count < 0 || (count > 0 && (!probs || !outs))) return fail(plan, LQT_EINVAL, "lqt_tune: bad count/arrays");
    for (int i = 0; i < count; ++i) {
        lqt_status st = validate(plan, probs[i], outs[i], i);
        if (st != LQT_OK) return st;
    }
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    graph_clear(plan);  // recorded launch sequences follow the chunk lengths
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(plan, LQT_EHIP, "lqt_tune: event creation failed");
    lqt_status st = LQT_OK;
    for (int key = 0; key < 8 && st == LQT_OK; ++key) {
        std::vector<lqt_problem> ps;
        std::vector<lqt_outputs> os;
        for (int i = 0; i < count; ++i)
            if (path_of(plan, probs[i]) == Path::Wave && group_key(plan->route, probs[i]) == key) {
                ps.push_back(probs[i]);
                os.push_back(outs[i]);
            }
        if (ps.empty()) continue;
        float best = 0.f;
        int best_div = 0;
        for (int div : kTuneDivs) {
            plan->tune_div[key] = div;
            float ms = 0.f;
            for (int rep = 0; rep < 2 && st == LQT_OK; ++rep) {  // the first run warms up
                (void)hipEventRecord(e0, s);
                st = solve_all(plan, plan->main, ps.data(), os.data(), (int32_t)ps.size(), s, nullptr);
                (void)hipEventRecord(e1, s);
                if (st == LQT_OK && hipEventSynchronize(e1) != hipSuccess)
                    st = fail(plan, LQT_EHIP, "lqt_tune: timing failed");
                if (st == LQT_OK) (void)hipEventElapsedTime(&ms, e0, e1);
            }
            if (st != LQT_OK) break;
            if (best == 0.f || ms < best) {
                best = ms;
                best_div = div;
            }
        }
        plan->tune_div[key] = best_div;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (chosen)
        for (int key = 0; key < 8; ++key) chosen[key] = plan->tune_div[key];
    return st;
}

lqt_status lqt_set_graphs(lqt_plan_t plan, int32_t enable) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_set_graphs: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    if (!enable) {
        graph_clear(plan);
        plan->graphs = false;
        return LQT_OK;
    }
    if (!plan->cap_stream && hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return fail(plan, LQT_EHIP, "lqt_set_graphs: capture stream creation failed");
    }
    plan->graphs = true;
    return LQT_OK;
}

int32_t lqt_graphs_recorded(lqt_plan_t plan) {
    if (!plan) return -(int32_t)fail(nullptr, LQT_EINVAL, "lqt_graphs_recorded: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    return (int32_t)plan->gcache.size();
}

lqt_status lqt_set_routing(lqt_plan_t plan, const lqt_routing* routing) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_set_routing: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    graph_clear(plan);  // recorded launch sequences follow the routing
    if (!routing) {
        plan->route = lqt_routing{};
        return LQT_OK;
    }
    const lqt_routing& r = *routing;
    if (r.path < 0 || r.path > 3 || r.block < 0 || r.block > 1 || r.lane_chunk < 0 || r.lane_chunk > 1024 ||
        r.wave_chunk < 0 || r.wave_chunk > 4096 || r.tree < 0 || r.tree > 2)
        return fail(plan, LQT_EINVAL,
                    "lqt_set_routing: path=%d block=%d lane_chunk=%d wave_chunk=%d tree=%d out of range", r.path,
                    r.block, r.lane_chunk, r.wave_chunk, r.tree);
    plan->route = r;
    return LQT_OK;
}

lqt_status lqt_submit(lqt_plan_t plan, const lqt_problem* prob, const lqt_outputs* out, uint64_t* ticket) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_submit: NULL plan");
    if (!prob || !out || !ticket) return fail(plan, LQT_EINVAL, "lqt_submit: NULL argument");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    lqt_status st = validate(plan, *prob, *out, 0);
    if (st != LQT_OK) return st;
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    st = serve_init(plan);
    if (st != LQT_OK) return st;
    (void)plan->core.pump(plan->ops);  // retire finished work first: it frees queue places
    const size_t need = serve_bytes(plan, *prob, *out);
    const uint64_t t = plan->next_ticket;
    const int code = plan->core.submit(t, serve_lane(plan, *prob), need, (size_t)t);
    if (code == LQT_ENOMEM)
        return fail(plan, LQT_ENOMEM, "lqt_submit: request needs %zu device bytes, the serving pool holds %zu", need,
                    plan->core.pool().size());
    if (code == LQT_EBUSY)
        return fail(plan, LQT_EBUSY, "lqt_submit: %zu requests queued or running (max %d)", plan->core.live(),
                    plan->desc.max_inflight);
    plan->payload[t] = PendingReq{*prob, *out};
    ++plan->next_ticket;
    *ticket = t;
    // a launch failure is the request's status (and that of its batch), read by lqt_poll
    (void)plan->core.pump(plan->ops);
    plan->wake.notify_all();
    return LQT_OK;
}

lqt_status lqt_poll(lqt_plan_t plan, uint64_t ticket) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_poll: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    if (!plan->core.known(ticket))
        return fail(plan, LQT_EINVAL, "lqt_poll: unknown ticket %llu", (unsigned long long)ticket);
    if (plan->core.pending(ticket)) {
        if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
        (void)plan->core.pump(plan->ops);
    }
    int code = 0;
    if (!plan->core.poll(ticket, code)) return LQT_EAGAIN;
    return (lqt_status)code;
}

lqt_status lqt_serve_stats_read(lqt_plan_t plan, lqt_serve_stats* out) {
    if (!plan || !out) return fail(plan, LQT_EINVAL, "lqt_serve_stats_read: NULL argument");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    const lqt::ServeCounters& c = plan->core.counters();
    *out = lqt_serve_stats{};
    out->submitted = c.submitted;
    out->completed = c.completed;
    out->batches = c.batches;
    out->queued = plan->core.queued();
    out->running_batches = c.running_batches;
    out->max_running_batches = c.max_running_batches;
    out->max_batch = c.max_batch;
    out->pool_bytes = plan->core.pool().size();
    out->pool_in_use = plan->core.pool().in_use();
    out->pool_peak = c.pool_peak;
    return LQT_OK;
}

lqt_status lqt_nl_iterate(lqt_plan_t plan, const lqt_nl_problem* prob, int32_t iterations, void* x, void* u,
                          double* change, int32_t* status, void* stream) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_nl_iterate: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (!prob || !x || !u) return fail(plan, LQT_EINVAL, "lqt_nl_iterate: NULL problem or trajectory");
    if (prob->model != LQT_NL_UNICYCLE) return fail(plan, LQT_EINVAL, "lqt_nl_iterate: unknown model %d",
                                                    (int)prob->model);
    if (iterations < 1) return fail(plan, LQT_EINVAL, "lqt_nl_iterate: iterations must be >= 1 (got %d)",
                                    iterations);
    if (prob->per_step & ~(uint32_t)(LQT_PS_H | LQT_PS_X | LQT_PS_U))
        return fail(plan, LQT_EINVAL, "lqt_nl_iterate: only H, X and U may carry a time axis (per_step=0x%x)",
                    prob->per_step);
    if (!prob->dt) return fail(plan, LQT_EINVAL, "lqt_nl_iterate: dt is NULL");
    const int n = 4, m = 2;
    const int64_t T = prob->T;
    // the instance of every round: the linearised model (workspace) and the cost
    lqt_problem p{};
    p.nx = n; p.nu = m; p.ny = prob->ny; p.nyT = prob->nyT; p.T = T;
    p.per_step = prob->per_step | LQT_PS_F | LQT_PS_c | LQT_PS_L;
    p.H = prob->H; p.X = prob->X; p.U = prob->U; p.r = prob->r;
    p.HT = prob->HT; p.XT = prob->XT; p.rT = prob->rT; p.x0 = prob->x0;
    lqt_outputs o{};
    o.x = x;
    o.u = u;
    // validation with stand-in model pointers (replaced below)
    p.F = p.L = p.c = prob->x0;
    lqt_status st = validate(plan, p, o, 0);
    if (st != LQT_OK) return st;
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    if (!plan->graphs || plan->prof.on) return nl_enqueue(plan, plan->nl, plan->main, *prob, p, o, iterations, x, u,
                                                          change, status, s);
    std::string key("nl");
    sig_nl(key, *prob);
    sig_val(key, iterations);
    void* ptrs[4] = {x, u, change, status};
    sig_add(key, ptrs, sizeof ptrs);
    return graph_run(plan, key, s, [&](GraphEntry& e, hipStream_t gs) {
        return nl_enqueue(plan, e.nl, e.main, *prob, p, o, iterations, x, u, change, status, gs);
    });
}

lqt_status lqt_fs_solve(lqt_plan_t plan, const lqt_fs_problem* prob, const lqt_fs_outputs* out, void* stream) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_fs_solve: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->err.clear();
    if (!prob || !out) return fail(plan, LQT_EINVAL, "lqt_fs_solve: NULL problem or outputs");
    const int D = prob->nstates, Du = prob->ncontrols;
    if (D < 1 || D > 32 || Du < 1 || Du > 32)
        return fail(plan, LQT_EINVAL, "lqt_fs_solve: states %d and controls %d must be in 1..32", D, Du);
    if (prob->T < 1) return fail(plan, LQT_EINVAL, "lqt_fs_solve: T must be >= 1 (got %lld)", (long long)prob->T);
    if (prob->x0 < 0 || prob->x0 >= D) return fail(plan, LQT_EINVAL, "lqt_fs_solve: x0=%d outside 0..%d", prob->x0,
                                                   D - 1);
    if (prob->per_step & ~(uint32_t)(LQT_FS_NEXT | LQT_FS_COST))
        return fail(plan, LQT_EINVAL, "lqt_fs_solve: unknown per_step bits 0x%x", prob->per_step);
    if (!prob->next || !prob->cost || !prob->cost_T)
        return fail(plan, LQT_EINVAL, "lqt_fs_solve: a table pointer is NULL");
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    lqt::FsArgs a{};
    a.next = prob->next; a.cost = prob->cost; a.cost_T = prob->cost_T;
    a.T = prob->T; a.D = D; a.Du = Du; a.per_step = prob->per_step; a.x0 = prob->x0;
    lqt::fs_shape(a.T, a.B, a.NC, a.NG);
    const size_t DD = (size_t)D * D;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t oP = take((size_t)a.NC * DD * sizeof(double));
    const size_t oQ = take((size_t)a.NG * DD * sizeof(double));
    const size_t oG = take((size_t)(a.NG + 1) * D * sizeof(double));
    const size_t oC = take((size_t)(a.NC + 1) * D * sizeof(double));
    const size_t oN = take((size_t)a.T * D * sizeof(int32_t));
    const size_t oF = take((size_t)a.NC * D * sizeof(int32_t));
    const size_t oX = take((size_t)(a.NC + 1) * sizeof(int32_t));
    const size_t oU = take(out->u ? 0 : (size_t)a.T * D * sizeof(int32_t));
    const size_t oGF = take((size_t)a.NG * D * sizeof(int32_t));
    const size_t oGX = take((size_t)(a.NG + 1) * sizeof(int32_t));
    lqt_status st = ensure_ws(plan, plan->fs, off);
    if (st != LQT_OK) return st;
    char* w = plan->fs.ws;
    a.P = (double*)(w + oP); a.Q = (double*)(w + oQ); a.gval = (double*)(w + oG); a.cval = (double*)(w + oC);
    a.nxt = (int32_t*)(w + oN); a.phi = (int32_t*)(w + oF); a.xs = (int32_t*)(w + oX);
    a.gphi = (int32_t*)(w + oGF); a.gxs = (int32_t*)(w + oGX);
    a.V = out->V;
    a.ulaw = out->u ? out->u : (int32_t*)(w + oU);
    a.x = out->x; a.ux = out->ux; a.status = out->status;
    lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
    hipError_t e = lqt::fs_solve(a, (hipStream_t)stream, plan->prof.on ? &hook : nullptr);
    if (e != hipSuccess) return fail(plan, LQT_EHIP, "finite-state launch failed: %s", hipGetErrorString(e));
    return LQT_OK;
}

lqt_status lqt_destroy(lqt_plan_t plan) {
    if (!plan) return LQT_OK;
    if (plan->progress.joinable()) {
        {
            std::lock_guard<std::recursive_mutex> lk(plan->mu);
            plan->stop = true;
        }
        plan->wake.notify_all();
        plan->progress.join();
    }
    (void)hipSetDevice(plan->desc.device);
    (void)hipDeviceSynchronize();
    graph_clear(plan);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    for (Slot& s : plan->slots) slot_release(s);
    if (plan->pool) (void)hipFree(plan->pool);
    if (plan->has_side) {
        (void)hipStreamDestroy(plan->side.side);
        (void)hipEventDestroy(plan->side.fork);
        (void)hipEventDestroy(plan->side.join);
    }
    for (auto& r : plan->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : plan->prof.pool) (void)hipEventDestroy(e);
    arena_release(plan->main);
    arena_release(plan->nl);
    arena_release(plan->fs);
    delete plan;
    return LQT_OK;
}

lqt_status lqt_profile_enable(lqt_plan_t plan, int32_t enable) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_profile_enable: NULL plan");
    plan->prof.on = enable != 0;
    return LQT_OK;
}

lqt_status lqt_profile_select(lqt_plan_t plan, const char* stage) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_profile_select: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    plan->prof.only = stage ? stage : "";
    return LQT_OK;
}

int32_t lqt_profile_read(lqt_plan_t plan, lqt_stage_time* out, int32_t max) {
    if (!plan) return -(int32_t)fail(nullptr, LQT_EINVAL, "lqt_profile_read: NULL plan");
    std::lock_guard<std::recursive_mutex> lk(plan->mu);
    Profiler& P = plan->prof;
    for (auto& r : P.pending) {
        if (hipEventSynchronize(r.b) != hipSuccess) return -(int32_t)fail(plan, LQT_EHIP, "event sync failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        auto it = P.acc.find(r.name);
        if (it == P.acc.end()) {
            P.names.push_back(r.name);
            P.acc[r.name] = {1, (double)ms};
        } else {
            it->second.first += 1;
            it->second.second += ms;
        }
        P.pool.push_back(r.a);
        P.pool.push_back(r.b);
    }
    P.pending.clear();
    int32_t n = 0;
    for (const std::string& nm : P.names) {
        if (n >= max) break;
        auto& v = P.acc[nm];
        out[n].name = nm.c_str();  // names vector owns the strings
        out[n].launches = v.first;
        out[n].total_ms = v.second;
        v = {0, 0.0};
        ++n;
    }
    return n;
}

const char* lqt_last_error(lqt_plan_t plan) {
    if (!plan) return g_create_error.c_str();
    return plan->err.c_str();
}

}  // extern "C"
