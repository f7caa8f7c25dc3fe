// Host runtime of the LQT solver: plans, validation, workspace, launches,
// status and the asynchronous submit/poll interface.  Implements include/lqt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lqt.h"
#include "lqt_internal.hpp"

namespace {

constexpr int kMaxNx = 32;         // largest state dimension of this build's kernels
constexpr int kWaveMaxN = 32;      // wavefront path: n, m, p, pT up to this
constexpr int64_t kSmallMinT = 8192;  // lane-per-element path for long n <= 4 instances

// Path of an instance: a function of the instance alone (never of the batch),
// so a result is the same alone and in any mix.  LQT_PATH=small|wave forces
// one path where it applies (tests).
enum class Path { Small, Wave };

Path path_of(const lqt_problem& p) {
    int force = 0;
    if (const char* e = getenv("LQT_PATH")) force = !strcmp(e, "small") ? 1 : (!strcmp(e, "wave") ? 2 : 0);
    const bool small_ok = lqt::small_supported(p.nx, p.nu);
    if (force == 1 && small_ok) return Path::Small;
    if (force == 2) return Path::Wave;
    return (small_ok && p.T >= kSmallMinT) ? Path::Small : Path::Wave;
}

int wave_chunk(int64_t T) {
    if (const char* e = getenv("LQT_WCHUNK")) {
        int b = atoi(e);
        if (b >= 1 && b <= 4096) return b;
    }
    int64_t b = (T + 63) / 64;
    return (int)std::max<int64_t>(16, std::min<int64_t>(256, b));
}

thread_local std::string g_create_error;

struct Request {
    uint64_t ticket;
    hipEvent_t done;
    int32_t* status_dev;  // plan-owned per-request status word
    int32_t* user_status;
};

}  // namespace

struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    bool on = false;
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
        p->cur_a = p->get();
        p->cur_name = name;
        (void)hipEventRecord(p->cur_a, s);
    }
    static void end(void* ctx, hipStream_t s) {
        Profiler* p = (Profiler*)ctx;
        hipEvent_t b = p->get();
        (void)hipEventRecord(b, s);
        p->pending.push_back({p->cur_name, p->cur_a, b});
    }
};

struct lqt_plan_s {
    lqt_plan_desc desc{};
    Profiler prof;
    char* ws = nullptr;
    size_t ws_cap = 0;
    std::string err;
    hipStream_t serve_stream = nullptr;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, Request> inflight;
    std::vector<int32_t*> free_status;
    // wavefront path: pinned host copy of the instance table and the event of
    // its last upload (the buffer is reused only after that copy finished)
    lqt::GInst* ginst_host = nullptr;
    size_t ginst_cap = 0;
    hipEvent_t ginst_done = nullptr;
};

namespace {

lqt_status fail(lqt_plan_t p, lqt_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

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

int chunk_length(int64_t T) {
    if (const char* e = getenv("LQT_CHUNK")) {
        int b = atoi(e);
        if (b >= 1 && b <= 1024) return b;
    }
    // About 64K lanes (one wavefront per SIMD on 256 CUs), at most 16 steps
    // per lane; measured best for the n = 4 pipeline at T = 1e6.
    int64_t b = (T + 65535) / 65536;
    return (int)std::max<int64_t>(1, std::min<int64_t>(16, b));
}

struct Layout {
    size_t cst, der, lane_el, wave_val, lane_aff, wave_x, K, d, total;
    int64_t NC;
    int B, NG;
};

Layout layout_for(const lqt_problem& p, bool need_K, bool need_d) {
    using namespace lqt;
    Layout L{};
    const int n = p.nx, m = p.nu;
    L.B = chunk_length(p.T);
    L.NC = (p.T + L.B - 1) / L.B;
    L.NG = (int)((L.NC + 63) / 64);
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
    L.K = take(need_K ? (size_t)p.T * m * n : 0);
    L.d = take(need_d ? (size_t)p.T * m : 0);
    L.total = off;
    return L;
}

lqt_status validate(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o, int idx) {
    if (p.nx < 1 || p.nu < 1 || p.ny < 1 || p.nyT < 1)
        return fail(plan, LQT_EINVAL, "instance %d: dimensions must be >= 1 (nx=%d nu=%d ny=%d nyT=%d)", idx,
                    p.nx, p.nu, p.ny, p.nyT);
    if (p.T < 1) return fail(plan, LQT_EINVAL, "instance %d: T must be >= 1 (got %lld)", idx, (long long)p.T);
    if (p.nx > plan->desc.max_nx || p.nu > plan->desc.max_nu)
        return fail(plan, LQT_EINVAL, "instance %d: nx=%d nu=%d exceed the plan's max_nx=%d max_nu=%d", idx, p.nx,
                    p.nu, plan->desc.max_nx, plan->desc.max_nu);
    if (path_of(p) == Path::Wave && std::max(std::max(p.nx, p.nu), std::max(p.ny, p.nyT)) > kWaveMaxN)
        return fail(plan, LQT_ENOTSUP, "instance %d: dimensions nx=%d nu=%d ny=%d nyT=%d exceed %d", idx, p.nx,
                    p.nu, p.ny, p.nyT, kWaveMaxN);
    if (p.per_step & ~63u) return fail(plan, LQT_EINVAL, "instance %d: unknown per_step bits 0x%x", idx, p.per_step);
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

lqt_status ensure_ws(lqt_plan_t plan, size_t bytes) {
    if (bytes <= plan->ws_cap) return LQT_OK;
    if (plan->desc.hbm_budget_bytes && bytes > plan->desc.hbm_budget_bytes)
        return fail(plan, LQT_ENOMEM, "workspace of %zu bytes exceeds the plan budget of %zu bytes", bytes,
                    plan->desc.hbm_budget_bytes);
    if (plan->ws) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(plan->ws) != hipSuccess)
            return fail(plan, LQT_EHIP, "hipFree of the old workspace failed");
        plan->ws = nullptr;
        plan->ws_cap = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(plan, LQT_ENOMEM, "hipMalloc of %zu workspace bytes failed", bytes);
    }
    plan->ws = (char*)p;
    plan->ws_cap = bytes;
    return LQT_OK;
}

lqt_status launch_one(lqt_plan_t plan, const lqt_problem& p, const lqt_outputs& o, hipStream_t s,
                      int32_t* status_override) {
    const bool fwd = o.x || o.u;
    const bool need_K = !o.K, need_d = !o.d;
    Layout L = layout_for(p, need_K, need_d);
    lqt_status st = ensure_ws(plan, L.total);
    if (st != LQT_OK) return st;
    lqt::SmallArgs a{};
    a.F = p.F; a.c = p.c; a.L = p.L; a.U = p.U; a.H = p.H; a.X = p.X; a.r = p.r;
    a.HT = p.HT; a.XT = p.XT; a.rT = p.rT; a.x0 = p.x0;
    a.T = p.T; a.n = p.nx; a.m = p.nu; a.p = p.ny; a.pT = p.nyT;
    a.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
    a.S = (double*)o.S; a.v = (double*)o.v;
    a.K = o.K ? (double*)o.K : (double*)(plan->ws + L.K);
    a.d = o.d ? (double*)o.d : (double*)(plan->ws + L.d);
    a.x = (double*)o.x; a.u = (double*)o.u;
    a.status = status_override ? status_override : o.status;
    a.cst = (double*)(plan->ws + L.cst);
    a.der = (double*)(plan->ws + L.der);
    a.lane_el = (double*)(plan->ws + L.lane_el);
    a.wave_val = (double*)(plan->ws + L.wave_val);
    a.lane_aff = (double*)(plan->ws + L.lane_aff);
    a.wave_x = (double*)(plan->ws + L.wave_x);
    a.NC = L.NC; a.B = L.B; a.NG = L.NG;
    a.want_fwd = fwd ? 1 : 0;
    lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
    hipError_t e = lqt::small_solve(a, s, plan->prof.on ? &hook : nullptr);
    if (e != hipSuccess) return fail(plan, LQT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
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
        return fail(nullptr, LQT_ENOTSUP, "lqt_plan: max_nx=%d exceeds this build's limit %d", desc->max_nx, kMaxNx);
    if (desc->prec != LQT_PREC_FP64)
        return fail(nullptr, LQT_ENOTSUP, "lqt_plan: precision %d is not provided by this build", (int)desc->prec);
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
    if (p->desc.max_inflight <= 0) p->desc.max_inflight = 64;
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
                    need = std::max(need, layout_for(probe, true, true).total);
                }
        // and for one wavefront-path instance of the largest dimensions
        {
            const int64_t B = wave_chunk(desc->max_steps);
            const int64_t NC = (desc->max_steps + B - 1) / B;
            const size_t w = (size_t)lqt::wave_inst_ws_doubles(desc->max_nx, desc->max_nu, desc->max_nx, NC) * 8 +
                             (size_t)desc->max_steps * (desc->max_nu * desc->max_nx + desc->max_nu) * 8 + 4096;
            need = std::max(need, w);
        }
        lqt_status st = ensure_ws(p, need);
        if (st != LQT_OK) {
            g_create_error = p->err;
            delete p;
            return st;
        }
    }
    *out = p;
    return LQT_OK;
}

}  // extern "C"

namespace {

// Solve a set of instances on stream s.  status_override (if not null) gives
// a per-instance device status word used instead of outs[i].status.
lqt_status solve_all(lqt_plan_t plan, const lqt_problem* probs, const lqt_outputs* outs, int32_t count,
                     hipStream_t s, int32_t* const* status_override) {
    // partition by path; wavefront instances ordered by size class
    std::vector<int> small, wave;
    for (int i = 0; i < count; ++i) (path_of(probs[i]) == Path::Small ? small : wave).push_back(i);
    auto cls = [&](int i) {
        const lqt_problem& p = probs[i];
        return lqt::tile_class(std::max(std::max(p.nx, p.nu), std::max(p.ny, p.nyT)));
    };
    std::stable_sort(wave.begin(), wave.end(), [&](int a, int b) { return cls(a) < cls(b); });
    // workspace: [small-path region (largest small instance)] [wave region]
    size_t small_need = 0;
    for (int i : small) small_need = std::max(small_need, layout_for(probs[i], !outs[i].K, !outs[i].d).total);
    small_need = align_up(small_need);
    size_t wave_need = 0;
    std::vector<int64_t> ws_off(wave.size()), kd_off(wave.size());
    for (size_t j = 0; j < wave.size(); ++j) {
        const lqt_problem& p = probs[wave[j]];
        const int B = wave_chunk(p.T);
        const int64_t NC = (p.T + B - 1) / B;
        ws_off[j] = (int64_t)wave_need;
        wave_need = align_up(wave_need + (size_t)lqt::wave_inst_ws_doubles(p.nx, p.nu, p.ny, NC) * sizeof(double));
        kd_off[j] = (int64_t)wave_need;
        const lqt_outputs& o = outs[wave[j]];
        if (!o.K || !o.d)
            wave_need = align_up(wave_need + (size_t)p.T * (p.nu * p.nx + p.nu) * sizeof(double));
    }
    const size_t inst_bytes = align_up(wave.size() * sizeof(lqt::GInst));
    const size_t total = small_need + (wave.empty() ? 0 : wave_need + inst_bytes);
    lqt_status st = ensure_ws(plan, total);
    if (st != LQT_OK) return st;
    for (int i : small) {
        st = launch_one(plan, probs[i], outs[i], s, status_override ? status_override[i] : nullptr);
        if (st != LQT_OK) return st;
    }
    if (wave.empty()) return LQT_OK;
    if (plan->ginst_cap < wave.size()) {
        if (plan->ginst_done) (void)hipEventSynchronize(plan->ginst_done);
        if (plan->ginst_host) (void)hipHostFree(plan->ginst_host);
        plan->ginst_host = nullptr;
        plan->ginst_cap = 0;
        if (hipHostMalloc((void**)&plan->ginst_host, wave.size() * sizeof(lqt::GInst), 0) != hipSuccess)
            return fail(plan, LQT_ENOMEM, "pinned instance table allocation failed");
        plan->ginst_cap = wave.size();
    } else if (plan->ginst_done) {
        (void)hipEventSynchronize(plan->ginst_done);  // previous upload has left the buffer
    }
    char* wbase = plan->ws + small_need;
    std::vector<char> want_fwd_c(wave.size(), 0);
    int64_t chunk0 = 0;
    for (size_t j = 0; j < wave.size(); ++j) {
        if (j > 0 && cls(wave[j]) != cls(wave[j - 1])) chunk0 = 0;  // each class numbers its own chunks
        const lqt_problem& p = probs[wave[j]];
        const lqt_outputs& o = outs[wave[j]];
        lqt::GInst& g = plan->ginst_host[j];
        g = lqt::GInst{};
        g.F = p.F; g.c = p.c; g.L = p.L; g.U = p.U; g.H = p.H; g.X = p.X; g.r = p.r;
        g.HT = p.HT; g.XT = p.XT; g.rT = p.rT; g.x0 = p.x0;
        g.S = (double*)o.S; g.v = (double*)o.v; g.x = (double*)o.x; g.u = (double*)o.u;
        double* kd = (double*)(wbase + kd_off[j]);
        g.K = o.K ? (double*)o.K : kd;
        g.d = o.d ? (double*)o.d : kd + (size_t)p.T * p.nu * p.nx;
        g.status = status_override ? status_override[wave[j]] : o.status;
        g.T = p.T; g.n = p.nx; g.m = p.nu; g.p = p.ny; g.pT = p.nyT;
        g.per_step = p.per_step & (p.c ? 63u : (63u & ~(uint32_t)LQT_PS_c));
        g.B = wave_chunk(p.T);
        g.NC = (p.T + g.B - 1) / g.B;
        g.chunk0 = chunk0;
        chunk0 += g.NC;
        g.ws = (double*)(wbase + ws_off[j]);
        // forward pass only if some instance of the launch wants it; instances
        // without x and u still get their (cheap) roll-out into K/d-free paths
        want_fwd_c[j] = (o.x || o.u) ? 1 : 0;
    }
    lqt::GInst* d_inst = (lqt::GInst*)(wbase + wave_need);
    if (hipMemcpyAsync(d_inst, plan->ginst_host, wave.size() * sizeof(lqt::GInst), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return fail(plan, LQT_EHIP, "instance table upload failed");
    if (!plan->ginst_done && hipEventCreateWithFlags(&plan->ginst_done, hipEventDisableTiming) != hipSuccess)
        return fail(plan, LQT_EHIP, "event creation failed");
    (void)hipEventRecord(plan->ginst_done, s);
    lqt::StageHook hook{&Profiler::begin, &Profiler::end, &plan->prof};
    for (size_t j0 = 0; j0 < wave.size();) {
        size_t j1 = j0;
        int64_t nch = 0;
        bool fwd = false;
        while (j1 < wave.size() && cls(wave[j1]) == cls(wave[j0])) {
            nch += plan->ginst_host[j1].NC;
            fwd = fwd || want_fwd_c[j1];
            ++j1;
        }
        hipError_t e = lqt::tile_solve(cls(wave[j0]), d_inst + j0, (int)(j1 - j0), nch, fwd, s,
                                       plan->prof.on ? &hook : nullptr);
        if (e != hipSuccess) return fail(plan, LQT_EHIP, "wavefront-path launch failed: %s", hipGetErrorString(e));
        j0 = j1;
    }
    return LQT_OK;
}

}  // namespace

extern "C" {

lqt_status lqt_solve(lqt_plan_t plan, const lqt_problem* probs, const lqt_outputs* outs, int32_t count,
                     void* stream) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_solve: NULL plan");
    plan->err.clear();
    if (count < 0 || (count > 0 && (!probs || !outs))) return fail(plan, LQT_EINVAL, "lqt_solve: bad count/arrays");
    for (int i = 0; i < count; ++i) {
        lqt_status st = validate(plan, probs[i], outs[i], i);
        if (st != LQT_OK) return st;
    }
    if (count == 0) return LQT_OK;
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    return solve_all(plan, probs, outs, count, (hipStream_t)stream, nullptr);
}

lqt_status lqt_submit(lqt_plan_t plan, const lqt_problem* prob, const lqt_outputs* out, uint64_t* ticket) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_submit: NULL plan");
    if (!prob || !out || !ticket) return fail(plan, LQT_EINVAL, "lqt_submit: NULL argument");
    plan->err.clear();
    lqt_status st = validate(plan, *prob, *out, 0);
    if (st != LQT_OK) return st;
    if ((int)plan->inflight.size() >= plan->desc.max_inflight)
        return fail(plan, LQT_EBUSY, "lqt_submit: %zu requests in flight (max %d)", plan->inflight.size(),
                    plan->desc.max_inflight);
    Layout L = layout_for(*prob, !out->K, !out->d);
    if (plan->desc.hbm_budget_bytes && L.total > plan->desc.hbm_budget_bytes)
        return fail(plan, LQT_ENOMEM, "lqt_submit: request needs %zu bytes, budget %zu", L.total,
                    plan->desc.hbm_budget_bytes);
    if (hipSetDevice(plan->desc.device) != hipSuccess) return fail(plan, LQT_EHIP, "hipSetDevice failed");
    if (!plan->serve_stream && hipStreamCreateWithFlags(&plan->serve_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(plan, LQT_EHIP, "hipStreamCreate failed");
    Request r{};
    if (!plan->free_status.empty()) {
        r.status_dev = plan->free_status.back();
        plan->free_status.pop_back();
    } else if (hipMalloc(&r.status_dev, sizeof(int32_t)) != hipSuccess) {
        return fail(plan, LQT_ENOMEM, "lqt_submit: status allocation failed");
    }
    int32_t* ovr[1] = {r.status_dev};
    st = solve_all(plan, prob, out, 1, plan->serve_stream, ovr);
    if (st == LQT_OK && out->status)
        if (hipMemcpyAsync(out->status, r.status_dev, sizeof(int32_t), hipMemcpyDeviceToDevice,
                           plan->serve_stream) != hipSuccess)
            st = fail(plan, LQT_EHIP, "status copy failed");
    if (st == LQT_OK && (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess ||
                         hipEventRecord(r.done, plan->serve_stream) != hipSuccess))
        st = fail(plan, LQT_EHIP, "event record failed");
    if (st != LQT_OK) {
        plan->free_status.push_back(r.status_dev);
        return st;
    }
    r.ticket = plan->next_ticket++;
    r.user_status = out->status;
    plan->inflight[r.ticket] = r;
    *ticket = r.ticket;
    return LQT_OK;
}

lqt_status lqt_poll(lqt_plan_t plan, uint64_t ticket) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_poll: NULL plan");
    auto it = plan->inflight.find(ticket);
    if (it == plan->inflight.end()) return fail(plan, LQT_EINVAL, "lqt_poll: unknown ticket %llu",
                                                (unsigned long long)ticket);
    hipError_t q = hipEventQuery(it->second.done);
    if (q == hipErrorNotReady) {
        (void)hipGetLastError();
        return LQT_EAGAIN;
    }
    if (q != hipSuccess) return fail(plan, LQT_EHIP, "lqt_poll: event query failed");
    int32_t code = 0;
    if (hipMemcpy(&code, it->second.status_dev, sizeof code, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(plan, LQT_EHIP, "lqt_poll: status read failed");
    (void)hipEventDestroy(it->second.done);
    plan->free_status.push_back(it->second.status_dev);
    plan->inflight.erase(it);
    return (lqt_status)code;
}

lqt_status lqt_destroy(lqt_plan_t plan) {
    if (!plan) return LQT_OK;
    (void)hipSetDevice(plan->desc.device);
    (void)hipDeviceSynchronize();
    for (auto& kv : plan->inflight) {
        (void)hipEventDestroy(kv.second.done);
        (void)hipFree(kv.second.status_dev);
    }
    for (int32_t* s : plan->free_status) (void)hipFree(s);
    if (plan->serve_stream) (void)hipStreamDestroy(plan->serve_stream);
    for (auto& r : plan->prof.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : plan->prof.pool) (void)hipEventDestroy(e);
    if (plan->ginst_done) (void)hipEventDestroy(plan->ginst_done);
    if (plan->ginst_host) (void)hipHostFree(plan->ginst_host);
    if (plan->ws) (void)hipFree(plan->ws);
    delete plan;
    return LQT_OK;
}

lqt_status lqt_profile_enable(lqt_plan_t plan, int32_t enable) {
    if (!plan) return fail(nullptr, LQT_EINVAL, "lqt_profile_enable: NULL plan");
    plan->prof.on = enable != 0;
    return LQT_OK;
}

int32_t lqt_profile_read(lqt_plan_t plan, lqt_stage_time* out, int32_t max) {
    if (!plan) return -(int32_t)fail(nullptr, LQT_EINVAL, "lqt_profile_read: NULL plan");
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
