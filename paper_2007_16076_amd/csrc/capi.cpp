// Host runtime and C ABI of libgapd.so (declared in include/gapd.h).
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "gapd_internal.h"
#include "capi_internal.h"
#include "gapd.h"

using namespace gapd;

namespace gapd {

thread_local std::string g_create_error;

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

int env_int(const char *name, int dflt) {
    const char *s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}

// Checks of the image and options that need no device (include/gapd.h, Limits).
int validate_image(const uint8_t *img, int H, int W, int C, int conn, int wmode, std::string &why) {
    if (!img) { why = "image is null"; return GAPD_EINVAL; }
    if (H < 1 || W < 1 || H > kMaxLine || W > kMaxLine) { why = "H and W must be in [1, 512]"; return GAPD_EINVAL; }
    if (conn != GAPD_CONN4 && conn != GAPD_CONN8) { why = "conn must be 4 or 8"; return GAPD_EINVAL; }
    if (wmode == GAPD_W_SUM) {
        if (C != 1) { why = "GAPD_W_SUM needs C == 1"; return GAPD_EINVAL; }
    } else if (wmode == GAPD_W_1PL1) {
        if (C < 1 || C > 256) { why = "GAPD_W_1PL1 needs 1 <= C <= 256"; return GAPD_EINVAL; }
    } else {
        why = "unknown weight_mode";
        return GAPD_EINVAL;
    }
    // Largest and smallest edge weight, by the same definition the kernels use.
    int64_t wmax = 0, wmin = INT64_MAX;
    auto w = [&](int p, int q) -> int64_t {
        if (wmode == GAPD_W_SUM) return (int64_t)img[p] + img[q];
        int64_t s = 1;
        for (int b = 0; b < C; ++b) s += std::abs((int)img[(size_t)p * C + b] - (int)img[(size_t)q * C + b]);
        return s;
    };
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int v = y * W + x;
            int64_t e[4];
            int n = 0;
            if (x + 1 < W) e[n++] = w(v, v + 1);
            if (y + 1 < H) e[n++] = w(v, v + W);
            if (conn == 8 && y + 1 < H && x + 1 < W) e[n++] = w(v, v + W + 1);
            if (conn == 8 && y + 1 < H && x >= 1) e[n++] = w(v, v + W - 1);
            for (int k = 0; k < n; ++k) { wmax = std::max(wmax, e[k]); wmin = std::min(wmin, e[k]); }
        }
    if (wmin < 1 && H * W > 1) { why = "an edge weighs 0 (two neighbouring zero pixels under GAPD_W_SUM)"; return GAPD_EINVAL; }
    const int64_t hops = conn == 4 ? (int64_t)H + W - 2 : (int64_t)std::max(H, W) - 1;
    if (hops * wmax >= kDistLimit) { why = "distances could reach 2^27"; return GAPD_ERANGE; }
    return GAPD_OK;
}

int max_rounds_for(int N) {
    const int cap = env_int("GAPD_MAX_ROUNDS", 512);
    return std::max(1, std::min(cap, N + 1));
}

StepGraph::~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
}

bool StepGraph::capture(int n, const std::function<hipError_t(hipStream_t)> &step) {
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { cs = nullptr; return false; }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    hipError_t le = hipSuccess;
    for (int i = 0; i < n && le == hipSuccess; ++i) le = step(cs);
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    (void)hipGetLastError();  // a failed capture leaves no error for later calls
    if (le != hipSuccess || ce != hipSuccess || !graph) return false;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        exec = nullptr;
        (void)hipGetLastError();
        return false;
    }
    return true;
}

bool use_step_graphs() { return env_int("GAPD_FR_GRAPH", 1) != 0; }

}  // namespace gapd

struct gapd_ctx {
    int H = 0, W = 0, C = 0, N = 0, conn = 4, wmode = 0;
    int device = 0;             // the device current at gapd_create
    hipStream_t stream = nullptr;
    void *dev = nullptr;
    uint8_t *img_dev = nullptr;
    GImg g{};
    FrCtl *ctl = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int max_rounds = 512;
    bool poisoned = false;
    std::string err;
};

namespace {

int fail(gapd_ctx *c, int st, const std::string &why) {
    if (c) c->err = why;
    return st;
}

int dev_fail(gapd_ctx *c, hipError_t e, const char *where) {
    c->poisoned = true;
    c->err = std::string(where) + ": " + hipGetErrorString(e);
    return GAPD_EDEVICE;
}

#define HIP_OR_FAIL(c, expr)                              \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return dev_fail(c, _e, #expr); \
    } while (0)

int ctx_check(gapd_ctx *c) {
    if (!c) return GAPD_EINVAL;
    if (c->poisoned) return fail(c, GAPD_EDEVICE, "context poisoned by an earlier device error");
    return GAPD_OK;
}

}  // namespace

extern "C" {

const char *gapd_strerror(int st) {
    switch (st) {
        case GAPD_OK: return "ok";
        case GAPD_PENDING: return "pending";
        case GAPD_EINVAL: return "invalid argument";
        case GAPD_ENOMEM: return "not enough memory";
        case GAPD_EDEVICE: return "device error";
        case GAPD_ERANGE: return "distance range exceeded";
        case GAPD_ENOCONV: return "propagation did not converge";
        case GAPD_EBUSY: return "busy";
        case GAPD_ENOTFOUND: return "not found";
        default: return "unknown status";
    }
}

const char *gapd_last_error(gapd_ctx *ctx) {
    if (!ctx) return gapd::g_create_error.c_str();
    return ctx->err.c_str();
}

int gapd_create(const uint8_t *image, int H, int W, int C, int conn, int weight_mode, gapd_ctx **out) {
    if (!out) return GAPD_EINVAL;
    *out = nullptr;
    std::string why;
    int st = validate_image(image, H, W, C, conn, weight_mode, why);
    if (st != GAPD_OK) { g_create_error = why; return st; }
    gapd_ctx *c = new gapd_ctx();
    c->H = H; c->W = W; c->C = C; c->N = H * W; c->conn = conn; c->wmode = weight_mode;
    c->max_rounds = max_rounds_for(c->N);
    if (hipGetDevice(&c->device) != hipSuccess) { g_create_error = "no current device"; delete c; return GAPD_EDEVICE; }
    const size_t nimg = al256((size_t)c->N * C);
    const size_t nw = weight_block_bytes(H, W);
    const size_t bytes = nimg + nw + al256(sizeof(FrCtl));
    hipError_t e = hipMalloc(&c->dev, bytes);
    if (e != hipSuccess) { g_create_error = hipGetErrorString(e); delete c; return GAPD_ENOMEM; }
    c->img_dev = (uint8_t *)c->dev;
    GImgW w = weight_block_layout((char *)c->dev + nimg, H, W, conn);
    c->g = as_const(w);
    c->ctl = (FrCtl *)((char *)c->dev + nimg + nw);
    e = hipMemcpy(c->img_dev, image, (size_t)c->N * C, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset((char *)c->dev + nimg, 0, nw);
    if (e == hipSuccess) e = launch_prep(w, c->img_dev, C, weight_mode, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        (void)hipFree(c->dev);
        delete c;
        return GAPD_EDEVICE;
    }
    *out = c;
    return GAPD_OK;
}

int gapd_set_stream(gapd_ctx *ctx, void *hip_stream) {
    int st = ctx_check(ctx);
    if (st) return st;
    ctx->stream = (hipStream_t)hip_stream;
    return GAPD_OK;
}

int gapd_workspace_size(gapd_ctx *ctx, int mode, size_t *bytes) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!bytes) return fail(ctx, GAPD_EINVAL, "bytes is null");
    if (mode == GAPD_MODE_NAIVE) { *bytes = 0; return GAPD_OK; }
    if (mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA && mode != GAPD_MODE_TREE_FILL_SPIRAL)
        return fail(ctx, GAPD_EINVAL, "unknown mode");
    *bytes = fr_workspace_bytes(ctx->N, true);
    return GAPD_OK;
}

int gapd_set_workspace(gapd_ctx *ctx, void *dev_ptr, size_t bytes) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (dev_ptr && ((uintptr_t)dev_ptr & 255)) return fail(ctx, GAPD_EINVAL, "workspace must be 256-byte aligned");
    ctx->ws = dev_ptr;
    ctx->ws_bytes = dev_ptr ? bytes : 0;
    return GAPD_OK;
}

int gapd_sssp(gapd_ctx *ctx, const int32_t *sources, int K, int32_t *out) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (K < 0) return fail(ctx, GAPD_EINVAL, "K < 0");
    if (K == 0) return GAPD_OK;
    if (!sources || !out) return fail(ctx, GAPD_EINVAL, "null pointer");
    std::vector<int32_t> hs(K);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(hs.data(), sources, sizeof(int32_t) * K, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < K; ++k)
        if (hs[k] < 0 || hs[k] >= ctx->N) return fail(ctx, GAPD_EINVAL, "source id out of range");
    return run_rows(ctx->g, sources, 0, K, out, ctx->max_rounds, ctx->ctl, ctx->stream, ctx->err, ctx->poisoned);
}

namespace {

// The API mode of a rule (-1: the naive method).
int mode_of_rule(int rule) {
    return rule < 0 ? GAPD_MODE_NAIVE
                    : rule == kRuleFilling ? GAPD_MODE_TREE_FILL_FR
                                           : rule == kRuleExtrema ? GAPD_MODE_TREE_FILL_EXTREMA : GAPD_MODE_TREE_FILL_SPIRAL;
}

// One all-pairs call: the naive method (rule < 0) or a tree-based method,
// with the autotuned launch shapes of this image and method, or *force.
int all_pairs_impl(gapd_ctx *ctx, int rule, int h, const uint32_t *draws, int32_t *out, gapd_stats *stp,
                   const Tuning *force = nullptr) {
    const Tuning tune = force ? *force : tuning_for(tune_key(ctx->H, ctx->W, ctx->C, ctx->conn, mode_of_rule(rule)));
    gapd_stats local{};
    gapd_stats &s = stp ? *stp : local;
    s.n_prop = 0; s.n_prop_setup = 0; s.rounds = 0; s.centroid = -1; s.ms_total = 0; s.ms_setup = 0;
    s.ms_kernel = 0; s.ms_step_kernels = 0; s.ms_fill_kernels = 0; s.n_prop_speculative = 0; s.n_cache_hits = 0;
    s.rounds_speculative = 0;
    s.graph_replays = 0;
    int st = GAPD_OK;
    hipEvent_t e0, e1, e2;
    HIP_OR_FAIL(ctx, hipEventCreate(&e0));
    HIP_OR_FAIL(ctx, hipEventCreate(&e1));
    HIP_OR_FAIL(ctx, hipEventCreate(&e2));
    struct EvGuard {
        hipEvent_t a, b, c;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); }
    } guard{e0, e1, e2};
    HIP_OR_FAIL(ctx, hipEventRecord(e0, ctx->stream));
    if (rule < 0) {
        st = run_rows(ctx->g, nullptr, 0, ctx->N, out, ctx->max_rounds, ctx->ctl, ctx->stream, ctx->err,
                      ctx->poisoned, &s.rounds, &s.ms_kernel, tune.naive_pfw,
                      tune.naive_check1);
        HIP_OR_FAIL(ctx, hipEventRecord(e2, ctx->stream));
        HIP_OR_FAIL(ctx, hipEventSynchronize(e2));
        s.n_prop = ctx->N;
    } else {
        if (!tree_methods_fit(ctx->H, ctx->W))
            return fail(ctx, GAPD_EINVAL, "the tree methods need both image sides <= 192 (distance field in LDS)");
        const size_t need = fr_workspace_bytes(ctx->N, true);
        if (!ctx->ws || ctx->ws_bytes < need) return fail(ctx, GAPD_ENOMEM, "tree-method workspace missing or too small");
        FrState fs = fr_workspace_layout(ctx->ws, ctx->N, true);
        fs.H = ctx->g.H;
        fs.W = ctx->g.W;
        fs.rule = rule;
        fs.rep_h = h;
        fs.draws = draws;
        fs.spec_cap = tune.spec_cap;
        if (rule == kRuleSpiral) fs.cache = nullptr;  // no speculation on random draws
        fs.D = out;
        fs.seq_out = s.sources_out;
        fs.filled_out = s.filled_out;
        fs.trace = s.step_trace;
        if (fs.trace)
            HIP_OR_FAIL(ctx, hipMemsetAsync(fs.trace, 0, sizeof(int64_t) * kTraceFields * (size_t)ctx->N, ctx->stream));
        FrCtl hc{};
        float kt[2] = {0.f, 0.f};
        st = run_filling_rate(ctx->g, fs, ctx->max_rounds, ctx->stream, e1, hc, ctx->err, ctx->poisoned,
                              s.time_kernels ? kt : nullptr, &s.graph_replays, tune);
        s.ms_step_kernels = kt[0];
        s.ms_fill_kernels = kt[1];
        HIP_OR_FAIL(ctx, hipEventRecord(e2, ctx->stream));
        HIP_OR_FAIL(ctx, hipEventSynchronize(e2));
        s.n_prop = hc.n_prop;
        s.rounds = hc.rounds;
        s.n_prop_speculative = hc.spec_props;
        s.n_cache_hits = hc.spec_hits;
        s.rounds_speculative = hc.spec_rounds;
        if (rule != kRuleSpiral) {
            s.n_prop_setup = 2;
            s.centroid = hc.centroid;
        }
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) s.ms_setup = ms;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e2) == hipSuccess) s.ms_total = ms;
    return st;
}

}  // namespace

int gapd_all_pairs(gapd_ctx *ctx, int mode, int32_t *out, gapd_stats *stp) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!out) return fail(ctx, GAPD_EINVAL, "out is null");
    if (mode == GAPD_MODE_TREE_FILL_SPIRAL)
        return fail(ctx, GAPD_EINVAL, "the spiral methods take draws: use gapd_all_pairs_spiral");
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return fail(ctx, GAPD_EINVAL, "unknown mode");
    const int rule = mode == GAPD_MODE_NAIVE ? -1 : mode == GAPD_MODE_TREE_FILL_FR ? kRuleFilling : kRuleExtrema;
    return all_pairs_impl(ctx, rule, 0, nullptr, out, stp);
}

int gapd_autotune(gapd_ctx *ctx, int mode, int32_t *out, gapd_tuning *best) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!out) return fail(ctx, GAPD_EINVAL, "out is null");
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return fail(ctx, GAPD_EINVAL, "only the naive, filling-rate and extrema modes are tuned");
    const int rule = mode == GAPD_MODE_NAIVE ? -1 : mode == GAPD_MODE_TREE_FILL_FR ? kRuleFilling : kRuleExtrema;
    // The candidates, the defaults first.
    std::vector<Tuning> cands;
    if (mode == GAPD_MODE_NAIVE) {
        for (int c1 : {kNaiveCheck1, 1 - kNaiveCheck1})
            for (int pfw : {4, 8}) {
                Tuning t;
                t.naive_pfw = pfw;
                t.naive_check1 = c1;
                cands.push_back(t);
            }
    } else {
        for (int lanes : {kFillLanes, 256})
            for (int pf : {16, 8})
                for (int cap : {kSpecK, kSpecK / 2}) {
                    Tuning t;
                    t.fill_lanes = lanes;
                    t.walk_pf = pf;
                    t.spec_cap = cap;
                    cands.push_back(t);
                }
    }
    gapd_stats s{};
    st = all_pairs_impl(ctx, rule, 0, nullptr, out, &s, &cands[0]);  // warm-up
    if (st) return st;
    float best_ms = 0, default_ms = 0;
    size_t bi = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        gapd_stats t{};
        st = all_pairs_impl(ctx, rule, 0, nullptr, out, &t, &cands[i]);
        if (st) return st;
        if (i == 0) default_ms = t.ms_total;
        if (i == 0 || t.ms_total < best_ms) {
            best_ms = t.ms_total;
            bi = i;
        }
    }
    store_tuning(tune_key(ctx->H, ctx->W, ctx->C, ctx->conn, mode), cands[bi], best_ms);
    if (best) {
        best->fill_lanes = cands[bi].fill_lanes;
        best->walk_pf = cands[bi].walk_pf;
        best->spec_cap = cands[bi].spec_cap;
        best->naive_pfw = cands[bi].naive_pfw;
        best->naive_check1 = cands[bi].naive_check1;
        best->ms = best_ms;
        best->ms_default = default_ms;
        best->candidates = (int32_t)cands.size();
    }
    return GAPD_OK;
}

int gapd_set_tuning(gapd_ctx *ctx, int mode, const gapd_tuning *t) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!t) return fail(ctx, GAPD_EINVAL, "tuning is null");
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return fail(ctx, GAPD_EINVAL, "only the naive, filling-rate and extrema modes are tuned");
    if ((t->fill_lanes != 128 && t->fill_lanes != 256) || (t->walk_pf != 8 && t->walk_pf != 16) ||
        t->spec_cap < 1 || t->spec_cap > kSpecK || (t->naive_pfw != 4 && t->naive_pfw != 8) ||
        (t->naive_check1 != 0 && t->naive_check1 != 1))
        return fail(ctx, GAPD_EINVAL, "unsupported launch shapes (fill_lanes 128|256, walk_pf 8|16, spec_cap 1..32, "
                                      "naive_pfw 4|8, naive_check1 0|1)");
    Tuning x;
    x.fill_lanes = t->fill_lanes;
    x.walk_pf = t->walk_pf;
    x.spec_cap = t->spec_cap;
    x.naive_pfw = t->naive_pfw;
    x.naive_check1 = t->naive_check1;
    store_tuning(tune_key(ctx->H, ctx->W, ctx->C, ctx->conn, mode), x, 0.0, false);
    return GAPD_OK;
}

int gapd_all_pairs_spiral(gapd_ctx *ctx, int h, const uint32_t *draws, int32_t *out, gapd_stats *stp) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!out || !draws) return fail(ctx, GAPD_EINVAL, "out or draws is null");
    if (h < 0 || h > 65536) return fail(ctx, GAPD_EINVAL, "repulsion distance out of range");
    return all_pairs_impl(ctx, kRuleSpiral, h, draws, out, stp);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// A fixed device scratch for callers that cannot allocate device memory.
// ---------------------------------------------------------------------------------------------
namespace {

// Largest tree-method workspace the fixed scratch holds: 64 MiB covers the
// filled-pairs matrix and the tree cache up to N of about 18000 pixels (the
// 128 x 128 workload needs 40.6 MiB).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

// Every device that loads the library holds its own copy of this array until
// the process ends.  In host code its name is only a host-side stand-in:
// kernels get the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device with
// that device current (the previous current device is restored).
int scratch_on(int device, void **ptr, std::string &why) {
    if (device < 0 || device >= kMaxDevices) { why = "device id out of range for the fixed scratch"; return GAPD_EINVAL; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            why = std::string("looking up the fixed scratch: ") + hipGetErrorString(e);
            return GAPD_EDEVICE;
        }
        g_scratch_dev[device] = p;
    }
    *ptr = g_scratch_dev[device];
    return GAPD_OK;
}

}  // namespace

extern "C" {

int gapd_all_pairs_noalloc(gapd_ctx *ctx, int mode, int32_t *out, gapd_stats *stp) {
    int st = ctx_check(ctx);
    if (st) return st;
    if (!out) return fail(ctx, GAPD_EINVAL, "out is null");
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return fail(ctx, GAPD_EINVAL, "unknown mode (the spiral methods are not offered here)");
    gapd_stats local{};
    gapd_stats &s = stp ? *stp : local;
    s.n_prop = 0; s.n_prop_setup = 0; s.rounds = 0; s.centroid = -1; s.ms_total = 0; s.ms_setup = 0;
    s.ms_kernel = 0; s.ms_step_kernels = 0; s.ms_fill_kernels = 0; s.n_prop_speculative = 0; s.n_cache_hits = 0;
    s.rounds_speculative = 0;
    s.graph_replays = 0;
    if (mode == GAPD_MODE_NAIVE) {
        // no scratch: the naive method only needs the context's control block
        st = run_rows(ctx->g, nullptr, 0, ctx->N, out, ctx->max_rounds, ctx->ctl, ctx->stream, ctx->err,
                      ctx->poisoned, &s.rounds);
        if (st == GAPD_OK) s.n_prop = ctx->N;
        return st;
    }
    if (!tree_methods_fit(ctx->H, ctx->W))
        return fail(ctx, GAPD_EINVAL, "the tree methods need both image sides <= 192 (distance field in LDS)");
    const size_t need = fr_workspace_bytes(ctx->N, true);
    if (need > kNoAllocScratchBytes)
        return fail(ctx, GAPD_ENOMEM, "the tree-method workspace (" + std::to_string(need) +
                                          " bytes) exceeds the fixed scratch of 64 MiB (N up to about 18000)");
    void *ws = nullptr;
    st = scratch_on(ctx->device, &ws, ctx->err);
    if (st) return st;
    FrState fs = fr_workspace_layout(ws, ctx->N, true);
    fs.H = ctx->g.H;
    fs.W = ctx->g.W;
    fs.rule = mode == GAPD_MODE_TREE_FILL_FR ? kRuleFilling : kRuleExtrema;
    fs.D = out;
    fs.seq_out = s.sources_out;
    fs.filled_out = s.filled_out;
    fs.trace = s.step_trace;
    if (fs.trace)
        HIP_OR_FAIL(ctx, hipMemsetAsync(fs.trace, 0, sizeof(int64_t) * kTraceFields * (size_t)ctx->N, ctx->stream));
    const Tuning tune = tuning_for(tune_key(ctx->H, ctx->W, ctx->C, ctx->conn, mode));
    fs.spec_cap = tune.spec_cap;
    FrCtl hc{};
    st = run_filling_rate(ctx->g, fs, ctx->max_rounds, ctx->stream, nullptr, hc, ctx->err, ctx->poisoned, nullptr,
                          &s.graph_replays, tune);
    s.n_prop = hc.n_prop;
    s.rounds = hc.rounds;
    s.n_prop_speculative = hc.spec_props;
    s.n_cache_hits = hc.spec_hits;
    s.rounds_speculative = hc.spec_rounds;
    s.n_prop_setup = 2;
    s.centroid = hc.centroid;
    return st;
}

void gapd_destroy(gapd_ctx *ctx) {
    if (!ctx) return;
    if (ctx->dev) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->dev);
    }
    delete ctx;
}

}  // extern "C"

namespace gapd {

int run_rows(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out, int max_rounds, FrCtl *ctl,
             hipStream_t stream, std::string &err, bool &poisoned, int64_t *rounds_out, float *ms_kernel, int pfw,
             int check1) {
    // Launch errors are read with hipGetLastError: drop one that an earlier,
    // unrelated call left pending so it is not taken for ours.
    (void)hipGetLastError();
    hipEvent_t k0 = nullptr, k1 = nullptr;
    if (ms_kernel) {
        if (hipEventCreate(&k0) != hipSuccess || hipEventCreate(&k1) != hipSuccess) ms_kernel = nullptr;
    }
    hipError_t e = hipMemsetAsync(ctl, 0, sizeof(FrCtl), stream);
    if (e == hipSuccess && ms_kernel) e = hipEventRecord(k0, stream);
    if (e == hipSuccess) e = launch_relax_rows(g, src_list, src_base, K, out, max_rounds, ctl, stream, pfw, check1);
    if (e == hipSuccess && ms_kernel) e = hipEventRecord(k1, stream);
    FrCtl hc{};
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, ctl, sizeof(FrCtl), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        poisoned = true;
        err = std::string("propagation kernels: ") + hipGetErrorString(e);
        return GAPD_EDEVICE;
    }
    if (rounds_out) *rounds_out = hc.rounds;
    if (ms_kernel) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, k0, k1) == hipSuccess) *ms_kernel = ms;
    }
    if (k0) (void)hipEventDestroy(k0);
    if (k1) (void)hipEventDestroy(k1);
    if (hc.err) { err = "a propagation hit the sweep-round cap"; return hc.err; }
    return GAPD_OK;
}

int run_filling_rate(const GImg &g, const FrState &fs, int max_rounds, hipStream_t stream, hipEvent_t setup_done,
                     FrCtl &hc, std::string &err, bool &poisoned, float *kt, int *graph_replays,
                     const Tuning &tune) {
    const int N = g.N;
    auto bad = [&](hipError_t e, const char *where) {
        poisoned = true;
        err = std::string(where) + ": " + hipGetErrorString(e);
        return GAPD_EDEVICE;
    };
    (void)hipGetLastError();  // as in run_rows
    hipError_t e = hipMemsetAsync(fs.mask, 0, (size_t)N * fs.MW * 4, stream);
    if (e != hipSuccess) return bad(e, "clearing the filled-pairs matrix");
    e = hipMemsetAsync(fs.ctl, 0, sizeof(FrCtl), stream);
    if (e != hipSuccess) return bad(e, "clearing the loop state");
    e = launch_fr_init(fs, stream);
    if (e != hipSuccess) return bad(e, "filling-rate init launch");
    if (fs.rule != kRuleSpiral) {
        e = launch_fr_setup(g, fs, max_rounds, stream);
        if (e != hipSuccess) return bad(e, "centroid and extrema launch");
    }
    if (setup_done) {
        e = hipEventRecord(setup_done, stream);
        if (e != hipSuccess) return bad(e, "setup event");
    }
    // The loop runs on the device: each step selects its own source, so the
    // host only enqueues steps in chunks and reads the done flag between them.
    const int chunk = std::max(1, env_int("GAPD_FR_CHUNK", 64));
    std::vector<hipEvent_t> ev;
    if (kt) {
        kt[0] = kt[1] = 0.f;
        ev.resize(3 * (size_t)chunk);
        for (auto &x : ev)
            if (hipEventCreate(&x) != hipSuccess) return bad(hipErrorOutOfMemory, "timing events");
    }
    struct EvFree {
        std::vector<hipEvent_t> &v;
        ~EvFree() { for (auto x : v) (void)hipEventDestroy(x); }
    } ev_free{ev};
    int64_t enq = 0;
    int status = GAPD_OK;
    // After the first chunk (direct launches, which also set the kernels'
    // attributes) the chunk is captured once into a graph and replayed.
    StepGraph sg;
    bool graphs = !kt && use_step_graphs();
    for (;;) {
        if (graphs && enq > 0 && !sg.exec &&
            !sg.capture(chunk, [&](hipStream_t s) { return launch_fr_step(g, fs, max_rounds, s, nullptr, tune); }))
            graphs = false;  // capture refused: keep launching directly
        if (graphs && sg.exec) {
            e = hipGraphLaunch(sg.exec, stream);
            if (e != hipSuccess) return bad(e, "filling-rate step graph");
            if (graph_replays) ++*graph_replays;
        } else {
            for (int i = 0; i < chunk; ++i) {
                if (kt) (void)hipEventRecord(ev[3 * i], stream);
                e = launch_fr_step(g, fs, max_rounds, stream, kt ? ev[3 * i + 1] : nullptr, tune);
                if (e != hipSuccess) return bad(e, "filling-rate step");
                if (kt) (void)hipEventRecord(ev[3 * i + 2], stream);
            }
        }
        e = hipMemcpyAsync(&hc, fs.ctl, sizeof(FrCtl), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return bad(e, "filling-rate poll");
        if (kt) {
            // Step enq+i did work if it ran before the loop finished.
            for (int i = 0; i < chunk; ++i) {
                if (enq + i >= hc.n_prop) break;
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]) == hipSuccess) kt[0] += a;
                if (hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]) == hipSuccess) kt[1] += b;
            }
        }
        enq += chunk;
        if (hc.err) { err = "a propagation hit the sweep-round cap"; status = hc.err; break; }
        if (hc.done) break;
        if (enq > (int64_t)N + 2 * chunk) { err = "filling-rate loop did not terminate"; return GAPD_EDEVICE; }
    }
    return status;
}

}  // namespace gapd

// ---------------------------------------------------------------------------------------------
// Batched all-pairs.
// ---------------------------------------------------------------------------------------------
namespace {

struct BatchPlan {
    std::vector<size_t> img_off, w_off, fr_off;
    size_t imgs_bytes = 0, w_bytes = 0, fr_bytes = 0, desc_bytes = 0, total = 0;
};

BatchPlan plan_batch(const int32_t *H, const int32_t *W, int B, int C, int mode) {
    BatchPlan p;
    p.img_off.resize(B); p.w_off.resize(B); p.fr_off.resize(B);
    for (int b = 0; b < B; ++b) {
        const size_t N = (size_t)H[b] * W[b];
        p.img_off[b] = p.imgs_bytes; p.imgs_bytes += N * C;
        p.w_off[b] = p.w_bytes; p.w_bytes += weight_block_bytes(H[b], W[b]);
        p.fr_off[b] = p.fr_bytes;
        if (mode != GAPD_MODE_NAIVE) p.fr_bytes += fr_workspace_bytes((int)N);
    }
    p.imgs_bytes = al256(p.imgs_bytes);
    p.desc_bytes = al256(sizeof(BImg) * B) + al256(sizeof(GImgW) * B) + al256(sizeof(int64_t) * B) +
                   al256(sizeof(FrCtl));
    p.total = p.imgs_bytes + p.w_bytes + p.fr_bytes + p.desc_bytes;
    return p;
}

}  // namespace

extern "C" {

int gapd_batched_workspace_size(const int32_t *H, const int32_t *W, int B, int C, int conn, int mode, size_t *bytes) {
    if (!H || !W || B < 0 || !bytes || C < 1) return GAPD_EINVAL;
    if (conn != 4 && conn != 8) return GAPD_EINVAL;
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return GAPD_EINVAL;
    for (int b = 0; b < B; ++b)
        if (H[b] < 1 || W[b] < 1 || H[b] > kMaxLine || W[b] > kMaxLine) return GAPD_EINVAL;
    *bytes = plan_batch(H, W, B, C, mode).total;
    return GAPD_OK;
}

int gapd_all_pairs_batched(const uint8_t *images_packed, const int32_t *H, const int32_t *W, int B, int C, int conn,
                           int weight_mode, int mode, int32_t *out, const int64_t *out_offsets, int64_t *n_prop_out,
                           int32_t *sources_out, void *workspace, size_t ws_bytes, void *hip_stream) {
    if (B < 0 || !H || !W || !out_offsets) return GAPD_EINVAL;
    if (B == 0) return GAPD_OK;
    if (!images_packed || !out || !workspace) return GAPD_EINVAL;
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return GAPD_EINVAL;
    if ((uintptr_t)workspace & 255) return GAPD_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    (void)hipGetLastError();  // as in run_rows
    BatchPlan p = plan_batch(H, W, B, C, mode);
    if (ws_bytes < p.total) return GAPD_ENOMEM;
    std::string why;
    size_t in_off = 0;
    for (int b = 0; b < B; ++b) {
        int s = validate_image(images_packed + in_off, H[b], W[b], C, conn, weight_mode, why);
        if (s != GAPD_OK) { g_create_error = "image " + std::to_string(b) + ": " + why; return s; }
        const int64_t N = (int64_t)H[b] * W[b];
        if (out_offsets[b] < 0 || out_offsets[b + 1] - out_offsets[b] < N * N) {
            g_create_error = "out_offsets too small for image " + std::to_string(b);
            return GAPD_EINVAL;
        }
        in_off += (size_t)N * C;
    }
    char *base = (char *)workspace;
    uint8_t *imgs_dev = (uint8_t *)base;
    char *wbase = base + p.imgs_bytes;
    char *frbase = wbase + p.w_bytes;
    char *desc = frbase + p.fr_bytes;
    BImg *bimg_dev = (BImg *)desc;
    GImgW *gw_dev = (GImgW *)(desc + al256(sizeof(BImg) * B));
    int64_t *ioff_dev = (int64_t *)((char *)gw_dev + al256(sizeof(GImgW) * B));
    FrCtl *ctl_dev = (FrCtl *)((char *)ioff_dev + al256(sizeof(int64_t) * B));

    // Largest images first, so the long items start early.
    std::vector<int> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b2) { return (int64_t)H[a] * W[a] > (int64_t)H[b2] * W[b2]; });
    std::vector<GImgW> gw(B);
    std::vector<BImg> bi(B);
    std::vector<int64_t> ioff(B);
    std::vector<int64_t> seq_off(B + 1, 0);
    for (int b = 0; b < B; ++b) seq_off[b + 1] = seq_off[b] + (int64_t)H[b] * W[b];
    int64_t items = 0;
    int max_line = 1, maxN = 1;
    size_t lds = 0, wbytes = 0;
    for (int i = 0; i < B; ++i) {
        const int b = order[i];
        const int N = H[b] * W[b];
        gw[i] = weight_block_layout(wbase + p.w_off[b], H[b], W[b], conn);
        ioff[i] = (int64_t)p.img_off[b];
        BImg &x = bi[i];
        memset(&x, 0, sizeof(x));
        x.g = as_const(gw[i]);
        x.Wp = lds_row_stride(W[b]);
        x.out_off = out_offsets[b];
        x.item0 = items;
        items += N;
        max_line = std::max(max_line, std::max(H[b], W[b]));
        const size_t l = (size_t)H[b] * x.Wp * 4;
        if (mode != GAPD_MODE_NAIVE) {
            x.fr = fr_workspace_layout(frbase + p.fr_off[b], N);
            x.fr.H = H[b];
            x.fr.W = W[b];
            x.fr.rule = mode == GAPD_MODE_TREE_FILL_EXTREMA ? kRuleExtrema : kRuleFilling;
            x.fr.D = out + out_offsets[b];
            x.fr.seq_out = sources_out ? sources_out + seq_off[b] : nullptr;
            wbytes = std::max(wbytes, (size_t)(conn == 8 ? 4 : 2) * ((N + 1) / 2) * 4);
        }
        lds = std::max(lds, l);
        maxN = std::max(maxN, N);
    }
    if (lds > kMaxLds) { g_create_error = "an image is too large for the batched kernels"; return GAPD_EINVAL; }
    const int max_rounds = max_rounds_for(1 << 30);
    hipError_t e = hipMemcpyAsync(imgs_dev, images_packed, in_off, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(wbase, 0, p.w_bytes, st);
    if (e == hipSuccess) e = hipMemcpyAsync(gw_dev, gw.data(), sizeof(GImgW) * B, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ioff_dev, ioff.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bimg_dev, bi.data(), sizeof(BImg) * B, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ctl_dev, 0, sizeof(FrCtl), st);
    if (e == hipSuccess && mode != GAPD_MODE_NAIVE) e = hipMemsetAsync(frbase, 0, p.fr_bytes, st);
    if (e == hipSuccess) e = launch_prep_batched(gw_dev, imgs_dev, ioff_dev, B, C, weight_mode, st);
    if (e == hipSuccess) {
        if (mode == GAPD_MODE_NAIVE) {
            e = launch_relax_rows_batched(bimg_dev, B, items, max_line, lds, conn, out, max_rounds, ctl_dev, st);
        } else {
            // Images run their loops in lockstep; the host enqueues steps in
            // chunks and reads how many images have finished between chunks.
            e = launch_fr_batched_setup(bimg_dev, B, max_line, maxN, lds, conn, max_rounds, st);
            const int chunk = std::max(1, env_int("GAPD_FR_CHUNK", 64));
            int64_t enq = 0;
            StepGraph sg;  // as in run_filling_rate: the chunk replayed as a graph after the first
            bool graphs = use_step_graphs();
            auto step = [&](hipStream_t s) {
                return launch_fr_batched_step(bimg_dev, B, max_line, maxN, lds, wbytes, conn, max_rounds,
                                              &ctl_dev->done, s);
            };
            while (e == hipSuccess) {
                if (graphs && enq > 0 && !sg.exec && !sg.capture(chunk, step)) graphs = false;
                if (graphs && sg.exec)
                    e = hipGraphLaunch(sg.exec, st);
                else
                    for (int i = 0; i < chunk && e == hipSuccess; ++i) e = step(st);
                enq += chunk;
                FrCtl hc{};
                if (e == hipSuccess) e = hipMemcpyAsync(&hc, ctl_dev, sizeof(FrCtl), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess || hc.done >= B) break;
                if (enq > (int64_t)maxN + 2 * chunk) {
                    g_create_error = "batched filling-rate loop did not terminate";
                    return GAPD_EDEVICE;
                }
            }
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { g_create_error = std::string("batched: ") + hipGetErrorString(e); return GAPD_EDEVICE; }
    int status = GAPD_OK;
    if (mode == GAPD_MODE_NAIVE) {
        FrCtl hc{};
        e = hipMemcpy(&hc, ctl_dev, sizeof(FrCtl), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return GAPD_EDEVICE;
        if (hc.err) status = hc.err;
        if (n_prop_out)
            for (int b = 0; b < B; ++b) n_prop_out[b] = (int64_t)H[b] * W[b];
    } else {
        for (int i = 0; i < B; ++i) {
            FrCtl hc{};
            e = hipMemcpy(&hc, bi[i].fr.ctl, sizeof(FrCtl), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return GAPD_EDEVICE;
            if (hc.err) status = hc.err;
            if (n_prop_out) n_prop_out[order[i]] = hc.n_prop;
        }
    }
    return status;
}

}  // extern "C"
