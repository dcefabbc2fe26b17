// C ABI of the general-graph path (declared in include/gapd.h): the
// propagations, geodesic trees, redundancy fill and deterministic selection
// rules on an undirected CSR graph whose boundary vertices stand in for the
// image border (Section 5).
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "capi_internal.h"
#include "gapd.h"
#include "gapd_internal.h"

using namespace gapd;

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Host checks of a CSR graph (include/gapd.h, gapd_graph_create).
int validate_graph(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw, std::string &why) {
    if (n < 1 || n > kGraphMaxN) { why = "n must be in [1, 32768]"; return GAPD_EINVAL; }
    if (!rp || rp[0] != 0) { why = "row_ptr is null or row_ptr[0] != 0"; return GAPD_EINVAL; }
    for (int64_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) { why = "row_ptr decreases"; return GAPD_EINVAL; }
    const int64_t m = rp[n];
    if (m > 0 && (!ci || !cw)) { why = "col_idx or weight is null"; return GAPD_EINVAL; }
    if (m > (int64_t)1 << 31) { why = "too many edges"; return GAPD_EINVAL; }
    std::vector<int64_t> mark(n, -1);
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int64_t u = ci[e];
            if (u < 0 || u >= n) { why = "a neighbour id is out of range"; return GAPD_EINVAL; }
            if (u == v) { why = "a self loop"; return GAPD_EINVAL; }
            if (cw[e] < 1) { why = "an edge weight is below 1"; return GAPD_EINVAL; }
            // No distance may reach 2^27 (the tree words keep 5 flag bits
            // above it), and the kernels add a weight to a distance in int32:
            // an edge at least that heavy is refused even off the spanning
            // tree checked below.
            if (cw[e] >= kDistLimit) { why = "an edge weighs 2^27 or more"; return GAPD_ERANGE; }
            if (mark[u] == v) { why = "a neighbour is listed twice"; return GAPD_EINVAL; }
            mark[u] = v;
        }
    }
    // every edge has its reverse with the same weight
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int64_t u = ci[e];
            bool ok = false;
            for (int64_t f = rp[u]; f < rp[u + 1] && !ok; ++f) ok = ci[f] == v && cw[f] == cw[e];
            if (!ok) { why = "an edge has no reverse of the same weight"; return GAPD_EINVAL; }
        }
    // connected; the breadth-first tree from vertex 0 spans the graph, and
    // every distance is at most its total weight
    std::vector<int32_t> q(n);
    std::vector<char> seen(n, 0);
    int64_t head = 0, tail = 0, span = 0;
    q[tail++] = 0;
    seen[0] = 1;
    while (head < tail) {
        const int64_t v = q[head++];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (!seen[ci[e]]) {
                seen[ci[e]] = 1;
                q[tail++] = ci[e];
                span += cw[e];
            }
    }
    if (tail != n) { why = "the graph is not connected"; return GAPD_EINVAL; }
    if (span >= kDistLimit) { why = "distances could reach 2^27"; return GAPD_ERANGE; }
    return GAPD_OK;
}

}  // namespace

struct gapd_graph {
    int n = 0;
    int64_t m = 0;
    hipStream_t stream = nullptr;
    void *dev = nullptr;
    GGraph g{};
    FrCtl *ctl = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    bool poisoned = false;
};

static int gfail(gapd_graph *G, int st, const std::string &msg) {
    if (G) G->err = msg;
    return st;
}

#define GHIP_OR_FAIL(G, expr)                                                              \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            (G)->poisoned = true;                                                          \
            return gfail((G), GAPD_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
        }                                                                                  \
    } while (0)

static int gcheck(gapd_graph *G) {
    if (!G) return GAPD_EINVAL;
    if (G->poisoned) return gfail(G, GAPD_EDEVICE, "graph context is poisoned by an earlier device error");
    return GAPD_OK;
}

static int graph_max_rounds(int n) { return std::max(2, std::min(env_int("GAPD_MAX_ROUNDS", n + 2), n + 2)); }

// The tree-method loop on a graph: setup, then steps enqueued in chunks until
// the done flag is seen (as the image loop does).  Synchronises the stream.
static int run_graph_tree(gapd_graph *G, const FrState &fs, hipEvent_t setup_done, FrCtl &hc, float *kt) {
    const int N = G->n, max_rounds = graph_max_rounds(N);
    hipStream_t stream = G->stream;
    auto bad = [&](hipError_t e, const char *where) {
        G->poisoned = true;
        G->err = std::string(where) + ": " + hipGetErrorString(e);
        return GAPD_EDEVICE;
    };
    (void)hipGetLastError();  // launch checks below read hipGetLastError
    hipError_t e = hipMemsetAsync(fs.mask, 0, (size_t)N * fs.MW * 4, stream);
    if (e != hipSuccess) return bad(e, "clearing the filled-pairs matrix");
    e = hipMemsetAsync(fs.ctl, 0, sizeof(FrCtl), stream);
    if (e != hipSuccess) return bad(e, "clearing the loop state");
    e = launch_fr_init(fs, stream);
    if (e != hipSuccess) return bad(e, "init launch");
    e = launch_graph_setup(G->g, fs, max_rounds, stream);
    if (e != hipSuccess) return bad(e, "centre and extrema launch");
    if (setup_done && (e = hipEventRecord(setup_done, stream)) != hipSuccess) return bad(e, "setup event");
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
    for (;;) {
        for (int i = 0; i < chunk; ++i) {
            if (kt) (void)hipEventRecord(ev[3 * i], stream);
            e = launch_graph_step(G->g, fs, max_rounds, stream, kt ? ev[3 * i + 1] : nullptr);
            if (e != hipSuccess) return bad(e, "graph step");
            if (kt) (void)hipEventRecord(ev[3 * i + 2], stream);
        }
        e = hipMemcpyAsync(&hc, fs.ctl, sizeof(FrCtl), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return bad(e, "graph loop poll");
        if (kt)
            for (int i = 0; i < chunk && enq + i < hc.n_prop; ++i) {
                float a = 0, b = 0;
                if (hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]) == hipSuccess) kt[0] += a;
                if (hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]) == hipSuccess) kt[1] += b;
            }
        enq += chunk;
        if (hc.err) { G->err = "a propagation hit the round cap"; return hc.err; }
        if (hc.done) return GAPD_OK;
        if (enq > (int64_t)N + 2 * chunk) { G->err = "graph loop did not terminate"; return GAPD_EDEVICE; }
    }
}

extern "C" {

int gapd_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const int32_t *weight,
                      const uint8_t *boundary, gapd_graph **out) {
    if (!out) return GAPD_EINVAL;
    *out = nullptr;
    std::string why;
    int st = validate_graph(n, row_ptr, col_idx, weight, why);
    if (st != GAPD_OK) { g_create_error = why; return st; }
    const int64_t m = row_ptr[n];
    // boundary: given, or the vertices of degree below the average (all when none is)
    std::vector<uint8_t> bnd(n);
    if (boundary) {
        int64_t any = 0;
        for (int64_t v = 0; v < n; ++v) any += bnd[v] = boundary[v] ? 1 : 0;
        if (!any) { g_create_error = "no boundary vertex"; return GAPD_EINVAL; }
    } else {
        int64_t any = 0;
        for (int64_t v = 0; v < n; ++v) {
            bnd[v] = (row_ptr[v + 1] - row_ptr[v]) * n < m;
            any += bnd[v];
        }
        if (!any) std::fill(bnd.begin(), bnd.end(), 1);
    }
    gapd_graph *G = new gapd_graph;
    G->n = (int)n;
    G->m = m;
    const size_t b_rp = al256((size_t)(n + 1) * 8), b_ci = al256((size_t)m * 4 + 4), b_cw = b_ci,
                 b_bnd = al256((size_t)n), b_ctl = al256(sizeof(FrCtl));
    hipError_t e = hipMalloc(&G->dev, b_rp + b_ci + b_cw + b_bnd + b_ctl);
    if (e != hipSuccess) {
        delete G;
        g_create_error = "device memory";
        return GAPD_ENOMEM;
    }
    char *p = (char *)G->dev;
    int64_t *rp = (int64_t *)p; p += b_rp;
    int32_t *ci = (int32_t *)p; p += b_ci;
    int32_t *cw = (int32_t *)p; p += b_cw;
    uint8_t *bd = (uint8_t *)p; p += b_bnd;
    G->ctl = (FrCtl *)p;
    e = hipMemcpy(rp, row_ptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && m) e = hipMemcpy(ci, col_idx, (size_t)m * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && m) e = hipMemcpy(cw, weight, (size_t)m * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bd, bnd.data(), (size_t)n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(G->dev);
        delete G;
        g_create_error = std::string("upload: ") + hipGetErrorString(e);
        return GAPD_EDEVICE;
    }
    G->g.n = (int)n;
    G->g.rp = rp;
    G->g.ci = ci;
    G->g.cw = cw;
    G->g.bnd = bd;
    *out = G;
    return GAPD_OK;
}

int gapd_graph_set_stream(gapd_graph *G, void *hip_stream) {
    int st = gcheck(G);
    if (st) return st;
    G->stream = (hipStream_t)hip_stream;
    return GAPD_OK;
}

int gapd_graph_workspace_size(gapd_graph *G, int mode, size_t *bytes) {
    int st = gcheck(G);
    if (st) return st;
    if (!bytes) return gfail(G, GAPD_EINVAL, "bytes is null");
    if (mode == GAPD_MODE_NAIVE) { *bytes = 0; return GAPD_OK; }
    if (mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return gfail(G, GAPD_EINVAL, "graphs support the naive, filling-rate and extrema modes");
    *bytes = graph_workspace_bytes(G->n);
    return GAPD_OK;
}

int gapd_graph_set_workspace(gapd_graph *G, void *dev_ptr, size_t bytes) {
    int st = gcheck(G);
    if (st) return st;
    if (dev_ptr && ((uintptr_t)dev_ptr & 255)) return gfail(G, GAPD_EINVAL, "workspace must be 256-byte aligned");
    G->ws = dev_ptr;
    G->ws_bytes = dev_ptr ? bytes : 0;
    return GAPD_OK;
}

int gapd_graph_sssp(gapd_graph *G, const int32_t *sources, int K, int32_t *out) {
    int st = gcheck(G);
    if (st) return st;
    if (K < 0) return gfail(G, GAPD_EINVAL, "K < 0");
    if (K == 0) return GAPD_OK;
    if (!sources || !out) return gfail(G, GAPD_EINVAL, "null pointer");
    std::vector<int32_t> hs(K);
    GHIP_OR_FAIL(G, hipMemcpyAsync(hs.data(), sources, sizeof(int32_t) * K, hipMemcpyDeviceToHost, G->stream));
    GHIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
    for (int k = 0; k < K; ++k)
        if (hs[k] < 0 || hs[k] >= G->n) return gfail(G, GAPD_EINVAL, "source id out of range");
    (void)hipGetLastError();
    GHIP_OR_FAIL(G, hipMemsetAsync(G->ctl, 0, sizeof(FrCtl), G->stream));
    GHIP_OR_FAIL(G, launch_graph_rows(G->g, sources, 0, K, out, graph_max_rounds(G->n), G->ctl, G->stream));
    FrCtl hc{};
    GHIP_OR_FAIL(G, hipMemcpyAsync(&hc, G->ctl, sizeof(FrCtl), hipMemcpyDeviceToHost, G->stream));
    GHIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
    if (hc.err) return gfail(G, hc.err, "a propagation hit the round cap");
    return GAPD_OK;
}

int gapd_graph_all_pairs(gapd_graph *G, int mode, int32_t *out, gapd_stats *stp) {
    int st = gcheck(G);
    if (st) return st;
    if (!out) return gfail(G, GAPD_EINVAL, "out is null");
    if (mode != GAPD_MODE_NAIVE && mode != GAPD_MODE_TREE_FILL_FR && mode != GAPD_MODE_TREE_FILL_EXTREMA)
        return gfail(G, GAPD_EINVAL, "graphs support the naive, filling-rate and extrema modes");
    gapd_stats local{};
    gapd_stats &s = stp ? *stp : local;
    s.n_prop = 0; s.n_prop_setup = 0; s.rounds = 0; s.centroid = -1; s.ms_total = 0; s.ms_setup = 0;
    s.ms_kernel = 0; s.ms_step_kernels = 0; s.ms_fill_kernels = 0; s.n_prop_speculative = 0; s.n_cache_hits = 0;
    s.rounds_speculative = 0;
    s.graph_replays = 0;
    hipEvent_t e0, e1, e2;
    GHIP_OR_FAIL(G, hipEventCreate(&e0));
    GHIP_OR_FAIL(G, hipEventCreate(&e1));
    GHIP_OR_FAIL(G, hipEventCreate(&e2));
    struct EvGuard {
        hipEvent_t a, b, c;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); }
    } guard{e0, e1, e2};
    GHIP_OR_FAIL(G, hipEventRecord(e0, G->stream));
    if (mode == GAPD_MODE_NAIVE) {
        (void)hipGetLastError();
        GHIP_OR_FAIL(G, hipMemsetAsync(G->ctl, 0, sizeof(FrCtl), G->stream));
        GHIP_OR_FAIL(G, hipEventRecord(e1, G->stream));
        GHIP_OR_FAIL(G, launch_graph_rows(G->g, nullptr, 0, G->n, out, graph_max_rounds(G->n), G->ctl, G->stream));
        GHIP_OR_FAIL(G, hipEventRecord(e2, G->stream));
        FrCtl hc{};
        GHIP_OR_FAIL(G, hipMemcpyAsync(&hc, G->ctl, sizeof(FrCtl), hipMemcpyDeviceToHost, G->stream));
        GHIP_OR_FAIL(G, hipStreamSynchronize(G->stream));
        s.n_prop = G->n;
        s.rounds = hc.rounds;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e1, e2) == hipSuccess) s.ms_kernel = ms;
        if (hc.err) return gfail(G, hc.err, "a propagation hit the round cap");
    } else {
        const size_t need = graph_workspace_bytes(G->n);
        if (!G->ws || G->ws_bytes < need) return gfail(G, GAPD_ENOMEM, "tree-method workspace missing or too small");
        FrState fs = graph_workspace_layout(G->ws, G->n);
        fs.H = 0;
        fs.W = 0;
        fs.rule = mode == GAPD_MODE_TREE_FILL_EXTREMA ? kRuleExtrema : kRuleFilling;
        fs.D = out;
        fs.seq_out = s.sources_out;
        fs.filled_out = s.filled_out;
        FrCtl hc{};
        float kt[2] = {0.f, 0.f};
        st = run_graph_tree(G, fs, e1, hc, s.time_kernels ? kt : nullptr);
        if (st == GAPD_EDEVICE) return st;
        s.ms_step_kernels = kt[0];
        s.ms_fill_kernels = kt[1];
        GHIP_OR_FAIL(G, hipEventRecord(e2, G->stream));
        GHIP_OR_FAIL(G, hipEventSynchronize(e2));
        s.n_prop = hc.n_prop;
        s.n_prop_setup = 2;
        s.rounds = hc.rounds;
        s.centroid = hc.centroid;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) s.ms_setup = ms;
        if (st) return st;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e2) == hipSuccess) s.ms_total = ms;
    return GAPD_OK;
}

const char *gapd_graph_last_error(gapd_graph *G) {
    if (!G) return g_create_error.c_str();
    return G->err.c_str();
}

void gapd_graph_destroy(gapd_graph *G) {
    if (!G) return;
    if (G->dev) {
        (void)hipStreamSynchronize(G->stream);
        (void)hipFree(G->dev);
    }
    delete G;
}

}  // extern "C"
