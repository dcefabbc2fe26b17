// Host-side helpers shared by the C ABI (capi.cpp) and the server (server.cpp).
#pragma once

#include <functional>
#include <string>

#include "gapd_internal.h"

namespace gapd {

extern thread_local std::string g_create_error;

int env_int(const char *name, int dflt);
int validate_image(const uint8_t *img, int H, int W, int C, int conn, int wmode, std::string &why);
int max_rounds_for(int N);

// A chunk of loop steps recorded once from a private stream (capture only,
// nothing runs there) and replayed on the caller's stream.  Only kernel
// launches are recorded: no memset or copy.
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;
    ~StepGraph();
    // Record n calls of step; false (and nothing to replay) if HIP refused.
    bool capture(int n, const std::function<hipError_t(hipStream_t)> &step);
};
// Whether loop chunks are replayed as graphs (GAPD_FR_GRAPH=0 turns it off).
bool use_step_graphs();

// Longest image side the tree-based methods accept on one image: their step
// kernel keeps the distance field in LDS.
constexpr int kTreeMaxSide = 192;
inline bool tree_methods_fit(int H, int W) { return H <= kTreeMaxSide && W <= kTreeMaxSide; }

// Propagations from K sources into K rows of out; synchronises the stream.
// pfw: the sweeps' weight prefetch depth (0: default); check1: check the
// edges after the first round already.
int run_rows(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out, int max_rounds, FrCtl *ctl,
             hipStream_t stream, std::string &err, bool &poisoned, int64_t *rounds_out = nullptr,
             float *ms_kernel = nullptr, int pfw = 0, int check1 = kNaiveCheck1);

// Autotuned launch shapes (tune.cpp): the cache key of an image and method,
// and the cached shapes for it (defaults when the cache has none).
std::string tune_key(int H, int W, int C, int conn, int mode);
Tuning tuning_for(const std::string &key);
// save: also rewrite the cache file (else this process only).
void store_tuning(const std::string &key, const Tuning &t, double ms, bool save = true);

// The filling-rate method on one image (workspace fs, output fs.D); the
// final control block is copied to hc.  Synchronises the stream.
// With kt non-null, every loop launch is bracketed by events and the summed
// durations of the launches that did work are returned in kt[0] (select +
// propagate) and kt[1] (fill).
int run_filling_rate(const GImg &g, const FrState &fs, int max_rounds, hipStream_t stream, hipEvent_t setup_done,
                     FrCtl &hc, std::string &err, bool &poisoned, float *kt = nullptr, int *graph_replays = nullptr,
                     const Tuning &tune = Tuning());

}  // namespace gapd
