// The tree-based methods on one image: setup (geodesic centroid and extrema
// ranks, Section 3.3), loop steps (selection + propagation + tree, Sections
// 3.1-3.4) and the redundancy fill beside the speculative propagations.
#include "dev_common.h"

namespace gapd {

namespace {

template <int CONN, int S>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_setup(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    fr_setup_block<CONN, S>(g, Wp, fs, smem, max_rounds, red);
}

template <int CONN, int S, bool kStageW>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_step(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    fr_step_block<CONN, S, kStageW>(g, Wp, fs, max_rounds, smem, red, nullptr);
}

// Static LDS of the speculation plan's sort keys (beyond the usual reserve).
constexpr size_t kSpecSortLds = (2 * kRelaxThreads + kSpecSlots) * sizeof(uint64_t);

template <int CONN, int S, bool kStageW>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_step_spec(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    __shared__ uint64_t keys[2 * kRelaxThreads];
    __shared__ uint64_t skeys[kSpecSlots];
    const int64_t t0 = fs.trace ? trace_clock() : 0;
    __shared__ int64_t ph[3];  // select phases (thread 0, when tracing)
    fr_step_block<CONN, S, kStageW, true>(g, Wp, fs, max_rounds, smem, red, nullptr, keys, skeys,
                                          fs.trace ? ph : nullptr);
    // thread 0 set the step's state; a step that found D complete records nothing
    if (fs.trace && threadIdx.x == 0 && !fs.ctl->done) {
        int64_t *tr = fs.trace + (fs.ctl->n_prop - 1) * kTraceFields;
        const int64_t t1 = trace_clock();
        tr[kTrSelect] = t1 - t0;
        tr[kTrHit] = fs.ctl->tree_slot >= 0;
        tr[kTrSelPass] = ph[0] - t0;
        tr[kTrSelMin] = ph[1] - ph[0];
        tr[kTrSelSort] = ph[2] - ph[1];
        tr[kTrSelRest] = t1 - ph[2];
    }
}

template <bool kLds, bool kLdsCount>
__global__ __launch_bounds__(256) void k_fr_fill(FrState fs, int W) {
    extern __shared__ uint32_t spk[];
    __shared__ int64_t red[4];
    fr_fill_block<kLds, kLdsCount>(fs, fs.packed, W, spk, red, blockIdx.x, gridDim.x);
}

// Fill variants of the speculative step: the link fill (when its tables fit
// LDS) with 128 or 256 walking threads per block and 8 or 16 ancestor pairs
// in flight per walk (the autotuner's choice), the walk with a grandparent
// table (kFillA2) or the plain walk with the tree words in LDS (kFillTree).
constexpr int kFillTree = 0, kFillA2 = 1, kFillLinks = 2;  // kFillLinks + (lanes == 256) + 2 * (pf == 8)
constexpr int kFillCompact = 6;  // the compact tables (parent table only, counts in global memory)
constexpr int fill_links_variant(int lanes, int pf) { return kFillLinks + (lanes == 256 ? 1 : 0) + (pf == 8 ? 2 : 0); }
constexpr int variant_lanes(int v) { return ((v - kFillLinks) & 1) ? 256 : 128; }
constexpr int variant_pf(int v) { return ((v - kFillLinks) & 2) ? 8 : 16; }

// The fill of the current step (blocks kSpecK..) beside the speculative
// propagations of the candidates it listed (blocks 0..kSpecK-1, first, so
// that the longer propagations start at once).  The link fill and the
// grandparent walk use kFillLanes (128) walking threads per 256-thread block:
// the walks then spread over twice the compute units, which pays for the
// extra staging.
template <int CONN, int S, bool kStageW, bool kLdsCount, int kFill = kFillTree>
__global__ __launch_bounds__(256) void k_fr_fill_spec(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ int64_t red[4];
    if (fs.ctl->done) return;
    if ((int)blockIdx.x < kSpecK) {
        const int64_t t0 = fs.trace ? trace_clock() : 0;
        const int r = fr_spec_block<CONN, S, kStageW>(g, Wp, fs, smem, blockIdx.x);
        if (fs.trace && threadIdx.x == 0 && r != -3) {
            int64_t *tr = fs.trace + (fs.ctl->n_prop - 1) * kTraceFields;
            const int64_t t1 = trace_clock();
            atomicAdd((unsigned long long *)&tr[kTrSpecPieces], 1ull);
            atomicMax((unsigned long long *)&tr[kTrSpecMax], (unsigned long long)(t1 - t0));
            if (r >= 0) atomicAdd((unsigned long long *)&tr[kTrSpecDone], 1ull);
            atomicMax((unsigned long long *)&tr[kTrSpecEnd], (unsigned long long)t1);
        }
        return;
    }
    const int slot = fs.ctl->tree_slot;
    const uint32_t *tree = slot >= 0 ? slot_tree(fs, slot) : fs.packed;
    if constexpr (kFill == kFillCompact) {
        fill_links_block<kCompactLanes, 16, true>(fs, tree, g.W, (uint32_t *)smem, red, blockIdx.x - kSpecK);
    } else if constexpr (kFill >= kFillLinks) {
        fill_links_block<variant_lanes(kFill), variant_pf(kFill)>(fs, tree, g.W, (uint32_t *)smem, red,
                                                                 blockIdx.x - kSpecK);
    } else {
        fr_fill_block<true, kLdsCount, kFill == kFillA2, kFill == kFillA2 ? 128 : 256>(
            fs, tree, g.W, (uint32_t *)smem, red, blockIdx.x - kSpecK, gridDim.x - kSpecK);
    }
}

template <int CONN, int S>
struct FrSetup {
    static hipError_t run(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        auto k1 = k_fr_setup<CONN, S>;
        hipError_t e = set_lds(k1, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k1, dim3(1), dim3(kRelaxThreads), lds, st, g, Wp, fs, max_rounds);
        hipLaunchKernelGGL(k_rank, dim3((g.N + 255) / 256), dim3(256), 0, st, fs.dbuf, g.N, fs.rank, fs.order);
        return hipGetLastError();
    }
};

template <int CONN, int S>
struct FrStep {
    template <bool kStageW, bool kLdsCount, int kFill = kFillTree>
    static hipError_t launch_fill_spec(const GImg &g, int Wp, const FrState &fs, int max_rounds, hipStream_t st,
                                       size_t lds, int blocks) {
        auto k = k_fr_fill_spec<CONN, S, kStageW, kLdsCount, kFill>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(kSpecK + blocks), dim3(256), lds, st, g, Wp, fs, max_rounds);
        return hipGetLastError();
    }

    template <bool kStageW>
    static hipError_t launch_step(const GImg &g, int Wp, const FrState &fs, int max_rounds, hipStream_t st,
                                  size_t lds, bool spec) {
        auto k1 = spec ? k_fr_step_spec<CONN, S, kStageW> : k_fr_step<CONN, S, kStageW>;
        hipError_t e = set_lds(k1, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k1, dim3(1), dim3(kRelaxThreads), lds, st, g, Wp, fs, max_rounds);
        return hipGetLastError();
    }

    template <bool kStageW>
    static hipError_t launch_links(const GImg &g, int Wp, const FrState &fs, int max_rounds, hipStream_t st,
                                   size_t lds, int lanes, int pf) {
        const int blocks = (g.N + lanes - 1) / lanes;
        switch (fill_links_variant(lanes, pf)) {
            case fill_links_variant(256, 16):
                return launch_fill_spec<kStageW, false, fill_links_variant(256, 16)>(g, Wp, fs, max_rounds, st, lds,
                                                                                    blocks);
            case fill_links_variant(128, 8):
                return launch_fill_spec<kStageW, false, fill_links_variant(128, 8)>(g, Wp, fs, max_rounds, st, lds,
                                                                                   blocks);
            case fill_links_variant(256, 8):
                return launch_fill_spec<kStageW, false, fill_links_variant(256, 8)>(g, Wp, fs, max_rounds, st, lds,
                                                                                   blocks);
            default:
                return launch_fill_spec<kStageW, false, fill_links_variant(128, 16)>(g, Wp, fs, max_rounds, st, lds,
                                                                                    blocks);
        }
    }

    static hipError_t run(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st, hipEvent_t mid,
                          const Tuning &tune) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        const size_t wbytes = (size_t)(CONN == 8 ? 4 : 2) * ((g.N + 1) / 2) * sizeof(uint32_t);
        const size_t pk = (size_t)g.N * sizeof(uint32_t);
        // speculation needs the fill to stage a tree in LDS and the select
        // kernel to hold its sort keys beside the field
        const bool spec = fs.cache && pk <= kMaxLds && lds + kSpecSortLds <= kMaxLds;
        const size_t extra = spec ? kSpecSortLds : 0;
        if (spec) {
            const hipError_t ep = launch_sel_part(fs, st);
            if (ep != hipSuccess) return ep;
        }
        hipError_t e = lds + wbytes + extra <= kMaxLds
                           ? launch_step<true>(g, Wp, fs, max_rounds, st, lds + wbytes, spec)
                           : launch_step<false>(g, Wp, fs, max_rounds, st, lds, spec);
        if (e != hipSuccess) return e;
        if (mid) {
            e = hipEventRecord(mid, st);
            if (e != hipSuccess) return e;
        }
        const int blocks = (g.N + 255) / 256;
        if (spec) {
            // the fill beside the speculative propagations
            const size_t sp = lds + (lds + wbytes <= kMaxLds ? wbytes : 0);
            const size_t a2 = pk + (size_t)g.N * 2;  // tree words + grandparents
            const int blocks2 = (g.N + kFillLanes - 1) / kFillLanes;
            const int lanes = tune.fill_lanes == 256 && link_fill_fits(g.N, 256) ? 256 : kFillLanes;
            const int pf = tune.walk_pf == 8 ? 8 : 16;
            if (link_fill_fits(g.N, lanes)) {
                const size_t ll = std::max(sp, link_fill_lds(g.N, lanes));
                if (lds + wbytes <= kMaxLds)
                    e = launch_links<true>(g, Wp, fs, max_rounds, st, ll, lanes, pf);
                else
                    e = launch_links<false>(g, Wp, fs, max_rounds, st, ll, lanes, pf);
            } else if (compact_fill_fits(g.N)) {
                const size_t cl = std::max(sp, compact_fill_lds(g.N));
                const int cb = (g.N + kCompactLanes - 1) / kCompactLanes;
                if (lds + wbytes <= kMaxLds)
                    e = launch_fill_spec<true, false, kFillCompact>(g, Wp, fs, max_rounds, st, cl, cb);
                else
                    e = launch_fill_spec<false, false, kFillCompact>(g, Wp, fs, max_rounds, st, cl, cb);
            } else if (a2 <= kMaxLds && g.N < 0xFFFF) {
                if (lds + wbytes <= kMaxLds)
                    e = launch_fill_spec<true, false, kFillA2>(g, Wp, fs, max_rounds, st, std::max(sp, a2), blocks2);
                else
                    e = launch_fill_spec<false, false, kFillA2>(g, Wp, fs, max_rounds, st, std::max(sp, a2), blocks2);
            } else if (2 * pk <= kMaxLds) {
                if (lds + wbytes <= kMaxLds)
                    e = launch_fill_spec<true, true>(g, Wp, fs, max_rounds, st, std::max(sp, 2 * pk), blocks);
                else
                    e = launch_fill_spec<false, true>(g, Wp, fs, max_rounds, st, std::max(sp, 2 * pk), blocks);
            } else {
                if (lds + wbytes <= kMaxLds)
                    e = launch_fill_spec<true, false>(g, Wp, fs, max_rounds, st, std::max(sp, pk), blocks);
                else
                    e = launch_fill_spec<false, false>(g, Wp, fs, max_rounds, st, std::max(sp, pk), blocks);
            }
            if (e != hipSuccess) return e;
        } else if (2 * pk <= kMaxLds) {
            auto k2 = k_fr_fill<true, true>;
            e = set_lds(k2, 2 * pk);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k2, dim3(blocks), dim3(256), 2 * pk, st, fs, g.W);
        } else if (pk <= kMaxLds) {
            auto k2 = k_fr_fill<true, false>;
            e = set_lds(k2, pk);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k2, dim3(blocks), dim3(256), pk, st, fs, g.W);
        } else {
            hipLaunchKernelGGL((k_fr_fill<false, false>), dim3(blocks), dim3(256), 0, st, fs, g.W);
        }
        return hipGetLastError();
    }
};

}  // namespace

// ---- launchers ----------------------------------------------------------------------------------
// This file is compiled once per (connectivity, size class) pair, given by
// GAPD_CONN and GAPD_S, so the instantiations build in parallel; the
// dispatch over the pairs is launch_fr_setup / launch_fr_step (k_misc.hip).
#if !defined(GAPD_CONN) || !defined(GAPD_S)
#error "k_fr.hip needs -DGAPD_CONN=<4|8> -DGAPD_S=<32|64|128|192>"
#endif
#define GAPD_PART_CAT2(a, b, c) a##_##b##_##c
#define GAPD_PART_CAT(a, b, c) GAPD_PART_CAT2(a, b, c)

hipError_t GAPD_PART_CAT(fr_setup_part, GAPD_CONN, GAPD_S)(const GImg &g, const FrState &fs, int max_rounds,
                                                           hipStream_t st) {
    return FrSetup<GAPD_CONN, GAPD_S>::run(g, fs, max_rounds, st);
}

hipError_t GAPD_PART_CAT(fr_step_part, GAPD_CONN, GAPD_S)(const GImg &g, const FrState &fs, int max_rounds,
                                                          hipStream_t st, hipEvent_t mid, const Tuning &tune) {
    return FrStep<GAPD_CONN, GAPD_S>::run(g, fs, max_rounds, st, mid, tune);
}

}  // namespace gapd
