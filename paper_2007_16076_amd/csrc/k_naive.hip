// The naive method and multi-source propagations (Section 1): one
// geodesic propagation per source, each writing its row of D; also over
// every (image, source) item of a batch.
#include "dev_common.h"

namespace gapd {

namespace {

// ---------------------------------------------------------------------------------------------
// Naive method / multi-source propagations: block b propagates from
// src_list[b] (or src_base + b) and writes row b of out (Section 1).
// With kGlobal the distance field lives in the output row itself (images too
// large for LDS); otherwise in LDS, and the row is written once at the end.
// PFW: the sweeps' weight prefetch depth (0: the default of 4 lines).
// check1: check the edges after the first round already (smooth images often
// reach the fixed point in one round, and a check costs far less than a
// round); else the second round runs unchecked.
// ---------------------------------------------------------------------------------------------
template <int CONN, int S, bool kGlobal, int PFW = 0>
__global__ __launch_bounds__(kRelaxThreads) void k_relax_rows(GImg g, int Wp, const int32_t *src_list,
                                                              int src_base, int32_t *out, int max_rounds,
                                                              FrCtl *ctl, int check1) {
    extern __shared__ int smem[];
    const int s = src_list ? src_list[blockIdx.x] : src_base + (int)blockIdx.x;
    int32_t *row = out + (size_t)blockIdx.x * g.N;
    int *d = kGlobal ? row : smem;
    const int Wd = kGlobal ? g.W : Wp;
    fill_inf(d, g.H * Wd);
    __syncthreads();
    if (threadIdx.x == 0) d[(s / g.W) * Wd + s % g.W] = 0;
    __syncthreads();
    const int r = relax_block<CONN, S, kGlobal, false, PFW>(g, d, Wd, max_rounds, nullptr, nullptr, nullptr,
                                                            check1 != 0);
    if (threadIdx.x == 0) {
        if (r < 0) atomicExch(&ctl->err, GAPD_ENOCONV);
        atomicAdd((unsigned long long *)&ctl->rounds, (unsigned long long)(r < 0 ? max_rounds : r));
    }
    if (!kGlobal) field_from_lds((uint32_t *)row, d, Wp, g.N, g.W);
}

template <int CONN, int S>
__global__ __launch_bounds__(kRelaxThreads) void k_relax_rows_batched(const BImg *imgs, int B, int32_t *out,
                                                                      int max_rounds, FrCtl *ctl, int check1) {
    extern __shared__ int smem[];
    const int64_t item = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    const int b = find_image(imgs, B, item);
    const BImg &bi = imgs[b];
    const GImg g = bi.g;
    const int s = (int)(item - bi.item0);
    if (s >= g.N) return;  // padding items of the 2-D grid
    const int Wp = bi.Wp;
    int *d = smem;
    fill_inf(d, g.H * Wp);
    __syncthreads();
    if (threadIdx.x == 0) d[(s / g.W) * Wp + s % g.W] = 0;
    __syncthreads();
    const int r = relax_block<CONN, S>(g, d, Wp, max_rounds, nullptr, nullptr, nullptr, check1 != 0);
    if (threadIdx.x == 0) {
        if (r < 0) atomicExch(&ctl->err, GAPD_ENOCONV);
        atomicAdd((unsigned long long *)&ctl->rounds, (unsigned long long)(r < 0 ? max_rounds : r));
    }
    field_from_lds((uint32_t *)(out + bi.out_off + (size_t)s * g.N), d, Wp, g.N, g.W);
}

template <int CONN, int S>
struct RelaxRows {
    static hipError_t run(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                          int max_rounds, FrCtl *ctl, hipStream_t st, int pfw, int check1) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        if (lds <= kMaxLds) {
            auto k = k_relax_rows<CONN, S, false>;
            if constexpr (S <= 128) {  // the deeper weight ring where a lane holds at most two elements
                if (pfw == 8) k = k_relax_rows<CONN, S, false, 8>;
            }
            hipError_t e = set_lds(k, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k, dim3(K), dim3(kRelaxThreads), lds, st, g, Wp, src_list, src_base, out,
                               max_rounds, ctl, check1);
        } else {
            hipLaunchKernelGGL((k_relax_rows<CONN, S, true>), dim3(K), dim3(kRelaxThreads), 0, st, g, g.W,
                               src_list, src_base, out, max_rounds, ctl, check1);
        }
        return hipGetLastError();
    }
};

template <int CONN, int S>
struct RelaxRowsBatched {
    static hipError_t run(const BImg *imgs, int B, int64_t n_items, size_t lds, int32_t *out, int max_rounds,
                          FrCtl *ctl, hipStream_t st, int check1) {
        auto k = k_relax_rows_batched<CONN, S>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        const int64_t gx = n_items < 65536 ? n_items : 65536;
        const int64_t gy = (n_items + gx - 1) / gx;
        hipLaunchKernelGGL(k, dim3((unsigned)gx, (unsigned)gy), dim3(kRelaxThreads), lds, st, imgs, B, out,
                           max_rounds, ctl, check1);
        return hipGetLastError();
    }
};

}  // namespace

// ---- launchers ----------------------------------------------------------------------------------
hipError_t launch_relax_rows(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                             int max_rounds, FrCtl *ctl, hipStream_t st, int pfw, int check1) {
    if (K <= 0) return hipSuccess;
    return dispatch<RelaxRows>(g.conn, g.H > g.W ? g.H : g.W, g, src_list, src_base, K, out, max_rounds, ctl,
                               st, pfw, check1);
}

hipError_t launch_relax_rows_batched(const BImg *imgs_dev, int B, int64_t n_items, int max_line, size_t lds_bytes,
                                     int conn, int32_t *out, int max_rounds, FrCtl *ctl, hipStream_t st,
                                     int check1) {
    if (n_items <= 0) return hipSuccess;
    return dispatch<RelaxRowsBatched>(conn, max_line, imgs_dev, B, n_items, lds_bytes, out, max_rounds, ctl, st,
                                      check1);
}

}  // namespace gapd
