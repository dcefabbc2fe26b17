// The tree-based methods over a batch of images, in lockstep.
#include "dev_common.h"

namespace gapd {

namespace {

__global__ void k_fr_init_b(const BImg *imgs) {
    fr_init_range(imgs[blockIdx.y].fr, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int CONN, int S>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_setup_b(const BImg *imgs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    const BImg &bi = imgs[blockIdx.x];
    fr_setup_block<CONN, S>(bi.g, bi.Wp, bi.fr, smem, max_rounds, red);
}

__global__ void k_rank_b(const BImg *imgs) {
    __shared__ int32_t tile[256];
    const FrState &fs = imgs[blockIdx.y].fr;
    if ((int)(blockIdx.x * blockDim.x) >= fs.N) return;
    rank_block(fs.dbuf, fs.N, fs.rank, fs.order, tile);
}

// Every image of a batch takes its step at once: block b is image b.
template <int CONN, int S, bool kStageW>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_step_b(const BImg *imgs, int max_rounds, int *batch_done) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    // the image's descriptors by value: kept in registers rather than re-read
    // through a pointer (or copied to the stack)
    const GImg g = imgs[blockIdx.x].g;
    const FrState fs = imgs[blockIdx.x].fr;
    fr_step_block<CONN, S, kStageW>(g, imgs[blockIdx.x].Wp, fs, max_rounds, smem, red, batch_done);
}

// Batched fill: blockIdx.y is the image, blockIdx.x a chunk of its pixels.
template <bool kLds, bool kLdsCount>
__global__ __launch_bounds__(256) void k_fr_fill_b(const BImg *imgs) {
    extern __shared__ uint32_t spk[];
    __shared__ int64_t red[4];
    const FrState fs = imgs[blockIdx.y].fr;
    if ((int)(blockIdx.x * blockDim.x) >= fs.N) return;
    fr_fill_block<kLds, kLdsCount>(fs, fs.packed, imgs[blockIdx.y].g.W, spk, red, blockIdx.x,
                                   (fs.N + blockDim.x - 1) / blockDim.x);
}

template <int CONN, int S>
struct FrBatchedSetup {
    static hipError_t run(const BImg *imgs, int B, int maxN, size_t lds, int max_rounds, hipStream_t st) {
        hipLaunchKernelGGL(k_fr_init_b, dim3((maxN + 255) / 256, B), dim3(256), 0, st, imgs);
        auto k = k_fr_setup_b<CONN, S>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(B), dim3(kRelaxThreads), lds, st, imgs, max_rounds);
        hipLaunchKernelGGL(k_rank_b, dim3((maxN + 255) / 256, B), dim3(256), 0, st, imgs);
        return hipGetLastError();
    }
};

template <int CONN, int S>
struct FrBatchedStep {
    static hipError_t run(const BImg *imgs, int B, int maxN, size_t lds, size_t wbytes, int max_rounds,
                          int *batch_done, hipStream_t st) {
        hipError_t e;
        if (lds + wbytes <= kMaxLds) {
            auto k1 = k_fr_step_b<CONN, S, true>;
            e = set_lds(k1, lds + wbytes);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k1, dim3(B), dim3(kRelaxThreads), lds + wbytes, st, imgs, max_rounds, batch_done);
        } else {
            auto k1 = k_fr_step_b<CONN, S, false>;
            e = set_lds(k1, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k1, dim3(B), dim3(kRelaxThreads), lds, st, imgs, max_rounds, batch_done);
        }
        const size_t pk = (size_t)maxN * sizeof(uint32_t);
        const dim3 grid((maxN + 255) / 256, B);
        if (2 * pk <= kMaxLds) {
            auto k2 = k_fr_fill_b<true, true>;
            e = set_lds(k2, 2 * pk);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k2, grid, dim3(256), 2 * pk, st, imgs);
        } else if (pk <= kMaxLds) {
            auto k2 = k_fr_fill_b<true, false>;
            e = set_lds(k2, pk);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k2, grid, dim3(256), pk, st, imgs);
        } else {
            hipLaunchKernelGGL((k_fr_fill_b<false, false>), grid, dim3(256), 0, st, imgs);
        }
        return hipGetLastError();
    }
};

}  // namespace

// ---- launchers ----------------------------------------------------------------------------------
hipError_t launch_fr_batched_setup(const BImg *imgs_dev, int B, int max_line, int maxN, size_t lds, int conn,
                                   int max_rounds, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    return dispatch<FrBatchedSetup>(conn, max_line, imgs_dev, B, maxN, lds, max_rounds, st);
}

hipError_t launch_fr_batched_step(const BImg *imgs_dev, int B, int max_line, int maxN, size_t lds, size_t wbytes,
                                  int conn, int max_rounds, int *batch_done, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    return dispatch<FrBatchedStep>(conn, max_line, imgs_dev, B, maxN, lds, wbytes, max_rounds, batch_done, st);
}

}  // namespace gapd
