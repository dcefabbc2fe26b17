// Edge-weight preparation, workspace layouts and the filling-rate
// initialisation (Section 2: D_mrk = identity, count = 1, D(i,i) = 0).
#include "dev_common.h"

namespace gapd {

namespace {

__global__ void k_prep(GImgW w, const uint8_t *img, int C, int wmode) {
    prep_pixels(w, img, C, wmode, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_prefix(GImgW w) { prefix_lines(w, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x); }

__global__ void k_prep_batched(const GImgW *ws, const uint8_t *imgs, const int64_t *img_off, int C, int wmode) {
    const GImgW w = ws[blockIdx.y];
    prep_pixels(w, imgs + img_off[blockIdx.y], C, wmode, blockIdx.x * blockDim.x + threadIdx.x,
                gridDim.x * blockDim.x);
}

__global__ void k_prefix_batched(const GImgW *ws) {
    const GImgW w = ws[blockIdx.x];
    prefix_lines(w, threadIdx.x, blockDim.x);
}

template <int RULE>
__global__ __launch_bounds__(256) void k_sel_part(FrState fs) {
    sel_part_block<RULE>(fs);
}

__global__ void k_fr_init(FrState fs) { fr_init_range(fs, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x); }

}  // namespace

// ---- layouts (host) ---------------------------------------------------------------------------
size_t weight_block_bytes(int H, int W) {
    const size_t n = (size_t)H * W;
    return 7 * al256(n * 2) + 2 * al256(n * 4);
}

GImgW weight_block_layout(void *dev, int H, int W, int conn) {
    char *p = (char *)dev;
    const size_t n = (size_t)H * W;
    GImgW w;
    w.H = H; w.W = W; w.N = H * W; w.conn = conn;
    uint16_t **u16[7] = {&w.wr, &w.wd, &w.wdr, &w.wdl, &w.cwv, &w.cwdr, &w.cwdl};
    for (auto **q : u16) { *q = (uint16_t *)p; p += al256(n * 2); }
    w.P = (int32_t *)p; p += al256(n * 4);
    w.cP = (int32_t *)p;
    return w;
}

size_t fr_workspace_bytes(int N, bool spec) {
    const size_t MW = ((size_t)N + 31) / 32;
    size_t b = al256((size_t)N * MW * 4) + 7 * al256((size_t)N * 4) + al256(sizeof(FrCtl));
    if (spec)
        b += al256((size_t)kSpecSlots * al4w(N) * 4) + al256((size_t)N * 4) + 2 * al256(kSpecSlots * 4) +
             al256(2 * kSpecK * 4) + al256((size_t)sel_part_waves(N) * (1 + kSelCand) * 8);
    return b;
}

FrState fr_workspace_layout(void *ws, int N, bool spec) {
    char *p = (char *)ws;
    FrState f{};
    f.N = N;
    f.MW = (N + 31) / 32;
    f.mask = (uint32_t *)p; p += al256((size_t)N * f.MW * 4);
    f.count = (int32_t *)p; p += al256((size_t)N * 4);
    f.rank = (int32_t *)p; p += al256((size_t)N * 4);
    f.order = (int32_t *)p; p += al256((size_t)N * 4);
    f.packed = (uint32_t *)p; p += al256((size_t)N * 4);
    f.dbuf = (int32_t *)p; p += al256((size_t)N * 4);
    f.full = (uint32_t *)p; p += al256((size_t)N * 4);
    f.sp_in = (int32_t *)p; p += al256((size_t)N * 4);  // a spiral turn has at most N pixels
    f.ctl = (FrCtl *)p; p += al256(sizeof(FrCtl));
    if (spec) {
        f.cache = (uint32_t *)p; p += al256((size_t)kSpecSlots * al4w(N) * 4);
        f.src_slot = (int32_t *)p; p += al256((size_t)N * 4);
        f.slot_src = (int32_t *)p; p += al256(kSpecSlots * 4);
        f.slot_state = (int32_t *)p; p += al256(kSpecSlots * 4);
        f.spec_list = (int32_t *)p; p += al256(2 * kSpecK * 4);
        f.part = (uint64_t *)p;
    }
    return f;
}

// ---- launchers ----------------------------------------------------------------------------------
hipError_t launch_sel_part(const FrState &fs, hipStream_t st) {
    if (fs.rule == kRuleExtrema)
        hipLaunchKernelGGL(k_sel_part<kRuleExtrema>, dim3(sel_part_blocks(fs.N)), dim3(256), 0, st, fs);
    else
        hipLaunchKernelGGL(k_sel_part<kRuleFilling>, dim3(sel_part_blocks(fs.N)), dim3(256), 0, st, fs);
    return hipGetLastError();
}


hipError_t launch_prep(const GImgW &w, const uint8_t *img_dev, int C, int wmode, hipStream_t st) {
    const int blocks = (w.N + 255) / 256;
    hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st, w, img_dev, C, wmode);
    hipLaunchKernelGGL(k_prefix, dim3((w.H + w.W + 63) / 64), dim3(64), 0, st, w);
    return hipGetLastError();
}

hipError_t launch_prep_batched(const GImgW *w_dev, const uint8_t *imgs_dev, const int64_t *img_off_dev, int B,
                               int C, int wmode, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_batched, dim3(64, B), dim3(256), 0, st, w_dev, imgs_dev, img_off_dev, C, wmode);
    hipLaunchKernelGGL(k_prefix_batched, dim3(B), dim3(256), 0, st, w_dev);
    return hipGetLastError();
}

hipError_t launch_fr_init(const FrState &fs, hipStream_t st) {
    hipLaunchKernelGGL(k_fr_init, dim3((fs.N + 255) / 256), dim3(256), 0, st, fs);
    return hipGetLastError();
}

// ---- tree-method launchers: one object of k_fr.hip per (connectivity, size class) --------------
#define GAPD_FR_PARTS(X) X(4, 32) X(4, 64) X(4, 128) X(4, 192) X(8, 32) X(8, 64) X(8, 128) X(8, 192)
#define GAPD_FR_DECL(C, S)                                                                                   \
    hipError_t fr_setup_part_##C##_##S(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st);   \
    hipError_t fr_step_part_##C##_##S(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st,     \
                                      hipEvent_t mid, const Tuning &tune);
GAPD_FR_PARTS(GAPD_FR_DECL)

hipError_t launch_fr_setup(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
    const int c = size_class(g.H > g.W ? g.H : g.W);
#define GAPD_FR_SETUP_CASE(C, S) \
    if (g.conn == C && c == S) return fr_setup_part_##C##_##S(g, fs, max_rounds, st);
    GAPD_FR_PARTS(GAPD_FR_SETUP_CASE)
    return hipErrorInvalidValue;  // the tree methods need the distance field in LDS (sides <= 192)
}

hipError_t launch_fr_step(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st, hipEvent_t mid,
                          const Tuning &tune) {
    const int c = size_class(g.H > g.W ? g.H : g.W);
#define GAPD_FR_STEP_CASE(C, S) \
    if (g.conn == C && c == S) return fr_step_part_##C##_##S(g, fs, max_rounds, st, mid, tune);
    GAPD_FR_PARTS(GAPD_FR_STEP_CASE)
    return hipErrorInvalidValue;
}

}  // namespace gapd
