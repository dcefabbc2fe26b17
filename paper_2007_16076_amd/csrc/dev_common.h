// Device code shared by the HIP translation units of libgapd.so (gfx950,
// CDNA4, wave64): edge weights of the pseudo-metric (Section 2, eq.
// distance_somme; 1 + L1 for multiband images), geodesic propagation as the
// fixed point of min-plus sweeps in LDS (Section 2, eqs. temps and distance),
// the geodesic tree (each pixel's parent is its smallest-index tight
// neighbour), the source-selection rules (Sections 3.1-3.4) and the
// redundancy fill along a tree (Property 1).  Everything here has internal
// linkage; each translation unit instantiates what its kernels use.
//
// No MFMA: the work is integer min-plus, not a dense contraction.
#pragma once
#include "gapd_internal.h"
#include "gapd.h"

#pragma clang diagnostic ignored "-Wunused-function"

namespace gapd {

namespace {

constexpr int kBig = 0x7FFFFFFF;

// Tree word of a pixel for one propagation: bits 0-3 the parent direction
// code (kRootCode at the root), bit 4 set when the pixel's row of the
// filled-pairs matrix was already complete before this step, bits 5-31 the
// distance from the source (< 2^27).
constexpr uint32_t kFilledBit = 16u;

// Slot states of the tree cache.
constexpr int kSlotFree = 0;     // no tree
constexpr int kSlotReady = 1;    // holds the tree words of slot_src
constexpr int kSlotRunning = 2;  // holds the partial distance field of slot_src's propagation

// floor(v / W) by a multiply: with m = floor(2^32 / W) + 1, (v * m) >> 32 is
// exact for v < 2^18 and W <= 512 (the product exceeds v / W by less than
// v / 2^32 < 1 / W).
__device__ __forceinline__ uint64_t divw_magic(int W) { return (1ull << 32) / (uint64_t)W + 1ull; }
__device__ __forceinline__ int divw(int v, uint64_t m) { return (int)(((uint64_t)(uint32_t)v * m) >> 32); }

__host__ __device__ inline uint32_t tree_word(int d, uint32_t code) { return ((uint32_t)d << 5) | code; }
__host__ __device__ inline int tw_dist(uint32_t w) { return (int)(w >> 5); }
__host__ __device__ inline uint32_t tw_code(uint32_t w) { return w & 15u; }

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Tree-cache slot sl: its tree words, or while running its partial distance field.
// Slots are al4w(N) words apart, so every tree starts 16-byte aligned.
__device__ __forceinline__ uint32_t *slot_tree(const FrState &fs, int sl) { return fs.cache + (size_t)sl * al4w(fs.N); }

// Constant-clock timestamp (100 MHz) for the optional per-step trace.
__device__ __forceinline__ int64_t trace_clock() { return (int64_t)wall_clock64(); }

// ---------------------------------------------------------------------------------------------
// Edge weights (Section 2, pseudo-metrics).
// ---------------------------------------------------------------------------------------------
__device__ inline int edge_weight(const uint8_t *img, int C, int wmode, int p, int q) {
    if (wmode == GAPD_W_SUM) return int(img[p]) + int(img[q]);
    int s = 1;
    for (int b = 0; b < C; ++b) s += abs(int(img[(size_t)p * C + b]) - int(img[(size_t)q * C + b]));
    return s;
}

__device__ void prep_pixels(const GImgW &w, const uint8_t *img, int C, int wmode, int v0, int stride) {
    const int H = w.H, W = w.W;
    for (int v = v0; v < w.N; v += stride) {
        const int y = v / W, x = v - (v / W) * W;
        const bool r = x + 1 < W, dn = y + 1 < H;
        const int wr = r ? edge_weight(img, C, wmode, v, v + 1) : 0;
        const int wd = dn ? edge_weight(img, C, wmode, v, v + W) : 0;
        const int wdr = (r && dn) ? edge_weight(img, C, wmode, v, v + W + 1) : 0;
        const int wdl = (dn && x >= 1) ? edge_weight(img, C, wmode, v, v + W - 1) : 0;
        w.wr[v] = (uint16_t)wr;
        w.wd[v] = (uint16_t)wd;
        w.wdr[v] = (uint16_t)wdr;
        w.wdl[v] = (uint16_t)wdl;
        // Column view: line x, element y.  Its "down" edges are the image's
        // right edges; its dr edges are the image's dr edges; its dl edge at
        // (line x, element y) joins image pixels (y, x) and (y-1, x+1).
        const int cv = x * H + y;
        w.cwv[cv] = (uint16_t)wr;
        w.cwdr[cv] = (uint16_t)wdr;
        w.cwdl[cv] = (uint16_t)((y >= 1 && r) ? edge_weight(img, C, wmode, v - W + 1, v) : 0);
    }
}


__device__ void prefix_lines(const GImgW &w, int t0, int stride) {
    const int H = w.H, W = w.W;
    for (int t = t0; t < H + W; t += stride) {
        if (t < H) {
            int acc = 0;
            for (int x = 0; x < W; ++x) { w.P[t * W + x] = acc; acc += w.wr[t * W + x]; }
        } else {
            const int x = t - H;
            int acc = 0;
            for (int y = 0; y < H; ++y) { w.cP[x * H + y] = acc; acc += w.wd[y * W + x]; }
        }
    }
}


// ---------------------------------------------------------------------------------------------
// Wave-level min scans over 64 lanes (DPP row shifts inside each 16-lane row,
// readlane for the carries between rows).
// ---------------------------------------------------------------------------------------------
// Distance-field load.  The field in global memory is updated by atomics
// performed in L2, so its reads bypass the per-CU L1 (agent scope); in LDS a
// workgroup-scope relaxed load is a plain ds_read.
template <bool G>
__device__ __forceinline__ int ldd(const int *p) {
    if (G) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Block-wide copy of n words from global memory into LDS: 16-byte loads, U
// in flight per thread before any is stored.  The stores take the same
// clamped index as the loads, so lanes past the end rewrite the last element
// with its own value: no branch, which keeps the compiler from moving each
// load next to its store (and waiting for it there).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int U = 8>
__device__ __forceinline__ void copy_to_lds(uint32_t *dst, const uint32_t *src, int n) {
    typedef const __attribute__((address_space(1))) u32x4 *gptr4;  // global memory: plain vector loads
    const int n4 = n / 4;
    const gptr4 s4 = (gptr4)src;
    u32x4 *d4 = reinterpret_cast<u32x4 *>(dst);
    const int nb = (int)blockDim.x;
    for (int base = threadIdx.x; base < n4; base += nb * U) {
        u32x4 t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) t[k] = s4[min(base + k * nb, n4 - 1)];
#pragma unroll
        for (int k = 0; k < U; ++k) d4[min(base + k * nb, n4 - 1)] = t[k];
    }
    for (int i = n4 * 4 + threadIdx.x; i < n; i += nb) dst[i] = src[i];
}

template <int CTRL>
__device__ __forceinline__ int dpp_mov(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}

// Lane masks of the 16-lane DPP row a lane sits in (row = lane / 16), used to
// pick the carry of the rows before / after it without branching.
struct RowMasks {
    int ge1, ge2, ge3, le0, le1, le2;
    __device__ explicit RowMasks(int row)
        : ge1(row >= 1 ? -1 : 0), ge2(row >= 2 ? -1 : 0), ge3(row >= 3 ? -1 : 0),
          le0(row <= 0 ? -1 : 0), le1(row <= 1 ? -1 : 0), le2(row <= 2 ? -1 : 0) {}
};

__device__ __forceinline__ int sel(int mask, int a, int b) { return (a & mask) | (b & ~mask); }

// Both exclusive scans at once: x = prefix minimum over lanes < l of p,
// y = suffix minimum over lanes > l of q.  Interleaving the two dependency
// chains hides most of the DPP latency.  The prefix scan crosses the 16-lane
// rows with the row broadcasts of lanes 15 and 31 and shifts by one lane over
// the whole wave; the suffix scan takes the first lane of each later row by
// readlane.
__device__ __forceinline__ int2 wave_excl_scans(int p, int q, const RowMasks &m) {
    p = min(p, dpp_mov<0x111>(kBig, p));
    q = min(q, dpp_mov<0x101>(kBig, q));
    p = min(p, dpp_mov<0x112>(kBig, p));
    q = min(q, dpp_mov<0x102>(kBig, q));
    p = min(p, dpp_mov<0x114>(kBig, p));
    q = min(q, dpp_mov<0x104>(kBig, q));
    p = min(p, dpp_mov<0x118>(kBig, p));
    q = min(q, dpp_mov<0x108>(kBig, q));
    // rows 1 and 3 take lane 15 of the row before, rows 2 and 3 lane 31
    p = min(p, __builtin_amdgcn_update_dpp(kBig, p, 0x142, 0xA, 0xF, false));
    const int b1 = __builtin_amdgcn_readlane(q, 16);
    const int b2 = __builtin_amdgcn_readlane(q, 32);
    const int b3 = __builtin_amdgcn_readlane(q, 48);
    p = min(p, __builtin_amdgcn_update_dpp(kBig, p, 0x143, 0xC, 0xF, false));
    const int b23 = min(b2, b3), b123 = min(b1, b23);
    q = min(q, sel(m.le0, b123, sel(m.le1, b23, sel(m.le2, b3, kBig))));
    // exclusive: the inclusive value of the lane before (wave_shr:1) / after (wave_shl:1)
    return make_int2(__builtin_amdgcn_update_dpp(kBig, p, 0x138, 0xF, 0xF, false),
                     __builtin_amdgcn_update_dpp(kBig, q, 0x130, 0xF, 0xF, false));
}

// base[idx] with the byte offset computed in 32 bits (arrays under 4 GiB), so
// that the load takes a scalar base and a 32-bit vector offset.
template <typename T>
__device__ __forceinline__ T ld_off(const T *__restrict__ base, uint32_t idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (idx * (uint32_t)sizeof(T)));
}

// A field of N values in pixel order (row stride W) from global memory into
// LDS rows of stride Wp, and back: U values per thread per batch, all loads of
// a batch issued before its stores.  Indices past the end are clamped (a
// repeated copy of the last value).
template <int U = 8>
__device__ __forceinline__ void field_to_lds(int *d, int Wp, const uint32_t *__restrict__ src, int N, int W) {
    const uint64_t mW = divw_magic(W);
    const int nb = (int)blockDim.x;
    for (int base = threadIdx.x; base < N; base += nb * U) {
        uint32_t t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) t[k] = ld_off(src, (uint32_t)min(base + k * nb, N - 1));
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int v = min(base + k * nb, N - 1), y = divw(v, mW);
            d[y * Wp + (v - y * W)] = (int)t[k];
        }
    }
}

template <int U = 8>
__device__ __forceinline__ void field_from_lds(uint32_t *dst, const int *d, int Wp, int N, int W) {
    const uint64_t mW = divw_magic(W);
    const int nb = (int)blockDim.x;
    for (int base = threadIdx.x; base < N; base += nb * U) {
        int t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int v = min(base + k * nb, N - 1), y = divw(v, mW);
            t[k] = d[y * Wp + (v - y * W)];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) dst[min(base + k * nb, N - 1)] = (uint32_t)t[k];
    }
}

// Inputs of one line of a sweep, prefetched into registers.
template <int C>
struct LineIn {
    int P[C];    // running weight sum along the line
    int wc[C];   // cross edge from the previous line, same element
    int wm[C];   // 8-neighbours: cross edge from element e-1 of the previous line
    int wp[C];   // 8-neighbours: cross edge from element e+1 of the previous line
};

// ---------------------------------------------------------------------------------------------
// One directional sweep over all lines of a view (rows of the image, or rows
// of its transpose = columns).  Line l is relaxed from the previous line of
// the sweep (cross edges), then exactly along itself: with R[e] the running
// weight sum along the line, min_{e'}(a[e'] + |R[e]-R[e']|) is a prefix
// minimum of a - R plus R and a suffix minimum of a + R minus R.  A lane owns
// C consecutive elements.  Stores go through an atomic min, so the four
// sweeps of a round may run concurrently on the same distance field: every
// stored value is the length of a real path, and values only decrease.
// Line weights are loaded PF lines ahead into a register ring (PFW, or 4
// by default: a lone workgroup per compute unit wants a deeper ring to cover
// the L2 latency), the field values at most 4 lines ahead, so they are read
// as late as possible; all addresses are clamped into the image, so the loads
// are unconditional.  FULL says that every line has exactly 64 * C elements,
// so no lane owns a slot past its end and the clamps drop out.  Returns true
// if this wave lowered a value it had read.
// ---------------------------------------------------------------------------------------------
template <int CONN, int C, bool FWD, bool G, int PFW = 0, bool FULL = false>
__device__ __forceinline__ bool sweep(int *d, int ls, int es, int NL, int L, const uint16_t *__restrict__ wv,
                      const uint16_t *__restrict__ wdr, const uint16_t *__restrict__ wdl,
                      const int32_t *__restrict__ P) {
    constexpr int PF = PFW > 0 ? PFW : (C <= 4 ? 4 : 2);
    constexpr int PD = PF < 4 ? PF : 4;
    static_assert(PF % PD == 0, "the weight ring must be a multiple of the field ring");
    const int lane = __lane_id();
    const RowMasks rm(lane >> 4);
    const int e0 = lane * C;
    int ec[C], em[C], ep[C], es_[C];
    bool ok[C], okm[C], okp[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int e = e0 + j;
        ok[j] = FULL || e < L;
        ec[j] = ok[j] ? e : L - 1;
        // store address: lanes past the end of the line spread over the line
        // (their atomic min of kInf changes nothing) instead of all hitting
        // its last element
        es_[j] = ok[j] ? e : e % L;
        okm[j] = ok[j] && e > 0;
        okp[j] = e + 1 < L;
        em[j] = okm[j] ? e - 1 : ec[j];
        ep[j] = okp[j] ? e + 1 : ec[j];
    }
    auto loadd = [&](int (&cur)[C], int step) {
        const int l = FWD ? step : NL - 1 - step;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int v = ldd<G>(&d[l * ls + ec[j] * es]);
            cur[j] = ok[j] ? v : kInf;
        }
    };
    // weight and prefix-sum offsets as unsigned 32-bit indices, so that the
    // loads take a scalar base plus a 32-bit vector offset
    auto load = [&](LineIn<C> &in, int step) {
        const int l = FWD ? step : NL - 1 - step;
        const int top = FWD ? (l > 0 ? l - 1 : 0) : l;  // line holding the cross edges into l
        const uint32_t lo = (uint32_t)(l * L), to = (uint32_t)(top * L);
#pragma unroll
        for (int j = 0; j < C; ++j) {
            in.P[j] = ld_off(P, lo + (uint32_t)ec[j]);
            in.wc[j] = ld_off(wv, to + (uint32_t)ec[j]);
            if (CONN == 8) {
                const int a = FWD ? ld_off(wdr, to + (uint32_t)em[j]) : ld_off(wdl, lo + (uint32_t)ec[j]);
                const int b = FWD ? ld_off(wdl, to + (uint32_t)ep[j]) : ld_off(wdr, lo + (uint32_t)ec[j]);
                in.wm[j] = okm[j] ? a : kInf;
                in.wp[j] = okp[j] ? b : kInf;
            }
        }
    };
    int prev[C];
    uint32_t chg = 0;
    auto process = [&](const LineIn<C> &in, const int (&cur)[C], int step, bool first) {
        const int l = FWD ? step : NL - 1 - step;
        int a[C], t[C];
#pragma unroll
        for (int j = 0; j < C; ++j) a[j] = first ? cur[j] : min(cur[j], prev[j] + in.wc[j]);
        if (CONN == 8 && !first) {
            int left_in = __shfl_up(prev[C - 1], 1);
            int right_in = __shfl_down(prev[0], 1);
            left_in = lane == 0 ? kInf : left_in;
            right_in = lane == 63 ? kInf : right_in;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int pm = j > 0 ? prev[j - 1] : left_in;
                const int pp = j < C - 1 ? prev[j + 1] : right_in;
                a[j] = min(a[j], min(pm + in.wm[j], pp + in.wp[j]));
            }
        }
        // Along the line: paths from e' <= e (prefix minimum of a - R) and
        // from e' >= e (suffix minimum of a + R) are independent, so the two
        // scans run interleaved.
        int u[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            t[j] = a[j] - in.P[j];
            u[j] = a[j] + in.P[j];
        }
#pragma unroll
        for (int j = 1; j < C; ++j) {
            t[j] = min(t[j], t[j - 1]);
            u[C - 1 - j] = min(u[C - 1 - j], u[C - j]);
        }
        const int2 ex = wave_excl_scans(t[C - 1], u[0], rm);
        // Lanes past the end of the line hold kInf: their atomic min changes
        // nothing, so every store is unconditional.
#pragma unroll
        for (int j = 0; j < C; ++j) {
            a[j] = ok[j] ? min(min(t[j], ex.x) + in.P[j], min(u[j], ex.y) - in.P[j]) : kInf;
            chg |= (uint32_t)(a[j] < cur[j]);
            atomicMin(&d[l * ls + es_[j] * es], a[j]);
            prev[j] = a[j];
        }
    };
    // Rings of prefetched lines: weight slot (step % PF) and field slot
    // (step % PD) hold line `step`.  Line indices past the end are clamped to
    // the last line, so every load in the steady-state loop is unconditional
    // and the wait counters stay exact.
    LineIn<C> S[PF];
    int F[PD][C];
#pragma unroll
    for (int i = 0; i < PF; ++i) load(S[i], min(i, NL - 1));
#pragma unroll
    for (int i = 0; i < PD; ++i) loadd(F[i], min(i, NL - 1));
    process(S[0], F[0], 0, true);
    load(S[0], min(PF, NL - 1));
    loadd(F[0], min(PD, NL - 1));
    int base = 1;
    for (; base + PF <= NL; base += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int step = base + k;
            process(S[(1 + k) % PF], F[(1 + k) % PD], step, false);
            load(S[(1 + k) % PF], min(step + PF, NL - 1));
            loadd(F[(1 + k) % PD], min(step + PD, NL - 1));
        }
    }
#pragma unroll
    for (int k = 0; k < PF - 1; ++k)
        if (base + k < NL) {
            process(S[(1 + k) % PF], F[(1 + k) % PD], base + k, false);
            loadd(F[(1 + k) % PD], min(base + k + PD, NL - 1));
        }
    return chg != 0;
}

// Neighbour k of pixel (y, x), in ascending pixel-index order:
// 0:(-1,-1) 1:(-1,0) 2:(-1,+1) 3:(0,-1) 4:(0,+1) 5:(+1,-1) 6:(+1,0) 7:(+1,+1).
// The 4-neighbourhood uses codes 1, 3, 4, 6.
// Decoded without branches: 2 bits per code hold dy + 1 and dx + 1; the root
// code (15) decodes to (0, 0), so its "parent" offset is 0.
constexpr uint32_t kCodeDy1 = 0u | 0u << 2 | 0u << 4 | 1u << 6 | 1u << 8 | 2u << 10 | 2u << 12 | 2u << 14 | 1u << 30;
constexpr uint32_t kCodeDx1 = 0u | 1u << 2 | 2u << 4 | 0u << 6 | 2u << 8 | 0u << 10 | 1u << 12 | 2u << 14 | 1u << 30;
__device__ __forceinline__ int code_dy(int k) { return (int)((kCodeDy1 >> (2 * k)) & 3u) - 1; }
__device__ __forceinline__ int code_dx(int k) { return (int)((kCodeDx1 >> (2 * k)) & 3u) - 1; }
// Pixel-index offset of neighbour k in an image of width W (< 2^23).
__device__ __forceinline__ int code_off(int k, int W) { return __mul24(code_dy(k), W) + code_dx(k); }

template <int CONN>
__device__ __forceinline__ bool code_used(int k) {
    return CONN == 8 || k == 1 || k == 3 || k == 4 || k == 6;
}

// The four edge-weight arrays of the 4-/8-neighbourhood, from global memory
// or from an LDS copy.
struct NbW {
    const uint16_t *wr, *wd, *wdr, *wdl;
};
__device__ inline NbW nbw_of(const GImg &g) { return NbW{g.wr, g.wd, g.wdr, g.wdl}; }

// Path lengths into (y, x) through each neighbour k: d(q) + w(q, v), or kBig
// where there is no such neighbour.  Loads use clamped in-image addresses and
// are issued unconditionally; absent neighbours are masked afterwards.
template <int CONN, bool G>
__device__ __forceinline__ void neighbour_paths(const GImg &g, const NbW &w, const int *d, int Wp, int y, int x,
                                                int cand[8]) {
    const int H = g.H, W = g.W;
    const bool up = y > 0, dn = y + 1 < H, lf = x > 0, rt = x + 1 < W;
    const int yu = up ? y - 1 : y, yd = dn ? y + 1 : y, xl = lf ? x - 1 : x, xr = rt ? x + 1 : x;
    const int du = ldd<G>(&d[yu * Wp + x]), dl = ldd<G>(&d[y * Wp + xl]);
    const int dr = ldd<G>(&d[y * Wp + xr]), dd = ldd<G>(&d[yd * Wp + x]);
    const uint32_t ou = (uint32_t)(yu * W), oy = (uint32_t)(y * W);
    const int wu = ld_off(w.wd, ou + x), wl = ld_off(w.wr, oy + xl), wr = ld_off(w.wr, oy + x),
              wdn = ld_off(w.wd, oy + x);
    cand[1] = up ? du + wu : kBig;
    cand[3] = lf ? dl + wl : kBig;
    cand[4] = rt ? dr + wr : kBig;
    cand[6] = dn ? dd + wdn : kBig;
    if (CONN == 8) {
        const int dul = ldd<G>(&d[yu * Wp + xl]), dur = ldd<G>(&d[yu * Wp + xr]);
        const int ddl = ldd<G>(&d[yd * Wp + xl]), ddr = ldd<G>(&d[yd * Wp + xr]);
        const int wul = ld_off(w.wdr, ou + xl), wur = ld_off(w.wdl, ou + xr);
        const int wdl_ = ld_off(w.wdl, oy + x), wdr_ = ld_off(w.wdr, oy + x);
        cand[0] = (up && lf) ? dul + wul : kBig;
        cand[2] = (up && rt) ? dur + wur : kBig;
        cand[5] = (dn && lf) ? ddl + wdl_ : kBig;
        cand[7] = (dn && rt) ? ddr + wdr_ : kBig;
    } else {
        cand[0] = cand[2] = cand[5] = cand[7] = kBig;
    }
}

// One pass over every pixel of the field: true if some edge still relaxes a
// distance.  With TREE it also writes each pixel's tree word (its distance
// and the code of its geodesic-tree parent: the first neighbour, in
// ascending index order, with d(q) + w(q, v) == d(v); kRootCode at distance
// 0) to tree[v]; once a pass finds no relaxable edge these words are final.
// Each thread takes U pixels at a time so that their loads overlap.
template <int CONN, bool G, bool TREE>
__device__ bool field_check(const GImg &g, const NbW &w, const int *d, int Wp, uint32_t *tree) {
    constexpr int U = 8;
    bool bad = false;
    const int N = g.N, W = g.W;
    const uint64_t mW = divw_magic(W);
    for (int base = threadIdx.x; base < N; base += blockDim.x * U) {
        int m[U], dv[U];
        uint32_t code[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int v = min(base + k * (int)blockDim.x, N - 1);
            const int y = divw(v, mW), x = v - y * W;
            int cand[8];
            neighbour_paths<CONN, G>(g, w, d, Wp, y, x, cand);
            dv[k] = ldd<G>(&d[y * Wp + x]);
            m[k] = cand[0];
#pragma unroll
            for (int j = 1; j < 8; ++j) m[k] = min(m[k], cand[j]);
            if (TREE) {
                code[k] = kRootCode;
#pragma unroll
                for (int j = 7; j >= 0; --j) code[k] = cand[j] == dv[k] ? (uint32_t)j : code[k];
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            bad |= m[k] < dv[k];
            if (TREE && base + k * (int)blockDim.x < N) tree[base + k * blockDim.x] = tree_word(dv[k], code[k]);
        }
    }
    return bad;
}

// Geodesic-tree parent of (y, x) (see field_check).
template <int CONN>
__device__ uint32_t parent_code(const GImg &g, const int *d, int Wp, int y, int x, int dv) {
    int cand[8];
    neighbour_paths<CONN, false>(g, nbw_of(g), d, Wp, y, x, cand);
    uint32_t code = kRootCode;
#pragma unroll
    for (int k = 7; k >= 0; --k) code = cand[k] == dv ? (uint32_t)k : code;
    return code;
}

// ---------------------------------------------------------------------------------------------
// One geodesic propagation by the whole workgroup (256 threads) on the
// distance field d (H rows of stride Wp; LDS or global).  d must already hold
// kInf everywhere except the seeds (0).  Each round runs the four directional
// sweeps concurrently, one wave each; after a round that changed something,
// a parallel check of every edge decides whether the fixed point is reached.
// Returns the number of rounds, or -1 if max_rounds was hit.
// ---------------------------------------------------------------------------------------------
// S is the size class of the image (its longer side is at most S); each
// lane owns C = S / 64 elements of a line (at least one).
//
// With TREE the edge checks also write the tree words to tree[]; *tree_done
// tells whether the last check (the one that ended the loop) wrote them.
//
// PFW is the sweeps' weight prefetch depth (0: the default).  With
// check_first the edge check also runs after the first round: a field resumed
// from an earlier round may already be the fixed point.  FULLOK allows the
// sweeps' full-line variant (more code; a kernel that inlines several
// propagations turns it off to stay within its registers).
template <int CONN, int S, bool G = false, bool TREE = false, int PFW = 0, bool FULLOK = true>
__device__ __forceinline__ int relax_block(const GImg &g, int *d, int Wp, int max_rounds, const NbW *nw = nullptr,
                                          uint32_t *tree = nullptr, bool *tree_done = nullptr,
                                          bool check_first = false) {
    constexpr int C = S >= 64 ? S / 64 : 1;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    // lines that fill every lane slot (rows of length W, columns of length H)
    const bool full_rows = FULLOK && S >= 64 && g.W == 64 * C, full_cols = FULLOK && S >= 64 && g.H == 64 * C;
    int rounds = 0;
    for (;;) {
        bool ch = false;
        if (wave == 0)
            ch = full_rows ? sweep<CONN, C, true, G, PFW, true>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P)
                           : sweep<CONN, C, true, G, PFW>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P);
        else if (wave == 1)
            ch = full_rows ? sweep<CONN, C, false, G, PFW, true>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P)
                           : sweep<CONN, C, false, G, PFW>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P);
        else if (wave == 2)
            ch = full_cols ? sweep<CONN, C, true, G, PFW, true>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP)
                           : sweep<CONN, C, true, G, PFW>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP);
        else if (wave == 3)
            ch = full_cols ? sweep<CONN, C, false, G, PFW, true>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP)
                           : sweep<CONN, C, false, G, PFW>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP);
        ++rounds;
        if (!__syncthreads_or(ch)) break;
        // A first round that changed anything is almost never the fixed point
        // (paths with turns need a second one): sweep again before checking.
        if (rounds == 1 && !check_first) {
            if (rounds >= max_rounds) return -1;
            continue;
        }
        const NbW w = nw ? *nw : nbw_of(g);
        if (!__syncthreads_or(field_check<CONN, G, TREE>(g, w, d, Wp, tree))) {
            if (TREE) *tree_done = true;
            break;
        }
        if (rounds >= max_rounds) return -1;
    }
    return rounds;
}

__device__ void fill_inf(int *d, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = kInf;
}

// Block-wide minimum of a 64-bit key (all threads get the result).
__device__ uint64_t block_min_u64(uint64_t k, uint64_t *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(k, off);
        k = o < k ? o : k;
    }
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) red[wave] = k;
    __syncthreads();
    uint64_t r = red[0];
    for (int i = 1; i < nw; ++i) r = red[i] < r ? red[i] : r;
    __syncthreads();
    return r;
}

// Block-wide sum of a 64-bit value (all threads get the result).
__device__ int64_t block_sum_i64(int64_t v, int64_t *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) red[wave] = v;
    __syncthreads();
    int64_t r = 0;
    for (int i = 0; i < nw; ++i) r += red[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------------------------
// Filling-rate method, one image.
// ---------------------------------------------------------------------------------------------

// D_mrk(i,i) = 1, count = 1, D(i,i) = 0 (Section 2; the filled-pairs matrix
// must already be zero).
__device__ void fr_init_range(const FrState &fs, int i0, int stride) {
    if (fs.src_slot)
        for (int i = i0; i < (fs.N > kSpecSlots ? fs.N : kSpecSlots); i += stride) {
            if (i < fs.N) fs.src_slot[i] = -1;
            if (i < kSpecSlots) {
                fs.slot_src[i] = -1;
                fs.slot_state[i] = kSlotFree;
            }
        }
    for (int i = i0; i < fs.N; i += stride) {
        fs.mask[(size_t)i * fs.MW + (i >> 5)] = 1u << (i & 31);
        fs.count[i] = 1;
        fs.D[(size_t)i * fs.N + i] = 0;
        if ((i & 31) == 0) fs.full[i >> 5] = fs.N == 1 ? 1u : 0u;
    }
}

// count[i] += inc, keeping the complete-row bitmap in step: the addition
// that brings the count to N sets bit i.
__device__ __forceinline__ void count_add(const FrState &fs, int i, int inc) {
    const int old = atomicAdd(&fs.count[i], inc);
    if (old < fs.N && old + inc >= fs.N) atomicOr(&fs.full[i >> 5], 1u << (i & 31));
}

// Geodesic centroid and the propagation from it (Section 3.3): propagate from
// every border pixel, take the first pixel of maximal distance as the
// centroid c, propagate from c into fs.dbuf.  One block.
template <int CONN, int S>
__device__ void fr_setup_block(const GImg &g, int Wp, const FrState &fs, int *d, int max_rounds,
                               uint64_t *red) {
    const int H = g.H, W = g.W, N = g.N;
    fill_inf(d, H * Wp);
    __syncthreads();
    for (int v = threadIdx.x; v < N; v += blockDim.x) {
        const int y = v / W, x = v - y * W;
        if (y == 0 || y == H - 1 || x == 0 || x == W - 1) d[y * Wp + x] = 0;
    }
    __syncthreads();
    int r1 = relax_block<CONN, S, false, false, 0, false>(g, d, Wp, max_rounds);
    // argmax with ties to the smallest index: minimise (INF - d, index)
    uint64_t best = ~0ull;
    for (int v = threadIdx.x; v < N; v += blockDim.x) {
        const int y = v / W, x = v - y * W;
        const uint64_t key = ((uint64_t)(uint32_t)(kInf - d[y * Wp + x]) << 32) | (uint32_t)v;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, red);
    const int c = (int)(best & 0xFFFFFFFFu);
    fill_inf(d, H * Wp);
    __syncthreads();
    if (threadIdx.x == 0) d[(c / W) * Wp + c % W] = 0;
    __syncthreads();
    int r2 = relax_block<CONN, S, false, false, 0, false>(g, d, Wp, max_rounds);
    for (int v = threadIdx.x; v < N; v += blockDim.x) {
        const int y = v / W, x = v - y * W;
        fs.dbuf[v] = d[y * Wp + x];
    }
    if (threadIdx.x == 0) {
        fs.ctl->centroid = c;
        if (r1 < 0 || r2 < 0) fs.ctl->err = GAPD_ENOCONV;
        fs.ctl->rounds += (r1 < 0 ? max_rounds : r1) + (r2 < 0 ? max_rounds : r2);
    }
}

// rank[x] = position of x in the list sorted by decreasing d_c, ties by
// increasing index (Section 3.3); order = inverse permutation.  Brute-force
// counting over all pairs (N^2 comparisons, once per run).
__device__ void rank_block(const int32_t *dc, int N, int32_t *rank, int32_t *order, int32_t *tile) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int dx = x < N ? dc[x] : 0;
    int cnt = 0;
    for (int base = 0; base < N; base += 256) {
        __syncthreads();
        if (base + (int)threadIdx.x < N) tile[threadIdx.x] = dc[base + threadIdx.x];
        __syncthreads();
        const int lim = min(256, N - base);
        for (int k = 0; k < lim; ++k) {
            const int dy = tile[k], y = base + k;
            cnt += (dy > dx) || (dy == dx && y < x);
        }
    }
    if (x < N) { rank[x] = cnt; order[cnt] = x; }
}

__global__ void k_rank(const int32_t *dc, int N, int32_t *rank, int32_t *order) {
    __shared__ int32_t tile[256];
    rank_block(dc, N, rank, order, tile);
}

// Least filled point (Section 3.4): argmin over x of (count[x], rank[x]).
// Returns the pixel, or -1 when that point is filled (D is complete).
// Selection keys of the deterministic rules; the smaller key wins.
//   filling rate (Section 3.4): count, then rank in the extrema list, 19 + 19
//     bits.  A point whose row is complete keeps its key: the loop ends when
//     the least key belongs to such a point.
//   extrema (Section 3.3): distance from the centroid (greatest first), then
//     count, then index, 27 + 18 + 18 bits.  Points whose rows are complete
//     are left out (kNoKey).
constexpr uint64_t kNoKey = ~0ull;
constexpr uint64_t kDcMax = (1u << 27) - 1;

template <int RULE>
__device__ __forceinline__ const int32_t *sel_aux(const FrState &fs) {
    return RULE == kRuleFilling ? fs.rank : fs.dbuf;
}

template <int RULE>
__device__ __forceinline__ uint64_t sel_key(const FrState &fs, int x, int c, int aux) {
    if (RULE == kRuleFilling) return ((uint64_t)(uint32_t)c << 19) | (uint32_t)aux;
    if (c >= fs.N) return kNoKey;
    return ((kDcMax - (uint32_t)aux) << 36) | ((uint64_t)(uint32_t)c << 18) | (uint32_t)x;
}

template <int RULE>
__device__ __forceinline__ bool key_done(const FrState &fs, uint64_t k) {
    return RULE == kRuleFilling ? (int)(k >> 19) >= fs.N : k == kNoKey;
}

template <int RULE>
__device__ __forceinline__ int key_point(const FrState &fs, uint64_t k) {
    return RULE == kRuleFilling ? fs.order[(int)(k & 0x7FFFFu)] : (int)(k & 0x3FFFFu);
}

// A coarser key of at most 46 bits that orders points the same way up to
// ties (for the cache's eviction order, a heuristic).
template <int RULE>
__device__ __forceinline__ uint64_t key_heur(uint64_t k) {
    return RULE == kRuleFilling ? k : k >> 18;
}

// The source of the step by a deterministic rule, -1 when D is filled.
template <int RULE>
__device__ int fr_select(const FrState &fs, uint64_t *red) {
    constexpr int U = 16;  // independent loads in flight per thread
    const int32_t *aux = sel_aux<RULE>(fs);
    uint64_t best = kNoKey;
    const int step = blockDim.x * U;
    for (int base = threadIdx.x; base < fs.N; base += step) {
        int c[U], a[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int x = min(base + k * (int)blockDim.x, fs.N - 1);
            c[k] = fs.count[x];
            a[k] = aux[x];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int x = min(base + k * (int)blockDim.x, fs.N - 1);
            const uint64_t key = sel_key<RULE>(fs, x, c[k], a[k]);
            best = key < best ? key : best;  // clamped duplicates change nothing
        }
    }
    best = block_min_u64(best, red);
    if (key_done<RULE>(fs, best)) return -1;
    return key_point<RULE>(fs, best);
}

// Block-wide exclusive prefix sum in thread order (red: one slot per wave);
// *total (optional) receives the block's sum.
__device__ int block_excl_scan(int v, int64_t *red, int *total = nullptr) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wave] = x;
    __syncthreads();
    int base = 0, all = 0;
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 0; w < nw; ++w) {
        const int r = (int)red[w];
        base += w < wave ? r : 0;
        all += r;
    }
    __syncthreads();
    if (total) *total = all;
    return base + x - v;
}

// Spiral turn k (Section 3.1): the frame of the pixels at distance k from
// the image border, walked clockwise from its top-left corner (top row,
// right column, bottom row, left column); a single row or column is walked
// left to right or top to bottom.
struct Turn {
    int top, left, bottom, right, len;
    bool cyclic;
};

__device__ __forceinline__ Turn turn_of(int H, int W, int k) {
    Turn t{k, k, H - 1 - k, W - 1 - k, 0, false};
    if (k < 0 || t.top > t.bottom || t.left > t.right) { t.len = 0; return t; }
    const int h = t.bottom - t.top + 1, w = t.right - t.left + 1;
    if (h == 1) t.len = w;
    else if (w == 1) t.len = h;
    else { t.len = 2 * (h + w) - 4; t.cyclic = true; }
    return t;
}

__device__ __forceinline__ int turn_pixel(const Turn &t, int W, int p) {
    const int h = t.bottom - t.top + 1, w = t.right - t.left + 1;
    if (h == 1) return t.top * W + t.left + p;
    if (w == 1) return (t.top + p) * W + t.left;
    if (p < w) return t.top * W + t.left + p;
    p -= w;
    if (p < h - 1) return (t.top + 1 + p) * W + t.right;
    p -= h - 1;
    if (p < w - 1) return t.bottom * W + t.right - 1 - p;
    p -= w - 1;
    return (t.bottom - 1 - p) * W + t.left;
}

// Source of a spiral step (Sections 3.1 and 3.2): drop the filled points
// from S; when S is empty, take the outermost turn that still has an
// unfilled point and set S to its unfilled points; draw number n_prop picks
// member floor(draw |S| / 2^32) of S in turn order; with repulsion h the
// turn pixels 1 .. h-1 positions away on either side leave S.  -1 when D is
// filled.
__device__ __forceinline__ int spiral_select(const FrState &fs, uint64_t *red) {
    __shared__ int sh_pos;
    FrCtl *ctl = fs.ctl;
    const int N = fs.N, W = fs.W;
    const int turn1 = ctl->sp_turn1;
    const int64_t t = ctl->n_prop;
    Turn tn = turn_of(fs.H, W, turn1 - 1);
    int mine = 0;
    for (int p = threadIdx.x; p < tn.len; p += blockDim.x) {
        int in = fs.sp_in[p];
        if (in && fs.count[turn_pixel(tn, W, p)] >= N) {
            in = 0;
            fs.sp_in[p] = 0;
        }
        mine += in;
    }
    int ns = (int)block_sum_i64(mine, (int64_t *)red);
    if (ns == 0) {
        uint64_t kb = kNoKey;
        for (int x = threadIdx.x; x < N; x += blockDim.x) {
            if (fs.count[x] >= N) continue;
            const int y = x / W, xx = x - y * W;
            const int b = min(min(y, xx), min(fs.H - 1 - y, W - 1 - xx));
            kb = (uint64_t)b < kb ? (uint64_t)b : kb;
        }
        kb = block_min_u64(kb, red);
        if (kb == kNoKey) return -1;
        tn = turn_of(fs.H, W, (int)kb);
        mine = 0;
        for (int p = threadIdx.x; p < tn.len; p += blockDim.x) {
            const int in = fs.count[turn_pixel(tn, W, p)] < N;
            fs.sp_in[p] = in;
            mine += in;
        }
        ns = (int)block_sum_i64(mine, (int64_t *)red);
        if (threadIdx.x == 0) ctl->sp_turn1 = (int)kb + 1;
    }
    const uint32_t r = t < N ? fs.draws[t] : 0u;
    const int j = (int)(((uint64_t)r * (uint64_t)ns) >> 32);
    // member j: each thread counts a contiguous run of positions
    const int C = (tn.len + blockDim.x - 1) / blockDim.x;
    const int p0 = min((int)threadIdx.x * C, tn.len), p1 = min(p0 + C, tn.len);
    int cnt = 0;
    for (int p = p0; p < p1; ++p) cnt += fs.sp_in[p];
    if (threadIdx.x == 0) sh_pos = 0;
    const int before = block_excl_scan(cnt, (int64_t *)red);
    if (j >= before && j < before + cnt) {
        int left = j - before, p = p0;
        for (; p < p1 - 1; ++p)
            if (fs.sp_in[p] && left-- == 0) break;
        sh_pos = p;
    }
    __syncthreads();
    const int pos = sh_pos;
    if (threadIdx.x == 0) {
        const int reach = min(fs.rep_h - 1, tn.len);
        for (int d = 1; d <= reach; ++d)
            for (int side = -1; side <= 1; side += 2) {
                int p = pos + side * d;
                if (tn.cyclic) p = ((p % tn.len) + tn.len) % tn.len;
                else if (p < 0 || p >= tn.len) continue;
                fs.sp_in[p] = 0;
            }
    }
    return turn_pixel(tn, W, pos);
}

// The value v of lane (lane ^ M).  Exchanges inside a 16-lane row use DPP
// (quad permutes for M = 1, 2; the two row shifts for M = 4; a row rotation
// for M = 8), which costs a few cycles; across rows the LDS crossbar
// (ds_bpermute).
template <int M>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v) {
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    } else if constexpr (M == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0xF, false);  // row_shl:4
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
        return (__lane_id() & 4) ? dn : up;
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else {
        return (uint32_t)__shfl_xor((int)v, M);
    }
}

template <int M>
__device__ __forceinline__ uint64_t xor_lane(uint64_t v) {
    return (uint64_t)xor_lane32<M>((uint32_t)v) | ((uint64_t)xor_lane32<M>((uint32_t)(v >> 32)) << 32);
}

// One compare-exchange stage of a bitonic sort of 128 keys held two per lane
// (lane l holds elements 2l and 2l+1), for a stride of 2M >= 2 elements:
// lane l pairs with lane l ^ M.
template <int SIZE, int M>
__device__ __forceinline__ void bitonic_lane_stage(uint64_t &a, uint64_t &b) {
    const int lane = __lane_id();
    const bool up = ((2 * lane) & SIZE) == 0;
    const uint64_t pa = xor_lane<M>(a), pb = xor_lane<M>(b);
    const bool keep_min = ((lane & M) == 0) == up;
    a = keep_min ? (pa < a ? pa : a) : (pa > a ? pa : a);
    b = keep_min ? (pb < b ? pb : b) : (pb > b ? pb : b);
}

template <int SIZE>
__device__ __forceinline__ void bitonic_lane_inner(uint64_t &a, uint64_t &b) {
    const bool up = ((2 * __lane_id()) & SIZE) == 0;
    const bool sw = (a > b) == up;
    const uint64_t lo = sw ? b : a, hi = sw ? a : b;
    a = lo;
    b = hi;
}

// The stages of one bitonic merge of blocks of SIZE elements: strides
// SIZE/2 .. 2 across lanes, then stride 1 inside each lane.
template <int SIZE, int M>
__device__ __forceinline__ void bitonic_merge_lanes(uint64_t &a, uint64_t &b) {
    if constexpr (M >= 1) {
        bitonic_lane_stage<SIZE, M>(a, b);
        bitonic_merge_lanes<SIZE, M / 2>(a, b);
    } else {
        bitonic_lane_inner<SIZE>(a, b);
    }
}

// Ascending bitonic sort of 128 keys held two per lane across one wave
// (lane l holds elements 2l and 2l+1): 28 compare-exchange stages, the
// stride-1 ones inside a lane, the others as lane exchanges (xor_lane).
__device__ __forceinline__ void wave_sort128(uint64_t &a, uint64_t &b) {
    bitonic_merge_lanes<2, 0>(a, b);
    bitonic_merge_lanes<4, 1>(a, b);
    bitonic_merge_lanes<8, 2>(a, b);
    bitonic_merge_lanes<16, 4>(a, b);
    bitonic_merge_lanes<32, 8>(a, b);
    bitonic_merge_lanes<64, 16>(a, b);
    bitonic_merge_lanes<128, 32>(a, b);
}

// The pass of the select with the speculation plan, spread over many
// workgroups (its own launch before the step kernel): each thread takes 4
// points, so each wave holds 4 runs of 64 consecutive points (one ballot per
// run rebuilds the complete-row bitmap); each wave writes its minimum key to
// fs.part[w] and its kSelCand smallest candidate keys (points whose row is
// incomplete and that have no cache slot; each lane keeps its best two) to
// fs.part[nw + w * kSelCand ...], in increasing order.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    v = min(v, xor_lane<32>(v));
    v = min(v, xor_lane<16>(v));
    v = min(v, xor_lane<8>(v));
    v = min(v, xor_lane<4>(v));
    v = min(v, xor_lane<2>(v));
    v = min(v, xor_lane<1>(v));
    return v;
}

template <int RULE>
__device__ void sel_part_block(const FrState &fs) {
    if (fs.ctl->done) return;
    constexpr int U = 4;
    const int32_t *aux = sel_aux<RULE>(fs);
    const int N = fs.N, nb = (int)blockDim.x;
    const int base = (int)blockIdx.x * nb * U + (int)threadIdx.x;
    int c[U], a[U], sl[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint32_t x = (uint32_t)min(base + k * nb, N - 1);
        c[k] = ld_off(fs.count, x);
        a[k] = ld_off(aux, x);
        sl[k] = ld_off(fs.src_slot, x);
    }
    uint64_t best = kNoKey, c1 = kNoKey, c2 = kNoKey;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int x = base + k * nb;
        // the complete-row bitmap, rebuilt from the counts (the link fill adds
        // to the counts without watching them reach N)
        const uint64_t fb = __ballot(x < N && c[k] >= N);
        if (__lane_id() == 0 && x < N) {
            fs.full[x >> 5] = (uint32_t)fb;
            if (x + 32 < N) fs.full[(x >> 5) + 1] = (uint32_t)(fb >> 32);
        }
        if (x >= N) continue;
        const uint64_t key = sel_key<RULE>(fs, x, c[k], a[k]);
        best = key < best ? key : best;
        if (sl[k] < 0 && c[k] < N) {
            if (key < c1) { c2 = c1; c1 = key; }
            else if (key < c2) c2 = key;
        }
    }
    const int nw = (int)gridDim.x * (nb >> 6), w = (int)blockIdx.x * (nb >> 6) + ((int)threadIdx.x >> 6);
    best = wave_min_u64(best);
    if (__lane_id() == 0) fs.part[w] = best;
#pragma unroll 1
    for (int r = 0; r < kSelCand; ++r) {
        const uint64_t m = wave_min_u64(c1);
        if (m != kNoKey && c1 == m) { c1 = c2; c2 = kNoKey; }
        if (__lane_id() == 0) fs.part[nw + w * kSelCand + r] = m;
    }
}

// fr_select, and from the same pass the speculation plan for this step: a
// list of at most kSpecK propagation pieces for the fill launch.  First every
// running propagation continues (those whose source's row became complete
// are dropped).  Then new candidates start: the points with the smallest keys
// other than the selected one, among those whose rows are incomplete and
// that have no slot (each thread keeps its two best; each wave sorts its
// 128, the block merges the four best 32s).  Each new candidate takes a
// victim slot, in eviction order: free slots, then ready slots whose
// source's row is complete, then ready slots by decreasing key of their
// source; running slots and the selected point's slot are never victims.
// Candidate j replaces victim j while its key is the smaller one.  The list
// goes to fs.spec_list (source, or -1 to continue; then the slot), its
// length to *n_plan.
template <int RULE>
__device__ int fr_select_spec(const FrState &fs, uint64_t *red, uint64_t *keys, uint64_t *skeys, int *n_plan,
                              int64_t *ph = nullptr) {
    const bool tr0 = ph && threadIdx.x == 0;
    constexpr uint64_t kTop = (1ull << 46) - 1, kPinned = (1ull << 50) - 1;
    const int32_t *aux = sel_aux<RULE>(fs);
    uint64_t best = kNoKey, c1 = kNoKey, c2 = kNoKey;
    // The slots' state (the first two waves, one slot each) does not depend
    // on the selected point: its loads go out first, beside the partials'.
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    int src = -1, st = kSlotFree, cs = 0, as = 0;
    if (wave < kSpecSlots / 64) {
        src = fs.slot_src[threadIdx.x];
        st = fs.slot_state[threadIdx.x];
        const int sc = src >= 0 ? src : 0;
        cs = fs.count[sc];
        as = aux[sc];
    }
    // the partial pass (sel_part_block) left each wave's minimum and best
    // candidates: the minimum over the minima, and each thread's best two of
    // the candidates it reads
    {
        const int nw = sel_part_waves(fs.N);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) {
            const uint64_t k = fs.part[i];
            best = k < best ? k : best;
        }
        for (int i = threadIdx.x; i < nw * kSelCand; i += blockDim.x) {
            const uint64_t key = fs.part[nw + i];
            if (key < c1) { c2 = c1; c1 = key; }
            else if (key < c2) c2 = key;
        }
    }
    if (tr0) ph[0] = trace_clock();
    best = block_min_u64(best, red);
    if (tr0) ph[1] = trace_clock();
    const int s = key_done<RULE>(fs, best) ? -1 : key_point<RULE>(fs, best);
    if (c1 == best) { c1 = c2; c2 = kNoKey; }
    else if (c2 == best) c2 = kNoKey;
    // slots (kSpecSlots = 128, the first two waves): running ones continue,
    // the others get an eviction key
    __shared__ int n_run;
    if (threadIdx.x == 0) n_run = 0;
    __syncthreads();
    uint64_t e0 = ~0ull, e1 = ~0ull;
    if (wave < kSpecSlots / 64) {
        const int t = threadIdx.x;
        if (src < 0) cs = 0;
        uint64_t keep;
        if (st == kSlotRunning && cs < fs.N) {
            keep = kPinned;
            const int j = atomicAdd(&n_run, 1);
            if (j < kSpecK) {
                fs.spec_list[j] = -1;
                fs.spec_list[kSpecK + j] = t;
            }
        } else if (src < 0 || st == kSlotFree || (st == kSlotRunning && cs >= fs.N)) {
            keep = 0;  // free, or a propagation no longer needed
        } else if (src == s) {
            keep = kPinned;
        } else {
            keep = cs >= fs.N ? 1 : 2 + (kTop - key_heur<RULE>(sel_key<RULE>(fs, src, cs, as)));
        }
        // two slot keys per lane: slot t goes to element t of the wave pair
        skeys[t] = (keep << 8) | (uint64_t)t;
    }
    __syncthreads();
    // candidates: each wave sorts its 128, keeps its best 32
    wave_sort128(c1, c2);
    if (lane < 16) {
        keys[wave * 32 + 2 * lane] = c1;
        keys[wave * 32 + 2 * lane + 1] = c2;
    }
    if (wave == 2) {  // the slot keys, two per lane
        e0 = skeys[2 * lane];
        e1 = skeys[2 * lane + 1];
        wave_sort128(e0, e1);
    }
    __syncthreads();
    if (wave == 2) {
        skeys[2 * lane] = e0;
        skeys[2 * lane + 1] = e1;
    }
    if (wave == 0) {
        uint64_t m0 = keys[2 * lane], m1 = keys[2 * lane + 1];
        wave_sort128(m0, m1);
        if (lane < 16) {
            keys[128 + 2 * lane] = m0;
            keys[128 + 2 * lane + 1] = m1;
        }
    }
    __syncthreads();
    if (tr0) ph[2] = trace_clock();
    const int nr = n_run < kSpecK ? n_run : kSpecK;
    if (threadIdx.x < kSpecK) {
        const int j = threadIdx.x;
        bool take = false;
        // new candidates: at most spec_cap of them (running pieces continue regardless)
        const int cap = fs.spec_cap > 0 ? fs.spec_cap : kSpecK;
        if (j >= nr && j - nr < cap) {
            const uint64_t ck = keys[128 + (j - nr)];
            const uint64_t keep = skeys[j - nr] >> 8;
            take = ck != kNoKey && keep != kPinned && (keep < 2 || key_heur<RULE>(ck) < kTop - (keep - 2));
            if (take) {
                fs.spec_list[j] = key_point<RULE>(fs, ck);
                fs.spec_list[kSpecK + j] = (int)(skeys[j - nr] & 0xFFu);
            }
        }
        keys[256 + j] = (j < nr || take) ? 1 : 0;  // 'take' is monotone in j: a prefix
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int n = 0;
        while (n < kSpecK && keys[256 + n]) ++n;
        *n_plan = n;
    }
    return s;
}

// One step of the filling-rate loop: select s, propagate from s, write the
// tree as packed (d << 4 | parent code) words.  One block.
// One step of the loop for one image, by one block.  batch_done (nullable)
// counts the images of a batch whose loop has ended.
template <int CONN, int S, bool kStageW, bool kSpec = false>
__device__ void fr_step_block(const GImg &g, int Wp, const FrState &fs, int max_rounds, int *smem, uint64_t *red,
                              int *batch_done, uint64_t *keys = nullptr, uint64_t *skeys = nullptr,
                              int64_t *ph = nullptr) {
    FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    if (threadIdx.x == 0 && fs.filled_out && ctl->n_prop > 0) fs.filled_out[ctl->n_prop - 1] = ctl->filled;
    __shared__ int n_cand;
    int s;
    if (fs.rule == kRuleSpiral) {
        s = spiral_select(fs, red);  // random draws: nothing to speculate on
        if (kSpec && threadIdx.x == 0) n_cand = 0;
    } else if (fs.rule == kRuleExtrema)
        s = kSpec ? fr_select_spec<kRuleExtrema>(fs, red, keys, skeys, &n_cand, ph) : fr_select<kRuleExtrema>(fs, red);
    else
        s = kSpec ? fr_select_spec<kRuleFilling>(fs, red, keys, skeys, &n_cand, ph) : fr_select<kRuleFilling>(fs, red);
    if (s < 0) {
        if (threadIdx.x == 0) {
            ctl->done = 1;
            if (batch_done) atomicAdd(batch_done, 1);
        }
        return;
    }
    int slot = kSpec ? fs.src_slot[s] : -1;
    if (slot >= 0 && fs.slot_state[slot] != kSlotReady) slot = -1;  // still propagating: compute it here
    if (threadIdx.x == 0) {
        if (fs.seq_out) fs.seq_out[ctl->n_prop] = s;
        ctl->s = s;
        ctl->n_prop += 1;
        ctl->tree_slot = slot;
        if (kSpec) {
            ctl->spec_n = n_cand;
            if (slot >= 0) ctl->spec_hits += 1;
        }
    }
    if (slot >= 0) return;  // the tree of s is already in the cache
    int *d = smem;
    NbW w = nbw_of(g);
    if (kStageW) {
        // The edge checks and the tree pass read every weight of the
        // neighbourhood: keep them in LDS next to the distance field.
        const int half = (g.N + 1) / 2;  // u16 pairs per array
        uint32_t *lw = (uint32_t *)(smem + g.H * Wp);
        copy_to_lds(lw, (const uint32_t *)g.wr, half);
        copy_to_lds(lw + half, (const uint32_t *)g.wd, half);
        w.wr = (const uint16_t *)lw;
        w.wd = (const uint16_t *)(lw + half);
        if (CONN == 8) {
            copy_to_lds(lw + 2 * half, (const uint32_t *)g.wdr, half);
            copy_to_lds(lw + 3 * half, (const uint32_t *)g.wdl, half);
            w.wdr = (const uint16_t *)(lw + 2 * half);
            w.wdl = (const uint16_t *)(lw + 3 * half);
        }
    }
    fill_inf(d, g.H * Wp);
    __syncthreads();
    if (threadIdx.x == 0) d[(s / g.W) * Wp + s % g.W] = 0;
    __syncthreads();
    bool tree_done = false;
    const int r = relax_block<CONN, S, false, true>(g, d, Wp, max_rounds, &w, fs.packed, &tree_done);
    if (!tree_done) field_check<CONN, false, true>(g, w, d, Wp, fs.packed);
    if (threadIdx.x == 0) {
        if (r < 0) ctl->err = GAPD_ENOCONV;
        ctl->rounds += r < 0 ? max_rounds : r;
    }
}

// Redundancy fill for pixel v along its ancestors (Property 1): every
// ancestor u on the tree path from the source gives d(u,v) = d(s,v) - d(s,u).
// pk holds the tree words with row stride pkW (W for global arrays, Wp for
// LDS).  Pairs already marked are skipped, so every entry of D is written
// once; an ancestor whose row was complete needs no look at the filled-pairs
// matrix.  The walk moves one ancestor per iteration and keeps PF of them in
// flight, so the loads of their filled-pairs words overlap.  Returns the
// number of new pairs.
template <int PF, bool kCntLds>
__device__ __forceinline__ int fill_from(const FrState &fs, const uint32_t *pk, int pkW, int W, int v, int s, int *cnt) {
    const int N = fs.N, MW = fs.MW;
    int uy = v / W, ux = v - uy * W;
    const uint32_t wv = pk[uy * pkW + ux];
    const int dv = tw_dist(wv);
    uint32_t code = tw_code(wv);
    uint32_t *mrow = fs.mask + (size_t)v * MW;
    int32_t *Drow = fs.D + (size_t)v * N;
    auto up = [&](int &u, int &du, uint32_t &bits) {
        if (code == kRootCode) {
            u = -1;
            return;
        }
        uy += code_dy((int)code);
        ux += code_dx((int)code);
        const uint32_t pu = pk[uy * pkW + ux];
        code = tw_code(pu);
        u = uy * W + ux;
        du = tw_dist(pu);
        bits = 0xFFFFFFFFu;
        if (!(pu & kFilledBit)) bits = mrow[u >> 5];
    };
    int ru[PF], rd[PF];
    uint32_t rb[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) up(ru[k], rd[k], rb[k]);
    int nnew = 0;
    bool alive = true;
    while (alive) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int u = ru[k];
            alive = alive && u >= 0;
            if (alive) {
                if (!((rb[k] >> (u & 31)) & 1u)) {
                    const int val = dv - rd[k];
                    Drow[u] = val;
                    fs.D[(size_t)u * N + v] = val;
                    atomicOr(&mrow[u >> 5], 1u << (u & 31));
                    if (u != s) {
                        atomicOr(&fs.mask[(size_t)u * MW + (v >> 5)], 1u << (v & 31));
                        if (kCntLds)
                            atomicAdd(&cnt[u], 1);
                        else
                            count_add(fs, u, 1);
                    }
                    ++nnew;
                }
                up(ru[k], rd[k], rb[k]);
            }
        }
    }
    return nnew;
}

// fill_from with a grandparent table a2 (0xFFFF: none) beside the tree words
// in LDS: one round of LDS reads (the tree words of the parent and of the
// grandparent, and the grandparent's own grandparent) advances the walk by
// two ancestors, so the dependent chain of reads is half as long.
template <int PF, bool kCntLds>
__device__ __forceinline__ int fill_from2(const FrState &fs, const uint32_t *pk, const uint16_t *a2, int W, int v, int s, int *cnt) {
    constexpr int P2 = PF / 2;
    const int N = fs.N, MW = fs.MW;
    const uint32_t wv = pk[v];
    const int dv = tw_dist(wv);
    uint32_t *mrow = fs.mask + (size_t)v * MW;
    int32_t *Drow = fs.D + (size_t)v * N;
    int cur = v;
    uint32_t tcur = wv;
    int gcur = a2[v] == 0xFFFFu ? -1 : (int)a2[v];
    // the next two ancestors a (parent of cur) and b (its parent, -1 past the root)
    auto gen = [&](int &a, int &b, int &da, int &db, uint32_t &ba, uint32_t &bb) {
        if (cur < 0) {
            a = b = -1;
            return;
        }
        const uint32_t code = tw_code(tcur);
        a = code == kRootCode ? -1 : cur + code_off((int)code, W);
        b = a < 0 ? -1 : gcur;
        const int ac = a < 0 ? v : a, bc = b < 0 ? v : b;  // in-range addresses
        const uint32_t ta = pk[ac], tb = pk[bc];
        const uint16_t gb = a2[bc];
        da = tw_dist(ta);
        db = tw_dist(tb);
        ba = 0xFFFFFFFFu;
        bb = 0xFFFFFFFFu;
        if (!(ta & kFilledBit)) ba = mrow[ac >> 5];
        if (!(tb & kFilledBit)) bb = mrow[bc >> 5];
        cur = b;
        tcur = tb;
        gcur = gb == 0xFFFFu ? -1 : (int)gb;
    };
    int nnew = 0;
    auto handle = [&](int u, int du, uint32_t bits) {
        if ((bits >> (u & 31)) & 1u) return;
        const int val = dv - du;
        Drow[u] = val;
        fs.D[(size_t)u * N + v] = val;
        atomicOr(&mrow[u >> 5], 1u << (u & 31));
        if (u != s) {
            atomicOr(&fs.mask[(size_t)u * MW + (v >> 5)], 1u << (v & 31));
            if (kCntLds)
                atomicAdd(&cnt[u], 1);
            else
                count_add(fs, u, 1);
        }
        ++nnew;
    };
    int pa[P2], pb[P2], qa[P2], qb[P2];
    uint32_t ra[P2], rb[P2];
#pragma unroll
    for (int k = 0; k < P2; ++k) gen(pa[k], pb[k], qa[k], qb[k], ra[k], rb[k]);
    bool alive = true;
    while (alive) {
#pragma unroll
        for (int k = 0; k < P2; ++k) {
            if (alive) {
                if (pa[k] < 0) {
                    alive = false;
                } else {
                    handle(pa[k], qa[k], ra[k]);
                    if (pb[k] < 0)
                        alive = false;
                    else
                        handle(pb[k], qb[k], rb[k]);
                }
                if (alive) gen(pa[k], pb[k], qa[k], qb[k], ra[k], rb[k]);
            }
        }
    }
    return nnew;
}

// Fill D along the current tree (many blocks).  The tree words are staged in
// LDS when they fit, and so are the count increments of the ancestors: the
// few ancestors near the source collect thousands of increments per step,
// which would serialise as same-address atomics in L2, so each block sums
// them in LDS and adds its totals once.  The source's own row becomes
// complete: block 0 marks it.
template <bool kLds, bool kLdsCount, bool kA2 = false, int kLanes = 256>
__device__ void fr_fill_block(const FrState &fs, const uint32_t *tree, int W, uint32_t *spk, int64_t *red, int chunk,
                              int nchunks) {
    const FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    const int s = ctl->s, N = fs.N;
    const uint32_t *pk = tree;
    int *cnt = fs.count;
    if (kLds) {
        copy_to_lds(spk, tree, N);
        pk = spk;
    }
    __syncthreads();
    // Flag the points whose rows were complete before this step (not the
    // source, whose row this step completes), from the complete-row bitmap.
    if (kLds) {
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            uint32_t b = fs.full[w];
            while (b) {
                const int i = w * 32 + __ffs(b) - 1;
                b &= b - 1;
                if (i != s) spk[i] |= kFilledBit;
            }
        }
    }
    if (kLdsCount) {
        cnt = (int *)(spk + (kLds ? N : 0));
        for (int i = threadIdx.x; i < N; i += blockDim.x) cnt[i] = 0;
    }
    __syncthreads();
    // grandparents, after the flags (which leave the parent codes alone)
    uint16_t *a2 = (uint16_t *)(spk + N);
    if (kA2) {
        for (int x = threadIdx.x; x < N; x += blockDim.x) {
            const uint32_t c1 = tw_code(spk[x]);
            uint16_t g = 0xFFFFu;
            if (c1 != kRootCode) {
                const int p = x + code_off((int)c1, W);
                const uint32_t c2 = tw_code(spk[p]);
                if (c2 != kRootCode) g = (uint16_t)(p + code_off((int)c2, W));
            }
            a2[x] = g;
        }
        __syncthreads();
    }
    int64_t mine = 0;
    for (int v = chunk * kLanes + threadIdx.x; threadIdx.x < kLanes && v < N; v += nchunks * kLanes) {
        if (v == s || (pk[v] & kFilledBit)) continue;
        const int n = kA2 ? fill_from2<16, kLdsCount>(fs, pk, a2, W, v, s, cnt)
                          : fill_from<16, kLdsCount>(fs, pk, W, W, v, s, cnt);
        if (n) count_add(fs, v, n);
        mine += n;
    }
    if (kLdsCount) {
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += blockDim.x)
            if (cnt[i]) count_add(fs, i, cnt[i]);
    }
    const int64_t tot = block_sum_i64(mine, red);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&fs.ctl->filled, (unsigned long long)tot);
    if (chunk == 0) {
        uint32_t *mrow = fs.mask + (size_t)s * fs.MW;
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            const int lo = w * 32;
            mrow[w] = (N - lo >= 32) ? 0xFFFFFFFFu : ((1u << (N - lo)) - 1u);
        }
        if (threadIdx.x == 0) {
            fs.count[s] = N;
            atomicOr(&fs.full[s >> 5], 1u << (s & 31));
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Link fill: the redundancy fill (Property 1) in two phases per pixel v.
// Each block first turns the step's tree words into two LDS tables: L[x] =
// parent(x) | (d(x) - d(parent(x))) << 16, the parent and the weight of the
// tree edge into x (kNoId at the root), and G[x] = grandparent(x).
//   detect: walk v's ancestors u two at a time (G is the chain: one
//           dependent LDS read per two ancestors; L gives the one between)
//           and test each pair (u, v) in row v of the filled-pairs matrix.
//           The loop issues loads only, so the compiler's wait counts stay
//           exact and PF pairs of ancestors with their matrix words stay in
//           flight; new pairs are flagged by ancestor position in LDS.
//   write:  walk again up to the last new pair (LDS only), keeping
//           d(s,u) = d(s,v) - (edge weights on the way), and for each new pair
//           write D(u,v) = D(v,u) = d(s,v) - d(s,u), set both matrix bits and
//           count it.  Stores and atomics are fire-and-forget.
// Counts: the block sums the increments of the ancestors in LDS (8-bit
// counters for up to 255 walking threads per block, else 16-bit) and adds
// them once; row v adds its own.  The complete-row bitmap is rebuilt from the counts by the next
// select.
// ---------------------------------------------------------------------------------------------
struct WalkOut {
    int nnew;     // new pairs
    int last;     // position (0-based ancestor index) of the last new pair, -1: none
    int walked;   // ancestors visited
    int fail;     // position of the first new pair the block's list had no room for (INT_MAX: none)
};

// The loads-only walk also appends each new pair (ancestor u, walker vi) to
// the block's list in LDS (list, *lcnt, cap entries): LDS atomics leave the
// wait counts of the global loads exact.
// kG: L holds parent | weight << 16 and G the grandparents; otherwise G is the
// parent table alone (the compact tables) and the grandparent is the
// parent's parent, one more dependent LDS read.
template <int PF, bool kG = true>
__device__ __forceinline__ WalkOut walk_detect(const uint32_t *L, const uint16_t *G, const uint32_t *mrow, int v,
                                               uint32_t *flags, uint32_t *list, int *lcnt, int cap, int vi) {
    constexpr int kCap = kFillFlagWords * 32;
    int cur = v;
    // the next two ancestors of cur and their words of row v; addresses are
    // clamped into range so that every load is issued
    auto gen = [&](int &a, int &b, uint32_t &ma, uint32_t &mb) {
        const int cc = cur < 0 ? v : cur;
        int pa, pb;
        if constexpr (kG) {
            pa = (int)(L[cc] & 0xFFFFu);
            pb = (int)G[cc];
        } else {
            pa = (int)G[cc];
            pb = (int)G[pa == (int)kNoId ? cc : pa];
        }
        a = (cur < 0 || pa == (int)kNoId) ? -1 : pa;
        b = (a < 0 || pb == (int)kNoId) ? -1 : pb;
        ma = mrow[(a < 0 ? v : a) >> 5];
        mb = mrow[(b < 0 ? v : b) >> 5];
        cur = b;
    };
    int ra[PF], rb[PF];
    uint32_t wa[PF], wb[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) gen(ra[k], rb[k], wa[k], wb[k]);
    WalkOut o{0, -1, 0, INT_MAX};
    uint32_t acc = 0;
    int pos = 0;
    auto append = [&](int u, int p) {
        const int i = atomicAdd(lcnt, 1);
        if (i < cap)
            list[i] = (uint32_t)u | ((uint32_t)vi << 16);
        else
            o.fail = min(o.fail, p);
    };
    // one pass over the ring: test each slot, then refill it
    auto group = [&]() {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int a = ra[k], b = rb[k];
            // integer flags (1: the ancestor exists / the pair is new)
            const uint32_t ea = 1u - ((uint32_t)a >> 31), eb = 1u - ((uint32_t)b >> 31);
            const uint32_t na = ea & ((~wa[k]) >> (a & 31)), nb = eb & ((~wb[k]) >> (b & 31));
            const uint32_t fa = na & 1u, fb = nb & 1u;
            acc |= (fa << (pos & 31)) | (fb << ((pos + 1) & 31));
            o.nnew += (int)(fa + fb);
            o.last = (fa | fb) ? pos + (int)fb : o.last;
            o.walked += (int)(ea + eb);
            if (fa | fb) {  // rare after the first steps
                if (fa) append(a, pos);
                if (fb) append(b, pos + 1);
            }
            pos += 2;
            if ((pos & 31) == 0) {
                if (pos <= kCap) flags[(pos >> 5) - 1] = acc;
                acc = 0;
            }
            gen(ra[k], rb[k], wa[k], wb[k]);
            // keep the program order: each slot is tested just before it is
            // refilled, so PF slots of loads stay in flight
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // Four passes per loop iteration: the compiler waits for every load at
    // the loop head, so the head comes once per 8 PF ancestors.
    while (ra[0] >= 0) {
        group();
        if (ra[0] < 0) break;
        group();
        if (ra[0] < 0) break;
        group();
        if (ra[0] < 0) break;
        group();
    }
    if ((pos & 31) != 0 && pos < kCap) flags[pos >> 5] = acc;
    return o;
}

// Pair (u, v) is new: D(u,v) = D(v,u) = dv - du, both matrix bits, counts
// (u's in the block's LDS counters, 1 << CS per word, never the source's:
// its row is completed by block 0).
template <int CS, bool kGlobalCnt = false>
__device__ __forceinline__ void write_pair(const FrState &fs, uint32_t *mrow, int32_t *Drow, uint32_t *cnt, int v,
                                           int dv, int u, int du, int s) {
    constexpr int kPer = 1 << CS, kBits = 32 / kPer;
    const int val = dv - du;
    Drow[u] = val;
    fs.D[(size_t)u * fs.N + v] = val;
    atomicOr(&mrow[u >> 5], 1u << (u & 31));
    if (u != s) {
        atomicOr(&fs.mask[(size_t)u * fs.MW + (v >> 5)], 1u << (v & 31));
        if constexpr (kGlobalCnt)
            atomicAdd(&fs.count[u], 1);
        else
            atomicAdd(&cnt[u >> CS], 1u << ((u & (kPer - 1)) * kBits));
    }
}

// Walk again from v to the last new pair and write the new pairs at
// positions from `from` on (those the block's list had no room for).
template <int CS>
__device__ __forceinline__ void walk_write(const FrState &fs, const uint32_t *L, const uint16_t *G, const uint32_t *flags,
                           uint32_t *cnt8, int v, int dv, int last, int s, int from) {
    constexpr int kCap = kFillFlagWords * 32;
    uint32_t *mrow = fs.mask + (size_t)v * fs.MW;
    int32_t *Drow = fs.D + (size_t)v * fs.N;
    int cur = v, dcur = dv;
    for (int p = 0; p <= last; p += 2) {
        const uint32_t l = L[cur];
        const int a = (int)(l & 0xFFFFu), b = (int)G[cur];
        const int da = dcur - (int)(l >> 16);
        bool na, nb;
        if (p < kCap) {
            const uint32_t fw = flags[p >> 5];
            na = (fw >> (p & 31)) & 1u;
            nb = (fw >> ((p + 1) & 31)) & 1u;
        } else {  // beyond the flags: the matrix still holds the answer for these pairs
            na = !((mrow[a >> 5] >> (a & 31)) & 1u);
            nb = b != (int)kNoId && !((mrow[b >> 5] >> (b & 31)) & 1u);
        }
        if (na && p >= from) write_pair<CS>(fs, mrow, Drow, cnt8, v, dv, a, da, s);
        if (b == (int)kNoId) break;
        const int db = da - (int)(L[a] >> 16);
        if (nb && p + 1 >= from) write_pair<CS>(fs, mrow, Drow, cnt8, v, dv, b, db, s);
        cur = b;
        dcur = db;
    }
}

// The compact tables' walk again from v to the last new pair, writing the
// pairs at positions from `from` on; d(s, u) comes from u's tree word.
__device__ __forceinline__ void walk_write_compact(const FrState &fs, const uint16_t *P, const uint32_t *tree,
                                                   const uint32_t *flags, int v, int dv, int last, int s, int from) {
    constexpr int kCap = kFillFlagWords * 32;
    uint32_t *mrow = fs.mask + (size_t)v * fs.MW;
    int32_t *Drow = fs.D + (size_t)v * fs.N;
    int cur = v;
    for (int p = 0; p <= last; ++p) {
        const int u = (int)P[cur];
        if (u == (int)kNoId) break;
        bool nu;
        if (p < kCap)
            nu = (flags[p >> 5] >> (p & 31)) & 1u;
        else
            nu = !((mrow[u >> 5] >> (u & 31)) & 1u);
        if (nu && p >= from) write_pair<0, true>(fs, mrow, Drow, nullptr, v, dv, u, tw_dist(tree[u]), s);
        cur = u;
    }
}

// The parent table of a tree from its words in global memory (kNoId at the
// root), 4 pixels per 16-byte load, U loads in flight per thread.
__device__ __forceinline__ void build_parents(const uint32_t *__restrict__ tree, uint16_t *P, int N, int W) {
    constexpr int U = 8;
    const int nb = (int)blockDim.x;
    const int N4 = N / 4;
    typedef const __attribute__((address_space(1))) u32x4 *gptr4;
    const gptr4 t4p = (gptr4)tree;
    auto par = [&](int x, uint32_t t) -> uint32_t {
        const uint32_t c = tw_code(t);
        return c == kRootCode ? kNoId : (uint32_t)(x + code_off((int)c, W));
    };
    for (int base = threadIdx.x; base < N4; base += nb * U) {
        u32x4 t[U];
#pragma unroll
        for (int k = 0; k < U; ++k) t[k] = t4p[min(base + k * nb, N4 - 1)];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = min(base + k * nb, N4 - 1), x = 4 * i;
            const uint32_t p0 = par(x, t[k].x), p1 = par(x + 1, t[k].y), p2 = par(x + 2, t[k].z), p3 = par(x + 3, t[k].w);
            *reinterpret_cast<uint2 *>(&P[x]) = make_uint2(p0 | (p1 << 16), p2 | (p3 << 16));
        }
    }
    for (int x = 4 * N4 + threadIdx.x; x < N; x += nb) P[x] = (uint16_t)par(x, tree[x]);
}

// The link tables of a tree, straight from its words in global memory:
// L[x] = parent(x) | (d(x) - d(parent(x))) << 16 and G[x] = parent(parent(x))
// (kNoId where there is none).  The parent's word holds both its distance
// and its own parent's direction, so one dependent load per pixel gives both
// tables.  The loads are latency-bound: each thread takes 4 * U pixels at a
// time (U 16-byte loads, then the 4 * U parents' words), which covers a
// 128 x 128 image in two round trips of each kind.
__device__ __forceinline__ void link_words(const uint32_t *__restrict__ tree, int x, uint32_t t, uint32_t tp, int W,
                                           uint32_t &l, uint32_t &gg) {
    const uint32_t c = tw_code(t);
    const int p = x + code_off((int)c, W);
    const uint32_t cp = tw_code(tp);
    l = c == kRootCode ? kNoId : ((uint32_t)p | ((uint32_t)(tw_dist(t) - tw_dist(tp)) << 16));
    gg = (c == kRootCode || cp == kRootCode) ? kNoId : (uint32_t)(p + code_off((int)cp, W));
}

__device__ __forceinline__ void build_links(const uint32_t *__restrict__ tree, uint32_t *L, uint16_t *G, int N, int W) {
    constexpr int U = 8;
    const int nb = (int)blockDim.x;
    const int N4 = N / 4;
    const uint4 *t4p = reinterpret_cast<const uint4 *>(tree);
    auto parent_of = [&](int x, uint32_t t) {
        const uint32_t c = tw_code(t);
        return x + code_off((int)c, W);  // the root's offset is 0
    };
    for (int base = threadIdx.x; base < N4; base += nb * U) {
        uint4 t[U];
        uint32_t tp[U][4];
#pragma unroll
        for (int k = 0; k < U; ++k) t[k] = t4p[min(base + k * nb, N4 - 1)];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int x = 4 * min(base + k * nb, N4 - 1);
            tp[k][0] = tree[parent_of(x, t[k].x)];
            tp[k][1] = tree[parent_of(x + 1, t[k].y)];
            tp[k][2] = tree[parent_of(x + 2, t[k].z)];
            tp[k][3] = tree[parent_of(x + 3, t[k].w)];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * nb;
            if (i >= N4) continue;
            const int x = 4 * i;
            uint4 l;
            uint32_t g0, g1, g2, g3;
            link_words(tree, x, t[k].x, tp[k][0], W, l.x, g0);
            link_words(tree, x + 1, t[k].y, tp[k][1], W, l.y, g1);
            link_words(tree, x + 2, t[k].z, tp[k][2], W, l.z, g2);
            link_words(tree, x + 3, t[k].w, tp[k][3], W, l.w, g3);
            *reinterpret_cast<uint4 *>(&L[x]) = l;
            *reinterpret_cast<uint2 *>(&G[x]) = make_uint2(g0 | (g1 << 16), g2 | (g3 << 16));
        }
    }
    for (int x = 4 * N4 + threadIdx.x; x < N; x += nb) {
        const uint32_t t = tree[x];
        uint32_t l, gg;
        link_words(tree, x, t, tree[parent_of(x, t)], W, l, gg);
        L[x] = l;
        G[x] = (uint16_t)gg;
    }
}

// The link fill of one block: pixels chunk * kLanes .. + kLanes, PF pairs of
// ancestors in flight per walk.  smem: link_fill_lds(N, kLanes) bytes: L (N
// words), G (N uint16), the ancestor counters and the new-pair flags.
// kCompact: the compact tables for images whose full tables do not fit LDS:
// the parent table alone (G), no L, the counts added straight to global
// memory; d(s, u) always comes from the tree words.
template <int kLanes = kFillLanes, int PF = 16, bool kCompact = false>
__device__ __forceinline__ void fill_links_block(const FrState &fs, const uint32_t *tree, int W, uint32_t *smem, int64_t *red,
                                 int chunk) {
    constexpr int CS = fill_cnt_shift(kLanes), kPer = 1 << CS, kBits = 32 / kPer;
    constexpr uint32_t kCntMask = (1u << kBits) - 1u;
    const FrCtl *ctl = fs.ctl;
    const int64_t t0 = fs.trace ? trace_clock() : 0;
    const int s = ctl->s, N = fs.N;
    const int ncw = kCompact ? 0 : (N + kPer - 1) / kPer;  // counter words
    uint32_t *L = smem;
    uint16_t *G = (uint16_t *)(kCompact ? smem : smem + al4w(N));
    uint32_t *C8 = kCompact ? smem + al4w((N + 1) / 2) : smem + al4w(N) + al4w((N + 1) / 2);
    uint32_t *FL = C8 + al4w(ncw);
    int *DV = (int *)(FL + kLanes * kFillFlagWords);  // each walker's d(s, v)
    uint32_t *LIST = (uint32_t *)(DV + kLanes);        // new pairs: u | walker << 16
    const int cap = kCompact ? compact_fill_list_cap(N, kLanes) : link_fill_list_cap(N, kLanes);
    __shared__ int lcnt;
    if (threadIdx.x == 0) lcnt = 0;
    // phase ticks, read by thread 0 when tracing (a traced block also waits
    // for every walker between the detect and write phases)
    int64_t ph[6] = {t0, 0, 0, 0, 0, 0};
    const bool tr0 = fs.trace && threadIdx.x == 0;
    if constexpr (kCompact)
        build_parents(tree, G, N, W);
    else
        build_links(tree, L, G, N, W);
    for (int i = threadIdx.x; i < ncw; i += blockDim.x) C8[i] = 0;
    const int v = chunk * kLanes + (int)threadIdx.x;
    // a complete row has nothing left to fill, whenever it became complete
    const bool walker = (int)threadIdx.x < kLanes && v < N && v != s && fs.count[v] < N;
    const int dv = walker ? tw_dist(tree[v]) : 0;
    if ((int)threadIdx.x < kLanes) DV[threadIdx.x] = dv;
    __syncthreads();
    if (tr0) ph[1] = trace_clock();
    WalkOut o{0, -1, 0, INT_MAX};
    uint32_t *flags = FL + (size_t)threadIdx.x * kFillFlagWords;
    if (walker)
        o = walk_detect<PF, !kCompact>(L, G, fs.mask + (size_t)v * fs.MW, v, flags, LIST, &lcnt, cap, (int)threadIdx.x);
    __syncthreads();
    if (tr0) ph[2] = trace_clock();
    // The listed pairs, spread over all threads of the block: each needs
    // d(s, u) (the tree word of u) and its walker's d(s, v); loads first.
    {
        constexpr int U = 4;
        const int n = min(lcnt, cap), nb = (int)blockDim.x;
        for (int base = threadIdx.x; base < n; base += nb * U) {
            uint32_t e[U], tu[U];
#pragma unroll
            for (int k = 0; k < U; ++k) e[k] = LIST[min(base + k * nb, n - 1)];
#pragma unroll
            for (int k = 0; k < U; ++k) tu[k] = ld_off(tree, e[k] & 0xFFFFu);
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (base + k * nb >= n) continue;
                const int u = (int)(e[k] & 0xFFFFu), wi = (int)(e[k] >> 16), vv = chunk * kLanes + wi;
                write_pair<CS, kCompact>(fs, fs.mask + (size_t)vv * fs.MW, fs.D + (size_t)vv * N, C8, vv, DV[wi], u,
                                         tw_dist(tu[k]), s);
            }
        }
    }
    // pairs the list had no room for: walk again from the first of them
    if (o.fail != INT_MAX) {
        if constexpr (kCompact)
            walk_write_compact(fs, G, tree, flags, v, dv, o.last, s, o.fail);
        else
            walk_write<CS>(fs, L, G, flags, C8, v, dv, o.last, s, o.fail);
    }
    if (o.nnew) atomicAdd(&fs.count[v], o.nnew);
    __syncthreads();
    if (tr0) ph[3] = trace_clock();
    for (int i = threadIdx.x; i < ncw; i += blockDim.x) {
        const uint32_t c = C8[i];
        if (c) {
#pragma unroll
            for (int j = 0; j < kPer; ++j)
                if ((c >> (kBits * j)) & kCntMask) atomicAdd(&fs.count[kPer * i + j], (int)((c >> (kBits * j)) & kCntMask));
        }
    }
    const int64_t tot = block_sum_i64(o.nnew, red);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&fs.ctl->filled, (unsigned long long)tot);
    if (chunk == 0) {
        uint32_t *mrow = fs.mask + (size_t)s * fs.MW;
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            const int lo = w * 32;
            mrow[w] = (N - lo >= 32) ? 0xFFFFFFFFu : ((1u << (N - lo)) - 1u);
        }
        if (threadIdx.x == 0) fs.count[s] = N;
    }
    if (fs.trace) {
        int64_t *tr = fs.trace + (ctl->n_prop - 1) * kTraceFields;
        const int64_t walked = block_sum_i64(o.walked, red);
        const int64_t walkers = block_sum_i64(walker ? 1 : 0, red);
        int mw = o.walked;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mw = max(mw, __shfl_xor(mw, off));
        if (__lane_id() == 0) atomicMax((unsigned long long *)&tr[kTrMaxWalk], (unsigned long long)mw);
        if (threadIdx.x == 0) {
            const int64_t t1 = trace_clock();
            ph[4] = t1;
            for (int i = 0; i < 4; ++i)
                atomicAdd((unsigned long long *)&tr[kTrPhTables + i], (unsigned long long)(ph[i + 1] - ph[i]));
            atomicMax((unsigned long long *)&tr[kTrPhDetectMax], (unsigned long long)(ph[2] - ph[1]));
            atomicMax((unsigned long long *)&tr[kTrPhWriteMax], (unsigned long long)(ph[3] - ph[2]));
            atomicAdd((unsigned long long *)&tr[kTrVisits], (unsigned long long)walked);
            atomicAdd((unsigned long long *)&tr[kTrNew], (unsigned long long)tot);
            atomicAdd((unsigned long long *)&tr[kTrWalkers], (unsigned long long)walkers);
            atomicMax((unsigned long long *)&tr[kTrBlockMax], (unsigned long long)(t1 - t0));
            atomicAdd((unsigned long long *)&tr[kTrBlockSum], (unsigned long long)(t1 - t0));
            atomicMax((unsigned long long *)&tr[kTrStartInv], (unsigned long long)(INT64_MAX - t0));
            atomicMax((unsigned long long *)&tr[kTrEnd], (unsigned long long)t1);
            atomicAdd((unsigned long long *)&tr[kTrFillBlocks], 1ull);
        }
    }
}

// Piece j of the speculation plan, one round of a propagation into its
// cache slot: a new candidate starts in its victim slot (source at 0, the
// rest infinite), a running one resumes from the partial distance field kept
// in its slot.  A round that changes nothing ends the propagation (the field
// is the fixed point): the tree words replace the field and the slot is
// ready.  Otherwise the field goes back to the slot.  Any state of the field
// is a set of real path lengths, so resuming converges to the same
// distances.  One round stays shorter than the fill it runs beside, so the
// speculation never lengthens a step.  One block.  Returns 1 when the piece
// reached the fixed point, -1 when the field goes back to the slot, -3 when
// the plan has no piece j.
template <int CONN, int S, bool kStageW>
__device__ __forceinline__ int fr_spec_block(const GImg &g, int Wp, const FrState &fs, int *smem, int j) {
    const int64_t tstart = fs.trace && threadIdx.x == 0 ? trace_clock() : 0;
    FrCtl *ctl = fs.ctl;
    if (j >= ctl->spec_n) return -3;
    const int c = fs.spec_list[j], sl = fs.spec_list[kSpecK + j];
    uint32_t *tree = slot_tree(fs, sl);
    int *d = smem;
    NbW w = nbw_of(g);
    if (kStageW) {
        const int half = (g.N + 1) / 2;
        uint32_t *lw = (uint32_t *)(smem + g.H * Wp);
        copy_to_lds(lw, (const uint32_t *)g.wr, half);
        copy_to_lds(lw + half, (const uint32_t *)g.wd, half);
        w.wr = (const uint16_t *)lw;
        w.wd = (const uint16_t *)(lw + half);
        if (CONN == 8) {
            copy_to_lds(lw + 2 * half, (const uint32_t *)g.wdr, half);
            copy_to_lds(lw + 3 * half, (const uint32_t *)g.wdl, half);
            w.wdr = (const uint16_t *)(lw + 2 * half);
            w.wdl = (const uint16_t *)(lw + 3 * half);
        }
    }
    if (c >= 0) {
        if (threadIdx.x == 0) {
            const int old = fs.slot_src[sl];
            if (old >= 0) fs.src_slot[old] = -1;
            fs.slot_src[sl] = c;
            fs.src_slot[c] = sl;
            fs.slot_state[sl] = kSlotRunning;
        }
        fill_inf(d, g.H * Wp);
        __syncthreads();
        if (threadIdx.x == 0) d[(c / g.W) * Wp + c % g.W] = 0;
    } else {
        field_to_lds(d, Wp, tree, g.N, g.W);
    }
    __syncthreads();
    const int64_t tp0 = fs.trace && threadIdx.x == 0 ? trace_clock() : 0;
    bool tree_done = false;
    // One sweep round.  A new propagation never converges in its first round;
    // a resumed field is checked right after it, which saves the round that
    // would otherwise only confirm the fixed point.
    const int r = relax_block<CONN, S, false, true>(g, d, Wp, 1, &w, tree, &tree_done, c < 0);
    const int64_t tp1 = fs.trace && threadIdx.x == 0 ? trace_clock() : 0;
    if (r >= 0) {
        if (!tree_done) field_check<CONN, false, true>(g, w, d, Wp, tree);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            fs.slot_state[sl] = kSlotReady;
            atomicAdd((unsigned long long *)&ctl->spec_props, 1ull);
        }
    } else {
        field_from_lds(tree, d, Wp, g.N, g.W);
    }
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&ctl->rounds, 1ull);
        atomicAdd((unsigned long long *)&ctl->spec_rounds, 1ull);
        if (fs.trace) {
            int64_t *tr = fs.trace + (ctl->n_prop - 1) * kTraceFields;
            atomicAdd((unsigned long long *)&tr[kTrSpecStage], (unsigned long long)(tp0 - tstart));
            atomicAdd((unsigned long long *)&tr[kTrSpecRound], (unsigned long long)(tp1 - tp0));
            atomicAdd((unsigned long long *)&tr[kTrSpecStore], (unsigned long long)(trace_clock() - tp1));
        }
    }
    return r;
}

// ---------------------------------------------------------------------------------------------
// Batched: naive over every (image, source) item, one block per item.
// ---------------------------------------------------------------------------------------------
__device__ int find_image(const BImg *imgs, int B, int64_t item) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------------------------
// Template dispatch on connectivity and elements per lane.
// ---------------------------------------------------------------------------------------------
// Size class: the smallest of 32, 64, 128, 192, 256, 512 that is >= the longer side.
inline int size_class(int max_line) {
    if (max_line <= 32) return 32;
    if (max_line <= 64) return 64;
    if (max_line <= 128) return 128;
    if (max_line <= 192) return 192;
    if (max_line <= 256) return 256;
    return 512;
}

template <template <int, int> class F, typename... A>
hipError_t dispatch(int conn, int max_line, A... args) {
    const int c = size_class(max_line);
    if (conn == 4) {
        switch (c) {
            case 32: return F<4, 32>::run(args...);
            case 64: return F<4, 64>::run(args...);
            case 128: return F<4, 128>::run(args...);
            case 192: return F<4, 192>::run(args...);
            case 256: return F<4, 256>::run(args...);
            default: return F<4, 512>::run(args...);
        }
    }
    switch (c) {
        case 32: return F<8, 32>::run(args...);
        case 64: return F<8, 64>::run(args...);
        case 128: return F<8, 128>::run(args...);
        case 192: return F<8, 192>::run(args...);
        case 256: return F<8, 256>::run(args...);
        default: return F<8, 512>::run(args...);
    }
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

}  // namespace gapd
