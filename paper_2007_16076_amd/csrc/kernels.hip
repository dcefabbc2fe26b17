// HIP kernels of libgapd.so for gfx950 (CDNA4, wave64).
//
// The hot path of the filling-rate method (Noyel, Angulo, Jeulin, "Fast
// computation of all pairs of geodesic distances", Section 3.4, algorithm
// "filling") and of the naive method (Section 1):
//   * k_prep / k_prefix   edge weights of the pseudo-metric (Section 2, eq.
//                         distance_somme; 1 + L1 for multiband images) and
//                         running sums along rows and columns;
//   * relax_block         one geodesic propagation (Section 2, eqs. temps and
//                         distance: minimum over paths of summed weights),
//                         computed as the fixed point of min-plus relaxation
//                         with the distance field resident in LDS;
//   * parent_code         the geodesic tree (Section 2): each pixel's parent
//                         is the smallest-index tight neighbour;
//   * k_fr_step           least-filled source selection (Section 3.4) +
//                         propagation + tree, for one step;
//   * k_fr_fill           redundancy fill along the tree (Property 1):
//                         d(u,v) = d(s,v) - d(s,u) for every ancestor u of v;
//   * k_fr_setup / k_rank geodesic centroid and extrema ranks (Section 3.3).
//
// No MFMA: the work is integer min-plus, not a dense contraction.
#include "gapd_internal.h"
#include "gapd.h"

namespace gapd {

namespace {

constexpr int kBig = 0x7FFFFFFF;

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

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

__global__ void k_prep(GImgW w, const uint8_t *img, int C, int wmode) {
    prep_pixels(w, img, C, wmode, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
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

template <int CTRL>
__device__ __forceinline__ int dpp_mov(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}

// Exclusive prefix minimum: lane l receives min over lanes < l (kBig for lane 0).
__device__ __forceinline__ int wave_excl_prefix_min(int x, int row) {
    x = min(x, dpp_mov<0x111>(kBig, x));  // row_shr:1
    x = min(x, dpp_mov<0x112>(kBig, x));  // row_shr:2
    x = min(x, dpp_mov<0x114>(kBig, x));  // row_shr:4
    x = min(x, dpp_mov<0x118>(kBig, x));  // row_shr:8
    const int t0 = __builtin_amdgcn_readlane(x, 15);
    const int t1 = __builtin_amdgcn_readlane(x, 31);
    const int t2 = __builtin_amdgcn_readlane(x, 47);
    const int c1 = t0, c2 = min(t0, t1), c3 = min(c2, t2);
    const int carry = row == 0 ? kBig : (row == 1 ? c1 : (row == 2 ? c2 : c3));
    x = min(x, carry);
    return dpp_mov<0x111>(carry, x);  // first lane of each row takes the carry
}

// Exclusive suffix minimum: lane l receives min over lanes > l (kBig for lane 63).
__device__ __forceinline__ int wave_excl_suffix_min(int x, int row) {
    x = min(x, dpp_mov<0x101>(kBig, x));  // row_shl:1
    x = min(x, dpp_mov<0x102>(kBig, x));  // row_shl:2
    x = min(x, dpp_mov<0x104>(kBig, x));  // row_shl:4
    x = min(x, dpp_mov<0x108>(kBig, x));  // row_shl:8
    const int t1 = __builtin_amdgcn_readlane(x, 16);
    const int t2 = __builtin_amdgcn_readlane(x, 32);
    const int t3 = __builtin_amdgcn_readlane(x, 48);
    const int c2 = t3, c1 = min(t2, t3), c0 = min(t1, c1);
    const int carry = row == 3 ? kBig : (row == 2 ? c2 : (row == 1 ? c1 : c0));
    x = min(x, carry);
    return dpp_mov<0x101>(carry, x);  // last lane of each row takes the carry
}

// ---------------------------------------------------------------------------------------------
// One directional sweep over all lines of a view (rows of the image, or rows
// of its transpose = columns).  Line l is relaxed from the previous line of
// the sweep (cross edges), then exactly along itself: with R[e] the running
// weight sum along the line, min_{e'}(a[e'] + |R[e]-R[e']|) is a prefix
// minimum of a - R plus R and a suffix minimum of a + R minus R.  A lane owns
// C consecutive elements.  Writes go through an atomic min, so the four
// sweeps of a round may run concurrently on the same distance field: every
// stored value is the length of a real path, and values only decrease.
// Returns true if this wave lowered any value.
// ---------------------------------------------------------------------------------------------
template <int CONN, int C, bool FWD, bool G>
__device__ bool sweep(int *d, int ls, int es, int NL, int L, const uint16_t *__restrict__ wv,
                      const uint16_t *__restrict__ wdr, const uint16_t *__restrict__ wdl,
                      const int32_t *__restrict__ P) {
    const int lane = __lane_id();
    const int row = lane >> 4;
    const int e0 = lane * C;
    bool changed = false;
    int prev[C];
#pragma unroll
    for (int j = 0; j < C; ++j) prev[j] = kInf;

    // Registers holding the next line's inputs (prefetched one line ahead).
    int ncur[C], nP[C], nwc[C], nwm[C], nwp[C];
    auto load = [&](int step) {
        const int l = FWD ? step : NL - 1 - step;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int e = e0 + j;
            const bool ok = e < L;
            ncur[j] = ok ? ldd<G>(&d[l * ls + e * es]) : kInf;
            nP[j] = P[l * L + (ok ? e : L - 1)];
            nwc[j] = kInf;
            nwm[j] = kInf;
            nwp[j] = kInf;
            if (step > 0 && ok) {
                const int top = FWD ? l - 1 : l;
                nwc[j] = wv[top * L + e];
                if (CONN == 8) {
                    if (FWD) {
                        if (e > 0) nwm[j] = wdr[(l - 1) * L + e - 1];
                        if (e + 1 < L) nwp[j] = wdl[(l - 1) * L + e + 1];
                    } else {
                        if (e > 0) nwm[j] = wdl[l * L + e];
                        if (e + 1 < L) nwp[j] = wdr[l * L + e];
                    }
                }
            }
        }
    };
    load(0);
    for (int step = 0; step < NL; ++step) {
        const int l = FWD ? step : NL - 1 - step;
        int cur[C], Pl[C], a[C];
        int wc[C], wm[C], wp[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            cur[j] = ncur[j]; Pl[j] = nP[j]; wc[j] = nwc[j]; wm[j] = nwm[j]; wp[j] = nwp[j];
        }
        if (step + 1 < NL) load(step + 1);

        // Cross edges from the previous line (unused weights are kInf).
#pragma unroll
        for (int j = 0; j < C; ++j) a[j] = min(cur[j], prev[j] + wc[j]);
        if (CONN == 8) {
            int left_in = __shfl_up(prev[C - 1], 1);
            int right_in = __shfl_down(prev[0], 1);
            if (lane == 0) left_in = kInf;
            if (lane == 63) right_in = kInf;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int pm = j > 0 ? prev[j - 1] : left_in;
                const int pp = j < C - 1 ? prev[j + 1] : right_in;
                a[j] = min(a[j], min(pm + wm[j], pp + wp[j]));
            }
        }
        // Along the line, increasing e.
        int t[C];
#pragma unroll
        for (int j = 0; j < C; ++j) t[j] = a[j] - Pl[j];
#pragma unroll
        for (int j = 1; j < C; ++j) t[j] = min(t[j], t[j - 1]);
        int ex = wave_excl_prefix_min(t[C - 1], row);
#pragma unroll
        for (int j = 0; j < C; ++j) {
            a[j] = min(t[j], ex) + Pl[j];
            if (e0 + j >= L) a[j] = kInf;
        }
        // Along the line, decreasing e.
#pragma unroll
        for (int j = 0; j < C; ++j) t[j] = a[j] + Pl[j];
#pragma unroll
        for (int j = C - 2; j >= 0; --j) t[j] = min(t[j], t[j + 1]);
        ex = wave_excl_suffix_min(t[0], row);
#pragma unroll
        for (int j = 0; j < C; ++j) a[j] = min(t[j], ex) - Pl[j];
        // Store improvements.
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int e = e0 + j;
            if (e < L && a[j] < cur[j]) {
                const int old = atomicMin(&d[l * ls + e * es], a[j]);
                if (a[j] < old) changed = true;
                a[j] = min(a[j], old);
            }
            prev[j] = a[j];
        }
    }
    return changed;
}

// Neighbour k of pixel (y, x), in ascending pixel-index order:
// 0:(-1,-1) 1:(-1,0) 2:(-1,+1) 3:(0,-1) 4:(0,+1) 5:(+1,-1) 6:(+1,0) 7:(+1,+1).
// The 4-neighbourhood uses codes 1, 3, 4, 6.
__device__ __forceinline__ int code_dy(int k) { return k < 3 ? -1 : (k < 5 ? 0 : 1); }
__device__ __forceinline__ int code_dx(int k) { return k < 3 ? k - 1 : (k == 3 ? -1 : (k == 4 ? 1 : k - 6)); }

// Weight of the edge between (y, x) and its neighbour in direction k.
__device__ __forceinline__ int nb_weight(const GImg &g, int y, int x, int k) {
    const int W = g.W;
    switch (k) {
        case 0: return g.wdr[(y - 1) * W + x - 1];
        case 1: return g.wd[(y - 1) * W + x];
        case 2: return g.wdl[(y - 1) * W + x + 1];
        case 3: return g.wr[y * W + x - 1];
        case 4: return g.wr[y * W + x];
        case 5: return g.wdl[y * W + x];
        case 6: return g.wd[y * W + x];
        default: return g.wdr[y * W + x];
    }
}

template <int CONN>
__device__ __forceinline__ bool code_used(int k) {
    return CONN == 8 || k == 1 || k == 3 || k == 4 || k == 6;
}

// True if some edge into (y, x) still relaxes its distance.
template <int CONN, bool G>
__device__ bool pixel_violates(const GImg &g, const int *d, int Wp, int y, int x) {
    const int dv = ldd<G>(&d[y * Wp + x]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!code_used<CONN>(k)) continue;
        const int ny = y + code_dy(k), nx = x + code_dx(k);
        if (ny < 0 || ny >= g.H || nx < 0 || nx >= g.W) continue;
        if (ldd<G>(&d[ny * Wp + nx]) + nb_weight(g, y, x, k) < dv) return true;
    }
    return false;
}

// Geodesic-tree parent of (y, x): the first neighbour, in ascending index
// order, with d(q) + w(q, v) == d(v); kRootCode for a pixel at distance 0.
template <int CONN>
__device__ uint32_t parent_code(const GImg &g, const int *d, int Wp, int y, int x, int dv) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!code_used<CONN>(k)) continue;
        const int ny = y + code_dy(k), nx = x + code_dx(k);
        if (ny < 0 || ny >= g.H || nx < 0 || nx >= g.W) continue;
        if (d[ny * Wp + nx] + nb_weight(g, y, x, k) == dv) return (uint32_t)k;
    }
    return kRootCode;
}

// ---------------------------------------------------------------------------------------------
// One geodesic propagation by the whole workgroup (256 threads) on the
// distance field d (H rows of stride Wp; LDS or global).  d must already hold
// kInf everywhere except the seeds (0).  Each round runs the four directional
// sweeps concurrently, one wave each; after a round that changed something,
// a parallel check of every edge decides whether the fixed point is reached.
// Returns the number of rounds, or -1 if max_rounds was hit.
// ---------------------------------------------------------------------------------------------
template <int CONN, int C, bool G = false>
__device__ int relax_block(const GImg &g, int *d, int Wp, int max_rounds) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    int rounds = 0;
    for (;;) {
        bool ch = false;
        if (wave == 0)
            ch = sweep<CONN, C, true, G>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P);
        else if (wave == 1)
            ch = sweep<CONN, C, false, G>(d, Wp, 1, g.H, g.W, g.wd, g.wdr, g.wdl, g.P);
        else if (wave == 2)
            ch = sweep<CONN, C, true, G>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP);
        else if (wave == 3)
            ch = sweep<CONN, C, false, G>(d, 1, Wp, g.W, g.H, g.cwv, g.cwdr, g.cwdl, g.cP);
        ++rounds;
        if (!__syncthreads_or(ch)) break;
        if (rounds >= max_rounds) return -1;
        bool bad = false;
        for (int v = tid; v < g.N && !bad; v += blockDim.x) {
            const int y = v / g.W, x = v - y * g.W;
            bad = pixel_violates<CONN, G>(g, d, Wp, y, x);
        }
        if (!__syncthreads_or(bad)) break;
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
// Naive method / multi-source propagations: block b propagates from
// src_list[b] (or src_base + b) and writes row b of out (Section 1).
// With kGlobal the distance field lives in the output row itself (images too
// large for LDS); otherwise in LDS, and the row is written once at the end.
// ---------------------------------------------------------------------------------------------
template <int CONN, int C, bool kGlobal>
__global__ __launch_bounds__(kRelaxThreads) void k_relax_rows(GImg g, int Wp, const int32_t *src_list,
                                                              int src_base, int32_t *out, int max_rounds,
                                                              FrCtl *ctl) {
    extern __shared__ int smem[];
    const int s = src_list ? src_list[blockIdx.x] : src_base + (int)blockIdx.x;
    int32_t *row = out + (size_t)blockIdx.x * g.N;
    int *d = kGlobal ? row : smem;
    const int Wd = kGlobal ? g.W : Wp;
    fill_inf(d, g.H * Wd);
    __syncthreads();
    if (threadIdx.x == 0) d[(s / g.W) * Wd + s % g.W] = 0;
    __syncthreads();
    const int r = relax_block<CONN, C, kGlobal>(g, d, Wd, max_rounds);
    if (threadIdx.x == 0) {
        if (r < 0) atomicExch(&ctl->err, GAPD_ENOCONV);
        atomicAdd((unsigned long long *)&ctl->rounds, (unsigned long long)(r < 0 ? max_rounds : r));
    }
    if (!kGlobal) {
        for (int v = threadIdx.x; v < g.N; v += blockDim.x) {
            const int y = v / g.W, x = v - y * g.W;
            row[v] = d[y * Wp + x];
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Filling-rate method, one image.
// ---------------------------------------------------------------------------------------------

// D_mrk(i,i) = 1, count = 1, D(i,i) = 0 (Section 2; the filled-pairs matrix
// must already be zero).
__global__ void k_fr_init(FrState fs) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < fs.N; i += gridDim.x * blockDim.x) {
        fs.mask[(size_t)i * fs.MW + (i >> 5)] = 1u << (i & 31);
        fs.count[i] = 1;
        fs.D[(size_t)i * fs.N + i] = 0;
    }
}

// Geodesic centroid and the propagation from it (Section 3.3): propagate from
// every border pixel, take the first pixel of maximal distance as the
// centroid c, propagate from c into fs.dbuf.  One block.
template <int CONN, int C>
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
    int r1 = relax_block<CONN, C>(g, d, Wp, max_rounds);
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
    int r2 = relax_block<CONN, C>(g, d, Wp, max_rounds);
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

template <int CONN, int C>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_setup(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    fr_setup_block<CONN, C>(g, Wp, fs, smem, max_rounds, red);
}

// rank[x] = position of x in the list sorted by decreasing d_c, ties by
// increasing index (Section 3.3); order = inverse permutation.  Brute-force
// counting over all pairs (N^2 comparisons, once per run).
__global__ void k_rank(const int32_t *dc, int N, int32_t *rank, int32_t *order) {
    __shared__ int32_t tile[256];
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

// Least filled point (Section 3.4): argmin over x of (count[x], rank[x]).
// Returns the pixel, or -1 when that point is filled (D is complete).
__device__ int fr_select(const FrState &fs, uint64_t *red) {
    uint64_t best = ~0ull;
    for (int x = threadIdx.x; x < fs.N; x += blockDim.x) {
        const uint64_t key = ((uint64_t)(uint32_t)fs.count[x] << 32) | (uint32_t)fs.rank[x];
        best = key < best ? key : best;
    }
    best = block_min_u64(best, red);
    if ((int)(best >> 32) >= fs.N) return -1;
    return fs.order[(int)(best & 0xFFFFFFFFu)];
}

// One step of the filling-rate loop: select s, propagate from s, write the
// tree as packed (d << 4 | parent code) words.  One block.
template <int CONN, int C>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_step(GImg g, int Wp, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    if (threadIdx.x == 0 && fs.filled_out && ctl->n_prop > 0) fs.filled_out[ctl->n_prop - 1] = ctl->filled;
    const int s = fr_select(fs, red);
    if (s < 0) {
        if (threadIdx.x == 0) ctl->done = 1;
        return;
    }
    if (threadIdx.x == 0) {
        if (fs.seq_out) fs.seq_out[ctl->n_prop] = s;
        ctl->s = s;
        ctl->n_prop += 1;
    }
    int *d = smem;
    fill_inf(d, g.H * Wp);
    __syncthreads();
    if (threadIdx.x == 0) d[(s / g.W) * Wp + s % g.W] = 0;
    __syncthreads();
    const int r = relax_block<CONN, C>(g, d, Wp, max_rounds);
    for (int v = threadIdx.x; v < g.N; v += blockDim.x) {
        const int y = v / g.W, x = v - y * g.W;
        const int dv = d[y * Wp + x];
        fs.packed[v] = ((uint32_t)dv << 4) | parent_code<CONN>(g, d, Wp, y, x, dv);
    }
    if (threadIdx.x == 0) {
        if (r < 0) ctl->err = GAPD_ENOCONV;
        ctl->rounds += r < 0 ? max_rounds : r;
    }
}

// Redundancy fill for pixel v along its ancestors (Property 1).  pk holds the
// packed tree with row stride pkW (W for global arrays, Wp for LDS).  Pairs
// already marked are skipped, so every entry of D is written once.  Ancestors
// are gathered KB at a time so their mask-word loads are in flight together.
// Returns the number of new pairs.
template <int KB>
__device__ int fill_from(const FrState &fs, const uint32_t *pk, int pkW, int W, int v, int s) {
    const int N = fs.N, MW = fs.MW;
    const int vy = v / W, vx = v - vy * W;
    int uy = vy, ux = vx;
    const uint32_t pv = pk[vy * pkW + vx];
    const int dv = (int)(pv >> 4);
    uint32_t code = pv & 15u;
    uint32_t *mrow = fs.mask + (size_t)v * MW;
    int32_t *Drow = fs.D + (size_t)v * N;
    int nnew = 0;
    bool end = (code == kRootCode);
    while (!end) {
        int ub[KB], du[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            ub[i] = -1;
            du[i] = 0;
            if (!end) {
                const int k = (int)code;
                uy += code_dy(k);
                ux += code_dx(k);
                const uint32_t pu = pk[uy * pkW + ux];
                ub[i] = uy * W + ux;
                du[i] = (int)(pu >> 4);
                code = pu & 15u;
                end = (code == kRootCode);
            }
        }
        uint32_t wbits[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) wbits[i] = ub[i] >= 0 ? mrow[ub[i] >> 5] : 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const int u = ub[i];
            if (u < 0 || ((wbits[i] >> (u & 31)) & 1u)) continue;
            const int val = dv - du[i];
            Drow[u] = val;
            fs.D[(size_t)u * N + v] = val;
            atomicOr(&mrow[u >> 5], 1u << (u & 31));
            if (u != s) {
                atomicOr(&fs.mask[(size_t)u * MW + (v >> 5)], 1u << (v & 31));
                atomicAdd(&fs.count[u], 1);
            }
            ++nnew;
        }
    }
    return nnew;
}

// Fill D along the current tree (many blocks).  The packed tree is staged in
// LDS when it fits.  The source's own row becomes complete: block 0 marks it.
template <bool kLds>
__global__ __launch_bounds__(256) void k_fr_fill(FrState fs, int W) {
    extern __shared__ uint32_t spk[];
    __shared__ int64_t red[4];
    const FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    const int s = ctl->s, N = fs.N;
    const uint32_t *pk = fs.packed;
    if (kLds) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) spk[i] = fs.packed[i];
        __syncthreads();
        pk = spk;
    }
    int64_t mine = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        if (v == s || fs.count[v] >= N) continue;
        const int n = fill_from<8>(fs, pk, W, W, v, s);
        if (n) atomicAdd(&fs.count[v], n);
        mine += n;
    }
    const int64_t tot = block_sum_i64(mine, red);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)&fs.ctl->filled, (unsigned long long)tot);
    if (blockIdx.x == 0) {
        uint32_t *mrow = fs.mask + (size_t)s * fs.MW;
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            const int lo = w * 32;
            mrow[w] = (N - lo >= 32) ? 0xFFFFFFFFu : ((1u << (N - lo)) - 1u);
        }
        if (threadIdx.x == 0) fs.count[s] = N;
    }
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

template <int CONN, int C>
__global__ __launch_bounds__(kRelaxThreads) void k_relax_rows_batched(const BImg *imgs, int B, int32_t *out,
                                                                      int max_rounds, FrCtl *ctl) {
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
    const int r = relax_block<CONN, C>(g, d, Wp, max_rounds);
    if (threadIdx.x == 0) {
        if (r < 0) atomicExch(&ctl->err, GAPD_ENOCONV);
        atomicAdd((unsigned long long *)&ctl->rounds, (unsigned long long)(r < 0 ? max_rounds : r));
    }
    int32_t *row = out + bi.out_off + (size_t)s * g.N;
    for (int v = threadIdx.x; v < g.N; v += blockDim.x) {
        const int y = v / g.W, x = v - y * g.W;
        row[v] = d[y * Wp + x];
    }
}

// Batched filling rate: block b owns image b's whole loop (setup, then
// select / propagate / tree / fill until D is complete).  The tree is packed
// in LDS in place of the distances, so the fill walks ancestors in LDS.
template <int CONN, int C>
__global__ __launch_bounds__(kRelaxThreads) void k_fr_batched(const BImg *imgs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    __shared__ int64_t red2[kRelaxThreads / 64];
    const BImg &bi = imgs[blockIdx.x];
    const GImg g = bi.g;
    const FrState fs = bi.fr;
    const int Wp = bi.Wp, H = g.H, W = g.W, N = g.N;
    int *d = smem;
    uint8_t *codes = (uint8_t *)(smem + H * Wp);
    // D_mrk = I, count = 1, D(i,i) = 0
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        fs.mask[(size_t)i * fs.MW + (i >> 5)] = 1u << (i & 31);
        fs.count[i] = 1;
        fs.D[(size_t)i * N + i] = 0;
    }
    fr_setup_block<CONN, C>(g, Wp, fs, d, max_rounds, red);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // ranks by counting (fs.dbuf holds d_c)
    for (int x = threadIdx.x; x < N; x += blockDim.x) {
        const int dx = fs.dbuf[x];
        int cnt = 0;
        for (int y = 0; y < N; ++y) {
            const int dy = fs.dbuf[y];
            cnt += (dy > dx) || (dy == dx && y < x);
        }
        fs.rank[x] = cnt;
        fs.order[cnt] = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    int64_t nprop = 0, filled = 0, rounds = 0;
    for (;;) {
        const int s = fr_select(fs, red);
        if (s < 0) break;
        ++nprop;
        fill_inf(d, H * Wp);
        __syncthreads();
        if (threadIdx.x == 0) d[(s / W) * Wp + s % W] = 0;
        __syncthreads();
        const int r = relax_block<CONN, C>(g, d, Wp, max_rounds);
        rounds += r < 0 ? max_rounds : r;
        if (r < 0) {
            if (threadIdx.x == 0) fs.ctl->err = GAPD_ENOCONV;
            break;
        }
        for (int v = threadIdx.x; v < N; v += blockDim.x) {
            const int y = v / W, x = v - y * W;
            codes[v] = (uint8_t)parent_code<CONN>(g, d, Wp, y, x, d[y * Wp + x]);
        }
        __syncthreads();
        for (int v = threadIdx.x; v < N; v += blockDim.x) {
            const int y = v / W, x = v - y * W;
            d[y * Wp + x] = (int)(((uint32_t)d[y * Wp + x] << 4) | codes[v]);
        }
        __syncthreads();
        int64_t mine = 0;
        for (int v = threadIdx.x; v < N; v += blockDim.x) {
            if (v == s || fs.count[v] >= N) continue;
            const int n = fill_from<8>(fs, (const uint32_t *)d, Wp, W, v, s);
            if (n) atomicAdd(&fs.count[v], n);
            mine += n;
        }
        filled += block_sum_i64(mine, red2);
        if (threadIdx.x == 0) fs.count[s] = N;
        uint32_t *mrow = fs.mask + (size_t)s * fs.MW;
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            const int lo = w * 32;
            mrow[w] = (N - lo >= 32) ? 0xFFFFFFFFu : ((1u << (N - lo)) - 1u);
        }
        // Counts and marks were updated by other waves through L2 atomics:
        // release ours, wait for all, and drop stale L1 lines before the next select.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (threadIdx.x == 0) {
        fs.ctl->n_prop = nprop;
        fs.ctl->filled = filled;
        fs.ctl->rounds += rounds;
        fs.ctl->done = 1;
    }
}

// ---------------------------------------------------------------------------------------------
// Template dispatch on connectivity and elements per lane.
// ---------------------------------------------------------------------------------------------
inline int lane_chunk(int max_line) {
    if (max_line <= 64) return 1;
    if (max_line <= 128) return 2;
    if (max_line <= 256) return 4;
    return 8;
}

template <template <int, int> class F, typename... A>
hipError_t dispatch(int conn, int max_line, A... args) {
    const int c = lane_chunk(max_line);
    if (conn == 4) {
        switch (c) {
            case 1: return F<4, 1>::run(args...);
            case 2: return F<4, 2>::run(args...);
            case 4: return F<4, 4>::run(args...);
            default: return F<4, 8>::run(args...);
        }
    }
    switch (c) {
        case 1: return F<8, 1>::run(args...);
        case 2: return F<8, 2>::run(args...);
        case 4: return F<8, 4>::run(args...);
        default: return F<8, 8>::run(args...);
    }
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int CONN, int C>
struct RelaxRows {
    static hipError_t run(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                          int max_rounds, FrCtl *ctl, hipStream_t st) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        if (lds <= kMaxLds) {
            auto k = k_relax_rows<CONN, C, false>;
            hipError_t e = set_lds(k, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k, dim3(K), dim3(kRelaxThreads), lds, st, g, Wp, src_list, src_base, out,
                               max_rounds, ctl);
        } else {
            hipLaunchKernelGGL((k_relax_rows<CONN, C, true>), dim3(K), dim3(kRelaxThreads), 0, st, g, g.W,
                               src_list, src_base, out, max_rounds, ctl);
        }
        return hipGetLastError();
    }
};

template <int CONN, int C>
struct FrSetup {
    static hipError_t run(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        auto k1 = k_fr_setup<CONN, C>;
        hipError_t e = set_lds(k1, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k1, dim3(1), dim3(kRelaxThreads), lds, st, g, Wp, fs, max_rounds);
        hipLaunchKernelGGL(k_rank, dim3((g.N + 255) / 256), dim3(256), 0, st, fs.dbuf, g.N, fs.rank, fs.order);
        return hipGetLastError();
    }
};

template <int CONN, int C>
struct FrStep {
    static hipError_t run(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
        const int Wp = lds_row_stride(g.W);
        const size_t lds = (size_t)g.H * Wp * sizeof(int);
        auto k1 = k_fr_step<CONN, C>;
        hipError_t e = set_lds(k1, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k1, dim3(1), dim3(kRelaxThreads), lds, st, g, Wp, fs, max_rounds);
        const size_t pk = (size_t)g.N * sizeof(uint32_t);
        const int blocks = (g.N + 255) / 256;
        if (pk <= kMaxLds) {
            auto k2 = k_fr_fill<true>;
            e = set_lds(k2, pk);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k2, dim3(blocks), dim3(256), pk, st, fs, g.W);
        } else {
            hipLaunchKernelGGL(k_fr_fill<false>, dim3(blocks), dim3(256), 0, st, fs, g.W);
        }
        return hipGetLastError();
    }
};

template <int CONN, int C>
struct RelaxRowsBatched {
    static hipError_t run(const BImg *imgs, int B, int64_t n_items, size_t lds, int32_t *out, int max_rounds,
                          FrCtl *ctl, hipStream_t st) {
        auto k = k_relax_rows_batched<CONN, C>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        const int64_t gx = n_items < 65536 ? n_items : 65536;
        const int64_t gy = (n_items + gx - 1) / gx;
        hipLaunchKernelGGL(k, dim3((unsigned)gx, (unsigned)gy), dim3(kRelaxThreads), lds, st, imgs, B, out,
                           max_rounds, ctl);
        return hipGetLastError();
    }
};

template <int CONN, int C>
struct FrBatched {
    static hipError_t run(const BImg *imgs, int B, size_t lds, int max_rounds, hipStream_t st) {
        auto k = k_fr_batched<CONN, C>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(B), dim3(kRelaxThreads), lds, st, imgs, max_rounds);
        return hipGetLastError();
    }
};

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

size_t fr_workspace_bytes(int N) {
    const size_t MW = ((size_t)N + 31) / 32;
    return al256((size_t)N * MW * 4) + 6 * al256((size_t)N * 4) + al256(sizeof(FrCtl));
}

FrState fr_workspace_layout(void *ws, int N) {
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
    p += al256((size_t)N * 4);  // reserved
    f.ctl = (FrCtl *)p;
    return f;
}

// ---- launchers ----------------------------------------------------------------------------------
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

hipError_t launch_relax_rows(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                             int max_rounds, FrCtl *ctl, hipStream_t st) {
    if (K <= 0) return hipSuccess;
    return dispatch<RelaxRows>(g.conn, g.H > g.W ? g.H : g.W, g, src_list, src_base, K, out, max_rounds, ctl,
                               st);
}

hipError_t launch_fr_init(const FrState &fs, hipStream_t st) {
    hipLaunchKernelGGL(k_fr_init, dim3((fs.N + 255) / 256), dim3(256), 0, st, fs);
    return hipGetLastError();
}

hipError_t launch_fr_setup(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
    return dispatch<FrSetup>(g.conn, g.H > g.W ? g.H : g.W, g, fs, max_rounds, st);
}

hipError_t launch_fr_step(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st) {
    return dispatch<FrStep>(g.conn, g.H > g.W ? g.H : g.W, g, fs, max_rounds, st);
}

hipError_t launch_relax_rows_batched(const BImg *imgs_dev, int B, int64_t n_items, int max_line, size_t lds_bytes,
                                     int conn, int32_t *out, int max_rounds, FrCtl *ctl, hipStream_t st) {
    if (n_items <= 0) return hipSuccess;
    return dispatch<RelaxRowsBatched>(conn, max_line, imgs_dev, B, n_items, lds_bytes, out, max_rounds, ctl, st);
}

hipError_t launch_fr_batched(const BImg *imgs_dev, int B, int max_line, size_t lds_bytes, int conn, int max_rounds,
                             hipStream_t st) {
    if (B <= 0) return hipSuccess;
    return dispatch<FrBatched>(conn, max_line, imgs_dev, B, lds_bytes, max_rounds, st);
}

}  // namespace gapd
