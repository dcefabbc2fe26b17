// General undirected graphs in CSR form (Section 5).
#include "dev_common.h"

namespace gapd {

namespace {

// ---------------------------------------------------------------------------------------------
// General graphs (Section 5): the same propagations, trees, fill and
// selection rules on an undirected CSR graph.
// ---------------------------------------------------------------------------------------------

// Frontier list capacity of a graph propagation: what LDS holds beside the
// n distances and the two frontier bitmaps, at most 8192 entries.
__host__ __device__ inline int graph_list_cap(int n) {
    const long long rest = (long long)kMaxLds - 4ll * n - 8ll * ((n + 31) / 32);
    return (int)(rest / 4 < 8192 ? rest / 4 : 8192);
}

__host__ __device__ inline size_t graph_prop_lds(int n) {
    return (size_t)n * 4 + 8 * (size_t)((n + 31) / 32) + 4 * (size_t)graph_list_cap(n);
}

// LDS of a graph propagation: n distances, two frontier bitmaps, the list.
struct GFront {
    uint32_t *cur, *nxt;
    int *list;
    int cap;
};

__device__ __forceinline__ GFront graph_lds(int n, int *smem, int *&d) {
    const int nw = (n + 31) >> 5;
    GFront f;
    d = smem;
    f.cur = (uint32_t *)(smem + n);
    f.nxt = f.cur + nw;
    f.list = (int *)(f.nxt + nw);
    f.cap = graph_list_cap(n);
    return f;
}

// Relax the edges of v (distance dv) in rows e0..e1, 8 edge loads in flight;
// improved vertices join the next frontier.
__device__ __forceinline__ void graph_relax_edges(const GGraph &g, int *d, uint32_t *nxt, int dv, int64_t e0,
                                                  int64_t e1, int &any) {
    for (int64_t e = e0; e < e1; e += 8) {
        int u[8], w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t ee = e + k < e1 ? e + k : e1 - 1;  // a repeated edge relaxes nothing new
            u[k] = g.ci[ee];
            w[k] = g.cw[ee];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int nd = dv + w[k];
            if (nd < d[u[k]] && nd < atomicMin(&d[u[k]], nd)) {
                atomicOr(&nxt[u[k] >> 5], 1u << (u[k] & 31));
                any = 1;
            }
        }
    }
}

// One propagation on a CSR graph by a frontier Bellman-Ford in LDS: every
// vertex whose distance dropped in the last round relaxes its edges (LDS
// atomic minimums; a vertex that improves joins the next frontier).  d and
// the bitmap f.cur hold the seeds on entry; f.nxt is zero.  Positive weights
// end it within n rounds.  Returns the rounds, or -1 at the cap.  Each round
// compacts the frontier into an LDS list (in passes of at most f.cap
// vertices) so that the threads share it evenly.
__device__ int graph_relax_block(const GGraph &g, int *d, GFront f, int max_rounds, int64_t *red) {
    const int nw = (g.n + 31) >> 5;
    for (int r = 1; r <= max_rounds; ++r) {
        int any = 0;
        for (;;) {
            int c = 0;
            for (int w = threadIdx.x; w < nw; w += blockDim.x) c += __popc(f.cur[w]);
            int total;
            int pos = block_excl_scan(c, red, &total);
            if (total == 0) break;
            for (int w = threadIdx.x; w < nw && pos < f.cap; w += blockDim.x) {
                uint32_t b = f.cur[w];
                while (b && pos < f.cap) {
                    f.list[pos++] = (w << 5) + __ffs(b) - 1;
                    b &= b - 1;
                }
                f.cur[w] = b;  // what did not fit waits for the next pass
            }
            __syncthreads();
            const int F = total < f.cap ? total : f.cap;
            for (int i = threadIdx.x; i < F; i += blockDim.x) {
                const int v = f.list[i];
                graph_relax_edges(g, d, f.nxt, d[v], g.rp[v], g.rp[v + 1], any);
            }
            __syncthreads();
            if (total <= f.cap) break;  // the whole frontier was listed
        }
        if (!__syncthreads_or(any)) return r;
        uint32_t *t = f.cur;
        f.cur = f.nxt;
        f.nxt = t;
    }
    return -1;
}

// d = INF, frontiers empty; then the seeds (seed < 0: the boundary vertices).
__device__ void graph_seed(const GGraph &g, int *d, const GFront &f, int seed) {
    const int nw = (g.n + 31) >> 5;
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) d[v] = kInf;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) { f.cur[w] = 0; f.nxt[w] = 0; }
    __syncthreads();
    if (seed >= 0) {
        if (threadIdx.x == 0) { d[seed] = 0; f.cur[seed >> 5] = 1u << (seed & 31); }
    } else {
        for (int v = threadIdx.x; v < g.n; v += blockDim.x)
            if (g.bnd[v]) { d[v] = 0; atomicOr(&f.cur[v >> 5], 1u << (v & 31)); }
    }
    __syncthreads();
}

// Block b propagates from src_list[b] (or src_base + b) and writes row b.
__global__ __launch_bounds__(kRelaxThreads) void k_graph_rows(GGraph g, const int32_t *src_list, int src_base,
                                                             int32_t *out, int max_rounds, FrCtl *ctl) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    int *d;
    const GFront f = graph_lds(g.n, smem, d);
    const int s = src_list ? src_list[blockIdx.x] : src_base + (int)blockIdx.x;
    graph_seed(g, d, f, s);
    const int r = graph_relax_block(g, d, f, max_rounds, (int64_t *)red);
    int32_t *row = out + (size_t)blockIdx.x * g.n;
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) row[v] = d[v];
    if (threadIdx.x == 0) {
        if (r < 0) atomicExch(&ctl->err, GAPD_ENOCONV);
        atomicAdd((unsigned long long *)&ctl->rounds, (unsigned long long)(r < 0 ? max_rounds : r));
    }
}

// Geodesic centre and extrema of a graph (Section 5): propagate from the
// boundary vertices, take the first vertex of maximal distance, propagate
// from it into fs.dbuf.  One block.
__global__ __launch_bounds__(kRelaxThreads) void k_graph_setup(GGraph g, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    int *d;
    const GFront f = graph_lds(g.n, smem, d);
    graph_seed(g, d, f, -1);
    const int r1 = graph_relax_block(g, d, f, max_rounds, (int64_t *)red);
    uint64_t best = ~0ull;
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) {
        const uint64_t key = ((uint64_t)(uint32_t)(kInf - d[v]) << 32) | (uint32_t)v;
        best = key < best ? key : best;
    }
    best = block_min_u64(best, red);
    const int c = (int)(best & 0xFFFFFFFFu);
    graph_seed(g, d, f, c);
    const int r2 = graph_relax_block(g, d, f, max_rounds, (int64_t *)red);
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) fs.dbuf[v] = d[v];
    if (threadIdx.x == 0) {
        fs.ctl->centroid = c;
        if (r1 < 0 || r2 < 0) fs.ctl->err = GAPD_ENOCONV;
        fs.ctl->rounds += (r1 < 0 ? max_rounds : r1) + (r2 < 0 ? max_rounds : r2);
    }
}

// Select by the filling-rate or extrema rule, propagate from the source and
// write the tree entries: parent = the smallest-index neighbour q with
// d(q) + w(q,v) = d(v), from the final distances.  One block.
__global__ __launch_bounds__(kRelaxThreads) void k_graph_step(GGraph g, FrState fs, int max_rounds) {
    extern __shared__ int smem[];
    __shared__ uint64_t red[kRelaxThreads / 64];
    FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    if (threadIdx.x == 0 && fs.filled_out && ctl->n_prop > 0) fs.filled_out[ctl->n_prop - 1] = ctl->filled;
    const int s = fs.rule == kRuleExtrema ? fr_select<kRuleExtrema>(fs, red) : fr_select<kRuleFilling>(fs, red);
    if (s < 0) {
        if (threadIdx.x == 0) ctl->done = 1;
        return;
    }
    if (threadIdx.x == 0) {
        if (fs.seq_out) fs.seq_out[ctl->n_prop] = s;
        ctl->s = s;
        ctl->n_prop += 1;
    }
    int *d;
    const GFront f = graph_lds(g.n, smem, d);
    graph_seed(g, d, f, s);
    const int r = graph_relax_block(g, d, f, max_rounds, (int64_t *)red);
    for (int v = threadIdx.x; v < g.n; v += blockDim.x) {
        const int dv = d[v];
        uint32_t par = 0xFFFFFFFFu;
        if (v != s) {
            const int64_t e1 = g.rp[v + 1];
            for (int64_t e = g.rp[v]; e < e1; ++e) {
                const int q = g.ci[e];
                if (d[q] + g.cw[e] == dv && (uint32_t)q < par) par = (uint32_t)q;
            }
        }
        fs.gtree[v] = ((uint64_t)(uint32_t)dv << 32) | par;
    }
    if (threadIdx.x == 0) {
        if (r < 0) ctl->err = GAPD_ENOCONV;
        ctl->rounds += r < 0 ? max_rounds : r;
    }
}

// Tree entry helpers: distance in bits 32..61, complete-row flag in bit 62
// (set only on the LDS copy), parent in the low 32 bits (-1 at the root).
constexpr uint64_t kGFilled = 1ull << 62;
__device__ __forceinline__ int gt_dist(uint64_t t) { return (int)((t >> 32) & 0x3FFFFFFFu); }
__device__ __forceinline__ int gt_parent(uint64_t t) { return (int)(uint32_t)t; }

// Redundancy fill for vertex v along its ancestors (Property 1), as
// fill_from, with the parent read from the tree entry.  Without the LDS copy
// an ancestor's complete row is read from the bitmap (never the source's:
// block 0 marks it complete while other blocks may still walk).
template <bool kLds, bool kCntLds>
__device__ int graph_fill_from(const FrState &fs, const uint64_t *tr, int v, int s, int *cnt) {
    const int N = fs.N, MW = fs.MW;
    const uint64_t tv = tr[v];
    const int dv = gt_dist(tv);
    uint32_t *mrow = fs.mask + (size_t)v * MW;
    int32_t *Drow = fs.D + (size_t)v * N;
    int nnew = 0;
    for (int u = gt_parent(tv); u >= 0;) {
        const uint64_t tu = tr[u];
        const bool complete = kLds ? (tu & kGFilled) != 0 : (u != s && ((fs.full[u >> 5] >> (u & 31)) & 1u));
        if (!complete && !((mrow[u >> 5] >> (u & 31)) & 1u)) {
            const int val = dv - gt_dist(tu);
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
        u = gt_parent(tu);
    }
    return nnew;
}

template <bool kLds, bool kLdsCount>
__global__ __launch_bounds__(256) void k_graph_fill(FrState fs) {
    extern __shared__ uint64_t sgt[];
    __shared__ int64_t red[4];
    const FrCtl *ctl = fs.ctl;
    if (ctl->done) return;
    const int s = ctl->s, N = fs.N;
    const uint64_t *tr = fs.gtree;
    int *cnt = fs.count;
    if (kLds) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) sgt[i] = fs.gtree[i];
        __syncthreads();
        for (int w = threadIdx.x; w < fs.MW; w += blockDim.x) {
            uint32_t b = fs.full[w];
            while (b) {
                const int i = w * 32 + __ffs(b) - 1;
                b &= b - 1;
                if (i != s) sgt[i] |= kGFilled;
            }
        }
        tr = sgt;
    }
    if (kLdsCount) {
        cnt = (int *)(sgt + (kLds ? N : 0));
        for (int i = threadIdx.x; i < N; i += blockDim.x) cnt[i] = 0;
    }
    __syncthreads();
    int64_t mine = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        if (v == s) continue;
        if (kLds ? (tr[v] & kGFilled) != 0 : ((fs.full[v >> 5] >> (v & 31)) & 1u) != 0) continue;
        const int n = graph_fill_from<kLds, kLdsCount>(fs, tr, v, s, cnt);
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
    if (blockIdx.x == 0) {
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

}  // namespace

size_t graph_workspace_bytes(int n) { return fr_workspace_bytes(n, false) + al256((size_t)n * 8); }

FrState graph_workspace_layout(void *ws, int n) {
    FrState f = fr_workspace_layout(ws, n, false);
    f.gtree = (uint64_t *)((char *)ws + fr_workspace_bytes(n, false));
    return f;
}


hipError_t launch_graph_rows(const GGraph &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                             int max_rounds, FrCtl *ctl, hipStream_t st) {
    if (K <= 0) return hipSuccess;
    const size_t lds = graph_prop_lds(g.n);
    hipError_t e = set_lds(k_graph_rows, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_graph_rows, dim3(K), dim3(kRelaxThreads), lds, st, g, src_list, src_base, out, max_rounds,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_graph_setup(const GGraph &g, const FrState &fs, int max_rounds, hipStream_t st) {
    const size_t lds = graph_prop_lds(g.n);
    hipError_t e = set_lds(k_graph_setup, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_graph_setup, dim3(1), dim3(kRelaxThreads), lds, st, g, fs, max_rounds);
    hipLaunchKernelGGL(k_rank, dim3((g.n + 255) / 256), dim3(256), 0, st, fs.dbuf, g.n, fs.rank, fs.order);
    return hipGetLastError();
}

template <bool kLds, bool kLdsCount>
static hipError_t launch_graph_fill(const FrState &fs, size_t lds, hipStream_t st) {
    auto k = k_graph_fill<kLds, kLdsCount>;
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((fs.N + 255) / 256), dim3(256), lds, st, fs);
    return hipGetLastError();
}

hipError_t launch_graph_step(const GGraph &g, const FrState &fs, int max_rounds, hipStream_t st, hipEvent_t mid) {
    const size_t lds = graph_prop_lds(g.n);
    hipError_t e = set_lds(k_graph_step, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_graph_step, dim3(1), dim3(kRelaxThreads), lds, st, g, fs, max_rounds);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (mid) {
        e = hipEventRecord(mid, st);
        if (e != hipSuccess) return e;
    }
    const size_t tb = (size_t)g.n * 8, cb = (size_t)g.n * 4;
    if (tb + cb <= kMaxLds) return launch_graph_fill<true, true>(fs, tb + cb, st);
    if (tb <= kMaxLds) return launch_graph_fill<true, false>(fs, tb, st);
    return launch_graph_fill<false, false>(fs, 0, st);
}

}  // namespace gapd
