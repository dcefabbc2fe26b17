/*
 * gapd_oracle.c -- plain, slow, CPU reference for all pairs of geodesic
 * distances on a pixel grid (Noyel, Angulo, Jeulin, "Fast computation of all
 * pairs of geodesic distances").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library, and the GPU library never calls it.
 *
 * What it computes, each function citing the passage it follows:
 *   - edge weights: the "sum of grey levels" pseudo-metric d_+ (Section 2, eq.
 *     distance_somme) and, for multiband images, 1 + L1 spectral difference
 *     (the paper's Section 5 leaves the multiband pseudo-metric open; this is
 *     the reading used throughout);
 *   - geodesic distance = minimum over paths of the summed edge weights
 *     (Section 2, eqs. temps and distance), by Dijkstra with a binary heap,
 *     and independently by Floyd-Warshall for tiny images;
 *   - the naive method: one propagation per pixel (Section 1);
 *   - the filling-rate method (Section 3.4, algorithm "filling"), with the
 *     geodesic centroid and the decreasing list of geodesic extrema
 *     (Section 3.3), and the redundancy fill along geodesic trees
 *     (Section 2, Property 1);
 *   - with the same fill, the geodesic extrema method (Section 3.3,
 *     algorithm "extrema") and the spiral methods without and with repulsion
 *     (Sections 3.1 and 3.2), whose random draws are inputs;
 *   - the same propagation, tree, fill and selection rules on a general
 *     undirected graph in CSR form, whose boundary vertices replace the image
 *     border (Section 5).
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - pixel index i = y*W + x; no wrap-around at the image border;
 *   - 4-neighbours in ascending index order: up, left, right, down;
 *     8-neighbours: (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1) (+1,-1) (+1,0) (+1,+1);
 *     diagonal edges use the same pseudo-metric (no Euclidean factor);
 *   - geodesic tree: the parent of v != root is the smallest-index neighbour q
 *     with d(q) + w(q,v) == d(v), computed from the final distances;
 *   - the tree fills exactly its ancestor/descendant pairs, both orientations;
 *   - "propagation from the edges": every border pixel starts at distance 0;
 *     the centroid is the first pixel (smallest index) of maximal distance;
 *   - the extrema list orders pixels by decreasing distance from the
 *     centroid, ties by increasing index; "Ext[x]" is x's position (rank);
 *   - the filling rate of a point is carried as the integer count of filled
 *     entries of its row (diagonal included), which has the same argmin;
 *   - extrema method: among the unfilled points at the greatest distance
 *     from the centroid, the least filled, then the smallest index;
 *   - spiral turns are listed clockwise from their top-left corner; a random
 *     draw r (uniform 32 bits) picks member floor(r |S| / 2^32) of S in that
 *     order; repulsion h removes from S the turn pixels 1 .. h-1 positions
 *     away from s on either side (cyclically on a closed frame); a point is
 *     "filled" when its row of D is complete;
 *   - general graphs: the boundary vertices are given, or by the example rule
 *     of Section 5 the vertices of degree below the average (all vertices
 *     when none is); weights are given per edge, symmetric, >= 1; the graph
 *     must be connected.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ERANGE (-4)
#define OR_TRUNCATED 2

#define OR_W_SUM 0
#define OR_W_1PL1 1

/* ORACLE_MUTANT plants one deliberate mistake (build with -DORACLE_MUTANT=k);
 * the test suite builds each mutant and checks that its pins reject it. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* The graph of a propagation: a pixel grid (img != NULL) or a general
 * undirected graph in CSR form (rp != NULL; the generalisation of Section 5). */
typedef struct {
    const uint8_t *img; /* H*W*C bytes, HWC row-major */
    int H, W, C, conn, wmode;
    const int64_t *rp;  /* CSR: row pointers (N+1) */
    const int32_t *ci;  /* CSR: neighbour ids */
    const int32_t *cw;  /* CSR: edge weights (>= 1) */
    const uint8_t *bnd; /* CSR: boundary flags (N) */
    int64_t N;
    int64_t maxdeg;
} or_graph;

static int or_check(const or_graph *g) {
    if (!g->img || g->H < 1 || g->W < 1 || g->C < 1) return OR_EINVAL;
    if (g->conn != 4 && g->conn != 8) return OR_EINVAL;
    if (g->wmode == OR_W_SUM && g->C != 1) return OR_EINVAL;
    if (g->wmode != OR_W_SUM && g->wmode != OR_W_1PL1) return OR_EINVAL;
    return OR_OK;
}

/* Edge weight between neighbouring pixels p and q.  d_+ is Section 2, eq.
 * distance_somme; the multiband weight is 1 + sum over bands |f_b(p)-f_b(q)|. */
static int64_t or_weight(const or_graph *g, int64_t p, int64_t q) {
    if (g->wmode == OR_W_SUM) {
        if (ORACLE_MUTANT == 2) return 2 * (int64_t)g->img[p];
        return (int64_t)g->img[p] + (int64_t)g->img[q];
    }
    int64_t s = ORACLE_MUTANT == 8 ? 0 : 1;
    for (int b = 0; b < g->C; ++b) {
        int64_t a = g->img[p * g->C + b], c = g->img[q * g->C + b];
        s += a > c ? a - c : c - a;
    }
    return s;
}

/* Neighbours of p and the weights of the edges to them.  Pixel grid: the
 * 4- or 8-neighbours (Section 2, eqs. voisinage_1/2) in ascending index order;
 * CSR graph: the row of p as given.  out and wout hold g->maxdeg entries. */
static int64_t or_neighbours(const or_graph *g, int64_t p, int64_t *out, int64_t *wout) {
    int64_t n = 0;
    if (g->rp) {
        for (int64_t e = g->rp[p]; e < g->rp[p + 1]; ++e) {
            out[n] = g->ci[e];
            wout[n++] = g->cw[e];
        }
        return n;
    }
    int y = (int)(p / g->W), x = (int)(p % g->W);
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dy == 0 && dx == 0) continue;
            if (g->conn == 4 && dy != 0 && dx != 0) continue;
            int yy = y + dy, xx = x + dx;
            if (yy < 0 || yy >= g->H || xx < 0 || xx >= g->W) continue;
            out[n] = (int64_t)yy * g->W + xx;
            wout[n] = or_weight(g, p, out[n]);
            ++n;
        }
    return n;
}

/* Boundary vertices: the image border pixels (Section 3.3), or the flags of
 * a CSR graph (Section 5). */
static int or_is_boundary(const or_graph *g, int64_t p) {
    if (g->rp) return g->bnd[p] != 0;
    int y = (int)(p / g->W), x = (int)(p % g->W);
    return y == 0 || (y == g->H - 1 && ORACLE_MUTANT != 7) || x == 0 || x == g->W - 1;
}

/* ---- binary heap of (distance, node), lazy deletion ---------------------------------- */
typedef struct { int64_t d; int64_t v; } or_item;
typedef struct { or_item *a; int64_t n, cap; } or_heap;

static int or_push(or_heap *h, int64_t d, int64_t v) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        or_item *na = (or_item *)realloc(h->a, (size_t)nc * sizeof(or_item));
        if (!na) return OR_ENOMEM;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].d <= d) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].d = d; h->a[i].v = v;
    return OR_OK;
}

static or_item or_pop(or_heap *h) {
    or_item top = h->a[0], last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        int64_t md = last.d;
        if (l < h->n && h->a[l].d < md) { m = l; md = h->a[l].d; }
        if (r < h->n && h->a[r].d < md) { m = r; }
        if (m == i) break;
        h->a[i] = h->a[m];
        i = m;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* Geodesic propagation (Section 1: "computing the geodesic distance from one
 * pixel to all others"): Dijkstra from a set of seeds at distance 0. */
static int or_dijkstra(const or_graph *g, const int64_t *seeds, int64_t nseeds, int64_t *dist) {
    const int64_t INF = INT64_MAX / 4;
    for (int64_t i = 0; i < g->N; ++i) dist[i] = INF;
    or_heap h = {0, 0, 0};
    for (int64_t k = 0; k < nseeds; ++k) {
        if (seeds[k] < 0 || seeds[k] >= g->N) { free(h.a); return OR_EINVAL; }
        dist[seeds[k]] = 0;
        if (or_push(&h, 0, seeds[k])) { free(h.a); return OR_ENOMEM; }
    }
    int64_t *nb = (int64_t *)malloc((size_t)(2 * g->maxdeg + 2) * sizeof(int64_t)), *wb = nb + g->maxdeg + 1;
    if (!nb) { free(h.a); return OR_ENOMEM; }
    while (h.n > 0) {
        or_item it = or_pop(&h);
        if (it.d != dist[it.v]) continue; /* stale entry */
        int64_t k = or_neighbours(g, it.v, nb, wb);
        for (int64_t j = 0; j < k; ++j) {
            int64_t nd = it.d + wb[j];
            if (nd < dist[nb[j]]) {
                dist[nb[j]] = nd;
                if (or_push(&h, nd, nb[j])) { free(h.a); free(nb); return OR_ENOMEM; }
            }
        }
    }
    free(h.a);
    free(nb);
    return OR_OK;
}

static int or_graph_init(or_graph *g, const uint8_t *img, int H, int W, int C, int conn, int wmode) {
    memset(g, 0, sizeof(*g));
    g->img = img; g->H = H; g->W = W; g->C = C; g->conn = conn; g->wmode = wmode;
    g->N = (int64_t)H * W;
    g->maxdeg = 8;
    return or_check(g);
}

/* ---- exported entry points ---------------------------------------------------------- */

/* Multi-seed propagation; dist receives N int64 distances. */
int gapd_oracle_dijkstra(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                         const int64_t *seeds, int64_t nseeds, int64_t *dist) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    if (!dist || nseeds < 1 || !seeds) return OR_EINVAL;
    return or_dijkstra(&g, seeds, nseeds, dist);
}

/* Floyd-Warshall on the same graph (textbook all-pairs shortest paths), int64,
 * for tiny images only: D receives N*N entries. */
int gapd_oracle_floyd(const uint8_t *img, int H, int W, int C, int conn, int wmode, int64_t *D) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    if (!D || g.N > 1024) return OR_EINVAL;
    const int64_t N = g.N, INF = INT64_MAX / 4;
    for (int64_t i = 0; i < N * N; ++i) D[i] = INF;
    int64_t nb[8], wb[8];
    for (int64_t p = 0; p < N; ++p) {
        D[p * N + p] = 0;
        int64_t k = or_neighbours(&g, p, nb, wb);
        for (int64_t j = 0; j < k; ++j) D[p * N + nb[j]] = wb[j];
    }
    for (int64_t k = 0; k < N; ++k)
        for (int64_t i = 0; i < N; ++i) {
            int64_t dik = D[i * N + k];
            if (dik >= INF) continue;
            for (int64_t j = 0; j < N; ++j) {
                int64_t c = dik + D[k * N + j];
                if (c < D[i * N + j]) D[i * N + j] = c;
            }
        }
    return OR_OK;
}

/* Rows of the distances array for K given sources (one propagation each);
 * out receives K*N int32.  The naive method (Section 1) is sources = 0..N-1. */
static int or_rows(const or_graph *gp, const int32_t *sources, int64_t K, int32_t *out, int nthreads) {
    const or_graph g = *gp;
    if (!out || K < 0 || (K > 0 && !sources)) return OR_EINVAL;
    for (int64_t k = 0; k < K; ++k)
        if (sources[k] < 0 || sources[k] >= g.N) return OR_EINVAL;
    int err = OR_OK;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *dist = (int64_t *)malloc((size_t)g.N * sizeof(int64_t));
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < K; ++k) {
            if (!dist) { err = OR_ENOMEM; continue; }
            int64_t s = sources[k];
            int e = or_dijkstra(&g, &s, 1, dist);
            if (e) { err = e; continue; }
            for (int64_t v = 0; v < g.N; ++v) {
                if (dist[v] > INT32_MAX) { err = OR_ERANGE; break; }
                out[k * g.N + v] = (int32_t)dist[v];
            }
        }
        free(dist);
    }
    return err;
}

int gapd_oracle_rows(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                     const int32_t *sources, int64_t K, int32_t *out, int nthreads) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_rows(&g, sources, K, out, nthreads);
}

/* The naive method (Section 1): N propagations, one per pixel; D is N*N int32. */
int gapd_oracle_naive(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                      int32_t *D, int nthreads) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    int32_t *src = (int32_t *)malloc((size_t)g.N * sizeof(int32_t));
    if (!src) return OR_ENOMEM;
    for (int64_t i = 0; i < g.N; ++i) src[i] = (int32_t)i;
    st = gapd_oracle_rows(img, H, W, C, conn, wmode, src, g.N, D, nthreads);
    free(src);
    return st;
}

/* Geodesic tree of a propagation (Section 2: root, nodes, leaves): parent of
 * v is the smallest-index neighbour q with dist(q) + w(q,v) == dist(v); the
 * root (dist 0, a seed) gets parent -1.  Computed from the final distances. */
static int or_parents(const or_graph *g, const int64_t *dist, int32_t *parent) {
    int64_t *nb = (int64_t *)malloc((size_t)(2 * g->maxdeg + 2) * sizeof(int64_t)), *wb = nb + g->maxdeg + 1;
    if (!nb) return OR_ENOMEM;
    for (int64_t v = 0; v < g->N; ++v) {
        parent[v] = -1;
        if (dist[v] == 0) continue;
        int64_t k = or_neighbours(g, v, nb, wb);
        for (int64_t j = 0; j < k; ++j)  /* the weights are symmetric: w(q,v) = w(v,q) */
            if (dist[nb[j]] + wb[j] == dist[v]) {
                const int better = ORACLE_MUTANT == 1 ? nb[j] > parent[v] : (parent[v] < 0 || nb[j] < parent[v]);
                if (better) parent[v] = (int32_t)nb[j];
            }
    }
    free(nb);
    return OR_OK;
}

int gapd_oracle_parents(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                        const int64_t *dist, int32_t *parent) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_parents(&g, dist, parent);
}

/* Geodesic centroid and decreasing list of geodesic extrema (Section 3.3):
 * a propagation from all border pixels, c = first pixel of maximal distance,
 * a propagation from c, rank[x] = position of x when pixels are sorted by
 * decreasing distance from c (ties: increasing index). */
static const int64_t *or_sort_key;
static int or_cmp_rank(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (or_sort_key[i] != or_sort_key[j]) return or_sort_key[i] > or_sort_key[j] ? -1 : 1;
    if (ORACLE_MUTANT == 3) return i > j ? -1 : (i < j ? 1 : 0);
    return i < j ? -1 : (i > j ? 1 : 0);
}

static int or_extrema(const or_graph *gp, int32_t *centroid, int64_t *d_edge, int64_t *d_c, int32_t *rank) {
    const or_graph g = *gp;
    int st;
    int64_t nb = 0;
    int64_t *seeds = (int64_t *)malloc((size_t)g.N * sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)g.N * sizeof(int64_t));
    if (!seeds || !order) { free(seeds); free(order); return OR_ENOMEM; }
    for (int64_t p = 0; p < g.N; ++p)
        if (or_is_boundary(&g, p)) seeds[nb++] = p;
    st = or_dijkstra(&g, seeds, nb, d_edge);
    if (!st) {
        int64_t c = 0;
        for (int64_t p = 1; p < g.N; ++p)
            if (d_edge[p] > d_edge[c] || (ORACLE_MUTANT == 6 && d_edge[p] == d_edge[c])) c = p;
        *centroid = (int32_t)c;
        st = or_dijkstra(&g, &c, 1, d_c);
    }
    if (!st) {
        for (int64_t p = 0; p < g.N; ++p) order[p] = p;
        or_sort_key = d_c;
        qsort(order, (size_t)g.N, sizeof(int64_t), or_cmp_rank);
        for (int64_t r = 0; r < g.N; ++r) rank[order[r]] = (int32_t)r;
    }
    free(seeds); free(order);
    return st;
}

int gapd_oracle_extrema(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                        int32_t *centroid, int64_t *d_edge, int64_t *d_c, int32_t *rank) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_extrema(&g, centroid, d_edge, d_c, rank);
}

/* ---- spiral turns (Section 3.1) ------------------------------------------------------- */

/* Spiral turn k of an H x W image: the one-pixel-wide frame of the pixels
 * whose distance to the image border, min(y, x, H-1-y, W-1-x), is k (k = 0 is
 * the outermost).  Listed clockwise from its top-left corner (k,k): the top
 * row left to right, the right column downwards, the bottom row right to
 * left, the left column upwards.  A turn of one row or one column is listed
 * left to right or top to bottom.  Returns the length, 0 if the turn does not
 * exist.  *cyclic is set when the list closes on itself (a proper frame). */
int gapd_oracle_spiral_turn(int H, int W, int k, int32_t *out, int *cyclic) {
    const int top = k, left = k, bottom = H - 1 - k, right = W - 1 - k;
    int n = 0;
    if (cyclic) *cyclic = 0;
    if (k < 0 || top > bottom || left > right) return 0;
    if (top == bottom) {
        for (int x = left; x <= right; ++x) out[n++] = top * W + x;
        return n;
    }
    if (left == right) {
        for (int y = top; y <= bottom; ++y) out[n++] = y * W + left;
        return n;
    }
    if (cyclic) *cyclic = 1;
    for (int x = left; x <= right; ++x) out[n++] = top * W + x;
    for (int y = top + 1; y <= bottom; ++y) out[n++] = y * W + right;
    for (int x = right - 1; x >= left; --x) out[n++] = bottom * W + x;
    if (ORACLE_MUTANT == 10) return n;  /* mutant: the left column is dropped */
    for (int y = bottom - 1; y > top; --y) out[n++] = y * W + left;
    return n;
}

/* ---- the tree-based methods: one loop, three selection rules --------------------------- */

#define OR_RULE_FILLING 0  /* Section 3.4, algorithm "filling"                          */
#define OR_RULE_EXTREMA 1  /* Section 3.3, algorithm "extrema"                          */
#define OR_RULE_SPIRAL  2  /* Section 3.1 "spiral" and 3.2 "spiral with repulsion"        */

/* State of the spiral selection: the current turn and the list S of its
 * pixels that are still candidates (in_s, by position along the turn). */
typedef struct {
    int turn;        /* -1: no turn selected yet */
    int len, cyclic;
    int32_t *pix;    /* pixels of the turn, in turn order */
    uint8_t *in_s;   /* membership in S, by position */
} or_spiral;

/* Every method below has the same body (Section 2): compute the geodesic
 * tree from the selected source s, fill D along it by Property 1, then update
 * the filled-pairs matrix D_mrk and the per-point counts.  Only the choice of
 * s differs.
 *   rule       OR_RULE_*
 *   h          spiral only: repulsion distance; after s is drawn, the turn
 *              pixels at 1 .. h-1 positions on either side of s leave S
 *              (h <= 1: plain spiral method)
 *   rnd        spiral only: one uniform 32-bit draw per selection; draw r
 *              picks the floor(r * |S| / 2^32)-th member of S in turn order
 *   n_rnd      length of rnd; the call fails with OR_EINVAL if it runs out
 * Returns OR_TRUNCATED when max_steps (>= 0) stops the loop early. */
static int or_tree_methods(const or_graph *gp, int rule, int h, const uint32_t *rnd, int64_t n_rnd, int32_t *D,
                           int32_t *seq_out, int64_t *a_out, int64_t *n_prop, int32_t *centroid_out,
                           int32_t *rank_out, int64_t max_steps) {
    const or_graph g = *gp;
    const int H = g.H, W = g.W;
    int st = OR_OK;
    if (!D || !n_prop) return OR_EINVAL;
    if (rule == OR_RULE_SPIRAL && g.rp) return OR_EINVAL; /* spiral turns need a pixel grid */
    if (rule == OR_RULE_SPIRAL && !rnd && n_rnd > 0) return OR_EINVAL;
    const int64_t N = g.N;
    uint8_t *mrk = (uint8_t *)calloc((size_t)(N * N), 1);
    int64_t *count = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int32_t *rank = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int32_t *parent = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int64_t *da = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t *dc = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    or_spiral sp = {-1, 0, 0, (int32_t *)malloc((size_t)(2 * (H + W) + 4) * sizeof(int32_t)),
                    (uint8_t *)calloc((size_t)(2 * (H + W) + 4), 1)};
    if (!mrk || !count || !rank || !parent || !da || !dc || !sp.pix || !sp.in_s) { st = OR_ENOMEM; goto done; }

    /* The geodesic centroid and the decreasing list of geodesic extrema
     * (Section 3.3); dc keeps the distances from the centroid. */
    int32_t c;
    st = or_extrema(&g, &c, da, dc, rank);
    if (st) goto done;
    if (centroid_out) *centroid_out = c;
    if (rank_out) memcpy(rank_out, rank, (size_t)N * sizeof(int32_t));

    /* D_mrk(i,i) = 1 by convention, so every point starts with one filled entry. */
    for (int64_t i = 0; i < N; ++i) { mrk[i * N + i] = 1; count[i] = 1; D[i * N + i] = 0; }
    int64_t filled = 0, t = 0;
    *n_prop = 0;
    for (;;) {
        int64_t s = -1;
        if (rule == OR_RULE_FILLING) {
            /* B = argmin tau; among several, the greatest extremum (smallest rank). */
            s = 0;
            for (int64_t x = 1; x < N; ++x)
                if (count[x] < count[s] || (count[x] == count[s] && ORACLE_MUTANT != 5 && rank[x] < rank[s])) s = x;
            if (count[s] == N) break; /* the least filled point is filled: D is filled */
        } else if (rule == OR_RULE_EXTREMA) {
            /* Ext without its filled points; B = its points at the greatest
             * distance from the centroid; s = the least filled of B (then the
             * smallest index). */
            for (int64_t x = 0; x < N; ++x) {
                if (count[x] == N) continue;
                if (s < 0 || dc[x] > dc[s]) { s = x; continue; }
                if (dc[x] == dc[s] && (ORACLE_MUTANT == 9 ? count[x] > count[s] : count[x] < count[s])) s = x;
            }
            if (s < 0) break; /* every point is filled */
        } else {
            /* Remove the points of S which are filled. */
            int64_t ns = 0;
            for (int p = 0; p < sp.len; ++p) {
                if (sp.in_s[p] && count[sp.pix[p]] == N) sp.in_s[p] = 0;
                ns += sp.in_s[p];
            }
            if (ns == 0) {
                /* S is empty: the most exterior turn that is not yet filled,
                 * and S = its pixels that are not yet filled. */
                int k = -1;
                for (int64_t x = 0; x < N; ++x) {
                    if (count[x] == N) continue;
                    const int y = (int)(x / W), xx = (int)(x % W);
                    int b = y < xx ? y : xx;
                    if (H - 1 - y < b) b = H - 1 - y;
                    if (W - 1 - xx < b) b = W - 1 - xx;
                    if (k < 0 || b < k) k = b;
                }
                if (k < 0) break; /* D is filled */
                sp.turn = k;
                sp.len = gapd_oracle_spiral_turn(H, W, k, sp.pix, &sp.cyclic);
                for (int p = 0; p < sp.len; ++p) {
                    sp.in_s[p] = count[sp.pix[p]] < N;
                    ns += sp.in_s[p];
                }
            }
            /* Select a source point s randomly in S. */
            if (t >= n_rnd) { st = OR_EINVAL; goto done; }
            int64_t j = (int64_t)(((uint64_t)rnd[t] * (uint64_t)ns) >> 32), pos = -1;
            for (int p = 0; p < sp.len; ++p)
                if (sp.in_s[p] && j-- == 0) { pos = p; break; }
            s = sp.pix[pos];
            /* Repulsion: the h-1 turn pixels on either side of s leave S. */
            for (int dd = 1; dd < h; ++dd)
                for (int side = -1; side <= 1; side += 2) {
                    int64_t p = pos + side * dd;
                    if (sp.cyclic) p = ((p % sp.len) + sp.len) % sp.len;
                    else if (p < 0 || p >= sp.len) continue;
                    if (ORACLE_MUTANT != 11 || side > 0) sp.in_s[p] = 0;
                }
        }
        if (max_steps >= 0 && t >= max_steps) { st = OR_TRUNCATED; break; }

        /* Compute the geodesic tree from s. */
        st = or_dijkstra(&g, &s, 1, da);
        if (st) goto done;
        st = or_parents(&g, da, parent);
        if (st) goto done;

        /* Fill D along the tree (Property 1): each ancestor u of v gives
         * d(u,v) = d(s,v) - d(s,u). */
        for (int64_t v = 0; v < N; ++v) {
            for (int64_t u = parent[v]; u >= 0; u = parent[u]) {
                if (mrk[u * N + v]) continue;
                int64_t duv = da[v] - da[u];
                if (duv > INT32_MAX) { st = OR_ERANGE; goto done; }
                D[u * N + v] = (int32_t)duv;
                if (ORACLE_MUTANT != 4) D[v * N + u] = (int32_t)duv;
                mrk[u * N + v] = 1;
                mrk[v * N + u] = 1;
                count[u] += 1;
                count[v] += 1;
                filled += 1;
            }
        }
        if (seq_out) seq_out[t] = (int32_t)s;
        if (a_out) a_out[t] = filled;
        ++t;
        *n_prop = t;
    }
done:
    free(mrk); free(count); free(rank); free(parent); free(da); free(dc); free(sp.pix); free(sp.in_s);
    return st;
}

/* The filling-rate method (Section 3.4, algorithm "filling").
 *   D          N*N int32 output (every entry written exactly once)
 *   seq_out    N int32, the source of each propagation (nullable)
 *   a_out      N int64, filled pairs a after each propagation (nullable;
 *              Section 2, eq. _a)
 *   n_prop     number of propagations in the loop (the two setup propagations
 *              of the centroid and extrema are not included)
 *   max_steps  stop after this many propagations (<0: no limit); the call then
 *              returns OR_TRUNCATED and D is only partly written
 * The filled-pairs matrix D_mrk (Section 2) is kept as one byte per entry and
 * the per-point filling rate tau(x) (eq. filling_rate_pt) as the integer
 * numerator count[x] = sum_k D_mrk(k, x).  */
int gapd_oracle_filling_rate(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                             int32_t *D, int32_t *seq_out, int64_t *a_out, int64_t *n_prop,
                             int32_t *centroid_out, int32_t *rank_out, int64_t max_steps) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_tree_methods(&g, OR_RULE_FILLING, 0, NULL, 0, D, seq_out, a_out, n_prop, centroid_out, rank_out,
                           max_steps);
}

/* The geodesic extrema method (Section 3.3, algorithm "extrema"): the source
 * is the unfilled point farthest from the geodesic centroid, the least filled
 * among equally far ones.  Arguments as for gapd_oracle_filling_rate. */
int gapd_oracle_extrema_method(const uint8_t *img, int H, int W, int C, int conn, int wmode,
                               int32_t *D, int32_t *seq_out, int64_t *a_out, int64_t *n_prop,
                               int32_t *centroid_out, int64_t max_steps) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_tree_methods(&g, OR_RULE_EXTREMA, 0, NULL, 0, D, seq_out, a_out, n_prop, centroid_out, NULL,
                           max_steps);
}

/* The spiral method (Section 3.1, algorithm "spiral"; h <= 1) and the spiral
 * method with repulsion (Section 3.2; the paper's h is 3): sources drawn at
 * random in the most exterior spiral turn not yet filled.  rnd holds n_rnd
 * uniform 32-bit draws, one per propagation (N always suffice). */
int gapd_oracle_spiral(const uint8_t *img, int H, int W, int C, int conn, int wmode, int h,
                       const uint32_t *rnd, int64_t n_rnd, int32_t *D, int32_t *seq_out, int64_t *a_out,
                       int64_t *n_prop, int64_t max_steps) {
    or_graph g;
    int st = or_graph_init(&g, img, H, W, C, conn, wmode);
    if (st) return st;
    return or_tree_methods(&g, OR_RULE_SPIRAL, h, rnd, n_rnd, D, seq_out, a_out, n_prop, NULL, NULL, max_steps);
}

/* ---- general graphs (Section 5: any graph, once its boundary vertices are known) ------- */

/* Boundary vertices by the example rule of Section 5: fewer neighbours than
 * the graph's average degree.  When no vertex qualifies (a regular graph),
 * every vertex is a boundary vertex.  out: n flags. */
int gapd_oracle_graph_boundary(int64_t n, const int64_t *rp, uint8_t *out) {
    if (n < 1 || !rp || !out) return OR_EINVAL;
    int64_t any = 0;
    for (int64_t v = 0; v < n; ++v) {
        /* deg(v) < m / n, in integers */
        out[v] = ORACLE_MUTANT == 12 ? (rp[v + 1] - rp[v]) * n <= rp[n] : (rp[v + 1] - rp[v]) * n < rp[n];
        any += out[v];
    }
    if (!any)
        for (int64_t v = 0; v < n; ++v) out[v] = 1;
    return OR_OK;
}

/* A CSR graph is accepted when: rp[0] = 0, rows are nondecreasing, every
 * neighbour id is in range and not the vertex itself, no row repeats a
 * neighbour, every weight is >= 1, every edge (u, v, w) has its reverse
 * (v, u, w), and the graph is connected.  bnd (nullable) gives the boundary
 * flags; without it the degree rule is used (*owned then holds the flags). */
static int or_csr_init(or_graph *g, int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                       const uint8_t *bnd, uint8_t **owned) {
    memset(g, 0, sizeof(*g));
    *owned = NULL;
    if (n < 1 || !rp || rp[0] != 0) return OR_EINVAL;
    for (int64_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return OR_EINVAL;
    const int64_t m = rp[n];
    if (m > 0 && (!ci || !cw)) return OR_EINVAL;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t deg = rp[v + 1] - rp[v];
        if (deg > maxdeg) maxdeg = deg;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int64_t u = ci[e];
            if (u < 0 || u >= n || u == v || cw[e] < 1) return OR_EINVAL;
            for (int64_t f = rp[v]; f < e; ++f)
                if (ci[f] == u) return OR_EINVAL;
            int found = 0;
            for (int64_t f = rp[u]; f < rp[u + 1]; ++f)
                if (ci[f] == v && cw[f] == cw[e]) { found = 1; break; }
            if (!found) return OR_EINVAL;
        }
    }
    /* connected: a breadth-first search from vertex 0 reaches every vertex */
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    if (!queue || !seen) { free(queue); free(seen); return OR_ENOMEM; }
    int64_t head = 0, tail = 0;
    queue[tail++] = 0;
    seen[0] = 1;
    while (head < tail) {
        const int64_t v = queue[head++];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (!seen[ci[e]]) { seen[ci[e]] = 1; queue[tail++] = ci[e]; }
    }
    free(queue);
    free(seen);
    if (tail != n) return OR_EINVAL;
    g->rp = rp; g->ci = ci; g->cw = cw; g->N = n; g->maxdeg = maxdeg;
    if (bnd) {
        g->bnd = bnd;
    } else {
        uint8_t *b = (uint8_t *)malloc((size_t)n);
        if (!b) return OR_ENOMEM;
        gapd_oracle_graph_boundary(n, rp, b);
        g->bnd = b;
        *owned = b;
    }
    return OR_OK;
}

/* Multi-seed propagation on a CSR graph (Section 1, on the graph of Section 5). */
int gapd_oracle_graph_dijkstra(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                               const int64_t *seeds, int64_t nseeds, int64_t *dist) {
    or_graph g;
    uint8_t *owned;
    int st = or_csr_init(&g, n, rp, ci, cw, NULL, &owned);
    if (!st) st = (!dist || nseeds < 1 || !seeds) ? OR_EINVAL : or_dijkstra(&g, seeds, nseeds, dist);
    free(owned);
    return st;
}

/* Canonical geodesic-tree parents on a CSR graph (smallest-index tight neighbour). */
int gapd_oracle_graph_parents(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                              const int64_t *dist, int32_t *parent) {
    or_graph g;
    uint8_t *owned;
    int st = or_csr_init(&g, n, rp, ci, cw, NULL, &owned);
    if (!st) st = or_parents(&g, dist, parent);
    free(owned);
    return st;
}

/* Rows of D for K sources on a CSR graph; the naive method is sources 0..n-1. */
int gapd_oracle_graph_rows(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                           const int32_t *sources, int64_t K, int32_t *out, int nthreads) {
    or_graph g;
    uint8_t *owned;
    int st = or_csr_init(&g, n, rp, ci, cw, NULL, &owned);
    if (!st) st = or_rows(&g, sources, K, out, nthreads);
    free(owned);
    return st;
}

/* Geodesic centre and extrema ranks of a CSR graph, the first propagation
 * starting from the boundary vertices (Section 5). */
int gapd_oracle_graph_extrema(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                              const uint8_t *bnd, int32_t *centroid, int64_t *d_edge, int64_t *d_c, int32_t *rank) {
    or_graph g;
    uint8_t *owned;
    int st = or_csr_init(&g, n, rp, ci, cw, bnd, &owned);
    if (!st) st = or_extrema(&g, centroid, d_edge, d_c, rank);
    free(owned);
    return st;
}

/* The filling-rate method (rule 0) or the geodesic extrema method (rule 1)
 * on a CSR graph.  Outputs as for gapd_oracle_filling_rate. */
int gapd_oracle_graph_tree_method(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *cw,
                                  const uint8_t *bnd, int rule, int32_t *D, int32_t *seq_out, int64_t *a_out,
                                  int64_t *n_prop, int32_t *centroid_out, int32_t *rank_out, int64_t max_steps) {
    if (rule != OR_RULE_FILLING && rule != OR_RULE_EXTREMA) return OR_EINVAL;
    or_graph g;
    uint8_t *owned;
    int st = or_csr_init(&g, n, rp, ci, cw, bnd, &owned);
    if (!st)
        st = or_tree_methods(&g, rule, 0, NULL, 0, D, seq_out, a_out, n_prop, centroid_out, rank_out, max_steps);
    free(owned);
    return st;
}
