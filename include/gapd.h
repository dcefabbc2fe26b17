/*
 * gapd.h -- all pairs of geodesic distances on a pixel grid, MI355X (gfx950).
 *
 * C ABI of libgapd.so.  The library computes, on the GPU, the N x N array of
 * geodesic distances between the N = H*W pixels of an image (Noyel, Angulo,
 * Jeulin, "Fast computation of all pairs of geodesic distances"), either by
 * the naive method (one geodesic propagation per pixel, Section 1) or by the
 * filling-rate method (Section 3.4, algorithm "filling"), which propagates
 * from one source at a time, fills the distances array along each
 * propagation's geodesic tree (Section 2, Property 1) and picks the next
 * source as the least filled point, ties broken by the geodesic-extrema list
 * of Section 3.3.
 *
 * Conventions shared by every entry point
 *   - pixel index i = y*W + x; images are HWC row-major uint8 (C bands);
 *   - the graph is the 4- or 8-neighbour grid without wrap-around
 *     (Section 2, eqs. voisinage_1/2); diagonal edges carry the plain
 *     pseudo-metric (no Euclidean factor);
 *   - edge weights are integers >= 1: GAPD_W_SUM is d_+(p,q) = f(p) + f(q)
 *     (Section 2, eq. distance_somme; one band, grey levels should be >= 1
 *     so that no edge weighs 0); GAPD_W_1PL1 is 1 + sum_b |f_b(p) - f_b(q)|
 *     for C >= 1 bands (the multiband pseudo-metric Section 5 leaves open);
 *   - distances are int32; D[i*N + j] is the geodesic distance (Section 2,
 *     eq. distance) between pixels i and j; D is symmetric with zero diagonal;
 *   - the geodesic tree of a propagation gives each pixel v != source the
 *     smallest-index neighbour q with d(q) + w(q,v) == d(v) as parent;
 *   - device pointers are HIP device addresses (e.g. torch tensor data
 *     pointers on a ROCm build); host pointers are ordinary process memory;
 *   - every call returns a status; nothing throws across the ABI.  A device
 *     error makes the context unusable (later calls return GAPD_EDEVICE).
 *
 * Limits: 1 <= H, W <= 512; the largest possible distance, hops * w_max with
 * hops = H+W-2 (4-neighbours) or max(H,W)-1 (8-neighbours), must be < 2^27,
 * else GAPD_ERANGE.
 *
 * Threading: a context belongs to one host thread and one stream at a time.
 * A server is safe to call from several host threads.
 */
#ifndef GAPD_H
#define GAPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define GAPD_OK        0
#define GAPD_PENDING   1   /* serving: job admitted or queued, not finished yet          */
#define GAPD_EINVAL   (-1) /* bad argument (sizes, modes, null pointers, sources range)   */
#define GAPD_ENOMEM   (-2) /* workspace / arena / budget too small                        */
#define GAPD_EDEVICE  (-3) /* HIP runtime or kernel error; the context is poisoned        */
#define GAPD_ERANGE   (-4) /* a distance could reach 2^27                                 */
#define GAPD_ENOCONV  (-5) /* a propagation hit its sweep-round cap                       */
#define GAPD_EBUSY    (-6) /* serving: the job is still running                           */
#define GAPD_ENOTFOUND (-7) /* serving: unknown or released ticket                        */

/* ---- options ----------------------------------------------------------------------------- */
#define GAPD_CONN4 4
#define GAPD_CONN8 8
#define GAPD_W_SUM  0
#define GAPD_W_1PL1 1
#define GAPD_MODE_NAIVE        0   /* N propagations, one row of D each (Section 1)          */
#define GAPD_MODE_TREE_FILL_FR 1   /* filling-rate method (Section 3.4, algorithm filling)  */
#define GAPD_MODE_TREE_FILL_EXTREMA 2 /* geodesic extrema method (Section 3.3, algorithm
                                         extrema): the unfilled point farthest from the
                                         geodesic centroid, the least filled (then the
                                         smallest index) among equally far ones         */
#define GAPD_MODE_TREE_FILL_SPIRAL 3 /* spiral methods (Sections 3.1, 3.2): only through
                                        gapd_all_pairs_spiral, which takes the draws  */

typedef struct gapd_ctx gapd_ctx;
typedef struct gapd_server gapd_server;

/* Statistics of one all-pairs call.  sources_out and filled_out are inputs:
 * optional DEVICE buffers of N elements each that receive, for the
 * filling-rate mode, the source of every propagation in order and a(t), the
 * number of filled pairs after each propagation (Section 2, eq. _a).  All
 * other fields are outputs. */
typedef struct {
    int64_t  n_prop;        /* propagations of the main loop (N for naive)                */
    int64_t  n_prop_setup;  /* 2 for the filling-rate mode (centroid and extrema), else 0  */
    int64_t  rounds;        /* sweep rounds summed over all propagations                  */
    int32_t  centroid;      /* geodesic centroid (filling-rate mode), else -1             */
    int32_t  _pad;
    int32_t *sources_out;   /* nullable device buffer, N int32 (input)                     */
    int64_t *filled_out;    /* nullable device buffer, N int64 (input)                     */
    float    ms_total;      /* wall time of the call, stream-event timed                   */
    float    ms_setup;      /* centroid and extrema propagations (filling-rate mode)       */
    float    ms_kernel;     /* naive mode: duration of its single propagation kernel,
                               timed by events on the context's stream                    */
    int32_t  time_kernels;  /* input: nonzero asks the filling-rate mode to time each
                               launch of its two loop kernels with events                 */
    float    ms_step_kernels; /* sum of durations of the select+propagate launches        */
    float    ms_fill_kernels; /* sum of durations of the redundancy-fill launches         */
    int32_t  graph_replays; /* tree modes: chunks of loop steps replayed as a HIP graph
                               (captured once per call; GAPD_FR_GRAPH=0 turns it off)    */
    int64_t  n_prop_speculative; /* filling-rate mode: propagations computed ahead for
                                    likely next sources (not counted in n_prop)          */
    int64_t  n_cache_hits;  /* filling-rate steps whose propagation was such a tree, taken
                               from the cache instead of being propagated again          */
    int64_t *step_trace;    /* input: nullable DEVICE buffer of 32*N int64, zeroed by the
                               call; for the filling-rate and extrema modes with the tree
                               cache, loop step t fills entries 32t..32t+31 with the
                               ancestors the fill walked, the new pairs, the longest walk,
                               the pixels that walked, the slowest fill block, the sum over
                               fill blocks, 2^63-1 minus the first block start, the last
                               block end, the speculative pieces run, the slowest piece,
                               the select kernel, the fill blocks, the pieces that reached
                               their fixed point, the last piece end, 1 if the step's tree
                               came from the cache, the speculative pieces' staging
                               summed over them, then the link fill's phases summed over
                               its workgroups (link tables built, loads-only walks,
                               writing walks, counters flushed), the pieces' sweep rounds
                               and write-backs summed over them, the slowest workgroup's
                               two walk phases, the select kernel's phases (pass over the
                               points, argmin, slot keys and sorts, the rest) and 4 zeros
                               (times in ticks of the device's constant clock,
                               hipDeviceAttributeWallClockRate kHz).  Tracing adds a
                               little work to those kernels.                             */
    int64_t  rounds_speculative; /* filling-rate and extrema modes: the sweep rounds of the
                                    speculative propagations (part of rounds)             */
} gapd_stats;

/* ---- single image ------------------------------------------------------------------------ */

/* Create a context for one image (Section 2: the image as a grid graph with a
 * pseudo-metric).  image: HOST pointer to H*W*C bytes, HWC row-major; it is
 * copied to the device together with the edge weights derived from it, in
 * device memory the context owns until gapd_destroy.  conn: GAPD_CONN4 or
 * GAPD_CONN8.  weight_mode: GAPD_W_SUM (requires C == 1) or GAPD_W_1PL1.
 * Runs on the null stream until gapd_set_stream.  On error *out is NULL. */
int gapd_create(const uint8_t *image, int H, int W, int C, int conn, int weight_mode, gapd_ctx **out);

/* Use this HIP stream (a hipStream_t passed as void*) for later calls. */
int gapd_set_stream(gapd_ctx *ctx, void *hip_stream);

/* Bytes of caller-provided device workspace that gapd_all_pairs(mode) or
 * gapd_all_pairs_spiral needs (0 for the naive mode; the same for the three
 * tree modes).  It holds the filled-pairs bit matrix D_mrk (Section 2),
 * N*ceil(N/32)*4 bytes, a cache of 128 geodesic trees (4N bytes each) and
 * O(N) arrays. */
int gapd_workspace_size(gapd_ctx *ctx, int mode, size_t *bytes);

/* Hand the context a DEVICE workspace of at least gapd_workspace_size bytes,
 * 256-byte aligned.  The caller owns it and must keep it alive while calls
 * that use it may run on the stream. */
int gapd_set_workspace(gapd_ctx *ctx, void *dev_ptr, size_t bytes);

/* One geodesic propagation per source (Section 1): out[k*N + v] = d(sources[k], v).
 * sources: DEVICE pointer to K int32 pixel ids in [0, N) (checked on the host
 * after a copy; out-of-range ids give GAPD_EINVAL and nothing is written);
 * out: DEVICE pointer to K*N int32.  Returns when the rows are complete (the
 * call synchronises the context's stream). */
int gapd_sssp(gapd_ctx *ctx, const int32_t *sources, int K, int32_t *out);

/* Every entry of the N x N distances array D.  out: DEVICE pointer to N*N
 * int32.  mode GAPD_MODE_NAIVE runs N propagations; GAPD_MODE_TREE_FILL_FR
 * runs the filling-rate method, GAPD_MODE_TREE_FILL_EXTREMA the geodesic
 * extrema method; both need the workspace.  All give the same, unique D
 * (Section 2, Property 1).  The tree modes need H <= 192 and W <= 192 (their
 * propagation keeps the distance field in LDS), else GAPD_EINVAL.
 * GAPD_MODE_TREE_FILL_SPIRAL is refused here
 * (GAPD_EINVAL): it needs draws.  st: nullable host struct.  Returns when the
 * result is complete on the stream (the call synchronises the stream). */
int gapd_all_pairs(gapd_ctx *ctx, int mode, int32_t *out, gapd_stats *st);

/* The spiral method (Section 3.1, algorithm spiral) for h <= 1, and the
 * spiral method with repulsion (Section 3.2; the paper uses h = 3) for h >= 2.
 * Turn k is the frame of the pixels at distance k from the image border,
 * listed clockwise from its top-left corner (one row or column: left to
 * right, top to bottom).  Each step removes the filled points from S; when S
 * is empty it takes the outermost turn with an unfilled point and sets S to
 * its unfilled points; draw t (the t-th propagation) picks member
 * floor(draws[t] * |S| / 2^32) of S in turn order; with repulsion the turn
 * pixels 1 .. h-1 positions away from the source on either side (cyclically
 * on a closed frame) leave S.
 *   h      0 <= h <= 65536
 *   draws  DEVICE pointer to N uniform uint32 draws, caller-owned, read only
 *          (N always suffice: every propagation completes its source's row)
 *   out    DEVICE pointer to N*N int32
 * Needs the workspace of gapd_workspace_size(GAPD_MODE_TREE_FILL_SPIRAL), and
 * H <= 192 and W <= 192 (GAPD_EINVAL otherwise).
 * No setup propagations (st->n_prop_setup = 0, st->centroid = -1). */
int gapd_all_pairs_spiral(gapd_ctx *ctx, int h, const uint32_t *draws, int32_t *out, gapd_stats *st);

/* gapd_all_pairs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results, with the tree modes' workspace taken from a fixed device
 * scratch of 64 MiB that the library holds on every device it runs on until
 * the process ends, instead of the caller's workspace.  It calls no
 * hipMalloc, hipFree, event creation or other allocating routine (the
 * first call on a device looks up the scratch's address once).  Tree modes
 * whose workspace (gapd_workspace_size) exceeds 64 MiB give GAPD_ENOMEM
 * (N up to about 18000 fit); the naive mode needs no scratch.  Every call on
 * one device shares that device's scratch, and each call clears what it
 * needs at its start, so calls that overlap on one device (several streams
 * or threads) race and must be serialised by the caller.  Timing fields of
 * st stay 0.  Returns when the result is complete (the call synchronises the
 * context's stream). */
int gapd_all_pairs_noalloc(gapd_ctx *ctx, int mode, int32_t *out, gapd_stats *st);

/* Launch shapes chosen by gapd_autotune. */
typedef struct {
    int32_t fill_lanes;   /* tree modes: walking threads per fill workgroup (128 or 256)   */
    int32_t walk_pf;      /* tree modes: ancestor pairs in flight per walk (8 or 16)       */
    int32_t spec_cap;     /* tree modes: new speculative propagations per step (16 or 32)  */
    int32_t naive_pfw;    /* naive mode: lines of edge weights each sweep loads ahead (4, 8) */
    float   ms;           /* the chosen shapes' call time                                  */
    float   ms_default;   /* the default shapes' call time                                 */
    int32_t candidates;   /* shapes timed                                                   */
    int32_t naive_check1; /* naive mode: check the edges after the first sweep round (1)
                             or only after the second (0)                              */
} gapd_tuning;

/* Time the candidate launch shapes of `mode` (GAPD_MODE_NAIVE,
 * GAPD_MODE_TREE_FILL_FR or GAPD_MODE_TREE_FILL_EXTREMA) with one whole
 * gapd_all_pairs call each on this context's image (after one warm-up call;
 * the tree modes need the workspace), and keep the fastest, in the process
 * and in a JSON cache file (GAPD_TUNE_FILE, else gapd_tune.json beside
 * libgapd.so), keyed by (device architecture, H x W x C, connectivity,
 * mode).  Every later call on an image of that key uses them.  The results
 * (D and the rest) are the same for every shape.  out: DEVICE N*N int32
 * that receives the calls' D.  best: nullable host struct.  Other modes give
 * GAPD_EINVAL. */
int gapd_autotune(gapd_ctx *ctx, int mode, int32_t *out, gapd_tuning *best);

/* Pin the launch shapes that `mode` uses on images of this context's key,
 * for the rest of the process (the cache file is not written).  Only
 * fill_lanes, walk_pf, spec_cap, naive_pfw and naive_check1 are read; values
 * outside fill_lanes {128, 256}, walk_pf {8, 16}, spec_cap 1..32, naive_pfw
 * {4, 8}, naive_check1 {0, 1} give GAPD_EINVAL. */
int gapd_set_tuning(gapd_ctx *ctx, int mode, const gapd_tuning *t);

/* Release the context and its device memory (not the caller's buffers). */
void gapd_destroy(gapd_ctx *ctx);

/* Text for a status code, and the context's last error message. */
const char *gapd_strerror(int status);
const char *gapd_last_error(gapd_ctx *ctx);

/* ---- general graphs (Section 5) --------------------------------------------------------- */

/* The paper's methods apply to any graph once its boundary vertices are
 * known: they replace the image border in the first propagation that finds
 * the geodesic centre (Section 5).  A graph context holds an undirected
 * graph in CSR form on the device.
 *   n         vertices, 1 <= n <= 32768 (one propagation's distances and
 *             frontier live in LDS)
 *   row_ptr   HOST, n+1 int64: row v lists col_idx[row_ptr[v] .. row_ptr[v+1])
 *   col_idx   HOST, int32 neighbour ids
 *   weight    HOST, int32 edge weights, >= 1
 *   boundary  HOST, nullable, n flags; null takes the example rule of
 *             Section 5: the vertices with fewer neighbours than the average
 *             degree (every vertex when none has); an all-zero mask is
 *             refused
 * Every edge must appear in both rows with the same weight, with no self
 * loop and no repeated neighbour, and the graph must be connected, else
 * GAPD_EINVAL.  Every distance is at most the total weight of the
 * breadth-first spanning tree from vertex 0; if that reaches 2^27, or any
 * single edge weighs 2^27 or more, the call gives GAPD_ERANGE.  The arrays are copied.  gapd_last_error(NULL) explains a failed create. */
typedef struct gapd_graph gapd_graph;
int gapd_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const int32_t *weight,
                      const uint8_t *boundary, gapd_graph **out);
int gapd_graph_set_stream(gapd_graph *g, void *hip_stream);
/* Workspace for GAPD_MODE_TREE_FILL_FR and _EXTREMA: the filled-pairs bit
 * matrix, O(n) arrays and n 8-byte tree entries (0 for naive). */
int gapd_graph_workspace_size(gapd_graph *g, int mode, size_t *bytes);
int gapd_graph_set_workspace(gapd_graph *g, void *dev_ptr, size_t bytes);
/* K propagations (Section 1): out[k*n + v] = d(sources[k], v); sources and
 * out are DEVICE pointers; ids out of range give GAPD_EINVAL. */
int gapd_graph_sssp(gapd_graph *g, const int32_t *sources, int K, int32_t *out);
/* All of D (n x n int32, DEVICE) by GAPD_MODE_NAIVE, GAPD_MODE_TREE_FILL_FR
 * or GAPD_MODE_TREE_FILL_EXTREMA (other modes: GAPD_EINVAL).  The geodesic
 * tree of a propagation gives each vertex the smallest-index neighbour q
 * with d(q) + w(q,v) = d(v) as parent; st as for gapd_all_pairs. */
int gapd_graph_all_pairs(gapd_graph *g, int mode, int32_t *out, gapd_stats *st);
const char *gapd_graph_last_error(gapd_graph *g);
void gapd_graph_destroy(gapd_graph *g);

/* ---- many images in one launch ------------------------------------------------------------ */

/* Workspace bytes for gapd_all_pairs_batched with these image sizes (host
 * arrays H[B], W[B]). */
int gapd_batched_workspace_size(const int32_t *H, const int32_t *W, int B, int C, int conn, int mode,
                                size_t *bytes);

/* All-pairs distances of B images in one pass: naive mode runs every
 * (image, source) propagation of the batch in one kernel launch; the tree
 * modes (GAPD_MODE_TREE_FILL_FR, GAPD_MODE_TREE_FILL_EXTREMA) run the images'
 * sequential loops in lockstep, each step one launch with a workgroup per
 * unfinished image (select and propagate) and one fill launch over all
 * images.  Other modes give GAPD_EINVAL.
 *   images_packed: HOST, the B images back to back (H[b]*W[b]*C bytes each);
 *   H, W:          HOST, B sizes each;
 *   out:           DEVICE int32; image b's N_b x N_b array starts at
 *                  out + out_offsets[b];
 *   out_offsets:   HOST, B+1 int64 element offsets (nondecreasing, the span
 *                  of image b at least N_b^2 elements);
 *   n_prop_out:    nullable HOST, B int64: loop propagations per image;
 *   sources_out:   nullable DEVICE int32, sum of N_b elements: tree modes
 *                  write image b's sources in order from element
 *                  N_0 + ... + N_(b-1) on (n_prop_out[b] of them);
 *   workspace:     DEVICE, gapd_batched_workspace_size bytes, 256-aligned.
 * Synchronises the stream before returning. */
int gapd_all_pairs_batched(const uint8_t *images_packed, const int32_t *H, const int32_t *W, int B, int C,
                           int conn, int weight_mode, int mode, int32_t *out, const int64_t *out_offsets,
                           int64_t *n_prop_out, int32_t *sources_out, void *workspace, size_t ws_bytes,
                           void *hip_stream);

/* ---- serving ---------------------------------------------------------------------------------- */

#define GAPD_JOB_ALL_PAIRS    0
#define GAPD_JOB_MULTI_SOURCE 1

typedef struct {
    int            kind;        /* GAPD_JOB_ALL_PAIRS or GAPD_JOB_MULTI_SOURCE              */
    int            H, W, C, conn, weight_mode;
    int            mode;        /* all-pairs jobs: GAPD_MODE_NAIVE, _TREE_FILL_FR or
                                   _TREE_FILL_EXTREMA (others: GAPD_EINVAL)                 */
    const uint8_t *image;       /* HOST, H*W*C bytes; copied at submit                      */
    const int32_t *sources;     /* HOST, K ids (multi-source jobs); copied at submit        */
    int            K;
} gapd_job;

typedef struct {
    int32_t *dev_out;           /* DEVICE result inside the arena: N*N or K*N int32          */
    size_t   elems;
    int64_t  n_prop;            /* all-pairs jobs: loop propagations (N for naive)          */
    double   t_submit, t_admit, t_done;  /* seconds, steady clock of the server           */
} gapd_result;

/* Create a server over a caller-owned DEVICE arena (arena_bytes, 256-aligned).
 * Jobs are admitted first come first served while their bytes fit in the arena
 * and a slot is free (max_slots running jobs); admitted jobs run concurrently
 * on max_slots streams of the current device.  The server owns a scheduler
 * thread until gapd_server_destroy.  The slot streams are non-blocking: work
 * the caller queued on the arena (a fill, a copy) must be complete before
 * this call, or it may land on top of the jobs' data. */
int gapd_server_create(void *arena_dev, size_t arena_bytes, int max_slots, gapd_server **out);

/* Queue a job; never blocks.  The image and sources are copied.  *ticket
 * identifies it.  GAPD_ENOMEM if the job alone can never fit in the arena. */
int gapd_serve_submit(gapd_server *srv, const gapd_job *job, uint64_t *ticket);

/* GAPD_PENDING while queued or running, GAPD_OK with *res filled when done
 * (the result stays valid until gapd_serve_release), or the job's error.  A
 * job is marked done or failed only once its slot's stream has drained.  A
 * device error fails that job with GAPD_EDEVICE and poisons the server: every
 * job admitted after it fails with GAPD_EDEVICE too. */
int gapd_serve_poll(gapd_server *srv, uint64_t ticket, gapd_result *res);

/* Block until the job is done (or failed); same results as gapd_serve_poll. */
int gapd_serve_wait(gapd_server *srv, uint64_t ticket, gapd_result *res);

/* Return a finished job's arena bytes so queued jobs can be admitted.
 * GAPD_EBUSY if it is still running. */
int gapd_serve_release(gapd_server *srv, uint64_t ticket);

/* Stop the scheduler (waits for running jobs) and free the server. */
void gapd_server_destroy(gapd_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GAPD_H */
