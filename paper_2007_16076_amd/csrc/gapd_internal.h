// Internal declarations shared by the HIP kernels and the host runtime of
// libgapd.so.  Not part of the public ABI (that is include/gapd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace gapd {

// Distances of unreached pixels.  Every real distance is < 2^27 (checked at
// context creation; it leaves room for 5 flag bits in the tree words), so
// INF + any prefix of edge weights stays below 2^31.
constexpr int kInf = 0x3FFFFFFF;
constexpr int kDistLimit = 1 << 27;
// Direction code of the geodesic-tree root in the packed (d << 4 | code) words.
constexpr uint32_t kRootCode = 15u;
constexpr int kRelaxThreads = 256;   // four waves: one per sweep direction
constexpr int kMaxLine = 512;        // longest image side supported

// Edge weights of one image, all arrays H*W, row-major.  The four weight
// arrays hold the edge from pixel (y,x) to (y,x+1) [wr], (y+1,x) [wd],
// (y+1,x+1) [wdr] and (y+1,x-1) [wdl]; entries for edges leaving the image
// are 0 and never read.  P is the running sum of wr along each row
// (P[y][x] = sum_{k<x} wr[y][k]).  The c* arrays are the same data for the
// transposed image (W*H, "column view"): column sweeps are row sweeps of it.
struct GImg {
    int H, W, N, conn;
    const uint16_t *wr, *wd, *wdr, *wdl;
    const int32_t *P;
    const uint16_t *cwv, *cwdr, *cwdl;
    const int32_t *cP;
};

// Writable twin used only while building the arrays.
struct GImgW {
    int H, W, N, conn;
    uint16_t *wr, *wd, *wdr, *wdl;
    int32_t *P;
    uint16_t *cwv, *cwdr, *cwdl;
    int32_t *cP;
};

// Bytes of the weight block of an H x W image (256-aligned sub-arrays).
size_t weight_block_bytes(int H, int W);
// Lay the weight arrays out in a device block of weight_block_bytes().
GImgW weight_block_layout(void *dev, int H, int W, int conn);
inline GImg as_const(const GImgW &w) {
    GImg g;
    g.H = w.H; g.W = w.W; g.N = w.N; g.conn = w.conn;
    g.wr = w.wr; g.wd = w.wd; g.wdr = w.wdr; g.wdl = w.wdl; g.P = w.P;
    g.cwv = w.cwv; g.cwdr = w.cwdr; g.cwdl = w.cwdl; g.cP = w.cP;
    return g;
}

// Device control block of one filling-rate run.
struct FrCtl {
    int32_t s;          // source of the current step
    int32_t done;       // 1 once the least filled point is filled
    int32_t centroid;
    int32_t err;        // GAPD_ENOCONV etc. from device code
    int64_t n_prop;     // propagations done by the main loop
    int64_t filled;     // a: filled unordered pairs
    int64_t rounds;     // sweep rounds summed over propagations
    int32_t tree_slot;  // tree-cache slot holding the current source's tree, -1: the packed array
    int32_t spec_n;     // candidates listed for speculation this step
    int32_t spec_hits;  // steps whose tree came from the cache
    int32_t sp_turn1;   // spiral rules: current turn + 1 (0: none yet)
    int32_t _pad;
    int64_t spec_props; // speculative propagations computed
    int64_t spec_rounds;  // sweep rounds of the speculative pieces (also counted in rounds)
};

// Device state of the filling-rate method for one image.
// Source-selection rules of the tree-based methods.
constexpr int kRuleFilling = 0;  // least filled, then greatest extremum (Section 3.4)
constexpr int kRuleExtrema = 1;  // greatest extremum, then least filled (Section 3.3)
constexpr int kRuleSpiral = 2;   // random in the outermost unfilled turn (Sections 3.1, 3.2)

struct FrState {
    int N, MW;                 // pixels; 32-bit words per row of the filled-pairs matrix
    int H, W;
    int rule;                  // kRule*
    int rep_h;                 // spiral: repulsion distance (<= 1: none)
    int spec_cap;              // new speculative propagations planned per step, at most (0: kSpecK)
    const uint32_t *draws;     // spiral: N uniform 32-bit draws, one per selection
    int32_t *sp_in;            // spiral: membership in S by position along the turn
    uint32_t *mask;            // N * MW bits: D_mrk
    int32_t *count;            // N: filled entries of each row (diagonal included)
    int32_t *rank;             // N: position in the decreasing geodesic-extrema list
    int32_t *order;            // N: inverse of rank
    uint32_t *packed;          // N: tree words (distance, complete-row flag, parent direction)
    uint32_t *full;            // ceil(N/32) words: bit i set once count[i] == N
    // Tree cache for speculative propagations (null when not used): kSpecSlots
    // slots of N words, the slot of each source (-1: none), the source and
    // state of each slot, and the current step's plan: kSpecK sources (-1:
    // continue the slot's propagation), then the kSpecK slots.
    uint32_t *cache;
    int32_t *src_slot;
    int32_t *slot_src;
    int32_t *slot_state;       // free, ready (tree words) or running (a partial distance field)
    int32_t *spec_list;
    uint64_t *part;            // the partial select pass: sel_part_waves(N) minima, then kSelCand keys per wave
    int32_t *dbuf;             // N: distances of the setup propagations
    uint64_t *gtree;           // general graphs: N tree entries, distance << 32 | parent (-1 at the root)
    int32_t *D;                // N * N output
    FrCtl *ctl;
    int32_t *seq_out;          // nullable, N
    int64_t *filled_out;       // nullable, N
    int64_t *trace;            // nullable, kTraceFields per loop step (see gapd_stats.step_trace)
};

// Per-step trace fields (int64) of the filling-rate loop.
constexpr int kTraceFields = 32;
enum TraceField {
    kTrVisits = 0,     // ancestors walked by the fill (pairs tested)
    kTrNew = 1,        // new pairs
    kTrMaxWalk = 2,    // longest walk (ancestors)
    kTrWalkers = 3,    // pixels that walked (incomplete rows)
    kTrBlockMax = 4,   // slowest fill block (constant-clock ticks)
    kTrBlockSum = 5,   // fill-block ticks summed over blocks
    kTrStartInv = 6,   // max over fill blocks of (2^63 - 1 - start tick)
    kTrEnd = 7,        // max over fill blocks of the end tick
    kTrSpecPieces = 8, // speculative pieces run beside the fill
    kTrSpecMax = 9,    // slowest speculative piece (ticks)
    kTrSelect = 10,    // select (+ propagation on a miss) kernel (ticks)
    kTrFillBlocks = 11,  // fill blocks that ran
    kTrSpecDone = 12,    // speculative pieces that reached their fixed point
    kTrSpecEnd = 13,     // max over speculative pieces of the end tick
    kTrHit = 14,         // 1: the step's tree came from the cache
    kTrSpecStage = 15,   // speculative pieces: weights staged and field loaded (ticks summed over pieces)
    kTrSpecRound = 20,   // ... the sweep round (and the edge check of a resumed field)
    kTrSpecStore = 21,   // ... the tree words or the field written back
    // link-fill phases, ticks summed over fill blocks:
    kTrPhTables = 16,    // link tables built, counters cleared
    kTrPhDetect = 17,    // loads-only walks (the block's slowest walker)
    kTrPhWrite = 18,     // writing walks
    kTrPhFlush = 19,     // counters flushed, totals
    kTrPhDetectMax = 22, // slowest block's detect phase
    kTrPhWriteMax = 23,  // slowest block's write phase
    // select kernel phases (ticks; 28..31 unused):
    kTrSelPass = 24,     // pass over the points (keys, complete-row bitmap)
    kTrSelMin = 25,      // block argmin
    kTrSelSort = 26,     // slot keys and candidate sorts
    kTrSelRest = 27      // speculation plan, step state, propagation on a miss
};

// The link fill (the redundancy fill with 16-bit pixel ids in LDS tables).
constexpr uint32_t kNoId = 0xFFFFu;   // no such pixel (the root's parent)
__host__ __device__ inline size_t al4w(size_t n) { return (n + 3) & ~size_t(3); }
// Walking threads per block of the link fill (the default; the autotuner may
// pick 256), and 32-bit words of new-pair flags each keeps in LDS (one flag
// per ancestor; longer walks fall back to re-reading the filled-pairs matrix).
constexpr int kFillLanes = 128;
constexpr int kFillFlagWords = 12;
// Largest dynamic LDS a workgroup may use.
constexpr size_t kMaxLds = 160 * 1024 - 1024;

// The partial select pass: 256-thread workgroups of 4 points per thread,
// kSelCand candidates kept per wave.
constexpr int kSelCand = 8;
__host__ __device__ inline int sel_part_blocks(int N) { return (N + 1023) / 1024; }
__host__ __device__ inline int sel_part_waves(int N) { return 4 * sel_part_blocks(N); }

// Per-pixel counters of a link-fill block: one ancestor gains at most one
// new pair per walking thread, so 8 bits hold up to 255 walkers and 16 bits
// the rest.  log2 of the counters per 32-bit word:
__host__ __device__ constexpr int fill_cnt_shift(int lanes) { return lanes < 256 ? 2 : 1; }
// LDS of a link-fill block: L (N words), G (N uint16), the counters, the
// flags, each walker's distance, then the list of new pairs: as many words as
// remain, up to kFillListMax (at least kFillListMin for the link fill to be
// used).
constexpr int kFillListMax = 8192, kFillListMin = 1024;
__host__ __device__ inline size_t link_fill_base_words(int N, int lanes) {
    const size_t per = (size_t)1 << fill_cnt_shift(lanes);
    return al4w(N) + al4w(((size_t)N + 1) / 2) + al4w(((size_t)N + per - 1) / per) +
           (size_t)lanes * (kFillFlagWords + 1);
}
__host__ __device__ inline int link_fill_list_cap(int N, int lanes = kFillLanes) {
    const size_t base = link_fill_base_words(N, lanes), room = (kMaxLds / 4) > base ? (kMaxLds / 4) - base : 0;
    return (int)((room < (size_t)kFillListMax ? room : (size_t)kFillListMax) & ~(size_t)3);
}
__host__ __device__ inline size_t link_fill_lds(int N, int lanes = kFillLanes) {
    return 4 * (link_fill_base_words(N, lanes) + (size_t)link_fill_list_cap(N, lanes));
}
// The compact tables (images whose full tables do not fit): the parent table
// (N uint16), the flags, each walker's distance, then the list; the counts
// go straight to global memory.  256 walking threads per block.
constexpr int kCompactLanes = 256;
__host__ __device__ inline size_t compact_fill_base_words(int N, int lanes = kCompactLanes) {
    return al4w(((size_t)N + 1) / 2) + (size_t)lanes * (kFillFlagWords + 1);
}
__host__ __device__ inline int compact_fill_list_cap(int N, int lanes = kCompactLanes) {
    const size_t base = compact_fill_base_words(N, lanes), room = kMaxLds / 4 > base ? kMaxLds / 4 - base : 0;
    return (int)((room < (size_t)kFillListMax ? room : (size_t)kFillListMax) & ~(size_t)3);
}
__host__ __device__ inline size_t compact_fill_lds(int N, int lanes = kCompactLanes) {
    return 4 * (compact_fill_base_words(N, lanes) + (size_t)compact_fill_list_cap(N, lanes));
}

// Whether propagations without a tree check their edges after the first
// round by default (else only after the second).
constexpr int kNaiveCheck1 = 0;

// Launch shapes the autotuner chooses (include/gapd.h, gapd_autotune).
struct Tuning {
    int fill_lanes = kFillLanes;  // link fill: walking threads per block (128 or 256)
    int walk_pf = 16;             // link fill: ancestor pairs in flight per walk (8 or 16)
    int spec_cap = 32;            // tree modes: new speculative propagations per step (<= kSpecK)
    int naive_pfw = 4;            // naive: lines of weights the sweeps load ahead (4 or 8)
    int naive_check1 = kNaiveCheck1;  // naive: check the edges after the first round (0 or 1)
};

// Speculation: each step lists the kSpecK least-filled points whose trees are
// not cached; their propagations run beside the fill, into a cache of
// kSpecSlots trees.  A tree depends on the image only, so a cached tree is
// exactly the tree the step would compute.
constexpr int kSpecK = 32;      // speculative propagations per filling-rate step, at most
constexpr int kSpecSlots = 128; // trees kept in the cache (at most 256, a power of two)

// Workspace layout of a single-image filling-rate run (spec: with the cache).
size_t fr_workspace_bytes(int N, bool spec = false);
FrState fr_workspace_layout(void *ws, int N, bool spec = false);

// A general undirected graph on the device, in CSR form (Section 5).
struct GGraph {
    int n;
    int _pad;
    const int64_t *rp;   // n + 1 row pointers
    const int32_t *ci;   // neighbour ids
    const int32_t *cw;   // edge weights, >= 1, symmetric
    const uint8_t *bnd;  // n boundary flags
};

// Vertices a graph may have: the distance array and two frontier bitmaps of
// one propagation live in LDS.
constexpr int kGraphMaxN = 32768;

// Workspace of a tree-method run on a graph: the grid layout plus the
// 64-bit tree entries.
size_t graph_workspace_bytes(int n);
FrState graph_workspace_layout(void *ws, int n);

// Graph launchers: K propagations into K rows; setup (boundary propagation,
// centre, propagation from it, ranks); one loop step (select + propagate +
// tree, then the fill).
hipError_t launch_graph_rows(const GGraph &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                             int max_rounds, FrCtl *ctl, hipStream_t st);
hipError_t launch_graph_setup(const GGraph &g, const FrState &fs, int max_rounds, hipStream_t st);
hipError_t launch_graph_step(const GGraph &g, const FrState &fs, int max_rounds, hipStream_t st,
                             hipEvent_t mid = nullptr);

// One image of a batch, as the batched kernels see it.
struct BImg {
    GImg g;
    int Wp;             // LDS row stride of the distance tile
    int _pad;
    int64_t out_off;    // element offset of the image's N*N block in the output
    int64_t item0;      // first global work item of the image (naive batched)
    FrState fr;         // filling-rate state (batched filling-rate mode)
};

// ---- launchers (defined in kernels.hip) -------------------------------------------------
struct LaunchStatus {
    hipError_t err;
};

// Build weights of one image from its HWC bytes on the device.
hipError_t launch_prep(const GImgW &w, const uint8_t *img_dev, int C, int wmode, hipStream_t st);
// Weights of B images at once: descriptors on the device (GImgW[B]), image offsets.
hipError_t launch_prep_batched(const GImgW *w_dev, const uint8_t *imgs_dev, const int64_t *img_off_dev,
                               int B, int C, int wmode, hipStream_t st);

// Propagations from sources (list or src_base + block) into K rows of out.
// pfw: the sweeps' weight prefetch depth (0: 4; the autotuner may pick 8);
// check1: check the edges after the first round already.
hipError_t launch_relax_rows(const GImg &g, const int32_t *src_list, int src_base, int K, int32_t *out,
                             int max_rounds, FrCtl *ctl, hipStream_t st, int pfw = 0, int check1 = kNaiveCheck1);

// Filling-rate method pieces for one image.
hipError_t launch_fr_init(const FrState &fs, hipStream_t st);
// The partial select pass of the speculative step (before its step kernel).
hipError_t launch_sel_part(const FrState &fs, hipStream_t st);
hipError_t launch_fr_setup(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st);
// One loop step: select + propagate + tree (one workgroup), then the fill.
// If mid is given it is recorded between the two launches.
hipError_t launch_fr_step(const GImg &g, const FrState &fs, int max_rounds, hipStream_t st, hipEvent_t mid = nullptr,
                          const Tuning &tune = Tuning());

// Batched naive: every (image, source) item in one launch.
hipError_t launch_relax_rows_batched(const BImg *imgs_dev, int B, int64_t n_items, int max_line,
                                     size_t lds_bytes, int conn, int32_t *out, int max_rounds, FrCtl *ctl,
                                     hipStream_t st, int check1 = kNaiveCheck1);
// Batched filling rate, images in lockstep: the setup of every image, then
// steps that each cover every image still running (one select+propagate
// block per image, then the fills of all images in one launch).  lds is the
// largest distance field (H * Wp * 4), wbytes the largest LDS weight copy;
// batch_done counts the images whose loop has ended.
hipError_t launch_fr_batched_setup(const BImg *imgs_dev, int B, int max_line, int maxN, size_t lds, int conn,
                                   int max_rounds, hipStream_t st);
hipError_t launch_fr_batched_step(const BImg *imgs_dev, int B, int max_line, int maxN, size_t lds, size_t wbytes,
                                  int conn, int max_rounds, int *batch_done, hipStream_t st);

// LDS row stride for an image of width W (odd, so column walks avoid bank conflicts).
inline int lds_row_stride(int W) { return (W & 1) ? W : W + 1; }
// The link fill needs 16-bit pixel ids and its tables, with a list of at
// least kFillListMin new pairs, in LDS.
__host__ __device__ inline bool link_fill_fits(int N, int lanes = kFillLanes) {
    return N >= 1 && N < (int)kNoId && link_fill_list_cap(N, lanes) >= kFillListMin;
}
__host__ __device__ inline bool compact_fill_fits(int N) {
    return N >= 1 && N < (int)kNoId && compact_fill_list_cap(N) >= kFillListMin;
}

}  // namespace gapd
