// Internal declarations of the gfx950 FMM library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "fmm2d.h"

#define FMM_PMAX 64             // largest expansion order supported
#define FMM_BN 132              // binomial table: C(n,k) for 0 <= n,k < FMM_BN
#define FMM_MAXL 15             // deepest tree (4^15 leaves)
#define FMM_DEFAULT_LIST_CAP 256

// status bits written by kernels into the handle's device status word
#define FMM_ST_LIST_OVERFLOW 1
#define FMM_ST_ORDERS_SHORT 2   // caller's pair orders shorter than the weak list
#define FMM_ST_TREE_INCONSISTENT 4 // internal check of the tree build failed
#define FMM_ST_NONFINITE 8      // a coordinate or strength is NaN or infinite
#define FMM_LB_TILE 4096         // records per tile of the one-pass partition

// learned truncation order
#define FMM_NF FMM2D_PORDER_NFEAT
#define FMM_HID FMM2D_PORDER_HIDDEN

static inline int64_t box_off(int l) { return ((((int64_t)1) << (2 * l)) - 1) / 3; }
static inline int64_t nbox(int l) { return ((int64_t)1) << (2 * l); }
static inline int64_t start_off(int l) { return box_off(l) + l; }

// Index of the calling wave in a 1-D grid of 64-wide waves.  readfirstlane
// tells the compiler the value is wave-uniform, so everything derived from it
// (loop bounds, list entries, source records) lives in scalar registers and is
// fetched with scalar loads.
// Position of block b among the blocks [b0, b1) of a launch, so that each
// XCD takes runs of XCD_RUN consecutive positions: workgroups go to the 8 XCDs
// round-robin (XCD = b mod 8), and a run of neighbouring leaves in one XCD
// finds the data it shares in that XCD's L2; runs go to the XCDs in turn,
// which spreads uneven work.  Blocks past the last whole group of 8 runs keep
// their place.  A bijection onto [0, b1 - b0) whatever the hardware order.
#define XCD_RUN 16
__device__ __forceinline__ int32_t xcd_order(int32_t b, int32_t b0, int32_t b1)
{
    const int32_t r = b - b0, n = b1 - b0;
    const int32_t full = n / (8 * XCD_RUN) * (8 * XCD_RUN);
    if (r >= full) return r;
    const int32_t x = r & 7, i = r >> 3; // XCD (relative to b0) and rank on it
    return ((i / XCD_RUN) * 8 + x) * XCD_RUN + i % XCD_RUN;
}

// Tile of block b of nb for work of equal size per tile: the blocks of one
// XCD (b mod 8) take one range of consecutive tiles, so that the cache lines
// which neighbouring tiles share (the ends of their output runs) are written
// through one L2.  A bijection onto [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + (b >> 3);
}

__device__ __forceinline__ int32_t wave_index()
{
    return __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64));
}

__device__ __forceinline__ int64_t d_box_off(int l) { return ((((int64_t)1) << (2 * l)) - 1) / 3; }
__device__ __forceinline__ int64_t d_start_off(int l) { return d_box_off(l) + l; }

// --------------------------------------------------------------------------
// Workspace layout: every array of one evaluation, carved out of the caller's
// buffer at 256-byte aligned offsets.  The layout depends only on the sizes
// and options, so fmm2d_workspace_size and fmm2d_eval agree.
struct fmm_layout {
    int64_t ns, nt;    // sources; separate targets (0 = at sources)
    int L, p, cap;     // levels, order, list capacity per box
    int mixed, learned;
    int64_t nb;        // boxes over all levels
    int64_t nleaf;
    int64_t nstart;    // entries of the per-level start arrays
    int64_t nstep;     // entries of the per-split-step start arrays
    int64_t listcap;   // entries of each global list array
    // offsets (bytes)
    size_t keys[2], vals[2];     // radix sort ping-pong (max(ns,nt) each)
    size_t hist;                 // radix histogram / scan block sums
    size_t hist2;                // radix histogram of the y presort when it runs beside the x one
    size_t srec, trec;           // 4 x n records (x- and y-ordered lists, ping-pong)
    size_t srank;                // x and y presort orders, x and y rank of every source (4 ns)
    size_t scoord;               // source x and y coordinates in sorted order (2 ns)
    size_t lbst;                 // partition tile states (4 lists) and tickets
    int64_t lbtiles;             // tiles per list
    size_t perm, tperm;          // leaf-order original indices (sources / targets)
    size_t bsum;                 // partition / scan block sums
    size_t sstep, tstep;         // per-step starts (sources / targets)
    size_t seg_axis, seg_pc, seg_pi, seg_nlo, seg_tlo, seg_LO, seg_TLO;
    size_t seg_nlox, seg_nloy, seg_LOy; // lo counts of the moving source lists, prefix of the y one
    size_t sbits;                // per segment and source list: the buffer holding it (current, next)
    size_t stseg;                // per source partition tile: the segment of its first position
    size_t stcnt;                // per source list and tile: moving lo count, then its prefix
    size_t sstart, tstart;       // per-level starts (output)
    size_t centre, radius;
    size_t wcnt, scnt;           // per-box list counts (current level)
    size_t woff, soff;           // per-level list offsets
    size_t widx, sidx;           // global list arrays
    size_t mcnt, pcnt, moff, poff, midx, pidx; // finest-level M2P / P2L lists
    int64_t leafcap;             // entries of each M2P / P2L array
    size_t lbsum;                // list scan block sums
    size_t lhvy, lhcnt;          // list build: heavy boxes per level (level-local ids), their counts
    size_t lhpart;               // list build: class counts per heavy box and part (16 parts)
    size_t srcs;                 // double4 sources in leaf order
    size_t tgts;                 // double2 targets in leaf order
    size_t m32;                  // float2 strengths in leaf order (mixed)
    size_t A, B;                 // FP64 multipoles / locals [nb][p+1] complex
    size_t A32;                  // FP32 radius-scaled multipoles (mixed)
    size_t n1, tail;             // per-box coefficient norms (order features)
    size_t vmin, budget;         // per-box label budget
    size_t hs, hoff, hbox, hpart; // M2L heavy-box segments (counts, offsets, box, partials)
    size_t nhw, nhoff, nuleaf, npart; // near-field units of heavy leaves
    int64_t nucap;               // capacity in near-field units
    size_t nsum;                 // near sums per leaf-order target: Phi' [n], then Phi [n] (double2)
    size_t mut_ucnt, mut_uoff, mut_rev; // mutual near field: upper entries per leaf, their scan, reverse sums
    int64_t mut_rcap;            // capacity of mut_rev in upper entries
    int64_t hmax;                // capacity in segments
    size_t qw;                   // uint8 order per weak pair, weak-list order
    size_t sw, sp;               // weak pairs sorted by order within a box: source, order
    size_t pbox;                 // target box of every weak pair (order phase)
    size_t total;
};

int fmm_plan_layout(int64_t ns, int64_t nt, int L, int p, int cap, int mixed, int learned,
                    fmm_layout *lay, int mutual);

// --------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All asynchronous on `st`.
struct fmm_tree_args {
    int64_t ns, nt;               // nt = 0 at sources
    int L;
    double theta;
    const double *src;            // [2 ns] caller order
    const double *tgt;            // [2 nt] or NULL
    char *ws;
    const fmm_layout *lay;
    int32_t *status;              // device status word
    int cap;
    int swap;                     // leaf-level swapped criterion (P2L / M2P)
    // side stream (or NULL): the y presort runs there beside the x presort,
    // forked and joined with the two events
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
};
// Builds perm/tperm, per-level starts, centres, radii and lists; gathers the
// sources (with strengths) and targets into leaf order.
hipError_t fmm_build_tree(const fmm_tree_args &a, const double *m, hipStream_t st);
hipError_t fmm_build_lists(const fmm_tree_args &a, hipStream_t st);

struct fmm_eval_args {
    int L, p, kernel, mixed;      // mixed: 0 FP64, 1 FP32 near and far field, 2 FP32 far field only
    int64_t ns, nt;               // nt == ns when at sources
    int at_sources;
    const char *ws;
    const fmm_layout *lay;
    const double *binom;          // [FMM_BN][FMM_BN] FP64
    int32_t cap;
    int swap;
    int porder;                   // per-pair orders (sorted lists sw/sp) in use
    int mutual;                   // mutual near field (at the sources, harmonic, FP64, leaves <= 64)
    int32_t *status;
    unsigned upward_blocks;       // grid cap of P2M and M2M (0: none)
};
hipError_t fmm_p2m(const fmm_eval_args &a, hipStream_t st);
hipError_t fmm_m2m(const fmm_eval_args &a, hipStream_t st);
hipError_t fmm_m2l_plan(const fmm_eval_args &a, hipStream_t st);
hipError_t fmm_m2l(const fmm_eval_args &a, hipStream_t st);
#define FMM_M2L_HEAVY 256  // weak pairs above which a box is cut into segments
#define FMM_M2L_SEG 512    // pairs per segment
hipError_t fmm_l2l(const fmm_eval_args &a, hipStream_t st);
hipError_t fmm_p2l(const fmm_eval_args &a, hipStream_t st);
hipError_t fmm_near_plan(const fmm_eval_args &a, hipStream_t st);
// part 0: the near-field kernel (part 2 then part 3: its heavy-leaf units,
// then its light leaves, as two launches); part 1: the output kernel
hipError_t fmm_p2p_l2p(const fmm_eval_args &a, double *phi, double *dphi, int part, hipStream_t st);

// learned / given per-pair orders (porder.hip)
struct fmm_porder_args {
    const double *centre, *radius, *n1, *tail;
    double *den;                  // per-box share denominators (scratch)
    double *dpart;                // heavy-segment partial denominators (scratch)
    int32_t *pbox;                // target box of every weak pair (scratch)
    const int32_t *woff, *widx;
    const float *model;           // device model or NULL
    float delta;
    const uint8_t *given;         // caller's orders or NULL
    int64_t ngiven;
    int p, L;
    int64_t nb;
    int32_t cap;
    uint8_t *qw;
    int32_t *sw;
    uint8_t *sp;
    int32_t *status;
    const int32_t *hoff, *hbox;   // M2L heavy-box segments (the sort's units)
    int64_t hmax;
};
hipError_t fmm_box_norms(const double2 *A, const double *radius, int p, int64_t nb, double *n1, double *tail,
                         hipStream_t st);
hipError_t fmm_features(const fmm_porder_args &a, int64_t nfeat_cap, float *feat, hipStream_t st);
hipError_t fmm_porder(const fmm_porder_args &a, hipStream_t st);
hipError_t fmm_labels(const fmm_porder_args &a, const double2 *A, const double *binom, const int32_t *tperm,
                      const int32_t *tstart, const double *val, double tol, int P, int kernel, int qmin, int qmax,
                      int64_t nlab_cap, double *vmin, double *budget, uint8_t *label, hipStream_t st);
int64_t fmm_mlp_grad_blocks(int64_t n);
hipError_t fmm_mlp_forward(const float *w, const float *x, int64_t n, float *y, hipStream_t st);
hipError_t fmm_mlp_grad(const float *w, const float *x, const float *q, int64_t n, float tau, float *part,
                        float *grad, float *loss, hipStream_t st);
hipError_t fmm_mlp_adam(float *w, const float *grad, float *m, float *v, int step, float lr, float b1, float b2,
                        float eps, hipStream_t st);

hipError_t fmm_direct(int64_t ns, const double *src, const double *m, int64_t nt,
                      const double *tgt, const int64_t *tsel, int64_t nsel, int kernel,
                      double *phi, double *dphi, hipStream_t st);

// device-wide exclusive scan of int32 (n entries) into out[0..n]; out[n] is
// the total; base (device, may be NULL) is added to every entry; blocksums
// holds fmm_scan_blocks(n) + 1 entries.
hipError_t fmm_scan_i32(const int32_t *in, int32_t *out, int64_t n, const int32_t *base,
                        int32_t *blocksums, hipStream_t st);
// up to FMM_SCAN_JOBS such scans of arrays of the same length, in one set of
// launches (each job with its own block sums)
#define FMM_SCAN_JOBS 4
struct fmm_scan_jobs {
    const int32_t *in[FMM_SCAN_JOBS];
    int32_t *out[FMM_SCAN_JOBS];
    const int32_t *base[FMM_SCAN_JOBS];
    int32_t *bs[FMM_SCAN_JOBS];
};
hipError_t fmm_scan_i32_jobs(const fmm_scan_jobs &J, int njobs, int64_t n, hipStream_t st);
__host__ __device__ int64_t fmm_scan_blocks(int64_t n);
