/*
 * fmm2d.h -- C ABI of the MI355X (gfx950) adaptive 2D fast multipole library.
 *
 * The library evaluates, for sources x_j with complex strengths m_j and
 * evaluation points y_i (Goude & Engblom, "Adaptive fast multipole methods on
 * the GPU", Sec. 1, eqs. (paireval) and (poteval)):
 *
 *     Phi (y_i) = sum_{j : x_j != y_i} m_j log(y_i - x_j)
 *     Phi'(y_i) = sum_{j : x_j != y_i} m_j / (y_i - x_j)
 *
 * with the adaptive, asymmetric (equal-count median split) FMM of Sec. 2-3:
 * tree build, theta-criterion interaction lists, P2M, M2M, M2L, L2L, L2P and
 * the near-field P2P, all as HIP kernels on one device.
 *
 * Conventions shared by every entry point
 *  - Complex arrays are interleaved FP64 pairs (re, im): a point z = x + iy is
 *    stored as {x, y}.  All data pointers are DEVICE pointers unless stated.
 *  - Every call that takes `stream` (a hipStream_t, may be NULL for the null
 *    stream) is asynchronous on that stream; the library never synchronises
 *    it except in fmm2d_get_stats / fmm2d_sync.
 *  - The library never allocates device memory on the evaluation path: the
 *    caller supplies a workspace sized by fmm2d_workspace_size.
 *  - Return value: 0 on success, a negative FMM2D_E* code otherwise; the
 *    message is available from fmm2d_last_error(handle).  On error the outputs
 *    are unspecified.  No C++ exception crosses this interface.
 *  - A handle may be used from one host thread at a time; calls that share a
 *    workspace must be ordered on one stream.
 */
#ifndef FMM2D_H
#define FMM2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define FMM2D_OK 0
#define FMM2D_EINVAL (-1)   /* invalid argument (sizes, theta, p, levels, NULL) */
#define FMM2D_ENOSPC (-2)   /* workspace too small, or interaction lists overflowed
                               the workspace's list capacity (reported by
                               fmm2d_sync / fmm2d_get_stats, since it is found on
                               the device) */
#define FMM2D_EHIP (-3)     /* a HIP runtime call failed */
#define FMM2D_ENOMODEL (-4) /* learned order requested but no model is loaded
                               (only when FMM2D_FLAG_REQUIRE_MODEL is set) */

/* ---- kernels (which potential) ---------------------------------------- */
#define FMM2D_KERNEL_LOG 1      /* Phi and Phi' (multipole carries a_0 log term) */
#define FMM2D_KERNEL_HARMONIC 2 /* Phi' only, a_0 = 0.  The harmonic potential of
                                   Sec. 5, G = Gamma_j/(z_j - z_i), equals -Phi'
                                   with m = Gamma. */

/* ---- precision -------------------------------------------------------- */
#define FMM2D_FP64 0  /* every step in FP64 */
#define FMM2D_MIXED 1 /* P2P and the M2L contraction in FP32 with compensated
                         sums and radius-scaled coefficients; geometry, theta
                         tests, the top tree levels and the final near+far sum
                         stay FP64 */

/* ---- truncation order policy ------------------------------------------ */
#define FMM2D_P_FIXED 0   /* one order p for every M2L interaction */
#define FMM2D_P_LEARNED 1 /* per-interaction order predicted by the loaded MLP,
                             falling back to the fixed p without a model */

/* ---- flags ------------------------------------------------------------ */
#define FMM2D_FLAG_TIMING 1u        /* record per-phase device times (events) */
#define FMM2D_FLAG_REQUIRE_MODEL 2u /* learned order without a model is an error */
#define FMM2D_FLAG_LEAF_SWAP 4u     /* finest-level strong pairs that pass the theta-
                                       criterion with the radii interchanged (Sec. 2)
                                       are handled by M2P (larger target box) or P2L
                                       (larger source box) instead of P2P */

typedef struct fmm2d_opts {
    double theta;        /* theta-criterion parameter, in (0,1); Sec. 2 uses 1/2 */
    double tol;          /* target tolerance; used only when p == 0 */
    int32_t p;           /* expansion order (highest coefficient index), 1..64;
                            0 = derive from tol by the a-priori rule
                            p = ceil(log(tol) / log(theta)) (Sec. 2) */
    int32_t levels;      /* tree depth L >= 0 (4^L leaves, 4^L <= n_src);
                            -1 = derive by eq. (Nlevels) from leaf_target */
    int32_t leaf_target; /* N_d of eq. (Nlevels), the desired sources per leaf */
    uint32_t kernel;     /* FMM2D_KERNEL_* */
    uint32_t precision;  /* FMM2D_FP64 or FMM2D_MIXED */
    uint32_t porder;     /* FMM2D_P_FIXED or FMM2D_P_LEARNED */
    uint32_t flags;      /* FMM2D_FLAG_* */
    int32_t list_cap;    /* capacity of the interaction lists, in entries per
                            box (weak and strong each); 0 = default (256) */
} fmm2d_opts;

/* Fill `o` with the defaults: theta 1/2, tol 1e-6, p 0, levels -1,
 * leaf_target 45 (the optimum reported in Sec. 5.1), LOG, FP64, fixed order. */
void fmm2d_default_opts(fmm2d_opts *o);

typedef struct fmm2d_handle fmm2d_handle;

/* Create a handle bound to HIP device `device` (made current for the call).
 * The handle owns a few events and a small device status block; it never owns
 * user data.  Returns FMM2D_EINVAL for a bad device, FMM2D_EHIP on HIP errors. */
int fmm2d_create(fmm2d_handle **h, int device);
void fmm2d_destroy(fmm2d_handle *h);
const char *fmm2d_last_error(const fmm2d_handle *h);

/* Levels that eq. (Nlevels) of Sec. 5.1 gives for n sources and leaf target
 * nd: ceil(0.5 log2(5 n / (8 nd))), clamped at 0 (evaluated exactly). */
int fmm2d_nlevels(int64_t n, int32_t nd);

/* Bytes of device workspace fmm2d_eval needs for n_src sources, n_tgt
 * separate evaluation points (0 = evaluate at the sources) and opts.  The
 * size depends only on these arguments, not on the data. */
int fmm2d_workspace_size(fmm2d_handle *h, int64_t n_src, int64_t n_tgt,
                         const fmm2d_opts *opts, size_t *bytes);

/* Evaluate Phi and/or Phi' (Sec. 1 eq. (poteval); eq. (paireval) when tgt is
 * NULL) by the adaptive FMM.
 *   src   [2*n_src] source positions (x, y), device, read-only, finite
 *   m     [2*n_src] complex strengths, device, read-only, finite
 *   tgt   [2*n_tgt] evaluation points, device, or NULL = at the sources (then
 *         n_tgt is ignored and a source does not act on itself)
 *   phi   [2*n_out] output Phi, or NULL (ignored for the harmonic kernel)
 *   dphi  [2*n_out] output Phi', or NULL
 *   ws    device workspace of ws_bytes >= fmm2d_workspace_size(...)
 * Pairs with coincident points (both coordinates equal) are excluded, so a
 * source never acts on itself.  Outputs are in the caller's target order.
 * Phi uses the principal Log in every near-field pair; in the far field it
 * follows the branch of Log(c_T - c_S) of the interacting box centres (the
 * log term of eq. (multipole)), so Phi is defined modulo 2 pi i m_j terms.
 * Errors: FMM2D_EINVAL (n_src < 1, 4^L > n_src, theta outside (0,1), p outside
 * 1..64, NULL src/m/ws, both outputs NULL, bad enum), FMM2D_ENOSPC (workspace
 * too small).  NaN/Inf coordinates are not checked on the device; they make
 * the outputs unspecified.  List overflow is detected on the device and
 * reported by fmm2d_sync. */
int fmm2d_eval(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
               int64_t n_tgt, const double *tgt, const fmm2d_opts *opts,
               double *phi, double *dphi, void *ws, size_t ws_bytes, void *stream);

/* Direct O(N M) summation of the same sums on the device (the near-field
 * kernel applied to all pairs, Sec. 5.3 "break-even").  tsel (device, int64,
 * optional) restricts the evaluation to targets tsel[0..n_sel); outputs are
 * then [2*n_sel].  No workspace. */
int fmm2d_direct(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
                 int64_t n_tgt, const double *tgt, const int64_t *tsel, int64_t n_sel,
                 uint32_t kernel, double *phi, double *dphi, void *stream);

/* Wait for `stream` and return the device status of the last evaluation:
 * FMM2D_OK, or FMM2D_ENOSPC if its interaction lists overflowed. */
int fmm2d_sync(fmm2d_handle *h, void *stream);

/* Device pointers into the workspace describing the tree and lists of the
 * last fmm2d_eval on this handle.  Valid until the workspace is reused.
 * Box b of level l has global index box_offset(l) + b, box_offset(l) =
 * (4^l - 1)/3; per-level start arrays have 4^l + 1 entries and are stored
 * back to back (level l at offset box_offset(l) + l). */
typedef struct fmm2d_topology {
    int32_t levels;        /* L */
    int32_t p;             /* order used */
    int64_t n_src, n_tgt;  /* n_tgt == n_src when evaluating at the sources */
    const int32_t *perm;   /* [n_src] source original index, leaf order */
    const int32_t *tperm;  /* [n_tgt] target original index, leaf order */
    const int32_t *sstart; /* per level, source segment starts */
    const int32_t *tstart; /* per level, target segment starts */
    const double *centre;  /* [nboxes][2] box centres */
    const double *radius;  /* [nboxes] box radii (half diagonals) */
    const int32_t *weak_off;   /* per level (4^l+1 entries, back to back):
                                  offsets into weak_idx (absolute) */
    const int32_t *weak_idx;   /* weak (M2L) source boxes, ascending per box,
                                  as per-level box numbers */
    const int32_t *strong_off; /* same layout for strong boxes (P2P at the finest level) */
    const int32_t *strong_idx;
    const int32_t *m2p_off;    /* finest level only (4^L + 1 entries, from 0): M2P */
    const int32_t *m2p_idx;    /*   source leaves (empty without FMM2D_FLAG_LEAF_SWAP) */
    const int32_t *p2l_off;    /* finest level only: P2L source leaves */
    const int32_t *p2l_idx;
    const double *mpole;   /* [nboxes][p+1] complex multipole coefficients */
    const double *local;   /* [nboxes][p+1] complex local coefficients */
    const uint8_t *porder; /* [n_weak_total] learned orders, or NULL */
} fmm2d_topology;
int fmm2d_get_topology(fmm2d_handle *h, fmm2d_topology *out);

/* Per-phase statistics of the last evaluation (synchronises the stream it
 * ran on).  Times are device milliseconds, recorded only with
 * FMM2D_FLAG_TIMING (else -1). */
enum {
    FMM2D_PH_TREE = 0, FMM2D_PH_LISTS, FMM2D_PH_P2M, FMM2D_PH_M2M,
    FMM2D_PH_PORDER, FMM2D_PH_M2L, FMM2D_PH_L2L, FMM2D_PH_P2L, FMM2D_PH_P2P, FMM2D_NPHASE
};
typedef struct fmm2d_stats {
    float ms[FMM2D_NPHASE];
    int64_t n_weak;      /* M2L pairs over all levels */
    int64_t n_strong;    /* P2P leaf pairs */
    int64_t n_m2p;       /* M2P leaf pairs */
    int64_t n_p2l;       /* P2L leaf pairs */
    int64_t n_p2p_pairs; /* point-point pair evaluations in P2P */
    int32_t status;      /* as fmm2d_sync */
    int32_t used_model;  /* 1 if the learned order was used */
    int64_t p_hist[65];  /* learned order histogram (p = 0..64) */
} fmm2d_stats;
int fmm2d_get_stats(fmm2d_handle *h, fmm2d_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* FMM2D_H */
