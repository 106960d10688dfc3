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
 *    it except in fmm2d_get_stats / fmm2d_sync.  fmm2d_eval without
 *    FMM2D_FLAG_TIMING also runs part of its work on a stream the handle owns
 *    (default priority), forked from and joined back into `stream` with
 *    events: when the last kernel on `stream` has finished, all of it has.
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
#define FMM2D_MIXED_FAR 2 /* the M2L contraction in FP32 (radius-scaled, as
                             above); the near field, L2P and everything else
                             in FP64 */

/* ---- truncation order policy ------------------------------------------ */
#define FMM2D_P_FIXED 0   /* one order p for every M2L interaction */
#define FMM2D_P_LEARNED 1 /* per-interaction order predicted by the loaded MLP
                             (fmm2d_set_porder_model), falling back to the
                             fixed p without a model or when p is below
                             FMM2D_PORDER_FEAT_K */
#define FMM2D_P_GIVEN 2   /* per-interaction orders supplied by the caller
                             (fmm2d_set_pair_orders) */

/* ---- flags ------------------------------------------------------------ */
#define FMM2D_FLAG_TIMING 1u        /* record per-phase device times (events); the
                                       phases then run one after another on the
                                       caller's stream, without the overlap of the
                                       far field with the lists and near field */
#define FMM2D_FLAG_REQUIRE_MODEL 2u /* learned order without a model is an error */
#define FMM2D_FLAG_LEAF_SWAP 4u     /* finest-level strong pairs that pass the theta-
                                       criterion with the radii interchanged (Sec. 2)
                                       are handled by M2P (larger target box) or P2L
                                       (larger source box) instead of P2P */
#define FMM2D_FLAG_MUTUAL 8u        /* evaluation at the sources with the harmonic kernel
                                       in FP64 and at most 64 sources per leaf: each
                                       unordered pair of near-field leaves is evaluated
                                       once for both directions (the pair symmetry of
                                       Sec. 4), with a deterministic sum of the reverse
                                       parts; ignored otherwise.  Its workspace holds
                                       list_cap / 16 (at least 4) upper leaf pairs per
                                       leaf; more is reported as FMM2D_ENOSPC */

typedef struct fmm2d_opts {
    double theta;        /* theta-criterion parameter, in (0,1); Sec. 2 uses 1/2 */
    double tol;          /* target tolerance; used only when p == 0 */
    int32_t p;           /* expansion order (highest coefficient index), 1..64;
                            0 = derive from tol by the a-priori rule
                            p = ceil(log(tol) / log(theta)) (Sec. 2) */
    int32_t levels;      /* tree depth L >= 0 (4^L leaves, 4^L <= n_src);
                            -1 = derive by eq. (Nlevels) from leaf_target */
    int32_t leaf_target; /* N_d of eq. (Nlevels), the desired sources per leaf;
                            0 = the value calibrated on MI355X for the order p
                            (45 for p <= 26, 100 for p >= 27) */
    uint32_t kernel;     /* FMM2D_KERNEL_* */
    uint32_t precision;  /* FMM2D_FP64 or FMM2D_MIXED */
    uint32_t porder;     /* FMM2D_P_FIXED or FMM2D_P_LEARNED */
    uint32_t flags;      /* FMM2D_FLAG_* */
    int32_t list_cap;    /* capacity of the interaction lists, in entries per
                            box (weak and strong each); 0 = default (256) */
} fmm2d_opts;

/* Fill `o` with the defaults: theta 1/2, tol 1e-6, p 0, levels -1,
 * leaf_target 0 (calibrated: 45, the optimum Sec. 5.1 reports, up to p = 26),
 * LOG, FP64, fixed order. */
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
 * The FP64 near field of the harmonic kernel evaluates 1/|w|^2 as
 * 1/(|w|^2 + 2^-255), four pairs per reciprocal: exact to rounding for point
 * separations above 2^-100, and it needs near-field separations (neighbouring
 * leaves) below 2^127.
 * Phi uses the principal Log in every near-field pair; in the far field it
 * follows the branch of Log(c_T - c_S) of the interacting box centres (the
 * log term of eq. (multipole)), so Phi is defined modulo 2 pi i m_j terms.
 * Errors returned by this call: FMM2D_EINVAL (n_src < 1, 4^L > n_src, theta
 * outside (0,1), p outside 1..64, NULL src/m/ws, both outputs NULL, bad enum),
 * FMM2D_ENOSPC (workspace too small); nothing is launched then.  Errors found
 * on the device and returned by the next fmm2d_sync / fmm2d_get_stats:
 * FMM2D_EINVAL if a source or target coordinate or a strength is NaN or
 * infinite (the evaluation still runs to completion and stays inside its
 * buffers; its outputs are unspecified), FMM2D_ENOSPC if the interaction lists
 * overflowed list_cap.  The handle and workspace stay usable after any of
 * these. */
int fmm2d_eval(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
               int64_t n_tgt, const double *tgt, const fmm2d_opts *opts,
               double *phi, double *dphi, void *ws, size_t ws_bytes, void *stream);

/* fmm2d_eval without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a static device array of
 * FMM2D_STATIC_WS_BYTES bytes inside the library: every device the library
 * runs on holds its own copy from the library's first use there (at
 * fmm2d_create) until the process ends.  The call allocates nothing and takes
 * the same arguments as fmm2d_eval apart from ws / ws_bytes; it returns
 * FMM2D_ENOSPC, launching nothing, when fmm2d_workspace_size(...) exceeds
 * FMM2D_STATIC_WS_BYTES (with the default options about 90,000 sources at the
 * sources, p = 20).  All calls on one device share that device's array, and
 * the topology of the last evaluation (fmm2d_get_topology) points into it:
 * calls that overlap on one device (other streams, other handles, other host
 * threads) race and must be ordered by the caller.  Every array that must
 * start at zero is cleared by the call itself. */
#define FMM2D_STATIC_WS_BYTES ((size_t)64 << 20)
int fmm2d_eval_static(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
                      int64_t n_tgt, const double *tgt, const fmm2d_opts *opts,
                      double *phi, double *dphi, void *stream);

/* Direct O(N M) summation of the same sums on the device (the near-field
 * kernel applied to all pairs, Sec. 5.3 "break-even").  tsel (device, int64,
 * optional) restricts the evaluation to targets tsel[0..n_sel); outputs are
 * then [2*n_sel].  No workspace. */
int fmm2d_direct(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
                 int64_t n_tgt, const double *tgt, const int64_t *tsel, int64_t n_sel,
                 uint32_t kernel, double *phi, double *dphi, void *stream);

/* Wait for `stream` and return the device status of the last evaluation:
 * FMM2D_OK; FMM2D_EINVAL if an input coordinate or strength was NaN or
 * infinite (or FMM2D_P_GIVEN orders were fewer than the weak pairs);
 * FMM2D_ENOSPC if its interaction lists overflowed.  The status is cleared by
 * the next fmm2d_eval. */
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
    const uint8_t *porder; /* [n_weak_total] per-pair M2L orders in weak_idx
                              order (learned or given), or NULL at fixed p */
} fmm2d_topology;
int fmm2d_get_topology(fmm2d_handle *h, fmm2d_topology *out);

/* Per-phase statistics of the last evaluation (synchronises the stream it
 * ran on).  Times are device milliseconds, recorded only with
 * FMM2D_FLAG_TIMING (else -1).  FMM2D_PH_P2P is the near-field kernel alone
 * (the P2P and M2P sums of every target: per light leaf, or per unit of a
 * heavy leaf's list); FMM2D_PH_NREDUCE adds a heavy leaf's unit sums and, for
 * every target, L2P and the output. */
enum {
    FMM2D_PH_TREE = 0, FMM2D_PH_LISTS, FMM2D_PH_P2M, FMM2D_PH_M2M,
    FMM2D_PH_PORDER, FMM2D_PH_M2L, FMM2D_PH_L2L, FMM2D_PH_P2L, FMM2D_PH_P2P, FMM2D_PH_NREDUCE, FMM2D_NPHASE
};
typedef struct fmm2d_stats {
    float ms[FMM2D_NPHASE];
    int64_t n_weak;      /* M2L pairs over all levels */
    int64_t n_strong;    /* P2P leaf pairs */
    int64_t n_m2p;       /* M2P leaf pairs */
    int64_t n_p2l;       /* P2L leaf pairs */
    int64_t n_p2p_pairs; /* point-point pair evaluations in P2P */
    int64_t n_m2p_evals; /* multipole evaluations at targets (M2P) */
    int64_t n_p2l_evals; /* source contributions to local expansions (P2L) */
    int32_t status;      /* as fmm2d_sync */
    int32_t used_model;  /* 1 if the learned order model was used */
    int64_t p_hist[65];  /* M2L pairs per order q = 0..64 (all at p when fixed) */
} fmm2d_stats;
int fmm2d_get_stats(fmm2d_handle *h, fmm2d_stats *out);

/* Per-phase device times of the last evaluation only (ms[FMM2D_NPHASE],
 * host array; -1 without FMM2D_FLAG_TIMING).  Waits for the last phase's
 * event, copies nothing else: cheap enough to call after every evaluation. */
int fmm2d_get_times(fmm2d_handle *h, float *ms);

/* ---- per-interaction truncation order ----------------------------------
 * The method uses one order p for all M2L interactions (the a-priori rule
 * p ~ log(TOL)/log(theta) of Sec. 2).  With FMM2D_P_LEARNED or FMM2D_P_GIVEN
 * each weak pair (T, S) gets its own order q in [1, p]: its M2L reads
 * a_0..a_q of S and adds to b_0..b_q of T only (eq. (multipole) and
 * eq. (local) truncated at q).  Storage, P2M, M2M, L2L and L2P stay at p.
 *
 * Learned orders come from an MLP on 8 features of the pair (schema 1):
 *   f0 rho_S/d, f1 rho_T/d, f2 (rho_S+rho_T)/d, f3 l/L,
 *   f4 log10(|ahat_S|_1 / |ahat_root|_1),
 *   f5 log10(sum_{k>K/2} |ahat_{S,k}| / |ahat_S|_1),
 *   f6 log10(|ahat_S|_1 / sum_{S' in weak(T)} |ahat_S'|_1),
 *   f7 log10(|weak(T)|),
 * where d = |c_T - c_S|, rho the box radii, l the level, ahat_k = a_k /
 * sigma^k for k = 0..K (K = FMM2D_PORDER_FEAT_K), sigma = max(rho,
 * 2^-20 rho_root), log10 arguments floored at 1e-300.
 * Model layout (FMM2D_PORDER_MODEL_FLOATS floats):
 *   [W1 32x8 row-major][b1 32][W2 32][b2 1]     trainable (FMM2D_PORDER_NPARAM)
 *   [mu 8][isd 8]                                  input standardisation
 *   [lo 8][hi 8]                                   feature range seen in training
 *   y = W2 . relu(W1 ((f - mu) * isd) + b1) + b2,
 *   q = clamp(ceil(y + delta), FMM2D_PORDER_QMIN, p); a pair with a feature
 *   outside [lo, hi] keeps q = p.  All MLP arithmetic is FP32. */
#define FMM2D_PORDER_SCHEMA 1
#define FMM2D_PORDER_NFEAT 8
#define FMM2D_PORDER_HIDDEN 32
#define FMM2D_PORDER_NPARAM 321
#define FMM2D_PORDER_MODEL_FLOATS 353
#define FMM2D_PORDER_FEAT_K 20
#define FMM2D_PORDER_QMIN 4

/* Load (copy to the device) or, with model == NULL, drop the order model.
 * model is a HOST array of n_floats == FMM2D_PORDER_MODEL_FLOATS; schema must
 * be FMM2D_PORDER_SCHEMA; delta is the calibrated offset added to y.
 * Allocates one small device buffer owned by the handle (this call is not on
 * the evaluation path).  FMM2D_EINVAL on a wrong size, schema or a non-finite
 * weight. */
int fmm2d_set_porder_model(fmm2d_handle *h, const float *model, int64_t n_floats, uint32_t schema, float delta);

/* Orders for FMM2D_P_GIVEN evaluations: orders is a DEVICE uint8 array of n
 * entries in weak_idx order (as exported by fmm2d_get_topology); values are
 * clamped to [1, p].  The caller keeps it alive while such evaluations run;
 * NULL clears it.  An evaluation with more weak pairs than n uses p for the
 * rest and fmm2d_sync reports FMM2D_EINVAL. */
int fmm2d_set_pair_orders(fmm2d_handle *h, const uint8_t *orders, int64_t n);

/* Features of every weak pair of the last evaluation (which must have used
 * p >= FMM2D_PORDER_FEAT_K), in weak_idx order: feat is a DEVICE float array
 * [n_cap][8]; pairs beyond n_cap are skipped.  Asynchronous on stream (the
 * evaluation's stream). */
int fmm2d_pair_features(fmm2d_handle *h, float *feat, int64_t n_cap, void *stream);

/* Training labels from the last evaluation, which must have used one fixed
 * order P <= 63 (a high order, e.g. 40).  For weak pair (T, S) with rho =
 * c_T - c_S, the truncation error bound at order q is
 *   e_q = sum_{l=0..P} |b_l^(q) - b_l^(P)| rho_T^l,
 * b^(q) the M2L of S truncated at q (as above), and the label is the smallest
 * q in [qmin, qmax] with e_q <= tol * min_{y in T} |val(y)| / max(|weak(T)|, 1),
 * else qmax.  val is a DEVICE array [2*n_tgt] in the caller's target order of
 * the function the expansions represent (Phi for FMM2D_KERNEL_LOG, Phi' for
 * FMM2D_KERNEL_HARMONIC), usually the output of that evaluation.  labels is a
 * DEVICE uint8 array of n_cap entries, weak_idx order.  Asynchronous.
 * FMM2D_EINVAL if the last evaluation used per-pair orders or P > 63, or
 * unless 0 <= qmin <= qmax <= P. */
int fmm2d_pair_labels(fmm2d_handle *h, const double *val, double tol, int32_t qmin, int32_t qmax,
                      uint8_t *labels, int64_t n_cap, void *stream);

/* MLP training kernels (FP32, DEVICE pointers, asynchronous on stream).
 *   forward: y[i] = MLP(x[i]) for x [n][8] raw features (the model's
 *            standardisation is applied), model as above.
 *   grad:    gradient of the pinball loss (1/n) sum_i rho_tau(q_i - y_i),
 *            rho_tau(u) = u (tau - [u < 0]), with respect to the
 *            FMM2D_PORDER_NPARAM trainable parameters -> grad [321]; the loss
 *            -> *loss (device, may be NULL).  work is a device buffer of
 *            fmm2d_mlp_work_size(n) bytes.  The sum runs in a fixed order
 *            (deterministic).
 *   adam:    one bias-corrected Adam step (step >= 1) on the trainable
 *            parameters of model, with moment buffers m, v [321] (zeroed by
 *            the caller before step 1). */
size_t fmm2d_mlp_work_size(int64_t n);
int fmm2d_mlp_forward(fmm2d_handle *h, const float *model, const float *x, int64_t n, float *y, void *stream);
int fmm2d_mlp_grad(fmm2d_handle *h, const float *model, const float *x, const float *q, int64_t n, float tau,
                   float *grad, float *loss, void *work, size_t work_bytes, void *stream);
int fmm2d_mlp_adam(fmm2d_handle *h, float *model, const float *grad, float *m, float *v, int32_t step, float lr,
                   float beta1, float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FMM2D_H */
