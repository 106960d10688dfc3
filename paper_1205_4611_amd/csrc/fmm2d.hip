// Host side of the C ABI (include/fmm2d.h): argument checks, workspace
// layout, and the order of the device phases of one evaluation.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "common.h"

// Workspace of fmm2d_eval_static: a static device array, one copy on every
// device the library runs on, held until the process ends.  Host code never
// uses the array's name as an address: each device's copy is looked up once
// (hipGetSymbolAddress, in fmm2d_create with that device current) and kept in
// g_scratch_ptr.
static __device__ __align__(256) char scratch[FMM2D_STATIC_WS_BYTES];
#define FMM_MAX_DEVICES 64
static void *g_scratch_ptr[FMM_MAX_DEVICES];
static std::mutex g_scratch_mu;

struct fmm2d_handle {
    int device;
    void *scratch;          // this device's copy of `scratch` (device address)
    char err[512];
    int32_t *d_status;      // device status word
    double *d_binom;        // [FMM_BN][FMM_BN]
    hipEvent_t ev[FMM2D_NPHASE + 1];
    // side stream and its fork / join events: y presort (0, 1), tree done (2),
    // M2L done (3), lists and plans done (4), far field done (5), leaf
    // multipoles done (6)
    hipStream_t side;
    hipEvent_t sev[7];
    int n_cu;               // compute units of the device
    int timing_valid;
    hipStream_t last_stream;
    // learned order model (device copy, owned) and caller-given orders (not owned)
    float *d_model;
    float delta;
    const uint8_t *given;
    int64_t ngiven;
    // last evaluation
    int have_topo;
    fmm_layout lay;
    const char *ws;
    int64_t ns, nt;
    int L, p, kernel, at_sources, used_orders, used_model;
};

static int fail(fmm2d_handle *h, int code, const char *fmt, ...)
{
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->err, sizeof(h->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(h, x)                                                                          \
    do {                                                                                      \
        hipError_t e__ = (x);                                                                 \
        if (e__ != hipSuccess)                                                                \
            return fail((h), FMM2D_EHIP, "%s: %s (%s:%d)", #x, hipGetErrorString(e__), __FILE__, \
                        __LINE__);                                                            \
    } while (0)

extern "C" void fmm2d_default_opts(fmm2d_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->theta = 0.5;
    o->tol = 1e-6;
    o->p = 0;
    o->levels = -1;
    o->leaf_target = 0;
    o->kernel = FMM2D_KERNEL_LOG;
    o->precision = FMM2D_FP64;
    o->porder = FMM2D_P_FIXED;
    o->flags = 0;
    o->list_cap = 0;
}

// eq. (Nlevels): the smallest L >= 0 with 8 nd 4^L >= 5 n (exact integers).
extern "C" int fmm2d_nlevels(int64_t n, int32_t nd)
{
    if (n <= 0 || nd <= 0) return -1;
    int L = 0;
    __int128 lhs = (__int128)8 * nd;
    while (lhs < (__int128)5 * n) {
        lhs *= 4;
        ++L;
    }
    return L;
}

// The leaf target N_d that eq. (Nlevels) uses when fmm2d_opts.leaf_target is
// 0: the calibration of Sec. 5.1 repeated on MI355X (FP64, harmonic kernel,
// 20-cluster sources at the sources, N from 2^20 to 2^24, fixed and learned
// orders): the fastest depth lies in N_d in [40, 79] up to p = 20 and in
// [80, 159] from p = 27 on (at p = 24 the two depths are within 2%), as the
// paper finds the optimum growing with p (Sec. 5.2); 45 is also the paper's
// optimum for its GPU.
static int32_t calibrated_nd(int p) { return p >= 27 ? 100 : 45; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The mutual near field applies (evaluation at the sources, harmonic, FP64,
// at most 64 sources per leaf; equal-count splits make every leaf hold at
// most ceil(ns / 4^L)).
static int use_mutual(const fmm2d_opts *o, int64_t nt, int64_t ns, int L)
{
    return (o->flags & FMM2D_FLAG_MUTUAL) && nt == 0 && o->kernel == FMM2D_KERNEL_HARMONIC &&
           o->precision == FMM2D_FP64 && (ns + nbox(L) - 1) / nbox(L) <= 64;
}

int fmm_plan_layout(int64_t ns, int64_t nt, int L, int p, int cap, int mixed, int learned,
                    fmm_layout *lay, int mutual)
{
    memset(lay, 0, sizeof(*lay));
    lay->ns = ns; lay->nt = nt; lay->L = L; lay->p = p; lay->cap = cap;
    lay->mixed = mixed; lay->learned = learned;
    lay->nb = box_off(L + 1);
    lay->nleaf = nbox(L);
    lay->nstart = start_off(L + 1);
    lay->nstep = (((int64_t)1) << (2 * L + 1)) + 2 * L + 2;
    lay->listcap = (int64_t)cap * lay->nb + 4;
    const int64_t nmax = ns > nt ? ns : nt;
    const int64_t P1 = p + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + (bytes ? bytes : 1)); return r; };
    const int64_t rs_blocks = (nmax + 4095) / 4096;
    const int64_t hist_n = 256 * rs_blocks + 256 * 8 + 1; // histograms and per-pass digit totals
    const int64_t seg_scan_n = fmm_scan_blocks(lay->nleaf + 1) + 1;
    lay->keys[0] = take(8 * nmax);
    lay->keys[1] = take(8 * nmax);
    lay->vals[0] = take(4 * nmax);
    lay->vals[1] = take(4 * nmax);
    lay->hist = take(4 * (hist_n > 3 * seg_scan_n ? hist_n : 3 * seg_scan_n)); // also 3 block-sum arrays
    lay->hist2 = take(4 * hist_n);
    {
        int64_t a = fmm_scan_blocks(hist_n) + 1;
        int64_t b = 4 * (fmm_scan_blocks(nmax) + 1);
        lay->bsum = take(4 * (a > b ? a : b));
    }
    lay->srec = take(8 * 4 * ns);
    lay->sbits = take(4 * (lay->nleaf + 1));
    lay->stseg = take(4 * ((ns + FMM_LB_TILE - 1) / FMM_LB_TILE + 1));
    lay->stcnt = take(4 * 2 * ((ns + FMM_LB_TILE - 1) / FMM_LB_TILE + 1));
    lay->trec = take(24 * 4 * nt);
    lay->srank = take(4 * 4 * ns);
    lay->scoord = take(8 * 2 * ns);
    lay->lbtiles = (nmax + FMM_LB_TILE - 1) / FMM_LB_TILE;
    lay->lbst = take(8 * (4 * lay->lbtiles + 2));
    lay->perm = take(4 * ns);
    lay->tperm = take(4 * nt);
    lay->sstep = take(4 * lay->nstep);
    lay->tstep = take(4 * lay->nstep);
    lay->seg_axis = take(lay->nleaf + 1);
    lay->seg_pc = take(8 * (lay->nleaf + 1));
    lay->seg_pi = take(4 * (lay->nleaf + 1));
    lay->seg_nlo = take(4 * (lay->nleaf + 1));
    lay->seg_tlo = take(4 * (lay->nleaf + 1));
    lay->seg_LO = take(4 * (lay->nleaf + 2));
    lay->seg_TLO = take(4 * (lay->nleaf + 2));
    lay->seg_nlox = take(4 * (lay->nleaf + 1));
    lay->seg_nloy = take(4 * (lay->nleaf + 1));
    lay->seg_LOy = take(4 * (lay->nleaf + 2));
    lay->sstart = take(4 * lay->nstart);
    lay->tstart = take(4 * lay->nstart);
    lay->centre = take(16 * lay->nb);
    lay->radius = take(8 * lay->nb);
    lay->wcnt = take(4 * lay->nleaf);
    lay->scnt = take(4 * lay->nleaf);
    lay->woff = take(4 * lay->nstart);
    lay->soff = take(4 * lay->nstart);
    lay->widx = take(4 * lay->listcap);
    lay->sidx = take(4 * lay->listcap);
    lay->leafcap = (int64_t)cap * lay->nleaf + 4;
    lay->mcnt = take(4 * lay->nleaf);
    lay->pcnt = take(4 * lay->nleaf);
    lay->moff = take(4 * (lay->nleaf + 1));
    lay->poff = take(4 * (lay->nleaf + 1));
    lay->midx = take(4 * lay->leafcap);
    lay->pidx = take(4 * lay->leafcap);
    lay->lbsum = take(4 * FMM_SCAN_JOBS * (fmm_scan_blocks(lay->nleaf) + 2));
    lay->lhvy = take(4 * lay->nb);
    lay->lhcnt = take(4 * (L + 2));
    lay->lhpart = take(4 * 4 * 16 * lay->nleaf); // heavy boxes of a level <= 4^L, 16 parts, 4 counts
    lay->srcs = take(32 * ns);
    lay->tgts = take(16 * nt);
    lay->m32 = mixed == 1 ? take(8 * ns) : 0;
    lay->A = take(16 * lay->nb * P1);
    lay->B = take(16 * lay->nb * P1);
    lay->A32 = mixed ? take(8 * lay->nb * P1) : 0;
    lay->n1 = take(8 * lay->nb);
    lay->tail = take(8 * lay->nb);
    lay->vmin = take(8 * lay->nb);
    lay->budget = take(8 * lay->nb);
    // heavy-box segments: ceil(cnt / 512) <= cnt / 512 + 1 per box of more
    // than 256 pairs, so at most listcap / 512 + listcap / 256 + 1 in total
    lay->hmax = lay->listcap / 512 + lay->listcap / 256 + 1;
    lay->hs = take(4 * (lay->nb + 1));
    lay->hoff = take(4 * (lay->nb + 2));
    lay->hbox = take(4 * lay->hmax);
    lay->hpart = take(16 * lay->hmax * P1);
    // near-field units of heavy leaves: about one per leaf (heavy leaves past
    // the capacity are evaluated whole)
    lay->nucap = lay->nleaf + 1024;
    lay->nhw = take(4 * (lay->nleaf + 1));
    lay->nhoff = take(4 * (lay->nleaf + 2));
    lay->nuleaf = take(4 * lay->nucap);
    lay->npart = take(8 * 4 * 64 * lay->nucap);
    lay->nsum = take(32 * (nt ? nt : ns));
    lay->mut_rcap = mutual ? lay->nleaf * (cap / 16 > 4 ? cap / 16 : 4) : 0;
    lay->mut_ucnt = mutual ? take(4 * lay->nleaf) : 0;
    lay->mut_uoff = mutual ? take(4 * (lay->nleaf + 1)) : 0;
    lay->mut_rev = mutual ? take(16 * 64 * (size_t)lay->mut_rcap) : 0;
    lay->qw = learned ? take(lay->listcap) : 0;
    lay->sw = learned ? take(4 * lay->listcap) : 0;
    lay->pbox = learned ? take(4 * lay->listcap) : 0;
    lay->sp = learned ? take(lay->listcap) : 0;
    lay->total = o;
    return 0;
}

extern "C" int fmm2d_create(fmm2d_handle **out, int device)
{
    if (!out) return FMM2D_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FMM2D_EINVAL;
    fmm2d_handle *h = (fmm2d_handle *)calloc(1, sizeof(fmm2d_handle));
    if (!h) return FMM2D_EINVAL;
    h->device = device;
    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_status, 64);
    if (e == hipSuccess) e = hipMemset(h->d_status, 0, 64);
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_binom, sizeof(double) * FMM_BN * FMM_BN);
    if (e == hipSuccess) {
        // Pascal's rule in FP64 (exact below 2^53)
        double *t = (double *)calloc(FMM_BN * FMM_BN, sizeof(double));
        for (int n = 0; n < FMM_BN; ++n) {
            t[n * FMM_BN] = 1.0;
            for (int k = 1; k <= n; ++k)
                t[n * FMM_BN + k] = t[(n - 1) * FMM_BN + k - 1] + (k < n ? t[(n - 1) * FMM_BN + k] : 0.0);
        }
        e = hipMemcpy(h->d_binom, t, sizeof(double) * FMM_BN * FMM_BN, hipMemcpyHostToDevice);
        free(t);
    }
    if (e == hipSuccess && device < FMM_MAX_DEVICES) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e == hipSuccess) g_scratch_ptr[device] = ptr;
        }
        h->scratch = g_scratch_ptr[device];
    }
    for (int i = 0; i <= FMM2D_NPHASE && e == hipSuccess; ++i) e = hipEventCreate(&h->ev[i]);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, device);
    for (int i = 0; i < 7 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&h->sev[i], hipEventDisableTiming);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        fmm2d_destroy(h);
        return FMM2D_EHIP;
    }
    *out = h;
    return FMM2D_OK;
}

extern "C" void fmm2d_destroy(fmm2d_handle *h)
{
    if (!h) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(h->device);
    for (int i = 0; i <= FMM2D_NPHASE; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    for (int i = 0; i < 7; ++i)
        if (h->sev[i]) (void)hipEventDestroy(h->sev[i]);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->d_status) (void)hipFree(h->d_status);
    if (h->d_binom) (void)hipFree(h->d_binom);
    if (h->d_model) (void)hipFree(h->d_model);
    (void)hipSetDevice(prev);
    free(h);
}

extern "C" const char *fmm2d_last_error(const fmm2d_handle *h) { return h ? h->err : "null handle"; }

// Resolve levels and order from opts; returns 0 or an error code.
static int resolve(fmm2d_handle *h, int64_t ns, const fmm2d_opts *o, int *L, int *p, int *cap)
{
    if (!o) return fail(h, FMM2D_EINVAL, "opts is NULL");
    if (ns < 1 || ns > ((int64_t)1 << 30)) return fail(h, FMM2D_EINVAL, "n_src must be in [1, 2^30]");
    if (!(o->theta > 0.0 && o->theta < 1.0)) return fail(h, FMM2D_EINVAL, "theta must be in (0,1)");
    if (o->kernel != FMM2D_KERNEL_LOG && o->kernel != FMM2D_KERNEL_HARMONIC)
        return fail(h, FMM2D_EINVAL, "unknown kernel %u", o->kernel);
    if (o->precision != FMM2D_FP64 && o->precision != FMM2D_MIXED && o->precision != FMM2D_MIXED_FAR)
        return fail(h, FMM2D_EINVAL, "unknown precision %u", o->precision);
    if (o->porder != FMM2D_P_FIXED && o->porder != FMM2D_P_LEARNED && o->porder != FMM2D_P_GIVEN)
        return fail(h, FMM2D_EINVAL, "unknown order policy %u", o->porder);
    int pp = o->p;
    if (pp == 0) {
        if (!(o->tol > 0.0 && o->tol < 1.0)) return fail(h, FMM2D_EINVAL, "tol must be in (0,1)");
        pp = (int)ceil(log(o->tol) / log(o->theta));
    }
    if (pp < 1 || pp > FMM_PMAX) return fail(h, FMM2D_EINVAL, "p=%d outside 1..%d", pp, FMM_PMAX);
    int LL = o->levels;
    if (LL < 0) {
        if (o->leaf_target < 0) return fail(h, FMM2D_EINVAL, "leaf_target must be >= 0");
        LL = fmm2d_nlevels(ns, o->leaf_target > 0 ? o->leaf_target : calibrated_nd(pp));
    }
    if (LL > FMM_MAXL) return fail(h, FMM2D_EINVAL, "levels=%d > %d", LL, FMM_MAXL);
    if (nbox(LL) > ns) return fail(h, FMM2D_EINVAL, "4^L = %lld exceeds n_src = %lld", (long long)nbox(LL), (long long)ns);
    int c = o->list_cap > 0 ? o->list_cap : FMM_DEFAULT_LIST_CAP;
    *L = LL;
    *p = pp;
    *cap = c;
    return 0;
}

extern "C" int fmm2d_workspace_size(fmm2d_handle *h, int64_t n_src, int64_t n_tgt, const fmm2d_opts *opts,
                                    size_t *bytes)
{
    if (!h || !bytes) return fail(h, FMM2D_EINVAL, "NULL argument");
    int L, p, cap;
    int rc = resolve(h, n_src, opts, &L, &p, &cap);
    if (rc) return rc;
    if (n_tgt < 0 || n_tgt > ((int64_t)1 << 30)) return fail(h, FMM2D_EINVAL, "n_tgt out of range");
    fmm_layout lay;
    fmm_plan_layout(n_src, n_tgt, L, p, cap, (int)opts->precision, opts->porder != FMM2D_P_FIXED, &lay,
                    use_mutual(opts, n_tgt, n_src, L));
    *bytes = lay.total;
    return FMM2D_OK;
}

__global__ void k_zero_status(int32_t *s) { s[threadIdx.x] = 0; }

static fmm_porder_args porder_args(fmm2d_handle *h, char *w, const fmm_layout &lay, int L, int p, int cap)
{
    fmm_porder_args a;
    memset(&a, 0, sizeof(a));
    a.centre = reinterpret_cast<const double *>(w + lay.centre);
    a.radius = reinterpret_cast<const double *>(w + lay.radius);
    a.n1 = reinterpret_cast<const double *>(w + lay.n1);
    a.tail = reinterpret_cast<const double *>(w + lay.tail);
    a.den = reinterpret_cast<double *>(w + lay.budget); // free outside the label computation
    a.dpart = reinterpret_cast<double *>(w + lay.hpart);  // M2L partials are written later
    a.pbox = lay.sw ? reinterpret_cast<int32_t *>(w + lay.pbox) : nullptr;
    a.woff = reinterpret_cast<const int32_t *>(w + lay.woff);
    a.widx = reinterpret_cast<const int32_t *>(w + lay.widx);
    a.p = p;
    a.L = L;
    a.nb = lay.nb;
    a.cap = (int32_t)lay.listcap;
    (void)cap;
    a.qw = lay.qw ? reinterpret_cast<uint8_t *>(w + lay.qw) : nullptr;
    a.sw = lay.sw ? reinterpret_cast<int32_t *>(w + lay.sw) : nullptr;
    a.sp = lay.sp ? reinterpret_cast<uint8_t *>(w + lay.sp) : nullptr;
    a.status = h->d_status;
    a.hoff = reinterpret_cast<const int32_t *>(w + lay.hoff);
    a.hbox = reinterpret_cast<const int32_t *>(w + lay.hbox);
    a.hmax = lay.hmax;
    return a;
}

extern "C" int fmm2d_eval(fmm2d_handle *h, int64_t n_src, const double *src, const double *m, int64_t n_tgt,
                          const double *tgt, const fmm2d_opts *opts, double *phi, double *dphi, void *ws,
                          size_t ws_bytes, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    h->err[0] = 0;
    int L, p, cap;
    int rc = resolve(h, n_src, opts, &L, &p, &cap);
    if (rc) return rc;
    if (!src || !m || !ws) return fail(h, FMM2D_EINVAL, "src, m and ws must be non-NULL");
    const bool LOG = opts->kernel == FMM2D_KERNEL_LOG;
    if (!dphi && !(LOG && phi)) return fail(h, FMM2D_EINVAL, "no output requested");
    const int64_t nt = tgt ? n_tgt : 0;
    if (tgt && (n_tgt < 1 || n_tgt > ((int64_t)1 << 30))) return fail(h, FMM2D_EINVAL, "n_tgt out of range");
    const int mixed = (int)opts->precision;
    const int learned = opts->porder != FMM2D_P_FIXED;
    // per-pair orders: the model needs the features' coefficients (k <= FEAT_K)
    const bool use_model = opts->porder == FMM2D_P_LEARNED && h->d_model && p >= FMM2D_PORDER_FEAT_K;
    const bool use_given = opts->porder == FMM2D_P_GIVEN;
    if (opts->porder == FMM2D_P_LEARNED && !use_model && (opts->flags & FMM2D_FLAG_REQUIRE_MODEL))
        return fail(h, FMM2D_ENOMODEL, h->d_model ? "learned order needs p >= %d" : "no order model is loaded",
                    FMM2D_PORDER_FEAT_K);
    if (use_given && !h->given) return fail(h, FMM2D_EINVAL, "FMM2D_P_GIVEN without fmm2d_set_pair_orders");
    fmm_layout lay;
    const int mutual = use_mutual(opts, nt, n_src, L);
    fmm_plan_layout(n_src, nt, L, p, cap, mixed, learned, &lay, mutual);
    if (ws_bytes < lay.total)
        return fail(h, FMM2D_ENOSPC, "workspace of %zu bytes < %zu needed", ws_bytes, lay.total);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(h, hipSetDevice(h->device));
    const bool timing = (opts->flags & FMM2D_FLAG_TIMING) != 0;
    // Without timing the far field (P2M ... P2L) and the y presort run on the
    // handle's side stream, beside the lists and the near field; the output
    // kernel waits for both.  With timing every phase runs in order on st, so
    // that the events between them measure one phase each.
    const bool fork = !timing;
    hipStream_t sb = fork ? h->side : st;
    k_zero_status<<<1, 16, 0, st>>>(h->d_status);
    if (timing) HIPCHK(h, hipEventRecord(h->ev[0], st));

    char *w = (char *)ws;
    fmm_tree_args ta;
    ta.ns = n_src; ta.nt = nt; ta.L = L; ta.theta = opts->theta;
    ta.src = src; ta.tgt = tgt; ta.ws = w; ta.lay = &lay; ta.status = h->d_status; ta.cap = cap;
    ta.swap = (opts->flags & FMM2D_FLAG_LEAF_SWAP) != 0;
    ta.side = fork ? h->side : nullptr;
    ta.ev_fork = h->sev[0];
    ta.ev_join = h->sev[1];
    HIPCHK(h, fmm_build_tree(ta, m, st));
    if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_TREE], st));

    fmm_eval_args ea;
    ea.L = L; ea.p = p; ea.kernel = (int)opts->kernel; ea.mixed = mixed;
    ea.ns = n_src; ea.nt = nt ? nt : n_src; ea.at_sources = nt == 0;
    ea.ws = w; ea.lay = &lay; ea.binom = h->d_binom; ea.cap = cap; ea.swap = ta.swap;
    ea.porder = use_model || use_given;
    ea.mutual = mutual;
    ea.status = h->d_status;
    // Beside the lists, P2M and M2M run on at most 4 workgroups per CU (grid-
    // stride loops), so that the lists' single-workgroup kernels find room on
    // the CUs instead of waiting for the upward pass to drain; the upward pass
    // still ends long before M2L needs it.
    ea.upward_blocks = fork ? 4u * (unsigned)h->n_cu : 0u;
    fmm_porder_args pa = porder_args(h, w, lay, L, p, cap);
    if (use_model) {
        pa.model = h->d_model;
        pa.delta = h->delta;
    } else {
        pa.given = h->given;
        pa.ngiven = h->ngiven;
    }
    // the multipoles, upward pass and coefficient norms need the tree only
    auto upward = [&]() -> int {
        HIPCHK(h, fmm_p2m(ea, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_P2M], sb));
        if (fork) HIPCHK(h, hipEventRecord(h->sev[6], sb));
        HIPCHK(h, fmm_m2m(ea, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_M2M], sb));
        if (use_model)
            HIPCHK(h, fmm_box_norms(reinterpret_cast<const double2 *>(w + lay.A), pa.radius, p, lay.nb,
                                    reinterpret_cast<double *>(w + lay.n1), reinterpret_cast<double *>(w + lay.tail),
                                    sb));
        return 0;
    };
    // orders, M2L, downward pass and P2L need the lists too
    auto downward = [&]() -> int {
        if (ea.porder) HIPCHK(h, fmm_porder(pa, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_PORDER], sb));
        HIPCHK(h, fmm_m2l(ea, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_M2L], sb));
        if (fork) HIPCHK(h, hipEventRecord(h->sev[3], sb));
        HIPCHK(h, fmm_l2l(ea, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_L2L], sb));
        HIPCHK(h, fmm_p2l(ea, sb));
        if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_P2L], sb));
        return 0;
    };
    int rc2 = 0;
    if (fork) {
        HIPCHK(h, hipEventRecord(h->sev[2], st));
        HIPCHK(h, hipStreamWaitEvent(sb, h->sev[2], 0));
        if ((rc2 = upward())) return rc2;
    }
    HIPCHK(h, fmm_build_lists(ta, st));
    if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_LISTS], st));
    HIPCHK(h, fmm_m2l_plan(ea, st));
    HIPCHK(h, fmm_near_plan(ea, st));
    if (fork) {
        HIPCHK(h, hipEventRecord(h->sev[4], st));
        HIPCHK(h, hipStreamWaitEvent(sb, h->sev[4], 0));
        if ((rc2 = downward())) return rc2;
        HIPCHK(h, hipEventRecord(h->sev[5], sb));
        // The near field needs only the lists and the leaf multipoles (M2P).
        // Its heavy-leaf units run beside the order phase; its light leaves
        // wait for M2L: M2L waves hold 168 VGPRs and find little room once
        // the near kernel's 49-VGPR waves fill the CUs, so side by side M2L
        // ran past the end of the near kernel; alone it runs at full rate,
        // and L2L and P2L run beside the light leaves.
        HIPCHK(h, hipStreamWaitEvent(st, h->sev[6], 0));
        HIPCHK(h, fmm_p2p_l2p(ea, LOG ? phi : nullptr, dphi, 2, st));
        HIPCHK(h, hipStreamWaitEvent(st, h->sev[3], 0));
        HIPCHK(h, fmm_p2p_l2p(ea, LOG ? phi : nullptr, dphi, 3, st));
    } else {
        if ((rc2 = upward())) return rc2;
        if ((rc2 = downward())) return rc2;
        HIPCHK(h, fmm_p2p_l2p(ea, LOG ? phi : nullptr, dphi, 0, st));
    }
    if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_P2P], st));
    if (fork) HIPCHK(h, hipStreamWaitEvent(st, h->sev[5], 0)); // L2P reads the local expansions
    HIPCHK(h, fmm_p2p_l2p(ea, LOG ? phi : nullptr, dphi, 1, st));
    if (timing) HIPCHK(h, hipEventRecord(h->ev[1 + FMM2D_PH_NREDUCE], st));

    h->timing_valid = timing;
    h->last_stream = st;
    h->have_topo = 1;
    h->lay = lay;
    h->ws = w;
    h->ns = n_src;
    h->nt = nt;
    h->L = L;
    h->p = p;
    h->kernel = (int)opts->kernel;
    h->at_sources = nt == 0;
    h->used_orders = ea.porder;
    h->used_model = use_model;
    return FMM2D_OK;
}

extern "C" int fmm2d_eval_static(fmm2d_handle *h, int64_t n_src, const double *src, const double *m,
                                 int64_t n_tgt, const double *tgt, const fmm2d_opts *opts, double *phi,
                                 double *dphi, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    h->err[0] = 0;
    if (!h->scratch)
        return fail(h, FMM2D_EINVAL, "no static workspace on device %d (devices 0..%d only)", h->device,
                    FMM_MAX_DEVICES - 1);
    size_t need = 0;
    int rc = fmm2d_workspace_size(h, n_src, tgt ? n_tgt : 0, opts, &need);
    if (rc) return rc;
    if (need > (size_t)FMM2D_STATIC_WS_BYTES)
        return fail(h, FMM2D_ENOSPC,
                    "fmm2d_eval_static: this problem needs %zu bytes of workspace, more than the %zu of the "
                    "static workspace; use fmm2d_eval with a caller workspace",
                    need, (size_t)FMM2D_STATIC_WS_BYTES);
    return fmm2d_eval(h, n_src, src, m, n_tgt, tgt, opts, phi, dphi, h->scratch, (size_t)FMM2D_STATIC_WS_BYTES,
                      stream);
}

extern "C" int fmm2d_direct(fmm2d_handle *h, int64_t n_src, const double *src, const double *m, int64_t n_tgt,
                            const double *tgt, const int64_t *tsel, int64_t n_sel, uint32_t kernel, double *phi,
                            double *dphi, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (n_src < 1 || !src || !m) return fail(h, FMM2D_EINVAL, "bad sources");
    if (kernel != FMM2D_KERNEL_LOG && kernel != FMM2D_KERNEL_HARMONIC) return fail(h, FMM2D_EINVAL, "bad kernel");
    if (!tgt) { tgt = src; n_tgt = n_src; }
    if (n_tgt < 1) return fail(h, FMM2D_EINVAL, "bad n_tgt");
    if (tsel && n_sel < 0) return fail(h, FMM2D_EINVAL, "bad n_sel");
    if (!dphi && !(kernel == FMM2D_KERNEL_LOG && phi)) return fail(h, FMM2D_EINVAL, "no output requested");
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, fmm_direct(n_src, src, m, n_tgt, tgt, tsel, n_sel, (int)kernel, phi, dphi, (hipStream_t)stream));
    return FMM2D_OK;
}

extern "C" int fmm2d_sync(fmm2d_handle *h, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, hipStreamSynchronize((hipStream_t)stream));
    int32_t s = 0;
    HIPCHK(h, hipMemcpy(&s, h->d_status, sizeof(s), hipMemcpyDeviceToHost));
    if (s & FMM_ST_NONFINITE)
        return fail(h, FMM2D_EINVAL, "a source or target coordinate or a strength is NaN or infinite");
    if (s & FMM_ST_LIST_OVERFLOW)
        return fail(h, FMM2D_ENOSPC, "interaction lists overflowed list_cap; raise fmm2d_opts.list_cap");
    if (s & FMM_ST_ORDERS_SHORT)
        return fail(h, FMM2D_EINVAL, "the pair orders given are fewer than the weak pairs");
    if (s & FMM_ST_TREE_INCONSISTENT)
        return fail(h, FMM2D_EHIP, "internal error: inconsistent point lists in the tree build");
    return FMM2D_OK;
}

extern "C" int fmm2d_get_topology(fmm2d_handle *h, fmm2d_topology *t)
{
    if (!h || !t) return FMM2D_EINVAL;
    if (!h->have_topo) return fail(h, FMM2D_EINVAL, "no evaluation yet");
    const fmm_layout &lay = h->lay;
    const char *w = h->ws;
    memset(t, 0, sizeof(*t));
    t->levels = h->L;
    t->p = h->p;
    t->n_src = h->ns;
    t->n_tgt = h->at_sources ? h->ns : h->nt;
    t->perm = reinterpret_cast<const int32_t *>(w + lay.perm);
    t->tperm = h->at_sources ? t->perm : reinterpret_cast<const int32_t *>(w + lay.tperm);
    t->sstart = reinterpret_cast<const int32_t *>(w + lay.sstart);
    t->tstart = h->at_sources ? t->sstart : reinterpret_cast<const int32_t *>(w + lay.tstart);
    t->centre = reinterpret_cast<const double *>(w + lay.centre);
    t->radius = reinterpret_cast<const double *>(w + lay.radius);
    t->weak_off = reinterpret_cast<const int32_t *>(w + lay.woff);
    t->weak_idx = reinterpret_cast<const int32_t *>(w + lay.widx);
    t->strong_off = reinterpret_cast<const int32_t *>(w + lay.soff);
    t->strong_idx = reinterpret_cast<const int32_t *>(w + lay.sidx);
    t->m2p_off = reinterpret_cast<const int32_t *>(w + lay.moff);
    t->m2p_idx = reinterpret_cast<const int32_t *>(w + lay.midx);
    t->p2l_off = reinterpret_cast<const int32_t *>(w + lay.poff);
    t->p2l_idx = reinterpret_cast<const int32_t *>(w + lay.pidx);
    t->mpole = reinterpret_cast<const double *>(w + lay.A);
    t->local = reinterpret_cast<const double *>(w + lay.B);
    t->porder = h->used_orders ? reinterpret_cast<const uint8_t *>(w + lay.qw) : nullptr;
    return FMM2D_OK;
}

extern "C" int fmm2d_get_stats(fmm2d_handle *h, fmm2d_stats *s)
{
    if (!h || !s) return FMM2D_EINVAL;
    memset(s, 0, sizeof(*s));
    for (int i = 0; i < FMM2D_NPHASE; ++i) s->ms[i] = -1.0f;
    if (!h->have_topo) return fail(h, FMM2D_EINVAL, "no evaluation yet");
    s->status = fmm2d_sync(h, h->last_stream);
    if (h->timing_valid) {
        for (int i = 0; i < FMM2D_NPHASE; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) s->ms[i] = ms;
        }
    }
    const fmm_layout &lay = h->lay;
    const int L = h->L;
    // list totals and the P2P pair count, from the device lists
    int32_t wend = 0, send_prev = 0, send = 0;
    const int32_t *woff = reinterpret_cast<const int32_t *>(h->ws + lay.woff);
    const int32_t *soff = reinterpret_cast<const int32_t *>(h->ws + lay.soff);
    HIPCHK(h, hipMemcpy(&wend, woff + start_off(L) + nbox(L), 4, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(&send, soff + start_off(L) + nbox(L), 4, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(&send_prev, soff + start_off(L), 4, hipMemcpyDeviceToHost));
    s->n_weak = wend;
    s->n_strong = (int64_t)send - send_prev;
    {
        int32_t mend = 0, pend = 0;
        HIPCHK(h, hipMemcpy(&mend, reinterpret_cast<const int32_t *>(h->ws + lay.moff) + nbox(L), 4,
                            hipMemcpyDeviceToHost));
        HIPCHK(h, hipMemcpy(&pend, reinterpret_cast<const int32_t *>(h->ws + lay.poff) + nbox(L), 4,
                            hipMemcpyDeviceToHost));
        s->n_m2p = mend;
        s->n_p2l = pend;
    }
    if (s->status == FMM2D_OK) {
        const int64_t nl = nbox(L);
        int32_t *so = (int32_t *)malloc(4 * (nl + 1));
        int32_t *ss = (int32_t *)malloc(4 * (nl + 1));
        int32_t *ts = (int32_t *)malloc(4 * (nl + 1));
        int32_t *si = (int32_t *)malloc(4 * (s->n_strong + 1));
        const char *w = h->ws;
        hipError_t e = hipMemcpy(so, soff + start_off(L), 4 * (nl + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(ss, reinterpret_cast<const int32_t *>(w + lay.sstart) + start_off(L), 4 * (nl + 1),
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(ts,
                          reinterpret_cast<const int32_t *>(w + (h->at_sources ? lay.sstart : lay.tstart)) + start_off(L),
                          4 * (nl + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess && s->n_strong > 0)
            e = hipMemcpy(si, reinterpret_cast<const int32_t *>(w + lay.sidx) + send_prev, 4 * s->n_strong,
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            int64_t pairs = 0;
            for (int64_t t = 0; t < nl; ++t) {
                int64_t nsrc = 0;
                for (int32_t k = so[t]; k < so[t + 1]; ++k) {
                    int32_t b = si[k - send_prev];
                    nsrc += ss[b + 1] - ss[b];
                }
                pairs += nsrc * (ts[t + 1] - ts[t]);
            }
            s->n_p2p_pairs = pairs;
        }
        // M2P evaluations (targets x source leaves) and P2L contributions
        // (sources of the P2L leaves, per target leaf)
        int32_t *mo = (int32_t *)malloc(4 * (nl + 1));
        int32_t *po = (int32_t *)malloc(4 * (nl + 1));
        int32_t *pi = (int32_t *)malloc(4 * (s->n_p2l + 1));
        if (e == hipSuccess) e = hipMemcpy(mo, w + lay.moff, 4 * (nl + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(po, w + lay.poff, 4 * (nl + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess && s->n_p2l > 0) e = hipMemcpy(pi, w + lay.pidx, 4 * s->n_p2l, hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            int64_t me = 0, pe = 0;
            for (int64_t t = 0; t < nl; ++t) {
                me += (int64_t)(mo[t + 1] - mo[t]) * (ts[t + 1] - ts[t]);
                for (int32_t k = po[t]; k < po[t + 1]; ++k) pe += ss[pi[k] + 1] - ss[pi[k]];
            }
            s->n_m2p_evals = me;
            s->n_p2l_evals = pe;
        }
        free(mo); free(po); free(pi);
        free(so); free(ss); free(ts); free(si);
        HIPCHK(h, e);
    }
    s->used_model = h->used_model;
    if (h->used_orders && s->n_weak > 0) {
        uint8_t *q = (uint8_t *)malloc((size_t)s->n_weak);
        hipError_t e = hipMemcpy(q, h->ws + lay.qw, (size_t)s->n_weak, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (int64_t i = 0; i < s->n_weak; ++i) s->p_hist[q[i]]++;
        free(q);
        HIPCHK(h, e);
    } else {
        s->p_hist[h->p] = s->n_weak;
    }
    return FMM2D_OK;
}

extern "C" int fmm2d_get_times(fmm2d_handle *h, float *ms)
{
    if (!h || !ms) return FMM2D_EINVAL;
    for (int i = 0; i < FMM2D_NPHASE; ++i) ms[i] = -1.0f;
    if (!h->have_topo) return fail(h, FMM2D_EINVAL, "no evaluation yet");
    if (!h->timing_valid) return FMM2D_OK;
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, hipEventSynchronize(h->ev[FMM2D_NPHASE]));
    for (int i = 0; i < FMM2D_NPHASE; ++i) HIPCHK(h, hipEventElapsedTime(&ms[i], h->ev[i], h->ev[i + 1]));
    return FMM2D_OK;
}

// ------------------------------------------------------- learned order --
extern "C" int fmm2d_set_porder_model(fmm2d_handle *h, const float *model, int64_t n_floats, uint32_t schema,
                                      float delta)
{
    if (!h) return FMM2D_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    if (!model) {
        if (h->d_model) HIPCHK(h, hipFree(h->d_model));
        h->d_model = nullptr;
        return FMM2D_OK;
    }
    if (schema != FMM2D_PORDER_SCHEMA) return fail(h, FMM2D_EINVAL, "unknown feature schema %u", schema);
    if (n_floats != FMM2D_PORDER_MODEL_FLOATS)
        return fail(h, FMM2D_EINVAL, "model has %lld floats, expected %d", (long long)n_floats,
                    FMM2D_PORDER_MODEL_FLOATS);
    for (int64_t i = 0; i < n_floats; ++i)
        if (!isfinite(model[i]) && i < FMM2D_PORDER_NPARAM + 2 * FMM2D_PORDER_NFEAT)
            return fail(h, FMM2D_EINVAL, "model entry %lld is not finite", (long long)i);
    if (!isfinite(delta)) return fail(h, FMM2D_EINVAL, "delta is not finite");
    if (!h->d_model) HIPCHK(h, hipMalloc((void **)&h->d_model, sizeof(float) * FMM2D_PORDER_MODEL_FLOATS));
    HIPCHK(h, hipMemcpy(h->d_model, model, sizeof(float) * FMM2D_PORDER_MODEL_FLOATS, hipMemcpyHostToDevice));
    h->delta = delta;
    return FMM2D_OK;
}

extern "C" int fmm2d_set_pair_orders(fmm2d_handle *h, const uint8_t *orders, int64_t n)
{
    if (!h) return FMM2D_EINVAL;
    if (orders && n < 0) return fail(h, FMM2D_EINVAL, "negative count");
    h->given = orders;
    h->ngiven = orders ? n : 0;
    return FMM2D_OK;
}

// weak-pair count of the last evaluation (synchronises its stream)
static int last_nweak(fmm2d_handle *h, int64_t *nw)
{
    HIPCHK(h, hipStreamSynchronize(h->last_stream));
    int32_t wend = 0;
    const int32_t *woff = reinterpret_cast<const int32_t *>(h->ws + h->lay.woff);
    HIPCHK(h, hipMemcpy(&wend, woff + start_off(h->L) + nbox(h->L), 4, hipMemcpyDeviceToHost));
    *nw = wend;
    return FMM2D_OK;
}

extern "C" int fmm2d_pair_features(fmm2d_handle *h, float *feat, int64_t n_cap, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (!h->have_topo) return fail(h, FMM2D_EINVAL, "no evaluation yet");
    if (!feat || n_cap < 0) return fail(h, FMM2D_EINVAL, "bad feature buffer");
    if (h->p < FMM2D_PORDER_FEAT_K)
        return fail(h, FMM2D_EINVAL, "features need an evaluation at p >= %d", FMM2D_PORDER_FEAT_K);
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    char *w = const_cast<char *>(h->ws);
    const fmm_layout &lay = h->lay;
    fmm_porder_args pa = porder_args(h, w, lay, h->L, h->p, h->lay.cap);
    HIPCHK(h, fmm_box_norms(reinterpret_cast<const double2 *>(w + lay.A), pa.radius, h->p, lay.nb,
                            reinterpret_cast<double *>(w + lay.n1), reinterpret_cast<double *>(w + lay.tail), st));
    HIPCHK(h, fmm_features(pa, n_cap, feat, st));
    return FMM2D_OK;
}

extern "C" int fmm2d_pair_labels(fmm2d_handle *h, const double *val, double tol, int32_t qmin, int32_t qmax,
                                 uint8_t *labels, int64_t n_cap, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (!h->have_topo) return fail(h, FMM2D_EINVAL, "no evaluation yet");
    if (!val || !labels || n_cap < 0) return fail(h, FMM2D_EINVAL, "bad buffers");
    if (!(tol > 0.0)) return fail(h, FMM2D_EINVAL, "tol must be > 0");
    if (h->used_orders) return fail(h, FMM2D_EINVAL, "labels need an evaluation at one fixed order");
    if (h->p > 63) return fail(h, FMM2D_EINVAL, "labels need p <= 63");
    if (qmin < 0 || qmax < qmin || qmax > h->p)
        return fail(h, FMM2D_EINVAL, "need 0 <= qmin <= qmax <= p (%d)", h->p);
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    char *w = const_cast<char *>(h->ws);
    const fmm_layout &lay = h->lay;
    fmm_porder_args pa = porder_args(h, w, lay, h->L, h->p, h->lay.cap);
    const int32_t *tperm = reinterpret_cast<const int32_t *>(w + (h->at_sources ? lay.perm : lay.tperm));
    const int32_t *tstart = reinterpret_cast<const int32_t *>(w + (h->at_sources ? lay.sstart : lay.tstart));
    HIPCHK(h, fmm_labels(pa, reinterpret_cast<const double2 *>(w + lay.A), h->d_binom, tperm, tstart, val, tol, h->p,
                         h->kernel, qmin, qmax, n_cap, reinterpret_cast<double *>(w + lay.vmin),
                         reinterpret_cast<double *>(w + lay.budget), labels, st));
    return FMM2D_OK;
}

extern "C" size_t fmm2d_mlp_work_size(int64_t n)
{
    return n < 0 ? 0 : (size_t)fmm_mlp_grad_blocks(n) * (FMM2D_PORDER_NPARAM + 1) * sizeof(float) + 256;
}

extern "C" int fmm2d_mlp_forward(fmm2d_handle *h, const float *model, const float *x, int64_t n, float *y,
                                 void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (!model || n < 0 || (n > 0 && (!x || !y))) return fail(h, FMM2D_EINVAL, "bad arguments");
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, fmm_mlp_forward(model, x, n, y, (hipStream_t)stream));
    return FMM2D_OK;
}

extern "C" int fmm2d_mlp_grad(fmm2d_handle *h, const float *model, const float *x, const float *q, int64_t n,
                              float tau, float *grad, float *loss, void *work, size_t work_bytes, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (!model || !grad || n < 1 || !x || !q || !work) return fail(h, FMM2D_EINVAL, "bad arguments");
    if (!(tau > 0.0f && tau < 1.0f)) return fail(h, FMM2D_EINVAL, "tau must be in (0,1)");
    if (work_bytes < fmm2d_mlp_work_size(n)) return fail(h, FMM2D_ENOSPC, "work buffer too small");
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, fmm_mlp_grad(model, x, q, n, tau, (float *)work, grad, loss, (hipStream_t)stream));
    return FMM2D_OK;
}

extern "C" int fmm2d_mlp_adam(fmm2d_handle *h, float *model, const float *grad, float *m, float *v, int32_t step,
                              float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!h) return FMM2D_EINVAL;
    if (!model || !grad || !m || !v || step < 1) return fail(h, FMM2D_EINVAL, "bad arguments");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(h, FMM2D_EINVAL, "bad Adam hyper-parameters");
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, fmm_mlp_adam(model, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return FMM2D_OK;
}
