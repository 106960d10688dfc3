/*
 * fmm2d_oracle.c -- plain, slow CPU reference for the adaptive 2D FMM of
 * Goude & Engblom, "Adaptive fast multipole methods on the GPU".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may link, load or call this file; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * code, header, table or helper with the GPU path.
 *
 * Everything is IEEE FP64.  The file is compiled with -ffp-contract=off so
 * that the box geometry and the theta-tests are evaluated exactly in the
 * order written here (the GPU tree must reproduce them bit for bit).
 *
 * Contents (each cites the passage it follows):
 *   orc_nlevels        level rule, eq. (Nlevels) of Sec. 5.1
 *   orc_direct         the definition, eqs. (paireval)/(poteval) of Sec. 1
 *   orc_build          tree (Sec. 2 and Sec. 3.2, readings T1-T7) and
 *                      interaction lists (Sec. 2, theta-criterion)
 *   orc_p2m/m2m/m2l/l2l/eval_*
 *                      closed-form expansions eqs. (multipole), (local),
 *                      written as binomial sums (Sec. 2, Sec. 3.3)
 *   orc_eval           the whole evaluation: upward pass, M2L, downward pass,
 *                      L2P and P2P (Sec. 2)
 *   orc_direct_branch  direct sum on the branch of log that the FMM far field
 *                      follows (reading of the log term of eq. (multipole))
 *   orc_eval_orders    orc_eval with one truncation order per M2L pair
 *   orc_pair_err       truncation error bound e_q of one M2L pair at order q
 *   orc_labels         the smallest order whose e_q meets a per-box budget
 *                      (training labels for the learned order)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_KERNEL_LOG 1      /* Phi = sum m log(y-x) and Phi' = sum m/(y-x) */
#define ORC_KERNEL_HARMONIC 2 /* Phi' only; multipole has a_0 = 0           */
#define ORC_MAXL 15

/* ------------------------------------------------------------------ */
/* Level rule, eq. (Nlevels): L = ceil(0.5 log2(5N / (8 N_d))), clamped at 0.
 * ceil(0.5 log2 x) is the smallest integer L with 4^L >= x, so the rule is
 * evaluated exactly in integers: the smallest L >= 0 with 8 N_d 4^L >= 5 N. */
int orc_nlevels(int64_t n, int64_t nd)
{
    if (n <= 0 || nd <= 0) return -1;
    int L = 0;
    __int128 lhs = (__int128)8 * nd;
    while (lhs < (__int128)5 * n) { lhs *= 4; ++L; }
    return L;
}

/* ------------------------------------------------------------------ */
/* Direct sums, the definition (eq. (poteval); eq. (paireval) when the targets
 * are the sources).  Coincident pairs (both coordinates equal) are skipped.
 * Each of Re/Im Phi and Re/Im Phi' is summed with Neumaier's compensated
 * summation.  tsel (optional) selects a subset of targets. */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

void orc_direct(int64_t ns, const double *src, const double *m, int64_t nt,
                const double *tgt, const int64_t *tsel, int64_t nsel,
                int kernel, double *phi, double *dphi)
{
    if (!tgt) { tgt = src; nt = ns; }
    int64_t nout = tsel ? nsel : nt;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t o = 0; o < nout; ++o) {
        int64_t i = tsel ? tsel[o] : o;
        double yx = tgt[2 * i], yy = tgt[2 * i + 1];
        nsum pr = {0, 0}, pi = {0, 0}, dr = {0, 0}, di = {0, 0};
        for (int64_t j = 0; j < ns; ++j) {
            double xx = src[2 * j], xy = src[2 * j + 1];
            if (xx == yx && xy == yy) continue;
            cplx w = (yx - xx) + I * (yy - xy);
            cplx mj = m[2 * j] + I * m[2 * j + 1];
            cplx d = mj / w;
            nadd(&dr, creal(d));
            nadd(&di, cimag(d));
            if (kernel == ORC_KERNEL_LOG) {
                cplx f = mj * clog(w);
                nadd(&pr, creal(f));
                nadd(&pi, cimag(f));
            }
        }
        if (dphi) { dphi[2 * o] = nval(&dr); dphi[2 * o + 1] = nval(&di); }
        if (phi && kernel == ORC_KERNEL_LOG) {
            phi[2 * o] = nval(&pr); phi[2 * o + 1] = nval(&pi);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Binomial coefficients C(n,k) in FP64 from Pascal's rule (exact while they
 * stay below 2^53, correctly rounded sums of exact values beyond). */
#define ORC_BMAX 192
static double g_binom[ORC_BMAX][ORC_BMAX];
static int g_binom_ready = 0;
static void binom_init(void)
{
    if (g_binom_ready) return;
    for (int n = 0; n < ORC_BMAX; ++n) {
        g_binom[n][0] = 1.0;
        for (int k = 1; k <= n; ++k)
            g_binom[n][k] = g_binom[n - 1][k - 1] + (k <= n - 1 ? g_binom[n - 1][k] : 0.0);
        for (int k = n + 1; k < ORC_BMAX; ++k) g_binom[n][k] = 0.0;
    }
    g_binom_ready = 1;
}
static double binom(int n, int k)
{
    if (k < 0 || n < 0 || k > n) return 0.0;
    return g_binom[n][k];
}
double orc_binom(int n, int k) { binom_init(); return binom(n, k); }

/* ------------------------------------------------------------------ */
/* Expansions (eq. (multipole), eq. (local)), closed-form binomial sums.
 * Coefficient arrays hold p+1 complex numbers, interleaved (re, im):
 *   M(z) = a_0 log(z - c) + sum_{k=1..p} a_k (z - c)^{-k}
 *   L(z) = sum_{l=0..p} b_l (z - c)^l                                    */

/* P2M (Alg. "Multipole initialization"): the Taylor coefficients of the
 * sources' field about the box centre c.
 *   LOG:      m log(z-x) = m log(z-c) - sum_k m (x-c)^k / k  (z-c)^{-k}
 *   HARMONIC: m/(z-x)    = sum_{k>=1} m (x-c)^{k-1} (z-c)^{-k}            */
void orc_p2m(int kernel, int p, double cx, double cy, int64_t n,
             const double *x, const double *m, double *a_out)
{
    cplx *a = (cplx *)a_out;
    for (int k = 0; k <= p; ++k) a[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        cplx d = (x[2 * j] - cx) + I * (x[2 * j + 1] - cy);
        cplx mj = m[2 * j] + I * m[2 * j + 1];
        if (kernel == ORC_KERNEL_LOG) {
            a[0] += mj;
            cplx pw = 1;
            for (int k = 1; k <= p; ++k) { pw *= d; a[k] -= mj * pw / (double)k; }
        } else {
            cplx pw = 1;
            for (int k = 1; k <= p; ++k) { a[k] += mj * pw; pw *= d; }
        }
    }
}

/* M2M (Alg. "Multipole to multipole translation"): re-expand a multipole
 * about c_c as one about c_p, r = c_c - c_p.  From
 *   log(z-c_c)       = log(z-c_p) - sum_{l>=1} r^l/l (z-c_p)^{-l}
 *   (z-c_c)^{-k}     = sum_{l>=k} C(l-1,k-1) r^{l-k} (z-c_p)^{-l}
 * so a'_0 = a_0 and a'_l = -a_0 r^l / l + sum_{k=1..l} C(l-1,k-1) a_k r^{l-k}.
 * This is exact (no truncation).  Accumulates into a_par. */
void orc_m2m(int p, const double *a_child, double rx, double ry, double *a_par)
{
    binom_init();
    const cplx *a = (const cplx *)a_child;
    cplx *o = (cplx *)a_par;
    cplx r = rx + I * ry;
    cplx rp[ORC_BMAX];
    rp[0] = 1;
    for (int l = 1; l <= p; ++l) rp[l] = rp[l - 1] * r;
    o[0] += a[0];
    for (int l = 1; l <= p; ++l) {
        cplx s = -a[0] * rp[l] / (double)l;
        for (int k = 1; k <= l; ++k) s += binom(l - 1, k - 1) * a[k] * rp[l - k];
        o[l] += s;
    }
}

/* M2L (Alg. "Multipole to local translation"; this is the textbook
 * re-expansion, which the printed listing intends): a multipole about c_S
 * re-expanded as a local expansion about c_T, rho = c_T - c_S.  With
 * w = z - c_T and z - c_S = rho (1 + w/rho):
 *   log(z-c_S)   = Log(rho) - sum_{l>=1} (-w/rho)^l / l
 *   (z-c_S)^{-k} = rho^{-k} sum_{l>=0} C(k+l-1, l) (-w/rho)^l
 * so b_0 += a_0 Log(rho) + sum_k a_k rho^{-k} and, for l >= 1,
 *    b_l += (-1)^l rho^{-l} [ -a_0/l + sum_{k=1..p} C(k+l-1,l) a_k rho^{-k} ].
 * Log is the principal branch.  Accumulates into b. */
void orc_m2l(int p, const double *a_src, double rhox, double rhoy, double *b_out)
{
    binom_init();
    const cplx *a = (const cplx *)a_src;
    cplx *b = (cplx *)b_out;
    cplx rho = rhox + I * rhoy;
    cplx ri = 1.0 / rho;
    cplx rp[ORC_BMAX]; /* rho^{-k} */
    rp[0] = 1;
    for (int k = 1; k <= p; ++k) rp[k] = rp[k - 1] * ri;
    cplx s0 = a[0] * clog(rho);
    for (int k = 1; k <= p; ++k) s0 += a[k] * rp[k];
    b[0] += s0;
    for (int l = 1; l <= p; ++l) {
        cplx s = -a[0] / (double)l;
        for (int k = 1; k <= p; ++k) s += binom(k + l - 1, l) * a[k] * rp[k];
        double sgn = (l & 1) ? -1.0 : 1.0;
        b[l] += sgn * rp[l] * s;
    }
}

/* L2L (Alg. "Local to local translation"): re-centre a polynomial from c_p to
 * c_c, r = c_c - c_p:  sum_j b_j (w + r)^j = sum_l [sum_{j>=l} C(j,l) b_j
 * r^{j-l}] w^l.  Exact.  Accumulates into b_child. */
void orc_l2l(int p, const double *b_par, double rx, double ry, double *b_child)
{
    binom_init();
    const cplx *b = (const cplx *)b_par;
    cplx *o = (cplx *)b_child;
    cplx r = rx + I * ry;
    cplx rp[ORC_BMAX];
    rp[0] = 1;
    for (int l = 1; l <= p; ++l) rp[l] = rp[l - 1] * r;
    for (int l = 0; l <= p; ++l) {
        cplx s = 0;
        for (int j = l; j <= p; ++j) s += binom(j, l) * b[j] * rp[j - l];
        o[l] += s;
    }
}

/* P2L (Sec. 2, leaf-level swapped criterion): the sources' field expanded
 * directly as a local expansion about c, valid for |z - c| < |x - c|:
 *   LOG:      m log(z-x) = m Log(c-x) - sum_{l>=1} m/(l (x-c)^l) (z-c)^l
 *   HARMONIC: m/(z-x)    = -sum_{l>=0} m/(x-c)^{l+1} (z-c)^l
 * Accumulates into b. */
void orc_p2l(int kernel, int p, double cx, double cy, int64_t n, const double *x,
             const double *m, double *b_out)
{
    cplx *b = (cplx *)b_out;
    for (int64_t j = 0; j < n; ++j) {
        cplx d = (x[2 * j] - cx) + I * (x[2 * j + 1] - cy); /* x - c */
        cplx mj = m[2 * j] + I * m[2 * j + 1];
        cplx di = 1.0 / d, pw = 1;
        if (kernel == ORC_KERNEL_LOG) {
            b[0] += mj * clog((cx - x[2 * j]) + I * (cy - x[2 * j + 1]));
            for (int l = 1; l <= p; ++l) { pw *= di; b[l] -= mj * pw / (double)l; }
        } else {
            for (int l = 0; l <= p; ++l) { pw *= di; b[l] -= mj * pw; }
        }
    }
}

/* Evaluate a multipole expansion at z (principal Log), and its derivative. */
void orc_eval_multipole(int p, const double *a_in, double cx, double cy,
                        double zx, double zy, double *val, double *der)
{
    const cplx *a = (const cplx *)a_in;
    cplx w = (zx - cx) + I * (zy - cy);
    cplx wi = 1.0 / w;
    cplx v = a[0] * clog(w), d = a[0] * wi, pw = 1;
    for (int k = 1; k <= p; ++k) {
        pw *= wi;
        v += a[k] * pw;
        d -= (double)k * a[k] * pw * wi;
    }
    if (val) { val[0] = creal(v); val[1] = cimag(v); }
    if (der) { der[0] = creal(d); der[1] = cimag(d); }
}

/* L2P: evaluate a local expansion and its derivative at z. */
void orc_eval_local(int p, const double *b_in, double cx, double cy,
                    double zx, double zy, double *val, double *der)
{
    const cplx *b = (const cplx *)b_in;
    cplx w = (zx - cx) + I * (zy - cy);
    cplx v = 0, d = 0, pw = 1;
    for (int l = 0; l <= p; ++l) {
        v += b[l] * pw;
        if (l + 1 <= p) d += (double)(l + 1) * b[l + 1] * pw;
        pw *= w;
    }
    if (val) { val[0] = creal(v); val[1] = cimag(v); }
    if (der) { der[0] = creal(d); der[1] = cimag(d); }
}

/* ------------------------------------------------------------------ */
/* Tree (Sec. 2 "asymmetric adaptivity", Sec. 3.2 "sorting"), under the
 * readings:
 *  T2 level 0 is one box with every point;
 *  T3 each box is split twice; children 4b+0..3 = lo.lo, lo.hi, hi.lo, hi.hi;
 *  T4 one split of a set with n sources: axis x if the tight rectangle of its
 *     sources and targets has w >= h, else y; sources ordered by (coordinate on
 *     the axis, original index); the first floor(n/2) go to lo; a target goes to
 *     hi iff its coordinate >= that of the first hi source;
 *  T5 every partition is stable, so inside a box points stay in ascending
 *     original index;
 *  T6 box geometry: tight rectangle of sources and targets, centre = midpoint,
 *     radius = half diagonal.
 * Interaction lists (Sec. 2, eq. (thetacriterion)): strong(root) = {root};
 * for box b at level l the candidates are the children of the parent's strong
 * boxes, in ascending order; candidate s is weak iff s != b, d > 0 and
 * R + theta r <= theta d, else strong.  strong at the finest level = P2P. */
typedef struct {
    int L;
    double theta;
    int64_t ns, nt;        /* nt == 0: evaluation at the sources            */
    const double *src;     /* borrowed, interleaved (x, y)                  */
    const double *tgt;
    int32_t *perm;         /* [ns] sources in leaf order                    */
    int32_t *tperm;        /* [nt]                                          */
    int64_t *sstart;       /* per level l: 4^l + 1 entries, concatenated    */
    int64_t *tstart;
    double *cen;           /* [nboxes][2]                                   */
    double *rad;           /* [nboxes]                                      */
    int64_t *woff[ORC_MAXL + 1], *soff[ORC_MAXL + 1];
    int32_t *widx[ORC_MAXL + 1], *sidx[ORC_MAXL + 1];
    int swap;              /* leaf-level swapped criterion in use            */
    int64_t *moff, *poff;  /* finest level: M2P and P2L lists (CSR)          */
    int32_t *midx, *pidx;
} orc_tree;

static int64_t box_off(int l) { return ((((int64_t)1) << (2 * l)) - 1) / 3; }
static int64_t nbox(int l) { return ((int64_t)1) << (2 * l); }
static int64_t start_off(int l) { return box_off(l) + l; } /* sum_{j<l} (4^j+1) */

typedef struct { double c; int32_t i; } keyed;
static int keyed_cmp(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->c < b->c) return -1;
    if (a->c > b->c) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

static void rect_of(const double *src, const int32_t *s, int64_t n,
                    const double *tgt, const int32_t *t, int64_t m, double r[4])
{
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t k = 0; k < n; ++k) {
        double x = src[2 * s[k]], y = src[2 * s[k] + 1];
        if (x < x0) x0 = x;
        if (x > x1) x1 = x;
        if (y < y0) y0 = y;
        if (y > y1) y1 = y;
    }
    for (int64_t k = 0; k < m; ++k) {
        double x = tgt[2 * t[k]], y = tgt[2 * t[k] + 1];
        if (x < x0) x0 = x;
        if (x > x1) x1 = x;
        if (y < y0) y0 = y;
        if (y > y1) y1 = y;
    }
    r[0] = x0; r[1] = x1; r[2] = y0; r[3] = y1;
}

/* Stable partition of idx[0..n) by pred; returns the number in front. */
static int64_t stable_partition(int32_t *idx, int64_t n, const char *lo, int32_t *tmp)
{
    int64_t a = 0, b = 0;
    for (int64_t k = 0; k < n; ++k) if (lo[k]) tmp[a++] = idx[k];
    for (int64_t k = 0; k < n; ++k) if (!lo[k]) tmp[a + b++] = idx[k];
    memcpy(idx, tmp, (size_t)n * sizeof(int32_t));
    return a;
}

/* One split (reading T4) of the source segment s[0..n) and target segment
 * t[0..m); both are reordered in place, lo part first. */
static void split_set(const double *src, int32_t *s, int64_t n,
                      const double *tgt, int32_t *t, int64_t m,
                      int64_t *nlo, int64_t *mlo)
{
    *nlo = 0; *mlo = 0;
    if (n == 0) return;
    double r[4];
    rect_of(src, s, n, tgt, t, m, r);
    int ax = (r[1] - r[0] >= r[3] - r[2]) ? 0 : 1;
    keyed *kv = (keyed *)malloc((size_t)n * sizeof(keyed));
    for (int64_t k = 0; k < n; ++k) { kv[k].c = src[2 * s[k] + ax]; kv[k].i = s[k]; }
    qsort(kv, (size_t)n, sizeof(keyed), keyed_cmp);
    keyed piv = kv[n / 2]; /* first source of the hi half */
    free(kv);
    char *lo = (char *)malloc((size_t)(n > m ? n : m) + 1);
    int32_t *tmp = (int32_t *)malloc(((size_t)(n > m ? n : m) + 1) * sizeof(int32_t));
    for (int64_t k = 0; k < n; ++k) {
        keyed e = {src[2 * s[k] + ax], s[k]};
        lo[k] = keyed_cmp(&e, &piv) < 0;
    }
    *nlo = stable_partition(s, n, lo, tmp);
    for (int64_t k = 0; k < m; ++k) lo[k] = !(tgt[2 * t[k] + ax] >= piv.c);
    *mlo = stable_partition(t, m, lo, tmp);
    free(lo);
    free(tmp);
}

static int theta_weak(const double *cb, double rb, const double *cs, double rs, double theta)
{
    double dx = cb[0] - cs[0];
    double dy = cb[1] - cs[1];
    double d = sqrt(dx * dx + dy * dy);
    double R = rb >= rs ? rb : rs;
    double r = rb >= rs ? rs : rb;
    return d > 0.0 && R + theta * r <= theta * d;
}

/* The criterion with the roles of the radii interchanged (Sec. 2, last
 * paragraph on the passes): r + theta R <= theta d. */
static int theta_swapped(const double *cb, double rb, const double *cs, double rs, double theta)
{
    double dx = cb[0] - cs[0];
    double dy = cb[1] - cs[1];
    double d = sqrt(dx * dx + dy * dy);
    double R = rb >= rs ? rb : rs;
    double r = rb >= rs ? rs : rb;
    return d > 0.0 && r + theta * R <= theta * d;
}

typedef struct { int32_t *v; int64_t n, cap; } ivec;
static void ipush(ivec *a, int32_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->v = (int32_t *)realloc(a->v, (size_t)a->cap * sizeof(int32_t));
    }
    a->v[a->n++] = x;
}

void orc_free(orc_tree *T);

orc_tree *orc_build(int64_t ns, const double *src, int64_t nt, const double *tgt,
                    int L, double theta, int swap)
{
    if (ns <= 0 || L < 0 || L > ORC_MAXL || nbox(L) > ns) return NULL;
    orc_tree *T = (orc_tree *)calloc(1, sizeof(orc_tree));
    T->L = L; T->theta = theta; T->ns = ns; T->src = src; T->swap = swap;
    T->nt = tgt ? nt : 0; T->tgt = tgt;
    int64_t nb = box_off(L + 1);
    T->perm = (int32_t *)malloc((size_t)ns * sizeof(int32_t));
    T->tperm = (int32_t *)malloc(((size_t)T->nt + 1) * sizeof(int32_t));
    T->sstart = (int64_t *)malloc((size_t)start_off(L + 1) * sizeof(int64_t));
    T->tstart = (int64_t *)malloc((size_t)start_off(L + 1) * sizeof(int64_t));
    T->cen = (double *)malloc((size_t)nb * 2 * sizeof(double));
    T->rad = (double *)malloc((size_t)nb * sizeof(double));
    for (int64_t k = 0; k < ns; ++k) T->perm[k] = (int32_t)k;
    for (int64_t k = 0; k < T->nt; ++k) T->tperm[k] = (int32_t)k;

    /* segments of the current split step */
    int64_t *ss = (int64_t *)malloc((size_t)(nbox(L) + 1) * sizeof(int64_t));
    int64_t *ts = (int64_t *)malloc((size_t)(nbox(L) + 1) * sizeof(int64_t));
    int64_t *ss2 = (int64_t *)malloc((size_t)(nbox(L) + 1) * sizeof(int64_t));
    int64_t *ts2 = (int64_t *)malloc((size_t)(nbox(L) + 1) * sizeof(int64_t));
    ss[0] = 0; ss[1] = ns; ts[0] = 0; ts[1] = T->nt;
    const double *tg = tgt ? tgt : src;
    for (int l = 0; l <= L; ++l) {
        int64_t nbl = nbox(l);
        for (int64_t b = 0; b <= nbl; ++b) {
            T->sstart[start_off(l) + b] = ss[b];
            T->tstart[start_off(l) + b] = ts[b];
        }
        for (int64_t b = 0; b < nbl; ++b) { /* geometry, reading T6 */
            double r[4];
            rect_of(src, T->perm + ss[b], ss[b + 1] - ss[b], tg, T->tperm + ts[b],
                    ts[b + 1] - ts[b], r);
            double w = r[1] - r[0], h = r[3] - r[2];
            int64_t g = box_off(l) + b;
            T->cen[2 * g] = 0.5 * (r[0] + r[1]);
            T->cen[2 * g + 1] = 0.5 * (r[2] + r[3]);
            T->rad[g] = 0.5 * sqrt(w * w + h * h);
        }
        if (l == L) break;
        /* two successive splits (reading T3) */
        int64_t nseg = nbl;
        for (int step = 0; step < 2; ++step) {
            for (int64_t j = 0; j < nseg; ++j) {
                int64_t nlo, mlo;
                split_set(src, T->perm + ss[j], ss[j + 1] - ss[j], tg,
                          T->tperm + ts[j], ts[j + 1] - ts[j], &nlo, &mlo);
                ss2[2 * j] = ss[j]; ss2[2 * j + 1] = ss[j] + nlo;
                ts2[2 * j] = ts[j]; ts2[2 * j + 1] = ts[j] + mlo;
            }
            nseg *= 2;
            ss2[nseg] = ns; ts2[nseg] = T->nt;
            memcpy(ss, ss2, (size_t)(nseg + 1) * sizeof(int64_t));
            memcpy(ts, ts2, (size_t)(nseg + 1) * sizeof(int64_t));
        }
    }
    free(ss); free(ts); free(ss2); free(ts2);

    /* interaction lists */
    T->woff[0] = (int64_t *)calloc(2, sizeof(int64_t));
    T->soff[0] = (int64_t *)malloc(2 * sizeof(int64_t));
    T->widx[0] = (int32_t *)malloc(sizeof(int32_t));
    T->sidx[0] = (int32_t *)malloc(sizeof(int32_t));
    T->soff[0][0] = 0; T->soff[0][1] = 1; T->sidx[0][0] = 0;
    ivec mv = {0, 0, 0}, pv = {0, 0, 0};
    T->moff = (int64_t *)calloc((size_t)nbox(L) + 1, sizeof(int64_t));
    T->poff = (int64_t *)calloc((size_t)nbox(L) + 1, sizeof(int64_t));
    for (int l = 1; l <= L; ++l) {
        int64_t nbl = nbox(l);
        ivec wv = {0, 0, 0}, sv = {0, 0, 0};
        T->woff[l] = (int64_t *)malloc((size_t)(nbl + 1) * sizeof(int64_t));
        T->soff[l] = (int64_t *)malloc((size_t)(nbl + 1) * sizeof(int64_t));
        const double *C = T->cen + 2 * box_off(l);
        const double *Rr = T->rad + box_off(l);
        for (int64_t b = 0; b < nbl; ++b) {
            T->woff[l][b] = wv.n;
            T->soff[l][b] = sv.n;
            if (l == L) { T->moff[b] = mv.n; T->poff[b] = pv.n; }
            int64_t q = b / 4;
            for (int64_t e = T->soff[l - 1][q]; e < T->soff[l - 1][q + 1]; ++e) {
                int64_t s = T->sidx[l - 1][e];
                for (int k = 0; k < 4; ++k) {
                    int64_t c = 4 * s + k;
                    if (c != b && theta_weak(C + 2 * b, Rr[b], C + 2 * c, Rr[c], theta))
                        ipush(&wv, (int32_t)c);
                    else if (l == L && swap && c != b &&
                             theta_swapped(C + 2 * b, Rr[b], C + 2 * c, Rr[c], theta))
                        ipush(Rr[b] > Rr[c] ? &mv : &pv, (int32_t)c);
                    else
                        ipush(&sv, (int32_t)c);
                }
            }
        }
        T->woff[l][nbl] = wv.n;
        T->soff[l][nbl] = sv.n;
        if (l == L) { T->moff[nbl] = mv.n; T->poff[nbl] = pv.n; }
        T->widx[l] = wv.v ? wv.v : (int32_t *)malloc(sizeof(int32_t));
        T->sidx[l] = sv.v ? sv.v : (int32_t *)malloc(sizeof(int32_t));
    }
    T->midx = mv.v ? mv.v : (int32_t *)malloc(sizeof(int32_t));
    T->pidx = pv.v ? pv.v : (int32_t *)malloc(sizeof(int32_t));
    return T;
}

void orc_free(orc_tree *T)
{
    if (!T) return;
    free(T->perm); free(T->tperm); free(T->sstart); free(T->tstart);
    free(T->cen); free(T->rad);
    for (int l = 0; l <= T->L; ++l) {
        free(T->woff[l]); free(T->soff[l]); free(T->widx[l]); free(T->sidx[l]);
    }
    free(T->moff); free(T->poff); free(T->midx); free(T->pidx);
    free(T);
}

/* Accessors for the Python wrapper. */
int orc_levels_of(const orc_tree *T) { return T->L; }
/* which: 0 weak, 1 strong (P2P at the finest level), 2 M2P, 3 P2L (the last
 * two exist at the finest level only). */
static void list_of(const orc_tree *T, int l, int which, const int64_t **o, const int32_t **v)
{
    switch (which) {
    case 0: *o = T->woff[l]; *v = T->widx[l]; break;
    case 1: *o = T->soff[l]; *v = T->sidx[l]; break;
    case 2: *o = T->moff; *v = T->midx; break;
    default: *o = T->poff; *v = T->pidx; break;
    }
}
int64_t orc_list_len(const orc_tree *T, int l, int which)
{
    const int64_t *o; const int32_t *v;
    list_of(T, l, which, &o, &v);
    return o[nbox(l)];
}
void orc_get_list(const orc_tree *T, int l, int which, int64_t *off, int32_t *idx)
{
    int64_t nbl = nbox(l);
    const int64_t *o; const int32_t *v;
    list_of(T, l, which, &o, &v);
    memcpy(off, o, (size_t)(nbl + 1) * sizeof(int64_t));
    memcpy(idx, v, (size_t)o[nbl] * sizeof(int32_t));
}
void orc_get_tree(const orc_tree *T, int32_t *perm, int32_t *tperm, int64_t *sstart,
                  int64_t *tstart, double *cen, double *rad)
{
    int L = T->L;
    if (perm) memcpy(perm, T->perm, (size_t)T->ns * sizeof(int32_t));
    if (tperm && T->nt) memcpy(tperm, T->tperm, (size_t)T->nt * sizeof(int32_t));
    if (sstart) memcpy(sstart, T->sstart, (size_t)start_off(L + 1) * sizeof(int64_t));
    if (tstart) memcpy(tstart, T->tstart, (size_t)start_off(L + 1) * sizeof(int64_t));
    if (cen) memcpy(cen, T->cen, (size_t)box_off(L + 1) * 2 * sizeof(double));
    if (rad) memcpy(rad, T->rad, (size_t)box_off(L + 1) * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* The whole evaluation (Sec. 2): P2M at the leaves, M2M upward through every
 * level, M2L over every weak pair of every level, L2L downward, then at each
 * leaf L2P plus P2P over its strong list.  A and B (optional outputs) receive
 * the multipole and local coefficients of every box, [nboxes][p+1] complex,
 * with B holding the complete local expansion (M2L plus inherited L2L). */
/* qw (optional): one order q in [1, p] per weak pair, in the order of the
 * weak lists of levels 1, 2, ..., L concatenated; pair (T, S) then adds
 * orc_m2l at order q (a_0..a_q of S into b_0..b_q of T). */
static int eval_impl(const orc_tree *T, const double *m, int kernel, int p, const unsigned char *qw,
                     double *phi, double *dphi, double *A_out, double *B_out);

int orc_eval(const orc_tree *T, const double *m, int kernel, int p,
             double *phi, double *dphi, double *A_out, double *B_out)
{
    return eval_impl(T, m, kernel, p, NULL, phi, dphi, A_out, B_out);
}

int orc_eval_orders(const orc_tree *T, const double *m, int kernel, int p, const unsigned char *qw,
                    double *phi, double *dphi, double *A_out, double *B_out)
{
    return eval_impl(T, m, kernel, p, qw, phi, dphi, A_out, B_out);
}

static int eval_impl(const orc_tree *T, const double *m, int kernel, int p, const unsigned char *qw,
                     double *phi, double *dphi, double *A_out, double *B_out)
{
    if (p < 1 || p >= ORC_BMAX / 2) return -1;
    binom_init();
    int L = T->L;
    int64_t nb = box_off(L + 1), P1 = p + 1;
    double *A = (double *)calloc((size_t)(nb * P1 * 2), sizeof(double));
    double *B = (double *)calloc((size_t)(nb * P1 * 2), sizeof(double));
    const double *tg = T->nt ? T->tgt : T->src;
    const int32_t *tperm = T->nt ? T->tperm : T->perm;
    const int64_t *tst = (T->nt ? T->tstart : T->sstart) + start_off(L);
    const int64_t *sst = T->sstart + start_off(L);
    int64_t nleaf = nbox(L), lo = box_off(L);

    /* P2M at the leaves */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nleaf; ++b) {
        int64_t n = sst[b + 1] - sst[b];
        double *xs = (double *)malloc((size_t)(2 * n + 1) * sizeof(double));
        double *ms = (double *)malloc((size_t)(2 * n + 1) * sizeof(double));
        for (int64_t k = 0; k < n; ++k) {
            int32_t j = T->perm[sst[b] + k];
            xs[2 * k] = T->src[2 * j]; xs[2 * k + 1] = T->src[2 * j + 1];
            ms[2 * k] = m[2 * j]; ms[2 * k + 1] = m[2 * j + 1];
        }
        int64_t g = lo + b;
        orc_p2m(kernel, p, T->cen[2 * g], T->cen[2 * g + 1], n, xs, ms, A + 2 * P1 * g);
        free(xs); free(ms);
    }
    /* M2M upward */
    for (int l = L - 1; l >= 0; --l) {
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < nbox(l); ++b) {
            int64_t g = box_off(l) + b;
            for (int k = 0; k < 4; ++k) {
                int64_t c = box_off(l + 1) + 4 * b + k;
                orc_m2m(p, A + 2 * P1 * c, T->cen[2 * c] - T->cen[2 * g],
                        T->cen[2 * c + 1] - T->cen[2 * g + 1], A + 2 * P1 * g);
            }
        }
    }
    /* M2L over every weak pair (at its own order if qw is given), then L2L
     * downward */
    int64_t qbase = 0;
    for (int l = 1; l <= L; ++l) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t b = 0; b < nbox(l); ++b) {
            int64_t g = box_off(l) + b;
            for (int64_t e = T->woff[l][b]; e < T->woff[l][b + 1]; ++e) {
                int64_t s = box_off(l) + T->widx[l][e];
                int q = p;
                if (qw) {
                    q = qw[qbase + e];
                    if (q < 1) q = 1;
                    if (q > p) q = p;
                }
                orc_m2l(q, A + 2 * P1 * s, T->cen[2 * g] - T->cen[2 * s],
                        T->cen[2 * g + 1] - T->cen[2 * s + 1], B + 2 * P1 * g);
            }
        }
        qbase += T->woff[l][nbox(l)];
    }
    for (int l = 1; l <= L; ++l) {
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < nbox(l); ++b) {
            int64_t g = box_off(l) + b, q = box_off(l - 1) + b / 4;
            orc_l2l(p, B + 2 * P1 * q, T->cen[2 * g] - T->cen[2 * q],
                    T->cen[2 * g + 1] - T->cen[2 * q + 1], B + 2 * P1 * g);
        }
    }
    /* P2L: sources of large boxes straight into the local expansions of the
     * small leaves that pass the swapped criterion */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nleaf; ++t) {
        int64_t g = lo + t;
        for (int64_t e = T->poff[t]; e < T->poff[t + 1]; ++e) {
            int64_t s = T->pidx[e];
            int64_t n = sst[s + 1] - sst[s];
            double *xs = (double *)malloc((size_t)(2 * n + 1) * sizeof(double));
            double *ms = (double *)malloc((size_t)(2 * n + 1) * sizeof(double));
            for (int64_t k = 0; k < n; ++k) {
                int32_t j = T->perm[sst[s] + k];
                xs[2 * k] = T->src[2 * j]; xs[2 * k + 1] = T->src[2 * j + 1];
                ms[2 * k] = m[2 * j]; ms[2 * k + 1] = m[2 * j + 1];
            }
            orc_p2l(kernel, p, T->cen[2 * g], T->cen[2 * g + 1], n, xs, ms, B + 2 * P1 * g);
            free(xs); free(ms);
        }
    }
    /* L2P + M2P + P2P at the leaves */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nleaf; ++t) {
        int64_t g = lo + t;
        for (int64_t k = tst[t]; k < tst[t + 1]; ++k) {
            int32_t i = tperm[k];
            double yx = tg[2 * i], yy = tg[2 * i + 1];
            double v[2], d[2];
            orc_eval_local(p, B + 2 * P1 * g, T->cen[2 * g], T->cen[2 * g + 1], yx, yy, v, d);
            cplx fv = v[0] + I * v[1], fd = d[0] + I * d[1];
            /* M2P: multipoles of small leaves evaluated at this target */
            for (int64_t e = T->moff[t]; e < T->moff[t + 1]; ++e) {
                int64_t gs = lo + T->midx[e];
                orc_eval_multipole(p, A + 2 * P1 * gs, T->cen[2 * gs], T->cen[2 * gs + 1], yx, yy, v, d);
                fv += v[0] + I * v[1];
                fd += d[0] + I * d[1];
            }
            cplx nv = 0, nd = 0;
            for (int64_t e = T->soff[L][t]; e < T->soff[L][t + 1]; ++e) {
                int64_t s = T->sidx[L][e];
                for (int64_t q = sst[s]; q < sst[s + 1]; ++q) {
                    int32_t j = T->perm[q];
                    double xx = T->src[2 * j], xy = T->src[2 * j + 1];
                    if (xx == yx && xy == yy) continue;
                    cplx w = (yx - xx) + I * (yy - xy);
                    cplx mj = m[2 * j] + I * m[2 * j + 1];
                    if (kernel == ORC_KERNEL_LOG) {
                        nv += mj * clog(w);
                        nd += mj / w;
                    } else {
                        nv += mj / w;
                    }
                }
            }
            if (kernel == ORC_KERNEL_LOG) {
                if (phi) { phi[2 * i] = creal(fv + nv); phi[2 * i + 1] = cimag(fv + nv); }
                if (dphi) { dphi[2 * i] = creal(fd + nd); dphi[2 * i + 1] = cimag(fd + nd); }
            } else {
                /* HARMONIC: the expansions represent Phi' itself */
                if (dphi) { dphi[2 * i] = creal(fv + nv); dphi[2 * i + 1] = cimag(fv + nv); }
            }
        }
    }
    if (A_out) memcpy(A_out, A, (size_t)(nb * P1 * 2) * sizeof(double));
    if (B_out) memcpy(B_out, B, (size_t)(nb * P1 * 2) * sizeof(double));
    free(A); free(B);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Direct sum of Phi on the branch the FMM far field follows.  For a pair
 * (y, x) whose leaves are P2P neighbours the principal Log(y-x) is used.
 * Otherwise the pair is handled at one level by an ancestor pair (T, S) with
 * S weak to T; the far field then carries Log(c_T - c_S) plus principal logs
 * of numbers close to 1, so its argument is Arg(c_T - c_S) plus the
 * difference Arg(y-x) - Arg(c_T - c_S) wrapped into (-pi, pi].
 * tsel selects targets (original indices); phi is [nsel] complex. */
static int in_sorted(const int32_t *v, int64_t n, int32_t x)
{
    int64_t a = 0, b = n;
    while (a < b) {
        int64_t c = (a + b) / 2;
        if (v[c] < x) a = c + 1; else b = c;
    }
    return a < n && v[a] == x;
}

int orc_direct_branch(const orc_tree *T, const double *m, const int64_t *tsel,
                      int64_t nsel, double *phi)
{
    int L = T->L;
    const double *tg = T->nt ? T->tgt : T->src;
    const int32_t *tperm = T->nt ? T->tperm : T->perm;
    const int64_t *tst = (T->nt ? T->tstart : T->sstart) + start_off(L);
    const int64_t *sst = T->sstart + start_off(L);
    int64_t nleaf = nbox(L), ntg = T->nt ? T->nt : T->ns;
    /* leaf of every target */
    int32_t *leaf_of = (int32_t *)malloc((size_t)ntg * sizeof(int32_t));
    for (int64_t t = 0; t < nleaf; ++t)
        for (int64_t k = tst[t]; k < tst[t + 1]; ++k) leaf_of[tperm[k]] = (int32_t)t;
    const double pi = 3.14159265358979323846;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : bad)
    for (int64_t o = 0; o < nsel; ++o) {
        int64_t i = tsel[o];
        double yx = tg[2 * i], yy = tg[2 * i + 1];
        int32_t t = leaf_of[i];
        nsum pr = {0, 0}, pim = {0, 0};
        for (int64_t s = 0; s < nleaf; ++s) {
            /* find the level at which this leaf pair is handled */
            int lev = -1;
            for (int l = 1; l <= L && lev < 0; ++l) {
                int sh = 2 * (L - l);
                int32_t Tb = t >> sh, Sb = (int32_t)(s >> sh);
                if (in_sorted(T->widx[l] + T->woff[l][Tb], T->woff[l][Tb + 1] - T->woff[l][Tb], Sb))
                    lev = l;
            }
            double ref = 0.0;
            int mode = 0; /* 0 P2P or M2L at lev, 1 M2P (reference Arg(y - c_s)), 2 P2L (Arg(c_t - x)) */
            if (lev < 0) {
                if (in_sorted(T->midx + T->moff[t], T->moff[t + 1] - T->moff[t], (int32_t)s)) {
                    int64_t gs = box_off(L) + s;
                    ref = atan2(yy - T->cen[2 * gs + 1], yx - T->cen[2 * gs]);
                    mode = 1;
                } else if (in_sorted(T->pidx + T->poff[t], T->poff[t + 1] - T->poff[t], (int32_t)s)) {
                    mode = 2;
                } else if (!in_sorted(T->sidx[L] + T->soff[L][t], T->soff[L][t + 1] - T->soff[L][t], (int32_t)s))
                    ++bad; /* not covered: lists are broken */
            } else {
                int sh = 2 * (L - lev);
                int64_t gT = box_off(lev) + (t >> sh), gS = box_off(lev) + (s >> sh);
                ref = atan2(T->cen[2 * gT + 1] - T->cen[2 * gS + 1], T->cen[2 * gT] - T->cen[2 * gS]);
            }
            for (int64_t q = sst[s]; q < sst[s + 1]; ++q) {
                int32_t j = T->perm[q];
                double xx = T->src[2 * j], xy = T->src[2 * j + 1];
                if (xx == yx && xy == yy) continue;
                cplx w = (yx - xx) + I * (yy - xy);
                double lr = log(cabs(w));
                double ar = carg(w);
                if (mode == 2) {
                    int64_t gt = box_off(L) + t;
                    ref = atan2(T->cen[2 * gt + 1] - xy, T->cen[2 * gt] - xx);
                }
                if (lev >= 0 || mode != 0) {
                    double dlt = ar - ref;
                    while (dlt > pi) dlt -= 2 * pi;
                    while (dlt <= -pi) dlt += 2 * pi;
                    ar = ref + dlt;
                }
                cplx f = (m[2 * j] + I * m[2 * j + 1]) * (lr + I * ar);
                nadd(&pr, creal(f));
                nadd(&pim, cimag(f));
            }
        }
        phi[2 * o] = nval(&pr);
        phi[2 * o + 1] = nval(&pim);
    }
    free(leaf_of);
    return bad ? -bad : 0;
}

/* ------------------------------------------------------------------ */
/* Truncation error bound of one M2L pair.  a: multipole at order P about c_S,
 * rho = c_T - c_S, rT the target radius.  b^(q) = orc_m2l at order q (a_0..a_q
 * into b_0..b_q, zero above), and
 *     e_q = sum_{l=0..P} |b_l^(q) - b_l^(P)| rT^l,
 * which bounds the error of the pair truncated at q (against order P) over
 * the disc |z - c_T| <= rT.  Writes e_q for q = qmin..qmax into e[]. */
void orc_pair_err(int P, const double *a, double rhox, double rhoy, double rT, int qmin, int qmax, double *e)
{
    double *bP = (double *)calloc((size_t)(2 * (P + 1)), sizeof(double));
    double *bq = (double *)calloc((size_t)(2 * (P + 1)), sizeof(double));
    orc_m2l(P, a, rhox, rhoy, bP);
    for (int q = qmin; q <= qmax; ++q) {
        memset(bq, 0, (size_t)(2 * (P + 1)) * sizeof(double));
        orc_m2l(q, a, rhox, rhoy, bq); /* q = 0: the log term of b_0 only */
        double eq = 0.0, rl = 1.0;
        for (int l = 0; l <= P; ++l) {
            eq += cabs((bq[2 * l] - bP[2 * l]) + I * (bq[2 * l + 1] - bP[2 * l + 1])) * rl;
            rl *= rT;
        }
        e[q - qmin] = eq;
    }
    free(bP); free(bq);
}

/* Training labels for a per-pair truncation order.  A holds the multipoles of
 * an evaluation at order P.  With V(T) = min over the targets y in box T of
 * |val(y)| (val in the original target order), the budget of T is
 * tol V(T) / max(|weak(T)|, 1), and the label of weak pair (T, S) is the
 * smallest q in [qmin, qmax] whose orc_pair_err e_q is <= that budget, else
 * qmax.  Outputs, per weak pair in the concatenated order of levels 1..L:
 * label[], and optionally err[pair][qmax - qmin + 1] and budget_out[pair]. */
int orc_labels(const orc_tree *T, const double *A, int P, const double *val, double tol, int qmin,
               int qmax, unsigned char *label, double *err, double *budget_out)
{
    if (P < 1 || P >= ORC_BMAX / 2 || qmin < 0 || qmax < qmin || qmax > P) return -1;
    binom_init();
    int L = T->L;
    int64_t P1 = P + 1, nq = qmax - qmin + 1;
    const int32_t *tperm = T->nt ? T->tperm : T->perm;
    const int64_t *tst = T->nt ? T->tstart : T->sstart;
    int64_t qbase = 0;
    for (int l = 1; l <= L; ++l) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < nbox(l); ++b) {
            int64_t g = box_off(l) + b;
            double vmin = INFINITY;
            for (int64_t k = tst[start_off(l) + b]; k < tst[start_off(l) + b + 1]; ++k) {
                int32_t i = tperm[k];
                double v = cabs(val[2 * i] + I * val[2 * i + 1]);
                if (v < vmin) vmin = v;
            }
            int64_t nw = T->woff[l][b + 1] - T->woff[l][b];
            double bud = tol * vmin / (double)(nw > 0 ? nw : 1);
            double *eq = (double *)malloc((size_t)nq * sizeof(double));
            for (int64_t e = T->woff[l][b]; e < T->woff[l][b + 1]; ++e) {
                int64_t s = box_off(l) + T->widx[l][e];
                orc_pair_err(P, A + 2 * P1 * s, T->cen[2 * g] - T->cen[2 * s], T->cen[2 * g + 1] - T->cen[2 * s + 1],
                             T->rad[g], qmin, qmax, eq);
                int lab = qmax;
                for (int q = qmax; q >= qmin; --q)
                    if (eq[q - qmin] <= bud) lab = q;
                label[qbase + e] = (unsigned char)lab;
                if (err) memcpy(err + (qbase + e) * nq, eq, (size_t)nq * sizeof(double));
                if (budget_out) budget_out[qbase + e] = bud;
            }
            free(eq);
        }
        qbase += T->woff[l][nbox(l)];
    }
    return 0;
}
