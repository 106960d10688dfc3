// Learned truncation order for M2L.  The method fixes one order p for every
// interaction (the a-priori rule of Sec. 2, p ~ log(TOL)/log(theta), is the
// fallback here); this file lets a small MLP choose, for every weak (M2L)
// pair, an order q <= p from 8 features of the pair, and lets the caller
// supply orders directly.  The M2L kernels then truncate each interaction at
// its own order: they read a_0..a_q of the source and produce b_0..b_q.
//
// Features (schema 1), FP32 from FP64 quantities, for target box T at level l
// of L and source box S in weak(T), d = |c_T - c_S|, rho = box radius,
// sigma = max(rho, 2^-20 rho_root) and ahat_k = a_k / sigma^k, k = 0..K with
// K = FMM2D_PORDER_FEAT_K:
//   f0 rho_S / d             f1 rho_T / d            f2 (rho_S + rho_T) / d
//   f3 l / L                 f4 log10(|ahat_S|_1 / |ahat_root|_1)
//   f5 log10(sum_{k > K/2} |ahat_{S,k}| / |ahat_S|_1)           (decay)
//   f6 log10(|ahat_S|_1 / sum_{S' in weak(T)} |ahat_S'|_1)       (share)
//   f7 log10(|weak(T)|)
// log10 arguments are floored at 1e-300.
//
// Model (FMM2D_PORDER_MODEL_FLOATS floats): the trainable part
//   W1 [32][8] row-major, b1 [32], W2 [32], b2 [1]          (321 floats)
// then fixed standardisation and training range
//   mu [8], isd [8], lo [8], hi [8]
// y = W2 . relu(W1 ((f - mu) * isd) + b1) + b2; the order is
// clamp(ceil(y + delta), FMM2D_PORDER_QMIN, p).  A pair with a feature
// outside [lo, hi] keeps the fixed order p.
#include "common.h"

#define WAVE 64

__device__ __forceinline__ float flog10(double v) { return (float)log10(fmax(v, 1e-300)); }

// log10 of a positive FP64 value from its exact binary exponent and an FP32
// log2 of the mantissa (absolute error ~1e-7); log10(0) = -inf.
__device__ __forceinline__ float lg10_fast(double x)
{
    int e;
    const double m = frexp(x, &e); // x = m 2^e, m in [0.5, 1)
    return ((float)e + __log2f((float)m)) * 0.30102999566398120f;
}
// log10(max(a / b, 1e-300)) with b floored at 1e-300, as a difference of logs
__device__ __forceinline__ float lg10_ratio(double a, double b)
{
    return fmaxf(lg10_fast(a) - lg10_fast(fmax(b, 1e-300)), -300.0f);
}
__device__ __forceinline__ double rcp_nr64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ int level_of_box(int64_t g, int L)
{
    int l = 0;
    while (l < L && d_box_off(l + 1) <= g) ++l;
    return l;
}

// Per box: n1 = |ahat|_1 over k = 0..K and the tail over k > K/2.  Each
// |a_k| is multiplied by 1/sigma k times (no power of 1/sigma is formed, so
// nothing overflows while |a_k| ~ sigma^k).
__global__ void k_box_norms(const double2 *__restrict__ A, const double *__restrict__ radius, int p, int64_t nb,
                            double *__restrict__ n1, double *__restrict__ tail)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb) return;
    const int K = p < FMM2D_PORDER_FEAT_K ? p : FMM2D_PORDER_FEAT_K;
    const double sig = fmax(radius[g], fmax(radius[0] * 0x1p-20, 1e-300));
    const double is = 1.0 / sig;
    const double2 *a = A + g * (p + 1);
    double s = 0.0, t = 0.0;
    for (int k = 0; k <= K; ++k) {
        double v = sqrt(a[k].x * a[k].x + a[k].y * a[k].y);
        for (int q = 0; q < k; ++q) v *= is;
        s += v;
        if (2 * k > K) t += v;
    }
    n1[g] = s;
    tail[g] = t;
}

struct feat_ctx {
    const double *centre, *radius, *n1, *tail;
    int64_t g, bo;
    int l, L;
    double n1root, den;
    int32_t nweak;
};

__device__ __forceinline__ void pair_features(const feat_ctx &c, int64_t gS, float f[FMM2D_PORDER_NFEAT])
{
    const double dx = c.centre[2 * c.g] - c.centre[2 * gS], dy = c.centre[2 * c.g + 1] - c.centre[2 * gS + 1];
    const double d = fmax(sqrt(dx * dx + dy * dy), 1e-300);
    const double id = rcp_nr64(d);
    const double rS = c.radius[gS], rT = c.radius[c.g];
    const double nS = c.n1[gS];
    f[0] = (float)(rS * id);
    f[1] = (float)(rT * id);
    f[2] = (float)((rS + rT) * id);
    f[3] = c.L > 0 ? (float)((double)c.l / (double)c.L) : 0.0f;
    f[4] = lg10_ratio(nS, c.n1root);
    f[5] = lg10_ratio(c.tail[gS], nS);
    f[6] = lg10_ratio(nS, c.den);
    f[7] = lg10_fast((double)(c.nweak > 0 ? c.nweak : 1));
}

// Sum of n1 over the weak list entries [e0, e1) of a box (the share
// denominator of feature f6), in every lane: lane i adds entries i, i + 64, ...
// in order, then a butterfly.  The lane loads 8 entries per round trip (a
// box's list can hold 16k pairs); padding adds exact zeros.
__device__ __forceinline__ double box_den(const double *__restrict__ n1, const int32_t *__restrict__ widx, int32_t e0,
                                          int32_t e1, int64_t bo, int32_t nbl)
{
    const int lane = threadIdx.x & (WAVE - 1);
    double den = 0.0;
    for (int32_t e = e0 + lane; e < e1; e += 8 * WAVE) {
        // all index loads, then all value loads (clamped, always valid), then
        // the sum with the entries past e1 as exact zeros
        int32_t ix[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ix[u] = widx[min(e + u * WAVE, e1 - 1)];
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = n1[bo + min(max(ix[u], 0), nbl - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) den += e + u * WAVE < e1 ? v[u] : 0.0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) den += __shfl_xor(den, o, WAVE);
    return den;
}

// Shared set-up of the wave-per-target-box kernels: the box's weak range and
// the feature context (the share denominator is a wave reduction).
__device__ __forceinline__ bool box_setup(const double *centre, const double *radius, const double *n1,
                                          const double *tail, const int32_t *woff, const int32_t *widx, int L,
                                          int64_t g, int32_t cap, int32_t &e0, int32_t &e1, int32_t &nbl,
                                          feat_ctx &c)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int l = level_of_box(g, L);
    const int64_t bo = d_box_off(l);
    const int64_t so = d_start_off(l);
    const int32_t b = (int32_t)(g - bo);
    e0 = min(woff[so + b], cap);
    e1 = min(woff[so + b + 1], cap);
    if (e0 >= e1) return false;
    nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double den = box_den(n1, widx, e0, e1, bo, nbl);
    c.centre = centre; c.radius = radius; c.n1 = n1; c.tail = tail;
    c.g = g; c.bo = bo; c.l = l; c.L = L;
    c.n1root = n1[0];
    c.den = den;
    c.nweak = woff[so + b + 1] - woff[so + b];
    return true;
}

// The MLP of one pair.  w must be 16-byte aligned: the rows of W1 and the
// blocks of b1 and W2 are read as float4 (half the LDS instructions of
// one-float reads); the operations and their order are those of the loop
// over hidden units j and inputs i.
__device__ __forceinline__ float mlp_eval(const float *__restrict__ w, const float f[FMM2D_PORDER_NFEAT])
{
    static_assert(FMM_NF == 8 && FMM_HID % 4 == 0, "float4 reads of the weights");
    const float *W1 = w, *b1 = W1 + FMM_HID * FMM_NF, *W2 = b1 + FMM_HID, *b2 = W2 + FMM_HID;
    const float *mu = b2 + 1, *isd = mu + FMM_NF;
    float x[FMM_NF];
#pragma unroll
    for (int i = 0; i < FMM_NF; ++i) x[i] = (f[i] - mu[i]) * isd[i];
    float y = b2[0];
    for (int j0 = 0; j0 < FMM_HID; j0 += 4) {
        const float4 bb = *reinterpret_cast<const float4 *>(b1 + j0);
        const float4 ww = *reinterpret_cast<const float4 *>(W2 + j0);
        const float bj[4] = {bb.x, bb.y, bb.z, bb.w}, w2[4] = {ww.x, ww.y, ww.z, ww.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float4 a0 = *reinterpret_cast<const float4 *>(W1 + (j0 + u) * FMM_NF);
            const float4 a1 = *reinterpret_cast<const float4 *>(W1 + (j0 + u) * FMM_NF + 4);
            const float wr[FMM_NF] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            float z = bj[u];
#pragma unroll
            for (int i = 0; i < FMM_NF; ++i) z = fmaf(wr[i], x[i], z);
            y = fmaf(w2[u], fmaxf(z, 0.0f), y);
        }
    }
    return y;
}

// Every feature inside the training range [lo, hi] (a NaN is outside).  The
// tests are combined without short-circuit, so that the check is
// straight-line code after all features are formed (a chain of && compiles
// to one branch and one LDS round trip per bound).
__device__ __forceinline__ bool in_range(const float *__restrict__ w, const float f[FMM_NF])
{
    const float *lo = w + FMM2D_PORDER_NPARAM + 2 * FMM_NF, *hi = lo + FMM_NF;
    uint32_t ok = 1u;
#pragma unroll
    for (int i = 0; i < FMM_NF; ++i) ok &= (uint32_t)(f[i] >= lo[i]) & (uint32_t)(f[i] <= hi[i]);
    return ok != 0u;
}

// Features of every weak pair, in weak-list order: feat[e][8].
__global__ void __launch_bounds__(256) k_features(const double *__restrict__ centre, const double *__restrict__ radius,
                                                  const double *__restrict__ n1, const double *__restrict__ tail,
                                                  const int32_t *__restrict__ woff, const int32_t *__restrict__ widx,
                                                  int L, int64_t nb, int32_t cap, int64_t nfeat_cap,
                                                  float *__restrict__ feat)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t g = wave_index();
    if (g >= nb) return;
    int32_t e0, e1, nbl;
    feat_ctx c;
    if (!box_setup(centre, radius, n1, tail, woff, widx, L, g, cap, e0, e1, nbl, c)) return;
    for (int32_t e = e0 + lane; e < e1; e += WAVE) {
        if (e >= nfeat_cap) break;
        float f[FMM_NF];
        pair_features(c, c.bo + min(max(widx[e], 0), nbl - 1), f);
#pragma unroll
        for (int i = 0; i < FMM_NF; ++i) feat[(int64_t)e * FMM_NF + i] = f[i];
    }
}

// Orders of every weak pair (from the model, or the caller's array).  The
// work is cut into the M2L work units (boxes of up to FMM_M2L_HEAVY weak pairs
// and segments of FMM_M2L_SEG pairs of longer lists) so that very long lists
// do not serialise:
//   k_porder         one wave per M2L work unit: features, MLP and order of
//                    every pair of the unit, then the unit's pairs re-ordered
//                    by increasing order (M2L chunks share similar orders).
#define PORDER_RCH 8 // chunks of 64 pairs per sort unit (FMM_M2L_SEG / 64)
static_assert(PORDER_RCH * 64 >= FMM_M2L_SEG && PORDER_RCH * 64 >= FMM_M2L_HEAVY,
              "a sort unit must fit the register window");

__device__ __forceinline__ bool box_range(const int32_t *__restrict__ woff, int L, int64_t g, int32_t cap,
                                          int &l, int64_t &bo, int32_t &e0, int32_t &e1)
{
    l = level_of_box(g, L);
    bo = d_box_off(l);
    const int64_t so = d_start_off(l) + (g - bo);
    e0 = min(woff[so], cap);
    e1 = min(woff[so + 1], cap);
    return e0 < e1;
}

// The M2L work units (a box of at most FMM_M2L_HEAVY weak pairs, or a segment
// of FMM_M2L_SEG pairs of a longer list): unit t < nb is box t, unit nb + s is
// heavy segment s.  Returns false for units that do not exist.
__device__ __forceinline__ bool porder_unit(const int32_t *__restrict__ woff, const int32_t *__restrict__ hoff,
                                            const int32_t *__restrict__ hbox, int L, int64_t nb, int32_t cap,
                                            int64_t t, int64_t &g, int &l, int64_t &bo, int32_t &e0,
                                            int32_t &e1)
{
    if (t < nb) {
        g = t;
    } else {
        if (t - nb >= hoff[nb]) return false;
        g = hbox[t - nb];
    }
    if (!box_range(woff, L, g, cap, l, bo, e0, e1)) return false;
    if (e1 - e0 > FMM_M2L_HEAVY) {
        if (t < nb) return false; // handled by its segments
        const int32_t s0 = min(e0 + (int32_t)(t - nb - hoff[g]) * FMM_M2L_SEG, e1);
        e1 = min(s0 + FMM_M2L_SEG, e1);
        e0 = s0;
    } else if (t >= nb) {
        return false;
    }
    return true;
}

// M2L body class of an order q: k-steps (q + 3) / 4 plus row tiles q / 16 + 1,
// less one.  Both counts are non-decreasing in q, so equal classes mean equal
// (row tiles, k-steps) and the class is non-decreasing in q; below 20 for q < 64.
__device__ __forceinline__ int order_class(int q)
{
    return ((q + 3) >> 2) + (q >> 4);
}

// One wave per M2L work unit (a box of at most FMM_M2L_HEAVY weak pairs, or
// a segment of FMM_M2L_SEG pairs of a longer list; units t < nb are boxes,
// t - nb indexes the segments).  The wave evaluates the order of each of the
// unit's pairs (features and MLP, the caller's orders, or p), writes it in
// weak-list order (qw) and re-orders the unit's pairs by increasing order
// (stable counting sort with ballots over the unit's range of orders) into sw
// (source) and sp (order), so that the pairs of an M2L chunk have similar
// orders.  The target box's context, including the share denominator over its
// whole weak list, is computed once per unit.
__global__ void __launch_bounds__(256) k_porder(fmm_porder_args a, const float *__restrict__ model)
{
    __shared__ __align__(16) float smodel[FMM2D_PORDER_MODEL_FLOATS];
    // per wave: the unit's sources and orders (lane i keeps entries i, i + 64, ...)
    __shared__ int32_t s_src[256 / WAVE][PORDER_RCH * WAVE];
    __shared__ uint8_t s_q[256 / WAVE][PORDER_RCH * WAVE];
    // the grid covers the capacity in heavy-box segments: a block past the
    // segments in use returns before it loads the model (block-uniform)
    {
        const int64_t t0 = (int64_t)blockIdx.x * (blockDim.x / WAVE);
        if (t0 >= a.nb && t0 - a.nb >= a.hoff[a.nb]) return;
    }
    if (model) {
        for (int k = threadIdx.x; k < FMM2D_PORDER_MODEL_FLOATS; k += blockDim.x) smodel[k] = model[k];
        __syncthreads();
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t t = wave_index();
    int64_t g, bo;
    int l;
    int32_t e0, e1;
    if (!porder_unit(a.woff, a.hoff, a.hbox, a.L, a.nb, a.cap, t, g, l, bo, e0, e1)) return;
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    int32_t *wsrc = s_src[wv];
    uint8_t *wq = s_q[wv];
    feat_ctx c;
    if (a.model) {
        // the whole box's list (a heavy box's segments each sum it, in one order)
        int32_t E0, E1;
        box_range(a.woff, a.L, g, a.cap, l, bo, E0, E1);
        const double den = box_den(a.n1, a.widx, E0, E1, bo, nbl);
        const int64_t so = d_start_off(l) + (g - bo);
        c.centre = a.centre; c.radius = a.radius; c.n1 = a.n1; c.tail = a.tail;
        c.g = g; c.bo = bo; c.l = l; c.L = a.L;
        c.n1root = a.n1[0];
        c.den = den;
        c.nweak = a.woff[so + 1] - a.woff[so];
    }
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
    const int32_t nent = min(e1 - e0, PORDER_RCH * WAVE); // <= FMM_M2L_SEG
    const int32_t kmax = (nent + WAVE - 1) / WAVE;
    bool short_given = false;
#pragma unroll 1
    for (int k = 0; k < kmax; ++k) {
        const int32_t i = k * WAVE + lane;
        wq[i] = 0; // 0 never matches an order
        if (i < nent) {
            const int32_t e = e0 + i;
            const int32_t s = a.widx[e];
            int q = a.p;
            if (a.model) {
                float f[FMM_NF];
                pair_features(c, bo + min(max(s, 0), nbl - 1), f);
                // an opaque zero offset keeps the weights in LDS, read where
                // they are used, instead of hoisted into registers
                uint32_t off = 0;
                asm volatile("" : "+v"(off));
                const float *mw = smodel + off;
                if (in_range(mw, f)) {
                    const float y = mlp_eval(mw, f) + a.delta;
                    const float yc = fminf(fmaxf(y, -1.0e6f), 1.0e6f); // NaN -> -1e6
                    const int qq = (int)ceilf(yc);
                    q = qq < FMM2D_PORDER_QMIN ? FMM2D_PORDER_QMIN : (qq > a.p ? a.p : qq);
                }
            } else if (a.given) {
                if ((int64_t)e < a.ngiven) {
                    const int qq = a.given[e];
                    q = qq < 1 ? 1 : (qq > a.p ? a.p : qq);
                } else {
                    short_given = true;
                }
            }
            a.qw[e] = (uint8_t)q;
            wq[i] = (uint8_t)q;
            wsrc[i] = s;
        }
    }
    if (short_given) atomicOr(a.status, FMM_ST_ORDERS_SHORT);
    // stable sort by the M2L body class of the order (row tiles, k-steps):
    // the classes present as a bit mask, then one pass per class
    uint64_t present = 0;
    for (int k = 0; k < kmax; ++k) {
        const int32_t i = k * WAVE + lane;
        if (i < nent) present |= 1ull << order_class(wq[i]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) present |= __shfl_xor(present, o, WAVE);
    int32_t run = e0;
    while (present) {
        const int cls = __builtin_ctzll(present);
        present &= present - 1;
        for (int k = 0; k < kmax; ++k) {
            const int32_t i = k * WAVE + lane;
            const int q = wq[i];
            const bool hit = i < nent && order_class(q) == cls;
            const uint64_t m = __ballot(hit);
            if (hit) {
                const int32_t dst = run + __popcll(m & lt);
                a.sw[dst] = wsrc[i];
                a.sp[dst] = (uint8_t)q;
            }
            run += __popcll(m);
        }
    }
}

// ------------------------------------------------------------------ labels --
// Label of one weak pair from an evaluation at order P (< 64).  With
// rho = c_T - c_S and c_{l,k} the contribution of a_k to b_l,
//   c_{l,0} = a_0 Log(rho) (l = 0),  (-1)^{l+1} a_0 rho^{-l} / l (l >= 1; LOG only)
//   c_{l,k} = (-1)^l C(k+l-1, l) a_k rho^{-(k+l)}  (k >= 1)
// the pair truncated at q has b_l^(q) = sum_{k<=q} c_{l,k} for l <= q and 0
// above, and
//   e_q = sum_{l=0..P} |b_l^(q) - b_l^(P)| rho_T^l,
// a bound of the truncation error over the disc of radius rho_T about c_T.
// The label is the smallest q in [qmin, qmax] with e_q <= budget(T), else
// qmax.  One wave per pair, lane l handles row l.
__global__ void __launch_bounds__(256) k_labels(const double *__restrict__ centre, const double *__restrict__ radius,
                                                const double2 *__restrict__ A, const double *__restrict__ binom,
                                                const int32_t *__restrict__ woff, const int32_t *__restrict__ widx,
                                                const double *__restrict__ budget, int P, int L, int kernel,
                                                int64_t nb, int32_t cap, int qmin, int qmax, int64_t nlab_cap,
                                                uint8_t *__restrict__ label)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t g = wave_index();
    if (g >= nb) return;
    const int l = level_of_box(g, L);
    const int64_t bo = d_box_off(l), so = d_start_off(l);
    const int32_t b = (int32_t)(g - bo);
    const int32_t e0 = min(woff[so + b], cap), e1 = min(woff[so + b + 1], cap);
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double bud = budget[g];
    const double rT = radius[g];
    const bool LOG = kernel == FMM2D_KERNEL_LOG;
    const int ll = lane;            // row of this lane
    const bool row = ll <= P;
    double rl = 1.0;                // rho_T^l
    for (int q = 0; q < ll && row; ++q) rl *= rT;
    for (int32_t e = e0; e < e1 && e < nlab_cap; ++e) {
        const int64_t gS = bo + min(max(widx[e], 0), nbl - 1);
        const double2 rho = make_double2(centre[2 * g] - centre[2 * gS], centre[2 * g + 1] - centre[2 * gS + 1]);
        const double iq = 1.0 / (rho.x * rho.x + rho.y * rho.y);
        const double2 ri = make_double2(rho.x * iq, -rho.y * iq);
        const double2 *a = A + gS * (P + 1);
        // rho^{-l} and rho^{-(P+l)}
        double2 pl = make_double2(1.0, 0.0);
        for (int q = 0; q < ll && row; ++q) pl = make_double2(pl.x * ri.x - pl.y * ri.y, pl.x * ri.y + pl.y * ri.x);
        double2 pk = pl;
        for (int q = 0; q < P; ++q) pk = make_double2(pk.x * ri.x - pk.y * ri.y, pk.x * ri.y + pk.y * ri.x);
        const double sg = (ll & 1) ? -1.0 : 1.0;
        // c_{l,0}
        double2 c0 = make_double2(0.0, 0.0);
        if (LOG && row) {
            if (ll == 0) {
                const double lr = 0.5 * log(rho.x * rho.x + rho.y * rho.y), ar = atan2(rho.y, rho.x);
                c0 = make_double2(a[0].x * lr - a[0].y * ar, a[0].x * ar + a[0].y * lr);
            } else {
                c0 = make_double2(-sg * (a[0].x * pl.x - a[0].y * pl.y) / ll, -sg * (a[0].x * pl.y + a[0].y * pl.x) / ll);
            }
        }
        // full row b_l^(P): sum over k descending (rho^{-(k+l)} from rho^{-(P+l)} by multiplying with rho)
        double2 full = c0;
        {
            double2 pw = pk;
            for (int k = P; k >= 1; --k) {
                const double cb = row ? sg * binom[(k + ll - 1) * FMM_BN + ll] : 0.0;
                const double2 ak = a[k];
                full.x += cb * (ak.x * pw.x - ak.y * pw.y);
                full.y += cb * (ak.x * pw.y + ak.y * pw.x);
                pw = make_double2(pw.x * rho.x - pw.y * rho.y, pw.x * rho.y + pw.y * rho.x);
            }
        }
        const double absfull = row ? sqrt(full.x * full.x + full.y * full.y) * rl : 0.0;
        // q descending: tail(q) = sum_{k=q+1..P} c_{l,k}
        double2 tl = make_double2(0.0, 0.0);
        double2 pw = pk; // rho^{-(q+l)} for the c_{l,q} added after step q
        int lab = qmax;
        for (int q = P; q >= 0; --q) {
            double term = 0.0;
            if (row) term = (ll <= q) ? sqrt(tl.x * tl.x + tl.y * tl.y) * rl : absfull;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) term += __shfl_xor(term, o, WAVE);
            if (q >= qmin && q <= qmax && term <= bud) lab = q;
            if (q >= 1) {
                const double cb = row ? sg * binom[(q + ll - 1) * FMM_BN + ll] : 0.0;
                const double2 ak = a[q];
                tl.x += cb * (ak.x * pw.x - ak.y * pw.y);
                tl.y += cb * (ak.x * pw.y + ak.y * pw.x);
                pw = make_double2(pw.x * rho.x - pw.y * rho.y, pw.x * rho.y + pw.y * rho.x);
            }
        }
        if (lane == 0) label[e] = (uint8_t)lab;
    }
}

// Budget per box: tol * min over the box's targets of |val| / max(|weak(T)|, 1).
// The minima are formed at the leaves, then up the pyramid (children 4b..4b+3).
__global__ void k_leaf_min(const double *__restrict__ val, const int32_t *__restrict__ tperm,
                           const int32_t *__restrict__ tst, int64_t nleaf, double *__restrict__ vmin)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf) return;
    double m = INFINITY;
    for (int32_t i = tst[t]; i < tst[t + 1]; ++i) {
        const int64_t o = tperm[i];
        m = fmin(m, sqrt(val[2 * o] * val[2 * o] + val[2 * o + 1] * val[2 * o + 1]));
    }
    vmin[t] = m;
}

__global__ void k_parent_min(const double *__restrict__ child, int64_t nparent, double *__restrict__ parent)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nparent) return;
    parent[b] = fmin(fmin(child[4 * b], child[4 * b + 1]), fmin(child[4 * b + 2], child[4 * b + 3]));
}

__global__ void k_budget(const double *__restrict__ vmin, const int32_t *__restrict__ woff, int L, int64_t nb,
                         double tol, double *__restrict__ budget)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb) return;
    const int l = level_of_box(g, L);
    const int64_t b = g - d_box_off(l);
    const int64_t so = d_start_off(l);
    const int32_t nw = woff[so + b + 1] - woff[so + b];
    budget[g] = tol * vmin[g] / (double)(nw > 0 ? nw : 1);
}

// ------------------------------------------------------------------ MLP --
#define MLP_BLOCK 256

// y[i] = MLP(x[i]) (standardisation included).
__global__ void __launch_bounds__(MLP_BLOCK) k_mlp_forward(const float *__restrict__ w, const float *__restrict__ x,
                                                           int64_t n, float *__restrict__ y)
{
    __shared__ __align__(16) float sw[FMM2D_PORDER_MODEL_FLOATS];
    for (int k = threadIdx.x; k < FMM2D_PORDER_MODEL_FLOATS; k += blockDim.x) sw[k] = w[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[FMM_NF];
#pragma unroll
    for (int k = 0; k < FMM_NF; ++k) f[k] = x[i * FMM_NF + k];
    y[i] = mlp_eval(sw, f);
}

// Gradient of the pinball loss (1/n) sum_i rho_tau(q_i - y_i), rho_tau(u) =
// u (tau - [u < 0]), with respect to the 321 trainable parameters, and the
// loss itself.  Each block writes its partial sums (one per parameter, plus
// the loss) to part[block][322]; k_mlp_grad_sum adds them in block order, so
// the result does not depend on scheduling.
__global__ void __launch_bounds__(MLP_BLOCK) k_mlp_grad_part(const float *__restrict__ w, const float *__restrict__ x,
                                                             const float *__restrict__ q, int64_t n, float tau,
                                                             float *__restrict__ part)
{
    __shared__ float sw[FMM2D_PORDER_MODEL_FLOATS];
    __shared__ float red[MLP_BLOCK / WAVE][FMM2D_PORDER_NPARAM + 1];
    for (int k = threadIdx.x; k < FMM2D_PORDER_MODEL_FLOATS; k += blockDim.x) sw[k] = w[k];
    __syncthreads();
    const float *W1 = sw, *b1 = W1 + FMM_HID * FMM_NF, *W2 = b1 + FMM_HID, *b2 = W2 + FMM_HID;
    const float *mu = b2 + 1, *isd = mu + FMM_NF;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    float xs[FMM_NF], h[FMM_HID];
    float y = b2[0];
#pragma unroll
    for (int k = 0; k < FMM_NF; ++k) xs[k] = act ? (x[i * FMM_NF + k] - mu[k]) * isd[k] : 0.0f;
    for (int j = 0; j < FMM_HID; ++j) {
        float z = b1[j];
#pragma unroll
        for (int k = 0; k < FMM_NF; ++k) z = fmaf(W1[j * FMM_NF + k], xs[k], z);
        h[j] = z; // pre-activation
        y = fmaf(W2[j], fmaxf(z, 0.0f), y);
    }
    float gy = 0.0f, loss = 0.0f;
    if (act) {
        const float u = q[i] - y;
        const float s = u >= 0.0f ? tau : tau - 1.0f; // d rho / du
        loss = s * u / (float)n;
        gy = -s / (float)n;                           // d loss / d y
    }
    auto wsum = [&](float v) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
        return v;
    };
    for (int j = 0; j < FMM_HID; ++j) {
        const float gz = h[j] > 0.0f ? gy * W2[j] : 0.0f; // d loss / d z_j
#pragma unroll
        for (int k = 0; k < FMM_NF; ++k) {
            const float v = wsum(gz * xs[k]);
            if (lane == 0) red[wv][j * FMM_NF + k] = v;
        }
        const float vb = wsum(gz);
        const float vw = wsum(gy * fmaxf(h[j], 0.0f));
        if (lane == 0) {
            red[wv][FMM_HID * FMM_NF + j] = vb;
            red[wv][FMM_HID * FMM_NF + FMM_HID + j] = vw;
        }
    }
    {
        const float vb2 = wsum(gy), vl = wsum(loss);
        if (lane == 0) {
            red[wv][FMM2D_PORDER_NPARAM - 1] = vb2;
            red[wv][FMM2D_PORDER_NPARAM] = vl;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= FMM2D_PORDER_NPARAM; k += blockDim.x) {
        float s = 0.0f;
#pragma unroll
        for (int q2 = 0; q2 < MLP_BLOCK / WAVE; ++q2) s += red[q2][k];
        part[(int64_t)blockIdx.x * (FMM2D_PORDER_NPARAM + 1) + k] = s;
    }
}

__global__ void k_mlp_grad_sum(const float *__restrict__ part, int64_t nblk, float *__restrict__ grad,
                               float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > FMM2D_PORDER_NPARAM) return;
    double s = 0.0;
    for (int64_t b = 0; b < nblk; ++b) s += part[b * (FMM2D_PORDER_NPARAM + 1) + k];
    if (k < FMM2D_PORDER_NPARAM) grad[k] = (float)s;
    else if (loss) *loss = (float)s;
}

// Adam (Kingma & Ba), bias-corrected, on the 321 trainable parameters.
__global__ void k_mlp_adam(float *__restrict__ w, const float *__restrict__ grad, float *__restrict__ m,
                           float *__restrict__ v, int step, float lr, float b1, float b2, float eps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= FMM2D_PORDER_NPARAM) return;
    const float gk = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float c1 = 1.0f - (float)pow((double)b1, (double)step);
    const float c2 = 1.0f - (float)pow((double)b2, (double)step);
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ------------------------------------------------------------ launchers --
hipError_t fmm_box_norms(const double2 *A, const double *radius, int p, int64_t nb, double *n1, double *tail,
                         hipStream_t st)
{
    k_box_norms<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(A, radius, p, nb, n1, tail);
    return hipGetLastError();
}

hipError_t fmm_features(const fmm_porder_args &a, int64_t nfeat_cap, float *feat, hipStream_t st)
{
    k_features<<<(unsigned)((a.nb + 3) / 4), 256, 0, st>>>(a.centre, a.radius, a.n1, a.tail, a.woff, a.widx, a.L,
                                                           a.nb, a.cap, nfeat_cap, feat);
    return hipGetLastError();
}

hipError_t fmm_porder(const fmm_porder_args &a, hipStream_t st)
{
    const unsigned nub = (unsigned)((a.nb + a.hmax + 3) / 4); // units: boxes, then heavy-box segments
    k_porder<<<nub, 256, 0, st>>>(a, a.model);
    return hipGetLastError();
}

hipError_t fmm_labels(const fmm_porder_args &a, const double2 *A, const double *binom, const int32_t *tperm,
                      const int32_t *tstart, const double *val, double tol, int P, int kernel, int qmin, int qmax,
                      int64_t nlab_cap, double *vmin, double *budget, uint8_t *label, hipStream_t st)
{
    const int L = a.L;
    const int64_t nleaf = nbox(L);
    k_leaf_min<<<(unsigned)((nleaf + 255) / 256), 256, 0, st>>>(val, tperm, tstart + start_off(L), nleaf,
                                                                 vmin + box_off(L));
    for (int l = L - 1; l >= 0; --l)
        k_parent_min<<<(unsigned)((nbox(l) + 255) / 256), 256, 0, st>>>(vmin + box_off(l + 1), nbox(l),
                                                                         vmin + box_off(l));
    k_budget<<<(unsigned)((a.nb + 255) / 256), 256, 0, st>>>(vmin, a.woff, L, a.nb, tol, budget);
    k_labels<<<(unsigned)((a.nb + 3) / 4), 256, 0, st>>>(a.centre, a.radius, A, binom, a.woff, a.widx, budget, P, L,
                                                         kernel, a.nb, a.cap, qmin, qmax, nlab_cap, label);
    return hipGetLastError();
}

int64_t fmm_mlp_grad_blocks(int64_t n) { return (n + MLP_BLOCK - 1) / MLP_BLOCK; }

hipError_t fmm_mlp_forward(const float *w, const float *x, int64_t n, float *y, hipStream_t st)
{
    if (n > 0) k_mlp_forward<<<(unsigned)((n + MLP_BLOCK - 1) / MLP_BLOCK), MLP_BLOCK, 0, st>>>(w, x, n, y);
    return hipGetLastError();
}

hipError_t fmm_mlp_grad(const float *w, const float *x, const float *q, int64_t n, float tau, float *part,
                        float *grad, float *loss, hipStream_t st)
{
    const int64_t nblk = fmm_mlp_grad_blocks(n);
    if (nblk > 0) k_mlp_grad_part<<<(unsigned)nblk, MLP_BLOCK, 0, st>>>(w, x, q, n, tau, part);
    k_mlp_grad_sum<<<(FMM2D_PORDER_NPARAM + 1 + 127) / 128, 128, 0, st>>>(part, nblk, grad, loss);
    return hipGetLastError();
}

hipError_t fmm_mlp_adam(float *w, const float *grad, float *m, float *v, int step, float lr, float b1, float b2,
                        float eps, hipStream_t st)
{
    k_mlp_adam<<<(FMM2D_PORDER_NPARAM + 127) / 128, 128, 0, st>>>(w, grad, m, v, step, lr, b1, b2, eps);
    return hipGetLastError();
}
