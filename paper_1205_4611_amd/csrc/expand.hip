// Expansion kernels on gfx950: P2M, M2M, M2L and L2L (Goude & Engblom,
// Sec. 2 eqs. (multipole), (local); Sec. 3.3 algorithms "Multipole
// initialization", "Multipole to multipole translation", "Multipole to local
// translation" and "Local to local translation").
//
// Coefficients are complex, [box][p+1], interleaved FP64 (double2).
//   multipole  M(z) = a_0 log(z-c) + sum_{k=1..p} a_k (z-c)^{-k}
//   local      L(z) = sum_{l=0..p} b_l (z-c)^l
//
// M2L is written as diagonal scalings around one fixed real matrix, so that
// all interactions of all levels form one dense batched contraction on the
// matrix cores.  With r = c_S - c_T:
//   beta_{k'} = (-1)^{k'+1} a_{k'+1} r^{-(k'+1)}          k' = 0..p-1
//   B_l       = sum_{k'} S_{l,k'} beta_{k'},  S_{l,k'} = C(l+k', l)
//   b_l      += r^{-l} (B_l - a_0/l)       (l >= 1),   b_0 += B_0 + a_0 Log(c_T - c_S)
// which is the re-expansion of (z-c_S)^{-k} and log(z-c_S) about c_T.  (The
// printed listing of the M2L algorithm has sign slips; this is the operator
// it describes.)  S is the same for every pair, so it is the MFMA A operand
// (read from a table in LDS) while the pre-scaled multipoles stream through the
// B operand: in FP64 (k_m2l64, v_mfma_f64_16x16x4f64) 16 pairs per chunk with
// the real and imaginary parts in two accumulators; in FP32 (k_m2l32, the mixed
// path, S in registers) 8 pairs per chunk as 16 real columns (re/im).
#include <string.h>

#include "common.h"

#define WAVE 64

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 a)
{
    double q = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * q, -a.y * q);
}

// 1/x from the hardware reciprocal and one Newton step (relative error
// ~1e-15, against ~5e-8 for the bare instruction); x > 0 finite.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double2 cinv_fast(double2 a)
{
    const double q = rcp_nr(a.x * a.x + a.y * a.y);
    return make_double2(a.x * q, -a.y * q);
}

// Cross-lane moves inside a row of 16 lanes through DPP (no LDS traffic).
// DPP_XOR1: lanes 2i <-> 2i+1 (quad_perm 1,0,3,2); DPP_XOR2: quad_perm
// 2,3,0,1; DPP_ROR4 / DPP_ROR8: rotate the row right by 4 / 8 lanes.
#define DPP_XOR1 0xB1
#define DPP_XOR2 0x4E
#define DPP_ROR4 0x124
#define DPP_ROR8 0x128
template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Sum over the 8 lanes of a row that share bit 0 of the lane index (the 8
// pairs of an M2L chunk, one component): xor 2, then rotations by 4 and 8.
__device__ __forceinline__ double sum8_64(double v)
{
    v += dpp64<DPP_XOR2>(v);
    v += dpp64<DPP_ROR4>(v);
    v += dpp64<DPP_ROR8>(v);
    return v;
}
// Sum and largest value over the 16 lanes of a row (the 16 pairs of an FP64
// M2L chunk): xor 1, xor 2, then rotations by 4 and 8.
__device__ __forceinline__ double sum16_64(double v)
{
    v += dpp64<DPP_XOR1>(v);
    v += dpp64<DPP_XOR2>(v);
    v += dpp64<DPP_ROR4>(v);
    v += dpp64<DPP_ROR8>(v);
    return v;
}
__device__ __forceinline__ int max16_i(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_XOR1, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_XOR2, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROR4, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROR8, 0xF, 0xF, false));
    return v;
}
// Largest value over the same 8 lanes (the pairs of a chunk).
__device__ __forceinline__ int max8_i(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_XOR2, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROR4, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, DPP_ROR8, 0xF, 0xF, false));
    return v;
}
__device__ __forceinline__ float sum8_32(float v)
{
    v += dpp32<DPP_XOR2>(v);
    v += dpp32<DPP_ROR4>(v);
    v += dpp32<DPP_ROR8>(v);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Lane layout of the leaf kernels (P2M, P2L): lane = 16 g + r, r a source
// slot, g a group of P2_KG consecutive expansion terms k = P2_KG g + t.  A lane
// takes the sources r, r + 16, ... and the terms of its group, so the sum over
// sources is a reduction over the 16 lanes of a DPP row.
template <int PM>
struct p2_groups {
    static constexpr int KG = (PM + 4) / 4; // 4 groups cover k = 0..PM
};

// z^E for a compile-time E by squaring
template <int E>
__device__ __forceinline__ double2 cpow_ct(double2 z)
{
    if constexpr (E == 0) {
        return make_double2(1.0, 0.0);
    } else if constexpr (E == 1) {
        return z;
    } else if constexpr ((E & 1) == 0) {
        const double2 h = cpow_ct<E / 2>(z);
        return cmul(h, h);
    } else {
        return cmul(z, cpow_ct<E - 1>(z));
    }
}
// zK^g for the lane's group g in 0..3
__device__ __forceinline__ double2 group_power(double2 zK, int g)
{
    const double2 z2 = cmul(zK, zK), z3 = cmul(z2, zK);
    return g == 0 ? make_double2(1.0, 0.0) : (g == 1 ? zK : (g == 2 ? z2 : z3));
}

// ------------------------------------------------------------------ P2M --
// One wave per leaf (a wave takes leaves w, w + waves of the grid, ...): s_k =
// sum m (x-c)^k, then
//   LOG:      a_0 = s_0, a_k = -s_k / k
//   HARMONIC: a_0 = 0,   a_k = s_{k-1}
template <int PM>
__global__ void __launch_bounds__(256) k_p2m(const double4 *__restrict__ srcs,
                                              const int32_t *__restrict__ sst,
                                              const double *__restrict__ centre,
                                              double2 *__restrict__ A, int p, int kernel,
                                              int32_t nleaf)
{
    constexpr int KG = p2_groups<PM>::KG;
    const int lane = threadIdx.x & (WAVE - 1);
    const int r = lane & 15, g = lane >> 4, kb = KG * g;
    const int32_t nwv = (int32_t)(gridDim.x * (blockDim.x / WAVE));
    for (int32_t b = wave_index(); b < nleaf; b += nwv) {
        const int32_t s0 = sst[b], s1 = sst[b + 1];
        const double cx = centre[2 * (int64_t)b], cy = centre[2 * (int64_t)b + 1];
        double sr[KG], si[KG];
#pragma unroll
        for (int t = 0; t < KG; ++t) { sr[t] = 0.0; si[t] = 0.0; }
        for (int32_t j = s0 + r; j < s1; j += 16) {
            const double4 d = srcs[j];
            const double2 w = make_double2(d.x - cx, d.y - cy);
            double2 pw = cmul(make_double2(d.z, d.w), group_power(cpow_ct<KG>(w), g));
#pragma unroll
            for (int t = 0; t < KG; ++t) {
                sr[t] += pw.x;
                si[t] += pw.y;
                if (t + 1 < KG) pw = cmul(pw, w);
            }
        }
        double2 *out = A + (int64_t)b * (p + 1);
#pragma unroll
        for (int t = 0; t < KG; ++t) {
            const double re = sum16_64(sr[t]), im = sum16_64(si[t]);
            const int k = kb + t;
            if (r == 0 && k <= p) {
                if (kernel == FMM2D_KERNEL_LOG) {
                    out[k] = (k == 0) ? make_double2(re, im) : make_double2(-re / k, -im / k);
                } else {
                    if (k < p) out[k + 1] = make_double2(re, im);
                    if (k == 0) out[0] = make_double2(0.0, 0.0);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ P2L --
// Leaf-level swapped criterion: sources of a larger box, outside the target
// leaf's disc, go straight into its local expansion (added after L2L).  With
// d = x - c and u = 1/d:
//   LOG:      b_0 += sum m Log(c - x),   b_l -= (sum m u^l) / l   (l >= 1)
//   HARMONIC: b_l -= sum m u^{l+1}                               (l >= 0)
// One wave per target leaf; the list entries are read once, up to 64 at a
// time.  Lane = 32 g + r: source slot r (sources r, r + 32, ...) and the
// terms k = g, g + 2, ... of parity g, so a lane starts at m u^g (LOG) or
// m u^(g+1) and steps by u^2; the sum over sources is a reduction over the 32
// lanes of its half.  The Log term of the log kernel is summed by all 64
// lanes apart.
template <int PM>
struct p2l_terms {
    static constexpr int KT = (PM + 2) / 2; // terms of parity 0 cover k = 0..PM
};
__device__ __forceinline__ double sum32_64(double v)
{
    v = sum16_64(v);
    return v + __shfl_xor(v, 16, WAVE);
}

template <int PM, bool LOG>
__global__ void __launch_bounds__(256) k_p2l(const double4 *__restrict__ srcs,
                                              const int32_t *__restrict__ sst,
                                              const int32_t *__restrict__ poff,
                                              const int32_t *__restrict__ pidx,
                                              const double *__restrict__ centre,
                                              double2 *__restrict__ B, int p, int32_t nleaf, int32_t lcap)
{
    constexpr int KT = p2l_terms<PM>::KT;
    const int lane = threadIdx.x & (WAVE - 1);
    const int r = lane & 31, g = lane >> 5;
    const int32_t t = wave_index();
    if (t >= nleaf) return;
    const int32_t e0 = min(poff[t], lcap), e1 = min(poff[t + 1], lcap);
    if (e0 >= e1) return;
    const double cx = centre[2 * (int64_t)t], cy = centre[2 * (int64_t)t + 1];
    double sr[KT], si[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) { sr[q] = 0.0; si[q] = 0.0; }
    double2 lg0 = make_double2(0.0, 0.0);
    for (int32_t ec = e0; ec < e1; ec += WAVE) {
        // this batch's source leaves and their ranges
        int32_t mj0 = 0, mj1 = 0;
        if (ec + lane < e1) {
            const int32_t s = min(max(pidx[ec + lane], 0), nleaf - 1);
            mj0 = sst[s];
            mj1 = sst[s + 1];
        }
        const int32_t ne = min(e1 - ec, WAVE);
        for (int32_t q = 0; q < ne; ++q) {
            const int32_t j0 = __builtin_amdgcn_readlane(mj0, q), j1 = __builtin_amdgcn_readlane(mj1, q);
            for (int32_t j = j0 + r; j < j1; j += 32) {
                const double4 d = srcs[j];
                const double2 u = cinv_fast(make_double2(d.x - cx, d.y - cy));
                const double2 u2 = cmul(u, u);
                // m u^g (LOG) or m u^(g+1)
                const double2 m = make_double2(d.z, d.w);
                const double2 mu = cmul(m, u);
                double2 pw = LOG ? (g ? mu : m) : (g ? cmul(mu, u) : mu);
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    sr[k] += pw.x;
                    si[k] += pw.y;
                    if (k + 1 < KT) pw = cmul(pw, u2);
                }
            }
            if (LOG) {
                for (int32_t j = j0 + lane; j < j1; j += WAVE) {
                    const double4 d = srcs[j];
                    const double lx = cx - d.x, ly = cy - d.y; // Log(c - x), formed as written
                    const double2 lg = make_double2(0.5 * log(lx * lx + ly * ly), atan2(ly, lx));
                    const double2 t0 = cmul(make_double2(d.z, d.w), lg);
                    lg0.x += t0.x;
                    lg0.y += t0.y;
                }
            }
        }
    }
    double2 *out = B + (int64_t)t * (p + 1);
    if (LOG) {
        lg0.x = wave_sum(lg0.x);
        lg0.y = wave_sum(lg0.y);
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) {
        const double re = sum32_64(sr[q]), im = sum32_64(si[q]);
        const int k = g + 2 * q;
        if (r == 0 && k <= p) {
            double2 o = out[k];
            if (LOG) {
                if (k == 0) {
                    o.x += lg0.x;
                    o.y += lg0.y;
                } else {
                    o.x -= re / k;
                    o.y -= im / k;
                }
            } else {
                o.x -= re;
                o.y -= im;
            }
            out[k] = o;
        }
    }
}

// ------------------------------------------------------------------ M2M --
// Thread per (parent, coefficient l), grid-stride: a'_l = sum over the 4
// children of -a_0 r^l / l + sum_{k=1..l} C(l-1,k-1) a_k r^{l-k},
// r = c_child - c_parent.
__global__ void k_m2m(const double *__restrict__ centre, double2 *__restrict__ A,
                      const double *__restrict__ binom, int p, int l, int64_t nbl)
{
    const int P1 = p + 1;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nbl * P1;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / P1;
        const int lc = (int)(t - b * P1);
        const int64_t g = d_box_off(l) + b;
        const double2 cp = make_double2(centre[2 * g], centre[2 * g + 1]);
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < 4; ++q) {
            const int64_t c = d_box_off(l + 1) + 4 * b + q;
            const double2 r = make_double2(centre[2 * c] - cp.x, centre[2 * c + 1] - cp.y);
            const double2 *a = A + c * P1;
            if (lc == 0) {
                acc.x += a[0].x;
                acc.y += a[0].y;
            } else {
                double2 s = make_double2(0.0, 0.0), pw = make_double2(1.0, 0.0);
                for (int k = lc; k >= 1; --k) {
                    const double cb = binom[(lc - 1) * FMM_BN + (k - 1)];
                    const double2 ak = a[k];
                    const double2 tk = cmul(ak, pw);
                    s.x += cb * tk.x;
                    s.y += cb * tk.y;
                    pw = cmul(pw, r);
                }
                const double2 a0 = cmul(a[0], pw); // a_0 r^l
                s.x -= a0.x / lc;
                s.y -= a0.y / lc;
                acc.x += s.x;
                acc.y += s.y;
            }
        }
        A[g * P1 + lc] = acc;
    }
}

// ------------------------------------------------------------------ L2L --
// Thread per (child, coefficient l): b'_l += sum_{j=l..p} C(j,l) b_j r^{j-l},
// r = c_child - c_parent.
__global__ void k_l2l(const double *__restrict__ centre, double2 *__restrict__ B,
                      const double *__restrict__ binom, int p, int l, int64_t nbl)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P1 = p + 1;
    if (t >= nbl * P1) return;
    const int64_t b = t / P1;
    const int lc = (int)(t - b * P1);
    const int64_t g = d_box_off(l) + b;
    const int64_t q = d_box_off(l - 1) + b / 4;
    const double2 r = make_double2(centre[2 * g] - centre[2 * q], centre[2 * g + 1] - centre[2 * q + 1]);
    const double2 *bp = B + q * P1;
    double2 s = make_double2(0.0, 0.0), pw = make_double2(1.0, 0.0);
    for (int j = lc; j <= p; ++j) {
        const double cb = binom[j * FMM_BN + lc];
        const double2 tj = cmul(bp[j], pw);
        s.x += cb * tj.x;
        s.y += cb * tj.y;
        pw = cmul(pw, r);
    }
    double2 o = B[g * P1 + lc];
    o.x += s.x;
    o.y += s.y;
    B[g * P1 + lc] = o;
}

// ------------------------------------------------------------------ M2L --
struct m2l_args {
    const double *centre;   // [nb][2]
    const double *radius;   // [nb]
    const double2 *A;       // FP64 multipoles (plain path, and a_0 for both)
    const float2 *A32;      // radius-scaled FP32 multipoles (mixed path)
    double2 *B;             // output, written (not accumulated)
    const int32_t *woff;    // per-level offsets
    const int32_t *widx;    // global weak list
    const int32_t *sw;      // per-pair orders: sources sorted by order within a box, or NULL
    const uint8_t *sp;      //   and their orders (ascending within a box)
    const double *binom;
    int64_t nb;
    int L, p, kernel;
    int32_t cap;
    // boxes with more than M2L_HEAVY weak pairs are cut into segments of
    // M2L_SEG pairs: hoff[g] = first segment of box g (exclusive scan, total
    // at hoff[nb]), hbox[s] = box of segment s, hpart[s][p+1] its partial sum
    const int32_t *hoff, *hbox;
    double2 *hpart;
};

__device__ __forceinline__ int level_of(int64_t g, int L)
{
    int l = 0;
    while (l < L && d_box_off(l + 1) <= g) ++l;
    return l;
}

__device__ __forceinline__ double2 clog_principal(double2 z)
{
    return make_double2(0.5 * log(z.x * z.x + z.y * z.y), atan2(z.y, z.x));
}

#define M2L_HEAVY FMM_M2L_HEAVY // boxes with more weak pairs are cut into segments
#define M2L_SEG FMM_M2L_SEG     // pairs per segment (one workgroup each)
#define M2L_WAVES 4

__device__ __forceinline__ int32_t m2l_range(const m2l_args &a, int64_t g, int &l, int32_t &e0, int32_t &e1)
{
    l = level_of(g, a.L);
    const int32_t b = (int32_t)(g - d_box_off(l));
    const int64_t so = d_start_off(l);
    e0 = min(a.woff[so + b], a.cap);
    e1 = min(a.woff[so + b + 1], a.cap);
    return e1 - e0;
}

// Radius used to scale the FP32 coefficients: the box radius, floored.
__device__ __forceinline__ double scale_radius(double rho, double rmin)
{
    return rho > rmin ? rho : rmin;
}
// Scaling radius floor: 2^-40 of the root radius (boxes of coincident points
// have radius 0; any positive scale is exact in exact arithmetic).
__device__ __forceinline__ double scale_floor(const double *radius)
{
    return fmax(radius[0] * 0x1p-40, 1e-300);
}

// Operands of one chunk of 8 pairs as this lane needs them, fetched one chunk
// ahead of its use (the list entry two chunks ahead) so that the loads of the
// next chunk overlap the contraction of the current one.
template <int KS, typename C2>
struct m2l_chunk {
    double2 cS;       // source centre
    C2 ak[KS];        // a_k (or ahat_k), k = 4 ks + kq + 1
    double2 a0;       // a_0 (log kernel)
    double sS;        // source scaling radius (FP32 path)
    int q, qc;        // this pair's order, the chunk's largest order
    bool valid;
};

template <int KS, bool LOG, bool F32, typename C2>
__device__ __forceinline__ void m2l_fetch(const m2l_args &a, int64_t bo, int32_t nbl, int32_t e, int32_t e1,
                                          int32_t sbraw, int ps, int kq, double rmin, m2l_chunk<KS, C2> &c)
{
    const int p = a.p, P1 = p + 1;
    const int32_t pe = e + ps;
    c.valid = pe < e1;
    const int32_t sb = min(max(c.valid ? sbraw : 0, 0), nbl - 1);
    const int64_t gS = bo + sb;
    c.cS = make_double2(a.centre[2 * gS], a.centre[2 * gS + 1]);
    c.q = p;
    c.qc = p;
    if (a.sp) {
        c.q = c.valid ? (int)a.sp[pe] : 0;
        // the chunk's largest order bounds its k-steps and row tiles
        c.qc = __builtin_amdgcn_readfirstlane(max8_i(c.q));
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int kk = 4 * ks + kq + 1;
        if (F32) {
            const float2 *As = a.A32 + gS * P1;
            const float2 v = (c.valid && kk <= p) ? As[kk] : make_float2(0.0f, 0.0f);
            c.ak[ks] = *reinterpret_cast<const C2 *>(&v);
        } else {
            const double2 *As = a.A + gS * P1;
            const double2 v = (c.valid && kk <= p) ? As[kk] : make_double2(0.0, 0.0);
            c.ak[ks] = *reinterpret_cast<const C2 *>(&v);
        }
    }
    c.a0 = (LOG && c.valid) ? a.A[gS * P1] : make_double2(0.0, 0.0);
    c.sS = F32 ? scale_radius(a.radius[gS], rmin) : 0.0;
}

// Operands of one chunk of 16 weak pairs for the FP64 contraction: lane
// (pr, kq) = (lane % 16, lane / 16) holds pair pr's source centre and its
// coefficients a_k, k = 4 ks + kq + 1, as full complex numbers; terms above
// the pair's order q are loaded as zero.
template <int KS>
struct m2l_chunk16 {
    double2 cS;
    double2 ak[KS];
    double2 a0; // a_0 (log kernel)
    int q, qc;  // this pair's order, the chunk's largest order
    bool valid;
};

// In two steps, so that no load of a chunk waits for another: m2l_issue16
// issues every load (all coefficients up to p at a clamped index, the pair's
// order); m2l_finish16 takes the orders and zeroes the terms above each
// pair's order.  (Loading the next chunk during the current one's
// contraction cost a wave per SIMD and was slower.)
template <int KS, bool LOG>
__device__ __forceinline__ void m2l_issue16(const m2l_args &a, int64_t bo, int32_t nbl, int32_t e, int32_t e1,
                                            int32_t sbraw, int pr, int kq, m2l_chunk16<KS> &c)
{
    const int p = a.p, P1 = p + 1;
    const int32_t pe = e + pr;
    c.valid = pe < e1;
    const int32_t sb = min(max(c.valid ? sbraw : 0, 0), nbl - 1);
    const int64_t gS = bo + sb;
    c.cS = make_double2(a.centre[2 * gS], a.centre[2 * gS + 1]);
    c.q = (a.sp && c.valid) ? (int)a.sp[pe] : p; // (the raw order; finished below)
    const double2 *As = a.A + gS * P1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) c.ak[ks] = As[min(4 * ks + kq + 1, p)];
    c.a0 = LOG ? As[0] : make_double2(0.0, 0.0);
}
template <int KS, bool LOG>
__device__ __forceinline__ void m2l_finish16(const m2l_args &a, int kq, m2l_chunk16<KS> &c)
{
    c.q = c.valid ? c.q : -1;
    // the chunk's largest order bounds its k-steps and row tiles
    c.qc = a.sp ? __builtin_amdgcn_readfirstlane(max16_i(c.q)) : a.p;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
        if (4 * ks + kq + 1 > c.q) c.ak[ks] = make_double2(0.0, 0.0);
    if (!c.valid) c.a0 = make_double2(0.0, 0.0);
}

// Rows 16 mt + 4 j + kq of an accumulator element exist only up to p <= 4 KS
// (the instance's k-steps bound the order): in the shapes of up to two row
// tiles the elements of higher rows are neither post-scaled, summed nor
// written (in the 5-tile shape of p <= 64 skipping them raised the spills).
template <int MT, int KS>
__host__ __device__ constexpr bool m2l_row_live(int mt, int j)
{
    return MT > 2 || 16 * mt + 4 * j <= 4 * KS;
}

// One chunk of 16 weak pairs in FP64 with MTN row tiles and KSN k-steps
// (the chunk's largest order qc needs rows 0..qc and a_1..a_qc).  Lane layout
// of v_mfma_f64_16x16x4f64: A operand lane i holds A[i%16][i/16], B operand
// lane i holds B[i/16][i%16], accumulator element j of lane i holds row
// 4j + i/16 of column i%16.  Columns are pairs; the real and imaginary parts
// of the scaled coefficients go through two accumulators, so every lane holds
// whole complex numbers of its pair and needs no lane exchange before the
// post-scaling.  Straight-line code for each (MTN, KSN): the accumulators are
// never merged across skipped products.
struct m2l_no_hook {
    __device__ void operator()() const {}
};
template <int MT, int KS, int MTN, int KSN, bool LOG, typename HOOK = m2l_no_hook>
__device__ __forceinline__ void m2l64_chunk(const double *Sl, const double *Il, const m2l_chunk16<KS> &c,
                                            double2 cT, int kq, double (&re)[MT][4], double (&im)[MT][4],
                                            HOOK hook = HOOK())
{
    const int qlim = c.q; // rows above the pair's order are dropped (-1: no pair)
    const double2 r = make_double2(c.cS.x - cT.x, c.cS.y - cT.y);
    const double2 r1 = c.valid ? cinv_fast(r) : make_double2(0.0, 0.0);
    const double2 r2 = cmul(r1, r1), r3 = cmul(r2, r1), r4 = cmul(r2, r2);
    // Pre-scale: beta_{k'} = (-1)^{k'+1} a_{k'+1} r^{-(k'+1)}, k' = 4 ks + kq;
    // the power advances by r^-4 per k-step (an even power: no sign change).
    const double2 p0 = kq == 0 ? r1 : (kq == 1 ? r2 : (kq == 2 ? r3 : r4)); // r^{-(kq+1)}
    const double sg = (kq & 1) ? 1.0 : -1.0;                                // (-1)^{kq+1}
    double2 W = make_double2(sg * p0.x, sg * p0.y);
    double bre[KSN], bim[KSN];
#pragma unroll
    for (int ks = 0; ks < KSN; ++ks) {
        const double2 ak = c.ak[ks];
        bre[ks] = fma(-ak.y, W.y, ak.x * W.x);
        bim[ks] = fma(ak.y, W.x, ak.x * W.y);
        if (ks + 1 < KSN) W = cmul(W, r4);
    }
    dbl4 Cr[MTN], Ci[MTN];
#pragma unroll
    for (int mt = 0; mt < MTN; ++mt) {
        const double sv = Sl[16 * mt * (4 * KS)];
        Cr[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv, bre[0], dbl4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
        Ci[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv, bim[0], dbl4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
    }
#pragma unroll
    for (int ks = 1; ks < KSN; ++ks)
#pragma unroll
        for (int mt = 0; mt < MTN; ++mt) {
            const double sv = Sl[16 * mt * (4 * KS) + 4 * ks];
            Cr[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv, bre[ks], Cr[mt], 0, 0, 0);
            Ci[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv, bim[ks], Ci[mt], 0, 0, 0);
        }
    // the products are issued: the hook (the next chunk's loads) runs while
    // they complete, in the registers of the operands no longer needed
    hook();
    // Post-scale: row l = 16 mt + 4 j + kq gets r^{-l} (B_l - a_0/l); the
    // power starts at r^{-kq} and advances by r^-4 per row, r^-16 per tile.
    double2 u = kq == 0 ? make_double2(1.0, 0.0) : (kq == 1 ? r1 : (kq == 2 ? r2 : r3)); // r^{-kq}
#pragma unroll
    for (int mt = 0; mt < MTN; ++mt) {
        double2 v = u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!m2l_row_live<MT, KS>(mt, j)) continue;
            const int row = 16 * mt + 4 * j + kq;
            double cr = Cr[mt][j], ci = Ci[mt][j];
            if (LOG) {
                const double il = Il[16 * mt + 4 * j]; // 1/l (0 for l = 0)
                cr = fma(-c.a0.x, il, cr);
                ci = fma(-c.a0.y, il, ci);
            }
            const double f = (row <= qlim) ? 1.0 : 0.0;
            re[mt][j] = fma(f, fma(-ci, v.y, cr * v.x), re[mt][j]);
            im[mt][j] = fma(f, fma(ci, v.x, cr * v.y), im[mt][j]);
            if (j < 3) v = cmul(v, r4);
        }
        if (mt + 1 < MTN) u = cmul(u, cmul(cmul(r4, r4), cmul(r4, r4)));
    }
    if (LOG && c.valid && kq == 0) {
        // Log(c_T - c_S), the difference formed as written: on the branch
        // cut the sign of a zero imaginary part decides between +pi and -pi
        const double2 lg = clog_principal(make_double2(cT.x - c.cS.x, cT.y - c.cS.y));
        const double2 t = cmul(c.a0, lg);
        re[0][0] += t.x;
        im[0][0] += t.y;
    }
}

// Chooses the straight-line body for the chunk's (mtn, ksn): the full one
// first (fixed orders), then the combinations a largest order can give
// (mtn tiles need 4 (mtn - 1) <= ksn <= 4 mtn k-steps).  The full body is
// correct for every chunk (terms above a pair's order are zero or masked),
// so it is also the fallback.
template <int MT, int KS, bool LOG, int MTN, int KSN>
__device__ __forceinline__ void m2l64_pick(int mtn, int ksn, const double *Sl, const double *Il,
                                           const m2l_chunk16<KS> &c, double2 cT, int kq, double (&re)[MT][4],
                                           double (&im)[MT][4])
{
    constexpr bool legal = KSN >= (MTN > 1 ? 4 * (MTN - 1) : 1) && KSN <= 4 * MTN;
    if constexpr (MTN == 0) {
        m2l64_chunk<MT, KS, MT, KS, LOG>(Sl, Il, c, cT, kq, re, im);
    } else if constexpr (!legal || (MTN == MT && KSN == KS)) {
        if constexpr (KSN > 1) m2l64_pick<MT, KS, LOG, MTN, KSN - 1>(mtn, ksn, Sl, Il, c, cT, kq, re, im);
        else m2l64_pick<MT, KS, LOG, MTN - 1, KS>(mtn, ksn, Sl, Il, c, cT, kq, re, im);
    } else {
        if (mtn == MTN && ksn == KSN) {
            m2l64_chunk<MT, KS, MTN, KSN, LOG>(Sl, Il, c, cT, kq, re, im);
        } else if constexpr (KSN > 1) {
            m2l64_pick<MT, KS, LOG, MTN, KSN - 1>(mtn, ksn, Sl, Il, c, cT, kq, re, im);
        } else {
            m2l64_pick<MT, KS, LOG, MTN - 1, KS>(mtn, ksn, Sl, Il, c, cT, kq, re, im);
        }
    }
}

// FP64 contraction for the chunks c = w, w + nw, ... of 16 weak pairs of box
// g.  On return (re, im)[mt][j] hold b_l, l = 16 mt + 4 j + kq, summed over
// the chunks' pairs (lane kq = lane / 16).
template <int MT, int KS, bool LOG>
__device__ __forceinline__ void m2l64_acc(const m2l_args &a, const double *Sop, int64_t g, int l, int32_t e0,
                                          int32_t e1, int w, int nw, double (&re)[MT][4], double (&im)[MT][4])
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t bo = d_box_off(l);
    const int pr = lane & 15, kq = lane >> 4;
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double2 cT = make_double2(a.centre[2 * g], a.centre[2 * g + 1]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            re[mt][j] = 0.0;
            im[mt][j] = 0.0;
        }
    // this lane's A operands S[16 mt + pr][4 ks + kq] and 1/l for its rows,
    // read from the block's tables
    const double *Sl = Sop + pr * (4 * KS) + kq;
    const double *Il = Sop + MT * 16 * 4 * KS + kq;
    const int32_t *wl = a.sw ? a.sw : a.widx;
    const int32_t step = 16 * nw;
    int32_t e = e0 + 16 * w;
    // the shapes of p <= 20 hold the next chunk's operands without spills
    constexpr bool PIPE = MT <= 2 && KS <= 5;
    if (PIPE && e < e1 && !a.sp) {
        // fixed order: every chunk takes the full body, and the next chunk's
        // loads are issued once this chunk's products are (m2l64_chunk's hook)
        int32_t sb1 = (e + step + pr < e1) ? wl[e + step + pr] : 0;
        m2l_chunk16<KS> cur, nxt;
        m2l_issue16<KS, LOG>(a, bo, nbl, e, e1, (e + pr < e1) ? wl[e + pr] : 0, pr, kq, cur);
        int32_t sb0 = sb1;
        sb1 = (e + 2 * step + pr < e1) ? wl[e + 2 * step + pr] : 0;
        m2l_finish16<KS, LOG>(a, kq, cur);
        for (; e < e1; e += step) {
            const int32_t en = e + step;
            const bool more = en < e1;
            m2l64_chunk<MT, KS, MT, KS, LOG>(Sl, Il, cur, cT, kq, re, im, [&]() {
                if (more) {
                    m2l_issue16<KS, LOG>(a, bo, nbl, en, e1, sb0, pr, kq, nxt);
                    sb0 = sb1;
                    sb1 = (en + 2 * step + pr < e1) ? wl[en + 2 * step + pr] : 0;
                }
            });
            if (more) {
                m2l_finish16<KS, LOG>(a, kq, nxt);
                cur = nxt;
            }
        }
    } else if (e < e1) {
        int32_t sb1 = (e + step + pr < e1) ? wl[e + step + pr] : 0;
        int32_t sb0 = (e + pr < e1) ? wl[e + pr] : 0;
        for (; e < e1; e += step) {
            m2l_chunk16<KS> cur;
            m2l_issue16<KS, LOG>(a, bo, nbl, e, e1, sb0, pr, kq, cur);
            sb0 = sb1;
            sb1 = (e + 2 * step + pr < e1) ? wl[e + 2 * step + pr] : 0;
            m2l_finish16<KS, LOG>(a, kq, cur);
            const int ksn = min(max((cur.qc + 3) >> 2, 1), KS), mtn = min((cur.qc >> 4) + 1, MT);
            m2l64_pick<MT, KS, LOG, MT, KS>(mtn, ksn, Sl, Il, cur, cT, kq, re, im);
        }
    }
    // sum over the 16 pairs of a tile (lane bits 0..3)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (m2l_row_live<MT, KS>(mt, j)) {
                re[mt][j] = sum16_64(re[mt][j]);
                im[mt][j] = sum16_64(im[mt][j]);
            }
}

// Waves per SIMD the register budget is sized for: three where the body fits
// in 168 VGPRs without spills (row tiles and k-steps of p <= 20, harmonic
// kernel), two (256 VGPRs) otherwise.  Workgroups are M2L_WAVES = 4 waves,
// one per SIMD, so that the groups resident on a CU reach that number (with
// 8-wave groups, 2 waves per SIMD each, a CU held one group at 168 VGPRs).
template <int MT, int KS, bool LOG>
constexpr int m2l_waves_per_simd()
{
    return (MT <= 2 && KS <= 5 && !LOG) ? 3 : 2;
}

// One launch: blocks [0, H) take the boxes with more than M2L_HEAVY weak pairs
// (M2L_WAVES waves per box, fixed-order LDS reduction); the other blocks take
// the light boxes, one wave per box.
template <int MT, int KS, bool LOG>
__global__ void __launch_bounds__(64 * M2L_WAVES) __attribute__((amdgpu_waves_per_eu(m2l_waves_per_simd<MT, KS, LOG>())))
k_m2l64(m2l_args a, int32_t H)
{
    __shared__ double part[M2L_WAVES][MT * 16][2];
    // S_{l,k} = C(l + k, l) for rows l < 16 MT, k < 4 KS (zero beyond p, and
    // for k = p: the highest coefficient a_{k+1} does not exist)
    // followed by 1/l for the rows (the a_0 term of the log kernel)
    __shared__ double Sop[MT * 16 * 4 * KS + MT * 16];
    for (int t = threadIdx.x; t < MT * 16 * 4 * KS; t += blockDim.x) {
        const int row = t / (4 * KS), kk = t % (4 * KS);
        Sop[t] = (row <= a.p && kk < a.p) ? a.binom[(row + kk) * FMM_BN + row] : 0.0;
    }
    for (int t = threadIdx.x; t < MT * 16; t += blockDim.x) Sop[MT * 16 * 4 * KS + t] = t ? 1.0 / t : 0.0;
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int pr = lane & 15, kq = lane >> 4;
    const int P1 = a.p + 1;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const bool light = (int32_t)blockIdx.x >= H;
    const int32_t nseg = light ? 0 : a.hoff[a.nb];
    // light blocks: one box per wave, one pass; heavy blocks: segments of the
    // heavy boxes (partial sums to hpart), blockIdx.x, + H, ...
    for (int32_t sg = blockIdx.x;; sg += H) {
        int64_t g;
        int l, ww = 0, nw = 1;
        int32_t e0, e1;
        if (light) {
            g = (int64_t)xcd_order((int32_t)blockIdx.x, H, (int32_t)gridDim.x) * M2L_WAVES + w;
            if (g >= a.nb) return;
            if (m2l_range(a, g, l, e0, e1) > M2L_HEAVY) return;
        } else {
            if (sg >= nseg) return; // uniform over the block
            g = a.hbox[sg];
            m2l_range(a, g, l, e0, e1);
            const int32_t s0 = min(e0 + (sg - a.hoff[g]) * M2L_SEG, e1);
            e1 = min(s0 + M2L_SEG, e1);
            e0 = s0;
            ww = w;
            nw = M2L_WAVES;
        }
        double re[MT][4], im[MT][4];
        m2l64_acc<MT, KS, LOG>(a, Sop, g, l, e0, e1, ww, nw, re, im);
        if (light) {
            double2 *Bt = a.B + g * P1;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * j + kq;
                    if (m2l_row_live<MT, KS>(mt, j) && pr == 0 && row <= a.p)
                        Bt[row] = make_double2(re[mt][j], im[mt][j]);
                }
            return;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (m2l_row_live<MT, KS>(mt, j) && pr == 0) {
                    part[w][16 * mt + 4 * j + kq][0] = re[mt][j];
                    part[w][16 * mt + 4 * j + kq][1] = im[mt][j];
                }
        __syncthreads();
        if (w == 0) {
            double2 *Bt = a.hpart + (int64_t)sg * P1;
            for (int k = lane; k < 2 * P1; k += WAVE) {
                double v = 0.0;
                for (int q = 0; q < M2L_WAVES; ++q) v += part[q][k >> 1][k & 1];
                reinterpret_cast<double *>(Bt)[k] = v;
            }
        }
        __syncthreads();
    }
}

// Accumulator layout of v_mfma_f32_16x16x4f32: element j of lane i holds row
// 4 (i/16) + j of column i%16.  acc0 collects the FP64 a_0 Log term of row 0.
// FP32 (mixed precision): the same contraction with radius-scaled
// coefficients.  With sigma_S, sigma_T the box radii, ahat_k = a_k /
// sigma_S^k, u = sigma_S / r and v = sigma_T / r:
//   beta_{k'} = (-1)^{k'+1} ahat_{k'+1} u^{k'+1},
//   bhat_l    = v^l (B_l - a_0/l),   b_l = bhat_l / sigma_T^l.
// The theta-criterion keeps |u|, |v| <= theta/(1+theta) < 1, so every scaled
// quantity stays O(1) in FP32.  Log(c_T - c_S) and the final unscaling are FP64.
template <int MT, int KS, bool LOG>
__device__ __forceinline__ void m2l32_acc(const m2l_args &a, int64_t g, int l, int32_t e0, int32_t e1, int w,
                                          int nw, float (&acc)[MT][4], double &acc0)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t bo = d_box_off(l);
    const int p = a.p;
    const int col = lane & 15, ps = col >> 1, comp = col & 1, kq = lane >> 4;
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double2 cT = make_double2(a.centre[2 * g], a.centre[2 * g + 1]);
    const double rmin = scale_floor(a.radius);
    const double sT = scale_radius(a.radius[g], rmin);
    float Sop[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int row = 16 * mt + col, kk = 4 * ks + kq;
            Sop[mt][ks] = (row <= p && kk < p) ? (float)a.binom[(row + kk) * FMM_BN + row] : 0.0f;
        }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mt][j] = 0.0f;
    acc0 = 0.0;
    float irow[MT][4]; // 1/l for the a_0 term (log kernel); rows 16 mt + 4 kq + j
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * mt + 4 * kq + j;
            irow[mt][j] = (LOG && row >= 1) ? 1.0f / (float)row : 0.0f;
        }
    const int32_t *wl = a.sw ? a.sw : a.widx;
    const int32_t step = 8 * nw;
    int32_t e = e0 + 8 * w;
    if (e < e1) {
        int32_t sb1 = (e + step + ps < e1) ? wl[e + step + ps] : 0;
        m2l_chunk<KS, float2> cur;
        m2l_fetch<KS, LOG, true>(a, bo, nbl, e, e1, (e + ps < e1) ? wl[e + ps] : 0, ps, kq, rmin, cur);
        for (; e < e1; e += step) {
            const int32_t en = e + step;
            const int32_t sb2 = (en + step + ps < e1) ? wl[en + step + ps] : 0;
            m2l_chunk<KS, float2> nxt;
            m2l_fetch<KS, LOG, true>(a, bo, nbl, en, e1, sb1, ps, kq, rmin, nxt);
            sb1 = sb2;

            const bool valid = cur.valid;
            const int qlim = valid ? cur.q : -1;
            const int ksn = (cur.qc + 3) >> 2, mtn = (cur.qc >> 4) + 1;
            const double2 r = make_double2(cur.cS.x - cT.x, cur.cS.y - cT.y);
            double2 u64 = make_double2(0.0, 0.0), v64 = make_double2(0.0, 0.0);
            if (valid) {
                const double2 ri = cinv_fast(r);
                u64 = make_double2(cur.sS * ri.x, cur.sS * ri.y);
                v64 = make_double2(sT * ri.x, sT * ri.y);
            }
            const float2 u1 = make_float2((float)u64.x, (float)u64.y);
            const float2 v = make_float2((float)v64.x, (float)v64.y);
            const float2 u2 = cmulf(u1, u1), u3 = cmulf(u2, u1), u4 = cmulf(u2, u2);
            // as in the FP64 kernel, with u = sigma_S / r in place of 1/r
            const float2 p0 = kq == 0 ? u1 : (kq == 1 ? u2 : (kq == 2 ? u3 : u4));
            const float sg = (kq & 1) ? 1.0f : -1.0f;
            float w1 = comp ? sg * p0.y : sg * p0.x;
            float w2 = comp ? sg * p0.x : -sg * p0.y;
            float bop[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                bop[ks] = 0.0f;
                if (ks < ksn) {
                    const float2 ak = cur.ak[ks];
                    bop[ks] = (4 * ks + kq + 1 <= qlim) ? fmaf(ak.y, w2, ak.x * w1) : 0.0f;
                    const float t = fmaf(w2, u4.y, w1 * u4.x);
                    w2 = fmaf(-w1, u4.y, w2 * u4.x);
                    w1 = t;
                }
            }
            flt4 C[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) C[mt] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    if (ks < ksn && mt < mtn)
                        C[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Sop[mt][ks], bop[ks], C[mt], 0, 0, 0);
            // post-scale with v = sigma_T / r: rows 16 mt + 4 kq + j
            const float2 v2 = cmulf(v, v), v4 = cmulf(v2, v2), v8 = cmulf(v4, v4), v16 = cmulf(v8, v8);
            const float2 b0 = kq == 0 ? make_float2(1.0f, 0.0f) : (kq == 1 ? v4 : (kq == 2 ? v8 : cmulf(v8, v4)));
            const float sc = comp ? 1.0f : -1.0f;
            const float d1 = sc * v.y, d16 = sc * v16.y;
            float e1v = b0.x, e2v = sc * b0.y;
            const float a0m = (float)(comp ? cur.a0.y : cur.a0.x), a0o = (float)(comp ? cur.a0.x : cur.a0.y);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                if (mt >= mtn) break;
                float g1 = e1v, g2 = e2v;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * kq + j;
                    float mine = C[mt][j];
                    float oth = dpp32<DPP_XOR1>(mine);
                    if (LOG) {
                        mine = fmaf(-a0m, irow[mt][j], mine);
                        oth = fmaf(-a0o, irow[mt][j], oth);
                    }
                    const float res = fmaf(oth, g2, mine * g1);
                    acc[mt][j] += (row <= qlim) ? res : 0.0f;
                    const float t = fmaf(-g2, d1, g1 * v.x);
                    g2 = fmaf(g1, d1, g2 * v.x);
                    g1 = t;
                }
                const float t = fmaf(-e2v, d16, e1v * v16.x);
                e2v = fmaf(e1v, d16, e2v * v16.x);
                e1v = t;
            }
            if (LOG && valid && kq == 0) {
                const double2 lg = clog_principal(make_double2(cT.x - cur.cS.x, cT.y - cur.cS.y));
                const double2 t = cmul(cur.a0, lg);
                acc0 += comp ? t.y : t.x;
            }
            cur = nxt;
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mt][j] = sum8_32(acc[mt][j]);
    acc0 = sum8_64(acc0);
}

// b_l = bhat_l / sigma_T^l in FP64, one factor at a time so that no
// intermediate power over- or underflows.
__device__ __forceinline__ double m2l32_unscale(double v, int row, double isT)
{
    for (int q = 0; q < row; ++q) v *= isT;
    return v;
}

// One launch: blocks [0, H) take the boxes with more than M2L_HEAVY weak pairs
// (M2L_WAVES waves per box, fixed-order LDS reduction); the other blocks take
// the light boxes, one wave per box.
template <int MT, int KS, bool LOG>
__global__ void __launch_bounds__(64 * M2L_WAVES) __attribute__((amdgpu_waves_per_eu(2))) k_m2l32(m2l_args a, int32_t H)
{
    __shared__ double part[M2L_WAVES][MT * 16][2];
    const int lane = threadIdx.x & (WAVE - 1);
    const int col = lane & 15, ps = col >> 1, comp = col & 1, kq = lane >> 4;
    const int P1 = a.p + 1;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    if ((int32_t)blockIdx.x >= H) {
        const int64_t g = (int64_t)(blockIdx.x - H) * M2L_WAVES + w;
        if (g >= a.nb) return;
        int l;
        int32_t e0, e1;
        if (m2l_range(a, g, l, e0, e1) > M2L_HEAVY) return;
        float acc[MT][4];
        double acc0;
        m2l32_acc<MT, KS, LOG>(a, g, l, e0, e1, 0, 1, acc, acc0);
        const double isT = 1.0 / scale_radius(a.radius[g], scale_floor(a.radius));
        double2 *Bt = a.B + g * P1;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * mt + 4 * kq + j;
                double d = (double)acc[mt][j];
                if (row == 0) d += acc0;
                if (ps == 0 && row <= a.p) reinterpret_cast<double *>(Bt + row)[comp] = m2l32_unscale(d, row, isT);
            }
    } else {
        // segments of the heavy boxes; partial sums (unscaled) go to hpart
        const int32_t nseg = a.hoff[a.nb];
        for (int32_t sg = blockIdx.x; sg < nseg; sg += H) {
            const int64_t g = a.hbox[sg];
            int l;
            int32_t e0, e1;
            m2l_range(a, g, l, e0, e1);
            const int32_t s0 = min(e0 + (sg - a.hoff[g]) * M2L_SEG, e1), s1 = min(s0 + M2L_SEG, e1);
            float acc[MT][4];
            double acc0;
            m2l32_acc<MT, KS, LOG>(a, g, l, s0, s1, w, M2L_WAVES, acc, acc0);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * kq + j;
                    double d = (double)acc[mt][j];
                    if (row == 0) d += acc0;
                    if (ps == 0) part[w][row][comp] = d;
                }
            __syncthreads();
            if (w == 0) {
                const double isT = 1.0 / scale_radius(a.radius[g], scale_floor(a.radius));
                double2 *Bt = a.hpart + (int64_t)sg * P1;
                for (int k = lane; k < 2 * P1; k += WAVE) {
                    double v = 0.0;
                    for (int q = 0; q < M2L_WAVES; ++q) v += part[q][k >> 1][k & 1];
                    reinterpret_cast<double *>(Bt)[k] = m2l32_unscale(v, k >> 1, isT);
                }
            }
            __syncthreads();
        }
    }
}

// Heavy-box segments: count per box, the box of every segment, and the
// final sum of each heavy box's segment partials in segment order.
__global__ void k_m2l_hcount(m2l_args a, int32_t *__restrict__ hs)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nb) return;
    int l;
    int32_t e0, e1;
    const int32_t cnt = m2l_range(a, g, l, e0, e1);
    hs[g] = cnt > M2L_HEAVY ? (cnt + M2L_SEG - 1) / M2L_SEG : 0;
}

__global__ void k_m2l_hfill(const int32_t *__restrict__ hs, const int32_t *__restrict__ hoff, int64_t nb,
                            int32_t *__restrict__ hbox)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb) return;
    for (int32_t k = 0; k < hs[g]; ++k) hbox[hoff[g] + k] = (int32_t)g;
}

__global__ void k_m2l_hreduce(const int32_t *__restrict__ hs, const int32_t *__restrict__ hoff,
                              const double2 *__restrict__ hpart, int P1, int64_t nb, double2 *__restrict__ B)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * P1) return;
    const int64_t g = t / P1;
    const int c = (int)(t - g * P1);
    const int32_t n = hs[g];
    if (n == 0) return;
    double2 v = make_double2(0.0, 0.0);
    for (int32_t k = 0; k < n; ++k) {
        const double2 u = hpart[(int64_t)(hoff[g] + k) * P1 + c];
        v.x += u.x;
        v.y += u.y;
    }
    B[t] = v;
}

// FP32 radius-scaled copy of the multipoles: ahat_k = a_k / sigma^k.
__global__ void k_scale_mpole(const double2 *__restrict__ A, const double *__restrict__ radius,
                              float2 *__restrict__ A32, int p, int64_t nb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P1 = p + 1;
    if (t >= nb * P1) return;
    const int64_t g = t / P1;
    const int k = (int)(t - g * P1);
    const double is = 1.0 / scale_radius(radius[g], scale_floor(radius));
    double2 v = A[t];
    for (int q = 0; q < k; ++q) { v.x *= is; v.y *= is; }
    A32[t] = make_float2((float)v.x, (float)v.y);
}

// ------------------------------------------------------------ launchers --
#define WSC(T, off) reinterpret_cast<T *>(const_cast<char *>(a.ws) + (off))

template <int PM>
static void launch_p2m(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    const int64_t nleaf = nbox(a.L);
    unsigned nblk = (unsigned)((nleaf + 3) / 4);
    if (a.upward_blocks && nblk > a.upward_blocks) nblk = a.upward_blocks;
    k_p2m<PM><<<nblk, 256, 0, st>>>(WSC(double4, lay.srcs),
                                    WSC(int32_t, lay.sstart) + start_off(a.L),
                                    WSC(double, lay.centre) + 2 * box_off(a.L),
                                    WSC(double2, lay.A) + box_off(a.L) * (a.p + 1), a.p, a.kernel,
                                    (int32_t)nleaf);
}

hipError_t fmm_p2m(const fmm_eval_args &a, hipStream_t st)
{
    if (a.p <= 20) launch_p2m<20>(a, st);
    else if (a.p <= 32) launch_p2m<32>(a, st);
    else if (a.p <= 44) launch_p2m<44>(a, st);
    else launch_p2m<64>(a, st);
    return hipGetLastError();
}

template <int PM>
static void launch_p2l(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    const int64_t nleaf = nbox(a.L);
    const unsigned nblk = (unsigned)((nleaf + 3) / 4);
    auto k = a.kernel == FMM2D_KERNEL_LOG ? k_p2l<PM, true> : k_p2l<PM, false>;
    k<<<nblk, 256, 0, st>>>(WSC(double4, lay.srcs), WSC(int32_t, lay.sstart) + start_off(a.L), WSC(int32_t, lay.poff),
                            WSC(int32_t, lay.pidx), WSC(double, lay.centre) + 2 * box_off(a.L),
                            WSC(double2, lay.B) + box_off(a.L) * (a.p + 1), a.p, (int32_t)nleaf,
                            (int32_t)lay.leafcap);
}

hipError_t fmm_p2l(const fmm_eval_args &a, hipStream_t st)
{
    if (!a.swap) return hipSuccess;
    if (a.p <= 20) launch_p2l<20>(a, st);
    else if (a.p <= 32) launch_p2l<32>(a, st);
    else if (a.p <= 44) launch_p2l<44>(a, st);
    else launch_p2l<64>(a, st);
    return hipGetLastError();
}

hipError_t fmm_m2m(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    for (int l = a.L - 1; l >= 0; --l) {
        const int64_t nt = nbox(l) * (a.p + 1);
        unsigned nblk = (unsigned)((nt + 255) / 256);
        if (a.upward_blocks && nblk > a.upward_blocks) nblk = a.upward_blocks;
        k_m2m<<<nblk, 256, 0, st>>>(WSC(double, lay.centre), WSC(double2, lay.A),
                                                            a.binom, a.p, l, nbox(l));
    }
    return hipGetLastError();
}

hipError_t fmm_l2l(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    for (int l = 1; l <= a.L; ++l) {
        const int64_t nt = nbox(l) * (a.p + 1);
        k_l2l<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(WSC(double, lay.centre), WSC(double2, lay.B),
                                                            a.binom, a.p, l, nbox(l));
    }
    return hipGetLastError();
}

template <int MT, int KS>
static void launch_m2l(const m2l_args &m, bool mixed, hipStream_t st)
{
    const int32_t H = (int32_t)(m.nb < 512 ? m.nb : 512);
    const unsigned nblk = (unsigned)(H + (m.nb + M2L_WAVES - 1) / M2L_WAVES);
    const bool LOG = m.kernel == FMM2D_KERNEL_LOG;
    if (mixed) {
        if (LOG) k_m2l32<MT, KS, true><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
        else k_m2l32<MT, KS, false><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
    } else {
        if (LOG) k_m2l64<MT, KS, true><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
        else k_m2l64<MT, KS, false><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
    }
}

// Segments of the heavy boxes (after the lists, before the order phase,
// whose sort works on the same units).
hipError_t fmm_m2l_plan(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    m2l_args m;
    memset(&m, 0, sizeof(m));
    m.woff = WSC(int32_t, lay.woff);
    m.nb = lay.nb;
    m.L = a.L;
    m.cap = (int32_t)lay.listcap;
    int32_t *hs = WSC(int32_t, lay.hs), *hoff = WSC(int32_t, lay.hoff), *hbox = WSC(int32_t, lay.hbox);
    const unsigned nbk = (unsigned)((lay.nb + 255) / 256);
    k_m2l_hcount<<<nbk, 256, 0, st>>>(m, hs);
    hipError_t e = fmm_scan_i32(hs, hoff, lay.nb, nullptr, WSC(int32_t, lay.bsum), st);
    if (e != hipSuccess) return e;
    k_m2l_hfill<<<nbk, 256, 0, st>>>(hs, hoff, lay.nb, hbox);
    return hipGetLastError();
}

hipError_t fmm_m2l(const fmm_eval_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    m2l_args m;
    m.centre = WSC(double, lay.centre);
    m.radius = WSC(double, lay.radius);
    m.A = WSC(double2, lay.A);
    m.A32 = a.mixed ? WSC(float2, lay.A32) : nullptr;
    m.B = WSC(double2, lay.B);
    m.woff = WSC(int32_t, lay.woff);
    m.widx = WSC(int32_t, lay.widx);
    m.sw = a.porder ? WSC(int32_t, lay.sw) : nullptr;
    m.sp = a.porder ? WSC(uint8_t, lay.sp) : nullptr;
    m.binom = a.binom;
    m.nb = lay.nb;
    m.L = a.L;
    m.p = a.p;
    m.kernel = a.kernel;
    m.cap = (int32_t)lay.listcap;
    int32_t *hs = WSC(int32_t, lay.hs), *hoff = WSC(int32_t, lay.hoff), *hbox = WSC(int32_t, lay.hbox);
    m.hoff = hoff;
    m.hbox = hbox;
    m.hpart = WSC(double2, lay.hpart);
    if (a.mixed) {
        const int64_t nt = lay.nb * (a.p + 1);
        k_scale_mpole<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(m.A, m.radius, WSC(float2, lay.A32),
                                                                     a.p, lay.nb);
    }
    const int p = a.p;
    const int MT = (p + 1 + 15) / 16, KS = (p + 3) / 4;
    // instantiate the shapes that cover p = 1..64
    if (MT == 1 && KS <= 4) launch_m2l<1, 4>(m, a.mixed, st);
    else if (MT <= 2 && KS <= 5) launch_m2l<2, 5>(m, a.mixed, st);
    else if (MT <= 2 && KS <= 8) launch_m2l<2, 8>(m, a.mixed, st);
    else if (MT <= 3 && KS <= 12) launch_m2l<3, 12>(m, a.mixed, st);
    else launch_m2l<5, 16>(m, a.mixed, st);
    const int64_t nc = lay.nb * (a.p + 1);
    k_m2l_hreduce<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(hs, hoff, m.hpart, a.p + 1, lay.nb, m.B);
    return hipGetLastError();
}
