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
// it describes.)  S is the same for every pair, so it stays in registers as
// the MFMA A operand while the pre-scaled multipoles of 8 pairs (16 real
// columns: re/im) stream through the B operand.
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

// ------------------------------------------------------------------ P2M --
// One wave per leaf, one source per lane: every lane accumulates
// s_k = sum m (x-c)^k in registers, then the wave reduces the 2(p+1) sums.
//   LOG:      a_0 = s_0, a_k = -s_k / k
//   HARMONIC: a_0 = 0,   a_k = s_{k-1}
template <int PM>
__global__ void __launch_bounds__(256) k_p2m(const double4 *__restrict__ srcs,
                                              const int32_t *__restrict__ sst,
                                              const double *__restrict__ centre,
                                              double2 *__restrict__ A, int p, int kernel,
                                              int32_t nleaf)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int32_t b = wave_index();
    if (b >= nleaf) return;
    const int32_t s0 = sst[b], s1 = sst[b + 1];
    const double cx = centre[2 * (int64_t)b], cy = centre[2 * (int64_t)b + 1];
    double sr[PM + 1], si[PM + 1];
#pragma unroll
    for (int k = 0; k <= PM; ++k) { sr[k] = 0.0; si[k] = 0.0; }
    for (int32_t j = s0 + lane; j < s1; j += WAVE) {
        const double4 d = srcs[j];
        const double2 w = make_double2(d.x - cx, d.y - cy);
        double2 pw = make_double2(d.z, d.w);
#pragma unroll
        for (int k = 0; k <= PM; ++k) {
            if (k <= p) {
                sr[k] += pw.x;
                si[k] += pw.y;
                pw = cmul(pw, w);
            }
        }
    }
    double2 *out = A + (int64_t)b * (p + 1);
#pragma unroll
    for (int k = 0; k <= PM; ++k) {
        if (k <= p) {
            const double r = wave_sum(sr[k]), i = wave_sum(si[k]);
            if (lane == 0) {
                if (kernel == FMM2D_KERNEL_LOG) {
                    out[k] = (k == 0) ? make_double2(r, i) : make_double2(-r / k, -i / k);
                } else {
                    if (k < p) out[k + 1] = make_double2(r, i);
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
//   LOG:      b_0 += m Log(c - x),   b_l -= m u^l / l      (l >= 1)
//   HARMONIC: b_l -= m u^{l+1}                            (l >= 0)
// One wave per leaf, one source per lane, wave reduction of the p+1 sums.
template <int PM>
__global__ void __launch_bounds__(256) k_p2l(const double4 *__restrict__ srcs,
                                              const int32_t *__restrict__ sst,
                                              const int32_t *__restrict__ poff,
                                              const int32_t *__restrict__ pidx,
                                              const double *__restrict__ centre,
                                              double2 *__restrict__ B, int p, int kernel,
                                              int32_t nleaf, int32_t lcap)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int32_t t = wave_index();
    if (t >= nleaf) return;
    const int32_t e0 = min(poff[t], lcap), e1 = min(poff[t + 1], lcap);
    if (e0 >= e1) return;
    const double cx = centre[2 * (int64_t)t], cy = centre[2 * (int64_t)t + 1];
    const bool LOG = kernel == FMM2D_KERNEL_LOG;
    double sr[PM + 1], si[PM + 1];
#pragma unroll
    for (int k = 0; k <= PM; ++k) { sr[k] = 0.0; si[k] = 0.0; }
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t s = __builtin_amdgcn_readfirstlane(min(max(pidx[e], 0), nleaf - 1));
        const int32_t j0 = sst[s], j1 = sst[s + 1];
        for (int32_t j = j0 + lane; j < j1; j += WAVE) {
            const double4 q = srcs[j];
            const double2 u = cinv(make_double2(q.x - cx, q.y - cy));
            double2 pw = make_double2(q.z, q.w);
            if (LOG) {
                const double lx = cx - q.x, ly = cy - q.y; // Log(c - x), formed as written
                const double2 lg = make_double2(0.5 * log(lx * lx + ly * ly), atan2(ly, lx));
                const double2 t0 = cmul(pw, lg);
                sr[0] += t0.x;
                si[0] += t0.y;
            }
#pragma unroll
            for (int k = 0; k <= PM; ++k) {
                if (k <= p) {
                    if (LOG) {
                        if (k >= 1) {
                            pw = cmul(pw, u);
                            sr[k] -= pw.x / k;
                            si[k] -= pw.y / k;
                        }
                    } else {
                        pw = cmul(pw, u);
                        sr[k] -= pw.x;
                        si[k] -= pw.y;
                    }
                }
            }
        }
    }
    double2 *out = B + (int64_t)t * (p + 1);
#pragma unroll
    for (int k = 0; k <= PM; ++k) {
        if (k <= p) {
            const double r = wave_sum(sr[k]), i = wave_sum(si[k]);
            if (lane == 0) {
                double2 o = out[k];
                o.x += r;
                o.y += i;
                out[k] = o;
            }
        }
    }
}

// ------------------------------------------------------------------ M2M --
// Thread per (parent, coefficient l): a'_l = sum over the 4 children of
// -a_0 r^l / l + sum_{k=1..l} C(l-1,k-1) a_k r^{l-k},  r = c_child - c_parent.
__global__ void k_m2m(const double *__restrict__ centre, double2 *__restrict__ A,
                      const double *__restrict__ binom, int p, int l, int64_t nbl)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P1 = p + 1;
    if (t >= nbl * P1) return;
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

#define M2L_HEAVY 256 // boxes with more weak pairs get an 8-wave workgroup
#define M2L_WAVES 8

__device__ __forceinline__ int32_t m2l_range(const m2l_args &a, int64_t g, int &l, int32_t &e0, int32_t &e1)
{
    l = level_of(g, a.L);
    const int32_t b = (int32_t)(g - d_box_off(l));
    const int64_t so = d_start_off(l);
    e0 = min(a.woff[so + b], a.cap);
    e1 = min(a.woff[so + b + 1], a.cap);
    return e1 - e0;
}

// FP64 contraction for the chunks c = w, w + nw, ... of 8 weak pairs of box g.
// Lane layout of v_mfma_f64_16x16x4f64: A operand lane i holds A[i%16][i/16],
// B operand lane i holds B[i/16][i%16], accumulator element j of lane i holds
// row 4j + i/16 of column i%16 (the FP64 instruction interleaves its rows).
// On return acc[mt][j] holds, summed over this lane's pairs, the re (even
// column) or im (odd column) part of b_l, l = 16 mt + 4 j + kq.
template <int MT, int KS>
__device__ __forceinline__ void m2l64_acc(const m2l_args &a, int64_t g, int l, int32_t e0, int32_t e1, int w,
                                          int nw, double (&acc)[MT][4])
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t bo = d_box_off(l);
    const int p = a.p, P1 = p + 1;
    const int col = lane & 15, ps = col >> 1, comp = col & 1, kq = lane >> 4;
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double2 cT = make_double2(a.centre[2 * g], a.centre[2 * g + 1]);
    const bool LOG = a.kernel == FMM2D_KERNEL_LOG;
    double Sop[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int row = 16 * mt + col, kk = 4 * ks + kq;
            Sop[mt][ks] = (row <= p && kk < p) ? a.binom[(row + kk) * FMM_BN + row] : 0.0;
        }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mt][j] = 0.0;
    // 1/l for the a_0 term of the rows this lane holds (LOG only)
    double irow[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * mt + 4 * j + kq;
            irow[mt][j] = (LOG && row >= 1) ? 1.0 / row : 0.0;
        }

    const int32_t *wl = a.sw ? a.sw : a.widx;
    // the next chunk's list entry is fetched one iteration ahead
    int32_t sb_next = (e0 + 8 * w + ps < e1) ? wl[e0 + 8 * w + ps] : 0;
    for (int32_t e = e0 + 8 * w; e < e1; e += 8 * nw) {
        const int32_t pe = e + ps;
        const bool valid = pe < e1;
        int32_t sb = valid ? sb_next : 0;
        const int32_t pn = pe + 8 * nw;
        sb_next = (pn < e1) ? wl[pn] : 0;
        sb = min(max(sb, 0), nbl - 1);
        // order of this lane's pair (q) and the largest order of the chunk
        // (qc, its last pair: orders ascend within a box), which bounds the
        // k-steps and row tiles the chunk needs
        int q = p, qc = p;
        if (a.sp) {
            q = valid ? (int)a.sp[pe] : 0;
            qc = __builtin_amdgcn_readfirstlane((int)a.sp[min(e + 7, e1 - 1)]);
        }
        const int ksn = (qc + 3) >> 2, mtn = (qc >> 4) + 1;
        const int64_t gS = bo + sb;
        const double2 r = make_double2(a.centre[2 * gS] - cT.x, a.centre[2 * gS + 1] - cT.y);
        const double2 rinv = valid ? cinv_fast(r) : make_double2(0.0, 0.0);
        const double2 *As = a.A + gS * P1;
        // pre-scale: lane holds beta_{k'} for k' = 4 ks + kq
        const double2 r2 = cmul(rinv, rinv);
        const double2 r4 = cmul(r2, r2);
        double2 pw = rinv;
        for (int t = 0; t < kq; ++t) pw = cmul(pw, rinv);
        double bop[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int kk = 4 * ks + kq + 1;
            bop[ks] = 0.0;
            if (ks < ksn) {
                const double2 ak = (valid && kk <= q) ? As[kk] : make_double2(0.0, 0.0);
                double2 v = cmul(ak, pw);
                if (kk & 1) { v.x = -v.x; v.y = -v.y; }
                bop[ks] = comp ? v.y : v.x;
                pw = cmul(pw, r4);
            }
        }
        dbl4 C[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) C[mt] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                if (ks < ksn && mt < mtn)
                    C[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Sop[mt][ks], bop[ks], C[mt], 0, 0, 0);
        // post-scale: row l = 16 mt + 4 j + kq gets r^{-l} (B_l - a_0/l)
        const double2 a0 = (valid && LOG) ? As[0] : make_double2(0.0, 0.0);
        const double2 r16 = cmul(cmul(r4, r4), cmul(r4, r4));
        double2 base = make_double2(1.0, 0.0);
        for (int t = 0; t < kq; ++t) base = cmul(base, rinv);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            if (mt >= mtn) break;
            double2 pr = base;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * mt + 4 * j + kq;
                const double mine = C[mt][j];
                const double oth = dpp64<DPP_XOR1>(mine);
                double2 Bl = comp ? make_double2(oth, mine) : make_double2(mine, oth);
                if (LOG) {
                    Bl.x -= a0.x * irow[mt][j];
                    Bl.y -= a0.y * irow[mt][j];
                }
                const double2 res = cmul(Bl, pr);
                if (valid && row <= q) acc[mt][j] += comp ? res.y : res.x;
                pr = cmul(pr, r4);
            }
            base = cmul(base, r16);
        }
        if (LOG && valid && kq == 0) {
            // Log(c_T - c_S), the difference formed as written: on the branch
            // cut the sign of a zero imaginary part decides between +pi and -pi
            const double2 lg = clog_principal(make_double2(cT.x - a.centre[2 * gS], cT.y - a.centre[2 * gS + 1]));
            const double2 t = cmul(a0, lg);
            acc[0][0] += comp ? t.y : t.x;
        }
    }
    // sum over the 8 pairs of a tile (lane bits 1..3)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mt][j] = sum8_64(acc[mt][j]);
}

// One launch: blocks [0, H) take the boxes with more than M2L_HEAVY weak pairs
// (M2L_WAVES waves per box, fixed-order LDS reduction); the other blocks take
// the light boxes, one wave per box.
template <int MT, int KS>
__global__ void __launch_bounds__(64 * M2L_WAVES) k_m2l64(m2l_args a, int32_t H)
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
        double acc[MT][4];
        m2l64_acc<MT, KS>(a, g, l, e0, e1, 0, 1, acc);
        double2 *Bt = a.B + g * P1;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * mt + 4 * j + kq;
                if (ps == 0 && row <= a.p) reinterpret_cast<double *>(Bt + row)[comp] = acc[mt][j];
            }
    } else {
        for (int64_t g = blockIdx.x; g < a.nb; g += H) {
            int l;
            int32_t e0, e1;
            if (m2l_range(a, g, l, e0, e1) <= M2L_HEAVY) continue;
            double acc[MT][4];
            m2l64_acc<MT, KS>(a, g, l, e0, e1, w, M2L_WAVES, acc);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (ps == 0) part[w][16 * mt + 4 * j + kq][comp] = acc[mt][j];
            __syncthreads();
            if (w == 0) {
                double2 *Bt = a.B + g * P1;
                for (int k = lane; k < 2 * P1; k += WAVE) {
                    double v = 0.0;
                    for (int q = 0; q < M2L_WAVES; ++q) v += part[q][k >> 1][k & 1];
                    reinterpret_cast<double *>(Bt)[k] = v;
                }
            }
            __syncthreads();
        }
    }
}

// FP32 (mixed precision): the same contraction on v_mfma_f32_16x16x4f32 with
// radius-scaled coefficients.  With sigma_S, sigma_T the box radii,
// ahat_k = a_k / sigma_S^k, u = sigma_S / r and v = sigma_T / r:
//   beta_{k'} = (-1)^{k'+1} ahat_{k'+1} u^{k'+1},
//   bhat_l    = v^l (B_l - a_0/l),   b_l = bhat_l / sigma_T^l.
// The theta-criterion keeps |u|, |v| <= theta/(1+theta) < 1, so every scaled
// quantity stays O(1) in FP32.  Log(c_T - c_S) and the final unscaling are FP64.
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

// Accumulator layout of v_mfma_f32_16x16x4f32: element j of lane i holds row
// 4 (i/16) + j of column i%16.  acc0 collects the FP64 a_0 Log term of row 0.
template <int MT, int KS>
__device__ __forceinline__ void m2l32_acc(const m2l_args &a, int64_t g, int l, int32_t e0, int32_t e1, int w,
                                          int nw, float (&acc)[MT][4], double &acc0)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t bo = d_box_off(l);
    const int p = a.p, P1 = p + 1;
    const int col = lane & 15, ps = col >> 1, comp = col & 1, kq = lane >> 4;
    const int32_t nbl = (int32_t)(((int64_t)1) << (2 * l));
    const double2 cT = make_double2(a.centre[2 * g], a.centre[2 * g + 1]);
    const double rmin = scale_floor(a.radius);
    const double sT = scale_radius(a.radius[g], rmin);
    const bool LOG = a.kernel == FMM2D_KERNEL_LOG;
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
    float irow[MT][4]; // 1/l for the a_0 term (LOG only); rows 16 mt + 4 kq + j
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * mt + 4 * kq + j;
            irow[mt][j] = (LOG && row >= 1) ? 1.0f / (float)row : 0.0f;
        }
    const int32_t *wl = a.sw ? a.sw : a.widx;
    // the next chunk's list entry is fetched one iteration ahead
    int32_t sb_next = (e0 + 8 * w + ps < e1) ? wl[e0 + 8 * w + ps] : 0;
    for (int32_t e = e0 + 8 * w; e < e1; e += 8 * nw) {
        const int32_t pe = e + ps;
        const bool valid = pe < e1;
        int32_t sb = valid ? sb_next : 0;
        const int32_t pn = pe + 8 * nw;
        sb_next = (pn < e1) ? wl[pn] : 0;
        sb = min(max(sb, 0), nbl - 1);
        int q = p, qc = p; // as in the FP64 kernel
        if (a.sp) {
            q = valid ? (int)a.sp[pe] : 0;
            qc = __builtin_amdgcn_readfirstlane((int)a.sp[min(e + 7, e1 - 1)]);
        }
        const int ksn = (qc + 3) >> 2, mtn = (qc >> 4) + 1;
        const int64_t gS = bo + sb;
        const double2 r = make_double2(a.centre[2 * gS] - cT.x, a.centre[2 * gS + 1] - cT.y);
        const double sS = scale_radius(a.radius[gS], rmin);
        double2 u64 = make_double2(0.0, 0.0), v64 = make_double2(0.0, 0.0);
        if (valid) {
            const double2 ri = cinv_fast(r);
            u64 = make_double2(sS * ri.x, sS * ri.y);
            v64 = make_double2(sT * ri.x, sT * ri.y);
        }
        const float2 u = make_float2((float)u64.x, (float)u64.y);
        const float2 v = make_float2((float)v64.x, (float)v64.y);
        const float2 *As = a.A32 + gS * P1;
        const float2 u2 = cmulf(u, u), u4 = cmulf(u2, u2);
        float2 pw = u;
        for (int t = 0; t < kq; ++t) pw = cmulf(pw, u);
        float bop[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int kk = 4 * ks + kq + 1;
            bop[ks] = 0.0f;
            if (ks < ksn) {
                const float2 ak = (valid && kk <= q) ? As[kk] : make_float2(0.0f, 0.0f);
                float2 t = cmulf(ak, pw);
                if (kk & 1) { t.x = -t.x; t.y = -t.y; }
                bop[ks] = comp ? t.y : t.x;
                pw = cmulf(pw, u4);
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
        const double2 a064 = (valid && LOG) ? a.A[gS * P1] : make_double2(0.0, 0.0);
        const float2 a0 = make_float2((float)a064.x, (float)a064.y);
        const float2 v2 = cmulf(v, v), v4 = cmulf(v2, v2);
        const float2 v16 = cmulf(cmulf(v4, v4), cmulf(v4, v4));
        float2 base = make_float2(1.0f, 0.0f);
        for (int t = 0; t < kq; ++t) base = cmulf(base, v4);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            if (mt >= mtn) break;
            float2 pr = base;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * mt + 4 * kq + j;
                const float mine = C[mt][j];
                const float oth = dpp32<DPP_XOR1>(mine);
                float2 Bl = comp ? make_float2(oth, mine) : make_float2(mine, oth);
                if (LOG) {
                    Bl.x -= a0.x * irow[mt][j];
                    Bl.y -= a0.y * irow[mt][j];
                }
                const float2 res = cmulf(Bl, pr);
                if (valid && row <= q) acc[mt][j] += comp ? res.y : res.x;
                pr = cmulf(pr, v);
            }
            base = cmulf(base, v16);
        }
        if (LOG && valid && kq == 0) {
            const double2 lg = clog_principal(make_double2(cT.x - a.centre[2 * gS], cT.y - a.centre[2 * gS + 1]));
            const double2 t = cmul(a064, lg);
            acc0 += comp ? t.y : t.x;
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
template <int MT, int KS>
__global__ void __launch_bounds__(64 * M2L_WAVES) k_m2l32(m2l_args a, int32_t H)
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
        m2l32_acc<MT, KS>(a, g, l, e0, e1, 0, 1, acc, acc0);
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
        for (int64_t g = blockIdx.x; g < a.nb; g += H) {
            int l;
            int32_t e0, e1;
            if (m2l_range(a, g, l, e0, e1) <= M2L_HEAVY) continue;
            float acc[MT][4];
            double acc0;
            m2l32_acc<MT, KS>(a, g, l, e0, e1, w, M2L_WAVES, acc, acc0);
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
                double2 *Bt = a.B + g * P1;
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
    const unsigned nblk = (unsigned)((nleaf + 3) / 4);
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
    k_p2l<PM><<<nblk, 256, 0, st>>>(WSC(double4, lay.srcs), WSC(int32_t, lay.sstart) + start_off(a.L),
                                    WSC(int32_t, lay.poff), WSC(int32_t, lay.pidx),
                                    WSC(double, lay.centre) + 2 * box_off(a.L),
                                    WSC(double2, lay.B) + box_off(a.L) * (a.p + 1), a.p, a.kernel,
                                    (int32_t)nleaf, (int32_t)lay.leafcap);
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
        k_m2m<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(WSC(double, lay.centre), WSC(double2, lay.A),
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
    if (mixed) k_m2l32<MT, KS><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
    else k_m2l64<MT, KS><<<nblk, 64 * M2L_WAVES, 0, st>>>(m, H);
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
    return hipGetLastError();
}
