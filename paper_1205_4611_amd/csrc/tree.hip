// Topological phase on gfx950: presort, equal-count median splits, box
// geometry and theta-criterion interaction lists (Goude & Engblom, Sec. 2 and
// Sec. 3.2).  Integer work plus FP64 compares; this file is compiled with
// -ffp-contract=off so the geometry and theta-tests round exactly as written.
//
// Design (replaces the paper's warp-32 pivot search, Alg. "Partitioning with
// successive splits", which is non-deterministic across blocks):
//  * a stable LSD radix sort of the order-preserving 64-bit key of each
//    coordinate (ties by index) gives every point its rank in the global
//    (x, index) and (y, index) orders; comparisons of ranks are exactly the
//    (coordinate, index) comparisons.
//  * each source set is then kept as two lists of 8-byte rank records
//    (rx, ry), one in x order and one in y order inside every segment.  One
//    split of every segment is data-parallel: the median is the record at
//    position floor(n/2) of the list of the split axis, which stays as it is
//    (its first floor(n/2) records are the lo side); only the other list is
//    stably partitioned by the side flag.  Both lists stay sorted inside every
//    segment, so the rectangles of the next step come from the segment ends
//    (coordinates are read from the sorted coordinate arrays at those ranks).
//  * the last splits of every segment of at most 2048 sources run in one
//    workgroup in LDS (k_subtree), which also writes the leaf order and the
//    leaf-ordered sources.  Targets (evaluation away from the sources) follow
//    the source splits by one pass per step (k_part_lb, decoupled look-back).
//  * the tree is a pyramid with children 4b..4b+3, so segment j of split step
//    k becomes segments 2j, 2j+1 of step k+1 and no host round-trip is needed.
// Kernels: the presort is k_rs_init (keys), then per 8-bit digit k_rs_hist
// (tile histograms), k_rs_colscan (per-digit scan over the tiles and the
// digit totals) and k_rs_scatter (stable, staged through LDS, tiles in an
// XCD-aware order; the last pass also writes every point's rank), then
// k_rs_decode (the sorted coordinates); k_srec_init builds the rank records; a
// global split step is k_seg (pivots and geometry of every segment) and
// k_part_src count / place (the list across the split); k_subtree finishes
// the segments in LDS; k_lists<false> counts and, after a scan of the counts,
// k_lists<true> writes the interaction lists of one level.
#pragma clang fp contract(off)

#include <string.h>

#include "common.h"

#define WAVE 64

// ---------------------------------------------------------------- scans --
#define SCAN_T 256
#define SCAN_I 8
#define SCAN_B (SCAN_T * SCAN_I)

__host__ __device__ int64_t fmm_scan_blocks(int64_t n) { return (n + SCAN_B - 1) / SCAN_B; }

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v)
{
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int32_t t = __shfl_up(v, o, WAVE);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; *total = block sum.
// sh must hold blockDim.x/64 ints.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *sh, int32_t *total)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    int32_t inc = wave_incl_scan(v);
    if (lane == WAVE - 1) sh[w] = inc;
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        int32_t s = sh[i];
        off += (i < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Up to 4 exclusive scans of arrays of the same length in one set of launches
// (grid row y: job y); job y's block sums live in bs[y].
__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(fmm_scan_jobs J, int64_t n)
{
    __shared__ int32_t sh[SCAN_T / WAVE];
    const int32_t *__restrict__ in = J.in[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i)
        if (base + i < n) s += in[base + i];
    int32_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) J.bs[blockIdx.y][blockIdx.x] = tot;
}

// One block per job: exclusive scan of the block sums in place (+ *base),
// the grand total to bs[nb] and to out[n].
__global__ void __launch_bounds__(1024) k_scan_sums(fmm_scan_jobs J, int64_t nb, int64_t n)
{
    __shared__ int32_t sh[1024 / WAVE];
    int32_t *__restrict__ bs = J.bs[blockIdx.y];
    int32_t carry = J.base[blockIdx.y] ? *J.base[blockIdx.y] : 0;
    for (int64_t c = 0; c < nb; c += blockDim.x) {
        int64_t k = c + threadIdx.x;
        int32_t v = k < nb ? bs[k] : 0;
        int32_t tot;
        int32_t ex = block_excl_scan(v, sh, &tot);
        if (k < nb) bs[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        bs[nb] = carry;
        J.out[blockIdx.y][n] = carry;
    }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_down(fmm_scan_jobs J, int64_t n)
{
    __shared__ int32_t sh[SCAN_T / WAVE];
    const int32_t *__restrict__ in = J.in[blockIdx.y];
    int32_t *__restrict__ out = J.out[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_I;
    int32_t v[SCAN_I];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int32_t tot;
    int32_t run = block_excl_scan(s, sh, &tot) + J.bs[blockIdx.y][blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// Small arrays (n <= SCAN_SMALL): one block of 1024 threads per job; thread t
// takes the SCAN_SMALL / 1024 consecutive elements from SCAN_SMALL/1024 t, all
// loaded before one block scan of the per-thread sums.
#define SCAN_SMALL 16384
#define SCAN_SMALL_I (SCAN_SMALL / 1024)
__global__ void __launch_bounds__(1024) k_scan_single(fmm_scan_jobs J, int64_t n)
{
    __shared__ int32_t sh[1024 / WAVE];
    const int32_t *__restrict__ in = J.in[blockIdx.y];
    int32_t *__restrict__ out = J.out[blockIdx.y];
    const int32_t base = J.base[blockIdx.y] ? *J.base[blockIdx.y] : 0;
    const int64_t k0 = (int64_t)threadIdx.x * SCAN_SMALL_I;
    int32_t v[SCAN_SMALL_I];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_SMALL_I; ++i) v[i] = k0 + i < n ? in[k0 + i] : 0;
#pragma unroll
    for (int i = 0; i < SCAN_SMALL_I; ++i) s += v[i];
    int32_t tot;
    int32_t run = base + block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_SMALL_I; ++i) {
        if (k0 + i < n) out[k0 + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) out[n] = base + tot;
}

hipError_t fmm_scan_i32_jobs(const fmm_scan_jobs &J, int njobs, int64_t n, hipStream_t st)
{
    if (njobs < 1 || njobs > FMM_SCAN_JOBS) return hipErrorInvalidValue;
    if (n <= SCAN_SMALL) {
        k_scan_single<<<dim3(1, njobs), 1024, 0, st>>>(J, n);
        return hipGetLastError();
    }
    const int64_t nb = fmm_scan_blocks(n);
    k_scan_reduce<<<dim3((unsigned)nb, njobs), SCAN_T, 0, st>>>(J, n);
    k_scan_sums<<<dim3(1, njobs), 1024, 0, st>>>(J, nb, n);
    k_scan_down<<<dim3((unsigned)nb, njobs), SCAN_T, 0, st>>>(J, n);
    return hipGetLastError();
}

hipError_t fmm_scan_i32(const int32_t *in, int32_t *out, int64_t n, const int32_t *base,
                        int32_t *blocksums, hipStream_t st)
{
    fmm_scan_jobs J;
    memset(&J, 0, sizeof(J));
    J.in[0] = in;
    J.out[0] = out;
    J.base[0] = base;
    J.bs[0] = blocksums;
    return fmm_scan_i32_jobs(J, 1, n, st);
}

// ------------------------------------------------------- radix presort --
// Stable LSD radix sort of (64-bit key, int32 value), 8-bit digits.  Starting
// from the identity order, equal keys stay in index order, which is exactly
// the (coordinate, index) order the split rule asks for.
__global__ void k_fill_u8(uint8_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

#define RS_T 256
#define RS_TILES 16
#define RS_BLOCK (RS_T * RS_TILES)

__device__ __forceinline__ uint64_t order_key(double x)
{
    if (x == 0.0) x = 0.0; // -0 and +0 compare equal: give them one key
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// One status bit per wave that saw a non-finite value (an error the host
// reports after the evaluation; the value itself is then used as 0 where it
// would steer the tree, so the build stays well formed).
__device__ __forceinline__ void flag_nonfinite(bool bad, int32_t *status)
{
    const uint64_t b = __ballot(bad);
    if (b && (threadIdx.x & (WAVE - 1)) == __ffsll((unsigned long long)b) - 1) atomicOr(status, FMM_ST_NONFINITE);
}

__global__ void k_rs_init(const double *__restrict__ pts, int64_t n, int axis,
                          uint64_t *__restrict__ keys, int32_t *__restrict__ vals, int32_t *__restrict__ status)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        double x = pts[2 * i + axis];
        bad = !isfinite(x);
        keys[i] = order_key(bad ? 0.0 : x);
        vals[i] = (int32_t)i;
    }
    flag_nonfinite(bad, status);
}

// Per-tile digit histogram of one pass: hist[digit][tile].
__global__ void __launch_bounds__(RS_T) k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                   int shift, int32_t *__restrict__ hist, int nblk)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, nblk);
    const int64_t base = (int64_t)tile * RS_BLOCK;
    for (int t = 0; t < RS_TILES; ++t) {
        int64_t k = base + (int64_t)t * RS_T + threadIdx.x;
        if (k < n) atomicAdd(&h[(keys[k] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + tile] = h[threadIdx.x];
}

// Column scan of one pass: block d scans column d of the histogram in place,
// off[d][b] = sum_{b' < b} hist[d][b'] (the position of block b's keys inside
// digit d's run), and writes the digit's total tot[d]; the scatter adds the
// digit bases (the exclusive scan of tot) itself.
__global__ void __launch_bounds__(1024) k_rs_colscan(int32_t *__restrict__ hist, int nblk, int32_t *__restrict__ tot)
{
    __shared__ int32_t sh[1024 / WAVE];
    const int d = blockIdx.x;
    int32_t *col = hist + (int64_t)d * nblk;
    int32_t carry = 0;
    for (int c0 = 0; c0 < nblk; c0 += blockDim.x) {
        const int k = c0 + threadIdx.x;
        const int32_t v = k < nblk ? col[k] : 0;
        int32_t t;
        const int32_t ex = block_excl_scan(v, sh, &t);
        if (k < nblk) col[k] = carry + ex;
        carry += t;
    }
    if (threadIdx.x == 0) tot[d] = carry;
}

// Scatter of one pass.  Wave w of a block takes the block's elements
// [w RS_BLOCK/4, (w+1) RS_BLOCK/4) 64 at a time and ranks each within its
// digit with wave-private counters (peers of a digit found by ballots over its
// 8 bits), so the loop has no block barrier; the four waves' counts then give
// every element its place in the block's digit-ordered tile, staged in LDS and
// written out so that consecutive threads write consecutive addresses of a
// digit's run.  Stable: the block's order is wave-major, then in order.
// Keys and values are staged one after the other through the same buffer,
// with the digit of every staged slot kept, so that the LDS use (39.9 KB) lets
// 4 blocks share a CU and a 4M-key pass runs in one round of blocks.
__global__ void __launch_bounds__(RS_T, 4) k_rs_scatter(const uint64_t *__restrict__ kin,
                                                      const int32_t *__restrict__ vin,
                                                      uint64_t *__restrict__ kout,
                                                      int32_t *__restrict__ vout, int64_t n,
                                                      int shift, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ tot, int nblk,
                                                      int32_t *__restrict__ rank)
{
    constexpr int NW = RS_T / WAVE, PER_W = RS_BLOCK / NW, IT = PER_W / WAVE;
    static_assert(PER_W <= 65535 && RS_BLOCK <= 65535, "per-wave counts and bases are 16-bit");
    __shared__ uint64_t sk[RS_BLOCK];   // staged keys, then (as int32) staged values
    __shared__ uint8_t sd[RS_BLOCK];    // digit of every staged slot
    __shared__ uint16_t wc[NW][256];    // per-wave digit counts, then per-wave digit bases
    __shared__ int32_t dstart[256];     // digit starts in the tile, then output base - start
    __shared__ int32_t sh[NW];
    int32_t *sv = reinterpret_cast<int32_t *>(sk);
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
#pragma unroll
    for (int q = 0; q < NW; ++q) wc[q][tid] = 0;
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, nblk);
    const int64_t base = (int64_t)tile * RS_BLOCK;
    const int64_t wbase = base + (int64_t)w * PER_W;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
    uint64_t key[IT];
    int32_t val[IT], rk[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const int64_t k = wbase + (int64_t)t * WAVE + lane;
        const bool valid = k < n;
        key[t] = valid ? kin[k] : 0ull;
        val[t] = valid ? vin[k] : 0;
    }
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        const bool valid = wbase + (int64_t)t * WAVE + lane < n;
        const int d = (int)((key[t] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const int32_t c = wc[w][d];
        rk[t] = valid ? c + __popcll(peers & lt) : -1;
        if (valid && __popcll(peers & lt) == 0) wc[w][d] = (uint16_t)(c + __popcll(peers));
    }
    __syncthreads();
    {
        // thread tid = digit: bases of the waves, the block's count, its start
        int32_t s = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int32_t v = wc[q][tid];
            wc[q][tid] = (uint16_t)s;
            s += v;
        }
        int32_t tot;
        dstart[tid] = block_excl_scan(s, sh, &tot);
    }
    __syncthreads();
    // rk[t] becomes the element's slot in the tile (-1: none)
#pragma unroll
    for (int t = 0; t < IT; ++t) {
        if (rk[t] >= 0) {
            const int d = (int)((key[t] >> shift) & 255);
            const int p = min(dstart[d] + (int)wc[w][d] + rk[t], RS_BLOCK - 1);
            rk[t] = p;
            sk[p] = key[t];
            sd[p] = (uint8_t)d;
        }
    }
    __syncthreads();
    // output base of every digit less its start in the tile: slot j of digit d
    // goes to position dstart[d] + j (the digit's base: the exclusive scan of
    // the totals, thread tid = digit)
    {
        int32_t all;
        const int32_t dbase = block_excl_scan(tot[tid], sh, &all);
        dstart[tid] = dbase + off[(int64_t)tid * nblk + tile] - dstart[tid];
    }
    __syncthreads();
    const int nvalid = (int)min((int64_t)RS_BLOCK, n - base);
    for (int j = tid; j < nvalid; j += RS_T) {
        int64_t pos = (int64_t)dstart[sd[j]] + j;
        pos = pos < 0 ? 0 : (pos >= n ? n - 1 : pos); // never leave the array
        kout[pos] = sk[j];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < IT; ++t)
        if (rk[t] >= 0) sv[rk[t]] = val[t];
    __syncthreads();
    for (int j = tid; j < nvalid; j += RS_T) {
        int64_t pos = (int64_t)dstart[sd[j]] + j;
        pos = pos < 0 ? 0 : (pos >= n ? n - 1 : pos);
        const int32_t v = sv[j];
        vout[pos] = v;
        // last pass of a presort: the values are the original indices, and
        // pos is the rank of that point
        if (rank) rank[v < 0 ? 0 : (v >= n ? n - 1 : v)] = (int32_t)pos;
    }
}

// LSD radix sort of (k0, v0) over `passes` 8-bit digits (ping-pong through
// k1, v1); the values end up in out.  Stable, so equal keys keep their order.
// hist holds 256 * nblk + 256 ints (histograms, scanned in place into the
// scatter offsets, then the digit totals).
static hipError_t radix_sort(int64_t n, int passes, uint64_t *k0, uint64_t *k1, int32_t *v0, int32_t *v1,
                             int32_t *hist, int32_t *bsum, int32_t *out, hipStream_t st, int32_t *rank = nullptr)
{
    if (n <= 0) return hipSuccess;
    if (passes <= 0) return hipMemcpyAsync(out, v0, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    const int nblk = (int)((n + RS_BLOCK - 1) / RS_BLOCK);
    int32_t *off = hist, *tot = hist + (int64_t)256 * nblk;
    uint64_t *ka = k0, *kb = k1;
    int32_t *va = v0, *vb = v1;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        k_rs_hist<<<nblk, RS_T, 0, st>>>(ka, n, shift, hist, nblk);
        k_rs_colscan<<<256, 1024, 0, st>>>(hist, nblk, tot);
        // the last pass writes the values to out (and, given rank, the inverse)
        const bool last = pass == passes - 1;
        k_rs_scatter<<<nblk, RS_T, 0, st>>>(ka, va, kb, last ? out : vb, n, shift, off, tot, nblk,
                                            last ? rank : nullptr);
        uint64_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    return hipGetLastError();
}

// Coordinate of each sorted key: the inverse of order_key, except that -0
// and +0 share a key, so a zero key takes the point's own coordinate.
__global__ void k_rs_decode(const uint64_t *__restrict__ keys, const int32_t *__restrict__ order,
                            const double *__restrict__ pts, int64_t n, int axis, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t k = keys[i];
        double x;
        if (k == 0x8000000000000000ull) {
            x = pts[2 * min(max((int64_t)order[i], (int64_t)0), n - 1) + axis];
            if (!isfinite(x)) x = 0.0; // a non-finite coordinate took the key of 0
        } else {
            const uint64_t u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
            x = __longlong_as_double((long long)u);
        }
        out[i] = x;
    }
}

// Indices 0..n-1 of pts ordered by (coordinate `axis`, index) into out, the
// inverse (rank of every index) into rank if not NULL and, if coord is not
// NULL, the coordinates in that order into coord.
static hipError_t presort(const double *pts, int64_t n, int axis, uint64_t *k0, uint64_t *k1,
                          int32_t *v0, int32_t *v1, int32_t *hist, int32_t *bsum, int32_t *out,
                          double *coord, int32_t *status, hipStream_t st, int32_t *rank = nullptr)
{
    if (n <= 0) return hipSuccess;
    k_rs_init<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(pts, n, axis, k0, v0, status);
    hipError_t e = radix_sort(n, 8, k0, k1, v0, v1, hist, bsum, out, st, rank);
    if (e != hipSuccess || !coord) return e;
    // an even number of passes leaves the sorted keys in k0
    k_rs_decode<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(k0, out, pts, n, axis, coord);
    return hipGetLastError();
}

// ------------------------------------------------------------ splits --
// Every point set is kept as two lists of self-describing records, one in
// (x, index) order and one in (y, index) order inside every segment.  A record
// carries its current segment, so the side of a split follows from comparing
// the record with its segment's pivot: no gathers through the original index,
// and stable partitions keep both lists sorted inside every new segment.
//
// Sources are records of ranks: rx, ry are the positions of the point in the
// global (x, index) and (y, index) orders, so (x, index) < (x', index') is
// exactly rx < rx'.  Coordinates are needed only at segment ends (rectangles)
// and come from xs[rx], ys[ry], the coordinates in sorted order; the original
// index is px[rx], px the x presort order.  A split along axis a leaves the
// segment's a-ordered list as it is (its first floor(n/2) records are the lo
// side), so only the other list moves: each list has two buffers and every
// segment a bit per list saying which buffer holds its records; a record's
// segment follows from its position.  Targets
// (evaluation away from the sources) go below a pivot by coordinate alone and
// keep their coordinates in the record.
struct src_rec {
    int32_t rx, ry;
};
struct pt_rec {
    double x, y;
    int32_t idx, seg;
};

__global__ void k_srec_init(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                            const int32_t *__restrict__ rxo, const int32_t *__restrict__ ryo, int64_t n,
                            src_rec *__restrict__ lx, src_rec *__restrict__ ly)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int64_t vx = min(max((int64_t)px[i], (int64_t)0), n - 1);
        const int64_t vy = min(max((int64_t)py[i], (int64_t)0), n - 1);
        lx[i] = src_rec{(int32_t)i, ryo[vx]};
        ly[i] = src_rec{rxo[vy], (int32_t)i};
    }
}

__global__ void k_trec_init(const double *__restrict__ pts, const int32_t *__restrict__ order, int64_t n,
                            pt_rec *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int32_t v = order[i];
        pt_rec r;
        r.x = pts[2 * (int64_t)v];
        r.y = pts[2 * (int64_t)v + 1];
        // (non-finite coordinates are flagged by the presort; as 0 they
        // cannot make a rectangle or a split comparison NaN)
        if (!isfinite(r.x)) r.x = 0.0;
        if (!isfinite(r.y)) r.y = 0.0;
        r.idx = v;
        r.seg = 0;
        out[i] = r;
    }
}

// partition tiles: LB_T threads, LB_I records each
#define LB_T 256
#define LB_I 16
#define LB_B (LB_T * LB_I)
static_assert(LB_B == FMM_LB_TILE, "partition tile size");
static_assert(LB_I * (LB_T / WAVE) == WAVE, "one wave scans the (stripe, wave) counts of a tile");

struct seg_args {
    const src_rec *slx[2], *sly[2]; // source lists (two buffers each)
    const uint8_t *bx, *by;       // per segment: the buffer holding its x / y list
    uint8_t *bx_next, *by_next;   // the same for the next step's segments
    int32_t *nlox, *nloy;         // lo counts of the lists that move (0 where a list stays)
    int32_t *tseg;                // per partition tile: the segment holding its first position, or NULL
    int32_t ntiles;               // tiles of the source lists
    int32_t *LOx, *LOy, *TLO;     // exclusive scans of nlox, nloy, tlo when one block holds every segment, else NULL
    const double *xs, *ys;        // source coordinates by rank
    const pt_rec *tlx, *tly;      // target lists (nt > 0)
    const int32_t *sst, *tst;     // step starts (nseg+1)
    int32_t *sst_next, *tst_next; // next step starts (2 nseg + 1), or NULL
    uint8_t *axis;
    double *pc;                   // pivot coordinate per segment
    int32_t *pi;                  // pivot rank (in the axis order) per segment
    int32_t *nlo, *tlo;
    double *centre, *radius;      // level arrays (already offset), or NULL
    int32_t *lvl_sst, *lvl_tst;   // per-level start output (already offset), or NULL
    uint64_t *lb_clear;           // partition tile states to zero, or NULL
    int64_t lb_n;
    int32_t nseg;
    int64_t ns, nt;
};

// One thread per segment: tight rectangle of its sources and targets, box
// geometry (on even steps), split axis, pivot (the record at rank floor(n/2)
// of the axis list) and the number of targets below the pivot coordinate.
// The grid also zeroes the tile states of this step's partition.
__device__ __forceinline__ void seg_work(const seg_args &a, int32_t j, int32_t &nlx, int32_t &nly, int32_t &tlv)
{
    const int32_t s0 = a.sst[j], s1 = a.sst[j + 1];
    const int32_t n = s1 - s0;
    const int32_t t0 = a.nt ? a.tst[j] : 0, t1 = a.nt ? a.tst[j + 1] : 0;
    const int32_t m = t1 - t0;
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    const src_rec *LX = a.slx[a.bx[j] & 1], *LY = a.sly[a.by[j] & 1];
    const int32_t rmax = (int32_t)a.ns - 1; // ranks index the sorted coordinates
    if (n > 0) {
        x0 = a.xs[min(max(LX[s0].rx, 0), rmax)];
        x1 = a.xs[min(max(LX[s1 - 1].rx, 0), rmax)];
        y0 = a.ys[min(max(LY[s0].ry, 0), rmax)];
        y1 = a.ys[min(max(LY[s1 - 1].ry, 0), rmax)];
    }
    if (m > 0) {
        double u;
        u = a.tlx[t0].x;      if (u < x0) x0 = u;
        u = a.tlx[t1 - 1].x;  if (u > x1) x1 = u;
        u = a.tly[t0].y;      if (u < y0) y0 = u;
        u = a.tly[t1 - 1].y;  if (u > y1) y1 = u;
    }
    const double w = x1 - x0, h = y1 - y0;
    if (a.centre) {
        a.centre[2 * (int64_t)j] = 0.5 * (x0 + x1);
        a.centre[2 * (int64_t)j + 1] = 0.5 * (y0 + y1);
        a.radius[j] = 0.5 * sqrt(w * w + h * h);
    }
    if (a.lvl_sst) {
        a.lvl_sst[j] = s0;
        if (j == a.nseg - 1) a.lvl_sst[a.nseg] = s1;
        if (a.nt) {
            a.lvl_tst[j] = t0;
            if (j == a.nseg - 1) a.lvl_tst[a.nseg] = t1;
        }
    }
    if (!a.sst_next) return;
    const int ax = (w >= h) ? 0 : 1;
    const int32_t nl = n / 2;
    int32_t tl = 0;
    double pcv = 0.0;
    int32_t prk = 0;
    if (n > 0) {
        const src_rec P = (ax ? LY : LX)[s0 + nl];
        prk = ax ? P.ry : P.rx;
        pcv = ax ? a.ys[min(max(prk, 0), rmax)] : a.xs[min(max(prk, 0), rmax)];
    }
    if (n > 0 && m > 0) {
        const pt_rec *TA = ax ? a.tly : a.tlx;
        int32_t lo = t0, hi = t1; // first position with coordinate >= pivot coordinate
        while (lo < hi) {
            int32_t mid = lo + ((hi - lo) >> 1);
            const double c = ax ? TA[mid].y : TA[mid].x;
            if (c >= pcv) hi = mid; else lo = mid + 1;
        }
        tl = lo - t0;
    }
    a.axis[j] = (uint8_t)ax;
    a.pc[j] = pcv;
    a.pi[j] = prk;
    a.nlo[j] = nl;
    a.tlo[j] = tl;
    // the list along the axis stays; the other moves to the other buffer
    nlx = ax ? nl : 0;
    nly = ax ? 0 : nl;
    tlv = tl;
    a.nlox[j] = nlx;
    a.nloy[j] = nly;
    const uint8_t nbx = ax ? (uint8_t)(1 - (a.bx[j] & 1)) : a.bx[j];
    const uint8_t nby = ax ? a.by[j] : (uint8_t)(1 - (a.by[j] & 1));
    a.bx_next[2 * j] = nbx;
    a.bx_next[2 * j + 1] = nbx;
    a.by_next[2 * j] = nby;
    a.by_next[2 * j + 1] = nby;
    a.sst_next[2 * j] = s0;
    a.sst_next[2 * j + 1] = s0 + nl;
    if (j == a.nseg - 1) a.sst_next[2 * a.nseg] = s1;
    if (a.nt) {
        a.tst_next[2 * j] = t0;
        a.tst_next[2 * j + 1] = t0 + tl;
        if (j == a.nseg - 1) a.tst_next[2 * a.nseg] = t1;
    }
}

// One thread per segment (seg_work), per tile of the source lists the segment
// of its first position, the clearing of the targets' partition states, and,
// when one block holds every segment, the exclusive scans of the lo counts.
__global__ void __launch_bounds__(1024) k_seg(seg_args a)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gt; i < a.lb_n; i += stride) a.lb_clear[i] = 0;
    if (a.tseg)
        for (int64_t t = gt; t < a.ntiles; t += stride) {
            const int64_t pos = t * LB_B;
            int32_t lo = 0, hi = a.nseg - 1; // the last segment starting at or before pos
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (a.sst[mid] <= pos) lo = mid; else hi = mid - 1;
            }
            a.tseg[t] = lo;
        }
    const int32_t j = (int32_t)gt;
    int32_t nlx = 0, nly = 0, tlv = 0;
    if (j < a.nseg) seg_work(a, j, nlx, nly, tlv);
    if (a.LOx) {
        __shared__ int32_t sh[1024 / WAVE];
        int32_t t;
        const int32_t ex = block_excl_scan(nlx, sh, &t);
        const int32_t ey = block_excl_scan(nly, sh, &t);
        if (j < a.nseg) {
            a.LOx[j] = ex;
            a.LOy[j] = ey;
        }
        if (a.TLO) {
            const int32_t et = block_excl_scan(tlv, sh, &t);
            if (j < a.nseg) a.TLO[j] = et;
        }
    }
}

// Stable partition of every segment of a list by the side of each record, in
// one pass (decoupled look-back).  Tiles of LB_B records are taken in the
// order of a ticket counter; a tile publishes its lo count (AGG), sums the
// counts of the tiles before it from their published states (stopping at the
// first inclusive prefix, INC), publishes its own inclusive prefix and
// scatters.  A tile only waits for tiles that took their ticket earlier and
// are therefore running, and every wait is bounded.
#define LB_AGG 1ull
#define LB_INC 2ull
#define LB_SPIN (1 << 20)

struct lb_list {
    const void *in;
    void *out;
    uint64_t *state;      // ntiles words, zero before the launch
    int32_t *ticket;      // zero before the launch
    const int32_t *start; // segment starts (nseg + 1)
    const int32_t *nlo;   // lo count per segment
    const int32_t *LO;    // exclusive scan of nlo
    int64_t n;
    int32_t nseg, ntiles;
};
struct lb_batch {
    lb_list l[2];
    const uint8_t *axis;
    const double *pc;
    const int32_t *pi;
    int32_t *status;
};

template <typename R>
__global__ void __launch_bounds__(LB_T) k_part_lb(lb_batch pb)
{
    const lb_list p = blockIdx.y ? pb.l[1] : pb.l[0]; // (a select keeps the fields in scalar registers)
    __shared__ int32_t s_tile, s_carry;
    __shared__ int32_t wc[LB_I * (LB_T / WAVE)]; // lo count per (stripe, wave), then its exclusive scan
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    if (tid == 0) s_tile = atomicAdd(p.ticket, 1);
    __syncthreads();
    const int32_t tile = s_tile;
    if (tile >= p.ntiles) return; // uniform over the block
    const R *in = reinterpret_cast<const R *>(p.in);
    R *out = reinterpret_cast<R *>(p.out);
    const int64_t base = (int64_t)tile * LB_B + tid;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
    R r[LB_I];
    uint64_t mk[LB_I];
    int32_t sg[LB_I];
    // three passes, so that the loads of a pass are in flight together: the
    // records, then the axis and pivot coordinate of their segments, then the
    // sides
#pragma unroll
    for (int i = 0; i < LB_I; ++i) r[i] = in[min(base + (int64_t)i * LB_T, p.n - 1)]; // (no branch: a valid index)
    uint8_t ax[LB_I];
    double pcv[LB_I];
#pragma unroll
    for (int i = 0; i < LB_I; ++i) {
        const int64_t pos = base + (int64_t)i * LB_T;
        const int32_t j = min(max(r[i].seg, 0), p.nseg - 1);
        sg[i] = pos < p.n ? j : -1;
        ax[i] = pb.axis[j];
        pcv[i] = pb.pc[j];
    }
#pragma unroll
    for (int i = 0; i < LB_I; ++i) {
        // lo iff the record's coordinate on its segment's axis is below the pivot coordinate
        const bool lo = sg[i] >= 0 && (ax[i] ? r[i].y : r[i].x) < pcv[i];
        mk[i] = __ballot(lo);
        if (lane == 0) wc[i * (LB_T / WAVE) + w] = __popcll(mk[i]);
    }
    __syncthreads();
    if (w == 0) {
        // exclusive scan of the 64 (stripe, wave) counts in stripe-major order
        const int32_t v = wc[lane];
        const int32_t inc = wave_incl_scan(v);
        wc[lane] = inc - v;
        const int32_t A = __shfl(inc, WAVE - 1, WAVE); // lo records of the tile
        if (lane == 0)
            __hip_atomic_store(p.state + tile, ((tile == 0 ? LB_INC : LB_AGG) << 32) | (uint32_t)A,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t prefix = 0;
        if (tile > 0) {
            int64_t t = tile - 1; // newest predecessor not yet summed
            int spins = 0;
            while (true) {
                const int64_t tt = t - lane;
                const uint64_t sv = tt >= 0 ? __hip_atomic_load(p.state + tt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                            : (LB_INC << 32);
                const uint32_t fl = (uint32_t)(sv >> 32);
                const uint64_t incm = __ballot(fl == LB_INC);
                const uint64_t notready = __ballot(fl == 0);
                const int k = incm ? (int)__builtin_ctzll(incm) : WAVE - 1; // lanes 0..k are summed
                const uint64_t need = (k == WAVE - 1) ? ~0ull : ((2ull << k) - 1);
                if (notready & need) {
                    if (++spins > LB_SPIN) {
                        if (lane == 0) atomicOr(pb.status, FMM_ST_TREE_INCONSISTENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                int32_t sum = (lane <= k) ? (int32_t)(uint32_t)sv : 0;
#pragma unroll
                for (int o = WAVE / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, WAVE);
                prefix += sum;
                if (incm) break;
                t -= WAVE;
            }
            if (lane == 0)
                __hip_atomic_store(p.state + tile, (LB_INC << 32) | (uint32_t)(prefix + A), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_carry = prefix;
    }
    __syncthreads();
    const int32_t carry = s_carry;
#pragma unroll
    for (int i = 0; i < LB_I; ++i) {
        if (sg[i] < 0) continue;
        const int64_t pos = base + (int64_t)i * LB_T;
        const int32_t j = sg[i];
        const bool lo = (mk[i] >> lane) & 1;
        const int32_t before = carry + wc[i * (LB_T / WAVE) + w] + __popcll(mk[i] & lt);
        const int32_t st = p.start[j];
        const int32_t rank = before - p.LO[j]; // lo records before pos in segment j
        int64_t dst = lo ? (int64_t)st + rank : (int64_t)st + p.nlo[j] + (pos - st - rank);
        dst = dst < 0 ? 0 : (dst >= p.n ? p.n - 1 : dst); // never leave the array
        R o = r[i];
        o.seg = 2 * j + (lo ? 0 : 1);
        out[dst] = o;
    }
}

// Source lists: per list (blockIdx.y: 0 x, 1 y) only the segments split across
// it move (from buffer bit[j] to the other); the tiles of LB_B positions find
// the segment of each position in an LDS window of the segment starts and
// skip the positions of segments that stay.  Two launches with a scan of the
// tile counts between them (no chain of waits between tiles): COUNT writes
// the tile's number of moving lo records, the second launch places every
// moving record stably (tile prefix from the scan; LO holds the exclusive
// prefix over segments of the moving lo counts).
#define LB_SEGW LB_T // segments of a tile held in LDS (one per thread)

struct ps_list {
    src_rec *buf0, *buf1;        // the list's two buffers
    const uint8_t *bit;          // per segment: the buffer holding this list
    const int32_t *LO;           // exclusive prefix of the moving lo counts
    int32_t *tcnt;               // per tile: moving lo records (written by the count pass)
};
struct ps_batch {
    ps_list l[2];
    const int32_t *start;        // segment starts (nseg + 1)
    const int32_t *nlo;          // lo count per segment
    const uint8_t *axis;
    const int32_t *pi;           // pivot rank in the axis order
    const int32_t *tseg;         // per tile: the segment holding its first position
    int64_t n;
    int32_t nseg, ntiles;
    int32_t *status;
};

template <bool COUNT>
__global__ void __launch_bounds__(LB_T) k_part_src(ps_batch pb)
{
    const int q = blockIdx.y; // 0: x list, 1: y list
    // the list's fields chosen by a select (not an index into the argument
    // struct), so that they stay in scalar registers
    const ps_list p = q ? pb.l[1] : pb.l[0];
    __shared__ int32_t wc[LB_I * (LB_T / WAVE)];
    // the segments j0, j0 + 1, ... that meet the tile: start, the record data
    // of their split (pivot rank, axis, buffer bit) and placement (LO, nlo)
    __shared__ int32_t win[LB_SEGW], wpi[LB_SEGW], wlo[LB_SEGW], wnl[LB_SEGW];
    __shared__ uint8_t wax[LB_SEGW], wbit[LB_SEGW];
    __shared__ int32_t wpre[LB_T / WAVE];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int32_t tile = blockIdx.x;
    if (!COUNT) {
        // moving lo records of the tiles before this one: the sum of their
        // counts (read from L2, reduced while the records load)
        int32_t part = 0;
        for (int32_t k = tid; k < tile; k += LB_T) part += p.tcnt[k];
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, WAVE);
        if (lane == 0) wpre[w] = part;
    }
    const int64_t tb = (int64_t)tile * LB_B, te = min(tb + LB_B, pb.n);
    const int32_t j0 = min(max(pb.tseg[tile], 0), pb.nseg - 1);
    {
        const int32_t jj = j0 + tid;
        const int32_t v = jj <= pb.nseg ? pb.start[jj] : INT32_MAX;
        win[tid] = v;
        if (jj < pb.nseg) {
            wpi[tid] = pb.pi[jj];
            wlo[tid] = p.LO[jj];
            wnl[tid] = pb.nlo[jj];
            wax[tid] = pb.axis[jj];
            wbit[tid] = p.bit[jj];
        }
        // segments of the window that begin before the tile's end
        const uint64_t in = __ballot(v < te);
        if (lane == 0) wc[w] = __popcll(in);
    }
    __syncthreads();
    int32_t nw = 0;
#pragma unroll
    for (int q2 = 0; q2 < LB_T / WAVE; ++q2) nw += wc[q2];
    __syncthreads();
    // fewer than LB_SEGW segments begin before the tile's end: the window holds
    // every segment of the tile; else (many small segments) look them up
    const bool inwin = nw < LB_SEGW;
    const int64_t base = tb + tid;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
    src_rec r[LB_I];
    uint64_t mk[LB_I];
    int32_t sg[LB_I]; // 2 x (window slot, or segment outside the window) + buffer bit of a moving record, else -1
    // three passes, so that the record loads are all in flight together: the
    // segment (window slot, or segment outside the window) and buffer of every
    // moving record, encoded 2 slot + bit (-1: the record stays or is past n);
    // the loads; the sides
    if (inwin) {
#pragma unroll
        for (int i = 0; i < LB_I; ++i) {
            const int64_t pos = base + (int64_t)i * LB_T;
            sg[i] = -1;
            if (pos < pb.n) {
                int32_t a0 = 0, a1 = nw - 1; // the last window entry <= pos
                while (a0 < a1) {
                    const int32_t mid = (a0 + a1 + 1) >> 1;
                    if (win[mid] <= pos) a0 = mid; else a1 = mid - 1;
                }
                if (wax[a0] != q) sg[i] = 2 * a0 + (wbit[a0] & 1); // this list moves in the segment
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < LB_I; ++i) {
            const int64_t pos = base + (int64_t)i * LB_T;
            sg[i] = -1;
            if (pos < pb.n) {
                int32_t a0 = j0, a1 = pb.nseg - 1;
                while (a0 < a1) {
                    const int32_t mid = (a0 + a1 + 1) >> 1;
                    if (pb.start[mid] <= pos) a0 = mid; else a1 = mid - 1;
                }
                if (pb.axis[a0] != q) sg[i] = 2 * a0 + (p.bit[a0] & 1);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < LB_I; ++i)
        if (sg[i] >= 0) r[i] = ((sg[i] & 1) ? p.buf1 : p.buf0)[base + (int64_t)i * LB_T];
#pragma unroll
    for (int i = 0; i < LB_I; ++i) {
        bool lo = false;
        if (sg[i] >= 0) {
            const int32_t j = sg[i] >> 1;
            const int ax = inwin ? wax[j] : pb.axis[j];
            lo = (ax ? r[i].ry : r[i].rx) < (inwin ? wpi[j] : pb.pi[j]);
        }
        mk[i] = __ballot(lo);
        if (lane == 0) wc[i * (LB_T / WAVE) + w] = __popcll(mk[i]);
    }
    __syncthreads();
    if (COUNT) {
        if (w == 0) {
            int32_t v = wc[lane];
#pragma unroll
            for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
            if (lane == 0) p.tcnt[tile] = v;
        }
        return;
    }
    if (w == 0) {
        // exclusive scan of the (stripe, wave) counts in stripe-major order
        const int32_t v = wc[lane];
        const int32_t inc = wave_incl_scan(v);
        wc[lane] = inc - v;
    }
    __syncthreads();
    int32_t carry = 0; // moving lo records of the tiles before
#pragma unroll
    for (int q2 = 0; q2 < LB_T / WAVE; ++q2) carry += wpre[q2];
#pragma unroll
    for (int i = 0; i < LB_I; ++i) {
        if (sg[i] < 0) continue;
        const int64_t pos = base + (int64_t)i * LB_T;
        const int32_t j = sg[i] >> 1;
        const bool lo = (mk[i] >> lane) & 1;
        const int32_t before = carry + wc[i * (LB_T / WAVE) + w] + __popcll(mk[i] & lt);
        const int32_t st = inwin ? win[j] : pb.start[j];
        const int32_t LOj = inwin ? wlo[j] : p.LO[j], nlj = inwin ? wnl[j] : pb.nlo[j];
        const uint8_t bj = (uint8_t)(sg[i] & 1);
        const int32_t rank = before - LOj; // lo records before pos in the segment
        int64_t dst = lo ? (int64_t)st + rank : (int64_t)st + nlj + (pos - st - rank);
        dst = dst < 0 ? 0 : (dst >= pb.n ? pb.n - 1 : dst); // never leave the array
        ((bj & 1) ? p.buf0 : p.buf1)[dst] = r[i];
    }
}

// ------------------------------------------------ subtree in LDS --
// Evaluation at the sources: once every segment holds at most SUB_S sources,
// one workgroup takes a segment through all its remaining splits in LDS and
// writes the box geometry, the per-level starts and the leaf order itself.
// Local point ids are positions in the segment's x list; the segment's y list
// is read too and mapped to local ids by binary search of its x ranks (the x
// list is sorted by x rank).  Sides are decided on ranks and rectangles come
// from the coordinates of the end points, as in the global steps, so the tree
// is the same.
#define SUB_S 2048
#define SUB_T 512
#define SUB_I (SUB_S / SUB_T)

struct subtree_args {
    const src_rec *lx[2], *ly[2]; // x and y lists after step k0 (two buffers each)
    const uint8_t *bx, *by;     // per step-k0 segment: the buffer holding its x / y list
    const double *xs, *ys;      // coordinates by rank
    const int32_t *px;          // original index by x rank
    const int32_t *sst;         // starts of the step-k0 segments (nseg0 + 1)
    int k0, L;
    int32_t nseg0;
    int64_t ns;
    double *centre, *radius;    // all levels
    int32_t *sstart;            // per-level starts, all levels
    int32_t *perm;
    int32_t *status;
    const double *src, *m;      // caller's sources and strengths
    double4 *srcs;              // sources with strengths in leaf order
    float2 *m32;                // FP32 strengths in leaf order, or NULL
};

__global__ void __launch_bounds__(SUB_T) k_subtree(subtree_args a)
{
    __shared__ int32_t rxl[SUB_S], ryl[SUB_S], pid[SUB_S]; // by local id
    __shared__ uint16_t lst[2][2][SUB_S];                   // [buffer][x or y list][position] -> local id
    __shared__ uint16_t st[2][SUB_S + 1];                   // sub-segment starts
    __shared__ uint16_t piv[SUB_S];                         // pivot local id per sub-segment
    __shared__ uint8_t axs[SUB_S];                          // split axis per sub-segment
    __shared__ uint16_t exs[2][SUB_S];                      // exclusive lo counts per position
    __shared__ int32_t sh[SUB_T / WAVE];
    const int tid = threadIdx.x;
    const int32_t g0 = blockIdx.x;
    const int32_t base = a.sst[g0];
    const int32_t n = min(max(a.sst[g0 + 1] - base, 0), SUB_S);
    const int32_t rmax = (int32_t)a.ns - 1; // ranks index the sorted coordinates
    // a thread's records, then their original indices, each set of loads in
    // flight together; position i = tid + u SUB_T
    {
        const src_rec *lx = a.lx[a.bx[g0] & 1] + base;
        int32_t rx[SUB_I], ry[SUB_I], ox[SUB_I];
#pragma unroll
        for (int u = 0; u < SUB_I; ++u) {
            const int i = tid + u * SUB_T;
            const src_rec r = i < n ? lx[i] : src_rec{0, 0};
            rx[u] = min(max(r.rx, 0), rmax);
            ry[u] = min(max(r.ry, 0), rmax);
        }
#pragma unroll
        for (int u = 0; u < SUB_I; ++u) ox[u] = a.px[rx[u]];
#pragma unroll
        for (int u = 0; u < SUB_I; ++u) {
            const int i = tid + u * SUB_T;
            if (i < n) {
                rxl[i] = rx[u];
                ryl[i] = ry[u];
                pid[i] = ox[u];
                lst[0][0][i] = (uint16_t)i;
            }
        }
    }
    // the y list of the same points, as local ids (its x ranks loaded first)
    int32_t yrx[SUB_I];
    {
        const src_rec *ly = a.ly[a.by[g0] & 1] + base;
#pragma unroll
        for (int u = 0; u < SUB_I; ++u) {
            const int i = tid + u * SUB_T;
            yrx[u] = i < n ? ly[i].rx : 0;
        }
    }
    __syncthreads();
    bool missing = false;
#pragma unroll
    for (int u = 0; u < SUB_I; ++u) {
        const int i = tid + u * SUB_T;
        if (i >= n) continue;
        const int32_t rx = yrx[u];
        int32_t lo_i = 0, hi_i = n - 1;
        while (lo_i < hi_i) {
            const int32_t mid = (lo_i + hi_i) >> 1;
            if (rxl[mid] < rx) lo_i = mid + 1; else hi_i = mid;
        }
        missing = missing || rxl[lo_i] != rx;
        lst[0][1][i] = (uint16_t)lo_i;
    }
    if (missing) atomicOr(a.status, FMM_ST_TREE_INCONSISTENT);
    if (tid == 0) {
        st[0][0] = 0;
        st[0][1] = (uint16_t)n;
    }
    __syncthreads();
    const int J = 2 * a.L - a.k0;
    int cur = 0;
    for (int j = 0; j <= J; ++j) {
        const int32_t nsub = 1 << j;
        const int kg = a.k0 + j;
        const bool even = (kg & 1) == 0, split = j < J;
        const int lev = kg >> 1;
        // (a) per sub-segment: rectangle, geometry on even steps, axis and pivot
        for (int32_t t = tid; t < nsub; t += SUB_T) {
            const int32_t s0 = st[cur][t], s1 = st[cur][t + 1], m = s1 - s0;
            double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
            if (m > 0) {
                x0 = a.xs[rxl[lst[cur][0][s0]]];
                x1 = a.xs[rxl[lst[cur][0][s1 - 1]]];
                y0 = a.ys[ryl[lst[cur][1][s0]]];
                y1 = a.ys[ryl[lst[cur][1][s1 - 1]]];
            }
            const double w = x1 - x0, h = y1 - y0;
            if (even) {
                const int64_t b = ((int64_t)g0 << j) + t;
                const int64_t gb = d_box_off(lev) + b;
                a.centre[2 * gb] = 0.5 * (x0 + x1);
                a.centre[2 * gb + 1] = 0.5 * (y0 + y1);
                a.radius[gb] = 0.5 * sqrt(w * w + h * h);
                a.sstart[d_start_off(lev) + b] = base + s0;
                if (g0 == a.nseg0 - 1 && t == nsub - 1)
                    a.sstart[d_start_off(lev) + (((int64_t)1) << (2 * lev))] = (int32_t)a.ns;
            }
            if (split) {
                const int ax = (w >= h) ? 0 : 1;
                axs[t] = (uint8_t)ax;
                piv[t] = m > 0 ? lst[cur][ax][s0 + m / 2] : 0;
            }
        }
        __syncthreads();
        if (!split) break;
        const int nxt = cur ^ 1;
        // (b) lo flags of both lists, block-wide exclusive scans.  The
        // sub-segment of position p is the last t with st[t] <= p; a thread's
        // positions are consecutive and both lists share the starts, so one
        // binary search and forward steps give all of them.
        bool lo[2][SUB_I];
        int32_t tseg[SUB_I];
        {
            const int p0 = tid * SUB_I;
            int32_t lo_t = 0, hi_t = nsub - 1;
            while (lo_t < hi_t) {
                const int32_t mid = (lo_t + hi_t + 1) >> 1;
                if (st[cur][mid] <= p0) lo_t = mid; else hi_t = mid - 1;
            }
#pragma unroll
            for (int u = 0; u < SUB_I; ++u) {
                while (lo_t + 1 < nsub && st[cur][lo_t + 1] <= p0 + u) ++lo_t;
                tseg[u] = lo_t;
            }
        }
        for (int q = 0; q < 2; ++q) {
            int32_t cnt = 0;
#pragma unroll
            for (int u = 0; u < SUB_I; ++u) {
                const int p = tid * SUB_I + u;
                bool f = false;
                if (p < n) {
                    const int32_t t = tseg[u];
                    const uint16_t id = lst[cur][q][p], pv = piv[t];
                    f = axs[t] ? (ryl[id] < ryl[pv]) : (rxl[id] < rxl[pv]);
                }
                lo[q][u] = f;
                cnt += f;
            }
            int32_t tot;
            int32_t e = block_excl_scan(cnt, sh, &tot);
#pragma unroll
            for (int u = 0; u < SUB_I; ++u) {
                const int p = tid * SUB_I + u;
                if (p < n) exs[q][p] = (uint16_t)e;
                e += lo[q][u];
            }
        }
        __syncthreads();
        // (c) stable partition of both lists into the other buffer
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int u = 0; u < SUB_I; ++u) {
                const int p = tid * SUB_I + u;
                if (p < n) {
                    const int32_t t = tseg[u];
                    const int32_t s0 = st[cur][t], m = st[cur][t + 1] - s0;
                    const int32_t r = exs[q][p] - exs[q][s0]; // lo positions before p in t
                    const int32_t dst = lo[q][u] ? s0 + r : s0 + m / 2 + (p - s0 - r);
                    lst[nxt][q][min(max(dst, 0), SUB_S - 1)] = lst[cur][q][p];
                }
            }
        }
        for (int32_t t = tid; t < nsub; t += SUB_T) {
            const int32_t s0 = st[cur][t], m = st[cur][t + 1] - s0;
            st[nxt][2 * t] = (uint16_t)s0;
            st[nxt][2 * t + 1] = (uint16_t)(s0 + m / 2);
        }
        if (tid == 0) st[nxt][2 * nsub] = (uint16_t)n;
        __syncthreads();
        cur = nxt;
    }
    // (d) leaf order: inside every leaf the sources by ascending original
    // index (rxl is free now: it holds the original index of each final position)
    int32_t *pidl = rxl;
    for (int p = tid; p < n; p += SUB_T) pidl[p] = pid[lst[cur][0][p]];
    __syncthreads();
    const int32_t nleaf = 1 << J;
    for (int p = tid; p < n; p += SUB_T) {
        int32_t lo_t = 0, hi_t = nleaf - 1;
        while (lo_t < hi_t) {
            const int32_t mid = (lo_t + hi_t + 1) >> 1;
            if (st[cur][mid] <= p) lo_t = mid; else hi_t = mid - 1;
        }
        const int32_t s0 = st[cur][lo_t], s1 = st[cur][lo_t + 1];
        const int32_t me = pidl[p];
        int32_t r = 0;
        for (int32_t k = s0; k < s1; ++k) r += pidl[k] < me;
        const int64_t pos = base + s0 + min(r, s1 - s0 - 1);
        a.perm[pos] = me;
        // the leaf-ordered sources (the gather of the global path)
        const int64_t j = min(max((int64_t)me, (int64_t)0), a.ns - 1);
        const double2 mm = reinterpret_cast<const double2 *>(a.m)[j];
        a.srcs[pos] = make_double4(a.src[2 * j], a.src[2 * j + 1], mm.x, mm.y);
        if (a.m32) a.m32[pos] = make_float2((float)mm.x, (float)mm.y);
        flag_nonfinite(!(isfinite(mm.x) && isfinite(mm.y)), a.status);
    }
}

// Leaf of every original index (as the sort key) and the identity values;
// a source's original index is px[rx].
__global__ void k_leaf_keys(const pt_rec *__restrict__ lx, int64_t n, uint64_t *__restrict__ keys,
                            int32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const pt_rec r = lx[i];
        const int64_t v = min(max((int64_t)r.idx, (int64_t)0), n - 1);
        keys[v] = (uint64_t)(uint32_t)r.seg;
        vals[i] = (int32_t)i;
    }
}
// For sources the leaf of position i is found in the leaf starts and the
// record read from the buffer that holds that leaf's x list.
__global__ void k_leaf_keys_src(const src_rec *__restrict__ lx0, const src_rec *__restrict__ lx1,
                                const uint8_t *__restrict__ bx, const int32_t *__restrict__ lst, int32_t nleaf,
                                const int32_t *__restrict__ px, int64_t n, uint64_t *__restrict__ keys,
                                int32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int32_t lo = 0, hi = nleaf - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (lst[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const src_rec r = ((bx[lo] & 1) ? lx1 : lx0)[i];
        const int64_t v = min(max((int64_t)px[min(max((int64_t)r.rx, (int64_t)0), n - 1)], (int64_t)0), n - 1);
        keys[v] = (uint64_t)(uint32_t)lo;
        vals[i] = (int32_t)i;
    }
}

// ------------------------------------------------------------- lists --
__device__ __forceinline__ bool theta_weak(double cbx, double cby, double rb, double csx,
                                           double csy, double rs, double theta)
{
    const double dx = cbx - csx;
    const double dy = cby - csy;
    const double d = sqrt(dx * dx + dy * dy);
    const double R = rb >= rs ? rb : rs;
    const double r = rb >= rs ? rs : rb;
    return d > 0.0 && R + theta * r <= theta * d;
}

// The criterion with the radii interchanged (leaf-level swap): r + theta R <= theta d.
__device__ __forceinline__ bool theta_swapped(double cbx, double cby, double rb, double csx,
                                              double csy, double rs, double theta)
{
    const double dx = cbx - csx;
    const double dy = cby - csy;
    const double d = sqrt(dx * dx + dy * dy);
    const double R = rb >= rs ? rb : rs;
    const double r = rb >= rs ? rs : rb;
    return d > 0.0 && r + theta * R <= theta * d;
}

struct list_args {
    const double *centre, *radius; // level l arrays (offset)
    const int32_t *psoff;          // level l-1 strong offsets (offset)
    const int32_t *sidx;           // global strong list array
    int32_t *wcnt, *scnt;          // counts (count pass)
    const int32_t *woff, *soff;    // level l offsets (fill pass, offset)
    int32_t *widx_out, *sidx_out;  // global arrays (fill pass)
    int32_t nbl;
    int32_t cap;
    double theta;
    int32_t *status;
    int swap;                      // finest level with the swapped criterion
    int32_t *mcnt, *pcnt;          // M2P / P2L counts (count pass)
    const int32_t *moff, *poff;    // M2P / P2L offsets (fill pass)
    int32_t *midx_out, *pidx_out;  // M2P / P2L lists (fill pass)
    int32_t lcap;                  // capacity of the M2P / P2L arrays
    const int32_t *hvy, *hcnt;     // heavy boxes of this level (level-local ids) and their count
    int32_t *hvy_next, *hcnt_next; // the same for the next level (fill pass appends), or NULL
    int32_t *hpart;                // per heavy box and part: its 4 class counts (count pass)
};

// A box whose candidate set (4 x its parent's strong count) exceeds
// LIST_HEAVY is shared by the 4 waves of a workgroup; the first LIST_HB
// workgroups of a launch take these boxes from the level's heavy list (filled
// by the previous level's fill pass), the others take one light box per wave.
// Clustered inputs put a few thousand strong boxes next to a large box, and
// one wave walking its children's candidates would set the launch's length.
#define LIST_HEAVY 512
#define LIST_HB 256
#define LIST_KP 16 // parts (of 4 waves) a heavy box is split into

struct list_cnt {
    int32_t w, s, m, p; // weak, strong, M2P, P2L
};

__device__ __forceinline__ bool list_heavy(const int32_t *psoff, int32_t b)
{
    const int32_t q = b >> 2;
    return 4 * (psoff[q + 1] - psoff[q]) > LIST_HEAVY;
}

// Candidates [kb, ke) of box b (candidate k: child k & 3 of the parent's strong
// entry e0 + k / 4): their class counts and, with FILL, the entries written
// from the positions in o on, in candidate order (ballot compaction).
// Classes: weak (M2L), strong (next level; P2P at the finest), and at the
// finest level with the swapped criterion M2P (this box larger) and P2L
// (candidate larger).
template <bool FILL>
__device__ __forceinline__ list_cnt list_range(const list_args &a, int32_t b, int32_t e0, int32_t kb, int32_t ke,
                                               double cbx, double cby, double rb, list_cnt o)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
    list_cnt n = {0, 0, 0, 0};
    for (int32_t k0 = kb; k0 < ke; k0 += WAVE) {
        const int32_t k = k0 + lane;
        const bool act = k < ke;
        int cls = 1; // 0 weak, 1 strong, 2 M2P, 3 P2L
        int32_t c = 0;
        if (act) {
            int32_t s = a.sidx[e0 + (k >> 2)];
            s = min(max(s, 0), (a.nbl >> 2) - 1);
            c = 4 * s + (k & 3);
            const double ccx = a.centre[2 * (int64_t)c], ccy = a.centre[2 * (int64_t)c + 1];
            const double rc = a.radius[c];
            if (c != b && theta_weak(cbx, cby, rb, ccx, ccy, rc, a.theta)) cls = 0;
            else if (a.swap && c != b && theta_swapped(cbx, cby, rb, ccx, ccy, rc, a.theta))
                cls = rb > rc ? 2 : 3;
        }
        const uint64_t mw = __ballot(act && cls == 0);
        const uint64_t ms = __ballot(act && cls == 1);
        const uint64_t mm = __ballot(act && cls == 2);
        const uint64_t mp = __ballot(act && cls == 3);
        if (FILL && act) {
            if (cls == 0) {
                const int32_t pos = o.w + n.w + __popcll(mw & lt);
                if (pos < a.cap) a.widx_out[pos] = c;
            } else if (cls == 1) {
                const int32_t pos = o.s + n.s + __popcll(ms & lt);
                if (pos < a.cap) a.sidx_out[pos] = c;
            } else if (cls == 2) {
                const int32_t pos = o.m + n.m + __popcll(mm & lt);
                if (pos < a.lcap) a.midx_out[pos] = c;
            } else {
                const int32_t pos = o.p + n.p + __popcll(mp & lt);
                if (pos < a.lcap) a.pidx_out[pos] = c;
            }
        }
        n.w += __popcll(mw);
        n.s += __popcll(ms);
        n.m += __popcll(mm);
        n.p += __popcll(mp);
    }
    return n;
}

// Fill pass: the list starts of box b, with the overflow check.
__device__ __forceinline__ list_cnt list_starts(const list_args &a, int32_t b, bool &over)
{
    list_cnt o = {a.woff[b], a.soff[b], 0, 0};
    over = a.woff[b + 1] > a.cap || a.soff[b + 1] > a.cap;
    if (a.swap) {
        o.m = a.moff[b];
        o.p = a.poff[b];
        over = over || a.moff[b + 1] > a.lcap || a.poff[b + 1] > a.lcap;
    }
    return o;
}

// Fill pass: a box whose children will be heavy at the next level enters that
// level's heavy list (the order of the list does not matter: each box writes
// its own positions).
__device__ __forceinline__ void list_next_heavy(const list_args &a, int32_t b, int32_t nstrong)
{
    if (a.hvy_next && 4 * nstrong > LIST_HEAVY) {
        const int32_t pos = atomicAdd(a.hcnt_next, 4);
        for (int i = 0; i < 4; ++i) {
            const int32_t c = 4 * b + i;
            a.hvy_next[pos + i] = c;
            // the next level's count pass adds the parts' counts to these
            a.wcnt[c] = 0;
            a.scnt[c] = 0;
            a.mcnt[c] = 0;
            a.pcnt[c] = 0;
        }
    }
}

template <bool FILL>
__global__ void __launch_bounds__(256) k_lists(list_args a)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const list_cnt zero = {0, 0, 0, 0};
    if ((int32_t)blockIdx.x >= LIST_HB) {
        // one light box per wave
        const int32_t b = ((int32_t)blockIdx.x - LIST_HB) * 4 + __builtin_amdgcn_readfirstlane(w);
        if (b >= a.nbl || list_heavy(a.psoff, b)) return;
        const int32_t q = b >> 2;
        const int32_t e0 = min(a.psoff[q], a.cap), e1 = min(a.psoff[q + 1], a.cap);
        const double cbx = a.centre[2 * (int64_t)b], cby = a.centre[2 * (int64_t)b + 1];
        const double rb = a.radius[b];
        list_cnt o = zero;
        if (FILL) {
            bool over;
            o = list_starts(a, b, over);
            if (lane == 0 && over) atomicOr(a.status, FMM_ST_LIST_OVERFLOW);
        }
        const list_cnt n = list_range<FILL>(a, b, e0, 0, 4 * (e1 - e0), cbx, cby, rb, o);
        if (lane == 0) {
            if (!FILL) {
                a.wcnt[b] = n.w;
                a.scnt[b] = n.s;
                if (a.swap) {
                    a.mcnt[b] = n.m;
                    a.pcnt[b] = n.p;
                }
            } else {
                list_next_heavy(a, b, n.s);
            }
        }
        return;
    }
    // heavy boxes: LIST_KP parts of 4 waves each; wave slot v = 4 part + wave
    // takes a contiguous range of 64-candidate chunks
    __shared__ list_cnt hc[4];
    const int32_t nh = min(*a.hcnt, a.nbl);
    for (int32_t it = blockIdx.x; it < nh * LIST_KP; it += LIST_HB) {
        const int32_t h = it / LIST_KP, part = it % LIST_KP;
        const int32_t b = min(max(a.hvy[h], 0), a.nbl - 1);
        const int32_t q = b >> 2;
        const int32_t e0 = min(a.psoff[q], a.cap), e1 = min(a.psoff[q + 1], a.cap);
        const int32_t ncand = 4 * (e1 - e0);
        const int32_t C = (ncand + 4 * LIST_KP * WAVE - 1) / (4 * LIST_KP * WAVE) * WAVE;
        const int32_t v = 4 * part + w;
        const int32_t kb = min(v * C, ncand), ke = min(kb + C, ncand);
        const double cbx = a.centre[2 * (int64_t)b], cby = a.centre[2 * (int64_t)b + 1];
        const double rb = a.radius[b];
        int32_t *hp = a.hpart + ((int64_t)h * LIST_KP) * 4;
        const list_cnt n = list_range<false>(a, b, e0, kb, ke, cbx, cby, rb, zero);
        if (lane == 0) hc[w] = n;
        __syncthreads();
        if (!FILL) {
            if (threadIdx.x == 0) {
                list_cnt t = zero;
                for (int u = 0; u < 4; ++u) {
                    t.w += hc[u].w; t.s += hc[u].s; t.m += hc[u].m; t.p += hc[u].p;
                }
                hp[4 * part] = t.w;
                hp[4 * part + 1] = t.s;
                hp[4 * part + 2] = t.m;
                hp[4 * part + 3] = t.p;
                // integer sums: exact in any order
                if (t.w) atomicAdd(a.wcnt + b, t.w);
                if (t.s) atomicAdd(a.scnt + b, t.s);
                if (a.swap) {
                    if (t.m) atomicAdd(a.mcnt + b, t.m);
                    if (t.p) atomicAdd(a.pcnt + b, t.p);
                }
            }
        } else {
            bool over;
            list_cnt o = list_starts(a, b, over);
            for (int k = 0; k < part; ++k) {
                o.w += hp[4 * k]; o.s += hp[4 * k + 1]; o.m += hp[4 * k + 2]; o.p += hp[4 * k + 3];
            }
            for (int u = 0; u < w; ++u) {
                o.w += hc[u].w; o.s += hc[u].s; o.m += hc[u].m; o.p += hc[u].p;
            }
            if (part == 0 && threadIdx.x == 0) {
                if (over) atomicOr(a.status, FMM_ST_LIST_OVERFLOW);
                int32_t ns = 0;
                for (int k = 0; k < LIST_KP; ++k) ns += hp[4 * k + 1];
                list_next_heavy(a, b, ns);
            }
            list_range<true>(a, b, e0, kb, ke, cbx, cby, rb, o);
        }
        __syncthreads();
    }
}


__global__ void k_root(int32_t *sstep, int32_t ns, int32_t *tstep, int32_t nt)
{
    sstep[0] = 0; sstep[1] = ns;
    tstep[0] = 0; tstep[1] = nt;
}

__global__ void k_lists_root(int32_t *woff, int32_t *soff, int32_t *sidx, int32_t *hcnt, int L)
{
    woff[0] = 0; woff[1] = 0;
    soff[0] = 0; soff[1] = 1;
    sidx[0] = 0;
    for (int l = 0; l <= L + 1; ++l) hcnt[l] = 0;
}

__global__ void k_gather(const double *__restrict__ src, const double *__restrict__ m,
                         const int32_t *__restrict__ perm, int64_t ns, double4 *__restrict__ srcs,
                         float2 *__restrict__ m32, const double *__restrict__ tgt,
                         const int32_t *__restrict__ tperm, int64_t nt, double2 *__restrict__ tgts,
                         int32_t *__restrict__ status)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < ns) {
        const int64_t j = min(max((int64_t)perm[i], (int64_t)0), ns - 1);
        srcs[i] = make_double4(src[2 * j], src[2 * j + 1], m[2 * j], m[2 * j + 1]);
        if (m32) m32[i] = make_float2((float)m[2 * j], (float)m[2 * j + 1]);
        bad = !(isfinite(m[2 * j]) && isfinite(m[2 * j + 1]));
    }
    flag_nonfinite(bad, status);
    if (i < nt) {
        const int64_t j = min(max((int64_t)tperm[i], (int64_t)0), nt - 1);
        tgts[i] = make_double2(tgt[2 * j], tgt[2 * j + 1]);
    }
}

#define WS(T, off) reinterpret_cast<T *>(a.ws + (off))
#define CK(x) do { hipError_t e__ = (x); if (e__ != hipSuccess) return e__; } while (0)

static inline unsigned nblk256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t fmm_build_tree(const fmm_tree_args &a, const double *m, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    const int L = a.L;
    const int64_t ns = a.ns, nt = a.nt;
    uint64_t *k0s = WS(uint64_t, lay.keys[0]), *k1 = WS(uint64_t, lay.keys[1]);
    int32_t *v0 = WS(int32_t, lay.vals[0]), *v1 = WS(int32_t, lay.vals[1]);
    int32_t *hist = WS(int32_t, lay.hist);
    int32_t *bsum = WS(int32_t, lay.bsum);
    int32_t *perm = WS(int32_t, lay.perm), *tperm = nt ? WS(int32_t, lay.tperm) : nullptr;
    // source lists: x in buffers xb[0], xb[1], y in yb[0], yb[1], with a
    // buffer bit per segment and list (current and next step); target lists:
    // [0] x-ordered, [1] y-ordered, [2], [3] partition outputs
    src_rec *xb[2], *yb[2];
    for (int i = 0; i < 2; ++i) {
        xb[i] = WS(src_rec, lay.srec) + (int64_t)i * ns;
        yb[i] = WS(src_rec, lay.srec) + (int64_t)(2 + i) * ns;
    }
    uint8_t *bits = WS(uint8_t, lay.sbits);
    const int64_t bstride = lay.nleaf + 1;
    uint8_t *bxc = bits, *byc = bits + bstride, *bxn = bits + 2 * bstride, *byn = bits + 3 * bstride;
    int32_t *nlox = WS(int32_t, lay.seg_nlox), *nloy = WS(int32_t, lay.seg_nloy);
    int32_t *LOY = WS(int32_t, lay.seg_LOy);
    int32_t *tsegm = WS(int32_t, lay.stseg);
    int32_t *tcnt = WS(int32_t, lay.stcnt);
    pt_rec *tl[4];
    for (int i = 0; i < 4; ++i) tl[i] = nt ? WS(pt_rec, lay.trec) + (int64_t)i * nt : nullptr;
    int32_t *px = WS(int32_t, lay.srank), *py = px + ns, *rxo = px + 2 * ns, *ryo = px + 3 * ns;
    double *xs = WS(double, lay.scoord), *ys = xs + ns;
    int32_t *sstep = WS(int32_t, lay.sstep), *tstep = WS(int32_t, lay.tstep);
    uint8_t *axis = WS(uint8_t, lay.seg_axis);
    double *pc = WS(double, lay.seg_pc);
    int32_t *pi = WS(int32_t, lay.seg_pi);
    int32_t *nlo = WS(int32_t, lay.seg_nlo), *tlo = WS(int32_t, lay.seg_tlo);
    int32_t *LO = WS(int32_t, lay.seg_LO), *TLO = WS(int32_t, lay.seg_TLO);
    int32_t *sstart = WS(int32_t, lay.sstart), *tstart = WS(int32_t, lay.tstart);
    double *centre = WS(double, lay.centre), *radius = WS(double, lay.radius);
    // partition tile states: 4 lists of lay.lbtiles words, then 4 tickets
    uint64_t *lbst = WS(uint64_t, lay.lbst);
    int32_t *ticket = reinterpret_cast<int32_t *>(lbst + 4 * lay.lbtiles);
    const int64_t lb_n = 4 * lay.lbtiles + 2;

    // presort into (coordinate, index) order; source records of ranks.  With
    // a side stream the y presort runs there, beside the x one, in the record
    // buffers (2 x 8 + 2 x 4 bytes per source of their 32, unused until the
    // records are built) with a histogram of its own.
    if (a.side) {
        uint64_t *ky0 = WS(uint64_t, lay.srec), *ky1 = ky0 + ns;
        int32_t *vy0 = reinterpret_cast<int32_t *>(ky1 + ns), *vy1 = vy0 + ns;
        CK(hipEventRecord(a.ev_fork, st));
        CK(hipStreamWaitEvent(a.side, a.ev_fork, 0));
        CK(presort(a.src, ns, 1, ky0, ky1, vy0, vy1, WS(int32_t, lay.hist2), bsum, py, ys, a.status, a.side, ryo));
        CK(presort(a.src, ns, 0, k0s, k1, v0, v1, hist, bsum, px, xs, a.status, st, rxo));
        CK(hipEventRecord(a.ev_join, a.side));
        CK(hipStreamWaitEvent(st, a.ev_join, 0));
    } else {
        CK(presort(a.src, ns, 0, k0s, k1, v0, v1, hist, bsum, px, xs, a.status, st, rxo));
        CK(presort(a.src, ns, 1, k0s, k1, v0, v1, hist, bsum, py, ys, a.status, st, ryo));
    }
    k_srec_init<<<nblk256(ns), 256, 0, st>>>(px, py, rxo, ryo, ns, xb[0], yb[0]);
    k_fill_u8<<<nblk256(2 * bstride), 256, 0, st>>>(bxc, 2 * bstride); // the root: both lists in buffer 0
    if (nt) {
        CK(presort(a.tgt, nt, 0, k0s, k1, v0, v1, hist, bsum, tperm, nullptr, a.status, st));
        k_trec_init<<<nblk256(nt), 256, 0, st>>>(a.tgt, tperm, nt, tl[0]);
        CK(presort(a.tgt, nt, 1, k0s, k1, v0, v1, hist, bsum, tperm, nullptr, a.status, st));
        k_trec_init<<<nblk256(nt), 256, 0, st>>>(a.tgt, tperm, nt, tl[1]);
    }
    k_root<<<1, 1, 0, st>>>(sstep, (int32_t)ns, tstep, (int32_t)nt);
    // At the sources, the steps from k0 on run in LDS (k_subtree): k0 is the
    // first step whose segments (at most ceil(ns / 2^k) sources) fit.
    int k0 = -1;
    if (nt == 0)
        for (int k = 0; k <= 2 * L; ++k)
            if (((ns + (((int64_t)1) << k) - 1) >> k) <= SUB_S && (((int64_t)1) << (2 * L - k)) <= SUB_S) {
                k0 = k;
                break;
            }
    const int32_t st_tiles = (int32_t)((ns + LB_B - 1) / LB_B), tt_tiles = (int32_t)((nt + LB_B - 1) / LB_B);
    int64_t soff_k = 0; // offset of step k's starts
    for (int k = 0; k <= 2 * L; ++k) {
        const int32_t nseg = (int32_t)(((int64_t)1) << k);
        if (k == k0) {
            subtree_args ta;
            ta.lx[0] = xb[0];
            ta.lx[1] = xb[1];
            ta.ly[0] = yb[0];
            ta.ly[1] = yb[1];
            ta.bx = bxc;
            ta.by = byc;
            ta.xs = xs;
            ta.ys = ys;
            ta.px = px;
            ta.status = a.status;
            ta.sst = sstep + soff_k;
            ta.k0 = k0;
            ta.L = L;
            ta.nseg0 = nseg;
            ta.ns = ns;
            ta.centre = centre;
            ta.radius = radius;
            ta.sstart = sstart;
            ta.perm = perm;
            ta.src = a.src;
            ta.m = m;
            ta.srcs = WS(double4, lay.srcs);
            ta.m32 = lay.mixed == 1 ? WS(float2, lay.m32) : nullptr;
            k_subtree<<<(unsigned)nseg, SUB_T, 0, st>>>(ta);
            CK(hipGetLastError());
            break;
        }
        const bool split = k < 2 * L;
        const bool even = (k % 2) == 0;
        const int l = k / 2;
        seg_args sa;
        sa.slx[0] = xb[0]; sa.slx[1] = xb[1];
        sa.sly[0] = yb[0]; sa.sly[1] = yb[1];
        sa.bx = bxc; sa.by = byc; sa.bx_next = bxn; sa.by_next = byn;
        sa.nlox = nlox; sa.nloy = nloy;
        sa.tseg = split ? tsegm : nullptr;
        sa.ntiles = st_tiles;
        const bool fuse = split && nseg <= 1024; // one block holds every segment: scans in k_seg
        sa.LOx = fuse ? LO : nullptr;
        sa.LOy = fuse ? LOY : nullptr;
        sa.TLO = fuse && nt ? TLO : nullptr;
        sa.xs = xs; sa.ys = ys;
        sa.tlx = tl[0]; sa.tly = tl[1];
        sa.sst = sstep + soff_k; sa.tst = tstep + soff_k;
        sa.sst_next = split ? sstep + soff_k + nseg + 1 : nullptr;
        sa.tst_next = split ? tstep + soff_k + nseg + 1 : nullptr;
        sa.axis = axis; sa.pc = pc; sa.pi = pi; sa.nlo = nlo; sa.tlo = tlo;
        sa.centre = even ? centre + 2 * box_off(l) : nullptr;
        sa.radius = even ? radius + box_off(l) : nullptr;
        sa.lvl_sst = even ? sstart + start_off(l) : nullptr;
        sa.lvl_tst = even ? tstart + start_off(l) : nullptr;
        sa.lb_clear = split ? lbst : nullptr;
        sa.lb_n = split ? lb_n : 0;
        sa.nseg = nseg; sa.ns = ns; sa.nt = nt;
        if (fuse) k_seg<<<1, 1024, 0, st>>>(sa);
        else k_seg<<<nblk256(nseg), 256, 0, st>>>(sa);
        CK(hipGetLastError());
        if (!split) break;
        // exclusive scans of the lo counts of the moving source lists (and the
        // targets' lo counts) over segments
        if (!fuse) {
            fmm_scan_jobs J;
            memset(&J, 0, sizeof(J));
            const int64_t bstr = fmm_scan_blocks(nseg) + 1;
            J.in[0] = nlox; J.out[0] = LO; J.bs[0] = hist;
            J.in[1] = nloy; J.out[1] = LOY; J.bs[1] = hist + bstr;
            J.in[2] = tlo; J.out[2] = TLO; J.bs[2] = hist + 2 * bstr;
            CK(fmm_scan_i32_jobs(J, nt ? 3 : 2, nseg, st));
        }
        {
            ps_batch pb;
            for (int q = 0; q < 2; ++q) {
                ps_list &p = pb.l[q];
                p.buf0 = q ? yb[0] : xb[0];
                p.buf1 = q ? yb[1] : xb[1];
                p.bit = q ? byc : bxc;
                p.LO = q ? LOY : LO;
                p.tcnt = tcnt + (int64_t)q * (st_tiles + 1);
            }
            pb.start = sstep + soff_k;
            pb.nlo = nlo;
            pb.axis = axis;
            pb.pi = pi;
            pb.tseg = tsegm;
            pb.n = ns;
            pb.nseg = nseg;
            pb.ntiles = st_tiles;
            pb.status = a.status;
            k_part_src<true><<<dim3((unsigned)st_tiles, 2), LB_T, 0, st>>>(pb);
            k_part_src<false><<<dim3((unsigned)st_tiles, 2), LB_T, 0, st>>>(pb);
            CK(hipGetLastError());
        }
        if (nt) {
            lb_batch pb;
            pb.axis = axis; pb.pc = pc; pb.pi = pi; pb.status = a.status;
            for (int q = 0; q < 2; ++q) {
                lb_list &p = pb.l[q];
                p.in = tl[q]; p.out = tl[2 + q];
                p.state = lbst + (int64_t)(2 + q) * lay.lbtiles;
                p.ticket = ticket + 2 + q;
                p.start = tstep + soff_k; p.nlo = tlo; p.LO = TLO;
                p.n = nt; p.nseg = nseg; p.ntiles = tt_tiles;
            }
            k_part_lb<pt_rec><<<dim3((unsigned)tt_tiles, 2), LB_T, 0, st>>>(pb);
            CK(hipGetLastError());
            for (int q = 0; q < 2; ++q) {
                pt_rec *u = tl[q]; tl[q] = tl[2 + q]; tl[2 + q] = u;
            }
        }
        uint8_t *tb = bxc; bxc = bxn; bxn = tb;
        tb = byc; byc = byn; byn = tb;
        soff_k += nseg + 1;
    }
    // leaf order with ascending original index inside every leaf: a stable
    // sort of the identity by leaf number
    const int passes = (2 * L + 7) / 8;
    if (k0 < 0) {
        // (the last step left the leaf starts at step 2L and their bits in bxc)
        k_leaf_keys_src<<<nblk256(ns), 256, 0, st>>>(xb[0], xb[1], bxc, sstep + soff_k, (int32_t)nbox(L), px, ns,
                                                     k0s, v0);
        if (passes > 0) CK(radix_sort(ns, passes, k0s, k1, v0, v1, hist, bsum, perm, st));
        else CK(hipMemcpyAsync(perm, v0, (size_t)ns * 4, hipMemcpyDeviceToDevice, st));
    }
    if (nt) {
        k_leaf_keys<<<nblk256(nt), 256, 0, st>>>(tl[0], nt, k0s, v0);
        if (passes > 0) CK(radix_sort(nt, passes, k0s, k1, v0, v1, hist, bsum, tperm, st));
        else CK(hipMemcpyAsync(tperm, v0, (size_t)nt * 4, hipMemcpyDeviceToDevice, st));
    }
    if (k0 < 0) { // (the LDS subtree writes the leaf-ordered sources itself)
        int64_t nmax = ns > nt ? ns : nt;
        k_gather<<<nblk256(nmax), 256, 0, st>>>(a.src, m, perm, ns, WS(double4, lay.srcs),
                                                lay.mixed == 1 ? WS(float2, lay.m32) : nullptr, a.tgt,
                                                tperm, nt, nt ? WS(double2, lay.tgts) : nullptr, a.status);
        CK(hipGetLastError());
    }
    return hipSuccess;
}

// Interaction lists, level by level (count, scan, fill).
hipError_t fmm_build_lists(const fmm_tree_args &a, hipStream_t st)
{
    const fmm_layout &lay = *a.lay;
    const int L = a.L;
    double *centre = WS(double, lay.centre), *radius = WS(double, lay.radius);
    int32_t *woff = WS(int32_t, lay.woff), *soff = WS(int32_t, lay.soff);
    int32_t *widx = WS(int32_t, lay.widx), *sidx = WS(int32_t, lay.sidx);
    int32_t *wcnt = WS(int32_t, lay.wcnt), *scnt = WS(int32_t, lay.scnt);
    int32_t *lbsum = WS(int32_t, lay.lbsum);
    int32_t *hvy = WS(int32_t, lay.lhvy), *hcnt = WS(int32_t, lay.lhcnt);
    k_lists_root<<<1, 1, 0, st>>>(woff, soff, sidx, hcnt, L);
    if (!a.swap) {
        k_fill_i32<<<nblk256(nbox(L) + 1), 256, 0, st>>>(WS(int32_t, lay.moff), nbox(L) + 1, 0);
        k_fill_i32<<<nblk256(nbox(L) + 1), 256, 0, st>>>(WS(int32_t, lay.poff), nbox(L) + 1, 0);
    }
    for (int l = 1; l <= L; ++l) {
        list_args la;
        la.centre = centre + 2 * box_off(l);
        la.radius = radius + box_off(l);
        la.psoff = soff + start_off(l - 1);
        la.sidx = sidx;
        la.wcnt = wcnt; la.scnt = scnt;
        la.woff = woff + start_off(l);
        la.soff = soff + start_off(l);
        la.widx_out = widx; la.sidx_out = sidx;
        la.nbl = (int32_t)nbox(l);
        la.cap = (int32_t)lay.listcap;
        la.theta = a.theta;
        la.status = a.status;
        la.swap = (l == L) && a.swap;
        la.mcnt = WS(int32_t, lay.mcnt);
        la.pcnt = WS(int32_t, lay.pcnt);
        la.moff = WS(int32_t, lay.moff);
        la.poff = WS(int32_t, lay.poff);
        la.midx_out = WS(int32_t, lay.midx);
        la.pidx_out = WS(int32_t, lay.pidx);
        la.lcap = (int32_t)lay.leafcap;
        la.hvy = hvy + box_off(l);
        la.hcnt = hcnt + l;
        la.hvy_next = l < L ? hvy + box_off(l + 1) : nullptr;
        la.hcnt_next = l < L ? hcnt + l + 1 : nullptr;
        la.hpart = WS(int32_t, lay.lhpart);
        // LIST_HB workgroups for the heavy boxes, then 4 light boxes per workgroup
        const unsigned nwb = (unsigned)(LIST_HB + (nbox(l) + 3) / 4);
        k_lists<false><<<nwb, 256, 0, st>>>(la);
        {
            // weak and strong offsets (and at the finest level M2P and P2L) in one set of launches
            fmm_scan_jobs J;
            memset(&J, 0, sizeof(J));
            const int64_t bstr = fmm_scan_blocks(nbox(l)) + 1;
            J.in[0] = wcnt; J.out[0] = woff + start_off(l); J.base[0] = woff + start_off(l - 1) + nbox(l - 1);
            J.in[1] = scnt; J.out[1] = soff + start_off(l); J.base[1] = soff + start_off(l - 1) + nbox(l - 1);
            J.in[2] = la.mcnt; J.out[2] = WS(int32_t, lay.moff);
            J.in[3] = la.pcnt; J.out[3] = WS(int32_t, lay.poff);
            for (int q = 0; q < 4; ++q) J.bs[q] = lbsum + q * bstr;
            CK(fmm_scan_i32_jobs(J, la.swap ? 4 : 2, nbox(l), st));
        }
        k_lists<true><<<nwb, 256, 0, st>>>(la);
        CK(hipGetLastError());
    }
    return hipSuccess;
}
