// HIP kernels (gfx950) for the filtered Paterson-Stockmeyer series.
//
// Every stage of the method is one "row-accumulation" stage:
//
//     out_r = D_tau( e_r + sum_t a_t * R_t )                          (*)
//
// where the terms (a_t, R_t) of output row r are
//   - product stage (eq. 11, eq. 14): a_t = A_rk, R_t = row k of B, for the
//     stored k of row r of A in ascending order;
//   - coefficient-sum stage (eq. 13): a_t = c_j, R_t = row r of P_j
//     (P_0 = I), in ascending j;
// e_r is row r of an optional extra matrix (the block Bhat in a Horner step)
// and D_tau drops x iff x == 0 or |x| < tau.  Each row is owned by one
// 64-lane wavefront, which accumulates the terms strictly in order with one
// fma per term into a per-row accumulator, so the result does not depend on
// the launch configuration and matches a sequential row-wise product.
//
// Per stage:  analyze  -> per-row column window [lo, lo+W), upper bound of
//                         stored entries, and the exact empty-row test
//             scan     -> slack output offsets
//             numeric  -> structure bitmap of the window, rank of every
//                         column = its slot in a dense sorted accumulator,
//                         ordered fma accumulation, drop test fused into
//                         the (sorted, coalesced) write-out.
// Rows whose window or structure does not fit the shared-memory workspace
// are finished by a second kernel with per-wave workspace in device memory.
#include "fps_device.h"

#include <algorithm>
#include <climits>

namespace fps {
namespace {

// Shared-memory tiers of the numeric kernel.  Narrow: windows of up to 6144
// columns and 320 structural entries, 19.5 KB per four-wavefront block and at
// most 64 VGPRs, so eight wavefronts per SIMD.  Wide (rows that do not fit
// the narrow tier): 6912 columns and 512 entries, 26.5 KB per block, six
// blocks per CU.  Larger rows take the device-memory kernel.
constexpr int kNarrowWords = 192, kNarrowCap = 320;
// small-row tier (four rows per wavefront): window words and entries per row
constexpr int kSmallWords = 96, kSmallCap = 96;
constexpr int kWideWords = 216, kWideCap = 512;
// Rows beyond the wide tier: in the device-memory kernel, with structure and
// accumulator still in shared memory up to 8192 columns and 2048 entries
// (77 KB per block, two blocks per CU), the parked values in device memory.
constexpr int kDevWords = 256, kDevCap = 2048;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Orders this wavefront's shared/device memory accesses around the call
// (lanes of one wavefront see each other's stores after it).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T x)
{
    const int l = lane();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T x)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, G);
    return x;
}
template <int G, typename T>
__device__ __forceinline__ T group_min(T x)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, G));
    return x;
}
template <int G, typename T>
__device__ __forceinline__ T group_max(T x)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) x = max(x, __shfl_xor(x, d, G));
    return x;
}

// ---- cross-lane operations on DPP (data-parallel primitives) ------------------
// A DPP row is 16 lanes.  These replace shuffles through the LDS crossbar
// (ds_bpermute, one LDS round trip per step) on the paths every row takes;
// all lanes of the wavefront must be active.
constexpr int kDppQuadSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;  // lane i <- lane 7 - i of its half row
constexpr int kDppRowMirror = 0x140;     // lane i <- lane 15 - i of its row
constexpr int kDppRowShr1 = 0x111;       // lane i <- lane i - n of its row (0 below)
constexpr int kDppRowBcast15 = 0x142;    // lanes of row k+1 <- lane 15 of row k
constexpr int kDppRowBcast31 = 0x143;    // lanes of rows 2, 3 <- lane 31

template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, kRowMask, 0xF, false);
}
template <int kCtrl, typename T>
__device__ __forceinline__ T dpp_val(T x)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp32<kCtrl>(__builtin_bit_cast(uint32_t, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint64_t lo = dpp32<kCtrl>((uint32_t)u), hi = dpp32<kCtrl>((uint32_t)(u >> 32));
        return __builtin_bit_cast(T, (hi << 32) | lo);
    }
}
struct OpMax {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpMin {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a < b ? a : b; }
};
struct OpSum {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a + b; }
};
// Every lane gets the reduction over its 16-lane row.
template <typename Op, typename T>
__device__ __forceinline__ T row_reduce(T x)
{
    const Op op;
    x = op(x, dpp_val<kDppQuadSwap1>(x));
    x = op(x, dpp_val<kDppQuadSwap2>(x));
    x = op(x, dpp_val<kDppRowHalfMirror>(x));
    x = op(x, dpp_val<kDppRowMirror>(x));
    return x;
}
// The reduction over the wavefront (uniform).
template <typename Op, typename T>
__device__ __forceinline__ T wave_reduce(T x)
{
    x = row_reduce<Op>(x);
    const Op op;
    T r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (sizeof(T) == 4) {
            r[k] = __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 16 * k));
        } else {
            const uint64_t u = __builtin_bit_cast(uint64_t, x);
            const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 16 * k);
            const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 16 * k);
            r[k] = __builtin_bit_cast(T, (hi << 32) | lo);
        }
    }
    return op(op(r[0], r[1]), op(r[2], r[3]));
}
// Inclusive prefix sum over the wavefront.
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x)
{
    x += dpp32<kDppRowShr1>(x);
    x += dpp32<kDppRowShr1 + 1>(x);
    x += dpp32<kDppRowShr1 + 3>(x);
    x += dpp32<kDppRowShr1 + 7>(x);
    x += dpp32<kDppRowBcast15, 0xA>(x);
    x += dpp32<kDppRowBcast31, 0xC>(x);
    return x;
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Block order that keeps consecutive logical blocks (consecutive rows) on one
// XCD: the hardware hands blocks to the 8 XCDs round-robin, so block b runs on
// XCD b % 8; logical ranges are contiguous per XCD and the map is a bijection.
__device__ __forceinline__ int64_t xcd_logical_block()
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / kXcds, rm = nb % kXcds, x = b % kXcds, i = b / kXcds;
    return (int64_t)x * q + (int64_t)min(x, rm) + i;
}

__device__ __forceinline__ void flag_error(const StageArgs& P, unsigned long long bit)
{
    atomicOr(&P.ctr->errors, bit);
}

// Block-wide sum of one value per thread; result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum_256(T x, T* sh)
{
    x = group_sum<kWave>(x);
    if (lane() == 0) sh[threadIdx.x / kWave] = x;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / kWave; ++i) t += sh[i];
    return t;
}

// Inclusive scan over the threads of a block; *total gets the block's sum.
__device__ __forceinline__ int64_t block_incl_scan(int64_t x, int64_t* sh, int64_t* total)
{
    const int64_t inc = wave_incl_sum(x);
    const int w = threadIdx.x / kWave;
    if (lane() == kWave - 1) sh[w] = inc;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int i = 0; i < kBlock / kWave; ++i) {
        const int64_t v = sh[i];
        pre += (i < w) ? v : 0;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + inc;
}

// Exclusive scan, in place, of the per-block totals x[0..nblk) written by a
// row kernel; the grand total goes to *grand.  One block.
__global__ void __launch_bounds__(kBlock) k_block_scan(int64_t* x, int64_t nblk, int64_t* grand)
{
    __shared__ int64_t sh[kBlock / kWave];
    // thread t owns the contiguous range [t * per, (t + 1) * per)
    const int64_t per = (nblk + kBlock - 1) / kBlock;
    const int64_t b = min<int64_t>((int64_t)threadIdx.x * per, nblk), e = min<int64_t>(b + per, nblk);
    int64_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += x[i];
    int64_t tot = 0;
    int64_t run = block_incl_scan(sum, sh, &tot) - sum;
    for (int64_t i = b; i < e; ++i) {
        const int64_t v = x[i];
        x[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) *grand = tot;
}

// ---------------------------------------------------------------------------
// Structure words of a row from its ascending columns, G lanes at a time (G a
// power of two up to 64; a group is G consecutive lanes that all make the
// same calls).  The columns of one word sit on consecutive lanes, so a
// segmented OR over lane distances 1, 2, 4, ... leaves each word's bits on
// its first lane.  The last word of a batch stays open, since the next batch
// may continue it.
// ---------------------------------------------------------------------------
template <int G>
struct WordBuilder {
    uint2* out;       // first word of the row
    int32_t n = 0;    // words written
    uint32_t cw = 0;  // the open word
    uint32_t cm = 0;  // its bits (0: no open word)

    // Columns c of group lanes [0, cnt), ascending, above the previous batch's.
    __device__ __forceinline__ void add(int32_t c, int32_t cnt)
    {
        if (cnt <= 0) return;
        const int gl = lane() & (G - 1);
        const int gb = lane() & (kWave - G);
        const bool v = gl < cnt;
        const uint32_t w = (uint32_t)c >> 5;
        uint32_t m = v ? (1u << (c & 31)) : 0u;
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const uint32_t ow = __shfl_down(w, d, G);
            const uint32_t om = __shfl_down(m, d, G);
            if (gl + d < cnt && ow == w) m |= om;
        }
        const uint32_t pw = __shfl_up(w, 1, G);
        const bool lead = v && (gl == 0 || pw != w);
        const unsigned long long bal = __ballot(lead);
        const unsigned long long gm = (G == kWave) ? bal : (bal >> gb) & ((1ull << (G & 63)) - 1ull);
        const int nseg = __popcll(gm);
        const int seg = __popcll(gm & ((1ull << gl) - 1ull));
        const uint32_t w0 = __shfl(w, 0, G), m0 = __shfl(m, 0, G);
        const bool cont = cm != 0u && w0 == cw;  // the first word continues the open one
        uint32_t om = cm;
        if (cont) om |= m0;
        const int first = cont ? 1 : 0;
        if (nseg == first) {  // the batch only continued the open word
            cm = om;
            return;
        }
        if (om != 0u) {
            if (gl == 0) out[n] = make_uint2(cw, om);
            n += 1;
        }
        if (lead && seg >= first && seg < nseg - 1) out[n + seg - first] = make_uint2(w, m);
        n += nseg - 1 - first;
        const int lastl = 63 - __clzll(gm);
        cw = __shfl(w, lastl, G);
        cm = __shfl(m, lastl, G);
    }
    // Closes the open word; returns the number of words of the row.
    __device__ __forceinline__ int32_t finish()
    {
        if (cm != 0u) {
            if ((lane() & (G - 1)) == 0) out[n] = make_uint2(cw, cm);
            n += 1;
            cm = 0u;
        }
        return n;
    }
};

// The same for a whole wavefront, with the ORs of each word's bits done in
// shared memory (`seg`: 64 words per wavefront) instead of by shuffles.
struct WaveWordBuilder {
    uint2* out;       // first word of the row
    uint32_t* seg;    // this wavefront's 64 segment masks
    int32_t n = 0;    // words written
    uint32_t cw = 0;  // the open word
    uint32_t cm = 0;  // its bits (0: no open word)

    // Columns c of lanes [0, cnt), ascending, above the previous batch's.
    __device__ __forceinline__ void add(int32_t c, int32_t cnt)
    {
        if (cnt <= 0) return;
        const int l = lane();
        const bool v = l < cnt;
        const uint32_t w = (uint32_t)c >> 5;
        const uint32_t pw = __shfl_up(w, 1, kWave);
        const bool lead = v && (l == 0 || pw != w);
        const unsigned long long L = __ballot(lead);
        const int nseg = __popcll(L);
        // segment of lane l: leaders at or below it, minus one
        const int si = (int)lanes_below(L) + (lead ? 1 : 0) - 1;
        if (l < nseg) seg[l] = 0u;
        wave_sync();
        if (v) atomicOr(&seg[si], 1u << (c & 31));
        wave_sync();
        const uint32_t m = lead ? seg[si] : 0u;
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)w, 0);
        const uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane((int)m, 0);
        const bool cont = cm != 0u && w0 == cw;  // the first word continues the open one
        uint32_t om = cm;
        if (cont) om |= m0;
        const int first = cont ? 1 : 0;
        if (nseg == first) {
            cm = om;
            return;
        }
        if (om != 0u) {
            if (l == 0) out[n] = make_uint2(cw, om);
            n += 1;
        }
        if (lead && si >= first && si < nseg - 1) out[n + si - first] = make_uint2(w, m);
        n += nseg - 1 - first;
        const int lastl = 63 - __clzll(L);
        cw = (uint32_t)__builtin_amdgcn_readlane((int)w, lastl);
        cm = (uint32_t)__builtin_amdgcn_readlane((int)m, lastl);
        wave_sync();  // the next batch clears seg
    }
    __device__ __forceinline__ int32_t finish()
    {
        if (cm != 0u) {
            if (lane() == 0) out[n] = make_uint2(cw, cm);
            n += 1;
            cm = 0u;
        }
        return n;
    }
};

// Row summary (a rounded-up float keeps amax an upper bound).
__device__ __forceinline__ RowInfo row_info(int64_t len, int32_t first, int32_t last, double amax)
{
    RowInfo q;
    q.len = (int32_t)len;
    q.first = len > 0 ? first : 1;
    q.last = len > 0 ? last : 0;
    q.amax = __double2float_ru(amax);
    return q;
}

// One 16-byte load of a row summary.
__device__ __forceinline__ RowInfo load_info(const RowInfo* p)
{
    const int4 v = *reinterpret_cast<const int4*>(p);
    RowInfo q;
    q.len = v.x;
    q.first = v.y;
    q.last = v.z;
    q.amax = __int_as_float(v.w);
    return q;
}

// ---------------------------------------------------------------------------
// Row summaries and structure words of a canonical CSR.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_rowinfo_csr(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, int64_t n, RowInfo* info,
                                                        uint2* sw, int32_t* nw)
{
    constexpr int G = 16;
    const int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
    const int gl = threadIdx.x % G;
    if (r >= n) return;
    const int64_t b = rp[r], e = rp[r + 1];
    double m = 0.0;
    WordBuilder<G> wb{sw + b};
    for (int64_t p0 = b; p0 < e; p0 += G) {
        const int64_t p = p0 + gl;
        int32_t c = 0;
        if (p < e) {
            c = col[p];
            m = fmax(m, fabs(val[p]));
        }
        wb.add(c, (int32_t)min<int64_t>(G, e - p0));
    }
    const int32_t words = wb.finish();
    m = row_reduce<OpMax>(m);
    if (gl == 0) {
        info[r] = row_info(e - b, e > b ? col[b] : 1, e > b ? col[e - 1] : 0, m);
        nw[r] = words;
    }
}

// ---------------------------------------------------------------------------
// Device-side check of a canonical CSR (row pointers, column order/range,
// finite values).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_validate_csr(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, int64_t n, int64_t nnz,
                                                         unsigned long long* err)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(err, kErrBadCsr);
    if (r >= n) return;
    const int64_t b = rp[r], e = rp[r + 1];
    if (b > e || b < 0 || e > nnz) {
        atomicOr(err, kErrBadCsr);
        return;
    }
    int32_t prev = -1;
    for (int64_t p = b; p < e; ++p) {
        const int32_t c = col[p];
        const double v = val[p];
        if (c <= prev || c >= n || !isfinite(v)) {
            atomicOr(err, kErrBadCsr);
            return;
        }
        prev = c;
    }
}

// ---------------------------------------------------------------------------
// Analysis: window, upper bound, exact empty-row test.
//
// For a product row, |e_r| + sum_k |A_rk| max|B_k,:| bounds every entry of
// (*) in exact arithmetic (the row maxima are stored rounded up to float,
// which only enlarges the bound); the computed values exceed it by at most a
// relative (terms+2) u, far below the 1e-6 margin folded into skip_tau, so a
// row whose bound is below skip_tau would be dropped entirely by D_tau and is
// marked empty without computing it.
// ---------------------------------------------------------------------------
constexpr int kAnalyzeLanes = 16;  // lanes per row in the product analysis
constexpr int kAnalyzeShiftProduct = 4;  // log2(kBlock / kAnalyzeLanes) rows per block
constexpr int kAnalyzeShiftSum = 8;      // log2(kBlock) rows per block
static_assert(kBlock / kAnalyzeLanes == (1 << kAnalyzeShiftProduct) && kBlock == (1 << kAnalyzeShiftSum),
              "analysis block geometry");

__global__ void __launch_bounds__(kBlock) k_analyze_product(StageArgs P)
{
    constexpr int G = kAnalyzeLanes;
    __shared__ unsigned long long sh[4][kBlock / G];
    __shared__ int64_t ubs[kBlock / G];
    __shared__ int64_t blk_total;
    const int64_t blk = xcd_logical_block();
    const int64_t r = (blk * kBlock + threadIdx.x) / G;
    const int gl = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    unsigned long long prod_done = 0, prod_skip = 0, row_skip = 0, a_nnz = 0;
    if (r < P.n) {
        int32_t lo = INT_MAX, hi = -1;
        int64_t prod = 0;
        double bnd = 0.0;
        const int64_t pb = P.A.beg[r], pe = P.A.end[r];
        a_nnz = (unsigned long long)(pe - pb);
#pragma unroll 4
        for (int64_t p = pb + gl; p < pe; p += G) {
            // an empty row adds nothing (len 0, amax 0); every field is
            // used unconditionally, so the summary is one 16-byte load
            const int32_t k = P.A.col[p];
            const RowInfo q = load_info(P.B.info + k);
            lo = min(lo, q.len > 0 ? q.first : INT_MAX);
            hi = max(hi, q.len > 0 ? q.last : -1);
            prod += q.len;
            bnd += fabs(P.A.val[p]) * (double)q.amax;
        }
        int64_t elen = 0;
        double emax = 0.0;
        if (P.has_e && gl == 0) {
            const RowInfo q = load_info(P.E.info + r);
            elen = q.len;
            if (elen > 0) {
                lo = min(lo, q.first);
                hi = max(hi, q.last);
                emax = (double)q.amax;
            }
        }
        if (P.has_blk) {  // fused coefficient block: |block entries| <= sum_t |c_t| max|M_t[r,:]|
            for (int t = gl; t < P.T.n; t += G) {  // the group's lanes share the terms
                if (P.T.beg[t] == nullptr) {
                    lo = min(lo, (int32_t)r);
                    hi = max(hi, (int32_t)r);
                    elen += 1;
                    emax += fabs(P.T.coef[t]);
                } else {
                    const RowInfo q = load_info(P.T.info[t] + r);
                    if (q.len > 0) {
                        lo = min(lo, q.first);
                        hi = max(hi, q.last);
                        elen += q.len;
                        emax += fabs(P.T.coef[t]) * (double)q.amax;
                    }
                }
            }
        }
        static_assert(G == 16, "a product row is one DPP row");
        lo = row_reduce<OpMin>(lo);
        hi = row_reduce<OpMax>(hi);
        prod = row_reduce<OpSum>(prod);
        bnd = row_reduce<OpSum>(bnd);
        elen = row_reduce<OpSum>(elen);
        emax = row_reduce<OpSum>(emax);
        if (gl == 0) {
            const bool empty = (prod == 0 && elen == 0);
            const double skip_tau = P.tau_row ? P.tau_row[r] * P.skip_rel : P.skip_tau;
            const bool skip = !empty && skip_tau > 0.0 && (emax + bnd) < skip_tau;
            int32_t W = 0;
            int64_t ub = 0;
            if (!empty && !skip) {
                // the window starts on a 32-column boundary, so that its bitmap
                // words are whole words of the column space
                ub = min(prod + elen, (int64_t)(hi - lo + 1));
                lo &= ~31;
                W = hi - lo + 1;
            }
            P.W[r] = W;
            P.lo[r] = lo;
            P.prod[r] = prod;
            ubs[grp] = ub;
            // products counted as multiply-adds: the B rows plus, when fused, the block terms
            const int64_t work = prod + (P.has_blk ? elen : 0);
            if (skip) {
                prod_skip = (unsigned long long)work;
                row_skip = 1;
            } else {
                prod_done = (unsigned long long)work;
                if (P.prod_acc) P.prod_acc[r] += work;
            }
        }
    }
    if (gl == 0) {
        sh[0][grp] = prod_done;
        sh[1][grp] = prod_skip;
        sh[2][grp] = row_skip;
        sh[3][grp] = a_nnz;
        if (r >= P.n) ubs[grp] = 0;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock / G; ++i) t += sh[threadIdx.x][i];
        // kPartProducts, kPartProductsSkipped, kPartRowsSkipped, then kPartANnz
        P.part[(threadIdx.x < 3 ? threadIdx.x : kPartANnz) * P.part_stride + blk] = t;
    }
    if (threadIdx.x == kBlock - 1) {  // offsets of the block's rows within the block
        int64_t run = 0;
        for (int i = 0; i < kBlock / G; ++i) {
            const int64_t t = ubs[i];
            ubs[i] = run;
            run += t;
        }
        blk_total = run;
    }
    __syncthreads();
    if (gl == 0 && r < P.n) P.out.off[r] = ubs[grp];
    if (threadIdx.x == 0) P.blk_pre[blk] = blk_total;
}

__global__ void __launch_bounds__(kBlock) k_analyze_sum(StageArgs P)
{
    __shared__ unsigned long long sh[kBlock / kWave];
    __shared__ int64_t osh[kBlock / kWave];
    const int64_t blk = xcd_logical_block();
    const int64_t r = blk * kBlock + threadIdx.x;
    unsigned long long prod_done = 0;
    int64_t ubv = 0;
    if (r < P.n) {
        int32_t lo = INT_MAX, hi = -1;
        int64_t prod = 0;
#pragma unroll 4
        for (int t = 0; t < P.T.n; ++t) {
            if (P.T.beg[t] == nullptr) {
                lo = min(lo, (int32_t)r);
                hi = max(hi, (int32_t)r);
                prod += 1;
            } else {
                const RowInfo q = load_info(P.T.info[t] + r);
                if (q.len > 0) {
                    lo = min(lo, q.first);
                    hi = max(hi, q.last);
                    prod += q.len;
                }
            }
        }
        int32_t W = 0;
        int64_t ub = 0;
        if (prod > 0) {
            ub = min(prod, (int64_t)(hi - lo + 1));
            lo &= ~31;  // whole words of the column space
            W = hi - lo + 1;
        }
        P.W[r] = W;
        P.lo[r] = lo;
        P.prod[r] = prod;
        ubv = ub;
        prod_done = (unsigned long long)prod;
        if (P.prod_acc) P.prod_acc[r] += prod;
    }
    const unsigned long long t = block_sum_256(prod_done, sh);
    if (threadIdx.x == 0) {
        P.part[kPartProducts * P.part_stride + blk] = t;
        P.part[kPartProductsSkipped * P.part_stride + blk] = 0;
        P.part[kPartRowsSkipped * P.part_stride + blk] = 0;
        P.part[kPartANnz * P.part_stride + blk] = 0;
    }
    int64_t total = 0;
    const int64_t inc = block_incl_scan(ubv, osh, &total);
    if (r < P.n) P.out.off[r] = inc - ubv;
    if (threadIdx.x == 0) P.blk_pre[blk] = total;
}

// ---------------------------------------------------------------------------
// Numeric stage.
// ---------------------------------------------------------------------------
constexpr int kChunk = kWave;  // terms handled per chunk: lane t holds term t

// Short-row batches look up the term of each product in the staged prefix
// counts of the chunk.
struct WaveStage {
    int32_t excl[kChunk];  // exclusive prefix of the term row lengths
    int64_t beg[kChunk];   // first entry of the term's row
};

// Once the row's values have moved to registers, the accumulator holds the
// structural column list of the row (int32, slot order) for the write-out.
template <int kWords, int kCap>
struct LdsWave {
    static_assert(kCap % kWave == 0, "the parked values cover the accumulator exactly");
    static constexpr int kPark = kCap / kWave;  // parked values per lane
    uint2 bmp[kWords + 1];  // per 32 window columns: .x structure bits, .y set bits in earlier words;
                            // then the guard word
    double acc[kCap + 1];   // then the spare slot
    WaveStage st;
};
constexpr int kU = 4;                     // flattened batch: kU sub-batches of 64 products
constexpr int kStep = 2 * kWave;          // per-term step: 128 entries of one term row

__device__ __forceinline__ uint32_t rank_of(const uint2* bmp, uint32_t d)
{
    const uint2 w = bmp[d >> 5];
    return w.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(w.x, 0u, d));
}

// The same by column: the window starts on a word boundary, so with
// bw = bmp - (lo >> 5) the column's word is bw[c >> 5] and its bit c & 31.
// The guard column lo + guard ranks to the spare slot.
__device__ __forceinline__ uint32_t rank_col(const uint2* bw, int32_t c)
{
    const uint2 w = bw[(uint32_t)c >> 5];
    return w.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(w.x, 0u, (uint32_t)c));
}

__device__ __forceinline__ int32_t sgpr(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t sgpr64(int64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t readlane64(int64_t x, int i)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)x, i);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)x >> 32), i);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlaned(double x, int i)
{
    return __longlong_as_double(readlane64(__double_as_longlong(x), i));
}

enum TermSource : int { kSrcProducts = 0, kSrcCoefs = 1 };

// Terms of row r: entries [tb, te) of row r of A (products) or the
// coefficient terms 0..T.n-1.
__device__ __forceinline__ void term_range(const StageArgs& P, int src, int64_t r, int64_t* tb, int64_t* te)
{
    if (src == kSrcProducts) {
        *tb = P.A.beg[r];
        *te = P.A.end[r];
    } else {
        *tb = 0;
        *te = P.T.n;
    }
}

// One chunk of terms in registers: lane t holds term t0 + t (zero-length
// padding past the last term).
struct Chunk {
    int32_t len;     // entries of the term row
    int32_t nw;      // structure words of the term row
    int32_t incl;    // inclusive prefix of len over the lanes
    int64_t beg;     // first entry of the term row; -1: identity row (P_0)
    double a;        // weight
    int32_t total;   // uniform: products of the chunk
    int32_t nterms;  // uniform
    int32_t maxlen;  // uniform: longest term row of the chunk
};

__device__ __forceinline__ Chunk load_chunk(const StageArgs& P, int src, int64_t r, int64_t t0, int64_t te)
{
    const int l = lane();
    const int64_t t = t0 + l;
    Chunk c;
    c.len = 0;
    c.nw = 0;
    c.beg = 0;
    c.a = 0.0;
    if (t < te) {
        if (src == kSrcProducts) {
            const int32_t k = P.A.col[t];
            c.a = P.A.val[t];
            c.beg = P.B.beg[k];
            c.len = (int32_t)(P.B.end[k] - c.beg);
            c.nw = P.B.nw[k];
        } else {
            // both row pointers of the term are read at once, then both
            // offsets of row r (the identity term reads zeros from the dummy
            // entries): two round trips instead of three
            const int ti = (int)t;
            c.a = P.T.coef[ti];
            const int64_t* bp = P.T.beg[ti];
            const int64_t* ep = P.T.end[ti];
            const bool ident = bp == nullptr;
            const int64_t* zero = reinterpret_cast<const int64_t*>(P.dummy_val);
            const int64_t b = *(ident ? zero : bp + r);
            const int64_t e = *(ident ? zero : ep + r);
            const int32_t nwv = *(ident ? reinterpret_cast<const int32_t*>(zero) : P.T.nw[ti] + r);
            c.beg = ident ? -1 : b;
            c.len = ident ? 1 : (int32_t)(e - b);
            c.nw = ident ? 1 : nwv;
        }
    }
    c.incl = (int32_t)wave_scan_u32((uint32_t)c.len);
    c.total = __builtin_amdgcn_readlane(c.incl, kWave - 1);
    c.maxlen = wave_reduce<OpMax>(c.len);
    c.nterms = (int32_t)min<int64_t>(kChunk, te - t0);
    return c;
}

__device__ __forceinline__ void stage_chunk(const Chunk& c, WaveStage& st)
{
    const int l = lane();
    wave_sync();  // earlier readers of the staging area are done
    st.excl[l] = c.incl - c.len;
    st.beg[l] = c.beg;
    wave_sync();
}

// Largest term index i of the chunk with excl[i] <= q.
__device__ __forceinline__ int find_term(const WaveStage& st, int32_t q)
{
    int k = 0;
#pragma unroll
    for (int step = kChunk / 2; step >= 1; step >>= 1)
        if (st.excl[k + step] <= q) k += step;
    return k;
}

// Marks window offset d (clamped to the guard offset: bit 0 of the guard word
// records a column outside the window, which the row information of
// consistent operands excludes).
template <bool kGlobal>
__device__ __forceinline__ void mark_d(uint32_t d, uint32_t guard, uint8_t* bytes, uint2* bmp)
{
    d = min(d, guard);
    if (kGlobal)
        bytes[d] = 1;
    else
        atomicOr(&bmp[d >> 5].x, 1u << (d & 31u));
}

// ---- flattened batches (short term rows) ------------------------------------
// Products q0 + j*64 + lane of the chunk.  Every lane issues its loads (lanes
// without a product read a zeroed dummy row), so loads stay in flight until
// the values are used.

template <int U>
struct Batch {
    int32_t c[U];
    double v[U];
    int kidx[U];
    bool ok[U];
};

// Products only: coefficient terms always take the per-term path, whose term
// index is uniform across the wavefront.
template <bool kNeedV, int U>
__device__ __forceinline__ void gather(const StageArgs& P, const WaveStage& st, int32_t q0, int32_t total, Batch<U>& b)
{
    const int l = lane();
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int32_t q = q0 + j * kWave + l;
        b.ok[j] = q < total;
        const int k = find_term(st, b.ok[j] ? q : total - 1);
        b.kidx[j] = k;
        const int64_t b0 = st.beg[k];
        const int32_t* cp = P.dummy_col;
        const double* vp = P.dummy_val;
        int64_t e = l;
        if (b.ok[j]) {
            cp = P.B.col;
            vp = P.B.val;
            e = b0 + (q - st.excl[k]);
        }
        b.c[j] = cp[e];
        b.v[j] = kNeedV ? vp[e] : 0.0;
    }
}

template <bool kGlobal, int U>
__device__ __forceinline__ void mark_batch(int32_t lo, uint32_t guard, const Batch<U>& b, uint8_t* bytes, uint2* bmp)
{
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (b.ok[j]) mark_d<kGlobal>((uint32_t)(b.c[j] - lo), guard, bytes, bmp);
}

// acc[rank] = fma(a, v, acc[rank]) in term order: each 64-product sub-batch
// is applied one term at a time (the products of one term have distinct
// columns, so a term's read-modify-writes never collide).
template <int U>
__device__ __forceinline__ void accumulate_batch(const Chunk& c, int32_t q0, int32_t lo, uint32_t guard,
                                                 const Batch<U>& b, const uint2* bmp, double* acc)
{
    const uint2* bw = bmp - (lo >> 5);
    const int32_t gcol = lo + (int32_t)guard;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int32_t qj = q0 + j * kWave;
        if (qj >= c.total) break;
        const double v = b.v[j];
        const bool ok = b.ok[j];
        const uint32_t slot = rank_col(bw, ok ? b.c[j] : gcol);
        const int last = min(kWave - 1, c.total - qj - 1);
        const int kf = __builtin_amdgcn_readlane(b.kidx[j], 0);
        const int kl = __builtin_amdgcn_readlane(b.kidx[j], last);
        for (int kk = kf; kk <= kl; ++kk) {
            const double a = readlaned(c.a, kk);
            if (ok && b.kidx[j] == kk) acc[slot] = fma(a, v, acc[slot]);
            wave_sync();
        }
    }
}

// ---- per-term groups (long term rows) ------------------------------------------
// kGroup terms at a time.  Each term row is addressed through a buffer
// resource whose size is the row's length, so the loads of lanes past the end
// of the row return zeros without touching memory; the first kStep entries of
// each of the group's rows are loaded together (two per lane), then the terms
// are applied one after the other.  Entries beyond kStep (rows longer than
// 128) are handled right after their term's first part.

constexpr int kGroup = 3;  // terms per group (products; coefficient terms go two at a time, which keeps
                           // the register budget while the main part is parked in registers)
__host__ __device__ constexpr int group_size(int src) { return src == 0 ? kGroup : 2; }
constexpr int kRsrcWord3 = 0x00020000;  // raw (unswizzled, stride 0) buffer of 32-bit elements

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, int32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kRsrcWord3);
}

// Uniform description of one term.
struct TermInfo {
    int32_t len;  // entries of the term row; 0: no term
    bool ident;   // identity row (coefficient term of P_0): the single entry (r, 1)
    double a;     // weight
};
struct TermDesc {
    TermInfo t;
    __amdgpu_buffer_rsrc_t rc, rv;
};

// Term i of the chunk (i may point past the chunk's terms: no term).
template <int SRC, bool kNeedV>
__device__ __forceinline__ TermDesc term_desc(const StageArgs& P, int64_t t0, const Chunk& c, int i)
{
    TermDesc h;
    const int il = min(i, kChunk - 1);
    h.t.len = (i < c.nterms) ? __builtin_amdgcn_readlane(c.len, il) : 0;
    const int64_t beg = readlane64(c.beg, il);
    h.t.a = kNeedV ? readlaned(c.a, il) : 0.0;
    h.t.ident = SRC == kSrcCoefs && h.t.len > 0 && beg < 0;
    // no term, or the identity (whose entry is not read): an empty buffer,
    // whose loads return zeros without touching memory, so the base address
    // does not matter
    const int32_t real = h.t.ident ? 0 : h.t.len;
    uintptr_t cb, vb;
    if (SRC == kSrcProducts) {
        cb = reinterpret_cast<uintptr_t>(P.B.col);
        vb = reinterpret_cast<uintptr_t>(P.B.val);
    } else {
        const int ti = min((int)t0 + il, kMaxTerms - 1);
        cb = reinterpret_cast<uintptr_t>(P.T.col[ti]);
        vb = reinterpret_cast<uintptr_t>(P.T.val[ti]);
    }
    h.rc = row_rsrc(reinterpret_cast<const void*>(cb + (uintptr_t)beg * 4u), real * 4);
    h.rv = row_rsrc(reinterpret_cast<const void*>(vb + (uintptr_t)beg * 8u), real * 8);
    return h;
}

// Entries e0 + lane and e0 + 64 + lane of a term row (zeros past its end).
struct Part {
    int32_t c0, c1;
    double v0, v1;
};

template <bool kNeedV>
__device__ __forceinline__ Part load_part(const TermDesc& h, int32_t e0)
{
    const int32_t i = e0 + lane();
    Part p;
    p.c0 = __builtin_amdgcn_raw_buffer_load_b32(h.rc, i * 4, 0, 0);
    p.c1 = __builtin_amdgcn_raw_buffer_load_b32(h.rc, i * 4 + kWave * 4, 0, 0);
    if (kNeedV) {
        p.v0 = __longlong_as_double((long long)__builtin_amdgcn_raw_buffer_load_b64(h.rv, i * 8, 0, 0));
        p.v1 = __longlong_as_double((long long)__builtin_amdgcn_raw_buffer_load_b64(h.rv, i * 8 + kWave * 8, 0, 0));
    } else {
        p.v0 = p.v1 = 0.0;
    }
    return p;
}

// Structure pass over one part.
template <bool kGlobal>
__device__ __forceinline__ void mark_part(const TermInfo& h, int32_t e0, const Part& p, int64_t r, int32_t lo,
                                          uint32_t guard, uint8_t* bytes, uint2* bmp)
{
    const int l = lane();
    const int32_t c0 = h.ident ? (int32_t)r : p.c0;
    if (e0 + l < h.len) mark_d<kGlobal>((uint32_t)(c0 - lo), guard, bytes, bmp);
    if (h.len > e0 + kWave && e0 + kWave + l < h.len) mark_d<kGlobal>((uint32_t)(p.c1 - lo), guard, bytes, bmp);
}

struct Slots {
    uint32_t s0, s1;
};

// Accumulator slots of a part's entries; lanes without an entry get the spare
// slot.  Every column of the row lies in the window (checked after the
// structure pass).  kBoth: the second half of the part as well (the spare
// slot for every lane if the row ends in the first half).  kFull: the row
// fills the first half (no lane of it needs the spare slot).
template <bool kBoth, bool kFull = false>
__device__ __forceinline__ Slots part_slots(const TermInfo& h, int32_t e0, const Part& p, int64_t r, int32_t lo,
                                            uint32_t guard, const uint2* bmp)
{
    const int l = lane();
    const int32_t c0 = h.ident ? (int32_t)r : p.c0;
    const uint2* bw = bmp - (lo >> 5);
    const int32_t gcol = lo + (int32_t)guard;
    Slots s;
    s.s0 = rank_col(bw, (kFull || e0 + l < h.len) ? c0 : gcol);
    s.s1 = kBoth ? rank_col(bw, (e0 + kWave + l < h.len) ? p.c1 : gcol) : 0u;
    return s;
}

// acc[slot] = fma(a, v, acc[slot]) for a part's entries (one term: distinct
// columns, so no two lanes touch one slot other than the spare).
__device__ __forceinline__ void accumulate_part(const TermInfo& h, int32_t e0, const Part& p, const Slots& s,
                                                double* acc)
{
    const double v0 = h.ident ? 1.0 : p.v0;
    if (h.len > e0 + kWave) {
        const double x0 = fma(h.a, v0, acc[s.s0]);
        const double x1 = fma(h.a, p.v1, acc[s.s1]);
        acc[s.s0] = x0;
        acc[s.s1] = x1;
    } else {
        acc[s.s0] = fma(h.a, v0, acc[s.s0]);
    }
}

// Issues the loads of the first part of the group's term rows.
template <int SRC, bool kNeedV>
__device__ __forceinline__ void issue_group(const StageArgs& P, int64_t t0, const Chunk& c, int i0, TermInfo* h,
                                            Part* p)
{
#pragma unroll
    for (int g = 0; g < group_size(SRC); ++g) {
        const TermDesc d = term_desc<SRC, kNeedV>(P, t0, c, i0 + g);
        h[g] = d.t;
        p[g] = load_part<kNeedV>(d, 0);
    }
}

// Applies a loaded group: structure marks, or the ranks of the whole group
// first (the bitmap is read-only then) and the read-modify-writes strictly
// term by term.  Rows longer than kStep continue right after their first part.
template <int SRC, bool kAccum, bool kGlobal>
__device__ __forceinline__ void run_group(const StageArgs& P, int64_t r, int64_t t0, const Chunk& c, int i0,
                                          const TermInfo* h, const Part* p, int32_t lo, uint32_t guard,
                                          uint8_t* bytes, uint2* bmp, double* acc)
{
    if (!kAccum) {
#pragma unroll
        for (int g = 0; g < group_size(SRC); ++g) {
            if (h[g].len == 0) continue;
            mark_part<kGlobal>(h[g], 0, p[g], r, lo, guard, bytes, bmp);
            if (h[g].len > kStep) {
                const TermDesc d = term_desc<SRC, false>(P, t0, c, i0 + g);
                for (int32_t e0 = kStep; e0 < h[g].len; e0 += kStep)
                    mark_part<kGlobal>(h[g], e0, load_part<false>(d, e0), r, lo, guard, bytes, bmp);
            }
        }
    } else {
        // the ranks of the whole group first, without branches between the
        // bitmap reads: second halves for every term if any term needs them
        Slots s[kGroup];
        bool two = false, full = true;
#pragma unroll
        for (int g = 0; g < group_size(SRC); ++g) {
            two = two || h[g].len > kWave;
            full = full && h[g].len >= kWave;
        }
        if (full) {  // every term row fills its first half (the usual case of long rows)
#pragma unroll
            for (int g = 0; g < group_size(SRC); ++g)
                s[g] = part_slots<true, true>(h[g], 0, p[g], r, lo, guard, bmp);
        } else if (two) {
#pragma unroll
            for (int g = 0; g < group_size(SRC); ++g) s[g] = part_slots<true>(h[g], 0, p[g], r, lo, guard, bmp);
        } else {
#pragma unroll
            for (int g = 0; g < group_size(SRC); ++g) s[g] = part_slots<false>(h[g], 0, p[g], r, lo, guard, bmp);
        }
#pragma unroll
        for (int g = 0; g < group_size(SRC); ++g) {
            if (h[g].len == 0) continue;
            accumulate_part(h[g], 0, p[g], s[g], acc);
            wave_sync();
            if (h[g].len > kStep) {
                const TermDesc d = term_desc<SRC, true>(P, t0, c, i0 + g);
                for (int32_t e0 = kStep; e0 < h[g].len; e0 += kStep) {
                    const Part q = load_part<true>(d, e0);
                    accumulate_part(h[g], e0, q, part_slots<true>(h[g], e0, q, r, lo, guard, bmp), acc);
                    wave_sync();
                }
            }
        }
    }
}

// The terms of one chunk, kGroup at a time.  (Keeping the next group's loads
// in flight as well costs more in occupancy than it saves.)
template <int SRC, bool kAccum, bool kGlobal>
__device__ __forceinline__ void per_term_pass(const StageArgs& P, int64_t r, int64_t t0, const Chunk& c, int32_t lo,
                                              uint32_t guard, uint8_t* bytes, uint2* bmp, double* acc)
{
    for (int i0 = 0; i0 < c.nterms; i0 += group_size(SRC)) {
        TermInfo h[kGroup];
        Part p[kGroup];
        issue_group<SRC, kAccum>(P, t0, c, i0, h, p);
        run_group<SRC, kAccum, kGlobal>(P, r, t0, c, i0, h, p, lo, guard, bytes, bmp, acc);
    }
}

// Chunks whose term rows all fit one wavefront (at most 64 entries)
// accumulate kShortGroup terms at a time, one load per lane and term: the
// same registers as a group of kGroup terms with two halves each, half the
// dependent round trips.
constexpr int kShortGroup = 6;

template <int SRC>
__device__ __forceinline__ void short_group_pass(const StageArgs& P, int64_t r, int64_t t0, const Chunk& c,
                                                 int32_t lo, uint32_t guard, const uint2* bmp, double* acc)
{
    const int l = lane();
    const uint2* bw = bmp - (lo >> 5);
    const int32_t gcol = lo + (int32_t)guard;
    for (int i0 = 0; i0 < c.nterms; i0 += kShortGroup) {
        TermInfo h[kShortGroup];
        int32_t cc[kShortGroup];
        double vv[kShortGroup];
#pragma unroll
        for (int g = 0; g < kShortGroup; ++g) {
            const TermDesc d = term_desc<SRC, true>(P, t0, c, i0 + g);
            h[g] = d.t;
            cc[g] = __builtin_amdgcn_raw_buffer_load_b32(d.rc, l * 4, 0, 0);
            vv[g] = __longlong_as_double((long long)__builtin_amdgcn_raw_buffer_load_b64(d.rv, l * 8, 0, 0));
        }
        uint32_t sl[kShortGroup];
#pragma unroll
        for (int g = 0; g < kShortGroup; ++g) {
            const int32_t col = h[g].ident ? (int32_t)r : cc[g];
            sl[g] = rank_col(bw, (l < h[g].len) ? col : gcol);
        }
#pragma unroll
        for (int g = 0; g < kShortGroup; ++g) {
            if (h[g].len == 0) continue;
            const double v = h[g].ident ? 1.0 : vv[g];
            acc[sl[g]] = fma(h[g].a, v, acc[sl[g]]);
            wave_sync();
        }
    }
}

// Short product term rows (at most kPackedMax entries) packed over the
// lanes: `per` terms per instruction with `wd` = the chunk's longest row
// lanes each, so each lane knows its term without a search.  The ranks of an
// instruction's entries come first, then one read-modify-write round per
// term, in term order (two terms may share a column).
constexpr int kPackedMax = 32;

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src)
{
    const uint32_t lo = __shfl((uint32_t)x, src, kWave);
    const uint32_t hi = __shfl((uint32_t)(x >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double shfl_f64(double x, int src)
{
    return __longlong_as_double((long long)shfl_u64((uint64_t)__double_as_longlong(x), src));
}

// With `seen` (one zeroed word per accumulator slot, or null), an
// instruction's entries are not applied one term per round: each lane ORs its
// term's bit into its slot's word, and its round is the number of earlier
// terms of the instruction on the same slot, so a round applies, for every
// slot, its next term in term order, and an instruction takes as many rounds
// as the most terms sharing one slot.
__device__ __forceinline__ void packed_pass(const StageArgs& P, const Chunk& c, int32_t lo, uint32_t guard,
                                            const uint2* bmp, double* acc, uint32_t* seen)
{
    const int l = lane();
    const int32_t wd = max(c.maxlen, 1);
    const int32_t per = kWave / wd;
    const int32_t sub = l / wd, idx = l - sub * wd;
    const bool lane_on = sub < per;
    const uint2* bw = bmp - (lo >> 5);
    const int32_t gcol = lo + (int32_t)guard;
    // entry idx of the term held by lane ti of the chunk
    auto fetch = [&](int32_t ti, bool* ok, double* a, int32_t* cl, double* v) {
        const int src = min(ti, kChunk - 1);
        const uint64_t beg = shfl_u64((uint64_t)c.beg, src);
        const int32_t len = __shfl(c.len, src, kWave);
        *a = shfl_f64(c.a, src);
        *ok = lane_on && ti < c.nterms && idx < len;
        const int64_t e = *ok ? (int64_t)beg + idx : 0;
        *cl = *ok ? P.B.col[e] : gcol;
        *v = *ok ? P.B.val[e] : 0.0;
    };
    // terms of an instruction by bit (sub < per <= 32)
    const bool multi = seen != nullptr && per <= 32;
    auto apply_rounds = [&](bool ok, uint32_t sl, double a, double v) {
        if (ok) atomicOr(&seen[sl], 1u << sub);
        wave_sync();
        const uint32_t rk = ok ? (uint32_t)__popc(seen[sl] & ((1u << sub) - 1u)) : 0u;
        for (uint32_t t = 0; __ballot(ok && rk >= t) != 0ull; ++t) {
            if (ok && rk == t) acc[sl] = fma(a, v, acc[sl]);
            wave_sync();
        }
        if (ok) seen[sl] = 0u;
        wave_sync();
    };
    for (int32_t i0 = 0; i0 < c.nterms; i0 += 2 * per) {
        bool ok0, ok1;
        double a0, a1, v0, v1;
        int32_t c0, c1;
        fetch(i0 + sub, &ok0, &a0, &c0, &v0);
        fetch(i0 + per + sub, &ok1, &a1, &c1, &v1);
        const uint32_t s0 = rank_col(bw, c0), s1 = rank_col(bw, c1);
        if (multi) {
            apply_rounds(ok0, s0, a0, v0);
            apply_rounds(ok1, s1, a1, v1);
            continue;
        }
        const int32_t n0 = min(per, c.nterms - i0);
        for (int32_t j = 0; j < n0; ++j) {
            if (ok0 && sub == j) acc[s0] = fma(a0, v0, acc[s0]);
            wave_sync();
        }
        const int32_t n1 = min(per, c.nterms - i0 - per);
        for (int32_t j = 0; j < n1; ++j) {
            if (ok1 && sub == j) acc[s1] = fma(a1, v1, acc[s1]);
            wave_sync();
        }
    }
}

// How the accumulation reads a chunk: term rows of 16 entries or more on
// average (coefficient terms always) go term by term, six at a time when they
// all fit one wavefront, otherwise three at a time (coefficient terms two) in
// steps of 128 entries; shorter product rows are packed over the lanes when
// the longest has at most kPackedMax entries, else read in flattened batches.
// The structure pass reads structure words instead (mark_words), except in
// the device-memory kernel.
__device__ __forceinline__ bool use_per_term(int src, const Chunk& c)
{
    return src == kSrcCoefs || c.total >= 16 * c.nterms;
}

// One pass over all terms of a source.  kAccum = false marks the structure,
// kAccum = true accumulates in term order.  If `have_first`, `first` is the
// chunk at the first term, already loaded (and staged if it takes the
// flattened path).
template <bool kAccum, bool kGlobal>
__device__ __forceinline__ void terms_pass(const StageArgs& P, int src, int64_t r, int32_t lo, uint32_t guard,
                                           uint8_t* bytes, uint2* bmp, double* acc, WaveStage& st,
                                           bool have_first, const Chunk& first, uint32_t* seen = nullptr,
                                           const int64_t* range = nullptr)
{
    int64_t tb, te;
    if (range != nullptr) {
        tb = range[0];
        te = range[1];
    } else {
        term_range(P, src, r, &tb, &te);
    }
    for (int64_t t0 = tb; t0 < te; t0 += kChunk) {
        const bool pre = have_first && t0 == tb;
        const Chunk c = pre ? first : load_chunk(P, src, r, t0, te);
        if (use_per_term(src, c)) {
            if (kAccum && c.maxlen <= kWave) {
                if (src == kSrcProducts)
                    short_group_pass<kSrcProducts>(P, r, t0, c, lo, guard, bmp, acc);
                else
                    short_group_pass<kSrcCoefs>(P, r, t0, c, lo, guard, bmp, acc);
            } else if (src == kSrcProducts) {
                per_term_pass<kSrcProducts, kAccum, kGlobal>(P, r, t0, c, lo, guard, bytes, bmp, acc);
            } else {
                per_term_pass<kSrcCoefs, kAccum, kGlobal>(P, r, t0, c, lo, guard, bytes, bmp, acc);
            }
        } else if (kAccum && src == kSrcProducts && c.maxlen <= kPackedMax) {
            packed_pass(P, c, lo, guard, bmp, acc, seen);
        } else {
            if (!pre) stage_chunk(c, st);
            for (int32_t q0 = 0; q0 < c.total; q0 += kWave * kU) {
                Batch<kU> b;
                gather<kAccum>(P, st, q0, c.total, b);
                if (kAccum)
                    accumulate_batch(c, q0, lo, guard, b, bmp, acc);
                else
                    mark_batch<kGlobal>(lo, guard, b, bytes, bmp);
            }
        }
    }
}

// ---- structure marks from structure words ------------------------------------
// A term row marks the output row's bitmap with one OR per structure word
// (the words of one row are distinct, so its ORs never meet on one address).
// The chunk's terms are spread over the lanes, `per` terms per instruction
// with `wd` lanes each, wd being the chunk's largest word count; term rows of
// more than 64 words go 64 words per step.  A word outside the window lands
// in the guard word.

// `first`, if given, is the chunk at the first term, already loaded.
template <int SRC>
__device__ __forceinline__ void mark_words(const StageArgs& P, int64_t r, int32_t lo, uint32_t words, uint2* bmp,
                                           const Chunk* first, const int64_t* range = nullptr)
{
    const int l = lane();
    const uint32_t lo_w = (uint32_t)lo >> 5;
    const uint2 ident = make_uint2((uint32_t)(r >> 5), 1u << (r & 31));
    int64_t tb, te;
    if (range != nullptr) {
        tb = range[0];
        te = range[1];
    } else {
        term_range(P, SRC, r, &tb, &te);
    }
    for (int64_t t0 = tb; t0 < te; t0 += kChunk) {
        const int64_t t = t0 + l;
        uint64_t wp = 0;  // address of the term row's first word; 0: the identity row
        int32_t nw = 0;
        if (first != nullptr && t0 == tb) {
            nw = first->nw;
            if (SRC == kSrcProducts) {
                wp = reinterpret_cast<uint64_t>(P.B.sw + first->beg);
            } else if (t < te && first->beg >= 0) {
                wp = reinterpret_cast<uint64_t>(P.T.sw[(int)t] + first->beg);
            }
        } else if (t < te) {
            if (SRC == kSrcProducts) {
                const int32_t k = P.A.col[t];
                wp = reinterpret_cast<uint64_t>(P.B.sw + P.B.beg[k]);
                nw = P.B.nw[k];
            } else {
                const int ti = (int)t;
                const int64_t* bp = P.T.beg[ti];
                if (bp == nullptr) {
                    nw = 1;
                } else {
                    wp = reinterpret_cast<uint64_t>(P.T.sw[ti] + bp[r]);
                    nw = P.T.nw[ti][r];
                }
            }
        }
        const int32_t nterms = (int32_t)min<int64_t>(kChunk, te - t0);
        const int32_t maxnw = sgpr(wave_reduce<OpMax>(nw));
        if (maxnw == 0) continue;
        const int32_t wd = min(maxnw, (int32_t)kWave);
        const int32_t per = kWave / wd;
        const int32_t sub = l / wd, idx = l - sub * wd;
        const bool lane_on = sub < per;
        // word e of the term held by lane ti of the chunk
        auto fetch = [&](int32_t ti, int32_t e, bool* ok) -> uint2 {
            const int src = min(ti, kChunk - 1);
            const uint64_t p = shfl_u64(wp, src);
            const int32_t n_t = __shfl(nw, src, kWave);
            *ok = lane_on && ti < nterms && e < n_t;
            if (!*ok) return make_uint2(0u, 0u);
            if (SRC == kSrcCoefs && p == 0) return ident;
            return reinterpret_cast<const uint2*>(p)[e];
        };
        auto mark = [&](bool ok, uint2 w) {
            if (ok) atomicOr(&bmp[min(w.x - lo_w, words)].x, w.y);
        };
        if (maxnw <= kWave) {
            for (int32_t i0 = 0; i0 < nterms; i0 += 2 * per) {
                bool ok0, ok1;
                const uint2 w0 = fetch(i0 + sub, idx, &ok0);
                const uint2 w1 = fetch(i0 + per + sub, idx, &ok1);
                mark(ok0, w0);
                mark(ok1, w1);
            }
        } else {
            for (int32_t i0 = 0; i0 < nterms; ++i0)
                for (int32_t e0 = 0; e0 < maxnw; e0 += kWave) {
                    bool ok;
                    const uint2 w = fetch(i0, e0 + l, &ok);
                    mark(ok, w);
                }
        }
    }
}

// Row r of the stage output left empty at offset o (one lane writes): every
// row gets its end, span, maximum and word count in every evaluation, so
// that later stages and the compaction never read a previous evaluation's
// values.
__device__ __forceinline__ void empty_row(const StageArgs& P, int64_t r, int64_t o)
{
    P.out.end[r] = o;
    P.out.info[r] = row_info(0, 1, 0, 0.0);
    P.out.nw[r] = 0;
}

// Computes output row r.  Returns false (with nothing written) if the row
// needs more workspace than max_words / cap provide.
//
// Phases: structure bitmap of the row's column window (the term rows'
// structure words ORed in; the device-memory kernel marks entries in a byte
// map); prefix counts so that rank(column) is the column's slot in a dense
// accumulator kept in column order; the main terms accumulated in order and
// parked (registers in the shared-memory kernel, `ebuf` in the device-memory
// kernel); the extra part (fused block terms or E) accumulated on its own;
// x = extra + main; the drop test and a sorted, coalesced write-out; the
// row's summary and structure words.  Rows whose main terms are at most 64
// short-row products keep them in registers from the structure pass to the
// accumulation.
// kGlobal: the structure in a device-memory byte map, bitmap and accumulator
// in device memory.  kDevPark: the main part parked in `ebuf` (device memory)
// rather than in kParked registers per lane.
template <bool kGlobal, bool kDevPark, int kParked>
__device__ __forceinline__ bool process_row(const StageArgs& P, int64_t r, int64_t o, uint8_t* bytes, uint2* bmp,
                                            double* acc, double* ebuf, WaveStage& st, int64_t max_words, int64_t cap,
                                            int64_t* kept_out, int64_t* ns_out)
{
    const int l = lane();
    *kept_out = 0;
    *ns_out = 0;
    // the row's analysis results and its range of main terms in one round trip
    const int main_src = (P.mode == kModeProduct) ? kSrcProducts : kSrcCoefs;
    const int32_t W = P.W[r];
    const int32_t lo = P.lo[r];
    const bool has_main = P.prod[r] > 0;
    int64_t range[2];
    term_range(P, main_src, r, &range[0], &range[1]);
    if (W <= 0) {
        if (l == 0) empty_row(P, r, o);
        return true;
    }
    const int64_t words = ((int64_t)W + 31) >> 5;
    if (words > max_words) return false;
    const uint32_t guard = (uint32_t)(words * 32);
    const bool has_extra = P.has_e || P.has_blk;

    // 1. structure of the row inside its window, guard word included
    if (kGlobal) {
        uint32_t* b4 = reinterpret_cast<uint32_t*>(bytes);
        for (int64_t i = l; i < (words + 1) * 8; i += kWave) b4[i] = 0u;
    } else {
        for (int64_t w = l; w <= words; w += kWave) bmp[w].x = 0u;
    }
    wave_sync();
    // rows whose main terms have no entries (known from the analysis) skip
    // them.  The first chunk of main terms is loaded before the block's marks
    // (its loads overlap theirs); the structure pass reuses it.
    const int64_t tb = range[0], te = range[1];
    Chunk c0{};
    if (has_main) c0 = load_chunk(P, main_src, r, tb, te);
    const Chunk none{};
    if (P.has_blk) {
        if (kGlobal)
            terms_pass<false, true>(P, kSrcCoefs, r, lo, guard, bytes, bmp, nullptr, st, false, none);
        else
            mark_words<kSrcCoefs>(P, r, lo, (uint32_t)words, bmp, nullptr);
    }
    if (P.has_e) {
        for (int64_t p = P.E.beg[r] + l; p < P.E.end[r]; p += kWave)
            mark_d<kGlobal>((uint32_t)(P.E.col[p] - lo), guard, bytes, bmp);
    }
    bool one_chunk = true, single = false;
    Batch<1> b1;
    if (has_main) {
        one_chunk = (te - tb <= kChunk);
        const bool flat0 = !use_per_term(main_src, c0);
        if (flat0) stage_chunk(c0, st);
        single = one_chunk && flat0 && (c0.total <= kWave);
        if (single) {
            if (c0.total > 0) {
                gather<true>(P, st, 0, c0.total, b1);
                mark_batch<kGlobal>(lo, guard, b1, bytes, bmp);
            }
        } else if (kGlobal) {
            terms_pass<false, true>(P, main_src, r, lo, guard, bytes, bmp, nullptr, st, true, c0, nullptr, range);
        } else if (main_src == kSrcProducts) {
            mark_words<kSrcProducts>(P, r, lo, (uint32_t)words, bmp, &c0, range);
        } else {
            mark_words<kSrcCoefs>(P, r, lo, (uint32_t)words, bmp, &c0);
        }
    }
    wave_sync();
    if (kGlobal) {  // pack the byte map into bits, guard word included
        const uint32_t* b4 = reinterpret_cast<const uint32_t*>(bytes);
        for (int64_t w = l; w <= words; w += kWave) {
            uint32_t bits = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t v = b4[w * 8 + j];
                bits |= ((v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u)) << (4 * j);
            }
            bmp[w].x = bits;
        }
        wave_sync();
    }

    // a column outside the row's window means the row information of an
    // operand was inconsistent: the stage reports an error, the row stays empty
    if (bmp[words].x != 0u) {
        flag_error(P, kErrColumnOutsideWindow);
        if (l == 0) empty_row(P, r, o);
        return true;
    }

    // 2. prefix counts of the bitmap words: rank(column) = slot; the guard
    //    word maps to the spare accumulator slot `cap`
    uint32_t running = 0;
    for (int64_t w0 = 0; w0 < words; w0 += kWave) {
        const int64_t w = w0 + l;
        const uint32_t cnt = (w < words) ? (uint32_t)__popc(bmp[w].x) : 0u;
        const uint32_t inc = wave_scan_u32(cnt);
        if (w < words) bmp[w].y = running + inc - cnt;
        running += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    }
    const int64_t ns = running;
    wave_sync();
    if (l == 0) bmp[words] = make_uint2(0u, (uint32_t)cap);
    *ns_out = ns;
    if (ns > cap) return false;
    // room of the row in the output: its stride, or up to the capacity
    if (ns > (P.row_stride > 0 ? P.row_stride : P.out.cap - o)) {
        flag_error(P, kErrCapacity);
        if (l == 0) empty_row(P, r, o);
        return true;
    }

    // the columns in slot order: lane w lists the set bits of word w
    auto list_cols = [&](int32_t* cols) {
        for (int64_t w = l; w < words; w += kWave) {
            const uint2 wd = bmp[w];
            uint32_t bits = wd.x;
            uint32_t base = wd.y;
            while (bits) {
                const int bt = __ffs((int)bits) - 1;
                cols[base++] = lo + (int32_t)(w * 32 + bt);
                bits &= bits - 1u;
            }
        }
    };

    // 3. zero the accumulator.  The device-memory kernel lists the columns
    //    now, in the row's output slot (compacted in place by the write-out);
    //    the shared-memory kernel lists them in shared memory after the
    //    accumulation (step 5).
    for (int64_t i = l; i < ns; i += kWave) acc[i] = 0.0;
    // the packed short-row path's slot words, zeroed, in the accumulator
    // beyond the row's slots when they fit below the spare slot (that path
    // leaves them zeroed)
    uint32_t* seen = nullptr;
    if (!kGlobal && ns + (ns + 1) / 2 <= cap) {
        seen = reinterpret_cast<uint32_t*>(acc + ns);
        for (int64_t i = l; i < ns; i += kWave) seen[i] = 0u;
    }
    if (kGlobal) list_cols(P.out.col + o);
    wave_sync();

    // 4. main terms in order, parked; then the extra part on its own
    if (!has_main) {
    } else if (single) {
        if (c0.total > 0) accumulate_batch(c0, 0, lo, guard, b1, bmp, acc);
    } else {
        terms_pass<true, kGlobal>(P, main_src, r, lo, guard, nullptr, bmp, acc, st, one_chunk, c0, seen, range);
    }
    wave_sync();
    double preg[kParked];
#pragma unroll
    for (int t = 0; t < kParked; ++t) preg[t] = 0.0;
    if (has_extra) {
        if (kDevPark) {
            for (int64_t i = l; i < ns; i += kWave) {
                ebuf[i] = acc[i];
                acc[i] = 0.0;
            }
        } else {
#pragma unroll
            for (int t = 0; t < kParked; ++t) {
                const int64_t i = (int64_t)t * kWave + l;
                if (i < ns) {
                    preg[t] = acc[i];
                    acc[i] = 0.0;
                }
            }
        }
        wave_sync();
        if (P.has_blk) terms_pass<true, kGlobal>(P, kSrcCoefs, r, lo, guard, nullptr, bmp, acc, st, false, none);
        if (P.has_e) {
            for (int64_t p = P.E.beg[r] + l; p < P.E.end[r]; p += kWave)
                acc[rank_of(bmp, (uint32_t)(P.E.col[p] - lo))] = P.E.val[p];
        }
        wave_sync();
    }
    // 5. x = extra + main, drop test, sorted write-out.  (Device-memory
    //    kernel: entry i moves to position kept-before-i <= i of the same
    //    slot; a batch reads its columns before any of its writes, which
    //    depend on the loaded values, and writes only below the next batch's
    //    reads.)
    int64_t kept = 0;
    double amx = 0.0;
    int32_t first = INT_MAX, last = -1;
    unsigned long long ndrop = 0;  // dropped-entry statistics
    double dmx = 0.0;
    const double tau = P.tau_row ? P.tau_row[r] : P.tau;
    auto emit = [&](int64_t i, double x, int32_t c) {
        bool keep = false;
        if (i < ns) {
            keep = (x != 0.0) && !(fabs(x) < tau);
            // the bitmap keeps the kept columns only, for the structure words
            if (!keep) atomicAnd(&bmp[(uint32_t)(c - lo) >> 5].x, ~(1u << (c & 31)));
        }
        if (P.dsum != nullptr) {
            const bool d = i < ns && x != 0.0 && (!keep || fabs(x) <= P.dthr);
            if (d) atomicAdd(&P.dsum[c], (unsigned long long)ceil(fabs(x) * P.dscale));
            if (P.dcount) {
                if (d) dmx = fmax(dmx, fabs(x));
                ndrop += __popcll(__ballot(d));
            }
        }
        const unsigned long long m = __ballot(keep);
        if (keep) {
            const int64_t pos = o + kept + (int64_t)lanes_below(m);
            P.out.col[pos] = c;
            P.out.val[pos] = x;
            amx = fmax(amx, fabs(x));
            first = min(first, c);
            last = max(last, c);
        }
        kept += __popcll(m);
    };
    if (kGlobal) {
        const int32_t* cols = P.out.col + o;
        for (int64_t i0 = 0; i0 < ns; i0 += kWave) {
            const int64_t i = i0 + l;
            double x = 0.0;
            int32_t c = 0;
            if (i < ns) {
                x = has_extra ? acc[i] + ebuf[i] : acc[i];
                c = cols[i];
            }
            emit(i, x, c);
        }
    } else if (kDevPark) {
        // the values move to `ebuf` (x = extra + parked main part), which
        // frees the accumulator for the column list
        for (int64_t i = l; i < ns; i += kWave) ebuf[i] = has_extra ? acc[i] + ebuf[i] : acc[i];
        wave_sync();
        int32_t* cols = reinterpret_cast<int32_t*>(acc);
        list_cols(cols);
        wave_sync();
        for (int64_t i0 = 0; i0 < ns; i0 += kWave) {
            const int64_t i = i0 + l;
            emit(i, i < ns ? ebuf[i] : 0.0, i < ns ? cols[i] : 0);
        }
    } else {
        // the values move to registers (x = extra + parked main part), which
        // frees the accumulator for the column list
#pragma unroll
        for (int t = 0; t < kParked; ++t) {
            const int64_t i = (int64_t)t * kWave + l;
            if (i < ns) preg[t] = has_extra ? acc[i] + preg[t] : acc[i];
        }
        wave_sync();
        int32_t* cols = reinterpret_cast<int32_t*>(acc);
        list_cols(cols);
        wave_sync();
#pragma unroll
        for (int t = 0; t < kParked; ++t) {
            const int64_t i = (int64_t)t * kWave + l;
            if ((int64_t)t * kWave < ns) emit(i, preg[t], i < ns ? cols[i] : 0);
        }
    }
    amx = wave_reduce<OpMax>(amx);
    first = wave_reduce<OpMin>(first);
    last = wave_reduce<OpMax>(last);
    if (P.dsum != nullptr && P.dcount) {
        dmx = wave_reduce<OpMax>(dmx);
        if (l == 0 && ndrop != 0) {
            atomicAdd(&P.ctr->n_dropped, ndrop);
            atomicMax(&P.ctr->dropped_max, (unsigned long long)__double_as_longlong(dmx));
        }
    }
    // 6. structure words of the row: the nonzero bitmap words, in order
    wave_sync();
    int32_t nwd = 0;
    for (int64_t w0 = 0; w0 < words; w0 += kWave) {
        const int64_t w = w0 + l;
        const uint32_t bits = (w < words) ? bmp[w].x : 0u;
        const unsigned long long m = __ballot(bits != 0u);
        if (bits != 0u) P.out.sw[o + nwd + (int64_t)lanes_below(m)] = make_uint2(((uint32_t)lo >> 5) + (uint32_t)w, bits);
        nwd += __popcll(m);
    }
    if (l == 0) {
        P.out.end[r] = o + kept;
        P.out.info[r] = row_info(kept, first, last, amx);
        P.out.nw[r] = nwd;
    }
    wave_sync();
    *kept_out = kept;
    return true;
}

// Appends row r (output offset o) to a fallback list, called by one lane.
// If the kernel that serves the list does not run for this stage (`planned`
// is 0), the row is left empty and flagged instead: the result query then
// repeats the evaluation with sizing, which plans that kernel.
__device__ __forceinline__ void defer_row(const StageArgs& P, int64_t r, int64_t o, unsigned long long* count,
                                          int64_t* list, int32_t planned)
{
    if (planned) {
        const unsigned long long i = atomicAdd(count, 1ull);
        list[i] = r;
    } else {
        empty_row(P, r, o);
        flag_error(P, kErrNeedsGlobal);
    }
}

// One row per wavefront, four rows per block, blocks in XCD-aware order, in
// the shared-memory tier kWords / kCap.  Rows that do not fit go to the next
// kernel's list: from the narrow tier the wide tier's (with
// FPS_FLAG_FORCE_GLOBAL every row the device-memory kernel's), from the wide
// tier the device-memory kernel's.
template <int kWords, int kCap, bool kNarrow>
__device__ __forceinline__ void numeric_rows(const StageArgs& P)
{
    using Ws = LdsWave<kWords, kCap>;
    __shared__ Ws lds[kWavesPerBlock];
    __shared__ unsigned long long kept_sh[kWavesPerBlock], ns_sh[kWavesPerBlock], words_sh[kWavesPerBlock];
    const int wv = sgpr((int32_t)(threadIdx.x / kWave));  // wave-uniform: row-level values live in scalar registers
    Ws& me = lds[wv];
    const int l = lane();
    const int64_t blk = xcd_logical_block();
    const int64_t r = blk * kWavesPerBlock + wv;
    int64_t kept = 0, ns = 0, words = 0;
    if (r < P.n) {
        words = ((int64_t)max(P.W[r], 0) + 31) >> 5;
        // the row's output offset: a fixed stride, or its block prefix plus
        // its offset in the block
        const int64_t o = P.row_stride > 0 ? r * P.row_stride : P.blk_pre[r >> P.scan_shift] + P.out.off[r];
        if (l == 0) P.out.off[r] = o;
        bool done = false;
        if (!P.force_global)
            done = process_row<false, false, Ws::kPark>(P, r, o, nullptr, me.bmp, me.acc, nullptr, me.st, kWords, kCap,
                                                 &kept, &ns);
        if (!done && l == 0) {
            const bool direct = !kNarrow || P.force_global != 0;
            defer_row(P, r, o, direct ? &P.ctr->fb2_count : &P.ctr->fb_count, direct ? P.fb2_list : P.fb_list,
                      direct ? P.global_planned : P.wide_planned);
        }
    }
    if (l == 0) {
        kept_sh[wv] = (unsigned long long)kept;
        ns_sh[wv] = (unsigned long long)ns;
        words_sh[wv] = (unsigned long long)words;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0, mx = 0, mw = 0, big = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) {
            t += kept_sh[i];
            mx = max(mx, ns_sh[i]);
            mw = max(mw, words_sh[i]);
            big += (ns_sh[i] > (unsigned long long)kSmallCap || words_sh[i] > (unsigned long long)kSmallWords) ? 1 : 0;
        }
        P.part[kPartKept * P.part_stride + blk] = t;
        P.part[kPartMaxNs * P.part_stride + blk] = mx;
        P.part[kPartMaxWords * P.part_stride + blk] = mw;
        P.part[kPartBig * P.part_stride + blk] = big;
    }
}

// Narrow tier, every row of a stage: the workspace (19.5 KB per block) and
// the register budget (64 per lane) are sized for eight wavefronts per SIMD.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) k_numeric_lds(StageArgs P)
{
    numeric_rows<kNarrowWords, kNarrowCap, true>(P);
}

// Wide tier, every row of a stage whose rows mostly exceed the narrow tier
// (26.5 KB per block, six wavefronts per SIMD).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) k_numeric_wide_rows(StageArgs P)
{
    numeric_rows<kWideWords, kWideCap, false>(P);
}

// ---- small rows: four rows per wavefront ---------------------------------------
// Rows with a narrow window and few structural entries (powers of a stencil
// operator, the start of the Horner recurrence) leave most lanes of a
// wavefront idle, and such a stage is bound by the latency of each row's
// chain of dependent loads.  Here each row is owned by one 16-lane DPP row
// of a wavefront, so four rows share one chain.  The steps and the order of
// every fma are those of process_row: structure bitmap of the window, ranks,
// the main terms in term order, the block terms on their own, x = extra +
// main, the drop test and a sorted write-out.  A stage runs in this tier
// only when its sizing run found every row within kSmallWords / kSmallCap
// (24.3 KB per block, six wavefronts per SIMD: a smaller workspace for
// eight measured no faster, the tier being bound by instruction issue; a
// larger one, 192 entries in 5120 columns at three wavefronts per SIMD, took
// rows of 85 terms of about 10 entries in 298 us against the 64-lane packed
// path's 172); a row beyond them later goes to the wide tier's list.
constexpr int kSmallLanes = 16;
constexpr int kSmallRowsPerWave = kWave / kSmallLanes;
constexpr int kSmallRowsPerBlock = kBlock / kSmallLanes;
// The tier pays only when a stage has more rows than the 64-lane kernel holds
// at once (eight wavefronts per SIMD on 256 CUs): with fewer, both finish in
// one round and a row's own chain, shorter on 64 lanes, sets the time.
constexpr int64_t kSmallMinRows = 256 * 4 * 8;
// ... and takes a stage most of whose rows fit it when at most one row in
// kSmallBigShare does not (those go to the wide tier's list)
constexpr int64_t kSmallBigShare = 16;
constexpr int kSmallU = 2;  // terms whose first 32 entries are loaded together

template <int kWords, int kCap>
struct SmallRow {
    static_assert(kCap % kSmallLanes == 0, "the values per lane cover the accumulator exactly");
    static constexpr int kPark = kCap / kSmallLanes;  // values per lane after the accumulation
    uint2 bmp[kWords + 1];  // as in LdsWave: structure bits, earlier set bits; then the guard word
    double acc[kCap + 1];   // then the spare slot
};

__device__ __forceinline__ int small_lane() { return lane() & (kSmallLanes - 1); }

// Inclusive prefix sum over the 16 lanes of a DPP row.
__device__ __forceinline__ uint32_t row_scan_u32(uint32_t x)
{
    x += dpp32<kDppRowShr1>(x);
    x += dpp32<kDppRowShr1 + 1>(x);
    x += dpp32<kDppRowShr1 + 3>(x);
    x += dpp32<kDppRowShr1 + 7>(x);
    return x;
}

// This lane's DPP row's 16 bits of a wavefront ballot.
__device__ __forceinline__ uint32_t row_bits(unsigned long long m)
{
    return (uint32_t)(m >> (lane() & (kWave - kSmallLanes))) & 0xFFFFu;
}

// Value of lane j of this lane's DPP row.
__device__ __forceinline__ int32_t row_bcast(int32_t x, int j) { return __shfl(x, j, kSmallLanes); }
__device__ __forceinline__ int64_t row_bcast64(int64_t x, int j)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)(uint64_t)x, j, kSmallLanes);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)((uint64_t)x >> 32), j, kSmallLanes);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double row_bcastd(double x, int j)
{
    return __longlong_as_double((long long)row_bcast64((int64_t)__double_as_longlong(x), j));
}

// One term of a chunk of up to 16, held by one lane of the row.
struct SmallTerm {
    int64_t beg;  // first entry of the term row; -1: the identity row (coefficient term of P_0)
    int32_t len;  // entries of the term row (0: no term)
    int32_t nw;   // structure words of the term row
    double a;     // weight
};

template <int SRC>
__device__ __forceinline__ SmallTerm small_term(const StageArgs& P, int64_t r, int64_t t, bool on)
{
    SmallTerm h{0, 0, 0, 0.0};
    if (!on) return h;
    if constexpr (SRC == kSrcProducts) {
        const int32_t k = P.A.col[t];
        h.a = P.A.val[t];
        h.beg = P.B.beg[k];
        h.len = (int32_t)(P.B.end[k] - h.beg);
        h.nw = P.B.nw[k];
    } else {
        const int ti = (int)t;
        h.a = P.T.coef[ti];
        const int64_t* bp = P.T.beg[ti];
        if (bp == nullptr) {
            h.beg = -1;
            h.len = 1;
            h.nw = 1;
        } else {
            h.beg = bp[r];
            h.len = (int32_t)(P.T.end[ti][r] - h.beg);
            h.nw = P.T.nw[ti][r];
        }
    }
    return h;
}

// Term j of the chunk starting at term t0: its row's columns, values and
// structure words (coefficient terms index the same term on every row, so
// their arrays are uniform).
template <int SRC>
__device__ __forceinline__ const uint2* small_sw(const StageArgs& P, int64_t t0, int j, int64_t beg)
{
    if constexpr (SRC == kSrcProducts)
        return P.B.sw + beg;
    else
        return P.T.sw[min((int)t0 + j, kMaxTerms - 1)] + beg;
}
template <int SRC>
__device__ __forceinline__ const int32_t* small_col(const StageArgs& P, int64_t t0, int j, int64_t beg)
{
    if constexpr (SRC == kSrcProducts)
        return P.B.col + beg;
    else
        return P.T.col[min((int)t0 + j, kMaxTerms - 1)] + beg;
}
template <int SRC>
__device__ __forceinline__ const double* small_val(const StageArgs& P, int64_t t0, int j, int64_t beg)
{
    if constexpr (SRC == kSrcProducts)
        return P.B.val + beg;
    else
        return P.T.val[min((int)t0 + j, kMaxTerms - 1)] + beg;
}

// Structure marks of terms [0, nt) of a chunk: kSmallU terms at a time, the
// first two words of each per lane loaded together, then the rest.
template <int SRC>
__device__ __forceinline__ void small_marks(const StageArgs& P, int64_t r, int64_t t0, int32_t nt, const SmallTerm& h,
                                            uint32_t lo_w, uint32_t words, uint2* bmp)
{
    const int gl = small_lane();
    const uint2 ident = make_uint2((uint32_t)(r >> 5), 1u << (r & 31));
    for (int32_t j0 = 0; j0 < nt; j0 += kSmallU) {
        uint2 w[kSmallU][2];
        int32_t nw[kSmallU];
        int64_t beg[kSmallU];
#pragma unroll
        for (int g = 0; g < kSmallU; ++g) {
            const int j = min(j0 + g, kSmallLanes - 1);
            beg[g] = row_bcast64(h.beg, j);
            nw[g] = (j0 + g < nt) ? row_bcast(h.nw, j) : 0;
            const bool id = SRC == kSrcCoefs && beg[g] < 0;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int e = gl + i * kSmallLanes;
                w[g][i] = make_uint2(0u, 0u);
                if (e < nw[g]) w[g][i] = id ? ident : small_sw<SRC>(P, t0, j, beg[g])[e];
            }
        }
#pragma unroll
        for (int g = 0; g < kSmallU; ++g)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                if (gl + i * kSmallLanes < nw[g]) atomicOr(&bmp[min(w[g][i].x - lo_w, words)].x, w[g][i].y);
#pragma unroll
        for (int g = 0; g < kSmallU; ++g) {
            for (int32_t e0 = 2 * kSmallLanes; e0 < nw[g]; e0 += kSmallLanes) {
                const int32_t e = e0 + gl;
                if (e < nw[g]) {
                    const uint2 x = small_sw<SRC>(P, t0, min(j0 + g, kSmallLanes - 1), beg[g])[e];
                    atomicOr(&bmp[min(x.x - lo_w, words)].x, x.y);
                }
            }
        }
    }
}

// acc[rank] = fma(a, v, acc[rank]) for terms [0, nt) of a chunk, strictly
// term by term (the entries of one term have distinct columns); lanes
// without an entry use the spare slot.
template <int SRC>
__device__ __forceinline__ void small_accumulate(const StageArgs& P, int64_t r, int64_t t0, int32_t nt,
                                                 const SmallTerm& h, const uint2* bw, int32_t gcol, double* acc)
{
    const int gl = small_lane();
    for (int32_t j0 = 0; j0 < nt; j0 += kSmallU) {
        int32_t cc[kSmallU][2];
        double vv[kSmallU][2];
        double aa[kSmallU];
        int32_t ln[kSmallU];
#pragma unroll
        for (int g = 0; g < kSmallU; ++g) {
            const int j = min(j0 + g, kSmallLanes - 1);
            const int64_t beg = row_bcast64(h.beg, j);
            ln[g] = (j0 + g < nt) ? row_bcast(h.len, j) : 0;
            aa[g] = row_bcastd(h.a, j);
            const bool id = SRC == kSrcCoefs && beg < 0;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int e = gl + i * kSmallLanes;
                cc[g][i] = gcol;
                vv[g][i] = 0.0;
                if (e < ln[g]) {
                    cc[g][i] = id ? (int32_t)r : small_col<SRC>(P, t0, j, beg)[e];
                    vv[g][i] = id ? 1.0 : small_val<SRC>(P, t0, j, beg)[e];
                }
            }
        }
        uint32_t sl[kSmallU][2];
#pragma unroll
        for (int g = 0; g < kSmallU; ++g)
#pragma unroll
            for (int i = 0; i < 2; ++i) sl[g][i] = rank_col(bw, cc[g][i]);
#pragma unroll
        for (int g = 0; g < kSmallU; ++g) {
            if (ln[g] == 0) continue;
            acc[sl[g][0]] = fma(aa[g], vv[g][0], acc[sl[g][0]]);
            if (ln[g] > kSmallLanes) acc[sl[g][1]] = fma(aa[g], vv[g][1], acc[sl[g][1]]);
            if (ln[g] > 2 * kSmallLanes) {
                const int j = min(j0 + g, kSmallLanes - 1);
                const int64_t beg = row_bcast64(h.beg, j);
                const int32_t* cp = small_col<SRC>(P, t0, j, beg);
                const double* vp = small_val<SRC>(P, t0, j, beg);
                for (int32_t e0 = 2 * kSmallLanes; e0 < ln[g]; e0 += kSmallLanes) {
                    const int32_t e = e0 + gl;
                    int32_t c = gcol;
                    double v = 0.0;
                    if (e < ln[g]) {
                        c = cp[e];
                        v = vp[e];
                    }
                    const uint32_t sv = rank_col(bw, c);
                    acc[sv] = fma(aa[g], v, acc[sv]);
                }
            }
            wave_sync();
        }
    }
}

// All terms of a source, chunk by chunk (16 terms per chunk, one per lane).
// `first` is the first chunk, already loaded.
template <int SRC, bool kAccum>
__device__ __forceinline__ void small_pass(const StageArgs& P, int64_t r, const SmallTerm& first, uint32_t lo_w,
                                           uint32_t words, uint2* bmp, const uint2* bw, int32_t gcol, double* acc)
{
    const int gl = small_lane();
    int64_t tb, te;
    term_range(P, SRC, r, &tb, &te);
    for (int64_t t0 = tb; t0 < te; t0 += kSmallLanes) {
        const int32_t nt = (int32_t)min<int64_t>(kSmallLanes, te - t0);
        const SmallTerm h = (t0 == tb) ? first : small_term<SRC>(P, r, t0 + gl, gl < nt);
        if (kAccum)
            small_accumulate<SRC>(P, r, t0, nt, h, bw, gcol, acc);
        else
            small_marks<SRC>(P, r, t0, nt, h, lo_w, words, bmp);
    }
}

// A row's analysis on its 16-lane DPP row, as the analysis kernels compute
// it: the same lanes take the same terms in the same order and reduce over
// the same DPP row, so the window, the product count and the empty-row test
// (a floating-point bound) come out identical.  Writes W, lo and the product
// count for the fallback tiers; also returns the row's multiply-adds and
// whether the empty-row test skipped them.
struct SmallAnalysis {
    int32_t W, lo;
    int64_t prod;
    int64_t work;  // multiply-adds of the row (done, or skipped if `skip`)
    bool skip;
};

// The first chunk of terms (16, one per lane) of the main part and of the
// block are read in the same pass: *mt and *bt are what small_term gives.
template <bool kBlk>
__device__ __forceinline__ SmallAnalysis small_analyze(const StageArgs& P, int64_t r, SmallTerm* mt, SmallTerm* bt)
{
    const int gl = small_lane();
    static_assert(kSmallLanes == kAnalyzeLanes, "one DPP row per row, as in the analysis");
    SmallAnalysis a{0, 0, 0, 0, false};
    int32_t lo = INT_MAX, hi = -1;
    int64_t prod = 0;
    *mt = SmallTerm{0, 0, 0, 0.0};
    *bt = SmallTerm{0, 0, 0, 0.0};
    // coefficient term t of row r: summary into the window and counts, and
    // (first chunk) the term itself
    auto coef_term = [&](int t, bool first, int64_t* len_sum, double* amax_sum, SmallTerm* h) {
        const int64_t* bp = P.T.beg[t];
        if (bp == nullptr) {
            lo = min(lo, (int32_t)r);
            hi = max(hi, (int32_t)r);
            *len_sum += 1;
            if (amax_sum) *amax_sum += fabs(P.T.coef[t]);
            if (first) *h = SmallTerm{-1, 1, 1, P.T.coef[t]};
        } else {
            const RowInfo q = load_info(P.T.info[t] + r);
            if (first) {
                const int64_t b = bp[r];
                *h = SmallTerm{b, (int32_t)(P.T.end[t][r] - b), P.T.nw[t][r], P.T.coef[t]};
            }
            if (q.len > 0) {
                lo = min(lo, q.first);
                hi = max(hi, q.last);
                *len_sum += q.len;
                if (amax_sum) *amax_sum += fabs(P.T.coef[t]) * (double)q.amax;
            }
        }
    };
    if (P.mode == kModeProduct) {
        double bnd = 0.0;
        const int64_t pb = P.A.beg[r], pe = P.A.end[r];
        int64_t p = pb + gl;
        if (p < pe) {  // the first chunk: the term as well
            const int32_t k = P.A.col[p];
            const double av = P.A.val[p];
            const RowInfo q = load_info(P.B.info + k);
            const int64_t b = P.B.beg[k];
            *mt = SmallTerm{b, (int32_t)(P.B.end[k] - b), P.B.nw[k], av};
            lo = min(lo, q.len > 0 ? q.first : INT_MAX);
            hi = max(hi, q.len > 0 ? q.last : -1);
            prod += q.len;
            bnd += fabs(av) * (double)q.amax;
        }
#pragma unroll 4
        for (p += kSmallLanes; p < pe; p += kSmallLanes) {
            const int32_t k = P.A.col[p];
            const RowInfo q = load_info(P.B.info + k);
            lo = min(lo, q.len > 0 ? q.first : INT_MAX);
            hi = max(hi, q.len > 0 ? q.last : -1);
            prod += q.len;
            bnd += fabs(P.A.val[p]) * (double)q.amax;
        }
        int64_t elen = 0;
        double emax = 0.0;
        if (kBlk) {
            for (int t = gl; t < P.T.n; t += kSmallLanes) coef_term(t, t == gl, &elen, &emax, bt);
        }
        lo = row_reduce<OpMin>(lo);
        hi = row_reduce<OpMax>(hi);
        prod = row_reduce<OpSum>(prod);
        bnd = row_reduce<OpSum>(bnd);
        elen = row_reduce<OpSum>(elen);
        emax = row_reduce<OpSum>(emax);
        const bool empty = (prod == 0 && elen == 0);
        const double skip_tau = P.tau_row ? P.tau_row[r] * P.skip_rel : P.skip_tau;
        const bool skip = !empty && skip_tau > 0.0 && (emax + bnd) < skip_tau;
        if (!empty && !skip) {
            lo &= ~31;
            a.W = hi - lo + 1;
        }
        a.work = prod + (kBlk ? elen : 0);
        a.skip = skip;
    } else {
        for (int t = gl; t < P.T.n; t += kSmallLanes) coef_term(t, t == gl, &prod, nullptr, mt);
        lo = row_reduce<OpMin>(lo);
        hi = row_reduce<OpMax>(hi);
        prod = row_reduce<OpSum>(prod);
        if (prod > 0) {
            lo &= ~31;
            a.W = hi - lo + 1;
        }
        a.work = prod;
    }
    a.lo = lo;
    a.prod = prod;
    if (gl == 0) {
        P.W[r] = a.W;
        P.lo[r] = lo;
        P.prod[r] = prod;
    }
    return a;
}

// Row r (output offset o) on this lane's DPP row.  Returns false, with
// nothing written, if the row does not fit the workspace.
// kBlk: the stage fuses a coefficient block (P.has_blk).
// With P.fuse_analysis the row's analysis comes first; lane 0 stores the
// row's multiply-adds in *work (their complement if the empty-row test
// skipped them).
template <int kWords, int kCap, bool kBlk>
__device__ __forceinline__ bool small_row(const StageArgs& P, int64_t r, int64_t o, SmallRow<kWords, kCap>& ws, int64_t* kept_out,
                                          int64_t* ns_out, long long* work)
{
    const int gl = small_lane();
    *kept_out = 0;
    *ns_out = 0;
    int32_t W, lo;
    int64_t prod;
    SmallTerm m0{0, 0, 0, 0.0}, b0{0, 0, 0, 0.0};  // first chunks of the main and block terms
    if (P.fuse_analysis) {
        const SmallAnalysis an = small_analyze<kBlk>(P, r, &m0, &b0);
        W = an.W;
        lo = an.lo;
        prod = an.prod;
        if (gl == 0) *work = an.skip ? ~(long long)an.work : (long long)an.work;
    } else {
        W = P.W[r];
        lo = P.lo[r];
        prod = P.prod[r];
    }
    if (W <= 0) {
        if (gl == 0) empty_row(P, r, o);
        return true;
    }
    const int32_t words = (W + 31) >> 5;
    if (words > kWords) return false;
    uint2* bmp = ws.bmp;
    double* acc = ws.acc;
    const uint32_t lo_w = (uint32_t)lo >> 5;
    const uint2* bw = bmp - (lo >> 5);
    const int32_t gcol = lo + words * 32;

    // 1. structure of the row inside its window, guard word included
    for (int32_t w = gl; w <= words; w += kSmallLanes) bmp[w].x = 0u;
    wave_sync();
    const bool product = P.mode == kModeProduct;
    const bool has_main = prod > 0;
    int64_t tb, te;
    term_range(P, product ? kSrcProducts : kSrcCoefs, r, &tb, &te);
    const int32_t nt0 = (int32_t)min<int64_t>(kSmallLanes, te - tb);
    if (has_main && !P.fuse_analysis)
        m0 = product ? small_term<kSrcProducts>(P, r, tb + gl, gl < nt0) : small_term<kSrcCoefs>(P, r, tb + gl, gl < nt0);
    if (kBlk) {
        if (!P.fuse_analysis) b0 = small_term<kSrcCoefs>(P, r, gl, gl < min(P.T.n, kSmallLanes));
        small_pass<kSrcCoefs, false>(P, r, b0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
    }
    if (has_main) {
        if (product)
            small_pass<kSrcProducts, false>(P, r, m0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
        else
            small_pass<kSrcCoefs, false>(P, r, m0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
    }
    wave_sync();
    if (bmp[words].x != 0u) {  // a column outside the window: inconsistent row information
        flag_error(P, kErrColumnOutsideWindow);
        if (gl == 0) empty_row(P, r, o);
        return true;
    }

    // 2. ranks: prefix counts of the bitmap words; the guard word maps to the spare slot
    uint32_t running = 0;
    for (int32_t w0 = 0; w0 < words; w0 += kSmallLanes) {
        const int32_t w = w0 + gl;
        const uint32_t cnt = (w < words) ? (uint32_t)__popc(bmp[w].x) : 0u;
        const uint32_t inc = row_scan_u32(cnt);
        if (w < words) bmp[w].y = running + inc - cnt;
        running += row_reduce<OpMax>(inc);
    }
    const int32_t ns = (int32_t)running;
    wave_sync();
    if (gl == 0) bmp[words] = make_uint2(0u, (uint32_t)kCap);
    *ns_out = ns;
    if (ns > kCap) return false;
    if (ns > (P.row_stride > 0 ? P.row_stride : P.out.cap - o)) {
        flag_error(P, kErrCapacity);
        if (gl == 0) empty_row(P, r, o);
        return true;
    }

    // 3. main terms in order, then the block terms on their own
    for (int32_t i = gl; i < ns; i += kSmallLanes) acc[i] = 0.0;
    wave_sync();
    if (has_main) {
        if (product)
            small_pass<kSrcProducts, true>(P, r, m0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
        else
            small_pass<kSrcCoefs, true>(P, r, m0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
    }
    wave_sync();
    double x[SmallRow<kWords, kCap>::kPark];
#pragma unroll
    for (int t = 0; t < SmallRow<kWords, kCap>::kPark; ++t) {
        const int32_t i = t * kSmallLanes + gl;
        x[t] = (i < ns) ? acc[i] : 0.0;
    }
    if (kBlk) {
        wave_sync();
        for (int32_t i = gl; i < ns; i += kSmallLanes) acc[i] = 0.0;
        wave_sync();
        small_pass<kSrcCoefs, true>(P, r, b0, lo_w, (uint32_t)words, bmp, bw, gcol, acc);
        wave_sync();
#pragma unroll
        for (int t = 0; t < SmallRow<kWords, kCap>::kPark; ++t) {
            const int32_t i = t * kSmallLanes + gl;
            if (i < ns) x[t] = acc[i] + x[t];  // x = extra + main
        }
    }
    wave_sync();

    // 4. the columns in slot order, in the accumulator's place
    int32_t* cols = reinterpret_cast<int32_t*>(acc);
    for (int32_t w = gl; w < words; w += kSmallLanes) {
        const uint2 wd = bmp[w];
        uint32_t bits = wd.x, base = wd.y;
        while (bits) {
            const int bt = __ffs((int)bits) - 1;
            cols[base++] = lo + w * 32 + bt;
            bits &= bits - 1u;
        }
    }
    wave_sync();

    // 5. drop test and sorted write-out
    const uint32_t below = (1u << gl) - 1u;
    const double tau = P.tau_row ? P.tau_row[r] : P.tau;
    int64_t kept = 0;
    double amx = 0.0, dmx = 0.0;
    int32_t first = INT_MAX, last = -1;
    unsigned long long ndrop = 0;
#pragma unroll
    for (int t = 0; t < SmallRow<kWords, kCap>::kPark; ++t) {
        if (t * kSmallLanes >= ns) break;
        const int32_t i = t * kSmallLanes + gl;
        const bool in = i < ns;
        const int32_t c = in ? cols[i] : 0;
        const double v = x[t];
        const bool keep = in && (v != 0.0) && !(fabs(v) < tau);
        // the bitmap keeps the kept columns only, for the structure words
        if (in && !keep) atomicAnd(&bmp[(uint32_t)(c - lo) >> 5].x, ~(1u << (c & 31)));
        if (P.dsum != nullptr) {
            const bool d = in && v != 0.0 && (!keep || fabs(v) <= P.dthr);
            if (d) atomicAdd(&P.dsum[c], (unsigned long long)ceil(fabs(v) * P.dscale));
            if (P.dcount) {
                if (d) dmx = fmax(dmx, fabs(v));
                ndrop += (unsigned long long)__popc(row_bits(__ballot(d)));
            }
        }
        const uint32_t m = row_bits(__ballot(keep));
        if (keep) {
            const int64_t pos = o + kept + (int64_t)__popc(m & below);
            P.out.col[pos] = c;
            P.out.val[pos] = v;
            amx = fmax(amx, fabs(v));
            first = min(first, c);
            last = max(last, c);
        }
        kept += __popc(m);
    }
    amx = row_reduce<OpMax>(amx);
    first = row_reduce<OpMin>(first);
    last = row_reduce<OpMax>(last);
    if (P.dsum != nullptr && P.dcount) {
        dmx = row_reduce<OpMax>(dmx);
        if (gl == 0 && ndrop != 0) {
            atomicAdd(&P.ctr->n_dropped, ndrop);
            atomicMax(&P.ctr->dropped_max, (unsigned long long)__double_as_longlong(dmx));
        }
    }

    // 6. structure words of the row: the nonzero bitmap words, in order
    wave_sync();
    int32_t nwd = 0;
    for (int32_t w0 = 0; w0 < words; w0 += kSmallLanes) {
        const int32_t w = w0 + gl;
        const uint32_t bits = (w < words) ? bmp[w].x : 0u;
        const uint32_t m = row_bits(__ballot(bits != 0u));
        if (bits != 0u) P.out.sw[o + nwd + (int64_t)__popc(m & below)] = make_uint2(lo_w + (uint32_t)w, bits);
        nwd += __popc(m);
    }
    if (gl == 0) {
        P.out.end[r] = o + kept;
        P.out.info[r] = row_info(kept, first, last, amx);
        P.out.nw[r] = nwd;
    }
    wave_sync();
    *kept_out = kept;
    return true;
}

// Four rows per wavefront, sixteen per block, blocks in XCD-aware order.  The
// per-block partial sums are written per wavefront, at the index of the
// four-row block of the other shared-memory tiers (same layout).
template <int kWords, int kCap, int kWaves, bool kBlk>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves, 8))) k_numeric_small(StageArgs P)
{
    __shared__ SmallRow<kWords, kCap> rows[kSmallRowsPerBlock];
    __shared__ long long work_sh[kSmallRowsPerBlock];
    const int wv = sgpr((int32_t)(threadIdx.x / kWave));
    const int l = lane();
    const int grp = l / kSmallLanes;
    const int64_t blk = xcd_logical_block();
    const int64_t r0 = (blk * kWavesPerBlock + wv) * kSmallRowsPerWave;  // first row of the wavefront
    const int64_t r = r0 + grp;
    int64_t kept = 0, ns = 0;
    long long* work = &work_sh[wv * kSmallRowsPerWave + grp];
    if (small_lane() == 0) *work = 0;
    if (r < P.n) {
        const int64_t o = P.row_stride > 0 ? r * P.row_stride : P.blk_pre[r >> P.scan_shift] + P.out.off[r];
        if (small_lane() == 0) P.out.off[r] = o;
        const bool done =
            small_row<kWords, kCap, kBlk>(P, r, o, rows[wv * kSmallRowsPerWave + grp], &kept, &ns, work);
        if (!done && small_lane() == 0) defer_row(P, r, o, &P.ctr->fb_count, P.fb_list, P.wide_planned);
    }
    wave_sync();
    if (r0 < P.n) {
        unsigned long long t = 0, mx = 0, pd = 0, ps = 0, rs = 0;
#pragma unroll
        for (int k = 0; k < kSmallRowsPerWave; ++k) {
            t += (unsigned long long)readlane64(kept, k * kSmallLanes);
            mx = max(mx, (unsigned long long)readlane64(ns, k * kSmallLanes));
            const long long w = work_sh[wv * kSmallRowsPerWave + k];
            pd += w >= 0 ? (unsigned long long)w : 0ull;
            ps += w < 0 ? (unsigned long long)~w : 0ull;
            rs += w < 0 ? 1ull : 0ull;
        }
        if (l == 0) {
            const int64_t pi = r0 / kSmallRowsPerWave;
            P.part[kPartKept * P.part_stride + pi] = t;
            P.part[kPartMaxNs * P.part_stride + pi] = mx;
            if (P.fuse_analysis) {
                P.part[kPartProducts * P.part_stride + pi] = pd;
                P.part[kPartProductsSkipped * P.part_stride + pi] = ps;
                P.part[kPartRowsSkipped * P.part_stride + pi] = rs;
            }
        }
    }
}

// Rows of the wide tier's list, fetched dynamically (few rows, usually): 26.5
// KB of shared memory per block; the register budget of four wavefronts per
// SIMD keeps the persistent loop free of spills.  Rows that do not fit
// either go to the device-memory kernel's list.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) k_numeric_wide(StageArgs P)
{
    using Ws = LdsWave<kWideWords, kWideCap>;
    __shared__ Ws lds[kWavesPerBlock];
    const int wv = sgpr((int32_t)(threadIdx.x / kWave));
    Ws& me = lds[wv];
    const int l = lane();
    const unsigned long long count = __hip_atomic_load(&P.ctr->fb_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long kept = 0, rows = 0, mx = 0;
    while (true) {
        unsigned long long i = 0;
        if (l == 0) i = atomicAdd(&P.ctr->fb_next, 1ull);
        i = __shfl(i, 0, kWave);
        if (i >= count) break;
        const int64_t r = sgpr64(P.fb_list[i]);
        const int64_t o = sgpr64(P.out.off[r]);
        int64_t k = 0, ns = 0;
        if (process_row<false, false, Ws::kPark>(P, r, o, nullptr, me.bmp, me.acc, nullptr, me.st, kWideWords, kWideCap,
                                          &k, &ns)) {
            kept += (unsigned long long)k;
            mx = max(mx, (unsigned long long)ns);
            ++rows;
        } else if (l == 0) {
            defer_row(P, r, o, &P.ctr->fb2_count, P.fb2_list, P.global_planned);
        }
    }
    if (l == 0 && kept) atomicAdd(&P.ctr->kept_global, kept);
    if (l == 0 && rows) atomicAdd(&P.ctr->rows_wide, rows);
    if (l == 0 && mx) atomicMax(&P.ctr->max_ns, mx);
}

// Rows that did not fit shared memory: per-wave workspace in device memory
// sized for a full row, rows fetched dynamically from the device-memory list.
__global__ void __launch_bounds__(kBlock) k_numeric_global(StageArgs P)
{
    using Ws = LdsWave<kDevWords, kDevCap>;
    __shared__ Ws lds[kWavesPerBlock];
    const int wv = sgpr((int32_t)(threadIdx.x / kWave));
    Ws& me = lds[wv];
    const int l = lane();
    const int64_t slot = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (slot >= P.g_slots) return;
    uint32_t* base = P.g_scratch + slot * P.g_slot_stride;
    uint8_t* bytes = reinterpret_cast<uint8_t*>(base);
    uint2* bmp = reinterpret_cast<uint2*>(base + (P.g_slot_words + 1) * 8);
    double* acc = reinterpret_cast<double*>(base + P.g_off_acc);
    double* ebuf = reinterpret_cast<double*>(base + P.g_off_ebuf);
    const unsigned long long count = __hip_atomic_load(&P.ctr->fb2_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long kept = 0, mx = 0;
    while (true) {
        unsigned long long i = 0;
        if (l == 0) i = atomicAdd(&P.ctr->fb2_next, 1ull);
        i = __shfl(i, 0, kWave);
        if (i >= count) break;
        const int64_t r = sgpr64(P.fb2_list[i]);
        const int64_t o = sgpr64(P.out.off[r]);
        int64_t k = 0, ns = 0;
        // rows of up to 2048 entries in a window of up to 8192 columns keep
        // their structure and accumulator in shared memory
        if (!process_row<false, true, 1>(P, r, o, nullptr, me.bmp, me.acc, ebuf, me.st, kDevWords, kDevCap, &k,
                                         &ns) &&
            !process_row<true, true, 1>(P, r, o, bytes, bmp, acc, ebuf, me.st, P.g_slot_words, P.g_slot_cap, &k,
                                        &ns)) {
            flag_error(P, kErrCapacity);
            if (l == 0) empty_row(P, r, o);
        }
        kept += (unsigned long long)k;
        mx = max(mx, (unsigned long long)ns);
    }
    if (l == 0 && kept) atomicAdd(&P.ctr->kept_global, kept);
    if (l == 0 && mx) atomicMax(&P.ctr->max_ns, mx);
}

// ---------------------------------------------------------------------------
// Compaction of a slack matrix into canonical CSR.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_row_offsets(const int64_t* __restrict__ beg, const int64_t* __restrict__ end,
                                                        int64_t n, int64_t* rp, int64_t* blk_pre)
{
    __shared__ int64_t sh[kBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t len = (r < n) ? end[r] - beg[r] : 0;
    int64_t total = 0;
    const int64_t inc = block_incl_scan(len, sh, &total);
    if (r < n) rp[r] = inc - len;
    if (threadIdx.x == 0) blk_pre[blockIdx.x] = total;
}

// One wavefront per row; the row's entries four per lane at a time, all
// loads issued before the stores (input and output never overlap).
__global__ void __launch_bounds__(kBlock) k_compact(const int64_t* __restrict__ beg, const int64_t* __restrict__ end,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    int64_t n, int64_t* rp, const int64_t* __restrict__ blk_pre,
                                                    int32_t* __restrict__ ocol, double* __restrict__ oval)
{
    constexpr int kU4 = 4;
    const int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (r >= n) return;
    const int64_t b = beg[r], e = end[r], d = blk_pre[r >> 8] + rp[r];
    if (lane() == 0) rp[r] = d;
    for (int64_t p0 = b; p0 < e; p0 += kU4 * kWave) {
        int32_t c[kU4];
        double v[kU4];
#pragma unroll
        for (int u = 0; u < kU4; ++u) {
            const int64_t p = p0 + u * kWave + lane();
            if (p < e) {
                c[u] = col[p];
                v[u] = val[p];
            }
        }
#pragma unroll
        for (int u = 0; u < kU4; ++u) {
            const int64_t p = p0 + u * kWave + lane();
            if (p < e) {
                ocol[d + (p - b)] = c[u];
                oval[d + (p - b)] = v[u];
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(unsigned long long* p, int64_t count, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Adaptive filter (Algorithm 1) on a stage output in slack layout.
//
// The candidate norm at entry threshold t is the largest column sum of
// ceil(|x| * scale) over the entries with 0 < |x| <= t, summed exactly in
// 64-bit integers (so the result does not depend on the order of the atomic
// additions), scale = 2^40 / eps_g.
// ---------------------------------------------------------------------------
constexpr int kAlg1Rows = 32;       // rows per block of the candidate column sums
constexpr int kAlg1Cols = 6144;     // widest column window summed in shared memory
constexpr int kAlg1Threads = 1024;   // threads per block of the candidate column sums
constexpr int kAlg1Waves = kAlg1Threads / kWave;
static_assert(kAlg1Threads >= kAlg1Rows, "one thread per row reads the row summaries");

// Candidate column sums of rows [blockIdx.x * kAlg1Rows, ...): every entry
// with 0 < |x| <= t adds ceil(|x| scale) to sums[col].  When the block's rows
// span at most kAlg1Cols columns (from their summaries), the block sums in
// shared memory first and adds each column to the device array once; the
// integer sums do not depend on the order of the additions.
__device__ __forceinline__ void alg1_block_colsums(const int64_t* __restrict__ beg, const int64_t* __restrict__ end,
                                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                                   const RowInfo* __restrict__ info, int64_t n, double t,
                                                   double scale, unsigned long long* sums)
{
    __shared__ unsigned long long sh[kAlg1Cols];
    __shared__ int32_t wlo[kAlg1Waves], whi[kAlg1Waves];
    const int wv = threadIdx.x / kWave;
    const int64_t r0 = (int64_t)blockIdx.x * kAlg1Rows;
    const int64_t r1 = min(r0 + (int64_t)kAlg1Rows, n);
    int32_t f = INT_MAX, g = -1;
    if (r0 + (int64_t)threadIdx.x < r1) {
        const RowInfo q = load_info(info + r0 + threadIdx.x);
        if (q.len > 0) {
            f = q.first;
            g = q.last;
        }
    }
    f = wave_reduce<OpMin>(f);
    g = wave_reduce<OpMax>(g);
    if (lane() == 0) {
        wlo[wv] = f;
        whi[wv] = g;
    }
    __syncthreads();
    int32_t lo = INT_MAX, hi = -1;
    for (int k = 0; k < kAlg1Waves; ++k) {
        lo = min(lo, wlo[k]);
        hi = max(hi, whi[k]);
    }
    const bool local = hi >= lo && hi - lo < kAlg1Cols;  // uniform over the block
    if (local)
        for (int j = threadIdx.x; j <= hi - lo; j += kAlg1Threads) sh[j] = 0ull;
    __syncthreads();
    for (int64_t r = r0 + wv; r < r1; r += kAlg1Waves) {
        auto add = [&](double a, int32_t c) {
            if (a > 0.0 && a <= t) {
                const unsigned long long v = (unsigned long long)ceil(a * scale);
                // (a column outside the summaries' window goes to the device array)
                if (local && (uint32_t)(c - lo) <= (uint32_t)(hi - lo))
                    atomicAdd(&sh[c - lo], v);
                else
                    atomicAdd(&sums[c], v);
            }
        };
        const int64_t pe = end[r];
        int64_t p = beg[r] + lane();
        for (; p + kWave < pe; p += 2 * kWave) {  // two entries per lane in flight
            const double a0 = fabs(val[p]), a1 = fabs(val[p + kWave]);
            const int32_t c0 = col[p], c1 = col[p + kWave];
            add(a0, c0);
            add(a1, c1);
        }
        if (p < pe) add(fabs(val[p]), col[p]);
    }
    if (local) {
        __syncthreads();
        for (int j = threadIdx.x; j <= hi - lo; j += kAlg1Threads)
            if (sh[j] != 0ull) atomicAdd(&sums[lo + j], sh[j]);
    }
}

__global__ void __launch_bounds__(kAlg1Threads) k_alg1_colsum(const int64_t* __restrict__ beg, const int64_t* __restrict__ end,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, const RowInfo* info,
                                                        int64_t n, double t, double scale, unsigned long long* colsum)
{
    alg1_block_colsums(beg, end, col, val, info, n, t, scale, colsum);
}

__global__ void __launch_bounds__(kBlock) k_max_u64(const unsigned long long* __restrict__ x, int64_t n,
                                                    unsigned long long* out)
{
    __shared__ unsigned long long sh[kBlock / kWave];
    unsigned long long m = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        m = max(m, x[i]);
    m = group_max<kWave>(m);
    if (lane() == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock / kWave; ++i) t = max(t, sh[i]);
        atomicMax(out, t);
    }
}

// ---- Algorithm 1 driven on the device -------------------------------------------
// Iteration i uses the state left by iteration i - 1 (slot (i-1)&1) and the
// candidate norm it measured (max slot (i-1)%3), applies the update of
// Algorithm 1 (every thread computes the same values), stores its own state
// in slot i&1 (block 0 thread 0), and, unless the stopping test held,
// accumulates the integer candidate column sums at its threshold into the
// column buffer i&1 while clearing the buffers of iteration i + 1; a second
// kernel takes the largest column sum.  Both run grid-stride loops over a
// bounded grid, so the launches of iterations that are not needed are cheap.

__device__ __forceinline__ void alg1_update(Alg1State& st, const Alg1Params& pr, unsigned long long mx)
{
    const double c = (double)mx / pr.scale;
    const double m = c / st.t;
    st.it += 1;
    if (c > pr.target && st.it < pr.max_iter) {
        st.t = pr.eps_g / m;
    } else {
        st.done = 1;
        st.c = c;
    }
}

__device__ __forceinline__ Alg1State alg1_state(const Alg1Params& pr, int i, const Alg1State* st,
                                                const unsigned long long* mxs)
{
    if (i == 0) return Alg1State{pr.eps_g, 0.0, 0, 0, 0, 0};  // m_0 = 1
    Alg1State cur = st[(i - 1) & 1];
    if (!cur.done) alg1_update(cur, pr, mxs[(i - 1) % 3]);
    return cur;
}

__global__ void __launch_bounds__(kAlg1Threads) k_alg1_iter(const int64_t* __restrict__ beg, const int64_t* __restrict__ end,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val, const RowInfo* info, int64_t n,
                                                      Alg1Params pr, int i, Alg1State* st, unsigned long long* cs,
                                                      int fused0, const unsigned long long* __restrict__ base)
{
    unsigned long long* mxs = cs + 2 * n;
    const Alg1State cur = alg1_state(pr, i, st, mxs);
    if (blockIdx.x == 0 && threadIdx.x == 0) st[i & 1] = cur;
    // (a first iteration summed by the numeric kernel's write-out is not
    // launched: the host cleared every buffer before it, and the maximum
    // kernel records its state)
    if (cur.done || (i == 0 && fused0)) return;
    const int64_t nthreads = (int64_t)gridDim.x * kAlg1Threads;
    unsigned long long* next = cs + (int64_t)((i + 1) & 1) * n;
    // (base: column sums of entries the numeric write-out already removed,
    // all below every threshold tried, so every iteration's sums start there)
    for (int64_t g = (int64_t)blockIdx.x * kAlg1Threads + threadIdx.x; g < n; g += nthreads)
        next[g] = base != nullptr ? base[g] : 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) mxs[(i + 1) % 3] = 0ull;
    alg1_block_colsums(beg, end, col, val, info, n, cur.t, pr.scale, cs + (int64_t)(i & 1) * n);
}

// first: iteration 0 whose sums the numeric write-out took (no iteration
// launch before this one); block 0 records the first state.
__global__ void __launch_bounds__(kBlock) k_alg1_max(int64_t n, int i, Alg1State* st, unsigned long long* cs,
                                                     int first, double eps_g)
{
    if (first) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = Alg1State{eps_g, 0.0, 0, 0, 0, 0};  // m_0 = 1
    } else if (st[i & 1].done) {
        return;
    }
    __shared__ unsigned long long sh[kBlock / kWave];
    const unsigned long long* sums = cs + (int64_t)(i & 1) * n;
    unsigned long long m = 0;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock)
        m = max(m, sums[g]);
    m = group_max<kWave>(m);
    if (lane() == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t = max(t, sh[k]);
        if (t) atomicMax(&cs[2 * n + i % 3], t);
    }
}

// One-iteration check for a stage whose write-out already dropped |x| <=
// eps_g and summed those entries into cs[0, n): the candidate norm (maximum
// column sum) and, in the last block to finish, the final state of
// Algorithm 1 and its flags, as the iteration, maximum and final-state
// kernels would record them.  cs[2n + 1] counts finished blocks (cleared with
// the sums; cleared again by the last block).
__global__ void __launch_bounds__(kBlock) k_alg1_check1(int64_t n, Alg1Params pr, Alg1State* st,
                                                        unsigned long long* cs, StageCounters* ctr)
{
    __shared__ unsigned long long sh[kBlock / kWave];
    __shared__ int last;
    unsigned long long* mxs = cs + 2 * n;
    unsigned long long m = 0;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock)
        m = max(m, cs[g]);
    m = group_max<kWave>(m);
    if (lane() == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kBlock / kWave; ++k) t = max(t, sh[k]);
        if (t) atomicMax(&mxs[0], t);
        __threadfence();
        last = atomicAdd(&mxs[1], 1ull) == (unsigned long long)(gridDim.x - 1);
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    const unsigned long long mx = atomicAdd(&mxs[0], 0ull);
    const Alg1State first{pr.eps_g, 0.0, 0, 0, 0, 0};  // m_0 = 1
    Alg1State fin = first;
    alg1_update(fin, pr, mx);
    const bool miss = fin.done && fin.t != pr.eps_g;  // never: a stop keeps the first threshold
    Alg1State rec = fin;
    rec.ok = fin.done && !miss;
    st[0] = first;
    st[2] = rec;
    if (!fin.done || miss) atomicOr(&ctr->errors, kErrAlg1Pending);
    if (rec.ok && fin.c > pr.target) atomicOr(&ctr->errors, kErrCapacity);  // iteration limit reached
    mxs[1] = 0ull;
}

// Drops the entries with |x| <= t of every row in place (the kept entries
// keep their order), updates end, span, amax and the structure words, and
// writes per-block kept counts into `part_kept` (same block layout as the
// numeric kernel).
template <bool kDevice>
__global__ void __launch_bounds__(kBlock) k_alg1_drop_t(const int64_t* __restrict__ beg, int64_t* end, int32_t* col,
                                                        double* val, RowInfo* info, uint2* sw, int32_t* nw,
                                                        int64_t n, double t,
                                                        unsigned long long* part_kept, Alg1Params pr, int iters,
                                                        Alg1State* st, const unsigned long long* cs,
                                                        StageCounters* ctr, int finalize_only)
{
    if (kDevice) {  // the final update; the threshold is the last one used
        const Alg1State fin = alg1_state(pr, iters, st, cs + 2 * n);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            // finalize_only: the write-out dropped at threshold t, which must
            // be the one the iteration ends with
            const bool miss = finalize_only && fin.done && fin.t != t;
            Alg1State rec = fin;
            rec.ok = fin.done && !miss;
            st[2] = rec;
            if (!fin.done || miss) atomicOr(&ctr->errors, kErrAlg1Pending);
            if (rec.ok && fin.c > pr.target) atomicOr(&ctr->errors, kErrCapacity);  // iteration limit reached
        }
        if (!fin.done || finalize_only) return;
        t = fin.t;
    }
    // the drop recounts every row (per-block partials), including those of
    // the fallback kernels, whose separate count is cleared
    if (ctr != nullptr && blockIdx.x == 0 && threadIdx.x == 0) ctr->kept_global = 0ull;
    __shared__ unsigned long long kept_sh[kWavesPerBlock];
    __shared__ uint32_t seg_sh[kWavesPerBlock][kWave];
    __shared__ uint32_t stage_sh[kWavesPerBlock][2 * kWave];
    const int wv = threadIdx.x / kWave;
    const int l = lane();
    const int64_t blk = xcd_logical_block();
    const int64_t r = blk * kWavesPerBlock + wv;
    int64_t kept = 0;
    if (r < n) {
        const int64_t b = beg[r], e = end[r];
        double amx = 0.0;
        int32_t first = INT_MAX, last = -1;
        // The kept columns are staged in order in shared memory and handed to
        // the word builder 64 at a time.
        WaveWordBuilder wb{sw + b, seg_sh[wv]};
        uint32_t* stg = stage_sh[wv];
        int32_t staged = 0;
        int32_t c = 0;
        double x = 0.0;
        if (b + l < e) {
            c = col[b + l];
            x = val[b + l];
        }
        for (int64_t p0 = b; p0 < e; p0 += kWave) {
            const int64_t p = p0 + l;
            const bool keep = p < e && fabs(x) > t;
            // The next 64 entries lie past every position this batch writes
            // (kept <= p0 - b), so they are loaded before its stores.
            int32_t cn = 0;
            double xn = 0.0;
            if (p + kWave < e) {
                cn = col[p + kWave];
                xn = val[p + kWave];
            }
            const unsigned long long m = __ballot(keep);
            const int32_t below = (int32_t)lanes_below(m);
            if (keep) {
                const int64_t q = b + kept + below;
                col[q] = c;
                val[q] = x;
                amx = fmax(amx, fabs(x));
                first = min(first, c);
                last = max(last, c);
                stg[staged + below] = (uint32_t)c;
            }
            kept += __popcll(m);
            staged += __popcll(m);
            if (staged >= kWave) {  // staged <= 127
                wave_sync();
                const int32_t cc = (int32_t)stg[l];
                const uint32_t rest = stg[kWave + l];
                wave_sync();
                if (l < staged - kWave) stg[l] = rest;
                staged -= kWave;
                wb.add(cc, kWave);
            }
            c = cn;
            x = xn;
        }
        if (staged > 0) {
            wave_sync();
            const int32_t cc = l < staged ? (int32_t)stg[l] : 0;
            wb.add(cc, staged);
        }
        amx = wave_reduce<OpMax>(amx);
        first = wave_reduce<OpMin>(first);
        last = wave_reduce<OpMax>(last);
        const int32_t words = wb.finish();
        if (l == 0) {
            end[r] = b + kept;
            info[r] = row_info(kept, first, last, amx);
            nw[r] = words;
        }
    }
    if (l == 0) kept_sh[wv] = (unsigned long long)kept;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) s += kept_sh[i];
        part_kept[blk] = s;
    }
}

inline unsigned blocks_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

}  // namespace

// ---- launch wrappers -------------------------------------------------------

hipError_t launch_rowinfo_csr(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n, RowInfo* info,
                              uint2* sw, int32_t* nw, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowinfo_csr, dim3(blocks_for(n * 16)), dim3(kBlock), 0, s, row_ptr, col, val, n, info, sw,
                       nw);
    return hipGetLastError();
}

hipError_t launch_validate_csr(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n, int64_t nnz,
                               unsigned long long* err, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate_csr, dim3(blocks_for(n > 0 ? n : 1)), dim3(kBlock), 0, s, row_ptr, col, val, n, nnz,
                       err);
    return hipGetLastError();
}

hipError_t launch_block_scan(int64_t* x, int64_t nblk, int64_t* grand, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_scan, dim3(1), dim3(kBlock), 0, s, x, nblk, grand);
    return hipGetLastError();
}

hipError_t launch_analyze(const StageArgs& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (a.mode == kModeProduct)
        hipLaunchKernelGGL(k_analyze_product, dim3((unsigned)analyze_blocks(a.mode, a.n)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_analyze_sum, dim3((unsigned)analyze_blocks(a.mode, a.n)), dim3(kBlock), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.row_stride > 0) return e;
    return launch_block_scan(a.blk_pre, analyze_blocks(a.mode, a.n), a.out.off + a.n, s);
}

int analyze_shift(int32_t mode) { return mode == kModeProduct ? kAnalyzeShiftProduct : kAnalyzeShiftSum; }

int64_t analyze_blocks(int32_t mode, int64_t n)
{
    return mode == kModeProduct ? (n * kAnalyzeLanes + kBlock - 1) / kBlock : (n + kBlock - 1) / kBlock;
}

int64_t numeric_blocks(int64_t n) { return (n + kWavesPerBlock - 1) / kWavesPerBlock; }

hipError_t launch_numeric_lds(const StageArgs& a, int grid, hipStream_t s)
{
    (void)grid;
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_numeric_lds, dim3((unsigned)numeric_blocks(a.n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_numeric_small(const StageArgs& a, int64_t max_ns, int64_t max_words, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = (a.n + kSmallRowsPerBlock - 1) / kSmallRowsPerBlock;
    (void)max_ns;
    (void)max_words;
    const dim3 g((unsigned)blocks), b(kBlock);
    if (a.has_blk)
        hipLaunchKernelGGL((k_numeric_small<kSmallWords, kSmallCap, 6, true>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((k_numeric_small<kSmallWords, kSmallCap, 6, false>), g, b, 0, s, a);
    return hipGetLastError();
}

bool small_tier_fits(int64_t n, int64_t max_ns, int64_t max_words)
{
    return n > kSmallMinRows && max_ns <= kSmallCap && max_words <= kSmallWords;
}

bool small_tier_most(int64_t n, int64_t big)
{
    return n > kSmallMinRows && big * kSmallBigShare <= n;
}

hipError_t launch_numeric_wide_rows(const StageArgs& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_numeric_wide_rows, dim3((unsigned)numeric_blocks(a.n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_numeric_wide(const StageArgs& a, int grid, hipStream_t s)
{
    if (a.n <= 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_numeric_wide, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_numeric_global(const StageArgs& a, int grid, hipStream_t s)
{
    if (a.n <= 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_numeric_global, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

int64_t offset_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

hipError_t launch_row_offsets(const int64_t* beg, const int64_t* end, int64_t n, int64_t* rp, int64_t* blk_pre,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_offsets, dim3(blocks_for(n)), dim3(kBlock), 0, s, beg, end, n, rp, blk_pre);
    return launch_block_scan(blk_pre, offset_blocks(n), rp + n, s);
}

hipError_t launch_compact(const int64_t* beg, const int64_t* end, const int32_t* col, const double* val, int64_t n,
                          int64_t* rp, const int64_t* blk_pre, int32_t* ocol, double* oval, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(blocks_for(n * kWave)), dim3(kBlock), 0, s, beg, end, col, val, n, rp,
                       blk_pre, ocol, oval);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(count)), dim3(kBlock), 0, s, p, count, v);
    return hipGetLastError();
}

int numeric_waves_per_block() { return kWavesPerBlock; }

hipError_t launch_alg1_colsum(const int64_t* beg, const int64_t* end, const int32_t* col, const double* val,
                              const RowInfo* info, int64_t n, double t, double scale, unsigned long long* colsum,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alg1_colsum, dim3((unsigned)((n + kAlg1Rows - 1) / kAlg1Rows)), dim3(kAlg1Threads), 0, s, beg, end,
                       col, val, info, n, t, scale, colsum);
    return hipGetLastError();
}

hipError_t launch_max_u64(const unsigned long long* x, int64_t n, unsigned long long* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_max_u64, dim3(blocks), dim3(kBlock), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_alg1_drop(const int64_t* beg, int64_t* end, int32_t* col, double* val, RowInfo* info, uint2* sw,
                            int32_t* nw, int64_t n, double t, unsigned long long* part_kept, StageCounters* ctr,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_alg1_drop_t<false>, dim3((unsigned)numeric_blocks(n)), dim3(kBlock), 0, s, beg, end, col, val,
                       info, sw, nw, n, t, part_kept, Alg1Params{}, 0, (Alg1State*)nullptr,
                       (const unsigned long long*)nullptr, ctr, 0);
    return hipGetLastError();
}

hipError_t launch_alg1_device(const int64_t* beg, int64_t* end, int32_t* col, double* val, RowInfo* info,
                              uint2* sw, int32_t* nw, int64_t n, const Alg1Params& pr, int iters, Alg1State* st, unsigned long long* cs,
                              unsigned long long* part_kept, StageCounters* ctr, int fused0, int finalize_only,
                              double t_dropped, const unsigned long long* base, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)numeric_blocks(n);
    const unsigned iter_blocks = (unsigned)((n + kAlg1Rows - 1) / kAlg1Rows);
    const unsigned max_blocks = (unsigned)std::min<int64_t>(256, (n + kBlock - 1) / kBlock);
    if (finalize_only && iters == 1 && base == nullptr && t_dropped == pr.eps_g) {
        hipLaunchKernelGGL(k_alg1_check1, dim3(max_blocks), dim3(kBlock), 0, s, n, pr, st, cs, ctr);
        return hipGetLastError();
    }
    for (int i = 0; i < iters; ++i) {
        // (the first iteration of a write-out that took its sums has only its
        // maximum to take)
        const int first = i == 0 && fused0 ? 1 : 0;
        if (!first)
            hipLaunchKernelGGL(k_alg1_iter, dim3(iter_blocks), dim3(kAlg1Threads), 0, s, (const int64_t*)beg,
                               (const int64_t*)end, (const int32_t*)col, (const double*)val, (const RowInfo*)info, n,
                               pr, i, st, cs, fused0, base);
        hipLaunchKernelGGL(k_alg1_max, dim3(max_blocks), dim3(kBlock), 0, s, n, i, st, cs, first, pr.eps_g);
    }
    // (finalize_only: the numeric write-out already applied the threshold; one
    // block records the final state and raises the flags)
    hipLaunchKernelGGL(k_alg1_drop_t<true>, dim3(finalize_only ? 1u : blocks), dim3(kBlock), 0, s, beg, end, col,
                       val, info, sw, nw, n, finalize_only ? t_dropped : 0.0,
                       part_kept, pr, iters, st, (const unsigned long long*)cs, ctr, finalize_only);
    return hipGetLastError();
}

int numeric_global_blocks(int slots) { return slots / kWavesPerBlock; }

int numeric_wide_blocks(int64_t n) { return (int)std::min<int64_t>(numeric_blocks(n), 1536); }

}  // namespace fps
