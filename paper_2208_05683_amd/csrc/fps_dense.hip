// HIP kernels (gfx950) of the dense path: a sparse product whose work has
// grown to a sizeable fraction of a dense one (the fill of the powers and of
// the Horner states that the paper notes after eq. 9) is computed as a dense
// FP64 matrix product on the matrix cores (v_mfma_f64_16x16x4f64), with the
// coefficient block added and the filter applied in the product's write-out:
//     C = D_tau(E + A B)            (eq. 11 with E = 0, eq. 14 with E = Bhat)
// The operands are stored dense and row-major with a leading dimension ld
// (n rounded up to 128, the padding zero), and the result is written back as
// the same slack-CSR rows the sparse kernels write (entries in column order,
// row summary, structure words, per-block counts), so later stages read it
// as any other stage output.  The products are summed in the matrix cores'
// order, not the ordered sparse one: results agree with the sparse path to
// rounding, not bit for bit.  Bhat itself is formed in the sparse path's
// order (ascending terms, one fused multiply-add each from +0), so it is
// bit-identical.
#include "fps_device.h"

#include <climits>

namespace fps {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kB = 256;
constexpr int kRowsPerBlock = 4;  // write-out: one wavefront per row, as the numeric kernels

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kB - 1) / kB); }

__device__ __forceinline__ unsigned lanes_below64(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// E[r][c] = sum_t coef_t M_t[r][c] for columns c < n, accumulated over
// ascending t with one fused multiply-add per stored entry from +0 (M_t the
// identity when beg[t] is null); every such entry of E is written, zeros
// included, so E needs no clearing.  One wavefront per (row, chunk of
// kTermCols columns): the chunk is summed in shared memory term by term (the
// entries of one term row have distinct columns, so its lanes never meet on
// one slot; terms are ordered by a wavefront barrier), then written out in
// one coalesced pass.
constexpr int kTermCols = 1024;  // 8 KB of shared memory per wavefront
constexpr int kTermWaves = kB / kWave;

__device__ __forceinline__ void dense_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The first position p in [lo, hi) of the sorted columns cl with
// cl[p] >= key, hi if there is none; the same on every lane.  Each round
// probes 64 evenly spaced positions at once and keeps the piece between the
// last probe below the key and the first one at or above it (a 64-fold
// narrowing per dependent load); the last piece, at most 64 positions, is
// read whole.
__device__ __forceinline__ int64_t first_at_least(const int32_t* __restrict__ cl, int64_t lo, int64_t hi, int32_t key)
{
    const int l = threadIdx.x % kWave;
    while (hi - lo > kWave) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t q = min(lo + (int64_t)(l + 1) * step - 1, hi - 1);
        const int j0 = __popcll(__ballot(cl[q] < key));  // probes below the key: a prefix
        if (j0 == kWave) return hi;  // the last probe is hi - 1
        const int64_t nlo = j0 > 0 ? min(lo + (int64_t)j0 * step - 1, hi - 1) + 1 : lo;
        hi = min(lo + (int64_t)(j0 + 1) * step - 1, hi - 1);  // a probe at or above the key
        lo = nlo;
    }
    const int64_t p = lo + l;
    return lo + __popcll(__ballot(p < hi && cl[p] < key));
}

__global__ void __launch_bounds__(kB) k_dense_terms(Terms T, int64_t n, int64_t ld, double* E)
{
    __shared__ double acc_sh[kTermWaves][kTermCols];
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int64_t chunks = (n + kTermCols - 1) / kTermCols;
    const int64_t item = (int64_t)blockIdx.x * kTermWaves + wv;
    if (item >= n * chunks) return;  // (no block-wide barrier below)
    const int64_t r = item / chunks;
    const int32_t c0 = (int32_t)((item % chunks) * kTermCols);
    const int32_t c1 = (int32_t)min<int64_t>((int64_t)c0 + kTermCols, n);
    double* acc = acc_sh[wv];
    for (int i = l; i < kTermCols; i += kWave) acc[i] = 0.0;
    dense_wave_sync();
    for (int t = 0; t < T.n; ++t) {
        const double c = T.coef[t];
        if (T.beg[t] == nullptr) {
            if (l == 0 && r >= c0 && r < c1) acc[r - c0] = fma(c, 1.0, acc[r - c0]);
        } else {
            const int32_t* __restrict__ cl = T.col[t];
            const double* __restrict__ vl = T.val[t];
            const int64_t e = T.end[t][r];
            int64_t p0 = T.beg[t][r];
            if (c0 > 0) p0 = first_at_least(cl, p0, e, c0);
            // the chunk's entries in batches of 4 x 64 (column and value
            // loads together); positions past the chunk come last in a sorted row
            for (; p0 < e; p0 += 4 * kWave) {
                int32_t k[4];
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t p = p0 + u * kWave + l;
                    k[u] = p < e ? cl[p] : INT_MAX;
                    v[u] = p < e ? vl[p] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (k[u] < c1) acc[k[u] - c0] = fma(c, v[u], acc[k[u] - c0]);
                if (__ballot(k[3] >= c1) != 0ull) break;  // the batch's last position is past the chunk
            }
        }
        dense_wave_sync();
    }
    double* row = E + r * ld;
    for (int32_t i = c0 + l; i < c1; i += kWave) row[i] = acc[i - c0];
}

// ---- densify --------------------------------------------------------------

// D = M as a dense ld x ld matrix with every entry written (zeros included,
// the padding rows and columns beyond n too), so D needs no clearing.  One
// wavefront per (row, chunk of kTermCols columns): the chunk is assembled in
// shared memory (a row's columns are distinct) and written out whole.
__global__ void __launch_bounds__(kB) k_densify(MatView M, int64_t n, int64_t ld, double* D)
{
    __shared__ double row_sh[kTermWaves][kTermCols];
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int64_t chunks = (ld + kTermCols - 1) / kTermCols;
    const int64_t item = (int64_t)blockIdx.x * kTermWaves + wv;
    if (item >= ld * chunks) return;  // (no block-wide barrier below)
    const int64_t r = item / chunks;
    const int32_t c0 = (int32_t)((item % chunks) * kTermCols);
    const int32_t c1 = (int32_t)min<int64_t>((int64_t)c0 + kTermCols, ld);
    double* sh = row_sh[wv];
    for (int i = l; i < kTermCols; i += kWave) sh[i] = 0.0;
    dense_wave_sync();
    if (r < n) {
        const int64_t e = M.end[r];
        int64_t p0 = M.beg[r];
        if (c0 > 0) p0 = first_at_least(M.col, p0, e, c0);
        for (; p0 < e; p0 += 4 * kWave) {
            int32_t k[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = p0 + u * kWave + l;
                k[u] = p < e ? M.col[p] : INT_MAX;
                v[u] = p < e ? M.val[p] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k[u] < c1) sh[k[u] - c0] = v[u];
            if (__ballot(k[3] >= c1) != 0ull) break;  // the batch's last position is past the chunk
        }
        dense_wave_sync();
    }
    double* row = D + r * ld;
    for (int32_t i = c0 + l; i < c1; i += kWave) row[i] = sh[i - c0];
}

// ---- the product on the matrix cores ----------------------------------------
//
// Block tile BM x BM of C (128, 64 or 32: the largest that gives the chip
// 512 blocks), four wavefronts in 2 x 2, each a (BM/2) x (BM/2) tile made
// of 16 x 16 MFMA tiles.  K advances in chunks of 16 staged in
// shared memory, A k-major and B row-major, so that the 16 lanes of a
// quarter-wave read 16 consecutive doubles.  Lane layout of
// v_mfma_f64_16x16x4f64 (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of the 16 x 4 and 4 x 16 operands, and item v of its
// result holds C[4 v + l / 16][l % 16].
// Two wavefronts per SIMD for the 128 x 128 tile: its accumulators then live
// in VGPRs (198 in all) instead of AGPRs next to 194 VGPRs, which left one.
template <int BM>
__global__ void __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(BM == 128 ? 2 : 4, 8)))
k_dgemm_mfma(const double* __restrict__ A, const double* __restrict__ B,
                                                   double* E, int64_t ld, int64_t n, int has_e, double tau,
                                                   const double* __restrict__ tau_row)
{
    constexpr int KC = 16;
    constexpr int WM = BM / 2;   // wave tile
    constexpr int TM = WM / 16;  // MFMA tiles per wave dimension
    constexpr int PAD = 2;
    constexpr int PER = BM * KC / kB;  // doubles of each operand chunk per thread
    __shared__ double As[KC][BM + PAD];
    __shared__ double Bs[KC][BM + PAD];
    const int t = threadIdx.x, l = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
    const int64_t row0 = (int64_t)blockIdx.y * BM, col0 = (int64_t)blockIdx.x * BM;
    v4d acc[TM][TM];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TM; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    // chunk loads: A rows (t / (KC / PER)), PER consecutive k; B row (t / (BM / PER)), PER consecutive columns
    constexpr int AQ = KC / PER;  // threads per A row
    constexpr int BQ = BM / PER;  // threads per B row
    const int ar = t / AQ, ak = (t % AQ) * PER;
    const int bk = t / BQ, bc = (t % BQ) * PER;
    const double* pa = A + (row0 + ar) * ld + ak;
    const double* pb = B + (int64_t)bk * ld + col0 + bc;
    double ra[PER], rb[PER];
#pragma unroll
    for (int i = 0; i < PER; i += 2) {
        const double2 x = *reinterpret_cast<const double2*>(pa + i);
        const double2 y = *reinterpret_cast<const double2*>(pb + i);
        ra[i] = x.x;
        ra[i + 1] = x.y;
        rb[i] = y.x;
        rb[i + 1] = y.y;
    }
    for (int64_t k0 = 0; k0 < ld; k0 += KC) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            As[ak + i][ar] = ra[i];
            Bs[bk][bc + i] = rb[i];
        }
        __syncthreads();
        if (k0 + KC < ld) {  // the next chunk's loads overlap this chunk's products
            const double* na = pa + (k0 + KC);
            const double* nb = pb + (k0 + KC) * ld;
#pragma unroll
            for (int i = 0; i < PER; i += 2) {
                const double2 x = *reinterpret_cast<const double2*>(na + i);
                const double2 y = *reinterpret_cast<const double2*>(nb + i);
                ra[i] = x.x;
                ra[i + 1] = x.y;
                rb[i] = y.x;
                rb[i + 1] = y.y;
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            double a[TM], b[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[kk + (l >> 4)][wr * WM + i * 16 + (l & 15)];
#pragma unroll
            for (int j = 0; j < TM; ++j) b[j] = Bs[kk + (l >> 4)][wc * WM + j * 16 + (l & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // write-out: x = E + product (one addition), then the filter
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TM; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = row0 + wr * WM + i * 16 + 4 * v + (l >> 4);
                const int64_t gj = col0 + wc * WM + j * 16 + (l & 15);
                if (gi < n && gj < n) {
                    double x = acc[i][j][v];
                    double* pe = E + gi * ld + gj;
                    if (has_e) x = *pe + x;
                    const double tr = tau_row ? tau_row[gi] : tau;
                    *pe = (x != 0.0 && !(fabs(x) < tr)) ? x : 0.0;
                }
            }
}

// ---- the dense product in k order on the vector units ---------------------------------
// C = D_tau(E + A B) with every entry's sum taken over k = 0, 1, ..., ld - 1
// in order, one fma per k from +0: the sparse path's fma chain over the
// stored entries of A's row (ascending columns) with exact zeros added for
// the others, so the sparse result bit for bit (as in k_spmm_rows below).
// FP64 fma on the vector units has the matrix cores' FP64 peak on this chip.
// Block tile BT x BT (128, or 64 when that gives the chip too few blocks),
// 256 threads as 16 x 16; thread (ty, tx) owns the row pairs
// 2 ty + 32 i + {0, 1} and the column pairs 2 tx + 32 j + {0, 1}
// (i, j < BT / 32), so that each k row of A and of B is read with 16-byte
// loads (a wavefront's reads of A are broadcasts, of B sixteen consecutive
// pairs); k in chunks of 16 staged in shared memory (A k-major), the next
// chunk's global loads in flight during the current chunk's fmas.
constexpr int kOK = 16;

template <int BT>
__global__ void __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(BT == 128 ? 2 : 4, 8)))
k_dgemm_ordered(const double* __restrict__ A, const double* __restrict__ B, double* E, int64_t ld, int64_t n,
                int has_e, double tau, const double* __restrict__ tau_row)
{
    constexpr int R = BT / 16;          // rows (and columns) per thread
    constexpr int PER = BT * kOK / kB;  // doubles of each operand chunk per thread
    constexpr int AQ = kOK / PER;       // threads per A row of a chunk
    constexpr int BQ = BT / PER;        // threads per B k row of a chunk
    __shared__ __align__(16) double As[2][kOK][BT];
    __shared__ __align__(16) double Bs[2][kOK][BT];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t row0 = (int64_t)blockIdx.y * BT, col0 = (int64_t)blockIdx.x * BT;
    double acc[R][R];  // [row 2 i + u][column 2 j + v] of the thread's pairs
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[i][j] = 0.0;
    const int ar = t / AQ, ak = (t % AQ) * PER;
    const int bk = t / BQ, bc = (t % BQ) * PER;
    const double* pa = A + (row0 + ar) * ld + ak;
    const double* pb = B + (int64_t)bk * ld + col0 + bc;
    double ra[PER], rb[PER];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < PER; i += 2) {
            const double2 x = *reinterpret_cast<const double2*>(pa + k0 + i);
            const double2 y = *reinterpret_cast<const double2*>(pb + k0 * ld + i);
            ra[i] = x.x;
            ra[i + 1] = x.y;
            rb[i] = y.x;
            rb[i + 1] = y.y;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            As[buf][ak + i][ar] = ra[i];
            Bs[buf][bk][bc + i] = rb[i];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    // two buffers: chunk c is read from buffer c & 1 while chunk c + 1 goes
    // to the other one, which every wavefront finished reading before the
    // barrier that ended chunk c - 1; one barrier per chunk
    for (int64_t k0 = 0, c = 0; k0 < ld; k0 += kOK, ++c) {
        const int buf = (int)(c & 1);
        const bool more = k0 + kOK < ld;
        if (more) fetch(k0 + kOK);
#pragma unroll 2
        for (int kk = 0; kk < kOK; ++kk) {
            double a[R], b[R];
#pragma unroll
            for (int i = 0; i < R / 2; ++i) {
                const double2 x = *reinterpret_cast<const double2*>(&As[buf][kk][2 * ty + 32 * i]);
                a[2 * i] = x.x;
                a[2 * i + 1] = x.y;
            }
#pragma unroll
            for (int j = 0; j < R / 2; ++j) {
                const double2 y = *reinterpret_cast<const double2*>(&Bs[buf][kk][2 * tx + 32 * j]);
                b[2 * j] = y.x;
                b[2 * j + 1] = y.y;
            }
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
    }
    // write-out: x = E + product (one addition), then the filter
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int64_t gi = row0 + 2 * ty + 32 * (i >> 1) + (i & 1);
        if (gi >= n) continue;
        const double tr = tau_row ? tau_row[gi] : tau;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t gj = col0 + 2 * tx + 32 * (j >> 1) + (j & 1);
            if (gj < n) {
                double x = acc[i][j];
                double* pe = E + gi * ld + gj;
                if (has_e) x = *pe + x;
                *pe = (x != 0.0 && !(fabs(x) < tr)) ? x : 0.0;
            }
        }
    }
}

// ---- sparse rows times dense rows -------------------------------------------------
// C = D_tau(E + A B) with A sparse (row-range CSR, rows < n) and B dense (ld
// columns).  Each output entry is the fma chain over row r's stored entries
// of A in column order from +0, as in the sparse kernels.  Where B[k][c] is
// zero (no stored entry) the fma adds an exact zero, which leaves the sum
// unchanged (+0 stays +0: the sum is never -0, a stored product being
// nonzero), so every entry the sparse path keeps has the same bits here,
// and every column it never forms is 0 here and dropped.  One block per
// (row, chunk of kRowsCols columns), kRowsPer columns per thread.
constexpr int kRowsPer = 8;
constexpr int kRowsCols = kB * kRowsPer;

__global__ void __launch_bounds__(kB) k_spmm_rows(MatView A, const double* __restrict__ B, double* E, int64_t ld,
                                                  int64_t n, int has_e, double tau, const double* __restrict__ tau_row)
{
    const int64_t r = blockIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * kRowsCols + threadIdx.x;
    double acc[kRowsPer];
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) acc[j] = 0.0;
    const int64_t pb = A.beg[r], pe = A.end[r];
    for (int64_t p = pb; p < pe; ++p) {
        const int64_t k = A.col[p];
        const double a = A.val[p];
        const double* bk = B + k * ld;
#pragma unroll
        for (int j = 0; j < kRowsPer; ++j) {
            const int64_t c = c0 + (int64_t)j * kB;
            if (c < n) acc[j] = fma(a, bk[c], acc[j]);
        }
    }
    double* er = E + r * ld;
    const double tr = tau_row ? tau_row[r] : tau;
#pragma unroll
    for (int j = 0; j < kRowsPer; ++j) {
        const int64_t c = c0 + (int64_t)j * kB;
        if (c < n) {
            double x = acc[j];
            if (has_e) x = er[c] + x;  // x = extra + main, one addition
            er[c] = (x != 0.0 && !(fabs(x) < tr)) ? x : 0.0;
        }
    }
}

// ---- back to slack-CSR rows -----------------------------------------------------

// Row r of the dense result C as a stage output row: placed as the numeric
// kernels place it (a fixed stride, or the analysis' block prefix plus its
// offset), its nonzero entries in column order, its summary and structure
// words; a row that does not fit its room is left empty and flagged.  The
// block's kept count and largest row go to the stage's partial sums.
__global__ void __launch_bounds__(kB) k_dense_to_slack(const double* __restrict__ C, int64_t ld, StageArgs P)
{
    __shared__ unsigned long long kept_sh[kRowsPerBlock];
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
    const int64_t blk = blockIdx.x;
    const int64_t r = blk * kRowsPerBlock + wv;
    int64_t kept = 0;
    if (r < P.n) {
        const int64_t o = P.row_stride > 0 ? r * P.row_stride : P.blk_pre[r >> P.scan_shift] + P.out.off[r];
        const int64_t room = P.row_stride > 0 ? P.row_stride : P.out.cap - o;
        if (l == 0) P.out.off[r] = o;
        const double* row = C + r * ld;
        double amx = 0.0;
        int32_t first = INT_MAX, last = -1, nwd = 0;
        // 64 columns per step, the loads of four steps issued together
        constexpr int kU = 4;
        for (int64_t cb = 0; cb < P.n; cb += kU * kWave) {
            double xs[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t c = cb + u * kWave + l;
                xs[u] = c < P.n ? row[c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t c0 = cb + u * kWave;
                const int64_t c = c0 + l;
                const double x = xs[u];
                const bool nz = x != 0.0;
                const unsigned long long m = __ballot(nz);
                if (nz) {
                    const int64_t pos = kept + (int64_t)lanes_below64(m);
                    if (pos < room) {
                        P.out.col[o + pos] = (int32_t)c;
                        P.out.val[o + pos] = x;
                    }
                    // Algorithm 1's first-iteration candidates (|x| <= dthr), as
                    // the sparse write-out sums them
                    if (P.dsum != nullptr && fabs(x) <= P.dthr)
                        atomicAdd(&P.dsum[c], (unsigned long long)ceil(fabs(x) * P.dscale));
                    amx = fmax(amx, fabs(x));
                    first = min(first, (int32_t)c);
                    last = max(last, (int32_t)c);
                }
                kept += __popcll(m);
                // structure words: the step's two 32-column words (c0 is a multiple of 64)
                const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
                if (l == 0) {
                    if (lo && nwd < room) P.out.sw[o + nwd] = make_uint2((uint32_t)(c0 >> 5), lo);
                    nwd += lo ? 1 : 0;
                    if (hi && nwd < room) P.out.sw[o + nwd] = make_uint2((uint32_t)(c0 >> 5) + 1u, hi);
                    nwd += hi ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) {
            amx = fmax(amx, __shfl_xor(amx, d, kWave));
            first = min(first, __shfl_xor(first, d, kWave));
            last = max(last, __shfl_xor(last, d, kWave));
        }
        if (l == 0) {
            RowInfo q;
            if (kept > room) {  // the row does not fit: left empty, the evaluation is repeated with sizing
                atomicOr(&P.ctr->errors, kErrCapacity);
                P.out.end[r] = o;
                q.len = 0;
                q.first = 1;
                q.last = 0;
                q.amax = 0.0f;
                P.out.nw[r] = 0;
                kept = 0;
            } else {
                P.out.end[r] = o + kept;
                q.len = (int32_t)kept;
                q.first = kept > 0 ? first : 1;
                q.last = kept > 0 ? last : 0;
                q.amax = __double2float_ru(amx);
                P.out.nw[r] = nwd;
            }
            P.out.info[r] = q;
        }
    }
    if (l == 0) kept_sh[wv] = (unsigned long long)kept;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0, mx = 0;
        for (int i = 0; i < kRowsPerBlock; ++i) {
            s += kept_sh[i];
            mx = max(mx, kept_sh[i]);
        }
        P.part[kPartKept * P.part_stride + blk] = s;
        P.part[kPartMaxNs * P.part_stride + blk] = mx;
    }
}

// Block tile of the dense products: the largest of 128, 64 and 32 whose
// tiles number at least 512 (two blocks per CU), else 32; ld is a multiple
// of 128.
int dense_tile(int64_t ld)
{
    for (int bm = 128; bm > 32; bm /= 2)
        if ((ld / bm) * (ld / bm) >= 512) return bm;
    return 32;
}

}  // namespace

int64_t dense_ld(int64_t n) { return (n + 127) / 128 * 128; }

hipError_t launch_densify(const MatView& M, int64_t n, int64_t ld, double* D, hipStream_t s)
{
    const int64_t items = ld * ((ld + kTermCols - 1) / kTermCols);
    hipLaunchKernelGGL(k_densify, dim3((unsigned)((items + kTermWaves - 1) / kTermWaves)), dim3(kB), 0, s, M, n, ld,
                       D);
    return hipGetLastError();
}

hipError_t launch_dense_terms(const Terms& T, int64_t n, int64_t ld, double* E, hipStream_t s)
{
    const int64_t items = n * ((n + kTermCols - 1) / kTermCols);
    hipLaunchKernelGGL(k_dense_terms, dim3((unsigned)((items + kTermWaves - 1) / kTermWaves)), dim3(kB), 0, s, T, n,
                       ld, E);
    return hipGetLastError();
}

hipError_t launch_dgemm_mfma(const double* A, const double* B, double* E, int64_t ld, int64_t n, int has_e, double tau,
                             const double* tau_row, hipStream_t s)
{
    // the largest tile (128, 64, 32) that gives the chip at least 512 blocks
    const int bm = dense_tile(ld);
    const unsigned t = (unsigned)(ld / bm);
    if (bm == 128)
        hipLaunchKernelGGL(k_dgemm_mfma<128>, dim3(t, t), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau, tau_row);
    else if (bm == 64)
        hipLaunchKernelGGL(k_dgemm_mfma<64>, dim3(t, t), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau, tau_row);
    else
        hipLaunchKernelGGL(k_dgemm_mfma<32>, dim3(t, t), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau, tau_row);
    return hipGetLastError();
}

hipError_t launch_dgemm_ordered(const double* A, const double* B, double* E, int64_t ld, int64_t n, int has_e,
                               double tau, const double* tau_row, hipStream_t s)
{
    // as the matrix-core product, but not below 64 (ld is a multiple of 128):
    // 32 x 32 tiles leave each thread four fma per two shared-memory reads
    const int bt = std::max(64, dense_tile(ld));
    const unsigned t = (unsigned)(ld / bt);
    if (bt == 128)
        hipLaunchKernelGGL(k_dgemm_ordered<128>, dim3(t, t), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau, tau_row);
    else
        hipLaunchKernelGGL(k_dgemm_ordered<64>, dim3(t, t), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau, tau_row);
    return hipGetLastError();
}

hipError_t launch_spmm_rows(const MatView& A, const double* B, double* E, int64_t ld, int64_t n, int has_e, double tau,
                            const double* tau_row, hipStream_t s)
{
    const int64_t chunks = (n + kRowsCols - 1) / kRowsCols;
    hipLaunchKernelGGL(k_spmm_rows, dim3((unsigned)n, (unsigned)chunks), dim3(kB), 0, s, A, B, E, ld, n, has_e, tau,
                       tau_row);
    return hipGetLastError();
}

hipError_t launch_dense_to_slack(const double* C, int64_t ld, const StageArgs& a, hipStream_t s)
{
    const int64_t blocks = (a.n + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(k_dense_to_slack, dim3((unsigned)blocks), dim3(kB), 0, s, C, ld, a);
    return hipGetLastError();
}

}  // namespace fps
