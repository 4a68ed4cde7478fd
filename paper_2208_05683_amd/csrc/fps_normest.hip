// HIP kernels (gfx950) of the 1-norm estimator used by the series mode
// (Section 3.2.2, eq. 37): the estimator of Higham and Tisseur with one
// column, applied to A = Z^p through p products with Z (A x) or with Z^T
// (A^T s).  Every reduction is exact or in a fixed order, so the estimate does
// not depend on the launch configuration:
//   - Z x and Z^T x accumulate each output entry over its stored terms in
//     ascending index order, one fused multiply-add each, from +0 (Z^T is
//     built once as a CSR whose rows list the rows of Z in ascending order);
//   - ||y||_1 adds |y_i| in ascending i (one wavefront);
//   - the largest |h_i| and the smallest index attaining it are exact
//     (integer atomics on the bit patterns of nonnegative doubles);
//   - the sign-vector comparison is a flag reduction.
#include "fps_device.h"

#include <climits>

namespace fps {
namespace {

constexpr int kB = 256;

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kB - 1) / kB); }

// ---- transpose (counting sort by column, then rows sorted within each column)

__global__ void __launch_bounds__(kB) k_col_counts(const int32_t* __restrict__ col, int64_t nnz,
                                                   unsigned long long* cnt)
{
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[col[p]], 1ull);
}

// Exclusive scan of cnt[0..n) into rp[0..n] in one block (setup path only):
// thread t scans the contiguous range [t * per, (t + 1) * per).
__global__ void __launch_bounds__(kB) k_scan_counts(const unsigned long long* __restrict__ cnt, int64_t n, int64_t* rp)
{
    __shared__ int64_t part[kB];
    const int64_t per = (n + kB - 1) / kB;
    const int64_t b = min<int64_t>((int64_t)threadIdx.x * per, n), e = min<int64_t>(b + per, n);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += (int64_t)cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < kB; ++i) {
            const int64_t t = part[i];
            part[i] = run;
            run += t;
        }
        rp[n] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t i = b; i < e; ++i) {
        rp[i] = run;
        run += (int64_t)cnt[i];
    }
}

// Entries scattered into their column segments in arrival order.
__global__ void __launch_bounds__(kB) k_scatter_t(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, int64_t n,
                                                  const int64_t* __restrict__ trp, unsigned long long* cursor,
                                                  int32_t* trow, double* tval)
{
    const int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (r >= n) return;
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
        const int32_t c = col[p];
        const int64_t pos = trp[c] + (int64_t)atomicAdd(&cursor[c], 1ull);
        trow[pos] = (int32_t)r;
        tval[pos] = val[p];
    }
}

// Each column segment reordered by row index (row indices within a column are
// distinct, so an entry's position is the number of smaller ones): one
// wavefront per column.
__global__ void __launch_bounds__(kB) k_sort_segments(const int64_t* __restrict__ trp, int64_t n,
                                                      const int32_t* __restrict__ trow_in,
                                                      const double* __restrict__ tval_in, int32_t* trow,
                                                      double* tval)
{
    const int64_t c = ((int64_t)blockIdx.x * kB + threadIdx.x) / kWave;
    const int l = threadIdx.x % kWave;
    if (c >= n) return;
    const int64_t b = trp[c], e = trp[c + 1];
    for (int64_t i = b + l; i < e; i += kWave) {
        const int32_t ri = trow_in[i];
        int64_t rank = 0;
        for (int64_t j = b; j < e; ++j) rank += (trow_in[j] < ri) ? 1 : 0;
        trow[b + rank] = ri;
        tval[b + rank] = tval_in[i];
    }
}

// ---- products, norms, signs, argmax ---------------------------------------------

__global__ void __launch_bounds__(kB) k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                             const double* __restrict__ val, int64_t n, const double* __restrict__ x,
                                             double* y)
{
    const int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (r >= n) return;
    double acc = 0.0;
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) acc = fma(val[p], x[col[p]], acc);
    y[r] = acc;
}

// ||y||_1 = sum_i |y_i| added in ascending index order from +0, by one
// wavefront: kSumBlock values at a time go through shared memory (the next
// block already loading, kSumBlock / 64 per lane, so that a load's latency is
// covered by a whole block of additions), and every lane runs the same chain
// of additions on broadcast reads of them in order; the padding past n adds
// +0, which leaves a sum of nonnegative terms unchanged
constexpr int kSumBlock = 4 * kWave;

__global__ void __launch_bounds__(kWave) k_abs_sum_ordered(const double* __restrict__ y, int64_t n, double* out)
{
    __shared__ double buf[kSumBlock];
    constexpr int kPer = kSumBlock / kWave;
    const int l = threadIdx.x;
    double acc = 0.0;
    double nxt[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) nxt[q] = (q * kWave + l < n) ? fabs(y[q * kWave + l]) : 0.0;
    for (int64_t b = 0; b < n; b += kSumBlock) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) buf[q * kWave + l] = nxt[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t i = b + kSumBlock + q * kWave + l;
            nxt[q] = (i < n) ? fabs(y[i]) : 0.0;
        }
        for (int j0 = 0; j0 < kSumBlock; j0 += kWave) {
            double v[kWave];
#pragma unroll
            for (int j = 0; j < kWave; ++j) v[j] = buf[j0 + j];
#pragma unroll
            for (int j = 0; j < kWave; ++j) acc = acc + v[j];
        }
        __syncthreads();
    }
    if (l == 0) *out = acc;
}

// s = sign(y) with sign(0) = +1; flags[0] (flags[1]) stays 1 iff s equals
// (the negation of) s_old
__global__ void __launch_bounds__(kB) k_sign(const double* __restrict__ y, int64_t n, const double* __restrict__ s_old,
                                             int check, double* s, unsigned int* flags)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    bool diff = false, notneg = false;
    if (i < n) {
        const double v = (y[i] >= 0.0) ? 1.0 : -1.0;
        s[i] = v;
        if (check) {
            diff = v != s_old[i];
            notneg = v != -s_old[i];
        }
    }
    // one atomic per wavefront that saw a difference
    const unsigned long long md = __ballot(diff), mn = __ballot(notneg);
    if ((threadIdx.x % kWave) == 0) {
        if (md) atomicAnd(&flags[0], 0u);
        if (mn) atomicAnd(&flags[1], 0u);
    }
}

// res[0] = bit pattern of max |h_i| (nonnegative doubles order like their
// bit patterns), then res[1] = smallest i attaining it
// (both reduce within the wavefront first: one atomic per wavefront)
__global__ void __launch_bounds__(kB) k_absmax_bits(const double* __restrict__ h, int64_t n, unsigned long long* res)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    unsigned long long v = (i < n) ? (unsigned long long)__double_as_longlong(fabs(h[i])) : 0ull;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    if ((threadIdx.x % kWave) == 0) atomicMax(&res[0], v);
}

__global__ void __launch_bounds__(kB) k_absmax_index(const double* __restrict__ h, int64_t n, unsigned long long* res)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    const bool hit = i < n && (unsigned long long)__double_as_longlong(fabs(h[i])) == res[0];
    const unsigned long long m = __ballot(hit);
    if ((threadIdx.x % kWave) == 0 && m)
        atomicMin(&res[1], (unsigned long long)(i + __builtin_ctzll(m)));
}

__global__ void __launch_bounds__(kB) k_fill_f64(double* x, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_set_one(double* x, int64_t i) { x[i] = 1.0; }

}  // namespace

// ---- launch wrappers -------------------------------------------------------

hipError_t launch_transpose(const int64_t* rp, const int32_t* col, const double* val, int64_t n, int64_t nnz,
                            unsigned long long* cnt, int64_t* trp, int32_t* trow_tmp, double* tval_tmp, int32_t* trow,
                            double* tval, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kB), 0, s, reinterpret_cast<double*>(cnt), n, 0.0);
    if (nnz > 0) hipLaunchKernelGGL(k_col_counts, dim3(grid_for(nnz)), dim3(kB), 0, s, col, nnz, cnt);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kB), 0, s, (const unsigned long long*)cnt, n, trp);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kB), 0, s, reinterpret_cast<double*>(cnt), n, 0.0);
    hipLaunchKernelGGL(k_scatter_t, dim3(grid_for(n)), dim3(kB), 0, s, rp, col, val, n, (const int64_t*)trp, cnt,
                       trow_tmp, tval_tmp);
    hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(n * kWave)), dim3(kB), 0, s, (const int64_t*)trp, n,
                       (const int32_t*)trow_tmp, (const double*)tval_tmp, trow, tval);
    return hipGetLastError();
}

hipError_t launch_spmv(const int64_t* rp, const int32_t* col, const double* val, int64_t n, const double* x, double* y,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(n)), dim3(kB), 0, s, rp, col, val, n, x, y);
    return hipGetLastError();
}

hipError_t launch_abs_sum_ordered(const double* y, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_abs_sum_ordered, dim3(1), dim3(kWave), 0, s, y, n, out);
    return hipGetLastError();
}

hipError_t launch_sign(const double* y, int64_t n, const double* s_old, int check, double* sv, unsigned int* flags,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sign, dim3(grid_for(n)), dim3(kB), 0, s, y, n, s_old, check, sv, flags);
    return hipGetLastError();
}

hipError_t launch_absmax(const double* h, int64_t n, unsigned long long* res, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_absmax_bits, dim3(grid_for(n)), dim3(kB), 0, s, h, n, res);
    hipLaunchKernelGGL(k_absmax_index, dim3(grid_for(n)), dim3(kB), 0, s, h, n, res);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* x, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kB), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_unit_vector(double* x, int64_t n, int64_t i, hipStream_t s)
{
    hipError_t e = launch_fill_f64(x, n, 0.0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, s, x, i);
    return hipGetLastError();
}

}  // namespace fps
