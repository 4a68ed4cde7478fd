// HIP kernels (gfx950) of the batched layer: many independent instances of
// the filtered PS evaluation are joined into one block-diagonal CSR per
// group (instances that share the schedule and the coefficients), so that
// every stage of the scheme is one launch over all the group's rows.  Rows
// of different instances never meet: a row's terms come from its own block,
// so each instance's result is the one a plan of its own gives, bit for bit.
//
// Kernels here: the join (row pointers, shifted columns, values and the
// per-row threshold), the per-instance sums of per-row counters (the
// autotuner's multiply-add counts), and the extraction of one instance's rows
// from a joined result.
#include "fps_device.h"

namespace fps {
namespace {

constexpr int kB = 256;

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kB - 1) / kB); }

// Instance holding joined row R: the largest i with base[i] <= R
// (base[0] = 0, base[count] = total rows, nondecreasing).
__device__ __forceinline__ int instance_of(const int64_t* __restrict__ base, int count, int64_t R)
{
    int lo = 0, hi = count;  // base[lo] <= R < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= R)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Joined row pointers (rp[R] = nnz_base[i] + row_ptr_i[r]; rp[total] by the
// last row) and per-row thresholds.
__global__ void __launch_bounds__(kB) k_batch_join_rows(const BatchSrc* __restrict__ src,
                                                        const int64_t* __restrict__ base, int count, int64_t total,
                                                        int64_t* rp, double* tau_row)
{
    const int64_t R = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (R >= total) return;
    const int i = instance_of(base, count, R);
    const BatchSrc s = src[i];
    const int64_t r = R - base[i];
    rp[R] = s.nnz_base + s.row_ptr[r];
    if (R == total - 1) rp[total] = s.nnz_base + s.row_ptr[r + 1];
    tau_row[R] = s.tau;
}

// Joined entries: one thread per row copies its entries, columns shifted by
// the instance's first row (the blocks are square and on the diagonal).
__global__ void __launch_bounds__(kB) k_batch_join_entries(const BatchSrc* __restrict__ src,
                                                           const int64_t* __restrict__ base, int count,
                                                           int64_t total, const int64_t* __restrict__ rp, int32_t* col,
                                                           double* val)
{
    const int64_t R = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (R >= total) return;
    const int i = instance_of(base, count, R);
    const BatchSrc s = src[i];
    const int64_t r = R - base[i];
    const int64_t b = s.row_ptr[r], e = s.row_ptr[r + 1];
    const int32_t shift = (int32_t)base[i];
    int64_t o = rp[R];
    for (int64_t p = b; p < e; ++p, ++o) {
        col[o] = s.col[p] + shift;
        val[o] = s.val[p];
    }
}

__global__ void __launch_bounds__(kB) k_batch_instance_sum(const int64_t* __restrict__ acc,
                                                           const int64_t* __restrict__ base, int count, int64_t total,
                                                           unsigned long long* out)
{
    const int64_t R = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (R >= total) return;
    const int64_t v = acc[R];
    if (v != 0) atomicAdd(&out[instance_of(base, count, R)], (unsigned long long)v);
}

// bounds[2i], bounds[2i+1] = first and one-past-last entry of instance i in
// a joined result with row pointers frp.
__global__ void __launch_bounds__(kB) k_batch_bounds(const int64_t* __restrict__ frp, const int64_t* __restrict__ base,
                                                     int count, int64_t* bounds)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= count) return;
    bounds[2 * i] = frp[base[i]];
    bounds[2 * i + 1] = frp[base[i + 1]];
}

// One instance's rows of a joined result: row pointers from 0, columns
// shifted back.
__global__ void __launch_bounds__(kB) k_batch_extract_rp(const int64_t* __restrict__ frp, int64_t row0, int64_t n,
                                                         int64_t* rp)
{
    const int64_t r = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (r > n) return;
    rp[r] = frp[row0 + r] - frp[row0];
}

__global__ void __launch_bounds__(kB) k_batch_extract_col(const int32_t* __restrict__ fcol, int64_t p0, int64_t cnt,
                                                          int32_t shift, int32_t* col)
{
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= cnt) return;
    col[p] = fcol[p0 + p] - shift;
}

}  // namespace

hipError_t launch_batch_join(const BatchSrc* src, const int64_t* base, int count, int64_t total, int64_t* rp,
                             int32_t* col, double* val, double* tau_row, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_join_rows, dim3(grid_for(total)), dim3(kB), 0, s, src, base, count, total, rp, tau_row);
    hipLaunchKernelGGL(k_batch_join_entries, dim3(grid_for(total)), dim3(kB), 0, s, src, base, count, total,
                       (const int64_t*)rp, col, val);
    return hipGetLastError();
}

hipError_t launch_batch_instance_sum(const int64_t* acc, const int64_t* base, int count, int64_t total,
                                     unsigned long long* out, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_instance_sum, dim3(grid_for(total)), dim3(kB), 0, s, acc, base, count, total, out);
    return hipGetLastError();
}

hipError_t launch_batch_bounds(const int64_t* frp, const int64_t* base, int count, int64_t* bounds, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_bounds, dim3(grid_for(count)), dim3(kB), 0, s, frp, base, count, bounds);
    return hipGetLastError();
}

hipError_t launch_batch_extract(const int64_t* frp, const int32_t* fcol, int64_t row0, int64_t n, int64_t p0,
                                int64_t cnt, int32_t shift, int64_t* rp, int32_t* col, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_extract_rp, dim3(grid_for(n + 1)), dim3(kB), 0, s, frp, row0, n, rp);
    if (cnt > 0)
        hipLaunchKernelGGL(k_batch_extract_col, dim3(grid_for(cnt)), dim3(kB), 0, s, fcol, p0, cnt, shift, col);
    return hipGetLastError();
}

}  // namespace fps
