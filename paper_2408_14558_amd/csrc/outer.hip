// The outer-product form of the 1D product (Alg. 3): with the inner
// dimension split into row blocks of B, process r forms the partial product
// A(:, K_r) * B(K_r, :) and the partial results are then summed.  On one GPU
// the two data-movement steps of Alg. 3 become device kernels:
//   - the row block B(K_r, :) with its global row ids (so a plan of
//     A * B(K_r, :) selects exactly the columns K_r of A, as Alg. 1 does);
//   - the partial results stacked side by side, [C_1 ... C_P], and the
//     selector [I; ...; I] whose product with the stack is their sum, so the
//     merge runs through the same Gustavson kernels as every product.
#include <algorithm>

#include "common.hpp"

namespace spg {

constexpr int kOuterThreads = 256;

// First position in rows[lo, hi) whose row is at least r (rows ascending).
__device__ __forceinline__ int64_t lower_row(const int32_t *__restrict__ rows, int64_t lo,
                                             int64_t hi, int64_t r) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rows[mid] < r) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// colptr_out[j + 1] = entries of column j in rows [r0, r1); colptr_out[0] = 0.
__global__ void k_row_block_count(int64_t n, const int64_t *__restrict__ colptr,
                                  const int32_t *__restrict__ rows, int64_t r0, int64_t r1,
                                  int64_t *__restrict__ colptr_out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) colptr_out[0] = 0;
    if (j >= n) return;
    const int64_t lo = colptr[j], hi = colptr[j + 1];
    colptr_out[j + 1] = lower_row(rows, lo, hi, r1) - lower_row(rows, lo, hi, r0);
}

// In-place inclusive scan of x[0, n) by one workgroup, a tile of
// kOuterThreads values at a time with the running total carried over.
__global__ __launch_bounds__(kOuterThreads) void k_scan_one_group(int64_t *__restrict__ x,
                                                                  int64_t n) {
    __shared__ long long s_tmp[kOuterThreads / kWave + 1];
    long long carry = 0;
    for (int64_t base = 0; base < n; base += kOuterThreads) {
        const int64_t i = base + threadIdx.x;
        const long long v = i < n ? x[i] : 0;
        long long total;
        const long long excl = group_excl_scan64<kOuterThreads>(v, s_tmp, &total);
        if (i < n) x[i] = carry + excl + v;
        carry += total;
    }
}

// One wave per column copies the column's entries in rows [r0, r1).
template <typename V>
__global__ __launch_bounds__(kOuterThreads) void k_row_block_fill(
    int64_t n, const int64_t *__restrict__ colptr, const int32_t *__restrict__ rows,
    const V *__restrict__ vals, int64_t r0, const int64_t *__restrict__ colptr_out,
    int32_t *__restrict__ rows_out, V *__restrict__ vals_out) {
    const int64_t j = (int64_t)blockIdx.x * (kOuterThreads / kWave) + threadIdx.x / kWave;
    if (j >= n) return;  // whole wave
    const int64_t src = lower_row(rows, colptr[j], colptr[j + 1], r0);
    const int64_t dst = colptr_out[j], cnt = colptr_out[j + 1] - dst;
    for (int64_t e = lane_id(); e < cnt; e += kWave) {
        rows_out[dst + e] = rows[src + e];
        vals_out[dst + e] = vals[src + e];
    }
}

// Column pointers of part r inside the stack: part r's column j is stack
// column r*n + j, its entries shifted by the entries of the parts before it.
__global__ void k_stack_colptr(int64_t n, const int64_t *__restrict__ colptr, int64_t shift,
                               int64_t *__restrict__ stack_colptr) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) stack_colptr[j] = shift + colptr[j];
}

// The selector S = [I_n; ...; I_n] (P blocks): column j holds a 1 in rows
// j, n + j, ..., (P-1) n + j.
template <typename V>
__global__ void k_selector(int64_t n, int32_t P, int64_t *__restrict__ colptr,
                           int32_t *__restrict__ rows, V *__restrict__ vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n) return;
    colptr[j] = (int64_t)P * j;
    if (j == n) return;
    for (int32_t r = 0; r < P; ++r) {
        rows[(int64_t)P * j + r] = (int32_t)(r * n + j);
        vals[(int64_t)P * j + r] = V(1);
    }
}

__global__ void k_set_i64(int64_t *__restrict__ p, int64_t v) {
    if (threadIdx.x == 0) *p = v;
}

static unsigned blocks_for(int64_t items, int per) {
    return (unsigned)std::max<int64_t>(1, (items + per - 1) / per);
}

}  // namespace spg

using namespace spg;

extern "C" int spgemm_row_block(const spgemm_csc *B, spgemm_dtype dtype, int64_t r0, int64_t r1,
                                int64_t *colptr_out, int32_t *rowidx_out, void *vals_out,
                                void *stream) {
    if (!B || !B->colptr || !colptr_out) return fail(SPGEMM_EINVAL, "B or colptr_out is NULL");
    if (dtype != SPGEMM_F32 && dtype != SPGEMM_F64) return fail(SPGEMM_EINVAL, "bad dtype");
    if (B->ncols < 0 || B->nnz < 0) return fail(SPGEMM_EINVAL, "B has a negative size");
    if (r0 < 0 || r1 < r0 || r1 > B->nrows) return fail(SPGEMM_EINVAL, "need 0 <= r0 <= r1 <= nrows");
    if (B->nnz > 0 && (!B->rowidx || !B->vals || !rowidx_out || !vals_out))
        return fail(SPGEMM_EINVAL, "B's or the output's row ids or values are NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = B->ncols;
    hipLaunchKernelGGL(k_row_block_count, dim3(blocks_for(n, kOuterThreads)),
                       dim3(kOuterThreads), 0, s, n, B->colptr, B->rowidx, r0, r1, colptr_out);
    SPG_LAUNCHED("k_row_block_count");
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_one_group, dim3(1), dim3(kOuterThreads), 0, s, colptr_out + 1,
                           n);
        SPG_LAUNCHED("k_scan_one_group");
        const unsigned g = blocks_for(n, kOuterThreads / kWave);
        if (dtype == SPGEMM_F64)
            hipLaunchKernelGGL(k_row_block_fill<double>, dim3(g), dim3(kOuterThreads), 0, s, n,
                               B->colptr, B->rowidx, (const double *)B->vals, r0, colptr_out,
                               rowidx_out, (double *)vals_out);
        else
            hipLaunchKernelGGL(k_row_block_fill<float>, dim3(g), dim3(kOuterThreads), 0, s, n,
                               B->colptr, B->rowidx, (const float *)B->vals, r0, colptr_out,
                               rowidx_out, (float *)vals_out);
        SPG_LAUNCHED("k_row_block_fill");
    }
    return SPGEMM_OK;
}

extern "C" int spgemm_stack_parts(int32_t P, const spgemm_csc *parts, spgemm_dtype dtype,
                                  int64_t *stack_colptr, int32_t *stack_rowidx, void *stack_vals,
                                  int64_t *sel_colptr, int32_t *sel_rowidx, void *sel_vals,
                                  void *stream) {
    if (P < 1 || !parts) return fail(SPGEMM_EINVAL, "need P >= 1 parts");
    if (dtype != SPGEMM_F32 && dtype != SPGEMM_F64) return fail(SPGEMM_EINVAL, "bad dtype");
    const int64_t m = parts[0].nrows, n = parts[0].ncols;
    if (m < 0 || n < 0) return fail(SPGEMM_EINVAL, "parts have a negative size");
    if ((int64_t)P * n >= (1ll << 31)) return fail(SPGEMM_EINVAL, "P * ncols must be below 2^31");
    if (!stack_colptr || !sel_colptr || (n > 0 && (!sel_rowidx || !sel_vals)))
        return fail(SPGEMM_EINVAL, "an output array is NULL");
    const size_t vs = dtype == SPGEMM_F64 ? sizeof(double) : sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    int64_t shift = 0;
    for (int32_t r = 0; r < P; ++r) {
        const spgemm_csc &c = parts[r];
        if (c.nrows != m || c.ncols != n || c.nnz < 0 || !c.colptr)
            return fail(SPGEMM_EINVAL, "part " + std::to_string(r) + " differs in shape");
        if (c.nnz > 0 && (!c.rowidx || !c.vals || !stack_rowidx || !stack_vals))
            return fail(SPGEMM_EINVAL, "row ids or values of part " + std::to_string(r) + " are NULL");
        if (n > 0) {
            hipLaunchKernelGGL(k_stack_colptr, dim3(blocks_for(n, kOuterThreads)),
                               dim3(kOuterThreads), 0, s, n, c.colptr, shift,
                               stack_colptr + (int64_t)r * n);
            SPG_LAUNCHED("k_stack_colptr");
        }
        if (c.nnz > 0) {
            SPG_HIP(hipMemcpyAsync(stack_rowidx + shift, c.rowidx, sizeof(int32_t) * c.nnz,
                                   hipMemcpyDeviceToDevice, s));
            SPG_HIP(hipMemcpyAsync((char *)stack_vals + shift * vs, c.vals, vs * c.nnz,
                                   hipMemcpyDeviceToDevice, s));
        }
        shift += c.nnz;
    }
    // the stack's last pointer: the total
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, stack_colptr + (int64_t)P * n, shift);
    SPG_LAUNCHED("k_set_i64");
    if (dtype == SPGEMM_F64)
        hipLaunchKernelGGL(k_selector<double>, dim3(blocks_for(n + 1, kOuterThreads)),
                           dim3(kOuterThreads), 0, s, n, P, sel_colptr, sel_rowidx,
                           (double *)sel_vals);
    else
        hipLaunchKernelGGL(k_selector<float>, dim3(blocks_for(n + 1, kOuterThreads)),
                           dim3(kOuterThreads), 0, s, n, P, sel_colptr, sel_rowidx,
                           (float *)sel_vals);
    SPG_LAUNCHED("k_selector");
    return SPGEMM_OK;
}
