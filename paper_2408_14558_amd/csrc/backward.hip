// Gradients of L = <dC, A * B_i> on the stored entries of A and B_i:
//   dB(k,l) = sum_i A(i,k) dC(i,l)   ((A^T dC) sampled on pattern(B_i))
//   dA(i,k) = sum_l dC(i,l) B(k,l)   ((dC B^T) sampled on pattern(A))
// Only the products that the forward pass forms are visited: for each stored
// b_kl and each stored a_ik, the entry dC(i,l) (which exists, since that
// product reaches row i of column l).  One workgroup per column l of B_i
// indexes dC(:,l) by a bitmap + rank over the rows in LDS.
#include "common.hpp"

namespace spg {

template <typename V>
__global__ void k_fill_zero(V *__restrict__ x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] = V(0);
}

constexpr int kBwdThreads = 256;

template <typename V, bool kBitmap>
__global__ __launch_bounds__(kBwdThreads) void k_backward(
    int64_t m, const int64_t *__restrict__ Acolptr, const int32_t *__restrict__ Arowidx,
    const V *__restrict__ Avals, const int64_t *__restrict__ Bcolptr,
    const int32_t *__restrict__ Browidx, const V *__restrict__ Bvals,
    const int64_t *__restrict__ Ccolptr, const int32_t *__restrict__ Crow,
    const V *__restrict__ dC, V *__restrict__ dA, V *__restrict__ dB) {
    extern __shared__ uint32_t s_bits[];
    __shared__ int s_tmp[kBwdThreads / kWave + 2];
    const int64_t l = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t c0 = Ccolptr[l], c1 = Ccolptr[l + 1];
    const int nw = (int)((m + 31) >> 5);
    int *wpre = reinterpret_cast<int *>(s_bits + (kBitmap ? nw : 0));
    if constexpr (kBitmap) {
        for (int i = tid; i < nw; i += kBwdThreads) s_bits[i] = 0u;
        __syncthreads();
        for (int64_t e = c0 + tid; e < c1; e += kBwdThreads) {
            const int32_t r = Crow[e];
            atomicOr(&s_bits[r >> 5], 1u << (r & 31));
        }
        __syncthreads();
        const int per = (nw + kBwdThreads - 1) / kBwdThreads;
        const int w0 = tid * per, w1 = min(nw, w0 + per);
        int c = 0;
        for (int w = w0; w < w1; ++w) c += __popc(s_bits[w]);
        int total;
        int run = group_excl_scan<kBwdThreads>(c, s_tmp, &total);
        for (int w = w0; w < w1; ++w) {
            wpre[w] = run;
            run += __popc(s_bits[w]);
        }
        __syncthreads();
    }
    const int64_t q1 = Bcolptr[l + 1];
    for (int64_t q = Bcolptr[l] + tid; q < q1; q += kBwdThreads) {
        const int32_t k = Browidx[q];
        const V bv = Bvals[q];
        V acc = V(0);
        const int64_t p1 = Acolptr[k + 1];
        for (int64_t p = Acolptr[k]; p < p1; ++p) {
            const int32_t i = Arowidx[p];
            int64_t e;
            if constexpr (kBitmap) {
                const uint32_t w = s_bits[i >> 5];
                if (!((w >> (i & 31)) & 1u)) continue;  // row not in C's pattern
                e = c0 + wpre[i >> 5] + __popc(w & ((1u << (i & 31)) - 1u));
            } else {
                int64_t lo = c0, hi = c1 - 1;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (Crow[mid] < i) lo = mid + 1; else hi = mid;
                }
                e = lo;
                if (e >= c1 || Crow[e] != i) continue;  // row not in C's pattern
            }
            const V g = dC[e];
            acc += Avals[p] * g;
            if (dA) atomicAdd(&dA[p], g * bv);
        }
        if (dB) dB[q] = acc;
    }
}

template <typename V>
static int backward_t(Plan &p, const int64_t *Ccolptr, const int32_t *Crow, const V *Avals,
                      const V *Bvals, const V *dC, V *dA, V *dB) {
    if (dA && p.nnzA > 0)
        hipLaunchKernelGGL(k_fill_zero<V>, dim3((unsigned)std::min<int64_t>(
                                               (p.nnzA + 255) / 256, 4096)),
                           dim3(256), 0, p.stream, dA, p.nnzA);
    if (p.n > 0) {
        if (p.m <= kMaxDenseRows) {
            const size_t lds = (size_t)((p.m + 31) / 32) * 8;
            hipLaunchKernelGGL((k_backward<V, true>), dim3((unsigned)p.n), dim3(kBwdThreads), lds,
                               p.stream, p.m, p.Acolptr, p.Arowidx, Avals, p.Bcolptr, p.Browidx,
                               Bvals, Ccolptr, Crow, dC, dA, dB);
        } else {
            hipLaunchKernelGGL((k_backward<V, false>), dim3((unsigned)p.n), dim3(kBwdThreads), 0,
                               p.stream, p.m, p.Acolptr, p.Arowidx, Avals, p.Bcolptr, p.Browidx,
                               Bvals, Ccolptr, Crow, dC, dA, dB);
        }
    }
    SPG_HIP(hipGetLastError());
    return SPGEMM_OK;
}

int launch_backward(Plan &p, const int64_t *Ccolptr, const int32_t *Crow, const void *Avals,
                    const void *Bvals, const void *dC, void *dA, void *dB) {
    if (p.dtype == SPGEMM_F64)
        return backward_t<double>(p, Ccolptr, Crow, (const double *)Avals,
                                  (const double *)Bvals, (const double *)dC, (double *)dA,
                                  (double *)dB);
    return backward_t<float>(p, Ccolptr, Crow, (const float *)Avals, (const float *)Bvals,
                             (const float *)dC, (float *)dA, (float *)dB);
}

}  // namespace spg
