// Gradients of L = <dC, A * B_i> on the stored entries of A and B_i:
//   dB(k,l) = sum_i A(i,k) dC(i,l)   ((A^T dC) sampled on pattern(B_i))
//   dA(i,k) = sum_l dC(i,l) B(k,l)   ((dC B^T) sampled on pattern(A))
// Only the products that the forward pass forms are visited: for each stored
// b_kl and each stored a_ik, the entry dC(i,l) (which exists, since that
// product reaches row i of column l).
#include "common.hpp"

namespace spg {

template <typename V>
__global__ void k_fill_zero(V *__restrict__ x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] = V(0);
}

constexpr int kBwdThreads = 256;
// Slots of the per-column table that finds dC(i,l) by row: a column of C
// with at most kBwdTable/2 entries is indexed by an LDS hash of its rows;
// longer ones by a binary search over its row ids.
constexpr int kBwdTable = 4096;

// One workgroup per column l of B_i.  The rows of C(:,l) are entered into an
// open-addressing LDS table (row -> position in C), sized by the column's
// entry count, so setting up a column costs O(nnz(C(:,l))), not O(m).  Each
// entry q of B(:,l) is walked by a team of L lanes: lane t of the team visits
// the terms t, t + L, ... of A(:,k) and the team sums its partial dB values
// in a fixed tree order, so every dB entry is reproducible bit for bit.
template <typename V, int L>
__global__ __launch_bounds__(kBwdThreads) void k_backward(
    const int64_t *__restrict__ Acolptr, const int32_t *__restrict__ Arowidx,
    const V *__restrict__ Avals, const int64_t *__restrict__ Bcolptr,
    const int32_t *__restrict__ Browidx, const V *__restrict__ Bvals,
    const int64_t *__restrict__ Ccolptr, const int32_t *__restrict__ Crow,
    const V *__restrict__ dC, V *__restrict__ dA, V *__restrict__ dB) {
    static_assert(L >= 1 && L <= kWave && (L & (L - 1)) == 0, "team width");
    __shared__ int s_key[kBwdTable];
    __shared__ int s_pos[kBwdTable];
    const int64_t l = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t c0 = Ccolptr[l], c1 = Ccolptr[l + 1];
    const int64_t cn = c1 - c0;
    const bool hashed = cn <= kBwdTable / 2;
    int T = 1;
    if (hashed) {
        while (T < 2 * cn) T <<= 1;
        const int bits = __builtin_ctz(T);
        for (int s = tid; s < T; s += kBwdThreads) s_key[s] = -1;
        __syncthreads();
        for (int64_t e = c0 + tid; e < c1; e += kBwdThreads) {
            const int32_t r = Crow[e];
            uint32_t h = bits ? ((uint32_t)r * 2654435761u) >> (32 - bits) : 0u;
            while (atomicCAS(&s_key[h], -1, r) != -1) h = (h + 1) & (T - 1);
            s_pos[h] = (int)(e - c0);
        }
        __syncthreads();
    }
    const int bits = __builtin_ctz(T);
    // position of row i in C(:,l), or -1 when the column has no such row
    auto find = [&](int32_t i) -> int64_t {
        if (hashed) {
            uint32_t h = bits ? ((uint32_t)i * 2654435761u) >> (32 - bits) : 0u;
            while (true) {
                const int key = s_key[h];
                if (key == i) return c0 + s_pos[h];
                if (key == -1) return -1;
                h = (h + 1) & (T - 1);
            }
        }
        int64_t lo = c0, hi = c1 - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (Crow[mid] < i) lo = mid + 1; else hi = mid;
        }
        return (lo < c1 && Crow[lo] == i) ? lo : -1;
    };
    const int team = tid / L, tl = tid % L;
    constexpr int kTeams = kBwdThreads / L;
    const int64_t q0 = Bcolptr[l], q1 = Bcolptr[l + 1];
    for (int64_t qb = q0; qb < q1; qb += kTeams) {
        const int64_t q = qb + team;
        const bool live = q < q1;  // uniform over the team
        V acc = V(0);
        if (live) {
            const int32_t k = Browidx[q];
            const V bv = Bvals[q];
            const int64_t p1 = Acolptr[k + 1];
            for (int64_t p = Acolptr[k] + tl; p < p1; p += L) {
                const int64_t e = find(Arowidx[p]);
                if (e < 0) continue;  // row not in C's pattern
                const V g = dC[e];
                acc += Avals[p] * g;
                if (dA) atomicAdd(&dA[p], g * bv);
            }
        }
        // fixed-order tree sum over the team (lanes of one wave)
#pragma unroll
        for (int d = L >> 1; d > 0; d >>= 1) acc += __shfl_xor(acc, d, L);
        if (live && tl == 0 && dB) dB[q] = acc;
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
        // team width: about the average column length of A
        const double avg = p.k > 0 ? (double)p.nnzA / (double)p.k : 0.0;
        const dim3 grid((unsigned)p.n), block(kBwdThreads);
#define SPG_BWD(Lw)                                                                         \
    hipLaunchKernelGGL((k_backward<V, Lw>), grid, block, 0, p.stream, p.Acolptr, p.Arowidx, \
                       Avals, p.Bcolptr, p.Browidx, Bvals, Ccolptr, Crow, dC, dA, dB)
        if (avg <= 4.0) SPG_BWD(4);
        else if (avg <= 8.0) SPG_BWD(8);
        else if (avg <= 16.0) SPG_BWD(16);
        else if (avg <= 32.0) SPG_BWD(32);
        else SPG_BWD(64);
#undef SPG_BWD
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
