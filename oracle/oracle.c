/*
 * CPU oracle for the local product of the sparsity-aware 1D SpGEMM
 * (Hong & Buluc, "A sparsity-aware distributed-memory algorithm for
 * sparse-sparse matrix multiplication").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * reference.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline use it; the product path never calls, links or loads it, and it
 * shares no code with the HIP library.
 *
 * Conventions (all arrays are host memory owned by the caller):
 *   CSC matrix: colptr int64[ncols+1], rowidx int32[nnz] (ascending, unique
 *   per column), vals double[nnz].  FP32 inputs are upcast by the caller.
 *   Every function returns 0 on success, -1 on a bad argument and -2 when a
 *   scratch allocation fails.
 *
 * Everything is computed in FP64 with the summation order stated at each
 * function; build with -ffp-contract=off so a*b+c is never fused.  The two
 * product passes (count, fill) hand output columns to OpenMP threads when
 * built with -fopenmp; one thread computes a whole column, so the results do
 * not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/*
 * H_i: dense boolean vector of length k marking the rows of B_i that hold a
 * stored entry (notation table, "H_i"; Alg. 1, the step that stores the
 * nonzero row ids of B_i).
 */
int oracle_rows_of_b(int64_t k, int64_t nnzB, const int32_t *Browidx, uint8_t *H)
{
    if (k < 0 || nnzB < 0 || (nnzB > 0 && !Browidx) || (k > 0 && !H))
        return ORACLE_EINVAL;
    memset(H, 0, (size_t)k);
    for (int64_t q = 0; q < nnzB; ++q) {
        int32_t r = Browidx[q];
        if (r < 0 || r >= k)
            return ORACLE_EINVAL;
        H[r] = 1;
    }
    return ORACLE_OK;
}

/*
 * Block fetching (Alg. 2), applied to every one of the P column partitions of
 * A (Alg. 1 splits A's k columns into P slices; the paper's example in
 * Sec. III-A fetches whole blocks of a slice whenever one of their columns
 * is needed).
 *
 * Reading of the algorithm used here:
 *   - the "ordered non-zero column ids" of partition r are the columns c in
 *     [offsets[r], offsets[r+1]) with at least one stored entry, ascending;
 *   - "split into K groups" cuts that list into consecutive runs of b ids,
 *     the last run possibly shorter, so K_r = ceil(nzc_r / b);
 *   - a group is chosen when any of its columns has H = 1; a chosen group
 *     adds the pair (first column, last column) to R and M grows by one;
 *   - the same rule is applied to every partition, the caller's own included,
 *     unless own_whole names a partition: that partition is local to the
 *     caller (Sec. III-A: only remote blocks are fetched), so all of its
 *     groups are chosen and its nonzero columns enter A~ whole.
 *
 * Outputs:
 *   sel[c]  = 1 when column c lies in a chosen group, else 0 (length k)
 *   map[c]  = index of c among the selected columns in ascending order, or -1
 *   *kt     = number of selected columns
 *   blocks  = the M pairs (first, last), partition-major, group order; the
 *             caller provides room for blocks_cap pairs
 *   *M      = number of chosen groups, *K = total number of groups
 */
int oracle_block_select(int64_t k, const int64_t *Acolptr, const uint8_t *H,
                        int32_t P, const int64_t *offsets, int64_t b, int32_t own_whole,
                        uint8_t *sel, int32_t *map, int64_t *kt,
                        int64_t *blocks, int64_t blocks_cap,
                        int64_t *M, int64_t *K)
{
    if (k < 0 || P < 1 || b < 1 || !Acolptr || !offsets || !kt || !M || !K)
        return ORACLE_EINVAL;
    if (k > 0 && (!H || !sel || !map))
        return ORACLE_EINVAL;
    if (offsets[0] != 0 || offsets[P] != k)
        return ORACLE_EINVAL;
    for (int32_t r = 0; r < P; ++r)
        if (offsets[r + 1] < offsets[r])
            return ORACLE_EINVAL;

    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    if (!ids)
        return ORACLE_ENOMEM;
    memset(sel, 0, (size_t)k);
    int64_t nM = 0, nK = 0;

    for (int32_t r = 0; r < P; ++r) {
        /* the ordered nonzero column ids of this partition */
        int64_t nzc = 0;
        for (int64_t c = offsets[r]; c < offsets[r + 1]; ++c)
            if (Acolptr[c + 1] > Acolptr[c])
                ids[nzc++] = c;
        int64_t groups = (nzc + b - 1) / b;
        nK += groups;
        for (int64_t g = 0; g < groups; ++g) {
            int64_t lo = g * b;
            int64_t hi = lo + b < nzc ? lo + b : nzc;
            int choose = r == own_whole;
            for (int64_t j = lo; j < hi && !choose; ++j) {
                if (H[ids[j]]) {
                    choose = 1;
                    break;
                }
            }
            if (choose) {
                if (nM < blocks_cap && blocks) {
                    blocks[2 * nM] = ids[lo];
                    blocks[2 * nM + 1] = ids[hi - 1];
                }
                nM += 1;
                for (int64_t j = lo; j < hi; ++j)
                    sel[ids[j]] = 1;
            }
        }
    }
    free(ids);

    int64_t count = 0;
    for (int64_t c = 0; c < k; ++c)
        map[c] = sel[c] ? (int32_t)(count++) : -1;
    *kt = count;
    *M = nM;
    *K = nK;
    return ORACLE_OK;
}

/*
 * The compacted matrix A~ of Alg. 1: the selected columns of A, in ascending
 * order, copied whole (row ids and values).  Atcolptr has kt+1 entries; the
 * caller sizes Atrowidx/Atvals with Atcolptr[kt], which this function fills
 * first when Atrowidx is NULL (a sizing call).
 */
int oracle_gather(int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                  const double *Avals, const int32_t *map,
                  int64_t *Atcolptr, int32_t *Atrowidx, double *Atvals)
{
    if (k < 0 || !Acolptr || !Atcolptr || (k > 0 && !map))
        return ORACLE_EINVAL;
    int64_t j = 0, pos = 0;
    Atcolptr[0] = 0;
    for (int64_t c = 0; c < k; ++c) {
        if (map[c] < 0)
            continue;
        if (map[c] != j)
            return ORACLE_EINVAL;
        for (int64_t p = Acolptr[c]; p < Acolptr[c + 1]; ++p) {
            if (Atrowidx) {
                Atrowidx[pos] = Arowidx[p];
                Atvals[pos] = Avals[p];
            }
            ++pos;
        }
        ++j;
        Atcolptr[j] = pos;
    }
    return ORACLE_OK;
}

/*
 * Sparse flops of each output column: the number of products a_ik * b_kj
 * with both entries stored (sparse-flops definition in Sec. III-B),
 * i.e. flop[j] = sum over stored b_kj of nnz(A(:,k)).
 */
int oracle_column_flops(int64_t k, const int64_t *Acolptr, int64_t n,
                        const int64_t *Bcolptr, const int32_t *Browidx,
                        int64_t *flop)
{
    if (k < 0 || n < 0 || !Acolptr || !Bcolptr || (n > 0 && !flop))
        return ORACLE_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        int64_t s = 0;
        for (int64_t q = Bcolptr[j]; q < Bcolptr[j + 1]; ++q) {
            int32_t r = Browidx[q];
            if (r < 0 || r >= k)
                return ORACLE_EINVAL;
            s += Acolptr[r + 1] - Acolptr[r];
        }
        flop[j] = s;
    }
    return ORACLE_OK;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/*
 * Output columns are independent (Sec. III-A computes C column by column),
 * so the two product passes below hand requested columns to OpenMP threads,
 * each with its own dense accumulator.  A column's own arithmetic and its
 * order are the same whatever the thread count.  oracle_set_threads(n)
 * fixes the thread count (n <= 0: OpenMP's default); oracle_threads()
 * returns the count the next pass will use.
 */
static int g_threads = 0;

void oracle_set_threads(int n) { g_threads = n > 0 ? n : 0; }

int oracle_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Number of distinct rows of column j of A*B: the union of A(:,k) over the
 * stored b_kj.  flag (m bytes, all 0 on entry and on return) and list (m
 * ints) are the caller's scratch.  Returns the count, or -1 for a row id of
 * B outside A's columns.
 */
static int64_t count_column(int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                            const int64_t *Bcolptr, const int32_t *Browidx, int64_t j,
                            uint8_t *flag, int32_t *list)
{
    int64_t len = 0;
    for (int64_t q = Bcolptr[j]; q < Bcolptr[j + 1]; ++q) {
        int32_t kk = Browidx[q];
        if (kk < 0 || kk >= k) {
            for (int64_t e = 0; e < len; ++e)
                flag[list[e]] = 0;
            return -1;
        }
        for (int64_t p = Acolptr[kk]; p < Acolptr[kk + 1]; ++p) {
            int32_t i = Arowidx[p];
            if (!flag[i]) {
                flag[i] = 1;
                list[len++] = i;
            }
        }
    }
    for (int64_t e = 0; e < len; ++e)
        flag[list[e]] = 0;
    return len;
}

/*
 * Number of stored entries of each requested column of C = A*B (Sec. III-A,
 * column-by-column formula C(:,j) = sum_k A(:,k) b_kj): the number of
 * distinct row ids in the union of A(:,k) over the stored b_kj.  A row is
 * stored whenever some product reaches it, even if the values cancel.
 *
 * cols lists the requested columns of B (NULL = all n columns, in order);
 * counts[t] receives the count of column cols[t].
 */
int oracle_spgemm_count(int64_t m, int64_t k, const int64_t *Acolptr,
                        const int32_t *Arowidx, int64_t n,
                        const int64_t *Bcolptr, const int32_t *Browidx,
                        int64_t ncols, const int64_t *cols, int64_t *counts)
{
    if (m < 0 || k < 0 || n < 0 || ncols < 0 || !Acolptr || !Bcolptr)
        return ORACLE_EINVAL;
    int rc = ORACLE_OK;
#pragma omp parallel num_threads(oracle_threads())
    {
        uint8_t *flag = (uint8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
        if (!flag || !list) {
#pragma omp atomic write
            rc = ORACLE_ENOMEM;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < ncols; ++t) {
            int bad;
#pragma omp atomic read
            bad = rc;
            if (bad != ORACLE_OK)
                continue;
            int64_t j = cols ? cols[t] : t;
            int64_t len = j < 0 || j >= n ? -1
                          : count_column(k, Acolptr, Arowidx, Bcolptr, Browidx, j, flag, list);
            if (len < 0) {
#pragma omp atomic write
                rc = ORACLE_EINVAL;
                continue;
            }
            counts[t] = len;
        }
        free(flag);
        free(list);
    }
    return rc;
}

/*
 * Values of column j of A*B into out (rows), outval and outabs (may be NULL)
 * at their final places: the dense accumulator spa/spa_abs (m doubles each),
 * flag (m bytes, 0 on entry and on return) and list (m ints) are the
 * caller's scratch.  want is the count the caller sized the column for.
 * Returns 0, or -1 on a bad row id of B or a count that differs from want.
 */
static int fill_column(int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                       const double *Avals, const int64_t *Bcolptr,
                       const int32_t *Browidx, const double *Bvals, int64_t j,
                       int64_t want, int32_t *outrow, double *outval, double *outabs,
                       uint8_t *flag, double *spa, double *spa_abs, int32_t *list)
{
    int64_t len = 0;
    int bad = 0;
    for (int64_t q = Bcolptr[j]; q < Bcolptr[j + 1] && !bad; ++q) {
        int32_t kk = Browidx[q];
        double bv = Bvals[q];
        if (kk < 0 || kk >= k) {
            bad = 1;
            break;
        }
        for (int64_t p = Acolptr[kk]; p < Acolptr[kk + 1]; ++p) {
            int32_t i = Arowidx[p];
            double prod = Avals[p] * bv;
            double mag = (Avals[p] < 0 ? -Avals[p] : Avals[p]) * (bv < 0 ? -bv : bv);
            if (!flag[i]) {
                flag[i] = 1;
                list[len++] = i;
                spa[i] = prod;
                spa_abs[i] = mag;
            } else {
                spa[i] = spa[i] + prod;
                spa_abs[i] = spa_abs[i] + mag;
            }
        }
    }
    if (bad || len != want) {
        for (int64_t e = 0; e < len; ++e)
            flag[list[e]] = 0;
        return -1;
    }
    qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
    for (int64_t e = 0; e < len; ++e) {
        int32_t i = list[e];
        outrow[e] = i;
        outval[e] = spa[i];
        if (outabs)
            outabs[e] = spa_abs[i];
        flag[i] = 0;
    }
    return 0;
}

/*
 * Values of the requested columns of C = A*B by a dense sparse accumulator
 * (Gustavson's column-by-column formula, Sec. III-A).  For each requested
 * column j, for each stored b_kj in ascending k, for each stored a_ik in
 * ascending i: the first product reaching row i sets spa[i] = a_ik*b_kj,
 * later ones add to it.  The touched rows are sorted ascending and written
 * at outptr[t]..outptr[t+1] (outptr from a prefix sum of
 * oracle_spgemm_count).  When outabs is not NULL it receives, in the same
 * slots, sum |a_ik|*|b_kj|, the magnitude used to bound rounding errors.
 */
int oracle_spgemm_fill(int64_t m, int64_t k, const int64_t *Acolptr,
                       const int32_t *Arowidx, const double *Avals, int64_t n,
                       const int64_t *Bcolptr, const int32_t *Browidx,
                       const double *Bvals, int64_t ncols, const int64_t *cols,
                       const int64_t *outptr, int32_t *outrow, double *outval,
                       double *outabs)
{
    if (m < 0 || k < 0 || n < 0 || ncols < 0 || !Acolptr || !Bcolptr || !outptr)
        return ORACLE_EINVAL;
    size_t mm = (size_t)(m > 0 ? m : 1);
    int rc = ORACLE_OK;
#pragma omp parallel num_threads(oracle_threads())
    {
        uint8_t *flag = (uint8_t *)calloc(mm, 1);
        double *spa = (double *)malloc(sizeof(double) * mm);
        double *spa_abs = (double *)malloc(sizeof(double) * mm);
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * mm);
        if (!flag || !spa || !spa_abs || !list) {
#pragma omp atomic write
            rc = ORACLE_ENOMEM;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < ncols; ++t) {
            int bad;
#pragma omp atomic read
            bad = rc;
            if (bad != ORACLE_OK)
                continue;
            int64_t j = cols ? cols[t] : t;
            int64_t o = outptr[t];
            if (j < 0 || j >= n ||
                fill_column(k, Acolptr, Arowidx, Avals, Bcolptr, Browidx, Bvals, j,
                            outptr[t + 1] - o, outrow + o, outval + o,
                            outabs ? outabs + o : NULL, flag, spa, spa_abs, list) != 0) {
#pragma omp atomic write
                rc = ORACLE_EINVAL;
            }
        }
        free(flag);
        free(spa);
        free(spa_abs);
        free(list);
    }
    return rc;
}

/*
 * Gradients of L = <dC, A*B> restricted to the stored patterns:
 *   dA(i,k) = sum_l dC(i,l) * B(k,l)   for every stored (i,k) of A,
 *   dB(k,l) = sum_i A(i,k) * dC(i,l)   for every stored (k,l) of B,
 * i.e. (dC*B^T) masked to pattern(A) and (A^T*dC) masked to pattern(B).
 * dC is given on the pattern of C (Ccolptr/Crowidx, n columns).  For each
 * column l of B, dC(:,l) is scattered into a dense vector; then for each
 * stored b_kl (ascending k) and each stored a_ik (ascending i) the two
 * products are added to dA and dB.  dA (nnz(A)) and dB (nnz(B)) are
 * overwritten.
 */
int oracle_backward(int64_t m, int64_t k, const int64_t *Acolptr,
                    const int32_t *Arowidx, const double *Avals, int64_t n,
                    const int64_t *Bcolptr, const int32_t *Browidx,
                    const double *Bvals, const int64_t *Ccolptr,
                    const int32_t *Crowidx, const double *dCvals, double *dA,
                    double *dB)
{
    if (m < 0 || k < 0 || n < 0 || !Acolptr || !Bcolptr || !Ccolptr)
        return ORACLE_EINVAL;
    size_t mm = (size_t)(m > 0 ? m : 1);
    double *spa = (double *)calloc(mm, sizeof(double));
    if (!spa)
        return ORACLE_ENOMEM;
    for (int64_t p = 0; p < Acolptr[k]; ++p)
        dA[p] = 0.0;
    for (int64_t q = 0; q < Bcolptr[n]; ++q)
        dB[q] = 0.0;
    int rc = ORACLE_OK;
    for (int64_t l = 0; l < n && rc == ORACLE_OK; ++l) {
        for (int64_t e = Ccolptr[l]; e < Ccolptr[l + 1]; ++e)
            spa[Crowidx[e]] = dCvals[e];
        for (int64_t q = Bcolptr[l]; q < Bcolptr[l + 1]; ++q) {
            int32_t kk = Browidx[q];
            if (kk < 0 || kk >= k) {
                rc = ORACLE_EINVAL;
                break;
            }
            double bv = Bvals[q];
            double acc = 0.0;
            for (int64_t p = Acolptr[kk]; p < Acolptr[kk + 1]; ++p) {
                double g = spa[Arowidx[p]];
                dA[p] = dA[p] + g * bv;
                acc = acc + Avals[p] * g;
            }
            dB[q] = acc;
        }
        for (int64_t e = Ccolptr[l]; e < Ccolptr[l + 1]; ++e)
            spa[Crowidx[e]] = 0.0;
    }
    free(spa);
    return rc;
}
