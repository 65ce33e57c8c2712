/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure only; run by the CPU test suite).  It calls
 * every oracle function on small pseudo-random CSC matrices, including empty
 * shapes and malformed inputs, and checks the consistency the functions
 * promise each other (counts against the filled column pointers, the gather
 * against the selection).  The sanitizers report any out-of-bounds access,
 * use of freed memory, leak or undefined operation on the way.
 *
 * Exit status 0 when every check holds.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_rows_of_b(int64_t k, int64_t nnzB, const int32_t *Browidx, uint8_t *H);
int oracle_block_select(int64_t k, const int64_t *Acolptr, const uint8_t *H, int32_t P,
                        const int64_t *offsets, int64_t b, int32_t own_whole, uint8_t *sel,
                        int32_t *map, int64_t *kt, int64_t *blocks, int64_t blocks_cap,
                        int64_t *M, int64_t *K);
int oracle_gather(int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                  const double *Avals, const int32_t *map, int64_t *Atcolptr,
                  int32_t *Atrowidx, double *Atvals);
int oracle_column_flops(int64_t k, const int64_t *Acolptr, int64_t n, const int64_t *Bcolptr,
                        const int32_t *Browidx, int64_t *flop);
int oracle_spgemm_count(int64_t m, int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                        int64_t n, const int64_t *Bcolptr, const int32_t *Browidx,
                        int64_t ncols, const int64_t *cols, int64_t *counts);
int oracle_spgemm_fill(int64_t m, int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                       const double *Avals, int64_t n, const int64_t *Bcolptr,
                       const int32_t *Browidx, const double *Bvals, int64_t ncols,
                       const int64_t *cols, const int64_t *outptr, int32_t *outrow,
                       double *outval, double *outabs);
int oracle_backward(int64_t m, int64_t k, const int64_t *Acolptr, const int32_t *Arowidx,
                    const double *Avals, int64_t n, const int64_t *Bcolptr,
                    const int32_t *Browidx, const double *Bvals, const int64_t *Ccolptr,
                    const int32_t *Crowidx, const double *dCvals, double *dA, double *dB);
void oracle_set_threads(int n);

typedef struct {
    int64_t m, n, nnz;
    int64_t *colptr;
    int32_t *rowidx;
    double *vals;
} csc;

static uint64_t g_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void)
{
    /* xorshift64*: a published generator, enough for test shapes */
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1Dull;
}

static csc random_csc(int64_t m, int64_t n, int density_pct)
{
    csc a;
    a.m = m;
    a.n = n;
    a.colptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    a.rowidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m * n));
    a.vals = (double *)malloc(sizeof(double) * (size_t)(m * n));
    int64_t nnz = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            if ((int)(next_u64() % 100) < density_pct) {
                a.rowidx[nnz] = (int32_t)i;
                a.vals[nnz] = (double)(int64_t)(next_u64() % 2001) / 1000.0 - 1.0;
                ++nnz;
            }
        }
        a.colptr[j + 1] = nnz;
    }
    a.nnz = nnz;
    return a;
}

static void free_csc(csc *a)
{
    free(a->colptr);
    free(a->rowidx);
    free(a->vals);
}

static int failures = 0;

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static void one_case(int64_t m, int64_t k, int64_t n, int dA, int dB, int32_t P, int64_t b)
{
    csc A = random_csc(m, k, dA);
    csc B = random_csc(k, n, dB);
    uint8_t *H = (uint8_t *)malloc((size_t)k);
    CHECK(oracle_rows_of_b(k, B.nnz, B.rowidx, H) == 0);

    int64_t *offs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P + 1));
    for (int32_t r = 0; r <= P; ++r)
        offs[r] = k * r / P;
    uint8_t *sel = (uint8_t *)malloc((size_t)k);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    int64_t cap = k + P;
    int64_t *blocks = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * cap));
    int64_t kt = -1, M = -1, K = -1;
    CHECK(oracle_block_select(k, A.colptr, H, P, offs, b, -1, sel, map, &kt, blocks, cap, &M,
                              &K) == 0);
    CHECK(M <= K && kt <= k);
    int64_t *atc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(kt + 1));
    CHECK(oracle_gather(k, A.colptr, A.rowidx, A.vals, map, atc, NULL, NULL) == 0);
    int32_t *atr = (int32_t *)malloc(sizeof(int32_t) * (size_t)atc[kt]);
    double *atv = (double *)malloc(sizeof(double) * (size_t)atc[kt]);
    CHECK(oracle_gather(k, A.colptr, A.rowidx, A.vals, map, atc, atr, atv) == 0);

    int64_t *flop = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    CHECK(oracle_column_flops(k, A.colptr, n, B.colptr, B.rowidx, flop) == 0);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    CHECK(oracle_spgemm_count(m, k, A.colptr, A.rowidx, n, B.colptr, B.rowidx, n, NULL, cnt) ==
          0);
    int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) {
        CHECK(cnt[j] <= flop[j] && cnt[j] <= m);
        cp[j + 1] = cp[j] + cnt[j];
    }
    int32_t *cr = (int32_t *)malloc(sizeof(int32_t) * (size_t)cp[n]);
    double *cv = (double *)malloc(sizeof(double) * (size_t)cp[n]);
    double *ca = (double *)malloc(sizeof(double) * (size_t)cp[n]);
    CHECK(oracle_spgemm_fill(m, k, A.colptr, A.rowidx, A.vals, n, B.colptr, B.rowidx, B.vals, n,
                             NULL, cp, cr, cv, ca) == 0);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t e = cp[j] + 1; e < cp[j + 1]; ++e)
            CHECK(cr[e - 1] < cr[e]);
    /* a wrong column size is reported, not written past */
    if (n > 0 && cnt[0] > 0) {
        int64_t *bad = (int64_t *)malloc(sizeof(int64_t) * 2);
        bad[0] = 0;
        bad[1] = cnt[0] - 1;
        int64_t col0 = 0;
        CHECK(oracle_spgemm_fill(m, k, A.colptr, A.rowidx, A.vals, n, B.colptr, B.rowidx, B.vals,
                                 1, &col0, bad, cr, cv, NULL) != 0);
        free(bad);
    }
    double *dC = (double *)malloc(sizeof(double) * (size_t)cp[n]);
    for (int64_t e = 0; e < cp[n]; ++e)
        dC[e] = (double)(e % 7) - 3.0;
    double *gA = (double *)malloc(sizeof(double) * (size_t)A.nnz);
    double *gB = (double *)malloc(sizeof(double) * (size_t)B.nnz);
    CHECK(oracle_backward(m, k, A.colptr, A.rowidx, A.vals, n, B.colptr, B.rowidx, B.vals, cp,
                          cr, dC, gA, gB) == 0);

    free(dC);
    free(gA);
    free(gB);
    free(cr);
    free(cv);
    free(ca);
    free(cp);
    free(cnt);
    free(flop);
    free(atc);
    free(atr);
    free(atv);
    free(blocks);
    free(map);
    free(sel);
    free(offs);
    free(H);
    free_csc(&A);
    free_csc(&B);
}

int main(void)
{
    static const int threads[2] = {1, 4};
    for (int t = 0; t < 2; ++t) {
        oracle_set_threads(threads[t]);
        one_case(0, 0, 0, 50, 50, 1, 1);
        one_case(5, 0, 3, 50, 50, 1, 2);
        one_case(0, 4, 3, 50, 50, 2, 1);
        one_case(7, 6, 0, 50, 50, 3, 2);
        one_case(30, 40, 25, 10, 15, 4, 3);
        one_case(64, 64, 64, 30, 5, 1, 64);
        one_case(100, 37, 50, 3, 40, 5, 1);
        one_case(1, 1, 1, 100, 100, 1, 1);
    }
    /* malformed input: a row id of B outside A's columns */
    {
        int64_t Acp[2] = {0, 1}, Bcp[2] = {0, 1}, cnt[1];
        int32_t Ar[1] = {0}, Br[1] = {5};
        CHECK(oracle_spgemm_count(1, 1, Acp, Ar, 1, Bcp, Br, 1, NULL, cnt) != 0);
        uint8_t H[1];
        CHECK(oracle_rows_of_b(1, 1, Br, H) != 0);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle checks passed\n");
    return 0;
}
