/*
 * CPU oracle for C = A*B on CSR matrices.  TEST INFRASTRUCTURE ONLY: the
 * library never links, loads or calls this file; only the test suite, the
 * package smoke check and the benchmark's CPU baseline do.
 *
 * What it computes (Kokkos Kernels paper, section 2.2.1, Eq. (1)):
 *     C(i,:) = sum over j in A(i,:) of A(i,j) * B(j,:)
 * row by row (Gustavson), with the paper's *dense* accumulator (same section:
 * a marker/bit per column for the structure, a scalar array for the values).
 * The two phases of the section are kept as two entry points:
 *   oracle_row_nnz -- symbolic: number of distinct columns in each C row;
 *   oracle_fill    -- numeric: sorted column indices and values of each row.
 * The row pointer is the exclusive prefix sum of the counts (section 2.2.1),
 * taken by the caller in 64-bit arithmetic.
 *
 * Conventions (readings of points the paper leaves open):
 *   - values are FP64; FP32 inputs are widened exactly by the caller;
 *   - each product A(i,j)*B(j,c) is rounded, then added to the accumulator in
 *     the stored order of A's row and then B's row; build with
 *     -ffp-contract=off so no fused multiply-add changes this;
 *   - explicit zeros (cancellation) are kept: the structure is the boolean
 *     product of the two patterns;
 *   - duplicate column entries in A or B rows contribute additively; columns
 *     in input rows need not be sorted;
 *   - columns of each C row are emitted in ascending order;
 *   - alongside each value the oracle returns sum |A(i,j)|*|B(j,c)|, the scale
 *     of the standard inner-product rounding-error bound, so that callers can
 *     compare values componentwise.
 * Rows are independent; OpenMP splits them across host threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Checks that rows [r0, r1) only reference valid columns.  0 on success. */
static int check_rows(int32_t n, int32_t k, const int32_t* rpA, const int32_t* ciA,
                      const int32_t* rpB, const int32_t* ciB, int32_t r0, int32_t r1) {
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(|:bad)
    for (int32_t i = r0; i < r1; ++i) {
        for (int32_t p = rpA[i]; p < rpA[i + 1]; ++p) {
            int32_t j = ciA[p];
            if (j < 0 || j >= n) { bad = 1; continue; }
            for (int32_t q = rpB[j]; q < rpB[j + 1]; ++q)
                if (ciB[q] < 0 || ciB[q] >= k) bad = 1;
        }
    }
    return bad ? -1 : 0;
}

/*
 * Symbolic phase: nnz_out[i - r0] = number of distinct columns of C(i,:),
 * i in [r0, r1).  Returns 0, or -1 on an out-of-range index, -2 on allocation
 * failure.
 */
int oracle_row_nnz(int32_t m, int32_t n, int32_t k,
                   const int32_t* rpA, const int32_t* ciA,
                   const int32_t* rpB, const int32_t* ciB,
                   int32_t r0, int32_t r1, int64_t* nnz_out) {
    (void)m;
    if (check_rows(n, k, rpA, ciA, rpB, ciB, r0, r1)) return -1;
    int fail = 0;
    #pragma omp parallel reduction(|:fail)
    {
        /* marker[c] == i  <=>  column c already seen in row i */
        int32_t* marker = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
        if (!marker) fail = 1;
        else {
            for (int32_t c = 0; c < k; ++c) marker[c] = -1;
            #pragma omp for schedule(dynamic, 64)
            for (int32_t i = r0; i < r1; ++i) {
                int64_t cnt = 0;
                for (int32_t p = rpA[i]; p < rpA[i + 1]; ++p) {
                    int32_t j = ciA[p];
                    for (int32_t q = rpB[j]; q < rpB[j + 1]; ++q) {
                        int32_t c = ciB[q];
                        if (marker[c] != i) { marker[c] = i; ++cnt; }
                    }
                }
                nnz_out[i - r0] = cnt;
            }
            free(marker);
        }
    }
    return fail ? -2 : 0;
}

/*
 * Numeric phase for rows [r0, r1): row i is written at positions
 * off[i - r0] .. off[i - r0 + 1] - 1 of cols / vals / absv (off comes from
 * the exclusive scan of oracle_row_nnz over the same rows).  vA and vB are
 * FP64 copies of the values.  Returns 0, -1 on a bad index, -2 on allocation
 * failure, -3 if a row's count disagrees with off.
 */
int oracle_fill(int32_t m, int32_t n, int32_t k,
                const int32_t* rpA, const int32_t* ciA, const double* vA,
                const int32_t* rpB, const int32_t* ciB, const double* vB,
                int32_t r0, int32_t r1, const int64_t* off,
                int32_t* cols, double* vals, double* absv) {
    (void)m;
    if (check_rows(n, k, rpA, ciA, rpB, ciB, r0, r1)) return -1;
    int fail = 0;
    #pragma omp parallel reduction(|:fail)
    {
        size_t kk = (size_t)(k > 0 ? k : 1);
        int32_t* marker = (int32_t*)malloc(sizeof(int32_t) * kk);
        double* acc = (double*)malloc(sizeof(double) * kk);
        double* mag = (double*)malloc(sizeof(double) * kk);
        int32_t* list = (int32_t*)malloc(sizeof(int32_t) * kk);
        if (!marker || !acc || !mag || !list) fail = 2;
        else {
            for (int32_t c = 0; c < k; ++c) marker[c] = -1;
            #pragma omp for schedule(dynamic, 64)
            for (int32_t i = r0; i < r1; ++i) {
                int64_t cnt = 0;
                for (int32_t p = rpA[i]; p < rpA[i + 1]; ++p) {
                    int32_t j = ciA[p];
                    double a = vA[p];
                    for (int32_t q = rpB[j]; q < rpB[j + 1]; ++q) {
                        int32_t c = ciB[q];
                        double prod = a * vB[q];
                        double pmag = fabs(a) * fabs(vB[q]);
                        if (marker[c] != i) {
                            marker[c] = i; acc[c] = 0.0; mag[c] = 0.0;
                            list[cnt++] = c;
                        }
                        acc[c] = acc[c] + prod;
                        mag[c] = mag[c] + pmag;
                    }
                }
                int64_t base = off[i - r0];
                if (off[i - r0 + 1] - base != cnt) { fail |= 4; continue; }
                qsort(list, (size_t)cnt, sizeof(int32_t), cmp_i32);
                for (int64_t t = 0; t < cnt; ++t) {
                    int32_t c = list[t];
                    cols[base + t] = c;
                    vals[base + t] = acc[c];
                    absv[base + t] = mag[c];
                }
            }
        }
        free(marker); free(acc); free(mag); free(list);
    }
    if (fail & 4) return -3;
    return fail ? -2 : 0;
}

/* Number of host threads OpenMP will use (reported beside CPU timings). */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Host threads later calls use (timing of the oracle with fewer threads). */
void oracle_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
