/*
 * Oracle (test infrastructure only): the residue product and the exact
 * integer product of Section 3.1 as plain C loops, for sizes that Python
 * loops cannot reach.  Nothing in the product path links this file.
 *
 * oracle_modmatmul: C = (A B) mod p for residue matrices in [0, p), p < 2^26.
 *   Each term is below 2^52, so 2048 terms sum below 2^63 < 2^64: the
 *   unsigned 64-bit running sum of each output is reduced mod p after every
 *   2048 terms and once at the end.  The sum runs over k in increasing order.
 * oracle_exact_matmul: C = A B in int64; the caller guarantees that no
 *   partial sum leaves the int64 range.
 *
 * Rows of C are independent, so they are shared among threads with OpenMP;
 * nothing else is reordered.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define K_CHUNK 2048

void oracle_modmatmul(const uint32_t *A, const uint32_t *B, uint32_t *C,
                      int64_t m, int64_t n, int64_t k, uint32_t p)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        uint64_t *acc = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
        for (int64_t k0 = 0; k0 < k; k0 += K_CHUNK) {
            int64_t k1 = k0 + K_CHUNK < k ? k0 + K_CHUNK : k;
            for (int64_t t = k0; t < k1; ++t) {
                uint64_t a = A[i * k + t];
                const uint32_t *brow = B + t * n;
                for (int64_t j = 0; j < n; ++j)
                    acc[j] += a * (uint64_t)brow[j];
            }
            for (int64_t j = 0; j < n; ++j)
                acc[j] %= p;
        }
        for (int64_t j = 0; j < n; ++j)
            C[i * n + j] = (uint32_t)(acc[j] % p);
        free(acc);
    }
}

void oracle_exact_matmul(const int64_t *A, const int64_t *B, int64_t *C,
                         int64_t m, int64_t n, int64_t k)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        int64_t *acc = C + i * n;
        memset(acc, 0, (size_t)n * sizeof(int64_t));
        for (int64_t t = 0; t < k; ++t) {
            int64_t a = A[i * k + t];
            const int64_t *brow = B + t * n;
            for (int64_t j = 0; j < n; ++j)
                acc[j] += a * brow[j];
        }
    }
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
