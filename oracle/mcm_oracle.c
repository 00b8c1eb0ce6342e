/*
 * Plain CPU oracle for the matrix-chain-multiplication (MCM) dynamic
 * programming table.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the benchmark's CPU-baseline leg are the only callers.  It shares no
 * code, header or helper with the GPU library.
 *
 * What it computes (Section IV of the paper, "Solving MCM Problem"): the
 * two-dimensional triangular solution table of the MCM problem, filled
 * along the diagonal direction (Fig. 5), where every element is the
 * smaller-operand operator applied over all splits of a binary function of
 * the left and right sub-results (Fig. 6, Eq. (2)).  The paper defers the
 * cost function to the textbook definition of MCM; written out:
 *
 *   matrix t (0-based) has p[t] rows and p[t+1] columns, t = 0..n-1;
 *   m[i][i] = 0;
 *   m[i][j] = min over k in [i, j-1] of
 *             m[i][k] + m[k+1][j] + p[i] * p[k+1] * p[j+1]      (i < j)
 *   s[i][j] = the smallest k attaining that minimum               (i < j)
 *
 * Output contract (shared with the GPU library by specification, not by
 * code): m is n*n int64 row-major and symmetric (m[j][i] = m[i][j], zero
 * diagonal); s is n*n int32 row-major, s[i][j] = split for i < j and -1
 * for i >= j.
 *
 * Arithmetic is exact int64.  The caller-side precondition that makes it
 * exact: every candidate for cell (i, j) is at most (j-i) * pmax^3 (by
 * induction on j-i), so (n-1) * pmax^3 < 2^63 rules out overflow.
 *
 * The only liberty taken: because m is symmetric by contract, the right
 * operand m[k+1][j] is read from its mirror m[j][k+1], so the inner loop
 * walks two rows instead of a row and a column.  The value read is the
 * same defined quantity.  With threads > 1 the cells of one diagonal
 * (which do not depend on each other) are split across OpenMP threads; the
 * arithmetic per cell is unchanged.
 */
#include <stdint.h>
#include <stddef.h>

#define MCM_ORACLE_OK 0
#define MCM_ORACLE_INVALID 1
#define MCM_ORACLE_OVERFLOW 2

/* 1 if (n-1) * pmax^3 < 2^63 for the dims p[0..n], else 0. */
static int oracle_fits_int64(const int32_t *p, int32_t n)
{
    int64_t pmax = 0;
    for (int32_t t = 0; t <= n; ++t)
        if (p[t] > pmax) pmax = p[t];
    unsigned __int128 bound = (unsigned __int128)(uint64_t)pmax * (uint64_t)pmax;
    bound *= (uint64_t)pmax;
    bound *= (uint64_t)(n - 1);
    return bound < ((unsigned __int128)1 << 63);
}

/* Validate p[0..n] for the oracle: n >= 1, all dims >= 1, no overflow. */
int mcm_oracle_validate(const int32_t *p, int32_t n)
{
    if (p == NULL || n < 1) return MCM_ORACLE_INVALID;
    for (int32_t t = 0; t <= n; ++t)
        if (p[t] < 1) return MCM_ORACLE_INVALID;
    if (!oracle_fits_int64(p, n)) return MCM_ORACLE_OVERFLOW;
    return MCM_ORACLE_OK;
}

/*
 * Fill m (n*n int64) and s (n*n int32) for the chain p[0..n].
 * threads <= 1: single thread.  Returns MCM_ORACLE_* codes.
 */
int mcm_oracle_fill(const int32_t *p, int32_t n, int64_t *m, int32_t *s,
                    int32_t threads)
{
    int rc = mcm_oracle_validate(p, n);
    if (rc != MCM_ORACLE_OK) return rc;
    if (m == NULL || s == NULL) return MCM_ORACLE_INVALID;
    const size_t N = (size_t)n;

    /* Base cases: the first n elements of the linearised table (the main
     * diagonal) are preset; s is -1 on and below the diagonal. */
    for (size_t i = 0; i < N; ++i) {
        for (size_t j = 0; j < N; ++j) {
            m[i * N + j] = 0;
            s[i * N + j] = -1;
        }
    }

    /* Diagonal order: every cell of diagonal d needs only diagonals < d. */
    for (int32_t d = 1; d < n; ++d) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads > 1 ? threads : 1) if (threads > 1)
        for (int32_t i = 0; i < n - d; ++i) {
            const int32_t j = i + d;
            const int64_t *row_i = m + (size_t)i * N;   /* m[i][k]           */
            const int64_t *row_j = m + (size_t)j * N;   /* m[j][k+1]=m[k+1][j] */
            const int64_t pij = (int64_t)p[i] * (int64_t)p[j + 1];
            int64_t best = INT64_MAX;
            int32_t arg = -1;
            for (int32_t k = i; k < j; ++k) {
                const int64_t c = row_i[k] + row_j[k + 1] + pij * (int64_t)p[k + 1];
                if (c < best) {          /* strict: the smallest k wins ties */
                    best = c;
                    arg = k;
                }
            }
            m[(size_t)i * N + j] = best;
            m[(size_t)j * N + i] = best;
            s[(size_t)i * N + j] = arg;
        }
    }
    return MCM_ORACLE_OK;
}

/*
 * Check the defining recurrence at selected cells of a complete table
 * (m, s) that someone else produced: for each (i, j) with i < j, recompute
 * min over k of m[i][k] + m[k+1][j] + p[i]p[k+1]p[j+1] and its smallest
 * argmin from the table's own entries, and compare with m[i][j], s[i][j].
 * If this holds at every cell and the diagonal is zero, the table equals
 * the oracle's by induction on j - i; on a sample it is a spot check.
 * cells holds `count` (i, j) pairs.  Returns the number of cells that fail
 * (also counting i >= j pairs as failures); -1 on invalid arguments.
 */
int64_t mcm_oracle_check_cells(const int32_t *p, int32_t n, const int64_t *m,
                               const int32_t *s, const int32_t *cells,
                               int64_t count, int32_t threads)
{
    if (mcm_oracle_validate(p, n) != MCM_ORACLE_OK) return -1;
    if (m == NULL || s == NULL || (cells == NULL && count > 0)) return -1;
    const size_t N = (size_t)n;
    int64_t bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(dynamic, 64) num_threads(threads > 1 ? threads : 1) if (threads > 1)
    for (int64_t c = 0; c < count; ++c) {
        const int32_t i = cells[2 * c], j = cells[2 * c + 1];
        if (i < 0 || j >= n || i >= j) { bad += 1; continue; }
        const int64_t pij = (int64_t)p[i] * (int64_t)p[j + 1];
        int64_t best = INT64_MAX;
        int32_t arg = -1;
        for (int32_t k = i; k < j; ++k) {
            const int64_t v = m[(size_t)i * N + k] + m[(size_t)(k + 1) * N + j] +
                              pij * (int64_t)p[k + 1];
            if (v < best) { best = v; arg = k; }
        }
        if (best != m[(size_t)i * N + j] || arg != s[(size_t)i * N + j]) bad += 1;
    }
    return bad;
}
