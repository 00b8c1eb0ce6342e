/*
 * Host-only run of the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer: fills of random, tie-heavy and range-limit
 * chains (single and multi-threaded), the cell checker on the oracle's own
 * tables (zero failures) and on planted mistakes (exactly the planted cells
 * fail), and the validation edge cases.  Any out-of-bounds access, overflow
 * or other undefined behaviour aborts with the sanitizer's report.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int mcm_oracle_validate(const int32_t *p, int32_t n);
int mcm_oracle_fill(const int32_t *p, int32_t n, int64_t *m, int32_t *s, int32_t threads);
int64_t mcm_oracle_check_cells(const int32_t *p, int32_t n, const int64_t *m, const int32_t *s,
                               const int32_t *cells, int64_t count, int32_t threads);

static uint64_t rng = 88172645463325252ull;
static uint32_t next_u32(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 11);
}

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                 \
        }                                                             \
    } while (0)

static int run_case(int32_t n, int32_t lo, int32_t hi, int threads)
{
    int32_t *p = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t *m = malloc(sizeof(int64_t) * (size_t)n * (size_t)n);
    int32_t *s = malloc(sizeof(int32_t) * (size_t)n * (size_t)n);
    int32_t *cells = malloc(sizeof(int32_t) * 2 * (size_t)n * (size_t)n);
    for (int32_t t = 0; t <= n; ++t) p[t] = lo + (int32_t)(next_u32() % (uint32_t)(hi - lo + 1));
    CHECK(mcm_oracle_fill(p, n, m, s, threads) == 0);
    int64_t count = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            cells[2 * count] = i;
            cells[2 * count + 1] = j;
            ++count;
        }
    CHECK(mcm_oracle_check_cells(p, n, m, s, cells, count, threads) == 0);
    if (n >= 3) {
        /* planted mistakes: a cost one too high, a split moved */
        m[(size_t)0 * n + (n - 1)] += 1;
        CHECK(mcm_oracle_check_cells(p, n, m, s, cells, count, threads) >= 1);
        m[(size_t)0 * n + (n - 1)] -= 1;
        s[(size_t)0 * n + 2] = (s[(size_t)0 * n + 2] == 0) ? 1 : 0;
        CHECK(mcm_oracle_check_cells(p, n, m, s, cells, count, threads) == 1);
    }
    free(p);
    free(m);
    free(s);
    free(cells);
    return 0;
}

int main(void)
{
    int32_t bad[3] = {3, 0, 4};
    CHECK(mcm_oracle_validate(bad, 2) == 1);
    CHECK(mcm_oracle_validate(NULL, 2) == 1);
    int32_t big[3] = {1 << 21, 1 << 21, 1 << 21};
    CHECK(mcm_oracle_validate(big, 2) == 2);
    int32_t edge[3] = {(1 << 21) - 1, (1 << 21) - 1, (1 << 21) - 1};
    CHECK(mcm_oracle_validate(edge, 2) == 0);
    for (int32_t n = 1; n <= 70; n += 3) {
        if (run_case(n, 1, 1024, 1)) return 1;
        if (run_case(n, 1, 2, 4)) return 1;
    }
    if (run_case(200, 1, 1024, 4)) return 1;
    /* near the int64 limit: (n-1) * pmax^3 just below 2^63 */
    if (run_case(8, (1 << 20) - 30, 1 << 20, 1)) return 1;
    printf("oracle checks passed\n");
    return 0;
}
