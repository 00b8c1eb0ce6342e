/*
 * mcm.h -- C ABI of the gfx950 matrix-chain-multiplication DP solver.
 *
 * The operation (Section IV of the paper, "Solving MCM Problem"; the paper
 * takes the cost function from the textbook MCM definition): for a chain of
 * n matrices where matrix t (0-based) has p[t] rows and p[t+1] columns,
 * fill the triangular solution table along the diagonal direction (Fig. 5),
 * each element being the minimum over its splits of a function of the left
 * and right sub-results (Fig. 6, Eq. (2)):
 *
 *   m[i][i] = 0
 *   m[i][j] = min_{i <= k < j} m[i][k] + m[k+1][j] + p[i]*p[k+1]*p[j+1]
 *   s[i][j] = the smallest k attaining the minimum              (i < j)
 *
 * Output contract (every byte of both buffers is written):
 *   m_out: int64, n*n, row-major, symmetric: m_out[i*n+j] = m_out[j*n+i] =
 *          the optimal cost of matrices min(i,j)..max(i,j); zero diagonal.
 *   s_out: int32, n*n, row-major: s_out[i*n+j] = 0-based split k (the
 *          product is (A_i..A_k)(A_k+1..A_j)) for i < j, and -1 for i >= j.
 * Results are exact integers and deterministic; every algorithm below
 * returns the same bytes.
 *
 * Preconditions checked on the host before anything is enqueued (on error
 * nothing is enqueued and the output buffers are not touched):
 *   n >= 1, every p[t] >= 1, and (n-1) * max(p)^3 < 2^63 (every candidate
 *   cost of cell (i, j) is at most (j-i) * max(p)^3, so int64 is exact).
 *
 * Threading and streams: calls are thread-safe.  Work is enqueued on
 * `stream` (0 = the null stream) and the call returns without waiting for
 * it; the caller synchronises the stream before reading the outputs.  The
 * library reads the host array p before returning, so the caller may reuse
 * it immediately.  Workspace is allocated stream-ordered on `stream` and
 * released on it.  Outputs of concurrent calls must not alias.
 *
 * Errors: MCM_ERR_INVALID_ARG / MCM_ERR_OVERFLOW for bad inputs (synchronous,
 * nothing enqueued); MCM_ERR_NO_MEMORY when workspace allocation fails;
 * MCM_ERR_DEVICE when the HIP runtime reports an error while enqueueing
 * (including errors left by earlier asynchronous work).
 */
#ifndef MCM_H_
#define MCM_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mcm_status {
    MCM_OK = 0,
    MCM_ERR_INVALID_ARG = 1,
    MCM_ERR_OVERFLOW = 2,
    MCM_ERR_NO_MEMORY = 3,
    MCM_ERR_DEVICE = 4,
    MCM_ERR_UNSUPPORTED = 5
} mcm_status;

/*
 * Kernel paths.  All produce identical bytes; they differ in speed and in
 * the inputs they accept.
 *   MCM_ALGO_AUTO       pick the fastest path for the input (the tiled path).
 *   MCM_ALGO_WAVEFRONT  one launch per diagonal of the table; every cell of
 *                       a diagonal is independent (Fig. 5 order), its splits
 *                       are scanned by a group of lanes and reduced in
 *                       registers.  int64 arithmetic; accepts every valid
 *                       input.
 *   MCM_ALGO_TILED      T x T tiles of the table in tile-diagonal order;
 *                       operand panels staged through LDS and reused across
 *                       a register microtile; split range spread over
 *                       workgroups; a per-tile closure pass in LDS.  When
 *                       (n-1) * max(p)^3 < 2^46, exact integers carried in
 *                       fp64 keys (cost * 2^kb + local split: one fma, add
 *                       and min per split); beyond that, up to the int64
 *                       limit, the same schedule with the split carried
 *                       beside the cost (the bulk in exact fp64 while
 *                       (n-1) * max(p)^3 < 2^53, the closure on int64 keys
 *                       while it is < 2^54, int64 pairs above).  Accepts
 *                       every valid input.
 *   MCM_ALGO_PIPELINE   the paper's pipeline (Section IV-B, Fig. 8): the
 *                       table linearised in diagonal order, thread j folding
 *                       split j of an element one step after thread j-1, a
 *                       barrier per step, in one workgroup; each element
 *                       starts once its operands are final (a stall where
 *                       the printed schedule would read too early).  An
 *                       ablation, far slower than the others; int64;
 *                       n <= 1025 (else MCM_ERR_UNSUPPORTED); never chosen
 *                       by AUTO.
 */
typedef enum mcm_algo {
    MCM_ALGO_AUTO = 0,
    MCM_ALGO_WAVEFRONT = 1,
    MCM_ALGO_TILED = 2,
    MCM_ALGO_PIPELINE = 3
} mcm_algo;

/* Static, NUL-terminated description of a status code (never NULL). */
const char *mcm_status_string(int32_t status);

/* ABI version: major * 10000 + minor * 100 + patch. */
int32_t mcm_version(void);

/*
 * Host-only validation of a chain (no device call): MCM_OK,
 * MCM_ERR_INVALID_ARG (p == NULL, n < 1, or some p[t] < 1) or
 * MCM_ERR_OVERFLOW ((n-1) * max(p)^3 >= 2^63).  p: host, n+1 entries.
 */
mcm_status mcm_check_chain(const int32_t *p, int32_t n);

/*
 * The algorithm MCM_ALGO_AUTO would use for this chain (host only), or a
 * negative status code (-MCM_ERR_*) if the chain is invalid.
 */
int32_t mcm_select_algo(const int32_t *p, int32_t n);

/*
 * Fill m_out and s_out for one chain (the operation above).
 *   p      host pointer, n+1 dimensions (read before return).
 *   n      number of matrices, >= 1.
 *   m_out  device pointer, n*n int64, 8-byte aligned, caller-owned.
 *   s_out  device pointer, n*n int32, 4-byte aligned, caller-owned.
 *   stream HIP stream, or 0.
 * Equivalent to mcm_solve_algo(..., MCM_ALGO_AUTO, stream).
 */
mcm_status mcm_solve(const int32_t *p, int32_t n, int64_t *m_out, int32_t *s_out,
                     hipStream_t stream);

/* mcm_solve with an explicit kernel path (mcm_algo).  MCM_ERR_UNSUPPORTED
 * if that path does not accept the input; MCM_ERR_INVALID_ARG for an
 * unknown algo. */
mcm_status mcm_solve_algo(const int32_t *p, int32_t n, int64_t *m_out, int32_t *s_out,
                          int32_t algo, hipStream_t stream);

/*
 * mcm_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * call allocates nothing (no hipMalloc / hipFree / pinned host memory, no
 * second stream or events): every buffer beyond p, m_out and s_out lives
 * in one fixed device array of MCM_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends.  Same arguments,
 * output contract and validation as mcm_solve (MCM_ALGO_TILED, its
 * schedule run on `stream` alone); the dims reach the device as kernel
 * arguments, so p may be reused at once.
 *   n > MCM_NOALLOC_MAX_N, or a chain whose tables and partial minima do
 *   not fit the array (none up to that n), returns MCM_ERR_UNSUPPORTED
 *   before anything is enqueued.
 * Every call on one device shares that device's array, which keeps the
 * last call's contents (nothing in it needs clearing: each call writes what
 * it reads).  Calls that overlap on one device -- on different streams, or
 * from different threads without ordering -- race on the array and must
 * not be issued; calls ordered on one stream are safe.
 */
#define MCM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define MCM_NOALLOC_MAX_N 8192
mcm_status mcm_solve_noalloc(const int32_t *p, int32_t n, int64_t *m_out, int32_t *s_out,
                             hipStream_t stream);

/*
 * Many independent chains in one call.  All chains advance together, one
 * tile-diagonal per iteration, each kernel launch serving every chain that
 * is still active, so a batch of thousands of small chains costs a few
 * dozen launches instead of thousands.  Chains beyond the fp64 keys' exact
 * range run the tiled path's int64 kernels, after the others.
 *   count   number of chains (>= 0; 0 is a no-op).
 *   n       host, count entries: matrices of chain b (>= 1).
 *   p_off   host, count entries: chain b's dims are p_all[p_off[b] ..
 *           p_off[b] + n[b]] (offsets may overlap; >= 0).
 *   p_all   host, dims of all chains (read before return).
 *   tab_off host, count entries: chain b's m table is m_all + tab_off[b]
 *           and its s table s_all + tab_off[b], n[b]*n[b] elements each,
 *           row-major, same contract as mcm_solve; tables of different
 *           chains must not overlap (checked: MCM_ERR_INVALID_ARG).
 *   m_all, s_all  device buffers (int64 / int32), caller-owned.
 * Every chain is validated before anything is enqueued; the first failure
 * is returned and nothing runs.
 */
mcm_status mcm_solve_batched(int32_t count, const int32_t *n, const int64_t *p_off,
                             const int32_t *p_all, const int64_t *tab_off, int64_t *m_all,
                             int32_t *s_all, hipStream_t stream);

/*
 * Reusable batched plan: the schedule of mcm_solve_batched (every chain's
 * tile-diagonals advanced together, Section IV-A's diagonal order per
 * chain) built once for a fixed batch shape, its launch tables kept in
 * device memory, then solved for any dims that respect the shape.
 *   mcm_plan_create   count, n, p_off and tab_off as in mcm_solve_batched
 *                     (host, read before return); max_dim >= 1 bounds every
 *                     dimension the plan will be solved with (the tiled
 *                     path's exact key width is sized for it, so a chain
 *                     whose (n-1) * max_dim^3 exceeds that range takes the
 *                     int64 tiled kernels).  Validates the shape (INVALID_ARG,
 *                     OVERFLOW as mcm_check_chain with every dim = max_dim)
 *                     before any HIP call, then allocates and copies the
 *                     tables synchronously on the current device.  *out
 *                     receives a handle owned by the caller.
 *   mcm_plan_solve    enqueues one batched solve on `stream` (current device
 *                     = the plan's): p_all (host) holds every chain's dims at
 *                     its p_off; m_all / s_all (device, caller-owned) receive
 *                     the tables at tab_off, same contract as
 *                     mcm_solve_batched.  A dim outside [1, max_dim] returns
 *                     MCM_ERR_INVALID_ARG before anything is enqueued.  The
 *                     plan is read only: solves of one plan may run on
 *                     several streams at once with distinct outputs.
 *   mcm_plan_autotune times every configuration the plan can run on the
 *                     given inputs and keeps the fastest for later solves.
 *                     Configurations: 64-edge tiles with paired closures
 *                     (two per compute unit) for launches above each of four
 *                     tile-count thresholds, and, when every tiled chain has
 *                     n <= 1024, 32-edge tiles (half the closure splits per
 *                     cell, 63 closure steps per tile).  Each runs once
 *                     untimed, then three times timed with events on
 *                     `stream`; its fastest run counts.  The choice is also
 *                     stored in a per-process tuning cache under the plan's
 *                     bucket (device architecture, ceil(log2) of its largest
 *                     tiled chain and of its tiled-chain count): plans
 *                     created later for the same bucket, and
 *                     mcm_solve_batched calls whose batch falls in it, start
 *                     from it.  Writes m_all / s_all as a solve does and
 *                     synchronises `stream`.  *choice (may be NULL) receives
 *                     the index of the chosen configuration in
 *                     mcm_plan_candidates' list (-1 if the plan has none).
 *                     Must not run concurrently with solves of the same plan.
 *   mcm_plan_config   the configuration solves use: tile edge (64 or 32),
 *                     the paired-closure threshold in tiles, and its source
 *                     (MCM_PLAN_DEFAULT: 64-edge tiles, threshold = the CU
 *                     count; MCM_PLAN_CACHED: the tuning cache;
 *                     MCM_PLAN_TUNED: this plan's autotune).  Any output
 *                     pointer may be NULL.
 *   mcm_plan_set_config  pins the configuration later solves use (tile
 *                     edge 64 or 32, threshold >= 0, 0 meaning the CU
 *                     count), e.g. one tuned elsewhere; MCM_ERR_UNSUPPORTED
 *                     if the plan has no schedule for that edge (32 needs
 *                     every tiled chain n <= 1024), MCM_ERR_INVALID_ARG for
 *                     another edge or a negative threshold.  Its source
 *                     becomes MCM_PLAN_TUNED, and the tuning cache keeps
 *                     it for the plan's bucket as an autotune would.  Must
 *                     not run concurrently with solves of the same plan.
 *   mcm_plan_candidates  the configurations the plan can run, in autotune
 *                     order: up to `cap` entries of tile edge, threshold (0:
 *                     the CU count) and the last autotune's time in ms (-1
 *                     if never timed); *count receives the full number.
 *   mcm_plan_graph_create  records the plan's whole solve -- the widening of
 *                     the dims and every launch of every tile-diagonal on both
 *                     streams, in the configuration in use at the call --
 *                     into a HIP graph by stream capture on `stream` (not the
 *                     null stream), for the fixed outputs m_all / s_all
 *                     (device, as in mcm_plan_solve).  The plan then owns the
 *                     graph, a second stream for it and the device buffers
 *                     it reads (dims, their fp64 copies, partial minima); an
 *                     earlier graph of the plan is released.  Cross-stream
 *                     edges are events.  Nothing runs on the device.
 *   mcm_plan_graph_solve  one solve by replay: copies p_all (host, checked
 *                     against max_dim as in mcm_plan_solve) to the plan's
 *                     dims buffer on `stream` and launches the graph there;
 *                     the tables land in the m_all / s_all the graph was
 *                     recorded for.  MCM_ERR_INVALID_ARG without a graph.
 *                     Replays of one plan must be ordered on one stream (they
 *                     share its buffers).
 *   mcm_plan_destroy  frees the plan (its device tables with hipFree, so
 *                     after the device has finished with them); NULL is
 *                     ignored.
 */
enum { MCM_PLAN_DEFAULT = 0, MCM_PLAN_CACHED = 1, MCM_PLAN_TUNED = 2 };
typedef struct mcm_plan mcm_plan;
mcm_status mcm_plan_create(int32_t count, const int32_t *n, const int64_t *p_off,
                           const int64_t *tab_off, int32_t max_dim, mcm_plan **out);
mcm_status mcm_plan_solve(const mcm_plan *plan, const int32_t *p_all, int64_t *m_all,
                          int32_t *s_all, hipStream_t stream);
mcm_status mcm_plan_autotune(mcm_plan *plan, const int32_t *p_all, int64_t *m_all,
                             int32_t *s_all, hipStream_t stream, int32_t *choice);
mcm_status mcm_plan_config(const mcm_plan *plan, int32_t *tile_edge, int32_t *pair_min_blocks,
                           int32_t *source);
mcm_status mcm_plan_set_config(mcm_plan *plan, int32_t tile_edge, int32_t pair_min_blocks);
mcm_status mcm_plan_candidates(const mcm_plan *plan, int32_t cap, int32_t *tile_edge,
                               int32_t *pair_min_blocks, float *ms, int32_t *count);
mcm_status mcm_plan_graph_create(mcm_plan *plan, int64_t *m_all, int32_t *s_all,
                                 hipStream_t stream);
mcm_status mcm_plan_graph_solve(const mcm_plan *plan, const int32_t *p_all, hipStream_t stream);
void mcm_plan_destroy(mcm_plan *plan);

/*
 * Device-resident chain: validated once, dimensions copied to device
 * memory, then solved any number of times without touching the host p.
 *   mcm_chain_create  validates p (host, n+1 entries, read before return)
 *                     and enqueues its upload on `stream`; *out receives an
 *                     opaque handle owned by the caller.  Same status codes
 *                     as mcm_check_chain, plus MCM_ERR_NO_MEMORY /
 *                     MCM_ERR_DEVICE.
 *   mcm_chain_solve   mcm_solve_algo on a created chain (m_out and s_out as
 *                     in mcm_solve).  `stream` must be the creation stream or
 *                     one ordered after it.
 *   mcm_chain_n       number of matrices of the chain (0 for NULL).
 *   mcm_chain_destroy releases the handle; its device memory is freed
 *                     stream-ordered on `stream`, after work already
 *                     enqueued there.  NULL is ignored.
 */
typedef struct mcm_chain mcm_chain;
mcm_status mcm_chain_create(const int32_t *p, int32_t n, hipStream_t stream, mcm_chain **out);
mcm_status mcm_chain_solve(const mcm_chain *chain, int32_t algo, int64_t *m_out, int32_t *s_out,
                           hipStream_t stream);
int32_t mcm_chain_n(const mcm_chain *chain);
void mcm_chain_destroy(mcm_chain *chain, hipStream_t stream);

/*
 * Optimal order read back from a split table.  Section IV of the paper
 * takes the MCM problem from the textbook formulation it cites, where the
 * optimal product order follows from s by recursion: matrices i..j are
 * multiplied as (i..s[i][j]) times (s[i][j]+1..j).  The n-1 products of the
 * tree are named by their split k (the product that joins matrix k to
 * matrix k+1); for each, the call reports the matrices it spans.
 *
 *   mcm_parens_length  characters of the parenthesized text of n matrices
 *                      (any order has the same length): 2(n-1) for the
 *                      parentheses plus, per matrix t, "A" and the decimal
 *                      digits of t.  -1 for n < 1.  Host only.
 *
 *   mcm_parenthesize   one chain.
 *     p      host, n+1 dims (read before return); required when cost is
 *            given (validated as in mcm_check_chain), else may be NULL.
 *     n      number of matrices, >= 1.
 *     s      device, n*n int32 split table, row-major, as written by
 *            mcm_solve (only s[i][j], i < j, on the tree's cells is read).
 *     lo, hi device, n-1 int32 each, 4-byte aligned, or both NULL: product
 *            k multiplies (A_lo[k] .. A_k) by (A_k+1 .. A_hi[k]).
 *     cost   device, one int64, or NULL: the scalar multiplications of the
 *            tree, sum over k of p[lo[k]] * p[k+1] * p[hi[k]+1]; equal to
 *            m[0][n-1] when s is the table mcm_solve wrote for p.
 *     text   device, mcm_parens_length(n)+1 bytes, or NULL: the fully
 *            parenthesized product, matrices written A0, A1, ... (0-based),
 *            e.g. "((A0A1)A2)", NUL-terminated; "A0" for n = 1.
 *   A table entry on the tree's path that is not a split of its cell
 *   (s[i][j] outside [i, j-1]) is not followed: lo/hi of the products below
 *   it stay -1, cost is -1 and text is the empty string.  Work is enqueued
 *   on `stream` like mcm_solve; workspace is stream-ordered.
 *
 *   mcm_parenthesize_batched  many chains, one workgroup each, one launch.
 *     count     chains (>= 0; 0 is a no-op).
 *     n         host, count entries (>= 1).
 *     tab_off   host: chain b's split table is s_all + tab_off[b] (n*n).
 *     node_off  host: chain b's products are lo_all/hi_all + node_off[b]
 *               (n[b]-1 entries each; ranges of different chains must not
 *               overlap: checked, MCM_ERR_INVALID_ARG).
 *     cost_all  device, count int64, or NULL: per-chain tree cost, needing
 *               p_off/p_all (host, as in mcm_solve_batched).
 *   Same invalid-table behaviour per chain.  All chains are validated
 *   before anything is enqueued.
 * Errors: MCM_ERR_INVALID_ARG (bad sizes, offsets, alignment, one of lo/hi
 * NULL, cost without p), MCM_ERR_OVERFLOW (from validating p),
 * MCM_ERR_NO_MEMORY, MCM_ERR_DEVICE.
 */
int64_t mcm_parens_length(int32_t n);
mcm_status mcm_parenthesize(const int32_t *p, int32_t n, const int32_t *s, int32_t *lo,
                            int32_t *hi, int64_t *cost, char *text, hipStream_t stream);
mcm_status mcm_parenthesize_batched(int32_t count, const int32_t *n, const int64_t *p_off,
                                    const int32_t *p_all, const int64_t *tab_off,
                                    const int32_t *s_all, const int64_t *node_off,
                                    int32_t *lo_all, int32_t *hi_all, int64_t *cost_all,
                                    hipStream_t stream);

/*
 * The simplified DP problem (S-DP) of Section II-A, Definition 1: a
 * one-dimensional table ST[0..n-1], offsets a_1 > a_2 > ... > a_k > 0 and a
 * semigroup operator (x); ST[0..a_1-1] are preset and, Eq. (1),
 *
 *   ST[i] = ST[i - a_1] (x) ST[i - a_2] (x) ... (x) ST[i - a_k],   a_1 <= i < n.
 *
 *   a    host, k offsets, strictly decreasing, a[k-1] >= 1, a[0] <= n (read
 *        before return).
 *   op   MCM_SDP_MIN (the operator of the paper's Table I), MCM_SDP_MAX or
 *        MCM_SDP_ADD (int32 addition modulo 2^32).
 *   st   device, n int32, 4-byte aligned, caller-owned: st[0..a[0]-1] hold
 *        the preset values on entry; the call writes st[a[0]..n-1] and
 *        nothing else.  Results are exact and deterministic.
 * Work is enqueued on `stream`; workspace (n int32 plus the offset tables)
 * is stream-ordered.  MCM_ERR_INVALID_ARG for bad sizes, offsets, op or
 * alignment (nothing enqueued); MCM_ERR_NO_MEMORY; MCM_ERR_DEVICE.
 */
typedef enum mcm_sdp_op { MCM_SDP_MIN = 0, MCM_SDP_MAX = 1, MCM_SDP_ADD = 2 } mcm_sdp_op;
mcm_status mcm_sdp_solve(const int32_t *a, int32_t k, int32_t op, int32_t *st, int32_t n,
                         hipStream_t stream);

/*
 * Optimal binary search tree: an interval DP with the split shape of MCM,
 * from the textbook the paper takes MCM from, for the paper's closing aim
 * (end of Section IV) of carrying its technique to more general DP
 * problems.  Keys k_1 < ... < k_n with search weights p_1..p_n and gaps
 * d_0..d_n (unsuccessful searches) with weights q_0..q_n; the cost of a
 * tree is the sum of (depth + 1) times the weight of every key and gap.
 * Cells are intervals of gaps: for 0 <= a <= b <= n, cell (a, b) is the
 * subtree over keys a+1..b, and
 *
 *   e[a][a] = q_a
 *   e[a][b] = min_{a <= k < b} e[a][k] + e[k+1][b] + W(a, b)
 *   W(a, b) = q_a + ... + q_b + p_{a+1} + ... + p_b
 *
 *   p         host, n int32 key weights p_1..p_n (>= 0; NULL when n = 0).
 *   q         host, n+1 int32 gap weights q_0..q_n (>= 0).
 *   n         number of keys, 0 <= n <= 2^30.
 *   e_out     device, (n+1)*(n+1) int64, row-major, symmetric: e_out[a][b] =
 *             e_out[b][a] = e[a][b]; the optimal tree's cost is e_out[0][n].
 *   root_out  device, (n+1)*(n+1) int32: for a < b the smallest optimal
 *             root key (1-based, in a+1..b); -1 for a >= b.
 * Validation (host, before anything is enqueued): negative weights give
 * MCM_ERR_INVALID_ARG; 2 (n+1) (2n+1) max(p, q) >= 4.6e18 gives
 * MCM_ERR_OVERFLOW.  Exact int64, deterministic; stream semantics as in
 * mcm_solve.
 */
mcm_status mcm_obst_solve(const int32_t *p, const int32_t *q, int32_t n, int64_t *e_out,
                          int32_t *root_out, hipStream_t stream);

/* mcm_obst_solve with an explicit kernel path (mcm_algo): the tiled kernels
 * in their weight-interval mode (W added once per cell after its minimum;
 * needs 2 (n+1) (2n+1) max(p, q) < 2^46, else MCM_ERR_UNSUPPORTED), or the
 * int64 diagonal launches, which accept every valid input.  AUTO takes the
 * tiled path when it accepts the input.  Both return the same bytes. */
mcm_status mcm_obst_solve_algo(const int32_t *p, const int32_t *q, int32_t n, int64_t *e_out,
                               int32_t *root_out, int32_t algo, hipStream_t stream);

/*
 * Request server: continuous batching of many chains on one device.
 *
 * The server owns one device arena of `mem_budget` bytes from which each
 * admitted request gets its dims and its m/s tables (n*n*12 bytes plus the
 * dims), a FIFO queue, and a scheduler thread.  Every iteration the
 * scheduler admits queued requests in arrival order while a slot (at most
 * `max_slots` requests hold memory at once) and arena memory are free,
 * then advances every admitted, unfinished request by one tile-diagonal:
 * one launch of each tiled kernel serves them all, each at its own
 * tile-diagonal, so requests that arrive while others run join the next
 * iteration and their work overlaps on the device.  Up to two iterations
 * are in flight; a request is complete when the iteration holding its last
 * tile-diagonal has finished on the device.  Results are bit-identical to
 * mcm_solve of the same chain.  Chains outside the tiled path's
 * fp64-exact range run the int64 wavefront in one iteration.
 *
 *   mcm_server_create  budget in bytes (> 0), max_slots >= 1; work runs on
 *                      `stream` (0 = null stream).  MCM_ERR_NO_MEMORY if
 *                      the arena cannot be allocated.
 *   mcm_server_submit  validates p (host, n+1 dims, copied before return)
 *                      and queues the request under the caller's `tag`.
 *                      A tag names one request from its submission until
 *                      its release: submitting under a live tag returns
 *                      MCM_ERR_INVALID_ARG.  MCM_ERR_INVALID_ARG /
 *                      MCM_ERR_OVERFLOW for a bad chain, MCM_ERR_NO_MEMORY
 *                      if the request alone exceeds the arena; never
 *                      blocks (the queue is unbounded, so admission
 *                      failure is a wait in the queue, not an error).
 *   mcm_server_poll    moves up to `cap` completed requests into `out`
 *                      (oldest first) and sets *count.  m and s are device
 *                      pointers into the arena, valid until released.
 *   mcm_server_release returns a completed (polled) request's memory to the
 *                      arena.  The caller must have finished every read of
 *                      its tables (work on the server's stream, or
 *                      synchronised).  MCM_ERR_INVALID_ARG for an unknown
 *                      tag.
 *   mcm_server_stats   counters; any pointer may be NULL.
 *   mcm_server_destroy stops the scheduler, waits for the device, frees
 *                      the arena; pending requests are dropped.
 *   mcm_clock_now      the steady clock the timestamps use, in seconds.
 * Times are seconds on mcm_clock_now's clock: t_submit when submitted,
 * t_admit when memory was granted, t_done when completion was observed.
 */
typedef struct mcm_server mcm_server;
typedef struct mcm_request_info {
    uint64_t tag;
    int32_t n;
    int32_t status;      /* mcm_status of the request */
    int64_t *m;          /* device, n*n int64 (arena memory) */
    int32_t *s;          /* device, n*n int32 (arena memory) */
    double t_submit, t_admit, t_done;
} mcm_request_info;

mcm_status mcm_server_create(size_t mem_budget, int32_t max_slots, hipStream_t stream,
                             mcm_server **out);
mcm_status mcm_server_submit(mcm_server *srv, const int32_t *p, int32_t n, uint64_t tag);
mcm_status mcm_server_poll(mcm_server *srv, mcm_request_info *out, int32_t cap, int32_t *count);
mcm_status mcm_server_release(mcm_server *srv, uint64_t tag);
/* Arena bytes a request for chain p (host, n+1 dims) holds while admitted:
 * its dims, m and s tables, and its partial minima.  0 if p is invalid. */
size_t mcm_server_request_bytes(const int32_t *p, int32_t n);
mcm_status mcm_server_stats(mcm_server *srv, int64_t *queued, int64_t *active,
                            int64_t *completed, int64_t *iterations, int64_t *bytes_in_use);
void mcm_server_destroy(mcm_server *srv);
double mcm_clock_now(void);

/*
 * Kernel-level profiling on the library's own launches (HIP events on the
 * stream each kernel is enqueued on).  Enabling clears the counters;
 * reading synchronises the recorded events.  Classes:
 *   0 setup (diagonal tiles / init), 1 tiled bulk, 2 tiled closure,
 *   3 wavefront diagonals, 4 batched.
 * mcm_profile_read returns MCM_OK and fills: total kernel milliseconds,
 * number of launches, and the split evaluations those launches performed
 * (the algorithmic count, not counting padding).
 */
void mcm_profile_enable(int32_t on);
/* Times only the classes whose bit is set (bit c: class c); 0 disables.
 * Each timed launch adds two event records to its stream, so a caller that
 * times one kernel class can leave the others unmarked.
 * MCM_PROFILE_SERIAL in the mask (with or without class bits) runs every
 * single-chain tiled solve as a serial schedule while it is set: every
 * launch on the caller's stream in schedule order, the bulk chunking fitted
 * to the whole device, so each timed launch has the device to itself and
 * its duration is the kernel's alone.  The bytes written are the same; the
 * solve is slower (nothing overlaps). */
#define MCM_PROFILE_SERIAL (1u << 16)
void mcm_profile_enable_mask(uint32_t mask);
mcm_status mcm_profile_read(int32_t kernel_class, double *total_ms, int64_t *launches,
                            double *split_evals);

#ifdef __cplusplus
}
#endif

#endif /* MCM_H_ */
