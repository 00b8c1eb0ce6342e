"""Readings of the paper that the oracle and the GPU path rely on (no GPU).

The MCM pipeline of Fig. 8 (Section IV-B) runs n-1 threads in lockstep:
at head position i, thread j folds split j of element i-j+1 into ST.
Theorem 1 (Section IV-C) shows that no two threads touch the same cell in a
substep; it does not show that the operands a thread reads are final.  This
test runs Fig. 8 literally, in lockstep (every read of a step sees the
table as it was before that step's writes), and shows it can read an
element before its last split has been folded in.  The defining recurrence
(Eq. (2) with the textbook cost function) is therefore what the oracle and
every kernel implement, and Fig. 8 is treated as a description of
parallelism, not as the definition of the result.
"""
from oracle import linear


def fig8_lockstep(p):
    """Fig. 8 executed step by step; returns the final ST (1-based list)."""
    n = len(p) - 1
    total = n * (n + 1) // 2
    ST = [0] * (total + 1)
    for i in range(n + 1, total + n - 1):          # head positions
        writes = []
        for j in range(1, n):                        # threads, in parallel
            x = i - j + 1
            if not (n + 1 <= x <= total):
                continue
            pairs = linear.operand_pairs(x, n)
            if j > len(pairs):                       # element has k_x < j splits
                continue
            a, b = linear.element_at(x, n)
            l, r = pairs[j - 1]
            v = ST[l] + ST[r] + p[a - 1] * p[a + j - 1] * p[b]   # substeps 1-3
            writes.append((x, j, v))
        for x, j, v in writes:                       # substep 4
            ST[x] = v if j == 1 else min(ST[x], v)
    return ST


def test_fig8_lockstep_reads_unfinished_operand():
    p = [50, 2, 50, 1, 1]       # 1-based dims: A1 50x2, A2 2x50, A3 50x1, A4 1x1
    n = 4
    ref, _ = linear.solve_linear(p)
    pipe = fig8_lockstep(p)
    x = linear.element_index(1, 4, n)
    assert ref[x] == 202        # (A1 (A2 A3 A4)) with A2 A3 A4 = (A2 A3) A4
    assert pipe[x] == 250       # split 1 read element (2,4) = 150 before its
                                # split 2 (cost 102) was folded in
    # Every other element agrees: the hazard is only on that read.
    assert all(pipe[y] == ref[y] for y in range(1, len(ref)) if y != x)


def test_fig8_step_count_and_distinct_reads():
    # The outer loop of Fig. 8 runs n(n+1)/2 - 2 steps (heads n+1 ..
    # n(n+1)/2 + n - 2), and within a step the left operands and the right
    # operands read by active threads are distinct (Lemmas 1 and 2).
    for n in range(3, 11):
        total = n * (n + 1) // 2
        heads = list(range(n + 1, total + n - 1))
        assert len(heads) == total - 2
        for i in heads:
            lefts, rights = [], []
            for j in range(1, n):
                x = i - j + 1
                if n + 1 <= x <= total and j <= len(linear.operand_pairs(x, n)):
                    l, r = linear.operand_pairs(x, n)[j - 1]
                    lefts.append(l)
                    rights.append(r)
            assert len(set(lefts)) == len(lefts)
            assert len(set(rights)) == len(rights)
