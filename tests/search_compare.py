"""Comparison of the library's lambda_k search with the oracle's (Sec. 4.3).

Tested points agree (to mid_tol where a float32-evaluated bracket enters),
counts agree to tol (1 + |count|), and every decision agrees unless the
oracle's count lies within twice that margin of k - 1/2, k + 1/2 or k; after
such a near-tie the two searches may part, and the estimates then lie within
the interval of that test.
"""
import math


def compare_search(trace, lam, steps, ref_trace, ref_intervals, ref_lam, ref_steps, k,
                   ref_missed=False, mid_tol=0.0, tol=1e-3):
    """Returns True when every decision agreed (then the estimates agree)."""
    for s, ((lg, cg), (lo_, co)) in enumerate(zip(trace, ref_trace)):
        assert abs(lg - lo_) <= mid_tol, (s, lg, lo_)
        assert abs(cg - co) <= tol * (1 + abs(co)), (s, cg, co)
        dg = (math.floor(cg + 0.5) == k, cg < k)
        do = (math.floor(co + 0.5) == k, co < k)
        if dg != do:
            near = min(abs(co - (k - 0.5)), abs(co - (k + 0.5)), abs(co - k))
            assert near <= 2 * tol * (1 + abs(co)), (s, cg, co)
            a, b = ref_intervals[s]
            if not ref_missed:
                assert abs(lam - ref_lam) <= (b - a) + mid_tol
            return False
    assert steps == ref_steps
    assert abs(lam - ref_lam) <= mid_tol
    return True


def compare_with(trace, lam, steps, ref, k, mid_tol=0.0, tol=1e-3):
    """compare_search against an oracle eigencount.Search."""
    return compare_search(trace, lam, steps, ref.trace, ref.intervals, ref.lam, ref.steps, k,
                          ref.missed, mid_tol, tol)
