"""Reporting helpers: the relative scaled efficiency of Table 1 and latency percentiles."""
import math


def effic_rel(T, N, P, T0, N0, P0):
    """Relative scaled efficiency (Table 1 caption): (T0 / T) * (N / N0) * (P0 / P)."""
    return (T0 / T) * (N / N0) * (P0 / P)


def percentile(values, q):
    """Nearest-rank percentile (q in (0, 100])."""
    xs = sorted(values)
    if not xs:
        raise ValueError("empty sample")
    k = max(1, int(math.ceil(q / 100.0 * len(xs))))
    return xs[k - 1]
