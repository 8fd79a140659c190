"""Algorithm 1 of the paper (Section 8.1), feature-wise variant learning: TEST
INFRASTRUCTURE ONLY (oracle of the library's hawk_learn_feature_wise).

Steps, in the paper's order:
  * the configuration starts at the first value of every dimension;
  * up to q iterations: remember the configuration, then for every dimension
    D_i try each of its values d with all other dimensions fixed, keep the
    value with the lowest workload time (a strictly lower time is needed to
    replace the incumbent, so equal times keep the earlier value), and store
    it in the configuration before moving to the next dimension;
  * stop as soon as a whole iteration leaves the configuration unchanged.

Readings (silent in the paper): measured configurations are memoised (a
configuration is timed once); a dimension whose values are all infeasible
(+inf) keeps its current value; `order` is the visiting order of the
dimensions (feature ordering, Section 8.2).
"""
from __future__ import annotations

import math


def learn_feature_wise(dim_sizes, cost, q=5, order=None):
    """Returns (configuration tuple, number of distinct configurations timed)."""
    n = len(dim_sizes)
    order = list(range(n)) if order is None else list(order)
    memo = {}

    def timed(cfg):
        if cfg not in memo:
            t = float(cost(cfg))
            memo[cfg] = math.inf if math.isnan(t) else t
        return memo[cfg]

    v = [0] * n
    for _ in range(q):
        last = list(v)
        for i in order:
            best_time, best_value = math.inf, None
            for d in range(dim_sizes[i]):
                w = list(v)
                w[i] = d
                t = timed(tuple(w))
                if t < best_time:
                    best_time, best_value = t, d
            if best_value is not None:
                v[i] = best_value
        if v == last:
            break
    return tuple(v), len(memo)
