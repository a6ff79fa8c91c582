"""The bound on how fast the recursion of eq. (new_weight) can move ln w: an
update subtracts ln h from each visited bin (1 <= h <= P M configurations of
one round) and leaves the unvisited ones, so the spread max ln w - min ln w
over the reachable bins grows by at most ln(P M) per iteration.  From ln w = 0
a flat histogram needs the spread of ln g, so at least about
(ln g_max - ln g_min) / ln(P M) iterations; the large-lattice records are
read against this bound.  Checked on the oracle's recursion, every iteration."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("L,P,M,bs", [(4, 8, 50, 0), (6, 16, 20, 1), (8, 4, 30, 1)])
def test_spread_of_ln_w_grows_at_most_ln_PM_per_iteration(L, P, M, bs):
    N = L * L
    reach = np.array([O.level_reachable(L, m) for m in range(N + 1)])
    nb = (N >> bs) + 1
    rb = np.zeros(nb, dtype=bool)
    rb[np.flatnonzero(reach) >> bs] = True
    R = O.Run(L, P, seed=3, bin_shift=bs)
    span_prev = 0.0
    bound = math.log(P * M)
    grew = []
    for it in range(12):
        tr, _ = R.run(M)
        R.join(tr)
        kept = R.retained
        H = R.H.copy()
        R.update()
        w = R.lnW[rb]
        span = float(w.max() - w.min())
        # the update moved each visited bin by -ln h with h <= kept <= P M
        assert kept <= P * M and H.max() <= P * M
        assert span - span_prev <= math.log(max(1, H.max())) + 1e-9 <= bound + 1e-9, (it, span, span_prev)
        grew.append(span - span_prev)
        span_prev = span
    # the recursion does move the weight: from ln w = 0 the first update's
    # spread is the log-ratio of its largest and smallest counts over the
    # reachable bins (an unvisited bin counts as one)
    assert grew[0] > 0
