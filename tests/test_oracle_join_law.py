"""The law of the first configuration a detailed-balance joint keeps
(Algorithm step 4 as the oracle reads it), checked on the exactly known
4 x 4 lattice.

The joint tests a chain's configurations in order against the seam with the
Metropolis rule min(1, w(E_k) / w(E_seam)) and keeps the first one accepted.
If the chain's configurations were independent draws from a law q(E), the
energy of the first kept one would follow q(E) min(1, w(E) / w(E_seam)),
normalised; with the exact multicanonical weight w = 1/g, q is flat over the
energies and the kept law is proportional to min(1, g(E_seam) / g(E)): it
favours energies rarer than the seam's.  Feeding the oracle's joint traces of
independent flat draws (one bin per level, exact g from enumeration of all
2^16 states) must reproduce that law, and differ from the flat one, which
confirms that the selection the joint applies (and the bias it gives short
segments) is the rule's, not a slip in the oracle."""
import numpy as np

import oracle as O
from paper_0812_2964_amd import exact as X

L, N = 4, 16


def _first_kept_levels(sigma, trials, M, seed):
    g = X.brute_force_dos(L).astype(np.float64)
    reach = np.array([O.level_reachable(L, m) for m in range(N + 1)])
    lnW = np.where(reach, -np.log(np.where(g > 0, g, 1.0)), 0.0)
    levels = np.flatnonzero(reach)
    rng = np.random.default_rng(seed)
    kept = []
    for t in range(trials):
        tr = (rng.choice(levels, size=(1, M)) - N // 2).astype(np.int32)
        cut, H, ret, _ = O.join(L, 0, 1, tr, lnW, sigma, t)
        if cut[0] > 0:
            m = int(tr[0, cut[0] - 1]) + N // 2
            kept.append(m)
            assert ret == M - cut[0] + 1 and H.sum() == ret
    return np.bincount(kept, minlength=N + 1), g, levels


def _chi2(obs, p):
    n = obs.sum()
    e = n * p
    return float(((obs - e) ** 2 / e).sum())


def test_first_kept_configuration_follows_the_selection_law():
    # seam at the ground state (g = 2): energies rarer than it are never
    # penalised, the others are accepted with probability 2 / g(E)
    for sigma, trials in ((0, 6000), (4, 6000)):
        obs, g, levels = _first_kept_levels(sigma, trials, 200, seed=sigma + 1)
        a = np.minimum(1.0, g[sigma] / g[levels])
        pred = a / a.sum()
        flat = np.full(levels.size, 1.0 / levels.size)
        c_pred = _chi2(obs[levels], pred)
        c_flat = _chi2(obs[levels], flat)
        # 14 degrees of freedom: 36.1 is the 0.1 % point
        assert c_pred < 36.1, (sigma, c_pred)
        assert c_flat > 1000.0, (sigma, c_flat)
