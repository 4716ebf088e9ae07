"""Pins of the sampling oracle (oracle/sampler.py): normalisation and
masking of the autoregressive model by enumeration, exactness of the pruned
search against the unpruned tree, and the sampling law of the Gumbel top-K
trick (Gumbel-max frequencies for K = 1, the without-replacement inclusion
probabilities for K = 2) over many seeds."""
import itertools

import numpy as np
import pytest

from oracle import sampler as S


def _model(N=8, D=3, H=16, seed=0, n_up=-1, n_down=-1, scale=1.5):
    return S.random_model(N, D, H, np.random.default_rng(seed), n_up, n_down, scale=scale)


@pytest.mark.parametrize("n_up,n_down", [(-1, -1), (2, 2), (1, 3)])
def test_model_normalised_and_masked(n_up, n_down):
    m = _model(n_up=n_up, n_down=n_down)
    total = 0.0
    for key in range(1 << m.N):
        lp = S.log_prob(m, key)
        up = sum((key >> q) & 1 for q in range(0, m.N, 2))
        dn = sum((key >> q) & 1 for q in range(1, m.N, 2))
        ok = n_up < 0 or (up == n_up and dn == n_down)
        assert np.isfinite(lp) == ok, (key, lp)
        if ok:
            total += np.exp(lp)
    assert abs(total - 1.0) < 1e-12


def test_conditioned_value():
    """The conditioned perturbed log-probability of the largest child is
    the parent's, and the others stay below it; the closed form equals the
    direct evaluation where the latter is representable."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        T = rng.normal(scale=3)
        L = np.sort(rng.normal(scale=3, size=4))
        Z = L[-1]
        assert S.conditioned(T, Z, Z) == T
        for x in L[:-1]:
            v = S.conditioned(T, Z, x)
            assert v < T
            assert abs(v - (-np.log(np.exp(-T) - np.exp(-Z) + np.exp(-x)))) < 1e-9 * max(1, abs(v))


@pytest.mark.parametrize("n_up,n_down,seed", [(-1, -1, 3), (2, 2, 4), (2, 1, 5)])
def test_pruned_search_is_exact(n_up, n_down, seed):
    """Keeping only K prefixes per qudit returns exactly the K best leaves of
    the unpruned tree (same keys, log-probabilities and perturbed values):
    the conditioning makes a prefix's value the maximum over its leaves."""
    m = _model(n_up=n_up, n_down=n_down, seed=seed)
    full_keys, full_l, full_T = S.ar_gumbel_top_k(m, 1 << m.N, seed=99)
    n_states = sum(np.isfinite(S.log_prob(m, k)) for k in range(1 << m.N))
    assert len(full_keys) == n_states
    for K in (1, 2, 5, 17, n_states // 2):
        keys, l, T = S.ar_gumbel_top_k(m, K, seed=99)
        assert keys == full_keys[:K]
        np.testing.assert_allclose(l, full_l[:K], atol=1e-12)
        np.testing.assert_allclose(T, full_T[:K], atol=1e-12)
        np.testing.assert_allclose(l, [S.log_prob(m, k) for k in keys], atol=1e-12)


def test_gumbel_max_frequencies():
    """K = 1: the sample is x with probability p(x)."""
    m = _model(N=6, D=3, H=8, seed=6, scale=1.0)
    p = np.array([np.exp(S.log_prob(m, k)) for k in range(64)])
    n = 6000
    counts = np.zeros(64)
    for s in range(n):
        keys, _, _ = S.ar_gumbel_top_k(m, 1, seed=1000 + s)
        counts[keys[0]] += 1
    sigma = np.sqrt(n * p * (1 - p))
    assert np.all(np.abs(counts - n * p) <= 5 * sigma + 1)
    chi2 = ((counts - n * p) ** 2 / (n * p)).sum()
    assert chi2 < 64 + 6 * np.sqrt(2 * 64)


def test_without_replacement_inclusion():
    """K = 2: P(x in U) = p(x) + sum_{y != x} p(y) p(x) / (1 - p(y)), the law
    of drawing two samples one by one without replacement."""
    m = _model(N=6, D=3, H=8, seed=7, scale=1.0)
    p = np.array([np.exp(S.log_prob(m, k)) for k in range(64)])
    incl = p + np.array([sum(p[y] * p[x] / (1 - p[y]) for y in range(64) if y != x) for x in range(64)])
    assert abs(incl.sum() - 2.0) < 1e-12
    n = 6000
    counts = np.zeros(64)
    for s in range(n):
        keys, _, _ = S.ar_gumbel_top_k(m, 2, seed=50000 + s)
        assert len(set(keys)) == 2
        for k in keys:
            counts[k] += 1
    sigma = np.sqrt(n * incl * (1 - incl))
    assert np.all(np.abs(counts - n * incl) <= 5 * sigma + 1)


def test_gumbel_noise_uniform():
    """The counter-based uniforms: mean 1/2, and G has the Gumbel mean (Euler's
    constant) and variance pi^2 / 6."""
    g = np.array([S.gumbel(5, lvl, [w], c) for lvl, w, c in itertools.product(range(4), range(50), range(50))])
    assert abs(g.mean() - np.euler_gamma) < 0.05
    assert abs(g.var() - np.pi ** 2 / 6) < 0.1
