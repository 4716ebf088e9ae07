"""Sampling without replacement on the GPU against the sampling oracle: the
same model weights and seed give the same samples in the same order, their
log-probabilities and conditioned perturbed log-probabilities within FP64
rounding (the perceptrons' sums run in a different order)."""
import numpy as np
import pytest
import torch

from oracle import sampler as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import paper_2408_07625_amd as pe
    e = pe.Engine(0)
    yield e
    e.close()


def _weights(m):
    return {n: torch.from_numpy(np.ascontiguousarray(getattr(m, n))).cuda()
            for n in ("W1", "b1", "W2", "b2", "W3", "b3")}


@pytest.mark.parametrize("N,D,K,n_up,n_down,seed", [
    (12, 3, 50, -1, -1, 1),        # four full qudits, no mask
    (12, 6, 100, 3, 3, 2),         # two qudits of 64 outcomes, (3, 3) electrons: 400 states
    (12, 6, 1000, 3, 3, 3),        # K above the number of allowed states
    (20, 6, 300, 5, 5, 4),         # ragged last qudit (2 qubits)
    (13, 4, 200, -1, -1, 5),       # ragged last qudit (1 qubit), odd N
    (70, 5, 40, 10, 9, 6),         # two-word keys, a qudit across the word boundary
])
def test_sample_matches_oracle(eng, N, D, K, n_up, n_down, seed):
    m = S.random_model(N, D, 64, np.random.default_rng(seed), n_up, n_down, scale=1.5)
    keys, logp, pert = eng.sample(N, D, _weights(m), K, seed=1000 + seed, n_up=n_up, n_down=n_down)
    ref_keys, ref_l, ref_T = S.ar_gumbel_top_k(m, K, seed=1000 + seed)
    ref = S.keys_to_words(ref_keys, N)
    got = keys.cpu().numpy().view(np.uint64)
    print(f"sample N={N} D={D} K={K}: {got.shape[0]} samples (oracle {ref.shape[0]})", flush=True)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_allclose(logp.cpu().numpy(), ref_l, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(pert.cpu().numpy(), ref_T, rtol=1e-10, atol=1e-10)
    assert np.unique(got, axis=0).shape[0] == got.shape[0]


def test_sample_all_states_when_k_covers_them(eng):
    """K at least the number of allowed states returns every state of the
    (n_up, n_down) sector once, and their probabilities add to one."""
    N, D = 10, 5
    m = S.random_model(N, D, 64, np.random.default_rng(9), 2, 3, scale=1.0)
    keys, logp, _ = eng.sample(N, D, _weights(m), 5000, seed=3, n_up=2, n_down=3)
    got = {int(k) for k in keys.cpu().numpy()[:, 0]}
    want = {x for x in range(1 << N)
            if sum((x >> q) & 1 for q in range(0, N, 2)) == 2 and sum((x >> q) & 1 for q in range(1, N, 2)) == 3}
    assert got == want and len(got) == keys.shape[0]
    assert abs(np.exp(logp.cpu().numpy()).sum() - 1.0) < 1e-10
