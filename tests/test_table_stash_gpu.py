"""Membership tables with keys in the stash, on the GPU, against the oracle.

Three sample keys whose hash differences vanish on the slot bits share both
cuckoo slots, so one of them must live in the table's stash; the same holds
for four XY masks in the group table.  The lanes past the last group (or
sample) of a chunk repeat that chunk's last candidate; a stashed candidate
found there must not be counted again.  The keys are built from the engine's
hash words (splitmix64 from a fixed seed, the first 32 independent in their
low halves and the first 64 as whole words), restated here to aim the
collisions; the test checks through ``samples_info`` that the stash is used.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import jw  # noqa: E402

M64 = (1 << 64) - 1


def _splitmix(state):
    state = (state + 0x9E3779B97F4A7C15) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def _independent(basis, v):
    """Adds v to a GF(2) basis keyed by leading bit; False if v depends on it."""
    while v:
        top = v.bit_length() - 1
        if top not in basis:
            basis[top] = v
            return True
        v ^= basis[top]
    return False


def hash_words():
    s, R, b32, b64 = 0x2408076250, [], {}, {}
    while len(R) < 32:
        s, v = _splitmix(s)
        if _independent(b32, v & 0xFFFFFFFF):
            _independent(b64, v)
            R.append(v)
    while len(R) < 64:
        s, v = _splitmix(s)
        if _independent(b64, v):
            R.append(v)
    while len(R) < 128:
        s, v = _splitmix(s)
        R.append(v)
    return np.array(R, dtype=np.uint64)


def lin(keys, R, n_qubits):
    """Linear hash of keys [n, W]: XOR of R[q] over the set qubits q."""
    h = np.zeros(keys.shape[0], dtype=np.uint64)
    for q in range(n_qubits):
        w, b = divmod(q, 64)
        bit = (keys[:, w] >> np.uint64(b)) & np.uint64(1)
        h ^= np.where(bit == 1, R[q], np.uint64(0))
    return h


def random_keys(rng, n, n_qubits):
    W = (n_qubits + 63) // 64
    k = rng.integers(0, 1 << 32, size=(n, W, 2), dtype=np.uint64)
    k = k[..., 0] | (k[..., 1] << np.uint64(32))
    for w in range(W):
        nb = n_qubits - 64 * w
        if nb < 64:
            k[:, w] &= np.uint64((1 << nb) - 1)
    return k


def colliding_workload(n_qubits, seed):
    """U = {a, b, c} (one shared slot pair), its shift by D, ten random keys;
    groups 0, a^b, a^c, b^c (one shared slot pair), three random masks, D last."""
    rng = np.random.default_rng(seed)
    R = hash_words()
    zero_bits = np.uint64((1 << 13) - 1)   # slot bits of both tables (<= 64 slots) and the tag's low bits
    a = random_keys(rng, 1, n_qubits)
    ha = lin(a, R, n_qubits)[0]
    found = []
    while len(found) < 2:
        cand = random_keys(rng, 1 << 16, n_qubits)
        d = lin(cand, R, n_qubits) ^ ha
        ok = np.nonzero((d & zero_bits) == 0)[0]
        for i in ok:
            if len(found) < 2 and not (cand[i] == a[0]).all():
                found.append(cand[i])
    b, c = found
    a = a[0]
    D = random_keys(rng, 1, n_qubits)[0]
    base = [a, b, c]
    keys = base + [k ^ D for k in base] + list(random_keys(rng, 10, n_qubits))
    keys = np.array(keys, dtype=np.uint64)
    assert len({tuple(k) for k in keys.tolist()}) == len(keys)
    xy = [np.zeros_like(a), a ^ b, a ^ c, b ^ c] + list(random_keys(rng, 3, n_qubits)) + [D]
    xy = np.array(xy, dtype=np.uint64)
    yz = random_keys(rng, len(xy), n_qubits)
    coeff = rng.normal(size=len(xy))
    ham = jw.PauliHamiltonian(n_qubits, coeff, xy, yz)
    logpsi = rng.normal(size=len(keys)) * 0.3 + 1j * rng.normal(size=len(keys))
    return ham, keys, logpsi


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_07625_amd as pe
    e = pe.Engine(0)
    yield e
    e.close()


@pytest.mark.parametrize("n_qubits", [20, 48, 100])
def test_stashed_keys_counted_once(eng, n_qubits):
    ham, keys, logpsi = colliding_workload(n_qubits, seed=n_qubits)
    eng.set_hamiltonian(ham.n_qubits, ham.coeff, ham.xy, ham.yz)
    eng.set_samples(torch.from_numpy(keys.view(np.int64)).cuda())
    info = eng.samples_info()
    assert info["n_unique"] == len(keys) and info["table_stash"] >= 1, info
    ref = oracle.local_energy(ham, keys, logpsi)
    pi, pj, pg = (a.astype(np.int64) for a in oracle.find_pairs(ham, keys))
    L = torch.from_numpy(logpsi).cuda()
    for variant in ("terms", "batch", "trie"):
        assert eng.count_pairs(variant) == pi.size, variant
        i, j, g = (t.cpu().numpy().astype(np.int64) for t in eng.find_pairs(variant))
        np.testing.assert_array_equal(i, pi)
        np.testing.assert_array_equal(j, pj)
        np.testing.assert_array_equal(g, pg)
        for prec, tol in (("fp64", 1e-9), ("fp32c", 1e-6)):
            e, _ = eng.local_energy(L, None, variant=variant, precision=prec)
            assert np.abs(e.cpu().numpy() - ref).max() <= tol, (variant, prec)
