"""Oracle for autoregressive sampling without replacement (test
infrastructure).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library's
sampler.  Only the tests and the benchmark's CPU-baseline leg may import it;
the library and its Python binding never do.

What it computes, in plain numpy FP64, following the paper's Methods
("Autoregressive sampling without replacement", Algorithm ARGumbelTopK) and
its ansatz description ("Ansatz architecture", "Local pruning strategy",
"Grouping qubits into qudits", "Global activation"):

  - the conditional distribution of one qudit (D consecutive qubits; the
    last qudit takes the remaining N mod D) given the qubits before it: a
    perceptron per qudit position with two hidden layers of width H, tanh
    activations and the first hidden layer's output added to the second
    layer's pre-activation; its 2^D outputs are log|psi| of the qudit's
    outcomes, shifted by their mean (the global activation, which does not
    change the normalised probabilities); outcomes that can no longer reach
    the target numbers of spin-up and spin-down electrons are masked (zero
    probability, the pruning of unphysical nodes); the rest are normalised:
    log p(c | x_<) = 2 z_c - log sum_{allowed c'} exp(2 z_c');
  - ARGumbelTopK: starting from the empty prefix with l = 0 and conditioned
    perturbed log-probability 0, every kept prefix expands into its allowed
    children with l' = l + log p(c | prefix) and unconditioned perturbed
    L' = l' + G (G a standard Gumbel variable); with Z the largest L' among
    the siblings, the conditioned value is
        Ltil' = -log(exp(-Ltil) - exp(-Z) + exp(-L')),
    evaluated as Ltil - softplus(Ltil - L' + log(1 - exp(L' - Z))); the K
    children with the largest Ltil' (ties to the smaller (parent, outcome))
    are kept; after the last qudit they are the sample set U;
  - Gumbel variables from a counter-based generator: the SplitMix64 output
    function (Steele, Lea, Flood, OOPSLA 2014) chained over (seed, qudit
    index, prefix words, outcome) gives 64 bits; u = (top 53 bits + 0.5)
    2^-53 and G = -log(-log u), so that the noise of a node depends only on
    the node, not on the order in which nodes are visited.

Qubit q is bit q % 64 of word q // 64; qudit k covers qubits [kD, kD + D_k),
outcome c sets qubit kD + t to bit t of c.  Spin orbitals are interleaved
(even qubits spin up, odd qubits spin down).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """SplitMix64 output function."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def gumbel(seed: int, level: int, prefix_words, outcome: int) -> float:
    h = mix64((seed + GOLDEN * (level + 1)) & MASK64)
    for w in prefix_words:
        h = mix64(h ^ int(w))
    h = mix64(h ^ int(outcome))
    u = ((h >> 11) + 0.5) * 2.0 ** -53
    return -np.log(-np.log(u))


class Model:
    """Per-qudit perceptrons.  Arrays (numpy float64):
    W1 [Q][H][N], b1 [Q][H], W2 [Q][H][H], b2 [Q][H], W3 [Q][2^D][H], b3 [Q][2^D]
    (the last qudit uses the first 2^{D_last} rows of W3 / b3)."""

    def __init__(self, n_qubits, qudit, W1, b1, W2, b2, W3, b3, n_up=-1, n_down=-1):
        self.N = n_qubits
        self.D = qudit
        self.Q = (n_qubits + qudit - 1) // qudit
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = W1, b1, W2, b2, W3, b3
        self.n_up, self.n_down = n_up, n_down

    def width(self, k: int) -> int:
        return min(self.D, self.N - k * self.D)

    def _allowed(self, bits_prefix: np.ndarray, k: int) -> np.ndarray:
        """Outcomes of qudit k that can still reach the electron targets."""
        Dk = self.width(k)
        out = np.ones(1 << Dk, dtype=bool)
        if self.n_up < 0:
            return out
        q0 = k * self.D
        up0 = int(sum(bits_prefix[q] for q in range(0, q0, 2)))
        dn0 = int(sum(bits_prefix[q] for q in range(1, q0, 2)))
        for c in range(1 << Dk):
            up, dn = up0, dn0
            for t in range(Dk):
                if (c >> t) & 1:
                    if (q0 + t) % 2 == 0:
                        up += 1
                    else:
                        dn += 1
            rest_up = sum(1 for q in range(q0 + Dk, self.N) if q % 2 == 0)
            rest_dn = sum(1 for q in range(q0 + Dk, self.N) if q % 2 == 1)
            out[c] = up <= self.n_up <= up + rest_up and dn <= self.n_down <= dn + rest_dn
        return out

    def cond_logp(self, bits_prefix: np.ndarray, k: int) -> np.ndarray:
        """log p(c | prefix) for every outcome c of qudit k (-inf if masked)."""
        inp = np.zeros(self.N)
        q0 = k * self.D
        inp[:q0] = 2.0 * bits_prefix[:q0] - 1.0
        h1 = np.tanh(self.W1[k] @ inp + self.b1[k])
        h2 = np.tanh(self.W2[k] @ h1 + self.b2[k] + h1)
        n_out = 1 << self.width(k)
        z = self.W3[k][:n_out] @ h2 + self.b3[k][:n_out]
        z = z - z.mean()
        allowed = self._allowed(bits_prefix, k)
        out = np.full(n_out, -np.inf)
        if not allowed.any():      # an infeasible prefix: no outcome has probability
            return out
        a = 2.0 * z[allowed]
        m = a.max()
        out[allowed] = a - (m + np.log(np.exp(a - m).sum()))
        return out


def random_model(n_qubits, qudit, hidden, rng, n_up=-1, n_down=-1, scale=1.0):
    Q = (n_qubits + qudit - 1) // qudit
    O = 1 << qudit
    W1 = rng.normal(scale=scale / np.sqrt(n_qubits), size=(Q, hidden, n_qubits))
    b1 = rng.normal(scale=0.1, size=(Q, hidden))
    W2 = rng.normal(scale=scale / np.sqrt(hidden), size=(Q, hidden, hidden))
    b2 = rng.normal(scale=0.1, size=(Q, hidden))
    W3 = rng.normal(scale=scale / np.sqrt(hidden), size=(Q, O, hidden))
    b3 = rng.normal(scale=0.5, size=(Q, O))
    return Model(n_qubits, qudit, W1, b1, W2, b2, W3, b3, n_up, n_down)


def _bits(key: int, N: int) -> np.ndarray:
    return np.array([(key >> q) & 1 for q in range(N)], dtype=np.float64)


def _words(key: int, N: int):
    W = (N + 63) // 64
    return [(key >> (64 * w)) & MASK64 for w in range(W)]


def log_prob(model: Model, key: int) -> float:
    """log p(x) = sum over qudits of log p(x_k | x_<k)."""
    bits = _bits(key, model.N)
    total = 0.0
    for k in range(model.Q):
        c = (key >> (k * model.D)) & ((1 << model.width(k)) - 1)
        total += model.cond_logp(bits, k)[c]
        if not np.isfinite(total):
            return -np.inf
    return total


def _softplus(v: float) -> float:
    return max(v, 0.0) + np.log1p(np.exp(-abs(v)))


def _log1mexp(a: float) -> float:
    """log(1 - exp(a)) for a <= 0 (-inf at a = 0)."""
    if a == 0.0:
        return -np.inf
    return np.log(-np.expm1(a)) if a > -np.log(2.0) else np.log1p(-np.exp(a))


def conditioned(T: float, Z: float, L: float) -> float:
    """-log(exp(-T) - exp(-Z) + exp(-L)) for L <= Z."""
    v = T - L + _log1mexp(L - Z)
    return T - (_softplus(v) if np.isfinite(v) else 0.0)


def ar_gumbel_top_k(model: Model, K: int, seed: int):
    """ARGumbelTopK: (keys as Python ints, log p, conditioned perturbed
    log-probability), in descending order of the latter."""
    N = model.N
    beam = [(0, 0.0, 0.0)]     # (prefix key, l, Ltil)
    for k in range(model.Q):
        cand = []
        for parent, (key, l, T) in enumerate(beam):
            bits = _bits(key, N)
            lp = model.cond_logp(bits, k)
            words = _words(key, N)
            kids = []
            for c in range(lp.size):
                if not np.isfinite(lp[c]):
                    continue
                lc = l + lp[c]
                kids.append((c, lc, lc + gumbel(seed, k, words, c)))
            Z = max(x[2] for x in kids)
            for c, lc, Lc in kids:
                cand.append((conditioned(T, Z, Lc), parent, c, key | (c << (k * model.D)), lc))
        cand.sort(key=lambda t: (-t[0], t[1], t[2]))
        beam = [(t[3], t[4], t[0]) for t in cand[:K]]
    keys = [b[0] for b in beam]
    return keys, np.array([b[1] for b in beam]), np.array([b[2] for b in beam])


def keys_to_words(keys, N: int) -> np.ndarray:
    W = (N + 63) // 64
    return np.array([_words(k, N) for k in keys], dtype=np.uint64).reshape(len(keys), W)
