"""Host replica of the chunked permutation kernels (solve.hip perm_chunk_kernel and
perm_apply_kernel), pinned to the definition of LAPACK's interchanges: rows k and
ipiv[k] - 1 trade places for k = 0, 1, ..., and perm[i] is the original row that
ends at position i.  The replica restates the kernels' steps (chunks of 256
interchanges; per chunk, the moves of its own positions and of its partners past
the chunk, each traced back through the chunk; moves applied in chunk order, every
source read before any write) and must agree with the sequential definition on
random, repeated and invalid pivot entries.  No GPU needed."""
import numpy as np
import pytest

PCH = 256


def sequential(ipiv, n):
    rows = list(range(n))
    for k in range(n):
        pv = ipiv[k] - 1
        if not (k < pv < n):
            pv = k          # an invalid entry is a no-op
        rows[k], rows[pv] = rows[pv], rows[k]
    return rows


def chunked(ipiv, n):
    content = list(range(n))
    for c in range((n + PCH - 1) // PCH):
        k0, kc = c * PCH, min(PCH, n - c * PCH)
        sp = []
        for t in range(PCH):
            k = k0 + t
            pv = ipiv[k] - 1 if t < kc else k
            sp.append(pv if (t < kc and k < pv < n) else k)
        moves = []
        for h in range(2):
            for t in range(PCH):
                p = k0 + t if h == 0 else sp[t]
                cand = t < kc and (h == 0 or p >= k0 + kc)
                src = p
                for i in range(kc - 1, -1, -1):
                    a, b = k0 + i, sp[i]
                    src = b if src == a else (a if src == b else src)
                if cand and src != p:
                    moves.append((p, src))
        vals = [(p, content[s]) for p, s in moves]     # every read before any write
        for p, v in vals:
            content[p] = v
    return content


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 513, 900])
def test_chunked_permutation_matches_the_interchanges(n):
    g = np.random.default_rng(n)
    cases = [
        [int(g.integers(k, n)) + 1 for k in range(n)],                              # any partner below
        [k + 1 if g.random() < 0.6 else int(g.integers(k, n)) + 1 for k in range(n)],  # many no-ops
        [min(n, k + 1 + int(g.integers(0, 3))) for k in range(n)],                   # short hops, repeats
        [int(g.integers(-3, n + 3)) for k in range(n)],                              # invalid entries too
    ]
    for ipiv in cases:
        assert chunked(ipiv, n) == sequential(ipiv, n)


def test_replica_catches_a_planted_mistake():
    """Tracing the chunk forwards instead of backwards (a plausible slip) gives a different order."""
    n = 300
    g = np.random.default_rng(5)
    ipiv = [int(g.integers(k, n)) + 1 for k in range(n)]
    ref = sequential(ipiv, n)

    def forward_trace(ipiv, n):
        content = list(range(n))
        for c in range((n + PCH - 1) // PCH):
            k0, kc = c * PCH, min(PCH, n - c * PCH)
            sp = [(ipiv[k0 + t] - 1) if (k0 + t < n and k0 + t < ipiv[k0 + t] - 1 < n) else k0 + t for t in range(kc)]
            moves = []
            for p in set(list(range(k0, k0 + kc)) + sp):
                src = p
                for i in range(kc):          # wrong direction
                    a, b = k0 + i, sp[i]
                    src = b if src == a else (a if src == b else src)
                if src != p:
                    moves.append((p, src))
            vals = [(p, content[s]) for p, s in moves]
            for p, v in vals:
                content[p] = v
        return content
    assert forward_trace(ipiv, n) != ref
