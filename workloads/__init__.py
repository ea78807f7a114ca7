"""Seeded synthetic inputs shared by the product path, the tests and the benchmark.

This module draws inputs only: graphs, angle sets and random matrices. It holds
none of the method's arithmetic (no gates, no tensors, no contraction), so the
oracle and the GPU path can both read the same inputs without sharing any code
that computes a result.

Workload recipe (the paper's benchmark family, QAOA Max-Cut on random regular
graphs, Sec. "QAOA / Max-Cut"):
  * graphs: random d-regular graphs on n vertices, drawn by random pairing of
    vertex "stubs" without self loops or repeated edges; a disconnected draw is
    rejected and redrawn, as the paper's generator does;
  * angles: (gamma_1..gamma_p, beta_1..beta_p) uniform in [0, pi);
  * every random number comes from SplitMix64 so the inputs do not depend on
    the numpy version.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), 64-bit output."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) (m <= 2**32, rejection-free multiply-shift)."""
        return ((self.next_u64() >> 32) * m) >> 32


def _connected(n: int, edges: Sequence[Tuple[int, int]]) -> bool:
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    seen = [False] * n
    stack = [0]
    seen[0] = True
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if not seen[y]:
                seen[y] = True
                stack.append(y)
    return all(seen)


def _try_pairing(n: int, d: int, rng: SplitMix64):
    """One attempt at a simple d-regular graph by pairing stubs at random.

    Pairs are drawn one at a time among the remaining stubs; a pair that would
    make a loop or a repeated edge is redrawn (bounded), otherwise the attempt
    fails and the caller starts over.
    """
    stubs = [v for v in range(n) for _ in range(d)]
    edges = set()
    while stubs:
        for _ in range(100):
            i = rng.below(len(stubs))
            j = rng.below(len(stubs))
            u, v = stubs[i], stubs[j]
            if i == j or u == v:
                continue
            e = (min(u, v), max(u, v))
            if e in edges:
                continue
            edges.add(e)
            for k in sorted((i, j), reverse=True):
                stubs[k] = stubs[-1]
                stubs.pop()
            break
        else:
            return None
    return sorted(edges)


def random_regular_graph(d: int, n: int, seed: int) -> List[Tuple[int, int]]:
    """Seeded random connected d-regular simple graph on vertices 0..n-1.

    Returns the sorted edge list (u < v). Disconnected or failed draws are
    redrawn from the same stream.
    """
    if d < 1 or d >= n or (n * d) % 2:
        raise ValueError(f"no {d}-regular graph on {n} vertices")
    rng = SplitMix64(seed * 0x100000001B3 + 1000003 * d + n)
    for _ in range(10000):
        edges = _try_pairing(n, d, rng)
        if edges is not None and _connected(n, edges):
            return edges
    raise RuntimeError("random_regular_graph: no connected draw")


def qaoa_angles(seed: int, n_sets: int, p: int) -> List[List[float]]:
    """n_sets angle vectors (gamma_1..gamma_p, beta_1..beta_p), uniform in [0, pi)."""
    rng = SplitMix64(seed ^ 0xA5A5A5A5DEADBEEF)
    return [[math.pi * rng.uniform() for _ in range(2 * p)] for _ in range(n_sets)]


def random_unitary(dim: int, seed: int):
    """Seeded random dim x dim unitary as nested lists of complex numbers.

    Gram-Schmidt on a matrix of uniform(-1, 1) real and imaginary parts; the
    distribution is not Haar, which does not matter for parity inputs.
    """
    rng = SplitMix64(seed ^ 0x5DEECE66D)
    cols = []
    for _ in range(dim):
        v = [complex(2 * rng.uniform() - 1, 2 * rng.uniform() - 1) for _ in range(dim)]
        for c in cols:
            dot = sum(ci.conjugate() * vi for ci, vi in zip(c, v))
            v = [vi - dot * ci for ci, vi in zip(c, v)]
        nrm = math.sqrt(sum(abs(x) ** 2 for x in v))
        cols.append([x / nrm for x in v])
    return [[cols[j][i] for j in range(dim)] for i in range(dim)]


def random_circuit(n: int, n_gates: int, seed: int, kinds_1q: Sequence[str] = ("H", "X", "Y", "Z", "RX", "RY", "RZ", "U1"),
                   kinds_2q: Sequence[str] = ("ZZ", "CNOT", "CZ", "U2")):
    """Seeded random circuit description: list of (kind, q0, q1, theta, matrix_seed).

    q1 is -1 for one-qubit gates; theta is used by rotations; matrix_seed by
    the custom U1/U2 gates (see random_unitary). Descriptions only: each side
    builds its own gate matrices from them.
    """
    rng = SplitMix64(seed ^ 0x1234567)
    out = []
    for _ in range(n_gates):
        if n >= 2 and rng.uniform() < 0.5:
            k = kinds_2q[rng.below(len(kinds_2q))]
            q0 = rng.below(n)
            q1 = rng.below(n - 1)
            if q1 >= q0:
                q1 += 1
        else:
            k = kinds_1q[rng.below(len(kinds_1q))]
            q0, q1 = rng.below(n), -1
        out.append((k, q0, q1, 2 * math.pi * rng.uniform(), rng.next_u64() & 0xFFFFFFFF))
    return out
