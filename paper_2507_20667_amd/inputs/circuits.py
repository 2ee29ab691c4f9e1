"""Seeded synthetic quantum circuits.

The paper evaluates on gate-level circuit networks (one tensor per gate plus a
rank-1 boundary tensor per qubit at input and output, 10-50 qubits, leg
dimension 2; Section 5.2, Table 1).  Its benchmark suite is not reproduced
here; these seeded families stand in for it with the same shape class.

This module only builds gate lists and gate matrices.  It holds none of the
contraction or planning arithmetic and is the one module shared by the oracle
and the product path.

Conventions (the paper does not fix them):
  * qubit q is bit q of an integer basis index (qubit 0 is the least
    significant bit);
  * H = [[1,1],[1,-1]]/sqrt2, RX(t) = [[c,-is],[-is,c]] with c=cos(t/2),
    s=sin(t/2), RZ(t) = diag(e^{-it/2}, e^{it/2}), CZ = diag(1,1,1,-1),
    CX = |0><0| (x) I + |1><1| (x) X with the first qubit as control;
  * a two-qubit matrix on (q1, q2) is indexed [2*o1+o2, 2*i1+i2].
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: tuple
    params: tuple = ()


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)
    name: str = ""

    def add(self, name, qubits, params=()):
        self.gates.append(Gate(name, tuple(int(q) for q in qubits),
                               tuple(float(p) for p in params)))


_SQ2 = 1.0 / math.sqrt(2.0)


def gate_matrix(name: str, params=()) -> np.ndarray:
    """Unitary of a gate as a complex128 matrix (2x2 or 4x4)."""
    if name == "H":
        return np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128)
    if name == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if name == "Z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if name == "I":
        return np.eye(2, dtype=np.complex128)
    if name == "RX":
        (t,) = params
        c, s = math.cos(t / 2.0), math.sin(t / 2.0)
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "RZ":
        (t,) = params
        return np.array([[complex(math.cos(t / 2.0), -math.sin(t / 2.0)), 0],
                         [0, complex(math.cos(t / 2.0), math.sin(t / 2.0))]],
                        dtype=np.complex128)
    if name == "CZ":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "CX":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[1, 1] = 1
        m[2, 3] = m[3, 2] = 1
        return m
    raise ValueError(f"unknown gate {name}")


def adjoint_gate(g: Gate) -> np.ndarray:
    return gate_matrix(g.name, g.params).conj().T


# ---------------------------------------------------------------- families

def ghz(n: int) -> Circuit:
    """H on qubit 0 then CX(k -> k+1): (|0..0> + |1..1>)/sqrt2."""
    c = Circuit(n, name=f"ghz{n}")
    c.add("H", (0,))
    for k in range(n - 1):
        c.add("CX", (k, k + 1))
    return c


def hadamard_layer(n: int) -> Circuit:
    c = Circuit(n, name=f"hlayer{n}")
    for q in range(n):
        c.add("H", (q,))
    return c


def graph_state_circuit(n: int, edges) -> Circuit:
    """H on every qubit, then CZ on each edge (i, j) in the order given."""
    c = Circuit(n, name=f"graph{n}_e{len(edges)}")
    for q in range(n):
        c.add("H", (q,))
    for i, j in edges:
        c.add("CZ", (i, j))
    return c


def brick_edges(n: int, layers: int) -> list:
    """The CZ bricks of brickwork_circuit's CZ layers: (2i, 2i+1) on even
    layers, (2i+1, 2i+2) on odd ones."""
    out = []
    for layer in range(layers):
        start = 0 if layer % 2 == 0 else 1
        out.extend((q, q + 1) for q in range(start, n - 1, 2))
    return out


def phase_poly_circuit(n: int, depth: int, seed: int) -> Circuit:
    """H on every qubit, then per layer: CX on the disjoint consecutive pairs
    of a random permutation (first of a pair is the control), then RZ(theta)
    on every qubit with theta ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, name=f"phasepoly_n{n}_d{depth}_s{seed}")
    for q in range(n):
        c.add("H", (q,))
    for _ in range(depth):
        perm = rng.permutation(n)
        for i in range(n // 2):
            c.add("CX", (perm[2 * i], perm[2 * i + 1]))
        thetas = rng.uniform(0.0, 2.0 * math.pi, size=n)
        for q in range(n):
            c.add("RZ", (q,), (thetas[q],))
    return c


def brickwork_circuit(n: int, depth: int, seed: int) -> Circuit:
    """Even layers: one rotation per qubit, RX or RZ by a seeded coin, angle
    ~ U[0, 2pi).  Odd layers: CZ bricks on (2i, 2i+1), then (2i+1, 2i+2) on
    the next CZ layer, alternating."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, name=f"brick_n{n}_d{depth}_s{seed}")
    cz_layer = 0
    for layer in range(depth):
        if layer % 2 == 0:
            coins = rng.integers(0, 2, size=n)
            thetas = rng.uniform(0.0, 2.0 * math.pi, size=n)
            for q in range(n):
                c.add("RX" if coins[q] == 0 else "RZ", (q,), (thetas[q],))
        else:
            start = 0 if cz_layer % 2 == 0 else 1
            for q in range(start, n - 1, 2):
                c.add("CZ", (q, q + 1))
            cz_layer += 1
    return c


def random_circuit(n: int, depth: int, seed: int, cx_per_layer: int | None = None,
                   p_nn: float = 0.7) -> Circuit:
    """Per layer: `cx_per_layer` disjoint CX pairs, each nearest-neighbour
    (q, q+1) with probability p_nn, otherwise long-range (|q1-q2| >= 2), with a
    random orientation; every qubit outside the pairs gets one of {H, RX, RZ}
    uniformly, angles ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    if cx_per_layer is None:
        cx_per_layer = max(1, n // 4)
    c = Circuit(n, name=f"rand_n{n}_d{depth}_s{seed}")
    for _ in range(depth):
        free = set(range(n))
        pairs = []
        for _ in range(cx_per_layer):
            want_nn = rng.random() < p_nn
            if want_nn:
                cand = [(q, q + 1) for q in range(n - 1) if q in free and q + 1 in free]
            else:
                fl = sorted(free)
                cand = [(a, b) for i, a in enumerate(fl) for b in fl[i + 1:] if b - a >= 2]
            if not cand:
                fl = sorted(free)
                cand = [(a, b) for i, a in enumerate(fl) for b in fl[i + 1:]]
            if not cand:
                break
            a, b = cand[int(rng.integers(0, len(cand)))]
            if rng.random() < 0.5:
                a, b = b, a
            pairs.append((a, b))
            free.discard(a)
            free.discard(b)
        for a, b in pairs:
            c.add("CX", (a, b))
        kinds = rng.integers(0, 3, size=n)
        thetas = rng.uniform(0.0, 2.0 * math.pi, size=n)
        for q in range(n):
            if q not in free:
                continue
            k = int(kinds[q])
            if k == 0:
                c.add("H", (q,))
            elif k == 1:
                c.add("RX", (q,), (thetas[q],))
            else:
                c.add("RZ", (q,), (thetas[q],))
    return c


def random_bitstrings(n: int, count: int, seed: int) -> list:
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(0, 1 << n, size=count, dtype=np.int64)]


def circuit_mix(count: int, seed0: int = 0, n_range=(12, 26), d_range=(8, 20)) -> list:
    """`count` circuits of the random family, circuit i drawn from seed
    seed0 + i: n ~ U{n_range}, depth ~ U{d_range}, floor(n/4) CX pairs per
    layer (70 % nearest-neighbour).  Returns (seed, circuit) pairs."""
    out = []
    for i in range(count):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        out.append((seed, random_circuit(n, d, seed, cx_per_layer=n // 4)))
    return out


def zipf_indices(count: int, num: int, s: float, seed: int) -> list:
    """`num` indices in [0, count) from a Zipf(s) law truncated to `count`
    values (draws above the range are redrawn): index 0 is the most likely."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < num:
        v = rng.zipf(s, size=num)
        out.extend(int(x) - 1 for x in v if x <= count)
    return out[:num]
