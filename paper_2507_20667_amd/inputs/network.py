"""Circuit -> labelled-leg tensor network (Section 2.1's G = (V, E)).

A network is a list of dense complex tensors, each with an ordered list of
integer edge labels.  A label on two tensor slots is a bound edge; a label on
one slot is an open edge (an edge to the dummy vertex).  Every leg here has
dimension 2.

The mapping of a circuit onto a network is not spelled out in the paper; the
one used here reproduces its tensor counts (Table 1: a GHZ circuit on n qubits
gives 3n tensors, i.e. one tensor per gate plus one rank-1 tensor per qubit at
the input and at the output):
  * input |0> on each qubit: rank 1, legs [wire];
  * one-qubit gate G: rank 2, legs (out, in), T[o, i] = G[o, i];
  * two-qubit gate on (q1, q2): rank 4, legs (o1, o2, i1, i2),
    T[o1, o2, i1, i2] = G[2*o1 + o2, 2*i1 + i2];
  * output <x_q| on each qubit: rank 1, legs [wire].
Tensors are listed in generation order: inputs, gates in time order, outputs.

Like circuits.py this holds no contraction arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuits import Circuit, Gate, gate_matrix


@dataclass
class Network:
    tensors: list = field(default_factory=list)   # np.ndarray complex128, shape (dims...)
    legs: list = field(default_factory=list)      # list[list[int]]
    tags: list = field(default_factory=list)      # 'in' / 'gate' / 'out' / 'obs'
    output_legs: list = field(default_factory=list)
    dims: dict = field(default_factory=dict)      # label -> dimension
    n_qubits: int = 0

    def add(self, data: np.ndarray, legs, tag: str) -> int:
        data = np.asarray(data, dtype=np.complex128)
        legs = [int(x) for x in legs]
        assert data.ndim == len(legs)
        for lab, d in zip(legs, data.shape):
            if lab in self.dims:
                assert self.dims[lab] == d
            self.dims[lab] = int(d)
        self.tensors.append(data)
        self.legs.append(legs)
        self.tags.append(tag)
        return len(self.tensors) - 1

    @property
    def num_tensors(self) -> int:
        return len(self.tensors)

    def flat(self):
        """Arrays in the layout the C ABI takes: ranks, concatenated labels,
        concatenated leg dims."""
        ranks = np.array([len(l) for l in self.legs], dtype=np.int32)
        labels = np.array([x for l in self.legs for x in l], dtype=np.int64)
        dims = np.array([self.dims[x] for l in self.legs for x in l], dtype=np.int64)
        return ranks, labels, dims

    def copy_with(self, overrides: dict) -> "Network":
        n = Network(list(self.tensors), [list(l) for l in self.legs], list(self.tags),
                    list(self.output_legs), dict(self.dims), self.n_qubits)
        for t, d in overrides.items():
            n.tensors[t] = np.asarray(d, dtype=np.complex128).reshape(self.tensors[t].shape)
        return n


def _gate_tensor(g: Gate, adjoint: bool = False) -> np.ndarray:
    m = gate_matrix(g.name, g.params)
    if adjoint:
        m = m.conj().T
    if len(g.qubits) == 1:
        return m.reshape(2, 2)
    return m.reshape(2, 2, 2, 2)


def basis_vec(bit: int) -> np.ndarray:
    v = np.zeros(2, dtype=np.complex128)
    v[int(bit)] = 1.0
    return v


def amplitude_network(circ: Circuit, bits: int | None = 0, open_qubits=()) -> Network:
    """Network for <x|U|0^n>.  Qubits listed in `open_qubits` get no output
    tensor; their final wire stays an open leg.  With bits=None every qubit is
    open (the network then yields the whole state vector).  Open legs are
    ordered most-significant qubit first, so the flattened result index equals
    the basis index restricted to the open qubits."""
    net = Network(n_qubits=circ.n)
    nxt = [0]

    def new():
        nxt[0] += 1
        return nxt[0] - 1

    wire = [new() for _ in range(circ.n)]
    for q in range(circ.n):
        net.add(basis_vec(0), [wire[q]], "in")
    for g in circ.gates:
        if len(g.qubits) == 1:
            (q,) = g.qubits
            o = new()
            net.add(_gate_tensor(g), [o, wire[q]], "gate")
            wire[q] = o
        else:
            q1, q2 = g.qubits
            o1, o2 = new(), new()
            net.add(_gate_tensor(g), [o1, o2, wire[q1], wire[q2]], "gate")
            wire[q1], wire[q2] = o1, o2
    opens = set(range(circ.n)) if bits is None else set(int(q) for q in open_qubits)
    for q in range(circ.n):
        if q in opens:
            continue
        net.add(basis_vec((bits >> q) & 1), [wire[q]], "out")
    net.output_legs = [wire[q] for q in sorted(opens, reverse=True)]
    return net


def output_tensor_ids(net: Network) -> list:
    """Ids of the rank-1 output tensors, qubit order (qubit 0 first among the
    non-open qubits)."""
    return [i for i, t in enumerate(net.tags) if t == "out"]


def amplitude_overrides(net: Network, circ: Circuit, bits: int, open_qubits=()) -> dict:
    """Leaf overrides that turn a network built for one bitstring into the
    network for `bits` (only the output tensors change)."""
    ids = output_tensor_ids(net)
    qs = [q for q in range(circ.n) if q not in set(open_qubits)]
    return {t: basis_vec((bits >> q) & 1) for t, q in zip(ids, qs)}


def lightcone(circ: Circuit, observed) -> list:
    """Indices of gates in the backward light cone of the observed qubits:
    scanning gates from last to first, a gate is kept if it touches an active
    qubit, and then all its qubits become active.  Gates outside the cone
    cancel against their adjoints in U^dag O U."""
    active = set(int(q) for q in observed)
    keep = []
    for idx in range(len(circ.gates) - 1, -1, -1):
        g = circ.gates[idx]
        if any(q in active for q in g.qubits):
            keep.append(idx)
            active.update(g.qubits)
    keep.reverse()
    return keep


def zz_network(circ: Circuit, i: int, j: int, prune: bool = True) -> Network:
    """Closed network for <0^n| U^dag Z_i Z_j U |0^n>.  With prune=True only the
    gates of the backward light cone of {i, j} are kept, and qubits outside it
    are dropped (their <0|0> factors are 1)."""
    gate_ids = lightcone(circ, (i, j)) if prune else list(range(len(circ.gates)))
    gates = [circ.gates[k] for k in gate_ids]
    qubits = set([i, j])
    for g in gates:
        qubits.update(g.qubits)
    if not prune:
        qubits = set(range(circ.n))
    net = Network(n_qubits=circ.n)
    nxt = [0]

    def new():
        nxt[0] += 1
        return nxt[0] - 1

    wire = {q: new() for q in sorted(qubits)}
    for q in sorted(qubits):
        net.add(basis_vec(0), [wire[q]], "in")

    def apply(g: Gate, adjoint: bool):
        t = _gate_tensor(g, adjoint)
        if len(g.qubits) == 1:
            (q,) = g.qubits
            o = new()
            net.add(t, [o, wire[q]], "gate")
            wire[q] = o
        else:
            q1, q2 = g.qubits
            o1, o2 = new(), new()
            net.add(t, [o1, o2, wire[q1], wire[q2]], "gate")
            wire[q1], wire[q2] = o1, o2

    for g in gates:
        apply(g, False)
    for q in (i, j):
        o = new()
        net.add(gate_matrix("Z"), [o, wire[q]], "obs")
        wire[q] = o
    for g in reversed(gates):
        apply(g, True)
    for q in sorted(qubits):
        net.add(basis_vec(0), [wire[q]], "out")
    net.output_legs = []
    return net
