"""Closed-form amplitudes used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

  * GHZ: H on qubit 0 then CX(k -> k+1) gives (|0..0> + |1..1>)/sqrt2.
  * A Hadamard layer gives every amplitude 2^(-n/2).
  * Phase-polynomial family (H layer, then layers of CX on disjoint pairs and
    RZ on every qubit): every CX layer permutes basis states and is its own
    inverse, every RZ layer is diagonal, so <x|U|0^n> = 2^(-n/2) e^{i Phi(x)}
    where Phi collects, layer by layer from the last, the RZ phase of the
    current bitstring and then maps the bitstring back through that layer's
    CX gates.  RZ(t) = diag(e^{-it/2}, e^{it/2}).
  * Single-qubit: <0|RX(t)|0> = cos(t/2), <1|RX(t)|0> = -i sin(t/2),
    <0|RZ(t)|0> = e^{-it/2}.
  * Graph state (H on every qubit, then CZ on the edges of a graph): H^n|0>
    is the uniform superposition and each CZ(i, j) multiplies basis state x
    by (-1)^(x_i x_j), so <x|U|0^n> = 2^(-n/2) (-1)^(sum over edges of
    x_i x_j).  It fixes the CZ matrix, and it does not depend on the
    orientation or the order of the CZ gates.
"""
from __future__ import annotations

import cmath
import math


def ghz_amplitude(n: int, x: int) -> complex:
    return 1.0 / math.sqrt(2.0) if x in (0, (1 << n) - 1) else 0.0


def hadamard_layer_amplitude(n: int, x: int) -> complex:
    return 2.0 ** (-n / 2.0)


def phase_poly_amplitude(circ, x: int) -> complex:
    """Exact amplitude of a phase_poly_circuit for bitstring x."""
    n = circ.n
    gates = list(circ.gates)
    assert all(g.name == "H" for g in gates[:n])
    layers = []
    cur = None
    for g in gates[n:]:
        if g.name == "CX":
            if cur is None or cur[1]:
                cur = ([], [])
                layers.append(cur)
            cur[0].append(g)
        elif g.name == "RZ":
            cur[1].append(g)
        else:
            raise ValueError("not a phase-polynomial circuit")
    z = [(x >> q) & 1 for q in range(n)]
    phi = 0.0
    for cxs, rzs in reversed(layers):
        for g in rzs:
            (q,) = g.qubits
            (t,) = g.params
            phi += t / 2.0 if z[q] else -t / 2.0
        for g in cxs:
            c, t = g.qubits
            z[t] ^= z[c]
    return 2.0 ** (-n / 2.0) * cmath.exp(1j * phi)


def rx_amplitudes(theta: float):
    return math.cos(theta / 2.0), -1j * math.sin(theta / 2.0)


def rz_amplitude0(theta: float) -> complex:
    return cmath.exp(-1j * theta / 2.0)


def graph_state_amplitude(circ, x: int) -> complex:
    """Exact amplitude of an H layer followed by CZ gates only (a graph state)
    for bitstring x: 2^(-n/2) times -1 for every CZ whose two qubits are 1 in x."""
    n = circ.n
    gates = list(circ.gates)
    if [g.name for g in gates[:n]] != ["H"] * n or sorted(g.qubits[0] for g in gates[:n]) != list(range(n)):
        raise ValueError("not a graph-state circuit: it must start with H on every qubit")
    sign = 1
    for g in gates[n:]:
        if g.name != "CZ":
            raise ValueError("not a graph-state circuit: only CZ after the H layer")
        i, j = g.qubits
        if (x >> i) & 1 and (x >> j) & 1:
            sign = -sign
    return sign * 2.0 ** (-n / 2.0)
