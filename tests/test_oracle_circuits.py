"""Pins of the circuit side of the oracle.

  * the state-vector simulator against textbook states (Bell, GHZ, H H = I,
    CX truth table, RX/RZ matrix elements) and norm preservation;
  * the network builder plus loop-nest contraction against the state vector
    (an independent algorithm) on every amplitude of <= 12-qubit circuits of
    each seeded family;
  * closed forms: GHZ amplitudes 1/sqrt2, Hadamard-layer amplitudes
    2^(-n/2), the exact phase-polynomial amplitudes (configuration-1 family,
    also at 20 qubits where no state vector is needed), graph-state signs
    (the CZ convention of the brickwork family), sum |amp|^2 = 1;
  * <Z_i Z_j>: light-cone-pruned network = unpruned network = state-vector
    expectation; GHZ gives 1 and a Hadamard layer 0.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_2507_20667_amd.inputs import (Circuit, amplitude_network, brick_edges, brickwork_circuit,
                                         ghz, graph_state_circuit, hadamard_layer, phase_poly_circuit, random_circuit,
                                         zz_network)
from paper_2507_20667_amd.planner import contiguous_partition, plan_from_partition


def sv_amplitude_via_network(circ, x):
    net = amplitude_network(circ, x)
    plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
    return complex(oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree))


def test_statevector_textbook_states():
    c = Circuit(2)
    c.add("H", (0,))
    c.add("CX", (0, 1))
    psi = oracle.statevector(c)
    s = 1 / math.sqrt(2)
    assert np.allclose(psi, [s, 0, 0, s], atol=1e-15)
    c = Circuit(1)
    c.add("H", (0,))
    c.add("H", (0,))
    assert np.allclose(oracle.statevector(c), [1, 0], atol=1e-15)
    # CX truth table: control qubit 1, target qubit 0, from |q1=1, q0=0> = index 2
    c = Circuit(2)
    c.add("X", (1,))
    c.add("CX", (1, 0))
    assert np.allclose(oracle.statevector(c), [0, 0, 0, 1], atol=0)
    # CX with control 0 leaves |q1=1,q0=0> unchanged
    c = Circuit(2)
    c.add("X", (1,))
    c.add("CX", (0, 1))
    assert np.allclose(oracle.statevector(c), [0, 0, 1, 0], atol=0)
    t = 1.234
    c = Circuit(1)
    c.add("RX", (0,), (t,))
    a0, a1 = cf.rx_amplitudes(t)
    assert np.allclose(oracle.statevector(c), [a0, a1], atol=1e-15)
    c = Circuit(1)
    c.add("RZ", (0,), (t,))
    assert np.allclose(oracle.statevector(c), [cf.rz_amplitude0(t), 0], atol=1e-15)


@pytest.mark.parametrize("n", [3, 7, 10])
def test_ghz_and_hadamard_closed_forms(n):
    psi = oracle.statevector(ghz(n))
    want = np.array([cf.ghz_amplitude(n, x) for x in range(1 << n)])
    assert np.allclose(psi, want, atol=1e-14)
    psi = oracle.statevector(hadamard_layer(n))
    assert np.allclose(psi, 2.0 ** (-n / 2), atol=1e-14)
    for x in (0, (1 << n) - 1, 5 % (1 << n)):
        assert abs(sv_amplitude_via_network(ghz(n), x) - cf.ghz_amplitude(n, x)) < 1e-14
        assert abs(sv_amplitude_via_network(hadamard_layer(n), x) - 2.0 ** (-n / 2)) < 1e-14


@pytest.mark.parametrize("family,seed", [("phase", 0), ("phase", 3), ("brick", 1),
                                         ("rand", 2), ("rand", 5)])
def test_network_matches_statevector_all_amplitudes(family, seed):
    if family == "phase":
        c = phase_poly_circuit(10, 6, seed)
    elif family == "brick":
        c = brickwork_circuit(10, 8, seed)
    else:
        c = random_circuit(10, 6, seed)
    psi = oracle.statevector(c)
    assert abs(np.vdot(psi, psi) - 1) < 1e-12
    net = amplitude_network(c, bits=None)          # every qubit open: the whole state
    plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
    full = oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree, net.output_legs)
    assert np.allclose(full.reshape(-1), psi, atol=1e-13)
    # closed networks for a few bitstrings, on two different trees
    rng = np.random.default_rng(seed)
    for x in rng.integers(0, 1 << c.n, size=4):
        net = amplitude_network(c, int(x))
        seq = oracle.contract_tree(net.legs, net.dims, net.tensors,
                                   oracle.sequential_tree(net.num_tensors))
        two = plan_from_partition(net.legs, net.dims, contiguous_partition(net.num_tensors, 2), 2)
        par = oracle.contract_tree(net.legs, net.dims, net.tensors, two.tree)
        assert abs(complex(seq) - psi[int(x)]) < 1e-13
        assert abs(complex(par) - psi[int(x)]) < 1e-13


def test_phase_polynomial_closed_form_small_and_large():
    c = phase_poly_circuit(10, 10, 0)
    psi = oracle.statevector(c)
    want = np.array([cf.phase_poly_amplitude(c, x) for x in range(1 << 10)])
    assert np.allclose(psi, want, atol=1e-13)
    assert np.allclose(np.abs(psi), 2 ** -5, atol=1e-13)
    c = phase_poly_circuit(20, 8, 1)
    rng = np.random.default_rng(11)
    for x in rng.integers(0, 1 << 20, size=3):
        got = sv_amplitude_via_network(c, int(x))
        assert abs(got - cf.phase_poly_amplitude(c, int(x))) < 1e-13


def test_graph_state_closed_form_pins_cz():
    """CZ-only circuits: the state vector and the network contraction equal
    2^(-n/2) (-1)^(sum over edges of x_i x_j) on every amplitude (brickwork
    CZ bricks, and a random graph with long-range edges in both orientations),
    and on sampled amplitudes of the 20-qubit brickwork layout through the
    network alone.  A wrong CZ matrix or leg convention flips some sign."""
    n = 10
    for edges in (brick_edges(n, 6),
                  [(0, 7), (7, 0), (3, 9), (2, 5), (9, 1), (4, 6), (6, 8), (5, 3)]):
        c = graph_state_circuit(n, edges)
        psi = oracle.statevector(c)
        want = np.array([cf.graph_state_amplitude(c, x) for x in range(1 << n)])
        assert np.allclose(psi, want, atol=1e-13)
        # the closed form is not trivial: both signs occur
        assert (want > 0).any() and (want < 0).any()
        for x in np.random.default_rng(5).integers(0, 1 << n, size=12):
            assert abs(sv_amplitude_via_network(c, int(x)) - want[int(x)]) < 1e-13
    c = graph_state_circuit(20, brick_edges(20, 7))
    for x in np.random.default_rng(12).integers(0, 1 << 20, size=4):
        got = sv_amplitude_via_network(c, int(x))
        assert abs(got - cf.graph_state_amplitude(c, int(x))) < 1e-13
    # a CZ that acted as diag(1, 1, -1, 1) would be caught: the closed form
    # with the sign on x_i (1 - x_j) differs from the state vector
    c = graph_state_circuit(4, [(0, 1)])
    psi = oracle.statevector(c)
    assert abs(psi[0b01] - (-0.25)) > 0.4 and abs(psi[0b11] - (-0.25)) < 1e-15


def test_norm_over_all_bitstrings():
    c = random_circuit(8, 5, 4)
    total = sum(abs(sv_amplitude_via_network(c, x)) ** 2 for x in range(1 << 8))
    assert abs(total - 1.0) < 1e-12


def test_open_legs_subset():
    c = random_circuit(9, 5, 9)
    psi = oracle.statevector(c).reshape([2] * 9)   # axes: qubit 8 .. qubit 0
    x_fixed = 0b101100000                           # qubits 5, 6, 8 set among the closed ones
    opens = (0, 2, 3)
    net = amplitude_network(c, x_fixed, open_qubits=opens)
    plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
    got = oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree, net.output_legs)
    idx = []
    for q in range(8, -1, -1):
        idx.append(slice(None) if q in opens else (x_fixed >> q) & 1)
    assert np.allclose(got, psi[tuple(idx)], atol=1e-13)


@pytest.mark.parametrize("seed,i,j", [(1, 0, 3), (2, 4, 7), (3, 2, 2 + 1)])
def test_zz_expectation(seed, i, j):
    c = random_circuit(8, 6, seed)
    psi = oracle.statevector(c)
    z = np.array([1.0 if not ((x >> i) & 1) ^ ((x >> j) & 1) else -1.0 for x in range(1 << 8)])
    want = float(np.sum(z * np.abs(psi) ** 2))
    vals = []
    for prune in (True, False):
        net = zz_network(c, i, j, prune=prune)
        plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
        vals.append(complex(oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree)))
    assert abs(vals[0] - want) < 1e-12 and abs(vals[1] - want) < 1e-12
    assert zz_network(c, i, j, True).num_tensors <= zz_network(c, i, j, False).num_tensors


def test_zz_closed_forms():
    for n in (4, 6):
        net = zz_network(ghz(n), 0, n - 1)
        plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
        assert abs(complex(oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree)) - 1) < 1e-14
        net = zz_network(hadamard_layer(n), 1, 2)
        plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
        assert abs(complex(oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree))) < 1e-14
