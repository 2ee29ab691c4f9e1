"""Pins of the oracle's loop-nest contractor (oracle_contract_tree).

  * the full contraction as its definition (a sum over every assignment of
    every bound edge of the product of entries, Section 2.2), both as the
    oracle's brute-force routine and as numpy.einsum over the whole network;
  * tree independence (Section 2.3: the result does not depend on the order of
    the pairwise contractions): two unrelated trees agree;
  * hand-worked networks: a ring is the trace of a matrix product, a chain a
    vector-matrix-vector product (numpy matmul);
  * degenerate inputs: a single tensor, scalars (degree-0 tensors are allowed,
    Section 2.1), dimension-1 legs, outer products of disconnected parts.
"""
import json
import os
import string

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cost_worked_examples.json")


def random_network(rng, nv, max_bound=10, max_open=3, dim_choices=(1, 2, 3)):
    """Random labelled-leg network: bound labels join two distinct tensors,
    open labels sit on one tensor."""
    legs = [[] for _ in range(nv)]
    dims = {}
    lab = 0
    nb = int(rng.integers(nv - 1, max_bound + 1))
    # a spanning chain keeps most cases connected, then extra random edges
    for e in range(nb):
        if e < nv - 1:
            u, v = e, e + 1
        else:
            u, v = rng.choice(nv, size=2, replace=False)
        legs[int(u)].append(lab)
        legs[int(v)].append(lab)
        dims[lab] = int(rng.choice(dim_choices))
        lab += 1
    opens = []
    for _ in range(int(rng.integers(0, max_open + 1))):
        u = int(rng.integers(0, nv))
        legs[u].append(lab)
        dims[lab] = int(rng.choice(dim_choices))
        opens.append(lab)
        lab += 1
    for l in legs:
        rng.shuffle(l)
    tensors = []
    for l in legs:
        shape = tuple(dims[x] for x in l)
        tensors.append(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    rng.shuffle(opens)
    return legs, dims, tensors, opens


def random_tree(rng, nv):
    alive = list(range(nv))
    tree = []
    nxt = nv
    while len(alive) > 1:
        i, j = rng.choice(len(alive), size=2, replace=False)
        a, b = alive[i], alive[j]
        tree.append((a, b))
        alive = [x for x in alive if x not in (a, b)] + [nxt]
        nxt += 1
    return tree


def einsum_reference(legs, dims, tensors, opens):
    letters = {}
    pool = iter(string.ascii_letters)
    for l in legs:
        for x in l:
            if x not in letters:
                letters[x] = next(pool)
    sub = ",".join("".join(letters[x] for x in l) for l in legs)
    sub += "->" + "".join(letters[x] for x in opens)
    return np.einsum(sub, *tensors, optimize=False)


@pytest.mark.parametrize("seed", range(12))
def test_loop_nest_matches_definition(seed):
    rng = np.random.default_rng(100 + seed)
    nv = int(rng.integers(2, 7))
    legs, dims, tensors, opens = random_network(rng, nv)
    ref = oracle.brute_force(legs, dims, tensors, opens)
    ein = einsum_reference(legs, dims, tensors, opens)
    t1 = oracle.contract_tree(legs, dims, tensors, random_tree(rng, nv), opens, nthreads=2)
    t2 = oracle.contract_tree(legs, dims, tensors, oracle.sequential_tree(nv), opens, nthreads=1)
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.allclose(ein, ref, rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(t1, ref, rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(t2, ref, rtol=1e-12, atol=1e-12 * scale)


def test_ring_is_trace_and_chain_is_matrix_product():
    gold = json.load(open(GOLD))
    rng = np.random.default_rng(7)
    for ex in gold["examples"]:
        names = sorted(ex["dims"])
        lab = {n: i for i, n in enumerate(names)}
        legs = [[lab[x] for x in l] for l in ex["legs"]]
        dims = {lab[k]: v for k, v in ex["dims"].items()}
        tensors = [rng.standard_normal(tuple(dims[x] for x in l))
                   + 1j * rng.standard_normal(tuple(dims[x] for x in l)) for l in legs]
        got = oracle.contract_tree(legs, dims, tensors, [tuple(p) for p in ex["tree"]])
        if ex["name"].startswith("W1"):
            want = np.trace(tensors[0] @ tensors[1] @ tensors[2] @ tensors[3])
        else:
            want = tensors[0] @ tensors[1] @ tensors[2] @ tensors[3] @ tensors[4]
        assert abs(complex(got) - complex(want)) <= 1e-12 * max(1.0, abs(want))


def test_degenerate_networks():
    rng = np.random.default_rng(3)
    # single tensor with open legs, returned in a permuted order
    t = rng.standard_normal((2, 3, 4)) + 0j
    got = oracle.contract_tree([[0, 1, 2]], {0: 2, 1: 3, 2: 4}, [t], [], output_legs=[2, 0, 1])
    assert np.array_equal(got, np.transpose(t, (2, 0, 1)))
    # scalars: degree-0 tensors multiply
    a, b = np.array(2.0 + 1j), np.array(-3.0 + 0.5j)
    got = oracle.contract_tree([[], []], {}, [a, b], [(0, 1)])
    assert complex(got) == complex(a * b)
    # disconnected parts: outer product
    u = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    got = oracle.contract_tree([[0], [1]], {0: 3, 1: 2}, [u, v], [(0, 1)], output_legs=[0, 1])
    assert np.allclose(got, np.outer(u, v), rtol=1e-15, atol=0)
    # dimension-1 legs
    x = rng.standard_normal((1, 2)) + 0j
    y = rng.standard_normal((2, 1)) + 0j
    got = oracle.contract_tree([[0, 1], [1, 2]], {0: 1, 1: 2, 2: 1}, [x, y], [(0, 1)],
                               output_legs=[0, 2])
    assert np.allclose(got, x @ y, rtol=1e-15, atol=0)


def test_malformed_tree_is_rejected():
    t = np.ones(2, dtype=np.complex128)
    with pytest.raises(RuntimeError):
        oracle.contract_tree([[0], [0]], {0: 2}, [t, t], [(0, 0)])
    with pytest.raises(RuntimeError):
        oracle.contract_tree([[0], [0]], {0: 2}, [t, t], [(0, 5)])
