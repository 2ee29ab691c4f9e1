"""Slicing (fixing legs, contracting each slice, adding the slices): host-side
pins against the oracle.  A contraction sums over every bound index, so the
sum over a leg's values of the contractions with that leg fixed is the
contraction itself."""
import numpy as np

import oracle
from paper_2507_20667_amd.inputs import amplitude_network, random_circuit
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.cost import largest_intermediate
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.slicing import choose_slices, largest_after, sliced_problem


def _setup(n=16, d=10, seed=3):
    circ = random_circuit(n, d, seed)
    net = amplitude_network(circ, 5)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 2), 2,
                               SAConfig(iterations=3, n_steps=16, workers=2, rg_samples=4, seed=seed))
    return circ, net, plan


def test_choose_slices_meets_target():
    circ, net, plan = _setup()
    top = largest_intermediate(net.legs, net.dims, plan.tree)
    target = top // 4
    sl = choose_slices(net.legs, net.dims, plan.tree, target)
    assert sl and len(set(sl)) == len(sl)
    assert largest_after(net.legs, net.dims, plan.tree, sl) <= target
    assert largest_after(net.legs, net.dims, plan.tree, []) == top


def test_sum_of_slices_is_the_contraction():
    circ, net, plan = _setup()
    ref = complex(oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree))
    sl = choose_slices(net.legs, net.dims, plan.tree, max(largest_intermediate(net.legs, net.dims, plan.tree) // 8, 2))
    d, base, ovrs = sliced_problem(net.legs, net.dims, net.tensors, sl)
    assert len(ovrs) == 2 ** len(sl)
    total = 0j
    for o in ovrs:
        ts = list(base)
        for t, v in o.items():
            ts[t] = v
        total += complex(oracle.contract_tree(net.legs, d, ts, plan.tree))
    assert abs(total - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-15
    # and one slice alone is not the whole (the slicing is real)
    one = list(base)
    assert abs(complex(oracle.contract_tree(net.legs, d, one, plan.tree)) - ref) > 1e-6 * abs(ref)


def test_library_slice_choice_matches_planner():
    """tn_plan_slice on a host-only plan chooses legs by the same greedy rule
    as choose_slices: the sliced plan's largest intermediate and con_serial
    are those of the network with choose_slices' legs at dimension 1; with
    the legs given explicitly the same sliced network results."""
    from paper_2507_20667_amd import lib
    from paper_2507_20667_amd.planner import cost
    for seed, div in ((3, 4), (4, 8), (6, 16)):
        circ, net, plan = _setup(seed=seed)
        top = largest_intermediate(net.legs, net.dims, plan.tree)
        target = max(top // div, 2)
        sl = choose_slices(net.legs, net.dims, plan.tree, target, max_legs=30)
        d = dict(net.dims)
        for l in sl:
            d[l] = 1
        p = lib.tn_plan_load(None, net.legs, net.dims, net.tensors, plan.partition_of, 2, plan.tree)
        for s in (lib.tn_plan_slice(p, (), target), lib.tn_plan_slice(p, sl)):
            c = lib.tn_plan_costs_get(s)
            assert c["largest_intermediate"] == largest_after(net.legs, net.dims, plan.tree, sl) <= target
            assert c["con_serial"] == cost.con_serial(net.legs, d, plan.tree)
            lib.tn_plan_free(s)
        # a leg that is not bound is refused
        open_like = max(max(l) for l in net.legs) + 1
        import pytest
        with pytest.raises(lib.TnError):
            lib.tn_plan_slice(p, [open_like])
        lib.tn_plan_free(p)
