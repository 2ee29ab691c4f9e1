"""GEMM epilogues that write the parent GEMM's operand planes (fused TTGT
permutation), on small networks built so that each configuration occurs:

  X(a, s) Y(s, b1, b2) -> P(a, b1, b2), a GEMM on k-tiled planes (K = |s|);
  P and Z(c, b2) -> the root, contracting b2; P is its A operand (tree
  (P, Z)) or its B operand (tree (Z, P)).

The producer P writes the root's planes; the root reads them as they are and
scales its result by the power of two instead.  Cases cover both operand
sides, tiles the producer fills only in part (|a| < the tile's rows, or |b1
b2| < its columns), one-bit and multi-bit contracted legs (the former let the
planner move row legs into the low result bits), a producer shared by every
query of a batch (its planes read with batch stride 0) and one computed per
query, in FP32 (4M, 3M) and BF16x3 (4M: four planes; 3M: six).  The CPU
test checks the plan decisions; the GPU tests check fused against unfused
results bit for bit and against the oracle's complex128 contraction of the
same tree.
"""
import math
import re

import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib

# name: (bits of a, of b1, of s, of b2, of c, side, b2 as one-bit legs)
CASES = {
    "b_side": (6, 6, 4, 5, 4, "B", True),
    "a_side": (6, 6, 4, 5, 4, "A", True),
    "b_side_multibit": (6, 6, 4, 5, 4, "B", False),
    "partial_rows": (5, 7, 4, 4, 5, "B", True),
    "partial_cols": (9, 1, 5, 4, 4, "A", True),
}


def _case(name, seed=0):
    """legs, dims, tensors, tree, output legs of a case; leaf 0 = X, 1 = Y,
    2 = Z; vertex 3 = P."""
    ab, b1b, sb, b2b, cb, side, onebit = CASES[name]
    dims = {}
    lab = [100]

    def leg(bits):
        lab[0] += 1
        dims[lab[0]] = 2 ** bits
        return lab[0]

    a, b1, c = leg(ab), leg(b1b), leg(cb)
    s = [leg(1) for _ in range(sb)]
    b2 = [leg(1) for _ in range(b2b)] if onebit else [leg(b2b)]
    legs = [[a] + s, s + [b1] + b2, [c] + b2]
    rng = np.random.default_rng(seed)
    ts = [rng.standard_normal(tuple(dims[x] for x in l)) + 1j * rng.standard_normal(tuple(dims[x] for x in l))
          for l in legs]
    tree = [(0, 1), (3, 2)] if side == "A" else [(0, 1), (2, 3)]
    return legs, dims, ts, tree, [a, b1, c]


def _load(ctx, name, flags, ts=None):
    legs, dims, ts0, tree, out = _case(name)
    return (lib.tn_plan_load(ctx, legs, dims, ts if ts is not None else ts0, [0, 0, 0], 1, tree, out, flags),
            legs, dims, ts0, tree, out)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("flags", [lib.TN_PREC_FP32, lib.TN_PREC_FP32 | lib.TN_FORM_3M, lib.TN_PREC_BF16X3,
                                   lib.TN_PREC_BF16X3 | lib.TN_FORM_3M])
def test_fusion_in_plan(name, flags, monkeypatch, capfd):
    """The producer writes planes, the root reads the designed operand raw,
    one permutation fewer than with TN_GEMM_FUSE=0."""
    side = CASES[name][5]
    monkeypatch.setenv("TN_DEBUG", "1")
    p = _load(None, name, flags)[0]
    fused = lib.tn_plan_costs_get(p)["num_permutations"]
    lib.tn_plan_free(p)
    err = capfd.readouterr().err
    assert re.search(r"gemm vertex 3: .* fused 00 writes 1", err), err
    assert re.search(r"gemm vertex 4: .* fused %s writes 0" % ("10" if side == "A" else "01"), err), err
    monkeypatch.setenv("TN_GEMM_FUSE", "0")
    p = _load(None, name, flags)[0]
    plain = lib.tn_plan_costs_get(p)["num_permutations"]
    lib.tn_plan_free(p)
    assert plain == fused + 1


def _tol(flags, p):
    if flags & lib.TN_PREC_BF16X3:
        return 1e-3
    return 64 * 2.0 ** -24 * math.sqrt(max(lib.tn_plan_costs_get(p)["con_serial"], 1))


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(4 << 30)
    yield c
    c.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("flags", [lib.TN_PREC_FP32, lib.TN_PREC_FP32 | lib.TN_FORM_3M, lib.TN_PREC_BF16X3,
                                   lib.TN_PREC_BF16X3 | lib.TN_FORM_3M])
def test_fused_single(ctx, name, flags, monkeypatch):
    """One query: fused and unfused bits agree, and both match the oracle."""
    got = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("TN_GEMM_FUSE", fuse)
        p, legs, dims, ts, tree, out = _load(ctx.handle, name, flags)
        shape = tuple(dims[x] for x in out)
        got[fuse] = lib.tn_contract(p, result_shape=shape)[0]
        tol = _tol(flags, p)
        lib.tn_plan_free(p)
    assert np.array_equal(got["0"].view(np.uint64), got["1"].view(np.uint64))
    ref = oracle.contract_tree(legs, dims, ts, tree, out)
    assert np.max(np.abs(got["1"] - ref)) / np.max(np.abs(ref)) < tol


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["b_side", "a_side", "partial_rows"])
@pytest.mark.parametrize("flags", [lib.TN_PREC_FP32, lib.TN_PREC_BF16X3, lib.TN_PREC_BF16X3 | lib.TN_FORM_3M])
@pytest.mark.parametrize("leaf", [2, 0])
def test_fused_batch(ctx, name, flags, leaf, monkeypatch):
    """Four queries in one batch, each overriding leaf Z (the producer P is
    then shared: computed once, its planes read by every query at stride 0)
    or leaf X (P per query): fused and unfused bits agree, and every result
    matches the oracle."""
    legs, dims, ts, tree, out = _case(name)
    shape = tuple(dims[x] for x in out)
    rng = np.random.default_rng(7)
    ovrs = []
    for _ in range(4):
        t = ts[leaf]
        ovrs.append({leaf: rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape)})
    got = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("TN_GEMM_FUSE", fuse)
        p = lib.tn_plan_load(ctx.handle, legs, dims, ts, [0, 0, 0], 1, tree, out, flags)
        res, _, st = lib.tn_contract_batch(ctx.handle, [(p, o) for o in ovrs], [shape] * len(ovrs))
        assert all(s == 0 for s in st)
        got[fuse] = np.stack(res)
        tol = _tol(flags, p)
        lib.tn_plan_free(p)
    assert np.array_equal(got["0"].view(np.uint64), got["1"].view(np.uint64))
    for q, o in enumerate(ovrs):
        tq = list(ts)
        tq[leaf] = o[leaf]
        ref = oracle.contract_tree(legs, dims, tq, tree, out)
        assert np.max(np.abs(got["1"][q] - ref)) / np.max(np.abs(ref)) < tol


@pytest.mark.parametrize("flags", [lib.TN_PREC_FP32, lib.TN_PREC_BF16X3])
def test_no_fusion_past_2pow29_entries(flags, monkeypatch, capfd):
    """T1[a, x] T2[b, x] T3[a] T4[b] with |a| = |b| = 2^16, |x| = 16 along
    ((T1, T2), T3), T4: the first GEMM's result (2^32 entries) is too large for
    32-bit plane offsets, so its parent permutes it instead of reading planes
    the first GEMM writes."""
    a, x = 1 << 16, 16
    legs = [[1, 3], [2, 3], [1], [2]]
    dims = {1: a, 2: a, 3: x}
    ts = [np.ones((a, x), np.complex64), np.ones((a, x), np.complex64), np.ones(a, np.complex64),
          np.ones(a, np.complex64)]
    monkeypatch.setenv("TN_DEBUG", "1")
    p = lib.tn_plan_load(None, legs, dims, ts, [0, 0, 0, 0], 1, [(0, 1), (4, 2), (5, 3)], None, flags,
                         lib.TN_C64)
    lib.tn_plan_free(p)
    err = capfd.readouterr().err
    assert re.search(r"gemm vertex 4: M 65536 N 65536 K 16 .* fused 00 writes 0", err), err
    assert re.search(r"gemm vertex 5: .* perm 1. .* fused 00 writes 0", err), err
