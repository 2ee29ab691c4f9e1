"""Tensors of 2^32 entries: 64-bit indexing in the GEMM, permutation and
reduction kernels.

T1[a, x] T2[b, x] T3[a] T4[b] with |a| = |b| = 2^16, |x| = 16, contracted
along the tree ((T1, T2), T3), T4: the first vertex is a complex GEMM with a
2^32-entry result (M = N = 2^16, K = 16), which the second vertex permutes
into k-tiled planes (2^32 entries moved) and reads as the A operand of a GEMM
with K = 2^16.  The value does not depend on the tree, so the oracle
evaluates it along ((T1, T3), (T2, T4)), whose intermediates hold 16 entries.
Entries have real parts in [0.5, 1) and imaginary parts in [0, 0.1), so the
sums do not cancel and the FP32 bound is relative to the result.
"""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib

pytestmark = pytest.mark.gpu

A, X = 1 << 16, 16
LEGS = [[1, 3], [2, 3], [1], [2]]
DIMS = {1: A, 2: A, 3: X}


@pytest.fixture(scope="module")
def network():
    rng = np.random.default_rng(20)

    def t(*shape):
        return (rng.uniform(0.5, 1.0, shape) + 1j * rng.uniform(0.0, 0.1, shape)).astype(np.complex64)

    ts = [t(A, X), t(A, X), t(A), t(A)]
    ref = complex(oracle.contract_tree(LEGS, DIMS, [x.astype(np.complex128) for x in ts],
                                       [(0, 2), (1, 3), (4, 5)]))
    return ts, ref


@pytest.fixture(scope="module")
def ctx():
    import torch
    c = lib.Context(96 << 30)
    yield c
    c.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("flags,tol", [(lib.TN_PREC_FP32, 1e-4), (lib.TN_FORM_3M, 1e-4),
                                       (lib.TN_PREC_BF16X3, 1e-3),
                                       (lib.TN_PREC_BF16X3 | lib.TN_FORM_3M, 1e-3)])
def test_2pow32_entry_intermediate(ctx, network, flags, tol):
    ts, ref = network
    p = ctx.plan_load(LEGS, DIMS, ts, [0, 0, 0, 0], 1, [(0, 1), (4, 2), (5, 3)], None, flags, lib.TN_C64)
    c = lib.tn_plan_costs_get(p)
    assert c["largest_intermediate"] == 1 << 32 and c["num_gemm_nodes"] == 2
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    got, _ = lib.tn_contract(p)
    st = lib.tn_profile_read(ctx.handle, reset=True)
    lib.tn_profile_enable(ctx.handle, False)
    ctx.free_plan(p)
    # both GEMMs on the k-tiled matrix-core kernels; the 2^32-entry result
    # permuted into planes (16 bytes per entry or more)
    assert st["gemm"]["launches"] == 2
    assert st["permute"]["algo_bytes"] >= 16.0 * (1 << 32)
    err = abs(complex(got) - ref) / abs(ref)
    assert err < tol, (complex(got), ref, err)
