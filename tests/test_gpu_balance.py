"""Parity of the balance study (the sample-size and investigator ablation of
Section V: Table 2 and the sample-size figures) at a size the oracle runs in
seconds: 10^6 keys, P = 10 as in Table 2, each of the four input
distributions, each investigator mode, and the sample sizes 0.004X ... 1.4X
with X = 256 KB / P of keys.  Every output is compared with the oracle bit for
bit; the count-based investigator must also meet its balance bound."""
import numpy as np
import pytest

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import check_case

pytestmark = pytest.mark.gpu

N, P = 1_000_000, 10
X = 262144 // (P * 8)  # samples per block at the paper's budget, u64 keys
FACTORS = (0.004, 0.04, 0.4, 1.0, 1.004, 1.04, 1.4)


@pytest.fixture(scope="module")
def ws():
    return L.Workspace("cuda")


@pytest.fixture(scope="module")
def inputs():
    return {d: datagen.balance_keys(d, N) for d in datagen.BALANCE_DISTS}


@pytest.mark.parametrize("dist", datagen.BALANCE_DISTS)
@pytest.mark.parametrize("mode", [O.INV_COUNT, O.INV_NONE, O.INV_PAPER])
def test_table2_distributions(ws, inputs, dist, mode):
    keys = inputs[dist]
    vals = datagen.index_values(N) if mode == O.INV_COUNT else None
    r, o = check_case(keys, vals, P, X, mode, ws=ws)
    if mode == O.INV_COUNT:
        counts = o.part_counts.astype(np.float64)
        assert counts.max() <= N / P + (N / X) * (1 + 1 / P) + 2 * P + 3


@pytest.mark.parametrize("dist", ["uniform", "exponential"])
@pytest.mark.parametrize("f", FACTORS)
def test_sample_size_sweep(ws, inputs, dist, f):
    s = max(1, int(f * X))
    r, o = check_case(inputs[dist], None, P, s, O.INV_COUNT, ws=ws)
    counts = o.part_counts.astype(np.float64)
    assert counts.max() <= N / P + (N / s) * (1 + 1 / P) + 2 * P + 3


@pytest.mark.parametrize("P_", [10, 52])
def test_default_budget(ws, inputs, P_):
    """s = 0 takes the default budget on both sides (a multiple of P within
    256 KB over all processors)."""
    check_case(inputs["uniform"], None, P_, 0, O.INV_COUNT, ws=ws)
