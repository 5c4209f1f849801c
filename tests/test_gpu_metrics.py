"""GPU normalised mutual information (lpa_nmi) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2312_08140_amd import abi, graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ka,kb,seed", [(1, 1, 1, 0), (2, 2, 1, 1), (1000, 10, 7, 2), (100_000, 300, 50, 3),
                                          (2_000_000, 5000, 1000, 4)])
def test_nmi_matches_oracle(n, ka, kb, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, ka, n).astype(np.int32)
    # b: a noisy copy of a, so the two share information
    b = np.where(rng.uniform(size=n) < 0.7, a % kb, rng.integers(0, kb, n)).astype(np.int32)
    got = abi.nmi(a, b)
    ref = oracle.nmi(a, b)
    assert abs(got - ref) <= 1e-10, (got, ref)


def test_nmi_identities():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 100, 50_000).astype(np.int32)
    perm = rng.permutation(100).astype(np.int32)
    assert abs(abi.nmi(a, a) - 1.0) <= 1e-12
    assert abs(abi.nmi(a, perm[a]) - 1.0) <= 1e-12          # relabelling does not matter
    one = np.zeros_like(a)
    assert abi.nmi(one, one) == 1.0                         # two single-class partitions
    assert abi.nmi(a, one) == 0.0                           # one side carries no information
    neg = np.array([-5, -5, 7, 7, -2147483648, 2147483647], np.int32)  # any int32 values
    assert abs(abi.nmi(neg, neg) - 1.0) <= 1e-12
    assert abi.nmi(np.zeros(0, np.int32), np.zeros(0, np.int32)) == 1.0


def test_nmi_of_lpa_result_vs_planted_partition():
    import torch
    g = gg.sbm(200_000, 200, 32 * 0.8 / 999, 32 * 0.2 / (200_000 - 1000), seed=5)
    G = abi.LPAGraph(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    G.run(0.05, 20, abi.LPA_MODE_ASYNC, True, labels_out=out)
    truth = gg.sbm_truth(g.n, 200)
    dev = abi.nmi(out, torch.from_numpy(truth.astype(np.int32)).cuda())
    ref = oracle.nmi(out.cpu().numpy(), truth)
    assert abs(dev - ref) <= 1e-10
    G.close()
