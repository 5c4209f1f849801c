"""The GPU R-MAT generator against the host generator: the same CSR, bit for bit."""
import sys

import numpy as np
import pytest

from paper_2312_08140_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scale,ef,seed,weighted,abc", [
    (1, 1, 1, True, (0.57, 0.19, 0.19)),       # two vertices: at most one edge
    (6, 4, 3, True, (0.57, 0.19, 0.19)),
    (10, 8, 1, True, (0.57, 0.19, 0.19)),
    (12, 16, 2, False, (0.57, 0.19, 0.19)),
    (13, 16, 7, "ones", (0.25, 0.25, 0.25)),   # Erdos-Renyi-like quadrants
    (16, 16, 4, True, (0.57, 0.19, 0.19)),
    (19, 16, 100, True, (0.57, 0.19, 0.19)),
])
def test_device_rmat_equals_host(scale, ef, seed, weighted, abc):
    print(f"R-MAT scale {scale} ef {ef} seed {seed} weighted {weighted} abc {abc}", flush=True)
    sys.stdout.flush()
    h = gg.rmat(scale, ef, *abc, seed=seed, weighted=weighted)
    d = gg.rmat_device(scale, ef, *abc, seed=seed, weighted=weighted)
    assert d.n == h.n and d.m == h.m
    assert np.array_equal(d.offsets.cpu().numpy(), h.offsets)
    assert np.array_equal(d.indices.cpu().numpy(), h.indices)
    if h.weights is None:
        assert d.weights is None
    else:
        assert np.array_equal(d.weights.cpu().numpy(), h.weights)


def test_device_rmat_rejects_bad_parameters():
    with pytest.raises(RuntimeError):
        gg.rmat_device(0, 16)
    with pytest.raises(RuntimeError):
        gg.rmat_device(10, 16, 0.6, 0.3, 0.3)
