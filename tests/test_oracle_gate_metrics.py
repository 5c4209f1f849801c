"""Pins of the FP64 gate-network oracle and the NMI oracle (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def _theta(seed, scale=0.5):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAMS)


def test_param_count():
    assert mlp.NPARAMS == 1377  # 8*32+32 + 32*32+32 + 32+1


@pytest.mark.parametrize("pw", [1.0, 3.5])
def test_gradient_matches_central_differences(pw):
    rng = np.random.default_rng(0)
    th = _theta(1)
    x = rng.normal(0, 1, (16, 8))
    y = (rng.random(16) < 0.4).astype(np.float64)
    g = mlp.backward(th, x, y, pw)
    h = 1e-6
    num = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        num[i] = (mlp.loss(th + e, x, y, pw) - mlp.loss(th - e, x, y, pw)) / (2 * h)
    # units on the ReLU kinks are measure-zero for Gaussian inputs
    assert np.linalg.norm(g - num) <= 1e-6 * max(1.0, np.linalg.norm(num))


def test_zero_weights_closed_form():
    """All weights and hidden biases zero: p = sigmoid(b3) for every input and
    dL/db3 = mean(p - y) (pw = 1); every other gradient is zero."""
    th = np.zeros(mlp.NPARAMS)
    th[-1] = 0.3
    x = np.random.default_rng(2).normal(0, 1, (10, 8))
    y = np.array([1, 0, 1, 1, 0, 0, 0, 1, 0, 1], np.float64)
    p, _ = mlp.forward(th, x)
    s = 1 / (1 + np.exp(-0.3))
    assert np.allclose(p, s, rtol=0, atol=1e-15)
    g = mlp.backward(th, x, y)
    assert g[-1] == pytest.approx(np.mean(s - y), abs=1e-15)
    assert np.all(g[:-1] == 0)


def test_forward_matches_torch_float64():
    import torch
    th = _theta(3)
    P = mlp.unpack(th)
    x = np.random.default_rng(4).normal(0, 1, (32, 8))
    net = torch.nn.Sequential(torch.nn.Linear(8, 32), torch.nn.ReLU(), torch.nn.Linear(32, 32), torch.nn.ReLU(),
                              torch.nn.Linear(32, 1)).double()
    with torch.no_grad():
        for lin, (w, b) in zip([net[0], net[2], net[4]], [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            lin.weight.copy_(torch.from_numpy(P[w]))
            lin.bias.copy_(torch.from_numpy(P[b]))
    xt = torch.from_numpy(x)
    yt = torch.from_numpy((np.arange(32) % 3 == 0).astype(np.float64))
    z = net(xt)[:, 0]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z, yt, pos_weight=torch.tensor(2.0, dtype=torch.float64))
    lt.backward()
    p, _ = mlp.forward(th, x)
    assert np.allclose(p, torch.sigmoid(z).detach().numpy(), rtol=1e-13, atol=1e-15)
    assert mlp.loss(th, x, yt.numpy(), 2.0) == pytest.approx(lt.item(), rel=1e-13)
    gt = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(), net[2].weight.grad.numpy().ravel(),
                         net[2].bias.grad.numpy(), net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
    assert np.allclose(mlp.backward(th, x, yt.numpy(), 2.0), gt, rtol=1e-11, atol=1e-14)


def test_adam_matches_torch():
    import torch
    th = _theta(5)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    t_param = torch.nn.Parameter(torch.from_numpy(th.copy()))
    opt = torch.optim.Adam([t_param], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(6)
    for t in range(1, 6):
        g = rng.normal(0, 1, th.size)
        th, m, v = mlp.adam_step(th, g, m, v, t)
        t_param.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.allclose(th, t_param.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_round_matches_torch():
    import torch
    x = np.concatenate([np.random.default_rng(7).normal(0, 3, 10000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, 1e-40], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)


# ---------------------------------------------------------------- NMI

def test_nmi_identities():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 7, 500)
    assert oracle.nmi(x, x) == pytest.approx(1.0, abs=1e-15)
    perm = rng.permutation(7) + 100
    assert oracle.nmi(x, perm[x]) == pytest.approx(1.0, abs=1e-15)
    assert oracle.nmi(np.zeros(10), np.zeros(10)) == 1.0


def test_nmi_against_singletons_closed_form():
    """Against all-singletons, I(X;Y) = H(X) and H(Y) = ln n, so
    NMI = 2 H(X) / (H(X) + ln n)."""
    x = np.repeat(np.arange(5), [1, 2, 3, 4, 10])
    n = x.size
    p = np.bincount(x) / n
    hx = -(p * np.log(p)).sum()
    assert oracle.nmi(x, np.arange(n)) == pytest.approx(2 * hx / (hx + np.log(n)), abs=1e-14)


def test_nmi_matches_sklearn():
    from sklearn.metrics import normalized_mutual_info_score
    rng = np.random.default_rng(1)
    for _ in range(5):
        x = rng.integers(0, 20, 2000)
        y = np.where(rng.random(2000) < 0.7, x, rng.integers(0, 30, 2000))
        assert oracle.nmi(x, y) == pytest.approx(normalized_mutual_info_score(x, y, average_method="arithmetic"),
                                                 abs=1e-12)


# ---------------------------------------------------------------- gate trace oracle

def test_trace_triangle_by_hand():
    """K3, id order, tau < 0: sweep 0 changes vertices 0 and 2 (to label 1);
    sweep 1 re-processes 0 and 1 (flagged by 2's change) and nothing changes."""
    from oracle.gate_trace import lpa_trace
    from paper_2312_08140_amd import graphgen as gg
    g = gg.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    r = lpa_trace(g, tau=-1.0, max_iters=3)
    assert list(r["labels"]) == [1, 1, 1]
    assert list(r["changed"]) == [2, 0, 0]
    l3 = np.log2(3.0)
    expect = np.array([[l3, 0.0, 0.0, 1.0, 1 / 3, 0.5, 1.0, 0.125],    # vertex 0: tie {1:1, 2:1}, changed 0 -> 1
                       [l3, 0.0, 0.5, 0.0, 1 / 3, 0.5, 1.0, 0.125]])   # vertex 1: tie, kept its own label 1
    assert np.allclose(r["X"], expect, atol=1e-15)
    assert list(r["y"]) == [0, 0] and list(r["sweep"]) == [1, 1]


@pytest.mark.parametrize("seed", [1, 2])
def test_trace_lpa_equals_c_oracle(seed):
    """The trace oracle's label process is the C oracle's, sweep for sweep, and
    its samples count exactly the re-processings (y = the changes among them)."""
    import oracle
    from oracle.gate_trace import lpa_trace
    from paper_2312_08140_amd import graphgen as gg
    g = gg.sbm(400, 4, 0.08, 0.01, seed=seed)
    order = oracle.color_order(*oracle.color(g, 0))
    ref = oracle.lpa(g, order=order, tau=0.0, max_iters=12)
    r = lpa_trace(g, order=order, tau=0.0, max_iters=12)
    assert np.array_equal(r["labels"], ref["labels"])
    assert np.array_equal(r["changed"], ref["changed"][:ref["iterations"]])
    iso = np.diff(np.asarray(g.offsets)) == 0
    for s in range(1, r["iterations"]):
        sel = r["sweep"] == s
        assert sel.sum() == ref["processed"][s]          # every vertex was processed in sweep 0
        assert r["y"][sel].sum() == ref["changed"][s]
    X = r["X"]
    assert np.all((X[:, 1:] >= 0) & (X[:, 1:] <= 1)) and not iso.all()
    assert np.all(X[:, 5] >= X[:, 1]) and np.all(X[:, 5] >= X[:, 2])  # W1 bounds W1 - W2 and W(own)
