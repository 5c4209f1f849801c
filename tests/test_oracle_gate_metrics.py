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


def test_trace_weighted_by_hand():
    """Weighted triangle 0-1-2 (w01 = w02 = 1, w12 = 2) with a pendant 3 on 2
    (w23 = 1), id order, tau < 0, three sweeps.  K = (2, 3, 4, 1).
    Sweep 0: 0 ties {1:1, 2:1} and takes 1; 1 sees {1:1, 2:2} and takes 2;
    2 (marked by 0) sees {1:1, 2:2, 3:1} and keeps 2; 3 takes 2.  Flags left:
    0 (marked by 1) and 2 (marked by 3).  Sweep 1: 0 sees {2:2} and changes;
    its mark re-flags 1 before its turn, so 1 is re-processed in the same
    sweep and keeps 2; 2 keeps 2.  The features divide by the weighted degree
    K (not by deg): vertex 1's margin (2 - 1)/3 and vertex 2's W(own)/K = 2/4."""
    from oracle.gate_trace import lpa_trace
    from paper_2312_08140_amd import graphgen as gg
    g = gg.from_edges(4, [(0, 1), (0, 2), (1, 2), (2, 3)], [1, 1, 2, 1])
    r = lpa_trace(g, tau=-1.0, max_iters=3)
    assert list(r["labels"]) == [2, 2, 2, 2]
    assert list(r["changed"]) == [3, 1, 0]
    l3 = np.log2(3.0)
    expect = np.array([[l3, 0.0, 0.0, 1.0, 1 / 3, 0.5, 1.0, 0.125],          # vertex 0: changed 0 -> 1 at sweep 0
                       [l3, 1 / 3, 1 / 3, 1.0, 1 / 3, 2 / 3, 1.0, 0.125],    # vertex 1: {1:1, 2:2}, took 2
                       [2.0, 0.25, 0.5, 0.0, 1 / 3, 0.5, 1.0, 0.125]])       # vertex 2: {1:1, 2:2, 3:1}, kept 2
    assert np.allclose(r["X"], expect, atol=1e-15)
    assert list(r["y"]) == [1, 0, 0] and list(r["sweep"]) == [1, 1, 1]


# ---------------------------------------------------------------- gated-method oracle

def _x3_gate():
    """Parameters whose logit is x3 - 0.5 (x3 = changed at the last processing):
    with threshold 0.5 a flagged vertex is skipped iff it kept its label last time."""
    from oracle import mlp
    P = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    P["W1"][0, 3] = 1.0
    P["W2"][0, 0] = 1.0
    P["W3"][0, 0] = 1.0
    P["b3"][0] = -0.5
    return mlp.pack(P).astype(np.float32)


def test_gated_path_by_hand():
    """Path 0-1-2-3, unit weights, id order, gate 'skip if unchanged last time'.
    Sweep 0 (ungated): 0 takes 1; 1 ties {1, 2} and keeps 1; 2 ties {1, 3} and
    takes 1 (re-flagging 1 and 3); 3 (already flagged) takes 1 and re-flags 2.
    Flagged at sweep 1: 1 (kept its label: skipped, stays flagged) and 2
    (changed: processed, keeps 1).  dN = 0 stops the run; the verification
    sweep processes the still-flagged 1, which keeps 1."""
    from oracle.gate_trace import lpa_gated
    from paper_2312_08140_amd import graphgen as gg
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    r = lpa_gated(g, _x3_gate(), 0.5, tau=0.05, max_iters=20)
    assert list(r["labels"]) == [1, 1, 1, 1]
    assert list(r["changed"]) == [3, 0] and list(r["processed"]) == [4, 1] and list(r["gated"]) == [0, 1]
    assert list(r["scanned"]) == [6, 2]
    assert r["converged"] and r["verified"] and r["verify_changed"] == 0 and r["verify_scanned"] == 2
    assert r["margin"] == pytest.approx(0.5)


def _sbm_colour_order(seed, n=400):
    from paper_2312_08140_amd import graphgen as gg
    g = gg.sbm(n, 4, 0.08, 0.01, seed=seed, weighted=seed % 2 == 0)
    return g, oracle.color_order(*oracle.color(g, 0))


@pytest.mark.parametrize("seed", [1, 2])
def test_gated_threshold_zero_is_plain_plus_verification(seed):
    """Threshold 0 gates nothing: the main loop is the C oracle's run, and the
    verification sweep is one more pruned sweep resumed from its state."""
    from oracle.gate_trace import lpa_gated
    g, order = _sbm_colour_order(seed)
    theta = np.random.default_rng(seed).normal(0, 0.3, 1377).astype(np.float32)
    r = lpa_gated(g, theta, 0.0, order=order, tau=0.05, max_iters=20)
    ref = oracle.lpa(g, order=order, tau=0.05, max_iters=20)
    k = ref["iterations"]
    assert r["iterations"] >= k
    assert list(r["changed"][:k]) == list(ref["changed"]) and list(r["processed"][:k]) == list(ref["processed"])
    assert list(r["scanned"][:k]) == list(ref["scanned"]) and not r["gated"].any()
    v = oracle.lpa(g, order=order, tau=-1.0, max_iters=1, init_labels=ref["labels"], init_flags=ref["flags"])
    assert r["verify_changed"] >= v["changed"][0]
    if v["changed"][0] <= 0.05 * g.n:
        assert r["verified"] and r["iterations"] == k and np.array_equal(r["labels"], v["labels"])


@pytest.mark.parametrize("seed", [1, 2])
def test_gated_threshold_one_stalls_then_falls_back(seed):
    """Threshold 1 skips every re-processing: sweep 1 processes nothing and
    stops the run; the verification sweep and the plain fallback are the C
    oracle resumed from the state after sweep 0 (cap: max_iters more sweeps,
    counted with the verification sweep), then verification again."""
    from oracle.gate_trace import lpa_gated
    g, order = _sbm_colour_order(seed)
    theta = np.random.default_rng(seed).normal(0, 0.3, 1377).astype(np.float32)
    tau, it = 0.05, 20
    r = lpa_gated(g, theta, 1.0, order=order, tau=tau, max_iters=it)
    s0 = oracle.lpa(g, order=order, tau=-1.0, max_iters=1)
    assert r["changed"][0] == s0["changed"][0] and r["changed"][1] == 0 and r["processed"][1] == 0
    assert r["gated"][1] == int(s0["flags"].sum())
    v1 = oracle.lpa(g, order=order, tau=-1.0, max_iters=1, init_labels=s0["labels"], init_flags=s0["flags"])
    assert v1["changed"][0] > tau * g.n      # sweep 0 leaves much to do: the fallback runs
    fb = oracle.lpa(g, order=order, tau=tau, max_iters=min(it, 2 * it - 3), init_labels=v1["labels"],
                    init_flags=v1["flags"])
    v2 = oracle.lpa(g, order=order, tau=-1.0, max_iters=1, init_labels=fb["labels"], init_flags=fb["flags"])
    assert list(r["changed"][2:]) == list(fb["changed"])
    assert r["verify_changed"] == v1["changed"][0] + v2["changed"][0]
    assert np.array_equal(r["labels"], v2["labels"])
    assert r["verified"] == (v2["changed"][0] <= tau * g.n)
