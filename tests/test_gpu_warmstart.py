"""Learned warm start (features, MFMA inference, training kernels, start
vector) against the FP64 references in oracle/mlp.py."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1709_07122_amd")

pytestmark = pytest.mark.gpu

# BF16 keeps 8 significant bits: unit roundoff u = 2^-9.  Along any path of
# the network a value meets at most 8 roundings (weights and activations of
# three layers, the features, the hidden outputs), so with ReLU 1-Lipschitz the
# error of the output is at most ((1+u)^8 - 1) times the same network evaluated
# on absolute values (|W|, |x|, |b|); FP32 accumulation adds ~1e-6 of that.
BF16_PATH_BOUND = (1 + 2.0 ** -9) ** 8 - 1 + 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def he_params(seed):
    return P.warmstart.init_params(seed).astype(np.float64)


def abs_network(p, X):
    w = mlp.unpack(p)
    a1 = np.abs(X) @ np.abs(w["W1"]).T + np.abs(w["b1"])
    a2 = a1 @ np.abs(w["W2"]).T + np.abs(w["b2"])
    return a2 @ np.abs(w["w3"]) + abs(w["b3"][0])


def exact_case(seed, b=256):
    """Parameters and inputs on which no rounding happens anywhere: small
    integer features and hidden units, weights in {0, +-1} (W2 with four
    nonzeros a row, w3 in {0, +-1/4}), a power-of-two batch and targets
    y + k/4.  Forward and gradient are then exact in BF16/FP32."""
    rng = np.random.default_rng(seed)
    w = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    w["W1"][:, :6] = rng.integers(-1, 2, (mlp.H, 6))
    w["b1"][:] = rng.integers(-2, 3, mlp.H)
    for i in range(mlp.H):
        w["W2"][i, rng.choice(mlp.H, 4, replace=False)] = rng.choice([-1.0, 1.0], 4)
    w["b2"][:] = rng.integers(-2, 3, mlp.H)
    w["w3"][:] = rng.integers(-1, 2, mlp.H) * 0.25
    w["b3"][0] = 0.5
    X = np.zeros((b, mlp.F))
    X[:, :6] = rng.integers(0, 4, (b, 6))
    p = mlp.pack(w)
    y, _ = mlp.forward(p, X)
    t = y + rng.integers(-2, 3, b) * 0.25
    return p, X, t


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_and_gradient_exact_where_nothing_rounds(seed):
    p, X, t = exact_case(seed)
    b = len(t)
    params, feat, tgt = dev(p.astype(np.float32)), dev(X.astype(np.float32)), dev(t.astype(np.float32))
    y = P.ws_forward(params, feat).cpu().numpy()
    yref, _ = mlp.forward(p, X)
    np.testing.assert_array_equal(y.astype(np.float64), yref)
    idx = dev(np.random.default_rng(seed).permutation(b).astype(np.int64))
    grad, loss = P.ws_backward(params, feat, tgt, idx)
    lref, gref = mlp.loss_and_grad(p, X, t)
    assert loss == lref
    g = grad.cpu().numpy().astype(np.float64)
    for name, (lo, hi) in _blocks().items():
        np.testing.assert_array_equal(g[lo:hi], gref[lo:hi], err_msg=name)
    assert np.abs(gref).max() > 0


def _blocks():
    out, o = {}, 0
    for name, shape in mlp.SIZES:
        size = int(np.prod(shape))
        out[name] = (o, o + size)
        o += size
    return out


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 70001])
def test_forward_within_bf16_bound(n):
    rng = np.random.default_rng(n)
    p = he_params(n % 7)
    w = mlp.unpack(p)
    w["b1"][:] = rng.normal(0, 0.3, mlp.H)
    w["b2"][:] = rng.normal(0, 0.3, mlp.H)
    w["b3"][0] = -1.0
    p = mlp.pack(w)
    X = np.zeros((n, mlp.F))
    X[:, :6] = rng.normal(0, 2, (n, 6))
    y = P.ws_forward(dev(p.astype(np.float32)), dev(X.astype(np.float32))).cpu().numpy().astype(np.float64)
    yref, _ = mlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    bound = BF16_PATH_BOUND * abs_network(p, X)
    err = np.abs(y - yref)
    assert np.all(err <= bound), (err / bound).max()
    # typical error is far below the worst case
    assert np.median(err / abs_network(p, X)) < 2e-3


def test_gradient_close_to_fp64_on_random_data():
    rng = np.random.default_rng(3)
    rows, b = 5000, 3000
    p = he_params(3)
    X = np.zeros((rows, mlp.F))
    X[:, :6] = rng.normal(0, 1.5, (rows, 6))
    t = rng.normal(0, 1, rows)
    idx = rng.choice(rows, b, replace=False)
    p32 = p.astype(np.float32)
    grad, loss = P.ws_backward(dev(p32), dev(X.astype(np.float32)), dev(t.astype(np.float32)), dev(idx.astype(np.int64)))
    lref, gref = mlp.loss_and_grad(p32.astype(np.float64), X[idx].astype(np.float32).astype(np.float64),
                                   t[idx].astype(np.float32).astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - lref) <= 2 * BF16_PATH_BOUND * lref
    for name, (lo, hi) in _blocks().items():
        rel = np.linalg.norm(g[lo:hi] - gref[lo:hi]) / np.linalg.norm(gref[lo:hi])
        assert rel < 0.02, (name, rel)
        cos = g[lo:hi] @ gref[lo:hi] / (np.linalg.norm(g[lo:hi]) * np.linalg.norm(gref[lo:hi]))
        assert cos > 0.999, (name, cos)


def test_gradient_is_deterministic_and_checks_indices():
    rng = np.random.default_rng(5)
    rows = 2000
    p = dev(P.warmstart.init_params(5))
    X = np.zeros((rows, mlp.F), np.float32)
    X[:, :6] = rng.normal(0, 1, (rows, 6))
    feat, tgt = dev(X), dev(rng.normal(0, 1, rows).astype(np.float32))
    idx = dev(rng.choice(rows, 1500).astype(np.int64))
    g1, l1 = P.ws_backward(p, feat, tgt, idx)
    g1 = g1.clone()
    g2, l2 = P.ws_backward(p, feat, tgt, idx)
    assert l1 == l2 and torch.equal(g1, g2)
    bad = idx.clone()
    bad[700] = rows
    with pytest.raises(P.PCPMError):
        P.ws_backward(p, feat, tgt, bad)
    bad[700] = -3
    with pytest.raises(P.PCPMError):
        P.ws_backward(p, feat, tgt, bad)


@pytest.mark.parametrize("step", [1, 7])
def test_adam_matches_oracle(step):
    rng = np.random.default_rng(step)
    n = P.WS_PARAMS
    p, g = rng.normal(0, 1, n), rng.normal(0, 1e-2, n)
    m, v = rng.normal(0, 1e-3, n), rng.uniform(0, 1e-4, n)
    if step == 1:
        m[:], v[:] = 0, 0
    p32, g32, m32, v32 = (a.astype(np.float32) for a in (p, g, m, v))
    tp, tm, tv = dev(p32), dev(m32), dev(v32)
    P.ws_adam(tp, dev(g32), tm, tv, step, 3e-3)
    rp, rm, rv = mlp.adam_step(*(a.astype(np.float64) for a in (p32, g32, m32, v32)), step, 3e-3)
    # FP32 moments: a few roundings relative to the size of the two terms
    # (the sum itself can cancel)
    u = 2.0 ** -24
    m64, v64, g64 = (a.astype(np.float64) for a in (m32, v32, g32))
    assert np.all(np.abs(tm.cpu().numpy() - rm) <= 4 * u * (0.9 * np.abs(m64) + 0.1 * np.abs(g64)))
    assert np.all(np.abs(tv.cpu().numpy() - rv) <= 4 * u * (0.999 * v64 + 0.001 * g64 * g64))
    # the update to 1e-4 of its size, plus the rounding of the stored weight
    upd = rp - p32
    assert np.all(np.abs(tp.cpu().numpy() - rp) <= 1e-4 * np.abs(upd) + np.spacing(np.abs(p32)))


def features_gpu(r, c, part_log2, d=0.85):
    png = P.build_png(dev(r), dev(c), part_log2=part_log2)
    f, ms = P.ws_features(png, d)
    f2, ms2 = P.ws_features(png, d)  # the graph sums are kept in the handle
    assert torch.equal(f, f2) and ms2 == ms
    out = f.cpu().numpy().astype(np.float64)
    png.close()
    return out


@pytest.mark.parametrize("scale,part_log2,relabel", [(12, 14, "random"), (14, 9, None), (15, 12, "random")])
def test_features_match_definitions(scale, part_log2, relabel):
    r, c = graphgen.rmat(scale, 16, seed=scale, relabel=relabel)
    got = features_gpu(r, c, part_log2)
    ref = mlp.features(r, c)
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=2e-6)


def test_features_of_a_small_hand_graph():
    # 0 -> 1, 0 -> 2, 1 -> 2, 2 -> 0, 3 -> 0 (3 has no in-edges), 4 dangling
    r = np.array([0, 2, 3, 4, 5, 5], np.int32)
    c = np.array([1, 2, 2, 0, 0], np.int32)
    got = features_gpu(r, c, 1, d=0.5)
    ref = mlp.features(r, c, d=0.5)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
    assert got[4, 2] == 1.0 and got[:4, 2].sum() == 0
    np.testing.assert_allclose(got[3], [0, np.log(2.0), 0, np.log(0.5 + 0.5 * 0.2), 0, 0, 0, 0], rtol=1e-6)
    # node 2: in-neighbours 0 (outdeg 2) and 1 (outdeg 1); 1/5 of the nodes dangle
    np.testing.assert_allclose(got[2, 3], np.log(0.5 + 0.5 * (0.5 + 1.0 + 0.2)), rtol=1e-6)


def test_features_need_a_single_graph():
    parts = [graphgen.rmat(8, 8, seed=s) for s in (1, 2)]
    row_off, col, offs, sizes = P.union_csr(parts, 8)
    png = P.build_png(dev(row_off), dev(col), part_log2=8, graph_node_off=offs, graph_nodes=sizes)
    with pytest.raises(P.PCPMError):
        P.ws_features(png)
    with pytest.raises(P.PCPMError):
        P.ws_predict(png, P.warmstart.load(P.warmstart.DEFAULT_WEIGHTS))
    png.close()


@pytest.mark.parametrize("scale,part_log2,d", [(10, 9, 0.85), (15, 14, 0.85), (13, 11, 0.5)])
def test_predict_equals_forward_of_the_features(scale, part_log2, d):
    """The fused prediction (features formed inside the forward kernel) is the
    forward pass of the feature matrix, bit for bit, on a fresh handle (the
    in-degree count runs inside it) and on a second call."""
    r, c = graphgen.rmat(scale, 16, seed=scale, relabel="random")
    params = P.warmstart.load(P.warmstart.DEFAULT_WEIGHTS)
    png = P.build_png(dev(r), dev(c), part_log2=part_log2)
    y1, _ = P.ws_predict(png, params, d)
    y2, _ = P.ws_predict(png, params, d)
    f, _ = P.ws_features(png, d)
    ref = P.ws_forward(params, f)
    assert torch.equal(y1, ref) and torch.equal(y2, ref)
    png.close()


def test_start_vector_is_softmax_and_falls_back():
    rng = np.random.default_rng(8)
    y = rng.normal(0, 3, 100003).astype(np.float32)
    pr0, fb = P.ws_init(dev(y))
    assert not fb
    e = np.exp(y.astype(np.float64) - y.max())
    np.testing.assert_allclose(pr0.cpu().numpy(), e / e.sum(), rtol=1e-5, atol=1e-12)
    for badv in (np.nan, np.inf, -np.inf):
        yb = y.copy()
        yb[777] = badv
        pr0, fb = P.ws_init(dev(yb))
        assert fb
        np.testing.assert_array_equal(pr0.cpu().numpy(), np.float32(1.0 / len(y)))


def test_targets_are_log_n_pr():
    pr = np.random.default_rng(9).dirichlet(np.ones(5000)).astype(np.float32)
    y = P.ws_targets(dev(pr)).cpu().numpy()
    np.testing.assert_allclose(y, np.log(pr.astype(np.float64) * 5000), rtol=1e-6, atol=1e-6)


def test_training_lowers_iterations_on_held_out_graphs():
    """Train on 16 small RMAT graphs, then solve two unseen ones from the
    predicted start: fewer iterations to the same FP64 residual, and a start
    vector closer (in L1) to the solution than the uniform one."""
    ws = P.warmstart
    specs = [ws.GraphSpec(int(s), 16, float(a), 300 + i)
             for i, (s, a) in enumerate(zip(np.tile([12, 13, 14, 13], 4), np.linspace(0.47, 0.63, 16)))]
    params, hist, info = ws.train(specs, epochs=40, batch=4096, lr=3e-3, log=None)
    assert hist[-1] < 0.5 * hist[0], hist
    for seed in (5000, 5001):
        r, c = graphgen.rmat(14, 16, seed=seed, relabel="random")
        png = P.build_png(dev(r), dev(c))
        pr0, fb = ws.warm_start(png, params)
        assert not fb
        cold = P.pagerank(png, tol=1e-6, max_iters=200)
        warm = P.pagerank(png, tol=1e-6, max_iters=200, init=pr0)
        assert cold.converged and warm.converged
        assert warm.iters < cold.iters, (warm.iters, cold.iters)
        star = oracle.pagerank(r, c, iters=200, tol=1e-12).x
        n = len(r) - 1
        e_warm = np.abs(pr0.cpu().numpy() - star).sum()
        e_cold = np.abs(1.0 / n - star).sum()
        assert e_warm < 0.5 * e_cold, (e_warm, e_cold)
        # the warm solve reaches the same fixed point: ||x - x*||_1 <= d res / (1 - d)
        # (plus FP32 rounding of the stored ranks)
        for res in (warm, cold):
            err = np.abs(res.pr.cpu().numpy().astype(np.float64) - star).sum()
            assert err <= 0.85 * res.resid / 0.15 + 1e-5, err
        png.close()
