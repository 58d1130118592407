"""Pin of the FP64 reference network: its analytic gradient against central
finite differences of its loss, and its forward pass against a plain loop."""
import numpy as np

from oracle import mlp_ref

NF, H = 44, 8


def random_params(seed):
    rng = np.random.default_rng(seed)
    n = NF * H + H + 2 * (H * H + H) + H + 1
    net = rng.normal(scale=0.3, size=n)
    xmean = rng.normal(size=NF)
    xstd = rng.uniform(0.5, 2.0, size=NF)
    return np.concatenate([net, xmean, xstd, [0.3, 1.7]])


def test_gradient_matches_central_differences():
    p = random_params(1)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(23, NF))
    y = rng.normal(size=23)
    g, nnet = mlp_ref.grad(p, X, y, NF, H)
    assert g.size == nnet
    eps = 1e-6
    idx = np.random.default_rng(3).choice(nnet, size=60, replace=False)
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = mlp_ref.loss(q, X, y, NF, H)
        q[i] -= 2 * eps
        lm = mlp_ref.loss(q, X, y, NF, H)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_matches_plain_loops():
    p = random_params(4)
    X = np.random.default_rng(5).normal(size=(3, NF))
    W, (xm, xs, ym, ys), _ = mlp_ref.unpack(p, NF, H)
    for r in range(3):
        a = [(X[r, k] - xm[k]) / xs[k] for k in range(NF)]
        for l in range(4):
            I, O = len(a), W[2 * l].shape[1]
            z = [W[2 * l + 1][o] + sum(a[k] * W[2 * l][k, o] for k in range(I)) for o in range(O)]
            a = [v / (1 + np.exp(-v)) for v in z] if l < 3 else z
        got = mlp_ref.predict_log_ms(p, X[r:r + 1], NF, H)[0]
        assert abs(got - (a[0] * ys + ym)) < 1e-12
