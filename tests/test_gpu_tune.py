"""GPU checks of the learned cost model's HIP kernels and of the tuners.

The MLP's FP32 gradient (hand-written HIP backward pass) is compared with
the FP64 reference network in oracle/mlp_ref.py; training must drive the
loss down; the exhaustive and model tuners must pick runnable plans whose
results match the oracle.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp_ref
from paper_2303_17510_amd import Plan, synth, tune

pytestmark = pytest.mark.gpu
NF, H = tune.NF, 64


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_setup(seed, n=257):
    """A network whose parameters are drawn here (numpy, seeded) and loaded
    into the library, so the reference sees only values this test made."""
    rng = np.random.default_rng(seed)
    shapes = [(NF, H), (H,), (H, H), (H,), (H, H), (H,), (H, 1), (1,)]
    parts = []
    for sh in shapes:
        fan = sh[0] if len(sh) == 2 else H
        parts.append(rng.uniform(-1, 1, size=sh).ravel() * math.sqrt(3.0 / fan))
    parts.append(rng.normal(size=NF))             # xmean
    parts.append(rng.uniform(0.5, 2, NF))         # xstd
    parts.append(np.array([0.4, 1.3]))            # ymean, ystd
    p = np.concatenate(parts).astype(np.float32)
    m = tune.CostModel(hidden=H, seed=seed)
    assert m.params().size == p.size
    m.load(p)
    X = rng.normal(size=(n, NF)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    return m, p.astype(np.float64), X, y


def test_mlp_gradient_matches_fp64_reference(gpu):
    m, p, X, y = random_setup(11)
    g_gpu, loss_gpu = m.grad(X, y)
    g_ref, nnet = mlp_ref.grad(p, X.astype(np.float64), y.astype(np.float64), NF, H)
    l_ref = mlp_ref.loss(p, X.astype(np.float64), y.astype(np.float64), NF, H)
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    say("gradient rel err %.2e, loss %.6f vs %.6f" % (rel, loss_gpu, l_ref))
    assert g_gpu.size == nnet
    assert rel < 1e-3
    assert abs(loss_gpu - l_ref) <= 1e-4 * max(1.0, l_ref)
    m.close()


def test_mlp_predict_matches_reference(gpu):
    m, p, X, y = random_setup(12, n=100)
    got = m.predict(X)
    ref = mlp_ref.predict_log_ms(p, X.astype(np.float64), NF, H)
    assert np.max(np.abs(got - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    m.close()


def test_mlp_training_fits_a_smooth_function(gpu):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(2000, NF)).astype(np.float32)
    w = rng.normal(size=NF)
    y = (np.tanh(X @ w / 6) + 0.1 * (X[:, 0] ** 2)).astype(np.float32)
    m = tune.CostModel(hidden=H, seed=5)
    before = float(np.mean((m.predict(X) - y) ** 2))
    loss = m.train(X, y, epochs=60, batch=128, lr=3e-3, seed=1)
    after = float(np.mean((m.predict(X) - y) ** 2))
    say("mse before %.4f after %.4f (normalised train loss %.4f)" % (before, after, loss))
    assert after < 0.05 * before and loss < 0.05
    m.close()


def test_exhaustive_tuner_picks_a_fast_correct_plan(gpu):
    import torch
    L = 30000
    xs = [synth.unit_disk((L,), 40 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((L,), (2 * L,), dtype="c64", tuner="exhaustive", tune_reps=3) as p:
        info = p.info()
        out = p(*dev)
        torch.cuda.synchronize()
    say("tuned", info["dims"][0]["variant"], info["dims"][0]["m"], info["tuned_ms"], info["timed_candidates"])
    assert info["tuner"] == "exhaustive" and info["timed_candidates"] == info["tuned_candidates"] > 1
    ref = oracle.conv_explicit([synth.as_oracle(x) for x in xs])
    assert oracle.rel_l2(out.cpu().numpy(), ref) < 1e-5
    # the chosen shape is at least as fast as the default within timing noise
    t_def = tune.time_shape((L,), (2 * L,), tune.candidates((L,), (2 * L,))[0][1], reps=5)
    assert info["tuned_ms"] <= 1.25 * t_def


def test_model_tuner_times_only_close_calls(gpu):
    import torch
    # a model trained on a few geometries' timings
    geoms = tune.geometries(12, 99, A_choices=(2,), mix=(1, 0, 0), l1=(1000, 200000))
    from paper_2303_17510_amd import costmodel
    data = costmodel.collect(geoms, reps=2)
    model, loss = costmodel.train(data, epochs=100, batch=64, lr=3e-3, seed=0)
    L = 50000
    xs = [synth.unit_disk((L,), 60 + a).astype(np.complex64) for a in range(2)]
    dev = [torch.from_numpy(x).cuda() for x in xs]
    with Plan((L,), (2 * L,), dtype="c64", tuner="model", model=model, margin=0.05) as p:
        info = p.info()
        out = p(*dev)
        torch.cuda.synchronize()
    say("model tuner: %d candidates, %d timed" % (info["tuned_candidates"], info["timed_candidates"]))
    assert info["tuner"] == "model" and info["timed_candidates"] < info["tuned_candidates"]
    ref = oracle.conv_explicit([synth.as_oracle(x) for x in xs])
    assert oracle.rel_l2(out.cpu().numpy(), ref) < 1e-5
    model.close()
