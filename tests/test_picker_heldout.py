"""Regret of the shipped picker on the stored held-out timings (CPU).

trained/heldout.npz holds the autotuner's timings of every candidate plan of
500 held-out geometries (seed 17510501 of the cost-model workload), written
by ``python -m paper_2303_17510_amd.costmodel collect``; trained/heldout3.npz
re-times the 2D/3D ones it reached on the current kernels (its rows replace
theirs); trained/picker_mlp.f32 is the network trained on 2000 other
geometries.  The shipped network is
evaluated here in FP64 with NumPy (the documented layout: normalised inputs,
three SiLU layers, linear output); the pick is the argmin of the predicted
log times, its regret t(pick)/t(best) - 1 against the timed exhaustive best;
the library's tuner decides per dimension, which is checked as well.  The
target is a geometric-mean regret within 5 %.
"""
import json
import math
import os

import numpy as np


HERE = os.path.dirname(os.path.abspath(__file__))
TRAINED = os.path.join(HERE, "..", "paper_2303_17510_amd", "trained")


def _model():
    with open(os.path.join(TRAINED, "picker_mlp.f32.json")) as fh:
        hdr = json.load(fh)
    p = np.fromfile(os.path.join(TRAINED, "picker_mlp.f32"), dtype="<f4").astype(np.float64)
    assert p.size == hdr["nparams"]
    return p, hdr


def _predict(p, X, nf, h):
    shapes = [(nf, h), (h,), (h, h), (h,), (h, h), (h,), (h, 1), (1,)]
    W, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        W.append(p[o:o + k].reshape(sh))
        o += k
    xm, xs = p[o:o + nf], p[o + nf:o + 2 * nf]
    ym, ys = p[o + 2 * nf], p[o + 2 * nf + 1]
    a = (X - xm) / xs
    for l in range(4):
        z = a @ W[2 * l] + W[2 * l + 1]
        a = z / (1.0 + np.exp(-z)) if l < 3 else z
    return a[:, 0] * ys + ym


def _load(names):
    # re-collected geometries (the later file) replace their older timings
    parts = [dict(np.load(os.path.join(TRAINED, n), allow_pickle=False)) for n in names]
    seen = set()
    for i in range(len(parts) - 1, -1, -1):
        keep = ~np.isin(parts[i]["gid"], np.array(sorted(seen), dtype=np.int64))
        seen.update(int(g) for g in np.unique(parts[i]["gid"]))
        parts[i] = {k: v[keep] for k, v in parts[i].items()}
    return {k: np.concatenate([q[k] for q in parts]) for k in parts[0]}


def _regrets(names):
    """Per geometry: regret of the least predicted candidate over all of
    them, gain over the default plan; per dimension of each geometry: regret
    of the tuner's decision (least predicted among the default and the
    variations of that dimension, against the least timed of the same)."""
    p, hdr = _model()
    d = _load(names)
    pred = _predict(p, d["X"].astype(np.float64), hdr["nfeatures"], hdr["hidden"])
    regrets, gains, decisions, guarded = [], [], [], []
    for g in np.unique(d["gid"]):
        idx = np.nonzero(d["gid"] == g)[0]
        t = np.exp(d["y"][idx].astype(np.float64))
        pick = t[np.argmin(pred[idx])]
        regrets.append(pick / t.min() - 1.0)
        var = d["varied"][idx]
        dflt = idx[var == -1]
        if len(dflt):
            gains.append(math.exp(float(d["y"][dflt[0]])) / pick)
        for dim in range(int(d["dims"][idx[0]])):
            sel = np.nonzero((var == -1) | (var == dim))[0]
            if len(sel) > 1:
                pick_t = t[sel][np.argmin(pred[idx][sel])]
                decisions.append(pick_t / t[sel].min() - 1.0)
                if len(dflt):
                    # the tuner times its pick against the default plan and keeps the faster
                    guarded.append(min(pick_t, math.exp(float(d["y"][dflt[0]]))) / t[sel].min() - 1.0)
    return regrets, gains, decisions, guarded


def _gm(r):
    return math.exp(np.mean(np.log1p(r))) - 1.0


def test_shipped_picker_regret_within_five_percent():
    regrets, gains, decisions, guarded = _regrets(["heldout.npz", "heldout3.npz"])
    print("geometries %d, geomean regret %.4f, median %.4f, gain over default %.3f; %d decisions, geomean %.4f, "
          "guarded %.4f" % (len(regrets), _gm(regrets), float(np.median(regrets)),
                            math.exp(np.mean(np.log(gains))), len(decisions), _gm(decisions), _gm(guarded)))
    assert len(regrets) >= 450
    assert _gm(regrets) <= 0.05
    assert _gm(decisions) <= 0.05
    assert _gm(guarded) <= _gm(decisions)


def test_shipped_picker_on_the_256_cube():
    # every candidate plan of the 3D 256^3 convolution (A = 2, M = 512^3), timed
    regrets, gains, decisions, _ = _regrets(["cube256.npz"])
    print("256^3: regret %.4f, gain over default %.3f, decisions %s" % (regrets[0], gains[0], decisions))
    assert regrets[0] <= 0.05
    assert len(decisions) == 3 and _gm(decisions) <= 0.05
