"""Learned parameter picker: data from the autotuner, training, regret.

Workflow (all GPU work runs in libhdconv's kernels):

1. ``collect``: for seeded geometries (``tune.geometries``), enumerate the
   planner's candidates (the default plan and every single-dimension
   variation, Sec. 7's decoupled search), time each on the device and store
   (features, log ms) rows.  The timings are the exhaustive search's.
2. ``train``: fit the library's MLP (HIP forward/backward/Adam) to predict
   log ms from features.
3. ``evaluate``: on held-out geometries, the model's pick (argmin predicted
   time over a geometry's candidates) against the exhaustive pick (argmin
   timed): regret = t(model pick) / t(best) - 1, and the gain over the
   planner's default (untuned) plan = t(default) / t(model pick).

CLI: ``python -m paper_2303_17510_amd.costmodel collect --seed S --start i
--count n --out file.npz`` (chunks of the geometry list), ``train`` and
``evaluate`` (see --help).
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np

from . import tune

SEED_TRAIN = 17510500
SEED_HELDOUT = 17510501
SEED_FLAGGED = 17510502  # centered and Hermitian training geometries
FLAG_MIX_FLAGGED = (0.5, 0.5)
FLAG_MIX_HELDOUT = (0.15, 0.15)
GID_FLAGGED = 100000     # geometry ids of the flagged list start here


SHAPE_FIELDS = ("variant", "m", "p", "q", "E_m", "E_p", "S", "rows_per_block", "centered")


def _shape_rows(shape):
    """Per-dimension shape fields as a 3 x 9 integer array (unused dimensions 0)."""
    out = np.zeros((3, len(SHAPE_FIELDS)), dtype=np.int64)
    for d, s in enumerate(shape):
        for k, f in enumerate(SHAPE_FIELDS):
            v = s.get(f, 0)
            if f == "variant":
                v = {"fused": 1, "multipass": 2, "outer": 3}.get(v, v)
            out[d, k] = int(v)
    return out


def _shape_of(rows, dims):
    names = {1: "fused", 2: "multipass", 3: "outer"}
    return [{f: (names[int(rows[d, k])] if f == "variant" else int(rows[d, k]))
             for k, f in enumerate(SHAPE_FIELDS) if k < rows.shape[1]} for d in range(dims)]


def _widen(data):
    """Shape rows of files written before the centered field: a zero column."""
    sh = data["shape"]
    if sh.shape[-1] < len(SHAPE_FIELDS):
        pad = np.zeros(sh.shape[:-1] + (len(SHAPE_FIELDS) - sh.shape[-1],), dtype=sh.dtype)
        data = dict(data)
        data["shape"] = np.concatenate([sh, pad], axis=-1)
    return data


def refeature(data, dtype="c64"):
    """Recompute the feature rows of stored candidates with this library's
    feature function (host-only plans): timings collected once stay usable
    when the feature set changes."""
    X = np.zeros((len(data["y"]), tune.NF), dtype=np.float32)
    for i in range(len(data["y"])):
        dims = int(data["dims"][i])
        L = [int(v) for v in data["L"][i][:dims]]
        M = [int(v) for v in data["M"][i][:dims]]
        X[i] = tune.features(L, M, _shape_of(data["shape"][i], dims), A=int(data["A"][i]), dtype=dtype)
    out = dict(data)
    out["X"] = X
    return out


def collect(geoms, reps=3, dtype="c64", log=None, time_budget_s=None, ids=None):
    """Rows of every candidate of every geometry: dict of numpy arrays (the
    features, log ms, geometry id, varied dimension, dimensions, and the
    geometry and per-dimension shape each row was timed with)."""
    X, y, gid, var, dims_l = [], [], [], [], []
    Ls, Ms, As, shp = [], [], [], []
    t0 = time.time()
    for i, g in enumerate(geoms):
        if time_budget_s and time.time() - t0 > time_budget_s:
            break
        gi = ids[i] if ids is not None else i
        try:
            cands = tune.candidates(g["L"], g["M"], A=g["A"], dtype=dtype, flags=g.get("flags", 0))
        except Exception as e:  # no plan for this geometry
            if log:
                log("geometry %d %s: no candidates (%s)" % (gi, g, e))
            continue
        n_ok = 0
        for v, shape in cands:
            try:
                ms = tune.time_shape(g["L"], g["M"], shape, A=g["A"], dtype=dtype, reps=reps)
            except Exception:
                continue
            if not (ms > 0):
                continue
            X.append(tune.features(g["L"], g["M"], shape, A=g["A"], dtype=dtype))
            y.append(math.log(ms))
            gid.append(gi)
            var.append(v)
            dims_l.append(len(g["L"]))
            Ls.append(list(g["L"]) + [1] * (3 - len(g["L"])))
            Ms.append(list(g["M"]) + [1] * (3 - len(g["M"])))
            As.append(g["A"])
            shp.append(_shape_rows(shape))
            n_ok += 1
        if log and (i % 20 == 0):
            log("geometry %d/%d L=%s A=%d: %d candidates timed, %.0f s" % (i, len(geoms), g["L"], g["A"], n_ok,
                                                                          time.time() - t0))
    return {"X": np.array(X, dtype=np.float32).reshape(-1, tune.NF), "y": np.array(y, dtype=np.float32),
            "gid": np.array(gid, dtype=np.int64), "varied": np.array(var, dtype=np.int64),
            "dims": np.array(dims_l, dtype=np.int64), "L": np.array(Ls, dtype=np.int64).reshape(-1, 3),
            "M": np.array(Ms, dtype=np.int64).reshape(-1, 3), "A": np.array(As, dtype=np.int64),
            "shape": np.array(shp, dtype=np.int64).reshape(-1, 3, len(SHAPE_FIELDS))}


def save(data, path):
    np.savez_compressed(path, **data)


def load(paths):
    """Rows of several files; a geometry id present in more than one file
    keeps only the rows of the last file that holds it (re-collected
    geometries replace their older timings)."""
    parts = [_widen({k: v for k, v in np.load(p, allow_pickle=False).items()}) for p in paths]
    later = set()
    for i in range(len(parts) - 1, -1, -1):
        gids = parts[i]["gid"]
        keep = ~np.isin(gids, np.array(sorted(later), dtype=gids.dtype))
        later.update(int(g) for g in np.unique(gids))
        parts[i] = {k: v[keep] for k, v in parts[i].items()}
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def train(data, hidden=64, epochs=300, batch=256, lr=2e-3, seed=0):
    m = tune.CostModel(hidden=hidden, seed=seed)
    loss = m.train(data["X"], data["y"], epochs=epochs, batch=batch, lr=lr, seed=seed)
    return m, loss


def evaluate(model, data):
    """Per held-out geometry: regret of the model's pick and gain over the default plan.

    Two readings of "the pick":
    * over all candidates of a geometry (the default plan and every
      single-dimension variation), the one of least predicted time;
    * per dimension, as the library's tuner decides: for each dimension d,
      the least predicted among the default and the variations of d, judged
      against the least timed of the same set ("decision" regret, one value
      per dimension of each geometry); "guarded": the faster of that pick
      and the default plan, as the tuner keeps it (close calls, where the
      tuner also times the predicted top three, are not modelled)."""
    pred = model.predict(data["X"])
    regrets, gains, rows, dec, guarded = [], [], [], [], []
    for g in np.unique(data["gid"]):
        idx = np.nonzero(data["gid"] == g)[0]
        t = np.exp(data["y"][idx].astype(np.float64))
        best = t.min()
        pick = t[np.argmin(pred[idx])]
        var = data["varied"][idx]
        dflt = idx[var == -1]
        t_def = math.exp(float(data["y"][dflt[0]])) if len(dflt) else float("nan")
        regrets.append(pick / best - 1.0)
        gains.append(t_def / pick)
        rows.append((int(g), int(data["dims"][idx[0]]), float(best), float(pick), float(t_def)))
        for d in range(int(data["dims"][idx[0]])):
            sel = np.nonzero((var == -1) | (var == d))[0]
            if len(sel) > 1:
                pick_t = t[sel][np.argmin(pred[idx][sel])]
                dec.append(pick_t / t[sel].min() - 1.0)
                if len(dflt):
                    guarded.append(min(pick_t, t_def) / t[sel].min() - 1.0)
    r = np.array(regrets)
    gm = float(np.exp(np.mean(np.log1p(r))) - 1.0)
    dr = np.array(dec) if dec else np.zeros(1)
    gr = np.array(guarded) if guarded else np.zeros(1)
    return {"geometries": len(r), "regret_geomean": gm, "regret_median": float(np.median(r)),
            "regret_p90": float(np.percentile(r, 90)), "regret_max": float(r.max()),
            "decision_regret_geomean": float(np.exp(np.mean(np.log1p(dr))) - 1.0),
            "decision_regret_p90": float(np.percentile(dr, 90)), "decision_regret_max": float(dr.max()),
            "decisions": len(dec),
            "guarded_decision_regret_geomean": float(np.exp(np.mean(np.log1p(gr))) - 1.0),
            "guarded_decision_regret_max": float(gr.max()),
            "gain_over_default_geomean": float(np.exp(np.mean(np.log(np.array(gains))))),
            "exhaustive_gain_over_default_geomean": float(np.exp(np.mean(
                [math.log(x[4] / x[2]) for x in rows if x[4] == x[4]]))),
            "rows": rows}


def _device_via_torch():
    """Start the device through PyTorch, as the front end runs (its tensors
    are PyTorch's): timings collected in a process where the library alone
    started the HIP runtime measured up to 30 % slower at 256^3 and ranked
    shapes differently from the same plans in a PyTorch process."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.zeros(1, device="cuda")
        torch.cuda.synchronize()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--geometry", default="", help="one geometry 'L1,L2,..:A' instead of the seeded list "
                   "(M = A L per dimension)")
    c.add_argument("--seed", type=int, default=SEED_TRAIN)
    c.add_argument("--total", type=int, default=2000, help="geometries in the seeded list")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=2000)
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--budget", type=float, default=0, help="stop after this many seconds (0: none)")
    c.add_argument("--min-dims", type=int, default=1, help="only geometries of at least this many dimensions")
    c.add_argument("--gid", type=int, default=0, help="geometry id of the rows of --geometry")
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--seed", type=int, default=0)
    r = sub.add_parser("refeature", help="recompute the features of stored timings (host only)")
    r.add_argument("--data", required=True)
    r.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", required=True)
    e.add_argument("--data", nargs="+", required=True)
    e.add_argument("--json", default="", help="also write the summary here")
    a = ap.parse_args(argv)
    log = lambda *s: print(*s, file=sys.stderr, flush=True)  # noqa: E731
    if a.cmd in ("collect", "train", "evaluate"):
        _device_via_torch()
    if a.cmd == "collect":
        if a.geometry:
            dims_s, A_s = a.geometry.split(":")
            L = [int(v) for v in dims_s.split(",")]
            geoms, sel = [{"L": L, "M": [int(A_s) * v for v in L], "A": int(A_s)}], [0]
            base = a.gid
        else:
            # the flagged and held-out lists mix in centered and Hermitian geometries
            fm = {SEED_FLAGGED: FLAG_MIX_FLAGGED, SEED_HELDOUT: FLAG_MIX_HELDOUT}.get(a.seed, (0.0, 0.0))
            geoms = tune.geometries(a.total, a.seed, flag_mix=fm)
            sel = [i for i in range(a.start, min(a.total, a.start + a.count)) if len(geoms[i]["L"]) >= a.min_dims]
            base = GID_FLAGGED if a.seed == SEED_FLAGGED else 0
        d = collect([geoms[i] for i in sel], reps=a.reps, log=log, time_budget_s=a.budget or None,
                    ids=[base + i for i in sel])
        save(d, a.out)
        log("saved %d rows from %d geometries to %s" % (len(d["y"]), len(np.unique(d["gid"])), a.out))
    elif a.cmd == "refeature":
        d = refeature(_widen({k: v for k, v in np.load(a.data, allow_pickle=False).items()}))
        save(d, a.out)
        log("recomputed %d feature rows into %s" % (len(d["y"]), a.out))
    elif a.cmd == "train":
        d = load(a.data)
        t0 = time.time()
        m, loss = train(d, epochs=a.epochs, seed=a.seed)
        m.save(a.out, meta={"train_rows": int(len(d["y"])), "train_geometries": int(len(np.unique(d["gid"]))),
                            "epochs": a.epochs, "seed": a.seed, "final_normalised_mse": loss,
                            "train_seconds": time.time() - t0, "data_seed": SEED_TRAIN})
        log("trained on %d rows in %.1f s, final normalised MSE %.4f, saved %s" % (len(d["y"]), time.time() - t0,
                                                                                   loss, a.out))
    else:
        m = tune.CostModel.load_file(a.model)
        r = evaluate(m, load(a.data))
        r.pop("rows")
        print(r)
        if a.json:
            import json
            with open(a.json, "w") as fh:
                json.dump(r, fh, indent=1)


if __name__ == "__main__":
    main()
