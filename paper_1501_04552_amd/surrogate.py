"""Blow-up surrogate built on the solver.

The paper motivates the benchmark with parametric studies of blow-up in the
cubic Klein-Gordon equation (Sec. 1).  Here the solver labels a sweep of
Gaussian initial data u0 = A exp(-(x^2/sx^2 + y^2/sy^2 + z^2/sz^2)) (blow-up
or not, and the blow-up time), a small MLP trained by the library's own HIP
kernels learns the map (A, sx, sy, sz) -> (blow-up logit, log blow-up time),
and queries the network is not confident about (|logit| < 2) are answered by
rerunning the solver, which remains the arbiter of every error reported.
"""
import time

import numpy as np
import torch

from . import kg as _kg

HIDDEN = 128
CONFIDENCE = 2.0


def sweep_labels(params, n=64, dt=0.005, max_steps=2000, threshold=1e3, chunk=1024, log=None):
    """Solver labels for parameter rows (A, sx, sy, sz): (blew_up, t_blowup, seconds)."""
    runs = [dict(n=n, A=float(p[0]), sigma=(float(p[1]), float(p[2]), float(p[3])), dt=dt,
                 max_steps=max_steps, threshold=threshold) for p in params]
    out, secs = [], 0.0
    for s in range(0, len(runs), chunk):
        r, t = _kg.kg_batch_run(runs[s:s + chunk])
        out += r
        secs += t
        if log:
            log(f"  labelled {len(out)}/{len(runs)} runs ({secs:.1f} s stepping)")
    blown = np.array([o["blew_up"] for o in out], dtype=bool)
    tb = np.array([o["t_blowup"] for o in out])
    return blown, tb, secs


def init_params(hidden, seed):
    """Uniform He-style initial weights, zero biases, in the library's flat
    layout (the GPU draws no random numbers; these values are its input)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in, is_w in ((hidden, 4, True), (hidden, 0, False), (hidden, hidden, True),
                                  (hidden, 0, False), (2, hidden, True), (2, 0, False)):
        if is_w:
            bound = np.sqrt(6.0 / fan_in) / np.sqrt(2.0)
            parts.append(rng.uniform(-bound, bound, size=fan_out * fan_in))
        else:
            parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    """The MLP on the GPU plus its input and target standardisation."""

    def __init__(self, hidden=HIDDEN, seed=0, max_batch=4096, params=None):
        self.hidden = hidden
        self.stream = torch.cuda.current_stream()
        p0 = init_params(hidden, seed) if params is None else np.asarray(params, np.float32)
        self.m = _kg.kg_mlp_create(hidden, max_batch, p0, self.stream.cuda_stream)
        self.tmean, self.tstd = 0.0, 1.0

    def close(self):
        if self.m:
            self.stream.synchronize()
            _kg.kg_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        return _kg.kg_mlp_get_params(self.m, self.hidden)

    def fit(self, X, blown, tb, epochs=300, lr=1e-3, batch=256, seed=0, log=None):
        """Adam on minibatches of a seeded shuffle; targets are standardised
        log blow-up times (used only where blown)."""
        X = np.asarray(X, np.float64)
        mean, std = X.mean(0), X.std(0)
        _kg.kg_mlp_set_norm(self.m, mean, std)
        logt = np.where(blown, np.log(np.where(blown, tb, 1.0)), 0.0)
        if blown.any():
            self.tmean, self.tstd = float(logt[blown].mean()), float(logt[blown].std() or 1.0)
        tgt = np.where(blown, (logt - self.tmean) / self.tstd, 0.0)
        Y = np.stack([blown.astype(np.float64), tgt], 1)
        rng = np.random.default_rng(seed)
        n = len(X)
        nb = n // batch
        history = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = rng.permutation(n)
            xd = torch.from_numpy(X[perm].astype(np.float32)).cuda()
            yd = torch.from_numpy(Y[perm].astype(np.float32)).cuda()
            last = None
            for b in range(nb):
                want = b == nb - 1
                last = _kg.kg_mlp_train_step(self.m, xd[b * batch:(b + 1) * batch],
                                             yd[b * batch:(b + 1) * batch], lr, want_loss=want)
            history.append(last)
            if log and (ep + 1) % max(1, epochs // 10) == 0:
                log(f"  epoch {ep + 1}/{epochs} loss {last:.4f}")
        torch.cuda.synchronize()
        return history, time.perf_counter() - t0

    def predict(self, X):
        """(logit, predicted blow-up time) for rows (A, sx, sy, sz)."""
        xd = torch.from_numpy(np.asarray(X, np.float32)).cuda()
        out = torch.empty((len(X), 2), dtype=torch.float32, device="cuda")
        _kg.kg_mlp_forward(self.m, xd, out)
        o = out.cpu().numpy().astype(np.float64)
        return o[:, 0], np.exp(o[:, 1] * self.tstd + self.tmean)


def evaluate(model, X, blown, tb, solver_seconds, n=64, dt=0.005, max_steps=2000, threshold=1e3,
             confidence=CONFIDENCE):
    """Accuracy against the solver's labels, the fraction deferred to the
    solver, the blow-up-time error, and runs/hour with and without the
    network (the deferred runs are actually rerun and timed)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logit, tpred = model.predict(X)
    t_infer = time.perf_counter() - t0
    pred = logit > 0
    conf = np.abs(logit) >= confidence
    deferred = np.flatnonzero(~conf)
    t_rerun = 0.0
    final = pred.copy()
    if len(deferred):
        rb, _, t_rerun = sweep_labels(X[deferred], n=n, dt=dt, max_steps=max_steps,
                                      threshold=threshold)
        final[deferred] = rb
    both = conf & pred & blown
    rel_t = np.abs(tpred[both] - tb[both]) / tb[both] if both.any() else np.array([np.nan])
    nq = len(X)
    return {
        "queries": nq,
        "accuracy_network": float(np.mean(pred == blown)),
        "accuracy_confident": float(np.mean(pred[conf] == blown[conf])) if conf.any() else None,
        "accuracy_with_fallback": float(np.mean(final == blown)),
        "deferred_fraction": float(np.mean(~conf)),
        "blowup_time_rel_err_median": float(np.median(rel_t)),
        "blowup_time_rel_err_p90": float(np.percentile(rel_t, 90)),
        "solver_only_runs_per_hour": nq / solver_seconds * 3600.0,
        "with_surrogate_runs_per_hour": nq / (t_infer + t_rerun) * 3600.0,
        "speedup": solver_seconds / (t_infer + t_rerun),
        "seconds": {"solver_all": solver_seconds, "inference": t_infer, "solver_deferred": t_rerun},
    }


def amortised(res, label_seconds, train_seconds):
    """What the surrogate costs to build (labelling its training sweep with
    the solver, then training) against what it saves per query: the number
    of queries after which answering with the surrogate (and rerunning the
    deferred ones) has paid for building it, and the speedup over the solver
    alone at the held-out set's size once the building cost is included.
    The per-query figures of `evaluate` leave the building cost out."""
    nq = res["queries"]
    t = res["seconds"]
    per_solver = t["solver_all"] / nq
    per_surrogate = (t["inference"] + t["solver_deferred"]) / nq
    build = label_seconds + train_seconds
    saving = per_solver - per_surrogate
    return {"build_seconds": build, "label_seconds": label_seconds,
            "train_seconds": train_seconds,
            "solver_seconds_per_query": per_solver,
            "surrogate_seconds_per_query": per_surrogate,
            "break_even_queries": build / saving if saving > 0 else None,
            "speedup_incl_build_at_held_out_size":
                t["solver_all"] / (build + t["inference"] + t["solver_deferred"])}


def main(argv=None):
    """Full pipeline: label a training sweep and a held-out sweep with the
    solver, train the MLP, evaluate it with solver fallback; prints JSON."""
    import argparse
    import json
    import sys

    import kg_inputs as ki

    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=8192)
    ap.add_argument("--test", type=int, default=1024)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--dt", type=float, default=0.005)
    ap.add_argument("--max-steps", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--save", default=None, help="write the labelled sweeps to this .npz")
    ap.add_argument("--quiet", action="store_true", help="no progress and no JSON output")
    args = ap.parse_args(argv)

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    cfg = dict(n=args.n, dt=args.dt, max_steps=args.max_steps, threshold=1e3)
    Xtr = ki.surrogate_params(args.train, seed=1)
    Xte = ki.surrogate_params(args.test, seed=2)
    log(f"labelling {args.train} training runs at {args.n}^3")
    btr, ttr, s_tr = sweep_labels(Xtr, log=log, **cfg)
    log(f"labelling {args.test} held-out runs")
    bte, tte, s_te = sweep_labels(Xte, log=log, **cfg)
    if args.save:
        np.savez(args.save, Xtr=Xtr, btr=btr, ttr=ttr, Xte=Xte, bte=bte, tte=tte)
    model = Surrogate(seed=0)
    log("training")
    hist, t_train = model.fit(Xtr, btr, ttr, epochs=args.epochs, lr=args.lr, batch=args.batch,
                              seed=0, log=log)
    res = evaluate(model, Xte, bte, tte, s_te, **cfg)
    model.close()
    res["amortised"] = amortised(res, s_tr, t_train)
    res.update({"workload": f"train {args.train} runs (seed 1), held out {args.test} (seed 2), "
                            f"{args.n}^3, dt={args.dt}, <= {args.max_steps} steps, blow-up at "
                            "max|u| > 1e3; MLP 4-128-128-2 GELU FP32, Adam lr "
                            f"{args.lr}, batch {args.batch}, {args.epochs} epochs",
                "blown_fraction_train": float(btr.mean()), "blown_fraction_test": float(bte.mean()),
                "label_seconds_train": s_tr, "train_seconds": t_train,
                "loss_first_last": [hist[0], hist[-1]]})
    if not args.quiet:
        print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
