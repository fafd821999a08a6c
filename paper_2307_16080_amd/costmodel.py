"""Leave-one-problem-out evaluation of the learned cost model against
exhaustive and random tile search.

For each problem h of a set: the model is trained (on the GPU, by the
library's own kernels) on the measured times of every problem of another
layer (h's layer is held out at every batch size), and the library's
model-guided search (mlk_tune, MLK_TUNE_MODEL) ranks all legal
configurations of h and "measures" the top ceil(budget * S_h), reading their
times from h's exhaustive table, so every strategy is judged on the same
measurements.  Regret = t(chosen) / t(exhaustive best) - 1.  The library's
random search at the same budget is the method without the model; its (1+1)
evolution strategy (MLK_TUNE_ES) is replayed on the same tables.

    times = exhaustive_tables(problems)          # one GPU tuning sweep per problem
    report = leave_one_out(problems, times)      # model vs random vs ES, per problem
"""
import math

import numpy as np

from . import MLK_OP_CONV2D, MLK_TUNE_ES, MLK_TUNE_EXHAUSTIVE, MLK_TUNE_MODEL, MLK_TUNE_RANDOM, CostModel, configs, tune


def exhaustive_tables(problems, reps=3, warmup=1, log=None):
    """Median time (us) of every legal configuration of every problem."""
    tables = []
    for p in problems:
        _, rep, t = tune(p, MLK_TUNE_EXHAUSTIVE, reps=reps, warmup=warmup, want_times=True)
        tables.append(np.array(t, dtype=np.float64))
        if log:
            log(f"exhaustive: {rep.n_legal} configs, best {rep.best_us:.2f} us")
    return tables


def layer_key(p):
    """What identifies a problem apart from its batch size: a conv layer at batch
    1 and at batch 32 is one layer (its held-out evaluation holds out both)."""
    if p.op == MLK_OP_CONV2D:
        return ("conv", p.in_, p.out, p.c, p.f, p.h, p.w, p.kh, p.kw, p.sh, p.sw, p.ph, p.pw)
    return ("op", p.op, p.in_, p.out, p.M, p.N, p.K, p.count)


def train_model(problems, tables, skip_key=None, hidden=64, epochs=200, batch=256, lr=2e-3, seed=0):
    """A cost model trained on the GPU on every measured (time > 0) configuration
    of the problems whose layer_key differs from skip_key."""
    model = CostModel(hidden=hidden, seed=seed)
    for q, t in zip(problems, tables):
        if skip_key is not None and layer_key(q) == skip_key:
            continue
        for c, v in zip(configs(q), t):
            if v > 0:
                model.add_sample(q, c, float(v))
    loss = model.train(epochs=epochs, batch=batch, lr=lr)
    return model, loss


def _regret(t, idx, best):
    return float(t[idx] / best - 1.0) if idx >= 0 and t[idx] > 0 else float("inf")


def leave_one_out(problems, tables, budget=0.2, hidden=64, epochs=200, batch=256, lr=2e-3,
                  random_seeds=20, seed=0, log=None):
    """Every strategy is the library's own (mlk_tune with MLK_TUNE_MODEL,
    MLK_TUNE_RANDOM and MLK_TUNE_ES), replayed on each problem's exhaustive
    table (configurations that failed there fail here too).  For problem h
    the model is trained on the tables of every problem of a different layer
    (both batch sizes of h's layer held out); the budget counts measurements
    on h only; regret = t(chosen) / t(exhaustive best) - 1 on h's table."""
    rows = []
    models = {}
    for h, p in enumerate(problems):
        t = np.asarray(tables[h], dtype=np.float64)
        ok = t > 0
        S = len(t)
        k = max(1, math.ceil(budget * S - 1e-9))
        best = float(np.min(t[ok]))
        key = layer_key(p)
        if key not in models:   # one model per held-out layer
            models[key] = train_model(problems, tables, skip_key=key, hidden=hidden, epochs=epochs,
                                      batch=batch, lr=lr, seed=seed + len(models))
        model, loss = models[key]
        _, rep, _ = tune(p, MLK_TUNE_MODEL, budget_frac=budget, model=model, table=list(t))
        model_regret = _regret(t, rep.best_index, best)
        rand, es = [], []
        for r in range(random_seeds):
            _, rr, _ = tune(p, MLK_TUNE_RANDOM, budget_frac=budget, seed=seed + 1000 + 97 * h + r, table=list(t))
            rand.append(_regret(t, rr.best_index, best))
            _, re_, _ = tune(p, MLK_TUNE_ES, budget_frac=budget, seed=seed + 2000 + 97 * h + r, table=list(t))
            es.append(_regret(t, re_.best_index, best))
        # rank correlation of prediction and measurement over the configurations that ran
        pred = np.array(model.predict(p, configs(p)))[ok]
        rp = np.argsort(np.argsort(pred))
        rt = np.argsort(np.argsort(t[ok]))
        spearman = float(np.corrcoef(rp, rt)[0, 1]) if ok.sum() > 1 else float("nan")
        row = {"configs": S, "measured": int(rep.n_measured), "budget": k, "best_us": best,
               "model_regret": model_regret,
               "random_regret_median": float(np.median(rand)), "random_regret_p90": float(np.percentile(rand, 90)),
               "es_regret_median": float(np.median(es)), "es_regret_p90": float(np.percentile(es, 90)),
               "train_loss": loss, "train_samples": int(model.sample_count()), "spearman": spearman}
        rows.append(row)
        if log:
            log(f"problem {h}: S={S} measured {rep.n_measured}/{k} model regret {model_regret:.3f}, random median "
                f"{row['random_regret_median']:.3f} p90 {row['random_regret_p90']:.3f}, spearman {spearman:.2f}")
    mr = np.array([r["model_regret"] for r in rows])
    rm = np.array([r["random_regret_median"] for r in rows])
    em = np.array([r["es_regret_median"] for r in rows])
    summary = {"problems": len(rows), "budget_frac": budget, "strategy": "mlk_tune replayed on exhaustive tables",
               "holdout": "both batch sizes of the layer",
               "max_measured_frac": max(r["measured"] / r["configs"] for r in rows),
               "model_regret_mean": float(mr.mean()), "model_regret_median": float(np.median(mr)),
               "model_regret_max": float(mr.max()), "model_within_5pct": int((mr <= 0.05).sum()),
               "random_regret_mean": float(rm.mean()), "random_regret_median": float(np.median(rm)),
               "random_within_5pct": int((rm <= 0.05).sum()),
               "es_regret_mean": float(em.mean()), "es_regret_median": float(np.median(em)),
               "es_within_5pct": int((em <= 0.05).sum())}
    return {"summary": summary, "per_problem": rows}
