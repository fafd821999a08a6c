"""Leave-one-problem-out evaluation of the learned cost model against
exhaustive and random tile search.

For each problem h of a set: the model is trained (on the GPU, by the
library's own kernels) on the measured times of every OTHER problem, ranks
all legal configurations of h, and the top ceil(budget * S_h) are "measured"
(their times are read from h's exhaustive table, so every strategy is judged
on the same measurements).  Regret = t(chosen) / t(exhaustive best) - 1.
Random search at the same budget is the method without the model; the
(1+1) evolution strategy (MLK_TUNE_ES) is replayed on the same tables.

    times = exhaustive_tables(problems)          # one GPU tuning sweep per problem
    report = leave_one_out(problems, times)      # model vs random vs ES, per problem
"""
import math

import numpy as np

from . import MLK_TUNE_ES, MLK_TUNE_EXHAUSTIVE, CostModel, configs, tune


def exhaustive_tables(problems, reps=3, warmup=1, log=None):
    """Median time (us) of every legal configuration of every problem."""
    tables = []
    for p in problems:
        _, rep, t = tune(p, MLK_TUNE_EXHAUSTIVE, reps=reps, warmup=warmup, want_times=True)
        tables.append(np.array(t, dtype=np.float64))
        if log:
            log(f"exhaustive: {rep.n_legal} configs, best {rep.best_us:.2f} us")
    return tables


def leave_one_out(problems, tables, budget=0.2, hidden=64, epochs=200, batch=256, lr=2e-3,
                  random_seeds=20, seed=0, log=None):
    cfgs = [configs(p) for p in problems]
    rows = []
    for h, p in enumerate(problems):
        model = CostModel(hidden=hidden, seed=seed + h)
        for q, (pq, tq) in enumerate(zip(problems, tables)):
            if q == h:
                continue
            for c, t in zip(cfgs[q], tq):
                if t > 0:
                    model.add_sample(pq, c, float(t))
        loss = model.train(epochs=epochs, batch=batch, lr=lr)
        t = tables[h]
        S = len(t)
        k = max(1, math.ceil(budget * S - 1e-9))
        best = float(np.min(t[t > 0]))
        pred = np.array(model.predict(p, cfgs[h]))
        order = np.argsort(pred, kind="stable")[:k]
        chosen = order[np.argmin(t[order])]
        model_regret = float(t[chosen] / best - 1.0)
        rng = np.random.default_rng(seed + 1000 + h)
        rand = []
        for _ in range(random_seeds):
            pick = rng.choice(S, size=k, replace=False)
            rand.append(float(np.min(t[pick]) / best - 1.0))
        # the (1+1) evolution strategy replayed on the same measured table
        es = []
        for r in range(random_seeds):
            _, _, seen = tune(p, MLK_TUNE_ES, budget_frac=budget, seed=seed + 2000 + 97 * h + r, table=list(t),
                              want_times=True)
            seen = np.array(seen)
            es.append(float(np.min(seen[seen > 0]) / best - 1.0))
        # rank correlation of prediction and measurement (Spearman)
        rp = np.argsort(np.argsort(pred))
        rt = np.argsort(np.argsort(t))
        spearman = float(np.corrcoef(rp, rt)[0, 1])
        row = {"configs": S, "measured": k, "best_us": best, "model_regret": model_regret,
               "random_regret_median": float(np.median(rand)), "random_regret_p90": float(np.percentile(rand, 90)),
               "es_regret_median": float(np.median(es)), "es_regret_p90": float(np.percentile(es, 90)),
               "train_loss": loss, "train_samples": int(model.sample_count()), "spearman": spearman}
        rows.append(row)
        if log:
            log(f"problem {h}: S={S} k={k} model regret {model_regret:.3f}, random median "
                f"{row['random_regret_median']:.3f} p90 {row['random_regret_p90']:.3f}, spearman {spearman:.2f}")
    mr = np.array([r["model_regret"] for r in rows])
    rm = np.array([r["random_regret_median"] for r in rows])
    em = np.array([r["es_regret_median"] for r in rows])
    summary = {"problems": len(rows), "budget_frac": budget,
               "model_regret_mean": float(mr.mean()), "model_regret_median": float(np.median(mr)),
               "model_regret_max": float(mr.max()), "model_within_5pct": int((mr <= 0.05).sum()),
               "random_regret_mean": float(rm.mean()), "random_regret_median": float(np.median(rm)),
               "random_within_5pct": int((rm <= 0.05).sum()),
               "es_regret_mean": float(em.mean()), "es_regret_median": float(np.median(em)),
               "es_within_5pct": int((em <= 0.05).sum())}
    return {"summary": summary, "per_problem": rows}
