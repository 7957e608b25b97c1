"""Train the cost model on the device and measure what it gains.

    python -m paper_1906_08687_amd.costmodel.build_model [--train 120] [--test 30]
    python -m paper_1906_08687_amd.costmodel.build_model --collect 0 60      (timings only)
    python -m paper_1906_08687_amd.costmodel.build_model --fit --test 30     (train and evaluate)

1. time every tile candidate of random training workloads 0..train-1 with
   the exhaustive autotuner (lmfao_autotune appends to the timing file);
2. fit the network to log(ms) with the library's forward/backward/Adam
   kernels and write the weights file;
3. on held-out workloads 150..150+test-1 compare the root-scan time of the
   heuristic tile choice, the learned choice and the autotuner's best:
   gain = sum t(heuristic) / sum t(learned), regret = sum t(learned) / sum t(best).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=120)
    ap.add_argument("--test", type=int, default=30)
    ap.add_argument("--collect", nargs=2, type=int, metavar=("J0", "J1"), default=None,
                    help="only time the candidates of training workloads J0..J1-1, appending to the timing file")
    ap.add_argument("--fit", action="store_true",
                    help="only train on the existing timing file and evaluate (no collection)")
    ap.add_argument("--max-rows", type=int, default=4_000_000)
    ap.add_argument("--hidden", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--timing-db", default=None)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    import torch
    from datagen.configs import random_workload
    from .. import lmfao
    from . import WEIGHTS, collect, load_db, save, train

    here = os.path.dirname(os.path.abspath(__file__))
    db_path = args.timing_db or os.path.join(here, "timings.csv")
    weights = args.weights or WEIGHTS

    def log(msg):
        print("[costmodel] " + msg, flush=True)

    if args.collect:
        t0 = time.time()
        for j in range(args.collect[0], args.collect[1]):
            collect([random_workload(j, args.max_rows)], db_path, log=lambda m, j=j: log("train %d: %s" % (j, m)))
        log("collected workloads %d..%d in %.0fs" % (args.collect[0], args.collect[1] - 1, time.time() - t0))
        return 0
    t0 = time.time()
    if not args.fit:
        if os.path.exists(db_path):
            os.remove(db_path)
        for j in range(args.train):
            collect([random_workload(j, args.max_rows)], db_path, log=lambda m, j=j: log("train %d: %s" % (j, m)))
    X, cfg, ms = load_db(db_path)
    log("collected %d timings in %.0fs" % (len(ms), time.time() - t0))
    norm, params, losses = train(X, ms, args.hidden, args.epochs, args.lr)
    save(weights, args.hidden, norm, params)
    log("trained: loss %.4f -> %.4f (standardised log ms)" % (losses[0], losses[-1]))

    stream = torch.cuda.Stream()
    rows = []
    for j in range(150, 150 + args.test):
        db, qs = random_workload(j, args.max_rows)
        eng = lmfao.Engine(db, qs, precision="bf16x3")
        eng.run(stream)
        t_h = eng.ctx.time_root_group(stream, 2, 10)
        best = eng.ctx.choose_learned(weights, stream)
        eng._bind()
        eng.run(stream)
        t_l = eng.ctx.time_root_group(stream, 2, 10)
        eng.ctx.autotune(stream, None, 3)
        eng._bind()
        eng.run(stream)
        t_b = eng.ctx.time_root_group(stream, 2, 10)
        rows.append((j, db.relations[0].n_rows, len(qs), t_h, t_l, t_b, best))
        log("test %d: heuristic %.3f ms, learned %.3f ms, autotuned %.3f ms" % (j, t_h, t_l, t_b))
        del eng
        torch.cuda.empty_cache()
    th = sum(r[3] for r in rows)
    tl = sum(r[4] for r in rows)
    tb = sum(r[5] for r in rows)
    geo_gain = float(np.exp(np.mean([np.log(r[3] / r[4]) for r in rows])))
    geo_regret = float(np.exp(np.mean([np.log(r[4] / r[5]) for r in rows])))
    report = {"train_workloads": args.train if not args.fit else "from " + os.path.basename(db_path),
              "timings": int(len(ms)), "test_workloads": args.test, "max_rows": args.max_rows,
              "hidden": args.hidden, "epochs": args.epochs, "final_loss": float(losses[-1]),
              "sum_ms": {"heuristic": th, "learned": tl, "autotune_best": tb},
              "gain_vs_heuristic": th / tl, "regret_vs_autotune": tl / tb,
              "geomean_gain": geo_gain, "geomean_regret": geo_regret,
              "per_workload": [dict(zip(["j", "fact_rows", "queries", "heuristic_ms", "learned_ms", "best_ms",
                                         "chosen"], r)) for r in rows]}
    out = json.dumps(report, indent=1)
    print(out)
    if args.report:
        with open(args.report, "w") as f:
            f.write(out)


if __name__ == "__main__":
    sys.exit(main())
