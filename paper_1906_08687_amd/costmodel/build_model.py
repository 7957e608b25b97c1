"""Train the cost model on the device and measure what it gains.

    python -m paper_1906_08687_amd.costmodel.build_model [--train 120] [--test 30]
    python -m paper_1906_08687_amd.costmodel.build_model --collect 0 60      (timings only)
    python -m paper_1906_08687_amd.costmodel.build_model --collect 0 30 --family cov
    python -m paper_1906_08687_amd.costmodel.build_model --fit --test 30     (train and evaluate)

1. time every tile candidate of training workloads 0..train-1 with the
   exhaustive autotuner (lmfao_autotune appends to the timing file): random
   mixed batches (datagen.configs.random_workload, general root scan) and
   random covariance-only star batches (random_covariance_workload, the
   dedicated covariance scan, up to 100M fact rows);
2. fit the network to log(ms) with the library's forward/backward/Adam
   kernels and write the weights file;
3. on held-out workloads 150.. of both families, and on the 100M-row
   covariance benchmark batch, compare the root-scan time of the heuristic
   tile choice, the learned choice and the autotuner's best:
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
    ap.add_argument("--family", choices=["random", "cov"], default="random",
                    help="training workloads of --collect: random mixed batches or covariance-only stars")
    ap.add_argument("--max-rows", type=int, default=None,
                    help="largest fact (default 8M for random batches, 100M for covariance stars)")
    ap.add_argument("--test-cov", type=int, default=10, help="held-out covariance-only workloads")
    ap.add_argument("--no-bench-workload", action="store_true",
                    help="skip the 100M-row covariance benchmark batch in the evaluation")
    ap.add_argument("--hidden", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--timing-db", default=None)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    import torch
    from datagen import make_batch, make_database
    from datagen.configs import random_covariance_workload, random_workload
    from .. import lmfao
    from . import WEIGHTS, collect, load_db, save, train

    here = os.path.dirname(os.path.abspath(__file__))
    db_path = args.timing_db or os.path.join(here, "timings.csv")
    weights = args.weights or WEIGHTS

    def log(msg):
        print("[costmodel] " + msg, flush=True)

    rand_rows = args.max_rows or 8_000_000
    cov_rows = args.max_rows or 100_000_000
    if args.collect:
        t0 = time.time()
        for j in range(args.collect[0], args.collect[1]):
            w = random_workload(j, rand_rows) if args.family == "random" else random_covariance_workload(j, cov_rows)
            collect([w], db_path, log=lambda m, j=j: log("train %s %d: %s" % (args.family, j, m)))
        log("collected workloads %d..%d in %.0fs" % (args.collect[0], args.collect[1] - 1, time.time() - t0))
        return 0
    t0 = time.time()
    if not args.fit:
        if os.path.exists(db_path):
            os.remove(db_path)
        for j in range(args.train):
            collect([random_workload(j, rand_rows)], db_path, log=lambda m, j=j: log("train %d: %s" % (j, m)))
    X, cfg, ms = load_db(db_path)
    log("collected %d timings in %.0fs" % (len(ms), time.time() - t0))
    norm, params, losses = train(X, ms, args.hidden, args.epochs, args.lr)
    save(weights, args.hidden, norm, params)
    log("trained: loss %.4f -> %.4f (standardised log ms)" % (losses[0], losses[-1]))

    stream = torch.cuda.Stream()

    def evaluate(name, db, qs):
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
        dedicated = int(eng.stats()["dedicated_scan"])
        log("test %s: %d fact rows, heuristic %.3f ms, learned %.3f ms, autotuned %.3f ms" %
            (name, db.relations[0].n_rows, t_h, t_l, t_b))
        del eng
        torch.cuda.empty_cache()
        return {"workload": name, "fact_rows": int(db.relations[0].n_rows), "queries": len(qs),
                "dedicated_scan": dedicated, "heuristic_ms": t_h, "learned_ms": t_l, "best_ms": t_b, "chosen": best}

    def summary(rows):
        th = sum(r["heuristic_ms"] for r in rows)
        tl = sum(r["learned_ms"] for r in rows)
        tb = sum(r["best_ms"] for r in rows)
        return {"workloads": len(rows), "sum_ms": {"heuristic": th, "learned": tl, "autotune_best": tb},
                "gain_vs_heuristic": th / tl, "regret_vs_autotune": tl / tb,
                "geomean_gain": float(np.exp(np.mean([np.log(r["heuristic_ms"] / r["learned_ms"]) for r in rows]))),
                "geomean_regret": float(np.exp(np.mean([np.log(r["learned_ms"] / r["best_ms"]) for r in rows])))}

    rand = [evaluate("random %d" % j, *random_workload(j, rand_rows)) for j in range(150, 150 + args.test)]
    cov = [evaluate("covariance %d" % j, *random_covariance_workload(j, cov_rows))
           for j in range(150, 150 + args.test_cov)]
    report = {"train_workloads": args.train if not args.fit else "from " + os.path.basename(db_path),
              "timings": int(len(ms)), "max_rows": {"random": rand_rows, "covariance": cov_rows},
              "hidden": args.hidden, "epochs": args.epochs, "final_loss": float(losses[-1]),
              "random": summary(rand), "covariance": summary(cov), "all": summary(rand + cov)}
    if not args.no_bench_workload:
        db = make_database(4, "full")
        report["benchmark_workload"] = evaluate("benchmark (workload 4, full size)", db, make_batch(4, db))
        del db
    report["per_workload"] = rand + cov
    out = json.dumps(report, indent=1)
    print(out)
    if args.report:
        with open(args.report, "w") as f:
            f.write(out)


if __name__ == "__main__":
    sys.exit(main())
