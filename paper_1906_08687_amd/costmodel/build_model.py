"""Train the cost model on the device and measure what it gains.

    python -m paper_1906_08687_amd.costmodel.build_model --collect 0 110                (random batches)
    python -m paper_1906_08687_amd.costmodel.build_model --collect 0 90 --family cov    (covariance stars)
    python -m paper_1906_08687_amd.costmodel.build_model --fit --test 50 --test-cov 20 --report eval.json

1. time every candidate (tile configuration and table grouping) of training
   workloads j < 150 with the exhaustive autotuner (lmfao_autotune appends to
   the timing file): random mixed batches (datagen.configs.random_workload,
   general root scan) and random covariance-only star batches
   (random_covariance_workload, the dedicated covariance scan, up to 100M fact
   rows), in the benchmark's precision;
2. train the network in the library (lmfao_train_cost_model: workload
   grouping, relative log-time targets, standardisation and Adam on the
   device) and write the weights file;
3. on held-out workloads 150.. of both families (random batches up to 20M
   fact rows), and on the 100M-row covariance benchmark batch, time the root
   scan under the heuristic choice, the model's top choice, the model's top
   four judged by timing together with the heuristic choice, and the
   autotuner's best: gain = t(heuristic) / t(learned), regret =
   t(learned) / t(autotuner's best), as sums and geometric means.
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
                    help="largest fact of the training workloads (default 8M for random batches, 100M for "
                         "covariance stars; held-out random batches go up to 20M)")
    ap.add_argument("--precision", default="bf16x6")
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
    from . import WEIGHTS, collect, load_db

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
            collect([w], db_path, precision=args.precision,
                    log=lambda m, j=j: log("train %s %d: %s" % (args.family, j, m)))
        log("collected workloads %d..%d in %.0fs" % (args.collect[0], args.collect[1] - 1, time.time() - t0))
        return 0
    t0 = time.time()
    if not args.fit:
        if os.path.exists(db_path):
            os.remove(db_path)
        for j in range(args.train):
            collect([random_workload(j, rand_rows)], db_path, precision=args.precision,
                    log=lambda m, j=j: log("train %d: %s" % (j, m)))
    X, cfg, ms = load_db(db_path)
    log("collected %d timings in %.0fs" % (len(ms), time.time() - t0))
    first = lmfao.train_cost_model(db_path, weights, args.hidden, 1, args.lr)
    loss = lmfao.train_cost_model(db_path, weights, args.hidden, args.epochs, args.lr)
    log("trained in the library: loss %.4f after one step, %.4f after %d (standardised relative log ms)" %
        (first, loss, args.epochs))

    stream = torch.cuda.Stream()

    def evaluate(name, db, qs):
        eng = lmfao.Engine(db, qs, precision=args.precision)
        eng.run(stream)
        t_h = eng.ctx.time_root_group(stream, 2, 10)
        top = eng.ctx.choose_learned(weights, stream)
        eng._bind()
        eng.run(stream)
        t_l = eng.ctx.time_root_group(stream, 2, 10)
        eng.replan()
        eng.run(stream)
        ver = eng.ctx.choose_learned_verified(weights, stream, 4, 3)
        eng._bind()
        eng.run(stream)
        t_v = eng.ctx.time_root_group(stream, 2, 10)
        eng.ctx.autotune(stream, None, 2)
        eng._bind()
        eng.run(stream)
        t_b = eng.ctx.time_root_group(stream, 2, 10)
        dedicated = int(eng.stats()["dedicated_scan"])
        n_cand = len(eng.ctx.candidates())
        log("test %s: %d fact rows, %d candidates, heuristic %.3f ms, learned %.3f ms, learned top-4 timed %.3f ms, "
            "autotuned %.3f ms" % (name, db.relations[0].n_rows, n_cand, t_h, t_l, t_v, t_b))
        del eng
        torch.cuda.empty_cache()
        return {"workload": name, "fact_rows": int(db.relations[0].n_rows), "queries": len(qs), "candidates": n_cand,
                "dedicated_scan": dedicated, "heuristic_ms": t_h, "learned_ms": t_l, "learned_top4_timed_ms": t_v,
                "best_ms": t_b, "chosen": top, "chosen_timed": ver}

    def summary(rows):
        out = {"workloads": len(rows)}
        th = [r["heuristic_ms"] for r in rows]
        tb = [r["best_ms"] for r in rows]
        for key, label in (("learned_ms", "learned"), ("learned_top4_timed_ms", "learned_top4_timed")):
            tl = [r[key] for r in rows]
            out[label] = {"sum_ms": sum(tl), "gain_vs_heuristic": sum(th) / sum(tl),
                          "regret_vs_autotune": sum(tl) / sum(tb),
                          "geomean_gain": float(np.exp(np.mean(np.log(np.array(th) / np.array(tl))))),
                          "geomean_regret": float(np.exp(np.mean(np.log(np.array(tl) / np.array(tb)))))}
        out["sum_ms"] = {"heuristic": sum(th), "autotune_best": sum(tb)}
        return out

    rand = [evaluate("random %d" % j, *random_workload(j, 20_000_000)) for j in range(150, 150 + args.test)]
    cov = [evaluate("covariance %d" % j, *random_covariance_workload(j, cov_rows))
           for j in range(150, 150 + args.test_cov)]
    report = {"train_workloads": args.train if not args.fit else "from " + os.path.basename(db_path),
              "timings": int(len(ms)), "max_rows": {"train random": rand_rows, "held-out random": 20_000_000,
                                                    "covariance": cov_rows},
              "precision": args.precision, "hidden": args.hidden, "epochs": args.epochs, "final_loss": loss,
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
