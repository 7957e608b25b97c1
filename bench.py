"""Benchmark: covariance batch over a 100M-row star join on one MI355X.

One step = one evaluation of the whole batch (every view of every level:
fills, dimension views, the fused root scan, fp64 merge, result assembly)
with all inputs resident in HBM.  Reported value = join tuples aggregated
per second (|J| = 100M tuples per step) of the full form (BF16 split
covariance on MFMA, batched schedule in a hipGraph, tile configuration
ranked by the learned cost model and judged by timing, else chosen by the
exhaustive autotuner), next to the plain form (fp32 FMAs, one launch per
view, heuristic tiles), the speedup between them, and an ablation of the
three choices one at a time (precision, batching, learned tiles) over the
plain form.  ms_per_step is the mean over the timed steps (one host clock
around all of them); the median of per-step HIP-event times is reported
beside it.

The CPU oracle runs only in the reported-baseline leg: it is timed on a
bounded sample of the workload (the first fact rows, every query), and the
same leg evaluates a seeded sample of queries over the whole join so that
each form's largest strict and normwise error against it is reported.  Full
parity in this launch configuration is tests/test_gpu_full_size.py.

`--batch cube` and `--batch ctree` time the other batch shapes the same way
(a three-dimensional data cube with five measures over workload 2's schema at
10M fact rows; a 32-node classification-tree level over workload 3's schema
at 50M fact rows), and `--batch w1|w2|w3|w5` the other workloads at full
size; the default is the covariance batch.  Table-bound batches also report
their grouped-table updates against the measured LDS atomic rate.
`--peaks` prints the measured unit rates (HBM read, LDS and L2 atomics) alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(ROOT, "paper_1906_08687_amd", "costmodel", "weights.bin")
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FULL_PRECISION = "bf16x6"     # the BF16 split the full form uses
ERR_SAMPLE = 24               # queries the oracle leg evaluates over the whole join for the error report


def algorithmic_bytes(db) -> int:
    """Bytes the root scan must move: every fact column once, plus every
    dimension view record once (the views are gathered through L2/MALL)."""
    fact = db.relations[0]
    b = sum(c.data.nbytes for c in fact.columns)
    for r in db.relations[1:]:
        nfeat = sum(1 for c in r.columns if c.kind == "cont")
        stride = ((1 + nfeat) + 3) // 4 * 4
        b += r.n_rows * stride * 4
    return int(b)


def referenced_bytes(db, queries) -> int:
    """Bytes a root scan of this batch must move: every fact column a query
    names and every foreign key of the fact once, plus every dimension view
    record once (count and the attributes the batch names below it, in whole
    16-byte quads)."""
    names = set()
    for q in queries:
        names.update(g.attr for g in q.groupby)
        names.update(p.attr for p in q.where)
        for a in q.aggs:
            for _, attrs in a.terms:
                names.update(attrs)
    fact = db.relations[0]
    keys = {c.attr for r in db.relations[1:] for c in r.columns if c.kind == "key"}
    b = sum(c.data.nbytes for c in fact.columns if c.attr in names or c.attr in keys)
    for r in db.relations[1:]:
        words = 1 + sum(1 for c in r.columns if c.attr in names)
        b += r.n_rows * ((words + 3) // 4 * 4) * 4
    return int(b)


def profiled_kernel(kernel_file: str, kernel: str):
    """The committed rocprofv3 summary of the scan (profiles/gram_scan_covariance_100M.json):
    its average kernel duration and its HBM bytes per launch (FETCH_SIZE and WRITE_SIZE scaled
    by a plain copy of known size), or None when the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gram_scan_covariance_100M.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if rec.get("kernel") != kernel or hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return {"traffic": rec["read_bytes"] + rec["write_bytes"], "kernel_ms": rec.get("kernel_trace_avg_ms")}


def time_app(batch, eng, db, qs, stream, reps=5):
    """Median host time of the application loop on the device over the engine's resident results
    (through the binding: its argument marshalling and one synchronisation are included)."""
    import torch
    from datagen.configs import cat_attrs, cont_attrs, tree_level
    from paper_1906_08687_amd import lmfao
    if batch in ("w1", "w2"):
        attrs = cont_attrs(db)
        name = "ridge regression (batch gradient descent with Barzilai-Borwein steps, lambda 0.1) of %s on the " \
               "other %d attributes, from the covariance block" % (attrs[0], len(attrs) - 1)

        def run():
            theta, info = lmfao.ridge_bgd(lmfao.covariance_matrix(eng, attrs), 1, 0.1, 5000, 1e-12)
            return {"iterations": int(info[1]), "objective": float(info[0])}
    elif batch == "w5":
        cats = cat_attrs(db)
        pairs = [i for i, q in enumerate(qs) if len(q.groupby) == 2]
        name = "mutual information of the %d pair-count tables and the Chow-Liu tree over %d attributes" % (len(pairs), len(cats))

        def run():
            mi = lmfao.mutual_information(eng, pairs)
            m = torch.zeros((len(cats), len(cats)), dtype=torch.float64, device=mi.device)
            for k, i in enumerate(pairs):
                a, b = cats.index(qs[i].groupby[0].attr), cats.index(qs[i].groupby[1].attr)
                m[a, b] = m[b, a] = mi[k]
            edges, total = lmfao.chow_liu(m)
            return {"edges": len(edges), "total_mi": total}
    elif batch in ("w3", "ctree"):
        level = tree_level(db, seed=3)
        crit = "variance" if batch == "w3" else "gini"
        name = "best %s split of each of the %d nodes over every split attribute and threshold" % (crit, len(level.nodes))
        # variance: every query of a node (COUNT, SUM(y), SUM(y^2) by attribute); gini: its
        # label-split counts; queries are laid out node after node
        qids = [i for i, q in enumerate(qs) if crit == "variance" or len(q.groupby) == 2]
        per = len(qs) // len(level.nodes)
        nodes = [i // per for i in qids]

        def run():
            res = lmfao.best_splits(eng, qids, nodes, crit, db.column("g3").domain if crit == "gini" else 0)
            return {"nodes": len(res)}
    else:
        return None
    info = run()
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        run()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t) * 1e3)
    out = {"loop": name, "ms_median": float(np.median(times)), "reps": reps}
    out.update(info)
    print("[bench] application loop: %s: %.3f ms" % (name, out["ms_median"]), file=sys.stderr, flush=True)
    return out


def time_steps(eng, stream, steps, warmup, median=False):
    """Mean seconds per step over `steps` executions after `warmup` (host clock around all of
    them, synchronised on both sides); with `median`, also the median of per-step HIP-event
    times recorded on the engine's stream (a second, separate run of `steps`)."""
    import torch
    for _ in range(warmup):
        eng.ctx.execute(stream)
    eng.ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eng.ctx.execute(stream)
    eng.ctx.sync()
    torch.cuda.synchronize()
    mean = (time.perf_counter() - t0) / steps
    if not median:
        return mean
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        eng.ctx.execute(stream)
        ev[i + 1].record(stream)
    eng.ctx.sync()
    torch.cuda.synchronize()
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    return mean, per[len(per) // 2] * 1e-3


def max_errors(got, ref, sample):
    """Largest strict relative error |got - ref| / |ref| and normwise error
    |got - ref| / sum|term| over the sampled queries' sums (ref = the oracle;
    sums whose reference is 0 count in the normwise figure only)."""
    strict = normwise = 0.0
    for i, r in zip(sample, ref):
        g = got[i]
        if not r.sums.size:
            continue
        d = np.abs(g.sums - r.sums)
        nz = r.sums != 0
        if nz.any():
            strict = max(strict, float(np.max(d[nz] / np.abs(r.sums[nz]))))
        a = r.abs_sums > 0
        if a.any():
            normwise = max(normwise, float(np.max(d[a] / r.abs_sums[a])))
    return {"max_strict": strict, "max_normwise": normwise}


def counts_exact(got, ref, sample):
    return all(np.array_equal(got[i].counts, r.counts) for i, r in zip(sample, ref))


def measure_peaks(dev, stream):
    """Unit rates on this GPU (lmfao_measure_peak): HBM read GB/s, LDS u32 atomics at random and
    at bank-distinct addresses, LDS fp64 atomics, device-scope u64 atomics on a 22 MB table."""
    import torch
    from paper_1906_08687_amd import lmfao
    out = {}
    big = torch.empty(1 << 32, dtype=torch.uint8, device=dev)
    small = torch.zeros(1 << 20, dtype=torch.uint8, device=dev)
    tab = torch.zeros(22 << 20, dtype=torch.uint8, device=dev)
    for kind, buf, iters in (("read", big, 3), ("lds_u32", small, 2000), ("lds_u32_spread", small, 2000),
                             ("lds_f64", small, 1000), ("global_u64", tab, 200)):
        lmfao.measure_peak(kind, buf, max(1, iters // 10), stream)
        best = None
        for _ in range(3):
            ms, units = lmfao.measure_peak(kind, buf, iters, stream)
            rate = units / (ms * 1e-3)
            best = rate if best is None else max(best, rate)
        out[kind] = best / 1e9 if kind == "read" else best
    del big, small, tab
    torch.cuda.empty_cache()
    return {"hbm_read_GBs": out["read"], "lds_u32_atomics_per_s": out["lds_u32"],
            "lds_u32_atomics_bank_distinct_per_s": out["lds_u32_spread"], "lds_f64_atomics_per_s": out["lds_f64"],
            "l2_u64_atomics_per_s": out["global_u64"]}


def table_updates(db, queries, results):
    """Grouped-table updates the batch defines: for every query with a group-by, one count and one
    update per aggregate for each join tuple it reaches (from the result counts), before the
    planner merges equal tables or derives coarser ones."""
    n = 0
    for q, r in zip(queries, results):
        if q.groupby:
            n += int(r.counts.sum()) * (1 + len(q.aggs))
    return n


WORKLOADS = {
    "w1": "tiny star: 100k-row fact, 2 dims; covariance of 9 attributes plus one grouped sum",
    "w2": "snowflake: 10M-row fact (Zipf(1.1) keys), 4 dims and a sub-dimension; ridge-regression batch with "
          "categorical group-bys and pairwise categorical counts",
    "w3": "regression-tree level: 50M-row fact, 3 dims; COUNT, SUM(y), SUM(y^2) grouped by bucket per "
          "(node, attribute) for 32 random nodes",
    "w5": "mutual-information counts: 50M-row fact, 3 dims; all marginal and pairwise COUNT GROUP BY over "
          "15 categorical attributes",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", default="covariance", choices=["covariance", "cube", "ctree", "w1", "w2", "w3", "w5", "m2m"],
                    help="covariance: the 861-aggregate covariance batch (workload 4, the benchmark); cube: data "
                         "cube; ctree: classification-tree level; wK: workload K's batch at full size")
    ap.add_argument("--n-fact", type=int, default=None, help="fact rows (default: the batch's full size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="no effect (accepted for recorded profiling command lines); parity with the oracle at full "
                         "size in this launch configuration is tests/test_gpu_full_size.py")
    ap.add_argument("--plan", default="auto", choices=["auto", "learned", "autotune", "heuristic"],
                    help="tile choice of the full form: auto = the cost model ranks the candidates, its top 4 "
                         "and the heuristic choice are timed and the fastest kept (exhaustive autotune without a model); learned = the model's top choice alone")
    ap.add_argument("--timing-db", default=None, help="autotune: append every candidate's timing to this file")
    ap.add_argument("--candidate", type=int, default=-1,
                    help="run tile candidate I of the full form instead of choosing one (profiling runs)")
    ap.add_argument("--precision", default=FULL_PRECISION, choices=["bf16x3", "bf16x4", "bf16x6"],
                    help="split form of the full form: hi+lo with three products (hi*hi + hi*lo + lo*hi) or four "
                         "(+ lo*lo), or hi+mid+lo with six (every term down to 2^-16 of a product)")
    ap.add_argument("--forms", default="both", choices=["both", "full"],
                    help="full: skip the plain form (profiling runs)")
    ap.add_argument("--peaks", action="store_true", help="print the measured unit rates alone and exit")
    ap.add_argument("--no-ablation", action="store_true", help="skip the one-choice-at-a-time forms")
    ap.add_argument("--root", default="tree", choices=["tree", "find"],
                    help="root of each query in the full form: the join tree's root, or the paper's root assignment")
    ap.add_argument("--app", action="store_true",
                    help="also time the application loop on the device over the full form's results: ridge "
                         "regression by gradient descent (w1, w2), mutual information and the Chow-Liu tree (w5), "
                         "best regression-tree splits (w3) or classification-tree splits (ctree)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device-to-device copy of 2 GiB (a plain copy kernel of known size, "
                         "used to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the engine shards by fact rows "
              "in design only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from datagen import make_batch, make_database
    from datagen.configs import (classification_tree_batch, data_cube_batch, many_to_many_batch, many_to_many_database,
                                 many_to_many_join_size, many_to_many_local_queries, tree_level)
    from paper_1906_08687_amd.lmfao import Engine, upload_columns

    if args.peaks:
        dev = torch.device("cuda", 0)
        print(json.dumps({"peaks": measure_peaks(dev, torch.cuda.Stream())}))
        return

    t = time.time()
    over = {"n_fact": args.n_fact} if args.n_fact else {}
    if args.batch == "covariance":
        db = make_database(4, "full", **over)
        qs = make_batch(4, db)
        precision = args.precision
        metric = "join tuples aggregated/sec (covariance batch, 100M fact) + speedup vs plain FP32"
        workload = ("covariance batch: 100M-row fact (16 fp32 attrs, 4 Zipf(1.2) keys) joined with 4 dims "
                    "(1M/100k/10k/1k rows, 6 fp32 attrs each), values N(100,1); 861 aggregates")
        cpu_rows = 25_000_000
    elif args.batch == "cube":
        db = make_database(2, "full", **over)
        qs = data_cube_batch(["c0", "c1", "c4"], ["f1", "f2", "d1_1", "d2_1", "d4_1"])
        precision = "fp32"
        metric = "join tuples aggregated/sec (data cube, 10M fact) + speedup vs plain"
        workload = ("data cube: 3 dimensions (c0 of the fact, c1 and c4 of two dimensions; 60/65/112 values "
                    "at this seed) x 5 measures, 8 group-bys, over workload 2's snowflake at 10M fact rows")
        cpu_rows = 10_000_000
    elif args.batch == "m2m":
        db = many_to_many_database(n_fact=args.n_fact or 6_000_000, n_users=1_300_000, n_business=170_000,
                                   mean_cat=4, mean_attr=15)
        qs = many_to_many_batch(db) + many_to_many_local_queries()
        precision = "fp32"       # a covariance block over count-weighted views runs in FP32
        metric = "join tuples aggregated/sec (many-to-many star, %s reviews)" % "{:,}".format(db.relations[0].n_rows)
        workload = ("many-to-many star (Yelp-like): Review (Zipf(1.1) user and business keys) joined with User "
                    "(1.3M) and Business (170k) on unique keys and with Category and Attribute on the repeated "
                    "business key (0-8 and 0-30 rows per business); covariance of 8 attributes, grouped sums, and "
                    "queries that group by, filter on or multiply the many-to-many attributes (evaluated at those "
                    "relations)")
        cpu_rows = 200_000
    elif args.batch in WORKLOADS:
        k = int(args.batch[1])
        db = make_database(k, "full", **over)
        qs = make_batch(k, db)
        has_gram = any(not q.groupby and not q.where and q.aggs for q in qs)
        precision = args.precision if has_gram else "fp32"
        metric = "join tuples aggregated/sec (workload %d, %s fact)" % (k, "{:,}".format(db.relations[0].n_rows))
        workload = WORKLOADS[args.batch]
        cpu_rows = {1: 100_000, 2: 2_000_000, 3: 1_000_000, 5: 2_000_000}[k]
    else:
        db = make_database(3, "full", **over)
        qs = classification_tree_batch(db, "g3", tree_level(db, seed=3))
        precision = "fp32"
        metric = "join tuples aggregated/sec (classification-tree level, 50M fact) + speedup vs plain"
        workload = ("classification-tree level: 32 nodes x 29 split attributes (20 bucketed continuous, 9 "
                    "categorical), COUNT GROUP BY (label g3, bucket) and GROUP BY bucket, over workload 3's star "
                    "at 50M fact rows")
        cpu_rows = 2_000_000
    print("[bench] generated %s batch: %d fact rows, %d queries in %.1fs" % (args.batch, db.relations[0].n_rows, len(qs),
                                                                             time.time() - t), file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    cols = upload_columns(db, dev)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    n_join = many_to_many_join_size(db) if args.batch == "m2m" else db.relations[0].n_rows

    if args.copy_calibration:
        src = torch.empty(1 << 31, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: %d bytes read, %d bytes written" % (src.numel(), dst.numel()),
              file=sys.stderr, flush=True)
        del src, dst
        # read-only rate: a device-wide sum over 8 GB of fp32 (context for the roofline)
        x = torch.ones(1 << 31, dtype=torch.float32, device=dev)
        for _ in range(2):
            x.sum()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            x.sum()
        torch.cuda.synchronize()
        print("[bench] read-only sum over %d bytes: %.1f GB/s" % (x.numel() * 4, x.numel() * 4 * 5 / (time.perf_counter() - t) / 1e9),
              file=sys.stderr, flush=True)
        del x

    # plain form: fp32 covariance, one launch per view, heuristic tiles, every table scanned
    t_plain, plain_root_ms, plain_stats, plain_res = None, None, {"launches": None}, None
    if args.forms == "both":
        plain = Engine(db, qs, precision="fp32", schedule="plain", columns=cols, rollup=False)
        # the tree levels' and pair counts' plain forms rescan the fact once per view (hundreds of scans)
        ps, pw = (args.steps, args.warmup) if args.batch not in ("ctree", "w3", "w5") else (2, 1)
        t_plain = time_steps(plain, stream, ps, pw)
        plain_root_ms = plain.ctx.time_root_group(stream, 1, 5)
        plain_stats = plain.stats()
        plain_res = plain.results()
        print("[bench] plain fp32: %.3f ms/step" % (t_plain * 1e3), file=sys.stderr, flush=True)
        del plain

    # full form: BF16 split on MFMA, batched in a hipGraph; tiles chosen by the cost model, its top
    # candidates judged by timing (every way of choosing is timed and reported; the one the
    # --plan option names runs last, so it is the plan the timed steps use)
    full = Engine(db, qs, precision=precision, schedule="batched", columns=cols, root=args.root)
    full.ctx.execute(stream)
    full.ctx.sync()
    plans = {}
    have_model = os.path.exists(WEIGHTS)
    if args.candidate >= 0:
        full.ctx.select_candidate(args.candidate)
        chosen, best = "fixed", args.candidate
    else:
        def heuristic():
            full.replan()
            full._bind()
            full.ctx.execute(stream)
            full.ctx.sync()
            return -1

        def learned():
            return full.ctx.choose_learned(WEIGHTS, stream)

        def verified():
            heuristic()
            return full.ctx.choose_learned_verified(WEIGHTS, stream, 4, 10)

        def autotune():
            return full.ctx.autotune(stream, args.timing_db, 3)

        ways = [("heuristic", heuristic)]
        if have_model:
            ways += [("learned", learned), ("learned_top4_timed", verified)]
        # the exhaustive autotuner is timed for reference when the plan has few candidates (the
        # dedicated scan has 15; a general scan of a large batch can have hundreds of slow ones)
        if args.plan == "autotune" or not have_model or len(full.ctx.candidates()) <= 32:
            ways.append(("autotune", autotune))
        chosen = {"auto": "learned_top4_timed" if have_model else "autotune",
                  "learned": "learned" if have_model else "heuristic",
                  "autotune": "autotune", "heuristic": "heuristic"}[args.plan]
        ways = [w for w in ways if w[0] != chosen] + [w for w in ways if w[0] == chosen]
        for name, fn in ways:
            idx = fn()
            full._bind()
            full.ctx.execute(stream)
            full.ctx.sync()
            plans[name] = {"candidate": idx, "root_scan_ms": full.ctx.time_root_group(stream, 2, 10)}
            print("[bench] tile choice %s: candidate %d, root scan %.3f ms" % (name, idx, plans[name]["root_scan_ms"]),
                  file=sys.stderr, flush=True)
        best = plans[chosen]["candidate"]
        print("[bench] tile choices: %s" % json.dumps(plans), file=sys.stderr, flush=True)
    full._bind()
    t_full, t_full_median = time_steps(full, stream, args.steps, args.warmup, median=True)
    root_ms = full.ctx.time_root_group(stream, 2, 10)
    stats = full.stats()
    full_res = full.results()
    print("[bench] full %s/batched/%s: %.3f ms/step (median %.3f), root scan %.3f ms" %
          (precision, chosen, t_full * 1e3, t_full_median * 1e3, root_ms), file=sys.stderr, flush=True)

    app = time_app(args.batch, full, db, qs, stream) if args.app else None

    # ablation: each of the three choices alone over the plain form (fp32, one launch per view,
    # heuristic tiles; the tables as the full form plans them)
    ablation = None
    if args.forms == "both" and not args.no_ablation:
        ablation = {}
        ab_steps = min(args.steps, 10) if args.batch not in ("ctree", "w3", "w5") else 2
        del full
        torch.cuda.empty_cache()
        for name, prec, sched, learned in (("precision", precision, "plain", False), ("batching", "fp32", "batched", False),
                                           ("learned_tiles", "fp32", "plain", True)):
            eng = Engine(db, qs, precision=prec, schedule=sched, columns=cols)
            eng.ctx.execute(stream)
            eng.ctx.sync()
            cand = -1
            if learned and have_model:
                cand = eng.ctx.choose_learned_verified(WEIGHTS, stream, 4, 3)
                eng._bind()
            t = time_steps(eng, stream, ab_steps, 1)
            ablation[name] = {"precision": prec, "schedule": sched, "tiles": "learned_top4_timed" if learned else "heuristic",
                              "candidate": cand, "ms_per_step": t * 1e3, "speedup_vs_plain_fp32": (t_plain / t)}
            print("[bench] ablation %s alone: %.3f ms/step" % (name, t * 1e3), file=sys.stderr, flush=True)
            del eng
            torch.cuda.empty_cache()

    # reported baseline: the oracle on the host cores, timed on a bounded sample; the same leg
    # evaluates a seeded sample of queries over the whole join for the error report of both forms
    cpu, errors = None, None
    if not args.no_cpu_baseline:
        import oracle
        rows = min(db.relations[0].n_rows, cpu_rows)        # about 10 s of the oracle on 16 host threads
        threads = os.cpu_count() or 1
        t = time.time()
        oracle.evaluate(db, qs, n_threads=threads, root_range=(0, rows))
        dt = time.time() - t
        tuples = rows
        if args.batch == "m2m":   # the sample's join tuples: its reviews times their businesses' row counts
            b = db.rel("Review").col("business").data[:rows]
            nb = db.rel("Business").n_rows
            c = np.bincount(db.rel("Category").col("business").data, minlength=nb).astype(np.int64)
            a = np.bincount(db.rel("Attribute").col("business").data, minlength=nb).astype(np.int64)
            tuples = int(np.sum(c[b] * a[b]))
        cpu = {"value": tuples / dt, "unit": "join tuples/s", "cores": threads, "kind": "oracle",
               "sample": "first %d fact rows (of %d; %d join tuples) joined with every other relation, all %d queries" %
                         (rows, db.relations[0].n_rows, tuples, len(qs))}
        print("[bench] cpu oracle: %.3g tuples/s on %d threads" % (cpu["value"], threads), file=sys.stderr, flush=True)
        rng = np.random.default_rng(2024)
        sample = sorted(set([0] + [int(i) for i in rng.choice(np.arange(1, len(qs)), min(ERR_SAMPLE, len(qs) - 1),
                                                                 replace=False)]))
        t = time.time()
        ref = oracle.evaluate(db, [qs[i] for i in sample], n_threads=threads)
        errors = {"sample": "%d of %d queries (seeded), every cell, over the whole join" % (len(sample), len(qs)),
                  "oracle_s": time.time() - t,
                  "full": dict(max_errors(full_res, ref, sample), counts_exact=counts_exact(full_res, ref, sample),
                               precision=precision)}
        if plain_res is not None:
            errors["plain_fp32"] = dict(max_errors(plain_res, ref, sample), counts_exact=counts_exact(plain_res, ref, sample))
        print("[bench] errors vs oracle: %s" % json.dumps(errors), file=sys.stderr, flush=True)

    alg = algorithmic_bytes(db) if args.batch == "covariance" else referenced_bytes(db, qs)
    achieved = alg / (root_ms * 1e-3) / 1e9
    prof = profiled_kernel("gram_scan.hip", "gram_scan_kernel") if stats["dedicated_scan"] else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": prof["traffic"] if prof else None,
                "kernel": ("gram_scan_kernel" if stats["dedicated_scan"] else "root_scan_kernel") + " (%s)" % precision,
                "algorithmic_bytes": alg, "kernel_ms": root_ms,
                "rocprof_kernel_ms": prof["kernel_ms"] if prof else None}
    extra = {}
    if args.batch == "covariance" and plain_root_ms:
        # the plain form's covariance is fp32 FMAs: 2 flops per monomial and joined row
        flops = 2.0 * sum(1 for q in qs if q.aggs) * n_join
        extra["plain_fp32_scan_fp32_roofline"] = {"bound": "alu", "achieved": flops / (plain_root_ms * 1e-3) / 1e12,
                                                  "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                  "frac": flops / (plain_root_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    if args.batch in ("w2", "w3", "w5", "cube", "ctree"):
        # grouped tables: their updates against the measured LDS atomic rate
        peaks = measure_peaks(dev, stream)
        upd = table_updates(db, qs, full_res)
        rate = upd / t_full
        extra["table_updates"] = {"bound": "lds_atomics", "updates_per_step": upd, "achieved_per_s": rate,
                                  "peak_per_s": peaks["lds_u32_atomics_per_s"],
                                  "frac": rate / peaks["lds_u32_atomics_per_s"],
                                  "hbm_frac": alg / t_full / 1e9 / HBM_PEAK_GBS, "peaks": peaks}
    line = {
        "metric": metric,
        "value": n_join / t_full,
        "unit": "join tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_full * 1e3,
        "ms_per_step_median": t_full_median * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("%s-split/f32-acc/f64-merge" % precision) if precision != "fp32" else "f32/u64-counts/f64-merge",
        "data": "synthetic (seeded; %s recipe)" % {"covariance": "workload 4", "cube": "workload 2", "ctree": "workload 3",
                                                    "m2m": "many-to-many star"}.get(args.batch, "workload " + args.batch[1:]),
        "config": {"workload": workload,
                   "fact_rows": n_join, "aggregates": len(qs), "plan": chosen, "candidate": best,
                   "plan_choices": plans,
                   "grid_blocks": stats["grid_blocks"], "gram_block": stats["gram_block"],
                   "waves_per_workgroup": stats["waves"], "staging_buffers": stats["nbuf"],
                   "lds_bytes": stats["lds_bytes"], "grouped_tables": stats["tables"],
                   "derived_tables": stats["derived_tables"], "count_table_scan": stats["hist_scan"],
                   "root_policy": args.root, "queries_at_other_roots": stats["target_queries"],
                   "launches": stats["launches"]},
        "speedup_vs_plain_fp32": (t_plain / t_full) if t_plain else None,
        "plain_fp32": ({"ms_per_step": t_plain * 1e3, "value": n_join / t_plain, "root_scan_ms": plain_root_ms,
                        "launches": plain_stats["launches"]} if t_plain else None),
        "ablation": ablation,
        "errors_vs_oracle": errors,
        "application_loop": app,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
