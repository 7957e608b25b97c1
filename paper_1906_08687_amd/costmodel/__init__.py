"""Learned cost model of the root view-group scan.

A small network (16 plan features -> relative log milliseconds) ranks the
candidate tile configurations of a plan (waves per workgroup, staging buffers,
workgroups, fp32 register block, table placement).  Only the ranking within a
plan matters, so the training target is a candidate's log time over the best
time among its workload's candidates, clipped at log 4: every candidate more
than 4x slower than the best is simply bad, and its exact slowdown does not
pull the fit away from the near-optimal ones (workloads are told apart by the
features that do not depend on the candidate).  Timings come from the
engine itself: the exhaustive autotuner appends one line per timed candidate
to a timing file; training runs on the device with the library's own
forward/backward/Adam kernels, inside the library (lmfao_train_cost_model
builds the targets and the standardisation from the timing file); the planner
queries the network through
lmfao_choose_learned and keeps the heuristic configuration whenever the
model is absent or predicts a non-finite time.

Weights file: b"LMFAOMLP", int32 hidden, float32 feature mean[16] and
std[16], float32 target mean and std, float32 parameters.
"""
from __future__ import annotations

import os
import struct
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .. import lmfao

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights.bin")
N_FEATURES = lmfao.N_FEATURES


def collect(workloads, timing_db: str, precision: str = "bf16x6", reps: int = 3, device: int = 0,
            log=None) -> List[Tuple[int, float]]:
    """Time every tile candidate of every workload (db, queries) and append
    the timings to ``timing_db``.  Returns (best candidate, best ms) per
    workload."""
    import torch
    out = []
    stream = torch.cuda.Stream(device=device)
    for i, (db, qs) in enumerate(workloads):
        eng = lmfao.Engine(db, qs, precision=precision, schedule="batched", device=device)
        eng.run(stream)
        best = eng.ctx.autotune(stream, timing_db, reps)
        ms = eng.ctx.time_root_group(stream, 1, reps)
        out.append((best, ms))
        if log:
            log("workload %d: %d fact rows, %d queries, best candidate %d at %.3f ms" %
                (i, db.relations[0].n_rows, len(qs), best, ms))
        del eng
        torch.cuda.empty_cache()
    return out


def load_db(path: str):
    """Features (n x 16), candidate configuration columns and milliseconds."""
    rows = [l.strip().split(",") for l in open(path) if l.strip()]
    a = np.array([[float(v) for v in r] for r in rows], dtype=np.float64)
    return a[:, :N_FEATURES], a[:, N_FEATURES:-1], a[:, -1]


def init_params(hidden: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2.0 / N_FEATURES), hidden * N_FEATURES), np.zeros(hidden),
             rng.normal(0, np.sqrt(2.0 / hidden), hidden * hidden), np.zeros(hidden),
             rng.normal(0, np.sqrt(1.0 / hidden), hidden), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


# features fixed by the workload and plan (the rest describe the tile candidate)
WORKLOAD_FEATURES = (0, 1, 3, 4, 5, 6, 7, 8, 12, 13)


def workload_groups(X: np.ndarray) -> np.ndarray:
    """Group index of every timing row: rows with equal workload features."""
    keys = np.round(np.asarray(X, np.float64)[:, WORKLOAD_FEATURES], 4)
    _, inv = np.unique(keys, axis=0, return_inverse=True)
    return inv.reshape(-1)


RELATIVE_CAP = float(np.log(4.0))


def relative_log_ms(X: np.ndarray, ms: np.ndarray) -> np.ndarray:
    """min(log(ms / best ms of the row's workload), log 4)."""
    y = np.log(np.asarray(ms, np.float64))
    g = workload_groups(X)
    best = np.full(g.max() + 1, np.inf)
    np.minimum.at(best, g, y)
    return np.minimum(y - best[g], RELATIVE_CAP)


def save(path: str, hidden: int, norm: np.ndarray, params: np.ndarray):
    """Write a weights file in the library's layout (used by tests that build a model by hand)."""
    with open(path, "wb") as f:
        f.write(b"LMFAOMLP")
        f.write(struct.pack("<i", hidden))
        f.write(np.asarray(norm, np.float32).tobytes())
        f.write(np.asarray(params, np.float32).tobytes())


def load(path: str = WEIGHTS):
    with open(path, "rb") as f:
        assert f.read(8) == b"LMFAOMLP"
        hidden = struct.unpack("<i", f.read(4))[0]
        norm = np.frombuffer(f.read(4 * (2 * N_FEATURES + 2)), np.float32)
        params = np.frombuffer(f.read(), np.float32)
    return hidden, norm, params
