"""Batched form: many clouds of uneven size in one set of launches.

Host-side orchestration only: FPS for all clouds in one batched call, one
Delaunay per cloud on a thread pool (the ctypes call releases the GIL), one
concatenated problem, and an optional HIP graph capture of the filtration
(the library allocates nothing and records no memset nodes, so the capture
replays cleanly).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import api


def prepare(clouds, n_lm, k, threads=16, sampling="grid", seed=0):
    """clouds: list of float32 [N_i, 3] arrays.  Returns (FloodProblem,
    host landmark arrays, complexes)."""
    dev = torch.device("cuda")
    x_off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    Xd = torch.from_numpy(np.ascontiguousarray(np.concatenate(clouds), np.float32)).to(dev)
    idx, _ = api.fps_batched(Xd, x_off, n_lm)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    l_off = np.concatenate([[0], np.cumsum(n_lm)]).astype(np.int64)
    Ls = [clouds[b][idx[l_off[b]:l_off[b + 1]]] for b in range(len(clouds))]
    with ThreadPoolExecutor(threads) as ex:
        cxs = list(ex.map(api.delaunay, Ls))
    gidx = np.concatenate([idx[l_off[b]:l_off[b + 1]] + x_off[b] for b in range(len(clouds))]).astype(np.int32)
    Ld = torch.from_numpy(np.concatenate(Ls)).to(dev)
    pb = api.problem_from_complexes(Xd, x_off, Ld, l_off, cxs, k, l_xidx=torch.from_numpy(gidx).to(dev),
                                    sampling=sampling, seed=seed)
    return pb, Ls, cxs


class GraphedFiltration:
    """The whole batched filtration captured once and replayed (with
    count_evals, the debug counters are captured too; they add per-wave
    atomics, so timed replays leave them out)."""

    def __init__(self, pb, tuning=None, count_evals=False):
        self.run = api.FloodRun(pb, tuning, count_evals=count_evals)
        self.run()  # warm-up outside capture
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
        return self.run.f
