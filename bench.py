#!/usr/bin/env python3
"""Benchmark of the flooding path on one MI355X.

Workload (default): N = 10,000,000 float32 points on 20 noisy primitive
surfaces in the unit cube, L = 10,000 farthest-point landmarks, k = 8
segments per edge.  One step = landmark selection (GPU) + the flooding
filtration (GPU: grid build, seeds, flooding search, winners) for every
simplex of Del(L).  Del(L) is computed once on the host before the timed
region (it is combinatorial and the landmarks are identical every step).

Prints one JSON line.  `value` is sample-point distance evaluations per
second over the whole step; the evaluations are counted by the kernels in a
separate instrumented run (the timed steps run without counters).  The
roofline block covers the flooding-search kernel, timed live with HIP
events the library records around each of its launches.  Beside it: the
FP64 oracle on a bounded sample of the same simplices (its throughput and,
element by element, the largest |df| / diam(X) per dimension), the batched
form (512 clouds, one HIP-graph replay, autotuned), and the differentiable
form (64 clouds, forward + backward).

`--sweep x|l|table` instead runs the stage breakdown and scaling sweeps on
swiss-cheese clouds and writes them as JSON to `--sweep-out`.
"""
import argparse
import ctypes
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flood distance evals/s + simplices/s at N=10M (% FP32 peak); batched clouds/s"
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
FLOP_PER_EVAL = 8  # 3 sub + 1 mul + 2 fma (2 each)
GRID_BYTES_PER_POINT = 100  # bbox 12 + count 12 + partition 12 + 16 + bucket sort 16 + 16 + 16
TOL = 1e-5  # |df| / diam(X)
TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")


def hip_runtime():
    for line in open("/proc/self/maps"):
        if "libamdhip64.so" in line:
            return ctypes.CDLL(line.split()[-1])
    return ctypes.CDLL("libamdhip64.so")


class HipEvents:
    """Raw hipEvent_t handles for the library's launch stream (torch's events
    see only torch's current stream, and the library records these itself)."""

    def __init__(self, n):
        self.rt = hip_runtime()
        self.ev = [ctypes.c_void_p() for _ in range(n)]
        for e in self.ev:
            assert self.rt.hipEventCreate(ctypes.byref(e)) == 0

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) == 0
        return ms.value

    def close(self):
        """Destroys the events (after the work that records them has finished)."""
        for e in self.ev:
            if e.value:
                assert self.rt.hipEventDestroy(e) == 0
                e.value = None


def measured_traffic(kernel, tuning=None):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain-copy calibration),
    or None when the kernel's sources changed since the counters were taken
    or the counters were taken at another tuning."""
    try:
        t = json.load(open(TRAFFIC_PATH))
        k = t["kernels"][kernel]
        m = hashlib.sha256()
        for f in k["sources"]:
            m.update(open(os.path.join(ROOT, "paper_2509_22432_amd", "csrc", f), "rb").read())
    except (OSError, KeyError, ValueError):
        return None
    if m.hexdigest() != k["sources_sha256"]:
        return None
    if "tuning" in k and k["tuning"] != (tuning or {}):
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


# source files each profiled kernel is compiled from (the traffic figures
# are dropped once any of them changes)
TRAFFIC_SOURCES = {
    "flood::k_flood_tiles<1>": ["flood.hip", "sample.hpp", "internal.hpp"],
    "flood::k_flood_deep": ["flood.hip", "sample.hpp", "internal.hpp"],
    "flood::k_winner_search": ["flood.hip", "sample.hpp", "internal.hpp"],
    "flood::k_fps_coop<0>": ["fps.hip", "internal.hpp"],
}


def _counter_rows(d):
    """(kernel name, dispatch id) -> counter value from one rocprofv3 --pmc
    csv directory (one counter per pass)."""
    import csv
    import glob
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            key = (name, int(r["Dispatch_Id"]))
            out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return out


def write_traffic(pmc_dir, tuning):
    """profiles/traffic.json from four rocprofv3 --pmc runs under pmc_dir:
    pmc_fetch / pmc_write (FETCH_SIZE / WRITE_SIZE of the bench), and
    pmc_copy_fetch / pmc_copy_write (the same counters for a plain copy of
    known size, `--calibrate-copy`), which give the KiB-to-bytes scale."""
    copy_bytes = 1 << 30
    cal = {}
    for c, sub in (("fetch", "pmc_copy_fetch"), ("write", "pmc_copy_write")):
        rows = _counter_rows(os.path.join(pmc_dir, sub))
        vals = [v for (n, _), v in rows.items() if "copy" in n.lower()]
        cal[c] = copy_bytes / (float(np.median(vals)) * 1024.0)
    kern = {}
    for c, sub in (("fetch", "pmc_fetch"), ("write", "pmc_write")):
        rows = _counter_rows(os.path.join(pmc_dir, sub))
        for name in TRAFFIC_SOURCES:
            vals = [v for (n, _), v in sorted(rows.items(), key=lambda kv: kv[0][1]) if n == name]
            if vals:
                kern.setdefault(name, {})[c] = (float(np.mean(vals)) * 1024.0 * cal[c], len(vals))
    out = {"calibration": {"copy_bytes": copy_bytes, "fetch_scale": cal["fetch"], "write_scale": cal["write"]},
           "kernels": {}}
    for name, v in kern.items():
        if "fetch" not in v or "write" not in v:
            continue
        m = hashlib.sha256()
        for f in TRAFFIC_SOURCES[name]:
            m.update(open(os.path.join(ROOT, "paper_2509_22432_amd", "csrc", f), "rb").read())
        out["kernels"][name] = {"fetch_bytes_per_launch": v["fetch"][0], "write_bytes_per_launch": v["write"][0],
                                "dispatches_averaged": v["fetch"][1],
                                "sources": TRAFFIC_SOURCES[name], "sources_sha256": m.hexdigest()}
        if "fps" not in name:  # the landmark kernel takes no tuning
            out["kernels"][name]["tuning"] = tuning or {}
    with open(TRAFFIC_PATH, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1, sort_keys=True))


# ---------------------------------------------------------------------------
# oracle legs (host)

def oracle_sample(X, Lxyz, cx, k, budget_s, xs, seed=0):
    """The oracle (masked FP64 mode, all host threads) on random simplices of
    the same complex, in growing rounds until `budget_s` of oracle time is
    spent.  Returns ({d: (rows, values)}, evaluations, seconds)."""
    from oracle import flood as OF
    rng = np.random.default_rng(seed)
    simp = {1: cx.E, 2: cx.F, 3: cx.T}
    tot = sum(len(simp[d]) for d in (1, 2, 3))
    rows = {d: [] for d in (1, 2, 3)}
    vals = {d: [] for d in (1, 2, 3)}
    done_s, ev, per = 0.0, np.zeros(1, np.int64), 16
    while done_s < budget_s:
        for d in (1, 2, 3):
            m = max(1, int(round(per * len(simp[d]) / tot)))
            pick = rng.choice(len(simp[d]), m, replace=False)
            t = time.time()
            v, _, _ = OF.flood_dim(X, Lxyz, simp[d][pick], d, k, "masked", xs, counter=ev)
            done_s += time.time() - t
            rows[d].append(pick)
            vals[d].append(v)
        per = min(per * 2, 4096)
    out = {d: (np.concatenate(rows[d]), np.concatenate(vals[d])) for d in (1, 2, 3)}
    return out, int(ev[0]), done_s


def parity_block(f_gpu, sample, diam):
    """Element-by-element FP32 GPU vs FP64 oracle on the sampled simplices."""
    err = []
    for d in (1, 2, 3):
        rows, ref = sample[d]
        err.append(float(np.abs(f_gpu[d][rows].astype(np.float64) - ref).max() / diam) if len(rows) else 0.0)
    err = [0.0] + err  # vertices: f = 0 exactly (checked on every vertex below)
    return {"max_df_over_diam_per_dim": err, "simplices_checked_per_dim": [0] + [int(len(sample[d][0]))
                                                                             for d in (1, 2, 3)],
            "tol_over_diam": TOL, "diam": diam, "ok": bool(max(err) <= TOL)}


def interior_compositions(d, k):
    """All a in N^{d+1} with a_i >= 1 and sum a = k."""
    out = []

    def rec(prefix, left, slots):
        if slots == 1:
            if left >= 1:
                out.append(prefix + [left])
            return
        for a in range(1, left - slots + 2):
            rec(prefix + [a], left - a, slots - 1)
    rec([], k, d + 1)
    return np.array(out, np.float64).reshape(-1, d + 1)


def culling_block(X, Lxyz, cx, k, sample, executed_per_dim, per_dim=150):
    """Executed evaluations against the evaluations an exact search needs:
    for every interior sample s (the samples the GPU evaluates; boundary
    samples belong to the faces), the points in the cells of a uniform grid
    with one cell per point on average that meet the closed ball
    B(s, d(s, X)).  Estimated on `per_dim` of the oracle's sampled simplices
    per dimension and scaled to the whole complex."""
    from scipy.spatial import cKDTree
    t0 = time.time()
    X64 = X.astype(np.float64)
    lo, hi = X64.min(0), X64.max(0)
    ext = np.maximum(hi - lo, 1e-9)
    h = float(np.cbrt(np.prod(ext) / len(X)))
    dims = np.floor(ext / h).astype(np.int64) + 1
    cell = np.minimum(np.floor((X64 - lo) / h).astype(np.int64), dims - 1)
    lin = (cell[:, 2] * dims[1] + cell[:, 1]) * dims[0] + cell[:, 0]
    counts = np.bincount(lin, minlength=int(np.prod(dims))).reshape(dims[2], dims[1], dims[0])
    del cell, lin
    tree = cKDTree(X64, balanced_tree=False, compact_nodes=False)
    simp = {1: cx.E, 2: cx.F, 3: cx.T}
    L64 = Lxyz.astype(np.float64)
    out = {}
    for d in (1, 2, 3):
        A = interior_compositions(d, k) / k
        rows = sample[d][0][:per_dim]
        if len(A) == 0 or len(rows) == 0:
            out[d] = 0.0
            continue
        S = np.einsum("sa,nac->nsc", A, L64[simp[d][rows]]).reshape(-1, 3)
        r, _ = tree.query(S, workers=-1)
        need = 0
        for s, rr in zip(S, r):
            c0 = np.floor((s - rr - lo) / h).astype(np.int64).clip(0, dims - 1)
            c1 = np.floor((s + rr - lo) / h).astype(np.int64).clip(0, dims - 1)
            zs, ys, xs = (np.arange(c0[2], c1[2] + 1), np.arange(c0[1], c1[1] + 1), np.arange(c0[0], c1[0] + 1))
            gx = np.maximum(np.maximum(lo[0] + xs * h - s[0], s[0] - (lo[0] + (xs + 1) * h)), 0.0) ** 2
            gy = np.maximum(np.maximum(lo[1] + ys * h - s[1], s[1] - (lo[1] + (ys + 1) * h)), 0.0) ** 2
            gz = np.maximum(np.maximum(lo[2] + zs * h - s[2], s[2] - (lo[2] + (zs + 1) * h)), 0.0) ** 2
            meet = (gz[:, None, None] + gy[None, :, None] + gx[None, None, :]) <= rr * rr
            need += int(counts[c0[2]:c1[2] + 1, c0[1]:c1[1] + 1, c0[0]:c1[0] + 1][meet].sum())
        out[d] = need / len(rows) * len(simp[d])
    necessary = [0.0] + [out[d] for d in (1, 2, 3)]
    ratio = [None] + [executed_per_dim[d] / necessary[d] if necessary[d] > 0 else None for d in (1, 2, 3)]
    tot_nec = sum(necessary)
    return {"necessary_evals_per_dim_est": necessary, "executed_evals_per_dim": executed_per_dim,
            "culling_ratio_per_dim": ratio,
            "culling_ratio": sum(executed_per_dim) / tot_nec if tot_nec else None,
            "definition": "executed / necessary; necessary = points in the cells (uniform grid, h = cbrt(bbox "
                          "volume / N) = %.3g) meeting B(s, d(s,X)) for every interior sample s, estimated on "
                          "%d sampled simplices per dimension (%.1f s host)" % (h, per_dim, time.time() - t0)}


# ---------------------------------------------------------------------------
# the headline workload

def main_block(args, torch, P, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    X = synth.config_cloud(3, args.n_points)
    gen_s = time.time() - t0
    Xd = torch.from_numpy(X).to(dev)
    print("bench: generated N=%d in %.1fs" % (len(X), gen_s), file=sys.stderr, flush=True)
    idx, rad = P.fps(Xd, args.n_landmarks)
    torch.cuda.synchronize()
    t0 = time.time()
    Lxyz = X[idx.cpu().numpy()]
    cx = P.delaunay(Lxyz)
    del_ms = (time.time() - t0) * 1e3
    V, E, F, T = cx.counts()
    print("bench: Del(L) %s in %.1f ms" % (cx.counts(), del_ms), file=sys.stderr, flush=True)
    Ld = Xd[idx.long()].contiguous()
    tuning = json.loads(args.tuning) if args.tuning else None
    pb = P.problem_from_complexes(Xd, [0, len(X)], Ld, [0, len(Lxyz)], [cx], args.k, l_xidx=idx.clone())
    tune_ms = {}
    if tuning is None and not args.no_autotune:
        from paper_2509_22432_amd import autotune
        tuning, tune_ms = autotune.autotune(pb, use_cache=False)
        print("bench: autotuned %s" % tuning, file=sys.stderr, flush=True)
    run = P.api.FloodRun(pb, tuning, count_evals=False)
    hev = HipEvents(14)
    for i in range(12):
        run.out.tile_events[i] = hev.ev[i].value
    run.out.grid_events[0], run.out.grid_events[1] = hev.ev[12].value, hev.ev[13].value
    s0, s1, s2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    last = {}

    def step():
        last["idx"], _ = P.fps(Xd, args.n_landmarks, check_indices=False)
        s1.record()
        run()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if "idx" in last:
        P.api.check_landmarks(last["idx"])
    fps_ms, flood_ms, tile_ms, grid_ms = [], [], [], []
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        s0.record()
        step()
        s2.record()
        torch.cuda.synchronize()
        fps_ms.append(s0.elapsed_time(s1))
        flood_ms.append(s1.elapsed_time(s2))
        grid_ms.append(hev.elapsed_ms(12, 13))
        tile_ms.append([(hev.elapsed_ms(3 * d, 3 * d + 1), hev.elapsed_ms(3 * d + 1, 3 * d + 2))
                        if (d == 0 or pb.n(d)) and P.n_interior(d, args.k) > 0 else (0.0, 0.0) for d in range(4)])
    t_end.record()
    torch.cuda.synchronize()
    P.api.check_landmarks(last["idx"])
    assert np.array_equal(last["idx"].cpu().numpy(), idx.cpu().numpy()), "landmarks changed between steps"
    total_ms = t_start.elapsed_time(t_end)
    ms = total_ms / args.steps
    for i in range(12):
        run.out.tile_events[i] = None
    run.out.grid_events[0] = run.out.grid_events[1] = None
    hev.close()
    f_gpu = [t.cpu().numpy() for t in run.f]

    # the instrumented run: evaluation counters (a separate run, the timed
    # steps carry no counters)
    irun = P.api.FloodRun(pb, tuning, count_evals=True)
    ev_runs, stats_runs = [], []
    for _ in range(3):
        irun.evals.zero_()
        irun.stats.zero_()
        irun()
        torch.cuda.synchronize()
        ev_runs.append(int(irun.evals.item()))
        stats_runs.append(irun.stats.view(8, 4).cpu().numpy().copy())
    same = all(np.array_equal(irun.f[d].cpu().numpy(), f_gpu[d]) for d in range(4))
    del irun
    ev = int(np.median(ev_runs))
    st = np.median(np.stack(stats_runs), axis=0)
    a_ms = float(np.mean([sum(t[d][0] for d in range(4)) for t in tile_ms]))
    b_ms = float(np.mean([sum(t[d][1] for d in range(4)) for t in tile_ms]))
    a_ev, b_ev = float(st[:4, 2].sum()), float(st[:4, 3].sum())
    dominant = ("k_flood_deep", b_ev, b_ms) if b_ms >= a_ms else ("k_flood_tiles<1>", a_ev, a_ms)
    achieved = FLOP_PER_EVAL * dominant[1] / (dominant[2] * 1e-3) / 1e12
    nsimp = V + E + F + T
    n_unique = [V] + [pb.n(d) * P.n_interior(d, args.k) for d in (1, 2, 3)]
    g_ms = float(np.mean(grid_ms))
    fps_mean = float(np.mean(fps_ms))
    traffic = measured_traffic("flood::" + dominant[0], tuning)
    fps_traffic = measured_traffic("flood::k_fps_coop<0>")
    out = {
        "metric": METRIC,
        "value": ev / (ms * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mix20 surfaces N=%d, L=%d FPS landmarks, k=%d (plain, single cloud)"
                               % (len(X), args.n_landmarks, args.k),
                   "N": len(X), "L": args.n_landmarks, "k": args.k, "simplices": [V, E, F, T],
                   "tuning": tuning},
        "autotune_ms": tune_ms,
        "simplices_per_s": nsimp / (ms * 1e-3),
        "evals_per_step": ev,
        "evals_counted_in": "a separate instrumented run (median of 3); the timed steps run without counters",
        "value_basis": ("executed sample-point distance evaluations per second of the whole step; the autotuner "
                        "picks the tuning by wall time, and a tuning that culls more (smaller tiles) executes "
                        "fewer evaluations, so this rate can fall while the step gets faster: simplices_per_s "
                        "and ms_per_step compare like with like"),
        "unique_samples_per_dim": n_unique,
        "brute_force_equivalent_evals": int(sum(n_unique)) * len(X),
        "search_stats_per_dim": {"per_sample_search_ring_steps": [int(v) for v in st[:4, 0]],
                                 "per_sample_search_samples": [int(v) for v in st[:4, 1]],
                                 "per_sample_search_longest_steps": [int(v) for v in st[4:, 1]],
                                 "per_sample_searches_over_32_steps": [int(v) for v in st[4:, 2]],
                                 "tile_evals": [int(v) for v in st[:4, 2]],
                                 "tile_lane_utilisation": [float(st[d, 2] / st[4 + d, 0]) if st[4 + d, 0] else None
                                                           for d in range(4)],
                                 "per_sample_evals": [int(v) for v in st[:4, 3]]},
        "fps": {"ms": fps_mean, "rounds": args.n_landmarks,
                "us_per_round": fps_mean * 1e3 / args.n_landmarks,
                "hbm_frac": (fps_traffic / (fps_mean * 1e-3) / 1e9 / HBM_PEAK_GBS) if fps_traffic else None,
                "hbm_frac_basis": "measured k_fps_coop bytes (profiles/traffic.json) / FPS call time"},
        "grid_build": {"ms": g_ms, "algorithmic_bytes": GRID_BYTES_PER_POINT * len(X),
                       "hbm_frac": GRID_BYTES_PER_POINT * len(X) / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "stage_ms": {"fps": fps_mean, "filtration": float(np.mean(flood_ms)), "grid_build": g_ms,
                     "tile_search_per_dim": [float(np.mean([t[d][0] for t in tile_ms])) for d in range(4)],
                     "per_sample_search_per_dim": [float(np.mean([t[d][1] for t in tile_ms])) for d in range(4)],
                     "delaunay_host_once": del_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "launches_per_step": 4,
                     "kernel": dominant[0], "kernel_ms_per_step": dominant[2], "flop_per_eval": FLOP_PER_EVAL,
                     "other_search_kernel": {"k_flood_tiles": {"ms": a_ms, "evals": a_ev},
                                             "k_flood_deep": {"ms": b_ms, "evals": b_ev}}},
        "instrumented_run_bitwise_equal": bool(same),
    }
    # the persistence step after the flooding (host), outside the timed step
    ph_ms = []
    for _ in range(3):
        t0 = time.time()
        dg = P.persistence(cx, f_gpu)
        ph_ms.append((time.time() - t0) * 1e3)
    out["persistence"] = {"host_ms": float(np.median(ph_ms)), "simplices": nsimp,
                          "diagram_points_per_dim": [int(len(dg[p]["birth"])) for p in range(3)],
                          "essential_per_dim": [int(np.isinf(dg[p]["death"]).sum()) for p in range(3)]}
    step_total = fps_mean + float(np.mean(flood_ms)) + del_ms + out["persistence"]["host_ms"]
    out["stage_share_pct"] = {
        "landmark_select": 100 * fps_mean / step_total, "delaunay_host": 100 * del_ms / step_total,
        "grid_build": 100 * g_ms / step_total, "filtration": 100 * (float(np.mean(flood_ms)) - g_ms) / step_total,
        "persistence_host": 100 * out["persistence"]["host_ms"] / step_total,
        "basis": "one FPS + Del(L) + filtration + persistence pass (Table 1's stages; Del(L) and persistence "
                 "on the host)"}
    vertices_zero = bool(np.all(f_gpu[0] == 0.0))
    if not args.no_cpu_baseline:
        from oracle import flood as OF
        from oracle import native
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        t0 = time.time()
        xs = OF.XSorted(X)
        prep = time.time() - t0
        sample, oev, osec = oracle_sample(X, Lxyz, cx, args.k, args.cpu_seconds, xs)
        ns = sum(len(sample[d][0]) for d in (1, 2, 3))
        out["cpu_baseline"] = {
            "value": oev / osec, "unit": "evals/s", "cores": native.threads(), "kind": "oracle",
            "sample": "masked FP64 oracle on %d random simplices of the same complex (%.1f s; x-presort %.1f s "
                      "excluded)" % (ns, osec, prep),
            "simplices_per_s": ns / osec}
        out["simplices_per_s_gpu_vs_oracle"] = {"gpu_step": nsimp / (ms * 1e-3), "oracle": ns / osec}
        diam = OF.diameter(X)
        out["parity"] = parity_block(f_gpu, sample, diam)
        out["parity"]["vertices_zero"] = vertices_zero
        out["parity"]["ok"] = out["parity"]["ok"] and vertices_zero
        print("bench: parity %s" % out["parity"]["max_df_over_diam_per_dim"], file=sys.stderr, flush=True)
        executed = [float(st[d, 2] + st[d, 3]) for d in range(4)]
        if not args.no_culling:
            out["culling"] = culling_block(X, Lxyz, cx, args.k, sample, executed)
        del xs
    del run, pb, Xd, Ld
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# batched and differentiable forms

def batched_block(args, reps):
    """Workload 'batch512': clouds/s of the batched filtration (one HIP graph
    replay at the autotuned tiles) against the same clouds run one plain call
    at a time, and the FP32 vs FP64 error per dimension of every cloud."""
    import torch
    import synth
    from paper_2509_22432_amd import api, autotune, batch
    t0 = time.time()
    clouds, lms = synth.batched_clouds(args.batched_clouds, scale=args.batched_scale)
    print("bench: batched: %d clouds, %d points generated in %.1fs" % (len(clouds), sum(map(len, clouds)),
                                                                      time.time() - t0), file=sys.stderr, flush=True)
    t0 = time.time()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    pb, Ls, cxs = batch.prepare(clouds, lms, 6)
    prep_s = time.time() - t0
    tuning, timings = None, {}
    if not args.no_autotune:
        tuning, timings = autotune.autotune(pb, use_cache=False)
        print("bench: batched: autotuned %s" % tuning, file=sys.stderr, flush=True)
    gf = batch.GraphedFiltration(pb, tuning)
    times = []
    for _ in range(reps):
        e0.record()
        gf.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    g_ms = float(np.median(times))
    f = [t.cpu().numpy() for t in gf.run.f]
    # the counts from a separate instrumented call (the replays run without counters)
    irun = api.FloodRun(pb, tuning, count_evals=True)
    irun()
    torch.cuda.synchronize()
    evals = int(irun.evals.item())
    stats = irun.stats.view(8, 4).cpu().numpy()
    counted_equal = all(np.array_equal(irun.f[d].cpu().numpy(), f[d]) for d in range(4))
    del irun
    # the same clouds as separate plain calls (one problem per cloud)
    singles = []
    for b in range(len(clouds)):
        xo = [0, len(clouds[b])]
        Xb = torch.from_numpy(clouds[b]).cuda()
        Lb = torch.from_numpy(Ls[b]).cuda()
        li = pb.l_xidx[int(pb.l_off[b]):int(pb.l_off[b + 1])] - int(pb.x_off[b])
        p1 = api.problem_from_complexes(Xb, xo, Lb, [0, len(Ls[b])], [cxs[b]], 6, l_xidx=li.contiguous())
        singles.append(api.FloodRun(p1, tuning, count_evals=False))
    for r in singles:
        r()
    torch.cuda.synchronize()
    e0.record()
    for r in singles:
        r()
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    del singles
    V = int(pb.l_off[-1])
    n_simp = V + sum(pb.n(d) for d in (1, 2, 3))
    out = {"workload": "batch512: %d clouds, N log-uniform in [1e4, 5e5] x %.2f, 1-6 primitives, "
                       "L = min(N/100, 4096), k=6" % (len(clouds), args.batched_scale),
           "clouds_per_s": len(clouds) / (g_ms * 1e-3), "graph_replay_ms": g_ms,
           "plain_per_cloud_calls_ms": plain_ms, "plain_clouds_per_s": len(clouds) / (plain_ms * 1e-3),
           "tuning": tuning, "autotune_ms": timings,
           "points": int(pb.x_off[-1]), "landmarks": V, "simplices": n_simp, "evals": evals, "evals_counted_in": "a separate instrumented call (bit-identical f: %s)" % counted_equal,
           "search_stats_per_dim": {"per_sample_search_samples": [int(v) for v in stats[:4, 1]],
                                    "tile_evals": [int(v) for v in stats[:4, 2]],
                                    "per_sample_evals": [int(v) for v in stats[:4, 3]]},
           "host_prepare_s (fps + delaunay, untimed)": prep_s}
    if not args.no_cpu_baseline:
        out["fp32_vs_fp64"] = batched_errors(clouds, Ls, cxs, pb, f, args.batched_check, args.errors_out)
    del gf, pb
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def batched_errors(clouds, Ls, cxs, pb, f, per_dim, path):
    """max |df| / diam per dimension of every cloud, on `per_dim` random
    simplices per dimension (masked FP64 oracle)."""
    from oracle import flood as OF
    t0 = time.time()
    rng = np.random.default_rng(11)
    table = np.zeros((len(clouds), 4))
    simp_of = {1: "E", 2: "F", 3: "T"}
    for b, X in enumerate(clouds):
        diam = OF.diameter(X)
        xs = OF.XSorted(X)
        for d in range(4):
            simp = np.arange(cxs[b].L).reshape(-1, 1) if d == 0 else getattr(cxs[b], simp_of[d])
            off = int(pb.l_off[b]) if d == 0 else int(pb.s_off[d][b])
            pick = rng.choice(len(simp), min(per_dim, len(simp)), replace=False)
            ref, _, _ = OF.flood_dim(X, Ls[b], simp[pick], d, 6, "masked", xs)
            table[b, d] = np.abs(f[d][off + pick].astype(np.float64) - ref).max() / diam
    if path:
        with open(path, "w") as fh:
            json.dump({"max_df_over_diam[cloud][dim]": table.tolist(), "simplices_per_dim_per_cloud": per_dim}, fh)
    return {"max_df_over_diam_per_dim": table.max(0).tolist(),
            "median_df_over_diam_per_dim": np.median(table, 0).tolist(),
            "clouds_over_tol": int((table.max(1) > TOL).sum()), "clouds": len(clouds),
            "simplices_per_dim_per_cloud": per_dim, "host_s": time.time() - t0, "ok": bool(table.max() <= TOL)}


def differentiable_block(args, reps):
    """Workload 'twotorus64': 64 clouds of 100k points (two random tori,
    noise 0.005), L = 512, k = 6; forward + backward of
    loss = sum_sigma w_sigma f(sigma), w ~ U(0, 1)."""
    import torch
    import synth
    from paper_2509_22432_amd import api, batch
    clouds = synth.differentiable_clouds(args.diff_clouds)
    pb, Ls, cxs = batch.prepare(clouds, [512] * len(clouds), 6)
    rng = np.random.default_rng(1005)
    w = [torch.from_numpy(rng.random(pb.n(d)).astype(np.float32)).cuda() for d in range(4)]
    run = api.FloodRun(pb, None, count_evals=False)
    gX = torch.zeros_like(pb.X)
    gL = torch.zeros_like(pb.Lxyz)

    def step():
        run()
        gX.zero_()
        gL.zero_()
        run.backward(w, gX, gL)

    step()
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    fw, bw = [], []
    for _ in range(reps):
        e0.record()
        run()
        e1.record()
        gX.zero_()
        gL.zero_()
        run.backward(w, gX, gL)
        e2.record()
        torch.cuda.synchronize()
        fw.append(e0.elapsed_time(e1))
        bw.append(e1.elapsed_time(e2))
    loss = float(sum((run.f[d] * w[d]).sum() for d in range(4)))
    out = {"workload": "twotorus64: %d clouds x 100k points (two random tori, noise 0.005), L=512, k=6, "
                       "loss = sum w f, w ~ U(0,1)" % len(clouds),
           "forward_ms": float(np.median(fw)), "backward_ms": float(np.median(bw)),
           "clouds_per_s_fwd_bwd": len(clouds) / (float(np.median(fw)) + float(np.median(bw))) * 1e3,
           "simplices": int(sum(pb.n(d) for d in range(4))), "loss": loss,
           "grad_finite": bool(torch.isfinite(gX).all() and torch.isfinite(gL).all())}
    del run, pb
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# swiss-cheese stage breakdown and scaling sweeps

def one_pipeline(torch, P, X, n_lm, k, reps=3, tuning=None):
    """FPS + Del(L) + filtration + persistence of one cloud; median times."""
    Xd = torch.from_numpy(X).cuda()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    idx, _ = P.fps(Xd, n_lm)
    torch.cuda.synchronize()
    t0 = time.time()
    Lxyz = X[idx.cpu().numpy()]
    cx = P.delaunay(Lxyz)
    del_ms = (time.time() - t0) * 1e3
    pb = P.problem_from_complexes(Xd, [0, len(X)], Xd[idx.long()].contiguous(), [0, n_lm], [cx], k,
                                  l_xidx=idx.clone())
    if tuning is None:
        # the autotuner on this problem (without the candidate that skips the
        # tile search, which hands every sample to the per-sample search)
        from paper_2509_22432_amd import autotune
        tuning, _ = autotune.autotune(pb, [c for c in autotune.DEFAULT_CANDIDATES if c.get("tile_shells") != -1],
                                      use_cache=False)
    run = P.api.FloodRun(pb, tuning, count_evals=False)
    hev = HipEvents(2)
    run.out.grid_events[0], run.out.grid_events[1] = hev.ev[0].value, hev.ev[1].value
    fps_ms, fl_ms, gr_ms = [], [], []
    for _ in range(reps + 1):
        e0.record()
        P.fps(Xd, n_lm, check_indices=False)
        e1.record()
        run()
        e2.record()
        torch.cuda.synchronize()
        fps_ms.append(e0.elapsed_time(e1))
        fl_ms.append(e1.elapsed_time(e2))
        gr_ms.append(hev.elapsed_ms(0, 1))
    run.out.grid_events[0] = run.out.grid_events[1] = None
    hev.close()
    f = [t.cpu().numpy() for t in run.f]
    t0 = time.time()
    P.persistence(cx, f)
    ph_ms = (time.time() - t0) * 1e3
    med = lambda v: float(np.median(v[1:]))
    res = {"N": len(X), "L": n_lm, "k": k, "tuning": tuning, "simplices": list(cx.counts()), "fps_ms": med(fps_ms),
           "delaunay_host_ms": del_ms, "grid_build_ms": med(gr_ms), "filtration_ms": med(fl_ms) - med(gr_ms),
           "persistence_host_ms": ph_ms}
    res["total_ms"] = res["fps_ms"] + del_ms + med(fl_ms) + ph_ms
    del run, pb, Xd
    torch.cuda.empty_cache()
    return res


def sweep(args, torch, P, synth):
    rows = []
    k = args.sweep_k
    tu = json.loads(args.tuning) if args.tuning else None
    if args.sweep in ("x", "all"):
        for n in (10_000, 30_000, 100_000, 300_000, 1_000_000, 3_000_000, 10_000_000):
            X, _, _ = synth.swisscheese(n, 10, seed=2000)
            rows.append(dict(sweep="|X| at |L|=1k", **one_pipeline(torch, P, X, 1000, k, tuning=tu)))
            print("sweep x:", rows[-1], file=sys.stderr, flush=True)
    if args.sweep in ("l", "all"):
        X, _, _ = synth.swisscheese(1_000_000, 10, seed=2000)
        for nl in (250, 500, 1000, 2000, 4000, 8000, 16000):
            rows.append(dict(sweep="|L| at |X|=1M", **one_pipeline(torch, P, X, nl, k, tuning=tu)))
            print("sweep l:", rows[-1], file=sys.stderr, flush=True)
    if args.sweep in ("table", "all"):
        X, _, _ = synth.swisscheese(1_000_000, 10, seed=2000)
        rows.append(dict(sweep="Table 1: swisscheese 1M / 2k", **one_pipeline(torch, P, X, 2000, k, tuning=tu)))
        print("table:", rows[-1], file=sys.stderr, flush=True)
        X = synth.config_cloud(3)
        for nl in (2000, 10_000):
            rows.append(dict(sweep="Table 1: mix20 10M / %dk" % (nl // 1000), **one_pipeline(torch, P, X, nl, k, tuning=tu)))
            print("table:", rows[-1], file=sys.stderr, flush=True)
    for r in rows:
        tot = r["total_ms"]
        r["share_pct"] = {s: 100 * r[s + "_ms"] / tot for s in ("fps", "delaunay_host", "grid_build", "filtration",
                                                                "persistence_host")}
    res = {"k": k, "points_per_edge": k + 1, "tuning": tu or "autotuned per row", "workload": "swiss-cheese clouds: uniform in [0,5]^3 minus 10 disjoint "
                                                           "balls of radius U[0.1, 0.5] (seed 2000)", "rows": rows}
    with open(args.sweep_out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps({"sweep": args.sweep, "rows": len(rows), "out": args.sweep_out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-points", type=int, default=10_000_000)
    ap.add_argument("--n-landmarks", type=int, default=10_000)
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--tuning", type=str, default=None, help="JSON dict of flood_tuning fields")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every oracle leg")
    ap.add_argument("--no-culling", action="store_true")
    ap.add_argument("--batched-clouds", type=int, default=512, help="0 skips the batched block")
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--batched-check", type=int, default=4, help="oracle simplices per dimension per cloud")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--errors-out", type=str, default=None, help="write the per-cloud error table here")
    ap.add_argument("--diff-clouds", type=int, default=64, help="0 skips the differentiable block")
    ap.add_argument("--sweep", choices=["x", "l", "table", "all"], default=None)
    ap.add_argument("--sweep-k", type=int, default=29, help="segments per edge in the sweeps (30 points per edge)")
    ap.add_argument("--sweep-out", type=str, default="sweep.json")
    ap.add_argument("--write-traffic", type=str, default=None, metavar="PMC_DIR",
                    help="write profiles/traffic.json from rocprofv3 FETCH_SIZE/WRITE_SIZE runs under PMC_DIR "
                         "(pmc_fetch, pmc_write, pmc_copy_fetch, pmc_copy_write) taken at --tuning; no GPU")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scale for the FETCH_SIZE / "
                         "WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the flooding path here is single-GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.write_traffic:
        write_traffic(args.write_traffic, json.loads(args.tuning) if args.tuning else None)
        return
    import torch
    if args.calibrate_copy:
        n = 1 << 28
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_per_launch": n * 4, "launches": 3}), flush=True)
        return
    import paper_2509_22432_amd as P
    import synth

    if args.sweep:
        sweep(args, torch, P, synth)
        return
    out = main_block(args, torch, P, synth)
    if args.batched_clouds > 0:
        out["batched"] = batched_block(args, max(args.steps, 3))
    if args.diff_clouds > 0:
        out["differentiable"] = differentiable_block(args, max(args.steps, 3))
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    ok = out.get("parity", {}).get("ok", True) and out.get("batched", {}).get("fp32_vs_fp64", {}).get("ok", True)
    if not ok:
        print("bench: FP32 vs FP64 parity above 1e-5 * diam(X)", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
