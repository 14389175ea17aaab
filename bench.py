#!/usr/bin/env python3
"""Benchmark of the flooding path on one MI355X.

Workload (default): N = 10,000,000 float32 points on 20 noisy primitive
surfaces in the unit cube, L = 10,000 farthest-point landmarks, k = 8
segments per edge.  One step = landmark selection (GPU) + the flooding
filtration (GPU: grid build, seeds, flooding search, winners) for every
simplex of Del(L).  Del(L) is computed once on the host before the timed
region (it is combinatorial and the landmarks are identical every step).

Prints one JSON line.  `value` is executed sample-point distance
evaluations per second over the whole step; the roofline block covers the
flooding-search kernel, timed live with HIP events recorded by the library
around each of its launches.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flood distance evals/s + simplices/s at N=10M (% FP32 peak); batched clouds/s"
FP32_PEAK_TFLOPS = 157.3
FLOP_PER_EVAL = 8  # 3 sub + 1 mul + 2 fma (2 each)


def hip_runtime():
    for line in open("/proc/self/maps"):
        if "libamdhip64.so" in line:
            return ctypes.CDLL(line.split()[-1])
    return ctypes.CDLL("libamdhip64.so")


class HipEvents:
    def __init__(self, n):
        self.rt = hip_runtime()
        self.ev = [ctypes.c_void_p() for _ in range(n)]
        for e in self.ev:
            assert self.rt.hipEventCreate(ctypes.byref(e)) == 0

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) == 0
        return ms.value


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain-copy calibration),
    or None when the kernel's sources changed since the counters were taken."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        k = t["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    srcs = {"flood::k_fps_coop<0>": ["fps.hip", "internal.hpp"]}.get(kernel, ["flood.hip", "sample.hpp", "internal.hpp"])
    m = hashlib.sha256()
    for f in srcs:
        m.update(open(os.path.join(ROOT, "paper_2509_22432_amd", "csrc", f), "rb").read())
    if m.hexdigest() != k["sources_sha256"]:
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def cpu_baseline(X, Lxyz, cx, k, budget_s):
    """The oracle (masked FP64 mode) on a bounded random sample of the same
    simplices; returns its distance evaluations per second."""
    from oracle import flood as OF
    from oracle import native
    t0 = time.time()
    xs = OF.XSorted(X)
    prep = time.time() - t0
    rng = np.random.default_rng(0)
    simp = {1: cx.E, 2: cx.F, 3: cx.T}
    tot = sum(len(simp[d]) for d in (1, 2, 3))
    done_s, ev, ns = 0.0, np.zeros(1, np.int64), 0
    per = 16
    while done_s < budget_s:
        for d in (1, 2, 3):
            m = max(1, int(round(per * len(simp[d]) / tot)))
            pick = rng.choice(len(simp[d]), m, replace=False)
            t = time.time()
            OF.flood_dim(X, Lxyz, simp[d][pick], d, k, "masked", xs, counter=ev)
            done_s += time.time() - t
            ns += m
        per = min(per * 2, 4096)
    return {"value": float(ev[0] / done_s), "unit": "evals/s", "cores": native.threads(), "kind": "oracle",
            "sample": "masked FP64 oracle on %d random simplices of the same complex (%.1f s, %.0f simplices/s; "
                      "x-presort %.1f s excluded)" % (ns, done_s, ns / done_s, prep)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-points", type=int, default=10_000_000)
    ap.add_argument("--n-landmarks", type=int, default=10_000)
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--tuning", type=str, default=None, help="JSON dict of flood_tuning fields")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-clouds", type=int, default=512, help="0 skips the batched block")
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scale for the FETCH_SIZE / "
                         "WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the flooding path here is single-GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

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
    run = P.api.FloodRun(pb, tuning, count_evals=True)
    hev = HipEvents(12)
    for i in range(12):
        run.out.tile_events[i] = hev.ev[i].value
    s0, s1, s2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))

    def step():
        P.fps(Xd, args.n_landmarks)
        s1.record()
        run.evals.zero_()
        run.stats.zero_()
        run()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fps_ms, flood_ms, tile_ms, step_ms, stats_steps = [], [], [], [], []
    evals = []
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
        step_ms.append(s0.elapsed_time(s2))
        tile_ms.append([(hev.elapsed_ms(3 * d, 3 * d + 1), hev.elapsed_ms(3 * d + 1, 3 * d + 2))
                        if (d == 0 or pb.n(d)) and P.n_interior(d, args.k) > 0 else (0.0, 0.0) for d in range(4)])
        stats_steps.append(run.stats.view(4, 4).cpu().numpy().copy())
        evals.append(int(run.evals.item()))
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms = total_ms / args.steps
    ev = int(np.median(evals))
    # per phase: cooperative tile search (k_flood_tiles) and per-sample search
    # (k_flood_deep), each summed over the four dimensions
    a_ms = float(np.mean([sum(t[d][0] for d in range(4)) for t in tile_ms]))
    b_ms = float(np.mean([sum(t[d][1] for d in range(4)) for t in tile_ms]))
    st = np.mean(stats_steps, axis=0)
    a_ev, b_ev = float(st[:, 2].sum()), float(st[:, 3].sum())
    dominant = ("k_flood_deep", b_ev, b_ms) if b_ms >= a_ms else ("k_flood_tiles<1>", a_ev, a_ms)
    achieved = FLOP_PER_EVAL * dominant[1] / (dominant[2] * 1e-3) / 1e12
    nsimp = V + E + F + T
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
        "simplices_per_s": nsimp / (ms * 1e-3),
        "evals_per_step": ev,
        "search_stats_per_dim": {"per_sample_search_samples": [int(v) for v in run.stats.view(4, 4)[:, 1].cpu()],
                                 "tile_evals": [int(v) for v in run.stats.view(4, 4)[:, 2].cpu()],
                                 "per_sample_evals": [int(v) for v in run.stats.view(4, 4)[:, 3].cpu()]},
        "fps": {"ms": float(np.mean(fps_ms)), "rounds": args.n_landmarks,
                "us_per_round": float(np.mean(fps_ms)) * 1e3 / args.n_landmarks},
        "stage_ms": {"fps": float(np.mean(fps_ms)), "filtration": float(np.mean(flood_ms)),
                     "tile_search_per_dim": [float(np.mean([t[d][0] for t in tile_ms])) for d in range(4)],
                     "per_sample_search_per_dim": [float(np.mean([t[d][1] for t in tile_ms])) for d in range(4)],
                     "delaunay_host_once": del_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic("flood::" + dominant[0]),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "launches_per_step": 4,
                     "kernel": dominant[0], "kernel_ms_per_step": dominant[2], "flop_per_eval": FLOP_PER_EVAL,
                     "other_search_kernel": {"k_flood_tiles": {"ms": a_ms, "evals": a_ev},
                                             "k_flood_deep": {"ms": b_ms, "evals": b_ev}}},
    }
    # the persistence step after the flooding (host), outside the timed step
    fh = [run.f[d].detach().cpu().numpy() for d in range(4)]
    ph_ms = []
    for _ in range(3):
        t0 = time.time()
        dg = P.persistence(cx, fh)
        ph_ms.append((time.time() - t0) * 1e3)
    out["persistence"] = {"host_ms": float(np.median(ph_ms)), "simplices": nsimp,
                          "diagram_points_per_dim": [int(len(dg[p]["birth"])) for p in range(3)],
                          "essential_per_dim": [int(np.isinf(dg[p]["death"]).sum()) for p in range(3)]}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(X, Lxyz, cx, args.k, args.cpu_seconds)
    if args.batched_clouds > 0:
        del run, pb, Xd, Ld
        torch.cuda.empty_cache()
        out["batched"] = batched_block(args.batched_clouds, args.batched_scale, max(args.steps, 3))
    print(json.dumps(out), flush=True)


def batched_block(n_clouds, scale, reps):
    """Workload 'batch512': clouds/s of the batched filtration (one HIP graph
    replay) against the same clouds run one plain call at a time."""
    import torch
    import synth
    from paper_2509_22432_amd import api, batch
    t0 = time.time()
    clouds, lms = synth.batched_clouds(n_clouds, scale=scale)
    print("bench: batched: %d clouds, %d points generated in %.1fs" % (len(clouds), sum(map(len, clouds)),
                                                                      time.time() - t0), file=sys.stderr, flush=True)
    t0 = time.time()
    pb, Ls, cxs = batch.prepare(clouds, lms, 6)
    prep_s = time.time() - t0
    gf = batch.GraphedFiltration(pb)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        gf.run.evals.zero_()
        gf.run.stats.zero_()
        e0.record()
        gf.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    g_ms = float(np.median(times))
    evals = int(gf.run.evals.item())
    # the same clouds as separate plain calls (one problem per cloud)
    singles = []
    for b in range(len(clouds)):
        xo = [0, len(clouds[b])]
        Xb = torch.from_numpy(clouds[b]).cuda()
        Lb = torch.from_numpy(Ls[b]).cuda()
        li = pb.l_xidx[int(pb.l_off[b]):int(pb.l_off[b + 1])] - int(pb.x_off[b])
        p1 = api.problem_from_complexes(Xb, xo, Lb, [0, len(Ls[b])], [cxs[b]], 6, l_xidx=li.contiguous())
        singles.append(api.FloodRun(p1, None, count_evals=False))
    for r in singles:
        r()
    torch.cuda.synchronize()
    e0.record()
    for r in singles:
        r()
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    V = int(pb.l_off[-1])
    n_simp = V + sum(pb.n(d) for d in (1, 2, 3))
    return {"workload": "batch512: %d clouds, N log-uniform in [1e4, 5e5] x %.2f, 1-6 primitives, L = min(N/100, 4096), k=6"
                        % (len(clouds), scale),
            "clouds_per_s": len(clouds) / (g_ms * 1e-3), "graph_replay_ms": g_ms,
            "plain_per_cloud_calls_ms": plain_ms, "plain_clouds_per_s": len(clouds) / (plain_ms * 1e-3),
            "points": int(pb.x_off[-1]), "landmarks": V, "simplices": n_simp, "evals": evals,
            "search_stats_per_dim": {"per_sample_search_samples": [int(v) for v in gf.run.stats.view(4, 4)[:, 1].cpu()],
                                     "tile_evals": [int(v) for v in gf.run.stats.view(4, 4)[:, 2].cpu()],
                                     "per_sample_evals": [int(v) for v in gf.run.stats.view(4, 4)[:, 3].cpu()]},
            "host_prepare_s (fps + delaunay, untimed)": prep_s}


if __name__ == "__main__":
    main()
