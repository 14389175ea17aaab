"""Shared set-up for the GPU parity tests: run the HIP path end to end and
the oracle beside it, on the same seeded inputs."""
import numpy as np
import torch

import paper_2509_22432_amd as P


def dev():
    return torch.device("cuda:0")


def run_single(X, n_lm, k, tuning=None, landmarks=None, sampling="grid", seed=0):
    """FPS (GPU) -> Delaunay (host lib) -> flooding (GPU) for one cloud.
    If `landmarks` (float32 [L,3]) is given, they are used instead and are
    not assumed to be points of X."""
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev())
    if landmarks is None:
        idx, rad = P.fps(Xd, n_lm)
        torch.cuda.synchronize()
        idx_h = idx.cpu().numpy()
        Lxyz = X[idx_h]
        Ld = Xd[idx.long()].contiguous()
        lx = idx.clone()
    else:
        idx_h = None
        Lxyz = np.ascontiguousarray(landmarks, np.float32)
        Ld = torch.from_numpy(Lxyz).to(dev())
        lx = None
    cx = P.delaunay(Lxyz)
    pb = P.problem_from_complexes(Xd, [0, len(X)], Ld, [0, len(Lxyz)], [cx], k, l_xidx=lx, sampling=sampling,
                                  seed=seed)
    run = P.filtration(pb, tuning)
    torch.cuda.synchronize()
    out = dict(f=[t.cpu().numpy() for t in run.f], win_x=[t.cpu().numpy() for t in run.win_x],
               win_a=[t.cpu().numpy().view(np.uint32) for t in run.win_a],
               win_w=[t.cpu().numpy() for t in run.win_w], evals=int(run.evals.item()))
    return dict(X=X, Lxyz=Lxyz, idx=idx_h, cx=cx, pb=pb, run=run, out=out)


def oracle_complex(cx):
    return dict(E=cx.E, F=cx.F, T=cx.T, tri_edges=cx.tri_edges, tet_tris=cx.tet_tris, L=cx.L)


def unpack(a, d):
    a = np.asarray(a, np.uint32)
    return np.stack([(a >> (8 * i)) & 255 for i in range(d + 1)], 1).astype(np.int64)
