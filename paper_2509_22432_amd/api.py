"""Argument marshalling for the flood library (see package docstring)."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import Outputs, Problem, Tuning, check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _i64_host(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _dev(t, dtype, device):
    return torch.as_tensor(t, dtype=dtype).to(device).contiguous()


def _check_points(X, name):
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.shape[1] == 3 and X.is_contiguous()):
        raise ValueError("%s must be a contiguous float32 CUDA tensor of shape [n, 3]" % name)
    if X.numel() and not bool(torch.isfinite(X).all()):
        raise ValueError("%s holds non-finite coordinates" % name)


# ---------------------------------------------------------------------------
# landmarks


def fps_batched(X: torch.Tensor, x_off, n_lm, start=None, check_indices: bool = True):
    """Farthest-point landmarks for B clouds concatenated in X ([sum N, 3]).
    Returns (idx int32 [sum n_lm] local to each cloud, radius float32).

    A cooperative launch that stops hearing from its workgroups leaves -1 for
    the landmarks it did not decide; with check_indices (the default) the call
    synchronises and raises FloodError(EHIP) in that case.  Callers that time
    repeated calls pass False and check the indices themselves."""
    _check_points(X, "X")
    dev = X.device
    x_off_h, x_off_p = _i64_host(x_off)
    B = len(x_off_h) - 1
    n_lm_h = np.ascontiguousarray(np.asarray(n_lm, dtype=np.int32))
    if len(n_lm_h) != B:
        raise ValueError("n_lm must have one entry per cloud")
    # the per-cloud arrays go up in one copy: x_off and start (int64), then
    # n_lm (int32), each at an 8-byte aligned offset of one byte buffer
    start_h = np.ascontiguousarray(np.asarray(start, np.int64)) if start is not None else np.zeros(0, np.int64)
    if start is not None and len(start_h) != B:
        raise ValueError("start must have one entry per cloud")
    o_start = 8 * (B + 1)
    o_nlm = o_start + 8 * len(start_h)
    packed = np.zeros(o_nlm + 4 * B, np.uint8)
    packed[:o_start] = x_off_h.view(np.uint8)
    packed[o_start:o_nlm] = start_h.view(np.uint8)
    packed[o_nlm:] = n_lm_h.view(np.uint8)
    packed_d = torch.from_numpy(packed).to(dev)
    base = packed_d.data_ptr()
    x_off_d = ctypes.c_void_p(base)
    start_d = ctypes.c_void_p(base + o_start) if start is not None else ctypes.c_void_p(0)
    n_lm_d = ctypes.c_void_p(base + o_nlm)
    tot = int(n_lm_h.sum())
    idx = torch.empty(tot, dtype=torch.int32, device=dev)
    radius = torch.empty(tot, dtype=torch.float32, device=dev)
    L = lib()
    n_lm_p = n_lm_h.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    ws_n = L.flood_fps_workspace_size(B, x_off_p, n_lm_p)
    ws = torch.empty(max(ws_n, 1), dtype=torch.uint8, device=dev)
    check(L.flood_fps(_ptr(X), B, x_off_p, x_off_d, n_lm_p, n_lm_d, start_d, _ptr(idx),
                      _ptr(radius), _ptr(ws), ws_n, _stream()))
    if check_indices:
        check_landmarks(idx)
    return idx, radius


def check_landmarks(idx: torch.Tensor):
    """Raises FloodError(EHIP) if any landmark index is negative (an exchange
    of the cooperative FPS launch was given up)."""
    if idx.numel() and int(idx.min()) < 0:
        bad = int((idx < 0).sum())
        raise _lib.FloodError(_lib.EHIP, "flood_fps: %d landmark(s) left undecided (cooperative exchange "
                                         "gave up)" % bad)


def fps(X: torch.Tensor, n_landmarks: int, start: int = 0, check_indices: bool = True):
    """Farthest-point landmarks of one cloud: (idx int32 [L], radius float32 [L])."""
    return fps_batched(X, [0, X.shape[0]], [n_landmarks], [start], check_indices)


# ---------------------------------------------------------------------------
# Delaunay


@dataclass
class Complex:
    """Del(L) as flat arrays (rows sorted, lexicographic order); facet i of a
    row omits its i-th vertex."""
    L: int
    E: np.ndarray
    F: np.ndarray
    T: np.ndarray
    tri_edges: np.ndarray
    tet_tris: np.ndarray
    fallbacks: int = 0

    def counts(self):
        return self.L, len(self.E), len(self.F), len(self.T)


def delaunay(Lxyz) -> Complex:
    """Delaunay triangulation of landmark coordinates (host, exact
    predicates): [L, 3] gives tetrahedra; [L, 2] (ambient dimension 2) gives
    triangles, and the complex has no tetrahedra."""
    P = np.ascontiguousarray(np.asarray(Lxyz.detach().cpu() if torch.is_tensor(Lxyz) else Lxyz, dtype=np.float32))
    if P.ndim != 2 or P.shape[1] not in (2, 3):
        raise ValueError("Lxyz must be [L, 3] or [L, 2]")
    L = lib()
    h = ctypes.c_void_p()
    call = L.flood_delaunay if P.shape[1] == 3 else L.flood_delaunay2d
    check(call(P.ctypes.data_as(ctypes.c_void_p), P.shape[0], ctypes.byref(h)))
    try:
        cnt = (ctypes.c_int64 * 5)()
        check(L.flood_complex_counts(h, cnt))
        E = np.zeros((cnt[1], 2), np.int32)
        F = np.zeros((cnt[2], 3), np.int32)
        T = np.zeros((cnt[3], 4), np.int32)
        te = np.zeros((cnt[2], 3), np.int32)
        tt = np.zeros((cnt[3], 4), np.int32)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        check(L.flood_complex_export(h, vp(E), vp(F), vp(T), vp(te), vp(tt)))
    finally:
        L.flood_complex_free(h)
    return Complex(P.shape[0], E, F, T, te, tt, int(cnt[4]))


def lift_2d(P) -> np.ndarray:
    """Planar coordinates [n, 2] as the library's [n, 3] rows with z = 0 (the
    flooding kernels, the grid and the landmark rule then work in the plane:
    every z difference is exactly 0)."""
    P = np.asarray(P.detach().cpu() if torch.is_tensor(P) else P, dtype=np.float32)
    if P.ndim != 2 or P.shape[1] != 2:
        raise ValueError("expected [n, 2] coordinates")
    out = np.zeros((P.shape[0], 3), np.float32)
    out[:, :2] = P
    return out


def persistence(cx: Complex, f):
    """Persistence diagrams of the flood filtration f = (f0, f1, f2, f3) on cx
    (host library call; arrays are copied to the host).  Returns
    {p: dict(birth, death, birth_row, death_row)} for p = 0, 1, 2; essential
    classes have death = +inf and death_row = -1."""
    fh = [np.ascontiguousarray(np.asarray(v.detach().cpu() if torch.is_tensor(v) else v, dtype=np.float32))
          for v in f]
    n = (ctypes.c_int64 * 4)(*[int(x) for x in cx.counts()])
    for d in range(4):
        if fh[d].shape != (n[d],):
            raise ValueError("f[%d] must have %d entries" % (d, n[d]))
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    E = np.ascontiguousarray(cx.E, dtype=np.int32)
    te = np.ascontiguousarray(cx.tri_edges, dtype=np.int32)
    tt = np.ascontiguousarray(cx.tet_tris, dtype=np.int32)
    fp = (ctypes.c_void_p * 4)(*[vp(a) for a in fh])
    L = lib()
    h = ctypes.c_void_p()
    check(L.flood_persistence(n, vp(E), vp(te), vp(tt), fp, ctypes.byref(h)))
    try:
        cnt = (ctypes.c_int64 * 3)()
        check(L.flood_diagram_counts(h, cnt))
        out = {}
        for p in range(3):
            m = int(cnt[p])
            b, dth = np.zeros(m, np.float32), np.zeros(m, np.float32)
            br, dr = np.zeros(m, np.int64), np.zeros(m, np.int64)
            check(L.flood_diagram_export(h, p, vp(b), vp(dth), vp(br), vp(dr)))
            out[p] = dict(birth=b, death=dth, birth_row=br, death_row=dr)
    finally:
        L.flood_diagram_free(h)
    return out


# ---------------------------------------------------------------------------
# flooding


def n_interior(d: int, k: int) -> int:
    """Interior samples (all a_i >= 1) of a d-simplex at k segments per edge."""
    if d == 0:
        return 1
    from math import comb
    return comb(k - 1, d) if k - 1 >= d else 0


def own_samples(d: int, k: int, sampling: str = "grid") -> int:
    """Samples a d-simplex evaluates itself: its interior grid points, or its
    k random points (a vertex: itself)."""
    if d == 0:
        return 1
    return k if sampling == "random" else n_interior(d, k)


@dataclass
class FloodProblem:
    """Device-resident description of B clouds and their complexes, reusable
    across forward / backward / graph replays.  k: segments per edge of the
    barycentric grid (sampling "grid") or samples per simplex (sampling
    "random", drawn with the counter-based generator keyed by `seed`)."""
    B: int
    k: int
    X: torch.Tensor
    Lxyz: torch.Tensor
    l_xidx: torch.Tensor | None
    x_off: np.ndarray
    l_off: np.ndarray
    s_off: list
    simp: list
    tri_edges: torch.Tensor
    tet_tris: torch.Tensor
    dev_off: dict = field(default_factory=dict)
    sampling: str = "grid"
    seed: int = 0
    _struct: Problem | None = None

    def n(self, d):
        return int(self.l_off[-1]) if d == 0 else int(self.s_off[d][-1])

    def struct(self) -> Problem:
        if self._struct is not None:
            return self._struct
        pb = Problem()
        pb.B, pb.k = self.B, self.k
        pb.sampling = {"grid": _lib.SAMPLING_GRID, "random": _lib.SAMPLING_RANDOM}[self.sampling]
        pb.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        pb.landmarks_in_x = 1 if self.l_xidx is not None else 0
        pb.X = self.X.data_ptr()
        self._keep = []
        xo, xop = _i64_host(self.x_off)
        lo, lop = _i64_host(self.l_off)
        self._keep += [xo, lo]
        pb.x_off = xop
        pb.l_off = lop
        pb.x_off_d = self.dev_off["x"].data_ptr()
        pb.l_off_d = self.dev_off["l"].data_ptr()
        pb.Lxyz = self.Lxyz.data_ptr()
        pb.l_xidx = self.l_xidx.data_ptr() if self.l_xidx is not None else None
        for d in range(1, 4):
            so, sop = _i64_host(self.s_off[d])
            self._keep.append(so)
            pb.s_off[d] = sop
            pb.s_off_d[d] = self.dev_off[d].data_ptr()
            pb.simp[d] = self.simp[d].data_ptr() if self.simp[d].numel() else None
        zero, zp = _i64_host(np.zeros(self.B + 1))
        self._keep.append(zero)
        pb.s_off[0] = zp
        pb.tri_edges = self.tri_edges.data_ptr() if self.tri_edges.numel() else None
        pb.tet_tris = self.tet_tris.data_ptr() if self.tet_tris.numel() else None
        self._struct = pb
        return pb


def problem_from_complexes(X: torch.Tensor, x_off, Lxyz: torch.Tensor, l_off, complexes, k: int,
                           l_xidx: torch.Tensor | None = None, sampling: str = "grid",
                           seed: int = 0) -> FloodProblem:
    """Concatenate per-cloud complexes (landmark ids local to each cloud) into
    one device problem with global landmark / edge / triangle rows.
    sampling "grid": k segments per edge (Lemma 6); "random": k points drawn
    uniformly from every simplex (Lemma 9), keyed by `seed`."""
    if sampling not in ("grid", "random"):
        raise ValueError("sampling must be 'grid' or 'random'")
    _check_points(X, "X")
    _check_points(Lxyz, "Lxyz")
    dev = X.device
    x_off = np.asarray(x_off, np.int64)
    l_off = np.asarray(l_off, np.int64)
    B = len(x_off) - 1
    if len(complexes) != B or len(l_off) != B + 1:
        raise ValueError("one complex and one landmark range per cloud")
    E, F, T, TE, TT = [], [], [], [], []
    s_off = {1: [0], 2: [0], 3: [0]}
    for b, cx in enumerate(complexes):
        lb = int(l_off[b])
        E.append(cx.E.astype(np.int64) + lb)
        F.append(cx.F.astype(np.int64) + lb)
        T.append(cx.T.astype(np.int64) + lb)
        TE.append(cx.tri_edges.astype(np.int64) + s_off[1][-1])
        TT.append(cx.tet_tris.astype(np.int64) + s_off[2][-1])
        s_off[1].append(s_off[1][-1] + len(cx.E))
        s_off[2].append(s_off[2][-1] + len(cx.F))
        s_off[3].append(s_off[3][-1] + len(cx.T))
    cat = lambda xs, w: np.concatenate(xs).reshape(-1, w) if xs else np.zeros((0, w), np.int64)
    simp = [None, _dev(cat(E, 2), torch.int32, dev), _dev(cat(F, 3), torch.int32, dev), _dev(cat(T, 4), torch.int32, dev)]
    so = [None] + [np.asarray(s_off[d], np.int64) for d in (1, 2, 3)]
    dev_off = {"x": _dev(x_off, torch.int64, dev), "l": _dev(l_off, torch.int64, dev)}
    for d in (1, 2, 3):
        dev_off[d] = _dev(so[d], torch.int64, dev)
    return FloodProblem(B, k, X, Lxyz, l_xidx, x_off, l_off, so, simp,
                        _dev(cat(TE, 3), torch.int32, dev), _dev(cat(TT, 4), torch.int32, dev), dev_off,
                        sampling, seed)


def _tuning(tuning):
    if tuning is None:
        return None
    t = Tuning()
    t.cells_per_point = float(tuning.get("cells_per_point", 0.0))
    t.samples_per_lane = int(tuning.get("samples_per_lane", 0))
    t.waves_per_block = int(tuning.get("waves_per_block", 0))
    t.tile_shells = int(tuning.get("tile_shells", 0))
    t.tile_extent = int(tuning.get("tile_extent", 0))
    t.queue_grab = int(tuning.get("queue_grab", 0))
    t.tile_lanes = int(tuning.get("tile_lanes", 0))
    return t


class FloodRun:
    """Pre-allocated outputs + workspace for repeated forward calls (and for
    HIP-graph capture: the call allocates nothing).  With noalloc=True no
    workspace is allocated: the calls go to flood_filtration_noalloc, whose
    workspace is the library's static device scratch."""

    def __init__(self, pb: FloodProblem, tuning=None, count_evals=True, noalloc=False):
        self.pb = pb
        dev = pb.X.device
        self.tuning = _tuning(tuning)
        self.f = [torch.empty(pb.n(d), dtype=torch.float32, device=dev) for d in range(4)]
        self.win_x = [torch.empty(pb.n(d), dtype=torch.int32, device=dev) for d in range(4)]
        self.win_a = [torch.empty(pb.n(d), dtype=torch.int32, device=dev) for d in range(4)]
        self.win_w = [torch.empty((pb.n(d), 4), dtype=torch.float32, device=dev) for d in range(4)]
        self.evals = torch.zeros(1, dtype=torch.int64, device=dev) if count_evals else None
        self.stats = torch.zeros(32, dtype=torch.int64, device=dev) if count_evals else None
        o = Outputs()
        for d in range(4):
            o.f[d] = self.f[d].data_ptr() if self.f[d].numel() else None
            o.win_x[d] = self.win_x[d].data_ptr() if self.win_x[d].numel() else None
            o.win_a[d] = self.win_a[d].data_ptr() if self.win_a[d].numel() else None
            o.win_w[d] = self.win_w[d].data_ptr() if self.win_w[d].numel() else None
        o.evals = self.evals.data_ptr() if self.evals is not None else None
        o.stats = self.stats.data_ptr() if self.stats is not None else None
        self.out = o
        tp = ctypes.byref(self.tuning) if self.tuning is not None else None
        self.noalloc = noalloc
        self.ws, self.ws_bytes = None, 0
        if noalloc:
            return
        self.ws_bytes = lib().flood_filtration_workspace_size(ctypes.byref(pb.struct()), tp)
        if self.ws_bytes == 0:
            check(lib().flood_filtration(ctypes.byref(pb.struct()), tp, ctypes.byref(o), None, 0, _stream()))
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)

    def __call__(self):
        tp = ctypes.byref(self.tuning) if self.tuning is not None else None
        if self.noalloc:
            check(lib().flood_filtration_noalloc(ctypes.byref(self.pb.struct()), tp, ctypes.byref(self.out),
                                                 _stream()))
        else:
            check(lib().flood_filtration(ctypes.byref(self.pb.struct()), tp, ctypes.byref(self.out),
                                         _ptr(self.ws), self.ws_bytes, _stream()))
        return self.f

    def backward(self, grad_f, grad_X, grad_L):
        g = (ctypes.c_void_p * 4)()
        keep = []
        for d in range(4):
            if grad_f[d] is not None and grad_f[d].numel():
                t = grad_f[d].contiguous().float()
                keep.append(t)
                g[d] = t.data_ptr()
        check(lib().flood_filtration_backward(ctypes.byref(self.pb.struct()), ctypes.byref(self.out), g,
                                              _ptr(grad_X), _ptr(grad_L), _stream()))


def filtration(pb: FloodProblem, tuning=None, count_evals=True):
    """One forward call.  Returns the FloodRun holding f, win_x, win_a, evals.
    count_evals turns on the kernels' evaluation and search counters (per-wave
    atomics: a diagnostic run; timed and production calls pass False)."""
    run = FloodRun(pb, tuning, count_evals)
    run()
    return run


class FloodFiltration(torch.autograd.Function):
    """f = FloodFiltration.apply(X, Lxyz, pb) -> (f0, f1, f2, f3).  The
    backward routes d f(sigma) to the argmin point x* and, with the
    barycentric weights a_i/k of the winning sample, to sigma's vertices.
    X and Lxyz must be the tensors `pb` was built on."""

    @staticmethod
    def forward(ctx, X, Lxyz, pb: FloodProblem, tuning=None):
        if X.data_ptr() != pb.X.data_ptr() or Lxyz.data_ptr() != pb.Lxyz.data_ptr():
            raise ValueError("X / Lxyz must be the tensors the problem was built on")
        run = FloodRun(pb, tuning, count_evals=False)
        run()
        ctx.run = run
        return tuple(t.clone() for t in run.f)

    @staticmethod
    def backward(ctx, g0, g1, g2, g3):
        run = ctx.run
        pb = run.pb
        gX = torch.zeros_like(pb.X)
        gL = torch.zeros_like(pb.Lxyz)
        run.backward([g0, g1, g2, g3], gX, gL)
        return gX, gL, None, None
