"""Exact geometric predicates on float32/float64 input (oracle).

orient(a,b,c,d) = det[a-d; b-d; c-d]; insph(a,b,c,d,e) = det of the 4x4
matrix with rows (p - e, |p - e|^2) for p in (a,b,c,d).  The point e lies
strictly inside the circumsphere of (a,b,c,d) iff insph * orient > 0.

Vectorised FP64 evaluation with a deliberately loose error filter
(|det| <= 1e-10 * permanent is "uncertain"); uncertain cases are decided in
exact rational arithmetic (every float converts exactly to a Fraction).
"""
from fractions import Fraction

import numpy as np

FILTER = 1e-10


def _det3(A, B, C):
    return (A[..., 0] * (B[..., 1] * C[..., 2] - B[..., 2] * C[..., 1])
            - A[..., 1] * (B[..., 0] * C[..., 2] - B[..., 2] * C[..., 0])
            + A[..., 2] * (B[..., 0] * C[..., 1] - B[..., 1] * C[..., 0]))


def _perm3(A, B, C):
    A, B, C = np.abs(A), np.abs(B), np.abs(C)
    return (A[..., 0] * (B[..., 1] * C[..., 2] + B[..., 2] * C[..., 1])
            + A[..., 1] * (B[..., 0] * C[..., 2] + B[..., 2] * C[..., 0])
            + A[..., 2] * (B[..., 0] * C[..., 1] + B[..., 1] * C[..., 0]))


def _fr(v):
    return [Fraction(float(x)) for x in v]


def _det3_exact(A, B, C):
    return (A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0])
            + A[2] * (B[0] * C[1] - B[1] * C[0]))


def orient_exact(a, b, c, d) -> int:
    a, b, c, d = _fr(a), _fr(b), _fr(c), _fr(d)
    A = [a[i] - d[i] for i in range(3)]
    B = [b[i] - d[i] for i in range(3)]
    C = [c[i] - d[i] for i in range(3)]
    v = _det3_exact(A, B, C)
    return (v > 0) - (v < 0)


def insph_exact(a, b, c, d, e) -> int:
    e = _fr(e)
    rows = []
    for p in (a, b, c, d):
        p = _fr(p)
        r = [p[i] - e[i] for i in range(3)]
        rows.append((r, r[0] * r[0] + r[1] * r[1] + r[2] * r[2]))
    (r0, w0), (r1, w1), (r2, w2), (r3, w3) = rows
    v = (-w0 * _det3_exact(r1, r2, r3) + w1 * _det3_exact(r0, r2, r3)
         - w2 * _det3_exact(r0, r1, r3) + w3 * _det3_exact(r0, r1, r2))
    return (v > 0) - (v < 0)


def orient_sign(a, b, c, d, skip=None):
    """Vectorised exact sign of orient; a..d are [..., 3] arrays.  Entries
    where `skip` is True are left at their FP64 sign (callers use it for
    degenerate-by-construction entries they ignore).
    Returns (int8 signs, number of exact fallbacks)."""
    a, b, c, d = (np.asarray(x, dtype=np.float64) for x in (a, b, c, d))
    a, b, c, d = np.broadcast_arrays(a, b, c, d)
    A, B, C = a - d, b - d, c - d
    det = _det3(A, B, C)
    perm = _perm3(A, B, C)
    s = np.asarray(np.sign(det), dtype=np.int8).copy()
    unsure = np.abs(det) <= FILTER * perm
    if skip is not None:
        unsure &= ~skip
    idx = np.argwhere(unsure)
    for ii in map(tuple, idx):
        s[ii] = orient_exact(a[ii], b[ii], c[ii], d[ii])
    return s, len(idx)


def insph_sign(a, b, c, d, e, skip=None):
    """Vectorised exact sign of insph (see module docstring); `skip` as in
    orient_sign."""
    a, b, c, d, e = (np.asarray(x, dtype=np.float64) for x in (a, b, c, d, e))
    a, b, c, d, e = np.broadcast_arrays(a, b, c, d, e)
    R = [p - e for p in (a, b, c, d)]
    W = [(r * r).sum(-1) for r in R]
    t0 = W[0] * _det3(R[1], R[2], R[3])
    t1 = W[1] * _det3(R[0], R[2], R[3])
    t2 = W[2] * _det3(R[0], R[1], R[3])
    t3 = W[3] * _det3(R[0], R[1], R[2])
    det = -t0 + t1 - t2 + t3
    perm = (W[0] * _perm3(R[1], R[2], R[3]) + W[1] * _perm3(R[0], R[2], R[3])
            + W[2] * _perm3(R[0], R[1], R[3]) + W[3] * _perm3(R[0], R[1], R[2]))
    s = np.asarray(np.sign(det), dtype=np.int8).copy()
    unsure = np.abs(det) <= FILTER * perm
    if skip is not None:
        unsure &= ~skip
    idx = np.argwhere(unsure)
    for ii in map(tuple, idx):
        s[ii] = insph_exact(a[ii], b[ii], c[ii], d[ii], e[ii])
    return s, len(idx)


# --------------------------------------------------------------------------
# the plane: orient2(a,b,c) = det[a-c; b-c] (positive for a counter-clockwise
# a, b, c); incircle(a,b,c,d) = det of the 3x3 matrix with rows
# (p - d, |p - d|^2), p in (a,b,c): d lies strictly inside the circle through
# a counter-clockwise (a,b,c) iff it is positive


def orient2_exact(a, b, c) -> int:
    a, b, c = _fr(a), _fr(b), _fr(c)
    v = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])
    return (v > 0) - (v < 0)


def incircle_exact(a, b, c, d) -> int:
    d = _fr(d)
    rows = []
    for p in (a, b, c):
        p = _fr(p)
        r = [p[0] - d[0], p[1] - d[1]]
        rows.append([r[0], r[1], r[0] * r[0] + r[1] * r[1]])
    v = _det3_exact(*rows)
    return (v > 0) - (v < 0)


def orient2_sign(a, b, c, skip=None):
    """Vectorised exact sign of orient2 on [..., 2] arrays; returns (int8
    signs, exact fallbacks)."""
    a, b, c = (np.asarray(x, dtype=np.float64) for x in (a, b, c))
    a, b, c = np.broadcast_arrays(a, b, c)
    A, B = a - c, b - c
    det = A[..., 0] * B[..., 1] - A[..., 1] * B[..., 0]
    perm = np.abs(A[..., 0] * B[..., 1]) + np.abs(A[..., 1] * B[..., 0])
    s = np.asarray(np.sign(det), dtype=np.int8).copy()
    unsure = np.abs(det) <= FILTER * perm
    if skip is not None:
        unsure &= ~skip
    idx = np.argwhere(unsure)
    for ii in map(tuple, idx):
        s[ii] = orient2_exact(a[ii], b[ii], c[ii])
    return s, len(idx)


def incircle_sign(a, b, c, d, skip=None):
    """Vectorised exact sign of incircle on [..., 2] arrays."""
    a, b, c, d = (np.asarray(x, dtype=np.float64) for x in (a, b, c, d))
    a, b, c, d = np.broadcast_arrays(a, b, c, d)
    R = []
    for p in (a, b, c):
        r = p - d
        R.append(np.concatenate([r, (r * r).sum(-1, keepdims=True)], axis=-1))
    det = _det3(R[0], R[1], R[2])
    perm = _perm3(R[0], R[1], R[2])
    s = np.asarray(np.sign(det), dtype=np.int8).copy()
    unsure = np.abs(det) <= FILTER * perm
    if skip is not None:
        unsure &= ~skip
    idx = np.argwhere(unsure)
    for ii in map(tuple, idx):
        s[ii] = incircle_exact(a[ii], b[ii], c[ii], d[ii])
    return s, len(idx)
