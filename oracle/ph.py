"""Persistent homology over Z/2 and bottleneck matching (oracle).

The filtration induced by f on the complex (Sec. 2, "Preliminaries": the
sublevel complexes f^{-1}((-inf, t])) is turned into a simplex order by
(f, dimension, sorted vertex tuple).  Diagrams come from the standard
column reduction of the boundary matrix (the algorithm the paper cites as
the cubic-worst-case reduction), with the clearing shortcut.  The bottleneck
test decides d_B <= tol as a perfect-matching feasibility question
(Sec. 2, definition of d_B: bijections with the diagonal of infinite
multiplicity).
"""
import numpy as np


def filtration_order(cx, fvals):
    """cx: dict with 'L' (number of vertices), 'E','F','T'; fvals: {d: f}.
    Returns (simplex list as tuples, dims, values) in filtration order."""
    simp = [(v,) for v in range(cx["L"])]
    dims = [0] * cx["L"]
    vals = list(np.asarray(fvals[0], dtype=np.float64))
    for d, key in ((1, "E"), (2, "F"), (3, "T")):
        rows = [tuple(int(x) for x in r) for r in np.asarray(cx[key])]
        simp += rows
        dims += [d] * len(rows)
        vals += list(np.asarray(fvals[d], dtype=np.float64))
    order = sorted(range(len(simp)), key=lambda i: (vals[i], dims[i], simp[i]))
    return [simp[i] for i in order], [dims[i] for i in order], [vals[i] for i in order]


def boundary_columns(simp):
    pos = {s: i for i, s in enumerate(simp)}
    cols = []
    for s in simp:
        if len(s) == 1:
            cols.append(set())
        else:
            cols.append({pos[s[:i] + s[i + 1:]] for i in range(len(s))})
    return cols


def reduce_pairs(simp, dims):
    """Column reduction with clearing.  Returns (pairs [(i, j)], essential [i])
    as positions in the filtration order."""
    cols = boundary_columns(simp)
    n = len(simp)
    low_of = {}
    cleared = [False] * n
    pairs = []
    maxd = max(dims) if dims else 0
    for d in range(maxd, 0, -1):
        for j in range(n):
            if dims[j] != d or cleared[j]:
                continue
            c = cols[j]
            while c:
                lo = max(c)
                if lo in low_of:
                    c ^= cols[low_of[lo]]
                else:
                    low_of[lo] = j
                    pairs.append((lo, j))
                    cleared[lo] = True
                    cols[lo] = set()
                    break
            cols[j] = c
    killed = set(i for i, _ in pairs)
    creators = set(j for _, j in pairs)
    essential = [i for i in range(n) if not cols[i] and i not in killed and i not in creators]
    return pairs, essential


def diagrams(cx, fvals, maxdim=2, drop_zero=True):
    """Persistence diagrams dims 0..maxdim: {p: (finite [m,2], essential births [e])}."""
    simp, dims, vals = filtration_order(cx, fvals)
    pairs, ess = reduce_pairs(simp, dims)
    out = {}
    for p in range(maxdim + 1):
        fin = [(vals[i], vals[j]) for i, j in pairs if dims[i] == p]
        if drop_zero:
            fin = [(b, d) for b, d in fin if d > b]
        out[p] = (np.array(fin, dtype=np.float64).reshape(-1, 2),
                  np.sort(np.array([vals[i] for i in ess if dims[i] == p], dtype=np.float64)))
    return out


def bottleneck_leq(A, B, tol) -> bool:
    """d_B(A, B) <= tol for diagrams given as (finite [m,2], essential births).
    Essential classes must match in number; sorted births pair off optimally
    in the sup norm.  Finite points: perfect matching in the bipartite graph
    A + diag(B) versus B + diag(A)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_bipartite_matching
    (fa, ea), (fb, eb) = A, B
    if len(ea) != len(eb):
        return False
    if len(ea) and np.max(np.abs(np.sort(ea) - np.sort(eb))) > tol:
        return False
    na, nb = len(fa), len(fb)
    n = na + nb
    if n == 0:
        return True
    rows, cols = [], []
    if na and nb:
        D = np.maximum(np.abs(fa[:, None, 0] - fb[None, :, 0]), np.abs(fa[:, None, 1] - fb[None, :, 1]))
        r, c = np.nonzero(D <= tol)
        rows += list(r)
        cols += list(c)
    # a_i -> its own diagonal slot (column nb + i) if close to the diagonal
    for i in range(na):
        if (fa[i, 1] - fa[i, 0]) / 2 <= tol:
            rows.append(i)
            cols.append(nb + i)
    # diagonal slot of b_j (row na + j) -> b_j if close to the diagonal
    for j in range(nb):
        if (fb[j, 1] - fb[j, 0]) / 2 <= tol:
            rows.append(na + j)
            cols.append(j)
    # diagonal to diagonal, always
    for j in range(nb):
        for i in range(na):
            rows.append(na + j)
            cols.append(nb + i)
    M = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    match = maximum_bipartite_matching(M, perm_type="column")
    return bool(np.all(match >= 0))


# ---------------------------------------------------------------------------
# independent check: persistence from ranks (tiny complexes only)


def _rank_gf2(M: np.ndarray) -> int:
    M = (np.asarray(M) % 2).astype(np.uint8).copy()
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = np.nonzero(M[r:, c])[0]
        if len(piv) == 0:
            continue
        p = r + piv[0]
        M[[r, p]] = M[[p, r]]
        others = np.nonzero(M[:, c])[0]
        others = others[others != r]
        M[others] ^= M[r]
        r += 1
        if r == rows:
            break
    return r


def rank_invariant_pairs(simp, dims, maxdim=2):
    """Index-persistence multiplicities mu_p(i, j) from persistent Betti
    numbers beta_p(i, j) = dim Z_p(K_i) - dim(B_p(K_j) cap C_p(K_i)),
    where K_i is the first i+1 simplices.  Returns {p: sorted list of (i, j)}
    with j = None for essential classes."""
    n = len(simp)
    pos = {s: i for i, s in enumerate(simp)}
    D = np.zeros((n, n), dtype=np.uint8)
    for j, s in enumerate(simp):
        if len(s) > 1:
            for t in range(len(s)):
                D[pos[s[:t] + s[t + 1:]], j] = 1
    dims = np.asarray(dims)

    def beta(p, i, j):
        if i < 0:
            return 0
        Ki = np.arange(n) <= i
        Kj = np.arange(n) <= j
        cp_i = np.nonzero(Ki & (dims == p))[0]
        cm = np.nonzero(dims == p - 1)[0]
        z = len(cp_i) - (_rank_gf2(D[np.ix_(cm, cp_i)]) if p > 0 and len(cp_i) else 0)
        cq_j = np.nonzero(Kj & (dims == p + 1))[0]
        if len(cq_j) == 0:
            return z
        Bj = D[np.ix_(np.nonzero(dims == p)[0], cq_j)]
        pdims = np.nonzero(dims == p)[0]
        outside = ~Ki[pdims]
        inter = _rank_gf2(Bj) - _rank_gf2(Bj[outside]) if outside.any() else _rank_gf2(Bj)
        return z - inter

    out = {}
    for p in range(maxdim + 1):
        res = []
        for i in range(n):
            if dims[i] != p:
                continue
            for j in range(i + 1, n):
                mu = beta(p, i, j - 1) - beta(p, i, j) - beta(p, i - 1, j - 1) + beta(p, i - 1, j)
                res += [(i, j)] * mu
            mu_inf = beta(p, i, n - 1) - beta(p, i - 1, n - 1)
            res += [(i, None)] * mu_inf
        out[p] = sorted(res, key=lambda t: (t[0], -1 if t[1] is None else t[1]))
    return out
