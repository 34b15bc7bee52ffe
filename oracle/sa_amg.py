"""Oracle inner solver: PCG with a plain smoothed-aggregation AMG (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use this module.  It is a deliberately different design from the library's
preconditioner: fully algebraic greedy aggregation on a strength graph of the
2x2 node blocks, a tentative prolongator from per-aggregate QR of the three
rigid-body modes (which the viscous part of the operator annihilates), one
damped-Jacobi smoothing of the prolongator, scipy Galerkin products, and a
symmetric damped-Jacobi V-cycle with a sparse direct coarse solve.  The paper's
preconditioner (Sec. 5.4) is classical AMG inside FGMRES; here it only has to
deliver Newton directions to a stated relative tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _node_strength(A, theta):
    """Node graph of strong couplings: |A_IJ|_F >= theta sqrt(|A_II|_F |A_JJ|_F)."""
    n = A.shape[0] // 2
    Ab = sp.bsr_matrix(A, blocksize=(2, 2))
    norms = np.sqrt((Ab.data ** 2).sum(axis=(1, 2)))
    S = sp.csr_matrix((norms, Ab.indices, Ab.indptr), shape=(n, n))
    d = np.asarray(S.diagonal()).copy()
    d[d == 0] = 1.0
    S = S.tocoo()
    keep = (S.row != S.col) & (S.data >= theta * np.sqrt(d[S.row] * d[S.col]))
    return sp.csr_matrix((np.ones(keep.sum()), (S.row[keep], S.col[keep])), shape=(n, n))


def _aggregate(S, skip):
    """Greedy aggregation: roots whose strong neighbourhood is free form
    aggregates; left-over nodes join a neighbouring aggregate or form their own."""
    n = S.shape[0]
    agg = -np.ones(n, dtype=np.int64)
    agg[skip] = -2
    indptr, indices = S.indptr, S.indices
    na = 0
    for i in range(n):
        if agg[i] != -1:
            continue
        nb = indices[indptr[i]:indptr[i + 1]]
        nb = nb[agg[nb] != -2]
        if np.all(agg[nb] == -1):
            agg[i] = na
            agg[nb] = na
            na += 1
    for i in range(n):
        if agg[i] != -1:
            continue
        nb = indices[indptr[i]:indptr[i + 1]]
        nb = nb[agg[nb] >= 0]
        if nb.size:
            agg[i] = agg[nb[0]]
    for i in range(n):
        if agg[i] == -1:
            agg[i] = na
            na += 1
    return agg, na


def _tentative(agg, na, B, nodes_dofs):
    """Per-aggregate QR of the near-null-space block B (rows of the aggregate's dofs)."""
    k = B.shape[1]
    rows, cols, vals = [], [], []
    Bc = np.zeros((na * k, k))
    order = np.argsort(agg, kind="stable")
    bounds = np.searchsorted(agg[order], np.arange(na + 1))
    for a in range(na):
        nodes = order[bounds[a]:bounds[a + 1]]
        if nodes.size == 0:
            continue
        dofs = nodes_dofs(nodes)
        Q, R = np.linalg.qr(B[dofs])
        kk = Q.shape[1]
        for c in range(kk):
            rows.extend(dofs)
            cols.extend([a * k + c] * len(dofs))
            vals.extend(Q[:, c])
        Bc[a * k:a * k + kk] = R
    T = sp.csr_matrix((vals, (rows, cols)), shape=(B.shape[0], na * k))
    return T, Bc


def _lmax(A, Dinv, iters=15, seed=0):
    x = np.random.default_rng(seed).standard_normal(A.shape[0])
    lam = 1.0
    for _ in range(iters):
        y = Dinv * (A @ x)
        lam = np.linalg.norm(y) / max(np.linalg.norm(x), 1e-300)
        x = y / max(np.linalg.norm(y), 1e-300)
    return lam


class SAAMG:
    """Symmetric SA-AMG V-cycle usable as a PCG preconditioner."""

    def __init__(self, K, nxn, nyn, hx, hy, boundary, theta=0.08, max_coarse=400,
                 max_levels=10, sweeps=2, omega_s=0.6):
        self.levels = []
        self.sweeps, self.omega_s = sweeps, omega_s
        A = K.tocsr()
        jj, ii = np.divmod(np.arange(nxn * nyn), nxn)
        x = ii * hx
        y = jj * hy
        n = nxn * nyn
        B = np.zeros((2 * n, 3))
        B[0::2, 0] = 1.0
        B[1::2, 1] = 1.0
        xc, yc = x - x.mean(), y - y.mean()
        scale = max(hx * nxn, hy * nyn)
        B[0::2, 2] = -yc / scale
        B[1::2, 2] = xc / scale
        free = np.repeat(~boundary, 2)
        B[~free] = 0.0
        skip = boundary.copy()
        bs = 2
        for lev in range(max_levels):
            d = A.diagonal().copy()
            d[d == 0] = 1.0
            Dinv = 1.0 / d
            if A.shape[0] <= max_coarse or lev == max_levels - 1:
                break
            if bs == 2:
                S = _node_strength(A, theta)
            else:
                S = _node_strength_k(A, theta, bs)
            agg, na = _aggregate(S, skip)
            kk = B.shape[1]
            T, Bc = _tentative(agg, na, B, lambda nodes, b=bs: (b * nodes[:, None] + np.arange(b)).ravel())
            lam = _lmax(A, Dinv)
            P = (T - (4.0 / (3.0 * lam)) * sp.diags(Dinv) @ (A @ T)).tocsr()
            Ac = (P.T @ A @ P).tocsr()
            # coarse dofs with an empty column (rank-deficient aggregate) get identity
            dc = Ac.diagonal()
            dead = np.abs(dc) < 1e-300
            if dead.any():
                Ac = (Ac + sp.diags(dead.astype(float))).tocsr()
            self.levels.append(dict(A=A, Dinv=Dinv, P=P, lam=lam))
            A, B, bs = Ac, Bc, kk
            skip = np.zeros(A.shape[0] // bs, dtype=bool)
        self.coarse = spla.splu(A.tocsc())
        self.Ac = A

    def vcycle(self, b, lev=0):
        if lev == len(self.levels):
            return self.coarse.solve(b)
        L = self.levels[lev]
        A, Dinv, P = L["A"], L["Dinv"], L["P"]
        w = self.omega_s / L["lam"]
        x = np.zeros_like(b)
        for _ in range(self.sweeps):
            x += w * Dinv * (b - A @ x)
        x += P @ self.vcycle(P.T @ (b - A @ x), lev + 1)
        for _ in range(self.sweeps):
            x += w * Dinv * (b - A @ x)
        return x

    def __call__(self, b):
        return self.vcycle(b)


def _node_strength_k(A, theta, k):
    n = A.shape[0] // k
    Ab = sp.bsr_matrix(A, blocksize=(k, k))
    norms = np.sqrt((Ab.data ** 2).sum(axis=(1, 2)))
    S = sp.csr_matrix((norms, Ab.indices, Ab.indptr), shape=(n, n))
    d = np.asarray(S.diagonal()).copy()
    d[d == 0] = 1.0
    S = S.tocoo()
    keep = (S.row != S.col) & (S.data >= theta * np.sqrt(d[S.row] * d[S.col]))
    return sp.csr_matrix((np.ones(keep.sum()), (S.row[keep], S.col[keep])), shape=(n, n))


def pcg(A, b, M, rtol=1e-8, maxit=1000):
    """Preconditioned conjugate gradients from x = 0; returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = M(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit
