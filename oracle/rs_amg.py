"""Oracle for classical (Ruge-Stueben) AMG with the paper's settings (test infrastructure).

Only the test suite may use this module.  It follows the preconditioner the
paper reports in Sec. 5.4: classical AMG in a V-cycle, strong threshold 0.5
instead of the usual 0.25, three symmetric Gauss-Seidel (SSOR with unit
relaxation) sweeps per smoothing on every level, and Gaussian elimination on the
coarsest level.  The pieces are the textbook ones, written plainly:

* strength of connection: j strongly influences i when -a_ij >= theta *
  max_{k != i} (-a_ik) (sign taken relative to a_ii); rows whose |row sum|
  exceeds max_row_sum |a_ii| (strongly diagonally dominant rows) have no strong
  connections;
* coarsening: the Ruge-Stueben first pass (largest measure first; new C point
  makes its strong dependents F; measures updated), sequential here;
* interpolation: classical interpolation with strong F neighbours distributed
  over the common strong C neighbours (only couplings of the sign opposite to the
  neighbour's diagonal count; a neighbour without such couplings is lumped into
  the diagonal) and weak connections lumped into the diagonal;
* Galerkin coarse operators P^T A P (scipy products: the definition);
* multicolour symmetric Gauss-Seidel: rows of one colour are not coupled, so a
  colour is relaxed at once; forward over the colours then backward is one
  symmetric sweep.

The coarsening and the colouring are not unique; functions that take a C/F
splitting or a colouring as an argument accept any valid one, so the GPU's
hierarchy can be rebuilt here from its own splitting and colouring.
"""
from __future__ import annotations

import heapq

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

C_PT, F_PT = 1, 0


def strength(A, theta=0.5, max_row_sum=0.9):
    """Boolean CSR S: S[i, j] true when j strongly influences i (i != j)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows, cols = [], []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        js, vs = A.indices[lo:hi], A.data[lo:hi]
        d = vs[js == i].sum()
        if max_row_sum < 1.0 and abs(vs.sum()) > max_row_sum * abs(d):
            continue
        sgn = -1.0 if d >= 0.0 else 1.0
        off = [(j, sgn * v) for j, v in zip(js, vs) if j != i]
        if not off:
            continue
        m = max(v for _, v in off)
        if m <= 0.0:
            continue
        for j, v in off:
            if v >= theta * m:
                rows.append(i)
                cols.append(j)
    return sp.csr_matrix((np.ones(len(rows), dtype=bool), (rows, cols)), shape=(n, n))


def rs_first_pass(S):
    """Sequential Ruge-Stueben first pass.  Measure lam_i = number of undecided
    points that strongly depend on i plus twice the F points that do; the largest
    undecided measure becomes C (ties: the lower index), its undecided strong
    dependents become F, and the measures of the points they depend on grow.
    Points that nothing depends on are F from the start."""
    S = sp.csr_matrix(S)
    n = S.shape[0]
    ST = sp.csr_matrix(S.T)
    lam = np.diff(ST.indptr).astype(np.int64)
    state = np.full(n, -1, dtype=np.int64)
    state[lam == 0] = F_PT
    heap = [(-lam[i], i) for i in range(n) if state[i] < 0]
    heapq.heapify(heap)
    while heap:
        ml, i = heapq.heappop(heap)
        if state[i] >= 0 or -ml != lam[i]:
            continue
        if lam[i] == 0:
            state[i] = F_PT
            continue
        state[i] = C_PT
        for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]]:
            if state[j] < 0:
                state[j] = F_PT
                for k in S.indices[S.indptr[j]:S.indptr[j + 1]]:
                    if state[k] < 0:
                        lam[k] += 1
                        heapq.heappush(heap, (-lam[k], k))
        for k in S.indices[S.indptr[i]:S.indptr[i + 1]]:
            if state[k] < 0:
                lam[k] -= 1
                heapq.heappush(heap, (-lam[k], k))
    return state


def interpolation(A, S, cf):
    """Classical interpolation P (n x nc); coarse points numbered in fine order."""
    A = sp.csr_matrix(A)
    S = sp.csr_matrix(S)
    n = A.shape[0]
    cidx = -np.ones(n, dtype=np.int64)
    cidx[cf == C_PT] = np.arange(int((cf == C_PT).sum()))
    rows, cols, vals = [], [], []

    def entry(r, c):
        lo, hi = A.indptr[r], A.indptr[r + 1]
        hit = np.nonzero(A.indices[lo:hi] == c)[0]
        return A.data[lo + hit[0]] if hit.size else 0.0

    for i in range(n):
        if cf[i] == C_PT:
            rows.append(i)
            cols.append(cidx[i])
            vals.append(1.0)
            continue
        strong = set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist())
        Ci = [j for j in sorted(strong) if cf[j] == C_PT]
        if not Ci:
            continue
        lo, hi = A.indptr[i], A.indptr[i + 1]
        diag = 0.0
        num = {k: 0.0 for k in Ci}
        strongF = []
        for j, a in zip(A.indices[lo:hi], A.data[lo:hi]):
            if j == i:
                diag += a
            elif j in strong and cf[j] == C_PT:
                num[j] += a
            elif j in strong:
                strongF.append((j, a))
            else:
                diag += a  # weak connection: lumped
        for m, aim in strongF:
            smm = np.sign(entry(m, m))
            amk = {k: entry(m, k) for k in Ci}
            use = [k for k in Ci if amk[k] * smm < 0.0]
            den = sum(amk[k] for k in use)
            if den == 0.0:
                diag += aim
                continue
            for k in use:
                num[k] += aim * amk[k] / den
        for k in Ci:
            rows.append(i)
            cols.append(cidx[k])
            vals.append(-num[k] / diag)
    nc = int((cf == C_PT).sum())
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def galerkin(A, P):
    """Coarse operator P^T A P."""
    return sp.csr_matrix(P.T @ sp.csr_matrix(A) @ P)


def is_valid_colouring(A, colours):
    A = sp.coo_matrix(A)
    off = A.row != A.col
    return bool(np.all(colours[A.row[off]] != colours[A.col[off]]))


def greedy_colouring(A):
    """Sequential first-fit colouring of the graph of A's off-diagonal entries."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    col = -np.ones(n, dtype=np.int64)
    for i in range(n):
        used = {col[j] for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j != i and col[j] >= 0}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def sgs(A, b, x, colours, sweeps):
    """`sweeps` symmetric multicolour Gauss-Seidel sweeps (forward over the colours,
    then backward), x updated from its value on entry."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    nc = int(colours.max()) + 1 if colours.size else 0
    groups = [np.nonzero(colours == c)[0] for c in range(nc)]
    x = x.copy()
    for _ in range(sweeps):
        for order in (range(nc), range(nc - 1, -1, -1)):
            for c in order:
                rows = groups[c]
                if rows.size == 0:
                    continue
                r = b[rows] - A[rows] @ x
                x[rows] += r / d[rows]
    return x


class RSHierarchy:
    """Levels (A_l, P_l, colours_l) and the V-cycle over them.  Built from the
    oracle's own sequential coarsening and colouring, or from given splittings and
    colourings (those of another implementation)."""

    def __init__(self, A, theta=0.5, max_row_sum=0.9, sweeps=3, max_coarse=140, max_levels=25,
                 splittings=None, colourings=None):
        self.sweeps = sweeps
        self.A, self.P, self.colours = [sp.csr_matrix(A)], [], []
        l = 0
        while self.A[-1].shape[0] > max_coarse and len(self.A) < max_levels:
            Al = self.A[-1]
            S = strength(Al, theta, max_row_sum)
            cf = splittings[l] if splittings is not None else rs_first_pass(S)
            nc = int((cf == C_PT).sum())
            if nc == 0 or nc == Al.shape[0]:
                break
            P = interpolation(Al, S, cf)
            self.P.append(P)
            self.colours.append(colourings[l] if colourings is not None else greedy_colouring(Al))
            self.A.append(galerkin(Al, P))
            l += 1
        self.coarse = np.linalg.inv(self.A[-1].toarray()) if self.A[-1].shape[0] else np.zeros((0, 0))

    def vcycle(self, b, l=0):
        if l == len(self.P):
            return self.coarse @ b
        A = self.A[l]
        x = sgs(A, b, np.zeros_like(b), self.colours[l], self.sweeps)
        r = b - A @ x
        xc = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return sgs(A, b, x, self.colours[l], self.sweeps)

    def operator(self):
        n = self.A[0].shape[0]
        return spla.LinearOperator((n, n), matvec=self.vcycle, dtype=np.float64)
