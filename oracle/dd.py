"""Oracle, domain decomposition: GMRES with an additive Schwarz preconditioner on physics-based
subdomains (the iterative alternative of Section 3.2 to one full LU per frequency).

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

Subdomains follow the physical domains (Section 3.2: one subdomain per domain, here the structure
DoFs and the fluid DoFs), each grown by `overlap` layers of neighbours in the graph of the
assembled matrices: DoFs i and j are neighbours when (i, j) is an entry of K or M as assembled
(the finite-element connectivity, explicit zeros included, e.g. the coupling entries of a face
normal's zero components). The
preconditioner is the additive Schwarz sum of Section 3.2,

    M^{-1} r = sum_j R_j^T A_j^{-1} R_j r,     A_j = R_j A R_j^T,

with R_j the restriction to the (grown) subdomain j; in the restricted variant (the paper's
GASM runs use PETSc's restricted type) the prolongation R_j^T writes only the DoFs that subdomain
j owns before growing. overlap = 0 is block Jacobi. Sub-solves are exact (SuperLU), as the paper
applies a full LU per subdomain. The system is the Jacobi-scaled one of oracle/krylov.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def structure(*mats):
    """0/1 matrix of the union of the stored entries of the given CSR matrices and their
    transposes (explicit zeros count: the graph is the assembled connectivity). Pass the matrices
    as assembled: a sparse product such as the Jacobi scaling drops stored zeros."""
    n = mats[0].shape[0]
    rows, cols = [], []
    for A in mats:
        A = A.tocsr()
        r = np.repeat(np.arange(n), np.diff(A.indptr))
        rows += [r, A.indices]
        cols += [A.indices, r]
    r, c = np.concatenate(rows), np.concatenate(cols)
    G = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    G.data[:] = 1.0
    return G


def subdomains(G, n_u, overlap):
    """[(idx_j, owned_j)]: grown index set (sorted) and the mask of its owned DoFs, per physical
    domain (structure DoFs < n_u, fluid DoFs >= n_u; an empty domain is left out); G is the
    connectivity (structure(K, M))."""
    n = G.shape[0]
    out = []
    for lo, hi in ((0, n_u), (n_u, n)):
        if hi <= lo:
            continue
        mark = np.zeros(n, bool)
        mark[lo:hi] = True
        for _ in range(overlap):
            mark = mark | (G @ mark.astype(float) > 0)
        idx = np.flatnonzero(mark)
        out.append((idx, (idx >= lo) & (idx < hi)))
    return out


def preconditioner(A, doms, restricted=True):
    """z = M^{-1} r as a function of r (n x k), with one SuperLU factor per subdomain."""
    A = A.tocsr()
    facs = [spla.splu(A[idx][:, idx].tocsc()) for idx, _ in doms]

    def apply(r):
        r = np.asarray(r, complex).reshape(A.shape[0], -1)
        z = np.zeros_like(r)
        for (idx, own), lu in zip(doms, facs):
            zj = lu.solve(r[idx])
            if restricted:
                z[idx[own]] += zj[own]
            else:
                z[idx] += zj
        return z
    return apply


def gmres_right(A, b, apply_m, tol, restart, max_iter):
    """Right-preconditioned GMRES(restart) for one right-hand side: A M^{-1} y = b, x = M^{-1} y,
    modified Gram-Schmidt Arnoldi, stop when ||b - A x|| <= tol ||b||. Returns (x, iterations)."""
    n = b.shape[0]
    x = np.zeros(n, complex)
    bn = np.linalg.norm(b)
    its = 0
    while its < max_iter:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            break
        m = min(restart, max_iter - its)
        V = np.zeros((n, m + 1), complex)
        H = np.zeros((m + 1, m), complex)
        V[:, 0] = r / beta
        k = 0
        for k in range(m):
            w = A @ apply_m(V[:, k]).ravel()
            for i in range(k + 1):
                H[i, k] = np.vdot(V[:, i], w)
                w = w - H[i, k] * V[:, i]
            H[k + 1, k] = np.linalg.norm(w)
            its += 1
            e1 = np.zeros(k + 2, complex)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)
            if np.linalg.norm(H[:k + 2, :k + 1] @ y - e1) <= tol * bn or H[k + 1, k] == 0:
                k += 1
                break
            V[:, k + 1] = w / H[k + 1, k]
        else:
            k = m
        e1 = np.zeros(k + 1, complex)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
        x = x + apply_m(V[:, :k] @ y).ravel()
    return x, its
