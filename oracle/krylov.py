"""Oracle, steps O4-O5: rational Krylov basis and Galerkin reduced model.

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

Subspace (paper Section 3.3, Eq. (10), first-order Krylov space for complex-stiffness damping):

    colspan V = U_j K_{k_j}( A_j^{-1} M , A_j^{-1} F ),   A_j = K - w_j^2 M,

i.e. for every expansion point w_j the blocks A_j^{-1} F, (A_j^{-1} M) A_j^{-1} F, ... up to k_j
blocks. (The minus signs of Eq. (10) do not change the span.) One factorisation is kept per
expansion point and reused for all its moments (Section 3.3, offline phase).

Construction: per expansion point, an Arnoldi recurrence that applies A_j^{-1} M to the most
recent orthonormalised block and orthogonalises the result against every column so far by
two passes of modified Gram-Schmidt, column by column. Because every A_j^{-1} M is a rational
function of the same pencil, continuing from already-orthogonalised vectors spans the same
space as the union of the raw Krylov spaces.

Deflation: a new column whose norm after orthogonalisation is below 1e-10 of its norm before
is dropped. If a whole block deflates, that expansion point contributes no further blocks.

Reduced model (Eq. (11)): K_R = V^H K V, M_R = V^H M V, F_R = V^H F, C_R = C^T V (rows of V at
the receiver DoFs). The printed f_R = V^T f is read as V^H f, the Galerkin choice that matches
[.]_R = V^H [.] V.

DoF scaling. Displacement rows carry stiffness entries ~ E t (1e8) while pressure rows carry
~ h (1e-2), the scale disparity the paper points out for the coupled system (Section 3.2,
where its solver applies diagonal scaling). The basis is therefore built for the symmetrically
Jacobi-scaled system  S K S, S M S, S F  with S = diag(|K_ii|^{-1/2}), and C_R = (S C)^T V.
Since S V spans the same Krylov space and the Galerkin model does not depend on the basis
chosen for that space, the reduced outputs y_R are unchanged in exact arithmetic; only the
orthonormalisation runs on commensurate entries.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DEFLATE_TOL = 1e-10


def _mgs2_column(V, ncols, w):
    """Two passes of modified Gram-Schmidt of w against V[:, :ncols]."""
    for _ in range(2):
        for k in range(ncols):
            w = w - V[:, k] * np.vdot(V[:, k], w)
    return w


class RationalBasis:
    """Growing orthonormal basis V (n x q, complex128) of the rational Krylov space."""

    def __init__(self, n, capacity):
        self.V = np.zeros((n, capacity), dtype=complex)
        self.q = 0
        self.deflated = 0
        self.shifts = []

    def add_block(self, W):
        """Orthonormalise the columns of W against V and each other; return the accepted block."""
        acc = []
        for c in range(W.shape[1]):
            w = W[:, c].copy()
            before = np.linalg.norm(w)
            if before == 0.0:
                self.deflated += 1
                continue
            w = _mgs2_column(self.V, self.q, w)
            after = np.linalg.norm(w)
            if after < DEFLATE_TOL * before:
                self.deflated += 1
                continue
            if self.q >= self.V.shape[1]:
                self.V = np.hstack([self.V, np.zeros_like(self.V)])
            self.V[:, self.q] = w / after
            acc.append(self.q)
            self.q += 1
        return self.V[:, acc]

    def add_shift(self, K, M, F, omega, blocks):
        """Append up to `blocks` Krylov blocks at expansion point omega (rad/s)."""
        lu = spla.splu((K - omega ** 2 * M).tocsc())
        Q = self.add_block(lu.solve(F.astype(complex)))
        for _ in range(1, blocks):
            if Q.shape[1] == 0:
                break
            Q = self.add_block(lu.solve(M @ Q))
        self.shifts.append(omega)
        return lu

    @property
    def basis(self):
        return self.V[:, :self.q]


def build_basis(sysd, omegas_shift, blocks):
    """Fixed expansion points: blocks is an int or a per-shift list. Pass the scaled system."""
    K, M, F = sysd["K"], sysd["M"], sysd["F"]
    n = K.shape[0]
    bl = [blocks] * len(omegas_shift) if np.isscalar(blocks) else list(blocks)
    rb = RationalBasis(n, max(1, sum(bl) * F.shape[1]))
    for w, b in zip(omegas_shift, bl):
        rb.add_shift(K, M, F, w, b)
    return rb


def jacobi_scaled(sysd):
    """The symmetrically scaled system S K S, S M S, S F with S = diag(|K_ii|^{-1/2})."""
    d = 1.0 / np.sqrt(np.abs(sysd["K"].diagonal()))
    S = sp.diags(d)
    out = dict(sysd)
    out.update(K=(S @ sysd["K"] @ S).tocsr(), M=(S @ sysd["M"] @ S).tocsr(),
               F=d[:, None] * sysd["F"], scale=d)
    return out


def project(sysd, V):
    """Galerkin reduced model of Eq. (11) (of the scaled system when sysd carries a scale)."""
    K, M, F, recv = sysd["K"], sysd["M"], sysd["F"], sysd["recv"]
    d = sysd.get("scale")
    sr = np.ones(len(recv)) if d is None else d[recv]
    Vh = V.conj().T
    return dict(KR=Vh @ (K @ V), MR=Vh @ (M @ V), FR=Vh @ F, CR=sr[:, None] * V[recv, :],
                flags=np.asarray(sysd["flags"]).copy())
