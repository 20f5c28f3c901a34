"""Oracle, second-order rational Krylov space for a system with viscous damping (D != 0).

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

Full-order model (Section 3.3, Eq. (8)): (K + i w D - w^2 M) x = f(w). Expanding x around an
expansion point w_j in s - s_j (s = i w) gives the second-order Krylov space of Eq. (9):

    A_j r_0 = F,   A_j r_1 = -D_j r_0,   A_j r_i = -(D_j r_(i-1) + M r_(i-2)),
    A_j = K + i w_j D - w_j^2 M,   D_j = 2 i w_j M + D,

(Eq. (9) writes the operators as -A_j^{-1} D_j and -A_j^{-1} M; the printed mix of w_i, w_j
and w is read as w_j throughout). The basis spans the union over the expansion points of
{r_0, ..., r_(k_j - 1)}: here the raw vectors of the recurrence, orthonormalised by two-pass
modified Gram-Schmidt with the 1e-10 deflation rule of oracle/krylov.py. The reduced model
adds D_R = V^H D V to Eq. (11); with Rayleigh damping D = alpha M + beta K this equals
alpha M_R + beta K_R, the form the paper gives after Eq. (11).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import RationalBasis


def rayleigh(sysd, alpha, beta, structure_only=False):
    """Rayleigh damping D = alpha M + beta K on the system's own matrices (a copy of sysd with D).
    structure_only keeps the displacement block only (rows and columns < n_u): viscous damping of
    the structure, which is not proportional for the coupled system."""
    D = (alpha * sysd["M"] + beta * sysd["K"]).tocsr()
    if structure_only:
        nu = sysd["n_u"]
        keep = np.zeros(D.shape[0])
        keep[:nu] = 1.0
        S = sp.diags(keep)
        D = (S @ D @ S).tocsr()
    out = dict(sysd)
    out["D"] = D
    return out


def jacobi_scaled_d(sysd):
    """S K S, S D S, S M S, S F with S = diag(|K_ii|^{-1/2}) (the scaling of oracle/krylov.py)."""
    d = 1.0 / np.sqrt(np.abs(sysd["K"].diagonal()))
    S = sp.diags(d)
    out = dict(sysd)
    out.update(K=(S @ sysd["K"] @ S).tocsr(), M=(S @ sysd["M"] @ S).tocsr(), D=(S @ sysd["D"] @ S).tocsr(),
               F=d[:, None] * sysd["F"], scale=d)
    return out


def second_order_vectors(K, D, M, F, omega, k):
    """r_0 .. r_(k-1) of the recurrence at expansion point omega (rad/s), each n x L."""
    Aj = (K + 1j * omega * D - omega ** 2 * M).tocsc()
    Dj = 2j * omega * M + D
    lu = spla.splu(Aj)
    r = [lu.solve(F.astype(complex))]
    if k > 1:
        r.append(lu.solve(-(Dj @ r[0])))
    for i in range(2, k):
        r.append(lu.solve(-(Dj @ r[i - 1] + M @ r[i - 2])))
    return r


def build_basis(sysd, omegas_shift, blocks):
    """Orthonormal basis of the union of the second-order spaces (pass the scaled system)."""
    K, D, M, F = sysd["K"], sysd["D"], sysd["M"], sysd["F"]
    rb = RationalBasis(K.shape[0], max(1, len(omegas_shift) * blocks * F.shape[1]))
    for w in omegas_shift:
        for r in second_order_vectors(K, D, M, F, w, blocks):
            rb.add_block(r)
        rb.shifts.append(w)
    return rb


def project(sysd, V):
    """Eq. (11) with D_R: K_R, D_R, M_R, F_R, C_R (scaled system, as oracle/krylov.project)."""
    from .krylov import project as project1
    r = project1(sysd, V)
    r["DR"] = V.conj().T @ (sysd["D"] @ V)
    return r


def full_solve(sysd, omega):
    """x(w) = (K + i w D - w^2 M)^{-1} f(w) by SuperLU."""
    from .solve import load_at
    A = (sysd["K"] + 1j * omega * sysd["D"] - omega ** 2 * sysd["M"]).tocsc()
    return spla.splu(A).solve(load_at(sysd["F"], sysd["flags"], omega))
