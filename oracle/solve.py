"""Oracle, step O3: full-order frequency response by a direct sparse solve per frequency.

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

The reference solution strategy of the paper (Section 2) factors A(w) = K - w^2 M at every
frequency and solves A(w) x = f(w); the output is y = C^T x, here the pressures at the
receiver DoFs (Eq. (8), D = 0 because damping is carried by the complex stiffness).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def load_at(F, flags, omega):
    """f(w) = (i w)^flag * F, column by column."""
    return F * np.where(np.asarray(flags) == 1, 1j * omega, 1.0)[None, :]


def system_matrix(K, M, omega):
    return (K - (omega ** 2) * M).tocsc()


def full_solve(K, M, F, flags, omega, dense=False):
    """x(w) = A(w)^{-1} f(w) with SuperLU (or LAPACK zgesv when dense=True)."""
    A = system_matrix(K, M, omega)
    b = load_at(F, flags, omega)
    if dense:
        return np.linalg.solve(A.toarray(), b)
    return spla.splu(A).solve(b)


def full_frf(sysd, omegas, dense=False):
    """Y[w, l, o] = receiver pressure o for load l at frequency w (complex128)."""
    K, M, F, flags, recv = sysd["K"], sysd["M"], sysd["F"], sysd["flags"], sysd["recv"]
    Y = np.empty((len(omegas), F.shape[1], len(recv)), dtype=complex)
    for i, w in enumerate(omegas):
        x = full_solve(K, M, F, flags, w, dense=dense)
        Y[i] = x[recv, :].T
    return Y
