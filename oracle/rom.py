"""Oracle, step O6: the reduced frequency sweep (the MOR online phase).

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

Per frequency w (paper Section 3.3, reduced system after Eq. (10), D_R = 0 or Rayleigh
D_R = alpha M_R + beta K_R):

    (K_R + i w D_R - w^2 M_R) x_R(w) = F_R (i w)^flag ,   y_R(w) = C_R x_R(w)

solved by LAPACK's zgesv (numpy.linalg.solve), one dense solve per frequency.
"""
from __future__ import annotations

import numpy as np


def sweep(rom, omegas, DR=None):
    """Y[w, l, o] (complex128) for every frequency, load and receiver."""
    KR, MR, FR, CR, flags = rom["KR"], rom["MR"], rom["FR"], rom["CR"], rom["flags"]
    L, n_o = FR.shape[1], CR.shape[0]
    Y = np.empty((len(omegas), L, n_o), dtype=complex)
    for i, w in enumerate(omegas):
        A = KR - (w ** 2) * MR
        if DR is not None:
            A = A + 1j * w * DR
        b = FR * np.where(np.asarray(flags) == 1, 1j * w, 1.0)[None, :]
        Y[i] = (CR @ np.linalg.solve(A, b)).T
    return Y


def relative_error(Y, Yref):
    """e[w, l] = ||y - y_ref||_2 / ||y_ref||_2 over receivers; the paper's eps(w) per load."""
    return np.linalg.norm(Y - Yref, axis=2) / np.linalg.norm(Yref, axis=2)
