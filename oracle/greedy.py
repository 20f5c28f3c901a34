"""Oracle, step O7: greedy (residual-maximum) choice of expansion points.

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

The paper picks expansion points iteratively in [w_min, w_max] with a greedy approach
(Section 3.3, after Eq. (9)) and notes that the classical error check by full solves can be
replaced by a cheaper estimate (Section 3.3, error-measure paragraph). This oracle uses the
relative residual of the reduced solution lifted to full order as that estimate:

    r(w_c) = || f(w_c) - A(w_c) V x_R(w_c) ||_F / || f(w_c) ||_F ,   A(w) = K - w^2 M,

taken in the Jacobi-scaled system (see oracle/krylov.py), i.e. a residual weighted by
S = diag(|K_ii|^{-1/2}) so that displacement and pressure rows count alike, and
evaluated at n_cand candidate frequencies linspace(f_lo, f_hi, n_cand). Start: the candidate
nearest the band centre (lower index on ties). Loop: add `blocks` Krylov blocks at the chosen
point, rebuild the Galerkin model, evaluate r at every candidate; stop when max r <= tol or
after max_shifts points; otherwise the next point is the unused candidate of largest r
(lower index on ties).
"""
from __future__ import annotations

import numpy as np

from .krylov import RationalBasis, jacobi_scaled, project
from .solve import load_at


def candidate_residuals(sysd, V, rom, omegas):
    K, M, F, flags = sysd["K"], sysd["M"], sysd["F"], sysd["flags"]
    KV, MV = K @ V, M @ V
    r = np.empty(len(omegas))
    for i, w in enumerate(omegas):
        f = load_at(F, flags, w)
        xr = np.linalg.solve(rom["KR"] - w ** 2 * rom["MR"], V.conj().T @ f)
        res = f - (KV @ xr - w ** 2 * (MV @ xr))
        r[i] = np.linalg.norm(res) / np.linalg.norm(f)
    return r


def first_candidate(cand_hz):
    centre = 0.5 * (cand_hz[0] + cand_hz[-1])
    d = np.abs(cand_hz - centre)
    return int(np.flatnonzero(d == d.min())[0])


def greedy(sysd, band_hz, n_cand, blocks, tol, max_shifts, stall_stop=0):
    """Return dict(basis, rom, shift_idx, shifts_hz, maxres (per iteration), res (last)).

    sysd is the assembled system; the loop runs on its Jacobi-scaled form. stall_stop > 0 also
    stops once that many expansion points in a row added no basis column (all their Krylov
    columns deflated, so the reduced model and its residuals cannot change any more)."""
    sysd = jacobi_scaled(sysd)
    cand_hz = np.linspace(band_hz[0], band_hz[1], n_cand)
    cand_w = 2 * np.pi * cand_hz
    n = sysd["K"].shape[0]
    rb = RationalBasis(n, blocks * sysd["F"].shape[1] * max_shifts)
    used, maxres = [], []
    j = first_candidate(cand_hz)
    res = None
    stalled = 0
    for _ in range(max_shifts):
        used.append(j)
        q_before = rb.q
        rb.add_shift(sysd["K"], sysd["M"], sysd["F"], cand_w[j], blocks)
        stalled = stalled + 1 if rb.q == q_before else 0
        rom = project(sysd, rb.basis)
        res = candidate_residuals(sysd, rb.basis, rom, cand_w)
        maxres.append(float(res.max()))
        if res.max() <= tol:
            break
        if stall_stop > 0 and stalled >= stall_stop:
            break
        masked = res.copy()
        masked[used] = -np.inf
        j = int(np.argmax(masked))
    rom = project(sysd, rb.basis)
    return dict(basis=rb, rom=rom, shift_idx=used, shifts_hz=cand_hz[used], maxres=maxres,
                res=res, cand_hz=cand_hz)
