"""Oracle, local reduced models on frequency windows (l-fROMs).

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

For high modal density the paper partitions the broad band into sub-intervals and builds one
local reduced model per window (Section 3.3, local-fROM paragraph and its schematic figure;
windows of Tab. 4); the paper chose its windows by hand and names an automated partition as
future work. The partition used here is automated by bisection:

  build(window):  run the residual-maximum greedy (oracle/greedy.py) on the window's own
                  candidates with at most max_shifts expansion points;
                  if its largest candidate residual is <= tol, or the window holds fewer than
                  2 min_cand - 1 candidates, keep the window and its model;
                  otherwise split the window's candidates at the middle index (the middle
                  candidate belongs to both halves) and build both halves, left first.

Windows are index ranges [i0, i1] of the global candidate grid linspace(f_lo, f_hi, n_cand); a
window's greedy sees the candidates linspace(cand[i0], cand[i1], i1 - i0 + 1). The stitched
sweep evaluates frequency f with the model of the first window (in increasing frequency) whose
upper edge is >= f, the last window above the band.
"""
from __future__ import annotations

import numpy as np

from .greedy import greedy
from .rom import sweep as rom_sweep


def local_roms(sysd, band_hz, n_cand, blocks, tol, max_shifts, min_cand):
    """Return a list of dict(i0, i1, lo_hz, hi_hz, greedy=<oracle greedy result>) in increasing
    frequency order."""
    cand = np.linspace(band_hz[0], band_hz[1], n_cand)
    out = []

    def build(i0, i1):
        k = i1 - i0 + 1
        g = greedy(sysd, (cand[i0], cand[i1]), k, blocks, tol, max_shifts)
        if g["maxres"][-1] <= tol or k < 2 * min_cand - 1:
            out.append(dict(i0=i0, i1=i1, lo_hz=cand[i0], hi_hz=cand[i1], greedy=g))
            return
        mid = (i0 + i1) // 2
        build(i0, mid)
        build(mid, i1)

    build(0, n_cand - 1)
    return out


def window_of(windows, f_hz):
    """Index of the window that evaluates frequency f_hz."""
    for k, w in enumerate(windows):
        if f_hz <= w["hi_hz"]:
            return k
    return len(windows) - 1


def sweep(windows, omegas):
    """Stitched sweep Y[w, l, o] of the local models."""
    omegas = np.asarray(omegas, float)
    owner = np.array([window_of(windows, om / (2 * np.pi)) for om in omegas], int)
    first = windows[0]["greedy"]["rom"]
    Y = np.empty((len(omegas), first["FR"].shape[1], first["CR"].shape[0]), dtype=complex)
    for k, w in enumerate(windows):
        sel = np.flatnonzero(owner == k)
        if len(sel):
            Y[sel] = rom_sweep(w["greedy"]["rom"], omegas[sel])
    return Y, owner
