"""Oracle, frequency-dependent materials (non-affine in the paper's sense): loss factors eta(f).

TEST INFRASTRUCTURE ONLY (see oracle/assembly.py).

The paper's matrices K(w), D(w), M(w) depend on frequency through material parameters, for
structural damping K(w) = K^ (1 + i eta(w)) (Section 3.3, text after Eq. (8)). Moments are computed
with the full-order matrices evaluated at each expansion point, and the reduced matrices are
[.]_R(w) = V^H [.](w) V at every frequency (Section 3.3, the paragraph and reduced system after
Eq. (10)). This oracle takes that literally: at every frequency it reassembles the model with
each table material's loss factor eta(f) (piecewise-linear interpolation of its (f_hz, eta)
samples, constant beyond the ends) and projects the assembled matrices onto V.

Scaling: the basis is built for S K S, S M S, S F with S = diag(|K_ii|^{-1/2}) taken from the
model assembled with every table material's loss factor set to zero (one S for all frequencies).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import assembly
from .krylov import RationalBasis


def eta_at(table, f_hz):
    f, e = table
    return float(np.interp(f_hz, f, e))


def mesh_at(mesh, f_hz, zero=False):
    """The mesh with every table material's eta replaced by eta(f_hz) (or by 0)."""
    mats = []
    for m in mesh.materials:
        tab = getattr(m, "eta_table", None)
        if tab is not None:
            m = dataclasses.replace(m, eta=0.0 if zero else eta_at(tab, f_hz), eta_table=None)
        mats.append(m)
    return dataclasses.replace(mesh, materials=mats)


def scale(mesh, loads, receivers):
    s0 = assembly.assemble(mesh_at(mesh, 0.0, zero=True), loads, receivers)
    return 1.0 / np.sqrt(np.abs(s0["K"].diagonal()))


def scaled_at(mesh, loads, receivers, f_hz, d):
    s = assembly.assemble(mesh_at(mesh, f_hz), loads, receivers)
    S = sp.diags(d)
    out = dict(s)
    out.update(K=(S @ s["K"] @ S).tocsr(), M=(S @ s["M"] @ S).tocsr(), F=d[:, None] * s["F"], scale=d)
    return out


def build_basis(mesh, loads, receivers, omegas_shift, blocks):
    """Eq. (10) with the matrices of each expansion point: A_j = K(w_j) - w_j^2 M(w_j), M(w_j).

    The pencils differ between expansion points, so the recurrence of one point continues from
    its own vectors only (orthonormalised among themselves), and each of its blocks is then added
    to the global basis; continuing from vectors orthogonalised against other points' vectors
    (valid for one fixed pencil, oracle/krylov.py) would leave this point's space."""
    import scipy.sparse.linalg as spla
    d = scale(mesh, loads, receivers)
    rb = None
    for w in omegas_shift:
        sj = scaled_at(mesh, loads, receivers, w / (2 * np.pi), d)
        n, L = sj["F"].shape
        if rb is None:
            rb = RationalBasis(n, max(1, len(omegas_shift) * blocks * L))
        lu = spla.splu((sj["K"] - w ** 2 * sj["M"]).tocsc())
        local = RationalBasis(n, max(1, blocks * L))
        X = lu.solve(sj["F"].astype(complex))
        for _ in range(blocks):
            Q = local.add_block(X)
            rb.add_block(Q)
            if Q.shape[1] == 0:
                break
            X = lu.solve(sj["M"] @ Q)
        rb.shifts.append(w)
    return rb, d


def sweep(mesh, loads, receivers, V, d, omegas):
    """Y[w, l, o]: K_R(w) = V^H K(w) V, M_R(w) = V^H M(w) V from the model reassembled at each w."""
    Vh = V.conj().T
    out = None
    for i, w in enumerate(omegas):
        s = scaled_at(mesh, loads, receivers, w / (2 * np.pi), d)
        KR, MR, FR = Vh @ (s["K"] @ V), Vh @ (s["M"] @ V), Vh @ s["F"]
        CR = d[s["recv"]][:, None] * V[s["recv"], :]
        b = FR * np.where(np.asarray(s["flags"]) == 1, 1j * w, 1.0)[None, :]
        y = (CR @ np.linalg.solve(KR - w ** 2 * MR, b)).T
        if out is None:
            out = np.empty((len(omegas),) + y.shape, dtype=complex)
        out[i] = y
    return out
