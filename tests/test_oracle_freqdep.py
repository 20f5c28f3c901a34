"""Pins of the oracle's frequency-dependent-material path (CPU)."""
import dataclasses

import numpy as np

import workloads as W
from oracle import assembly, freqdep, krylov, rom, solve


def _model(table_plate, table_air):
    w = W.small_plate_cavity()
    mats = []
    for m in w.mesh.materials:
        tab = table_plate if m.kind == 1 else table_air
        mats.append(dataclasses.replace(m, eta_table=tab) if tab is not None else m)
    return w, dataclasses.replace(w.mesh, materials=mats)


def test_constant_tables_reproduce_the_constant_model():
    """Tables that hold the material's own eta give exactly the frequency-independent model."""
    w, mesh = _model(((10.0, 400.0), (0.02, 0.02)), ((10.0, 400.0), (0.01, 0.01)))
    s_ref = assembly.assemble(w.mesh, w.loads, w.receivers)
    for f in (5.0, 123.0, 999.0):
        s = assembly.assemble(freqdep.mesh_at(mesh, f), w.loads, w.receivers)
        assert abs(s["K"] - s_ref["K"]).max() == 0 and abs(s["M"] - s_ref["M"]).max() == 0
    assert np.isclose(freqdep.eta_at(((10.0, 400.0), (0.01, 0.05)), 205.0), 0.03, rtol=1e-15)
    assert freqdep.eta_at(((10.0, 400.0), (0.01, 0.05)), 1.0) == 0.01
    assert freqdep.eta_at(((10.0, 400.0), (0.01, 0.05)), 1e4) == 0.05


def test_interpolation_and_moments_with_frequency_dependent_matrices():
    """The reduced model reproduces the full response (matrices at that frequency) at every
    expansion point, the first-order moments there match in backward-error form, and off the
    points the residual is larger."""
    w, mesh = _model(((10.0, 400.0), (0.005, 0.06)), ((10.0, 400.0), (0.002, 0.03)))
    shifts = 2 * np.pi * np.array([70.0, 260.0])
    rb, d = freqdep.build_basis(mesh, w.loads, w.receivers, shifts, 4)
    V = rb.basis
    assert rb.deflated == 0 and rb.q == 8
    for wj in shifts:
        s = assembly.assemble(freqdep.mesh_at(mesh, wj / (2 * np.pi)), w.loads, w.receivers)
        y = solve.full_frf(s, [wj])
        yr = freqdep.sweep(mesh, w.loads, w.receivers, V, d, [wj])
        assert rom.relative_error(yr, y).max() < 1e-9
        ss = freqdep.scaled_at(mesh, w.loads, w.receivers, wj / (2 * np.pi), d)
        A, M = ss["K"] - wj ** 2 * ss["M"], ss["M"]
        Vh = V.conj().T
        AR, MR = Vh @ (A @ V), Vh @ (M @ V)
        xr, b = np.linalg.solve(AR, Vh @ ss["F"]), ss["F"]
        for i in range(4):
            x = V @ xr
            be = np.abs(A @ x - b).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())
            assert be <= 1e-13, (wj, i)
            b, xr = M @ x, np.linalg.solve(AR, MR @ xr)
    wo = 2 * np.pi * 161.0
    ss = freqdep.scaled_at(mesh, w.loads, w.receivers, 161.0, d)
    A = ss["K"] - wo ** 2 * ss["M"]
    x = V @ np.linalg.solve(V.conj().T @ (A @ V), V.conj().T @ ss["F"])
    be = np.abs(A @ x - ss["F"]).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(ss["F"]).max())
    assert be >= 1e-10


def test_frequency_dependent_damping_changes_the_response():
    """Growing structural loss lowers the response where it grows (sanity of the direction)."""
    w, mesh = _model(((10.0, 400.0), (0.02, 0.2)), None)
    f = np.linspace(300, 400, 11)
    s0 = assembly.assemble(w.mesh, w.loads, w.receivers)
    y0 = np.array([np.abs(solve.full_frf(s0, [2 * np.pi * x])).max() for x in f])
    y1 = np.array([np.abs(solve.full_frf(assembly.assemble(freqdep.mesh_at(mesh, x), w.loads, w.receivers),
                                         [2 * np.pi * x])).max() for x in f])
    assert y1.max() < y0.max()
