"""Pins of the oracle's second-order Krylov space (viscous damping, Eq. (9)) on the CPU."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assembly, krylov, rom, soar, solve


@pytest.fixture(scope="module")
def damped():
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    sd = soar.rayleigh(s, 40.0, 2e-5, structure_only=True)
    return w, s, sd, soar.jacobi_scaled_d(sd)


def test_second_order_moments_match_in_backward_error(damped):
    """The lifted reduced moments satisfy the full second-order recurrence at every expansion
    point (normwise backward error at rounding level); off the points the model's own residual
    is far larger, so the check discriminates."""
    _, _, _, ss = damped
    shifts = 2 * np.pi * np.array([60.0, 250.0])
    k = 4
    rb = soar.build_basis(ss, shifts, k)
    assert rb.deflated == 0 and rb.q == len(shifts) * k
    V, r = rb.basis, soar.project(ss, rb.basis)
    K, D, M, F = ss["K"], ss["D"], ss["M"], ss["F"]

    def berr(A, x, b):
        return np.abs(A @ x - b).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())

    for w in shifts:
        A, Dj = K + 1j * w * D - w ** 2 * M, 2j * w * M + D
        AR, DjR = r["KR"] + 1j * w * r["DR"] - w ** 2 * r["MR"], 2j * w * r["MR"] + r["DR"]
        xr = [np.linalg.solve(AR, r["FR"])]
        xr.append(np.linalg.solve(AR, -(DjR @ xr[0])))
        for i in range(2, k):
            xr.append(np.linalg.solve(AR, -(DjR @ xr[i - 1] + r["MR"] @ xr[i - 2])))
        x = [V @ v for v in xr]
        assert berr(A, x[0], F) <= 1e-13
        assert berr(A, x[1], -(Dj @ x[0])) <= 1e-13
        for i in range(2, k):
            assert berr(A, x[i], -(Dj @ x[i - 1] + M @ x[i - 2])) <= 1e-13, (w, i)
    w = 2 * np.pi * 151.0
    A = K + 1j * w * D - w ** 2 * M
    xr = np.linalg.solve(r["KR"] + 1j * w * r["DR"] - w ** 2 * r["MR"], r["FR"])
    assert berr(A, V @ xr, F) >= 1e-9


def test_interpolation_of_the_damped_response(damped):
    """The reduced model reproduces the full damped FRF at every expansion point."""
    _, s, sd, ss = damped
    shifts = 2 * np.pi * np.array([60.0, 250.0])
    rb = soar.build_basis(ss, shifts, 3)
    r = soar.project(ss, rb.basis)
    for w in shifts:
        y = soar.full_solve(sd, w)[s["recv"]].T[None]
        yr = rom.sweep(r, [w], DR=r["DR"])
        assert rom.relative_error(yr, y).max() < 1e-9


def test_without_damping_the_second_order_space_is_the_first_order_one(damped):
    """D = 0: the Taylor coefficients in s = i w and in w^2 at w_j != 0 span the same space, so
    the second-order basis equals the first-order one of Eq. (10) (all principal angles ~ 0)."""
    _, s, _, _ = damped
    s0 = soar.rayleigh(s, 0.0, 0.0)
    ss0 = soar.jacobi_scaled_d(s0)
    shifts = 2 * np.pi * np.array([80.0, 300.0])
    V2 = soar.build_basis(ss0, shifts, 3).basis
    V1 = krylov.build_basis(krylov.jacobi_scaled(s), shifts, 3).basis
    sv = sla.svdvals(V1.conj().T @ V2)
    assert V1.shape == V2.shape and sv.min() > 1 - 1e-8


def test_rayleigh_projection_equals_the_reduced_rayleigh_form(damped):
    """D = alpha M + beta K gives D_R = alpha M_R + beta K_R (the paper's reduced Rayleigh form)."""
    _, s, _, _ = damped
    ss = soar.jacobi_scaled_d(soar.rayleigh(s, 4.0, 2e-6))
    rb = soar.build_basis(ss, 2 * np.pi * np.array([100.0]), 3)
    r = soar.project(ss, rb.basis)
    assert np.abs(r["DR"] - (4.0 * r["MR"] + 2e-6 * r["KR"])).max() <= 1e-12 * np.abs(r["DR"]).max()


def test_damping_lowers_the_resonance_peak(damped):
    """Added viscous damping reduces the largest receiver response over the band (passivity sign)."""
    w, s, sd, _ = damped
    om = 2 * np.pi * np.linspace(10, 400, 80)
    y0 = np.array([np.abs(solve.full_solve(s["K"], s["M"], s["F"], s["flags"], o)[s["recv"]]).max() for o in om])
    y1 = np.array([np.abs(soar.full_solve(sd, o)[s["recv"]]).max() for o in om])
    assert y1.max() < y0.max()
