"""Pins of the oracle's full solve, rational Krylov basis, reduced model, sweep and greedy."""
import numpy as np
import pytest

import workloads as W
from workloads.meshes import FLUID, LOAD_VOLUME_VELOCITY, Load, Material, air_box
from oracle import assembly, greedy, krylov, rom, solve


def _m1d(m, h):
    """1D consistent linear-element mass matrix (textbook h/6 [2 1; 1 2] per element)."""
    M = np.zeros((m + 1, m + 1))
    for e in range(m):
        M[e:e + 2, e:e + 2] += h / 6 * np.array([[2, 1], [1, 2]])
    return M


def test_box_full_solve_equals_closed_form_modal_sum():
    """Discrete modal expansion with tensor-cosine eigenvectors, built without the oracle.

    A = K_f - w^2 M0 / c~^2, K_f phi = mu M0 phi with phi = cos_x (x) cos_y (x) cos_z and
    mu = sum_d (6/h_d^2)(1 - cos t_d)/(2 + cos t_d). Then x = sum phi phi^T f / ((mu - w^2/c~^2) n_phi),
    f = i w rho0 Q e_s.
    """
    cells, dims = (5, 4, 3), (1.0, 0.7, 0.5)
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    mesh = air_box(*dims, *cells, air)
    src, rec = 17, np.array([3, 40, 77, 101])
    s = assembly.assemble(mesh, [Load(kind=LOAD_VOLUME_VELOCITY, node=src, value=1.0)], rec)
    c2 = 343.0 ** 2 * (1 + 0.01j)
    phis, mus, norms = [], [], []
    for m, Ld in zip(cells, dims):
        h = Ld / m
        t = np.arange(m + 1) * np.pi / m
        j = np.arange(m + 1)
        P = np.cos(np.outer(j, t))                         # columns = eigenvectors
        phis.append(P)
        mus.append((6 / h ** 2) * (1 - np.cos(t)) / (2 + np.cos(t)))
        norms.append(np.einsum("ja,jk,ka->a", P, _m1d(m, h), P))
    # node id = i + (mx+1)(j + (my+1) k): x fastest -> kron order z, y, x
    Phi = np.kron(np.kron(phis[2], phis[1]), phis[0])
    mu = (mus[2][:, None, None] + mus[1][None, :, None] + mus[0][None, None, :]).ravel()
    nrm = (norms[2][:, None, None] * norms[1][None, :, None] * norms[0][None, None, :]).ravel()
    for f_hz in (33.0, 171.0, 290.0, 444.0):
        om = 2 * np.pi * f_hz
        x = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)[:, 0]
        f = np.zeros(mesh.n_nodes, complex)
        f[src] = 1j * om * 1.21
        xm = Phi @ ((Phi.T @ f) / ((mu - om ** 2 / c2) * nrm))
        assert np.allclose(x, xm, rtol=1e-10, atol=1e-12 * np.abs(xm).max())


def test_sparse_lu_equals_dense_solve():
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    om = 2 * np.pi * 211.0
    a = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
    b = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om, dense=True)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-13 * np.abs(b).max())


@pytest.fixture(scope="module")
def small_rom():
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    shifts = 2 * np.pi * np.array([30.0, 90.0, 150.0, 210.0, 270.0, 330.0, 390.0])
    rb = krylov.build_basis(ss, shifts, 5)
    return w, s, ss, shifts, rb, krylov.project(ss, rb.basis)


def test_orthonormal_basis(small_rom):
    _, _, _, _, rb, _ = small_rom
    V = rb.basis
    assert np.abs(V.conj().T @ V - np.eye(rb.q)).max() < 1e-13


def test_moment_matching(small_rom):
    """Zeroth moment (interpolation) at every expansion point of the converged 7-point model."""
    _, s, _, shifts, rb, r = small_rom
    K, M, F = s["K"].toarray(), s["M"].toarray(), s["F"]
    recv = s["recv"]
    for om in shifts:
        yf = np.linalg.solve(K - om ** 2 * M, F)[recv]
        yr = r["CR"] @ np.linalg.solve(r["KR"] - om ** 2 * r["MR"], r["FR"])
        assert np.abs(yf - yr).max() <= 1e-10 * np.abs(yf).max()


@pytest.mark.parametrize("shifts_hz,blocks", [((30.0, 200.0, 370.0), 4), ((60.0, 180.0, 300.0), 3)])
def test_higher_moments_match_in_backward_error(shifts_hz, blocks):
    """Moment matching of Eq. (10)-(11) for every moment i < k_j, in the scaled system.

    The ROM's moments x_R,0 = A_Rj^{-1} F_R, x_R,i+1 = A_Rj^{-1} M_R x_R,i, lifted by V, satisfy the
    full-order recurrence A_j x_0 = F, A_j x_i+1 = M x_i exactly (the Krylov blocks lie in span V
    and the model is a Galerkin projection), so their normwise backward errors against the full
    matrices are at rounding level. The check is in backward-error form because the forward
    error of high moments carries kappa(A_j) ~ 1e6. Off the expansion points the same quantity
    is the model's own residual (>= 1e-9 here), which shows that the check discriminates.
    (When a block nearly deflates, i.e. a norm ratio close to 1e-10, the continuation vector
    of the next block is accurate to eps / ratio only and later moments match to that level;
    these two models are far from converged so no block comes close to deflating.)"""
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    K, M, F = ss["K"], ss["M"], ss["F"]
    shifts = 2 * np.pi * np.array(shifts_hz)
    rb = krylov.build_basis(ss, shifts, blocks)
    assert rb.deflated == 0 and rb.q == len(shifts) * blocks
    V, r = rb.basis, krylov.project(ss, rb.basis)

    def berr(A, x, b):
        nA = abs(A).sum(axis=1).max()
        return np.abs(A @ x - b).max() / (nA * np.abs(x).max() + np.abs(b).max())

    for om in shifts:
        A, AR = K - om ** 2 * M, r["KR"] - om ** 2 * r["MR"]
        xr, b = np.linalg.solve(AR, r["FR"]), F
        for i in range(blocks):
            x = V @ xr
            assert berr(A, x, b) <= 1e-13, (om, i)
            # the same moment at the receivers, forward error bounded by kappa(A_j) eps
            yf = np.linalg.solve(A.toarray(), b)[ss["recv"]] * ss["scale"][ss["recv"]][:, None]
            assert np.abs(r["CR"] @ xr - yf).max() <= 1e-9 * np.abs(yf).max(), (om, i)
            b, xr = M @ x, np.linalg.solve(AR, r["MR"] @ xr)
    om = 2 * np.pi * 123.0
    A = K - om ** 2 * M
    x = V @ np.linalg.solve(r["KR"] - om ** 2 * r["MR"], r["FR"])
    assert berr(A, x, F) >= 1e-9


def test_interpolation_and_galerkin(small_rom):
    w, s, ss, shifts, rb, r = small_rom
    for om in shifts:
        y = solve.full_frf(s, [om])
        yr = rom.sweep(r, [om])
        assert rom.relative_error(yr, y).max() < 1e-10
    om = 2 * np.pi * 123.4
    V = rb.basis
    f = solve.load_at(ss["F"], ss["flags"], om)
    xr = np.linalg.solve(r["KR"] - om ** 2 * r["MR"], r["FR"] * np.where(s["flags"] == 1, 1j * om, 1))
    res = f - (ss["K"] - om ** 2 * ss["M"]) @ (V @ xr)
    assert np.abs(V.conj().T @ res).max() < 1e-9 * np.abs(f).max()


def test_full_dimension_rom_is_exact():
    """q = n: the Galerkin model reproduces every full solve."""
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    mesh = air_box(0.5, 0.4, 0.3, 2, 2, 1, air)
    src = 4
    s = assembly.assemble(mesh, [Load(kind=LOAD_VOLUME_VELOCITY, node=src, value=1.0)],
                          np.arange(mesh.n_nodes))
    n = s["K"].shape[0]
    rb = krylov.RationalBasis(n, n)
    rb.add_block(np.eye(n, dtype=complex))
    assert rb.q == n
    r = krylov.project(s, rb.basis)
    om = 2 * np.pi * np.array([50.0, 400.0, 900.0])
    assert rom.relative_error(rom.sweep(r, om), solve.full_frf(s, om)).max() < 1e-12


def test_basis_invariance_householder(small_rom):
    """The same recurrence orthonormalised by Householder QR (LAPACK) instead of MGS spans the
    same space: y_R agrees wherever the model has converged."""
    _, _, ss, shifts, rb, r = small_rom
    K, M, F = ss["K"].toarray(), ss["M"].toarray(), ss["F"]
    Q = np.zeros((K.shape[0], 0), complex)
    for om in shifts:
        A = K - om ** 2 * M
        x = np.linalg.solve(A, F)
        for i in range(5):
            Q, _ = np.linalg.qr(np.hstack([Q, x]))
            x = np.linalg.solve(A, M @ Q[:, -1:])
    r2 = krylov.project(ss, Q)
    om = 2 * np.pi * np.linspace(12, 398, 25)
    y1, y2 = rom.sweep(r, om), rom.sweep(r2, om)
    # where the model has converged to the full solution both bases must give the same
    # outputs; elsewhere y_R carries the model's own approximation error and is sensitive
    # to rounding in the basis
    conv = rom.relative_error(y1, solve.full_frf(small_rom[1], om)) < 1e-8
    assert conv.sum() >= 15
    assert rom.relative_error(y1, y2)[conv].max() < 1e-8


def test_deflation_of_duplicate_direction():
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    mesh = air_box(0.5, 0.4, 0.3, 3, 2, 2, air)
    s = assembly.assemble(mesh, [Load(kind=LOAD_VOLUME_VELOCITY, node=3, value=1.0),
                                 Load(kind=LOAD_VOLUME_VELOCITY, node=3, value=2.0)], np.array([0]))
    rb = krylov.build_basis(s, [2 * np.pi * 100.0], 2)
    assert rb.deflated == 1 and rb.q == 2     # the parallel column is dropped once


def test_greedy_properties():
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    rp = w.rom
    g = greedy.greedy(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], rp["max_shifts"])
    cand = g["cand_hz"]
    assert g["shift_idx"][0] == greedy.first_candidate(cand) == 31    # nearest the centre, lower index
    assert g["maxres"][-1] <= rp["tol"]
    # the residual estimate vanishes at every expansion point (interpolation)
    assert np.all(g["res"][g["shift_idx"]] < 1e-9)
    # the converged model agrees with full solves on the candidate grid
    om = 2 * np.pi * cand[::7]
    err = rom.relative_error(rom.sweep(g["rom"], om), solve.full_frf(s, om))
    assert err.max() < 1e-4


def test_greedy_stops_when_the_space_saturates():
    """With an unreachable tolerance, stall_stop = 2 ends the greedy after two expansion points in
    a row that add no column (their Krylov columns all deflate), with the residual unchanged
    since the last point that added columns; without it the loop runs to the cap."""
    w = W.box()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    g = greedy.greedy(s, (20.0, 500.0), 64, 10, 1e-15, 30, stall_stop=2)
    k = len(g["shift_idx"])
    assert 3 <= k < 30
    assert g["maxres"][-1] == g["maxres"][-2] == g["maxres"][-3]
    g0 = greedy.greedy(s, (20.0, 500.0), 64, 10, 1e-15, 8)
    assert len(g0["shift_idx"]) == 8 and g0["basis"].q == g["basis"].q
    assert list(g0["shift_idx"][:k]) == list(g["shift_idx"])
