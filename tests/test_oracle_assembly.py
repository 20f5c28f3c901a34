"""Pins of the oracle's assembly against closed forms and physical identities (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from workloads.meshes import (FLUID, SOLID, LOAD_POINT_FORCE, LOAD_VOLUME_VELOCITY, Load,
                              Material, Mesh, air_box, grid_elems, grid_nodes)
from oracle import assembly, solve


def _box(cells, dims, c=343.0, eta=0.0, rho=1.21):
    return air_box(*dims, *cells, Material(kind=FLUID, rho=rho, eta=eta, c=c))


def _lam1d(m, h):
    """1D linear-element Neumann eigenvalues of (K1, M1): (6/h^2)(1-cos t)/(2+cos t), t = l pi / m."""
    t = np.arange(m + 1) * np.pi / m
    return (6.0 / h ** 2) * (1 - np.cos(t)) / (2 + np.cos(t))


def test_acoustic_discrete_closed_form():
    """Eigenvalues of (K_f, M_f) on a tensor box equal c^2 * sum_d lam_d exactly."""
    cells, dims, c = (4, 3, 2), (1.0, 0.7, 0.5), 343.0
    mesh = _box(cells, dims, c=c)
    s = assembly.assemble(mesh, [], np.array([0]))
    K = s["K"].toarray().real
    M = s["M"].toarray().real
    ev = np.sort(sla.eigh(K, M, eigvals_only=True))
    lx, ly, lz = (_lam1d(m, L / m) for m, L in zip(cells, dims))
    ref = np.sort((lx[:, None, None] + ly[None, :, None] + lz[None, None, :]).ravel()) * c ** 2
    assert np.allclose(ev, ref, rtol=1e-12, atol=1e-6)


def test_acoustic_continuum_mode_convergence():
    """Lowest non-zero mode -> c/(2 Lx); the error drops ~4x when h halves (O(h^2))."""
    c, dims = 343.0, (1.0, 0.7, 0.5)
    exact = c / (2 * dims[0])
    errs = []
    for cells in [(5, 4, 3), (10, 7, 5)]:
        s = assembly.assemble(_box(cells, dims, c=c), [], np.array([0]))
        ev = np.sort(sla.eigh(s["K"].toarray().real, s["M"].toarray().real, eigvals_only=True))
        f1 = np.sqrt(ev[1]) / (2 * np.pi)
        errs.append(abs(f1 - exact) / exact)
    assert errs[1] < 0.006
    assert 3.0 < errs[0] / errs[1] < 5.0


def _solid_block(E=70e9, nu=0.3, rho=2700.0, distort=True):
    coords = grid_nodes(np.linspace(0, 0.3, 3), np.linspace(0, 0.2, 3), np.linspace(0, 0.1, 2))
    if distort:   # move interior-ish nodes so elements are non-rectangular
        rng = W.SplitMix64(12345)
        coords = coords + 0.01 * (rng.uniforms(coords.size).reshape(coords.shape) - 0.5)
    nid = lambda i, j, k: i + 3 * (j + 3 * k)
    elems = grid_elems(2, 2, 1, nid)
    mat = Material(kind=SOLID, rho=rho, eta=0.0, E=E, nu=nu)
    return Mesh(coords=coords, elems=elems, elem_mat=np.zeros(len(elems), np.int32),
                materials=[mat], clamped=np.zeros(0, np.int64), iface=np.zeros((0, 4), np.int64))


def _volume(mesh):
    # volume of each hex from its outward-oriented boundary: sum of origin tetrahedra (24 triangles)
    faces = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
    vol = 0.0
    for el in mesh.elems:
        X = mesh.coords[el]
        for f in faces:
            a, b, c, d = (X[i] for i in f)
            ctr = (a + b + c + d) / 4
            for p, q in [(a, b), (b, c), (c, d), (d, a)]:
                vol += np.dot(ctr, np.cross(p, q)) / 6.0
    return vol


def test_solid_rigid_modes_mass_and_energy():
    E, nu, rho = 70e9, 0.3, 2700.0
    mesh = _solid_block(E, nu, rho)
    dm = assembly.DofMap(mesh)
    Ke, Me = assembly.solid_element_matrices(mesh.coords[mesh.elems], E, nu, rho)
    n = dm.n_u
    K = np.zeros((n, n)); Mm = np.zeros((n, n))
    for e, el in enumerate(mesh.elems):
        d = dm.u[el].ravel()
        K[np.ix_(d, d)] += Ke[e].real
        Mm[np.ix_(d, d)] += Me[e].real
    X = mesh.coords
    u = lambda f: np.array([f(x) for x in X]).ravel()
    rigid = [u(lambda x: [1, 0, 0]), u(lambda x: [0, 1, 0]), u(lambda x: [0, 0, 1]),
             u(lambda x: [-x[1], x[0], 0]), u(lambda x: [0, -x[2], x[1]]), u(lambda x: [x[2], 0, -x[0]])]
    scale = np.abs(K).max()
    for r in rigid:
        assert np.abs(K @ r).max() < 1e-9 * scale * np.abs(r).max()
    ev = np.sort(np.abs(np.linalg.eigvalsh(K)))
    assert ev[5] < 1e-8 * ev[-1] and ev[6] > 1e-6 * ev[-1]
    vol = _volume(mesh)
    for d in range(3):
        one = np.zeros((len(X), 3)); one[:, d] = 1
        assert np.isclose(one.ravel() @ Mm @ one.ravel(), rho * vol, rtol=1e-12)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu)); mu = E / (2 * (1 + nu))
    eps, gam = 1e-4, 2e-4
    ux = u(lambda x: [eps * x[0], 0, 0])
    assert np.isclose(ux @ K @ ux, vol * (lam + 2 * mu) * eps ** 2, rtol=1e-10)
    us = u(lambda x: [gam * x[1], 0, 0])
    assert np.isclose(us @ K @ us, vol * mu * gam ** 2, rtol=1e-10)
    uv = u(lambda x: [eps * x[0], eps * x[1], eps * x[2]])
    assert np.isclose(uv @ K @ uv, vol * 3 * (3 * lam + 2 * mu) * eps ** 2, rtol=1e-10)


def test_coupling_area_and_direction():
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    n_u = s["n_u"]
    Kc = -s["K"][:n_u, n_u:].toarray()             # = C restricted to free u DoFs
    Mc = s["M"][n_u:, :n_u].toarray()              # = rho0 C^T
    assert np.allclose(Mc, 1.21 * Kc.T, rtol=0, atol=1e-15)
    # every interface face has normal +z: x and y rows vanish, z rows integrate to the area
    dm = s["dof"]
    lx, ly = w.mesh.meta["dims"][:2]
    mesh_nodes = np.unique(w.mesh.iface.ravel())
    zrows = dm.u[mesh_nodes, 2]; zrows = zrows[zrows >= 0]
    xrows = dm.u[mesh_nodes, 0]; xrows = xrows[xrows >= 0]
    assert np.abs(Kc[xrows]).max() == 0.0
    # clamped edge nodes drop part of the area: compare with an unclamped assembly of C
    Wf = assembly.face_integrals(w.mesh.coords[w.mesh.iface])
    assert np.isclose(Wf[..., 2].sum(), lx * ly, rtol=1e-13)
    assert abs(Wf[..., 0].sum()) < 1e-15 and abs(Wf[..., 1].sum()) < 1e-15
    assert Kc[zrows].sum().real <= lx * ly


def test_volume_balance_and_reciprocity():
    """Fluid-row and structure-row coupling signs and the rho0 / i w scale.

    Volume balance: summing the fluid rows, K_f 1 = 0 leaves
        -w^2 [ 1^T M_f p + rho0 1^T C^T u ] = 1^T f_p   (holds for every solution).
    Reciprocity of the u-p system: p_b(F_a = 1) = -i w u_a(Q_b = 1).
    """
    w = W.small_plate_cavity()
    mesh = w.mesh
    fa = w.loads[0].node
    fn = W.fluid_nodes(mesh)
    qb = int(fn[len(fn) // 3])
    loads = [Load(kind=LOAD_POINT_FORCE, node=fa, dir=2, value=1.0),
             Load(kind=LOAD_VOLUME_VELOCITY, node=qb, value=1.0)]
    s = assembly.assemble(mesh, loads, np.array([qb]))
    dm = s["dof"]
    n_u = s["n_u"]
    for f_hz in (37.0, 151.0, 333.0):
        om = 2 * np.pi * f_hz
        x = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
        p_b = x[dm.p[qb], 0]
        u_a = x[dm.u[fa, 2], 1]
        assert np.isclose(p_b, -1j * om * u_a, rtol=1e-9)
        for l in range(2):
            xu, xp = x[:n_u, l], x[n_u:, l]
            t1 = s["M"][n_u:, n_u:] @ xp
            t2 = s["M"][n_u:, :n_u] @ xu
            lhs = -om ** 2 * (t1 + t2).sum()
            rhs = solve.load_at(s["F"], s["flags"], om)[n_u:, l].sum()
            scale = om ** 2 * (np.abs(t1).sum() + np.abs(t2).sum())
            assert abs(lhs - rhs) <= 1e-9 * scale


def test_passivity():
    """With e^{+i w t} and positive loss factors the sources inject positive power."""
    w = W.small_plate_cavity()
    fn = W.fluid_nodes(w.mesh)
    qb = int(fn[5])
    loads = [w.loads[0], Load(kind=LOAD_VOLUME_VELOCITY, node=qb, value=1.0)]
    s = assembly.assemble(w.mesh, loads, np.array([qb]))
    dm = s["dof"]
    fa = w.loads[0].node
    for f_hz in np.linspace(15, 395, 13):
        om = 2 * np.pi * f_hz
        x = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
        assert (np.conj(1.0) * 1j * om * x[dm.u[fa, 2], 0]).real > 0    # Re(F^* v) > 0
        assert (x[dm.p[qb], 1] * np.conj(1.0)).real > 0                 # Re(p Q^*) > 0


def test_dof_counts_plate_cavity():
    w = W.plate_cavity_workload()
    dm = assembly.DofMap(w.mesh)
    assert dm.n_u == 2070 and dm.n_p == 5525 and dm.n == 7595
