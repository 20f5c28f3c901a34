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


# ------------------------------------------------------------------ skin-pressure load
# f_u = -int N_s^T p n_out dGamma with n_out pointing away from the structure. Because the
# element is isoparametric, sum_a N_a X_a = X on every face, so weighted sums of the nodal
# forces are exact surface integrals that can be written out without the oracle:
#   sum_a f_a            = -int p n_out dGamma
#   sum_a (f_a . X_a)    = -int p (n_out . X) dGamma


def _plate_patch(lx=0.3, ly=0.2, t=0.002, nx=3, ny=2):
    coords = grid_nodes(np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1), np.array([0.0, t]))
    nid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    elems = grid_elems(nx, ny, 1, nid)
    top = np.array([[nid(i, j, 1), nid(i + 1, j, 1), nid(i + 1, j + 1, 1), nid(i, j + 1, 1)]
                    for j in range(ny) for i in range(nx)], np.int64)   # right-hand normal +z
    mat = Material(kind=SOLID, rho=2700.0, eta=0.02, E=70e9, nu=0.3)
    mesh = Mesh(coords=coords, elems=elems, elem_mat=np.zeros(len(elems), np.int32), materials=[mat],
                clamped=np.zeros(0, np.int64), iface=np.zeros((0, 4), np.int64))
    return mesh, top


def _nodal_forces(s, mesh, l=0):
    dm = s["dof"]
    f = np.zeros((mesh.n_nodes, 3), complex)
    ok = dm.u[:, 0] >= 0
    f[ok] = s["F"][dm.u[ok], l]
    return f


def test_skin_pressure_flat_patch_total_force_and_moment():
    """Uniform p on a flat top face (normal +z, away from the plate): total force -p A e_z.
    Linear p = a + b x + c y: sum f_z = -int p dA and sum x_a f_z,a = -int x p dA in closed form."""
    from workloads.meshes import LOAD_SKIN_PRESSURE
    lx, ly = 0.3, 0.2
    mesh, top = _plate_patch(lx, ly)
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    a, b, c = 2.0 - 1.0j, 3.0 + 0.5j, -1.5 + 2.0j
    loads = [Load(kind=LOAD_SKIN_PRESSURE, faces=top, amp=np.full(mesh.n_nodes, 1.0 + 0j)),
             Load(kind=LOAD_SKIN_PRESSURE, faces=top, amp=a + b * x + c * y)]
    s = assembly.assemble(mesh, loads, np.zeros(0, np.int64))
    assert np.array_equal(s["flags"], [0, 0])
    A = lx * ly
    f0 = _nodal_forces(s, mesh, 0)
    assert np.allclose(f0.sum(axis=0), [0.0, 0.0, -A], rtol=0, atol=1e-15)
    # only the loaded face's nodes carry force
    loaded = np.unique(top)
    assert np.all(f0[np.setdiff1d(np.arange(mesh.n_nodes), loaded)] == 0)
    f1 = _nodal_forces(s, mesh, 1)
    int_p = a * A + b * lx ** 2 / 2 * ly + c * ly ** 2 / 2 * lx
    int_xp = a * lx ** 2 / 2 * ly + b * lx ** 3 / 3 * ly + c * (lx ** 2 / 2) * (ly ** 2 / 2)
    assert np.isclose(f1[:, 2].sum(), -int_p, rtol=1e-13)
    assert np.isclose((x * f1[:, 2]).sum(), -int_xp, rtol=1e-13)
    assert np.allclose(f1[:, :2], 0, atol=1e-15)


def test_skin_pressure_closed_cylinder_net_force_and_virial():
    """Uniform unit pressure on the fuselage skin (faces as the workload generator orients them):
    the net force vanishes, and sum_a f_a . X_a = -sum_faces A_f (n_f . X_f), with n_f the plane
    normal of each (planar) face taken pointing AWAY FROM THE AXIS (computed here from the face
    corners, not from the generator's orientation). A face list oriented into the structure, or a
    factor of two in the face integrals, fails this."""
    from workloads.fuselage import fuselage
    from workloads.meshes import LOAD_SKIN_PRESSURE
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    alu = Material(kind=SOLID, rho=2700.0, eta=0.02, E=70e9, nu=0.3)
    mesh = fuselage(length=1.0, frame_z=(0.5,), n_core=4, n_ring=2, h_z=0.25, air=air, metal=alu)
    mesh.clamped = np.zeros(0, np.int64)          # every skin node free, so no force is dropped
    faces = mesh.meta["skin_faces"]
    s = assembly.assemble(mesh, [Load(kind=LOAD_SKIN_PRESSURE, faces=faces, amp=np.ones(mesh.n_nodes, complex))],
                          np.zeros(0, np.int64))
    f = _nodal_forces(s, mesh)
    X = mesh.coords
    expect, area = 0.0, 0.0
    for q in faces:
        c = X[q]
        d1, d2 = c[2] - c[0], c[3] - c[1]
        nv = np.cross(d1, d2)
        Af = 0.5 * np.linalg.norm(nv)                 # planar quad: half the diagonals' cross product
        n = nv / np.linalg.norm(nv)
        mid = c.mean(axis=0)
        if np.dot(n[:2], mid[:2]) < 0:
            n = -n
        assert abs(np.dot(c - c[0], n)).max() < 1e-12   # the face is planar
        expect += -Af * np.dot(n, mid)
        area += Af
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * area
    assert np.isclose(np.einsum("ad,ad->", f, X), expect, rtol=1e-12)
    assert expect < 0


def test_skin_pressure_power_is_positive():
    """A skin pressure on a damped coupled model injects positive time-averaged power:
    Re(f^H v) > 0 with v = i w u (e^{+i w t}); checked on a small fuselage segment."""
    from workloads.fuselage import fuselage
    from workloads.meshes import LOAD_SKIN_PRESSURE
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    alu = Material(kind=SOLID, rho=2700.0, eta=0.02, E=70e9, nu=0.3)
    mesh = fuselage(length=1.0, frame_z=(0.5,), n_core=3, n_ring=1, h_z=0.25, air=air, metal=alu)
    faces = mesh.meta["skin_faces"]
    rng = W.SplitMix64(4242)
    amp = np.exp(2j * np.pi * rng.uniforms(mesh.n_nodes))
    s = assembly.assemble(mesh, [Load(kind=LOAD_SKIN_PRESSURE, faces=faces, amp=amp)], np.zeros(0, np.int64))
    n_u = s["n_u"]
    for f_hz in (23.0, 97.0, 211.0, 289.0):
        om = 2 * np.pi * f_hz
        x = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)[:, 0]
        power = np.vdot(s["F"][:n_u, 0], 1j * om * x[:n_u]).real
        assert power > 0
