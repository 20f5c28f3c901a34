"""The seeded input generators: SplitMix64 against its published reference outputs, and the
geometric invariants of the fuselage meshes (interface and skin orientation, clamping, DoF
counts of the full-size segment)."""
import numpy as np

import workloads as W
from workloads.fuselage import HEX_FACES, fuselage
from workloads.meshes import FLUID, SOLID, Material


def test_splitmix64_reference_outputs():
    # published SplitMix64 outputs for seed 0 (Vigna's reference implementation)
    r = W.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = W.SplitMix64(1).uniforms(1000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.05


def _face_normal(c):
    return np.cross(c[1] - c[0], c[3] - c[0])


def test_fuselage_interface_and_skin_orientation():
    air = Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    alu = Material(kind=SOLID, rho=2700.0, eta=0.02, E=70e9, nu=0.3)
    mesh = fuselage(length=2.0, frame_z=(0.6, 1.4), n_core=4, n_ring=2, h_z=0.25, air=air, metal=alu)
    kinds = np.array([m.kind for m in mesh.materials])[mesh.elem_mat]
    # every interface face lies on a fluid element and on a solid element, and its right-hand
    # normal points out of the fluid element
    fluid_faces = {}
    for e in np.nonzero(kinds == FLUID)[0]:
        for f in HEX_FACES:
            fluid_faces[frozenset(mesh.elems[e][f])] = e
    solid_faces = {frozenset(mesh.elems[e][f]) for e in np.nonzero(kinds == SOLID)[0] for f in HEX_FACES}
    assert len(mesh.iface) > 0
    for quad in mesh.iface:
        key = frozenset(quad)
        assert key in fluid_faces and key in solid_faces
        c = mesh.coords[quad]
        centre = mesh.coords[mesh.elems[fluid_faces[key]]].mean(axis=0)
        assert np.dot(_face_normal(c), c.mean(axis=0) - centre) > 0
    # outer skin faces point away from the axis; the skin ends are clamped
    sf = mesh.meta["skin_faces"]
    for quad in sf:
        c = mesh.coords[quad]
        mid = c.mean(axis=0)
        assert np.dot(_face_normal(c)[:2], mid[:2]) > 0
        assert np.allclose(np.hypot(c[:, 0], c[:, 1]), 1.4, atol=1e-9)   # corners on the outer circle
    z = mesh.coords[mesh.clamped, 2]
    assert np.all((np.abs(z) < 1e-12) | (np.abs(z - 2.0) < 1e-12))


def test_full_size_fuselage_dof_counts():
    from oracle.assembly import DofMap
    w = W.fuselage_workload(n_loads=1)
    d = DofMap(w.mesh)
    assert (d.n, d.n_u, d.n_p) == (529306, 94176, 435130)
