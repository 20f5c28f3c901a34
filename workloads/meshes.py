"""Structured hex8 meshes and load descriptions for the synthetic vibro-acoustic workloads.

Only geometry and bookkeeping live here (node coordinates, element connectivity, material
tags, clamped nodes, fluid-solid interface faces, load descriptors). No finite-element or
solver arithmetic: the oracle and the GPU library each assemble the matrices on their own.

Conventions shared by both consumers:
  * hex8 node order in natural coordinates (xi, eta, zeta):
      (-,-,-) (+,-,-) (+,+,-) (-,+,-) (-,-,+) (+,-,+) (+,+,+) (-,+,+)
  * interface faces list 4 node ids around the perimeter such that the right-hand normal
    (x1 - x0) x (x3 - x0) points OUT of the fluid (into the structure);
  * skin-pressure faces list 4 node ids such that the right-hand normal points OUT of the
    structure (away from the cabin, into the exterior where the pressure acts);
  * nodes are shared between a solid and a fluid element on the interface: such a node
    carries 3 displacement DoFs and 1 pressure DoF.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FLUID = 0
SOLID = 1

LOAD_VOLUME_VELOCITY = 0
LOAD_POINT_FORCE = 1
LOAD_SKIN_PRESSURE = 2


@dataclass
class Material:
    kind: int            # FLUID or SOLID
    rho: float
    eta: float           # loss factor
    c: float = 0.0       # fluid speed of sound
    E: float = 0.0       # solid Young's modulus
    nu: float = 0.0      # solid Poisson ratio
    # frequency-dependent loss factor: (f_hz, eta) sample points, piecewise linear and constant
    # beyond the ends; None = the constant eta above
    eta_table: tuple | None = None


@dataclass
class Load:
    kind: int
    node: int = -1
    dir: int = 2
    value: complex = 1.0 + 0.0j
    faces: np.ndarray | None = None     # (nf, 4) int64, SKIN_PRESSURE only
    amp: np.ndarray | None = None       # (n_nodes,) complex128 nodal pressure, SKIN_PRESSURE only


@dataclass
class Mesh:
    coords: np.ndarray                  # (n_nodes, 3) float64
    elems: np.ndarray                   # (n_el, 8) int64
    elem_mat: np.ndarray                # (n_el,) int32, index into materials
    materials: list
    clamped: np.ndarray                 # node ids whose displacement DoFs are fixed
    iface: np.ndarray                   # (n_if, 4) int64 fluid-solid faces
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])


def grid_nodes(xs, ys, zs) -> np.ndarray:
    """Tensor-product node coordinates, x fastest, then y, then z."""
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    return np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                     Z.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)


def grid_elems(nx, ny, nz, node_id) -> np.ndarray:
    """hex8 connectivity of an nx*ny*nz block; node_id(i, j, k) maps grid indices to node ids."""
    out = np.empty((nx * ny * nz, 8), dtype=np.int64)
    e = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                out[e] = [node_id(i, j, k), node_id(i + 1, j, k), node_id(i + 1, j + 1, k),
                          node_id(i, j + 1, k), node_id(i, j, k + 1), node_id(i + 1, j, k + 1),
                          node_id(i + 1, j + 1, k + 1), node_id(i, j + 1, k + 1)]
                e += 1
    return out


def air_box(lx, ly, lz, nx, ny, nz, air: Material) -> Mesh:
    """Rigid-walled fluid box [0,lx]x[0,ly]x[0,lz] meshed by nx*ny*nz hex8."""
    coords = grid_nodes(np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1),
                        np.linspace(0, lz, nz + 1))
    nid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    elems = grid_elems(nx, ny, nz, nid)
    return Mesh(coords=coords, elems=elems, elem_mat=np.zeros(len(elems), np.int32),
                materials=[air], clamped=np.zeros(0, np.int64), iface=np.zeros((0, 4), np.int64),
                meta=dict(kind="box", dims=(lx, ly, lz), cells=(nx, ny, nz)))


def plate_cavity(lx, ly, lz, nx, ny, nz, t, air: Material, plate: Material) -> Mesh:
    """Fluid box with a one-element-thick solid plate of thickness t on its top face z = lz.

    The plate's bottom node layer is the fluid's top node layer (shared nodes). The plate is
    clamped along its four edges (every plate node with x in {0, lx} or y in {0, ly}).
    """
    box = air_box(lx, ly, lz, nx, ny, nz, air)
    nf = box.n_nodes
    xs, ys = np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1)
    top = grid_nodes(xs, ys, np.array([lz + t]))
    coords = np.vstack([box.coords, top])
    fid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)

    def pid(i, j, k):
        return fid(i, j, nz) if k == 0 else nf + i + (nx + 1) * j

    pel = grid_elems(nx, ny, 1, pid)
    elems = np.vstack([box.elems, pel])
    elem_mat = np.concatenate([box.elem_mat, np.ones(len(pel), np.int32)])
    plate_nodes = np.unique(pel.ravel())
    px, py = coords[plate_nodes, 0], coords[plate_nodes, 1]
    edge = (np.isclose(px, 0) | np.isclose(px, lx) | np.isclose(py, 0) | np.isclose(py, ly))
    clamped = np.sort(plate_nodes[edge])
    iface = np.array([[fid(i, j, nz), fid(i + 1, j, nz), fid(i + 1, j + 1, nz), fid(i, j + 1, nz)]
                      for j in range(ny) for i in range(nx)], dtype=np.int64)
    top_ids = nf + np.arange((nx + 1) * (ny + 1), dtype=np.int64)
    return Mesh(coords=coords, elems=elems, elem_mat=elem_mat, materials=[air, plate],
                clamped=clamped, iface=iface,
                meta=dict(kind="plate_cavity", dims=(lx, ly, lz), cells=(nx, ny, nz), t=t,
                          top_nodes=top_ids))


def fluid_nodes(mesh: Mesh) -> np.ndarray:
    fl = [i for i, m in enumerate(mesh.materials) if m.kind == FLUID]
    return np.unique(mesh.elems[np.isin(mesh.elem_mat, fl)].ravel())


def solid_nodes(mesh: Mesh) -> np.ndarray:
    so = [i for i, m in enumerate(mesh.materials) if m.kind == SOLID]
    if not so:
        return np.zeros(0, np.int64)
    return np.unique(mesh.elems[np.isin(mesh.elem_mat, so)].ravel())
