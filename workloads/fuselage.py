"""Fuselage-like segment: air-filled cylinder with a thin metal skin and ring frames.

Cross-section: an O-grid (square core of n_core x n_core cells, n_ring blended rings from the
square to the circle r1 = R - t_skin - d_frame, one ring r1..r2 = R - t_skin that is air except
inside a frame, one skin ring r2..R). The section is extruded along z with layers of about h_z
plus the two planes of every frame (frames are 2 mm thick axially). Skin and frames are solid
hex8, everything else fluid hex8. Skin ends (z = 0 and z = L) are clamped; the end caps are
rigid walls for the air (natural boundary). Interface faces (solid element face shared with a
fluid element) and the outer skin faces are found by matching element faces.

Only geometry and bookkeeping; no finite-element arithmetic.
"""
from __future__ import annotations

import numpy as np

from .meshes import FLUID, SOLID, Material, Mesh

# hex8 faces with outward right-hand orientation: (x1 - x0) x (x3 - x0) points out of the element
HEX_FACES = np.array([[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]])


def _z_planes(length, h_z, frame_z, frame_t):
    base = np.linspace(0.0, length, max(2, int(np.ceil(length / h_z))) + 1)
    fb = np.sort(np.concatenate([[z - frame_t / 2, z + frame_t / 2] for z in frame_z])) if len(frame_z) else np.zeros(0)
    keep = [z for z in base if np.all(np.abs(fb - z) > 0.25 * h_z) or z in (0.0, length)]
    zs = np.unique(np.concatenate([keep, fb]))
    return zs


def fuselage(R=1.4, length=4.0, skin_t=0.002, frame_z=(0.4, 1.2, 2.0, 2.8, 3.6), frame_depth=0.06,
             frame_t=0.002, n_core=8, n_ring=4, h_z=0.2, air: Material = None, metal: Material = None,
             core_frac=0.5) -> Mesh:
    r1 = R - skin_t - frame_depth
    r2 = R - skin_t
    a = core_frac * r1 / np.sqrt(2.0)   # half-width of the square core
    n = n_core
    Nc = 4 * n
    # core grid
    xs = np.linspace(-a, a, n + 1)
    core = np.array([[xs[i], xs[j]] for j in range(n + 1) for i in range(n + 1)])
    ncore = (n + 1) ** 2

    def core_id(i, j):
        return i + (n + 1) * j

    # square boundary, counter-clockwise from the corner (a, -a)
    sq_id = np.empty(Nc, np.int64)
    sq_xy = np.empty((Nc, 2))
    for s in range(Nc):
        side, k = divmod(s, n)
        if side == 0:
            i, j = n, k
        elif side == 1:
            i, j = n - k, n
        elif side == 2:
            i, j = 0, n - k
        else:
            i, j = k, 0
        sq_id[s] = core_id(i, j)
        sq_xy[s] = core[sq_id[s]]
    th = -np.pi / 4 + 2 * np.pi * np.arange(Nc) / Nc
    circ = np.stack([np.cos(th), np.sin(th)], axis=1)
    rings = []
    for k in range(1, n_ring + 1):
        rings.append(sq_xy + (k / n_ring) * (r1 * circ - sq_xy))
    rings.append(r2 * circ)
    rings.append(R * circ)
    sec = np.vstack([core] + rings)             # plane nodes
    Np = sec.shape[0]

    def ring_id(k, s):                          # ring 0 = square boundary (core nodes)
        s = s % Nc
        return sq_id[s] if k == 0 else ncore + (k - 1) * Nc + s

    zs = _z_planes(length, h_z, np.asarray(frame_z, float), frame_t)
    nz = len(zs)
    coords = np.empty((Np * nz, 3))
    for kz, z in enumerate(zs):
        coords[kz * Np:(kz + 1) * Np, :2] = sec
        coords[kz * Np:(kz + 1) * Np, 2] = z
    # section cells (CCW corner node ids) with their kind: 0 fluid, 1 frame zone, 2 skin
    cells, kind = [], []
    for j in range(n):
        for i in range(n):
            cells.append([core_id(i, j), core_id(i + 1, j), core_id(i + 1, j + 1), core_id(i, j + 1)])
            kind.append(0)
    for k in range(n_ring + 2):
        for s in range(Nc):
            cells.append([ring_id(k, s), ring_id(k + 1, s), ring_id(k + 1, s + 1), ring_id(k, s + 1)])
            kind.append(0 if k < n_ring else (1 if k == n_ring else 2))
    cells = np.array(cells, np.int64)
    kind = np.array(kind)
    fz = np.asarray(frame_z, float)
    elems, emat = [], []
    for kz in range(nz - 1):
        zc = 0.5 * (zs[kz] + zs[kz + 1])
        in_frame = len(fz) > 0 and np.min(np.abs(fz - zc)) < 0.5 * frame_t + 1e-12 and (zs[kz + 1] - zs[kz]) <= frame_t + 1e-9
        bot, top = cells + kz * Np, cells + (kz + 1) * Np
        elems.append(np.hstack([bot, top]))
        m = np.where(kind == 2, 1, np.where(kind == 1, 1 if in_frame else 0, 0))
        emat.append(m)
    elems = np.vstack(elems)
    emat = np.concatenate(emat).astype(np.int32)
    # drop nodes that no element uses (none here, kept for safety) -> keep numbering as is
    solid = np.unique(elems[emat == 1].ravel())
    zc = coords[solid, 2]
    clamped = np.sort(solid[np.isclose(zc, 0.0) | np.isclose(zc, length)])
    # faces
    F = elems[:, HEX_FACES]                      # (ne, 6, 4) outward
    key = np.sort(F, axis=2).reshape(-1, 4)
    owner = np.repeat(np.arange(len(elems)), 6)
    order = np.lexsort(key.T[::-1])
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    pairs = np.flatnonzero(same)
    a_idx, b_idx = order[pairs], order[pairs + 1]
    ea, eb = owner[a_idx], owner[b_idx]
    fl_a = emat[ea] == 0
    fl_b = emat[eb] == 0
    mixed = fl_a != fl_b
    fluid_face = np.where(fl_a[mixed], a_idx[mixed], b_idx[mixed])
    iface = F.reshape(-1, 4)[fluid_face]
    # boundary faces of skin elements on the outer radius
    single = np.ones(len(key), bool)
    single[order[pairs]] = False
    single[order[pairs + 1]] = False
    bf = np.flatnonzero(single)
    bf = bf[emat[owner[bf]] == 1]
    fn = F.reshape(-1, 4)[bf]
    rr = np.hypot(coords[fn, 0], coords[fn, 1])
    outer = np.all(np.abs(rr - R) < 1e-9, axis=1)
    skin_faces = fn[outer]
    air = air or Material(kind=FLUID, rho=1.21, eta=0.01, c=343.0)
    metal = metal or Material(kind=SOLID, rho=2700.0, eta=0.02, E=70e9, nu=0.3)
    return Mesh(coords=coords, elems=elems, elem_mat=emat, materials=[air, metal], clamped=clamped, iface=iface,
                meta=dict(kind="fuselage", R=R, length=length, skin_t=skin_t, frame_z=list(fz),
                          skin_faces=skin_faces, n_planes=nz, plane_nodes=Np))
