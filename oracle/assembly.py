"""Oracle, step O2: finite-element assembly of the coupled structural-acoustic (u-p) system.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, FP64 CPU definition that the GPU
library is checked against. It shares no code with the library and must never be imported
by the product path.

What it builds (paper, Section 2, Eq. (1)-(3), two-domain subset; damping as complex
stiffness, Section 3.3 text after Eq. (8)):

    K = [ K_s   -C  ]      M = [ M_s        0  ]      A(w) = K - w^2 M
        [ 0     K_f ]          [ rho0 C^T  M_f ]

  K_f = int grad N^T grad N dV                    (fluid, pressure DoF)
  M_f = (1 / c~^2) int N^T N dV,  c~^2 = c^2 (1 + i eta_f)
  K_s = int B^T D(E~, nu) B dV,   E~ = E (1 + i eta_s)       (solid, 3 displacement DoF / node)
  M_s = rho_s int N^T N dV (x) I_3
  C   = int_Gamma N_s^T n_f N_f dGamma, n_f the unit normal pointing out of the fluid.

Elements are trilinear hex8 with 2 x 2 x 2 Gauss points at +-1/sqrt(3) (weight 1); interface
and skin faces are bilinear quads with 2 x 2 Gauss points. Clamped displacement DoFs are
eliminated (their rows and columns are dropped).

Global DoF order (structure first, cabin last, as in the paper's domain numbering):
  u DoFs: for each solid node that is not clamped, in increasing node id, components x, y, z;
  p DoFs: for each fluid node, in increasing node id.

Loads (one column of F per load; f(w) = (i w)^flag * F[:, l]):
  volume velocity Q at fluid node s:  F[p(s)] = rho0 Q, flag 1  (f = i w rho0 Q e_s)
  point force F_d at solid node a:    F[u(a, d)] = F_d, flag 0
  skin pressure p_ext (nodal amplitudes, bilinear interpolation) on faces whose normal points
  away from the structure:            f_u = - int N_s^T p_ext n_out dGamma, flag 0
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

G = 1.0 / np.sqrt(3.0)
_XI = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
_GP3 = np.array([[a, b, c] for c in (-G, G) for b in (-G, G) for a in (-G, G)])
_XI2 = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
_GP2 = np.array([[a, b] for b in (-G, G) for a in (-G, G)])


def hex8_shape(p):
    """N_a = 1/8 (1 + xi xi_a)(1 + eta eta_a)(1 + zeta zeta_a) and its natural gradient."""
    xi, eta, ze = p
    f = [1 + xi * _XI[:, 0], 1 + eta * _XI[:, 1], 1 + ze * _XI[:, 2]]
    N = 0.125 * f[0] * f[1] * f[2]
    dN = np.stack([0.125 * _XI[:, 0] * f[1] * f[2],
                   0.125 * _XI[:, 1] * f[0] * f[2],
                   0.125 * _XI[:, 2] * f[0] * f[1]], axis=1)      # (8, 3)
    return N, dN


def quad4_shape(p):
    s, t = p
    f = [1 + s * _XI2[:, 0], 1 + t * _XI2[:, 1]]
    N = 0.25 * f[0] * f[1]
    dN = np.stack([0.25 * _XI2[:, 0] * f[1], 0.25 * _XI2[:, 1] * f[0]], axis=1)  # (4, 2)
    return N, dN


def _geometry(X):
    """Per element and Gauss point: shape values, physical gradients and detJ.

    X: (ne, 8, 3). Returns N (8g, 8), dNdx (ne, 8g, 8, 3), detJ (ne, 8g).
    """
    Ns, dNx, dets = [], [], []
    for p in _GP3:
        N, dN = hex8_shape(p)
        J = np.einsum("ai,eaj->eij", dN, X)            # J_ij = d x_j / d xi_i
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("inverted or degenerate hex8 element")
        dNdx = np.einsum("eij,aj->eai", np.linalg.inv(J), dN)
        Ns.append(N)
        dNx.append(dNdx)
        dets.append(det)
    return np.array(Ns), np.stack(dNx, axis=1), np.stack(dets, axis=1)


def fluid_element_matrices(X):
    """(K_e, M0_e) with K_e = int grad N grad N^T, M0_e = int N N^T (no 1/c^2)."""
    N, dNdx, det = _geometry(X)
    Ke = np.einsum("eg,egai,egbi->eab", det, dNdx, dNdx)
    Me = np.einsum("eg,ga,gb->eab", det, N, N)
    return Ke, Me


def isotropic_D(E, nu):
    """Voigt order (xx, yy, zz, xy, yz, xz), engineering shear strains."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6), dtype=np.result_type(E, 1.0))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def solid_element_matrices(X, E, nu, rho):
    """(K_e, M_e), 24 x 24 with DoF order (node a, component d) -> 3a + d."""
    N, dNdx, det = _geometry(X)
    ne = X.shape[0]
    B = np.zeros((ne, 8, 6, 24))
    for a in range(8):
        gx, gy, gz = dNdx[:, :, a, 0], dNdx[:, :, a, 1], dNdx[:, :, a, 2]
        B[:, :, 0, 3 * a] = gx
        B[:, :, 1, 3 * a + 1] = gy
        B[:, :, 2, 3 * a + 2] = gz
        B[:, :, 3, 3 * a] = gy
        B[:, :, 3, 3 * a + 1] = gx
        B[:, :, 4, 3 * a + 1] = gz
        B[:, :, 4, 3 * a + 2] = gy
        B[:, :, 5, 3 * a] = gz
        B[:, :, 5, 3 * a + 2] = gx
    D = isotropic_D(E, nu)
    Ke = np.einsum("eg,egki,kl,eglj->eij", det, B, D, B)
    M8 = rho * np.einsum("eg,ga,gb->eab", det, N, N)
    Me = np.einsum("eab,cd->eacbd", M8, np.eye(3)).reshape(ne, 24, 24)
    return Ke, Me


def face_integrals(Xf):
    """For quads Xf (nf, 4, 3): W[f, a, b, d] = int N_a N_b n_d dGamma (n unnormalised x dGamma)."""
    W = np.zeros((Xf.shape[0], 4, 4, 3))
    for p in _GP2:
        N, dN = quad4_shape(p)
        ts = np.einsum("a,fai->fi", dN[:, 0], Xf)
        tt = np.einsum("a,fai->fi", dN[:, 1], Xf)
        nvec = np.cross(ts, tt)                       # = n dGamma / (ds dt)
        W += np.einsum("a,b,fd->fabd", N, N, nvec)
    return W


class DofMap:
    """Global numbering: free solid-node displacements first, then fluid-node pressures."""

    def __init__(self, mesh):
        from workloads.meshes import FLUID, SOLID
        n = mesh.n_nodes
        kinds = np.array([m.kind for m in mesh.materials])
        el_fluid = kinds[mesh.elem_mat] == FLUID
        el_solid = kinds[mesh.elem_mat] == SOLID
        is_f = np.zeros(n, bool)
        is_s = np.zeros(n, bool)
        is_f[mesh.elems[el_fluid].ravel()] = True
        is_s[mesh.elems[el_solid].ravel()] = True
        free_s = is_s.copy()
        free_s[mesh.clamped] = False
        self.u = -np.ones((n, 3), np.int64)
        su = np.nonzero(free_s)[0]
        self.u[su] = 3 * np.arange(len(su))[:, None] + np.arange(3)[None, :]
        self.n_u = 3 * len(su)
        self.p = -np.ones(n, np.int64)
        fp = np.nonzero(is_f)[0]
        self.p[fp] = self.n_u + np.arange(len(fp))
        self.n_p = len(fp)
        self.n = self.n_u + self.n_p
        self.el_fluid, self.el_solid = el_fluid, el_solid


def _fluid_material(mesh):
    from workloads.meshes import FLUID
    fl = [m for m in mesh.materials if m.kind == FLUID]
    if len(fl) != 1:
        raise ValueError("exactly one fluid material is supported")
    return fl[0]


def assemble(mesh, loads, receivers):
    """Return dict(K, M: csr complex128 n x n, F: n x L complex128, flags: (L,) int,
    recv: (n_o,) int64 DoF ids, n_u, n_p, dof: DofMap)."""
    from workloads.meshes import LOAD_POINT_FORCE, LOAD_SKIN_PRESSURE, LOAD_VOLUME_VELOCITY
    dm = DofMap(mesh)
    rows, cols, kv, mv = [], [], [], []

    def add(r, c, kval, mval):
        keep = (r >= 0) & (c >= 0)
        rows.append(r[keep]); cols.append(c[keep])
        kv.append(np.asarray(kval)[keep]); mv.append(np.asarray(mval)[keep])

    for mi, mat in enumerate(mesh.materials):
        sel = mesh.elem_mat == mi
        if not np.any(sel):
            continue
        conn = mesh.elems[sel]
        X = mesh.coords[conn]
        if mat.kind == 0:     # fluid
            Ke, M0 = fluid_element_matrices(X)
            c2 = mat.c ** 2 * (1 + 1j * mat.eta)
            d = dm.p[conn]                                   # (ne, 8)
            r = np.repeat(d[:, :, None], 8, 2).ravel()
            c = np.repeat(d[:, None, :], 8, 1).ravel()
            add(r, c, Ke.ravel().astype(complex), (M0 / c2).ravel())
        else:                 # solid
            Et = mat.E * (1 + 1j * mat.eta)
            Ke, Me = solid_element_matrices(X, Et, mat.nu, mat.rho)
            d = dm.u[conn].reshape(len(conn), 24)
            r = np.repeat(d[:, :, None], 24, 2).ravel()
            c = np.repeat(d[:, None, :], 24, 1).ravel()
            add(r, c, Ke.ravel(), Me.ravel().astype(complex))

    if len(mesh.iface):
        rho0 = _fluid_material(mesh).rho
        W = face_integrals(mesh.coords[mesh.iface])           # (nf, 4, 4, 3)
        ud = dm.u[mesh.iface]                                 # (nf, 4, 3)
        pd = dm.p[mesh.iface]                                 # (nf, 4)
        r = np.broadcast_to(ud[:, :, None, :], W.shape).ravel()
        c = np.broadcast_to(pd[:, None, :, None], W.shape).ravel()
        w = W.ravel().astype(complex)
        add(r, c, -w, np.zeros_like(w))                       # K: -C in (u, p)
        add(c, r, np.zeros_like(w), rho0 * w)                 # M: rho0 C^T in (p, u)

    n = dm.n
    R, Cc = np.concatenate(rows), np.concatenate(cols)
    K = sp.csr_matrix((np.concatenate(kv), (R, Cc)), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv), (R, Cc)), shape=(n, n))
    K.sum_duplicates(); M.sum_duplicates()

    L = len(loads)
    F = np.zeros((n, L), dtype=complex)
    flags = np.zeros(L, np.int64)
    for l, ld in enumerate(loads):
        if ld.kind == LOAD_VOLUME_VELOCITY:
            F[dm.p[ld.node], l] = _fluid_material(mesh).rho * ld.value
            flags[l] = 1
        elif ld.kind == LOAD_POINT_FORCE:
            F[dm.u[ld.node, ld.dir], l] = ld.value
        elif ld.kind == LOAD_SKIN_PRESSURE:
            W = face_integrals(mesh.coords[ld.faces])         # (nf, 4, 4, 3)
            P = ld.amp[ld.faces]                              # (nf, 4) nodal pressure
            fa = -np.einsum("fabd,fb->fad", W, P)             # (nf, 4, 3)
            ud = dm.u[ld.faces]
            keep = ud >= 0
            np.add.at(F[:, l], ud[keep], fa[keep])
        else:
            raise ValueError("unknown load kind")
    recv = dm.p[np.asarray(receivers)]
    if np.any(recv < 0):
        raise ValueError("receiver without a pressure DoF")
    return dict(K=K, M=M, F=F, flags=flags, recv=recv.astype(np.int64), n_u=dm.n_u,
                n_p=dm.n_p, dof=dm)
