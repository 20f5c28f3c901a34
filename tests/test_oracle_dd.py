"""Pins of the oracle's additive Schwarz preconditioner and GMRES (CPU)."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import assembly, dd, krylov, solve


def _scaled_at(om):
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    return s, ss, (ss["K"] - om ** 2 * ss["M"]).tocsr()


def test_block_jacobi_is_the_inverse_of_the_diagonal_blocks():
    """overlap 0: M^{-1} = blockdiag(A_uu^{-1}, A_pp^{-1}) (dense inverses on the small model)."""
    om = 2 * np.pi * 140.0
    s, ss, A = _scaled_at(om)
    nu = s["n_u"]
    doms = dd.subdomains(dd.structure(s["K"], s["M"]), nu, 0)
    assert [len(i) for i, _ in doms] == [nu, A.shape[0] - nu]
    Ad = A.toarray()
    Minv = np.zeros_like(Ad)
    Minv[:nu, :nu] = np.linalg.inv(Ad[:nu, :nu])
    Minv[nu:, nu:] = np.linalg.inv(Ad[nu:, nu:])
    r = W.SplitMix64(5).uniforms(2 * A.shape[0])
    r = r[:A.shape[0]] + 1j * r[A.shape[0]:]
    for restricted in (True, False):
        z = dd.preconditioner(A, doms, restricted)(r).ravel()
        assert np.allclose(z, Minv @ r, rtol=1e-10, atol=1e-12 * np.abs(z).max())


def test_overlap_grows_by_graph_layers_and_restriction_owns_each_dof_once():
    om = 2 * np.pi * 140.0
    s, ss, A = _scaled_at(om)
    nu = s["n_u"]
    G = dd.structure(s["K"], s["M"])
    # the coupling entries of a face normal's zero components are stored zeros: the assembled
    # connectivity holds more neighbours than the nonzero values of A
    assert G.nnz > (abs(A) > 0).sum()
    for ov in (1, 2):
        doms = dd.subdomains(G, nu, ov)
        prev = dd.subdomains(G, nu, ov - 1)
        for (idx, own), (pidx, _) in zip(doms, prev):
            mark = np.zeros(A.shape[0])
            mark[pidx] = 1
            assert np.array_equal(idx, np.flatnonzero((G @ mark) > 0))
        owners = np.zeros(A.shape[0], int)
        for idx, own in doms:
            owners[idx[own]] += 1
        assert np.all(owners == 1)


def test_whole_domain_subdomain_gives_one_iteration():
    """A subdomain holding every DoF makes M^{-1} = A^{-1}: GMRES converges in one step."""
    om = 2 * np.pi * 140.0
    s, ss, A = _scaled_at(om)
    doms = [(np.arange(A.shape[0]), np.ones(A.shape[0], bool))]
    b = ss["F"][:, 0].astype(complex)
    x, its = dd.gmres_right(A, b, dd.preconditioner(A, doms), 1e-9, 50, 50)
    assert its == 1
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_schwarz_gmres_converges_to_the_direct_solution():
    """Physics-based subdomains without and with one layer of overlap: GMRES reaches the direct
    solution, in a few iterations (the preconditioner captures most of the coupled operator)."""
    om = 2 * np.pi * 211.0
    s, ss, A = _scaled_at(om)
    b = solve.load_at(ss["F"], ss["flags"], om)[:, 0]
    xd = sp.linalg.spsolve(A.tocsc(), b)
    its = {}
    for ov in (0, 1):
        doms = dd.subdomains(dd.structure(s["K"], s["M"]), s["n_u"], ov)
        x, its[ov] = dd.gmres_right(A, b, dd.preconditioner(A, doms), 1e-8, 100, 200)
        assert np.linalg.norm(A @ x - b) <= 1e-8 * np.linalg.norm(b)
        assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
        assert its[ov] <= 20
