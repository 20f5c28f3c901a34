"""Domain decomposition (GMRES + additive Schwarz on the structure / fluid subdomains) through the
library against the oracle: the preconditioner's action on random vectors, and solves against the
oracle's direct SuperLU solution."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assembly, dd, krylov, solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.mark.parametrize("overlap,restricted", [(0, True), (1, True), (1, False), (2, True)])
def test_preconditioner_matches_oracle(P, ctx, overlap, restricted):
    print(f"dd preconditioner overlap={overlap} restricted={restricted}", flush=True)
    w = W.small_plate_cavity()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    om = 2 * np.pi * 140.0
    A = (ss["K"] - om ** 2 * ss["M"]).tocsr()
    doms = dd.subdomains(dd.structure(s["K"], s["M"]), s["n_u"], overlap)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    D = P.DomainDecomposition(g, overlap=overlap, restricted=restricted)
    u = W.SplitMix64(11).uniforms(4 * A.shape[0])
    R = (u[:2 * A.shape[0]] + 1j * u[2 * A.shape[0]:]).reshape(A.shape[0], 2)
    Zo = dd.preconditioner(A, doms, restricted)(R)
    Z = D.precondition(om, torch.from_numpy(R).to(ctx.device)).cpu().numpy()
    # two backward-stable solves of each subdomain system differ by up to kappa(A_j) u
    kappa = max(np.linalg.cond(A[idx][:, idx].toarray()) for idx, _ in doms)
    assert np.abs(Z - Zo).max() <= 50 * kappa * 2.2e-16 * np.abs(Zo).max(), kappa


@pytest.mark.parametrize("name", ["plate_cavity_small", "plate_cavity"])
def test_dd_solve_matches_direct(P, ctx, name):
    print(f"dd solve {name}", flush=True)
    w = {"plate_cavity_small": W.small_plate_cavity, "plate_cavity": W.plate_cavity_workload}[name]()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    an = g.analyse()
    D = P.DomainDecomposition(g, overlap=1, restricted=True, restart=100, max_iter=400, tol=1e-9)
    for f_hz in (37.0, 211.0):
        om = 2 * np.pi * f_hz
        b = solve.load_at(s["F"], s["flags"], om)
        x = D.solve(om, torch.from_numpy(b).to(ctx.device)).cpu().numpy()
        xo = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
        assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max(), f_hz
        info = D.last_info
        assert info["n_sub"] == 2 and info["rel_residual"] <= 1e-9
    print(f"dd {name}: iterations {info['iterations']}, subdomain factor entries {info['sub_factor_entries']} "
          f"vs full {an['factor_entries']}", flush=True)
