"""The reduced sweep's Hessenberg-triangular path (models without damping matrix or
frequency-dependent terms, FP64): against the oracle's LAPACK solve at every frequency, and
against the dense-LU path with refinement, over orders that cover one and two rows per thread,
the smallest models and mixed load flags."""
import numpy as np
import pytest

import workloads as W
from oracle import rom

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


def _pencil(q, L, n_o, seed):
    """A seeded reduced model with a resonant band: K = diag(1..100) plus a complex perturbation
    (loss), M = I plus a small complex perturbation; random loads and receivers, mixed flags."""
    g = W.SplitMix64(seed)

    def cplx(*shape):
        u = g.uniforms(2 * int(np.prod(shape))) - 0.5
        return (u[: u.size // 2] + 1j * u[u.size // 2:]).reshape(shape)
    KR = np.diag(np.linspace(1.0, 100.0, q)).astype(complex) + 0.1 * cplx(q, q) + 0.02j * np.eye(q)
    MR = np.eye(q, dtype=complex) + 0.05 * cplx(q, q)
    FR = cplx(q, L)
    CR = cplx(n_o, q)
    flags = (np.arange(L) % 2).astype(np.int32)
    return dict(KR=KR, MR=MR, FR=FR, CR=CR, flags=flags)


@pytest.mark.parametrize("q,L,n_o", [(1, 1, 1), (2, 3, 4), (3, 16, 7), (97, 16, 50), (256, 5, 50), (257, 16, 50),
                                     (400, 16, 256)])
def test_hessenberg_sweep_matches_oracle(P, ctx, q, L, n_o):
    print(f"hessenberg sweep q={q} L={L} n_o={n_o}", flush=True)
    r = _pencil(q, L, n_o, 2310047340 + 7 * q + L)
    om = np.sqrt(np.linspace(0.3, 120.0, 37))
    R = P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"])
    Y = R.sweep(om, prec=P.CR_FP64).cpu().numpy()
    Yo = rom.sweep(r, om)
    err = rom.relative_error(Y, Yo)
    assert err.max() <= 1e-9, err.max()
    # the dense path with refinement (forced through the batched call's refine flag)
    Ys, info = P.sweep_batched(ctx, [R], om[None, :], prec=P.CR_FP64, tune=dict(variant=2, refine=1))
    assert rom.relative_error(Ys[0].cpu().numpy(), Yo).max() <= 1e-9
    assert info["n_perturbed"] == 0 and info["not_converged"] == 0


def test_hessenberg_batched_mixed_paths(P, ctx):
    """One batched launch with Hessenberg models and models that need the dense path (a damping
    matrix; an order above the Hessenberg limit): every model against the oracle."""
    print("hessenberg batched mixed paths", flush=True)
    specs = [(40, 4, 9), (600, 3, 9), (130, 16, 30), (64, 2, 5)]
    rs = [_pencil(q, L, n_o, 99 + q) for q, L, n_o in specs]
    roms = [P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"]) for r in rs]
    DR = 0.01 * np.eye(64, dtype=complex)
    roms[3] = P.Rom.from_arrays(ctx, rs[3]["KR"], rs[3]["MR"], rs[3]["FR"], rs[3]["CR"], rs[3]["flags"], DR=DR)
    om = np.stack([np.sqrt(np.linspace(0.5, 110.0, 23)) + 0.01 * k for k in range(len(rs))])
    Ys, info = P.sweep_batched(ctx, roms, om, prec=P.CR_FP64)
    for k, r in enumerate(rs):
        Yo = rom.sweep(r, om[k], DR=DR if k == 3 else None)
        assert rom.relative_error(Ys[k].cpu().numpy(), Yo).max() <= 1e-9, k
    assert info["not_converged"] == 0
