"""The allocation-free sweep entry point (cr_sweep_noalloc) against cr_sweep, through the C ABI.

Both entry points run the same sweep kernel; every (model, frequency) item is computed by one
workgroup whatever the launch shape, so the outputs agree bit for bit. Two calls in a row (the
second on a smaller model, so stale contents of the shared static scratch would show), both
precisions, and the size limit."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, krylov, rom

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


def _box_rom():
    w = W.box()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    rb = krylov.build_basis(ss, 2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"])
    return w.omegas, krylov.project(ss, rb.basis)


def _small_rom(q=17, L=3, n_o=5):
    rng = W.SplitMix64(991)
    u = rng.uniforms(3 * q * q + 2 * q * L + 2 * n_o * q)
    G = (u[:q * q] - 0.5).reshape(q, q) + 1j * (u[q * q:2 * q * q] - 0.5).reshape(q, q)
    H = (u[2 * q * q:3 * q * q] - 0.5).reshape(q, q)
    o = 3 * q * q
    FR = (u[o:o + q * L] - 0.5).reshape(q, L) + 1j * (u[o + q * L:o + 2 * q * L] - 0.5).reshape(q, L)
    o += 2 * q * L
    CR = (u[o:o + n_o * q] - 0.5).reshape(n_o, q) + 1j * (u[o + n_o * q:o + 2 * n_o * q] - 0.5).reshape(n_o, q)
    return dict(KR=G @ G.conj().T + q * np.eye(q) * (1 + 0.02j), MR=(H @ H.T + q * np.eye(q)) * 1e-5, FR=FR, CR=CR,
                flags=np.arange(L) % 2)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_sweep_two_calls(P, ctx, prec):
    print(f"noalloc sweep prec={prec}", flush=True)
    om1, r1 = _box_rom()
    r2 = _small_rom()
    om2 = 2 * np.pi * np.linspace(5, 300, 37)
    for om, r in ((om1, r1), (om2, r2)):          # second call: smaller order, fewer frequencies
        R = P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"])
        ref = R.sweep(om, prec=prec).cpu().numpy()
        got = R.sweep_noalloc(om, prec=prec).cpu().numpy()
        if prec == 1:
            assert np.array_equal(got, ref)   # same kernels: complex-FP32 LU + FP64 refinement
        else:
            # cr_sweep solves an FP64 model without damping through its Hessenberg-triangular
            # form, which needs device memory of its own; the allocation-free call keeps the dense
            # LU: the two agree to rounding
            assert rom.relative_error(got, ref).max() <= 1e-10
        assert R.last_info["not_converged"] == 0
        assert rom.relative_error(got, rom.sweep(r, om)).max() <= 1e-6
    # an empty sweep is a no-op
    assert R.sweep_noalloc(np.zeros(0), prec=prec).shape[0] == 0


def test_noalloc_rejects_sizes_beyond_its_scratch(P, ctx):
    print("noalloc size limit", flush=True)
    q = 2900          # 16 q^2 bytes per workgroup exceed the 128 MiB scratch
    KR = np.eye(q, dtype=complex)
    R = P.Rom.from_arrays(ctx, KR, 1e-6 * KR, np.ones((q, 1), complex), np.ones((1, q), complex), np.zeros(1))
    with pytest.raises(P.CabinRomError) as e:
        R.sweep_noalloc(np.array([100.0]), prec=0)
    assert e.value.name == "CR_E_UNSUPPORTED" and "scratch" in str(e.value)
    y = R.sweep(np.array([100.0]), prec=0)      # the allocating entry point still serves it
    assert torch.isfinite(torch.view_as_real(y)).all()
