"""Frequency-dependent loss factors (plate and air eta(f) tables) through the library against the
oracle, which reassembles the model at every frequency: the same subspace at fixed expansion
points (each with its own matrices) and reduced outputs within 1e-6, where the library forms
K_R(w), M_R(w) from per-term projections."""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assembly, freqdep, rom, solve

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


def _model():
    w = W.small_plate_cavity()
    tabs = {1: ((10.0, 150.0, 400.0), (0.005, 0.03, 0.06)), 0: ((10.0, 400.0), (0.002, 0.03))}
    mats = [dataclasses.replace(m, eta_table=tabs[m.kind]) for m in w.mesh.materials]
    return w, dataclasses.replace(w.mesh, materials=mats)


def test_frequency_dependent_materials_match_oracle(P, ctx):
    print("frequency-dependent materials", flush=True)
    w, mesh = _model()
    shifts = 2 * np.pi * np.array([70.0, 260.0])
    g = P.assemble(ctx, mesh, w.loads, w.receivers)
    g.analyse()
    B = g.basis(shifts, 4, prec=P.CR_FP64)
    rb, d = freqdep.build_basis(mesh, w.loads, w.receivers, shifts, 4)
    assert B.q == rb.q == 8
    sv = sla.svdvals(rb.basis.conj().T @ B.V().cpu().numpy())
    assert sv.min() > 1 - 1e-8
    R = B.project()
    om = 2 * np.pi * np.linspace(12.0, 398.0, 24)
    Yo = freqdep.sweep(mesh, w.loads, w.receivers, rb.basis, d, om)
    for prec in (P.CR_FP64, P.CR_MIXED):
        Y = R.sweep(om, prec=prec).cpu().numpy()
        assert rom.relative_error(Y, Yo).max() <= 1e-6, prec
    Yb, _ = P.sweep_batched(ctx, [R], om[None, :], prec=P.CR_MIXED)
    assert rom.relative_error(Yb[0].cpu().numpy(), Yo).max() <= 1e-6
    for wj in shifts:   # interpolation: the full response with the matrices at w_j
        s = assembly.assemble(freqdep.mesh_at(mesh, wj / (2 * np.pi)), w.loads, w.receivers)
        y = solve.full_frf(s, [wj])
        assert rom.relative_error(R.sweep([wj], prec=P.CR_FP64).cpu().numpy(), y).max() < 1e-8
    with pytest.raises(P.CabinRomError) as e:
        g.basis_greedy((10.0, 400.0), 16, 2, 1e-6, 2, prec=P.CR_FP64)
    assert e.value.name == "CR_E_UNSUPPORTED"
    with pytest.raises(P.CabinRomError) as e:
        R.sweep_noalloc(om, prec=P.CR_FP64)
    assert e.value.name == "CR_E_UNSUPPORTED"
