"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances: reduced outputs y_R within 1e-6 relative (per frequency and load, 2-norm over the
receivers), the bar the method is held to; assembled matrices entrywise within 1e-13 of the
largest entry (both sides sum the same element integrals in a different order); shifted solves
within a backward error of 1e-14 after FP64 refinement.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import assembly, greedy, krylov, rom, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _oracle_box_rom():
    w = W.box()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    rb = krylov.build_basis(ss, 2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"])
    return w, s, rb, krylov.project(ss, rb.basis)


def _rel(Y, Yref):
    return rom.relative_error(np.asarray(Y), np.asarray(Yref))


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_parity_box_rom(P, ctx, prec):
    _flush(f"sweep parity box prec={prec}")
    w, s, rb, r = _oracle_box_rom()
    R = P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"])
    Y = R.sweep(w.omegas, prec=prec).cpu().numpy()
    Yo = rom.sweep(r, w.omegas)
    assert _rel(Y, Yo).max() <= 1e-6
    if prec == 1:
        assert R.last_info["not_converged"] == 0


def test_sweep_edge_cases(P, ctx):
    """q = 1, q not a multiple of the panel width, several loads, Rayleigh damping, empty sweep."""
    rng = W.SplitMix64(77)
    for q, L, n_o in [(1, 1, 1), (17, 3, 5), (70, 2, 9), (130, 1, 4)]:
        _flush(f"sweep edge q={q} L={L}")
        u = rng.uniforms(4 * q * q + 2 * q * L + 2 * n_o * q)
        G = (u[:q * q] - 0.5).reshape(q, q) + 1j * (u[q * q:2 * q * q] - 0.5).reshape(q, q)
        KR = G @ G.conj().T + q * np.eye(q) * (1 + 0.02j)
        H = (u[2 * q * q:3 * q * q] - 0.5).reshape(q, q)
        MR = (H @ H.T + q * np.eye(q)) * 1e-5
        o = 4 * q * q
        FR = (u[o:o + q * L] - 0.5).reshape(q, L) + 1j * (u[o + q * L:o + 2 * q * L] - 0.5).reshape(q, L)
        o += 2 * q * L
        CR = (u[o:o + n_o * q] - 0.5).reshape(n_o, q) + 1j * (u[o + n_o * q:o + 2 * n_o * q] - 0.5).reshape(n_o, q)
        flags = np.arange(L) % 2
        DR = 1e-4 * MR + 1e-6 * KR
        oms = 2 * np.pi * np.linspace(5, 300, 37)
        for prec in (0, 1):
            R = P.Rom.from_arrays(ctx, KR, MR, FR, CR, flags, DR=DR)
            Y = R.sweep(oms, prec=prec).cpu().numpy()
            Yo = rom.sweep(dict(KR=KR, MR=MR, FR=FR, CR=CR, flags=flags), oms, DR=DR)
            assert _rel(Y, Yo).max() <= 1e-6, (q, L, prec)
    R = P.Rom.from_arrays(ctx, KR, MR, FR, CR, flags)
    assert R.sweep(np.zeros(0), prec=1).shape[0] == 0


def _fuselage_small():
    """A short coarse fuselage segment with three random-phase skin-pressure loads."""
    return W.fuselage_workload(n_core=4, n_ring=2, h_z=0.25, n_loads=3, n_freq=16, length=1.0, frame_z=(0.5,))


@pytest.mark.parametrize("name", ["box", "plate_cavity_small", "plate_cavity", "fuselage_small_skin_load"])
def test_assembly_parity(P, ctx, name):
    _flush(f"assembly parity {name}")
    w = {"box": W.box, "plate_cavity_small": W.small_plate_cavity, "plate_cavity": W.plate_cavity_workload,
         "fuselage_small_skin_load": _fuselage_small}[name]()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    e = g.export()
    import scipy.sparse as sp
    n = g.n
    assert n == s["K"].shape[0] and g.n_u == s["n_u"]
    Kg = sp.csr_matrix((e["K"], e["col"], e["rowptr"]), shape=(n, n))
    Mg = sp.csr_matrix((e["M"], e["col"], e["rowptr"]), shape=(n, n))
    for A, B in ((Kg, s["K"]), (Mg, s["M"])):
        scale = abs(B).max()
        assert abs(A - B).max() <= 1e-13 * scale
    assert np.abs(e["F"] - s["F"]).max() <= 1e-13 * max(np.abs(s["F"]).max(), 1e-300)
    assert np.array_equal(e["recv"], s["recv"]) and np.array_equal(e["flags"], s["flags"])


@pytest.mark.parametrize("prec", [0, 1])
def test_factor_solve_plate_cavity(P, ctx, prec):
    _flush(f"factor/solve plate_cavity prec={prec}")
    w = W.plate_cavity_workload()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    info = g.analyse()
    assert info["n_fronts"] > 1
    for f_hz in (12.0, 211.0, 399.0):
        om = 2 * np.pi * f_hz
        b = solve.load_at(s["F"], s["flags"], om)
        x_ref = solve.full_solve(s["K"], s["M"], s["F"], s["flags"], om)
        fac = g.factor(om, prec)
        x = fac.solve(torch.from_numpy(b).to(ctx.device)).cpu().numpy()
        assert fac.last_info["backward_error"] <= 1e-14
        # certificate computed by the oracle: normwise backward error of the GPU solution in
        # the Jacobi-scaled norm the library refines in, and forward error against SuperLU
        # (which carries the condition number of A near the resonances, ~1e7-1e8 here)
        ss = krylov.jacobi_scaled(s)
        d = ss["scale"]
        A = (ss["K"] - om ** 2 * ss["M"]).tocsr()
        xs, bs = x / d[:, None], d[:, None] * b
        r = bs - A @ xs
        be = np.abs(r).max() / (abs(A).sum(axis=1).max() * np.abs(xs).max() + np.abs(bs).max())
        assert be <= 1e-14, (f_hz, be)
        err = np.abs(x - x_ref).max() / np.abs(x_ref).max()
        assert err <= 1e-6, (f_hz, err)


def test_basis_fixed_box(P, ctx):
    _flush("basis fixed box")
    w, s, rb, r = _oracle_box_rom()
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    for prec in (0, 1):
        B = g.basis(2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"], prec=prec)
        assert B.q == rb.q and B.info["deflated"] == rb.deflated
        V = B.V().cpu().numpy()
        assert np.abs(V.conj().T @ V - np.eye(B.q)).max() < 1e-12
        R = B.project()
        Y = R.sweep(w.omegas, prec=1).cpu().numpy()
        Yo = rom.sweep(r, w.omegas)
        assert _rel(Y, Yo).max() <= 1e-6


def test_basis_partial_blocks(P, ctx):
    """13 loads of which 3 repeat earlier ones: the first block at each point deflates, so the
    Gram products run on blocks of 13 and 10 columns (the matrix-core path for 5..16 columns with
    a ragged column count), and the box's 528 rows leave a ragged last row chunk."""
    _flush("basis partial blocks")
    w = W.box()
    fn = W.fluid_nodes(w.mesh)
    nodes = [int(v) for v in W.SplitMix64(W.stream_seed(9, 1)).sample(fn, 10)]
    nodes += nodes[:3]
    w.loads = [W.Load(kind=W.LOAD_VOLUME_VELOCITY, node=nd, value=1.0 + 0.0j) for nd in nodes]
    shifts, blocks = 2 * np.pi * np.array([80.0, 200.0, 320.0]), 3
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    ss = krylov.jacobi_scaled(s)
    rb = krylov.build_basis(ss, shifts, blocks)
    r = krylov.project(ss, rb.basis)
    assert rb.deflated >= 3
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    B = g.basis(shifts, blocks, prec=P.CR_FP64)
    assert B.q == rb.q and B.info["deflated"] == rb.deflated
    V = B.V().cpu().numpy()
    assert np.abs(V.conj().T @ V - np.eye(B.q)).max() < 1e-12
    Y = B.project().sweep(w.omegas, prec=P.CR_FP64).cpu().numpy()
    assert _rel(Y, rom.sweep(r, w.omegas)).max() <= 1e-6


def test_greedy_plate_cavity(P, ctx):
    _flush("greedy plate_cavity")
    w = W.plate_cavity_workload()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    rp = w.rom
    go = greedy.greedy(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], rp["max_shifts"])
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    B = g.basis_greedy(rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], rp["max_shifts"], prec=1)
    assert list(B.trace["shift_idx"]) == list(go["shift_idx"])
    assert B.q == go["basis"].q
    # the residual estimate agrees with the oracle's while it is above rounding level (an
    # unconverged model is evaluated next to its own spurious poles, where x_R is sensitive to
    # the rounding of the basis); once the model has converged both are below the tolerance
    for a, b in zip(B.trace["max_res"], go["maxres"]):
        if b > 1e-5:
            assert abs(a - b) <= 1e-4 * b, (a, b)
    assert B.trace["max_res"][-1] <= rp["tol"] and go["maxres"][-1] <= rp["tol"]
    R = B.project()
    Y = R.sweep(w.omegas, prec=1).cpu().numpy()
    Yo = rom.sweep(go["rom"], w.omegas)
    assert _rel(Y, Yo).max() <= 1e-6


def test_batched_sweep(P, ctx):
    _flush("batched sweep")
    w, s, rb, r = _oracle_box_rom()
    ss = krylov.jacobi_scaled(s)
    roms_o, roms_g = [], []
    for k, blocks in enumerate([2, 5, 3, 8, 10, 1]):
        shifts = 2 * np.pi * np.array([80.0, 200.0, 320.0, 440.0])[: 1 + k % 4]
        b = krylov.build_basis(ss, shifts, blocks)
        ro = krylov.project(ss, b.basis)
        roms_o.append(ro)
        roms_g.append(P.Rom.from_arrays(ctx, ro["KR"], ro["MR"], ro["FR"], ro["CR"], ro["flags"]))
    oms = np.stack([2 * np.pi * np.linspace(20 + 3 * k, 500 - 5 * k, 211) for k in range(len(roms_o))])
    for prec in (0, 1):
        Ys, info = P.sweep_batched(ctx, roms_g, oms, prec=prec)
        for k in range(len(roms_o)):
            Yo = rom.sweep(roms_o[k], oms[k])
            assert _rel(Ys[k].cpu().numpy(), Yo).max() <= 1e-6, (k, prec)


def test_greedy_stall_stop_box(P, ctx):
    """The saturation stop of the greedy: the same points up to saturation and the same stop as the
    oracle (past saturation every residual is at rounding level, so which candidate the maximum
    picks there is not compared)."""
    _flush("greedy stall stop")
    w = W.box()
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    go = greedy.greedy(s, (20.0, 500.0), 64, 10, 1e-15, 30, stall_stop=2)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    B = g.basis_greedy((20.0, 500.0), 64, 10, 1e-15, 30, prec=P.CR_FP64, stall_stop=2)
    k = len(go["shift_idx"])
    assert len(B.trace["shift_idx"]) == k and B.q == go["basis"].q
    assert list(B.trace["shift_idx"][:k - 2]) == list(go["shift_idx"][:k - 2])


def test_greedy_residuals_many_loads(P, ctx):
    """Candidate residuals with 16 loads (q L above the single-pass kernel's LDS budget, so the
    matrix-core residual kernel runs): the same points and the same residual at every candidate
    as the oracle greedy on a thin-skin fuselage variant."""
    _flush("greedy residuals 16 loads")
    vs, _, _ = W.fuselage_variants()
    w, _geom = vs[0]
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    go = greedy.greedy(s, (20.0, 300.0), 256, 2, 1e-3, 2)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    B = g.basis_greedy((20.0, 300.0), 256, 2, 1e-3, 2, prec=P.CR_FP64)
    assert B.q == go["basis"].q and B.q * g.L > 512
    assert list(B.trace["shift_idx"]) == list(go["shift_idx"])
    a, b = np.asarray(B.trace["res"]), np.asarray(go["res"])
    # at the expansion points both residuals are at rounding level (~1e-8 relative to ||f||);
    # x_R next to the unconverged model's spurious poles is sensitive to the rounding of the
    # basis (see the plate-cavity greedy above); elsewhere the two agree to many digits
    big = b > 1e-5
    rel = np.abs(a - b)[big] / b[big]
    assert big.sum() >= 200 and np.median(rel) <= 1e-9 and rel.max() <= 1e-4, (np.median(rel), rel.max())
    assert np.all(a[~big] <= 1e-5)
