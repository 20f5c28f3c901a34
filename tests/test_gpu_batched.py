"""GPU parity of the batched sweep (many reduced models of uneven order in one persistent
launch) against per-model LAPACK sweeps of the FP64 oracle, the LDS-resident variant, the
autotuner, and HIP-graph replay against the eager launch."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, krylov, rom

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.fixture(scope="module")
def variant_roms():
    """Oracle ROMs of six seeded variants (coarse plate-cavity mesh), truncated to their q."""
    out = []
    for w, q in W.batched_variants(n_rom=6, q_range=(20, 140), n_freq=61, n_loads=4, plate_cells=(6, 4, 3)):
        s = assembly.assemble(w.mesh, w.loads, w.receivers)
        ss = krylov.jacobi_scaled(s)
        rb = krylov.build_basis(ss, 2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"] + 2)
        V = rb.basis[:, :min(q, rb.q)]
        out.append((w, krylov.project(ss, V)))
    return out


def _rel(Y, Yref):
    return rom.relative_error(np.asarray(Y), np.asarray(Yref))


def test_batched_variants_parity(P, ctx, variant_roms):
    _flush("batched variants parity")
    roms = [P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"]) for _, r in variant_roms]
    oms = np.stack([w.omegas for w, _ in variant_roms])
    qs = [r.q for r in roms]
    assert len(set(qs)) > 1
    refs = [rom.sweep(r, w.omegas) for w, r in variant_roms]
    for prec in (0, 1):
        Ys, info = P.sweep_batched(ctx, roms, oms, prec=prec)
        for k in range(len(roms)):
            assert _rel(Ys[k].cpu().numpy(), refs[k]).max() <= 1e-6, (k, prec)
        assert info["not_converged"] == 0


@pytest.mark.parametrize("tune", [{"variant": 1, "grid_per_cu": 2, "nb": 96}, {"variant": 2, "grid_per_cu": 1, "nb": 0},
                                  None])
def test_plan_graph_replay(P, ctx, variant_roms, tune):
    """A plan (explicit LDS-resident shape, explicit global shape, autotuned) replays its graph
    several times with eager library work in between; every replay equals the eager batched
    result bit for bit, and the oracle within 1e-6."""
    _flush(f"plan graph replay tune={tune}")
    roms = [P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"]) for _, r in variant_roms]
    oms = np.stack([w.omegas for w, _ in variant_roms])
    eager, _ = P.sweep_batched(ctx, roms, oms, prec=1)
    eager = [y.cpu().numpy() for y in eager]
    plan = P.SweepPlan(ctx, roms, oms, prec=1, tune=tune)
    if tune is None:
        t = plan.tuning()
        assert len(t["sample_ms"]) == 12 and t["grid_per_cu"] in (1, 2, 4)
    for rep in range(3):
        for Y in plan.outs:
            Y.zero_()
        info = plan.execute()
        assert info["not_converged"] == 0
        got = [y.cpu().numpy() for y in plan.outs]
        for k in range(len(roms)):
            assert np.array_equal(got[k], eager[k]), (rep, k)
        # eager work between replays: a single-model sweep and torch arithmetic
        roms[rep].sweep(oms[rep][:7], prec=1)
        torch.cuda.synchronize()
    for k, (w, r) in enumerate(variant_roms):
        assert _rel(plan.outs[k].cpu().numpy(), rom.sweep(r, w.omegas)).max() <= 1e-6


@pytest.fixture(scope="module")
def large_variant_roms():
    """Oracle ROMs of four seeded plate-cavity / box variants with 16 loads and orders above 256
    (the reduced LU's long-column panel path), truncated to their q."""
    out = []
    for w, q in W.batched_variants(n_rom=4, q_range=(257, 400), n_freq=41, n_loads=16, plate_cells=(12, 8, 6)):
        s = assembly.assemble(w.mesh, w.loads, w.receivers)
        ss = krylov.jacobi_scaled(s)
        rb = krylov.build_basis(ss, 2 * np.pi * w.rom["shifts_hz"], w.rom["blocks"])
        assert rb.q >= q
        out.append((w, krylov.project(ss, rb.basis[:, :q])))
    return out


def test_batched_large_orders_16_loads(P, ctx, large_variant_roms):
    """q in (256, 400] with 16 loads of very different response size per model: every result
    within 1e-6 of the oracle's LAPACK sweep in both precisions, refinement converged per load."""
    _flush("batched large orders, 16 loads")
    roms = [P.Rom.from_arrays(ctx, r["KR"], r["MR"], r["FR"], r["CR"], r["flags"]) for _, r in large_variant_roms]
    assert min(r.q for r in roms) > 256 and all(r.L == 16 for r in roms)
    oms = np.stack([w.omegas for w, _ in large_variant_roms])
    refs = [rom.sweep(r, w.omegas) for w, r in large_variant_roms]
    for prec in (0, 1):
        Ys, info = P.sweep_batched(ctx, roms, oms, prec=prec)
        for k in range(len(roms)):
            e = _rel(Ys[k].cpu().numpy(), refs[k])
            assert e.max() <= 1e-6, (k, prec, e.max())
        assert info["not_converged"] == 0 and info["n_perturbed"] == 0


def test_batched_loads_of_different_size(P, ctx, variant_roms):
    """Load columns scaled over twelve orders of magnitude: refinement must converge each column
    on its own (a backward error pooled over the columns would stop on the largest ones)."""
    _flush("batched loads of different size")
    out, refs, roms = [], [], []
    for w, r in variant_roms[:3]:
        sc = 10.0 ** (-np.arange(r["FR"].shape[1]) * 4.0)
        rr = dict(r, FR=r["FR"] * sc[None, :])
        roms.append(P.Rom.from_arrays(ctx, rr["KR"], rr["MR"], rr["FR"], rr["CR"], rr["flags"]))
        refs.append(rom.sweep(rr, w.omegas))
    oms = np.stack([w.omegas for w, _ in variant_roms[:3]])
    Ys, info = P.sweep_batched(ctx, roms, oms, prec=1)
    for k in range(len(roms)):
        assert _rel(Ys[k].cpu().numpy(), refs[k]).max() <= 1e-6, k
