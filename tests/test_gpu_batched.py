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
