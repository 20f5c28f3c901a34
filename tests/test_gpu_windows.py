"""Local reduced models on frequency windows (automated bisection partition) against the oracle's
windows: the same partition, the same expansion points per window, and the stitched sweep within
1e-6 of the oracle's per-window LAPACK sweeps."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, rom, windows

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


@pytest.mark.parametrize("max_shifts", [4, 2])
def test_local_windows_match_oracle(P, ctx, max_shifts):
    print(f"local windows max_shifts={max_shifts}", flush=True)
    w = W.small_plate_cavity()
    rp = w.rom
    s = assembly.assemble(w.mesh, w.loads, w.receivers)
    wo = windows.local_roms(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], max_shifts, 4)
    g = P.assemble(ctx, w.mesh, w.loads, w.receivers)
    g.analyse()
    lr = g.local_roms(rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], max_shifts, min_cand=4, prec=P.CR_FP64)
    assert [tuple(c) for c in lr.cand] == [(x["i0"], x["i1"]) for x in wo]
    assert lr.info["n_windows"] == len(wo) and lr.info["unconverged"] == sum(
        x["greedy"]["maxres"][-1] > rp["tol"] for x in wo)
    for k, x in enumerate(wo):
        assert lr.roms[k].q == x["greedy"]["basis"].q
        # converged windows agree on their residual level; unconverged ones are both above tol
        a, b = lr.max_res[k], x["greedy"]["maxres"][-1]
        assert (a <= rp["tol"]) == (b <= rp["tol"])
    om = 2 * np.pi * np.linspace(rp["band_hz"][0], rp["band_hz"][1], 301)
    Yo, owner = windows.sweep(wo, om)
    for prec in (P.CR_FP64, P.CR_MIXED):
        Y = lr.sweep(om, prec=prec).cpu().numpy()
        assert rom.relative_error(Y, Yo).max() <= 1e-6, prec
