"""The learned expansion-point proposer: what the trained network gains over the residual-max
greedy on the 16 held-out fuselage variants, at equal stopping tolerance (the greedy's residual
maximum stays the judge), and that the training data respect the split."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


def test_proposer_saves_expansion_points_on_held_out_variants(P):
    from paper_2310_04734_amd import proposer
    ctx = P.Context(0)
    variants, tr_idx, te_idx = W.fuselage_variants()
    assert len(set(tr_idx) & set(te_idx)) == 0 and len(te_idx) == 16
    net = proposer.load_trained(ctx)
    rows = proposer.compare(ctx, variants, te_idx, net)
    g = sum(r["greedy_factorizations"] for r in rows)
    m = sum(r["mlp_factorizations"] for r in rows)
    print(f"held-out variants: greedy {g} factorizations, with proposer {m}", flush=True)
    tol = variants[te_idx[0]][0].rom["tol"]
    for r in rows:
        # equal error: whenever a run stops before the cap it has reached the tolerance
        for k in ("greedy", "mlp"):
            if r[f"{k}_shifts"] < variants[r["variant"]][0].rom["max_shifts"]:
                assert r[f"{k}_maxres"] <= tol, r
    assert sum(r["mlp_converged"] for r in rows) >= sum(r["greedy_converged"] for r in rows)
    assert m < g
