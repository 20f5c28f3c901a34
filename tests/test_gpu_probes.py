"""Achievable-peak probes used by the rooflines: plausible rates and argument checks."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2310_04734_amd as P
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return P


def test_probes_report_plausible_peaks(P):
    ctx = P.Context(0)
    print("probes", flush=True)
    gbs = ctx.probe_copy(64 << 20, 5)
    f64 = ctx.probe_mfma(P.CR_FP64, 2)
    f32 = ctx.probe_mfma(P.CR_MIXED, 2)
    # below the published peaks (8 TB/s; 78.6 and 157.3 TFLOP/s dense) and far above host rates
    assert 500.0 < gbs < 8000.0 * 1.05, gbs
    assert 5.0 < f64 < 78.6 * 1.05, f64
    assert 5.0 < f32 < 157.3 * 1.05, f32
    with pytest.raises(P.CabinRomError):
        ctx.probe_copy(100, 1)   # not a multiple of 16 bytes
