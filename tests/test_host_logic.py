"""Host-side logic of the library that needs no GPU: the proposer's input features."""
import numpy as np
import pytest

P = pytest.importorskip("paper_2310_04734_amd")


def test_mlp_features_definition():
    rng = np.random.default_rng(7)
    res = 10.0 ** rng.uniform(-9, -1, 256)
    res[17] = 0.0                                   # clamped at 1e-300
    used = np.array([0, 100, 255], np.int32)
    geom = np.array([0.25, -1.0, 0.5])
    x, m = P.mlp_features(res, used, geom)
    lg = np.log10(np.maximum(res, 1e-300))
    np.testing.assert_allclose(x[:256], (lg - lg.max()).astype(np.float32), rtol=0, atol=1e-5)
    np.testing.assert_array_equal(x[256:], geom.astype(np.float32))
    assert x[:256].max() == 0.0
    banned = {0, 1, 99, 100, 101, 254, 255}
    assert set(np.flatnonzero(m == 0)) == banned
    assert np.all(m[[i for i in range(256) if i not in banned]] == 1)


def test_mlp_features_rejects_bad_arguments():
    with pytest.raises(P.CabinRomError):
        P.mlp_features(np.zeros(0), np.zeros(0, np.int32))


def test_trained_proposer_weights_file():
    import os
    path = os.path.join(os.path.dirname(P.__file__), "data", "proposer_fuselage.npy")
    p = np.load(path, allow_pickle=False)
    n_params = 259 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 256 + 256
    assert p.dtype == np.float32 and p.shape == (n_params,) and np.isfinite(p).all()
