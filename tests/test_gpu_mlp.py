"""GPU parity of the proposer network's own forward/backward kernels against the FP64 oracle
(same BF16-rounded weights), and training by the library's Adam kernel."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp

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


def _case(n_in, H, n_out, B, seed=3):
    _, n = mlp.layout(n_in, H, n_out)
    rng = W.SplitMix64(seed)
    p = ((rng.uniforms(n) - 0.5) * (2 * np.sqrt(6.0 / n_in))).astype(np.float32)
    X = (rng.uniforms(B * n_in).reshape(B, n_in) * -4.0).astype(np.float32)   # log-residual-like inputs
    labels = np.array([rng.randint(n_out) for _ in range(B)], np.int32)
    mask = np.ones((B, n_out), np.float32)
    for b in range(B):
        for _ in range(5):
            j = rng.randint(n_out)
            if j != labels[b]:
                mask[b, j] = 0.0
    return p, X, labels, mask


def test_forward_and_gradients_match_oracle(P, ctx):
    n_in, H, n_out, B = 259, 256, 256, 64
    p, X, labels, mask = _case(n_in, H, n_out, B)
    net = P.Mlp(ctx, n_in, H, n_out)
    net.set_params(p)
    pe = mlp.effective(p, n_in, H, n_out)
    logits_o, _, _ = mlp.forward(pe, X, n_in, H, n_out)
    logits_g = net.forward(torch.from_numpy(X).to(ctx.device)).cpu().numpy()
    assert np.abs(logits_g - logits_o).max() <= 1e-4 * np.abs(logits_o).max()
    loss_o, g_o = mlp.loss_and_grad(pe, X, labels, mask, n_in, H, n_out)
    loss_g, g_g = net.gradients(torch.from_numpy(X).to(ctx.device), torch.from_numpy(labels).to(ctx.device),
                                torch.from_numpy(mask).to(ctx.device))
    g_g = g_g.cpu().numpy().astype(np.float64)
    assert abs(loss_g - loss_o) <= 1e-5 * abs(loss_o)
    lay, _ = mlp.layout(n_in, H, n_out)
    for k, (o, sh) in enumerate(lay):
        nk = int(np.prod(sh))
        a, b = g_g[o:o + nk], g_o[o:o + nk]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-9, k


def test_training_reduces_loss(P, ctx):
    n_in, H, n_out, B = 259, 256, 256, 128
    p, X, labels, mask = _case(n_in, H, n_out, B, seed=9)
    net = P.Mlp(ctx, n_in, H, n_out, seed=1)
    Xt, lt, mt = (torch.from_numpy(a).to(ctx.device) for a in (X, labels, mask))
    first = net.train_step(Xt, lt, mt, lr=1e-3)
    for _ in range(60):
        last = net.train_step(Xt, lt, mt, lr=1e-3)
    assert last < 0.5 * first
    # the updated masters are finite and their BF16 copies are what the forward pass uses
    p2 = net.get_params()
    assert np.all(np.isfinite(p2))
    pe = mlp.effective(p2, n_in, H, n_out)
    logits_o, _, _ = mlp.forward(pe, X, n_in, H, n_out)
    logits_g = net.forward(Xt).cpu().numpy()
    assert np.abs(logits_g - logits_o).max() <= 1e-4 * np.abs(logits_o).max()
