"""Radiance-cache network on the matrix cores against the FP64 oracle (oracle/mlp.py).

Bar: forward outputs and weight gradients agree with the oracle (BF16 rounding
emulated at the same points) with cosine similarity > 0.999 and relative L2
error < 2e-2; Adam matches its closed form; training on the GPU lowers the loss.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as M
from paper_1504_03151_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def _flat(ws):
    return np.concatenate([np.asarray(w, np.float32).reshape(-1) for w in ws])


def _unflat(v):
    out, o = [], 0
    for shape in [(64, 64)] * 5 + [(3, 64)]:
        k = shape[0] * shape[1]
        out.append(np.asarray(v[o:o + k], np.float64).reshape(shape))
        o += k
    return out


def _close(a, b, what):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
    rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
    assert cos > 0.999 and rel < 2e-2, (what, cos, rel)


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    ws = S.mlp_init_weights(seed)
    x = rng.uniform(-1, 1, size=(n, 3)) * 20
    nf = rng.normal(size=(n, 3))
    nf /= np.linalg.norm(nf, axis=1, keepdims=True)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    feats = M.encode(x, nf, v, [-20, -20, -20], [20, 20, 20])
    target = rng.uniform(0, 2, size=(n, 3))
    return ws, feats, target


# 200,003: more tiles than one round of the persistent grid (2,048 waves x 32 samples), ragged tail
@pytest.mark.parametrize("n", [1, 31, 100, 4099, 200003])
def test_forward_matches_oracle(rt, n):
    ws, feats, _ = _problem(1, n)
    w = rt.bf16_bits(torch.from_numpy(_flat(ws)).cuda())
    x = rt.bf16_bits(torch.from_numpy(feats.astype(np.float32)).cuda())
    y = rt.mlp_forward(w, x).cpu().numpy()
    yo, _ = M.forward(ws, feats)
    _close(y, yo, "forward")
    assert np.abs(y - yo).max() < 2e-2 * (np.abs(yo).max() + 1e-3)


# 70,001: more two-wave groups than training blocks (each block loops), ragged tail
@pytest.mark.parametrize("n", [32, 1000, 70001])
def test_gradients_match_oracle(rt, n):
    ws, feats, target = _problem(2, n)
    w = rt.bf16_bits(torch.from_numpy(_flat(ws)).cuda())
    x = rt.bf16_bits(torch.from_numpy(feats.astype(np.float32)).cuda())
    t = torch.from_numpy(target.astype(np.float32)).cuda()
    dw = torch.zeros(rt.mlp_num_params(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rt.mlp_grad(w, x, t, dw, loss)
    lo, go, _ = M.loss_and_grads(ws, feats, target)
    assert abs(loss.item() / (3 * n) - lo) <= 2e-2 * lo
    g = _unflat(dw.cpu().numpy())
    for l in range(6):
        _close(g[l], go[l], f"dW{l + 1}")


def test_adam_matches_closed_form_and_training_lowers_the_loss(rt):
    ws, feats, target = _problem(3, 2048)
    wm = torch.from_numpy(_flat(ws)).cuda()
    wb = rt.bf16_bits(wm)
    m = torch.zeros_like(wm)
    v = torch.zeros_like(wm)
    g = torch.randn_like(wm) * 1e-3
    g0 = g.clone()
    w0 = wm.clone()
    rt.mlp_adam(wm, wb, m, v, g, 1, lr=1e-3)
    torch.cuda.synchronize()
    step = (wm - w0).cpu().numpy()
    exp = -1e-3 * g0.cpu().numpy() / (np.abs(g0.cpu().numpy()) + 1e-8)
    np.testing.assert_allclose(step, exp, rtol=2e-3, atol=2e-9)
    assert (g == 0).all()
    assert torch.equal(wb, rt.bf16_bits(wm))
    # a few hundred steps on one batch
    x = rt.bf16_bits(torch.from_numpy(feats.astype(np.float32)).cuda())
    t = torch.from_numpy(target.astype(np.float32)).cuda()
    wm = torch.from_numpy(_flat(ws)).cuda()
    wb = rt.bf16_bits(wm)
    m.zero_()
    v.zero_()
    dw = torch.zeros_like(wm)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for s in range(1, 301):
        loss.zero_()
        rt.mlp_grad(wb.view(torch.int16), x, t, dw, loss)
        rt.mlp_adam(wm, wb, m, v, dw, s, lr=1e-3)
        if s in (1, 300):
            losses.append(loss.item() / (3 * 2048))
    assert losses[1] < 0.5 * losses[0], losses
