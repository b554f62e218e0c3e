"""Pins of the oracle's surrogate network: the hand-written backward pass
against central finite differences of the forward pass, and the bfloat16
rounding against PyTorch's conversion."""
import numpy as np
import pytest

from oracle import mlp


def _params(seed):
    r = np.random.default_rng(seed)
    p = np.empty(mlp.NPARAMS, dtype=np.float64)
    off = 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        fan = shape[1] if len(shape) == 2 else 1
        p[off:off + n] = r.uniform(-1, 1, n) * (np.sqrt(6.0 / fan) if len(shape) == 2 else 0.3)
        off += n
    return p


def _set(n, seed):
    r = np.random.default_rng(seed)
    inp = np.stack([r.uniform(3, 8, n), 10 ** r.uniform(0, 2, n), 10 ** r.uniform(-2, 6, n),
                    np.cos(r.uniform(0, np.pi, n))], 1)
    integ = 10 ** r.normal(-3, 2, (n, 8))
    norm = np.concatenate([np.full(8, -3.0), np.linspace(0.5, 3.0, 8), r.normal(0, 0.5, 160)])
    return inp, integ, norm


def test_backprop_matches_finite_differences():
    p = _params(3)
    inp, integ, norm = _set(16, 4)
    loss, g = mlp.loss_and_grad(p, norm, inp, integ, rounded=False)
    r = np.random.default_rng(5)
    idx = np.concatenate([r.choice(np.arange(0, 256), 6), r.choice(np.arange(256, 320), 3),
                          r.choice(np.arange(320, 4416), 8), r.choice(np.arange(4480, 8576), 8),
                          r.choice(np.arange(8640, 9152), 6), np.arange(9152, 9160)])
    for k in idx:
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_and_grad(pp, norm, inp, integ, rounded=False)[0] -
              mlp.loss_and_grad(pm, norm, inp, integ, rounded=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-7 * abs(g[k]), (k, fd, g[k])


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(9)
    a = np.concatenate([r.normal(0, 1, 10000), r.normal(0, 1e-3, 1000), [0.0, -0.0, 1.0, 65504.0]]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(a), ref)


def test_forward_definition_small_case():
    """One hidden unit path by hand: with all weights zero except a chain of
    single entries, z is the composition of three SiLUs."""
    p = np.zeros(mlp.NPARAMS)
    d = mlp.unpack(p, rounded=False)
    d["W1"][0, 0] = 1.0
    d["W2"][0, 0] = 2.0
    d["W3"][0, 0] = 0.5
    d["W4"][3, 0] = 4.0
    d["b4"][:] = 0.25
    p = mlp.pack(d)
    inp = np.array([[8.0, 10.0, 100.0, 0.0]])
    x = (8.0 - 5.5) / 2.5   # exact in FP32
    s = lambda t: t / (1 + np.exp(-t))
    z3 = 4.0 * s(0.5 * s(2.0 * s(x))) + 0.25
    norm = np.concatenate([np.zeros(8), np.ones(8), np.zeros(160)])
    out = mlp.predict_log10(p, norm, inp)[0]
    assert abs(out[3] - z3) < 1e-15 and np.allclose(out[[0, 1, 2, 4, 5, 6, 7]], 0.25, rtol=0, atol=1e-15)
