"""Nonthermal (kappa) module on the GPU against the oracle.

- exact integrator (HIP) vs the oracle's integrator, element by element;
- general constant-coefficient Stokes update vs the oracle's matrix
  exponential;
- the surrogate's backward pass (HIP training kernel) vs the oracle's FP64
  backpropagation, its MFMA forward pass vs the oracle's forward pass, and a
  short training run on the GPU that must reduce the loss.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import mlp as omlp
from paper_2302_02733_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(f"[gpu-kappa] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_02733_amd import krt
    c = krt.Context(0)
    yield c
    c.close()


def _box_and_edges(n, seed):
    inp = W.kappa_inputs(n, seed)[:, :3].copy()
    edges = np.array([[3.0, 1.0, 1e-2], [8.0, 100.0, 1e6], [3.0, 100.0, 1e-2], [8.0, 1.0, 1e6],
                      [12.0, 0.3, 1e8], [3.05, 150.0, 1e-4], [5.0, 10.0, 700.0 * 10.0 / 100.0]])
    return np.concatenate([inp, edges])


def test_kappa_integrals_match_oracle(ctx):
    inp = _box_and_edges(249, 21)
    ref = oracle.kappa_integrals(inp)
    _log(f"exact integrator on {len(inp)} points")
    got = ctx.kappa_integrals(torch.tensor(inp, device=ctx.device)).cpu().numpy()
    rel = np.abs(got / ref - 1)
    _log(f"max rel err per integral {rel.max(0)}")
    assert np.all(np.isfinite(got))
    assert rel.max() < 1e-9


def _mueller_cases():
    r = np.random.default_rng(31)
    cases = []
    for regime in range(7):
        for _ in range(24):
            AI = 10 ** r.uniform(-3, 1)
            frac = r.uniform(0, 0.95)
            ang = r.uniform(0, 2 * np.pi)
            AQ, AV = AI * frac * np.cos(ang), AI * frac * np.sin(ang)
            if regime == 0:      # small invariants (series branch)
                RQ, RV = r.normal(0, 0.05, 2)
                AQ, AV = AQ * 0.01, AV * 0.01
            elif regime == 1:    # strong rotation
                RQ, RV = r.normal(0, 30, 2)
            elif regime == 2:    # pure rotation (x = 0)
                AQ = AV = 0.0
                RQ, RV = r.normal(0, 5, 2)
            elif regime == 3:    # pure dichroism (y = 0)
                RQ = RV = 0.0
            elif regime == 4:    # rotation along the dichroism axis (small x or y)
                RQ, RV = 3.0 * AQ + 1e-3, 3.0 * AV
            elif regime == 5:    # optically thick
                AI = 10 ** r.uniform(1, 2.5)
                AQ, AV = AI * 0.5, -AI * 0.3
                RQ, RV = r.normal(0, 10, 2)
            else:                # optical depth 1-20 with small invariants (series branch
                AI = 10 ** r.uniform(0.2, 1.3)    # with high-order Taylor terms of phi1)
                AQ, AV = r.uniform(-0.2, 0.2, 2)
                RQ, RV = r.uniform(-0.15, 0.15, 2)
            J = r.normal(0, 1, 3) * 10 ** r.uniform(-2, 1)
            J[0] = abs(J[0]) + np.hypot(J[1], J[2])
            S = r.normal(0, 1, 4)
            S[0] = abs(S[0]) + np.linalg.norm(S[1:])
            cases.append((np.array([J[0], J[1], J[2], AI, AQ, AV, RQ, RV]), S))
    return cases


@pytest.mark.parametrize("w", [0.0, 0.05, 1.0, 3.0])
def test_mueller_general_matches_oracle(ctx, w):
    cases = _mueller_cases()
    coef = np.array([c for c, _ in cases])
    S = np.array([s for _, s in cases])
    got = ctx.mueller_general(torch.tensor(coef, device=ctx.device), torch.tensor(S, device=ctx.device),
                              w).cpu().numpy()
    ref = np.array([oracle.mueller_step(c, s, w) for c, s in cases])
    # error relative to the output, with a floor at 1e-14 of the inputs' scale
    scale = np.abs(S).max(1) + np.abs(coef[:, :3]).max(1) * w
    err = np.abs(got - ref).max(1) / (np.abs(ref).max(1) + 1e-3 * scale)
    _log(f"w={w}: max rel err {err.max():.2e}")
    assert np.all(np.isfinite(got))
    assert err.max() <= 1e-11


def test_mueller_general_reduces_to_thermal(ctx):
    """With J = S_eq (A_I, A_Q, A_V) the general update equals the thermal one."""
    r = np.random.default_rng(5)
    n = 64
    AI = 10 ** r.uniform(-2, 1, n)
    AQ, AV = AI * 0.4, -AI * 0.2
    RQ, RV = r.normal(0, 3, n), r.normal(0, 3, n)
    seq = 10 ** r.uniform(-1, 1, n)
    S = np.abs(r.normal(0, 1, (n, 4)))
    gen = np.stack([seq * AI, seq * AQ, seq * AV, AI, AQ, AV, RQ, RV], 1)
    th = np.stack([seq, AI, AQ, AV, RQ, RV], 1)
    for w in (0.1, 2.0):
        a = ctx.mueller_general(torch.tensor(gen, device=ctx.device), torch.tensor(S, device=ctx.device), w)
        b = ctx.mueller_step(torch.tensor(th, device=ctx.device), torch.tensor(S, device=ctx.device), w)
        d = (a - b).abs().max().item() / b.abs().max().item()
        assert d < 1e-12


@pytest.fixture(scope="module")
def small_set(ctx):
    inp = W.kappa_inputs(2048, 77)
    integ = ctx.kappa_integrals(torch.tensor(inp[:, :3].copy(), device=ctx.device))
    return torch.tensor(inp, device=ctx.device), integ


def test_mlp_gradient_matches_cpu_backprop(ctx, small_set):
    inp, integ = small_set
    ctx.mlp_init(123)
    logs = np.log10(integ.cpu().numpy())
    # a baseline with nonzero coefficients, so that the residual targets are exercised
    cb = np.zeros((8, 20))
    cb[:, 0] = logs.mean(0)
    cb[:, 3] = 0.5
    cb[:, 6] = -0.25
    norm = np.concatenate([np.zeros(8), logs.std(0), cb.ravel()])
    p0, _ = ctx.mlp_get_params()
    ctx.mlp_set_params(p0, norm)
    n = 1000   # ragged: not a multiple of the 32-sample tile
    g, loss = ctx.mlp_grad(inp[:n].contiguous(), integ[:n].contiguous())
    g = g.cpu().numpy().astype(np.float64)
    loss_c, g_c = omlp.loss_and_grad(p0.astype(np.float64), norm, inp[:n].cpu().numpy(), integ[:n].cpu().numpy())
    _log(f"loss gpu {loss:.8e} cpu {loss_c:.8e}; max |dg| {np.abs(g - g_c).max():.2e} of {np.abs(g_c).max():.2e}")
    assert abs(loss / loss_c - 1) < 1e-5
    assert np.abs(g - g_c).max() <= 2e-5 * np.abs(g_c).max()
    for off, size in ((0, 256), (256, 64), (320, 4096), (4416, 64), (4480, 4096), (8576, 64), (8640, 512),
                      (9152, 8)):
        blk = slice(off, off + size)
        assert np.abs(g[blk] - g_c[blk]).max() <= 1e-4 * np.abs(g_c[blk]).max() + 1e-7 * np.abs(g_c).max()


def test_mlp_mfma_forward_matches_cpu(ctx, small_set):
    inp, integ = small_set
    ctx.mlp_init(7)
    logs = np.log10(integ.cpu().numpy())
    cb = np.zeros((8, 20))
    cb[:, 2] = 0.3
    cb[:, 19] = -0.1
    norm = np.concatenate([logs.mean(0), logs.std(0), cb.ravel()])
    p0, _ = ctx.mlp_get_params()
    ctx.mlp_set_params(p0, norm)
    n = 2048 - 37   # ragged against the 64-lane waves
    got = np.log10(ctx.mlp_eval(inp[:n].contiguous()).cpu().numpy())
    ref = omlp.predict_log10(p0, norm, inp[:n].cpu().numpy())
    dz = np.abs(got - ref) / norm[8:16]
    _log(f"MFMA forward: max |dz| {dz.max():.2e}, max |d log10| {np.abs(got - ref).max():.2e}")
    assert dz.max() < 1e-4


def test_mlp_training_reduces_loss(ctx, small_set):
    inp, integ = small_set
    ctx.mlp_init(11)
    # one epoch at a vanishing step fits the baseline and gives the initial loss
    loss0 = ctx.mlp_train(inp, integ, epochs=1, batch=256, lr_max=1e-12, lr_min=0.0, seed=3)
    _, norm0 = ctx.mlp_get_params()
    loss = ctx.mlp_train(inp, integ, epochs=200, batch=256, lr_max=3e-3, lr_min=1e-5, seed=3, set_norm=False)
    _log(f"training loss {loss0:.4e} -> {loss:.4e}")
    assert loss < 0.1 * loss0
    p1, norm1 = ctx.mlp_get_params()
    assert np.array_equal(norm1, norm0)
    # the fitted baseline is the least-squares cubic of log10 I in the features
    from oracle import mlp as om
    M = om.monomials(om.features(inp.cpu().numpy()))
    y = np.log10(integ.cpu().numpy())
    c_ls, *_ = np.linalg.lstsq(M, y, rcond=None)
    assert np.abs(norm1[16:].reshape(8, 20) - c_ls.T).max() < 1e-8 * max(1.0, np.abs(c_ls).max())
    assert np.allclose(norm1[8:16], (y - M @ c_ls).std(0), rtol=1e-6)
    loss_c = omlp.loss_and_grad(p1.astype(np.float64), norm1, inp.cpu().numpy(), integ.cpu().numpy())[0]
    assert abs(loss_c / loss - 1) < 1e-3
