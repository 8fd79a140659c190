"""GPU cost-model kernels against the FP64 reference (oracle/mlp_ref.py):
forward values and gradients within 1e-4 relative, Adam steps, training and
the argmin pick."""
import ctypes

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = hawk.Context(0)
    yield c
    c.close()


def _data(seed, m):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-3, 12, size=(m, 12)).astype(np.float32)
    y = (0.4 * X[:, 0] - 0.3 * X[:, 7] + np.sin(X[:, 2]) + 0.1 * X[:, 11] ** 2).astype(np.float32)
    mu = X.mean(0).astype(np.float32)
    sd = (X.std(0) + 0.3).astype(np.float32)
    return X, y, mu, sd


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_matches_fp64_reference(ctx, seed):
    X, _, mu, sd = _data(seed, 1000)
    theta = M.init(seed).astype(np.float32)
    model = hawk.Model(ctx)
    model.set_params(theta, mu, sd)
    got = model.predict(X)
    ref, _ = M.forward(theta.astype(np.float64), X.astype(np.float64), mu.astype(np.float64), sd.astype(np.float64))
    assert np.all(np.abs(got - ref) <= 1e-4 * np.abs(ref) + 1e-4 * np.abs(ref).max())


@pytest.mark.parametrize("m", [1, 37, 3000])
def test_gradient_matches_fp64_reference(ctx, m):
    import torch
    X, y, mu, sd = _data(10 + m, m)
    theta = M.init(3).astype(np.float32)
    model = hawk.Model(ctx)
    model.set_params(theta, mu, sd)
    dX = torch.from_numpy(X).cuda()
    dy = torch.from_numpy(y).cuda()
    g = torch.zeros(M.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hawk.check(hawk.L().hawk_mlp_grad_dev(model.handle, ctypes.c_void_p(dX.data_ptr()), ctypes.c_void_p(dy.data_ptr()),
                                          m, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr())))
    torch.cuda.synchronize()
    gref, lref = M.grad(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64),
                        mu.astype(np.float64), sd.astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    scale = np.abs(gref).max()
    assert np.all(np.abs(gg - gref) <= 1e-4 * np.abs(gref) + 1e-4 * scale), np.abs(gg - gref).max() / scale
    assert abs(float(loss.item()) - lref) <= 1e-4 * lref


def test_adam_steps_match_reference(ctx):
    X, y, _, _ = _data(7, 500)
    theta0 = M.init(5)
    model = hawk.Model(ctx)
    model.set_params(theta0.astype(np.float32), np.zeros(12, np.float32), np.ones(12, np.float32))
    model.train(X, y, epochs=5, batch=500, lr=1e-3, seed=0)     # 5 full-batch steps
    p, mu, sd = model.get_params()
    # the library standardises with the training mean and population std
    Xd = X.astype(np.float64)
    mu_r = Xd.mean(0)
    sd_r = np.sqrt(np.maximum(0, (Xd ** 2).mean(0) - mu_r ** 2))
    assert np.allclose(mu, mu_r, rtol=1e-5, atol=1e-5) and np.allclose(sd, sd_r, rtol=1e-4)
    th = theta0.astype(np.float32).astype(np.float64)
    m1 = np.zeros_like(th)
    m2 = np.zeros_like(th)
    for t in range(1, 6):
        g, _ = M.grad(th, Xd, y.astype(np.float64), mu.astype(np.float64), sd.astype(np.float64))
        th, m1, m2 = M.adam_step(th, g, m1, m2, t, lr=1e-3)
    assert np.max(np.abs(p - th)) < 1e-4


def test_training_fits_and_pick_is_argmin(ctx):
    X, y, _, _ = _data(21, 4000)
    model = hawk.Model(ctx, seed=2)
    first = float(np.mean((model.predict(X) - y) ** 2))
    final = model.train(X, y, epochs=60, batch=256, lr=3e-3, seed=1)
    assert final < 0.05 * first
    pred = model.predict(X)
    assert np.mean((pred - y) ** 2) == pytest.approx(final, rel=1e-3)
    # the pick over a query's variant space is the argmin of the predictions
    tables, spec = dg.c2_aggregation(n=1000)
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    vs = hawk.variant_space(q)
    feats = np.stack([q.features(v) for v in vs])
    picked, pred_ms = model.pick([q])
    p = model.predict(feats)
    i = int(np.argmin(p))
    assert hawk.format_variant(picked[0]) == hawk.format_variant(vs[i])
    assert pred_ms[0] == pytest.approx(np.exp(p[i]), rel=1e-5)
    # a constant model ties everywhere: the first variant is chosen
    params = np.zeros(M.N_PARAMS, np.float32)
    params[-1] = 1.0
    model.set_params(params, np.zeros(12, np.float32), np.ones(12, np.float32))
    picked, _ = model.pick([q, q])
    assert all(hawk.format_variant(v) == hawk.format_variant(vs[0]) for v in picked)
