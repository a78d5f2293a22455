"""GPU checks of the learned-bounds path.

Features (FP64) against the CPU reference computed from their definitions;
MLP forward, gradients and Adam (FP32 kernels) against the FP64 CPU MLP whose
gradient is pinned by finite differences; the prediction's fallback; and what
the trained network gains over Lanczos bounds with xi = 0 on held-out
operators (prediction quality itself is parity unpinned).
"""
import os

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2208_01339_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_01339_amd import binding

    binding.lib()
    return binding


def cases():
    return {
        "hetero21_jac": (lambda: (W.hetero_diffusion(21, 2.0, 5), None), True),
        "poisson12": (lambda: (W.poisson3d(12), None), False),
        "dfn_small_jac": (lambda: (None, W.dfn_schur(n_frac=13, G=16, n_traces=30, L_lo=3, L_hi=12, seed=2)), True),
    }


@pytest.mark.parametrize("name", list(cases()))
def test_features_match_reference(B, name):
    build, jac = cases()[name]
    a, s = build()
    if s is not None:
        op = B.Operator(schur=s, flags=B.PP_JACOBI if jac else 0)
        orc = O.Operator(s.a, s.c, s.m, jacobi=jac)
        ref = M.features(orc, s.a, s.c, s.m, power_steps=8)
    else:
        op = B.Operator(a=a, flags=B.PP_JACOBI if jac else 0)
        orc = O.Operator(a, jacobi=jac)
        ref = M.features(orc, a, power_steps=8)
    got = B.pp_features(op.handle, 8)
    op.close()
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-12), np.max(np.abs(got - ref) / (np.abs(ref) + 1e-12))


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_mlp_forward_and_gradient(B):
    h = B.pp_mlp_create(16, 128, 3, 3, seed=3)
    npar = B.pp_mlp_num_params(h)
    shapes = M.layer_shapes(16, 128, 3, 3)
    assert npar == sum(fi * fo + fo for fi, fo in shapes) == 35587
    p = torch.empty(npar, dtype=torch.float32, device="cuda")
    B.pp_mlp_get_params(h, p)
    torch.cuda.synchronize()
    params = p.cpu().numpy().astype(np.float64)
    X = _rand((64, 16), 1).astype(np.float32)
    T = _rand((64, 3), 2).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    Y = torch.empty(64, 3, dtype=torch.float32, device="cuda")
    B.pp_mlp_forward(h, Xd, Y)
    torch.cuda.synchronize()
    Yr, _ = M.forward(params, shapes, X.astype(np.float64))
    assert np.max(np.abs(Y.cpu().numpy() - Yr)) <= 1e-4 * (1 + np.max(np.abs(Yr)))
    g = torch.empty(npar, dtype=torch.float32, device="cuda")
    loss = B.pp_mlp_loss_grad(h, Xd, Td, g)
    torch.cuda.synchronize()
    Lr, gr = M.loss_grad(params, shapes, X.astype(np.float64), T.astype(np.float64))
    assert loss == pytest.approx(Lr, rel=1e-4)
    gg = g.cpu().numpy()
    assert np.linalg.norm(gg - gr) <= 1e-4 * np.linalg.norm(gr)
    B.pp_mlp_destroy(h)


def test_mlp_adam_step(B):
    h = B.pp_mlp_create(16, 32, 2, 3, seed=5)
    npar = B.pp_mlp_num_params(h)
    shapes = M.layer_shapes(16, 32, 2, 3)
    p = torch.empty(npar, dtype=torch.float32, device="cuda")
    B.pp_mlp_get_params(h, p)
    torch.cuda.synchronize()
    p0 = p.cpu().numpy().astype(np.float64)
    X = _rand((32, 16), 7).astype(np.float32)
    T = _rand((32, 3), 8).astype(np.float32)
    lr = 1e-3
    B.pp_mlp_train_step(h, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), lr)
    B.pp_mlp_get_params(h, p)
    torch.cuda.synchronize()
    p1 = p.cpu().numpy().astype(np.float64)
    _, g = M.loss_grad(p0, shapes, X.astype(np.float64), T.astype(np.float64))
    pr, _, _ = M.adam(p0, g, np.zeros(npar), np.zeros(npar), 1, lr)
    live = np.abs(g) > 1e-5 * np.max(np.abs(g))  # where the FP32 gradient's sign is reliable
    assert np.allclose((p1 - p0)[live], (pr - p0)[live], atol=2e-3 * lr)
    B.pp_mlp_destroy(h)


def test_mlp_training_reduces_loss(B):
    h = B.pp_mlp_create(16, 64, 2, 3, seed=9)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(256, 16)).astype(np.float32)
    A = rng.normal(size=(16, 3))
    T = (np.tanh(X @ A) + 0.1 * X[:, :3] ** 2).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = B.pp_mlp_loss_grad(h, Xd, Td)
    for _ in range(300):
        last = B.pp_mlp_train_step(h, Xd, Td, 3e-3)
    assert last < 0.1 * first
    B.pp_mlp_destroy(h)


def test_predict_bounds_fallback_and_pass(B):
    a = W.hetero_diffusion(20, 1.5, 4)
    op = B.Operator(a=a, flags=B.PP_JACOBI)
    lo, hi = B.pp_estimate_bounds(op.handle, 20)
    h = B.pp_mlp_create(16, 32, 2, 3, seed=1)
    # output std tiny: the prediction is the output mean whatever the features
    B.pp_mlp_set_normalization(h, np.zeros(16), np.ones(16), [np.log(lo), np.log(hi), np.log10(1e-3 + 1e-5)],
                               [1e-7, 1e-7, 1e-7])
    plo, phi, pxi, fb = B.pp_predict_bounds(op.handle, h, 8)
    assert not fb
    assert plo == pytest.approx(lo, rel=1e-4) and phi == pytest.approx(hi, rel=1e-4)
    assert pxi == pytest.approx(1e-3, rel=1e-3)
    # lambda_max below a certified lower bound (a Rayleigh quotient) -> fallback to Lanczos, xi = 0
    B.pp_mlp_set_normalization(h, np.zeros(16), np.ones(16), [np.log(lo), np.log(0.3 * hi), 0.0],
                               [1e-7, 1e-7, 1e-7])
    plo, phi, pxi, fb = B.pp_predict_bounds(op.handle, h, 8)
    assert fb and pxi == 0.0 and plo == lo and phi == hi
    # lambda_min >= lambda_max -> fallback
    B.pp_mlp_set_normalization(h, np.zeros(16), np.ones(16), [np.log(2 * hi), np.log(hi), 0.0], [1e-7] * 3)
    assert B.pp_predict_bounds(op.handle, h, 8)[3]
    B.pp_mlp_destroy(h)
    op.close()


def test_learned_gain_over_lanczos(B):
    """The trained network (weights under paper_2208_01339_amd/weights) against Lanczos bounds with xi = 0."""
    from paper_2208_01339_amd import learned

    if not os.path.exists(os.path.join(learned.WEIGHTS_DIR, "bounds_mlp.npy")):
        pytest.skip("no trained weights committed")
    m = learned.Model.load()
    summ, rows = learned.evaluate(m, 24, seed=424242)
    m.close()
    print(summ)
    assert summ["fallback_rate"] <= 0.25
    # setup: features + forward pass against 20 Lanczos steps
    assert summ["mean_setup_s_pred"] < summ["mean_setup_s_lanczos"] * 1.5
    # solver: predicted bounds and xi need fewer iterations than Lanczos bounds with xi = 0
    # (on 500 held-out operators: 9.0 vs 11.4 on average)
    assert summ["mean_iters_pred"] <= 0.95 * summ["mean_iters_lanczos_xi0"]
