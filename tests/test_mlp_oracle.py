"""Pins of the learned estimator's CPU oracle (oracle/mlp.py): bfloat16
rounding against hand-worked values and torch's conversion, the gradient
against central finite differences, Adam against torch.optim.Adam."""

import numpy as np
import pytest

from oracle import mlp as M


def test_param_count_and_layout():
    for F in (1, 4, 6, 8):
        assert M.n_params(F) == 64 * F + 64 + 64 * 64 + 64 + 64 + 1
        theta = np.arange(M.n_params(F), dtype=np.float64)
        W1, b1, W2, b2, w3, b3 = M.split(theta, F)
        assert W1.shape == (64, F) and W2.shape == (64, 64) and b3.shape == (1,)
        assert M.weight_mask(F).sum() == 64 * F + 64 * 64 + 64


def test_bf16_rounding_hand_values():
    # spacing at 1.0 is 2^-7; exact halves go to the even mantissa
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 0.0],
                    np.float32)
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 0.0], np.float32)
    assert np.array_equal(M.to_bf16(vals), want)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    t = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.to_bf16(x), t)


@pytest.mark.parametrize("F", [4, 6])
def test_gradient_matches_finite_differences(F):
    rng = np.random.default_rng(F)
    theta = rng.standard_normal(M.n_params(F)) * 0.3
    x = rng.uniform(0, 1, (40, F))
    t = rng.uniform(0, 8, 40)
    loss, g = M.loss_and_grad(theta, F, x, t, act_bf16=False)
    idx = rng.choice(M.n_params(F), 120, replace=False)
    fd = M.finite_difference_grad(theta, F, x, t, idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-8)
    assert loss > 0


def test_bf16_activations_of_the_second_layer():
    """The device's definition of layer 2's inputs: z1 in fp32 (bias, then the
    products in input order) agrees with fp64 to fp32 rounding; h1 enters z2
    rounded to bf16, shown on a hand-built network whose output is h1[0]
    itself: x = 1 + 2^-8 + 2^-10 gives z1 = x exactly in fp32, which rounds to
    the bf16 value 1 + 2^-7; and the bf16-mode gradient stays within the
    rounding of h1 of the fp64 network's."""
    F = 1
    theta = np.zeros(M.n_params(F))
    W1, b1, W2, b2, w3, b3 = M.split(theta, F)   # views into theta
    W1[:] = 1.0
    W2[0, 0] = 1.0
    w3[0] = 1.0
    x = np.array([[1 + 2 ** -8 + 2 ** -10]], np.float32)
    y_bf, _ = M.forward(theta, F, x)
    y_ex, _ = M.forward(theta, F, x, act_bf16=False)
    assert y_bf[0] == 1 + 2 ** -7
    assert y_ex[0] == 1 + 2 ** -8 + 2 ** -10
    rng = np.random.default_rng(9)
    F = 6
    theta = M.compute_params(rng.standard_normal(M.n_params(F)).astype(np.float32) * 0.3, F)
    x = rng.uniform(0, 1, (300, F)).astype(np.float32)
    z32 = M.layer1_fp32(theta, F, x).astype(np.float64)
    W1, b1 = (a.astype(np.float64) for a in M.split(theta, F)[:2])
    z64 = x.astype(np.float64) @ W1.T + b1
    assert np.max(np.abs(z32 - z64)) <= 1e-6 * (np.max(np.abs(z64)) + 1)
    t = rng.uniform(0, 8, 300)
    _, g_bf = M.loss_and_grad(theta, F, x, t)
    _, g_ex = M.loss_and_grad(theta, F, x, t, act_bf16=False)
    assert np.max(np.abs(g_bf - g_ex)) <= 2 ** -7 * 4 * np.max(np.abs(g_ex))
    assert not np.array_equal(g_bf, g_ex)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    P = 500
    w = rng.standard_normal(P)
    m = np.zeros(P)
    v = np.zeros(P)
    p = torch.nn.Parameter(torch.from_numpy(w.copy()))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 4):
        g = rng.standard_normal(P)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        w, m, v = M.adam_step(w, g, m, v, step, 1e-2)
        assert np.allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_features_hand_values():
    """Feature values worked by hand at g = 4096 (each is ln(1 + g u) with u
    the log ratio of the column's zeros to its no-sharing expectation):
    z = g gives u = 0; z = g/2 gives u = ln 2, so ln(1 + 4096 ln 2) =
    7.951605...; z = g/4 gives ln(1 + 4096 ln 4) = 8.644576...; z = 0 is read
    as one zero, ln(1 + 4096 ln 4096) = 10.436189.... The union column's count
    divides by g - g eps (Thm. 2): with eps = 1/4, Z = 3072 is exactly the
    expected shared fill (u = 0), Z = 1536 gives ln 2 again, and Z above
    g - g eps is clamped to 0 rather than going negative; g eps = 1024. The
    row-aware pair divides by g - shared instead."""
    layer = np.array([[4096, 2048, 1024, 0]] * 3, np.uint16)
    union = np.array([3072, 1536, 4096], np.uint16)
    eps = np.full(3, 0.25)
    shared = np.array([1024.0, 2048.0, 0.0])
    x = M.features(layer, union, eps, 4096, extended=True, shared=shared)
    assert x.dtype == np.float32 and x.shape == (3, 8)
    per = np.array([0.0, 7.951605404591579, 8.64457652142652, 10.436189247200675], np.float32)
    for k in range(3):
        assert np.allclose(x[k, :4], per, rtol=1e-6, atol=0)
    assert np.allclose(x[:, 4], [0.0, 7.951605404591579, 0.0], rtol=1e-6, atol=0)
    assert np.all(x[:, 5] == 1024.0)
    # row-aware: Z = 3072 against g - 1024 = 3072 -> 0; Z = 1536 against
    # g - 2048 = 2048 -> ln(1 + 4096 ln(4/3)); Z = 4096 against g -> 0
    assert np.allclose(x[:, 6], [0.0, np.log1p(4096 * np.log(4 / 3)), 0.0], rtol=1e-6, atol=0)
    assert np.array_equal(x[:, 7], shared.astype(np.float32))
    base = M.features(layer, union, eps, 4096, extended=False)
    assert base.shape == (3, 4) and np.array_equal(base, x[:, :4])
