"""Learned estimator on the GPU: kernels against the fp64 oracle
(oracle/mlp.py), features against the CBAA oracle, and a trained network
against the paper's linear count on a held-out window.

Tolerances: forward outputs and the loss within 1e-5 relative, gradients
within 1e-4 of the largest gradient entry (fp32 accumulation in a different
order than the oracle's fp64 sums, same bf16-rounded weights on both
sides); Adam's master within 1e-6 relative plus 1e-9; the bf16 copy is
exactly the round-to-nearest-even of the device master."""

import json

import numpy as np
import pytest

import oracle as O
import tracegen
from conftest import default_params
from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06207_amd import cbaa
    cbaa.lib()
    return cbaa


def _model(cb, F, seed):
    """A network with every layer random (the output layer too)."""
    import torch
    from paper_1901_06207_amd import learned
    P = cb.cbaa_mlp_param_count(F)
    m = learned.Model(F, torch.empty(P, dtype=torch.float32, device="cuda"),
                      torch.empty(P, dtype=torch.int16, device="cuda"))
    cb.cbaa_mlp_init(F, seed, m.master, m.wbf)
    return m


def _np(t):
    return t.detach().cpu().numpy()


def _bf16_bits_to_f32(bits):
    return (bits.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("F", [4, 6])
def test_init_and_bf16_copy(cb, F):
    m = _model(cb, F, 7)
    master = _np(m.master)
    wbf = _bf16_bits_to_f32(_np(m.wbf).view(np.uint16))
    mask = M.weight_mask(F)
    assert np.all(master[~mask] == 0)
    assert np.all(np.abs(master[mask][: 64 * F]) <= np.sqrt(6 / F))
    assert np.array_equal(wbf[mask], M.to_bf16(master[mask]))
    assert np.std(master[mask][: 64 * F]) > 0.1


def test_zero_output_init_is_the_linear_count(cb):
    import torch
    from paper_1901_06207_amd import learned
    m = learned.Model.new(6, seed=5)
    x = torch.rand(1000, 6, device="cuda") * 8
    assert torch.equal(learned.predict_log(m, x), learned.base_log(x))


@pytest.mark.parametrize("F,n", [(4, 1), (4, 1000), (6, 4097), (8, 200003)])
def test_forward_matches_oracle(cb, F, n):
    import torch
    m = _model(cb, F, 11)
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 1, (n, F)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    cb.cbaa_mlp_forward(F, m.master, m.wbf, xt, y)
    want, _ = M.forward(M.compute_params(_np(m.master), F), F, x)
    assert np.allclose(_np(y), want, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("F,n", [(4, 64), (6, 1000), (6, 65536), (8, 100001)])
def test_loss_and_gradient_match_oracle(cb, F, n):
    import torch
    m = _model(cb, F, 13)
    rng = np.random.default_rng(F + n)
    x = rng.uniform(0, 1, (n, F)).astype(np.float32)
    t = rng.uniform(0, 12, n).astype(np.float32)
    P = cb.cbaa_mlp_param_count(F)
    grad = torch.empty(P, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    cb.cbaa_mlp_loss_grad(F, m.master, m.wbf, torch.from_numpy(x).cuda(),
                          torch.from_numpy(t).cuda(), grad, loss)
    wl, wg = M.loss_and_grad(M.compute_params(_np(m.master), F), F, x, t)
    assert abs(float(_np(loss)[0]) - wl) <= 1e-5 * abs(wl)
    g = _np(grad)
    assert np.max(np.abs(g - wg)) <= 1e-4 * np.max(np.abs(wg)) + 1e-7


def test_adam_step_matches_oracle(cb):
    import torch
    F = 6
    m = _model(cb, F, 17)
    P = cb.cbaa_mlp_param_count(F)
    rng = np.random.default_rng(5)
    mom = torch.zeros(P, dtype=torch.float32, device="cuda")
    vel = torch.zeros(P, dtype=torch.float32, device="cuda")
    w = _np(m.master).astype(np.float64)
    mm = np.zeros(P)
    vv = np.zeros(P)
    for step in range(1, 4):
        g = rng.standard_normal(P).astype(np.float32)
        cb.cbaa_mlp_adam(F, m.master, m.wbf, torch.from_numpy(g).cuda(), mom, vel, step, 1e-3)
        w, mm, vv = M.adam_step(w, g, mm, vv, step, 1e-3)
        got = _np(m.master)
        assert np.allclose(got, w, rtol=1e-6, atol=1e-9)
        w = got.astype(np.float64)   # follow the device's fp32 state
    bits = _bf16_bits_to_f32(_np(m.wbf).view(np.uint16))
    assert np.array_equal(bits, M.to_bf16(_np(m.master)))


@pytest.mark.parametrize("rows", [False, True])
def test_features_match_oracle(cb, rows):
    from paper_1901_06207_amd import learned
    p = default_params()
    t = tracegen.window_core_edge(6, scale=1 / 32)    # fan-in hosts: uneven rows
    cube = cb.new_cube(p)
    cb.cbaa_update(p, cube, cb.pairs_to_device(t.pairs), 0)
    hosts = np.concatenate([t.planted_ips, t.bg_ips[:3000]])
    x = _np(learned.features(p, cube, hosts, extended=True, rows=rows))
    cube_np = O.cube_of(p, t.pairs, 0)
    g = 1 << p["log2_g"]
    lz = O.host_layer_zeros(p, cube_np, hosts)
    _, uz, _ = O.estimate(p, cube_np, hosts)
    _, ones = O.column_zeros(p, cube_np)
    eps, _ = O.thresholds(p, ones, 1024.0)
    cs = np.array([O.host_columns(p, int(h))[0] for h in hosts])
    shared = O.row_shared(p, O.row_ones(p, cube_np)) if rows else None
    want = M.features(lz, uz, eps[cs], g, extended=True,
                      shared=shared[cs] if rows else None)
    assert x.shape == want.shape
    # device log vs libm log, a parallel sum of the row mass, rounding to fp32
    assert np.allclose(x, want, rtol=2e-6, atol=1e-6)
    if rows:
        assert shared.min() > 0.0


def _window_rows(cb, learned, p, seed, scale, side, per_bin, rng):
    """Features and construction truth for hosts of one window and side, up to
    per_bin hosts from each power-of-two cardinality bin (per_bin None: a
    uniform sample of 1M hosts, the natural mix)."""
    import torch
    print(f"[case] learned window seed={seed} scale={scale} side={side}", flush=True)
    t = tracegen.window_core_edge(seed, scale=scale)
    a, b = cb.new_cube(p), cb.new_cube(p)
    cb.cbaa_update2(p, a, b, cb.pairs_to_device(t.pairs))
    cube = a if side == 0 else b
    hosts, counts = tracegen.construction_truth(t, side)
    if per_bin is None:
        sel = rng.choice(hosts.size, min(hosts.size, 1_000_000), replace=False)
    else:
        sel = learned.stratified_rows(counts, per_bin, rng)
    x = learned.features(p, cube, hosts[sel], extended=True)
    torch.cuda.synchronize()
    return cube, hosts[sel], counts[sel], x


def test_trained_network_against_linear_count(cb):
    """Trains on core-edge windows (both sides) and compares with the paper's
    Thm. 2 estimate and the row-aware count on a held-out window at equal
    false-negative rate. The network must lower the log-scale error overall
    and the mean relative error below 64 peers, where rows set by fan-in
    hosts bias the linear count upwards."""
    import torch
    from paper_1901_06207_amd import learned
    p = default_params()
    rng = np.random.default_rng(0)
    xs, ts = [], []
    for seed, side in ((21, 0), (21, 1), (22, 0), (22, 1), (24, 0), (25, 0)):
        _, _, c, x = _window_rows(cb, learned, p, seed, 0.5, side, 100_000, rng)
        xs.append(x)
        ts.append(torch.from_numpy(np.log1p(c).astype(np.float32)).cuda())
    X = torch.cat(xs)
    T = torch.cat(ts)
    model = learned.Model.new(X.shape[1], seed=3)
    log = learned.train(model, X, T, epochs=20, batch=16384)
    cube, hosts, counts, xe = _window_rows(cb, learned, p, 23, 0.5, 0, None, rng)
    est_ml = learned.predict(model, xe).cpu().numpy()
    est_lc = learned.linear_count(p, cube, hosts)
    est_row = learned.row_aware_count(xe).cpu().numpy()
    rep = learned.compare(est_lc, est_ml, counts, 1024.0, est_row=est_row)
    rep["train"] = {"rows": int(X.shape[0]), "epochs": log.epochs, "steps": log.steps,
                    "loss_by_epoch": log.losses}
    print(json.dumps({k: v for k, v in rep.items() if k != "bins"}), flush=True)
    for row in rep["bins"]:
        print(row, flush=True)
    assert log.losses[-1] < log.losses[0]
    assert rep["mlp"]["log_mse"] < rep["lc"]["log_mse"]
    assert rep["row"]["log_mse"] < rep["lc"]["log_mse"]
    small = [r for r in rep["bins"] if r["card_hi"] < 64]
    assert sum(r["mlp_mean_rel_err"] * r["hosts"] for r in small) < \
        sum(r["lc_mean_rel_err"] * r["hosts"] for r in small)
    assert abs(rep["mlp"]["fnr"] - rep["lc"]["fnr"]) <= 2.0 / max(1, int((counts >= 1024).sum()))
