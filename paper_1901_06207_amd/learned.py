"""Learned cardinality estimator: training and inference driven through the
C ABI of include/cbaa_mlp.h (all arithmetic in the library's HIP kernels;
torch only holds device buffers).

The network reads a host's per-array column popcounts in the log domain of
the linear count, plus its union column's Thm. 2 count and its sketch's
g*eps (features of cbaa_mlp_features), and outputs a correction in log space
of the paper's estimate: ln(1 + n_hat) = x_uc + y, where x_uc = ln(1 + Thm. 2
estimate) is the union-column feature. A network whose output is zero is the
paper's estimator, which therefore stays both the starting point and the
fallback. Labels are supplied by the caller.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import cbaa


@dataclasses.dataclass
class Model:
    n_features: int
    master: torch.Tensor   # fp32 [P]
    wbf: torch.Tensor      # bf16 bits [P] (int16 storage)

    @classmethod
    def new(cls, n_features: int, seed: int = 1, device="cuda") -> "Model":
        """A fresh network for the extended features (n_ra + n_va + 2)."""
        P = cbaa.cbaa_mlp_param_count(n_features)
        if P == 0 or n_features < 3:
            raise ValueError("3 <= n_features <= 8 (extended features)")
        m = cls(n_features, torch.empty(P, dtype=torch.float32, device=device),
                torch.empty(P, dtype=torch.int16, device=device))
        # zero output layer: an untrained network is exactly the linear count
        cbaa.cbaa_mlp_init(n_features, seed, m.master, m.wbf, zero_output=True)
        return m

    def state(self) -> dict:
        return {"n_features": self.n_features, "master": self.master.cpu().numpy().tolist()}


def features(cfg, cube: torch.Tensor, hosts: np.ndarray, extended: bool = True) -> torch.Tensor:
    """fp32 [n, F] features of the given inner IPs, computed on the device."""
    c = cfg if isinstance(cfg, cbaa.Config) else cbaa.Config.from_dict(cfg)
    F = c.n_arrays + (2 if extended else 0)
    n = len(hosts)
    dev = cube.device
    h = torch.from_numpy(np.ascontiguousarray(hosts, dtype=np.uint32).view(np.int32)).to(dev)
    x = torch.empty((max(n, 1), F), dtype=torch.float32, device=dev)
    scratch = cbaa.scratch_tensor(cbaa.cbaa_restore_scratch_bytes(cfg, 0), dev)
    cbaa.cbaa_mlp_features(cfg, cube, h, F, x, scratch)
    return x[:n]


def base_log(x: torch.Tensor) -> torch.Tensor:
    """ln(1 + Thm. 2 estimate): the union-column feature (second to last)."""
    return x[:, -2]


def predict_log(model: Model, x: torch.Tensor) -> torch.Tensor:
    """ln(1 + n_hat): the linear count's log plus the network's correction."""
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    cbaa.cbaa_mlp_forward(model.n_features, model.master, model.wbf, x.contiguous(), y)
    return base_log(x) + y


def predict(model: Model, x: torch.Tensor) -> torch.Tensor:
    """Cardinality estimates exp(y) - 1, clamped at 0."""
    return torch.clamp(torch.expm1(predict_log(model, x).double()), min=0.0)


@dataclasses.dataclass
class TrainLog:
    steps: int
    epochs: int
    final_loss: float
    losses: list


def train(model: Model, x: torch.Tensor, target_log: torch.Tensor, epochs: int = 20,
          batch: int = 65536, lr: float = 2e-3, lr_final: float = 1e-4, seed: int = 0) -> TrainLog:
    """Adam on mean (y - (t - x_uc))^2 / 2, i.e. the log-space error of the
    corrected estimate, with a cosine learning-rate decay; minibatches drawn
    by a seeded permutation each epoch. target_log = ln(1 + n)."""
    dev = x.device
    target_log = (target_log - base_log(x)).contiguous()
    n = x.shape[0]
    P = model.master.numel()
    grad = torch.empty(P, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros(P, dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = max(1, math.ceil(n / batch))
    total = epochs * steps_per_epoch
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        xs = x[perm].contiguous()
        ts = target_log[perm].contiguous()
        ep_loss = torch.zeros(1, dtype=torch.float32, device=dev)
        for b0 in range(0, n, batch):
            step += 1
            xb, tb = xs[b0:b0 + batch], ts[b0:b0 + batch]
            cbaa.cbaa_mlp_loss_grad(model.n_features, model.master, model.wbf, xb, tb, grad, loss)
            frac = (step - 1) / max(total - 1, 1)
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
            cbaa.cbaa_mlp_adam(model.n_features, model.master, model.wbf, grad, m, v, step, cur)
            ep_loss += loss * (xb.shape[0] / n)
        losses.append(float(ep_loss.item()))
    return TrainLog(steps=step, epochs=epochs, final_loss=losses[-1], losses=losses)


def stratified_rows(counts: np.ndarray, per_bin: int, rng: np.random.Generator) -> np.ndarray:
    """Indices of up to per_bin hosts from every power-of-two cardinality bin,
    so training is not dominated by the many single-peer hosts."""
    b = np.floor(np.log2(np.maximum(counts, 1))).astype(np.int64)
    out = []
    for v in np.unique(b):
        idx = np.flatnonzero(b == v)
        out.append(idx if idx.size <= per_bin else rng.choice(idx, per_bin, replace=False))
    return rng.permutation(np.concatenate(out))


def linear_count(cfg, cube: torch.Tensor, hosts: np.ndarray) -> np.ndarray:
    """The paper's estimate (Thm. 2) for the same hosts, for comparison."""
    est, _ = cbaa.estimate(cfg, cube, hosts)
    return est


def compare(est_lc: np.ndarray, est_mlp: np.ndarray, truth: np.ndarray, theta: float,
            bins=(1, 4, 16, 64, 256, 1024, 4096, 16384, 65536, 500001)) -> dict:
    """Error of both estimators by cardinality bin, and detection at equal FNR:
    the learned estimator's threshold is set so its false-negative rate over
    hosts with >= theta peers equals linear counting's at theta."""
    truth = truth.astype(np.float64)
    rel_lc = np.abs(est_lc - truth) / truth
    rel_ml = np.abs(est_mlp - truth) / truth
    rows = []
    for lo, hi in zip(bins[:-1], bins[1:]):
        sel = (truth >= lo) & (truth < hi)
        if not sel.any():
            continue
        rows.append({"card_lo": lo, "card_hi": hi - 1, "hosts": int(sel.sum()),
                     "lc_mean_rel_err": float(rel_lc[sel].mean()),
                     "mlp_mean_rel_err": float(rel_ml[sel].mean()),
                     "lc_median_rel_err": float(np.median(rel_lc[sel])),
                     "mlp_median_rel_err": float(np.median(rel_ml[sel]))})
    pos = truth >= theta
    npos = max(int(pos.sum()), 1)
    fnr_lc = float(((est_lc < theta) & pos).sum()) / npos
    fpr_lc = float(((est_lc >= theta) & ~pos).sum()) / npos
    # smallest threshold on the learned estimate reaching the same FNR
    sc = np.sort(est_mlp[pos])
    k = int(math.floor(fnr_lc * npos))
    thr = float(sc[k]) if k < sc.size else float("inf")
    fnr_ml = float(((est_mlp < thr) & pos).sum()) / npos
    fpr_ml = float(((est_mlp >= thr) & ~pos).sum()) / npos
    log_mse_lc = float(np.mean((np.log1p(est_lc) - np.log1p(truth)) ** 2))
    log_mse_ml = float(np.mean((np.log1p(est_mlp) - np.log1p(truth)) ** 2))
    return {"bins": rows, "theta": theta, "lc": {"fnr": fnr_lc, "fpr": fpr_lc, "log_mse": log_mse_lc,
                                                  "mean_rel_err": float(rel_lc.mean())},
            "mlp": {"threshold": thr, "fnr": fnr_ml, "fpr": fpr_ml, "log_mse": log_mse_ml,
                    "mean_rel_err": float(rel_ml.mean())}}
