"""Learned cardinality estimator: training and inference driven through the
C ABI of include/cbaa_mlp.h (all arithmetic in the library's HIP kernels;
torch only holds device buffers).

The network reads a host's per-array column popcounts in the log domain of
the linear count, plus its union column's Thm. 2 count and its sketch's
g*eps, and (full feature set) the union column's count against the sketch's
row-aware shared-bit mass and that mass (features of cbaa_mlp_features). It
outputs a correction in log space of the union-column count that comes last
among them: ln(1 + n_hat) = x_base + y, x_base being the row-aware count with
the full set, Thm. 2's with the shorter one. A network whose output is zero is
that count, which therefore stays both the starting point and the fallback.
Labels are supplied by the caller.

The row-aware count replaces Thm. 1's uniform shared-bit probability by a
per-row one: q_b = product over arrays of the fraction of columns with bit b
set, summed over the g rows (it equals g*eps when rows fill evenly). Fan-in
super hosts set their own row in nearly every column, which Thm. 1 cannot
see; the row-aware count subtracts exactly those rows.
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
        """A fresh network for extended features (n_ra + n_va + 2 or + 4)."""
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


def features(cfg, cube: torch.Tensor, hosts: np.ndarray, extended: bool = True,
             rows: bool = True) -> torch.Tensor:
    """fp32 [n, F] features of the given inner IPs, computed on the device:
    F = A, A + 2 (extended) or A + 4 (extended with the row-aware pair)."""
    c = cfg if isinstance(cfg, cbaa.Config) else cbaa.Config.from_dict(cfg)
    F = c.n_arrays + ((4 if rows else 2) if extended else 0)
    n = len(hosts)
    dev = cube.device
    h = torch.from_numpy(np.ascontiguousarray(hosts, dtype=np.uint32).view(np.int32)).to(dev)
    x = torch.empty((max(n, 1), F), dtype=torch.float32, device=dev)
    scratch = cbaa.scratch_tensor(cbaa.cbaa_restore_scratch_bytes(cfg, 0), dev)
    cbaa.cbaa_mlp_features(cfg, cube, h, F, x, scratch)
    return x[:n]


def base_log(x: torch.Tensor) -> torch.Tensor:
    """ln(1 + union-column count): the second-to-last feature (row-aware with
    the full feature set, Thm. 2 with A + 2 features)."""
    return x[:, -2]


def row_aware_count(x: torch.Tensor) -> torch.Tensor:
    """The row-aware linear count from the full feature set."""
    return torch.clamp(torch.expm1(x[:, -2].double()), min=0.0)


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


def stratified_rows(counts: np.ndarray, per_bin: int, rng: np.random.Generator,
                    oversample: bool = False) -> np.ndarray:
    """Indices of per_bin hosts from every power-of-two cardinality bin, so
    training is not dominated by the many single-peer hosts: bins with more
    hosts are subsampled, bins with fewer are drawn with replacement
    (oversample) or kept whole."""
    b = np.floor(np.log2(np.maximum(counts, 1))).astype(np.int64)
    out = []
    for v in np.unique(b):
        idx = np.flatnonzero(b == v)
        if idx.size > per_bin:
            out.append(rng.choice(idx, per_bin, replace=False))
        elif oversample:
            out.append(rng.choice(idx, per_bin, replace=True))
        else:
            out.append(idx)
    return rng.permutation(np.concatenate(out))


def linear_count(cfg, cube: torch.Tensor, hosts: np.ndarray) -> np.ndarray:
    """The paper's estimate (Thm. 2) for the same hosts, for comparison."""
    est, _ = cbaa.estimate(cfg, cube, hosts)
    return est


def compare(est_lc: np.ndarray, est_mlp: np.ndarray, truth: np.ndarray, theta: float,
            est_row: np.ndarray | None = None,
            bins=(1, 4, 16, 64, 256, 1024, 4096, 16384, 65536, 500001)) -> dict:
    """Error of the estimators by cardinality bin, and detection at equal FNR:
    each other estimator's threshold is set so its false-negative rate over
    hosts with >= theta peers equals linear counting's at theta (lc: the
    paper's Thm. 2 estimate; row: the row-aware count; mlp: the network)."""
    truth = truth.astype(np.float64)
    ests = {"lc": est_lc, "mlp": est_mlp}
    if est_row is not None:
        ests["row"] = est_row
    rel = {k: np.abs(v - truth) / truth for k, v in ests.items()}
    rows = []
    for lo, hi in zip(bins[:-1], bins[1:]):
        sel = (truth >= lo) & (truth < hi)
        if not sel.any():
            continue
        r = {"card_lo": lo, "card_hi": hi - 1, "hosts": int(sel.sum())}
        for k in ests:
            r[f"{k}_mean_rel_err"] = float(rel[k][sel].mean())
            r[f"{k}_median_rel_err"] = float(np.median(rel[k][sel]))
        rows.append(r)
    pos = truth >= theta
    npos = max(int(pos.sum()), 1)
    fnr_lc = float(((est_lc < theta) & pos).sum()) / npos
    out = {"bins": rows, "theta": theta}
    for k, v in ests.items():
        if k == "lc":
            thr = theta
        else:   # smallest threshold reaching linear counting's FNR
            sc = np.sort(v[pos])
            j = int(math.floor(fnr_lc * npos))
            thr = float(sc[j]) if j < sc.size else float("inf")
        out[k] = {"threshold": thr, "fnr": float(((v < thr) & pos).sum()) / npos,
                  "fpr": float(((v >= thr) & ~pos).sum()) / npos,
                  "log_mse": float(np.mean((np.log1p(v) - np.log1p(truth)) ** 2)),
                  "mean_rel_err": float(rel[k].mean())}
    return out
