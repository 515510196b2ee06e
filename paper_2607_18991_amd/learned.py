"""Learned prefill: a small MLP predicts, for a lattice (zone mask, L), the mean
and the spread of n*/N; each sample then starts its Newman-Ziff sweep (Sec. II.B)
from a bulk state with n0 = (mean - k std) N sites already occupied and
labelled (k = 3 unless a tuned batch says otherwise).  The prediction only moves work between the bulk and the sequential
phase: a sample whose bulk state already spans backs off, so n* and the mass
never depend on it.

Every arithmetic step of training and inference runs in the MLP kernels of
libnz (forward, loss, backward, Adam); PyTorch holds the device buffers.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import nz

IN, H, OUT = 8, 64, 2
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prefill_mlp.json")


def zone_bits(mask: int) -> list[float]:
    return [float((mask >> k) & 1) for k in range(7)]


def to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even (host copy of the
    rounding the Adam kernel applies on the device)."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases; float32 flat vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((IN, H), (H, H), (H, OUT)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == nz.NZ_MLP_NPARAM
    return flat


# The size input is the finite-size-scaling variable L^(-1/nu), standardised
# over the training set; the library forms it (nz_mlp_features).
NU5 = 0.5720


class PrefillModel:
    def __init__(self, params: np.ndarray, size_mean: float, size_std: float, meta: dict | None = None):
        self.params = np.asarray(params, dtype=np.float32)
        self.size_mean = float(size_mean)
        self.size_std = float(size_std)
        self.meta = meta or {}

    @property
    def params(self) -> np.ndarray:
        return self._params

    @params.setter
    def params(self, value) -> None:
        self._params = np.asarray(value, dtype=np.float32)
        self._dev_params = {}   # device -> these weights in bf16 on it, uploaded at the first prediction

    # ---------------------------------------------------------------- io
    def save(self, path: str = DEFAULT_PATH) -> None:
        with open(path, "w") as f:
            json.dump({"size_feature": "L^(-1/nu)", "nu": NU5, "size_mean": self.size_mean,
                       "size_std": self.size_std, "meta": self.meta,
                       "params_fp32": [float(v) for v in self.params]}, f)

    @classmethod
    def load(cls, path: str = DEFAULT_PATH) -> "PrefillModel":
        with open(path) as f:
            d = json.load(f)
        return cls(np.array(d["params_fp32"], dtype=np.float32), d["size_mean"], d["size_std"], d.get("meta"))

    # ---------------------------------------------------------------- inference
    def features(self, masks, Ls) -> np.ndarray:
        return nz.nz_mlp_features(masks, Ls, self.size_mean, self.size_std)

    def forward(self, masks, Ls, stream=None) -> np.ndarray:
        """The MLP's outputs (ln mean, ln std of n*/N) per (mask, L), via the
        forward kernel."""
        import torch

        x = torch.from_numpy(self.features(masks, Ls)).cuda()
        dev = torch.cuda.current_device()
        pb = self._dev_params.get(dev)
        if pb is None:
            pb = torch.from_numpy(to_bf16_bits(self.params).view(np.int16)).cuda()
            self._dev_params[dev] = pb
        B = x.shape[0]
        y = torch.empty((B, OUT), dtype=torch.float32, device="cuda")
        act = torch.empty((B, nz.NZ_MLP_NACT), dtype=torch.float32, device="cuda")
        nz.nz_mlp_forward(pb, x, y, act, stream=stream)
        return y.cpu().numpy()

    def predict(self, masks, Ls, stream=None):
        """Predicted (mean, std) of n*/N per (mask, L)."""
        out = self.forward(masks, Ls, stream).astype(np.float64)
        return np.exp(out[:, 0]), np.exp(out[:, 1])

    def plan(self, jobs, k_sigma: float = 3.0, band_sigma: float = 5.0, k_sigma_wide: float | None = None,
             split_z: int | None = None):
        """Copies of the job dicts with the learned n0, backoff step and band
        (nz_prefill_plan).  k_sigma_wide: the prefill depth of the jobs wider
        than split_z (the second group when a batch runs as two groups)."""
        y = self.forward([j["zone_mask"] for j in jobs], [j["L"] for j in jobs])
        return plan_outputs(y, jobs, k_sigma, band_sigma, k_sigma_wide, split_z)


# widest neighbourhood of the first group when the library splits a batch and
# no split is given (nz_tuning.split_z = 0)
SPLIT_Z_DEFAULT = 64


def plan_outputs(y, jobs, k_sigma: float, band_sigma: float = 5.0, k_sigma_wide: float | None = None,
                 split_z: int | None = None):
    """nz_prefill_plan of the MLP outputs y (one row per job), with prefill
    depth k_sigma_wide for the jobs whose coordination number exceeds split_z
    when it is given."""
    if k_sigma_wide is None:
        return nz.nz_prefill_plan(y, jobs, k_sigma, band_sigma)
    sz = int(split_z) if split_z else SPLIT_Z_DEFAULT
    yy = np.asarray(y, dtype=np.float32).reshape(-1, OUT)
    wide = [nz.nz_coordination(int(j["zone_mask"])) > sz for j in jobs]
    out = [None] * len(jobs)
    for flag, k in ((False, k_sigma), (True, k_sigma_wide)):
        idx = [i for i, w in enumerate(wide) if w == flag]
        if idx:
            for i, p in zip(idx, nz.nz_prefill_plan(yy[idx], [jobs[i] for i in idx], k, band_sigma)):
                out[i] = p
    return out


def plan_band_only(model: PrefillModel, jobs, band_sigma: float = 5.0):
    """Plain sweeps (no prefill) with the learned band size, so that plain and
    learned runs differ only in the prefill."""
    y = model.forward([j["zone_mask"] for j in jobs], [j["L"] for j in jobs])
    return nz.nz_prefill_plan(y, jobs, 0.0, band_sigma, plain=True)


def aggregate(L: int, mask: int, nstar: np.ndarray) -> dict:
    """Training target of one lattice: mean and std of n*/N over the samples
    that span (nz_prefill_target)."""
    count, mean, sd, ln_mean, ln_sd = nz.nz_prefill_target(nstar, L)
    return {"L": L, "mask": mask, "count": count, "mean": mean, "std": sd, "ln_mean": ln_mean, "ln_std": ln_sd}


def train(points, steps: int = 3000, lr: float = 3e-3, seed: int = 0, log_every: int = 0,
          wd: float = 0.0) -> PrefillModel:
    """Fit the MLP to aggregates [{'L','mask','count','ln_mean','ln_std'}] with the
    device kernels: forward, weighted squared error, backward, Adam."""
    import torch

    Ls = np.array([p["L"] for p in points], dtype=np.int32)
    w = np.array([p["count"] for p in points], dtype=np.float64)
    s_mean, s_std = nz.nz_mlp_size_stats(Ls)
    model = PrefillModel(init_params(seed), s_mean, s_std)
    x = torch.from_numpy(model.features([p["mask"] for p in points], [p["L"] for p in points])).cuda()
    tgt = torch.from_numpy(np.array([[p["ln_mean"], p["ln_std"]] for p in points],
                                    dtype=np.float32)).cuda()
    # every lattice counts, with a mild preference for the better-sampled ones
    wt = torch.from_numpy(np.sqrt(w).astype(np.float32)).cuda()
    B = x.shape[0]
    w32 = torch.from_numpy(model.params.copy()).cuda()
    wb = torch.from_numpy(to_bf16_bits(model.params).view(np.int16)).cuda()
    m = torch.zeros_like(w32)
    v = torch.zeros_like(w32)
    g = torch.zeros_like(w32)
    y = torch.empty((B, OUT), dtype=torch.float32, device="cuda")
    act = torch.empty((B, nz.NZ_MLP_NACT), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hyper = [lr, 0.9, 0.999, 1e-8, wd]
    history = []
    for step in range(1, steps + 1):
        nz.nz_mlp_forward(wb, x, y, act)
        nz.nz_mlp_loss(y, tgt, wt, dy, loss)
        nz.nz_mlp_backward(wb, x, act, dy, g)
        nz.nz_mlp_adam(w32, wb, g, m, v, hyper, step)
        if step == 1 or step == steps or (log_every and step % log_every == 0):
            history.append((step, float(loss.item())))
    model.params = w32.cpu().numpy()
    model.meta = {"steps": steps, "lr": lr, "seed": seed, "loss_history": history,
                  "points": len(points), "L_values": sorted(set(int(L) for L in Ls))}
    return model
