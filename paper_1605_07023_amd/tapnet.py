"""Learned tap network (GR_MLP): weights, training loop and kernel descriptor.

The network replaces the oversampled 2-D W-kernel table (the precomputed GCF
of Merry 2016, Section 2.2) by a function of the tap's coordinates
(w_hat, d_u, d_v); the blob layout, inputs and encoding are those of
``gr_mlp_eval`` in include/gridder.h.  Every computation (dataset, forward,
gradients, Adam, evaluation, gridding) runs in libgridder.so; this module
initialises the weights from a seeded host generator, draws the minibatch
indices, watches the loss and keeps checkpoints.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np
import torch

from . import binding as B

HIDDEN = 64
D_IN = 64
N_FEAT = 36
HDR = 4


class TrainingDiverged(RuntimeError):
    """The training loss became NaN or infinite; the run is abandoned."""


def check_loss(value: float, step: int) -> float:
    if not math.isfinite(value):
        raise TrainingDiverged(f"training loss is {value} at step {step}")
    return value


def _offsets() -> dict:
    o = {"W1": HDR}
    o["b1"] = o["W1"] + D_IN * HIDDEN
    o["W2"] = o["b1"] + HIDDEN
    o["b2"] = o["W2"] + HIDDEN * HIDDEN
    o["W3"] = o["b2"] + HIDDEN
    o["b3"] = o["W3"] + HIDDEN * HIDDEN
    o["W4"] = o["b3"] + HIDDEN
    o["b4"] = o["W4"] + HIDDEN * 2
    return o


OFFSETS = _offsets()
SHAPES = {"W1": (D_IN, HIDDEN), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,),
          "W3": (HIDDEN, HIDDEN), "b3": (HIDDEN,), "W4": (HIDDEN, 2), "b4": (2,)}


def params_to_blob(params: dict, n_floats: int, header=(0.0, 0.0, 1.0, 0.0)) -> np.ndarray:
    blob = np.zeros(n_floats, np.float32)
    blob[:HDR] = header
    for k, shp in SHAPES.items():
        a = np.asarray(params[k], np.float64).reshape(shp)
        blob[OFFSETS[k]:OFFSETS[k] + a.size] = a.ravel()
    return blob


def blob_to_params(blob: np.ndarray) -> dict:
    blob = np.asarray(blob, np.float64)
    return {k: blob[OFFSETS[k]:OFFSETS[k] + int(np.prod(shp))].reshape(shp).copy()
            for k, shp in SHAPES.items()}


def init_params(seed: int = 0) -> dict:
    """Weights uniform in +-1/sqrt(fan-in of live inputs), zero biases.  (He
    scaling, 2.45 times larger, trains this network to an about ten times
    larger tap error.)"""
    rng = np.random.default_rng(seed)
    fan = {"W1": N_FEAT, "W2": HIDDEN, "W3": HIDDEN, "W4": HIDDEN}
    p = {}
    for k in ("W1", "W2", "W3", "W4"):
        lim = 1.0 / math.sqrt(fan[k])
        p[k] = rng.uniform(-lim, lim, size=SHAPES[k])
    p["W1"][N_FEAT:] = 0.0
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = np.zeros(SHAPES[k])
    return p


@dataclass
class TrainLog:
    steps: List[int] = field(default_factory=list)
    losses: List[float] = field(default_factory=list)


class TapNet:
    """Device-resident weights blob plus Adam state."""

    def __init__(self, device="cuda:0", seed: int = 0, params: Optional[dict] = None):
        self.device = torch.device(device)
        self.n_floats = B.gr_mlp_blob_floats()
        p = params if params is not None else init_params(seed)
        blob = params_to_blob(p, self.n_floats)
        self.blob = torch.from_numpy(blob).to(self.device)
        self.m = torch.zeros(self.n_floats, dtype=torch.float32, device=self.device)
        self.v = torch.zeros_like(self.m)
        self.grads = torch.zeros_like(self.m)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0
        self.meta: dict = {}

    # --- header -----------------------------------------------------------
    def set_header(self, x0_offset: float, x0_step: float, out_scale: float) -> None:
        h = torch.tensor([x0_offset, x0_step, out_scale, 0.0], dtype=torch.float32)
        self.blob[:HDR].copy_(h.to(self.device))

    def header(self) -> Tuple[float, float, float]:
        h = self.blob[:3].cpu().numpy()
        return float(h[0]), float(h[1]), float(h[2])

    def params(self) -> dict:
        return blob_to_params(self.blob.cpu().numpy())

    # --- training ---------------------------------------------------------
    def train(self, inputs: torch.Tensor, targets: torch.Tensor, steps: int, batch: int = 16384,
              lr: float = 2e-3, lr_final: float = 2e-5, seed: int = 0, log_every: int = 100,
              stream=None) -> TrainLog:
        """Adam on minibatches drawn without replacement (a fresh permutation per
        epoch, seeded); learning rate decays as a cosine from lr to lr_final over
        ``steps``.  The loss is read back every ``log_every`` steps; a non-finite
        loss raises TrainingDiverged.  Continues from self.step (resume)."""
        n = int(targets.shape[0])
        if inputs.shape[0] != n or inputs.shape[1] != 3 or targets.shape[1] != 2:
            raise ValueError("inputs must be [n, 3] and targets [n, 2]")
        if batch < 1 or n < 1:
            raise ValueError("empty training set or batch")
        batch = min(batch, n)
        rng = np.random.default_rng(seed + self.step)
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(self.device)
        pos = 0
        log = TrainLog()
        start = self.step
        for i in range(steps):
            if pos + batch > n:
                perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(self.device)
                pos = 0
            idx = perm[pos:pos + batch]
            pos += batch
            frac = i / max(steps - 1, 1)
            lr_i = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            self.step += 1
            B.gr_mlp_train_step(self.blob, self.m, self.v, self.grads, inputs, targets, idx, batch,
                                self.step, lr_i, self.loss_buf, stream)
            if (i + 1) % log_every == 0 or i == steps - 1:
                val = float(self.loss_buf.item())
                log.steps.append(self.step)
                log.losses.append(check_loss(val, self.step))
        self.meta["trained_steps"] = self.step - start + self.meta.get("trained_steps", 0)
        return log

    def grads_of(self, inputs, targets, idx, batch: int) -> torch.Tensor:
        B.gr_mlp_grads(self.blob, inputs, targets, idx, batch, self.grads, self.loss_buf)
        return self.grads

    def eval(self, inputs: torch.Tensor) -> torch.Tensor:
        out = torch.empty((inputs.shape[0], 2), dtype=torch.float32, device=self.device)
        B.gr_mlp_eval(self.blob, inputs, int(inputs.shape[0]), out)
        return out

    # --- checkpoints --------------------------------------------------------
    def save(self, path: str) -> None:
        """Weights, Adam moments and step as .npz (no pickled objects)."""
        d = os.path.dirname(path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = path + ".tmp.npz"
        np.savez(tmp, blob=self.blob.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.array([self.step], np.int64),
                 meta=np.frombuffer(json.dumps(self.meta).encode(), dtype=np.uint8))
        os.replace(tmp, path)

    @classmethod
    def load(cls, path: str, device="cuda:0") -> "TapNet":
        z = np.load(path, allow_pickle=False)
        net = cls(device=device)
        if z["blob"].size != net.n_floats:
            raise ValueError(f"{path}: blob has {z['blob'].size} floats, the library expects {net.n_floats}")
        net.blob.copy_(torch.from_numpy(z["blob"].astype(np.float32)).to(net.device))
        net.m.copy_(torch.from_numpy(z["m"].astype(np.float32)).to(net.device))
        net.v.copy_(torch.from_numpy(z["v"].astype(np.float32)).to(net.device))
        net.step = int(z["step"][0])
        net.meta = json.loads(bytes(z["meta"]).decode()) if "meta" in z else {}
        return net

    # --- gridding ---------------------------------------------------------
    def kernel(self, support: int, oversample: int, n_planes: int, w_min: float, inv_dw: float) -> B.GrKernel:
        """GR_MLP kernel descriptor (the blob header must map the plane index)."""
        return B.make_kernel(self.blob, support, oversample, n_planes, True, B.GR_F32, w_min, inv_dw,
                             kind=B.GR_MLP)


def dataset_from_table(table: torch.Tensor, support: int, oversample: int, w_hats: np.ndarray,
                       w_hat_range: float, out_scale: float, stream=None):
    """(inputs [n, 3], targets [n, 2]) device tensors for every entry of a complex
    FP32 2-D table [planes][O][O][S][S] (gr_mlp_dataset); w_hats are the plane
    centres, equally spaced."""
    w_hats = np.asarray(w_hats, np.float64)
    P = w_hats.size
    n = P * oversample * oversample * support * support
    dev = table.device
    inputs = torch.empty((n, 3), dtype=torch.float32, device=dev)
    targets = torch.empty((n, 2), dtype=torch.float32, device=dev)
    step = float(w_hats[1] - w_hats[0]) if P > 1 else 0.0
    B.gr_mlp_dataset(table, support, oversample, P, float(w_hats[0]), step, w_hat_range, out_scale,
                     inputs, targets, stream)
    return inputs, targets


def fine_planes(w_min: float, inv_dw: float, n_planes: int, n_fine: int) -> Tuple[float, float]:
    """(w_min, inv_dw) of a grid of n_fine planes whose rounding cells cover exactly
    the interval the n_planes grid covers, [w_min - dw/2, w_min + (n_planes - 1/2) dw),
    so both grids keep the same visibilities."""
    inv_f = inv_dw * n_fine / n_planes
    return w_min - 0.5 / inv_dw + 0.5 / inv_f, inv_f


def header_for_planes(w_min: float, inv_dw: float, w_hat_scale: float, w_hat_range: float) -> Tuple[float, float]:
    """(x0 offset, x0 step) so that x0 = w_hat(plane) / w_hat_range with
    w_hat(plane) = (w_min + plane / inv_dw) * w_hat_scale."""
    return w_min * w_hat_scale / w_hat_range, w_hat_scale / (inv_dw * w_hat_range)
