"""Parameters of the learned initial-normal MLP (48 -> 128 -> 128 -> 3): initialisation,
save / load (safetensors, no pickle). The arithmetic is in csrc/dwg_mlp.hip."""
from __future__ import annotations

import math

import numpy as np
import torch

IN, HID, OUT = 48, 128, 3
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)),
          ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, as one float32 blob in ABI order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in SHAPES:
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp) * math.sqrt(2.0 / shp[1]))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def save_params(path: str, blob, meta: dict | None = None) -> None:
    from safetensors.numpy import save_file
    blob = np.asarray(blob, np.float32)
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = blob[o:o + k].reshape(shp).copy()
        o += k
    save_file(out, path, metadata={k: str(v) for k, v in (meta or {}).items()})


def load_params(path: str, device=None) -> torch.Tensor:
    from safetensors.numpy import load_file
    d = load_file(path)
    blob = np.concatenate([np.asarray(d[name], np.float32).ravel() for name, _ in SHAPES])
    assert blob.size == N_PARAMS
    t = torch.from_numpy(blob)
    return t.to(device) if device is not None else t
