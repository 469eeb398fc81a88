"""Training of the refinement-order network (all arithmetic in the library's
kernels; torch only holds device memory).

The network scores the vertices of a coarse level by how likely their cell
holds a critical point of the exact classification (inputs, targets and
architecture are defined with ``pcrit_mlp_features`` in ``include/pcrit.h``);
``progressive_timeline(..., params=...)`` refines the regions with the
highest summed scores first.  The paper has no such part: it classifies
every vertex at once, so its previews are not ordered at all.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import binding as B


def init_params(seed: int = 0, device="cuda"):
    """Random initial parameters (FP32, device): weights N(0, 1/fan_in),
    biases 0."""
    import torch
    rng = np.random.default_rng(seed)
    p = np.zeros(B.MLP_PARAMS, np.float32)
    nin, nh = B.MLP_INPUTS, 64
    o = 0
    for fan_in, fan_out in ((nin, nh), (nh, nh), (nh, 1)):
        p[o:o + fan_in * fan_out] = rng.standard_normal(fan_in * fan_out) / np.sqrt(fan_in)
        o += fan_in * fan_out + fan_out
    assert o == B.MLP_PARAMS
    return torch.from_numpy(p).to(device)


@dataclass
class TrainingSet:
    X: "object"        # n x 32 bfloat16 (device)
    y: "object"        # n uint8 (device)
    level: int


def training_set(field, *, ctx: Optional[B.Context] = None,
                 level: Optional[int] = None) -> TrainingSet:
    """Inputs of the vertices of the scoring level of ``field`` (a 3D device
    tensor) and their targets from its level-0 classification."""
    if level is None:
        level = B.mlp_feature_level(field.shape)
    r = B.classify(field, 0, ctx=ctx)
    X = B.mlp_features(field, level, ctx=ctx)
    y = B.mlp_labels(r.codes, level, ctx=ctx)
    return TrainingSet(X, y, level)


def train(params, sets: Sequence[TrainingSet], *, steps: int = 3000, lr: float = 1e-2,
          ctx: Optional[B.Context] = None) -> List[float]:
    """Full-batch Adam on the union of ``sets``; updates ``params`` in place
    and returns the mean loss before every step."""
    import torch
    X = torch.cat([s.X for s in sets]) if len(sets) > 1 else sets[0].X
    y = torch.cat([s.y for s in sets]) if len(sets) > 1 else sets[0].y
    n = X.shape[0]
    grad = torch.empty_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    losses = torch.empty(steps, dtype=torch.float32, device=params.device)
    for t in range(1, steps + 1):
        B.mlp_backward(params, X, y, ctx=ctx, grad=grad, loss=losses[t - 1:t])
        B.mlp_adam(params, grad, m, v, lr, t, ctx=ctx)
    return (losses.cpu().numpy() / n).tolist()
