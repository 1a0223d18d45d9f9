"""Training loop of the learned destroy proposal (marshalling only).

Every step calls the library: a batch of recorded (removal set, makespan
change) pairs drawn on the device (alns_record_batch), the network's forward
pass, set loss, backward pass and momentum step (vrprpd_mlp_*).  The host
only sequences the calls and reads the loss back now and then.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import AlnsState, Mlp


def record(state: AlnsState, iterations: int, stream=None) -> int:
    """Run `iterations` plain ALNS iterations recording one set per chain per
    iteration; returns the number of sets recorded."""
    state.record(state.chains * iterations, stream=stream)
    state.step(iterations, stream=stream)
    return state.record_info()[0]


def set_loss(mlp: Mlp, x, seg, target, stream=None) -> float:
    """Mean squared error of the network's set scores on one batch."""
    mlp.forward(x, stream=stream)
    return float(mlp.loss(seg, target, stream=stream).mean().item())


def baseline_loss(target) -> float:
    """Error of always predicting the batch's mean change."""
    t = target.double()
    return float(((t - t.mean()) ** 2).mean().item())


def train(mlp: Mlp, source: AlnsState, steps: int, batch_sets: int = 512, lr: float = 1e-3,
          momentum: float = 0.9, seed: int = 0, log_every: int = 0, stream=None):
    """`steps` momentum SGD steps on batches drawn from `source`'s records.
    Returns the losses read back every `log_every` steps (none if 0)."""
    losses = []
    for s in range(steps):
        x, seg, tgt = source.record_batch(batch_sets, seed=(seed << 20) + s, stream=stream)
        mlp.forward(x, stream=stream)           # padding rows lie outside every set
        sq = mlp.loss(seg, tgt, stream=stream)
        mlp.backward(stream=stream)
        mlp.sgd_step(lr, momentum, stream=stream)
        if log_every and s % log_every == 0:
            losses.append(float(sq.mean().item()))
    return losses


def held_out(mlp: Mlp, source: AlnsState, batches: int = 8, batch_sets: int = 512, seed: int = 99):
    """(network loss, mean-predictor loss) averaged over batches of another
    run's records."""
    a, b = [], []
    for i in range(batches):
        x, seg, tgt = source.record_batch(batch_sets, seed=seed + i)
        a.append(set_loss(mlp, x, seg, tgt))
        b.append(baseline_loss(tgt))
    return float(np.mean(a)), float(np.mean(b))
