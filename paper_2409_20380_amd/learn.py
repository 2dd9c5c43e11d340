"""Training driver of the learned node-wise predictor.

The network's training data are trajectories the solver generates itself
(plain snapshot predictor, Algorithm 1 to the tolerance); samples are gathered
on the device during ``ebe_step`` and the network is trained on the device by
the library's own forward / backward / Adam kernels.  This module only
orchestrates those calls: it holds no arithmetic of the method.
"""
from __future__ import annotations

import time

import numpy as np

from . import ebe, inputs


def generate(sol, wl, seeds, steps, nodes, capacity, log=None):
    """Run one trajectory per seed from rest, collecting samples at `nodes`
    (int32 CUDA tensor of node ids) on every step from the fifth on."""
    sol.set_predictor(ebe.PRED_SNAPSHOT)
    sol.collect(capacity, nodes)
    t0 = time.time()
    iters = []
    for k, seed in enumerate(seeds):
        wave = inputs.base_wave(seed, steps, wl.dt, *wl.f_band)
        sol.reset()
        for it in range(1, steps + 1):
            st = sol.step(base_acc=wave[it])
            iters.append(st.iters)
        if log:
            log(f"trajectory {k + 1}/{len(seeds)} (seed {seed}) done; {sol.samples().shape[0]} samples; "
                f"{time.time() - t0:.1f} s")
    sol.collect(capacity, None)
    return float(np.mean(iters))


def train(sol, seed, schedule, batch, init_seed=0, log=None):
    """Fit the scales to the samples, initialise the weights (Glorot) and run
    Adam phases [(steps, lr), ...]; returns the per-step losses."""
    import torch
    scales = sol.mlp_fit_scales()
    sol.mlp_set(inputs.mlp_init(init_seed), scales)
    count = sol.samples().shape[0]
    losses = []
    for k, (steps, lr) in enumerate(schedule):
        idx = torch.from_numpy(inputs.minibatches(seed + k, steps, batch, count)).cuda()
        t0 = time.time()
        losses.append(sol.mlp_train(idx, lr))
        if log:
            log(f"phase {k}: {steps} Adam steps (batch {batch}, lr {lr:g}) in {time.time() - t0:.2f} s; "
                f"loss {losses[-1][:8].mean():.4f} -> {losses[-1][-8:].mean():.4f}")
    return np.concatenate(losses) if losses else np.zeros(0)
