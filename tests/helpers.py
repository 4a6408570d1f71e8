"""Shared helpers of the test suite: problem construction through the oracle
(test infrastructure) and comparison metrics."""

import sys

import numpy as np

import inputs
from oracle import csa, ita, sim


def rel_l2(a, b):
    """||a - b|| / ||b||."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def say(msg):
    """Progress line that names the case, flushed before any GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


def point_problem(params, shape, targets, rate, snr_db, seed, echo="exact"):
    """Point-target scene, sampled raw data and lambda by the sparsity rule
    (Section IV.B) with k = number of targets.

    Returns (x_true, y (zero-filled, complex128), mask (bool), lam)."""
    g = csa.Geometry(params, shape)
    rows, cols, sig = inputs.point_targets(shape, targets, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    if echo == "exact":
        clean = sim.echo(params, shape, rows, cols, sig)
    else:
        clean = csa.G(xt, g)
    mask = inputs.random_mask(shape, rate, seed=seed + 1000)
    noise = inputs.circular_noise(shape, seed=seed + 2000)
    y = sim.add_noise(clean, mask, snr_db, noise)
    lam = ita.lambda_from_sparsity(y, mask, targets, g)
    return xt, y, mask, lam
