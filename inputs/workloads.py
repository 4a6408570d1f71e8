"""Workload descriptions (plain data): grid shape, scene recipe, mask rate,
SNR, iteration count and seed.  Simulation of the raw data from a scene is
method arithmetic and lives with whoever consumes these records."""

import numpy as np

from .params import RADAR_STRIPMAP
from .scenes import circular_noise, point_targets, random_mask, rng, targets_to_image

WORKLOADS = {
    # 256 x 256 stripmap scene, 20 point targets, exact point-target echoes.
    "stripmap_256": dict(
        shape=(256, 256), params=RADAR_STRIPMAP, scene="points", targets=20,
        amp=(0.5, 1.0), mask_rate=0.5, snr_db=20.0, iters=100, seed=1,
        echo="exact"),
    # 2048 x 2048: 200 point targets plus extended patches over 2 % of pixels.
    "stripmap_2048": dict(
        shape=(2048, 2048), params=RADAR_STRIPMAP, scene="points+patches",
        targets=200, amp=(0.5, 1.0), patch_coverage=0.02, mask_rate=0.3,
        snr_db=15.0, iters=200, seed=2, echo="operator"),
    # 4096 x 4096: 1 % sparse log-normal field, 50 % mask, 20 dB.
    "sparse_4096": dict(
        shape=(4096, 4096), params=RADAR_STRIPMAP, scene="sparse",
        density=0.01, mask_rate=0.5, snr_db=20.0, iters=100, seed=6,
        echo="operator"),
    # 8192 x 8192 wide swath: same recipe as the 4096 scene.
    "sparse_8192": dict(
        shape=(8192, 8192), params=RADAR_STRIPMAP, scene="sparse",
        density=0.01, mask_rate=0.5, snr_db=20.0, iters=100, seed=3,
        echo="operator"),
    # 64 scenes with per-dimension sizes from {512, 1024, 1536, 2048}.
    "batched_64": dict(
        count=64, sizes=(512, 1024, 1536, 2048), params=RADAR_STRIPMAP,
        scene="points", targets=(50, 300), amp=(0.5, 1.0),
        mask_rate=(0.3, 0.7), snr_db=20.0, iters=100, seed=4,
        echo="operator"),
    # 1024 x 1024, 100 targets, K = 20 unrolled iterations, checkpoint every 5.
    "grad_1024": dict(
        shape=(1024, 1024), params=RADAR_STRIPMAP, scene="points",
        targets=100, amp=(0.5, 1.0), mask_rate=0.5, snr_db=20.0, iters=20,
        every=5, seed=5, echo="exact"),
}


def workload(name):
    """A copy of one workload record."""
    return dict(WORKLOADS[name])


def gradient_problem_parts(name="grad_1024", samples=256):
    """The seeded parts of a differentiated workload: the record, the true
    scene x* (point targets), the mask, unit circular noise and ``samples``
    sorted sampled positions (flat indices) at which dL/dy is compared."""
    wl = workload(name)
    shape = wl["shape"]
    rows, cols, sig = point_targets(shape, wl["targets"], seed=wl["seed"], amp=wl["amp"])
    xt = targets_to_image(shape, rows, cols, sig)
    mask = random_mask(shape, wl["mask_rate"], seed=wl["seed"] + 1)
    noise = circular_noise(shape, seed=wl["seed"] + 2)
    sampled = np.flatnonzero(mask.ravel())
    pick = np.sort(rng(wl["seed"] + 3).choice(sampled, samples, replace=False))
    return wl, xt, mask, noise, pick
