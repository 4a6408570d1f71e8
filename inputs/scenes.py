"""Seeded random scene content, masks and noise (numpy only).

Every generator takes an explicit integer seed and returns numpy arrays in
float64/complex128/bool; callers convert to the precision they compute in.
"""

import numpy as np


def rng(seed):
    """The one random generator used everywhere: PCG64 via default_rng."""
    return np.random.default_rng(int(seed))


def random_complex(shape, seed, scale=1.0):
    """Circular complex Gaussian array with E|z|^2 = scale^2."""
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) * (scale / np.sqrt(2.0))


def point_targets(shape, count, seed, amp=(0.5, 1.0), margin=0):
    """``count`` distinct integer pixel positions with uniform amplitude and
    uniform phase.  Returns (rows, cols, sigma) with sigma complex128.

    ``margin`` keeps positions that many pixels away from the grid border
    (used where a test wants to look at a chip around each target).
    """
    na, nr = shape
    g = rng(seed)
    h = na - 2 * margin
    w = nr - 2 * margin
    if count > h * w:
        raise ValueError("more targets than admissible pixels")
    flat = g.choice(h * w, size=count, replace=False)
    rows = flat // w + margin
    cols = flat % w + margin
    a = g.uniform(amp[0], amp[1], size=count)
    ph = g.uniform(0.0, 2.0 * np.pi, size=count)
    return rows.astype(np.int64), cols.astype(np.int64), a * np.exp(1j * ph)


def targets_to_image(shape, rows, cols, sigma):
    """Place point reflectivities on an otherwise zero scene."""
    x = np.zeros(shape, dtype=np.complex128)
    x[rows, cols] = sigma
    return x


def sparse_field(shape, density, seed, log_sigma=1.0):
    """Sparse complex field: a ``density`` fraction of pixels (chosen without
    replacement) carry log-normal magnitude exp(N(0, log_sigma^2)) and uniform
    phase; the rest are zero."""
    na, nr = shape
    n = na * nr
    k = int(round(density * n))
    g = rng(seed)
    idx = g.choice(n, size=k, replace=False)
    mag = np.exp(log_sigma * g.standard_normal(k))
    ph = g.uniform(0.0, 2.0 * np.pi, size=k)
    x = np.zeros(n, dtype=np.complex128)
    x[idx] = mag * np.exp(1j * ph)
    return x.reshape(shape)


def extended_patches(shape, coverage, seed, patch=16):
    """Square patches of circular complex Gaussian CN(0,1) amplitude at
    random positions until about ``coverage`` of the pixels are covered.
    Patches may overlap and wrap around the (periodic) grid."""
    na, nr = shape
    g = rng(seed)
    npatch = max(1, int(round(coverage * na * nr / (patch * patch))))
    x = np.zeros(shape, dtype=np.complex128)
    for _ in range(npatch):
        r0 = int(g.integers(0, na))
        c0 = int(g.integers(0, nr))
        rr = (r0 + np.arange(patch)) % na
        cc = (c0 + np.arange(patch)) % nr
        vals = (g.standard_normal((patch, patch))
                + 1j * g.standard_normal((patch, patch))) / np.sqrt(2.0)
        x[np.ix_(rr, cc)] = vals
    return x


def random_mask(shape, rate, seed):
    """Elementwise Bernoulli(rate) raw-domain sampling mask (True = kept)."""
    g = rng(seed)
    return g.random(shape) < rate


def circular_noise(shape, seed):
    """Unit-variance circular complex Gaussian noise (E|n|^2 = 1)."""
    return random_complex(shape, seed, 1.0)


def batched_shapes(count, seed, sizes=(512, 1024, 1536, 2048)):
    """``count`` (N_a, N_r) pairs, each dimension drawn independently and
    uniformly from ``sizes``."""
    g = rng(seed)
    na = g.choice(np.asarray(sizes), size=count)
    nr = g.choice(np.asarray(sizes), size=count)
    return [(int(a), int(b)) for a, b in zip(na, nr)]
