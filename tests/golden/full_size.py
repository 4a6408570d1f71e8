"""Full-size oracle goldens for the GPU parity tests (test infrastructure).

The FP64 oracle needs minutes to hours for the iterations of the full-size
workloads (naive DFT matrices at 2048, 4096 and 8192 points), so its results
are computed once by this script and stored here as small ``.npz`` files:
residual histories, step and threshold histories, and sampled columns of the
final image.  The script calls only ``oracle/`` and ``inputs/``; nothing it
stores comes from the HIP path.  The GPU tests rebuild the same input y with
the same functions (the seeded recipe below, simulated through the oracle's
G), check it against the digest stored with the golden, run the HIP solver
on it and compare.

    python tests/golden/full_size.py sparse_4096_ita       # eq. (th2d), 100 iterations
    python tests/golden/full_size.py sparse_4096_adaptive  # Section IV.B, 5 iterations
    python tests/golden/full_size.py stripmap_2048_ita     # eq. (th2d), 200 iterations
    python tests/golden/full_size.py sparse_8192_ita       # eq. (th2d), 3 iterations
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import inputs  # noqa: E402
from oracle import csa, ita, sim  # noqa: E402

# Sampled columns: both edges of the grid, column-tile edges of two- and
# four-column tiles, the reference column N_r/2 and its neighbours.
COLS = {
    2048: [0, 1, 2, 3, 4, 5, 255, 256, 1023, 1024, 1025, 1535, 2044, 2045, 2046, 2047],
    4096: [0, 1, 2, 3, 4, 5, 511, 512, 1023, 1024, 2047, 2048, 2049, 3071, 4094, 4095],
    8192: [0, 1, 3, 4, 4095, 4096, 4097, 8191],
}


def path(name):
    return os.path.join(HERE, f"{name}.npz")


def sparse_problem(name):
    """The sparse-field workload ``name`` (sparse_4096, sparse_8192): scene
    x (a density fraction of pixels, log-normal magnitude, uniform phase),
    mask, and y = m o (G x + s n) through the oracle's G at the stated SNR.
    Returns (geometry, x, y, mask, k = nonzero count)."""
    wl = inputs.workload(name)
    shape = wl["shape"]
    g = csa.Geometry(wl["params"], shape)
    x = inputs.sparse_field(shape, wl["density"], wl["seed"])
    k = int(np.count_nonzero(x))
    mask = inputs.random_mask(shape, wl["mask_rate"], wl["seed"] + 1)
    noise = inputs.circular_noise(shape, wl["seed"] + 2)
    y = sim.add_noise(csa.G(x, g), mask, wl["snr_db"], noise)
    return g, x, y, mask, k


def stripmap_2048_problem():
    """The 2048 x 2048 workload: 200 point targets plus extended patches over
    2 % of the pixels, echo through the oracle's G, 30 % mask, 15 dB.
    Returns (geometry, x, y, mask, k = nonzero count)."""
    wl = inputs.workload("stripmap_2048")
    shape = wl["shape"]
    g = csa.Geometry(wl["params"], shape)
    rows, cols, sig = inputs.point_targets(shape, wl["targets"], seed=wl["seed"])
    x = inputs.targets_to_image(shape, rows, cols, sig)
    x = x + inputs.extended_patches(shape, wl["patch_coverage"], seed=wl["seed"] + 1)
    mask = inputs.random_mask(shape, wl["mask_rate"], seed=wl["seed"] + 2)
    noise = inputs.circular_noise(shape, wl["seed"] + 3)
    y = sim.add_noise(csa.G(x, g), mask, wl["snr_db"], noise)
    return g, x, y, mask, int(np.count_nonzero(x))


def y_digest(y):
    """||y||^2 and 64 spread samples: enough to tell that a rebuilt y is the
    one the golden was computed from."""
    flat = np.asarray(y).ravel()
    idx = np.linspace(0, flat.size - 1, 64).astype(np.int64)
    return float(np.vdot(flat, flat).real), idx, flat[idx].astype(np.complex128)


def check_digest(y, gold):
    """True when y matches the digest stored with the golden (to FP64
    rounding differences between machines)."""
    n2, idx, vals = y_digest(y)
    ok = abs(n2 - float(gold["y_norm2"])) <= 1e-9 * float(gold["y_norm2"])
    return ok and np.allclose(vals, gold["y_samples"], rtol=1e-9, atol=1e-12) and \
        np.array_equal(idx, gold["y_index"])


def _save(name, **arrays):
    np.savez_compressed(path(name), **arrays)
    print(f"wrote {path(name)}", flush=True)


def make_ita(name, iters):
    """Eq. (th2d), Algorithm 1 with the lambda of the sparsity rule."""
    t0 = time.time()
    if name.startswith("stripmap_2048"):
        g, x, y, mask, k = stripmap_2048_problem()
    else:
        g, x, y, mask, k = sparse_problem(name.rsplit("_", 1)[0])
    lam = ita.lambda_from_sparsity(y, mask, k, g)
    print(f"{name}: problem built, lambda {lam:.6g}, k {k} ({time.time() - t0:.0f} s)", flush=True)
    xo, hist = ita.ita(y, mask, lam, iters, g)
    cols = COLS[y.shape[1]]
    n2, idx, vals = y_digest(y)
    _save(name, iters=iters, lam=lam, k=k, resid=np.asarray(hist), cols=np.asarray(cols),
          x_cols=xo[:, cols].astype(np.complex64), x_norm2=float(np.vdot(xo, xo).real),
          nnz=int(np.count_nonzero(xo)), y_norm2=n2, y_index=idx, y_samples=vals)
    print(f"{name}: {iters} iterations in {time.time() - t0:.0f} s", flush=True)


def make_adaptive(name, iters):
    """Section IV.B: mu_t and lambda_t per iteration, k = the nonzero count."""
    t0 = time.time()
    g, x, y, mask, k = sparse_problem(name.rsplit("_", 1)[0])
    xo, resid, mus, lams = ita.ita_adaptive(y, mask, k, iters, g)
    cols = COLS[y.shape[1]]
    n2, idx, vals = y_digest(y)
    _save(name, iters=iters, k=k, resid=np.asarray(resid), mu=np.asarray(mus), lam=np.asarray(lams),
          cols=np.asarray(cols), x_cols=xo[:, cols].astype(np.complex64),
          nnz=int(np.count_nonzero(xo)), y_norm2=n2, y_index=idx, y_samples=vals)
    print(f"{name}: {iters} iterations in {time.time() - t0:.0f} s", flush=True)


MAKERS = {
    "sparse_4096_ita": lambda: make_ita("sparse_4096_ita", 100),
    "sparse_4096_adaptive": lambda: make_adaptive("sparse_4096_adaptive", 5),
    "stripmap_2048_ita": lambda: make_ita("stripmap_2048_ita", 200),
    "sparse_8192_ita": lambda: make_ita("sparse_8192_ita", 3),
}


if __name__ == "__main__":
    for n in sys.argv[1:] or list(MAKERS):
        MAKERS[n]()
