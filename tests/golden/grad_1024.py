"""Oracle gradient of the differentiated workload, for the benchmark's
accuracy figure (test infrastructure).

The workload (1024 x 1024, 100 point targets, 50 % mask, 20 dB, K = 20
unrolled iterations of eq. (th2d) / Algorithm 1, loss ||X^(K) - x*||^2)
with its raw data simulated through the operator G (y = m o (G x* + s n)),
so that the benchmark can rebuild the same input with the GPU's G.  The
FP64 oracle (``oracle.grad``, pinned by finite differences and tangents)
gives the loss, the derivatives in lambda, K_a and K_r, and dL/dy on 256
seeded positions; this script stores them in ``grad_1024.npz``.  It calls
only ``oracle/`` and ``inputs/``.

    python tests/golden/grad_1024.py
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
from oracle import csa, grad, ita  # noqa: E402

PATH = os.path.join(HERE, "grad_1024.npz")
SAMPLES = 256


def main():
    wl, xt, mask, noise, pick = inputs.gradient_problem_parts("grad_1024", SAMPLES)
    shape, K, p = wl["shape"], wl["iters"], wl["params"]
    g = csa.Geometry(p, shape)
    clean = csa.G(xt, g)
    s = np.sqrt(np.mean(np.abs(clean[mask]) ** 2) / 10.0 ** (wl["snr_db"] / 10.0))
    y = np.where(mask, clean + s * noise, 0.0)
    lam = ita.lambda_from_sparsity(y, mask, wl["targets"], g)
    t0 = time.time()
    L, (ybar, lbar, kabar, krbar) = grad.loss_and_grad(y, mask, lam, K, p, shape, xt)
    print(f"oracle gradient: {time.time() - t0:.0f} s; L {L:.6g} lambda {lam:.6g} "
          f"dL/dlambda {lbar:.6g} dL/dKa {kabar:.6g} dL/dKr {krbar:.6g}")
    np.savez(PATH, loss=L, lam=lam, lbar=lbar, kabar=kabar, krbar=krbar, pick=pick,
             ybar=ybar.ravel()[pick], ybar_norm=float(np.linalg.norm(ybar)),
             y_norm=float(np.linalg.norm(y)), noise_scale=s)


if __name__ == "__main__":
    main()
