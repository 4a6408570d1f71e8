"""Iterative thresholding for the approximated-observation CS-SAR model
(FP64, test infrastructure only).

Model eq. (model), Section IV.A: min_X ||Y_s - Theta G(X)||_F^2 + lambda ||X||_1,
with the sampling operators Theta_eta, Theta_tau generalised to an
elementwise raw-domain mask m (Theta^T Theta = multiplication by m, i.e.
zero fill).  Iteration eq. (th2d) / Algorithm 1:

    X^(0) = 0
    R^(i)   = m o (Y_s - G(X^(i)))            (residue)
    dX^(i)  = M(R^(i))                          (matched filter on residue)
    X^(i+1) = E_{1, lambda mu}(X^(i) + mu dX^(i))   (thresholding)

``iters`` counts the updates X^(1) .. X^(iters).
"""

import numpy as np

from . import csa as _csa


def soft_threshold(v, sigma):
    """Complex soft threshold e_{1,sigma} of eq. (L12), with sgn(x) = x/|x|:
    sgn(v)(|v| - sigma) where |v| >= sigma, else 0 (0 maps to 0)."""
    v = np.asarray(v, dtype=np.complex128)
    a = np.abs(v)
    out = np.zeros_like(v)
    keep = a >= sigma
    keep &= a > 0
    out[keep] = v[keep] / a[keep] * (a[keep] - sigma)
    return out


def ita(y, mask, lam, iters, geom, mu=1.0, x0=None):
    """Algorithm 1.  Returns (X^(iters), [||R^(0)||^2, ..., ||R^(iters-1)||^2]).

    ``y`` is the zero-filled sampled raw data, ``mask`` the sampling mask.
    ``x0`` (default 0) is the starting iterate.
    """
    y = np.asarray(y, dtype=np.complex128)
    m = np.asarray(mask, dtype=np.float64)
    x = np.zeros_like(y) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    for _ in range(int(iters)):
        if np.any(x):
            r = m * (y - _csa.G(x, geom))
        else:
            r = m * y  # G is linear, so G(0) = 0
        hist.append(float(np.vdot(r, r).real))
        dx = _csa.M(r, geom)
        x = soft_threshold(x + mu * dx, lam * mu)
    return x, hist


def lambda_from_sparsity(y, mask, k, geom, mu=1.0):
    """Section IV.B: lambda = |b_mu(x)|_{k+1} / mu, the (k+1)-th largest
    magnitude of b_mu(x) = x + mu dx, taken once at x = X^(0) = 0, where
    b_mu(0) = mu M(m o y)."""
    b = mu * _csa.M(np.asarray(mask, dtype=np.float64) * np.asarray(y), geom)
    mags = np.sort(np.abs(b).ravel())[::-1]
    return float(mags[int(k)] / mu)


def objective(x, y, mask, lam, geom):
    """1/2 ||m o (y - G x)||^2 + lambda ||x||_1, the objective whose
    proximal-gradient step with threshold lambda*mu is eq. (th2d)."""
    r = np.asarray(mask, dtype=np.float64) * (y - _csa.G(x, geom))
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.abs(x).sum())
