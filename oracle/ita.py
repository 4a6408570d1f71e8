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

``iters`` counts the updates X^(1) .. X^(iters).  ``geom`` is an
oracle.csa.Geometry (chirp-scaling chain) or an oracle.rda.RdaGeometry
(range-Doppler chain of eq. (RDA)); the iteration is the same.
"""

import numpy as np

from . import csa as _csa
from . import rda as _rda


def _sampled(mask, a):
    """Theta^T Theta a: the entries of a at sampled positions, 0 elsewhere.
    Entries outside the mask are dropped whatever their value (the sampling
    operator of eq. (model) selects the measured samples, and its transpose
    zero-fills), so a non-finite value there does not reach the result."""
    return np.where(np.asarray(mask, dtype=bool), a, 0.0)


def _G(x, geom):
    """G of the focusing chain geom describes (chirp scaling or range-Doppler)."""
    return _rda.G(x, geom) if isinstance(geom, _rda.RdaGeometry) else _csa.G(x, geom)


def _M(y, geom):
    """M = G^H of the focusing chain geom describes."""
    return _rda.M(y, geom) if isinstance(geom, _rda.RdaGeometry) else _csa.M(y, geom)


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


def ita(y, mask, lam, iters, geom, mu=1.0, x0=None, trace=None):
    """Algorithm 1.  Returns (X^(iters), [||R^(0)||^2, ..., ||R^(iters-1)||^2]).

    ``y`` is the zero-filled sampled raw data, ``mask`` the sampling mask.
    ``x0`` (default 0) is the starting iterate.  ``trace``, if a dict,
    receives the lists "l1" (||X^(t+1)||_1, the sum of magnitudes) and "nnz"
    (the nonzero count of X^(t+1)), t = 0 .. iters-1.
    """
    y = np.asarray(y, dtype=np.complex128)
    x = np.zeros_like(y) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    for _ in range(int(iters)):
        if np.any(x):
            r = _sampled(mask, y - _G(x, geom))
        else:
            r = _sampled(mask, y)  # G is linear, so G(0) = 0
        hist.append(float(np.vdot(r, r).real))
        dx = _M(r, geom)
        x = soft_threshold(x + mu * dx, lam * mu)
        if trace is not None:
            trace.setdefault("l1", []).append(float(np.abs(x).sum()))
            trace.setdefault("nnz", []).append(int(np.count_nonzero(x)))
    return x, hist


def lambda_from_sparsity(y, mask, k, geom, mu=1.0):
    """Section IV.B: lambda = |b_mu(x)|_{k+1} / mu, the (k+1)-th largest
    magnitude of b_mu(x) = x + mu dx, taken once at x = X^(0) = 0, where
    b_mu(0) = mu M(m o y)."""
    b = mu * _M(_sampled(mask, np.asarray(y, dtype=np.complex128)), geom)
    mags = np.sort(np.abs(b).ravel())[::-1]
    return float(mags[int(k)] / mu)


def objective(x, y, mask, lam, geom):
    """1/2 ||m o (y - G x)||^2 + lambda ||x||_1, the objective whose
    proximal-gradient step with threshold lambda*mu is eq. (th2d)."""
    r = _sampled(mask, y - _G(x, geom))
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.abs(x).sum())


def kth_largest_magnitude(v, r):
    """|v|_r: the r-th largest magnitude of v (r counted from 1), or 0 when
    v has fewer than r entries."""
    a = np.sort(np.abs(np.asarray(v)).ravel())[::-1]
    return float(a[r - 1]) if 1 <= r <= a.size else 0.0


def normalized_step(dx, support, mask, geom):
    """Step mu_i of Section IV.B (eq. (mure), adaptive form), read as the
    normalized step of the cited iterative hard thresholding: the printed
    ratio is inverted, and with it mu_i would be at most 1 and shrink as the
    mask thins, against the condition 0 < mu^-1 < ||A||^2 it is meant to meet
    (Section IV.B).  So

        mu = ||dX_G||^2 / ||m o G(dX_G)||^2,

    dX_G = dX on the support G of the current iterate and 0 elsewhere.  It is
    the exact minimiser of the data term 1/2 ||m o (y - G(X + t dX_G))||^2
    over t.  With an empty support (the first iteration) the ratio is 0/0;
    mu = 1 there, which is the same ratio over the whole image (G M = I and
    M is unitary, so ||m o G M(m o R)|| = ||m o R|| = ||M(m o R)||).  A zero
    denominator also gives mu = 1."""
    dxk = np.where(support, np.asarray(dx, dtype=np.complex128), 0.0)
    num = float(np.vdot(dxk, dxk).real)
    if num == 0.0:
        return 1.0
    gk = _sampled(mask, _G(dxk, geom))
    den = float(np.vdot(gk, gk).real)
    return num / den if den > 0.0 else 1.0


def ita_adaptive(y, mask, k, iters, geom, x0=None):
    """Eq. (th2d) with both parameters of Section IV.B set per iteration:

        R      = m o (Y_s - G(X))
        dX     = M(R)
        mu_i   = normalized_step(dX, supp X, m)
        V      = X + mu_i dX                       (= b_mu(X))
        lambda_i mu_i = |V|_{k+1}                  (the (k+1)-th largest magnitude)
        X+     = E_{1, lambda_i mu_i}(V)            (keeps the k largest, shrunk)

    ``x0`` (default 0) is the starting iterate.
    Returns (X^(iters), [||R^(i)||^2], [mu_i], [lambda_i])."""
    y = np.asarray(y, dtype=np.complex128)
    x = np.zeros_like(y) if x0 is None else np.array(x0, dtype=np.complex128)
    resid, mus, lams = [], [], []
    for _ in range(int(iters)):
        r = _sampled(mask, y - _G(x, geom)) if np.any(x) else _sampled(mask, y)
        resid.append(float(np.vdot(r, r).real))
        dx = _M(r, geom)
        mu = normalized_step(dx, x != 0, mask, geom)
        v = x + mu * dx
        sigma = kth_largest_magnitude(v, int(k) + 1)
        x = soft_threshold(v, sigma)
        mus.append(mu)
        lams.append(sigma / mu)
    return x, resid, mus, lams


def safeguard_bound(x_new, x, mask, geom, c):
    """The step bound of the support-change safeguard of the cited normalized
    iterative hard thresholding (Section IV.B cites it for mu_i):

        omega = (1 - c) ||X+ - X||^2 / ||m o G(X+ - X)||^2,

    +inf when the denominator is 0 (no measured change: no bound)."""
    d = np.asarray(x_new, dtype=np.complex128) - np.asarray(x, dtype=np.complex128)
    num = float(np.vdot(d, d).real)
    gd = _sampled(mask, _G(d, geom))
    den = float(np.vdot(gd, gd).real)
    return (1.0 - c) * num / den if den > 0.0 else np.inf


def ita_adaptive_safeguarded(y, mask, k, iters, geom, c=0.01, kappa=2.0, max_shrinks=2, x0=None):
    """ita_adaptive with the support-change safeguard of the cited normalized
    iterative hard thresholding, applied to the paper's soft-threshold step
    (whose support is the k largest |V|, as the hard threshold's):

        V = X + mu dX,  X+ = E_{1, |V|_{k+1}}(V)
        while supp X+ != supp X and fewer than max_shrinks shrinks so far:
            if mu <= safeguard_bound(X+, X): stop
            mu <- mu / (kappa (1 - c));  V, X+ again with the new mu

    kappa (1 - c) > 1.  With mu <= omega the step satisfies the descent
    condition of that method; max_shrinks bounds the loop (the cited method
    has no bound).  Returns (X^(iters), [||R^(i)||^2], [mu_i], [lambda_i],
    [shrinks_i], [mu / omega at each bound test])."""
    if not (0.0 < c < 1.0) or not (kappa * (1.0 - c) > 1.0):
        raise ValueError("need 0 < c < 1 and kappa (1 - c) > 1")
    y = np.asarray(y, dtype=np.complex128)
    x = np.zeros_like(y) if x0 is None else np.array(x0, dtype=np.complex128)
    resid, mus, lams, shrinks, ratios = [], [], [], [], []
    for _ in range(int(iters)):
        r = _sampled(mask, y - _G(x, geom)) if np.any(x) else _sampled(mask, y)
        resid.append(float(np.vdot(r, r).real))
        dx = _M(r, geom)
        mu = normalized_step(dx, x != 0, mask, geom)
        support = x != 0

        def step(mu):
            v = x + mu * dx
            sigma = kth_largest_magnitude(v, int(k) + 1)
            return soft_threshold(v, sigma), sigma

        x_new, sigma = step(mu)
        s = 0
        while s < max_shrinks and np.any((x_new != 0) != support):
            omega = safeguard_bound(x_new, x, mask, geom, c)
            ratios.append(mu / omega)
            if mu <= omega:
                break
            mu = mu / (kappa * (1.0 - c))
            s += 1
            x_new, sigma = step(mu)
        x = x_new
        mus.append(mu)
        lams.append(sigma / mu)
        shrinks.append(s)
    return x, resid, mus, lams, shrinks, ratios
