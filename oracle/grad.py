"""Gradients of a loss of the unrolled iterative thresholding (FP64, test
infrastructure only).

The method (eq. (th2d), Algorithm 1) run for K iterations from X^(0) = 0 is
a differentiable map of the raw data y, the threshold lambda and the radar
parameters through which G and M = G^H are built.  The gradient is not in
the paper; it is defined here by plain calculus:

  * the loss gradient convention is the real pair dL/dRe z + i dL/dIm z;
  * the radar parameters are the azimuth FM rate K_a = 2 V^2 / (lambda_w
    r_ref) (so V = sqrt(K_a lambda_w r_ref / 2); the stripmap model of
    Section II.A) and the range chirp rate K_r;
  * the derivative of a phase screen exp(i arg(theta)) is
    i (d arg / d theta) exp(i arg), with d arg / d theta written out below
    from the screen definitions of oracle.csa;
  * M and G are differentiated by the product rule along their chains
    (forward mode), and the iteration by reverse accumulation: with V the
    value before the threshold (V = X + mu M(m o (y - G X))),
      Vbar = J_S(V)^T Xbar_next   (J_S the real 2x2 Jacobian of the complex
                                   soft threshold, zero off its support)
      Xbar = Vbar - mu M(m o G Vbar)          (the iteration map is
                                               I - mu M m G, self-adjoint)
      ybar += mu m o G Vbar
      lambdabar += -mu sum_support Re(conj(Xbar_next) V / |V|)
      thetabar += Re <Vbar, mu dM(R) - mu M(m o dG(X))>.
"""

import numpy as np

from . import csa as _csa
from . import dft as _dft
from . import ita as _ita

C_LIGHT = _csa.C_LIGHT


def ka_of(params):
    """Azimuth FM rate at the reference range, K_a = 2 V^2 / (lambda_w r_ref)."""
    lam = C_LIGHT / params["fc"]
    return 2.0 * params["v"] ** 2 / (lam * params["r_ref"])


def with_theta(params, Ka=None, Kr=None):
    """A copy of params with K_a (through V) and/or K_r replaced."""
    p = dict(params)
    if Ka is not None:
        lam = C_LIGHT / p["fc"]
        p["v"] = float(np.sqrt(Ka * lam * p["r_ref"] / 2.0))
    if Kr is not None:
        p["Kr"] = float(Kr)
    return p


def arg_derivatives(geom):
    """d arg_k / d K_a and d arg_k / d K_r for the three screens (radians per
    unit of the parameter), each [N_a, N_r]: {"Ka": (d1, d2, d3), "Kr": ...}."""
    p = geom.p
    v, fc, r_ref, Kr = p["v"], p["fc"], p["r_ref"], p["Kr"]
    lam = C_LIGHT / fc
    f = geom.f_eta
    D = geom.D
    w = lam * f / (2.0 * v)
    dD_dv = w ** 2 / (v * D)
    if p.get("src", 1):
        z = C_LIGHT * r_ref * f ** 2 / (2.0 * v ** 2 * fc ** 3 * D ** 3)
        den = 1.0 - Kr * z
        Km = Kr / den
        dz_dv = z * (-2.0 / v - 3.0 * dD_dv / D)
        dKm_dv = Km ** 2 * dz_dv
        dKm_dKr = 1.0 / den ** 2
    else:
        Km = np.full_like(f, Kr)
        dKm_dv = np.zeros_like(f)
        dKm_dKr = np.ones_like(f)
    e = 1.0 / D - 1.0
    de_dv = -dD_dv / D ** 2
    col = lambda a: a[:, None]
    tau = geom.tau[None, :]
    s = tau - 2.0 * r_ref / (C_LIGHT * col(D))
    ds_dv = 2.0 * r_ref / (C_LIGHT * col(D) ** 2) * col(dD_dv)
    # arg1 = pi Km e s^2
    d1_dv = np.pi * (col(dKm_dv * e + Km * de_dv) * s ** 2 + col(Km * e) * 2.0 * s * ds_dv)
    d1_dKr = np.pi * col(dKm_dKr * e) * s ** 2
    # arg2 = pi D / Km f_tau^2 + 4 pi r_ref f_tau e / c
    ft = geom.f_tau[None, :]
    d2_dv = (np.pi * col((dD_dv * Km - D * dKm_dv) / Km ** 2) * ft ** 2
             + 4.0 * np.pi * r_ref * ft * col(de_dv) / C_LIGHT)
    d2_dKr = -np.pi * col(D * dKm_dKr / Km ** 2) * ft ** 2
    # arg3 = 4 pi fc R0 D / c - 4 pi Km / c^2 h(D) (R0 - r_ref)^2, h = (1 - D) / D^2
    r0 = geom.r0[None, :]
    h = (1.0 - D) / D ** 2
    dh_dv = (D - 2.0) / D ** 3 * dD_dv
    q = (r0 - r_ref) ** 2
    d3_dv = (4.0 * np.pi * fc * r0 * col(dD_dv) / C_LIGHT
             - 4.0 * np.pi / C_LIGHT ** 2 * q * col(dKm_dv * h + Km * dh_dv))
    d3_dKr = -4.0 * np.pi / C_LIGHT ** 2 * q * col(dKm_dKr * h)
    dv_dKa = lam * r_ref / (4.0 * v)
    return {"Ka": (d1_dv * dv_dKa, d2_dv * dv_dKa, d3_dv * dv_dKa),
            "Kr": (d1_dKr, d2_dKr, d3_dKr)}


def M_tangent(r, geom, dargs):
    """(M r, dM r): the chain of M with its derivative carried alongside
    (product rule at each phase stage, transforms linear)."""
    p1, p2, p3 = geom.screens()
    d1, d2, d3 = dargs
    a = _dft.dft(np.asarray(r, dtype=np.complex128), axis=0)
    da = np.zeros_like(a)
    a, da = p1 * a, p1 * da + 1j * d1 * p1 * a
    a, da = _dft.dft(a, axis=1), _dft.dft(da, axis=1)
    a, da = p2 * a, p2 * da + 1j * d2 * p2 * a
    a, da = _dft.idft(a, axis=1), _dft.idft(da, axis=1)
    a, da = p3 * a, p3 * da + 1j * d3 * p3 * a
    return _dft.idft(a, axis=0), _dft.idft(da, axis=0)


def G_tangent(x, geom, dargs):
    """(G x, dG x), with d exp(-i arg) = -i (d arg) exp(-i arg)."""
    p1, p2, p3 = geom.screens()
    d1, d2, d3 = dargs
    c1, c2, c3 = np.conj(p1), np.conj(p2), np.conj(p3)
    a = _dft.dft(np.asarray(x, dtype=np.complex128), axis=0)
    da = np.zeros_like(a)
    a, da = c3 * a, c3 * da - 1j * d3 * c3 * a
    a, da = _dft.dft(a, axis=1), _dft.dft(da, axis=1)
    a, da = c2 * a, c2 * da - 1j * d2 * c2 * a
    a, da = _dft.idft(a, axis=1), _dft.idft(da, axis=1)
    a, da = c1 * a, c1 * da - 1j * d1 * c1 * a
    return _dft.idft(a, axis=0), _dft.idft(da, axis=0)


def ita_states(y, mask, lam, iters, geom, mu=1.0):
    """Forward pass keeping every iterate: (X[0..K], V[0..K-1], R[0..K-1]),
    the same iteration as oracle.ita.ita."""
    y = np.asarray(y, dtype=np.complex128)
    X = [np.zeros_like(y)]
    V, R = [], []
    for _ in range(int(iters)):
        x = X[-1]
        r = _ita._sampled(mask, y - _csa.G(x, geom)) if np.any(x) else _ita._sampled(mask, y)
        v = x + mu * _csa.M(r, geom)
        R.append(r)
        V.append(v)
        X.append(_ita.soft_threshold(v, lam * mu))
    return X, V, R


def threshold_vjp(v, xbar, sigma):
    """(J_S(v)^T xbar, dS/dsigma . xbar) for the complex soft threshold at
    sigma: on |v| > sigma, S(v) = v (1 - sigma/|v|), whose real Jacobian is
    (1 - sigma/|v|) I + sigma v v^T / |v|^3 (symmetric), and dS/dsigma = -v/|v|;
    off the support both are zero."""
    a = np.abs(v)
    on = a > sigma
    vbar = np.zeros_like(v)
    av = a[on]
    vv, xb = v[on], xbar[on]
    dot = (vv.real * xb.real + vv.imag * xb.imag)
    vbar[on] = (1.0 - sigma / av) * xb + sigma * dot / av ** 3 * vv
    dsig = -float(np.sum(dot / av))
    return vbar, dsig


def ita_grad(y, mask, lam, iters, params, shape, xbar, mu=1.0):
    """Gradient of a loss L(X^(K)) given xbar = dL/dX^(K): returns
    (ybar, lambdabar, Kabar, Krbar)."""
    geom = _csa.Geometry(params, shape)
    dargs = arg_derivatives(geom)
    m = np.asarray(mask, dtype=np.float64)
    X, V, R = ita_states(y, mask, lam, iters, geom, mu)
    xbar = np.asarray(xbar, dtype=np.complex128)
    ybar = np.zeros_like(xbar)
    lbar = 0.0
    tbar = {"Ka": 0.0, "Kr": 0.0}
    sigma = lam * mu
    for t in range(int(iters) - 1, -1, -1):
        vbar, dsig = threshold_vjp(V[t], xbar, sigma)
        lbar += mu * dsig
        gv = _csa.G(vbar, geom)
        ybar += mu * m * gv
        for name in ("Ka", "Kr"):
            _, dmr = M_tangent(R[t], geom, dargs[name])
            if np.any(X[t]):
                _, dgx = G_tangent(X[t], geom, dargs[name])
                dv = mu * (dmr - _csa.M(m * dgx, geom))
            else:
                dv = mu * dmr
            tbar[name] += float(np.sum(vbar.real * dv.real + vbar.imag * dv.imag))
        xbar = vbar - mu * _csa.M(m * gv, geom)
    return ybar, lbar, tbar["Ka"], tbar["Kr"]


def loss_and_grad(y, mask, lam, iters, params, shape, x_true, mu=1.0):
    """L = ||X^(K) - x_true||^2 and its gradient (ybar, lambdabar, Kabar, Krbar)."""
    geom = _csa.Geometry(params, shape)
    xk, _ = _ita.ita(y, mask, lam, iters, geom, mu)
    d = xk - x_true
    L = float(np.vdot(d, d).real)
    return L, ita_grad(y, mask, lam, iters, params, shape, 2.0 * d, mu)


def loss(y, mask, lam, iters, params, shape, x_true, mu=1.0):
    """L = ||X^(K) - x_true||^2 for the given parameters (for finite differences)."""
    xk, _ = _ita.ita(y, mask, lam, iters, _csa.Geometry(params, shape), mu)
    d = xk - x_true
    return float(np.vdot(d, d).real)
