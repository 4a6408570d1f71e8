"""Range-Doppler focusing chain M and its approximated observation G = M^H
(FP64, test infrastructure only).

Section III.C works the approximated observation for the range-Doppler
algorithm, eq. (RDA):

    M(Y) = F_eta^H { P_eta o C< F_eta [ P_tau o (Y F_tau) ] F_tau^H > }

range compression P_tau in the range-frequency domain, range cell migration
correction C in the range-Doppler domain (a space-variant shift by truncated
sinc interpolation, eq. (RCMCs)), azimuth compression P_eta in the
range-Doppler domain.  Its inverse is built step by step (rules i)-iii)),
with the interpolation inverted by D = C^T (eq. (CD)), eq. (apob):

    G(X) = { P_tau^* o < F_eta^H D[ P_eta^* o (F_eta X) ] F_tau > } F_tau^H

so G = M^H exactly (Theorem 1) while G is only close to M^-1 (D inverts C up
to the interpolation error).  Arrays are [N_a, N_r]; the DFTs are unitary;
the azimuth and range transforms act on different axes and commute.

Readings (the paper leaves these open):
  * P_tau(f_tau) = exp(+i pi f_tau^2 / K_r): the matched filter of the
    up-chirp exp(+i pi K_r t^2) under the DFT kernel exp(-2 pi i k n / N)
    (the sign printed in eq. (amf) fits the opposite kernel), as for the
    chirp-scaling chain;
  * P_eta(f_eta; tau) = exp(-i pi f_eta^2 / K_a(tau)) as printed, with
    K_a(tau) = 2 V^2 / (lambda_w R0(tau)); no constant phase, so a focused
    target keeps the phase -4 pi R0 / lambda_w of its echo;
  * the migration of eq. (RCMCs), measured in range samples:
    delta(f_eta, tau_j) = tau_j (1/D(f_eta) - 1) f_s, D the migration factor
    of the chirp-scaling chain (target at range time tau_j / D in the
    range-Doppler domain);
  * the truncated sinc uses K taps (K even, default 8): output j of C takes
    V at (p + t) mod N_r, p = floor(j + delta_j), t = -K/2 + 1 .. K/2, with
    weight sinc(t - (j + delta_j - p)), sinc(x) = sin(pi x) / (pi x).
"""

import numpy as np

from . import csa as _csa
from . import dft as _dft

C_LIGHT = _csa.C_LIGHT
DEFAULT_TAPS = 8


class RdaGeometry:
    """Grids, filters and migration of the range-Doppler chain for one
    (params, shape) pair (the grids of oracle.csa.Geometry)."""

    def __init__(self, params, shape, taps=DEFAULT_TAPS):
        if taps < 2 or taps % 2:
            raise ValueError("taps must be even and >= 2")
        self.g = _csa.Geometry(params, shape)
        self.p = self.g.p
        self.shape = self.g.shape
        self.taps = int(taps)
        p = self.p
        ka = 2.0 * p["v"] ** 2 / (self.g.lam * self.g.r0)  # [N_r]
        self.p_tau = np.exp(1j * np.pi * self.g.f_tau ** 2 / p["Kr"])  # [N_r]
        self.p_eta = np.exp(-1j * np.pi * self.g.f_eta[:, None] ** 2 / ka[None, :])  # [N_a, N_r]
        # migration in range samples, [N_a, N_r]
        self.delta = self.g.tau[None, :] * (1.0 / self.g.D[:, None] - 1.0) * p["fs"]


def _taps(delta_row, taps):
    """Per output j: (indices (p + t) mod N, weights sinc(t - fr)), each [N, K]."""
    n = delta_row.size
    pos = np.arange(n) + delta_row
    p = np.floor(pos)
    fr = pos - p
    t = np.arange(-taps // 2 + 1, taps // 2 + 1)
    idx = (p[:, None].astype(np.int64) + t[None, :]) % n
    w = np.sinc(t[None, :] - fr[:, None])
    return idx, w


def rcmc(v, delta, taps):
    """C of eq. (RCMCs): per Doppler row, U[j] = sum_t V[(p_j + t) mod N] w_jt
    (a gather)."""
    v = np.asarray(v, dtype=np.complex128)
    u = np.zeros_like(v)
    for i in range(v.shape[0]):
        idx, w = _taps(delta[i], taps)
        u[i] = np.sum(v[i][idx] * w, axis=1)
    return u


def rcmc_transpose(u, delta, taps):
    """D = C^T (eq. (CD)): per Doppler row, V[(p_j + t) mod N] += U[j] w_jt
    (the same index pairs and weights, scattered)."""
    u = np.asarray(u, dtype=np.complex128)
    v = np.zeros_like(u)
    for i in range(u.shape[0]):
        idx, w = _taps(delta[i], taps)
        np.add.at(v[i], idx.ravel(), (u[i][:, None] * w).ravel())
    return v


def M(y, rg):
    """eq. (RDA): range compression, azimuth DFT, range IDFT, RCMC, azimuth
    compression, azimuth IDFT."""
    a = _dft.dft(np.asarray(y, dtype=np.complex128), axis=1)
    a = rg.p_tau[None, :] * a
    a = _dft.dft(a, axis=0)
    a = _dft.idft(a, axis=1)
    a = rcmc(a, rg.delta, rg.taps)
    a = rg.p_eta * a
    return _dft.idft(a, axis=0)


def G(x, rg):
    """eq. (apob): every step of eq. (RDA) replaced by its adjoint, in reverse
    order (conjugate filters, D = C^T for the interpolation)."""
    a = _dft.dft(np.asarray(x, dtype=np.complex128), axis=0)
    a = np.conj(rg.p_eta) * a
    a = rcmc_transpose(a, rg.delta, rg.taps)
    a = _dft.dft(a, axis=1)
    a = _dft.idft(a, axis=0)
    a = np.conj(rg.p_tau)[None, :] * a
    return _dft.idft(a, axis=1)
