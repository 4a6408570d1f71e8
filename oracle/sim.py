"""Exact stripmap echo model, periodised on the grid (FP64, test
infrastructure only).

Eq. (obf), Section II.A: the echo is the reflectivity convolved with a
time-variant kernel h = h1 (x) h2 (azimuth modulation times the transmitted
pulse, eq. (kncomp)).  Section V.A generates raw data "in time domain by exact
slant range".  For a point target k at pixel (i_k, j_k) with reflectivity
sigma_k, closest-approach range R0_k = R0(tau_{j_k}), the baseband echo at
azimuth time offset d_eta and range time tau is

    sigma_k * w_a(d_eta) * w_r(tau - 2 R_k(d_eta)/c)
            * exp(-i 4 pi fc R_k(d_eta) / c) * exp(i pi Kr (tau - 2 R_k/c)^2)

with exact slant range R_k(d_eta) = sqrt(R0_k^2 + V^2 d_eta^2), a rectangular
pulse window of length Tp and a rectangular azimuth window of length
T_a = ba / K_a(R0_k), K_a = 2 V^2 / (lambda R0_k) (the beam is held constant,
so the processed Doppler bandwidth is ba).  The grid is periodic in both axes
(a DFT-based G models exactly that), so samples falling outside the grid
wrap around.  Each target echo is divided by sqrt(number of window samples)
so that a column of H has unit norm before wrapping.
"""

import numpy as np

C_LIGHT = 299792458.0


def _range_time(params, nr):
    return 2.0 * params["r_ref"] / C_LIGHT + (np.arange(nr) - nr / 2) / params["fs"]


def target_echo_samples(params, shape, i_k, j_k):
    """Unwrapped samples of one unit target: (rows, cols, values) with rows
    and cols already reduced modulo the grid."""
    na, nr = shape
    p = params
    lam = C_LIGHT / p["fc"]
    tau0 = 2.0 * p["r_ref"] / C_LIGHT - (nr / 2) / p["fs"]  # tau of column 0
    r0k = C_LIGHT * (tau0 + j_k / p["fs"]) / 2.0
    ka = 2.0 * p["v"] ** 2 / (lam * r0k)
    ta = p["ba"] / ka
    half_a = int(np.floor(ta * p["prf"] / 2.0))
    d = np.arange(-half_a, half_a + 1)
    deta = d / p["prf"]
    keep_a = np.abs(deta) <= ta / 2.0
    d = d[keep_a]
    deta = deta[keep_a]
    rk = np.sqrt(r0k ** 2 + (p["v"] * deta) ** 2)          # exact slant range
    tc = 2.0 * rk / C_LIGHT                                   # echo delay
    # unwrapped range sample u has time tau0 + u / fs
    u_lo = np.ceil((tc - p["Tp"] / 2.0 - tau0) * p["fs"]).astype(np.int64)
    width = int(np.ceil(p["Tp"] * p["fs"])) + 2
    u = u_lo[:, None] + np.arange(width)[None, :]
    dt = tau0 + u / p["fs"] - tc[:, None]
    keep = np.abs(dt) <= p["Tp"] / 2.0
    phase = (-4.0 * np.pi * p["fc"] * rk / C_LIGHT)[:, None] + np.pi * p["Kr"] * dt ** 2
    val = np.exp(1j * phase)
    rows = np.broadcast_to(((i_k + d) % na)[:, None], u.shape)
    cols = u % nr
    rows, cols, val = rows[keep], cols[keep], val[keep]
    return rows, cols, val / np.sqrt(val.size)


def echo(params, shape, rows, cols, sigma):
    """Raw data Y = H x for point targets (rows, cols, sigma)."""
    na, nr = shape
    y = np.zeros(na * nr, dtype=np.complex128)
    for i_k, j_k, s in zip(np.asarray(rows), np.asarray(cols), np.asarray(sigma)):
        r, c, v = target_echo_samples(params, shape, int(i_k), int(j_k))
        np.add.at(y, r * nr + c, s * v)
    return y.reshape(shape)


def dense_H(params, shape):
    """Dense exact observation matrix H of eq. (ob2d) (row-major vec), one
    column per scene pixel.  Tiny grids only."""
    na, nr = shape
    n = na * nr
    h = np.zeros((n, n), dtype=np.complex128)
    for i_k in range(na):
        for j_k in range(nr):
            r, c, v = target_echo_samples(params, shape, i_k, j_k)
            np.add.at(h[:, i_k * nr + j_k], r * nr + c, v)
    return h


def add_noise(clean, mask, snr_db, noise):
    """Sampled data m o (clean + s n), with s^2 = mean over sampled pixels of
    |clean|^2 / 10^(snr/10); ``noise`` is unit-variance circular Gaussian."""
    m = np.asarray(mask, dtype=bool)
    p_sig = float(np.mean(np.abs(clean[m]) ** 2)) if m.any() else 0.0
    s = np.sqrt(p_sig / 10.0 ** (snr_db / 10.0))
    return np.where(m, clean + s * noise, 0.0)
