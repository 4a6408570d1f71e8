"""Chirp-scaling focusing chain M and approximated observation G = M^{-1}
(FP64, test infrastructure only).

Paper: Section III.B defines the approximated observation as G = M^{-1} for a
high-precision matched-filter focusing procedure M; Section III.C works the
construction for the range-Doppler algorithm (eq. (RDA)) with the inversion
rules i) FFT pairs and ii) conjugate phases; Section III.D.1 names the
chirp-scaling algorithm (CSA) as a focusing chain whose inverse is obtained
the same way.  The paper prints no CSA formula, so the chain below is the
standard low-squint CSA (chirp scaling in the range-Doppler domain; range
compression, secondary range compression and bulk RCMC in the 2-D frequency
domain; azimuth compression and residual-phase removal in the range-Doppler
domain), all three steps being unimodular phase multiplies:

    M(Y) = F_eta^H [ Phi3 o F_tau^H [ Phi2 o F_tau [ Phi1 o F_eta [Y] ] ] ]
    G(X) = F_eta^H [ Phi1* o F_tau^H [ Phi2* o F_tau [ Phi3* o F_eta [X] ] ] ]

With unitary DFTs this makes G = M^{-1} = M^H exactly (Theorem 1 without its
approximation).  Arrays are [N_a, N_r]: axis 0 = azimuth (eta), axis 1 =
range (tau).  Sign conventions (readings of the paper, pinned by the
focusing tests): DFT kernel exp(-2 pi i k n / N), transmitted up-chirp
exp(+i pi Kr t^2), so the range matched filter is exp(+i pi f^2 / K) (the
sign printed for P_tau in eq. (amf) corresponds to the opposite DFT sign);
the azimuth matched filter reduces to exp(-i pi f_eta^2 / K_a) up to a
constant, as printed for P_eta in eq. (amf).
"""

import numpy as np

from . import dft as _dft

C_LIGHT = 299792458.0


class Geometry:
    """Grids and per-Doppler-bin coefficients of the CSA chain for one
    (params, shape) pair.

    Azimuth frequency f_eta[k] = prf * nu(k) / N_a, range frequency
    f_tau[l] = fs * nu(l) / N_r (nu = signed index, fftfreq order).  Range
    time tau_j = 2 r_ref / c + (j - N_r/2) / fs, slant range R0_j = c tau_j/2,
    so the scene centre (reference range) sits at column N_r/2.
    """

    def __init__(self, params, shape):
        self.p = dict(params)
        na, nr = int(shape[0]), int(shape[1])
        self.shape = (na, nr)
        p = self.p
        if p.get("f_dc", 0.0) != 0.0:
            raise ValueError("only zero Doppler centroid is modelled")
        self.lam = C_LIGHT / p["fc"]
        self.f_eta = p["prf"] * _dft.freq_index(na) / na
        self.f_tau = p["fs"] * _dft.freq_index(nr) / nr
        self.tau = 2.0 * p["r_ref"] / C_LIGHT + (np.arange(nr) - nr / 2) / p["fs"]
        self.r0 = C_LIGHT * self.tau / 2.0
        v = p["v"]
        # Migration factor D(f_eta) = sqrt(1 - (lambda f_eta / (2 V))^2).
        self.D = np.sqrt(1.0 - (self.lam * self.f_eta / (2.0 * v)) ** 2)
        self.D_ref = 1.0  # D at the (zero) Doppler centroid
        # Modified range FM rate including secondary range compression,
        # evaluated at the reference range.
        if p.get("src", 1):
            z = (C_LIGHT * p["r_ref"] * self.f_eta ** 2
                 / (2.0 * v ** 2 * p["fc"] ** 3 * self.D ** 3))
            self.Km = p["Kr"] / (1.0 - p["Kr"] * z)
        else:
            self.Km = np.full(na, p["Kr"], dtype=np.float64)

    # -- phase arguments (radians, each [N_a, N_r]) ------------------------
    def arg1(self):
        """Chirp scaling, range-Doppler domain:
        pi Km (D_ref/D - 1) (tau - 2 r_ref / (c D))^2."""
        D = self.D[:, None]
        Km = self.Km[:, None]
        tref = 2.0 * self.p["r_ref"] / (C_LIGHT * D)
        return np.pi * Km * (self.D_ref / D - 1.0) * (self.tau[None, :] - tref) ** 2

    def arg2(self):
        """Range compression + SRC + bulk RCMC, 2-D frequency domain:
        pi D/(Km D_ref) f_tau^2 + 4 pi r_ref f_tau (1/D - 1/D_ref)/c."""
        D = self.D[:, None]
        Km = self.Km[:, None]
        f = self.f_tau[None, :]
        return (np.pi * D / (Km * self.D_ref) * f ** 2
                + 4.0 * np.pi * self.p["r_ref"] * f * (1.0 / D - 1.0 / self.D_ref) / C_LIGHT)

    def arg3(self):
        """Azimuth compression + residual phase, range-Doppler domain:
        4 pi fc R0 D / c - 4 pi Km/c^2 (1 - D/D_ref) (R0 - r_ref)^2 / D^2."""
        D = self.D[:, None]
        Km = self.Km[:, None]
        r0 = self.r0[None, :]
        return (4.0 * np.pi * self.p["fc"] * r0 * D / C_LIGHT
                - 4.0 * np.pi * Km / C_LIGHT ** 2 * (1.0 - D / self.D_ref)
                * (r0 - self.p["r_ref"]) ** 2 / D ** 2)

    # -- phase screens (each [N_a, N_r], unit modulus) ---------------------
    def phi1(self):
        return np.exp(1j * self.arg1())

    def phi2(self):
        return np.exp(1j * self.arg2())

    def phi3(self):
        return np.exp(1j * self.arg3())

    def screens(self):
        """(Phi1, Phi2, Phi3), computed once and cached."""
        if not hasattr(self, "_screens"):
            self._screens = (self.phi1(), self.phi2(), self.phi3())
        return self._screens


def M(y, geom):
    """Matched-filter focusing chain (Section III.B eq. (focus), CSA form)."""
    p1, p2, p3 = geom.screens()
    a = _dft.dft(np.asarray(y, dtype=np.complex128), axis=0)
    a = p1 * a
    a = _dft.dft(a, axis=1)
    a = p2 * a
    a = _dft.idft(a, axis=1)
    a = p3 * a
    return _dft.idft(a, axis=0)


def G(x, geom):
    """Approximated observation G = M^{-1}: every step of M inverted in
    reverse order (Section III.C rules i) and ii))."""
    p1, p2, p3 = geom.screens()
    a = _dft.dft(np.asarray(x, dtype=np.complex128), axis=0)
    a = np.conj(p3) * a
    a = _dft.dft(a, axis=1)
    a = np.conj(p2) * a
    a = _dft.idft(a, axis=1)
    a = np.conj(p1) * a
    return _dft.idft(a, axis=0)


def M_cols(y, geom, cols):
    """Columns ``cols`` of M(y): the same chain, with the last range inverse
    DFT evaluated only at those output columns (everything after it acts
    column by column)."""
    cols = np.asarray(cols)
    p1, p2, p3 = geom.screens()
    a = _dft.dft(np.asarray(y, dtype=np.complex128), axis=0)
    a = p1 * a
    a = _dft.dft(a, axis=1)
    a = p2 * a
    a = _dft.idft_rows_at(a, cols)
    a = p3[:, cols] * a
    return _dft.idft(a, axis=0)


def G_cols(x, geom, cols):
    """Columns ``cols`` of G(x), evaluated like :func:`M_cols`."""
    cols = np.asarray(cols)
    p1, p2, p3 = geom.screens()
    a = _dft.dft(np.asarray(x, dtype=np.complex128), axis=0)
    a = np.conj(p3) * a
    a = _dft.dft(a, axis=1)
    a = np.conj(p2) * a
    a = _dft.idft_rows_at(a, cols)
    a = np.conj(p1[:, cols]) * a
    return _dft.idft(a, axis=0)
