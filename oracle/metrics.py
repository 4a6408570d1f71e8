"""Point-target quality metrics (test infrastructure only).

Section V.A.2 scores a focused point target with two numbers.  PSLR (dB)
compares the strongest side lobe with the main-lobe peak, in intensity, so a
more negative value is better.  IRW counts how wide the main lobe is where it
has fallen 3 dB from its peak.  Both are read on cuts through the peak of a
16 x 16 chip around the target, interpolated 16-fold.

Two readings of that interpolation are implemented.  point_response takes it
as exact band-limited (trigonometric) interpolation of the complex chip:
zero padding of its unitary DFT (naive DFT matrices from ``oracle.dft``),
with the Nyquist bin split evenly.  point_response_linear takes it as
bilinear interpolation of the chip's magnitude, the grid an image viewer
draws between pixels.
"""

import numpy as np

from . import dft as _dft


def _zero_pad_1d(spec, m):
    """Place an n-point spectrum (DFT order) into an m-point one."""
    n = spec.shape[0]
    out = np.zeros((m,) + spec.shape[1:], dtype=np.complex128)
    h = n // 2
    out[:h] = spec[:h]
    out[m - h:] = spec[n - h:]
    if n % 2 == 0:  # split the Nyquist bin between +n/2 and -n/2
        out[h] = 0.5 * spec[h]
        out[m - h] = 0.5 * spec[h]
    else:
        out[h] = spec[h]
    return out


def upsample_2d(chip, factor):
    """Band-limited interpolation of a chip by ``factor`` in both axes."""
    chip = np.asarray(chip, dtype=np.complex128)
    a, b = chip.shape
    s = _dft.dft(_dft.dft(chip, axis=0), axis=1)
    s = _zero_pad_1d(s, a * factor)
    s = np.swapaxes(_zero_pad_1d(np.swapaxes(s, 0, 1), b * factor), 0, 1)
    up = _dft.idft(_dft.idft(s, axis=0), axis=1)
    return up * factor  # keeps sample values (unitary DFTs change length)


def chip_around(img, center, size):
    """size x size chip of a periodic image centred on ``center``."""
    na, nr = img.shape
    rr = (center[0] - size // 2 + np.arange(size)) % na
    cc = (center[1] - size // 2 + np.arange(size)) % nr
    return img[np.ix_(rr, cc)]


def irw_samples(cut):
    """Number of samples of a 1-D magnitude cut within 3 dB of its maximum,
    counted contiguously around the maximum."""
    p = np.abs(cut) ** 2
    k = int(np.argmax(p))
    thr = p[k] / 2.0
    lo = k
    while lo - 1 >= 0 and p[lo - 1] >= thr:
        lo -= 1
    hi = k
    while hi + 1 < p.size and p[hi + 1] >= thr:
        hi += 1
    return hi - lo + 1


def irw_fractional(cut):
    """3 dB width of the main lobe in samples, with linear interpolation of
    the power between samples at both crossings."""
    p = np.abs(cut) ** 2
    k = int(np.argmax(p))
    thr = p[k] / 2.0
    lo = k
    while lo - 1 >= 0 and p[lo - 1] >= thr:
        lo -= 1
    hi = k
    while hi + 1 < p.size and p[hi + 1] >= thr:
        hi += 1
    left = lo - (p[lo] - thr) / (p[lo] - p[lo - 1]) if lo > 0 else float(lo)
    right = hi + (p[hi] - thr) / (p[hi] - p[hi + 1]) if hi + 1 < p.size else float(hi)
    return right - left


def pslr_db(cut):
    """Peak side-lobe ratio in dB: highest power outside the main lobe (the
    lobe between the first minima on either side of the maximum) divided by
    the maximum power."""
    p = np.abs(cut) ** 2
    k = int(np.argmax(p))
    lo = k
    while lo - 1 >= 0 and p[lo - 1] < p[lo]:
        lo -= 1
    hi = k
    while hi + 1 < p.size and p[hi + 1] < p[hi]:
        hi += 1
    side = np.concatenate([p[:lo], p[hi + 1:]])
    if side.size == 0 or side.max() <= 0.0:
        return -np.inf
    return 10.0 * np.log10(side.max() / p[k])


def demodulate(chip):
    """Remove the mean linear phase ramp of a chip along each axis (the
    circular centroid of its power spectrum), so that its spectrum is centred
    on zero frequency before band-limited interpolation.  A focused image
    keeps a per-pixel carrier phase (the azimuth filter restores each
    target's own phase), which offsets the range spectrum; magnitudes are
    unchanged by this step."""
    chip = np.asarray(chip, dtype=np.complex128)
    out = chip
    for axis in (0, 1):
        n = chip.shape[axis]
        spec = _dft.dft(out, axis=axis)
        pw = (np.abs(spec) ** 2).sum(axis=1 - axis)
        k = np.arange(n)
        centroid = np.angle(np.sum(pw * np.exp(2j * np.pi * k / n))) * n / (2 * np.pi)
        ramp = np.exp(-2j * np.pi * centroid * np.arange(n) / n)
        out = out * (ramp[:, None] if axis == 0 else ramp[None, :])
    return out


def point_response(img, center, chip=16, factor=16):
    """PSLR (dB) and IRW (upsampled samples) along range and azimuth for the
    target at ``center``: a chip x chip window around it is demodulated,
    upsampled by ``factor`` and cut through its maximum."""
    c = demodulate(chip_around(img, center, chip))
    up = upsample_2d(c, factor)
    pk = np.unravel_index(int(np.argmax(np.abs(up))), up.shape)
    rng_cut = up[pk[0], :]
    az_cut = up[:, pk[1]]
    return dict(
        pslr_r=pslr_db(rng_cut), pslr_a=pslr_db(az_cut),
        irw_r=irw_samples(rng_cut), irw_a=irw_samples(az_cut),
        irw_r_frac=irw_fractional(rng_cut), irw_a_frac=irw_fractional(az_cut),
    )


def upsample_linear_magnitude(chip, factor):
    """Bilinear interpolation of |chip| by ``factor``: samples at t = i/factor,
    i = 0 .. (n - 1) factor, along each axis (separable, piecewise linear
    between the pixel centres)."""
    m = np.abs(np.asarray(chip))
    n0, n1 = m.shape
    t0 = np.arange((n0 - 1) * factor + 1) / factor
    t1 = np.arange((n1 - 1) * factor + 1) / factor
    rows = np.array([np.interp(t1, np.arange(n1), m[i]) for i in range(n0)])
    return np.array([np.interp(t0, np.arange(n0), rows[:, j]) for j in range(rows.shape[1])]).T


def point_response_linear(img, center, chip=16, factor=16):
    """point_response under the second reading of the 16-fold interpolation
    of Section V.A.2 (bilinear interpolation of the chip's magnitude).  A cut
    with no side lobe gives a PSLR of -inf."""
    up = upsample_linear_magnitude(chip_around(img, center, chip), factor)
    pk = np.unravel_index(int(np.argmax(up)), up.shape)
    rng_cut = up[pk[0], :]
    az_cut = up[:, pk[1]]
    return dict(pslr_r=pslr_db(rng_cut), pslr_a=pslr_db(az_cut),
                irw_r=irw_samples(rng_cut), irw_a=irw_samples(az_cut))
