"""GPU parity of the range-Doppler operator (eq. (RDA), cssar_make_operator_rda)
against the FP64 oracle (oracle/rda.py, pinned on the CPU by Theorem 1, brute
force and the paper's printed point response).

Bars as for the chirp-scaling operator: relative L2 <= 1e-5 per operator
application, <= 1e-4 on final images."""

import numpy as np
import pytest

import inputs
from oracle import ita, rda
from tests.helpers import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OP_TOL = 1e-5
IMG_TOL = 1e-4
STRIP = inputs.RADAR_STRIPMAP
STRESS = inputs.RADAR_LBAND_STRESS


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _h(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("params,shape,taps", [
    (STRIP, (64, 64), 8), (STRIP, (256, 512), 8), (STRIP, (512, 256), 4),
    (STRIP, (768, 1536), 8), (STRESS, (128, 256), 8), (STRESS, (256, 1024), 16),
    (STRIP, (128, 8192), 8), (STRESS, (64, 128), 32),
])
def test_rda_apply_G_and_GH_match_oracle(dev, params, shape, taps):
    import paper_1302_3120_amd as pk
    say(f"[gpu] rda apply_G/apply_GH {shape} taps={taps} fc={params['fc']:.3g}")
    rg = rda.RdaGeometry(params, shape, taps)
    op = pk.make_operator(params, shape, chain="rda", taps=taps)
    x = inputs.random_complex(shape, seed=shape[0] + 3 * shape[1])
    y = inputs.random_complex(shape, seed=shape[0] + 5 * shape[1] + 1)
    gx = _h(op.apply_G(_d(x, dev)))
    my = _h(op.apply_GH(_d(y, dev)))
    e1, e2 = rel_l2(gx, rda.G(x, rg)), rel_l2(my, rda.M(y, rg))
    # Theorem 1 on the GPU's own results
    adj = abs(np.vdot(gx, y) - np.vdot(x, my)) / (np.linalg.norm(gx) * np.linalg.norm(y))
    say(f"    rel L2 G {e1:.2e} G^H {e2:.2e}; adjointness {adj:.2e}")
    assert e1 <= OP_TOL and e2 <= OP_TOL and adj <= OP_TOL


def test_rda_ita_matches_oracle(dev):
    import paper_1302_3120_amd as pk
    shape = (256, 256)
    say(f"[gpu] rda ITA {shape}, 20 targets, 50% mask, 10 iterations")
    rg = rda.RdaGeometry(STRIP, shape)
    rows, cols, sig = inputs.point_targets(shape, 20, seed=11)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, 0.5, seed=12)
    clean = rda.G(xt, rg)
    n = inputs.circular_noise(shape, 13)
    y = mask * (clean + 0.1 * np.sqrt(np.mean(np.abs(clean) ** 2)) * n)
    lam = ita.lambda_from_sparsity(y, mask, 20, rg)
    op = pk.make_operator(STRIP, shape, chain="rda")
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    x, res = op.ita_solve(_d(y, dev), bits, lam, 10, resid=True)
    wx, wres = ita.ita(y, mask, lam, 10, rg)
    e_x, e_r = rel_l2(_h(x), wx), rel_l2(res.cpu().numpy(), wres)
    xa, mu, lamh, _ = op.ita_solve_adaptive(_d(y, dev), bits, 20, 6)
    wxa, _, wmu, _ = ita.ita_adaptive(y, mask, 20, 6, rg)
    e_a = rel_l2(_h(xa), wxa)
    e_mu = np.max(np.abs(mu.cpu().numpy() - wmu) / np.abs(wmu))
    say(f"    fixed lambda: X {e_x:.2e} resid {e_r:.2e}; adaptive: X {e_a:.2e} mu {e_mu:.2e}")
    assert e_x <= IMG_TOL and e_r <= IMG_TOL and e_a <= IMG_TOL and e_mu <= 1e-5


def test_rda_at_4096_full_size(dev):
    # The 4096 x 4096 grid of the headline workload: M and G against the
    # full oracle chain (one application each on the host).
    import paper_1302_3120_amd as pk
    shape = (4096, 4096)
    say(f"[gpu] rda apply_G/apply_GH {shape} (oracle on the host)")
    rg = rda.RdaGeometry(STRIP, shape)
    op = pk.make_operator(STRIP, shape, chain="rda")
    x = inputs.random_complex(shape, seed=91)
    e1 = rel_l2(_h(op.apply_G(_d(x, dev))), rda.G(x, rg))
    e2 = rel_l2(_h(op.apply_GH(_d(x, dev))), rda.M(x, rg))
    say(f"    rel L2 G {e1:.2e} G^H {e2:.2e}")
    assert e1 <= OP_TOL and e2 <= OP_TOL


def test_rda_rejections(dev):
    import paper_1302_3120_amd as pk
    for taps in (0, 3, 34, -2):
        with pytest.raises(pk.CssarError):
            pk.make_operator(STRIP, (64, 64), chain="rda", taps=taps)
    with pytest.raises(pk.CssarError):  # migration beyond half the range extent
        pk.make_operator(STRESS, (64, 64), chain="rda")
    op = pk.make_operator(STRIP, (128, 128), chain="rda")
    with pytest.raises(pk.CssarError):
        pk.make_batch([op])
    y = _d(inputs.random_complex((128, 128), seed=1), dev)
    bits = op.pack_mask(torch.ones((128, 128), dtype=torch.bool, device=dev))
    with pytest.raises(pk.CssarError):
        op.ita_forward(y, bits, 0.1, 4, 2)
