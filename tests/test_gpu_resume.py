"""GPU tests of cssar_ita_solve_ex: warm start (Algorithm 1 from a given
X^(0)) and the per-iteration ||X^(t+1)||_1 and nonzero counts.

Bars: a solve split as n1 + n2 iterations equals the n1 + n2 solve bit for
bit (image and residual norms); against the FP64 oracle, relative L2 <= 1e-4
on the image, rtol 1e-4 on residual norms and l1 norms, and nonzero counts
within a few pixels (the FP32 and FP64 thresholds may decide pixels within
rounding of sigma differently)."""

import numpy as np
import pytest

import inputs
from oracle import csa, ita
from tests.helpers import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = inputs.RADAR_STRIPMAP


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _h(t):
    return t.cpu().numpy().astype(np.complex128)


def _gpu_problem(shape, seed, dev):
    """A 1 % sparse log-normal scene, 50 % mask, y = m o (G x + n) at 20 dB
    through the GPU operator, lambda by the sparsity rule."""
    import paper_1302_3120_amd as pk
    op = pk.make_operator(P, shape)
    x = inputs.sparse_field(shape, 0.01, seed)
    k = int(np.count_nonzero(x))
    mask = inputs.random_mask(shape, 0.5, seed + 1)
    md = torch.from_numpy(mask).to(dev)
    clean = op.apply_G(_d(x, dev))
    s = float((clean.abs() ** 2)[md].mean() / 100.0) ** 0.5
    n = _d(inputs.circular_noise(shape, seed + 2), dev)
    y = torch.where(md, clean + s * n, torch.zeros_like(clean))
    lam = float(torch.topk(op.apply_GH(y).abs().flatten(), k + 1).values[-1])
    return op, y, op.pack_mask(md), lam


@pytest.mark.parametrize("shape,n1,n2", [((512, 1024), 3, 4), ((4096, 512), 5, 5),
                                         ((2048, 256), 1, 6), ((8192, 64), 2, 3),
                                         ((4096, 4096), 50, 50)])
def test_split_solve_equals_whole_solve(dev, shape, n1, n2):
    say(f"[gpu] warm start {shape}: {n1} + {n2} iterations vs {n1 + n2}")
    op, y, bits, lam = _gpu_problem(shape, 31, dev)
    xw, hw, lw, nw = op.ita_solve_ex(y, bits, lam, n1 + n2)
    x1, h1, l1, c1 = op.ita_solve_ex(y, bits, lam, n1)
    x2, h2, l2, c2 = op.ita_solve_ex(y, bits, lam, n2, x0=x1)
    op.sync_status()
    say(f"    nonzeros {int(nw[-1])}, equal image {torch.equal(x2, xw)}")
    assert torch.equal(x2, xw)
    assert torch.equal(torch.cat([h1, h2]), hw)
    # (the last iterate of a solve is totalled from the image, the others from
    # the sparse iterate: the same FP64 terms in another order)
    assert torch.equal(torch.cat([c1, c2]), nw)
    torch.testing.assert_close(torch.cat([l1, l2]), lw, rtol=1e-6, atol=0.0)
    # the plain entry point gives the same image and residuals
    xp, hp = op.ita_solve(y, bits, lam, n1 + n2, resid=True)
    assert torch.equal(xp, xw) and torch.equal(hp, hw)
    # metrics of the last iterate are those of the returned image
    xa = _h(xw)
    assert int(nw[-1]) == np.count_nonzero(xa)
    assert abs(float(lw[-1]) - np.abs(xa).sum()) <= 1e-5 * np.abs(xa).sum()


def test_metrics_and_warm_start_match_oracle(dev):
    import paper_1302_3120_amd as pk
    shape = (256, 512)
    say(f"[gpu] per-iteration l1 / nnz and a warm start vs oracle {shape}")
    g = csa.Geometry(P, shape)
    mask = inputs.random_mask(shape, 0.5, seed=41)
    y = np.where(mask, csa.G(inputs.sparse_field(shape, 0.02, 40), g), 0)
    lam = 0.02
    op = pk.make_operator(P, shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    tr = {}
    xo, ho = ita.ita(y, mask, lam, 8, g, trace=tr)
    xg, hg, lg, ng = op.ita_solve_ex(_d(y, dev), bits, lam, 8)
    op.sync_status()
    e = rel_l2(_h(xg), xo)
    lg, ng = lg.cpu().numpy(), ng.cpu().numpy()
    say(f"    image rel L2 {e:.2e}; l1 {lg[-1]:.6g} (oracle {tr['l1'][-1]:.6g}); "
        f"nnz {ng.tolist()} (oracle {tr['nnz']})")
    assert e <= 1e-4
    np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-4)
    np.testing.assert_allclose(lg, tr["l1"], rtol=1e-4)
    assert np.all(np.abs(ng - np.array(tr["nnz"])) <= 3)
    # warm start from a given iterate: a dense one (every element nonzero,
    # so every thread of the update pass stores its values densely), and the
    # oracle's X^(3) (sparse)
    for tag, x0 in (("dense", inputs.random_complex(shape, seed=42, scale=0.1)),
                    ("sparse", ita.ita(y, mask, lam, 3, g)[0])):
        xo, ho = ita.ita(y, mask, lam, 4, g, x0=x0)
        xg, hg, _, _ = op.ita_solve_ex(_d(y, dev), bits, lam, 4, x0=_d(x0, dev))
        op.sync_status()
        e = rel_l2(_h(xg), xo)
        say(f"    from a {tag} X(0): image rel L2 {e:.2e}")
        assert e <= 1e-4
        np.testing.assert_allclose(hg.cpu().numpy(), ho, rtol=1e-4)


def test_warm_start_rejects_aliasing(dev):
    import paper_1302_3120_amd as pk
    shape = (256, 256)
    op = pk.make_operator(P, shape)
    y = torch.zeros(shape, dtype=torch.complex64, device=dev)
    bits = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    with pytest.raises(pk.CssarError):
        op.ita_solve_ex(y, bits, 0.1, 2, x0=y)
    x, h, l1, nnz = op.ita_solve_ex(y, bits, 0.1, 2)
    assert float(x.abs().max()) == 0.0 and int(nnz.abs().max()) == 0 and float(l1.abs().max()) == 0.0
