"""GPU parity at the full sizes of the workloads, against stored oracle
results (tests/golden/*.npz, written by tests/golden/full_size.py, which
calls only the oracle and the input generators).

Each test rebuilds the workload's input y through the oracle's G (seeded
recipe), checks it against the digest stored with the golden, runs the HIP
solver through the C ABI and compares element by element on the sampled
columns: relative L2 <= 1e-4 on the final image (eq. (th2d), Algorithm 1)
and rtol 1e-4 on the residual norms.
"""

import os

import numpy as np
import pytest

from tests.golden import full_size as fs
from tests.helpers import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

IMG_TOL = 1e-4
RES_RTOL = 1e-4


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gold(name):
    p = fs.path(name)
    if not os.path.exists(p):
        pytest.fail(f"golden {p} missing: run python tests/golden/full_size.py {name}")
    return np.load(p, allow_pickle=False)


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


@pytest.fixture(scope="module")
def sparse_4096():
    say("[gpu] building the sparse_4096 input through the oracle's G")
    g, x, y, mask, k = fs.sparse_problem("sparse_4096")
    return y, mask, k


def _solve(dev, shape, y, mask, lam, iters):
    import paper_1302_3120_amd as pk
    op = pk.make_operator(fs.inputs.RADAR_STRIPMAP, shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    xg, hg = op.ita_solve(_d(y, dev), bits, lam, iters, resid=True)
    op.sync_status()
    return xg, hg.cpu().numpy().astype(np.float64)


def _compare(name, gold, xg, hg):
    cols = gold["cols"]
    xc = xg[:, torch.from_numpy(cols).to(xg.device)].cpu().numpy().astype(np.complex128)
    want = gold["x_cols"].astype(np.complex128)
    e = rel_l2(xc, want)
    worst = max(rel_l2(xc[:, i], want[:, i]) for i in range(len(cols)) if np.any(want[:, i]))
    say(f"    {name}: X sampled columns rel L2 {e:.2e} (worst column {worst:.2e}), "
        f"residual max rel {np.max(np.abs(hg - gold['resid']) / gold['resid']):.2e}")
    assert e <= IMG_TOL
    np.testing.assert_allclose(hg, gold["resid"], rtol=RES_RTOL)


def test_headline_4096_100_iterations_partial_mask(dev, sparse_4096):
    # The 4096 x 4096 headline workload (1 % log-normal field, 50 % mask,
    # 20 dB), 100 iterations with the sparsity-rule lambda: every residual
    # norm and 16 sampled columns of X(100), through the unsampled-entry
    # branch of the residual pass in every iteration.
    gold = _gold("sparse_4096_ita")
    y, mask, k = sparse_4096
    assert fs.check_digest(y, gold), "rebuilt y differs from the golden's input"
    say(f"[gpu] sparse_4096 ITA x{int(gold['iters'])} vs golden")
    xg, hg = _solve(dev, y.shape, y, mask, float(gold["lam"]), int(gold["iters"]))
    _compare("sparse_4096", gold, xg, hg)
    nnz = int(torch.count_nonzero(xg))
    say(f"    nonzeros {nnz} (oracle {int(gold['nnz'])})")
    assert abs(nnz - int(gold["nnz"])) <= max(50, int(gold["nnz"]) // 1000)


def test_adaptive_4096_five_iterations(dev, sparse_4096):
    # Section IV.B at full size: mu_t, lambda_t, the residuals and sampled
    # columns of X(5), k = the scene's nonzero count.
    gold = _gold("sparse_4096_adaptive")
    y, mask, k = sparse_4096
    assert fs.check_digest(y, gold)
    assert k == int(gold["k"])
    import paper_1302_3120_amd as pk
    say(f"[gpu] sparse_4096 adaptive x{int(gold['iters'])} vs golden")
    op = pk.make_operator(fs.inputs.RADAR_STRIPMAP, y.shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    xa, mu, lam, res = op.ita_solve_adaptive(_d(y, dev), bits, k, int(gold["iters"]))
    op.sync_status()
    mu = mu.cpu().numpy().astype(np.float64)
    lam = lam.cpu().numpy().astype(np.float64)
    res = res.cpu().numpy().astype(np.float64)
    say(f"    mu {mu.tolist()} oracle {gold['mu'].tolist()}")
    np.testing.assert_allclose(mu, gold["mu"], rtol=1e-5)
    np.testing.assert_allclose(lam, gold["lam"], rtol=1e-4)
    _compare("sparse_4096 adaptive", gold, xa, res)


def test_stripmap_2048_200_iterations(dev):
    # The 2048 x 2048 configuration (points + 2 % extended patches, 30 %
    # mask, 15 dB): all 200 residual norms and 16 sampled columns of X(200).
    gold = _gold("stripmap_2048_ita")
    say("[gpu] building the stripmap_2048 input through the oracle's G")
    g, x, y, mask, k = fs.stripmap_2048_problem()
    assert fs.check_digest(y, gold)
    say(f"[gpu] stripmap_2048 ITA x{int(gold['iters'])} vs golden")
    xg, hg = _solve(dev, y.shape, y, mask, float(gold["lam"]), int(gold["iters"]))
    _compare("stripmap_2048", gold, xg, hg)


def test_wide_swath_8192_three_iterations(dev):
    # The 8192 x 8192 wide-swath configuration with its 50 % mask: three
    # iterations (G, the residual pass on 8192-point columns and the split
    # 8192 row plan inside iterations 2 and 3), sampled columns of X(3).
    gold = _gold("sparse_8192_ita")
    say("[gpu] building the sparse_8192 input through the oracle's G")
    g, x, y, mask, k = fs.sparse_problem("sparse_8192")
    del x
    assert fs.check_digest(y, gold)
    say(f"[gpu] sparse_8192 ITA x{int(gold['iters'])} vs golden")
    xg, hg = _solve(dev, y.shape, y, mask, float(gold["lam"]), int(gold["iters"]))
    del y
    _compare("sparse_8192", gold, xg, hg)
