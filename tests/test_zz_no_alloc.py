"""The allocation-free solver entry point (cssar_ita_solve_static: the
workspace is the library's fixed device array) against cssar_ita_solve with
a caller workspace, through the C ABI: the same kernels on the same inputs,
so the results must be equal bit for bit, on two calls in a row (the second
smaller, over the contents the first left in the array), and a solve larger
than the array is refused before any launch."""

import ctypes

import numpy as np
import pytest

import inputs
from tests.helpers import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = inputs.RADAR_STRIPMAP


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _static_fn():
    from paper_1302_3120_amd import cssar
    f = cssar.lib().cssar_ita_solve_static
    vp = ctypes.c_void_p
    f.argtypes = [vp, vp, vp, ctypes.c_float, ctypes.c_int, vp, vp, vp]
    f.restype = ctypes.c_int
    return f


def _problem(shape, seed, dev):
    y = inputs.random_complex(shape, seed=seed)
    mask = inputs.random_mask(shape, 0.5, seed=seed + 1)
    ym = torch.from_numpy(np.where(mask, y, 0).astype(np.complex64)).to(dev)
    return ym, torch.from_numpy(mask).to(dev)


def test_static_workspace_equals_caller_workspace(dev):
    import paper_1302_3120_amd as pk
    from paper_1302_3120_amd import cssar
    f = _static_fn()
    iters = 6
    for shape, seed, lam in (((1024, 1536), 71, 0.9), ((512, 256), 73, 0.7)):
        say(f"[gpu] cssar_ita_solve_static {shape} x{iters} vs cssar_ita_solve")
        op = pk.make_operator(P, shape)
        assert op.workspace_size(1) <= (64 << 20)
        y, m = _problem(shape, seed, dev)
        bits = op.pack_mask(m)
        want, hw = op.ita_solve(y, bits, lam, iters, resid=True)
        out = torch.empty_like(y)
        hist = torch.empty(iters, dtype=torch.float32, device=dev)
        rc = f(op.handle, y.data_ptr(), bits.data_ptr(), lam, iters, out.data_ptr(), hist.data_ptr(),
               cssar._stream())
        assert rc == 0, cssar.lib().cssar_last_error()
        torch.cuda.synchronize()
        op.sync_status()
        nz = int(torch.count_nonzero(out))
        say(f"    equal image {torch.equal(out, want)} residuals {torch.equal(hist, hw)} nonzeros {nz}")
        assert nz > 0
        assert torch.equal(out, want) and torch.equal(hist, hw)


def test_static_workspace_refuses_larger_solves(dev):
    import paper_1302_3120_amd as pk
    from paper_1302_3120_amd import cssar
    f = _static_fn()
    shape = (2048, 2048)
    op = pk.make_operator(P, shape)
    assert op.workspace_size(1) > (64 << 20)
    y = torch.zeros(shape, dtype=torch.complex64, device=dev)
    bits = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    out = torch.empty_like(y)
    rc = f(op.handle, y.data_ptr(), bits.data_ptr(), 0.5, 2, out.data_ptr(), None, cssar._stream())
    msg = cssar.lib().cssar_last_error().decode()
    say(f"    {shape}: rc {rc}: {msg}")
    assert rc == cssar.EINVAL and "static workspace" in msg
