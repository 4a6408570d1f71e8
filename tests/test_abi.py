"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cssar.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(cssar_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1302_3120_amd import cssar
    if not os.path.exists(cssar.LIB_PATH):
        pytest.fail("libcssar.so is not built (run __graft_entry__.build())")
    return cssar.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "cssar_ita_solve" in names and "cssar_apply_G" in names
    for n in names:
        assert hasattr(L, n), n


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "cssar.h"\nint main(void){cssar_params p={0};(void)p;return 0;}\n')
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                        "-c", str(src), "-o", str(tmp_path / "t.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_supported_lengths_and_plans(L):
    from paper_1302_3120_amd import cssar
    for n in (64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096, 8192):
        assert cssar.supported_length(n)
        e, radices = cssar.plan_info(n)
        prod = 1
        for r in radices:
            prod *= r
            assert e % r == 0
        assert prod == n
    for n in (0, 1, 100, 1000, 1536 * 3, 16384, -4):
        assert not cssar.supported_length(n)
    with pytest.raises(cssar.CssarError) as ei:
        cssar.plan_info(1000)
    assert ei.value.code == cssar.EUNSUPPORTED


def _params(**kw):
    import inputs
    from paper_1302_3120_amd import cssar
    d = dict(inputs.RADAR_STRIPMAP)
    d.update(kw)
    return cssar.Params.from_dict(d)


@pytest.mark.parametrize("kw,shape,code", [
    (dict(fc=0.0), (256, 256), -1),
    (dict(v=-1.0), (256, 256), -1),
    (dict(prf=float("nan")), (256, 256), -1),
    (dict(f_dc=5.0), (256, 256), -2),
    (dict(prf=1e9), (256, 256), -1),          # Doppler beyond the migration singularity
    ({}, (0, 256), -1),
    ({}, (256, -8), -1),
    ({}, (1000, 256), -2),
    ({}, (256, 1000), -2),
    ({}, (256, 100), -2),
])
def test_make_operator_rejects_before_any_hip_call(L, kw, shape, code):
    p = _params(**kw)
    h = ctypes.c_void_p()
    rc = L.cssar_make_operator(ctypes.byref(p), shape[0], shape[1], ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert len(L.cssar_last_error()) > 0


@pytest.mark.parametrize("taps", [0, 3, 34, -2])
def test_make_operator_rda_rejects_taps_before_any_hip_call(L, taps):
    p = _params()
    h = ctypes.c_void_p()
    assert L.cssar_make_operator_rda(ctypes.byref(p), 256, 256, taps, ctypes.byref(h)) == -1
    assert h.value is None


def test_null_arguments(L):
    h = ctypes.c_void_p()
    assert L.cssar_make_operator(None, 256, 256, ctypes.byref(h)) == -1
    p = _params()
    assert L.cssar_make_operator(ctypes.byref(p), 256, 256, None) == -1
    assert L.cssar_apply_G(None, None, None, None, None) == -1
    assert L.cssar_apply_GH(None, None, None, None, None) == -1
    assert L.cssar_ita_solve(None, None, None, 0.1, 10, None, None, None, None) == -1
    assert L.cssar_ita_solve_adaptive(None, None, None, 10, 10, None, None, None, None, None,
                                      None) == -1
    assert L.cssar_ita_solve_safeguarded(None, None, None, 10, 10, 0.01, 2.0, 2, None, None, None,
                                         None, None, None, None) == -1
    assert L.cssar_workspace_size(None, 3) == 0
    assert L.cssar_workspace_size(None, 2) == 0
    assert L.cssar_make_operator_rda(None, 256, 256, 8, ctypes.byref(h)) == -1
    assert L.cssar_make_operator_rda(ctypes.byref(p), 256, 256, 8, None) == -1
    assert L.cssar_operator_chain(None) == -1
    assert L.cssar_pack_mask(None, None, None, None) == -1
    assert L.cssar_sync_status(None, None) == -1
    assert L.cssar_destroy_operator(None) == 0
    assert L.cssar_workspace_size(None, 1) == 0
    # batch entry points
    hb = ctypes.c_void_p()
    assert L.cssar_make_batch(None, 1, ctypes.byref(hb)) == -1
    ops = (ctypes.c_void_p * 2)(None, None)
    assert L.cssar_make_batch(ops, 2, ctypes.byref(hb)) == -1
    assert L.cssar_make_batch(ops, 0, ctypes.byref(hb)) == -1
    assert L.cssar_make_batch(ops, 2, None) == -1
    assert hb.value is None
    assert L.cssar_destroy_batch(None) == 0
    assert L.cssar_batch_workspace_size(None) == 0
    assert L.cssar_batch_set_graph(None, 1) == -1
    assert L.cssar_batch_autotune(None, None, None, None) == -1
    assert L.cssar_batch_describe(None, None, 0) == -1
    assert L.cssar_ita_solve_batched(None, None, None, None, 3, None, None, None) == -1
    # gradient entry points
    assert L.cssar_checkpoint_size(None, 10, 5) == 0
    assert L.cssar_grad_workspace_size(None, 5) == 0
    assert L.cssar_ita_forward(None, None, None, 0.1, 10, 5, None, None, None, None) == -1
    assert L.cssar_ita_backward(None, None, None, 0.1, 10, 5, None, None, None, None, None, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    from paper_1302_3120_amd import cssar
    op = cssar.Operator.__new__(cssar.Operator)
    op.shape = (64, 64)
    with pytest.raises(ValueError):
        op._arr(torch.zeros(64, 64, dtype=torch.complex64), "x")
    with pytest.raises(TypeError):
        op._arr(torch.zeros(64, 64, dtype=torch.complex128), "x")


def test_rate_parameterisation_round_trip(L):
    # cssar_azimuth_fm_rate / cssar_params_with_rates (host calls): K_a =
    # 2 v^2 / (lambda_w r_ref) and its inverse, against the oracle's geometry
    import inputs
    from oracle import csa
    from paper_1302_3120_amd import cssar
    P = inputs.RADAR_STRIPMAP
    ka = cssar.ka_of(P)
    g = csa.Geometry(P, (64, 64))
    assert abs(ka - 2.0 * P["v"] ** 2 / (g.lam * P["r_ref"])) <= 1e-12 * ka
    q = cssar.params_with_theta(P, 1.1 * ka, 0.9 * P["Kr"])
    assert abs(cssar.ka_of(q) - 1.1 * ka) <= 1e-12 * ka
    assert q["Kr"] == 0.9 * P["Kr"]
    assert abs(q["v"] - P["v"] * 1.1 ** 0.5) <= 1e-12 * P["v"]
    for k in ("fc", "fs", "prf", "r_ref"):
        assert q[k] == P[k]
    for bad in ((0.0, P["Kr"]), (ka, -1.0), (float("nan"), P["Kr"]), (ka, float("inf"))):
        with pytest.raises(cssar.CssarError) as ei:
            cssar.params_with_theta(P, *bad)
        assert ei.value.code == cssar.EINVAL
