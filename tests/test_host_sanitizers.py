"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The entry points' sources are compiled with the sanitizers on hipcc's host
pass only (-Xarch_host; the device code is unchanged), linked with the
in-tree kernel objects and the C driver tests/host/abi_driver.c, and run.  The driver exercises plan inspection,
the (K_a, K_r) parameterisation and the argument validation of every entry
point that answers without a GPU; any sanitizer report fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1302_3120_amd", "csrc")
HIPCC = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    import sys
    sys.path.insert(0, ROOT)
    from paper_1302_3120_amd import build as B
    # the kernel objects of the plans (their host part is the launch tables)
    # from the in-tree build; the entry points' sources with the sanitizers
    kobjs = [os.path.join(B.BUILD, f"kern_{n}_{v}.o") for n, v in B.PLANS]
    if not all(os.path.exists(o) for o in kobjs):
        B.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Wno-unused-command-line-argument", *san]
    jobs = [[HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", str(tmp_path / src.replace(".hip", ".o"))]
            for src in ("cssar_api.hip", "cssar_batch.hip", "cssar_grad.hip", "cssar_adaptive.hip",
                        "cssar_noalloc.hip")]
    procs = [subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for j in jobs]
    for p, j in zip(procs, jobs):
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, " ".join(j) + "\n" + out[-3000:]
    drv = tmp_path / "abi_driver.o"
    r = subprocess.run(["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
                        f"-I{os.path.join(ROOT, 'include')}", "-c",
                        os.path.join(ROOT, "tests", "host", "abi_driver.c"), "-o", str(drv)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = tmp_path / "abi_driver"
    objs = kobjs + [j[-1] for j in jobs] + [str(drv)]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address,undefined", *objs,
                        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
                        "-lm", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "all checks passed" in out
