"""Build libcssar.so for gfx950 with hipcc (in-tree).

The pass kernels of every compiled plan (supported line length and plan
variant) are compiled from one source (csrc/kern_inst.hip) with different
CSSAR_N / CSSAR_V, in parallel, then linked with the C-ABI objects
(csrc/cssar_api.hip, csrc/cssar_batch.hip, csrc/cssar_grad.hip,
csrc/cssar_adaptive.hip) into
paper_1302_3120_amd/libcssar.so.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcssar.so")
LENGTHS = (64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096, 8192)
# (length, variant) pairs: every length has variant 0; these also have 1
VARIANT1 = (512, 1024, 1536, 2048, 4096, 8192)
VARIANT2 = (4096,)
PLANS = (tuple((n, 0) for n in LENGTHS) + tuple((n, 1) for n in VARIANT1) +
         tuple((n, 2) for n in VARIANT2))
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


ROCM_LIB = "/opt/rocm/lib"


def common_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # no packed FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build(jobs=None, verbose=False, report=False):
    """Compile every kernel object and link the shared library.  Always
    rebuilds.  Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    flags = common_flags()
    extra = ["-Rpass-analysis=kernel-resource-usage"] if report else []
    cmds = []
    for n, v in PLANS:
        obj = os.path.join(BUILD, f"kern_{n}_{v}.o")
        cmds.append([cc, *flags, *extra, f"-DCSSAR_N={n}", f"-DCSSAR_V={v}", "-c",
                     os.path.join(CSRC, "kern_inst.hip"), "-o", obj])
    for src in ("cssar_api.hip", "cssar_batch.hip", "cssar_grad.hip", "cssar_adaptive.hip",
                "cssar_noalloc.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmds.append([cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    outs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            outs.append(out)
    if verbose or report:
        print("\n".join(o for o in outs if o.strip()))
    objs = [c[-1] for c in cmds]
    tmp = LIB + ".tmp"
    # roctx: the named host ranges of the entry points and pass launches
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, f"-L{ROCM_LIB}",
          "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    report = "--report" in sys.argv
    print(build(verbose=True, report=report))
