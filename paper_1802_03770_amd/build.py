"""Build the HIP library libfraclap.so for gfx950 in-tree (hipcc, no JIT cache).

The library is split into translation units compiled in parallel: the host
driver and C ABI, and the operator-application and preconditioner launch
sequences once per precision (explicit template instantiations).
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfraclap.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep hipcc from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-Wno-unused-value", "-Wno-unused-result",
]
UNITS = [
    ("fl_host.hip", []),
    ("fl_apply.hip", ["-DFL_T=float"]),
    ("fl_apply.hip", ["-DFL_T=double"]),
    ("fl_precond.hip", ["-DFL_T=float"]),
    ("fl_precond.hip", ["-DFL_T=double"]),
    ("fl_batch.hip", ["-DFL_T=float"]),
    ("fl_batch.hip", ["-DFL_T=double"]),
    ("fl_batch.hip", ["-DFL_BATCH_HOST"]),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    return r


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmpdir = tempfile.mkdtemp(prefix="fraclap_build_")
    cmds = []
    for i, (src, defs) in enumerate(UNITS):
        obj = os.path.join(tmpdir, f"u{i}.o")
        cmds.append((obj, [hipcc] + FLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", obj]))
    if verbose:
        for _, c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 4)) as ex:
        list(ex.map(lambda oc: _run(oc[1]), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in cmds] + ["-o", tmp])
    os.replace(tmp, LIB)
    for o, _ in cmds:
        os.remove(o)
    os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
