"""Build the HIP library libfraclap.so for gfx950 in-tree (hipcc, no JIT cache).

The library is split into translation units compiled in parallel: the host
driver and C ABI, and the operator-application and preconditioner launch
sequences once per precision (explicit template instantiations).
"""
import hashlib
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
    ("fl_net.hip", []),
    ("fl_capacity.hip", []),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    return r


def _unit_key(src, defs):
    h = hashlib.sha1()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hpp") or name == src:
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    with open(os.path.join(ROOT, "include", "fraclap.h"), "rb") as f:
        h.update(f.read())
    h.update(" ".join(FLAGS + defs).encode())
    return h.hexdigest()[:16]


def build(verbose=False, jobs=None, reuse=False):
    """Compile every unit and link the library.  reuse=True (development
    only) keeps objects in _build/ and recompiles only units whose sources or
    headers changed."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmpdir = tempfile.mkdtemp(prefix="fraclap_build_")
    cache = os.path.join(HERE, "_build")
    cmds, objs = [], []
    for i, (src, defs) in enumerate(UNITS):
        if reuse:
            os.makedirs(cache, exist_ok=True)
            obj = os.path.join(cache, f"{os.path.splitext(src)[0]}_{_unit_key(src, defs)}.o")
            objs.append(obj)
            if os.path.exists(obj):
                continue
        else:
            obj = os.path.join(tmpdir, f"u{i}.o")
            objs.append(obj)
        cmds.append((obj, [hipcc] + FLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", obj + ".part"]))
    if verbose:
        for _, c in cmds:
            print(" ".join(c), flush=True)
    if cmds:
        with ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 4)) as ex:
            list(ex.map(lambda oc: (_run(oc[1]), os.replace(oc[0] + ".part", oc[0])), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    if not reuse:
        for o in objs:
            os.remove(o)
    os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
