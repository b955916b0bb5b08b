"""Build librve.so for gfx950 with hipcc (in-tree, no JIT cache): every source is
compiled to an object in parallel, then linked."""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/rve.hip", "csrc/passes.hip", "csrc/xpass.hip", "csrc/zfused.hip",
           "csrc/spectral.hip", "csrc/voxel.hip", "csrc/vector.hip", "csrc/macro.hip",
           "csrc/gmres.hip", "csrc/pfdir.hip", "csrc/finite.hip"]
FLAGS = ["-O3", "-std=c++20", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stderr[-4000:])


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = os.path.join(HERE, "librve.so")
    tmp = out + ".tmp"
    with tempfile.TemporaryDirectory(prefix="rve_build_") as d:
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[hipcc] + FLAGS + ["-c", os.path.join(HERE, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            list(ex.map(_run, cmds))
        _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
