"""Compile the HIP sources of the library for gfx950 into lib/libibfsi.so.

Each source is compiled to an object in parallel, then linked.  The flags disable
packed FP32 instructions (-packed-fp32-ops) for all device code.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["ib_flow.hip", "ib_flow_tuned.hip", "ib_flow_multi.hip", "ib_flow_multi_tuned.hip", "ib_body.hip", "ib_engine.hip", "ib_serve.hip", "ib_gemm.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose=False):
    out_dir = os.path.join(HERE, "lib")
    os.makedirs(out_dir, exist_ok=True)
    target = os.path.join(out_dir, "libibfsi.so")
    with tempfile.TemporaryDirectory() as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC] + FLAGS + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, r
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for src, _, r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            if verbose:
                sys.stderr.write(r.stderr)
        tmp_target = target + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_target] + \
              [obj for _, obj, _ in results]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError("link failed")
        os.replace(tmp_target, target)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
