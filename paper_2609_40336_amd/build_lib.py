"""Compile the HIP library liblrh.so for gfx950 (in-tree, next to this file).

Every translation unit under csrc/ is compiled to an object in parallel (the cluster kernel
families are split by precision and mode so that they do), then the objects are linked."""
import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
TARGET = os.path.join(HERE, "liblrh.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wno-unused-value",
    # packed FP32 instructions stay disabled for every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# the matrix-core kernels (scaling and squaring; the sustained-rate probe in lrh_kernels.hip) keep
# their results in ordinary VGPRs (the unified register file of gfx950): no copies through the
# accumulation registers between instructions
FILE_FLAGS = {f: ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
              for f in ("lrh_k_f32_gibbs.hip", "lrh_k_f64_gibbs.hip", "lrh_kernels.hip")}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="lrh_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + r.stdout[-4000:] + r.stderr[-8000:])
            return obj
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(compile_one, sources()))
        tmp = TARGET + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout[-4000:] + r.stderr[-8000:])
    os.replace(tmp, TARGET)
    return TARGET


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
