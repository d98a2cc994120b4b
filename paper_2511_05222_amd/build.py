"""Build the HIP library libvmcx.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvmcx.so")
SOURCES = ["vmc_abi.hip", "vmc_pipeline.hip", "vmc_mo.hip", "vmc_adjoint.hip", "vmc_dense.hip", "vmc_sweep.hip", "vmc_reduce.hip", "vmc_jastrow.hip", "vmc_ecp.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def build(verbose=False, jobs=None):
    """Compile every source (in parallel, one hipcc per source) and link."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    objs = [os.path.join(tmp, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(i):
        cmd = [hipcc, *[f for f in HIPCC_FLAGS if f != "-shared"], "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(compile_one, i) for i in range(len(SOURCES))]:
            f.result()
    out_tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
