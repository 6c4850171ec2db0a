"""Build libbfpfft.so (gfx950) in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled (-Xclang -target-feature -Xclang
-packed-fp32-ops) and default denormal handling (FP16 subnormals matter for
the 2^-log2N prescale).  Objects go to ``_build/``; the library lands next to
this file as ``libbfpfft.so``.  Run ``python -m paper_2605_28451_amd.build_lib``.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbfpfft.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Wall", "-Wno-unused-function"]
# -packed-fp32-ops: no v_pk_*_f32 selection.  -dot5-insts: select the VOP3P
# v_dot2_f32_f16 (inline zero accumulator) instead of the VOP2 v_dot2c form,
# which needs a register copy per product.  amdgpu-mfma-vgpr-form: MFMA
# accumulators in VGPRs (no accvgpr moves).
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xclang", "-target-feature", "-Xclang", "-dot5-insts",
          "-mllvm", "-amdgpu-mfma-vgpr-form"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]

# (source, object name, extra defines, is_device)
UNITS = [("rows.hip", f"rows_m{m}.o", [f"-DBFP_MODE_ID={m}"], True) for m in range(6)] + [
    ("uneven.hip", f"uneven_m{m}.o", [f"-DBFP_MODE_ID={m}"], True) for m in range(6)] + [
    ("dispatch.hip", "dispatch.o", [], True),
    ("sar.hip", "sar.o", [], True),
    ("autofocus.hip", "autofocus.o", [], True),
    ("api.cpp", "api.o", [], False),
    ("uneven_api.cpp", "uneven_api.o", [], False),
    ("host_tables.cpp", "host_tables.o", [], False),
]


def _headers():
    return [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + \
        [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]


def _compile(unit, force):
    src, obj, defs, dev = unit
    srcp = os.path.join(CSRC, src)
    objp = os.path.join(BUILD, obj)
    if not force and os.path.exists(objp):
        newest = max([os.path.getmtime(srcp)] + [os.path.getmtime(h) for h in _headers()])
        if os.path.getmtime(objp) >= newest:
            return objp, ""
    cmd = [HIPCC] + (DEVICE if dev else HOST) + COMMON + defs + ["-c", srcp, "-o", objp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32-ops feature: harmless
    err = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and "dot5-insts" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return objp, err


def build(force: bool = True, jobs: int = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, force), UNITS))
    for _, err in results:
        if err.strip():
            sys.stderr.write(err + "\n")
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv))
