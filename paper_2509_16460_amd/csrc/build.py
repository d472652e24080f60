"""Build libpwdf.so for gfx950 with hipcc (in-tree, next to the Python binding)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libpwdf.so")
SOURCES = ["capi.cpp", "plan.cpp", "kernels_fp64.hip", "kernels_fp32.hip", "kernels_head.hip", "kernels_grad.hip", "kernels_cd.hip", "kernels_gpw.hip", "static_ws.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # packed FP32 instructions stay off (hipcc emits them from scalar float code otherwise)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]

# The MFMA kernels keep their accumulators in VGPRs (the MFMA's C/D operands in
# the VGPR form): with AGPR operands the register allocator moved every
# accumulator between a single AGPR tile and VGPRs around each MFMA in several of
# their instances, which also exposed each MFMA's full latency.
MFMA_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
MFMA_SOURCES = {"kernels_fp32.hip", "kernels_head.hip"}


def build(jobs: int = 8) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + (MFMA_FLAGS if src in MFMA_SOURCES else []) + ["-c", os.path.join(HERE, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        if pr.returncode != 0:
            failed.append((src, text))
        elif "error" in text.lower():
            sys.stderr.write(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"---- {src}\n{text}\n")
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
