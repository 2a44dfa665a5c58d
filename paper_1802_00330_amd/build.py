"""Build step of the HIP library: compiles csrc/*.hip and csrc/*.cpp with hipcc
for gfx950 into libibb.so next to this file."""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libibb.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no contraction into fused multiply-adds, IEEE single-precision denormals
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
]
SOURCES = ["kernels.hip", "api.cpp"]


def check_no_scratch(remarks: str) -> None:
    """The persistent search kernels must keep every value in registers or
    LDS: a variant that spilled to scratch memory gave run-to-run different
    trees, so a build whose search kernels use scratch is rejected."""
    current = None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            current = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and current and "solve_kernel" in current and int(m.group(1)) != 0:
            raise RuntimeError(f"{current} uses {m.group(1)} bytes of scratch per lane")


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link libibb.so."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        else:
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        res = subprocess.run(cmd, capture_output=True, text=True)
        text = res.stdout + res.stderr
        out = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and "remark:" not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if not src.endswith(".cpp"):
            check_no_scratch(text)
        if verbose and out.strip():
            print(out, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
