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
SOURCES = ["kernels.hip", "api.cpp", "backtrack.cpp"]


# Kernels that run a whole search in one persistent launch.
SEARCH_KERNELS = ("solve_kernel", "queue_kernel")


def check_no_scratch(remarks: str) -> None:
    """The persistent search kernels must keep every value in registers or
    LDS (a build whose search kernels use scratch memory is rejected): their
    register budget is chosen for a number of resident waves, and a variant
    that spilled gave run-to-run different trees."""
    current = None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            current = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and current and any(k in current for k in SEARCH_KERNELS) and int(m.group(1)) != 0:
            raise RuntimeError(f"{current} uses {m.group(1)} bytes of scratch per lane")


# FP64 instructions whose result depends on the rounding mode.  In kernels
# that run with the FP64 rounding field set toward -infinity, each of them
# must come from the hand-written one-instruction statements (inline
# assembly), never from the compiler, which assumes round-to-nearest.
_ROUNDED_F64 = re.compile(r"^v_(add|sub|subrev|mul|fma|fmac|div_scale|div_fmas|div_fixup|ldexp|sqrt|rsq|"
                          r"fract|trig_preop|frexp_mant)_f64")
# Packed FP32 arithmetic is not used anywhere.
_PACKED_F32 = re.compile(r"^v_pk_(add|mul|fma)_f32")
_MODE_WRITE = re.compile(r"^s_(setreg|setreg_imm32|round_mode|denorm_mode)")


def check_isa(asm: str) -> None:
    """Checks the device assembly of kernels.hip:

    * every kernel that sets the FP64 rounding field has exactly that one
      MODE write (inline assembly at entry) and no other, so the mode holds
      for the whole kernel;
    * such kernels contain no compiler-generated rounding-dependent FP64
      instruction (exact conversions, compares, min/max and the reciprocal
      seed of the directed division, which exact residual tests correct,
      are allowed);
    * no kernel uses packed FP32 arithmetic.
    """
    fn = None
    in_asm = False
    funcs = {}
    for raw in asm.splitlines():
        m = re.match(r"^([A-Za-z_][\w.$]*):", raw)
        if m and not raw.startswith("."):
            fn = m.group(1)
            funcs.setdefault(fn, {"mode_asm": 0, "mode_cc": 0, "f64_cc": [], "pk": []})
            continue
        if "ASMSTART" in raw:
            in_asm = True
            continue
        if "ASMEND" in raw:
            in_asm = False
            continue
        line = raw.strip()
        if fn is None or not line or line[0] in ";." or line.endswith(":"):
            continue
        op = line.split()[0]
        f = funcs[fn]
        if _MODE_WRITE.match(op):
            f["mode_asm" if in_asm else "mode_cc"] += 1
        elif _ROUNDED_F64.match(op) and not in_asm:
            f["f64_cc"].append(line)
        if _PACKED_F32.match(op):
            f["pk"].append(line)
    for name, f in funcs.items():
        if f["pk"]:
            raise RuntimeError(f"{name} uses packed FP32 arithmetic: {f['pk'][0]}")
        if f["mode_asm"] == 0 and f["mode_cc"] == 0:
            continue
        if f["mode_cc"] or f["mode_asm"] != 1:
            raise RuntimeError(f"{name} writes the MODE register {f['mode_asm']} + {f['mode_cc']} times")
        if f["f64_cc"]:
            raise RuntimeError(f"{name} has compiler-generated rounded FP64 arithmetic: {f['f64_cc'][0]}")


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
            # the device assembly is kept (for check_isa) beside the object
            cmd += ["-Rpass-analysis=kernel-resource-usage", "-save-temps=obj"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        text = res.stdout + res.stderr
        out = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and "remark:" not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if not src.endswith(".cpp"):
            check_no_scratch(text)
            stem = os.path.splitext(src)[0]
            with open(os.path.join(build_dir, f"{stem}-hip-amdgcn-amd-amdhsa-gfx950.s")) as f:
                check_isa(f.read())
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
