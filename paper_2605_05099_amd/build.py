"""Build the gfx950 HIP library paper_2605_05099_amd/librp.so with hipcc.

Every source in csrc/*.hip is compiled for gfx950 (objects in
paper_2605_05099_amd/_build/) and linked into one shared library exporting the
C ABI of include/rp.h.  Flags:
  -ffp-contract=off   no fused multiply-add: floating point is rounded exactly
                      as written (the serial definition is bit-reproducible)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep the compiler from emitting packed-FP32 instructions
Run: python -m paper_2605_05099_amd.build [--incremental]
(--incremental recompiles only objects older than their source or any csrc/
header).
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librp.so")
ARCH = os.environ.get("RP_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas"]


# per-source flags: the gradient kernels flush binary32 subnormals (their
# binary32 series run an order of magnitude slower on subnormal terms;
# binary64 keeps gradual underflow, and elements whose binary32 evaluation
# could meet a subnormal are evaluated in binary64)
EXTRA = {"k_grad.hip": ["-fgpu-flush-denormals-to-zero"]}


def hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _stale(src, obj):
    """An object is stale when it is missing or older than its source or any
    header or table in csrc/ (every .hip may include them)."""
    if not os.path.exists(obj):
        return True
    deps = [src] + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(CSRC, "*.inc"))
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and not _stale(src, obj):
        return obj, ""
    cmd = [hipcc(), *COMMON, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose=True, incremental=False):
    """Compiles every source (incremental=True: only stale objects) and links."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda s: _compile(s, incremental), srcs))
    for _, err in results:
        if err.strip() and verbose:
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *COMMON, "-shared", *[o for o, _ in results], "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
