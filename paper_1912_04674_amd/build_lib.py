"""Build libenvpic.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1912_04674_amd.build_lib

Objects go to paper_1912_04674_amd/_build/, the library next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libenvpic.so")
SOURCES = ["particles.hip", "grid.hip", "sort_diag.hip", "beam.hip", "bunch.hip", "api.hip", "copy.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, csrc=CSRC, out=LIB, build_dir=BUILD, defines=()):
    """Compile the sources of `csrc` into the shared library `out` (by
    default the package's own sources and library); `defines` are extra
    -D options."""
    os.makedirs(build_dir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, *(f"-D{d}" for d in defines), "-I", os.path.join(HERE, "..", "include"), "-c",
               os.path.join(csrc, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        log, _ = pr.communicate()
        text = log.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 target feature
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if pr.returncode != 0:
            failed.append(src)
            sys.stderr.write(f"[build] {src} failed:\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write(f"[build] {src}:\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = out + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
