"""Build liblrcc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2604_12914_amd.build      # or build() from Python

Every source under csrc/ is compiled to an object in csrc/_build/ (in
parallel) and linked into paper_2604_12914_amd/liblrcc.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblrcc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # keep packed-FP32 VALU instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, obj: str, extra=()) -> None:
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    noise = "is not a recognized feature for this target"
    for line in (r.stderr or "").splitlines():
        if line.strip() and noise not in line:
            print(line, file=sys.stderr)


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the debug
# library liblrcc_san.so (the device code is built as usual): the host
# validation paths of the C ABI run under it in the CPU tests, with the
# shared sanitizer runtime preloaded (SANITIZER_RUNTIME).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-O1"]
SAN_OUT = os.path.join(HERE, "liblrcc_san.so")
SANITIZER_RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def _link(objs, out, extra=()):
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def _objects(bdir, flags):
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(bdir, f[:-4] + ".o") for f in srcs]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(jobs, 1)) as ex:
        list(ex.map(lambda a: _compile(*a, extra=flags),
                    [(os.path.join(CSRC, s), o) for s, o in zip(srcs, objs)]))
    return objs


def build(verbose: bool = True, sanitized: bool = True) -> str:
    _link(_objects(os.path.join(CSRC, "_build"), []), OUT)
    if verbose:
        print(f"built {OUT}")
    if sanitized:
        _link(_objects(os.path.join(CSRC, "_build_san"), SAN_FLAGS), SAN_OUT,
              ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-shared-libsan"])
        if verbose:
            print(f"built {SAN_OUT}")
    return OUT


if __name__ == "__main__":
    build()
