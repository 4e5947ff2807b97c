"""Build libdmul.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdmul.so")
# the same sources with primes below 2^62 and redundant-range butterflies
LIB_LAZY = os.path.join(HERE, "libdmul_lazy.so")
SOURCES = ["api.hip", "batch.hip", "ntt.hip", "carry.hip", "small.hip", "transpose.hip"]
HEADERS = ["field.hpp", "internal.hpp", "ctx.hpp", "batch.hpp", "ntt_dev.hpp", "rec_dev.hpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed-FP32 instructions are never wanted in this integer code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "dmul.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False) -> str:
    """Compiles every source to an object (in parallel), once for each
    library, then links them: libdmul.so and libdmul_lazy.so."""
    import concurrent.futures
    import tempfile
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    libs = ((LIB, []), (LIB_LAZY, ["-DDMUL_LAZY_FIELD=1"]))
    with tempfile.TemporaryDirectory(prefix="dmul_build_") as tmpdir:
        def compile_one(job):
            li, src = job
            obj = os.path.join(tmpdir, f"{li}_{os.path.basename(src)}.o")
            cmd = [hipcc()] + compile_flags + libs[li][1] + inc + ["-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
            return obj
        jobs = [(li, src) for li in range(len(libs)) for src in sources()]
        workers = max(1, min(len(jobs), os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            objs = list(ex.map(compile_one, jobs))
        for li, (path, _) in enumerate(libs):
            tmp = path + ".tmp"
            mine = [o for (lj, _), o in zip(jobs, objs) if lj == li]
            cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + mine
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
            os.replace(tmp, path)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
