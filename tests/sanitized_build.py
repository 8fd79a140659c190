"""Builds the library with its host code (the .cpp sources: plan lowering,
planner, variant space and search, cost-model host logic, batch set-up,
run-time source generation) instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer, into _build_san/libhawk_san.so. The device code
objects are those of the regular build (paper_1709_00700_amd/build.py); the
sanitizers apply to host code only. Test infrastructure: loaded by
tests/test_library_sanitized.py through HAWK_LIBRARY, in a process started
with clang's ASan runtime preloaded."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

from paper_1709_00700_amd import build as hb

OUT = os.path.join(hb.ROOT, "_build_san")
LIB = os.path.join(OUT, "libhawk_san.so")
# every sanitizer flag applies to the host compilation only
HOST_SAN = []
for _f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"):
    HOST_SAN += ["-Xarch_host", _f]


def asan_runtime() -> str | None:
    """clang's ASan runtime of the ROCm toolchain (preloaded by the test)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build() -> str:
    host = [s for s in hb.SOURCES if s.endswith(".cpp")]
    stems = {os.path.splitext(s)[0] for s in host}
    os.makedirs(OUT, exist_ok=True)

    def device_objects():
        objs = glob.glob(os.path.join(hb.OBJ, "*.o"))
        return [o for o in objs if os.path.splitext(os.path.basename(o))[0] not in stems]

    dev = device_objects()
    if len(dev) < len(hb.SOURCES) - len(host) + len(hb.SHAPED) * len(hb.SHAPES):
        hb.build()
        dev = device_objects()

    def compile_one(src: str) -> str:
        obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        cmd = [hb.HIPCC, "-x", "hip"] + hb.FLAGS + HOST_SAN + ["-c", os.path.join(hb.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(host))) as ex:
        objs = list(ex.map(compile_one, host))
    cmd = [hb.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + dev + ["-lhiprtc"] + \
        HOST_SAN[:4]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(LIB + ".tmp", LIB)
    return LIB
