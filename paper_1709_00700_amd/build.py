"""Builds libhawk.so (gfx950) in-tree: each source compiled by hipcc in
parallel, then linked into one shared library beside this file."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhawk.so")

SOURCES = ["hk_batch.hip", "hk_common.hip", "hk_dispatch.hip", "hk_mlp.hip", "hawk_api.cpp", "hawk_explore.cpp",
           "hawk_model.cpp", "hawk_batch.cpp", "hawk_jit.cpp", "hawk_planner.cpp"]
# device headers embedded into the library for run-time compilation (hawk_jit.cpp)
EMBEDDED = [("kSrcPlan", "hawk_plan.h"), ("kSrcDevice", "hawk_device.h"), ("kSrcAggBody", "hk_agg_body.h"),
            ("kSrcProjBody", "hk_proj_body.h"), ("kSrcScalarBody", "hk_scalar_body.h")]
# kernel families compiled once per shape class (see HkShape in hawk_plan.h)
SHAPED = ["hk_agg.hip", "hk_proj.hip", "hk_scalar.hip"]
SHAPES = ["A", "F", "J", "W", "G"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (no fp32 math on the hot path needs them)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", OBJ]


def _compile(job) -> str:
    src, shape = job if isinstance(job, tuple) else (job, None)
    stem = os.path.splitext(src)[0] + (f"_{shape}" if shape else "")
    obj = os.path.join(OBJ, stem + ".o")
    path = os.path.join(CSRC, src)
    cmd = [HIPCC] + FLAGS + (["-DHK_SHAPE_CLASS=HkShape" + shape] if shape else []) + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
    return obj


def _embed_headers() -> None:
    """Writes hk_jit_sources.inc: each embedded header as a raw string literal."""
    out = []
    for var, name in EMBEDDED:
        with open(os.path.join(CSRC, name)) as f:
            text = f.read()
        if ')HKSRC"' in text:
            raise RuntimeError(f"{name} contains the raw-string delimiter")
        out.append(f'const char {var}[] = R"HKSRC({text})HKSRC";\n')
    path = os.path.join(OBJ, "hk_jit_sources.inc")
    with open(path + ".tmp", "w") as f:
        f.write("".join(out))
    os.replace(path + ".tmp", path)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    _embed_headers()
    jobs = SOURCES[:1] + [(s, sh) for s in SHAPED for sh in SHAPES] + SOURCES[1:]  # longest first
    with ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16, len(jobs))) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
