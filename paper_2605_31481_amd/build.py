"""Build libbard.so (HIP kernels for gfx950 + host compiler + C ABI) in-tree."""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc")
_OUT = os.path.join(_HERE, "libbard.so")
_BUILD = os.path.join(os.path.dirname(_HERE), "_build", "bard")

SOURCES = ["kernels.hip", "adjoint.hip", "tiers.hip", "path.hip", "api.cpp", "compiler.cpp", "plan.cpp", "specialize.cpp"]
_GEN = os.path.join(_BUILD, "gen")

# Packed FP32 instructions are turned off for every HIP translation unit.
# Multiply-adds are fused only within one expression (-ffp-contract=on), so a
# quantity rounds the same way in every kernel instantiation that computes it:
# state one operator stores in a workspace tier has the bits another
# operator would have computed itself.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def library_path() -> str:
    return _OUT


def _embed_headers():
    """spatial.h as a C++ string literal: the model specialiser hands its text
    to hipRTC, so generated kernels compile against the library's own device
    helpers."""
    os.makedirs(_GEN, exist_ok=True)
    text = open(os.path.join(_SRC, "spatial.h")).read()
    if ")BARDSRC" in text:
        raise RuntimeError("spatial.h contains the raw-string delimiter")
    out = os.path.join(_GEN, "spatial_h.inc")
    body = 'R"BARDSRC(' + text + ')BARDSRC"\n'
    if not os.path.exists(out) or open(out).read() != body:
        with open(out, "w") as f:
            f.write(body)


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(_BUILD, src.replace(".", "_") + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc", *lang, *HIP_FLAGS, "-I", _GEN, "-c", os.path.join(_SRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


_PEAKS_OUT = os.path.join(_HERE, "libbard_peaks.so")


def build_peaks(verbose: bool = False) -> str:
    """The benchmark's peak probe (csrc/peaks.hip), a library of its own."""
    tmp = _PEAKS_OUT + ".tmp"
    cmd = ["hipcc", "-x", "hip", *HIP_FLAGS, "-shared", os.path.join(_SRC, "peaks.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _PEAKS_OUT)
    return _PEAKS_OUT


def build(verbose: bool = False) -> str:
    os.makedirs(_BUILD, exist_ok=True)
    _embed_headers()
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = _OUT + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lhiprtc", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _OUT)
    build_peaks(verbose)
    return _OUT


if __name__ == "__main__":
    print(build(verbose=True))
