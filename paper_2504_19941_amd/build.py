"""Builds libdsm.so, the gfx950 HIP library behind include/dsm.h, in-tree.

    python -m paper_2504_19941_amd.build        # or: python paper_2504_19941_amd/build.py
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdsm.so")
SOURCES = ["dsm_api.hip", "dsm_kernels.hip", "dsm_fused.hip", "dsm_links.hip", "dsm_batch.hip"]
# streaming reference kernels the benchmark times beside the step (measurement only)
PROBE_LIB = os.path.join(PKG, "libdsm_probe.so")
PROBE_SOURCES = ["dsm_probe.hip"]
ARCH = "gfx950"


def hipcc_command(out: str = LIB, extra=(), sources=SOURCES):
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # no contraction of a*b + c into FMAs: each kernel's rounding is then
        # fixed by its source, so the single-lattice and batched kernels,
        # which share the per-node code, give bit-identical results
        "-ffp-contract=off",
        "-Wall", "-I", os.path.join(ROOT, "include"),
        *extra,
        "-o", out, *[os.path.join(CSRC, s) for s in sources],
    ]


def _build_one(out, sources, verbose, extra):
    cmd = hipcc_command(out, extra=extra, sources=sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = out + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.run(cmd, check=True, cwd=PKG)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra=()) -> str:
    """Builds libdsm.so and the benchmark's streaming-probe library."""
    _build_one(PROBE_LIB, PROBE_SOURCES, verbose, extra)
    return _build_one(LIB, SOURCES, verbose, extra)


if __name__ == "__main__":
    print(build(verbose=True))
