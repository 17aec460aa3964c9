"""Build libpfl.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["pfl_api.hip", "pfl_step2d.hip", "pfl_step2d_lowp.hip", "pfl_step3d.hip", "pfl_step3d_lowp.hip",
       "pfl_adj2d.hip", "pfl_adj2d_lowp.hip", "pfl_aux.hip"]
# FP32-compute instantiations of the step and its adjoint: contraction (FMA)
# and reassociation are allowed; the FP64 parity form and everything else is
# built without them.
LOWP = {"pfl_step2d_lowp.hip", "pfl_step3d_lowp.hip", "pfl_adj2d_lowp.hip"}
LOWP_FLAGS = ["-ffp-contract=fast", "-fassociative-math", "-fno-signed-zeros", "-fno-trapping-math",
              "-freciprocal-math", "-ffinite-math-only"]
# The step and adjoint kernels see finite values only (non-finite states are
# detected by the reduction kernels, built strict).  Assuming so lets the
# compiler drop products with a zero lattice component, x * 0 -> 0, which it
# must keep under IEEE rules for the case x = inf or nan.  In the FP64 units
# no contraction or reassociation comes with it: every finite result equals the
# strict IEEE one, up to the sign of a zero.
FINITE = {"pfl_step2d.hip", "pfl_step3d.hip", "pfl_adj2d.hip"}
FINITE_FLAGS = ["-fno-honor-nans", "-fno-honor-infinities", "-fno-signed-zeros"]
OUT = os.path.join(HERE, "libpfl.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-shared",
    "-ffp-contract=off",
    # packed FP32 instructions disabled
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs = []
    procs = []
    for s in SRC:
        obj = os.path.join(HERE, "csrc", s.replace(".hip", ".o"))
        flags = [f for f in FLAGS if f != "-shared"]
        if s in LOWP:
            flags = [f for f in flags if f != "-ffp-contract=off"] + LOWP_FLAGS
        elif s in FINITE:
            flags = flags + FINITE_FLAGS
        cmd = [hipcc, "-c", os.path.join(HERE, "csrc", s), "-o", obj] + flags + inc
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    err = False
    for s, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            err = True
            sys.stderr.write(f"--- {s} failed ---\n" + out.decode(errors="replace"))
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    if err:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    for o in objs:
        os.remove(o)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
