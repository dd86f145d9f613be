"""Build the HIP library ``libpdfcbm.so`` for gfx950 with hipcc.

Called by ``__graft_entry__.build()``; also runnable as
``python -m paper_2105_06055_amd.build``.  The C entry points (pd_fcbm.hip)
and fourteen instantiation units of the per-dtype implementation (pd_inst.hip
with PD_INST_T = float / double and PD_INST_PART = 0 .. 6) compile in
parallel to objects, which are linked into the library, written in-tree next
to this file so it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdfcbm.so")
HEADERS = ["pd_fft.hpp", "pd_ops.hpp", "pd_passes.hpp", "pd_plan.hpp", "pd_impl.hpp"]
UNITS = [("pd_fcbm.hip", [])] + [
    ("pd_inst.hip", ["-DPD_INST_T=%s" % t, "-DPD_INST_PART=%d" % part, "-DPD_INST_F32=%d" % (t == "float")])
    for t in ("float", "double") for part in range(7)]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="pdfcbm_build_") as tmpd:
        jobs = []
        for k, (src, defs) in enumerate(UNITS):
            obj = os.path.join(tmpd, "u%d.o" % k)
            jobs.append(([hipcc] + HIPCC_FLAGS + inc + defs + ["-c", "-o", obj, os.path.join(CSRC, src)], obj))

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
            list(ex.map(run, [c for c, _ in jobs]))
        tmp = LIB + ".tmp%d" % os.getpid()
        run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] +
            [o for _, o in jobs])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
