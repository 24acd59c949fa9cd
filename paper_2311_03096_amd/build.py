"""Build the gfx950 HIP library libwsr.so in-tree with hipcc (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwsr.so")
SOURCES = ["wsr_small.hip", "wsr_big.hip", "wsr_api.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wno-unused-command-line-argument",
]


PROBE_LIB = os.path.join(HERE, "libwsr_probe.so")  # LDS throughput probes (measurement only)
PROBE_SOURCES = ["wsr_lds_probe.hip"]
# the same sources with phase timestamps in the short-segment forward (measurement only)
PHASE_LIB = os.path.join(HERE, "libwsr_phases.so")


def _hipcc(sources, lib, verbose, defines=()):
    """Start hipcc on `sources` into `lib`; returns a function that waits for it and installs it."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + ["-D" + m for m in defines] + [os.path.join(CSRC, s) for s in sources] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)

    def finish():
        _, stderr = proc.communicate()
        err = "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)
        if proc.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + err)
        os.replace(tmp, lib)
        return lib
    return finish


def build(verbose: bool = False) -> str:
    """Compile the three libraries side by side (each hipcc run is single-threaded)."""
    jobs = [_hipcc(SOURCES, LIB, verbose), _hipcc(PROBE_SOURCES, PROBE_LIB, verbose),
            _hipcc(SOURCES, PHASE_LIB, verbose, defines=("WSR_PHASE_CLOCKS",))]
    errors = []
    for finish in jobs:  # wait for every job before reporting, so no compiler is left running
        try:
            finish()
        except RuntimeError as e:
            errors.append(str(e))
    if errors:
        raise RuntimeError("\n".join(errors))
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
