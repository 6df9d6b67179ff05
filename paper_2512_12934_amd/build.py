"""Build the HIP library ``liblbm.so`` for gfx950 (in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
# the measurement library (streaming probes), linked on its own
PROBE_LIB = os.path.join(HERE, "libprobe.so")
SOURCES = ["lbm_api.hip", "k2d.hip", "k3d.hip", "surrogate.hip"]
PROBE_SOURCES = ["probe.hip"]
HEADERS = ["kernels.h", "lattice.h", "params.h", "launch.h", "launch_impl.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds are fused only where one source expression has them, so
    # every kernel that inlines the same node update (the single-context and
    # the batched launch, every tile configuration) rounds identically
    "-ffp-contract=on",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False, extra=()) -> str:
    """Compile every translation unit in parallel, then link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES + PROBE_SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *extra, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    for p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, "hipcc")
    for lib, srcs in ((LIB, SOURCES), (PROBE_LIB, PROBE_SOURCES)):
        lib_objs = [o for o, s in zip(objs, SOURCES + PROBE_SOURCES) if s in srcs]
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp", *lib_objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB) or not os.path.exists(PROBE_LIB):
        return True
    t = min(os.path.getmtime(LIB), os.path.getmtime(PROBE_LIB))
    deps = [os.path.join(CSRC, s) for s in SOURCES + PROBE_SOURCES + HEADERS]
    deps += [os.path.join(HERE, "..", "include", h) for h in ("lbm.h", "lbm_probe.h")]
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
