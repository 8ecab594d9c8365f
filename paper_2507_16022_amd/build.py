"""Build the HIP library libdotpe.so in-tree for gfx950 (hipcc, no JIT).

The host runtime (csrc/dotpe.hip), the pre-selection kernels
(csrc/preselect.hip) and two instantiation units per (precision, number of
m groups) -- the fused kernel and bound pass (csrc/fused_inst.hip), the
marginalisation kernels (csrc/marg_inst.hip) -- are compiled to objects in
parallel, then linked into one shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdotpe.so")
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(os.path.dirname(HERE), "_build", "dotpe")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]

PRECISIONS = (0, 1, 2)     # FP64, FP16x2, BF16x2
GROUPS = (1, 2, 3, 4)      # distinct m values


def units():
    """(source, object, extra flags) of every translation unit."""
    out = [(os.path.join(CSRC, "dotpe.hip"), os.path.join(OBJ, "dotpe.o"), []),
           (os.path.join(CSRC, "preselect.hip"), os.path.join(OBJ, "preselect.o"), [])]
    for p in PRECISIONS:
        for g in GROUPS:
            inst = [f"-DDOTPE_INST_PREC={p}", f"-DDOTPE_INST_G={g}"]
            out.append((os.path.join(CSRC, "fused_inst.hip"), os.path.join(OBJ, f"fused_p{p}_g{g}.o"),
                        inst))
            # the marginalisation kernels: no machine-level hoisting of constants
            out.append((os.path.join(CSRC, "marg_inst.hip"), os.path.join(OBJ, f"marg_p{p}_g{g}.o"),
                        inst + ["-mllvm", "-disable-machine-licm"]))
    return out


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, r.stdout + r.stderr


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(16, max(1, len(os.sched_getaffinity(0))))
    cmds = [[HIPCC] + FLAGS + extra + ["-c", "-o", obj, src] for src, obj, extra in units()]
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    for cmd, (rc, log) in zip(cmds, results):
        if rc != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + log)
            raise RuntimeError("hipcc failed compiling " + cmd[-1])
        if verbose and log.strip():
            sys.stderr.write(log)
    tmp = LIB + ".tmp"
    rc, log = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp]
                   + [obj for _, obj, _ in units()])
    if rc != 0:
        sys.stderr.write(log)
        raise RuntimeError("hipcc failed linking libdotpe.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
