"""Build the HIP shared library (gfx950) in-tree: paper_2003_03508_amd/libhmm.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhmm.so")
# (source, extra flags): small tiles keep MFMA results in VGPRs (they are
# read by VALU code every step); large tiles need AGPRs for their accumulators.
UNITS = [(os.path.join(CSRC, "hmm_api.hip"), ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
         (os.path.join(CSRC, "hmm_large.hip"), []),
         (os.path.join(CSRC, "hmm_batch.hip"), []),
         (os.path.join(CSRC, "hmm_sampler.hip"), []),
         (os.path.join(CSRC, "hmm_posterior.hip"), []),
         (os.path.join(CSRC, "hmm_viterbi.hip"), []),
         (os.path.join(CSRC, "hmm_forecast.hip"), [])]
SOURCES = [u[0] for u in UNITS]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "hmm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=False):
    """Compile each unit to an object (in parallel), then link the shared library."""
    objs, procs = [], []
    for src, extra in UNITS:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + extra + ["-c", "-o", obj, src]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    for cmd, pr in procs:
        _, err = pr.communicate()
        err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l)
        if pr.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + err)
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
