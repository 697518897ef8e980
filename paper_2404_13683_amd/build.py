"""Build libovfem.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2404_13683_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libovfem.so")
OBJ_DIR = os.path.join(HERE, "_build")

COMPILE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # the reference matrices are derived by constexpr evaluation of the element integrals
    "-fconstexpr-steps=100000000",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep MFMA accumulators in architectural VGPRs (fewer copies, fewer registers)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"),
]
# kept for callers that build single sources by hand
HIPCC_FLAGS = COMPILE_FLAGS + ["-shared"]


def sources():
    """Translation units: the host library and one per kernel instantiation group."""
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _messages(res):
    return [ln for ln in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in ln and ln.strip()]


def build(verbose=False, jobs=None):
    """Compile libovfem.so; always recompiles (the translation units in parallel).
    Returns the library path."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or max(1, min(len(sources()), os.cpu_count() or 1, 16))
    cc = hipcc()
    pending, objs, msgs = list(sources()), [], []
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            src = pending.pop(0)
            obj = os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")
            cmd = [cc] + COMPILE_FLAGS + ["-c", "-o", obj, src]
            running.append((src, obj, subprocess.Popen(cmd, cwd=HERE, stdout=subprocess.PIPE,
                                                       stderr=subprocess.PIPE, text=True)))
        src, obj, proc = running.pop(0)
        out, err = proc.communicate()
        m = [ln for ln in (out + err).splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if proc.returncode != 0:
            for _, _, p in running:
                p.kill()
            raise RuntimeError("hipcc failed on %s:\n%s" % (os.path.basename(src), "\n".join(m)))
        msgs += m
        objs.append(obj)
    tmp = LIB + ".tmp"
    res = subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + sorted(objs), cwd=HERE,
                         capture_output=True, text=True)
    m = _messages(res)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + "\n".join(m))
    msgs += m
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
