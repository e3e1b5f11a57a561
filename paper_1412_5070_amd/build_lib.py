"""Build libf12int.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel, the shape-specialised
contraction kernels (f12_big_unit.hip) once per (l_a + l_b, ket precision),
then linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libf12int.so")
# (source, object name, extra defines)
SOURCES = [(s, os.path.splitext(s)[0], []) for s in ("f12_host.cpp", "f12_batch.cpp", "f12_kernels.hip", "f12_k2.hip", "f12_sph.hip", "f12_hobson.hip", "f12_digest.hip")]
SOURCES += [("f12_big_unit.hip", "f12_big_unit_%d_%d" % (lab, prec), ["-DF12_LAB=%d" % lab, "-DF12_PREC=%d" % prec])
            for prec in (0, 1) for lab in range(7)]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    # with F12_INCREMENTAL=1, an object newer than its source and every header
    # is kept (a development aid; the default always compiles everything)
    incremental = os.environ.get("F12_INCREMENTAL") == "1"
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(os.path.dirname(HERE), "include", "f12int.h"))
    newest_h = max(os.path.getmtime(h) for h in headers)

    def compile_one(job):
        src, name, defs = job
        obj = os.path.join(objdir, name + ".o")
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t > os.path.getmtime(os.path.join(CSRC, src)) and t > newest_h:
                return src, obj, subprocess.CompletedProcess([], 0, "", "")
        cmd = [hipcc] + FLAGS + defs + ["-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, r in failed:
        sys.stderr.write("== %s\n%s%s" % (s, r.stdout, r.stderr))
    if failed:
        raise RuntimeError("hipcc failed building libf12int.so")
    if verbose:
        for s, _, r in results:
            if r.stderr.strip():
                sys.stderr.write(r.stderr)
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + [o for _, o, _ in results] + ["-o", LIB + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libf12int.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
