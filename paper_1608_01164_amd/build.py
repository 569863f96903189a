"""Build libhqdwh.so (HIP for gfx950 + host C++) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhqdwh.so")
SOURCES = ["kernels.hip", "engine.hip", "mlp.hip", "noalloc.hip", "givens.cpp", "predictor.cpp", "tuning.cpp", "zolo.cpp", "hmatrix.cpp", "tree.cpp", "api.cpp"]
ARCH = os.environ.get("HQ_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(force: bool = True, jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        s = os.path.join(CSRC, src)
        deps = [s] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
        deps.append(os.path.join(HERE, "..", "include", "hq.h"))
        if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
            continue
        cmd = ["hipcc", *FLAGS, "-c", s, "-o", obj]
        if src.endswith(".cpp"):
            # host-only translation units: no device code, so no offload target
            cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-fopenmp", "--offload-arch=" + ARCH, "-c", s, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = OUT + ".tmp%d" % os.getpid()
    link = ["hipcc", "-shared", "-fPIC", "-fopenmp", f"--offload-arch={ARCH}", *objs, "-o", tmp,
            "-Wl,-rpath,/opt/rocm/lib:/opt/rocm/llvm/lib", "-ldl"]
    subprocess.check_call(link)
    os.replace(tmp, OUT)
    return OUT


def _wait(item):
    src, p = item
    _, err = p.communicate()
    err = "\n".join(l for l in err.splitlines() if "packed-fp32" not in l and "feature" not in l)
    if p.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv))
