"""Build libdctkrylov.so (HIP, gfx950) in-tree: python -m paper_2103_11847_amd.build

Every source under csrc/ is compiled with hipcc for gfx950 into _build/ and
linked into paper_2103_11847_amd/libdctkrylov.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdctkrylov.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(HERE, "..", "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    return r.returncode, obj, out


def _stale(src, headers_mtime):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return os.path.getmtime(src) > t or headers_mtime > t


def build(verbose=True, incremental=False):
    """Compile every source (incremental=True: only those older than their object
    or than any header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = srcs
    if incremental:
        hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
        hdrs.append(os.path.join(HERE, "..", "include", "dctkrylov.h"))
        hm = max(os.path.getmtime(h) for h in hdrs)
        todo = [s_ for s_ in srcs if _stale(s_, hm)]
    with ThreadPoolExecutor(max_workers=max(1, min(8, len(todo)))) as ex:
        results = list(ex.map(_compile, todo))
    results_by_src = dict(zip(todo, results))
    results = [results_by_src.get(s_, (0, os.path.join(BUILD, os.path.basename(s_)[:-4] + ".o"), ""))
               for s_ in srcs]
    objs = []
    failed = False
    for (rc, obj, out), src in zip(results, srcs):
        if out.strip() and verbose:
            print(out, file=sys.stderr)
        if rc != 0:
            failed = True
            print("build failed: %s" % os.path.basename(src), file=sys.stderr)
        objs.append(obj)
    if failed:
        raise RuntimeError("libdctkrylov: compilation failed")
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stdout + r.stderr, file=sys.stderr)
        raise RuntimeError("libdctkrylov: link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
