"""Build step for the gfx950 library: hipcc -> paper_2008_07437_amd/libmvgeo.so.

Every source is compiled to an object in parallel (each file's kernels and
device functions are self-contained, so no relocatable device code is
needed), then the objects are linked into the shared library."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
SO = os.path.join(HERE, "libmvgeo.so")
SOURCES = ["capi.hip", "matern.hip", "dense.hip", "solve.hip", "mixed.hip", "morton.hip", "tlr.hip",
           "tlr_kernels.hip", "tlr_gemm.hip", "tlr_update.hip", "batched.hip", "noalloc.hip", "serve.cpp", "mle.cpp"]
CFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-Wno-unused-value"]
LDFLAGS = ["--offload-arch=gfx950", "-shared", "-fPIC",
           "-Wl,-z,defs"]  # an unresolved symbol fails the link, not the first load


def _obj(src: str) -> str:
    return os.path.join(OBJ, os.path.splitext(src)[0] + ".o")


def _compile(src: str, verbose: bool) -> None:
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc", *CFLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *lang, "-c",
           os.path.join(CSRC, src), "-o", _obj(src)]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)


def _stale(src: str) -> bool:
    """The object is missing or older than its source or any header (every
    source includes the shared headers, so a header change rebuilds all)."""
    obj = _obj(src)
    if not os.path.exists(obj):
        return True
    heads = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    heads += [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))]
    newest = max(os.path.getmtime(f) for f in heads + [os.path.join(CSRC, src)])
    return os.path.getmtime(obj) < newest


def build(verbose: bool = False, only=None) -> str:
    """Compiles the sources (all of them, or those named in `only` plus any
    whose object is stale) and links libmvgeo.so."""
    os.makedirs(OBJ, exist_ok=True)
    todo = [s for s in SOURCES if only is None or s in only or _stale(s)]
    jobs = max(1, min(len(todo), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, s, verbose) for s in todo]:
            f.result()
    cmd = ["hipcc", *LDFLAGS, *[_obj(s) for s in SOURCES], "-o", SO + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    import sys
    print(build(verbose=True, only=sys.argv[1:] or None))
