"""CPU build of the library's HIP sources (csrc/*.hip) with the SIMT shim in
tests/simt/hip/, under AddressSanitizer and UndefinedBehaviorSanitizer, as
one shared library exporting the same C ABI as libdmn.so.

Test infrastructure: it checks every global, LDS and array index the kernels
use on the host, where an out-of-bounds access stops the run with a report
instead of faulting a device.  The build is cached in tests/simt/_build under
a hash of the sources and flags.
"""
import concurrent.futures as cf
import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2103_08253_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "_build")
CXX = os.environ.get("CXX_SIMT", "g++")

FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC",
         "-I", HERE, "-I", INCLUDE, "-I", CSRC]

# Gauss-point kernel variants of this build: the device build's list plus the
# (8, 3) lane split, which the device build leaves out after a device fault
VARIANTS = ("-DDMN_GP_VARIANTS(X)=X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(4, 2) "
            "X(5, 1) X(5, 2) X(6, 1) X(6, 2) X(7, 1) X(7, 2) X(8, 2) X(8, 3)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# ThreadSanitizer instead of ASan/UBSan: a data race between GPU threads (for
# example LDS written by one lane and read by another with no barrier between)
SANITIZERS = {"address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
              "thread": ["-fsanitize=thread"]}


def _digest(defines, srcs):
    h = hashlib.sha256()
    for f in list(srcs) + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                                 if f.endswith(".hpp")) + [
            os.path.join(INCLUDE, "dmn.h"), os.path.join(HERE, "hip", "hip_runtime.h")]:
        with open(f, "rb") as fh:
            h.update(f.encode() + fh.read())
    h.update(" ".join(FLAGS + list(defines) + [CXX]).encode())
    return h.hexdigest()[:16]


def _compile(src, obj, defines):
    cmd = [CXX, *FLAGS, *defines, "-x", "c++", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stderr[-4000:]}")


def build(defines=(VARIANTS,), jobs=None, srcs=None, name="libdmn_simt", sanitizer="address"):
    """Return the path of a sanitised CPU library, building it if needed: by
    default the whole library (every csrc/*.hip), else the given sources."""
    srcs = list(srcs) if srcs is not None else sources()
    san = SANITIZERS[sanitizer]
    defines = tuple(defines) + tuple(san)
    if sanitizer != "address":
        name = f"{name}_{sanitizer}"
    tag = _digest(defines, srcs)
    lib = os.path.join(OUT, f"{name}_{tag}.so")
    if os.path.exists(lib):
        return lib
    os.makedirs(OUT, exist_ok=True)
    objs = [os.path.join(OUT, f"{tag}_{os.path.basename(s)}.o") for s in srcs]
    jobs = jobs or max(1, min(6, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], defines), zip(srcs, objs)))
    tmp = lib + ".tmp"
    r = subprocess.run([CXX, "-shared", san[0], "-Wl,--no-undefined",
                        "-o", tmp, *objs, "-lpthread"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    stale = re.compile(rf"^{re.escape(name)}_[0-9a-f]{{16}}\.so$")
    for f in os.listdir(OUT):  # builds of earlier sources
        if stale.match(f) and os.path.join(OUT, f) != lib:
            os.remove(os.path.join(OUT, f))
    return lib


def build_f32_kernel():
    """The FP32-storage Gauss-point kernel (tests/simt/fp32_kernel.cpp, which
    includes the kernel source) with the table-prep kernels it needs."""
    return build(defines=(), srcs=[os.path.join(HERE, "fp32_kernel.cpp"),
                                   os.path.join(CSRC, "dmn_prep.hip")],
                 name="libdmn_simt_f32")


def asan_runtime(sanitizer="address"):
    """Path of the compiler's sanitizer runtime, preloaded into the Python
    process that loads the library."""
    lib = {"address": "libasan.so", "thread": "libtsan.so"}[sanitizer]
    return subprocess.run([CXX, f"-print-file-name={lib}"], capture_output=True,
                          text=True, check=True).stdout.strip()


if __name__ == "__main__":
    print(build(tuple(sys.argv[1:]) or (VARIANTS,)))
