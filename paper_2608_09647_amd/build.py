"""Build libcgmi.so in-tree: HIP kernels with hipcc for gfx950, the host
runtime with g++ (OpenMP), linked by hipcc.

    python -m paper_2608_09647_amd.build                      # libcgmi.so
    python -m paper_2608_09647_amd.build --sanitize address   # libcgmi_asan.so
    python -m paper_2608_09647_amd.build --sanitize thread    # libcgmi_tsan.so

The sanitizer builds instrument the host runtime only (the C ABI, argument
validation, the Matrix Market reader, the host complement's OpenMP loops,
the p exchange); the device code objects are the ordinary ones.  address:
AddressSanitizer + UndefinedBehaviorSanitizer with g++; thread:
ThreadSanitizer with LLVM's clang++ and its OpenMP runtime (whose barriers
ThreadSanitizer understands through the libarcher tool).  Load one in place
of libcgmi.so with CGMI_LIBRARY=<path> and the matching runtime preloaded
(see README)."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libcgmi.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_SOURCES = ["kernels_cg.hip", "kernels_small.hip", "kernels_fsai.hip", "kernels_batch.hip", "kernels_util.hip",
               "scratch.hip"]
HOST_SOURCES = ["cgmi.cpp", "devmatrix.cpp", "fsai.cpp", "batch.cpp", "mmio.cpp"]

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               # keep packed-float32 instructions out of the device code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-Wall",
              "-Wno-unused-function", "-Wno-unused-result"]
GXX_FLAGS = ["-O3", "-fopenmp", *HOST_FLAGS]

SANITIZERS = {
    # name: (host compiler, compile flags, link flags, library file)
    "address": ("g++", ["-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", *HOST_FLAGS],
                ["-fsanitize=address,undefined", "-fopenmp"], "libcgmi_asan.so"),
    "thread": (f"{ROCM}/llvm/bin/clang++", ["-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp=libomp",
                                            "-fsanitize=thread", *HOST_FLAGS],
               ["-fsanitize=thread", "-fopenmp=libomp", f"-L{ROCM}/llvm/lib", f"-Wl,-rpath,{ROCM}/llvm/lib"],
               "libcgmi_tsan.so"),
}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    noise = "is not a recognized feature for this target"
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if l.strip() and noise not in l]
    if msgs and verbose:
        print("\n".join(msgs))


def _device_objects(verbose):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run(["hipcc", *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    return objs


def build(verbose: bool = False) -> str:
    objs = _device_objects(verbose)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", ".host.o"))
        _run(["g++", *GXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lgomp", "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(kind: str, verbose: bool = False) -> str:
    """The library with its host runtime instrumented by a sanitizer (the
    device objects are the ordinary ones); linked by the host compiler."""
    cxx, cflags, lflags, name = SANITIZERS[kind]
    objs = _device_objects(verbose)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src.replace(".cpp", f".{kind}.o"))
        _run([cxx, *cflags, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    lib = os.path.join(PKG, name)
    tmp = lib + ".tmp"
    _run([cxx, "-shared", "-fPIC", *objs, *lflags, f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib",
          "-o", tmp], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--sanitize":
        print(build_sanitized(sys.argv[2], verbose=True))
    else:
        print(build(verbose=True))
