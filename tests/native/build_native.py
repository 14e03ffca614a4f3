"""Build the C drivers of the C ABI into tests/native/bin (gcc; with
--sanitize thread also a ThreadSanitizer build, clang, linked against
libcgmi_tsan.so from `python -m paper_2608_09647_amd.build --sanitize thread`).

    python tests/native/build_native.py [--sanitize thread]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2608_09647_amd")
BIN = os.path.join(HERE, "bin")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
DRIVERS = ["cabi_split"]


def build(sanitize: str | None = None, verbose: bool = False) -> list:
    os.makedirs(BIN, exist_ok=True)
    out = []
    for name in DRIVERS:
        src = os.path.join(HERE, name + ".c")
        if sanitize == "thread":
            exe = os.path.join(BIN, name + "_tsan")
            cmd = [f"{ROCM}/llvm/bin/clang", "-O1", "-g", "-std=c11", "-fsanitize=thread", src, "-o", exe,
                   f"-L{PKG}", "-l:libcgmi_tsan.so", f"-Wl,-rpath,{PKG}", "-lm"]
        else:
            exe = os.path.join(BIN, name)
            cmd = ["gcc", "-O2", "-std=c11", "-Wall", src, "-o", exe, f"-L{PKG}", "-l:libcgmi.so",
                   f"-Wl,-rpath,{PKG}", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        out.append(exe)
    return out


if __name__ == "__main__":
    san = sys.argv[2] if len(sys.argv) > 2 and sys.argv[1] == "--sanitize" else None
    print(build(san, verbose=True))
