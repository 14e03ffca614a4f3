"""The C ABI driven from C alone (tests/native/cabi_split.c): host-pointer
vectors, GPU shares 0, 1/2 (three memory modes, a non-prefix range) and 1,
each solve of b = A 1 returning x = 1 and A 1 = b exactly."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "native", "bin", "cabi_split")


def test_c_driver_split_modes_with_host_vectors(require_gpu):
    if not os.path.exists(EXE):
        import importlib.util
        spec = importlib.util.spec_from_file_location("build_native", os.path.join(HERE, "native", "build_native.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    print("[native] cabi_split 24 4", flush=True)
    r = subprocess.run([EXE, "24", "4"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0 and "all checks passed" in r.stdout
