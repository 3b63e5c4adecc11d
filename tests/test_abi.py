"""The C-ABI library loads and exports every entry point its header declares (no GPU calls)."""
import ast
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "filterreg.h")
LIB = os.path.join(ROOT, "paper_1811_10136_amd", "libfilterreg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z_0-9]+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        # the build script by path: the package itself refuses to import without the library
        import importlib.util
        spec = importlib.util.spec_from_file_location("_fr_build", os.path.join(ROOT, "paper_1811_10136_amd",
                                                                                "build.py"))
        hipbuild = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(hipbuild)
        hipbuild.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path_boundary():
    names = declared_functions()
    for f in ("fr_lattice_build", "fr_estep", "fr_mstep_reduce", "fr_register"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_library_exports_nothing_but_the_declared_symbols():
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if len(ln.split()) == 3 and ln.split()[1] == "T"})
    assert exported == declared_functions()


def test_binding_covers_every_declared_symbol():
    import paper_1811_10136_amd as fr
    assert sorted(fr.ABI_FUNCTIONS) == declared_functions()


def test_binding_shares_torchs_hip_runtime():
    """Importing the binding first still leaves one HIP runtime in the process (torch's): two
    runtimes under one soname leave torch without a device."""
    import subprocess
    import sys
    code = ("import paper_1811_10136_amd, torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    paths = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths
    import torch
    assert os.path.dirname(paths[0]) == os.path.join(os.path.dirname(torch.__file__), "lib"), paths


def test_version_and_error_string_without_gpu():
    lib = _lib()
    lib.fr_version.restype = ctypes.c_int32
    assert lib.fr_version() >= 100
    lib.fr_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.fr_last_error(), bytes)


def test_argument_errors_are_reported_before_any_device_work():
    """Entry points reject bad arguments without touching the device (works with no GPU)."""
    import paper_1811_10136_amd as fr
    lib = fr._lib
    # NULL lattice handle
    st = lib.fr_estep(None, None, None, None, None, None, None)
    assert st == fr.FR_EINVAL
    # bad residual kind in the reduce
    off = (ctypes.c_int64 * 2)(0, 0)
    cloud = fr.fr_cloud(None, None, None, None, None, None, off, 1)
    prm = fr.fr_mstep_params(7, 0, 0.0, 0.1, None)
    st = lib.fr_mstep_reduce(ctypes.byref(cloud), None, None, None, None, ctypes.byref(prm), None, None, None, None)
    assert st == fr.FR_EINVAL
    assert b"residual" in lib.fr_last_error()
    # negative sizes to the solver
    assert lib.fr_solve_rigid(-1, None, None, None, None, None, None, None, None) == fr.FR_EINVAL
    # destroying a NULL context
    assert lib.fr_ctx_destroy(None) == fr.FR_EINVAL
