"""The C ABI library loads and exports every function include/nfvm.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "nfvm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nfvm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("nfvm_init_grid", "nfvm_step", "nfvm_mg_solve", "nfvm_submit", "nfvm_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2603_21869_amd import nfvm
    path = nfvm.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libnfvm.so not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(nfvm.EXPORTS) == set(declared())


def test_footprint_and_validation_without_gpu():
    """Descriptor validation and the footprint model are host code."""
    from paper_2603_21869_amd import cases as C, nfvm
    if not os.path.exists(nfvm.LIB_PATH):
        pytest.skip("libnfvm.so not built")
    d = nfvm.Desc(C.channel3d(64, 16, 16, n_levels=3))
    b64 = nfvm.nfvm_grid_footprint(d)
    d32 = nfvm.Desc(C.channel3d(64, 16, 16, n_levels=3), precision=nfvm.NFVM_FP32)
    assert 0 < nfvm.nfvm_grid_footprint(d32) < b64
    bad = nfvm.Desc(C.channel3d(64, 16, 16, n_levels=6))
    with pytest.raises(nfvm.NfvmError) as e:
        nfvm.nfvm_grid_footprint(bad)
    assert e.value.status == nfvm.NFVM_E_INVAL


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises instead of falling
    back to anything (run in a fresh interpreter so the loaded library of
    this process is not reused)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2603_21869_amd import nfvm\n"
            "nfvm.LIB_PATH = '/nonexistent/libnfvm.so'\n"
            "try:\n    nfvm.lib()\nexcept OSError as e:\n    print('raised', e)\n    sys.exit(0)\n"
            "sys.exit(1)\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "raised" in r.stdout, r.stdout + r.stderr


def test_reduction_scratch_covers_every_tiling_of_odd_shapes():
    """The partial buffer of the device reductions holds the largest launch
    any tile choice can make: tile counts are rounded up to a multiple of 8
    workgroups, every one of which stores its partial, so shapes whose column
    and plane counts multiply to a non-multiple of 8 need the rounded count
    (host code, no device work)."""
    from paper_2603_21869_amd import cases as C, nfvm
    if not os.path.exists(nfvm.LIB_PATH):
        pytest.skip("libnfvm.so not built")
    shapes2 = [(90, 18), (64, 2), (66, 6), (130, 34), (8, 8), (256, 64), (4, 4)]
    shapes3 = [(64, 32, 32), (96, 32, 32), (66, 6, 3), (130, 10, 7), (200, 12, 5), (8, 8, 1),
               (1024, 512, 256)]
    seen_round = False
    for nx, ny in shapes2:
        c = C.channel2d(nx, ny, n_levels=1, n_steps=1)
        need, cap = nfvm.nfvm_reduction_blocks(nfvm.Desc(c))
        assert 0 < need <= cap, (nx, ny, need, cap)
        cols = -(-nx // 64) * -(-ny // 4)
        seen_round |= need > cols
    for nx, ny, nz in shapes3:
        c = C.channel3d(nx, ny, nz, n_levels=1, n_steps=1)
        need, cap = nfvm.nfvm_reduction_blocks(nfvm.Desc(c))
        assert 0 < need <= cap, (nx, ny, nz, need, cap)
        assert need % 8 == 0 and cap % 8 == 0
    assert seen_round  # some 2D shape needs more workgroups than it has columns


def test_null_arguments_are_rejected_without_gpu():
    """The reverse-mode, probe and tuning entry points reject a null grid or
    descriptor with NFVM_E_INVAL and a message, before any device work."""
    from paper_2603_21869_amd import nfvm
    if not os.path.exists(nfvm.LIB_PATH):
        pytest.skip("libnfvm.so not built")
    L = nfvm.lib()
    f = nfvm.nfvm_fields()
    st = nfvm.nfvm_step_stats()
    calls = [
        lambda: L.nfvm_explicit_adjoint_device(None, ctypes.byref(f), ctypes.byref(f),
                                               ctypes.byref(f)),
        lambda: L.nfvm_destroy_adjoint_device(None, ctypes.byref(f), 0.1, None, None,
                                              ctypes.byref(f)),
        lambda: L.nfvm_step_adjoint_device(None, ctypes.byref(f), ctypes.byref(f),
                                           ctypes.byref(f), 1e-10, 10, -1, ctypes.byref(st)),
        lambda: L.nfvm_pressure_adjoint_device(None, None, None, None, None, None, None, None,
                                               1e-10, 10, -1, None),
        lambda: L.nfvm_line_probe(None, None, 0, None),
        lambda: L.nfvm_tune(None),
    ]
    for call in calls:
        assert call() == nfvm.NFVM_E_INVAL
        assert nfvm.nfvm_last_error()
