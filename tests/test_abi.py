"""The C ABI loads, exports every declared symbol and rejects bad arguments
without touching a GPU (argument checks run before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "perks.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(perks_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2204_02064_amd as pk
    return pk.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "perks_stencil_run" in names and "perks_cg_solve" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror(L):
    assert L.perks_strerror(0) == b"success"
    assert L.perks_strerror(-1) == b"invalid argument"


def test_invalid_arguments_are_rejected(L):
    import paper_2204_02064_amd as pk
    w = np.zeros(9)
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(0x1000)
    assert L.perks_stencil_run(None, wp, pk.Shape(2, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(4, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 2, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), -1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), 1, 7, None, None) == -1
    w27 = np.zeros(27)
    w27[0] = 1.0           # a 3D corner weight: the radius-1 box kernel is disabled
    assert L.perks_stencil_run(fake, w27.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(3, 0, 8, 8, 8), 1, 1, None, None) == -5
    w343 = np.zeros(343)   # 3D radius 3: no kernel
    assert L.perks_stencil_run(fake, w343.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(3, 3, 8, 8, 8), 1, 1, None, None) == -5
    # radius: 0..4; ring of width r; 3D only radius 1; boxes only radius 2
    w25 = np.zeros(25)
    w25[12] = 1.0
    w25p = w25.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.perks_stencil_run(fake, w25p, pk.Shape(2, 5, 64, 64, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, w25p, pk.Shape(2, -1, 64, 64, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, w25p, pk.Shape(2, 2, 4, 64, 1), 1, 1, None, None) == -1
    w125 = np.zeros(125)
    w125[0] = 1.0          # a corner of the radius-2 3D box: only the 3D radius-2 star is built
    assert L.perks_stencil_run(fake, w125.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(3, 2, 16, 16, 16), 1, 1, None, None) == -5
    w49 = np.zeros(49)
    w49[0] = 1.0           # a corner of the radius-3 box: no 7x7 box kernel
    assert L.perks_stencil_run(fake, w49.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(2, 3, 64, 64, 1), 1, 1, None, None) == -5
    assert L.perks_stencil_run_batched((ctypes.c_void_p * 1)(fake), (pk.Shape * 1)(pk.Shape(2, 2, 64, 64, 1)), 1,
                                       w25p, 1, 1, None) == -5
    tu = pk.Tuning()
    tu.kernel = 4          # only 0, 1, 2, 3
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), 1, 1, None, ctypes.byref(tu)) == -1
    tu = pk.Tuning()
    tu.steps_per_sync = 4  # for kernel 3 only
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), 1, 1, None, ctypes.byref(tu)) == -1
    wn = np.full(9, np.nan)
    assert L.perks_stencil_run(fake, wn.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(2, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert b"finite" in L.perks_last_error()


def test_solver_arguments_are_rejected_before_any_device_call(L):
    import paper_2204_02064_amd as pk
    fake = ctypes.c_void_p(0x1000)
    rp = np.array([0, 1], np.int32)
    A = pk.Csr(1, 1, rp.ctypes.data, rp.ctypes.data, rp.ctypes.data, pk.PERKS_F64, 0)
    res = pk.CgResult()
    r = ctypes.byref(res)
    assert L.perks_cg_solve(None, fake, fake, 1e-8, 10, 0, 0, None, r) == -1
    assert L.perks_cg_solve(ctypes.byref(A), fake, fake, -1.0, 10, 0, 0, None, r) == -1
    assert L.perks_cg_solve(ctypes.byref(A), fake, fake, 1e-8, -1, 0, 0, None, r) == -1
    assert L.perks_cg_solve(ctypes.byref(A), fake, fake, 1e-8, 10, 5, 0, None, r) == -1
    assert L.perks_cg_solve(ctypes.byref(A), fake, fake, 1e-8, 10, 0, 7, None, r) == -1
    assert L.perks_cg_solve(ctypes.byref(A), None, fake, 1e-8, 10, 0, 0, None, r) == -1
    A32 = pk.Csr(1, 1, rp.ctypes.data, rp.ctypes.data, rp.ctypes.data, pk.PERKS_F32, 0)
    assert L.perks_cg_solve(ctypes.byref(A32), fake, fake, 1e-8, 10, 0, 0, None, r) == -5
    assert L.perks_cg_solve_baseline(ctypes.byref(A), fake, fake, 1e-8, 10, 0, 0, 0, None, r) == -1
    assert L.perks_cg_solve_capture(ctypes.byref(A), fake, fake, 1e-8, 10, 0, None, 2, None, None, None, r) == -1
    # FCG: the grid must hold the unknowns; a network needs log k
    assert L.perks_fcg_solve(ctypes.byref(A), fake, fake, 1e-8, 10, None, None, 2, 2, 20, None, r) == -1
    assert L.perks_fcg_solve(ctypes.byref(A), fake, fake, 1e-8, 10, fake, None, 1, 1, 20, None, r) == -1
    assert L.perks_fcg_solve(ctypes.byref(A), fake, fake, 1e-8, 10, None, None, 1, 1, 0, None, r) == -1
    # batched
    plan = ctypes.c_void_p()
    assert L.perks_cg_batch_create(None, None, None, -1, 1e-8, 10, 0, 0, ctypes.byref(plan)) == -1
    arr = (pk.Csr * 1)(A)
    ptrs = (ctypes.c_void_p * 1)(fake)
    assert L.perks_cg_batch_create(arr, ptrs, ptrs, 1, -1.0, 10, 0, 0, ctypes.byref(plan)) == -1
    assert L.perks_cg_batch_create(arr, ptrs, ptrs, 1, 1e-8, 10, 0, 0, None) == -1
    assert L.perks_cg_batch_run(None, None) == -1
    assert L.perks_cg_batch_results(None, None, None) == -1
    assert L.perks_cg_batch_destroy(None) == 0
    # network
    assert L.perks_nn_forward(None, fake, 1, 4, 4, fake, None) == -1
    assert L.perks_nn_forward(fake, fake, 0, 4, 4, fake, None) == -1
    assert L.perks_nn_loss_grad(fake, fake, fake, 1, 3, 4, fake, None, None) == -5   # H must be even
    assert L.perks_nn_loss_grad(fake, fake, fake, 1, 4, 600, fake, None, None) == -5  # W <= 512
    assert L.perks_nn_adam(fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    st = ctypes.c_int32(0)
    # nn_train: exactly one of target / planes; planes need field; batch <= P
    assert L.perks_nn_train(fake, fake, fake, fake, fake, 4, 4, 4, 1, 2, 1e-3, 0, fake, fake, ctypes.byref(st), None,
                            None) == -1
    assert L.perks_nn_train(fake, fake, None, fake, None, 4, 4, 4, 1, 2, 1e-3, 0, fake, fake, ctypes.byref(st), None,
                            None) == -1
    assert L.perks_nn_train(fake, fake, fake, None, None, 4, 4, 4, 1, 8, 1e-3, 0, fake, fake, ctypes.byref(st), None,
                            None) == -1
    assert L.perks_nn_train(fake, fake, fake, None, None, 4, 3, 4, 1, 2, 1e-3, 0, fake, fake, ctypes.byref(st), None,
                            None) == -5


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes
    and field offsets (a host-only C program built with gcc prints them)."""
    import shutil
    import subprocess
    import paper_2204_02064_amd as pk
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"perks_cg_result": pk.CgResult, "perks_barrier_stats_t": pk.BarrierStats, "perks_tuning": pk.Tuning,
               "perks_stencil_plan": pk.StencilPlan, "perks_csr": pk.Csr, "perks_shape": pk.Shape,
               "perks_device_info": pk.DeviceInfo}
    lines = ['#include <stddef.h>', '#include <stdio.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
