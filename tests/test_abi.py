"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/lsr.h declares, its struct layouts match a C compiler's, and the argument
validation lsr_run applies (through lsr_check_args) rejects every invalid case."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1609_04567_amd as L
from paper_1609_04567_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsr.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lsr_status|const char \*)\s*(lsr_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 10
    lib = C.CDLL(N.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(N._SIGS), "binding and header disagree"


def test_version_and_last_error_without_device():
    assert "gfx950" in L.lsr_version()
    assert isinstance(L.lsr_last_error(), str)


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lsr.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lsr_grid), sizeof(lsr_cond),'
                   ' sizeof(lsr_config), sizeof(lsr_job_result), sizeof(lsr_tuning),'
                   ' offsetof(lsr_grid, param), offsetof(lsr_job_result, device_ms));return 0;}')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(N.lsr_grid), C.sizeof(N.lsr_cond), C.sizeof(N.lsr_config),
            C.sizeof(N.lsr_job_result), C.sizeof(N.lsr_tuning), N.lsr_grid.param.offset,
            N.lsr_job_result.device_ms.offset]
    assert got == want


FAKE = 0x10000  # never dereferenced: validation only looks at the descriptor


def _g(rows=64, cols=64, pitch=None, dtype=L.LSR_F64, bc=L.LSR_BC_RING, env0=None, param=(1.0, 0.1)):
    return L.make_grid(FAKE, rows, cols, pitch or cols, dtype, bc, env0, param)


def _c(kind=L.LSR_COND_BELOW, thr=1e-6, every=1, window=10):
    return L.make_cond(kind, thr, every, window)


def _sep(dtype=L.LSR_F64, env1=True, param=(1.0, 0.1, 20.7, 0.01)):
    g = _g(dtype=dtype, env0=FAKE, param=param)
    g.env1 = FAKE if env1 else None
    return g


VALID = [
    (_g(), L.LSR_ST_LAPLACE5, L.LSR_RED_MAX_ABS_DELTA, _c()),
    (_g(dtype=L.LSR_F32), L.LSR_ST_LAPLACE5, L.LSR_RED_L2_DELTA, _c(L.LSR_COND_NEVER)),
    (_g(env0=FAKE), L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, _c(every=10)),
    (_g(dtype=L.LSR_F32, env0=FAKE), L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, _c(every=10)),
    # alpha h^2 = 4 and -4/3: the ends of the FP32 form's range; FP64 takes any finite 1/(4 + alpha h^2)
    (_g(dtype=L.LSR_F32, env0=FAKE, param=(4.0, 1.0)), L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, _c()),
    (_g(dtype=L.LSR_F32, env0=FAKE, param=(-4.0 / 3.0, 1.0)), L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA,
     _c()),
    (_g(env0=FAKE, param=(100.0, 1.0)), L.LSR_ST_HELMHOLTZ5, L.LSR_RED_L2_DELTA, _c()),
    (_g(dtype=L.LSR_U8, bc=L.LSR_BC_TORUS), L.LSR_ST_LIFE, L.LSR_RED_SUM, _c(L.LSR_COND_STABLE_FOR)),
    (_g(1, 1, dtype=L.LSR_U8, bc=L.LSR_BC_BOTTOM), L.LSR_ST_LIFE, L.LSR_RED_SUM, _c(L.LSR_COND_NEVER)),
    (_g(dtype=L.LSR_F32, bc=L.LSR_BC_BOTTOM, env0=FAKE, param=(100.0,)), L.LSR_ST_RESTORE,
     L.LSR_RED_MEAN_ABS_DELTA, _c(thr=0.1)),
    (_g(1, 1, dtype=L.LSR_U8, bc=L.LSR_BC_BOTTOM), L.LSR_ST_SOBEL, L.LSR_RED_SUM, _c(L.LSR_COND_NEVER)),
    (_sep(), L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_L2_DELTA, _c(every=10)),
    (_sep(dtype=L.LSR_F32), L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_MAX_ABS_DELTA, _c()),
    (_g(9, 9, param=(4.0,)), L.LSR_ST_BOX, L.LSR_RED_MAX_ABS_DELTA, _c()),
    (_g(dtype=L.LSR_F32, param=(1.0,)), L.LSR_ST_BOX, L.LSR_RED_L2_DELTA, _c(L.LSR_COND_NEVER)),
    (_g(12, 5, param=(4.0,)), L.LSR_ST_LAPLACE7_3D, L.LSR_RED_MAX_ABS_DELTA, _c()),
    (_g(9, 3, dtype=L.LSR_F32, param=(3.0,)), L.LSR_ST_LAPLACE7_3D, L.LSR_RED_MEAN_ABS_DELTA, _c()),
]


@pytest.mark.parametrize("i", range(len(VALID)))
def test_valid_combinations(i):
    g, st, red, cond = VALID[i]
    assert L.lsr_check_args(g, st, red, cond, 100) == L.LSR_OK, L.lsr_last_error()


INVALID = [
    ("null data", L.make_grid(0, 8, 8, 8, L.LSR_F64, L.LSR_BC_RING), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("pitch < cols", _g(pitch=10), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("rows < 3", _g(rows=2), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("cols < 3", _g(cols=2), L.LSR_ST_HELMHOLTZ5, 2, _c(), 10),
    ("u8 jacobi", _g(dtype=L.LSR_U8), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("torus jacobi", _g(bc=L.LSR_BC_TORUS), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("helmholtz no env", _g(), L.LSR_ST_HELMHOLTZ5, 2, _c(), 10),
    ("f32 helmholtz alpha h^2 > 4", _g(dtype=L.LSR_F32, env0=FAKE, param=(4.5, 1.0)),
     L.LSR_ST_HELMHOLTZ5, 2, _c(), 10),
    ("f32 helmholtz alpha h^2 < -4/3", _g(dtype=L.LSR_F32, env0=FAKE, param=(-1.5, 1.0)),
     L.LSR_ST_HELMHOLTZ5, 2, _c(), 10),
    ("laplace with env", _g(env0=FAKE), L.LSR_ST_LAPLACE5, 1, _c(), 10),
    ("jacobi sum reduce", _g(), L.LSR_ST_LAPLACE5, L.LSR_RED_SUM, _c(), 10),
    ("jacobi stable cond", _g(), L.LSR_ST_LAPLACE5, 1, _c(L.LSR_COND_STABLE_FOR), 10),
    ("check_every 0", _g(), L.LSR_ST_LAPLACE5, 1, _c(every=0), 10),
    ("max_iter 0", _g(), L.LSR_ST_LAPLACE5, 1, _c(), 0),
    ("nan threshold", _g(), L.LSR_ST_LAPLACE5, 1, _c(thr=float("nan")), 10),
    ("f64 life", _g(bc=L.LSR_BC_TORUS), L.LSR_ST_LIFE, L.LSR_RED_SUM, _c(L.LSR_COND_STABLE_FOR), 10),
    ("ring life", _g(dtype=L.LSR_U8), L.LSR_ST_LIFE, L.LSR_RED_SUM, _c(L.LSR_COND_STABLE_FOR), 10),
    ("life max reduce", _g(dtype=L.LSR_U8, bc=L.LSR_BC_TORUS), L.LSR_ST_LIFE, 1,
     _c(L.LSR_COND_STABLE_FOR), 10),
    ("life window 0", _g(dtype=L.LSR_U8, bc=L.LSR_BC_TORUS), L.LSR_ST_LIFE, L.LSR_RED_SUM,
     _c(L.LSR_COND_STABLE_FOR, window=0), 10),
    ("life below", _g(dtype=L.LSR_U8, bc=L.LSR_BC_TORUS), L.LSR_ST_LIFE, L.LSR_RED_SUM, _c(), 10),
    ("restore no mask", _g(bc=L.LSR_BC_BOTTOM, param=(100.0,)), L.LSR_ST_RESTORE, 1, _c(), 10),
    ("restore ring", _g(env0=FAKE, param=(100.0,)), L.LSR_ST_RESTORE, 1, _c(), 10),
    ("restore beta 0", _g(bc=L.LSR_BC_BOTTOM, env0=FAKE, param=(0.0,)), L.LSR_ST_RESTORE, 1, _c(), 10),
    ("restore l2", _g(bc=L.LSR_BC_BOTTOM, env0=FAKE, param=(100.0,)), L.LSR_ST_RESTORE, 2, _c(), 10),
    ("sobel f64", _g(bc=L.LSR_BC_BOTTOM), L.LSR_ST_SOBEL, L.LSR_RED_SUM, _c(L.LSR_COND_NEVER), 1),
    ("sobel torus", _g(dtype=L.LSR_U8, bc=L.LSR_BC_TORUS), L.LSR_ST_SOBEL, L.LSR_RED_SUM,
     _c(L.LSR_COND_NEVER), 1),
    ("sobel max reduce", _g(dtype=L.LSR_U8, bc=L.LSR_BC_BOTTOM), L.LSR_ST_SOBEL, 1,
     _c(L.LSR_COND_NEVER), 1),
    ("sobel below", _g(dtype=L.LSR_U8, bc=L.LSR_BC_BOTTOM), L.LSR_ST_SOBEL, L.LSR_RED_SUM, _c(), 1),
    ("sobel env", _g(dtype=L.LSR_U8, bc=L.LSR_BC_BOTTOM, env0=FAKE), L.LSR_ST_SOBEL, L.LSR_RED_SUM,
     _c(L.LSR_COND_NEVER), 1),
    ("sep without q", _sep(env1=False), L.LSR_ST_HELMHOLTZ5_SEP, 2, _c(), 10),
    ("sep without p", _g(), L.LSR_ST_HELMHOLTZ5_SEP, 2, _c(), 10),
    ("sep nan c1", _sep(param=(1.0, 0.1, float("nan"), 1.0)), L.LSR_ST_HELMHOLTZ5_SEP, 2, _c(), 10),
    ("sep f32 alpha h^2 > 4", _sep(dtype=L.LSR_F32, param=(4.5, 1.0, 1.0, 1.0)),
     L.LSR_ST_HELMHOLTZ5_SEP, 2, _c(), 10),
    ("sep sum reduce", _sep(), L.LSR_ST_HELMHOLTZ5_SEP, L.LSR_RED_SUM, _c(), 10),
    ("env1 on helmholtz", _sep(), L.LSR_ST_HELMHOLTZ5, 2, _c(), 10),
    ("box radius 5", _g(param=(5.0,)), L.LSR_ST_BOX, 1, _c(), 10),
    ("box radius 1.5", _g(param=(1.5,)), L.LSR_ST_BOX, 1, _c(), 10),
    ("box too small", _g(8, 8, param=(4.0,)), L.LSR_ST_BOX, 1, _c(), 10),
    ("box u8", _g(dtype=L.LSR_U8, param=(1.0,)), L.LSR_ST_BOX, 1, _c(), 10),
    ("box torus", _g(bc=L.LSR_BC_TORUS, param=(1.0,)), L.LSR_ST_BOX, 1, _c(), 10),
    ("3d ny not dividing", _g(10, 5, param=(4.0,)), L.LSR_ST_LAPLACE7_3D, 1, _c(), 10),
    ("3d nz < 3", _g(8, 5, param=(4.0,)), L.LSR_ST_LAPLACE7_3D, 1, _c(), 10),
    ("3d ny < 3", _g(8, 5, param=(2.0,)), L.LSR_ST_LAPLACE7_3D, 1, _c(), 10),
    ("3d sum reduce", _g(12, 5, param=(4.0,)), L.LSR_ST_LAPLACE7_3D, L.LSR_RED_SUM, _c(), 10),
    ("unknown stencil", _g(), 99, 1, _c(), 10),
    ("env1 set", None, L.LSR_ST_LAPLACE5, 1, _c(), 10),
]


@pytest.mark.parametrize("case", INVALID, ids=[c[0] for c in INVALID])
def test_invalid_arguments_are_rejected(case):
    name, g, st, red, cond, mi = case
    if g is None:
        g = _g()
        g.env1 = FAKE
    assert L.lsr_check_args(g, st, red, cond, mi) == L.LSR_EINVAL
    assert len(L.lsr_last_error()) > 0


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(L.LsrError) as ei:
        L.lsr_create(0)
    assert ei.value.status in (L.LSR_EDEVICE, L.LSR_EINVAL)
