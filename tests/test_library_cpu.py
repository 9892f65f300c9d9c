"""Host-side checks of the C ABI (no device work): every entry point declared in
include/hfdib.h is exported by the built library, defaults, workspace sizing and
argument validation, call-order errors."""

import ctypes as C
import os
import re

import pytest

import synth
from paper_2606_06135_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hfdib.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hfdib_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(hiplib):
    names = _declared()
    assert "hfdib_init_grid" in names and "hfdib_simple_iterate" in names
    for n in names:
        assert hasattr(hiplib, n), f"{n} declared in include/hfdib.h but not exported"
    assert sorted(B.EXPORTED) == names


def test_abi_version_and_defaults(hiplib):
    assert hiplib.hfdib_abi_version() == 4
    c = B.default_config()
    assert c.abi_version == 4 and c.n_sweeps == 2 and c.recorrect == 1 and c.continuity == 0
    assert c.yplus_dist == 0 and c.conv_scheme == 0
    # the library's defaults are the constants the oracle receives
    for n in B._CONST_NAMES:
        assert getattr(c, n) == synth.DEFAULT_CONSTANTS[n], n
    assert (c.urf_u, c.urf_p, c.urf_t) == (0.7, 0.3, 0.85)
    assert (c.Cmu, c.kappa, c.E, c.ylam) == (0.09, 0.41, 9.8, 11.0)


def _ws(d, c):
    n = C.c_size_t(0)
    st = B.lib().hfdib_workspace_bytes(C.byref(d), C.byref(c), C.byref(n))
    return st, n.value


def test_workspace_bytes_scale_with_grid(hiplib):
    d1, c1 = B.make_desc_config(synth.case_bfs(nx=80, ny=20))
    d2, c2 = B.make_desc_config(synth.case_bfs(nx=160, ny=40))
    st1, n1 = _ws(d1, c1)
    st2, n2 = _ws(d2, c2)
    assert st1 == 0 and st2 == 0
    assert n2 > 3.5 * n1 > 0
    # about 50 FP64 arrays per cell
    assert 40 * 8 * 6400 < n2 < 120 * 8 * 6400


def test_mixed_workspace_adds_fp32_arrays(hiplib):
    """The mixed policy adds FP32 defects, corrections and mirrors (about 16
    N-sized FP32 arrays incl. faces) and stores the coarse levels in FP32; it
    has no FP64 colour-split copies of the pressure correction, its residual,
    u, v, w and the transported scalar (6 arrays of N doubles on this even
    grid), which its FP32 correction sweeps do not use."""
    spec = synth.case_bfs(nx=160, ny=40)
    d, c = B.make_desc_config(spec)
    dm, cm = B.make_desc_config(spec, precision="mixed")
    st, n64 = _ws(d, c)
    stm, nmx = _ws(dm, cm)
    assert st == 0 and stm == 0
    N = spec.ncells
    assert 12 * 4 * N < nmx - n64 + 6 * 8 * N < 20 * 4 * N


@pytest.mark.parametrize("mutate", [
    lambda d, c: setattr(d, "dim", 4),
    lambda d, c: setattr(d, "nx", 2),
    lambda d, c: setattr(d, "dx", -1.0),
    lambda d, c: d.bc.__setitem__(4, 0),          # 2D grid with a non-empty z face
    lambda d, c: d.bc.__setitem__(0, 9),
    lambda d, c: setattr(c, "urf_u", 1.5),
    lambda d, c: setattr(c, "nu", 0.0),
    lambda d, c: setattr(c, "n_sweeps", 0),
    lambda d, c: setattr(c, "precision", 2),
    lambda d, c: setattr(c, "continuity", 7),
    lambda d, c: setattr(c, "yplus_dist", 2),
    lambda d, c: setattr(c, "conv_scheme", 3),
    lambda d, c: setattr(c, "model", 5),
    lambda d, c: setattr(c, "abi_version", 99),
])
def test_invalid_arguments_rejected(hiplib, mutate):
    d, c = B.make_desc_config(synth.case_bfs(nx=80, ny=20))
    mutate(d, c)
    st, _ = _ws(d, c)
    assert st == -1


def test_init_validation_and_call_order(hiplib):
    L = B.lib()
    d, c = B.make_desc_config(synth.case_bfs(nx=80, ny=20))
    st, need = _ws(d, c)
    assert st == 0
    fake = C.c_void_p(1 << 20)  # aligned host-side stand-in: init enqueues no device work
    ctx = C.c_void_p()
    assert L.hfdib_init_grid(C.byref(d), C.byref(c), fake, need - 1, None, C.byref(ctx)) == -2
    assert L.hfdib_init_grid(C.byref(d), C.byref(c), C.c_void_p((1 << 20) + 8), need, None, C.byref(ctx)) == -1
    assert L.hfdib_init_grid(C.byref(d), C.byref(c), fake, need, None, C.byref(ctx)) == 0
    done = C.c_int(-1)
    assert L.hfdib_simple_iterate(ctx, 1, 0.0, 0, C.byref(done), None) == -5
    assert b"set_indicator" in L.hfdib_last_error(ctx)
    counts = (C.c_int * 3)()
    assert L.hfdib_get_counts(ctx, counts) == -5
    assert L.hfdib_status_string(-4) == b"diverged"
    # kernel timing: a recording period >= 1, or 0 (off); host-side state only
    assert L.hfdib_timing_enable(ctx, -1) == -1
    assert L.hfdib_timing_enable(ctx, 3) == 0 and L.hfdib_timing_enable(ctx, 0) == 0
    L.hfdib_destroy(ctx)
