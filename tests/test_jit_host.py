"""Host-side checks of the runtime stencil compiler (no GPU needed: hipRTC
compiles for gfx950 on the host): programs that parse compile, every
malformed program the interpreter rejects is rejected with a position, and
the generated kernel reads each (field, dx, dy) column once per level."""

import re

import pytest
import torch

from oracle import stencil_lang as sl
from stencil_programs import JACOBI, advection, random_program

import paper_2310_01882_amd as ms


def test_jacobi_program_compiles_with_its_signature():
    j = ms.JitStencil(JACOBI)
    assert (j.fields, j.params, j.profiles, j.outputs) == (["u", "f"], [], [], ["v"])
    src = j.source
    assert "typedef double T;" in src
    scalar = src[src.index("ms_jit_kernel_s"):src.index("ms_jit_kernel_v")]
    vector = src[src.index("ms_jit_kernel_v"):]
    # scalar kernel: six (field, dx, dy) columns: u at x+-1, y+-1, the
    # centre column, and f
    assert len(re.findall(r"const T\* __restrict__ c\d+ =", scalar)) == 6
    # vector kernel, two rows per lane: six rows (u at rows -1, 0, 1, 2 and
    # f at rows 0, 1); x neighbours by DPP for u's two own rows, in each of
    # the two unrolled steps
    assert len(re.findall(r"const T\* __restrict__ c\d+ =", vector)) == 6
    assert vector.count("ms_from_left(") == 4 and vector.count("ms_from_right(") == 4
    assert "ext_vector_type(2)" in src
    # the constant is the double nearest 1/6, as a hex literal
    assert "0x1.5555555555555p-3" in src


def test_float32_program_and_the_advection_program_compile():
    j = ms.JitStencil(JACOBI, dtype=torch.float32)
    assert "typedef float T;" in j.source and "0x1.555556p-3f" in j.source
    assert "ext_vector_type(4)" in j.source
    a = ms.JitStencil(advection())
    assert a.fields == ["u", "v", "w"] and a.params == ["tcx", "tcy"]
    assert a.profiles == ["tzc1", "tzc2"] and a.outputs == ["su", "sv", "sw"]


@pytest.mark.parametrize("seed", range(3))
def test_random_programs_compile(seed):
    text = random_program(seed)
    sl.parse(text)
    j = ms.JitStencil(text, dtype=torch.float32 if seed % 2 else torch.float64)
    assert j.outputs == ["o0", "o1"]


@pytest.mark.parametrize("bad", ["field u; out v = u[2,0,0];", "field u; out v = w;",
                                 "field u; out v = u + ;", "field u out v = u;",
                                 "field u; out v = 1e999;", "field u; param u; out v = u;",
                                 "field u; let a = u; out v = a[1,0,0];", "field u;",
                                 "field u; out v = 1x;", "field u; out o = u; out p = o;",
                                 "field let; out o = 1;", "field u; out v = u[1,0];"])
def test_malformed_programs_are_rejected_by_both(bad):
    with pytest.raises(ValueError):
        sl.parse(bad)
    with pytest.raises(ms.MsError) as e:
        ms.JitStencil(bad)
    assert e.value.code == ms.MS_EINVAL and "line 1 col" in str(e.value)


def test_limits_and_bad_arguments():
    many = "field " + ", ".join(f"f{i}" for i in range(9)) + "; out o = f0;"
    with pytest.raises(ms.MsError, match="too many field"):
        ms.JitStencil(many)
    with pytest.raises(ms.MsError, match="line 3 col"):
        ms.JitStencil("field u;\n# comment\nout o = u * ;")
    with pytest.raises(ms.MsError):
        ms.JitStencil("out o = " + "(" * 300 + "1" + ")" * 300 + ";")
    j = ms.JitStencil(JACOBI)
    assert ms.lib.ms_jit_name(j._h, ms.MS_JIT_FIELD, 2) is None
    assert ms.lib.ms_jit_name(j._h, 7, 0) is None
    rc = ms.lib.ms_jit_compile(b"out o = 1;", 5, ms.ctypes.byref(ms.ctypes.c_void_p()))
    assert rc == ms.MS_EUNSUPPORTED
