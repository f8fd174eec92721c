"""The C-ABI boundary on the CPU: symbols, struct layout, host-side validation (no GPU).

Every validation error is returned before any HIP call, so these run without a device.
"""

import ctypes
import os
import re
import subprocess

import pytest

from paper_2003_09468_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc_kpt.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.library_path()):
        from paper_2003_09468_amd import build
        build.build()
    return B.lib()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(afqmc_kpt_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert set(names) == set(B.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", B.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (afqmc_kpt_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_struct_layout_matches_header(tmp_path):
    fields = [f for f, _ in B.Problem._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
           'printf("size %zu\\n", sizeof(afqmc_kpt_problem));']
    for f in fields:
        src.append(f'printf("{f} %zu\\n", offsetof(afqmc_kpt_problem, {f}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    assert int(got["size"]) == ctypes.sizeof(B.Problem)
    for f in fields:
        assert int(got[f]) == getattr(B.Problem, f).offset, f


def good_problem():
    p = B.Problem()
    p.mesh[0], p.mesh[1], p.mesh[2] = 3, 3, 3
    p.nk, p.m, p.nocc, p.nchol, p.nwalk = 27, 26, 4, 208, 64
    p.prec, p.dt = 0, 0.005
    addr = 0x10000
    for name in ("L", "A", "Lh", "h1h", "bhalf", "L32", "Lh32", "U", "Gh", "logdet", "weight",
                 "status"):
        setattr(p, name, addr)
        addr += 0x10000
    return p


def call(L, name, p, *args):
    f = getattr(L, name)
    return f(ctypes.byref(p), 1, *args)


def test_workspace_sizes_positive_and_stable(L):
    p = good_problem()
    out = ctypes.c_size_t()
    sizes = []
    for e in range(8):
        assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, e, ctypes.byref(out)) == 0
        sizes.append(out.value)
        assert out.value % 256 == 0
    assert all(s > 0 for s in sizes)
    assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 8, ctypes.byref(out)) == -1
    assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 0, None) == -2


@pytest.mark.parametrize("field,value,code", [
    ("nk", 26, -1),       # nk != prod(mesh)
    ("nocc", 27, -1),     # nocc > m
    ("m", 0, -1),
    ("nchol", 0, -1),
    ("nwalk", 0, -1),
    ("prec", 5, -1),
    ("dt", -0.1, -1),
    ("dt", float("nan"), -1),
    ("nocc", 17, -7),     # beyond the exchange kernel (needs m >= 17: set below)
])
def test_bad_dimensions(L, field, value, code):
    p = good_problem()
    if field == "nocc" and value == 17:
        p.m = 40
    setattr(p, field, value)
    ws = ctypes.c_void_p(0x100000)
    assert call(L, "afqmc_kpt_greens", p, ws, 1 << 40, None) == code
    assert call(L, "afqmc_kpt_energy", p, ctypes.c_void_p(0x2000), ws, 1 << 40, None) == code


def test_unsupported_sizes(L):
    p = good_problem()
    p.mesh[0], p.mesh[1], p.mesh[2], p.nk, p.m = 4, 4, 4, 64, 52  # nk*nocc = 256 > 128
    assert call(L, "afqmc_kpt_greens", p, ctypes.c_void_p(0x100000), 1 << 40, None) == -7
    p = good_problem()
    p.m = 65
    assert call(L, "afqmc_kpt_energy", p, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000),
                1 << 40, None) == -7


def test_null_and_alignment(L):
    ws = ctypes.c_void_p(0x100000)
    p = good_problem()
    p.Gh = None
    assert call(L, "afqmc_kpt_greens", p, ws, 1 << 40, None) == -2
    p = good_problem()
    p.U = 0x10008  # not 16-byte aligned
    assert call(L, "afqmc_kpt_greens", p, ws, 1 << 40, None) == -3
    p = good_problem()
    assert call(L, "afqmc_kpt_vbias", p, None, None, ws, 1 << 40, None) == -2
    assert L.afqmc_kpt_greens(None, 1, ws, 1 << 40, None) == -2
    assert L.afqmc_kpt_greens(ctypes.byref(p), 0, ws, 1 << 40, None) == -1
    # FP32 needs the complex64 copies
    p = good_problem()
    p.prec = 1
    p.Lh32 = None
    assert call(L, "afqmc_kpt_energy", p, ctypes.c_void_p(0x2000), ws, 1 << 40, None) == -2
    # propagate rejects unknown flags
    p = good_problem()
    assert call(L, "afqmc_kpt_propagate", p, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000),
                ctypes.c_void_p(0x4000), 2, ws, 1 << 40, None) == -1


def test_workspace_checks(L):
    p = good_problem()
    out = ctypes.c_size_t()
    L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 6, ctypes.byref(out))
    need = out.value
    E = ctypes.c_void_p(0x2000)
    assert call(L, "afqmc_kpt_energy", p, E, None, need, None) == -4
    assert call(L, "afqmc_kpt_energy", p, E, ctypes.c_void_p(0x100000), need - 1, None) == -4
    assert call(L, "afqmc_kpt_energy", p, E, ctypes.c_void_p(0x100010), need, None) == -3


def test_strerror_and_version(L):
    for code in range(-7, 1):
        assert isinstance(L.afqmc_kpt_strerror(code), bytes)
    assert L.afqmc_kpt_strerror(-99) == b"unknown status"
    assert b"gfx950" in L.afqmc_kpt_version()


def test_no_device_reported_after_validation(L):
    """With valid arguments the first HIP call is the device check: ENODEV without a GPU."""
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    p = good_problem()
    assert call(L, "afqmc_kpt_greens", p, ctypes.c_void_p(0x100000), 1 << 40, None) == -5


def test_product_path_has_no_cpu_fallback():
    """The binding imports nothing from the oracle and needs the built library."""
    import paper_2003_09468_amd.binding as mod
    src = open(mod.__file__).read()
    assert "oracle" not in src and "numpy" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2003_09468_amd")):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_2003_09468_amd", f)).read()
