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
    for e in range(10):
        assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, e, ctypes.byref(out)) == 0
        sizes.append(out.value)
        assert out.value % 256 == 0
    assert all(s > 0 for s in sizes)
    # population control holds a copy of U and Gh
    assert sizes[9] >= 2 * 16 * 64 * (27 * 26) * (27 * 4)
    assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 10, ctypes.byref(out)) == -1
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
    p.mesh[0], p.mesh[1], p.mesh[2], p.nk, p.m, p.nocc = 4, 4, 4, 64, 52, 5  # nk*nocc > 256
    assert call(L, "afqmc_kpt_greens", p, ctypes.c_void_p(0x100000), 1 << 40, None) == -7
    assert call(L, "afqmc_kpt_orthonormalize", p, ctypes.c_void_p(0x100000), 1 << 40,
                None) == -7
    assert call(L, "afqmc_kpt_propagate", p, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000),
                ctypes.c_void_p(0x4000), 1, ctypes.c_void_p(0x100000), 1 << 40, None) == -7
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
        assert L.afqmc_kpt_strerror(code) != b"unknown status"
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


# ---------------------------------------------------------------------------
# batches: packed buffers, the step block, the captured block and the autotuner

def two_problems():
    a, b = good_problem(), good_problem()
    b.mesh[0], b.mesh[1], b.mesh[2], b.nk, b.m, b.nchol, b.nwalk = 2, 2, 2, 8, 26, 208, 128
    b.prec = 1
    arr = (B.Problem * 2)(a, b)
    return arr


def one_slice(p, buf):
    W, nk, C = p.nwalk, p.nk, p.nchol
    N, n = nk * p.m, nk * p.nocc
    return {0: 8 * W * nk * C * 2, 1: 16 * W * nk * C * 2, 2: 16 * W * nk * C,
            3: (8 if p.prec == 1 else 16) * W * N * N, 4: 48 * W, 5: 16 * W,
            6: 16 * W * n * N}[buf]


@pytest.mark.parametrize("buf", range(7))
def test_buffer_layout_packs_problems(L, buf):
    arr = two_problems()
    off = (ctypes.c_size_t * 3)()
    assert L.afqmc_kpt_buffer_layout(arr, 2, buf, off) == 0
    s0, s1 = one_slice(arr[0], buf), one_slice(arr[1], buf)
    assert off[0] == 0
    assert off[1] % 256 == 0 and s0 <= off[1] < s0 + 256
    assert off[2] == off[1] + s1
    assert L.afqmc_kpt_buffer_layout(arr, 2, 7, off) == -1
    assert L.afqmc_kpt_buffer_layout(arr, 2, buf, None) == -2


def test_batch_workspace_is_sum_of_parts(L):
    arr = two_problems()
    out = ctypes.c_size_t()
    for e in range(9):
        parts = []
        for i in range(2):
            assert L.afqmc_kpt_workspace_bytes(ctypes.byref(arr[i]), 1, e, ctypes.byref(out)) == 0
            parts.append(out.value)
        assert L.afqmc_kpt_workspace_bytes(arr, 2, e, ctypes.byref(out)) == 0
        assert out.value == sum(parts)


def test_batch_validates_every_problem(L):
    arr = two_problems()
    arr[1].nocc = 30  # > m
    ws = ctypes.c_void_p(0x100000)
    assert L.afqmc_kpt_greens(arr, 2, ws, 1 << 40, None) == -1
    arr = two_problems()
    arr[1].Lh32 = None  # FP32 system without its complex64 copy
    assert L.afqmc_kpt_energy(arr, 2, ctypes.c_void_p(0x2000), ws, 1 << 40, None) == -2


def step_args(**kw):
    a = dict(x=0x2000, nsteps=10, xbar=0x4000, vhs=0x8000, E=0xc000, flags=3, ws=0x100000,
             nbytes=1 << 40)
    a.update(kw)
    return a


def call_step(L, arr, n, a):
    return L.afqmc_kpt_step(arr, n, a["x"], a["nsteps"], a["xbar"], a["vhs"], a["E"], a["flags"],
                            a["ws"], a["nbytes"], None)


def test_step_validation(L):
    arr = two_problems()
    assert call_step(L, arr, 2, step_args(nsteps=0)) == -1
    assert call_step(L, arr, 2, step_args(flags=4)) == -1
    assert call_step(L, arr, 2, step_args(xbar=None)) == -2
    assert call_step(L, arr, 2, step_args(vhs=0x8008)) == -3
    assert call_step(L, arr, 2, step_args(E=None)) == -2           # energy requested
    assert call_step(L, arr, 2, step_args(ws=None)) == -4
    assert call_step(L, arr, 2, step_args(nbytes=256)) == -4
    h = ctypes.c_void_p()
    a = step_args()
    assert L.afqmc_kpt_graph_create(arr, 2, a["x"], a["nsteps"], a["xbar"], a["vhs"], a["E"],
                                    a["flags"], a["ws"], a["nbytes"], None) == -2
    assert L.afqmc_kpt_graph_create(arr, 2, a["x"], 0, a["xbar"], a["vhs"], a["E"], a["flags"],
                                    a["ws"], a["nbytes"], ctypes.byref(h)) == -1
    assert h.value is None
    assert L.afqmc_kpt_graph_launch(None, None) == -2
    assert L.afqmc_kpt_graph_destroy(None) == -2
    assert L.afqmc_kpt_autotune(arr, 2, None, a["ws"], a["nbytes"], None) == -2
    assert L.afqmc_kpt_autotune(arr, 2, a["vhs"], a["ws"], 256, None) == -4


def test_step_reaches_device_check(L):
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    arr = two_problems()
    assert call_step(L, arr, 2, step_args()) == -5
    assert call_step(L, arr, 2, step_args(E=None, flags=1)) == -5  # no energy: E unused
    h = ctypes.c_void_p()
    a = step_args()
    assert L.afqmc_kpt_graph_create(arr, 2, a["x"], a["nsteps"], a["xbar"], a["vhs"], a["E"],
                                    a["flags"], a["ws"], a["nbytes"], ctypes.byref(h)) == -5
    assert L.afqmc_kpt_autotune(arr, 2, a["vhs"], a["ws"], a["nbytes"], None) == -5


def test_mixed_energy_validation(L):
    arr = two_problems()
    assert L.afqmc_kpt_mixed_energy(arr, 2, None, ctypes.c_void_p(0x2000), None) == -2
    assert L.afqmc_kpt_mixed_energy(arr, 2, ctypes.c_void_p(0x2008), ctypes.c_void_p(0x2000),
                                    None) == -3
    arr[1].weight = None
    assert L.afqmc_kpt_mixed_energy(arr, 2, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x4000),
                                    None) == -2


def test_population_control_validation(L):
    p = good_problem()
    out = ctypes.c_size_t()
    assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 9, ctypes.byref(out)) == 0
    need = out.value
    ws = ctypes.c_void_p(0x1000000)
    f = L.afqmc_kpt_population_control

    def xs(v):
        return (ctypes.c_double * 1)(v)

    assert f(ctypes.byref(p), 1, None, None, ws, need, None) == -2
    for bad in (1.0, -0.25, float("nan"), float("inf")):
        assert f(ctypes.byref(p), 1, xs(bad), None, ws, need, None) == -1
    misaligned = (ctypes.c_void_p * 1)(0x2002)
    assert f(ctypes.byref(p), 1, xs(0.5), misaligned, ws, need, None) == -3
    assert f(ctypes.byref(p), 1, xs(0.5), None, ws, need - 1, None) == -4
    assert f(ctypes.byref(p), 1, xs(0.5), None, None, need, None) == -4
    q = good_problem()
    q.status = None
    assert f(ctypes.byref(q), 1, xs(0.5), None, ws, need, None) == -2
    assert f(ctypes.byref(p), 0, xs(0.5), None, ws, need, None) == -1
    # valid arguments: the device check comes first (only without a GPU: the pointers
    # here are fake)
    from tests.conftest import gpu_available
    if not gpu_available():
        aligned = (ctypes.c_void_p * 1)(0x2000)
        assert f(ctypes.byref(p), 1, xs(0.0), aligned, ws, need, None) == -5
        assert f(ctypes.byref(p), 1, xs(0.999), None, ws, need, None) == -5


def bf16x3_problem():
    p = good_problem()
    p.prec = 2
    p.Lhs, p.Ls = 0xd00000, 0xe00000
    return p


def test_bf16x3_split_planes_required(L):
    """Every entry whose BF16X3 kernels read the split planes rejects NULL planes before any
    HIP call: the force bias (every step) and the Coulomb trace of the energy and its adjoint
    read Lhs, the HS potential reads Ls."""
    ws = ctypes.c_void_p(0x1000000)
    buf = [ctypes.c_void_p(0x2000 * (i + 1)) for i in range(4)]
    for missing in ("Lhs", "Ls"):
        p = bf16x3_problem()
        setattr(p, missing, None)
        if missing == "Lhs":
            assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -2
            assert call(L, "afqmc_kpt_energy", p, buf[0], ws, 1 << 40, None) == -2
            assert call(L, "afqmc_kpt_energy_backward", p, None, buf[0], ws, 1 << 40,
                        None) == -2
        else:
            assert call(L, "afqmc_kpt_vhs", p, buf[0], buf[1], buf[2], ws, 1 << 40, None) == -2
        arr = (B.Problem * 1)(p)
        # a step block without the energy still runs the force bias and the HS potential
        assert call_step(L, arr, 1, step_args(E=None, flags=1)) == -2
        h = ctypes.c_void_p()
        a = step_args(E=None, flags=1)
        assert L.afqmc_kpt_graph_create(arr, 1, a["x"], a["nsteps"], a["xbar"], a["vhs"],
                                        a["E"], a["flags"], a["ws"], a["nbytes"],
                                        ctypes.byref(h)) == -2
        assert L.afqmc_kpt_autotune(arr, 1, a["vhs"], a["ws"], a["nbytes"], None) == -2
    # an FP64 problem never reads the planes: NULL is fine up to the device check
    from tests.conftest import gpu_available
    if not gpu_available():
        p = good_problem()
        assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -5
        p = bf16x3_problem()
        assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -5



def test_placed_precision_encoding(L):
    """AFQMC_PREC_PLACE(step, energy) is accepted for every pair of precisions; other bits,
    step values above BF16X3 and energy codes above BF16X3 + 1 are rejected."""
    ws = ctypes.c_void_p(0x1000000)
    out = ctypes.c_size_t()
    for sp in range(3):
        for ep in range(3):
            p = good_problem()
            p.prec = B.prec_place(sp, ep)
            assert B.step_prec(p.prec) == sp and B.energy_prec(p.prec) == ep
            assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 8, ctypes.byref(out)) == 0
    for bad in (3, 4, 15, B.prec_place(0, 5), B.prec_place(3, 0), 0x80, 0x100, -1):
        p = good_problem()
        p.prec = bad
        assert call(L, "afqmc_kpt_greens", p, ws, 1 << 40, None) == -1, bad
    # a plain value is its own step and energy precision
    assert B.step_prec(2) == 2 and B.energy_prec(2) == 2


def test_placed_precision_workspaces(L):
    """Each stage is sized in its own precision: the step workspace of BF16X3 propagation
    with an FP64 energy is the larger of the BF16X3 step stages and the FP64 energy; the
    energy and adjoint entries are sized as FP64, the propagation as BF16X3; the HS
    potential buffer is complex64 (BF16X3 step)."""
    def ws(prec, entry):
        p = good_problem()
        p.prec = prec
        out = ctypes.c_size_t()
        assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, entry, ctypes.byref(out)) == 0
        return out.value
    pl = B.prec_place(2, 0)
    for e in (B.ENTRIES["energy"], B.ENTRIES["energy_backward"]):
        assert ws(pl, e) == ws(0, e)
    for e in (B.ENTRIES["propagate"], B.ENTRIES["vhs"], B.ENTRIES["vbias"]):
        assert ws(pl, e) == ws(2, e)
    step = B.ENTRIES["step"]
    assert ws(pl, step) == max([ws(2, B.ENTRIES[e]) for e in ("vbias", "vhs", "propagate")]
                               + [ws(0, B.ENTRIES["energy"])])
    for prec, nb in ((pl, 8), (B.prec_place(0, 2), 16), (0, 16), (2, 8)):
        p = good_problem()
        p.prec = prec
        off = (ctypes.c_size_t * 2)()
        assert L.afqmc_kpt_buffer_layout(ctypes.byref(p), 1, 3, off) == 0
        assert off[1] == nb * 64 * (27 * 26) ** 2


def test_placed_precision_checks_each_stage(L):
    """With BF16X3 propagation and an FP64 energy the energy entries need neither split
    planes nor complex64 copies, the step entries need the BF16X3 planes; with an FP64 step
    and a BF16X3 energy it is the other way round."""
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("the device check would pass and launch")
    ws = ctypes.c_void_p(0x1000000)
    buf = [ctypes.c_void_p(0x2000 * (i + 1)) for i in range(4)]
    p = good_problem()
    p.prec = B.prec_place(2, 0)
    p.Lh32 = p.Lhs = p.Ls = None
    assert call(L, "afqmc_kpt_energy", p, buf[0], ws, 1 << 40, None) == -5
    assert call(L, "afqmc_kpt_energy_backward", p, None, buf[0], ws, 1 << 40, None) == -5
    assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -2
    assert call(L, "afqmc_kpt_vhs", p, buf[0], buf[1], buf[2], ws, 1 << 40, None) == -2
    p.Lh32, p.Lhs, p.Ls = 0xc00000, 0xd00000, 0xe00000
    assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -5
    arr = (B.Problem * 1)(p)
    assert call_step(L, arr, 1, step_args(E=buf[3], flags=3)) == -5
    # FP64 step, BF16X3 energy: the energy needs Lhs, the step does not
    p = good_problem()
    p.prec = B.prec_place(0, 2)
    p.Lhs = p.Ls = None
    assert call(L, "afqmc_kpt_vbias", p, buf[0], buf[1], ws, 1 << 40, None) == -5
    assert call(L, "afqmc_kpt_energy", p, buf[0], ws, 1 << 40, None) == -2
    arr = (B.Problem * 1)(p)
    assert call_step(L, arr, 1, step_args(E=None, flags=1)) == -5
    assert call_step(L, arr, 1, step_args(E=buf[3], flags=3)) == -2
    # prepare needs the union of both stages' arrays
    H1 = buf[3]
    assert call(L, "afqmc_kpt_prepare", p, H1, ws, 1 << 40, None) == -2
    p.Lhs = 0xd00000
    assert call(L, "afqmc_kpt_prepare", p, H1, ws, 1 << 40, None) == -5


def test_energy_noalloc_validation(L):
    """The entry point without a workspace validates like afqmc_kpt_energy and rejects a
    batch whose energy scratch exceeds its fixed array, all before any HIP call."""
    from tests.conftest import gpu_available
    cap = 64 << 20  # AFQMC_ENERGY_NOALLOC_MAX_BYTES
    assert f"({cap >> 20}u << 20)" in open(HEADER).read()
    E = ctypes.c_void_p(0x2000)
    p = good_problem()
    assert L.afqmc_kpt_energy_noalloc(ctypes.byref(p), 1, None, None) == -2
    assert L.afqmc_kpt_energy_noalloc(ctypes.byref(p), 1, ctypes.c_void_p(0x2008), None) == -3
    assert L.afqmc_kpt_energy_noalloc(None, 1, E, None) == -2
    assert L.afqmc_kpt_energy_noalloc(ctypes.byref(p), 0, E, None) == -1
    q = good_problem()
    q.Gh = None
    assert L.afqmc_kpt_energy_noalloc(ctypes.byref(q), 1, E, None) == -2
    # the 3x3x3, m = 26, 64-walker energy fits; twice the walkers do not
    out = ctypes.c_size_t()
    L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, 6, ctypes.byref(out))
    assert out.value <= cap
    big = good_problem()
    big.nwalk = 128
    L.afqmc_kpt_workspace_bytes(ctypes.byref(big), 1, 6, ctypes.byref(out))
    assert out.value > cap
    assert L.afqmc_kpt_energy_noalloc(ctypes.byref(big), 1, E, None) == -4
    pair = (B.Problem * 2)(good_problem(), good_problem())
    assert L.afqmc_kpt_energy_noalloc(pair, 2, E, None) == -4
    if not gpu_available():
        assert L.afqmc_kpt_energy_noalloc(ctypes.byref(p), 1, E, None) == -5


def test_reblock_matches_oracle(L):
    """The library's host blocking analysis against the oracle's: same levels and the same
    chosen level (sums in a different order: 1e-12 relative)."""
    import numpy as np
    from oracle import blocking as blk
    import paper_2003_09468_amd as lib
    rng = np.random.default_rng(2)
    for n in (2, 3, 17, 1000, 4097):
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0]
        for t in range(1, n):
            x[t] = 0.7 * x[t - 1] + e[t]
        x = 5.0 + 0.01 * x
        got, opt = lib.reblock(x)
        ref = blk.reblock(x)
        assert len(got) == len(ref)
        for (n1, m1, e1, ee1), (n2, m2, e2, ee2) in zip(got, ref):
            assert n1 == n2
            assert m1 == pytest.approx(m2, rel=1e-12)
            assert e1 == pytest.approx(e2, rel=1e-9, abs=1e-300)
            assert ee1 == pytest.approx(ee2, rel=1e-9, abs=1e-300)
        assert opt == blk.optimal_level(ref)
    got, opt = lib.reblock([4.0])
    assert got == [] and opt == -1


def test_reblock_and_etrial_validation(L):
    import numpy as np
    lv = (B.ReblockLevel * 4)()
    nl, opt = ctypes.c_int(0), ctypes.c_int(0)
    x = np.array([1.0, float("nan"), 2.0])
    assert L.afqmc_kpt_reblock(x.ctypes.data, 3, lv, 4, ctypes.byref(nl), ctypes.byref(opt)) == -1
    x = np.array([1.0, 2.0, 3.0, 4.0])
    assert L.afqmc_kpt_reblock(None, 4, lv, 4, ctypes.byref(nl), ctypes.byref(opt)) == -2
    assert L.afqmc_kpt_reblock(x.ctypes.data, 0, lv, 4, ctypes.byref(nl), ctypes.byref(opt)) == -1
    assert L.afqmc_kpt_reblock(x.ctypes.data, 4, None, 4, ctypes.byref(nl), ctypes.byref(opt)) == -2
    # a short output array: only the first levels are written, the count is complete
    assert L.afqmc_kpt_reblock(x.ctypes.data, 4, lv, 1, ctypes.byref(nl), ctypes.byref(opt)) == 0
    assert nl.value == 2 and lv[0].n == 4 and lv[1].n == 0
    # the energy shift: needs etrial and Emix, blend in (0, 1]
    p = good_problem()
    Em = ctypes.c_void_p(0x2000)
    assert call(L, "afqmc_kpt_update_etrial", p, Em, 1.0, None) == -2
    p.etrial = 0x3008
    assert call(L, "afqmc_kpt_update_etrial", p, None, 1.0, None) == -2
    for bad in (0.0, 1.5, float("nan")):
        assert call(L, "afqmc_kpt_update_etrial", p, Em, bad, None) == -1
    p.etrial = 0x3004  # not 8-byte aligned
    assert call(L, "afqmc_kpt_update_etrial", p, Em, 1.0, None) == -3
    assert call(L, "afqmc_kpt_propagate", p, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000),
                ctypes.c_void_p(0x4000), 0, ctypes.c_void_p(0x100000), 1 << 40, None) == -3


@pytest.mark.parametrize("ep", [3, 4], ids=["int8x5", "int8x4"])
def test_int8_energy_precision(L, ep):
    """INT8X5 and INT8X4 are energy precisions only: PLACE(step, INT8Xn) is valid, as a plain
    value or a step precision they are not; the energy needs the digit array Lh8 (the
    adjoint, FP64, does not); workspaces are those of FP64."""
    ws = ctypes.c_void_p(0x1000000)
    E = ctypes.c_void_p(0x2000)
    out = ctypes.c_size_t()
    for sp in range(3):
        p = good_problem()
        p.prec = B.prec_place(sp, ep)
        assert B.energy_prec(p.prec) == ep
        for e in range(10):
            assert L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, e, ctypes.byref(out)) == 0
        q = good_problem()
        q.prec = sp
        for e in (B.ENTRIES["energy"], B.ENTRIES["energy_backward"]):
            L.afqmc_kpt_workspace_bytes(ctypes.byref(q), 1, e, ctypes.byref(out))
            want = out.value
            L.afqmc_kpt_workspace_bytes(ctypes.byref(p), 1, e, ctypes.byref(out))
            if sp == 0:
                assert out.value == want
        # Lh8 missing
        assert call(L, "afqmc_kpt_energy", p, E, ws, 1 << 40, None) == -2
        assert L.afqmc_kpt_energy_noalloc(ctypes.byref(p), 1, E, None) == -2
        p.Lh8 = 0x5008  # misaligned
        assert call(L, "afqmc_kpt_energy", p, E, ws, 1 << 40, None) == -3
        p.Lh8 = 0x5000
        p.Lhs = p.Ls = 0x6000
        from tests.conftest import gpu_available
        if not gpu_available():
            assert call(L, "afqmc_kpt_energy", p, E, ws, 1 << 40, None) == -5
        # the adjoint does not read Lh8
        p.Lh8 = None
        if not gpu_available():
            assert call(L, "afqmc_kpt_energy_backward", p, None, ctypes.c_void_p(0x3000), ws,
                        1 << 40, None) == -5
    for bad in (ep, B.prec_place(ep, 0)):
        p = good_problem()
        p.prec = bad
        assert call(L, "afqmc_kpt_energy", p, E, ws, 1 << 40, None) == -1


@pytest.mark.parametrize("mesh", [(1, 1, 1), (2, 2, 2), (3, 3, 3), (4, 4, 4), (2, 3, 1),
                                  (1, 2, 3), (3, 1, 1), (2, 1, 1), (4, 3, 2)])
def test_half_store_slots(mesh):
    """The half store of L keeps one block per time-reversal pair: its slot count equals the
    number of Q whose index does not exceed that of -Q (brute force over the oracle's -Q
    table), i.e. (nk + #{Q = -Q}) / 2."""
    from oracle import kpoint as kp
    _, negq = kp.kpoint_tables(mesh)
    brute = sum(1 for Q in range(len(negq)) if Q <= negq[Q])
    assert B.ls_slots(mesh) == brute
    pairs = sum(1 for Q in range(len(negq)) if Q < negq[Q])
    assert brute == pairs + sum(1 for Q in range(len(negq)) if Q == negq[Q])


# ---------------------------------------------------------------------------
# two-determinant (collinear) walkers
# ---------------------------------------------------------------------------

def spin_pair():
    """A valid up/down pair: one system (same L), own walker arrays, different nocc."""
    a, b = good_problem(), good_problem()
    a.spin, b.spin = 1, 2
    b.nocc = 3
    addr = 0x1000000
    for name in ("A", "Lh", "h1h", "Lh32", "U", "Gh", "logdet", "weight", "status"):
        setattr(b, name, addr)
        addr += 0x10000
    return (B.Problem * 2)(a, b)


def test_spin_pair_validation(L):
    from tests.conftest import gpu_available
    ws = ctypes.c_void_p(0x10000000)
    g = L.afqmc_kpt_greens
    if not gpu_available():
        # valid: the device check is the first failure
        assert g(spin_pair(), 2, ws, 1 << 40, None) == -5
    for mutate in (
            lambda a: setattr(a[0], "spin", 3),            # no such spin
            lambda a: setattr(a[0], "spin", -1),
            lambda a: setattr(a[1], "spin", 0),            # up half without its down half
            lambda a: setattr(a[0], "spin", 2),            # down half first
            lambda a: setattr(a[1], "m", 20),              # different systems
            lambda a: setattr(a[1], "nchol", 100),
            lambda a: setattr(a[1], "nwalk", 32),
            lambda a: setattr(a[1], "prec", 1),
            lambda a: setattr(a[1], "dt", 0.01),
            lambda a: setattr(a[1], "L", 0x7770000),
            lambda a: setattr(a[1], "U", a[0].U),          # shared walker arrays
            lambda a: setattr(a[1], "weight", a[0].weight),
            lambda a: setattr(a[1], "logdet", a[0].logdet),
            lambda a: setattr(a[1], "status", a[0].status),
            lambda a: setattr(a[1], "Lh", a[0].Lh)):
        arr = spin_pair()
        mutate(arr)
        assert g(arr, 2, ws, 1 << 40, None) == -1
    arr = spin_pair()
    arr[1].mesh[2] = 1
    arr[1].nk = 9
    assert g(arr, 2, ws, 1 << 40, None) == -1
    # a lone half
    one = spin_pair()
    assert g(ctypes.byref(one[0]), 1, ws, 1 << 40, None) == -1
    assert g(ctypes.byref(one[1]), 1, ws, 1 << 40, None) == -1
    # a pair inside a larger batch, after a closed-shell problem
    arr3 = (B.Problem * 3)(good_problem(), *spin_pair())
    if not gpu_available():
        assert g(arr3, 3, ws, 1 << 40, None) == -5
    arr3 = (B.Problem * 3)(*spin_pair(), good_problem())
    arr3[2].spin = 2
    assert g(arr3, 3, ws, 1 << 40, None) == -1


def test_spin_pair_population_ignores_down_xi(L):
    """The down half draws with the up half's xi: its own entry is not read or checked."""
    from tests.conftest import gpu_available
    arr = spin_pair()
    out = ctypes.c_size_t()
    assert L.afqmc_kpt_workspace_bytes(arr, 2, 9, ctypes.byref(out)) == 0
    ws = ctypes.c_void_p(0x10000000)
    f = L.afqmc_kpt_population_control
    xs = (ctypes.c_double * 2)(0.5, float("nan"))
    if not gpu_available():
        assert f(arr, 2, xs, None, ws, out.value, None) == -5
    xs = (ctypes.c_double * 2)(1.5, 0.5)
    assert f(arr, 2, xs, None, ws, out.value, None) == -1


def test_band_padding_validation(L):
    from tests.conftest import gpu_available
    p = good_problem()
    p.mesh[0], p.mesh[1], p.mesh[2], p.nk, p.m, p.nocc = 2, 1, 1, 2, 8, 2
    mk = (ctypes.c_int32 * 2)(5, 8)
    a, b = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    f, g = L.afqmc_kpt_pad_bands, L.afqmc_kpt_unpad_bands
    n = None
    if not gpu_available():
        assert f(ctypes.byref(p), 1, mk, a, n, n, n, b, n, n, n, None) == -5
        assert g(ctypes.byref(p), 1, mk, a, n, b, n, None) == -5
    assert f(ctypes.byref(p), 1, None, a, n, n, n, b, n, n, n, None) == -2
    assert f(ctypes.byref(p), 1, mk, a, n, n, n, None, n, n, n, None) == -2  # no output
    assert f(ctypes.byref(p), 1, mk, ctypes.c_void_p(0x10008), n, n, n, b, n, n, n, None) == -3
    assert f(ctypes.byref(p), 2, mk, a, n, n, n, b, n, n, n, None) == -1
    for bad in ((1, 8), (5, 9)):  # below nocc, above m
        mb = (ctypes.c_int32 * 2)(*bad)
        assert f(ctypes.byref(p), 1, mb, a, n, n, n, b, n, n, n, None) == -1
        assert g(ctypes.byref(p), 1, mb, a, n, b, n, None) == -1
    big = good_problem()
    big.mesh[0], big.mesh[1], big.mesh[2], big.nk, big.nocc = 4, 4, 9, 144, 1
    mkb = (ctypes.c_int32 * 144)(*([26] * 144))
    assert f(ctypes.byref(big), 1, mkb, a, n, n, n, b, n, n, n, None) == -7


def test_dense_system_validation(L):
    from tests.conftest import gpu_available
    p = good_problem()  # 3x3x3, m = 26: the dense problem (702 orbitals) is out of range
    a = ctypes.c_void_p(0x10000)
    f = L.afqmc_kpt_dense_system
    assert f(ctypes.byref(p), 1, a, a, a, a, None) == -7
    q = good_problem()
    q.mesh[0], q.mesh[1], q.mesh[2], q.nk, q.m, q.nocc = 2, 2, 2, 8, 8, 2
    if not gpu_available():
        assert f(ctypes.byref(q), 1, a, a, a, a, None) == -5
    q.nocc = 3  # 24 occupied orbitals in the dense problem
    assert f(ctypes.byref(q), 1, a, a, a, a, None) == -7
    q.nocc = 2
    assert f(ctypes.byref(q), 1, None, a, a, a, None) == -2
    arr = (B.Problem * 2)(q, q)
    assert f(arr, 2, a, a, a, a, None) == -1
