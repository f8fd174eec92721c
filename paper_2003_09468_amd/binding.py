"""ctypes binding of libafqmc_kpt.so (argument marshalling only).

Each method of KptProblem fills the C problem descriptor from the torch tensors
it owns, calls the entry point of the same name on the current torch stream,
and raises AfqmcError on a negative status.  All arithmetic runs in the gfx950
kernels of the library.
"""

from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libafqmc_kpt.so"

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2
PREC_INT8X5 = 3  # energy precision only (prec_place(step, PREC_INT8X5))
PREC_INT8X4 = 4  # energy precision only


def prec_place(step: int, energy: int) -> int:
    """AFQMC_PREC_PLACE: the step contractions in one precision, the local energy and its
    adjoint in another."""
    return int(step) | ((int(energy) + 1) << 4)


def ls_slots(mesh) -> int:
    """Slots of the half store of L: (nk + number of Q with -Q = Q) / 2."""
    nk, self_inv = 1, 1
    for d in mesh:
        nk *= int(d)
        self_inv *= 2 if int(d) % 2 == 0 else 1
    return (nk + self_inv) // 2


def step_prec(prec: int) -> int:
    return int(prec) & 15


def energy_prec(prec: int) -> int:
    prec = int(prec)
    return (prec >> 4) - 1 if prec >> 4 else prec & 15

WALKER_SINGULAR = 1
WALKER_NONFINITE = 2
WALKER_KILLED = 4

# spins of a problem's walkers (afqmc_spin): one determinant for both spins, or the up and
# down halves of a two-determinant (collinear) walker set, held as consecutive problems
SPIN_CLOSED = 0
SPIN_UP = 1
SPIN_DOWN = 2

PROPAGATE_ORTHO = 1
PROPAGATE_REDUCED_GH = 4
STEP_ENERGY = 2

ENTRIES = {
    "prepare": 0,
    "greens": 1,
    "vbias": 2,
    "vhs": 3,
    "propagate": 4,
    "ortho": 5,
    "energy": 6,
    "energy_backward": 7,
    "step": 8,
    "population": 9,
}

BUFFERS = {"fields": 0, "xbar": 1, "X": 2, "vhs": 3, "energy": 4, "gE": 5, "gGh": 6}

EXPORTS = [
    "afqmc_kpt_workspace_bytes",
    "afqmc_kpt_prepare",
    "afqmc_kpt_greens",
    "afqmc_kpt_vbias",
    "afqmc_kpt_vhs",
    "afqmc_kpt_propagate",
    "afqmc_kpt_orthonormalize",
    "afqmc_kpt_energy",
    "afqmc_kpt_energy_noalloc",
    "afqmc_kpt_energy_backward",
    "afqmc_kpt_mixed_energy",
    "afqmc_kpt_population_control",
    "afqmc_kpt_update_etrial",
    "afqmc_kpt_reblock",
    "afqmc_kpt_dense_system",
    "afqmc_kpt_dense_fields",
    "afqmc_kpt_pad_bands",
    "afqmc_kpt_unpad_bands",
    "afqmc_kpt_buffer_layout",
    "afqmc_kpt_step",
    "afqmc_kpt_autotune",
    "afqmc_kpt_graph_create",
    "afqmc_kpt_graph_launch",
    "afqmc_kpt_graph_destroy",
    "afqmc_kpt_timing_enable",
    "afqmc_kpt_timing_read",
    "afqmc_kpt_strerror",
    "afqmc_kpt_version",
]

KERNEL_CLASSES = ["taylor", "vhs", "vbias", "greens", "bhalf", "weights", "ortho", "exchange",
                  "energy_rest", "exchange_bwd"]


class AfqmcError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    """Mirror of afqmc_kpt_problem (include/afqmc_kpt.h)."""

    _fields_ = [
        ("mesh", ctypes.c_int32 * 3),
        ("nk", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("nocc", ctypes.c_int32),
        ("nchol", ctypes.c_int32),
        ("nwalk", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("L", ctypes.c_void_p),
        ("A", ctypes.c_void_p),
        ("Lh", ctypes.c_void_p),
        ("h1h", ctypes.c_void_p),
        ("bhalf", ctypes.c_void_p),
        ("L32", ctypes.c_void_p),
        ("Lh32", ctypes.c_void_p),
        ("Lhs", ctypes.c_void_p),
        ("Ls", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("Gh", ctypes.c_void_p),
        ("logdet", ctypes.c_void_p),
        ("weight", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("etrial", ctypes.c_void_p),
        ("Lh8", ctypes.c_void_p),
        ("spin", ctypes.c_int32),
    ]


_lib = None


def library_path() -> str:
    return os.path.join(HERE, _LIBNAME)


def lib():
    """Load the library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2003_09468_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(Problem)
    vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    sig = {
        "afqmc_kpt_workspace_bytes": [P, i, i, ctypes.POINTER(sz)],
        "afqmc_kpt_prepare": [P, i, vp, vp, sz, vp],
        "afqmc_kpt_greens": [P, i, vp, sz, vp],
        "afqmc_kpt_vbias": [P, i, vp, vp, vp, sz, vp],
        "afqmc_kpt_vhs": [P, i, vp, vp, vp, vp, sz, vp],
        "afqmc_kpt_propagate": [P, i, vp, vp, vp, i, vp, sz, vp],
        "afqmc_kpt_orthonormalize": [P, i, vp, sz, vp],
        "afqmc_kpt_energy": [P, i, vp, vp, sz, vp],
        "afqmc_kpt_energy_noalloc": [P, i, vp, vp],
        "afqmc_kpt_energy_backward": [P, i, vp, vp, vp, sz, vp],
        "afqmc_kpt_mixed_energy": [P, i, vp, vp, vp],
        "afqmc_kpt_population_control": [P, i, vp, vp, vp, sz, vp],
        "afqmc_kpt_update_etrial": [P, i, vp, ctypes.c_double, vp],
        "afqmc_kpt_dense_system": [P, i, vp, vp, vp, vp, vp],
        "afqmc_kpt_dense_fields": [P, i, vp, vp, vp],
        "afqmc_kpt_pad_bands": [P, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "afqmc_kpt_unpad_bands": [P, i, vp, vp, vp, vp, vp, vp],
        "afqmc_kpt_reblock": [vp, ctypes.c_int64, vp, i, ctypes.POINTER(i),
                              ctypes.POINTER(i)],
        "afqmc_kpt_buffer_layout": [P, i, i, ctypes.POINTER(sz)],
        "afqmc_kpt_step": [P, i, vp, i, vp, vp, vp, i, vp, sz, vp],
        "afqmc_kpt_autotune": [P, i, vp, vp, sz, vp],
        "afqmc_kpt_graph_create": [P, i, vp, i, vp, vp, vp, i, vp, sz, ctypes.POINTER(vp)],
        "afqmc_kpt_graph_launch": [vp, vp],
        "afqmc_kpt_graph_destroy": [vp],
        "afqmc_kpt_timing_enable": [i, i],
        "afqmc_kpt_timing_read": [i, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_longlong)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.afqmc_kpt_strerror.argtypes = [ctypes.c_int]
    L.afqmc_kpt_strerror.restype = ctypes.c_char_p
    L.afqmc_kpt_version.argtypes = []
    L.afqmc_kpt_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != 0:
        msg = lib().afqmc_kpt_strerror(status).decode()
        raise AfqmcError(fn, status, msg)


def timing_enable(enable: bool, capacity: int = 65536) -> None:
    """Bracket every kernel launch with HIP events on its stream (see the header)."""
    check("afqmc_kpt_timing_enable", lib().afqmc_kpt_timing_enable(int(enable), int(capacity)))


def timing_read(kclass: str) -> tuple[float, int]:
    """(total ms, launches) of a kernel class since timing was enabled."""
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    check("afqmc_kpt_timing_read",
          lib().afqmc_kpt_timing_read(KERNEL_CLASSES.index(kclass), ctypes.byref(ms),
                                      ctypes.byref(n)))
    return float(ms.value), int(n.value)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class ReblockLevel(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_double), ("err", ctypes.c_double),
                ("err_err", ctypes.c_double)]


def reblock(x):
    """Blocking analysis of a host series (afqmc_kpt_reblock): a list of levels
    (n, mean, err, err_err) and the index of the level to quote (-1: none)."""
    vals = [float(v) for v in x]
    xs = (ctypes.c_double * max(len(vals), 1))(*vals)
    cap = 64
    lv = (ReblockLevel * cap)()
    nl, opt = ctypes.c_int(0), ctypes.c_int(0)
    check("afqmc_kpt_reblock",
          lib().afqmc_kpt_reblock(ctypes.addressof(xs), len(vals), lv, cap, ctypes.byref(nl),
                                  ctypes.byref(opt)))
    out = [(int(l.n), float(l.mean), float(l.err), float(l.err_err))
           for l in lv[:min(nl.value, cap)]]
    return out, int(opt.value)


class KptProblem:
    """One k-point system and its walker batch, with device buffers owned by torch.

    L: [nk][nk][m][m][nchol] complex128, A: [nk][m][nocc] complex128 (device tensors).
    """

    def __init__(self, mesh, m, nocc, nchol, nwalk, dt, L, A, prec=PREC_FP64, device="cuda",
                 spin=SPIN_CLOSED, share=None):
        """spin: SPIN_CLOSED, or SPIN_UP / SPIN_DOWN for a half of a two-determinant walker
        set (see KptSpinPair); share: another problem of the same system whose arrays
        derived from L and H1 alone (L, bhalf, L32, Ls) this one uses instead of its own."""
        self.spin = int(spin)
        self.mesh = tuple(int(v) for v in mesh)
        self.nk = self.mesh[0] * self.mesh[1] * self.mesh[2]
        self.m, self.nocc, self.nchol, self.nwalk = int(m), int(nocc), int(nchol), int(nwalk)
        self.dt = float(dt)
        self.prec = int(prec)
        self.device = torch.device(device)
        nk, c128 = self.nk, torch.complex128
        kw = dict(device=self.device)
        self.L = share.L if share is not None else L.to(**kw, dtype=c128).contiguous()
        self.A = A.to(**kw, dtype=c128).contiguous()
        self.Lh = torch.empty((nk, nk, nocc, m, nchol), dtype=c128, **kw)
        self.h1h = torch.empty((nk, nocc, m), dtype=c128, **kw)
        self.bhalf = (share.bhalf if share is not None
                      else torch.empty((nk, m, m), dtype=c128, **kw))
        # complex64 copies: L for the FP32 HS potential, Lh for the FP32 force bias and
        # exchange and for the adjoint of both reduced modes (BF16X3 reads split planes of L)
        sp, ep = step_prec(self.prec), energy_prec(self.prec)
        self.L32 = (torch.empty(self.L.shape, dtype=torch.complex64, **kw)
                    if sp == PREC_FP32 and share is None else
                    (share.L32 if share is not None else None))
        low = (PREC_FP32, PREC_BF16X3)
        self.Lh32 = (torch.empty(self.Lh.shape, dtype=torch.complex64, **kw)
                     if sp in low or ep in low else None)
        self.Lhs = self.Ls = self.Lh8 = None
        if ep in (PREC_INT8X5, PREC_INT8X4):
            # five int8 digits per element of [Re | Im] rows padded to 64, then int32 exponents
            kp8 = 64 * ((2 * m + 63) // 64)
            rows = nk * nk * nchol * nocc
            self.Lh8 = torch.empty(rows * (5 * kp8 + 4), dtype=torch.int8, **kw)
        if PREC_BF16X3 in (sp, ep):
            kp = 32 * ((m + 31) // 32)
            self.Lhs = torch.empty((nk, nk, nchol, nocc, 4, kp), dtype=torch.int16, **kw)
        if sp == PREC_BF16X3 and share is not None:
            self.Ls = share.Ls
        elif sp == PREC_BF16X3:
            cp = 32 * ((nchol + 31) // 32)
            # half store: one slot per time-reversal pair (Q <= -Q), then int32 Q per slot
            nq = ls_slots(self.mesh)
            self.Ls = torch.empty(nq * (cp // 32) * nk * m * m * 4 * 32 + 2 * nq,
                                  dtype=torch.int16, **kw)
        N, n = nk * m, nk * nocc
        self.U = torch.zeros((nwalk, N, n), dtype=c128, **kw)
        self.Gh = torch.zeros((nwalk, n, N), dtype=c128, **kw)
        self.logdet = torch.zeros(nwalk, dtype=c128, **kw)
        self.weight = torch.ones(nwalk, dtype=torch.float64, **kw)
        self.status = torch.zeros(nwalk, dtype=torch.int32, **kw)
        self.etrial = torch.zeros(1, dtype=torch.float64, **kw)  # E_T per supercell
        self._ws = None
        self.struct = self._make_struct()

    # -- descriptor and workspace ------------------------------------------------
    def _make_struct(self, Gh=None) -> Problem:
        p = Problem()
        p.mesh[0], p.mesh[1], p.mesh[2] = self.mesh
        p.nk, p.m, p.nocc, p.nchol, p.nwalk = self.nk, self.m, self.nocc, self.nchol, self.nwalk
        p.prec, p.dt = self.prec, self.dt
        p.L, p.A, p.Lh, p.h1h, p.bhalf = (_ptr(self.L), _ptr(self.A), _ptr(self.Lh),
                                          _ptr(self.h1h), _ptr(self.bhalf))
        p.Lh8 = _ptr(self.Lh8)
        p.L32, p.Lh32, p.Lhs, p.Ls = (_ptr(self.L32), _ptr(self.Lh32), _ptr(self.Lhs),
                                      _ptr(self.Ls))
        p.U = _ptr(self.U)
        p.Gh = _ptr(self.Gh if Gh is None else Gh)
        p.logdet, p.weight, p.status = _ptr(self.logdet), _ptr(self.weight), _ptr(self.status)
        p.etrial = _ptr(self.etrial)
        p.spin = self.spin
        return p

    def workspace_bytes(self, entry: str) -> int:
        out = ctypes.c_size_t(0)
        check("afqmc_kpt_workspace_bytes",
              lib().afqmc_kpt_workspace_bytes(ctypes.byref(self.struct), 1, ENTRIES[entry],
                                              ctypes.byref(out)))
        return int(out.value)

    def workspace(self):
        if self._ws is None:
            need = max(self.workspace_bytes(e) for e in ENTRIES)
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def _ws_args(self):
        ws = self.workspace()
        return ws.data_ptr(), ws.numel()

    # -- entry points ----------------------------------------------------------------
    def set_walkers(self, U, weight=None):
        self.U.copy_(U.to(self.U.dtype))
        if weight is not None:
            self.weight.copy_(weight)
        self.status.zero_()

    def prepare(self, H1):
        H1 = H1.to(device=self.device, dtype=torch.complex128).contiguous()
        ws, nb = self._ws_args()
        check("afqmc_kpt_prepare",
              lib().afqmc_kpt_prepare(ctypes.byref(self.struct), 1, H1.data_ptr(), ws, nb,
                                      _stream()))

    def greens(self):
        ws, nb = self._ws_args()
        check("afqmc_kpt_greens",
              lib().afqmc_kpt_greens(ctypes.byref(self.struct), 1, ws, nb, _stream()))

    def vbias(self, xbar=None, X=None):
        W, nk, C = self.nwalk, self.nk, self.nchol
        if xbar is None:
            xbar = torch.empty((W, nk, C, 2), dtype=torch.complex128, device=self.device)
        if X is None:
            X = torch.empty((W, nk, C), dtype=torch.complex128, device=self.device)
        ws, nb = self._ws_args()
        check("afqmc_kpt_vbias",
              lib().afqmc_kpt_vbias(ctypes.byref(self.struct), 1, xbar.data_ptr(),
                                    X.data_ptr(), ws, nb, _stream()))
        return xbar, X

    def vhs(self, x, xbar, out=None):
        N = self.nk * self.m
        dt = torch.complex64 if step_prec(self.prec) != PREC_FP64 else torch.complex128
        if out is None:
            out = torch.empty((self.nwalk, N, N), dtype=dt, device=self.device)
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        ws, nb = self._ws_args()
        check("afqmc_kpt_vhs",
              lib().afqmc_kpt_vhs(ctypes.byref(self.struct), 1, x.data_ptr(), xbar.data_ptr(),
                                  out.data_ptr(), ws, nb, _stream()))
        return out

    def propagate(self, vhs, x, xbar, ortho=False, reduced_gh=False):
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        ws, nb = self._ws_args()
        check("afqmc_kpt_propagate",
              lib().afqmc_kpt_propagate(ctypes.byref(self.struct), 1, vhs.data_ptr(),
                                        x.data_ptr(), xbar.data_ptr(),
                                        (PROPAGATE_ORTHO if ortho else 0) |
                                        (PROPAGATE_REDUCED_GH if reduced_gh else 0),
                                        ws, nb, _stream()))

    def orthonormalize(self):
        ws, nb = self._ws_args()
        check("afqmc_kpt_orthonormalize",
              lib().afqmc_kpt_orthonormalize(ctypes.byref(self.struct), 1, ws, nb, _stream()))

    def energy(self, out=None, Gh=None):
        if out is None:
            out = torch.empty((self.nwalk, 3), dtype=torch.complex128, device=self.device)
        st = self.struct if Gh is None else self._make_struct(Gh)
        ws, nb = self._ws_args()
        check("afqmc_kpt_energy",
              lib().afqmc_kpt_energy(ctypes.byref(st), 1, out.data_ptr(), ws, nb, _stream()))
        return out

    def energy_noalloc(self, out=None, Gh=None):
        """The local energy through the entry point that allocates nothing (fixed device
        scratch instead of this problem's workspace)."""
        if out is None:
            out = torch.empty((self.nwalk, 3), dtype=torch.complex128, device=self.device)
        st = self.struct if Gh is None else self._make_struct(Gh)
        check("afqmc_kpt_energy_noalloc",
              lib().afqmc_kpt_energy_noalloc(ctypes.byref(st), 1, out.data_ptr(), _stream()))
        return out

    def energy_backward(self, gE=None, out=None, Gh=None):
        if gE is not None:
            gE = gE.resolve_conj().to(device=self.device, dtype=torch.complex128).contiguous()
        if out is None:
            out = torch.empty_like(self.Gh)
        st = self.struct if Gh is None else self._make_struct(Gh)
        ws, nb = self._ws_args()
        check("afqmc_kpt_energy_backward",
              lib().afqmc_kpt_energy_backward(ctypes.byref(st), 1, _ptr(gE), out.data_ptr(),
                                              ws, nb, _stream()))
        return out

    def mixed_energy(self, E):
        """Weighted average of the walkers' local energies (current weights)."""
        out = torch.empty(1, dtype=torch.complex128, device=self.device)
        check("afqmc_kpt_mixed_energy",
              lib().afqmc_kpt_mixed_energy(ctypes.byref(self.struct), 1, E.data_ptr(),
                                           out.data_ptr(), _stream()))
        return out[0]

    def dense(self, H1, prec=None):
        """The standard (dense) representation of this system as a 1x1x1-mesh problem (same
        walkers, same Hamiltonian): Cholesky vectors, one-body matrix and trial from
        afqmc_kpt_dense_system, prepared; the walkers of this problem are copied in."""
        N, n = self.nk * self.m, self.nk * self.nocc
        kw = dict(device=self.device, dtype=torch.complex128)
        Ld = torch.empty((1, 1, N, N, self.nk * self.nchol), **kw)
        H1d = torch.empty((1, N, N), **kw)
        Ad = torch.empty((1, N, n), **kw)
        H1 = H1.to(**kw).contiguous()
        check("afqmc_kpt_dense_system",
              lib().afqmc_kpt_dense_system(ctypes.byref(self.struct), 1, H1.data_ptr(),
                                           Ld.data_ptr(), H1d.data_ptr(), Ad.data_ptr(),
                                           _stream()))
        d = KptProblem((1, 1, 1), N, n, self.nk * self.nchol, self.nwalk, self.dt, Ld, Ad,
                       prec=self.prec if prec is None else prec, device=self.device)
        d.prepare(H1d)
        d.set_walkers(self.U, self.weight)
        return d

    def dense_fields(self, x):
        """The dense system's fields for the k-point fields x ([nwalk][nk][nchol][2])."""
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        xd = torch.empty((self.nwalk, 1, self.nk * self.nchol, 2), dtype=torch.float64,
                         device=self.device)
        check("afqmc_kpt_dense_fields",
              lib().afqmc_kpt_dense_fields(ctypes.byref(self.struct), 1, x.data_ptr(),
                                           xd.data_ptr(), _stream()))
        return xd

    def set_etrial(self, value):
        """Energy shift E_T (per supercell) of the projector exp(-dt (H - E_T))."""
        self.etrial.fill_(float(value))

    def update_etrial(self, Emix, blend=1.0):
        """E_T <- (1 - blend) E_T + blend Re(Emix) on the device (Emix: [1] complex128 from
        mixed_energy, e.g. a view of its result); a non-finite Emix leaves E_T."""
        Emix = Emix.reshape(1).to(dtype=torch.complex128)
        check("afqmc_kpt_update_etrial",
              lib().afqmc_kpt_update_etrial(ctypes.byref(self.struct), 1, Emix.data_ptr(),
                                            float(blend), _stream()))

    def population_control(self, xi):
        """Comb population control with the uniform number xi in [0, 1): resamples U, Gh,
        logdet and status in place, sets every weight to the mean weight; returns the
        parent index of each new walker (int32, device)."""
        parent = torch.empty(self.nwalk, dtype=torch.int32, device=self.device)
        xs = (ctypes.c_double * 1)(float(xi))
        pp = (ctypes.c_void_p * 1)(parent.data_ptr())
        ws, nb = self._ws_args()
        check("afqmc_kpt_population_control",
              lib().afqmc_kpt_population_control(ctypes.byref(self.struct), 1, xs, pp, ws, nb,
                                                 _stream()))
        return parent

    def step(self, x, ortho=False, bufs=None, reduced_gh=False):
        """force bias -> HS potential -> propagate (new Gh, logdet, weights); reduced_gh:
        the new Gh by the FP32 product in the FP32 and BF16X3 modes (for a Gh that only
        feeds the next force bias; with ortho the re-orthonormalisation forms it in FP64)."""
        if bufs is None:
            bufs = {}
        xbar, _ = self.vbias(bufs.get("xbar"), bufs.get("X"))
        v = self.vhs(x, xbar, bufs.get("vhs"))
        self.propagate(v, x, xbar, ortho=ortho, reduced_gh=reduced_gh)
        return xbar, v


def _band_problem(mesh, m, nocc, nchol, nwalk):
    p = Problem()
    p.mesh[0], p.mesh[1], p.mesh[2] = (int(v) for v in mesh)
    p.nk = p.mesh[0] * p.mesh[1] * p.mesh[2]
    p.m, p.nocc, p.nchol, p.nwalk = int(m), int(nocc), int(nchol), max(int(nwalk), 1)
    p.prec, p.dt = 0, 1.0
    return p


def _band_counts(mk):
    return (ctypes.c_int32 * len(mk))(*[int(v) for v in mk])


def pad_bands(mesh, mk, m, nocc, nchol, L_r=None, H1_r=None, A_r=None, U_r=None,
              device="cuda"):
    """Uniform arrays with m bands per k-point from packed ragged ones (afqmc_kpt_pad_bands):
    returns (L, H1, A, U), None for each input not given.  L_r, H1_r, A_r: the flat packed
    blocks; U_r: [nwalk][sum mk][nk*nocc]."""
    dev = torch.device(device)
    nk = int(mesh[0]) * int(mesh[1]) * int(mesh[2])
    c128 = dict(dtype=torch.complex128, device=dev)
    ins = [None if t is None else t.to(**c128).contiguous() for t in (L_r, H1_r, A_r, U_r)]
    nwalk = 1 if ins[3] is None else int(ins[3].shape[0])
    shapes = [(nk, nk, m, m, nchol), (nk, m, m), (nk, m, nocc), (nwalk, nk * m, nk * nocc)]
    outs = [None if t is None else torch.empty(sh, **c128) for t, sh in zip(ins, shapes)]
    p = _band_problem(mesh, m, nocc, nchol, nwalk)
    check("afqmc_kpt_pad_bands",
          lib().afqmc_kpt_pad_bands(ctypes.byref(p), 1, _band_counts(mk),
                                    *[_ptr(t) for t in ins], *[_ptr(t) for t in outs],
                                    _stream()))
    return tuple(outs)


def unpad_bands(problem, mk, U=None, Gh=None):
    """Ragged walkers [nwalk][sum mk][n] and half-rotated Green's functions
    [nwalk][n][sum mk] of a padded problem (afqmc_kpt_unpad_bands)."""
    M = sum(int(v) for v in mk)
    n = problem.nk * problem.nocc
    c128 = dict(dtype=torch.complex128, device=problem.device)
    Ur = None if U is None else torch.empty((problem.nwalk, M, n), **c128)
    Gr = None if Gh is None else torch.empty((problem.nwalk, n, M), **c128)
    p = _band_problem(problem.mesh, problem.m, problem.nocc, problem.nchol, problem.nwalk)
    check("afqmc_kpt_unpad_bands",
          lib().afqmc_kpt_unpad_bands(ctypes.byref(p), 1, _band_counts(mk), _ptr(U), _ptr(Gh),
                                      _ptr(Ur), _ptr(Gr), _stream()))
    return Ur, Gr


class KptBatch:
    """Several systems (KptProblem objects, possibly of different sizes and precisions)
    driven as one batch: each stage of an entry point is one launch for up to 8 systems.

    Per-call buffers are packed problem after problem at the offsets the library reports
    (afqmc_kpt_buffer_layout); xbar(i), vhs(i) and energy(i) are views of system i's slice.
    """

    def __init__(self, problems):
        self.problems = list(problems)
        if not self.problems:
            raise ValueError("empty batch")
        self.n = len(self.problems)
        self.device = self.problems[0].device
        self.arr = (Problem * self.n)(*[p.struct for p in self.problems])
        self.layout = {b: self.buffer_layout(b) for b in BUFFERS}
        self._xbar = self._alloc("xbar")
        self._vhs = self._alloc("vhs")
        self._E = self._alloc("energy")
        self._ws = None

    def buffer_layout(self, buf: str) -> list[int]:
        off = (ctypes.c_size_t * (self.n + 1))()
        check("afqmc_kpt_buffer_layout",
              lib().afqmc_kpt_buffer_layout(self.arr, self.n, BUFFERS[buf], off))
        return [int(v) for v in off]

    def _alloc(self, buf: str, count: int = 1):
        nbytes = self.layout[buf][-1] * count
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def _view(self, raw, buf: str, i: int, dtype, shape):
        off = self.layout[buf][i]
        count = 1
        for v in shape:
            count *= v
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return raw[off:off + nbytes].view(dtype).view(shape)

    def workspace_bytes(self, entry: str) -> int:
        out = ctypes.c_size_t(0)
        check("afqmc_kpt_workspace_bytes",
              lib().afqmc_kpt_workspace_bytes(self.arr, self.n, ENTRIES[entry], ctypes.byref(out)))
        return int(out.value)

    def workspace(self):
        if self._ws is None:
            need = max(self.workspace_bytes(e) for e in ENTRIES)
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def fields(self, xs):
        """Pack per-system fields ([nsteps][W][nk][C][2] float64 each) for step()/graph()."""
        nsteps = int(xs[0].shape[0])
        raw = self._alloc("fields", nsteps)
        stride = self.layout["fields"][-1]
        for i, x in enumerate(xs):
            off = self.layout["fields"][i]
            nb = x[0].numel() * 8
            xd = x.to(device=self.device, dtype=torch.float64).contiguous()
            for s_ in range(nsteps):
                raw[s_ * stride + off:s_ * stride + off + nb].view(torch.float64).copy_(
                    xd[s_].reshape(-1))
        return raw, nsteps

    def xbar(self, i):
        p = self.problems[i]
        return self._view(self._xbar, "xbar", i, torch.complex128, (p.nwalk, p.nk, p.nchol, 2))

    def vhs(self, i):
        p = self.problems[i]
        N = p.nk * p.m
        dt = torch.complex64 if step_prec(p.prec) != PREC_FP64 else torch.complex128
        return self._view(self._vhs, "vhs", i, dt, (p.nwalk, N, N))

    def energy(self, i):
        p = self.problems[i]
        return self._view(self._E, "energy", i, torch.complex128, (p.nwalk, 3))

    def mixed_energy(self):
        """Mixed estimate per system from the last step's energies (afqmc_kpt_mixed_energy)."""
        out = torch.empty(self.n, dtype=torch.complex128, device=self.device)
        check("afqmc_kpt_mixed_energy",
              lib().afqmc_kpt_mixed_energy(self.arr, self.n, self._E.data_ptr(), out.data_ptr(),
                                           _stream()))
        return out

    def population_control(self, xis):
        """Comb population control of every system (one uniform number per system); returns
        the parent indices per system."""
        parents = [torch.empty(p.nwalk, dtype=torch.int32, device=self.device)
                   for p in self.problems]
        xs = (ctypes.c_double * self.n)(*[float(x) for x in xis])
        pp = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in parents])
        ws = self.workspace()
        check("afqmc_kpt_population_control",
              lib().afqmc_kpt_population_control(self.arr, self.n, xs, pp, ws.data_ptr(),
                                                 ws.numel(), _stream()))
        return parents

    def greens(self):
        ws = self.workspace()
        check("afqmc_kpt_greens",
              lib().afqmc_kpt_greens(self.arr, self.n, ws.data_ptr(), ws.numel(), _stream()))

    def prepare(self, H1):
        """afqmc_kpt_prepare of every system with the one-body blocks H1 (equal shapes)."""
        H1 = H1.to(device=self.device, dtype=torch.complex128).contiguous()
        ws = self.workspace()
        check("afqmc_kpt_prepare",
              lib().afqmc_kpt_prepare(self.arr, self.n, H1.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream()))

    def vbias(self):
        """Force bias of every system (afqmc_kpt_vbias) into the batch's xbar and X slices."""
        if getattr(self, "_X", None) is None:
            self._X = self._alloc("X")
        ws = self.workspace()
        check("afqmc_kpt_vbias",
              lib().afqmc_kpt_vbias(self.arr, self.n, self._xbar.data_ptr(), self._X.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream()))

    def X(self, i):
        p = self.problems[i]
        return self._view(self._X, "X", i, torch.complex128, (p.nwalk, p.nk, p.nchol))

    def local_energy(self):
        """Local energy of every system (afqmc_kpt_energy) into the batch's energy slices."""
        ws = self.workspace()
        check("afqmc_kpt_energy",
              lib().afqmc_kpt_energy(self.arr, self.n, self._E.data_ptr(), ws.data_ptr(),
                                     ws.numel(), _stream()))

    def energy_backward(self, gEs):
        """dE/dGh of every system (afqmc_kpt_energy_backward) for the per-walker cotangents
        gEs[i] ([nwalk] complex128, None for ones); returns one gradient view per system."""
        gE = self._alloc("gE")
        for i, g in enumerate(gEs):
            p = self.problems[i]
            v = self._view(gE, "gE", i, torch.complex128, (p.nwalk,))
            if g is None:
                v.fill_(1.0)
            else:
                v.copy_(g.resolve_conj().to(device=self.device, dtype=torch.complex128))
        out = self._alloc("gGh")
        ws = self.workspace()
        check("afqmc_kpt_energy_backward",
              lib().afqmc_kpt_energy_backward(self.arr, self.n, gE.data_ptr(), out.data_ptr(),
                                              ws.data_ptr(), ws.numel(), _stream()))
        return [self._view(out, "gGh", i, torch.complex128, tuple(p.Gh.shape))
                for i, p in enumerate(self.problems)]

    def step(self, fields, ortho=False, energy=False):
        """Run the packed fields' nsteps steps of every system (afqmc_kpt_step)."""
        raw, nsteps = fields
        ws = self.workspace()
        flags = (PROPAGATE_ORTHO if ortho else 0) | (STEP_ENERGY if energy else 0)
        check("afqmc_kpt_step",
              lib().afqmc_kpt_step(self.arr, self.n, raw.data_ptr(), nsteps, self._xbar.data_ptr(),
                                   self._vhs.data_ptr(), self._E.data_ptr(), flags,
                                   ws.data_ptr(), ws.numel(), _stream()))

    def autotune(self):
        ws = self.workspace()
        check("afqmc_kpt_autotune",
              lib().afqmc_kpt_autotune(self.arr, self.n, self._vhs.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream()))

    def graph(self, fields, ortho=False, energy=False):
        """Capture the step block over these packed fields (refresh them between launches)."""
        return KptGraph(self, fields, ortho, energy)


class KptSpinPair(KptBatch):
    """Collinear walkers with one determinant per spin (afqmc_spin): one system, held as
    the up half (nocc_up electrons of spin up per k-point, trial A_up) followed by the down
    half (nocc_dn, A_dn), which shares L and the arrays derived from L and H1.  Every entry
    of the batch couples the halves: one field per walker, the force bias and the energy of
    both spins, one weight per walker (kept equal in both halves)."""

    def __init__(self, mesh, m, nocc_up, nocc_dn, nchol, nwalk, dt, L, A_up, A_dn,
                 prec=PREC_FP64, device="cuda"):
        up = KptProblem(mesh, m, nocc_up, nchol, nwalk, dt, L, A_up, prec=prec, device=device,
                        spin=SPIN_UP)
        dn = KptProblem(mesh, m, nocc_dn, nchol, nwalk, dt, None, A_dn, prec=prec,
                        device=device, spin=SPIN_DOWN, share=up)
        super().__init__([up, dn])
        self.up, self.dn = up, dn

    def set_walkers(self, U_up, U_dn, weight=None):
        self.up.set_walkers(U_up, weight)
        self.dn.set_walkers(U_dn, weight)

    def step_fields(self, x):
        """Packed fields of one walker set ([nsteps][W][nk][C][2]) for step()/graph(); the
        down half's slot is not read, so it is left as a copy."""
        return self.fields([x, x])


class KptGraph:
    """A captured block of steps of a KptBatch (afqmc_kpt_graph_*)."""

    def __init__(self, batch, fields, ortho, energy):
        raw, nsteps = fields
        ws = batch.workspace()
        flags = (PROPAGATE_ORTHO if ortho else 0) | (STEP_ENERGY if energy else 0)
        h = ctypes.c_void_p()
        check("afqmc_kpt_graph_create",
              lib().afqmc_kpt_graph_create(batch.arr, batch.n, raw.data_ptr(), nsteps,
                                           batch._xbar.data_ptr(), batch._vhs.data_ptr(),
                                           batch._E.data_ptr(), flags, ws.data_ptr(), ws.numel(),
                                           ctypes.byref(h)))
        self.handle = h
        self._keep = (batch, raw, ws)  # the graph holds their addresses

    def launch(self):
        check("afqmc_kpt_graph_launch", lib().afqmc_kpt_graph_launch(self.handle, _stream()))

    def close(self):
        if self.handle is not None and self.handle.value:
            check("afqmc_kpt_graph_destroy", lib().afqmc_kpt_graph_destroy(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _LocalEnergy(torch.autograd.Function):
    """E_L[w] = E1B + EC + EX as a holomorphic function of Gh.

    Backward follows torch's convention for complex inputs:
    grad_Gh = grad_E * conj(dE/dGh) = conj(conj(grad_E) * dE/dGh); the library
    returns gE * dE/dGh for a given per-walker cotangent gE.
    """

    @staticmethod
    def forward(ctx, Gh, problem):
        Gh = Gh.contiguous()
        E = problem.energy(Gh=Gh)
        ctx.problem = problem
        ctx.save_for_backward(Gh)
        return E.sum(dim=1)

    @staticmethod
    def backward(ctx, grad):
        (Gh,) = ctx.saved_tensors
        # resolve_conj: a lazy conjugate view would hand the library unconjugated memory
        gE = grad.conj().resolve_conj().to(torch.complex128).contiguous()
        g = ctx.problem.energy_backward(gE=gE, Gh=Gh)
        return g.conj(), None


def local_energy(problem: KptProblem, Gh) -> torch.Tensor:
    """Differentiable local energy per walker (recomputes the exchange intermediates in backward)."""
    return _LocalEnergy.apply(Gh, problem)
