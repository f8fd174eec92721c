"""The local energy through the entry point that allocates nothing (afqmc_kpt_energy_noalloc)
against afqmc_kpt_energy on the same problems: the same kernels, so the same energies bit
for bit, over two calls in a row whose second problem is smaller than the first (the fixed
scratch keeps the first call's contents), and against the FP64 oracle."""

import ctypes

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from paper_2003_09468_amd import binding as B
    from oracle import kpoint as kp
    from tests.gpu_cases import build, host, energy_err, overlap_cond


NOALLOC_MAX = 64 << 20  # AFQMC_ENERGY_NOALLOC_MAX_BYTES


def _noalloc(p, E):
    """Direct C-ABI call (no workspace argument)."""
    st = B.lib().afqmc_kpt_energy_noalloc(ctypes.byref(p.struct), 1, E.data_ptr(),
                                          torch.cuda.current_stream().cuda_stream)
    assert st == 0, B.lib().afqmc_kpt_strerror(st)
    return E


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_energy_noalloc_matches_energy(prec):
    pr = {"fp64": lib.PREC_FP64, "bf16x3": lib.PREC_BF16X3}[prec]
    # the larger problem first, then a smaller one on the same scratch
    for case in ("wide", "c0"):
        s, U, x, p, pre = build(case, prec=pr)
        need = p.workspace_bytes("energy")
        assert need <= NOALLOC_MAX
        E_ws = host(p.energy()).copy()
        E_na = torch.full((p.nwalk, 3), complex("nan"), dtype=torch.complex128, device="cuda")
        E_na = host(_noalloc(p, E_na)).copy()
        torch.cuda.synchronize()
        assert np.array_equal(E_na, E_ws), case
        if prec == "fp64":
            Gh, _ = kp.greens(U, s.A)
            Eref = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
            assert energy_err(E_na, Eref, s.nk, overlap_cond(U, s.A)) <= 1.0
        del p
        torch.cuda.empty_cache()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_energy_noalloc_after_a_step():
    """After a propagation step (dense Gh) and on a Gh passed in place of the problem's."""
    s, U, x, p, pre = build("m40")
    p.step(torch.from_numpy(x[0]))
    E_ws = host(p.energy()).copy()
    E_na = host(p.energy_noalloc()).copy()
    assert np.array_equal(E_na, E_ws)
    G = p.Gh.clone() * 0.5
    assert np.array_equal(host(p.energy_noalloc(Gh=G)), host(p.energy(Gh=G)))
