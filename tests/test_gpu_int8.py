"""The local energy with its exchange on the int8 split (energy precisions INT8X5 and
INT8X4) against the FP64 oracle, with a bar derived from the split's truncation bound; the
rest of the energy and the adjoint are the FP64 kernels, bit for bit.

Bound.  Every real row x of [Re Lh | Im Lh] (per Q, k, a, g) and of [Re G | Im G] (per
walker, row and column block of Gh) is scaled by s = 2^e with 2^(e-2) <= max|x| < 2^(e-1)
and kept to S 7-bit digits (S = 5 or 4).  The two truncated operands cost at most
2 * (128^-S / 2) * (1/2) s s' per real product and the dropped digit levels S+2 .. 2S at
most (S-1) 4096 128^-(S+2) (128/127) s s', together (1/2 + (S-1)/4 * 128/127) 2^-7S s s'
(about 1.5 * 2^-35 for S = 5, 1.25 * 2^-28 for S = 4); over kk < 2m each complex T1 entry
is off by at most delta = sqrt(2) * 2m * (that factor) * s s'.  The exchange sums
T1_t[b,a,g] T2_t[a,b,g] over the triples t, so
  |dEX| <= sum_t sum_{g,a,b} delta_t |T2_t| + |T1_t| delta'_t + delta_t delta'_t,
with |T1|, |T2| bounded by the sums of |Lh| |G| over r.  The test takes twice that.
"""

import math

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from oracle import kpoint as kp
    from tests.gpu_cases import build, host

CASESEL = (["c0", "mol", "aniso", "line3", "mixed", "wide", "m40", "m52", "m64", "occ10"]
           if gpu_available() else [])


def _scale(x, axis):
    """2^e per row: 2^(e-2) <= max(|Re|, |Im|) < 2^(e-1) over the axis (1 for a zero row)."""
    amax = np.maximum(np.abs(x.real), np.abs(x.imag)).max(axis=axis)
    _, E = np.frexp(amax)  # amax = f 2^E, 0.5 <= f < 1: ilogb = E - 1
    return np.where(amax > 0, np.ldexp(1.0, E + 1), 1.0)


def exchange_bound(Lh, Gh, mesh, S=5):
    nk, _, nocc, m, nchol = Lh.shape
    kmq, negq = kp.kpoint_tables(mesh)
    nw = Gh.shape[0]
    G = kp.blocked(Gh, nk, nocc, m).transpose(1, 3, 0, 2, 4)  # [k1, k2, w, a, r]
    sL = _scale(Lh, 3)                                         # [Q, k, a, g]
    sG = _scale(G, 4)                                          # [k1, k2, w, b]
    eps = math.sqrt(2.0) * 2 * m * (0.5 + (S - 1) / 4.0 * 128.0 / 127.0) * 2.0 ** (-7 * S)
    aL, aG = np.abs(Lh), np.abs(G)
    out = np.zeros(nw)
    for Q in range(nk):
        mQ = negq[Q]
        for k in range(nk):
            kq = kmq[Q, k]
            for kpt in range(nk):
                kpq = kmq[Q, kpt]
                P1 = np.einsum("arg,wbr->wbag", aL[Q, k], aG[kpq, kq])
                P2 = np.einsum("bsg,was->wabg", aL[mQ, kpq], aG[k, kpt])
                d1 = eps * np.einsum("ag,wb->wbag", sL[Q, k], sG[kpq, kq])
                d2 = eps * np.einsum("bg,wa->wabg", sL[mQ, kpq], sG[k, kpt])
                d2t = d2.transpose(0, 2, 1, 3)  # [w, b, a, g]
                P2t = P2.transpose(0, 2, 1, 3)
                out += (d1 * P2t + P1 * d2t + d1 * d2t).sum(axis=(1, 2, 3))
    return out


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("digits", [5, 4])
@pytest.mark.parametrize("case", CASESEL)
def test_int8_energy_against_oracle(case, digits):
    ep = lib.PREC_INT8X5 if digits == 5 else lib.PREC_INT8X4
    pl = lib.prec_place(lib.PREC_FP64, ep)
    s, U, x, p, pre = build(case, prec=pl)
    _, _, _, pd, _ = build(case, prec=lib.PREC_FP64)
    assert p.Lh8 is not None and p.Lh32 is None and p.Lhs is None
    for it in range(2):  # the initial walkers, then after one (FP64) step
        if it == 1:
            xt = torch.from_numpy(x[0])
            p.step(xt)
            pd.step(xt)
            torch.cuda.synchronize()
            assert torch.equal(p.U, pd.U) and torch.equal(p.Gh, pd.Gh)
        Gh = host(p.Gh).copy()
        E, Ed = host(p.energy()).copy(), host(pd.energy()).copy()
        # one-body and Coulomb parts: the FP64 kernels
        assert np.array_equal(E[:, :2], Ed[:, :2])
        Eref = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
        bound = exchange_bound(pre["Lh"], Gh, s.mesh, S=digits)
        dEX = np.abs(E[:, 2] - Eref[:, 2])
        # twice the derived bound, plus the FP64 evaluation's own rounding
        bar = 2.0 * bound + 1e-12 * np.abs(Eref).sum(axis=1)
        assert np.all(dEX <= bar), (case, it, dEX, bar)
        # the split is far closer than the bar suggests on these inputs, and (five digits)
        # far closer than an FP32 contraction (relative 6e-8 per product)
        rel_bar = 1e-9 if digits == 5 else 1e-7
        assert np.all(dEX <= rel_bar * np.abs(Eref).sum(axis=1) + 1e-12), (case, it, dEX)
        # the adjoint stays FP64
        assert np.array_equal(host(p.energy_backward()), host(pd.energy_backward()))


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_int8x5_placed_with_bf16x3_step_block():
    """BF16X3 steps with the INT8X5 energy in afqmc_kpt_step: the steps are the BF16X3
    problem's bit for bit, the energy is within the bound of the FP64 oracle's on the
    propagated state."""
    pl = lib.prec_place(lib.PREC_BF16X3, lib.PREC_INT8X5)
    s, U, x, p, pre = build("wide", prec=pl)
    _, _, _, pb, _ = build("wide", prec=lib.PREC_BF16X3)
    b = lib.KptBatch([p])
    f = b.fields([torch.from_numpy(x)])
    b.step(f, ortho=True, energy=True)
    E = host(b.energy(0)).copy()
    bb = lib.KptBatch([pb])
    bb.step(bb.fields([torch.from_numpy(x)]), ortho=True, energy=False)
    torch.cuda.synchronize()
    assert torch.equal(p.U, pb.U) and torch.equal(p.Gh, pb.Gh)
    Gh = host(p.Gh).copy()
    Eref = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    bar = 2.0 * exchange_bound(pre["Lh"], Gh, s.mesh) + 1e-12 * np.abs(Eref).sum(axis=1)
    assert np.all(np.abs(E[:, 2] - Eref[:, 2]) <= bar)
    assert np.all(np.abs(E[:, :2] - Eref[:, :2]).max(axis=1) <= 1e-10 * np.abs(Eref).sum(axis=1))


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("digits", [5, 4])
@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_int8_nonfinite_green_function_gives_nonfinite_energy(digits, bad):
    """A non-finite Gh entry of one walker gives that walker a non-finite exchange and leaves
    the others finite (both digit counts: INT8X4 forms its digits in a second pass)."""
    ep = lib.PREC_INT8X5 if digits == 5 else lib.PREC_INT8X4
    s, U, x, p, pre = build("c0", prec=lib.prec_place(lib.PREC_FP64, ep))
    G = p.Gh.clone()
    G[1, 0, 3] = complex(bad)
    E = host(p.energy(Gh=G))
    assert not np.isfinite(E[1, 2]) and np.all(np.isfinite(E[[0, 2, 3], 2]))
