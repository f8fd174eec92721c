"""The block driver around the step on the GPU: the energy shift E_T in the weight update,
its update from the mixed estimate between blocks, and several blocks of steps, local
energy, mixed estimate, E_T update and comb population control against the same loop of
the FP64 oracle."""

import math

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from oracle import kpoint as kp
    from oracle import walkers as wk
    from tests.gpu_cases import build, host, rel


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", ["c0", "wide"])
def test_step_with_energy_shift(case):
    s, U, x, p, pre = build(case)
    ET = -41.5
    p.set_etrial(ET)
    p.step(torch.from_numpy(x[0]))
    w = host(p.weight).copy()
    _, ld = kp.greens(U, s.A)
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt, etrial=ET)
    assert rel(w, out["weight"]) < 1e-10
    # against the same step without the shift: the common factor exp(dt E_T)
    _, _, _, q, _ = build(case)
    q.step(torch.from_numpy(x[0]))
    np.testing.assert_allclose(w, host(q.weight) * math.exp(s.dt * ET), rtol=1e-13)
    assert torch.equal(p.U, q.U) and torch.equal(p.Gh, q.Gh)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_update_etrial_from_mixed_estimate():
    s, U, x, p, pre = build("c0")
    p.set_etrial(2.0)
    E = p.energy()
    em = p.mixed_energy(E).reshape(1).clone()
    p.update_etrial(em, blend=0.25)
    torch.cuda.synchronize()
    want = 0.75 * 2.0 + 0.25 * em.real.item()
    assert abs(p.etrial.item() - want) <= 1e-15 * max(1.0, abs(want))
    # a non-finite estimate leaves E_T as it is
    p.update_etrial(torch.full((1,), complex("nan"), dtype=torch.complex128, device="cuda"))
    torch.cuda.synchronize()
    assert p.etrial.item() == want


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_blocks_with_shift_and_comb_match_oracle():
    """Three blocks of two steps each (QR after the second), then the local energy, the
    mixed estimate, E_T <- Re E_mix and the comb, on the GPU and in the oracle."""
    s, U, _, p, pre = build("c0")
    rng = np.random.default_rng(21)
    nb, ns, W = 3, 2, U.shape[0]
    xs = rng.standard_normal((nb, ns, W, s.nk, s.nchol, 2))
    xis = [0.37, 0.81, 0.05]
    # oracle loop
    Uo = U.copy()
    Gh, ld = kp.greens(Uo, s.A)
    wo = np.ones(W)
    ETo = 0.0
    ref = []
    for b in range(nb):
        for t in range(ns):
            out = kp.step(Uo, ld, wo, xs[b, t], pre, s.A, s.L, s.mesh, s.dt, etrial=ETo)
            Uo, ld, wo = out["U"], out["logdet"], out["weight"]
        Uo = kp.orthonormalize(Uo)
        Gh, ld = kp.greens(Uo, s.A)
        E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
        em = kp.mixed_energy(E, wo)
        ETo = em.real
        st = np.zeros(W, dtype=np.int32)
        Uo, Gh, ld, st, wo, par = wk.population_control(Uo, Gh, ld, st, wo, xis[b])
        ref.append((E, em, ETo, wo.copy(), par))
    # GPU loop
    for b in range(nb):
        for t in range(ns):
            p.step(torch.from_numpy(xs[b, t]), ortho=(t == ns - 1))
        E = p.energy()
        em = p.mixed_energy(E).reshape(1)
        p.update_etrial(em, blend=1.0)
        par = p.population_control(xis[b])
        torch.cuda.synchronize()
        Er, emr, ETr, wr, parr = ref[b]
        assert rel(host(E), Er) < 1e-10, b
        assert abs(em.item() - emr) <= 1e-10 * max(1.0, abs(emr)), b
        assert abs(p.etrial.item() - ETr) <= 1e-10 * max(1.0, abs(ETr)), b
        assert np.array_equal(host(par), parr), b
        assert rel(host(p.weight), wr) < 1e-10, b
    # with the shift the weights stay moderate (E_L falls from about -130 to -200 Ha per
    # supercell here: without it every step would scale them by exp(0.65) to exp(1))
    w = host(p.weight)
    assert np.all(np.isfinite(w)) and 1e-3 < w.max() < 1e3
