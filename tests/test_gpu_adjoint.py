"""The energy adjoint on the GPU: central differences of the GPU local energy on the
2x2x2 system, and the full 3x3x3, m=26, 16-walker workload (FP64 and FP32 contractions)
against the oracle's analytic generalized Fock matrix, at the trial determinant and at
perturbed walkers.

E_L is a quadratic polynomial in Gh, so the central difference with h = 1e-6 is exact up
to rounding (|E| eps / h ~ 1e-9).  FP32 bar: the FP32 contractions carry a relative
error of order sqrt(K) * 2^-24 with K = m or nocc * nchol terms; 2e-5 relative to the
largest gradient entry leaves a margin of ten over what the 2x2x2 cases show.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import kpoint as kp
    from tests.gpu_cases import build, host, rel

SAMPLE = [0, 9, 15]


def test_adjoint_central_difference_c0():
    s, U, x, p, pre = build("c0")
    G0 = p.Gh.clone()
    D = host(p.energy_backward())
    W, n, N = G0.shape
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(6):
        w, i, j = int(rng.integers(W)), int(rng.integers(n)), int(rng.integers(N))
        for d in (1.0, 1j):
            Gp, Gm = G0.clone(), G0.clone()
            Gp[w, i, j] += h * d
            Gm[w, i, j] -= h * d
            Ep = host(p.energy(Gh=Gp)).sum(1)[w]
            Em = host(p.energy(Gh=Gm)).sum(1)[w]
            fd = (Ep - Em) / (2 * h)
            assert abs(fd - D[w, i, j] * d) < 1e-6 * max(1.0, abs(D[w, i, j]))
    # a dense random direction: dE = sum D V
    V = torch.from_numpy(rng.standard_normal(G0.shape) + 1j * rng.standard_normal(G0.shape))
    V = V.to(G0.device)
    Ep = host(p.energy(Gh=G0 + h * V)).sum(1)
    Em = host(p.energy(Gh=G0 - h * V)).sum(1)
    lin = (D * host(V)).sum(axis=(1, 2))
    assert np.abs((Ep - Em) / (2 * h) - lin).max() < 1e-6 * max(1.0, np.abs(lin).max())


@pytest.fixture(scope="module")
def c4():
    from synth.kpt_inputs import config_shapes, make_system, make_walkers
    from paper_2003_09468_amd import KptProblem, PREC_FP32
    cfg = config_shapes("c4")
    s, rng = make_system(cfg["mesh"], cfg["m"], cfg["nocc"], cfg["nchol"], seed=cfg["seed"])
    U = make_walkers(s, cfg["nwalk"], rng)
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    out = {}
    for name, prec in (("fp64", 0), ("fp32", PREC_FP32)):
        p = KptProblem(s.mesh, s.m, s.nocc, s.nchol, cfg["nwalk"], s.dt,
                       torch.from_numpy(s.L), torch.from_numpy(s.A), prec=prec)
        p.prepare(torch.from_numpy(s.H1))
        p.set_walkers(torch.from_numpy(U))
        p.greens()
        out[name] = (host(p.Gh).copy(), host(p.energy_backward()).copy())
        # trial determinant: every walker = A (block diagonal)
        Ut = np.zeros_like(U)
        for k in range(s.nk):
            Ut[:, k * s.m:(k + 1) * s.m, k * s.nocc:(k + 1) * s.nocc] = s.A[k]
        p.set_walkers(torch.from_numpy(Ut))
        p.greens()
        out[name + "_trial"] = (host(p.Gh).copy(), host(p.energy_backward()).copy())
        del p
        torch.cuda.empty_cache()
    return s, pre, out


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_c4_adjoint_sampled_walkers(c4, prec, bar):
    s, pre, out = c4
    Gh, D = out[prec]
    ref = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh[SAMPLE], s.mesh)
    assert rel(D[SAMPLE], ref) < bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_c4_adjoint_at_trial_is_fock(c4, prec, bar):
    s, pre, out = c4
    Gh, D = out[prec + "_trial"]
    ref = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh[:1], s.mesh)
    assert rel(D[0], ref[0]) < bar
    # every walker sits on the trial: identical rows
    assert rel(D, np.broadcast_to(D[:1], D.shape)) < bar
