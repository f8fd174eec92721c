"""Full-size parity on the 3x3x3, m=26, 64-walker workload, in the launch configuration the
benchmark times (FP64 path): all 64 walkers on the GPU; the oracle recomputes sampled walkers.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

SAMPLE = [0, 37, 63]


@pytest.fixture(scope="module")
def c1():
    import torch
    from synth.kpt_inputs import config_shapes, make_system, make_walkers, make_fields
    from oracle import kpoint as kp
    from paper_2003_09468_amd import KptProblem
    cfg = config_shapes("c1")
    s, rng = make_system(cfg["mesh"], cfg["m"], cfg["nocc"], cfg["nchol"], seed=cfg["seed"])
    U = make_walkers(s, cfg["nwalk"], rng)
    x = make_fields(s, cfg["nwalk"], 2, rng)
    p = KptProblem(s.mesh, s.m, s.nocc, s.nchol, cfg["nwalk"], s.dt, torch.from_numpy(s.L),
                   torch.from_numpy(s.A))
    p.prepare(torch.from_numpy(s.H1))
    p.set_walkers(torch.from_numpy(U))
    p.greens()
    xbar_g, X_g = p.vbias()
    xbar_g, X_g = xbar_g.cpu().numpy(), X_g.cpu().numpy()
    p.step(torch.from_numpy(x[0]))
    E = p.energy().cpu().numpy()
    res = dict(U=p.U.cpu().numpy(), Gh=p.Gh.cpu().numpy(), logdet=p.logdet.cpu().numpy(),
               weight=p.weight.cpu().numpy(), E=E, xbar=xbar_g, X=X_g)
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    del p
    return s, U, x, pre, res


def test_c1_step_sampled_walkers(c1):
    from oracle import kpoint as kp
    s, U, x, pre, res = c1
    Us = U[SAMPLE]
    Gh, ld = kp.greens(Us, s.A)
    xbar, X = kp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    assert np.abs(res["X"][SAMPLE] - X).max() / np.abs(X).max() < 1e-11
    assert np.abs(res["xbar"][SAMPLE] - xbar).max() / np.abs(xbar).max() < 1e-11
    out = kp.step(Us, ld, np.ones(len(SAMPLE)), x[0][SAMPLE], pre, s.A, s.L, s.mesh, s.dt)
    assert np.abs(res["U"][SAMPLE] - out["U"]).max() < 1e-11
    assert np.abs(res["Gh"][SAMPLE] - out["Gh"]).max() / np.abs(out["Gh"]).max() < 1e-10
    assert np.abs(np.exp(res["logdet"][SAMPLE] - out["logdet"]) - 1).max() < 1e-10
    np.testing.assert_allclose(res["weight"][SAMPLE], out["weight"], rtol=1e-10)
    E = kp.local_energy(pre["Lh"], pre["h1h"], out["Gh"], s.mesh)
    assert np.abs(res["E"][SAMPLE] - E).max() / s.nk < 1e-10


def test_c1_properties_all_walkers(c1):
    """Properties that hold for every walker at any size."""
    s, U, x, pre, res = c1
    from oracle.supercell import block_diag
    Af = block_diag(s.A)
    GA = np.einsum("wir,rj->wij", res["Gh"], Af.conj())
    assert np.abs(GA - np.eye(Af.shape[1])[None]).max() < 1e-10  # Gh A* = 1
    assert np.all(np.isfinite(res["E"]))
    assert np.all(np.isfinite(res["U"])) and np.all(res["weight"] >= 0.0)
