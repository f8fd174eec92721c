"""Full-size parity of the batched path and of the reduced-precision modes.

* Systems A (2x2x2, m=26, 128 walkers) and B (3x3x3, m=26, 64 walkers) of the uneven
  batch run as one batch for two steps (QR after the last) and the energy; sampled walkers
  of each are recomputed by the oracle (FP64 bars as in the other parity tests).  System C
  (3x3x3, m=52, nchol=416, 32 walkers: the 16-step exchange kernel) runs batched with A
  and is checked the same way.
* The 3x3x3, m=26 system with FP32 and BF16X3 contractions: energies of sampled initial
  walkers against the oracle, with the bars of test_gpu_precision (relative to the summed
  magnitude of the energy parts), and one BF16X3 propagation step.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import kpoint as kp
    from tests.gpu_cases import host, rel, phase_err


def system(name, prec=0):
    from synth.kpt_inputs import config_shapes, make_system, make_walkers, make_fields
    from paper_2003_09468_amd import KptProblem
    c = config_shapes(name)
    s, rng = make_system(c["mesh"], c["m"], c["nocc"], c["nchol"], seed=c["seed"])
    U = make_walkers(s, c["nwalk"], rng)
    x = make_fields(s, c["nwalk"], 2, rng)
    p = KptProblem(s.mesh, s.m, s.nocc, s.nchol, c["nwalk"], s.dt, torch.from_numpy(s.L),
                   torch.from_numpy(s.A), prec=prec)
    p.prepare(torch.from_numpy(s.H1))
    p.set_walkers(torch.from_numpy(U))
    p.greens()
    return s, U, x, p


@pytest.fixture(scope="module")
def batch_ab():
    from paper_2003_09468_amd import KptBatch
    sysd = [system("c3A"), system("c3B")]
    b = KptBatch([d[3] for d in sysd])
    b.step(b.fields([torch.from_numpy(d[2]) for d in sysd]), ortho=True, energy=True)
    torch.cuda.synchronize()
    out = []
    for i, (s, U, x, p) in enumerate(sysd):
        out.append((s, U, x, dict(U=host(p.U), logdet=host(p.logdet), weight=host(p.weight),
                                  E=host(b.energy(i)).copy())))
    del b, sysd
    torch.cuda.empty_cache()
    return out


@pytest.fixture(scope="module")
def batch_ac():
    """Systems A and C as one batch (different band counts: every stage groups them into
    separate kernel variants of one call)."""
    from paper_2003_09468_amd import KptBatch
    sysd = [system("c3A"), system("c3C")]
    print("batch A+C: systems prepared", flush=True)
    b = KptBatch([d[3] for d in sysd])
    b.step(b.fields([torch.from_numpy(d[2]) for d in sysd]), ortho=True, energy=True)
    torch.cuda.synchronize()
    s, U, x, p = sysd[1]
    out = (s, U, x, dict(U=host(p.U), logdet=host(p.logdet), weight=host(p.weight),
                         E=host(b.energy(1)).copy()))
    del b, sysd, p
    torch.cuda.empty_cache()
    return out


def check_sampled(sysres, sample):
    s, U, x, res = sysres
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    print(f"oracle prepared (mesh {s.mesh}, m={s.m}); walkers {sample}", flush=True)
    Us = U[sample]
    _, ld = kp.greens(Us, s.A)
    w = np.ones(len(sample))
    for it in range(2):
        o = kp.step(Us, ld, w, x[it][sample], pre, s.A, s.L, s.mesh, s.dt)
        Us, ld, w = o["U"], o["logdet"], o["weight"]
    Us = kp.orthonormalize(Us)
    Gr, ldr = kp.greens(Us, s.A)
    assert rel(res["U"][sample], Us) < 1e-10
    assert phase_err(res["logdet"][sample], ldr) < 1e-9
    np.testing.assert_allclose(res["weight"][sample], w, rtol=1e-9, atol=1e-14)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gr, s.mesh)
    scale = np.abs(E).sum(1)
    assert (np.abs(res["E"][sample] - E).sum(1) / scale).max() < 1e-11


@pytest.mark.parametrize("which,sample", [(0, [0, 127]), (1, [5, 60])], ids=["A", "B"])
def test_batch_sampled_walkers(batch_ab, which, sample):
    check_sampled(batch_ab[which], sample)


def test_batch_c3C_sampled_walkers(batch_ac):
    check_sampled(batch_ac, [0, 31])


@pytest.mark.parametrize("prec,bar", [(1, 5e-6), (2, 5e-5)], ids=["fp32", "bf16x3"])
def test_reduced_precision_energy_c1(prec, bar):
    s, U, x, p = system("c3B", prec=prec)
    E = host(p.energy())
    del p
    torch.cuda.empty_cache()
    sample = [3, 41]
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, _ = kp.greens(U[sample], s.A)
    Er = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    scale = np.abs(Er).sum(1)
    assert (np.abs(E[sample].sum(1) - Er.sum(1)) / scale).max() < bar


def test_bf16x3_step_full_size():
    """One BF16X3 step of the 3x3x3, m=26, 64-walker system (702 x 702 potential, 108 walker
    columns: the launch uses the 96-row Taylor tiles) against the oracle on sampled walkers,
    with the one-step bar of test_gpu_precision."""
    s, U, x, p = system("c3B", prec=2)
    p.step(torch.from_numpy(x[0]))
    torch.cuda.synchronize()
    Ug = host(p.U)
    del p
    torch.cuda.empty_cache()
    sample = [0, 33, 63]
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    _, ld = kp.greens(U[sample], s.A)
    out = kp.step(U[sample], ld, np.ones(len(sample)), x[0][sample], pre, s.A, s.L, s.mesh, s.dt)
    assert rel(Ug[sample], out["U"]) < 5e-5
