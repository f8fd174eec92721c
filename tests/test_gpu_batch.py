"""Batches of uneven systems in one call, the captured step block and the autotuner.

A batch mixes meshes, band counts, Cholesky ranks, walker counts, one FP32 and two BF16X3
systems.
Every system's result must equal what the same system gives when run alone through the
single-problem entry points (same kernels, same reduction order: agreement to rounding
noise), and the FP64 systems must match the oracle to the FP64 bar.  The captured block
is replayed several times, with eager library work and synchronisations between the
replays, and every replay is compared with the eager result.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import kpoint as kp
    from paper_2003_09468_amd import KptBatch
    from tests.gpu_cases import build, host, rel, phase_err, energy_err, overlap_cond

# (case, precision): uneven sizes; one FP32 and two BF16X3 systems share the batch (the two
# BF16X3 systems differ in mesh and Cholesky padding but share each BF16X3 launch)
BATCH = [("aniso", 0), ("line3", 0), ("wide", 0), ("mixed", 1), ("c0", 0), ("mol", 2),
         (((2, 2, 1), 9, 3, 40, 7, "random", "dense"), 2)]
NSTEPS = 2  # the fields drawn by build() cover two steps


def make():
    return [build(case, seed=10 + i, prec=prec) for i, (case, prec) in enumerate(BATCH)]


def state(p):
    return [host(t).copy() for t in (p.U, p.Gh, p.logdet, p.weight, p.status)]


def run_single(items):
    """Each system alone: two steps (re-orthonormalise after the last) and the energy; as in
    the block entry, the reduced precisions form each step's Gh by the FP32 product."""
    out = []
    for s, U, x, p, pre in items:
        for it in range(NSTEPS):
            p.step(torch.from_numpy(x[it]), ortho=(it == NSTEPS - 1), reduced_gh=True)
        E = p.energy()
        torch.cuda.synchronize()
        out.append(state(p) + [host(E)])
    return out


def run_batch(items):
    batch = KptBatch([it[3] for it in items])
    fields = batch.fields([torch.from_numpy(it[2]) for it in items])
    batch.step(fields, ortho=True, energy=True)
    torch.cuda.synchronize()
    return batch, fields, [state(it[3]) + [host(batch.energy(i))] for i, it in enumerate(items)]


def close(a, b, tol):
    for x, y in zip(a, b):
        if x.dtype.kind in "iu":
            assert np.array_equal(x, y)
        else:
            assert rel(x, y) <= tol


def test_batch_equals_single_systems():
    _, _, got = run_batch(make())
    ref = run_single(make())
    for g, r in zip(got, ref):
        close(g, r, 1e-13)


def test_batch_fp64_systems_match_oracle():
    items = make()
    _, _, got = run_batch(items)
    for (case, prec), (s, U, x, p, pre), g in zip(BATCH, items, got):
        if prec != 0:
            continue
        Gh, ld = kp.greens(U, s.A)
        w = np.ones(U.shape[0])
        Ur = U
        for it in range(NSTEPS):
            o = kp.step(Ur, ld, w, x[it], pre, s.A, s.L, s.mesh, s.dt)
            Ur, ld, w = o["U"], o["logdet"], o["weight"]
        Ur = kp.orthonormalize(Ur)
        Gr, ldr = kp.greens(Ur, s.A)
        E = kp.local_energy(pre["Lh"], pre["h1h"], Gr, s.mesh)
        assert rel(g[0], Ur) < 1e-10, case
        assert phase_err(g[2], ldr) < 1e-9, case
        np.testing.assert_allclose(g[3], w, rtol=1e-10, atol=1e-14)
        # the energy kernels at the state the GPU reached: the FP64 bar
        Eg = kp.local_energy(pre["Lh"], pre["h1h"], g[1], s.mesh)
        assert energy_err(g[5], Eg, s.nk, overlap_cond(g[0], s.A)) <= 1.0, case
        # against the oracle's own trajectory: two steps amplify rounding differences of
        # the walkers (1e-13 -> 1e-11 relative) and the parts of E cancel, so the bar is
        # relative to the size of the parts
        scale = np.abs(E).sum(1)
        assert (np.abs(g[5] - E).sum(1) / scale).max() < 1e-11, case


def tensors(p):
    return (p.U, p.Gh, p.logdet, p.weight, p.status)


def test_graph_replays_match_eager():
    items = make()
    ps = [it[3] for it in items]
    init = [[t.clone() for t in tensors(p)] for p in ps]
    batch = KptBatch(ps)
    fields = batch.fields([torch.from_numpy(it[2]) for it in items])
    batch.step(fields, ortho=True, energy=True)
    torch.cuda.synchronize()
    ref = [state(p) + [host(batch.energy(i))] for i, p in enumerate(ps)]
    g = batch.graph(fields, ortho=True, energy=True)
    try:
        for rep in range(3):
            for p, st in zip(ps, init):
                for dst, src in zip(tensors(p), st):
                    dst.copy_(src)
            # eager library work between replays (its result is overwritten by the replay)
            batch.greens()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for i, p in enumerate(ps):
                close(state(p) + [host(batch.energy(i))], ref[i], 0.0)
    finally:
        g.close()


def test_autotune_keeps_results_and_state():
    items = make()
    ps = [it[3] for it in items]
    batch = KptBatch(ps)
    before = [state(p) for p in ps]
    batch.autotune()
    torch.cuda.synchronize()
    for p, b in zip(ps, before):
        close(state(p), b, 0.0)  # the walker state is untouched
    fields = batch.fields([torch.from_numpy(it[2]) for it in items])
    batch.step(fields, ortho=True, energy=True)
    torch.cuda.synchronize()
    got = [state(p) + [host(batch.energy(i))] for i, p in enumerate(ps)]
    ref = run_single(make())
    # another tile shape changes which workgroup computes an entry, not its K order
    for g_, r in zip(got, ref):
        close(g_, r, 1e-13)
