"""Shared set-up for the GPU parity tests: seeded inputs -> GPU problem and oracle data."""

from __future__ import annotations

import numpy as np
import torch

from synth import make_system, make_walkers, make_fields
from oracle import kpoint as kp

# (mesh, m, nocc, nchol, nwalk, trial, walkers): meshes cover the molecular limit, self-inverse
# Q, anisotropic linearisation; sizes leave ragged MFMA tiles (m, nchol not multiples of 16).
CASES = {
    "c0": ((2, 2, 2), 8, 2, 24, 4, "identity", "blockdiag"),
    "mol": ((1, 1, 1), 11, 3, 13, 5, "random", "dense"),
    "aniso": ((2, 3, 1), 5, 3, 7, 6, "random", "dense"),
    "line3": ((3, 1, 1), 9, 4, 20, 7, "random", "dense"),
    "mixed": ((1, 2, 3), 6, 2, 17, 3, "random", "dense"),
    "wide": ((2, 2, 1), 26, 4, 40, 33, "random", "dense"),
}


def build(case, seed=0, prec=0):
    from paper_2003_09468_amd import KptProblem
    mesh, m, nocc, nchol, nw, trial, wk = CASES[case] if isinstance(case, str) else case
    s, rng = make_system(mesh, m, nocc, nchol, seed=seed, trial=trial)
    U = make_walkers(s, nw, rng, kind=wk)
    x = make_fields(s, nw, 2, rng)
    p = KptProblem(s.mesh, s.m, s.nocc, s.nchol, nw, s.dt, torch.from_numpy(s.L),
                   torch.from_numpy(s.A), prec=prec)
    p.prepare(torch.from_numpy(s.H1))
    p.set_walkers(torch.from_numpy(U))
    p.greens()
    torch.cuda.synchronize()
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    return s, U, x, p, pre


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


def phase_err(ld_gpu, ld_ref):
    """max |exp(ld_gpu - ld_ref) - 1|: log determinants agree modulo 2 pi i."""
    return np.abs(np.exp(np.asarray(ld_gpu) - np.asarray(ld_ref)) - 1.0).max()


def energy_err(Eg, E, nk):
    """Max over walkers of |dE| per cell divided by the FP64 bar for that walker.

    The bar is 1e-10 Ha/cell; for walkers with |E| > 1000 Ha/cell (near-singular overlaps,
    where FP64 rounding of the overlap inverse alone exceeds the absolute bar) it is 1e-13
    relative.  A value <= 1 passes.
    """
    Eg, E = np.asarray(Eg), np.asarray(E)
    d = np.abs(Eg - E) / nk
    mag = np.abs(E) / nk
    bar = np.maximum(1e-10, 1e-13 * mag)
    return float((d / bar).max())
