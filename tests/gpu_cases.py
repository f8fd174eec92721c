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
    # band counts past 32 (the exchange and its adjoint with 16 K steps, 3 and 4 column
    # tiles), the largest band count, and nocc > 8 (one g and one walker per 16-wide tile)
    "m40": ((2, 1, 1), 40, 4, 37, 5, "random", "dense"),
    "m52": ((1, 2, 1), 52, 4, 45, 6, "random", "dense"),
    "m64": ((1, 1, 2), 64, 5, 30, 3, "random", "dense"),
    "occ10": ((2, 1, 1), 14, 10, 19, 3, "random", "dense"),
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


def overlap_cond(U, A):
    """2-norm condition number of each walker's overlap matrix A^H U (A block diagonal)."""
    nk, m, nocc = A.shape
    U = np.asarray(U).reshape(U.shape[0], nk, m, -1)
    O = np.einsum("kpa,wkpj->wkaj", A.conj(), U).reshape(U.shape[0], nk * nocc, -1)
    return np.linalg.cond(O)


def energy_bar(E, nk, cond):
    """FP64 energy bar per walker, Ha per cell: 1e-10, or the rounding floor of the walker's
    overlap inverse where that is larger.

    Gh = (U O^-1)^T computed in FP64 carries a relative error up to about eps cond(O); every
    part of E_L is a sum of products of two Gh entries, so the parts move by up to
    2 eps cond(O) times their magnitude.  Where that floor exceeds 1e-10 Ha/cell no FP64
    evaluation can meet the absolute bar, and the bar becomes the floor itself.
    """
    S = np.abs(np.asarray(E)).sum(axis=-1) / nk
    floor = 2.0 * np.finfo(np.float64).eps * np.asarray(cond) * S
    return np.maximum(1e-10, floor)


def energy_err(Eg, E, nk, cond):
    """Max over walkers and parts of |dE| per cell divided by energy_bar; <= 1 passes."""
    Eg, E = np.asarray(Eg), np.asarray(E)
    d = np.abs(Eg - E).max(axis=-1) / nk
    return float((d / energy_bar(E, nk, cond)).max())
