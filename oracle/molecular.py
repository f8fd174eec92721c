"""Standard (molecular) representation, used for the Nk = 1 reduction (test infrastructure only).

Only tests, the repository smoke check and the benchmark's CPU-baseline leg
may import this module.

Follows the standard-representation section with half-rotated intermediates:
  Lh_ar,g  = sum_p L_pr,g conj(A_pa),     Lbar_bs,g = sum_q conj(L_sq,g) conj(A_qb)
  X_g = sum_ar Lh_ar,g Gh_ar,             Xbar_g = sum_bs Lbar_bs,g Gh_bs
  EC  = 1/2 sum_{g, sigma, sigma'} X_g Xbar_g
  T_ab,g = sum_r Lh_ar,g Gh_br,           Tbar_ba,g = sum_s Lbar_bs,g Gh_as
  EX  = -1/2 sum_{a b g sigma} T_ab,g Tbar_ba,g
with both spins equal.
"""

from __future__ import annotations

import numpy as np


def energy_standard(L, h, A, Gh):
    """(E1B, EC, EX) for one walker; L[p, r, g], h[p, q], A[p, a], Gh[a, r]."""
    Lh = np.einsum("prg,pa->arg", L, A.conj())
    Lbar = np.einsum("sqg,qb->bsg", L.conj(), A.conj())
    X = np.einsum("arg,ar->g", Lh, Gh)
    Xb = np.einsum("bsg,bs->g", Lbar, Gh)
    EC = 0.5 * 4.0 * np.sum(X * Xb)  # sigma, sigma' both run over 2 spins
    T = np.einsum("arg,br->abg", Lh, Gh)
    Tb = np.einsum("bsg,as->bag", Lbar, Gh)
    EX = -0.5 * 2.0 * np.einsum("abg,bag->", T, Tb)
    G = A.conj() @ Gh
    E1 = 2.0 * np.sum(h * G)
    return np.array([E1, EC, EX])


def force_bias_standard(L, A, Gh, dt):
    """xbar_g,+/- = -sqrt(dt) c+/- sum_{a r sigma} [Lh+/-]_ar,g Gh_ar with c+ = i, c- = 1."""
    LH = L.conj().transpose(1, 0, 2)
    Lp = 0.5 * (L + LH)
    Lm = 0.5 * (L - LH)
    Lhp = np.einsum("prg,pa->arg", Lp, A.conj())
    Lhm = np.einsum("prg,pa->arg", Lm, A.conj())
    sdt = np.sqrt(dt)
    xp = -sdt * 1j * 2.0 * np.einsum("arg,ar->g", Lhp, Gh)
    xm = -sdt * 1.0 * 2.0 * np.einsum("arg,ar->g", Lhm, Gh)
    return np.stack([xp, xm], axis=-1)
