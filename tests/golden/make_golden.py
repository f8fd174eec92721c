"""Write the stored oracle results of the 2x2x2 parity workload (calls only the oracle).

Run from the repository root:  python tests/golden/make_golden.py
The file it writes pins the oracle against accidental drift: any later change
of the oracle's arithmetic shows up as a failure of the regression test and has
to be justified by the passage of the paper it follows.
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth.kpt_inputs import make_config  # noqa: E402
from oracle import kpoint as kp  # noqa: E402


def compute():
    s, U, x = make_config("c0")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, logdet = kp.greens(U, s.A)
    E0 = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    out = kp.step(U, logdet, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    E1 = kp.local_energy(pre["Lh"], pre["h1h"], out["Gh"], s.mesh)
    return dict(
        config="mesh 2x2x2, m=8, nocc=2, nchol=24, 4 walkers, dt=0.005, seed 0",
        energy_initial=[[[c.real, c.imag] for c in row] for row in E0],
        energy_after_step=[[[c.real, c.imag] for c in row] for row in E1],
        logdet_after_step=[[c.real, c.imag] for c in out["logdet"]],
        weight_after_step=list(out["weight"]),
    )


if __name__ == "__main__":
    res = compute()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c0_oracle.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", path)
