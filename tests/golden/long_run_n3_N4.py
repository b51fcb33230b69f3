"""Writes long_run_n3_N4.npz: the oracle's state after 1000 LSRK(5,4) steps.

Recipe: Kuhn periodic cube n=3 (162 tets), N=4, the smooth heterogeneous
medium (mu = 1 + 0.5 sin 2 pi x cos 2 pi y, lambda = 2 + 0.5 cos 2 pi z,
rho = 1 + 0.3 sin 2 pi (x+y+z) at the Stroud points), Ricker point force
f0 = 5, t0 = 0.2, amp 1, direction z at (0.05, -0.10, 0.15), zero initial
state at t = 0, dt at CFL 0.5 (Sec. 4.4 scaling), upwind flux.  Stores the
final modal coefficients; tests compare at the quadrature points.
Calls only oracle/ and the input generators.  Run from the repository root:
    python tests/golden/long_run_n3_N4.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import timestep  # noqa: E402
from oracle.dg import Elastic  # noqa: E402
from oracle.reference import stroud_rule  # noqa: E402
from workloads import media  # noqa: E402
from workloads.mesh import kuhn_periodic_mesh  # noqa: E402

N, NHEX, NSTEPS = 4, 3, 1000
SRC = dict(xs=(0.05, -0.10, 0.15), direction=(0.0, 0.0, 1.0), amp=1.0, f0=5.0, t0=0.2)


def quad_xyz(VXYZ, N):
    xq, _ = stroud_rule(N)
    X0 = VXYZ[:, 0]
    A = np.stack([VXYZ[:, 1] - X0, VXYZ[:, 2] - X0, VXYZ[:, 3] - X0], axis=-1) / 2.0
    return np.einsum('qd,kjd->kqj', xq + 1.0, A) + X0[:, None, :]


def main():
    EToV, VXYZ = kuhn_periodic_mesh(NHEX)
    op = Elastic(N, VXYZ, *media.smooth(quad_xyz(VXYZ, N)))
    src = timestep.Source(SRC["xs"], SRC["direction"], SRC["amp"], SRC["f0"], SRC["t0"])
    dt = timestep.cfl_dt(op, 0.5)
    c, t, _ = timestep.run(op, np.zeros((op.K, 9, op.Np)), dt, NSTEPS, t=0.0, source=src)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_run_n3_N4.npz")
    np.savez_compressed(out, c=c, dt=dt, t=t, nsteps=NSTEPS, energy=op.energy(c))
    print("wrote", out, "dt", dt, "t", t, "energy", op.energy(c))


if __name__ == "__main__":
    main()
