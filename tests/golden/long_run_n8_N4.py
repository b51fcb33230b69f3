"""Writes long_run_n8_N4.npz: the oracle after 1000 LSRK(5,4) steps on the
heterogeneous cube of 8^3 x 6 = 3,072 tets at N=4.

Recipe (the bench workload's medium and source on a smaller cube): Kuhn
periodic cube n=8, N=4, mu = 1 + 0.5 sin 2 pi x cos 2 pi y,
lambda = 2 + 0.5 cos 2 pi z, rho = 1 + 0.3 sin 2 pi (x+y+z) at the Stroud
points, Ricker point force f0 = 5, t0 = 0.2, amp 1, direction z at
(0.05, -0.10, 0.15), zero initial state at t = 0, dt at CFL 0.5 (Sec. 4.4
scaling), upwind flux, four receivers recorded after every full step.

Stored: the final modal coefficients of 256 elements (the source element,
elements 0 and K-1, the four receivers' elements and a seeded sample), their
values at the Stroud quadrature points, the total energy (Sec. 2 weighted
norm) and the receiver traces.  Tests compare the GPU state on the stored
elements at the quadrature points, element by element, and the energy and
traces globally; the benchmark reads the stored quadrature values.

Calls only oracle/ and the input generators.  Run from the repository root:
    python tests/golden/long_run_n8_N4.py
or, to add the quadrature values to an existing file without rerunning:
    python tests/golden/long_run_n8_N4.py --quadrature-values
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

N, NHEX, NSTEPS, NSAMPLE = 4, 8, 1000, 256
SRC = dict(xs=(0.05, -0.10, 0.15), direction=(0.0, 0.0, 1.0), amp=1.0, f0=5.0, t0=0.2)
RECEIVERS = np.array([[0.30, -0.10, 0.15], [0.05, 0.40, -0.20], [-0.60, 0.55, 0.70], [0.05, -0.10, 0.15]])


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

    def progress(n, t, c):
        if (n + 1) % 100 == 0:
            print("step", n + 1, "t", t, flush=True)

    c, t, traces = timestep.run(op, np.zeros((op.K, 9, op.Np)), dt, NSTEPS, t=0.0, source=src,
                                receivers=RECEIVERS, callback=progress)
    fixed = [op.locate(np.array(SRC["xs"]))[0], 0, op.K - 1] + [op.locate(x)[0] for x in RECEIVERS]
    fixed = np.unique(np.array(fixed, dtype=np.int64))
    rng = np.random.default_rng(8)
    rest = np.setdiff1d(np.arange(op.K), fixed)
    elems = np.sort(np.concatenate([fixed, rng.choice(rest, NSAMPLE - len(fixed), replace=False)]))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_run_n8_N4.npz")
    np.savez_compressed(out, elems=elems, c=c[elems], fq=op.to_q(c[elems]), dt=dt, t=t, nsteps=NSTEPS,
                        energy=op.energy(c), receivers=RECEIVERS, traces=traces)
    print("wrote", out, "dt", dt, "t", t, "energy", op.energy(c))


def add_quadrature_values():
    """Values at the quadrature points of the stored coefficients (the
    oracle's modal-to-quadrature evaluation), added to the existing file."""
    from oracle.reference import Reference
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_run_n8_N4.npz")
    g = dict(np.load(out))
    g["fq"] = Reference(N).to_q(g["c"])
    np.savez_compressed(out, **g)
    print("added fq", g["fq"].shape, "to", out)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--quadrature-values":
        add_quadrature_values()
    else:
        main()
