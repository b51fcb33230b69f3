"""Seeded stream of independent forward-solve requests for the serving loop.

Each request is a periodic cube of n^3 hexahedra x 6 tetrahedra at degree N
with its own smooth heterogeneous medium (random phases and amplitude
factors of the reference medium), a Ricker point source at a random
position, a number of time steps and an arrival time.  Arrivals are a
Poisson process of the given rate (exponential inter-arrival times).
"""
from dataclasses import dataclass, field

import numpy as np

from . import media
from .mesh import kuhn_periodic_mesh


@dataclass
class Request:
    rid: int
    n: int
    N: int
    nsteps: int
    xs: np.ndarray
    phases: tuple
    amps: tuple
    arrival: float = 0.0
    direction: tuple = (0.0, 0.0, 1.0)
    f0: float = 5.0
    t0: float = 0.2
    receivers: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))

    def mesh(self):
        return kuhn_periodic_mesh(self.n)

    def material(self, xyz):
        return media.smooth(xyz, phases=self.phases, amps=self.amps)


def request_stream(count, n_range=(8, 24), degrees=(3, 4, 5), nsteps=500, rate=None,
                   seed0=4, receivers=None):
    """Requests seeded individually with numpy.random.default_rng(seed0 + i).

    rate: arrivals per second (None: all arrive at t = 0).  Inter-arrival
    times come from numpy.random.default_rng(seed0).
    """
    reqs = []
    t = 0.0
    arr_rng = np.random.default_rng(seed0)
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        N = int(rng.choice(np.asarray(degrees)))
        xs = rng.uniform(-0.9, 0.9, size=3)
        phases = tuple(rng.uniform(0.0, 2.0 * np.pi, size=4))
        amps = tuple(rng.uniform(0.5, 1.5, size=3))
        if rate is not None and i > 0:
            t += float(arr_rng.exponential(1.0 / rate))
        rec = np.zeros((0, 3)) if receivers is None else np.asarray(receivers, float)
        reqs.append(Request(i, n, N, nsteps, xs, phases, amps, arrival=t, receivers=rec))
    return reqs
