"""Writes wave16_p3_cfl_dt.txt: the CFL time step (Sec. 4.2, eqn. timestep,
with the cell diameter as h) of the density wave on the periodic Voronoi mesh
of 16^3 jittered seeds at N = 3 and CFL 0.004, computed by the oracle over all
4096 cells.  The full-size GPU test reads it instead of rebuilding every cell
of the oracle (about a minute of CPU).  Run from the repository root:

    python tests/golden/make_cfl_dt.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from afe_inputs.fields import density_wave  # noqa: E402
from afe_inputs.mesh import jittered_lattice_seeds, periodic_voronoi  # noqa: E402
from oracle.scheme import Oracle, Params  # noqa: E402

RECIPE = dict(n=16, jitter=0.25, seed=1, N=3, cfl=0.004)


def main():
    r = RECIPE
    mesh = periodic_voronoi(jittered_lattice_seeds(r["n"], r["jitter"], r["seed"]))
    o = Oracle(mesh, r["N"], Params())
    dt = o.cfl_dt(o.initial_state(density_wave), r["cfl"])
    with open(os.path.join(HERE, "wave16_p3_cfl_dt.txt"), "w") as f:
        f.write("# CFL time step of the density wave (amplitude 0.2, velocity (1,1,1), p = 1) on the\n")
        f.write("# periodic Voronoi mesh of 16^3 seeds jittered by +-0.25h (seed 1), N = 3, CFL 0.004;\n")
        f.write("# Sec. 4.2 eqn. timestep with h the cell diameter, written by make_cfl_dt.py (oracle only)\n")
        f.write(f"{dt!r}\n")
    print(dt)


if __name__ == "__main__":
    main()
