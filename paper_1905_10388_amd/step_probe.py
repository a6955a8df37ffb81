"""Run a few SBDF steps of one 2-D workload (for profilers and counters).

    python3 -m paper_1905_10388_amd.step_probe [fp64|mixed] [NxxNz] [steps]

Synthetic conductive state plus seeded noise; Ra = 1e8, Pr = 1, dt = 1e-5;
Lx = 4 (16 when Nx > 1024).
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import seeded_inputs as si  # noqa: E402
from paper_1905_10388_amd import RBSolver  # noqa: E402


def main(argv):
    prec = argv[1] if len(argv) > 1 else "fp64"
    Nx, Nz = (1024, 256) if len(argv) < 3 else tuple(int(v) for v in argv[2].split("x"))
    steps = int(argv[3]) if len(argv) > 3 else 12
    g = RBSolver(Nx, Nz, 4.0 if Nx <= 1024 else 16.0, 1e8, 1.0, precision=prec)
    j = np.arange(Nz)
    z = 0.5 * (1.0 - np.cos(np.pi * (j + 0.5) / Nz))
    g.initial_state(torch.from_numpy((1.0 - z) + 1e-3 * z * (1.0 - z) * si.workload_noise((Nx, Nz), 0)))
    for _ in range(steps):
        g.step(1e-5)
    torch.cuda.synchronize()
    g.check()
    print("done", prec, Nx, Nz, steps, flush=True)


if __name__ == "__main__":
    main(sys.argv)
