"""Writes tests/golden/rising_bubble_128x128x256_100steps.json: the FP64 oracle
run of the rising-bubble workload (128 x 128 x 256, no-slip walls on every
face, density ratio 1000, dynamic viscosity ratio 100, Eo 10, Mo 1e-3; the
Sec. III.A set-up) over 100 time steps of Sec. II.D, evaluated at fixed
sample nodes.

Calls only the oracle (oracle/scheme.py) and the seeded input generator
(paper_2501_00846_amd/workloads.py).  Stored per sample node: the 11 state
fields (phi, P, Jx, Jy, Jz, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz) and the observables
rho, u, p; and per field the maximum magnitude and the L2 norm over the whole
box, which the parity test uses as the scale of its relative tolerance.

Run from the repository root:  python tests/golden/make_rising_bubble_100.py
(about 75 minutes on one core, ~8 GB of memory)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import scheme as S  # noqa: E402
from paper_2501_00846_amd import workloads  # noqa: E402

STEPS = 100
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rising_bubble_128x128x256_100steps.json")


def sample_nodes(nx, ny, nz):
    """Corners, every wall face, the bubble's poles and equator (R 16 at
    z = 48), the column above it, and seeded random nodes."""
    pts = {(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, 0), (nx - 1, 0, nz - 1),
           (nx // 2, ny // 2, 0), (nx // 2, ny // 2, 1), (nx // 2, ny // 2, nz - 1),
           (nx // 2, ny // 2, nz - 2), (0, ny // 3, nz // 2), (nx - 1, ny // 3, nz // 2),
           (nx // 3, 0, nz // 2), (nx // 3, ny - 1, nz // 2), (1, 1, 1),
           (64, 64, 32), (64, 64, 48), (64, 64, 64), (48, 64, 48), (80, 64, 48), (64, 48, 48),
           (64, 80, 48), (64, 64, 30), (64, 64, 66), (64, 64, 100), (63, 63, 49), (70, 58, 55)}
    rng = np.random.default_rng(2024)
    while len(pts) < 64:
        pts.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return sorted(pts)


def main():
    case = workloads.rising_bubble()
    prob = case.problem
    st = S.initial_state(case.phi, case.u, case.pstar)
    t0 = time.time()
    for k in range(STEPS):
        st = S.step(st, prob)
        print("step %d done (%.0f s)" % (k + 1, time.time() - t0), flush=True)
    ob = S.observables(st, prob)
    state = np.concatenate([st.phi[None], st.P[None], st.J, S.q_six(st.Q)])
    names = ["phi", "P", "Jx", "Jy", "Jz", "Qxx", "Qyy", "Qzz", "Qxy", "Qxz", "Qyz"]
    obs = {"rho": ob["rho"], "ux": ob["u"][0], "uy": ob["u"][1], "uz": ob["u"][2], "p": ob["p"]}
    pts = sample_nodes(prob.nx, prob.ny, prob.nz)
    idx = tuple(np.array([[z for x, y, z in pts], [y for x, y, z in pts], [x for x, y, z in pts]]))
    out = {
        "description": ("FP64 oracle, rising bubble 128x128x256 with walls, 100 steps from the seeded "
                        "initial fields (workloads.rising_bubble(), seed 2); written by "
                        "tests/golden/make_rising_bubble_100.py"),
        "steps": STEPS,
        "nodes": [list(p) for p in pts],
        "state": {n: [float(v) for v in state[k][idx]] for k, n in enumerate(names)},
        "observables": {n: [float(v) for v in a[idx]] for n, a in obs.items()},
        "max_abs": {**{n: float(np.abs(state[k]).max()) for k, n in enumerate(names)},
                    **{n: float(np.abs(a).max()) for n, a in obs.items()}},
        "l2": {**{n: float(np.linalg.norm(state[k])) for k, n in enumerate(names)},
               **{n: float(np.linalg.norm(a)) for n, a in obs.items()}},
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
