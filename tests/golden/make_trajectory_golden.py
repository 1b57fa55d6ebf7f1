"""Write the FP64 oracle's long-run references of the two larger workloads.
Calls only oracle/ and the workload definitions.  Run from the repository
root (about 40 minutes on 8 cores):

    python tests/golden/make_trajectory_golden.py [single128] [pair_collinear] [pair_side]

single128_x_2000.txt   the 128^3 swimmer (seed 0): swimmer centre X(n) at
                       every step n = 0..2000 (the first actuation period).
pair256_<arrangement>_10000.npz
                       the 256x128x128 pair (seed 0), 10000 steps: both
                       swimmer centres every 10 steps, every marker at the
                       end, and the final velocity field on every fourth node
                       per axis (u[:, ::4, ::4, ::4], layout [3][z][y][x]).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import orc  # noqa: E402
from paper_2202_12147_amd import workloads  # noqa: E402


def _oracle(case):
    o = orc.Oracle(case["shape"], case["tau"], case["forcing"], case["width"])
    for sw in case["swimmers"]:
        o.add_swimmer_desc(sw)
    return o


def single128(steps=2000):
    case = workloads.single_128(seed=0)
    o = _oracle(case)
    X = [o.swimmer_centres()[0].copy()]
    t0 = time.time()
    for n in range(steps):
        o.step(1)
        X.append(o.swimmer_centres()[0].copy())
        if n % 200 == 199:
            print(f"single128 step {n + 1} ({time.time() - t0:.0f} s)", flush=True)
    X = np.array(X)
    assert np.isfinite(X).all()
    with open(os.path.join(HERE, f"single128_x_{steps}.txt"), "w") as f:
        f.write("# FP64 oracle, workloads.single_128(seed=0): 128^3, tau 0.8, Guo, 4-point kernel,\n")
        f.write(f"# radius-4 beads (1280 triangles), spacing 16, A = B = 5e-4, T = 2000; swimmer centre"
                f" X(n), n = 0..{steps}\n")
        f.write("# n x y z\n")
        for n, x in enumerate(X):
            f.write(f"{n} {x[0]:.17e} {x[1]:.17e} {x[2]:.17e}\n")


def pair256(arrangement, steps=10000, every=10):
    case = workloads.pair_256(seed=0, arrangement=arrangement)
    o = _oracle(case)
    X = [o.swimmer_centres().copy()]
    t0 = time.time()
    for n in range(0, steps, every):
        o.step(every)
        X.append(o.swimmer_centres().copy())
        if (n + every) % 1000 == 0:
            print(f"pair {arrangement} step {n + every} |u|max {np.abs(o.velocity()).max():.3e}"
                  f" ({time.time() - t0:.0f} s)", flush=True)
    u = o.velocity()
    X = np.array(X)
    assert np.isfinite(X).all() and np.isfinite(u).all()
    np.savez_compressed(os.path.join(HERE, f"pair256_{arrangement}_{steps}.npz"), X=X, every=every,
                        markers=o.markers(), u_sub=u[:, ::4, ::4, ::4].copy(),
                        u_l2=np.linalg.norm(u), u_max=np.abs(u).max())


def main():
    orc.set_threads(min(16, len(os.sched_getaffinity(0))))
    which = sys.argv[1:] or ["single128", "pair_collinear", "pair_side"]
    if "single128" in which:
        single128()
    for arr in ("collinear", "side"):
        if f"pair_{arr}" in which:
            pair256(arr)


if __name__ == "__main__":
    main()
