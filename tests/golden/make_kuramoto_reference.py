"""Writes kuramoto_n4096_ref.npy: the oracle's Dormand-Prince 5(4) solution (FP64,
rtol = atol = 1e-12) of the default benchmark workload, Kuramoto N = 4096 with
dense weights, K = 2, seed 2000, t in [0, 50], at t = 50.  The reference
integrator of the accuracy comparisons (the paper measures its solvers against
a fifth-order Dormand-Prince solution at a tight tolerance, Sec. 2.4); this
script calls only the oracle and the seeded input generator.

Usage: python tests/golden/make_kuramoto_reference.py   (several minutes of CPU)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "kuramoto_n4096_ref.npy")


def main():
    w = workloads.kuramoto(4096, seed=2000, K=2.0, t1=50.0, rtol=1e-6)
    t = time.time()
    y, st = oracle.dp54_solve(w["kind"], w["n"], w["y0"], 0.0, 50.0, 1e-12, 1e-12, A=w["A"], param=w["param"],
                              gain=w["gain"], i_max=10_000_000)
    assert st["status"] == 0 and st["t_reached"] == 50.0, st
    np.save(OUT, y)
    print(f"wrote {OUT}: {st['n_accept']} accepted, {st['n_reject']} rejected, {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()
