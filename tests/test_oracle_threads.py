"""The OpenMP build of oracle.c (used only to time the benchmark's CPU
baseline on several host cores) computes the same bits as the plain
single-threaded build the tests use: sites are independent, and a site's
arithmetic does not depend on the thread that runs it."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
rng = np.random.default_rng(3)
for dim, shape, ushape in ((2, (81, 7, 13), (2, 2, 7, 13)),
                           (1, (17, 50), (2, 1, 50))):
    f = rng.random(shape)
    u = 0.4 * rng.standard_normal(ushape)
    out = oracle.step(f, u, dim=dim, dx=0.2, tau_p=2.0, kappa=0.01, dt=0.1,
                      nsteps=5, u_hold=3, nsub=2)
    np.save(sys.argv[2] + f"_{dim}.npy", out)
"""


def _run(tmp, lib, threads):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    if lib:
        env["ORACLE_LIB"] = lib
    else:
        env.pop("ORACLE_LIB", None)
    subprocess.check_call([sys.executable, "-c", SCRIPT, ROOT, str(tmp)],
                          env=env)
    return [np.load(f"{tmp}_{d}.npy") for d in (1, 2)]


def test_openmp_build_gives_the_plain_builds_bits(tmp_path):
    import oracle
    oracle.build()
    plain = _run(tmp_path / "plain", None, 1)
    omp = _run(tmp_path / "omp", oracle.OMP_SO, 4)
    for a, b in zip(plain, omp):
        assert np.array_equal(a, b)
