"""The pins must catch plausible mistakes in the oracle: each mutation below
plants one mistake (at every place the pattern occurs) in a copy of
oracle/oracle.c (on the CPU), builds it, and runs the pin suites against it;
at least one pin must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "koren_sixth": ("theta / 6.0", "theta / 5.0"),
    "koren_third": ("1.0 / 3.0 + theta", "1.0 / 2.0 + theta"),
    "koren_no_theta_cap": ("if (theta < psi) psi = theta;", ""),
    "drift_sign_1d": ("(u[site] - vj)", "(vj - u[site])"),
    "u_component_2d": ("const double uy = u[sites + site];",
                       "const double uy = u[site];"),
    "upwind_donor": ("double fp = P[k - 1];", "double fp = P[k];"),
    "minus_stencil": ("koren_correction(M[k - 1] - M[k], M[k] - M[k + 1])",
                      "koren_correction(M[k] - M[k - 1], M[k] - M[k + 1])"),
    "open_boundary_face": ("F[nv] = 0.0;", "F[nv] = F[nv - 1];"),
    "diffusion_sign": ("F[k] = -D * (c[k] - c[k - 1]);",
                       "F[k] = D * (c[k] - c[k - 1]);"),
    "diffusion_number": ("double D = kappa * dts / (dv * dv);",
                         "double D = kappa * dts / dv;"),
    "stream_direction_1d": ("wrap(x - s * (j - h), nx)",
                            "wrap(x + s * (j - h), nx)"),
    "stream_y_index_2d": ("wrap(y - s * (jy - h), ny)",
                          "wrap(y - s * (jx - h), ny)"),
    "order_diffusion_first": (
        "orc_drift_line(line, nv, nu, scheme);\n      orc_diffuse_line(line, nv, D);",
        "orc_diffuse_line(line, nv, D);\n      orc_drift_line(line, nv, nu, scheme);"),
    "flow_slice_ignored": ("long sl = u_hold > 0 ? step / u_hold : 0;",
                           "long sl = 0;"),
    "substep_length": ("double dts = dt / (double)nsub;", "double dts = dt;"),
    "second_moment_y": ("Q[1] += m * vy * vy;", "Q[1] += m * vy;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {old!r}"
    mut_c = tmp_path / "oracle_mut.c"
    mut_c.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o",
                           str(so), str(mut_c), "-lm"])
    env = dict(os.environ, ORACLE_LIB=str(so))
    rc = 0
    for suite in ("tests/test_oracle_pins.py", "tests/test_oracle_montecarlo.py"):
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                            "-p", "no:cacheprovider", "-m", "not gpu", suite],
                           cwd=ROOT, env=env, capture_output=True, text=True)
        assert r.returncode in (0, 1), r.stdout[-2000:] + r.stderr[-2000:]
        if r.returncode == 1:
            rc = 1
            break
    assert rc == 1, f"no pin caught the mutation {name}"
