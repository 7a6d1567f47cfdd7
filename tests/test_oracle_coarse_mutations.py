"""The corrected-site pins must catch plausible mistakes in
oracle/coarse.corrected_site: each mutation plants one mistake in a copy of
oracle/coarse.py (in memory, on the CPU), and at least one of the pins must
fail against the mutated module."""
import importlib.util
import os

import pytest

import test_oracle_coarse as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "coarse.py")

MUTATIONS = {
    "flux_sign": ("G = np.where(use, sg * ms *", "G = np.where(use, -sg * ms *"),
    "xy_faces_swapped": (
        "Gx = G[:nfx].reshape(nv, nv - 1).copy()   # [jy, k-1]\n"
        "    Gy = G[nfx:].reshape(nv - 1, nv).T.copy()",
        "Gx = G[nfx:].reshape(nv, nv - 1).copy()   # [jy, k-1]\n"
        "    Gy = G[:nfx].reshape(nv - 1, nv).T.copy()"),
    "y_faces_untransposed": ("Gy = G[nfx:].reshape(nv - 1, nv).T.copy()",
                             "Gy = G[nfx:].reshape(nv, nv - 1).copy()"),
    "x_donor_side": ("donor = c[a, k - 1] if gx > 0 else c[a, k]",
                     "donor = c[a, k] if gx > 0 else c[a, k - 1]"),
    "y_donor_side": ("donor = c[k - 1, a] if gy > 0 else c[k, a]",
                     "donor = c[k, a] if gy > 0 else c[k - 1, a]"),
    "limit_fraction": ("np.clip(gx, -0.25 * donor, 0.25 * donor)",
                       "np.clip(gx, -0.5 * donor, 0.5 * donor)"),
    "threshold_not_relative": ("(ms >= line_eps * M)", "(ms >= line_eps)"),
    "no_stencil_mass_scale": ("sg * ms * np.asarray(y", "sg * np.asarray(y"),
}

CHECKS = [pins.check_corrected_site_hand_example,
          pins.check_corrected_site_closes_min_norm_targets]


def _mutant(name, src):
    spec = importlib.util.spec_from_loader(f"coarse_mut_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src, f"<coarse mutant {name}>", "exec"), mod.__dict__)
    return mod


def test_unmutated_copy_passes():
    mod = _mutant("none", open(SRC).read())
    for check in CHECKS:
        check(mod)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_corrected_site_pins_catch_mutation(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {old!r}"
    mod = _mutant(name, src.replace(old, new))
    caught = 0
    for check in CHECKS:
        try:
            check(mod)
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught the mutation {name}"
