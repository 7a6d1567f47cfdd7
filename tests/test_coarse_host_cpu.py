"""Host logic of the coarse-model workflow (no GPU): the rollout loss and
error tallies, the shifted flow view, the choice of face threshold and
output scale, and the argument checks that run before any lattice is
made."""
import math

import numpy as np
import pytest

from paper_1508_02899_amd import coarse as CC


def _track(variances, rho):
    T = CC.Track()
    for i, v in enumerate(variances):
        T.steps.append(25 * (i + 1))
        T.variance.append(v)
        T.rho_r2.append(np.asarray(rho[i], dtype=np.float64))
    return T


def test_rollout_loss_and_errors_by_hand():
    """Recorded steps 25, 50, 75; from step 50 on the variances are off by
    +10 % and -10 % and <rho_r^2> matches: mean squared relative error
    0.01, mean absolute relative error 0.1, no <rho_r^2> error."""
    rho = [[1.0, 2.0, 3.0]] * 3
    ref = _track([1.0, 1.0, 1.0], rho)
    run = _track([5.0, 1.1, 0.9], rho)
    assert CC.rollout_loss(run, ref, 0.1, 50) == pytest.approx(0.01)
    e = CC.errors({"ref": ref, "run": run}, "ref", 0.1, from_step=50)["run"]
    assert e["variance"] == pytest.approx(0.1)
    assert e["rho_r2"] == 0.0
    # the step before from_step counts once it is included
    assert CC.rollout_loss(run, ref, 0.1, 0) == pytest.approx(
        (16.0 + 0.01 + 0.01) / 3)


def test_rollout_loss_adds_the_squared_density_error():
    """<rho_r^2> off by 10 % at every scale: the distance-averaged error is
    0.1 whatever the weights, so it adds 0.01 to the loss."""
    ref = _track([1.0, 1.0], [[1.0, 2.0, 4.0]] * 2)
    run = _track([1.0, 1.0], [[1.1, 2.2, 4.4]] * 2)
    assert CC.rollout_loss(run, ref, 0.05, 0) == pytest.approx(0.01)


def test_shifted_flow_view():
    u = np.arange(10 * 2).reshape(10, 2)
    fl = (lambda k: u[k:k + 1])
    fl.all = u
    sh = CC._shifted(fl, 4)
    assert sh.all.shape[0] == 6
    assert np.array_equal(sh(0), u[4:5])
    assert np.array_equal(sh(5), u[9:10])


def test_choose_setting():
    table = {(0.01, 1.0): (0.03, 0.001), (0.01, 1.25): (0.02, 0.001),
             (0.05, 1.0): (0.025, 0.03), (0.05, 1.25): (0.028, 0.002)}
    # both thresholds fast enough: the smallest larger error wins
    assert CC.choose_setting(table, {0.01: 4.5, 0.05: 5.0}, 4.1) == \
        (0.01, 1.25)
    # only the larger threshold reaches the bound
    assert CC.choose_setting(table, {0.01: 3.9, 0.05: 4.3}, 4.1) == \
        (0.05, 1.25)
    # none reaches it: the fastest threshold's best pair
    assert CC.choose_setting(table, {0.01: 3.0, 0.05: 3.5}, 4.1) == \
        (0.05, 1.25)


def _fake_flows(lengths):
    out = {}
    for k, n in lengths.items():
        fl = (lambda k_: None)
        fl.all = np.zeros((n, 1))
        out[k] = fl
    return out


def test_workflow_refuses_short_flows_and_bad_thresholds():
    flows = _fake_flows({"train": 100, "valid": 225, "eval": 225})
    with pytest.raises(ValueError, match="train flow"):
        CC.build_and_evaluate(32, 65, 2.0, 1e-4, 3.0, flows)
    flows = _fake_flows({"train": 400, "valid": 100, "eval": 225})
    with pytest.raises(ValueError, match="valid flow"):
        CC.build_and_evaluate(32, 65, 2.0, 1e-4, 3.0, flows)
    flows = _fake_flows({"train": 400, "valid": 225, "eval": 225})
    with pytest.raises(ValueError, match="train_eps"):
        CC.build_and_evaluate(32, 65, 2.0, 1e-4, 3.0, flows,
                              train_eps=0.02, thresholds=(0.01, 0.03))


def test_initial_params_layout():
    p = CC.initial_params(3)
    assert p.shape == (4801,) and p.dtype == np.float32
    # biases zero, output layer small
    assert not p[512:576].any() and not p[4672:4736].any() and p[4800] == 0
    assert np.abs(p[4736:4800]).max() < 0.05
    assert math.isclose(float(np.std(p[:512])), 1 / math.sqrt(8), rel_tol=0.2)
