"""Pins of the coarse-lattice / correction-network oracle (oracle/coarse.py)."""
import math

import numpy as np
import pytest

from oracle import coarse as C


def test_restrict_weights_partition_each_fine_cell():
    R = C.restrict_weights(65)
    assert R.shape == (17, 65)
    np.testing.assert_array_equal(R.sum(axis=0), np.ones(65))
    # coarse centre J sits on fine index 4J; symmetric weights
    np.testing.assert_array_equal(R, R[::-1, ::-1])
    assert R[3, 12] == 1 and R[3, 14] == 0.5 and R[4, 14] == 0.5


def test_restrict_conserves_mass():
    rng = np.random.default_rng(1)
    nvf = 33
    f = rng.random((nvf * nvf, 3, 4))
    fc = C.restrict(f, 2)
    # masses: fine cells weigh dv^2, coarse cells (4 dv)^2
    assert fc.sum() * 16 == pytest.approx(f.sum(), rel=1e-14)


def test_restrict_maps_coarse_centred_mass_exactly():
    """Mass sitting on fine cells 4J (the coarse centres) lands unchanged in
    coarse cell J (density divided by 4 per axis)."""
    nvf = 17
    f = np.zeros((nvf * nvf, 2))
    f[(4 * 2) * nvf + 4 * 3, 0] = 8.0   # (jy, jx) = (8, 12) -> (2, 3)
    f[(4 * 0) * nvf + 4 * 4, 1] = 16.0  # (0, 16) -> (0, 4)
    fc = C.restrict(f, 2)
    want = np.zeros((25, 2))
    want[2 * 5 + 3, 0] = 0.5
    want[0 * 5 + 4, 1] = 1.0
    np.testing.assert_array_equal(fc, want)


def test_minnorm_fluxes_reproduce_residual_and_lie_in_range():
    rng = np.random.default_rng(2)
    n = 7
    r = rng.standard_normal((n * n, 5))
    r -= r.mean(axis=0)
    Gx, Gy = C.minnorm_fluxes(r, n)
    G = np.concatenate([Gx.reshape(-1, 5), Gy.reshape(-1, 5)])
    D = C.divergence_matrix(n)
    np.testing.assert_allclose(-D @ G, r, atol=1e-12)
    # least norm <=> G = D^T psi for some psi
    psi, *_ = np.linalg.lstsq(D.T, G, rcond=None)
    np.testing.assert_allclose(D.T @ psi, G, atol=1e-12)


def test_divergence_matrix_is_conservative():
    D = C.divergence_matrix(5)
    np.testing.assert_array_equal(D.sum(axis=0), np.zeros(D.shape[1]))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = C.init_params(rng, scale=1.5)
    P["b1"] = rng.standard_normal(C.NH) * 0.3
    P["b2"] = rng.standard_normal(C.NH) * 0.3
    X = rng.standard_normal((40, C.NF))
    t = rng.standard_normal(40)
    w = rng.random(40)
    L, g = C.loss_and_grads(P, X, t, w, quantize=False)
    h = 1e-6
    for k, idx in [("W1", (3, 7)), ("b1", (11,)), ("W2", (5, 40)),
                   ("b2", (63,)), ("w3", (17,)), ("b3", ())]:
        Pp = {q: v.copy() for q, v in P.items()}
        Pm = {q: v.copy() for q, v in P.items()}
        Pp[k][idx] += h
        Pm[k][idx] -= h
        Lp, _ = C.loss_and_grads(Pp, X, t, w, quantize=False)
        Lm, _ = C.loss_and_grads(Pm, X, t, w, quantize=False)
        assert g[k][idx] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-5, abs=1e-9)


def test_gelu_closed_forms():
    z = np.array([0.0, 1e-8, 30.0, -30.0])
    g = C.gelu(z)
    assert g[0] == 0.0 and g[2] == pytest.approx(30.0) and abs(g[3]) < 1e-12
    assert C.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5)
    # tanh form vs the exact erf form: |diff| < 1e-3 (published bound ~5e-4)
    from scipy.special import erf
    zz = np.linspace(-5, 5, 1001)
    exact = 0.5 * zz * (1 + erf(zz / math.sqrt(2)))
    assert np.abs(C.gelu(zz) - exact).max() < 1e-3


def test_bf16_rounding():
    assert C.bf16(1.0) == 1.0
    assert C.bf16(1.0 + 2 ** -9) == 1.0          # ties to even
    assert C.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7
    assert C.bf16(-3.0) == -3.0


def test_adam_first_step_is_sign_step():
    P = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-3])}
    st = {}
    C.adam(P, g, st, lr=0.01)
    np.testing.assert_allclose(P["a"], [0.99, -1.99, 0.49], atol=1e-7)


def test_divergence_matrix_hand_example():
    """n = 2 by hand: unknowns x-face (row 0, k = 1), x-face (row 1, k = 1),
    y-face (k = 1, column 0), y-face (k = 1, column 1); (D G)_J is the flux
    out of cell J through its upper faces minus the flux into it through
    its lower faces."""
    D = C.divergence_matrix(2)
    want = np.array([[1, 0, 1, 0],      # cell (jy, jx) = (0, 0)
                     [-1, 0, 0, 1],     # (0, 1)
                     [0, 1, -1, 0],     # (1, 0)
                     [0, -1, 0, -1]])   # (1, 1)
    np.testing.assert_array_equal(D, want)


def check_corrected_site_hand_example(C):
    """3 x 3 square c[jy, jx] = 1..9 (mass 45), stencil masses 1 (one face
    0.01), line_eps 0.01 (threshold 0.45).  Face index: x-face (row a, face
    k) = 2 a + k - 1; y-face (face k, column a) = 6 + 3 (k - 1) + a.  A
    positive flux moves mass toward larger velocity index, a negative one
    toward smaller; each face moves at most a quarter of its donor.
      x (1, 1): +0.5 from (1,0) to (1,1), donor 4 -> not limited;
      y (2, 2): -1.0 from (2,2) to (1,2), donor 9 -> not limited;
      x (0, 2): +1.0 from (0,1) to (0,2), donor 2 -> limited to 0.5;
      y (1, 0): -3.0 from (1,0) to (0,0), donor 4 -> limited to 1.0;
      x (2, 1): stencil mass 0.01 < 0.45 -> no correction."""
    nv = 3
    c = np.arange(1.0, 10.0)
    nf = 2 * nv * (nv - 1)
    y = np.zeros(nf)
    ms = np.ones(nf)
    sg = np.ones(nf)
    y[2], sg[2] = 0.5, 1.0
    y[11], sg[11] = 1.0, -1.0
    y[1], sg[1] = 1.0, 1.0
    y[6], sg[6] = 3.0, -1.0
    y[4], ms[4] = 70.0, 0.01
    out = C.corrected_site(c, nv, y, ms, sg, line_eps=0.01)
    want = np.array([[2.0, 1.5, 3.5],
                     [2.5, 5.5, 7.0],
                     [7.0, 8.0, 8.0]])
    np.testing.assert_allclose(out.reshape(nv, nv), want, rtol=0,
                               atol=1e-15)


def check_corrected_site_closes_min_norm_targets(C):
    """With y set to the least-norm face fluxes of f_true - f_pred divided by
    sign x stencil mass, no face excluded and every flux below a quarter of
    its donor, the corrected f_pred is f_true."""
    rng = np.random.default_rng(11)
    nv = 9
    fp = 1.0 + rng.random(nv * nv)
    ft = fp + 1e-3 * rng.standard_normal(nv * nv)
    ft += (fp.sum() - ft.sum()) / ft.size
    Gx, Gy = C.minnorm_fluxes((ft - fp).reshape(-1, 1), nv)
    G = np.concatenate([Gx.reshape(-1), Gy.reshape(-1)])
    _, ms, sg = C.face_features(fp, nv, 0.3, -0.2, 0.5, 0.1, 1.0, 2.0)
    assert np.all(ms > 0) and np.abs(G).max() < 0.25
    out = C.corrected_site(fp, nv, G / (sg * ms), ms, sg, line_eps=0.0)
    np.testing.assert_allclose(out, ft, rtol=0, atol=1e-13)
    assert np.abs(out - fp).max() > 1e-4    # the correction did something


def test_corrected_site_hand_example():
    check_corrected_site_hand_example(C)


def test_corrected_site_closes_min_norm_targets():
    check_corrected_site_closes_min_norm_targets(C)


def test_corrected_site_conserves_mass_and_positivity():
    rng = np.random.default_rng(4)
    nv = 9
    fc = rng.random(nv * nv) ** 3
    X, ms, sg = C.face_features(fc, nv, 0.4, -0.3, 0.5, 0.1, 1.0, 2.0)
    y = rng.standard_normal(len(ms)) * 5  # large corrections get limited
    out = C.corrected_site(fc, nv, y, ms, sg)
    assert out.sum() == pytest.approx(fc.sum(), rel=1e-13)
    assert out.min() >= -1e-15


def test_face_features_hand_example():
    """Hand-built 5x5 square (rows jy, columns jx), u = 0: the stencil is
    read from the upwind side (donor first), normalised by its mass; the
    drift feature is |nu| = dt |u - v_face| / (tau_p dv)."""
    nv, dv, dt, tau, St = 5, 0.5, 0.2, 2.0, 3.0
    c = np.zeros((nv, nv))
    c[0, :] = [1, 2, 3, 4, 5]          # row jy = 0 carries the x-faces checked
    X, ms, sg = C.face_features(c.ravel(), nv, 0.0, 0.0, dv, dt, tau, St)
    assert X.shape == (2 * nv * (nv - 1), 8)
    # x-face k = 2 of row 0 (index 1): v_face = -dv/2 < u -> nu > 0, donor
    # cell 1; stencil cells (-1, 0, 1, 2, 3) = (0, 1, 2, 3, 4), mass 10
    assert ms[1] == 10 and sg[1] == 1
    assert np.allclose(X[1], [0, .1, .2, .3, .4, 0.5 * dt / tau, np.log(St), 0])
    # x-face k = 3 (index 2): v_face = +dv/2 -> nu < 0, donor cell 3;
    # stencil cells (5, 4, 3, 2, 1) = (0, 5, 4, 3, 2), mass 14
    assert ms[2] == 14 and sg[2] == -1
    assert np.allclose(X[2, :5], np.array([0, 5, 4, 3, 2]) / 14)
    assert X[2, 5] == pytest.approx(0.5 * dt / tau)
    # y-faces of an empty column carry no mass and zero stencil features
    ny0 = nv * (nv - 1)
    assert ms[ny0 + 1 * nv + 4] > 0      # column 4: row 0 holds 5
    assert ms[ny0 + 3 * nv + 4] == 0     # face 4 of column 4: cells 1..4 empty
    assert np.all(X[ny0 + 3 * nv + 4, :5] == 0)


@pytest.mark.parametrize("nv,s,nsub,scheme", [(65, 1, 3, "koren"),
                                              (17, 4, 2, "koren"),
                                              (9, 1, 2, "upwind")])
def test_collide_site_is_the_lattice_step_of_a_one_site_lattice(nv, s, nsub,
                                                                scheme):
    """On a 1 x 1 periodic lattice streaming is the identity, so a full
    lattice step of the C oracle is the collision alone; the recorded face
    fluxes reproduce the change exactly (c0 - div F = c1)."""
    import oracle
    rng = np.random.default_rng(nv + s)
    c0 = rng.random((nv, nv)) ** 3
    ux, uy = 0.7, -0.4
    dx, dt, tau = 0.1, 0.05, 3.0
    dv = s * dx / dt
    kappa = 0.02 * dv * dv / dt
    dts = dt / nsub
    c1, Fx, Fy = C.collide_site(c0, ux, uy, dts / (dv * tau), dts / tau,
                                kappa * dts / dv ** 2, nsub,
                                scheme == "koren")
    want = oracle.step(c0.reshape(nv * nv, 1, 1),
                       np.array([ux, uy]).reshape(1, 2, 1, 1), dim=2, dx=dx,
                       tau_p=tau, kappa=kappa, dt=dt, nsteps=1, scheme=scheme,
                       s=s, nsub=nsub).reshape(nv, nv)
    assert np.abs(c1 - want).max() <= 1e-14 * np.abs(want).max()
    div = (Fx[:, 1:] - Fx[:, :-1]) + (Fy[1:, :] - Fy[:-1, :])
    assert np.abs(c0 - div - c1).max() <= 1e-14 * np.abs(c0).max()
    assert not Fx[:, 0].any() and not Fx[:, -1].any()
    assert not Fy[0, :].any() and not Fy[-1, :].any()


def test_natural_coarse_fluxes_carry_the_restricted_divergence():
    """div_c G = R div F for any fine face fluxes (outer faces closed), and a
    single fine flux phi through fine face 4k-1 or 4k-2 shows up as phi/8
    through coarse face k (and 0 through the faces inside a coarse cell)."""
    rng = np.random.default_rng(5)
    nvf, nvc = 65, 17
    Fx = rng.standard_normal((nvf, nvf + 1))
    Fy = rng.standard_normal((nvf + 1, nvf))
    Fx[:, 0] = Fx[:, -1] = 0.0
    Fy[0, :] = Fy[-1, :] = 0.0
    Gx, Gy = C.natural_coarse_fluxes(Fx, Fy)
    divf = (Fx[:, 1:] - Fx[:, :-1]) + (Fy[1:, :] - Fy[:-1, :])
    divc = (Gx[:, 1:] - Gx[:, :-1]) + (Gy[1:, :] - Gy[:-1, :])
    Rdiv = C.restrict(divf.reshape(-1, 1), 2).reshape(nvc, nvc)
    assert np.allclose(divc, Rdiv, rtol=0, atol=1e-13)
    # 1D reading of the same map: one fine flux at a time, fine row 8 (a
    # coarse-centred row, restriction weight 1/4 across the other axis)
    for m, want in [(4 * 3 - 1, 1 / 8), (4 * 3 - 2, 1 / 8), (4 * 3, 0.0),
                    (4 * 3 + 1, 0.0)]:
        Fx = np.zeros((nvf, nvf + 1))
        Fx[8, m] = 1.0
        Gx, _ = C.natural_coarse_fluxes(Fx, np.zeros((nvf + 1, nvf)))
        k = 3
        assert Gx[2, k] == pytest.approx(want / 4.0)


def test_natural_targets_close_the_coarse_step():
    """pred - div T = R (fine collision of g): the targets map the coarse
    collision of the restricted state onto the restricted fine collision."""
    rng = np.random.default_rng(9)
    g = rng.random(65 * 65) ** 4
    dt, tau, kappa, dvf = 0.3, 4 * math.pi, 1e-4, 3.0 / 32
    fine = dict(alpha_scale=(dt / 3) / (dvf * tau), beta=(dt / 3) / tau,
                D=kappa * (dt / 3) / dvf ** 2, nsub=3, koren=True)
    dvc = 4 * dvf
    coarse = dict(alpha_scale=dt / (dvc * tau), beta=dt / tau,
                  D=kappa * dt / dvc ** 2, nsub=1, koren=True)
    T, pred, true = C.natural_targets(g, 0.6, -0.8, fine, coarse)
    D = C.divergence_matrix(17)
    assert np.abs(pred.reshape(-1) - D @ T - true.reshape(-1)).max() <= \
        1e-15 * np.abs(true).max() * 100
