"""GPU checks of the coarse lattice and its learned face-flux correction
against the FP64 oracle (oracle/coarse.py): restriction, the matrix-core
network forward pass, gradients, Adam, training samples, the fused
correction pass."""
import math

import numpy as np
import pytest

from helpers import rel_l2, say

pytestmark = pytest.mark.gpu


def _params(rng, scale=1.0):
    from oracle import coarse as C
    P = C.init_params(rng, scale=scale)
    P["b1"] = rng.standard_normal(C.NH) * 0.2
    P["b2"] = rng.standard_normal(C.NH) * 0.2
    P["b3"] = np.array(0.1)
    return P


def _pack(P):
    return np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"],
                           P["w3"], np.atleast_1d(P["b3"])]).astype(np.float32)


def _unpack(a):
    a = np.asarray(a, dtype=np.float64)
    o = 0
    out = {}
    for k, shape in [("W1", (8, 64)), ("b1", (64,)), ("W2", (64, 64)),
                     ("b2", (64,)), ("w3", (64,)), ("b3", ())]:
        n = int(np.prod(shape)) if shape else 1
        out[k] = a[o:o + n].reshape(shape) if shape else np.array(a[o])
        o += n
    return out


@pytest.mark.parametrize("dim,nvf", [(1, 33), (2, 65), (2, 17)])
def test_restrict_matches_oracle(dim, nvf):
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import restrict
    rng = np.random.default_rng(31)
    shape = (nvf, 37) if dim == 1 else (nvf * nvf, 5, 7)
    f = rng.random(shape).astype(np.float32)
    got = restrict(torch.from_numpy(f).cuda(), dim).cpu().numpy()
    want = C.restrict(f.astype(np.float64), dim)
    assert rel_l2(got, want) < 1e-6


def test_mlp_forward_matrix_cores_match_oracle():
    """bf16 weights and layer inputs, FP32 accumulation on the matrix cores
    vs the FP64 oracle with the same bf16 roundings."""
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Mlp
    rng = np.random.default_rng(32)
    P = _params(rng, 1.5)
    X = rng.standard_normal((1000, 8)).astype(np.float32)
    X[:, 7] = 0.0
    m = Mlp()
    m.set_params(_pack(P))
    y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = C.forward(_unpack(_pack(P)), X.astype(np.float64))
    err = rel_l2(y, want)
    say(f"  forward rel L2 {err:.2e}, max abs {np.abs(y - want).max():.2e}")
    assert err < 5e-3
    m.close()


def test_mlp_gradient_matches_oracle():
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Mlp
    rng = np.random.default_rng(33)
    P = _params(rng, 1.2)
    n = 3000
    X = rng.standard_normal((n, 8)).astype(np.float32)
    X[:, 7] = 0.0
    t = rng.standard_normal(n).astype(np.float32)
    w = rng.random(n).astype(np.float32)
    m = Mlp()
    m.set_params(_pack(P))
    loss, g = m.grad(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(),
                     torch.from_numpy(w).cuda())
    L, go = C.loss_and_grads(_unpack(_pack(P)), X.astype(np.float64),
                             t.astype(np.float64), w.astype(np.float64))
    gw = _pack(go)
    err = rel_l2(g.cpu().numpy(), gw)
    say(f"  loss {loss:.6f} vs {L:.6f}; gradient rel L2 {err:.2e}")
    assert loss == pytest.approx(L, rel=1e-4)
    assert err < 1e-4
    m.close()


def test_adam_training_reduces_loss_on_teacher_targets():
    """Targets from a random 'teacher' network: Adam on the GPU must cut the
    loss of a differently initialised student by 10x."""
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Mlp
    rng = np.random.default_rng(34)
    teacher = _params(rng, 1.0)
    n = 16384
    X = rng.standard_normal((n, 8)).astype(np.float32)
    X[:, 7] = 0.0
    t, _ = C.forward(_unpack(_pack(teacher)), X.astype(np.float64))
    w = np.ones(n, dtype=np.float32)
    m = Mlp()
    m.set_params(_pack(_params(np.random.default_rng(35), 0.5)))
    Xd, td, wd = (torch.from_numpy(a).cuda() for a in
                  (X, t.astype(np.float32), w))
    l0, _ = m.grad(Xd, td, wd)
    m.train(Xd, td, wd, batch=1024, steps=600, lr=3e-3)
    l1, _ = m.grad(Xd, td, wd)
    say(f"  teacher loss {l0:.4e} -> {l1:.4e}")
    assert l1 < 0.1 * l0
    m.close()


def test_adam_step_matches_oracle():
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Mlp
    rng = np.random.default_rng(36)
    P = _params(rng, 1.0)
    n = 512
    X = rng.standard_normal((n, 8)).astype(np.float32)
    X[:, 7] = 0
    t = rng.standard_normal(n).astype(np.float32)
    w = np.ones(n, dtype=np.float32)
    m = Mlp()
    m.set_params(_pack(P))
    m.train(*(torch.from_numpy(a).cuda() for a in (X, t, w)), batch=n,
            steps=3, lr=1e-3)
    got = m.get_params()
    Po = _unpack(_pack(P))
    st = {}
    for _ in range(3):
        _, g = C.loss_and_grads(Po, X.astype(np.float64), t.astype(np.float64),
                                w.astype(np.float64))
        C.adam(Po, g, st, lr=1e-3)
    # Adam's first steps are close to sign steps: compare the updates
    d_gpu = got - _pack(P)
    d_ora = _pack(Po) - _pack(P)
    err = rel_l2(d_gpu, d_ora)
    say(f"  3 Adam steps: update rel L2 {err:.2e}")
    assert err < 2e-2
    m.close()


def _coarse_case(rng, n=6, ny=None):
    """A coarse 17^2 state at n x ny sites (ny = n by default) and a 'true'
    state of equal mass."""
    nv = 17
    ny = n if ny is None else ny
    f_pred = (rng.random((nv * nv, ny, n)) ** 3).astype(np.float32)
    f_true = (f_pred * (1 + 0.1 * rng.standard_normal(f_pred.shape))).astype(np.float32)
    f_true = np.abs(f_true)
    s_p = f_pred.sum(axis=0, dtype=np.float64)
    s_t = f_true.sum(axis=0, dtype=np.float64)
    f_true = (f_true * (s_p / s_t)[None]).astype(np.float32)
    u = (0.8 * np.tanh(rng.standard_normal((1, 2, ny, n)))).astype(np.float32)
    return f_pred, f_true, u


def test_flux_samples_match_oracle():
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Lattice, LatticeSpec, Mlp
    rng = np.random.default_rng(37)
    n, nv = 6, 17
    f_pred, f_true, u = _coarse_case(rng, n)
    dx, dt, tau_p, St = 2 * math.pi / n, 0.05, 1.3, 2.0
    lat = Lattice(LatticeSpec(dim=2, nx=n, ny=n, nv=nv, dx=dx, vstride=4))
    m = Mlp()
    sites = np.array([0, 7, 35], dtype=np.int32)
    X, t, w = m.samples(lat, dt, tau_p, St, torch.from_numpy(f_pred).cuda(),
                        torch.from_numpy(f_true).cuda(), torch.from_numpy(u).cuda(),
                        torch.from_numpy(sites).cuda())
    X, t, w = X.cpu().numpy(), t.cpu().numpy(), w.cpu().numpy()
    dv = 4 * dx / dt
    for q, s in enumerate(sites):
        y, x = divmod(int(s), n)
        fp = f_pred[:, y, x].astype(np.float64)
        ft = f_true[:, y, x].astype(np.float64)
        Xo, ms, sg = C.face_features(fp, nv, float(u[0, 0, y, x]),
                                     float(u[0, 1, y, x]), dv, dt, tau_p, St)
        Gx, Gy = C.minnorm_fluxes(ft - fp, nv)
        G = np.concatenate([Gx.ravel(), Gy.ravel()])
        to = np.where(ms > 0, sg * G / np.where(ms > 0, ms, 1), 0)
        sl = slice(q * 544, (q + 1) * 544)
        np.testing.assert_allclose(X[sl], Xo, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(w[sl], ms, rtol=1e-5)
        err = rel_l2(t[sl], to)
        say(f"  site {s}: target rel L2 {err:.2e}")
        assert err < 1e-4
    m.close()
    lat.close()


@pytest.mark.parametrize("scheme,nsf,nsc", [("koren", 3, 1),
                                            ("upwind", 2, 2)])
def test_natural_flux_samples_match_oracle(scheme, nsf, nsc):
    """Natural flux targets: the fine collision of each listed site redone
    with its face fluxes recorded, restricted to coarse faces, minus the
    coarse collision's fluxes -- against the oracle's FP64 version from the
    same streamed fine state; features and weights from the coarse
    collision the library computed."""
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Lattice, LatticeSpec, Mlp, restrict
    rng = np.random.default_rng(41 + nsf)
    n, nvf, nvc = 6, 65, 17
    L = 2 * math.pi
    dx = L / n
    dvf = 3.0 / 32
    dt = dx / dvf
    tau_p, kappa, St = 400.0, 2e-4, 2.0  # coarse CFL ~0.3 at nsub 1
    g = (rng.random((nvf * nvf, n, n)) ** 4).astype(np.float32)
    u = (0.8 * np.tanh(rng.standard_normal((1, 2, n, n)))).astype(np.float32)
    fs = LatticeSpec(dim=2, nx=n, ny=n, nv=nvf, dx=dx, scheme=scheme,
                     nsub=nsf)
    cs = LatticeSpec(dim=2, nx=n, ny=n, nv=nvc, dx=dx, vstride=4,
                     scheme=scheme, nsub=nsc)
    fine, coarse, m = Lattice(fs), Lattice(cs), Mlp()
    gd = torch.from_numpy(g).cuda()
    ud = torch.from_numpy(u).cuda()
    fc = restrict(gd, 2)
    coarse.collide(fc, ud, tau_p, kappa, dt, 1)
    sites = np.array([0, 9, 35], dtype=np.int32)
    X, t, w = m.samples_natural(fine, coarse, dt, tau_p, kappa, St, gd, fc,
                                ud, torch.from_numpy(sites).cuda())
    X, t, w = X.cpu().numpy(), t.cpu().numpy(), w.cpu().numpy()
    pred_gpu = fc.cpu().numpy()
    dvc = 4 * dvf
    koren = scheme == "koren"
    fine_c = dict(alpha_scale=(dt / nsf) / (dvf * tau_p), beta=(dt / nsf) / tau_p,
                  D=kappa * (dt / nsf) / dvf ** 2, nsub=nsf, koren=koren)
    coarse_c = dict(alpha_scale=(dt / nsc) / (dvc * tau_p),
                    beta=(dt / nsc) / tau_p, D=kappa * (dt / nsc) / dvc ** 2,
                    nsub=nsc, koren=koren)
    for q, s_ in enumerate(sites):
        y, x = divmod(int(s_), n)
        ux, uy = float(u[0, 0, y, x]), float(u[0, 1, y, x])
        T, pred, _ = C.natural_targets(g[:, y, x], ux, uy, fine_c, coarse_c)
        # the oracle's coarse collision agrees with the library's
        pg = pred_gpu[:, y, x].astype(np.float64)
        assert rel_l2(pg, pred.reshape(-1)) < 1e-5
        Xo, ms, sg = C.face_features(pg, nvc, ux, uy, dvc, dt, tau_p, St)
        use = ms > 0
        to = np.where(use, sg * T / np.where(use, ms, 1), 0)
        sl = slice(q * 544, (q + 1) * 544)
        np.testing.assert_allclose(X[sl], Xo, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(w[sl], ms, rtol=1e-5)
        err = np.sqrt(np.sum(ms * (t[sl] - to) ** 2) / np.sum(ms * to ** 2))
        say(f"  site {s_}: mass-weighted target rel L2 {err:.2e}")
        assert err < 1e-3
    m.close()
    fine.close()
    coarse.close()


@pytest.mark.parametrize("n,ny", [(8, 8), (12, 7)])
def test_correction_pass_matches_oracle_and_conserves_mass(n, ny):
    """A coarse 2D step with the network attached vs plain step + the
    oracle's correction of every site.  12 x 7 = 84 sites: the correction
    kernel's last tile of 32 sites is partly empty."""
    import torch
    from oracle import coarse as C
    from paper_1508_02899_amd import Lattice, LatticeSpec, Mlp
    rng = np.random.default_rng(38)
    nv = 17
    say(f"  correction pass, {n} x {ny} sites")
    f0, _, u = _coarse_case(rng, n, ny)
    dx = 2 * math.pi / n
    dt, tau_p, St, kappa, eps = 0.05, 40.0, 1.5, 0.0, 1e-3
    spec = LatticeSpec(dim=2, nx=n, ny=ny, nv=nv, dx=dx, vstride=4)
    P = _params(rng, 0.3)
    P["b3"] = np.array(0.05)
    plain = Lattice(spec)
    fa = torch.from_numpy(f0.copy()).cuda()
    plain.step(fa, torch.from_numpy(u).cuda(), tau_p, kappa, dt, 1)
    plain.sync()
    mid = fa.cpu().numpy().astype(np.float64)
    corr = Lattice(spec)
    m = Mlp()
    m.set_params(_pack(P))
    m.attach(corr, St, eps)
    fb = torch.from_numpy(f0.copy()).cuda()
    corr.step(fb, torch.from_numpy(u).cuda(), tau_p, kappa, dt, 1)
    corr.sync()
    got = fb.cpu().numpy()
    dv = 4 * dx / dt
    Pq = _unpack(_pack(P))
    want = np.empty_like(mid)
    for y in range(ny):
        for x in range(n):
            c = mid[:, y, x]
            Xo, ms, sg = C.face_features(c, nv, float(u[0, 0, y, x]),
                                         float(u[0, 1, y, x]), dv, dt, tau_p, St)
            yo, _ = C.forward(Pq, Xo)
            want[:, y, x] = C.corrected_site(c, nv, yo, ms, sg, line_eps=eps)
    err = rel_l2(got, want)
    corr_size = rel_l2(want, mid)
    say(f"  corrected state rel L2 {err:.2e} (correction size {corr_size:.2e})")
    assert err < 2e-3 * max(1.0, corr_size / 1e-2)
    assert err < 0.1 * corr_size
    assert abs(got.sum(dtype=np.float64) - mid.sum()) / mid.sum() < 1e-6
    assert got.min() >= 0.0
    m.close()
    plain.close()
    corr.close()
