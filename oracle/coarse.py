"""FP64 oracle of the coarse-velocity-lattice form -- TEST INFRASTRUCTURE ONLY.

Only tests/ (and the benchmark's CPU baseline) may import this module; the
GPU library never does.  Plain numpy in double precision.

Coarse lattice (a reading of Sec. 2, dx = dv dt): the coarse velocity
lattice keeps dx and dt and uses every 4th fine velocity (stride 4), so its
streaming is still an exact integer shift.  Fine nv_f = 4 (nv_c - 1) + 1.

* restrict: mass-conservative fine -> coarse map.  Coarse cell J spans
  fine centres 4J-2 .. 4J+2; fine cells 4J-1, 4J, 4J+1 lie inside, fine
  cells 4J+-2 are split half/half with the neighbour.  In 2D the weights
  are the tensor product.
* min-norm face fluxes: the face fluxes G (x-faces and y-faces of the coarse
  velocity square, outer faces closed) whose conservative update
  f_J -= div G reproduces a given zero-sum residual r, with the smallest
  sum of squares -- solved here by least squares on the explicit
  divergence matrix.
* the flux-correction MLP: x (8) -> 64 -> 64 -> 1, GELU (tanh form,
  Hendrycks & Gimpel 2016: 0.5 z (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3)))),
  forward and hand-derived backward, weighted squared loss, Adam.
* natural flux targets: the collision of a site with its face fluxes
  recorded, and the coarse fluxes those imply under the restriction
  (div_c G = R div F), minus the coarse collision's own fluxes.
* face features and the corrected coarse update.
"""
from __future__ import annotations

import math

import numpy as np

NF = 8      # input features (7 used + 1 zero pad)
NH = 64     # hidden width


# ---------------------------------------------------------------------------
# restriction
def restrict_weights(nv_f: int) -> np.ndarray:
    """R[J, j]: fraction of fine cell j's mass that lands in coarse cell J."""
    assert (nv_f - 1) % 4 == 0
    nv_c = (nv_f - 1) // 4 + 1
    R = np.zeros((nv_c, nv_f))
    for j in range(nv_f):
        J, o = divmod(j, 4)
        if o == 0:
            R[J, j] = 1.0
        elif o == 1:
            R[J, j] = 1.0
        elif o == 3:
            R[J + 1, j] = 1.0
        else:  # o == 2: exactly between coarse centres J and J+1
            R[J, j] = 0.5
            R[J + 1, j] = 0.5
    return R


def restrict(f_fine: np.ndarray, dim: int) -> np.ndarray:
    """Coarse state (same sites) of a fine state; values are densities, the
    coarse cell being 4x (per axis) wider: f_c = (R f_f) / 4^dim."""
    f = np.asarray(f_fine, dtype=np.float64)
    if dim == 1:
        nv_f = f.shape[0]
        R = restrict_weights(nv_f)
        return (R @ f.reshape(nv_f, -1)).reshape((R.shape[0],) + f.shape[1:]) / 4.0
    nvv = f.shape[0]
    nv_f = int(round(nvv ** 0.5))
    R = restrict_weights(nv_f)
    nv_c = R.shape[0]
    g = f.reshape(nv_f, nv_f, -1)                 # [jy, jx, site]
    g = np.einsum("Yy,Xx,yxs->YXs", R, R, g)
    return g.reshape((nv_c * nv_c,) + f.shape[1:]) / 16.0


# ---------------------------------------------------------------------------
# min-norm face fluxes
def divergence_matrix(n: int) -> np.ndarray:
    """D (n^2 x 2 n (n-1)): (D G)_J = G^x_{Jy,Jx+1} - G^x_{Jy,Jx}
    + G^y_{Jy+1,Jx} - G^y_{Jy,Jx}, outer faces zero.  Unknown order: x-faces
    (Jy, k) k = 1..n-1, then y-faces (k, Jx)."""
    nfx = n * (n - 1)
    D = np.zeros((n * n, 2 * nfx))
    for jy in range(n):
        for jx in range(n):
            J = jy * n + jx
            if jx + 1 <= n - 1:
                D[J, jy * (n - 1) + jx] += 1.0          # face jx+1 of row jy
            if jx >= 1:
                D[J, jy * (n - 1) + jx - 1] -= 1.0      # face jx of row jy
            if jy + 1 <= n - 1:
                D[J, nfx + jy * n + jx] += 1.0          # face jy+1 of col jx
            if jy >= 1:
                D[J, nfx + (jy - 1) * n + jx] -= 1.0    # face jy of col jx
    return D


def minnorm_fluxes(r: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """G minimising |G|^2 subject to -div G = r for each site (r[n*n, sites]).
    Returns (Gx[n, n-1 (faces 1..n-1), sites], Gy[n-1 (faces 1..n-1), n, sites])."""
    D = divergence_matrix(n)
    r = np.asarray(r, dtype=np.float64).reshape(n * n, -1)
    G, *_ = np.linalg.lstsq(D, -r, rcond=None)
    nfx = n * (n - 1)
    return G[:nfx].reshape(n, n - 1, -1), G[nfx:].reshape(n - 1, n, -1)


# ---------------------------------------------------------------------------
# collision of one site with its face fluxes, and the natural coarse fluxes
def _limiter(dp, dm):
    """Koren limiter in the division-free form: dp > 0: max(0, min(dp,
    dp/3 + dm/6, dm)); dp < 0: min(0, max(...)); dp = 0: 0."""
    t = dp / 3.0 + dm / 6.0
    up = np.maximum(0.0, np.minimum(np.minimum(dp, t), dm))
    dn = np.minimum(0.0, np.maximum(np.maximum(dp, t), dm))
    return np.where(dp > 0, up, np.where(dp < 0, dn, 0.0))


def _drift_faces(c, nu, koren):
    """Split drift fluxes of lines c[..., n] with cell-centred nu[n] (Eq. 5
    force in cells per sub-step): F[..., k] through face k (cells k-1 | k),
    k = 0..n, the outer faces closed, cells outside the line empty."""
    n = c.shape[-1]
    pad = [(0, 0)] * (c.ndim - 1) + [(2, 2)]
    gp = np.pad(np.maximum(nu, 0.0) * c, pad)   # gp[i + 2] = g+ of cell i
    gm = np.pad(np.minimum(nu, 0.0) * c, pad)
    F = np.zeros(c.shape[:-1] + (n + 1,))
    for k in range(1, n):
        fp = gp[..., k + 1]                     # g+ of cell k-1
        fm = gm[..., k + 2]                     # g- of cell k
        if koren:
            fp = fp + _limiter(gp[..., k + 2] - gp[..., k + 1],
                               gp[..., k + 1] - gp[..., k])
            fm = fm + _limiter(gm[..., k + 1] - gm[..., k + 2],
                               gm[..., k + 2] - gm[..., k + 3])
        F[..., k] = fp + fm
    return F


def _diffusion_faces(c, D):
    """Diffusion fluxes D (c_{k-1} - c_k) through faces k = 1..n-1."""
    n = c.shape[-1]
    F = np.zeros(c.shape[:-1] + (n + 1,))
    F[..., 1:n] = D * (c[..., :-1] - c[..., 1:])
    return F


def collide_site(c, ux, uy, alpha_scale, beta, D, nsub, koren=True):
    """The collision part of one 2D time step at one site (Sec. 2: nsub x
    [drift along vx, drift along vy, diffusion along vx, along vy], the
    force at cell centres, nu_j = alpha_scale u - beta (j - h)), on its
    velocity square c[jy, jx].  Returns (c after, Fx[jy, 0..nv] summed over
    the sub-steps, Fy[0..nv, jx] summed): c_after = c - div F exactly."""
    c = np.asarray(c, dtype=np.float64).copy()
    nv = c.shape[0]
    h = (nv - 1) // 2
    j = np.arange(nv) - h
    nux = alpha_scale * ux - beta * j
    nuy = alpha_scale * uy - beta * j
    Fx = np.zeros((nv, nv + 1))
    Fy = np.zeros((nv + 1, nv))
    for _ in range(nsub):
        F = _drift_faces(c, nux, koren)                 # rows: along vx
        c -= F[:, 1:] - F[:, :-1]
        Fx += F
        F = _drift_faces(c.T, nuy, koren).T             # columns: along vy
        c -= F[1:, :] - F[:-1, :]
        Fy += F
        F = _diffusion_faces(c, D)
        c -= F[:, 1:] - F[:, :-1]
        Fx += F
        F = _diffusion_faces(c.T, D).T
        c -= F[1:, :] - F[:-1, :]
        Fy += F
    return c, Fx, Fy


def natural_coarse_fluxes(Fx, Fy):
    """Coarse face fluxes G with div_c G = R (div F) for the stride-4
    restriction R (restrict_weights, densities / 4 per axis): coarse face k
    (coarse cells k-1 | k) collects the fine faces 4k-2 and 4k-1 on either
    side of the shared fine cell 4k-2, G_k = (F_{4k-2} + F_{4k-1}) / 8 per
    fine line, and the lines are combined with the restriction weights
    across the other axis.  Fx[jy, 0..nv_f], Fy[0..nv_f, jx] ->
    (Gx[Jy, 0..nv_c], Gy[0..nv_c, Jx])."""
    nv_f = Fx.shape[0]
    R = restrict_weights(nv_f) / 4.0
    nv_c = R.shape[0]
    k = np.arange(1, nv_c)
    ax = np.zeros((nv_f, nv_c + 1))
    ax[:, 1:nv_c] = (Fx[:, 4 * k - 2] + Fx[:, 4 * k - 1]) / 8.0
    Gx = R @ ax                                      # [Jy, faces]
    ay = np.zeros((nv_c + 1, nv_f))
    ay[1:nv_c, :] = (Fy[4 * k - 2, :] + Fy[4 * k - 1, :]) / 8.0
    Gy = ay @ R.T                                    # [faces, Jx]
    return Gx, Gy


def natural_targets(g_fine, ux, uy, fine, coarse):
    """Target face fluxes of one site from its streamed fine velocity square
    g_fine[nv_f*nv_f]: the natural coarse fluxes of the fine collision minus
    the coarse collision's own fluxes on R g.  fine / coarse: dicts with
    alpha_scale, beta, D, nsub, koren.  Returns (T in the face order of
    face_features / divergence_matrix, pred = coarse collision of R g,
    true = R (fine collision of g)); pred - div T = true."""
    nv_f = int(round(len(g_fine) ** 0.5))
    c = np.asarray(g_fine, dtype=np.float64).reshape(nv_f, nv_f)
    cf, Fx, Fy = collide_site(c, ux, uy, fine["alpha_scale"], fine["beta"],
                              fine["D"], fine["nsub"], fine["koren"])
    Gx, Gy = natural_coarse_fluxes(Fx, Fy)
    rg = restrict(c.reshape(-1, 1), 2).reshape(Gx.shape[0], -1)
    pred, Cx, Cy = collide_site(rg, ux, uy, coarse["alpha_scale"],
                                coarse["beta"], coarse["D"], coarse["nsub"],
                                coarse["koren"])
    nv = rg.shape[0]
    Tx, Ty = Gx - Cx, Gy - Cy
    T = np.concatenate([Tx[:, 1:nv].reshape(-1), Ty[1:nv, :].reshape(-1)])
    true = restrict(cf.reshape(-1, 1), 2).reshape(nv, nv)
    return T, pred, true


# ---------------------------------------------------------------------------
# MLP
def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(math.sqrt(2.0 / math.pi) * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    a = math.sqrt(2.0 / math.pi)
    t = np.tanh(a * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * a * (1.0 + 3 * 0.044715 * z * z)


def bf16(x):
    """Round to bfloat16 (round to nearest even), returned as float64."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, X, quantize=True):
    """X [N, 8] -> y [N] and the cache for backward.  With quantize, the
    weights and every layer input are rounded to bf16 (as on the GPU)."""
    W1, b1, W2, b2, w3, b3 = (params[k] for k in ("W1", "b1", "W2", "b2", "w3", "b3"))
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    X0 = q(X)
    z1 = X0 @ q(W1) + b1
    h1 = q(gelu(z1))
    z2 = h1 @ q(W2) + b2
    h2 = q(gelu(z2))
    y = h2 @ q(w3) + b3
    return y, (X0, z1, h1, z2, h2)


def loss_and_grads(params, X, t, w, quantize=True):
    """L = sum_i w_i (y_i - t_i)^2 / sum_i w_i and its gradients (the
    rounding to bf16 is passed straight through)."""
    y, (X0, z1, h1, z2, h2) = forward(params, X, quantize)
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W = float(np.sum(w))
    e = y - t
    L = float(np.sum(w * e * e) / W)
    dy = 2.0 * w * e / W                      # [N]
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array(np.sum(dy))
    dh2 = np.outer(dy, q(params["w3"]))
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ q(params["W2"]).T
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = X0.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return L, g


def init_params(rng, scale=1.0):
    return {
        "W1": rng.standard_normal((NF, NH)) * scale / math.sqrt(NF),
        "b1": np.zeros(NH),
        "W2": rng.standard_normal((NH, NH)) * scale / math.sqrt(NH),
        "b2": np.zeros(NH),
        "w3": rng.standard_normal(NH) * scale / math.sqrt(NH),
        "b3": np.zeros(()),
    }


def adam(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


# ---------------------------------------------------------------------------
# features and the corrected update (2D coarse lattice, one site at a time)
def face_features(fc, nv, ux, uy, dv, dt, tau_p, St):
    """For one site's coarse velocity square fc[nv*nv], the 8 features,
    stencil masses and orientation of every interior face.
    Returns X[2 nv (nv-1), 8], ms[...], sgn[...] in the face order of
    divergence_matrix (x-faces (Jy, k), then y-faces (k, Jx))."""
    h = (nv - 1) // 2
    c = np.asarray(fc, dtype=np.float64).reshape(nv, nv)  # [jy, jx]
    rows = []
    order = [(0, a, k) for a in range(nv) for k in range(1, nv)]      # x: (Jy, k)
    order += [(1, a, k) for k in range(1, nv) for a in range(nv)]     # y: (k, Jx)
    for axis, a, k in order:
        line = c[a, :] if axis == 0 else c[:, a]
        u = ux if axis == 0 else uy
        vface = (k - 0.5 - h) * dv
        nu = dt * (u - vface) / (tau_p * dv)
        if nu >= 0:
            idx, sg = [k - 3, k - 2, k - 1, k, k + 1], 1.0
        else:
            idx, sg = [k + 2, k + 1, k, k - 1, k - 2], -1.0
        st = np.array([line[i] if 0 <= i < nv else 0.0 for i in idx])
        ms = st.sum()
        feat = np.zeros(NF)
        if ms > 0:
            feat[:5] = st / ms
        feat[5] = abs(nu)
        feat[6] = math.log(St)
        rows.append((feat, ms, sg))
    X = np.array([r[0] for r in rows])
    ms = np.array([r[1] for r in rows])
    sg = np.array([r[2] for r in rows])
    return X, ms, sg


def corrected_site(fc, nv, y, ms, sg, line_eps=0.0):
    """Apply the face fluxes G = sg * ms * y, each limited to a quarter of
    its donor cell's mass, as the conservative update f -= div G.  Faces
    whose stencil holds less than line_eps of the site's mass (or none) get
    no correction: the faces the network is trained on are exactly the
    others (the training samples use the same rule)."""
    c = np.asarray(fc, dtype=np.float64).reshape(nv, nv).copy()
    M = c.sum()
    ms = np.asarray(ms, dtype=np.float64)
    use = (ms > 0) & (ms >= line_eps * M)
    G = np.where(use, sg * ms * np.asarray(y, dtype=np.float64), 0.0)
    nfx = nv * (nv - 1)
    Gx = G[:nfx].reshape(nv, nv - 1).copy()   # [jy, k-1]
    Gy = G[nfx:].reshape(nv - 1, nv).T.copy()  # -> [jx, k-1]
    Gx2 = np.zeros((nv, nv + 1))
    Gy2 = np.zeros((nv + 1, nv))
    for a in range(nv):
        for k in range(1, nv):
            gx = Gx[a, k - 1]
            donor = c[a, k - 1] if gx > 0 else c[a, k]
            Gx2[a, k] = np.clip(gx, -0.25 * donor, 0.25 * donor)
            gy = Gy[a, k - 1]
            donor = c[k - 1, a] if gy > 0 else c[k, a]
            Gy2[k, a] = np.clip(gy, -0.25 * donor, 0.25 * donor)
    c -= (Gx2[:, 1:] - Gx2[:, :-1]) + (Gy2[1:, :] - Gy2[:-1, :])
    return c.reshape(nv * nv)
