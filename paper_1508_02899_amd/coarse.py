"""Coarse velocity lattice with the learned face-flux correction: training
data from fine runs, training and a side-by-side comparison.

The coarse lattice keeps dx and dt and uses every 4th fine velocity
(stride 4), so its streaming stays an exact integer shift (Sec. 2).  The
correction network adds face fluxes in velocity space once per stream step;
it is trained a priori: for fine states f_n, f_{n+1} and the restriction R,
the targets are the minimum-norm face fluxes that map the plain coarse step
C(R f_n) onto R f_{n+1}.

Everything here only orchestrates library calls (restriction, steps,
sample extraction, training, moments, density statistics); all arithmetic
runs in the GPU kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

from .lattice import Lattice, LatticeSpec, Mlp, restrict


def coarse_spec(fine: LatticeSpec, nsub: int = 1) -> LatticeSpec:
    """The stride-4 coarse lattice of a fine lattice (same sites, dx)."""
    if (fine.nv - 1) % 4:
        raise ValueError("fine nv must be 4 (nv_c - 1) + 1")
    return replace(fine, nv=(fine.nv - 1) // 4 + 1, vstride=4 * fine.vstride,
                   nsub=nsub)


def nsub_for(spec: LatticeSpec, u, tau_p: float, kappa: float, dt: float,
             bound: float | None = None) -> int:
    """Smallest number of collision sub-steps that keeps the drift CFL of
    Eq. 3 within the scheme's bound (1/2 Koren, 1 upwind; 0.9 of it here)
    and the diffusion number of Eq. 4 below 1/2, for the flow slices u."""
    if bound is None:
        bound = 0.45 if spec.scheme == "koren" else 0.9
    lat = Lattice(replace(spec, nsub=1))
    cfl, dnum = lat.stability(u, tau_p, kappa, dt)
    lat.close()
    return max(1, math.ceil(cfl / bound), math.ceil(dnum / 0.45))


def collect_samples(fine: Lattice, coarse: Lattice, mlp: Mlp, f_fine, flow,
                    *, steps: int, dt: float, tau_p: float, kappa: float,
                    St: float, sites_per_step: int, seed: int = 0,
                    first_step: int = 0, rel_eps: float = 1e-3,
                    collision_only: bool = True, targets: str = "minnorm"):
    """Advance the fine state ``steps`` steps (in place) and return the
    training samples (X, t, w) of ``sites_per_step`` random sites per step.
    ``flow(n)`` gives the flow slice [1, dim, ny, nx] of step n; the coarse
    lattice must have no network attached.  Faces with stencil mass below
    rel_eps x site mass carry no weight.

    collision_only: the targets compare the two collision parts on the same
    streamed state, R C_f (S_f f_n) against C_c (R S_f f_n), which leaves
    out the (velocity-space unrepresentable) difference between fine and
    coarse streaming; otherwise the whole steps, R f_{n+1} against
    C(R f_n).

    targets: "minnorm" (default): the least-norm face fluxes of the
    residual; "natural" (collision_only only): the coarse face fluxes
    implied by the fine collision's own face fluxes under the restriction,
    minus the coarse collision's fluxes.  Both have the same divergence;
    the natural ones are face-local and fit far better (about 70 % of
    their weighted variance explained against 31 %), but the coarse runs
    corrected by a network trained on them drift further from the fine
    state (128^2, St = 2: variance error 25 % against 19 %)."""
    if targets not in ("natural", "minnorm"):
        raise ValueError("targets: 'natural' or 'minnorm'")
    if targets == "natural" and not collision_only:
        raise ValueError("natural targets compare the collision parts")
    torch = _torch()
    dim = fine.spec.dim
    nsites = fine.spec.nx * (fine.spec.ny if dim == 2 else 1)
    gen = torch.Generator(device=f_fine.device)
    gen.manual_seed(seed)
    streamer = Lattice(replace(fine.spec, nsub=1)) if collision_only else None
    Xs, ts, ws = [], [], []
    for n in range(first_step, first_step + steps):
        u = flow(n)
        if collision_only and targets == "natural":
            streamer.step(f_fine, u, math.inf, 0.0, dt, 1)  # S_f f_n
            fc = restrict(f_fine, dim)                      # R S_f f_n
            coarse.collide(fc, u, tau_p, kappa, dt, 1)      # C_c(R S_f f_n)
            sites = torch.randint(0, nsites, (sites_per_step,), generator=gen,
                                  device=f_fine.device, dtype=torch.int32)
            X, t, w = mlp.samples_natural(fine, coarse, dt, tau_p, kappa, St,
                                          f_fine, fc, u, sites, rel_eps)
            fine.collide(f_fine, u, tau_p, kappa, dt, 1)    # f_{n+1}
            Xs.append(X)
            ts.append(t)
            ws.append(w)
            continue
        if collision_only:
            streamer.step(f_fine, u, math.inf, 0.0, dt, 1)  # S_f f_n
            fc = restrict(f_fine, dim)                      # R S_f f_n
            fine.collide(f_fine, u, tau_p, kappa, dt, 1)    # f_{n+1}
            ft = restrict(f_fine, dim)                      # R f_{n+1}
            coarse.collide(fc, u, tau_p, kappa, dt, 1)      # C_c(R S_f f_n)
        else:
            fc = restrict(f_fine, dim)                      # R f_n
            fine.step(f_fine, u, tau_p, kappa, dt, 1)       # f_{n+1}
            ft = restrict(f_fine, dim)                      # R f_{n+1}
            coarse.step(fc, u, tau_p, kappa, dt, 1)         # C(R f_n)
        sites = torch.randint(0, nsites, (sites_per_step,), generator=gen,
                              device=f_fine.device, dtype=torch.int32)
        X, t, w = mlp.samples(coarse, dt, tau_p, St, fc, ft, u, sites,
                              rel_eps)
        Xs.append(X)
        ts.append(t)
        ws.append(w)
    fine.sync()
    coarse.sync()
    if streamer is not None:
        streamer.sync()
        streamer.close()
    # shuffled, so that the consecutive training windows mix steps and sites
    X, t, w = torch.cat(Xs), torch.cat(ts), torch.cat(ws)
    perm = torch.randperm(t.numel(), generator=gen, device=t.device)
    return X[perm].contiguous(), t[perm].contiguous(), w[perm].contiguous()


def initial_params(seed: int = 0, out_scale: float = 0.01):
    """Random starting weights for the correction network (Glorot-style
    normal layers, a small output layer so that the initial correction is
    close to zero), packed as W1[8][64], b1, W2[64][64], b2, w3, b3."""
    import numpy as np
    rng = np.random.default_rng(seed)
    nf, nh = 8, 64
    parts = [rng.standard_normal(nf * nh) / math.sqrt(nf), np.zeros(nh),
             rng.standard_normal(nh * nh) / math.sqrt(nh), np.zeros(nh),
             out_scale * rng.standard_normal(nh) / math.sqrt(nh), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Track:
    """Time series of the observables of one run."""
    steps: list = field(default_factory=list)
    variance: list = field(default_factory=list)
    rho_r2: list = field(default_factory=list)  # one array of levels each


def observe(lat: Lattice, f, dt: float, levels: int, track: Track, n: int):
    m = lat.moments(f, dt)
    rho = lat.density(f, dt)
    track.steps.append(n)
    track.variance.append(m["variance"])
    track.rho_r2.append(lat.rho_r2(rho, levels))


def compare(fine: Lattice, coarse_runs: dict, f0_fine, flow, *, steps: int,
            dt: float, tau_p: float, kappa: float, levels: int, every: int):
    """Run the fine lattice and each coarse lattice of ``coarse_runs``
    (name -> Lattice, with or without a network attached) from the same
    initial state (restricted for the coarse ones) under the same flow;
    record variance and <rho_r^2> every ``every`` steps.  The track
    "fine_R" holds the restricted fine state seen on the coarse lattice
    (what a coarse run can represent at best)."""
    dim = fine.spec.dim
    f = f0_fine.clone()
    states = {k: restrict(f0_fine, dim) for k in coarse_runs}
    tracks = {"fine": Track(), "fine_R": Track(),
              **{k: Track() for k in coarse_runs}}
    any_coarse = next(iter(coarse_runs.values()))
    for n in range(1, steps + 1):
        u = flow(n - 1)
        fine.step(f, u, tau_p, kappa, dt, 1)
        for k, lat in coarse_runs.items():
            lat.step(states[k], u, tau_p, kappa, dt, 1)
        if n % every == 0:
            observe(fine, f, dt, levels, tracks["fine"], n)
            observe(any_coarse, restrict(f, dim), dt, levels,
                    tracks["fine_R"], n)
            for k, lat in coarse_runs.items():
                observe(lat, states[k], dt, levels, tracks[k], n)
    return tracks, f, states


def calibrate_output_scale(fine: Lattice, coarse_spec: LatticeSpec, mlp: Mlp,
                           St: float, f0_fine, flow, *, steps: int, dt: float,
                           tau_p: float, kappa: float, line_eps: float = 1e-3,
                           scales=(1.0, 1.25, 1.5, 2.0, 2.5, 3.0),
                           from_step: int = 50, every: int = 25):
    """A-posteriori calibration of the trained network's output scale: the
    coarse lattice runs once per candidate scale c (correction c * G; c is
    folded into the output layer w3, b3) beside the fine lattice, from
    f0_fine under ``flow`` (the training flow, or any flow other than the
    one the model is evaluated on, within the lattices' CFL bounds), and
    the scale with the smallest mean velocity-variance error against the
    restricted fine state (steps >= from_step) is written into ``mlp``.
    Returns (best scale, {scale: error})."""
    import numpy as np
    P0 = np.asarray(mlp.get_params(), dtype=np.float32)
    nets, runs = {}, {}
    for c in scales:
        m = Mlp()
        P = P0.copy()
        P[-65:] *= c          # w3[64] and b3, the last 65 parameters
        m.set_params(P)
        lat = Lattice(coarse_spec)
        m.attach(lat, St, line_eps)
        nets[c], runs[f"s{c}"] = m, lat
    levels = 1
    tracks, _, _ = compare(fine, runs, f0_fine, flow, steps=steps, dt=dt,
                           tau_p=tau_p, kappa=kappa, levels=levels,
                           every=every)
    err = errors({k: v for k, v in tracks.items() if k != "fine"}, "fine_R",
                 coarse_spec.dx, from_step=from_step)
    scores = {c: err[f"s{c}"]["variance"] for c in scales}
    best = min(scores, key=scores.get)
    P = P0.copy()
    P[-65:] *= best
    mlp.set_params(P)
    for c in scales:
        runs[f"s{c}"].close()
        nets[c].close()
    return best, scores


def errors(tracks: dict, ref: str, dx: float, from_step: int = 0):
    """Per run: mean relative error of the velocity variance and the mean
    distance-averaged relative error of <rho_r^2> against the reference
    run, over the recorded steps >= from_step (weights r^2 on the tiling
    scales r = 2^k dx, the discrete form of the r dr average of Sec. 4.2.1).
    """
    import numpy as np
    from .lattice import rho_r2_error
    R = tracks[ref]
    sel = [i for i, s in enumerate(R.steps) if s >= from_step]
    out = {}
    for k, T in tracks.items():
        if k == ref:
            continue
        ev = [abs(T.variance[i] - R.variance[i]) / R.variance[i] for i in sel]
        er = [rho_r2_error(T.rho_r2[i], R.rho_r2[i], dx) for i in sel]
        out[k] = {"variance": float(np.mean(ev)), "rho_r2": float(np.mean(er))}
    return out


def _torch():
    import torch
    return torch
