"""Pins of the oracle's field feedback (Sec. 3.2: the macro-particles' current on the grid, then
Maxwell's equations for E and B), against facts that do not come from the oracle's formulas:

- the continuity equation node by node for the charge density of the gather's own shape
  (cloud-in-cell), with the density written out here;
- the total current of a move, Q times the velocity;
- the out-of-plane current as the time average of the linearly interpolated shape product
  (quadrature here);
- the Yee scheme's vacuum plane waves, both polarisations, with the frequency of its discrete
  dispersion relation;
- Gauss's law: div E - rho keeps its value through a coupled run with emission and pairs;
- the plasma frequency of a cold electron plasma, omega_p^2 = kappa Q n, from the Lorentz force
  of code units and Gauss's law.

Each planted mistake a plausible bug would make (a sign, a half, an offset, a wrong cumulative
direction, the current's sign in Ampere's law, the charge normalisation) fails one of them."""
import math

import numpy as np
import pytest

import oracle

NX, NY, DX, DY = 12, 10, 0.3, 0.4
DT = 0.1


def _cfg(nx=NX, ny=NY, dx=DX, dy=DY, dt=DT, q=1.0, **kw):
    return oracle.RunConfig(field_kind=oracle.FIELD_GRID_FDTD, field=(q,), dt=dt, n_steps=kw.pop("n_steps", 1),
                            dims=2, grid=(nx, ny, dx, dy, 0.0, 0.0), **kw)


def _rho(Q, x, y, nx=NX, ny=NY, dx=DX, dy=DY):
    """Cloud-in-cell charge density of point charges Q at (x, y) on the nodes (i dx, j dy),
    periodic: each node gets Q (1 - |x/dx - i|)(1 - |y/dy - j|)/(dx dy) from a charge within a cell."""
    rho = np.zeros((ny, nx))
    for q, xx, yy in np.broadcast(Q, x, y):
        gx, gy = xx / dx, yy / dy
        i0, j0 = math.floor(gx), math.floor(gy)
        for a in (0, 1):
            for b in (0, 1):
                w = (1 - abs(gx - (i0 + a))) * (1 - abs(gy - (j0 + b)))
                rho[(j0 + b) % ny, (i0 + a) % nx] += q * w / (dx * dy)
    return rho


def _div(Jx, Jy, dx=DX, dy=DY):
    """Divergence at the nodes (i, j) of fields on the Ex / Ey nodes (i + 1/2, j) / (i, j + 1/2)."""
    return (Jx - np.roll(Jx, 1, axis=1)) / dx + (Jy - np.roll(Jy, 1, axis=0)) / dy


MOVES = [  # (x0, y0, x1, y1): inside a cell, across x, across y, across both, across the periodic edge
    (1.05, 1.30, 1.17, 1.33),
    (1.25, 1.30, 1.36, 1.22),
    (2.10, 1.18, 2.04, 1.25),
    (0.88, 2.39, 0.95, 2.43),
    (3.55, 3.95, 3.64, 4.07),
    (0.02, 0.05, -0.07, -0.08),
]


@pytest.mark.parametrize("move", MOVES)
def test_deposit_satisfies_continuity_node_by_node(move):
    x0, y0, x1, y1 = move
    Q = -1.7
    J = oracle.deposit(_cfg(), Q, x0, y0, x1, y1, 0.4)
    drho = _rho(Q, x1, y1) - _rho(Q, x0, y0)
    res = drho / DT + _div(J[0], J[1])
    scale = np.abs(drho / DT).max()
    assert np.abs(res).max() <= 1e-13 * scale


@pytest.mark.parametrize("move", MOVES)
def test_deposit_total_current_is_charge_times_velocity(move):
    x0, y0, x1, y1 = move
    Q, vz = 0.8, -0.37
    J = oracle.deposit(_cfg(), Q, x0, y0, x1, y1, vz)
    tot = J.sum(axis=(1, 2)) * DX * DY
    want = np.array([Q * (x1 - x0) / DT, Q * (y1 - y0) / DT, Q * vz])
    np.testing.assert_allclose(tot, want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("move", MOVES)
def test_out_of_plane_current_is_the_path_average_of_the_shape(move):
    # Jz(i, j) = Q vz/(dx dy) * int_0^1 Sx_i(t) Sy_j(t) dt with S(t) = S0 + t (S1 - S0) the linear
    # interpolation of each node's shape factor between the old and new positions
    x0, y0, x1, y1 = move
    Q, vz = 1.3, 0.6
    J = oracle.deposit(_cfg(), Q, x0, y0, x1, y1, vz)
    r0, r1 = _rho(1.0, x0, y0) * DX * DY, _rho(1.0, x1, y1) * DX * DY  # node shape products
    # separable factors: S(x)S(y) per node; build the 1-D factors to interpolate each linearly
    def fac(x, n, d):
        f = np.zeros(n)
        g = x / d
        i0 = math.floor(g)
        f[i0 % n] += 1 - abs(g - i0)
        f[(i0 + 1) % n] += 1 - abs(g - i0 - 1)
        return f
    sx0, sx1, sy0, sy1 = fac(x0, NX, DX), fac(x1, NX, DX), fac(y0, NY, DY), fac(y1, NY, DY)
    assert np.allclose(np.outer(sy0, sx0), r0) and np.allclose(np.outer(sy1, sx1), r1)
    ts, ws = np.polynomial.legendre.leggauss(4)  # exact for the quadratic integrand
    ts, ws = 0.5 * (ts + 1), 0.5 * ws
    avg = sum(w * np.outer(sy0 + t * (sy1 - sy0), sx0 + t * (sx1 - sx0)) for t, w in zip(ts, ws))
    np.testing.assert_allclose(J[2], Q * vz * avg / (DX * DY), rtol=0, atol=1e-14 * abs(Q * vz) / (DX * DY))


def _mode(kind, mx, my, n, nx=32, ny=16, dx=0.25, dy=0.3, dt=0.12):
    """Planes (9, ny, nx) of a vacuum eigenmode of the Yee scheme at step n: wave numbers of the
    periodic box, frequency from sin^2(w dt/2)/dt^2 = sum sin^2(k d/2)/d^2.  E sits at whole
    steps; the solver's B at whole steps is the mean of its half-step values, cos(w dt/2) times
    the half-step amplitude.  kind 'TM': Ez, Bx, By; 'TE': Bz, Ex, Ey."""
    kx, ky = 2 * math.pi * mx / (nx * dx), 2 * math.pi * my / (ny * dy)
    Kx, Ky = 2 * math.sin(kx * dx / 2) / dx, 2 * math.sin(ky * dy / 2) / dy
    Om = math.hypot(Kx, Ky)
    w = 2 * math.asin(Om * dt / 2) / dt
    t = n * dt
    c = math.cos(w * dt / 2)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    ph = lambda ox, oy: kx * (i + ox) * dx + ky * (j + oy) * dy - w * t
    F = np.zeros((9, ny, nx))
    if kind == "TM":
        F[2] = np.cos(ph(0, 0))                       # Ez (i, j)
        F[3] = c * (Ky / Om) * np.cos(ph(0, 0.5))     # Bx (i, j+1/2)
        F[4] = -c * (Kx / Om) * np.cos(ph(0.5, 0))    # By (i+1/2, j)
    else:
        F[5] = c * np.cos(ph(0.5, 0.5))               # Bz (i+1/2, j+1/2)
        F[0] = -(Ky / Om) * np.cos(ph(0.5, 0))        # Ex (i+1/2, j)
        F[1] = (Kx / Om) * np.cos(ph(0, 0.5))         # Ey (i, j+1/2)
    return F, (nx, ny, dx, dy, dt)


@pytest.mark.parametrize("kind,mx,my", [("TM", 1, 0), ("TM", 2, 3), ("TE", 0, 1), ("TE", 3, 2)])
def test_yee_vacuum_modes_follow_the_discrete_dispersion_relation(kind, mx, my):
    F0, (nx, ny, dx, dy, dt) = _mode(kind, mx, my, 0)
    cfg = _cfg(nx, ny, dx, dy, dt)
    F = F0
    steps = 27  # no whole number of periods for these modes
    for _ in range(steps):
        F = oracle.fdtd_step(cfg, F)
    want, _ = _mode(kind, mx, my, steps)
    assert np.abs(F[:6] - want[:6]).max() < 1e-12
    # the mode moved: far from its start
    assert np.abs(F[:6] - F0[:6]).max() > 0.1


def test_gauss_law_residual_is_kept_by_a_coupled_run_with_events(oracle_tables_small):
    # electrons in a strong grid field with emission and pairs: the residual div E - rho of the
    # initial state (here a field that does not satisfy Gauss's law) must persist unchanged
    nx, ny, dx, dy = 16, 12, 0.5, 0.5
    dt = 0.2  # below the Courant limit dx / sqrt(2)
    rng = np.random.default_rng(7)
    n = 40
    Q = 2e-6
    e = dict(x=rng.uniform(0, nx * dx, n), y=rng.uniform(0, ny * dy, n), ux=rng.normal(0, 300, n),
             uy=rng.normal(0, 300, n), uz=rng.normal(0, 300, n),
             uid=np.arange(1, n + 1, dtype=np.uint64))
    F = np.zeros((9, ny, nx))
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    F[1] = 2e-3 * np.cos(2 * math.pi * i / nx)
    F[2] = 2e-3 * np.sin(2 * math.pi * j / ny)
    F[5] = 1.5e-3 * np.cos(2 * math.pi * (i + 0.5) / nx)
    cfg = oracle.RunConfig(field_kind=oracle.FIELD_GRID_FDTD, field=(Q,), dt=dt, n_steps=25, dims=2,
                           grid=(nx, ny, dx, dy, 0.0, 0.0))
    res, led = oracle.run(cfg, oracle_tables_small, electrons=e, fields=F)
    assert led["n_emit"] > 0 and led["n_pair"] > 0
    kw = dict(nx=nx, ny=ny, dx=dx, dy=dy)
    r0 = _rho(-Q, e["x"], e["y"], **kw)
    el, po = res["electron"], res["positron"]
    r1 = _rho(-Q, el["x"], el["y"], **kw) + _rho(Q, po["x"], po["y"], **kw)
    g0 = _div(F[0], F[1], dx, dy) - r0
    F1 = led["fields"]
    g1 = _div(F1[0], F1[1], dx, dy) - r1
    scale = np.abs(r0).max()
    assert np.abs(g1 - g0).max() < 1e-9 * scale
    # the particles did change the field (feedback is on): E moved by more than the residual check
    assert np.abs(F1[0] - F[0]).max() > 0.0


def test_cold_plasma_oscillates_at_the_plasma_frequency(oracle_tables_small):
    # electrons displaced by xi(x) = d sin(k x) over a neutralising background oscillate at
    # omega_p^2 = kappa Q n (Lorentz force du/dt = q kappa E in code units, Gauss div E = rho,
    # n macro-particles per unit area); E starts as the solution of Gauss's law
    nx, ny, dx, dy = 64, 2, 0.2, 0.2
    dt = 0.05
    kappa = 1e-6 / 2.42631023867e-12
    per = 8
    x0 = (np.arange(nx * per) + 0.5) * dx / per
    xs = np.concatenate([x0, x0])
    ys = np.concatenate([np.full_like(x0, 0.5 * dy), np.full_like(x0, 1.5 * dy)])
    n_area = len(xs) / (nx * dx * ny * dy)
    wp = 0.5
    Q = wp ** 2 / (kappa * n_area)
    k = 2 * math.pi / (nx * dx)
    xs = xs + 0.01 * dx * np.sin(k * xs)
    kw = dict(nx=nx, ny=ny, dx=dx, dy=dy)
    rho = _rho(-Q, xs, ys, **kw)
    rho -= rho.mean()
    Ex = np.cumsum(rho.mean(axis=0)) * dx  # (Ex(i+1/2) - Ex(i-1/2))/dx = rho(i)
    Ex -= Ex.mean()
    F = np.zeros((9, ny, nx))
    F[0] = Ex[None, :]
    e = dict(x=xs, y=ys, ux=np.zeros_like(xs), uy=np.zeros_like(xs), uz=np.zeros_like(xs),
             uid=np.arange(1, len(xs) + 1, dtype=np.uint64))
    xe = (np.arange(nx) + 0.5) * dx
    amp = []
    chunk = 10
    for c in range(32):
        cfg = oracle.RunConfig(field_kind=oracle.FIELD_GRID_FDTD, field=(Q,), dt=dt, n_steps=chunk, step0=c * chunk,
                               dims=2, grid=(nx, ny, dx, dy, 0.0, 0.0), flags=0, draw_initial_tau=False)
        e["tau"] = np.ones(len(e["x"]))
        amp.append(float((F[0].mean(axis=0) * np.sin(k * xe)).sum()))
        res, led = oracle.run(cfg, oracle_tables_small, electrons=e, fields=F)
        order = np.argsort(res["electron"]["uid"])
        e = {key: res["electron"][key][order] for key in ("x", "y", "ux", "uy", "uz", "uid")}
        F = led["fields"]
    t = np.arange(len(amp)) * chunk * dt
    a = np.array(amp)
    ws = np.linspace(0.4, 0.6, 2001)
    err = [np.linalg.lstsq(np.stack([np.cos(w * t), np.sin(w * t)], 1), a, rcond=None)[1].sum() for w in ws]
    w_fit = ws[int(np.argmin(err))]
    # finite-k and leapfrog corrections are below a per cent at k dx = 0.1, w dt = 0.025
    assert abs(w_fit / wp - 1) < 0.01, w_fit
