"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds only input recipes (initial particles, field parameters, time
steps, run lengths).  It holds none of the method's arithmetic: no rates, no
tables, no sampling, no push.  Both the GPU path and the oracle consume what it
produces, so it is the one module they share.

Code units: time t' = w t with w = 2 pi c / lambda_L, length x' = w x / c,
momentum u = p / (m c), fields E' = E / E_s and B' = c B / E_s.  Converting the
physical inputs (a0, field in units of E_s, pulse length in fs, beam size in um)
needs kappa = lambda_L / lambda_c, defined here for that purpose only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dfield

import numpy as np

LAMBDA_L = 1.0e-6                 # laser wavelength defining the code units (m)
LAMBDA_COMPTON = 2.42631023867e-12  # h / (m_e c), CODATA 2018 (m)
KAPPA = LAMBDA_L / LAMBDA_COMPTON   # m c^2 / (hbar w): converts a0 <-> E'
C_LIGHT = 299792458.0
OMEGA = 2.0 * math.pi * C_LIGHT / LAMBDA_L  # rad/s per unit code time

FIELD_UNIFORM = 0
FIELD_LP_PULSE = 1
FIELD_CP_WAVE = 2
FIELD_CP_STANDING = 3
FIELD_GRID_CP_STANDING = 4
FIELD_GRID_FDTD = 5

FLAG_EMIT = 1
FLAG_PAIRS = 2
FLAG_PROPAGATE = 4


def fs_to_code(t_fs: float) -> float:
    return OMEGA * t_fs * 1e-15


def um_to_code(x_um: float) -> float:
    return 2.0 * math.pi * x_um * 1e-6 / LAMBDA_L


@dataclass
class Workload:
    """One instance: initial particles plus everything a run needs besides tables."""
    name: str
    field_kind: int
    field: tuple
    dt: float
    n_steps: int
    flags: int
    electrons: dict
    dims: int = 3
    seed: int = 1
    instance: int = 0
    t0: float = 0.0
    weight: float = 1.0
    grid: tuple = (0, 0, 0.0, 0.0, 0.0, 0.0)   # nx, ny, dx, dy, x0, y0
    fields: np.ndarray | None = None           # field feedback: initial planes (9, ny, nx), Ex..Bz, Jx..Jz
    capacity: dict = dfield(default_factory=dict)  # per species: electron, positron, photon
    notes: str = ""

    @property
    def n(self) -> int:
        return len(self.electrons["uid"])


def _beam(n, gamma, direction, pos, dims, uid0=0):
    """Electrons moving along `direction` with Lorentz factors `gamma` at positions `pos`."""
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (n,)).copy()
    p = np.sqrt(gamma * gamma - 1.0)
    d = np.asarray(direction, dtype=np.float64)
    e = {"x": pos[0].copy(), "y": pos[1].copy(),
         "ux": p * d[0], "uy": p * d[1], "uz": p * d[2],
         "uid": np.arange(uid0, uid0 + n, dtype=np.uint64)}
    if dims == 3:
        e["z"] = pos[2].copy()
    return e


# ---------------------------------------------------------------------------
# uniform static magnetic field (paper tests 1 and 3)
# ---------------------------------------------------------------------------
def gyro_period(gamma0: float, b: float) -> float:
    """Code-time gyration period 2 pi gamma / (kappa B') of a lepton in B'."""
    return 2.0 * math.pi * gamma0 / (KAPPA * b)


def uniform_b(n: int, gamma0: float, b: float, dt: float, n_steps: int, flags: int,
              seed: int = 1, name: str = "uniform_b") -> Workload:
    """Electrons at the origin with u perpendicular to a uniform B' = b z_hat."""
    zeros = np.zeros(n)
    e = _beam(n, gamma0, (1.0, 0.0, 0.0), (zeros, zeros, zeros), 3)
    w = Workload(name=name, field_kind=FIELD_UNIFORM, field=(0.0, 0.0, 0.0, 0.0, 0.0, b), dt=dt,
                 n_steps=n_steps, flags=flags, electrons=e, seed=seed)
    # at most one emission per particle per step (Sec. 3.1); pairs per photon
    ph = n * n_steps + 1024
    w.capacity = dict(electron=n + 2 * ph if flags & FLAG_PAIRS else n + 1024,
                      positron=2 * ph if flags & FLAG_PAIRS else 1024, photon=ph)
    return w


def dt_qed(field_max: float, h0: float = 5.24) -> float:
    """Code-time Delta t_QED = 1 / Max lambda_gamma for a peak field Max(E, cB)/E_s
    (Sec. 3.1, with the paper's h0 = 5.24), used to set the step of the physics presets."""
    alpha = 7.2973525693e-3
    return 1.0 / (2.0 * math.sqrt(3.0) * alpha * KAPPA / (2.0 * math.pi) * field_max * h0)


def uniform_b_config1() -> Workload:
    """Uniform B, 1e4 electrons, gamma0 = 1000 perpendicular to B (eta0 = 1), dt = 0.01
    gyro-periods, 1000 steps, photons emitted but not propagated, seed 1."""
    b = 1e-3
    return uniform_b(10_000, 1000.0, b, 0.01 * gyro_period(1000.0, b), 1000, FLAG_EMIT, 1,
                     name="uniform_b_1e4")


def paper_test(test: int, n: int, dt_over_qed: float, seed: int = 1, pairs: bool = True) -> Workload:
    """Paper tests 1 and 3 (Table 1): gamma0 = 1000 perpendicular to B' = 1e-3 or 9e-3, run
    to t0 = 1 fs or 0.1 fs with dt = dt_over_qed * Delta t_QED."""
    b, t_end = {1: (1e-3, 1.0), 3: (9e-3, 0.1)}[test]
    dt_q = dt_qed(b)
    n_steps = max(1, int(round(fs_to_code(t_end) / (dt_over_qed * dt_q))))
    dt = fs_to_code(t_end) / n_steps
    flags = FLAG_EMIT | (FLAG_PAIRS | FLAG_PROPAGATE if pairs else 0)
    return uniform_b(n, 1000.0, b, dt, n_steps, flags, seed, name="paper_test%d" % test)


# ---------------------------------------------------------------------------
# circularly polarised plane wave (paper test 2)
# ---------------------------------------------------------------------------
def cp_wave_test2(n: int, dt_over_qed: float = 0.3, seed: int = 1, pairs: bool = True) -> Workload:
    """Paper test 2: gamma0 = 4120 counter-propagating against a CP wave with
    |E|/E_s = c|B|/E_s = 1.22e-4 (a = 50), run to 3 fs."""
    e0 = 1.22e-4
    dt_q = dt_qed(e0)
    t_end = fs_to_code(3.0)
    n_steps = max(1, int(round(t_end / (dt_over_qed * dt_q))))
    zeros = np.zeros(n)
    e = _beam(n, 4120.0, (-1.0, 0.0, 0.0), (zeros, zeros, zeros), 3)
    flags = FLAG_EMIT | (FLAG_PAIRS | FLAG_PROPAGATE if pairs else 0)
    w = Workload(name="paper_test2", field_kind=FIELD_CP_WAVE, field=(e0, 0.0), dt=t_end / n_steps,
                 n_steps=n_steps, flags=flags, electrons=e, seed=seed)
    ph = n * n_steps + 1024
    w.capacity = dict(electron=n + 2 * ph, positron=2 * ph, photon=ph)
    return w


# ---------------------------------------------------------------------------
# head-on collision with a linearly polarised sin^2 pulse
# ---------------------------------------------------------------------------
def lp_pulse_duration(fwhm_fs: float) -> float:
    """Full code-time length Psi of a sin^2 field envelope whose intensity (sin^4) has the
    given FWHM: sin^4(pi psi / Psi) = 1/2 at psi / Psi = asin(2^-1/4) / pi."""
    frac = 1.0 - 2.0 * math.asin(2.0 ** -0.25) / math.pi
    return fs_to_code(fwhm_fs / frac)


def collision(n: int, a0: float = 200.0, gamma_mean: float = 2000.0, gamma_rel_sd: float = 0.1,
              sigma_um: float = 2.0, fwhm_fs: float = 30.0, dt: float = 2.0 * math.pi / 200.0,
              n_steps: int = 20_000, meet_step: int | None = None, seed: int = 1, instance: int = 0,
              flags: int = FLAG_EMIT | FLAG_PAIRS | FLAG_PROPAGATE, uid0: int = 0,
              name: str = "collision_lp") -> Workload:
    """Electron beam along -x meeting an LP pulse travelling along +x (E_y, B_z).

    Beam: gamma ~ N(gamma_mean, gamma_rel_sd * gamma_mean) (truncated at 1.5), Gaussian
    positions with sigma = sigma_um in x, y and z, centred on the origin at t = 0.  The
    pulse peak meets the beam centre at step `meet_step` (default n_steps / 2).
    """
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, instance], dtype=np.uint64)))
    gam = rng.normal(gamma_mean, gamma_rel_sd * gamma_mean, n)
    gam = np.maximum(gam, 1.5)
    sig = um_to_code(sigma_um)
    pos = (rng.normal(0.0, sig, n), rng.normal(0.0, sig, n), rng.normal(0.0, sig, n))
    e = _beam(n, gam, (-1.0, 0.0, 0.0), pos, 3, uid0)
    e0 = a0 / KAPPA
    psi_len = lp_pulse_duration(fwhm_fs)
    m = n_steps // 2 if meet_step is None else meet_step
    t_m = m * dt
    beta = math.sqrt(1.0 - 1.0 / (gamma_mean * gamma_mean))
    # envelope argument psi = t - x - psi0; the peak (psi = Psi/2) reaches x = -beta t_m at t_m
    psi0 = t_m + beta * t_m - 0.5 * psi_len
    w = Workload(name=name, field_kind=FIELD_LP_PULSE, field=(e0, psi_len, psi0, 0.0), dt=dt,
                 n_steps=n_steps, flags=flags, electrons=e, seed=seed, instance=instance,
                 notes="a0=%g gamma=%g" % (a0, gamma_mean))
    # room for the emission and pair yield of a0 <= 500, gamma <= 5000 beams
    w.capacity = dict(electron=3 * n + 4096, positron=2 * n + 4096, photon=160 * n + 8192)
    return w


def photon_population(n: int, eps_min: float = 10.0, eps_max: float = 1e5, sigma_um: float = 2.0,
                      comoving_x: tuple | None = None, seed: int = 1, uid0: int = 1 << 40) -> dict:
    """Photons (birth step 0) around the origin for the collision geometry: energies
    log-uniform in [eps_min, eps_max]; directions 60% along -x, 20% isotropic, 10% at a small
    angle to +x (1 - n_x log-uniform in [1e-12, 1e-4]) and 10% exactly along +x (moving with
    the pulse); Gaussian positions with sigma = sigma_um, except that the photons moving along
    +x are spread uniformly in x over `comoving_x` when it is given."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0xF0700], dtype=np.uint64)))
    eps = 10.0 ** rng.uniform(math.log10(eps_min), math.log10(eps_max), n)
    kind = rng.uniform(0.0, 1.0, n)
    d = np.zeros((n, 3))
    d[:, 0] = -1.0
    iso = (kind >= 0.6) & (kind < 0.8)
    c = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s_ = np.sqrt(1.0 - c * c)
    d[iso] = np.stack([c, s_ * np.cos(phi), s_ * np.sin(phi)], axis=1)[iso]
    near = (kind >= 0.8) & (kind < 0.9)
    om = 10.0 ** rng.uniform(-12.0, -4.0, n)         # 1 - cos(theta)
    sn = np.sqrt(om * (2.0 - om))
    d[near] = np.stack([1.0 - om, sn * np.cos(phi), sn * np.sin(phi)], axis=1)[near]
    d[kind >= 0.9] = (1.0, 0.0, 0.0)
    sig = um_to_code(sigma_um)
    x = rng.normal(0.0, sig, n)
    if comoving_x is not None:
        x = np.where(kind >= 0.8, rng.uniform(comoving_x[0], comoving_x[1], n), x)
    return {"x": x, "y": rng.normal(0.0, sig, n), "z": rng.normal(0.0, sig, n),
            "ux": eps * d[:, 0], "uy": eps * d[:, 1], "uz": eps * d[:, 2],
            "uid": np.arange(uid0, uid0 + n, dtype=np.uint64), "birth_step": np.zeros(n, dtype=np.int64)}


def collision_config2(n: int = 1_000_000, n_steps: int = 20_000) -> Workload:
    """1e6 electrons, gamma ~ N(2000, 10%), sigma = 2 um, LP a0 = 200, lambda = 1 um,
    30 fs (intensity FWHM) sin^2 envelope, dt = lambda/(200 c), 20000 steps, pairs on."""
    w = collision(n, n_steps=n_steps, meet_step=10_000 if n_steps >= 20_000 else None,
                  name="collision_lp_a200")
    w.capacity = dict(electron=n * 3 + 1024, positron=n * 2 + 1024, photon=n * 120 + 4096)
    return w


def batched_config5(n_inst: int = 256, seed: int = 1, n_scale: float = 1.0, n_steps: int = 20_000) -> list:
    """256 independent collisions: N_i = floor(10^U(3,6)), a0 ~ U(50, 500), gamma0 log-uniform
    in [500, 5000] with a 10% spread, geometry of the collision preset."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0xBA7C4], dtype=np.uint64)))
    logn = rng.uniform(3.0, 6.0, n_inst)
    a0 = rng.uniform(50.0, 500.0, n_inst)
    g0 = 10.0 ** rng.uniform(math.log10(500.0), math.log10(5000.0), n_inst)
    out = []
    for i in range(n_inst):
        n = max(1, int(math.floor(10.0 ** logn[i] * n_scale)))
        w = collision(n, a0=float(a0[i]), gamma_mean=float(g0[i]), n_steps=n_steps, seed=seed,
                      instance=i, name="batched_%d" % i)
        out.append(w)
    return out


# ---------------------------------------------------------------------------
# standing wave of two counter-propagating CP lasers on a 2-D Yee grid
# ---------------------------------------------------------------------------
def grid_config3(n: int = 16_000_000, nx: int = 4096, ny: int = 2048, cells_per_lambda: int = 128,
                 a0: float = 500.0, dt: float = 2.0 * math.pi / 400.0, n_steps: int = 2000,
                 seed: int = 1) -> Workload:
    """Electrons at rest, uniform over a periodic nx x ny grid with dx = dy = lambda/128,
    in the standing wave of two CP lasers of amplitude a0 each; 2-D3V."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 0x3D], dtype=np.uint64)))
    dx = 2.0 * math.pi / cells_per_lambda
    lx, ly = nx * dx, ny * dx
    pos = (rng.uniform(0.0, lx, n), rng.uniform(0.0, ly, n), None)
    e = {"x": pos[0], "y": pos[1], "ux": np.zeros(n), "uy": np.zeros(n), "uz": np.zeros(n),
         "uid": np.arange(n, dtype=np.uint64)}
    w = Workload(name="grid_cp_standing_a500", field_kind=FIELD_GRID_CP_STANDING, field=(a0 / KAPPA,),
                 dt=dt, n_steps=n_steps, flags=FLAG_EMIT | FLAG_PAIRS | FLAG_PROPAGATE, electrons=e,
                 dims=2, seed=seed, grid=(nx, ny, dx, dx, 0.0, 0.0))
    w.capacity = dict(electron=4 * n, positron=2 * n, photon=4 * n)
    return w


def standing_wave_planes(e0: float, nx: int, ny: int, dx: float, dy: float, x0: float = 0.0) -> np.ndarray:
    """Initial planes (9, ny, nx) of the solver grid: the standing wave of two CP lasers at t = 0
    (E_y = 2 e0 cos x, B_y = 2 e0 sin x, the rest zero) at the Yee nodes, zero current."""
    F = np.zeros((9, ny, nx))
    xa = x0 + np.arange(nx) * dx          # nodes of Ey, Ez, Bx
    xb = x0 + (np.arange(nx) + 0.5) * dx  # nodes of Ex, By, Bz
    F[1] = 2.0 * e0 * np.cos(xa)[None, :]
    F[4] = 2.0 * e0 * np.sin(xb)[None, :]
    return F


def feedback_config(n: int = 16_000_000, nx: int = 4096, ny: int = 2048, cells_per_lambda: int = 128,
                    a0: float = 500.0, density: float = 1e-3, dt: float = 2.0 * math.pi / 400.0,
                    n_steps: int = 2000, seed: int = 1) -> Workload:
    """Configuration 3 with field feedback: the electrons (at rest, uniform) are a plasma of
    `density` times the critical density n_c whose current drives the grid's fields; the grid
    starts with the standing wave of two CP lasers of amplitude a0 each.  An immobile ion
    background neutralises the plasma (its charge never enters: the solver advances E with the
    current only).  Charge per macro-particle in code units: from omega_p^2 = kappa Q n_m (n_m
    macro-particles per unit area) and omega_p^2 / omega^2 = n / n_c, Q = (n/n_c) / (kappa n_m)."""
    w = grid_config3(n=n, nx=nx, ny=ny, cells_per_lambda=cells_per_lambda, a0=a0, dt=dt, n_steps=n_steps, seed=seed)
    dx = w.grid[2]
    n_m = n / (nx * dx * ny * dx)
    q = density / (KAPPA * n_m)
    w.name = "feedback_cp_standing_a500"
    w.field_kind = FIELD_GRID_FDTD
    w.field = (q,)
    w.fields = standing_wave_planes(a0 / KAPPA, nx, ny, dx, dx)
    w.notes = "plasma density %g n_c, charge per macro-particle %.4g (code units)" % (density, q)
    return w


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to the initial electrons `idx` (uids preserved)."""
    idx = np.asarray(idx)
    e = {k: v[idx].copy() for k, v in w.electrons.items()}
    return Workload(name=w.name + "_subset", field_kind=w.field_kind, field=w.field, dt=w.dt,
                    n_steps=w.n_steps, flags=w.flags, electrons=e, dims=w.dims, seed=w.seed,
                    instance=w.instance, t0=w.t0, weight=w.weight, grid=w.grid,
                    capacity=dict(w.capacity), notes=w.notes,
                    fields=None if w.fields is None else w.fields.copy())
