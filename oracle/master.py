"""Direct solution of the energy-space kinetic equations (eqs. 6 and 7, Sec. 2.4) for electrons,
positrons and photons moving perpendicular to a uniform magnetic field B' (in units of the
Schwinger field), the paper's own check of its Monte-Carlo (Sec. 4: first-order in time, with
dt < 0.1 Delta t_QED).  Test infrastructure: the tests compare the Monte-Carlo's ensemble
spectra with these solutions; nothing here is used by the library.

Readings (the equations are written for ultra-relativistic particles):
  * eta = gamma B' for a lepton and chi = eps B'/2 for a photon; a photon of chi emitted by a
    lepton of gamma takes energy eps = 2 chi / B' from it (eq. 1 with eta = gamma B').
  * rates in code time (omega = 2 pi c / lambda_L): lambda_gamma = A_g (eta/gamma) h(eta) with
    A_g = sqrt(3) alpha kappa / (2 pi) (eq. 2); lambda_pm = A_p chi T(chi) / eps with
    A_p = alpha kappa (eq. 3); p_chi = F/(chi h) (Sec. 2.1); p_f from Appendix B, the positron
    taking f and the electron 1 - f (p_f is symmetric, so both gain the same spectrum).

Discretisation: energies on cells with log-spaced edges from gamma_min to just above gamma0
(gamma0 is the top cell's centre); a cell holds the probability Phi * d(gamma) of its interval.
  * An emission that takes a lepton below its own cell's lower edge is a jump to the cell that
    holds gamma - eps (the emitted number integrated over that cell's range of eps); the smaller
    emissions, which cannot leave the cell, act as a continuous energy loss (their radiated power)
    moved to the next cell down by a first-order upwind flux.  Leptons that fall below gamma_min
    collect in the lowest cell.
  * A photon is counted in the cell holding its energy (photons below gamma_min are dropped: they
    carry a negligible share of the energy).
  * Pair creation moves a photon's probability to the lepton cells of f eps and (1 - f) eps.
  * Explicit Euler steps in time.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import energy_below, h as h_fn, number_cumulative, pf_cumulative, T as T_fn

ALPHA = 7.2973525693e-3
LAMBDA_COMPTON = 2.42631023867e-12  # h/(m_e c), metres


@dataclass
class MasterSolution:
    edges: np.ndarray     # cell edges (energy, m c^2)
    centres: np.ndarray   # geometric cell centres
    t: float              # time reached (code units)
    electron: np.ndarray  # probability per cell, per initial electron
    positron: np.ndarray
    photon: np.ndarray

    def energy(self, which: str) -> float:
        return float(np.sum(self.centres * getattr(self, which)))

    def number(self, which: str) -> float:
        return float(np.sum(getattr(self, which)))


def _grid(gamma0: float, gamma_min: float, cells_per_e: int):
    n = int(math.ceil(math.log(gamma0 / gamma_min) * cells_per_e))
    r = math.exp(math.log(gamma0 / gamma_min) / n)
    # gamma0 at the centre of the top cell
    top = gamma0 * math.sqrt(r)
    edges = top / r ** np.arange(n + 1)[::-1]
    centres = np.sqrt(edges[:-1] * edges[1:])
    return edges, centres


def _kernels(b: float, edges: np.ndarray, centres: np.ndarray, kappa: float, pairs: bool, t_end: float = 0.0,
             threads: int = 8):
    """Rates between cells (per unit code time), built from the oracle's F/chi, F, T, p_f."""
    from concurrent.futures import ThreadPoolExecutor
    n = len(centres)
    a_g = math.sqrt(3.0) * ALPHA * kappa / (2.0 * math.pi)
    a_p = ALPHA * kappa
    jump = np.zeros((n, n))    # lepton cell j -> lepton cell i < j
    emit = np.zeros((n, n))    # lepton cell j -> photon cell m (rate of photons per lepton)
    drift = np.zeros(n)        # upwind rate from cell j to j - 1 (sub-cell emissions)

    def lepton_row(j):
        g = centres[j]
        eta = g * b
        pre = a_g * eta / g                      # times the emitted number int F/chi dchi
        # lepton targets: eps = g - gamma' at the edges below the cell
        eps_l = g - edges[: j + 1]               # eps at edges 0..j (largest first)
        cum_l = number_cumulative(eta, eps_l[::-1] * b / 2.0)[::-1]  # N(eps at edge i)
        hh = h_fn(eta)
        # cell i < j receives eps in [g - e_{i+1}, g - e_i]; below edge 0 collects in cell 0
        for i in range(j):
            jump[i, j] = pre * ((cum_l[i] if i > 0 else hh) - cum_l[i + 1])
        # sub-cell emissions (eps < g - e_j): their power moves the lepton down continuously
        if j > 0:
            chi_sub = (g - edges[j]) * b / 2.0
            p_sub = pre * energy_below(eta, chi_sub) * 2.0 / b   # energy per unit time (m c^2)
            drift[j] = p_sub / (centres[j] - centres[j - 1])
        # photons: eps in [e_m, e_{m+1}] (and eps <= g)
        emit[:, j] = pre * np.diff(number_cumulative(eta, np.minimum(edges, g) * b / 2.0))

    pair = np.zeros((n, n))    # photon cell k -> lepton cell i (per lepton species)
    absorb = np.zeros(n)       # photon cell k: pair rate

    def photon_row(k):
        eps = centres[k]
        chi = eps * b / 2.0
        rate = a_p * chi * T_fn(chi) / eps
        if not rate * max(t_end, 1.0) > 1e-14:  # photons that (practically) never convert
            return
        absorb[k] = rate
        cum = pf_cumulative(chi, np.clip(edges / eps, 0.0, 1.0))
        pair[:, k] = rate * np.diff(cum)
        pair[0, k] += rate * cum[0]              # leptons below gamma_min

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lepton_row, range(n)))
        if pairs:
            list(ex.map(photon_row, range(n)))
    return jump, emit, drift, pair, absorb


def _kernels_cached(b, gamma0, gamma_min, cells_per_e, kappa, pairs, t_end):
    """_kernels, stored on disk per (oracle source, parameters): building them takes minutes."""
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    src = b"".join(open(os.path.join(here, f), "rb").read() for f in ("qed_oracle.cpp", "master.py"))
    key = hashlib.sha1(src + repr((b, gamma0, gamma_min, cells_per_e, kappa, pairs, t_end)).encode()).hexdigest()[:16]
    path = os.path.join(here, "_cache", "master_%s.npz" % key)
    edges, centres = _grid(gamma0, gamma_min, cells_per_e)
    if os.path.exists(path):
        d = np.load(path)
        return edges, centres, (d["jump"], d["emit"], d["drift"], d["pair"], d["absorb"])
    k = _kernels(b, edges, centres, kappa, pairs, t_end)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, jump=k[0], emit=k[1], drift=k[2], pair=k[3], absorb=k[4])
    os.replace(tmp, path)
    return edges, centres, k


def solve(b: float, gamma0: float, t_end: float, dt_over_qed: float = 0.05, cells_per_e: int = 20,
          gamma_min: float = 1.0, pairs: bool = True, lambda_L: float = 1e-6, h0: float = 5.24) -> MasterSolution:
    """Phi_-, Phi_+ and Phi_gamma at t_end for electrons starting at gamma0 perpendicular to B'."""
    kappa = lambda_L / LAMBDA_COMPTON
    edges, centres, (jump, emit, drift, pair, absorb) = _kernels_cached(b, gamma0, gamma_min, cells_per_e, kappa,
                                                                         pairs, t_end)
    out_jump = jump.sum(axis=0)
    # Delta t_QED = 1 / max lambda_gamma with the paper's h0 (Sec. 3.1), as the Monte-Carlo presets
    dt_qed = 1.0 / (2.0 * math.sqrt(3.0) * ALPHA * kappa / (2.0 * math.pi) * b * h0)
    n_steps = max(1, int(math.ceil(t_end / (dt_over_qed * dt_qed))))
    dt = t_end / n_steps
    n = len(centres)
    e = np.zeros(n)
    e[-1] = 1.0
    p = np.zeros(n)
    g = np.zeros(n)
    for _ in range(n_steps):
        de = jump @ e - out_jump * e
        dp = jump @ p - out_jump * p
        de[:-1] += drift[1:] * e[1:]
        de -= drift * e
        dp[:-1] += drift[1:] * p[1:]
        dp -= drift * p
        dg = emit @ (e + p) - absorb * g
        if pairs:
            src = pair @ g
            de += src
            dp += src
        e = e + dt * de
        p = p + dt * dp
        g = g + dt * dg
    return MasterSolution(edges=edges, centres=centres, t=t_end, electron=e, positron=p, photon=g)


def mean_loss_rate(b: float, gamma0: float, cells_per_e: int = 20, gamma_min: float = 1.0,
                   lambda_L: float = 1e-6) -> float:
    """d<gamma>/dt at t = 0 from the discretised lepton operator (jumps + drift), per electron."""
    kappa = lambda_L / LAMBDA_COMPTON
    edges, centres = _grid(gamma0, gamma_min, cells_per_e)
    jump, _, drift, _, _ = _kernels(b, edges, centres, kappa, pairs=False)
    j = len(centres) - 1
    return float(np.sum((centres - centres[j]) * jump[:, j]) + (centres[j - 1] - centres[j]) * drift[j])
