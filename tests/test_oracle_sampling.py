"""Pins of the oracle's two sampling steps against the paper's spectra evaluated independently
(scipy Bessel functions and quadrature, not the oracle's special functions or tables):

  * photon chi drawn from the tabulated 2-D inverse CDF (Sec. 3, Appendix A): one step of
    forced emission at fixed eta, KS test of the sampled chi against the cumulative of F/chi
    above the 1e-9 energy cut, and the fraction of null events (draws below the cut) against
    the share of the rate below chi_min;
  * the positron energy fraction drawn from P_f (Sec. 3, Appendix B): one step of forced pair
    creation at fixed chi, KS test against the cumulative of the unnormalised p_f.
Events are forced by a vanishing initial optical depth, so every particle has its event in the
first step with the state it starts with."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from paper_1311_5551_amd import workloads as W
from test_oracle_special import F_scipy


def _simpson_cumulative(x, y):
    return np.concatenate([[0.0], integrate.cumulative_simpson(y, x=x)])


@pytest.mark.parametrize("eta", [1.0, 10.0])
def test_sampled_chi_follows_the_emission_spectrum(eta, oracle_tables):
    n, g0 = 300_000, 1000.0  # a 2% scale error of chi fails the KS test at this size
    b = eta / math.sqrt(g0 * g0 - 1.0)  # |u| b = eta with u perpendicular to B
    w = W.uniform_b(n, g0, b, 1e-7, 1, W.FLAG_EMIT)
    e = {k: np.asarray(v).copy() for k, v in w.electrons.items()}
    assert np.all(e["ux"] == e["ux"][0])
    e["tau"] = np.full(n, 1e-300)
    cfg = oracle.RunConfig(field_kind=w.field_kind, field=w.field, dt=w.dt, n_steps=1, flags=w.flags, seed=3,
                           draw_initial_tau=False)
    res, led = oracle.run(cfg, oracle_tables, electrons=e)
    assert led["n_emit"] + led["n_null"] == n
    ph = res["photon"]
    umag = math.sqrt(g0 * g0 - 1.0)  # the push in B keeps |u|; dt is negligible
    chi = 0.5 * eta * np.sqrt(ph["ux"] ** 2 + ph["uy"] ** 2 + ph["uz"] ** 2) / umag

    # independent cumulative of F/chi in s = ln chi, from chi_min to eta/2
    chi_min = oracle.cutoff_chi(eta)
    s = np.linspace(math.log(chi_min), math.log(0.5 * eta) - 1e-9, 1601)
    f = np.array([F_scipy(eta, math.exp(v)) for v in s])
    cum = _simpson_cumulative(s, f)
    cdf = lambda c: np.interp(np.log(c), s, cum / cum[-1])
    assert chi.min() >= chi_min * (1 - 1e-9) and chi.max() <= 0.5 * eta
    ks = stats.kstest(chi, cdf)
    assert ks.pvalue > 1e-3, ks

    # null events: share of the full rate below chi_min (F ~ chi^{1/3} there, so the part below
    # a tiny chi_lo is 3 F(chi_lo))
    lo = math.log(chi_min) - math.log(1e3)
    s_lo = np.linspace(lo, math.log(chi_min), 401)
    below = 3.0 * F_scipy(eta, math.exp(lo)) + integrate.simpson([F_scipy(eta, math.exp(v)) for v in s_lo], x=s_lo)
    p0 = below / (below + cum[-1])
    frac = led["n_null"] / n
    assert abs(frac - p0) < 5 * math.sqrt(p0 / n) + 1e-4, (frac, p0)


@pytest.mark.parametrize("chi", [1.0, 10.0])
def test_sampled_pair_split_follows_p_f(chi, oracle_tables):
    n, eps = 60_000, 2000.0
    b = 2.0 * chi / eps  # photon along x in B along z: chi = eps b / 2
    zeros = np.zeros(n)
    ph = {"x": zeros, "y": zeros, "z": zeros, "ux": np.full(n, eps), "uy": zeros, "uz": zeros,
          "uid": np.arange(n, dtype=np.uint64), "tau": np.full(n, 1e-300)}
    cfg = oracle.RunConfig(field_kind=W.FIELD_UNIFORM, field=(0, 0, 0, 0, 0, b), dt=1e-7, n_steps=1,
                           flags=W.FLAG_PAIRS | W.FLAG_PROPAGATE, seed=5, draw_initial_tau=False)
    res, led = oracle.run(cfg, oracle_tables, photons=ph)
    assert led["n_pair"] == n
    fpos = np.asarray(res["positron"]["ux"]) / eps  # the positron takes f k

    # independent cumulative of the unnormalised p_f (Appendix B) on (0, 1)
    q = lambda f: (2 + f * (1 - f)) / (f * (1 - f)) * special.kv(2 / 3, 1 / (3 * chi * f * (1 - f)))
    fg = np.linspace(1e-6, 1 - 1e-6, 4001)
    cum = _simpson_cumulative(fg, np.array([q(v) for v in fg]))
    cdf = lambda f: np.interp(f, fg, cum / cum[-1])
    ks = stats.kstest(fpos, cdf)
    assert ks.pvalue > 1e-3, ks
    # the electron takes the rest
    np.testing.assert_allclose(np.sort(res["electron"]["ux"]) / eps, np.sort(1.0 - fpos), atol=1e-12)
