"""Pins of the oracle's look-up tables (Sec. 3: h, T_pm, P_chi, P_f) against the
functions they tabulate (pinned in test_oracle_special.py), closed-form moments,
the energy cut-off definition and the symmetry of p_f."""
import math

import numpy as np
import pytest

import oracle


def eta_grid(t):
    p = t["params"]
    return np.exp(np.linspace(math.log(p["eta_min"]), math.log(p["eta_max"]), p["n_eta"]))


def chi_pair_grid(t):
    p = t["params"]
    return np.exp(np.linspace(math.log(p["chi_pair_min"]), math.log(p["chi_pair_max"]), p["n_chi_pair"]))


def test_h_table_is_h(oracle_tables_small):
    t = oracle_tables_small
    eta = eta_grid(t)
    for i in (0, 7, 20, 33, len(eta) - 1):
        assert t["h"][i] == pytest.approx(oracle.h(eta[i]), rel=1e-12)


def test_chi_rows_span_cutoff_to_half_eta(oracle_tables_small):
    t = oracle_tables_small
    eta = eta_grid(t)
    n = t["params"]["n_chi"]
    for i in (0, 10, 25, len(eta) - 1):
        top = t["lnchi_min"][i] + (n - 1) * t["dlnchi"][i]
        assert top == pytest.approx(math.log(eta[i] / 2), abs=1e-12)
        chimin = math.exp(t["lnchi_min"][i])
        # Sec. 3: the ignored photons carry 1e-9 of the spectrum's energy
        assert oracle.energy_below(eta[i], chimin) / oracle.energy_below(eta[i], eta[i] / 2) == pytest.approx(
            1e-9, rel=1e-9)


def test_cdf_rows_monotone_and_normalised(oracle_tables):
    P = oracle_tables["P_chi"]
    assert np.all(np.diff(P, axis=1) >= 0)
    assert np.all(P[:, -1] == 1.0)
    # below-cut share: F ~ chi^{1/3} at chi_min, so int_0^{chi_min} F/chi = 3 F(chi_min) (1 + O(y^{2/3}))
    eta = eta_grid(oracle_tables)
    for i in (0, 64, 128, 200, 255):
        chimin = math.exp(oracle_tables["lnchi_min"][i])
        assert P[i, 0] == pytest.approx(3 * oracle.F(eta[i], chimin) / oracle_tables["h"][i], rel=1e-4)
    # about 0.6-0.7 % of emissions fall below the cut (energy share 1e-9, number share ~ (1e-9)^{1/4})
    assert np.all((P[:, 0] > 0.004) & (P[:, 0] < 0.008))


@pytest.mark.parametrize("i", [0, 60, 128, 170, 212])
def test_cdf_mean_photon_fraction(oracle_tables, i):
    # <2 chi/eta> over p_chi = (2/eta) int F dchi / h = (4 pi / 3 sqrt3) eta g(eta) / h(eta)
    t = oracle_tables
    eta = eta_grid(t)[i]
    n = t["params"]["n_chi"]
    P = t["P_chi"][i]
    lnchi = t["lnchi_min"][i] + np.arange(n) * t["dlnchi"][i]
    chi = np.exp(lnchi)
    # the inverse is linear in ln chi on each segment: int chi du = dP (chi_{j+1} - chi_j) / dlnchi
    mean_chi = np.sum(np.diff(P) * np.diff(chi) / t["dlnchi"][i])
    expect = 4 * math.pi / (3 * math.sqrt(3)) * eta * oracle.g(eta) / t["h"][i]
    assert 2 * mean_chi / eta == pytest.approx(expect, rel=2e-3)


def test_T_table_is_T(oracle_tables_small):
    t = oracle_tables_small
    chi = chi_pair_grid(t)
    np.testing.assert_allclose(t["T"], oracle.T(chi), rtol=1e-12)


def test_pair_split_rows_symmetric(oracle_tables):
    # p_f(f) = p_f(1 - f) and the f grid sin^2(pi l / 2(n-1)) is symmetric, so P_f(f_l) + P_f(f_{n-1-l}) = 1
    Pf = oracle_tables["P_f"]
    f = oracle_tables["f_grid"]
    np.testing.assert_allclose(f + f[::-1], 1.0, atol=2e-16)
    np.testing.assert_allclose(Pf + Pf[:, ::-1], 1.0, atol=1e-13)
    assert np.all(np.diff(Pf, axis=1) >= 0)
    assert np.all(Pf[:, 0] == 0.0) and np.all(Pf[:, -1] == 1.0)


def test_pair_split_table_matches_density(oracle_tables_small):
    from scipy import integrate
    t = oracle_tables_small
    chi = chi_pair_grid(t)
    f = t["f_grid"]
    for k in (5, 24, 40):
        # each CDF step is the integral of p_f over its segment
        for j in (1, 10, len(f) // 2, len(f) - 3):
            seg = integrate.quad(lambda x: oracle.pf(x, chi[k]), f[j], f[j + 1], epsrel=1e-12)[0]
            assert t["P_f"][k, j + 1] - t["P_f"][k, j] == pytest.approx(seg, rel=1e-9, abs=1e-15)
        assert t["k_norm"][k] == pytest.approx(oracle.pair_k(chi[k]), rel=1e-12)
