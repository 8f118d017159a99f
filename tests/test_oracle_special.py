"""Pins of the oracle's special functions (Appendices A and B) and of its Philox and
quadrature primitives, against closed forms, the paper's printed numbers and
independent library routines (scipy's AMOS Bessel functions, numpy's Philox and
Gauss-Legendre rules)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle

H0 = 5.0 * math.pi / 3.0  # classical h: int_0^inf t K_{5/3}(t) dt = Gamma(1/6) Gamma(11/6)


# ---- independent reference: F(eta, chi) from scipy's kv and quad ------------
def kv_tail_scipy(nu, y):
    """int_y^inf K_nu(t) dt by adaptive quadrature of scipy's kv (in ln t below t = 1)."""
    lo = max(y, 1.0)
    val = integrate.quad(lambda t: special.kv(nu, t), lo, lo + 50.0, epsabs=0, epsrel=1e-13, limit=400)[0]
    if y < 1.0:
        g = lambda s: special.kv(nu, math.exp(s)) * math.exp(s)
        a = math.log(y)
        cuts = np.linspace(a, 0.0, max(2, int(-a) + 2))
        val += sum(integrate.quad(g, u, v, epsabs=0, epsrel=1e-13, limit=200)[0] for u, v in zip(cuts[:-1], cuts[1:]))
    return val


def F_scipy(eta, chi):
    xi = 2 * chi / eta
    if xi >= 1:
        return 0.0
    y = 4 * chi / (3 * eta * (eta - 2 * chi))
    return xi * xi * y * special.kv(2 / 3, y) + (1 - xi) * y * kv_tail_scipy(5 / 3, y)


@pytest.mark.parametrize("nu", [1 / 3, 2 / 3, 5 / 3])
def test_bessel_k_matches_scipy(nu):
    for y in [1e-8, 1e-3, 0.1, 1.0, 5.0, 30.0, 200.0]:
        assert oracle.bessel_k(nu, y) == pytest.approx(special.kv(nu, y), rel=1e-13)


def test_bessel_k_tail_matches_quadrature_of_kv():
    for y in [1e-6, 1e-2, 0.3, 1.0, 4.0, 20.0, 100.0]:
        assert oracle.bessel_k_tail(5 / 3, y) == pytest.approx(kv_tail_scipy(5 / 3, y), rel=1e-11)
    # small-y behaviour: int_y^inf K_{5/3} -> (3/2) Gamma(5/3) 2^{2/3} y^{-2/3}
    y = 1e-12
    lead = 1.5 * special.gamma(5 / 3) * 2 ** (2 / 3) * y ** (-2 / 3)
    assert oracle.bessel_k_tail(5 / 3, y) == pytest.approx(lead, rel=1e-6)


def test_classical_spectrum_integral_closed_form():
    # int_0^inf y int_y^inf K_{5/3} dy = (1/2) int_0^inf t^2 K_{5/3}(t) dt = 8 pi / (9 sqrt 3)
    f = lambda y: y * oracle.bessel_k_tail(5 / 3, y)
    val = integrate.quad(f, 0, 1, epsrel=1e-12, limit=200)[0] + integrate.quad(f, 1, 60, epsrel=1e-12)[0]
    assert val == pytest.approx(8 * math.pi / (9 * math.sqrt(3)), rel=1e-10)


@pytest.mark.parametrize("eta,chi", [(1.0, 0.01), (1.0, 0.1), (1.0, 0.25), (1.0, 0.45), (0.01, 1e-5),
                                     (9.0, 1.0), (100.0, 49.0), (1e-4, 1e-9)])
def test_F_matches_independent_evaluation(eta, chi):
    assert oracle.F(eta, chi) == pytest.approx(F_scipy(eta, chi), rel=1e-11)


def test_F_vanishes_above_half_eta():
    # Appendix A: F = 0 for chi >= eta/2 (no photon carries more than the emitter's energy)
    assert oracle.F(1.0, 0.5) == 0.0
    assert oracle.F(1.0, 0.7) == 0.0
    assert oracle.F(1.0, 0.5 - 1e-6) >= 0.0


def test_F_classical_limit():
    # Appendix A: F -> y_c int_{y_c}^inf K_{5/3}, y_c = 4 chi / (3 eta^2), as hbar -> 0 (eta -> 0)
    eta = 1e-7
    for yc in [1e-3, 0.1, 1.0, 3.0]:
        chi = 0.75 * eta * eta * yc
        assert oracle.F(eta, chi) == pytest.approx(yc * kv_tail_scipy(5 / 3, yc), rel=1e-5)


def test_h_and_g_classical_limits():
    # h(eta -> 0) = int_0^inf t K_{5/3}(t) dt = 5 pi/3 ("h0 = 5.24", Sec. 3.1); g(0) = 1
    eta = 1e-6
    assert oracle.h(eta) == pytest.approx(H0, rel=2e-6)
    assert oracle.g(eta) == pytest.approx(1.0, rel=1e-5)
    assert round(H0, 2) == 5.24
    # first-order quantum corrections: 1 - g ~ (55 sqrt3/16) eta, 1 - h/h0 ~ (8/(5 sqrt3)) eta
    eta = 1e-5
    assert (1 - oracle.g(eta)) / eta == pytest.approx(55 * math.sqrt(3) / 16, rel=2e-4)
    assert (1 - oracle.h(eta) / H0) / eta == pytest.approx(8 / (5 * math.sqrt(3)), rel=2e-4)


def _h_g_scipy(eta):
    """h and g by nested adaptive quadrature of F_scipy over ln chi."""
    top = math.log(eta / 2)
    fh = lambda s: F_scipy(eta, math.exp(s))
    fg = lambda s: F_scipy(eta, math.exp(s)) * math.exp(s)
    pts = [top - 60, top - 20, top - 5, top - 1, top - 0.1, top - 1e-3, top]
    h = 3 * F_scipy(eta, math.exp(top - 60))
    e = 0.75 * math.exp(top - 60) * F_scipy(eta, math.exp(top - 60))
    for a, b in zip(pts[:-1], pts[1:]):
        h += integrate.quad(fh, a, b, epsrel=1e-11, limit=200)[0]
        e += integrate.quad(fg, a, b, epsrel=1e-11, limit=200)[0]
    return h, 3 * math.sqrt(3) / (2 * math.pi * eta * eta) * e


@pytest.mark.parametrize("eta", [0.1, 1.0, 9.0])
def test_h_and_g_match_independent_quadrature(eta):
    h, g = _h_g_scipy(eta)
    assert oracle.h(eta) == pytest.approx(h, rel=1e-8)
    assert oracle.g(eta) == pytest.approx(g, rel=1e-8)


def test_g_fit_and_g1():
    # Sec. 2.1: g ~ [1 + 4.8 (1 + eta) ln(1 + 1.7 eta) + 2.44 eta^2]^{-2/3}, and g(1) ~ 0.2
    for eta in np.logspace(-4, 2, 13):
        fit = (1 + 4.8 * (1 + eta) * math.log(1 + 1.7 * eta) + 2.44 * eta * eta) ** (-2 / 3)
        assert oracle.g(eta) == pytest.approx(fit, rel=0.015)
    assert abs(oracle.g(1.0) - 0.2) < 0.02


def test_cutoff_energy_fraction_independent():
    # Sec. 3: photons below chi_min carry 1e-9 of the spectrum's energy
    eta = 1.0
    chimin = oracle.cutoff_chi(eta, 1e-9)
    f = lambda s: F_scipy(eta, math.exp(s)) * math.exp(s)
    s0 = math.log(chimin) - 60
    below = 0.75 * math.exp(s0) * F_scipy(eta, math.exp(s0)) + integrate.quad(
        f, s0, math.log(chimin), epsrel=1e-11, limit=200)[0]
    _, g = _h_g_scipy(eta)
    total = g * 2 * math.pi * eta * eta / (3 * math.sqrt(3))
    assert below / total == pytest.approx(1e-9, rel=1e-7)


def test_pair_T_paper_statements():
    chi = np.logspace(-1, 2, 301)
    T = oracle.T(chi)
    k = int(np.argmax(T))
    # Sec. 3.1 footnote: Max(T_pm) = 0.2
    assert abs(T[k] - 0.2) < 0.01
    assert 4.0 < chi[k] < 9.0
    # Appendix B: T falls off as chi^{-1/3} at high chi; coefficient from K_{1/3}(z) ~ Gamma(1/3)/2 (2/z)^{1/3}
    c_hi = 0.04 * special.gamma(1 / 3) ** 2 * 3 ** (2 / 3)
    assert oracle.T(1e4) * 1e4 ** (1 / 3) == pytest.approx(c_hi, rel=0.01)
    # low chi: exponential suppression; with K_{1/3}(z) ~ sqrt(pi/2z) e^{-z} the formula gives
    # T ~ 0.12 pi exp(-4/(3 chi)) (the square of K doubles the exponent)
    for c in (0.01, 0.02):
        assert oracle.T(c) / (0.12 * math.pi * math.exp(-4 / (3 * c))) == pytest.approx(1.0, rel=0.02)


@pytest.mark.parametrize("chi", [0.1, 1.0, 10.0, 100.0])
def test_pair_split_normalisation_and_symmetry(chi):
    q = lambda f: (2 + f * (1 - f)) / (f * (1 - f)) * special.kv(2 / 3, 1 / (3 * chi * f * (1 - f)))
    k_ref = 2 * integrate.quad(q, 0, 0.5, epsrel=1e-12, limit=400, points=[1e-4, 1e-3, 1e-2, 0.1])[0]
    assert oracle.pair_k(chi) == pytest.approx(k_ref, rel=1e-10)
    for f in [0.01, 0.1, 0.3]:
        assert oracle.pf(f, chi) == pytest.approx(oracle.pf(1 - f, chi), rel=1e-12)
    total = 2 * integrate.quad(lambda f: oracle.pf(f, chi), 0, 0.5, epsrel=1e-10, limit=400,
                               points=[1e-4, 1e-3, 1e-2, 0.1])[0]
    assert total == pytest.approx(1.0, rel=1e-9)


def test_pair_split_limits():
    # Appendix B: peaked at f = 1/2 for chi << 1, at f -> 0, 1 for chi >> 1
    assert oracle.pf(0.5, 0.05) > 10 * oracle.pf(0.3, 0.05)
    assert oracle.pf(0.02, 1e3) > oracle.pf(0.5, 1e3)
    # chi >> 1/(f(1-f)): p_f ~ (2 + f(1-f)) / (f(1-f))^{1/3} up to normalisation
    shape = lambda f: (2 + f * (1 - f)) / (f * (1 - f)) ** (1 / 3)
    assert oracle.pf(0.1, 1e5) / oracle.pf(0.5, 1e5) == pytest.approx(shape(0.1) / shape(0.5), rel=0.01)
    # chi << 1: p_f ~ (2 + g) g^{-1/2} exp(-1/(3 chi g)) up to normalisation, g = f(1-f)
    lo = lambda f, c: (2 + f * (1 - f)) / math.sqrt(f * (1 - f)) * math.exp(-1 / (3 * c * f * (1 - f)))
    c = 0.01
    assert oracle.pf(0.45, c) / oracle.pf(0.5, c) == pytest.approx(lo(0.45, c) / lo(0.5, c), rel=0.01)


def test_philox_matches_numpy():
    # numpy's Philox (4x64, 10 rounds) increments its 256-bit counter before each block
    rng = np.random.default_rng(7)
    cases = [([0, 0, 0, 0], [1, 2]), ([2 ** 64 - 1, 5, 0, 0], [0, 0]), ([2 ** 64 - 1, 2 ** 64 - 1, 3, 0], [9, 2 ** 63])]
    for _ in range(20):
        cases.append((list(rng.integers(0, 2 ** 63, 4)), list(rng.integers(0, 2 ** 63, 2))))
    for ctr, key in cases:
        ctr = np.array(ctr, dtype=np.uint64)
        key = np.array(key, dtype=np.uint64)
        ref = np.random.Philox(counter=ctr, key=key).random_raw(4)
        # counter + 1 as a 256-bit little-endian integer
        c = [int(x) for x in ctr]
        v = (c[0] | c[1] << 64 | c[2] << 128 | c[3] << 192) + 1
        nxt = np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
        assert np.array_equal(oracle.philox(nxt, key), ref)


def test_gauss_legendre_matches_numpy():
    for n in (10, 16, 20):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(x, xr, rtol=0, atol=4e-15)
        np.testing.assert_allclose(w, wr, rtol=0, atol=4e-15)
