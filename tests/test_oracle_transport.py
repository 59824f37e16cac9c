"""Pins of the oracle's transport post-processing: the integrated DOS against the
DOS it integrates (derivative and quadrature), the band edges and the level count of
a ring; the frame average, plateau and unit factor of the mobility against SI
arithmetic."""
import numpy as np
import pytest
from scipy import constants, integrate

from oracle import oracle as O


def exact_moments(eps, a, b, M):
    """mu_n = sum_k T_n((eps_k - b)/a) (the exact trace of T_n)."""
    x = (np.asarray(eps) - b) / a
    return np.cos(np.arange(M)[:, None] * np.arccos(x)[None, :]).sum(axis=1)


def ring_levels(n, t=-1.0):
    return 2.0 * t * np.cos(2.0 * np.pi * np.arange(n) / n)


def test_edges_and_total():
    rng = np.random.default_rng(3)
    eps = rng.uniform(-2.0, 2.0, 40)
    a, b = 2.6, 0.1
    mu = exact_moments(eps, a, b, 300)
    N = O.integrated_dos(mu, a, b, np.array([b - a, b - 2 * a, b + a, b + 3 * a]))
    assert N[0] == 0.0 and N[1] == 0.0
    assert N[2] == pytest.approx(40.0, abs=1e-12) and N[3] == N[2]


@pytest.mark.parametrize("kernel", [0, 1])
def test_derivative_is_the_dos(kernel):
    rng = np.random.default_rng(5)
    eps = rng.normal(0.0, 0.8, 60)
    a, b = 4.0, 0.0
    mu = exact_moments(eps, a, b, 128)
    E = np.linspace(-3.5, 3.5, 41)
    h = 1e-5
    dN = (O.integrated_dos(mu, a, b, E + h, kernel) - O.integrated_dos(mu, a, b, E - h, kernel)) / (2 * h)
    rho = O.kpm_dos(mu, a, b, E, kernel)
    assert np.abs(dN - rho).max() <= 1e-6 * np.abs(rho).max()


def test_quadrature_of_the_dos():
    rng = np.random.default_rng(8)
    eps = rng.uniform(-1.5, 1.5, 25)
    a, b = 2.0, 0.0
    mu = exact_moments(eps, a, b, 200)
    lo, hi = -1.2, 0.9
    q, _ = integrate.quad(lambda e: O.kpm_dos(mu, a, b, np.array([e]))[0], lo, hi, limit=400,
                          epsabs=1e-11, epsrel=1e-11)
    N = O.integrated_dos(mu, a, b, np.array([lo, hi]))
    assert N[1] - N[0] == pytest.approx(q, abs=1e-8)


def test_ring_level_count():
    """Between the levels of an 8-site ring, N counts the levels below (Jackson width
    ~ pi a / M = 0.002 eV against gaps of 0.6 eV)."""
    a, b = 2.5, 0.0
    mu = exact_moments(ring_levels(8), a, b, 4000)
    E = np.array([-1.707, -0.707, 0.707, 1.707, -2.3, 2.3])
    N = O.integrated_dos(mu, a, b, E)
    np.testing.assert_allclose(N, [1, 3, 5, 7, 0, 8], atol=1e-6)


def test_mobility_plateau_frame_mean_and_nan():
    # frame 0 peaks at t1, frame 1 at t2: the plateau of the mean differs from the mean of the maxima
    sigma = np.zeros((2, 3, 3))
    sigma[0, :, 0] = [0.0, 4.0, 1.0]
    sigma[1, :, 0] = [0.0, 0.0, 5.0]
    sigma[:, :, 1] = [[0.0, 1.0, 2.0], [0.0, 1.0, 2.0]]
    sigma[:, :, 2] = 3.0
    N = np.array([[10.0, 12.0, 7.0], [12.0, 12.0, 9.0]])
    ssc, car, mob = O.mobility(sigma, N, 8.0)
    np.testing.assert_allclose(ssc, [3.0, 2.0, 3.0])       # max_t of (4, 1 | 0, 5) mean = (2, 3) -> 3
    np.testing.assert_allclose(car, [3.0, 4.0, 0.0])
    np.testing.assert_allclose(mob[:2], [0.1 * 3.0 / 3.0, 0.1 * 2.0 / 4.0])
    assert np.isnan(mob[2])


def test_mobility_unit_factor_against_si():
    """sigma = (2 e^2 / A) X and n = 2 c / A; mu = sigma / (e n) in SI, converted to cm^2/(V s)."""
    X = 37.5          # Angstrom^2 / (eV fs): the running conductivity without 2 e^2 / A
    c = 1234.0        # carriers (states, no spin)
    A = 2.6e6         # area, Angstrom^2
    e = constants.e
    x_si = X * 1e-20 / (e * 1e-15)                 # m^2 / (J s)
    sig = 2.0 * e * e * x_si / (A * 1e-20)          # S (sheet)
    n = 2.0 * c / (A * 1e-20)                       # 1 / m^2
    mu_cm2 = sig / (e * n) * 1e4
    _, _, mob = O.mobility(np.full((1, 1, 1), X), np.array([[c + 10.0]]), 10.0)
    assert mob[0] == pytest.approx(mu_cm2, rel=1e-12)
