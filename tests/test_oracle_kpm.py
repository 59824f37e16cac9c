"""Pins of the oracle's Chebyshev moments (CPU only).

Sec. 2.4 names Chebyshev expansion, KPM and random phases; the moments are
mu_n = <r|T_n(Htilde)|r>, Htilde = (H - b)/a, T_{n+1} = 2 Htilde T_n - T_{n-1}.
Full traces are obtained by using the N unit vectors as the "random" vectors.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_06525_amd import synth
from tests import ref_numpy as ref


def full_trace(csr, a, b, M):
    n = csr.n
    mu_re, mu_im = O.kpm_moments(csr, a, b, np.eye(n, dtype=np.complex128), M)
    return mu_re.sum(axis=0), mu_im


def ring(n, t=-2.7):
    pos = np.zeros((n, 3))
    pos[:, 0] = np.arange(n) * synth.R0
    pos[:, 1:] = 5.0
    box = np.array([n * synth.R0, 10.0, 10.0])
    return O.hamiltonian(pos, np.zeros(n, np.int32), box, np.array([1, 0, 0], np.int32),
                         [0.0], [[t]], r_cut=2.0)[0]


@pytest.mark.parametrize("n", [7, 8, 12])
def test_ring_closed_form(n):
    """Ring of n sites, a = 2|t|: Tr T_m = (-1)^m n when n | m, else 0."""
    csr = ring(n)
    M = 3 * n + 2
    tr, im = full_trace(csr, 5.4, 0.0, M)
    m = np.arange(M)
    expect = np.where(m % n == 0, (-1.0) ** m * n, 0.0)
    np.testing.assert_allclose(tr, expect, atol=1e-10)
    assert np.abs(im).max() < 1e-12


@pytest.mark.parametrize("nx,ny,sigma,kind", [(2, 2, 0.0, "sheet"), (3, 2, 0.1, "sheet"),
                                              (4, 3, 0.05, "stripes")])
def test_moments_match_dense_spectrum(nx, ny, sigma, kind):
    if kind == "sheet":
        s = synth.graphene_sheet(nx, ny, sigma, 11)
    else:
        s = synth.hbn_stripes(nx, ny, stripe_cells=2, sigma=sigma, seed=12)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    lo, hi = O.gershgorin(csr)
    a, b = 1.01 * (hi - lo) / 2, (hi + lo) / 2
    M = 64
    tr, _ = full_trace(csr, a, b, M)
    eig = np.linalg.eigvalsh(csr.dense())
    expect = ref.trace_moments_from_eigs(eig, a, b, M)
    np.testing.assert_allclose(tr, expect, atol=1e-12 * s.n)


def test_c1_full_trace_equals_bloch_sum():
    """2304-atom pristine sheet, a = 9 eV: full trace vs the 4x4 Bloch k-sum spectrum."""
    w = synth.WORKLOADS["graphene_pristine_2304"]
    s = synth.graphene_sheet(w["nx"], w["ny"])
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    M = 48
    tr, _ = full_trace(csr, 9.0, 0.0, M)
    eig = ref.supercell_spectrum(w["nx"], w["ny"])
    assert eig.size == s.n
    np.testing.assert_allclose(np.sort(eig), np.sort(np.linalg.eigvalsh(csr.dense())), atol=1e-12)
    expect = ref.trace_moments_from_eigs(eig, 9.0, 0.0, M)
    np.testing.assert_allclose(tr, expect, atol=1e-11 * s.n)
    # closed forms: mu_0 = N, mu_2/N = 2 (3 t^2/a^2) - 1, mu_4/N from 15 closed 4-walks
    assert tr[0] == pytest.approx(s.n, abs=1e-9)
    assert tr[2] / s.n == pytest.approx(-0.46, abs=1e-13)
    assert tr[4] / s.n == pytest.approx(-0.188, abs=1e-13)
    np.testing.assert_allclose(tr[1::2], 0.0, atol=1e-9)    # bipartite: odd traces vanish


def test_random_phase_estimate_within_statistical_bound():
    """|mean_v mu_n^(v) - Tr T_n| / N <= 5 / sqrt(N R) (Var <r|A|r> <= N for |A_ij| <= 1)."""
    s = synth.graphene_sheet(12, 12, 0.05, 5)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    lo, hi = O.gershgorin(csr)
    a, b = 1.01 * (hi - lo) / 2, (hi + lo) / 2
    R, M = 4, 40
    r = synth.random_phase(s.n, R, 21)
    mu, im = O.kpm_moments(csr, a, b, r, M)
    eig = np.linalg.eigvalsh(csr.dense())
    exact = ref.trace_moments_from_eigs(eig, a, b, M)
    assert np.all(np.abs(mu.mean(0) - exact) / s.n <= 5.0 / math.sqrt(s.n * R))
    np.testing.assert_allclose(mu[:, 0], s.n, rtol=1e-14)          # mu_0 = sum |r_i|^2
    assert np.all(np.abs(mu) <= mu[:, :1] * (1 + 1e-12))           # spectrum guard holds
    # Hermitian H: <r|T_n|r> is real up to rounding
    assert np.abs(im).max() < 1e-9 * s.n


def test_moments_independent_per_vector_and_linear_in_phase():
    """Each vector's moments depend only on that vector; a global phase drops out."""
    s = synth.graphene_sheet(5, 5, 0.05, 8)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    r = synth.random_phase(s.n, 3, 9)
    mu3, _ = O.kpm_moments(csr, 9.0, 0.1, r, 20)
    mu1, _ = O.kpm_moments(csr, 9.0, 0.1, np.ascontiguousarray(r[:, 1:2] * np.exp(0.7j)), 20)
    np.testing.assert_allclose(mu3[1], mu1[0], rtol=1e-12, atol=1e-12)


def test_guard_violated_when_scale_too_small():
    """With a below the spectral radius the recurrence leaves [-mu_0, mu_0]."""
    s = synth.graphene_sheet(4, 4, 0.05, 4)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    lo, hi = O.gershgorin(csr)
    a = 0.5 * (hi - lo) / 2
    mu, _ = O.kpm_moments(csr, a, 0.0, synth.random_phase(s.n, 1, 3), 64)
    assert np.abs(mu).max() > mu[0, 0] * 10


@pytest.mark.parametrize("split", [(2,), (37,), (2, 3, 50, 99), (98,)])
def test_split_run_equals_one_shot_exactly(split):
    """Checkpoint/resume of the recurrence (Sec. 2.4's Chebyshev expansion, continued
    from its last two vectors): a run split at any k repeats the one-shot run's
    operations, so every moment is bit for bit the one-shot moment."""
    s = synth.graphene_sheet(5, 4, 0.05, 21)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    lo, hi = O.gershgorin(csr)
    a, b = 1.01 * (hi - lo) / 2, (hi + lo) / 2 + 0.1
    r = synth.random_phase(s.n, 3, 5, np.complex128)
    M = 100
    re1, im1 = O.kpm_moments(csr, a, b, r, M)
    stops = list(split) + [M]
    re2, im2, state = O.kpm_moments_state(csr, a, b, r, stops[0])
    mu_re, mu_im = np.full((3, M), np.nan), np.full((3, M), np.nan)
    mu_re[:, :stops[0]], mu_im[:, :stops[0]] = re2, im2
    for k0, k1 in zip(stops[:-1], stops[1:]):
        part_re, part_im = np.full((3, k1), np.nan), np.full((3, k1), np.nan)
        O.kpm_moments_state(csr, a, b, r, k1, n_start=k0, state=state, mu_re=part_re, mu_im=part_im)
        assert np.isnan(part_re[:, :k0]).all()          # nothing below n_start is written
        mu_re[:, k0:k1], mu_im[:, k0:k1] = part_re[:, k0:], part_im[:, k0:]
    np.testing.assert_array_equal(mu_re, re1)
    np.testing.assert_array_equal(mu_im, im1)


def test_split_run_keeps_the_ring_closed_form():
    """The continued recurrence still gives Tr T_m = (-1)^m n for n | m on a ring
    (a pin of the continuation that does not go through the one-shot routine)."""
    n = 9
    csr = ring(n)
    eye = np.eye(n, dtype=np.complex128)
    M = 3 * n + 2
    re, _, st = O.kpm_moments_state(csr, 5.4, 0.0, eye, 10)
    full = np.full((n, M), np.nan)
    full[:, :10] = re
    O.kpm_moments_state(csr, 5.4, 0.0, eye, M, n_start=10, state=st, mu_re=full, mu_im=np.empty((n, M)))
    m = np.arange(M)
    expect = np.where(m % n == 0, (-1.0) ** m * n, 0.0)
    np.testing.assert_allclose(full.sum(axis=0), expect, atol=1e-10)


def test_split_run_rejects_bad_starts():
    s = synth.graphene_sheet(2, 2)
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    r = np.ones((s.n, 1), np.complex128)
    st = np.zeros((1, 2, s.n), np.complex128)
    for k in (1, 10, 11, -1):
        with pytest.raises(O.OracleError):
            O.kpm_moments_state(csr, 9.0, 0.0, r, 10, n_start=k, state=st)
