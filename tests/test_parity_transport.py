"""GPU parity of the transport post-processing: the integrated DOS (closed form,
FP64) against the oracle's within 1e-11 of mu_0, including the band edges and
ragged energy counts; the frame-averaged plateau conductivity, carriers and
mobility bit for bit where defined (same sums in the same order), NaN where the
carriers vanish; and the whole multi-frame workflow (Hamiltonian, velocity,
correlation moments, running conductivity, DOS moments, integrated DOS,
mobility; FP64) against the oracle chain on the same frames and vectors."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def exact_moments(eps, a, b, M):
    x = (np.asarray(eps) - b) / a
    return np.cos(np.arange(M)[:, None] * np.arccos(x)[None, :]).sum(axis=1)


@pytest.mark.parametrize("M,nE,kernel", [(1, 5, 0), (37, 300, 0), (300, 257, 1), (1000, 2001, 0), (3000, 513, 0)])
def test_integrated_dos_matches_oracle(M, nE, kernel):
    rng = np.random.default_rng(M)
    eps = rng.uniform(-2.0, 2.0, 50)
    a, b = 2.3, 0.05
    mu = exact_moments(eps, a, b, M)
    E = np.concatenate([np.linspace(b - 1.2 * a, b + 1.2 * a, nE - 2), [b - a, b + a]])
    N = tbkpm.integrated_dos(G.to_dev(mu), a, b, G.to_dev(E), kernel).cpu().numpy()
    No = O.integrated_dos(mu, a, b, E, kernel)
    assert np.abs(N - No).max() <= 1e-11 * mu[0]
    assert N[-2] == 0.0 and N[-1] == mu[0]


def test_mobility_matches_oracle():
    rng = np.random.default_rng(4)
    F, n_t, nE = 3, 17, 300
    sigma = rng.uniform(0.0, 5.0, (F, n_t, nE))
    N = rng.uniform(0.0, 100.0, (F, nE))
    N[:, 7] = 40.0                                     # carriers exactly 0 at energy 7
    ssc, car, mob = (x.cpu().numpy() for x in tbkpm.mobility(G.to_dev(sigma), G.to_dev(N), 40.0))
    so, co, mo = O.mobility(sigma, N, 40.0)
    np.testing.assert_array_equal(ssc, so)
    np.testing.assert_array_equal(car, co)
    np.testing.assert_array_equal(mob, mo)               # NaN at the same place
    assert np.isnan(mob[7])


def test_errors():
    mu = G.to_dev(np.ones(8))
    E = G.to_dev(np.zeros(4))
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.integrated_dos(mu, -1.0, 0.0, E)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.mobility(G.to_dev(np.zeros((1, 2, 3))), G.to_dev(np.zeros((1, 3))), float("nan"))
    assert e.value.name == "NOT_FINITE"


def test_multi_frame_workflow_matches_oracle():
    F, M, n_t, dt, R, R_dos = 2, 40, 4, 0.4, 2, 3
    frames = [synth.graphene_sheet(6, 5, 0.06, 50 + f) for f in range(F)]
    n = frames[0].n
    r = synth.random_phase(n, R, 9)
    rd = synth.random_phase(n, R_dos, 10)
    Hs, scales = [], []
    for s in frames:
        Hs.append(G.build(s, fmt="sell_f64", slice=16))
        scales.append(G.oracle_ab_of(s))
    lo = max(b - 0.99 * a for a, b in scales)
    hi = min(b + 0.99 * a for a, b in scales)
    E = np.linspace(lo, hi, 301)
    nc = tbkpm.chebyshev_terms(max(a for a, _ in scales), dt)
    sig_g, n_g, sig_o, n_o = [], [], [], []
    for s, H, (a, b) in zip(frames, Hs, scales):
        vx = tbkpm.build_velocity(H, G.to_dev(s.pos), s.box, s.periodic, 0)
        nu = tbkpm.vac_moments(H, vx, a, b, G.to_dev(r), M, n_t, dt, nc)
        sig_g.append(tbkpm.vac_sigma(nu.mean(1).contiguous(), a, b, dt, G.to_dev(E)))
        mu = tbkpm.kpm_moments(H, a, b, G.to_dev(rd), M, "f64")
        n_g.append(tbkpm.integrated_dos(mu.mean(0).contiguous(), a, b, G.to_dev(E)))
        csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
        vo = O.velocity_values(csr, s.pos, s.box, s.periodic, 0)
        nuo = O.vac_moments(csr, vo, a, b, r, M, n_t, dt, nc)
        sig_o.append(O.vac_sigma(nuo.mean(1), a, b, dt, E))
        mo, _ = O.kpm_moments(csr, a, b, rd, M)
        n_o.append(O.integrated_dos(mo.mean(0), a, b, E))
    ssc, car, mob = (x.cpu().numpy() for x in tbkpm.mobility(torch.stack(sig_g), torch.stack(n_g), 0.5 * n))
    so, co, mo = O.mobility(np.stack(sig_o), np.stack(n_o), 0.5 * n)
    assert np.abs(ssc - so).max() <= 1e-9 * np.abs(so).max()
    assert np.abs(car - co).max() <= 1e-9 * n
    ok = np.abs(co) > 1e-2 * n
    assert ok.sum() > 100
    np.testing.assert_allclose(mob[ok], mo[ok], rtol=1e-6)
