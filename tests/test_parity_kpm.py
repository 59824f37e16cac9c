"""GPU parity of the Hamiltonian builder, the Chebyshev moments and the DOS
against the serial FP64 oracle, through the C ABI.

Tolerances: FP64 moments |mu_gpu - mu_oracle| <= 1e-10 mu_0 (rounding-order
differences only); complex-float recurrence: DOS relative L2 <= 1e-4; builder:
identical sparsity pattern (bit-exact), values within 2e-15 relative (exp and
sqrt may differ by an ulp between the host and device libraries).
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def oracle_setup(s):
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    return csr


@pytest.mark.parametrize("name,kw", [
    ("pristine_3x3", dict(nx=3, ny=3, sigma=0.0)),
    ("displaced_7x5", dict(nx=7, ny=5, sigma=0.08)),
    ("displaced_40x33", dict(nx=40, ny=33, sigma=0.05)),
])
@pytest.mark.parametrize("fmt,slice", [("csr_f64", 1), ("sell_f64", 64), ("sell_f32", 256),
                                       ("sell_f64", 8)])
@pytest.mark.parametrize("reorder", [True, False])
def test_builder_matches_oracle(name, kw, fmt, slice, reorder):
    s = synth.graphene_sheet(kw["nx"], kw["ny"], kw["sigma"], 17)
    H = G.build(s, fmt=fmt, slice=slice, reorder=reorder)
    csr = oracle_setup(s)
    rows, cols, vals, onsite = G.entries_in_atom_order(H)
    orow, ocol, oval = G.csr_entries(csr)
    o1 = np.lexsort((cols, rows))
    o2 = np.lexsort((ocol, orow))
    np.testing.assert_array_equal(rows[o1], orow[o2])
    np.testing.assert_array_equal(cols[o1], ocol[o2])
    tol = 1e-6 if fmt == "sell_f32" else 2e-15
    np.testing.assert_allclose(vals[o1], oval[o2], rtol=tol)
    np.testing.assert_array_equal(onsite, csr.diag)
    lo, hi = O.gershgorin(csr)
    assert H.bounds[0] == pytest.approx(lo, rel=1e-14)
    assert H.bounds[1] == pytest.approx(hi, rel=1e-14)
    assert H.st.n_bonds == len(orow) // 2
    assert H.st.max_degree == np.diff(csr.row_ptr).max()
    perm = H.perm.cpu().numpy()
    np.testing.assert_array_equal(np.sort(perm), np.arange(s.n))
    if not reorder:
        np.testing.assert_array_equal(perm, np.arange(s.n))


def test_builder_stripes_species_and_onsite():
    s = synth.hbn_stripes(12, 9, stripe_cells=3, sigma=0.03, seed=5)
    H = G.build(s, fmt="sell_f64", slice=32)
    csr = oracle_setup(s)
    rows, cols, vals, onsite = G.entries_in_atom_order(H)
    orow, ocol, oval = G.csr_entries(csr)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((ocol, orow))
    np.testing.assert_array_equal(cols[o1], ocol[o2])
    np.testing.assert_allclose(vals[o1], oval[o2], rtol=2e-15)
    np.testing.assert_array_equal(onsite, csr.diag)
    assert H.st.has_onsite == 1


def _moments_pair(s, fmt, slice, R, M, precision, a=None, b=None, seed=3, reorder=True):
    H = G.build(s, fmt=fmt, slice=slice, reorder=reorder)
    csr = oracle_setup(s)
    if a is None:
        lo, hi = O.gershgorin(csr)
        a, b = 1.01 * (hi - lo) / 2, (hi + lo) / 2
    cdt = np.complex64 if precision == "c32" else np.complex128
    r = synth.random_phase(s.n, R, seed, cdt)
    mu_gpu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), M, precision).cpu().numpy()
    mu_orc, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), M)
    return mu_gpu, mu_orc, a, b


def test_c1_moments_and_dos_fp64():
    """2304-atom pristine sheet, CSR FP64, a = 9 eV, b = 0, M = 256, R = 4."""
    w = synth.WORKLOADS["graphene_pristine_2304"]
    s = synth.graphene_sheet(w["nx"], w["ny"])
    mu_g, mu_o, a, b = _moments_pair(s, "csr_f64", 1, w["R"], w["M"], "f64", a=w["a"], b=w["b"],
                                     seed=w["seed"] + synth.VECTOR_SEED_OFFSET)
    assert np.abs(mu_g - mu_o).max() <= 1e-10 * s.n
    E = np.linspace(w["e_lo"], w["e_hi"], w["n_e"])
    rho_g = tbkpm.kpm_dos(G.to_dev(mu_g.mean(0)), a, b, G.to_dev(E)).cpu().numpy()
    rho_o = O.kpm_dos(mu_o.mean(0), a, b, E)
    assert G.rel_l2(rho_g, rho_o) < 1e-12


@pytest.mark.parametrize("R", [1, 3, 4, 8, 16])
@pytest.mark.parametrize("fmt,slice", [("sell_f64", 1), ("sell_f64", 32), ("csr_f64", 1)])
def test_fp64_moments_ragged(R, fmt, slice):
    s = synth.graphene_sheet(23, 17, 0.06, 29)          # 1564 rows: ragged against every tile
    mu_g, mu_o, _, _ = _moments_pair(s, fmt, slice, R, 97, "f64")
    assert np.abs(mu_g - mu_o).max() <= 1e-10 * s.n


@pytest.mark.parametrize("R", [1, 2, 5, 16, 32])
@pytest.mark.parametrize("slice", [8, 64, 256])
def test_c32_dos_within_1e_4(R, slice):
    s = synth.graphene_sheet(31, 29, 0.05, 41)
    M = 300
    mu_g, mu_o, a, b = _moments_pair(s, "sell_f32", slice, R, M, "c32")
    E = synth.energy_grid(a, b)
    rho_g = O.kpm_dos(mu_g.mean(0), a, b, E)
    rho_o = O.kpm_dos(mu_o.mean(0), a, b, E)
    assert G.rel_l2(rho_g, rho_o) <= 1e-4
    assert np.abs(mu_g - mu_o).max() <= 1e-4 * s.n


def test_stripes_onsite_shift_fp64_and_c32():
    s = synth.hbn_stripes(20, 18, stripe_cells=4, sigma=0.03, seed=6)
    mu_g, mu_o, a, b = _moments_pair(s, "sell_f64", 16, 4, 128, "f64")
    assert b != 0.0
    assert np.abs(mu_g - mu_o).max() <= 1e-10 * s.n
    mu_g, mu_o, a, b = _moments_pair(s, "sell_f32", 64, 4, 128, "c32")
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mu_g.mean(0), a, b, E), O.kpm_dos(mu_o.mean(0), a, b, E)) <= 1e-4


def test_reorder_does_not_change_moments():
    s = synth.graphene_sheet(15, 14, 0.05, 8)
    m1, mo, _, _ = _moments_pair(s, "sell_f64", 64, 4, 64, "f64", reorder=True)
    m0, _, _, _ = _moments_pair(s, "sell_f64", 64, 4, 64, "f64", reorder=False)
    assert np.abs(m1 - m0).max() <= 1e-10 * s.n


def test_bitwise_reproducible():
    s = synth.graphene_sheet(30, 30, 0.05, 9)
    H = G.build(s, fmt="sell_f32", slice=256)
    a, b = H.scale()
    r = G.to_dev(synth.random_phase(s.n, 8, 1, np.complex64))
    m1 = tbkpm.kpm_moments(H, a, b, r, 200).cpu().numpy()
    m2 = tbkpm.kpm_moments(H, a, b, r, 200).cpu().numpy()
    np.testing.assert_array_equal(m1, m2)


def test_spectrum_guard_raises():
    s = synth.graphene_sheet(10, 10, 0.05, 4)
    H = G.build(s, fmt="sell_f64", slice=64)
    a, b = H.scale()
    r = G.to_dev(synth.random_phase(s.n, 1, 2))
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.kpm_moments(H, 0.5 * a, b, r, 128)
    assert e.value.name == "SPECTRUM"


def test_error_statuses():
    s = synth.graphene_sheet(4, 4)
    pos = s.pos.copy()
    pos[5, 0] = np.nan
    bad = synth.Structure(pos=pos, species=s.species, box=s.box, periodic=s.periodic)
    with pytest.raises(tbkpm.TBKError) as e:
        G.build(bad)
    assert e.value.name == "NOT_FINITE"
    small = synth.graphene_sheet(2, 1)            # periodic y length 2.46 < 2 r_cut
    with pytest.raises(tbkpm.TBKError) as e:
        G.build(small)
    assert e.value.name == "INVALID_ARG"
    sp = s.species.copy()
    sp[0] = 3
    with pytest.raises(tbkpm.TBKError) as e:
        G.build(synth.Structure(pos=s.pos, species=sp, box=s.box, periodic=s.periodic))
    assert e.value.name == "INVALID_ARG"
    H = G.build(s, fmt="sell_f64", slice=64)
    r = G.to_dev(synth.random_phase(s.n, 2, 2))
    work = torch.empty(64, dtype=torch.uint8, device=G.DEV)
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.kpm_moments(H, 9.0, 0.0, r, 16, work=work)
    assert e.value.name == "BUFFER_TOO_SMALL"
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.kpm_moments(H, 9.0, 0.0, r.to(torch.complex64), 16)     # float vectors, double H
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.kpm_moments(H, -1.0, 0.0, r, 16)
    assert e.value.name == "INVALID_ARG"


def test_single_atom_and_isolated_rows():
    """Open boundaries far apart: every row has degree 0 (H = onsite), a 1x1 case too."""
    pos = np.array([[1.0, 1.0, 1.0], [10.0, 1.0, 1.0], [1.0, 10.0, 1.0]])
    s = synth.Structure(pos=pos, species=np.array([0, 1, 2], np.int32), box=np.array([0., 0., 0.]),
                        periodic=np.array([0, 0, 0], np.int32), onsite=synth.ONSITE_EV,
                        t_pair=synth.T_PAIR_EV)
    H = G.build(s, fmt="sell_f64", slice=4)
    assert H.st.n_entries == 0 and H.st.max_degree == 0
    a, b = 3.0, 0.1
    r = synth.random_phase(3, 2, 5)
    mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 40).cpu().numpy()
    x = (synth.ONSITE_EV - b) / a
    expect = np.cos(np.arange(40)[:, None] * np.arccos(x)[None, :]).sum(1)
    np.testing.assert_allclose(mu, np.broadcast_to(expect, (2, 40)), atol=1e-12)
    one = synth.Structure(pos=pos[:1], species=np.array([1], np.int32), box=np.zeros(3),
                          periodic=np.array([0, 0, 0], np.int32), onsite=synth.ONSITE_EV,
                          t_pair=synth.T_PAIR_EV)
    H1 = G.build(one, fmt="csr_f64")
    mu1 = tbkpm.kpm_moments(H1, a, b, G.to_dev(synth.random_phase(1, 1, 1)), 10).cpu().numpy()
    np.testing.assert_allclose(mu1[0], np.cos(np.arange(10) * math.acos((2.3 - b) / a)), atol=1e-14)


def test_dos_kernel_matches_oracle_on_device():
    mu = np.random.default_rng(3).normal(size=500) * np.exp(-np.arange(500) / 80.0)
    mu[0] = 1.0
    E = np.linspace(-3.2, 3.2, 777)
    for kernel in (0, 1):
        rho_g = tbkpm.kpm_dos(G.to_dev(mu), 3.0, 0.1, G.to_dev(E), kernel=kernel).cpu().numpy()
        rho_o = O.kpm_dos(mu, 3.0, 0.1, E, kernel=kernel)
        np.testing.assert_allclose(rho_g, rho_o, rtol=1e-11, atol=1e-13)
