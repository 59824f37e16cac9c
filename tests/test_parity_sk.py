"""GPU parity of the s, p Slater-Koster orbital Hamiltonian and of the DOS and
VAC paths on it.

Builder: the same (orbital row, orbital column) pattern as the oracle, values
within 2e-15 (FP64 storage) or 1e-6 (FP32 storage) relative; Gershgorin
bounds; moments FP64 within 1e-10 of the row count, complex float DOS within
1e-4 relative L2; VAC moments FP64 within 1e-10 of the largest.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

V = (-5.7, 5.4, 6.2, -2.7)
ES, EP = -7.3, 0.0


def build(s, fmt, slice, reorder=True):
    return tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic, *V, ES, EP,
                                      fmt=fmt, slice=slice, reorder=reorder)


def oracle_csr(s):
    return O.sk_hamiltonian(s.pos, s.box, s.periodic, V, ES, EP)[0]


@pytest.mark.parametrize("fmt,slice", [("sell_f64", 16), ("sell_f32", 64), ("csr_f64", 1), ("sell_f64", 256)])
@pytest.mark.parametrize("reorder", [True, False])
def test_sk_builder_matches_oracle(fmt, slice, reorder):
    s = synth.graphene_sheet(9, 7, 0.08, 21)
    H = build(s, fmt, slice, reorder)
    assert H.st.n_rows == 4 * s.n and H.st.n_orb == 4
    csr = oracle_csr(s)
    rows, cols, vals, onsite = G.entries_in_atom_order(H)
    orow, ocol, oval = G.csr_entries(csr)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((ocol, orow))
    np.testing.assert_array_equal(rows[o1], orow[o2])
    np.testing.assert_array_equal(cols[o1], ocol[o2])
    tol = 1e-6 if fmt == "sell_f32" else 2e-15
    np.testing.assert_allclose(vals[o1], oval[o2], rtol=tol, atol=tol * np.abs(oval).max())
    odiag = csr.diag.astype(np.float32).astype(np.float64) if fmt == "sell_f32" else csr.diag
    np.testing.assert_array_equal(onsite, odiag)
    lo, hi = O.gershgorin(csr)
    assert H.bounds[0] == pytest.approx(lo, rel=1e-12)
    assert H.bounds[1] == pytest.approx(hi, rel=1e-12)


@pytest.mark.parametrize("R", [1, 4])
def test_sk_fp64_moments_and_c32_dos(R):
    s = synth.graphene_sheet(13, 11, 0.06, 4)
    csr = oracle_csr(s)
    H = build(s, "sell_f64", 32)
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(4 * s.n, R, 7)
    mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 96, "f64").cpu().numpy()
    mo, _ = O.kpm_moments(csr, a, b, r, 96)
    assert np.abs(mu - mo).max() <= 1e-10 * 4 * s.n
    H32 = build(s, "sell_f32", 64)
    r32 = synth.random_phase(4 * s.n, R, 7, np.complex64)
    m32 = tbkpm.kpm_moments(H32, a, b, G.to_dev(r32), 256, "c32").cpu().numpy()
    mo32, _ = O.kpm_moments(csr, a, b, r32.astype(np.complex128), 256)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(m32.mean(0), a, b, E), O.kpm_dos(mo32.mean(0), a, b, E)) <= 1e-4


def test_sk_vac_moments_match_oracle():
    s = synth.graphene_sheet(6, 5, 0.07, 9)
    csr = oracle_csr(s)
    H = build(s, "sell_f64", 16)
    a, b = G.oracle_ab(csr)
    vx = tbkpm.build_velocity(H, G.to_dev(s.pos), s.box, s.periodic, 1)
    rows, cols, vals, _ = G.entries_in_atom_order(H, vx)
    vo = O.velocity_values(csr, s.pos, s.box, s.periodic, 1, n_orb=4)
    orow, ocol, _ = G.csr_entries(csr)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((ocol, orow))
    np.testing.assert_allclose(vals[o1], vo[o2], rtol=1e-14, atol=1e-14 * np.abs(vo).max())
    r = synth.random_phase(4 * s.n, 2, 5)
    M, n_t, dt = 40, 3, 0.3
    nc = tbkpm.chebyshev_terms(a, dt)
    nu = tbkpm.vac_moments(H, vx, a, b, G.to_dev(r), M, n_t, dt).cpu().numpy()
    nuo = O.vac_moments(csr, vo, a, b, r, M, n_t, dt, nc)
    assert np.abs(nu - nuo).max() <= 1e-10 * np.abs(nuo).max()


def test_sk_errors():
    s = synth.graphene_sheet(4, 4)
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic, float("nan"), 1, 1, 1,
                                   0, 0, fmt="sell_f64", slice=8)
    assert e.value.name == "NOT_FINITE"
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic, *V, ES, EP,
                                   fmt="sell_f64", slice=3)
    assert e.value.name == "INVALID_ARG"


@pytest.mark.parametrize("vpt,tpb,nt,xr", [(1, 1, 1, 0), (2, 2, 0, 1), (2, 4, 1, 1)])
def test_sk_uniform_width_12_shapes(vpt, tpb, nt, xr):
    """Pristine periodic sheet: every orbital row has 12 entries (uniform slice width)."""
    s = synth.graphene_sheet(11, 10, 0.0, 1)
    csr = oracle_csr(s)
    H = build(s, "sell_f32", 64)
    assert H.st.max_degree == 12 and H.st.n_entries == 12 * 64 * (-(-4 * s.n // 64))   # slices of 64 rows
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(4 * s.n, 8, 3, np.complex64)
    mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 200, "c32", config=tbkpm.make_config(vpt, tpb, nt, xr, 1))
    mo, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), 200)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mu.cpu().numpy().mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4


@pytest.mark.parametrize("fmt,slice", [("bsell4_f64", 16), ("bsell4_f32", 32), ("bsell4_f64", 1)])
def test_block_builder_matches_oracle(fmt, slice):
    s = synth.graphene_sheet(9, 7, 0.08, 21)
    H = build(s, fmt, slice)
    assert H.st.n_rows == 4 * s.n and H.st.n_orb == 4 and H.st.max_degree == 3
    csr = oracle_csr(s)
    rows, cols, vals, onsite = G.block_entries(H)
    orow, ocol, oval = G.csr_entries(csr)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((ocol, orow))
    np.testing.assert_array_equal(rows[o1], orow[o2])
    np.testing.assert_array_equal(cols[o1], ocol[o2])
    tol = 1e-6 if fmt.endswith("f32") else 2e-15
    np.testing.assert_allclose(vals[o1], oval[o2], rtol=tol, atol=tol * np.abs(oval).max())
    lo, hi = O.gershgorin(csr)
    assert H.bounds[0] == pytest.approx(lo, rel=1e-12)
    assert H.bounds[1] == pytest.approx(hi, rel=1e-12)


@pytest.mark.parametrize("atom", [0, 1])
@pytest.mark.parametrize("R,tpb,nt,xr,dbl", [(1, 1, 1, 0, 0), (3, 2, 0, 1, 0), (16, 2, 1, 0, 1), (64, 1, 1, 1, 0),
                                             (1, 2, 1, 0, 1), (1, 3, 0, 1, 0)])
def test_block_fp64_moments(R, tpb, nt, xr, dbl, atom):
    s = synth.graphene_sheet(13, 11, 0.06, 4)        # 2288 orbital rows: ragged tiles
    csr = oracle_csr(s)
    H = build(s, "bsell4_f64", 32)
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(4 * s.n, R, 7)
    mo, _ = O.kpm_moments(csr, a, b, r, 61)
    for rows in ((2, 4) if atom else (1,)):   # atom form, one vector: staged rows and direct
        cfg = tbkpm.make_config(1, tpb, nt, xr, rows, doubling=dbl, atom_rows=atom)
        mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 61, "f64", config=cfg).cpu().numpy()
        assert np.abs(mu - mo).max() <= 1e-10 * 4 * s.n


@pytest.mark.parametrize("atom", [0, 1])
@pytest.mark.parametrize("R,vpt", [(2, 2), (16, 2), (8, 1), (32, 2)])
def test_block_c32_dos_and_scalar_agreement(R, vpt, atom):
    s = synth.graphene_sheet(12, 10, 0.05, 8)
    csr = oracle_csr(s)
    Hb = build(s, "bsell4_f32", 64)
    Hs = build(s, "sell_f32", 64)
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(4 * s.n, R, 3, np.complex64)
    cfg = tbkpm.make_config(vpt, 2, 1, 0, 1, atom_rows=atom)
    mb = tbkpm.kpm_moments(Hb, a, b, G.to_dev(r), 256, "c32", config=cfg).cpu().numpy()
    ms = tbkpm.kpm_moments(Hs, a, b, G.to_dev(r), 256, "c32", config=cfg).cpu().numpy()
    mo, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), 256)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mb.mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4
    assert np.abs(mb - ms).max() <= 1e-4 * 4 * s.n


def test_block_default_shape_is_atom_form():
    s = synth.graphene_sheet(5, 4, 0.03, 1)
    H = build(s, "bsell4_f32", 8)
    assert tbkpm.default_config(H, 8, "c32").atom_rows == 1
    Hs = build(s, "sell_f32", 8)
    assert tbkpm.default_config(Hs, 8, "c32").atom_rows == 0


def test_block_rejections():
    s = synth.graphene_sheet(5, 4, 0.03, 1)
    H = build(s, "bsell4_f64", 8)
    a, b = H.scale()
    r = G.to_dev(synth.random_phase(4 * s.n, 1, 2))
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.kpm_moments(H, a, b, r, 16, "f64", config=tbkpm.make_config(1, 2, 1, 0, 1, uniform_values=1))
    assert e.value.name == "INVALID_ARG"


@pytest.mark.parametrize("R", [1, 2])
@pytest.mark.parametrize("atom", [0, 1])
def test_block_vac_moments_match_oracle(atom, R):
    s = synth.graphene_sheet(6, 5, 0.07, 9)
    csr = oracle_csr(s)
    H = build(s, "bsell4_f64", 16)
    a, b = G.oracle_ab(csr)
    vx = tbkpm.build_velocity(H, G.to_dev(s.pos), s.box, s.periodic, 1)
    rows, cols, vals, _ = G.block_entries(H, vx)
    vo = O.velocity_values(csr, s.pos, s.box, s.periodic, 1, n_orb=4)
    orow, ocol, _ = G.csr_entries(csr)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((ocol, orow))
    np.testing.assert_allclose(vals[o1], vo[o2], rtol=1e-15, atol=1e-15 * np.abs(vo).max())
    r = synth.random_phase(4 * s.n, R, 5)
    M, n_t, dt = 40, 3, 0.3
    nc = tbkpm.chebyshev_terms(a, dt)
    nuo = O.vac_moments(csr, vo, a, b, r, M, n_t, dt, nc)
    # the row groupings, and launch shapes of the kind a block-shape search picks
    # (several tiles per block, XCD orders)
    cfgs = [tbkpm.make_config(1, 2, 1, 0, rows, atom_rows=atom) for rows in ((2, 4) if atom else (1,))]
    cfgs += [tbkpm.make_config(1, 1, 0, 2, 1, atom_rows=atom), tbkpm.make_config(1, 4, 1, 1, 1, atom_rows=atom)]
    for cfg in cfgs:
        nu = tbkpm.vac_moments(H, vx, a, b, G.to_dev(r), M, n_t, dt, config=cfg).cpu().numpy()
        assert np.abs(nu - nuo).max() <= 1e-10 * np.abs(nuo).max(), cfg.as_dict()


@pytest.mark.parametrize("slice_", [16, 32])
@pytest.mark.parametrize("atom", [0, 1])
def test_block_c32_vac_launch_shapes(atom, slice_):
    """C32 VAC on stored s, p blocks in the launch shapes a block-shape search picks from
    (two vectors per thread, tiles per block, XCD orders), against the FP64 oracle."""
    s = synth.graphene_sheet(12, 10, 0.05, 8)
    csr = oracle_csr(s)
    H = build(s, "bsell4_f32", slice_)
    a, b = G.oracle_ab(csr)
    vx = tbkpm.build_velocity(H, G.to_dev(s.pos), s.box, s.periodic, 0)
    vo = O.velocity_values(csr, s.pos, s.box, s.periodic, 0, n_orb=4)
    r = synth.random_phase(4 * s.n, 1, 6, np.complex64)
    M, n_t, dt = 64, 5, 0.3
    nc = tbkpm.chebyshev_terms(a, dt)
    nuo = O.vac_moments(csr, vo, a, b, r.astype(np.complex128), M, n_t, dt, nc)
    for cfg in (tbkpm.make_config(1, 2, 1, 0, 1, atom_rows=atom), tbkpm.make_config(2, 1, 0, 2, 1, atom_rows=atom),
                tbkpm.make_config(2, 4, 1, 1, 1, atom_rows=atom), tbkpm.make_config(2, 2, 0, 0, 1, atom_rows=atom)):
        nu = tbkpm.vac_moments(H, vx, a, b, G.to_dev(r), M, n_t, dt, nc, "c32", config=cfg).cpu().numpy()
        assert np.abs(nu - nuo).max() <= 1e-4 * np.abs(nuo).max(), cfg.as_dict()
