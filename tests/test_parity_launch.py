"""GPU parity of every recurrence launch shape and of the autotuner's choice.

Each shape computes the same T_n; moments may differ only in the order of the
double partial sums, so shapes agree to 1e-12 mu_0 and each matches the oracle
to the FP64 bar (1e-10 mu_0).  Structures with irregular degrees (strong
displacements) exercise the general-width path; ragged row counts exercise
the clamped tail.
"""
import itertools

import numpy as np
import torch
import pytest

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

SHAPES = [tbkpm.make_config(1, tpb, nt, xr, rpt)
          for tpb, nt, xr, rpt in itertools.product([1, 2, 3], [0, 1], [0, 1, 2, 3], [1, 2]) if rpt <= tpb]


def _oracle_mu(s, a, b, r, M):
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    return O.kpm_moments(csr, a, b, r.astype(np.complex128), M)[0]


@pytest.mark.parametrize("sigma,slice", [(0.0, 64), (0.05, 256), (0.15, 32), (0.15, 1)])
@pytest.mark.parametrize("R", [1, 4])
def test_fp64_every_shape_matches_oracle(sigma, slice, R):
    s = synth.graphene_sheet(19, 13, sigma, 77)          # 988 rows
    H = G.build(s, fmt="sell_f64", slice=slice)
    if sigma == 0.15:
        assert H.st.max_degree > 3                         # irregular widths
    a, b = G.oracle_ab_of(s)
    M = 48
    r = synth.random_phase(s.n, R, 4)
    mu_o = _oracle_mu(s, a, b, r, M)
    rd = G.to_dev(r)
    first = None
    for cfg in SHAPES:
        mu = tbkpm.kpm_moments(H, a, b, rd, M, "f64", config=cfg).cpu().numpy()
        assert np.abs(mu - mu_o).max() <= 1e-10 * s.n, cfg.as_dict()
        if first is None:
            first = mu
        assert np.abs(mu - first).max() <= 1e-12 * s.n, cfg.as_dict()


@pytest.mark.parametrize("R,vpt", [(1, 1), (2, 2), (8, 1), (8, 2), (32, 2)])
def test_c32_shapes_agree(R, vpt):
    s = synth.hbn_stripes(22, 15, stripe_cells=5, sigma=0.12, seed=3)
    H = G.build(s, fmt="sell_f32", slice=16)
    a, b = G.oracle_ab_of(s)
    M = 64
    r = synth.random_phase(s.n, R, 9, np.complex64)
    mu_o = _oracle_mu(s, a, b, r, M)
    rd = G.to_dev(r)
    base = None
    for tpb, nt, xr, rpt in [(1, 1, 1, 1), (2, 0, 0, 2), (3, 1, 0, 2), (4, 0, 1, 1), (2, 1, 2, 2), (1, 0, 3, 1)]:
        cfg = tbkpm.make_config(vpt, tpb, nt, xr, rpt)
        mu = tbkpm.kpm_moments(H, a, b, rd, M, "c32", config=cfg).cpu().numpy()
        assert np.abs(mu - mu_o).max() <= 1e-4 * s.n
        if base is None:
            base = mu
        assert np.abs(mu - base).max() <= 1e-12 * s.n


@pytest.mark.parametrize("R,tpb,rpt", [(1, 4, 4), (1, 1, 1), (16, 2, 2)])
def test_xcd_block_orders_are_bitwise_neutral(R, tpb, rpt):
    """Every block order over the XCDs (dispatch order, contiguous eighths, runs of 16
    or 64 blocks) gives the same moments bit for bit: a block's tiles and the order
    in which block partials are summed do not change; blocks past the last tile add
    exact zeros."""
    s = synth.graphene_sheet(70, 50, 0.05, 8)          # 14,000 rows: grids of 14 to 55 blocks
    H = G.build(s, fmt="sell_f32", slice=64 if R == 1 else 16)
    a, b = G.oracle_ab_of(s)
    rd = G.to_dev(synth.random_phase(s.n, R, 3, np.complex64))
    vpt = 2 if R > 1 else 1
    mus = [tbkpm.kpm_moments(H, a, b, rd, 150, "c32", config=tbkpm.make_config(vpt, tpb, 1, xr, rpt))
           for xr in (0, 1, 2, 3)]
    for m in mus[1:]:
        assert torch.equal(m, mus[0])


def test_autotune_choice_is_valid_and_cached(tmp_path, monkeypatch):
    s = synth.graphene_sheet(40, 40, 0.05, 5)
    pos, sp = G.to_dev(s.pos), G.to_dev(s.species)
    res = tbkpm.autotune(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, R=4, precision="c32", steps=2)
    assert res.ms_per_step > 0 and res.candidates >= 10 and res.from_cache == 0
    again = tbkpm.autotune(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, R=4, precision="c32", steps=2)
    assert again.from_cache == 1 and again.slice == res.slice
    H = tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, fmt="sell_f32",
                                slice=res.slice)
    a, b = G.oracle_ab_of(s)
    r = synth.random_phase(s.n, 4, 2, np.complex64)
    mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 100, "c32", config=res.config).cpu().numpy()
    mu_o = _oracle_mu(s, a, b, r, 100)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mu.mean(0), a, b, E), O.kpm_dos(mu_o.mean(0), a, b, E)) <= 1e-4


def test_bad_shape_rejected():
    s = synth.graphene_sheet(5, 5)
    H = G.build(s, fmt="sell_f64", slice=64)
    r = G.to_dev(synth.random_phase(s.n, 2, 1))
    for bad in (tbkpm.make_config(2, 1, 1, 0, 1), tbkpm.make_config(1, 0, 1, 0, 1),
                tbkpm.make_config(1, 1, 2, 0, 1), tbkpm.make_config(1, 1, 1, 0, 3),
                tbkpm.make_config(1, 1, 1, 4, 1), tbkpm.make_config(1, 1, 1, -1, 1)):
        with pytest.raises(tbkpm.TBKError) as e:
            tbkpm.kpm_moments(H, 9.0, 0.0, r, 8, "f64", config=bad)
        assert e.value.name == "INVALID_ARG"
