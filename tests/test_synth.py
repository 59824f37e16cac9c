"""Checks of the seeded input generators (CPU only)."""
import math

import numpy as np

from paper_2509_06525_amd import synth


def test_sheet_counts_box_and_order():
    s = synth.graphene_sheet(5, 3)
    assert s.n == 60
    np.testing.assert_allclose(s.box, [5 * 4.26, 3 * math.sqrt(3) * 1.42, synth.SHEET_LZ])
    # cell-major order: atom 4*(cy*nx+cx)+b sits at the cell origin plus basis b
    i = 4 * (2 * 5 + 3) + 2
    np.testing.assert_allclose(s.pos[i, :2], [3 * 4.26 + 1.5 * 1.42, 2 * s.box[1] / 3 + 0.5 * s.box[1] / 3])


def test_displacements_are_seeded_gaussian():
    a = synth.graphene_sheet(40, 40, 0.05, 9)
    b = synth.graphene_sheet(40, 40, 0.05, 9)
    c = synth.graphene_sheet(40, 40)
    np.testing.assert_array_equal(a.pos, b.pos)
    d = a.pos - c.pos
    assert abs(d.std() - 0.05) < 0.002 and abs(d.mean()) < 0.002


def test_stripes_species_layout():
    s = synth.hbn_stripes(200, 2, 50)
    cx = (np.arange(s.n) // 4) % 200
    b = np.arange(s.n) % 4
    bn = (cx // 50) % 2 == 1
    assert np.all(s.species[~bn] == 0)
    assert np.all(s.species[bn & (b % 2 == 0)] == 1)
    assert np.all(s.species[bn & (b % 2 == 1)] == 2)


def test_snapshot_sizes_log_uniform_and_square():
    snaps = synth.snapshot_set(256, 3004)
    n = np.array([s.n for s in snaps])
    assert n.min() >= 900 and n.max() <= 52000
    assert 2.6e6 < n.sum() < 3.8e6
    for s in snaps[:20]:
        assert 0.9 < s.box[0] / s.box[1] < 1.1
        assert 0.02 <= s.sigma <= 0.08


def test_random_phase_unit_modulus():
    r = synth.random_phase(1000, 3, 5)
    np.testing.assert_allclose(np.abs(r), 1.0, rtol=1e-15)
    r64 = synth.random_phase(1000, 3, 5, np.complex64)
    np.testing.assert_allclose(r64, r, rtol=1e-7)
