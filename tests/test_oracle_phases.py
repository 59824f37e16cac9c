"""Pins of the oracle's counter-based random phases.

The generator is SplitMix64 (Steele, Lea & Flood 2014): output k is the mixed
state after k + 1 advances.  Its first outputs from state 0 are the published
reference values of the generator (Vigna's splitmix64.c, also the seeding
sequence of the xoshiro family), so a wrong constant, shift or order of the
mixing steps fails here.  The phases then only rescale the top 53 bits to
[0, 2 pi): |r| = 1, and the mean of exp(i phi) over many draws is within the
statistical bound of zero.
"""
import numpy as np

from oracle import oracle as O

# SplitMix64 from state 0: the first three outputs of the reference implementation
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_reference_outputs():
    assert [O.splitmix64(0, k) for k in range(3)] == SPLITMIX64_SEED0


def test_counter_form_equals_sequential_stream():
    """Output k from state s equals output 0 from state s + k * gamma (one shared stream)."""
    gamma = 0x9E3779B97F4A7C15
    for seed in (0, 1, 12345, 2**63 + 7):
        for k in (0, 1, 5, 1000, 2**40):
            assert O.splitmix64(seed, k) == O.splitmix64((seed + k * gamma) % 2**64, 0)


def test_phases_layout_unit_modulus_and_mean():
    n, R, seed = 4000, 3, 99
    r = O.random_phase(n, R, seed)
    np.testing.assert_allclose(np.abs(r), 1.0, atol=1e-15)
    # element (i, v) uses output i R + v
    x = O.splitmix64(seed, 7 * R + 2)
    phi = 2 * np.pi * ((x >> 11) * 2.0**-53)
    assert abs(r[7, 2] - np.exp(1j * phi)) < 1e-15
    assert abs(r.mean()) < 5.0 / np.sqrt(r.size)
    assert abs((r**2).mean()) < 5.0 / np.sqrt(r.size)     # phases uniform, not only balanced
    # different seeds give unrelated vectors
    r2 = O.random_phase(n, R, seed + 1)
    assert abs(np.vdot(r, r2)) / r.size < 5.0 / np.sqrt(r.size)
