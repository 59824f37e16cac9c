"""The library's step-kernel timer (kpm_step_timer): events around the step
launches only, on the caller's stream, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def test_step_timer_counts_step_launches_only():
    s = synth.graphene_sheet(60, 50, 0.05, 3)
    H = G.build(s, fmt="sell_f32", slice=64)
    a, b = H.scale()
    r = G.to_dev(synth.random_phase(s.n, 4, 5, np.complex64))
    M = 300                                            # > 64 steps: several stretches between reductions
    tbkpm.kpm_moments(H, a, b, r, M, "c32")            # warm-up
    tbkpm.step_timer(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    tbkpm.kpm_moments(H, a, b, r, M, "c32")
    e1.record()
    torch.cuda.synchronize()
    ms, n = tbkpm.step_timer_read()
    assert n == M - 1
    assert 0.0 < ms <= e0.elapsed_time(e1)
    assert tbkpm.step_timer_read() == (0.0, 0)         # read clears
    tbkpm.step_timer(False)
    tbkpm.kpm_moments(H, a, b, r, M, "c32")
    assert tbkpm.step_timer_read() == (0.0, 0)         # off: nothing timed
    # a stacked Hamiltonian, one launch per step
    snaps = [synth.graphene_sheet(9, 8, 0.05, k) for k in range(3)]
    pos, sp, seg, boxes = synth.stack(snaps)
    Hb = tbkpm.build_hamiltonian_batched(G.to_dev(pos), G.to_dev(sp), seg, boxes, (1, 1, 0), [0.0], [[-2.7]],
                                         fmt="sell_f32", slice=64)
    ab, bb = Hb.scales()
    rb = G.to_dev(synth.random_phase(int(seg[-1]), 2, 1, np.complex64))
    tbkpm.step_timer(True)
    tbkpm.kpm_moments_batched(Hb, ab, bb, rb, 100, "c32")
    ms, n = tbkpm.step_timer_read()
    tbkpm.step_timer(False)
    assert n == 99 and ms > 0.0


def test_scale_matches_the_bounds():
    s = synth.hbn_stripes(10, 8, stripe_cells=2, sigma=0.03, seed=4)
    H = G.build(s, fmt="sell_f64", slice=32)
    lo, hi = H.bounds
    a, b = H.scale(1.01)
    assert a == 1.01 * (hi - lo) / 2.0 and b == (hi + lo) / 2.0
