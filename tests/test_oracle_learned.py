"""Pins of the oracle's learned-hopping pieces (CPU only).

Eq. (2): f_k(r) = [T_k(2 (r/rc - 1)^2 - 1) + 1] / 2 * f_c(r), v_i = sum_j f(r_ij).
MLP backward against central finite differences; bfloat16 rounding against
torch's own conversion; AdamW against torch.optim.AdamW.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_06525_amd import synth
from tests import ref_numpy as ref


@pytest.mark.parametrize("r", [0.0, 0.3, 1.42, 2.0, 2.4595, 3.2, 3.999, 4.0, 4.5])
def test_radial_matches_chebyshev_series(r):
    got = O.radial(r, 4.0, 8)
    np.testing.assert_allclose(got, ref.cheb_radial_ref(r, 4.0, 8), atol=1e-15)


def test_cutoff_special_values():
    """f_c(0) = 1, f_c(rc/2) = 1/2, f_c(rc) = 0 and f_k(0) = 1 for every k."""
    rc = 4.0
    np.testing.assert_allclose(O.radial(0.0, rc, 8), 1.0, atol=1e-15)
    assert O.radial(rc / 2, rc, 1)[0] == pytest.approx(0.5, abs=1e-15)
    np.testing.assert_array_equal(O.radial(rc, rc, 8), 0.0)
    # T_1(x) = x: f_1(rc/2) = (2 * 0.25 - 1 + 1)/2 * 1/2 = 1/8
    assert O.radial(rc / 2, rc, 2)[1] == pytest.approx(0.125, abs=1e-15)


def test_pristine_descriptor_shells():
    s = synth.graphene_sheet(6, 8)
    pairs = O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_DESC)
    v = O.descriptor(s.n, pairs, synth.R_DESC, synth.N_RADIAL)
    a = synth.A_CC
    expect = sum(m * ref.cheb_radial_ref(r, 4.0, 8)
                 for m, r in [(3, a), (6, math.sqrt(3) * a), (3, 2 * a), (6, math.sqrt(7) * a)])
    np.testing.assert_allclose(v, np.broadcast_to(expect, v.shape), rtol=1e-12, atol=1e-13)
    assert v[0, 0] == pytest.approx(4.7357, abs=1e-4)    # z0 of the coordination target


def test_bond_features_and_target_scale():
    s = synth.graphene_sheet(4, 6, 0.05, 3)
    pairs_d = O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_DESC)
    v = O.descriptor(s.n, pairs_d, synth.R_DESC, 8)
    hop = O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_HOP)
    X = O.bond_features(hop, v, synth.R_DESC)
    p = 5
    i, j, r = hop[0][p], hop[1][p], hop[2][p]
    np.testing.assert_allclose(X[p, :8], ref.cheb_radial_ref(r, 4.0, 8), atol=1e-15)
    np.testing.assert_allclose(X[p, 8:], v[i] + v[j], rtol=1e-15)
    shift = np.arange(16.0)
    scale = np.full(16, 2.0)
    X2 = O.bond_features(hop, v, synth.R_DESC, shift, scale)
    np.testing.assert_allclose(X2, (X - shift) / scale, rtol=1e-15)
    sc = O.target_scale(hop, v, 0.25, 4.7357)
    assert sc[p] == pytest.approx(1 + 0.25 * (v[i, 0] + v[j, 0] - 2 * 4.7357), rel=1e-15)
    s0 = synth.graphene_sheet(4, 6)
    pd0 = O.neighbor_pairs(s0.pos, s0.box, s0.periodic, synth.R_DESC)
    v0 = O.descriptor(s0.n, pd0, synth.R_DESC, 8)
    h0 = O.neighbor_pairs(s0.pos, s0.box, s0.periodic, synth.R_HOP)
    np.testing.assert_allclose(O.target_scale(h0, v0, 0.25, v0[0, 0]), 1.0, atol=1e-13)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-30, 30, size=2000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e-39, -1e-40]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.bf16(x32.astype(np.float64))
    np.testing.assert_array_equal(got, want)


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, O.N_PARAMS)


def test_mlp_forward_special_case():
    """Only b3 and one path W1[0,0] -> W2[0,0] -> W3[0] nonzero: closed form."""
    p = np.zeros(O.N_PARAMS)
    W1, b1 = 0, 512
    W2, b2 = 544, 1568
    W3, b3 = 1600, 1632
    p[W1] = 0.7; p[b1] = 0.1; p[W2] = -1.3; p[b2] = 0.05; p[W3] = 2.0; p[b3] = -0.4
    X = np.array([[0.5] + [9.0] * 15, [-1.0] + [0.0] * 15])
    y = O.mlp_forward(X, p, bf16_ops=False)
    for e in range(2):
        h1 = math.tanh(0.7 * X[e, 0] + 0.1)
        h2 = math.tanh(-1.3 * h1 + 0.05)
        assert y[e] == pytest.approx(2.0 * h2 - 0.4 + 31 * 0.0, rel=1e-14)
    # other hidden units: tanh(b) = 0 feeds nothing since W3[k>0] = 0


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, 16))
    tgt = rng.normal(size=7) * 0.1
    w = rng.uniform(0.5, 1.5, size=7)
    p = _params(2)
    loss, g = O.mlp_loss_grad(X, tgt, p, w=w, bf16_ops=False)
    h = 1e-6
    idx = list(range(0, O.N_PARAMS, 37)) + [511, 543, 1567, 1599, 1631, 1632]
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = O.mlp_loss_grad(X, tgt, pp, w=w, bf16_ops=False)
        lm, _ = O.mlp_loss_grad(X, tgt, pm, w=w, bf16_ops=False)
        fd = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i
    y = O.mlp_forward(X, p, bf16_ops=False)
    assert loss == pytest.approx(np.mean(w * (y - tgt) ** 2), rel=1e-14)


def test_bf16_forward_rounds_operands_only():
    """With weights and inputs already bfloat16, rounding changes only hidden activations."""
    rng = np.random.default_rng(3)
    p = O.bf16(_params(4))
    X = O.bf16(rng.normal(size=(5, 16)))
    y16, h1, h2 = O.mlp_forward(X, p, bf16_ops=True, keep=True)
    y64, g1, g2 = O.mlp_forward(X, p, bf16_ops=False, keep=True)
    np.testing.assert_allclose(h1, g1, rtol=1e-15)          # first layer: exact operands
    assert np.abs(y16 - y64).max() < 2e-2
    assert np.abs(y16 - y64).max() > 0


def test_adamw_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    grads = rng.normal(size=(4, 50))
    p = p0.copy(); m = np.zeros(50); v = np.zeros(50)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.05)
    for t in range(4):
        O.adamw_step(p, grads[t], m, v, t + 1, 1e-2, 0.9, 0.999, 1e-8, 0.05)
        opt.zero_grad()
        tp.grad = torch.tensor(grads[t], dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Species-dependent descriptor coefficients c_nk of Eq. (2)
# ---------------------------------------------------------------------------

def _stripes():
    s = synth.hbn_stripes(6, 4, stripe_cells=2, sigma=0.1, seed=3)
    return s, O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_DESC)


def test_identity_coefficients_reproduce_the_plain_descriptor():
    s, pd = _stripes()
    eye = np.broadcast_to(np.eye(8), (3, 3, 8, 8))
    np.testing.assert_array_equal(O.descriptor(s.n, pd, synth.R_DESC, 8, s.species, eye),
                                  O.descriptor(s.n, pd, synth.R_DESC, 8))
    np.testing.assert_array_equal(O.bond_features(pd, np.ones((s.n, 8)), synth.R_DESC, species=s.species, cnk=eye),
                                  O.bond_features(pd, np.ones((s.n, 8)), synth.R_DESC))


def test_coefficients_against_brute_force():
    """Pair by pair: C(r) = c[s_i][s_j] f(r), summed onto both atoms; bond features
    carry C of the bond's own species pair."""
    s, pd = _stripes()
    rng = np.random.default_rng(2)
    c = rng.normal(size=(3, 3, 8, 8))
    c = 0.5 * (c + c.transpose(1, 0, 2, 3))              # symmetric in the species pair
    v = np.zeros((s.n, 8))
    C = []
    for i, j, r in zip(*pd):
        g = c[s.species[i], s.species[j]] @ O.radial(r, synth.R_DESC)
        v[i] += g
        v[j] += g
        C.append(g)
    np.testing.assert_allclose(O.descriptor(s.n, pd, synth.R_DESC, 8, s.species, c), v, rtol=1e-13, atol=1e-13)
    X = O.bond_features(pd, v, synth.R_DESC, species=s.species, cnk=c)
    np.testing.assert_allclose(X[:, :8], np.array(C), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(X[:, 8:], v[pd[0]] + v[pd[1]], rtol=1e-14)
