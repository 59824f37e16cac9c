"""GPU parity and behaviour of the learned-hopping path (descriptor, bond MLP,
training, fused learned assembly) against the BF16-emulating FP64 oracle.

Bars (derived from the arithmetic): descriptor and bond geometry are FP64 on
both sides (1e-12 relative); the bfloat16 feature codes are decided from FP64
values on both sides (bit-exact except at ties within FP64 rounding, allowed
for at most 1 in 10^4 codes, one bf16 step apart); MLP outputs differ by FP32
accumulation (~1e-6) and by rare one-ulp flips of a bf16 activation
(2^-8 relative of one hidden value): 99.9% of bonds within 2e-5, all within
1e-2 (1 + |y|); gradients within 1e-3 relative L2 (the flips average out);
AdamW within 1e-6 relative (FP32 state).  The learned DOS must be within 1e-2
relative L2 of the oracle DOS of the target Hamiltonian and closer to it than
the plain-formula DOS.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

PER = (1, 1, 0)


def sheets_small():
    return [synth.graphene_sheet(9, 14, 0.05, 1), synth.graphene_sheet(6, 11, 0.08, 2),
            synth.graphene_sheet(14, 23, 0.02, 3)]


def oracle_parts(s):
    pd = O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_DESC)
    v = O.descriptor(s.n, pd, synth.R_DESC, 8)
    hop = O.neighbor_pairs(s.pos, s.box, s.periodic, synth.R_HOP)
    o = np.lexsort((hop[1], hop[0]))
    hop = (hop[0][o], hop[1][o], hop[2][o])
    return v, hop


def gpu_parts(structs):
    pos, sp, seg, boxes = synth.stack(structs)
    pd = G.to_dev(pos)
    v = tbkpm.descriptor(pd, seg, boxes, PER, synth.R_DESC, 8)
    b = tbkpm.bonds(pd, seg, boxes, PER, synth.R_HOP)
    return pos, sp, seg, boxes, v, b


def bf16_bits_to_float(X):
    u = X.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def test_descriptor_and_bonds_match_oracle():
    ss = sheets_small()
    pos, sp, seg, boxes, v, (bi, bj, br) = gpu_parts(ss)
    v = v.cpu().numpy()
    bi, bj, br = bi.cpu().numpy(), bj.cpu().numpy(), br.cpu().numpy()
    for k, s in enumerate(ss):
        vo, hop = oracle_parts(s)
        np.testing.assert_allclose(v[seg[k]:seg[k + 1]], vo, rtol=1e-12, atol=1e-13)
        m = (bi >= seg[k]) & (bi < seg[k + 1])
        np.testing.assert_array_equal(bi[m] - seg[k], hop[0])
        np.testing.assert_array_equal(bj[m] - seg[k], hop[1])
        np.testing.assert_allclose(br[m], hop[2], rtol=1e-15)


def oracle_moments(ss):
    """Mean and standard deviation of the oracle's raw bond features over the structures."""
    raw = np.concatenate([O.bond_features(oracle_parts(s)[1], oracle_parts(s)[0], synth.R_DESC) for s in ss])
    return raw.mean(0), raw.std(0)


def test_features_moments_and_targets_match_oracle():
    ss = sheets_small()
    pos, sp, seg, boxes, v, b = gpu_parts(ss)
    mean_o, std_o = oracle_moments(ss)
    mean, std = tbkpm.feature_moments(b, v, synth.R_DESC)
    np.testing.assert_allclose(mean, mean_o, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(std, std_o, rtol=1e-8, atol=1e-12)
    # both sides standardise with the oracle's moments
    X = bf16_bits_to_float(tbkpm.bond_features(b, v, mean_o, std_o, synth.R_DESC))
    y = tbkpm.coordination_target(b, v, synth.COORD_KAPPA, synth.COORD_Z0).cpu().numpy()
    Xo, yo = [], []
    for s in ss:
        vo, hop = oracle_parts(s)
        Xo.append(O.bf16(O.bond_features(hop, vo, synth.R_DESC, mean_o, std_o)))
        yo.append(O.target_scale(hop, vo, synth.COORD_KAPPA, synth.COORD_Z0) - 1.0)
    Xo = np.concatenate(Xo)
    mism = X != Xo
    assert mism.mean() <= 1e-4
    if mism.any():
        np.testing.assert_allclose(X[mism], Xo[mism], rtol=2 ** -7)
    np.testing.assert_allclose(y, np.concatenate(yo), rtol=1e-6, atol=1e-7)


def _rand_inputs(nb, seed):
    rng = np.random.default_rng(seed)
    Xf = O.bf16(rng.normal(size=(nb, 16)))
    bits = (Xf.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return Xf, torch.from_numpy(bits.copy()).to(G.DEV)


@pytest.mark.parametrize("nb", [1, 15, 16, 17, 1000, 20011])
def test_mlp_forward_matches_bf16_oracle(nb):
    Xf, Xd = _rand_inputs(nb, nb)
    p = synth.init_mlp_params(7, out_scale=1.0)
    y = tbkpm.mlp_forward(Xd, G.to_dev(p)).cpu().numpy().astype(np.float64)
    yo, h1, h2 = O.mlp_forward(Xf, p.astype(np.float64), bf16_ops=True, keep=True)
    d = np.abs(y - yo)
    clear = G.bf16_decisions_clear(h1, h2)
    assert nb < 256 or clear.mean() >= 0.5
    assert np.all(d[clear] <= 2e-5)
    assert np.all(d <= 1e-2 * (1 + np.abs(yo)))


@pytest.mark.parametrize("nb,weighted", [(33, False), (5000, True)])
def test_mlp_grad_matches_bf16_oracle(nb, weighted):
    Xf, Xd = _rand_inputs(nb, 100 + nb)
    p = synth.init_mlp_params(8, out_scale=1.0)
    rng = np.random.default_rng(9)
    tgt = rng.normal(size=nb).astype(np.float32) * 0.1
    w = rng.uniform(0.5, 1.5, size=nb).astype(np.float32) if weighted else None
    loss, g = tbkpm.mlp_loss_grad(Xd, G.to_dev(tgt), G.to_dev(p), None if w is None else G.to_dev(w))
    lo, go = O.mlp_loss_grad(Xf, tgt.astype(np.float64), p.astype(np.float64),
                             w=None if w is None else w.astype(np.float64), bf16_ops=True)
    g = g.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(lo, rel=1e-4)
    assert np.linalg.norm(g - go) <= 1e-3 * np.linalg.norm(go)
    # every parameter block is covered (a mis-mapped layout leaves blocks wrong)
    for a, b in [(0, 512), (512, 544), (544, 1568), (1568, 1600), (1600, 1632), (1632, 1633)]:
        assert np.linalg.norm(g[a:b] - go[a:b]) <= 5e-3 * max(np.linalg.norm(go[a:b]), 1e-12), (a, b)


def test_adamw_matches_oracle():
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=1633)
    p = G.to_dev(p0.astype(np.float32))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    po, mo, vo = p0.astype(np.float32).astype(np.float64), np.zeros(1633), np.zeros(1633)
    for t in range(1, 4):
        g = rng.normal(size=1633).astype(np.float32)
        tbkpm.adamw_step(p, G.to_dev(g), m, v, t, 1e-2, 0.9, 0.999, 1e-8, 1e-2)
        O.adamw_step(po, g.astype(np.float64), mo, vo, t, 1e-2, 0.9, 0.999, 1e-8, 1e-2)
    np.testing.assert_allclose(p.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


def _training_set(count=24, seed=4004):
    snaps = synth.snapshot_set(count, seed, n_min=1000, n_max=8000)
    pos, sp, seg, boxes, v, b = gpu_parts(snaps)
    mean, std = tbkpm.feature_moments(b, v, synth.R_DESC)
    std = [max(s, 1e-6) for s in std]
    X = tbkpm.bond_features(b, v, mean, std, synth.R_DESC)
    y = tbkpm.coordination_target(b, v, synth.COORD_KAPPA, synth.COORD_Z0)
    return X, y, mean, std


def train_model(epochs=120, seed=11):
    X, y, mean, std = _training_set()
    tr = tbkpm.MlpTrainer(G.to_dev(synth.init_mlp_params(seed)))
    hist = tr.train(X, y, epochs=epochs, batch=2048, lr=2e-3, wd=1e-5)
    return tr.params, mean, std, hist, X, y


def test_training_lowers_the_loss_and_is_deterministic():
    X, y, mean, std = _training_set(count=6)
    p0 = G.to_dev(synth.init_mlp_params(5))
    t1, t2 = tbkpm.MlpTrainer(p0.clone()), tbkpm.MlpTrainer(p0.clone())
    h1 = t1.train(X, y, epochs=40, batch=1024, lr=2e-3, wd=1e-5)
    h2 = t2.train(X, y, epochs=40, batch=1024, lr=2e-3, wd=1e-5)
    assert h1 == h2
    torch.testing.assert_close(t1.params, t2.params, rtol=0, atol=0)
    assert h1[-1] < 0.05 * h1[0]
    var = float(torch.var(y).item())
    assert h1[-1] < 0.05 * var


def test_learned_assembly_matches_oracle():
    ss = sheets_small()
    p = synth.init_mlp_params(21, out_scale=1.0)
    pos, sp, seg, boxes, v, b = gpu_parts(ss)
    mean, std = oracle_moments(ss)
    H = tbkpm.build_hamiltonian_learned(G.to_dev(pos), G.to_dev(sp), seg, boxes, PER, [0.0], [[-2.7]],
                                        G.to_dev(p), mean, std, fmt="sell_f64", slice=32, with_bond_y=True)
    rows, cols, vals, _ = G.entries_in_atom_order(H)
    H32 = tbkpm.build_hamiltonian_learned(G.to_dev(pos), G.to_dev(sp), seg, boxes, PER, [0.0], [[-2.7]],
                                          G.to_dev(p), mean, std, fmt="sell_f32", slice=64)
    r32, c32, v32, _ = G.entries_in_atom_order(H32)
    o1, o2 = np.lexsort((cols, rows)), np.lexsort((c32, r32))
    np.testing.assert_allclose(v32[o2], vals[o1], rtol=1e-6)
    for k, s in enumerate(ss):
        vo, hop = oracle_parts(s)
        Xo = O.bf16(O.bond_features(hop, vo, synth.R_DESC, mean, std))
        yo, h1, h2 = O.mlp_forward(Xo, p.astype(np.float64), bf16_ops=True, keep=True)
        csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair, t_scale=1.0 + yo,
                               pairs=hop)
        orow, ocol, oval = G.csr_entries(csr)
        m = (rows >= seg[k]) & (rows < seg[k + 1])
        r, c, vv = rows[m] - seg[k], cols[m] - seg[k], vals[m]
        a1, a2 = np.lexsort((c, r)), np.lexsort((ocol, orow))
        np.testing.assert_array_equal(c[a1], ocol[a2])
        rel = np.abs(vv[a1] - oval[a2]) / np.abs(oval[a2])
        # entries of bonds whose activations sit clear of a bf16 rounding boundary
        clear = G.bf16_decisions_clear(h1, h2)
        bond_of = {(int(i), int(j)): e for e, (i, j) in enumerate(zip(hop[0], hop[1]))}
        ent_clear = np.array([clear[bond_of[(min(i, j), max(i, j))]] for i, j in zip(orow[a2], ocol[a2])])
        assert ent_clear.mean() >= 0.3
        assert rel[ent_clear].max() <= 5e-5
        assert rel.max() <= 1e-2
        np.testing.assert_array_equal(vv.reshape(-1) != 0, True)
    # learned bounds bound the learned values
    for k in range(len(ss)):
        lo, hi = H.bounds[k]
        assert lo < 0 < hi


def test_learned_hoppings_beat_the_plain_formula():
    """DOS of H_learned vs the oracle DOS of the coordination-corrected target H."""
    params, mean, std, hist, X, y = train_model()
    assert hist[-1] < 0.02 * hist[0]
    evals = synth.snapshot_set(256, 3004)[:4]
    pos, sp, seg, boxes = synth.stack(evals)
    Hl = tbkpm.build_hamiltonian_learned(G.to_dev(pos), G.to_dev(sp), seg, boxes, PER, [0.0], [[-2.7]], params,
                                         mean, std, fmt="sell_f32", slice=64)
    Hp = tbkpm.build_hamiltonian_batched(G.to_dev(pos), G.to_dev(sp), seg, boxes, PER, [0.0], [[-2.7]],
                                         fmt="sell_f32", slice=64)
    M, R = 1024, 8
    r = synth.random_phase(pos.shape[0], R, 77, np.complex64)
    a, b, rho_t = [], [], []
    for k, s in enumerate(evals):
        vo, hop = oracle_parts(s)
        scale_t = O.target_scale(hop, vo, synth.COORD_KAPPA, synth.COORD_Z0)
        csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair, t_scale=scale_t, pairs=hop)
        lo, hi = O.gershgorin(csr)
        ak, bk = 1.05 * (hi - lo) / 2, (hi + lo) / 2
        a.append(ak)
        b.append(bk)
        mu_t, _ = O.kpm_moments(csr, ak, bk, r[seg[k]:seg[k + 1]].astype(np.complex128), M)
        rho_t.append(O.kpm_dos(mu_t.mean(0), ak, bk, synth.energy_grid(ak, bk)))
    rd = G.to_dev(r)
    mu_l = tbkpm.kpm_moments_batched(Hl, a, b, rd, M, "c32").cpu().numpy()
    mu_p = tbkpm.kpm_moments_batched(Hp, a, b, rd, M, "c32").cpu().numpy()
    for k in range(len(evals)):
        E = synth.energy_grid(a[k], b[k])
        err_l = G.rel_l2(O.kpm_dos(mu_l[k].mean(0), a[k], b[k], E), rho_t[k])
        err_p = G.rel_l2(O.kpm_dos(mu_p[k].mean(0), a[k], b[k], E), rho_t[k])
        print(f"[learned] snapshot {k}: N={evals[k].n} err_learned={err_l:.3e} err_plain={err_p:.3e}", flush=True)
        assert err_l <= 1e-2
        assert err_l < err_p
