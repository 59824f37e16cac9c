"""Pins of the oracle's s, p Slater-Koster orbital Hamiltonian.

* a dimer along z has the textbook block: ss sigma, sp sigma on s-p_z only, pp
  sigma on p_z-p_z, pp pi on p_x-p_x and p_y-p_y;
* the Hamiltonian is rotation covariant: rotating the structure by Q turns each
  atom-pair block B into D B D^T with D = diag(1, Q) (s is a scalar, p a vector);
  a wrong sign or a swapped direction cosine breaks this;
* for a flat sheet the p_z orbitals decouple (sigma-pi separation) and their
  block is exactly the one-orbital Hamiltonian with t_pair = V_pp_pi;
* H is symmetric and its onsite part is diag(e_s, e_p, e_p, e_p).
"""
import numpy as np
import pytest
import scipy.spatial.transform

from oracle import oracle as O
from paper_2509_06525_amd import synth

V = np.array([-5.7, 5.4, 6.2, -2.7])        # V_ss_sigma, V_sp_sigma, V_pp_sigma, V_pp_pi (eV)
ES, EP = -7.3, 0.0
OPEN = np.array([0, 0, 0], np.int32)


def test_dimer_along_z():
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.42]])
    csr, _ = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V, ES, EP)
    H = csr.dense()
    vss, vsp, vpps, vppp = V
    want = np.array([[vss, 0, 0, vsp], [0, vppp, 0, 0], [0, 0, vppp, 0], [-vsp, 0, 0, vpps]])
    np.testing.assert_allclose(H[0:4, 4:8], want, atol=1e-15)
    np.testing.assert_allclose(H[4:8, 0:4], want.T, atol=1e-15)
    np.testing.assert_allclose(np.diag(H), [ES, EP, EP, EP] * 2)


def test_rotation_covariance():
    s = synth.graphene_sheet(2, 2, 0.15, 5)
    pos = s.pos - s.pos.mean(0)
    Q = scipy.spatial.transform.Rotation.from_euler("zyx", [0.7, -0.4, 1.1]).as_matrix()
    h1, pairs = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V, ES, EP)
    h2, _ = O.sk_hamiltonian(pos @ Q.T, np.zeros(3), OPEN, V, ES, EP, pairs=pairs)
    D = np.eye(4)
    D[1:, 1:] = Q
    Dn = np.kron(np.eye(s.n), D)
    np.testing.assert_allclose(h2.dense(), Dn @ h1.dense() @ Dn.T, atol=1e-12)
    assert np.abs(h1.dense()).max() > 1.0


def test_flat_sheet_pz_block_is_the_one_orbital_hamiltonian():
    s = synth.graphene_sheet(4, 5)                  # pristine, all atoms at the same z
    sk, _ = O.sk_hamiltonian(s.pos, s.box, s.periodic, V, ES, EP)
    H = sk.dense()
    z = np.arange(s.n) * 4 + 3
    others = np.setdiff1d(np.arange(4 * s.n), z)
    assert np.abs(H[np.ix_(z, others)]).max() == 0.0
    h1, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, [EP], [[V[3]]])
    np.testing.assert_allclose(H[np.ix_(z, z)], h1.dense(), rtol=0, atol=1e-15)


def test_symmetric_with_periodic_images():
    s = synth.graphene_sheet(3, 3, 0.08, 2)
    sk, _ = O.sk_hamiltonian(s.pos, s.box, s.periodic, V, ES, EP)
    H = sk.dense()
    np.testing.assert_array_equal(H, H.T)
    assert abs(np.trace(H) - s.n * (ES + 3 * EP)) < 1e-12
    assert np.all(np.diff(sk.row_ptr) == 12)          # 3 neighbours x 4 orbitals per row


def test_orbital_velocity_is_commutator_with_atom_positions():
    """V = (i/hbar)[H, X] with X = diag(x of each orbital's atom), on an open flake."""
    s = synth.graphene_sheet(2, 2, 0.1, 8)
    csr, _ = O.sk_hamiltonian(s.pos, np.zeros(3), OPEN, V, ES, EP)
    vx = O.velocity_values(csr, s.pos, np.zeros(3), OPEN, 0, n_orb=4)
    Vd = np.zeros((csr.n, csr.n), complex)
    for i in range(csr.n):
        for q in range(csr.row_ptr[i], csr.row_ptr[i + 1]):
            Vd[i, csr.col[q]] += 1j * vx[q]
    H = csr.dense()
    X = np.diag(np.repeat(s.pos[:, 0], 4))
    np.testing.assert_allclose(Vd, 1j / O.HBAR_EV_FS * (H @ X - X @ H), atol=1e-12)


# s, p, d: V_ss_s, V_sp_s, V_pp_s, V_pp_p, V_sd_s, V_pd_s, V_pd_p, V_dd_s, V_dd_p, V_dd_d
V10 = np.array([-5.7, 5.4, 6.2, -2.7, -3.1, -2.4, 1.6, -1.9, 1.3, -0.4])
ED = 4.0


def d_harmonics(x):
    """Real d orbitals of the Slater-Koster table at unit vectors x [k][3]."""
    a, b, c = x[:, 0], x[:, 1], x[:, 2]
    s3 = np.sqrt(3.0)
    return np.stack([s3 * a * b, s3 * b * c, s3 * c * a, 0.5 * s3 * (a * a - b * b), c * c - 0.5 * (a * a + b * b)],
                    axis=1)


def d_rotation(Q):
    """D2 with d(Q x) = D2 d(x) for every unit x (least squares over many directions)."""
    rng = np.random.default_rng(0)
    x = rng.normal(size=(400, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    A, B = d_harmonics(x), d_harmonics(x @ Q.T)
    D2T, *_ = np.linalg.lstsq(A, B, rcond=None)
    assert np.abs(A @ D2T - B).max() < 1e-12          # the five functions span an invariant space
    return D2T.T


def test_spd_dimer_along_z():
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.42]])
    csr, _ = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V10, ES, EP, e_d=ED)
    H = csr.dense()[0:9, 9:18]
    ss, sp, pps, ppp, sd, pds, pdp, dds, ddp, ddd = V10
    want = np.zeros((9, 9))
    want[0, 0], want[0, 3], want[0, 8] = ss, sp, sd
    want[3, 0], want[8, 0] = -sp, sd
    want[1, 1] = want[2, 2] = ppp
    want[3, 3] = pps
    want[3, 8], want[8, 3] = pds, -pds
    want[1, 6], want[6, 1] = pdp, -pdp            # px - dzx
    want[2, 5], want[5, 2] = pdp, -pdp            # py - dyz
    want[8, 8] = dds
    want[5, 5] = want[6, 6] = ddp
    want[4, 4] = want[7, 7] = ddd
    np.testing.assert_allclose(H, want, atol=1e-14)
    np.testing.assert_allclose(np.diag(csr.dense())[:9], [ES, EP, EP, EP, ED, ED, ED, ED, ED])


def test_spd_rotation_covariance():
    s = synth.graphene_sheet(2, 2, 0.2, 6)
    pos = s.pos - s.pos.mean(0)
    Q = scipy.spatial.transform.Rotation.from_euler("zyx", [-0.3, 0.9, 2.1]).as_matrix()
    h1, pairs = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V10, ES, EP, e_d=ED)
    h2, _ = O.sk_hamiltonian(pos @ Q.T, np.zeros(3), OPEN, V10, ES, EP, e_d=ED, pairs=pairs)
    D = np.zeros((9, 9))
    D[0, 0] = 1.0
    D[1:4, 1:4] = Q
    D[4:9, 4:9] = d_rotation(Q)
    Dn = np.kron(np.eye(s.n), D)
    np.testing.assert_allclose(h2.dense(), Dn @ h1.dense() @ Dn.T, atol=1e-12)


def test_spd_mirror_parity_and_sp_restriction():
    s = synth.graphene_sheet(3, 4)                  # flat: z -> -z is a symmetry
    h9, _ = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, ES, EP, e_d=ED)
    H = h9.dense()
    odd = np.array([3, 5, 6])                       # pz, dyz, dzx
    even = np.setdiff1d(np.arange(9), odd)
    oi = (np.arange(s.n)[:, None] * 9 + odd).ravel()
    ei = (np.arange(s.n)[:, None] * 9 + even).ravel()
    assert np.abs(H[np.ix_(oi, ei)]).max() < 1e-14
    np.testing.assert_array_equal(H, H.T)
    h4, _ = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10[:4], ES, EP)
    sp = (np.arange(s.n)[:, None] * 9 + np.arange(4)).ravel()
    np.testing.assert_allclose(H[np.ix_(sp, sp)], h4.dense(), atol=1e-15)


# ---------------------------------------------------------------------------
# Learned form of Eq. (2): per-bond scales of the two-centre integrals
# ---------------------------------------------------------------------------

def test_unit_scales_reproduce_the_plain_table():
    s = synth.graphene_sheet(3, 2, 0.1, 7)
    plain, pairs = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, ES, EP, e_d=ED)
    ones, _ = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, ES, EP, e_d=ED, pairs=pairs,
                               scale=np.ones((pairs[0].shape[0], 10)))
    np.testing.assert_array_equal(plain.val, ones.val)
    np.testing.assert_array_equal(plain.col, ones.col)


def test_scaled_spd_dimer_puts_each_scale_on_its_integral():
    """Dimer along z: each textbook entry carries the scale of its own integral (a swapped
    integral index moves a scale onto the wrong entries)."""
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.42]])
    sc = np.array([1.5, 0.5, 2.0, 0.25, 3.0, 0.75, 1.25, 0.6, 1.8, 2.5])
    csr, _ = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V10, ES, EP, e_d=ED, scale=sc[None, :])
    H = csr.dense()[0:9, 9:18]
    ss, sp, pps, ppp, sd, pds, pdp, dds, ddp, ddd = V10 * sc
    want = np.zeros((9, 9))
    want[0, 0], want[0, 3], want[0, 8] = ss, sp, sd
    want[3, 0], want[8, 0] = -sp, sd
    want[1, 1] = want[2, 2] = ppp
    want[3, 3] = pps
    want[3, 8], want[8, 3] = pds, -pds
    want[1, 6], want[6, 1] = pdp, -pdp
    want[2, 5], want[5, 2] = pdp, -pdp
    want[8, 8] = dds
    want[5, 5] = want[6, 6] = ddp
    want[4, 4] = want[7, 7] = ddd
    np.testing.assert_allclose(H, want, atol=1e-14)
    np.testing.assert_allclose(np.diag(csr.dense())[:9], [ES, EP, EP, EP, ED, ED, ED, ED, ED])


def test_per_pair_scales_keep_h_symmetric_and_linear():
    """Distinct scales on every pair: H stays symmetric (both entries of a pair scaled
    alike), and H is the sum over integrals of the one-integral Hamiltonians with the
    same per-pair scales (the scales enter linearly, one per integral)."""
    s = synth.graphene_sheet(3, 3, 0.12, 2)
    pairs = O.neighbor_pairs(s.pos, s.box, s.periodic, 2.0)
    rng = np.random.default_rng(1)
    sc = rng.uniform(0.5, 1.5, (pairs[0].shape[0], 10))
    H = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, 0.0, 0.0, pairs=pairs, scale=sc)[0].dense()
    np.testing.assert_allclose(H, H.T, atol=1e-14)
    total = np.zeros_like(H)
    for lam in range(10):
        v1 = np.zeros(10)
        v1[lam] = V10[lam]
        total += O.sk_hamiltonian(s.pos, s.box, s.periodic, v1, 0.0, 0.0, pairs=pairs, scale=sc)[0].dense()
    np.testing.assert_allclose(H, total, atol=1e-13)


# ---------------------------------------------------------------------------
# Several species: integrals per ordered species pair, onsite energies per species
# ---------------------------------------------------------------------------

def species_tables(ns, seed, norb=9):
    """Random pair tables with the same-l integrals (ss, pp, dd) symmetric in the pair."""
    rng = np.random.default_rng(seed)
    K = 4 if norb == 4 else 10
    pv = rng.uniform(-6.0, 6.0, (ns, ns, K))
    for l in (0, 2, 3, 7, 8, 9)[: 3 if K == 4 else 6]:
        pv[:, :, l] = 0.5 * (pv[:, :, l] + pv[:, :, l].T)
    se = rng.uniform(-8.0, 8.0, (ns, 3))
    return pv, se


def test_hetero_dimer_along_z():
    """A (row) - B dimer along z: s_A-pz_B carries V_sp of (A, B), pz_A-s_B minus V_sp of
    (B, A); s-d and p-d likewise with their parities; onsite per species."""
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.42]])
    pv, se = species_tables(2, 3)
    csr, _ = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V10, 0.0, 0.0, species=np.array([0, 1]), pair_v=pv,
                              species_e=se)
    H = csr.dense()
    B = H[0:9, 9:18]
    ab, ba = pv[0, 1], pv[1, 0]
    assert B[0, 0] == pytest.approx(ab[0])
    assert B[0, 3] == pytest.approx(ab[1]) and B[3, 0] == pytest.approx(-ba[1])
    assert B[0, 8] == pytest.approx(ab[4]) and B[8, 0] == pytest.approx(ba[4])
    assert B[3, 8] == pytest.approx(ab[5]) and B[8, 3] == pytest.approx(-ba[5])
    assert B[1, 6] == pytest.approx(ab[6]) and B[6, 1] == pytest.approx(-ba[6])
    assert B[3, 3] == pytest.approx(ab[2]) and B[1, 1] == pytest.approx(ab[3])
    assert B[8, 8] == pytest.approx(ab[7]) and B[5, 5] == pytest.approx(ab[8]) and B[4, 4] == pytest.approx(ab[9])
    np.testing.assert_allclose(H, H.T, atol=1e-14)
    np.testing.assert_allclose(np.diag(H), np.concatenate([se[k][[0, 1, 1, 1, 2, 2, 2, 2, 2]] for k in (0, 1)]))


def test_species_relabelling_and_single_species_limit():
    s = synth.hbn_stripes(6, 4, stripe_cells=2, sigma=0.1, seed=3)
    pairs = O.neighbor_pairs(s.pos, s.box, s.periodic, 2.0)
    pv, se = species_tables(3, 8)
    H = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, 0.0, 0.0, pairs=pairs, species=s.species, pair_v=pv,
                         species_e=se)[0].dense()
    np.testing.assert_allclose(H, H.T, atol=1e-13)
    perm = np.array([2, 0, 1])                   # species k becomes perm[k]
    pv2 = np.empty_like(pv)
    se2 = np.empty_like(se)
    for a in range(3):
        se2[perm[a]] = se[a]
        for b in range(3):
            pv2[perm[a], perm[b]] = pv[a, b]
    H2 = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, 0.0, 0.0, pairs=pairs, species=perm[s.species],
                          pair_v=pv2, species_e=se2)[0].dense()
    np.testing.assert_array_equal(H, H2)
    one = np.broadcast_to(np.asarray(V10), (3, 3, 10))
    H1 = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, ES, EP, e_d=ED, pairs=pairs, species=s.species,
                          pair_v=one, species_e=np.tile([ES, EP, ED], (3, 1)))[0].dense()
    H0 = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, ES, EP, e_d=ED, pairs=pairs)[0].dense()
    np.testing.assert_array_equal(H1, H0)


def test_onsite_addition_and_node_features():
    """The onsite network's output is added per atom and shell; its inputs are the
    standardised node features in the first eight slots, bfloat16-rounded."""
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.42]])
    add = np.array([[0.5, -0.25, 1.0], [0.125, 0.75, -2.0]])
    csr, _ = O.sk_hamiltonian(pos, np.zeros(3), OPEN, V10, ES, EP, e_d=ED, onsite_add=add)
    np.testing.assert_array_equal(np.diag(csr.dense())[:9], [ES + 0.5] + [EP - 0.25] * 3 + [ED + 1.0] * 5)
    np.testing.assert_array_equal(np.diag(csr.dense())[9:], [ES + 0.125] + [EP + 0.75] * 3 + [ED - 2.0] * 5)
    v = np.array([[1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0]])
    X = O.node_features(v, np.full(8, 1.0), np.full(8, 2.0))
    np.testing.assert_array_equal(X[0, :8], (v[0] - 1.0) / 2.0)        # exact in bfloat16
    np.testing.assert_array_equal(X[0, 8:], 0.0)
    assert O.node_features(np.array([[1.0 + 2 ** -12] + [0.0] * 7]), np.zeros(8), np.ones(8))[0, 0] == 1.0
