"""GPU parity of the displacement (matrix-free) form of the Slater-Koster block
Hamiltonian: each bond stores (dx, dy, dz), the recurrence forms the block.

Stored displacements against the minimum-image differences of the positions
(FP64: exact to rounding); the pattern equals the block format's; FP64 moments
within 1e-10 of the row count against the oracle (s, p and s, p, d); complex
float DOS within 1e-4 relative L2 and moments within 1e-4 of the row count of
the stored-block form; the forms that need stored values are refused."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def build(s, norb, fmt, slice_=16, model=None):
    return tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic, *synth.SK_V,
                                      synth.SK_ES, synth.SK_EP, r_cut=synth.R_HOP, r0=synth.R0, beta=synth.BETA,
                                      fmt=fmt, slice=slice_, d=synth.SK_D if norb == 9 else None, e_d=synth.SK_ED,
                                      model=model)


def oracle_csr(s, norb):
    vv = (synth.SK_V + synth.SK_D) if norb == 9 else synth.SK_V
    return O.sk_hamiltonian(s.pos, s.box, s.periodic, vv, synth.SK_ES, synth.SK_EP, r_cut=synth.R_HOP,
                            r0=synth.R0, beta=synth.BETA, e_d=synth.SK_ED)[0]


@pytest.mark.parametrize("norb", [4, 9])
def test_displacements_and_pattern(norb):
    s = synth.graphene_sheet(7, 6, 0.08, 3)
    Hg = build(s, norb, "bgeom_f64", 16)
    Hb = build(s, norb, "bsell4_f64", 16)
    assert Hg.st.n_entries == Hb.st.n_entries and Hg.st.n_orb == norb
    tg = {k: v.cpu().numpy() for k, v in Hg.tensors.items()}
    tb = {k: v.cpu().numpy() for k, v in Hb.tensors.items()}
    ne = Hg.st.n_entries
    np.testing.assert_array_equal(tg["ptr"], tb["ptr"])
    # slots of real atoms (lanes past the last atom of the last slice are never written)
    C = Hg.st.slice
    ptr = tg["ptr"]
    valid = np.zeros(ne, bool)
    for sl in range(ptr.shape[0] - 1):
        w = (ptr[sl + 1] - ptr[sl]) // C
        lanes = min(C, s.n - sl * C)
        for k in range(w):
            valid[ptr[sl] + k * C: ptr[sl] + k * C + lanes] = True
    np.testing.assert_array_equal(tg["col"][:ne][valid], tb["col"][:ne][valid])
    np.testing.assert_array_equal(tg["onsite"], tb["onsite"])
    assert Hg.bounds == Hb.bounds
    assert list(Hg.st.sk_geom)[:4] == list(synth.SK_V)
    geo = tg["val"][: 3 * ne].reshape(ne, 3)
    perm = tg["perm"][::norb] // norb                      # atom row -> caller's atom
    n_at = s.n
    col = tg["col"]
    for sl in range(ptr.shape[0] - 1):
        w = (ptr[sl + 1] - ptr[sl]) // C
        for lane in range(C):
            r = sl * C + lane
            if r >= n_at:
                break
            for k in range(w):
                q = ptr[sl] + k * C + lane
                if col[q] == r:
                    np.testing.assert_array_equal(geo[q], 0.0)        # padding
                    continue
                d = s.pos[perm[col[q]]] - s.pos[perm[r]]
                for ax in range(3):
                    if s.periodic[ax]:
                        d[ax] -= s.box[ax] * np.rint(d[ax] / s.box[ax])
                np.testing.assert_allclose(geo[q], d, rtol=0, atol=1e-14)
    # float form: one 16-byte record per slot, (dx, dy, dz) rounded to float and the
    # column's bits, on every slot of the atoms' rows (padding included)
    Hf = build(s, norb, "bgeom_f32", 16)
    tf = {k: v.cpu().numpy() for k, v in Hf.tensors.items()}
    assert Hf.st.n_entries == ne and tf["val"].size >= 4 * ne
    rec = tf["val"][: 4 * ne].reshape(ne, 4)
    np.testing.assert_array_equal(tf["col"][:ne][valid], col[:ne][valid])
    np.testing.assert_array_equal(rec[valid, :3], geo[valid].astype(np.float32))
    np.testing.assert_array_equal(rec[valid, 3].view(np.int32), col[:ne][valid])


@pytest.mark.parametrize("norb,R,tpb,nt,xr,dbl", [(4, 1, 1, 1, 0, 0), (4, 3, 2, 0, 1, 0), (9, 1, 2, 1, 0, 0),
                                                  (9, 4, 1, 1, 1, 1), (9, 16, 2, 1, 0, 0), (9, 1, 1, 1, 0, 1),
                                                  (4, 1, 3, 0, 1, 1)])
def test_geom_fp64_moments(norb, R, tpb, nt, xr, dbl):
    s = synth.graphene_sheet(9, 7, 0.06, 4)
    csr = oracle_csr(s, norb)
    H = build(s, norb, "bgeom_f64", 32)
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(norb * s.n, R, 7)
    mo, _ = O.kpm_moments(csr, a, b, r, 61)
    for rows in (2, 4):                # one-vector rows staged through LDS, and direct
        cfg = tbkpm.make_config(1, tpb, nt, xr, rows, doubling=dbl, atom_rows=1)
        mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), 61, "f64", config=cfg).cpu().numpy()
        assert np.abs(mu - mo).max() <= 1e-10 * norb * s.n


@pytest.mark.parametrize("norb,R,vpt", [(4, 8, 2), (9, 1, 1), (9, 16, 2)])
def test_geom_c32_dos_and_stored_block_agreement(norb, R, vpt):
    s = synth.graphene_sheet(12, 10, 0.05, 8)
    csr = oracle_csr(s, norb)
    Hg = build(s, norb, "bgeom_f32", 64)
    Hb = build(s, norb, "bsell4_f32", 64)
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(norb * s.n, R, 3, np.complex64)
    cfg = tbkpm.make_config(vpt, 2, 1, 0, 1, atom_rows=1)
    mg = tbkpm.kpm_moments(Hg, a, b, G.to_dev(r), 256, "c32", config=cfg).cpu().numpy()
    mb = tbkpm.kpm_moments(Hb, a, b, G.to_dev(r), 256, "c32", config=cfg).cpu().numpy()
    mo, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), 256)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mg.mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4
    assert np.abs(mg - mb).max() <= 1e-4 * norb * s.n


def test_geom_refusals():
    s = synth.graphene_sheet(5, 4, 0.03, 1)
    H = build(s, 4, "bgeom_f64", 8)
    with pytest.raises(tbkpm.TBKError) as e:
        tbkpm.build_velocity(H, G.to_dev(s.pos), s.box, s.periodic, 0)
    assert e.value.name == "UNSUPPORTED"
    P = np.repeat(synth.init_mlp_params(1)[None, :], 4, axis=0)
    with pytest.raises(tbkpm.TBKError) as e:
        build(s, 4, "bgeom_f64", 8, model=dict(params=G.to_dev(P), shift=np.zeros(16), scale=np.ones(16)))
    assert e.value.name == "INVALID_ARG"


V10 = synth.SK_V + synth.SK_D
R3NN = 3.0                        # third-neighbour cutoff (shells at 1.42, 2.46, 2.84 A)


@pytest.mark.parametrize("rows", [2, 4])
def test_geom_third_neighbours_against_oracle_and_stored_blocks(rows):
    """s, p, d with the third-neighbour cutoff: C32 DOS of the displacement form within 1e-4
    of the oracle's, moments within 1e-4 of the row count of the stored-block form."""
    s = synth.graphene_sheet(24, 14, 0.05, 12)
    mk = lambda fmt: tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic,
                                                *synth.SK_V, synth.SK_ES, synth.SK_EP, r_cut=R3NN, r0=synth.R0,
                                                beta=synth.BETA, fmt=fmt, slice=64, d=synth.SK_D, e_d=synth.SK_ED)
    Hg, Hb = mk("bgeom_f32"), mk("bsell4_f32")
    assert Hg.st.max_degree >= 11
    csr = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, synth.SK_ES, synth.SK_EP, r_cut=R3NN, r0=synth.R0,
                           beta=synth.BETA, e_d=synth.SK_ED)[0]
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(9 * s.n, 1, 21, np.complex64)
    cfg = tbkpm.make_config(1, 2, 1, 0, rows, atom_rows=1)
    mg = tbkpm.kpm_moments(Hg, a, b, G.to_dev(r), 128, "c32", config=cfg).cpu().numpy()
    mb = tbkpm.kpm_moments(Hb, a, b, G.to_dev(r), 128, "c32", config=cfg).cpu().numpy()
    assert np.abs(mg - mb).max() <= 1e-4 * 9 * s.n
    mo, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), 128)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mg.mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4


@pytest.mark.parametrize("rows", [1, 2])
def test_geom_partial_last_tile_with_a_vacancy(rows):
    """A sheet with one atom removed (1343 atoms, 63 in the last 256-atom tile, so the
    tile's rows of T_{n-1}, r and the onsite energies end on a partial 16-byte chunk):
    the staged form (rows_per_thread 2, whose FP32 streams are copied to LDS at the
    tile's start) and the direct form agree with the stored blocks and the oracle, the
    doubling form (T_n copied instead of r) too."""
    base = synth.graphene_sheet(24, 14, 0.05, 17)
    keep = np.arange(base.n) != 700
    s = synth.Structure(pos=np.ascontiguousarray(base.pos[keep]), species=base.species[keep],
                        box=base.box, periodic=base.periodic)
    assert s.n % 256 == 63
    mk = lambda fmt: tbkpm.build_hamiltonian_sk(G.to_dev(s.pos), G.to_dev(s.species), s.box, s.periodic,
                                                *synth.SK_V, synth.SK_ES, synth.SK_EP, r_cut=R3NN, r0=synth.R0,
                                                beta=synth.BETA, fmt=fmt, slice=64, d=synth.SK_D, e_d=synth.SK_ED)
    Hg, Hb, Hg64 = mk("bgeom_f32"), mk("bsell4_f32"), mk("bgeom_f64")
    csr = O.sk_hamiltonian(s.pos, s.box, s.periodic, V10, synth.SK_ES, synth.SK_EP, r_cut=R3NN, r0=synth.R0,
                           beta=synth.BETA, e_d=synth.SK_ED)[0]
    a, b = G.oracle_ab(csr)
    r = synth.random_phase(9 * s.n, 1, 23, np.complex64)
    cfg = tbkpm.make_config(1, 1, 1, 2, rows, atom_rows=1)
    mg = tbkpm.kpm_moments(Hg, a, b, G.to_dev(r), 96, "c32", config=cfg).cpu().numpy()
    mb = tbkpm.kpm_moments(Hb, a, b, G.to_dev(r), 96, "c32", config=cfg).cpu().numpy()
    assert np.abs(mg - mb).max() <= 1e-4 * 9 * s.n
    mo, _ = O.kpm_moments(csr, a, b, r.astype(np.complex128), 96)
    E = synth.energy_grid(a, b)
    assert G.rel_l2(O.kpm_dos(mg.mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4
    md = tbkpm.kpm_moments(Hg, a, b, G.to_dev(r), 96, "c32", config=tbkpm.with_doubling(cfg)).cpu().numpy()
    assert G.rel_l2(O.kpm_dos(md.mean(0), a, b, E), O.kpm_dos(mo.mean(0), a, b, E)) <= 1e-4
    m64 = tbkpm.kpm_moments(Hg64, a, b, G.to_dev(r.astype(np.complex128)), 96, "f64", config=cfg).cpu().numpy()
    assert np.abs(m64 - mo).max() <= 1e-10 * 9 * s.n


def bloch_spectrum(cell, tx, ty):
    """Exact spectrum of the pristine s, p, d third-neighbour sheet on a torus of tx x ty copies
    of the small periodic sheet `cell`, from the oracle's blocks of the small sheet and the
    commensurate Bloch phases (each entry's minimum-image lattice shift)."""
    csr = O.sk_hamiltonian(cell.pos, cell.box, cell.periodic, V10, synth.SK_ES, synth.SK_EP, r_cut=R3NN,
                           r0=synth.R0, beta=synth.BETA, e_d=synth.SK_ED)[0]
    nr = 9 * cell.n
    rows = np.repeat(np.arange(nr), np.diff(csr.row_ptr))
    cols = csr.col.astype(np.int64)
    d = cell.pos[cols // 9] - cell.pos[rows // 9]
    img = np.zeros_like(d)
    for ax in range(2):                              # periodic x, y
        img[:, ax] = -cell.box[ax] * np.rint(d[:, ax] / cell.box[ax])
    idx = rows * nr + cols
    eigs = []
    kx = 2 * np.pi * np.arange(tx) / (tx * cell.box[0])
    ky = 2 * np.pi * np.arange(ty) / (ty * cell.box[1])
    K = np.array([(x, y) for x in kx for y in ky])
    for s0 in range(0, K.shape[0], 100):
        Hk = []
        for k in K[s0:s0 + 100]:
            ph = np.exp(1j * (img[:, 0] * k[0] + img[:, 1] * k[1])) * csr.val
            h = (np.bincount(idx, weights=ph.real, minlength=nr * nr)
                 + 1j * np.bincount(idx, weights=ph.imag, minlength=nr * nr)).reshape(nr, nr)
            h[np.arange(nr), np.arange(nr)] += csr.diag
            Hk.append(h)
        eigs.append(np.linalg.eigvalsh(np.array(Hk)).reshape(-1))
    return np.concatenate(eigs), csr


def test_geom_100M_third_neighbours_against_exact_spectrum():
    """100 M atoms (900 M orbital rows), pristine s, p, d third-neighbour sheet, displacement
    form, the launch path of the benchmark (one vector, rows staged): moments n < 150 against
    the exact spectrum of a 200 x 200-cell torus (walks shorter than ~164 hops do not wrap
    it), |mu_n / N - tau_n| <= 5 / sqrt(N)."""
    from tests import ref_numpy as ref
    cell = synth.graphene_sheet(2, 4)                # 8.52 x 9.84 A: above twice the cutoff
    eigs, csr = bloch_spectrum(cell, 100, 50)        # 200 x 200 unit cells
    assert eigs.size == 9 * 4 * 200 * 200
    a, b = G.oracle_ab(csr)                          # every atom is equivalent: the same bounds
    Mc = 150
    tau = ref.trace_moments_from_eigs(eigs, a, b, Mc) / eigs.size
    s = synth.graphene_sheet(5000, 5000)
    n = 9 * s.n
    print(f"[fullsize] spd 3nn: N={s.n} atoms, {n} rows, M={Mc}", flush=True)
    pos, sp = G.to_dev(s.pos), G.to_dev(s.species)
    H = tbkpm.build_hamiltonian_sk(pos, sp, s.box, s.periodic, *synth.SK_V, synth.SK_ES, synth.SK_EP, r_cut=R3NN,
                                   r0=synth.R0, beta=synth.BETA, fmt="bgeom_f32", slice=64, d=synth.SK_D,
                                   e_d=synth.SK_ED)
    del s, pos, sp
    assert H.st.max_degree == 12
    cfg = tbkpm.make_config(1, 1, 0, 1, 1, atom_rows=1)
    mu = tbkpm.kpm_moments_seeded(H, a, b, 77, 1, Mc, "c32", config=cfg).cpu().numpy()[0]
    dev = np.abs(mu / n - tau)
    bound = 5.0 / np.sqrt(n)
    print(f"[fullsize] spd 3nn vs exact: max dev {dev.max():.3e} (bound {bound:.3e})", flush=True)
    assert np.all(dev <= bound)
