"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (the slice height and launch shape of the shipped MI355X tuning
table, which bench.py starts from).

The expected moments are the serial FP64 oracle's, stored under tests/golden/
by tests/golden/make_golden.py for the leading random vectors of each workload
(the complex64 phases widened to complex128), together with the (a, b) the
oracle derived; the GPU runs with that same (a, b).

Bars: complex-float path, DOS relative L2 <= 1e-4 on 2001 energies and
|mu_gpu - mu_oracle| <= 1e-4 mu_0 per moment; FP64 path <= 1e-10 mu_0.
The 100M-atom pristine sheet is also checked against its exact spectrum
(commensurate Bloch sum of a smaller periodic sheet, exact for walks shorter
than the smaller sheet's period): |mu_n/N - tau_n| <= 5/sqrt(N) for n < 300.
"""
import math
import os

import numpy as np
import pytest
import torch

from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G
from tests import ref_numpy as ref
from tests.golden import make_golden

pytestmark = pytest.mark.gpu

WORKLOADS = ["graphene_thermal_1M", "hbn_graphene_stripes_4M", "graphene_pristine_100M"]


def _have(name):
    return os.path.exists(make_golden.golden_path(name))


def shipped_shape(n, R, precision="c32", fmt=2, degree=3, onsite=0):
    """(slice, launch shape) of the shipped MI355X tuning table's entry for this
    problem class: the shape bench.py times (it starts from the same table)."""
    path = os.path.join(os.path.dirname(tbkpm.LIB_PATH), "tuned_gfx950.txt")
    lg = int(math.floor(math.log2(n)))
    p = {"f64": 0, "c32": 1}[precision]
    suffix = f"/n2^{lg}/R{R}/p{p}/f{fmt}/deg{degree}/ons{onsite}"
    for line in open(path):
        parts = line.split()
        if parts and parts[0].endswith(suffix):
            sl, vpt, tpb, nt, xcd, rpt = (int(v) for v in parts[1:7])
            compact = int(parts[8]) if len(parts) > 8 else 0
            return sl, tbkpm.make_config(vpt, tpb, nt, xcd, rpt, compact_columns=compact)
    raise AssertionError(f"no shipped tuning entry for {suffix}")


def _run(name, precision):
    w = synth.WORKLOADS[name]
    a, b, mu_o = make_golden.load(name)
    nv = mu_o.shape[0]
    s = synth.make_structure(name)
    print(f"[fullsize] {name}: N={s.n} M={w['M']} R={w['R']} {precision}", flush=True)
    r = synth.random_phase(s.n, w["R"], w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)
    pos, sp = G.to_dev(s.pos), G.to_dev(s.species)
    if precision == "c32":
        sl, cfg = shipped_shape(s.n, w["R"], onsite=int(np.any(s.onsite != 0)))
        print(f"[fullsize] {name}: shipped shape slice {sl} {cfg.as_dict()}", flush=True)
        H = tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, fmt="sell_f32", slice=sl)
        rd = G.to_dev(r)
    else:
        H = tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, fmt="sell_f64", slice=64)
        rd = G.to_dev(r.astype(np.complex128))
        cfg = None
    n = s.n
    del s, pos, sp
    mu = tbkpm.kpm_moments(H, a, b, rd, w["M"], precision, config=cfg).cpu().numpy()
    return n, a, b, mu, mu_o, nv


@pytest.mark.parametrize("name", WORKLOADS)
def test_fullsize_c32_against_oracle(name):
    if not _have(name):
        pytest.skip(f"golden moments for {name} not generated")
    n, a, b, mu, mu_o, nv = _run(name, "c32")
    E = synth.energy_grid(a, b)
    from oracle import oracle as O
    rho_g = O.kpm_dos(mu[:nv].mean(0), a, b, E)
    rho_o = O.kpm_dos(mu_o.mean(0), a, b, E)
    err = G.rel_l2(rho_g, rho_o)
    dmu = np.abs(mu[:nv] - mu_o).max() / n
    print(f"[fullsize] {name}: DOS relL2 {err:.3e}, max|dmu|/N {dmu:.3e}", flush=True)
    assert err <= 1e-4
    assert dmu <= 1e-4
    np.testing.assert_allclose(mu[:, 0], n, rtol=1e-6)        # mu_0 = sum |r|^2 for every vector


def test_fullsize_fp64_against_oracle():
    name = "graphene_thermal_1M"
    if not _have(name):
        pytest.skip("golden moments not generated")
    n, a, b, mu, mu_o, nv = _run(name, "f64")
    dmu = np.abs(mu[:nv] - mu_o).max() / n
    print(f"[fullsize] {name} FP64: max|dmu|/N {dmu:.3e}", flush=True)
    assert dmu <= 1e-10


def test_fullsize_100M_against_exact_spectrum():
    name = "graphene_pristine_100M"
    w = synth.WORKLOADS[name]
    s = synth.make_structure(name)
    n = s.n
    r = synth.random_phase(n, 1, w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)
    pos, sp = G.to_dev(s.pos), G.to_dev(s.species)
    sl, cfg = shipped_shape(n, 1)
    H = tbkpm.build_hamiltonian(pos, sp, s.box, s.periodic, s.onsite, s.t_pair, fmt="sell_f32", slice=sl)
    del s, pos, sp
    a, b = H.scale()
    assert abs(b) < 1e-12 and a == pytest.approx(1.01 * 8.1, rel=1e-10)
    Mc = 300
    mu = tbkpm.kpm_moments(H, a, b, G.to_dev(r), Mc, "c32", config=cfg).cpu().numpy()[0]
    # 200 x 200 cells: closed walks that wrap the torus need > 300 hops, so moments n < 300 are exact
    eig = ref.supercell_spectrum(200, 200)
    tau = ref.trace_moments_from_eigs(eig, a, b, Mc) / eig.size
    bound = 5.0 / math.sqrt(n)
    dev = np.abs(mu / n - tau)
    print(f"[fullsize] 100M vs exact: max dev {dev.max():.3e} (bound {bound:.3e})", flush=True)
    assert np.all(dev <= bound)
    assert tau[2] == pytest.approx(2 * 3 * 2.7 ** 2 / a ** 2 - 1, abs=1e-12)


def test_fullsize_snapshot_batch():
    """All 256 snapshots of the learned-hopping workload (3.43 M atoms, M = 1024,
    R = 8) with plain hoppings, in one batched recurrence per launch shape the
    benchmark chooses from: the XCD-aware block orders at 1, 2 and 4 tiles per
    block equal the plain order bitwise, and three sampled snapshots (the first,
    the last and the smallest) match the oracle, DOS relative L2 <= 1e-4."""
    from oracle import oracle as O
    w = synth.WORKLOADS["graphene_snapshots_256"]
    snaps = synth.snapshot_set(w["count"], w["seed"])
    pos, sp, seg, boxes = synth.stack(snaps)
    N, M, R = int(seg[-1]), w["M"], w["R"]
    print(f"[fullsize] snapshot batch: {len(snaps)} structures, N={N} M={M} R={R}", flush=True)
    a, b = G.oracle_scales(snaps)
    H = tbkpm.build_hamiltonian_batched(G.to_dev(pos), G.to_dev(sp), seg, boxes, (1, 1, 0), [0.0],
                                        [[synth.T_CC_EV]], fmt="sell_f32", slice=64)
    r = synth.random_phase(N, R, w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)
    rd = G.to_dev(r)
    mu0 = tbkpm.kpm_moments_batched(H, a, b, rd, M, "c32", config=tbkpm.make_config(2, 2, 1, 0, 1, 0))
    for tpb in (1, 2, 4):
        for xr in (1, 2):
            mu1 = tbkpm.kpm_moments_batched(H, a, b, rd, M, "c32", config=tbkpm.make_config(2, tpb, 1, xr, 1, 0))
            torch.testing.assert_close(mu0, mu1, rtol=0, atol=0)
    mu = mu0.cpu().numpy()
    for k in sorted({0, len(snaps) - 1, int(np.argmin([s.n for s in snaps]))}):
        s = snaps[k]
        csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
        mu_o, _ = O.kpm_moments(csr, a[k], b[k], r[seg[k]:seg[k + 1]].astype(np.complex128), M)
        E = synth.energy_grid(a[k], b[k])
        err = G.rel_l2(O.kpm_dos(mu[k].mean(0), a[k], b[k], E), O.kpm_dos(mu_o.mean(0), a[k], b[k], E))
        print(f"[fullsize] snapshot {k}: N={s.n} DOS relL2={err:.2e}", flush=True)
        assert err <= 1e-4, (k, err)
