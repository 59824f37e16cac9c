"""Seeded synthetic inputs: graphene-family structures and random-phase vectors.

This module only generates inputs (coordinates, species, model parameter
tables, random phases).  It contains none of the method's arithmetic and is the
one module that both the HIP path's callers and the oracle's callers use.

The paper's structures come from NEP molecular dynamics and DFT data that are
not available; thermally displaced sheets are modelled here by independent
Gaussian displacements of every coordinate of a periodic rectangular sheet.

Sheet geometry: rectangular 4-atom cells of graphene (C-C bond a = 1.42 A),
cell 3a x sqrt(3)a, zigzag direction along y.  Atoms are numbered cell-major:
index = 4 * (cy * nx + cx) + basis.  Sublattice A = basis {0, 2}, B = {1, 3}.
"""
from dataclasses import dataclass, field
import math

import numpy as np

A_CC = 1.42                                   # C-C bond length (A)
CELL_X = 3.0 * A_CC                           # 4.26 A
CELL_Y = math.sqrt(3.0) * A_CC                # 2.4595 A
BASIS = np.array([[0.0, 0.0],
                  [0.5 * A_CC, 0.5 * CELL_Y],
                  [1.5 * A_CC, 0.5 * CELL_Y],
                  [2.0 * A_CC, 0.0]])
SHEET_LZ = 20.0                               # open (non-periodic) z extent (A)

# Species table of the heterojunction model: 0 = C, 1 = B, 2 = N.
SPECIES = ("C", "B", "N")
ONSITE_EV = np.array([0.0, 2.3, -1.9])
T_PAIR_EV = np.array([[-2.7, -2.2, -2.5],
                      [-2.2, 0.0, -2.6],
                      [-2.5, -2.6, 0.0]])
T_CC_EV = -2.7

# Distance-scaled hopping model: t(r) = t_pair * exp(-BETA (r / R0 - 1)), r < R_HOP.
R0 = 1.42
BETA = 3.37
R_HOP = 2.0
R_DESC = 4.0        # descriptor cutoff of the learned model
N_RADIAL = 8        # Chebyshev radial functions per descriptor


@dataclass
class Structure:
    pos: np.ndarray            # [N][3] float64 (A)
    species: np.ndarray        # [N] int32
    box: np.ndarray            # [3] float64 (A)
    periodic: np.ndarray       # [3] int32
    onsite: np.ndarray = field(default_factory=lambda: np.array([0.0]))   # [S] eV
    t_pair: np.ndarray = field(default_factory=lambda: np.array([[T_CC_EV]]))  # [S][S] eV
    nx: int = 0
    ny: int = 0
    sigma: float = 0.0

    @property
    def n(self):
        return int(self.pos.shape[0])


def graphene_sheet(nx, ny, sigma=0.0, seed=None):
    """Periodic nx x ny sheet of 4-atom cells; Gaussian displacements of std sigma (A)."""
    cx = np.arange(nx, dtype=np.float64)
    cy = np.arange(ny, dtype=np.float64)
    n = 4 * nx * ny
    pos = np.empty((ny, nx, 4, 3), np.float64)
    pos[..., 0] = cx[None, :, None] * CELL_X + BASIS[None, None, :, 0]
    pos[..., 1] = cy[:, None, None] * CELL_Y + BASIS[None, None, :, 1]
    pos[..., 2] = 0.5 * SHEET_LZ
    pos = pos.reshape(n, 3)
    if sigma > 0.0:
        rng = np.random.default_rng(seed)
        pos += rng.normal(0.0, sigma, size=pos.shape)
    return Structure(pos=pos, species=np.zeros(n, np.int32),
                     box=np.array([nx * CELL_X, ny * CELL_Y, SHEET_LZ]),
                     periodic=np.array([1, 1, 0], np.int32),
                     onsite=np.array([0.0]), t_pair=np.array([[T_CC_EV]]),
                     nx=nx, ny=ny, sigma=sigma)


def hbn_stripes(nx, ny, stripe_cells=50, sigma=0.0, seed=None):
    """h-BN/graphene stripes normal to x, each `stripe_cells` cells wide.

    Even stripes are carbon; in odd stripes sublattice A (basis 0, 2) is boron
    and sublattice B (basis 1, 3) is nitrogen, so B-B and N-N bonds never occur.
    """
    s = graphene_sheet(nx, ny, sigma, seed)
    cx = np.broadcast_to(np.arange(nx)[None, :, None], (ny, nx, 4)).reshape(-1)
    b = np.broadcast_to(np.arange(4)[None, None, :], (ny, nx, 4)).reshape(-1)
    bn = (cx // stripe_cells) % 2 == 1
    sp = np.zeros(s.n, np.int32)
    sp[bn & ((b == 0) | (b == 2))] = 1
    sp[bn & ((b == 1) | (b == 3))] = 2
    s.species = sp
    s.onsite = ONSITE_EV.copy()
    s.t_pair = T_PAIR_EV.copy()
    return s


def sheet_dims_for(n_atoms):
    """Cells (nx, ny) of a near-square sheet with about n_atoms atoms."""
    nx = max(3, int(round(math.sqrt(n_atoms / (4.0 * math.sqrt(3.0))))))
    ny = max(3, int(round(math.sqrt(3.0) * nx)))
    return nx, ny


def snapshot_set(count, seed, n_min=1000, n_max=50000, sigma_lo=0.02, sigma_hi=0.08):
    """`count` thermally displaced sheets, sizes log-uniform on [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=count)
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for k in range(count):
        nx, ny = sheet_dims_for(sizes[k])
        out.append(graphene_sheet(nx, ny, float(sigmas[k]), int(seeds[k])))
    return out


def random_phase(n, R, seed, dtype=np.complex128):
    """Random-phase vectors r[i, v] = exp(i phi), phi ~ U[0, 2 pi): shape [n][R]."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n, R))
    out = np.empty((n, R), dtype)
    out.real = np.cos(phi)
    out.imag = np.sin(phi)
    return out


def energy_grid(a, b, n=2001, lo=None, hi=None):
    """Uniform grid; defaults to [b - 0.99 a, b + 0.99 a]."""
    if lo is None:
        lo = b - 0.99 * a
    if hi is None:
        hi = b + 0.99 * a
    return np.linspace(lo, hi, n)


# ---------------------------------------------------------------------------
# Named workloads (sizes, seeds and KPM settings).
# ---------------------------------------------------------------------------

WORKLOADS = {
    "graphene_pristine_2304": dict(kind="sheet", nx=24, ny=24, sigma=0.0, M=256, R=4,
                                   fmt="csr_f64", precision="f64", a=9.0, b=0.0,
                                   e_lo=-8.5, e_hi=8.5, n_e=2001, seed=1000),
    "graphene_thermal_1M": dict(kind="sheet", nx=500, ny=500, sigma=0.05, M=3000, R=16,
                                fmt="sell_f32", precision="c32", seed=1001),
    "hbn_graphene_stripes_4M": dict(kind="stripes", nx=1000, ny=1000, sigma=0.03, M=2000,
                                    R=32, fmt="sell_f32", precision="c32", seed=1002),
    "graphene_snapshots_256": dict(kind="snapshots", count=256, M=1024, R=8,
                                   fmt="sell_f32", precision="c32", seed=3004,
                                   train_seed=4004),
    "graphene_pristine_100M": dict(kind="sheet", nx=5000, ny=5000, sigma=0.0, M=1000, R=1,
                                   fmt="sell_f32", precision="c32", seed=1004),
    # s, p Slater-Koster orbital Hamiltonian (4 orbitals per atom: 4,000,000 rows)
    "graphene_sp3_thermal_1M": dict(kind="sheet", nx=500, ny=500, sigma=0.05, M=3000, R=16,
                                    fmt="bsell4_f32", precision="c32", seed=1006, sk=True),
    # s, p, d Slater-Koster orbital Hamiltonian (9 orbitals per atom: 9,000,000 rows)
    "graphene_spd_thermal_1M": dict(kind="sheet", nx=500, ny=500, sigma=0.05, M=1000, R=16,
                                    fmt="bsell4_f32", precision="c32", seed=1007, sk=True, orbitals=9),
    # s, p, d model with a third-neighbour cutoff on 100 M atoms (900 M orbital rows), the size of
    # the paper's largest DOS; bonds stored as displacements, blocks formed in the recurrence
    "graphene_spd_3nn_100M": dict(kind="sheet", nx=5000, ny=5000, sigma=0.05, M=1000, R=1,
                                  fmt="bgeom_f32", precision="c32", seed=1008, sk=True, orbitals=9, r_cut=3.0),
    # velocity autocorrelation: 200 propagation steps of 0.1 fs (20 fs of correlation time)
    "graphene_thermal_1M_vac": dict(kind="sheet", nx=500, ny=500, sigma=0.05, M=1000, R=1,
                                    fmt="sell_f32", precision="c32", seed=1005, vac=True,
                                    n_t=200, dt=0.1),
    # velocity autocorrelation on the s, p block Hamiltonian (100,800 atoms, 403,200 orbital rows)
    "graphene_sp3_thermal_100k_vac": dict(kind="sheet", nx=160, ny=158, sigma=0.05, M=1000, R=1,
                                          fmt="bsell4_f32", precision="c32", seed=1009, vac=True, sk=True,
                                          orbitals=4, n_t=200, dt=0.1),
    # four thermal frames of a 1 M-atom sheet (seeds 1010..1013): VAC conductivity and integrated
    # DOS of each frame, frame average, carriers and mobility
    "graphene_mobility_frames_1M": dict(kind="frames", frames=4, nx=500, ny=500, sigma=0.05, M=1000, R=1,
                                        R_dos=16, fmt="sell_f32", precision="c32", seed=1010, vac=True,
                                        n_t=200, dt=0.1),
}
VECTOR_SEED_OFFSET = 1000   # vector seed = structure seed + 1000

# Synthetic s, p Slater-Koster parameters of carbon (eV at R0): V_ss_sigma, V_sp_sigma,
# V_pp_sigma, V_pp_pi, and onsite e_s, e_p.  Round stand-ins of the magnitudes of
# published sp3 carbon sets, not a fit.
SK_V = (-5.7, 5.4, 6.2, -2.7)
SK_ES, SK_EP = -7.3, 0.0
# d-orbital integrals at r0 (sd_sigma, pd_sigma, pd_pi, dd_sigma, dd_pi, dd_delta) and the d
# onsite energy of the synthetic nine-orbital model: magnitudes and signs of typical s, p, d
# tight-binding sets, not fitted to any material
SK_D = (-3.1, -2.4, 1.3, -1.9, 1.05, -0.21)
SK_ED = 6.5


def make_structure(name):
    w = WORKLOADS[name]
    if w["kind"] == "sheet":
        return graphene_sheet(w["nx"], w["ny"], w["sigma"], w["seed"])
    if w["kind"] == "stripes":
        return hbn_stripes(w["nx"], w["ny"], 50, w["sigma"], w["seed"])
    if w["kind"] == "frames":
        return graphene_sheet(w["nx"], w["ny"], w["sigma"], w["seed"])
    raise ValueError("use snapshot_set for the snapshot workload")


def make_frames(name):
    """The frames of a multi-frame workload: the same sheet with independent
    displacements (seeds seed, seed + 1, ...)."""
    w = WORKLOADS[name]
    return [graphene_sheet(w["nx"], w["ny"], w["sigma"], w["seed"] + f) for f in range(w.get("frames", 1))]


# ---------------------------------------------------------------------------
# Learned-hopping workload: seeded initial MLP parameters and target constants.
# ---------------------------------------------------------------------------

MLP_SHAPES = ((32, 16), (32,), (32, 32), (32,), (32,), (1,))   # W1, b1, W2, b2, W3, b3
MLP_N_PARAMS = 1633
COORD_KAPPA = 0.25          # strength of the coordination correction of the target hoppings
COORD_Z0 = 4.7357           # pristine coordination sum_j f_c(r_ij) within 4.0 A (rounded)
# per-integral strengths of the coordination correction of the learned Slater-Koster
# workload's target (ss_sigma, sp_sigma, pp_sigma, pp_pi, then the six d integrals)
SK_COORD_KAPPA = (0.25, -0.15, 0.2, 0.3, 0.1, -0.2, 0.15, 0.25, -0.1, 0.05)


# Training of the snapshot workload's learned-hopping network: bonds of 128 sheets of the
# seed-4004 set (sizes log-uniform on 1k-50k atoms, sigma in [0.02, 0.08] A, disjoint from
# the evaluation set), minibatches of 2048 bonds in a shuffled order, AdamW with a learning
# rate stepped down over 150 epochs (epochs, rate).
LEARNED_TRAINING = dict(count=128, seed=4004, n_min=1000, n_max=50000, batch=2048, shuffle_seed=5,
                        schedule=((80, 2e-3), (40, 5e-4), (30, 1e-4)), wd=1e-5, init_seed=11)


def init_mlp_params(seed, out_scale=0.1):
    """Seeded initial parameters (float32): uniform(+-1/sqrt(fan_in)) weights, zero biases,
    output layer scaled by out_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = 1.0 / math.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        elif shape == (32,) and len(parts) == 4:       # W3
            parts.append(rng.uniform(-out_scale, out_scale, size=shape) / math.sqrt(32))
        else:
            parts.append(np.zeros(shape))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_N_PARAMS
    return p


def stack(structures):
    """Concatenate structures: positions, species, segment offsets, boxes."""
    pos = np.concatenate([s.pos for s in structures])
    sp = np.concatenate([s.species for s in structures])
    seg = np.concatenate([[0], np.cumsum([s.n for s in structures])]).astype(np.int64)
    boxes = np.array([s.box for s in structures])
    return pos, sp, seg, boxes
