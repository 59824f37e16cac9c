"""Independent references that pin the oracle (test code, numpy only).

None of these call the oracle: they are closed forms, library routines (dense
eigvalsh, numpy's Chebyshev series) and brute-force geometry, chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand) disagrees with at least one of them.
"""
import math

import numpy as np
from numpy.polynomial import chebyshev as npcheb

from paper_2509_06525_amd import synth


def cheb_T(n_max, x):
    """T_n(x) for n = 0..n_max-1 and |x| <= 1 via cos(n arccos x): [n_max][len(x)]."""
    x = np.clip(np.asarray(x, np.float64), -1.0, 1.0)
    th = np.arccos(x)
    n = np.arange(n_max, dtype=np.float64)[:, None]
    return np.cos(n * th[None, :])


def trace_moments_from_eigs(eigs, a, b, M, chunk=200000):
    """Full-trace moments sum_k T_n((lambda_k - b)/a), n < M, from a spectrum."""
    x = (np.asarray(eigs, np.float64) - b) / a
    out = np.zeros(M)
    for s in range(0, x.size, chunk):
        out += cheb_T(M, x[s:s + chunk]).sum(axis=1)
    return out


def brute_pairs(pos, box, periodic, r_cut):
    """All i<j pairs with minimum-image distance < r_cut, by a dense distance matrix."""
    pos = np.asarray(pos, np.float64)
    d = pos[None, :, :] - pos[:, None, :]
    for k in range(3):
        if periodic[k]:
            d[..., k] -= box[k] * np.round(d[..., k] / box[k])
    r = np.sqrt((d * d).sum(-1))
    i, j = np.nonzero(np.triu(r < r_cut, 1))
    return i, j, r[i, j]


def pristine_neighbors(nx, ny):
    """Nearest-neighbour table of the rectangular-cell sheet derived from its geometry.

    Basis 0 (0,0) bonds to basis 1 of its cell, basis 1 of the cell below and
    basis 3 of the cell to the left; the other three bonds of each atom follow.
    Returns the set of unordered pairs.
    """
    def idx(cx, cy, b):
        return 4 * ((cy % ny) * nx + (cx % nx)) + b
    pairs = set()
    for cy in range(ny):
        for cx in range(nx):
            for (i, j) in [(idx(cx, cy, 0), idx(cx, cy, 1)),
                           (idx(cx, cy, 0), idx(cx, cy - 1, 1)),
                           (idx(cx, cy, 0), idx(cx - 1, cy, 3)),
                           (idx(cx, cy, 1), idx(cx, cy, 2)),
                           (idx(cx, cy, 2), idx(cx, cy, 3)),
                           (idx(cx, cy, 2), idx(cx, cy + 1, 3))]:
                pairs.add((min(i, j), max(i, j)))
    return pairs


def bloch_hamiltonian(kx, ky, t=synth.T_CC_EV):
    """4x4 Bloch H(k) of the rectangular 4-atom cell (nearest neighbours only).

    Built by enumerating the images of each basis atom in the 3x3 block of
    neighbouring cells and keeping those at the bond length; H_bc(k) =
    sum_R t exp(i k . R) in the periodic gauge.  kx, ky are arrays.
    """
    kx = np.atleast_1d(np.asarray(kx, np.float64))
    ky = np.atleast_1d(np.asarray(ky, np.float64))
    H = np.zeros(kx.shape + (4, 4), np.complex128)
    tau = synth.BASIS
    for b in range(4):
        for c in range(4):
            for mx in (-1, 0, 1):
                for my in (-1, 0, 1):
                    R = np.array([mx * synth.CELL_X, my * synth.CELL_Y])
                    d = tau[c] + R - tau[b]
                    if abs(math.hypot(d[0], d[1]) - synth.A_CC) < 1e-6:
                        H[..., b, c] += t * np.exp(1j * (kx * R[0] + ky * R[1]))
    return H


def supercell_spectrum(nx, ny, t=synth.T_CC_EV):
    """Exact spectrum of the periodic nx x ny pristine sheet via commensurate k points."""
    mx, my = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    kx = 2.0 * math.pi * mx.reshape(-1) / (nx * synth.CELL_X)
    ky = 2.0 * math.pi * my.reshape(-1) / (ny * synth.CELL_Y)
    out = []
    for s in range(0, kx.size, 100000):
        out.append(np.linalg.eigvalsh(bloch_hamiltonian(kx[s:s + 100000], ky[s:s + 100000], t)).reshape(-1))
    return np.concatenate(out)


def cheb_radial_ref(r, rc, nk):
    """f_k(r) from numpy's Chebyshev series evaluation and the cosine cutoff."""
    x = 2.0 * (r / rc - 1.0) ** 2 - 1.0
    fc = 0.5 * (1.0 + math.cos(math.pi * r / rc)) if r < rc else 0.0
    return np.array([0.5 * (npcheb.chebval(x, np.eye(nk)[k]) + 1.0) * fc for k in range(nk)])
