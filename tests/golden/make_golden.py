"""Write the oracle's full-size Chebyshev moments for vector subsets of the large workloads.

Calls only the serial FP64 oracle (oracle/) and the seeded input generators.
For each workload the oracle builds the Hamiltonian from the generated
structure, takes its Gershgorin bounds, sets a = 1.01 (E_hi - E_lo)/2 and
b = (E_hi + E_lo)/2, and runs the recurrence on the first few random-phase
vectors (the complex64 phases of the workload, widened to complex128, so the
GPU's complex-float path sees identical inputs).  Output: one text file per
workload with a header (workload, N, M, vectors, a, b) and one line per moment.

Usage: python tests/golden/make_golden.py [workload ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_2509_06525_amd import synth              # noqa: E402

# workload -> number of leading vectors the oracle follows
SUBSETS = {"graphene_thermal_1M": 2, "hbn_graphene_stripes_4M": 1, "graphene_pristine_100M": 1}


def golden_path(name):
    return os.path.join(HERE, f"oracle_moments_{name}.txt")


def make(name):
    w = synth.WORKLOADS[name]
    t0 = time.time()
    s = synth.make_structure(name)
    nv = SUBSETS[name]
    r = synth.random_phase(s.n, w["R"], w["seed"] + synth.VECTOR_SEED_OFFSET, np.complex64)
    r = np.ascontiguousarray(r[:, :nv]).astype(np.complex128)
    print(f"{name}: N={s.n}, building H", flush=True)
    csr, pairs = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    del pairs, s
    lo, hi = O.gershgorin(csr)
    a, b = 1.01 * (hi - lo) / 2.0, (hi + lo) / 2.0
    print(f"{name}: a={a!r} b={b!r}, recurrence M={w['M']} over {nv} vectors", flush=True)
    mu, im = O.kpm_moments(csr, a, b, r, w["M"])
    with open(golden_path(name), "w") as f:
        f.write(f"# oracle moments (serial FP64 oracle), written by tests/golden/make_golden.py\n")
        f.write(f"# workload {name} N {csr.n} M {w['M']} vectors {nv}\n")
        f.write(f"# a {a!r} b {b!r}\n")
        f.write(f"# max|Im| {np.abs(im).max()!r}\n")
        for n in range(w["M"]):
            f.write(" ".join(f"{mu[v, n]:.17e}" for v in range(nv)) + "\n")
    print(f"{name}: done in {time.time() - t0:.0f} s", flush=True)


def load(name):
    """(a, b, mu[v][n], n_vectors) from a golden file."""
    with open(golden_path(name)) as f:
        lines = f.readlines()
    hdr = {}
    for ln in lines[:4]:
        parts = ln[1:].split()
        for k in range(0, len(parts) - 1, 2):
            hdr[parts[k]] = parts[k + 1]
    a, b = float(hdr["a"]), float(hdr["b"])
    mu = np.loadtxt(lines[4:], ndmin=2).T
    return a, b, mu


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(SUBSETS)):
        make(name)
