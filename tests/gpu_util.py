"""Helpers shared by the GPU tests: device transfers and decoding of the library's
Hamiltonian arrays into the caller's atom order (test code only)."""
import numpy as np
import torch

from paper_2509_06525_amd import synth, tbkpm

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def build(s, fmt="sell_f64", slice=64, reorder=True, r_cut=synth.R_HOP):
    return tbkpm.build_hamiltonian(to_dev(s.pos, torch.float64), to_dev(s.species, torch.int32),
                                   s.box, s.periodic, s.onsite, s.t_pair, r_cut=r_cut,
                                   r0=synth.R0, beta=synth.BETA, fmt=fmt, slice=slice, reorder=reorder)


def entries_in_atom_order(H, values=None):
    """(rows, cols, vals, onsite) of the stored non-padding entries, mapped back to atom indices.
    `values` (a tensor in H's entry layout, e.g. velocity coefficients) replaces H's values."""
    t = {k: v.cpu().numpy() for k, v in H.tensors.items()}
    n = H.n_rows
    C = 1 if H.fmt == tbkpm.FORMATS["csr_f64"] else H.st.slice
    with np.errstate(invalid="ignore"):      # lanes past the last row of the last slice are never written
        ptr, col, val, perm = t["ptr"], t["col"], t["val"].astype(np.float64), t["perm"]
    other = None if values is None else values.cpu().numpy().astype(np.float64)
    rows, cols, vals = [], [], []
    for s in range(ptr.shape[0] - 1):
        w = (ptr[s + 1] - ptr[s]) // C
        for lane in range(C):
            i = s * C + lane
            if i >= n:
                break
            for k in range(w):
                q = ptr[s] + k * C + lane
                if col[q] == i and val[q] == 0.0:
                    continue        # padding
                rows.append(perm[i]); cols.append(perm[col[q]])
                vals.append(val[q] if other is None else other[q])
    onsite = np.empty(n)
    onsite[perm] = t["onsite"].astype(np.float64)
    return np.array(rows), np.array(cols), np.array(vals), onsite


def block_entries(H, values=None):
    """(rows, cols, vals, onsite) in the caller's orbital order from a block Hamiltonian;
    `values` (a tensor in H's block value layout, e.g. velocity coefficients) replaces H's values."""
    t = {k: v.cpu().numpy() for k, v in H.tensors.items()}
    no = H.st.n_orb
    n_at = H.n_rows // no
    C = H.st.slice
    ptr, col, perm = t["ptr"], t["col"], t["perm"]
    nv = no * no * H.st.n_entries
    with np.errstate(invalid="ignore"):      # lanes past the last atom of the last slice are never written
        val = t["val"][:nv].astype(np.float64).reshape(-1, no, no)
        other = None if values is None else values.cpu().numpy()[:nv].astype(np.float64).reshape(-1, no, no)
    rows, cols, vals = [], [], []
    for sl in range(ptr.shape[0] - 1):
        w = (ptr[sl + 1] - ptr[sl]) // C
        for lane in range(C):
            r = sl * C + lane
            if r >= n_at:
                break
            for k in range(w):
                q = ptr[sl] + k * C + lane
                c = col[q]
                if c == r and not val[q].any():
                    continue                     # padding block
                rr = perm[no * r + np.arange(no)]
                cc = perm[no * c + np.arange(no)]
                rows.append(np.repeat(rr, no)); cols.append(np.tile(cc, no))
                vals.append((val[q] if other is None else other[q]).reshape(-1))
    onsite = np.empty(H.n_rows)
    onsite[perm] = t["onsite"].astype(np.float64)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), onsite


def oracle_ab(csr, margin=1.01):
    """(a, b) from the oracle's Gershgorin bounds of csr: the scale a parity test gives
    both sides (the GPU's own bounds are tested against the same oracle bounds)."""
    from oracle import oracle as O
    lo, hi = O.gershgorin(csr)
    return margin * (hi - lo) / 2.0, (hi + lo) / 2.0


def oracle_ab_of(s, margin=1.01):
    """oracle_ab of the one-orbital Hamiltonian of structure s."""
    from oracle import oracle as O
    csr, _ = O.hamiltonian(s.pos, s.species, s.box, s.periodic, s.onsite, s.t_pair)
    return oracle_ab(csr, margin)


def oracle_scales(structures, margin=1.01):
    """Lists (a, b) of oracle_ab_of over stacked structures."""
    ab = [oracle_ab_of(s, margin) for s in structures]
    return [x[0] for x in ab], [x[1] for x in ab]


def csr_entries(csr):
    rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    return rows, csr.col.astype(np.int64), csr.val


def rel_l2(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def bf16_decisions_clear(h1, h2, eps=1e-6):
    """Per bond: True when every hidden activation (oracle, FP64) lies more than
    eps from a bfloat16 rounding boundary.  The GPU forms these activations in
    FP32 (error ~1e-8), so for such bonds both sides round every MFMA operand
    the same way and the outputs agree to FP32 accumulation error; a bond with
    an activation inside the band may round it one bf16 ulp apart."""
    h = np.concatenate([h1, h2], axis=1)
    from oracle import oracle as O
    flip = O.bf16(h + eps) != O.bf16(h - eps)
    return ~flip.any(axis=1)
