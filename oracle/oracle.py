"""ctypes binding of the serial FP64 oracle (test infrastructure only).

Each function passes numpy arrays to one C routine of tbkpm_oracle.c and
returns numpy arrays; there is no arithmetic of the method here beyond
argument marshalling, except the small compositions at the bottom that chain
oracle routines in the order the path runs them.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f64 = ctypes.c_double


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    L = ctypes.CDLL(path)
    L.orc_neighbor_pairs.restype = _i64
    L.orc_neighbor_pairs.argtypes = [_i64, _f64p, _f64p, _i32p, _f64, _i64, _i32p, _i32p, _f64p]
    L.orc_assemble_csr.restype = ctypes.c_int
    L.orc_assemble_csr.argtypes = [_i64, _i32p, _i32, _f64p, _f64p, _f64, _f64, _i64,
                                   _i32p, _i32p, _f64p, ctypes.c_void_p,
                                   _i64p, _i32p, _f64p, _f64p]
    L.orc_gershgorin.restype = None
    L.orc_gershgorin.argtypes = [_i64, _i64p, _f64p, _f64p, _f64p]
    L.orc_kpm_moments.restype = ctypes.c_int
    L.orc_kpm_moments.argtypes = [_i64, _i64p, _i32p, _f64p, _f64p, _f64, _f64,
                                  _c128p, _i32, _i32, _f64p, _f64p]
    L.orc_kpm_moments_state.restype = ctypes.c_int
    L.orc_kpm_moments_state.argtypes = [_i64, _i64p, _i32p, _f64p, _f64p, _f64, _f64,
                                        _c128p, _i32, _i32, _i32, _c128p, _f64p, _f64p]
    L.orc_jackson.restype = None
    L.orc_jackson.argtypes = [_i32, _f64p]
    L.orc_kpm_dos.restype = ctypes.c_int
    L.orc_kpm_dos.argtypes = [_f64p, _i32, _f64, _f64, _i32, _f64p, _i32, _f64p]
    L.orc_radial.restype = None
    L.orc_radial.argtypes = [_f64, _f64, _i32, _f64p]
    L.orc_descriptor.restype = None
    L.orc_descriptor.argtypes = [_i64, _i64, _i32p, _i32p, _f64p, _f64, _i32, ctypes.c_void_p, _i32,
                                 ctypes.c_void_p, _f64p]
    L.orc_bf16.restype = _f64
    L.orc_bf16.argtypes = [_f64]
    L.orc_mlp_forward.restype = None
    L.orc_mlp_forward.argtypes = [_i64, _f64p, _f64p, _i32, _f64p, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_mlp_loss_grad.restype = _f64
    L.orc_mlp_loss_grad.argtypes = [_i64, _f64p, _f64p, ctypes.c_void_p, _f64p, _i32, _f64p]
    L.orc_bond_features.restype = None
    L.orc_bond_features.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64, _i32, ctypes.c_void_p, _i32,
                                    ctypes.c_void_p, _f64p, _f64p, _f64p]
    L.orc_target_scale.restype = None
    L.orc_target_scale.argtypes = [_i64, _i32p, _i32p, _f64p, _i32, _f64, _f64, _f64p]
    L.orc_adamw_step.restype = None
    L.orc_adamw_step.argtypes = [_i64, _f64p, _f64p, _f64p, _f64p, _i64, _f64, _f64, _f64, _f64, _f64]
    L.orc_velocity_values.restype = None
    L.orc_velocity_values.argtypes = [_i64, _i64p, _i32p, _f64p, _f64p, _f64p, _i32p, _i32, _i32, _f64p]
    L.orc_evolve.restype = ctypes.c_int
    L.orc_evolve.argtypes = [_i64, _i64p, _i32p, _f64p, _f64p, _f64, _f64, _f64, _i32, _c128p]
    L.orc_vac_moments.restype = ctypes.c_int
    L.orc_vac_moments.argtypes = [_i64, _i64p, _i32p, _f64p, _f64p, _f64p, _f64, _f64, _c128p, _i32, _i32,
                                  _i32, _f64, _i32, _f64p]
    L.orc_vac_sigma.restype = ctypes.c_int
    L.orc_vac_sigma.argtypes = [_f64p, _i32, _i32, _f64, _f64, _f64, _i32, _f64p, _i32, _f64p]
    L.orc_assemble_sk.restype = ctypes.c_int
    L.orc_integrated_dos.restype = ctypes.c_int
    L.orc_integrated_dos.argtypes = [_f64p, _i32, _f64, _f64, _i32, _f64p, _i32, _f64p]
    L.orc_mobility.restype = ctypes.c_int
    L.orc_mobility.argtypes = [_f64p, _i32, _i32, _i32, _f64p, _f64, _f64p, _f64p, _f64p]
    L.orc_assemble_sk.argtypes = [_i64, _f64p, _f64p, _i32p, _i64, _i32p, _i32p, _i32, _f64p, ctypes.c_void_p,
                                  _f64p, ctypes.c_void_p, _i32, ctypes.c_void_p, ctypes.c_void_p, _f64, _f64,
                                  _i64p, _i32p, _f64p, _f64p]
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_random_phase.restype = None
    L.orc_random_phase.argtypes = [_i64, _i32, ctypes.c_uint64, _f64p, _f64p]
    _LIB = L
    return L


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Geometry and Hamiltonian
# --------------------------------------------------------------------------

def neighbor_pairs(pos, box, periodic, r_cut):
    """Pairs i<j with minimum-image distance < r_cut: (pi, pj, dist)."""
    pos = _c(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    box = _c(box, np.float64)
    per = _c(periodic, np.int32)
    cap = max(16, 4 * n)
    while True:
        pi = np.empty(cap, np.int32)
        pj = np.empty(cap, np.int32)
        d = np.empty(cap, np.float64)
        cnt = _lib().orc_neighbor_pairs(n, pos.reshape(-1), box, per, float(r_cut), cap, pi, pj, d)
        if cnt < 0:
            raise OracleError("orc_neighbor_pairs: invalid argument")
        if cnt <= cap:
            return pi[:cnt].copy(), pj[:cnt].copy(), d[:cnt].copy()
        cap = int(cnt)


class CSR:
    """Off-diagonal CSR part plus the onsite diagonal of H (both FP64)."""

    def __init__(self, row_ptr, col, val, diag):
        self.row_ptr, self.col, self.val, self.diag = row_ptr, col, val, diag

    @property
    def n(self):
        return self.diag.shape[0]

    def dense(self):
        n = self.n
        H = np.zeros((n, n))
        for i in range(n):
            for q in range(self.row_ptr[i], self.row_ptr[i + 1]):
                H[i, self.col[q]] += self.val[q]
            H[i, i] += self.diag[i]
        return H


def assemble_csr(n, species, n_species, onsite, t_pair, r0, beta, pairs, t_scale=None):
    pi, pj, d = pairs
    npairs = pi.shape[0]
    row_ptr = np.empty(n + 1, np.int64)
    col = np.empty(2 * npairs, np.int32)
    val = np.empty(2 * npairs, np.float64)
    diag = np.empty(n, np.float64)
    ts = None
    if t_scale is not None:
        ts = _c(t_scale, np.float64)
        assert ts.shape[0] == npairs
    rc = _lib().orc_assemble_csr(n, _c(species, np.int32), int(n_species), _c(onsite, np.float64),
                                 _c(t_pair, np.float64).reshape(-1), float(r0), float(beta), npairs,
                                 pi, pj, d, None if ts is None else ts.ctypes.data,
                                 row_ptr, col, val, diag)
    if rc != 0:
        raise OracleError("orc_assemble_csr: invalid argument")
    return CSR(row_ptr, col, val, diag)


def gershgorin(csr):
    out = np.empty(2)
    _lib().orc_gershgorin(csr.n, csr.row_ptr, csr.val, csr.diag, out)
    return float(out[0]), float(out[1])


# --------------------------------------------------------------------------
# KPM
# --------------------------------------------------------------------------

def kpm_moments(csr, a, b, r, M):
    """mu_re, mu_im of shape [R][M] for vectors r [N][R] (complex128)."""
    r = _c(r, np.complex128)
    if r.ndim == 1:
        r = r.reshape(-1, 1)
    n, R = r.shape
    assert n == csr.n
    mu_re = np.empty((R, M))
    mu_im = np.empty((R, M))
    rc = _lib().orc_kpm_moments(n, csr.row_ptr, csr.col, csr.val, csr.diag, float(a), float(b),
                                r.reshape(-1), R, M, mu_re, mu_im)
    if rc != 0:
        raise OracleError("orc_kpm_moments: invalid argument")
    return mu_re, mu_im


def kpm_moments_state(csr, a, b, r, M, n_start=0, state=None, mu_re=None, mu_im=None):
    """The recurrence split over calls: moments n_start..M-1 written into mu_re, mu_im [R][M]
    (allocated when None), state [R][2][N] complex128 carrying the last two vectors (allocated
    when None and n_start = 0).  Returns (mu_re, mu_im, state)."""
    r = _c(r, np.complex128)
    if r.ndim == 1:
        r = r.reshape(-1, 1)
    n, R = r.shape
    assert n == csr.n
    if state is None:
        state = np.zeros((R, 2, n), dtype=np.complex128)
    mu_re = np.full((R, M), np.nan) if mu_re is None else mu_re
    mu_im = np.full((R, M), np.nan) if mu_im is None else mu_im
    rc = _lib().orc_kpm_moments_state(n, csr.row_ptr, csr.col, csr.val, csr.diag, float(a), float(b),
                                      r.reshape(-1), R, M, int(n_start), state.reshape(-1), mu_re, mu_im)
    if rc != 0:
        raise OracleError("orc_kpm_moments_state: invalid argument")
    return mu_re, mu_im, state


def jackson(M):
    g = np.empty(M)
    _lib().orc_jackson(M, g)
    return g


def kpm_dos(mu, a, b, E, kernel=0):
    mu = _c(mu, np.float64)
    E = _c(E, np.float64)
    rho = np.empty(E.shape[0])
    rc = _lib().orc_kpm_dos(mu, mu.shape[0], float(a), float(b), int(kernel), E, E.shape[0], rho)
    if rc != 0:
        raise OracleError("orc_kpm_dos: invalid argument")
    return rho


# --------------------------------------------------------------------------
# Learned hoppings
# --------------------------------------------------------------------------

def radial(r, rc, nk=8):
    f = np.empty(nk)
    _lib().orc_radial(float(r), float(rc), nk, f)
    return f


def _species_cnk(species, cnk, nk):
    if cnk is None:
        return None, 0, None
    c = np.ascontiguousarray(np.asarray(cnk, np.float64))
    ns = c.shape[0]
    assert c.shape == (ns, ns, nk, nk)
    return np.ascontiguousarray(np.asarray(species, np.int32)), ns, c


def descriptor(n, pairs, rc, nk=8, species=None, cnk=None):
    """Node features v [n][nk] = sum_j C(r_ij); cnk [ns][ns][nk][nk] per species pair
    (None: identity)."""
    pi, pj, d = pairs
    v = np.empty((n, nk))
    sp, ns, c = _species_cnk(species, cnk, nk)
    _lib().orc_descriptor(n, pi.shape[0], pi, pj, d, float(rc), nk, None if sp is None else sp.ctypes.data, ns,
                          None if c is None else c.ctypes.data, v.reshape(-1))
    return v


def bf16(x):
    f = _lib().orc_bf16
    x = np.asarray(x, np.float64)
    return np.vectorize(f, otypes=[np.float64])(x) if x.ndim else f(float(x))


N_PARAMS = 1633


def bond_features(pairs, v, rc, shift=None, scale=None, species=None, cnk=None):
    """[npairs][2 nk] MLP inputs [C(r_ij) || v_i + v_j], standardised by (shift, scale);
    C = f without cnk."""
    pi, pj, d = pairs
    nk = v.shape[1]
    shift = np.zeros(2 * nk) if shift is None else _c(shift, np.float64)
    scale = np.ones(2 * nk) if scale is None else _c(scale, np.float64)
    X = np.empty((pi.shape[0], 2 * nk))
    sp, ns, c = _species_cnk(species, cnk, nk)
    _lib().orc_bond_features(pi.shape[0], pi, pj, d, _c(v, np.float64).reshape(-1), float(rc), nk,
                             None if sp is None else sp.ctypes.data, ns, None if c is None else c.ctypes.data,
                             shift, scale, X.reshape(-1))
    return X


def target_scale(pairs, v, kappa, z0):
    """Coordination-corrected hopping factor 1 + kappa (z_i + z_j - 2 z0) per pair."""
    pi, pj, _ = pairs
    out = np.empty(pi.shape[0])
    _lib().orc_target_scale(pi.shape[0], pi, pj, _c(v, np.float64).reshape(-1), v.shape[1],
                            float(kappa), float(z0), out)
    return out


HBAR_EV_FS = 0.6582119569


def velocity_values(csr, pos, box, periodic, axis=0, n_orb=1):
    """vx[q] = H_ij (x_j - x_i) / hbar per CSR entry (V = i vx), Angstrom / fs; with
    n_orb orbitals per atom the positions are those of the orbitals' atoms."""
    vx = np.empty(csr.col.shape[0])
    _lib().orc_velocity_values(csr.n, csr.row_ptr, csr.col, csr.val, _c(pos, np.float64).reshape(-1),
                               _c(box, np.float64), _c(periodic, np.int32), int(axis), int(n_orb), vx)
    return vx


def evolve(csr, a, b, dt, n_cheb, psi):
    """exp(-i H dt / hbar) psi (dt in fs) by a Chebyshev-Bessel series of n_cheb terms."""
    out = _c(psi, np.complex128).copy()
    rc = _lib().orc_evolve(csr.n, csr.row_ptr, csr.col, csr.val, csr.diag, float(a), float(b), float(dt),
                           int(n_cheb), out)
    if rc != 0:
        raise OracleError("orc_evolve: invalid argument")
    return out


def vac_moments(csr, vx, a, b, r, M, n_t, dt, n_cheb):
    """nu [n_t][R][M] = Re <phi_L(t_j)| T_m(Ht) V |phi_R(t_j)> for start vectors r [N][R]."""
    r = _c(r, np.complex128)
    if r.ndim == 1:
        r = r.reshape(-1, 1)
    n, R = r.shape
    nu = np.empty((n_t, R, M))
    rc = _lib().orc_vac_moments(n, csr.row_ptr, csr.col, csr.val, csr.diag, _c(vx, np.float64), float(a),
                                float(b), r.reshape(-1), R, M, n_t, float(dt), int(n_cheb), nu.reshape(-1))
    if rc != 0:
        raise OracleError("orc_vac_moments: invalid argument")
    return nu


def vac_sigma(nu, a, b, dt, E, kernel=0):
    """Running time integral s [n_t][nE] of the KPM-reconstructed correlation (nu [n_t][M])."""
    nu = _c(nu, np.float64)
    n_t, M = nu.shape
    E = _c(E, np.float64)
    s = np.empty((n_t, E.shape[0]))
    rc = _lib().orc_vac_sigma(nu.reshape(-1), M, n_t, float(dt), float(a), float(b), int(kernel), E,
                              E.shape[0], s.reshape(-1))
    if rc != 0:
        raise OracleError("orc_vac_sigma: invalid argument")
    return s


def integrated_dos(mu, a, b, E, kernel=0):
    """N(E): states below E of the kernel-damped expansion (closed form), whole system."""
    mu = _c(mu, np.float64)
    E = _c(E, np.float64)
    N = np.empty(E.shape[0])
    if _lib().orc_integrated_dos(mu, mu.shape[0], float(a), float(b), int(kernel), E, E.shape[0], N) != 0:
        raise OracleError("orc_integrated_dos: invalid argument")
    return N


def mobility(sigma, N, n_ref):
    """Frame-averaged semiclassical conductivity, carriers and mobility (cm^2/(V s)):
    sigma [F][n_t][nE] running conductivities, N [F][nE] integrated DOS of each frame."""
    sigma = _c(sigma, np.float64)
    N = _c(N, np.float64)
    F, n_t, nE = sigma.shape
    ssc, car, mob = np.empty(nE), np.empty(nE), np.empty(nE)
    if _lib().orc_mobility(sigma.reshape(-1), F, n_t, nE, N.reshape(-1), float(n_ref), ssc, car, mob) != 0:
        raise OracleError("orc_mobility: invalid argument")
    return ssc, car, mob


def node_features(v, shift, scale):
    """Onsite-network inputs of Eq. (2) (the node feature v_i): [(v_i - shift) / scale || 0 x 8],
    rounded to bfloat16 (16 inputs, as the bond network's)."""
    v = np.asarray(v, np.float64)
    X = np.zeros((v.shape[0], 16))
    X[:, :8] = (v - np.asarray(shift, np.float64)) / np.asarray(scale, np.float64)
    return bf16(X)


def sk_hamiltonian(pos, box, periodic, v, e_s, e_p, r_cut=2.0, r0=1.42, beta=3.37, pairs=None, e_d=0.0,
                   scale=None, species=None, pair_v=None, species_e=None, onsite_add=None):
    """Slater-Koster orbital Hamiltonian as a CSR: v holds 4 integrals (s, p: orbital 4 i + a,
    a = s, x, y, z) or 10 (s, p, d: orbital 9 i + a, then dxy, dyz, dzx, dx2-y2, d3z2-r2)
    at r0; scale [npairs][len(v)] (optional) multiplies each pair's integrals (learned form).
    Several species: species [n], pair_v [ns][ns][len(v)] (ordered pair, lower angular
    momentum on the first species), species_e [ns][3] replace v and e_s, e_p, e_d.
    onsite_add [n][3] (optional): added to the onsite energy of each atom's s, p, d shell
    (the onsite network of Eq. (2)).  Returns (csr, pairs)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    if pairs is None:
        pairs = neighbor_pairs(pos, box, periodic, r_cut)
    pi, pj, _ = pairs
    v = np.asarray(v, np.float64)
    norb = 4 if v.size == 4 else 9
    if pair_v is not None:
        norb = 4 if np.asarray(pair_v).shape[2] == 4 else 9
    v10 = np.zeros(10)
    v10[: v.size] = v
    n = pos.shape[0]
    npairs = pi.shape[0]
    row_ptr = np.empty(norb * n + 1, np.int64)
    col = np.empty(2 * norb * norb * npairs, np.int32)
    val = np.empty(2 * norb * norb * npairs)
    diag = np.empty(norb * n)
    sc = None
    if scale is not None:
        scale = np.asarray(scale, np.float64).reshape(npairs, -1)
        sc = np.ones((npairs, 10))
        sc[:, : scale.shape[1]] = scale
    sp_a = pv = se = None
    ns = 0
    if pair_v is not None:
        pv0 = np.asarray(pair_v, np.float64)
        ns = pv0.shape[0]
        pv = np.zeros((ns, ns, 10))
        pv[:, :, : pv0.shape[2]] = pv0
        se = np.ascontiguousarray(np.asarray(species_e, np.float64).reshape(ns, 3))
        sp_a = np.ascontiguousarray(np.asarray(species, np.int32))
    rc = _lib().orc_assemble_sk(n, _c(pos, np.float64).reshape(-1), _c(box, np.float64), _c(periodic, np.int32),
                                npairs, pi, pj, norb, v10, None if sc is None else sc.ctypes.data,
                                np.array([e_s, e_p, e_d], np.float64),
                                None if sp_a is None else sp_a.ctypes.data, ns,
                                None if pv is None else pv.ctypes.data, None if se is None else se.ctypes.data,
                                float(r0), float(beta), row_ptr, col, val, diag)
    if rc != 0:
        raise OracleError("orc_assemble_sk failed")
    if onsite_add is not None:
        add = np.asarray(onsite_add, np.float64).reshape(n, 3)
        shell = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2])[:norb]
        diag = diag + add[:, shell].reshape(-1)
    return CSR(row_ptr, col, val, diag), pairs


def splitmix64(seed, k):
    """Output number k of SplitMix64 started at state `seed`."""
    return int(_lib().orc_splitmix64(int(seed) & (2**64 - 1), int(k)))


def random_phase(n, R, seed):
    """complex128 [n, R] counter-based random phases exp(2 pi i u(seed, i R + v))."""
    re = np.empty(n * R)
    im = np.empty(n * R)
    _lib().orc_random_phase(n, R, int(seed) & (2**64 - 1), re, im)
    return (re + 1j * im).reshape(n, R)


def mlp_forward(X, prm, bf16_ops=True, keep=False):
    X = _c(X, np.float64)
    B = X.shape[0]
    y = np.empty(B)
    h1 = np.empty((B, 32)) if keep else None
    h2 = np.empty((B, 32)) if keep else None
    _lib().orc_mlp_forward(B, X.reshape(-1), _c(prm, np.float64), int(bool(bf16_ops)), y,
                           None if h1 is None else h1.ctypes.data,
                           None if h2 is None else h2.ctypes.data)
    return (y, h1, h2) if keep else y


def mlp_loss_grad(X, target, prm, w=None, bf16_ops=True):
    X = _c(X, np.float64)
    B = X.shape[0]
    g = np.empty(N_PARAMS)
    wv = None if w is None else _c(w, np.float64)
    loss = _lib().orc_mlp_loss_grad(B, X.reshape(-1), _c(target, np.float64),
                                    None if wv is None else wv.ctypes.data,
                                    _c(prm, np.float64), int(bool(bf16_ops)), g)
    return loss, g


def adamw_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-2):
    """In-place AdamW update of float64 arrays p, m, v (step count t after the update)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _lib().orc_adamw_step(p.shape[0], p, _c(g, np.float64), m, v, int(t), float(lr),
                          float(beta1), float(beta2), float(eps), float(wd))


# --------------------------------------------------------------------------
# Compositions in path order
# --------------------------------------------------------------------------

def hamiltonian(pos, species, box, periodic, onsite, t_pair, r_cut=2.0, r0=1.42, beta=3.37,
                t_scale=None, pairs=None):
    """Neighbour pairs, then the CSR Hamiltonian of Eq. (1); returns (csr, pairs)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    if pairs is None:
        pairs = neighbor_pairs(pos, box, periodic, r_cut)
    t_pair = np.asarray(t_pair, np.float64)
    S = int(round(np.sqrt(t_pair.size)))
    csr = assemble_csr(pos.shape[0], species, S, onsite, t_pair, r0, beta, pairs, t_scale)
    return csr, pairs
