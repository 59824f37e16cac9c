"""Thin ctypes binding of libtbkpm.so (C ABI in include/tbkpm.h).

Arguments are marshalled from torch tensors (device memory) and Python
numbers; every step of the computation runs in the library's HIP kernels.
The binding raises TBKError when the library reports an error and refuses to
run when the library is not built: there is no fallback path.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtbkpm.so")

TBK_OK = 0
TBK_ERR_INVALID_ARG = 1
TBK_ERR_BUFFER_TOO_SMALL = 2
TBK_ERR_NOT_FINITE = 3
TBK_ERR_SPECTRUM = 4
TBK_MLP_PARAMS = 1633      # parameters of one per-bond network (W1, b1, W2, b2, W3, b3)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "BUFFER_TOO_SMALL", 3: "NOT_FINITE",
                4: "SPECTRUM", 5: "UNSUPPORTED", 6: "DEVICE"}
FORMATS = {"csr_f64": 0, "sell_f64": 1, "sell_f32": 2, "bsell4_f64": 3, "bsell4_f32": 4, "bgeom_f64": 5, "bgeom_f32": 6}
PRECISIONS = {"f64": 0, "c32": 1}


class TBKError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))


class TbParams(ctypes.Structure):
    _fields_ = [("r_cut", ctypes.c_double), ("r0", ctypes.c_double), ("beta", ctypes.c_double),
                ("n_species", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("onsite", ctypes.POINTER(ctypes.c_double)),
                ("t_pair", ctypes.POINTER(ctypes.c_double))]


class HamStruct(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("slice", ctypes.c_int32),
                ("n_rows", ctypes.c_int64), ("n_ptr", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("n_bonds", ctypes.c_int64),
                ("max_degree", ctypes.c_int32), ("has_onsite", ctypes.c_int32),
                ("n_seg", ctypes.c_int32),
                ("ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("onsite", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("seg_rows", ctypes.c_void_p), ("uniform_hop", ctypes.c_int32), ("hop_value", ctypes.c_double),
                ("col16", ctypes.c_void_p), ("n_orb", ctypes.c_int32), ("sk_geom", ctypes.c_double * 12)]


_LIB = None
ABI_SYMBOLS = ("tbk_last_error", "tbk_abi_version",
               "tbk_hamiltonian_size", "tb_build_hamiltonian",
               "tbk_hamiltonian_size_batched", "tb_build_hamiltonian_batched",
               "tbk_hamiltonian_size_sk", "tb_build_hamiltonian_sk",
               "kpm_default_config", "kpm_workspace_size", "kpm_workspace_size_config",
               "kpm_scale", "kpm_moments", "kpm_moments_config", "kpm_moments_seeded", "tbk_random_phase",
               "kpm_mean_moments", "kpm_step_timer", "kpm_step_timer_read", "tbk_bandwidth_probe",
               "tbk_bandwidth_probe_words", "kpm_moments_noalloc",
               "kpm_workspace_size_batched", "kpm_moments_batched",
               "kpm_dos", "kpm_dos_batched", "tbk_autotune", "tbk_autotune_form",
               "tbk_descriptor", "tbk_bonds", "tbk_bond_features", "tbk_feature_moments",
               "tbk_coordination_target", "tbk_mlp_forward", "tbk_mlp_workspace_size",
               "tbk_mlp_loss_grad", "tbk_adamw_step", "tbk_mlp_train", "tb_build_hamiltonian_learned",
               "tb_build_velocity", "lsqt_chebyshev_terms", "lsqt_workspace_size", "lsqt_vac_moments",
               "lsqt_sigma", "kpm_integrated_dos", "lsqt_mobility", "tb_build_hamiltonian_sk_learned",
               "tbk_node_features", "tbk_descriptor_species", "tbk_bond_features_species")


class SkParams(ctypes.Structure):
    _fields_ = [("r_cut", ctypes.c_double), ("r0", ctypes.c_double), ("beta", ctypes.c_double),
                ("e_s", ctypes.c_double), ("e_p", ctypes.c_double),
                ("v_ss_sigma", ctypes.c_double), ("v_sp_sigma", ctypes.c_double),
                ("v_pp_sigma", ctypes.c_double), ("v_pp_pi", ctypes.c_double), ("reorder", ctypes.c_int32),
                ("orbitals", ctypes.c_int32), ("e_d", ctypes.c_double),
                ("v_sd_sigma", ctypes.c_double), ("v_pd_sigma", ctypes.c_double), ("v_pd_pi", ctypes.c_double),
                ("v_dd_sigma", ctypes.c_double), ("v_dd_pi", ctypes.c_double), ("v_dd_delta", ctypes.c_double),
                ("n_species", ctypes.c_int32), ("pair_v", ctypes.POINTER(ctypes.c_double)),
                ("species_e", ctypes.POINTER(ctypes.c_double))]


class MlpModel(ctypes.Structure):
    _fields_ = [("r_cut", ctypes.c_double), ("n_radial", ctypes.c_int32),
                ("shift", ctypes.POINTER(ctypes.c_double)), ("scale", ctypes.POINTER(ctypes.c_double)),
                ("params", ctypes.c_void_p), ("n_species", ctypes.c_int32),
                ("c_nk", ctypes.POINTER(ctypes.c_double))]


class OnsiteModel(ctypes.Structure):
    _fields_ = [("r_cut", ctypes.c_double), ("shift", ctypes.POINTER(ctypes.c_double)),
                ("scale", ctypes.POINTER(ctypes.c_double)), ("params", ctypes.c_void_p),
                ("n_species", ctypes.c_int32), ("c_nk", ctypes.POINTER(ctypes.c_double))]


def _cnk_arg(cnk):
    """(n_species, host array, pointer) of descriptor coefficients [ns][ns][8][8], or (0, None, NULL)."""
    if cnk is None:
        return 0, None, None
    import numpy as np
    c = np.ascontiguousarray(np.asarray(cnk, np.float64))
    ns = c.shape[0]
    if c.shape != (ns, ns, 8, 8):
        raise ValueError(f"c_nk has shape {c.shape}, expected ({ns}, {ns}, 8, 8)")
    arr = _f64arr(c.reshape(-1))
    return ns, arr, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))


class KpmConfig(ctypes.Structure):
    _fields_ = [("vectors_per_thread", ctypes.c_int32), ("tiles_per_block", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("doubling", ctypes.c_int32), ("uniform_values", ctypes.c_int32),
                ("compact_columns", ctypes.c_int32), ("atom_rows", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("slice", ctypes.c_int32), ("config", KpmConfig), ("ms_per_step", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


def make_config(vectors_per_thread=1, tiles_per_block=2, nontemporal=1, xcd_remap=0, rows_per_thread=1,
                persistent=0, doubling=0, uniform_values=0, compact_columns=0, atom_rows=0):
    return KpmConfig(vectors_per_thread, tiles_per_block, nontemporal, xcd_remap, rows_per_thread, persistent,
                     doubling, uniform_values, compact_columns, atom_rows)


def with_doubling(cfg, on=1):
    """A copy of a launch shape with the doubling identities switched on or off."""
    return with_fields(cfg, doubling=int(on))


def with_fields(cfg, **fields):
    """A copy of a launch shape with some fields replaced."""
    d = cfg.as_dict()
    d.update(fields)
    return KpmConfig(**d)


def lib():
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python paper_2509_06525_amd/build.py first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.tbk_last_error.restype = ctypes.c_char_p
    L.tbk_last_error.argtypes = []
    L.tbk_abi_version.restype = i32
    L.tbk_hamiltonian_size.restype = ctypes.c_int
    L.tbk_hamiltonian_size.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                       ctypes.POINTER(TbParams), ctypes.POINTER(HamStruct), vp]
    L.tb_build_hamiltonian.restype = ctypes.c_int
    L.tb_build_hamiltonian.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                       ctypes.POINTER(TbParams), ctypes.POINTER(HamStruct),
                                       ctypes.POINTER(f64), vp]
    L.kpm_default_config.restype = ctypes.c_int
    L.kpm_default_config.argtypes = [ctypes.POINTER(HamStruct), i32, i32, ctypes.POINTER(KpmConfig)]
    L.kpm_workspace_size.restype = ctypes.c_int
    L.kpm_workspace_size.argtypes = [ctypes.POINTER(HamStruct), i32, i32, i32, ctypes.POINTER(i64)]
    L.kpm_moments.restype = ctypes.c_int
    L.kpm_moments.argtypes = [ctypes.POINTER(HamStruct), ctypes.POINTER(f64), ctypes.POINTER(f64), vp,
                              i32, i32, i32, i32, vp, i64, vp, vp]
    L.kpm_scale.restype = ctypes.c_int
    L.kpm_scale.argtypes = [i32, ctypes.POINTER(f64), f64, ctypes.POINTER(f64), ctypes.POINTER(f64)]
    L.kpm_moments_noalloc.restype = ctypes.c_int
    L.kpm_moments_noalloc.argtypes = [ctypes.POINTER(HamStruct), ctypes.POINTER(f64), ctypes.POINTER(f64), vp,
                                      i32, i32, i32, ctypes.POINTER(KpmConfig), i32, vp, vp]
    L.tbk_bandwidth_probe.restype = ctypes.c_int
    L.tbk_bandwidth_probe.argtypes = [vp, vp, i64, i32, vp]
    L.tbk_bandwidth_probe_words.restype = i64
    L.tbk_bandwidth_probe_words.argtypes = []
    L.kpm_step_timer.restype = ctypes.c_int
    L.kpm_step_timer.argtypes = [i32]
    L.kpm_step_timer_read.restype = ctypes.c_int
    L.kpm_step_timer_read.argtypes = [ctypes.POINTER(f64), ctypes.POINTER(i64)]
    L.kpm_mean_moments.restype = ctypes.c_int
    L.kpm_mean_moments.argtypes = [vp, i32, i32, i32, vp, vp]
    L.kpm_workspace_size_config.restype = ctypes.c_int
    L.kpm_workspace_size_config.argtypes = [ctypes.POINTER(HamStruct), i32, i32, i32,
                                            ctypes.POINTER(KpmConfig), ctypes.POINTER(i64)]
    L.kpm_moments_config.restype = ctypes.c_int
    L.kpm_moments_config.argtypes = [ctypes.POINTER(HamStruct), ctypes.POINTER(f64), ctypes.POINTER(f64),
                                     vp, i32, i32, i32, ctypes.POINTER(KpmConfig), i32, vp, i64, vp, vp]
    L.tbk_autotune.restype = ctypes.c_int
    L.tbk_autotune.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32), ctypes.POINTER(TbParams),
                               i32, i32, i32, i32, ctypes.POINTER(TuneResult), vp]
    L.tbk_autotune_form.restype = ctypes.c_int
    L.tbk_autotune_form.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                    ctypes.POINTER(TbParams), i32, i32, i32, i32, ctypes.POINTER(KpmConfig),
                                    ctypes.POINTER(TuneResult), vp]
    L.tbk_hamiltonian_size_batched.restype = ctypes.c_int
    L.tbk_hamiltonian_size_batched.argtypes = [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64),
                                               ctypes.POINTER(i32), ctypes.POINTER(TbParams),
                                               ctypes.POINTER(HamStruct), vp]
    L.tb_build_hamiltonian_batched.restype = ctypes.c_int
    L.tb_build_hamiltonian_batched.argtypes = [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64),
                                               ctypes.POINTER(i32), ctypes.POINTER(TbParams),
                                               ctypes.POINTER(HamStruct), ctypes.POINTER(f64), vp]
    L.kpm_workspace_size_batched.restype = ctypes.c_int
    L.kpm_workspace_size_batched.argtypes = [ctypes.POINTER(HamStruct), i32, i32, i32, ctypes.POINTER(KpmConfig),
                                             ctypes.POINTER(i64), vp]
    L.kpm_moments_batched.restype = ctypes.c_int
    L.kpm_moments_batched.argtypes = [ctypes.POINTER(HamStruct), ctypes.POINTER(f64), ctypes.POINTER(f64), vp,
                                      i32, i32, i32, ctypes.POINTER(KpmConfig), vp, i64, vp, vp]
    u16p = vp
    L.tbk_descriptor.restype = ctypes.c_int
    L.tbk_descriptor.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64), ctypes.POINTER(i32), f64, i32,
                                 vp, vp]
    L.tbk_bonds.restype = ctypes.c_int
    L.tbk_bonds.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64), ctypes.POINTER(i32), f64, i64,
                            vp, vp, vp, ctypes.POINTER(i64), vp]
    L.tbk_bond_features.restype = ctypes.c_int
    L.tbk_bond_features.argtypes = [i64, vp, vp, vp, vp, i32, f64, ctypes.POINTER(f64), ctypes.POINTER(f64),
                                    u16p, vp]
    L.tbk_descriptor_species.restype = ctypes.c_int
    L.tbk_descriptor_species.argtypes = [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64), ctypes.POINTER(i32),
                                         f64, i32, i32, ctypes.POINTER(f64), vp, vp]
    L.tbk_bond_features_species.restype = ctypes.c_int
    L.tbk_bond_features_species.argtypes = [i64, vp, vp, vp, vp, vp, i32, f64, i32, ctypes.POINTER(f64),
                                            ctypes.POINTER(f64), ctypes.POINTER(f64), u16p, vp]
    L.tbk_feature_moments.restype = ctypes.c_int
    L.tbk_feature_moments.argtypes = [i64, vp, vp, vp, vp, i32, f64, ctypes.POINTER(f64), ctypes.POINTER(f64), vp]
    L.tbk_coordination_target.restype = ctypes.c_int
    L.tbk_coordination_target.argtypes = [i64, vp, vp, vp, i32, f64, f64, vp, vp]
    L.tbk_mlp_forward.restype = ctypes.c_int
    L.tbk_mlp_forward.argtypes = [i64, u16p, vp, vp, vp]
    L.tbk_mlp_workspace_size.restype = ctypes.c_int
    L.tbk_mlp_workspace_size.argtypes = [i64, ctypes.POINTER(i64)]
    L.tbk_mlp_loss_grad.restype = ctypes.c_int
    L.tbk_mlp_loss_grad.argtypes = [i64, u16p, vp, vp, vp, vp, vp, vp, i64, vp]
    L.tbk_adamw_step.restype = ctypes.c_int
    L.tbk_adamw_step.argtypes = [i64, vp, vp, vp, vp, i64, f64, f64, f64, f64, f64, vp]
    L.tbk_mlp_train.restype = ctypes.c_int
    L.tbk_mlp_train.argtypes = [i64, u16p, vp, vp, vp, vp, vp, ctypes.POINTER(i64), i32, i64, ctypes.c_uint64, f64,
                                f64, f64, f64, f64, ctypes.POINTER(f64), vp, i64, vp]
    L.tb_build_hamiltonian_learned.restype = ctypes.c_int
    L.tb_build_hamiltonian_learned.argtypes = [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(f64),
                                               ctypes.POINTER(i32), ctypes.POINTER(TbParams),
                                               ctypes.POINTER(MlpModel), ctypes.POINTER(HamStruct),
                                               ctypes.POINTER(f64), vp, i64, ctypes.POINTER(i64), vp]
    L.kpm_moments_seeded.restype = ctypes.c_int
    L.kpm_moments_seeded.argtypes = [ctypes.POINTER(HamStruct), ctypes.POINTER(f64), ctypes.POINTER(f64),
                                     ctypes.c_uint64, i32, i32, i32, ctypes.POINTER(KpmConfig), i32, vp, i64, vp,
                                     vp]
    L.tbk_random_phase.restype = ctypes.c_int
    L.tbk_random_phase.argtypes = [ctypes.c_uint64, i64, i32, i32, vp, vp]
    L.tb_build_velocity.restype = ctypes.c_int
    L.tb_build_velocity.argtypes = [vp, ctypes.POINTER(f64), ctypes.POINTER(i32), i32, ctypes.POINTER(HamStruct),
                                    vp, vp]
    L.lsqt_chebyshev_terms.restype = i32
    L.lsqt_chebyshev_terms.argtypes = [f64, f64]
    L.lsqt_workspace_size.restype = ctypes.c_int
    L.lsqt_workspace_size.argtypes = [ctypes.POINTER(HamStruct), i32, i32, i32, i32, ctypes.POINTER(KpmConfig),
                                      ctypes.POINTER(i64)]
    L.lsqt_vac_moments.restype = ctypes.c_int
    L.lsqt_vac_moments.argtypes = [ctypes.POINTER(HamStruct), vp, f64, f64, vp, i32, i32, i32, f64, i32, i32,
                                   i32, ctypes.POINTER(KpmConfig), vp, i64, vp, vp]
    L.lsqt_sigma.restype = ctypes.c_int
    L.lsqt_sigma.argtypes = [vp, i32, i32, f64, f64, f64, i32, vp, i32, vp, vp]
    L.kpm_integrated_dos.restype = ctypes.c_int
    L.kpm_integrated_dos.argtypes = [vp, i32, f64, f64, i32, vp, i32, vp, vp]
    L.lsqt_mobility.restype = ctypes.c_int
    L.lsqt_mobility.argtypes = [vp, i32, i32, i32, vp, f64, vp, vp, vp, vp]
    L.tbk_hamiltonian_size_sk.restype = ctypes.c_int
    L.tbk_hamiltonian_size_sk.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                          ctypes.POINTER(SkParams), ctypes.POINTER(HamStruct), vp]
    L.tb_build_hamiltonian_sk_learned.restype = ctypes.c_int
    L.tb_build_hamiltonian_sk_learned.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                                  ctypes.POINTER(SkParams), ctypes.POINTER(MlpModel),
                                                  ctypes.POINTER(OnsiteModel), ctypes.POINTER(HamStruct),
                                                  ctypes.POINTER(f64), vp, i64, ctypes.POINTER(i64), vp]
    L.tbk_node_features.restype = ctypes.c_int
    L.tbk_node_features.argtypes = [i64, vp, i32, ctypes.POINTER(f64), ctypes.POINTER(f64), vp, vp]
    L.tb_build_hamiltonian_sk.restype = ctypes.c_int
    L.tb_build_hamiltonian_sk.argtypes = [vp, vp, i64, ctypes.POINTER(f64), ctypes.POINTER(i32),
                                          ctypes.POINTER(SkParams), ctypes.POINTER(HamStruct),
                                          ctypes.POINTER(f64), vp]
    L.kpm_dos.restype = ctypes.c_int
    L.kpm_dos.argtypes = [vp, i32, f64, f64, i32, vp, i32, vp, vp]
    L.kpm_dos_batched.restype = ctypes.c_int
    L.kpm_dos_batched.argtypes = [vp, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(f64), i32, vp, i32, vp, vp]
    _LIB = L
    return L


def _check(status):
    if status != TBK_OK:
        raise TBKError(status, lib().tbk_last_error().decode(errors="replace"))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, dtype):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor, got {t.dtype} on {t.device}")
    return t


def _f64arr(x):
    a = (ctypes.c_double * len(x))(*[float(v) for v in x])
    return a


def _params(onsite, t_pair, r_cut, r0, beta, reorder):
    onsite = [float(v) for v in onsite]
    flat = [float(v) for row in t_pair for v in (row if hasattr(row, "__len__") else [row])]
    S = len(onsite)
    if len(flat) != S * S:
        raise ValueError("t_pair must be S x S")
    on = _f64arr(onsite)
    tp = _f64arr(flat)
    p = TbParams(r_cut=r_cut, r0=r0, beta=beta, n_species=S, reorder=int(bool(reorder)),
                 onsite=ctypes.cast(on, ctypes.POINTER(ctypes.c_double)),
                 t_pair=ctypes.cast(tp, ctypes.POINTER(ctypes.c_double)))
    return p, (on, tp)


class Hamiltonian:
    """A Hamiltonian built by tb_build_hamiltonian; owns its device tensors."""

    def __init__(self, st, tensors, bounds):
        self.st = st
        self.tensors = tensors
        self.bounds = bounds

    @property
    def n_rows(self):
        return self.st.n_rows

    @property
    def n_entries(self):
        return self.st.n_entries

    @property
    def fmt(self):
        return self.st.fmt

    @property
    def perm(self):
        return self.tensors["perm"]

    def scale(self, margin=1.01):
        """(a, b) of the library's kpm_scale from the Gershgorin bounds:
        a = margin (E_hi - E_lo)/2, b = (E_hi + E_lo)/2."""
        a, b = kpm_scale([self.bounds], margin)
        return a[0], b[0]

    def nbytes(self):
        return sum(t.numel() * t.element_size() for t in self.tensors.values())


def build_hamiltonian(pos, species, box, periodic, onsite, t_pair, r_cut=2.0, r0=1.42, beta=3.37,
                      fmt="sell_f32", slice=256, reorder=True, stream=None, into=None):
    """Neighbour list + Eq. (1) assembly on the GPU.  pos: float64 [N,3], species: int32 [N].

    `into`: a Hamiltonian from an earlier call with the same N, format and slice
    height whose buffers are overwritten (no size pass) when they are large
    enough; `into` must not be used afterwards."""
    L = lib()
    pos = _dev(pos, torch.float64)
    species = _dev(species, torch.int32)
    n = pos.shape[0]
    p, keep = _params(onsite, t_pair, r_cut, r0, beta, reorder)
    boxa = _f64arr(box)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    s = _stream(stream)
    if into is not None and into.st.fmt == FORMATS[fmt] and into.st.slice == int(slice) and into.n_rows == n:
        t = into.tensors
        st = HamStruct(fmt=FORMATS[fmt], slice=int(slice), n_rows=n, n_ptr=t["ptr"].numel(),
                       n_entries=t["col"].numel())
        st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
        st.onsite, st.perm, st.col16 = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["col16"].data_ptr()
        bounds = (ctypes.c_double * 2)()
        rc = L.tb_build_hamiltonian(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(p), ctypes.byref(st),
                                    bounds, s)
        if rc != TBK_ERR_BUFFER_TOO_SMALL:
            _check(rc)
            del keep
            return Hamiltonian(st, t, (bounds[0], bounds[1]))
    st = HamStruct(fmt=FORMATS[fmt], slice=int(slice))
    _check(L.tbk_hamiltonian_size(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(p),
                                  ctypes.byref(st), s))
    dev = pos.device
    vdt = torch.float32 if fmt == "sell_f32" else torch.float64
    t = {
        "ptr": torch.empty(st.n_ptr, dtype=torch.int64, device=dev),
        "col": torch.empty(max(st.n_entries, 1), dtype=torch.int32, device=dev),
        "val": torch.empty(max(st.n_entries, 1), dtype=vdt, device=dev),
        "onsite": torch.empty(n, dtype=vdt, device=dev),
        "perm": torch.empty(n, dtype=torch.int32, device=dev),
        "col16": torch.empty(max(st.n_entries, 1), dtype=torch.int16, device=dev),
    }
    st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
    st.onsite, st.perm, st.col16 = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["col16"].data_ptr()
    bounds = (ctypes.c_double * 2)()
    _check(L.tb_build_hamiltonian(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(p),
                                  ctypes.byref(st), bounds, s))
    del keep
    return Hamiltonian(st, t, (bounds[0], bounds[1]))


def build_hamiltonian_sk(pos, species, box, periodic, v_ss_sigma, v_sp_sigma, v_pp_sigma, v_pp_pi, e_s, e_p,
                         r_cut=2.0, r0=1.42, beta=3.37, fmt="sell_f32", slice=256, reorder=True, stream=None,
                         d=None, e_d=0.0, model=None, with_bond_y=False, pair_v=None, species_e=None,
                         onsite_model=None):
    """Slater-Koster orbital Hamiltonian on the GPU: s, p (4 rows per atom), or
    s, p, d (9 rows per atom) when d = (v_sd_sigma, v_pd_sigma, v_pd_pi,
    v_dd_sigma, v_dd_pi, v_dd_delta) is given.

    model = dict(params=[K][1633] float32 tensor, shift=[16], scale=[16], r_desc=4.0):
    the learned form, each bond's integral l scaled by 1 + y_l from network l
    (K = 4 or 10).  with_bond_y also returns y [K][n_bonds].

    pair_v [ns][ns][K], species_e [ns][3]: several species (species indices in
    `species`), integrals per ordered species pair (lower angular momentum on
    the first species), onsite energies per species; the single-species
    integrals and onsite energies are then unused.

    onsite_model = dict(params=[ns][n_shells][1633] float32 tensor, shift=[8], scale=[8],
    r_desc=4.0): onsite energies e + y from one network per species and shell
    (n_shells = 2 for s, p, 3 for s, p, d)."""
    L = lib()
    pos = _dev(pos, torch.float64)
    species = _dev(species, torch.int32)
    n = pos.shape[0]
    dv = [0.0] * 6 if d is None else [float(x) for x in d]
    if len(dv) != 6:
        raise ValueError("d takes six integrals: sd_sigma, pd_sigma, pd_pi, dd_sigma, dd_pi, dd_delta")
    norb = 4 if d is None else 9
    sk = SkParams(float(r_cut), float(r0), float(beta), float(e_s), float(e_p), float(v_ss_sigma),
                  float(v_sp_sigma), float(v_pp_sigma), float(v_pp_pi), int(bool(reorder)), norb, float(e_d), *dv)
    keep = None
    if pair_v is not None:
        import numpy as np
        pv0 = np.asarray(pair_v, np.float64)
        ns = pv0.shape[0]
        if pv0.shape != (ns, ns, 4 if norb == 4 else 10):
            raise ValueError(f"pair_v has shape {pv0.shape}, expected ({ns}, {ns}, {4 if norb == 4 else 10})")
        pv = np.zeros((ns, ns, 10))
        pv[:, :, : pv0.shape[2]] = pv0
        se = np.asarray(species_e, np.float64).reshape(ns, 3)
        keep = (_f64arr(pv.reshape(-1)), _f64arr(se.reshape(-1)))
        sk.n_species = ns
        sk.pair_v = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_double))
        sk.species_e = ctypes.cast(keep[1], ctypes.POINTER(ctypes.c_double))
    boxa = _f64arr(box)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    s = _stream(stream)
    st = HamStruct(fmt=FORMATS[fmt], slice=int(slice))
    _check(L.tbk_hamiltonian_size_sk(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(sk), ctypes.byref(st), s))
    dev = pos.device
    vdt = torch.float32 if fmt in ("sell_f32", "bsell4_f32", "bgeom_f32") else torch.float64
    # norb x norb blocks, or the bond's displacement (3 values) for the matrix-free form
    # displacement form: (dx, dy, dz) per slot; float slots carry the column as a 4th value
    per_entry = norb * norb if fmt.startswith("bsell4") else (
        (4 if fmt == "bgeom_f32" else 3) if fmt.startswith("bgeom") else 1)
    t = {
        "ptr": torch.empty(st.n_ptr, dtype=torch.int64, device=dev),
        "col": torch.empty(max(st.n_entries, 1), dtype=torch.int32, device=dev),
        "val": torch.empty(max(per_entry * st.n_entries, 1), dtype=vdt, device=dev),
        "onsite": torch.empty(st.n_rows, dtype=vdt, device=dev),
        "perm": torch.empty(st.n_rows, dtype=torch.int32, device=dev),
        "col16": torch.empty(max(st.n_entries, 1), dtype=torch.int16, device=dev),
    }
    st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
    st.onsite, st.perm, st.col16 = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["col16"].data_ptr()
    bounds = (ctypes.c_double * 2)()
    if model is None and onsite_model is None:
        _check(L.tb_build_hamiltonian_sk(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(sk),
                                         ctypes.byref(st), bounds, s))
        return Hamiltonian(st, t, (bounds[0], bounds[1]))
    K = 4 if norb == 4 else 10
    mm = None
    if model is not None:
        params = _dev(model["params"], torch.float32)
        if tuple(params.shape) != (K, TBK_MLP_PARAMS):
            raise ValueError(f"params has shape {tuple(params.shape)}, expected {(K, TBK_MLP_PARAMS)}")
        sh, sc = _f64arr(model["shift"]), _f64arr(model["scale"])
        mns, marr, mcp = _cnk_arg(model.get("cnk"))
        mm = MlpModel(r_cut=float(model.get("r_desc", 4.0)), n_radial=8,
                      shift=ctypes.cast(sh, ctypes.POINTER(ctypes.c_double)),
                      scale=ctypes.cast(sc, ctypes.POINTER(ctypes.c_double)), params=params.data_ptr(),
                      n_species=mns, c_nk=mcp)
    om = None
    if onsite_model is not None:
        ns = 1 if pair_v is None else sk.n_species
        op = _dev(onsite_model["params"], torch.float32)
        want = (ns, 2 if norb == 4 else 3, TBK_MLP_PARAMS)
        if tuple(op.shape) != want:
            raise ValueError(f"onsite params have shape {tuple(op.shape)}, expected {want}")
        osh, osc = _f64arr(onsite_model["shift"]), _f64arr(onsite_model["scale"])
        ons, oarr, ocp = _cnk_arg(onsite_model.get("cnk"))
        om = OnsiteModel(r_cut=float(onsite_model.get("r_desc", 4.0)),
                         shift=ctypes.cast(osh, ctypes.POINTER(ctypes.c_double)),
                         scale=ctypes.cast(osc, ctypes.POINTER(ctypes.c_double)), params=op.data_ptr(),
                         n_species=ons, c_nk=ocp)
    if mm is None:
        with_bond_y = False
    nbonds = st.n_bonds
    y = torch.empty((K, max(nbonds, 1)), dtype=torch.float32, device=dev) if with_bond_y else None
    nb_out = ctypes.c_int64(0)
    _check(L.tb_build_hamiltonian_sk_learned(_ptr(pos), _ptr(species), n, boxa, per, ctypes.byref(sk),
                                             None if mm is None else ctypes.byref(mm),
                                             None if om is None else ctypes.byref(om), ctypes.byref(st), bounds,
                                             _ptr(y), K * nbonds if y is not None else 0, ctypes.byref(nb_out), s))
    H = Hamiltonian(st, t, (bounds[0], bounds[1]))
    if with_bond_y:
        return H, y[:, : nb_out.value]
    return H


def _cfg_ref(config):
    return ctypes.byref(config) if config is not None else None


def default_config(H, R, precision):
    """The launch shape kpm_moments uses for (H, R, precision) when given none."""
    out = KpmConfig()
    _check(lib().kpm_default_config(ctypes.byref(H.st), int(R), PRECISIONS[precision], ctypes.byref(out)))
    return out


def workspace_size(H, R, M, precision, config=None):
    out = ctypes.c_int64(0)
    _check(lib().kpm_workspace_size_config(ctypes.byref(H.st), int(R), int(M), PRECISIONS[precision],
                                           _cfg_ref(config), ctypes.byref(out)))
    return out.value


def alloc_workspace(H, R, M, precision, device=None, config=None):
    nbytes = workspace_size(H, R, M, precision, config)
    dev = device if device is not None else H.tensors["ptr"].device
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def kpm_scale(bounds, margin=1.01):
    """Lists (a, b) from spectral bounds [(E_lo, E_hi), ...] by the library's kpm_scale."""
    n = len(bounds)
    sb = _f64arr([float(v) for lo_hi in bounds for v in lo_hi])
    a, b = (ctypes.c_double * n)(), (ctypes.c_double * n)()
    _check(lib().kpm_scale(n, sb, float(margin), a, b))
    return list(a), list(b)


def kpm_moments(H, a, b, r, M, precision=None, work=None, mu=None, stream=None, config=None, n_start=0, R=None):
    """Chebyshev moments mu[v][n] (float64, device) of Ht = (H - b)/a for vectors r [N, R].

    n_start > 0 continues the run whose state `work` holds (r may then be None,
    with R given); only mu[:, n_start:] is written."""
    L = lib()
    if r is not None:
        if precision is None:
            precision = "c32" if r.dtype == torch.complex64 else "f64"
        want = torch.complex64 if precision == "c32" else torch.complex128
        r = _dev(r, want)
        if r.dim() == 1:
            r = r.reshape(-1, 1)
        R = r.shape[1]
    elif R is None or precision is None or work is None:
        raise ValueError("continuing a run without r needs R, precision and its work")
    dev = H.tensors["ptr"].device
    if work is None:
        work = alloc_workspace(H, R, M, precision, dev, config)
    if mu is None:
        mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    av = (ctypes.c_double * 1)(float(a))
    bv = (ctypes.c_double * 1)(float(b))
    _check(L.kpm_moments_config(ctypes.byref(H.st), av, bv, _ptr(r), int(R), int(M), PRECISIONS[precision],
                                _cfg_ref(config), int(n_start), _ptr(work), work.numel(), _ptr(mu),
                                _stream(stream)))
    return mu


def bandwidth_probe(src, dst, mode, stream=None):
    """One probe launch over src's bytes: mode "copy" (src -> dst) or "read" (dst receives
    tbk_bandwidth_probe_words() 32-bit folds)."""
    _check(lib().tbk_bandwidth_probe(_ptr(src), _ptr(dst), src.numel() * src.element_size(),
                                     1 if mode == "copy" else 0, _stream(stream)))


def bandwidth_probe_words():
    return int(lib().tbk_bandwidth_probe_words())


def step_timer(enable):
    """Switch the library's step-kernel timer on (cleared) or off for this thread."""
    _check(lib().kpm_step_timer(1 if enable else 0))


def step_timer_read():
    """(milliseconds, step launches) timed since the last read or enable; clears them."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().kpm_step_timer_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def kpm_moments_noalloc(H, a, b, r, M, precision=None, mu=None, stream=None, config=None, n_start=0, R=None):
    """kpm_moments with the library's static workspace (no allocation in the call; mu must
    then be given).  n_start > 0 continues the run the last call on this GPU left there."""
    if r is not None:
        if precision is None:
            precision = "c32" if r.dtype == torch.complex64 else "f64"
        r = _dev(r, torch.complex64 if precision == "c32" else torch.complex128)
        if r.dim() == 1:
            r = r.reshape(-1, 1)
        R = r.shape[1]
    elif R is None or precision is None:
        raise ValueError("continuing a run without r needs R and precision")
    if mu is None:
        mu = torch.empty((R, M), dtype=torch.float64, device=H.tensors["ptr"].device)
    av, bv = (ctypes.c_double * 1)(float(a)), (ctypes.c_double * 1)(float(b))
    _check(lib().kpm_moments_noalloc(ctypes.byref(H.st), av, bv, _ptr(r), int(R), int(M), PRECISIONS[precision],
                                     _cfg_ref(config), int(n_start), _ptr(mu), _stream(stream)))
    return mu


def mean_moments(mu, stream=None):
    """Average over the vectors on the device: mu [R, M] -> [M], or [S, R, M] -> [S, M]."""
    mu = _dev(mu, torch.float64)
    one = mu.dim() == 2
    m3 = mu.reshape(1, *mu.shape) if one else mu
    S, R, M = m3.shape
    out = torch.empty((S, M), dtype=torch.float64, device=mu.device)
    _check(lib().kpm_mean_moments(_ptr(m3), S, R, M, _ptr(out), _stream(stream)))
    return out[0] if one else out


def random_phase(seed, n, R, precision="c32", device="cuda", stream=None):
    """Counter-based random phases [n, R] (complex64 for c32, complex128 for f64) on the device."""
    dt = torch.complex64 if precision == "c32" else torch.complex128
    r = torch.empty((n, R), dtype=dt, device=device)
    _check(lib().tbk_random_phase(int(seed) & (2**64 - 1), int(n), int(R), PRECISIONS[precision], _ptr(r),
                                  _stream(stream)))
    return r


def kpm_moments_seeded(H, a, b, seed, R, M, precision="c32", work=None, mu=None, stream=None, config=None,
                       n_start=0):
    """kpm_moments with the random-phase start vectors generated on the device from `seed`."""
    L = lib()
    dev = H.tensors["ptr"].device
    if work is None:
        work = alloc_workspace(H, R, M, precision, dev, config)
    if mu is None:
        mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    av, bv = (ctypes.c_double * 1)(float(a)), (ctypes.c_double * 1)(float(b))
    _check(L.kpm_moments_seeded(ctypes.byref(H.st), av, bv, int(seed) & (2**64 - 1), int(R), int(M),
                                PRECISIONS[precision], _cfg_ref(config), int(n_start), _ptr(work), work.numel(),
                                _ptr(mu), _stream(stream)))
    return mu


def kpm_dos(mu, a, b, E, kernel=0, stream=None):
    """Jackson-damped DOS (Eq. (4)) on the energies E (float64 device tensors)."""
    mu = _dev(mu, torch.float64)
    E = _dev(E, torch.float64)
    rho = torch.empty_like(E)
    _check(lib().kpm_dos(_ptr(mu), mu.numel(), float(a), float(b), int(kernel), _ptr(E), E.numel(),
                         _ptr(rho), _stream(stream)))
    return rho


def kpm_dos_batched(mu, a, b, E, kernel=0, stream=None):
    """DOS of every structure: mu [S, M] (vector-averaged), a, b [S] (host), E [S, nE] -> rho [S, nE]."""
    mu = _dev(mu, torch.float64)
    E = _dev(E, torch.float64)
    S, M = mu.shape
    assert E.dim() == 2 and E.shape[0] == S
    rho = torch.empty_like(E)
    _check(lib().kpm_dos_batched(_ptr(mu), M, S, _f64arr(a), _f64arr(b), int(kernel), _ptr(E), E.shape[1],
                                 _ptr(rho), _stream(stream)))
    return rho


def autotune(pos, species, box, periodic, onsite, t_pair, R, precision="c32", r_cut=2.0, r0=1.42,
             beta=3.37, reorder=True, steps=8, stream=None, doubling=0, uniform_values=0):
    """Fastest (slice, launch shape) for this structure, R and form of the
    recurrence (doubling identities, uniform values); returns a TuneResult."""
    L = lib()
    pos = _dev(pos, torch.float64)
    species = _dev(species, torch.int32)
    p, keep = _params(onsite, t_pair, r_cut, r0, beta, reorder)
    boxa = _f64arr(box)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    out = TuneResult()
    fmt = "sell_f32" if precision == "c32" else "sell_f64"
    form = make_config(doubling=int(doubling), uniform_values=int(uniform_values))
    _check(L.tbk_autotune_form(_ptr(pos), _ptr(species), pos.shape[0], boxa, per, ctypes.byref(p),
                               FORMATS[fmt], int(R), PRECISIONS[precision], int(steps), ctypes.byref(form),
                               ctypes.byref(out), _stream(stream)))
    del keep
    return out


class BatchedHamiltonian(Hamiltonian):
    """Stacked Hamiltonian of several structures; bounds is a list of (E_lo, E_hi)."""

    @property
    def n_seg(self):
        return self.st.n_seg

    def scales(self, margin=1.01):
        """Lists (a, b) of kpm_scale over the structures' Gershgorin bounds."""
        return kpm_scale(self.bounds, margin)


def build_hamiltonian_batched(pos, species, seg_atoms, boxes, periodic, onsite, t_pair, r_cut=2.0, r0=1.42,
                              beta=3.37, fmt="sell_f32", slice=64, reorder=True, stream=None):
    """Stacked structures: atoms [seg_atoms[s], seg_atoms[s+1]) form structure s with box boxes[s]."""
    L = lib()
    pos = _dev(pos, torch.float64)
    species = _dev(species, torch.int32)
    n_seg = len(seg_atoms) - 1
    p, keep = _params(onsite, t_pair, r_cut, r0, beta, reorder)
    seg = (ctypes.c_int64 * (n_seg + 1))(*[int(v) for v in seg_atoms])
    bx = (ctypes.c_double * (3 * n_seg))(*[float(v) for b3 in boxes for v in b3])
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    st = HamStruct(fmt=FORMATS[fmt], slice=int(slice))
    s = _stream(stream)
    _check(L.tbk_hamiltonian_size_batched(_ptr(pos), _ptr(species), n_seg, seg, bx, per, ctypes.byref(p),
                                          ctypes.byref(st), s))
    dev = pos.device
    n = pos.shape[0]
    vdt = torch.float32 if fmt == "sell_f32" else torch.float64
    t = {
        "ptr": torch.empty(st.n_ptr, dtype=torch.int64, device=dev),
        "col": torch.empty(max(st.n_entries, 1), dtype=torch.int32, device=dev),
        "val": torch.empty(max(st.n_entries, 1), dtype=vdt, device=dev),
        "onsite": torch.empty(n, dtype=vdt, device=dev),
        "perm": torch.empty(n, dtype=torch.int32, device=dev),
        "seg_rows": torch.empty(n_seg + 1, dtype=torch.int64, device=dev),
    }
    st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
    st.onsite, st.perm, st.seg_rows = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["seg_rows"].data_ptr()
    bounds = (ctypes.c_double * (2 * n_seg))()
    _check(L.tb_build_hamiltonian_batched(_ptr(pos), _ptr(species), n_seg, seg, bx, per, ctypes.byref(p),
                                          ctypes.byref(st), bounds, s))
    del keep
    return BatchedHamiltonian(st, t, [(bounds[2 * k], bounds[2 * k + 1]) for k in range(n_seg)])


def workspace_size_batched(H, R, M, precision, config=None, stream=None):
    out = ctypes.c_int64(0)
    _check(lib().kpm_workspace_size_batched(ctypes.byref(H.st), int(R), int(M), PRECISIONS[precision],
                                            _cfg_ref(config), ctypes.byref(out), _stream(stream)))
    return out.value


def kpm_moments_batched(H, a, b, r, M, precision=None, work=None, mu=None, stream=None, config=None):
    """mu[s][v][n] (float64, device) for every structure s of a stacked Hamiltonian."""
    L = lib()
    if precision is None:
        precision = "c32" if r.dtype == torch.complex64 else "f64"
    want = torch.complex64 if precision == "c32" else torch.complex128
    r = _dev(r, want)
    if r.dim() == 1:
        r = r.reshape(-1, 1)
    R = r.shape[1]
    ns = H.n_seg
    if work is None:
        work = torch.empty(workspace_size_batched(H, R, M, precision, config, stream), dtype=torch.uint8,
                           device=r.device)
    if mu is None:
        mu = torch.empty((ns, R, M), dtype=torch.float64, device=r.device)
    av = (ctypes.c_double * ns)(*[float(v) for v in a])
    bv = (ctypes.c_double * ns)(*[float(v) for v in b])
    _check(L.kpm_moments_batched(ctypes.byref(H.st), av, bv, _ptr(r), R, int(M), PRECISIONS[precision],
                                 _cfg_ref(config), _ptr(work), work.numel(), _ptr(mu), _stream(stream)))
    return mu


# ---------------------------------------------------------------------------
# Learned hoppings
# ---------------------------------------------------------------------------

def _segs(seg_atoms, boxes):
    n_seg = len(seg_atoms) - 1
    seg = (ctypes.c_int64 * (n_seg + 1))(*[int(v) for v in seg_atoms])
    bx = (ctypes.c_double * (3 * n_seg))(*[float(v) for b3 in boxes for v in b3])
    return n_seg, seg, bx


def descriptor(pos, seg_atoms, boxes, periodic, r_cut=4.0, n_radial=8, stream=None, species=None, cnk=None):
    """Node features v [N][n_radial] (float64, device); with species (int32 device) and
    cnk [ns][ns][8][8] the descriptor coefficients per species pair of Eq. (2)."""
    pos = _dev(pos, torch.float64)
    n_seg, seg, bx = _segs(seg_atoms, boxes)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    v = torch.empty((pos.shape[0], n_radial), dtype=torch.float64, device=pos.device)
    if cnk is None:
        _check(lib().tbk_descriptor(_ptr(pos), n_seg, seg, bx, per, float(r_cut), int(n_radial), _ptr(v),
                                    _stream(stream)))
        return v
    ns, arr, cp = _cnk_arg(cnk)
    _check(lib().tbk_descriptor_species(_ptr(pos), _ptr(_dev(species, torch.int32)), n_seg, seg, bx, per,
                                        float(r_cut), int(n_radial), ns, cp, _ptr(v), _stream(stream)))
    return v


def bonds(pos, seg_atoms, boxes, periodic, r_cut=2.0, stream=None):
    """Unordered bonds i < j within r_cut: (bi, bj, br) device tensors ordered by (i, j)."""
    pos = _dev(pos, torch.float64)
    n_seg, seg, bx = _segs(seg_atoms, boxes)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    nb = ctypes.c_int64(0)
    L = lib()
    # size query: a zero-capacity call reports the count (BUFFER_TOO_SMALL when non-zero)
    st = L.tbk_bonds(_ptr(pos), n_seg, seg, bx, per, float(r_cut), 0, None, None, None, ctypes.byref(nb),
                     _stream(stream))
    if st not in (TBK_OK, 2):
        _check(st)
    n = nb.value
    dev = pos.device
    bi = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    bj = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    br = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    _check(L.tbk_bonds(_ptr(pos), n_seg, seg, bx, per, float(r_cut), n, _ptr(bi), _ptr(bj), _ptr(br),
                       ctypes.byref(nb), _stream(stream)))
    return bi[:n], bj[:n], br[:n]


def feature_moments(bonds_, v, r_cut=4.0, stream=None):
    bi, bj, br = bonds_
    mean = (ctypes.c_double * 16)()
    std = (ctypes.c_double * 16)()
    _check(lib().tbk_feature_moments(bi.numel(), _ptr(bi), _ptr(bj), _ptr(br), _ptr(v), v.shape[1], float(r_cut),
                                     mean, std, _stream(stream)))
    return list(mean), list(std)


def bond_features(bonds_, v, shift, scale, r_cut=4.0, stream=None, species=None, cnk=None):
    """Standardised MLP inputs as bfloat16 bits: int16 tensor [nb][16] (with species and
    cnk the bond descriptor of each bond's species pair)."""
    bi, bj, br = bonds_
    nb = bi.numel()
    X = torch.empty((nb, 16), dtype=torch.int16, device=bi.device)
    if cnk is None:
        _check(lib().tbk_bond_features(nb, _ptr(bi), _ptr(bj), _ptr(br), _ptr(v), v.shape[1], float(r_cut),
                                       _f64arr(shift), _f64arr(scale), _ptr(X), _stream(stream)))
        return X
    ns, arr, cp = _cnk_arg(cnk)
    _check(lib().tbk_bond_features_species(nb, _ptr(bi), _ptr(bj), _ptr(br), _ptr(_dev(species, torch.int32)),
                                           _ptr(v), v.shape[1], float(r_cut), ns, cp, _f64arr(shift),
                                           _f64arr(scale), _ptr(X), _stream(stream)))
    return X


def coordination_target(bonds_, v, kappa, z0, stream=None):
    bi, bj, _ = bonds_
    y = torch.empty(bi.numel(), dtype=torch.float32, device=bi.device)
    _check(lib().tbk_coordination_target(bi.numel(), _ptr(bi), _ptr(bj), _ptr(v), v.shape[1], float(kappa),
                                         float(z0), _ptr(y), _stream(stream)))
    return y


def mlp_forward(X, params, stream=None):
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib().tbk_mlp_forward(X.shape[0], _ptr(X), _ptr(_dev(params, torch.float32)), _ptr(y), _stream(stream)))
    return y


def mlp_workspace_size(nb):
    out = ctypes.c_int64(0)
    _check(lib().tbk_mlp_workspace_size(int(nb), ctypes.byref(out)))
    return out.value


def mlp_loss_grad(X, target, params, weight=None, stream=None):
    nb = X.shape[0]
    grad = torch.empty(1633, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float64, device=X.device)
    work = torch.empty(mlp_workspace_size(nb), dtype=torch.uint8, device=X.device)
    _check(lib().tbk_mlp_loss_grad(nb, _ptr(X), _ptr(target), _ptr(weight), _ptr(params), _ptr(grad), _ptr(loss),
                                   _ptr(work), work.numel(), _stream(stream)))
    return float(loss.item()), grad


def adamw_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-2, stream=None):
    _check(lib().tbk_adamw_step(p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(t), float(lr), float(beta1),
                                float(beta2), float(eps), float(wd), _stream(stream)))


class MlpTrainer:
    """FP32 parameters and AdamW state on the device; training runs in the library."""

    def __init__(self, params):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0

    def train(self, X, target, epochs, batch, lr=3e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4,
              weight=None, stream=None, shuffle_seed=0):
        nb = X.shape[0]
        bsz = min(batch, nb)
        work = torch.empty(mlp_workspace_size(bsz) + 256 + ((1633 * 4 + 255) // 256) * 256,
                           dtype=torch.uint8, device=X.device)
        hist = (ctypes.c_double * epochs)()
        st = ctypes.c_int64(self.step)
        _check(lib().tbk_mlp_train(nb, _ptr(X), _ptr(target), _ptr(weight), _ptr(self.params), _ptr(self.m),
                                   _ptr(self.v), ctypes.byref(st), int(epochs), int(batch),
                                   int(shuffle_seed) & (2**64 - 1), float(lr), float(beta1),
                                   float(beta2), float(eps), float(wd), hist, _ptr(work), work.numel(),
                                   _stream(stream)))
        self.step = st.value
        return list(hist)


def build_hamiltonian_learned(pos, species, seg_atoms, boxes, periodic, onsite, t_pair, params, shift, scale,
                              r_cut=2.0, r0=1.42, beta=3.37, r_desc=4.0, fmt="sell_f32", slice=64, reorder=True,
                              with_bond_y=False, stream=None, into=None):
    """Stacked structures with MLP hoppings t = t_plain (1 + y) (inference fused into assembly).

    `into`: a Hamiltonian from an earlier call with the same atom count, structure
    count, format and slice height whose buffers are overwritten (no size pass)
    when they are large enough; `into` must not be used afterwards (not with
    with_bond_y)."""
    L = lib()
    pos = _dev(pos, torch.float64)
    species = _dev(species, torch.int32)
    n_seg, seg, bx = _segs(seg_atoms, boxes)
    p, keep = _params(onsite, t_pair, r_cut, r0, beta, reorder)
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    sh, sc = _f64arr(shift), _f64arr(scale)
    model = MlpModel(r_cut=float(r_desc), n_radial=8, shift=ctypes.cast(sh, ctypes.POINTER(ctypes.c_double)),
                     scale=ctypes.cast(sc, ctypes.POINTER(ctypes.c_double)),
                     params=_dev(params, torch.float32).data_ptr())
    s = _stream(stream)
    n = pos.shape[0]
    if (into is not None and not with_bond_y and isinstance(into, BatchedHamiltonian)
            and into.st.fmt == FORMATS[fmt] and into.st.slice == int(slice) and into.n_rows == n
            and into.tensors["seg_rows"].numel() == n_seg + 1):
        t = into.tensors
        st = HamStruct(fmt=FORMATS[fmt], slice=int(slice), n_rows=n, n_ptr=t["ptr"].numel(),
                       n_entries=t["col"].numel())
        st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
        st.onsite, st.perm, st.seg_rows = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["seg_rows"].data_ptr()
        bounds = (ctypes.c_double * (2 * n_seg))()
        rc = L.tb_build_hamiltonian_learned(_ptr(pos), _ptr(species), n_seg, seg, bx, per, ctypes.byref(p),
                                            ctypes.byref(model), ctypes.byref(st), bounds, None, 0, None, s)
        if rc != TBK_ERR_BUFFER_TOO_SMALL:
            _check(rc)
            del keep
            return BatchedHamiltonian(st, t, [(bounds[2 * k], bounds[2 * k + 1]) for k in range(n_seg)])
    st = HamStruct(fmt=FORMATS[fmt], slice=int(slice))
    _check(L.tbk_hamiltonian_size_batched(_ptr(pos), _ptr(species), n_seg, seg, bx, per, ctypes.byref(p),
                                          ctypes.byref(st), s))
    dev = pos.device
    vdt = torch.float32 if fmt == "sell_f32" else torch.float64
    t = {
        "ptr": torch.empty(st.n_ptr, dtype=torch.int64, device=dev),
        "col": torch.empty(max(st.n_entries, 1), dtype=torch.int32, device=dev),
        "val": torch.empty(max(st.n_entries, 1), dtype=vdt, device=dev),
        "onsite": torch.empty(n, dtype=vdt, device=dev),
        "perm": torch.empty(n, dtype=torch.int32, device=dev),
        "seg_rows": torch.empty(n_seg + 1, dtype=torch.int64, device=dev),
    }
    st.ptr, st.col, st.val = t["ptr"].data_ptr(), t["col"].data_ptr(), t["val"].data_ptr()
    st.onsite, st.perm, st.seg_rows = t["onsite"].data_ptr(), t["perm"].data_ptr(), t["seg_rows"].data_ptr()
    nbonds = st.n_bonds
    y = torch.empty(max(nbonds, 1), dtype=torch.float32, device=dev) if with_bond_y else None
    bounds = (ctypes.c_double * (2 * n_seg))()
    nb_out = ctypes.c_int64(0)
    _check(L.tb_build_hamiltonian_learned(_ptr(pos), _ptr(species), n_seg, seg, bx, per, ctypes.byref(p),
                                          ctypes.byref(model), ctypes.byref(st), bounds, _ptr(y),
                                          nbonds if y is not None else 0, ctypes.byref(nb_out), s))
    del keep
    H = BatchedHamiltonian(st, t, [(bounds[2 * k], bounds[2 * k + 1]) for k in range(n_seg)])
    if with_bond_y:
        H.bond_y = y[:nb_out.value]
    return H


# --------------------------------------------------------------------------
# Velocity autocorrelation conductivity (Eq. (3))
# --------------------------------------------------------------------------

def build_velocity(H, pos, box, periodic, axis=0, stream=None):
    """vx [n_entries] (type of H's values): V = i vx in H's layout, Angstrom / fs."""
    pos = _dev(pos, torch.float64)
    vx = torch.empty_like(H.tensors["val"])
    per = (ctypes.c_int32 * 3)(*[int(v) for v in periodic])
    _check(lib().tb_build_velocity(_ptr(pos), _f64arr(box), per, int(axis), ctypes.byref(H.st), _ptr(vx),
                                   _stream(stream)))
    return vx


def chebyshev_terms(a, dt):
    """Terms of the propagator series lsqt_vac_moments uses by default."""
    return int(lib().lsqt_chebyshev_terms(float(a), float(dt)))


def vac_time_batch(R, time_batch=0):
    """Time steps per recurrence lsqt_vac_moments uses (0: automatic, max(1, 16 // R))."""
    return int(time_batch) if time_batch > 0 else max(1, 16 // int(R))


def vac_moments(H, vx, a, b, r, M, n_t, dt, n_cheb=0, precision=None, config=None, work=None, stream=None,
                time_batch=0):
    """nu [n_t][R][M] (float64, device): Re <phi_L(t_j)| T_m(Ht) V |phi_R(t_j)> for start vectors r [N, R].
    time_batch: time steps whose recurrences run as one of R * time_batch vectors (0: automatic);
    config is the launch shape of that recurrence."""
    L = lib()
    if precision is None:
        precision = "c32" if r.dtype == torch.complex64 else "f64"
    want = torch.complex64 if precision == "c32" else torch.complex128
    r = _dev(r, want)
    if r.dim() == 1:
        r = r.reshape(-1, 1)
    R = r.shape[1]
    if work is None:
        nbytes = ctypes.c_int64(0)
        _check(L.lsqt_workspace_size(ctypes.byref(H.st), R, int(M), PRECISIONS[precision], int(time_batch),
                                     _cfg_ref(config), ctypes.byref(nbytes)))
        work = torch.empty(nbytes.value, dtype=torch.uint8, device=r.device)
    nu = torch.empty((int(n_t), R, int(M)), dtype=torch.float64, device=r.device)
    _check(L.lsqt_vac_moments(ctypes.byref(H.st), _ptr(vx), float(a), float(b), _ptr(r), R, int(M), int(n_t),
                              float(dt), int(n_cheb), PRECISIONS[precision], int(time_batch), _cfg_ref(config),
                              _ptr(work), work.numel(), _ptr(nu), _stream(stream)))
    return nu


def node_features(v, shift, scale, stream=None):
    """Onsite-network inputs (bf16 bits, int16 [n][16]) of node features v [n][8]."""
    v = _dev(v, torch.float64)
    X = torch.empty((v.shape[0], 16), dtype=torch.int16, device=v.device)
    _check(lib().tbk_node_features(v.shape[0], _ptr(v), 8, _f64arr(shift), _f64arr(scale), _ptr(X),
                                   _stream(stream)))
    return X


def integrated_dos(mu, a, b, E, kernel=0, stream=None):
    """States below each energy of E (float64, device) from vector-averaged moments mu [M]."""
    mu = _dev(mu, torch.float64)
    E = _dev(E, torch.float64)
    N = torch.empty(E.numel(), dtype=torch.float64, device=E.device)
    _check(lib().kpm_integrated_dos(_ptr(mu), mu.numel(), float(a), float(b), int(kernel), _ptr(E), E.numel(),
                                    _ptr(N), _stream(stream)))
    return N


def mobility(sigma, N, n_ref, stream=None):
    """Frame-averaged plateau conductivity, carriers and mobility (cm^2/(V s)) from
    sigma [F][n_t][nE] and integrated DOS N [F][nE] on one energy grid."""
    sigma = _dev(sigma, torch.float64)
    N = _dev(N, torch.float64)
    F, n_t, nE = sigma.shape
    if tuple(N.shape) != (F, nE):
        raise ValueError(f"N has shape {tuple(N.shape)}, expected {(F, nE)}")
    out = [torch.empty(nE, dtype=torch.float64, device=sigma.device) for _ in range(3)]
    _check(lib().lsqt_mobility(_ptr(sigma), F, n_t, nE, _ptr(N), float(n_ref), _ptr(out[0]), _ptr(out[1]),
                               _ptr(out[2]), _stream(stream)))
    return tuple(out)


def vac_sigma(nu, a, b, dt, E, kernel=0, stream=None):
    """Running conductivity integral [n_t][nE] from vector-averaged moments nu [n_t][M]."""
    nu = _dev(nu, torch.float64)
    E = _dev(E, torch.float64)
    n_t, M = nu.shape
    sig = torch.empty((n_t, E.numel()), dtype=torch.float64, device=E.device)
    _check(lib().lsqt_sigma(_ptr(nu), M, n_t, float(dt), float(a), float(b), int(kernel), _ptr(E), E.numel(),
                            _ptr(sig), _stream(stream)))
    return sig
