"""kpm_moments_noalloc (the moments with the library's static workspace, for
callers that cannot allocate) against kpm_moments_config through the C ABI:
bit for bit the same moments for the same launch shape, on two calls in a row
(the second on a smaller Hamiltonian), a continued run, and the size limit."""
from ctypes import c_double

import numpy as np
import pytest
import torch

from paper_2509_06525_amd import synth, tbkpm
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _case(nx, ny, fmt, R, seed):
    s = synth.graphene_sheet(nx, ny, 0.05, seed)
    H = G.build(s, fmt=fmt, slice=64)
    a, b = H.scale()
    cdt = np.complex64 if fmt == "sell_f32" else np.complex128
    r = G.to_dev(synth.random_phase(s.n, R, seed + 1, cdt))
    return H, a, b, r


@pytest.mark.parametrize("fmt,precision", [("sell_f32", "c32"), ("sell_f64", "f64")])
def test_noalloc_equals_the_workspace_entry_point(fmt, precision):
    cfg = tbkpm.make_config(vectors_per_thread=1, tiles_per_block=2, nontemporal=1)
    for nx, ny, R, M in ((40, 31, 4, 300), (11, 7, 3, 130)):      # second call: smaller input
        H, a, b, r = _case(nx, ny, fmt, R, 11 + nx)
        want = tbkpm.kpm_moments(H, a, b, r, M, precision, config=cfg)
        mu = torch.full((R, M), float("nan"), dtype=torch.float64, device=G.DEV)
        got = tbkpm.kpm_moments_noalloc(H, a, b, r, M, precision, mu=mu, config=cfg)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (nx, ny)


def test_noalloc_continues_its_own_run_and_refuses_what_does_not_fit():
    H, a, b, r = _case(30, 20, "sell_f32", 2, 5)
    M = 200
    want = tbkpm.kpm_moments(H, a, b, r, M, "c32")
    first = torch.empty((2, 80), dtype=torch.float64, device=G.DEV)
    tbkpm.kpm_moments_noalloc(H, a, b, r, 80, "c32", mu=first)
    rest = torch.empty((2, M), dtype=torch.float64, device=G.DEV)
    tbkpm.kpm_moments_noalloc(H, a, b, None, M, "c32", mu=rest, n_start=80, R=2)
    assert torch.equal(first, want[:, :80])
    assert torch.equal(rest[:, 80:], want[:, 80:])
    # 4 M rows x 16 vectors need far more than the 64 MiB static workspace
    big = tbkpm.HamStruct(fmt=2, slice=64, n_rows=4_000_000, n_ptr=4_000_000 // 64 + 1, n_entries=12_000_000,
                          max_degree=3, n_seg=1)
    big.ptr = big.col = big.val = big.onsite = big.perm = 1
    av, bv = (c_double * 1)(9.0), (c_double * 1)(0.0)
    out = torch.empty((16, 10), dtype=torch.float64, device=G.DEV)
    st = tbkpm.lib().kpm_moments_noalloc(big, av, bv, tbkpm._ptr(out), 16, 10, 1, None, 0, tbkpm._ptr(out),
                                         tbkpm._stream(None))
    assert st == tbkpm.TBK_ERR_BUFFER_TOO_SMALL
    assert b"static workspace" in tbkpm.lib().tbk_last_error()

