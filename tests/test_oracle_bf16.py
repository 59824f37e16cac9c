"""Pin of the oracle's bfloat16 MLP arithmetic (CPU only).

The per-bond network of Eq. (2) runs on bf16 MFMA: every product takes operands
rounded to bfloat16 (round to nearest even) and accumulates in higher precision.
The oracle reproduces that in FP64 (`orc_mlp_forward`, `orc_mlp_loss_grad` with
bf16 = 1).  Here an independent reference pins it: float64 torch autograd over a
matrix product whose forward multiplies round(A) @ round(B) and whose backward
returns round(g) @ round(B)^T and round(A)^T @ round(g) -- the rounding rule of a
bf16-operand GEMM applied to the three forward and the five backward products
(dL/dW3, the delta through W3, dL/dW2, the delta through W2, dL/dW1).  The
rounding itself is a bit-level round-to-nearest-even of the float64 significand
to 8 bits, checked against torch's float32 -> bfloat16 conversion.

Mutants: each of the sixteen operand roundings of the oracle (two per product) is
removed in turn from a copy of the oracle's source, compiled on the CPU, and the
reference must tell the mutant from the oracle.
"""
import ctypes
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from oracle import build as oracle_build
from oracle import oracle as O
from tests import mlp_ref
from tests.mlp_ref import bf16_rne

NI, NH, NP = 16, 32, 1633


def test_reference_rounding_matches_torch_bf16():
    """bf16_rne agrees with torch's float32 -> bfloat16 conversion (one rounding)
    on float32 inputs, and has the defining properties on float64 inputs: at most
    8 significant bits, within half a bf16 ulp, ties to the even neighbour."""
    rng = np.random.default_rng(0)
    x32 = (rng.normal(size=20000) * 10.0 ** rng.integers(-20, 20, size=20000)).astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16_rne(x32.astype(np.float64)), want)
    x = rng.normal(size=20000) * 10.0 ** rng.integers(-20, 20, size=20000)
    y = bf16_rne(x)
    m, e = np.frexp(y)
    assert np.all(m * 256 == np.round(m * 256))                     # 8 significant bits
    ulp = np.ldexp(1.0, np.frexp(x)[1] - 8)
    assert np.all(np.abs(y - x) <= ulp / 2)
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(2.0 + 2.0 ** -7)])
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 (even: 1); 1 + 3 2^-8 halfway
    # between 1 + 2^-7 and 1 + 2^-6 (even: the latter); 2 + 2^-7 between 2 and 2 + 2^-6
    np.testing.assert_array_equal(bf16_rne(ties), [1.0, 1.0 + 2.0 ** -6, -2.0])


def _rt(t):
    return torch.from_numpy(bf16_rne(t.detach().numpy()))


class _Bf16Product(torch.autograd.Function):
    """A @ B with bfloat16-rounded operands in the forward and backward products."""

    @staticmethod
    def forward(ctx, A, B):
        ctx.save_for_backward(A, B)
        return _rt(A) @ _rt(B)

    @staticmethod
    def backward(ctx, g):
        A, B = ctx.saved_tensors
        rg = _rt(g)
        return rg @ _rt(B).T, _rt(A).T @ rg


def _mm(A, B, bf16):
    return _Bf16Product.apply(A, B) if bf16 else A @ B


def reference(X, p, target, w, bf16=True):
    """(y, loss, grad) of the network 16 -> 32 -> tanh -> 32 -> tanh -> 1 with the
    parameter layout W1 [32][16], b1, W2 [32][32], b2, W3 [32], b3."""
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    W1 = P[0:512].reshape(NH, NI)
    b1 = P[512:544]
    W2 = P[544:1568].reshape(NH, NH)
    b2 = P[1568:1600]
    W3 = P[1600:1632].reshape(1, NH)
    b3 = P[1632]
    Xt = torch.tensor(X, dtype=torch.float64)
    h1 = torch.tanh(_mm(Xt, W1.T, bf16) + b1)
    h2 = torch.tanh(_mm(h1, W2.T, bf16) + b2)
    y = (_mm(h2, W3.T, bf16)).reshape(-1) + b3
    wt = torch.ones(len(X), dtype=torch.float64) if w is None else torch.tensor(w)
    loss = (wt * (y - torch.tensor(target)) ** 2).sum() / len(X)
    loss.backward()
    return y.detach().numpy(), float(loss.detach()), P.grad.numpy().copy()


def _case(seed, B=64, weighted=True):
    """Inputs, parameters and targets that are not bfloat16 values (so every
    operand rounding changes something) with outputs away from the targets."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, NI))
    p = rng.normal(0.0, 0.35, NP)
    t = rng.normal(0.0, 0.5, B)
    w = rng.uniform(0.5, 1.5, B) if weighted else None
    return X, p, t, w


BLOCKS = [(0, 512), (512, 544), (544, 1568), (1568, 1600), (1600, 1632), (1632, 1633)]


def _close(got, want, rel=1e-12):
    return all(np.max(np.abs(got[a:b] - want[a:b])) <= rel * max(np.max(np.abs(want[a:b])), 1e-300)
               for a, b in BLOCKS)


@pytest.mark.parametrize("seed,weighted,B", [(1, True, 64), (2, False, 33), (3, True, 1)])
def test_oracle_bf16_forward_and_gradient_match_reference(seed, weighted, B):
    X, p, t, w = _case(seed, B, weighted)
    y_ref, l_ref, g_ref = reference(X, p, t, w, bf16=True)
    y = O.mlp_forward(X, p, bf16_ops=True)
    np.testing.assert_allclose(y, y_ref, rtol=1e-12, atol=1e-14)
    loss, g = O.mlp_loss_grad(X, t, p, w=w, bf16_ops=True)
    assert loss == pytest.approx(l_ref, rel=1e-12)
    assert _close(g, g_ref)


def test_oracle_plain_path_matches_reference_without_rounding():
    X, p, t, w = _case(4)
    y_ref, l_ref, g_ref = reference(X, p, t, w, bf16=False)
    np.testing.assert_allclose(O.mlp_forward(X, p, bf16_ops=False), y_ref, rtol=1e-12, atol=1e-14)
    loss, g = O.mlp_loss_grad(X, t, p, w=w, bf16_ops=False)
    assert loss == pytest.approx(l_ref, rel=1e-12)
    assert _close(g, g_ref)


# Each mutant removes one operand rounding from the oracle's source: (name, text, replacement).
_W1X = "s += orc_rnd(W1[h * ORC_NI + k], bf16) * orc_rnd(x[k], bf16);"
_W2A = "s += orc_rnd(W2[h * ORC_NH + k], bf16) * orc_rnd(a1[k], bf16);"
_W3A = "s += orc_rnd(W3[k], bf16) * orc_rnd(a2[k], bf16);"
_GW3 = "gW3[k] += orc_rnd(dy, bf16) * orc_rnd(h2[k], bf16);"
_D2 = "d2[k] = orc_rnd(W3[k], bf16) * orc_rnd(dy, bf16) *"
_GW2 = "gW2[h * ORC_NH + k] += orc_rnd(d2[h], bf16) * orc_rnd(h1[k], bf16);"
_D1 = "s += orc_rnd(W2[h * ORC_NH + k], bf16) * orc_rnd(d2[h], bf16);"
_GW1 = "gW1[h * ORC_NI + k] += orc_rnd(d1[h], bf16) * orc_rnd(x[k], bf16);"
MUTANTS = [
    ("fwd1_W1", _W1X, "s += W1[h * ORC_NI + k] * orc_rnd(x[k], bf16);"),
    ("fwd1_x", _W1X, "s += orc_rnd(W1[h * ORC_NI + k], bf16) * x[k];"),
    ("fwd2_W2", _W2A, "s += W2[h * ORC_NH + k] * orc_rnd(a1[k], bf16);"),
    ("fwd2_h1", _W2A, "s += orc_rnd(W2[h * ORC_NH + k], bf16) * a1[k];"),
    ("fwd3_W3", _W3A, "s += W3[k] * orc_rnd(a2[k], bf16);"),
    ("fwd3_h2", _W3A, "s += orc_rnd(W3[k], bf16) * a2[k];"),
    ("dW3_dy", _GW3, "gW3[k] += dy * orc_rnd(h2[k], bf16);"),
    ("dW3_h2", _GW3, "gW3[k] += orc_rnd(dy, bf16) * h2[k];"),
    ("delta2_W3", _D2, "d2[k] = W3[k] * orc_rnd(dy, bf16) *"),
    ("delta2_dy", _D2, "d2[k] = orc_rnd(W3[k], bf16) * dy *"),
    ("dW2_d2", _GW2, "gW2[h * ORC_NH + k] += d2[h] * orc_rnd(h1[k], bf16);"),
    ("dW2_h1", _GW2, "gW2[h * ORC_NH + k] += orc_rnd(d2[h], bf16) * h1[k];"),
    ("delta1_W2", _D1, "s += W2[h * ORC_NH + k] * orc_rnd(d2[h], bf16);"),
    ("delta1_d2", _D1, "s += orc_rnd(W2[h * ORC_NH + k], bf16) * d2[h];"),
    ("dW1_d1", _GW1, "gW1[h * ORC_NI + k] += d1[h] * orc_rnd(x[k], bf16);"),
    ("dW1_x", _GW1, "gW1[h * ORC_NI + k] += orc_rnd(d1[h], bf16) * x[k];"),
]


def _compile_mutant(src_text, name, old, new, tmp):
    assert src_text.count(old) == 1, (name, src_text.count(old))
    path = os.path.join(tmp, f"m_{name}.c")
    with open(path, "w") as f:
        f.write(src_text.replace(old, new))
    lib = os.path.join(tmp, f"m_{name}.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", lib, path, "-lm"], check=True)
    return lib


def _run(lib_path, X, p, t, w):
    L = ctypes.CDLL(lib_path)
    dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    L.orc_mlp_forward.restype = None
    L.orc_mlp_forward.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int32, dp, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_mlp_loss_grad.restype = ctypes.c_double
    L.orc_mlp_loss_grad.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_void_p, dp, ctypes.c_int32, dp]
    B = X.shape[0]
    y = np.empty(B)
    L.orc_mlp_forward(B, np.ascontiguousarray(X.reshape(-1)), p, 1, y, None, None)
    g = np.empty(NP)
    wa = None if w is None else np.ascontiguousarray(w)
    L.orc_mlp_loss_grad(B, np.ascontiguousarray(X.reshape(-1)), t,
                        None if wa is None else wa.ctypes.data_as(ctypes.c_void_p), p, 1, g)
    return y, g


@pytest.fixture(scope="module")
def mutant_libs():
    src = open(oracle_build.SRC).read()
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(8) as ex:
            libs = list(ex.map(lambda m: _compile_mutant(src, *m, tmp), MUTANTS))
        # the unmutated source through the same path must pass
        libs.append(_compile_mutant(src, "none", _W1X, _W1X, tmp))
        yield dict(zip([m[0] for m in MUTANTS] + ["none"], libs))


def test_unmutated_copy_passes(mutant_libs):
    X, p, t, w = _case(7)
    y_ref, _, g_ref = reference(X, p, t, w)
    y, g = _run(mutant_libs["none"], X, p, t, w)
    np.testing.assert_allclose(y, y_ref, rtol=1e-12, atol=1e-14)
    assert _close(g, g_ref)


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_every_dropped_rounding_is_caught(mutant_libs, name):
    """Without one rounding the forward output or the gradient moves by far more
    than the 1e-12 bar (here > 1e-6 relative in some parameter block)."""
    X, p, t, w = _case(7)
    y_ref, _, g_ref = reference(X, p, t, w)
    y, g = _run(mutant_libs[name], X, p, t, w)
    dy = np.max(np.abs(y - y_ref)) / np.max(np.abs(y_ref))
    dg = max(np.max(np.abs(g[a:b] - g_ref[a:b])) / np.max(np.abs(g_ref[a:b])) for a, b in BLOCKS)
    assert max(dy, dg) > 1e-6, (name, dy, dg)
    assert not _close(g, g_ref)


def test_decision_model_is_the_oracle_with_its_own_decisions():
    """tests/mlp_ref.py (used by the GPU parity tests to enumerate the rounding
    decisions a GPU may take) reproduces the oracle's bf16 forward, and every
    bond's candidate set holds the oracle's output; clear bonds have exactly one."""
    rng = np.random.default_rng(11)
    X = bf16_rne(rng.normal(size=(3000, NI)))
    p = rng.normal(0.0, 0.3, NP)
    yo = O.mlp_forward(X, p, bf16_ops=True)
    y, h1, h2 = mlp_ref.forward(X, p)
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-14)
    cands, clear = mlp_ref.forward_candidates(X, p, eps=1e-6)
    assert 0.2 < clear.mean() < 1.0                  # both kinds occur in this batch
    for (c, slack), v, cl in zip(cands, yo, clear):
        assert np.min(np.abs(c - v)) <= 1e-12 * max(1.0, abs(v))
        if cl:
            assert len(c) == 1 and slack == 0.0
        assert slack < 1e-5
    multi = [c for c, _ in cands if len(c) > 1]
    # another decision nearly always moves the output (a flip in the first layer can leave
    # every second-layer decision, and so the output, unchanged)
    assert len(multi) > 100 and np.mean([np.ptp(c) > 0 for c in multi]) > 0.5
    exc, _ = mlp_ref.excess(cands, yo)
    assert np.all(exc <= 1e-12)
    _, clear0 = mlp_ref.forward_candidates(X, p, eps=0.0)
    assert clear0.all()
