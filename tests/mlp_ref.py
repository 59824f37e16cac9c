"""Test-side FP64 model of the bf16-operand MLP (16 -> 32 -> tanh -> 32 -> tanh -> 1) that
enumerates the rounding decisions a GPU computing its activations in FP32 may take.

The GPU rounds every MFMA operand to bfloat16.  Its activations carry FP32 error (about
1e-7), so an activation within `eps` of a bfloat16 rounding boundary may round to either
neighbour; every other decision is the oracle's.  `forward_candidates` returns, per bond,
the outputs of all such decision sets (one for a bond whose decisions are all clear), so
a parity test can hold every bond to a tight bar.  `grad_clear` marks the bonds whose
forward and backward decisions are all clear for a given batch size.

Test infrastructure: numpy only; the oracle is the reference this module is checked
against (tests/test_oracle_bf16.py), it does not replace it.
"""
import numpy as np

NI, NH = 16, 32
FP32_U = 2.0 ** -24


def bf16_rne(x):
    """float64 -> nearest bfloat16 value (ties to even) as float64, by integer arithmetic
    on the IEEE bits: keep sign, exponent and the top 7 stored significand bits, rounding
    the 45 dropped bits half to even.  Valid in the normal float32 range."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = x.view(np.uint64)
    lsb = (u >> np.uint64(45)) & np.uint64(1)
    u = (u + np.uint64((1 << 44) - 1) + lsb) & ~np.uint64((1 << 45) - 1)
    return np.where(x == 0.0, x, u.view(np.float64))


def layers(p):
    p = np.asarray(p, dtype=np.float64)
    return (bf16_rne(p[0:512].reshape(NH, NI)), p[512:544], bf16_rne(p[544:1568].reshape(NH, NH)),
            p[1568:1600], bf16_rne(p[1600:1632]), p[1632])


def _sides(h, unc):
    """The bf16 values below and above h +- unc (equal where the decision is clear)."""
    return bf16_rne(h - unc), bf16_rne(h + unc)


def forward(X, p):
    """Oracle-decision forward: (y, h1, h2) with FP64 activations."""
    W1, b1, W2, b2, W3, b3 = layers(p)
    h1 = np.tanh(bf16_rne(X) @ W1.T + b1)
    h2 = np.tanh(bf16_rne(h1) @ W2.T + b2)
    return bf16_rne(h2) @ W3 + b3, h1, h2


def _bf16_ulp(v):
    """Spacing of bfloat16 values at |v| (v != 0)."""
    return np.ldexp(1.0, np.frexp(np.abs(v))[1] - 8)


def _ambiguity(h, eps):
    """(lo, hi, two, wide): the bf16 values of h - eps and h + eps; `two` marks a window
    holding exactly two neighbouring bf16 values (one boundary), `wide` one holding more
    (an activation so small that its spacing is below eps)."""
    lo, hi = _sides(h, eps)
    amb = lo != hi
    gap = np.where(amb, hi - lo, 0.0)
    step = np.maximum(_bf16_ulp(np.where(lo != 0, lo, 1.0)), _bf16_ulp(np.where(hi != 0, hi, 1.0)))
    wide = amb & ((gap > step) | (lo == 0) | (hi == 0) | (np.sign(lo) != np.sign(hi)))
    return lo, hi, amb & ~wide, wide


def forward_candidates(X, p, eps=1e-6, cap=12):
    """Per bond: (outputs over every admissible set of rounding decisions, slack), and a
    mask of the bonds whose decisions are all clear (one output, zero slack).

    An activation is ambiguous when a bfloat16 rounding boundary lies within eps of it.
    With one boundary in the window both neighbours are enumerated (the second layer's
    ambiguity is taken for each choice of the first).  An activation so small that the
    window holds several bf16 values keeps the oracle's value and adds to the bond's
    slack the largest output change a value in the window can cause: |W3_j| (hi - lo) in
    the second layer, sum_j |W3_j| |W2_jk| (hi - lo) in the first (|tanh'| <= 1).
    Bonds with more than `cap` enumerated decisions raise."""
    W1, b1, W2, b2, W3, b3 = layers(p)
    y, h1, h2 = forward(X, p)
    lo1, hi1, two1, wide1 = _ambiguity(h1, eps)
    lo2, hi2, two2, wide2 = _ambiguity(h2, eps)
    clear = ~((two1 | wide1).any(1) | (two2 | wide2).any(1))
    sens1 = np.abs(W3) @ np.abs(W2)                  # bound of |dy/dh1_k|
    cands = [(np.array([v]), 0.0) for v in y]
    for e in np.nonzero(~clear)[0]:
        u1 = np.nonzero(two1[e])[0]
        slack1 = float(np.sum(sens1[wide1[e]] * (hi1[e] - lo1[e])[wide1[e]]))
        base1 = bf16_rne(h1[e])
        out, slack = [], 0.0
        for m1 in range(1 << len(u1)):
            h1r = base1.copy()
            for t, k in enumerate(u1):
                h1r[k] = hi1[e, k] if (m1 >> t) & 1 else lo1[e, k]
            g2 = np.tanh(W2 @ h1r + b2)
            l2, u2v, t2, w2 = _ambiguity(g2[None, :], eps)
            l2, u2v, t2, w2 = l2[0], u2v[0], t2[0], w2[0]
            u2 = np.nonzero(t2)[0]
            if len(u1) + len(u2) > cap:
                raise ValueError(f"bond {e}: {len(u1) + len(u2)} ambiguous decisions")
            slack = max(slack, float(np.sum(np.abs(W3[w2]) * (u2v - l2)[w2])))
            base2 = bf16_rne(g2)
            y0 = base2 @ W3 + b3
            for m2 in range(1 << len(u2)):
                d = 0.0
                for t, j in enumerate(u2):
                    d += W3[j] * ((u2v[j] if (m2 >> t) & 1 else l2[j]) - base2[j])
                out.append(y0 + d)
        cands[e] = (np.array(out), slack1 + slack)
    return cands, clear


def excess(cands, y):
    """Per bond: distance from y[e] to its nearest candidate output, less the bond's slack
    (<= 0 when y lies within the slack of an admissible output), and that candidate."""
    best = np.array([c[np.argmin(np.abs(c - v))] for (c, _), v in zip(cands, y)])
    slack = np.array([sl for _, sl in cands])
    return np.abs(best - y) - slack, best


def grad_clear(X, p, target, w, B, eps=1e-6, y_err=1e-6):
    """Bonds whose every bf16 decision of the loss gradient is clear when the batch has B
    bonds: the forward activations (within eps of a boundary = ambiguous, as above), the
    output delta dy = 2 w (y - y*) / B, the deltas d2 = bf16(W3) bf16(dy) (1 - h2^2) and
    d1 = (bf16(W2)^T bf16(d2)) (1 - h1^2).  Each backward quantity gets an uncertainty from
    the GPU's FP32 arithmetic: y within y_err, tanh values within eps, a sum of K exact
    bf16 products within K u sum|terms| (u = 2^-24), a product of a few factors within
    4 u of its value.  For B a power of two the decisions do not depend on B (a factor
    2^-k is exact), so a subset of 2^k clear bonds stays clear as a batch of its own."""
    W1, b1, W2, b2, W3, b3 = layers(p)
    y, h1, h2 = forward(X, p)
    lo1, hi1 = _sides(h1, eps)
    lo2, hi2 = _sides(h2, eps)
    clear = ~((lo1 != hi1).any(1) | (lo2 != hi2).any(1))
    wv = np.ones(len(y)) if w is None else np.asarray(w, dtype=np.float64)
    dy = 2.0 * wv * (y - target) / B
    unc = 2.0 * wv / B * y_err + 4 * FP32_U * np.abs(dy)
    lo, hi = _sides(dy, unc)
    clear &= lo == hi
    dyr = bf16_rne(dy)
    t2 = 1.0 - h2 * h2
    d2 = W3[None, :] * dyr[:, None] * t2
    unc2 = np.abs(W3[None, :] * dyr[:, None]) * (2.0 * np.abs(h2) * eps + 4 * FP32_U * np.abs(t2))
    lo, hi = _sides(d2, unc2)
    clear &= (lo == hi).all(1)
    d2r = bf16_rne(d2)
    S = d2r @ W2                                    # S[e, k] = sum_j d2r[e, j] W2r[j, k]
    Sabs = np.abs(d2r) @ np.abs(W2)
    t1 = 1.0 - h1 * h1
    d1 = S * t1
    unc1 = NH * FP32_U * Sabs * np.abs(t1) + np.abs(S) * (2.0 * np.abs(h1) * eps + 4 * FP32_U * np.abs(t1))
    lo, hi = _sides(d1, unc1)
    clear &= (lo == hi).all(1)
    return clear
