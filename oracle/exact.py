"""Exact-rational brute force of the DSGM update (TEST INFRASTRUCTURE).

The same steps as the FP64 oracle -- Sec. 2.2's mean, variance and capped age
equations and Sec. 2.3's dual-model tests, reset and swap, with the appendix's
variance floor and background rule -- carried out in ``fractions.Fraction`` so
that no rounding happens anywhere.  Used on tiny inputs with dyadic values to
pin the FP64 oracle's decisions and values.

All inputs are Fractions (or ints); ``params`` is an ``oracle.Params`` whose
float fields must be exactly representable (they are converted exactly).
"""
from __future__ import annotations

from fractions import Fraction

from . import FG, HIT_A, HIT_C, MASK_PRINTED, RESET, SWAP, WEIGHT_APPENDIX


def _F(v) -> Fraction:
    return v if isinstance(v, Fraction) else Fraction(v)


def weight(age: int, params) -> Fraction:
    """Sec. 2.2: 1/(a+1); the appendix's reading: 1/a."""
    if params.weight_rule == WEIGHT_APPENDIX:
        return Fraction(1, age)
    return Fraction(1, age + 1)


def sgm_update(model: list, x: Fraction, params) -> None:
    """model = [mean, var, age]; Sec. 2.2 update in place."""
    w = weight(model[2], params)
    u = 1 - w
    mean = u * model[0] + w * x
    V = (mean - x) ** 2
    model[0] = mean
    model[1] = u * model[1] + w * V
    model[2] = min(model[2] + 1, params.age_max)


def step(A: list, C: list, x, params) -> tuple[int, tuple]:
    """One frame for one pixel; returns (code, exact margins (a, c, d))."""
    x = _F(x)
    ts, td_, vf, mf = (_F(params.theta_s), _F(params.theta_d), _F(params.var_floor),
                       _F(params.mask_floor))
    qa = (x - A[0]) ** 2
    ta = ts * max(A[1], vf)
    qc = (x - C[0]) ** 2
    tc = ts * max(C[1], vf)
    code = 0
    if qa < ta:
        code |= HIT_A
        sgm_update(A, x, params)
    elif qc < tc:
        code |= HIT_C
        sgm_update(C, x, params)
    else:
        code |= RESET
        C[:] = [x, _F(params.var_init), 1]
    if C[2] > A[2]:
        code |= SWAP
        A[:] = C[:]
        C[:] = [x, _F(params.var_init), 1]
    qd = (A[0] - x) ** 2
    ref = x if params.mask_rule == MASK_PRINTED else A[1]
    td = td_ * max(mf, ref)
    if not (qd <= td):
        code |= FG
    return code, (qa - ta, qc - tc, qd - td)


def forward(frames, state: dict, params) -> dict:
    """frames: list over t of lists over pixels.  Returns exact results."""
    T = len(frames)
    N = len(state["mean_a"])
    models = [([_F(state["mean_a"][i]), _F(state["var_a"][i]), int(state["age_a"][i])],
               [_F(state["mean_c"][i]), _F(state["var_c"][i]), int(state["age_c"][i])])
              for i in range(N)]
    codes = [[0] * N for _ in range(T)]
    bg = [[None] * N for _ in range(T)]
    margins = [[None] * N for _ in range(T)]
    for t in range(T):
        for i in range(N):
            A, C = models[i]
            c, m = step(A, C, frames[t][i], params)
            codes[t][i] = c
            bg[t][i] = A[0]
            margins[t][i] = m
    return {
        "codes": codes, "bg": bg, "margins": margins,
        "masks": [[255 if c & FG else 0 for c in row] for row in codes],
        "mean_a": [m[0][0] for m in models], "var_a": [m[0][1] for m in models],
        "age_a": [m[0][2] for m in models], "mean_c": [m[1][0] for m in models],
        "var_c": [m[1][1] for m in models], "age_c": [m[1][2] for m in models],
    }
