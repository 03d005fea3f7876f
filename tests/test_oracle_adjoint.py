"""Pins of the oracle's derivatives (reverse and forward mode).

With the decisions held fixed, every mean is affine and every variance is a
sum of squares of affine forms in (frames, initial state, var_init): the map is
exactly quadratic, so a central difference has no truncation error, only
rounding.  The derivatives are checked against central differences of the
pinned forward oracle, against each other (dot-product test), and against the
closed form of the running-mean case.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _case(seed, T=50, H=4, W=16, rule=oracle.WEIGHT_EQ):
    x = synth.frames(seed, T, H, W, "f64")
    st = synth.state(seed, H, W, "f64", 30)
    p = oracle.default_params(2.0)
    p.weight_rule = rule
    gbg = synth.grad_bg(seed, T, H, W)
    gsT = synth.grad_state(seed, H, W)
    return x, st, p, gbg, gsT


def _objective(x, st, p, forced, gbg, gsT):
    r = oracle.forward(x, st, p, forced=forced)
    terms = (gbg * r["bg"]).ravel().tolist()
    for j, k in enumerate(("mean_a", "var_a", "mean_c", "var_c")):
        terms += (gsT[j] * r[k]).tolist()
    return math.fsum(terms)


def _perturb(st, ds, s):
    out = dict(st)
    for j, k in enumerate(("mean_a", "var_a", "mean_c", "var_c")):
        out[k] = st[k] + s * ds[j]
    return out


@pytest.mark.parametrize("seed,rule", [(0, oracle.WEIGHT_EQ), (1, oracle.WEIGHT_APPENDIX), (2, oracle.WEIGHT_EQ)])
def test_adjoint_matches_central_difference(seed, rule):
    x, st, p, gbg, gsT = _case(seed, rule=rule)
    forced = oracle.forward(x, st, p)["codes"]
    codes = forced & 0x0F
    for bit in (oracle.HIT_A, oracle.HIT_C, oracle.RESET):
        assert np.any(codes & bit)
    g = oracle.backward(x, st, p, gbg, gsT, forced=forced)
    rng = np.random.default_rng(100 + seed)
    dx = rng.standard_normal(x.shape)
    ds = rng.standard_normal((4, x.shape[1]))
    dvi = float(rng.standard_normal())
    h = 1e-6
    pp, pm = oracle.Params(**vars(p)), oracle.Params(**vars(p))
    pp.var_init += h * dvi
    pm.var_init -= h * dvi
    fp = _objective(x + h * dx, _perturb(st, ds, h), pp, forced, gbg, gsT)
    fm = _objective(x - h * dx, _perturb(st, ds, -h), pm, forced, gbg, gsT)
    fd = (fp - fm) / (2 * h)
    an = math.fsum((dx * g["grad_frames"]).ravel().tolist() + (ds * g["grad_state0"]).ravel().tolist()
                   + [dvi * g["grad_var_init"]])
    assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (fd, an)


def test_forced_run_reproduces_natural_run():
    x, st, p, _, _ = _case(3)
    r = oracle.forward(x, st, p)
    rf = oracle.forward(x, st, p, forced=r["codes"])
    for k in ("bg", "codes", "masks", "mean_a", "var_a", "age_a", "mean_c", "var_c", "age_c"):
        np.testing.assert_array_equal(r[k], rf[k])


@pytest.mark.parametrize("seed", [4, 5])
def test_dot_product_jvp_vs_vjp(seed):
    x, st, p, gbg, gsT = _case(seed, T=80)
    forced = oracle.forward(x, st, p)["codes"]
    rng = np.random.default_rng(seed)
    dx = rng.standard_normal(x.shape)
    ds = rng.standard_normal((4, x.shape[1]))
    dvi = 0.7
    j = oracle.jvp(x, st, p, dx, ds, dvi, forced=forced)
    g = oracle.backward(x, st, p, gbg, gsT, forced=forced)
    lhs = math.fsum((j["dbg"] * gbg).ravel().tolist() + (j["dstate_T"] * gsT).ravel().tolist())
    rhs = math.fsum((dx * g["grad_frames"]).ravel().tolist() + (ds * g["grad_state0"]).ravel().tolist()
                    + [dvi * g["grad_var_init"]])
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_running_mean_gradient_closed_form():
    """theta_s = inf, EQ weights, no cap: bg_t = (a0*m0 + sum_{j<=t} x_j)/(a0+t)
    (1-based t), so dL/dx_j = sum_{t>=j} g_t/(a0+t) and dL/dm0 = sum_t g_t*a0/(a0+t)."""
    T, N, a0 = 60, 8, 3
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (T, N))
    st = {"mean_a": rng.uniform(-1, 1, N), "var_a": rng.uniform(0, 1, N), "age_a": np.full(N, a0),
          "mean_c": np.zeros(N), "var_c": np.ones(N), "age_c": np.ones(N, np.int32)}
    p = oracle.Params(theta_s=np.inf, theta_d=4.0, var_init=1.0, var_floor=0.1, mask_floor=0.25,
                      age_max=10 ** 6)
    gbg = rng.standard_normal((T, N))
    g = oracle.backward(x, st, p, gbg, None)
    wts = gbg / (a0 + np.arange(1, T + 1))[:, None]
    gx_ref = np.cumsum(wts[::-1], axis=0)[::-1]
    np.testing.assert_allclose(g["grad_frames"], gx_ref, atol=1e-13)
    np.testing.assert_allclose(g["grad_state0"][0], a0 * wts.sum(0), atol=1e-13)
    np.testing.assert_array_equal(g["grad_state0"][2:], 0.0)  # C never influences the outputs
    assert g["grad_var_init"] == 0.0


def test_reset_and_swap_routes():
    """Hand-checked routes: a reset makes the candidate mean a copy of x and its
    variance a copy of var_init; a swap moves the candidate into A."""
    p = oracle.Params(theta_s=2.0, theta_d=4.0, var_init=1.0, var_floor=0.0, mask_floor=0.0, age_max=30)
    # frame 1: A (age 5, far away) no match, C no match -> reset C = (x1, var_init, 1)
    # frame 2: C (x1, 1) matches x2 -> w = 1/2: mC = (x1+x2)/2, vC = 1/2 + (x2-x1)^2/8
    st = {"mean_a": [9.0], "var_a": [0.0], "age_a": [5], "mean_c": [-9.0], "var_c": [0.0], "age_c": [1]}
    x = np.array([[0.25], [0.5]])
    r = oracle.forward(x, st, p)
    assert r["codes"][0, 0] & oracle.RESET and r["codes"][1, 0] & oracle.HIT_C
    gsT = np.array([[0.0], [0.0], [1.0], [1.0]])  # L = mC + vC
    g = oracle.backward(x, st, p, None, gsT)
    d = 0.5 - 0.25
    # dL/dx1 = 1/2 - 2*d/8 ; dL/dx2 = 1/2 + 2*d/8 ; dL/dvar_init = 1/2
    np.testing.assert_allclose(g["grad_frames"][:, 0], [0.5 - d / 4, 0.5 + d / 4], atol=1e-15)
    assert g["grad_var_init"] == pytest.approx(0.5)
    np.testing.assert_array_equal(g["grad_state0"], 0.0)
