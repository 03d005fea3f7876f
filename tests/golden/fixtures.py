"""Parser of the hand-derived worked examples in this folder."""
from __future__ import annotations

import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str) -> dict:
    params, init, steps = {}, {}, []
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            kind, rest = line.split(None, 1)
            if kind in ("params", "init"):
                d = params if kind == "params" else init
                for kv in rest.split():
                    k, v = kv.split("=")
                    d[k] = v
            elif kind == "step":
                left, right = rest.split("|")
                t, x, code, mask, bg = left.split()
                mA, vA, aA, mC, vC, aC = right.split()
                steps.append({"t": int(t), "x": Fraction(x), "code": int(code), "mask": int(mask),
                              "bg": Fraction(bg), "mean_a": Fraction(mA), "var_a": Fraction(vA),
                              "age_a": int(aA), "mean_c": Fraction(mC), "var_c": Fraction(vC),
                              "age_c": int(aC)})
    return {"params": params, "init": init, "steps": steps}


def to_oracle_params(pd: dict):
    import oracle
    return oracle.Params(
        theta_s=float(Fraction(pd["theta_s"])), theta_d=float(Fraction(pd["theta_d"])),
        var_init=float(Fraction(pd["var_init"])), var_floor=float(Fraction(pd["var_floor"])),
        mask_floor=float(Fraction(pd["mask_floor"])), age_max=int(pd["age_max"]),
        weight_rule={"eq": oracle.WEIGHT_EQ, "appendix": oracle.WEIGHT_APPENDIX}[pd["weight_rule"]],
        mask_rule={"variance": oracle.MASK_VARIANCE, "printed": oracle.MASK_PRINTED}[pd["mask_rule"]])


def init_state(init: dict) -> dict:
    return {"mean_a": [Fraction(init["mean_a"])], "var_a": [Fraction(init["var_a"])],
            "age_a": [int(init["age_a"])], "mean_c": [Fraction(init["mean_c"])],
            "var_c": [Fraction(init["var_c"])], "age_c": [int(init["age_c"])]}


FIXTURES = ["worked_eq_variance.txt", "worked_appendix_printed.txt"]
