"""The oracle against the values the paper prints (no GPU).

Fixtures under tests/golden/ hold the paper's numbers verbatim with their
citations: the three worked examples of the Algorithms section and the
application logs (twofold clock accumulator, 3x3 Jordan-block solve,
quadratic equation).  Logs print 6 significant digits, so a logged number
matches when it agrees to one unit in its 6th significant digit (the paper
truncates at least once, in the double 100-hour clock).
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from exact import F, rn

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EXAMPLES = json.load(open(os.path.join(GOLDEN, "paper_examples.json")))
LOGS = json.load(open(os.path.join(GOLDEN, "paper_logs.json")))

TYPES = {"float": np.float32, "double": np.float64}


def eps_of(dtype):
    return 2.0 ** -53 if np.dtype(dtype) == np.float64 else 2.0 ** -24


def expand(coef, dtype):
    """[c0, c1, c2] -> c0 + c1 eps + c2 eps^2 as an exact value in dtype."""
    e = eps_of(dtype)
    v = F(coef[0]) + F(coef[1]) * F(e) + F(coef[2]) * F(e) * F(e)
    out = rn(v, dtype)
    assert F(out) == v, "fixture value not representable"
    return out


def one(v, dtype):
    return np.array([v], dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("ex", EXAMPLES["examples"], ids=lambda e: e["name"])
def test_worked_examples(ex, dtype):
    if ex["op"] in ("add", "div"):
        x0, x1 = (expand(c, dtype) for c in ex["x"])
        y0, y1 = (expand(c, dtype) for c in ex["y"])
        z0, z1 = getattr(oracle, ex["op"])(one(x0, dtype), one(x1, dtype), one(y0, dtype), one(y1, dtype))
        assert z0[0] == expand(ex["z"][0], dtype)
        assert z1[0] == expand(ex["z"][1], dtype)
        # the fixture's true deviation is the exact one
        xs, ys = F(x0) + F(x1), F(y0) + F(y1)
        true = xs + ys if ex["op"] == "add" else xs / ys
        assert true - F(z0[0]) == F(expand(ex["true_dz0"], dtype))
    else:  # sqrt
        x0, x1 = (expand(c, dtype) for c in ex["x"])
        z0, z1 = oracle.sqrt(one(x0, dtype), one(x1, dtype))
        assert z0[0] == expand(ex["z0"], dtype)
        mpmath.mp.prec = 300
        target = mpmath.sqrt(2) - 1
        assert z1[0] == rn(_mp_to_frac(target), dtype)


def _mp_to_frac(v):
    from fractions import Fraction
    m, e = mpmath.mpf(v).man_exp
    return Fraction(int(m)) * Fraction(2) ** int(e)


def test_dtf1_example_is_the_true_deviation():
    """The paper's claim: the computed z1 = -2 eps is exactly dz0 (binary64)."""
    e = 2.0 ** -53
    z0, z1 = oracle.div(one(1.0, np.float64), one(0.0, np.float64),
                        one(1 - e, np.float64), one(e, np.float64))
    exact = (F(1)) / (F(1 - e) + F(e)) - F(z0[0])
    assert F(z1[0]) == exact


# ---------------------------------------------------------------------------
# application logs
# ---------------------------------------------------------------------------

def parse(s):
    """'96.3958[3.54008]' -> (96.3958, 3.54008); 'nan' parses to NaN."""
    v, err = s.rstrip("]").split("[")
    return float(v), float(err)


def close6(ours, printed):
    """Agreement to one unit in the 6th significant digit."""
    ours = float(ours)
    if math.isnan(printed):
        return math.isnan(ours)
    if printed == 0:
        return ours == 0
    unit = 10.0 ** (math.floor(math.log10(abs(printed))) - 5)
    return abs(ours - printed) <= unit


def twofold_of_double(v64, dtype):
    """The paper's float initialisation: the double value rounded to float,
    its error part the float of the (exact) double difference; a double
    value enters with a zero error part."""
    if np.dtype(dtype) == np.float64:
        return np.float64(v64), np.float64(0.0)
    hi = np.float32(v64)
    return hi, np.float32(np.float64(v64) - np.float64(hi))


@pytest.mark.parametrize("run", LOGS["accumulator"]["runs"], ids=lambda r: "%s-%dh" % (r["type"], r["hours"]))
def test_accumulator_log(run):
    dt = TYPES[run["type"]]
    t0, t1 = twofold_of_double(0.1, dt)
    pt0, pt1 = parse(run["tenth"])
    assert close6(t0, pt0) and close6(t1, pt1)
    s0, s1 = oracle.accumulate(run["hours"] * 36000, t0, t1)
    h0, h1 = oracle.div(one(s0, dt), one(s1, dt), one(3600, dt), one(0, dt))
    p0, p1 = parse(run["result"])
    assert close6(h0[0], p0), (h0[0], p0)
    assert close6(h1[0], p1), (h1[0], p1)


def _tf(x, dt):
    return one(x[0], dt), one(x[1], dt)


def _op(name, a, b, dt):
    z0, z1 = getattr(oracle, name)(*_tf(a, dt), *_tf(b, dt))
    return (z0[0], z1[0])


@pytest.mark.parametrize("run", LOGS["gauss"]["runs"], ids=lambda r: "%s-%g" % (r["type"], r["lambda"]))
def test_jordan_block_log(run):
    """Back-substitution on the upper-triangular Jordan block with twofold
    sub, mul and div; every entry a twofold (zero error parts where exact)."""
    dt = TYPES[run["type"]]
    lam = twofold_of_double(run["lambda"], dt)
    pl = parse(run["diag"])
    assert close6(lam[0], pl[0]) and close6(lam[1], pl[1])
    zero, unit = (dt(0), dt(0)), (dt(1), dt(0))
    A = [[lam, unit, zero], [zero, lam, unit], [zero, zero, lam]]
    f = [(dt(v), dt(0)) for v in run["f"]]
    x = [None] * 3
    for i in (2, 1, 0):
        s = f[i]
        for j in range(i + 1, 3):
            s = _op("sub", s, _op("mul", A[i][j], x[j], dt), dt)
        x[i] = _op("div", s, A[i][i], dt)
    for i in range(3):
        p0, p1 = parse(run["x"][i])
        assert close6(x[i][0], p0), (i, x[i], run["x"][i])
        assert close6(x[i][1], p1), (i, x[i], run["x"][i])


@pytest.mark.parametrize("run", LOGS["quadratic"]["runs"], ids=lambda r: "%s-%s" % (r["type"], r["c"]))
def test_quadratic_log(run):
    """x = (-b +- sqrt(b^2 - 4ac)) / 2a with a = 1, b = 2 and twofold c."""
    dt = TYPES[run["type"]]
    c64 = {"1e-08": 1e-08, "1+1e-08": 1 + 1e-08}[run["c"]]
    c = twofold_of_double(c64, dt)
    pc = parse(run["c_twofold"])
    assert close6(c[0], pc[0]) and close6(c[1], pc[1])
    a, b = (dt(1), dt(0)), (dt(2), dt(0))
    four, two = (dt(4), dt(0)), (dt(2), dt(0))
    disc = _op("sub", _op("mul", b, b, dt), _op("mul", _op("mul", four, a, dt), c, dt), dt)
    d = oracle.sqrt(*_tf(disc, dt))
    d = (d[0][0], d[1][0])
    nb = (-b[0], -b[1])
    den = _op("mul", two, a, dt)
    x0 = _op("div", _op("sub", nb, d, dt), den, dt)
    x1 = _op("div", _op("add", nb, d, dt), den, dt)
    sign = -1.0 if run["negated_error_sign"] else 1.0
    for name, got in (("d", d), ("x0", x0), ("x1", x1)):
        p0, p1 = parse(run[name])
        assert close6(got[0], p0), (name, got)
        assert close6(got[1], sign * p1), (name, got)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dtf1_example_with_dotted_dividend(dtype):
    """The Divide example's dividend is the plain 1, so the dotted-dividend
    form (DTF1 with x1 = +0) must give the printed z0 = 1 + 2 eps and
    z1 = -2 eps too; dropping y1 gives z1 close to -eps instead."""
    ex = next(e for e in EXAMPLES["examples"] if e["name"] == "dtf1_example")
    x0 = expand(ex["x"][0], dtype)
    y0, y1 = (expand(c, dtype) for c in ex["y"])
    z0, z1 = oracle.div(one(x0, dtype), None, one(y0, dtype), one(y1, dtype))
    assert z0[0] == expand(ex["z"][0], dtype)
    assert z1[0] == expand(ex["z"][1], dtype)
