"""The oracle's pins catch plausible mistakes: each case plants one mistake
into a copy of the oracle's source (a flipped Householder sign, a wrong row
range, a dropped power iteration, a reused Gaussian slab, a transposed
rotation, a wrong tau, a flipped canonical sign, an early-stop off by one,
mistakes in the RSVD and lower-triangular functions, and in the U / V flop
count), runs the pins of
tests/test_oracle_pins.py against the copy, and requires that several of
them fail.  CPU only; the real oracle is untouched.

Not a mistake, and so not planted: flipping the signs of the over-sampled
basis vectors before their Householder QR.  A Householder reflector is the
same for x and -x (alpha and beta change sign together, so v and tau do
not), so the factorization does not depend on that sign convention."""
import os
import types

import numpy as np
import pytest

import tests.test_oracle_pins as pins

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                      "randutv_ref.py")

# (name, text in the oracle, replacement)
MUTATIONS = [
    ("householder sign", "sgn = 1.0 if np.real(alpha) >= 0.0 else -1.0",
     "sgn = -1.0 if np.real(alpha) >= 0.0 else 1.0"),
    ("tau denominator", "tau = (beta - alpha) / beta", "tau = (beta - alpha) / alpha"),
    ("right update rows", "apply_right(T[:, r0:], reflV)", "apply_right(T[r0:, r0:], reflV)"),
    ("power iteration dropped", "            for _ in range(q):\n                Y = X.T @ (X @ Y)",
     "            for _ in range(0):\n                Y = X.T @ (X @ Y)"),
    ("gaussian slab reused", "Gi = g_slab(G, m, b, i, p)", "Gi = g_slab(G, m, b, 0, p)"),
    ("fold-back Us not transposed", "T[r0:r1, c1:] = Us.T @ T[r0:r1, c1:]",
     "T[r0:r1, c1:] = Us @ T[r0:r1, c1:]"),
    ("fold-back Vs transposed", "T[:r0, r0:c1] = T[:r0, r0:c1] @ Vs",
     "T[:r0, r0:c1] = T[:r0, r0:c1] @ Vs.T"),
    ("canonical sign flipped", "if Vs[idx, j] < 0.0:", "if Vs[idx, j] > 0.0:"),
    ("early stop off by one", "c1 >= k_stop", "c1 > k_stop"),
    ("rsvd basis truncated early", "Q @ W[:, :k], Q", "Q[:, :k] @ W[:k, :k], Q"),
    ("lower form swaps U and V", "return V1, T1.T.copy(), U1, k", "return U1, T1.T.copy(), V1, k"),
    ("U/V flop count sign of 2mn^2", "- 2.0 * m * n * n + 2.0 * n ** 3",
     "+ 2.0 * m * n * n + 2.0 * n ** 3"),
    ("U/V flop count drops 2n^3", "- 2.0 * m * n * n + 2.0 * n ** 3", "- 2.0 * m * n * n"),
]


def _pin_calls():
    """Every pin of test_oracle_pins, each parametrized one with every
    argument set."""
    calls = []
    for name in sorted(dir(pins)):
        fn = getattr(pins, name)
        if not name.startswith("test_") or not callable(fn):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if params:
            argnames, values = params[0].args[0], params[0].args[1]
            names = [a.strip() for a in argnames.split(",")]
            for v in values:
                calls.append((name, fn, dict(zip(names, v if len(names) > 1 else (v,)))))
        else:
            calls.append((name, fn, {}))
    return calls


def _mutant(old, new):
    src = open(ORACLE).read()
    assert src.count(old) >= 1, f"mutation target not found: {old!r}"
    mod = types.ModuleType("randutv_ref_mutant")
    mod.__file__ = ORACLE
    exec(compile(src.replace(old, new, 1), ORACLE, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_pins(name, old, new):
    mutant = _mutant(old, new)
    real = pins.ref
    failed = []
    try:
        pins.ref = mutant
        for pname, fn, kw in _pin_calls():
            try:
                with np.errstate(all="ignore"):
                    fn(**kw)
            except Exception:  # an assertion, or the mutant breaking a shape
                failed.append(pname)
    finally:
        pins.ref = real
    assert len(failed) >= 2, f"{name}: only {failed} failed"


def test_unmutated_oracle_passes_every_pin():
    """The same harness on an unmodified copy: no pin fails."""
    mutant = _mutant("import math", "import math")
    real = pins.ref
    failed = []
    try:
        pins.ref = mutant
        for pname, fn, kw in _pin_calls():
            try:
                fn(**kw)
            except Exception:
                failed.append(pname)
    finally:
        pins.ref = real
    assert failed == []
