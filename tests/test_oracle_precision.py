"""Pins of the oracle's higher-precision builds, the truth of the FP64 parity bars.

The "ld" (x87 extended) and "quad" (binary128) builds run the oracle's
algorithm on the same FP64 inputs in more precise arithmetic.  They are pinned
(1) to the FP64 oracle, which the brute force and the closed forms of
test_oracle_pins pin in turn: same algorithm, so they agree to FP64 rounding;
and (2) to each other: the extended build must sit far closer to binary128
than the FP64 build does, which is what makes it a truth for FP64 errors.
Cases span d = 1, 2, 3, both stencils, both integrators, both boundary
conditions and the three quantities on tiny boxes.
"""
import numpy as np
import pytest

from oracle import micro
from paper_2108_09463_amd import inputs

CASES = [(d, order, bc, q, integ) for d in (1, 2, 3) for order in (2, 4) for bc in (0, 1)
         for q in (0, 1, 2) for integ in (1, 2) if not (d == 3 and (q, integ) != (0, 2) and order == 4)]


def _case(d, order, bc, q, integ):
    eps = 0.05
    n = {1: 16, 2: 10, 3: 8}[d]
    b = inputs.make_box(dim=d, n=n, order=order, bc=bc, quantity=q, integrator=integ, eps=eps, alpha=0.3,
                        mu=0.8 * 3 * eps, mu_box=3 * eps, eta=0.3 * eps ** 2, n_steps=6,
                        center=(0.137, 0.41, 0.29), a_max=1.6)
    coef = {1: inputs.coef_ex1(eps), 2: inputs.coef_ex2(eps), 3: inputs.coef_product3(eps)}[d]
    init = {1: inputs.InitEX1(), 2: inputs.InitEX2(), 3: inputs.InitSmooth3D()}[d]
    return b, coef, init


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("d,order,bc,q,integ", CASES)
def test_extended_and_binary128_builds(d, order, bc, q, integ):
    b, coef, init = _case(d, order, bc, q, integ)
    r = {v: micro.solve_box(b, coef, init_fn=init, want_state=True, variant=v)
         for v in ("plain", "ld", "quad")}
    e_plain = _rel(r["plain"]["out"], r["quad"]["out"])
    e_ld = _rel(r["ld"]["out"], r["quad"]["out"])
    s_plain = np.abs(r["plain"]["mfinal"] - r["quad"]["mfinal"]).max()
    s_ld = np.abs(r["ld"]["mfinal"] - r["quad"]["mfinal"]).max()
    # (1) same algorithm: the FP64 build is within its rounding of binary128
    assert e_plain < 1e-10 and s_plain < 1e-14
    # (2) the extended build is within its own, 2048x finer, rounding (allowing
    # a factor 8 of noise); its outputs are FP64 numbers, so agreement is also
    # limited by that last rounding (the floors, a few FP64 ulps)
    assert e_ld <= max(4e-3 * e_plain, 1e-15)
    assert s_ld <= max(4e-3 * s_plain, 4.5e-16)


def test_truth_resolves_fp64_errors_on_an_ill_conditioned_box():
    """A 2-D box whose average cancels several digits: the FP64 build's error
    against binary128 is far above FP64 unit roundoff, and the extended build
    resolves it to better than 1%."""
    eps = 1.0 / 200.0
    b = inputs.make_box(dim=2, n=32, order=2, bc=1, quantity=0, integrator=2, eps=eps, alpha=0.01,
                        mu=2 * eps, mu_box=3 * eps, eta=0.5 * eps ** 2, a_max=1.65, center=(0.31, 0.77))
    coef, init = inputs.coef_quasi(eps), inputs.InitEX2()
    r = {v: micro.solve_box(b, coef, init_fn=init, variant=v)["out"] for v in ("plain", "fma", "ld", "quad")}
    e_plain = _rel(r["plain"], r["quad"])
    e_fma = _rel(r["fma"], r["quad"])
    e_ld = _rel(r["ld"], r["quad"])
    print("errors against binary128: plain", e_plain, "fma", e_fma, "ld", e_ld)
    assert max(e_plain, e_fma) > 1e-14
    assert e_ld < 0.01 * max(e_plain, e_fma)
