"""Boxes for the final-state checks (status bits 4 and 8): a 2-D 32^2 and a
1-D 64-point box, each at the step count the stability rule plans and forced
to half of it, where dt is above the stability radius of Section 3.2."""
from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

EPS = 1.0 / 200.0


def case(dim, forced):
    n = 32 if dim == 2 else 64
    b = inputs.make_box(dim=dim, n=n, order=2, bc=0, quantity=inputs.Q_FIELD, integrator=inputs.RK4P,
                        eps=EPS, alpha=0.1, mu=3 * EPS, mu_box=3 * EPS, eta=EPS ** 2, a_max=1.65,
                        center=(0.31, 0.77))
    if forced:
        b["n_steps"] = int(L.llhmm_plan([b])[0][0]) // 2
    coef = inputs.coef_quasi(EPS) if dim == 2 else inputs.coef_ex1(EPS)
    init = inputs.InitEX2() if dim == 2 else inputs.InitEX1()
    return b, coef, init
