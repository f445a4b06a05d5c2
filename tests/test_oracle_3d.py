"""Pins of the oracle for d = 3 micro boxes (the problem allows d <= 3,
Section 2.1): dense brute force on tiny grids, exact reduction to the 2-D
problem when the data do not depend on one coordinate, the laminate's
homogenized matrix diag(harmonic mean, mean, mean), energy decay and the
projection."""
import numpy as np
import pytest

import bruteforce as bf
from oracle import micro
from paper_2108_09463_amd import inputs


def box3(**kw):
    kw.setdefault("center", (0.137, 0.41, 0.29))
    kw.setdefault("macro_index", (0, 0, 0))
    return inputs.make_box(dim=3, **kw)


CASES = [(order, bc, q, integ) for order in (2, 4) for bc in (0, 1) for q in (0, 1, 2)
         for integ in (1, 2) if not (order == 4 and integ == 1)]


@pytest.mark.parametrize("order,bc,q,integ", CASES)
def test_oracle_3d_matches_bruteforce(order, bc, q, integ):
    eps = 0.05
    b = box3(n=6, order=order, bc=bc, quantity=q, integrator=integ, eps=eps, alpha=0.3,
             mu=0.8 * 2 * eps, mu_box=2 * eps, eta=0.2 * eps ** 2, n_steps=4, a_max=1.5)
    coef = inputs.coef_product3(eps)
    init = inputs.InitSmooth3D()
    ora = micro.solve_box(b, coef, init_fn=init, want_state=True)
    ref, mref = bf.solve(b, coef, init_fn=init, M=4, integ=integ)
    assert np.abs(ora["out"] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(ora["mfinal"].reshape(3, -1) - mref).max() <= 1e-13


def _weight_sum(b):
    M = micro.plan(b)[1]
    w, _, _ = micro.weights(b, (3, 7, 3, 7), M)
    return float(np.sum(w))


@pytest.mark.parametrize("free_axis", [2, 0])
@pytest.mark.parametrize("bc,q", [(0, 0), (0, 2)])
def test_3d_reduces_to_2d(free_axis, bc, q):
    """Data and coefficient independent of x_free, periodic box (Dirichlet ghosts
    would pin the outer layers to m_init): every layer evolves exactly
    like the 2-D problem in the other two coordinates, and the 3-D average is the
    2-D one times the kernel weight sum along the free axis (same forced step
    count: the step rule itself depends on d)."""
    eps = 1.0 / 100.0
    a2 = inputs.coef_ex2(eps)
    i2 = inputs.InitEX2()
    if free_axis == 2:
        coef3 = lambda x, y, z: a2(x, y)
        init3 = lambda x, y, z: i2(x, y)
        c2 = (0.3, 0.6)
        c3 = (0.3, 0.6, 0.45)
    else:
        coef3 = lambda x, y, z: a2(y, z)
        init3 = lambda x, y, z: i2(y, z)
        c2 = (0.6, 0.45)
        c3 = (0.3, 0.6, 0.45)
    kw = dict(n=16, order=2, bc=bc, quantity=q, integrator=2, n_steps=40, eps=eps, alpha=0.2,
              mu=2.5 * eps, mu_box=3 * eps, eta=0.3 * eps ** 2, a_max=1.6)
    r3 = micro.solve_box(box3(center=c3, **kw), coef3, init_fn=init3, want_state=True)
    r2 = micro.solve_box(inputs.make_box(dim=2, center=c2, **kw), a2, init_fn=i2, want_state=True)
    S = _weight_sum(box3(center=c3, **kw))
    assert np.abs(r3["out"] - S * r2["out"]).max() <= 1e-12 * np.abs(r2["out"]).max()
    m3 = r3["mfinal"]                         # [3, i2, i1, i0]
    for layer in range(16):
        sl = m3[:, layer] if free_axis == 2 else m3[:, :, :, layer]
        assert np.array_equal(sl, r2["mfinal"])


def test_laminate_homogenized_matrix():
    """3-D laminate a = 1 + 0.5 sin(2 pi x1/eps): the field average approaches
    div(grad m A^H) with A^H = diag(sqrt(0.75), 1, 1)."""
    eps = 1.0 / 100.0
    init = inputs.InitSmooth3D()
    xc = (0.4, 0.3, 0.2)
    b = box3(n=48, order=2, bc=1, quantity=0, eps=eps, alpha=1.2, mu=3.9 * eps, mu_box=6 * eps,
             eta=1.0 * eps ** 2, a_max=1.5, center=xc)
    r = micro.solve_box(b, inputs.coef_layered3(eps), init_fn=init)
    h = 1e-4
    f = lambda *p: init(*[np.array([v]) for v in p])[:, 0]
    d2 = []
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        d2.append((f(*(np.array(xc) + e)) - 2 * f(*xc) + f(*(np.array(xc) - e))) / h ** 2)
    target = np.sqrt(0.75) * d2[0] + d2[1] + d2[2]
    naive = d2[0] + d2[1] + d2[2]                 # the arithmetic mean in every direction
    err = np.linalg.norm(r["out"] - target)
    assert err < 0.015 * np.linalg.norm(target), err
    assert err < 0.25 * np.linalg.norm(naive - target)


def test_3d_energy_decay_and_projection():
    eps = 0.05
    b = box3(n=8, order=2, bc=0, quantity=0, eps=eps, alpha=0.3, mu=2 * eps, mu_box=2 * eps,
             eta=0.5 * eps ** 2, a_max=1.5)
    r = micro.solve_box(b, inputs.coef_product3(eps), init_fn=inputs.InitSmooth3D(), want_trace=True)
    assert np.all(np.diff(r["energy"]) < 0)
    assert r["normdev"].max() < 1e-14
