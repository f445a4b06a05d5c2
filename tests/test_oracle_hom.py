"""Pins of the homogenized-problem oracle (oracle/homogenized.py): closed-form
plane waves of eq. (hom), the energy law, E_disc values printed in the paper
(tab:e1), a brute-force derivative of the interpolant, and the fourth-order
convergence of the E_avg = 0 macro loop (eq. (e_macro) with MPEA and l = 4)."""
import numpy as np
import pytest

from conftest import golden
from oracle import cell, homogenized as hg, macro, micro
from paper_2108_09463_amd import inputs

A2 = np.array([[0.62, 0.03], [0.03, 0.71]])


def grid(n, d=2):
    x = np.arange(n) / n
    return (x,) if d == 1 else tuple(np.meshgrid(x, x, indexing="ij"))


@pytest.mark.parametrize("alpha", [0.0, 0.3])
@pytest.mark.parametrize("d", [1, 2])
def test_solver_matches_plane_wave(d, alpha):
    """Spectral/RK4P solution of eq. (hom) against the closed-form damped,
    precessing plane wave (anisotropic A, wave vector along both axes)."""
    N, T = 32, 0.01
    xs = grid(N, d)
    k = 2 * np.pi * (np.array([3.0]) if d == 1 else np.array([1.0, 2.0]))
    A = 0.866 if d == 1 else A2
    M0 = hg.plane_wave(xs, k, A, alpha, 0.7, 0.2, 0.0)
    M = hg.solve_hom(M0, A, alpha, T, 2 * hg.stable_steps(A, N, alpha, T, d))
    want = hg.plane_wave(xs, k, A, alpha, 0.7, 0.2, T)
    assert np.abs(M - want).max() < 1e-8
    # the wave must actually move: precession and (for alpha > 0) tilt
    assert np.abs(want - M0).max() > 0.1


def test_plane_wave_solves_the_equation():
    """The closed form itself: its time derivative (central difference) equals
    the LL right-hand side with the field F = -(k^T A k)(m - c e3)."""
    xs = grid(16)
    k = 2 * np.pi * np.array([1.0, 1.0])
    alpha, t, h = 0.2, 0.004, 1e-6
    m = hg.plane_wave(xs, k, A2, alpha, 0.6, 0.0, t)
    dmdt = (hg.plane_wave(xs, k, A2, alpha, 0.6, 0.0, t + h)
            - hg.plane_wave(xs, k, A2, alpha, 0.6, 0.0, t - h)) / (2 * h)
    aeff = k @ A2 @ k
    F = -aeff * (m - m[2:3] * np.array([0, 0, 1.0])[:, None, None])
    c = np.cross(m, F, axis=0)
    rhs = -c - alpha * np.cross(m, c, axis=0)
    assert np.abs(dmdt - rhs).max() < 1e-5 * np.abs(rhs).max()
    assert np.abs(hg.hom_field(m, A2) - F).max() < 1e-9 * np.abs(F).max()


def test_energy_law():
    """E = 1/2 int grad M A grad M is conserved for alpha = 0 and decays for alpha > 0."""
    N = 32
    M = inputs.InitEX2()(*grid(N))
    for alpha in (0.0, 0.1):
        E = [hg.energy(M, A2)]
        Mt = M
        for _ in range(4):
            Mt = hg.solve_hom(Mt, A2, alpha, 0.002, hg.stable_steps(A2, N, alpha, 0.002, 2))
            E.append(hg.energy(Mt, A2))
        E = np.array(E)
        if alpha == 0.0:
            assert np.abs(E - E[0]).max() < 1e-9 * E[0]
        else:
            assert np.all(np.diff(E) < -1e-4 * E[0])


def test_edisc_matches_paper_table():
    """E_disc at (0,0) for EX2 with the paper's A^H reproduces tab:e1 to the
    printed digits."""
    want = golden("EX2_EDISC_Q4")
    AH = np.array(golden("EX2_AH")).reshape(2, 2)
    Nf = 96
    F_exact = hg.hom_field(inputs.InitEX2()(*grid(Nf)), AH)[:, 0, 0]
    half_digit = (0.05e-2, 0.05e-3, 0.5e-4)           # half a unit of the last printed digit
    for n, w, tol in zip((12, 24, 48), want, half_digit):
        F = hg.q4_node_field(inputs.InitEX2()(*grid(n)), AH, 1.0 / n)[:, 0, 0]
        e = np.linalg.norm(F - F_exact)
        assert abs(e - w) <= tol, (n, e, w)


def test_q4_field_matches_bruteforce_derivatives():
    """div(grad Q A) at a node from the quotient rule against central finite
    differences of the separately written interpolant micro.q4_interpolant."""
    n = 12
    M = inputs.InitEX2()(*grid(n))
    F = hg.q4_node_field(M, A2, 1.0 / n)
    mac = dict(n=n, dX=1.0 / n, M=M)
    h = 2e-3 / n
    xs = np.array([-h, 0.0, h])
    for k in ((0, 0), (5, 7), (11, 3)):
        Q = micro.q4_interpolant(mac, k, (xs, xs))        # [3, x2, x1]
        d11 = (Q[:, 1, 2] - 2 * Q[:, 1, 1] + Q[:, 1, 0]) / h ** 2
        d22 = (Q[:, 2, 1] - 2 * Q[:, 1, 1] + Q[:, 0, 1]) / h ** 2
        d12 = (Q[:, 2, 2] - Q[:, 2, 0] - Q[:, 0, 2] + Q[:, 0, 0]) / (4 * h * h)
        want = A2[0, 0] * d11 + A2[1, 1] * d22 + 2 * A2[0, 1] * d12
        assert np.abs(F[:, k[0], k[1]] - want).max() < 1e-5 * np.abs(want).max(), k


def test_q4_field_of_uniform_state_is_zero():
    M = np.broadcast_to(np.array([0.6, 0.0, 0.8])[:, None, None], (3, 12, 12))
    assert np.abs(hg.q4_node_field(M, A2, 1.0 / 12)).max() < 1e-10


def test_ideal_loop_is_fourth_order():
    """The macro loop with the E_avg = 0 field (MPEA after HeunP start-up steps)
    converges to M0 like dX^4 (eq. (e_macro): MPEA k = 2, Q_[4] gives l = 4)."""
    A = cell.homogenized_2d(inputs.coef_ex2(1.0), 6)
    T, alpha, Nf = 0.02, 0.01, 48
    M0 = hg.solve_hom(inputs.InitEX2()(*grid(Nf)), A, alpha, T,
                      hg.stable_steps(A, Nf, alpha, T, 2))
    errs = []
    for n in (12, 24):
        steps = int(np.ceil(T / (0.08 / n ** 2)))
        M = hg.run_loop(inputs.InitEX2()(*grid(n)),
                        lambda Y: hg.q4_node_field(Y.reshape(3, n, n), A, 1.0 / n).reshape(3, -1),
                        alpha, T / steps, steps).reshape(3, n, n)
        ref = M0[:, ::Nf // n, ::Nf // n]
        errs.append(np.sqrt(np.mean(np.sum((M - ref) ** 2, axis=0))))
    assert errs[0] / errs[1] > 12.0, errs
    assert errs[0] < 2e-3, errs


def test_batched_midpoint_solve_matches_pointwise():
    """The stacked 3 x 3 solve of the MPEA update equals solving point by point."""
    rng = np.random.default_rng(0)
    M = rng.normal(size=(3, 40))
    h = 30 * rng.normal(size=(3, 40))
    out = macro.implicit_midpoint_solve(M, h, 0.01)
    for i in range(40):
        S = macro.skew(h[:, i])
        ref = np.linalg.solve(np.eye(3) - 0.005 * S, (np.eye(3) + 0.005 * S) @ M[:, i])
        assert np.abs(out[:, i] - ref).max() < 1e-14


def test_stagger_flux_matches_bruteforce_derivatives():
    """Flux model: column j of grad Q A half a cell off the node against central
    finite differences of micro.q4_interpolant evaluated there."""
    n = 12
    dX = 1.0 / n
    M = inputs.InitEX2()(*grid(n))
    mac = dict(n=n, dX=dX, M=M)
    h = 2e-3 / n
    for axis in (0, 1):
        F = hg.q4_stagger_flux(M, A2, dX, axis)
        for k in ((0, 0), (5, 7), (11, 3)):
            o = [0.5 * dX if a == axis else 0.0 for a in (0, 1)]
            x0 = o[0] + np.array([-h, 0.0, h])
            x1 = o[1] + np.array([-h, 0.0, h])
            Q = micro.q4_interpolant(mac, k, (x0, x1))          # [3, x2, x1]
            g0 = (Q[:, 1, 2] - Q[:, 1, 0]) / (2 * h)
            g1 = (Q[:, 2, 1] - Q[:, 0, 1]) / (2 * h)
            want = A2[0, axis] * g0 + A2[1, axis] * g1
            assert np.abs(F[:, k[0], k[1]] - want).max() < 1e-6 * np.abs(want).max(), (axis, k)


def test_staggered_divergence_is_fourth_order():
    """The staggered difference of exact plane-wave fluxes converges to the exact
    field like dX^4 (and like dX^2 for the second-order stencil)."""
    k = 2 * np.pi * np.array([1.0, 2.0])
    errs = {2: [], 4: []}
    for n in (16, 32, 64):
        xs = grid(n)
        F = []
        for j in range(2):
            sh = [x + (0.5 / n if a == j else 0.0) for a, x in enumerate(xs)]
            m = hg.plane_wave(tuple(sh), k, A2, 0.0, 0.7, 0.3, 0.0)
            grads = [kk * np.stack([-m[1], m[0], 0 * m[2]]) for kk in k]   # d_a m
            F.append(sum(A2[a, j] * grads[a] for a in range(2)))
        m = hg.plane_wave(xs, k, A2, 0.0, 0.7, 0.3, 0.0)
        exact = -(k @ A2 @ k) * (m - m[2:3] * np.array([0, 0, 1.0])[:, None, None])
        for order in (2, 4):
            errs[order].append(np.abs(hg.staggered_divergence(F, 1.0 / n, order) - exact).max())
    for order in (2, 4):
        e = errs[order]
        for a, b in zip(e, e[1:]):
            assert abs(np.log2(a / b) - order) < 0.2, (order, e)


def test_torque_stepper_follows_the_plane_wave():
    """The torque-model stepping (RK4P on dM/dt = -T - alpha M x T) driven by the
    exact torque M x F(M) reproduces the closed-form plane wave."""
    N, T, alpha = 16, 0.004, 0.3
    xs = grid(N)
    k = 2 * np.pi * np.array([1.0, 1.0])
    M0 = hg.plane_wave(xs, k, A2, alpha, 0.7, 0.2, 0.0)
    steps = 2 * hg.stable_steps(A2, N, alpha, T, 2)
    M = hg.run_loop(M0, lambda Y: np.cross(Y, hg.hom_field(Y.reshape(3, N, N), A2).reshape(3, -1),
                                           axis=0),
                    alpha, T / steps, steps, startup="rk4p", model="torque").reshape(3, N, N)
    want = hg.plane_wave(xs, k, A2, alpha, 0.7, 0.2, T)
    assert np.abs(M - want).max() < 1e-8
    assert np.abs(want - M0).max() > 0.05


@pytest.mark.parametrize("model", ["flux", "torque"])
def test_ideal_flux_and_torque_loops_are_fourth_order(model):
    """Flux model (staggered fluxes, fourth-order divergence, MPEA) and torque
    model (RK4P) with E_avg = 0 converge to M0 like dX^4."""
    A = cell.homogenized_2d(inputs.coef_ex2(1.0), 6)
    T, alpha, Nf = 0.02, 0.01, 48
    M0 = hg.solve_hom(inputs.InitEX2()(*grid(Nf)), A, alpha, T,
                      hg.stable_steps(A, Nf, alpha, T, 2))
    errs = []
    for n in (12, 24):
        steps = int(np.ceil(T / (0.08 / n ** 2)))
        if model == "flux":
            f = lambda Y: hg.q4_flux_field(Y.reshape(3, n, n), A, 1.0 / n).reshape(3, -1)
            kw = dict(startup="heunp", model="field")
        else:
            f = lambda Y: hg.q4_node_torque(Y.reshape(3, n, n), A, 1.0 / n).reshape(3, -1)
            kw = dict(startup="rk4p", model="torque")
        M = hg.run_loop(inputs.InitEX2()(*grid(n)), f, alpha, T / steps, steps, **kw)
        ref = M0[:, ::Nf // n, ::Nf // n]
        errs.append(np.sqrt(np.mean(np.sum((M.reshape(3, n, n) - ref) ** 2, axis=0))))
    assert errs[0] / errs[1] > 12.0, errs


def test_offset_centre_interpolates_at_absolute_positions():
    """Micro initial data of a box centred between macro nodes: with macro values
    sampled from a polynomial of degree 4 per component, P_[4] reproduces the
    polynomial, so Q_[4] must equal the normalized polynomial at the box's
    absolute grid positions (centre on the node, half a cell off along x1,
    along x2, or a third of a cell off along both)."""
    n = 12
    dX = 1.0 / n

    def poly(x1, x2):
        return np.stack([0.3 + x1 - 2 * x1 ** 2 + 3 * x1 ** 3 * x2 - x2 ** 4,
                         0.5 - x2 + x1 * x2 + 0.7 * x2 ** 2 - x1 ** 4,
                         1.0 + 0.2 * x1 + 0.1 * x2 ** 3 + x1 ** 2 * x2 ** 2])

    x = np.arange(n) * dX
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    mac = dict(n=n, dX=dX, M=poly(X1, X2))
    k = (5, 6)
    for off in ((0.0, 0.0), (0.5, 0.0), (0.0, 0.5), (1 / 3, 1 / 3)):
        c = (k[0] * dX + off[0] * dX, k[1] * dX + off[1] * dX)
        b = inputs.make_box(dim=2, n=16, init_mode=1, macro_index=k, center=c, mu=0.01,
                            mu_box=0.01)
        mi = micro.initial_data(b, macro=mac).reshape(3, 22, 22)      # [3][i1][i0]
        xi, _ = micro.grid_positions(16, 0.01)
        G0, G1 = np.meshgrid(c[0] + xi, c[1] + xi, indexing="xy")
        want = poly(G0, G1)
        want = want / np.sqrt(np.sum(want * want, axis=0, keepdims=True))
        assert np.abs(mi - want).max() < 1e-12, off
