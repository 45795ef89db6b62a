"""Pins of the CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own formulas (no GPU needed)."""
from fractions import Fraction
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import lem_inputs as L
import oracle
from oracle import expm as E
from oracle import globalexp as ge
from oracle import halo as H
from oracle import krylov as K
from oracle import lem
from oracle import operator as op
from oracle import partition as P
from oracle import phi as PHI
from oracle import rosenbrock as ROS
from oracle import schrodinger as SCH
from oracle.metrics import rel_l2, rel_linf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = v
    return out


# ---------------------------------------------------------------- expm ----

def test_pade_coefficients_match_published_table():
    g = _golden("pade13_higham2005.txt")
    assert [int(x) for x in g["b"]] == [int(c) for c in E.pade_coefficients()]
    assert float(g["theta13"][0]) == E.THETA_13


def _rational_taylor_expm(A_frac, terms_tol=Fraction(1, 10 ** 30)):
    """exp(A) by its Taylor series in exact rational arithmetic."""
    n = len(A_frac)
    nrm = max(sum(abs(x) for x in row) for row in A_frac)
    S = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    T = [row[:] for row in S]
    k = 0
    while True:
        k += 1
        T = [[sum(T[i][l] * A_frac[l][j] for l in range(n)) / k for j in range(n)]
             for i in range(n)]
        S = [[S[i][j] + T[i][j] for j in range(n)] for i in range(n)]
        # tail bound: sum_{j>k} nrm^j/j! <= 2 nrm^{k+1}/(k+1)! once nrm < k/2
        tail = 2 * nrm ** (k + 1) / math.factorial(k + 1)
        if k > 2 * nrm and tail < terms_tol:
            return S


@pytest.mark.parametrize("C,mu", [(Fraction(1, 2), Fraction(1, 4)),
                                  (Fraction(2), Fraction(1, 2)),
                                  (Fraction(1), Fraction(2))])
def test_local_expm_matches_exact_rational_taylor(C, mu):
    # tiny 1D grid n=8, core 2, halo 2 -> local 6x6; dx = 1/8, a = 1
    n, dx = 8, Fraction(1, 8)
    dt = C * dx
    nu = mu * dx * dx / dt
    W = op.weights(1, n, float(dx), float(dt), (1.0, 0.0), nu=float(nu))
    box = P.uniform_boxes(1, n, 2, 2)[1]
    G = P.gather_map(box, 1, n)
    A_loc = lem.local_matrix(op.sparse(W), G)
    # exact local matrix: tridiagonal, west mu + C/2, east mu - C/2, diag -2 mu
    Af = [[Fraction(0)] * 6 for _ in range(6)]
    for i in range(6):
        Af[i][i] = -2 * mu
        if i > 0:
            Af[i][i - 1] = mu + C / 2
        if i < 5:
            Af[i][i + 1] = mu - C / 2
    assert np.array_equal(A_loc, np.array([[float(x) for x in r] for r in Af]))
    exact = np.array([[float(x) for x in r] for r in _rational_taylor_expm(Af)])
    assert np.abs(E.expm(A_loc) - exact).max() <= 4e-16 * max(1.0, np.abs(exact).max())


def test_pure_diffusion_block_matches_dst_closed_form():
    # symmetric tridiagonal Toeplitz (-2mu, mu): eigenvalues -2mu + 2mu cos(j pi/(m+1)),
    # eigenvectors sqrt(2/(m+1)) sin(i j pi/(m+1)) (the DST-I basis)
    n, c, h = 256, 64, 16
    mu = 4.096
    dx = 1.0 / n
    dt = 4 * dx
    W = op.weights(1, n, dx, dt, (0.0, 0.0), nu=mu * dx * dx / dt)
    box = P.uniform_boxes(1, n, c, h)[2]
    A_loc = lem.local_matrix(op.sparse(W), P.gather_map(box, 1, n))
    m = A_loc.shape[0]
    j = np.arange(1, m + 1)
    lam = -2 * mu + 2 * mu * np.cos(j * np.pi / (m + 1))
    Q = np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * np.pi / (m + 1))
    closed = Q @ np.diag(np.exp(lam)) @ Q
    assert np.abs(E.expm(A_loc) - closed).max() < 1e-14


def test_expm_matches_library_on_random_and_large_norm():
    rng = np.random.default_rng(7)
    for n, scale in [(5, 0.1), (30, 3.0), (40, 60.0)]:
        A = rng.standard_normal((n, n)) * scale / np.sqrt(n)
        ref = sla.expm(A)
        assert np.abs(E.expm(A) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert E.expm(np.zeros((0, 0))).shape == (0, 0)
    assert np.abs(E.expm(np.zeros((3, 3))) - np.eye(3)).max() <= 4.5e-16


def test_semigroup_local_and_global():
    p = L.workload_1d(n=256)
    W1 = op.from_problem(p)
    W2 = op.weights(1, p.n, p.dx, 2 * p.dt, p.vel, nu=p.nu)
    box = P.uniform_boxes(1, p.n, 64, 16)[0]
    G = P.gather_map(box, 1, p.n)
    E1 = E.expm(lem.local_matrix(op.sparse(W1), G))
    E2 = E.expm(lem.local_matrix(op.sparse(W2), G))
    assert np.abs(E1 @ E1 - E2).max() < 1e-13
    # two FFT half steps = one step (2D)
    q = L.workload_2d_ensemble(n=32, n_states=3)
    Wf = op.from_problem(q)
    Wh = op.weights(2, q.n, q.dx, q.dt / 2, q.vel, nu=q.nu)
    u = q.states
    assert rel_l2(ge.fft_steps(Wh, ge.fft_steps(Wh, u)), ge.fft_steps(Wf, u)) < 1e-14


# ------------------------------------------------------------ operator ----

def test_fft_global_matches_dense_expm_1d_2d():
    for ndim, n, k in [(1, 16, 2), (2, 8, 3)]:
        W = op.weights(ndim, n, 1.0 / n, 2.0 / n, (1.0, 0.5), nu=3e-2)
        u = np.random.default_rng(1).standard_normal((W.N, k))
        ref = sla.expm(op.dense(W)) @ u
        assert rel_l2(ge.fft_steps(W, u), ref) < 5e-14
        assert rel_l2(ge.dense_step(W, u), ref) < 5e-14


def test_operator_matches_continuum_derivatives():
    """dt*A u approximates dt(-a.grad u + nu lap u) to second order: this fixes
    the sign and scale of every stencil weight independently of the weights'
    formulas (a swapped east/west or a missing factor fails)."""
    errs = []
    for n in (64, 128):
        dx = 1.0 / n
        dt = 0.5 * dx
        a, b, nu = 1.3, -0.7, 0.02
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        f = np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y) + np.cos(2 * np.pi * (X + Y))
        fx = 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(4 * np.pi * Y) - 2 * np.pi * np.sin(2 * np.pi * (X + Y))
        fy = -4 * np.pi * np.sin(2 * np.pi * X) * np.sin(4 * np.pi * Y) - 2 * np.pi * np.sin(2 * np.pi * (X + Y))
        lap = -(4 + 16) * np.pi ** 2 * np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y) \
              - 8 * np.pi ** 2 * np.cos(2 * np.pi * (X + Y))
        W = op.weights(2, n, dx, dt, (a, b), nu=nu)
        got = op.apply(W, f.reshape(-1))
        want = dt * (-a * fx - b * fy + nu * lap).reshape(-1)
        errs.append(np.abs(got - want).max() / np.abs(want).max())
    assert errs[0] < 5e-3 and errs[1] < errs[0] / 3.5  # second-order convergence


def test_advection_moves_downstream():
    # pure advection of a smooth bump by the global exponential shifts it by a*t
    n = 512
    dx = 1.0 / n
    W = op.weights(1, n, dx, 64 * dx, (1.0, 0.0), nu=0.0)
    x = np.arange(n) * dx
    u0 = np.exp(-((x - 0.3) ** 2) / (2 * 0.03 ** 2))
    u1 = ge.fft_steps(W, u0)
    assert abs(x[np.argmax(u1)] - (0.3 + 64 * dx)) <= 2 * dx


def test_sparse_and_shift_application_agree_and_variable_nu_conservative():
    p = L.workload_2d_variable(n=32)
    W = op.from_problem(p)
    A = op.sparse(W)
    u = p.states
    assert np.abs(A @ u - op.apply(W, u)).max() < 1e-15
    # conservative flux form: column sums vanish, and exp(dt A) preserves mass
    assert np.abs(np.asarray(A.sum(axis=0))).max() < 1e-12
    Ed = E.expm(A.toarray())
    assert abs((Ed @ u).sum() - u.sum()) < 1e-12 * np.abs(u).sum()


def test_mass_conservation_global_constant():
    q = L.workload_2d_ensemble(n=64, n_states=4)
    W = op.from_problem(q)
    out = ge.fft_steps(W, q.states, 10)
    assert np.abs(out.sum(axis=0) - q.states.sum(axis=0)).max() < 1e-10


# ----------------------------------------------------------- partition ----

def test_kronecker_identity_2d_local_block():
    # 2D constant-coefficient box operator = A_x (+) A_y, so expm = expm(A_y) kron expm(A_x)
    n, c, h = 64, 16, 4
    dx = 1.0 / n
    dt = 2 * dx
    vel = (1.0, 0.5)
    nu = 1e-3 * 4  # mu = 0.128 * ...
    W2 = op.weights(2, n, dx, dt, vel, nu=nu)
    box = P.uniform_boxes(2, n, c, h)[5]
    A2 = lem.local_matrix(op.sparse(W2), P.gather_map(box, 2, n))
    Wx = op.weights(1, n, dx, dt, (vel[0], 0.0), nu=nu)
    Wy = op.weights(1, n, dx, dt, (vel[1], 0.0), nu=nu)
    b1 = P.uniform_boxes(1, n, c, h)[1]
    Ax = lem.local_matrix(op.sparse(Wx), P.gather_map(b1, 1, n))
    Ay = lem.local_matrix(op.sparse(Wy), P.gather_map(b1, 1, n))
    assert A2.shape == (576, 576)
    ref = np.kron(E.expm(Ay), E.expm(Ax))
    assert np.abs(E.expm(A2) - ref).max() < 1e-14


def test_maps_are_consistent_permutations():
    for ndim, n, c, h in [(1, 1024, 64, 16), (2, 64, 16, 4), (2, 48, 16, 7)]:
        boxes = P.uniform_boxes(ndim, n, c, h)
        P.check_tiling(boxes, ndim, n)
        Gc, goff, Sc, soff = P.all_maps(boxes, ndim, n)
        assert np.array_equal(np.sort(Sc), np.arange(n ** ndim))
        for k, b in enumerate(boxes):
            G = Gc[goff[k]:goff[k + 1]]
            S = Sc[soff[k]:soff[k + 1]]
            Lx, Ly = P.box_dims(b, ndim)
            assert len(G) == Lx * Ly
            assert np.array_equal(G[P.core_local_rows(b, ndim)], S)
            assert len(np.unique(G)) == len(G)
    with pytest.raises(ValueError):
        P.gather_map(P.Box(0, 0, 16, 16, 24), 2, 64)  # 16 + 48 >= 64
    with pytest.raises(ValueError):
        P.check_tiling(P.uniform_boxes(2, 64, 16, 4)[1:], 2, 64)


def test_uneven_boxes_tile():
    boxes = [P.Box(0, 0, 32, 32, 4), P.Box(32, 0, 32, 32, 5),
             P.Box(0, 32, 16, 16, 6), P.Box(16, 32, 16, 16, 4),
             P.Box(0, 48, 16, 16, 4), P.Box(16, 48, 16, 16, 8),
             P.Box(32, 32, 32, 32, 7)]
    P.check_tiling(boxes, 2, 64)


# ----------------------------------------------------------------- LEM ----

def test_single_domain_lem_equals_global():
    for ndim, n in [(1, 64), (2, 16)]:
        W = op.weights(ndim, n, 1.0 / n, 4.0 / n, (1.0, 0.5), nu=5e-3)
        u = np.random.default_rng(3).standard_normal((W.N, 2))
        boxes = [P.Box(0, 0, n, n if ndim == 2 else 1, 0)]
        got = lem.step(op.sparse(W), boxes, ndim, n, u)
        assert rel_l2(got, ge.fft_steps(W, u)) < 1e-14


def test_lem_error_decreases_with_halo_to_roundoff():
    p = L.workload_1d()
    W = op.from_problem(p)
    A = op.sparse(W)
    u0 = p.states[:, 0]
    g10 = ge.fft_steps(W, u0, 10)
    errs = [rel_l2(lem.run(A, P.uniform_boxes(1, p.n, 64, h), 1, p.n, u0, 10), g10)
            for h in (4, 8, 12, 16, 20, 24, 28)]
    assert all(b < a / 3 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


def test_lem_huge_halo_matches_fft_over_100_steps():
    p = L.workload_1d()
    W = op.from_problem(p)
    u = lem.run(op.sparse(W), P.uniform_boxes(1, p.n, 64, 32), 1, p.n,
                p.states[:, 0], 100)
    assert rel_l2(u, ge.fft_steps(W, p.states[:, 0], 100)) < 4e-13


def test_paper_buffer_example():
    g = _golden("paper_buffer_example.txt")
    n = int(g["n"][0]); Ld = float(g["L"][0]); D = int(g["subdomains"][0])
    dx = Ld / n
    dt = float(g["C"][0]) * dx
    nu = float(g["mu"][0]) * dx * dx / dt
    steps = int(round(float(g["T"][0]) / dt))
    x = np.arange(n) * dx
    u0 = np.exp(-(x - Ld / 2) ** 2)
    W = op.weights(1, n, dx, dt, (1.0, 0.0), nu=nu)
    A = op.sparse(W)
    ref = ge.fft_steps(W, u0, steps)
    good = lem.run(A, P.uniform_boxes(1, n, n // D, int(g["good_buffer"][0])), 1, n, u0, steps)
    bad = lem.run(A, P.uniform_boxes(1, n, n // D, int(g["bad_buffer"][0])), 1, n, u0, steps)
    level = float(g["paper_error_level"][0])
    assert rel_l2(good, ref) < level / 10      # indistinguishable from the global method
    assert rel_linf(bad, ref) > 0.1            # visibly wrong


def test_exp_euler_form_equals_exp_form():
    p = L.workload_1d(n=256)
    W = op.from_problem(p)
    box = P.uniform_boxes(1, p.n, 64, 16)[1]
    G = P.gather_map(box, 1, p.n)
    B = lem.local_matrix(op.sparse(W), G)
    v = p.states[G, 0]
    assert np.abs(PHI.exp_euler_step(B, v) - E.expm(B) @ v).max() < 1e-13
    # phi_1 scalar check: z phi_1(z) = e^z - 1
    z = np.array([[0.7]])
    assert abs(PHI.phi1_action(z, np.array([1.0]))[0] * 0.7 - math.expm1(0.7)) < 1e-15


# ------------------------------------------------------------ forcing ----
# Update (5) of section 3 with a forcing g constant over the step:
# exp(dt A_M) v + phi_1(dt A_M)(dt g_M).

def _smooth_field(W, seed):
    rng = np.random.default_rng(seed)
    n = W.n
    x = np.arange(n) / n
    if W.ndim == 1:
        return np.cos(2 * np.pi * 3 * x + rng.uniform(0, 6.3)) + 0.3
    X, Y = np.meshgrid(x, x)
    return (np.cos(2 * np.pi * (2 * X + Y) + rng.uniform(0, 6.3)) + 0.3).reshape(-1)


def test_phi1_closed_form_scalar_and_matrix():
    # phi_1(z) = (e^z - 1)/z on scalars, including z -> 0 and complex z
    z = np.array([0.0, 1e-9, -3.5, 2.0 + 1.0j])
    want = np.array([1.0, 1.0 + 5e-10, (math.exp(-3.5) - 1) / -3.5,
                     (np.exp(2.0 + 1.0j) - 1) / (2.0 + 1.0j)])
    assert np.abs(PHI.phi1_scalar(z) - want).max() < 1e-15
    # on a diagonalizable matrix: V phi_1(D) V^{-1}
    rng = np.random.default_rng(5)
    V = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    d = np.array([-4.0, -1.0, -0.1, 0.0, 0.5, 1.5])
    B = V @ np.diag(d) @ np.linalg.inv(V)
    want = V @ np.diag(PHI.phi1_scalar(d)) @ np.linalg.inv(V)
    assert np.abs(PHI.phi1_matrix(B) - want).max() < 1e-12


def test_forcing_constant_field_grows_linearly():
    # A annihilates constants (rows of the periodic stencil sum to zero), so
    # u = c, g = k gives exactly u(t + dt) = c + dt k on the global problem
    for ndim, n in [(1, 64), (2, 16)]:
        W = op.weights(ndim, n, 1.0 / n, 4.0 / n, (1.0, 0.5), nu=5e-3)
        u = np.full(W.N, 0.75)
        dtg = np.full(W.N, 0.2)
        assert np.abs(ge.fft_steps(W, u, 3, dtg) - (0.75 + 3 * 0.2)).max() < 1e-14
        assert np.abs(ge.dense_step(W, u, dtg) - 0.95).max() < 1e-13


def test_forced_steady_state_is_preserved():
    # with dt g = -dt A u*, u* is a fixed point of the exact step
    for ndim, n in [(1, 128), (2, 32)]:
        W = op.weights(ndim, n, 1.0 / n, 2.0 / n, (1.0, 0.5), nu=2e-3)
        us = _smooth_field(W, 7)
        dtg = -op.apply(W, us)
        assert rel_l2(ge.fft_steps(W, us, 5, dtg), us) < 1e-13
        if W.N <= 2048:
            assert rel_l2(ge.dense_step(W, us, dtg), us) < 1e-13
        assert rel_l2(ge.krylov_step(W, us, dtg=dtg), us) < 1e-13


def test_forced_single_domain_lem_equals_fft_and_mass_balance():
    # one box holding the whole periodic grid: LEM with forcing is the global
    # exponential-Euler step; the total grows by dt * sum(g) exactly
    for ndim, n in [(1, 64), (2, 16)]:
        W = op.weights(ndim, n, 1.0 / n, 4.0 / n, (1.0, 0.5), nu=5e-3)
        rng = np.random.default_rng(11)
        u = rng.standard_normal((W.N, 2))
        dtg = rng.standard_normal((W.N, 2)) * 0.1
        boxes = [P.Box(0, 0, n, n if ndim == 2 else 1, 0)]
        got = lem.step(op.sparse(W), boxes, ndim, n, u, dtg=dtg)
        assert rel_l2(got, ge.fft_steps(W, u, 1, dtg)) < 1e-14
        assert np.abs(got.sum(0) - (u.sum(0) + dtg.sum(0))).max() < 1e-11


def test_forced_lem_superposition_and_krylov_route():
    # the forced local update is affine: LEM(u, g) = LEM(u, 0) + LEM(0, g); the
    # augmented Krylov route agrees with the dense phi_1 route
    p = L.workload_2d_variable(n=32)
    W = op.from_problem(p)
    A = op.sparse(W)
    boxes = P.uniform_boxes(2, 32, 16, 4)
    u = p.states
    dtg = 0.05 * _smooth_field(W, 3)
    full = lem.step(A, boxes, 2, 32, u, dtg=dtg)
    parts = lem.step(A, boxes, 2, 32, u) + lem.step(A, boxes, 2, 32, 0 * u, dtg=dtg)
    assert rel_l2(full, parts) < 1e-14
    kry = lem.step(A, boxes, 2, 32, u, dtg=dtg, krylov_above=100, krylov_tol=1e-16)
    assert rel_l2(kry, full) < 1e-13


def test_forced_lem_converges_to_global_with_halo():
    p = L.workload_1d()
    W = op.from_problem(p)
    A = op.sparse(W)
    u0 = p.states[:, 0]
    dtg = p.dt * (0.5 + _smooth_field(W, 2))
    ref = ge.fft_steps(W, u0, 10, dtg)
    errs = [rel_l2(lem.run(A, P.uniform_boxes(1, p.n, 64, h), 1, p.n, u0, 10, dtg=dtg), ref)
            for h in (4, 12, 20, 28)]
    assert all(b < a / 10 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


# --------------------------------------------- exponential Rosenbrock ----
# Burgers u_t = -(u^2/2)_x + nu u_xx (section 4.2), exponential
# Rosenbrock-Euler steps u + dt phi_1(dt J) F(u) with J frozen between
# refreshes (sections 3 and 4).

def _gauss(n, L, amp=1.0, x0=3.0):
    x = np.arange(n) * (L / n)
    return amp * np.exp(-(x - x0) ** 2)


def test_burgers_jacobian_is_the_derivative_of_F():
    # F is quadratic, so the central difference is exact up to rounding
    n, dx, nu = 64, 10.0 / 64, 0.05
    rng = np.random.default_rng(4)
    u, d = rng.standard_normal(n), rng.standard_normal(n)
    eps = 1e-3
    fd = (ROS.burgers_F(u + eps * d, dx, nu) - ROS.burgers_F(u - eps * d, dx, nu)) / (2 * eps)
    assert np.abs(fd - ROS.burgers_J(u, dx, nu) @ d).max() < 1e-9
    # at a constant state c the Jacobian is the linear advection-diffusion
    # operator with speed c (an independently written stencil)
    c = 0.7
    W = op.weights(1, n, dx, 1.0, (c, 0.0), nu=nu)
    assert np.abs((ROS.burgers_J(np.full(n, c), dx, nu) - op.sparse(W)).toarray()).max() < 1e-12
    # and constant states are steady: F(c) = 0, so every step keeps them
    u1 = ROS.ere_global_run(np.full(n, c), dx, nu, 0.1, 3)
    assert np.abs(u1 - c).max() < 1e-14


def test_exponential_rosenbrock_euler_is_second_order():
    n, L, nu = 128, 10.0, 0.05
    dx = L / n
    u0 = _gauss(n, L)
    T = 0.8
    ref = ROS.rk4_reference(u0, dx, nu, T, 4000)
    errs = [rel_l2(ROS.ere_global_run(u0, dx, nu, T / s, s), ref) for s in (8, 16, 32)]
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.3 for r in rates), rates


def test_exponential_rosenbrock_conserves_mass_globally():
    # sum(F) = 0 and 1^T J = 0 for the periodic conservative stencil, so the
    # total is kept exactly, with a fresh or a frozen Jacobian
    n, L, nu = 100, 10.0, 0.05
    dx = L / n
    u0 = _gauss(n, L) + 0.2
    for K in (1, 4):
        u = ROS.ere_global_run(u0, dx, nu, 0.05, 9, refresh=K)
        assert abs(u.sum() - u0.sum()) < 1e-11


def test_lem_rosenbrock_single_domain_and_halo_convergence():
    n, L, nu, dt = 200, 10.0, 0.05, 0.05
    dx = L / n
    rng = np.random.default_rng(2)
    u0 = np.column_stack([_gauss(n, L, 1.0, 3.0), _gauss(n, L, 0.6, 5.5) + 0.1])
    glob = ROS.ere_global_run(u0, dx, nu, dt, 10, refresh=5)
    one = ROS.ere_lem_run(u0, [P.Box(0, 0, n, 1, 0)], n, dx, nu, dt, 10, refresh=5)
    assert rel_l2(one, glob) < 1e-13
    errs = [rel_l2(ROS.ere_lem_run(u0, P.uniform_boxes(1, n, 25, h), n, dx, nu, dt, 10, refresh=5), glob)
            for h in (2, 4, 8, 16)]
    assert all(b < a / 5 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-13


def test_nonnegative_local_exponential_when_mu_ge_half_c():
    p = L.workload_1d()
    W = op.from_problem(p)  # C = 4, mu = 4.096 >= C/2
    box = P.uniform_boxes(1, p.n, 64, 20)[0]
    Ek = E.expm(lem.local_matrix(op.sparse(W), P.gather_map(box, 1, p.n)))
    assert Ek.min() > -1e-15
    assert Ek.sum(axis=1).max() <= 1.0 + 1e-13


# -------------------------------------------------------------- Krylov ----

def test_krylov_full_dimension_reproduces_dense():
    p = L.workload_1d(n=256)
    W = op.from_problem(p)
    box = P.uniform_boxes(1, p.n, 32, 8)[0]
    B = lem.local_matrix(op.sparse(W), P.gather_map(box, 1, p.n))
    v = np.random.default_rng(5).standard_normal(B.shape[0])
    beta, V, Hm, k = K.arnoldi(lambda x: B @ x, v, B.shape[0])
    approx = beta * V[:, :k] @ E.expm(Hm[:k, :k])[:, 0]
    assert rel_l2(approx, E.expm(B) @ v) < 1e-13
    got = K.expv(lambda x: B @ x, v, m=30, tol=1e-15)
    assert rel_l2(got, E.expm(B) @ v) < 1e-13


def test_krylov_fourier_mode_happy_breakdown():
    W = op.weights(2, 32, 1 / 32, 2 / 32, (1.0, 0.5), nu=1e-2)
    j = np.arange(32 * 32)
    th = 2 * np.pi * 3 / 32
    v = np.exp(1j * th * (j % 32))  # an eigenvector of the circulant operator
    beta, V, Hm, k = K.arnoldi(lambda x: op.apply(W, x), v, 10)
    assert k == 1
    lam = ge.symbol(W)[0, 3]
    got = beta * V[:, :1] @ E.expm(Hm[:1, :1])[:, 0]
    assert np.abs(got - np.exp(lam) * v).max() < 1e-13


def _dst_diffusion_box(mu, n=256, c=64, h=16):
    """1D pure-diffusion box (C = 0): dt*A_M is symmetric tridiagonal Toeplitz
    (-2mu, mu) with the DST-I eigenbasis."""
    dx = 1.0 / n
    dt = 4 * dx
    W = op.weights(1, n, dx, dt, (0.0, 0.0), nu=mu * dx * dx / dt)
    box = P.uniform_boxes(1, n, c, h)[1]
    A = lem.local_matrix(op.sparse(W), P.gather_map(box, 1, n))
    m = A.shape[0]
    j = np.arange(1, m + 1)
    lam = -2 * mu + 2 * mu * np.cos(j * np.pi / (m + 1))
    Q = np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * np.pi / (m + 1))
    return A, Q, lam


@pytest.mark.parametrize("m,want_sub", [(12, 64), (24, 8), (40, 2)])
def test_krylov_substeps_match_dst_closed_form(m, want_sub):
    # ||dt A_M||_1 = 4 mu = 50: a Krylov space of dimension m cannot meet the
    # tolerance in one step, so the action is taken as a product of equal
    # sub-steps exp(A) = exp(A/k)^k (section 4.3 with Saad's estimate).  A
    # sub-step that forgets to scale H, or miscounts the part of the step
    # already done, misses the closed form by O(1).
    A, Q, lam = _dst_diffusion_box(12.5)
    assert abs(np.abs(A).sum(axis=0).max() - 50.0) < 1e-12
    v = np.random.default_rng(3).standard_normal(A.shape[0])
    closed = Q @ (np.exp(lam) * (Q @ v))
    got, info = K.expv(lambda x: A @ x, v, m=m, tol=1e-14, return_info=True)
    assert info["substeps"] == want_sub
    assert rel_l2(got, closed) <= 1e-13
    # the same sub-steps taken by hand from the closed form of each fraction
    part = v.copy()
    for _ in range(want_sub):
        part = Q @ (np.exp(lam / want_sub) * (Q @ part))
    assert rel_l2(got, part) <= 1e-13


def test_krylov_substeps_variable_nu_box_match_dense_pade():
    # nonsymmetric 2D box (lognormal nu, advection (1, 0.5)) with a norm that
    # needs several sub-steps at m = 20 and 30; reference: the dense Pade
    # exponential (pinned against exact rational Taylor series and the DST
    # closed form above) and, independently, SciPy's expm
    n = 64
    dx = 1.0 / n
    nuf = L.lognormal_field_2d(n, 2) * 4.0
    W = op.weights(2, n, dx, 2 * dx, (1.0, 0.5), nu_field=nuf)
    box = P.uniform_boxes(2, n, 16, 4)[5]
    A = lem.local_matrix(op.sparse(W), P.gather_map(box, 2, n))
    v = np.random.default_rng(4).standard_normal(A.shape[0])
    ref = E.expm(A) @ v
    assert rel_l2(ref, sla.expm(A) @ v) <= 1e-13
    subs = []
    for m in (20, 30):
        got, info = K.expv(lambda x: A @ x, v, m=m, tol=1e-14, return_info=True)
        subs.append(info["substeps"])
        assert info["substeps"] > 1
        assert rel_l2(got, ref) <= 1e-13
    assert subs[0] > subs[1]  # a larger space takes fewer sub-steps


def test_global_krylov_matches_fft_2d():
    q = L.workload_2d_ensemble(n=64, n_states=2)
    W = op.from_problem(q)
    got = ge.krylov_step(W, q.states, m=30, tol=1e-14)
    assert rel_l2(got, ge.fft_steps(W, q.states)) < 1e-12


# ---------------------------------------------------------------- halo ----

def _per_step_inf_error(W, ndim, n, c, h, u):
    boxes = P.uniform_boxes(ndim, n, c, h)
    got = lem.step(op.sparse(W), boxes, ndim, n, u)
    ref = ge.fft_steps(W, u)
    return np.abs(got - ref).max() / np.abs(u).max()


@pytest.mark.parametrize("case", ["1d", "2d"])
def test_decay_bound_dominates_actual_error(case):
    if case == "1d":
        p = L.workload_1d()
        W, ndim, n, c = op.from_problem(p), 1, p.n, 64
        u = p.states[:, 0]
        hs = (8, 12, 16, 20)
    else:
        q = L.workload_2d_ensemble(n=64, n_states=1)
        W, ndim, n, c = op.from_problem(q), 2, q.n, 16
        u = L.white_noise_states(q.N, 1, 9)[:, 0]
        hs = (2, 4, 6, 8)
    G = H.growth_factor(W)
    for h in hs:
        box = P.uniform_boxes(ndim, n, c, h)[0]
        bound = H.eps(H.block_coefficients(W, box, ndim), h, ndim, G)
        actual = _per_step_inf_error(W, ndim, n, c, h, u)
        assert actual <= bound
        assert bound < 1e3 * actual  # and it is not vacuous


def test_decay_bound_minimizer_vs_brute_force():
    for (ws, wsb, w0, Pp, h) in [(6.096, 2.096, -8.192, 0.0, 16),
                                 (1.512, 0.488, -2.048, 1.024, 9),
                                 (0.5, 0.0, -1.0, 0.0, 5)]:
        t = np.linspace(-6, 6, 400001)
        phi = w0 + Pp + ws * np.exp(t) + wsb * np.exp(-t)
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            vals = np.log(np.expm1(phi) / phi) - h * t
        vals = vals[np.isfinite(vals)]
        brute = math.log(ws) + vals.min()
        assert abs(H.side_log_bound(ws, wsb, w0, Pp, h) - brute) < 1e-6


def test_halo_rule_and_tie_acceptance():
    p = L.workload_1d()
    W = op.from_problem(p)
    co = H.block_coefficients(W, P.uniform_boxes(1, p.n, 64, 16)[0], 1)
    h, clamped = H.halo_width(co, 1, 1e-6, 4, 40)
    assert not clamped and H.eps(co, h, 1) <= 1e-6 < H.eps(co, h - 1, 1)
    assert H.accepts(co, 1, 1e-6, 4, h) and not H.accepts(co, 1, 1e-6, 4, h + 1)
    assert H.halo_width(co, 1, 1e-30, 4, 10) == (10, True)


# --------------------------------------------------------- Schroedinger ----

def test_schrodinger_propagator_matches_eigendecomposition():
    """exp(-i dt H) of the oracle (complex Pade) against V exp(-i dt Lambda) V^T
    from the symmetric eigendecomposition of H, a different route."""
    n, Lx, kappa = 64, 10.0, 10.0
    dx = Lx / n
    dt = 4.0 * dx * dx
    H = SCH.hamiltonian(n, Lx, kappa).toarray()
    assert np.array_equal(H, H.T)
    lam, V = np.linalg.eigh(H)
    want = (V * np.exp(-1j * dt * lam)) @ V.T
    got = SCH.global_propagator(n, Lx, kappa, dt)
    assert np.abs(got - want).max() <= 1e-12
    # unitary: the global step conserves the l2 norm
    c = SCH.coherent_state(SCH.grid(n, Lx), kappa, 1.0, 2.0)
    assert abs(np.linalg.norm(got @ c) - np.linalg.norm(c)) <= 1e-12 * np.linalg.norm(c)


def test_schrodinger_free_plane_wave_closed_form():
    """kappa = 0: a discrete plane wave exp(i k x_j), k = 2 pi m / L, is an
    eigenvector of H with eigenvalue (1 - cos(k dx)) / dx^2."""
    n, Lx = 48, 10.0
    dx = Lx / n
    dt = 0.3
    x = SCH.grid(n, Lx)
    for m in (0, 1, 5, n // 2 - 1):
        k = 2 * np.pi * m / Lx
        c0 = np.exp(1j * k * x)
        lam = (1.0 - np.cos(k * dx)) / (dx * dx)
        got = SCH.global_run(c0, Lx, 0.0, dt, 3)
        assert np.abs(got - np.exp(-3j * dt * lam) * c0).max() <= 1e-11


def _phase_aligned_rel(a, ref):
    ph = np.vdot(ref, a)
    return np.linalg.norm(a - ref * ph / abs(ph)) / np.linalg.norm(a)


def test_schrodinger_coherent_state_second_order_in_space():
    """The semi-discrete solution of a coherent state follows the continuous
    one (Gaussian of fixed width whose centre moves as x0 cos(sqrt(kappa) t))
    with the O(dx^2) error of centered differences: halving dx divides the
    error at T = 0.5 by about 4."""
    Lx, kappa, T = 10.0, 10.0, 0.5
    errs = []
    for n in (100, 200):
        dx = Lx / n
        steps = 50
        dt = T / steps
        x = SCH.grid(n, Lx)
        c = SCH.global_run(SCH.coherent_state(x, kappa, 1.0), Lx, kappa, dt, steps)
        errs.append(_phase_aligned_rel(c, SCH.coherent_state_exact(x, kappa, 1.0, T)))
    assert errs[1] < 0.05
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_schrodinger_lem_single_domain_and_halo_convergence():
    """D = 1 (core = n, halo = 0) is the global method; with D > 1 the LEM
    error against it falls as the buffer widens."""
    n, Lx, kappa = 120, 10.0, 10.0
    dx = Lx / n
    dt = 2 * 4 * dx * dx  # mu = 4
    x = SCH.grid(n, Lx)
    c0 = np.column_stack([SCH.coherent_state(x, kappa, 1.0), SCH.coherent_state(x, kappa, -2.0, 3.0)])
    g = SCH.global_run(c0, Lx, kappa, dt, 6)

    def crel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)

    assert crel(SCH.lem_run(c0, Lx, kappa, dt, 6, n, 0), g) <= 1e-13
    errs = [crel(SCH.lem_run(c0, Lx, kappa, dt, 6, 30, h), g) for h in (4, 8, 12, 16, 20)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[0] > 1e-2 and errs[-1] < 1e-6


# ------------------------------------------- variable velocity, anisotropy ----

def test_vortex_advection_is_skew_steady_and_norm_preserving():
    """Centered conservative advection by face velocities taken from a stream
    function: dt*A is skew-symmetric (so exp(dt A) is orthogonal), rows sum
    to zero (the discrete divergence vanishes: constants are steady) and
    columns sum to zero (mass)."""
    n = 20
    dx = 1.0 / n
    F = L.vortex_faces(n, speed=1.3)
    A = op.dense(op.weights(2, n, dx, 2.0 * dx, (0.0, 0.0), nu=0.0, vel_faces=F))
    scale = np.abs(A).max()
    assert np.abs(A + A.T).max() <= 1e-14 * scale
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * scale
    assert np.abs(A.sum(axis=0)).max() <= 1e-13 * scale
    u = L.gaussian_blobs_2d(n, 3, seed=1)
    v = E.expm(A) @ u
    assert np.abs(np.linalg.norm(v, axis=0) / np.linalg.norm(u, axis=0) - 1).max() <= 1e-12
    # with diffusion the l2 norm decays and the mass stays
    Ad = op.dense(op.weights(2, n, dx, 2.0 * dx, (0.0, 0.0), nu=1e-2, vel_faces=F))
    w = E.expm(Ad) @ u
    assert np.all(np.linalg.norm(w, axis=0) < np.linalg.norm(u, axis=0))
    assert np.abs(w.sum(0) - u.sum(0)).max() <= 1e-12 * np.abs(u.sum(0)).max()


def test_vortex_turns_a_blob_about_the_centre():
    """psi = (1/pi) sin^2(pi x) sin^2(pi y) turns counter-clockwise about the
    centre with angular velocity omega(r) = sin(2 pi r) / r on the horizontal
    axis (2 pi at the centre): a small blob started at distance r0 to the
    right of the centre is, after the time of a quarter turn at omega(r0),
    above the centre (angle pi/2) at the same distance, within the
    discretization, shear and blob-size errors."""
    n = 96
    dx = 1.0 / n
    F = L.vortex_faces(n)
    r0, sig = 0.08, 0.02
    omega = np.sin(2 * np.pi * r0) / r0
    T = 0.5 * np.pi / omega
    steps = 40
    A = op.sparse(op.weights(2, n, dx, T / steps, (0.0, 0.0), nu=0.0, vel_faces=F))
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    u = np.exp(-((X - 0.5 - r0) ** 2 + (Y - 0.5) ** 2) / (2 * sig ** 2)).reshape(-1)
    from scipy.sparse.linalg import expm_multiply
    v = expm_multiply(A, u, start=0, stop=steps, num=2, endpoint=True)[-1]
    m = v.sum()
    cx = (v * X.reshape(-1)).sum() / m - 0.5
    cy = (v * Y.reshape(-1)).sum() / m - 0.5
    assert abs(np.arctan2(cy, cx) - np.pi / 2) < 0.06
    assert abs(np.hypot(cx, cy) - r0) < 0.006


def test_anisotropic_fourier_mode_closed_form():
    """dy != dx: a discrete Fourier mode exp(i (kx x + ky y)) is an
    eigenvector of the constant-coefficient operator with eigenvalue
    -4 nu sin^2(kx dx/2)/dx^2 - 4 nu sin^2(ky dy/2)/dy^2
    - i (a_x sin(kx dx)/dx + a_y sin(ky dy)/dy)."""
    n = 16
    dx, dy = 1.0 / n, 0.01 / n
    nu, vel, dt = 1e-4, (0.7, 0.02), 0.5 * (1.0 / n)
    A = op.dense(op.weights(2, n, dx, dt, vel, nu=nu, dy=dy))
    x = np.arange(n) * dx
    y = np.arange(n) * dy
    X, Y = np.meshgrid(x, y)
    for m, l in ((1, 0), (0, 1), (3, 2), (5, 7)):
        kx, ky = 2 * np.pi * m, 2 * np.pi * l / (n * dy)
        u = np.exp(1j * (kx * X + ky * Y)).reshape(-1)
        lam = (-4 * nu * np.sin(kx * dx / 2) ** 2 / dx ** 2 - 4 * nu * np.sin(ky * dy / 2) ** 2 / dy ** 2
               - 1j * (vel[0] * np.sin(kx * dx) / dx + vel[1] * np.sin(ky * dy) / dy))
        got = E.expm(A) @ u
        want = np.exp(dt * lam) * u
        assert np.abs(got - want).max() <= 1e-11


def test_vortex_lem_converges_to_global_with_halo():
    n = 24
    dx = 1.0 / n
    F = L.vortex_faces(n)
    A = op.sparse(op.weights(2, n, dx, 1.5 * dx, (0.0, 0.0), nu=1e-3, vel_faces=F))
    u = L.gaussian_blobs_2d(n, 2, seed=3)
    g = E.expm(A.toarray()) @ u
    errs = [rel_l2(lem.step(A, P.uniform_boxes(2, n, 8, h), 2, n, u), g) for h in (1, 2, 4, 7)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-5


def test_column_boxes_keep_the_vertical_wrap():
    """Column-wise decomposition (cores of c x n): with no coupling across
    columns (vertical advection-diffusion only, a_x = 0 and the x part of the
    diffusion switched off by a huge dx) the columns decouple, so column LEM
    with h = 0 equals the global exponential exactly -- which requires the
    periodic vertical couplings inside every column box."""
    n = 24
    dx, dy = 1e6, 1.0 / n
    W = op.weights(2, n, dx, 0.9 * dy, (0.0, 1.0), nu=2e-3, dy=dy)
    assert np.abs(W.wW).max() < 1e-12 and np.abs(W.wE).max() < 1e-12
    A = op.sparse(W)
    u = L.gaussian_blobs_2d(n, 2, seed=4)
    g = E.expm(A.toarray()) @ u
    boxes = P.column_boxes(n, 6, 0)
    P.check_tiling(boxes, 2, n)
    assert rel_l2(lem.step(A, boxes, 2, n, u), g) <= 1e-13
    # a square decomposition of the same problem cuts the columns and is not exact
    assert rel_l2(lem.step(A, P.uniform_boxes(2, n, 6, 2), 2, n, u), g) > 1e-6


def test_column_lem_converges_with_horizontal_buffer():
    """Anisotropic mesh (dy = dx / 8), large vertical Courant number, column
    boxes with buffers only across columns: the error falls with h, and the
    bound without y cuts dominates it."""
    n = 32
    dx, dy = 1.0 / n, 1.0 / (8 * n)
    F = L.vortex_faces(n, height=1.0 / 8)
    W = op.weights(2, n, dx, 0.5 * dx, (0.0, 0.0), nu=1e-5, vel_faces=F, dy=dy)
    A = op.sparse(W)
    u = L.gaussian_blobs_2d(n, 2, seed=6)
    g = E.expm(A.toarray()) @ u
    G = H.growth_factor(W)
    errs = []
    for h in (1, 2, 4, 6):
        boxes = P.column_boxes(n, 8, h)
        errs.append(rel_l2(lem.step(A, boxes, 2, n, u), g))
        co = H.block_coefficients(W, boxes[1], 2)
        assert H.eps(co, h, 2, G, cut_y=False) >= errs[-1] * 0.5
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6
