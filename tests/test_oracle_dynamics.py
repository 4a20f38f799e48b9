"""Pins for the oracle's dynamics (eq. 1) and integrators (PropagateODE, eq. 2).

Double integrator: Euler's recursion has a closed form; RK4 is exact for the
quadratic trajectory p0 + v0 t + a t^2 / 2.

Quadcopter: the oracle's component formulas are checked against an
independent numpy construction (rotation-matrix product, inverse of the
angular-rate matrix, cross product), against special cases with closed
forms (hover, vertical thrust, pure yaw torque, torque-free principal-axis
spin), and its RK4 against scipy's DOP853 driven by the numpy construction.
"""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from workloads import problem_small_di, problem_small_quad, RK4, EULER


def di(integrator=EULER):
    return problem_small_di(integrator=integrator)


def quad():
    return problem_small_quad()


def integrate(p, x0, u, k):
    x = np.array(x0, np.float64)
    for _ in range(k):
        x = oracle.step(p, x, u)
    return x


@pytest.mark.parametrize("seed", range(5))
def test_di_euler_closed_form(seed):
    p = di(EULER)
    h = float(np.float32(p["h"]))
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-5, 5, 6)
    u = rng.uniform(-1, 1, 3)
    K = 10
    x = integrate(p, x0, u, K)
    # v_K = v0 + K h u ; p_K = p0 + K h v0 + h^2 u K (K - 1) / 2
    v_want = x0[3:] + K * h * u
    p_want = x0[:3] + K * h * x0[3:] + h * h * u * K * (K - 1) / 2
    np.testing.assert_allclose(x[3:], v_want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x[:3], p_want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_di_rk4_exact_for_quadratics(seed):
    p = di(RK4)
    h = float(np.float32(p["h"]))
    rng = np.random.default_rng(seed + 10)
    x0 = rng.uniform(-5, 5, 6)
    u = rng.uniform(-1, 1, 3)
    K = 10
    x = integrate(p, x0, u, K)
    t = K * h
    np.testing.assert_allclose(x[:3], x0[:3] + x0[3:] * t + 0.5 * u * t * t, atol=1e-12)
    np.testing.assert_allclose(x[3:], x0[3:] + u * t, atol=1e-12)


# --- independent quadcopter construction -----------------------------------
def Rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def Ry(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def Rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def quad_rhs_numpy(p, x, u):
    m, g, Ixx, Iyy, Izz = [float(v) for v in np.asarray(p["dyn_params"], np.float32)[:5]]
    phi, th, psi = x[3:6]
    w = x[9:12]
    R = Rz(psi) @ Ry(th) @ Rx(phi)                  # body -> inertial, ZYX
    acc = R @ np.array([0.0, 0.0, u[0] / m]) - np.array([0.0, 0.0, g])
    # body rates from Euler-angle rates: w = E(phi, th) dTheta
    E = np.array([[1, 0, -np.sin(th)],
                  [0, np.cos(phi), np.sin(phi) * np.cos(th)],
                  [0, -np.sin(phi), np.cos(phi) * np.cos(th)]])
    dTheta = np.linalg.solve(E, w)
    I = np.diag([Ixx, Iyy, Izz])
    dw = np.linalg.solve(I, np.array(u[1:4]) - np.cross(w, I @ w))
    return np.concatenate([x[6:9], dTheta, acc, dw])


def random_quad_state(rng):
    x = np.zeros(12)
    x[:3] = rng.uniform(10, 90, 3)
    x[3:5] = rng.uniform(-0.9, 0.9, 2)
    x[5] = rng.uniform(-3, 3)
    x[6:9] = rng.uniform(-8, 8, 3)
    x[9:12] = rng.uniform(-4, 4, 3)
    return x


@pytest.mark.parametrize("seed", range(10))
def test_quad_deriv_matches_matrix_construction(seed):
    p = quad()
    rng = np.random.default_rng(seed)
    x = random_quad_state(rng)
    u = np.array([rng.uniform(0, 19.62), *rng.uniform(-0.1, 0.1, 3)])
    np.testing.assert_allclose(oracle.deriv(p, x, u), quad_rhs_numpy(p, x, u), rtol=1e-12,
                               atol=1e-12)


def test_quad_hover_fixed_point():
    p = quad()
    m, g = [float(v) for v in np.asarray(p["dyn_params"], np.float32)[:2]]
    x0 = np.zeros(12)
    x0[:3] = [50, 50, 50]
    x0[5] = 0.7  # yaw does not matter at hover
    u = np.array([m * g, 0, 0, 0])
    assert np.max(np.abs(oracle.deriv(p, x0, u))) < 1e-14
    x = integrate(p, x0, u, 20)
    np.testing.assert_allclose(x, x0, atol=1e-12)


def test_quad_vertical_thrust_closed_form():
    p = quad()
    m, g = [float(v) for v in np.asarray(p["dyn_params"], np.float32)[:2]]
    h = float(np.float32(p["h"]))
    T = 13.0
    x0 = np.zeros(12)
    x0[:3] = [30, 40, 20]
    x0[8] = 1.5
    x = integrate(p, x0, np.array([T, 0, 0, 0]), 20)
    t = 20 * h
    a = T / m - g
    assert x[2] == pytest.approx(20 + 1.5 * t + 0.5 * a * t * t, abs=1e-12)
    assert x[8] == pytest.approx(1.5 + a * t, abs=1e-12)
    np.testing.assert_allclose(x[[0, 1, 3, 4, 5, 6, 7, 9, 10, 11]],
                               x0[[0, 1, 3, 4, 5, 6, 7, 9, 10, 11]], atol=1e-14)


def test_quad_pure_yaw_torque():
    p = quad()
    Izz = float(np.float32(p["dyn_params"][4]))
    m, g = [float(v) for v in np.asarray(p["dyn_params"], np.float32)[:2]]
    h = float(np.float32(p["h"]))
    tz = 0.07
    x0 = np.zeros(12)
    x0[:3] = [50, 50, 50]
    x = integrate(p, x0, np.array([m * g, 0, 0, tz]), 20)
    t = 20 * h
    assert x[5] == pytest.approx(0.5 * tz / Izz * t * t, abs=1e-12)
    assert x[11] == pytest.approx(tz / Izz * t, abs=1e-12)


@pytest.mark.parametrize("axis", [9, 10, 11])
def test_quad_torque_free_principal_spin(axis):
    p = quad()
    x0 = np.zeros(12)
    x0[:3] = [50, 50, 50]
    x0[axis] = 2.0
    d = oracle.deriv(p, x0, np.array([0.0, 0, 0, 0]))
    assert np.all(d[9:12] == 0.0)


def test_quad_rk4_vs_dop853_and_order():
    p = quad()
    rng = np.random.default_rng(3)
    h = float(np.float32(p["h"]))
    for _ in range(4):
        x0 = random_quad_state(rng)
        x0[3:5] *= 0.5
        u = np.array([rng.uniform(5, 15), *rng.uniform(-0.1, 0.1, 3)])
        T = 20 * h
        ref = solve_ivp(lambda t, y: quad_rhs_numpy(p, y, u), (0, T), x0, method="DOP853",
                        rtol=1e-12, atol=1e-12).y[:, -1]
        x_h = integrate(p, x0, u, 20)
        err_h = np.max(np.abs(x_h - ref))
        assert err_h < 1e-5  # RK4 truncation at h = 0.02 over 0.4 s
        # halve the step: global error should shrink ~16x (4th order)
        p2 = dict(p)
        p2["h"] = np.float32(h / 2)
        x_h2 = integrate(p2, x0, u, 40)
        err_h2 = np.max(np.abs(x_h2 - ref))
        if err_h > 1e-10:
            assert 10.0 < err_h / err_h2 < 24.0


def test_di_euler_vs_exact_deviation_bound():
    # Euler's end point differs from the exact double-integrator trajectory by
    # u h^2 K / 2 per axis: 0.05 |u| for K = 10, h = 0.1.
    p = di(EULER)
    h = float(np.float32(p["h"]))
    u = np.array([1.0, -1.0, 0.5])
    x0 = np.zeros(6)
    x = integrate(p, x0, u, 10)
    exact = 0.5 * u * (10 * h) ** 2
    np.testing.assert_allclose(exact - x[:3], u * h * h * 10 / 2, atol=1e-12)


@pytest.mark.parametrize("integrator", [RK4, EULER])
def test_quad_displacement_bound(integrator):
    """The bound the expansion's obstacle culling rests on.  The acceleration
    is thrust / m times a rotation-matrix column, less g along z, so per axis
    it lies in [-A, A] (x, y) and [-A - g, A - g] (z), A = max thrust / m; then
    after j steps p_j - p0 - j h v0 lies in [a_lo, a_hi] (j h)^2 / 2 per axis,
    from any start state (angles and rates unbounded) and any admissible
    control."""
    from workloads import problem_c2
    p = problem_c2(integrator=integrator)
    h = float(np.float32(p["h"]))
    K = int(p["steps"])
    A = float(p["u_hi"][0]) / float(p["dyn_params"][0])
    g = float(p["dyn_params"][1])
    a_lo = np.array([-A, -A, -A - g])
    a_hi = np.array([A, A, A - g])
    rng = np.random.default_rng(7)
    worst_lo = worst_hi = 0.0
    for _ in range(150):
        x0 = np.zeros(12)
        x0[:3] = rng.uniform(20.0, 80.0, 3)
        x0[3:6] = rng.uniform(-3.0, 3.0, 3)
        x0[6:9] = rng.uniform(-10.0, 10.0, 3)
        x0[9:] = rng.uniform(-8.0, 8.0, 3)
        u = rng.uniform(p["u_lo"], p["u_hi"])
        x = x0.copy()
        for j in range(1, K + 1):
            x = oracle.step(p, x, u)
            dev = x[:3] - x0[:3] - j * h * x0[6:9]
            w = (j * h) ** 2 / 2
            assert np.all(dev >= a_lo * w - 1e-12 * (1 + np.abs(a_lo * w))), (j, dev, a_lo * w)
            assert np.all(dev <= a_hi * w + 1e-12 * (1 + np.abs(a_hi * w))), (j, dev, a_hi * w)
            worst_lo = max(worst_lo, float(np.max(dev[:2] / (a_lo[:2] * w))))
            worst_hi = max(worst_hi, float(np.max(dev[:2] / (a_hi[:2] * w))))
    # not vacuous: horizontal displacements come within a factor 3 of both ends
    assert worst_lo > 1.0 / 3.0 and worst_hi > 1.0 / 3.0
