"""Pins of the oracle's barycentric solvers and closest-point routine against
mathematics that does not come from the oracle itself.

* App. B coefficients (eqs A11-A16) == the symbolic expansion of
  adj(F(t)) p and det F(t) under linear vertex motion (eq 7 -> eq 8), done by
  sympy here.
* Barycentric identities (eq 1): sum w = 1, F(t) w(t) = p, w(v_i(t)) = e_i.
* App. B closest point by edge projections == the solution of the convex QP
  min |F w - q|^2 over the simplex (solved by scipy here).
"""
import numpy as np
import pytest
import sympy as sp

import oracle


def _sym_coeffs():
    t, u, v = sp.symbols("t u v")
    x0 = sp.symbols("x0_0 x1_0 x2_0")
    y0 = sp.symbols("y0_0 y1_0 y2_0")
    x1 = sp.symbols("x0_1 x1_1 x2_1")
    y1 = sp.symbols("y0_1 y1_1 y2_1")
    xt = [(1 - t) * a + t * b for a, b in zip(x0, x1)]
    yt = [(1 - t) * a + t * b for a, b in zip(y0, y1)]
    F = sp.Matrix([xt, yt, [1, 1, 1]])
    N = F.adjugate() * sp.Matrix([u, v, 1])
    D = F.det()
    polyN = [sp.Poly(sp.expand(N[i]), t) for i in range(3)]
    polyD = sp.Poly(sp.expand(D), t)
    syms = list(x0) + list(y0) + list(x1) + list(y1) + [u, v]

    def coef(p, deg):
        return sp.lambdify(syms, p.coeff_monomial(t ** deg), "numpy")

    A = [[coef(polyN[i], d) for i in range(3)] for d in (2, 1, 0)]
    a = [coef(polyD, d) for d in (2, 1, 0)]
    return A, a


@pytest.fixture(scope="module")
def sym():
    return _sym_coeffs()


def test_appendix_b_coefficients_match_symbolic_expansion(sym):
    A, a = sym
    rng = np.random.default_rng(11)
    for _ in range(25):
        x0, y0, x1, y1 = (rng.uniform(-1, 1, 3) for _ in range(4))
        u, v = rng.uniform(-1, 1, 2)
        A1, A2, A3, av = oracle.fast_coeffs(x0, y0, x1, y1, u, v)
        args = list(x0) + list(y0) + list(x1) + list(y1) + [u, v]
        for d, got in enumerate((A1, A2, A3)):
            want = np.array([A[d][i](*args) for i in range(3)], float)
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)
        want_a = np.array([a[d](*args) for d in range(3)], float)
        np.testing.assert_allclose(av, want_a, rtol=1e-12, atol=1e-13)


def _w_fast(x0, y0, x1, y1, u, v, t):
    A1, A2, A3, a = oracle.fast_coeffs(x0, y0, x1, y1, u, v)
    return (A1 * t * t + A2 * t + A3) / (a[0] * t * t + a[1] * t + a[2])


def test_barycentric_identities_of_fast_solver():
    rng = np.random.default_rng(12)
    for _ in range(50):
        x0, y0, x1, y1 = (rng.uniform(-1, 1, 3) for _ in range(4))
        t = rng.uniform(0, 1)
        u, v = rng.uniform(-1, 1, 2)
        w = _w_fast(x0, y0, x1, y1, u, v, t)
        xt, yt = (1 - t) * x0 + t * x1, (1 - t) * y0 + t * y1
        area = abs((xt[1] - xt[0]) * (yt[2] - yt[0]) - (xt[2] - xt[0]) * (yt[1] - yt[0]))
        if area < 1e-3:
            continue
        assert abs(w.sum() - 1) < 1e-11
        np.testing.assert_allclose([w @ xt, w @ yt], [u, v], atol=1e-10)
        for i in range(3):
            wi = _w_fast(x0, y0, x1, y1, xt[i], yt[i], t)
            np.testing.assert_allclose(wi, np.eye(3)[i], atol=1e-10)


def _qp_closest(tri, q):
    from scipy.optimize import minimize
    tri = np.asarray(tri, float)

    def f(ab):
        p = tri[0] + ab[0] * (tri[1] - tri[0]) + ab[1] * (tri[2] - tri[0])
        return float(np.sum((p - q) ** 2))

    best = None
    for x0 in ([0.2, 0.2], [0.9, 0.05], [0.05, 0.9], [0.0, 0.0]):
        r = minimize(f, x0, method="SLSQP", bounds=[(0, 1), (0, 1)],
                     constraints=[{"type": "ineq", "fun": lambda ab: 1 - ab[0] - ab[1]}],
                     options={"ftol": 1e-15, "maxiter": 500})
        if best is None or r.fun < best.fun:
            best = r
    return best.fun


def test_closest_point_by_edge_projection_equals_simplex_qp():
    rng = np.random.default_rng(13)
    n = 0
    while n < 60:
        tri = rng.uniform(-1, 1, (3, 2))
        q = rng.uniform(-2, 2, 2)
        # App. B uses the edge search only for points outside the triangle
        M = np.array([[tri[0, 0], tri[1, 0], tri[2, 0]], [tri[0, 1], tri[1, 1], tri[2, 1]], [1, 1, 1]])
        if abs(np.linalg.det(M)) < 1e-2:
            continue
        w = np.linalg.solve(M, [q[0], q[1], 1.0])
        if w.min() >= 0:
            continue
        ws = oracle.closest_point(tri, q)
        assert ws.min() >= 0 and abs(ws.sum() - 1) < 1e-12 and (ws == 0).sum() >= 1
        d_edge = float(np.sum((ws @ tri - q) ** 2))
        d_qp = _qp_closest(tri, q)
        assert d_edge <= d_qp + 1e-9
        assert d_edge >= d_qp - 1e-7 * max(1.0, d_qp)
        n += 1


def test_schedule_matches_global_uniform_times():
    # t_k = k/(K-1) (Sec. 3.2) spread over S equal segments: t_k = (s + tau)/S
    for K in (1, 2, 5, 16, 64, 65, 512):
        for S in (1, 2, 3, 12, 36, 60):
            for k in range(K):
                s, tau, X = oracle.schedule(k, K, S)
                t = 0.0 if K == 1 else k / (K - 1)
                assert 0 <= s < S and 0.0 <= tau <= 1.0
                assert abs((s + tau) / S - t) < 1e-14
                assert X == (0 if tau <= 0.5 else 1)
