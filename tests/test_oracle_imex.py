"""Pins of the spinodal-decomposition oracle with IMEX Runge-Kutta steps.

* the tableau pairs satisfy the Runge-Kutta order conditions of their order
  for each tableau and for the coupling terms (exact rationals for orders 1
  and 3), and are stiffly accurate (the last stage is the new value);
* with the non-linear part switched off (rho = 0) one step multiplies a
  periodic Fourier mode by the implicit method's stability function
  R(z) = 1 + z b^T (I - z A)^-1 1 at z = dt times the mode's eigenvalue of
  -M kappa L o L, the eigenvalue being the square of the Laplacian's symbol;
* the observed temporal orders against a fine-step reference are 1, 2 and 3;
* mass is conserved and the free energy decreases along the benchmark's
  trajectory; the free energy's gradient term equals -(kappa/2) <c, L c>
  (summation by parts);
* the initial condition has mean about 0.5, as the benchmark states.
"""

import math
from fractions import Fraction as F

import numpy as np
import pytest

import synthetic as S
from oracle import imex as I


def _conditions(b, A, bh, Ah):
    c = [sum(r) for r in A]
    ch = [sum(r) for r in Ah]
    n = len(b)
    out = {}
    out["c=chat"] = all(c[i] == ch[i] for i in range(n)) if isinstance(c[0], F) else \
        max(abs(c[i] - ch[i]) for i in range(n))
    for name, u in (("b", b), ("bhat", bh)):
        out[f"sum {name}"] = sum(u)
        out[f"sum {name} c"] = sum(u[i] * c[i] for i in range(n))
        out[f"sum {name} c^2"] = sum(u[i] * c[i] * c[i] for i in range(n))
        for vn, V in (("A", A), ("Ahat", Ah)):
            out[f"sum {name} {vn} c"] = sum(u[i] * V[i][j] * c[j] for i in range(n) for j in range(n))
    return out


@pytest.mark.parametrize("order", [1, 3])
def test_exact_tableaux_satisfy_order_conditions(order):
    Ah, bh, A, b = I.tableau_exact(order)
    n = len(b)
    for i in range(n):
        assert all(Ah[i][j] == 0 for j in range(i, n))  # explicit: strictly lower
        assert all(A[i][j] == 0 for j in range(i + 1, n))  # implicit: lower
    assert A[0][0] == 0
    assert b == A[-1] and bh == Ah[-1]  # stiffly accurate
    cond = _conditions(b, A, bh, Ah)
    assert cond["c=chat"] is True
    for u in ("b", "bhat"):
        assert cond[f"sum {u}"] == 1
        if order >= 2:
            assert cond[f"sum {u} c"] == F(1, 2)
        if order >= 3:
            assert cond[f"sum {u} c^2"] == F(1, 3)
            assert cond[f"sum {u} A c"] == F(1, 6)
            assert cond[f"sum {u} Ahat c"] == F(1, 6)
    if order == 1:  # and not more
        assert cond["sum b c"] != F(1, 2) or cond["sum bhat c"] != F(1, 2)


def test_order2_tableau_conditions():
    T = I.tableau(2)
    cond = _conditions(T.b, T.A, T.bhat, T.Ahat)
    assert cond["c=chat"] <= 1e-16
    for u in ("b", "bhat"):
        assert abs(cond[f"sum {u}"] - 1) <= 1e-15
        assert abs(cond[f"sum {u} c"] - 0.5) <= 1e-15
    # the diagonal makes the implicit part L-stable: R(z) -> 0 as z -> -inf
    assert T.b == T.A[-1] and T.bhat == T.Ahat[-1]


def _stability(T, z):
    A = np.array(T.A)
    b = np.array(T.b)
    n = len(b)
    return 1.0 + z * b @ np.linalg.solve(np.eye(n) - z * A, np.ones(n))


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("dim", [2, 3])
def test_linear_mode_follows_the_stability_function(order, dim):
    p = I.Params(h=0.5, M=5.0, kappa=2.0, rho=0.0)
    n = 12
    k = (1, 2, 3)[:dim]
    idx = np.indices((n,) * dim)  # axis 0 is z (3D) or y (2D); x last
    theta = [2 * math.pi * k[a] / n for a in range(dim)]
    phase = sum(theta[a] * idx[dim - 1 - a] for a in range(dim))
    c = np.cos(phase)
    sym = -(4.0 / p.h ** 2) * sum(math.sin(t / 2) ** 2 for t in theta)
    lam = -p.M * p.kappa * sym * sym
    dt = 0.01
    got, _ = I.imex_step(c, dt, order, p, tol=1e-14)
    assert np.max(np.abs(got - _stability(I.tableau(order), dt * lam) * c)) <= 1e-11


@pytest.mark.parametrize("order,lo,hi", [(1, 0.9, 1.1), (2, 1.9, 2.1)])
def test_temporal_order_on_the_benchmark(order, lo, hi):
    # the benchmark's coefficients (stiff: dt |lambda_max| up to 40 here)
    p = I.Params()
    c0 = S.spinodal_initial(2, 24)
    T = 0.25
    ref, _ = I.integrate(c0, T / 512, 512, 3, p, tol=1e-13)
    errs = []
    for m in (16, 32, 64):
        c, _ = I.integrate(c0, T / m, m, order, p, tol=1e-13)
        errs.append(float(np.max(np.abs(c - ref))))
    rate = math.log(errs[1] / errs[2]) / math.log(2.0)
    assert lo <= rate <= hi, (errs, rate)


def test_temporal_order_three():
    # a milder stiffness (M kappa = 0.01) shows the third order of the pair
    # without the reduction the stiff regime brings to a method of stage
    # order one (the benchmark's coefficients give rates 2.7-2.9 over
    # dt |lambda_max| = 10 .. 0.3)
    p = I.Params(kappa=0.02, M=0.5)
    c0 = S.spinodal_initial(2, 24)
    T = 2.0
    ref, _ = I.integrate(c0, T / 1024, 1024, 3, p, tol=1e-14)
    errs = []
    for m in (32, 64, 128):
        c, _ = I.integrate(c0, T / m, m, 3, p, tol=1e-14)
        errs.append(float(np.max(np.abs(c - ref))))
    rate = math.log(errs[1] / errs[2]) / math.log(2.0)
    assert 2.8 <= rate <= 3.2, (errs, rate)


def test_mass_and_energy_along_the_benchmark():
    p = I.Params()
    c = S.spinodal_initial(2, 40)
    m0, e0 = I.free_energy(c, p)
    prev = e0
    for _ in range(10):
        c, _ = I.imex_step(c, 0.05, 2, p, tol=1e-13)
        m, e = I.free_energy(c, p)
        assert abs(m - m0) <= 1e-12 * abs(m0)
        assert e <= prev + 1e-12 * abs(prev)
        prev = e
    assert prev < e0


def test_free_energy_summation_by_parts():
    from oracle import capi
    from oracle import rational as R

    p = I.Params(h=0.5)
    c = S.spinodal_initial(3, 10, h=0.5)
    _, e = I.free_energy(c, p)
    bulk = p.h ** 3 * float(np.sum(p.rho * (c - p.ca) ** 2 * (c - p.cb) ** 2))
    Lc = capi.apply(R.laplacian(3), c, capi.PERIODIC, 0, p.h)
    grad = -0.5 * p.kappa * p.h ** 3 * float(np.sum(c * Lc))
    assert abs(e - (bulk + grad)) <= 1e-12 * abs(e)


def test_initial_condition_mean():
    for dim, n in ((2, 200), (3, 64)):
        c = S.spinodal_initial(dim, n)
        assert abs(float(np.mean(c)) - 0.5) < 0.01
        # the three terms lie in [-1, 1], [0, 1], [-1, 1] and all equal 1 at the origin
        assert float(np.min(c)) >= 0.5 - 0.02 and float(np.max(c)) <= 0.5 + 0.03
        assert c.flat[0] == 0.5 + 0.01 * 3
