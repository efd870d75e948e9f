"""Pins of the oracle's exact stencil algebra against values the paper prints.

Every expected value here is either printed in the paper (loaded from
tests/golden/paper_values.json, which cites the section/equation/table) or a
closed form derived in the test from first principles (trigonometric
symbols, factorial expansions); none comes from the code under test.
"""

import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import rational as R

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _from_golden_1d(e):
    offs = range(e["first_offset"], e["first_offset"] + len(e["weights"]))
    return R.stencil1d(offs, [F(w, e["den"]) for w in e["weights"]], e["p"])


def _from_rows(e):
    rows = e["rows_top_to_bottom"]
    r = len(rows) // 2
    pts = {}
    for a, row in enumerate(rows):
        y = r - a
        for b, w in enumerate(row):
            x = b - r
            if w:
                pts[(x, y)] = F(w, e["den"])
    return R.RStencil(2, e["p"], pts)


NAMED_1D = {
    "D1 o D1 (central)": lambda: R.compose(R.central_first(), R.central_first()),
    "forward D2 o forward D1": lambda: R.compose(R.forward_second(), R.forward_first()),
    "central D1 (2nd order) o central D1 (4th order)": lambda: R.compose(R.central_first(), R.central_first_4th()),
    "d/dx o d2/dx2 (central)": lambda: R.compose(R.central_first(), R.central_second()),
    "d/dx o d/dx o d2/dx2 (central)": lambda: R.compose(R.central_first(), R.compose(R.central_first(), R.central_second())),
    "d2/dx2 o d2/dx2 (central)": lambda: R.compose(R.central_second(), R.central_second()),
}


@pytest.mark.parametrize("entry", GOLD["stencils_1d"], ids=lambda e: e["name"])
def test_printed_1d_compositions(entry):
    assert NAMED_1D[entry["name"]]() == _from_golden_1d(entry)


def test_printed_laplacian_and_bilaplacian():
    lap, bilap = GOLD["stencils_2d"]
    L = R.laplacian(2)
    assert L == _from_rows(lap)
    assert R.compose(L, L) == _from_rows(bilap)
    assert R.compose(L, L).npts() == 13


def test_derived_closed_forms_25pt_and_33pt():
    # Derived by hand from the definition (each axis pair of the two factors):
    # 3D: centre 6*6 + 6 = 42, axis-1: -12, edge diagonals 2, axis-2: 1.
    B3 = R.biharmonic(3)
    nums, den = B3.integer_form()
    assert den == 1 and B3.p == 4 and B3.npts() == 25
    for off, w in nums.items():
        a = sorted(abs(c) for c in off)
        expect = {(0, 0, 0): 42, (0, 0, 1): -12, (0, 1, 1): 2, (0, 0, 2): 1}[tuple(a)]
        assert w == expect
    # 2D fourth-order cross (-1,16,-30,16,-1)/12 composed with itself, /144 h^4
    B33 = R.biharmonic(2, fourth_order=True)
    nums, den = B33.integer_form()
    assert den == 144 and B33.npts() == 33
    table = {(0, 0): 4628, (0, 1): -1952, (1, 1): 512, (0, 2): 376, (1, 2): -32,
             (0, 3): -32, (2, 2): 2, (0, 4): 1}
    for off, w in nums.items():
        assert w == table[tuple(sorted(abs(c) for c in off))]
    assert sum(nums.values()) == 0
    assert sum(abs(v) for v in nums.values()) == 16384


TAYLOR_STENCILS = {
    "central_first": R.central_first,
    "central_second": R.central_second,
    "D1oD1": lambda: R.compose(R.central_first(), R.central_first()),
    "fwdD2ofwdD1": lambda: R.compose(R.forward_second(), R.forward_first()),
    "central_first_4th": R.central_first_4th,
    "D1oD1_4th": lambda: R.compose(R.central_first(), R.central_first_4th()),
    "central_first_ex1": R.central_first,
    "central_second_ex1": R.central_second,
    "D2oD1_ex1": lambda: R.compose(R.central_second(), R.central_first()),
    "D2_4th_o_D2_4th": lambda: R.compose(R.central_second_4th(), R.central_second_4th()),
    "D1_4th_o_D2_4th": lambda: R.compose(R.central_first_4th(), R.central_second_4th()),
}


@pytest.mark.parametrize("entry", GOLD["taylor_1d"], ids=lambda e: e["stencil"])
def test_printed_taylor_series(entry):
    T, beta = R.normalized_series1d(TAYLOR_STENCILS[entry["stencil"]](), len(entry["T"]))
    assert beta == entry["beta"]
    assert T == [F(v) for v in entry["T"]]


def test_taylor_of_single_source_point_matches_factorials():
    # eq. (taylor2): a single source point at u contributes u^k/k!
    for u in (-3, -1, 2, 5):
        s = R.stencil1d([u], [1], 0)
        assert R.taylor1d(s, 6) == [F(u) ** k / math.factorial(k) for k in range(7)]


def test_commutativity_and_associativity():
    A, B, C = R.forward_first(), R.central_second(), R.central_first_4th()
    assert R.compose(A, B) == R.compose(B, A)  # the lemma of Sec. 2.2.1
    assert R.compose(R.compose(A, B), C) == R.compose(A, R.compose(B, C))
    L2 = R.laplacian(2)
    X = R.embed(R.forward_first(), 0, 2)
    assert R.compose(L2, X) == R.compose(X, L2)


def test_order_lemma_and_coefficient_proposition():
    # Lemma (Accuracy) and Proposition (CoeffAccuracy): q_c = min(q_a, q_b),
    # t_qc = t_qa, t_qb or their sum.
    cases = [
        (R.central_first(), R.central_first_4th()),
        (R.central_second(), R.central_first()),
        (R.central_second_4th(), R.central_first_4th()),
        (R.forward_first(), R.forward_second()),
        (R.central_second(), R.central_second_4th()),
    ]
    for a, b in cases:
        pa, qa, ta = R.derivative_and_accuracy(a)
        pb, qb, tb = R.derivative_and_accuracy(b)
        pc, qc, tc = R.derivative_and_accuracy(R.compose(b, a))
        assert pc == pa + pb
        assert qc == min(qa, qb)
        if qa < qb:
            assert tc == ta
        elif qb < qa:
            assert tc == tb
        else:
            assert tc == ta + tb


def test_composed_series_is_cauchy_product():
    # eq. (AccuracyComposition): T_{B(A)} is the Cauchy product of T_A and T_B.
    for a, b in [(R.central_first(), R.central_second()), (R.forward_first(), R.forward_second()),
                 (R.central_first_4th(), R.central_second_4th())]:
        Ta, _ = R.normalized_series1d(a, 10)
        Tb, _ = R.normalized_series1d(b, 10)
        Tc, _ = R.normalized_series1d(R.compose(b, a), 10)
        assert Tc == R.cauchy_product(Ta, Tb, 10)


def test_retarget_example():
    e = GOLD["retarget_example"]
    T = [F(v) for v in e["T"]]
    corr = R.retarget_correction(T, e["shift"], len(e["correction"]))
    assert corr == [F(v) for v in e["correction"]]
    assert [x + y for x, y in zip(T, corr)] == [F(v) for v in e["sum"]]


def test_retarget_matches_shifted_stencil():
    # Re-targeting the second derivative from y0 = x0 + h equals the Taylor
    # series of the same weights placed at offsets shifted by +1.
    shifted = R.stencil1d([2, 1, 0], [1, -2, 1], 2)
    raw = R.taylor1d(shifted, 8)[2:]
    T, _ = R.normalized_series1d(R.central_second(), 6)
    corr = R.retarget_correction(T, 1, 6)
    assert [x + y for x, y in zip(T, corr)] == raw[:6]


def _array2d(s, px, py, size):
    raw = R.taylor(s, px + py + 2 * size)
    return {(i, j): raw[(px + i, py + j)] for i in range(size) for j in range(size)}


def test_two_dimensional_outer_products():
    # Sec. 2.3: composing stencils along different axes multiplies their series.
    dx = R.embed(R.central_first(), 0, 2)
    dy = R.embed(R.central_first(), 1, 2)
    arr = _array2d(R.compose(dy, dx), 1, 1, 5)
    for key, val in GOLD["taylor_2d_mixed_first"]["entries"].items():
        i, j = map(int, key.split(","))
        assert arr[(i, j)] == F(val)
    # Sec. 3.2: f^(4,3) from fourth-order factors
    d4 = R.compose(R.central_second_4th(), R.central_second_4th())
    d3 = R.compose(R.central_first_4th(), R.central_second_4th())
    st = R.compose(R.embed(d3, 1, 2), R.embed(d4, 0, 2))
    arr = _array2d(st, 4, 3, 5)
    for key, val in GOLD["taylor_2d_corner"]["entries"].items():
        i, j = map(int, key.split(","))
        assert arr[(i, j)] == F(val)
    # the whole 5x5 corner is the outer product of the 1D series
    T4, _ = R.normalized_series1d(d4, 5)
    T3, _ = R.normalized_series1d(d3, 5)
    for i in range(5):
        for j in range(5):
            assert arr[(i, j)] == T4[i] * T3[j]


def _fit(hs, errs):
    A = np.vstack([np.log(hs), np.ones(len(hs))]).T
    p, logc = np.linalg.lstsq(A, np.log(errs), rcond=None)[0]
    return p, math.exp(logc)


def _eval_at(st, f, x0, h):
    offs, w = st.float_weights(h)
    return sum(wk * f(*(np.asarray(x0) + h * o)) for o, wk in zip(offs, w))


def test_one_dimensional_example_fit():
    # Sec. 3.1: f = sin x cos x, f''' at pi by central D2 o central D1;
    # expected order 2 with coefficient f^(5)(pi)/4 = 4 (printed fit 1.9976 / 3.9432).
    st = R.compose(R.central_second(), R.central_first())
    f = lambda x: math.sin(x) * math.cos(x)
    exact = 4 * math.sin(math.pi) ** 2 - 4 * math.cos(math.pi) ** 2
    hs = np.array([2.0 ** -k for k in range(3, 8)])
    errs = np.array([abs(_eval_at(st, f, [math.pi], h) - exact) for h in hs])
    p, C = _fit(hs, errs)
    assert abs(p - 2) < 0.01
    assert abs(C - GOLD["fits"]["ex1_expected_coeff"]) < 0.05


def test_two_dimensional_example_fit():
    # Sec. 3.2: f = sin(x+y), f^(4,3) at (2 pi, pi/3), fourth order with
    # coefficient 1/30 (printed fit 3.9997 / 3.324e-2).
    d4 = R.compose(R.central_second_4th(), R.central_second_4th())
    d3 = R.compose(R.central_first_4th(), R.central_second_4th())
    st = R.compose(R.embed(d3, 1, 2), R.embed(d4, 0, 2))
    f = lambda x, y: math.sin(x) * math.cos(y) + math.cos(x) * math.sin(y)
    x0 = (2 * math.pi, math.pi / 3)
    exact = math.sin(x0[0]) * math.sin(x0[1]) - math.cos(x0[0]) * math.cos(x0[1])
    hs = np.array([0.2, 0.16, 0.125, 0.1])
    errs = np.array([abs(_eval_at(st, f, x0, h) - exact) for h in hs])
    p, C = _fit(hs, errs)
    assert abs(p - 4) < 0.02
    assert abs(C - 1 / 30) < 0.002


def test_stability_constants():
    # Table (stability) and App. B: dt <= alpha h^4 from the Fourier symbol.
    e = GOLD["stability"]
    th = np.linspace(0, 2 * math.pi, 200001)[:, None]
    comp = R.compose(R.central_first(), R.compose(R.central_first(), R.central_second()))
    s = R.symbol(comp, th).real  # symbol of d/dx o d/dx o d2/dx2 (h = 1)
    # f_t = -D f gives xi = 1 - dt sigma_D / h^4; the printed bracket
    # (cos + 2cos2 - cos3 - 2) is -2 sigma_D
    assert abs(-2 * s.max() - float(F(e["symbol_min_dx_o_dx_o_dxx"]))) < 1e-8
    assert abs(2.0 / s.max() - float(F(e["alpha_dx_o_dx_o_dxx"]))) < 1e-8
    d4 = R.compose(R.central_second(), R.central_second())
    s4 = R.symbol(d4, th).real
    assert abs(2.0 / s4.max() - float(F(e["alpha_dxx_o_dxx"]))) < 1e-12
    # heat equation (Sec. 2.2.3)
    s_c = R.symbol(R.compose(R.central_first(), R.central_first()), th).real
    s_k = R.symbol(R.central_second(), th).real
    assert abs(2.0 / (-s_c.min()) - float(F(e["heat_composed_dt_over_h2"]))) < 1e-12
    assert abs(2.0 / (-s_k.min()) - float(F(e["heat_compact_dt_over_h2"]))) < 1e-12


def test_symbol_of_composition_is_product():
    rng = np.random.default_rng(5)
    th = rng.uniform(-math.pi, math.pi, size=(64, 2))
    A = R.compose(R.embed(R.forward_first(), 0, 2), R.laplacian(2))
    B = R.embed(R.central_first_4th(), 1, 2)
    np.testing.assert_allclose(R.symbol(R.compose(B, A), th), R.symbol(A, th) * R.symbol(B, th),
                               rtol=1e-12, atol=1e-12)


def test_table_bilaplacian_spectrum():
    # Sec. 4.6, Table (bilap_prop). Periodic [0,200]^2, n = 200/h: the
    # eigenvalues of a periodic convolution are its symbol at theta = 2 pi k/n.
    B = R.biharmonic(2)
    for row in GOLD["table_bilaplacian"]["rows"]:
        h, dt = row["h"], row["dt"]
        n = int(round(200 / h))
        k = 2 * math.pi * np.arange(n) / n
        th = np.stack(np.meshgrid(k, k, indexing="ij"), axis=-1)
        lam = R.symbol(B, th, h).real
        rho = np.abs(lam).max()
        step = 1 + dt * lam
        tol = 5e-5 if row["rho_B"] < 1 else 1e-9 * row["rho_B"]
        assert abs(rho - row["rho_B"]) <= tol
        assert abs(np.abs(step).max() - row["rho_step"]) <= 5e-4
        assert abs(np.abs(step).max() / np.abs(step).min() - row["cond_step"]) <= 5e-4


def test_table_sparsity():
    # Sec. 4.7, Table (sparsity): 5 n^2 vs 13 n^2 non-zeros.
    L = R.laplacian(2)
    B = R.compose(L, L)
    for row in GOLD["table_sparsity"]["rows"][:3]:
        n = int(round(200 / row["h"]))
        assert n * n == row["size"]
        assert R.nnz_of_assembled(L, (n, n)) == row["nnz_lap"]
        assert R.nnz_of_assembled(B, (n, n)) == row["nnz_bilap"]
    for row in GOLD["table_sparsity"]["rows"][3:]:
        n = int(round(200 / row["h"]))
        assert 5 * n * n == row["nnz_lap"] and 13 * n * n == row["nnz_bilap"]


@pytest.mark.parametrize("n", [3, 4, 5, 7, 9])
def test_bruteforce_periodic_matrix_product(n):
    # Composition replaces the sparse matrix-matrix product (Sec. 1): on a
    # periodic grid the composed stencil's matrix is the product of the
    # factor matrices, including aliasing when n < 2R+1.
    pairs = [
        (R.laplacian(2), R.laplacian(2)),
        (R.embed(R.forward_first(), 0, 2), R.laplacian(2)),
        (R.laplacian(2, True), R.laplacian(2, True)),
        (R.embed(R.central_first_4th(), 1, 2), R.embed(R.forward_second(), 0, 2)),
    ]
    for A, B in pairs:
        C = R.compose(B, A)
        MA = R.assemble_dense(A, (n, n), True)
        MB = R.assemble_dense(B, (n, n), True)
        MC = R.assemble_dense(C, (n, n), True)
        np.testing.assert_allclose(MC, MB @ MA, rtol=0, atol=1e-12)


def test_bruteforce_ring_matrix_product():
    # With prescribed ring values the composed stencil on the unknowns equals
    # the inner stencil evaluated on unknowns + ring R_outer, followed by the
    # outer stencil: a product of rectangular matrices.
    def rect(st, n, ring_out, ring_in):
        rows = [(i, j) for j in range(-ring_out, n + ring_out) for i in range(-ring_out, n + ring_out)]
        cols = {(i, j): c for c, (i, j) in enumerate((i, j) for j in range(-ring_in, n + ring_in)
                                                     for i in range(-ring_in, n + ring_in))}
        M = np.zeros((len(rows), len(cols)))
        offs, w = st.float_weights()
        for r, (i, j) in enumerate(rows):
            for o, wk in zip(offs, w):
                M[r, cols[(i + o[0], j + o[1])]] += wk
        return M
    for A, B in [(R.laplacian(2), R.laplacian(2)), (R.laplacian(2, True), R.laplacian(2))]:
        C = R.compose(B, A)
        ra, rb = A.radius(), B.radius()
        for n in (4, 7):
            MC = rect(C, n, 0, ra + rb)
            prod = rect(B, n, 0, rb) @ rect(A, n, rb, ra + rb)
            np.testing.assert_allclose(MC, prod, rtol=0, atol=1e-12)


def test_lincomb_ch_operator_weights():
    # I + dt eps^2 L o L - dt S L with eps = 4h, dt = h^2/10, S = 2 in grid
    # units: centre 1 + 1.6*20 + 0.2*4, axis-1 1.6*(-8) - 0.2, diagonal 3.2,
    # axis-2 1.6; the row sum is 1.
    A = R.ch_operator(2, F(4), F(1, 10), F(2))
    w = A.weights
    assert w[(0, 0)] == F(338, 10) and w[(1, 0)] == F(-13) and w[(1, 1)] == F(32, 10) and w[(2, 0)] == F(16, 10)
    assert sum(w.values()) == 1
    A3 = R.ch_operator(3, F(4), F(1, 10), F(2))
    assert sum(A3.weights.values()) == 1 and A3.npts() == 25
    assert A3.weights[(0, 0, 0)] == 1 + F(16, 10) * 42 + F(2, 10) * 6
