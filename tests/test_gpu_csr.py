"""GPU parity of the assembled (CSR) form of composed stencils.

Structure is index work and must be bit-exact: the row pointers and column
indices equal those read off the oracle's assembly on small grids (taps that
alias on grids narrower than the stencil merge into one entry), and the
entry count equals Table 3's (13 n^2 for the 13-point bi-Laplacian on a
periodic grid) and the closed form sum_t prod_a (n_a - |u_t,a|) with a zero
ring. Values equal the dense matrix's (bit-exact for integer weights, to
rounding where aliased weights are summed). y = A x by rocSPARSE is compared
with the oracle's apply under the same bar as the matrix-free sweeps
(bit-exact on integer inputs, 1e-12 of max |W||x| in FP64, 1e-5 in FP32).
"""

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import capi
from oracle import rational as R
from tests.gpu_util import lib_stencil, scaled_error

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def native():
    from paper_2205_03354_amd import _native

    return _native


def _ops():
    return {
        "bilap2": R.biharmonic(2),
        "bilap2_4th": R.biharmonic(2, True),
        "bilap3": R.biharmonic(3),
        "lap2": R.laplacian(2),
        "fwd": R.compose(R.embed(R.forward_first(), 0, 2), R.embed(R.forward_second(), 1, 2)),
    }


def _oracle_rows(op, n, periodic):
    # columns of every row from the definition (x fastest), duplicates merged
    dim = op.dim
    strides = [int(np.prod(n[:k])) for k in range(dim)]
    rows = []
    for lin in range(int(np.prod(n))):
        idx = [(lin // strides[a]) % n[a] for a in range(dim)]
        cols = set()
        for off in op.weights:
            nb = [idx[a] + off[a] for a in range(dim)]
            if periodic:
                nb = [v % m for v, m in zip(nb, n)]
            elif any(v < 0 or v >= m for v, m in zip(nb, n)):
                continue
            cols.add(sum(v * s for v, s in zip(nb, strides)))
        rows.append(sorted(cols))
    return rows


@pytest.mark.parametrize("name,n,periodic", [
    ("bilap2", (7, 6), True), ("bilap2", (7, 6), False), ("bilap2", (3, 4), True),
    ("bilap2_4th", (9, 10), True), ("bilap2_4th", (5, 3), True), ("bilap2_4th", (6, 11), False),
    ("bilap3", (5, 4, 6), True), ("bilap3", (3, 5, 4), False), ("bilap3", (2, 3, 2), True),
    ("fwd", (6, 5), True), ("fwd", (6, 5), False),
])
def test_structure_and_values_match_the_oracle_assembly(native, name, n, periodic):
    op = _ops()[name]
    bc = native.SC_CSR_PERIODIC if periodic else native.SC_CSR_ZERO_RING
    h = 0.25
    A = native.Csr(lib_stencil(native, op), tuple(reversed(n)), bc, h=h)
    rp, col, val = A.export()
    rows = _oracle_rows(op, list(n), periodic)
    assert A.rows == len(rows)
    assert A.nnz == R.nnz_of_assembled(op, n, periodic) == sum(len(r) for r in rows)
    assert np.array_equal(rp, np.cumsum([0] + [len(r) for r in rows]))
    assert np.array_equal(col, np.concatenate([np.array(r, dtype=np.int32) for r in rows]))
    dense = R.assemble_dense(op, n, periodic, h)
    ref = np.concatenate([dense[i, r] for i, r in enumerate(rows)])
    aliased = periodic and A.nnz < op.npts() * A.rows
    if not aliased and op.integer_form()[1] == 1:
        assert np.array_equal(val, ref)  # one exactly representable weight per entry
    else:  # weights num/den rounded once; aliased ones summed
        assert np.max(np.abs(val - ref)) <= 4.5e-16 * np.max(np.abs(ref))
    A.close()


@pytest.mark.parametrize("n", [64, 1025])
def test_table3_nnz_at_scale(native, n):
    for op, per_row in ((R.laplacian(2), 5), (R.biharmonic(2), 13)):
        A = native.Csr(lib_stencil(native, op), (n, n), native.SC_CSR_PERIODIC)
        assert A.nnz == per_row * n * n
        A.close()
    op = R.biharmonic(2, True)
    A = native.Csr(lib_stencil(native, op), (n, n + 3), native.SC_CSR_ZERO_RING)
    closed = sum((n + 3 - abs(o[0])) * (n - abs(o[1])) for o in op.weights)
    assert A.nnz == closed
    A.close()


@pytest.mark.parametrize("name,shape", [("bilap2", (77, 301)), ("bilap2_4th", (130, 257)),
                                        ("bilap3", (20, 17, 33)), ("fwd", (35, 70))])
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("alg", ["rowsplit", "adaptive"])
def test_spmv_parity(native, name, shape, periodic, alg):
    op = _ops()[name]
    bc = native.SC_CSR_PERIODIC if periodic else native.SC_CSR_ZERO_RING
    mode = capi.PERIODIC if periodic else capi.ZERO_RING
    a = native.SC_CSR_ROWSPLIT if alg == "rowsplit" else native.SC_CSR_ADAPTIVE
    st = lib_stencil(native, op)
    h = 1.0 / 64
    x = S.uniform_field(shape, seed=51)
    ref = capi.apply(op, x, mode, 0, h)
    A = native.Csr(st, shape, bc, h=h, alg=a)
    y = torch.full(shape, float("nan"), dtype=torch.float64, device=DEV)
    for _ in range(2):  # the second product reuses the prepared workspace
        A.spmv(torch.from_numpy(x).to(DEV), y)
        torch.cuda.synchronize()
        assert scaled_error(y.cpu().numpy(), ref, op, x, mode, 0, h) <= 1e-12
    A.close()
    A32 = native.Csr(st, shape, bc, h=h, dtype=torch.float32, alg=a)
    y32 = torch.empty(shape, dtype=torch.float32, device=DEV)
    A32.spmv(torch.from_numpy(x).to(DEV, torch.float32), y32)
    torch.cuda.synchronize()
    assert scaled_error(y32.double().cpu().numpy(), ref, op, x, mode, 0, h) <= 1e-5
    A32.close()


@pytest.mark.parametrize("name,shape", [("bilap2", (64, 129)), ("bilap3", (16, 9, 33))])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_integer_bit_exact(native, name, shape, dtype):
    op = _ops()[name]
    x = S.integer_field(shape, seed=52)
    for periodic in (True, False):
        bc = native.SC_CSR_PERIODIC if periodic else native.SC_CSR_ZERO_RING
        mode = capi.PERIODIC if periodic else capi.ZERO_RING
        A = native.Csr(lib_stencil(native, op), shape, bc, dtype=dtype)
        y = torch.empty(shape, dtype=dtype, device=DEV)
        A.spmv(torch.from_numpy(x).to(DEV, dtype), y)
        torch.cuda.synchronize()
        assert np.array_equal(y.double().cpu().numpy(), capi.apply(op, x, mode))
        A.close()


def test_spmv_matches_matrix_free_apply(native):
    # the assembled and the matrix-free forms of one operator on one input
    from paper_2205_03354_amd import stencils

    st = stencils.biharmonic(2, True)
    shape = (257, 300)
    x = torch.from_numpy(S.uniform_field(shape, seed=53)).to(DEV)
    y_mf = torch.empty_like(x)
    native.apply_composed(st, x, y_mf, native.SC_BC_PERIODIC)
    A = native.Csr(st, shape, native.SC_CSR_PERIODIC)
    y_csr = torch.empty_like(x)
    A.spmv(x, y_csr)
    torch.cuda.synchronize()
    op = R.biharmonic(2, True)
    xs = x.cpu().numpy()
    assert scaled_error(y_csr.cpu().numpy(), y_mf.cpu().numpy(), op, xs, capi.PERIODIC) <= 1e-13
    A.close()


def test_csr_errors(native):
    op = R.biharmonic(2)
    st = lib_stencil(native, op)
    A = native.Csr(st, (16, 16), native.SC_CSR_PERIODIC)
    x = torch.zeros((16, 16), dtype=torch.float64, device=DEV)
    with pytest.raises(native.ScError):  # y aliases x
        A.spmv(x, x)
    with pytest.raises(native.ScError):  # dtype mismatch
        A.spmv(x, torch.zeros((16, 16), dtype=torch.float32, device=DEV))
    with pytest.raises(native.ScError):  # shape mismatch
        A.spmv(x, torch.zeros((16, 17), dtype=torch.float64, device=DEV))
    with pytest.raises(native.ScError):  # non-contiguous rows
        big = torch.zeros((16, 20), dtype=torch.float64, device=DEV)
        A.spmv(x, big[:, :16])
    A.close()
    with pytest.raises(native.ScError):  # dimension mismatch with the stencil
        native.Csr(st, (4, 4, 4), native.SC_CSR_PERIODIC)
