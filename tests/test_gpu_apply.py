"""GPU parity of the composed-stencil apply against the CPU oracle.

Bars: integer-valued inputs with integer weights are bit-exact (FP64 and
FP32: every partial sum is an integer below 2^24); random FP64 inputs agree
to 1e-12 of max(|W| |x|) (the scaled error of the apply); random FP32
inputs to 2e-6 of the same scale (a few FP32 ulps of the summed terms).
"""

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import capi
from oracle import rational as R
from tests.gpu_util import lib_stencil, padded, scaled_error

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def native():
    from paper_2205_03354_amd import _native

    return _native


def _random_stencil(dim, R_, seed, pattern="box"):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = {}
    rngs = [range(-R_, R_ + 1)] * dim
    import itertools

    for off in itertools.product(*rngs):
        if pattern == "box" or sum(abs(o) for o in off) <= R_:
            w[tuple(reversed(off))] = int(rng.integers(-9, 10))
    return R.RStencil(dim, 0, w)


STENCILS_2D = {
    "lap5": lambda: R.laplacian(2),
    "lap9_4th": lambda: R.laplacian(2, True),
    "bilap13": lambda: R.biharmonic(2),
    "bilap33": lambda: R.biharmonic(2, True),
    "fwd_mixed": lambda: R.compose(R.embed(R.forward_first(), 0, 2), R.embed(R.central_second_4th(), 1, 2)),
    "box1": lambda: _random_stencil(2, 1, 1),
    "box3": lambda: _random_stencil(2, 3, 3),
    "box4": lambda: _random_stencil(2, 4, 4),
}

SIZES_2D = [(5, 7), (63, 65), (257, 129), (1000, 37), (1030, 300)]


def _run(native, st, x_np, bc, halo, dtype, h=1.0):
    x = torch.from_numpy(x_np).to(DEV, dtype)
    y = torch.full_like(x, float("nan"))
    native.apply_composed(lib_stencil(native, st), x, y, bc, h=h, halo=halo)
    torch.cuda.synchronize()
    out = y.double().cpu().numpy()
    if halo:
        inner = tuple(slice(halo, s - halo) for s in out.shape)
        out = out[inner]
    return out


@pytest.mark.parametrize("name", list(STENCILS_2D))
@pytest.mark.parametrize("size", SIZES_2D)
def test_apply2d_periodic_f64_random(native, name, size):
    st = STENCILS_2D[name]()
    n0, n1 = size
    x = S.uniform_field((n1, n0), seed=n0 * 7 + n1)
    got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64)
    ref = capi.apply(st, x, capi.PERIODIC)
    assert scaled_error(got, ref, st, x, capi.PERIODIC) <= 1e-12


@pytest.mark.parametrize("name", list(STENCILS_2D))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_apply2d_integer_bit_exact(native, name, dtype):
    st = STENCILS_2D[name]()
    nums, den = st.integer_form()
    sti = R.RStencil(2, 0, dict(nums))  # integer weights, h = 1
    for (n0, n1), halo in [((70, 33), 0), ((257, 19), 4)]:
        x = S.integer_field((n1 + 2 * halo, n0 + 2 * halo), seed=n0, lo=-64, hi=64)
        bc = native.SC_BC_HALO if halo else native.SC_BC_PERIODIC
        got = _run(native, sti, x, bc, halo, dtype)
        ref = capi.apply(sti, x, capi.HALO if halo else capi.PERIODIC, halo)
        assert np.array_equal(got, ref), (n0, n1, halo)


@pytest.mark.parametrize("name", ["bilap13", "bilap33", "box4", "fwd_mixed"])
@pytest.mark.parametrize("size", [(63, 65), (1030, 300)])
def test_apply2d_halo_f64_and_f32(native, name, size):
    st = STENCILS_2D[name]()
    r = st.radius()
    n0, n1 = size
    x = padded(S.uniform_field((n1, n0), seed=5), r, fill_seed=6)
    ref = capi.apply(st, x, capi.HALO, r)
    got = _run(native, st, x, native.SC_BC_HALO, r, torch.float64)
    assert scaled_error(got, ref, st, x, capi.HALO, r) <= 1e-12
    got32 = _run(native, st, x, native.SC_BC_HALO, r, torch.float32)
    x32 = x.astype(np.float32).astype(np.float64)
    ref32 = capi.apply(st, x32, capi.HALO, r)
    assert scaled_error(got32, ref32, st, x32, capi.HALO, r) <= 2e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9])
def test_apply2d_tiny_periodic_aliasing(native, n):
    # grids smaller than the stencil: offsets alias modulo n
    for st in (R.biharmonic(2, True), _random_stencil(2, 4, 9)):
        x = S.uniform_field((n, n + 1), seed=n)
        got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64)
        ref = capi.apply(st, x, capi.PERIODIC)
        assert scaled_error(got, ref, st, x, capi.PERIODIC) <= 1e-12


def test_apply2d_scaled_weights_h(native):
    st = R.biharmonic(2, True)
    x, h = S.periodic_sin_mode(2, 64)
    got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64, h=h)
    ref = capi.apply(st, x, capi.PERIODIC, 0, h)
    assert scaled_error(got, ref, st, x, capi.PERIODIC, 0, h) <= 1e-12


def test_composed_equals_sequential_on_gpu(native):
    # one pass of L o L == two passes of L (bit-exact for integer data)
    from paper_2205_03354_amd import stencils

    L = stencils.laplacian(2)
    LL = stencils.biharmonic(2)
    n0, n1 = 301, 77
    x = torch.from_numpy(S.integer_field((n1 + 4, n0 + 4), seed=2, lo=-100, hi=100)).to(DEV)
    mid = torch.zeros((n1 + 2, n0 + 2), dtype=torch.float64, device=DEV)
    # inner pass on unknowns + ring 1: view the halo-2 input as a halo-1 grid
    # around the (n0+2, n1+2) block, writing into `mid`
    native.apply_composed(L, x, mid, native.SC_BC_HALO, h=1.0, halo=1, out_halo=0)
    out_seq = torch.zeros((n1, n0), dtype=torch.float64, device=DEV)
    native.apply_composed(L, mid, out_seq, native.SC_BC_HALO, h=1.0, halo=1, out_halo=0)
    out_c = torch.zeros_like(out_seq)
    native.apply_composed(LL, x, out_c, native.SC_BC_HALO, h=1.0, halo=2, out_halo=0)
    torch.cuda.synchronize()
    assert torch.equal(out_seq, out_c)


STENCILS_3D = {
    "lap7": lambda: R.laplacian(3),
    "bilap25": lambda: R.biharmonic(3),
    "box1": lambda: _random_stencil(3, 1, 11),
    "box2": lambda: _random_stencil(3, 2, 12),
    "lap13_4th": lambda: R.laplacian(3, True),
}


@pytest.mark.parametrize("name", list(STENCILS_3D))
@pytest.mark.parametrize("size", [(5, 6, 7), (33, 17, 20), (70, 9, 40)])
def test_apply3d_f64(native, name, size):
    st = STENCILS_3D[name]()
    n0, n1, n2 = size
    x = S.uniform_field((n2, n1, n0), seed=n0 + n1 + n2)
    got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64)
    ref = capi.apply(st, x, capi.PERIODIC)
    assert scaled_error(got, ref, st, x, capi.PERIODIC) <= 1e-12
    r = st.radius()
    xh = padded(x, r, fill_seed=3)
    got = _run(native, st, xh, native.SC_BC_HALO, r, torch.float64)
    ref = capi.apply(st, xh, capi.HALO, r)
    assert scaled_error(got, ref, st, xh, capi.HALO, r) <= 1e-12


@pytest.mark.parametrize("name", ["lap7", "bilap25", "box1"])
@pytest.mark.parametrize("size", [(256, 13, 37), (128, 128, 40), (130, 9, 21)])
def test_apply3d_f64_multi_tile(native, name, size):
    # Mirror-symmetric 3D stencils take the wave-per-tile DMA-ring sweep:
    # several x strips, a ragged last row tile and several ragged z chunks;
    # (130, ...) has a partial last strip.
    st = STENCILS_3D[name]()
    n0, n1, n2 = size
    x = S.uniform_field((n2, n1, n0), seed=n0 + 3 * n1 + 7 * n2)
    got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64)
    ref = capi.apply(st, x, capi.PERIODIC)
    assert scaled_error(got, ref, st, x, capi.PERIODIC) <= 1e-12
    r = st.radius()
    xh = padded(x, r, fill_seed=5)
    got = _run(native, st, xh, native.SC_BC_HALO, r, torch.float64)
    ref = capi.apply(st, xh, capi.HALO, r)
    assert scaled_error(got, ref, st, xh, capi.HALO, r) <= 1e-12


@pytest.mark.parametrize("name", ["lap7", "bilap25"])
def test_apply3d_integer_bit_exact_f32_multi_tile(native, name):
    st = STENCILS_3D[name]()
    nums, den = st.integer_form()
    sti = R.RStencil(3, 0, dict(nums))
    x = S.integer_field((23, 18, 512), seed=6, lo=-32, hi=32)
    got = _run(native, sti, x, native.SC_BC_PERIODIC, 0, torch.float32)
    assert np.array_equal(got, capi.apply(sti, x, capi.PERIODIC))


@pytest.mark.parametrize("name", list(STENCILS_3D))
def test_apply3d_integer_bit_exact_f32(native, name):
    st = STENCILS_3D[name]()
    nums, den = st.integer_form()
    sti = R.RStencil(3, 0, dict(nums))
    x = S.integer_field((19, 23, 70), seed=4, lo=-32, hi=32)
    got = _run(native, sti, x, native.SC_BC_PERIODIC, 0, torch.float32)
    assert np.array_equal(got, capi.apply(sti, x, capi.PERIODIC))


def test_apply_full_size_4097_33pt(native):
    # The benchmark workload in its launch configuration: 4097^2 FP64,
    # periodic, fourth-order biharmonic (33 taps), checked at every point.
    st = R.biharmonic(2, True)
    n = 4097
    x = S.uniform_field((n, n), seed=0)
    got = _run(native, st, x, native.SC_BC_PERIODIC, 0, torch.float64, h=1.0 / n)
    ref = capi.apply(st, x, capi.PERIODIC, 0, 1.0 / n)
    assert scaled_error(got, ref, st, x, capi.PERIODIC, 0, 1.0 / n) <= 1e-12


def test_apply_rejects_unsupported(native):
    st = _random_stencil(3, 3, 1)  # 3D radius 3: no kernel
    x = torch.zeros((8, 8, 8), dtype=torch.float64, device=DEV)
    y = torch.zeros_like(x)
    with pytest.raises(native.ScError) as e:
        native.apply_composed(lib_stencil(native, st), x, y, native.SC_BC_PERIODIC)
    assert e.value.status == native.SC_EUNSUPPORTED
