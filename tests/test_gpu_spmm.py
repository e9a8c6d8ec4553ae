"""GPU checks of the sparse-times-block product kernels (CSR, diagonal form, grid stencil
with registers, grid stencil staged in LDS) on the products the solver takes (Alg. 1 and 3:
Z = A P on an n x t block).

The diagonal-form and both grid-stencil kernels sum the same terms in the same ascending
column order as the CSR kernel, so for finite inputs they must agree bitwise, in FP64 and in
FP32.  The FP64 product is also held to the forward error bound of a dot product of at
most 7 terms against SciPy: |Y - A X| <= 16 u |A| |X|.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

pytestmark = pytest.mark.gpu

CSR_K, DIA_K, GRID_K, LDS_K, DMA_K = 0, 1, 2, 3, 4
TS = [1, 2, 4, 8, 16, 32, 64]
# cases where the LDS-staged grid kernel applies (3-D 7-point, unit x stride, nx a multiple
# of the 16-byte coefficient chunk); it needs at least 4 lanes per block row: t >= 8 in
# FP64, t >= 16 in FP32
LDS_CASES = {"box_20x12x7", "box_24x13x40", "box_64x6x33"}


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2305_19013_amd import ecg

    ecg.lib()
    return torch, torch.device("cuda:0")


def _csr(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return W.CSR(A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


def _products(torch, dev, csr, t, dtype, kernels, seed):
    from paper_2305_19013_amd import ecg

    op = ecg.Operator.from_csr(csr)
    X = np.random.default_rng(seed).standard_normal((csr.n, t)).astype(dtype)
    Xt = torch.from_numpy(X).to(dev)
    out = {}
    for k in kernels:
        Yt = torch.full_like(Xt, np.nan)
        ecg.debug_spmm_kernel(op, k, t, Xt, Yt)
        out[k] = Yt.cpu().numpy()
    return X, out


def _grid3d(nz, ny, nx, seed):
    """7-point operator with random coefficients per row (not symmetric: any matrix with
    these diagonals takes the grid kernel)."""
    A = W.fd_operator((nz, ny, nx), (0.3, 2.0, 1.0)).to_scipy().tocsr()
    A.data = A.data * np.random.default_rng(seed).uniform(0.5, 1.5, A.nnz)
    return A


CASES = {
    # nx not a multiple of the x tile, ny even, nz < one z segment
    "box_20x12x7": lambda: _grid3d(7, 12, 20, 1),
    # ny odd (ragged y pair), nz = 40: three z segments, the last one ragged
    "box_17x13x40": lambda: _grid3d(40, 13, 17, 2),
    # one x line per plane row pair, many planes
    "box_3x2x50": lambda: _grid3d(50, 2, 3, 3),
    # ny not a multiple of the LDS tile's 4 y rows, nz = 40: ragged y tiles and z segments
    "box_24x13x40": lambda: _grid3d(40, 13, 24, 4),
    # several x tiles per line, ny = 6 (one full and one ragged y tile), nz = 33
    "box_64x6x33": lambda: _grid3d(33, 6, 64, 5),
    # the 2-D jumping-coefficient operator (5 diagonals: the 2-D form of the kernel)
    "jump2d_64": lambda: W.config("jump2d512", scale=8).A.to_scipy(),
    # 2-D, lines of 33, 17 lines
    "fd2d_33x17": lambda: W.fd_operator((17, 33), (1.0, 4.0)).to_scipy(),
    # general offsets -60, -6, -2, 0, 2, 6, 60 with n = 7 * 60: b = 6, c = 60, a = 2
    "offsets_2_6_60": lambda: sp.diags([np.random.default_rng(9).uniform(-1, 1, 420 - abs(o)) + (5.0 if o == 0 else 0.0)
                                        for o in (-60, -6, -2, 0, 2, 6, 60)], [-60, -6, -2, 0, 2, 6, 60],
                                       shape=(420, 420), format="csr"),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("t", TS)
def test_grid_stencil_product_fp64(torch_dev, case, t):
    torch, dev = torch_dev
    A = CASES[case]()
    lds = case in LDS_CASES and t >= 8
    X, Y = _products(torch, dev, _csr(A), t, np.float64, (GRID_K, DIA_K, CSR_K) + ((LDS_K, DMA_K) if lds else ()),
                     seed=t)
    assert np.array_equal(Y[GRID_K], Y[DIA_K]) and np.array_equal(Y[DIA_K], Y[CSR_K])
    if lds:
        assert np.array_equal(Y[LDS_K], Y[DIA_K]) and np.array_equal(Y[DMA_K], Y[DIA_K])
    bound = 16 * 2.0 ** -53 * (abs(A) @ np.abs(X))
    assert np.all(np.abs(Y[GRID_K] - A @ X) <= bound + 1e-300)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("t", [1, 4, 16, 32, 64])
def test_grid_stencil_product_fp32(torch_dev, case, t):
    torch, dev = torch_dev
    A = CASES[case]()
    lds = case in LDS_CASES and t >= 16
    X, Y = _products(torch, dev, _csr(A), t, np.float32, (GRID_K, DIA_K, CSR_K) + ((LDS_K, DMA_K) if lds else ()),
                     seed=100 + t)
    assert np.array_equal(Y[GRID_K], Y[DIA_K]) and np.array_equal(Y[DIA_K], Y[CSR_K])
    if lds:
        assert np.array_equal(Y[LDS_K], Y[DIA_K]) and np.array_equal(Y[DMA_K], Y[DIA_K])
    A32 = A.astype(np.float32).astype(np.float64)  # the FP32 copy of the values
    bound = 16 * 2.0 ** -24 * (abs(A32) @ np.abs(X.astype(np.float64)))
    assert np.all(np.abs(Y[GRID_K] - A32 @ X.astype(np.float64)) <= bound)


@pytest.mark.parametrize("t", [8, 32])
def test_diagonal_form_with_many_diagonals_matches_csr(torch_dev, t):
    """11 diagonals (the 16-diagonal instance of the diagonal kernel), no grid form."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    offs = [-40, -21, -9, -3, -1, 0, 1, 3, 9, 21, 40]
    n = 997
    rng = np.random.default_rng(t)
    A = sp.diags([rng.uniform(-1, 1, n - abs(o)) for o in offs], offs, shape=(n, n), format="csr")
    X, Y = _products(torch, dev, _csr(A), t, np.float64, (DIA_K, CSR_K, ecg.SPMM_AUTO), seed=t)
    assert np.array_equal(Y[DIA_K], Y[CSR_K]) and np.array_equal(Y[ecg.SPMM_AUTO], Y[DIA_K])
    with pytest.raises(ecg.EcgError, match="grid"):
        _products(torch, dev, _csr(A), t, np.float64, (GRID_K,), seed=t)


def test_kernel_availability(torch_dev):
    """The grid form needs b | c and c | n; the diagonal form at most 16 diagonals."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    A = sp.diags([np.ones(421 - abs(o)) for o in (-60, -6, -2, 0, 2, 6, 60)], [-60, -6, -2, 0, 2, 6, 60],
                 shape=(421, 421), format="csr")  # 60 does not divide 421
    _products(torch, dev, _csr(A), 4, np.float64, (DIA_K,), seed=1)
    with pytest.raises(ecg.EcgError, match="grid"):
        _products(torch, dev, _csr(A), 4, np.float64, (GRID_K,), seed=1)
    R = sp.random(500, 500, density=0.05, random_state=np.random.default_rng(3), format="csr")
    S = _csr(R + R.T + sp.eye(500))
    with pytest.raises(ecg.EcgError, match="diagonal"):
        _products(torch, dev, S, 4, np.float64, (DIA_K,), seed=1)
    with pytest.raises(ecg.EcgError):
        _products(torch, dev, _csr(_grid3d(4, 4, 4, 0)), 4, np.float64, (6,), seed=1)
    # the SELL-C-sigma form is kept only for matrices without a diagonal form
    with pytest.raises(ecg.EcgError, match="SELL"):
        _products(torch, dev, _csr(_grid3d(4, 4, 4, 0)), 4, np.float64, (5,), seed=1)
    # the LDS-staged grid kernel: not for 2 lanes per row (FP64 t = 4), an odd nx, a non-unit
    # x stride or a 2-D operator
    for A, t in ((_grid3d(4, 4, 8, 0), 4), (_grid3d(4, 4, 17, 0), 32), (CASES["offsets_2_6_60"](), 32),
                 (CASES["jump2d_64"](), 32)):
        for kern in (LDS_K, DMA_K):
            with pytest.raises(ecg.EcgError, match="LDS"):
                _products(torch, dev, _csr(A), t, np.float64, (kern,), seed=1)


@pytest.mark.parametrize("t", [16, 32, 64])
def test_grid_stencil_full_size_equals_diagonal_form(torch_dev, t):
    """The 128^3 anisotropic operator of the benchmark: both grid kernels and the diagonal
    kernel bitwise equal on the whole block, FP64 and FP32."""
    torch, dev = torch_dev
    from paper_2305_19013_amd import ecg

    p = W.config("aniso3d128")
    op = ecg.Operator.from_csr(p.A)
    for dt in (torch.float64, torch.float32):
        g = torch.Generator(device=dev).manual_seed(t)
        Xt = torch.randn((p.n, t), dtype=dt, device=dev, generator=g)
        Yg, Yd, Yl, Ym = (torch.empty_like(Xt) for _ in range(4))
        ecg.debug_spmm_kernel(op, GRID_K, t, Xt, Yg)
        ecg.debug_spmm_kernel(op, DIA_K, t, Xt, Yd)
        ecg.debug_spmm_kernel(op, LDS_K, t, Xt, Yl)
        ecg.debug_spmm_kernel(op, DMA_K, t, Xt, Ym)
        torch.cuda.synchronize()
        assert bool(torch.equal(Yg, Yd)) and bool(torch.equal(Yl, Yd)) and bool(torch.equal(Ym, Yd))
        del Xt, Yg, Yd, Yl, Ym


@pytest.mark.parametrize("variant", [0, 1])
def test_fp32_refined_solve_on_3d_stencil(torch_dev, variant):
    """The FP32 form on a 3-D 7-point operator (32^3 anisotropic, t = 32 -> 16), so that its
    products run on the FP32 grid-stencil kernel; SRE-CG2 and MSDO-CG: the FP64 true
    residual recomputed on the host reaches 1e-8."""
    torch, dev = torch_dev
    from oracle import ecg as ora
    from paper_2305_19013_amd import ecg

    p = W.config("aniso3d128", scale=4)
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    bt = torch.from_numpy(p.b).to(dev)
    xt = torch.zeros_like(bt)
    rep, _ = ecg.solve(op, P, bt, xt, ecg.options(tol=1e-8, precision=1, inner_tol=1e-4, variant=variant,
                                                  reduce=p.reduce, switch_tol=p.switch_tol, t_min=p.t_min))
    assert rep["status"] == "ok"
    assert ora.true_relres(p.A.to_scipy(), p.b, xt.cpu().numpy()) <= 1.01e-8
