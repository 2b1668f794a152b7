"""GPU FP64 band solve (the macro linear solve of every Newton update) through
the C ABI, against a dense FP64 solve of the same matrix.

Block cyclic reduction cuts the matrix into blocks of the bandwidth rounded up
to 16; the cases cover one block, a ragged last block, block counts that are
not powers of two, bandwidths below, at and just above a tile boundary, the
three factor placements (a block's lower triangle in LDS; its first steps in
global memory and the trailing triangle in LDS; all of it in global memory),
the 2D macro tangent's size (8450 unknowns, half bandwidth 133) with a
grid-Laplacian-like matrix, and the non-positive-definite report.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe2():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2312_12771_amd import fe2 as f
    return f


def band_of(A, bw):
    n = A.shape[0]
    band = np.zeros((n, bw + 1))
    for d in range(bw + 1):
        band[: n - d, d] = np.diagonal(A, -d)
    return band


def random_spd_band(n, bw, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for d in range(1, bw + 1):
        v = rng.uniform(-1.0, 1.0, n - d)
        A += np.diag(v, -d) + np.diag(v, d)
    # symmetric, diagonally dominant with a spread of scales
    A += np.diag(np.abs(A).sum(1) + rng.uniform(0.5, 2.0, n))
    s = np.exp(rng.uniform(-3.0, 3.0, n))
    return A * s[:, None] * s[None, :]


def solve_gpu(fe2, n, bw, band, b, allow=False):
    bd = torch.tensor(band.ravel(), dtype=torch.float64, device="cuda")
    x = torch.tensor(b, dtype=torch.float64, device="cuda")
    st, piv = fe2.fe2_band_solve(n, bw, bd, x, allow_notspd=allow)
    return st, piv, x.cpu().numpy(), bd.cpu().numpy()


# (2187, 275): blocks of 18 tile rows, factored first in global memory and
# then with the trailing triangle in LDS; (2300, 1100): blocks too wide for
# any tile of the triangle next to the panel, factored in global memory
@pytest.mark.parametrize("n,bw", [(1, 0), (7, 0), (16, 15), (17, 3), (100, 7), (301, 16), (513, 17),
                                  (1000, 33), (2187, 275), (2300, 1100)])
def test_band_solve_matches_dense(fe2, n, bw):
    A = random_spd_band(n, bw, seed=n + bw)
    b = np.random.default_rng(1).standard_normal(n)
    band = band_of(A, bw)
    st, piv, x, band_after = solve_gpu(fe2, n, bw, band, b)
    assert st == fe2.FE2_OK and piv == 0
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.array_equal(band_after, band.ravel())   # the input is read only


def test_band_solve_grid_laplacian_at_macro_size(fe2):
    """Two unknowns per node of a 65x65 grid, numbered row by row (half
    bandwidth 133): a vector Laplacian with a small shift, checked through
    the residual and against a dense solve."""
    m = 65
    n = 2 * m * m
    bw = 2 * (m + 1) + 1
    rng = np.random.default_rng(5)
    A = np.zeros((n, n))
    for y in range(m):
        for xg in range(m):
            p = y * m + xg
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dx or dy) and 0 <= xg + dx < m and 0 <= y + dy < m:
                        q = (y + dy) * m + xg + dx
                        w = 1.0 if (dx == 0 or dy == 0) else 0.5
                        for c in range(2):
                            A[2 * p + c, 2 * q + c] -= w
                            A[2 * p + c, 2 * p + c] += w
    A += 1e-3 * np.eye(n)
    A[0::2, 1::2] += 0.0
    b = rng.standard_normal(n)
    st, piv, x, _ = solve_gpu(fe2, n, bw, band_of(A, bw), b)
    assert st == fe2.FE2_OK
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.abs(A @ x - b).max() <= 1e-10 * np.abs(b).max() * np.abs(A).max()


def test_band_solve_reports_indefinite(fe2):
    n, bw = 200, 9
    A = random_spd_band(n, bw, seed=3)
    A[150, 150] = -1.0
    b = np.ones(n)
    st, piv, _, _ = solve_gpu(fe2, n, bw, band_of(A, bw), b, allow=True)
    assert st == fe2.FE2_ENOCONV
    assert 1 <= piv <= n


def test_band_solve_rejects_bad_arguments(fe2):
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(fe2.FE2Error):
        fe2.fe2_band_solve(0, 1, x, x)
    with pytest.raises(fe2.FE2Error):
        fe2.fe2_band_solve(4, 2000, x, x)
