"""fe2_band_solve_noalloc (the FP64 band solve of the macro Newton update with
its workspace in the library's static device scratch) through the C ABI,
against fe2_band_solve on the same systems.

Both entry points run the same kernels on the same block plan, so the
solutions must agree bit for bit.  Two calls in a row, the second on a smaller
system, show that the scratch left by the first call does not leak into the
second; the macro-mesh-sized case shows the 64 MiB limit admits the 64 x 64
Q4 macro tangent; a system beyond the limit is refused on the host.
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


def random_spd_band(n, bw, seed):
    """Lower band storage [n][bw + 1] of a symmetric, diagonally dominant
    matrix with scaled rows and columns."""
    rng = np.random.default_rng(seed)
    band = np.zeros((n, bw + 1))
    for d in range(1, bw + 1):
        band[: n - d, d] = rng.uniform(-1.0, 1.0, n - d)
    rowsum = np.zeros(n)
    for d in range(1, bw + 1):
        rowsum[: n - d] += np.abs(band[: n - d, d])
        rowsum[d:] += np.abs(band[: n - d, d])
    band[:, 0] = rowsum + rng.uniform(0.5, 2.0, n)
    s = np.exp(rng.uniform(-2.0, 2.0, n))
    for d in range(bw + 1):
        band[: n - d, d] *= s[: n - d] * s[d:]
    return band


def dense_of(band):
    n, w = band.shape
    A = np.diag(band[:, 0]).copy()
    for d in range(1, w):
        A += np.diag(band[: n - d, d], -d) + np.diag(band[: n - d, d], d)
    return A


def both(fe2, n, bw, band, b):
    bd = torch.tensor(band.ravel(), dtype=torch.float64, device="cuda")
    x_ref = torch.tensor(b, dtype=torch.float64, device="cuda")
    x_na = x_ref.clone()
    st_ref, piv_ref = fe2.fe2_band_solve(n, bw, bd, x_ref)
    st_na, piv_na = fe2.fe2_band_solve_noalloc(n, bw, bd, x_na)
    assert st_ref == st_na == fe2.FE2_OK and piv_ref == piv_na == 0
    return x_ref.cpu().numpy(), x_na.cpu().numpy()


def test_noalloc_matches_allocating_entry_on_two_calls(fe2):
    # first a large system (fills much of the scratch), then a smaller one
    for n, bw, seed in [(3000, 61, 11), (517, 19, 12)]:
        print(f"band solve noalloc n={n} bw={bw} seed={seed}", flush=True)
        band = random_spd_band(n, bw, seed)
        b = np.random.default_rng(seed + 100).standard_normal(n)
        x_ref, x_na = both(fe2, n, bw, band, b)
        assert np.array_equal(x_na, x_ref)
        ref = np.linalg.solve(dense_of(band), b)
        assert np.abs(x_na - ref).max() <= 1e-11 * np.abs(ref).max()


def test_noalloc_at_macro_mesh_size(fe2):
    # 8450 unknowns, half bandwidth 133: the 64 x 64 Q4 macro tangent's shape
    n, bw = 8450, 133
    print(f"band solve noalloc n={n} bw={bw}", flush=True)
    band = random_spd_band(n, bw, 21)
    b = np.random.default_rng(22).standard_normal(n)
    x_ref, x_na = both(fe2, n, bw, band, b)
    assert np.array_equal(x_na, x_ref)
    # residual through the band (no dense n x n matrix)
    r = band[:, 0] * x_na
    for d in range(1, bw + 1):
        r[d:] += band[: n - d, d] * x_na[: n - d]
        r[: n - d] += band[: n - d, d] * x_na[d:]
    assert np.abs(r - b).max() <= 1e-12 * np.abs(band).max() * np.abs(x_na).max() * (2 * bw + 1)


def test_noalloc_reports_indefinite_like_the_allocating_entry(fe2):
    n, bw = 200, 9
    band = random_spd_band(n, bw, 3)
    band[150, 0] = -1.0
    bd = torch.tensor(band.ravel(), dtype=torch.float64, device="cuda")
    x1 = torch.ones(n, dtype=torch.float64, device="cuda")
    x2 = x1.clone()
    st1, piv1 = fe2.fe2_band_solve(n, bw, bd, x1, allow_notspd=True)
    st2, piv2 = fe2.fe2_band_solve_noalloc(n, bw, bd, x2, allow_notspd=True)
    assert st1 == st2 == fe2.FE2_ENOCONV
    assert piv1 == piv2 and 1 <= piv2 <= n


def test_noalloc_refuses_systems_beyond_the_scratch(fe2):
    # 33282 unknowns at half bandwidth 261 (a 128 x 128 Q4 macro mesh) need
    # about 360 MB of workspace: refused before any device work
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(fe2.FE2Error, match="static scratch"):
        fe2.fe2_band_solve_noalloc(33282, 261, x, x)
    with pytest.raises(fe2.FE2Error):
        fe2.fe2_band_solve_noalloc(0, 1, x, x)
