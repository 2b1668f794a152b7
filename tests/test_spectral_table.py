"""The RVE solver's spectral preconditioner table (fe2_spectral_table, host
code, no GPU) against the oracle's periodic stiffness.

For a homogeneous RVE (mu = 1, lambda = rho) the oracle's assembled K_ww has
a translation-invariant stencil; its Fourier transform is the real symmetric
2x2 symbol S(k).  The table stores, at every position of the transformed
field, alpha = (a + c)/2 and beta = (a - c)/2 + i b of S^-1 = [a b; b c] at
the frequency held there (bit-reversed along each axis; for n = 48 position
p holds 3 rev(p mod 16) + p / 16), zero at k = 0, then the twiddles.  The
test decodes every entry and compares it with the inverse of the symbol
summed from the oracle's stencil, so a wrong element matrix, a wrong
frequency map or a wrong packing fails it.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import rve as R

LIB = os.path.join(os.path.dirname(__file__), "..", "paper_2312_12771_amd", "libfe2.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfe2.so not built")


def oracle_symbol(n, rho):
    """S[ky][kx] (2x2) from the column of K_ww at an interior node."""
    s = R.assemble_rve((n, n), np.zeros(n * n, np.uint8), np.array([[rho, 1.0], [rho, 1.0]]), "small", "linear",
                       np.zeros(3))
    K = s.K_ww.tocsc()
    red = {int(f): r for r, f in enumerate(s.free)}
    mx = my = n // 2
    m = my * n + mx
    k = 2.0 * np.pi * np.arange(n) / n
    S = np.zeros((n, n, 2, 2))
    for e in range(2):
        col = K[:, red[2 * m + e]].toarray().ravel()
        for r in np.nonzero(col)[0]:
            f = int(s.free[r])
            node, c = divmod(f, 2)
            dx, dy = node % n - mx, node // n - my
            S[:, :, c, e] += col[r] * np.cos(k[None, :] * dx + k[:, None] * dy)
    return S


def freq_of(n):
    if n == 48:
        rev = [int(format(x, "04b")[::-1], 2) for x in range(16)]
        return [3 * rev[p % 16] + p // 16 for p in range(n)]
    m = n.bit_length() - 1
    return [int(format(p, f"0{m}b")[::-1], 2) for p in range(n)]


@pytest.mark.parametrize("n", [8, 16, 32, 48])
@pytest.mark.parametrize("rho", [1.5, 4.0])
def test_table_inverts_the_oracle_symbol(n, rho):
    from paper_2312_12771_amd import fe2
    t = fe2.fe2_spectral_table(n, rho)
    nt = 32 if n == 48 else n // 2
    assert t.size == 4 * n * n + 2 * nt
    S = oracle_symbol(n, rho)
    fr = freq_of(n)
    assert sorted(fr) == list(range(n))
    tab = t[:4 * n * n].reshape(n, n, 4)
    worst = 0.0
    for q in range(n):
        for p in range(n):
            kx, ky = fr[p], fr[q]
            al, br, bi, z = tab[q, p]
            assert z == 0.0
            if kx == 0 and ky == 0:
                assert al == br == bi == 0.0
                continue
            Sinv = np.array([[al + br, bi], [bi, al - br]])
            ref = np.linalg.inv(S[ky, kx])
            worst = max(worst, np.abs(Sinv - ref).max() / np.abs(ref).max())
    assert worst < 1e-11, worst
    tw = t[4 * n * n:].reshape(-1, 2)
    ang = 2.0 * np.pi * np.arange(nt) / n
    np.testing.assert_allclose(tw[:, 0], np.cos(ang), atol=1e-15)
    np.testing.assert_allclose(tw[:, 1], -np.sin(ang), atol=1e-15)


def test_table_rejects_other_sizes():
    from paper_2312_12771_amd import fe2
    out = ctypes.c_int()
    assert fe2._lib.fe2_spectral_table(30, 2.0, None, ctypes.byref(out)) == fe2.FE2_ENOTSUP
    assert fe2._lib.fe2_spectral_table(32, 0.0, None, ctypes.byref(out)) == fe2.FE2_EINVAL
