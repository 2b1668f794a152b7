"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (laminate, homogeneous cell, uniaxial macro field, patch test, the
isotropic small-strain limit), invariants (Voigt/Reuss bounds, symmetry,
Hill-Mandel, microstructure symmetry), brute force (finite differences of an
independently written discrete energy) and algebraic identities of the
method (full block solve = null-space step = nested scheme).
"""
import numpy as np
import pytest

import workloads as W
from oracle import macro as M
from oracle import rve as R
from oracle import tensors as T

RNG = np.random.default_rng(2312)


# --------------------------------------------------------------------------
# tensor algebra and constitutive laws
# --------------------------------------------------------------------------

def test_cofactor_and_determinant_match_adjugate():
    """Eqs. (1)-(2) against the textbook adjugate: cof F = det(F) F^-T."""
    for _ in range(20):
        F = np.eye(3) + 0.3 * RNG.standard_normal((3, 3))
        H = T.cofactor(F)
        J = T.det(F)
        assert abs(J - np.linalg.det(F)) < 1e-13
        np.testing.assert_allclose(H, np.linalg.det(F) * np.linalg.inv(F).T, atol=1e-13)


@pytest.mark.parametrize("law", ["nh", "mr"])
def test_finite_strain_law_fd_stress_free_and_linear_limit(law):
    """P = dPsi/dF and A = dP/dF by central differences; P(I) = 0; A(I)
    equals the isotropic small-strain tensor lam d_ij d_kl + mu (d_ik d_jl +
    d_il d_jk) with mu = 2(a+b), lam = k + 4b for the Cook family."""
    if law == "nh":
        lam, mu = 2.0, 1.3
        energy = lambda F: T.nh_energy(F, lam, mu)
        st = lambda F: T.nh_stress_tangent(F, lam, mu)
        lam0, mu0 = lam, mu
    else:
        a, b, k = 27.0, 18.0, 60.0
        energy = lambda F: T.mr_energy(F, a, b, k)
        st = lambda F: T.mr_stress_tangent(F, a, b, k)
        lam0, mu0 = k + 4 * b, 2 * (a + b)
    e = 1e-6
    for _ in range(5):
        F = np.eye(2) + 0.2 * RNG.standard_normal((2, 2))
        if np.linalg.det(F) < 0.3:
            continue
        P, A = st(F)
        Fv = F.ravel()
        for c in range(4):
            d = np.zeros(4)
            d[c] = e
            fd = (energy((Fv + d).reshape(2, 2)) - energy((Fv - d).reshape(2, 2))) / (2 * e)
            assert abs(fd - P[c]) < 1e-7 * max(1, abs(P[c]))
            Pp, _ = st((Fv + d).reshape(2, 2))
            Pm, _ = st((Fv - d).reshape(2, 2))
            np.testing.assert_allclose((Pp - Pm) / (2 * e), A[:, c], rtol=1e-6, atol=1e-6)
    P0, A0 = st(np.eye(2))
    assert np.abs(P0).max() < 1e-13
    d = np.eye(2)
    Aiso = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k_ in range(2):
                for l in range(2):
                    Aiso[i, j, k_, l] = lam0 * d[i, j] * d[k_, l] + mu0 * (d[i, k_] * d[j, l] + d[i, l] * d[j, k_])
    np.testing.assert_allclose(A0, Aiso.reshape(4, 4), atol=1e-12)


# --------------------------------------------------------------------------
# RVE level
# --------------------------------------------------------------------------

def laminate_closed_form(lam, mu, frac):
    """Exact effective plane-strain stiffness of a laminate with layers
    normal to X2 (eps11 continuous; sigma22, sigma12 continuous)."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    Mm = lam + 2 * mu
    avg = lambda v: float(np.dot(frac, v))
    iM = avg(1 / Mm)
    C22 = 1 / iM
    C12 = avg(lam / Mm) / iM
    C11 = avg(Mm - lam ** 2 / Mm) + avg(lam / Mm) ** 2 / iM
    C66 = 1 / avg(1 / mu)
    return np.array([[C11, C12, 0], [C12, C22, 0], [0, 0, C66]])


def test_laminate_matches_closed_form_every_rve():
    p = W.config("cfg1")
    lam, mu = W.lame_from_young(np.array([1.0, 10.0]), 0.3)
    Cex = laminate_closed_form(lam, mu, [0.5, 0.5])
    frac = np.array([[500 / 77, 150 / 143, 0], [150 / 143, 350 / 143, 0], [0, 0, 100 / 143]])
    np.testing.assert_allclose(Cex, frac, rtol=1e-14, atol=1e-15)
    for b in range(0, p.n_rve, 7):
        c = R.homogenize_rve(p, b, np.zeros(3))
        assert np.abs(c.C - Cex).max() <= 1e-13 * np.abs(Cex).max()


@pytest.mark.parametrize("n1,n2", [(8, 8), (6, 10)])
def test_laminate_any_grid(n1, n2):
    lam, mu = W.lame_from_young(np.array([2.0, 7.0]), 0.25)
    ph = W.phases_laminate(n1, n2)
    params = np.stack([lam, mu], axis=1)
    c = R.condense(R.assemble_rve((n1, n2), ph, params, "small", "linear", np.zeros(3)))
    frac = np.array([n2 // 2, n2 - n2 // 2]) / n2
    Cex = laminate_closed_form(lam, mu, frac)
    assert np.abs(c.C - Cex).max() <= 1e-12 * np.abs(Cex).max()


def _hooke_voigt_3d(lam, mu):
    """Isotropic stiffness built column by column from Hooke's law in tensor
    form, sigma = lam tr(eps) I + 2 mu eps, with the Voigt strain
    [e11, e22, e33, g23, g13, g12] (engineering shear: eps_ij = g_ij / 2) and
    the stress read back in the same order.  Written without the oracle's
    Voigt matrix."""
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    C = np.zeros((6, 6))
    for c, (i, j) in enumerate(pairs):
        eps = np.zeros((3, 3))
        if i == j:
            eps[i, i] = 1.0
        else:
            eps[i, j] = eps[j, i] = 0.5
        sig = lam * np.trace(eps) * np.eye(3) + 2.0 * mu * eps
        C[:, c] = [sig[a, b] for a, b in pairs]
    return C


def test_voigt_3d_is_hookes_law_in_tensor_form():
    """The oracle's 3D Voigt stiffness against the tensor form of Hooke's law
    (a shear diagonal of 2 mu or a misplaced lambda block fails here)."""
    for lam, mu in [(1.7, 0.9), (0.0, 2.5), (12.0, 0.3)]:
        np.testing.assert_allclose(T.voigt_C(lam, mu, 3), _hooke_voigt_3d(lam, mu), rtol=0, atol=1e-15)
    rng = np.random.default_rng(31)
    for _ in range(5):
        lam, mu = rng.uniform(0.1, 5.0, 2)
        e = rng.standard_normal(6)
        eps = np.array([[e[0], e[5] / 2, e[4] / 2], [e[5] / 2, e[1], e[3] / 2], [e[4] / 2, e[3] / 2, e[2]]])
        sig = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
        s = T.voigt_C(lam, mu, 3) @ e
        np.testing.assert_allclose(s, [sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]],
                                   rtol=1e-14, atol=1e-14)
        # strain energy density eps:sigma/2 equals the Voigt quadratic form
        assert abs(T.linear_energy(e, lam, mu, 3) - 0.5 * np.sum(eps * sig)) < 1e-13 * (1 + abs(np.sum(eps * sig)))


def laminate_closed_form_3d(lam, mu, frac):
    """Exact effective stiffness of an isotropic laminate with layers normal
    to X3 (eps11, eps22, g12 continuous; sigma33, sigma23, sigma13
    continuous), in the Voigt order [11, 22, 33, 23, 13, 12]; written out in
    scalars, with M = lam + 2 mu per layer."""
    lam = np.asarray(lam, dtype=float)
    mu = np.asarray(mu, dtype=float)
    Mm = lam + 2 * mu
    avg = lambda v: float(np.dot(frac, v))
    iM = avg(1 / Mm)
    C33 = 1 / iM
    C13 = avg(lam / Mm) / iM
    C11 = avg(Mm - lam ** 2 / Mm) + avg(lam / Mm) ** 2 / iM
    C12 = avg(lam - lam ** 2 / Mm) + avg(lam / Mm) ** 2 / iM
    C44 = 1 / avg(1 / mu)
    C66 = avg(mu)
    return np.array([[C11, C12, C13, 0, 0, 0],
                     [C12, C11, C13, 0, 0, 0],
                     [C13, C13, C33, 0, 0, 0],
                     [0, 0, 0, C44, 0, 0],
                     [0, 0, 0, 0, C44, 0],
                     [0, 0, 0, 0, 0, C66]])


@pytest.mark.parametrize("res,n_lo", [((2, 2, 4), 2), ((2, 3, 5), 2), ((3, 2, 6), 4)])
def test_laminate_3d_matches_closed_form(res, n_lo):
    """hex8 RVE of two isotropic layers normal to X3 (interfaces on element
    faces, so the piecewise-linear exact fluctuation is in the trilinear
    space): the condensed tangent equals the layered-medium closed form."""
    n1, n2, n3 = res
    k = np.repeat(np.arange(n3), n1 * n2)   # element layer index (x fastest, then y, then z)
    ph = (k >= n_lo).astype(np.uint8)
    lam, mu = W.lame_from_young(np.array([1.0, 10.0]), 0.3)
    params = np.stack([lam, mu], axis=1)
    c = R.condense(R.assemble_rve(res, ph, params, "small", "linear", np.zeros(6)))
    frac = np.array([n_lo, n3 - n_lo]) / n3
    Cex = laminate_closed_form_3d(lam, mu, frac)
    assert np.abs(c.C - Cex).max() <= 1e-12 * np.abs(Cex).max(), (c.C, Cex)


def _voigt_reuss(ph, params, dim):
    Cs = [T.voigt_C(params[i, 0], params[i, 1], dim) for i in range(2)]
    f1 = float(np.mean(ph))
    CV = (1 - f1) * Cs[0] + f1 * Cs[1]
    CR = np.linalg.inv((1 - f1) * np.linalg.inv(Cs[0]) + f1 * np.linalg.inv(Cs[1]))
    return CV, CR


@pytest.mark.parametrize("seed", range(4))
def test_voigt_reuss_bounds_symmetry_pd(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([8, 12, 16]))
    ph = W.phases_circle(n, n, rng.uniform(0.1, 0.45))
    lam, mu = W.lame_from_young(np.array([1.0, rng.uniform(2, 50)]), rng.uniform(0.1, 0.4))
    params = np.stack([lam, mu], axis=1)
    c = R.condense(R.assemble_rve((n, n), ph, params, "small", "linear", np.zeros(3)))
    CV, CR = _voigt_reuss(ph, params, 2)
    s = np.abs(c.C).max()
    assert np.linalg.eigvalsh(CV - 0.5 * (c.C + c.C.T)).min() > -1e-12 * s
    assert np.linalg.eigvalsh(0.5 * (c.C + c.C.T) - CR).min() > -1e-12 * s
    assert np.abs(c.C - c.C.T).max() < 1e-12 * s
    assert np.linalg.eigvalsh(c.C).min() > 0
    # centred circle on an even grid: square symmetry
    assert abs(c.C[0, 0] - c.C[1, 1]) < 1e-12 * s
    assert abs(c.C[0, 2]) < 1e-12 * s and abs(c.C[1, 2]) < 1e-12 * s


def test_homogeneous_rve_recovers_phase_stiffness():
    for dim, res in [(2, (6, 6)), (3, (3, 3, 3))]:
        ph = np.zeros(int(np.prod(res)), dtype=np.uint8)
        params = np.array([[1.7, 0.9], [9.0, 9.0]])
        nF = 3 if dim == 2 else 6
        c = R.condense(R.assemble_rve(res, ph, params, "small", "linear", np.zeros(nF)))
        np.testing.assert_allclose(c.C, T.voigt_C(1.7, 0.9, dim), atol=1e-13)
        assert np.abs(c.X_F).max() < 1e-13


def test_sphere_cubic_symmetry_and_bounds():
    p = W.config("cfg4", macro=(1, 1, 1))
    c = R.homogenize_rve(p, 0, np.zeros(6))
    C = c.C
    s = np.abs(C).max()
    assert abs(C[0, 0] - C[1, 1]) < 1e-12 * s and abs(C[0, 0] - C[2, 2]) < 1e-12 * s
    assert abs(C[0, 1] - C[0, 2]) < 1e-12 * s and abs(C[3, 3] - C[5, 5]) < 1e-12 * s
    off = C.copy()
    off[:3, :3] = 0
    off[3, 3] = off[4, 4] = off[5, 5] = 0
    assert np.abs(off).max() < 1e-12 * s
    CV, CR = _voigt_reuss(p.rve_phases(0).ravel(), p.phase_params[0], 3)
    assert np.linalg.eigvalsh(CV - C).min() > -1e-12 * s
    assert np.linalg.eigvalsh(C - CR).min() > -1e-12 * s


def test_hill_mandel_discrete():
    """Eq. (18): with the equilibrated periodic fluctuation the volume
    average of sigma~:eps~ equals sigma:eps (here: 2 W / |Omega| =
    eps^T C eps and <sigma~> = C eps)."""
    p = W.config("cfg2", macro=(1, 1), rve=16)
    eps = np.array([1e-3, -4e-4, 7e-4])
    c0 = R.homogenize_rve(p, 0, np.zeros(3))
    w = R.expand(c0.system, -c0.X_F @ eps)
    s = R.assemble_rve(*R.rve_problem_args(p, 0)[:3], "small", "linear", eps, w, 1.0)
    sig = s.P_int / s.volume
    assert abs(2 * s.energy / s.volume - eps @ sig) < 1e-13 * abs(eps @ sig)
    np.testing.assert_allclose(sig, c0.C @ eps, rtol=1e-12, atol=1e-17)
    assert np.linalg.norm(s.r) < 1e-12 * np.linalg.norm(c0.system.K_wF @ eps)


# --------------------------------------------------------------------------
# brute force: finite differences of an independently written energy
# --------------------------------------------------------------------------

def _interp_grad_fd(wn, x, y, hx, hy):
    """Gradient of the bilinear interpolant of the nodal values wn
    (corners (0,0), (hx,0), (hx,hy), (0,hy) of an element) by central
    differences (exact for a bilinear field)."""
    def val(xx, yy):
        s, t = xx / hx, yy / hy
        return ((1 - s) * (1 - t) * wn[0] + s * (1 - t) * wn[1]
                + s * t * wn[2] + (1 - s) * t * wn[3])
    dx = 1e-3 * hx
    dy = 1e-3 * hy
    gx = (val(x + dx, y) - val(x - dx, y)) / (2 * dx)
    gy = (val(x, y + dy) - val(x, y - dy)) / (2 * dy)
    return gx, gy


def _brute_energy_2d(res, ph, params, macro, w_full, kin, L=1.0):
    n1, n2 = res
    hx, hy = L / n1, L / n2
    g = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    Wtot = 0.0
    for j in range(n2):
        for i in range(n1):
            nodes = [(i % n1) + n1 * (j % n2), ((i + 1) % n1) + n1 * (j % n2),
                     ((i + 1) % n1) + n1 * ((j + 1) % n2), (i % n1) + n1 * ((j + 1) % n2)]
            wx = np.array([w_full[2 * a] for a in nodes])
            wy = np.array([w_full[2 * a + 1] for a in nodes])
            p = params[ph[j * n1 + i]]
            for yy in g * hy:
                for xx in g * hx:
                    ux_x, ux_y = _interp_grad_fd(wx, xx, yy, hx, hy)
                    uy_x, uy_y = _interp_grad_fd(wy, xx, yy, hx, hy)
                    wq = 0.25 * hx * hy
                    if kin == "small":
                        e = macro + np.array([ux_x, uy_y, ux_y + uy_x])
                        Wtot += wq * float(T.linear_energy(e, p[0], p[1], 2))
                    else:
                        F = macro.reshape(2, 2) + np.array([[ux_x, ux_y], [uy_x, uy_y]])
                        Wtot += wq * float(T.nh_energy(F, p[0], p[1]))
    return Wtot


def test_brute_force_small_strain_blocks():
    """K_ww, K_wF and r against second/first differences of the discrete
    energy evaluated point by point (3x4 periodic grid, random phases)."""
    rng = np.random.default_rng(5)
    res = (3, 4)
    ph = rng.integers(0, 2, size=12).astype(np.uint8)
    params = np.array([[1.0, 0.7], [4.0, 2.5]])
    eps0 = np.array([1e-2, -3e-3, 5e-3])
    w0 = 1e-2 * rng.standard_normal(24)
    w0[:2] = 0
    s = R.assemble_rve(res, ph, params, "small", "linear", eps0, w0, 1.0)
    E = lambda eps, w: _brute_energy_2d(res, ph, params, eps, w, "small")
    free = s.free
    h = 1e-3
    # residual = gradient in w; quadratic energy -> central differences exact
    for k, dof in enumerate(free[::3]):
        d = np.zeros(24)
        d[dof] = h
        g = (E(eps0, w0 + d) - E(eps0, w0 - d)) / (2 * h)
        assert abs(g - s.r[list(free).index(dof)]) < 1e-9
    for a in free[::4]:
        for b in free[::5]:
            da = np.zeros(24)
            db = np.zeros(24)
            da[a] = h
            db[b] = h
            hess = (E(eps0, w0 + da + db) - E(eps0, w0 + da - db)
                    - E(eps0, w0 - da + db) + E(eps0, w0 - da - db)) / (4 * h * h)
            ia, ib = list(free).index(a), list(free).index(b)
            assert abs(hess - s.K_ww[ia, ib]) < 1e-6
    for a in free[::4]:
        for c in range(3):
            da = np.zeros(24)
            da[a] = h
            de = np.zeros(3)
            de[c] = h
            hess = (E(eps0 + de, w0 + da) - E(eps0 - de, w0 + da)
                    - E(eps0 + de, w0 - da) + E(eps0 - de, w0 - da)) / (4 * h * h)
            assert abs(hess - s.K_wF[list(free).index(a), c]) < 1e-6
    np.testing.assert_allclose(s.P_int, [(E(eps0 + np.eye(3)[c] * h, w0) - E(eps0 - np.eye(3)[c] * h, w0)) / (2 * h)
                                         for c in range(3)], rtol=1e-8, atol=1e-12)


def test_brute_force_finite_strain_residual_and_tangent():
    rng = np.random.default_rng(9)
    res = (3, 3)
    ph = rng.integers(0, 2, size=9).astype(np.uint8)
    params = np.array([[2.0, 1.0], [40.0, 20.0]])
    F0 = np.array([1.05, 0.02, -0.03, 0.98])
    w0 = 2e-2 * rng.standard_normal(18)
    w0[:2] = 0
    s = R.assemble_rve(res, ph, params, "finite", "neohooke", F0, w0, 1.0)
    E = lambda F, w: _brute_energy_2d(res, ph, params, F, w, "finite")
    free = list(s.free)
    h = 1e-5
    for dof in free:
        d = np.zeros(18)
        d[dof] = h
        g = (E(F0, w0 + d) - E(F0, w0 - d)) / (2 * h)
        assert abs(g - s.r[free.index(dof)]) < 1e-6
    for c in range(4):
        dF = np.zeros(4)
        dF[c] = h
        g = (E(F0 + dF, w0) - E(F0 - dF, w0)) / (2 * h)
        assert abs(g - s.P_int[c]) < 1e-6
    # tangent = derivative of the oracle residual (independent FD of r)
    for dof in free[::3]:
        d = np.zeros(18)
        d[dof] = 1e-6
        sp_ = R.assemble_rve(res, ph, params, "finite", "neohooke", F0, w0 + d, 1.0)
        sm_ = R.assemble_rve(res, ph, params, "finite", "neohooke", F0, w0 - d, 1.0)
        col = (sp_.r - sm_.r) / 2e-6
        np.testing.assert_allclose(col, s.K_ww[:, free.index(dof)].toarray().ravel(), atol=1e-6)


def test_brute_force_hex8_stiffness():
    """3D: K_ww entries against second differences of an energy built from a
    finite-difference gradient of the trilinear interpolant."""
    rng = np.random.default_rng(3)
    res = (2, 2, 3)
    ne = 12
    ph = rng.integers(0, 2, size=ne).astype(np.uint8)
    params = np.array([[1.0, 0.6], [3.0, 1.1]])
    L = 1.0
    hE = np.array([L / r for r in res])
    s = R.assemble_rve(res, ph, params, "small", "linear", np.zeros(6), None, L)
    g = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    en = R.element_nodes(res)
    corners = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                        [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])

    def energy(w):
        tot = 0.0
        for e in range(ne):
            wn = w.reshape(-1, 3)[en[e]]
            p = params[ph[e]]

            def val(x):
                s_ = x / hE
                wts = np.prod(np.where(corners == 1, s_, 1 - s_), axis=1)
                return wts @ wn
            for z in g * hE[2]:
                for y in g * hE[1]:
                    for x in g * hE[0]:
                        pt = np.array([x, y, z])
                        grad = np.zeros((3, 3))
                        for J in range(3):
                            d = np.zeros(3)
                            d[J] = 1e-3 * hE[J]
                            grad[:, J] = (val(pt + d) - val(pt - d)) / (2e-3 * hE[J])
                        e6 = np.array([grad[0, 0], grad[1, 1], grad[2, 2], grad[1, 2] + grad[2, 1],
                                       grad[0, 2] + grad[2, 0], grad[0, 1] + grad[1, 0]])
                        tot += np.prod(hE / 2) * float(T.linear_energy(e6, p[0], p[1], 3))
        return tot
    free = list(s.free)
    n = 36
    hh = 1e-3
    for a in free[::7]:
        for b in free[::11]:
            da = np.zeros(n)
            db = np.zeros(n)
            da[a] = hh
            db[b] = hh
            hess = (energy(da + db) - energy(da - db) - energy(-da + db) + energy(-da - db)) / (4 * hh * hh)
            assert abs(hess - s.K_ww[free.index(a), free.index(b)]) < 1e-6


# --------------------------------------------------------------------------
# macro level
# --------------------------------------------------------------------------

def test_cfg1_macro_uniaxial_closed_form():
    """Homogeneous orthotropic C: the exact macro field is linear,
    u_x = d X, u_y = -(C12/C22) d Y with C12/C22 = 3/7 for the laminate;
    sigma11 = (C11 - C12^2/C22) d = 550/91 * 1e-3."""
    p = W.config("cfg1")
    st, hist = M.solve(p)
    assert len(hist[0]) == 2
    np.testing.assert_allclose(st.u[0::2], 1e-3 * p.X[:, 0], atol=1e-17)
    np.testing.assert_allclose(st.u[1::2], -3.0 / 7.0 * 1e-3 * p.X[:, 1], atol=1e-17)
    geo = M.macro_geometry(p)
    c = M.linearize(p, geo, st)
    for b in range(0, p.n_rve, 5):
        assert abs(c[b].P_bar[0] - 550 / 91 * 1e-3) < 1e-15
        assert abs(c[b].P_bar[1]) < 1e-16 and abs(c[b].P_bar[2]) < 1e-16


def test_macro_patch_test_distorted_mesh():
    """Distorted 3x3 Q4 mesh, identical RVEs, u = eps0 X on the whole
    boundary: interior nodes exact and P_bar = C eps0 at every point."""
    p = W.config("cfg1", macro=(3, 3))
    X = p.X.copy()
    interior = np.where((X[:, 0] > 1e-9) & (X[:, 0] < 1 - 1e-9) & (X[:, 1] > 1e-9) & (X[:, 1] < 1 - 1e-9))[0]
    X[interior] += 0.08 * RNG.uniform(-1, 1, size=(len(interior), 2))
    eps0 = np.array([2e-3, -1e-3, 1.5e-3])
    Gd = np.array([[eps0[0], 0.5 * eps0[2]], [0.5 * eps0[2], eps0[1]]])
    bnd = np.setdiff1d(np.arange(X.shape[0]), interior)
    dofs = np.sort(np.concatenate([2 * bnd, 2 * bnd + 1])).astype(np.int32)
    uex = (X @ Gd.T).ravel()
    import dataclasses
    q = dataclasses.replace(p, X=X, dir_dofs=dofs, dir_vals=uex[dofs])
    st, _ = M.solve(q)
    np.testing.assert_allclose(st.u, uex, atol=1e-15)
    lam, mu = W.lame_from_young(np.array([1.0, 10.0]), 0.3)
    Cex = laminate_closed_form(lam, mu, [0.5, 0.5])
    c = M.linearize(q, M.macro_geometry(q), st)
    for b in range(q.n_rve):
        np.testing.assert_allclose(c[b].P_bar, Cex @ eps0, atol=1e-15)


def test_full_block_equals_null_space_step_linear_and_nonlinear():
    """Eq. (42) solved directly == Eqs. (46)-(49) per RVE."""
    for name, kw in [("cfg2", dict(macro=(2, 1), rve=6)), ("cfg5", dict(macro=(2, 1), rve=6))]:
        p = W.config(name, **kw)
        geo = M.macro_geometry(p)
        st = M.initial_state(p)
        if name == "cfg5":   # move away from the reference state first
            M.generalized_step(p, geo, st, 0.3)
        import copy
        st_fb = copy.deepcopy(st)
        du_fb, dw_fb = M.full_block_step(p, st_fb, 0.5)
        _, du, dws, _ = M.generalized_step(p, geo, st, 0.5)
        assert np.abs(du - du_fb).max() <= 1e-11 * np.abs(du).max()
        for a, b in zip(dws, dw_fb):
            assert np.abs(a - b).max() <= 1e-11 * max(1e-30, np.abs(du).max())


def test_linear_monolithic_equals_nested_in_one_step():
    p = W.config("cfg2", macro=(2, 2), rve=8)
    st1, h1 = M.solve(p, "generalized")
    st2, h2 = M.solve(p, "classical")
    assert len(h1[0]) == 2 and len(h2[0]) == 2
    assert np.abs(st1.u - st2.u).max() <= 1e-13 * np.abs(st1.u).max()
    for a, b in zip(st1.w, st2.w):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(st1.u).max()


@pytest.mark.slow
def test_nonlinear_monolithic_equals_nested_and_converges_quadratically():
    p = W.config("cfg5", macro=(2, 2), rve=8, n_steps=2)
    st1, h1 = M.solve(p, "generalized", tol=1e-12)
    st2, h2 = M.solve(p, "classical", tol=1e-12)
    assert np.abs(st1.u - st2.u).max() <= 1e-10 * np.abs(st1.u).max()
    for a, b in zip(st1.w, st2.w):
        assert np.abs(a - b).max() <= 1e-10 * np.abs(st1.u).max()
    for h in h1:   # quadratic rate of the generalized scheme
        r = [n.total / n.scale for n in h[1:]]
        for a, b in zip(r[:-1], r[1:]):
            if b > 1e-13:
                assert b <= 50.0 * a * a


@pytest.mark.slow
def test_homogenized_tangent_is_derivative_of_averaged_stress():
    """Finite strain: at equilibrium C = dP_bar/dF_bar (central differences
    of the equilibrated stress), and at F = I it equals the small-strain
    homogenized tensor of the same phases."""
    p = W.config("cfg5", macro=(1, 1), rve=8)
    F0 = np.array([1.04, 0.01, -0.02, 0.99])
    w, _ = R.equilibrate_rve(p, 0, F0, tol=1e-14)
    c = R.homogenize_rve(p, 0, F0, w)
    h = 1e-6
    for k in range(4):
        d = np.zeros(4)
        d[k] = h
        wp, _ = R.equilibrate_rve(p, 0, F0 + d, w, tol=1e-14)
        wm, _ = R.equilibrate_rve(p, 0, F0 - d, w, tol=1e-14)
        Pp = R.homogenize_rve(p, 0, F0 + d, wp).P_bar
        Pm = R.homogenize_rve(p, 0, F0 - d, wm).P_bar
        np.testing.assert_allclose((Pp - Pm) / (2 * h), c.C[:, k], rtol=2e-6, atol=2e-6)
    cI = R.homogenize_rve(p, 0, np.eye(2).ravel())
    res, ph, par, L = R.rve_problem_args(p, 0)
    cl = R.condense(R.assemble_rve(res, ph, par, "small", "linear", np.zeros(3), None, L))
    # small-strain Voigt C (11, 22, 12 eng.) -> 4th-order tensor in row-major F
    V = {(0, 0): 0, (1, 1): 1, (0, 1): 2, (1, 0): 2}
    A = np.zeros((4, 4))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    A[2 * i + j, 2 * k + l] = cl.C[V[(i, j)], V[(k, l)]]
    np.testing.assert_allclose(cI.C, A, atol=1e-12 * np.abs(A).max())
