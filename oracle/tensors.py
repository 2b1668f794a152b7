"""Tensor algebra and constitutive laws (FP64), oracle side.

* Tensor cross product, cofactor and determinant follow Sec. 2.1, Eqs. (1)
  and (2): [A x B]_iJ = eps_ijk eps_JMN A_jM B_kN, H = (F x F)/2,
  J = F:(F x F)/6.
* The polyconvex stress P = dPsi/dF + dPsi/dH x F + dPsi/dJ H of Eq. (8).
* Two-dimensional problems are plane strain: a 2x2 gradient is embedded in 3D
  as diag(F, 1).
* The Cook law, Eq. (59): Psi = a (F:F - 2) + b (F:F + J^2 - 3)
  + k/2 (J - 1)^2 - 2 (a + 2 b) ln J, written with the 2D F:F.  Its 3D reading
  (F:F_3D = F:F + 1, H:H_3D = F:F + J^2) is the Mooney-Rivlin form of Eq. (7),
  a F:F + b H:H + f(J).
* The compressible Neo-Hookean law is this family with b = 0, a = mu/2,
  k = lambda: Psi = mu/2 (F:F - 2) - mu ln J + lambda/2 (J - 1)^2.
* Small strain: linear isotropic elasticity, Voigt order [11, 22, 12] in 2D
  (plane strain) and [11, 22, 33, 23, 13, 12] in 3D, engineering shear.

Finite-strain quantities use the row-major 2D component order
[F11, F12, F21, F22].
"""
from __future__ import annotations

import numpy as np

# Levi-Civita symbol
EPS = np.zeros((3, 3, 3))
EPS[0, 1, 2] = EPS[1, 2, 0] = EPS[2, 0, 1] = 1.0
EPS[0, 2, 1] = EPS[2, 1, 0] = EPS[1, 0, 2] = -1.0


def cross(A, B):
    """Tensor cross product of Eq. (1), batched over leading axes."""
    return np.einsum("ijk,JMN,...jM,...kN->...iJ", EPS, EPS, A, B)


def cofactor(F):
    """H = (F x F) / 2, Eq. (1)."""
    return 0.5 * cross(F, F)


def det(F):
    """J = F : (F x F) / 6, Eq. (2)."""
    return np.einsum("...iJ,...iJ->...", F, cross(F, F)) / 6.0


def embed2(F2):
    """Plane-strain embedding of a (..., 2, 2) gradient into (..., 3, 3)."""
    F = np.zeros(F2.shape[:-2] + (3, 3))
    F[..., :2, :2] = F2
    F[..., 2, 2] = 1.0
    return F


# --------------------------------------------------------------------------
# Mooney-Rivlin family (Eq. (59)), plane strain, 2D gradient
# --------------------------------------------------------------------------

def mr_energy(F2, a, b, k):
    """Strain energy of Eq. (59) for a (..., 2, 2) gradient."""
    F = embed2(F2)
    J = det(F)
    FF = np.einsum("...iJ,...iJ->...", F2, F2)
    return a * (FF - 2.0) + b * (FF + J * J - 3.0) + 0.5 * k * (J - 1.0) ** 2 \
        - 2.0 * (a + 2.0 * b) * np.log(J)


def _dH_dF_2d(F2):
    """Linear map dF -> dH = F x dF (3D cross product with plane-strain
    embedding, dF33 = 0), returned as a (..., 4, 4) matrix acting on the
    row-major components of the 2D blocks."""
    F = embed2(F2)
    out = np.zeros(F2.shape[:-2] + (4, 4))
    for c in range(4):
        dF = np.zeros(F2.shape[:-2] + (3, 3))
        dF[..., c // 2, c % 2] = 1.0
        dH = cross(F, dF)
        out[..., :, c] = dH[..., :2, :2].reshape(F2.shape[:-2] + (4,))
    return out


def mr_stress_tangent(F2, a, b, k):
    """First Piola-Kirchhoff stress (Eq. (8)) and tangent dP/dF of the Cook
    law for (..., 2, 2) gradients; returns P (..., 4) and A (..., 4, 4).

    With Psi = a F:F_3D + b H:H_3D + f(J) (plus constants) the three partial
    derivatives of Eq. (8) are 2 a F, 2 b H and f'(J); in 2D plane strain
    H:H_3D = F:F + J^2 (the 33 entry of H is J), so dPsi/dF collects
    2 (a + b) F and the J^2 part joins f'(J):
    P = 2 (a + b) F + (2 b J + k (J - 1) - 2 (a + 2 b) / J) H.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    F = embed2(F2)
    H3 = cofactor(F)
    J = det(F)
    H = H3[..., :2, :2].reshape(F2.shape[:-2] + (4,))
    Fv = F2.reshape(F2.shape[:-2] + (4,))
    c0 = 2.0 * (a + b)
    c1 = 2.0 * b * J + k * (J - 1.0) - 2.0 * (a + 2.0 * b) / J
    dc1 = 2.0 * b + k + 2.0 * (a + 2.0 * b) / (J * J)
    P = np.asarray(c0)[..., None] * Fv + c1[..., None] * H
    dH = _dH_dF_2d(F2)
    eye = np.eye(4)
    A = (np.asarray(c0)[..., None, None] * eye + c1[..., None, None] * dH
         + dc1[..., None, None] * np.einsum("...i,...j->...ij", H, H))
    return P, A


def nh_params(lam, mu):
    """Neo-Hookean law as a member of the Cook family: (a, b, k)."""
    return 0.5 * np.asarray(mu), np.zeros_like(np.asarray(mu, dtype=float)), np.asarray(lam)


def nh_energy(F2, lam, mu):
    a, b, k = nh_params(lam, mu)
    return mr_energy(F2, a, b, k)


def nh_stress_tangent(F2, lam, mu):
    a, b, k = nh_params(lam, mu)
    return mr_stress_tangent(F2, a, b, k)


# --------------------------------------------------------------------------
# linear isotropic elasticity (Voigt, engineering shear)
# --------------------------------------------------------------------------

def voigt_C(lam, mu, dim):
    """Isotropic stiffness in Voigt form; 2D is plane strain."""
    if dim == 2:
        return np.array([[lam + 2 * mu, lam, 0.0],
                         [lam, lam + 2 * mu, 0.0],
                         [0.0, 0.0, mu]])
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def linear_energy(eps_voigt, lam, mu, dim):
    C = voigt_C(lam, mu, dim)
    return 0.5 * np.einsum("...i,ij,...j->...", eps_voigt, C, eps_voigt)
