"""Pins of the oracle's stiffness layouts (Sec. 3, eq. hooke; Sec. 3.3.1).

* Isotropic material in Voigt form, c11 = c22 = lambda + 2 mu, c12 = lambda,
  c66 = mu, c16 = c26 = 0, is the isotropic tensor of Sec. 3.3.1,
  lambda d_IJ d_KL + mu (d_IK d_JL + d_IL d_JK).
* Voigt notation is defined by Hooke's law on the vectors
  (sigma_11, sigma_22, sigma_12) = V (eps_11, eps_22, 2 eps_12) for a
  symmetric strain (engineering shear strain; stiffness carries no factor 2).
  Stress and strain energy from the full tensor must equal those from the
  6-entry matrix for every entry, c16 and c26 included.
* The compact major-symmetric layout round-trips and fills both halves.
"""
import numpy as np

from oracle import material as M
from paper_2003_12811_amd import workloads as W


def test_isotropic_voigt_is_the_isotropic_tensor():
    lam, mu = 1.7, 0.45
    V = np.array([lam + 2 * mu, lam, 0.0, lam + 2 * mu, 0.0, mu])
    C = M.full_from_voigt(V)
    d = np.eye(2)
    for I in range(2):
        for J in range(2):
            for K in range(2):
                for L in range(2):
                    ref = lam * d[I, J] * d[K, L] + mu * (d[I, K] * d[J, L] + d[I, L] * d[J, K])
                    assert abs(C[I, J, K, L] - ref) < 1e-15
    assert np.allclose(C, M.isotropic(lam, mu), rtol=0, atol=1e-15)


def test_voigt_is_hookes_law_with_engineering_shear():
    rng = np.random.default_rng(7)
    for _ in range(20):
        c11, c12, c16, c22, c26, c66 = rng.uniform(-1, 1, 6)
        V = np.array([c11, c12, c16, c22, c26, c66])
        Vm = np.array([[c11, c12, c16], [c12, c22, c26], [c16, c26, c66]])
        C = M.full_from_voigt(V)
        e = rng.normal(size=(2, 2))
        eps = 0.5 * (e + e.T)
        sig = np.zeros((2, 2))
        for I in range(2):
            for J in range(2):
                for K in range(2):
                    for L in range(2):
                        sig[I, J] += C[I, J, K, L] * eps[K, L]
        ev = np.array([eps[0, 0], eps[1, 1], 2 * eps[0, 1]])
        sv = Vm @ ev
        assert np.allclose([sig[0, 0], sig[1, 1], sig[0, 1]], sv, rtol=0, atol=1e-14)
        assert abs(sig[0, 1] - sig[1, 0]) < 1e-15               # minor symmetry
        energy = np.einsum('IJ,IJKL,KL->', eps, C, eps)
        assert abs(energy - ev @ Vm @ ev) < 1e-13


def test_c10_layout_round_trip_and_workload_helper():
    rng = np.random.default_rng(3)
    C10 = rng.normal(size=(10, 4))
    C = M.full_from_c10(C10)
    assert np.array_equal(M.c10_from_full(C), C10)
    # major symmetry C_IJKL = C_KLIJ holds, minor symmetry is not imposed
    assert np.array_equal(C, np.transpose(C, (2, 3, 0, 1, 4)))
    assert not np.allclose(C, np.transpose(C, (1, 0, 2, 3, 4)))
    # the workloads' Voigt helper gives the same tensor as the oracle's
    V = rng.normal(size=(6, 5))
    assert np.allclose(M.full_from_c10(W.voigt_to_c10(V)), M.full_from_voigt(V), rtol=0, atol=0)
