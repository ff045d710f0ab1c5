"""Pins of the FFTLog oracle (oracle/fftlog.py), independent of its own code, for the
synthetic model P(k) = exp(-beta k^2), F(chi) = q_A q_B q_C D_+^4 = chi^p exp(-chi / lam):

* the k integrals have elementary closed forms (Gaussian-Bessel integrals):
      int k e^{-b k^2} J_0(x k) dk   = e^{-x^2/4b} / (2b)
      int k^2 e^{-b k^2} J_1(x k) dk = x e^{-x^2/4b} / (4 b^2)
      int e^{-b k^2} J_1(x k) dk     = (1 - e^{-x^2/4b}) / x
      int k e^{-b k^2} J_2(x k) dk   = 2 (1 - e^{-x^2/4b}) / x^2 - e^{-x^2/4b} / (2b)
  (the last from J_2(z) = (2/z) J_1(z) - J_0(z)); the expansion of eqs. pklfft/cm with the
  term-by-term Gamma-ratio integral must reproduce them within the FFTLog discretisation
  error on 0.03 <= x <= 3 (max-normalised 1e-4, observed ~1e-5 or better);
* A_{s1 s2} = int_0^inf chi^{p - a1 - a2 - 2} e^{-chi/lam} dchi = lam^{p-a1-a2-1} Gamma(p-a1-a2-1);
* the whole chain: I^{(n1,mt1)}_{(n2,mt2)}(th1, th2) = int dchi F chi^{mt1+mt2} H1(th1 chi) H2(th2 chi)
  with the closed-form H, by an independent dense quadrature;
* I is real for real P; A_0 and A_2 are symmetric in (theta1, theta2).
"""

import numpy as np
import pytest
from scipy.special import loggamma

from oracle import fftlog as F

BETA, KMIN, KMAX, N = 1.0, 1e-6, 30.0, 512
P_EXP, LAM = 3.0, 1.0


def closed_hankel(n, mt, x):
    e = np.exp(-x * x / (4 * BETA))
    f = {(0, 0): e / (2 * BETA), (1, 1): x / (4 * BETA ** 2) * e, (1, -1): (1 - e) / x,
         (2, 0): 2 * (1 - e) / x ** 2 - e / (2 * BETA)}[(n, mt)]
    return f / (2 * np.pi)


def _P():
    k = F.k_grid(KMIN, KMAX, N)
    return np.exp(-BETA * k * k)


@pytest.mark.parametrize("n,mt,nu", [(0, 0, -1.3), (1, 1, -2.5), (1, -1, -1.3), (2, 0, -1.3)])
def test_hankel_factor_closed_forms(n, mt, nu):
    c, eta = F.coefficients(_P(), KMIN, KMAX, nu)
    x = np.logspace(np.log10(0.03), np.log10(3.0), 25)
    H = F.hankel_factor(c, eta, nu, n, mt, x).sum(axis=1)
    ref = closed_hankel(n, mt, x)
    assert np.abs(H.imag).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(H.real - ref).max() < 1e-4 * np.abs(ref).max()


def test_a_matrix_closed_form():
    chi = np.logspace(-5, np.log10(60.0), 4000)
    Fchi = chi ** P_EXP * np.exp(-chi / LAM)
    _, eta = F.coefficients(_P(), KMIN, KMAX, -1.3)
    a1 = 1.0 - 1.3 + 1j * eta[::37]
    _, eta2 = F.coefficients(_P(), KMIN, KMAX, -2.5)
    a2 = 1.0 - 2.5 + 1j * eta2[::41]
    A = F.a_matrix(chi, Fchi, a1, a2)
    z = P_EXP - a1[:, None] - a2[None, :] - 1.0
    ref = np.exp(z * np.log(LAM) + loggamma(z))
    assert np.abs(A - ref).max() < 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("n1,mt1,nu1,n2,mt2,nu2", [(0, 0, -1.3, 0, 0, -1.3), (1, 1, -2.5, 1, -1, -1.3),
                                                 (2, 0, -1.3, 2, 0, -1.3)])
def test_i_matrix_against_closed_form_quadrature(n1, mt1, nu1, n2, mt2, nu2):
    th = np.array([0.02, 0.05, 0.11, 0.2])
    chi = np.logspace(-1.5, np.log10(15.0), 1024)   # theta chi within the accurate x range
    Fchi = chi ** P_EXP * np.exp(-chi / LAM)
    I = F.i_matrix(_P(), KMIN, KMAX, chi, Fchi, th, th, n1, mt1, nu1, n2, mt2, nu2)
    # independent: dense trapezoid in ln chi of the closed-form factors over the same range
    cq = np.logspace(-1.5, np.log10(15.0), 200001)
    w = np.gradient(np.log(cq)) * cq
    Fq = cq ** P_EXP * np.exp(-cq / LAM) * cq ** (mt1 + mt2)
    ref = np.array([[np.sum(w * Fq * closed_hankel(n1, mt1, t1 * cq) * closed_hankel(n2, mt2, t2 * cq))
                     for t2 in th] for t1 in th])
    assert np.abs(I.imag).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(I.real - ref).max() < 1e-4 * np.abs(ref).max()


def test_a_functions_real_and_symmetric():
    th = np.logspace(-2, -0.7, 12)
    chi = np.logspace(-1.5, np.log10(15.0), 512)
    Fchi = chi ** P_EXP * np.exp(-chi / LAM)
    A = F.a_functions(_P(), KMIN, KMAX, chi, Fchi, th)
    scale = np.abs(A.real).max(axis=(1, 2))
    assert np.all(np.abs(A.imag).max(axis=(1, 2)) < 1e-10 * scale)
    for f in (0, 1, 2):
        assert np.abs(A[f] - A[f].T).max() < 1e-12 * scale[f]
