"""FFTLog evaluation of the line-of-sight integrals of the modelling appendix ("FFTLog for the
line-of-sight integral") -- test infrastructure only (see oracle/__init__.py).

Steps, in the appendix's order and notation, written out in NumPy/SciPy:

1. eq. pklfft / pklfft_eta / cm: N samples P(k_l) on k_l = k_min (k_max/k_min)^{l/(N-1)}
   (N log-spaced wave-numbers including both ends) give
       c_m = W_m k_min^{-nu - i eta_m} (1/N) sum_l P(k_l) (k_l/k_min)^{-nu} exp(-2 pi i m l / N),
       eta_m = ((N-1)/N) 2 pi m / ln(k_max/k_min),  m = -N/2 .. N/2,  W_{+-N/2} = 1/2, else 1,
   so that P(k) ~ sum_m c_m k^{nu + i eta_m};
2. the k integral of one factor, term by term with the closed form the appendix gives,
       int dk/(2 pi) k^{mu} J_n(x k) = 2^{mu-1} x^{-mu-1} Gamma((n+mu+1)/2) / (pi Gamma((n-mu+1)/2)),
   mu = mt + a_s, a_s = 1 + nu + i eta_s (mt the power of l, i.e. of k, in the integrand):
       g_{n,mt}(a_s) = 2^{mt+a_s-1} Gamma((1+mt+a_s+n)/2) / (pi Gamma((1-a_s-mt+n)/2));
3. A_{s1 s2} = int dchi F(chi) chi^{-a_{s1} - a_{s2} - 2}, F = q_A q_B q_C D_+^4, by the
   trapezoid rule in ln chi on a log-spaced chi grid;
4. I^{(n1,mt1)}_{(n2,mt2)}(theta1, theta2) = sum_{s1,s2} c_{s1} c_{s2} A_{s1 s2}
       g_{n1,mt1}(a_{s1}) g_{n2,mt2}(a_{s2}) theta1^{-(1 + a_{s1} + mt1)} theta2^{-(1 + a_{s2} + mt2)},
   with separate biases nu1, nu2 (hence separate c and a) for the two factors;
5. A_0 = I^{(0,0)}_{(0,0)},  A_1 = I^{(1,1)}_{(1,-1)}(th1, th2) + I^{(1,1)}_{(1,-1)}(th2, th1),
   A_2 = I^{(2,0)}_{(2,0)}.

Readings: the appendix's bias "nu_{b_m}" is the nu of step 1 for the factor with power mt;
a_s = 1 + nu + i eta_s (the k^{mt+1} of the integrand supplies the 1).  The result is real
for real P (the s and -s terms are conjugate); the imaginary part is returned for checking.
"""

from __future__ import annotations

import numpy as np
from scipy.special import loggamma


def k_grid(k_min, k_max, N):
    """The N log-spaced wave-numbers of eq. pklfft, both ends included."""
    return k_min * (k_max / k_min) ** (np.arange(N) / (N - 1))


def coefficients(Pk, k_min, k_max, nu):
    """c_m and eta_m of eqs. cm and pklfft_eta, m = -N/2..N/2 (N + 1 values, N even)."""
    Pk = np.asarray(Pk, dtype=np.float64)
    N = len(Pk)
    if N % 2:
        raise ValueError("N must be even")
    k = k_grid(k_min, k_max, N)
    m = np.arange(-N // 2, N // 2 + 1)
    eta = (N - 1) / N * 2.0 * np.pi * m / np.log(k_max / k_min)
    l = np.arange(N)
    f = Pk * (k / k_min) ** (-nu)
    dft = np.exp(-2j * np.pi * np.outer(m, l) / N) @ f / N     # plain DFT, no wrap-around
    W = np.ones(N + 1)
    W[0] = W[-1] = 0.5
    c = W * k_min ** (-nu - 1j * eta) * dft
    return c, eta


def gamma_factor(a, n, mt):
    """g_{n,mt}(a) = 2^{mt+a-1} Gamma((1+mt+a+n)/2) / (pi Gamma((1-a-mt+n)/2))."""
    a = np.asarray(a, dtype=np.complex128)
    return np.exp((mt + a - 1.0) * np.log(2.0) + loggamma(0.5 * (1 + mt + a + n))
                  - loggamma(0.5 * (1 - a - mt + n))) / np.pi


def hankel_factor(c, eta, nu, n, mt, x):
    """int dk/(2 pi) k^{mt+1} P(k) J_n(x k) from the expansion: sum_s c_s g(a_s) x^{-(1+a_s+mt)}."""
    a = 1.0 + nu + 1j * eta
    g = gamma_factor(a, n, mt)
    x = np.asarray(x, dtype=np.float64)
    return (c * g)[None, :] * np.exp(-(1.0 + a[None, :] + mt) * np.log(x)[:, None])


def a_matrix(chi, F, a1, a2):
    """A_{s1 s2} = int dchi F chi^{-a1 - a2 - 2}, trapezoid in ln chi on the log-spaced grid chi."""
    chi = np.asarray(chi, dtype=np.float64)
    lc = np.log(chi)
    w = np.full(len(chi), lc[1] - lc[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    d = w * chi * np.asarray(F, dtype=np.float64) * chi ** -2.0       # dchi = chi dln chi
    X1 = np.exp(-np.outer(lc, a1))
    X2 = np.exp(-np.outer(lc, a2))
    return (X1 * d[:, None]).T @ X2


def i_matrix(P, k_min, k_max, chi, F, theta1, theta2, n1, mt1, nu1, n2, mt2, nu2):
    """I^{(n1,mt1)}_{(n2,mt2)}(theta1_i, theta2_j) of step 4, complex [len(theta1), len(theta2)]."""
    c1, eta1 = coefficients(P, k_min, k_max, nu1)
    c2, eta2 = coefficients(P, k_min, k_max, nu2)
    a1 = 1.0 + nu1 + 1j * eta1
    a2 = 1.0 + nu2 + 1j * eta2
    A = a_matrix(chi, F, a1, a2)
    U1 = hankel_factor(c1, eta1, nu1, n1, mt1, theta1)
    U2 = hankel_factor(c2, eta2, nu2, n2, mt2, theta2)
    return U1 @ A @ U2.T


def a_functions(P, k_min, k_max, chi, F, theta, nu0=-1.3, nu1p=-2.5, nu1m=-1.3, nu2=-1.3):
    """A_0, A_1, A_2 on theta x theta (step 5), complex arrays [3, T, T]."""
    A0 = i_matrix(P, k_min, k_max, chi, F, theta, theta, 0, 0, nu0, 0, 0, nu0)
    I11 = i_matrix(P, k_min, k_max, chi, F, theta, theta, 1, 1, nu1p, 1, -1, nu1m)
    A1 = I11 + I11.T
    A2 = i_matrix(P, k_min, k_max, chi, F, theta, theta, 2, 0, nu2, 2, 0, nu2)
    return np.stack([A0, A1, A2])
