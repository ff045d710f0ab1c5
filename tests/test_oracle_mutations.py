"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each test swaps one oracle function for a plausibly wrong version and checks that a
pin from tests/pins.py raises.  This shows the pins constrain every step: the bearing
(sign and handedness), the exponent sign, the bin rule, the normaliser, the
contraction's operand order, the pivot weight and the removal of the k = j terms, the operand order of the multi-field contraction and the
planar bearing.
"""

import numpy as np
import pytest

from oracle import ref
from tests import pins


def _mirror_basis(orig):
    def f(piv):
        e_n, e_e = orig(piv)
        return e_n, -e_e
    return f


def test_mirrored_bearing_fails_three_point(monkeypatch):
    monkeypatch.setattr(ref, "bearing_basis", _mirror_basis(ref.bearing_basis))
    with pytest.raises(AssertionError):
        pins.check_three_point()


def test_swapped_north_east_fails_three_point(monkeypatch):
    orig = ref.bearing_basis
    monkeypatch.setattr(ref, "bearing_basis", lambda piv: orig(piv)[::-1])
    with pytest.raises(AssertionError):
        pins.check_three_point()


def test_positive_exponent_fails_three_point(monkeypatch):
    orig = ref.multipoles

    def plus(*a, **k):
        am, W, N = orig(*a, **k)
        return np.conj(am), W, N
    monkeypatch.setattr(ref, "multipoles", plus)
    with pytest.raises(AssertionError):
        pins.check_three_point()


def test_transposed_contraction_fails_three_point(monkeypatch):
    orig = ref.contract
    monkeypatch.setattr(ref, "contract", lambda X, vp: np.swapaxes(orig(X, vp), 1, 2))
    with pytest.raises(AssertionError):
        pins.check_three_point()


def test_dropped_normaliser_fails_weight_invariance(monkeypatch):
    monkeypatch.setattr(ref, "normalise", lambda a, W: a)
    with pytest.raises(AssertionError):
        pins.check_weight_invariance()


def test_total_weight_normaliser_fails_m0_means(monkeypatch):
    # per-pivot total weight instead of the per-bin weight
    monkeypatch.setattr(ref, "normalise", lambda a, W: a / np.maximum(W.sum(1), 1e-300)[:, None, None])
    with pytest.raises(AssertionError):
        pins.check_m0_annulus_means()


def test_closed_bins_fail_brute(monkeypatch):
    def closed(d2, edges):
        nb = len(edges) - 1
        b = np.searchsorted(edges, d2, side="left") - 1
        b[(b < 0) | (b >= nb)] = -1
        return b
    monkeypatch.setattr(ref, "bin_index", closed)
    xyz, w, x = pins.random_cap(40, 2.0, 21)
    d = xyz[:, 1] - xyz[:, 0]
    d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    E = np.array([d2 / 3, d2, 3 * d2])
    _, _, N = ref.multipoles(xyz[:, :1], xyz[:, :2], w[:2], x[:2], E, 0)
    assert N[0].tolist() != [0, 1]


def test_doubled_phase_fails_brute(monkeypatch):
    orig = ref.bearing
    monkeypatch.setattr(ref, "bearing", lambda d, n, e: 2.0 * orig(d, n, e))
    with pytest.raises(AssertionError):
        pins.check_brute(n=120, seed=3, m_max=3)


def test_unweighted_pivots_fail_brute(monkeypatch):
    orig = ref.contract
    monkeypatch.setattr(ref, "contract", lambda X, vp: orig(X, np.sign(vp)))
    with pytest.raises(AssertionError):
        pins.check_brute(n=120, seed=4, m_max=3)


def test_self_term_with_one_normaliser_fails_brute(monkeypatch):
    # k = j terms divided by W instead of W^2
    def wrong(W, Q, vp):
        safe = np.where(W > 0, W, 1.0)
        return np.where(W > 0, Q / safe, 0.0).T @ vp
    monkeypatch.setattr(ref, "self_pair_term", wrong)
    with pytest.raises(AssertionError):
        pins.check_brute_no_self()


def test_self_term_of_the_plain_field_fails_brute(monkeypatch):
    # Q taken as sum w |x| instead of sum (w x)^2 (the square dropped from the field)
    orig = ref.multipoles

    def wrong(piv, nbr, w, x, edges, m_max, block=128):
        if m_max == 0:
            x = np.sqrt(np.abs(x / w)) * np.sign(x)
        return orig(piv, nbr, w, x, edges, m_max, block)
    monkeypatch.setattr(ref, "multipoles", wrong)
    with pytest.raises(AssertionError):
        pins.check_brute_no_self()


def test_cross_conjugate_on_the_wrong_field_fails_brute(monkeypatch):
    def wrong(Xa, Xb, vp):
        M1, nb = Xa.shape[1], Xa.shape[2]
        out = np.zeros((M1, nb, nb), dtype=np.complex128)
        for p in range(Xa.shape[0]):
            out += vp[p] * (np.conj(Xa[p][:, :, None]) * Xb[p][:, None, :])
        return out
    monkeypatch.setattr(ref, "contract_cross", wrong)
    with pytest.raises(AssertionError):
        pins.check_cross_brute()


def test_cross_pivot_field_swapped_fails_brute(monkeypatch):
    orig = ref.estimate_cross

    def wrong(piv, nbr, w, fields, edges, m_max, wp, pivot_fields, cyclic=False):
        # the pivot takes field B instead of A
        pf = (pivot_fields[1], pivot_fields[1], pivot_fields[2])
        return orig(piv, nbr, w, fields, edges, m_max, wp, pf, cyclic)
    monkeypatch.setattr(ref, "estimate_cross", wrong)
    with pytest.raises(AssertionError):
        pins.check_cross_brute()


def test_planar_bearing_from_the_x_axis_fails_three_point(monkeypatch):
    # angle measured from +x counter-clockwise instead of from +y towards +x
    monkeypatch.setattr(ref, "planar_bearing", lambda dx, dy: np.arctan2(dy, dx))
    with pytest.raises(AssertionError):
        pins.check_three_point_planar()


def test_cross_catalogues_shared_normaliser_fails_brute(monkeypatch):
    # X^C normalised by catalogue B's bin weights instead of its own
    orig = ref.estimate_cross_catalogues

    def wrong(piv, wp, xp, nbr_b, w_b, x_b, nbr_c, w_c, x_c, edges, m_max):
        a_b, W_b, N_b = ref.multipoles(piv, nbr_b, w_b, x_b, edges, m_max)
        a_c, W_c, N_c = ref.multipoles(piv, nbr_c, w_c, x_c, edges, m_max)
        z = ref.contract_cross(ref.normalise(a_b, W_b), ref.normalise(a_c, W_b), wp * xp)
        return z / np.sum(wp), int(N_b.sum()), int(N_c.sum())
    monkeypatch.setattr(ref, "estimate_cross_catalogues", wrong)
    with pytest.raises(AssertionError):
        pins.check_cross_catalogues_brute()


# ---- angular-histogram estimator (oracle/hist.py) ------------------------------------------

from oracle import hist  # noqa: E402
from tests import test_oracle_hist as H  # noqa: E402


def test_hist_bin_start_phase_fails_ring_closed_form(monkeypatch):
    def start(Hh, m_max):
        F = np.fft.fft(Hh, axis=-1)
        return F[..., :m_max + 1]  # every pair at its bin's start, no half-bin phase
    monkeypatch.setattr(hist, "fourier_over_bins", start)
    with pytest.raises(AssertionError):
        H.test_ring_closed_form(8, 5, 3)


def test_hist_conjugated_transform_fails_three_point(monkeypatch):
    orig = hist.fourier_over_bins
    monkeypatch.setattr(hist, "fourier_over_bins", lambda Hh, m: np.conj(orig(Hh, m)))
    with pytest.raises(AssertionError):
        H.test_three_point_golden(8)


def test_hist_mirrored_boundaries_fail_bearing_bins(monkeypatch):
    orig = hist.angular_bin
    monkeypatch.setattr(hist, "angular_bin", lambda u1, u2, b: orig(u1, u2, b * np.array([1.0, -1.0])))
    with pytest.raises(AssertionError):
        H.test_bins_match_direct_bearing(16)


def test_hist_flipped_east_fails_bearing_bins(monkeypatch):
    orig = hist.frame_unnormalised
    monkeypatch.setattr(hist, "frame_unnormalised", lambda piv: (orig(piv)[0], -orig(piv)[1]))
    with pytest.raises(AssertionError):
        H.test_bins_match_direct_bearing(16)


# ---- FFTLog chain (oracle/fftlog.py) --------------------------------------------------------

from oracle import fftlog  # noqa: E402
from tests import test_oracle_fftlog as FL  # noqa: E402


def test_fftlog_phases_without_n_minus_1_over_n_fail(monkeypatch):
    orig = fftlog.coefficients

    def wrong(Pk, kmin, kmax, nu):
        c, eta = orig(Pk, kmin, kmax, nu)
        N = len(Pk)
        return c * (kmin ** (-1j * eta)) * kmin ** (1j * eta * N / (N - 1)), eta * N / (N - 1)
    monkeypatch.setattr(fftlog, "coefficients", wrong)
    with pytest.raises(AssertionError):
        FL.test_hankel_factor_closed_forms(0, 0, -1.3)


def test_fftlog_gamma_factor_without_pi_fails(monkeypatch):
    orig = fftlog.gamma_factor
    monkeypatch.setattr(fftlog, "gamma_factor", lambda a, n, mt: orig(a, n, mt) * np.pi)
    with pytest.raises(AssertionError):
        FL.test_hankel_factor_closed_forms(1, 1, -2.5)


def test_fftlog_quadrature_measure_fails(monkeypatch):
    orig = fftlog.a_matrix
    monkeypatch.setattr(fftlog, "a_matrix", lambda chi, Fc, a1, a2: orig(chi, np.asarray(Fc) / chi, a1, a2))
    with pytest.raises(AssertionError):
        FL.test_a_matrix_closed_form()
