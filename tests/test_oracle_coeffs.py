"""Pins for the oracle's coefficient fit (Section III), each against something
other than the oracle itself: numpy's Chebyshev routines, the Bessel-function
series of exp, the orthogonality the paper states (eq. 14), the interpolation
property, the classical error bound, and numbers printed in the paper."""
import math

import mpmath
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import polynomial as nppoly
from scipy import special

from oracle import coeffs as K


def _poly_mp(c, x):
    with mpmath.workdps(60):
        return mpmath.fsum(mpmath.mpf(cn) * mpmath.mpf(x) ** n for n, cn in enumerate(c))


def test_monomial_table_matches_numpy_cheb2poly():
    a = K.chebyshev_monomial_table(30)
    for l in range(31):
        ref = npcheb.cheb2poly([0] * l + [1])
        got = np.array(a[l][: l + 1], dtype=np.float64)
        np.testing.assert_array_equal(got, ref)
        assert all(v == 0 for v in a[l][l + 1:])


@pytest.mark.parametrize("l", [3, 11, 29])
def test_discrete_orthogonality_eq14(l):
    xi = K.chebyshev_zeros(l)
    for i in range(l):
        for j in range(l):
            s = float(mpmath.fsum(K.chebyshev_T(i, x) * K.chebyshev_T(j, x) for x in xi))
            want = 0.0 if i != j else (l if i == 0 else l / 2)
            assert abs(s - want) < 1e-12


def test_zeros_are_roots_and_T_matches_numpy():
    with mpmath.workdps(50):
        for l in (1, 4, 17):
            for x in K.chebyshev_zeros(l):
                assert abs(float(K.chebyshev_T(l, x))) < 1e-40
    for l in range(12):
        for x in np.linspace(-1, 1, 9):
            assert abs(float(K.chebyshev_T(l, x)) - npcheb.chebval(x, [0] * l + [1])) < 1e-13


def _aliased_bessel(mu, N, terms=40):
    """Interpolation coefficients of exp(mu y) at the zeros of T_{N+1}, from
    the Chebyshev series exp(mu y) = I_0 + 2 sum_k I_k(mu) T_k(y) and the
    aliasing T_{2m(N+1) +- l} -> (-1)^m T_l at those zeros."""
    cc = lambda k: special.iv(0, mu) if k == 0 else 2.0 * special.iv(k, mu)
    M = 2 * (N + 1)
    d = []
    for l in range(N + 1):
        s = cc(l)
        for m in range(1, terms):
            if l == 0:
                s += (-1) ** m * cc(M * m)
            else:
                s += (-1) ** m * (cc(M * m - l) + cc(M * m + l))
        d.append(s)
    return np.array(d)


@pytest.mark.parametrize("sigma_r,N", [(30.0, 28), (30.0, 10), (50.0, 11), (20.0, 62), (60.0, 8)])
def test_fit_equals_bessel_aliasing(sigma_r, N):
    _, d = K.gcf_coefficients(sigma_r, N)
    _, mu = K.gcf_params(sigma_r)
    ref = _aliased_bessel(mu, N)
    scale = special.iv(0, mu)
    assert np.max(np.abs(np.array(d) - ref)) <= 1e-13 * scale


@pytest.mark.parametrize("sigma_r,N", [(30.0, 28), (40.0, 16), (30.0, 12)])
def test_interpolates_exp_at_scaled_nodes(sigma_r, N):
    c, _ = K.gcf_coefficients(sigma_r, N)
    _, mu = K.gcf_params(sigma_r)
    with mpmath.workdps(60):
        for x in K.chebyshev_zeros(N + 1):
            y = mu * x
            got = mpmath.fsum(mpmath.mpf(cn) * y ** n for n, cn in enumerate(c))
            # c_n are rounded to FP64: the monomial sum carries up to
            # sum_n |c_n| |y|^n * 2^-53 of rounding.
            slack = mpmath.fsum(abs(mpmath.mpf(cn)) * abs(y) ** n for n, cn in enumerate(c)) * 2.0 ** -53
            assert abs(got - mpmath.exp(y)) <= slack


@pytest.mark.parametrize("mu,N", [(1.0, 10), (18.0625, 28), (6.5025, 11), (10.16015625, 16)])
def test_error_within_chebyshev_tail_bound(mu, N):
    sigma_r = 127.5 / math.sqrt(mu)
    c, _ = K.gcf_coefficients(sigma_r, N)
    y = np.linspace(-1, 1, 2001)
    with mpmath.workdps(40):
        err = max(abs(_poly_mp(c, mu * yy) - mpmath.exp(mu * yy)) for yy in y)
    tail = 2.0 * sum(2.0 * special.iv(k, mu) for k in range(N + 1, N + 80))
    assert float(err) <= tail * (1 + 1e-9)
    # and the first neglected term sets its size: near-minimax behaviour
    assert float(err) >= 2.0 * special.iv(N + 1, mu) * 0.5


@pytest.mark.parametrize("mu,N", [(1.0, 10), (18.0625, 28), (6.5025, 11)])
def test_error_alternates_at_extrema(mu, N):
    """The interpolation error changes sign between consecutive extrema
    cos(k pi/(N+1)) of T_{N+1}: the near-minimax shape (Section III-A)."""
    sigma_r = 127.5 / math.sqrt(mu)
    c, _ = K.gcf_coefficients(sigma_r, N)
    signs = []
    for k in range(N + 2):
        yk = math.cos(k * math.pi / (N + 1))
        e = mpmath.exp(mu * yk) - _poly_mp(c, mu * yk)
        signs.append(mpmath.sign(e))
    assert all(signs[k] == -signs[k + 1] for k in range(N + 1)), signs


def test_fig1_chebyshev_beats_taylor_on_unit_interval():
    """Fig. 1 (Section III-B): exp on [-1, 1] at N = 10. Taylor's l_inf error
    is its remainder at x = 1, e - sum 1/n!; Chebyshev's is bracketed by the
    first neglected Bessel coefficient and twice the tail."""
    N = 10
    mu = 1.0
    sigma_r = 127.5 / math.sqrt(mu)
    c, _ = K.gcf_coefficients(sigma_r, N)
    x = np.linspace(-1, 1, 2001)
    cheb = max(abs(float(_poly_mp(c, v)) - math.exp(v)) for v in x)
    t = K.taylor_coefficients(N)
    taylor = max(abs(float(_poly_mp(t, v)) - math.exp(v)) for v in x)
    assert abs(taylor - (math.e - sum(1 / math.factorial(n) for n in range(N + 1)))) < 1e-15
    assert 2 * special.iv(N + 1, 1.0) * 0.9 <= cheb <= 2 * sum(2 * special.iv(k, 1.0) for k in range(N + 1, 40))
    assert cheb < taylor / 100.0


def test_fig2_fig3_translated_kernels(golden):
    """Figs. 2-3: g_30(t - tau) approximated through eq. (4) over the centred
    range [-t_c, t_c] at N = 20. The paper's point (Section III-B, Section IV)
    is that Taylor degrades away from the origin while Chebyshev holds over
    the whole interval, most of all for large tau. Pinned: at the far ends of
    the range (|t| >= 0.8 t_c) Chebyshev is the more accurate for every tau
    the figures show, and for |tau| >= 110 it is the more accurate over the
    whole range. (For tau in {+-100, 90} the Chebyshev error peaks mid-range
    and its maximum exceeds Taylor's; the figures themselves are not
    available to settle what they plot.)"""
    spec = golden["fig_translated_kernels"]
    sr, N = spec["sigma_r"], spec["N"]
    t_c = golden["intensity_range"]["t_c"]
    cheb, _ = K.gcf_coefficients(sr, N)
    tayl = K.taylor_coefficients(N)
    t = np.linspace(-t_c, t_c, 2041)
    far = np.abs(t) >= 0.8 * t_c
    for tau in spec["tau"]:
        exact = np.exp(-(t - tau) ** 2 / (2 * sr * sr))
        x = tau * t / (sr * sr)
        pre = np.exp(-tau * tau / (2 * sr * sr)) * np.exp(-t * t / (2 * sr * sr))
        e_c = np.abs(pre * nppoly.polyval(x, cheb) - exact)
        e_t = np.abs(pre * nppoly.polyval(x, tayl) - exact)
        assert e_c[far].max() < 0.3 * e_t[far].max(), (tau, e_c[far].max(), e_t[far].max())
        if abs(tau) >= 120:
            assert e_c.max() < 0.3 * e_t.max(), (tau, e_c.max(), e_t.max())


def test_centre_and_mu(golden):
    rng = golden["intensity_range"]
    t_c, mu = K.gcf_params(30.0, rng["L"], rng["U"])
    assert t_c == rng["t_c"]
    # g(i) g(i-j) / sigma_r^2 spans exactly [-mu, mu] over the centred range
    assert mu == pytest.approx(t_c * t_c / 900.0, rel=1e-15)


def test_degree_rule_keeps_paper_operating_point(golden):
    """Table 2 runs at sigma_r = 30 with N = 28; the rule must return that,
    stay there for small moves of sigma_r, and grow as sigma_r shrinks."""
    assert K.degree_rule(golden["table2"]["sigma_r"]) == golden["table2"]["N"]
    assert K.degree_rule(29.8) == 28 and K.degree_rule(30.2) == 28
    sr = [10, 12, 15, 20, 25, 30, 35, 40, 50, 60]
    Ns = [K.degree_rule(s) for s in sr]
    assert all(a >= b for a, b in zip(Ns, Ns[1:]))
    assert Ns[0] > 200 and Ns[-1] < 12


def test_kernel_error_gap_matches_fig5_vs_table2(golden):
    """Soft pin: Fig. 5 (N = 26) and Table 2 at sigma_s = 5 (N = 28) differ
    by about 20 dB; MSE scales as the square of the weighted kernel error
    eps_N = max_y exp(-mu|y|) |p_N(mu y) - exp(mu y)|."""
    def eps(N):
        c, _ = K.gcf_coefficients(30.0, N)
        _, mu = K.gcf_params(30.0)
        y = np.linspace(-1, 1, 20001)
        with mpmath.workdps(40):
            return max(float(mpmath.exp(-mu * abs(v)) * abs(_poly_mp(c, mu * v) - mpmath.exp(mu * v)))
                       for v in y[::10])
    pred = 20 * math.log10(eps(26) / eps(28))
    paper = golden["fig_testpat"]["GCF_dB"] - golden["table2"]["GCF_dB"][golden["table2"]["sigma_s"].index(5)]
    assert abs(pred - paper) < 3.0, (pred, paper)


def test_bad_arguments():
    with pytest.raises(ValueError):
        K.gcf_coefficients(30.0, 0)
    with pytest.raises(ValueError):
        K.gcf_coefficients(-1.0, 5)


# ---- minimax (Remez) coefficients: pinned by the alternation theorem, a
# closed form at degree 1, and the de la Vallee Poussin bracket.

def _dense_max_error(mu, coeffs_T, n=6001):
    import mpmath
    from oracle import coeffs as K
    with mpmath.workdps(40):
        ys = [mpmath.mpf(-1) + 2 * mpmath.mpf(i) / (n - 1) for i in range(n)]
        return max(abs(mpmath.exp(mu * y) - K._clenshaw(coeffs_T, y)) for y in ys)


@pytest.mark.parametrize("mu,N", [(1.0, 5), (6.5025, 11), (18.0625, 16)])
def test_minimax_equioscillates(mu, N):
    """Alternation theorem: the error takes the values (-1)^k E at N+2
    increasing points and nowhere exceeds |E|, which makes the polynomial the
    unique best uniform approximation of degree N."""
    import mpmath
    from oracle import coeffs as K
    e, E, ref = K.minimax_fit(mu, N)
    assert len(ref) == N + 2 and all(ref[k] < ref[k + 1] for k in range(N + 1))
    with mpmath.workdps(40):
        vals = [mpmath.exp(mu * x) - K._clenshaw(e, x) for x in ref]
        for k, v in enumerate(vals):
            assert abs(v - (-1) ** k * E) <= 1e-25 * abs(E) + mpmath.mpf(10) ** -35
        assert _dense_max_error(mu, e) <= abs(E) * (1 + 1e-9)


@pytest.mark.parametrize("mu", [1.0, 2.5])
def test_minimax_linear_closed_form(mu):
    """Degree 1, convex exp(mu y): slope = the secant's, intercept halfway
    between the secant and the tangent of that slope (touching at x* with
    mu exp(mu x*) = slope)."""
    import math
    from oracle import coeffs as K
    e, E, _ = K.minimax_fit(mu, 1)
    m = (math.exp(mu) - math.exp(-mu)) / 2
    xs = math.log(m / mu) / mu
    c = (math.exp(-mu) + m + math.exp(mu * xs) - m * xs) / 2
    assert abs(float(e[1]) - m) <= 1e-13 * m
    assert abs(float(e[0]) - c) <= 1e-13 * abs(c)
    assert abs(abs(float(E)) - abs(math.exp(-mu) - (c - m))) <= 1e-13


@pytest.mark.parametrize("mu,N", [(1.0, 6), (18.0625, 20), (18.0625, 28)])
def test_minimax_bracketed_by_interpolant(mu, N):
    """min_k |r(x_k)| over the N+2 Chebyshev extrema, where the interpolant's
    error r alternates in sign, is a lower bound for the minimax error (de la
    Vallee Poussin); the interpolant's own maximum error is an upper bound."""
    import mpmath
    from oracle import coeffs as K
    _, E, _ = K.minimax_fit(mu, N)
    with mpmath.workdps(60):
        d = K.chebyshev_fit(mpmath.exp, mpmath.mpf(mu), N)     # coefficients of T_l(x / mu)
        ext = [mpmath.cos(mpmath.pi * k / (N + 1)) for k in range(N + 2)]
        r = [mpmath.exp(mu * x) - K._clenshaw(d, x) for x in ext]
        assert all(r[k] * r[k + 1] < 0 for k in range(N + 1))
        lower = min(abs(v) for v in r)
        upper = _dense_max_error(mu, d)
    assert lower <= abs(E) * (1 + 1e-12)
    assert abs(E) <= upper
    assert abs(E) < upper          # strictly better than node interpolation


def test_minimax_monomial_coefficients_evaluate_the_fit():
    """The monomial c_n (scaled as in eq. 19) evaluate to the same polynomial
    as the Chebyshev-basis fit."""
    import mpmath
    from oracle import coeffs as K
    sr, N = 50.0, 11
    _, mu = K.gcf_params(sr)
    c = K.minimax_coefficients(sr, N)
    e, _, _ = K.minimax_fit(mu, N)
    for y in np.linspace(-1, 1, 41):
        x = mu * y
        mono = sum(cn * x ** n for n, cn in enumerate(c))
        with mpmath.workdps(40):
            ref = float(K._clenshaw(e, mpmath.mpf(y)))
        assert abs(mono - ref) <= 1e-12 * math.exp(mu)


def test_minimax_coefficient_derivative_matches_implicit_form():
    """dc/dsigma_r of the minimax fit by central differences (the oracle)
    against the implicit-function form: with the reference frozen, the
    levelled system with right-hand side y_k exp(mu y_k) gives de_l/dmu (the
    interior reference points are extrema of the error, so their motion
    drops out to first order)."""
    import mpmath
    sr, N = 50.0, 7
    c, dc = K.minimax_coefficients_with_derivative(sr, N)
    with mpmath.workdps(60):
        mu = mpmath.mpf(255) ** 2 / (4 * mpmath.mpf(sr) ** 2)
        e, E, ref = K.minimax_fit(mu, N, tol=1e-40)
        A = mpmath.matrix(N + 2, N + 2)
        rhs = mpmath.matrix(N + 2, 1)
        for k, x in enumerate(ref):
            for l in range(N + 1):
                A[k, l] = K.chebyshev_T(l, x)
            A[k, N + 1] = (-1) ** k
            rhs[k] = x * mpmath.exp(mu * x)
        de = mpmath.lu_solve(A, rhs)
        a = K.chebyshev_monomial_table(N)
        dmu = -2 * mu / sr
        for n in range(N + 1):
            b = mpmath.fsum(e[l] * a[l][n] for l in range(n, N + 1))
            db = mpmath.fsum(de[l] * a[l][n] for l in range(n, N + 1))
            want = (db - n * b / mu) / mu ** n * dmu           # c_n = mu^-n b_n
            assert abs(float(want) - dc[n]) <= 1e-10 * abs(float(want)) + 1e-300
