// Host planning: coefficient fit (Section III), taps (Section I), plane
// scales and the parameter block. Pure C++, no HIP.
#include "plan.hpp"

#include <quadmath.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

namespace bfgc {

int radius_of(double sigma_s) { return (int)std::ceil(3.0 * sigma_s - 1e-12); }

// Modified Bessel function of the first kind, I_nu(x) for integer nu >= 0 and
// x >= 0, by its power series sum_k (x/2)^{2k+nu} / (k! (k+nu)!). All terms
// are positive, so the sum carries no cancellation.
static long double bessel_i(int nu, long double x) {
    if (x == 0.0L) return nu == 0 ? 1.0L : 0.0L;
    const long double h = 0.5L * x;
    long double term = std::exp((long double)nu * std::log(h) - std::lgamma((long double)nu + 1.0L));
    long double sum = term;
    for (int k = 1; k < 100000; ++k) {
        term *= h * h / ((long double)k * (long double)(k + nu));
        sum += term;
        if (term < 1e-22L * sum && k > h) break;
    }
    return sum;
}

// The rule's threshold: the geometric mean of the first neglected Chebyshev
// coefficients at N = 28 and 29 for sigma_r = 30.
static long double rule_eps0() {
    static const long double eps0 = [] {
        const long double mu30 = (long double)kTh * kTh / (30.0L * 30.0L);
        return std::sqrt(2.0L * bessel_i(28, mu30) * 2.0L * bessel_i(29, mu30));
    }();
    return eps0;
}

// Smallest N <= max_degree with 2 I_{N+1}(mu) <= eps0, else -1; results are
// cached per (mu, max_degree): the batch planner asks for the same values
// on every call.
static int rule_at_mu(long double mu, int max_degree) {
    static std::mutex mtx;
    static std::map<std::pair<long double, int>, int> cache;
    const auto key = std::make_pair(mu, max_degree);
    {
        std::lock_guard<std::mutex> lock(mtx);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const long double eps0 = rule_eps0();
    int n = -1;
    for (int N = 1; N <= max_degree; ++N)
        if (2.0L * bessel_i(N + 1, mu) <= eps0) {
            n = N;
            break;
        }
    std::lock_guard<std::mutex> lock(mtx);
    cache.emplace(key, n);
    return n;
}

int degree_rule(double sigma_r, int max_degree) {
    if (!(sigma_r > 0.0) || !std::isfinite(sigma_r)) return -1;
    return rule_at_mu((long double)kTh * kTh / ((long double)sigma_r * sigma_r), max_degree);
}

// Conditioning of the double coefficients the kernels use, on a grid of y:
// the weighted error of the polynomial against exp(mu y) and kappa.
static void condition(Fit &F, int N) {
    typedef long double ld;
    const int K = N + 1;
    std::vector<ld> b(K);
    for (int n = 0; n < K; ++n) b[n] = F.b[n];
    const ld mul = (ld)F.mu;
    const int M = 4000;
    ld kerr = 0.0L, kap = 0.0L;
    for (int m = 0; m <= M; ++m) {
        const ld y = -1.0L + 2.0L * m / M;
        ld p = 0.0L, q = 0.0L;
        const ld ay = std::fabs(y);
        for (int n = N; n >= 0; --n) {
            p = p * y + b[n];
            q = q * ay + std::fabs(b[n]);
        }
        const ld wgt = std::exp(-mul * ay);
        const ld err = wgt * std::fabs(p - std::exp(mul * y));
        if (err > kerr) kerr = err;
        if (wgt * q > kap) kap = wgt * q;
    }
    F.kernel_err = (double)kerr;
    F.kappa = (double)kap;
}

// The fit of exp(mu y), y in [-1, 1], at the N+1 zeros of T_{N+1}:
//   xi_k = cos(pi (2k-1) / (2(N+1))),  k = 1..N+1
//   d_0 = 1/(N+1) sum_k e^{mu xi_k},  d_l = 2/(N+1) sum_k e^{mu xi_k} T_l(xi_k)
// (eq. 16 in its rescaled form), T_l(xi_k) = cos(l theta_k) (eq. 11); then the
// monomial coefficients of T_l from T_{l+1} = 2x T_l - T_{l-1} (eqs. 12-13) and
// b_n = sum_{l >= n} d_l a_{l,n} (eq. 19 with mu^n folded into y = x/mu).
// The last sum cancels heavily (its terms reach I_0(mu) 2^{N-1} while b_n can
// be tiny), so the fit runs in binary128 and is rounded to double at the end.
static Fit compute_fit_q(__float128 mu, int N) {
    typedef __float128 qd;
    Fit F;
    F.mu = (double)mu;
    const int K = N + 1;
    std::vector<qd> theta(K), e(K), xe(K);
    for (int k = 1; k <= K; ++k) {
        theta[k - 1] = M_PIq * (qd)(2 * k - 1) / (qd)(2 * K);
        const qd xi = cosq(theta[k - 1]);
        e[k - 1] = expq(mu * xi);
        xe[k - 1] = xi * e[k - 1];                 // d/dmu of e^{mu xi_k}
    }
    std::vector<qd> d(K), dd(K);
    for (int l = 0; l <= N; ++l) {
        qd s = 0, sd = 0;
        for (int k = 0; k < K; ++k) {
            const qd t = cosq((qd)l * theta[k]);
            s += e[k] * t;
            sd += xe[k] * t;
        }
        d[l] = (l == 0 ? (qd)1 : (qd)2) * s / (qd)K;
        dd[l] = (l == 0 ? (qd)1 : (qd)2) * sd / (qd)K;
    }
    // a[l][n] row by row; three rows are enough to accumulate b_n.
    std::vector<qd> bq(K, (qd)0), bdq(K, (qd)0), am1(K, (qd)0), a0(K, (qd)0), ap1(K, (qd)0);
    a0[0] = 1;                                     // T_0 = 1
    for (int n = 0; n < K; ++n) {
        bq[n] += d[0] * a0[n];
        bdq[n] += dd[0] * a0[n];
    }
    if (N >= 1) {
        am1 = a0;
        std::fill(a0.begin(), a0.end(), (qd)0);
        a0[1] = 1;                                 // T_1 = x
        for (int n = 0; n < K; ++n) {
            bq[n] += d[1] * a0[n];
            bdq[n] += dd[1] * a0[n];
        }
        for (int l = 1; l < N; ++l) {              // T_{l+1} = 2x T_l - T_{l-1}
            for (int n = 0; n < K; ++n) ap1[n] = (n >= 1 ? 2 * a0[n - 1] : (qd)0) - am1[n];
            for (int n = 0; n < K; ++n) {
                bq[n] += d[l + 1] * ap1[n];
                bdq[n] += dd[l + 1] * ap1[n];
            }
            am1.swap(a0);
            a0.swap(ap1);
        }
    }
    F.b.resize(K);
    F.bd.resize(K);
    for (int n = 0; n < K; ++n) {
        F.b[n] = (double)bq[n];
        F.bd[n] = (double)bdq[n];
    }

    condition(F, N);
    return F;
}

// Monomial coefficients of sum_l c_l T_l(y), from the rows of the T_l table
// (T_{l+1} = 2y T_l - T_{l-1}, eqs. 12-13), accumulated in binary128.
static std::vector<__float128> monomial_of(const std::vector<__float128> &c) {
    typedef __float128 qd;
    const int K = (int)c.size();
    std::vector<qd> out(K, (qd)0), am1(K, (qd)0), a0(K, (qd)0), ap1(K, (qd)0);
    a0[0] = 1;
    for (int n = 0; n < K; ++n) out[n] += c[0] * a0[n];
    if (K >= 2) {
        am1 = a0;
        std::fill(a0.begin(), a0.end(), (qd)0);
        a0[1] = 1;
        for (int n = 0; n < K; ++n) out[n] += c[1] * a0[n];
        for (int l = 1; l + 1 < K; ++l) {
            for (int n = 0; n < K; ++n) ap1[n] = (n >= 1 ? 2 * a0[n - 1] : (qd)0) - am1[n];
            for (int n = 0; n < K; ++n) out[n] += c[l + 1] * ap1[n];
            am1.swap(a0);
            a0.swap(ap1);
        }
    }
    return out;
}

static __float128 clenshaw_q(const std::vector<__float128> &c, __float128 y) {
    __float128 b1 = 0, b2 = 0;
    for (int l = (int)c.size() - 1; l >= 1; --l) {
        const __float128 t = 2 * y * b1 - b2 + c[l];
        b2 = b1;
        b1 = t;
    }
    return y * b1 - b2 + c[0];
}

// Solves A x = r in place (Gaussian elimination, partial pivoting). n x n, row-major.
static bool solve_q(std::vector<__float128> &A, std::vector<__float128> &r, int n) {
    typedef __float128 qd;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (fabsq(A[(size_t)i * n + col]) > fabsq(A[(size_t)piv * n + col])) piv = i;
        if (A[(size_t)piv * n + col] == 0) return false;
        if (piv != col) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)piv * n + j], A[(size_t)col * n + j]);
            std::swap(r[piv], r[col]);
        }
        const qd inv = 1 / A[(size_t)col * n + col];
        for (int i = col + 1; i < n; ++i) {
            const qd m = A[(size_t)i * n + col] * inv;
            if (m == 0) continue;
            for (int j = col; j < n; ++j) A[(size_t)i * n + j] -= m * A[(size_t)col * n + j];
            r[i] -= m * r[col];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        qd s = r[i];
        for (int j = i + 1; j < n; ++j) s -= A[(size_t)i * n + j] * r[j];
        r[i] = s / A[(size_t)i * n + i];
    }
    return true;
}

// Minimax (best uniform) polynomial of degree N for exp(mu y) on [-1, 1]
// (the ideal choice Section III names), by the Remez exchange algorithm in
// binary128, Chebyshev basis:
//   1. reference: the N+2 extrema of T_{N+1};
//   2. level: sum_l c_l T_l(y_k) + (-1)^k E = e^{mu y_k} on the reference;
//   3. the error r = e^{mu y} - p alternates over the reference, so it has a
//      zero in each gap (bisection); between consecutive zeros (and the ends)
//      its extremum (golden section) gives the next reference;
//   4. repeat until max |r| exceeds |E| by at most 1e-15 relative, then level
//      once more on the final reference.
// db_n/dmu: at the optimum the interior reference points are extrema of r, so
// to first order only the right-hand side moves: the levelled system with
// right-hand side y_k e^{mu y_k} gives dc_l/dmu. Returns false where the
// levelled error falls below 1e-28 of e^mu (binary128 would not resolve it)
// or the exchange does not converge.
static bool compute_remez(double sigma_r, int N, Fit &F) {
    typedef __float128 qd;
    const qd mu = (qd)kTh * (qd)kTh / ((qd)sigma_r * (qd)sigma_r);
    F.mu = (double)mu;
    const int K = N + 1, M = N + 2;
    std::vector<qd> ref(M), c(K), dc(K);
    for (int k = 0; k < M; ++k) ref[k] = -cosq(M_PIq * (qd)k / (qd)(N + 1));
    qd E = 0;
    auto level = [&](const std::vector<qd> &pts, bool deriv) -> bool {
        std::vector<qd> A((size_t)M * M), r(M), A2, r2(M);
        for (int k = 0; k < M; ++k) {
            const qd y = pts[k];
            qd tm1 = 1, t0 = y;
            for (int l = 0; l < K; ++l) {
                qd t;
                if (l == 0) t = 1;
                else if (l == 1) t = y;
                else {
                    t = 2 * y * t0 - tm1;
                    tm1 = t0;
                    t0 = t;
                }
                A[(size_t)k * M + l] = t;
            }
            A[(size_t)k * M + K] = (k & 1) ? -1 : 1;
            r[k] = expq(mu * y);
            r2[k] = y * r[k];
        }
        if (deriv) A2 = A;
        if (!solve_q(A, r, M)) return false;
        for (int l = 0; l < K; ++l) c[l] = r[l];
        E = r[K];
        if (deriv) {
            if (!solve_q(A2, r2, M)) return false;
            for (int l = 0; l < K; ++l) dc[l] = r2[l];
        }
        return true;
    };
    auto err = [&](qd y) { return expq(mu * y) - clenshaw_q(c, y); };
    bool converged = false;
    for (int it = 0; it < 60 && !converged; ++it) {
        if (!level(ref, false)) return false;
        std::vector<qd> edges(M + 1);
        edges[0] = -1;
        edges[M] = 1;
        for (int k = 0; k + 1 < M; ++k) {          // zero of r in (ref[k], ref[k+1])
            qd a = ref[k], b = ref[k + 1];
            const bool neg_a = err(a) < 0;
            for (int i = 0; i < 80; ++i) {
                const qd m = (a + b) / 2;
                if ((err(m) < 0) == neg_a) a = m;
                else b = m;
            }
            edges[k + 1] = (a + b) / 2;
        }
        std::vector<qd> next(M);
        qd emax = 0;
        const qd g = (sqrtq((qd)5) - 1) / 2;
        for (int k = 0; k < M; ++k) {              // extremum of sgn r on [edges[k], edges[k+1]]
            qd a = edges[k], b = edges[k + 1];
            const qd sgn = err((a + b) / 2) >= 0 ? 1 : -1;
            qd x1 = b - g * (b - a), x2 = a + g * (b - a);
            qd f1 = sgn * err(x1), f2 = sgn * err(x2);
            for (int i = 0; i < 110; ++i) {
                if (f1 >= f2) {
                    b = x2; x2 = x1; f2 = f1;
                    x1 = b - g * (b - a); f1 = sgn * err(x1);
                } else {
                    a = x1; x1 = x2; f1 = f2;
                    x2 = a + g * (b - a); f2 = sgn * err(x2);
                }
            }
            qd x = (a + b) / 2;
            if (k == 0 && sgn * err((qd)-1) >= sgn * err(x)) x = -1;
            if (k == M - 1 && sgn * err((qd)1) >= sgn * err(x)) x = 1;
            next[k] = x;
            const qd v = fabsq(err(x));
            if (v > emax) emax = v;
        }
        ref = next;
        converged = emax - fabsq(E) <= (qd)1e-15 * fabsq(E);
    }
    if (!converged || !level(ref, true)) return false;
    if (!(fabsq(E) > (qd)1e-28 * expq(mu))) return false;
    const std::vector<qd> bq = monomial_of(c), bdq = monomial_of(dc);
    F.b.resize(K);
    F.bd.resize(K);
    for (int n = 0; n < K; ++n) {
        F.b[n] = (double)bq[n];
        F.bd[n] = (double)bdq[n];
    }
    condition(F, N);
    return true;
}

static Fit compute_fit(double sigma_r, int N) {
    typedef __float128 qd;
    return compute_fit_q((qd)kTh * (qd)kTh / ((qd)sigma_r * (qd)sigma_r), N);
}

// Taylor coefficients of exp(mu y): b_n = mu^n / n!, db_n/dmu = mu^{n-1}/(n-1)!.
static Fit compute_taylor(double sigma_r, int N) {
    typedef __float128 qd;
    Fit F;
    const qd mu = (qd)kTh * (qd)kTh / ((qd)sigma_r * (qd)sigma_r);
    F.mu = (double)mu;
    F.b.resize(N + 1);
    F.bd.resize(N + 1);
    qd t = 1;                                      // mu^n / n!
    for (int n = 0; n <= N; ++n) {
        if (n > 0) t = t * mu / (qd)n;
        F.b[n] = (double)t;
        F.bd[n] = n == 0 ? 0.0 : (double)(t * (qd)n / mu);
    }
    condition(F, N);
    return F;
}

const Fit &fit(double sigma_r, int N, int kind) {
    static std::mutex mtx;
    static std::map<std::pair<double, int>, Fit> cache[3];
    std::lock_guard<std::mutex> lock(mtx);
    const int slot = kind == kFitTaylor ? 1 : kind == kFitMinimax ? 2 : 0;
    auto &C = cache[slot];
    auto key = std::make_pair(sigma_r, N);
    auto it = C.find(key);
    if (it != C.end()) return it->second;
    Fit F;
    if (slot == 1) F = compute_taylor(sigma_r, N);
    else if (slot == 2) {
        if (!compute_remez(sigma_r, N, F)) {   // marked unusable: the caller reports it
            F = Fit();
            F.mu = (double)kTh * kTh / (sigma_r * sigma_r);
            F.kappa = INFINITY;
            F.kernel_err = INFINITY;
        }
    } else F = compute_fit(sigma_r, N);
    return C.emplace(key, std::move(F)).first->second;
}

const Fit &fit_mu(double mu, int N) {
    static std::mutex mtx;
    static std::map<std::pair<double, int>, Fit> cache;
    std::lock_guard<std::mutex> lock(mtx);
    auto key = std::make_pair(mu, N);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    return cache.emplace(key, compute_fit_q((__float128)mu, N)).first->second;
}

int degree_rule_mu(double mu, int max_degree) {
    if (!(mu > 0.0) || !std::isfinite(mu)) return -1;
    return rule_at_mu((long double)mu, max_degree);
}

std::vector<Pivot> pivot_plan(double sigma_r, int K, int N, int max_degree) {
    std::vector<Pivot> out;
    const double L0 = kTc - kTh, U0 = kTc + kTh;
    const double h = (U0 - L0) / (2.0 * K);
    for (int k = 0; k < K; ++k) {
        Pivot p;
        p.lo = L0 + (U0 - L0) * k / K;
        p.hi = L0 + (U0 - L0) * (k + 1) / K;
        p.t = 0.5 * (p.lo + p.hi);
        p.h = h;
        p.R = std::max(p.t - L0, U0 - p.t);
        p.mu = h * p.R / (sigma_r * sigma_r);
        p.nu = p.R * p.R / (sigma_r * sigma_r);
        p.N = N > 0 ? N : degree_rule_mu(p.mu, max_degree);
        out.push_back(p);
    }
    return out;
}

// b_n and the taps rounded to float for the fused kernels.
static void store_float_coefficients(const ParamLayout &L, const std::vector<double> &b, const std::vector<double> &w,
                                     std::vector<double> &out) {
    std::vector<float> bf((size_t)2 * (((L.N + 3) / 2 + 7) & ~7), 0.0f);
    for (int n = 0; n <= L.N; ++n) bf[n] = (float)b[n];
    std::memcpy(out.data() + L.off_bf, bf.data(), bf.size() * sizeof(float));
    std::vector<float> tf((size_t)2 * (((2 * L.W + 2) / 2 + 7) & ~7), 0.0f);
    for (int t = 0; t <= 2 * L.W; ++t) tf[t] = (float)w[t];
    std::memcpy(out.data() + L.off_tf, tf.data(), tf.size() * sizeof(float));
}

void fill_params_pivot(const ParamLayout &L, double sigma_s, double mu, double nu, int stack_dtype,
                       std::vector<double> &out) {
    out.assign(L.total, 0.0);
    const std::vector<double> w = spatial_taps(sigma_s);
    for (int t = 0; t <= 2 * L.W; ++t) out[L.off_taps + t + (kTapPad - 1)] = w[t];
    const Fit &F = fit_mu(mu, L.N);
    const std::vector<int> k = plane_exponents(nu, L.N, stack_dtype);
    for (int n = 0; n <= L.N; ++n) {
        out[L.off_cq + n] = std::ldexp(F.b[n], -k[n]);
        out[L.off_cp + n] = std::ldexp(F.b[n], -k[n + 1]);
    }
    for (int n = 0; n <= L.N + 1; ++n) out[L.off_scale + n] = std::ldexp(1.0, k[n]);
    for (int n = 0; n <= L.N; ++n) out[L.off_bd + n] = F.bd[n];
    store_float_coefficients(L, F.b, w, out);
}

// Each damped-cosine section r^n (A cos(t n) + B sin(t n)), n >= 0, has the
// z-transform (A + r (B sin t - A cos t) z^-1) / (1 - 2 r cos t z^-1 + r^2 z^-2)
// with r = e^{-b/s}, t = w/s; the causal filter is the sum of the two sections
// over the product of their denominators. The anticausal part is h(n) for
// n <= -1, i.e. the causal transform in z minus its n = 0 term. k makes the
// full response sum to 1.
Recursive recursive_coefficients(double sigma) {
    const double A[2] = {1.680, -0.6803}, B[2] = {3.735, -0.2598};
    const double b[2] = {1.783, 1.723}, w[2] = {0.6318, 1.997};
    double num[2][2], den[2][3];
    for (int i = 0; i < 2; ++i) {
        const double r = std::exp(-b[i] / sigma), t = w[i] / sigma;
        num[i][0] = A[i];
        num[i][1] = r * (B[i] * std::sin(t) - A[i] * std::cos(t));
        den[i][0] = 1.0;
        den[i][1] = -2.0 * r * std::cos(t);
        den[i][2] = r * r;
    }
    double D[5] = {0, 0, 0, 0, 0}, Nm[4] = {0, 0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[i + j] += den[0][i] * den[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) Nm[i + j] += num[0][i] * den[1][j] + num[1][i] * den[0][j];
    Recursive R;
    for (int j = 0; j < 4; ++j) {
        R.num[j] = Nm[j];
        R.den[j] = D[j + 1];
    }
    R.anum[0] = Nm[1] - Nm[0] * D[1];
    R.anum[1] = Nm[2] - Nm[0] * D[2];
    R.anum[2] = Nm[3] - Nm[0] * D[3];
    R.anum[3] = -Nm[0] * D[4];
    double sn = 0, sd = 0;
    for (int j = 0; j < 4; ++j) sn += Nm[j];
    for (int j = 0; j < 5; ++j) sd += D[j];
    R.k = sd / (2.0 * sn - Nm[0] * sd);
    R.P = (int)std::ceil(14.0 * sigma);
    return R;
}

std::vector<double> spatial_taps(double sigma_s) {
    const int W = radius_of(sigma_s);
    std::vector<long double> w(2 * W + 1);
    long double sum = 0.0L;
    for (int k = -W; k <= W; ++k) {
        w[k + W] = std::exp(-(long double)k * k / (2.0L * sigma_s * sigma_s));
        sum += w[k + W];
    }
    std::vector<double> out(2 * W + 1);
    for (int i = 0; i < 2 * W + 1; ++i) out[i] = (double)(w[i] / sum);
    return out;
}

std::vector<int> plane_exponents(double mu, int N, int stack_dtype) {
    std::vector<int> k(N + 2, 0);
    if (stack_dtype != 1) return k;                 // FP16 only
    for (int n = 0; n <= N + 1; ++n) {
        double lg;                                   // log2 of the plane's largest |value|
        if (n == 0) lg = 0.0;
        else if (n <= mu) lg = 0.5 * n * std::log2(n / (M_E * mu));
        else lg = -0.5 * mu / M_LN2;
        int kn = (int)std::floor(14.0 - lg);
        if (kn < 0) kn = 0;
        if (kn > 120) kn = 120;
        k[n] = kn;
    }
    return k;
}

ParamLayout param_layout(int W, int N) {
    ParamLayout L;
    L.W = W;
    L.N = N;
    L.off_taps = 0;
    L.n_taps = 2 * W + 1 + 2 * (kTapPad - 1);
    L.off_cq = L.off_taps + ((L.n_taps + 7) & ~7);
    L.off_cp = L.off_cq + ((N + 1 + 7) & ~7);
    L.off_scale = L.off_cp + ((N + 1 + 7) & ~7);
    L.off_bd = L.off_scale + ((N + 2 + 7) & ~7);
    L.off_bf = L.off_bd + ((N + 1 + 7) & ~7);
    L.off_tf = L.off_bf + (((N + 3) / 2 + 7) & ~7);
    L.total = L.off_tf + (((2 * W + 2) / 2 + 7) & ~7);
    return L;
}

void fill_params(const ParamLayout &L, double sigma_s, double sigma_r, int stack_dtype,
                 std::vector<double> &out, int kind) {
    out.assign(L.total, 0.0);
    const std::vector<double> w = spatial_taps(sigma_s);
    for (int t = 0; t <= 2 * L.W; ++t) out[L.off_taps + t + (kTapPad - 1)] = w[t];
    const Fit &F = fit(sigma_r, L.N, kind);
    const std::vector<int> k = plane_exponents(F.mu, L.N, stack_dtype);
    for (int n = 0; n <= L.N; ++n) {
        out[L.off_cq + n] = std::ldexp(F.b[n], -k[n]);
        out[L.off_cp + n] = std::ldexp(F.b[n], -k[n + 1]);
    }
    for (int n = 0; n <= L.N + 1; ++n) out[L.off_scale + n] = std::ldexp(1.0, k[n]);
    for (int n = 0; n <= L.N; ++n) out[L.off_bd + n] = F.bd[n];
    store_float_coefficients(L, F.b, w, out);
}

}  // namespace bfgc
