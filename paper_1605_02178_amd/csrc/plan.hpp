// Host-side planning for the Gauss-Chebyshev bilateral filter: radius and
// spatial taps, the Chebyshev coefficient fit, conditioning figures, FP16
// plane scales, and the parameter block the kernels read.
#pragma once

#include <cstddef>
#include <vector>

namespace bfgc {

// Intensity range of an 8-bit image, [L, U] = [0, 255] (Section II); the
// centring of eq. (17) uses t_c = (L + U)/2 and the half range t_h = (U - L)/2.
constexpr double kTc = 127.5;
constexpr double kTh = 127.5;

// Largest register block the kernels use; the padded tap array carries this
// many zeros minus one on each side.
constexpr int kTapPad = 16;

// W = 3 sigma_s (Section I), rounded up for non-integer sigma_s.
int radius_of(double sigma_s);

// Degree rule (see bf_gc_degree_rule in bfgc.h). -1 if none <= max_degree.
int degree_rule(double sigma_r, int max_degree);

struct Fit {
    double mu = 0.0;              // t_h^2 / sigma_r^2
    std::vector<double> b;        // b_n = c_n mu^n, n = 0..N
    std::vector<double> bd;       // db_n/dmu
    double kernel_err = 0.0;      // max_y e^{-mu|y|} |p(mu y) - e^{mu y}|
    double kappa = 0.0;           // max_y e^{-mu|y|} sum |b_n| |y|^n
};

// Polynomial for the cross term exp(mu y) of the range kernel, in the
// monomial basis: kind 0 = the Chebyshev interpolant at the zeros of T_{N+1}
// (Section III), kind 1 = the Taylor polynomial of the Gauss-polynomial
// filter, b_n = mu^n / n! (Section II), kind 2 = the minimax polynomial
// (Remez exchange; Section III names it the ideal choice). Cached per
// (sigma_r, N, kind); thread safe. A minimax fit that cannot be computed has
// empty b and infinite kappa.
enum { kFitChebyshev = 0, kFitTaylor = 1, kFitMinimax = 2 };
const Fit &fit(double sigma_r, int N, int kind = kFitChebyshev);

// The Chebyshev fit of exp(mu y) on [-1, 1] for a given mu (the pivoted form
// below); cached per (mu, N).
const Fit &fit_mu(double mu, int N);

// The degree rule for a given mu. -1 if none <= max_degree.
int degree_rule_mu(double mu, int max_degree);

// Pivoted form for small sigma_r: [L, U] = [0, 255] split into K equal
// sub-ranges [lo, hi) with midpoint t and half-width h; neighbour offsets from
// t reach R = max(t - L, U - t). The cross term exp(mu y), y = s_i s_j with
// s_i = (f_i - t)/h and s_j = (f_j - t)/R, has mu = h R / sigma_r^2; the
// planes carry e^{-nu s_j^2/2} s_j^n with nu = R^2 / sigma_r^2. N: the given
// degree, or the rule at mu when N <= 0 (-1 where none <= max_degree).
struct Pivot {
    double lo, hi, t, h, R, mu, nu;
    int N;
};
std::vector<Pivot> pivot_plan(double sigma_r, int K, int N, int max_degree);

// Recursive Gaussian (the recursion Section I cites, Deriche's): impulse
// response [a0 cos(w0 n/s) + a1 sin(w0 n/s)] e^{-b0|n|/s}
// + [c0 cos(w1 n/s) + c1 sin(w1 n/s)] e^{-b1|n|/s}, as a causal recursion
// y+[i] = sum_{j<4} num[j] x[i-j] - sum_{j<4} den[j] y+[i-1-j] and an
// anticausal one y-[i] = sum_{j<4} anum[j] x[i+1+j] - sum_{j<4} den[j] y-[i+1+j];
// y = k (y+ + y-). P: samples of symmetric extension per side (14 sigma).
struct Recursive {
    double num[4], anum[4], den[4], k;
    int P;
};
Recursive recursive_coefficients(double sigma);

// Normalised spatial taps exp(-k^2/2 sigma_s^2) / sum, k = -W..W.
std::vector<double> spatial_taps(double sigma_s);

// Power-of-two exponents k_n, n = 0..N+1: plane n is stored as 2^k_n H_n.
// Non-zero only for FP16, where they keep every plane's largest value near
// 2^14 (max over |s| <= 1 of e^{-mu s^2/2}|s|^n is (n/(e mu))^{n/2} for
// n <= mu, else e^{-mu/2}).
std::vector<int> plane_exponents(double mu, int N, int stack_dtype);

// Parameter block layout (all doubles) in device memory.
struct ParamLayout {
    int W = 0, N = 0;
    int off_taps = 0, n_taps = 0;   // taps padded: index u <-> tap t = u - (kTapPad-1) - W, zero outside |t| <= W
    int off_cq = 0;                 // cq_n = b_n 2^-k_n        (weight of Hbar_n in Q), n = 0..N
    int off_cp = 0;                 // cp_n = b_n 2^-k_{n+1}    (weight of Hbar_{n+1} in P), n = 0..N
    int off_scale = 0;              // 2^k_n, n = 0..N+1
    int off_bd = 0;                 // db_n/dmu, n = 0..N (gradient with respect to sigma_r)
    int off_bf = 0;                 // b_n as floats, n = 0..N+1 with b_{N+1} = 0, two per double slot
    int off_tf = 0;                 // taps as floats, t = 0..2W (tap t - W), two per double slot
    int total = 0;                  // doubles
};
ParamLayout param_layout(int W, int N);

// Fills `out` (layout.total doubles).
void fill_params(const ParamLayout &L, double sigma_s, double sigma_r, int stack_dtype,
                 std::vector<double> &out, int kind = kFitChebyshev);

// Parameter block of one pivot (Chebyshev coefficients at mu, plane scales
// from nu).
void fill_params_pivot(const ParamLayout &L, double sigma_s, double mu, double nu, int stack_dtype,
                       std::vector<double> &out);

}  // namespace bfgc
