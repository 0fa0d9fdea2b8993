// Drives the host planner (coefficient fits, conditioning, pivots, plane
// scales, parameter blocks, recursive coefficients) over a grid of arguments
// under AddressSanitizer and UndefinedBehaviorSanitizer. Exits non-zero on a
// failed sanity check; the sanitizers abort on the first memory or UB error.
#include <cmath>
#include <cstdio>
#include <vector>

#include "plan.hpp"

using namespace bfgc;

static int fails = 0;
static void expect(bool ok, const char *what, double a, double b) {
    if (!ok) {
        std::fprintf(stderr, "check failed: %s (%g, %g)\n", what, a, b);
        ++fails;
    }
}

int main() {
    const double srs[] = {8.0, 10.0, 12.5, 20.0, 25.0, 30.0, 41.0, 60.0, 1e6};
    const double sss[] = {0.2, 1.0, 2.5, 3.0, 10.0, 16.0, 32.0};
    for (double ss : sss) {
        const std::vector<double> w = spatial_taps(ss);
        double sum = 0.0;
        for (double x : w) sum += x;
        expect((int)w.size() == 2 * radius_of(ss) + 1, "tap count", (double)w.size(), ss);
        expect(std::fabs(sum - 1.0) < 1e-12, "taps sum to 1", sum, ss);
        const Recursive R = recursive_coefficients(ss < 1.0 ? 1.0 : ss);
        expect(std::isfinite(R.k) && R.P > 0, "recursive coefficients", R.k, R.P);
    }
    for (double sr : srs) {
        const int Nr = degree_rule(sr, 320);
        expect(Nr == -1 || (Nr >= 1 && Nr <= 320), "degree rule range", Nr, sr);
        const int Ns[] = {1, 2, 8, 28, 33, 64};
        for (int N : Ns) {
            for (int kind = 0; kind < 3; ++kind) {
                if (kind == kFitMinimax && N > 40) continue;
                const Fit &F = fit(sr, N, kind);
                if (kind == kFitMinimax && F.b.empty()) continue;
                expect((int)F.b.size() == N + 1, "fit size", (double)F.b.size(), N);
                for (double b : F.b) expect(std::isfinite(b), "finite b_n", b, N);
            }
            for (int dt = 0; dt < 3; ++dt) {
                const std::vector<int> k = plane_exponents(127.5 * 127.5 / (sr * sr), N, dt);
                expect((int)k.size() == N + 2, "plane exponents", (double)k.size(), N);
            }
            for (double ss : sss) {
                const int W = radius_of(ss);
                if (W > 96) continue;
                const ParamLayout L = param_layout(W, N);
                std::vector<double> pv;
                fill_params(L, ss, sr, 1, pv, kFitChebyshev);
                expect((int)pv.size() == L.total, "parameter block size", (double)pv.size(), L.total);
            }
        }
        for (int K = 1; K <= 64; K *= 2) {
            const std::vector<Pivot> pl = pivot_plan(sr, K, 0, 320);
            expect((int)pl.size() == K, "pivot count", (double)pl.size(), K);
            for (const Pivot &p : pl) {
                if (p.N < 1) continue;
                const ParamLayout L = param_layout(radius_of(3.0), p.N);
                std::vector<double> pv;
                fill_params_pivot(L, 3.0, p.mu, p.nu, 1, pv);
                expect((int)pv.size() == L.total, "pivot parameter block", (double)pv.size(), L.total);
            }
        }
    }
    std::printf("planner driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
