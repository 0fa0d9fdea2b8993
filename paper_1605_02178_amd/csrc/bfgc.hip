// Gauss-Chebyshev bilateral filter: HIP kernels for gfx950 and the C ABI
// declared in include/bfgc.h.
//
// Forward pipeline (Section III-B procedure over the fast algorithm of
// Section II):
//   k_put_params    parameter block (taps, b_n, plane scales) into device memory
//   k_stack_build   H_n = e^{-mu s^2/2} s^n, n = 0..N+1        (eq. 6, eq. 17)
//   k_vpass         column pass of the separable Gaussian      (eq. 7)
//   k_hpass<true>   row pass fused with the combine and divide (eqs. 7-10)
// With BF_FLAG_STAGED the last step is k_hpass<false> (row pass back into the
// stack) followed by k_combine, one kernel per stage.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bfgc.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace bfgc {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_put_params(double *__restrict__ prm, unsigned *__restrict__ flag,
                                                    ParamChunk chunk) {
    for (int i = threadIdx.x; i < chunk.count; i += blockDim.x) prm[chunk.offset + i] = chunk.v[i];
    if (chunk.clear_flag && threadIdx.x == 0 && flag) *flag = 0u;
}

// One thread per pixel; planes written one after another, coalesced along rows.
template <class S>
__global__ __launch_bounds__(256) void k_stack_build(const float *__restrict__ f, int H, int Wd, int ld,
                                                      typename S::T *__restrict__ stack, long long ps, int lds,
                                                      int P, const double *__restrict__ scale, double mu,
                                                      unsigned *__restrict__ flag) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
        bool bad = false;
        if (c < Wd) {
            const float fv = f[(long long)r * ld + c];
            bad = !(fv >= 0.0f && fv <= 255.0f);
            const double s = ((double)fv - kTc) * (1.0 / kTh);           // eq. (17), scaled
            double v = exp(-0.5 * mu * s * s);                           // H_0 = e^{-mu s^2/2}
            typename S::T *dst = stack + (long long)r * lds + c;
            for (int n = 0; n < P; ++n) {
                dst[n * ps] = S::enc(v * scale[n]);
                v *= s;                                                  // H_{n+1} = H_n s
            }
        }
        if (flag && __any(bad) && (threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(bad)) - 1)
            atomicOr(flag, BF_DEVFLAG_RANGE);
    }
}

// One line of the separable Gaussian (eq. 7) for R consecutive outputs of a
// lane. The line has `len` elements; element p sits at base[p * stride], with
// p taken through the symmetric extension. Output o (o0 <= o < o0+R) is
// sum_{t=0}^{2W} w[t] x[o - W + t], w[t] the normalised tap of offset t - W.
// Input-stationary: each input position is loaded once (U loads in flight at a
// time) and FMA'd in FP64 into every output it reaches; the head and tail of
// the window touch only the outputs inside the band, so no zero tap is
// multiplied. `w` points at tap t = 0 inside the zero-padded tap array.
template <class S, int R, int U>
__device__ __forceinline__ void conv_line(const typename S::T *__restrict__ plane, int laneoff, long long stride,
                                          int o0, int len, int W, const double *__restrict__ w, double (&acc)[R]) {
    // o0, len, W, stride and plane are wave-uniform: the line position p and
    // the row pointer stay in scalar registers, each load is a uniform base
    // plus the lane's own offset.
    const int p0 = o0 - W;
    const bool interior = p0 >= 0 && o0 + R + W <= len;
    auto ld = [&](int i) -> double {
        const int p = interior ? p0 + i : mirror(p0 + i, len);
        const typename S::T *row = plane + (long long)p * stride;
        return (double)S::dec(row[laneoff]);
    };
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    const int T = 2 * W;
    if (T + 1 >= R) {
        // head: inputs 0..R-2 reach outputs r <= i
        double xh[R - 1];
#pragma unroll
        for (int i = 0; i < R - 1; ++i) xh[i] = ld(i);
        // middle: inputs R-1..T reach every output; chunks of U, the next
        // chunk's loads issued before the current chunk's FMAs
        const int nM = (T - R + 2 + U - 1) / U;
        double xa[U], xb[U];
        auto ldchunk = [&](double (&x)[U], int k) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = R - 1 + k * U + u;
                x[u] = ld(i <= T ? i : T);
            }
        };
        auto fmachunk = [&](const double (&x)[U], int k) {
            const int i0 = R - 1 + k * U;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u <= T) {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] = fma(w[i0 + u - r], x[u], acc[r]);
                }
        };
        ldchunk(xa, 0);
#pragma unroll
        for (int i = 0; i < R - 1; ++i)
#pragma unroll
            for (int r = 0; r <= i; ++r) acc[r] = fma(w[i - r], xh[i], acc[r]);
        // tail inputs T+1..T+R-1 go into xh once the last middle chunk's
        // loads are out
        auto ldtail = [&]() {
#pragma unroll
            for (int u = 0; u < R - 1; ++u) xh[u] = ld(T + 1 + u);
        };
        if (nM == 1) ldtail();
        int k = 0;
        for (; k + 1 < nM; k += 2) {
            ldchunk(xb, k + 1);
            if (k + 2 == nM) ldtail();
            fmachunk(xa, k);
            if (k + 2 < nM) {
                ldchunk(xa, k + 2);
                if (k + 3 == nM) ldtail();
            }
            fmachunk(xb, k + 1);
        }
        if (k < nM) fmachunk(xa, k);
#pragma unroll
        for (int u = 0; u < R - 1; ++u)
#pragma unroll
            for (int r = u + 1; r < R; ++r) acc[r] = fma(w[T + 1 + u - r], xh[u], acc[r]);
    } else {
        // 2W+1 < R: every input against every output; the padding zeros of
        // the tap array cover offsets outside the band.
        for (int i = 0; i < R + T; ++i) {
            const double x = ld(i);
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = fma(w[i - r], x, acc[r]);
        }
    }
}

// Stores R consecutive elements (dst 16-byte aligned when full).
template <class S, int R>
__device__ __forceinline__ void store_run(typename S::T *__restrict__ dst, const double (&v)[R], int count) {
    typedef typename S::T T;
    if (count >= R && (R * sizeof(T)) % 16 == 0) {
        T tmp[R];
#pragma unroll
        for (int q = 0; q < R; ++q) tmp[q] = S::enc(v[q]);
#pragma unroll
        for (int q = 0; q < (int)(R * sizeof(T) / 16); ++q)
            reinterpret_cast<uint4 *>(dst)[q] = reinterpret_cast<const uint4 *>(tmp)[q];
    } else {
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (q < count) dst[q] = S::enc(v[q]);
    }
}

// Column pass: lane = column, each wave R consecutive rows, one plane per
// blockIdx.z. Output written transposed, [n][col][row] with row stride ldt,
// so that the row pass reads it with consecutive lanes on consecutive rows.
template <class S, int R>
__global__ __launch_bounds__(256) void k_vpass(const typename S::T *__restrict__ in,
                                                typename S::T *__restrict__ outT, int H, int Wd, long long ps,
                                                int lds, long long pst, int ldt, const double *__restrict__ taps,
                                                int W) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = blockIdx.x * 64 + lane;
    const int r0 = (blockIdx.y * 4 + wave) * R;
    const long long n = blockIdx.z;
    if (r0 >= H) return;
    const int cl = c < Wd ? c : Wd - 1;
    double acc[R];
    conv_line<S, R, 8>(in + n * ps, cl, lds, r0, H, W, taps + (kTapPad - 1), acc);
    if (c < Wd) store_run<S, R>(outT + n * pst + (long long)c * ldt + r0, acc, H - r0);
}

// Row pass on the transposed planes: lane = row, each wave R consecutive
// columns. COMBINE = false writes each filtered plane back as [n][row][col].
// COMBINE = true visits the planes from n = N+1 down to 0 and folds them in by
// Horner's rule in s,
//   P <- P s + cp_{n-1} Hbar_n  (n >= 1),   Q <- Q s + cq_n Hbar_n  (n <= N),
// which leaves P = sum_n cp_n s^n Hbar_{n+1} and Q = sum_n cq_n s^n Hbar_n
// (eqs. 8-9); then y = t_c + t_h P/Q (eq. 10, centring undone).
template <class S, int R, bool COMBINE>
__global__ __launch_bounds__(256) void k_hpass(const typename S::T *__restrict__ inT,
                                                typename S::T *__restrict__ out_stack,
                                                const float *__restrict__ f, float *__restrict__ out,
                                                float *__restrict__ Pout, float *__restrict__ Qout, int H,
                                                int Wd, int ld, long long ps, int lds, long long pst, int ldt,
                                                int P, int N, const double *__restrict__ taps,
                                                const double *__restrict__ cq, const double *__restrict__ cp,
                                                int W) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = blockIdx.x * 64 + lane;
    const int c0 = (blockIdx.y * 4 + wave) * R;
    if (c0 >= Wd) return;
    const int rl = r < H ? r : H - 1;
    double s[R], Pa[R], Qa[R];
    if (COMBINE) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int cc = c0 + q < Wd ? c0 + q : Wd - 1;
            s[q] = ((double)f[(long long)rl * ld + cc] - kTc) * (1.0 / kTh);
            Pa[q] = 0.0;
            Qa[q] = 0.0;
        }
    }
    for (int k = 0; k < P; ++k) {
        const int n = COMBINE ? P - 1 - k : k;
        double acc[R];
        conv_line<S, R, 8>(inT + (long long)n * pst, rl, ldt, c0, Wd, W, taps + (kTapPad - 1), acc);
        if (COMBINE) {
            const double cpn = n >= 1 ? cp[n - 1] : 0.0;
            const double cqn = n <= N ? cq[n] : 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (n >= 1) Pa[q] = fma(Pa[q], s[q], cpn * acc[q]);
                if (n <= N) Qa[q] = fma(Qa[q], s[q], cqn * acc[q]);
            }
        } else if (r < H) {
            store_run<S, R>(out_stack + (long long)n * ps + (long long)r * lds + c0, acc, Wd - c0);
        }
    }
    if (COMBINE && r < H) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (c0 + q < Wd) {
                const long long o = (long long)r * ld + c0 + q;
                out[o] = (float)(kTc + kTh * (Pa[q] / Qa[q]));
                if (Pout) Pout[o] = (float)Pa[q];
                if (Qout) Qout[o] = (float)Qa[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Backward: gradients of L = sum_i ybar_i y_i with respect to f and sigma_r.
// The paper has no backward pass; this is the adjoint of the forward above.
// With P' = sum cp_n s^n Hbar_{n+1}, Q = sum cq_n s^n Hbar_n, y = t_c + t_h P'/Q:
//   alpha = dL/dP' = ybar t_h / Q,   beta = dL/dQ = -ybar t_h P' / Q^2
//   R_m   = dL/dHbar_m = alpha cp_{m-1} s^{m-1} [m >= 1] + beta cq_m s^m [m <= N]
//   dL/dH_m = G R_m (the mirrored, normalised Gaussian is a symmetric matrix)
//   dL/ds_j = alpha dP'/ds + beta dQ/ds (centre pixel's powers)
//           + sum_m (G R_m)(j) (m H_{m-1}(j) - mu H_{m+1}(j))   (dH_m/ds)
//   dL/dmu  = sum_i alpha sum bd_n s^n Hbar_{n+1} + beta sum bd_n s^n Hbar_n
//           - 1/2 sum_j sum_m (G R_m)(j) H_{m+2}(j)              (dH_m/dmu)
//   dL/df = dL/ds / t_h,  dL/dsigma_r = dL/dmu (-2 mu / sigma_r).
// ---------------------------------------------------------------------------

// Row pass of the recomputed forward, folded per pixel into six Horner sums:
// P', Q, their derivatives in s (Horner value-and-derivative), and the
// coefficient-derivative sums Pmu, Qmu. Writes alpha, beta, the direct term of
// dL/ds and the coefficient term of dL/dmu (FP64, row pitch Wd).
template <class S, int R>
__global__ __launch_bounds__(256) void k_hpass_adj(const typename S::T *__restrict__ inT,
                                                    const float *__restrict__ f, const float *__restrict__ ybar,
                                                    int H, int Wd, int ld, long long pst, int ldt, int N,
                                                    const double *__restrict__ taps, const double *__restrict__ cq,
                                                    const double *__restrict__ cp, const double *__restrict__ bd,
                                                    int W, double *__restrict__ alpha, double *__restrict__ beta,
                                                    double *__restrict__ gdir, double *__restrict__ gmu) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = blockIdx.x * 64 + lane;
    const int c0 = (blockIdx.y * 4 + wave) * R;
    if (c0 >= Wd) return;
    const int rl = r < H ? r : H - 1;
    double s[R], Pa[R], Qa[R], dP[R], dQ[R], Pm[R], Qm[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int cc = c0 + q < Wd ? c0 + q : Wd - 1;
        s[q] = ((double)f[(long long)rl * ld + cc] - kTc) * (1.0 / kTh);
        Pa[q] = Qa[q] = dP[q] = dQ[q] = Pm[q] = Qm[q] = 0.0;
    }
    const int P = N + 2;
    for (int k = 0; k < P; ++k) {
        const int n = P - 1 - k;
        double acc[R];
        conv_line<S, R, 8>(inT + (long long)n * pst, rl, ldt, c0, Wd, W, taps + (kTapPad - 1), acc);
        if (n >= 1) {
            const double cpn = cp[n - 1], bdn = bd[n - 1];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                dP[q] = fma(dP[q], s[q], Pa[q]);
                Pa[q] = fma(Pa[q], s[q], cpn * acc[q]);
                Pm[q] = fma(Pm[q], s[q], bdn * acc[q]);
            }
        }
        if (n <= N) {
            const double cqn = cq[n], bdn = bd[n];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                dQ[q] = fma(dQ[q], s[q], Qa[q]);
                Qa[q] = fma(Qa[q], s[q], cqn * acc[q]);
                Qm[q] = fma(Qm[q], s[q], bdn * acc[q]);
            }
        }
    }
    if (r < H) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (c0 + q < Wd) {
                const double yb = (double)ybar[(long long)r * ld + c0 + q];
                const double a = yb * kTh / Qa[q];
                const double b = -a * Pa[q] / Qa[q];
                const long long o = (long long)r * Wd + c0 + q;
                alpha[o] = a;
                beta[o] = b;
                gdir[o] = a * dP[q] + b * dQ[q];
                gmu[o] = a * Pm[q] + b * Qm[q];
            }
        }
    }
}

// Adjoint planes R_m(i) = alpha cp_{m-1} s^{m-1} [m >= 1] + beta cq_m s^m [m <= N].
template <class S>
__global__ __launch_bounds__(256) void k_adj_build(const float *__restrict__ f, int H, int Wd, int ld,
                                                    const double *__restrict__ alpha, const double *__restrict__ beta,
                                                    typename S::T *__restrict__ stack, long long ps, int lds, int N,
                                                    const double *__restrict__ cq, const double *__restrict__ cp) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Wd) return;
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
        const double s = ((double)f[(long long)r * ld + c] - kTc) * (1.0 / kTh);
        const long long o = (long long)r * Wd + c;
        const double a = alpha[o], b = beta[o];
        typename S::T *dst = stack + (long long)r * lds + c;
        double pw = 1.0, pm1 = 0.0;                                   // s^m, s^{m-1}
        for (int m = 0; m <= N + 1; ++m) {
            double v = 0.0;
            if (m >= 1) v = a * cp[m - 1] * pm1;
            if (m <= N) v = fma(b * cq[m], pw, v);
            dst[m * ps] = S::enc(v);
            pm1 = pw;
            pw *= s;
        }
    }
}

// Per pixel j: dL/df_j from the direct term and sum_m (G R_m)(j) dH_m/ds with
// H_m recomputed in FP64; per-block partial sums of the dL/dmu terms.
template <class S>
__global__ __launch_bounds__(256) void k_adj_neighbor(const float *__restrict__ f, int H, int Wd, int ld,
                                                       const typename S::T *__restrict__ rbar, long long ps, int lds,
                                                       int N, double mu, const double *__restrict__ gdir,
                                                       const double *__restrict__ gmu, float *__restrict__ grad_f,
                                                       double *__restrict__ partial) {
    __shared__ double red[256];
    double local = 0.0;
    const long long npx = (long long)H * Wd;
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < npx;
         o += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(o / Wd), c = (int)(o - (long long)r * Wd);
        const double s = ((double)f[(long long)r * ld + c] - kTc) * (1.0 / kTh);
        const double E = exp(-0.5 * mu * s * s);
        double hm1 = 0.0, h0 = E, h1 = E * s, h2 = E * s * s;        // H_{m-1}, H_m, H_{m+1}, H_{m+2}
        double gs = 0.0, gm = 0.0;
        const typename S::T *src = rbar + (long long)r * lds + c;
        for (int m = 0; m <= N + 1; ++m) {
            const double rb = (double)S::dec(src[m * ps]);
            gs = fma(rb, fma((double)m, hm1, -mu * h1), gs);
            gm = fma(rb, h2, gm);
            hm1 = h0;
            h0 = h1;
            h1 = h2;
            h2 *= s;
        }
        grad_f[(long long)r * ld + c] = (float)((gdir[o] + gs) * (1.0 / kTh));
        local += gmu[o] - 0.5 * gm;
    }
    red[threadIdx.x] = local;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dL/dsigma_r = (sum of the partials) (-2 mu / sigma_r); fixed summation order.
__global__ __launch_bounds__(256) void k_reduce_f64(const double *__restrict__ partial, int n, double scale,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += partial[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Staged combine: one thread per pixel, planes read in order (eqs. 8-10).
template <class S>
__global__ __launch_bounds__(256) void k_combine(const float *__restrict__ f, const typename S::T *__restrict__ stack,
                                                  int H, int Wd, int ld, long long ps, int lds, int N,
                                                  const double *__restrict__ cq, const double *__restrict__ cp,
                                                  float *__restrict__ out, float *__restrict__ Pout,
                                                  float *__restrict__ Qout) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
        if (c >= Wd) continue;
        const long long o = (long long)r * ld + c;
        const double s = ((double)f[o] - kTc) * (1.0 / kTh);
        const typename S::T *src = stack + (long long)r * lds + c;
        double Q = 0.0, Pn = 0.0, sn = 1.0;                    // sn = s^n
        for (int n = 0; n <= N; ++n) {
            Q = fma(cq[n] * sn, (double)S::dec(src[n * ps]), Q);
            Pn = fma(cp[n] * sn, (double)S::dec(src[(n + 1) * ps]), Pn);
            sn *= s;
        }
        out[o] = (float)(kTc + kTh * (Pn / Q));
        if (Pout) Pout[o] = (float)Pn;
        if (Qout) Qout[o] = (float)Q;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static bf_status fail(bf_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

static bf_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return BF_OK;
}

// Optional per-kernel timing: when enabled, every launch is bracketed by a
// pair of HIP events on its own stream; bf_profile_stop waits for them and
// sums the elapsed times per kernel name.
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
struct ProfStat {
    std::string name;
    long long count;
    double total_ms;
};
static std::mutex g_prof_mtx;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof_recs;
static std::vector<hipEvent_t> g_prof_pool;
static std::vector<ProfStat> g_prof_stats;

static hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    const char *name;
    hipStream_t stream;
    hipEvent_t a = nullptr;
    ProfScope(const char *n, hipStream_t s) : name(n), stream(s) {
        std::lock_guard<std::mutex> lock(g_prof_mtx);
        if (!g_prof_on) return;
        a = prof_event();
        if (a) (void)hipEventRecord(a, stream);
    }
    ~ProfScope() {
        if (!a) return;
        std::lock_guard<std::mutex> lock(g_prof_mtx);
        hipEvent_t b = prof_event();
        if (!b) return;
        (void)hipEventRecord(b, stream);
        g_prof_recs.push_back({name, a, b});
    }
};

constexpr int kVR = 16;   // rows per lane in k_vpass
constexpr int kHR = 16;   // columns per lane in k_hpass (staged)
constexpr int kHRC = 8;   // columns per lane in k_hpass (fused with the combine)
constexpr size_t kFlagBytes = 256;

static size_t esize(int dtype) { return dtype == BF_STACK_F32 ? 4 : 2; }
static int lds_of(int width) { return (width + 63) & ~63; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool finite_pos(double x) { return x > 0.0 && std::isfinite(x); }

static bf_status check_common(int height, int width, double sigma_s, double sigma_r, int N, int dtype) {
    if (height < 0 || width < 0) return fail(BF_ERR_INVALID_ARG, "height and width must be >= 0");
    if (!finite_pos(sigma_s)) return fail(BF_ERR_INVALID_ARG, "sigma_s must be positive and finite");
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (N < 1 || N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N out of [1, BF_MAX_DEGREE]");
    if (dtype < BF_STACK_F32 || dtype > BF_STACK_BF16) return fail(BF_ERR_INVALID_ARG, "unknown stack dtype");
    if (radius_of(sigma_s) > BF_MAX_RADIUS) return fail(BF_ERR_UNSUPPORTED, "radius ceil(3 sigma_s) above BF_MAX_RADIUS");
    if ((long long)height * lds_of(width) > (1LL << 40)) return fail(BF_ERR_UNSUPPORTED, "image too large");
    return BF_OK;
}

// Storage rounding unit of each stack type.
static double unit_roundoff(int dtype) {
    return dtype == BF_STACK_F32 ? std::ldexp(1.0, -24) : dtype == BF_STACK_F16 ? std::ldexp(1.0, -11)
                                                                                : std::ldexp(1.0, -8);
}

static bf_status check_conditioning(double sigma_r, int N, int dtype, unsigned flags) {
    if (flags & BF_FLAG_ALLOW_ILL_CONDITIONED) return BF_OK;
    const Fit &F = fit(sigma_r, N);
    if (!std::isfinite(F.kappa) || F.kappa * unit_roundoff(dtype) > 1e-2) {
        char buf[200];
        snprintf(buf, sizeof buf, "ill-conditioned: kappa=%.3g times the stack rounding unit exceeds 1e-2 "
                                  "(sigma_r=%g, N=%d)", F.kappa, sigma_r, N);
        return fail(BF_ERR_ILL_CONDITIONED, buf);
    }
    return BF_OK;
}

static bf_status upload_params(double *prm, unsigned *flag, double sigma_s, double sigma_r, int N, int dtype,
                               hipStream_t stream, ParamLayout *Lout) {
    const int W = radius_of(sigma_s);
    ParamLayout L = param_layout(W, N);
    std::vector<double> host;
    fill_params(L, sigma_s, sigma_r, dtype, host);
    ParamChunk ch;
    int off = 0;
    do {
        std::memset(&ch, 0, sizeof ch);
        ch.offset = off;
        ch.count = std::min(400, L.total - off);
        ch.clear_flag = off == 0 ? 1 : 0;
        for (int i = 0; i < ch.count; ++i) ch.v[i] = host[off + i];
        ProfScope prof_("k_put_params", stream);
        hipLaunchKernelGGL(k_put_params, dim3(1), dim3(256), 0, stream, prm, flag, ch);
        off += 400;
    } while (off < L.total);
    *Lout = L;
    return check_launch("k_put_params");
}

struct Plan {
    int W = 0, N = 0, P = 0;
    double mu = 0.0;
    ParamLayout L;
};

template <class S>
static bf_status launch_build(const float *f, int H, int Wd, int ld, void *stack, long long ps, int lds, int P,
                              const double *prm, const ParamLayout &L, double mu, unsigned *flag,
                              hipStream_t stream) {
    dim3 grid((Wd + 255) / 256, std::min(H, 65535));
    ProfScope prof_("k_stack_build", stream);
    hipLaunchKernelGGL(k_stack_build<S>, grid, dim3(256), 0, stream, f, H, Wd, ld,
                       (typename S::T *)stack, ps, lds, P, prm + L.off_scale, mu, flag);
    return check_launch("k_stack_build");
}

static int ldt_of(int height) { return (height + 63) & ~63; }

template <class S>
static bf_status launch_vpass(const void *stack, void *tmpT, int planes, int H, int Wd, long long ps, int lds,
                              long long pst, int ldt, const double *prm, const ParamLayout &L, hipStream_t stream) {
    dim3 gv((Wd + 63) / 64, (H + 4 * kVR - 1) / (4 * kVR), planes);
    ProfScope prof_("k_vpass", stream);
    hipLaunchKernelGGL((k_vpass<S, kVR>), gv, dim3(256), 0, stream, (const typename S::T *)stack,
                       (typename S::T *)tmpT, H, Wd, ps, lds, pst, ldt, prm + L.off_taps, L.W);
    return check_launch("k_vpass");
}

template <class S>
static bf_status launch_gauss(void *stack, void *tmpT, int planes, int H, int Wd, long long ps, int lds,
                              const double *prm, const ParamLayout &L, hipStream_t stream) {
    const int ldt = ldt_of(H);
    const long long pst = (long long)Wd * ldt;
    bf_status st = launch_vpass<S>(stack, tmpT, planes, H, Wd, ps, lds, pst, ldt, prm, L, stream);
    if (st != BF_OK) return st;
    dim3 gh((H + 63) / 64, (Wd + 4 * kHR - 1) / (4 * kHR));
    ProfScope prof_("k_hpass", stream);
    hipLaunchKernelGGL((k_hpass<S, kHR, false>), gh, dim3(256), 0, stream, (const typename S::T *)tmpT,
                       (typename S::T *)stack, (const float *)nullptr, (float *)nullptr, (float *)nullptr,
                       (float *)nullptr, H, Wd, 0, ps, lds, pst, ldt, planes, 0, prm + L.off_taps,
                       prm + L.off_cq, prm + L.off_cp, L.W);
    return check_launch("k_hpass");
}

template <class S>
static bf_status launch_hpass_combine(const void *tmpT, const float *f, float *out, float *Pout, float *Qout, int H,
                                      int Wd, int ld, long long pst, int ldt, const double *prm,
                                      const ParamLayout &L, hipStream_t stream) {
    dim3 gh((H + 63) / 64, (Wd + 4 * kHRC - 1) / (4 * kHRC));
    ProfScope prof_("k_hpass_combine", stream);
    hipLaunchKernelGGL((k_hpass<S, kHRC, true>), gh, dim3(256), 0, stream, (const typename S::T *)tmpT,
                       (typename S::T *)nullptr, f, out, Pout, Qout, H, Wd, ld, 0LL, 0, pst, ldt, L.N + 2, L.N,
                       prm + L.off_taps, prm + L.off_cq, prm + L.off_cp, L.W);
    return check_launch("k_hpass(combine)");
}

template <class S>
static bf_status launch_combine(const float *f, const void *stack, int H, int Wd, int ld, long long ps, int lds,
                                const double *prm, const ParamLayout &L, float *out, float *Pout, float *Qout,
                                hipStream_t stream) {
    dim3 grid((Wd + 255) / 256, std::min(H, 65535));
    ProfScope prof_("k_combine", stream);
    hipLaunchKernelGGL(k_combine<S>, grid, dim3(256), 0, stream, f, (const typename S::T *)stack, H, Wd, ld, ps,
                       lds, L.N, prm + L.off_cq, prm + L.off_cp, out, Pout, Qout);
    return check_launch("k_combine");
}

template <class S>
static bf_status run_forward(const float *f, float *out, int H, int Wd, int ld, double sigma_s, double sigma_r,
                             int N, int dtype, unsigned flags, char *ws, hipStream_t stream) {
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, dtype, stream, &L);
    if (st != BF_OK) return st;
    const int lds = lds_of(Wd);
    const long long ps = (long long)H * lds;
    const int P = N + 2;
    char *stackA = ws + kFlagBytes + align256(sizeof(double) * L.total);
    char *stackB = stackA + align256((size_t)P * ps * sizeof(typename S::T));
    const double mu = fit(sigma_r, N).mu;
    if ((st = launch_build<S>(f, H, Wd, ld, stackA, ps, lds, P, prm, L, mu, flag, stream)) != BF_OK) return st;
    if (flags & BF_FLAG_STAGED) {
        if ((st = launch_gauss<S>(stackA, stackB, P, H, Wd, ps, lds, prm, L, stream)) != BF_OK) return st;
        return launch_combine<S>(f, stackA, H, Wd, ld, ps, lds, prm, L, out, nullptr, nullptr, stream);
    }
    const int ldt = ldt_of(H);
    const long long pst = (long long)Wd * ldt;
    if ((st = launch_vpass<S>(stackA, stackB, P, H, Wd, ps, lds, pst, ldt, prm, L, stream)) != BF_OK) return st;
    return launch_hpass_combine<S>(stackB, f, out, nullptr, nullptr, H, Wd, ld, pst, ldt, prm, L, stream);
}

constexpr int kAdjR = 4;            // columns per lane in k_hpass_adj
constexpr int kNeighborBlocks = 2048;

struct BwdLayout {
    size_t params, stackA, stackB, perpx, partial, total;
};

static BwdLayout bwd_layout(int H, int Wd, double sigma_s, int N) {
    BwdLayout B;
    const size_t P = (size_t)N + 2;
    B.params = align256(sizeof(double) * (size_t)param_layout(radius_of(sigma_s), N).total);
    B.stackA = align256(P * H * lds_of(Wd) * sizeof(double));
    B.stackB = align256(P * Wd * ldt_of(H) * sizeof(double));
    B.perpx = align256((size_t)H * Wd * sizeof(double));
    B.partial = align256(kNeighborBlocks * sizeof(double));
    B.total = kFlagBytes + B.params + B.stackA + B.stackB + 4 * B.perpx + B.partial;
    return B;
}

static bf_status run_backward(const float *f, const float *ybar, float *grad_f, double *grad_sr, int H, int Wd,
                              int ld, double sigma_s, double sigma_r, int N, char *ws, hipStream_t stream) {
    const BwdLayout B = bwd_layout(H, Wd, sigma_s, N);
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, BF_STACK_F32, stream, &L);
    if (st != BF_OK) return st;
    char *stackA = ws + kFlagBytes + B.params;
    char *stackB = stackA + B.stackA;
    double *alpha = (double *)(stackB + B.stackB);
    double *beta = (double *)((char *)alpha + B.perpx);
    double *gdir = (double *)((char *)beta + B.perpx);
    double *gmu = (double *)((char *)gdir + B.perpx);
    double *partial = (double *)((char *)gmu + B.perpx);
    const int P = N + 2;
    const int lds = lds_of(Wd), ldt = ldt_of(H);
    const long long ps = (long long)H * lds, pst = (long long)Wd * ldt;
    const double mu = fit(sigma_r, N).mu;
    // Recompute the forward stack and its column pass in FP64: the derivative
    // sums below cancel strongly, and FP32 planes cost them three to four
    // digits (measured against the FP64 gradient oracle).
    if ((st = launch_build<StF64>(f, H, Wd, ld, stackA, ps, lds, P, prm, L, mu, flag, stream)) != BF_OK) return st;
    if ((st = launch_vpass<StF64>(stackA, stackB, P, H, Wd, ps, lds, pst, ldt, prm, L, stream)) != BF_OK) return st;
    {
        dim3 g((H + 63) / 64, (Wd + 4 * kAdjR - 1) / (4 * kAdjR));
        ProfScope prof_("k_hpass_adj", stream);
        hipLaunchKernelGGL((k_hpass_adj<StF64, kAdjR>), g, dim3(256), 0, stream, (const double *)stackB, f, ybar, H,
                           Wd, ld, pst, ldt, N, prm + L.off_taps, prm + L.off_cq, prm + L.off_cp, prm + L.off_bd,
                           L.W, alpha, beta, gdir, gmu);
        if ((st = check_launch("k_hpass_adj")) != BF_OK) return st;
    }
    {
        dim3 g((Wd + 255) / 256, std::min(H, 65535));
        ProfScope prof_("k_adj_build", stream);
        hipLaunchKernelGGL(k_adj_build<StF64>, g, dim3(256), 0, stream, f, H, Wd, ld, (const double *)alpha,
                           (const double *)beta, (double *)stackA, ps, lds, N, prm + L.off_cq, prm + L.off_cp);
        if ((st = check_launch("k_adj_build")) != BF_OK) return st;
    }
    if ((st = launch_gauss<StF64>(stackA, stackB, P, H, Wd, ps, lds, prm, L, stream)) != BF_OK) return st;
    const long long npx = (long long)H * Wd;
    const int nb = (int)std::min<long long>(kNeighborBlocks, (npx + 255) / 256);
    {
        ProfScope prof_("k_adj_neighbor", stream);
        hipLaunchKernelGGL(k_adj_neighbor<StF64>, dim3(nb), dim3(256), 0, stream, f, H, Wd, ld,
                           (const double *)stackA, ps, lds, N, mu, (const double *)gdir, (const double *)gmu,
                           grad_f, partial);
        if ((st = check_launch("k_adj_neighbor")) != BF_OK) return st;
    }
    {
        ProfScope prof_("k_reduce_f64", stream);
        hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, stream, (const double *)partial, nb,
                           -2.0 * mu / sigma_r, grad_sr);
        return check_launch("k_reduce_f64");
    }
}

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

}  // namespace bfgc

using namespace bfgc;

extern "C" {

int bf_gc_degree_rule(double sigma_r) { return degree_rule(sigma_r, BF_MAX_DEGREE); }

bf_status bf_gc_coefficients(double sigma_r, int N, double *b_out, double *mu_out) {
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (N < 1 || N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N out of [1, BF_MAX_DEGREE]");
    if (!b_out) return fail(BF_ERR_INVALID_ARG, "b_out is null");
    const Fit &F = fit(sigma_r, N);
    for (int n = 0; n <= N; ++n) b_out[n] = F.b[n];
    if (mu_out) *mu_out = F.mu;
    return BF_OK;
}

bf_status bf_gc_query(double sigma_r, int N, int stack_dtype, double *kernel_err, double *kappa) {
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (N < 1 || N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N out of [1, BF_MAX_DEGREE]");
    if (stack_dtype < BF_STACK_F32 || stack_dtype > BF_STACK_BF16) return fail(BF_ERR_INVALID_ARG, "unknown stack dtype");
    const Fit &F = fit(sigma_r, N);
    if (kernel_err) *kernel_err = F.kernel_err;
    if (kappa) *kappa = F.kappa;
    return BF_OK;
}

size_t bf_gc_param_bytes(double sigma_s, int N) {
    if (!finite_pos(sigma_s) || N < 1 || N > BF_MAX_DEGREE || radius_of(sigma_s) > BF_MAX_RADIUS) return 0;
    return sizeof(double) * (size_t)param_layout(radius_of(sigma_s), N).total;
}

size_t bf_gc_workspace_bytes(int height, int width, double sigma_s, int N, int stack_dtype, int for_backward) {
    if (check_common(height, width, sigma_s, 30.0, N, stack_dtype) != BF_OK) return 0;
    if (for_backward) return bwd_layout(height, width, sigma_s, N).total;
    const size_t planesA = (size_t)(N + 2) * height * lds_of(width) * esize(stack_dtype);
    const size_t planesB = (size_t)(N + 2) * width * ldt_of(height) * esize(stack_dtype);
    return kFlagBytes + align256(bf_gc_param_bytes(sigma_s, N)) + align256(planesA) + align256(planesB);
}

bf_status bf_gc_forward(const float *f, float *out, int height, int width, int ld, double sigma_s,
                        double sigma_r, int N, int stack_dtype, unsigned flags, void *ws, size_t ws_bytes,
                        void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (height == 0 || width == 0) return BF_OK;
    if (!f || !out) return fail(BF_ERR_INVALID_ARG, "f and out must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const size_t img = ((size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, img, out, img)) return fail(BF_ERR_INVALID_ARG, "out overlaps f");
    if ((st = check_conditioning(sigma_r, N, stack_dtype, flags)) != BF_OK) return st;
    const size_t need = bf_gc_workspace_bytes(height, width, sigma_s, N, stack_dtype, 0);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null, misaligned or too small");
    hipStream_t s = (hipStream_t)stream;
    switch (stack_dtype) {
    case BF_STACK_F32: return run_forward<StF32>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    case BF_STACK_F16: return run_forward<StF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    default: return run_forward<StBF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    }
}

bf_status bf_gc_backward(const float *f, const float *grad_out, float *grad_f, double *grad_sigma_r, int height,
                         int width, int ld, double sigma_s, double sigma_r, int N, int stack_dtype, unsigned flags,
                         void *ws, size_t ws_bytes, void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (stack_dtype != BF_STACK_F32) return fail(BF_ERR_UNSUPPORTED, "the backward runs with an FP32 stack only");
    if (!grad_sigma_r) return fail(BF_ERR_INVALID_ARG, "grad_sigma_r must be non-null");
    if (height == 0 || width == 0) {   // empty image: dL/dsigma_r = 0 (a kernel, so the call can be graph-captured)
        hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, (hipStream_t)stream, (const double *)nullptr, 0, 0.0,
                           grad_sigma_r);
        return check_launch("k_reduce_f64");
    }
    if (!f || !grad_out || !grad_f) return fail(BF_ERR_INVALID_ARG, "f, grad_out and grad_f must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const size_t img = ((size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, img, grad_f, img) || overlaps(grad_out, img, grad_f, img))
        return fail(BF_ERR_INVALID_ARG, "grad_f overlaps f or grad_out");
    if ((st = check_conditioning(sigma_r, N, stack_dtype, flags)) != BF_OK) return st;
    const size_t need = bf_gc_workspace_bytes(height, width, sigma_s, N, stack_dtype, 1);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null, misaligned or too small");
    return run_backward(f, grad_out, grad_f, grad_sigma_r, height, width, ld, sigma_s, sigma_r, N, (char *)ws,
                        (hipStream_t)stream);
}

bf_status bf_gc_plane_scales(double sigma_r, int N, int stack_dtype, int *k_out) {
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (N < 1 || N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N out of [1, BF_MAX_DEGREE]");
    if (!k_out) return fail(BF_ERR_INVALID_ARG, "k_out is null");
    const std::vector<int> k = plane_exponents(fit(sigma_r, N).mu, N, stack_dtype);
    for (int n = 0; n <= N + 1; ++n) k_out[n] = k[n];
    return BF_OK;
}

static bf_status check_stack_args(const void *stack, int height, int width, long long plane_stride, int lds,
                                  int planes, const void *prm) {
    if (!stack || !prm) return fail(BF_ERR_INVALID_ARG, "stack and prm must be non-null");
    if (lds < width) return fail(BF_ERR_INVALID_ARG, "lds must be >= width");
    if (plane_stride < (long long)height * lds) return fail(BF_ERR_INVALID_ARG, "plane_stride < height * lds");
    if (planes < 1) return fail(BF_ERR_INVALID_ARG, "planes must be >= 1");
    if ((lds & 15) || (plane_stride & 15) || ((uintptr_t)stack & 15))
        return fail(BF_ERR_INVALID_ARG, "stack must be 16-byte aligned with lds and plane_stride multiples of 16");
    return BF_OK;
}

bf_status bf_gc_stack_build(const float *f, int height, int width, int ld, double sigma_r, int N, int stack_dtype,
                            void *stack, long long plane_stride, int lds, unsigned *devflag, void *prm,
                            void *stream) {
    bf_status st = check_common(height, width, 1.0, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (height == 0 || width == 0) return BF_OK;
    if (!f) return fail(BF_ERR_INVALID_ARG, "f must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    if ((st = check_stack_args(stack, height, width, plane_stride, lds, N + 2, prm)) != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    ParamLayout L;
    if ((st = upload_params((double *)prm, devflag, 1.0, sigma_r, N, stack_dtype, s, &L)) != BF_OK) return st;
    const double mu = fit(sigma_r, N).mu;
    switch (stack_dtype) {
    case BF_STACK_F32: return launch_build<StF32>(f, height, width, ld, stack, plane_stride, lds, N + 2, (double *)prm, L, mu, devflag, s);
    case BF_STACK_F16: return launch_build<StF16>(f, height, width, ld, stack, plane_stride, lds, N + 2, (double *)prm, L, mu, devflag, s);
    default: return launch_build<StBF16>(f, height, width, ld, stack, plane_stride, lds, N + 2, (double *)prm, L, mu, devflag, s);
    }
}

size_t bf_gc_gauss_tmp_bytes(int planes, int height, int width, int stack_dtype) {
    if (planes < 1 || height < 0 || width < 0 || stack_dtype < BF_STACK_F32 || stack_dtype > BF_STACK_BF16) return 0;
    return (size_t)planes * width * ldt_of(height) * esize(stack_dtype);
}

bf_status bf_gc_gauss_planes(void *stack, void *tmp, size_t tmp_bytes, int planes, int height, int width,
                             long long plane_stride, int lds, double sigma_s, int stack_dtype, void *prm,
                             void *stream) {
    bf_status st = check_common(height, width, sigma_s, 30.0, 1, stack_dtype);
    if (st != BF_OK) return st;
    if (height == 0 || width == 0) return BF_OK;
    if ((st = check_stack_args(stack, height, width, plane_stride, lds, planes, prm)) != BF_OK) return st;
    if (!tmp || tmp_bytes < bf_gc_gauss_tmp_bytes(planes, height, width, stack_dtype) || ((uintptr_t)tmp & 15))
        return fail(BF_ERR_WORKSPACE, "tmp null, not 16-byte aligned or smaller than bf_gc_gauss_tmp_bytes()");
    hipStream_t s = (hipStream_t)stream;
    ParamLayout L;
    if ((st = upload_params((double *)prm, nullptr, sigma_s, 30.0, 1, stack_dtype, s, &L)) != BF_OK) return st;
    switch (stack_dtype) {
    case BF_STACK_F32: return launch_gauss<StF32>(stack, tmp, planes, height, width, plane_stride, lds, (double *)prm, L, s);
    case BF_STACK_F16: return launch_gauss<StF16>(stack, tmp, planes, height, width, plane_stride, lds, (double *)prm, L, s);
    default: return launch_gauss<StBF16>(stack, tmp, planes, height, width, plane_stride, lds, (double *)prm, L, s);
    }
}

bf_status bf_gc_combine(const float *f, const void *stack, int height, int width, int ld, long long plane_stride,
                        int lds, double sigma_r, int N, int stack_dtype, float *out, float *P_out, float *Q_out,
                        void *prm, void *stream) {
    bf_status st = check_common(height, width, 1.0, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (height == 0 || width == 0) return BF_OK;
    if (!f || !out) return fail(BF_ERR_INVALID_ARG, "f and out must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    if ((st = check_stack_args(stack, height, width, plane_stride, lds, N + 2, prm)) != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    ParamLayout L;
    if ((st = upload_params((double *)prm, nullptr, 1.0, sigma_r, N, stack_dtype, s, &L)) != BF_OK) return st;
    switch (stack_dtype) {
    case BF_STACK_F32: return launch_combine<StF32>(f, stack, height, width, ld, plane_stride, lds, (double *)prm, L, out, P_out, Q_out, s);
    case BF_STACK_F16: return launch_combine<StF16>(f, stack, height, width, ld, plane_stride, lds, (double *)prm, L, out, P_out, Q_out, s);
    default: return launch_combine<StBF16>(f, stack, height, width, ld, plane_stride, lds, (double *)prm, L, out, P_out, Q_out, s);
    }
}

bf_status bf_gc_read_flags(const void *ws, unsigned *flags_out, void *stream) {
    if (!ws || !flags_out) return fail(BF_ERR_INVALID_ARG, "ws and flags_out must be non-null");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(flags_out, ws, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string("bf_gc_read_flags: ") + hipGetErrorString(e));
    return BF_OK;
}

bf_status bf_profile_start(void) {
    std::lock_guard<std::mutex> lock(g_prof_mtx);
    g_prof_stats.clear();
    g_prof_on = true;
    return BF_OK;
}

bf_status bf_profile_stop(void *stream) {
    (void)stream;
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lock(g_prof_mtx);
        g_prof_on = false;
        recs.swap(g_prof_recs);
    }
    bf_status st = BF_OK;
    std::vector<ProfStat> stats;
    for (const ProfRec &r : recs) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            st = fail(BF_ERR_DEVICE, std::string("bf_profile_stop: ") + hipGetErrorString(e));
            continue;
        }
        bool found = false;
        for (ProfStat &p : stats)
            if (p.name == r.name) {
                p.count += 1;
                p.total_ms += ms;
                found = true;
            }
        if (!found) stats.push_back({r.name, 1, (double)ms});
    }
    std::lock_guard<std::mutex> lock(g_prof_mtx);
    for (const ProfRec &r : recs) {
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_stats = stats;
    return st;
}

int bf_profile_count(void) {
    std::lock_guard<std::mutex> lock(g_prof_mtx);
    return (int)g_prof_stats.size();
}

bf_status bf_profile_entry(int i, char *name, int name_len, long long *count, double *total_ms) {
    std::lock_guard<std::mutex> lock(g_prof_mtx);
    if (i < 0 || i >= (int)g_prof_stats.size() || !name || name_len < 1 || !count || !total_ms)
        return fail(BF_ERR_INVALID_ARG, "bf_profile_entry: bad index or null output");
    snprintf(name, name_len, "%s", g_prof_stats[i].name.c_str());
    *count = g_prof_stats[i].count;
    *total_ms = g_prof_stats[i].total_ms;
    return BF_OK;
}

const char *bf_status_string(int status) {
    switch (status) {
    case BF_OK: return "BF_OK";
    case BF_ERR_INVALID_ARG: return "BF_ERR_INVALID_ARG";
    case BF_ERR_UNSUPPORTED: return "BF_ERR_UNSUPPORTED";
    case BF_ERR_ILL_CONDITIONED: return "BF_ERR_ILL_CONDITIONED";
    case BF_ERR_WORKSPACE: return "BF_ERR_WORKSPACE";
    case BF_ERR_DEVICE: return "BF_ERR_DEVICE";
    default: return "BF_UNKNOWN_STATUS";
    }
}

const char *bf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
