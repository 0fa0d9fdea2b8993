// Device kernels of the Gauss-Chebyshev bilateral filter for gfx950 (CDNA4).
//
// Data layout in HBM:
//   image f, output y: FP32, row-major, row stride ld;
//   stack: N+2 planes, plane-major [n][row][col], row stride lds (a multiple
//          of 64 elements), plane stride ps = height * lds elements;
//   parameter block: doubles (see plan.hpp ParamLayout), read through the
//          scalar cache (every index the kernels use is wave-uniform).
//
// Arithmetic: the power chain s^n, the convolution sums and the combine run in
// FP64; the stack itself is stored in FP32, FP16 (scaled by 2^k_n) or BF16.
// Rounding of the stored planes is then the only per-plane error.
//
// Every kernel is a thin wrapper over a tile function (one 256-thread block's
// share of the work); the persistent batched kernel runs the same tile
// functions, so a batch reproduces the per-image results bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfgc.h"
#include "plan.hpp"

namespace bfgc {

// Stack element encodings.
struct StF32 {
    typedef float T;
    static __device__ __forceinline__ T enc(double v) { return (float)v; }
    static __device__ __forceinline__ float dec(T x) { return x; }
};
struct StF64 {
    typedef double T;
    static __device__ __forceinline__ T enc(double v) { return v; }
    static __device__ __forceinline__ double dec(T x) { return x; }
};
struct StF16 {
    typedef _Float16 T;
    static __device__ __forceinline__ T enc(double v) { return (_Float16)(float)v; }
    static __device__ __forceinline__ float dec(T x) { return (float)x; }
};
struct StBF16 {
    typedef uint16_t T;
    static __device__ __forceinline__ T enc(double v) {
        uint32_t u = __float_as_uint((float)v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // keep NaN a NaN
        u += 0x7fffu + ((u >> 16) & 1u);                                              // round to nearest even
        return (uint16_t)(u >> 16);
    }
    static __device__ __forceinline__ float dec(T x) { return __uint_as_float((uint32_t)x << 16); }
};

// Symmetric extension of a line of length M (half-sample mirror, period 2M).
__device__ __forceinline__ int mirror(int i, int M) {
    if ((unsigned)i < (unsigned)M) return i;
    int p = i % (2 * M);
    if (p < 0) p += 2 * M;
    return p >= M ? 2 * M - 1 - p : p;
}

struct ParamChunk {
    int offset;
    int count;
    int clear_flag;
    int pad_;
    double v[400];
};


// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_put_params(double *__restrict__ prm, unsigned *__restrict__ flag,
                                                    ParamChunk chunk) {
    for (int i = threadIdx.x; i < chunk.count; i += blockDim.x) prm[chunk.offset + i] = chunk.v[i];
    if (chunk.clear_flag && threadIdx.x == 0 && flag) *flag = 0u;
}

// Centring of the expansion (eq. 17) and the output mask. The plain filter
// centres every pixel at t_c = (L+U)/2 with half range t_h; the pivoted form
// (small sigma_r) runs once per sub-range k with its midpoint t_k, scales the
// neighbour offsets by 1/R_k and the centre offsets by 1/h, and keeps the
// output only where the centre value lies in the sub-range.
struct Centring {
    double tc;         // centre t
    double inv_s;      // build: s_j = (f_j - tc) inv_s
    double inv_c;      // combine: s_i = (f_i - tc) inv_c
    double out_scale;  // y = tc + out_scale P / Q
    float lo, hi;      // sub-range of the centre value
    int mask;          // 0: store every output; 1: lo <= f_i < hi; 2: f_i < hi; 3: !(f_i < lo)
};
__host__ __device__ inline Centring plain_centring() {
    return Centring{kTc, 1.0 / kTh, 1.0 / kTh, kTh, 0.0f, 0.0f, 0};
}
__device__ __forceinline__ bool centring_keeps(const Centring &C, float fi) {
    return C.mask == 0 || (C.mask == 1 && fi >= C.lo && fi < C.hi) || (C.mask == 2 && fi < C.hi) ||
           (C.mask == 3 && !(fi < C.lo));
}

constexpr int kBuildRows = 8;   // rows per block in the stack build

// Stack build for rows [r0, r1) of the 256-column block cb: one thread per
// pixel, planes written one after another, coalesced along rows.
template <class S>
__device__ __forceinline__ void build_tile(const float *__restrict__ f, int H, int Wd, int ld,
                                           typename S::T *__restrict__ stack, long long ps, int lds, int P,
                                           const double *__restrict__ scale, double mu, unsigned *__restrict__ flag,
                                           int cb, int r0, int r1, const Centring &C) {
    const int c = cb * 256 + threadIdx.x;
    for (int r = r0; r < r1; ++r) {
        bool bad = false;
        if (c < Wd) {
            const float fv = f[(long long)r * ld + c];
            bad = !(fv >= 0.0f && fv <= 255.0f);
            const double s = ((double)fv - C.tc) * C.inv_s;               // eq. (17), scaled
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

template <class S>
__global__ __launch_bounds__(256) void k_stack_build(const float *__restrict__ f, int H, int Wd, int ld,
                                                      typename S::T *__restrict__ stack, long long ps, int lds,
                                                      int P, const double *__restrict__ scale, double mu,
                                                      unsigned *__restrict__ flag, Centring C) {
    const int r0 = blockIdx.y * kBuildRows;
    build_tile<S>(f, H, Wd, ld, stack, ps, lds, P, scale, mu, flag, blockIdx.x, r0, min(H, r0 + kBuildRows), C);
}

// One line of the separable Gaussian (eq. 7) for R consecutive outputs of a
// lane. The line has `len` elements; element p sits at base[p * stride], with
// p taken through the symmetric extension. Output o (o0 <= o < o0+R) is
// sum_{t=0}^{2W} w[t] x[o - W + t], w[t] the normalised tap of offset t - W.
// Input-stationary: each input position is loaded once (U loads in flight at a
// time) and FMA'd in FP64 into every output it reaches; the head and tail of
// the window touch only the outputs inside the band, so no zero tap is
// multiplied. `w` points at tap t = 0 inside the zero-padded tap array.
// The accumulation itself, with ld(i) giving input p0 + i (already through
// the symmetric extension): conv_line reads the plane in global memory, the
// LDS-staged passes read their tile, in the same FMA order.
template <int R, int U, class LD>
__device__ __forceinline__ void conv_core(LD ld, int W, const double *__restrict__ w, double (&acc)[R]) {
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
    conv_core<R, U>(ld, W, w, acc);
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

// Column pass: lane = column, each wave R consecutive rows; the block covers
// columns [64 bx, 64 bx + 64) and rows [4R by, 4R by + 4R) of plane n. Output
// written transposed, [n][col][row] with row stride ldt, so that the row pass
// reads it with consecutive lanes on consecutive rows.
template <class S, int R>
__device__ __forceinline__ void vpass_tile(const typename S::T *__restrict__ in, typename S::T *__restrict__ outT,
                                           int H, int Wd, long long ps, int lds, long long pst, int ldt,
                                           const double *__restrict__ taps, int W, int bx, int by, int n) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = bx * 64 + lane;
    const int r0 = (by * 4 + wave) * R;
    if (r0 >= H) return;
    const int cl = c < Wd ? c : Wd - 1;
    double acc[R];
    conv_line<S, R, 8>(in + (long long)n * ps, cl, lds, r0, H, W, taps + (kTapPad - 1), acc);
    if (c < Wd) store_run<S, R>(outT + (long long)n * pst + (long long)c * ldt + r0, acc, H - r0);
}

template <class S, int R>
__global__ __launch_bounds__(256) void k_vpass(const typename S::T *__restrict__ in,
                                                typename S::T *__restrict__ outT, int H, int Wd, long long ps,
                                                int lds, long long pst, int ldt, const double *__restrict__ taps,
                                                int W) {
    vpass_tile<S, R>(in, outT, H, Wd, ps, lds, pst, ldt, taps, W, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Row pass on the transposed planes: lane = row, each wave R consecutive
// columns. COMBINE = false writes each filtered plane back as [n][row][col].
// COMBINE = true visits the planes from n = N+1 down to 0 and folds them in by
// Horner's rule in s,
//   P <- P s + cp_{n-1} Hbar_n  (n >= 1),   Q <- Q s + cq_n Hbar_n  (n <= N),
// which leaves P = sum_n cp_n s^n Hbar_{n+1} and Q = sum_n cq_n s^n Hbar_n
// (eqs. 8-9); then y = t_c + t_h P/Q (eq. 10, centring undone).
template <class S, int R, bool COMBINE>
__device__ __forceinline__ void hpass_tile(const typename S::T *__restrict__ inT,
                                           typename S::T *__restrict__ out_stack, const float *__restrict__ f,
                                           float *__restrict__ out, float *__restrict__ Pout,
                                           float *__restrict__ Qout, int H, int Wd, int ld, long long ps, int lds,
                                           long long pst, int ldt, int P, int N, const double *__restrict__ taps,
                                           const double *__restrict__ cq, const double *__restrict__ cp, int W,
                                           int bx, int by, const Centring &C) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = bx * 64 + lane;
    const int c0 = (by * 4 + wave) * R;
    if (c0 >= Wd) return;
    const int rl = r < H ? r : H - 1;
    double s[R], Pa[R], Qa[R];
    if (COMBINE) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int cc = c0 + q < Wd ? c0 + q : Wd - 1;
            s[q] = ((double)f[(long long)rl * ld + cc] - C.tc) * C.inv_c;
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
                if (C.mask != 0 && !centring_keeps(C, f[o])) continue;
                out[o] = (float)(C.tc + C.out_scale * (Pa[q] / Qa[q]));
                if (Pout) Pout[o] = (float)Pa[q];
                if (Qout) Qout[o] = (float)Qa[q];
            }
        }
    }
}

template <class S, int R, bool COMBINE>
__global__ __launch_bounds__(256) void k_hpass(const typename S::T *__restrict__ inT,
                                                typename S::T *__restrict__ out_stack,
                                                const float *__restrict__ f, float *__restrict__ out,
                                                float *__restrict__ Pout, float *__restrict__ Qout, int H,
                                                int Wd, int ld, long long ps, int lds, long long pst, int ldt,
                                                int P, int N, const double *__restrict__ taps,
                                                const double *__restrict__ cq, const double *__restrict__ cp,
                                                int W, Centring C) {
    hpass_tile<S, R, COMBINE>(inT, out_stack, f, out, Pout, Qout, H, Wd, ld, ps, lds, pst, ldt, P, N, taps, cq, cp,
                              W, blockIdx.x, blockIdx.y, C);
}

// ---------------------------------------------------------------------------
// LDS-staged column and row passes (single image). A block first copies the
// input lines it needs (its 64-element segment of each line, through the
// symmetric extension) into LDS with 16-byte loads, all of them in flight at
// once, then convolves from there with conv_core in the FMA order of
// vpass_tile / hpass_tile: the outputs are bit-identical to those kernels
// (which the batched phases use). Reading from LDS takes the global-load
// latency off the FMA loop, the limit of the unstaged passes.
// ---------------------------------------------------------------------------

// Copies lines [0, nlines) of a 64-element-wide tile into LDS (line k from
// rowp(k): 64 elements, 16-byte aligned, inside the allocation), UNROLL
// 16-byte loads in flight per thread (256 threads).
template <class T, int UNROLL, class ROWP>
__device__ __forceinline__ void stage_lines(T *__restrict__ tile, int nlines, ROWP rowp) {
    constexpr int EPL = 16 / (int)sizeof(T);   // elements per 16-byte load
    constexpr int LPL = 64 / EPL;              // threads per line
    constexpr int LPB = 256 / LPL;             // lines per block-wide load
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // stays in registers (a uint4 array did not)
    const int lk = threadIdx.x / LPL, cc = (threadIdx.x % LPL) * EPL;
    for (int k0 = 0; k0 < nlines; k0 += LPB * UNROLL) {
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int k = k0 + u * LPB + lk;
            v[u] = k < nlines ? *reinterpret_cast<const u32x4 *>(rowp(k) + cc) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int k = k0 + u * LPB + lk;
            if (k < nlines) *reinterpret_cast<u32x4 *>(tile + k * 64 + cc) = v[u];
        }
    }
}

// Column pass (as vpass_tile) through the block's LDS tile: 64 columns
// [64 bx, 64 bx + 64) x 4R rows [4R by, 4R by + 4R) of plane n; the tile holds
// (4R + 2W) x 64 elements. Every thread meets the one barrier.
template <class S, int R>
__device__ __forceinline__ void vpass_tile_lds(typename S::T *__restrict__ tile,
                                               const typename S::T *__restrict__ in,
                                               typename S::T *__restrict__ outT, int H, int Wd, long long ps,
                                               int lds, long long pst, int ldt, const double *__restrict__ taps,
                                               int W, int bx, int by, int n) {
    typedef typename S::T T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = bx * 64, r0 = by * 4 * R;
    const T *plane = in + (long long)n * ps + c0;
    stage_lines<T, 8>(tile, 4 * R + 2 * W,
                      [&](int k) { return plane + (long long)mirror(r0 - W + k, H) * lds; });
    __syncthreads();
    const int rw = r0 + wave * R;
    if (rw < H) {
        const T *col = tile + wave * R * 64 + lane;
        double acc[R];
        conv_core<R, 8>([&](int i) { return (double)S::dec(col[i * 64]); }, W, taps + (kTapPad - 1), acc);
        const int c = c0 + lane;
        if (c < Wd) store_run<S, R>(outT + (long long)n * pst + (long long)c * ldt + rw, acc, H - rw);
    }
}

// Row pass (as hpass_tile) through the block's LDS tile: 64 rows
// [64 bx, 64 bx + 64) x 4R columns [4R by, 4R by + 4R), planes in
// hpass_tile's order, each staged as (4R + 2W) lines of 64 rows, with a
// barrier before each staging after the first; every thread meets all of them.
template <class S, int R, bool COMBINE>
__device__ __forceinline__ void hpass_tile_lds(typename S::T *__restrict__ tile,
                                               const typename S::T *__restrict__ inT,
                                               typename S::T *__restrict__ out_stack, const float *__restrict__ f,
                                               float *__restrict__ out, float *__restrict__ Pout,
                                               float *__restrict__ Qout, int H, int Wd, int ld, long long ps,
                                               int lds, long long pst, int ldt, int P, int N,
                                               const double *__restrict__ taps, const double *__restrict__ cq,
                                               const double *__restrict__ cp, int W, int bx, int by,
                                               const Centring &C) {
    typedef typename S::T T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = bx * 64, cb = by * 4 * R;
    const int r = r0 + lane;
    const int c0 = cb + wave * R;
    const bool active = c0 < Wd;   // wave-uniform; inactive waves still stage and meet the barriers
    const int rl = r < H ? r : H - 1;
    double s[R], Pa[R], Qa[R];
    if (COMBINE) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int cc = c0 + q < Wd ? c0 + q : Wd - 1;
            s[q] = ((double)f[(long long)rl * ld + cc] - C.tc) * C.inv_c;
            Pa[q] = 0.0;
            Qa[q] = 0.0;
        }
    }
    const T *line = tile + wave * R * 64 + lane;
    for (int k = 0; k < P; ++k) {
        const int n = COMBINE ? P - 1 - k : k;
        const T *plane = inT + (long long)n * pst + r0;
        if (k > 0) __syncthreads();   // every wave is done with the previous plane's tile
        stage_lines<T, 8>(tile, 4 * R + 2 * W,
                          [&](int j) { return plane + (long long)mirror(cb - W + j, Wd) * ldt; });
        __syncthreads();
        if (!active) continue;
        double acc[R];
        conv_core<R, 8>([&](int i) { return (double)S::dec(line[i * 64]); }, W, taps + (kTapPad - 1), acc);
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
    if (COMBINE && active && r < H) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (c0 + q < Wd) {
                const long long o = (long long)r * ld + c0 + q;
                if (C.mask != 0 && !centring_keeps(C, f[o])) continue;
                out[o] = (float)(C.tc + C.out_scale * (Pa[q] / Qa[q]));
                if (Pout) Pout[o] = (float)Pa[q];
                if (Qout) Qout[o] = (float)Qa[q];
            }
        }
    }
}

// Column pass (as k_vpass), LDS-staged: dynamic LDS (4R + 2W) x 64 elements.
template <class S, int R>
__global__ __launch_bounds__(256) void k_vpass_lds(const typename S::T *__restrict__ in,
                                                    typename S::T *__restrict__ outT, int H, int Wd, long long ps,
                                                    int lds, long long pst, int ldt,
                                                    const double *__restrict__ taps, int W) {
    extern __shared__ __align__(16) unsigned char s_lds[];
    vpass_tile_lds<S, R>(reinterpret_cast<typename S::T *>(s_lds), in, outT, H, Wd, ps, lds, pst, ldt, taps, W,
                         blockIdx.x, blockIdx.y, blockIdx.z);
}

// Row pass (as k_hpass), LDS-staged: dynamic LDS (4R + 2W) x 64 elements.
template <class S, int R, bool COMBINE>
__global__ __launch_bounds__(256) void k_hpass_lds(const typename S::T *__restrict__ inT,
                                                    typename S::T *__restrict__ out_stack,
                                                    const float *__restrict__ f, float *__restrict__ out,
                                                    float *__restrict__ Pout, float *__restrict__ Qout, int H,
                                                    int Wd, int ld, long long ps, int lds, long long pst, int ldt,
                                                    int P, int N, const double *__restrict__ taps,
                                                    const double *__restrict__ cq, const double *__restrict__ cp,
                                                    int W, Centring C) {
    extern __shared__ __align__(16) unsigned char s_lds[];
    hpass_tile_lds<S, R, COMBINE>(reinterpret_cast<typename S::T *>(s_lds), inT, out_stack, f, out, Pout, Qout, H,
                                  Wd, ld, ps, lds, pst, ldt, P, N, taps, cq, cp, W, blockIdx.x, blockIdx.y, C);
}

// ---------------------------------------------------------------------------
// Batched launch: many images of uneven sizes, each with its own sigma_s,
// sigma_r and N. Work items are the per-image kernels' blocks. Each of the
// three phases (build, column pass, row pass + combine) is one persistent
// kernel whose blocks stride over that phase's items of the whole batch
// (item t goes to block t mod gridDim.x); the kernel boundary between phases
// is the only synchronisation, so no block ever waits on another.
// ---------------------------------------------------------------------------

// Pointers read from the descriptor blob are generic to the compiler, which
// then emits flat loads with a 64-bit address per lane. Every buffer the
// batched kernels touch is device (global) memory, so they are cast to the
// global address space first; the tile code then gets global loads with a
// scalar base, as in the single-image kernels.
template <class T>
__device__ __forceinline__ T *as_global(T *p) {
    // Through an integer, so that the cast pair is not folded away before the
    // address-space inference sees the global pointer.
    return (T *)(__attribute__((address_space(1))) T *)(unsigned long long)p;
}

// Wave-uniform copies of descriptor fields: the descriptors sit in a blob the
// kernels also write (flags), so the compiler loads them per lane; reading
// the first lane puts them in scalar registers.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform(unsigned long long v) {
    return ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
           (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uniform(double v) {
    return __builtin_bit_cast(double, uniform(__builtin_bit_cast(unsigned long long, v)));
}
template <class T>
__device__ __forceinline__ T *uniform(T *p) {
    return (T *)uniform((unsigned long long)p);
}

struct BatchImage {
    const float *f;
    float *out;
    void *stackA;
    void *stackB;
    const double *prm;
    long long ps, pst;
    double mu;
    int H, Wd, ld, lds, ldt, W, N, P;
    int off_taps, off_cq, off_cp, off_scale, off_bf, off_tf;
    int gbx, gvx, gvy, ghx;    // tile grid widths: build, column pass, row pass (fused form: gvx = tiles per row)
    // Three-kernel form: the centring and output mask of the image's expansion
    // (the plain one, or one sub-range of the pivoted form, which then runs as
    // an image of its own writing only its pixels). Fused pivoted classes: K
    // sub-ranges, K / 255 for pivot_of, and the FusedPivot table at prm +
    // off_piv (taps at off_tf, coefficients at off_bf, as floats).
    Centring C;
    int K, off_piv;
    float kscale;
};

// Phases of the three-kernel form (build, column pass, row pass + combine) or
// classes of the fused form: the six geometry classes of the plain tile, then
// the same six for images routed to the pivoted form. A form uses the first 3
// or all 12.
constexpr int kFusedClasses = 6;
constexpr int kBatchPhases = 2 * kFusedClasses;

struct BatchHeader {
    unsigned flags;            // BF_DEVFLAG_RANGE from the builds
    int count;                 // images
    long long items[kBatchPhases];   // items in each phase
    long long queue[kBatchPhases];   // fused form: next item of each class (zero in every upload)
};
// device blob: BatchHeader | BatchImage[count] | long long start[12][count] |
//              int order[12][count] | parameter blocks
// In phase p the images are visited in order[p][0..count): item t belongs to
// image order[p][k] for the last k with start[p][k] <= t. The host orders each
// phase by decreasing cost per item (images with no items in a phase last), so
// the round-robin assignment of items to blocks gives every block a similar
// mix, heaviest items first.

constexpr int kMaxBatch = 2048;   // images per batched call

// Dynamic LDS for the phase's item table: count starts and count image indices.
__host__ __device__ constexpr size_t batch_lds_bytes(int count) {
    return (size_t)count * (sizeof(long long) + sizeof(int));
}

template <class S, int RV, int RH, int PHASE>
__global__ __launch_bounds__(256) void k_batched(char *__restrict__ blob) {
    extern __shared__ long long s_start[];
    BatchHeader *hdr = (BatchHeader *)blob;
    const BatchImage *img = (const BatchImage *)(blob + sizeof(BatchHeader));
    const int count = hdr->count;
    int *s_order = (int *)(s_start + count);
    const long long *start = (const long long *)(blob + sizeof(BatchHeader) + sizeof(BatchImage) * count);
    const int *order = (const int *)(start + kBatchPhases * count);
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        s_start[k] = start[PHASE * count + k];
        s_order[k] = order[PHASE * count + k];
    }
    __syncthreads();
    const long long items = hdr->items[PHASE];
    for (long long t = blockIdx.x; t < items; t += gridDim.x) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        // The decode reads LDS, so the compiler cannot see that it is the same in
        // every lane; readfirstlane keeps the image index (and so every field of
        // its descriptor and everything the tile derives from them) in scalar
        // registers, as in the single-image kernels.
        lo = __builtin_amdgcn_readfirstlane(lo);
        const int ii = __builtin_amdgcn_readfirstlane(s_order[lo]);
        const BatchImage &B = img[ii];
        const int l = (int)(t - s_start[lo]);
        typedef typename S::T T;
        const double *prm = as_global(B.prm);
        if (PHASE == 0) {
            const int cb = l % B.gbx, rb = l / B.gbx;
            const int r0 = rb * kBuildRows;
            build_tile<S>(as_global(B.f), B.H, B.Wd, B.ld, as_global((T *)B.stackA), B.ps, B.lds, B.P,
                          prm + B.off_scale, B.mu, as_global(&hdr->flags), cb, r0, min(B.H, r0 + kBuildRows),
                          B.C);
        } else if (PHASE == 1) {
            const int per_plane = B.gvx * B.gvy;
            const int n = l / per_plane, rem = l - n * per_plane;
            vpass_tile<S, RV>(as_global((const T *)B.stackA), as_global((T *)B.stackB), B.H, B.Wd, B.ps, B.lds,
                              B.pst, B.ldt, prm + B.off_taps, B.W, rem % B.gvx, rem / B.gvx, n);
        } else {
            hpass_tile<S, RH, true>(as_global((const T *)B.stackB), (T *)nullptr, as_global(B.f),
                                    as_global(B.out), nullptr, nullptr, B.H, B.Wd, B.ld, 0LL, 0, B.pst, B.ldt, B.P,
                                    B.N, prm + B.off_taps, prm + B.off_cq, prm + B.off_cp, B.W, l % B.ghx,
                                    l / B.ghx, B.C);
        }
    }
}

// Column and row passes of a batch (PHASE 1, 2) with one block per item
// (grid = the phase's items, set at every launch) and the LDS-staged tile
// functions of the single-image kernels, so each image equals its
// single-image result bit for bit. The phase's item table (starts and visiting
// order) is copied into LDS, the staged tile follows it (16-byte aligned; the
// launch sizes both). For batches whose table is small (the persistent
// k_batched serves the others).
template <class S, int RV, int RH, int PHASE>
__global__ __launch_bounds__(256) void k_batched_items(char *__restrict__ blob) {
    typedef typename S::T T;
    extern __shared__ long long s_start[];
    BatchHeader *hdr = (BatchHeader *)blob;
    const long long t = blockIdx.x;
    if (t >= hdr->items[PHASE]) return;
    const BatchImage *img = (const BatchImage *)(blob + sizeof(BatchHeader));
    const int count = hdr->count;
    int *s_order = (int *)(s_start + count);
    T *stile = reinterpret_cast<T *>((reinterpret_cast<uintptr_t>(s_order + count) + 15) & ~(uintptr_t)15);
    const long long *start = (const long long *)(blob + sizeof(BatchHeader) + sizeof(BatchImage) * count);
    const int *order = (const int *)(start + kBatchPhases * count);
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        s_start[k] = start[PHASE * count + k];
        s_order[k] = order[PHASE * count + k];
    }
    __syncthreads();
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int ii = __builtin_amdgcn_readfirstlane(s_order[lo]);
    const BatchImage &B = img[ii];
    const int l = (int)(t - s_start[lo]);
    const double *prm = as_global(B.prm);
    if (PHASE == 1) {
        const int per_plane = B.gvx * B.gvy;
        const int n = l / per_plane, rem = l - n * per_plane;
        vpass_tile_lds<S, RV>(stile, as_global((const T *)B.stackA), as_global((T *)B.stackB), B.H, B.Wd, B.ps,
                              B.lds, B.pst, B.ldt, prm + B.off_taps, B.W, rem % B.gvx, rem / B.gvx, n);
    } else {
        hpass_tile_lds<S, RH, true>(stile, as_global((const T *)B.stackB), (T *)nullptr, as_global(B.f),
                                    as_global(B.out), nullptr, nullptr, B.H, B.Wd, B.ld, 0LL, 0, B.pst, B.ldt, B.P,
                                    B.N, prm + B.off_taps, prm + B.off_cq, prm + B.off_cp, B.W, l % B.ghx,
                                    l / B.ghx, B.C);
    }
}

// ---------------------------------------------------------------------------
// Recursive variant of eq. 7 (Section I names recursion as the O(1) way to
// apply the Gaussian): Deriche's recursive Gaussian, a causal 4th-order
// recursion plus an anticausal one, per line, in FP64. Each line is extended
// by P samples per side through the symmetric extension and both recursions
// start from zero at the far ends; y = k (y+ + y-) on the line itself. This
// approximates the untruncated Gaussian, so it is a different filter from the
// truncated convolution (its own reference). FP32 stack; y+ is parked in the
// output plane (one extra FP32 rounding).
// ---------------------------------------------------------------------------

struct IirCoef {
    double n0, n1, n2, n3;   // causal numerator
    double m1, m2, m3, m4;   // anticausal numerator
    double d1, d2, d3, d4;   // common denominator 1 + sum d_i z^-i
    double k;                // unit DC gain
    int P;                   // extension per side
};

// Columns: one thread per column (coalesced along rows), plane blockIdx.y.
// The recursion is serial along the column and there are only Wd x P
// columns, so the inputs of the next kIirPrefetch samples are loaded while the
// current ones are processed (their latency would otherwise be paid per
// sample); the arithmetic is the plain sample-by-sample recursion.
constexpr int kIirPrefetch = 16;
template <class S>
__global__ __launch_bounds__(256) void k_iir_col(const typename S::T *__restrict__ in, typename S::T *__restrict__ out,
                                                  int H, int Wd, long long ps, int lds, IirCoef c) {
    typedef typename S::T T;
    constexpr int U = kIirPrefetch;
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= Wd) return;
    const T *src = in + (long long)blockIdx.y * ps + col;
    T *dst = out + (long long)blockIdx.y * ps + col;
    double x1 = 0, x2 = 0, x3 = 0, x4 = 0, y1 = 0, y2 = 0, y3 = 0, y4 = 0;
    T cur[U], nxt[U];
    // causal, rows -P .. H-1 (through the symmetric extension)
    const int i0 = -c.P;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (i0 + u < H) cur[u] = src[(long long)mirror(i0 + u, H) * lds];
    for (int ib = i0; ib < H; ib += U) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ib + U + u < H) nxt[u] = src[(long long)mirror(ib + U + u, H) * lds];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = ib + u;
            if (i < H) {
                const double x = S::dec(cur[u]);
                const double y = c.n0 * x + c.n1 * x1 + c.n2 * x2 + c.n3 * x3 - c.d1 * y1 - c.d2 * y2 - c.d3 * y3 -
                                 c.d4 * y4;
                x3 = x2; x2 = x1; x1 = x;
                y4 = y3; y3 = y2; y2 = y1; y1 = y;
                if (i >= 0) dst[(long long)i * lds] = S::enc(y);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
    // anticausal, rows H+P-1 .. 0; y+ read back from dst (this thread wrote it)
    x1 = x2 = x3 = x4 = y1 = y2 = y3 = y4 = 0;
    T ycur[U], ynxt[U];
    const int j0 = H + c.P - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = j0 - u;
        if (i >= 0) {
            cur[u] = src[(long long)mirror(i, H) * lds];
            if (i < H) ycur[u] = dst[(long long)i * lds];
        }
    }
    for (int ib = j0; ib >= 0; ib -= U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = ib - U - u;
            if (i >= 0) {
                nxt[u] = src[(long long)mirror(i, H) * lds];
                if (i < H) ynxt[u] = dst[(long long)i * lds];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = ib - u;
            if (i >= 0) {
                const double y = c.m1 * x1 + c.m2 * x2 + c.m3 * x3 + c.m4 * x4 - c.d1 * y1 - c.d2 * y2 - c.d3 * y3 -
                                 c.d4 * y4;
                const double x = S::dec(cur[u]);
                x4 = x3; x3 = x2; x2 = x1; x1 = x;
                y4 = y3; y3 = y2; y2 = y1; y1 = y;
                if (i < H) dst[(long long)i * lds] = S::enc(c.k * ((double)S::dec(ycur[u]) + y));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cur[u] = nxt[u];
            ycur[u] = ynxt[u];
        }
    }
}

// Ordering of a one-wave block's LDS accesses: a wave issues its LDS operations
// in order, so a counter wait and a compiler barrier suffice; unlike
// __syncthreads() this does not wait for the global loads in flight (the next
// tile's prefetch).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), other counters unconstrained (gfx9 encoding)
    __builtin_amdgcn_wave_barrier();
}

// The lane index, made where it is used: the compiler cannot hoist it out of
// a loop and hold it in a register across the loop.
__device__ __forceinline__ int fresh_lane_id() {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// Block barrier for LDS traffic only: the fences are limited to the local
// address space, so outstanding global loads (a prefetch) stay in flight
// across it; __syncthreads would wait for them as well.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Rows: one wave per block owns 64 rows; 64 x 32 tiles of the line are staged
// through LDS (coalesced loads and stores, row pitch 33 so a lane walking its
// row hits its own bank), and each lane runs the recursion along its row. The
// next tile's loads are issued before the current tile is processed.
constexpr int kIirChunk = 32;
template <class S>
__global__ __launch_bounds__(64) void k_iir_row(const typename S::T *__restrict__ in, typename S::T *__restrict__ out,
                                                 int H, int Wd, long long ps, int lds, IirCoef c) {
    typedef typename S::T T;
    __shared__ float X[64][kIirChunk + 1];
    __shared__ float Y[64][kIirChunk + 1];
    const int lane = threadIdx.x;
    const int r0 = blockIdx.x * 64;                         // < H by the grid
    const T *src = in + (long long)blockIdx.y * ps;
    T *dst = out + (long long)blockIdx.y * ps;
    constexpr int RPA = 64 / kIirChunk;                     // rows per access (kIirChunk lanes per row)
    constexpr int NR = 64 / RPA;                            // rows per lane per tile
    const int half = lane / kIirChunk, cc = lane % kIirChunk;
    auto row_of = [&](int q) { return (long long)min(r0 + half + RPA * q, H - 1) * lds; };
    // tile loads into registers: x (columns j0 + cc through the symmetric extension), and y+ when asked
    auto load_x = [&](int j0, T (&v)[NR]) {
        const int jm = mirror(j0 + cc, Wd);
#pragma unroll
        for (int q = 0; q < NR; ++q) v[q] = src[row_of(q) + jm];
    };
    auto load_y = [&](int j0, T (&v)[NR]) {
        if (j0 + cc < Wd) {
#pragma unroll
            for (int q = 0; q < NR; ++q) v[q] = dst[row_of(q) + j0 + cc];
        }
    };
    auto put = [&](float (&A)[64][kIirChunk + 1], const T (&v)[NR]) {
#pragma unroll
        for (int q = 0; q < NR; ++q) A[half + RPA * q][cc] = S::dec(v[q]);
    };
    auto store_y = [&](int j0) {
        if (j0 + cc >= 0 && j0 + cc < Wd)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (r0 + half + RPA * q < H)
                    dst[(long long)(r0 + half + RPA * q) * lds + j0 + cc] = S::enc(Y[half + RPA * q][cc]);
    };
    const int jlo = -((c.P + kIirChunk - 1) / kIirChunk) * kIirChunk;
    double x1 = 0, x2 = 0, x3 = 0, x4 = 0, y1 = 0, y2 = 0, y3 = 0, y4 = 0;
    T vx[NR], vy[NR];
    load_x(jlo, vx);
    for (int j0 = jlo; j0 < Wd; j0 += kIirChunk) {         // causal, left to right
        put(X, vx);
        if (j0 + kIirChunk < Wd) load_x(j0 + kIirChunk, vx);
        wave_lds_sync();
        for (int k = 0; k < kIirChunk; ++k) {
            const double x = X[lane][k];
            const double y = c.n0 * x + c.n1 * x1 + c.n2 * x2 + c.n3 * x3 - c.d1 * y1 - c.d2 * y2 - c.d3 * y3 - c.d4 * y4;
            x3 = x2; x2 = x1; x1 = x;
            y4 = y3; y3 = y2; y2 = y1; y1 = y;
            Y[lane][k] = (float)S::dec(S::enc(y));
        }
        wave_lds_sync();
        store_y(j0);
        wave_lds_sync();
    }
    const int jhi = ((Wd + c.P + kIirChunk - 1) / kIirChunk) * kIirChunk;
    x1 = x2 = x3 = x4 = y1 = y2 = y3 = y4 = 0;
    load_x(jhi - kIirChunk, vx);
    load_y(jhi - kIirChunk, vy);
    for (int j0 = jhi - kIirChunk; j0 >= 0; j0 -= kIirChunk) {   // anticausal, right to left
        put(X, vx);
        if (j0 + cc < Wd) put(Y, vy);
        if (j0 - kIirChunk >= 0) {
            load_x(j0 - kIirChunk, vx);
            load_y(j0 - kIirChunk, vy);
        }
        wave_lds_sync();
        for (int k = kIirChunk - 1; k >= 0; --k) {
            const double y = c.m1 * x1 + c.m2 * x2 + c.m3 * x3 + c.m4 * x4 - c.d1 * y1 - c.d2 * y2 - c.d3 * y3 - c.d4 * y4;
            const double x = X[lane][k];
            x4 = x3; x3 = x2; x2 = x1; x1 = x;
            y4 = y3; y3 = y2; y2 = y1; y1 = y;
            Y[lane][k] = (float)(c.k * ((double)Y[lane][k] + y));
        }
        wave_lds_sync();
        store_y(j0);
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Joint (cross) filter: the range variable comes from a guide g, the averaged
// values from f. Planes 0..N hold A_n = e^{-mu s^2/2} s^n with s from g (eq. 6
// on the guide), planes N+1..2N+1 hold B_n = A_n ft with ft = (f - t_c)/t_h;
// both carry the plane scale 2^k_n. Q = sum cq_n s^n Abar_n and
// Pt = sum cq_n s^n Bbar_n (eqs. 8-9 with f in place of the image), and
// y = t_c + t_h Pt/Q (eq. 10).
// ---------------------------------------------------------------------------

template <class S>
__global__ __launch_bounds__(256) void k_joint_build(const float *__restrict__ g, const float *__restrict__ f,
                                                      int H, int Wd, int ld, typename S::T *__restrict__ stack,
                                                      long long ps, int lds, int N,
                                                      const double *__restrict__ scale, double mu,
                                                      unsigned *__restrict__ flag) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r0 = blockIdx.y * kBuildRows, r1 = min(H, r0 + kBuildRows);
    for (int r = r0; r < r1; ++r) {
        bool bad = false;
        if (c < Wd) {
            const float gv = g[(long long)r * ld + c], fv = f[(long long)r * ld + c];
            bad = !(gv >= 0.0f && gv <= 255.0f) || !(fv >= 0.0f && fv <= 255.0f);
            const double s = ((double)gv - kTc) * (1.0 / kTh);          // eq. (17) on the guide
            const double ft = ((double)fv - kTc) * (1.0 / kTh);
            double v = exp(-0.5 * mu * s * s);
            typename S::T *dst = stack + (long long)r * lds + c;
            for (int n = 0; n <= N; ++n) {
                dst[n * ps] = S::enc(v * scale[n]);
                dst[(N + 1 + n) * ps] = S::enc(v * ft * scale[n]);
                v *= s;
            }
        }
        if (flag && __any(bad) && (threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(bad)) - 1)
            atomicOr(flag, BF_DEVFLAG_RANGE);
    }
}

// Row pass of the joint filter on the transposed planes (lane = row, R
// columns per wave), A_n and B_n together, folded by Horner's rule over
// descending n.
template <class S, int R>
__global__ __launch_bounds__(256) void k_hpass_joint(const typename S::T *__restrict__ inT,
                                                      const float *__restrict__ g, float *__restrict__ out,
                                                      int H, int Wd, int ld, long long pst, int ldt, int N,
                                                      const double *__restrict__ taps,
                                                      const double *__restrict__ cq, int W) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = blockIdx.x * 64 + lane;
    const int c0 = (blockIdx.y * 4 + wave) * R;
    if (c0 >= Wd) return;
    const int rl = r < H ? r : H - 1;
    double s[R], Pa[R], Qa[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int cc = c0 + q < Wd ? c0 + q : Wd - 1;
        s[q] = ((double)g[(long long)rl * ld + cc] - kTc) * (1.0 / kTh);
        Pa[q] = 0.0;
        Qa[q] = 0.0;
    }
    for (int n = N; n >= 0; --n) {
        double a[R], b[R];
        conv_line<S, R, 8>(inT + (long long)n * pst, rl, ldt, c0, Wd, W, taps + (kTapPad - 1), a);
        conv_line<S, R, 8>(inT + (long long)(N + 1 + n) * pst, rl, ldt, c0, Wd, W, taps + (kTapPad - 1), b);
        const double c = cq[n];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            Qa[q] = fma(Qa[q], s[q], c * a[q]);
            Pa[q] = fma(Pa[q], s[q], c * b[q]);
        }
    }
    if (r < H) {
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (c0 + q < Wd) out[(long long)r * ld + c0 + q] = (float)(kTc + kTh * (Pa[q] / Qa[q]));
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

// ---------------------------------------------------------------------------
// Fused FP64 adjoint tiles (radius W <= 16). One 1024-thread block per 64 x 32
// output tile (rows x columns). The planes (H_n in k_adj_forward_tile, R_m in
// k_adj_backward_tile) are generated one at a time over the tile and its
// W-halo, filtered in LDS (column pass, then row pass) and folded into
// per-pixel sums, so no plane stack goes through HBM. The tap loops are
// unrolled for the compile-time radius.
//
// The 16 waves take two roles. Waves 0-7 keep the generator state of the halo
// pixels in registers (halo row 8k + wave, halo column lane) and run the
// column pass with 8 rows per lane; waves 8-15 run the row pass with 4
// columns per lane and keep the output sums, one plane behind, reading the
// other of two column-pass buffers. Each role has its own loop (the role is
// wave-uniform, so each wave branches as a whole) with the same barriers:
//   step t:  generators: column pass of plane t (pl -> vt[t & 1])
//            row waves:  row pass + fold of plane t - 1 (vt[(t - 1) & 1])
//            barrier
//            generators: plane t + 1 into pl
//            barrier
// for t = 0..P, so every wave meets 1 + 2(P + 1) barriers.
// ---------------------------------------------------------------------------
constexpr int kAdjRows = 64;
constexpr int kAdjCols = 32;
constexpr int kAdjMaxRadius = BF_ADJ_MAX_RADIUS;
constexpr int kAdjPitch = kAdjCols + 2 * kAdjMaxRadius + 1;   // 65: odd in doubles, so lanes on consecutive rows start in distinct banks
constexpr int kAdjThreads = 1024;

// The W + 1 distinct taps (offsets -W..0; the Gaussian is symmetric), loaded
// once per block into (scalar) registers; tap t (offset t - W) of 2W + 1.
template <int W>
struct AdjTaps {
    double v[W + 1];
    __device__ __forceinline__ explicit AdjTaps(const double *__restrict__ w) {
#pragma unroll
        for (int t = 0; t <= W; ++t) v[t] = w[t];
    }
    __device__ __forceinline__ double operator[](int t) const { return v[t <= W ? t : 2 * W - t]; }
};

// acc[r] = sum_t tap(t - r) x(t), t in [0, R + 2W), x(t) = ld(t) from LDS:
// loads in chunks of U, the next chunk's loads issued before the current
// chunk's FMAs. Compiler and scheduling barriers between the chunks keep the
// loads from being merged and hoisted all ahead (2 registers per value).
template <int W, int R, int U, class LD>
__device__ __forceinline__ void adj_conv(LD ld, const AdjTaps<W> &w, double (&acc)[R]) {
    constexpr int T = R + 2 * W;
    constexpr int NC = (T + U - 1) / U;
    double buf[2][U];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (u < T) buf[0][u] = ld(u);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c + 1 < NC) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if ((c + 1) * U + u < T) buf[(c + 1) & 1][u] = ld((c + 1) * U + u);
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = c * U + u;
            if (t < T) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (t - r >= 0 && t - r <= 2 * W) acc[r] = fma(w[t - r], buf[c & 1][u], acc[r]);
            }
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    }
}

// alpha = dL/dP' = ybar t_h / Q and beta = dL/dQ = -alpha P'/Q of one pixel.
__device__ __forceinline__ void adj_alpha_beta(double yb, double Pa, double Qa, double &a, double &b) {
    a = yb * kTh / Qa;
    b = -a * Pa / Qa;
}

constexpr int kSplitWaves = 8;                                // waves per role
constexpr int kSplitRV = kAdjRows / kSplitWaves;              // 8 rows per lane, column pass
constexpr int kSplitRH = kAdjCols / kSplitWaves;              // 4 columns per lane, row pass

struct AdjLds {
    double pl[(kAdjRows + 2 * kAdjMaxRadius) * kAdjPitch];   // the current plane over the halo
    double vt[2][kAdjRows * kAdjPitch];                      // two column-pass results
};

template <int W>
constexpr int adj_own() {
    return (kAdjRows + 2 * W + kSplitWaves - 1) / kSplitWaves;
}

// Generator wave g, lane: its halo pixels k (halo row 8k + g, column lane).
template <int W>
__device__ __forceinline__ bool adj_split_in(int k, int g, int lane) {
    return kSplitWaves * k + g < kAdjRows + 2 * W && lane < kAdjCols + 2 * W;
}

// Column pass of the generator wave g: tile rows [8g, 8g + 8), lane = halo column.
template <int W>
__device__ __forceinline__ void adj_split_column(AdjLds &S, const AdjTaps<W> &w, int g, int lane, int b) {
    if (lane < kAdjCols + 2 * W) {
        double acc[kSplitRV];
        const double *src = S.pl + g * kSplitRV * kAdjPitch + lane;
        adj_conv<W, kSplitRV, 4>([&](int t) { return src[t * kAdjPitch]; }, w, acc);
#pragma unroll
        for (int r = 0; r < kSplitRV; ++r) S.vt[b][(g * kSplitRV + r) * kAdjPitch + lane] = acc[r];
    }
}

// Row pass of the row wave v: tile row lane, columns [4v, 4v + 4).
template <int W>
__device__ __forceinline__ void adj_split_row(const AdjLds &S, const AdjTaps<W> &w, int v, int lane, int b,
                                              double (&x)[kSplitRH]) {
    const double *src = S.vt[b] + lane * kAdjPitch + v * kSplitRH;
    adj_conv<W, kSplitRH, 4>([&](int t) { return src[t]; }, w, x);
}

// Forward in FP64, fused: the filtered planes Hbar_n at each output pixel,
// folded in ascending n into six sums (with explicit powers s^n, s^{n-1},
// s^{n-2} of the output pixel):
//   P' = sum cp_{n-1} s^{n-1} Hbar_n,  Q = sum cq_n s^n Hbar_n,
//   dP'/ds, dQ/ds (the explicit powers only),
//   Pm = sum bd_{n-1} s^{n-1} Hbar_n,  Qm = sum bd_n s^n Hbar_n,
// written to saved ([6][H][Wd] per image, FP64) when saved is non-null, and
// y = t_c + t_h P'/Q to out when out is non-null. Image z = blockIdx.z of a
// strided batch.
template <int W>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_adj_forward_tile(
    const float *__restrict__ f, float *__restrict__ out, double *__restrict__ saved, int H, int Wd, int ld,
    long long image_stride, int N, double mu, const double *__restrict__ taps, const double *__restrict__ cq,
    const double *__restrict__ cp, const double *__restrict__ bd, unsigned *__restrict__ flag) {
    __shared__ AdjLds S;
    const int r0 = blockIdx.y * kAdjRows, c0 = blockIdx.x * kAdjCols;
    const long long npx = (long long)H * Wd;
    f += blockIdx.z * image_stride;
    if (out) out += blockIdx.z * image_stride;
    if (saved) saved += blockIdx.z * 6 * npx;
    const AdjTaps<W> w(taps);   // taps points at the tap of offset -W
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = N + 2;
    if (wave < kSplitWaves) {
        constexpr int OWN = adj_own<W>();
        const int g = wave;
        double *own = S.pl + g * kAdjPitch + lane;
        double s[OWN], h[OWN];
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
            const bool in = adj_split_in<W>(k, g, lane);
            const int gi = in ? mirror(r0 - W + kSplitWaves * k + g, H) : 0;
            const int gj = in ? mirror(c0 - W + lane, Wd) : 0;
            const double sv = ((double)f[(long long)gi * ld + gj] - kTc) * (1.0 / kTh);
            s[k] = sv;
            h[k] = exp(-0.5 * mu * sv * sv);                                 // H_0
            if (in) own[k * kSplitWaves * kAdjPitch] = h[k];
        }
        __syncthreads();
        for (int t = 0; t <= P; ++t) {
            if (t < P) adj_split_column<W>(S, w, g, lane, t & 1);
            __syncthreads();
            if (t + 1 < P) {
#pragma unroll
                for (int k = 0; k < OWN; ++k) {
                    h[k] *= s[k];                                             // H_{t+1} = H_t s
                    if (adj_split_in<W>(k, g, lane)) own[k * kSplitWaves * kAdjPitch] = h[k];
                }
            }
            __syncthreads();
        }
    } else {
        const int v = wave - kSplitWaves;
        const int i = lane, j0 = v * kSplitRH;
        const int gr = min(r0 + i, H - 1);
        double so[kSplitRH], p2[kSplitRH];   // s and s^{max(n-2,0)} of the output pixel
        double Pa[kSplitRH], Qa[kSplitRH], dP[kSplitRH], dQ[kSplitRH], Pm[kSplitRH], Qm[kSplitRH];
#pragma unroll
        for (int q = 0; q < kSplitRH; ++q) {
            const int gc = min(c0 + j0 + q, Wd - 1);
            so[q] = ((double)f[(long long)gr * ld + gc] - kTc) * (1.0 / kTh);
            p2[q] = 1.0;
            Pa[q] = Qa[q] = dP[q] = dQ[q] = Pm[q] = Qm[q] = 0.0;
        }
        __syncthreads();
        for (int t = 0; t <= P; ++t) {
            if (t >= 1) {
                const int n = t - 1;
                const double cqn = n <= N ? cq[min(n, N)] : 0.0, bqn = n <= N ? bd[min(n, N)] : 0.0;
                const double cpn = n >= 1 ? cp[max(n - 1, 0)] : 0.0, bpn = n >= 1 ? bd[max(n - 1, 0)] : 0.0;
                double x[kSplitRH];
                adj_split_row<W>(S, w, v, lane, n & 1, x);
                const double ncq = (double)n * cqn, ncp = (double)(n - 1) * cpn;
#pragma unroll
                for (int q = 0; q < kSplitRH; ++q) {
                    // v0 = s^n x, v1 = s^{n-1} x, v2 = s^{n-2} x (p2 = s^{max(n-2,0)}).
                    // Below n = 2 a missing (negative) power is replaced by the next
                    // one: only zero coefficients meet it (cpn and ncq at n = 0, ncp
                    // at n <= 1). The selects are on n, uniform: no branches.
                    const double v2 = p2[q] * x[q];
                    const double v1 = n >= 2 ? so[q] * v2 : v2;
                    const double v0 = n >= 1 ? so[q] * v1 : v1;
                    if (n >= 2) p2[q] *= so[q];
                    Qa[q] = fma(cqn, v0, Qa[q]);
                    Qm[q] = fma(bqn, v0, Qm[q]);
                    dQ[q] = fma(ncq, v1, dQ[q]);
                    Pa[q] = fma(cpn, v1, Pa[q]);
                    Pm[q] = fma(bpn, v1, Pm[q]);
                    dP[q] = fma(ncp, v2, dP[q]);
                }
            }
            __syncthreads();
            __syncthreads();
        }
        const int r = r0 + i;
        bool bad = false;
#pragma unroll
        for (int q = 0; q < kSplitRH; ++q) {
            const int c = c0 + j0 + q;
            if (r < H && c < Wd) {
                const long long o = (long long)r * Wd + c;
                if (saved) {
                    saved[o] = Pa[q];
                    saved[npx + o] = Qa[q];
                    saved[2 * npx + o] = dP[q];
                    saved[3 * npx + o] = dQ[q];
                    saved[4 * npx + o] = Pm[q];
                    saved[5 * npx + o] = Qm[q];
                }
                if (out) out[(long long)r * ld + c] = (float)(kTc + kTh * (Pa[q] / Qa[q]));   // eq. 10
                const float fv = f[(long long)r * ld + c];
                bad |= !(fv >= 0.0f && fv <= 255.0f);
            }
        }
        if (flag && __any(bad) && lane == __ffsll((unsigned long long)__ballot(bad)) - 1)
            atomicOr(flag, BF_DEVFLAG_RANGE);
    }
}

// Adjoint, fused: the planes R_m (from alpha, beta of the halo pixels, formed
// from the saved sums and ybar) filtered by the same mirrored Gaussian, folded
// at each output pixel j with H_m(j) recomputed in FP64 into dL/df_j; one
// partial sum of the dL/dmu terms per tile and image (summed in a fixed order
// by k_reduce_f64). Image z = blockIdx.z of a strided batch.
template <int W>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_adj_backward_tile(
    const float *__restrict__ f, const float *__restrict__ ybar, const double *__restrict__ saved,
    float *__restrict__ grad_f, double *__restrict__ partial, int H, int Wd, int ld, long long image_stride, int N,
    double mu, const double *__restrict__ taps, const double *__restrict__ cq, const double *__restrict__ cp) {
    __shared__ AdjLds S;
    const int r0 = blockIdx.y * kAdjRows, c0 = blockIdx.x * kAdjCols;
    const long long npx = (long long)H * Wd;
    f += blockIdx.z * image_stride;
    ybar += blockIdx.z * image_stride;
    grad_f += blockIdx.z * image_stride;
    saved += blockIdx.z * 6 * npx;
    const AdjTaps<W> w(taps);   // taps points at the tap of offset -W
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = N + 2;
    double local = 0.0;
    if (wave < kSplitWaves) {
        constexpr int OWN = adj_own<W>();
        const int g = wave;
        double *own = S.pl + g * kAdjPitch + lane;
        double s[OWN], A[OWN], B[OWN];   // A = alpha s^{m-1} (from m = 1), B = beta s^m
        const double cq0 = cq[0];
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
            const bool in = adj_split_in<W>(k, g, lane);
            const int gi = in ? mirror(r0 - W + kSplitWaves * k + g, H) : 0;
            const int gj = in ? mirror(c0 - W + lane, Wd) : 0;
            s[k] = ((double)f[(long long)gi * ld + gj] - kTc) * (1.0 / kTh);
            const long long o = (long long)gi * Wd + gj;
            adj_alpha_beta((double)ybar[(long long)gi * ld + gj], saved[o], saved[npx + o], A[k], B[k]);
            if (in) own[k * kSplitWaves * kAdjPitch] = cq0 * B[k];          // R_0
        }
        __syncthreads();
        for (int t = 0; t <= P; ++t) {
            if (t < P) adj_split_column<W>(S, w, g, lane, t & 1);
            __syncthreads();
            if (t + 1 < P) {
                const double cpm = cp[min(t, N)], cqm = t + 1 <= N ? cq[min(t + 1, N)] : 0.0;
#pragma unroll
                for (int k = 0; k < OWN; ++k) {
                    if (t >= 1) A[k] *= s[k];
                    B[k] *= s[k];
                    if (adj_split_in<W>(k, g, lane))
                        own[k * kSplitWaves * kAdjPitch] = fma(cpm, A[k], cqm * B[k]);   // R_{t+1}
                }
            }
            __syncthreads();
        }
    } else {
        const int v = wave - kSplitWaves;
        const int i = lane, j0 = v * kSplitRH;
        const int gr = min(r0 + i, H - 1);
        double so[kSplitRH], hm1[kSplitRH], h0[kSplitRH], h1[kSplitRH], h2[kSplitRH], gs[kSplitRH], gm[kSplitRH];
#pragma unroll
        for (int q = 0; q < kSplitRH; ++q) {
            const int gc = min(c0 + j0 + q, Wd - 1);
            const double sv = ((double)f[(long long)gr * ld + gc] - kTc) * (1.0 / kTh);
            const double E = exp(-0.5 * mu * sv * sv);
            so[q] = sv;
            hm1[q] = 0.0;                                                     // H_{m-1}, H_m, H_{m+1}, H_{m+2}
            h0[q] = E;
            h1[q] = E * sv;
            h2[q] = E * sv * sv;
            gs[q] = gm[q] = 0.0;
        }
        __syncthreads();
        for (int t = 0; t <= P; ++t) {
            if (t >= 1) {
                const int m = t - 1;
                double x[kSplitRH];
                adj_split_row<W>(S, w, v, lane, m & 1, x);
                const double md = (double)m;
#pragma unroll
                for (int q = 0; q < kSplitRH; ++q) {
                    gs[q] = fma(x[q], fma(md, hm1[q], -mu * h1[q]), gs[q]);
                    gm[q] = fma(x[q], h2[q], gm[q]);
                    hm1[q] = h0[q];
                    h0[q] = h1[q];
                    h1[q] = h2[q];
                    h2[q] *= so[q];
                }
            }
            __syncthreads();
            __syncthreads();
        }
        const int r = r0 + i;
#pragma unroll
        for (int q = 0; q < kSplitRH; ++q) {
            const int c = c0 + j0 + q;
            if (r < H && c < Wd) {
                const long long o = (long long)r * Wd + c;
                double a, b;
                adj_alpha_beta((double)ybar[(long long)r * ld + c], saved[o], saved[npx + o], a, b);
                const double gdir = a * saved[2 * npx + o] + b * saved[3 * npx + o];   // alpha dP'/ds + beta dQ/ds
                const double gmu = a * saved[4 * npx + o] + b * saved[5 * npx + o];    // coefficient term of dL/dmu
                grad_f[(long long)r * ld + c] = (float)((gdir + gs[q]) * (1.0 / kTh));
                local += gmu - 0.5 * gm[q];
            }
        }
    }
    // every wave has met the loop's last barrier: the LDS is free
    double *red = S.pl;
    red[threadIdx.x] = local;
    __syncthreads();
    for (int v = kAdjThreads / 2; v > 0; v >>= 1) {
        if ((int)threadIdx.x < v) red[threadIdx.x] += red[threadIdx.x + v];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// dL/dsigma_r = (sum of the partials) (-2 mu / sigma_r); fixed summation order.
__global__ __launch_bounds__(256) void k_reduce_f64(const double *__restrict__ partial, long long n, double scale,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    double v = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) v += partial[i];
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
// Fused reduced-precision path (FP16 / BF16 stack): one kernel per 64-row
// output tile runs build, both Gaussian passes and the combine for every
// plane, so the stack never leaves the chip.
//
// Each plane H_n (scaled by 2^k_n for FP16, eq. 6 in scaled form) is made in
// registers by the running product H <- H s and rounded to the stack type; the
// two passes of eq. 7 are banded Toeplitz products on the matrix cores
// (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation); the combine of eqs. 8-9
// adds cq_n s^n Hbar_n to Q and cp_{n-1} s^{n-1} Hbar_n to P in FP32 as the
// planes go by; eq. 10 gives y.
//
// Geometry. Output tile: rows [r0, r0+64), columns [c0, c0+TC). The column
// pass covers the halo columns c0-W+[0,128) (8 blocks of 16, one per wave)
// and the halo rows r0-W+[0,32Q) in chunks of 32 (the MFMA K dimension). For
// output row block j (16 rows) and input chunk q the Toeplitz operand is
//   B[k][n] = w[32q + k - 16j - n]   (k: row in the chunk, n: row in the block),
// zero outside [0, 2W]; it depends only on d = 2q - j, so the 2Q fragments
// d = -1 .. 2Q-2 are made once per tile and serve both passes (the row pass
// has the same structure along columns). The column pass computes the
// transposed product (M = halo columns, N = output rows), which leaves each
// lane four consecutive columns of one row; these go through LDS as the row
// pass's row-major A operand.
// ---------------------------------------------------------------------------

typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_b8 __attribute__((ext_vector_type(8)));
typedef __bf16 mf_b4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

struct MmaF16 {
    // every FP16 plane carries 2^14: plane 0 peaks there, and the smallest
    // plane maximum e^{-mu/2} 2^14 stays a normal FP16 number while sigma_r >= 21
    static constexpr float kPrescale = 16384.0f;
    // the running plane H_{n+1} = H_n s is kept in FP16 (packed multiplies;
    // the rounding this adds is far below the stack's own, see filter())
    static constexpr bool kHalfPlanes = true;
    typedef _Float16 E;
    typedef mf_h8 V;
    typedef mf_h4 V4;
    static __device__ __forceinline__ E cvt(float x) { return (_Float16)x; }
    static __device__ __forceinline__ mf_f4 mma(V a, V b, mf_f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
struct MmaBF16 {
    static constexpr float kPrescale = 1.0f;   // BF16 has the FP32 exponent range
    static constexpr bool kHalfPlanes = false;  // an 8-bit significand would compound over n
    typedef __bf16 E;
    typedef mf_b8 V;
    typedef mf_b4 V4;
    static __device__ __forceinline__ E cvt(float x) { return (__bf16)x; }
    static __device__ __forceinline__ mf_f4 mma(V a, V b, mf_f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// An MFMA operand (8 elements) from the column-pass tile in LDS, as two
// 8-byte reads: the row pitch below is a multiple of 8 bytes but not of 16.
template <class M>
__device__ __forceinline__ typename M::V ld_frag(const typename M::E *p) {
    const typename M::V4 lo = *(const typename M::V4 *)p, hi = *(const typename M::V4 *)(p + 4);
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

constexpr int kFusedRows = 64;               // output rows per tile
constexpr int kFusedHaloC = 128;             // halo columns of the column pass
// LDS row pitch (elements) of the column-pass result: 70 words, 6 mod 32.
// The column pass writes 8 bytes per lane to rows li = 0..15 and the row
// pass reads 8 bytes per lane from rows li = 0..15; with this pitch both
// spread over all 32 banks (SQ_LDS_BANK_CONFLICT reads 0; a 16-byte aligned
// pitch of 136 leaves the writes two-way conflicted).
constexpr int kFusedPitch = kFusedHaloC + 12;

// Chunk ranges. Output block j (16 rows or columns) needs the halo positions
// [16j, 16j + 15 + 2W], i.e. chunks j/2 .. j/2 + A for even j and
// j/2 .. j/2 + B for odd j, with A = (2W+15)/32 and B = (2W+31)/32. For each
// kernel geometry B = Q - 2 and A is Q - 3 or Q - 2 (template parameter QA).
__host__ __device__ constexpr int fused_qa(int W) { return (2 * W + 15) / 32; }

// Symmetric extension for |overhang| <= M (one reflection).
__device__ __forceinline__ int mirror1(int i, int M) { return i < 0 ? -1 - i : (i >= M ? 2 * M - 1 - i : i); }

// Halo index -> image index. Positions at or beyond M + W only feed outputs at
// or beyond M, which are not stored, so they are clamped to M + W - 1 first;
// with W < M one reflection then suffices.
__device__ __forceinline__ int halo_index(int i, int M, int W, bool one_reflection) {
    return one_reflection ? mirror1(min(i, M + W - 1), M) : mirror(i, M);
}

constexpr int kFusedTabPad = 32;             // zero taps below t = 0 in the LDS tap table

// Constants of one fused launch, passed by value (kernel arguments): taps
// w[t], t = 0..2W (tap t - W), and b_n, n = 0..N+1 with b_{N+1} = 0.
struct FusedConsts {
    float taps[2 * BF_FUSED_F16_MAX_RADIUS + 1];
    float b[BF_MAX_DEGREE + 2];
};

// Range flag of a wave: with slots (single-image launches) every wave
// writes its own word slot[wave], 0 or BF_DEVFLAG_RANGE, so no word needs
// clearing first; without (batched) the flag word is or-ed.
__device__ __forceinline__ void report_range(bool bad, unsigned *flag, unsigned *slot) {
    if (slot) {
        const bool any = __any(bad);
        if ((threadIdx.x & 63) == 0) slot[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)] = any ? BF_DEVFLAG_RANGE : 0u;
    } else if (flag && __any(bad) && (threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(bad)) - 1) {
        atomicOr(flag, BF_DEVFLAG_RANGE);
    }
}
constexpr int kFusedSlots = 8;    // range words per tile of a single-image fused launch (one per wave)
constexpr int kFusedYElems = kFusedRows * kFusedPitch;
__host__ __device__ constexpr int fused_tab_len(int Q) { return kFusedTabPad + 32 * Q; }   // t in [-32, 32Q)

// Centring of one expansion in the fused tile (eq. 17 with a centre t and
// scales): the planes are built from s_j = f_j sb + ob, with 2^K e^{-nu s^2/2}
// computed as 2^{e2 s_j^2 + k2}; the combine takes s_i = f_i sc + oc and
// gives y = yo + ys Ps / (s_i Q).
struct FusedCentre {
    float sb, ob, e2, k2, sc, oc, ys, yo;
};

// One sub-range of the pivoted form for the fused tile (device memory):
// its centring, the lower end lo of [lo, hi) as the selection compares it,
// the degree N and the offset (floats) of its coefficients, n = 0..N+1.
struct FusedPivot {
    FusedCentre c;
    float lo;
    int N, boff, pad;
};

// Sub-range of a centre value x among K equal sub-ranges with lower ends
// lo[k] (the partition of the pivoted form: the number of k >= 1 with
// !(x < lo[k]), so NaN goes to the last): a first guess from the equal widths
// (kscale = K / 255), then one step each way against the exact ends.
__device__ __forceinline__ int pivot_of(float x, const float *lo, int K, float kscale) {
    int g = x == x ? (int)fminf(fmaxf(x * kscale, 0.0f), (float)(K - 1)) : K - 1;
    if (g > 0 && x < lo[g]) --g;
    else if (g < K - 1 && !(x < lo[g + 1])) ++g;
    return g;
}

// Fused tile machinery; all 64 NW threads of the block use it together.
// setup() makes the Toeplitz fragments of one image (through the LDS tap
// table tab, fused_tab_len(Q) elements); load() issues the global loads of
// one TR x TC output tile's inputs (halo column values and the lane's own
// output pixels) into registers; run() filters that tile through ybuf
// (kBufs LDS buffers of kYElems elements) and stores it. Blocks that run
// several tiles or centrings back to back continue the buffer parity (base)
// and use two buffers (the 8-wave forms).
// Geometry: NW waves (8 or 16) per block; output tiles of TR rows (64 or 32)
// by TC columns. The column pass runs on the first kNCW waves, each over 16
// halo columns and the tile's TR/16 row blocks; the row pass gives each wave
// JB of the tile's (TR/16) x (TC/16) output blocks, in one row block rb.
template <class M, int Q, int TC, int QA, int NW = 8, int TR = kFusedRows,
          int BUFS = (NW == 16 && TR == 64) ? 4 : 2>
struct FusedTile {
    typedef typename M::E E;
    typedef typename M::V V;
    static constexpr int QB = Q - TR / 32;       // chunk range of odd row blocks (see fused_qa)
    static constexpr int kNRB = TR / 16;         // row blocks
    static constexpr int kNCB = TC / 16;         // output column blocks
    static constexpr int kWPR = NW / kNRB;       // waves per row block in the row pass
    static constexpr int JB = kNCB / kWPR;       // output column blocks per wave in the row pass
    // halo columns the row pass reads: column blocks up to kNCB - 1 from
    // their 32-column chunk base, QB + 1 chunks each
    static constexpr int kNCW = kNCB + 2 * QB;
    // LDS row pitch (elements): the 16 kNCW columns the column waves write,
    // rounded up to 6 words mod 32
    static constexpr int kPitch = 2 * (8 * kNCW + ((6 - 8 * kNCW) % 32 + 32) % 32);
    static constexpr int kYElems = TR * kPitch;
    static constexpr int kSlots = NW;            // range words per tile (one per wave)
    // LDS buffers of the column-pass result: with four, two planes per
    // barrier phase (the single-image 64-row tiles on 16 waves); with two,
    // one (every other form)
    static constexpr int kBufs = BUFS;
    static_assert(BUFS == 2 || BUFS == 4, "buffers");
    static_assert(TR == 64 || TR == 32, "tile rows");
    static_assert(JB == 1 || JB == 2, "row-pass blocks per wave");
    static_assert(kNCW <= NW, "halo columns");
    static_assert(QA == QB - 1 || QA == QB, "chunk range");

    // Inputs of one tile: h[q][jj] = f at halo column 16 wave + li, halo row
    // 32q + 8lg + jj; c[b][v] = f at output row 16 rb + 4 lg + v, column
    // 16 (jc0 + b) + li (clamped into the image).
    struct Raw {
        float h[Q][8];
        float c[JB][4];
    };

    const float *__restrict__ f;
    float *__restrict__ out;
    const float *__restrict__ bt;                // b_n as floats, n = 0..N+1 (b_{N+1} = 0)
    E *__restrict__ ybuf;
    int H, Wd, ld, W, N;
    float mu, prescale;
    int lane, wave, li, lg, rb, p, jc0;
    bool one_ref;
    V tf[2 * Q];

    __device__ __forceinline__ FusedTile(const float *f_, float *out_, int H_, int Wd_, int ld_, int W_, int N_,
                                         float mu_, float prescale_, const float *bt_, E *ybuf_)
        : f(f_), out(out_), bt(bt_), ybuf(ybuf_), H(H_), Wd(Wd_), ld(ld_), W(W_), N(N_), mu(mu_),
          prescale(prescale_) {
        lane = threadIdx.x & 63;
        wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        li = lane & 15;
        lg = lane >> 4;
        // Row-pass assignment: row block rb = wave / kWPR, m = wave % kWPR.
        // With JB = 2 the wave takes column blocks 2m, 2m+1, which read the
        // halo chunks from column 32m and use the fragments of blocks 0, 1.
        // With JB = 1 it takes block jc = m, reading chunks from 32 (m / 2);
        // its fragment for chunk q, w[32q + 8lg + jj - 16 (m & 1) - li], is
        // tf[2q + 1 - (m & 1)].
        rb = wave / kWPR;
        p = wave % kWPR;
        jc0 = p * JB;
        one_ref = W < H && W < Wd;
    }

    // Tap table in LDS, tab[kFusedTabPad + t] = w[t] for t in [0, 2W] and zero
    // elsewhere, then the Toeplitz fragments tf[d+1], d = -1 .. 2Q-2: element
    // jj of lane (li, lg) is w[16d + 8lg + jj - li].
    __device__ __forceinline__ void setup(const float *__restrict__ taps, E *__restrict__ tab) {
        constexpr int kTabPad = kFusedTabPad;
        for (int i = threadIdx.x; i < fused_tab_len(Q); i += blockDim.x) {
            const int t = i - kTabPad;
            tab[i] = M::cvt(t >= 0 && t <= 2 * W ? taps[t] : 0.0f);
        }
        __syncthreads();
#pragma unroll
        for (int d = -1; d < 2 * Q - 1; ++d)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) tf[d + 1][jj] = tab[kTabPad + 16 * d + 8 * lg + jj - li];
    }

    __device__ __forceinline__ void load(int r0, int c0, Raw &R) const {
        const int mc = halo_index(c0 - W + 16 * wave + li, Wd, W, one_ref);
        const int cr = r0 + 16 * rb + 4 * lg;                    // first output row of the lane
        const bool colw = kNCW == NW || wave < kNCW;              // (uniform) a column-pass wave
        if (r0 - W >= 0 && r0 - W + 32 * Q <= H && r0 + TR <= H && (long long)H * ld < (1LL << 29)) {
            // Most tiles: every halo row and output row inside the image, and
            // byte offsets within 32 bits, so each load is one add from the
            // lane's first offset (the row steps are uniform).
            const char *base = (const char *)f;
            const unsigned o = 4u * (unsigned)((r0 - W + 8 * lg) * ld + mc);
            const unsigned ld4 = 4u * (unsigned)ld;
            if (colw) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        R.h[q][jj] = *(const float *)(base + o + (unsigned)(32 * q + jj) * ld4);
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) R.h[q][jj] = 0.0f;
            }
#pragma unroll
            for (int b = 0; b < JB; ++b) {
                const unsigned oc = 4u * (unsigned)(cr * ld + min(c0 + 16 * (jc0 + b) + li, Wd - 1));
#pragma unroll
                for (int v = 0; v < 4; ++v) R.c[b][v] = *(const float *)(base + oc + (unsigned)v * ld4);
            }
        } else {
            // symmetric extension of the halo rows; output rows clamped
            const float *col = f + mc;
            if (colw) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        R.h[q][jj] = col[(long long)halo_index(r0 - W + 32 * q + 8 * lg + jj, H, W, one_ref) * ld];
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) R.h[q][jj] = 0.0f;
            }
#pragma unroll
            for (int b = 0; b < JB; ++b) {
                const int c = min(c0 + 16 * (jc0 + b) + li, Wd - 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) R.c[b][v] = f[(long long)min(cr + v, H - 1) * ld + c];
            }
        }
    }

    // The lane's output pixels alone (Raw::c, the same values load() gives),
    // by 32-bit byte offsets: H ld < 2^29.
    // ln: the lane index (threadIdx.x mod 64).
    __device__ __forceinline__ void load_pixels(int r0, int c0, float (&c)[JB][4], int ln) const {
        const char *base = (const char *)f;
        const int cr = r0 + 16 * rb + 4 * (ln >> 4);
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const int col = min(c0 + 16 * (jc0 + b) + (ln & 15), Wd - 1);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                c[b][v] = *(const float *)(base + 4u * (unsigned)(min(cr + v, H - 1) * ld + col));
        }
    }

    // Range check on the lane's own output pixels: every pixel of the image
    // is the output of exactly one lane of one tile.
    __device__ __forceinline__ void check_range(const Raw &R, unsigned *__restrict__ flag,
                                                unsigned *__restrict__ slot) const {
        bool bad = false;
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) bad |= !(R.c[b][v] >= 0.0f && R.c[b][v] <= 255.0f);
        report_range(bad, flag, slot);
    }

    // Column-pass A operand state of one centring: s and the running 2^K H_n
    // for the lane's 8Q halo values (one scale 2^K for every plane keeps FP16
    // planes normal: it cancels in P/Q), with 2^K e^{-nu s^2/2} =
    // 2^{e2 s^2 + k2}. FP32 state (BF16), rounded once per plane; or (FP16,
    // kHalfPlanes) s and H_n held in FP16 and H_{n+1} = H_n s as packed FP16
    // products, which halves the state and needs no conversion per plane.
    // There H_0 is taken at the FP16 value of s too, so every plane is that of
    // one halo value moved by about |f - t| 2^-12 (one FP16 ulp of s), plus one
    // rounding per product; at 4096^2, sigma_s = 10, sigma_r = 30, N = 32 the
    // error against the direct filter stays 0.11 max-abs, 98.7 dB PSNR (98.8
    // with the FP32 recursion).
    static constexpr bool kH16 = M::kHalfPlanes;
    struct State {
        float sv[kH16 ? 1 : Q][8], hv[kH16 ? 1 : Q][8];
        V sv16[kH16 ? Q : 1], hv16[kH16 ? Q : 1];
    };
    static __device__ __forceinline__ float h0_of(float s, const FusedCentre &C) {
        return __builtin_amdgcn_exp2f(fmaf(C.e2 * s, s, C.k2));                  // 2^K H_0
    }
    // FP16 s of one halo value f (eq. 17).
    static __device__ __forceinline__ E s16_of(float f, const FusedCentre &C) { return M::cvt(fmaf(f, C.sb, C.ob)); }

    // State from the halo values h (the lane's Raw::h).
    __device__ __forceinline__ void build_state(const float (&h)[Q][8], const FusedCentre &C, State &S) const {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                if constexpr (kH16) {
                    const E s16 = s16_of(h[q][jj], C);
                    S.sv16[q][jj] = s16;
                    S.hv16[q][jj] = M::cvt(h0_of((float)s16, C));
                } else {
                    const float s = fmaf(h[q][jj], C.sb, C.ob);                  // eq. (17)
                    S.sv[q][jj] = s;
                    S.hv[q][jj] = h0_of(s, C);
                }
            }
        }
    }
    // Filters the N+2 planes of one centring (coefficients bt[n], n = 0..N+1,
    // with bt[N+1] = 0) and leaves the lane's outputs (rows 16 rb + 4 lg + v,
    // columns 16 (jc0 + b) + li) in y.
    // base: parity of the buffer the tile's plane 0 goes to. A block that
    // runs tiles (or centrings) back to back continues the alternation (base
    // = planes run before), so that the next first column pass writes the
    // buffer the last row pass did not read and needs no barrier before it.
    __device__ __forceinline__ void filter(const Raw &R, const FusedCentre &C, const float *__restrict__ bt, int N,
                                           int base, float (&y)[JB][4]) {
        const int P = N + 2;
        // The column-pass A operand state of State, built as build_state does
        // (local arrays: the other geometries keep fewer registers so).
        float sv[kH16 ? 1 : Q][8], hv[kH16 ? 1 : Q][8];
        V sv16[kH16 ? Q : 1], hv16[kH16 ? Q : 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                if constexpr (kH16) {
                    const E s16 = s16_of(R.h[q][jj], C);
                    sv16[q][jj] = s16;
                    hv16[q][jj] = M::cvt(h0_of((float)s16, C));
                } else {
                    const float s = fmaf(R.h[q][jj], C.sb, C.ob);                 // eq. (17)
                    sv[q][jj] = s;
                    hv[q][jj] = h0_of(s, C);
                }
            }
        }

        // With u_n = s^n Hbar_n the sums are accumulated as
        //   Q = sum_n b_n u_n,   Ps = sum_n b_{n-1} u_n = s P,
        // so one product serves both, and P = Ps / s. Where s = 0 the sums take
        // s = 2^-64 instead: Ps / s is then b_0 Hbar_1, the value of P at s = 0,
        // up to terms 2^-64 smaller, and Q moves by as little. (Where b_0 2^-64
        // Hbar_1 underflows, P/Q lies far below FP32 resolution: the pixel's own
        // term keeps Q >= w_0 b_0 2^K.)
        float sc[JB][4], pw[JB][4], Ps[JB][4], Qa[JB][4];
#pragma unroll
        for (int b = 0; b < JB; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float s = fmaf(R.c[b][v], C.sc, C.oc);
                sc[b][v] = s != 0.0f ? s : 0x1p-64f;
                pw[b][v] = sc[b][v];
                Ps[b][v] = 0.0f;
                Qa[b][v] = 0.0f;
            }
        }

        // Column pass of plane n into its LDS buffer; advances H to plane n+1.
        // Waves past kNCW hold no halo columns the row pass reads.
        auto column_pass = [&](int n) {
            if (kNCW < NW && wave >= kNCW) return;
            V a[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if constexpr (kH16) {
                    a[q] = hv16[q];
                    hv16[q] = hv16[q] * sv16[q];                          // H_{n+1} = H_n s
                } else {
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        a[q][jj] = M::cvt(hv[q][jj]);
                        hv[q][jj] *= sv[q][jj];                           // H_{n+1} = H_n s
                    }
                }
            }
            E *yb = ybuf + ((n + base) & (kBufs - 1)) * kYElems;
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int j = 0; j < kNRB; ++j) {
                const int qlast = min(Q - 1, j / 2 + ((j & 1) ? QB : QA));
                mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = j / 2; q <= qlast; ++q) acc = M::mma(a[q], tf[2 * q - j + 1], acc);
                typename M::V4 o;
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = M::cvt(acc[v]);
                *(typename M::V4 *)(yb + (16 * j + li) * kPitch + 16 * wave + 4 * lg) = o;
            }
            __builtin_amdgcn_s_setprio(0);
        };
        // Row pass of plane n from ybuf[n & 1]: the lane's filtered values z.
        auto row_pass = [&](int n, mf_f4 (&z)[JB]) {
            const E *src = ybuf + ((n + base) & (kBufs - 1)) * kYElems + (16 * rb + li) * kPitch + 8 * lg;
            if constexpr (JB == 2) {
                V ya[QB + 1];
#pragma unroll
                for (int q = 0; q <= QB; ++q) ya[q] = ld_frag<M>(src + 32 * (q + p));
                mf_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q <= QA; ++q) acc0 = M::mma(ya[q], tf[2 * q + 1], acc0);
#pragma unroll
                for (int q = 0; q <= QB; ++q) acc1 = M::mma(ya[q], tf[2 * q], acc1);
                z[0] = acc0;
                z[JB - 1] = acc1;
            } else {
                // p is uniform: one branch per wave, no fragment selected per lane
                src += 32 * (p >> 1);
                mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
                if ((p & 1) == 0) {
#pragma unroll
                    for (int q = 0; q <= QA; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q + 1], acc);
                } else {
#pragma unroll
                    for (int q = 0; q <= QB; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q], acc);
                }
                z[0] = acc;
            }
        };
        // Eqs. 8-9 for plane n >= 1 (pw = s^n on entry).
        auto combine = [&](int n, const mf_f4 (&z)[JB]) {
            const float bp = bt[n - 1];
            const float bq = bt[n];
#pragma unroll
            for (int b = 0; b < JB; ++b) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float u = pw[b][v] * z[b][v];
                    Ps[b][v] = fmaf(bp, u, Ps[b][v]);
                    Qa[b][v] = fmaf(bq, u, Qa[b][v]);
                    pw[b][v] *= sc[b][v];
                }
            }
        };

        // Eq. 9's first term (plane 0).
        auto first = [&](const mf_f4 (&z)[JB]) {
            const float b0 = bt[0];
#pragma unroll
            for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) Qa[b][v] = b0 * z[b][v];
        };
        if constexpr (kBufs == 4) {
            // Software pipeline, two planes per phase: the row passes of
            // planes 2k-2, 2k-1 and the column passes of 2k, 2k+1 sit between
            // the same two barriers (four LDS buffers), which halves the
            // barriers of a 16-wave block.
            column_pass(0);
            column_pass(1);
            lds_barrier();
            for (int k = 1; 2 * k - 2 < P; ++k) {
                if (2 * k < P) column_pass(2 * k);
                if (2 * k + 1 < P) column_pass(2 * k + 1);
                {
                    mf_f4 z[JB];
                    row_pass(2 * k - 2, z);
                    if (k == 1) first(z);
                    else combine(2 * k - 2, z);
                }
                if (2 * k - 1 < P) {
                    mf_f4 z[JB];
                    row_pass(2 * k - 1, z);
                    combine(2 * k - 1, z);
                }
                if (2 * k < P) lds_barrier();
            }
        } else {
            // Software pipeline: the row pass of plane n-1 and the column pass of
            // plane n sit between the same two barriers (different LDS buffers).
            column_pass(0);
            lds_barrier();
            column_pass(1);
            {
                mf_f4 z[JB];
                row_pass(0, z);
                first(z);
            }
            lds_barrier();
            for (int n = 2; n < P; ++n) {
                column_pass(n);
                mf_f4 z[JB];
                row_pass(n - 1, z);
                combine(n - 1, z);
                lds_barrier();
            }
            {
                mf_f4 z[JB];
                row_pass(P - 1, z);
                combine(P - 1, z);
            }
        }

#pragma unroll
        for (int b = 0; b < JB; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // a reduced-precision stack: the reciprocal's ulp is far below its error
                const float ratio = Ps[b][v] * __frcp_rn(sc[b][v] * Qa[b][v]);
                y[b][v] = C.yo + C.ys * ratio;                                   // eq. (10)
            }
        }
    }

    // The sums' start from the lane's output pixels cpx (s, the running s^n,
    // Ps = 0), and their range check (every pixel of the image is the output
    // of exactly one lane of one tile) to flag / slot.
    __device__ __forceinline__ void start_sums(const float (&cpx)[JB][4], const FusedCentre &C, float (&sc)[JB][4],
                                               float (&pw)[JB][4], float (&Ps)[JB][4], unsigned *__restrict__ flag,
                                               unsigned *__restrict__ slot) const {
        bool bad = false;
#pragma unroll
        for (int b = 0; b < JB; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                bad |= !(cpx[b][v] >= 0.0f && cpx[b][v] <= 255.0f);
                const float s = fmaf(cpx[b][v], C.sc, C.oc);
                sc[b][v] = s != 0.0f ? s : 0x1p-64f;
                pw[b][v] = sc[b][v];
                Ps[b][v] = 0.0f;
            }
        }
        report_range(bad, flag, slot);
    }

    // filter() for the strip kernel (FP16 state, four LDS buffers), on a
    // state S it keeps between tiles (H advances, s is kept), with three
    // changes that leave every value as filter() has it: H_n is the MFMA
    // operand in place and becomes H_{n+1} after the column pass's products
    // (fewer registers); the lane's output pixels cpx are first read after
    // the first barrier, where their range check goes to flag / slot; and
    // hook(k) runs at the start of each barrier phase k >= 1, all waves
    // together (k uniform). (A separate function: as one body with filter(),
    // the other geometries lose registers.)
    template <class Hook>
    __device__ __forceinline__ void strip_planes(State &S, const float (&cpx)[JB][4], const FusedCentre &C,
                                                 const float *__restrict__ bt, int N, int base, float (&y)[JB][4],
                                                 unsigned *__restrict__ flag, unsigned *__restrict__ slot,
                                                 Hook &&hook) {
        static_assert(kH16 && kBufs == 4, "FP16 plane state, four LDS buffers");
        const int P = N + 2;

        // With u_n = s^n Hbar_n the sums are accumulated as
        //   Q = sum_n b_n u_n,   Ps = sum_n b_{n-1} u_n = s P,
        // so one product serves both, and P = Ps / s. Where s = 0 the sums take
        // s = 2^-64 instead: Ps / s is then b_0 Hbar_1, the value of P at s = 0,
        // up to terms 2^-64 smaller, and Q moves by as little. (Where b_0 2^-64
        // Hbar_1 underflows, P/Q lies far below FP32 resolution: the pixel's own
        // term keeps Q >= w_0 b_0 2^K.) Set in first().
        float sc[JB][4], pw[JB][4], Ps[JB][4], Qa[JB][4];

        // Column pass of plane n into its LDS buffer; advances H to plane n+1.
        // Waves past kNCW hold no halo columns the row pass reads.
        auto column_pass = [&](int n) {
            if (kNCW < NW && wave >= kNCW) return;
            E *yb = ybuf + ((n + base) & (kBufs - 1)) * kYElems;
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int j = 0; j < kNRB; ++j) {
                const int qlast = min(Q - 1, j / 2 + ((j & 1) ? QB : QA));
                mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = j / 2; q <= qlast; ++q) acc = M::mma(S.hv16[q], tf[2 * q - j + 1], acc);
                typename M::V4 o;
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = M::cvt(acc[v]);
                *(typename M::V4 *)(yb + (16 * j + li) * kPitch + 16 * wave + 4 * lg) = o;
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int q = 0; q < Q; ++q) S.hv16[q] = S.hv16[q] * S.sv16[q];          // H_{n+1} = H_n s
        };
        // Row pass of plane n from ybuf[n & 1]: the lane's filtered values z.
        auto row_pass = [&](int n, mf_f4 (&z)[JB]) {
            const E *src = ybuf + ((n + base) & (kBufs - 1)) * kYElems + (16 * rb + li) * kPitch + 8 * lg;
            if constexpr (JB == 2) {
                V ya[QB + 1];
#pragma unroll
                for (int q = 0; q <= QB; ++q) ya[q] = ld_frag<M>(src + 32 * (q + p));
                mf_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q <= QA; ++q) acc0 = M::mma(ya[q], tf[2 * q + 1], acc0);
#pragma unroll
                for (int q = 0; q <= QB; ++q) acc1 = M::mma(ya[q], tf[2 * q], acc1);
                z[0] = acc0;
                z[JB - 1] = acc1;
            } else {
                // p is uniform: one branch per wave, no fragment selected per lane
                src += 32 * (p >> 1);
                mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
                if ((p & 1) == 0) {
#pragma unroll
                    for (int q = 0; q <= QA; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q + 1], acc);
                } else {
#pragma unroll
                    for (int q = 0; q <= QB; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q], acc);
                }
                z[0] = acc;
            }
        };
        // Eqs. 8-9 for plane n >= 1 (pw = s^n on entry).
        auto combine = [&](int n, const mf_f4 (&z)[JB]) {
            const float bp = bt[n - 1];
            const float bq = bt[n];
#pragma unroll
            for (int b = 0; b < JB; ++b) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float u = pw[b][v] * z[b][v];
                    Ps[b][v] = fmaf(bp, u, Ps[b][v]);
                    Qa[b][v] = fmaf(bq, u, Qa[b][v]);
                    pw[b][v] *= sc[b][v];
                }
            }
        };

        // Eq. 9's first term (plane 0).
        auto first = [&](const mf_f4 (&z)[JB]) {
            start_sums(cpx, C, sc, pw, Ps, flag, slot);
            const float b0 = bt[0];
#pragma unroll
            for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) Qa[b][v] = b0 * z[b][v];
        };
        // Software pipeline, two planes per phase, as in filter().
        column_pass(0);
        column_pass(1);
        lds_barrier();
        for (int k = 1; 2 * k - 2 < P; ++k) {
            hook(k);
            if (2 * k < P) column_pass(2 * k);
            if (2 * k + 1 < P) column_pass(2 * k + 1);
            {
                mf_f4 z[JB];
                row_pass(2 * k - 2, z);
                if (k == 1) first(z);
                else combine(2 * k - 2, z);
            }
            if (2 * k - 1 < P) {
                mf_f4 z[JB];
                row_pass(2 * k - 1, z);
                combine(2 * k - 1, z);
            }
            if (2 * k < P) lds_barrier();
        }

#pragma unroll
        for (int b = 0; b < JB; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // a reduced-precision stack: the reciprocal's ulp is far below its error
                const float ratio = Ps[b][v] * __frcp_rn(sc[b][v] * Qa[b][v]);
                y[b][v] = C.yo + C.ys * ratio;                                   // eq. (10)
            }
        }
    }

    __device__ __forceinline__ void store(int r0, int c0, const float (&y)[JB][4]) const {
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const int c = c0 + 16 * (jc0 + b) + li;
            if (c >= Wd) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 16 * rb + 4 * lg + v;
                if (r < H) out[(long long)r * ld + c] = y[b][v];
            }
        }
    }
    // store() by 32-bit byte offsets: H ld < 2^29. ln: the lane index.
    __device__ __forceinline__ void store32(int r0, int c0, const float (&y)[JB][4], int ln) const {
        char *base = (char *)out;
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const int c = c0 + 16 * (jc0 + b) + (ln & 15);
            if (c >= Wd) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 16 * rb + 4 * (ln >> 4) + v;
                if (r < H) *(float *)(base + 4u * (unsigned)(r * ld + c)) = y[b][v];
            }
        }
    }

    // The filter of eqs. (6)-(10) centred at t_c with half range t_h.
    __device__ __forceinline__ FusedCentre plain_centre() const {
        FusedCentre C;
        C.sb = C.sc = (float)(1.0 / kTh);
        C.ob = C.oc = (float)(-kTc / kTh);
        C.e2 = -0.5f * mu * 1.4426950408889634f;
        C.k2 = __log2f(prescale);
        C.ys = (float)kTh;
        C.yo = (float)kTc;
        return C;
    }
    __device__ __forceinline__ void run(int r0, int c0, const Raw &R, unsigned *__restrict__ flag,
                                        unsigned *__restrict__ slot, int base = 0) {
        const FusedCentre C = plain_centre();
        check_range(R, flag, slot);
        float y[JB][4];
        filter(R, C, bt, N, base, y);
        store(r0, c0, y);
    }

    // Mask of the sub-ranges present among the tile's output pixels (the
    // lane's pixels, clamped into the image as load() reads them), or-ed over
    // the block through m2 (two LDS words, zero on entry); one barrier. The
    // same set k_pivot_masks finds for the tile.
    __device__ __forceinline__ unsigned long long pivot_mask(const Raw &R, const float *lo, int K, float kscale,
                                                             unsigned *m2) const {
        unsigned long long m = 0;
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) m |= 1ull << pivot_of(R.c[b][v], lo, K, kscale);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m |= __shfl_xor(m, off);
        if (lane == 0) {
            if ((unsigned)m) atomicOr(&m2[0], (unsigned)m);
            if ((unsigned)(m >> 32)) atomicOr(&m2[1], (unsigned)(m >> 32));
        }
        __syncthreads();
        return ((unsigned long long)__builtin_amdgcn_readfirstlane(m2[1]) << 32) |
               (unsigned)__builtin_amdgcn_readfirstlane(m2[0]);
    }

    // Pivoted form: the sub-range of each of the lane's output pixels
    // (pivot_of), then the planes of each sub-range in the tile's mask (every
    // sub-range some output pixel of the tile falls in, uniform), every pixel
    // keeping the outputs of its own. lo: the sub-ranges' lower ends in LDS;
    // base: buffer parity, continued from tile to tile.
    __device__ __forceinline__ void run_pivots(int r0, int c0, const Raw &R, const FusedPivot *__restrict__ piv,
                                               const float *__restrict__ coef, int K, float kscale,
                                               const float *lo, unsigned long long todo,
                                               unsigned *__restrict__ flag, unsigned *__restrict__ slot,
                                               int &base) {
        check_range(R, flag, slot);
        int kb[JB][4];
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) kb[b][v] = pivot_of(R.c[b][v], lo, K, kscale);
        float y[JB][4] = {};
        while (todo) {
            const int k = __builtin_amdgcn_readfirstlane(__ffsll(todo) - 1);
            todo &= todo - 1;
            const FusedPivot &Pk = piv[k];
            const int Nk = Pk.N;
            float yk[JB][4];
            filter(R, Pk.c, coef + Pk.boff, Nk, base, yk);
            base += Nk + 2;
#pragma unroll
            for (int b = 0; b < JB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (kb[b][v] == k) y[b][v] = yk[b][v];
        }
        store(r0, c0, y);
    }
};

// Whether the single-image fused kernel of a geometry is persistent with
// prefetch (see k_fused_mfma): where one block per tile would not fit two
// blocks per CU anyway (BF16, with its FP32 plane state, at Q >= 4; FP16
// fits everywhere, 92-126 VGPRs).
template <class M>
__host__ __device__ constexpr bool fused_persistent(int Q) { return !M::kHalfPlanes && Q >= 4; }

// Single-image fused kernel over the tiles_x-wide grid of TR x TC tiles,
// NW waves per block (FusedTile).
// Where a block needs more than 128 VGPRs (one block per CU) it is
// persistent: block b takes tiles b, b + grid, ..., makes the fragments once,
// and loads the inputs of its next tile while the current one runs, so that
// no block waits for its halo at the start of a tile. Where one block per
// tile fits in 128 (FP16, and BF16 with Q = 3: 92-126 VGPRs) the
// registers of that prefetch would cost the second block per CU, which hides
// those loads instead (and runs the other block's VALU work beside this
// one's matrix-core work): one block per tile.
template <class M, int Q, int TC, int QA, int NW = 8, int TR = kFusedRows>
__global__ __launch_bounds__(NW * 64) void k_fused_mfma(const float *__restrict__ f, float *__restrict__ out, int H,
                                                        int Wd, int ld, FusedConsts C, int W, int N, float mu,
                                                        float prescale, unsigned *__restrict__ slots, int tiles_x,
                                                        int tiles) {
    typedef typename M::E E;
    typedef FusedTile<M, Q, TC, QA, NW, TR> T;
    __shared__ __align__(16) E ybuf[T::kBufs * T::kYElems];
    __shared__ E tab[fused_tab_len(Q)];
    T tile(f, out, H, Wd, ld, W, N, mu, prescale, C.b, ybuf);
    tile.setup(C.taps, tab);
    if constexpr (!fused_persistent<M>(Q) || NW != 8) {
        const int t = blockIdx.x;
        const int r0 = (t / tiles_x) * TR, c0 = (t % tiles_x) * TC;
        typename T::Raw cur;
        tile.load(r0, c0, cur);
        tile.run(r0, c0, cur, nullptr, slots + T::kSlots * t);
    } else {
        typename T::Raw next;
        int t = blockIdx.x;
        int base = 0;
        if (t < tiles) tile.load((t / tiles_x) * kFusedRows, (t % tiles_x) * TC, next);
        for (; t < tiles; t += gridDim.x) {
            const int r0 = (t / tiles_x) * kFusedRows, c0 = (t % tiles_x) * TC;
            const typename T::Raw cur = next;
            const int tn = t + gridDim.x;
            if (tn < tiles) tile.load((tn / tiles_x) * kFusedRows, (tn % tiles_x) * TC, next);
            tile.run(r0, c0, cur, nullptr, slots + kFusedSlots * t, base);
            base += N + 2;
        }
    }
}

// Single-image fused kernel on vertical strips of tiles (FP16 plane state,
// 64-row tiles on 16 waves, four LDS buffers): block b filters up to
// strip_len tiles of one tile column, top to bottom. Consecutive tiles share
// 2W halo rows, and with 64-row tiles and 32-row chunks the next tile's
// chunks 0..Q-3 are this tile's chunks 2..Q-1: each lane keeps their s (FP16)
// in its registers and their H_0 in its own LDS slots (written when the tile
// starts, before H advances), and loads only the two new chunks, 64 halo rows.
// Those loads go out in eight slices of two values during the plane loop,
// each one barrier phase before its s is written to the lane's LDS slots (no
// other lane reads any of them); the loop's barriers do not wait for them.
// (Where those rows reach the image's last row, the loads wait for the
// tile's end.)
// When the next tile starts the lane reads them back and takes H_0 of the
// new s: the state build_state gives for the same halo. Its output pixels
// are loaded then and first read after its first barrier. The strip's first
// tile loads its whole halo, before the tap setup. Images with W < H and
// W < Wd (one reflection at the edges) and H ld < 2^29 (32-bit byte offsets)
// only.
template <class M, int Q, int TC, int QA>
__global__ __launch_bounds__(1024) void k_fused_strip(const float *__restrict__ f, float *__restrict__ out, int H,
                                                      int Wd, int ld, FusedConsts C, int W, int N, float mu,
                                                      float prescale, unsigned *__restrict__ slots, int tiles_x,
                                                      int tiles_y, int strip_len) {
    typedef typename M::E E;
    typedef typename M::V V;
    typedef typename M::E E2 __attribute__((ext_vector_type(2)));
    typedef FusedTile<M, Q, TC, QA, 16, kFusedRows> T;
    static_assert(M::kHalfPlanes && T::kBufs == 4 && Q >= 3, "FP16 plane state, 64-row tiles on 16 waves");
    constexpr int kLanes = T::kNCW * 64;         // column-wave lanes
    constexpr int kSlices = 8;                   // two values each: new chunk sl / 4, rows 2 (sl % 4), +1
    constexpr int kKept = Q - 2;                 // chunks the next tile takes over
    __shared__ __align__(16) E ybuf[T::kBufs * T::kYElems];
    __shared__ E tab[fused_tab_len(Q)];
    __shared__ __align__(16) E2 s_new[kSlices * kLanes];
    __shared__ __align__(16) V h_kept[kKept * kLanes];
    T tile(f, out, H, Wd, ld, W, N, mu, prescale, C.b, ybuf);
    tile.one_ref = true;                         // W < H and W < Wd here
    // Strip order: blocks go to the 8 XCDs in turn (block b to XCD b mod 8);
    // each XCD takes a contiguous range of strips in row-major order, so
    // strips side by side, which share 2W halo columns, run in one L2.
    const int G = gridDim.x, gq = G / 8, gr = G % 8, xcd = blockIdx.x % 8;
    const int strip = xcd * gq + min(xcd, gr) + blockIdx.x / 8;
    const int cx = strip % tiles_x;
    const int ty0 = (strip / tiles_x) * strip_len;
    const int ty1 = min(ty0 + strip_len, tiles_y);
    const int c0 = cx * TC;
    const bool colw = tile.wave < T::kNCW;       // uniform
    typename T::Raw R;
    tile.load(ty0 * kFusedRows, c0, R);
    tile.setup(C.taps, tab);
    const FusedCentre Cn = tile.plain_centre();
    typename T::State S;
    tile.build_state(R.h, Cn, S);
    int base = 0;
    for (int ty = ty0; ty < ty1; ++ty) {
        const int r0 = ty * kFusedRows;
        const bool more = ty + 1 < ty1;
        // The lane's indices, from a copy of threadIdx.x the compiler cannot
        // see through: they are made again for each tile instead of being
        // held in registers across the plane loop.
        unsigned tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63;
        const int lg = lane >> 4;
        if (more && colw) {
#pragma unroll
            for (int q = 0; q < kKept; ++q) h_kept[q * kLanes + tid] = S.hv16[q + 2];
        }
        // halo column of a lane (lane index l)
        auto col_of = [&](int l) { return halo_index(c0 - W + 16 * tile.wave + (l & 15), Wd, W, true); };
        // first new halo row of the next tile; all its new rows inside the image or not (uniform)
        const int rb0 = r0 + kFusedRows - W + 32 * (Q - 2);
        const bool inside = rb0 + 63 < H;
        const unsigned lane_off = 4u * (unsigned)(8 * lg * ld + col_of(lane));
        float pf[2];
        int issued = 0, written = 0;
        auto load_slice = [&](int sl) {
            const int r = rb0 + 32 * (sl >> 2) + 2 * (sl & 3);
            if (inside) {
                const char *row = (const char *)f + 4u * (unsigned)(r * ld);
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
                    pf[jj] = *(const float *)(row + 4u * (unsigned)(jj * ld) + lane_off);
            } else {
                const int l = fresh_lane_id();
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
                    pf[jj] = *(const float *)((const char *)f +
                                              4u * (unsigned)(halo_index(r + 8 * (l >> 4) + jj, H, W, true) * ld +
                                                              col_of(l)));
            }
        };
        auto write_slice = [&](int sl) {
            E2 o;
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) o[jj] = T::s16_of(pf[jj], Cn);
            s_new[sl * kLanes + 64 * tile.wave + fresh_lane_id()] = o;
        };
        // (where the next tile's new rows reach the image's last row, all the
        // loads wait for the tile's end)
        auto hook = [&](int k) {
            if (!more || !colw || !inside) return;
            if (issued > written) {
                write_slice(written);
                ++written;
            }
            if (k >= 2 && issued < kSlices) {
                load_slice(issued);
                ++issued;
            }
        };
        float y[T::JB][4];
        tile.strip_planes(S, R.c, Cn, tile.bt, N, base, y, nullptr, slots + T::kSlots * (ty * tiles_x + cx), hook);
        {
            unsigned t2 = threadIdx.x;
            asm volatile("" : "+v"(t2));
            tile.store32(r0, c0, y, t2 & 63);
        }
        base += N + 2;
        if (more) {
            if (colw) {
                for (; written < kSlices; ++written) {
                    if (issued == written) {
                        load_slice(issued);
                        ++issued;
                    }
                    write_slice(written);
                }
                unsigned t3 = threadIdx.x;
                asm volatile("" : "+v"(t3));
#pragma unroll
                for (int q = 0; q < kKept; ++q) {
                    S.sv16[q] = S.sv16[q + 2];
                    S.hv16[q] = h_kept[q * kLanes + t3];
                }
#pragma unroll
                for (int sl = 0; sl < kSlices; ++sl) {
                    const E2 v = s_new[sl * kLanes + t3];
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        const int q = kKept + (sl >> 2), e = 2 * (sl & 3) + jj;
                        S.sv16[q][e] = v[jj];
                        S.hv16[q][e] = M::cvt(T::h0_of((float)v[jj], Cn));
                    }
                }
            }
            tile.load_pixels(r0 + kFusedRows, c0, R.c, lane);
        }
    }
}

// The or of `words` range words into *flag (one block of 256 threads; a
// plain store of 0 or BF_DEVFLAG_RANGE, so *flag needs no clearing).
__global__ __launch_bounds__(256) void k_or_range_words(const unsigned *__restrict__ words, int count,
                                                        unsigned *__restrict__ flag) {
    __shared__ unsigned s_or;
    if (threadIdx.x == 0) s_or = 0u;
    __syncthreads();
    unsigned acc = 0u;
    for (int i = threadIdx.x; i < count; i += blockDim.x) acc |= words[i];
    if (acc) atomicOr(&s_or, acc);
    __syncthreads();
    if (threadIdx.x == 0) *flag = s_or;
}

// Pivoted form on the fused tile, in three launches.
// k_pivot_masks: the mask of the sub-ranges present among each tile's output
// pixels (one block of 256 threads per tile).
template <int TC>
__global__ __launch_bounds__(256) void k_pivot_masks(const float *__restrict__ f, int H, int Wd, int ld,
                                                     const FusedPivot *__restrict__ piv, int K, float kscale,
                                                     int tiles_x, unsigned long long *__restrict__ masks) {
    __shared__ float s_lo[BF_MAX_PIVOTS];
    __shared__ unsigned s_mask[2];
    for (int i = threadIdx.x; i < K; i += blockDim.x) s_lo[i] = piv[i].lo;
    if (threadIdx.x < 2) s_mask[threadIdx.x] = 0u;
    __syncthreads();
    const int t = blockIdx.x;
    const int r0 = (t / tiles_x) * kFusedRows, c0 = (t % tiles_x) * TC;
    // thread i takes column i % TC of rows i / TC + (256 / TC) j; all loads
    // first, then the classification
    constexpr int kRowsPer = 256 / TC, kSteps = kFusedRows / kRowsPer;
    const int c = min(c0 + (int)threadIdx.x % TC, Wd - 1), rr = threadIdx.x / TC;
    float x[kSteps];
#pragma unroll
    for (int j = 0; j < kSteps; ++j) x[j] = f[(long long)min(r0 + rr + kRowsPer * j, H - 1) * ld + c];
    unsigned long long m = 0;
#pragma unroll
    for (int j = 0; j < kSteps; ++j) m |= 1ull << pivot_of(x[j], s_lo, K, kscale);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m |= __shfl_xor(m, off);
    if ((threadIdx.x & 63) == 0) {
        if ((unsigned)m) atomicOr(&s_mask[0], (unsigned)m);
        if ((unsigned)(m >> 32)) atomicOr(&s_mask[1], (unsigned)(m >> 32));
    }
    __syncthreads();
    if (threadIdx.x == 0) masks[t] = ((unsigned long long)s_mask[1] << 32) | s_mask[0];
}

// k_pivot_order (one block of 1024 threads): the tiles ordered by the number
// of sub-ranges they run, most first (a counting sort; order within a count
// is arbitrary and does not change any output), and the queue counter reset.
__global__ __launch_bounds__(1024) void k_pivot_order(const unsigned long long *__restrict__ masks, int tiles,
                                                      int *__restrict__ order, int *__restrict__ counter) {
    __shared__ int s_cnt[BF_MAX_PIVOTS + 1];
    for (int i = threadIdx.x; i <= BF_MAX_PIVOTS; i += blockDim.x) s_cnt[i] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < tiles; t += blockDim.x) atomicAdd(&s_cnt[__popcll(masks[t])], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int at = 0;
        for (int c = BF_MAX_PIVOTS; c >= 0; --c) {
            const int n = s_cnt[c];
            s_cnt[c] = at;
            at += n;
        }
        *counter = 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < tiles; t += blockDim.x) order[atomicAdd(&s_cnt[__popcll(masks[t])], 1)] = t;
}

// k_fused_pivots: persistent blocks take tiles from the queue (order,
// counter) and run each one's sub-ranges (FusedTile::run_pivots). Where the
// registers allow (Q <= 4) a block loads the next tile's inputs while the
// current one runs. piv: K sub-ranges; coef: their coefficients; taps: w[t],
// t = 0..2W (all in device memory).
template <class M, int Q, int TC, int QA>
__global__ __launch_bounds__(512) void k_fused_pivots(const float *__restrict__ f, float *__restrict__ out, int H,
                                                      int Wd, int ld, const FusedPivot *__restrict__ piv,
                                                      const float *__restrict__ coef, const float *__restrict__ taps,
                                                      int K, float kscale, int W, unsigned *__restrict__ slots,
                                                      int tiles_x, int tiles,
                                                      const unsigned long long *__restrict__ masks,
                                                      const int *__restrict__ order, int *__restrict__ counter) {
    typedef typename M::E E;
    typedef FusedTile<M, Q, TC, QA> T;
    constexpr bool kPrefetch = Q <= 4;
    __shared__ __align__(16) E ybuf[2 * kFusedYElems];
    __shared__ E tab[fused_tab_len(Q)];
    __shared__ float s_lo[BF_MAX_PIVOTS];
    __shared__ int s_ticket[2];
    T tile(f, out, H, Wd, ld, W, 0, 0.0f, M::kPrescale, nullptr, ybuf);
    for (int i = threadIdx.x; i < K; i += blockDim.x) s_lo[i] = piv[i].lo;
    // Ticket slot j & 1 is written at the top of step j and read after the
    // barrier that follows; the tile's own barriers separate those reads
    // from the write of step j + 2.
    if (threadIdx.x == 0) s_ticket[0] = atomicAdd(counter, 1);
    tile.setup(taps, tab);                     // its barrier also publishes s_lo and s_ticket[0]
    int ticket = __builtin_amdgcn_readfirstlane(s_ticket[0]);
    if (ticket >= tiles) return;
    int t = __builtin_amdgcn_readfirstlane(order[ticket]);
    typename T::Raw cur;
    tile.load((t / tiles_x) * kFusedRows, (t % tiles_x) * TC, cur);
    int base = 0;
    for (int step = 1;; ++step) {
        if (threadIdx.x == 0) s_ticket[step & 1] = atomicAdd(counter, 1);
        __syncthreads();
        ticket = __builtin_amdgcn_readfirstlane(s_ticket[step & 1]);
        const int tn = ticket < tiles ? __builtin_amdgcn_readfirstlane(order[ticket]) : -1;
        const int r0 = (t / tiles_x) * kFusedRows, c0 = (t % tiles_x) * TC;
        const unsigned long long m = masks[t];
        const unsigned long long todo =
            ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(m >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((unsigned)m);
        if constexpr (kPrefetch) {
            typename T::Raw next;
            if (tn >= 0) tile.load((tn / tiles_x) * kFusedRows, (tn % tiles_x) * TC, next);
            tile.run_pivots(r0, c0, cur, piv, coef, K, kscale, s_lo, todo, nullptr, slots + kFusedSlots * t, base);
            cur = next;
        } else {
            tile.run_pivots(r0, c0, cur, piv, coef, K, kscale, s_lo, todo, nullptr, slots + kFusedSlots * t, base);
            if (tn >= 0) tile.load((tn / tiles_x) * kFusedRows, (tn % tiles_x) * TC, cur);
        }
        if (tn < 0) break;
        t = tn;
    }
}

// Joint filter on the matrix cores: the plain tile's schedule with two operand
// sets per plane, A_n = 2^K e^{-mu s^2/2} s^n (s from the guide g) and
// B_n = A_n ft (ft = (v - t_c)/t_h from the averaged image v), both filtered
// (two MFMA chains per block, two LDS buffers per plane), then
// Q = sum b_n s_i^n Abar_n, P = sum b_n s_i^n Bbar_n, y = t_c + t_h P/Q.
// Planes n = 0..N. Geometries as the plain tile: 64-column tiles for
// radius <= 32, 32-column tiles (Q = 5) for radius <= 48.
template <class M, int Q, int TC, int QA>
__device__ __forceinline__ void fused_joint_tile(const float *__restrict__ g, const float *__restrict__ v,
                                                 float *__restrict__ out, int H, int Wd, int ld,
                                                 const float *__restrict__ taps, const float *__restrict__ bt,
                                                 int W, int N, float mu, float prescale,
                                                 unsigned *__restrict__ slot, int r0, int c0,
                                                 typename M::E *__restrict__ ybuf_base,
                                                 typename M::E *__restrict__ tab) {
    typedef typename M::E E;
    typedef typename M::V V;
    constexpr int QB = Q - 2;
    constexpr int JB = TC / 32;                 // output column blocks per wave in the row pass
    constexpr int kTabPad = kFusedTabPad;
    constexpr int kTab = fused_tab_len(Q);
    static_assert((TC == 64 && Q <= 4) || (TC == 32 && Q == 5), "joint geometry");
    static_assert(QA == Q - 3 || QA == Q - 2, "chunk range");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    for (int i = threadIdx.x; i < kTab; i += blockDim.x) {
        const int t = i - kTabPad;
        tab[i] = M::cvt(t >= 0 && t <= 2 * W ? taps[t] : 0.0f);
    }
    __syncthreads();
    V tf[2 * Q];
#pragma unroll
    for (int d = -1; d < 2 * Q - 1; ++d)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) tf[d + 1][jj] = tab[kTabPad + 16 * d + 8 * lg + jj - li];
    const int rb = wave >> 1;
    const int p = wave & 1;
    const int jc0 = p * JB;

    const bool one_ref = W < H && W < Wd;
    const int mc = halo_index(c0 - W + 16 * wave + li, Wd, W, one_ref);
    const int cr = r0 + 16 * rb + 4 * lg;                        // first output row of the lane
    // Inputs: halo column values of g and v, and the lane's own output pixels
    // (as in FusedTile::load: one add per load where everything lies inside
    // the image and byte offsets fit 32 bits).
    float gx[Q][8], vx[Q][8], gc[JB][4], vc[JB][4];
    if (r0 - W >= 0 && r0 - W + 32 * Q <= H && r0 + kFusedRows <= H && (long long)H * ld < (1LL << 29)) {
        const unsigned o = 4u * (unsigned)((r0 - W + 8 * lg) * ld + mc), ld4 = 4u * (unsigned)ld;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const unsigned oo = o + (unsigned)(32 * q + jj) * ld4;
                gx[q][jj] = *(const float *)((const char *)g + oo);
                vx[q][jj] = *(const float *)((const char *)v + oo);
            }
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const unsigned oc = 4u * (unsigned)(cr * ld + min(c0 + 16 * (jc0 + b) + li, Wd - 1));
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                gc[b][vv] = *(const float *)((const char *)g + oc + (unsigned)vv * ld4);
                vc[b][vv] = *(const float *)((const char *)v + oc + (unsigned)vv * ld4);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const long long o = (long long)halo_index(r0 - W + 32 * q + 8 * lg + jj, H, W, one_ref) * ld + mc;
                gx[q][jj] = g[o];
                vx[q][jj] = v[o];
            }
#pragma unroll
        for (int b = 0; b < JB; ++b) {
            const int c = min(c0 + 16 * (jc0 + b) + li, Wd - 1);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const long long o = (long long)min(cr + vv, H - 1) * ld + c;
                gc[b][vv] = g[o];
                vc[b][vv] = v[o];
            }
        }
    }
    // s (eq. 17 on the guide) by one fma, 2^K e^{-mu s^2/2} by one exp2. FP16
    // (kHalfPlanes, as in FusedTile::State): s, ft and the running A_n held
    // in FP16, A_0 taken at the FP16 s, A_{n+1} = A_n s and B_n = A_n ft as
    // packed FP16 products.
    constexpr bool kH16 = M::kHalfPlanes;
    const float e2 = -0.5f * mu * 1.4426950408889634f, k2 = __log2f(prescale);
    float sv[kH16 ? 1 : Q][8], hv[kH16 ? 1 : Q][8], fv[kH16 ? 1 : Q][8];
    V sv16[kH16 ? Q : 1], hv16[kH16 ? Q : 1], fv16[kH16 ? Q : 1];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const float s = fmaf(gx[q][jj], (float)(1.0 / kTh), (float)(-kTc / kTh));
            const float ft = fmaf(vx[q][jj], (float)(1.0 / kTh), (float)(-kTc / kTh));
            if constexpr (kH16) {
                sv16[q][jj] = M::cvt(s);
                const float sr = (float)sv16[q][jj];
                hv16[q][jj] = M::cvt(__builtin_amdgcn_exp2f(fmaf(e2 * sr, sr, k2)));
                fv16[q][jj] = M::cvt(ft);
            } else {
                const float h0 = __builtin_amdgcn_exp2f(fmaf(e2 * s, s, k2));
                sv[q][jj] = s;
                hv[q][jj] = h0;
                fv[q][jj] = ft;
            }
        }
    // range check on the lane's own output pixels (each image pixel is one)
    bool bad = false;
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
            bad |= !(gc[b][vv] >= 0.0f && gc[b][vv] <= 255.0f) || !(vc[b][vv] >= 0.0f && vc[b][vv] <= 255.0f);
    report_range(bad, nullptr, slot);

    float sc[JB][4], pw[JB][4], Pa[JB][4], Qa[JB][4];
#pragma unroll
    for (int b = 0; b < JB; ++b) {
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            sc[b][vv] = fmaf(gc[b][vv], (float)(1.0 / kTh), (float)(-kTc / kTh));
            pw[b][vv] = 1.0f;
            Pa[b][vv] = 0.0f;
            Qa[b][vv] = 0.0f;
        }
    }
    // buffers: plane n's A result in buffer 2 (n & 1), its B result in 2 (n & 1) + 1
    auto column_pass = [&](int n) {
        V a[Q], bo[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if constexpr (kH16) {
                a[q] = hv16[q];
                bo[q] = hv16[q] * fv16[q];
                hv16[q] = hv16[q] * sv16[q];
            } else {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    a[q][jj] = M::cvt(hv[q][jj]);
                    bo[q][jj] = M::cvt(hv[q][jj] * fv[q][jj]);
                    hv[q][jj] *= sv[q][jj];
                }
            }
        }
        E *ya = ybuf_base + (2 * (n & 1)) * kFusedYElems;
        E *yb = ya + kFusedYElems;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int qlast = min(Q - 1, j / 2 + ((j & 1) ? QB : QA));
            mf_f4 acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = j / 2; q <= qlast; ++q) {
                acc = M::mma(a[q], tf[2 * q - j + 1], acc);
                accb = M::mma(bo[q], tf[2 * q - j + 1], accb);
            }
            typename M::V4 o, ob;
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                o[vv] = M::cvt(acc[vv]);
                ob[vv] = M::cvt(accb[vv]);
            }
            const int off = (16 * j + li) * kFusedPitch + 16 * wave + 4 * lg;
            *(typename M::V4 *)(ya + off) = o;
            *(typename M::V4 *)(yb + off) = ob;
        }
    };
    auto row_pass = [&](int n) {
        const E *base = ybuf_base + (2 * (n & 1)) * kFusedYElems + (16 * rb + li) * kFusedPitch + 8 * lg;
        mf_f4 z[2][JB];
#pragma unroll
        for (int set = 0; set < 2; ++set) {
            const E *src = base + set * kFusedYElems;
            if (TC == 64) {
                V ya[QB + 1];
#pragma unroll
                for (int q = 0; q <= QB; ++q) ya[q] = ld_frag<M>(src + 32 * (q + p));
                mf_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q <= QA; ++q) acc0 = M::mma(ya[q], tf[2 * q + 1], acc0);
#pragma unroll
                for (int q = 0; q <= QB; ++q) acc1 = M::mma(ya[q], tf[2 * q], acc1);
                z[set][0] = acc0;
                z[set][JB - 1] = acc1;
            } else {
                // the wave's column block p: fragment tf[2q + 1 - p] (uniform branch)
                mf_f4 acc = {0.f, 0.f, 0.f, 0.f};
                if (p == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q + 1], acc);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc = M::mma(ld_frag<M>(src + 32 * q), tf[2 * q], acc);
                }
                z[set][0] = acc;
            }
        }
        const float bn = bt[n];
#pragma unroll
        for (int b = 0; b < JB; ++b) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                Qa[b][vv] = fmaf(bn, pw[b][vv] * z[0][b][vv], Qa[b][vv]);
                Pa[b][vv] = fmaf(bn, pw[b][vv] * z[1][b][vv], Pa[b][vv]);
                pw[b][vv] *= sc[b][vv];
            }
        }
    };
    column_pass(0);
    __syncthreads();
    for (int n = 1; n <= N; ++n) {
        column_pass(n);
        row_pass(n - 1);
        __syncthreads();
    }
    row_pass(N);
#pragma unroll
    for (int b = 0; b < JB; ++b) {
        const int c = c0 + 16 * (jc0 + b) + li;
        if (c >= Wd) continue;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const int r = r0 + 16 * rb + 4 * lg + vv;
            if (r < H) out[(long long)r * ld + c] = (float)kTc + (float)kTh * (Pa[b][vv] * __frcp_rn(Qa[b][vv]));   // eq. (10)
        }
    }
}

template <class M, int Q, int TC, int QA>
__global__ __launch_bounds__(512) void k_fused_joint(const float *__restrict__ g, const float *__restrict__ v,
                                                     float *__restrict__ out, int H, int Wd, int ld,
                                                     FusedConsts C, int W, int N, float mu,
                                                     unsigned *__restrict__ slots) {
    typedef typename M::E E;
    __shared__ __align__(16) E ybuf[4 * kFusedYElems];
    __shared__ E tab[fused_tab_len(Q)];
    fused_joint_tile<M, Q, TC, QA>(g, v, out, H, Wd, ld, C.taps, C.b, W, N, mu, M::kPrescale,
                                   slots + kFusedSlots * (blockIdx.y * gridDim.x + blockIdx.x),
                                   blockIdx.y * kFusedRows, blockIdx.x * TC, ybuf, tab);
}

// Geometry classes of the fused kernel, in the order the batched form keeps
// them: (Q, TC, QA) = (3,64,0) (3,64,1) (4,64,1) (4,64,2) (5,32,2) (5,32,3).
__host__ __device__ constexpr int fused_class(int Q, int QA) { return 2 * (Q - 3) + (QA - (Q - 3)); }
__host__ __device__ constexpr int fused_class_of_radius(int W) {
    return W <= 16 ? fused_class(3, fused_qa(W)) : W <= 32 ? fused_class(4, fused_qa(W)) : fused_class(5, fused_qa(W));
}

// Batched fused kernel for the BF16 classes (FP32 plane state, one block per
// CU): persistent blocks take the class's (image, tile) items from
// a queue (the header's counter, in the order of the item numbering: images
// by decreasing cost), load the next item's inputs while the current one
// runs, and rebuild the tap fragments only when the image changes. Items are decoded as in k_batched; the tiles
// are the single-image kernel's, so every image matches its bf_gc_forward
// result bit for bit.
template <class M, int Q, int TC, int QA>
__global__ __launch_bounds__(512) void k_fused_batched(char *__restrict__ blob) {
    typedef typename M::E E;
    typedef FusedTile<M, Q, TC, QA> T;
    constexpr int C = fused_class(Q, QA);
    const float prescale = M::kPrescale;
    extern __shared__ long long s_start[];
    __shared__ __align__(16) E ybuf[2 * kFusedYElems];
    __shared__ E tab[fused_tab_len(Q)];
    __shared__ long long s_ticket[2];
    BatchHeader *hdr = (BatchHeader *)blob;
    const BatchImage *img = (const BatchImage *)(blob + sizeof(BatchHeader));
    const int count = hdr->count;
    int *s_order = (int *)(s_start + count);
    const long long *start = (const long long *)(blob + sizeof(BatchHeader) + sizeof(BatchImage) * count);
    const int *order = (const int *)(start + kBatchPhases * count);
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        s_start[k] = start[C * count + k];
        s_order[k] = order[C * count + k];
    }
    const long long items = hdr->items[C];
    long long *queue = &hdr->queue[C];
    unsigned *flags = as_global(&hdr->flags);
    // Ticket slot j & 1 is written at the top of step j and read after the
    // barrier that follows; the item's own barriers separate those reads
    // from the write of step j + 2.
    if (threadIdx.x == 0) s_ticket[0] = (long long)atomicAdd((unsigned long long *)queue, 1ull);
    __syncthreads();
    auto ticket_of = [&](int slot) {
        const long long v = s_ticket[slot];
        return ((long long)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
               (unsigned)__builtin_amdgcn_readfirstlane((int)v);
    };
    // item t -> image (uniform) and its tile
    auto decode = [&](long long t, int &ii, int &r0, int &c0) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        ii = __builtin_amdgcn_readfirstlane(s_order[lo]);
        const int l = (int)(t - s_start[lo]);
        const int gvx = uniform(img[ii].gvx);
        r0 = (l / gvx) * kFusedRows;
        c0 = (l % gvx) * TC;
    };
    auto make = [&](int ii) {
        const BatchImage &B = img[ii];
        const double *prm = as_global(uniform(B.prm));
        return T(as_global(uniform(B.f)), as_global(uniform(B.out)), uniform(B.H), uniform(B.Wd), uniform(B.ld),
                 uniform(B.W), uniform(B.N), (float)uniform(B.mu), prescale, (const float *)(prm + uniform(B.off_bf)),
                 ybuf);
    };
    auto taps_of = [&](int ii) {
        const double *prm = as_global(uniform(img[ii].prm));
        return (const float *)(prm + uniform(img[ii].off_tf));
    };
    long long t = ticket_of(0);
    if (t >= items) return;
    int ii, r0, c0;
    decode(t, ii, r0, c0);
    T tile = make(ii);
    tile.setup(taps_of(ii), tab);
    typename T::Raw cur;
    tile.load(r0, c0, cur);
    int base = 0;
    for (int step = 1;; ++step) {
        if (threadIdx.x == 0) s_ticket[step & 1] = (long long)atomicAdd((unsigned long long *)queue, 1ull);
        __syncthreads();
        const long long tn = ticket_of(step & 1);
        int ni = -1, nr0 = 0, nc0 = 0;
        if (tn < items) decode(tn, ni, nr0, nc0);
        typename T::Raw next;
        if (tn < items) make(ni).load(nr0, nc0, next);
        tile.run(r0, c0, cur, flags, nullptr, base);
        cur = next;
        base += tile.N + 2;
        if (tn >= items) break;
        if (ni != ii) {
            tile = make(ni);
            tile.setup(taps_of(ni), tab);       // its barrier: every wave has read the old fragments long before
            ii = ni;
        }
        r0 = nr0;
        c0 = nc0;
    }
}

// Batched fused kernel for the FP16 classes, where the single-image kernel
// runs two blocks per CU: one block per (image, tile) item (grid = the
// class's items, set at every launch), as the single-image kernel, held to
// 128 VGPRs (four waves per SIMD: two blocks per CU; 94-124 used).
template <class M, int Q, int TC, int QA, int NW = 8>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_fused_batched_items(
    char *__restrict__ blob) {
    typedef typename M::E E;
    typedef FusedTile<M, Q, TC, QA, NW, kFusedRows, 2> T;
    constexpr int C = fused_class(Q, QA);
    const float prescale = M::kPrescale;
    extern __shared__ long long s_start[];
    __shared__ __align__(16) E ybuf[2 * T::kYElems];
    __shared__ E tab[fused_tab_len(Q)];
    BatchHeader *hdr = (BatchHeader *)blob;
    const long long t = blockIdx.x;
    if (t >= hdr->items[C]) return;
    const BatchImage *img = (const BatchImage *)(blob + sizeof(BatchHeader));
    const int count = hdr->count;
    int *s_order = (int *)(s_start + count);
    const long long *start = (const long long *)(blob + sizeof(BatchHeader) + sizeof(BatchImage) * count);
    const int *order = (const int *)(start + kBatchPhases * count);
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        s_start[k] = start[C * count + k];
        s_order[k] = order[C * count + k];
    }
    __syncthreads();
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int ii = __builtin_amdgcn_readfirstlane(s_order[lo]);
    const BatchImage &B = img[ii];
    const int l = (int)(t - s_start[lo]);
    const int gvx = uniform(B.gvx);
    const double *prm = as_global(uniform(B.prm));
    T tile(as_global(uniform(B.f)), as_global(uniform(B.out)), uniform(B.H), uniform(B.Wd), uniform(B.ld),
           uniform(B.W), uniform(B.N), (float)uniform(B.mu), prescale, (const float *)(prm + uniform(B.off_bf)), ybuf);
    tile.setup((const float *)(prm + uniform(B.off_tf)), tab);
    typename T::Raw raw;
    tile.load((l / gvx) * kFusedRows, (l % gvx) * TC, raw);
    tile.run((l / gvx) * kFusedRows, (l % gvx) * TC, raw, as_global(&hdr->flags), nullptr);
}

// Batched fused kernel for images routed to the pivoted form (their single
// expansion fails the conditioning check): one block per (image, tile) item
// of the class, as k_fused_batched_items. The block finds the sub-ranges its
// tile's output pixels fall in (FusedTile::pivot_mask, the set k_pivot_masks
// gives the single-image form) and runs them with the image's sub-range
// table (FusedTile::run_pivots), so each image equals its
// bf_gc_forward_pivots result bit for bit.
template <class M, int Q, int TC, int QA>
__global__ __launch_bounds__(512) void k_fused_batched_pivot_items(char *__restrict__ blob) {
    typedef typename M::E E;
    typedef FusedTile<M, Q, TC, QA> T;
    constexpr int C = kFusedClasses + fused_class(Q, QA);
    extern __shared__ long long s_start[];
    __shared__ __align__(16) E ybuf[2 * kFusedYElems];
    __shared__ E tab[fused_tab_len(Q)];
    __shared__ float s_lo[BF_MAX_PIVOTS];
    __shared__ unsigned s_mask[2];
    BatchHeader *hdr = (BatchHeader *)blob;
    const long long t = blockIdx.x;
    if (t >= hdr->items[C]) return;
    const BatchImage *img = (const BatchImage *)(blob + sizeof(BatchHeader));
    const int count = hdr->count;
    int *s_order = (int *)(s_start + count);
    const long long *start = (const long long *)(blob + sizeof(BatchHeader) + sizeof(BatchImage) * count);
    const int *order = (const int *)(start + kBatchPhases * count);
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        s_start[k] = start[C * count + k];
        s_order[k] = order[C * count + k];
    }
    if (threadIdx.x < 2) s_mask[threadIdx.x] = 0u;
    __syncthreads();
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int ii = __builtin_amdgcn_readfirstlane(s_order[lo]);
    const BatchImage &B = img[ii];
    const int l = (int)(t - s_start[lo]);
    const int gvx = uniform(B.gvx);
    const int K = uniform(B.K);
    const float kscale = __builtin_bit_cast(float, uniform(__builtin_bit_cast(int, B.kscale)));
    const double *prm = as_global(uniform(B.prm));
    const FusedPivot *piv = (const FusedPivot *)(prm + uniform(B.off_piv));
    for (int i = threadIdx.x; i < K; i += blockDim.x) s_lo[i] = piv[i].lo;
    T tile(as_global(uniform(B.f)), as_global(uniform(B.out)), uniform(B.H), uniform(B.Wd), uniform(B.ld),
           uniform(B.W), 0, 0.0f, M::kPrescale, nullptr, ybuf);
    tile.setup((const float *)(prm + uniform(B.off_tf)), tab);   // its barrier publishes s_lo
    const int r0 = (l / gvx) * kFusedRows, c0 = (l % gvx) * TC;
    typename T::Raw raw;
    tile.load(r0, c0, raw);
    const unsigned long long todo = tile.pivot_mask(raw, s_lo, K, kscale, s_mask);
    int base = 0;
    tile.run_pivots(r0, c0, raw, piv, (const float *)(prm + uniform(B.off_bf)), K, kscale, s_lo, todo,
                    as_global(&hdr->flags), nullptr, base);
}

}  // namespace bfgc
