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
// FP64, which issues at the same rate as unpacked FP32 on this GPU; the stack
// itself is stored in FP32, FP16 (scaled by 2^k_n) or BF16. Rounding of the
// stored planes is then the only per-plane error.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace bfgc
