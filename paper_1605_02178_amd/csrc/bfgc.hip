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

#include <climits>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "bfgc.h"
#include "device.hpp"
#include "plan.hpp"

namespace bfgc {

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

// Coefficient kind selected by the flags.
static int kind_of(unsigned flags) {
    return (flags & BF_FLAG_TAYLOR) ? kFitTaylor : (flags & BF_FLAG_MINIMAX) ? kFitMinimax : kFitChebyshev;
}

// The coefficient kind the flags select must be available for (sigma_r, N);
// checked whatever BF_FLAG_ALLOW_ILL_CONDITIONED says.
static bf_status check_kind(double sigma_r, int N, unsigned flags) {
    if ((flags & BF_FLAG_TAYLOR) && (flags & BF_FLAG_MINIMAX))
        return fail(BF_ERR_INVALID_ARG, "BF_FLAG_TAYLOR and BF_FLAG_MINIMAX exclude each other");
    if (flags & BF_FLAG_MINIMAX) {
        if (N > BF_MINIMAX_MAX_DEGREE) return fail(BF_ERR_UNSUPPORTED, "minimax fit: N above BF_MINIMAX_MAX_DEGREE");
        if (fit(sigma_r, N, kFitMinimax).b.empty())
            return fail(BF_ERR_UNSUPPORTED, "minimax fit: not resolvable in binary128 at this (sigma_r, N)");
    }
    return BF_OK;
}

// Tile configuration index from the flags: -1 when none is given, -2 if out of range.
static int tile_config_of(unsigned flags) {
    const unsigned c = (flags >> 8) & 0xfu;
    if (c == 0) return -1;
    return c - 1 < BF_TILE_CONFIGS ? (int)(c - 1) : -2;
}

constexpr int kJointFusedMaxRadius = BF_FUSED_MAX_RADIUS;   // the joint fused tile: the plain tile's geometries

// The fused matrix-core kernels cover FP16/BF16 stacks up to
// BF_FUSED_MAX_RADIUS; the single-image forward takes FP16 stacks up to
// BF_FUSED_F16_MAX_RADIUS.
static bool fused_applies(int dtype, double sigma_s) {
    return dtype != BF_STACK_F32 && radius_of(sigma_s) <= BF_FUSED_MAX_RADIUS;
}
static bool fused_forward_applies(int dtype, double sigma_s) {
    return fused_applies(dtype, sigma_s) || (dtype == BF_STACK_F16 && radius_of(sigma_s) <= BF_FUSED_F16_MAX_RADIUS);
}

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
    if (height > BF_MAX_SIDE || width > BF_MAX_SIDE) return fail(BF_ERR_UNSUPPORTED, "image side above BF_MAX_SIDE");
    if ((long long)height * lds_of(width) > (1LL << 40)) return fail(BF_ERR_UNSUPPORTED, "image too large");
    return BF_OK;
}

// Storage rounding unit of each stack type.
static double unit_roundoff(int dtype) {
    return dtype == BF_STACK_F32 ? std::ldexp(1.0, -24) : dtype == BF_STACK_F16 ? std::ldexp(1.0, -11)
                                                                                : std::ldexp(1.0, -8);
}

static bf_status check_conditioning(double sigma_r, int N, int dtype, unsigned flags) {
    bf_status st = check_kind(sigma_r, N, flags);
    if (st != BF_OK || (flags & BF_FLAG_ALLOW_ILL_CONDITIONED)) return st;
    const Fit &F = fit(sigma_r, N, kind_of(flags));
    if (!std::isfinite(F.kappa) || F.kappa * unit_roundoff(dtype) > 1e-2) {
        char buf[200];
        snprintf(buf, sizeof buf, "ill-conditioned: kappa=%.3g times the stack rounding unit exceeds 1e-2 "
                                  "(sigma_r=%g, N=%d)", F.kappa, sigma_r, N);
        return fail(BF_ERR_ILL_CONDITIONED, buf);
    }
    return BF_OK;
}

// Where the range flags of a workspace's last call sit: the flag word at its
// start (cleared by the parameter upload, or by the batched blob), or, after a
// single-image fused launch, one word per wave of each tile right after the
// flag area (every wave writes its word, so nothing is cleared first). The
// map holds the workspaces of the second kind with their word counts.
static std::mutex g_range_mtx;
static std::unordered_map<const void *, long long> g_range_words;
static void note_range_words(const void *ws, long long words) {
    std::lock_guard<std::mutex> lock(g_range_mtx);
    if (words > 0) g_range_words[ws] = words;
    else g_range_words.erase(ws);
}

static bf_status upload_params(double *prm, unsigned *flag, double sigma_s, double sigma_r, int N, int dtype,
                               hipStream_t stream, ParamLayout *Lout, int kind = kFitChebyshev) {
    if (flag) note_range_words(flag, 0);
    const int W = radius_of(sigma_s);
    ParamLayout L = param_layout(W, N);
    std::vector<double> host;
    fill_params(L, sigma_s, sigma_r, dtype, host, kind);
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
                              hipStream_t stream, const Centring &C = plain_centring()) {
    dim3 grid((Wd + 255) / 256, (H + kBuildRows - 1) / kBuildRows);
    ProfScope prof_("k_stack_build", stream);
    hipLaunchKernelGGL(k_stack_build<S>, grid, dim3(256), 0, stream, f, H, Wd, ld,
                       (typename S::T *)stack, ps, lds, P, prm + L.off_scale, mu, flag, C);
    return check_launch("k_stack_build");
}

static int ldt_of(int height) { return (height + 63) & ~63; }

// LDS bytes of a staged pass over 4R lines plus the 2W halo, 64 elements
// each; 0 where the unstaged kernel runs instead (above the 64 KiB of
// dynamic LDS a launch gets without an attribute: FP64 planes at large radii).
template <class S>
static size_t staged_lds_bytes(int R, int W) {
    const size_t b = (size_t)(4 * R + 2 * W) * 64 * sizeof(typename S::T);
    return b <= 65536 ? b : 0;
}

// The column pass: k_vpass_lds where its 64-element line segments stay inside
// each row (lds a multiple of 64, as the library's own stacks), else k_vpass;
// the two give identical outputs.
template <class S, int RV = kVR>
static bf_status launch_vpass(const void *stack, void *tmpT, int planes, int H, int Wd, long long ps, int lds,
                              long long pst, int ldt, const double *prm, const ParamLayout &L, hipStream_t stream) {
    dim3 gv((Wd + 63) / 64, (H + 4 * RV - 1) / (4 * RV), planes);
    ProfScope prof_("k_vpass", stream);
    const size_t sh = (lds & 63) == 0 ? staged_lds_bytes<S>(RV, L.W) : 0;
    if (sh)
        hipLaunchKernelGGL((k_vpass_lds<S, RV>), gv, dim3(256), sh, stream, (const typename S::T *)stack,
                           (typename S::T *)tmpT, H, Wd, ps, lds, pst, ldt, prm + L.off_taps, L.W);
    else
        hipLaunchKernelGGL((k_vpass<S, RV>), gv, dim3(256), 0, stream, (const typename S::T *)stack,
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
    const size_t sh = staged_lds_bytes<S>(kHR, L.W);
    if (sh)
        hipLaunchKernelGGL((k_hpass_lds<S, kHR, false>), gh, dim3(256), sh, stream, (const typename S::T *)tmpT,
                           (typename S::T *)stack, (const float *)nullptr, (float *)nullptr, (float *)nullptr,
                           (float *)nullptr, H, Wd, 0, ps, lds, pst, ldt, planes, 0, prm + L.off_taps,
                           prm + L.off_cq, prm + L.off_cp, L.W, plain_centring());
    else
        hipLaunchKernelGGL((k_hpass<S, kHR, false>), gh, dim3(256), 0, stream, (const typename S::T *)tmpT,
                           (typename S::T *)stack, (const float *)nullptr, (float *)nullptr, (float *)nullptr,
                           (float *)nullptr, H, Wd, 0, ps, lds, pst, ldt, planes, 0, prm + L.off_taps,
                           prm + L.off_cq, prm + L.off_cp, L.W, plain_centring());
    return check_launch("k_hpass");
}

template <class S, int RH = kHRC>
static bf_status launch_hpass_combine(const void *tmpT, const float *f, float *out, float *Pout, float *Qout, int H,
                                      int Wd, int ld, long long pst, int ldt, const double *prm,
                                      const ParamLayout &L, hipStream_t stream,
                                      const Centring &C = plain_centring()) {
    dim3 gh((H + 63) / 64, (Wd + 4 * RH - 1) / (4 * RH));
    ProfScope prof_("k_hpass_combine", stream);
    const size_t sh = staged_lds_bytes<S>(RH, L.W);
    if (sh)
        hipLaunchKernelGGL((k_hpass_lds<S, RH, true>), gh, dim3(256), sh, stream, (const typename S::T *)tmpT,
                           (typename S::T *)nullptr, f, out, Pout, Qout, H, Wd, ld, 0LL, 0, pst, ldt, L.N + 2, L.N,
                           prm + L.off_taps, prm + L.off_cq, prm + L.off_cp, L.W, C);
    else
        hipLaunchKernelGGL((k_hpass<S, RH, true>), gh, dim3(256), 0, stream, (const typename S::T *)tmpT,
                           (typename S::T *)nullptr, f, out, Pout, Qout, H, Wd, ld, 0LL, 0, pst, ldt, L.N + 2, L.N,
                           prm + L.off_taps, prm + L.off_cq, prm + L.off_cp, L.W, C);
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

// Constants of a fused launch: taps and b_n rounded to float, b_{N+1} = 0.
static FusedConsts fused_consts(double sigma_s, double sigma_r, int N, int kind) {
    FusedConsts C;
    std::memset(&C, 0, sizeof C);
    const std::vector<double> w = spatial_taps(sigma_s);
    for (size_t t = 0; t < w.size(); ++t) C.taps[t] = (float)w[t];
    const Fit &F = fit(sigma_r, N, kind);
    for (int n = 0; n <= N; ++n) C.b[n] = (float)F.b[n];
    return C;
}

// Blocks that fit on the device at once for a 512-thread kernel (CUs times
// its occupancy), looked up once per kernel.
static int resident_blocks(const void *kernel, int *cache) {
    if (*cache > 0) return *cache;
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 512, 0);
    *cache = std::max(1, cus) * std::max(1, per);
    return *cache;
}

// Strip length of k_fused_strip (one block per CU): the longest strip among
// those that give the fewest tile rounds, a round being one tile on every CU
// (ceil(strips / CUs) strips per CU, of at most L tiles each).
static int strip_length(int tiles_x, int tiles_y) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    cus = std::max(cus, 1);
    long long best = LLONG_MAX;
    int len = 1;
    for (int L = 1; L <= tiles_y; ++L) {
        const long long strips = (long long)tiles_x * ((tiles_y + L - 1) / L);
        const long long rounds = (strips + cus - 1) / cus * L;
        if (rounds <= best) {
            best = rounds;
            len = L;
        }
    }
    return len;
}

// Whether a single-image fused geometry runs on strips (k_fused_strip): the
// FP16 64-row tiles on 16 waves whose registers leave room for the prefetch.
template <class M, int Q, int NW, int TR>
__host__ __device__ constexpr bool fused_strips() { return M::kHalfPlanes && NW == 16 && TR == 64 && Q <= 4; }

template <class M, int Q, int TC, int QA, int NW, int TR>
static bf_status launch_fused_tiles(const float *f, float *out, int H, int Wd, int ld, const FusedConsts &C, int W,
                                    int N, float mu, char *ws, hipStream_t stream);

template <class M, int Q, int TC, int QA, int NW = 8, int TR = kFusedRows>
static bf_status launch_fused_q(const float *f, float *out, int H, int Wd, int ld, const FusedConsts &C, int W,
                                int N, float mu, char *ws, hipStream_t stream) {
    if constexpr (fused_strips<M, Q, NW, TR>()) {
        if (W >= H || W >= Wd || (long long)H * ld >= (1LL << 29))
            return launch_fused_tiles<M, Q, TC, QA, NW, TR>(f, out, H, Wd, ld, C, W, N, mu, ws, stream);
        const int tiles_x = (Wd + TC - 1) / TC, tiles_y = (H + TR - 1) / TR;
        const long long tiles = (long long)tiles_x * tiles_y;
        if (tiles > INT_MAX / 16) return fail(BF_ERR_UNSUPPORTED, "fused path: too many tiles");
        const int len = strip_length(tiles_x, tiles_y);
        const int grid = tiles_x * ((tiles_y + len - 1) / len);
        note_range_words(ws, (long long)NW * tiles);
        ProfScope prof_("k_fused_strip", stream);
        hipLaunchKernelGGL((k_fused_strip<M, Q, TC, QA>), dim3(grid), dim3(1024), 0, stream, f, out, H, Wd, ld, C, W,
                           N, mu, M::kPrescale, (unsigned *)(ws + kFlagBytes), tiles_x, tiles_y, len);
        return check_launch("k_fused_strip");
    } else {
        return launch_fused_tiles<M, Q, TC, QA, NW, TR>(f, out, H, Wd, ld, C, W, N, mu, ws, stream);
    }
}

template <class M, int Q, int TC, int QA, int NW, int TR>
static bf_status launch_fused_tiles(const float *f, float *out, int H, int Wd, int ld, const FusedConsts &C, int W,
                                    int N, float mu, char *ws, hipStream_t stream) {
    static int resident = 0;
    const void *kernel = (const void *)k_fused_mfma<M, Q, TC, QA, NW, TR>;
    const int tiles_x = (Wd + TC - 1) / TC;
    const long long tiles = (long long)tiles_x * ((H + TR - 1) / TR);
    if (tiles > INT_MAX) return fail(BF_ERR_UNSUPPORTED, "fused path: too many tiles");
    const bool persistent = fused_persistent<M>(Q) && NW == 8;
    const int grid = persistent ? (int)std::min<long long>(tiles, resident_blocks(kernel, &resident)) : (int)tiles;
    const float prescale = M::kPrescale;
    note_range_words(ws, (long long)NW * tiles);
    ProfScope prof_("k_fused_mfma", stream);
    hipLaunchKernelGGL((k_fused_mfma<M, Q, TC, QA, NW, TR>), dim3(grid), dim3(NW * 64), 0, stream, f, out, H, Wd, ld,
                       C, W, N, mu, prescale, (unsigned *)(ws + kFlagBytes), tiles_x, (int)tiles);
    return check_launch("k_fused_mfma");
}

// Tile geometry of the single-image fused forward: waves per block, tile
// rows and columns. FP16 (FP16 plane state, at most 128 VGPRs at 16 waves):
// 64 x 128 tiles up to radius 32, 64 x 64 up to 48, 32 x 128 up to 64, all
// on 16 waves, whose halo of 256 columns keeps the column pass's share of
// halo columns low; BF16 (FP32 plane state): 64 x 64 tiles up to radius 32
// and 64 x 32 up to 48 on 8 waves.
struct FusedGeom {
    int NW, TR, TC;
};
static FusedGeom fused_geom(int dtype, int W) {
    if (dtype == BF_STACK_F16) return W <= 32 ? FusedGeom{16, 64, 128} : W <= 48 ? FusedGeom{16, 64, 64}
                                                                        : FusedGeom{16, 32, 128};
    return W <= 32 ? FusedGeom{8, 64, 64} : FusedGeom{8, 64, 32};
}
static long long fused_tiles(const FusedGeom &G, int H, int Wd) {
    return (long long)((Wd + G.TC - 1) / G.TC) * ((H + G.TR - 1) / G.TR);
}

// Fused FP16/BF16 forward: one kernel (see k_fused_mfma), its constants
// passed by value. The workspace holds only the waves' range words (32 bytes
// per 64 x TC tile, far below bf_gc_workspace_bytes).
template <class M>
static bf_status run_fused(const float *f, float *out, int H, int Wd, int ld, double sigma_s, double sigma_r,
                           int N, int dtype, unsigned flags, char *ws, hipStream_t stream) {
    (void)dtype;
    const FusedConsts C = fused_consts(sigma_s, sigma_r, N, kind_of(flags));
    const float mu = (float)fit(sigma_r, N).mu;
    const int W = radius_of(sigma_s), qa = fused_qa(W);
    // geometry (fused_geom): TC + 2W halo columns within the block's 16 NW,
    // TR + 2W halo rows within 32 Q; QA = (2W + 15)/32 is QB - 1 or QB
#define BF_FUSED(Q, TC, NW, TR)                                                                                   \
    return qa == (Q) - (TR) / 32 - 1                                                                              \
               ? launch_fused_q<M, Q, TC, (Q) - (TR) / 32 - 1, NW, TR>(f, out, H, Wd, ld, C, W, N, mu, ws, stream) \
               : launch_fused_q<M, Q, TC, (Q) - (TR) / 32, NW, TR>(f, out, H, Wd, ld, C, W, N, mu, ws, stream)
    if constexpr (M::kHalfPlanes) {
        if (W <= 16) BF_FUSED(3, 128, 16, 64);
        if (W <= 32) BF_FUSED(4, 128, 16, 64);
        if (W <= 48) BF_FUSED(5, 64, 16, 64);
        if (W <= BF_FUSED_F16_MAX_RADIUS) BF_FUSED(5, 128, 16, 32);
    } else {
        if (W <= 16) BF_FUSED(3, 64, 8, 64);
        if (W <= 32) BF_FUSED(4, 64, 8, 64);
        if (W <= 48) BF_FUSED(5, 32, 8, 64);
    }
#undef BF_FUSED
    return fail(BF_ERR_UNSUPPORTED, "fused path: radius above the stack type's fused maximum");
}

// Scratch of bf_gc_forward_noalloc: the range words of one fused launch in a
// file-scope device array (each device that runs the library holds its own
// copy until the process ends). Host code uses the device address that
// hipGetSymbolAddress returns for the current device, never the array's
// name, which is a host-side stand-in.
constexpr size_t kNoAllocScratchBytes = (size_t)BF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mtx;
static std::unordered_map<int, void *> g_scratch_ptr;

static bf_status noalloc_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string("bf_gc_forward_noalloc: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return BF_OK;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(BF_ERR_DEVICE, std::string("bf_gc_forward_noalloc: scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return BF_OK;
}

template <class S, int RV, int RH>
static bf_status run_forward(const float *f, float *out, int H, int Wd, int ld, double sigma_s, double sigma_r,
                             int N, int dtype, unsigned flags, char *ws, hipStream_t stream) {
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, dtype, stream, &L, kind_of(flags));
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
    if ((st = launch_vpass<S, RV>(stackA, stackB, P, H, Wd, ps, lds, pst, ldt, prm, L, stream)) != BF_OK) return st;
    return launch_hpass_combine<S, RH>(stackB, f, out, nullptr, nullptr, H, Wd, ld, pst, ldt, prm, L, stream);
}

// Joint filter: build both plane sets, column pass over all 2(N+1) planes,
// row pass + combine of A_n and B_n together.
template <class S, int RV, int RH>
static bf_status run_joint_forward(const float *g, const float *f, float *out, int H, int Wd, int ld,
                                   double sigma_s, double sigma_r, int N, int dtype, unsigned flags, char *ws,
                                   hipStream_t stream) {
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, dtype, stream, &L, kind_of(flags));
    if (st != BF_OK) return st;
    const int lds = lds_of(Wd);
    const long long ps = (long long)H * lds;
    const int planes = 2 * (N + 1);
    char *stackA = ws + kFlagBytes + align256(sizeof(double) * L.total);
    char *stackB = stackA + align256((size_t)planes * ps * sizeof(typename S::T));
    const double mu = fit(sigma_r, N).mu;
    {
        dim3 grid((Wd + 255) / 256, (H + kBuildRows - 1) / kBuildRows);
        ProfScope prof_("k_joint_build", stream);
        hipLaunchKernelGGL((k_joint_build<S>), grid, dim3(256), 0, stream, g, f, H, Wd, ld,
                           (typename S::T *)stackA, ps, lds, N, prm + L.off_scale, mu, flag);
        if ((st = check_launch("k_joint_build")) != BF_OK) return st;
    }
    const int ldt = ldt_of(H);
    const long long pst = (long long)Wd * ldt;
    if ((st = launch_vpass<S, RV>(stackA, stackB, planes, H, Wd, ps, lds, pst, ldt, prm, L, stream)) != BF_OK)
        return st;
    dim3 gh((H + 63) / 64, (Wd + 4 * RH - 1) / (4 * RH));
    ProfScope prof_("k_hpass_joint", stream);
    hipLaunchKernelGGL((k_hpass_joint<S, RH>), gh, dim3(256), 0, stream, (const typename S::T *)stackB, g, out, H,
                       Wd, ld, pst, ldt, N, prm + L.off_taps, prm + L.off_cq, L.W);
    return check_launch("k_hpass_joint");
}

// Uploads a filled parameter vector (k_put_params chunks); clears the device
// flag only when asked.
static bf_status upload_vector(double *prm, unsigned *flag, const std::vector<double> &host, bool clear_flag,
                               hipStream_t stream) {
    if (flag && clear_flag) note_range_words(flag, 0);
    ParamChunk ch;
    int off = 0;
    const int total = (int)host.size();
    do {
        std::memset(&ch, 0, sizeof ch);
        ch.offset = off;
        ch.count = std::min(400, total - off);
        ch.clear_flag = (off == 0 && clear_flag) ? 1 : 0;
        for (int i = 0; i < ch.count; ++i) ch.v[i] = host[off + i];
        ProfScope prof_("k_put_params", stream);
        hipLaunchKernelGGL(k_put_params, dim3(1), dim3(256), 0, stream, prm, flag, ch);
        off += 400;
    } while (off < total);
    return check_launch("k_put_params");
}

static int pivot_nmax(const std::vector<Pivot> &plan) {
    int n = 0;
    for (const Pivot &p : plan) n = std::max(n, p.N);
    return n;
}

// Whether K sub-ranges at the rule's degree each have kappa times the stack
// type's rounding unit at most `limit` (1e-2: the conditioning check).
static bool pivots_conditioned(double sigma_r, int K, int dtype, double limit = 1e-2) {
    for (const Pivot &p : pivot_plan(sigma_r, K, 0, BF_MAX_DEGREE)) {
        if (p.N < 1) return false;
        const double kappa = fit_mu(p.mu, p.N).kappa;
        if (!std::isfinite(kappa) || kappa * unit_roundoff(dtype) > limit) return false;
    }
    return true;
}

// Accuracy domain of a stack type in a batch, as a limit on kappa times its
// rounding unit. The storage rounding reaches the output as about
// kappa u t_h (measured 0.1-1.3 kappa u t_h over the uneven batch), so FP32
// holds a 1e-3 max-abs error where kappa u <= 1e-5 (sigma_r >= 25 at the
// rule's degree); the 16-bit stacks, whose own rounding is far above that,
// keep the conditioning check's 1e-2.
static double batch_limit(int dtype) { return dtype == BF_STACK_F32 ? 1e-5 : 1e-2; }

// Route of one image of a batch whose host checks passed except, possibly,
// the conditioning check: 1 = its own expansion (degree N); K >= 2 = the
// pivoted form with K sub-ranges at the rule's degree each, for an image
// whose own expansion lies outside the stack type's accuracy domain
// (Chebyshev coefficients, no BF_FLAG_ALLOW_ILL_CONDITIONED), K the smallest
// power of two whose sub-ranges lie inside; 0 = neither (the image keeps its
// conditioning status, BF_ERR_ILL_CONDITIONED if its own expansion fails the
// check, else it runs its own expansion). *st: the image's status.
static int batch_route_uncached(double sigma_r, int N, int dtype, unsigned flags, bf_status *st) {
    *st = check_conditioning(sigma_r, N, dtype, flags);
    if ((*st != BF_OK && *st != BF_ERR_ILL_CONDITIONED) || (flags & BF_FLAG_ALLOW_ILL_CONDITIONED) ||
        (flags & (BF_FLAG_TAYLOR | BF_FLAG_MINIMAX)))
        return *st == BF_OK ? 1 : 0;
    const double limit = batch_limit(dtype);
    if (*st == BF_OK && fit(sigma_r, N).kappa * unit_roundoff(dtype) <= limit) return 1;
    for (int K = 2; K <= BF_MAX_PIVOTS; K *= 2)
        if (pivots_conditioned(sigma_r, K, dtype, limit)) {
            *st = BF_OK;
            return K;
        }
    return *st == BF_OK ? 1 : 0;
}

// batch_route with its results cached per (sigma_r, N, stack type, the flags
// that matter): a batch asks for the same images on every call.
static int batch_route(double sigma_r, int N, int dtype, unsigned flags, bf_status *st) {
    static std::mutex mtx;
    static std::map<std::tuple<double, int, int, unsigned>, std::pair<int, bf_status>> cache;
    const unsigned f = flags & (BF_FLAG_ALLOW_ILL_CONDITIONED | BF_FLAG_TAYLOR | BF_FLAG_MINIMAX);
    const auto key = std::make_tuple(sigma_r, N, dtype, f);
    {
        std::lock_guard<std::mutex> lock(mtx);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *st = it->second.second;
            if (*st != BF_OK) fail(*st, "ill-conditioned or unsupported coefficients for this image");
            return it->second.first;
        }
    }
    const int K = batch_route_uncached(sigma_r, N, dtype, flags, st);
    std::lock_guard<std::mutex> lock(mtx);
    cache.emplace(key, std::make_pair(K, *st));
    return K;
}

// Fused pivoted form: the range words of the tiles, then the sub-range table
// (K FusedPivot entries, the taps, the coefficients of every sub-range), the
// tiles' sub-range masks, their order and the queue counter.
static long long fused_pivot_tiles(int H, int Wd, int W) {
    const int TC = W <= 32 ? 64 : 32;
    return (long long)((Wd + TC - 1) / TC) * ((H + kFusedRows - 1) / kFusedRows);
}
static size_t fused_pivot_table_bytes(int K, int W, int Nmax) {
    return sizeof(FusedPivot) * K + sizeof(float) * (size_t)(((2 * W + 1) + 3) & ~3) +
           sizeof(float) * (size_t)K * (Nmax + 2);
}

static size_t pivots_ws_bytes(int H, int Wd, int W, int K, int Nmax, int dtype) {
    const size_t P = (size_t)Nmax + 2;
    const size_t staged = kFlagBytes + align256(sizeof(double) * (size_t)param_layout(W, Nmax).total) +
                          align256(P * H * lds_of(Wd) * esize(dtype)) + align256(P * Wd * ldt_of(H) * esize(dtype));
    const size_t tiles = (size_t)fused_pivot_tiles(H, Wd, W);
    const size_t fused = kFlagBytes + align256(sizeof(unsigned) * kFusedSlots * tiles) +
                         align256(fused_pivot_table_bytes(K, W, Nmax)) + align256(sizeof(unsigned long long) * tiles) +
                         align256(sizeof(int) * tiles) + 256;
    return std::max(staged, fused);
}

// Pivoted forward: per sub-range, the three-kernel forward centred at its
// midpoint, writing only the outputs whose centre value lies in it.
template <class S, int RV, int RH>
static bf_status run_pivots(const float *f, float *out, int H, int Wd, int ld, double sigma_s,
                            const std::vector<Pivot> &plan, int dtype, char *ws, hipStream_t stream) {
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    const int W = radius_of(sigma_s);
    const int Nmax = pivot_nmax(plan);
    const int lds = lds_of(Wd);
    const long long ps = (long long)H * lds;
    const int ldt = ldt_of(H);
    const long long pst = (long long)Wd * ldt;
    char *stackA = ws + kFlagBytes + align256(sizeof(double) * (size_t)param_layout(W, Nmax).total);
    char *stackB = stackA + align256((size_t)(Nmax + 2) * ps * sizeof(typename S::T));
    const int K = (int)plan.size();
    for (int k = 0; k < K; ++k) {
        const Pivot &p = plan[k];
        const ParamLayout L = param_layout(W, p.N);
        std::vector<double> host;
        fill_params_pivot(L, sigma_s, p.mu, p.nu, dtype, host);
        bf_status st = upload_vector(prm, flag, host, k == 0, stream);
        if (st != BF_OK) return st;
        const int mask = K == 1 ? 0 : k == 0 ? 2 : k == K - 1 ? 3 : 1;
        const Centring C{p.t, 1.0 / p.R, 1.0 / p.h, p.R, (float)p.lo, (float)p.hi, mask};
        if ((st = launch_build<S>(f, H, Wd, ld, stackA, ps, lds, p.N + 2, prm, L, p.nu, flag, stream, C)) != BF_OK)
            return st;
        if ((st = launch_vpass<S, RV>(stackA, stackB, p.N + 2, H, Wd, ps, lds, pst, ldt, prm, L, stream)) != BF_OK)
            return st;
        if ((st = launch_hpass_combine<S, RH>(stackB, f, out, nullptr, nullptr, H, Wd, ld, pst, ldt, prm, L, stream,
                                              C)) != BF_OK)
            return st;
    }
    return BF_OK;
}

// Pivoted form on the fused tile. Per sub-range the planes are built from
// c s_j with one geometric scale c = g(N+1)^{-1/(N+1)}, g(n) = max over |s| <= 1
// of e^{-nu s^2/2} |s|^n (= (n/(e nu))^{n/2} for n <= nu, else e^{-nu/2}): since
// log g is convex in n, every plane's peak c^n g(n) then lies in (0, 1], the
// top and bottom planes at 1, and the 16-bit planes stay normal without a
// scale per plane. c^{-n} goes into the coefficients (b_n c^{-n}, so the
// combine's Ps comes out c times too large) and 1/c into the output scale.
template <class M, int Q, int TC, int QA>
static bf_status launch_fused_pivots_q(const float *f, float *out, int H, int Wd, int ld, char *table,
                                       size_t table_bytes, int K, int W, char *ws, hipStream_t stream) {
    static int resident = 0;
    const void *kernel = (const void *)k_fused_pivots<M, Q, TC, QA>;
    const int tiles_x = (Wd + TC - 1) / TC;
    const long long tiles = (long long)tiles_x * ((H + kFusedRows - 1) / kFusedRows);
    if (tiles > INT_MAX) return fail(BF_ERR_UNSUPPORTED, "fused path: too many tiles");
    const FusedPivot *piv = (const FusedPivot *)table;
    const float *taps = (const float *)(table + sizeof(FusedPivot) * K);
    const float *coef = taps + (((2 * W + 1) + 3) & ~3);
    unsigned long long *masks = (unsigned long long *)(table + align256(table_bytes));
    int *order = (int *)((char *)masks + align256(sizeof(unsigned long long) * tiles));
    int *counter = (int *)((char *)order + align256(sizeof(int) * tiles));
    const float kscale = (float)(K / (kTc + kTh));
    note_range_words(ws, kFusedSlots * tiles);
    {
        ProfScope prof_("k_pivot_masks", stream);
        hipLaunchKernelGGL((k_pivot_masks<TC>), dim3((unsigned)tiles), dim3(256), 0, stream, f, H, Wd, ld, piv, K,
                           kscale, tiles_x, masks);
    }
    bf_status st = check_launch("k_pivot_masks");
    if (st != BF_OK) return st;
    {
        ProfScope prof_("k_pivot_order", stream);
        hipLaunchKernelGGL(k_pivot_order, dim3(1), dim3(1024), 0, stream, masks, (int)tiles, order, counter);
    }
    if ((st = check_launch("k_pivot_order")) != BF_OK) return st;
    const int grid = (int)std::min<long long>(tiles, resident_blocks(kernel, &resident));
    ProfScope prof_("k_fused_pivots", stream);
    hipLaunchKernelGGL((k_fused_pivots<M, Q, TC, QA>), dim3(grid), dim3(512), 0, stream, f, out, H, Wd, ld, piv, coef,
                       taps, K, kscale, W, (unsigned *)(ws + kFlagBytes), tiles_x, (int)tiles, masks, order, counter);
    return check_launch("k_fused_pivots");
}

// Host image of the fused pivoted form's sub-range table: K FusedPivot
// entries, the taps as floats (padded to a multiple of 4), then each
// sub-range's coefficients b_n c^{-n}, n = 0..N_k+1 (b_{N_k+1} = 0), as
// floats. prescale: the stack type's common plane scale 2^K.
static std::vector<char> fused_pivot_table(double sigma_s, const std::vector<Pivot> &plan, float prescale) {
    const int W = radius_of(sigma_s);
    const int K = (int)plan.size();
    std::vector<FusedPivot> piv(K);
    const std::vector<double> w = spatial_taps(sigma_s);
    const int ntap = ((2 * W + 1) + 3) & ~3;
    std::vector<float> coef;
    const double k2 = std::log2((double)prescale);
    for (int k = 0; k < K; ++k) {
        const Pivot &p = plan[k];
        const int n1 = p.N + 1;
        const double lg = n1 <= p.nu ? 0.5 * n1 * std::log(n1 / (std::exp(1.0) * p.nu)) : -0.5 * p.nu;
        const double c = std::exp(-lg / n1);
        FusedCentre &C = piv[k].c;
        C.sb = (float)(c / p.R);
        C.ob = (float)(-c * p.t / p.R);
        C.e2 = (float)(-0.5 * p.nu / (c * c) / std::log(2.0));
        C.k2 = (float)k2;
        C.sc = (float)(1.0 / p.h);
        C.oc = (float)(-p.t / p.h);
        C.ys = (float)(p.R / c);
        C.yo = (float)p.t;
        piv[k].lo = (float)p.lo;
        piv[k].N = p.N;
        piv[k].boff = (int)coef.size();
        piv[k].pad = 0;
        const Fit &F = fit_mu(p.mu, p.N);
        for (int n = 0; n <= p.N; ++n) coef.push_back((float)(F.b[n] * std::pow(c, -n)));
        coef.push_back(0.0f);
    }
    std::vector<char> bytes(sizeof(FusedPivot) * K + sizeof(float) * (ntap + coef.size()), 0);
    std::memcpy(bytes.data(), piv.data(), sizeof(FusedPivot) * K);
    float *tp = (float *)(bytes.data() + sizeof(FusedPivot) * K);
    for (int t = 0; t <= 2 * W; ++t) tp[t] = (float)w[t];
    std::memcpy(tp + ntap, coef.data(), sizeof(float) * coef.size());
    return bytes;
}

template <class M>
static bf_status run_fused_pivots(const float *f, float *out, int H, int Wd, int ld, double sigma_s,
                                  const std::vector<Pivot> &plan, char *ws, hipStream_t stream) {
    const int W = radius_of(sigma_s), qa = fused_qa(W);
    const int K = (int)plan.size();
    const long long tiles = fused_pivot_tiles(H, Wd, W);
    char *table = ws + kFlagBytes + align256(sizeof(unsigned) * kFusedSlots * (size_t)tiles);
    const std::vector<char> bytes = fused_pivot_table(sigma_s, plan, M::kPrescale);
    std::vector<double> host((bytes.size() + 7) / 8, 0.0);
    std::memcpy(host.data(), bytes.data(), bytes.size());
    bf_status st = upload_vector((double *)table, nullptr, host, false, stream);
    if (st != BF_OK) return st;
    const size_t tb = bytes.size();
#define BF_FPIV(Q, TC)                                                                                           \
    return qa == (Q) - 3 ? launch_fused_pivots_q<M, Q, TC, (Q) - 3>(f, out, H, Wd, ld, table, tb, K, W, ws, stream) \
                         : launch_fused_pivots_q<M, Q, TC, (Q) - 2>(f, out, H, Wd, ld, table, tb, K, W, ws, stream)
    if (W <= 16) BF_FPIV(3, 64);
    if (W <= 32) BF_FPIV(4, 64);
    if (W <= 48) BF_FPIV(5, 32);
#undef BF_FPIV
    return fail(BF_ERR_UNSUPPORTED, "fused path: radius above BF_FUSED_MAX_RADIUS");
}

// Recursive variant: build, recursive Gaussian along columns (stack A -> B)
// and rows (B -> A), then the combine of the staged path.
template <class S>
static bf_status run_recursive(const float *f, float *out, int H, int Wd, int ld, double sigma_s, double sigma_r,
                               int N, int dtype, unsigned flags, char *ws, hipStream_t stream) {
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, dtype, stream, &L, kind_of(flags));
    if (st != BF_OK) return st;
    const int lds = lds_of(Wd);
    const long long ps = (long long)H * lds;
    const int P = N + 2;
    char *stackA = ws + kFlagBytes + align256(sizeof(double) * L.total);
    char *stackB = stackA + align256((size_t)P * ps * sizeof(typename S::T));
    const double mu = fit(sigma_r, N).mu;
    if ((st = launch_build<S>(f, H, Wd, ld, stackA, ps, lds, P, prm, L, mu, flag, stream)) != BF_OK) return st;
    const Recursive R = recursive_coefficients(sigma_s);
    const IirCoef c{R.num[0], R.num[1], R.num[2], R.num[3], R.anum[0], R.anum[1], R.anum[2], R.anum[3],
                    R.den[0], R.den[1], R.den[2], R.den[3], R.k, R.P};
    {
        ProfScope prof_("k_iir_col", stream);
        hipLaunchKernelGGL((k_iir_col<S>), dim3((Wd + 255) / 256, P), dim3(256), 0, stream,
                           (const typename S::T *)stackA, (typename S::T *)stackB, H, Wd, ps, lds, c);
        if ((st = check_launch("k_iir_col")) != BF_OK) return st;
    }
    {
        ProfScope prof_("k_iir_row", stream);
        hipLaunchKernelGGL((k_iir_row<S>), dim3((H + 63) / 64, P), dim3(64), 0, stream,
                           (const typename S::T *)stackB, (typename S::T *)stackA, H, Wd, ps, lds, c);
        if ((st = check_launch("k_iir_row")) != BF_OK) return st;
    }
    return launch_combine<S>(f, stackA, H, Wd, ld, ps, lds, prm, L, out, nullptr, nullptr, stream);
}

// Joint filter on the fused kernel (FP16/BF16, radius <= 32).
template <class M>
static bf_status run_joint_fused(const float *g, const float *v, float *out, int H, int Wd, int ld, double sigma_s,
                                 double sigma_r, int N, int dtype, unsigned flags, char *ws, hipStream_t stream) {
    (void)dtype;
    const FusedConsts C = fused_consts(sigma_s, sigma_r, N, kind_of(flags));
    const float mu = (float)fit(sigma_r, N).mu;
    const int W = radius_of(sigma_s), qa = fused_qa(W);
    const int TC = W <= 32 ? 64 : 32;
    dim3 grid((Wd + TC - 1) / TC, (H + kFusedRows - 1) / kFusedRows);
    unsigned *slots = (unsigned *)(ws + kFlagBytes);
    if (W > kJointFusedMaxRadius) return fail(BF_ERR_UNSUPPORTED, "fused joint filter: radius above BF_FUSED_MAX_RADIUS");
    note_range_words(ws, (long long)kFusedSlots * grid.x * grid.y);
    ProfScope prof_("k_fused_joint", stream);
#define BF_JF(Q, TCC, QA) \
    hipLaunchKernelGGL((k_fused_joint<M, Q, TCC, QA>), grid, dim3(512), 0, stream, g, v, out, H, Wd, ld, C, W, N, mu, slots)
    if (W <= 16) {
        if (qa == 0) BF_JF(3, 64, 0);
        else BF_JF(3, 64, 1);
    } else if (W <= 32) {
        if (qa == 1) BF_JF(4, 64, 1);
        else BF_JF(4, 64, 2);
    } else {
        if (qa == 2) BF_JF(5, 32, 2);
        else BF_JF(5, 32, 3);
    }
#undef BF_JF
    return check_launch("k_fused_joint");
}

constexpr int kAdjR = 4;            // columns per lane in k_hpass_adj
constexpr int kNeighborBlocks = 2048;
constexpr size_t kBatchItemsMaxTable = 256;   // descriptors up to which the three-kernel batch runs one block per item

struct BwdLayout {
    size_t params, stackA, stackB, perpx, partial, total;
};

// Radii up to kAdjMaxRadius run the two fused tile kernels (no plane stacks;
// one partial sum per 64 x 32 tile); larger radii the staged passes over two
// FP64 stacks.
static bool bwd_fused(double sigma_s) { return radius_of(sigma_s) <= kAdjMaxRadius; }
static long long bwd_tiles(int H, int Wd) {
    return (long long)((Wd + kAdjCols - 1) / kAdjCols) * ((H + kAdjRows - 1) / kAdjRows);
}

// Fused form: the six saved sums per pixel (k_adj_forward_tile) take the
// place of the four per-pixel arrays.
static BwdLayout bwd_layout(int H, int Wd, double sigma_s, int N) {
    BwdLayout B;
    const size_t P = (size_t)N + 2;
    const bool fused = bwd_fused(sigma_s);
    B.params = align256(sizeof(double) * (size_t)param_layout(radius_of(sigma_s), N).total);
    B.stackA = fused ? 0 : align256(P * H * lds_of(Wd) * sizeof(double));
    B.stackB = fused ? 0 : align256(P * Wd * ldt_of(H) * sizeof(double));
    B.perpx = align256((size_t)H * Wd * sizeof(double));
    B.partial = align256((size_t)(fused ? bwd_tiles(H, Wd) : kNeighborBlocks) * sizeof(double));
    B.total = kFlagBytes + B.params + B.stackA + B.stackB + (fused ? 6 : 4) * B.perpx + B.partial;
    return B;
}

// The fused FP64 tile kernels over `count` images of one shape (image z at
// image_stride floats from image z - 1; saved sums 6 H Wd doubles apart).
static bf_status launch_adj_forward(const float *f, float *out, double *saved, int count, long long stride, int H,
                                    int Wd, int ld, int N, double mu, const double *prm, const ParamLayout &L,
                                    unsigned *flag, hipStream_t stream) {
    const dim3 g((Wd + kAdjCols - 1) / kAdjCols, (H + kAdjRows - 1) / kAdjRows, count);
    const double *taps = prm + L.off_taps + (kTapPad - 1);
    ProfScope prof_("k_adj_forward_tile", stream);
#define BF_ADJ_F(WW)                                                                                              \
    case WW:                                                                                                      \
        hipLaunchKernelGGL(k_adj_forward_tile<WW>, g, dim3(kAdjThreads), 0, stream, f, out, saved, H, Wd, ld,      \
                           stride, N, mu, taps, prm + L.off_cq, prm + L.off_cp, prm + L.off_bd, flag);              \
        break;
    switch (L.W) {
        BF_ADJ_F(1) BF_ADJ_F(2) BF_ADJ_F(3) BF_ADJ_F(4) BF_ADJ_F(5) BF_ADJ_F(6) BF_ADJ_F(7) BF_ADJ_F(8)
        BF_ADJ_F(9) BF_ADJ_F(10) BF_ADJ_F(11) BF_ADJ_F(12) BF_ADJ_F(13) BF_ADJ_F(14) BF_ADJ_F(15) BF_ADJ_F(16)
        default: return fail(BF_ERR_UNSUPPORTED, "fused FP64 tiles: radius above BF_ADJ_MAX_RADIUS");
    }
#undef BF_ADJ_F
    return check_launch("k_adj_forward_tile");
}

// The adjoint tiles and the fixed-order sum of their partials:
// grad_sr = sum over the count images of dL/dsigma_r.
static bf_status launch_adj_backward(const float *f, const float *ybar, const double *saved, float *grad_f,
                                     double *grad_sr, double *partial, int count, long long stride, int H, int Wd,
                                     int ld, int N, double mu, double sigma_r, const double *prm,
                                     const ParamLayout &L, hipStream_t stream) {
    const dim3 g((Wd + kAdjCols - 1) / kAdjCols, (H + kAdjRows - 1) / kAdjRows, count);
    const double *taps = prm + L.off_taps + (kTapPad - 1);
    {
        ProfScope prof_("k_adj_backward_tile", stream);
#define BF_ADJ_B(WW)                                                                                              \
    case WW:                                                                                                      \
        hipLaunchKernelGGL(k_adj_backward_tile<WW>, g, dim3(kAdjThreads), 0, stream, f, ybar, saved, grad_f,       \
                           partial, H, Wd, ld, stride, N, mu, taps, prm + L.off_cq, prm + L.off_cp);                \
        break;
        switch (L.W) {
            BF_ADJ_B(1) BF_ADJ_B(2) BF_ADJ_B(3) BF_ADJ_B(4) BF_ADJ_B(5) BF_ADJ_B(6) BF_ADJ_B(7) BF_ADJ_B(8)
            BF_ADJ_B(9) BF_ADJ_B(10) BF_ADJ_B(11) BF_ADJ_B(12) BF_ADJ_B(13) BF_ADJ_B(14) BF_ADJ_B(15) BF_ADJ_B(16)
            default: return fail(BF_ERR_UNSUPPORTED, "fused FP64 tiles: radius above BF_ADJ_MAX_RADIUS");
        }
#undef BF_ADJ_B
        bf_status st = check_launch("k_adj_backward_tile");
        if (st != BF_OK) return st;
    }
    ProfScope prof_("k_reduce_f64", stream);
    hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, stream, (const double *)partial,
                       (long long)count * bwd_tiles(H, Wd), -2.0 * mu / sigma_r, grad_sr);
    return check_launch("k_reduce_f64");
}

static bf_status run_backward(const float *f, const float *ybar, float *grad_f, double *grad_sr, int H, int Wd,
                              int ld, double sigma_s, double sigma_r, int N, unsigned flags, char *ws,
                              hipStream_t stream) {
    const BwdLayout B = bwd_layout(H, Wd, sigma_s, N);
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)(ws + kFlagBytes);
    ParamLayout L;
    bf_status st = upload_params(prm, flag, sigma_s, sigma_r, N, BF_STACK_F32, stream, &L, kind_of(flags));
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
    if (bwd_fused(sigma_s)) {
        // The forward recomputed in FP64 (the derivative sums cancel strongly;
        // FP32 planes cost them three to four digits) into the six saved sums,
        // then the adjoint planes, both per tile.
        double *saved = alpha;
        double *psum = (double *)((char *)saved + 6 * B.perpx);
        if ((st = launch_adj_forward(f, nullptr, saved, 1, 0, H, Wd, ld, N, mu, prm, L, nullptr, stream)) != BF_OK)
            return st;
        return launch_adj_backward(f, ybar, saved, grad_f, grad_sr, psum, 1, 0, H, Wd, ld, N, mu, sigma_r, prm, L,
                                   stream);
    }
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
        hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, stream, (const double *)partial, (long long)nb,
                           -2.0 * mu / sigma_r, grad_sr);
        return check_launch("k_reduce_f64");
    }
}

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

// ---------------------------------------------------------------------------
// Batched host side
// ---------------------------------------------------------------------------

struct BatchPlan {
    std::vector<int> status;
    std::vector<BatchImage> img;        // device descriptors (pointers filled in)
    std::vector<long long> start;       // [kBatchPhases][n] item starts in each phase's visiting order
    std::vector<int> order;             // [kBatchPhases][n] images in each phase's visiting order
    std::vector<std::vector<double>> prm;
    size_t blob_bytes = 0, blob_cap = 0, total = 0;
    long long items = 0, phase_items[kBatchPhases] = {};
};

static size_t batch_blob_cap(size_t bytes) {
    size_t cap = 64 * 1024;
    while (cap < bytes) cap *= 2;
    return cap;
}

static size_t batch_head_bytes(size_t n) {
    return align256(sizeof(BatchHeader) + sizeof(BatchImage) * n + (sizeof(long long) + sizeof(int)) * kBatchPhases * n);
}

// Plans a batch: per-image status, descriptors, parameter blocks and the
// workspace layout [blob (capacity blob_cap) | per image: stack A, stack B]
// (three-kernel form) or [blob] (fused form, phases = geometry classes).
// An image whose single expansion fails the conditioning check is routed to
// the pivoted form (batch_route): on the fused tile one descriptor in the
// pivoted class of its geometry, carrying the sub-range table; in the
// three-kernel form one descriptor per sub-range (its centring, degree and
// coefficients, stacks of its own), each writing only its own pixels. When
// sizing, pointers are not read.
static void plan_batch(const bf_image_desc *d, int count, int dtype, unsigned flags, int RV, int RH, bool fused,
                       char *ws, BatchPlan &B, bool sizing = false) {
    B.status.assign(count, BF_OK);
    B.img.clear();
    B.prm.clear();
    std::vector<int> ok, route;
    for (int i = 0; i < count; ++i) {
        const bf_image_desc &x = d[i];
        bf_status st = check_common(x.height, x.width, x.sigma_s, x.sigma_r, x.N, dtype);
        if (st == BF_OK && fused && radius_of(x.sigma_s) > BF_FUSED_MAX_RADIUS)
            st = fail(BF_ERR_UNSUPPORTED, "fused tile: radius above BF_FUSED_MAX_RADIUS");
        int K = 1;
        if (st == BF_OK && x.height > 0 && x.width > 0) {
            if (!sizing) {
                const size_t img = ((size_t)(x.height - 1) * x.ld + x.width) * sizeof(float);
                if (!x.f || !x.out) st = fail(BF_ERR_INVALID_ARG, "f and out must be non-null");
                else if (x.ld < x.width) st = fail(BF_ERR_INVALID_ARG, "ld must be >= width");
                else if (overlaps(x.f, img, x.out, img)) st = fail(BF_ERR_INVALID_ARG, "out overlaps f");
            }
            if (st == BF_OK) K = batch_route(x.sigma_r, x.N, dtype, flags, &st);
        }
        B.status[i] = st;
        if (st == BF_OK && x.height > 0 && x.width > 0) {
            ok.push_back(i);
            route.push_back(K);
        }
    }
    // descriptors: (image, pivot plan) pairs; an empty plan is the plain expansion
    struct Entry {
        int i;
        std::vector<Pivot> plan;   // fused: all sub-ranges; three-kernel: the one sub-range
        int k;                     // three-kernel: its index, for the output mask
    };
    std::vector<Entry> ent;
    for (size_t j = 0; j < ok.size(); ++j) {
        const bf_image_desc &x = d[ok[j]];
        if (route[j] == 1) {
            ent.push_back({ok[j], {}, 0});
            continue;
        }
        const std::vector<Pivot> plan = pivot_plan(x.sigma_r, route[j], 0, BF_MAX_DEGREE);
        if (fused) ent.push_back({ok[j], plan, 0});
        else
            for (int k = 0; k < route[j]; ++k) ent.push_back({ok[j], {plan[k]}, k});
    }
    const int n = (int)ent.size();
    const float prescale = dtype == BF_STACK_F16 ? MmaF16::kPrescale : MmaBF16::kPrescale;
    // parameter blocks
    for (int e = 0; e < n; ++e) {
        const bf_image_desc &x = d[ent[e].i];
        const int W = radius_of(x.sigma_s);
        std::vector<double> pv;
        if (ent[e].plan.empty()) {
            fill_params(param_layout(W, x.N), x.sigma_s, x.sigma_r, dtype, pv, kind_of(flags));
        } else if (fused) {
            const std::vector<char> bytes = fused_pivot_table(x.sigma_s, ent[e].plan, prescale);
            pv.assign((bytes.size() + 7) / 8, 0.0);
            std::memcpy(pv.data(), bytes.data(), bytes.size());
        } else {
            const Pivot &p = ent[e].plan[0];
            fill_params_pivot(param_layout(W, p.N), x.sigma_s, p.mu, p.nu, dtype, pv);
        }
        B.prm.push_back(pv);
    }
    size_t prm_bytes = 0;
    for (const std::vector<double> &pv : B.prm) prm_bytes += align256(sizeof(double) * pv.size());
    const size_t head_bytes = batch_head_bytes(n);
    B.blob_bytes = head_bytes + prm_bytes;
    B.blob_cap = batch_blob_cap(B.blob_bytes);
    size_t off = B.blob_cap;
    size_t poff = head_bytes;
    std::vector<long long> cnt[kBatchPhases], cost[kBatchPhases];
    for (int e = 0; e < n; ++e) {
        const Entry &E = ent[e];
        const bf_image_desc &x = d[E.i];
        const bool piv = !E.plan.empty();
        const int Ne = piv && !fused ? E.plan[0].N : x.N;
        const ParamLayout L = param_layout(radius_of(x.sigma_s), Ne);
        BatchImage I;
        std::memset(&I, 0, sizeof I);
        I.f = x.f;
        I.out = x.out;
        I.H = x.height;
        I.Wd = x.width;
        I.ld = x.ld;
        I.lds = lds_of(x.width);
        I.ldt = ldt_of(x.height);
        I.W = L.W;
        I.N = Ne;
        I.P = Ne + 2;
        I.ps = (long long)I.H * I.lds;
        I.pst = (long long)I.Wd * I.ldt;
        I.mu = piv ? (fused ? 0.0 : E.plan[0].nu) : fit(x.sigma_r, x.N).mu;
        I.off_taps = L.off_taps;
        I.off_cq = L.off_cq;
        I.off_cp = L.off_cp;
        I.off_scale = L.off_scale;
        I.off_bf = L.off_bf;
        I.off_tf = L.off_tf;
        I.C = plain_centring();
        I.K = 1;
        I.prm = (const double *)((uintptr_t)ws + poff);   // ws may be null when only sizing
        poff += align256(sizeof(double) * B.prm[e].size());
        for (int p = 0; p < kBatchPhases; ++p) {
            cnt[p].push_back(0);
            cost[p].push_back(0);
        }
        if (fused) {
            // tile columns of the class kernel (batched_fused_kernel,
            // k_fused_batched_pivot_items): wider FP16 tiles on 16 waves
            const int TC = dtype == BF_STACK_F16 && !piv ? (L.W <= 32 ? 128 : 64) : (L.W <= 32 ? 64 : 32);
            int c = fused_class_of_radius(L.W);
            I.gvx = (I.Wd + TC - 1) / TC;
            if (!piv) {
                cost[c].back() = I.P;                             // per tile: planes
            } else {
                const int K = (int)E.plan.size();
                c += kFusedClasses;
                I.K = K;
                I.kscale = (float)(K / (kTc + kTh));
                I.off_piv = 0;
                I.off_tf = (int)(sizeof(FusedPivot) * K / sizeof(double));
                I.off_bf = I.off_tf + (((2 * L.W + 1) + 3) & ~3) / 2;
                long long planes = 0;
                for (const Pivot &p : E.plan) planes += p.N + 2;
                cost[c].back() = planes;                          // per tile: at most every sub-range's planes
            }
            cnt[c].back() = (long long)I.gvx * ((I.H + kFusedRows - 1) / kFusedRows);
        } else {
            if (piv) {
                const Pivot &p = E.plan[0];
                const int K = route[std::find(ok.begin(), ok.end(), E.i) - ok.begin()];
                const int mask = E.k == 0 ? 2 : E.k == K - 1 ? 3 : 1;
                I.C = Centring{p.t, 1.0 / p.R, 1.0 / p.h, p.R, (float)p.lo, (float)p.hi, mask};
            }
            I.stackA = (void *)((uintptr_t)ws + off);
            off += align256((size_t)I.P * I.ps * esize(dtype));
            I.stackB = (void *)((uintptr_t)ws + off);
            off += align256((size_t)I.P * I.pst * esize(dtype));
            I.gbx = (I.Wd + 255) / 256;
            I.gvx = (I.Wd + 63) / 64;
            I.gvy = (I.H + 4 * RV - 1) / (4 * RV);
            I.ghx = (I.H + 63) / 64;
            const int ghy = (I.Wd + 4 * RH - 1) / (4 * RH);
            cnt[0].back() = (long long)I.gbx * ((I.H + kBuildRows - 1) / kBuildRows);
            cnt[1].back() = (long long)I.gvx * I.gvy * I.P;
            cnt[2].back() = (long long)I.ghx * ghy;
            cost[0].back() = I.P;                                   // per item: planes written
            cost[1].back() = 2LL * L.W + 1;                         // taps per output
            cost[2].back() = (long long)I.P * (2LL * L.W + 1);      // planes x taps per output
        }
        B.img.push_back(I);
    }
    B.start.assign((size_t)kBatchPhases * n, 0);
    B.order.assign((size_t)kBatchPhases * n, 0);
    B.items = 0;
    for (int p = 0; p < kBatchPhases; ++p) {
        std::vector<int> ord(n);
        for (int k = 0; k < n; ++k) ord[k] = k;
        // decreasing cost; images without items in this phase (cost 0) last,
        // where their start equals the phase's item count
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[p][a] > cost[p][b]; });
        long long acc = 0;
        for (int k = 0; k < n; ++k) {
            B.order[(size_t)p * n + k] = ord[k];
            B.start[(size_t)p * n + k] = acc;
            acc += cnt[p][ord[k]];
        }
        B.phase_items[p] = acc;
        B.items += acc;
    }
    B.total = off;
}

// The last few plans, reused when a call repeats one exactly (the same
// descriptor bytes, stack type, flags, tile form and workspace): a serving
// loop filters batches of the same images, and planning them costs host time
// that would otherwise sit in front of every launch.
struct PlanKey {
    std::vector<char> descs;
    int dtype, RV, RH;
    unsigned flags;
    bool fused;
    const char *ws;
    bool operator==(const PlanKey &o) const {
        return dtype == o.dtype && RV == o.RV && RH == o.RH && flags == o.flags && fused == o.fused && ws == o.ws &&
               descs == o.descs;
    }
};
static std::mutex g_plan_mtx;
static std::vector<std::pair<PlanKey, std::shared_ptr<const BatchPlan>>> g_plans;

static std::shared_ptr<const BatchPlan> cached_plan(const bf_image_desc *d, int count, int dtype, unsigned flags,
                                                    int RV, int RH, bool fused, char *ws) {
    PlanKey key{std::vector<char>((const char *)d, (const char *)(d + count)), dtype, RV, RH, flags, fused, ws};
    {
        std::lock_guard<std::mutex> lock(g_plan_mtx);
        for (size_t i = 0; i < g_plans.size(); ++i)
            if (g_plans[i].first == key) return g_plans[i].second;
    }
    auto B = std::make_shared<BatchPlan>();
    plan_batch(d, count, dtype, flags, RV, RH, fused, ws, *B);
    std::lock_guard<std::mutex> lock(g_plan_mtx);
    if (g_plans.size() >= 8) g_plans.erase(g_plans.begin());
    g_plans.emplace_back(std::move(key), B);
    return B;
}

static void pack_blob(const BatchPlan &B, char *host) {
    std::memset(host, 0, B.blob_bytes);
    const size_t n = B.img.size();
    BatchHeader *h = (BatchHeader *)host;
    h->flags = 0;
    h->count = (int)n;
    for (int p = 0; p < kBatchPhases; ++p) h->items[p] = B.phase_items[p];
    char *q = host + sizeof(BatchHeader);
    std::memcpy(q, B.img.data(), sizeof(BatchImage) * n);
    q += sizeof(BatchImage) * n;
    std::memcpy(q, B.start.data(), sizeof(long long) * kBatchPhases * n);
    q += sizeof(long long) * kBatchPhases * n;
    std::memcpy(q, B.order.data(), sizeof(int) * kBatchPhases * n);
    size_t poff = batch_head_bytes(n);
    for (const std::vector<double> &pv : B.prm) {
        std::memcpy(host + poff, pv.data(), sizeof(double) * pv.size());
        poff += align256(sizeof(double) * pv.size());
    }
}

// Pinned staging for the blob: two slots used in turn, each guarded by an
// event, so a slot is rewritten only after the copy that read it has run.
struct StageSlot {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
// Phase kernels of one batched launch (each takes the device blob).
struct BatchKernels {
    int n = 0;
    const void *func[kBatchPhases];
    int grid[kBatchPhases];
    bool items_grid[kBatchPhases] = {};   // grid = the phase's item count (set at every graph launch)
    int block[kBatchPhases];
    size_t lds = 0;
};
struct GraphEntry {
    void *ws;
    hipStream_t stream;
    size_t cap;
    int slot;
    BatchKernels k;
    hipGraphNode_t nodes[kBatchPhases];
    hipGraphExec_t exec;
    hipGraph_t graph;
};
static std::mutex g_batch_mtx;
static StageSlot g_slots[2];
static int g_next_slot = 0;
static std::vector<GraphEntry> g_graphs;

// Same kernels and launch shape; grids that follow the item count may differ
// (the cached graph's nodes are updated to the new grid before its launch).
static bool same_kernels(const BatchKernels &a, const BatchKernels &b) {
    if (a.n != b.n || a.lds != b.lds) return false;
    for (int i = 0; i < a.n; ++i)
        if (a.func[i] != b.func[i] || a.block[i] != b.block[i] || a.items_grid[i] != b.items_grid[i] ||
            (!a.items_grid[i] && a.grid[i] != b.grid[i]))
            return false;
    return true;
}

static hipKernelNodeParams kernel_node(const BatchKernels &K, int p, void **args) {
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.func = (void *)K.func[p];
    kp.gridDim = dim3(K.grid[p]);
    kp.blockDim = dim3(K.block[p]);
    kp.sharedMemBytes = (unsigned)K.lds;
    kp.kernelParams = args;
    return kp;
}

static bf_status stage_slot(size_t cap, int *slot_out) {
    const int k = g_next_slot;
    g_next_slot ^= 1;
    StageSlot &S = g_slots[k];
    hipError_t e = hipSuccess;
    if (S.pending) {
        e = hipEventSynchronize(S.ev);
        S.pending = false;
    }
    if (e == hipSuccess && S.cap < cap) {
        if (S.host) {
            e = hipHostFree(S.host);
            // graphs that copy from the old buffer are stale
            for (size_t i = 0; i < g_graphs.size();)
                if (g_graphs[i].slot == k) {
                    (void)hipGraphExecDestroy(g_graphs[i].exec);
                    (void)hipGraphDestroy(g_graphs[i].graph);
                    g_graphs.erase(g_graphs.begin() + i);
                } else ++i;
        }
        S.host = nullptr;
        S.cap = 0;
        if (e == hipSuccess) e = hipHostMalloc((void **)&S.host, cap, hipHostMallocDefault);
        if (e == hipSuccess) S.cap = cap;
    }
    if (e == hipSuccess && !S.ev) e = hipEventCreateWithFlags(&S.ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string("batched staging: ") + hipGetErrorString(e));
    *slot_out = k;
    return BF_OK;
}

// Blocks for a phase kernel: enough to fill every CU at its occupancy, never
// more than the phase has items.
static int phase_grid(const void *kernel, long long items, int block, size_t lds) {
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, lds);
    const long long full = (long long)std::max(1, cus) * std::max(block >= 512 ? 1 : 4, per);
    return (int)std::max(1LL, std::min(full, items));
}

// Uploads the planned blob and runs the phase kernels, through a cached
// hipGraph (memcpy node + one kernel node per phase) or as plain launches.
static bf_status launch_batch(const BatchPlan &B, const BatchKernels &K, unsigned flags, char *ws,
                              hipStream_t stream) {
    note_range_words(ws, 0);
    std::lock_guard<std::mutex> lock(g_batch_mtx);
    int slot = 0;
    bf_status st = stage_slot(B.blob_cap, &slot);
    if (st != BF_OK) return st;
    pack_blob(B, g_slots[slot].host);
    hipError_t e = hipSuccess;
    if (flags & BF_FLAG_GRAPH) {
        char *blob = ws;
        void *args[] = {&blob};
        GraphEntry *G = nullptr;
        for (size_t i = 0; i < g_graphs.size() && !G; ++i) {
            GraphEntry &g = g_graphs[i];
            if (g.ws != ws || g.stream != stream || g.cap != B.blob_cap || g.slot != slot || !same_kernels(g.k, K))
                continue;
            bool ok = true;
            for (int p = 0; p < K.n && ok; ++p)
                if (K.items_grid[p] && K.grid[p] != g.k.grid[p]) {
                    const hipKernelNodeParams kp = kernel_node(K, p, args);
                    ok = hipGraphExecKernelNodeSetParams(g.exec, g.nodes[p], &kp) == hipSuccess;
                    if (ok) g.k.grid[p] = K.grid[p];
                }
            if (ok) {
                G = &g;
            } else {                          // not updatable: rebuild below
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(g.exec);
                (void)hipGraphDestroy(g.graph);
                g_graphs.erase(g_graphs.begin() + i);
                break;
            }
        }
        if (!G) {
            GraphEntry g;
            g.ws = ws;
            g.stream = stream;
            g.cap = B.blob_cap;
            g.slot = slot;
            g.k = K;
            hipGraphNode_t prev;
            e = hipGraphCreate(&g.graph, 0);
            if (e == hipSuccess)
                e = hipGraphAddMemcpyNode1D(&prev, g.graph, nullptr, 0, ws, g_slots[slot].host, B.blob_cap,
                                            hipMemcpyHostToDevice);
            for (int p = 0; p < K.n && e == hipSuccess; ++p) {
                const hipKernelNodeParams kp = kernel_node(K, p, args);
                e = hipGraphAddKernelNode(&g.nodes[p], g.graph, &prev, 1, &kp);
                prev = g.nodes[p];
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string("batched graph: ") + hipGetErrorString(e));
            if (g_graphs.size() >= 32) {
                (void)hipGraphExecDestroy(g_graphs.front().exec);
                (void)hipGraphDestroy(g_graphs.front().graph);
                g_graphs.erase(g_graphs.begin());
            }
            g_graphs.push_back(g);
            G = &g_graphs.back();
        }
        ProfScope prof_("k_batched(graph)", stream);
        e = hipGraphLaunch(G->exec, stream);
    } else {
        e = hipMemcpyAsync(ws, g_slots[slot].host, B.blob_bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) {
            ProfScope prof_("k_batched", stream);
            char *blob = ws;
            void *args[] = {&blob};
            for (int p = 0; p < K.n && e == hipSuccess; ++p)
                e = hipLaunchKernel(K.func[p], dim3(K.grid[p]), dim3(K.block[p]), args, K.lds, stream);
            if (e == hipSuccess) e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(g_slots[slot].ev, stream);
    if (e != hipSuccess) return fail(BF_ERR_DEVICE, std::string("bf_gc_batched: ") + hipGetErrorString(e));
    g_slots[slot].pending = true;
    return BF_OK;
}

template <class S, int RV, int RH>
static bf_status run_batched(const bf_image_desc *descs, int count, int dtype, unsigned flags, int *status,
                             char *ws, size_t ws_bytes, hipStream_t stream) {
    const std::shared_ptr<const BatchPlan> plan = cached_plan(descs, count, dtype, flags, RV, RH, false, ws);
    const BatchPlan &B = *plan;
    for (int i = 0; i < count; ++i) status[i] = B.status[i];
    // descriptors (sub-ranges of routed images count one each) bound the item table in LDS
    if (B.img.size() > 2 * (size_t)kMaxBatch)
        return fail(BF_ERR_UNSUPPORTED, "batch: more than 2 BF_MAX_BATCH descriptors after the pivoted routing");
    if (ws_bytes < B.total) return fail(BF_ERR_WORKSPACE, "workspace smaller than bf_gc_batched_workspace_bytes()");
    if (B.items == 0) return BF_OK;
    BatchKernels K;
    K.n = 3;
    K.func[0] = (const void *)k_batched<S, RV, RH, 0>;
    K.func[1] = (const void *)k_batched<S, RV, RH, 1>;
    K.func[2] = (const void *)k_batched<S, RV, RH, 2>;
    K.lds = batch_lds_bytes((int)B.img.size());
    for (int p = 0; p < 3; ++p) {
        K.block[p] = 256;
        K.grid[p] = phase_grid(K.func[p], B.phase_items[p], K.block[p], K.lds);
    }
    // Small item tables: the column and row passes one block per item on the
    // LDS-staged tiles (the single-image kernels' form; the persistent
    // phases would wait on every item's staging in turn).
    int wmax = 0;
    for (const BatchImage &I : B.img) wmax = std::max(wmax, I.W);
    const size_t table = (batch_lds_bytes((int)B.img.size()) + 15) & ~(size_t)15;
    const size_t tile = (size_t)(4 * std::max(RV, RH) + 2 * wmax) * 64 * sizeof(typename S::T);
    if (B.img.size() <= kBatchItemsMaxTable && table + tile <= 65536) {
        K.func[1] = (const void *)k_batched_items<S, RV, RH, 1>;
        K.func[2] = (const void *)k_batched_items<S, RV, RH, 2>;
        K.lds = table + tile;   // the build phase needs only the table; one LDS size serves the graph's nodes
        for (int p = 1; p < 3; ++p) {
            if (B.phase_items[p] > INT_MAX) return fail(BF_ERR_UNSUPPORTED, "batch: too many tiles in a phase");
            K.grid[p] = (int)std::max(1LL, B.phase_items[p]);
            K.items_grid[p] = true;
        }
        K.grid[0] = phase_grid(K.func[0], B.phase_items[0], K.block[0], K.lds);
    }
    return launch_batch(B, K, flags, ws, stream);
}

// Fused FP16/BF16 form: one kernel per non-empty geometry class.
// The batched fused kernel of a plain class: one 16-wave block per item for
// FP16, on the single-image kernel's tiles (fused_geom: 64 x 128 to radius
// 32, 64 x 64 to 48), the persistent prefetching 8-wave form for BF16.
template <class M, int Q, int QA>
static const void *batched_fused_kernel() {
    if constexpr (M::kHalfPlanes) return (const void *)k_fused_batched_items<M, Q, (Q <= 4 ? 128 : 64), QA, 16>;
    else return (const void *)k_fused_batched<M, Q, (Q <= 4 ? 64 : 32), QA>;
}

template <class M>
static bf_status run_batched_fused(const bf_image_desc *descs, int count, int dtype, unsigned flags, int *status,
                                   char *ws, size_t ws_bytes, hipStream_t stream) {
    const std::shared_ptr<const BatchPlan> plan = cached_plan(descs, count, dtype, flags, 0, 0, true, ws);
    const BatchPlan &B = *plan;
    for (int i = 0; i < count; ++i) status[i] = B.status[i];
    if (ws_bytes < B.total) return fail(BF_ERR_WORKSPACE, "workspace smaller than bf_gc_batched_workspace_bytes()");
    if (B.items == 0) return BF_OK;
    const void *cls[kBatchPhases] = {
        batched_fused_kernel<M, 3, 0>(), batched_fused_kernel<M, 3, 1>(),
        batched_fused_kernel<M, 4, 1>(), batched_fused_kernel<M, 4, 2>(),
        batched_fused_kernel<M, 5, 2>(), batched_fused_kernel<M, 5, 3>(),
        (const void *)k_fused_batched_pivot_items<M, 3, 64, 0>, (const void *)k_fused_batched_pivot_items<M, 3, 64, 1>,
        (const void *)k_fused_batched_pivot_items<M, 4, 64, 1>, (const void *)k_fused_batched_pivot_items<M, 4, 64, 2>,
        (const void *)k_fused_batched_pivot_items<M, 5, 32, 2>, (const void *)k_fused_batched_pivot_items<M, 5, 32, 3>};
    BatchKernels K;
    K.lds = batch_lds_bytes((int)B.img.size());
    for (int c = 0; c < kBatchPhases; ++c)
        if (B.phase_items[c] > 0) {
            K.func[K.n] = cls[c];
            K.block[K.n] = M::kHalfPlanes && c < kFusedClasses ? 1024 : 512;
            if (M::kHalfPlanes || c >= kFusedClasses) {   // one block per item
                if (B.phase_items[c] > INT_MAX) return fail(BF_ERR_UNSUPPORTED, "fused batch: too many tiles in a class");
                K.grid[K.n] = (int)B.phase_items[c];
                K.items_grid[K.n] = true;
            } else {
                K.grid[K.n] = phase_grid(cls[c], B.phase_items[c], K.block[K.n], K.lds);
            }
            ++K.n;
        }
    return launch_batch(B, K, flags, ws, stream);
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

bf_status bf_gc_fit(double sigma_r, int N, unsigned flags, double *b_out, double *db_out, double *mu_out,
                    double *kernel_err, double *kappa) {
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (N < 1 || N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N out of [1, BF_MAX_DEGREE]");
    if (!b_out) return fail(BF_ERR_INVALID_ARG, "b_out is null");
    bf_status st = check_kind(sigma_r, N, flags);
    if (st != BF_OK) return st;
    const Fit &F = fit(sigma_r, N, kind_of(flags));
    for (int n = 0; n <= N; ++n) {
        b_out[n] = F.b[n];
        if (db_out) db_out[n] = F.bd[n];
    }
    if (mu_out) *mu_out = F.mu;
    if (kernel_err) *kernel_err = F.kernel_err;
    if (kappa) *kappa = F.kappa;
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
    // stack B holds the transposed column-filtered planes, or (recursive
    // variant) the planes in stack A's layout
    const size_t planesB = (size_t)(N + 2) * std::max((size_t)width * ldt_of(height),
                                                      (size_t)height * lds_of(width)) * esize(stack_dtype);
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
    int cfg = tile_config_of(flags);
    if (cfg == -2) return fail(BF_ERR_INVALID_ARG, "tile configuration out of range");
    if (flags & BF_FLAG_RECURSIVE) {
        if (stack_dtype != BF_STACK_F32) return fail(BF_ERR_UNSUPPORTED, "the recursive variant takes the FP32 stack");
        if (cfg != -1 || (flags & BF_FLAG_STAGED))
            return fail(BF_ERR_INVALID_ARG, "the recursive variant has its own kernels (no tile or staged flag)");
        return run_recursive<StF32>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    }
    if (cfg == -1) cfg = (fused_forward_applies(stack_dtype, sigma_s) && !(flags & BF_FLAG_STAGED)) ? BF_TILE_FUSED : 0;
    if (cfg == BF_TILE_FUSED) {
        if (!fused_forward_applies(stack_dtype, sigma_s))
            return fail(BF_ERR_UNSUPPORTED, "fused tile: FP16 stacks with radius <= BF_FUSED_F16_MAX_RADIUS or BF16 "
                                            "with radius <= BF_FUSED_MAX_RADIUS only");
        if (flags & BF_FLAG_STAGED) return fail(BF_ERR_INVALID_ARG, "fused tile and BF_FLAG_STAGED exclude each other");
        if (stack_dtype == BF_STACK_F16)
            return run_fused<MmaF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
        return run_fused<MmaBF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    }
#define BF_FWD(S, RV, RH) run_forward<S, RV, RH>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s)
#define BF_FWD_CFG(S)                                   \
    switch (cfg) {                                      \
    case 0: return BF_FWD(S, 16, 8);                    \
    case 1: return BF_FWD(S, 8, 8);                     \
    case 2: return BF_FWD(S, 16, 4);                    \
    default: return BF_FWD(S, 8, 4);                    \
    }
    switch (stack_dtype) {
    case BF_STACK_F32: BF_FWD_CFG(StF32)
    case BF_STACK_F16: BF_FWD_CFG(StF16)
    default: BF_FWD_CFG(StBF16)
    }
#undef BF_FWD_CFG
#undef BF_FWD
}

bf_status bf_gc_forward_noalloc(const float *f, float *out, int height, int width, int ld, double sigma_s,
                                double sigma_r, int N, int stack_dtype, unsigned flags, unsigned *range_flag,
                                void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    const int cfg = tile_config_of(flags);
    if (cfg == -2 || (cfg != -1 && cfg != BF_TILE_FUSED) || (flags & (BF_FLAG_STAGED | BF_FLAG_RECURSIVE)))
        return fail(BF_ERR_INVALID_ARG, "bf_gc_forward_noalloc runs the fused tile only (no staged, recursive or "
                                        "three-kernel tile flags)");
    if (!fused_forward_applies(stack_dtype, sigma_s))
        return fail(BF_ERR_UNSUPPORTED, "bf_gc_forward_noalloc: FP16 stacks with radius <= BF_FUSED_F16_MAX_RADIUS "
                                        "or BF16 with radius <= BF_FUSED_MAX_RADIUS only");
    if (height == 0 || width == 0) return BF_OK;
    const FusedGeom G = fused_geom(stack_dtype, radius_of(sigma_s));
    const long long words = (long long)G.NW * fused_tiles(G, height, width);
    if (kFlagBytes + sizeof(unsigned) * (size_t)words > kNoAllocScratchBytes)
        return fail(BF_ERR_UNSUPPORTED, "bf_gc_forward_noalloc: image needs more than BF_NOALLOC_SCRATCH_BYTES of "
                                        "scratch (4 bytes per wave and tile: 32 bytes per 4096 output pixels for FP16, per 4096 "
                                        "up to radius 32 and 2048 above for BF16)");
    if (!f || !out) return fail(BF_ERR_INVALID_ARG, "f and out must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const size_t img = ((size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, img, out, img)) return fail(BF_ERR_INVALID_ARG, "out overlaps f");
    if ((st = check_conditioning(sigma_r, N, stack_dtype, flags)) != BF_OK) return st;
    void *ws = nullptr;
    if ((st = noalloc_scratch(&ws)) != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = stack_dtype == BF_STACK_F16
             ? run_fused<MmaF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s)
             : run_fused<MmaBF16>(f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s);
    if (st != BF_OK || !range_flag) return st;
    ProfScope prof_("k_or_range_words", s);
    hipLaunchKernelGGL(k_or_range_words, dim3(1), dim3(256), 0, s, (const unsigned *)((char *)ws + kFlagBytes),
                       (int)words, range_flag);
    return check_launch("k_or_range_words");
}

int bf_gc_pivot_count(double sigma_r, int stack_dtype) {
    if (!finite_pos(sigma_r) || stack_dtype < BF_STACK_F32 || stack_dtype > BF_STACK_BF16) return -1;
    for (int K = 1; K <= BF_MAX_PIVOTS; K *= 2)
        if (pivots_conditioned(sigma_r, K, stack_dtype)) return K;
    return -1;
}

int bf_gc_batched_route(double sigma_r, int N, int stack_dtype, unsigned flags) {
    if (check_common(1, 1, 1.0, sigma_r, N, stack_dtype) != BF_OK) return 0;
    bf_status st;
    return batch_route(sigma_r, N, stack_dtype, flags, &st);
}

bf_status bf_gc_pivot_plan(double sigma_r, int K, int N, int *N_out, double *mu_out, double *kappa_out) {
    if (!finite_pos(sigma_r)) return fail(BF_ERR_INVALID_ARG, "sigma_r must be positive and finite");
    if (K < 1 || K > BF_MAX_PIVOTS) return fail(BF_ERR_INVALID_ARG, "K out of [1, BF_MAX_PIVOTS]");
    if (N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N above BF_MAX_DEGREE");
    const std::vector<Pivot> plan = pivot_plan(sigma_r, K, N, BF_MAX_DEGREE);
    for (int k = 0; k < K; ++k) {
        if (N_out) N_out[k] = plan[k].N;
        if (mu_out) mu_out[k] = plan[k].mu;
        if (kappa_out) kappa_out[k] = plan[k].N >= 1 ? fit_mu(plan[k].mu, plan[k].N).kappa : INFINITY;
    }
    return BF_OK;
}

size_t bf_gc_pivots_workspace_bytes(int height, int width, double sigma_s, double sigma_r, int K, int N,
                                    int stack_dtype) {
    if (check_common(height, width, sigma_s, sigma_r, 1, stack_dtype) != BF_OK) return 0;
    if (K < 1 || K > BF_MAX_PIVOTS || N > BF_MAX_DEGREE) return 0;
    const std::vector<Pivot> plan = pivot_plan(sigma_r, K, N, BF_MAX_DEGREE);
    for (const Pivot &p : plan)
        if (p.N < 1) return 0;
    return pivots_ws_bytes(height, width, radius_of(sigma_s), K, pivot_nmax(plan), stack_dtype);
}

bf_status bf_gc_forward_pivots(const float *f, float *out, int height, int width, int ld, double sigma_s,
                               double sigma_r, int K, int N, int stack_dtype, unsigned flags, void *ws,
                               size_t ws_bytes, void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, 1, stack_dtype);
    if (st != BF_OK) return st;
    if (K < 1 || K > BF_MAX_PIVOTS) return fail(BF_ERR_INVALID_ARG, "K out of [1, BF_MAX_PIVOTS]");
    if (N > BF_MAX_DEGREE) return fail(BF_ERR_INVALID_ARG, "degree N above BF_MAX_DEGREE");
    if (flags & (BF_FLAG_TAYLOR | BF_FLAG_MINIMAX | BF_FLAG_STAGED))
        return fail(BF_ERR_INVALID_ARG, "the pivoted form takes the Chebyshev coefficients and no staged flag");
    int cfg = tile_config_of(flags);
    if (cfg == -2) return fail(BF_ERR_INVALID_ARG, "tile configuration out of range");
    if (cfg == -1) cfg = fused_applies(stack_dtype, sigma_s) ? BF_TILE_FUSED : 0;
    if (cfg == BF_TILE_FUSED && !fused_applies(stack_dtype, sigma_s))
        return fail(BF_ERR_UNSUPPORTED, "fused tile: FP16/BF16 stacks with radius <= BF_FUSED_MAX_RADIUS only");
    if (height == 0 || width == 0) return BF_OK;
    if (!f || !out) return fail(BF_ERR_INVALID_ARG, "f and out must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const size_t img = ((size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, img, out, img)) return fail(BF_ERR_INVALID_ARG, "out overlaps f");
    const std::vector<Pivot> plan = pivot_plan(sigma_r, K, N, BF_MAX_DEGREE);
    for (const Pivot &p : plan) {
        if (p.N < 1) return fail(BF_ERR_UNSUPPORTED, "no degree <= BF_MAX_DEGREE meets the rule for a sub-range");
        if (!(flags & BF_FLAG_ALLOW_ILL_CONDITIONED)) {
            const double kappa = fit_mu(p.mu, p.N).kappa;
            if (!std::isfinite(kappa) || kappa * unit_roundoff(stack_dtype) > 1e-2) {
                char buf[200];
                snprintf(buf, sizeof buf, "ill-conditioned sub-range: kappa=%.3g at mu=%g, N=%d (more sub-ranges "
                                          "lower mu)", kappa, p.mu, p.N);
                return fail(BF_ERR_ILL_CONDITIONED, buf);
            }
        }
    }
    const size_t need = pivots_ws_bytes(height, width, radius_of(sigma_s), K, pivot_nmax(plan), stack_dtype);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null, misaligned or too small");
    hipStream_t s = (hipStream_t)stream;
    if (cfg == BF_TILE_FUSED) {
        if (stack_dtype == BF_STACK_F16)
            return run_fused_pivots<MmaF16>(f, out, height, width, ld, sigma_s, plan, (char *)ws, s);
        return run_fused_pivots<MmaBF16>(f, out, height, width, ld, sigma_s, plan, (char *)ws, s);
    }
#define BF_PIV(S, RV, RH) run_pivots<S, RV, RH>(f, out, height, width, ld, sigma_s, plan, stack_dtype, (char *)ws, s)
#define BF_PIV_CFG(S)                                   \
    switch (cfg) {                                      \
    case 0: return BF_PIV(S, 16, 8);                    \
    case 1: return BF_PIV(S, 8, 8);                     \
    case 2: return BF_PIV(S, 16, 4);                    \
    default: return BF_PIV(S, 8, 4);                    \
    }
    switch (stack_dtype) {
    case BF_STACK_F32: BF_PIV_CFG(StF32)
    case BF_STACK_F16: BF_PIV_CFG(StF16)
    default: BF_PIV_CFG(StBF16)
    }
#undef BF_PIV_CFG
#undef BF_PIV
}

size_t bf_gc_joint_workspace_bytes(int height, int width, double sigma_s, int N, int stack_dtype) {
    if (check_common(height, width, sigma_s, 30.0, N, stack_dtype) != BF_OK) return 0;
    const size_t planes = 2 * ((size_t)N + 1);
    const size_t A = planes * height * lds_of(width) * esize(stack_dtype);
    const size_t B = planes * width * ldt_of(height) * esize(stack_dtype);
    return kFlagBytes + align256(bf_gc_param_bytes(sigma_s, N)) + align256(A) + align256(B);
}

bf_status bf_gc_joint_forward(const float *g, const float *f, float *out, int height, int width, int ld,
                              double sigma_s, double sigma_r, int N, int stack_dtype, unsigned flags, void *ws,
                              size_t ws_bytes, void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (height == 0 || width == 0) return BF_OK;
    if (!g || !f || !out) return fail(BF_ERR_INVALID_ARG, "g, f and out must be non-null");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const size_t img = ((size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, img, out, img) || overlaps(g, img, out, img))
        return fail(BF_ERR_INVALID_ARG, "out overlaps f or g");
    if (flags & BF_FLAG_STAGED) return fail(BF_ERR_INVALID_ARG, "the joint filter has no staged form");
    if ((st = check_conditioning(sigma_r, N, stack_dtype, flags)) != BF_OK) return st;
    const size_t need = bf_gc_joint_workspace_bytes(height, width, sigma_s, N, stack_dtype);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null, misaligned or too small");
    int cfg = tile_config_of(flags);
    if (cfg == -2) return fail(BF_ERR_INVALID_ARG, "tile configuration out of range");
    const bool fusable = stack_dtype != BF_STACK_F32 && radius_of(sigma_s) <= kJointFusedMaxRadius;
    if (cfg == -1) cfg = fusable ? BF_TILE_FUSED : 0;
    hipStream_t s = (hipStream_t)stream;
    if (cfg == BF_TILE_FUSED) {
        if (!fusable) return fail(BF_ERR_UNSUPPORTED, "fused joint filter: FP16/BF16 stacks with radius <= BF_FUSED_MAX_RADIUS only");
        if (stack_dtype == BF_STACK_F16)
            return run_joint_fused<MmaF16>(g, f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags,
                                           (char *)ws, s);
        return run_joint_fused<MmaBF16>(g, f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags,
                                        (char *)ws, s);
    }
#define BF_JNT(S, RV, RH) run_joint_forward<S, RV, RH>(g, f, out, height, width, ld, sigma_s, sigma_r, N, stack_dtype, flags, (char *)ws, s)
#define BF_JNT_CFG(S)                                   \
    switch (cfg) {                                      \
    case 0: return BF_JNT(S, 16, 8);                    \
    case 1: return BF_JNT(S, 8, 8);                     \
    case 2: return BF_JNT(S, 16, 4);                    \
    default: return BF_JNT(S, 8, 4);                    \
    }
    switch (stack_dtype) {
    case BF_STACK_F32: BF_JNT_CFG(StF32)
    case BF_STACK_F16: BF_JNT_CFG(StF16)
    default: BF_JNT_CFG(StBF16)
    }
#undef BF_JNT_CFG
#undef BF_JNT
}

bf_status bf_gc_backward(const float *f, const float *grad_out, float *grad_f, double *grad_sigma_r, int height,
                         int width, int ld, double sigma_s, double sigma_r, int N, int stack_dtype, unsigned flags,
                         void *ws, size_t ws_bytes, void *stream) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, stack_dtype);
    if (st != BF_OK) return st;
    if (stack_dtype != BF_STACK_F32) return fail(BF_ERR_UNSUPPORTED, "the backward runs with an FP32 stack only");
    if (!grad_sigma_r) return fail(BF_ERR_INVALID_ARG, "grad_sigma_r must be non-null");
    if (height == 0 || width == 0) {   // empty image: dL/dsigma_r = 0 (a kernel, so the call can be graph-captured)
        hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, (hipStream_t)stream, (const double *)nullptr, 0LL,
                           0.0, grad_sigma_r);
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
    return run_backward(f, grad_out, grad_f, grad_sigma_r, height, width, ld, sigma_s, sigma_r, N, flags,
                        (char *)ws, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Forward with saved sums + backward from them (the fused FP64 tiles)
// ---------------------------------------------------------------------------

static size_t saving_partial_bytes(int count, int height, int width) {
    return align256((size_t)count * bwd_tiles(height, width) * sizeof(double));
}

size_t bf_gc_saving_workspace_bytes(int count, int height, int width, double sigma_s, int N) {
    if (count < 0 || check_common(height, width, sigma_s, 30.0, N, BF_STACK_F32) != BF_OK) return 0;
    const size_t params = align256(sizeof(double) * (size_t)param_layout(radius_of(sigma_s), N).total);
    return kFlagBytes + params + saving_partial_bytes(count, height, width);
}

// Shared argument checks of the two calls; *empty when there is nothing to do.
// out (the forward's y, the backward's grad_f) and saved: both required when
// `both`, else at least one (the forward may keep either).
static bf_status check_saving(const float *f, const void *out, const void *saved, bool both, int count,
                              long long stride, int height, int width, int ld, double sigma_s, double sigma_r, int N,
                              unsigned flags, void *ws, size_t ws_bytes, bool *empty) {
    bf_status st = check_common(height, width, sigma_s, sigma_r, N, BF_STACK_F32);
    if (st != BF_OK) return st;
    if (count < 0 || count > 65535) return fail(BF_ERR_INVALID_ARG, "count out of [0, 65535]");
    if (radius_of(sigma_s) > kAdjMaxRadius) return fail(BF_ERR_UNSUPPORTED, "radius W above BF_ADJ_MAX_RADIUS");
    *empty = count == 0 || height == 0 || width == 0;
    if (*empty) return BF_OK;
    if (!f || (both ? !out || !saved : !out && !saved))
        return fail(BF_ERR_INVALID_ARG, both ? "image, output and saved pointers must be non-null"
                                             : "f must be non-null, and out or saved");
    if (ld < width) return fail(BF_ERR_INVALID_ARG, "ld must be >= width");
    const long long img = (long long)(height - 1) * ld + width;
    if (count > 1 && stride < img) return fail(BF_ERR_INVALID_ARG, "image_stride smaller than one image");
    if ((st = check_conditioning(sigma_r, N, BF_STACK_F32, flags)) != BF_OK) return st;
    const size_t need = bf_gc_saving_workspace_bytes(count, height, width, sigma_s, N);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null, misaligned or too small");
    return BF_OK;
}

bf_status bf_gc_forward_saving(const float *f, float *out, double *saved, int count, long long image_stride,
                               int height, int width, int ld, double sigma_s, double sigma_r, int N, unsigned flags,
                               void *ws, size_t ws_bytes, void *stream) {
    bool empty = false;
    bf_status st = check_saving(f, out, saved, false, count, image_stride, height, width, ld, sigma_s, sigma_r, N,
                                flags, ws, ws_bytes, &empty);
    if (st != BF_OK || empty) return st;
    const size_t span = ((size_t)(count - 1) * image_stride + (size_t)(height - 1) * ld + width) * sizeof(float);
    const size_t sbytes = (size_t)count * 6 * height * width * sizeof(double);
    if ((out && overlaps(f, span, out, span)) || (saved && overlaps(saved, sbytes, f, span)) ||
        (out && saved && overlaps(saved, sbytes, out, span)))
        return fail(BF_ERR_INVALID_ARG, "out, saved and f overlap");
    hipStream_t s = (hipStream_t)stream;
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)((char *)ws + kFlagBytes);
    ParamLayout L;
    if ((st = upload_params(prm, flag, sigma_s, sigma_r, N, BF_STACK_F32, s, &L, kind_of(flags))) != BF_OK) return st;
    return launch_adj_forward(f, out, saved, count, image_stride, height, width, ld, N, fit(sigma_r, N).mu, prm, L,
                              flag, s);
}

bf_status bf_gc_backward_saving(const float *f, const float *grad_out, const double *saved, float *grad_f,
                                double *grad_sigma_r, int count, long long image_stride, int height, int width,
                                int ld, double sigma_s, double sigma_r, int N, unsigned flags, void *ws,
                                size_t ws_bytes, void *stream) {
    if (!grad_sigma_r) return fail(BF_ERR_INVALID_ARG, "grad_sigma_r must be non-null");
    bool empty = false;
    bf_status st = check_saving(f, grad_f, saved, true, count, image_stride, height, width, ld, sigma_s, sigma_r, N,
                                flags, ws, ws_bytes, &empty);
    if (st != BF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (empty) {   // dL/dsigma_r = 0 (a kernel, so the call can be graph-captured)
        hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, s, (const double *)nullptr, 0LL, 0.0, grad_sigma_r);
        return check_launch("k_reduce_f64");
    }
    if (!grad_out) return fail(BF_ERR_INVALID_ARG, "grad_out must be non-null");
    const size_t span = ((size_t)(count - 1) * image_stride + (size_t)(height - 1) * ld + width) * sizeof(float);
    if (overlaps(f, span, grad_f, span) || overlaps(grad_out, span, grad_f, span) ||
        overlaps(saved, (size_t)count * 6 * height * width * sizeof(double), grad_f, span))
        return fail(BF_ERR_INVALID_ARG, "grad_f overlaps f, grad_out or saved");
    unsigned *flag = (unsigned *)ws;
    double *prm = (double *)((char *)ws + kFlagBytes);
    ParamLayout L;
    if ((st = upload_params(prm, flag, sigma_s, sigma_r, N, BF_STACK_F32, s, &L, kind_of(flags))) != BF_OK) return st;
    double *partial = (double *)((char *)prm + align256(sizeof(double) * (size_t)L.total));
    return launch_adj_backward(f, grad_out, saved, grad_f, grad_sigma_r, partial, count, image_stride, height, width,
                               ld, N, fit(sigma_r, N).mu, sigma_r, prm, L, s);
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

size_t bf_gc_batched_workspace_bytes(const bf_image_desc *descs, int count, int stack_dtype) {
    if (count < 0 || count > kMaxBatch || (count > 0 && !descs) || stack_dtype < BF_STACK_F32 ||
        stack_dtype > BF_STACK_BF16)
        return 0;
    // the three-kernel layout (blob and stacks) covers the fused one (blob
    // only); images are sized both as their own expansion and as routed to
    // the pivoted form
    BatchPlan A, B;
    plan_batch(descs, count, stack_dtype, BF_FLAG_ALLOW_ILL_CONDITIONED, 16, 8, false, nullptr, A, true);
    plan_batch(descs, count, stack_dtype, 0, 16, 8, false, nullptr, B, true);
    return std::max(A.total, B.total);
}

bf_status bf_gc_batched(const bf_image_desc *descs, int count, int stack_dtype, unsigned flags,
                        int *per_image_status, void *ws, size_t ws_bytes, void *stream) {
    if (count < 0) return fail(BF_ERR_INVALID_ARG, "count must be >= 0");
    if (count == 0) return BF_OK;
    if (count > kMaxBatch) return fail(BF_ERR_UNSUPPORTED, "more images than BF_MAX_BATCH");
    if (!descs || !per_image_status) return fail(BF_ERR_INVALID_ARG, "descs and per_image_status must be non-null");
    if (stack_dtype < BF_STACK_F32 || stack_dtype > BF_STACK_BF16) return fail(BF_ERR_INVALID_ARG, "unknown stack dtype");
    int cfg = tile_config_of(flags);
    if (cfg == -2) return fail(BF_ERR_INVALID_ARG, "tile configuration out of range");
    if (cfg == -1) {
        // the fused form where it covers every image the call would filter
        bool fused = stack_dtype != BF_STACK_F32;
        for (int i = 0; i < count && fused; ++i) {
            const bf_image_desc &x = descs[i];
            if (x.height > 0 && x.width > 0 && finite_pos(x.sigma_s) && radius_of(x.sigma_s) > BF_FUSED_MAX_RADIUS)
                fused = false;
        }
        cfg = fused ? BF_TILE_FUSED : 0;
    }
    if (!ws || ((uintptr_t)ws & 255)) return fail(BF_ERR_WORKSPACE, "workspace null or misaligned");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    if (cfg == BF_TILE_FUSED) {
        if (stack_dtype == BF_STACK_F32) return fail(BF_ERR_UNSUPPORTED, "fused tile: FP16/BF16 stacks only");
        if (stack_dtype == BF_STACK_F16)
            return run_batched_fused<MmaF16>(descs, count, stack_dtype, flags, per_image_status, w, ws_bytes, s);
        return run_batched_fused<MmaBF16>(descs, count, stack_dtype, flags, per_image_status, w, ws_bytes, s);
    }
#define BF_BAT(S, RV, RH) run_batched<S, RV, RH>(descs, count, stack_dtype, flags, per_image_status, w, ws_bytes, s)
#define BF_BAT_CFG(S)                                   \
    switch (cfg) {                                      \
    case 0: return BF_BAT(S, 16, 8);                    \
    case 1: return BF_BAT(S, 8, 8);                     \
    case 2: return BF_BAT(S, 16, 4);                    \
    default: return BF_BAT(S, 8, 4);                    \
    }
    switch (stack_dtype) {
    case BF_STACK_F32: BF_BAT_CFG(StF32)
    case BF_STACK_F16: BF_BAT_CFG(StF16)
    default: BF_BAT_CFG(StBF16)
    }
#undef BF_BAT_CFG
#undef BF_BAT
}

bf_status bf_gc_read_flags(const void *ws, unsigned *flags_out, void *stream) {
    if (!ws || !flags_out) return fail(BF_ERR_INVALID_ARG, "ws and flags_out must be non-null");
    long long words = 0;
    {
        std::lock_guard<std::mutex> lock(g_range_mtx);
        auto it = g_range_words.find(ws);
        if (it != g_range_words.end()) words = it->second;
    }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess && words > 0) {
        std::vector<unsigned> w((size_t)words);
        e = hipMemcpy(w.data(), (const char *)ws + kFlagBytes, sizeof(unsigned) * w.size(), hipMemcpyDeviceToHost);
        unsigned acc = 0;
        for (unsigned x : w) acc |= x;
        *flags_out = acc;
    } else if (e == hipSuccess) {
        e = hipMemcpy(flags_out, ws, sizeof(unsigned), hipMemcpyDeviceToHost);
    }
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
