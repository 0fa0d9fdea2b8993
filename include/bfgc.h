/*
 * bfgc: Gauss-Chebyshev bilateral filter on AMD Instinct MI355X (gfx950).
 *
 * Method (Ghosh & Chaudhury, "Fast and High-Quality Bilateral Filtering Using
 * Gauss-Chebyshev Approximation", 2016):
 *
 *   B[f](i) = sum_j g_s(j) g_r(f(i-j) - f(i)) f(i-j) / sum_j g_s(j) g_r(f(i-j) - f(i))
 *
 * over the square Omega = [-W, W]^2, W = ceil(3 sigma_s), with the image
 * extended outside its rectangle by symmetry (Section I, eq. 1). The range
 * kernel is factored (eq. 2) and its cross term exp(x), x in [-mu, mu],
 * mu = (U-L)^2 / (4 sigma_r^2), is replaced by the degree-N polynomial that
 * interpolates it at the scaled zeros of T_{N+1} (Section III, eq. 16 rescaled,
 * eq. 19). The filter then becomes (Section II, eqs. 6-10, centring eq. 17):
 *
 *   1. a stack of N+2 pointwise images of the centred input,
 *   2. the same truncated spatial Gaussian applied to every image,
 *   3. a per-pixel combine into numerator P and denominator Q, and P/Q.
 *
 * The library computes in the scaled variables s = (f - t_c)/t_h,
 * t_c = t_h = 127.5 ([L, U] = [0, 255]), H_n = exp(-mu s^2/2) s^n,
 * b_n = c_n mu^n; F_n of eq. (6) equals mu^{n/2} H_n, and
 *   y = t_c + t_h * (sum_n b_n s^n Hbar_{n+1}) / (sum_n b_n s^n Hbar_n),
 * which is eq. (10) with the centring undone.
 *
 * Conventions for every entry point below:
 *   - Images are FP32, row-major, row stride `ld` >= width (elements).
 *   - Device pointers are HIP device memory owned by the caller; the library
 *     never allocates device memory in these calls.
 *   - `stream` is a hipStream_t (NULL = the null stream). All GPU work is
 *     enqueued on it asynchronously; a returned BF_OK means the work was
 *     enqueued, not that it has finished.
 *   - Host-side argument checks run before anything is enqueued; on an error
 *     nothing is enqueued and bf_last_error() holds a message (per thread).
 *   - Inputs are expected in [0, 255]. A pixel outside it (or NaN) is not
 *     corrected; it sets bit BF_DEVFLAG_RANGE in the workspace flag word.
 *   - No entry point aborts or throws.
 */
#ifndef BFGC_H
#define BFGC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BF_OK = 0,
    BF_ERR_INVALID_ARG = 1,      /* null pointer, bad size, sigma <= 0 or not finite, N out of range, overlap */
    BF_ERR_UNSUPPORTED = 2,      /* radius W above BF_MAX_RADIUS, size beyond the index range */
    BF_ERR_ILL_CONDITIONED = 3,  /* (sigma_r, N, stack type) outside the numerically usable domain */
    BF_ERR_WORKSPACE = 4,        /* workspace null or smaller than bf_gc_workspace_bytes() */
    BF_ERR_DEVICE = 5            /* a HIP call failed; bf_last_error() has the HIP message */
} bf_status;

typedef enum {
    BF_STACK_F32 = 0,            /* stack planes stored in FP32 */
    BF_STACK_F16 = 1,            /* FP16, each plane scaled by a power of two 2^k_n */
    BF_STACK_BF16 = 2            /* BF16 */
} bf_stack_dtype;

/* flags */
#define BF_FLAG_ALLOW_ILL_CONDITIONED 0x1u  /* compute even where the conditioning check fails */
#define BF_FLAG_STAGED                0x2u  /* materialise the stack: build | filter | combine (one kernel each) */
#define BF_FLAG_GRAPH                 0x4u  /* bf_gc_batched: launch through a cached hipGraph */
/* Gauss-polynomial filter: the cross term exp(x) is replaced by its Taylor
 * polynomial, c_n = 1/n! (Section II), instead of the Chebyshev interpolant
 * of eq. 19. Accepted by bf_gc_forward, bf_gc_backward and bf_gc_batched. */
#define BF_FLAG_TAYLOR                0x8u
/* Minimax filter: the cross term is replaced by the best uniform polynomial
 * approximation of exp on [-mu, mu] of degree N (Remez exchange; Section III
 * names it the ideal choice, of which the Chebyshev interpolant is a near
 * version). Degrees up to BF_MINIMAX_MAX_DEGREE; where binary128 cannot
 * resolve the levelled error (the error below 1e-28 of e^mu) the call returns
 * BF_ERR_UNSUPPORTED. Accepted by bf_gc_forward, bf_gc_backward and
 * bf_gc_batched; with BF_FLAG_TAYLOR it is BF_ERR_INVALID_ARG. */
#define BF_FLAG_MINIMAX               0x10u
/* Recursive variant of eq. 7 (Section I: recursion as the O(1) way to apply
 * the Gaussian): Deriche's recursive Gaussian along columns and rows (causal
 * + anticausal 4th-order recursions in FP64, each line extended by 14 sigma_s
 * through the symmetric extension), then the combine. It approximates the
 * untruncated Gaussian (within 5e-4 of the peak), so it is a different filter
 * from the truncated convolution of the other paths. bf_gc_forward only, FP32
 * stack (others: BF_ERR_UNSUPPORTED), without tile or staged flags
 * (BF_ERR_INVALID_ARG). */
#define BF_FLAG_RECURSIVE             0x20u
#define BF_MINIMAX_MAX_DEGREE         100
/* Tile configuration c in [0, BF_TILE_CONFIGS).
 *   c = 0..3: the three-kernel path (stack in HBM); output rows per lane in
 *             the column pass and output columns per lane in the row pass +
 *             combine, {16,8}, {8,8}, {16,4}, {8,4}.
 *   c = BF_TILE_FUSED: FP16/BF16 stacks with radius ceil(3 sigma_s) <= 48
 *             only; one kernel per 64-row tile makes each plane in registers,
 *             runs both passes of eq. 7 on the matrix cores (FP32
 *             accumulation) and folds eqs. 8-10 in, so the stack never reaches
 *             HBM. Not combinable with BF_FLAG_STAGED; bf_gc_batched does not
 *             take it (BF_ERR_UNSUPPORTED).
 * Without the flag: BF_TILE_FUSED where it applies (FP16/BF16, radius <= 48,
 * no BF_FLAG_STAGED), else c = 0. */
#define BF_TILE_CONFIGS 5
#define BF_TILE_FUSED   4
#define BF_FUSED_MAX_RADIUS 48
/* bf_gc_forward and bf_gc_forward_noalloc run FP16 stacks on the fused tile up
 * to this radius (64 x 128 tiles on 16 waves up to radius 32, one block per
 * CU walking a vertical strip of tiles; 64 x 64 up to 48, 32 x 128 above);
 * BF16 stacks, and the other entry points, up to BF_FUSED_MAX_RADIUS. */
#define BF_FUSED_F16_MAX_RADIUS 64
#define BF_FLAG_TILE(c)               ((((unsigned)(c)) + 1u) << 8)

/* device flag word bits (read with bf_gc_read_flags) */
#define BF_DEVFLAG_RANGE 0x1u               /* some input pixel was outside [0, 255] or not finite */

#define BF_MAX_DEGREE 320                   /* largest N accepted */
#define BF_MAX_RADIUS 96                    /* largest W = ceil(3 sigma_s) accepted */
/* Largest image side: the launch grids put up to side/32 blocks in a 16-bit
 * grid dimension. Larger sides: BF_ERR_UNSUPPORTED. */
#define BF_MAX_SIDE 2097152
#define BF_MAX_BATCH 2048                   /* most images in one bf_gc_batched call */

/*
 * Degree for a given sigma_r when the caller has none. The paper fixes N per
 * experiment (N = 28 at sigma_r = 30, Table 2) and states no rule; this one
 * keeps that point and scales it through the first neglected Chebyshev
 * coefficient of exp(mu y): the smallest N with 2 I_{N+1}(mu) <= eps0, eps0 =
 * sqrt(2 I_28(mu30) 2 I_29(mu30)), I_k the modified Bessel function.
 * Returns N >= 1, or -1 for sigma_r <= 0 / not finite / N above BF_MAX_DEGREE.
 */
int bf_gc_degree_rule(double sigma_r);

/*
 * Monomial coefficients b_n = c_n mu^n, n = 0..N, of the interpolant of
 * exp(mu y) at the zeros of T_{N+1} (Section III-B, eq. 19 with the mu^-n
 * moved into the scaled variables). b_out: host array of N+1 doubles.
 * mu_out: host double (may be NULL).
 */
bf_status bf_gc_coefficients(double sigma_r, int N, double *b_out, double *mu_out);

/*
 * The polynomial the flags select (the Chebyshev interpolant of Section III;
 * BF_FLAG_TAYLOR: Taylor, Section II; BF_FLAG_MINIMAX: minimax), in the same
 * scaled monomial form: b_out[n] = b_n and db_out[n] = db_n/dmu, n = 0..N
 * (host arrays of N+1 doubles; db_out may be NULL), mu_out, kernel_err and
 * kappa as in bf_gc_query (each may be NULL). Errors as the forward's flag
 * and degree checks.
 */
bf_status bf_gc_fit(double sigma_r, int N, unsigned flags, double *b_out, double *db_out, double *mu_out,
                    double *kernel_err, double *kappa);

/*
 * Conditioning of the approximation for (sigma_r, N): kernel_err = max over
 * y in [-1,1] of exp(-mu|y|) |p_N(mu y) - exp(mu y)| (largest error of the
 * approximate range kernel, relative to its peak 1) and kappa = max over y of
 * exp(-mu|y|) sum_n |b_n| |y|^n (how much a relative rounding of the stack
 * grows in the kernel). Either output pointer may be NULL. stack_dtype is
 * accepted for symmetry and does not change the values.
 */
bf_status bf_gc_query(double sigma_r, int N, int stack_dtype, double *kernel_err, double *kappa);

/*
 * Workspace bytes needed by bf_gc_forward (for_backward = 0) or
 * bf_gc_backward (for_backward = 1) for one height x width image. Includes
 * the parameter block, the device flag word, N+2 stack planes and N+2
 * transposed column-filtered planes (for the backward: both in FP64, plus
 * four FP64 per-pixel arrays and the reduction partials). Returns 0 for
 * invalid arguments.
 */
size_t bf_gc_workspace_bytes(int height, int width, double sigma_s, int N, int stack_dtype,
                             int for_backward);

/*
 * Forward filter (Section III-B procedure: centre, fast algorithm with the
 * coefficients of eq. 19, undo the centring).
 *   f      device, height x width FP32 with row stride ld, read only
 *   out    device, height x width FP32 with row stride ld; must not overlap f
 *   height, width >= 0 (0 means nothing to do, BF_OK); ld >= width
 *   sigma_s > 0: spatial std. dev.; W = ceil(3 sigma_s) <= BF_MAX_RADIUS
 *   sigma_r > 0: range std. dev.
 *   N: degree, 1 <= N <= BF_MAX_DEGREE (bf_gc_degree_rule gives the default)
 *   stack_dtype: bf_stack_dtype
 *   flags: BF_FLAG_*
 *   ws, ws_bytes: device workspace of at least bf_gc_workspace_bytes(..., 0)
 *     bytes, 256-byte aligned; its contents on entry are ignored.
 * The range flags in ws describe this call only (bf_gc_read_flags): the
 * three-kernel paths clear the flag word before their kernels set it; the
 * fused path (one kernel, taps and coefficients passed as kernel arguments)
 * has every wave write its own flag word after the first 256 bytes.
 * Path: see BF_TILE_CONFIGS. BF_FLAG_TILE(BF_TILE_FUSED) with an FP32 stack
 * or a radius above BF_FUSED_MAX_RADIUS is BF_ERR_UNSUPPORTED, with
 * BF_FLAG_STAGED BF_ERR_INVALID_ARG.
 */
bf_status bf_gc_forward(const float *f, float *out, int height, int width, int ld,
                        double sigma_s, double sigma_r, int N, int stack_dtype, unsigned flags,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * Pivoted forward for small sigma_r (not in the paper). The single expansion
 * centres every pixel at t_c = 127.5, so the cross term spans [-mu, mu] with
 * mu = t_h^2/sigma_r^2, which grows as 1/sigma_r^2 and makes the monomial sums
 * ill-conditioned (FP32 fails below sigma_r ~ 20). Here [0, 255] is split
 * into K equal sub-ranges; for a pixel whose value lies in sub-range k the
 * expansion is centred at its midpoint t_k (eq. 17 with t_k), so the centre
 * offset is at most h = 127.5/K and the cross term spans [-mu_k, mu_k],
 * mu_k = h R_k / sigma_r^2 (R_k = max(t_k, 255 - t_k)). Each sub-range runs
 * the three-kernel forward over the whole image and keeps the outputs whose
 * centre value lies in it ([lo, hi); values below 0 go to the first, values
 * from 255 up and NaN to the last). With BF_TILE_FUSED (the default for
 * FP16/BF16 stacks with radius <= BF_FUSED_MAX_RADIUS; otherwise
 * BF_ERR_UNSUPPORTED) the sub-ranges run on the fused matrix-core tile
 * instead, each 64-row tile only those its own output pixels fall in, with
 * the same partition; the workspace then holds the range words, the
 * sub-range table, the tiles' sub-range masks, their order and a queue
 * counter (three launches after the table upload: masks, order, filter).
 *   K: sub-ranges, 1..BF_MAX_PIVOTS (K = 1 is the plain expansion)
 *   N: the degree of every sub-range, or <= 0 for the degree rule at mu_k
 *   other arguments as bf_gc_forward (Chebyshev coefficients only:
 *   BF_FLAG_TAYLOR, BF_FLAG_MINIMAX, BF_FLAG_STAGED are BF_ERR_INVALID_ARG).
 *   The conditioning check applies to every sub-range. ws: at least
 *   bf_gc_pivots_workspace_bytes(...) bytes (enough for either tile form).
 * bf_gc_pivot_count: the smallest K in {1, 2, 4, ..., BF_MAX_PIVOTS} whose
 * sub-ranges pass the conditioning check for the stack type at the rule's
 * degrees, or -1. bf_gc_pivot_plan: per sub-range (host arrays of K, each may
 * be NULL) its degree (-1 where the rule finds none), mu_k and kappa.
 */
#define BF_MAX_PIVOTS 64
int bf_gc_pivot_count(double sigma_r, int stack_dtype);
bf_status bf_gc_pivot_plan(double sigma_r, int K, int N, int *N_out, double *mu_out, double *kappa_out);
size_t bf_gc_pivots_workspace_bytes(int height, int width, double sigma_s, double sigma_r, int K, int N,
                                    int stack_dtype);
bf_status bf_gc_forward_pivots(const float *f, float *out, int height, int width, int ld, double sigma_s,
                               double sigma_r, int K, int N, int stack_dtype, unsigned flags, void *ws,
                               size_t ws_bytes, void *stream);

/*
 * Joint (cross) bilateral filter: the range kernel is evaluated on the guide
 * g and the values of f are averaged (the use the conclusion points to, e.g.
 * aggregation with an image as guide). Same expansion as bf_gc_forward with
 * the range variable from g: planes A_n = e^{-mu s^2/2} s^n (s from g) and
 * B_n = A_n (f - t_c)/t_h, both filtered (eq. 7), Q = sum b_n s_i^n Abar_n,
 * P = sum b_n s_i^n Bbar_n, y = t_c + t_h P/Q.
 *   g, f   device, height x width FP32, row stride ld (the same for both),
 *          read only; values in [0, 255] (others set BF_DEVFLAG_RANGE)
 *   out    device, same layout; must overlap neither g nor f
 *   other arguments as bf_gc_forward; 2(N+1) planes per stack. FP16/BF16
 *   stacks with radius <= BF_FUSED_MAX_RADIUS default to the fused
 *   matrix-core kernel (two operand sets per plane); BF_TILE_FUSED elsewhere
 *   is BF_ERR_UNSUPPORTED.
 *   No staged form (BF_FLAG_STAGED: BF_ERR_INVALID_ARG). ws: at least
 *   bf_gc_joint_workspace_bytes(...) bytes, 256-byte aligned.
 */
size_t bf_gc_joint_workspace_bytes(int height, int width, double sigma_s, int N, int stack_dtype);
bf_status bf_gc_joint_forward(const float *g, const float *f, float *out, int height, int width, int ld,
                              double sigma_s, double sigma_r, int N, int stack_dtype, unsigned flags,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * Backward of bf_gc_forward (not in the paper): for L = sum_i grad_out_i y_i
 * with y the forward output, writes grad_f = dL/df (device FP32, height x
 * width, row stride ld) and *grad_sigma_r = dL/dsigma_r (device double;
 * written, not accumulated). sigma_s and N are constants. The stack is
 * recomputed in FP64 (nothing is kept from the forward); the adjoint planes
 * R_m = dL/dHbar_m are filtered with the same Gaussian, which is its own
 * adjoint under the symmetric extension (radius <= BF_ADJ_MAX_RADIUS: two
 * fused FP64 tile kernels; larger radii: staged passes over two FP64 plane
 * stacks in the workspace). Arguments as bf_gc_forward;
 * stack_dtype must be BF_STACK_F32, the forward's stack type the gradient is
 * taken for (BF_ERR_UNSUPPORTED otherwise); ws of at
 * least bf_gc_workspace_bytes(..., 1) bytes. grad_f must not overlap f or
 * grad_out.
 */
bf_status bf_gc_backward(const float *f, const float *grad_out, float *grad_f, double *grad_sigma_r,
                         int height, int width, int ld, double sigma_s, double sigma_r, int N,
                         int stack_dtype, unsigned flags, void *ws, size_t ws_bytes, void *stream);

/*
 * Training pair (not in the paper): a forward that keeps what the backward
 * needs, and that backward. Radius W = ceil(3 sigma_s) <= BF_ADJ_MAX_RADIUS;
 * larger radii are BF_ERR_UNSUPPORTED (bf_gc_forward / bf_gc_backward serve
 * them). Both run on count images of one shape: image z starts image_stride
 * floats after image z - 1 (f, out, grad_out, grad_f alike; image_stride >=
 * (height - 1) ld + width when count > 1), count in [0, 65535].
 *
 * bf_gc_forward_saving: the filter of eqs. 7-10 (plain centring, coefficients
 * as flags select, the conditioning check of the FP32 stack) with the planes
 * H_n = e^{-mu s^2/2} s^n generated and filtered in FP64, tile by tile; y to
 * out (FP32, as bf_gc_forward) and six sums per pixel to saved (device
 * doubles, count x 6 x height x width, [count][6][height][width],
 * caller-allocated): P' = sum b_n s^n Hbar_{n+1}, Q = sum b_n s^n Hbar_n,
 * their derivatives in the explicit powers of s, and the same sums with
 * db_n/dmu. Either of out and saved may be null (y only, for a forward that
 * keeps nothing; the sums only, to recompute them in a backward), not both.
 * Inputs outside [0, 255] set BF_DEVFLAG_RANGE in the workspace's flag word.
 * out and saved must overlap neither f nor each other.
 *
 * bf_gc_backward_saving: for L = sum_z sum_i grad_out_{z,i} y_{z,i}, grad_f =
 * dL/df (FP32, layout of f) and *grad_sigma_r = dL/dsigma_r summed over the
 * count images (one device double; written, not accumulated; 0 for an empty
 * batch), from f, grad_out and the saved sums of the forward with the same
 * f, sigma_s, sigma_r, N and flags. The adjoint planes R_m are filtered in FP64
 * tile by tile (as in bf_gc_backward). grad_f must not overlap f, grad_out
 * or saved.
 *
 * ws (both): device, 256-byte aligned, at least
 * bf_gc_saving_workspace_bytes(count, height, width, sigma_s, N) bytes (0 for
 * invalid sizes); it holds the flag word, the parameters and one partial sum
 * per 64 x 32 tile and image.
 */
#define BF_ADJ_MAX_RADIUS 16
size_t bf_gc_saving_workspace_bytes(int count, int height, int width, double sigma_s, int N);
bf_status bf_gc_forward_saving(const float *f, float *out, double *saved, int count, long long image_stride,
                               int height, int width, int ld, double sigma_s, double sigma_r, int N,
                               unsigned flags, void *ws, size_t ws_bytes, void *stream);
bf_status bf_gc_backward_saving(const float *f, const float *grad_out, const double *saved, float *grad_f,
                                double *grad_sigma_r, int count, long long image_stride, int height, int width,
                                int ld, double sigma_s, double sigma_r, int N, unsigned flags, void *ws,
                                size_t ws_bytes, void *stream);

/*
 * Stages of the forward filter, for callers that want the stack itself. These
 * are the kernels bf_gc_forward runs with BF_FLAG_STAGED. The stack is N+2
 * planes of height x width, plane stride `plane_stride` and row stride `lds`
 * elements (both multiples of 16, lds >= width, stack 16-byte aligned),
 * element type per stack_dtype; plane n holds 2^k_n H_n (k_n = 0 except for
 * FP16, see bf_gc_plane_scales).
 *
 * bf_gc_stack_build: H_n = exp(-mu s^2/2) s^n, n = 0..N+1 (eq. 6 scaled,
 *   centring eq. 17). Sets the range flag in *devflag (device unsigned, may
 *   be NULL).
 * bf_gc_gauss_planes: Hbar_n = G H_n for every plane (eq. 7, separable,
 *   taps normalised to sum 1), in place. tmp is device scratch of at least
 *   bf_gc_gauss_tmp_bytes(planes, height, width, stack_dtype) bytes, 16-byte
 *   aligned; it holds the column-filtered planes transposed between the two
 *   passes, and its contents afterwards are unspecified.
 * bf_gc_combine: y = t_c + t_h P/Q from the filtered planes (eqs. 8-10);
 *   P_out and Q_out (device FP32 height x width with row stride ld, may be
 *   NULL) receive the scaled P' = sum b_n s^n Hbar_{n+1} and
 *   Q' = sum b_n s^n Hbar_n, P = t_h S P', Q = S Q' with S the sum of the
 *   unnormalised 2-D spatial weights.
 * prm is a device buffer of bf_gc_param_bytes() bytes that the call fills and
 * the kernels read; it must stay untouched until the kernels have run.
 */
size_t bf_gc_param_bytes(double sigma_s, int N);
bf_status bf_gc_plane_scales(double sigma_r, int N, int stack_dtype, int *k_out);
bf_status bf_gc_stack_build(const float *f, int height, int width, int ld, double sigma_r, int N,
                            int stack_dtype, void *stack, long long plane_stride, int lds,
                            unsigned *devflag, void *prm, void *stream);
size_t bf_gc_gauss_tmp_bytes(int planes, int height, int width, int stack_dtype);
bf_status bf_gc_gauss_planes(void *stack, void *tmp, size_t tmp_bytes, int planes, int height, int width,
                             long long plane_stride, int lds, double sigma_s, int stack_dtype,
                             void *prm, void *stream);
bf_status bf_gc_combine(const float *f, const void *stack, int height, int width, int ld,
                        long long plane_stride, int lds, double sigma_r, int N, int stack_dtype,
                        float *out, float *P_out, float *Q_out, void *prm, void *stream);

/*
 * Batched forward: `count` images of uneven sizes, each with its own sigma_s,
 * sigma_r and N, in one graph after one copy of a small descriptor blob.
 * Three-kernel form (tile configurations 0-3, and the FP32 stack): three
 * persistent kernels (build, column pass, row pass + combine), each striding
 * over that phase's tiles of the whole batch. Fused form (BF_TILE_FUSED, the
 * default for FP16/BF16 stacks when every image's radius is at most
 * BF_FUSED_MAX_RADIUS; with the flag given, larger radii get
 * BF_ERR_UNSUPPORTED): one persistent kernel per geometry class present
 * (radius ranges with their own tile shape), striding over the class's tiles.
 * descs and per_image_status are host arrays, read and written before
 * return. Each image gets the status its own bf_gc_forward would return from
 * the host checks, with one exception: an image whose own expansion lies
 * outside the stack type's accuracy domain (sigma_r too small for it,
 * Section III-B: mu grows as 1/sigma_r^2; kappa times the rounding unit above
 * 1e-5 for FP32, where its 1e-3 max-abs error holds, and above the
 * conditioning check's 1e-2 for FP16/BF16) is routed to the pivoted form of
 * bf_gc_forward_pivots with the sub-range count bf_gc_batched_route returns
 * and the rule's degree per sub-range, and gets BF_OK (without
 * BF_FLAG_ALLOW_ILL_CONDITIONED, Chebyshev coefficients only; where no count
 * up to BF_MAX_PIVOTS reaches the domain, the image keeps its own expansion,
 * or BF_ERR_ILL_CONDITIONED if that fails the conditioning check). Images whose status is
 * not BF_OK are skipped (their out is untouched) and the call still returns
 * BF_OK. Tiles are the per-image kernels' blocks, so each output equals the
 * single-image forward's (a routed image: bf_gc_forward_pivots's) bit for
 * bit under the same tile configuration. On the fused tile a routed image
 * runs in a class of its own (one block per tile, each running the
 * sub-ranges present among its output pixels); in the three-kernel form each
 * of its sub-ranges runs as an image of its own that writes only its pixels
 * (at most 2 BF_MAX_BATCH such descriptors, BF_ERR_UNSUPPORTED beyond). BF_FLAG_GRAPH launches through a
 * hipGraph cached per (workspace, stream, capacity, tile configuration,
 * stack type) and replayed with the new descriptors. ws: device, 256-byte
 * aligned, at least bf_gc_batched_workspace_bytes(descs, count, stack_dtype)
 * bytes; its flag word (bf_gc_read_flags) collects BF_DEVFLAG_RANGE. Calls
 * that share a workspace must not overlap. count <= BF_MAX_BATCH
 * (BF_ERR_UNSUPPORTED otherwise). Within each phase the images are visited
 * in decreasing cost per tile, so the blocks' shares stay balanced.
 */
typedef struct {
    const float *f;            /* device, height x width, row stride ld */
    float *out;                /* device, same layout, must not overlap f */
    int height, width, ld;
    double sigma_s, sigma_r;
    int N;
} bf_image_desc;

/* Workspace for a batch: sizes every image with valid dimensions and
 * parameters (pointers are not read), whatever its conditioning (as its own
 * expansion and as routed to the pivoted form), for the three-kernel form
 * (which needs more than the fused form). */
size_t bf_gc_batched_workspace_bytes(const bf_image_desc *descs, int count, int stack_dtype);

/* How bf_gc_batched runs an image with these parameters under `flags`:
 * 1 = its own expansion of degree N; K >= 2 = the pivoted form with K
 * sub-ranges (the smallest power of two whose sub-ranges, at the rule's
 * degree each, lie in the stack type's accuracy domain); 0 = skipped
 * (invalid sigma_r, N or stack type, or no well-conditioned form). Host
 * only. */
int bf_gc_batched_route(double sigma_r, int N, int stack_dtype, unsigned flags);
bf_status bf_gc_batched(const bf_image_desc *descs, int count, int stack_dtype, unsigned flags,
                        int *per_image_status, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of bf_gc_forward on the fused tile (FP16 stacks with radius
 * ceil(3 sigma_s) <= BF_FUSED_F16_MAX_RADIUS, BF16 with radius <=
 * BF_FUSED_MAX_RADIUS; other stacks or radii: BF_ERR_UNSUPPORTED; staged,
 * recursive or three-kernel tile flags: BF_ERR_INVALID_ARG), with no
 * workspace argument. Its only scratch, the per-wave range words of the
 * launch (4 bytes per wave and tile: 32 bytes per 4096 output pixels, per
 * 2048 for BF16 above radius 32), lives in a
 * library-owned device array of BF_NOALLOC_SCRATCH_BYTES per GPU, held until
 * the process ends; an image that needs more gets BF_ERR_UNSUPPORTED. The call
 * allocates no device memory and calls no allocating routine; the array's
 * device address is looked up once per device on the first call there.
 * Every word the call reads back is written by the same launch, so nothing
 * needs clearing. Arguments, checks and output as bf_gc_forward; out equals
 * bf_gc_forward's bit for bit. range_flag: device unsigned or NULL; if given,
 * it receives BF_DEVFLAG_RANGE or 0 (a plain store, after the filter, on
 * `stream`). Calls that overlap on one GPU share its scratch and race (their
 * range flags may mix; outputs are unaffected); order them on one stream.
 */
#define BF_NOALLOC_SCRATCH_BYTES (4u << 20)
bf_status bf_gc_forward_noalloc(const float *f, float *out, int height, int width, int ld, double sigma_s,
                                double sigma_r, int N, int stack_dtype, unsigned flags, unsigned *range_flag,
                                void *stream);

/* Reads the range flags of the last call that used workspace ws
 * (bf_gc_forward, bf_gc_joint_forward, bf_gc_forward_pivots, bf_gc_backward
 * or bf_gc_batched): the flag word, or the or of the per-wave words a fused
 * launch wrote (the library remembers, per workspace address, which applies).
 * Waits for `stream` first. flags_out: host unsigned. */
bf_status bf_gc_read_flags(const void *ws, unsigned *flags_out, void *stream);

/*
 * Kernel timing for profiling. bf_profile_start() turns it on for every later
 * launch of this library (all streams): each kernel is bracketed by two HIP
 * events on the stream it runs on. bf_profile_stop() turns it off, waits for
 * the recorded events and sums the elapsed times per kernel name; read the
 * sums with bf_profile_count() and bf_profile_entry(i, ...), which copies the
 * name (NUL-terminated, at most name_len bytes), the launch count and the
 * total milliseconds. `stream` is unused (kept for symmetry).
 */
bf_status bf_profile_start(void);
bf_status bf_profile_stop(void *stream);
int bf_profile_count(void);
bf_status bf_profile_entry(int i, char *name, int name_len, long long *count, double *total_ms);

/* Text for a status code; the last error message of the calling thread. */
const char *bf_status_string(int status);
const char *bf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BFGC_H */
