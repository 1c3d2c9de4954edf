/*
 * ozemu.h - FP64 matrix multiplication emulated on low-precision matrix
 * units of AMD Instinct MI355X (gfx950), residue-number-system style.
 *
 * Method (Mazumder, Calotoiu, Hoefler, "FP64 Is All You Want, INT8 Is All
 * You Need, FP4/6/8 Is All You Have"): rows of A and columns of B are scaled
 * by powers of two and truncated to integers A', B' (Sec. II-A, eq.
 * "convert"); A' and B' are reduced modulo pairwise-coprime moduli (Sec.
 * II-B); each modulus's product runs as an exact INT8 GEMM with INT32
 * accumulation (Sec. IV-C); the epilogue reduces each product modulo its
 * modulus (Sec. V-D); Reconstruct applies the CRT, rounds once and unscales
 * (Sec. V-A, V-D). The result is C = RN(A'B' * 2^-(s_i + t_j)) entry by
 * entry, one rounding, whenever the CRT window (eq. "ov-crtgen") and the
 * accumulator bound (eq. "ov-accgen") hold; the library checks both before
 * any launch.
 *
 * Conventions for every entry point:
 *  - Matrices are row-major FP64 with a leading dimension (elements between
 *    consecutive rows): A is m x k (lda >= k), B is k x n (ldb >= n), C is
 *    m x n (ldc >= n). Leading dimensions are ignored for empty operands.
 *  - Pointers named A, B, C, workspace, shifts, planes and residues are
 *    device pointers owned by the caller; the library never allocates device
 *    memory and never frees caller memory. Host arrays are marked "host".
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream). All
 *    launches are asynchronous on it; no entry point synchronizes.
 *  - Every entry point returns an ozemu_status; arguments are validated on
 *    the host before any launch, and on an error nothing is launched.
 *    ozemu_last_error() gives a message for the calling thread's last error.
 *  - m = 0 or n = 0 is a no-op; k = 0 writes zeros to C.
 */
#ifndef OZEMU_H
#define OZEMU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OZEMU_OK = 0,
    OZEMU_ERR_INVALID_ARG = -1,  /* bad pointer, size, leading dimension, mode */
    OZEMU_ERR_K_TOO_LARGE = -2,  /* k above the exactness caps of the plan     */
    OZEMU_ERR_UNSUPPORTED = -3,  /* format or option not built                  */
    OZEMU_ERR_WORKSPACE = -4,    /* workspace NULL or smaller than required     */
    OZEMU_ERR_HIP = -5           /* a HIP launch or runtime call failed         */
} ozemu_status;

/* Low-precision format of the residue GEMMs (Sec. III-A alphabets). */
typedef enum {
    OZEMU_INT8 = 0,  /* one INT8 GEMM per modulus, moduli <= 256 (Sec. IV-C)      */
    OZEMU_E4M3 = 1,  /* FP8 limb channels, FP32 accumulation (Sec. III-B, IV-A)  */
    OZEMU_E2M3 = 2,  /* FP6 limb channels, FP32 accumulation (Sec. III-B, IV-A)  */
    OZEMU_E2M1 = 3   /* FP4 limb channels, FP32 accumulation (Sec. III-B, IV-B)  */
} ozemu_format;

/* How many bits of each row of A / column of B are kept (Sec. II-A).
 *  F53:    53 bits, the paper's scaling (mu, nu of eq. "convert"); refused
 *          when 2 k (2^53 - 1)^2 >= P (eq. "ov-crt").
 *  WINDOW: the moduli count is the accuracy knob: with
 *          w = floor(log2((P - 1) / (2 k))), A keeps ceil(w / 2) bits and B
 *          floor(w / 2), so the CRT window holds for any data.
 *  BOUND:  bound-adaptive: one extra INT8 GEMM of 6-bit magnitude bounds
 *          |A| |B| entrywise and sets per-row / per-column bits so that
 *          sum_h |A'_ih| |B'_hj| <= (P - 1) / 2 for every entry. */
typedef enum {
    OZEMU_SCALE_F53 = 0,
    OZEMU_SCALE_WINDOW = 1,
    OZEMU_SCALE_BOUND = 2
} ozemu_scaling;

/* Row or column shift written for a row of A / column of B holding a NaN or
 * an infinity; every entry of C it touches is NaN. */
#define OZEMU_SHIFT_NONFINITE INT32_MIN

typedef struct ozemu_plan_s* ozemu_plan;

/* Create a plan: the `num_moduli` pairwise-coprime moduli in [2, 256] of
 * largest product (Sec. III-A configuration; 2 <= num_moduli <= 32), the
 * scaling mode, CRT constants and caps. Host memory only; the plan owns it
 * and ozemu_plan_destroy frees it. *out is set to NULL on failure. */
ozemu_status ozemu_plan_create(ozemu_plan* out, int format, int num_moduli, int scaling);

/* Same with an explicit modulus list (host array of `count` ints, pairwise
 * coprime, each in [2, 256]; any order; stored sorted descending). */
ozemu_status ozemu_plan_create_moduli(ozemu_plan* out, int format, int count,
                                      const int32_t* moduli, int scaling);

/* Plan over limb channels of a float alphabet (format OZEMU_E4M3,
 * OZEMU_E2M3 or OZEMU_E2M1), for ozemu_dgemm (the other entry points take
 * INT8 plans). E2M3 scales its values by 2^3 and, within radius 32, holds
 * the same 49 integers as E4M3 (Example "equivalence"), so both pick the
 * same channels at k_slab = 2^14; its GEMMs run on the FP6 matrix cores.
 * The accumulation slab is k_slab terms (a multiple of 128, at most 2^24):
 * every stored plane value lies within r = floor(sqrt(2^24 / k_slab)), so
 * each FP32 accumulator stays exact (eq. "ov-accgen"); a longer k runs in
 * slabs whose residues add modulo m (Sec. V-B). The pool holds, per
 * modulus, the one-limb form if the alphabet within r meets every class,
 * else the two-limb Toom form at points 0, 1, infinity (three GEMMs,
 * weights 1 - b, b, b^2 - b) at the least base b that does and meets the
 * reduce-then-combine bound (eq. "ov-comrtc"). From the pool, pairwise-
 * coprime channels: with gemms > 0 the largest modulus product within
 * that many GEMMs (the accuracy knob of mode WINDOW); with gemms = 0 the
 * least GEMM count whose product exceeds k_slab * 2^107 (the window of
 * eq. "ov-crt" at K = k_slab, as Table "moduli" counts). Ties between
 * products are decided on a 32-fraction-bit fixed-point log2 computed by
 * repeated squaring, the first candidate in a fixed order winning. */
ozemu_status ozemu_plan_create_fp(ozemu_plan* out, int format, int gemms, int64_t k_slab,
                                  int scaling);

/* Channels of a plan into host arrays of capacity `cap` (any may be NULL):
 * modulus, rank (GEMMs: 1 one-limb, 3 two-limb Toom) and base (0 for one
 * limb), by decreasing modulus; an INT8 plan reports its moduli at rank 1.
 * *count receives the number of channels. */
ozemu_status ozemu_plan_channels(ozemu_plan plan, int32_t* moduli, int32_t* ranks,
                                 int32_t* bases, int cap, int* count);

ozemu_status ozemu_plan_destroy(ozemu_plan plan);

/* Moduli of the plan, descending, into host array `out` of capacity `cap`;
 * *count receives the number of moduli. */
ozemu_status ozemu_plan_moduli(ozemu_plan plan, int32_t* out, int cap, int* count);

/* Kept bits (beta_A, beta_B) the plan uses at inner dimension k in modes F53
 * and WINDOW (BOUND decides them per row and column on the device). For
 * INT8 plans k may exceed the accumulation cap (ozemu_plan_k_max), up to the
 * reconstruction cap: such k runs in the blocked call. */
ozemu_status ozemu_plan_kept_bits(ozemu_plan plan, int64_t k, int* beta_a, int* beta_b);

/* Largest k the plan accepts: min(kappa_rec, kappa_acc) of eq. "caps"
 * (kappa_rec only limits F53; WINDOW and BOUND adapt their bits to k). */
ozemu_status ozemu_plan_k_max(ozemu_plan plan, int64_t* k_max);

/* Padded sizes of the residue planes. Plane l of A holds m_pad x k_pad int8
 * (rows i of A'), plane l of B n_pad x k_pad (columns j of B'), each plane
 * m_pad * k_pad (n_pad * k_pad) bytes, planes back to back. Inside a plane
 * the bytes are in GEMM block order: entry (row, h) is at byte
 *   ((row / 256) * (k_pad / 64) + h / 64) * 16384 + (row % 256) * 64
 *   + ((((h % 64) / 16) ^ (((row % 256) / 4) % 4)) * 16) + h % 16,
 * i.e. blocks of 256 rows x 64 K-bytes, each contiguous, with the four
 * 16-byte chunks of a row permuted by an XOR. Residues are [N][m_pad][n_pad]
 * uint8, row-major. m_pad and n_pad are multiples of 256, k_pad of 64. */
ozemu_status ozemu_plane_dims(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                              int64_t* m_pad, int64_t* n_pad, int64_t* k_pad);

/* Bytes of device workspace ozemu_dgemm needs for this shape. */
ozemu_status ozemu_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                  size_t* bytes);

/* C = A B, emulated (Sec. V-A: Scale, Reduce, GEMMs, Epilogue, Reconstruct).
 * `workspace` must hold ozemu_workspace_size bytes, 256-byte aligned. */
ozemu_status ozemu_dgemm(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                         const double* A, int64_t lda, const double* B, int64_t ldb,
                         double* C, int64_t ldc, void* workspace, size_t ws_bytes);

/* Blocked call (Sec. V-B, "Slabs"): C = A B with the inner dimension cut
 * into slabs of k_slab terms (the last may be shorter). Each slab's residue
 * GEMMs accumulate on their own, so only k_slab is held to the INT32
 * accumulation cap (ozemu_plan_k_max); k itself may exceed it, up to the
 * reconstruction cap of the modulus set (the kept bits are those of the
 * whole k, as in ozemu_dgemm). Each slab's residues are added into a running
 * residue mod m_l, so the result is bitwise that of the unblocked definition;
 * the planes of one slab exist at a time, so k may also be longer than
 * the planes of a whole call could hold. INT8 plans in modes F53 and W
 * (OZEMU_ERR_UNSUPPORTED otherwise); k_slab > cap: OZEMU_ERR_K_TOO_LARGE.
 * Pointers, strides, stream and workspace rules as for ozemu_dgemm, with
 * ozemu_blocked_workspace_size bytes of workspace. */
ozemu_status ozemu_blocked_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                          int64_t k_slab, size_t* bytes);
ozemu_status ozemu_dgemm_blocked(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                 int64_t k_slab, const double* A, int64_t lda, const double* B,
                                 int64_t ldb, double* C, int64_t ldc, void* workspace,
                                 size_t ws_bytes);

/* ---- The five phases as separate calls (Sec. V-A), for callers that keep
 * intermediates (autograd, verification). Shapes and strides as in
 * ozemu_plane_dims. ---- */

/* Scale (Sec. V-A phase 1): shift_a[i] = s_i (A' = trunc(A * 2^s_i) per row),
 * shift_b[j] = t_j per column; 0 for a zero row/column,
 * OZEMU_SHIFT_NONFINITE for one with a NaN or infinity. Mode BOUND runs its
 * bound GEMM here and needs `workspace` (ozemu_workspace_size bytes); the
 * other modes accept NULL. */
ozemu_status ozemu_scale(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                         const double* A, int64_t lda, const double* B, int64_t ldb,
                         int32_t* shift_a, int32_t* shift_b, void* workspace, size_t ws_bytes);

/* Reduce (phase 2): plane l of A gets, at entry (i, h), the balanced residue
 * of A'_ih modulo m_l in [-floor(m/2), ceil(m/2) - 1] as int8 (two's
 * complement); plane l of B gets B'_hj at entry (j, h) (a transpose). Layout
 * as in ozemu_plane_dims; padding entries are written as 0. */
ozemu_status ozemu_reduce(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                          const double* A, int64_t lda, const double* B, int64_t ldb,
                          const int32_t* shift_a, const int32_t* shift_b,
                          int8_t* planes_a, int8_t* planes_b);

/* GEMMs and epilogue (phases 3-4): residues[l][i][j] = (sum_h
 * A-plane_l(i, h) B-plane_l(j, h)) mod m_l in [0, m_l), exact INT32 sums. */
ozemu_status ozemu_residue_gemm(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                const int8_t* planes_a, const int8_t* planes_b,
                                uint8_t* residues);

/* Reconstruct (phase 5): C_ij = RN(X_ij * 2^-(s_i + t_j)), X_ij the
 * balanced CRT solution of residues[.][i][j], one rounding (ties to even,
 * subnormals and overflow included). */
ozemu_status ozemu_reconstruct(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                               const uint8_t* residues, const int32_t* shift_a,
                               const int32_t* shift_b, double* C, int64_t ldc);

/* ---- Training: a forward that keeps what its backward reuses. The paper
 * covers one product; the two gradient products of Y = X W are emulated
 * with the same scheme (Sec. II-A scaling, Sec. II-B residues, Sec. V-A
 * phases), reusing the forward's truncated operands X', W' as cached
 * residue planes. Modes F53 and WINDOW; BOUND returns UNSUPPORTED. ---- */

/* Y = X W (X m x k, W k x n, Y m x n, row-major with leading dimensions),
 * emulated as ozemu_dgemm except that the kept bits are those of
 * ozemu_plan_kept_bits at K* = max(m, n, k), the largest inner dimension
 * of the forward and of both backward products (so Y may carry fewer bits
 * than ozemu_dgemm gives when m or n exceeds k). Also writes the cache:
 *   shift_x[m]   row shifts s_i of X (as ozemu_scale's shift_a),
 *   shift_w[n]   column shifts t_j of W,
 *   planes_x     residue planes of X' (ozemu_reduce's planes_a layout,
 *                N x m_pad x k_pad bytes from ozemu_plane_dims(m, n, k)),
 *   planes_w     residue planes of W' (planes_b layout, N x n_pad x k_pad).
 * All device buffers owned by the caller. `workspace` holds
 * ozemu_workspace_size(m, n, k) bytes, 256-byte aligned. The caps of the
 * plan must hold at K* (OZEMU_ERR_K_TOO_LARGE otherwise). When m, n or k
 * is 0 the cache is not written (both gradients are then empty or zero). */
ozemu_status ozemu_dgemm_fwd_cache(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                                   const double* X, int64_t ldx, const double* W, int64_t ldw,
                                   double* Y, int64_t ldy, int32_t* shift_x, int32_t* shift_w,
                                   int8_t* planes_x, int8_t* planes_w, void* workspace,
                                   size_t ws_bytes);

/* Bytes of device workspace ozemu_dgemm_bwd needs for forward shape (m, n, k). */
ozemu_status ozemu_bwd_workspace_size(ozemu_plan plan, int64_t m, int64_t n, int64_t k,
                                      size_t* bytes);

/* Gradients of Y = X W from dY (m x n) and the cache of
 * ozemu_dgemm_fwd_cache with the same plan and (m, n, k):
 *   dX (m x k, lddx >= k) = dY W^T: dY is folded by the cached column
 *     shifts (entry (i, j) taken as dY_ij 2^-t_j, exactly), row-scaled to
 *     keep the bits the CRT window leaves at inner dimension n beside W's
 *     cached bits, truncated and reduced; the cached W' planes are
 *     transposed on the device and multiplied per modulus;
 *     dX_ih = RN((D W'^T)_ih 2^-s''_i), one rounding.
 *   dW (k x n, lddw >= n) = X^T dY: the same with the rows of dY folded by
 *     the cached row shifts s_i, column scaling, and X' transposed.
 * Either output may be NULL to skip it. A NaN or infinity in a row of dY
 * makes that row of dX NaN (a column of dY: that column of dW); a row of X
 * or column of W that held one in the forward makes all of dW (all of dX)
 * NaN. `workspace`: ozemu_bwd_workspace_size bytes, 256-byte aligned. */
ozemu_status ozemu_dgemm_bwd(ozemu_plan plan, void* stream, int64_t m, int64_t n, int64_t k,
                             const double* dY, int64_t lddy, const int32_t* shift_x,
                             const int32_t* shift_w, const int8_t* planes_x,
                             const int8_t* planes_w, double* dX, int64_t lddx, double* dW,
                             int64_t lddw, void* workspace, size_t ws_bytes);

/* ---- Grouped products: many independent C_p = A_p B_p of different shapes
 * and plans in one set of launches (the paper treats one product at a time).
 * Scale, Reduce and Reconstruct run over the work of all problems at once;
 * the residue GEMM is one persistent launch whose workgroups take
 * (problem, modulus, tile) items from a counter, longest K first. A group
 * fixes shapes, plans and operand pointers; running it issues one
 * host-to-device copy of the group's tables (from pinned host memory the
 * group owns) and kernels, so a run can be captured in a HIP graph. ---- */
typedef struct ozemu_group_s* ozemu_group;

/* Build a group of `count` (0..4096) problems. Host arrays of length count:
 * plans[p] (a plan per problem, repeats allowed, F53 or WINDOW; the group
 * copies what it needs, so plans may be destroyed afterwards), shapes
 * m/n/k, device pointers A/B/C with leading dimensions (row-major, as for
 * ozemu_dgemm; pointers of empty problems are ignored). Each problem is
 * validated as ozemu_dgemm validates it (the message names the problem).
 * Host memory only. */
ozemu_status ozemu_group_create(ozemu_group* out, int count, const ozemu_plan* plans,
                                const int64_t* m, const int64_t* n, const int64_t* k,
                                const double* const* A, const int64_t* lda,
                                const double* const* B, const int64_t* ldb, double* const* C,
                                const int64_t* ldc);

/* Bytes of device workspace ozemu_group_run needs (tables, then every
 * problem's shifts, planes and residues). */
ozemu_status ozemu_group_workspace_size(ozemu_group group, size_t* bytes);

/* C_p = A_p B_p for every problem (results as ozemu_dgemm with the
 * problem's plan). `workspace`: ozemu_group_workspace_size bytes, 256-byte
 * aligned. The first run of a group makes the pinned host copy of its
 * tables (hipHostMalloc), so run once before capturing a run in a graph.
 * Runs of one group or workspace on different streams race. */
ozemu_status ozemu_group_run(ozemu_group group, void* stream, void* workspace, size_t ws_bytes);

/* Free the group; work launched by ozemu_group_run must have completed. */
ozemu_status ozemu_group_destroy(ozemu_group group);

const char* ozemu_status_string(int status);
const char* ozemu_last_error(void);
const char* ozemu_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OZEMU_H */
