/*
 * mach.h - C ABI of the MACH hot path on AMD MI355X (gfx950).
 *
 * MACH (Tsourakakis, "MACH: Fast Randomized Tensor Decompositions") keeps
 * every tensor entry with probability p, rescales the kept ones by 1/p, and
 * runs HOSVD (Algorithm 1) or HOOI (Algorithm 2) on the sparsified tensor.
 * This library runs that path in hand-written HIP kernels:
 *   mach_sample      the coin toss over a dense device tensor (Alg. 1/2,
 *                    "MACH" block; Theorem 1; Remark 1) and the sparse
 *                    layouts every later step reads;
 *   mach_hosvd       factors A^(n) = leading left singular vectors of each
 *                    matricization of the sampled tensor (Alg. 1, HOSVD
 *                    loop; Alg. 2 initialisation);
 *   mach_hooi_sweep  one pass of Alg. 2's REPEAT body: for each mode n,
 *                    Y = Xhat x_{k != n} A^(k)T, then A^(n) = leading left
 *                    singular vectors of Y_(n);
 *   mach_core        G = Xhat x_1 A^(1)T ... x_d A^(d)T (eq. eqcore; the
 *                    last line of Alg. 1 and Alg. 2) and ||G||^2.
 *
 * Conventions
 *  - Tensors are dense, C order: the LAST mode varies fastest.  Linear
 *    index l = sum_k i_k * prod_{m > k} I_m, and N = prod I_k < 2^31.
 *  - Factor matrices A^(n) are I_n x R_n, row-major, float64, orthonormal
 *    columns, ordered by descending singular value; in every column the
 *    entry of largest magnitude is positive (lowest row on ties).
 *  - The core is R_1 x ... x R_d, C order, float64, and includes the 1/p
 *    rescale of the kept entries.
 *  - Device pointers are plain device addresses (e.g. a torch tensor's
 *    data_ptr()); `stream` is a hipStream_t passed as void* (NULL = the
 *    null stream).  Every call only enqueues work on `stream` (mach_hosvd
 *    also on an internal stream joined back into it) and returns; nothing
 *    synchronises except mach_read_status.
 *  - The library allocates nothing.  The caller owns every buffer, sized
 *    with the *_workspace_bytes queries; a workspace may be reused for any
 *    later call with the same shape, ranks and capacity.  Two calls that
 *    share a workspace must not run concurrently.
 *  - Errors the host can see (bad arguments, small workspace) return a
 *    negative status at once and enqueue nothing.  Errors found on the
 *    device (kept count above capacity, degenerate Gram, eigensolver not
 *    converged) set a status word in the workspace; later calls on that
 *    workspace skip their work, and mach_read_status reports it.
 */
#ifndef MACH_H
#define MACH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mach_status;
#define MACH_OK            0
#define MACH_EINVAL       -1  /* an argument is out of range                    */
#define MACH_ENOMEM       -2  /* workspace too small, or kept count > capacity  */
#define MACH_EDEVICE      -3  /* a HIP runtime call failed                      */
#define MACH_EUNSUPPORTED -4  /* valid input the library does not handle        */
#define MACH_EDEGENERATE  -5  /* a Gram matrix has rank below R_n               */
#define MACH_ENOCONV      -6  /* eigensolver residual tolerance not reached     */

typedef int32_t mach_dtype;
#define MACH_F64     0
#define MACH_F32     1
#define MACH_BF16    2
#define MACH_FP8E4M3 3

#define MACH_MAX_D 8

typedef struct {
  int32_t d;                   /* number of modes, 2..MACH_MAX_D          */
  int32_t pad_;
  int64_t dims[MACH_MAX_D];    /* I_1..I_d (C order: dims[d-1] fastest)    */
} mach_shape;

/* Bytes of the sample workspace for a tensor of shape `s` holding at most
 * `nnz_cap` kept entries.  Kept counts are Binomial(N, p): a capacity of
 * ceil(pN + 8 sqrt(N p (1-p))) + 256 is exceeded with negligible
 * probability (mach_nnz_capacity computes it).  Returns 0 if `s` is invalid. */
size_t mach_sample_workspace_bytes(const mach_shape* s, uint64_t nnz_cap);
uint64_t mach_nnz_capacity(const mach_shape* s, double p);

/* The coin toss (Alg. 1/2, MACH block; Theorem 1).
 * X_dev      device tensor of shape s, dtype x_dtype (MACH_F64 or MACH_F32),
 *            read only.
 * p          keep probability in (0, 1].  Entry l is kept iff the 32-bit
 *            word of Philox4x32-10 (Salmon et al., SC'11) at counter
 *            (l/4 lo, l/4 hi, window lo, window hi), key (seed lo, seed hi),
 *            output number l mod 4, is below T = min(2^32, floor(p 2^32)).
 *            Every entry gets a coin, zeros included.
 * ws         sample workspace (>= mach_sample_workspace_bytes bytes).  It
 *            receives the kept entries in linear-index order as
 *            (uint32 l, float32 x_l) pairs (x is NOT divided by p), the
 *            same entries regrouped for the other modes, sum x_l^2 in
 *            float64, and the kept count.
 * Returns MACH_OK or MACH_EINVAL / MACH_ENOMEM / MACH_EUNSUPPORTED /
 * MACH_EDEVICE.  On the device (read with mach_read_status): a kept count
 * above nnz_cap sets MACH_ENOMEM; else a kept value that is not finite sets
 * MACH_EINVAL; else a sample whose kept values are all zero (none kept, or
 * X zero there) sets MACH_EDEGENERATE, since every Gram is then zero.  The
 * layouts are still written; solver calls on such a sample do nothing. */
mach_status mach_sample(const mach_shape* s, mach_dtype x_dtype, const void* X_dev,
                        double p, uint64_t seed, uint64_t window_id,
                        void* ws, size_t ws_bytes, uint64_t nnz_cap, void* stream);

/* The coin toss for windows of a stream (Remark 2: a coin per measurement as
 * it arrives, so that windows which share measurements share their coins).
 * The last mode of s is time: X_dev holds ticks tick0 .. tick0 + I_d - 1 of
 * the series indexed by the other modes.  Entry (j, t), j the C-order flat
 * index of the other coordinates, is kept iff word (tau mod 4) of the
 * Philox4x32-10 block at counter (q lo, q hi, j, 0), q = tau / 4,
 * tau = tick0 + t, key (seed lo, seed hi), is below T (as for mach_sample).
 * The coin of a measurement thus depends on its series, its absolute tick
 * and the seed only: two windows of the same series layout that overlap in
 * time keep exactly the same measurements in the overlap.  Workspace,
 * outputs, errors and every later call are as for mach_sample;
 * tick0 + I_d must not exceed 2^64 (MACH_EINVAL). */
mach_status mach_sample_ticks(const mach_shape* s, mach_dtype x_dtype, const void* X_dev, double p,
                              uint64_t seed, uint64_t tick0, void* ws, size_t ws_bytes,
                              uint64_t nnz_cap, void* stream);

/* The tick-keyed toss of a window that slides along a stream (Remark 2: the
 * coin of a measurement is tossed once, when it arrives), reusing an
 * earlier window's sample.  ws_prev holds a completed mach_sample_ticks (or
 * mach_sample_ticks_slide) of a window of the same shape s, the same seed,
 * p and nnz_cap, at its own first tick tick0p (read on the device).  Every
 * measurement (j, tau) of the new window that lies in the earlier window
 * takes its coin and its kept value (float32 input) from ws_prev: no
 * Philox block and no read of X_dev for it; the others are tossed as in
 * mach_sample_ticks and their values read from X_dev.  For float64 input
 * only the coins are reused (the sum of squares needs the float64 values).
 * The result - mask, kept list, layouts, sum of squares, kept count - is
 * bit for bit that of mach_sample_ticks on the new window, provided X_dev
 * holds, in the overlap, the values the earlier window was sampled from.
 * If ws_prev is not a valid tick-keyed sample with the same seed, p and
 * capacity (its header is checked on the device), every measurement is
 * tossed afresh, with the same result.  ws_prev is read only and must not
 * be ws; arguments and errors otherwise as for mach_sample_ticks. */
mach_status mach_sample_ticks_slide(const mach_shape* s, mach_dtype x_dtype, const void* X_dev,
                                    double p, uint64_t seed, uint64_t tick0, const void* ws_prev,
                                    void* ws, size_t ws_bytes, uint64_t nnz_cap, void* stream);

/* Bytes of the solver workspace for shape s and ranks R_1..R_d (host array
 * of d int32).  prec is the precision mach_hooi_sweep will be called with
 * (MACH_F32, MACH_BF16 or MACH_FP8E4M3; the workspace serves all three).
 * Returns 0 if the arguments are invalid or prec is not supported.
 *
 * Tucker-n (Section 2.1: compressing n of the d modes): R_d = 0 leaves the
 * last mode uncompressed - its factor is the identity, HOSVD and HOOI do
 * not compute or update it (its A_dev entry may be NULL), and the core is
 * R_1 x ... x R_{d-1} x I_d.  Supported when the last mode is the layouts'
 * only tail mode (mach_layout_info gives h = d - 1, e.g. hosts x metrics x
 * time, sensors x types x time) and every other mode's Gram is on the row
 * side (I_n <= prod of the other modes' ranks, the uncompressed mode
 * counting with I_d); else 0.  The sweep then works on the dense sampled
 * tensor (4 N bytes of the workspace). */
size_t mach_solver_workspace_bytes(const mach_shape* s, const int32_t* ranks,
                                   mach_dtype prec, uint64_t nnz_cap);

/* MACH-HOSVD factors (Alg. 1, the HOSVD loop): for every mode n,
 * A^(n) = R_n leading left singular vectors of Xhat_(n), from the Gram
 * matrix of the sampled matricization on its smaller side and a float64
 * eigensolve.  The Gram of the layouts' single tail mode on its column side
 * with more than 2048 head rows is not formed: its eigensolve applies it as
 * two sparse products (Remark 4; the workspace then holds no such Gram).
 * ws_sample must hold a completed mach_sample of the same
 * shape.  A_dev is a host array of d device pointers, each I_n x R_n
 * float64 row-major, written.  nnz_cap is the capacity ws_sample was built
 * with (it fixes where the sparse arrays sit).  Requires
 * 1 <= R_n <= min(I_n, N / I_n, 16) and d <= 4, except for an uncompressed
 * last mode (R_d = 0, see mach_solver_workspace_bytes), whose A_dev entry
 * may be NULL and is not written.  Resets the solver
 * workspace first.  The last mode's HOSVD runs on an auxiliary HIP stream
 * (one per caller stream and device, created on the first call, default
 * priority, kept for the life of the process), forked from and joined into
 * `stream` by events: work enqueued on `stream` after the call still sees
 * every factor; the call remains asynchronous.  If the auxiliary stream
 * cannot be created, all modes run on `stream`. */
mach_status mach_hosvd(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                       const int32_t* ranks, double* const* A_dev, void* ws, size_t ws_bytes,
                       void* stream);

/* One HOOI sweep (Alg. 2, one pass of the REPEAT body) over modes
 * first_mode..d-1 in order, each update seen by the next.  For mode n:
 * Y = Xhat x_{k != n} A^(k)T (sparse tensor-times-matrix chain), the Gram
 * of Y_(n) on its smaller side on MFMA, its top R_n eigenvectors in
 * float64, and (for the column-side Gram) back-projection and float64
 * re-orthonormalisation.  prec selects the arithmetic of the first two:
 *   MACH_F32      factor entries and Gram inputs float32;
 *   MACH_BF16     factor entries of the sparse passes and the Gram's inputs
 *                 rounded to bfloat16 (nearest even);
 *   MACH_FP8E4M3  factor entries as for MACH_BF16, the Gram's inputs in OCP
 *                 float8 e4m3 (nearest even, saturating at 448), each
 *                 staged tile of rows x summation indices scaled by its
 *                 largest magnitude / 448;
 * products and sums in float32 (the Gram over runs of 32 summation
 * indices, then float64) in every case.  Other prec values return
 * MACH_EUNSUPPORTED.  A short column-side mode (I_n <= 128,
 * 16 <= K_n <= 64, R_n <= 8) forms no Gram: its factor comes from a block
 * subspace iteration on Y Y^T in float64.  The float64 eigensolve stops at
 * an accuracy matched to its input: with MACH_F32 at off-diagonal mass
 * 1e-16 of the diagonal (Jacobi) or Ritz residuals 1e-10 of the largest
 * Ritz value (block and subspace iterations), with the other two at 1e-12
 * and 1e-6, far below the rounding of their bfloat16 / e4m3 inputs.
 * A_dev (host array of d device pointers, I_n x R_n float64) is read and
 * the updated factors written back.  If fit_dev is not NULL, the device
 * double it points to receives 1 - ||Xhat - G x A|| / ||Xhat|| after the
 * last update (with ||Xhat - G x A||^2 = ||Xhat||^2 - ||G||^2).
 * nnz_cap as for mach_hosvd.  Requires 1 <= R_n <= min(I_n, prod_{k != n}
 * R_k, 16) and d <= 4; with an uncompressed last mode (R_d = 0) the sweep
 * updates modes first_mode..d-2 (first_mode <= d - 2) and the fit is taken
 * after mode d-1's update. */
mach_status mach_hooi_sweep(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                            const int32_t* ranks, double* const* A_dev, mach_dtype prec,
                            int32_t first_mode, void* ws, size_t ws_bytes, double* fit_dev,
                            void* stream);

/* The core G = Xhat x_1 A^(1)T ... x_d A^(d)T (eq. eqcore), float64, C
 * order R_1 x ... x R_d, written to G_dev; ||G||^2 to *core_norm2_dev if
 * not NULL.  Uses the factors in A_dev.  With an uncompressed last mode
 * (R_d = 0) the core is R_1 x ... x R_{d-1} x I_d (no product along it). */
mach_status mach_core(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                      const int32_t* ranks, double* const* A_dev, double* G_dev,
                      double* core_norm2_dev, void* ws, size_t ws_bytes, void* stream);

/* mach_core without a solver workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * mach_core minus the workspace; the core's scratch (status word, float32
 * factor copies, the partial product over the tail modes, the last mode's
 * Y) lives in a fixed 16 MiB device array of the library, one per GPU, held
 * until the process ends.  The scratch needed is
 *   256 + sum_k 64 I_k + 4 MT KH  (+ 4 I_d K_d when the last mode is one of
 *   two tail modes)
 * bytes, each term rounded up to 256, with MT the product of the tail
 * dimensions and KH the product of the head ranks (mach_layout_info gives
 * the split); above 16 MiB the call returns MACH_ENOMEM and enqueues
 * nothing.  The call allocates nothing (no hipMalloc or hipFree, no
 * allocating library routine) and clears what must start at zero with a
 * kernel, not a memset.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams, or threads) race and
 * must be serialised by the caller.  The first call on a device looks up
 * the array's device address (hipGetSymbolAddress) and may return
 * MACH_EDEVICE if that fails. */
mach_status mach_core_noalloc(const void* ws_sample, uint64_t nnz_cap, const mach_shape* s,
                              const int32_t* ranks, double* const* A_dev, double* G_dev,
                              double* core_norm2_dev, void* stream);

/* Clears the solver workspace's status word and eigen warm-start state.
 * A fresh solver workspace must be reset (mach_hosvd does it) before
 * mach_hooi_sweep or mach_core use it. */
mach_status mach_solver_reset(const mach_shape* s, const int32_t* ranks, void* ws,
                              size_t ws_bytes, void* stream);

/* The head/tail split of the sparse layouts for shape s: *h_out receives h
 * (entries are grouped as a matrix of head modes 0..h-1 by tail modes
 * h..d-1) and headperm_out[0..h-1] the order in which the head coordinates
 * of one tail column are sorted in the column-grouped copy (outermost
 * first). */
mach_status mach_layout_info(const mach_shape* s, int32_t* h_out, int32_t* headperm_out);

/* Byte offsets, inside a sample workspace of shape s and capacity nnz_cap,
 * of (in this order): the kept entries in linear-index order (nnz_cap
 * pairs of uint32 l, float32 x), the CSR row pointers (MH+1 uint32, MH =
 * prod of head dims), the column-grouped copy of the entries (nnz_cap
 * pairs), its column pointers (MT+1 uint32, MT = N / MH), the keep bitmap
 * (uint64 words, bit l of word l/64) and the word ranks (uint32 per word:
 * kept entries before the word).  Writes min(n, 6) values to offsets_out.
 * For tests and tools that inspect the layouts; returns MACH_EINVAL on a
 * bad shape. */
mach_status mach_sample_offsets(const mach_shape* s, uint64_t nnz_cap, uint64_t* offsets_out,
                                int32_t n);

/* Synchronises `stream`, then reads the device status words of the sample
 * workspace (and of the solver workspace if ws_solver is not NULL).
 * *status_out receives the first non-zero status (or MACH_OK), *nnz_out
 * the kept count (may exceed the capacity), *sumsq_out sum x_l^2 over kept
 * entries.  Any out pointer may be NULL. */
mach_status mach_read_status(const void* ws_sample, const void* ws_solver, void* stream,
                             int32_t* status_out, uint64_t* nnz_out, double* sumsq_out);

/* Kernel timing for measurement tools.  mach_timing_enable(n), n >= 1:
 * from now on one sparse tensor-times-matrix pass in every n of each kind
 * (the 1st, (n+1)-th, ...) is launched with a start/stop event pair that
 * brackets exactly its dispatch; the call also clears the record.  n = 0
 * turns timing off; n < 0 is MACH_EINVAL.  mach_timing_read waits for the
 * recorded events of one pass kind (which = 0: the pass over head rows, 1:
 * the pass over tail columns) and returns their summed duration in
 * milliseconds and their number.  Events are created once and reused (no
 * device memory), without a system-scope fence on record, so timing adds
 * no cache writeback between kernels; sampling 1 in n keeps the markers'
 * own cost out of the surrounding work.  Not thread safe. */
mach_status mach_timing_enable(int32_t every);
mach_status mach_timing_read(int32_t which, double* total_ms, int32_t* count);

/* Static description of a status code. */
const char* mach_status_string(mach_status st);

/* Host-only self test of the library's integer helpers (fast division,
 * workspace layouts, the Jacobi round-robin schedule).  Needs no GPU.
 * Returns 0 on success, else the number of the first failed check. */
int32_t mach_host_selftest(void);

#ifdef __cplusplus
}
#endif
#endif /* MACH_H */
