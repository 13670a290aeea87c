/*
 * cmg.h — C ABI of the compact (linear-storage) multigrid library for AMD
 * MI355X (gfx950).
 *
 * The method is the one of "Multigrid with Linear Storage Complexity"
 * (Bauer, Kohl, McCormick, Tamstorf, arXiv 2511.19036): a full-multigrid
 * (FMG) solver whose solution, residual and correction are stored as
 * per-level "sections" (Sec. 2, eq. compact-to-standard) in block floating
 * point (Sec. 6.1.3) with regressive precision (Sec. 2.1, eq. regressive).
 *
 * Problem class: -div(kappa grad u) = f (kappa = 1: Poisson) on the unit
 * square/cube, zero Dirichlet boundary, finite differences on the node grid
 * with N = 2^L + 1 points per axis (h = 2^-L), rediscretised on every level.
 *
 * Conventions shared by every entry point
 *  - Node arrays (f, u, r, y, lambda, dJdu) are float64, N^dim values, C order
 *    with x fastest (index [z][y][x]); batched arrays are [batch][N^dim].
 *    Boundary entries of inputs are ignored; boundary entries of outputs are
 *    written as 0.
 *  - Cell arrays (kappa, grad_kappa) are float64, (2^L)^dim values, C order;
 *    cell c spans nodes c..c+1 on every axis.
 *  - Pointers named "device" must be device memory of the current HIP device;
 *    "host" pointers are ordinary host memory.  The caller owns every array it
 *    passes; the library never frees or retains them past the call (kappa is
 *    copied at setup).  The context owns all its internal buffers.
 *  - All GPU work is enqueued on the stream given to cmg_setup (or to the
 *    codec calls).  Calls return after enqueueing, except those that fill
 *    host memory (exports, stats with recording, memory stats), which
 *    synchronise the stream first.
 *  - Every call returns a cmg_status; cmg_last_error gives the message of the
 *    last failure on that context (or on the calling thread for ctx = NULL).
 *    After CMG_ERR_INVALID_ARG / CMG_ERR_UNSUPPORTED / CMG_ERR_NONFINITE the
 *    context stays usable; after CMG_ERR_HIP / CMG_ERR_OUT_OF_MEMORY only
 *    cmg_destroy is valid.  No C++ exception crosses this interface.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CMG_H
#define CMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmg_ctx_s* cmg_ctx;

typedef enum {
  CMG_OK = 0,
  CMG_ERR_INVALID_ARG = 1,   /* bad pointer, size, option or state           */
  CMG_ERR_UNSUPPORTED = 2,   /* valid in principle, not implemented           */
  CMG_ERR_OUT_OF_MEMORY = 3, /* device allocation failed                      */
  CMG_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed    */
  CMG_ERR_NONFINITE = 5,     /* NaN/Inf in an input (f, kappa, codec input)   */
  CMG_ERR_NOT_CONVERGED = 6  /* residual grew during iterative refinement:
                                an IR residual norm above 4 times the
                                smallest one of its FMG level (the solve
                                ran to its end; its output is unreliable) */
} cmg_status;

enum { CMG_POISSON = 0, CMG_DIFFUSION = 1 };          /* cmg_problem.op           */
enum { CMG_WJACOBI = 0, CMG_RBGS = 1 };               /* cmg_opts.smoother        */
enum { CMG_PLAIN_FP64 = 0, CMG_COMPACT_BFP = 1 };     /* cmg_opts.storage         */
enum { CMG_FP32 = 0, CMG_FP64 = 1 };                  /* cmg_opts.vcycle_prec     */
enum { CMG_SECTION_U = 0, CMG_SECTION_R = 1, CMG_SECTION_Y = 2, CMG_SECTION_YPRE = 3 }; /* section kind:
   solution u', residual g = r - s, correction y' after post-smoothing, y' after pre-smoothing */

typedef struct {
  int32_t dim;      /* 2 or 3                                                 */
  int32_t L;        /* finest level; N = 2^L + 1 nodes per axis, 2 <= L <= 10 */
  int32_t coarsest; /* coarsest level: 1 (one interior node) or 2 (3^dim
                       interior nodes, dense L D L^T solve), < L              */
  int32_t op;       /* CMG_POISSON or CMG_DIFFUSION                           */
  int32_t batch;    /* number of right-hand sides solved per call, >= 1      */
} cmg_problem;

/*
 * Solver options.  Alg. 3 (cFmg) with N = ir_iters IR iterations per FMG
 * level and nu = vcycles = 1 V-cycle per IR iteration (the paper fixes
 * nu = 1, Sec. 4); the V-cycle is Alg. 1 generalised to nu_pre/nu_post
 * sweeps of the smoother (eq. smoother).  Widths: section u' on level l at
 * FMG level Lp carries bits_u + inc_u (Lp - l) bits, residual and correction
 * bits_r/bits_y + inc_ry (Lp - l) bits (Table 1 with p + 1 = inc_u,
 * m = inc_ry), sign included (Table 2 caption); u' is capped at 53 bits,
 * r and y' at 24 bits with an FP32 V-cycle (53 with FP64).
 */
typedef struct {
  int32_t smoother;    /* CMG_WJACOBI or CMG_RBGS                              */
  double omega;        /* weighted-Jacobi weight (ignored by RB-GS)            */
  int32_t nu_pre;      /* pre-smoothing sweeps, >= 0                           */
  int32_t nu_post;     /* post-smoothing sweeps, >= 0                          */
  int32_t ir_iters;    /* N: IR iterations per FMG level, >= 1                 */
  int32_t vcycles;     /* nu: V-cycles per IR iteration, must be 1             */
  int32_t final_iters; /* extra IR iterations on the finest level, >= 0       */
  int32_t storage;     /* CMG_COMPACT_BFP, or CMG_PLAIN_FP64 (Alg. SM2)        */
  int32_t bfp_block;   /* BFP block length: 32 or 64                           */
  int32_t bits_u;      /* width of the finest solution section, 2..53          */
  int32_t bits_r;      /* width of the finest residual section, 2..24 (53)     */
  int32_t bits_y;      /* width of the finest correction section, 2..24 (53)   */
  int32_t inc_u;       /* regressive increment of u' (k = p + 1), >= 0        */
  int32_t inc_ry;      /* regressive increment of r, y' (k = m), >= 0         */
  int32_t vcycle_prec; /* CMG_FP32 or CMG_FP64 arithmetic inside the V-cycle   */
  int32_t keep_correction; /* 1: keep the pre- and post-smoothed corrections of
                              every level in sections of their own, for
                              inspection (CMG_SECTION_Y / _YPRE exports; one
                              more section of the correction's width).  0
                              (default): the post-smoothed correction is only
                              added to u' and not stored where the cycle does
                              not read it again, and those exports fail with
                              CMG_ERR_UNSUPPORTED.  Results are identical.   */
} cmg_opts;

/* Optional per-solve statistics (host struct). */
typedef struct {
  int32_t record;             /* in: 1 = record residual norms (synchronises)   */
  int32_t count;              /* out: residual norms written                    */
  double residual_norm[256];  /* out: FP64 2-norm of each IR residual f - A u   */
} cmg_stats;

/* Device memory held by a context, in bytes. */
typedef struct {
  int64_t sections;      /* BFP codes + exponents of u', r, y' on all levels  */
  int64_t coarse_fp64;   /* float64 temporaries of levels below the finest    */
  int64_t coarse_work;   /* V-cycle temporaries of levels below the finest    */
  int64_t fine_work;     /* temporaries on the finest level                   */
  int64_t kappa;         /* coefficient hierarchy (diffusion)                 */
  int64_t total;         /* everything the context allocated                  */
  int64_t interior_dofs; /* (2^L - 1)^dim                                      */
  double logical_bits_per_dof; /* mantissa + exponent bits of u', r, y' at the
                                  finest FMG level per interior DoF          */
} cmg_mem;

/* Fill *o with the defaults: RB-GS V(2,2), N = 2, nu = 1, compact BFP,
 * B = 64, b = 16 for u', r, y', increments 2 and 1, FP32 V-cycle,
 * keep_correction = 0. */
cmg_status cmg_default_opts(cmg_opts* o);

/*
 * Create a solver context for one problem shape.  Validates p and o, copies
 * kappa (device, (2^L)^dim float64 cells, must be > 0 and finite; NULL for
 * Poisson), builds the coefficient hierarchy (coarse cell = mean of its 2^d
 * children) and allocates every buffer with hipMalloc.  hip_stream is a
 * hipStream_t (NULL = default stream).  On success *out receives the context.
 */
cmg_status cmg_setup(const cmg_problem* p, const cmg_opts* o, const double* kappa_cells,
                     void* hip_stream, cmg_ctx* out);

/*
 * Compact FMG (Alg. 3, with Alg. 2 for the residual and the generalised
 * Alg. 1 for the V-cycle), or plain FP64 FMG (Alg. SM2) when storage is
 * CMG_PLAIN_FP64.  f: device [batch][N^dim]; u: device [batch][N^dim], the
 * decoded standard representation (eq. compact-to-standard).  st: host,
 * nullable.  Right-hand sides are injected to coarser FMG levels.
 */
cmg_status cmg_fmg_solve(cmg_ctx ctx, const double* f, double* u, cmg_stats* st);

/*
 * One compact V-cycle from a zero correction (generalised Alg. 1) on a
 * given fine residual: r (device, [batch][N^dim]) is rounded to the finest
 * residual width, the cycle runs on a zero solution, and y (device,
 * [batch][N^dim]) receives the decoded correction.  Overwrites the
 * context's sections.
 */
cmg_status cmg_vcycle(cmg_ctx ctx, const double* r, double* y);

/*
 * Adjoint solve and coefficient gradient for a loss J(u) (diffusion only).
 * Solves A lambda_b = dJdu_b for every batch item with the same FMG as
 * cmg_fmg_solve (A is symmetric), then forms
 *   dJ/dkappa_c = -h^-2 2^-(d-1) sum_b sum_{edges (p,q) of cell c}
 *                 (lambda_q - lambda_p)(u_q - u_p).
 * u: device forward solution [batch][N^dim]; dJdu: device [batch][N^dim];
 * lambda: device out [batch][N^dim]; grad_kappa: device out (2^L)^dim cells
 * (summed over the batch), nullable.
 */
cmg_status cmg_adjoint_solve(cmg_ctx ctx, const double* u, const double* dJdu, double* lambda,
                             double* grad_kappa);

/* Release the context and everything it allocated (synchronises). */
cmg_status cmg_destroy(cmg_ctx ctx);

/* Message of the last failure (never NULL; empty if none). */
const char* cmg_last_error(cmg_ctx ctx);

/* ---------------------------------------------------------------------------
 * Block floating point codec (Sec. 6.1.3 format; Sec. 4 rounding: round to
 * nearest, ties to even; the width includes the sign, Table 2 caption).
 * Blocks are `block` consecutive values (32 or 64), the last one zero-padded.
 * Block exponent e: frexp exponent of the block's largest magnitude, raised
 * by one if that magnitude rounds up to 2^(bits-1); value = m * 2^(e-bits+1);
 * all-zero blocks store e = -32768.  Codes are stored in a container of 8,
 * 12 (two values per three bytes, value t at bit 12t, little endian), 16, 32
 * or 64 bits (the smallest that holds `bits`), sign-extended.
 * ------------------------------------------------------------------------- */

/* Bytes of the code buffer for n values (padding to whole blocks included). */
int64_t cmg_bfp_code_bytes(int64_t n, int32_t block, int32_t bits);

/* Encode n values x (device, float64 if x_is_f64 else float32) into codes
 * (device, cmg_bfp_code_bytes) and exps (device, ceil(n/block) int16).
 * Returns CMG_ERR_NONFINITE (after synchronising) if x holds NaN/Inf. */
cmg_status cmg_bfp_encode(const void* x, int32_t x_is_f64, int64_t n, int32_t block, int32_t bits,
                          void* codes, int16_t* exps, void* hip_stream);

/* Decode n values into x (device float64); exact for bits <= 53. */
cmg_status cmg_bfp_decode(const void* codes, const int16_t* exps, int64_t n, int32_t block,
                          int32_t bits, double* x, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Adaptive-exponent BFP codec (Sec. 6.1.3, Exponents: the exponent need not
 * be known in advance).  Entries are visited in index order and normalised
 * to the largest exponent seen so far (the running exponent R_i); a block
 * starts wherever R_i rises, and only the last `bits` blocks (the `bits`
 * largest exponents) are kept: every other block's entries would round to
 * zero at the largest exponent.  An entry's exponent is the fixed-block
 * exponent of a block holding that entry alone (frexp exponent of |x|,
 * plus one if |x| rounds to 2^(bits-1)); code m_i = RNE(x_i 2^(bits-1-R_i)),
 * 0 before the first nonzero entry, in the containers of the fixed-block
 * codec; a kept block is an int64 start index and an int16 exponent.
 * Entries before the first kept block decode to 0.  One pass over x
 * (decoupled look-back scan over tiles of 4096 values).
 * ------------------------------------------------------------------------- */

/* Bytes of the code buffer for n values (ceil(n/64)*64 codes). */
int64_t cmg_abfp_code_bytes(int64_t n, int32_t bits);

/* Bytes of the device workspace an encode of n values needs. */
int64_t cmg_abfp_workspace_bytes(int64_t n);

/* Encode n values x (device, float64 if x_is_f64 else float32) into codes
 * (device, cmg_abfp_code_bytes, 16-byte aligned), starts (device, `bits`
 * int64) and exps (device, `bits` int16); *nblocks (device int32) receives
 * the number of kept blocks, or -1 if x held NaN/Inf, or -2 if the scan
 * failed.  workspace: device, cmg_abfp_workspace_bytes(n), owned by the
 * caller and not shared by overlapping calls.  Asynchronous on hip_stream
 * (read *nblocks after synchronising).  CMG_ERR_INVALID_ARG for a bad size,
 * width, NULL or misaligned buffer. */
cmg_status cmg_abfp_encode(const void* x, int32_t x_is_f64, int64_t n, int32_t bits, void* codes, int64_t* starts,
                           int16_t* exps, int32_t* nblocks, void* workspace, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * encode as cmg_abfp_encode, with the same outputs, but no workspace
 * argument: its workspace is one static device array per GPU (about 4 MiB,
 * held until the process ends) for n of at most 2^31 values; larger n fails
 * with CMG_ERR_INVALID_ARG.  Allocates nothing.  Calls that overlap on one
 * GPU (other streams or threads) share that array and race; calls in stream
 * order do not.  Asynchronous on hip_stream. */
cmg_status cmg_abfp_encode_noalloc(const void* x, int32_t x_is_f64, int64_t n, int32_t bits, void* codes,
                                   int64_t* starts, int16_t* exps, int32_t* nblocks, void* hip_stream);

/* Decode n values into x (device float64) from an encode's outputs (a
 * negative *nblocks decodes as no block: all zeros); exact for bits <= 53. */
cmg_status cmg_abfp_decode(const void* codes, const int64_t* starts, const int16_t* exps, const int32_t* nblocks,
                           int64_t n, int32_t bits, double* x, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Section inspection and stepwise driving (tests, checkpoint/resume).
 * Sections use the padded level layout: level l holds (2^l)^dim values, C
 * order; index 0 on each axis is the boundary node (always 0), the node at
 * 2^l is implicit.  `which` is CMG_SECTION_U / _R / _Y, or _YPRE: the
 * correction as the down sweep left it (the up sweep reads it and writes
 * its post-smoothed value to _Y).  _Y and _YPRE exist only in contexts set
 * up with keep_correction = 1 (else CMG_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------------- */

/* Shape of a stored section: values, current width, container bits, bytes of
 * the code buffer and number of blocks.  Any output pointer may be NULL. */
cmg_status cmg_section_info(cmg_ctx ctx, int32_t which, int32_t level, int64_t* n_values,
                            int32_t* bits, int32_t* container_bits, int64_t* code_bytes,
                            int64_t* n_blocks);

/* Copy a section to host memory (codes: code_bytes; exps: n_blocks). */
cmg_status cmg_export_section(cmg_ctx ctx, int32_t which, int32_t level, void* codes_host,
                              int16_t* exps_host);

/* Overwrite a section from host memory; `bits` sets its current width and
 * must fit the section's container. */
cmg_status cmg_import_section(cmg_ctx ctx, int32_t which, int32_t level, int32_t bits,
                              const void* codes_host, const int16_t* exps_host);

/* Enter FMG level `level` (Alg. 3): at the coarsest level, the exact coarse
 * solve of the injected f (device [N^dim]) into u'; above it, widen every
 * coarser u' section by inc_u bits and append a zero section. */
cmg_status cmg_fmg_enter_level(cmg_ctx ctx, int32_t level, const double* f);

/* IR residual at the current FMG level (Alg. 2): decode u', form f - A u in
 * float64, round it into the residual section of that level. */
cmg_status cmg_ir_residual(cmg_ctx ctx, const double* f);

/* One V-cycle from zero on the current residual section, followed by the
 * section-wise correction u' += y' (Alg. 1 generalised; Alg. 3). */
cmg_status cmg_vcycle_correct(cmg_ctx ctx);

/* The up sweep and correction of one level alone (Alg. 1 coarse to fine;
 * Alg. 3 apply correction), for inspection: with the coarse correction
 * e_{l-1} = y'_{l-1} + z_{l-1} given by the caller (e_coarse: device, the
 * padded layout of level - 1, float32 or float64 as the V-cycle type),
 * z = P e_{l-1}, y = S^nu_post(dec y'_l; g_l - A z) from the current
 * residual and pre-smoothed correction sections, y'_l = Q(y) (kept in the
 * _Y section with keep_correction = 1), u'_l = Q(dec u'_l + dec y'_l).
 * level: coarsest + 1 .. the current FMG level. */
cmg_status cmg_up_sweep(cmg_ctx ctx, int32_t level, const void* e_coarse);

/* Decode u' at the current FMG level Lp into u (device, (2^Lp + 1)^dim). */
cmg_status cmg_decode_solution(cmg_ctx ctx, double* u);

/* Device memory of the context by category. */
cmg_status cmg_memory_stats(cmg_ctx ctx, cmg_mem* out);

/* ---------------------------------------------------------------------------
 * Kernel timing for benchmarks.  While enabled, every kernel launch the
 * context makes (or only launches of the kernel named `kernel`, if not NULL)
 * is bracketed by two HIP events on the context stream, and its algorithmic
 * bytes (each operand read or written once) are recorded.  `kernel` may also
 * be "name@l" (that kernel's launches on level l only) or "@" (every kernel,
 * with separate totals per level, named "name@l", for the fused 3-D level
 * kernels).  Each API call
 * that launches kernels waits for its events before returning and adds the
 * durations to per-kernel totals.  Enabling (or disabling) clears the totals.
 * ------------------------------------------------------------------------- */
cmg_status cmg_timing_enable(cmg_ctx ctx, int32_t enable, const char* kernel);

/* Number of distinct kernels with recorded launches. */
cmg_status cmg_timing_count(cmg_ctx ctx, int32_t* count);

/* Totals of one kernel: name (NUL-terminated, truncated to name_len), launch
 * count, summed event time in milliseconds and summed algorithmic bytes. */
cmg_status cmg_timing_entry(cmg_ctx ctx, int32_t index, char* name, int32_t name_len, int64_t* launches,
                            double* total_ms, double* total_bytes);

#ifdef __cplusplus
}
#endif

#endif /* CMG_H */
