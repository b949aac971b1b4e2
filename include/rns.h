/*
 * rns.h -- C ABI of the MI355X (gfx950) exact multi-modular integer matrix
 * product and the Smith-form driver built on it.
 *
 * The method (Section 3.1 of Wang, Birmpilis, Labahn, Storjohann, "A C
 * implementation of the Smith massager algorithm"): an integer matrix is
 * reduced modulo L word-size primes, the L residue matrices are multiplied
 * independently modulo their prime, and the integer product is rebuilt by the
 * Chinese Remainder Theorem.  The Smith normal form (Section 1) is the
 * consumer: its lifting and massager steps reduce to such products.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are row-major.  A "plane stride" is the distance, in
 *   elements, between the residue matrices of consecutive primes.
 * - Residues are uint32 in the canonical range [0, p).
 * - Pointers named d_* or documented as device pointers are HIP device
 *   memory owned by the caller; the library never frees caller memory.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is enqueued asynchronously on it; the return code reports argument
 *   validation and launch errors only.  Device-side conditions (CRT overflow)
 *   are reported through a status word read after synchronisation.
 * - A primes range (prime_begin, L) selects the basis primes
 *   prime_begin .. prime_begin+L-1 of the context; plane j of every operand
 *   belongs to prime prime_begin+j.
 * - No call throws; every failure is a status code (rns_strerror names it).
 * - A context may be used by one host thread at a time.  Independent
 *   contexts may be used concurrently from different threads.
 */
#ifndef RNS_H
#define RNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    RNS_OK = 0,
    RNS_EINVAL = 1,     /* bad argument: null pointer, negative size, bad range */
    RNS_ENOMEM = 2,     /* device or host allocation failed */
    RNS_EDEVICE = 3,    /* a HIP call failed */
    RNS_EBOUND = 4,     /* an exactness bound of the chosen path is violated */
    RNS_EOVERFLOW = 5,  /* a reconstructed value does not fit the output words */
    RNS_ESINGULAR = 6,  /* the input matrix is singular */
    RNS_ERETRY = 7,     /* the Las Vegas restart budget was exhausted */
    RNS_ENOTSUP = 8,    /* the request is outside what this build implements */
    RNS_EPENDING = 9,   /* a served request has not finished within the wait */
    RNS_ESCRATCH = 10   /* larger than the fixed scratch of modmatmul_batched_noalloc */
};

/* Product paths of modmatmul_batched. */
enum {
    RNS_PATH_AUTO = 0,  /* the library chooses (autotuned per shape class) */
    RNS_PATH_FP64 = 1,  /* balanced residues in FP64 MFMA, reduced every 8 terms */
    RNS_PATH_INT8 = 2   /* 4 signed byte digits per residue, INT8 MFMA, int32 sums */
};

typedef struct rns_ctx rns_ctx;

/* Human-readable name of a status code.  Never NULL. */
const char *rns_strerror(int status);

/*
 * rns_primes_below -- the `count` largest primes strictly below `bound`,
 * descending (Section 3.1: primes are taken consecutively below a bound).
 * `out` is a host array of `count` entries.  bound <= 2^32.
 * Returns RNS_EINVAL if there are fewer than `count` primes below `bound`.
 */
int rns_primes_below(uint64_t bound, int count, uint32_t *out);

/*
 * rns_ctx_create -- a context on HIP device `device` holding an RNS basis and
 * the constants derived from it (Section 3.1, the bullet on precomputed RNS
 * constants): per prime p, its double and double reciprocal, 2^(8s) mod p for
 * the byte-digit recombination, the pairwise inverses of the Garner form of
 * the CRT, and the symmetric-range constants.
 *   primes: host array of L distinct odd primes, each < 2^26; NULL selects the
 *           L largest primes below 2^26.
 *   L:      1 <= L <= 4096.
 *   flags:  0, or RNS_CTX_PATH_FP64 / RNS_CTX_PATH_INT8: the path that
 *           RNS_PATH_AUTO resolves to in every product of this context (and
 *           of the Smith-form driver working on it), optionally or'ed with
 *           RNS_CTX_SEPARATE_CRT: whole-product plans of this context keep
 *           the CRT as a launch of its own even where they could fuse it
 *           into the GEMM launch (see rns_matmul_plan_create); other bits
 *           are reserved and rejected with RNS_EINVAL.
 * The context owns its device tables and a growable workspace; free it with
 * rns_ctx_destroy.  Returns RNS_EINVAL for a bad basis, RNS_EDEVICE or
 * RNS_ENOMEM on HIP failures.
 */
/* rns_ctx_create flags (low two bits: the default product path). */
#define RNS_CTX_PATH_FP64 1u
#define RNS_CTX_PATH_INT8 2u
#define RNS_CTX_SEPARATE_CRT 4u

int rns_ctx_create(rns_ctx **out, int device, const uint32_t *primes, int L,
                   uint64_t flags);
void rns_ctx_destroy(rns_ctx *ctx);

/* Number of primes and the primes themselves (host array of L entries). */
int rns_ctx_num_primes(const rns_ctx *ctx);
int rns_ctx_primes(const rns_ctx *ctx, uint32_t *out);

/*
 * rns_ctx_reserve -- grow the context's device workspace to at least `bytes`
 * now, so that later calls of that size allocate nothing.  modmatmul_batched
 * grows the workspace by itself when needed (a synchronous allocation).
 */
int rns_ctx_reserve(rns_ctx *ctx, size_t bytes);

/*
 * rns_primes_for_bound -- smallest L such that the product of the first L
 * basis primes is at least 2*B + 1, where B is the non-negative integer given
 * by `W` little-endian 64-bit words.  Every integer of absolute value at most
 * B is then determined by its residues modulo those primes.
 * Returns RNS_EBOUND if the whole basis is too short.
 */
int rns_primes_for_bound(const rns_ctx *ctx, const uint64_t *bound_words,
                         int W, int *L_out);

/*
 * rns_reduce -- Section 3.1, reduction of an integer matrix modulo each prime:
 *   res[j*plane_stride + i*ldr + c] = x[i*ldx + c] mod p_{prime_begin+j},
 * floor semantics (the result is in [0, p) also for negative x).
 *   x:   device int64, rows x cols, leading dimension ldx >= cols.
 *   res: device uint32, L planes, leading dimension ldr >= cols,
 *        plane_stride >= rows*ldr (planes must not overlap).
 * rows == 0 or cols == 0 is a no-op.
 */
int rns_reduce(rns_ctx *ctx, const int64_t *x, int64_t rows, int64_t cols,
               int64_t ldx, int prime_begin, int L, uint32_t *res,
               int64_t ldr, int64_t plane_stride, void *stream);

/*
 * rns_reduce_mw -- the same reduction (Section 3.1) for multiword integers:
 * entry (i, c) is the W-word two's-complement integer whose 64-bit words,
 * least significant first, are x[(i*ldx + c)*W + w], w = 0 .. W-1 (the
 * layout crt_reconstruct writes), so crt_reconstruct(rns_reduce_mw(x)) = x
 * whenever |x| < M/2 for the product M of the primes.
 *   x:   device uint64, 1 <= W <= 32, ldx >= cols (in entries).
 *   res: as for rns_reduce.
 * Computed on the INT8 matrix cores: the 8W+1 signed base-256 digits of x
 * times a table of the digits of 2^(8k) mod p_j (one int32 column sum per
 * digit of each 2^(8k) mod p_j), then sum_b T_b 2^(8b) mod p_j exactly in
 * doubles.
 */
int rns_reduce_mw(rns_ctx *ctx, const uint64_t *x, int W, int64_t rows, int64_t cols,
                  int64_t ldx, int prime_begin, int L, uint32_t *res,
                  int64_t ldr, int64_t plane_stride, void *stream);

/*
 * One residue product problem of modmatmul_batched:
 *   for j in [0, L):  C_j = A_j * B_j mod p_{prime_begin+j}
 * with A_j = A + j*a_plane_stride (m x k, leading dimension lda),
 *      B_j = B + j*b_plane_stride (k x n, leading dimension ldb),
 *      C_j = C + j*c_plane_stride (m x n, leading dimension ldc).
 * A and B hold residues in [0, p); C receives residues in [0, p).
 * All three are device pointers.
 */
typedef struct rns_gemm_desc {
    int64_t m, n, k;
    const uint32_t *A;
    int64_t lda, a_plane_stride;
    const uint32_t *B;
    int64_t ldb, b_plane_stride;
    uint32_t *C;
    int64_t ldc, c_plane_stride;
    int32_t prime_begin;
    int32_t L;
    int32_t flags;         /* 0, or RNS_GEMM_SUBTRACT */
    int32_t reserved;      /* 0 */
} rns_gemm_desc;

/* rns_gemm_desc.flags: C := (C - A B) mod p instead of C := A B mod p (C must
 * then hold residues in [0, p) on entry). */
#define RNS_GEMM_SUBTRACT 1

/* Workspace bytes modmatmul_batched needs for these problems on this path. */
int rns_workspace_bytes(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                        int path, size_t *bytes);

/*
 * modmatmul_batched -- Section 3.1, one independent product per prime, for
 * `count` problems of any sizes, all primes of all problems in one pass.
 *   descs: host array of `count` descriptors (read during the call only).
 *   path:  RNS_PATH_FP64, RNS_PATH_INT8 or RNS_PATH_AUTO.
 * Exactness: the FP64 path keeps every partial sum an integer below 2^53 by
 * reducing every 8 terms, for any k.  The INT8 path keeps every int32 digit
 * sum exact for k <= 43690 and returns RNS_EBOUND beyond.
 * The result is bit-exact and does not depend on the path, the tiling, the
 * launch order or the number of problems in the batch.  count == 0 is a
 * no-op.  Input residues outside [0, p) give unspecified (but in-range)
 * outputs.
 */
int modmatmul_batched(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                      int path, void *stream);

/*
 * modmatmul_batched_noalloc -- modmatmul_batched for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and exactness
 * bounds; it calls no hipMalloc, hipFree or other device allocation.  Its
 * scratch (the tiled digit or balanced operands, the problem table and the
 * work counter) is a fixed array of rns_noalloc_scratch_bytes() bytes (64 MiB)
 * per device, set up once per device by rns_ctx_create and held by the
 * process until it ends; problems whose tiled operands and table do not fit
 * return RNS_ESCRATCH and touch nothing.  The problem table is copied from
 * host memory and the stream is synchronised once after that copy; the
 * kernels then run asynchronously on `stream`.  Every call on one device
 * shares the array: calls that overlap on one device (other streams, other
 * threads, other contexts) race and give unspecified results; the array
 * keeps the last call's contents.  With kernel tracing (rns_ctx_profile) on,
 * each traced launch creates two HIP events.
 */
int modmatmul_batched_noalloc(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                              int path, void *stream);
/* Size in bytes of that fixed per-device scratch. */
int rns_noalloc_scratch_bytes(size_t *bytes);

/* ------------------------------------------------------------------------
 * Plans: the same products as modmatmul_batched, set up once and run many
 * times.  Creation validates the problems, sorts them by decreasing tile cost,
 * allocates a plan-owned workspace and uploads the problem table; execution
 * only enqueues kernels (one operand-conversion launch and one GEMM launch for
 * the whole batch), so it may be captured into a HIP graph.  The operand and
 * result pointers are fixed at creation: an executed plan reads A and B and
 * writes C as they are at execution time.
 * ---------------------------------------------------------------------- */
typedef struct rns_gemm_plan rns_gemm_plan;

typedef struct rns_plan_info {
    int path;              /* RNS_PATH_FP64 or RNS_PATH_INT8 */
    int variant;           /* INT8 GEMM kernel (all compute the same 64 x 128
                              output tiles):
                              0 LDS-staged, four waves of 32 x 64 outputs;
                              1 operands straight from L2, four waves;
                              2 as 4, persistent: two work-groups per CU take
                                half-tiles, longest first, from a counter;
                              3 LDS-staged, eight waves of 32 x 32 outputs;
                              4 (default) two independent four-wave
                                work-groups per tile, one per 64-column half,
                                two work-groups per CU;
                              RNS_I8_HALF_CRT (5): whole-product plans that
                                fuse the CRT: as 4, each work-group taking
                                both primes of its half-tile and writing
                                int64 (not selectable by set_variant) */
    int64_t tiles;         /* work-group tiles over all primes and problems */
    size_t workspace_bytes;
    double residue_ops;    /* 2*m*n*k*L summed over the problems */
} rns_plan_info;

int rns_gemm_plan_create(rns_ctx *ctx, const rns_gemm_desc *descs, int count,
                         int path, rns_gemm_plan **out);
int rns_gemm_plan_execute(rns_gemm_plan *plan, void *stream);
int rns_gemm_plan_info(const rns_gemm_plan *plan, rns_plan_info *info);
int rns_gemm_plan_set_variant(rns_gemm_plan *plan, int variant);
void rns_gemm_plan_destroy(rns_gemm_plan *plan);

/*
 * Autotuner.  rns_autotune times every INT8 GEMM variant on these problems
 * (it runs them: C is overwritten), records the fastest for the batch's shape
 * class (path, number of problems, largest dimension and total work, on log2
 * scales) in the context, and appends it to the cache file if one is set.
 * Plans and modmatmul_batched created afterwards use the recorded variant.
 * rns_ctx_set_tune_cache loads an existing cache file ("key variant" lines).
 */
int rns_ctx_set_tune_cache(rns_ctx *ctx, const char *path);
int rns_autotune(rns_ctx *ctx, const rns_gemm_desc *descs, int count, int path,
                 void *stream, int *variant_out);
/* The same for an existing plan (which then keeps the chosen variant). */
int rns_gemm_plan_autotune(rns_gemm_plan *plan, void *stream, int *variant_out);

/*
 * Whole-product plans (Section 3.1 end to end): C = A B over the integers for
 * `count` independent problems.  One execution runs three launches: one
 * conversion launch that reduces every A and B modulo each of its primes
 * straight into the GEMM's tiled operand layouts (no residue planes of A and
 * B are written), one GEMM launch over all primes and problems, and one CRT
 * launch over all C.  The plan owns the tiled operands and the residue planes
 * of every C; they stay resident in HBM between executions.
 *   A, B: device int64, row-major (m x k, k x n), leading dimensions lda, ldb.
 *   C:    device uint64, W words per entry (entry (i, j) at
 *         C[(i*ldc + j)*W + w]), two's complement; W == 1 is an int64 matrix.
 *   bound: a promise |C_ij| <= bound for every entry (0 = no promise).  When
 *         every problem has a promise with margin the Lagrange CRT form is used,
 *         otherwise the exact mixed-radix form.
 *   prime_begin, L: the primes of the problem, 1 <= L <= 64.
 * Overflow of W words is reported through the context status word.
 * When W == 1, every problem has L <= 2 and the INT8 path is taken (and the
 * context lacks RNS_CTX_SEPARATE_CRT), the plan fuses the CRT into the GEMM:
 * each work-group computes its output tile for both primes, keeps the first
 * prime's products in registers and writes the CRT of the pair (the unique
 * x with |x| <= (p0 p1 - 1)/2, exact whatever `bound` says; it always fits
 * one word) straight into C.  Execution is then two launches and the plan
 * holds no residue planes of C; rns_matmul_plan_info reports variant
 * RNS_I8_HALF_CRT.
 */
/* rns_plan_info.variant of a whole-product plan that fuses the CRT. */
#define RNS_I8_HALF_CRT 5

typedef struct rns_matmul_desc {
    int64_t m, n, k;
    const int64_t *A;
    int64_t lda;
    const int64_t *B;
    int64_t ldb;
    uint64_t *C;
    int64_t ldc;
    int32_t prime_begin;
    int32_t L;
    uint64_t bound;
} rns_matmul_desc;

typedef struct rns_matmul_plan rns_matmul_plan;

int rns_matmul_plan_create(rns_ctx *ctx, const rns_matmul_desc *descs, int count,
                           int path, int W, rns_matmul_plan **out);
int rns_matmul_plan_execute(rns_matmul_plan *plan, void *stream);
int rns_matmul_plan_info(const rns_matmul_plan *plan, rns_plan_info *info);
rns_gemm_plan *rns_matmul_plan_gemm(rns_matmul_plan *plan);
void rns_matmul_plan_destroy(rns_matmul_plan *plan);

/*
 * crt_reconstruct -- Section 3.1, Chinese-remainder reconstruction of every
 * entry of an L-plane residue matrix: the unique integer x with
 * |x| <= (M-1)/2, M = p_{prime_begin} ... p_{prime_begin+L-1}, and
 * x = res_j (mod p_{prime_begin+j}) for all j.
 *   res:  device uint32, L planes (rows x cols, leading dimension ldr,
 *         plane_stride apart), residues in [0, p).
 *   out:  device uint64; entry (i, c) occupies the W words
 *         out[(i*ldo + c)*W + 0 .. W-1], little-endian two's complement
 *         (W == 1 is a plain int64 matrix with leading dimension ldo).
 *   bound_words / Wb: optional promise |x| <= B (Wb little-endian words; NULL
 *         for none).  A promise that leaves a margin selects the Lagrange form
 *         with a floating-point correction (Section 3.1, the bullet on fast
 *         base conversion), one thread per entry; otherwise the exact form
 *         runs on the INT8 matrix cores: S = sum_j y_j (M/p_j) from the digits
 *         of y_j = r_j (M/p_j)^-1 mod p_j times a table of the digits of M/p_j,
 *         then x = S - a M with a = round(sum_j y_j / p_j), where a double
 *         value of that sum within 2^-40 of a half-integer is settled by an
 *         exact comparison with (M-1)/2.  (RNS_CRT_GARNER=1 in the environment
 *         at context creation selects the mixed-radix form instead.)  A false
 *         promise gives unspecified outputs.
 *   d_status: optional device int32; the kernel ORs 1 into it when some x
 *         does not fit in W words (that entry holds x mod 2^(64W)).  NULL
 *         uses the context's status word, read by rns_ctx_status.
 * Limits: 1 <= L <= 64 primes, 1 <= W <= 32 words.
 */
int crt_reconstruct(rns_ctx *ctx, const uint32_t *res, int64_t rows,
                    int64_t cols, int64_t ldr, int64_t plane_stride,
                    int prime_begin, int L, const uint64_t *bound_words,
                    int Wb, uint64_t *out, int W, int64_t ldo,
                    int32_t *d_status, void *stream);

/*
 * rns_base_convert -- Section 3.1, the bullet on fast RNS base conversion:
 * residues of x in the primes range (begin, L) to residues of the same x in
 * the range (begin_out, L_out), where x is the symmetric representative,
 * |x| <= (M-1)/2 for M = p_begin ... p_(begin+L-1):
 *     x mod q_i = sum_j y_j (M/p_j mod q_i) - a (M mod q_i),
 *     y_j = r_j (M/p_j)^-1 mod p_j,  a = round(sum_j y_j / p_j),
 * on the INT8 matrix cores (the digits of the y_j times a constant table).
 *   res:  device uint32, L planes (rows x cols, leading dimension ldr,
 *         plane_stride apart), residues in [0, p).
 *   out:  device uint32, L_out planes (leading dimension ldo,
 *         out_plane_stride apart), residues in [0, q).
 *   bound_words / Wb: optional promise |x| <= B.  A promise that leaves the
 *         margin of the Lagrange CRT (2B/M <= 1 - 2^-39) makes the
 *         floating-point correction exact and the conversion one pass that
 *         never forms x; without one x is rebuilt exactly (crt_reconstruct's
 *         exact form, into the context workspace, which may grow) and then
 *         reduced (rns_reduce_mw's kernel).  A false promise gives unspecified
 *         outputs.
 *   d_status: as for crt_reconstruct (unused on the one-pass form).
 * Limits: 1 <= L <= 64, 1 <= L_out.  The ranges may overlap.
 */
int rns_base_convert(rns_ctx *ctx, const uint32_t *res, int64_t rows, int64_t cols, int64_t ldr,
                     int64_t plane_stride, int begin, int L, const uint64_t *bound_words, int Wb,
                     uint32_t *out, int64_t ldo, int64_t out_plane_stride, int begin_out, int L_out,
                     int32_t *d_status, void *stream);

/*
 * rns_ctx_status -- synchronise `stream`, then read and clear the context's
 * device status word.  Returns RNS_EOVERFLOW if a CRT call that used it
 * overflowed since the last read, RNS_OK otherwise.
 */
int rns_ctx_status(rns_ctx *ctx, void *stream);

/* ------------------------------------------------------------------------
 * Smith normal form driver (Section 2.2, the three-phase Las Vegas method,
 * in a reduced form that calls the RNS primitives above for every product).
 * ---------------------------------------------------------------------- */

typedef struct rns_smith_result rns_smith_result;

typedef struct rns_smith_stats {
    double t_lif;          /* seconds: largest invariant factor (Phase 1) */
    double t_im;           /* seconds: projection and modular Smith form (Phase 2) */
    double t_uc;           /* seconds: certification (Phase 3) */
    double t_total;        /* seconds: whole call */
    int restarts;          /* Las Vegas restarts taken */
    int lift_steps;        /* path 0: primes for which A^-1 mod q was
                              computed; path 1: p-adic lifting steps */
    int64_t products;      /* modmatmul_batched calls issued */
    double residue_ops;    /* 2*m*n*k*L summed over all products */
    int cert_primes;       /* path 0: primes of the exact check A X = s I;
                              path 1: primes of det A / s */
    int columns;           /* columns of the projection J (n: J = I; massager:
                              summed over the batches) */
    int path;              /* 0: residues of s A^-1 (J = I); 1: p-adic lifting;
                              2: Smith massager (rns_smith_massager) */
    int cert_exact;        /* 1: the result is certified (path 0: A X = s I
                              exactly; path 1: |det A| = prod s_i with det A / s
                              reconstructed from enough primes to be exact);
                              0: not certified (rns_largest_invariant) */
    int lift_a_bytes;      /* path 1: 2 when A was stored as int16 for the
                              lifting kernels, 4 for int32; 0 on path 0 */
    int lift_kernels;      /* path 1: the lifting kernels of the last
                              lifting, as rns_lift_step's `kernels` bits */
    double t_host_cpu;     /* CPU seconds of the calling thread and of the
                              helper threads it started for this call */
    int batches;           /* path 2: index-massager batches of Phase 2 */
    int cert_kind;         /* 0: |det A| = prod s_i (determinant modulo
                              primes); 1 (path 2): the massaged matrix B of
                              Eq. (1) certified unimodular by high-order
                              residues (rns_unimodular_certify's method) */
    int uc_steps;          /* cert_kind 1: double-plus-one steps of the last
                              certificate */
    int uc_rejects;        /* cert_kind 1: massagers the certificate rejected
                              (each followed by a restart) */
    int64_t uc_dim;        /* cert_kind 1: dimension of the linearized B */
    double t_uc_cert;      /* cert_kind 1: seconds of the certificate proper
                              (inverse mod X and the steps); the rest of t_uc
                              builds the reduced massager and linearized B */
    int uc_x_primes;       /* cert_kind 1: primes in the lifting modulus X */
    int uc_lambda;         /* cert_kind 1: linearization base 2^uc_lambda */
} rns_smith_stats;

/*
 * rns_ctx_set_smith_path -- which Smith-form path smith_form takes:
 * 0 (default) chooses, 1 residue reconstruction of s A^-1 only, 2 p-adic
 * lifting only (RNS_ENOTSUP from smith_form where that path does not apply).
 */
int rns_ctx_set_smith_path(rns_ctx *ctx, int path);

/*
 * smith_form -- the Smith normal form S = diag(s_1, ..., s_n),
 * s_1 | s_2 | ... | s_n, s_i > 0, of a nonsingular n x n integer matrix
 * (Section 1), by the phases of Section 2.2 in reduced form: the largest
 * invariant factor s from rational reconstruction of A^-1 b; X = s A^-1 from
 * residues (A^-1 mod q by GPU Gauss-Jordan, products by modmatmul_batched,
 * combination by crt_reconstruct), certified by an exact check A X = s I on
 * fresh primes; the Smith form of X over Z/sZ gives s_i.  This path (0)
 * uses at most 64 primes per CRT, so |s A^-1| and the numerators and
 * denominators of A^-1 b must stay below about 2^1600.
 * Larger invariants take the p-adic lifting path (1) when n >= 16 and
 * n max|a_ij| < 2^36: one inverse C = A^-1 mod p stays resident and
 * Y = A^-1 J for a random n x t matrix J is lifted p-adically on the GPU; the
 * common denominator of random projections of Y gives s; the Smith form over
 * Z/sZ of s R Y (R random t+2 x n) gives the t largest invariants (t doubles
 * up to 16 while fewer than two of them are 1); the certificate checks
 * prod s_i = |det A| with det A / s rebuilt from det A mod primes, enough of
 * them (the product above 2 H / s + 1 for Hadamard's bound H) for the check to
 * be exact.  RNS_ENOTSUP when neither path applies;
 * entries must not be INT64_MIN.
 *   A_host: host int64, n x n row-major (copied during the call).
 *   seed:   drives the random choices only; S does not depend on it.
 *   out:    receives a library-allocated result; free with rns_smith_free.
 * Returns RNS_ESINGULAR when det A = 0, RNS_ERETRY when the restart budget is
 * exhausted.  Uses the context's stream-less default stream internally and
 * synchronises before returning.
 */
int smith_form(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
               rns_smith_result **out);

/*
 * rns_largest_invariant -- Phase 1 alone (Section 2.2): the largest
 * invariant factor s_n of a nonsingular A by p-adic lifting of A^-1 J for a
 * random n x 4 matrix J and rational reconstruction of random combinations of
 * the solution (the path-1 machinery of smith_form).  Monte Carlo: the value
 * returned divides s_n and equals it with high probability.  Requires n >= 16
 * and n max|a_ij| < 2^36 (RNS_ENOTSUP otherwise).  The result holds one
 * entry (read it with rns_smith_get(r, 0, ...)); free with rns_smith_free.
 */
int rns_largest_invariant(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
                          rns_smith_result **out);

/*
 * rns_smith_massager -- the Smith form S of a nonsingular A together with a
 * Smith massager (U, M, T, S) (Section 2.1, Eq. (1)): n x n integer matrices
 * with T unit upper triangular such that
 *     B = [A, A M S^-1; U, (T + U M) S^-1]
 * is integral and unimodular, i.e. A M S^-1 and (T + U M) S^-1 are integral
 * and |det A| = prod s_i (Section 4.2's checks).  By the three phases of
 * Section 2.2: Phase 1, s_n from p-adic lifting (as rns_largest_invariant);
 * Phase 2, index-(m, r) Smith massagers (Definition 2) in batches: each
 * batch lifts A^-1 J for a random J on the GPU (the resident C = A^-1 mod p),
 * projects it through the earlier batches (the first block of B^-1 of the
 * current massaged matrix), takes the Smith form of the n x t projection
 * over Z/sZ with its transforms (U and M of the batch), and continues with
 * s = the smallest invariant found; batch sizes grow with how far s fell, and
 * once s fits a machine word one batch takes all remaining invariants
 * (Section 3.2); Phase 3, |det A| = prod s_i checked exactly from det A mod
 * primes (stands in for the unimodularity certification of B; a failure
 * restarts, Las Vegas).
 * Positions: the invariants equal to 1 first (their U rows and M columns are
 * zero, their T columns unit vectors), then each batch in ascending order,
 * later batches first.  Entries are non-negative and reduced: column j of M
 * and T modulo s_j, row i of U modulo the modulus of its batch.
 * Requires n >= 16 and n max|a_ij| < 2^36 (RNS_ENOTSUP otherwise; n = 0 gives
 * an empty result); entries must not be INT64_MIN.  Read S with
 * rns_smith_get, the massager with rns_smith_massager_vector; free with
 * rns_smith_free.  Returns RNS_ESINGULAR when det A = 0, RNS_ERETRY when the
 * restart budget is exhausted.
 */
int rns_smith_massager(rns_ctx *ctx, const int64_t *A_host, int64_t n, uint64_t seed,
                       rns_smith_result **out);

#define RNS_MASSAGER_U 0   /* rows of U */
#define RNS_MASSAGER_M 1   /* columns of M */
#define RNS_MASSAGER_T 2   /* columns of T */

/*
 * rns_smith_massager_width -- 64-bit words per entry of row `index` of U
 * (which = RNS_MASSAGER_U) or column `index` of M or T; at least 1.  Returns
 * -RNS_EINVAL for a bad argument or a result without a massager.
 */
int rns_smith_massager_width(const rns_smith_result *r, int which, int64_t index);

/*
 * rns_smith_massager_vector -- copies row `index` of U, or column `index` of
 * M or T, to out: n entries of W words each (entry k at out[k W ..]),
 * little-endian, zero-extended.  RNS_EBOUND if W is below the width;
 * RNS_EINVAL for a bad argument or a result without a massager.
 */
int rns_smith_massager_vector(const rns_smith_result *r, int which, int64_t index, uint64_t *out, int W);

/* Invariant factor i (0-based) as little-endian 64-bit magnitude words. */
int rns_smith_get(const rns_smith_result *r, int64_t i, const uint64_t **words,
                  int *nwords);
int64_t rns_smith_size(const rns_smith_result *r);
int rns_smith_stats_get(const rns_smith_result *r, rns_smith_stats *st);
void rns_smith_free(rns_smith_result *r);

/* ------------------------------------------------------------------------
 * Kernel timing (tracing).  When enabled, every kernel the library launches
 * is bracketed by two HIP events recorded on the caller's stream (for
 * smith_form and rns_largest_invariant: on the solve's stream, including
 * the products they run on their internal basis; a run of lifting steps is
 * one record counting all its launches, and the lifting graphs are not
 * captured while tracing).
 * rns_ctx_profile_read synchronises those events and returns, for kernels
 * whose name contains `name` (NULL or "" = all), the summed duration in
 * milliseconds and the number of launches, then forgets them.
 * ---------------------------------------------------------------------- */
int rns_ctx_profile(rns_ctx *ctx, int enable);
int rns_ctx_profile_read(rns_ctx *ctx, const char *name, double *total_ms,
                         int64_t *launches);

/* ------------------------------------------------------------------------
 * Calibration: the sustained rate of one arithmetic unit on this device, to
 * state achieved rates beside the published peaks.  Every wave (eight per
 * CU) runs independent accumulation chains with register operands, no memory
 * traffic in the timed loop; `iters` iterations of 16 instructions per wave.
 * kind 0: v_mfma_i32_16x16x64_i8 (the instruction of the INT8-limb GEMM),
 *      1: v_mfma_i32_32x32x32_i8, 2: v_mfma_f64_16x16x4f64 (FP64 GEMM),
 *      3: vector v_fma_f64.
 * random_operands != 0 fills the operand registers with random bits (the
 * switching activity of real data, which decides the clock the chip holds
 * under load); 0 uses constant operands.  One untimed warm-up launch, then
 * one launch timed with HIP events on `stream`.  Outputs: integer ops (or
 * flops) per second and the timed launch in milliseconds.  Allocates and
 * frees a small device buffer.  Blocks until the timed launch ends.
 * ---------------------------------------------------------------------- */
int rns_calibrate(rns_ctx *ctx, int kind, int iters, int random_operands, void *stream,
                  double *ops_per_s, double *ms);

/* ------------------------------------------------------------------------
 * Serving: Smith-form requests of different sizes from a queue, several at
 * once on one GPU.  Worker threads each own a context (so their streams are
 * separate and admitted requests overlap on the device); a request is
 * admitted when its estimated device-memory footprint fits the budget
 * (oldest first, later requests may pass an older one that does not fit
 * until the older one has waited `aging` seconds, default 2).  A request
 * larger than the whole budget runs alone.  Each request has its own status;
 * a singular or failing request does not affect the others.
 * ---------------------------------------------------------------------- */
typedef struct rns_server rns_server;

typedef struct rns_request_info {
    int status;            /* smith_form status of this request */
    double t_submit;       /* seconds since the server started */
    double t_start;        /* admitted (work began) */
    double t_end;          /* finished */
    size_t footprint;      /* bytes reserved for it at admission */
    int worker;
} rns_request_info;

typedef struct rns_server_counters {
    size_t budget, in_use, high_water;
    int running, max_running, queued;
} rns_server_counters;

/* hbm_budget 0 = seven eighths of the device memory free at creation. */
int rns_server_create(int device, int workers, size_t hbm_budget, rns_server **out);
int rns_server_set_aging(rns_server *s, double seconds);
/* Copies A (n x n, host int64); *ticket identifies the request. */
int rns_server_submit(rns_server *s, const int64_t *A_host, int64_t n, uint64_t seed,
                      uint64_t *ticket);
/* Waits up to timeout_s seconds (negative = no limit).  Returns the request's
 * status (RNS_EPENDING if still running: wait again); on RNS_OK *out receives
 * the result (free with rns_smith_free).  A ticket can be waited for once. */
int rns_server_wait(rns_server *s, uint64_t ticket, double timeout_s,
                    rns_smith_result **out, rns_request_info *info);
int rns_server_stats(rns_server *s, rns_server_counters *st);
/* Estimated device bytes of one request of size n (the admission charge). */
int rns_server_footprint(int64_t n, size_t *bytes);
/* Stops the workers after the requests they are running; queued requests
 * are dropped. */
void rns_server_destroy(rns_server *s);

/*
 * rns_lift_step -- one step of Dixon's p-adic lifting (Section 3 names it as
 * the solver of the method's linear systems), run by the same kernels and the
 * same set-up as the Smith-form driver's lifting, on caller-given operands:
 *     X  = C (R mod p) mod p,
 *     R' = (R - A X) / p      (rounded toward zero; exact when C = A^-1 mod p),
 *     Rm' = R' mod p.
 * With C = A^-1 mod p this is the step the driver repeats; for other C the
 * division is inexact somewhere and *inexact is set.  It exists so that the
 * step kernels can be checked against a CPU computation at any n up to their
 * exactness bound.
 *   C:  device uint32, n x n row-major, residues in [0, p).
 *   A:  device int64, n x n row-major; stored as int16 when every |a| < 32640
 *       (the driver's rule), else int32 (entries must fit int32).
 *   R:  device int64, t vectors of n entries ([t][n]); |R| + n max|A| p < 2^63.
 *   X, Rm_next: device uint32 [t][n]; R_next: device int64 [t][n].
 *   form: 0 vector units only; 1 matrix cores (C Rm on INT8 MFMA; A X on
 *       INT8 MFMA as well when A is int16, with packed right operands when
 *       t <= 4).  n <= 43690 for form 1 (RNS_EBOUND beyond), n <= 65536.
 *   inexact: host int32, 1 if p does not divide some R - A X.
 *   kernels: host int, bit 0 C Rm on the matrix cores, bit 1 A X on the matrix
 *       cores, bit 2 packed right operands, bit 3 A stored as int16.
 * 1 <= t <= 16, p an odd prime below 2^26.  Allocates and frees its own work
 * buffers and synchronises `stream` before returning.
 */
int rns_lift_step(int device, const uint32_t *C, const int64_t *A, const int64_t *R, int64_t n, int t,
                  uint32_t p, int form, uint32_t *X, int64_t *R_next, uint32_t *Rm_next, int32_t *inexact,
                  int *kernels, void *stream);

/*
 * rns_unimodular_certify -- Section 2.2, Phase 3: decides whether the integer
 * matrix D is unimodular (|det D| = 1), deterministically, from high-order
 * X-adic residues computed by double-plus-one lifting (the certification the
 * paper takes from Pauderis and Storjohann; this library's reading):
 *   X = p_0 ... p_{j-1} (the first primes of the internal basis) with
 *   X >= 4 n^2 max|D|, C = D^-1 mod X, Z_0 = I and
 *       Z_{2e+1} = (Z_e Z_e - D cmod(C Z_e Z_e, X)) / X      (exact),
 *   which keeps I - D P_e = X^e Z_e for an integer P_e = D^-1 mod X^e with
 *   |P_e| < X^e and |Z_e| <= n max|D|.  Z_e = 0 proves D^-1 = P_e integral;
 *   a unimodular D reaches Z_e = 0 once X^e >= 4 H (H: Hadamard's bound on
 *   the (n-1)-minors), so the verdict is exact.  Each step is three residue
 *   products of n x n x n on the matrix cores (Z Z over j + l primes, C Y over
 *   j, D K over l) and two elementwise passes.
 *   D_host:    host int64, n x n row-major (leading dimension n); entries
 *              other than INT64_MIN, with n max|D| < 2^61.
 *   max_steps: < 0 runs the certificate (until Z_e = 0 or the bound's
 *              precision); >= 0 runs at most that many steps (Z_e = 0 ends
 *              early: it stays 0).
 *   Z_host:    optional host int64 n x n: the last residue Z_e.
 *   info:      verdict 1 (unimodular), 0 (not), -1 (steps ran out before the
 *              bound's precision); reason 0 residue vanished, 1 residue
 *              nonzero at the bound's precision, 2 D singular modulo a prime
 *              of X (then p | det D), 3 a zero column, 4 step limit; the
 *              primes of X and of the exact basis, steps run and needed,
 *              log2 H, log2 X, seconds, residue products.
 * n = 0 is unimodular.  n <= 43690 (the products' exact depth), else
 * RNS_ENOTSUP; RNS_EBOUND if n max|D| >= 2^61.  Synchronous.
 */
typedef struct rns_unimod_info {
    int32_t verdict, reason, steps, steps_needed;
    int32_t x_primes, q_primes;
    uint32_t x_prime[4], q_prime[4];
    double log2_bound, log2_x, seconds, residue_ops;
    int32_t products, reserved;
} rns_unimod_info;

int rns_unimodular_certify(rns_ctx *ctx, const int64_t *D_host, int64_t n, int max_steps,
                           int64_t *Z_host, rns_unimod_info *info);

/* Test hook: make the next `count` certifications of this context fail, to
 * exercise the Las Vegas restart (Section 2.2, Phase 3).  0 disables. */
int rns_ctx_force_cert_failures(rns_ctx *ctx, int count);

#ifdef __cplusplus
}
#endif

#endif /* RNS_H */
