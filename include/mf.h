/*
 * mf.h - C ABI of the fast bilinear matrix-multiplication library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library executes a fast algorithm <n0,n0,n0;R>, given by its factor
 * matrices U, V, W, on square row-major matrices: C = A B with A, B, C of
 * size n x n.  With the split factor p the operands are partitioned into
 * p x p blocks numbered row-major (A_k, k = i*p + j; the partition equations
 * of Section 2 of D'Alberto, "Strassen's Matrix Multiplication Algorithm Is
 * Still Faster", arXiv 2312.12732) and the algorithm computes (equation
 * "strassen" of Section 2)
 *
 *     T_r = sum_k U[k,r] A_k,   S_r = sum_l V[l,r] B_l,   P_r = T_r S_r,
 *     C_c = sum_r W[c,r] P_r,                             r = 0..R-1.
 *
 * Execution is a data flow of three phases on the caller's HIP stream:
 * pre-additions (linear combinations of operand blocks, one launch per
 * recursion level), the R^d leaf block products (one grouped MFMA GEMM
 * launch whose epilogue stores every product once in the workspace) and
 * post-additions (one launch per level, innermost first, combining the
 * stored products into the blocks of C).  Recursion to depth d runs level by
 * level; to run it as one level of the composed algorithm of split factor
 * p^d (the Kronecker construction of Section 2), compose the algorithm with
 * mf_algo_compose and call it at depth 1.
 *
 * Conventions for every entry point:
 *  - Device pointers are HIP device allocations; host pointers are ordinary
 *    host memory.  The library never takes ownership of caller memory.
 *  - Matrices are dense, row-major, contiguous (leading dimension n), with
 *    at least 8-byte alignment.  C must not overlap A or B (MF_ERR_ARG).
 *  - `stream` is a hipStream_t passed as a pointer; NULL means the default
 *    stream.  Calls are asynchronous with respect to the host: launch errors
 *    are returned as MF_ERR_HIP; faults surface at the caller's
 *    synchronisation.
 *  - Every entry point returns an mf_status; on error mf_last_error() gives a
 *    message for the calling thread.  Nothing aborts or throws across the
 *    ABI.
 *  - An mf_algo is immutable once created and may be shared between threads
 *    and streams.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_algo mf_algo;
typedef void* mf_stream; /* a hipStream_t */

typedef enum {
  MF_OK = 0,
  MF_ERR_ARG = -1,         /* invalid argument (null, negative size, overlap, unknown code) */
  MF_ERR_BRENT = -2,       /* U, V, W do not define a correct product algorithm */
  MF_ERR_SHAPE = -3,       /* sizes inconsistent with the algorithm or the workspace */
  MF_ERR_NOMEM = -4,       /* device or host allocation failed */
  MF_ERR_HIP = -5,         /* a HIP runtime call or kernel launch failed */
  MF_ERR_UNSUPPORTED = -6  /* valid request that the library does not implement */
} mf_status;

/* Element type of A, B, C (low byte) and precision of the leaf products
 * (second byte).  Pre- and post-additions always run in the storage type. */
enum {
  MF_F64 = 1,               /* double storage */
  MF_F32 = 2,               /* float storage */
  MF_LEAF_NATIVE = 0 << 8,  /* leaves in the storage type (FP64 or FP32 MFMA) */
  MF_LEAF_F32 = 1 << 8,     /* FP32 MFMA leaves (FP32 storage only) */
  MF_LEAF_BF16 = 2 << 8,    /* BF16 MFMA, FP32 accumulation (FP32 storage only) */
  MF_LEAF_BF16X3 = 3 << 8,  /* split-BF16 x3 compensated products, FP32 accumulation (FP32 storage only) */
  /* Schedule (third byte).  Default: the pre-additions run as linear-
   * combination launches that store each combined operand, every leaf
   * product is stored, and the post-additions run as launches after the
   * GEMM.  MF_SCHED_FUSED: one level of the algorithm (compose it for a
   * deeper split) with the pre-additions done inside the GEMM's operand load
   * (each operand tile summed from its <= 16 block terms in registers before
   * the LDS store) and the post-additions in the GEMM epilogue (a workgroup
   * runs every product at its tile position of all C blocks, in product
   * order: the first product feeding a block stores, later ones add), so no
   * workspace and no addition launches.  Leaves in the storage type only
   * (MF_ERR_UNSUPPORTED otherwise, and for more levels or more terms). */
  MF_SCHED_FUSED = 1 << 16
};

/* Row convention of W handed to mf_algo_from_uvw. */
enum {
  MF_W_ROWMAJOR_C = 0,  /* row c of W gives the coefficients of C_c (c = i*n0 + j) */
  MF_W_DEEPMIND_CT = 1  /* row t gives the coefficients of the C block with the transposed
                           2-d index, as in the c^t matrix printed in Section 2 (rows
                           labelled C_0, C_2, C_1, C_3 for n0 = 2) */
};

/* Build an algorithm from host arrays U, V, W, each n0*n0 x R, row-major
 * (entry [k*R + r]).  Coefficients are real; integer coefficients are checked
 * exactly.  The Brent equations (sum_r U[a,r] V[b,r] W[c,r] equals 1 when the
 * blocks a = (i,k), b = (k,j), c = (i,j) match and 0 otherwise; Section 2,
 * "prove them correct") are verified for all n0^6 index triples; a failure
 * returns MF_ERR_BRENT and no handle.  1 <= n0 <= 8, 1 <= R <= 4096.  The
 * caller owns *out and releases it with mf_algo_free. */
mf_status mf_algo_from_uvw(int n0, int R, const double* U, const double* V, const double* W,
                           int w_convention, mf_algo** out);

/* Built-in algorithms: "strassen" (the paper's printed form), "winograd"
 * (Strassen-Winograd), "strassen1969", "classical2", "classical3"
 * (the textbook <p,p,p;p^3> of equation "recursion"). */
mf_status mf_algo_builtin(const char* name, mf_algo** out);

/* Compose: apply `outer` first and `inner` to each of its products
 * (Kronecker construction of Section 2); split factors multiply dimension by
 * dimension (n0_outer*n0_inner for square algorithms, each at most 8),
 * R_outer*R_inner products.  The result is Brent-checked. */
mf_status mf_algo_compose(const mf_algo* outer, const mf_algo* inner, mf_algo** out);

/* Re-base by integer n0 x n0 matrices X, Y, Z with determinant +-1 (host,
 * row-major int64): the algorithm applied to X A Y^-1 and Y B Z^-1 yields
 * U'_r = X^T U_r Y^-T, V'_r = Y^T V_r Z^-T, W'_r = X^-1 W_r Z (U_r = column r
 * of U as an n0 x n0 matrix).  MF_ERR_ARG if a matrix is not unimodular. */
mf_status mf_algo_rebase(const mf_algo* a, const int64_t* X, const int64_t* Y, const int64_t* Z,
                         mf_algo** out);

/* Shape and sparsity of an algorithm (any output pointer may be NULL); *n0
 * is 0 for a rectangular algorithm (see mf_algo_shape). */
mf_status mf_algo_info(const mf_algo* a, int* n0, int* R, int* nnz_u, int* nnz_v, int* nnz_w);

/* Copy the canonical coefficients (W rows index C row-major) into host arrays
 * of m0*k0*R (U), k0*n0*R (V) and m0*n0*R (W) doubles (n0*n0*R each for a
 * square algorithm; any pointer may be NULL). */
mf_status mf_algo_get_uvw(const mf_algo* a, double* U, double* V, double* W);

/* Release an algorithm (NULL is ignored). */
void mf_algo_free(mf_algo* a);

/* ---- Rectangular algorithms ---------------------------------------------------
 * An algorithm <m0,k0,n0;R> splits A (M x K) into m0 x k0 blocks, B (K x N)
 * into k0 x n0 blocks and C (M x N) into m0 x n0 blocks, each numbered
 * row-major (A_(i,k) has index i*k0 + k, B_(k,j) index k*n0 + j, C_(i,j)
 * index i*n0 + j).  Equation "strassen" of Section 2 then reads
 *     T_r = sum U[(i,k), r] A_(i,k),   S_r = sum V[(k,j), r] B_(k,j),
 *     P_r = T_r S_r,                   C_(i,j) = sum_r W[(i,j), r] P_r,
 * and the Brent equations sum_r U[(i,k),r] V[(k',j),r] W[(i',j'),r] =
 * [i = i'][k = k'][j = j'] are checked for every index triple.  Square
 * algorithms are the case m0 = k0 = n0.  Section 2 builds a 6 x 6 x 6
 * product from non-square pieces by the Kronecker product of their factor
 * matrices (mf_algo_compose); the direct sum (mf_algo_concat) builds
 * rectangular algorithms from smaller ones, e.g. <2,2,3;11> from Strassen's
 * <2,2,2;7> and the textbook <2,2,1;4>.  Every level of a rectangular
 * algorithm needs a linear-combination kernel for m0*k0, k0*n0 and R inputs
 * per set (4, 6, 7, 8, 9, 11, 12, 16, 17, 27, 36, 49, 64, 81; a composition
 * runs as its factors when it has none of its own), else MF_ERR_UNSUPPORTED
 * at planning. */

/* U (m0*k0 x R), V (k0*n0 x R), W (m0*n0 x R): host arrays, row-major, W rows
 * indexing C row-major.  1 <= m0, k0, n0 <= 8, 1 <= R <= 4096; MF_ERR_BRENT
 * if the Brent equations fail. */
mf_status mf_algo_from_uvw_rect(int m0, int k0, int n0, int R, const double* U, const double* V,
                                const double* W, mf_algo** out);

/* The textbook partitioned product <m0,k0,n0; m0*k0*n0>: one product
 * A_(i,k) B_(k,j) per (i, j, k), added into C_(i,j) (the definition of
 * Section 2, partitioned). */
mf_status mf_algo_classical(int m0, int k0, int n0, mf_algo** out);

/* Direct sum of two algorithms along one dimension, the products of `a`
 * first: axis 0 stacks the rows of A and C (a's m0 rows of blocks, then
 * b's), axis 1 splits the inner dimension (C = A_a B_a + A_b B_b), axis 2
 * places the columns of B and C side by side.  The other two split factors
 * must agree (MF_ERR_ARG).  The result is Brent-checked. */
mf_status mf_algo_concat(const mf_algo* a, const mf_algo* b, int axis, mf_algo** out);

/* Split factors and rank (any output pointer may be NULL). */
mf_status mf_algo_shape(const mf_algo* a, int* m0, int* k0, int* n0, int* R);

/* C = A B with up to `depth` levels of `algo` (equation "strassen" of
 * Section 2 applied recursively: T_r, S_r from the blocks of the level above,
 * P_r = T_r S_r by recursion or by the leaf GEMM, C_c = sum_r W[c,r] P_r).
 * A level is taken while levels remain, the current size exceeds `cutoff`
 * and the 128 leaf tile, and the number of leaf products stays within 2^16
 * (sizes are rounded up at each split); depth 0 (or cutoff >= n) is the
 * classical product.  Sizes that the split factor does not divide are
 * handled by virtual zero padding (no copy of A, B or C).  Temporaries come
 * from a stream-ordered pool owned by the library, one per device, which
 * keeps the memory it has reserved until the process ends (so repeated calls
 * do not map fresh device memory).  A, B, C: device pointers to n x n
 * matrices of the storage type of `dtype`. */
mf_status mf_fastmm(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B, void* C,
                    int64_t n, int dtype, mf_stream stream);

/* C = A B by the library's own MFMA GEMM, no fast algorithm: the definition
 * C_ij = sum_k A_ik B_kj (Section 2, equation "basic"; the same product as
 * the classical blocked recursion of equation "recursion").  dtype as for
 * mf_fastmm.  BF16 leaves stage the operands in workspace from the library's
 * pool.  Rows that are not 16-byte aligned (n odd in FP64, not a multiple of
 * 4 in FP32, or a base of A or B off a 16-byte boundary) are copied, for
 * n >= 192, into aligned workspace blocks from that pool first (one launch;
 * the GEMM then loads whole K steps straight into LDS).  mf_fastmm copies
 * them at its first level in the same cases. */
mf_status mf_classical_mm(const void* A, const void* B, void* C, int64_t n, int dtype, mf_stream stream);

/* The general product C = alpha A B + beta C (Section 3 states the
 * operation as C = alpha A B) for row-major A (M x K, leading dimension
 * lda >= K), B (K x N, ldb >= N) and C (M x N, ldc >= N), with up to `depth`
 * levels of `algo` (square or rectangular; NULL with depth 0 for the
 * classical product).  M, N, K <= 2^20; lda, ldb <= 2^21 and ldc < 2^31
 * (MF_ERR_SHAPE beyond).  A level is taken while levels remain and every
 * dimension the algorithm splits exceeds `cutoff` and the 128 leaf tile;
 * dimensions the splits do not divide are padded virtually with zeros.  The
 * scaling is applied where results are written into C (the last
 * post-addition, or the GEMM epilogue of a classical product); beta = 0 does
 * not read C.  dtype MF_F64 or MF_F32 (leaves in the storage type; reduced
 * precision leaves are available through mf_fastmm).  M or N = 0: nothing to
 * do; K = 0: MF_ERR_SHAPE.  C must not overlap A or B (MF_ERR_ARG, by the
 * byte ranges the three views span).  Workspace from the library's pool, as
 * for mf_fastmm; a classical product whose A or B rows are not 16-byte
 * aligned (leading dimension or base) copies both operands into it first
 * when M, N and K are all at least 192. */
mf_status mf_gemm(const mf_algo* algo, int depth, int cutoff, int64_t M, int64_t N, int64_t K, double alpha,
                  const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                  int dtype, mf_stream stream);

/* Bytes of device workspace mf_fastmm_ws needs for this request (0 for a
 * classical product with leaves in the storage type, except that rows which
 * are not 16-byte aligned, at n >= 192, take two aligned copies of
 * ceil(n / 16)^2 * 256 elements (mf_fastmm_ws plans from n alone, so
 * operand bases off a 16-byte boundary are read in place there); BF16 leaves stage every leaf operand as BF16
 * planes, and their last pre-addition level writes those planes directly, so
 * its FP32 sums take no workspace). */
mf_status mf_workspace_bytes(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype,
                             size_t* bytes);

/* Shape and algorithmic cost of the plan mf_fastmm uses for a request (host
 * only).  Byte counts are what the addition stages must move at least: every
 * valid element of every input view read once and every element of every
 * output written once.  Input views exclude virtual padding; an output that
 * is a workspace block is written whole (zeros in its padding), since the
 * leaf GEMM reads whole blocks. */
typedef struct {
  int levels;          /* recursion levels taken (0: classical) */
  int levels_outer;    /* levels whose post-additions run as separate stages */
  int groups;          /* products are grouped by the outer levels */
  int pre_stages, post_stages;
  int64_t leaf_m;      /* leaf rows: a multiple of 16 with FP64 / FP32 leaves (the GEMM covers
                          them with whole 128 x 128 tiles), of 128 with BF16 leaves or fused
                          operands */
  int64_t products;    /* R^levels leaf products */
  double gemm_flops;   /* MFMA work as executed: per product 2 M' N' K, M' and N' the leaf
                          rows and columns rounded up to whole 128 tiles,
                          K = the product's valid inner size rounded up to 16 (FP64 / FP32
                          leaves) or the padded leaf K (BF16 leaves, fused operands) */
  double pre_bytes;    /* algorithmic bytes of all pre-addition stages */
  double post_bytes;   /* algorithmic bytes of all post-addition stages */
  size_t ws_bytes;     /* as mf_workspace_bytes */
} mf_plan_info;
mf_status mf_plan_query(const mf_algo* algo, int depth, int cutoff, int64_t n, int dtype, mf_plan_info* out);

/* As mf_fastmm, with caller-owned device workspace of ws_bytes bytes
 * (256-byte aligned; MF_ERR_SHAPE if smaller than mf_workspace_bytes).  The
 * first mf_workspace_bytes bytes must not overlap A, B or C (MF_ERR_ARG,
 * detected by address range).  The workspace must not be used by other work
 * until the call has completed on `stream`. */
mf_status mf_fastmm_ws(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B, void* C,
                       int64_t n, int dtype, void* workspace, size_t ws_bytes, mf_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * mf_fastmm, but the plan's descriptors and its workspace live in one fixed
 * device array of MF_NOALLOC_SCRATCH_BYTES bytes per GPU, which the library
 * holds from the first call on that GPU until the process ends; the call
 * itself allocates no device memory (the descriptors are copied into the
 * array on `stream`).  A request whose descriptors (rounded up to 256 bytes)
 * plus mf_workspace_bytes exceed the array is rejected with MF_ERR_SHAPE
 * before anything is enqueued (FP64, Strassen depth 1: up to n of about
 * 2900), unless it fits once operands whose rows are not 16-byte aligned are
 * read in place instead of copied into aligned blocks (then it runs so).  Every call on one GPU uses the same array, and nothing in it is
 * assumed to be zero: calls on one stream are ordered, but calls that
 * overlap on one GPU (other streams, other host threads) race on it and give
 * wrong results.  The result is bitwise that of mf_fastmm with the same
 * arguments.  No phase timing is recorded. */
#define MF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
mf_status mf_fastmm_noalloc(const mf_algo* algo, int depth, int cutoff, const void* A, const void* B, void* C,
                            int64_t n, int dtype, mf_stream stream);

/* ---- Batched execution ----------------------------------------------------
 * Many independent products C_i = A_i B_i (i < count) of sizes n[i], each
 * with its own algorithm (algos[i], NULL when depth[i] == 0), depth and
 * cutoff, all with storage dtype MF_F64 or MF_F32 (leaves in the storage
 * type).  The plan is a task list (addition chunks and GEMM tiles of every
 * instance) in topological order, split into phases: pre-addition level 0 of
 * every instance, level 1, ..., all GEMM tiles (largest leaves first), then
 * the post-addition levels.  A run launches each phase once over all
 * instances (one workgroup per task), so instances of different sizes share
 * the GPU within every launch.  Every instance runs the plan mf_fastmm uses
 * for the same arguments, so its result is bitwise that of the standalone
 * call.  Supported algorithm shapes: combinations of 4, 7, 8, 9 or 16
 * inputs, and of 27 (at most 9 outputs), 49 or 64 (at most 16 outputs)
 * inputs; other shapes give MF_ERR_UNSUPPORTED.  The persistent form
 * (mf_batch_create_form) runs the same task list in one launch.  A batch
 * plan is immutable; its runs are ordered (see mf_batch_run). */
typedef struct mf_batch mf_batch;

/* Plan a batch (host only; device state is made on the first run).  The
 * algorithm handles must outlive the batch.  1 <= n[i] <= 65536.  The batch
 * runs in the phase form (MF_BATCH_PHASES below). */
mf_status mf_batch_create(int count, const int64_t* n, const mf_algo* const* algos, const int* depth,
                          const int* cutoff, int dtype, mf_batch** out);

/* Execution form of a batch. */
enum {
  MF_BATCH_PHASES = 0,     /* one launch per phase, one workgroup per task; no waits */
  MF_BATCH_PERSISTENT = 1  /* the whole task list in ONE launch of about two workgroups per compute
                              unit: each takes the next task from a global ticket, waits until the
                              per-instance counter of the stage it depends on is complete, runs the
                              task and counts it done.  A task waits only on tasks with smaller
                              tickets, held by running workgroups, so the schedule cannot deadlock;
                              every wait is bounded (a few seconds), after which the run aborts
                              (mf_batch_aborted) instead of hanging.  Supports combinations of 4, 7,
                              8, 9 or 16 inputs (MF_ERR_UNSUPPORTED otherwise). */
};

/* As mf_batch_create with the execution form `form` (MF_ERR_ARG if unknown).
 * Both forms run the same tasks on the same plans, so their results are
 * bitwise equal. */
mf_status mf_batch_create_form(int count, const int64_t* n, const mf_algo* const* algos, const int* depth,
                               const int* cutoff, int dtype, int form, mf_batch** out);

/* Device workspace bytes a run needs (0 if every instance is a classical
 * product that copies nothing, as mf_workspace_bytes). */
mf_status mf_batch_workspace_bytes(const mf_batch* b, size_t* bytes);

/* Run the batch on `stream`.  A, B, C: host arrays of `count` device
 * pointers to n[i] x n[i] row-major matrices (C_i must not overlap A_i or
 * B_i).  workspace: NULL (stream-ordered pool of the library) or a caller
 * buffer of at least mf_batch_workspace_bytes, 256-byte aligned, whose first
 * mf_batch_workspace_bytes bytes overlap no A_i, B_i or C_i (MF_ERR_ARG).
 * Runs of one batch are ordered: a run issued on another stream (or from
 * another host thread) starts after the previous run has finished, since
 * every run rewrites the batch's device instance table. */
mf_status mf_batch_run(const mf_batch* b, const void* const* A, const void* const* B, void* const* C,
                       void* workspace, size_t ws_bytes, mf_stream stream);

/* Waits for the device and reports whether the last run aborted (a wait of
 * the persistent form exceeded its bound; the results of that run are then
 * incomplete); a run of the phase form never aborts, so *aborted is 0. */
mf_status mf_batch_aborted(const mf_batch* b, int* aborted);

/* The task graph, for host-side schedule checks: *ntasks tasks and *nctr
 * counters; if desc is not NULL it receives 5 ints per task in launch order:
 * type (0 addition chunk, 1 GEMM tile), instance, wait counter (-1: none),
 * wait value, done counter. */
mf_status mf_batch_tasks(const mf_batch* b, int* ntasks, int* nctr, int32_t* desc);

/* The phases of the task list: *nphases phases; if desc is not NULL it
 * receives 3 ints per phase: first task, end task (exclusive), 1 if the phase
 * holds GEMM tiles (else addition chunks).  The phases partition the list. */
mf_status mf_batch_phases(const mf_batch* b, int* nphases, int32_t* desc);

/* Release a batch (NULL is ignored). */
void mf_batch_free(mf_batch* b);

/* ---- Autotuner of the batched form ------------------------------------------
 * For each of nsizes sizes n[i], measures every candidate plan where it will
 * run, in a batch of many products of that size, and picks the
 * one with the least device time per product; a fast plan is taken only if it
 * beats the classical GEMM by at least 5% (the margin pays for the addition
 * launches it adds to a mixed batch).  Candidates, ncand =
 * 1 + nalgos * max_depth of them: index 0 is the classical GEMM; index
 * 1 + j * max_depth + (d - 1) is algos[j] at depth d (1 <= d <= max_depth).
 * A depth whose levels the plan would not take for that size (see
 * mf_fastmm) repeats a shallower plan and is skipped (time -1).  Each
 * measurement plans a batch of copies = ceil(work_flops / (2 n^3)) products
 * (at most max_copies, at most 8 GiB of operands, and for a fast candidate
 * at most 8 GiB of workspace), fills distinct
 * operands on the device with the counter-based generator, runs it once
 * untimed and then `reps` times between two HIP events on `stream`.
 * Outputs: out_choice[i] = index of the fastest candidate for n[i];
 * out_ms[i * ncand + c] = device ms per product of candidate c (or -1).
 * Allocates and frees its own device memory and synchronises before it
 * returns.  Errors: MF_ERR_ARG / MF_ERR_SHAPE / MF_ERR_UNSUPPORTED for bad
 * arguments, MF_ERR_NOMEM, MF_ERR_HIP (including an aborted batch). */
mf_status mf_autotune_batch(int nsizes, const int64_t* n, int dtype, const mf_algo* const* algos, int nalgos,
                            int max_depth, double work_flops, int max_copies, int reps, mf_stream stream,
                            int* out_choice, double* out_ms);

/* ---- Serving -----------------------------------------------------------------
 * A request loop for fast-multiply requests of different sizes.  The server
 * owns one device arena of hbm_budget bytes.  Requests wait in a FIFO queue;
 * the head request is admitted when one of max_slots slots (HIP streams) is
 * free and the HBM it needs (A, B, C and the temporaries of its plan) fits in
 * the arena as one block, first fit (allow_overtake lets later requests that
 * fit pass a blocked head).  An admitted request generates A and B in its
 * block on the device from its seed (mf_fill_uniform with seeds 2*seed and
 * 2*seed+1), runs its product and copies C out if asked, all on its slot's
 * stream, so requests on different slots overlap; its block is released when
 * its completion is observed.  The plan is a pure function of (n, dtype):
 * depth k+1 is used when n >= depth_min_n_*[k] (0 disables a level; algo
 * NULL means classical only); results are therefore identical alone and among
 * other requests. */
typedef struct {
  int max_slots;                /* 1..64 concurrent requests */
  size_t hbm_budget;            /* bytes for all admitted requests together */
  int allow_overtake;           /* 0: strict FIFO admission */
  int64_t depth_min_n_f64[4];   /* depth policy for MF_F64 requests */
  int64_t depth_min_n_f32[4];   /* depth policy for MF_F32 requests */
} mf_server_config;
typedef struct mf_server mf_server;

/* Start a server (a worker thread, max_slots streams and the arena on the
 * current device; MF_ERR_NOMEM if the arena cannot be allocated).  algo (may
 * be NULL) must outlive the server. */
mf_status mf_server_create(const mf_server_config* cfg, const mf_algo* algo, mf_server** out);
/* HBM bytes a request of this size and dtype is admitted against. */
mf_status mf_server_need_bytes(const mf_server* s, int64_t n, int dtype, size_t* bytes);
/* Enqueue a request (dtype MF_F64 or MF_F32).  host_out: NULL, or pinned
 * host memory of n*n elements that receives C.  MF_ERR_NOMEM if the request
 * alone exceeds the budget.  *id: request index (may be NULL). */
mf_status mf_server_submit(mf_server* s, int64_t n, int dtype, uint64_t seed, void* host_out, int64_t* id);
/* Enqueue a request on caller-owned device operands: C = A B for n x n
 * row-major A, B, C of the storage type of dtype (MF_F64 or MF_F32; C must not
 * overlap A or B, MF_ERR_ARG).  The request is admitted against the HBM of its
 * workspace only; A and B must stay valid and unchanged, and C untouched by
 * other work, until the request has completed (mf_server_drain).  Its plan is
 * the same pure function of (n, dtype) as for mf_server_submit, so C is
 * bitwise what mf_server_submit would give for the same operands. */
mf_status mf_server_submit_operands(mf_server* s, int64_t n, int dtype, const void* A, const void* B, void* C,
                                    int64_t* id);
/* Submit `count` requests from a replay thread at arrival times t_arrive[k]
 * seconds after the call (host arrays are copied). */
mf_status mf_server_replay(mf_server* s, int count, const double* t_arrive, const int64_t* n, const int* dtype,
                           const uint64_t* seed);
/* Wait until every submitted request has completed (including a replay). */
mf_status mf_server_drain(mf_server* s);
/* Per request (in id order; any pointer may be NULL): arrival, admission and
 * completion times in seconds since the server started (-1 if not done),
 * size and depth used; *count = number of requests. */
mf_status mf_server_stats(mf_server* s, int64_t* count, double* t_arrive, double* t_admit, double* t_done, int64_t* n,
                          int* depth);
/* Per request (in id order): device time in ms from the start of its first
 * operation on its slot's stream to its completion, -1 if not done; ms must
 * hold as many entries as mf_server_stats reports requests. */
mf_status mf_server_device_ms(mf_server* s, double* ms);
/* Per request (in id order): the start and end of its device work on the
 * device's own timeline, in ms since an origin event recorded when the
 * server started (-1 if not done); requests whose intervals intersect ran on
 * the device at the same time.  Arrays as for mf_server_device_ms. */
mf_status mf_server_device_interval(mf_server* s, double* start_ms, double* end_ms);
/* Stop the worker after the queue drains and release the server. */
void mf_server_free(mf_server* s);

/* Host-only simulation of the admission controller (the same policy and
 * first-fit arena as the server) with given arrival times, service times and
 * HBM needs (for tests and capacity planning): fills admission and
 * completion times and the peak arena bytes in use. */
mf_status mf_admission_simulate(int count, const double* t_arrive, const double* service, const size_t* need,
                                int slots, size_t budget, int allow_overtake, double* t_admit, double* t_done,
                                size_t* peak_used);

/* Fill count elements of device memory p (dtype MF_F64 or MF_F32) with the
 * counter-based generator of the serving runtime: element i is 2u - 1 where
 * u is the top 53 bits of the SplitMix64 output function applied to
 * seed + (i + 1) * 0x9e3779b97f4a7c15, times 2^-53. */
mf_status mf_fill_uniform(void* p, int64_t count, int dtype, uint64_t seed, mf_stream stream);

/* Phase timing (tracing).  While enabled, every mf_fastmm / mf_fastmm_ws /
 * mf_classical_mm call records HIP events on its stream around its three
 * phases: 0 pre-additions, 1 grouped leaf GEMM with the fused epilogue
 * post-addition, 2 outer post-addition.  mf_phase_timing_read waits for the
 * recorded calls, writes the summed milliseconds of each phase to ms[0..2]
 * and the number of calls to *calls (either pointer may be NULL), and
 * forgets them. */
mf_status mf_phase_timing(int enable);
mf_status mf_phase_timing_read(double* ms, int* calls);

/* Message of the last error on the calling thread ("" if none). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
