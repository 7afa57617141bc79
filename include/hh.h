/*
 * hh.h - adaptive mixed-precision hybrid hierarchical (H_h) matrices on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Khan & Carson, "Hybrid hierarchical matrices with adaptive mixed
 * precision storage". The library builds the H_h representation of a dense
 * kernel matrix H_ij = f(|p_i - p_j|) (eq:kernel_mat) and applies it, or its
 * transpose, to one or many vectors with hand-written gfx950 kernels.
 *
 * Conventions shared by every entry point
 *   - Status codes: every function returns hh_status; on failure the
 *     thread-local message of hh_last_error() says what was wrong. Inputs are
 *     validated on the host before any device work is queued.
 *   - Handles are opaque, own all their device memory and are immutable after
 *     hh_build / hh_derive. Two threads may call hh_matvec on one handle only
 *     on the same stream (the handle's workspace is shared).
 *   - Vectors x and y of the products are DEVICE pointers, row-major
 *     N x nrhs (a contiguous (N, nrhs) tensor), in the caller's point order.
 *     y is overwritten (never accumulated into); x and y must not alias.
 *   - Products are asynchronous on the given HIP stream (0 = null stream). A
 *     device fault surfaces as HH_EHIP at the next synchronising call.
 *   - The current HIP device at hh_build time is the device of the handle;
 *     products must be called with that device current.
 */
#ifndef HH_H
#define HH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hh_handle hh_handle;
typedef struct hh_plan hh_plan;

typedef enum {
    HH_OK = 0,
    HH_EINVAL = 1,     /* invalid argument (checked on the host, nothing queued) */
    HH_ENOMEM = 2,     /* device or host allocation failed; nothing leaked       */
    HH_EHIP = 3,       /* a HIP / rocBLAS / rocSOLVER call failed                 */
    HH_ENOTSUP = 4,    /* valid but unsupported combination                       */
    HH_EINTERNAL = 5   /* internal consistency check failed                       */
} hh_status;

/* Kernel functions of the paper's numerical section (Sec. 5) and the
 * nonsymmetric double-layer kernel. Every entry is multiplied by `scale`.
 *   HH_LOG          log r                       (singular: H_ii = 0)
 *   HH_INV_R        1 / r                       (singular)
 *   HH_INV_R2       1 / r^2                     (singular)
 *   HH_GAUSS        exp(-r^2 / h^2)             (regular: H_ii = scale)
 *   HH_MATERN       exp(-r / h)                 (regular)
 *   HH_DOUBLE_LAYER n_j . (p_i - p_j) / r^3     (singular, nonsymmetric)
 * For singular kernels the diagonal and the entries of coincident distinct
 * points are 0 (the paper sets H_ii = 0 for singular f). */
typedef enum {
    HH_LOG = 1, HH_INV_R = 2, HH_INV_R2 = 3, HH_GAUSS = 4, HH_MATERN = 5,
    HH_DOUBLE_LAYER = 6
} hh_kernel_type;

/* Storage formats of Table tab:precisions used for the low-rank factors, and
 * the continuum format of the accessor remark of Sec. 4.3: per block t
 * fraction bits (7 <= t <= 23) behind a sign and an 8-bit exponent with fp32's
 * range and gradual underflow, 9 + t bits per entry, round to nearest even
 * (t = 7 is bf16, t = 23 fp32). HH_FMT_Q43 is the 8-bit row of the table: a
 * sign, 4 exponent bits (bias 7) and 3 fraction bits, gradual underflow below
 * 2^-6, largest value 240, one byte per entry. */
enum { HH_FMT_FP64 = 0, HH_FMT_FP32 = 1, HH_FMT_FP16 = 2, HH_FMT_BF16 = 3, HH_FMT_CONT = 4,
       HH_FMT_Q43 = 5 };
/* Element type of x and y in the products. */
enum { HH_IO_F64 = 0, HH_IO_F32 = 1 };

/* Block kinds (Alg. 1). */
enum {
    HH_BLK_FAR = 0,        /* standard-admissible interaction list IL_s, levels 1..ell */
    HH_BLK_NEAR = 1,       /* compressed finer neighbours N_s at the switching level    */
    HH_BLK_WEAK = 2,       /* weak-admissible siblings IL_w, levels ell+1..L            */
    HH_BLK_DIAG = 3,       /* dense leaf diagonal block                                  */
    HH_BLK_DENSE_NEAR = 4  /* dense leaf neighbour (only when ell == L)                  */
};

typedef struct {
    int type;                /* hh_kernel_type                                        */
    double scale;            /* multiplies every entry (e.g. 1/(4 pi)); 0 means 1     */
    double h;                /* length scale of HH_GAUSS / HH_MATERN; 0 means 1       */
    const double* normals;   /* HOST, N x d row-major, HH_DOUBLE_LAYER only; copied   */
} hh_kernel;

typedef struct {
    uint32_t precision_mask; /* bit f set = format f available to the rule
                                (bits 0-3: fp64, fp32, fp16, bf16; bit 5: q43,
                                the 8-bit row of Table tab:precisions, tried
                                first); fp64 is always available. 0 means 0xF */
    int uniform_fp64;        /* 1: store every factor in fp64 (same tree, partition
                                and ranks); the uniform-precision baseline        */
    int io_dtype;            /* HH_IO_F64 (default) or HH_IO_F32 for x and y       */
    uint64_t seed;           /* key of the randomized-compression sketches          */
    int continuum;           /* 1: continuum storage (HH_FMT_CONT) instead of the
                                mask's formats (q43 included): each block takes the fewest
                                fraction bits t in [7, 23] whose unit roundoff
                                2^-(t+1) passes the rule, else fp64. 2: the same
                                with t in {7, 15, 23} only (16-, 24- and 32-bit
                                entries, whole bytes: faster to load)          */
    int64_t unit_bytes;      /* factor bytes per work unit of the single-vector
                                accumulation; 0 = 1 MiB (hh_autotune picks one)  */
    int64_t dot_task_elems;  /* stored entries per single-vector inner-product
                                task; 0 = 65536 (hh_autotune picks one)         */
} hh_options;

typedef struct {
    int32_t n, d, L, ell;                 /* points, dimension, depth, switching level */
    int32_t leaf_size, max_rank;
    int64_t n_blocks_lowrank;             /* low-rank blocks with rank > 0             */
    int64_t n_blocks_rank0;               /* admissible blocks compressed to rank 0    */
    int64_t n_blocks_dense;               /* dense blocks (diagonal + dense neighbours) */
    int64_t blocks_by_format[6];          /* low-rank blocks per HH_FMT_*              */
    int64_t factor_bytes_by_format[6];    /* device bytes of U and V per format        */
    int64_t dense_bytes;                  /* device bytes of dense blocks (fp64)       */
    int64_t lowrank_entries;              /* sum_b k_b (m_b + n_b)                     */
    int64_t dense_entries;                /* sum m n over dense blocks                 */
    int64_t total_columns;                /* sum_b k_b                                  */
    double storage_words;                 /* paper's bit-weighted storage, 64-bit words:
                                             sum k (m + n) b / 64 + sum m n (Sec. 5.2)  */
    double storage_words_fp64;            /* the same with every factor in fp64        */
    double matvec_bytes;                  /* algorithmic HBM bytes of one nrhs = 1
                                             product: factors (k (m + n) bits / 8 per
                                             block) + dense + x + y                    */
    double norm2_total;                   /* ||H~||_F^2 from Alg. 5                    */
    double build_seconds;                 /* wall time of hh_build / hh_derive         */
    double phase_bytes[3];                /* algorithmic HBM bytes of the three kernels
                                             of one nrhs = 1 product: [0] gather (x in,
                                             gathered x out), [1] inner products (V
                                             factors), [2] leaf accumulation (U factors,
                                             dense blocks, y out)                      */
} hh_stats;

typedef struct {                          /* one block, canonical order (level, i, j)  */
    int32_t level, kind, rank, format;    /* kind HH_BLK_*, format HH_FMT_*           */
    int64_t box_i, box_j;                 /* Morton indices of the two tree boxes     */
    int64_t row_begin, row_end;           /* row range [begin, end) in tree order     */
    int64_t col_begin, col_end;           /* column range in tree order               */
    int32_t exp_u, exp_v;                 /* stored factor = value * 2^-exp            */
    int32_t lowrank;                      /* 1 = U V^T factors, 0 = dense              */
    int32_t frac_bits;                    /* t of an HH_FMT_CONT block, else 0         */
    double norm2;                         /* ||H~_b||^2 (truncated) or ||H_b||^2        */
    double entry_norm2;                   /* ||H_b||_F^2 summed from the entries       */
    double tail_prev, tail;               /* discarded tail at rank-1 and at rank      */
} hh_block_info;

/* ------------------------------------------------------------------ build */

/* hh_build: H_h representation of the kernel matrix of `points`.
 * Follows Alg. 1 (tree of Sec. 2.1, hybrid admissibility eq:hybrid_admiss,
 * truncated-SVD compression with accuracy tol per admissible block, Def. of
 * H_h(p, eps)), Alg. 5 (norms from singular values) and Alg. 3 (per-block
 * storage precision: the largest unit roundoff u <= tol / (2^(d l / 2) xi_b)).
 * Blocks with min(m, n) <= 512 take the truncated SVD itself; larger blocks a
 * randomized range finder (Rademacher sketch keyed by opt->seed, one power
 * iteration) whose discarded tail includes the directly summed residual
 * ||H_b - Q Q^T H_b||_F^2, so ||H_b - U_b V_b^T||_F <= tol ||H_b||_F holds for
 * every block. HH_ENOTSUP if one factor column would span 2^31 bytes or more
 * (the product kernels address factors with 32-bit offsets).
 *   points        HOST, n x d row-major float64; copied.
 *   n             number of points, >= 1.     d in {1, 2, 3}.
 *   k             kernel description (not NULL).
 *   tol           target accuracy eps, 2^-52 < tol < 1.
 *   eta           admissibility parameter of eq:H_admiss, > 0.
 *   switch_level  ell in [0, L]; -1 selects the paper's default L - 1. ell = L
 *                 gives the H_s matrix, ell = 0 the HODLR matrix. L is the
 *                 smallest L >= 0 with leaf_size * 2^(dL) >= n.
 *   leaf_size     n_max >= 1.
 *   opt           NULL for defaults.
 *   out           receives the handle (set to NULL on failure).
 * Runs synchronously on the current device; needs roughly
 * 8 (sum_b k_b (m_b + n_b)) bytes of device memory beyond the result. */
hh_status hh_build(const double* points, int64_t n, int d, const hh_kernel* k,
                   double tol, double eta, int switch_level, int leaf_size,
                   const hh_options* opt, hh_handle** out);

/* hh_derive: a new handle with the same tree, partition and low-rank factors
 * as `src`, re-stored under the precision rule of Alg. 3 with options `opt`.
 * `src` must hold every low-rank factor in fp64 (built with uniform_fp64 = 1,
 * or with precision_mask = fp64 only); HH_ENOTSUP otherwise, and when src
 * has ell == L (its dense neighbours carry no factors). */
hh_status hh_derive(const hh_handle* src, const hh_options* opt, hh_handle** out);

/* hh_switch_level_search: the switching level of Sec. 3.3 (Alg. 2) that the
 * walk from ell = L downward finds for the storage gain S1(ell) - S2(ell) of
 * H_h over H_s (eq:S1, eq:S2). Builds H_s (switching level L) with hh_build's
 * arguments and reads S1(ell) for every ell from it (interaction lists of
 * levels ell+1..L plus the leaf neighbours); then, for ell = L-1, L-2, ...,
 * builds H_h(ell) and reads S2(ell) (compressed neighbours N_s(ell) plus the
 * sibling lists of levels ell+1..L), stopping at the first level whose gain
 * does not exceed the previous one (a tie stops the walk). Storage is counted
 * in 64-bit words weighted by each block's storage bits (k (m + n) bits / 64
 * for factors, m n for dense blocks), so opt->uniform_fp64 = 1 gives the
 * paper's uniform-precision choice and the adaptive rule the mixed-precision
 * one. Every handle is freed before returning; each build needs the device
 * memory hh_build needs, and the call takes the time of all its builds.
 *   points, n, d, k, tol, eta, leaf_size, opt   as for hh_build.
 *   level_out   HOST, receives ell* (-1 on failure).
 *   s1, s2      HOST arrays of cap doubles, or NULL. On success
 *               s1[ell] = S1(ell) for ell = 0..L; s2[ell] = S2(ell) for the
 *               levels the walk built, s2[L] = S1(L), NaN elsewhere.
 *   cap         entries of s1 / s2; HH_EINVAL if either is non-NULL and
 *               cap < L + 1 (hh_plan_info gives L).
 * Errors of a build are returned as hh_build returns them. */
hh_status hh_switch_level_search(const double* points, int64_t n, int d, const hh_kernel* k,
                                 double tol, double eta, int leaf_size, const hh_options* opt,
                                 int32_t* level_out, double* s1, double* s2, int32_t cap);

/* -------------------------------------------------------------- products */

/* hh_matvec: y = H^ x (Alg. 4): for every low-rank block y_I += U_b (V_b^T x_J),
 * for every dense block y_I += H_IJ x_J. x, y DEVICE, n x nrhs row-major in the
 * handle's io_dtype. Low-rank blocks stored in fp32 / fp64 and all dense blocks
 * are applied in fp64 arithmetic; fp16 / bf16 blocks multiply and accumulate
 * their inner products in fp32. Rows are accumulated in fp64, without atomics:
 * results are bitwise reproducible run to run.  nrhs >= 1. */
hh_status hh_matvec(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream);

/* hh_matvec_t: y = H^^T x: y_J += V_b (U_b^T x_I), y_J += H_IJ^T x_I. The
 * dense blocks of H^T are applied from transposed copies that hh_build stores
 * beside the originals (fp64, 8 sum n_i^2 extra bytes), so the transpose runs
 * the same kernels as the forward product. Same conventions as hh_matvec. */
hh_status hh_matvec_t(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream);

/* hh_matvec_timed: one product (trans = 0: H^ x, 1: H^^T x) exactly as
 * hh_matvec / hh_matvec_t, with HIP events recorded on `stream` around each of
 * its three kernels; waits for the stream and returns the elapsed milliseconds
 * of [gather, inner products, leaf accumulation] in phase_ms (HOST, 3). */
hh_status hh_matvec_timed(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream,
                          int trans, double* phase_ms);

/* hh_matvec_batch: y_t = H_t^ x_t (Alg. 4) for `count` independent handles in
 * one pass of the kernels (one launch per phase over all handles). Every
 * handle must share io_dtype and the device, and either all or none of them
 * may hold continuum storage (HH_ENOTSUP otherwise; handles with and without
 * q43 blocks mix freely); x[t], y[t] are DEVICE pointers
 * sized for handle t (N_t x nrhs, row-major). The task tables of the last
 * batch (same handles in the same order, same nrhs) stay on the device, so a
 * repeated call only uploads the x / y descriptors on `stream` and returns
 * without waiting. Calls that overlap in time (other streams, other threads)
 * share that descriptor table and the handles' workspaces, and race. Freeing
 * a handle of the batch drops the tables. The descriptor upload is a copy from
 * pageable host memory, so this call must not be recorded into a HIP graph. */
hh_status hh_matvec_batch(const hh_handle* const* hs, int count, const void* const* x,
                          void* const* y, int64_t nrhs, void* stream);

/* Bytes of the fixed device array behind hh_matvec_noalloc (one per device). */
#define HH_NOALLOC_SCRATCH_BYTES (64u << 20)

/* hh_matvec_noalloc: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). The product of hh_matvec (trans = 0) or hh_matvec_t (trans = 1),
 * with the same kernels and bit for bit the same result, but its workspace
 * (gathered x, the nrhs coefficients of every stored column, and for nrhs = 1
 * the partial rows of the work units) lives in a fixed device array of
 * HH_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it runs
 * on until the process ends, not in the handle. The call allocates nothing and
 * never grows the handle's workspace. It needs 8 nrhs (Np + C) bytes, plus
 * 8 Q bytes when nrhs = 1, each part rounded up to 256 bytes (Np = N padded to
 * 4 rows per leaf, C = sum_b k_b = hh_stats.total_columns, Q = partial rows,
 * about 2 N at leaf 256); a product needing more returns HH_ENOTSUP with
 * nothing queued. Every call on one device shares that array and nothing in it
 * needs clearing between calls: calls in one stream order are safe, calls
 * that overlap in time on one device (other streams or threads, replays of
 * captured graphs on several streams) race and give wrong results. Arguments
 * and other errors as for hh_matvec. */
hh_status hh_matvec_noalloc(const hh_handle* h, const void* x, void* y, int64_t nrhs, int trans,
                            void* stream);

/* hh_solve: restarted GMRES (Saad & Schultz) for (H^ + shift I) x = b, or
 * (H^^T + shift I) x = b when trans != 0, with the handle's product as the
 * operator: the iterative use of the fast product that closes Sec. 5.3.
 * Krylov basis orthonormalised by classical Gram-Schmidt applied twice, least
 * squares kept triangular by Givens rotations.
 *   b, x       DEVICE, N fp64 in caller order (handle with HH_IO_F64, else
 *              HH_ENOTSUP); x holds the initial guess on entry (zero it for
 *              none) and the solution on return. b and x must not alias.
 *   shift      real diagonal shift (0 for H^ itself).
 *   rtol       stop when ||b - A x|| <= rtol ||b|| (the recurrence's residual
 *              inside a cycle, the true residual between cycles).
 *   restart    Krylov dimension per cycle, 1..1000; max_iter >= 0 products.
 *   iters      HOST, receives the number of Krylov steps (may be NULL).
 *   relres     HOST, receives ||b - A x|| / ||b|| recomputed after the last
 *              cycle (may be NULL).
 * Runs on `stream` and returns after synchronising it; allocates its basis
 * (8 N (restart + 1) bytes) for the call. */
hh_status hh_solve(const hh_handle* h, const void* b, void* x, double shift, double rtol,
                   int restart, int max_iter, int trans, int32_t* iters, double* relres,
                   void* stream);

/* One setting of the task-table sizes and its measured product time. */
typedef struct {
    int64_t unit_bytes;      /* factor bytes per single-vector accumulation unit */
    int64_t dot_task_elems;  /* stored entries per single-vector inner-product task */
    double ms;               /* median time of one y = H^ x product, milliseconds */
} hh_tuning;

/* hh_autotune: picks the task-table sizes of the single-vector product for
 * this handle by measurement: work units of 256 KiB .. 4 MiB of factor data
 * with the default inner-product tasks, then inner-product tasks of 16K ..
 * 256K stored entries with the best unit size; each setting gets new task
 * tables (host work, no change to the stored matrix) and five timed products
 * after a warm-up (median of HIP events on `stream`, synchronised). The
 * handle keeps the fastest setting (the tables of both directions are rebuilt
 * with it); pass best->unit_bytes / dot_task_elems as hh_options of later
 * builds of similar matrices to skip the search. Products of any nrhs stay
 * correct; several-RHS tiles are not affected. Allocates temporary x, y.
 *   best       HOST, receives the chosen setting (not NULL).
 *   tried      HOST array of cap entries (may be NULL): every setting timed,
 *              in order; ntried (may be NULL) receives their number.
 * Must not overlap other calls on the handle; drops the cached batch tables. */
hh_status hh_autotune(hh_handle* h, void* stream, hh_tuning* best, hh_tuning* tried,
                      int32_t cap, int32_t* ntried);

/* hh_reserve: size the product workspace for up to max_nrhs right-hand sides
 * now (products with larger nrhs allocate on first use, which is not allowed
 * under HIP graph capture). */
hh_status hh_reserve(hh_handle* h, int64_t max_nrhs);

/* ------------------------------------------------------------ inspection */

hh_status hh_get_stats(const hh_handle* h, hh_stats* out);
/* Number of blocks (low-rank, rank-0 and dense), canonical order (level, i, j). */
hh_status hh_block_count(const hh_handle* h, int64_t* count);
hh_status hh_get_block(const hh_handle* h, int64_t index, hh_block_info* out);
/* Stored factors of a low-rank block, decoded to float64 (value = stored * 2^exp):
 * U HOST m x rank, V HOST n x rank, both column-major. For a dense block U
 * receives the m x n block column-major and V is ignored. */
hh_status hh_get_block_factors(const hh_handle* h, int64_t index, double* U, double* V);
/* Tree order: perm[t] = caller index of the point at tree position t (HOST, n). */
hh_status hh_get_perm(const hh_handle* h, int64_t* perm);
int hh_io_dtype(const hh_handle* h);
int64_t hh_size(const hh_handle* h);

/* hh_free: release the handle and its device memory; NULL is a no-op. */
void hh_free(hh_handle* h);

/* ------------------------------------------------- host-only structure */

/* hh_plan_*: the tree (Sec. 2.1) and block partition (Alg. 1) alone, computed
 * on the host without a GPU; the same code hh_build uses. */
hh_status hh_plan_create(const double* points, int64_t n, int d, double eta,
                         int switch_level, int leaf_size, hh_plan** out);
hh_status hh_plan_info(const hh_plan* p, int32_t* L, int32_t* ell, int64_t* n_blocks);
/* Arrays of length n_blocks (any may be NULL): level, kind, Morton boxes i and
 * j, tree-order row range [ib, ie) and column range [jb, je). */
hh_status hh_plan_blocks(const hh_plan* p, int32_t* level, int32_t* kind, int64_t* box_i,
                         int64_t* box_j, int64_t* ib, int64_t* ie, int64_t* jb, int64_t* je);
hh_status hh_plan_perm(const hh_plan* p, int64_t* perm);
void hh_plan_free(hh_plan* p);

/* hh_quantize: the library's storage rounding on the host: out[i] = round(in[i]
 * 2^-e) 2^e with round-to-nearest-even straight from float64 to `format`
 * (HH_FMT_*, not HH_FMT_CONT), gradual underflow kept. This is the arithmetic
 * hh_build applies to every factor (e = 0 for fp64 / fp32; the build picks e
 * per factor so that the largest entry lands in [2^14, 2^15) for fp16, in
 * [1, 2) for bf16 and in [64, 128) for q43, whose magnitudes past 240 saturate
 * to 240). */
hh_status hh_quantize(const double* in, int64_t n, int format, int e, double* out);

/* hh_quantize_cont: the continuum storage rounding on the host: out[i] = the
 * nearest value (ties to even) with t fraction bits (7 <= t <= 23), fp32's
 * exponent range and gradual underflow below 2^-126; magnitudes rounding past
 * (2 - 2^-t) 2^127 become infinite. The arithmetic hh_build applies to every
 * factor of an HH_FMT_CONT block (the accessor remark of Sec. 4.3). */
hh_status hh_quantize_cont(const double* in, int64_t n, int t, double* out);

/* Message of the last failing call on this thread ("" if none). */
const char* hh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HH_H */
