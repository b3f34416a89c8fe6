/*
 * hm.h -- C ABI of the MI355X (gfx950) hierarchical-matrix product engine.
 *
 * The library computes the update  y := alpha * M * x + y  (eq. 4 of
 * Kriemann, "Floating Point Compression of Hierarchical Matrix Formats and
 * its Impact on Matrix-Vector Multiplication", Sec. 3) for a hierarchical
 * matrix M stored in one of three forms:
 *   H   (Sec. 2.2, Def. 2.3, eq. 3): dense inadmissible leaves D and
 *        low-rank admissible leaves U V^T,
 *   UH  (Sec. 2.3): shared orthonormal cluster bases W_t, X_s and a
 *        coupling matrix S per admissible leaf, M_b = W_t S_b X_s^T,
 *   H2  (Sec. 2.4): nested bases; explicit bases at leaf clusters only and
 *        transfer matrices E (rows) / F (columns) above them:
 *        W_t = [W_t0 E_t0 ; W_t1 E_t1].
 * The block structure is a block tree over a cluster tree (Def. 2.1, 2.2).
 *
 * Conventions for every call:
 *   - Every call returns an hm_status; nothing aborts or throws across the ABI.
 *     On failure hm_last_error() returns a thread-local message.
 *   - Callers own every array they pass; the library copies what it keeps.
 *     Objects returned through out-pointers are owned by the library until
 *     the matching *_free / *_destroy call.
 *   - Matrices are column-major with leading dimension = row count.
 *   - Index vectors are in original point order unless HM_CLUSTER_ORDER is
 *     given; perm[i] is the original index of cluster position i.
 *   - Device work is enqueued on the given HIP stream and never synchronises
 *     the host, except hm_upload which returns after the copy completes.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hm_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
    HM_OK = 0,
    HM_EINVAL = -1,     /* bad argument (null pointer, size, id, dtype) */
    HM_ENOMEM = -2,     /* host or device allocation failed */
    HM_EDEVICE = -3,    /* a HIP runtime call failed */
    HM_ELAYOUT = -4,    /* partition or value set inconsistent with the layout */
    HM_EBUSY = -5,      /* serving queue full */
    HM_ENOTREADY = -6   /* result not available yet */
} hm_status;

typedef enum { HM_FMT_H = 0, HM_FMT_UH = 1, HM_FMT_H2 = 2 } hm_format;

/* Storage formats.  Hardware formats (Table 1): FP8 is OCP E4M3 (no
 * infinities, max 448).  HM_VALR_AUTO picks per column the cheapest of them
 * whose measured error meets delta_i = delta / sigma_i (Sec. 4.2, eq. 6-7).
 *
 * Byte-aligned codecs of Sec. 4.1 (a stored value of B bytes; a 16-byte
 * tile row holds floor(16 / B) of them at byte offsets 0, B, 2B, ..., each
 * least significant byte first, the rest of the row zero):
 *   FPX (the table of Sec. 4.1): the leading B bytes of the FP32 (8 exponent
 *   bits) or FP64 (11 bits) encoding, rounded to nearest, ties to even:
 *   HM_FPX24 = (8, 15), HM_FPX40 = (11, 28), HM_FPX48 = (11, 36),
 *   HM_FPX56 = (11, 44) (exponent, mantissa bits); the other rows are
 *   HM_BF16 = (8, 7), HM_F32 = (8, 23) and HM_F64 = (11, 52).
 *   AFLP (HM_AFLP8 ... HM_AFLP56, B = 1 ... 7): code = sign | z (e bits) |
 *   M (m' = 8B - 1 - e bits), value = sign * 2^k * 2^(z-1) * (1 + M/2^m'),
 *   z = 0 (with M = 0) is zero.  k (per column, a power-of-two scale) is
 *   floor(log2) of the column's smallest nonzero magnitude; e (per stored
 *   matrix) is the bit length of the largest code z = floor(log2(vmax/2^k))
 *   + 1 over its columns.  M is rounded to nearest (ties to even, a carry
 *   moves to z + 1); codes beyond the largest saturate.  Widths up to 3
 *   bytes need e <= 7, wider ones e <= 10.
 * Policies (not storage formats), valid in every hm_precision field:
 *   HM_AFLP_AUTO / HM_FPX_AUTO: direct compression at eps (AFLP: width
 *   B = ceil((1 + e + m_eps) / 8), m_eps = ceil(-log2 eps); FPX: the first
 *   row with m >= m_eps) for dense, coupling and transfer matrices, and VALR
 *   over the codec's widths (the narrowest whose measured column error meets
 *   delta_i) for low-rank factors and cluster bases.  A fixed AFLP width is
 *   raised to the first width that holds the matrix's e; past 7 bytes, and
 *   for eps below 2^-52, FP64 is stored. */
typedef enum {
    HM_F64 = 0, HM_F32 = 1, HM_BF16 = 2, HM_F16 = 3, HM_FP8E4M3 = 4, HM_VALR_AUTO = 5,
    HM_FPX24 = 6, HM_FPX40 = 7, HM_FPX48 = 8, HM_FPX56 = 9,
    HM_AFLP8 = 10, HM_AFLP16 = 11, HM_AFLP24 = 12, HM_AFLP32 = 13, HM_AFLP40 = 14, HM_AFLP48 = 15,
    HM_AFLP56 = 16,
    HM_AFLP_AUTO = 17, HM_FPX_AUTO = 18
} hm_dtype;

/* number of storage dtype codes (arrays indexed by dtype; code 5 is unused) */
#define HM_NDTYPES 17

typedef enum { HM_ACC_AUTO = 0, HM_ACC_F32 = 1, HM_ACC_F64 = 2 } hm_accum;

/* hm_mvm flags */
#define HM_CLUSTER_ORDER 1u   /* x and y are already in cluster order */
#define HM_TIMING 2u          /* record HIP events around every phase kernel (hm_timing_read) */
#define HM_ADJOINT 4u         /* y := alpha * M^T * x + y (needs hm_upload_opts.adjoint) */

/* ---------------------------------------------------------------- layout */

/* Partitions (Sec. 2.2; its remark names BLR and HODLR as members of the
 * same set of matrices, obtained by the choice of clustering and
 * admissibility alone). */
#define HM_PART_STANDARD 0   /* geometric bisection, standard admissibility */
#define HM_PART_HODLR 1      /* balanced bisection, off-diagonal admissibility: t != s */
#define HM_PART_BLR 2        /* balanced bisection, one level: all pairs of leaf clusters,
                                low rank where the standard condition holds */

typedef struct {
    int32_t leaf_size;   /* a cluster with at most leaf_size points is a leaf (default 64) */
    double eta;          /* admissibility min(diam) <= eta * dist (default 2) */
    int32_t partition;   /* HM_PART_* (default HM_PART_STANDARD) */
} hm_layout_opts;

typedef struct hm_layout hm_layout;

/* Cluster tree by geometric bisection and block tree with standard
 * admissibility (Def. 2.1, 2.2), for HM_PART_STANDARD:
 *   - a cluster's box is the tight axis-aligned box of its points;
 *   - clusters larger than leaf_size split along the axis of largest extent
 *     (lowest axis on ties) at 0.5*(lo+hi); points with coordinate < mid go
 *     to son 0, keeping their order; an empty side splits at half the size;
 *   - a block (t,s) is low rank if min(diam_t^2, diam_s^2) <= eta^2 dist^2
 *     and dist^2 > 0 (squared box diameters/distance, summed x,y,z), else a
 *     dense leaf if t or s is a leaf, else it recurses over son pairs.
 * HM_PART_HODLR and HM_PART_BLR use a balanced tree instead: every cluster
 * above level d splits (along its box's axis of largest extent, lowest axis
 * on ties) into the first floor(m/2) of its points ordered by that
 * coordinate (stable) and the rest, d being the smallest depth with
 * ceil(n / 2^d) <= leaf_size (a single point is always a leaf).  HODLR then
 * makes every block (t, s) with t != s low rank; BLR recurses down to the
 * pairs of leaf clusters and makes a pair low rank where the standard
 * condition holds, dense otherwise.
 * points: n x 3 row-major float64, caller-owned, n >= 1.  opts may be NULL.
 * Deterministic: the same points give bit-identical layouts.
 * Errors: HM_EINVAL (n < 1, null, non-finite point, leaf_size < 1, eta <= 0,
 * unknown partition). */
hm_status hm_build_layout(const double* points, int64_t n, const hm_layout_opts* opts,
                          hm_layout** out);

/* Read-only view of a layout (arrays owned by the layout).  Nodes are in
 * depth-first pre-order (node 0 = root); node t covers cluster positions
 * [node_begin[t], node_end[t]).  Blocks are the block-tree leaves in
 * depth-first order (son pairs tau-son major). */
typedef struct {
    int64_t n, nnodes, nblocks;
    int32_t depth;                  /* largest node level */
    const int64_t* perm;            /* [n] original index of cluster position i */
    const int64_t* node_begin;      /* [nnodes] */
    const int64_t* node_end;        /* [nnodes] */
    const int32_t* node_level;      /* [nnodes] */
    const int32_t* node_parent;     /* [nnodes] -1 at the root */
    const int32_t* node_son0;       /* [nnodes] -1 at leaves */
    const int32_t* node_son1;       /* [nnodes] -1 at leaves */
    const int32_t* blk_tau;         /* [nblocks] row cluster */
    const int32_t* blk_sigma;       /* [nblocks] column cluster */
    const int32_t* blk_adm;         /* [nblocks] 1 = admissible (low rank) */
} hm_layout_view;

hm_status hm_layout_export(const hm_layout* layout, hm_layout_view* view);
void hm_layout_free(hm_layout* layout);

/* Structure statistics of a layout (Def. 2.1, 2.2), from the partition
 * alone: no values are needed.  Per level l (distance from the root):
 * cluster-tree nodes, dense (inadmissible) and low-rank (admissible) block
 * leaves, and the areas sum |t|*|s| those leaves cover.  The areas of all
 * leaves add up to n*n (exact cover).  Levels at or beyond
 * HM_MAX_LEVELS - 1 are counted in the last entry.
 * Errors: HM_EINVAL (null argument). */
#define HM_MAX_LEVELS 64
typedef struct {
    int64_t n, nnodes, nleaves, nblocks, ndense, nlowrank;
    int64_t ndiag;                  /* dense leaves with t == s */
    int32_t depth;                  /* largest node level */
    int32_t min_leaf, max_leaf;     /* smallest / largest leaf cluster size */
    double dense_area;              /* sum over dense leaves of |t|*|s| */
    double lowrank_area;            /* sum over admissible leaves of |t|*|s| */
    int64_t nodes_per_level[HM_MAX_LEVELS];
    int64_t dense_per_level[HM_MAX_LEVELS];
    int64_t lowrank_per_level[HM_MAX_LEVELS];
    double dense_area_per_level[HM_MAX_LEVELS];
    double lowrank_area_per_level[HM_MAX_LEVELS];
} hm_layout_info;

hm_status hm_layout_stats(const hm_layout* layout, hm_layout_info* info);

/* --------------------------------------------------------------- values */

/* float64 values of one matrix, indexed by the layout's node and block ids.
 * Entries not used by the chosen format may be NULL.  All matrices are
 * column-major.
 *   dense[b]           inadmissible b: |t| x |s|
 *   H:   rank[b], W[b] (|t| x k, orthonormal columns), sigma[b] (k),
 *        X[b] (|s| x k); the block is W diag(sigma) X^T (Sec. 4.2 form)
 *   UH:  row_rank[v], col_rank[v]; row_basis[v] (|v| x k_v) and
 *        col_basis[v] for every node; coupling[b] (k_t x k_s)
 *   H2:  row_rank, col_rank; row_basis / col_basis at leaf nodes only;
 *        row_transfer[v] = E_v (k_v x k_parent) and col_transfer[v] = F_v
 *        (k_v x k_parent) at every non-root node; coupling[b]
 *   row_sv / col_sv (optional): per-node weights of the basis columns
 *        (singular values from the basis construction), used by VALR. */
typedef struct {
    const double* const* dense;
    const int32_t* rank;
    const double* const* W;
    const double* const* sigma;
    const double* const* X;
    const int32_t* row_rank;
    const int32_t* col_rank;
    const double* const* row_basis;
    const double* const* col_basis;
    const double* const* row_transfer;
    const double* const* col_transfer;
    const double* const* row_sv;
    const double* const* col_sv;
    const double* const* coupling;
} hm_values;

/* Storage policy.  Dense leaves with t == s use diag_dtype, other dense
 * leaves dense_dtype; low-rank factors (H), cluster bases (UH) and leaf
 * bases (H2) use factor_dtype; coupling and transfer matrices use
 * coupling_dtype (direct compression, Sec. 4.1).  Stored columns in FP16
 * or FP8 carry one scale c = max(fl32(max|col| / largest finite), 2^-126);
 * codes are round-to-nearest-even of col/c, saturated (FP64/FP32/BF16: c = 1).
 * For H2 column transfers the scaled axis is the row of F (the column of
 * F^T).  The singular values of H factors are folded into the column
 * scales of W.
 * accum: HM_ACC_AUTO = float64 accumulators if eps < 1e-7 or every dtype is
 * HM_F64, else float32 accumulators (float64 dense diagonal leaves keep a
 * float64 accumulator). */
typedef struct {
    double eps;
    int32_t dense_dtype;
    int32_t diag_dtype;
    int32_t factor_dtype;
    int32_t coupling_dtype;
    int32_t accum;
} hm_precision;

typedef struct hm_matrix hm_matrix;

/* Engine options of hm_upload (NULL, or every field 0, gives the defaults).
 * None of them changes what is computed; they change how the work is cut
 * into tasks and launches, and valr_promote the storage choice.
 *   task_bytes     target stored bytes per task (one wavefront); 0 = 32768 for
 *                  float64 data and 16384 for the narrower formats, else at
 *                  least 1024 (for every format)
 *   chain_task_bytes  the same for the tasks of the dependent stages only;
 *                  0 = task_bytes when that is set, else the format's
 *                  default, doubled for matrices with at least 2048 leaf
 *                  clusters
 *   spread_dense   1 = spread the dense leaves over the dependent stages
 *                  instead of one stage on a second stream
 *   dense_grid     cap on the workgroups of that second-stream stage (0 = none)
 *   fork_after     initial fork point of that stage (see hm_tune_mvm)
 *   schedule / dense_after / spin_limit_us: see the fields below
 *   valr_promote   1 = under HM_VALR_AUTO, a format used by fewer columns of
 *                  a factor than one 16-byte tile holds is stored in the
 *                  factor's next more precise format present when that costs
 *                  no extra tile.  Such columns are stored more precisely
 *                  than their budget delta_i asks (Sec. 4.2), so the bounds
 *                  of eq. 6 and eq. 7 still hold.  0 = the paper's rule:
 *                  every column in its own cheapest format. */
typedef struct {
    int64_t task_bytes;
    int32_t spread_dense;
    int32_t dense_grid;
    int32_t fork_after;
    int32_t valr_promote;
    int32_t schedule;       /* HM_SCHED_STAGED (default) or HM_SCHED_PERSISTENT (also builds the
                               persistent queue, so hm_tune_mvm can time both), see hm_mvm */
    int32_t dense_after;    /* persistent schedule: first boundary between dependent stages from
                               which the dense near-field tasks are interleaved (see hm_tune_mvm) */
    int32_t spin_limit_us;  /* persistent schedule: bound of one dependency wait in microseconds
                               (0 = 2 000 000); a wait past it aborts the launch (hm_matrix_check) */
    int32_t tickets_per_grab; /* persistent schedule: queue items a wavefront takes per atomic
                                 (0 = 4, at most 256) */
    int32_t sync;           /* how tasks that share output rows combine them (Sec. 3.1 discusses
                               the collision problem and three remedies), for comparison:
                               HM_SYNC_OWNER (default) one owner per row cluster, split owners'
                               partial sums added in a fixed order (deterministic);
                               HM_SYNC_ATOMIC every task adds its rows with float64 atomic adds
                               (no partial sums, no reduction launches; summation order varies);
                               HM_SYNC_PRIVATE y rows are added atomically into eight private
                               copies of y, summed by one final launch (the paper's thread-local
                               copies).  Staged schedule only. */
    int32_t adjoint;        /* 1 = also upload the adjoint M^T (the remark after Alg. 3: the
                               product over block columns) for HM_ADJOINT products: every block
                               transposed, stored under the same precision policy; doubles the
                               device memory of the matrix */
    int32_t h2_levels;      /* H2 downward pass: 0 = the coupling products of every level in one
                               launch right after the upward pass (each row cluster's couplings as
                               partial sums of its coefficients), then one small launch per level
                               for the transfers (default); 1 = couplings and transfers together,
                               one launch per level.  The same products; the transfer product is
                               its own partial sum in the first, so results agree to rounding. */
    int64_t chain_task_bytes; /* target stored bytes per task of the dependent stages (every task but
                                 the dense near field's); 0 = task_bytes if set, else the format's
                                 default, doubled from 2048 leaf clusters on; else at least 1024 */
} hm_upload_opts;

#define HM_SCHED_STAGED 0
#define HM_SCHED_PERSISTENT 1
#define HM_SYNC_OWNER 0
#define HM_SYNC_ATOMIC 1
#define HM_SYNC_PRIVATE 2

/* Quantise on the host per `prec`, pack into level- and row-cluster-ordered
 * streams and copy to the current HIP device.  opts may be NULL (defaults).
 * Blocks whose value pointers are required but NULL, ranks that are
 * negative or exceed the block size, non-finite values and out-of-range
 * options give HM_EINVAL / HM_ELAYOUT.  The layout must stay alive as long
 * as the matrix.  Returns after the copy has completed. */
hm_status hm_upload(const hm_layout* layout, int32_t format, const hm_values* values,
                    const hm_precision* prec, const hm_upload_opts* opts, hm_stream_t stream,
                    hm_matrix** out);
void hm_matrix_free(hm_matrix* m);

/* Storage statistics of an uploaded matrix (bytes as stored on the device). */
typedef struct {
    int64_t n, nblocks, ndense, nlowrank;
    int64_t bytes_dense, bytes_factors, bytes_coupling, bytes_transfer, bytes_scales;
    int64_t bytes_meta, bytes_workspace;
    int64_t bytes_per_dtype[HM_NDTYPES];     /* stored matrix data by dtype (16-byte tiles) */
    int64_t entries_per_dtype[HM_NDTYPES];   /* stored matrix entries by dtype, each source matrix
                                                once, without tile padding */
    int64_t sum_rank;               /* sum of block ranks (H) or basis ranks (UH/H2) */
    int32_t max_rank;
    int32_t accum;                  /* resolved accumulation (HM_ACC_F32 / HM_ACC_F64) */
    int32_t nlaunch;                /* kernel launches per hm_mvm (persistent schedule: 2) */
    int64_t nowners, nitems, ntasks; /* single-vector plan: output owners, stored slices, wavefront tasks */
    double algorithmic_bytes;       /* bytes one hm_mvm moves: stored data (16-byte tiles, padding
                                       included) + scales + vectors + coefficients + plan metadata */
    double method_bytes;            /* bytes the product itself needs: every stored entry once at its
                                       element size (codecs: B bytes), a float32 scale per FP16/FP8/
                                       AFLP column, x read,
                                       y read and written, every coefficient written and read once */
} hm_stats;

hm_status hm_matrix_stats(const hm_matrix* m, hm_stats* s);

/* Host-only dry run of hm_upload: quantise and pack exactly as hm_upload
 * would (same storage choices, same plan), fill *out with the statistics
 * of the resulting matrix and release everything.  Touches no device; the
 * errors are those of hm_upload.  Used to inspect the per-dtype storage
 * that VALR (Sec. 4.2) selects before committing device memory. */
hm_status hm_plan_stats(const hm_layout* layout, int32_t format, const hm_values* values,
                        const hm_precision* prec, const hm_upload_opts* opts, hm_stats* out);

/* ------------------------------------------------------------- products */

/* y := alpha * M * x + y, or with HM_ADJOINT y := alpha * M^T * x + y (the
 * transposed matrix uploaded with hm_upload_opts.adjoint; its blocks are
 * the transposes of M's, stored under the same policy: for FP64, FP32 and
 * BF16 storage exactly the transpose of M as stored; FP16/FP8 columns take
 * the range scales of the transposed columns).  x, y: device float64 arrays
 * of length n (caller-owned, e.g. PyTorch tensors), x != y.  Enqueued on
 * `stream`; calls on one matrix must not overlap in time (they share its
 * workspace).
 *
 * Schedules (the arithmetic and its order are the same, results are
 * bitwise identical):
 *   HM_SCHED_STAGED      one launch per stage of the data flow of Sec. 3
 *                        (forward transform / upward pass, couplings,
 *                        downward pass level by level, leaf rows), the
 *                        dense near field on a second stream, a final
 *                        reduction of split output rows;
 *   HM_SCHED_PERSISTENT  a gather launch, then one launch whose wavefronts
 *                        take the same tasks from a ticket queue in a
 *                        topological order; each task waits only for the
 *                        owners whose outputs it reads.  Every wait is
 *                        bounded (spin_limit_us): past it the launch aborts
 *                        and records an error for hm_matrix_check. */
hm_status hm_mvm(hm_matrix* m, double alpha, const double* x, double* y, uint32_t flags,
                 hm_stream_t stream);

/* Waits for the device (hipDeviceSynchronize) and reports whether a
 * persistent-schedule launch of this matrix was aborted since the last call
 * (a dependency wait exceeded its bound; the products of that launch are
 * wrong).  Clears the record.  Errors: HM_EINVAL, HM_EDEVICE (aborted, or a
 * HIP call failed). */
hm_status hm_matrix_check(hm_matrix* m);

/* Many right-hand sides (the paper's product applied to every column of a
 * block of vectors, eq. 4 per column): for i < nmat,
 *     Y_i := alpha * M_i * X_i + Y_i,
 * X_i, Y_i device arrays of n_i x nrhs[i] values, column-major with leading
 * dimensions ldx[i], ldy[i] >= n_i, in float64 (vec_dtype HM_F64) or
 * float32 (HM_F32).  mats, X, ldx, nrhs, Y, ldy are host arrays of nmat
 * entries; the vectors are caller-owned and X_i must not overlap Y_i.
 * nrhs[i] in [0, HM_MAX_NRHS]; 0 skips the entry.  One matrix may appear
 * only once per call.  flags: HM_CLUSTER_ORDER and HM_TIMING as for hm_mvm.
 * A single float64 column runs the hm_mvm kernels; wider blocks run the
 * matrix-core path (16x16x4 MFMA, float32 products and accumulation, or
 * float64 throughout for float64 data and for matrices that accumulate in
 * float64).  Each matrix keeps a workspace sized for the widest block seen;
 * growing it synchronises the device and allocates, so the first call at a
 * new width must not be inside a graph capture, and it invalidates every
 * graph captured earlier from a product of that matrix (hm_graph_launch
 * then refuses them).  Enqueued on `stream`;
 * calls on one matrix must not overlap in time.
 * Errors: HM_EINVAL (arguments), HM_ENOMEM (workspace), HM_EDEVICE. */
#define HM_MAX_NRHS 1024
hm_status hm_mvm_batch(hm_matrix* const* mats, int32_t nmat, double alpha, const void* const* X,
                       const int64_t* ldx, const int32_t* nrhs, void* const* Y, const int64_t* ldy,
                       int32_t vec_dtype, uint32_t flags, hm_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * products as hm_mvm_batch, bitwise, with every many-RHS workspace taken
 * from one library-owned device array of HM_NOALLOC_SCRATCH_BYTES (64 MiB)
 * instead of the matrices' own workspaces.  The call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.
 *   - Limit: the workspaces of one call (for matrix i, about
 *     (12 * (coefficient entries + n_i) + 8 * (n_i + partial sums)) * R_i
 *     bytes, R_i = nrhs[i] rounded up to 16 or a multiple of 32) must fit the
 *     array together; a larger call fails with HM_EINVAL before launching.
 *   - Every matrix with more than one column (or float32 vectors) needs its
 *     many-RHS plan already built (hm_tune_batch, or one earlier
 *     hm_mvm_batch call), else HM_EINVAL.  Single float64 columns run the
 *     hm_mvm kernels on the matrix's own workspace, as in hm_mvm_batch.
 *   - HM_TIMING is not accepted (timing events are allocated).
 *   - Each GPU has one array, shared by every call on it and holding the
 *     last call's contents; each call clears the part it uses before its
 *     products.  Calls that overlap in time on one GPU (on different streams
 *     or from different threads) race on the array and give wrong results:
 *     serialise them.
 * Arguments, layouts and the other errors are those of hm_mvm_batch. */
#define HM_NOALLOC_SCRATCH_BYTES (64ll << 20)
hm_status hm_mvm_batch_noalloc(hm_matrix* const* mats, int32_t nmat, double alpha, const void* const* X,
                               const int64_t* ldx, const int32_t* nrhs, void* const* Y, const int64_t* ldy,
                               int32_t vec_dtype, uint32_t flags, hm_stream_t stream);

/* Autotuner of the many-right-hand-side path.  The engine's two free
 * parameters are the column-chunk size of a task (bytes of stored data per
 * 64-row group: 64 KiB ... 1 MiB) and the number of 16-wide right-hand-side
 * blocks one wave carries (1 or 2, per stage).  For every chunk size
 * hm_tune_batch times each stage with both block counts (`reps` event-timed
 * products of an nrhs-wide zero block, allocated and freed here), keeps the
 * faster per stage, times that combination, and keeps the fastest chunk
 * size for this matrix.  It allocates,
 * synchronises and rebuilds the plan: call it outside graph capture, before
 * creating graphs of the matrix (graphs of its many-RHS products captured
 * earlier are invalidated, as when the workspace grows).  Results of later products may differ from
 * earlier ones in rounding (a different summation order), within the
 * accumulation tolerance. */
typedef struct {
    int64_t target_bytes;   /* chosen column-chunk size */
    int32_t nrb;            /* blocks per wave chosen for the stage with the most data */
    double ms;              /* its mean time per product */
    int32_t ncandidates;    /* candidates timed */
} hm_tune_result;
hm_status hm_tune_batch(hm_matrix* m, int32_t nrhs, int32_t vec_dtype, int32_t reps, hm_stream_t stream,
                        hm_tune_result* out);

/* Autotuner of the single-vector product.  Staged schedule: the dependent
 * chain of stages (cluster-basis and coupling passes) runs on the caller's
 * stream and the dense near-field stage, which reads only x, on a second
 * stream; the free parameter is the fork point, how many chain stages
 * complete before the dense stage starts (0 = right after x is gathered).
 * Persistent schedule: the free parameter is dense_after, the first boundary
 * between chain stages from which the dense tasks are interleaved into the
 * queue.  In the staged schedule the dense stage may also run as two
 * launches on the second stream: its first dense_split tasks from the fork
 * point, the rest once fork2 chain stages are done (after the first part);
 * the tuner tries split fractions 1/4, 1/2, 3/4 at later second fork
 * points.  Every fork point is timed with the upload's dense_grid and with
 * caps of 1, 2 and 3 workgroups per compute unit on the dense stage; the
 * chosen cap replaces dense_grid.  hm_tune_mvm times every candidate of both schedules (`reps`
 * replays of a captured graph of the product on a zero vector, allocated and
 * freed here; a matrix uploaded with HM_SCHED_STAGED has no persistent
 * candidates) and keeps the fastest for this matrix.  No candidate changes
 * the arithmetic: products are bitwise identical for every choice.  It
 * allocates and synchronises: call it outside graph capture, before
 * creating graphs of the matrix (graphs keep the schedule they were
 * captured with).  Errors: HM_EINVAL, HM_ENOMEM, HM_EDEVICE. */
typedef struct {
    int32_t fork_after;     /* staged schedule: chain stages completed before the dense stage starts */
    int32_t ncandidates;    /* candidates timed */
    double ms;              /* mean time per product of the chosen candidate */
    double ms_first;        /* ... of the staged schedule at fork point 0 */
    int32_t schedule;       /* chosen schedule (HM_SCHED_*) */
    int32_t dense_after;    /* persistent schedule: chosen interleave point */
    double ms_staged;       /* best staged candidate */
    double ms_persistent;   /* best persistent candidate (0 if none) */
    int32_t fork2;          /* staged schedule: chain stages completed before the second part of the
                               dense stage starts (meaningful when dense_split > 0) */
    int32_t dense_split;    /* staged schedule: dense tasks in the first part (0 = one launch) */
    int32_t dense_grid;     /* staged schedule: workgroup cap of the dense stage's launches (0 = none) */
} hm_tune_mvm_result;
hm_status hm_tune_mvm(hm_matrix* m, int32_t reps, hm_stream_t stream, hm_tune_mvm_result* out);

/* A product captured into a HIP graph: the kernels of one hm_mvm call with
 * fixed (alpha, x, y, flags) recorded once and replayed with one launch.
 * Replays read x and update y in place exactly like hm_mvm; results are
 * bitwise identical to the eager call.  The matrix must outlive the graph.
 * The graph records no memset nodes.  Errors: HM_EINVAL, HM_EDEVICE. */
/* Sets the single-vector schedule of a matrix without timing anything:
 * HM_SCHED_STAGED with param = fork point (0 ... number of dependent
 * stages; the dense stage as one launch), or HM_SCHED_PERSISTENT with param = dense_after (any value >= 0;
 * a matrix uploaded with HM_SCHED_STAGED has no persistent queue).  Changes
 * no arithmetic.  Synchronous (the queue order is copied); not inside graph
 * capture.  Errors: HM_EINVAL, HM_ELAYOUT, HM_EDEVICE. */
hm_status hm_set_schedule(hm_matrix* m, int32_t schedule, int32_t param);

/* Staged schedule: run the dense stage as two launches on the second stream,
 * its first `first_tasks` tasks from the fork point and the rest once `fork2`
 * dependent stages are done (first_tasks = 0: one launch).  The dense tasks
 * are independent, so the products are bitwise identical for every choice;
 * hm_tune_mvm picks these values by timing.  Not inside graph capture
 * (graphs keep the schedule they were captured with).  Errors: HM_EINVAL
 * (negative values, or first_tasks not below the dense stage's tasks). */
hm_status hm_set_dense_split(hm_matrix* m, int32_t fork2, int32_t first_tasks);

typedef struct hm_graph hm_graph;
hm_status hm_graph_create(hm_matrix* m, double alpha, const double* x, double* y, uint32_t flags,
                          hm_stream_t stream, hm_graph** out);
/* The same for one hm_mvm_batch call (fixed matrices, blocks and alpha).
 * The matrices' many-RHS workspaces are sized before the capture, so the
 * recorded work allocates nothing and holds no memset nodes. */
hm_status hm_graph_create_batch(hm_matrix* const* mats, int32_t nmat, double alpha, const void* const* X,
                                const int64_t* ldx, const int32_t* nrhs, void* const* Y, const int64_t* ldy,
                                int32_t vec_dtype, uint32_t flags, hm_stream_t stream, hm_graph** out);
/* Replays a graph.  Graphs hold device addresses of the matrices' buffers:
 * a graph whose matrices have since replaced a many-RHS workspace or plan
 * (a wider hm_mvm_batch, hm_tune_batch) is refused with HM_EINVAL before
 * anything is launched; capture it again. */
hm_status hm_graph_launch(hm_graph* g, hm_stream_t stream);
void hm_graph_free(hm_graph* g);

/* Per-phase kernel timing.  Every hm_mvm (or hm_mvm_batch) call made with HM_TIMING records a
 * HIP event pair on its stream around each phase's main kernel; this call
 * waits for the recorded events, returns the accumulated times and clears
 * them.  The phases of the single-vector plan come first, then those of
 * the many-right-hand-side plan (empty until hm_mvm_batch has run a block
 * wider than one float64 column).  out[i] for i < min(cap, number of
 * phases); *nphase = number of phases.  Names are owned by the matrix.
 * algorithmic_bytes is what a single-vector phase kernel must move per
 * launch: its stored matrix data, the scales and distinct input elements it
 * reads, and the outputs it writes. */
typedef struct {
    const char* name;
    double ms_total;
    int64_t launches;
    double algorithmic_bytes;
    int32_t ntasks;
    int32_t nowners;
    int64_t data_bytes;      /* stored matrix bytes its tasks stream per launch */
    int64_t data_entries;    /* stored matrix entries streamed (tile padding included) */
    int32_t nrhs;            /* padded block width of the timed launches (1 = single vector);
                                launches of different widths are not mixed: timing
                                an hm_mvm_batch call discards pending hm_mvm timings */
    double method_bytes;     /* algorithmic_bytes without tile padding and task descriptors */
} hm_phase_timing;

hm_status hm_timing_read(hm_matrix* m, hm_phase_timing* out, int32_t cap, int32_t* nphase);

/* --------------------------------------------------------------- serving */

/* A request loop over resident matrices (continuous batching).  A server
 * owns one scheduler thread, two HIP streams, a device arena of mem_budget
 * bytes for request blocks and a pinned host staging arena of the same
 * size.  Requests wait in FIFO order; the scheduler repeatedly forms a
 * launch group from the queued requests whose matrix is not in flight,
 * concatenating the columns of requests for the same matrix into one block,
 * as long as slots (max_slots requests in flight) and arena memory allow
 * (memory admission).  A group is copied in, multiplied with the
 * many-right-hand-side engine (hm_mvm_batch's merged launches) and copied
 * out on one stream while the next group forms and runs on the other, so
 * requests that arrive while others run join the next launch.
 *
 * Every product runs the same per-column arithmetic whatever the group:
 * a request's result is bitwise the same alone and in any mix (alpha is
 * applied on the host after the device product with alpha = 1).
 *
 * Matrices stay owned by the caller and must outlive the server.  fake = 1
 * runs the scheduler without a device (dry runs and tests): products are not
 * computed and results are zero, a group "runs" for fake_us microseconds. */
typedef struct {
    int64_t mem_budget;     /* device bytes for request blocks (and pinned host staging) */
    int32_t max_slots;      /* requests in flight at most (> 0) */
    int32_t max_queue;      /* queued requests at most; submit returns HM_EBUSY beyond */
    int32_t max_cols;       /* columns per matrix and launch group at most, and the widest request */
    int32_t fake;           /* 1 = no device work (see above) */
    int32_t fake_us;        /* duration of a fake launch group */
} hm_serve_opts;

typedef struct {
    double queue_ms;        /* submit -> admitted into a launch group */
    double run_ms;          /* admitted -> results copied out */
    double latency_ms;      /* submit -> done */
    int64_t group_id;       /* launch group that ran it */
    int32_t group_requests; /* requests in that group */
    int32_t group_cols;     /* columns of its matrix in that group */
} hm_req_stats;

typedef struct {
    int64_t submitted, completed, groups;
    int64_t peak_arena_bytes;   /* device arena high-water mark */
    int32_t peak_inflight;      /* requests in flight at most */
    int32_t max_group_requests; /* largest launch group */
} hm_serve_stats;

typedef struct hm_server hm_server;
hm_status hm_serve_create(const hm_serve_opts* opts, hm_server** out);
/* Register a resident matrix (its many-RHS workspace is sized for max_cols
 * here, so serving never allocates); *matrix_id identifies it in
 * hm_serve_submit. */
hm_status hm_serve_register(hm_server* s, hm_matrix* m, int32_t* matrix_id);
/* Register a placeholder of n rows for a fake server (no matrix). */
hm_status hm_serve_register_shape(hm_server* s, int64_t n, int32_t* matrix_id);
/* Y_host := alpha * M * X_host.  X_host, Y_host: host float64 arrays of
 * n x nrhs values, column-major (leading dimension n), caller-owned and
 * valid until hm_serve_poll reports the ticket done; nrhs in
 * [1, max_cols] (wider: HM_EINVAL).  Non-blocking; HM_EBUSY when max_queue
 * requests wait, HM_ENOMEM when the request could never fit mem_budget. */
hm_status hm_serve_submit(hm_server* s, int32_t matrix_id, double alpha, const double* X_host, int32_t nrhs,
                          double* Y_host, uint64_t* ticket);
/* Non-blocking.  *done = 1 once Y_host holds the result (the ticket is then
 * released and *st, if not NULL, filled); 0 while queued or running.
 * Unknown or released tickets give HM_EINVAL; a failed product returns its
 * error status (and releases the ticket). */
hm_status hm_serve_poll(hm_server* s, uint64_t ticket, int32_t* done, hm_req_stats* st);
hm_status hm_serve_stats_read(hm_server* s, hm_serve_stats* out);
/* Waits for every submitted request, then stops the thread and frees all. */
void hm_serve_destroy(hm_server* s);

/* Host-side helper used by tests: round float64 values to `dtype` exactly as
 * hm_upload does (scale already applied); writes float64 results.  Hardware
 * formats and FPX codes only (AFLP needs a whole column: hm_codec_column). */
hm_status hm_round_host(int32_t dtype, const double* in, double* out, int64_t count);

/* Host-side codec of one column exactly as hm_upload stores it (Sec. 4.1).
 * dtype: a storage format, or HM_AFLP_AUTO / HM_FPX_AUTO with eps > 0 (direct
 * compression).  ebits: the AFLP exponent width to use (<= 0: the column's
 * own).  col: m float64 values (host).  On return stored[i] is the value the
 * product multiplies, codes[i] (may be NULL) the B-byte code word (FP64 and
 * the hardware formats: their bit pattern), and info[0..3] = stored dtype,
 * bytes per value, AFLP e (0 otherwise), AFLP scale exponent k (0 otherwise).
 * HM_EINVAL: bad dtype, null pointers, non-finite data, an AFLP width that
 * cannot hold the requested e. */
hm_status hm_codec_column(int32_t dtype, double eps, int32_t ebits, const double* col, int64_t m, double* stored,
                          uint64_t* codes, int32_t* info);

const char* hm_last_error(void);
const char* hm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H */
