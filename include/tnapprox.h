/*
 * tnapprox.h - C ABI of the MI355X density-matrix approximate contraction.
 *
 * The library approximately contracts a closed tensor network to a scalar Z along
 * a caller-given contraction path (the inputs of the paper's partitioned_contract,
 * section 4.2: a network with its data, a partition and a path over it; the output
 * is the contraction value, reported as ln|Z| as in the experiments of section 8).
 *
 * Consecutive path slices are fused env_size at a time into partitions; the path
 * over partitions is maximally unbalanced (one partition absorbed per step). After
 * each absorption the intermediate is compressed into an MPS (the MPS tree of the
 * appendix on embedding trees) by the density-matrix algorithm (Algorithm
 * density_matrix_alg with the memoised density matrices of Eq. dm_cache): every
 * density matrix L = C R C^T is diagonalised and its leading eigenvectors, at most
 * max_rank of them, are applied as projectors along the path.
 *
 * All entry points return an int status (TN_OK = 0). Nothing throws across the
 * ABI. Host pointers are read during the call only; the caller keeps ownership.
 * A handle must not be used by two threads at once; distinct handles may run on
 * distinct threads and streams.
 */
#ifndef TNAPPROX_H
#define TNAPPROX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TN_OK = 0,
  TN_EINVAL = 1,    /* malformed network, path or argument (message via tn_last_error) */
  TN_ENOMEM = 2,    /* device or host allocation failed */
  TN_EDEVICE = 3,   /* a HIP runtime call failed, or no usable gfx950 device */
  TN_ENUMERIC = 4,  /* an input tensor holds a non-finite value */
  TN_EUNSUPPORTED = 5 /* valid input outside this build's limits (e.g. a density
                         matrix larger than 512 x 512, or an intermediate of 2^31
                         elements or more) */
};

/* One input tensor: host memory, row-major FP64, dims[order]. order 0 is a scalar. */
typedef struct {
  int32_t order;
  const int64_t *dims;
  const double *data;
} tn_tensor;

/* Edge: mode m0 of tensor t0 is contracted with mode m1 of tensor t1 (t0 != t1).
 * Every mode of every tensor must appear in exactly one edge (closed networks). */
typedef struct {
  int32_t t0, m0, t1, m1;
} tn_edge;

/* Contraction path: n_slices ordered slices in CSR form. slice_ptr has n_slices+1
 * entries; slice_vertices[slice_ptr[i] .. slice_ptr[i+1]) lists slice i's tensors.
 * The slices must partition the tensor set. */
typedef struct {
  int32_t n_slices;
  const int32_t *slice_ptr;
  const int32_t *slice_vertices;
} tn_path;

typedef enum {
  TN_FP64 = 0,          /* every contraction in FP64 on the FP64 matrix cores */
  TN_SPLIT_BF16X3 = 1,  /* the contractions that build right environments and density
                           matrices (Eq. dm_cache and the density matrix definition) run on
                           the BF16 matrix cores: each operand scaled by a power of two to
                           max |x| in [1/2, 1), split into three BF16 parts, the six part
                           products of order <= 2 accumulated in FP32. Their rounding only
                           moves the kept subspaces. The main chain (projector application,
                           the carried block, closing contractions), the eigensolve,
                           rescaling and log accumulation stay FP64. */
  TN_SPLIT_FP16X3 = 2,  /* the same with FP16 parts on the FP16 matrix cores */
  TN_SPLIT_BF16X3_ALL = 3, /* BF16 x3 split on every contraction, the main chain included */
  TN_SPLIT_FP16X3_ALL = 4  /* FP16 x3 split on every contraction */
} tn_precision;

typedef enum {
  TN_EIG_EXACT = 0,     /* full symmetric eigensolve of every density matrix */
  TN_EIG_LEARNED = 1    /* MLP warm start + subspace iteration, exact solve as fallback */
} tn_eig_mode;

typedef enum {
  TN_TRIDIAG_AUTO = 0,  /* tridiagonal eigensolve by divide and conquer for density matrices
                           of order up to 128 (Cuppen's tearing, eigenvectors from the roots by
                           the Loewner formula of Gu and Eisenstat), implicit QL above */
  TN_TRIDIAG_QL = 1     /* implicit QL with Wilkinson shifts for every order */
} tn_tridiag;

typedef struct tn_model_s *tn_model;      /* warm-start MLP weights on the device */
typedef struct tn_dataset_s *tn_dataset;  /* harvested (features, leverage) rows on the device */

/* Options; pass NULL for the defaults (FP64, exact eigensolve, tau_rel = 1e-12,
 * tau_deg = 0.1, the null stream). The rank rule (leading_eigenvectors of Algorithm
 * density_matrix_alg, which leaves ties and numerical zeros open): keep at most
 * max_rank eigenvectors, drop eigenvalues <= tau_rel * w1, and never cut where the
 * spectrum does not separate: while w_k - w_{k+1} <= tau_deg * w_k and w_{k+1} exceeds
 * 0.1 * tau_rel * w1, the cut moves up by one. With the defaults every cut is fixed by
 * FP64 arithmetic (a cut at relative gap g moves the result by about eps / g under the
 * backward error of any FP64 eigensolver). */
typedef struct {
  int32_t precision;      /* tn_precision */
  int32_t eig;            /* tn_eig_mode */
  double residual_tol;    /* learned mode: accepted max ||L x - theta x|| / theta over the kept
                             Ritz pairs (1e-6) */
  double tau_rel;         /* eigenvalues <= tau_rel * w1 are dropped */
  double tau_deg;         /* no cut where w_k - w_{k+1} <= tau_deg * w_k (see above) */
  void *hip_stream;       /* hipStream_t the work is queued on (NULL = null stream) */
  tn_model model;         /* learned mode: the MLP that ranks the warm-start columns */
  int32_t gemm_config[3]; /* FP64 contraction block shape for ops of <= 16, <= 32 and more
                             rows: 0 = built-in, k = 1..6 the k-th of 16x512/k8, 16x256/k16,
                             32x128/k32, 32x128/k16, 64x64/k32, 64x64/k16 (the autotuner's
                             choices, paper_2406_09769_amd/autotune.py) */
  int32_t chunks;         /* > 1: the persistent launch of a batch runs as this many
                             launches, each over the next part of every network's op list
                             (eager launches, same results bit for bit); 0 or 1: one launch,
                             replayed from a captured HIP graph */
  void (*progress)(void *ctx, int32_t done, int32_t total); /* chunks > 1: called on the host
                             after each part has finished (may be NULL) */
  void *progress_ctx;     /* passed to progress */
  int32_t tridiag;        /* tn_tridiag: solver of the tridiagonal eigenproblem in the exact
                             eigensolve (both reach the accuracy of a backward-stable FP64
                             solve; the kept subspaces agree to rounding) */
} tn_options;

/* Result of one contraction. log_abs = ln|Z| (natural log), sign in {-1, 0, +1};
 * Z == 0 gives sign 0 and log_abs = -inf. */
typedef struct {
  double log_abs;
  int32_t sign;
  int32_t _pad;
  double seconds;         /* device time of the call (HIP events) */
  int64_t flops;          /* algorithmic flops of the executed contractions (sum 2mnk) */
  int64_t eig_flops;      /* nominal eigensolver flops (9 n^3 per density matrix) */
  int64_t n_eig;          /* density matrices diagonalised */
  int64_t n_fallback;     /* keep() fallbacks (all eigenvalues below the floors) */
  double max_residual;    /* learned mode: largest accepted relative subspace residual */
  int64_t n_learned;      /* learned mode: density matrices solved by the warm start */
  int64_t split_flops;    /* the part of flops run in 16-bit parts by a split form (each such
                             contraction issues six 16-bit matrix products per FP64 one) */
} tn_result;

typedef struct tn_net_s *tn_net;

/* Copy a closed network to the device. Validates: t0 != t1, every mode used exactly
 * once, dims agree across each edge, dims >= 1, data finite (TN_ENUMERIC
 * otherwise). On success *out owns the device copy until tn_destroy. */
int tn_create(const tn_tensor *tensors, int32_t n_tensors, const tn_edge *edges,
              int32_t n_edges, tn_net *out);

/* Approximate ln|Z| of net along path (section 4.2 with the MPS ansatz), keeping at
 * most max_rank eigenvectors per density matrix (max_rank >= 1, env_size >= 1).
 * Blocks until the result is on the host. Plans are cached on the handle per
 * (path, max_rank, env_size). */
int tn_contract_approx(tn_net net, const tn_path *path, int32_t max_rank,
                       int32_t env_size, const tn_options *opt, tn_result *out);

/* The same for n networks in one persistent launch (one workgroup per network;
 * uneven sizes and mixed max_rank / env_size allowed). paths[i], max_ranks[i] and
 * env_sizes[i] belong to nets[i]; outs has n entries. A handle may appear once. */
int tn_contract_approx_batch(const tn_net *nets, const tn_path *paths,
                             const int32_t *max_ranks, const int32_t *env_sizes, int32_t n,
                             const tn_options *opt, tn_result *outs);

/* tn_contract_approx for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree or allocating library routine. The op list, index tables,
 * launch descriptor and workspace go into a static device array of 256 MiB that each
 * GPU the library runs on holds from the library's load until the process ends (its
 * address is looked up once per device, on the first call there). The network's
 * tensors and result scalars are the handle's, allocated by tn_create; the plan is
 * built on the host on first use and cached on the handle as usual.
 * Same arguments, result and numbers as tn_contract_approx (the same kernels on the
 * same op list; tn_result.seconds is host wall time of the launch here).
 * TN_EUNSUPPORTED: the plan needs more than 256 MiB of scratch, or has contractions
 * large enough to run over the whole chip (those need the grid scratch of the
 * allocating entry point). Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents (nothing in it needs clearing: every op writes what later
 * ops read); calls that overlap on one GPU, from any thread or stream, race. */
int tn_contract_approx_noalloc(tn_net net, const tn_path *path, int32_t max_rank,
                               int32_t env_size, const tn_options *opt, tn_result *out);

/* ---------------------------------------------------------------- learned warm start
 * The learned eigensolve (TN_EIG_LEARNED) starts subspace iteration from the columns
 * of a density matrix L that a small MLP ranks highest, computed row by row from
 * bond-local features (diagonal and row weight of L, position of the row's bond and
 * leaf index, size). It accepts the Ritz vectors when every kept residual satisfies
 * ||L x - theta x|| <= residual_tol * theta and otherwise falls back to the exact
 * solve (tn_result.n_learned counts the accepted warm starts). Training data come
 * from the method itself: tn_harvest runs an exact
 * contraction and records, for every row of every density matrix, its 8 features
 * and its leverage in the kept subspace (sum over kept vectors of U_ij^2). */

/* A model with Glorot-uniform layers and zero biases drawn from splitmix64(seed). */
int tn_model_create(uint64_t seed, tn_model *out);
/* Copy n = 1377 weights in (layout W1[8][32], b1[32], W2[32][32], b2[32], W3[32], b3). */
int tn_model_set(tn_model m, const float *w, int64_t n);
int tn_model_get(tn_model m, float *w, int64_t n);
/* Mean squared error and its gradient for the given rows (rows <= 128, X row-major
 * rows x 8, y rows), computed by the device training kernel without an update. */
int tn_model_grad(tn_model m, const float *X, const float *y, int32_t rows, float *grad, double *loss);
/* steps Adam updates (lr) on minibatches of `batch` rows (<= 128) drawn from ds with
 * splitmix64(seed); *final_loss is the loss of the last minibatch. */
int tn_model_train(tn_model m, tn_dataset ds, int32_t steps, int32_t batch, double lr, uint64_t seed,
                   double *final_loss);
void tn_model_destroy(tn_model m);

int tn_dataset_create(int64_t capacity_rows, tn_dataset *out);
/* Rows recorded so far (capped at the capacity). */
int tn_dataset_size(tn_dataset ds, int64_t *rows);
int tn_dataset_read(tn_dataset ds, float *X, float *y, int64_t rows);
void tn_dataset_destroy(tn_dataset ds);
/* Exact FP64 contraction that also appends training rows to ds. */
int tn_harvest(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size, tn_dataset ds,
               tn_result *out);

/* Structural plan for inspection and testing: writes a JSON text with, per
 * partition, the leaf edges in order and the position of every tensor of the
 * union network. Needs no device. *len is the buffer size on input and the
 * length needed (including the terminating 0) on output. */
int tn_plan_json(const int64_t *dims_flat, const int32_t *orders, int32_t n_tensors,
                 const tn_edge *edges, int32_t n_edges, const tn_path *path,
                 int32_t env_size, char *buf, int64_t *len);

void tn_destroy(tn_net net);

/* Static text for a status code. */
const char *tn_error_string(int status);

/* Text of the last error raised on the calling thread ("" if none). */
const char *tn_last_error(void);

/* ---------------------------------------------------------------- diagnostics
 * Used by the kernel tests; each runs one device op of the contraction program on
 * host data (copied in and out) and blocks. */

/* Plan statistics for (path, max_rank, env_size) on net: stats[0..8] = op count,
 * index-table entries, workspace doubles, GEMM flops (sum 2mnk), eigensolver flops
 * (9 n^3 per density matrix and 4 m c q per QR factorisation), density matrices,
 * largest density-matrix dimension, ops run over the whole chip (in a network with an
 * op whose output exceeds 2^21 elements: every contraction or rescaling with at least
 * 2^13 output elements and every contraction of at least 2^24 flops; a network with none
 * runs in one workgroup's pass), and vertices that take the QR-SVD branch of Algorithm
 * density_matrix_alg (open size above the crossing size: C = Q R, the leading
 * eigenvectors of R R_k R^T mapped back through Q, instead of forming C R_k C^T). */
int tn_plan_stats(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size,
                  int64_t *stats);

/* C (M x N, row-major) = A B with A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn],
 * through the contraction GEMM in the given tn_precision (FP64 matrix cores, or the
 * split BF16 / FP16 products). lo_split sets the inner size of the two-level
 * row/column index maps. chip_wide = 0 runs the product in one workgroup, as a
 * network's pass does; nonzero runs it over the whole chip with the launch a
 * contraction too large for one workgroup gets. */
int tn_debug_gemm(const double *A, int64_t sam, int64_t sak, const double *B, int64_t sbk,
                  int64_t sbn, double *C, int32_t M, int32_t N, int32_t K, int32_t lo_split,
                  int32_t precision, int32_t chip_wide);

/* U (n x ucols, row-major) = the kept leading eigenvectors of (L + L^T)/2 (n x n),
 * zero columns past the kept rank, under opt's tau_rel and tau_deg (NULL: defaults).
 * n <= 512 (orders above 128 are solved in global scratch). rest = 0: plain rows;
 * rest > 0: rows are (bond, leaf) pairs with leaf
 * dimension rest (must divide n), the layout the learned warm start reads its row
 * features from. With opt->eig = TN_EIG_LEARNED and opt->model set, the warm start is
 * tried first, as in a contraction. stats (8 entries, may be NULL): no eigenvalue
 * survived the rank rule (0/1), warm start accepted (0/1), kept rank, and the four
 * rejection counters of tn_profile_last entries 9-12, then 0. */
int tn_debug_eig(const double *L, int32_t n, int32_t ucols, int32_t rest, const tn_options *opt, double *U,
                 int64_t *stats);

/* Device time of the last contraction of net, split by op kind: seconds_by_kind[k]
 * for k = 1 GEMM, 2 eigensolve, 3 rescale, 4 closing scalar, 5 identity; inside the
 * eigensolve, 0 = tridiagonal reduction, 6 = QL iteration, 7 = ordering and
 * back-transformation; entry 8 holds the number of QL rotations; entries 9-12 count
 * the learned warm starts handed to the exact solve because the subspace would not be
 * smaller than the matrix, every start column was dependent, the weight outside the
 * subspace could change the cut, or a Ritz residual was too large; entries 13-16 split
 * the time of the warm starts (accepted or not) into scoring and start basis, products
 * with L, the small eigensolve, and Ritz vectors with residuals; entry 17 is the time of
 * the QR factorisations of the QR-SVD branch (18 entries; times measured by the first
 * thread of the network's workgroup with the wall clock). */
int tn_profile_last(tn_net net, double *seconds_by_kind);

/* x <- x * 2^-e with e the frexp exponent of max|x|; returns e. */
int tn_debug_rescale(double *x, int64_t count, int64_t *exponent);

#ifdef __cplusplus
}
#endif

#endif /* TNAPPROX_H */
