/*
 * stdecomp.h -- C ABI of libstdecomp: the SGD_Tucker minibatch update for
 * sparse Tucker decomposition (arXiv 2012.03550) on one MI355X (gfx950).
 *
 * Problem (Section "Notation and Preliminaries"): an N-order sparse tensor X
 * of size I_1 x ... x I_N, observed on a set Omega of T entries (COO), is
 * approximated by X_hat = G x_1 A(1) x_2 ... x_N A(N) (Definition "Sparse
 * Tucker Decomposition") with a core G of size J_1 x ... x J_N and factor
 * matrices A(n) of size I_n x J_n.  The parameters are fitted by averaged
 * minibatch SGD (Eq. SGD) on randomly ordered minibatches Psi of M entries:
 * each minibatch takes one step on the core objective (Eq.
 * approximated_core_tensor_optimization, dense core) and then, mode by mode,
 * one step on every sampled factor row (Eq. SGD_factor_matrix, Algorithm 1).
 *
 * Conventions
 *  - Indices are 0-based.  COO indices are SoA: idx[n*T + t] is i_n of entry t.
 *  - A(n) is exchanged row-major I_n x J_n (float32).  G is exchanged flat with
 *    j_1 fastest: G[j_1 + J_1*(j_2 + J_2*(...))] (Definitions "Tensor
 *    Unfolding" and "Vectorization" applied to the core).
 *  - Every function returns STD_OK (0) or a negative STD_E_* code and throws
 *    no C++ exception.  A handle is used by one host thread at a time, with
 *    one exception: stdecomp_predict / stdecomp_predict_noalloc run on the
 *    handle's own query stream and may be called from one other thread while
 *    a training call (stdecomp_epoch, stdecomp_run_minibatches,
 *    stdecomp_epoch_batched) runs on the handle; they then read the
 *    parameters as the chain updates them (every value is the one before or
 *    after an update) and change nothing the training reads.  Distinct
 *    handles are independent.
 *  - Device work runs on the handle's HIP stream (predictions: on a second
 *    stream of the handle, created with the same default priority); every
 *    call returns after its work has finished (the calls are synchronous).
 */
#ifndef STDECOMP_H
#define STDECOMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STD_OK 0
#define STD_E_INVAL (-1)    /* bad order, rank, size, index, hyper-parameter or pointer */
#define STD_E_NOMEM (-2)    /* host or device allocation failed */
#define STD_E_DEVICE (-3)   /* HIP error or a kernel gave up; see stdecomp_last_error */
#define STD_E_STATE (-4)    /* handle misuse (e.g. NULL handle) */
#define STD_E_DIVERGED (-5) /* non-finite parameters or loss */

#define STD_DTYPE_F32 0  /* FP32 parameters and arithmetic */
#define STD_DTYPE_BF16 1 /* BF16 read copies, FP32 master, FP32 accumulation */

#define STD_INIT_SCALED 0 /* entries N(0, 1/J_n) (core: 1/J_1), host RNG seeded by seed_init */
#define STD_INIT_PAPER 1  /* entries N(0.5, 0.1^2): the paper's experimental setting */
#define STD_INIT_CALLER 2 /* zeros until stdecomp_set_params */

/* Where the chain's workgroups run (options.placement).  A chain whose W
 * workgroups fit the compute units of one XCC can run on one XCC: its grid
 * barriers then order memory in that XCC's L2 instead of at device scope, and
 * the values its workgroups exchange stay in L2.  Results are bit-identical
 * either way. */
#define STD_PLACE_AUTO 0    /* one XCC when W fits one, the core is dense (r_core = 0) and
                               the dispatch was found to deal blocks to the XCCs in turn,
                               else spread */
#define STD_PLACE_SPREAD 1  /* blocks 0..W-1, spread over the XCCs, device-scope barriers */
#define STD_PLACE_ONE_XCC 2 /* one XCC, or STD_E_INVAL from stdecomp_init when it cannot
                               (also with r_core > 0) */

typedef struct stdecomp_handle stdecomp_handle;

/* Caller-supplied device memory (e.g. a framework's caching allocator).
 * alloc returns a device pointer to at least `bytes` bytes, aligned to 256
 * bytes, that work on `stream` (the handle's hipStream_t) may use, or NULL on
 * failure; free releases a pointer alloc returned, after all work the handle
 * queued on `stream` has finished.  Both are called from the thread that calls
 * the library, with `ctx` as given in the options. */
typedef void* (*stdecomp_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*stdecomp_free_fn)(void* ctx, void* ptr, void* stream);

/* The tensor (Section "Notation and Preliminaries"). */
typedef struct {
  int32_t order;        /* N, 2 <= N <= 8 */
  const int64_t* dims;  /* I_n, [N], 1 <= I_n < 2^31 */
  const int32_t* ranks; /* J_n, [N], 1 <= J_n <= 32; prod J_n limited by LDS (see stdecomp_init) */
  int64_t nnz;          /* T = |Omega| >= 1 */
  const int32_t* idx;   /* SoA [N][nnz], each 0 <= idx < I_n */
  const float* vals;    /* [nnz] */
} stdecomp_problem;

/* Solver options (Algorithm 1 inputs and the paper's hyper-parameters). */
typedef struct {
  int64_t batch;          /* M, entries per minibatch, 1 <= M <= 16384 */
  float lr_factor;        /* gamma_A >= 0 */
  float lr_core;          /* gamma_G (the paper's gamma_B) >= 0 */
  float lambda_factor;    /* lambda_A >= 0 */
  float lambda_core;      /* lambda_G (the paper's lambda_B) >= 0 */
  uint64_t seed_sample;   /* key of the epoch permutations */
  uint64_t seed_init;     /* seed of the host initialiser */
  int32_t init_kind;      /* STD_INIT_* */
  int32_t dtype;          /* STD_DTYPE_* */
  int32_t r_core;         /* 0: dense core G updated by SGD on Eq. approximated_core_tensor_optimization.
                             1..64: the paper's Kruskal core, G = sum_r b(1)_r o ... o b(N)_r
                             (Eq. CP-Decomposition) with B(n) in R^{J_n x R}: each minibatch
                             takes the column steps of Algorithm 1's core loop on B (Eqs.
                             eventual_approximated, Gradient_core_tensor; lr_core and
                             lambda_core are gamma_B and lambda_B) and then the factor steps
                             with the core they form.  R J_max + 1 columns of a Gram matrix
                             must fit one workgroup's LDS (STD_E_INVAL otherwise) */
  int32_t inputs_on_device; /* 1: problem.idx / problem.vals are device pointers */
  void* stream;           /* hipStream_t to run on, or NULL for a private stream */
  int32_t chain_chunk;    /* entries per workgroup per sub-step; 0: automatic, about M/32,
                             halved while chunk * prod(J) > 2^18 (three modes; 2^19
                             otherwise) or the rows of one
                             workgroup exceed its LDS */
  stdecomp_alloc_fn dev_alloc; /* NULL: hipMalloc.  Otherwise every device buffer the handle
                                  holds or a call of it needs comes from dev_alloc and goes
                                  back through dev_free (both must be given); a NULL return
                                  makes the call fail with STD_E_NOMEM, releasing what it
                                  had allocated */
  stdecomp_free_fn dev_free;
  void* alloc_ctx;             /* passed to dev_alloc / dev_free */
  int32_t report_train_rmse;   /* 1: stdecomp_epoch also evaluates the RMSE over Omega after
                                  its last epoch (one pass of the loss kernel over T entries) */
  float momentum;              /* mu, 0 <= mu < 1: heavy-ball momentum on every sub-step
                                  (Section "Conclusion and Future Works" names momentum as
                                  an extension without fixing it): v <- mu v + g,
                                  theta <- theta - gamma v, one velocity for the core,
                                  updated once per minibatch, and one per factor row,
                                  updated only when the row is sampled.  0: the plain
                                  method, no velocity buffers.  With mu > 0 the handle holds
                                  velocities of the size of the parameters (zero at init;
                                  stdecomp_get/set_velocity); the Kruskal core (r_core > 0)
                                  is refused (STD_E_INVAL) */
  int32_t placement;           /* STD_PLACE_*: the chain's workgroups on one XCC or spread
                                  (stdecomp_step_batched / stdecomp_epoch_batched put every
                                  slot on one XCC when every handle of the batch is on one
                                  and none has momentum, else spread them) */
  int32_t reserved[9];         /* must be zero */
} stdecomp_options;

typedef struct {
  int64_t epochs_run;      /* epochs completed by the call */
  int64_t updates;         /* nonzero-updates = T * epochs_run */
  int64_t minibatches;     /* minibatches run */
  double device_seconds;   /* HIP-event time of the whole call on the stream */
  double schedule_seconds; /* part spent in the sampler and row-set sort */
  double chain_seconds;    /* part spent in the minibatch chain */
  int64_t chain_launches;  /* chain kernel launches */
  double bytes_alg;        /* algorithmic bytes of the chain (COO read + rows read/written + core) */
  double flops_alg;        /* algorithmic flops of the chain: (2N+4) prod(J) per update with a dense
                              core; with the Kruskal core 2N prod(J) plus, per mode n, the row of
                              [W | x] and its Gram matrix, 2R sum_{k!=n} J_k + R J_n + (R J_n + 1)(R J_n + 2) */
  double train_rmse;       /* RMSE over Omega after the last epoch (Section "Experimental
                              Settings"), FP64 sums; NaN unless options.report_train_rmse */
} stdecomp_epoch_stats;

typedef struct {
  double rmse;      /* sqrt(SSE / n) (Section "Experimental Settings") */
  double mae;       /* sum |r| / n */
  double sse;       /* sum r^2, accumulated in FP64 */
  double objective; /* 0.5 SSE / n + 0.5 lambda_A sum ||A(n)||^2 + 0.5 lambda_G ||G||^2 */
  int64_t count;    /* n */
  int64_t nonfinite;/* residuals that were not finite */
} stdecomp_loss_out;

typedef struct {
  int32_t workgroups;      /* W: workgroups of the chain */
  int32_t chunk;           /* entries per workgroup per sub-step */
  int32_t threads;         /* threads per chain workgroup */
  int32_t variant;         /* common rank of the specialised kernel, 0 = generic */
  int64_t lds_bytes;       /* LDS per chain workgroup */
  int64_t device_bytes;    /* device memory held by the handle */
  int64_t minibatches;     /* per epoch: ceil(T / M) */
  int64_t epoch;           /* next epoch index (the current one inside stdecomp_step_batched's windows) */
  int64_t cursor;          /* next minibatch of that epoch for stdecomp_step_batched (0 at an epoch start) */
  int32_t placement;       /* STD_PLACE_ONE_XCC or STD_PLACE_SPREAD: where stdecomp_epoch runs the chain */
} stdecomp_info_out;

/* Fill *o with the defaults: M = 256, gamma = lambda = 0.01, seeds 0, scaled
 * init, FP32, dense core, host inputs, private stream, automatic chunk. */
int stdecomp_default_options(stdecomp_options* o);

/* Create a handle: validates the problem (every index < I_n), copies the COO
 * entries to device memory (the caller may free its arrays on return),
 * initialises the parameters and sizes the epoch schedule and chain.
 * Returns STD_E_INVAL when prod(J) or sum(J) exceed what one workgroup's LDS
 * holds.  *out is NULL on error. */
int stdecomp_init(const stdecomp_problem* p, const stdecomp_options* o, stdecomp_handle** out);

/* Run n_epochs epochs (Algorithm 1 applied to every minibatch of the epoch
 * order pi_e, e = the handle's epoch counter).  An epoch is one pass over all
 * T entries without replacement: minibatch b holds positions
 * [bM, min((b+1)M, T)) of pi_e.  st (nullable) receives counters and times.
 * STD_E_DIVERGED when a parameter became non-finite. */
int stdecomp_epoch(stdecomp_handle* h, int32_t n_epochs, stdecomp_epoch_stats* st);

/* Minibatches [b_begin, b_end) of epoch `epoch` only (a partial epoch, e.g.
 * to resume mid-epoch or to compare a prefix with a reference).  The epoch
 * counter is not changed.  0 <= b_begin <= b_end <= ceil(T / M). */
int stdecomp_run_minibatches(stdecomp_handle* h, int64_t epoch, int64_t b_begin, int64_t b_end,
                             stdecomp_epoch_stats* st);

/* x_hat for q entries (Definition "Sparse Tucker Decomposition").  idx is SoA
 * [N][q]; out is [q]; both host or both device memory (on_device).  An index
 * out of range gives STD_E_INVAL and writes nothing. */
int stdecomp_predict(stdecomp_handle* h, int64_t q, const int32_t* idx, float* out, int32_t on_device);

/* stdecomp_predict for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results as stdecomp_predict, but the
 * packed queries (and, for host buffers, the staged indices and outputs) live
 * in a fixed 16 MiB device array of the library, one per device, resolved at
 * stdecomp_init; the call allocates nothing.  The caller still owns idx and
 * out (both host or both device memory, as in stdecomp_predict).  Limit: the
 * queries must fit the array, pad256(4 q (N + 1)) bytes with device buffers
 * plus pad256(4 q N) + 4 q with host buffers (e.g. 1048576 queries of a
 * three-mode model from device memory, 524288 from host memory); a larger q
 * gives STD_E_INVAL and writes nothing.  Every handle on a device shares that
 * device's array: calls that overlap on one device (from several host
 * threads) race. */
int stdecomp_predict_noalloc(stdecomp_handle* h, int64_t q, const int32_t* idx, float* out, int32_t on_device);

/* RMSE, MAE and SSE over n entries (host or device, SoA idx [N][n], vals
 * [n]); idx == NULL and vals == NULL evaluates the training set Omega. */
int stdecomp_loss(stdecomp_handle* h, int64_t n, const int32_t* idx, const float* vals, int32_t on_device,
                  stdecomp_loss_out* out);

/* Copy the FP32 master parameters out of / into the handle (host memory).
 * A[n] points to I_n x J_n row-major floats; G to prod(J) floats (j_1 fastest).
 * Both are synchronous: each factor goes in one contiguous copy (rows are
 * padded or unpacked on the host), and set_params zeroes the row padding.
 * Errors: STD_E_INVAL for NULL pointers, STD_E_DEVICE if a copy fails. */
int stdecomp_get_params(stdecomp_handle* h, float* const* A, float* G);
int stdecomp_set_params(stdecomp_handle* h, const float* const* A, const float* G);

/* Heavy-ball velocities (options.momentum > 0): copy them out of / into the
 * handle (host memory), laid out as the parameters of stdecomp_get_params:
 * VA[n] points to I_n x J_n row-major floats, VG to prod(J) floats.  They
 * start at zero; with the parameters they make a checkpoint from which the
 * run resumes bit for bit.  stdecomp_set_params leaves them as they are.
 * STD_E_STATE for a handle without momentum, STD_E_INVAL for NULL pointers,
 * STD_E_DEVICE if a copy fails. */
int stdecomp_get_velocity(stdecomp_handle* h, float* const* VA, float* VG);
int stdecomp_set_velocity(stdecomp_handle* h, const float* const* VA, const float* VG);

/* Kruskal core (options.r_core = R > 0): copy the FP32 masters of B(n)
 * (B[n] points to J_n x R row-major floats) out of / into the handle.
 * set_kruskal also sets the core to their Kruskal product (Eq.
 * CP-Decomposition, computed on the host in FP64 and rounded to FP32), so
 * that predictions and losses before the next epoch use it.  STD_E_STATE for
 * a dense-core handle, STD_E_INVAL for NULL pointers. */
int stdecomp_get_kruskal(stdecomp_handle* h, float* const* B);
int stdecomp_set_kruskal(stdecomp_handle* h, const float* const* B);

/* Epoch counter: the next stdecomp_epoch runs epoch e.  Resuming from saved
 * parameters at epoch e reproduces the uninterrupted run bit for bit. */
int stdecomp_set_epoch(stdecomp_handle* h, int64_t e);

/* Schedule of one minibatch as the GPU computes it (host outputs, for
 * bit-exact comparison with the CPU definition): entries[p] = the entry at
 * position p of minibatch `batch` of epoch `epoch` (pi_e(bM + p)); sigma =
 * positions sorted by (i_mode, position); seg_off[0..nseg] and seg_row[0..nseg)
 * = the row runs.  Array sizes: entries, sigma, seg_row >= M; seg_off >= M+1. */
int stdecomp_debug_schedule(stdecomp_handle* h, int64_t epoch, int64_t batch, int32_t mode, int64_t* entries,
                            int32_t* sigma, int32_t* seg_off, int32_t* seg_row, int32_t* nseg, int32_t* m_out);

/* n_epochs epochs of each of n independent models, as stdecomp_epoch on each
 * (Algorithm 1 on every tensor; results identical to running the handles
 * alone), with all of their minibatch chains in one cooperative launch when
 * they share a kernel (equal ranks 4, 8 or 16 in every mode, the same class
 * of order, three or other, the same dtype and device), the handles are
 * distinct, and their workgroups fit the device at once; otherwise the
 * handles run one after another.  hs: n >= 1 handles (caller-owned); st:
 * NULL or n caller-owned records, where chain_seconds and device_seconds are
 * the time of the whole batched launch.  Allocates two small device buffers
 * per call.  STD_E_INVAL for n < 1 or a null array, STD_E_STATE for a null
 * handle; otherwise as stdecomp_epoch (reported on hs[0]). */
int stdecomp_epoch_batched(stdecomp_handle* const* hs, int32_t n, int32_t n_epochs, stdecomp_epoch_stats* st);

/* Continuous batching: advance each of n models by up to max_minibatches
 * minibatches of its current epoch, from where its previous call of this kind
 * stopped (the cursor of stdecomp_info_out), in the launches of
 * stdecomp_epoch_batched (one launch series when the models can share it,
 * else one model after another); a model whose epoch completes moves to the
 * next one (its epoch counter advances, the cursor returns to 0).  Windows of
 * an epoch give the same result, bit for bit, as the whole epoch.  Jobs can
 * thus join and leave a training batch every window instead of every epoch.
 * While a model's cursor is not 0, stdecomp_epoch and stdecomp_epoch_batched
 * refuse it (STD_E_STATE); stdecomp_set_epoch resets the cursor.  st: NULL or
 * n records (minibatches and updates run; epochs_run = epochs completed).
 * STD_E_INVAL for n < 1, a null array or max_minibatches < 1; otherwise as
 * stdecomp_epoch_batched. */
int stdecomp_step_batched(stdecomp_handle* const* hs, int32_t n, int64_t max_minibatches, stdecomp_epoch_stats* st);

/* Measurement aid: the chain's grid barrier alone (the handle's W workgroups,
 * `reps` barriers in a row, 1 <= reps <= 1000000), timed with events on the
 * handle's stream; *us_per_barrier receives the mean time of one barrier in
 * microseconds.  With N + 1 dependent sub-steps per minibatch of m entries a
 * chain cannot exceed m / ((N + 1) t_sync) updates/s.  STD_E_INVAL for a bad
 * reps or a null output, STD_E_DEVICE if a workgroup gave up waiting. */
int stdecomp_debug_barrier(stdecomp_handle* h, int32_t reps, double* us_per_barrier);

/* Self-test of the grid barrier's memory ordering in the handle's placement
 * (STD_PLACE_*): `reps` rounds (1 <= reps <= 1000000) in which every chain
 * workgroup writes the round number into its own word of a device buffer with
 * a plain store, passes the barrier, reads all W words with plain loads and
 * passes a second barrier.  *stale receives how many reads returned an older
 * round (0 when the barrier orders memory as the chain needs).  STD_E_INVAL
 * for a bad reps or a null output, STD_E_DEVICE if a workgroup gave up
 * waiting. */
int stdecomp_debug_barrier_check(stdecomp_handle* h, int32_t reps, int64_t* stale);

/* The GPU sampler alone: out[q] = pi_e(q) for q in [0, T) (the epoch order of
 * Section "Stochastic Optimization", minibatch b = positions [bM, (b+1)M)).
 * out: T int64 values, device memory when out_on_device (written by a kernel
 * on `stream`, nothing allocated), else host memory (a temporary device
 * buffer is allocated and freed).  stream: a hipStream_t or NULL (the null
 * stream).  Returns after the work has finished.  STD_E_INVAL for T < 1,
 * epoch < 0 or out == NULL, STD_E_NOMEM, STD_E_DEVICE. */
int stdecomp_sample_order(int64_t T, uint64_t seed, int64_t epoch, int64_t* out, int32_t out_on_device,
                          void* stream);

int stdecomp_info(const stdecomp_handle* h, stdecomp_info_out* out);

/* Release the handle and its device memory (NULL is accepted). */
int stdecomp_free(stdecomp_handle* h);

/* Static message for a return code; the handle's last error message (for
 * h == NULL: why the calling thread's last stdecomp_init failed). */
const char* stdecomp_strerror(int code);
const char* stdecomp_last_error(const stdecomp_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* STDECOMP_H */
