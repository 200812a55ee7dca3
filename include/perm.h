/*
 * perm.h -- C ABI of libpermgpu: Store-zechin permanents on MI355X (gfx950).
 *
 * The problem (Su & Zheng, section 3.1, eq. (1)): the permanent
 *     per(A) = sum over permutations s of {1..n} of prod_i a[i, s(i)]
 * of an n x n matrix A = (a_ij).
 *
 * The method (section 4, "Store-zechin"): develop per(A) along its last row
 * (property 4 of section 3.1), recursively, storing every sub-permanent the
 * first time it is evaluated and reusing it afterwards (sections 4.2-4.3:
 * each repeated minor is computed once).  A stored sub-permanent is
 *     F(S) = per(rows 1..|S| of A, columns S),  S a subset of the columns,
 * so that F(S) = sum over j in S (ascending) of a[|S|, j] * F(S \ {j}) and
 * per(A) = F({1..n}).  The library evaluates all F(S) with |S| = k before
 * those with |S| = k+1 ("layers" k = 1..n) on the GPU.
 *
 * Numbers:
 *   PERM_COMPLEX128 -- fp64 complex; each F(S) is one fixed chain of fused
 *     multiply-adds over j ascending (re += a.re*p.re; re += -a.im*p.im;
 *     im += a.re*p.im; im += a.im*p.re), so results do not depend on the
 *     launch configuration and are bitwise reproducible.
 *   PERM_INT64 -- exact: per(A) mod several primes p < 2^61 (largest first),
 *     chosen so their product exceeds twice a bound on |per(A)|, plus one
 *     redundant prime that must agree; recombined by Chinese remaindering on
 *     the host into a signed multi-limb integer (perm_int_t).  The layers
 *     whose stored values are bounded below 2^63 (by the row sums and by
 *     k! times the row maxima of |A|) are computed exactly in 64-bit
 *     integers and reduced mod the primes once, after the last of them.
 *
 * Conventions shared by every call:
 *   - Return value: PERM_OK (0), PERM_PENDING (1, server only) or a negative
 *     error code; perm_last_error() then holds a message (thread-local).
 *     No C++ exception ever crosses this boundary.
 *   - Matrices are row-major: entry (i, j) at a[i * lda + j], 0-based,
 *     lda >= n.  int64 entries are int64_t; complex entries perm_c128_t.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *   - The caller owns every buffer it passes, including the device
 *     workspace; the library never frees caller memory.
 *   - NaN/Inf inputs are outside the contract (they propagate by IEEE rules).
 */
#ifndef PERM_H
#define PERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_N_MAX 34        /* largest order accepted by perm_solve (colex ranks stay below 2^32) */
#define PERM_BATCH_N_MAX 12  /* largest order accepted by perm_solve_batch */
#define PERM_INT_LIMBS 36    /* 2304-bit magnitude: enough for any int64 input at n = 34 */
#define PERM_MAX_PRIMES 40   /* primes the integer path may use */

typedef enum { PERM_INT64 = 0, PERM_COMPLEX128 = 1 } perm_dtype_t;

typedef struct {
    double re, im;
} perm_c128_t;

/* value = sign * sum_{i < nlimbs} limb[i] * 2^(64 i); sign is -1, 0 or +1. */
typedef struct {
    int32_t sign;
    uint32_t nlimbs;
    uint64_t limb[PERM_INT_LIMBS];
} perm_int_t;

enum {
    PERM_OK = 0,
    PERM_PENDING = 1,      /* server: ticket not finished yet */
    PERM_EINVAL = -1,      /* null pointer, bad dtype, n < 0, lda < n, bad flags */
    PERM_ERANGE = -2,      /* n above the limit of the call */
    PERM_ENOMEM = -3,      /* workspace too small / footprint above the budget */
    PERM_EDEVICE = -4,     /* a HIP call failed, or the redundant prime disagreed */
    PERM_EAGAIN = -5,      /* server queue full (back-pressure) */
    PERM_ENOTFOUND = -6,   /* unknown or already consumed ticket */
    PERM_ECANCELLED = -7   /* server destroyed before the request finished */
};

/* ------------------------------------------------------------ library --- */

/* Message of the last non-OK return on the calling thread ("" if none). */
const char *perm_last_error(void);

/* ABI version (major * 10000 + minor * 100 + patch). */
int perm_version(void);

/* The i-th prime of the integer path (i = 0 is 2^61 - 1, then descending).
 * Returns PERM_EINVAL if i is outside [0, PERM_MAX_PRIMES) or p is NULL. */
int perm_prime(int i, uint64_t *p);

/* ------------------------------------------------- single-matrix solve --- */

/* Device workspace bytes perm_solve / perm_solve_async need for order n
 * (two layer tables of the largest layer, C(n, n/2) entries, plus the matrix
 * and the scalars).  For PERM_INT64 the size lets three primes share one
 * sweep; a smaller workspace still works (fewer primes per sweep, more
 * sweeps) as long as it holds one prime's tables.  Returns 0 for a bad
 * dtype or n outside [0, PERM_N_MAX]. */
size_t perm_workspace_bytes(perm_dtype_t dt, int n);

/* per(A) of one n x n matrix, 0 <= n <= PERM_N_MAX.
 *   a         host matrix (int64_t or perm_c128_t), row-major with lda.
 *   result    host output: perm_int_t* (PERM_INT64) or perm_c128_t*.
 *   workspace device memory of at least perm_workspace_bytes(dt, n) bytes
 *             (ws_bytes says how much there is); contents are scratch.
 *   stream    the stream every copy and kernel is ordered on.
 * Host-synchronous: returns after the result is in *result.  Re-entrant when
 * calls use distinct workspaces.  n = 0 gives 1 (empty product); n = 1 gives
 * a[0].  Errors: PERM_EINVAL, PERM_ERANGE (n > PERM_N_MAX), PERM_ENOMEM
 * (ws_bytes too small), PERM_EDEVICE. */
int perm_solve(perm_dtype_t dt, int n, const void *a, int64_t lda, void *result,
               void *workspace, size_t ws_bytes, void *stream);

/* Stream-ordered complex128 solve with device input and output: reads the
 * device matrix a_dev (row-major, lda), writes per(A) to *result_dev (device),
 * and returns as soon as the work is queued on `stream`.  Same workspace
 * rules and result bits as perm_solve(PERM_COMPLEX128, ...).  The caller
 * must keep a_dev, result_dev and the workspace alive until the stream has
 * passed the work. */
int perm_solve_async(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev,
                     void *workspace, size_t ws_bytes, void *stream);

/* Allocation-free variant of perm_solve_async, for callers that cannot
 * allocate device memory (code being captured into a HIP graph, serving
 * loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result bits, but the layer tables and the packed matrix live in a fixed
 * device array of PERM_NOALLOC_SCRATCH_BYTES bytes inside the library (one
 * per device, held until the process ends) instead of a caller workspace.
 * The call itself allocates nothing and frees nothing.
 *   n          0 <= n <= PERM_NOALLOC_N_MAX (the largest order whose two
 *              layer tables fit the array).
 *   a_dev      device complex128 matrix, row-major, lda >= n.
 *   result_dev device perm_c128_t output.
 *   stream     the stream every kernel is ordered on.
 * Stream-ordered; returns once the work is queued.  The first call on a
 * device also builds the library's rank tables and synchronizes `stream`
 * (make that call outside any graph capture).  Every call on one device
 * shares its array, so calls that may overlap on that device (different
 * streams, or threads) race and give undefined results: order them on one
 * stream.  Nothing in the array has to start at zero (each layer is fully
 * written before it is read).  Errors: PERM_EINVAL (null pointer, n < 0,
 * lda < n), PERM_ERANGE (n > PERM_NOALLOC_N_MAX), PERM_EDEVICE. */
#define PERM_NOALLOC_N_MAX 22
#define PERM_NOALLOC_SCRATCH_BYTES ((size_t)24 << 20)
int perm_solve_async_noalloc(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev,
                             void *stream);

/* ------------------------------------------------------------- batch --- */

#define PERM_BATCH_SYNC 1u   /* wait for completion before returning */
#define PERM_BATCH_GRAPH 2u  /* launch through a captured HIP graph (replayed on repeat calls) */
#define PERM_BATCH_REUSE 4u  /* with PERM_BATCH_GRAPH: ns/offsets are the same as in the
                              * previous call with this workspace, so the captured graph is
                              * replayed without rebuilding or re-uploading the work list
                              * (ignored without PERM_BATCH_GRAPH) */

/* ----------------------------------------------------------- Ryser --- */

/* The permanent by Ryser's inclusion-exclusion formula (eq. 4 of the paper,
 * the comparison method of its section 3 and Table 4):
 *   per(A) = (-1)^n sum_{S subset of columns} (-1)^|S| prod_i sum_{j in S} a_ij,
 * evaluated with FP64 complex arithmetic over the 2^n subsets in
 * binary-reflected Gray-code order (one column changes between consecutive
 * subsets), in fixed per-thread ranges that each start from directly
 * computed row sums, summed in a fixed order.  O(n^2) memory, no tables; the
 * result is deterministic but, unlike perm_solve, not a Store-zechin chain:
 * inclusion-exclusion cancels, so it agrees with perm_solve only to within
 * the rounding bound derived for it (see the tests).  dt = PERM_INT64 gives
 * the exact permanent (perm_int_t result) from the same walk on residues mod
 * the 61-bit primes perm_solve uses (as many as the entry bound asks for,
 * plus one redundant prime that must agree), recombined on the host.
 *
 * perm_ryser_workspace_bytes: device workspace needed for order n (0 for a
 * bad dtype or n outside 0..PERM_N_MAX).
 * perm_ryser: host matrix a (row-major, a[i*lda + j]: perm_c128_t or
 * int64_t) -> host *result (perm_c128_t or perm_int_t); synchronizes the
 * stream.  Errors as perm_solve (PERM_EDEVICE also when the redundant prime
 * disagrees).
 * perm_ryser_async: complex128, device matrix -> device *result_dev,
 * stream-ordered.  */
size_t perm_ryser_workspace_bytes(perm_dtype_t dt, int n);
int perm_ryser(perm_dtype_t dt, int n, const void *a, int64_t lda, void *result, void *workspace,
               size_t ws_bytes, void *stream);
int perm_ryser_async(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev, void *workspace,
                     size_t ws_bytes, void *stream);

/* ------------------------------------------------- repeated columns --- */

#define PERM_MULTI_N_MAX 64  /* largest n accepted by perm_solve_multi */

/* Permanent of the n x n matrix whose columns are column j of the n x m
 * matrix a repeated mult[j] times, in order (j = 0..m-1): the output
 * amplitudes of bosons that bunch in the detectors (section 2: an amplitude
 * is proportional to the permanent of a submatrix of the interferometer
 * unitary; an output mode hit by t photons contributes its column t times).
 *
 * Identical columns give identical stored minors for every column subset
 * with the same number c_j of copies of each column, so the section-4 table
 * keeps one value per count vector c (0 <= c_j <= mult[j]) instead of one per
 * subset:
 *     G(c) = sum over j ascending with c_j > 0 of a[|c|-1][j] * G(c - e_j),
 *     G(e_j) = a[0][j],  per = G(mult) * prod_j mult[j]!,
 * prod_j (mult[j] + 1) values instead of 2^n.  Layer k (|c| = k) is laid out
 * in colex order of count vectors (the last column most significant); its
 * size must stay below 2^32.
 *
 * Numbers: complex128 uses the perm_solve chain on G, then multiplies both
 * parts by f = 1.0 * 2 * ... * mult[0] * 2 * ... * mult[1] * ... (in double,
 * in that order); with every mult[j] = 1 the result is bitwise perm_solve's
 * (that case runs the subset path).  int64 is exact: G mod the 61-bit primes
 * (bound of the expanded matrix, one redundant prime), recombined on the
 * host, times prod_j mult[j]!; as for perm_solve, the layers whose values are
 * bounded below 2^63 run in exact 64-bit integers first.
 *
 * Arguments: n >= 0 rows (= sum of mult), m distinct columns (0 <= m <= n;
 * m = 0 only with n = 0), mult host int32_t[m], every entry >= 1; a row-major
 * a[i*lda + j], lda >= m.
 * Plan: the tables that map every output to its predecessors depend only on
 * mult; the library builds them on the host at the first call for a mult,
 * uploads them once per device into memory it allocates itself, and keeps
 * them (at most 16 plans and 2 GiB of device copies; beyond that the oldest
 * plan no call is using is dropped, after a device synchronization).
 * perm_multi_workspace_bytes: device workspace for (n, m, mult): the matrix
 * and the pair of largest layers (for int64 per group of primes); 0 when
 * the arguments are invalid or the layer size or the plan exceeds the limits.
 * perm_solve_multi: host matrix (perm_c128_t or int64_t) -> host *result
 * (perm_c128_t or perm_int_t); synchronizes the stream.
 * perm_solve_multi_async: complex128, device matrix -> device *result_dev,
 * stream-ordered (the first call for a mult also builds and uploads its plan,
 * synchronously).
 * Errors: PERM_EINVAL for a null pointer, lda < m, a multiplicity below 1 or
 * a sum other than n; PERM_ERANGE for n > PERM_MULTI_N_MAX, every
 * multiplicity 1 with n > PERM_N_MAX, a layer of 2^32 or more count vectors,
 * a plan beyond its limits (more than 2^24 high parts, or no split whose low
 * window fits 3072 entries), or (int64) a result beyond PERM_INT_LIMBS limbs
 * or PERM_MAX_PRIMES primes;
 * PERM_ENOMEM for a workspace below perm_multi_workspace_bytes;
 * PERM_EDEVICE as perm_solve. */
size_t perm_multi_workspace_bytes(perm_dtype_t dt, int n, int m, const int32_t *mult);
int perm_solve_multi(perm_dtype_t dt, int n, int m, const int32_t *mult, const void *a, int64_t lda, void *result,
                     void *workspace, size_t ws_bytes, void *stream);
int perm_solve_multi_async(int n, int m, const int32_t *mult, const perm_c128_t *a_dev, int64_t lda,
                           perm_c128_t *result_dev, void *workspace, size_t ws_bytes, void *stream);

/* Repeated rows and columns: the permanent of the n x n matrix in which row i
 * of the r x c host matrix a (row-major, lda >= c) is repeated row_mult[i]
 * times and column j col_mult[j] times (every multiplicity >= 1, both sums
 * equal n): the amplitude, up to 1 / sqrt(prod row_mult! prod col_mult!), of
 * bosons entering r modes and leaving c modes with those occupations
 * (section 2).  per(A) = per(A^T) (property 1 of section 3.1), so one side is
 * expanded and the other compressed into count vectors, and the call runs
 * perm_solve_multi on the result.  The side compressed is the one with fewer
 * count vectors, prod(mult + 1) compared exactly (ties compress the
 * columns); the orientation also fixes the fp64 chain, so a complex result
 * is a deterministic function of the inputs (perm_bunched_orientation
 * reports it: *rows = 1 when the rows are compressed).
 * perm_bunched_workspace_bytes: device workspace of that perm_solve_multi
 * call (0 for invalid arguments).  Result and errors as perm_solve_multi;
 * PERM_EINVAL also when the sums differ. */
size_t perm_bunched_workspace_bytes(perm_dtype_t dt, int r, const int32_t *row_mult, int c, const int32_t *col_mult);
int perm_bunched_orientation(int r, const int32_t *row_mult, int c, const int32_t *col_mult, int *rows);
int perm_solve_bunched(perm_dtype_t dt, int r, const int32_t *row_mult, int c, const int32_t *col_mult, const void *a,
                       int64_t lda, void *result, void *workspace, size_t ws_bytes, void *stream);

/* Shape of the repeated-column plan for (n, m, mult), built on the host (no
 * device needed).  With check != 0 the plan is also verified against the
 * closed-form colex ranking of count vectors: the tiles of each layer must
 * cover its ranks exactly once, and every output of every layer (above 2^22
 * outputs in all: up to about 512 tiles per layer and 64 outputs per tile)
 * is unranked, and the rank of each predecessor c - e_j is compared with what
 * the tables give; the number of outputs checked is returned.  PERM_EDEVICE when a check fails (message names the layer and
 * rank).  With every mult[j] = 1 no plan exists (the subset path runs):
 * fields are zero except states = 2^n.  */
typedef struct {
    int L;                /* low columns (0..L-1) */
    uint64_t states;      /* prod_j (mult[j] + 1) */
    uint64_t low_states;  /* prod_{j<L} (mult[j] + 1) */
    uint32_t max_layer;   /* count vectors in the largest layer */
    uint64_t tiles;       /* over layers 2..n */
    uint64_t windows;     /* high windows over layers 2..n */
    uint64_t plan_bytes;  /* device image of the tables */
    uint64_t checked;     /* outputs verified */
} perm_multi_plan_info_t;
int perm_multi_plan_info(int n, int m, const int32_t *mult, int check, perm_multi_plan_info_t *out);

/* Measurement probe: the FP64 rate (TFLOP/s, a fused multiply-add counted
 * as 2 flops) that independent FMA chains sustain on the current device --
 * the measured counterpart of the spec-sheet FP64 vector peak, for the
 * roofline fractions of the FP64-bound paths.  Runs about 10 ms of work on
 * `stream`, synchronizes it, allocates and frees a small device buffer.
 * PERM_EINVAL for a null pointer, PERM_EDEVICE on a HIP failure. */
int perm_probe_fp64(double *tflops, void *stream);

/* Measurement probe for the exact integer sweep: the rate (terms per second,
 * in units of 1e9) of its per-term arithmetic on independent chains --
 * mac_fold_gops: a 64 x 64 -> 128-bit product added into a 128-bit sum, the
 * sum folded mod 2^61 - 1 after every 16 terms (the residue layers);
 * add64_gops: a 64-bit addition (0/1 rows, plain 64-bit layers).  Runs a few
 * ms of work on `stream`, synchronizes it, allocates and frees a small
 * device buffer.  PERM_EINVAL for a null pointer, PERM_EDEVICE on a HIP
 * failure. */
int perm_probe_int(double *mac_fold_gops, double *add64_gops, void *stream);

/* Inspection of the cache-aware tile order (layer_flags bit 2).  The list
 * that a tiled layer launch reads for layer k (2..n) of order n with a low
 * window of t columns: in workgroup order, the high part of each workgroup's
 * tile as a mask of the n - t high columns (bit i = column t + i), or
 * 0xffffffff for an empty padding slot; the tiled k' groups in increasing
 * k', each padded to a multiple of 8 slots.  value_bytes is the size of one
 * stored value (16 for the complex sweep, 8 per prime for the integer
 * sweep); it sets how many high columns a family of tiles may span.  Uses
 * the tuning table's XCD run length and thin-tile threshold for n.  Host
 * only: no device call.  Writes min(cap, length) entries to out (which may
 * be null when cap is 0) and the length to *len.  PERM_EINVAL for a null
 * len, n - t above 18, or n, t, k or value_bytes out of range. */
int perm_layer_tile_order(int n, int t, int k, int value_bytes, uint32_t *out, size_t cap, size_t *len);

/* Device workspace bytes for a batch (host array ns of `count` orders). */
size_t perm_batch_workspace_bytes(perm_dtype_t dt, int count, const int32_t *ns);

/* Many independent permanents of orders 0..PERM_BATCH_N_MAX in one
 * persistent launch.  The paper's workload (section 2) is the boson-sampling
 * amplitude: one permanent of an n x n submatrix of the interferometer's
 * unitary per output pattern, so a sampler needs very many small ones; the
 * paper evaluates one at a time (sections 4-5), the batching is this
 * library's.  The matrices are dealt to workgroups from a work list
 * sorted by cost (largest first); each workgroup keeps a matrix's whole table
 * of stored sub-permanents on chip.
 *   ns[count]      host, orders.
 *   offsets[count] host, element offset of matrix i inside mats.
 *   mats           PERM_COMPLEX128: device perm_c128_t array;
 *                  PERM_INT64: HOST int64_t array (bounds and primes are
 *                  chosen on the host).  Matrices are row-major, lda = n.
 *   results        PERM_COMPLEX128: device perm_c128_t[count];
 *                  PERM_INT64: host perm_int_t[count] (the call is then
 *                  always synchronous).
 *   flags          PERM_BATCH_* bits.
 * Complex results are bitwise equal to perm_solve on the same matrix.
 * Stream-ordered unless PERM_BATCH_SYNC is given.  With PERM_BATCH_GRAPH the
 * launch is captured once per (workspace, mats, results, count) and replayed;
 * PERM_BATCH_REUSE then skips the host work entirely, including the checks of
 * ns and offsets (done when the graph was captured). */
int perm_solve_batch(perm_dtype_t dt, int count, const int32_t *ns, const int64_t *offsets,
                     const void *mats, void *results, void *workspace, size_t ws_bytes,
                     void *stream, uint32_t flags);

/* ------------------------------------------------------------ server --- */
/* Continuous batching of single permanents (not in the paper, which
 * evaluates one permanent at a time): requests of mixed order arrive while
 * others run and are admitted by the footprint of their table of stored
 * sub-permanents (16 * 2^n bytes: section 4 stores every minor once); small
 * orders share launches of the batched kernel, large ones run the layer
 * sweep on their own streams. */

typedef struct perm_server perm_server_t;

typedef struct {
    void *pool;             /* device arena the server carves tables from (caller-owned) */
    size_t pool_bytes;      /* its size */
    size_t budget_bytes;    /* admission budget: sum of 16 * 2^n over admitted requests;
                               0 means pool_bytes */
    int max_large_slots;    /* concurrent large solves (each on its own stream); >= 1 */
    int queue_capacity;     /* pending requests before submit returns PERM_EAGAIN; >= 1 */
    int small_n_max;        /* orders <= this go through the batched kernel (<= 12) */
    int max_small_batch;    /* most small requests in one batched launch; >= 1 */
} perm_server_config_t;

typedef struct {
    double t_submit, t_admit, t_start, t_done; /* seconds on a monotonic clock */
    int n;
    int status;                                /* PERM_OK or the request's error */
} perm_req_stats_t;

/* Start a server (complex128 requests) with its own scheduler thread and
 * streams.  The pool must stay allocated until perm_server_destroy returns. */
int perm_server_create(const perm_server_config_t *cfg, perm_server_t **out);

/* Queue per(A) of a host complex128 matrix (copied before return; the caller
 * may reuse `a` at once).  Returns PERM_EAGAIN when the queue is full,
 * PERM_ENOMEM when 16 * 2^n exceeds the whole budget, PERM_ERANGE for
 * n > PERM_N_MAX.  *ticket identifies the request. */
int perm_server_submit(perm_server_t *s, perm_dtype_t dt, int n, const void *a, int64_t lda,
                       uint64_t *ticket);

/* PERM_PENDING while the request runs; once finished, writes the
 * perm_c128_t result and (if stats != NULL) its timings, releases the ticket
 * and returns the request's status.  PERM_ENOTFOUND for unknown or consumed
 * tickets. */
int perm_server_poll(perm_server_t *s, uint64_t ticket, void *result, perm_req_stats_t *stats);

/* Stop the scheduler, wait for work on the device, fail still-queued
 * requests with PERM_ECANCELLED, free the server.  Unpolled results are
 * dropped. */
int perm_server_destroy(perm_server_t *s);

/* ------------------------------------------------------ tuning / stats --- */

/* Tile and schedule parameters (none of them changes any result bit).
 *   layer_t[n]         columns of the low window of the layer sweep for order
 *                      n (the other columns form a tile's fixed high part);
 *                      0 = library default.
 *   layer_xcd_remap[n] tiles dealt to each of the 8 XCDs in runs of this many
 *                      consecutive tiles; 0 = hardware order, -1 = default.
 *   layer_flags[n]     bit 0: non-temporal stores of layer outputs;
 *                      bit 1: the exact integer sweep's plain 64-bit layers
 *                      (those bounded below 2^63) use layer_t + 1 low columns;
 *                      bit 2: cache-aware tile order (both sweeps, orders
 *                      with at most 18 high columns): tiles that share high
 *                      windows are dealt to one XCD together (see
 *                      perm_layer_tile_order).  The first solve of an order
 *                      with this bit builds the order on the host and uploads
 *                      it into library-owned device memory (an allocation
 *                      and a stream synchronization, once per device, order
 *                      and schedule); perm_solve_async_noalloc never uses it.
 *   layer_thin[n]      tiles with fewer outputs than this are computed one
 *                      output per thread instead of staging a window in LDS;
 *                      0 = library default (128), -1 = never.
 *   batch_group[n]     threads that share one matrix in the batched kernel
 *                      (power of two, 16..512); 0 = library default. */
typedef struct {
    int layer_t[PERM_N_MAX + 1];
    int layer_xcd_remap[PERM_N_MAX + 1];
    int layer_flags[PERM_N_MAX + 1];
    int layer_thin[PERM_N_MAX + 1];
    int batch_group[PERM_BATCH_N_MAX + 1];
} perm_tuning_t;

/* Read / replace the process-wide tuning table (values are validated;
 * PERM_EINVAL on an impossible entry).  perm_tuning_load/_save use a small
 * JSON file keyed by GPU architecture, CU count and HIP runtime version; a
 * file for another key is ignored (returns PERM_ENOTFOUND). */
int perm_tuning_get(perm_tuning_t *out);
int perm_tuning_set(const perm_tuning_t *in);
int perm_tuning_load(const char *path);
int perm_tuning_save(const char *path);
/* The key string the tuning file must carry for the current device. */
int perm_tuning_key(char *buf, size_t len);

/* Per-kernel timing with HIP events on the launch stream.  While enabled,
 * every layer-sweep launch is bracketed by events; perm_profile_read
 * synchronizes on them and returns the summed duration (ms) and the number
 * of launches per kernel family since the last read. */
typedef struct {
    double layer_c128_ms;
    int64_t layer_c128_launches;
    double layer_modp_ms;
    int64_t layer_modp_launches;
    double batch_ms;
    int64_t batch_launches;
    double ryser_ms;        /* transpose + Gray-code walk + final sum, per call */
    int64_t ryser_launches;
    double multi_c128_ms;   /* repeated-column layer sweeps, complex, per layer launch */
    int64_t multi_c128_launches;
    double multi_modp_ms;   /* the same, residues */
    int64_t multi_modp_launches;
    int64_t int_plain_layers; /* layers of perm_solve's exact integer sweep run in plain
                                 64-bit arithmetic (counted once per run of the plain
                                 prefix, which serves every prime) */
} perm_profile_t;

int perm_profile_enable(int on);
int perm_profile_read(perm_profile_t *out);

#ifdef __cplusplus
}
#endif

#endif /* PERM_H */
