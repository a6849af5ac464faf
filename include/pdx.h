/*
 * pdx.h -- C ABI of libpdx: the PDX dimension-by-dimension K-nearest-
 * neighbour scan on one AMD Instinct MI355X (gfx950).
 *
 * Method: Kuffo, Krippner, Boncz, "PDX: A Data Layout for Vector
 * Similarity Search" (SIGMOD 2025).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Problem (Section 2.1): a collection of n vectors of D float32
 *   coordinates and a query q; the k vectors minimising the squared
 *   Euclidean distance sum_i (v_i - q_i)^2 are returned.
 * - Every data pointer is a DEVICE pointer owned by the caller (e.g. a
 *   torch tensor), 16-byte aligned.  Matrices are row-major float32,
 *   contiguous.  Indexes and search buffers are caller memory: the index
 *   lives in a caller buffer sized with the *_bytes query, and each search
 *   uses a caller workspace sized with the *_workspace query.  The only
 *   device memory the library takes itself is rocBLAS's handle (its GEMM
 *   workspace), once per device on the first IVF build or search or exact
 *   search on the bucket layout, held until the process ends;
 *   pdx_search_exact_noalloc does not use it.
 * - `stream` is a hipStream_t passed as void*; NULL means the default
 *   stream.  Search calls only enqueue work on it (no host sync): outputs
 *   are valid once the caller synchronises the stream.  Build calls are
 *   synchronous (they wait on `stream` before returning).
 * - Results: ids are int64 row numbers into the rows given to the build
 *   call; distances are float32 squared L2, ascending by (distance, id).
 *   If fewer than k candidates exist, the tail holds id -1 and +inf.
 * - Errors: every call returns a pdx_status and never throws.  Argument
 *   errors are detected on the host before anything is enqueued.
 *   pdx_last_error() returns a thread-local description of the last
 *   non-OK status.  A HIP error raised by an enqueue is returned as
 *   PDX_EHIP; faults during execution surface at the caller's sync.
 * - Concurrency: an index is read-only after its build; concurrent
 *   searches on it are allowed, each with its own workspace and stream.
 * - Limits: 1 <= k <= PDX_MAX_K, 1 <= D <= PDX_MAX_DIM, n < 2^31.
 */
#ifndef PDX_H
#define PDX_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define PDX_API __attribute__((visibility("default")))
#else
#define PDX_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdx_status;
#define PDX_OK 0
#define PDX_EINVAL (-1)        /* bad argument, or non-finite data at build */
#define PDX_EWORKSPACE (-2)    /* index buffer or workspace too small */
#define PDX_EHIP (-3)          /* a HIP runtime call or launch failed */
#define PDX_EUNSUPPORTED (-4)  /* valid request outside what is implemented */

#define PDX_MAX_K 64
#define PDX_MAX_RERANK 8192  /* candidates re-ranked by the IVF search (rerank) */
#define PDX_MAX_DIM 4096

/* Opaque host-side handle.  It points into the caller's index buffer,
 * which must outlive it; pdx_free releases only the handle. */
typedef struct pdx_index pdx_index;

/* ---------------------------------------------------------------------
 * Flat (exact-search) index
 * ------------------------------------------------------------------ */

typedef struct {
    int32_t group;      /* vectors per vectorgroup; 0 = 64 (Section 3). Only 64. */
    int32_t start_rows; /* rows of the START block (Section 4 PHASE 0, Section
                           6.5: blocks of at most 10K vectors); 0 = 10000 */
} pdx_build_params;

/* Device bytes pdx_build needs for n rows of d dimensions. */
PDX_API size_t pdx_build_bytes(int64_t n, int32_t d, const pdx_build_params *params);

/* pdx_build -- store the collection in the PDX layout.
 *
 * Section 3 and its kernel listing: rows are cut into vectorgroups of G=64
 * and inside a group the values of one dimension are contiguous (value of
 * dimension j of the group's i-th vector at j*64 + i); the last group is
 * zero-padded.  Section 5: the per-dimension collection means used by the
 * PDX-BOND order are computed (float64 accumulation, stored as float32).
 *
 * x           [n][d] float32 device, read only.
 * index_mem   device buffer of index_bytes >= pdx_build_bytes(n, d, params);
 *             owned by the caller, must stay alive while *out is used.
 * out         receives a new handle (release with pdx_free).
 * Returns PDX_EINVAL for n < 1, d < 1 or d > PDX_MAX_DIM, n >= 2^31, null
 * pointers, or any non-finite value in x; PDX_EWORKSPACE if index_bytes is
 * too small.  Synchronous. */
PDX_API pdx_status pdx_build(const float *x, int64_t n, int32_t d, const pdx_build_params *params,
                     void *index_mem, size_t index_bytes, void *stream, pdx_index **out);

enum {
    PDX_MODE_LINEAR = 0, /* PDX linear scan, every dimension of every vector */
    PDX_MODE_BOND = 1    /* PDXearch with the PDX-BOND bound and order */
};

/* Distances of the exact search (the L2, L1 and IP kernels of Section 3's
 * listing).  Results are ascending in the reported value in every case. */
enum {
    PDX_METRIC_L2 = 0, /* sum_j (q_j - v_j)^2                                  */
    PDX_METRIC_L1 = 1, /* sum_j |q_j - v_j|; PDX-BOND prunes it like L2: its
                          partial sums are lower bounds too                      */
    PDX_METRIC_IP = 2  /* -sum_j q_j v_j (largest inner product first);
                          PDX_MODE_LINEAR only: a partial inner product bounds
                          nothing.  Flat index: a matrix-core scan of every
                          row.  Bucket layout with D % 32 == 0: whole tiles
                          are skipped by q.v <= q.c + |q| r (Cauchy-Schwarz,
                          c the bucket centroid, r the tile radius) and the
                          rest scanned in full                                   */
};

typedef struct {
    int32_t mode;        /* PDX_MODE_LINEAR or PDX_MODE_BOND */
    int32_t chunk;       /* dimensions per pruning step; 0 = 32 */
    int32_t tile_groups; /* vectorgroups per wave task; 0 = library default */
    int32_t queries_per_block; /* queries per workgroup (1, 2, 4, 8); 0 = default */
    /* Optional instrumentation (NULL = off); neither changes the result.   */
    void **phase_events; /* 4 hipEvent_t recorded on `stream`: at the start,
                            after query preparation + START, after the pruned
                            scan, at the end */
    unsigned long long *counters; /* device [4], added to (not cleared):
                            [0] values (vector x dimension) evaluated by START,
                            [1] lane slots START issued, [2] values evaluated
                            by the pruned scan (live lanes only), [3] lane
                            slots it issued (live and pruned lanes) */
    int32_t metric;      /* PDX_METRIC_*; 0 = L2 */
    int32_t start_rows;  /* bucket layout (IVF index): rows of the query's
                            nearest bucket (inner product: the bucket with
                            the largest q.c) that START scans, in whole
                            vectorgroups (Section 6.5 bounds the START
                            block's size); 0 = 128.  The flat index takes
                            its START block from pdx_build_params. */
    /* Optional instrumentation (NULL = off; does not change the result):
     * device [ceil(D / chunk)], added to (not cleared).  Entry c counts the
     * (query, vector) pairs of the pruned scan (PDX_MODE_BOND after START;
     * L2 and L1) whose partial distance after the c-th chunk of the visit
     * order is still at or below the threshold the scan compares it with,
     * i.e. the survivors of each chunk (Section 2.3's pruning power per
     * step).  Pairs the bucket layout's centroid bound skips are never
     * evaluated and count nowhere.  Slows the scan (atomics per chunk). */
    unsigned long long *chunk_survivors;
    /* Schedule of the LDS-tile scan (PDX_MODE_BOND, L2 and L1; no effect on
     * the result, which is exact whatever the schedule; pdx_exact_tune picks
     * them).  rounds: launches the pruned range is split into, the k-th
     * distances refreshed from the candidates in between (1..64; 0 = 2
     * on the bucket layout, 4 on the flat one).
     * dense_min, bucket layout: a (query, 32-row tile) pair with at least
     * this many survivors after the first chunk is finished by the wave
     * that found them, the rest queued (1..33, 33 = always queue; 0 = 4). */
    int32_t rounds;
    int32_t dense_min;
} pdx_search_params;

/* Workspace bytes for pdx_search_exact with these arguments. */
PDX_API size_t pdx_search_exact_workspace(const pdx_index *index, int64_t nq, int32_t k,
                                  const pdx_search_params *params);

/* pdx_search_exact -- exact K-nearest neighbours of nq queries.
 *
 * PDX_MODE_LINEAR: the kernel listing of Section 3 (L2) over every
 * vectorgroup.  For L2 with D % 4 == 0 (and no counters asked for) every
 * vector's distance is evaluated on the matrix cores in the expanded form
 * |q|^2 + |x|^2 - 2 q.x, within a margin that covers its rounding: a pass
 * over every 8th vectorgroup bounds each query's k-th distance from above,
 * a pass over all of them lists the vectors whose lower bound reaches it,
 * and those are summed exactly in the vectorgroup path's order, so the
 * answer is the same.  PDX_MODE_BOND: PDXearch (Section 4) with PDX-BOND
 * (Section 5): dimensions visited by |q_j - mean_j| descending (ties by j),
 * START scans the first start_rows rows without pruning, every later
 * vector is dropped as soon as its partial distance after a chunk is
 * strictly above the running k-th distance.  Both modes return the exact
 * answer; partial sums are accumulated chunk by chunk in a fixed order per
 * (query, vector), so the result does not depend on scheduling.
 *
 * index: flat (pdx_build), or IVF (pdx_ivf_build), whose rows are stored
 * bucket by bucket.  On the bucket layout the scan still visits every
 * vector (the answer is the exact k-NN of all n rows), but a query's own
 * cluster arrives as whole vectorgroups, and START scans the query's
 * nearest bucket (Section 2.1 probe order) instead of the first rows; the
 * BOND means are those of the stored rows; a rotated index rotates the
 * queries first and reports distances in rotated space.
 *
 * Metrics (params->metric): L2 as above; L1 with the same phases (the
 * LDS-tile kernel is L2 only, so L1 scans vectorgroups per wave); IP in
 * linear mode as one matrix-core pass, 16 queries x 64 vectors per wave,
 * reporting -q.v.  A rotated index preserves L2 and IP, not L1: L1 on it
 * is measured in rotated space.
 *
 * q         [nq][d] float32 device.
 * ws        device workspace of ws_bytes >= pdx_search_exact_workspace(...).
 * out_ids   [nq][k] int64 device;  out_dist [nq][k] float32 device.
 * A query holding a non-finite value gets ids -1 and NaN distances (the
 * check runs on the device; the call still returns PDX_OK).
 * nq = 0 is a successful no-op.  Returns PDX_EINVAL (null pointers, nq < 0,
 * k < 1, unknown mode or metric), PDX_EUNSUPPORTED (k > PDX_MAX_K, IP with
 * PDX_MODE_BOND), PDX_EWORKSPACE. */
PDX_API pdx_status pdx_search_exact(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                            const pdx_search_params *params, void *ws, size_t ws_bytes,
                            int64_t *out_ids, float *out_dist, void *stream);

/* pdx_exact_tune -- pick the fastest tile-scan schedule for an exact search.
 *
 * Times pdx_search_exact on the caller's queries (one warm-up, then the
 * best of `reps` timed runs, HIP events on `stream`, synchronous) for each
 * candidate: START block (start_rows 64, 128, 256; bucket layout), rounds
 * (2, 4, 8) and dense_min (4, 8, 16; bucket layout), the 27 combinations
 * in that nesting (start_rows outermost).  A candidate whose value cannot
 * change this search (a flat index's start_rows and dense_min, a search
 * that does not take the tile path) is timed only with that value at its
 * default, and skipped otherwise.  Every schedule returns the same exact
 * answer; only the time differs.
 * params: in, the search to tune (mode, metric, chunk, tile_groups,
 * queries_per_block kept); out, start_rows, rounds and dense_min of the
 * fastest candidate.  table (may be NULL): PDX_EXACT_TUNE_CANDIDATES
 * entries, filled in candidate order (ms < 0: skipped).  ws: at least
 * pdx_exact_tune_workspace bytes, 16-byte aligned.  Returns PDX_EINVAL
 * (null pointers, nq < 1, reps < 1, arguments pdx_search_exact rejects),
 * PDX_EWORKSPACE, PDX_EHIP, or the search's own error. */
#define PDX_EXACT_TUNE_CANDIDATES 27
typedef struct {
    int32_t start_rows, rounds, dense_min;
    float ms; /* best timed run */
} pdx_exact_schedule;

PDX_API size_t pdx_exact_tune_workspace(const pdx_index *index, int64_t nq, int32_t k,
                                        const pdx_search_params *params);
PDX_API pdx_status pdx_exact_tune(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                                  pdx_search_params *params, int32_t reps, pdx_exact_schedule *table, void *ws,
                                  size_t ws_bytes, void *stream);

/* Static device scratch of pdx_search_exact_noalloc, per GPU. */
#define PDX_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* pdx_search_exact_noalloc -- pdx_search_exact with no workspace argument,
 * for callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * Same arguments, results and errors as pdx_search_exact, minus ws and
 * ws_bytes: the workspace is a static device array of
 * PDX_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on
 * holds until the process ends.  The call allocates nothing (no hipMalloc,
 * no library allocator).  Returns PDX_EWORKSPACE when
 * pdx_search_exact_workspace(...) for the same arguments exceeds the
 * scratch (e.g. about 250 queries per call on a 1M x 960 bucket layout;
 * search fewer queries per call).  Every call on one GPU shares that GPU's
 * scratch and leaves its contents behind (the search initialises what it
 * reads): calls that overlap on one GPU, on any streams or threads, race
 * and must be serialised by the caller. */
PDX_API pdx_status pdx_search_exact_noalloc(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                                            const pdx_search_params *params, int64_t *out_ids, float *out_dist,
                                            void *stream);

/* Dimension visit orders (pdx_query_order). */
enum {
    PDX_ORDER_NATURAL = 0, /* stored dimension order (linear scan, ADSampling) */
    PDX_ORDER_BOND = 1,    /* PDX-BOND, Section 5: |q_j - mean_j| descending,
                              equal keys by j ascending (keys in float32)      */
    PDX_ORDER_ZONES = 2    /* dimension zones, Section 5 and Figure "dz": zones
                              of 32 consecutive stored dimensions by
                              sum_j |q_j - mean_j| descending (float32 sums, j
                              ascending), equal scores by zone; storage order
                              inside a zone; a shorter last zone (D % 32 != 0)
                              is visited last                                   */
};

/* Workspace bytes for pdx_query_order over nq queries (0 for bad arguments). */
PDX_API size_t pdx_query_order_workspace(const pdx_index *index, int64_t nq);

/* pdx_query_order -- the dimension visit order each query's search uses.
 *
 * Section 5 (PDX-BOND, "distance to means"; dimension zones): runs the
 * query preparation of pdx_search_exact (PDX_ORDER_BOND: mode BOND) and of
 * pdx_search_ivf's PDX-BOND bounds (PDX_ORDER_BOND: bound 1,
 * PDX_ORDER_ZONES: bound 2) and returns what it produced: means are the
 * index's (flat: the collection's; IVF: those of the stored rows), and a
 * rotated IVF index rotates the queries first (dimensions are then the
 * rotated ones).
 *
 * q            [nq][d] float32 device, read only.
 * order        PDX_ORDER_*.
 * out_perm     [nq][d] int32 device: the j-th visited dimension.
 * out_qval     [nq][d] float32 device or NULL: the (rotated) query value
 *              at that dimension.
 * out_tile_off [nq][d] uint16 device or NULL: the LDS row offsets
 *              (32 * dimension) the exact search's tile scan reads for that
 *              order; needs d * 32 < 65536.
 * ws           pdx_query_order_workspace(index, nq) bytes, 16-byte aligned.
 * Asynchronous on `stream`.  nq = 0 is a no-op.  Returns PDX_EINVAL (null
 * pointers, nq < 0, unknown order), PDX_EUNSUPPORTED (out_tile_off with
 * d * 32 >= 65536), PDX_EWORKSPACE. */
PDX_API pdx_status pdx_query_order(const pdx_index *index, const float *q, int64_t nq, int32_t order,
                                   int32_t *out_perm, float *out_qval, uint16_t *out_tile_off, void *ws,
                                   size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * IVF index with ADSampling
 * ------------------------------------------------------------------ */

enum { PDX_DTYPE_F32 = 0, PDX_DTYPE_BF16 = 1, PDX_DTYPE_FP8 = 2 };

typedef struct {
    int32_t kmeans_iters;   /* Lloyd iterations; 0 = 20 */
    int32_t lowp_mask;      /* extra low-precision copies of the rotated vectors:
                               (1 << PDX_DTYPE_BF16) | (1 << PDX_DTYPE_FP8); 0 = none */
    /* Random numbers are drawn by the caller and passed in:             */
    const double *gaussian; /* [d][d] iid N(0,1) float64 device, rotated with
                               the Q of its QR (Haar sign fix); NULL = no rotation */
    const int64_t *init_rows; /* [nlist] device: rows seeding k-means */
    /* Optional precomputed parts (all device; NULL = compute):            */
    const float *rotation;  /* [d][d] used as is (overrides gaussian)     */
    const float *centroids; /* [nlist][d], in rotated space: skip k-means */
    const int32_t *assign;  /* [n] bucket of each row (needs centroids)   */
    /* Rotation kind (ignored when `rotation` is given):                    */
    int32_t rotation_kind;  /* PDX_ROTATION_RANDOM: Q of the QR of `gaussian`
                               (none when gaussian is NULL); PDX_ROTATION_PCA:
                               the principal directions of the rows, largest
                               variance first (BSA's PCA projection, Section
                               2.3, in place of the random one): float32
                               covariance, cyclic Jacobi sweeps, the float64
                               Householder QR to re-orthonormalise, rows
                               ordered by their Rayleigh quotient; gaussian
                               is then unused                                */
    int32_t pca_iters;      /* PCA: Jacobi sweeps; 0 = 12                    */
} pdx_ivf_params;

enum { PDX_ROTATION_RANDOM = 0, PDX_ROTATION_PCA = 1 };

PDX_API size_t pdx_ivf_build_bytes(int64_t n, int32_t d, int32_t nlist, const pdx_ivf_params *params);

/* pdx_ivf_build -- IVF buckets over randomly rotated vectors, each bucket
 * stored as PDX vectorgroups.
 *
 * Section 2.3 (ADSampling): a random orthogonal rotation R (float64
 * Householder QR on the device) is applied to every row; Section 2.1
 * (IVF): non-optimised Lloyd k-means with nlist buckets, each row in the
 * bucket of its nearest centroid (ties: lower id); an empty bucket keeps
 * its previous centroid.  Section 2.1 / Figure "IVF-PDX": every bucket is
 * a PDX block.  Synchronous.
 *
 * Low precision (lowp_mask): besides the f32 vectorgroups, the rotated rows
 * can be stored as bfloat16 (round to nearest even) and/or float8 e4m3 with
 * a per-dimension scale s_j = max_i |x_ij| / 448 (codes of x_ij / s_j, round
 * to nearest even, saturating); a row-major f32 copy is kept for rerank.
 * Compressed PDX blocks are the paper's future work (Section 7).
 *
 * Returns PDX_EINVAL for bad sizes (nlist < 1 or nlist > n), null required
 * pointers, or non-finite data; PDX_EWORKSPACE if index_bytes is short. */
PDX_API pdx_status pdx_ivf_build(const float *x, int64_t n, int32_t d, int32_t nlist,
                         const pdx_ivf_params *params, void *index_mem, size_t index_bytes,
                         void *stream, pdx_index **out);

/* Copy the IVF index's parts out (any pointer may be NULL):
 * rotation [d][d] f32, centroids [nlist][d] f32 (rotated space),
 * assign [n] int32 (bucket of each row), list_sizes [nlist] int32. */
PDX_API pdx_status pdx_ivf_export(const pdx_index *index, float *rotation, float *centroids,
                          int32_t *assign, int32_t *list_sizes, void *stream);

typedef struct {
    float eps0;        /* ADSampling error bound (Section 6.1: 2.1);
                          +INFINITY: exact within the probed buckets */
    int32_t delta_d;   /* dimensions between tests; 0 = 32, D/4 if D < 128 */
    int32_t dtype;     /* PDX_DTYPE_* copy to scan (must have been stored) */
    int32_t rerank;    /* BF16/FP8 scans: the R best by the scanned distance are
                          re-ranked with exact f32 distances (k <= R <=
                          PDX_MAX_RERANK); 0 = min(4k, PDX_MAX_K); -1 = no
                          rerank (distances are then the scanned low-precision
                          ones).  Ignored for F32.  R > PDX_MAX_K: the scans
                          append every vector that passes the test and lies
                          below tau to a per-query candidate buffer (tau: an
                          upper bound of the R-th smallest buffered distance,
                          from a histogram of the buffered distances; a full
                          buffer is compacted to its R best and the scan
                          resumed, so every probed vector is seen).  On the
                          matrix cores (16 queries per wave, no bucket_split,
                          bfloat16 MFMA on the codes: delta_d a multiple of
                          32; else the vector ALU) resumed vectors are
                          scanned on the vector ALU, whose rounding differs,
                          so there the candidate set can depend on the
                          buffer size at the rounding level.  No learned
                          networks or traces.                               */
    /* Optional instrumentation (NULL = off); neither changes the result.   */
    void **phase_events; /* 4 hipEvent_t recorded on `stream`: at the start,
                            after rotation + bucket selection + START, after
                            the pruned scan, at the end */
    unsigned long long *counters; /* device [4], added to: [0] values evaluated
                            by START, [1] its lane slots, [2] values evaluated
                            by the pruned scan (live lanes), [3] its lane slots */
    /* Learned early termination (see pdx_mlp_*; NULL = plain search).      */
    const void *mlp;       /* network state: after START the query probes the
                              smallest r in 1..nprobe-1 with sigmoid(z_r) >
                              mlp_threshold, else all nprobe buckets        */
    float mlp_threshold;
    /* Traces for training (NULL = off; the search then ignores mlp):       */
    float *trace_features; /* [nq][nprobe][72]: row r - 1 = the network's
                              inputs for "stop after r buckets", r < nprobe;
                              the last row zero                             */
    int32_t *trace_need;   /* [nq]: buckets the result needed, 1 + the
                              largest probe rank holding one of the returned
                              ids (0: no result); stopping after r buckets
                              loses nothing exactly when r >= this          */
    /* Scan schedule; neither changes the exact (eps0 = INF) result.        */
    int32_t queries_per_wave; /* queries of one bucket scanned together by
                                 one wave, each loaded value reused across
                                 them: vector ALU 1, 2, 4, 8 or 16 (0 = 4);
                                 matrix cores 16 or 32 (0 = 16)           */
    int32_t bucket_order;     /* 0: larger buckets first (their work items
                                 start first); 1: by bucket id              */
    int32_t engine;           /* 1: vector ALU (queries_per_wave);
                                 2: matrix cores, 16 or 32 queries per wave,
                                 the dot products of each chunk as MFMA tiles
                                 (F32: the k reported distances recomputed
                                 exactly); 0: automatic, 2 when
                                 queries_per_wave is 0 and nq * nprobe >=
                                 8 * nlist, else 1                         */
    int32_t bucket_split;     /* matrix cores: waves sharing one (query,
                                 bucket) item, each scanning every split-th
                                 vectorgroup with its own k-best list: 1, 2,
                                 4 or 8; 0: automatic (about 8 waves per SIMD
                                 for each phase)                           */
    int32_t bound;            /* 0: the ADSampling test (Section 2.3; its
                                 statistics assume a rotated index);
                                 1: PDX-BOND (Section 5) inside the probed
                                 buckets: each query visits dimensions by
                                 |q'_j - mean_j| descending and drops a
                                 vector once its partial distance exceeds
                                 the running k-th distance, so the result
                                 is exact within the probed buckets (eps0,
                                 engine and queries_per_wave are ignored;
                                 f32 storage only);
                                 2: PDX-BOND with dimension zones (Section
                                 5, Figure "dz"): zones of 32 consecutive
                                 stored dimensions visited by
                                 sum_j |q'_j - mean_j| descending (ties by
                                 zone; a shorter last zone last), one zone
                                 per 32-dimension fetch (delta_d ignored);
                                 exact within the probed buckets as for 1;
                                 3: BSA's test by error quantiles from the
                                 Cauchy-Schwarz inequality (Section 2.3,
                                 with a PCA index its projection): after d
                                 < D dimensions in natural order a vector
                                 is dropped when partial + max(|q_r|^2 +
                                 |x_r|^2 - 2 bsa_m |q_r| |x_r| - err, 0)
                                 > tau (1 + 2^-16), r the dimensions not
                                 yet seen (the build stores |x_r| at each
                                 test point of the default delta_d), err =
                                 2 (D + 4) 2^-24 (|q_r| + |x_r|)^2 covers
                                 float32 rounding; exact at d = D.
                                 bsa_m = 1 makes it a lower bound: exact
                                 within the probed buckets.  Vector ALU
                                 engine only; delta_d must be the
                                 default                                  */
    /* Learned prune bound (see pdx_mlp_*; NULL = ADSampling's eps0).       */
    const void *prune_mlp;    /* network state: after START every (query,
                                 rank r >= 1) gets its own eps, the
                                 multiplier at test point c being
                                 max(1 + eps/sqrt(c1), 0)^2 (bound 0 only;
                                 eps0 is then unused)                       */
    float prune_scale;        /* eps = prune_scale * z; > 0; 0 = 1          */
    float *prune_table;       /* optional out, [nq][nprobe-1][C]: the
                                 multiplier of rank r (row r - 1) at test
                                 point c; needs prune_mlp                    */
    /* Prune-network traces (NULL = off; the search itself is unchanged):   */
    float *trace_prune_features; /* [nq][k][72]: the inputs for (query,
                                    rank of the bucket of the i-th
                                    returned id)                             */
    float *trace_prune_target;   /* [nq][k]: the smallest eps keeping the
                                    i-th returned id at every test point
                                    (partials in the rotated space,
                                    dimensions in natural order); NaN where
                                    there is no sample: no id, an id of the
                                    START bucket, tau_k not positive and
                                    finite.  Targets hold for the exact
                                    result when the search is exact within
                                    the probed buckets (eps0 = +INFINITY,
                                    bound 1 or 2)                            */
    int32_t zone_rows;        /* bound 2: once a vectorgroup has at most this
                                 many surviving vectors, each survivor's
                                 zone is read from the row-major f32 copy
                                 (one 128-byte line) instead of 32
                                 dimension rows of the group; 0 = 32,
                                 < 0 = never.  Needs D % 4 == 0 (else never).
                                 Does not change the result, bit for bit.  */
    float bsa_m;              /* bound 3: the multiplier m in [0, 1]; 0 = 1 */
    int32_t rerank_capacity;  /* rerank > PDX_MAX_K: candidate-buffer slots
                                 per query (8 bytes each, in the workspace):
                                 0 = max(4 rerank, 16384), else at least
                                 max(2 rerank, rerank + 256); capped at what
                                 the nprobe largest buckets hold.  A smaller
                                 buffer costs more compaction rounds (at most
                                 1024, else PDX_EINVAL), never results.     */
} pdx_ivf_search_params;

/* pdx_ivf_tune -- pick the fastest scan schedule for a workload.
 *
 * Times pdx_search_ivf on the caller's queries (one warm-up, then the best
 * of `reps` timed runs, HIP events on `stream`, synchronous) for each
 * candidate schedule: vector ALU with 1, 2, 4 or 8 queries per wave, or
 * matrix cores; buckets by size or by id; and, when tune_delta_d is set
 * and eps0 is finite, ADSampling test intervals delta_d of 32 and 64
 * dimensions (a longer interval tests less often, each test on more
 * dimensions).  The vectorgroup stays 64 vectors: one per lane of a wave.
 * params: in, the search to tune (eps0, dtype, rerank; mlp, prune_mlp,
 * prune_table and every trace must be NULL); out, engine,
 * queries_per_wave, bucket_order and delta_d set to
 * the fastest candidate.  table (may be NULL): PDX_TUNE_CANDIDATES entries,
 * filled in candidate order (ms < 0: candidate skipped).  ws: at least
 * pdx_ivf_tune_workspace bytes, 16-byte aligned.  Errors as pdx_search_ivf. */
#define PDX_TUNE_CANDIDATES 14
typedef struct {
    int32_t engine, queries_per_wave, bucket_order, delta_d;
    float ms; /* best timed run */
} pdx_ivf_schedule;

PDX_API size_t pdx_ivf_tune_workspace(const pdx_index *index, int64_t nq, int32_t k, int32_t nprobe,
                                      const pdx_ivf_search_params *params);
PDX_API pdx_status pdx_ivf_tune(const pdx_index *index, const float *q, int64_t nq, int32_t k, int32_t nprobe,
                                pdx_ivf_search_params *params, int32_t tune_delta_d, int32_t reps,
                                pdx_ivf_schedule *table, void *ws, size_t ws_bytes, void *stream);

PDX_API size_t pdx_search_ivf_workspace(const pdx_index *index, int64_t nq, int32_t k, int32_t nprobe,
                                const pdx_ivf_search_params *params);

/* pdx_search_ivf -- approximate K nearest neighbours with IVF + ADSampling.
 *
 * Section 2.1 (IVF): the rotated query's distances to every centroid; the
 * nprobe nearest buckets (ties by bucket id) are searched nearest first.
 * Section 4 (PDXearch): the first probed bucket is scanned fully (START),
 * every other one chunk by chunk in the rotated (natural) dimension order.
 * Section 2.3 (ADSampling): after d < D dimensions a vector is dropped when
 * partial*D/d > tau*(1 + eps0/sqrt(d))^2, tau the running k-th distance;
 * at d = D the comparison is exact.  Distances are reported in rotated
 * space (equal to the original up to rounding).  Low-precision scans
 * accumulate in f32 over the decoded values; with rerank the returned
 * distances are exact f32 distances.
 *
 * Returns PDX_EINVAL (null pointers, k < 1, nprobe outside [1, nlist],
 * not an IVF index), PDX_EUNSUPPORTED (k > PDX_MAX_K, dtype not stored),
 * PDX_EWORKSPACE. */
PDX_API pdx_status pdx_search_ivf(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                          int32_t nprobe, const pdx_ivf_search_params *params, void *ws,
                          size_t ws_bytes, int64_t *out_ids, float *out_dist, void *stream);

/* ---------------------------------------------------------------------
 * Learned networks for the IVF search
 *
 * Two small networks of one architecture are additions beside the paper's
 * fixed-nprobe IVF search (Section 2.1) and its ADSampling test (Section
 * 2.3), which remain the fallback: with no network the search is the plain
 * one.  Architecture: x (72) -> relu(64) -> relu(64) -> z, float16
 * weights, float32 accumulation.  In the inputs below, tau is the k-th
 * distance in the START bucket (the nearest bucket, scanned whole), d_i
 * the squared distance to the i-th nearest centroid (0-based), and each
 * ratio is clamped to [0, 1e4].
 *
 * Probe budget (pdx_ivf_search_params.mlp).  After START the network is
 * evaluated for r = 1 .. nprobe-1 on: the first 64 rotated query
 * coordinates (zero-padded when D < 64), then tau/d_r, d_r/d_0,
 * d_last/d_0, tau/d_0 and log2(r)/log2(nprobe) (d_r: the first bucket not
 * probed), then 3 zeros; z is a logit.  The query probes the smallest r
 * whose output fires.
 *
 * Prune bound (pdx_ivf_search_params.prune_mlp).  For the bucket of probe
 * rank r >= 1 the network sees the same 64 coordinates, then tau/d_r,
 * d_r/d_0, tau/d_0 and log2(r)/log2(nprobe) (d_r: the bucket being
 * scanned), then 4 zeros; eps = prune_scale * z is that (query, bucket)'s
 * error bound.  After c1 < D dimensions (test points c1 =
 * (c + 1) delta_d; C = ceil(D / delta_d) - 1 of them) a vector of the
 * bucket is dropped when partial * D/c1 > tau_now * m with
 * m = max(1 + eps/sqrt(c1), 0)^2 (capped at 1e30), ADSampling's
 * (1 + eps0/sqrt(c1))^2 with a learned eps in place of eps0; the test after
 * all D dimensions stays exact.  Its training target for a returned
 * neighbour outside the START bucket is the smallest eps that keeps it at
 * every test point, max over c of (sqrt(partial(c1) * D / (c1 * tau_k)) -
 * 1) * sqrt(c1), tau_k being the search's final k-th distance (the running
 * threshold never falls below it); the network is trained for a high
 * quantile of it (PDX_LOSS_PINBALL).
 *
 * State buffer (pdx_mlp_bytes): float32 parameters W1[64][72] b1[64]
 * W2[64][64] b2[64] w3[64] b3 (8897 used, 8960 padded), Adam moments,
 * gradient, and the float16 copy the search and pdx_mlp_forward use.
 * ------------------------------------------------------------------ */

#define PDX_LOSS_BCE 0     /* L = (1/n) sum(-y log p - w (1-y) log(1-p)), p = sigmoid(z),
                              y in {0, 1}, w >= 0 weighting the negatives */
#define PDX_LOSS_PINBALL 1 /* L = (1/n) sum(u (w - [u < 0])), u = y - z, level w in (0, 1):
                              z estimates the w-quantile of y; dL/dz = ([z > y] - w)/n */

PDX_API size_t pdx_mlp_bytes(void);
/* Device workspace for pdx_mlp_grad / pdx_mlp_train_step over n samples. */
PDX_API size_t pdx_mlp_workspace(int64_t n);
/* Set the parameters to theta0 [8960] float32 device (random numbers drawn
 * by the caller), zero the Adam moments, refresh the float16 copy. */
PDX_API pdx_status pdx_mlp_init(void *mlp, const float *theta0, void *stream);
/* z [n] = outputs for x [n][72] with the float16 weights. */
PDX_API pdx_status pdx_mlp_forward(const void *mlp, const float *x, int64_t n, float *z, void *stream);
/* Gradient [8960] of the loss PDX_LOSS_* (parameter w) over samples x [n][72],
 * targets y [n], with respect to the parameters, the network evaluated with
 * its float16 weights; loss (device float, may be NULL) receives L.
 * Deterministic.  PDX_EINVAL for an unknown loss or w out of its range. */
PDX_API pdx_status pdx_mlp_grad(const void *mlp, const float *x, const float *y, int64_t n, int32_t loss_kind,
                                float w, void *ws, size_t ws_bytes, float *grad, float *loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on the
 * full batch x [n][72], targets y [n]; refreshes the float16 copy. */
PDX_API pdx_status pdx_mlp_train_step(void *mlp, const float *x, const float *y, int64_t n, int32_t loss_kind,
                                      float w, float lr, int64_t step, void *ws, size_t ws_bytes, float *loss,
                                      void *stream);
/* Copy the float32 parameters [8960] to theta (device), e.g. to save them;
 * pdx_mlp_init with the same vector restores the network. */
PDX_API pdx_status pdx_mlp_export(const void *mlp, float *theta, void *stream);

/* ---------------------------------------------------------------------
 * Distance kernels without a search (the kernel study of Section 6.4,
 * Tables "kernels" and "block"; the kernels of Section 3's listing)
 * ------------------------------------------------------------------ */

typedef enum {
    PDX_LAYOUT_NARY = 0, /* row-major [n][d] ("horizontal"), one vector per lane */
    PDX_LAYOUT_PDX = 1   /* PDX blocks of `block` vectors (pdx_layout_blocks)  */
} pdx_layout;

/* Bytes of the PDX block layout of n x d float32 rows with blocks of
 * `block` vectors: ceil(n / block) * block * d * 4; 0 for bad arguments. */
PDX_API size_t pdx_layout_blocks_bytes(int64_t n, int32_t d, int32_t block);

/* pdx_layout_blocks -- Section 3: the rows x [n][d] (device, float32,
 * row-major) cut into blocks of `block` vectors; inside a block, dimension
 * j of the block's v-th vector sits at offset j * block + v, i.e. out is
 * [ceil(n / block)][d][block], the last block's missing vectors zero.
 * block: 16, 32, 64, 128, 256 or 512.  out: device, caller-owned,
 * pdx_layout_blocks_bytes bytes.  Asynchronous on `stream`.  PDX_EINVAL for
 * bad sizes, a bad block or null pointers. */
PDX_API pdx_status pdx_layout_blocks(const float *x, int64_t n, int32_t d, int32_t block, float *out, void *stream);

/* pdx_distances -- the L2 (squared), L1 or inner-product (reported as
 * -q.v) score of every vector for each query, no search: out[i][v] for
 * query i and vector v, [nq][n] float32 (device, caller-owned).
 * data: PDX_LAYOUT_NARY, the rows [n][d] (16-byte aligned when d % 4 == 0);
 * PDX_LAYOUT_PDX, the output of pdx_layout_blocks with the same block.
 * q: [nq][d] row-major, 0 <= nq <= 65535.  Both layouts sum a vector's
 * terms in one fixed order (32-dimension chunks, sequential inside a chunk,
 * chunk sums added in order), so they return the same bits.  Non-finite
 * inputs give non-finite scores.  Asynchronous on `stream`.  PDX_EINVAL for
 * bad sizes, an unknown layout or metric, a bad block, null pointers or
 * misaligned row-major data; nq = 0 is a no-op. */
PDX_API pdx_status pdx_distances(const float *data, int32_t layout, int32_t block, int64_t n, int32_t d,
                                 const float *q, int64_t nq, int32_t metric, float *out, void *stream);

/* ---------------------------------------------------------------------
 * Handles and diagnostics
 * ------------------------------------------------------------------ */

/* Releases the host handle only (the caller frees its device buffers). */
PDX_API void pdx_free(pdx_index *index);

/* Thread-local text of the last non-OK status of this thread. */
PDX_API const char *pdx_last_error(void);

/* Library version, e.g. "pdx 0.1.0 gfx950". */
PDX_API const char *pdx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDX_H */
