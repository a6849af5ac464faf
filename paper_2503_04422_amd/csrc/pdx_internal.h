// Internal declarations shared by the libpdx translation units.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pdx.h"

namespace pdx {

constexpr int kGroup = 64;          // vectors per vectorgroup == wave width
constexpr int kWave = 64;
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits
constexpr uint64_t kEmptyKey = ~0ull;       // empty top-k slot

enum IndexKind { kFlat = 1, kIvf = 2 };

}  // namespace pdx

struct pdx_index {
    int kind;
    int64_t n;
    int32_t d;
    int32_t group;
    int32_t ngroups;     // vectorgroups stored
    int32_t start_rows;  // flat: START block, rounded up to whole groups
    float *pdx;          // [ngroups][d][64] float32
    float *means;        // [d] float32 (flat)
    // IVF
    int32_t nlist;
    int32_t dtype_mask;  // bit i set: PDX_DTYPE i stored
    int32_t has_rot;     // 0: rows stored unrotated (rot holds the identity)
    float *rot;          // [d][d] rotation (row j = j-th output coordinate)
    float *centroids;    // [nlist][d] rotated space
    int32_t *list_goff;  // [nlist+1] first vectorgroup of each bucket
    int32_t *list_size;  // [nlist]
    int32_t *slot_id;    // [ngroups*64] original row of each slot (-1 = pad)
    int32_t *assign;     // [n] bucket of each row
    uint16_t *pdx_bf16;  // [ngroups][d][64] (optional)
    uint8_t *pdx_fp8;    // [ngroups][d][64] (optional)
    float *fp8_scale;    // [d] per-dimension scale (optional)
    float *xrow;         // [n][d] rotated rows, row-major (rerank)
    int32_t max_list;    // largest bucket, rows
    int32_t *group_bucket;  // [ngroups] bucket of each vectorgroup
    float *tile_rad;        // [2 ngroups] radius of each 32-vector tile around its centroid
    float *tile_rad1;       // [2 ngroups] the same in the L1 norm
    float *xn_bf16;         // [ngroups][lp_nsub][64] |x_C|^2 of the decoded bfloat16 vectors per 32 dimensions
    float *xn_fp8;          // the same for the decoded e4m3 vectors
    int32_t lp_nsub;        // ceil(d / 32)
    float *xres;            // [ngroups][res_ntp][64] |x| over the dimensions after each test point (BSA)
    int32_t res_ntp;        // test points of the residual norms (delta_d = res_dd)
    int32_t res_dd;
};

namespace pdx {

void set_error(const char *fmt, ...);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Hands out aligned sub-ranges of one caller buffer (or only sizes them
// when base is null).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return align_up(off, 256); }
};

// ---- launchers (each returns hipSuccess or the launch error) ----
hipError_t launch_finite_check(const float *x, int64_t count, int32_t *flag, hipStream_t s);
hipError_t launch_transpose_pdx(const float *x, int64_t n, int32_t d, float *pdx, hipStream_t s);
hipError_t launch_column_means(const float *x, int64_t n, int32_t d, double *partial,
                               int32_t nchunks, float *means, hipStream_t s);

struct ExactPlan {
    int64_t nq;
    int32_t k;
    int32_t mode;
    int32_t chunk;
    int32_t tile_groups;
    int32_t qpb;           // queries per workgroup (waves per block)
    int32_t rounds;        // tile path (L2, L1): launches over the pruned range, threshold refreshed between
    int32_t dense_min;     // bucket-layout tile path: first-chunk survivors that keep a (query, tile) pair in its wave
    int32_t start_groups;  // groups scanned by START
    int32_t tiles_start;
    int32_t tiles_main;
    int32_t nslots;
    bool use_tiles;        // LDS tile path (else the group path only)
    bool ivf;              // bucket layout (IVF index): rows in bucket order, ids through slot_id
    bool library_gemm;     // centroid products on rocBLAS (else the library's own GEMM kernel, which allocates nothing)
    bool lin_mx;           // L2 linear mode on the matrix cores (bound pass, listing pass, exact re-sum)
    float *lin_mins;       // its bound pass: [nq][ip_parts][16] lane minima
    int32_t start_parts;   // bucket layout: waves per query in START
    int32_t start_maxg;    // bucket layout: vectorgroups of the nearest bucket START scans
    int32_t metric;        // PDX_METRIC_*
    int32_t ip_parts;      // inner product: vectorgroup ranges (a multiple of 8)
    uint64_t *ip_slots;    // inner product: [nq][ip_parts][k] k-best lists
    // workspace parts
    uint32_t *tau;
    int32_t *bad;
    int32_t *perm;         // [nq][d] visited dimension order
    float *qperm;          // [nq][d] query values in that order
    uint16_t *poff;        // tile path: [nq][d] LDS tile row offsets of that order
    uint64_t *slots;       // [nq][nslots][k] group-path k-best lists
    uint64_t *cand;        // [nq][cap] tile-path candidates
    int32_t *cand_cnt;     // [nq]
    int32_t *over_list;    // [nq] queries whose candidates overflowed
    int32_t *over_count;
    int32_t tile_grid;     // tile-path workgroups per launch
    int32_t cand_cap;      // tile path: candidate buffer entries per query
    uint64_t *gqueue;      // [tile_grid][overflow cap] survivor entries
    int32_t *tile_ctr;     // tile path: [64] next-tile counters, one per launch
    float *qrot;           // bucket layout, rotated: [nq][d] rotated queries
    float *cd;             // bucket layout: [nq][nlist] centroid distances
    float *dql;            // bucket layout: [nlist][nq] |q - c| lowered (centroid bound)
    float *qn;             // bucket layout: [nq] |q| (inner product, rounded up) or |q|^2 (L2)
    float *qshift;         // inner product, tile path: [nq] B_q, the score shift
    float *cn;             // bucket layout: [nlist] |c| (inner product) or |c|^2 (L2)
    uint32_t *mbits;       // inner product, tile path: bits of M >= every |x|
    int32_t *nearest;      // bucket layout: [nq] START bucket
    uint64_t *start_slots; // bucket layout: [nq][start_parts][k] START lists
    hipEvent_t *events;              // optional [4]
    unsigned long long *counters;    // optional [4]
    unsigned long long *surv;        // optional [ceil(d / chunk)] per-chunk survivors (BOND)
};

constexpr int32_t kDefaultQueriesPerWave = 4;
constexpr int32_t kDefaultRounds = 4;     // exact tile path, flat layout: threshold refreshes
constexpr int32_t kDefaultRoundsBuckets = 2;  // the same on the bucket layout (the centroid bound prunes early)
constexpr int32_t kDefaultDenseMin = 4;   // exact tile path, bucket layout: dense continuation from this many survivors
constexpr int32_t kMaxTileRounds = 64;    // exact tile path: next-tile counters in the workspace
constexpr int32_t kMaxSplit = 8;
constexpr int32_t kMaxWideRounds = 1024;  // compaction + resume rounds of the candidate buffer

// Compute units of the current device (256, the MI355X count, if the query fails).
inline int32_t device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

// Where the scans put each work item's k-best list: [nq][ranks][parts][kk]
// keys, `parts` waves sharing one (query, rank) item (each scans every
// parts-th vectorgroup of the bucket and keeps its own list).
struct SlotMap {
    uint64_t *base;
    int32_t ranks;  // probe ranks held
    int32_t r0;     // first rank held
    int32_t parts;
    int32_t kk;     // list length
    __host__ __device__ uint64_t *at(int64_t q, int32_t r, int32_t part) const {
        return base + (((size_t)q * ranks + (r - r0)) * parts + part) * kk;
    }
};

// The multiplier after c1 dimensions for an error bound eps:
// max(1 + eps/sqrt(c1), 0)^2, capped at 1e30 (ADSampling's shape).  rs is
// 1/sqrt(c1) (prune_rs), computed once per test point by the scans.
__device__ __forceinline__ float prune_rs(int32_t c1) { return 1.0f / sqrtf((float)c1); }
__device__ __forceinline__ float prune_mult(float eps, float rs) {
    const float b = fmaxf(fmaf(eps, rs, 1.0f), 0.0f);
    return fminf(b * b, 1.0e30f);
}

// The test of a bucket of probe rank r >= 1 after c1 < D dimensions: drop
// a vector when its partial distance exceeds tau_now * factor, with factor
// (c1/D) (1 + eps0/sqrt(c1))^2 (ADSampling), or (c1/D) prune_mult(eps, c1)
// with the learned bound eps [nq][nprobe-1] of the (query, bucket).  After
// all D dimensions the factor is 1 (exact).
struct PruneRule {
    float eps0;
    const float *eps;  // null: ADSampling
    // BSA (xres non-null): drop when partial + max(qr^2 + xr^2 - 2 m qr xr
    // - err (qr + xr)^2, 0) exceeds tau (1 + 2^-16); qr, xr: the query's
    // and the vector's norm over the dimensions not yet seen
    const float *xres = nullptr;  // [groups][ntp][64]
    const float *qres = nullptr;  // [nq][ntp]
    int32_t ntp = 0;
    float m = 1.0f;
    float err = 0.0f;  // 2 (D + 4) 2^-24: rounding of the norms and of the estimate
    __device__ __forceinline__ bool bsa_drop(float partial, float tau, float qr, float xr) const {
        const float sum = qr + xr;
        const float rest = fmaxf(fmaf(-2.0f * m * qr, xr, fmaf(qr, qr, xr * xr)) - err * sum * sum, 0.0f);
        return (partial + rest) * (1.0f - 0x1p-16f) > tau;
    }
    __device__ __forceinline__ float ads(int32_t c1, int32_t d) const {
        const float dc = (float)c1;
        const float f = 1.0f + eps0 / sqrtf(dc);
        return (dc / (float)d) * f * f;
    }
    __device__ __forceinline__ float eps_at(int64_t q, int32_t r, int32_t nprobe) const {
        return eps[(size_t)q * (nprobe - 1) + (r - 1)];
    }
    // (c1/D) prune_mult(e, rs): cd = c1/D and rs = 1/sqrt(c1) of the test point
    __device__ __forceinline__ static float learned(float e, float cd, float rs) { return cd * prune_mult(e, rs); }
};

// Operands of the matrix-core scan over low-precision codes (bfloat16
// MFMA on the stored codes): qs [nq][3][dpad] the bfloat16 terms of each
// query, qn [nq][nsub] |q_C|^2 per 32-dimension sub-chunk, xn
// [groups][nsub][64] |x_C|^2 of the decoded stored vectors.  qs null: the
// scan decodes to f32 instead.
struct LpOperands {
    const uint16_t *qs;
    const float *qn;
    const float *xn;
    int32_t nsub;
    int32_t dpad;
};

// Candidate buffer of the IVF search when more than PDX_MAX_K candidates
// are re-ranked (R > 64): every (query, vectorgroup) appends the keys of its
// surviving vectors whose scanned distance is below tau, reserving its slots
// with one atomic add (all or nothing).  A per-query histogram of the stored
// distances (kWideBins bins, 1/64 of an octave each, placed around the
// farthest probed centroid's distance) lowers tau to the upper edge of the
// bin holding the R-th smallest stored distance: at least R stored keys lie
// below it, so no key at or above it can enter the R best.  A full buffer
// stops the (query, bucket) item at the vectorgroup that did not fit; the
// query is then compacted to its R best and the item resumed (bounded
// number of rounds, sized by the planner), so every probed vector is seen.
constexpr int32_t kWideBins = 1024;

struct WideSink {
    uint64_t *buf;    // [nq][cap] keys (distance bits << 32 | id), kEmptyKey = unused
    int32_t *cnt;     // [nq] slots reserved (may exceed cap after an overflow)
    uint32_t *hist;   // [nq][kWideBins] stored keys per distance bin
    int32_t *hbase;   // [nq] bin 0 = distance bits >> 17 at or below this value
    int32_t *resume;  // [nq][nprobe] first vectorgroup not stored (-1: done)
    int32_t *over;    // [nq] 1 while the query has items to resume
    int32_t *olist;   // [2][nq] queries that overflowed, by round parity
    int32_t *ocnt;    // [rounds + 1] entries of each round's list
    int32_t cap;      // buffer slots per query
    int32_t r;        // candidates re-ranked
    int32_t nprobe;
    int32_t round;    // scans: the round their overflows are listed under
    int64_t nq;
};

// Candidate-buffer slots per query for a re-rank of r > PDX_MAX_K: the
// caller's request (0: max(4r, 16384)), at most what the nprobe largest
// buckets can hold (plus one reservation), at least r.
inline int32_t wide_capacity(const pdx_index *ix, int32_t nprobe, int32_t r, int32_t req) {
    const int64_t pmax = ix->n < (int64_t)nprobe * ix->max_list ? ix->n : (int64_t)nprobe * ix->max_list;
    int64_t cap = req > 0 ? req : (4ll * r > 16384 ? 4ll * r : 16384);
    if (cap > pmax + 64) cap = pmax + 64;
    if (cap < r) cap = r;
    return (int32_t)cap;
}

// Compaction + resume rounds that make every probed vector seen: a query
// that fills its buffer has stored at least cap - 63 vectors in the first
// pass and at least cap - r - 63 more in each round that fills it again,
// all distinct, so with pmax vectors probed at most (pmax - cap + 63) /
// (cap - r - 63) rounds can fill it and one more completes it.  -1: the
// capacity leaves no room (cap - r - 63 < 1).
inline int32_t wide_rounds(const pdx_index *ix, int32_t nprobe, int32_t r, int32_t cap) {
    const int64_t pmax = ix->n < (int64_t)nprobe * ix->max_list ? ix->n : (int64_t)nprobe * ix->max_list;
    if (pmax <= cap) return 0;
    const int64_t per = (int64_t)cap - r - 63;
    if (per < 1) return -1;
    const int64_t rounds = (pmax - cap + 63) / per + 1;
    return rounds > (1 << 20) ? (1 << 20) : (int32_t)rounds;
}

hipError_t launch_wide_init(const WideSink &w, const float *cd, int32_t nlist, const int32_t *probe, int32_t rounds,
                            hipStream_t s);
hipError_t launch_wide_select(const WideSink &w, int32_t list_round, uint32_t *tau, hipStream_t s);
hipError_t launch_wide_rerank(const WideSink &w, const float *xrow, const float *qrot, int32_t d, int32_t chunk,
                              const int32_t *bad, int32_t k, int64_t *out_ids, float *out_dist, hipStream_t s);

struct IvfPlan {
    int64_t nq;
    int32_t k;
    int32_t nprobe;
    int32_t chunk;  // dimensions between ADSampling tests
    int32_t dtype;  // storage scanned
    int32_t rerank; // > 0: keep this many candidates and rerank them in f32
    int32_t kk;     // list length kept per work item (k, or rerank)
    float eps0;
    float *qrot;       // [nq][d]
    float *cd;         // [nq][nlist]
    float *qsq, *csq;  // [nq] |q'|^2, [nlist] |c|^2 (centroid products on the matrix cores; null: vector ALU)
    int32_t *probe;    // [nq][nprobe]
    int32_t *bad;      // [nq]
    uint32_t *tau;     // [nq]
    int32_t *cnt0, *cnt1;  // [nlist] item cursors
    int2 *items0, *items1;
    int32_t *budget;   // [nq] buckets the query probes (learned; else nprobe)
    int32_t *xcd;      // matrix engine: [2][9] item ranges per XCD (START, later ranks)
    const __half *w16; // network weights (null: plain search)
    float zthr;        // stop when the logit exceeds this
    float *trace_f;
    int32_t *trace_need;
    const __half *pw16;   // prune-multiplier network (null: ADSampling)
    float pscale;         // multiplier scale
    float *peps;          // [nq][nprobe-1] learned error bounds
    float *ptable;        // optional out: the multipliers
    float *trace_pf;      // prune traces: [nq][k][npt][72] inputs
    float *trace_pt;      // [nq][k][npt] targets
    float *tau0;          // [nq] k-th distance after START (prune network / traces)
    int32_t npt;          // test points per bucket
    PruneRule rule;
    int32_t matrix;    // bucket scan on the matrix cores (16 queries per wave)
    int32_t qb0, qb1;  // queries per wave in the START / later bucket scans
    int32_t bond;      // PDX-BOND bound instead of ADSampling
    int32_t zones;     // with bond: dimension-zone order (chunks of 32 = zones)
    int32_t zone_rows; // with zones: row-major zone reads at or below this many survivors
    int32_t *perm;     // bond: [nq][d] visited dimension order
    float *qperm;      // bond: [nq][d] rotated query values in that order
    int32_t by_size;   // lay buckets out larger first
    int64_t cap0;      // START item slots (counts rounded up to qb per bucket)
    int64_t cap1;      // item slots of ranks >= 1
    SlotMap slots0;    // START lists [nq][1][s0][kk]
    SlotMap slots1;    // lists of ranks >= 1 [nq][nprobe-1][s1][kk]
    uint64_t *rkeys;   // [nq][kk] candidates to rerank
    int32_t wide;      // rerank > PDX_MAX_K: the candidate buffer (WideSink)
    int32_t wide_rounds;  // compaction + resume rounds after the scans
    WideSink ws;
    float *qres;       // BSA: [nq][ntp] query norms over the dimensions after each test point
    LpOperands lp;     // matrix-core scan of low-precision codes on bfloat16 MFMA
    hipEvent_t *events;
    unsigned long long *counters;
};

// Exact inner-product search on the matrix cores (k_exact_ip.hip): 64
// queries x the vectorgroups of one of `parts` ranges per workgroup, then
// the per-range lists merged; -q.v reported.
hipError_t launch_ip_scan(const pdx_index *ix, const float *q, int64_t nq, const int32_t *bad, int32_t parts,
                          uint64_t *slots, int32_t k, hipStream_t s);
hipError_t launch_ip_merge(const uint64_t *slots, int64_t nq, int32_t parts, int32_t k, const int32_t *bad,
                           int64_t *out_ids, float *out_dist, hipStream_t s);
int32_t ip_parts_for(int64_t nq, int32_t ngroups, int32_t d);

// L2 linear mode on the matrix cores (k_lin.hip).  Bound pass over every
// stride-th vectorgroup: per query, each lane's smallest upper bound into
// mins[q][parts][16], their k-th smallest into tau (float bits, +inf when
// fewer than k are finite).
// Listing pass over every vectorgroup: the row slots whose lower bound is
// at or below tau, appended to cand[q][0..cap) with cand_cnt counting on
// past cap (cand_cnt zeroed by the caller).  sid: slot -> row id on the
// bucket layout, null on the flat one; qn: each query's squared norm.
int32_t lin_bound_parts(int64_t nq, int32_t ngroups);
hipError_t launch_lin_bound(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                            const int32_t *bad, int32_t parts, int32_t stride, float *mins, int32_t k,
                            uint32_t *tau, hipStream_t s);
hipError_t launch_lin_list(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                           const int32_t *bad, const uint32_t *tau, uint64_t *cand, int32_t *cand_cnt, int32_t cap,
                           hipStream_t s);

// PDX-BOND inside IVF (k_exact.hip): query order and per-item bucket scans.
// zones: the dimension-zone order (32 consecutive dimensions per zone)
// instead of the per-dimension one
hipError_t launch_bond_prep(const float *q, int64_t nq, int32_t d, const float *means, bool zones, int32_t *perm,
                            float *qperm, uint32_t *tau, int32_t *bad, hipStream_t s);
// pdx_query_order: rotation (qrot [nq][d], rotated bucket layouts only) and
// the query preparation of the searches; off may be null
hipError_t launch_query_order(const pdx_index *ix, const float *q, int64_t nq, int32_t order, float *qrot,
                              int32_t *perm, float *qval, uint16_t *off, uint32_t *tau, int32_t *bad,
                              hipStream_t s);
// survivors at or below which a vectorgroup reads zones from the row-major
// copy (0: never); requested 0 = 32, < 0 = never
int32_t bond_zone_rows(int32_t d, int32_t requested);
hipError_t launch_bond_items(bool prune, const pdx_index *ix, const int2 *items, int64_t nitems,
                             const int32_t *probe, int32_t nprobe, const int32_t *perm, const float *qperm,
                             uint32_t *tau, const int32_t *bad, SlotMap slots, int32_t chunk,
                             unsigned long long *counters, bool zones, int32_t zone_rows, hipStream_t s);

// Bucket scan on the matrix cores (k_ivf_mscan.hip): batches of 16 * tiles
// queries (tiles = 1 or 2) per wave.  wide (non-null): survivors go to the
// candidate buffers (tiles 1, one wave per batch, low-precision codes with
// their LpOperands).
hipError_t launch_ivf_mscan(bool prune, int32_t store, int32_t tiles, const void *data, const float *scale,
                            int32_t d, const int32_t *slot_id, const int32_t *goff, const float *cen,
                            const int2 *items, int64_t nbatch, const int32_t *xcd_range, const int32_t *probe,
                            int32_t nprobe, const float *qrot, uint32_t *tau, const int32_t *bad, SlotMap slots,
                            int32_t chunk, PruneRule rule, unsigned long long *counters, const LpOperands &lp,
                            const WideSink *wide, hipStream_t s);
// The query operands of LpOperands (scale: the e4m3 scales, or null for bfloat16).
hipError_t launch_lp_query(const float *qrot, int64_t nq, int32_t d, const float *scale, const LpOperands &lp,
                           hipStream_t s);

// Item slots for nq queries x `ranks` probe ranks when every bucket's count
// is rounded up to a multiple of qb (at most qb - 1 padding slots per bucket).
inline int64_t ivf_item_capacity(int64_t nq, int32_t ranks, int32_t qb, int32_t nlist) {
    if (ranks <= 0) return 0;
    const int64_t c = nq * ranks + (int64_t)(qb - 1) * nlist;
    return (c + qb - 1) / qb * qb;
}

size_t ivf_plan(const pdx_index *ix, int64_t nq, int32_t k, int32_t nprobe, const pdx_ivf_search_params *p,
                void *ws, IvfPlan *plan);
hipError_t run_ivf(const pdx_index *ix, const float *q, const IvfPlan &plan, int64_t *out_ids,
                   float *out_dist, hipStream_t s);

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s);
// C = A B^T on the matrix cores (A [m][k], B [n][k], C [m][ldc]).
hipError_t launch_gemm_abt(const float *A, int64_t m, const float *B, int64_t n, int32_t k, float *C, int64_t ldc,
                           hipStream_t s);
// The same through rocBLAS's f32 GEMM (allocates its handle on a device's
// first call): the IVF search and build; the exact search keeps the kernel
// above so that its no-allocation entry point allocates nothing.
hipError_t launch_sgemm_abt(const float *A, int64_t m, const float *B, int64_t n, int32_t k, float *C, int64_t ldc,
                            hipStream_t s);
hipError_t launch_pair(int mode, int out, const float *A, int64_t m, const float *B, int64_t nb, int32_t k,
                       float *C, int64_t ldc, unsigned long long *best, hipStream_t s);
hipError_t launch_qr_rotation(const double *gauss, int32_t d, double *acm, double *q, double *v, double *diag,
                              float *rot, hipStream_t s);
hipError_t launch_gather_rows(const float *x, int64_t n, int32_t d, const int64_t *rows, int32_t count,
                              float *out, int32_t *flag, hipStream_t s);
hipError_t launch_labels_from_keys(const unsigned long long *best, int64_t n, int32_t *lab, hipStream_t s);
hipError_t launch_kmeans_update(const float *x, int64_t n, int32_t d, const int32_t *lab, int32_t nlist,
                                double *sums, int32_t *cnt, float *cen, hipStream_t s);
hipError_t launch_check_labels(const int32_t *lab, int64_t n, int32_t nlist, int32_t *flag, hipStream_t s);
hipError_t launch_bucketize(const float *xrot, int64_t n, int32_t d, const int32_t *lab, int32_t nlist,
                            int32_t *blk_cnt, int32_t *size, int32_t *goff, int32_t *stats, int32_t *slot_id,
                            int64_t max_slots, float *pdx, int64_t max_groups, hipStream_t s);

// Residual norms for BSA's test (k_pca.hip): per stored vector and test
// point c (after c1 = (c + 1) dd dimensions, c1 < d), |x| over [c1, d);
// ntp = ceil(d / dd) - 1 test points.  And the same per query.
int32_t res_test_points(int32_t d, int32_t dd);
hipError_t launch_residual_norms(const float *pdx, int32_t d, int64_t ngroups, const int32_t *ngroups_dev,
                                 int32_t dd, float *xres, hipStream_t s);
hipError_t launch_query_residuals(const float *q, int64_t nq, int32_t d, int32_t dd, float *qres, hipStream_t s);

// PCA rotation (k_pca.hip): float32 covariance of the rows x (mu: their
// column means), cyclic Jacobi sweeps, the float64 QR to re-orthonormalise,
// rows by Rayleigh quotient; scratch sized by pca_part_floats (part),
// d x d (cov, h, r2, tmp), d x d float64 (w64, acm, qd), d (v, diag, rho,
// perm), 3 d (cs).
size_t pca_part_floats(int64_t n, int32_t d);
hipError_t launch_pca_rotation(const float *x, int64_t n, int32_t d, int32_t sweeps, const float *mu, float *part,
                               float *cov, float *h, float *r2, double *w64, double *acm, double *qd, double *v,
                               double *diag, float *tmp, float *rho, int32_t *perm, float *cs, float *rot,
                               hipStream_t s);

size_t exact_plan(const pdx_index *ix, int64_t nq, int32_t k, const pdx_search_params *p,
                  void *ws, ExactPlan *plan);
hipError_t run_exact(const pdx_index *ix, const float *q, const ExactPlan &plan,
                     int64_t *out_ids, float *out_dist, hipStream_t s);
// pdx_search_exact; library_gemm false keeps rocBLAS (which may allocate) out of the search
pdx_status search_exact(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                        const pdx_search_params *params, void *ws, size_t ws_bytes, int64_t *out_ids,
                        float *out_dist, void *stream, bool library_gemm);

}  // namespace pdx

namespace pdx {

// ---- low-precision codes (round to nearest even) ----
// bfloat16: upper 16 bits of the float32 pattern after rounding.
__host__ __device__ inline uint16_t bf16_encode(float x) {
    uint32_t b;
    __builtin_memcpy(&b, &x, 4);
    uint32_t lsb = (b >> 16) & 1u;
    return static_cast<uint16_t>((b + 0x7fffu + lsb) >> 16);
}
__host__ __device__ inline float bf16_decode(uint32_t c) {
    uint32_t b = c << 16;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}
// float8 e4m3 ("fn": no infinities, largest finite 448): 1 sign, 4 exponent
// bits with bias 7, 3 mantissa bits, subnormals m * 2^-9; saturates at 448.
__device__ inline uint32_t e4m3_encode(float v) {
    const uint32_t b = __float_as_uint(v);
    const uint32_t sign = (b >> 24) & 0x80u;
    const float a = fabsf(v);
    if (a == 0.0f) return sign;
    if (a >= 448.0f) return sign | 0x7eu;
    const uint32_t ab = __float_as_uint(a);
    const int e = static_cast<int>(ab >> 23) - 127;
    if (e < -6) return sign | static_cast<uint32_t>(rintf(a * 512.0f));  // multiples of 2^-9
    const uint32_t mant = ab & 0x7fffffu;
    uint32_t r = mant >> 20;
    const uint32_t rem = mant & 0xfffffu;
    if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) r += 1;  // carries into the exponent
    uint32_t code = (static_cast<uint32_t>(e + 7) << 3) + r;
    return sign | (code > 0x7eu ? 0x7eu : code);
}
// Decoding is exact (every code is a float32 value); gfx950's conversion
// instruction reads the OCP e4m3 format from the low byte.
__device__ inline float e4m3_decode(uint32_t c) { return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(c), 0); }

// Bucket layout: the bucket of every vectorgroup, and the radius of every
// 32-vector tile around its bucket's centroid (rounded up).
hipError_t launch_tile_radii(const float *pdx, const int32_t *slot_id, const int32_t *goff, int32_t nlist,
                             const float *cen, int32_t d, int64_t max_groups, int32_t *gb, float *rad,
                             float *rad1, hipStream_t s);
hipError_t launch_lowp_store(const float *xrow, int64_t n, int32_t d, const int32_t *slot_id, const int32_t *stats,
                             int64_t max_groups, uint16_t *pdx16, uint8_t *pdx8, float *scale, uint32_t *maxbits,
                             hipStream_t s);
// |x_C|^2 of the decoded low-precision vectors per 32-dimension sub-chunk
// ([max_groups][ceil(d / 32)][64]; either code array may be null).
hipError_t launch_lowp_norms(const uint16_t *pdx16, const uint8_t *pdx8, const float *scale, int32_t d,
                             const int32_t *stats, int64_t max_groups, float *xn16, float *xn8, hipStream_t s);

}  // namespace pdx

namespace pdx {

// ---- learned early-termination network ----
constexpr int kMlpIn = 72;     // inputs: 64 query coordinates + 5 ratios + 3 zero pads
constexpr int kMlpH = 64;      // hidden width (= wave width)
constexpr int kMlpPad = 8960;  // padded parameter count

struct MlpLayout {
    float *theta, *m, *v, *g;
    __half *w16;
    float *loss;
    size_t bytes;
};
MlpLayout mlp_layout(void *base);
hipError_t launch_mlp_init(const MlpLayout &L, const float *theta0, hipStream_t s);
hipError_t launch_mlp_forward(const __half *w16, const float *x, int64_t n, float *z, hipStream_t s);
hipError_t launch_mlp_grad(const MlpLayout &L, const float *x, const float *y, int64_t n, int32_t kind, float w0,
                           float *work, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(const MlpLayout &L, float lr, int64_t step, hipStream_t s);
size_t mlp_work_floats(int64_t n);

}  // namespace pdx
