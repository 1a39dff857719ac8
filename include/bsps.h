/*
 * bsps.h -- C ABI of the MI355X BSP sample sort library (libbsps.so).
 *
 * The library sorts keys on one GPU with the deterministic regular-
 * oversampling method Sort_Det_BSP (Gerbessiotis & Siniolakis, Section 5.1,
 * Figure SortD) or its randomized oversampling variant Sort_IRan_BSP
 * (Section 5.2, Figure SortRI), both with the duplicate-key handling of
 * Section 5.1.1. The paper's p BSP processors are p virtual processors on one
 * GPU: processor k owns the contiguous block [floor(k n / p), floor((k+1) n / p))
 * of the input and bucket k of the output. Also selectable: the iterative
 * version of Sort_Det_BSP (Section 5.1, m rounds of k-way partitioning,
 * bsps_params.rounds), the Sort_Ran_BSP ordering (Section 5.2, Figure SortR:
 * sample, route, then sort; BSPS_RAN_SR), and the duplicate handling switched
 * off (the ablation of Section 6.4, bsps_params.untagged).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless a comment says HOST. The caller owns
 *    all memory; the library allocates no device memory on any sort path and
 *    frees nothing it did not allocate. (bsps_sort_noalloc instead uses a
 *    fixed scratch array that the library's code holds on every GPU.) State
 *    the library does own: the cached graph executables of the segmented sort,
 *    their capture stream and a pinned host buffer for its segment tables
 *    (all released by bsps_release_cache), the events of the diagnostic stage
 *    timer, and, during a diagnostic call only, a pinned staging buffer
 *    (allocated and freed inside that call).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream). Work is
 *    enqueued asynchronously and the call returns after enqueueing, except in
 *    diagnostic mode (a non-NULL bsps_stats*), where the call synchronizes the
 *    stream before it returns so that the statistics can be filled.
 *  - Every argument check is done on the host before any HIP call; a rejected
 *    call leaves all buffers untouched. Return codes only, no exceptions.
 *  - Key order: int32 and int64 keys sort numerically; float32 keys sort by
 *    IEEE-754 totalOrder of their bit patterns (-0 < +0; NaN patterns sort
 *    outside the finite values, -NaN first and +NaN last).
 *  - The result is the STABLE ascending order: equal keys keep their input
 *    order, which is exactly the order the paper's tie rule (processor
 *    identifier, then local index, Section 5.1.1) produces.
 *  - Limits: n < 2^32 - 1 (positions are 32-bit) and 1 <= p <= 1024. The
 *    local sort by tiles + merge takes blocks of at most 1024 tiles (16K keys
 *    for 4-byte keys, 8K for int64), i.e. n/p <= 2^24 (2^23 for int64):
 *    local_sort = MERGE rejects larger blocks, AUTO sorts them by LSD passes.
 */
#ifndef BSPS_H
#define BSPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSPS_OK = 0,
    BSPS_EINVAL = 1,       /* an argument is out of range (see each call) */
    BSPS_EWORKSPACE = 2,   /* workspace NULL, not 256-byte aligned, or smaller than bsps_workspace_bytes() */
    BSPS_EDEVICE = 3,      /* a HIP call failed */
    BSPS_EUNSUPPORTED = 4  /* valid but outside the library limits (n, p) */
} bsps_status;

/* The method: Sort_Det_BSP (Figure SortD) and Sort_IRan_BSP (Figure SortRI)
 * sort every block first and merge the routed runs; Sort_Ran_BSP (Figure
 * SortR, Section 5.2) samples the unsorted input, ranks and routes every key,
 * then sorts every bucket (route and local sort are its own, so `route` must be
 * BSPS_ROUTE_FUSED; `bucketing` picks the per-key ranking). */
typedef enum { BSPS_DET = 0, BSPS_RAN = 1, BSPS_RAN_SR = 2 } bsps_variant;
typedef enum { BSPS_I32 = 0, BSPS_I64 = 1, BSPS_F32 = 2 } bsps_dtype;

/* How keys are assigned to buckets when every key is ranked on its own. */
typedef enum {
    BSPS_SPLITTER = 0,  /* branch-free binary search of the splitters held in LDS */
    BSPS_LEARNED = 1    /* CDF model prediction, then the exact splitter check */
} bsps_bucketing;

/* How the sorted blocks reach their buckets (Figure SortD steps 9-12). */
typedef enum {
    /* Bucket boundaries come from binary searches of the splitters into each
     * sorted block (the paper's own choice, Section 5.2, Figure SortRI), and the
     * routing is carried out by the final per-bucket merge, which reads each
     * run where it lies in the block-sorted array. */
    BSPS_ROUTE_FUSED = 0,
    /* Every key is ranked against the splitters (or the learned model), the
     * p x p counts are prefix-summed and the keys are scattered into their
     * buckets before the per-bucket merge. */
    BSPS_ROUTE_SCATTER = 1
} bsps_route;

/* How every virtual processor sorts its block (Figure SortD step 3; any stable
 * sequential sort may be used). Both give the same block-sorted array. */
typedef enum {
    BSPS_LOCAL_AUTO = 0,   /* the faster one on MI355X: tiles + merge */
    BSPS_LOCAL_MERGE = 1,  /* stable LDS sort of every tile, then a sample-guided multiway merge of
                              the block's tiles, chunk by chunk */
    BSPS_LOCAL_LSD = 2     /* stable LSD radix sort of every block through HBM, 8-bit digits, one
                              pass per digit position at which the block's keys differ */
} bsps_local_sort;

typedef struct bsps_params {
    int32_t p;          /* virtual processors = blocks = buckets; 1 <= p <= max(n, 1) */
    int32_t s;          /* oversampling: sample records per bucket, i.e. the splitter
                           stride in the sorted sample. DET draws s keys per block
                           (p*s in all); RAN draws s*p - 1 keys. s >= 1. */
    int32_t variant;    /* bsps_variant */
    int32_t bucketing;  /* bsps_bucketing; applies to route = BSPS_ROUTE_SCATTER */
    int32_t route;      /* bsps_route */
    int32_t leaves;     /* learned model: leaf models, 1..4096 (0 = 4096) */
    uint64_t seed;      /* RAN: key of the sample permutation */
    int32_t chunk_cap;  /* 0 = default. Largest merge chunk sorted in LDS; a smaller
                           value routes more chunks through the global-memory path
                           (used to test that path). */
    int32_t local_sort; /* bsps_local_sort: how each block is sorted (step 3) */
    int32_t untagged;   /* 0: the duplicate handling of Section 5.1.1 (splitters carry their
                           tags and ties are broken by position). 1: switched off (the
                           ablation of Section 6.4): splitters compare by key alone, so all
                           keys equal to a splitter go to the bucket it closes. The output
                           is the same stable sort either way; buckets may be uneven with
                           duplicates. */
    int32_t rounds;     /* 0 or 1: Sort_Det_BSP as in Figure SortD. m >= 2: its iterative
                           version (Section 5.1): after the local sort, m rounds each
                           split every current bucket into k = p^(1/m) further buckets
                           and merge every processor's share of them. Needs p = k^m
                           (k >= 2), variant DET, route FUSED, bucketing SPLITTER,
                           untagged 0; m <= 10. Same output (the stable sort). */
    int32_t reserved[4];/* must be zero */
} bsps_params;

/*
 * Diagnostic statistics, HOST memory. Every pointer member may be NULL (not
 * filled). Passing a non-NULL bsps_stats* makes the call synchronous; the
 * arrays are copied out through a pinned staging buffer (hipHostMalloc,
 * freed before the call returns), 8 MiB at a time.
 */
typedef struct bsps_stats {
    void* splitter_keys;       /* p-1 keys of the call's dtype */
    int64_t* splitter_pos;     /* p-1 tags: positions in the block-sorted array */
    void* sample_keys;         /* sorted sample: DET p*s, RAN and RAN_SR p*s-1 keys */
    int64_t* sample_pos;       /* their positions in the block-sorted array (RAN_SR: in the input) */
    int64_t* bucket_sizes;     /* p */
    int64_t* count_matrix;     /* p*p, row k = source block, column i = bucket */
    void* block_sorted;        /* n keys: every block sorted (Figure SortD step 3); with a block
                                  shift D > 0 (reserved_i[3] bits 8-15) sorted on the order key
                                  >> D only, equal keys in input order: a stable sort of each
                                  block by key gives the exactly sorted block */
    uint32_t* block_sorted_values; /* n payloads, kv calls only */
    void* routed;              /* n keys after routing (route = SCATTER, or variant RAN_SR) */
    uint32_t* buckets;         /* n bucket ids of block_sorted (route = SCATTER), of the input (RAN_SR) */
    double max_bucket_ratio;   /* largest bucket / (n/p) */
    double mispredict_rate;    /* learned bucketing: fraction of keys corrected */
    double mean_fix_dist;      /* learned bucketing: mean |predicted - true| */
    int64_t oversize_chunks;   /* merge chunks sorted by the global-memory path */
    int64_t reserved_i[4];     /* bsps_sort: [0] oversize chunks of the block merge, [1] of the
                                  bucket merge, [2] keys in the largest one, [3] bits 0-7: the most
                                  low key bits the tile sort left to the block merge in any block
                                  (0: every block's tiles fully sorted), bits 8-15: the block shift
                                  D, the low key bits the block merge left to the bucket merge
                                  (route FUSED, one round). bsps_sort_segmented:
                                  [0] blocks, [1] merged segments, [2] 1 if the graph was captured
                                  and launched by this call, 2 if a cached graph was launched,
                                  [3] segments with learned bucketing (NL) */
    /* bsps_sort_segmented only: the training state of the learned models of its NL
     * large segments, in segment order, for checking the batched training kernels.
     * Filled when non-NULL and seg_capacity >= NL (else left untouched). */
    void* seg_models;          /* NL models of bsps_model_bytes(64) bytes each (layout of bsps_fit_model) */
    float* seg_grad;           /* NL * 64 * 2: leaf-stage gradient (dLoss/dc, dLoss/dd) at c = d = 0 */
    float* seg_gram;           /* NL * 64 * 3: leaf-stage Gram sums, as bsps_model_grad's out_gram */
    int64_t seg_capacity;      /* models the three buffers hold */
} bsps_stats;

/* Bytes of device workspace a sort of n keys needs (values: 0 or 1). Returns
 * 0 for invalid arguments. */
size_t bsps_workspace_bytes(int64_t n, int32_t dtype, int32_t with_values, const bsps_params* prm);

/*
 * Sort n keys in place (Figure SortD / Figure SortRI).
 *  keys      device, n keys of `dtype`; replaced by the sorted keys
 *  ws        device workspace, 256-byte aligned, of ws_bytes >= bsps_workspace_bytes(n, dtype, 0, prm)
 * Errors: EINVAL for n < 0, p < 1, p > max(n, 1), s < 1, RAN with s*p - 1 > n,
 * unknown dtype/variant/route/bucketing, leaves < 0 or > 4096, nonzero reserved fields;
 * EWORKSPACE; EUNSUPPORTED beyond the limits above. n = 0 and n = 1 are
 * valid no-ops.
 */
bsps_status bsps_sort(void* keys, int64_t n, int32_t dtype, const bsps_params* prm,
                      void* ws, size_t ws_bytes, void* stream, bsps_stats* st);

/* As bsps_sort, carrying a uint32 payload per key (values, device, n); equal
 * keys keep their input order, so payloads of equal keys keep theirs. */
bsps_status bsps_sort_kv(void* keys, uint32_t* values, int64_t n, int32_t dtype, const bsps_params* prm,
                         void* ws, size_t ws_bytes, void* stream, bsps_stats* st);

/*
 * Allocation-free sort, for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): bsps_sort (values == NULL) or bsps_sort_kv (values != NULL)
 * with the workspace taken from a scratch array that the library holds
 * statically on every GPU it runs on (BSPS_NOALLOC_SCRATCH_BYTES per GPU,
 * reserved when the library's code is loaded on that GPU and kept until the
 * process ends). The call allocates and frees nothing and records no timing
 * events. The scratch address of the current device is looked up on the first
 * call on that device (the device current at the call must be the one
 * `stream` belongs to). Every call on one GPU shares that GPU's scratch:
 * calls that overlap in time on one GPU (two host threads, or two streams
 * whose work runs concurrently) race and give wrong results; calls in order
 * on one stream are safe. The sort clears everything it reads before use, so
 * the previous call's contents do not matter.
 * Errors: as bsps_sort; EUNSUPPORTED when the workspace the sort needs,
 * bsps_workspace_bytes(n, dtype, values != NULL, prm), exceeds
 * BSPS_NOALLOC_SCRATCH_BYTES (checked on the host before any HIP call).
 */
#define BSPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bsps_status bsps_sort_noalloc(void* keys, uint32_t* values, int64_t n, int32_t dtype, const bsps_params* prm,
                              void* stream);

/*
 * Sort nseg independent segments [h_offsets[i], h_offsets[i+1]) of one key
 * array (and payload array if values != NULL), each with its own (p, s)
 * chosen per size class by the built-in tuning table or by tuning_json. All
 * segments go through one captured graph launch, cached by the exact call
 * signature (pointers, dtype, offsets, table) until bsps_release_cache().
 * The per-call segment tables are uploaded into the workspace from a pinned
 * host buffer the library owns; a call waits for the previous call's upload
 * before refilling it. Not thread safe (shared cache and staging buffer).
 *  h_offsets   HOST, nseg + 1 non-decreasing entries, h_offsets[0] = 0
 *  tuning_json HOST, NULL for the built-in table (format: bsps_tuning_format())
 * Errors: EINVAL for nseg < 0, offsets not non-decreasing or not starting at 0,
 * unknown dtype, malformed tuning_json; EWORKSPACE; EUNSUPPORTED as bsps_sort.
 */
bsps_status bsps_sort_segmented(void* keys, uint32_t* values, const int64_t* h_offsets, int32_t nseg,
                                int32_t dtype, const char* tuning_json, void* ws, size_t ws_bytes,
                                void* stream, bsps_stats* st);
size_t bsps_segmented_workspace_bytes(const int64_t* h_offsets, int32_t nseg, int32_t dtype,
                                      int32_t with_values, const char* tuning_json);

/*
 * Bucket of every key of a block-sorted array (Figure SortD step 9, tie rule
 * of Section 5.1.1): bucket(g) = number of splitter records (key, tag) that
 * are strictly below the record (keys[g], g).
 *  keys        device, n keys of dtype, every block of the p-way split sorted
 *  spl_keys    device, p-1 keys of dtype; spl_pos device, p-1 uint32 tags
 *  model       device learned model from bsps_fit_model (bucketing = LEARNED),
 *              ignored for SPLITTER
 *  out_bucket  device, n uint32 (may be NULL)
 *  out_counts  device, p*p uint32 count matrix, row = block (may be NULL)
 *  st          HOST, optional: mispredict_rate / mean_fix_dist (synchronizes)
 * Errors: EINVAL as bsps_sort, or model NULL with LEARNED; EWORKSPACE.
 */
bsps_status bsps_rank(const void* keys, int64_t n, int32_t dtype, int32_t p, const void* spl_keys,
                      const uint32_t* spl_pos, int32_t bucketing, const void* model,
                      uint32_t* out_bucket, uint32_t* out_counts, void* ws, size_t ws_bytes,
                      void* stream, bsps_stats* st);
size_t bsps_rank_workspace_bytes(int64_t n, int32_t p);

/*
 * Learned bucketing model (not in the paper): a linear root model choosing one
 * of L linear leaf models of the cumulative distribution, trained on the
 * sorted sample by the library's forward, backward (gradient and Gram sums)
 * and Newton-update kernels. Layout of the device model buffer
 * (bsps_model_bytes(L) = 48 + 12 L bytes, float32 unless noted):
 *   bytes  0..15  lo, hi as float64 (order-key range of the sample)
 *   bytes 16..31  root a, b, mu_r and inv_range = 1 / (hi - lo) (4 floats)
 *   bytes 32..47  L, p, s and a zero pad (4 int32)
 *   bytes 48..    L leaf triples (c, d, mu), 12 bytes each.
 * A leaf predicts c * (x - mu) + d for x = (u - lo) * inv_range.
 *  smp_keys  device, N sorted keys of dtype (the sorted sample)
 *  N, p, s   sample size and sort parameters (targets y_t = (t + 0.5) / (p s))
 *  iters     Newton iterations per stage (>= 1)
 *  model     device, bsps_model_bytes(L)
 */
size_t bsps_model_bytes(int32_t leaves);
bsps_status bsps_fit_model(const void* smp_keys, int64_t N, int32_t dtype, int32_t p, int32_t s,
                           int32_t leaves, int32_t iters, void* model, void* ws, size_t ws_bytes,
                           void* stream);
size_t bsps_fit_workspace_bytes(int64_t N, int32_t leaves);

/*
 * One forward + backward evaluation of the leaf stage for the gradient check:
 * for the N sorted sample keys and the model's current root and leaf
 * parameters, writes out_leaf[t] (device, N int32), out_grad (device, 2L
 * float: dLoss/dc, dLoss/dd per leaf) and out_gram (device, 3L float:
 * sum (x-mu)^2, sum (x-mu), count, all times 2/N), and the loss to *out_loss
 * (device, 1 float). Loss = (1/N) sum_t (f(x_t) - y_t)^2. ws: device,
 * bsps_fit_workspace_bytes(N, leaves) bytes.
 */
bsps_status bsps_model_grad(const void* smp_keys, int64_t N, int32_t dtype, int32_t p, int32_t s,
                            int32_t leaves, const void* model, int32_t* out_leaf, float* out_grad,
                            float* out_gram, float* out_loss, void* ws, size_t ws_bytes, void* stream);

/* Reference copy used to measure the attainable HBM bandwidth next to the
 * sort's kernels: copies `bytes` from src to dst (device pointers, both
 * 16-byte aligned, not overlapping; bytes a multiple of 16) with 16-byte
 * nontemporal vector loads and stores, asynchronously on `stream`. EINVAL for
 * misaligned pointers or sizes (checked on the host before any HIP call);
 * EUNSUPPORTED above 2^31 workgroups (32 TiB). */
bsps_status bsps_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/*
 * Host dry runs of the sort and of the segmented sort: the call plans the work
 * exactly as bsps_sort[_kv] / bsps_sort_segmented would for these sizes and
 * parameters, with fake buffer addresses, and instead of launching each kernel
 * it checks the launch: every pointer argument, and every table pointer inside
 * the argument structs, must be null or lie inside the keys, payload or
 * workspace buffer together with the whole extent the kernel indexes
 * (e.g. G*R run entries of a merge, p*256 digit starts per position of the LSD
 * passes), and grids must be non-empty. The segmented planner's host tables
 * are checked for consistency (blocks inside their segments, groups naming a
 * merged segment's bucket, prefix tables matching the sizes). No HIP call is
 * made; this runs without a GPU.
 *  report  HOST, report_len bytes (may be NULL): one line per finding, or
 *          "ok: N launches checked"
 * Returns the number of findings (0 = clean) or -status for arguments the real
 * call would reject (as bsps_sort / bsps_sort_segmented).
 */
int64_t bsps_check_sort(int64_t n, int32_t dtype, int32_t with_values, const bsps_params* prm, char* report,
                        size_t report_len);
int64_t bsps_check_segmented(const int64_t* h_offsets, int32_t nseg, int32_t dtype, int32_t with_values,
                             const char* tuning_json, char* report, size_t report_len);

/* Human-readable name of a status code (static storage). */
const char* bsps_status_string(int32_t status);
/* Format of the tuning table accepted by bsps_sort_segmented (static storage). */
const char* bsps_tuning_format(void);
/* Frees the library's owned state: the cached graph executables of the
 * segmented sort, their capture stream and the pinned table-staging buffer. */
void bsps_release_cache(void);

/*
 * Diagnostics: per-stage timing with HIP events recorded on the caller's
 * stream around every stage of the following calls. Stages (index):
 *   0 local sort (tile sorts; any LSD sort, local or Sort_Ran_BSP's bucket
 *     sort, with its digit counts and passes), 1 block merge,
 *   2 sample + sample sort + splitters,
 *   3 bucket ranking (bucket boundaries, the learned model's fit, per-key
 *     ranking), 4 prefix sums / routing, 5 bucket merge (every round of the
 *     iterative version; Sort_Ran_BSP: the sort of its buckets),
 *   6 merge kernel of the block merge, 7 merge kernel of the bucket merge,
 *   8 per-key ranking kernel, 9 the LSD passes (tile-parallel sweeps).
 * bsps_timing_read waits for the recorded events and returns, for the first
 * nstage stages, the summed milliseconds (ms, HOST) and launch counts
 * (launches, HOST); reset != 0 clears the record. Not thread safe.
 */
int bsps_timing(int enable);
int bsps_timing_read(double* ms, int64_t* launches, int nstage, int reset);

#ifdef __cplusplus
}
#endif

#endif /* BSPS_H */
