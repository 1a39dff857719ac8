/*
 * bsp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-thread CPU simulation of the two BSP sorting
 * algorithms of Gerbessiotis & Siniolakis, "BSP Sorting: An Experimental
 * Study": Sort_Det_BSP (Section 5.1, Figure SortD) and Sort_IRan_BSP
 * (Section 5.2, Figure SortRI), both with the duplicate-key handling of
 * Section 5.1.1. The p BSP processors are simulated one after the other.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may call this library. It shares no code, header or table with the GPU
 * library; the two are compared on the same inputs.
 *
 * Working representation. Every key is first mapped to an unsigned 64-bit
 * "order key" whose unsigned order is the key order (int32/int64: numeric;
 * float32: IEEE-754 totalOrder of the bit pattern, so -0 < +0). The sort
 * carries, with each key, its original index; the caller gathers raw keys and
 * payloads with the returned permutation.
 *
 * Parity status: every function below is pinned by the CPU tests (brute
 * force on tiny inputs, closed forms of Lemma `balance`, library sorts), except
 * that the random sample positions of Sort_IRan_BSP cannot be compared with the
 * paper's own runs (its generator is not given): parity unpinned for the
 * choice of RAN sample, self-consistent only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORA_OK 0
#define ORA_EINVAL 1
#define ORA_ENOMEM 2

enum { ORA_DET = 0, ORA_RAN = 1 };

/* ------------------------------------------------------------------------ */
/* Key order                                                                 */
/* ------------------------------------------------------------------------ */

/* int32: two's complement numeric order == unsigned order after flipping the sign bit. */
uint64_t ora_order_i32(int32_t v) { return (uint64_t)((uint32_t)v ^ 0x80000000u); }

/* int64: same, 64-bit. */
uint64_t ora_order_i64(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }

/* float32 bits: negative patterns are reversed (all bits flipped), non-negative
 * ones get the sign bit set, which is IEEE-754 totalOrder on the bit pattern. */
uint64_t ora_order_f32(uint32_t bits) {
    return (bits & 0x80000000u) ? (uint64_t)(uint32_t)~bits : (uint64_t)(bits | 0x80000000u);
}

/* kind: 0 int32, 1 int64, 2 float32 (raw bits). */
void ora_order_keys(int kind, const void* keys, int64_t n, uint64_t* out) {
    for (int64_t i = 0; i < n; i++) {
        if (kind == 0) out[i] = ora_order_i32(((const int32_t*)keys)[i]);
        else if (kind == 1) out[i] = ora_order_i64(((const int64_t*)keys)[i]);
        else out[i] = ora_order_f32(((const uint32_t*)keys)[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Keyed permutation for the random sample                                   */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t ora_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* A permutation of [0, n): a 4-round balanced Feistel network on 2h bits
 * (2h >= ceil(log2 n)), round function mix64(seed + golden*(round+1) + right),
 * restricted to [0, n) by cycle walking (Black & Rogaway 2002). */
int64_t ora_feistel(uint64_t seed, int64_t n, int64_t t) {
    if (n <= 1) return 0;
    int bits = 0;
    while (((int64_t)1 << bits) < n) bits++;
    int h = (bits + 1) / 2;
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t x = (uint64_t)t;
    do {
        uint64_t L = x >> h, R = x & mask;
        for (uint64_t j = 0; j < 4; j++) {
            uint64_t f = ora_mix64(seed + 0x9E3779B97F4A7C15ull * (j + 1) + R) & mask;
            uint64_t nl = R;
            R = L ^ f;
            L = nl;
        }
        x = (L << h) | R;
    } while (x >= (uint64_t)n);
    return (int64_t)x;
}

/* ------------------------------------------------------------------------ */
/* Records: a key tagged with its position g in the block-sorted array       */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t pos; } rec_t;

/* Record order of the duplicate handling (Section 5.1.1): key first, then
 * the tag. With contiguous blocks the tag (processor, local index) orders
 * exactly like the global position g in the block-sorted array. */
static int rec_less(rec_t a, rec_t b) { return a.key < b.key || (a.key == b.key && a.pos < b.pos); }

static int rec_cmp(const void* pa, const void* pb) {
    rec_t a = *(const rec_t*)pa, b = *(const rec_t*)pb;
    if (rec_less(a, b)) return -1;
    if (rec_less(b, a)) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step O0/O1: validation and blocks                                          */
/* ------------------------------------------------------------------------ */

/* Processor k owns positions [ora_block_start(k), ora_block_start(k+1)):
 * the input is evenly distributed, sizes differ by at most one. */
int64_t ora_block_start(int64_t n, int p, int k) { return (int64_t)(((__int128)k * n) / p); }

int ora_validate(int64_t n, int p, int s, int variant) {
    if (n < 0 || p < 1 || s < 1) return ORA_EINVAL;
    if ((int64_t)p > (n > 1 ? n : 1)) return ORA_EINVAL;       /* the method needs p <= n */
    if (variant != ORA_DET && variant != ORA_RAN) return ORA_EINVAL;
    if (variant == ORA_RAN && (int64_t)s * p - 1 > n) return ORA_EINVAL;  /* without replacement */
    return ORA_OK;
}

int64_t ora_sample_size(int p, int s, int variant) {
    return variant == ORA_DET ? (int64_t)p * s : (int64_t)p * s - 1;
}

/* ------------------------------------------------------------------------ */
/* Step O2: local sort (Figure SortD steps 2-3; Sort_Seq must be stable)      */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t idx; } item_t;

static int item_cmp(const void* pa, const void* pb) {
    const item_t* a = (const item_t*)pa;
    const item_t* b = (const item_t*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);  /* ties keep input order */
}

/* One simulated run: the arrays every step reads and writes. Each step below
 * is the work of ONE virtual processor and touches only that processor's
 * share of the output arrays, so the p processors may be simulated one after
 * the other (ora_sort) or on host threads (the driver in bsp_oracle_mt.c)
 * with the same result. */
typedef struct ora_run {
    const uint64_t* ok;  /* input order keys */
    int64_t n;
    int p;
    uint64_t* B_key;     /* block-sorted keys */
    int64_t* B_idx;      /* their original indices */
    const rec_t* S;      /* the p-1 splitters */
    int64_t* bucket;     /* bucket of every block-sorted record */
    int64_t* C;          /* C[k*p + i] */
    const int64_t* off;  /* routing offsets off[k*p + i] */
    uint64_t* Z_key;     /* routed array */
    int64_t* Z_idx;
    int64_t* perm;       /* output: original index of output element j */
    int bad;             /* set when a step finds an inconsistency */
} ora_run_t;

/* Scratch one processor needs for any step: ceil(n/p) items (local sort)
 * or the heap of the p-way merge. */
size_t ora_step_scratch_bytes(int64_t n, int p) {
    size_t a = sizeof(item_t) * (size_t)((n + p - 1) / p);
    size_t b = (sizeof(int) + 2 * sizeof(int64_t)) * (size_t)p;
    return (a > b ? a : b) + 64;
}

/* O2 for processor k: sort its share stably; B receives the sorted keys and
 * the original index of each. */
void ora_step_local_sort(ora_run_t* R, int k, void* scratch) {
    item_t* tmp = (item_t*)scratch;
    int64_t a = ora_block_start(R->n, R->p, k), b = ora_block_start(R->n, R->p, k + 1);
    for (int64_t g = a; g < b; g++) { tmp[g - a].key = R->ok[g]; tmp[g - a].idx = g; }
    qsort(tmp, (size_t)(b - a), sizeof(item_t), item_cmp);
    for (int64_t g = a; g < b; g++) { R->B_key[g] = tmp[g - a].key; R->B_idx[g] = tmp[g - a].idx; }
}

/* ------------------------------------------------------------------------ */
/* Step O3: sample extraction                                                 */
/* ------------------------------------------------------------------------ */

/* Regular oversampling (Figure SortD step 4; proof of Lemma `balance`):
 * block k of size m_k is cut into s segments of x = ceil(ceil(n/p)/s) keys,
 * the key closing each segment is taken, and the last one is the block
 * maximum. Positions past the end of a short block are clamped to its last
 * key, which stands in for the padding by the maximum key of the proof. */
static void det_sample(const uint64_t* B_key, int64_t n, int p, int s, rec_t* smp) {
    int64_t m = (n + p - 1) / p;
    int64_t x = (m + s - 1) / s;
    int64_t t = 0;
    for (int k = 0; k < p; k++) {
        int64_t a = ora_block_start(n, p, k), mk = ora_block_start(n, p, k + 1) - a;
        for (int64_t j = 1; j <= s; j++) {
            int64_t q = j * x < mk ? j * x : mk;
            smp[t].pos = a + q - 1;
            smp[t].key = B_key[a + q - 1];
            t++;
        }
    }
}

/* Random oversampling (Figure SortRI step 4): s*p - 1 distinct positions of
 * the block-sorted array, drawn uniformly without replacement as the images
 * of 0..s*p-2 under a keyed permutation of [0, n). */
static void ran_sample(const uint64_t* B_key, int64_t n, int p, int s, uint64_t seed, rec_t* smp) {
    int64_t ns = (int64_t)s * p - 1;
    for (int64_t t = 0; t < ns; t++) {
        int64_t g = ora_feistel(seed, n, t);
        smp[t].pos = g;
        smp[t].key = B_key[g];
    }
}

/* ------------------------------------------------------------------------ */
/* Steps O4-O6: sample sort, splitters, bucket of every record               */
/* ------------------------------------------------------------------------ */

/* Number of splitters strictly below record r: the splitters are sorted, so
 * this is a lower-bound search (records equal to a splitter go left). */
static int64_t bucket_of(rec_t r, const rec_t* S, int64_t nsplit) {
    int64_t lo = 0, hi = nsplit;  /* answer in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (rec_less(S[mid], r)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Steps O6, O8, O9 for one processor                                        */
/* ------------------------------------------------------------------------ */

/* O6 for processor k: partition its sorted keys by the splitters (Figure
 * SortD step 9) and count C[k][i]. The bucket ids along a sorted block never
 * decrease; a decrease would mean the block is not sorted. */
void ora_step_partition(ora_run_t* R, int k) {
    int p = R->p;
    int64_t a = ora_block_start(R->n, p, k), b = ora_block_start(R->n, p, k + 1);
    int64_t prev = 0;
    for (int64_t g = a; g < b; g++) {
        rec_t r = {R->B_key[g], g};
        int64_t bk = bucket_of(r, R->S, p - 1);
        if (bk < prev) R->bad = 1;
        prev = bk;
        R->bucket[g] = bk;
        R->C[(int64_t)k * p + bk]++;
    }
}

/* O8 for processor k: send each of its runs to its offset, order preserving
 * (Figure SortD steps 10-11). */
void ora_step_route(ora_run_t* R, int k, void* scratch) {
    int p = R->p;
    int64_t* cur = (int64_t*)scratch;  /* next free slot of each of k's runs */
    for (int i = 0; i < p; i++) cur[i] = R->off[(int64_t)k * p + i];
    int64_t a = ora_block_start(R->n, p, k), b = ora_block_start(R->n, p, k + 1);
    for (int64_t g = a; g < b; g++) {
        int64_t d = cur[R->bucket[g]]++;
        R->Z_key[d] = R->B_key[g];
        R->Z_idx[d] = R->B_idx[g];
    }
}

/* O9 for processor i: merge the sorted runs it received; on equal keys the
 * run from the lower-numbered processor goes first (Section 5.1.1). A binary
 * heap over the p run heads, ordered by (key, source). Bucket i's output
 * starts where its first run starts, off[0][i]. */
void ora_step_merge(ora_run_t* R, int i, void* scratch) {
    int p = R->p;
    int* heap = (int*)scratch;
    int64_t* head = (int64_t*)((char*)scratch + ((sizeof(int) * (size_t)p + 7) & ~(size_t)7));
    int64_t* end = head + p;
    const uint64_t* Z_key = R->Z_key;
    int64_t outpos = R->off[i];
    int hn = 0;
    for (int k = 0; k < p; k++) {
        head[k] = R->off[(int64_t)k * p + i];
        end[k] = head[k] + R->C[(int64_t)k * p + i];
        if (head[k] < end[k]) {
            /* sift up */
            int c = hn++;
            heap[c] = k;
            while (c > 0) {
                int par = (c - 1) / 2;
                int u = heap[c], v = heap[par];
                int less = Z_key[head[u]] < Z_key[head[v]] ||
                           (Z_key[head[u]] == Z_key[head[v]] && u < v);
                if (!less) break;
                heap[c] = v; heap[par] = u; c = par;
            }
        }
    }
    while (hn > 0) {
        int k = heap[0];
        R->perm[outpos++] = R->Z_idx[head[k]];
        head[k]++;
        if (head[k] == end[k]) heap[0] = heap[--hn];
        /* sift down */
        int c = 0;
        for (;;) {
            int l = 2 * c + 1, r = l + 1, m = c;
            if (l < hn) {
                int u = heap[l], v = heap[m];
                if (Z_key[head[u]] < Z_key[head[v]] || (Z_key[head[u]] == Z_key[head[v]] && u < v)) m = l;
            }
            if (r < hn) {
                int u = heap[r], v = heap[m];
                if (Z_key[head[u]] < Z_key[head[v]] || (Z_key[head[u]] == Z_key[head[v]] && u < v)) m = r;
            }
            if (m == c) break;
            int t = heap[c]; heap[c] = heap[m]; heap[m] = t; c = m;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Whole method                                                               */
/* ------------------------------------------------------------------------ */

/* Runs step(R, q, scratch) for q = 0..count-1. ora_sort passes the plain loop
 * below; bsp_oracle_mt.c passes one that spreads q over host threads. */
typedef void (*ora_step_fn)(ora_run_t* R, int q, void* scratch);
typedef int (*ora_each_fn)(ora_run_t* R, int count, ora_step_fn step, size_t scratch_bytes, void* ctx);

static int each_sequential(ora_run_t* R, int count, ora_step_fn step, size_t scratch_bytes, void* ctx) {
    (void)ctx;
    void* scratch = malloc(scratch_bytes);
    if (!scratch) return ORA_ENOMEM;
    for (int q = 0; q < count; q++) step(R, q, scratch);
    free(scratch);
    return ORA_OK;
}

static void step_partition(ora_run_t* R, int k, void* scratch) { (void)scratch; ora_step_partition(R, k); }

/*
 * The method with a given way of running the per-processor steps (see
 * ora_sort for the arguments).
 */
int ora_sort_driver(const uint64_t* ok, int64_t n, int p, int s, int variant, uint64_t seed,
                    int64_t* perm, int64_t* B_idx_out, uint64_t* smp_key, int64_t* smp_pos,
                    uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out,
                    int untagged, ora_each_fn each, void* ctx) {
    int rc = ora_validate(n, p, s, variant);
    if (rc) return rc;
    if (n <= 1) {
        if (n == 1) perm[0] = 0;
        if (n == 1 && B_idx_out) B_idx_out[0] = 0;
        if (n == 1 && Z_idx_out) Z_idx_out[0] = 0;
        if (C_out) C_out[0] = n;
        int64_t ns = n == 1 ? ora_sample_size(p, s, variant) : 0;
        for (int64_t t = 0; t < ns; t++) {
            if (smp_key) smp_key[t] = ok[0];
            if (smp_pos) smp_pos[t] = 0;
        }
        return ORA_OK;
    }
    int64_t ns = ora_sample_size(p, s, variant);
    size_t scr = ora_step_scratch_bytes(n, p);
    uint64_t* B_key = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t* B_idx = (int64_t*)malloc(sizeof(int64_t) * n);
    rec_t* smp = (rec_t*)malloc(sizeof(rec_t) * (ns > 0 ? ns : 1));
    rec_t* S = (rec_t*)malloc(sizeof(rec_t) * p);
    int64_t* C = (int64_t*)calloc((size_t)p * p, sizeof(int64_t));
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * p * p);
    int64_t* Z_idx = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* Z_key = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t* bucket = (int64_t*)malloc(sizeof(int64_t) * n);
    ora_run_t R;
    memset(&R, 0, sizeof(R));
    if (!B_key || !B_idx || !smp || !S || !C || !off || !Z_idx || !Z_key || !bucket) {
        rc = ORA_ENOMEM;
        goto done;
    }
    R.ok = ok; R.n = n; R.p = p; R.B_key = B_key; R.B_idx = B_idx; R.S = S; R.bucket = bucket;
    R.C = C; R.off = off; R.Z_key = Z_key; R.Z_idx = Z_idx; R.perm = perm;

    /* O2: every processor sorts its share (stable). */
    rc = each(&R, p, ora_step_local_sort, scr, ctx);
    if (rc) goto done;
    if (B_idx_out) memcpy(B_idx_out, B_idx, sizeof(int64_t) * n);

    /* O3: sample. O4: sort it by (key, tag). */
    if (variant == ORA_DET) det_sample(B_key, n, p, s, smp);
    else ran_sample(B_key, n, p, s, seed, smp);
    qsort(smp, (size_t)ns, sizeof(rec_t), rec_cmp);
    for (int64_t t = 0; t < ns; t++) {
        if (smp_key) smp_key[t] = smp[t].key;
        if (smp_pos) smp_pos[t] = smp[t].pos;
    }

    /* O5: p-1 evenly spaced splitters, the sample records at 1-based ranks
     * s, 2s, ..., (p-1)s (Figure SortD step 6, Figure SortRI step 7). */
    for (int i = 1; i < p; i++) S[i - 1] = smp[(int64_t)i * s - 1];
    for (int i = 1; i < p; i++) {
        if (spl_key) spl_key[i - 1] = S[i - 1].key;
        if (spl_pos) spl_pos[i - 1] = S[i - 1].pos;
    }
    /* Duplicate handling switched off (the ablation of Section 6.4): the
     * splitters lose their tags, so a key equal to a splitter is never above
     * it: every splitter compares as (key, +infinity) and buckets are decided
     * by the key alone. */
    if (untagged)
        for (int i = 1; i < p; i++) S[i - 1].pos = INT64_MAX;

    /* O6: partition each processor's sorted keys by the splitters and count. */
    rc = each(&R, p, step_partition, 64, ctx);
    if (rc) goto done;
    if (R.bad) { rc = ORA_EINVAL; goto done; }  /* cannot happen: blocks are sorted */
    if (C_out) memcpy(C_out, C, sizeof(int64_t) * p * p);

    /* O7: the p independent prefix computations: bucket i starts after all
     * smaller buckets, and within bucket i the keys from processor k follow
     * those of processors 0..k-1. */
    {
        int64_t base = 0;
        for (int i = 0; i < p; i++) {
            int64_t run = base;
            for (int k = 0; k < p; k++) {
                off[(int64_t)k * p + i] = run;
                run += C[(int64_t)k * p + i];
            }
            base = run;
        }
    }

    /* O8: routing, order preserving. */
    rc = each(&R, p, ora_step_route, scr, ctx);
    if (rc) goto done;
    if (Z_idx_out) memcpy(Z_idx_out, Z_idx, sizeof(int64_t) * n);

    /* O9: every processor merges the runs it received. */
    rc = each(&R, p, ora_step_merge, scr, ctx);

done:
    free(B_key); free(B_idx); free(smp); free(S); free(C); free(off);
    free(Z_idx); free(Z_key); free(bucket);
    return rc;
}

/*
 * ora_sort: sorts n order keys with p simulated processors and oversampling
 * parameter s (the splitter stride of the sorted sample), the processors
 * simulated one after the other.
 *   perm[j]     original index of output element j (required)
 *   B_idx[g]    original index of the block-sorted array element g (optional)
 *   smp_key/pos sorted sample records (optional, ora_sample_size entries)
 *   spl_key/pos the p-1 splitters (optional)
 *   C[k*p+i]    keys of processor k that fall in bucket i (optional)
 *   Z_idx[j]    original index of element j after routing (optional)
 * Returns ORA_OK, ORA_EINVAL (arguments) or ORA_ENOMEM.
 */
int ora_sort(const uint64_t* ok, int64_t n, int p, int s, int variant, uint64_t seed,
             int64_t* perm, int64_t* B_idx_out, uint64_t* smp_key, int64_t* smp_pos,
             uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out) {
    return ora_sort_driver(ok, n, p, s, variant, seed, perm, B_idx_out, smp_key, smp_pos, spl_key, spl_pos,
                           C_out, Z_idx_out, 0, each_sequential, NULL);
}

/* ora_sort with the duplicate handling switched off (untagged splitters). */
int ora_sort_untagged(const uint64_t* ok, int64_t n, int p, int s, int variant, uint64_t seed,
                      int64_t* perm, int64_t* B_idx_out, uint64_t* smp_key, int64_t* smp_pos,
                      uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out) {
    return ora_sort_driver(ok, n, p, s, variant, seed, perm, B_idx_out, smp_key, smp_pos, spl_key, spl_pos,
                           C_out, Z_idx_out, 1, each_sequential, NULL);
}

/* ------------------------------------------------------------------------ */
/* Sort_Ran_BSP (Figure SortR): sample, route, then sort locally             */
/* ------------------------------------------------------------------------ */

/*
 * ora_sort_sr: the sample-sort ordering of Section 5.2, Figure SortR, with the
 * duplicate handling of Section 5.1.1, for p simulated processors holding
 * the contiguous blocks of the UNSORTED input:
 *   R1 (step 2)    a sample of s*p - 1 input positions drawn uniformly without
 *                  replacement: the images of 0..s*p-2 under the keyed
 *                  permutation of [0, n); each is the record (key, g) with g its
 *                  input position, which orders like the tag (processor, local
 *                  index) since there is no local sort before the sample.
 *   R2 (steps 5-6) the sample sorted by (key, g); splitters at 1-based ranks
 *                  s, 2s, ..., (p-1)s.
 *   R3 (step 9)    the bucket of every input record: the number of splitters
 *                  strictly below it; C[k][i] counts processor k's records of
 *                  bucket i.
 *   R4 (steps 10-11) routing, order preserving: bucket i gathers processor 0's
 *                  records of bucket i in input order, then processor 1's, ...
 *   R5 (step 12)   every processor sorts what it received, stably by key, so
 *                  equal keys keep the routed order, which is input order.
 * The output is therefore the stable sort of the input. Outputs as ora_sort
 * (perm, sample records, splitters, C, Z_idx); the sample positions and
 * Z_idx are input positions.
 */
int ora_sort_sr(const uint64_t* ok, int64_t n, int p, int s, uint64_t seed,
                int64_t* perm, uint64_t* smp_key, int64_t* smp_pos,
                uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* Z_idx_out) {
    int rc = ora_validate(n, p, s, ORA_RAN);
    if (rc) return rc;
    if (n <= 1) {
        if (n == 1) perm[0] = 0;
        if (n == 1 && Z_idx_out) Z_idx_out[0] = 0;
        if (C_out) C_out[0] = n;
        return ORA_OK;
    }
    int64_t ns = (int64_t)s * p - 1;
    rec_t* smp = (rec_t*)malloc(sizeof(rec_t) * (ns > 0 ? ns : 1));
    rec_t* S = (rec_t*)malloc(sizeof(rec_t) * p);
    int64_t* C = (int64_t*)calloc((size_t)p * p, sizeof(int64_t));
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * p * p);
    int64_t* bucket = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* Z_idx = (int64_t*)malloc(sizeof(int64_t) * n);
    item_t* tmp = (item_t*)malloc(sizeof(item_t) * n);
    if (!smp || !S || !C || !off || !bucket || !Z_idx || !tmp) { rc = ORA_ENOMEM; goto done_sr; }

    /* R1, R2 */
    for (int64_t t = 0; t < ns; t++) {
        int64_t g = ora_feistel(seed, n, t);
        smp[t].pos = g;
        smp[t].key = ok[g];
    }
    qsort(smp, (size_t)ns, sizeof(rec_t), rec_cmp);
    for (int64_t t = 0; t < ns; t++) {
        if (smp_key) smp_key[t] = smp[t].key;
        if (smp_pos) smp_pos[t] = smp[t].pos;
    }
    for (int i = 1; i < p; i++) {
        S[i - 1] = smp[(int64_t)i * s - 1];
        if (spl_key) spl_key[i - 1] = S[i - 1].key;
        if (spl_pos) spl_pos[i - 1] = S[i - 1].pos;
    }

    /* R3 */
    for (int k = 0; k < p; k++) {
        int64_t a = ora_block_start(n, p, k), b = ora_block_start(n, p, k + 1);
        for (int64_t g = a; g < b; g++) {
            rec_t r = {ok[g], g};
            bucket[g] = bucket_of(r, S, p - 1);
            C[(int64_t)k * p + bucket[g]]++;
        }
    }
    if (C_out) memcpy(C_out, C, sizeof(int64_t) * p * p);

    /* R4: offsets as in Figure SortD step 9, then the order-preserving route */
    {
        int64_t base = 0;
        for (int i = 0; i < p; i++) {
            int64_t run = base;
            for (int k = 0; k < p; k++) {
                off[(int64_t)k * p + i] = run;
                run += C[(int64_t)k * p + i];
            }
            base = run;
        }
        for (int k = 0; k < p; k++) {
            int64_t a = ora_block_start(n, p, k), b = ora_block_start(n, p, k + 1);
            for (int64_t g = a; g < b; g++) Z_idx[off[(int64_t)k * p + bucket[g]]++] = g;
        }
    }
    if (Z_idx_out) memcpy(Z_idx_out, Z_idx, sizeof(int64_t) * n);

    /* R5: bucket i now spans [base_i, base_i + size_i) of Z (off[k][i] has
     * advanced to the end of processor k's run): sort it stably by key. */
    {
        int64_t lo = 0;
        for (int i = 0; i < p; i++) {
            int64_t hi = off[(int64_t)(p - 1) * p + i];
            for (int64_t j = lo; j < hi; j++) { tmp[j - lo].key = ok[Z_idx[j]]; tmp[j - lo].idx = j; }
            /* ties by routed position: the stable order */
            qsort(tmp, (size_t)(hi - lo), sizeof(item_t), item_cmp);
            for (int64_t j = lo; j < hi; j++) perm[j] = Z_idx[tmp[j - lo].idx];
            lo = hi;
        }
    }

done_sr:
    free(smp); free(S); free(C); free(off); free(bucket); free(Z_idx); free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Iterative Sort_Det_BSP: m rounds of partitioning and merging               */
/* ------------------------------------------------------------------------ */

/* k with k^m = p (k >= 2 unless p = 1), or 0 when p is not an m-th power. */
int ora_iter_k(int p, int m) {
    if (p < 1 || m < 1) return 0;
    if (p == 1) return 1;
    for (int k = 2; k <= p; k++) {
        int64_t v = 1;
        for (int r = 0; r < m && v <= p; r++) v *= k;
        if (v == p) return k;
        if (v > p) return 0;
    }
    return 0;
}

/*
 * ora_sort_iter: the iterative version of Sort_Det_BSP (Section 5.1): the
 * local sort, then m iterations of partitioning and merging; each iteration
 * splits every current bucket into k further buckets, p = k^m processors,
 * regular oversampling s. The paper describes the iteration in words only;
 * this is the reading implemented here (m = 1 is exactly ora_sort, DET):
 *   I0 (phase 1)  every processor sorts its block stably (as O2): array A;
 *                 one group, the whole array, held by all p processors.
 * Round r = 1..m, for every group g (its segment of A, z records, held by q
 * processors; processor j owns the share [ora_block_start(z, q, j),
 * ora_block_start(z, q, j + 1)) of the segment, sorted):
 *   I1 (phase 2)  regular sample of each share, as O3 with the share length
 *                 bound ceil(z/q). No share is ever empty: a record fills at
 *                 most s sample slots (the clamped last position of its
 *                 share), and a sub-bucket takes at least t - (s - 1) of the
 *                 t sample ranks between its splitters (only copies of the
 *                 lower splitter are lost), so it holds at least
 *                 ceil((t - s + 1) / s) = q/k records, one per processor of
 *                 the next round; round 1 has p <= n.
 *   I2            the q*s sample records of the group sorted by (key, tag);
 *                 k-1 splitters at the 1-based ranks t, 2t, ..., (k-1)t,
 *                 t = q*s/k (for m = 1: t = s, as O5).
 *   I3            every processor partitions its share by the splitters,
 *                 ties decided by the tag (as O6), and counts.
 *   I4            routing, order preserving (as O7-O8 inside the group):
 *                 sub-bucket b gathers the processors' runs of bucket b in
 *                 processor order; the sub-buckets follow each other in b
 *                 order in the group's segment; sub-bucket b becomes group
 *                 g*k + b, held by q/k processors.
 *   I5 (phase 3)  every processor of a new group takes its even share of the
 *                 routed sequence and merges the sorted pieces it holds, the
 *                 earlier piece first on equal keys (a stable sort of the
 *                 share, which is the same thing since the pieces are sorted).
 * Tags are positions in the current array: every round keeps equal keys in
 * input order, so they order exactly like the original (processor, index).
 * Outputs (optional unless stated):
 *   perm[j]                original index of output element j (required)
 *   spl_key/spl_pos[p-1]   the splitters of round 1 (k-1), then of the k groups
 *                          of round 2 (k-1 each, in group order), ...; pos is
 *                          the position in the round's input array
 *   C[m*p*k]               round r, processor (global number g*q + j), bucket b
 *   A_idx[m*n]             original index of every element after round r
 * Returns ORA_OK, ORA_EINVAL (arguments) or ORA_ENOMEM.
 */
int ora_sort_iter(const uint64_t* ok, int64_t n, int p, int s, int m, int64_t* perm,
                  uint64_t* spl_key, int64_t* spl_pos, int64_t* C_out, int64_t* A_idx_out) {
    int rc = ora_validate(n, p, s, ORA_DET);
    if (rc) return rc;
    const int k = ora_iter_k(p, m);
    if (k == 0) return ORA_EINVAL;
    if (n <= 1 || p == 1) {
        /* one processor: its local sort is the output */
        item_t* tmp = (item_t*)malloc(sizeof(item_t) * (size_t)(n > 0 ? n : 1));
        if (!tmp) return ORA_ENOMEM;
        for (int64_t g = 0; g < n; g++) { tmp[g].key = ok[g]; tmp[g].idx = g; }
        qsort(tmp, (size_t)n, sizeof(item_t), item_cmp);
        for (int64_t g = 0; g < n; g++) perm[g] = tmp[g].idx;
        for (int r = 0; r < m && A_idx_out; r++) memcpy(A_idx_out + (int64_t)r * n, perm, sizeof(int64_t) * n);
        if (C_out)
            for (int r = 0; r < m; r++)
                for (int64_t e = 0; e < (int64_t)p * k; e++) C_out[(int64_t)r * p * k + e] = e == 0 ? n : 0;
        free(tmp);
        return ORA_OK;
    }
    uint64_t* A_key = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t* A_idx = (int64_t*)malloc(sizeof(int64_t) * n);
    uint64_t* Z_key = (uint64_t*)malloc(sizeof(uint64_t) * n);
    int64_t* Z_idx = (int64_t*)malloc(sizeof(int64_t) * n);
    item_t* tmp = (item_t*)malloc(sizeof(item_t) * n);
    int64_t* gst = (int64_t*)malloc(sizeof(int64_t) * ((size_t)p + 1));   /* group starts */
    int64_t* ngst = (int64_t*)malloc(sizeof(int64_t) * ((size_t)p + 1));
    rec_t* smp = (rec_t*)malloc(sizeof(rec_t) * (size_t)p * s);
    rec_t* S = (rec_t*)malloc(sizeof(rec_t) * (size_t)k);
    int64_t* C = (int64_t*)malloc(sizeof(int64_t) * (size_t)p * k);      /* one group: q x k */
    int64_t* rs = (int64_t*)malloc(sizeof(int64_t) * (size_t)p * k);     /* run starts in Z */
    if (!A_key || !A_idx || !Z_key || !Z_idx || !tmp || !gst || !ngst || !smp || !S || !C || !rs) {
        rc = ORA_ENOMEM;
        goto done_it;
    }
    /* I0: local sort of the p blocks */
    for (int j = 0; j < p; j++) {
        int64_t a = ora_block_start(n, p, j), b = ora_block_start(n, p, j + 1);
        for (int64_t g = a; g < b; g++) { tmp[g - a].key = ok[g]; tmp[g - a].idx = g; }
        qsort(tmp, (size_t)(b - a), sizeof(item_t), item_cmp);
        for (int64_t g = a; g < b; g++) { A_key[g] = tmp[g - a].key; A_idx[g] = tmp[g - a].idx; }
    }
    int G = 1, q = p;
    int64_t nspl = 0;
    gst[0] = 0;
    gst[1] = n;
    for (int r = 0; r < m; r++) {
        const int q2 = q / k;
        for (int g = 0; g < G; g++) {
            const int64_t gs = gst[g], z = gst[g + 1] - gs;
            /* I1: regular sample of every share */
            const int64_t xm = (z + q - 1) / q, x = (xm + s - 1) / s;
            int64_t t = 0;
            for (int j = 0; j < q; j++) {
                const int64_t a = gs + ora_block_start(z, q, j), mj = ora_block_start(z, q, j + 1) - (a - gs);
                if (mj == 0) { rc = ORA_EINVAL; goto done_it; }  /* cannot happen (I1) */
                for (int64_t i = 1; i <= s; i++) {
                    const int64_t qq = i * x < mj ? i * x : mj;
                    smp[t].key = A_key[a + qq - 1];
                    smp[t].pos = a + qq - 1;
                    t++;
                }
            }
            /* I2: sort, splitters */
            qsort(smp, (size_t)t, sizeof(rec_t), rec_cmp);
            const int64_t stride = (int64_t)q * s / k;
            for (int i = 1; i < k; i++) {
                S[i - 1] = smp[(int64_t)i * stride - 1];
                if (spl_key) spl_key[nspl] = S[i - 1].key;
                if (spl_pos) spl_pos[nspl] = S[i - 1].pos;
                nspl++;
            }
            /* I3: partition every share, count */
            memset(C, 0, sizeof(int64_t) * (size_t)q * k);
            for (int j = 0; j < q; j++) {
                const int64_t a = gs + ora_block_start(z, q, j), b = gs + ora_block_start(z, q, j + 1);
                int64_t prev = 0;
                for (int64_t x2 = a; x2 < b; x2++) {
                    rec_t rr = {A_key[x2], x2};
                    int64_t bk = bucket_of(rr, S, k - 1);
                    if (bk < prev) { rc = ORA_EINVAL; goto done_it; }  /* cannot happen: shares are sorted */
                    prev = bk;
                    C[(int64_t)j * k + bk]++;
                }
            }
            if (C_out)
                for (int64_t e = 0; e < (int64_t)q * k; e++) C_out[(int64_t)r * p * k + (int64_t)g * q * k + e] = C[e];
            /* I4: route, order preserving; sub-bucket b = new group g*k + b */
            {
                int64_t base = gs;
                for (int b = 0; b < k; b++) {
                    ngst[(int64_t)g * k + b] = base;
                    for (int j = 0; j < q; j++) {
                        rs[(int64_t)j * k + b] = base;
                        base += C[(int64_t)j * k + b];
                    }
                }
                for (int j = 0; j < q; j++) {
                    const int64_t a = gs + ora_block_start(z, q, j), b = gs + ora_block_start(z, q, j + 1);
                    for (int64_t x2 = a; x2 < b; x2++) {
                        rec_t rr = {A_key[x2], x2};
                        const int64_t bk = bucket_of(rr, S, k - 1);
                        const int64_t d = rs[(int64_t)j * k + bk]++;
                        Z_key[d] = A_key[x2];
                        Z_idx[d] = A_idx[x2];
                    }
                }
            }
        }
        ngst[(int64_t)G * k] = n;
        /* I5: every processor of every new group merges its share */
        for (int g2 = 0; g2 < G * k; g2++) {
            const int64_t us = ngst[g2], z2 = ngst[g2 + 1] - us;
            for (int j = 0; j < q2; j++) {
                const int64_t a = us + ora_block_start(z2, q2, j), b = us + ora_block_start(z2, q2, j + 1);
                for (int64_t x2 = a; x2 < b; x2++) { tmp[x2 - a].key = Z_key[x2]; tmp[x2 - a].idx = x2; }
                qsort(tmp, (size_t)(b - a), sizeof(item_t), item_cmp);
                for (int64_t x2 = a; x2 < b; x2++) {
                    A_key[x2] = tmp[x2 - a].key;
                    A_idx[x2] = Z_idx[tmp[x2 - a].idx];
                }
            }
        }
        if (A_idx_out) memcpy(A_idx_out + (int64_t)r * n, A_idx, sizeof(int64_t) * n);
        G *= k;
        q = q2;
        memcpy(gst, ngst, sizeof(int64_t) * ((size_t)G + 1));
    }
    memcpy(perm, A_idx, sizeof(int64_t) * n);

done_it:
    free(A_key); free(A_idx); free(Z_key); free(Z_idx); free(tmp); free(gst); free(ngst);
    free(smp); free(S); free(C); free(rs);
    return rc;
}

/* Bucket of each record (key, g) of a block-sorted array against given
 * splitters: the definition used by step O6, exported so that a per-key GPU
 * ranking can be compared against it. */
void ora_rank(const uint64_t* B_key, int64_t n, const uint64_t* spl_key, const int64_t* spl_pos,
              int nsplit, int64_t* bucket) {
    rec_t* S = (rec_t*)malloc(sizeof(rec_t) * (nsplit > 0 ? nsplit : 1));
    for (int i = 0; i < nsplit; i++) { S[i].key = spl_key[i]; S[i].pos = spl_pos[i]; }
    for (int64_t g = 0; g < n; g++) {
        rec_t r = {B_key[g], g};
        bucket[g] = bucket_of(r, S, nsplit);
    }
    free(S);
}

/* ------------------------------------------------------------------------ */
/* Learned bucketing reference (not in the paper): a two-stage CDF model      */
/* ------------------------------------------------------------------------ */

/*
 * The model maps a key to a predicted bucket; the exact splitter check then
 * corrects it, so it only affects speed. Definitions (double precision):
 *   x(u)  = (u - lo) / (hi - lo) for an order key u, lo/hi the smallest and
 *           largest sorted-sample key (x = 0 when hi == lo)
 *   root  r(x) = a (x - mu_r) + b ; leaf(x) = clamp(floor(L r(x)), 0, L-1)
 *   leaf  f_l(x) = c_l (x - mu_l) + d_l ; bucket(x) = clamp(floor(p f), 0, p-1)
 * Training data: the sorted sample, record t with target y_t = (t+0.5)/(p s),
 * whose bucket under the splitter rule is floor(t/s).
 * Loss: (1/N) sum_t (f(x_t) - y_t)^2 over the N sample records.
 */

/* Gradient and Gram (Hessian) sums of the loss of one linear model
 * f(x) = c (x - mu) + d over the records t with leaf[t] == l, for all L
 * models at once. Outputs per model (all scaled by 2/N):
 *   g[2l]   = dLoss/dc, g[2l+1] = dLoss/dd
 *   h[3l..] = (sum (x-mu)^2, sum (x-mu), count)
 * Also returns the loss. */
double ora_rmi_grad(const double* x, const double* y, const int32_t* leaf, int64_t N, int L,
                    const double* c, const double* d, const double* mu, double* g, double* h) {
    double loss = 0.0;
    for (int l = 0; l < L; l++) { g[2 * l] = g[2 * l + 1] = 0.0; h[3 * l] = h[3 * l + 1] = h[3 * l + 2] = 0.0; }
    for (int64_t t = 0; t < N; t++) {
        int l = leaf[t];
        double dx = x[t] - mu[l];
        double r = c[l] * dx + d[l] - y[t];
        loss += r * r;
        g[2 * l] += r * dx;
        g[2 * l + 1] += r;
        h[3 * l] += dx * dx;
        h[3 * l + 1] += dx;
        h[3 * l + 2] += 1.0;
    }
    double sc = N > 0 ? 2.0 / (double)N : 0.0;
    for (int l = 0; l < L; l++) {
        g[2 * l] *= sc; g[2 * l + 1] *= sc;
        h[3 * l] *= sc; h[3 * l + 1] *= sc; h[3 * l + 2] *= sc;
    }
    return N > 0 ? loss / (double)N : 0.0;
}

/* One Newton step per model from gradient g and Gram h: for a quadratic loss
 * this lands on the least-squares solution. A model whose Gram matrix is
 * singular (fewer than two distinct x) only moves its intercept; a model with
 * no records keeps its parameters. */
void ora_rmi_newton(int L, const double* g, const double* h, double* c, double* d) {
    for (int l = 0; l < L; l++) {
        double sxx = h[3 * l], sx = h[3 * l + 1], sn = h[3 * l + 2];
        if (sn <= 0.0) continue;
        double det = sxx * sn - sx * sx;
        if (det > 1e-300 && sxx > 0.0 && det > 1e-12 * sxx * sn) {
            double dc = (sn * g[2 * l] - sx * g[2 * l + 1]) / det;
            double dd = (-sx * g[2 * l] + sxx * g[2 * l + 1]) / det;
            c[l] -= dc;
            d[l] -= dd;
        } else {
            d[l] -= g[2 * l + 1] / sn;
        }
    }
}

/* Full reference fit on sorted sample order keys; writes the model.
 * root: (a, b, mu_r); leaves: c[L], d[L], mu[L]; lo/hi as defined above.
 * Leaves with no sample take c = 0 and d = (number of samples in lower
 * leaves) / (p s), so that they predict the bucket where their keys belong. */
void ora_rmi_fit(const uint64_t* smp_key, int64_t N, int p, int s, int L, int iters,
                 double* root3, double* c, double* d, double* mu, double* lohi) {
    double lo = N ? (double)smp_key[0] : 0.0, hi = N ? (double)smp_key[N - 1] : 0.0;
    double inv = hi > lo ? 1.0 / (hi - lo) : 0.0;
    lohi[0] = lo; lohi[1] = hi;
    double* x = (double*)malloc(sizeof(double) * (N ? N : 1));
    double* y = (double*)malloc(sizeof(double) * (N ? N : 1));
    int32_t* lf = (int32_t*)malloc(sizeof(int32_t) * (N ? N : 1));
    double* g = (double*)malloc(sizeof(double) * 2 * (L > 1 ? L : 1));
    double* h = (double*)malloc(sizeof(double) * 3 * (L > 1 ? L : 1));
    for (int64_t t = 0; t < N; t++) {
        x[t] = ((double)smp_key[t] - lo) * inv;
        y[t] = ((double)t + 0.5) / ((double)p * (double)s);
        lf[t] = 0;
    }
    /* root */
    double mur = 0.0;
    for (int64_t t = 0; t < N; t++) mur += x[t];
    mur = N ? mur / (double)N : 0.0;
    double ra = 0.0, rb = 0.0;
    for (int it = 0; it < iters; it++) {
        double gg[2], hh[3];
        ora_rmi_grad(x, y, lf, N, 1, &ra, &rb, &mur, gg, hh);
        ora_rmi_newton(1, gg, hh, &ra, &rb);
    }
    root3[0] = ra; root3[1] = rb; root3[2] = mur;
    /* leaf assignment by the fitted root */
    for (int64_t t = 0; t < N; t++) {
        double r = ra * (x[t] - mur) + rb;
        double f = floor(r * (double)L);
        lf[t] = f < 0 ? 0 : (f > L - 1 ? L - 1 : (int32_t)f);
    }
    /* leaf centres: mean x of the leaf's records */
    int64_t* cnt = (int64_t*)calloc((size_t)L, sizeof(int64_t));
    for (int l = 0; l < L; l++) { mu[l] = 0.0; c[l] = 0.0; d[l] = 0.0; }
    for (int64_t t = 0; t < N; t++) { mu[lf[t]] += x[t]; cnt[lf[t]]++; }
    for (int l = 0; l < L; l++) mu[l] = cnt[l] ? mu[l] / (double)cnt[l] : 0.0;
    for (int it = 0; it < iters; it++) {
        ora_rmi_grad(x, y, lf, N, L, c, d, mu, g, h);
        ora_rmi_newton(L, g, h, c, d);
    }
    int64_t below = 0;
    for (int l = 0; l < L; l++) {
        if (cnt[l] == 0) { c[l] = 0.0; d[l] = (double)below / ((double)p * (double)s); }
        below += cnt[l];
    }
    free(cnt); free(x); free(y); free(lf); free(g); free(h);
}

/* Predicted bucket of an order key under a fitted model (double precision). */
int64_t ora_rmi_predict(uint64_t u, int p, int L, const double* root3, const double* c, const double* d,
                        const double* mu, const double* lohi) {
    double inv = lohi[1] > lohi[0] ? 1.0 / (lohi[1] - lohi[0]) : 0.0;
    double x = ((double)u - lohi[0]) * inv;
    double r = root3[0] * (x - root3[2]) + root3[1];
    double fl = floor(r * (double)L);
    int l = fl < 0 ? 0 : (fl > L - 1 ? L - 1 : (int)fl);
    double f = c[l] * (x - mu[l]) + d[l];
    double fb = floor(f * (double)p);
    return fb < 0 ? 0 : (fb > p - 1 ? p - 1 : (int64_t)fb);
}
