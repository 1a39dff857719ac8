// bsps_segmented.h -- batched sort of many independent segments.
//
// Segment i of n_i keys is sorted with its own p_i virtual processors and
// oversampling s_i (Figure SortD per segment). p_i is chosen so that every
// block fits one tile: each block is then sorted by one workgroup, and a
// segment with p_i = 1 is finished by that sort. The other steps run for all
// segments in one launch each, driven by tables:
//   seg[8*i .. 8*i+7] = start, n, p, s, first block, large, -, -
//   (large = 1: the segment's bucket counts come from the learned model below)
//   soff[i] / poff[i] / coff[i]: prefix offsets of the segments' samples
//   (p*s), splitters (p-1) and count rows ((p+1)*p); zero-sized for p = 1
//   btab[4*b ..]      = block start, size, segment, block-sample offset
#pragma once
#include "bsps_kernels.h"
#include "bsps_learned.h"

constexpr int SEGW = 8;

// Largest segment index s in [0, nseg) with off[s] <= idx (a segment that owns idx).
__device__ __forceinline__ int seg_of(const u32* off, int nseg, u32 idx) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Regular sample of every segment (Figure SortD step 4 inside each segment).
template <typename K>
__global__ void k_seg_det_sample(const K* B, const u32* seg, const u32* soff, int nseg, K* skey, u32* spos) {
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= soff[nseg]) return;
    const int sg = seg_of(soff, nseg, t);
    const u32* d = seg + SEGW * sg;
    const i64 start = d[0], n = d[1];
    const int p = (int)d[2], s = (int)d[3];
    const u32 local = t - soff[sg];
    const int k = (int)(local / s), j = (int)(local % s) + 1;
    const i64 st = start + blk_start(n, p, k), mk = blk_start(n, p, k + 1) - blk_start(n, p, k);
    const i64 m = (n + p - 1) / p, x = (m + s - 1) / s;
    const i64 q = ((i64)j * x < mk ? (i64)j * x : mk) - 1;
    skey[t] = B[st + q];
    spos[t] = (u32)(st + q);
}

template <typename K>
__global__ void k_seg_splitters(const K* ssk, const u32* ssp, const u32* seg, const u32* soff, const u32* poff,
                                int nseg, K* pk, u32* pp) {
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= poff[nseg]) return;
    const int sg = seg_of(poff, nseg, t);
    const int s = (int)seg[SEGW * sg + 3];
    const u32 i = t - poff[sg] + 1;
    pk[t] = ssk[soff[sg] + i * s - 1];
    pp[t] = ssp[soff[sg] + i * s - 1];
}

// cntT of every segment: row i, column k = keys of block k at or below splitter i.
template <typename K>
__global__ void k_seg_count(const K* B, const u32* seg, const u32* poff, const u32* coff, int nseg, const K* pk,
                            const u32* pp, u32* cntT) {
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= coff[nseg]) return;
    const int sg = seg_of(coff, nseg, t);
    const u32* d = seg + SEGW * sg;
    if (d[5]) return;  // counted by k_sl_rank
    const i64 start = d[0], n = d[1];
    const int p = (int)d[2];
    const u32 local = t - coff[sg];
    const int i = (int)(local / p), k = (int)(local % p);
    const i64 st = start + blk_start(n, p, k), mk = blk_start(n, p, k + 1) - blk_start(n, p, k);
    u32 res;
    if (i == 0) res = 0;
    else if (i == p) res = (u32)mk;
    else {
        const K sk = pk[poff[sg] + i - 1];
        const u32 sp = pp[poff[sg] + i - 1];
        u32 lo = 0, hi = (u32)mk;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (rec_le<K>(B[st + mid], (u32)(st + mid), sk, sp)) lo = mid + 1; else hi = mid;
        }
        res = lo;
    }
    cntT[t] = res;
}

// Merge tables of one size class: group g = (segment, bucket) from gtab,
// runs = the segment's blocks, padded with empty runs up to R. Samples of a
// run are the block samples (every yb-th key of the block) inside it.
__global__ __launch_bounds__(256) void k_seg_bucket_tables(const u32* gtab, int R, const u32* seg, const u32* coff,
                                                           const u32* cntT, const u32* btab, u32 yb, u32* run_start,
                                                           u32* run_len, u32* out_base, u32* sdesc) {
    __shared__ u32 red[4];
    const int g = blockIdx.x, t = threadIdx.x;
    const int sg = (int)gtab[2 * g], i = (int)gtab[2 * g + 1];
    const u32* d = seg + SEGW * sg;
    const int p = (int)d[2];
    const u32 blk0 = d[4];
    const u32* ct = cntT + coff[sg];
    u32 acc = 0;
    for (int k = t; k < R; k += 256) {
        const i64 gk = (i64)g * R + k;
        u32* sd = sdesc + gk * 4;
        if (k < p) {
            const u32 a0 = ct[(i64)i * p + k], a1 = ct[(i64)(i + 1) * p + k];
            const u32* bt = btab + 4 * (i64)(blk0 + k);
            const u32 bs = bt[0], bo = bt[3];
            acc += a0;
            run_start[gk] = bs + a0;
            run_len[gk] = a1 - a0;
            const u32 jlo = a0 / yb, jhi = a1 / yb;
            sd[0] = bo + jlo;
            sd[1] = jhi - jlo;
            sd[2] = bs + (jlo + 1) * yb - 1;
            sd[3] = yb;
        } else {
            run_start[gk] = 0;
            run_len[gk] = 0;
            sd[0] = 0; sd[1] = 0; sd[2] = 0; sd[3] = yb;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) out_base[g] = d[0] + red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- learned bucketing of large segments
//
// Segments above a size threshold get their own model (the two-stage CDF
// model of k_rank, SEG_LEAVES leaves), trained on the segment's sorted
// sample by batched forward / backward / Newton-update kernels, and every key
// of their blocks is ranked by it with the exact splitter check. The block's
// bucket histogram gives its column of the count table, so the fused merge
// reads the same runs as with the splitter search. Tables:
//   lseg[j]         segment of large segment j (j < NL)
//   lcs[j]          prefix of their sample sizes (NL + 1 entries)
//   lblk[2e], [2e+1] block (btab index) and its large-segment number
// Models: NL records of SEG_MODEL_BYTES (header, then SEG_LEAVES triples).
// Model indices: stage 0 = j (the root), stage 1 = j * SEG_LEAVES + leaf.

constexpr int SEG_LEAVES = 64;
constexpr u32 SEG_MODEL_BYTES = (u32)sizeof(ModelHdr) + 12u * SEG_LEAVES;

__device__ __forceinline__ ModelHdr* seg_model(void* models, u32 j) {
    return (ModelHdr*)((char*)models + (size_t)j * SEG_MODEL_BYTES);
}
__device__ __forceinline__ float* sl_params(void* models, int stage, u32 m) {
    if (stage == 0) return &seg_model(models, m)->a;  // a, b, mu_r
    return (float*)(seg_model(models, m / SEG_LEAVES) + 1) + 3 * (m % SEG_LEAVES);
}

template <typename K>
__global__ void k_sl_init(const K* ssk, const u32* seg, const u32* soff, const u32* lseg, int NL, void* models) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NL) return;
    const u32 sg = lseg[j];
    ModelHdr* h = seg_model(models, (u32)j);
    const K lo = ssk[soff[sg]], hi = ssk[soff[sg + 1] - 1];
    h->lo = (double)lo;
    h->hi = (double)hi;
    h->inv = hi > lo ? (float)(1.0 / ((double)hi - (double)lo)) : 0.0f;
    h->a = h->b = h->mur = 0.0f;
    h->L = SEG_LEAVES;
    h->p = (int32_t)seg[SEGW * sg + 2];
    h->s = (int32_t)seg[SEGW * sg + 3];
    h->pad = 0;
}

// x of every sample of the large segments (compact index q) and its model.
template <typename K>
__global__ void k_sl_x(const K* ssk, const u32* soff, const u32* lseg, const u32* lcs, int NL, void* models,
                       int stage, float* x, int32_t* mid) {
    const u32 q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= lcs[NL]) return;
    const int j = seg_of(lcs, NL, q);
    const ModelHdr h = *seg_model(models, (u32)j);
    const float xv = model_x<K>(ssk[soff[lseg[j]] + (q - lcs[j])], h);
    x[q] = xv;
    mid[q] = stage == 0 ? j : j * SEG_LEAVES + model_leaf(xv, h);
}

// Centre of every model's samples [lo[m], lo[m+1]); parameters start at zero.
__global__ __launch_bounds__(64) void k_sl_centres(const float* x, const int32_t* lo, int nmod, void* models,
                                                     int stage) {
    __shared__ float red[1];
    const int m = blockIdx.x;
    if (m >= nmod) return;
    const int32_t a = lo[m], b = lo[m + 1];
    float sx = 0.0f;
    for (int32_t t = a + (int32_t)threadIdx.x; t < b; t += 64) sx += x[t];
    sx = wg_sum<64>(sx, red);
    if (threadIdx.x != 0) return;
    float* q = sl_params(models, stage, (u32)m);
    q[0] = 0.0f;
    q[1] = 0.0f;
    q[2] = b > a ? sx / (float)(b - a) : 0.0f;
}

// Forward: residual of every sample; target (t + 0.5) / (samples of its segment).
__global__ void k_sl_forward(const float* x, const int32_t* mid, const u32* lcs, int NL, void* models, int stage,
                             float* r) {
    const u32 q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= lcs[NL]) return;
    const u32 m = (u32)mid[q];
    const u32 j = stage == 0 ? m : m / SEG_LEAVES;
    const float* c = sl_params(models, stage, m);
    const float y = ((float)(q - lcs[j]) + 0.5f) / (float)(lcs[j + 1] - lcs[j]);
    r[q] = c[0] * (x[q] - c[2]) + c[1] - y;
}

// Backward: per model, gradient and Gram sums of its segment's loss (times
// 2 / samples of the segment), one 64-thread workgroup per model.
__global__ __launch_bounds__(64) void k_sl_backward(const float* x, const float* r, const int32_t* lo, int nmod,
                                                      const u32* lcs, void* models, int stage, float* g, float* hs) {
    __shared__ float red[1];
    const int m = blockIdx.x;
    if (m >= nmod) return;
    const float* c = sl_params(models, stage, (u32)m);
    const float mu = c[2];
    float s_rx = 0, s_r = 0, s_xx = 0, s_x = 0;
    const int32_t a = lo[m], b = lo[m + 1];
    for (int32_t t = a + (int32_t)threadIdx.x; t < b; t += 64) {
        const float dx = x[t] - mu, rv = r[t];
        s_rx += rv * dx;
        s_r += rv;
        s_xx += dx * dx;
        s_x += dx;
    }
    s_rx = wg_sum<64>(s_rx, red);
    s_r = wg_sum<64>(s_r, red);
    s_xx = wg_sum<64>(s_xx, red);
    s_x = wg_sum<64>(s_x, red);
    if (threadIdx.x != 0) return;
    const u32 j = stage == 0 ? (u32)m : (u32)m / SEG_LEAVES;
    const float sc = 2.0f / (float)(lcs[j + 1] - lcs[j]);
    g[2 * m] = s_rx * sc;
    g[2 * m + 1] = s_r * sc;
    hs[3 * m] = s_xx * sc;
    hs[3 * m + 1] = s_x * sc;
    hs[3 * m + 2] = (float)(b - a) * sc;
}

// Update: one Newton step per model; an empty leaf predicts the fraction of
// its segment's samples below it.
__global__ void k_sl_update(const float* g, const float* hs, const int32_t* lo, int nmod, const u32* lcs,
                            void* models, int stage) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmod) return;
    float* q = sl_params(models, stage, (u32)m);
    const float sxx = hs[3 * m], sx = hs[3 * m + 1], sn = hs[3 * m + 2];
    if (sn <= 0.0f) {
        const u32 j = stage == 0 ? (u32)m : (u32)m / SEG_LEAVES;
        q[0] = 0.0f;
        q[1] = (float)((u32)lo[m] - lcs[j]) / (float)(lcs[j + 1] - lcs[j]);
        return;
    }
    const float det = sxx * sn - sx * sx;
    if (sxx > 0.0f && det > 1e-6f * sxx * sn) {
        q[0] -= (sn * g[2 * m] - sx * g[2 * m + 1]) / det;
        q[1] -= (-sx * g[2 * m] + sxx * g[2 * m + 1]) / det;
    } else {
        q[1] -= g[2 * m + 1] / sn;
    }
}

// One workgroup per block of a large segment: every key ranked by the
// segment's model, corrected against its splitters (records of the tie
// rule), and the block's column of the count table from the histogram.
constexpr int SL_NT = 1024;
template <typename K>
__global__ __launch_bounds__(SL_NT) void k_sl_rank(const K* B, const u32* seg, const u32* btab, const u32* lblk,
                                                     const u32* poff, const u32* coff, const K* pk, const u32* pp,
                                                     void* models, u32* cntT, unsigned long long* lstats) {
    __shared__ SplitLds<K> S;
    __shared__ u32 hist[MAXR];
    __shared__ float2 lf2[SEG_LEAVES];
    __shared__ u32 wsum[SL_NT / 64 + 2];
    __shared__ unsigned long long wst[2];
    const int t = threadIdx.x, lane = t & 63;
    const u32 b = lblk[2 * blockIdx.x], j = lblk[2 * blockIdx.x + 1];
    const u32* bt = btab + 4 * (i64)b;
    const u32 start = bt[0], m = bt[1], sg = bt[2];
    const u32* d = seg + SEGW * sg;
    const int p = (int)d[2];
    const int k = (int)(b - d[4]);
    int P2 = 1;
    while (P2 < p) P2 <<= 1;
    const u32 po = poff[sg];
    for (int i = t; i < P2; i += SL_NT) {
        if (i < p - 1) S.set(i, pk[po + i], pp[po + i]);
        else S.set_inf(i);
        if (i < p) hist[i] = 0;
    }
    const ModelHdr mh = *seg_model(models, j);
    if (t < SEG_LEAVES) {
        const float* lf = (const float*)(seg_model(models, j) + 1);
        const float c = lf[3 * t], dd = lf[3 * t + 1], mu = lf[3 * t + 2];
        lf2[t] = make_float2(c, dd - c * mu);
    }
    if (t == 0) wst[0] = wst[1] = 0;
    __syncthreads();
    unsigned long long miss = 0, dist = 0;
    constexpr int RG = sizeof(K) == 8 ? 4 : 8;  // keys whose loads are issued together
    for (u32 i0 = 0; i0 < m; i0 += SL_NT * RG) {
        K kg[RG];
#pragma unroll
        for (int u = 0; u < RG; u++) {
            const u32 i = i0 + (u32)u * SL_NT + t;
            kg[u] = i < m ? B[start + i] : (K)0;
        }
#pragma unroll
        for (int u = 0; u < RG; u++) {
            const u32 i = i0 + (u32)u * SL_NT + t;
            const bool valid = i < m;
            int bk = p;
            if (valid) {
                const K key = kg[u];
                const typename SplitLds<K>::Q q = SplitLds<K>::query(key, start + i);
                const float x = model_x<K>(key, mh);
                const float2 ce = lf2[model_leaf(x, mh)];
                const float f = fminf(fmaxf((ce.x * x + ce.y) * (float)p, 0.0f), (float)(p - 1));
                const int pred = (int)f;
                bk = pred;
                while (bk > 0 && !S.lt(bk - 1, q)) bk--;
                while (bk < p - 1 && S.lt(bk, q)) bk++;
                miss += bk != pred;
                dist += (unsigned long long)(bk > pred ? bk - pred : pred - bk);
            }
            const int bprev = __shfl_up(bk, 1, 64);
            const bool head = valid && (lane == 0 || bprev != bk);
            const unsigned long long bound = __ballot(head || !valid);
            if (head) {
                const unsigned long long above = lane == 63 ? 0ull : (bound >> (lane + 1));
                const int len = above ? __ffsll((long long)above) : 64 - lane;
                atomicAdd(&hist[bk], (u32)len);
            }
        }
    }
    atomicAdd(&wst[0], miss);
    atomicAdd(&wst[1], dist);
    __syncthreads();
    // column k of the count table: row r = keys of the block in buckets < r
    u32 total;
    const u32 h = t < p ? hist[t] : 0u;
    const u32 ex = block_excl_scan<SL_NT>(h, total, wsum);
    u32* col = cntT + coff[sg] + k;
    if (t < p) col[(i64)t * p] = ex;
    if (t == 0) {
        col[(i64)p * p] = m;
        atomicAdd(&lstats[0], wst[0]);
        atomicAdd(&lstats[1], wst[1]);
    }
}
