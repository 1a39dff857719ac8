// bsps_learned.h -- per-key bucket ranking (splitter search or learned model)
// and the learned CDF model's training kernels.
//
// Bucket of a record (key, g) of the block-sorted array: the number of
// splitter records (key_i, g_i) strictly below it (tie rule of Section 5.1.1:
// key first, then the position tag), i.e. a lower-bound search.
//
// Learned bucketing (not in the paper): a two-stage model of the key
// distribution. With x = (u - lo) / (hi - lo) for an order key u and lo/hi the
// smallest and largest sample keys, a linear root r(x) = a (x - mu_r) + b picks
// leaf l = clamp(floor(L r), 0, L-1), whose linear model
// f(x) = c_l (x - mu_l) + d_l predicts the fraction of keys below x. The
// predicted bucket clamp(floor(p f), 0, p-1) is then checked exactly against
// the splitters and moved to the true bucket, so the result always equals the
// splitter search. Training data: the sorted sample, record t with target
// y_t = (t + 0.5) / (p s) (its bucket under the splitter rule is floor(t/s)).
// Loss (1/N) sum (f(x_t) - y_t)^2; forward = residuals, backward = gradient and
// Gram (Hessian) sums per leaf, update = one Newton step per leaf.
#pragma once
#include "bsps_device.h"

// Device model buffer: header then L leaf triples.
struct ModelHdr {
    double lo, hi;          // order-key range of the sorted sample
    float a, b, mur, inv;   // root model and 1 / (hi - lo) (0 when hi == lo)
    int32_t L, p, s, pad;   // leaves, processors, oversampling
};
static_assert(sizeof(ModelHdr) == 48, "model header layout");

extern "C" size_t bsps_model_bytes(int32_t leaves) {
    return sizeof(ModelHdr) + (size_t)(leaves > 0 ? leaves : 4096) * 3 * sizeof(float);
}
extern "C" size_t bsps_fit_workspace_bytes(int64_t N, int32_t leaves);

template <typename K>
__device__ __forceinline__ float model_x(K u, const ModelHdr& h) {
    const u64 lo = (u64)h.lo;
    const float d = (u64)u >= lo ? (float)((u64)u - lo) : -(float)(lo - (u64)u);
    return d * h.inv;
}

// 4-byte keys: the offset from lo in 32-bit integer arithmetic (exact), then
// one conversion; training and inference use the same function.
template <>
__device__ __forceinline__ float model_x<u32>(u32 u, const ModelHdr& h) {
    const u32 lo = (u32)h.lo;
    const float d = u >= lo ? (float)(u - lo) : -(float)(lo - u);
    return d * h.inv;
}

__device__ __forceinline__ int model_leaf(float x, const ModelHdr& h) {
    float r = (h.a * (x - h.mur) + h.b) * (float)h.L;
    r = fminf(fmaxf(r, 0.0f), (float)(h.L - 1));
    return (int)r;
}


// ---------------------------------------------------------------- per-key rank

// One workgroup per RANK_TILE keys of one block: bucket of every key, the
// block's row of the count matrix (atomics), and for the learned model the
// number of corrected predictions and their total distance.
// Splitter search: 256-thread workgroups (12 KB of LDS, 8 per CU). Learned:
// 1024-thread workgroups that also hold the leaf table (32 KB), 2 per CU.
// A tile is 32 keys per thread of one block.
constexpr int RANK_IT = 32;
constexpr int MAX_LEAVES = 4096;
template <bool LEARNED> struct RankShape;
template <> struct RankShape<false> { static constexpr int NT = 256, WG_PER_CU = 8; };
template <> struct RankShape<true> { static constexpr int NT = 1024, WG_PER_CU = 2; };
template <bool LEARNED> constexpr int rank_tile() { return RankShape<LEARNED>::NT * RANK_IT; }

// ---------------------------------------------------------------- training

// x_t of every sample and the leaf each sample uses at this stage (stage 0:
// the root, one model; stage 1: leaf chosen by the root).
template <typename K>
__global__ void k_model_x(const K* smp, i64 N, int dt, const void* model, int stage, float* x, int32_t* leafid) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const ModelHdr h = *(const ModelHdr*)model;
    const float xv = model_x<K>(okey<K>(smp[t], dt), h);
    x[t] = xv;
    leafid[t] = stage == 0 ? 0 : model_leaf(xv, h);
}

// Leaf ranges: the leaf id is non-decreasing along the sorted sample, so
// leaf l owns the samples [lo_l, lo_{l+1}).
__global__ void k_model_ranges(const int32_t* leafid, i64 N, int L, int32_t* lo) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > L) return;
    i64 a = 0, b = N;  // first t with leafid[t] >= l
    while (a < b) {
        const i64 m = (a + b) >> 1;
        if (leafid[m] < l) a = m + 1; else b = m;
    }
    lo[l] = (int32_t)a;
}

// Sum over the workgroup (NTR threads, a multiple of 64); every thread gets
// the total. red: NTR/64 floats of LDS.
template <int NTR>
__device__ __forceinline__ float wg_sum(float v, float* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (NTR == 64) return v;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < NTR / 64; i++) acc += red[i];
    return acc;
}

// Loss = (sum of the models' r^2 shares) / N; one workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_sum_loss(const float* lossp, int nmod, i64 N, float* out) {
    __shared__ float red[4];
    float acc = 0.0f;
    for (int l = threadIdx.x; l < nmod; l += 256) acc += lossp[l];
    acc = wg_sum<256>(acc, red);
    if (threadIdx.x == 0) *out = N > 0 ? acc / (float)N : 0.0f;
}

// Splitter records in LDS, compared with a record (key, pos) by the tie rule.
// 4-byte keys pack (key, pos) into one u64, so a comparison is one 64-bit
// compare and one LDS read; 8-byte keys keep key and tag apart.
template <typename K> struct SplitLds;
template <>
struct SplitLds<u32> {
    u64 kp[MAXR];
    typedef u64 Q;
    __device__ __forceinline__ void set(int i, u32 k, u32 pos) { kp[i] = ((u64)k << 32) | pos; }
    __device__ __forceinline__ void set_inf(int i) { kp[i] = ~0ull; }
    __device__ __forceinline__ static Q query(u32 key, u32 pos) { return ((u64)key << 32) | pos; }
    __device__ __forceinline__ bool lt(int i, Q q) const { return kp[i] < q; }  // S_i <_rec (key, pos)
};
template <>
struct SplitLds<u64> {
    u64 k[MAXR];
    u32 ps[MAXR];
    struct Q { u64 key; u32 pos; };
    __device__ __forceinline__ void set(int i, u64 kk, u32 pos) { k[i] = kk; ps[i] = pos; }
    __device__ __forceinline__ void set_inf(int i) { k[i] = ~0ull; ps[i] = 0xffffffffu; }
    __device__ __forceinline__ static Q query(u64 key, u32 pos) { return Q{key, pos}; }
    __device__ __forceinline__ bool lt(int i, Q q) const { return rec_lt<u64>(k[i], ps[i], q.key, q.pos); }
};

// Bucket of every key of the block-sorted array B and the count matrix.
// Keys and splitters of dtype dt (BSPS_DT_NONE: already order keys). Tiles of
// rank_tile() keys of one block; each workgroup loads the splitters (and the
// learned model) once and walks tiles with a grid stride. Splitter
// bucketing: branch-free binary search over the p - 1 records padded to a
// power of two. Learned bucketing: root, then the leaf line held in LDS as
// (c, d - c mu) so that f(x) = c x + (d - c mu), then the exact check against
// the two neighbouring splitters, walking to the true bucket when the
// prediction is off. Counts: lanes holding a run of equal buckets add its
// length once.
// dt: dtype of the keys, sdt: of the splitter keys (BSPS_DT_NONE: order keys).
template <typename K, bool LEARNED>
__global__ __launch_bounds__(RankShape<LEARNED>::NT) void k_rank(const K* B, i64 n, int p, int tpb, const K* spk,
                                                                     const u32* spp, int dt, int sdt,
                                                                     const void* model, u32* bucket, u32* counts,
                                                                     unsigned long long* lstats) {
    constexpr int NT = RankShape<LEARNED>::NT, TILE = NT * RANK_IT;
    __shared__ SplitLds<K> S;
    __shared__ u32 hist[MAXR];
    __shared__ float2 lf2[LEARNED ? MAX_LEAVES : 1];
    __shared__ unsigned long long wst[2];
    const int t = threadIdx.x, lane = t & 63;
    int P2 = 1;
    while (P2 < p) P2 <<= 1;
    for (int i = t; i < P2; i += NT) {
        if (i < p - 1) S.set(i, okey<K>(spk[i], sdt), spp[i]);
        else S.set_inf(i);
        if (i < p) hist[i] = 0;
    }
    if (t == 0) wst[0] = wst[1] = 0;
    ModelHdr mh;
    if (LEARNED) {
        mh = *(const ModelHdr*)model;
        mh.L = mh.L < 1 ? 1 : (mh.L > MAX_LEAVES ? MAX_LEAVES : mh.L);  // leaf ids stay inside the table
        const float* lf = (const float*)((const ModelHdr*)model + 1);
        for (int l = t; l < mh.L; l += NT) {
            const float c = lf[3 * l], d = lf[3 * l + 1], mu = lf[3 * l + 2];
            lf2[l] = make_float2(c, d - c * mu);
        }
    }
    __syncthreads();
    unsigned long long miss = 0, dist = 0;
    const int ntile = p * tpb;
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int k = tile / tpb, tt = tile % tpb;
        const i64 st = (i64)(((u64)k * (u64)n) / (u64)p), en = (i64)(((u64)(k + 1) * (u64)n) / (u64)p);
        const i64 base = st + (i64)tt * TILE;
        const i64 cnt64 = en - base;
        const int cnt = cnt64 <= 0 ? 0 : (cnt64 > TILE ? TILE : (int)cnt64);
        constexpr int RG = sizeof(K) == 8 ? 4 : 8;  // keys whose loads are issued together
        for (int j0 = 0; j0 < RANK_IT; j0 += RG) {
            if (j0 * NT + (t & ~63) >= cnt) break;  // the whole wave is past the tile's end
            K kg[RG];
#pragma unroll
            for (int u = 0; u < RG; u++) {
                const int i = (j0 + u) * NT + t;
                kg[u] = i < cnt ? B[base + i] : (K)0;
            }
#pragma unroll
            for (int u = 0; u < RG; u++) {
                const int i = (j0 + u) * NT + t;
                const bool valid = i < cnt;
                const i64 g = base + i;
                int b = p;
                if (valid) {
                    const K key = okey<K>(kg[u], dt);
                    const typename SplitLds<K>::Q q = SplitLds<K>::query(key, (u32)g);
                    if (!LEARNED) {
                        b = 0;
                        for (int h = P2 >> 1; h >= 1; h >>= 1) b += S.lt(b + h - 1, q) ? h : 0;
                    } else {
                        const float x = model_x<K>(key, mh);
                        const float2 ce = lf2[model_leaf(x, mh)];
                        const float f = fminf(fmaxf((ce.x * x + ce.y) * (float)p, 0.0f), (float)(p - 1));
                        const int pred = (int)f;
                        b = pred;
                        while (b > 0 && !S.lt(b - 1, q)) b--;
                        while (b < p - 1 && S.lt(b, q)) b++;
                        miss += b != pred;
                        dist += (unsigned long long)(b > pred ? b - pred : pred - b);
                    }
                    if (bucket) bucket[g] = (u32)b;
                }
                const int bprev = __shfl_up(b, 1, 64);
                const bool head = valid && (lane == 0 || bprev != b);
                const unsigned long long bound = __ballot(head || !valid);
                if (head) {
                    const unsigned long long above = lane == 63 ? 0ull : (bound >> (lane + 1));
                    const int len = above ? __ffsll((long long)above) : 64 - lane;
                    atomicAdd(&hist[b], (u32)len);
                }
            }
        }
        __syncthreads();
        for (int i = t; i < p; i += NT) {
            const u32 h = hist[i];
            if (h) {
                if (counts) atomicAdd(&counts[(i64)k * p + i], h);
                hist[i] = 0;
            }
        }
        __syncthreads();
    }
    if (LEARNED) {
        atomicAdd(&wst[0], miss);
        atomicAdd(&wst[1], dist);
        __syncthreads();
        if (t == 0 && lstats) {
            atomicAdd(&lstats[0], wst[0]);
            atomicAdd(&lstats[1], wst[1]);
        }
    }
}

// Routing with per-key ranking (the scatter route, Figure SortD steps 9-11):
// every key of the block-sorted array B is given its bucket, by the branch-free
// splitter search or by the learned model with the exact check, and is copied
// to its run's destination, order kept. The run boundaries inside each sorted
// block come from the splitter searches into the blocks (cntT), so the keys
// are read once, by this kernel. Each workgroup takes a share of one block and
// holds the block's run starts (rs) and destinations (od) in LDS with the
// splitters (and the leaf table): key at block position c of bucket b goes to
// od[b] + (c - rs[b]). The loads of RG keys are issued before they are ranked.
template <typename K, bool LEARNED, bool HASV>
__global__ __launch_bounds__(RankShape<LEARNED>::NT) void k_scatter_rank(
    const K* B, const u32* Bv, i64 n, int p, int wpb, const K* spk, const u32* spp, const void* model,
    const u32* cntT, const u32* off, K* Z, u32* Zv, u32* bucket, unsigned long long* lstats) {
    constexpr int NT = RankShape<LEARNED>::NT;
    constexpr int RG = sizeof(K) == 8 ? 4 : 8;
    __shared__ SplitLds<K> S;
    __shared__ u32 rs[MAXR], od[MAXR];
    __shared__ float2 lf2[LEARNED ? MAX_LEAVES : 1];
    __shared__ unsigned long long wst[2];
    const int t = threadIdx.x;
    const int k = blockIdx.x / wpb, w = blockIdx.x % wpb;
    int P2 = 1;
    while (P2 < p) P2 <<= 1;
    for (int i = t; i < P2; i += NT) {
        if (i < p - 1) S.set(i, spk[i], spp[i]);
        else S.set_inf(i);
        if (i < p) {
            rs[i] = cntT[(i64)i * p + k];
            od[i] = off[(i64)k * p + i];
        }
    }
    if (t == 0) wst[0] = wst[1] = 0;
    ModelHdr mh;
    if (LEARNED) {
        mh = *(const ModelHdr*)model;
        mh.L = mh.L < 1 ? 1 : (mh.L > MAX_LEAVES ? MAX_LEAVES : mh.L);  // leaf ids stay inside the table
        const float* lf = (const float*)((const ModelHdr*)model + 1);
        for (int l = t; l < mh.L; l += NT) {
            const float c = lf[3 * l], d = lf[3 * l + 1], mu = lf[3 * l + 2];
            lf2[l] = make_float2(c, d - c * mu);
        }
    }
    __syncthreads();
    const i64 st = (i64)(((u64)k * (u64)n) / (u64)p), m = (i64)(((u64)(k + 1) * (u64)n) / (u64)p) - st;
    const i64 lo = m * w / wpb, hi = m * (w + 1) / wpb;
    unsigned long long miss = 0, dist = 0;
    for (i64 c0 = lo; c0 < hi; c0 += (i64)NT * RG) {
        K kg[RG];
        u32 vg[RG];
#pragma unroll
        for (int u = 0; u < RG; u++) {
            const i64 c = c0 + (i64)u * NT + t;
            kg[u] = c < hi ? B[st + c] : (K)0;
            vg[u] = (HASV && c < hi) ? Bv[st + c] : 0u;
        }
#pragma unroll
        for (int u = 0; u < RG; u++) {
            const i64 c = c0 + (i64)u * NT + t;
            if (c >= hi) continue;
            const K key = kg[u];
            const typename SplitLds<K>::Q q = SplitLds<K>::query(key, (u32)(st + c));
            int b;
            if (!LEARNED) {
                b = 0;
                for (int h = P2 >> 1; h >= 1; h >>= 1) b += S.lt(b + h - 1, q) ? h : 0;
            } else {
                const float x = model_x<K>(key, mh);
                const float2 ce = lf2[model_leaf(x, mh)];
                const float f = fminf(fmaxf((ce.x * x + ce.y) * (float)p, 0.0f), (float)(p - 1));
                const int pred = (int)f;
                b = pred;
                while (b > 0 && !S.lt(b - 1, q)) b--;
                while (b < p - 1 && S.lt(b, q)) b++;
                miss += b != pred;
                dist += (unsigned long long)(b > pred ? b - pred : pred - b);
            }
            const u32 dst = od[b] + ((u32)c - rs[b]);
            Z[dst] = key;
            if (HASV) Zv[dst] = vg[u];
            if (bucket) bucket[st + c] = (u32)b;
        }
    }
    if (LEARNED) {
        atomicAdd(&wst[0], miss);
        atomicAdd(&wst[1], dist);
        __syncthreads();
        if (t == 0 && lstats) {
            atomicAdd(&lstats[0], wst[0]);
            atomicAdd(&lstats[1], wst[1]);
        }
    }
}

// Routing offsets from the bucket boundaries of every sorted block (cntT, row
// i = keys of each block below bucket i): bucket i starts after all smaller
// buckets, and within it the keys of block k follow those of blocks 0..k-1:
// off[k*p + i]. One workgroup per bucket.
__global__ __launch_bounds__(256) void k_route_offsets_T(const u32* cntT, int p, u32* off) {
    __shared__ u32 wsum[8];
    const int i = blockIdx.x, t = threadIdx.x;
    const int per = (p + 255) / 256;
    u32 loc = 0, lb = 0;
    for (int k = t * per; k < (t + 1) * per && k < p; k++) {
        loc += cntT[(i64)(i + 1) * p + k] - cntT[(i64)i * p + k];
        lb += cntT[(i64)i * p + k];
    }
    u32 tot, base;
    u32 ex = block_excl_scan<256>(loc, tot, wsum);
    __syncthreads();
    (void)block_excl_scan<256>(lb, base, wsum);
    for (int k = t * per; k < (t + 1) * per && k < p; k++) {
        off[(i64)k * p + i] = base + ex;
        ex += cntT[(i64)(i + 1) * p + k] - cntT[(i64)i * p + k];
    }
}

// The fit in three launches (the same forward residuals, backward gradient
// and Gram sums times 2/N, and Newton update as the kernels above, `iters`
// steps per stage): the root on one workgroup of FIT_NT threads, which also
// writes x of every record; the first record of every leaf; then every leaf
// on one wave (its lanes split the leaf's records and reduce by shuffles).
// An empty leaf takes c = 0 and d = (records below it) / (p s).
constexpr int FIT_NT = 1024;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One Newton step of a linear model from its gradient (gc, gd) and Gram sums
// (sxx, sx, sn), all times 2/N (exact for the quadratic loss): a singular Gram
// matrix moves only the intercept d.
__device__ __forceinline__ void newton_step(float& c, float& d, float gc, float gd, float sxx, float sx, float sn) {
    const float det = sxx * sn - sx * sx;
    if (sxx > 0.0f && det > 1e-6f * sxx * sn) {
        c -= (sn * gc - sx * gd) / det;
        d -= (-sx * gc + sxx * gd) / det;
    } else {
        d -= gd / sn;
    }
}

// Forward and backward of one linear model f(x) = c (x - mu) + d over the
// records [a, b) of the sorted sample this thread takes (first, first +
// stride, ...): the residual r = f(x_t) - y_t with y_t = (t + 0.5) / (p s),
// then the partial sums of the gradient (r dx, r), of the Gram matrix (dx^2,
// dx) and of the loss (r^2), dx = x - mu. The fit and the gradient check
// (bsps_model_grad) both use it.
struct FitSums {
    float rx, r, xx, x, rr;
};

__device__ __forceinline__ FitSums fit_partials(const float* x, i64 first, i64 b, int stride, float c, float d,
                                                float mu, float ps) {
    FitSums f{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (i64 i = first; i < b; i += stride) {
        const float dx = x[i] - mu;
        const float r = c * dx + d - ((float)i + 0.5f) / ps;  // forward
        f.rx += r * dx;                                        // backward
        f.r += r;
        f.xx += dx * dx;
        f.x += dx;
        f.rr += r * r;
    }
    return f;
}

template <typename K>
__global__ __launch_bounds__(FIT_NT) void k_fit_root(const K* smp, i64 N, int dt, int p, int s, int L, int iters,
                                                     void* model, float* x) {
    __shared__ float red[FIT_NT / 64];
    __shared__ ModelHdr sh;
    const int t = threadIdx.x;
    ModelHdr* h = (ModelHdr*)model;
    if (t == 0) {
        const K klo = N > 0 ? okey<K>(smp[0], dt) : (K)0;
        const K khi = N > 0 ? okey<K>(smp[N - 1], dt) : (K)0;
        sh.lo = (double)klo;
        sh.hi = (double)khi;
        sh.inv = khi > klo ? (float)(1.0 / ((double)khi - (double)klo)) : 0.0f;
        sh.a = sh.b = sh.mur = 0.0f;
        sh.L = L;
        sh.p = p;
        sh.s = s;
        sh.pad = 0;
    }
    __syncthreads();
    const float ps = (float)p * (float)s;
    const float sc = N > 0 ? 2.0f / (float)N : 0.0f;
    float sx = 0.0f;
    for (i64 i = t; i < N; i += FIT_NT) {
        const float xv = model_x<K>(okey<K>(smp[i], dt), sh);
        x[i] = xv;
        sx += xv;
    }
    sx = wg_sum<FIT_NT>(sx, red);
    const float mur = N > 0 ? sx / (float)N : 0.0f;
    float ra = 0.0f, rb = 0.0f;
    for (int it = 0; it < iters; it++) {
        const FitSums f = fit_partials(x, t, N, FIT_NT, ra, rb, mur, ps);
        const float s_rx = wg_sum<FIT_NT>(f.rx, red), s_r = wg_sum<FIT_NT>(f.r, red);
        const float s_xx = wg_sum<FIT_NT>(f.xx, red), s_x = wg_sum<FIT_NT>(f.x, red);
        if (N > 0) newton_step(ra, rb, s_rx * sc, s_r * sc, s_xx * sc, s_x * sc, (float)N * sc);
    }
    if (t == 0) {
        h->lo = sh.lo;
        h->hi = sh.hi;
        h->inv = sh.inv;
        h->a = ra;
        h->b = rb;
        h->mur = mur;
        h->L = L;
        h->p = p;
        h->s = s;
        h->pad = 0;
    }
}

// lo[l] = first record of leaf l (l = 0..L; lo[L] = N). The root's leaf never
// decreases along the sorted sample, so record i starts every leaf in
// (leaf(i-1), leaf(i)]; one thread per record boundary i = 0..N. Leaf ids are
// capped at L, so only lo[0..L] is written whatever the model holds.
__global__ void k_fit_ranges(const float* x, i64 N, const void* model, int L, int32_t* lo) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const ModelHdr h = *(const ModelHdr*)model;
    const int a = i > 0 ? min(model_leaf(x[i - 1], h), L) : -1;
    const int b = i < N ? min(model_leaf(x[i], h), L) : L;
    for (int l = a + 1; l <= b; l++) lo[l] = (int32_t)i;
}

constexpr int FIT_LEAF_NT = 256;

__global__ __launch_bounds__(FIT_LEAF_NT) void k_fit_leaves(const float* x, const int32_t* lo, i64 N, int L, int p,
                                                           int s, int iters, void* model) {
    const ModelHdr* h = (const ModelHdr*)model;
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.x * (FIT_LEAF_NT / 64) + (threadIdx.x >> 6);
    if (l >= L) return;
    const float ps = (float)p * (float)s;
    const float sc = N > 0 ? 2.0f / (float)N : 0.0f;
    float* q = (float*)(h + 1);
    // (clamped: with a model whose leaves do not follow the sample order, lo is
    // not a partition, and the reads must still stay inside the sample)
    const int32_t a = (int32_t)max((i64)0, min((i64)lo[l], N)), b = (int32_t)max((i64)a, min((i64)lo[l + 1], N));
    if (b <= a) {
        if (lane == 0) {
            q[3 * l] = 0.0f;
            q[3 * l + 1] = (float)a / ps;
            q[3 * l + 2] = 0.0f;
        }
        return;
    }
    float cx = 0.0f;
    for (int32_t i = a + lane; i < b; i += 64) cx += x[i];
    const float mu = wave_sum(cx) / (float)(b - a);
    float c = 0.0f, d = 0.0f;
    for (int it = 0; it < iters; it++) {
        const FitSums f = fit_partials(x, a + lane, b, 64, c, d, mu, ps);
        newton_step(c, d, wave_sum(f.rx) * sc, wave_sum(f.r) * sc, wave_sum(f.xx) * sc, wave_sum(f.x) * sc,
                    (float)(b - a) * sc);
    }
    if (lane == 0) {
        q[3 * l] = c;
        q[3 * l + 1] = d;
        q[3 * l + 2] = mu;
    }
}

// Gradient check of the leaf stage (bsps_model_grad): for every leaf, at the
// model's current parameters, the same forward and backward as the fit, the
// gradient and Gram sums times 2/N (g[2l], g[2l+1]; hs[3l], hs[3l+1],
// hs[3l+2] = count times 2/N) and the leaf's share of the loss sum r^2. One
// wave per leaf.
__global__ __launch_bounds__(FIT_LEAF_NT) void k_grad_leaves(const float* x, const int32_t* lo, i64 N, int L,
                                                            int p, int s, const void* model, float* g, float* hs,
                                                            float* lossp) {
    const ModelHdr* h = (const ModelHdr*)model;
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.x * (FIT_LEAF_NT / 64) + (threadIdx.x >> 6);
    if (l >= L) return;
    const float ps = (float)p * (float)s;
    const float sc = N > 0 ? 2.0f / (float)N : 0.0f;
    const float* q = (const float*)(h + 1);
    const int32_t a = (int32_t)max((i64)0, min((i64)lo[l], N)), b = (int32_t)max((i64)a, min((i64)lo[l + 1], N));
    const FitSums f = fit_partials(x, a + lane, b, 64, q[3 * l], q[3 * l + 1], q[3 * l + 2], ps);
    const float rx = wave_sum(f.rx), r = wave_sum(f.r), xx = wave_sum(f.xx), xs = wave_sum(f.x), rr = wave_sum(f.rr);
    if (lane == 0) {
        g[2 * l] = rx * sc;
        g[2 * l + 1] = r * sc;
        hs[3 * l] = xx * sc;
        hs[3 * l + 1] = xs * sc;
        hs[3 * l + 2] = (float)(b - a) * sc;
        lossp[l] = rr;
    }
}
