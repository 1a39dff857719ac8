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

__device__ __forceinline__ int model_leaf(float x, const ModelHdr& h) {
    float r = (h.a * (x - h.mur) + h.b) * (float)h.L;
    r = fminf(fmaxf(r, 0.0f), (float)(h.L - 1));
    return (int)r;
}

__device__ __forceinline__ int model_bucket(float x, int l, const float* leaf, int p) {
    float f = leaf[3 * l] * (x - leaf[3 * l + 2]) + leaf[3 * l + 1];
    f = fminf(fmaxf(f * (float)p, 0.0f), (float)(p - 1));
    return (int)f;
}

// ---------------------------------------------------------------- per-key rank

// One workgroup per RANK_TILE keys of one block: bucket of every key, the
// block's row of the count matrix (atomics), and for the learned model the
// number of corrected predictions and their total distance.
constexpr int RANK_NT = 256, RANK_IT = 16, RANK_TILE = RANK_NT * RANK_IT;

// ---------------------------------------------------------------- training

// Header: range of the sorted sample (order keys) and the model's shape.
template <typename K>
__global__ void k_model_init(const K* smp, i64 N, int dt, int p, int s, int L, void* model) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ModelHdr* h = (ModelHdr*)model;
    const K lo = N > 0 ? okey<K>(smp[0], dt) : (K)0;
    const K hi = N > 0 ? okey<K>(smp[N - 1], dt) : (K)0;
    h->lo = (double)lo;
    h->hi = (double)hi;
    h->inv = hi > lo ? (float)(1.0 / ((double)hi - (double)lo)) : 0.0f;
    h->a = h->b = h->mur = 0.0f;
    h->L = L;
    h->p = p;
    h->s = s;
    h->pad = 0;
}

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

// Parameter views: stage 0 uses the root (a, b, mu_r) as one "leaf"; stage 1
// the L leaf triples (c, d, mu).
__device__ __forceinline__ float* stage_params(void* model, int stage) {
    ModelHdr* h = (ModelHdr*)model;
    return stage == 0 ? &h->a : (float*)(h + 1);
}

// Leaf centres mu = mean x over each leaf's samples (0 for an empty leaf);
// parameters start at zero.
__global__ void k_model_centres(const float* x, const int32_t* lo, int nmod, void* model, int stage) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nmod) return;
    float* q = stage_params(model, stage);
    const int32_t a = lo[l], b = lo[l + 1];
    float sx = 0.0f;
    for (int32_t t = a; t < b; t++) sx += x[t];
    const float mu = b > a ? sx / (float)(b - a) : 0.0f;
    if (stage == 0) {
        q[0] = 0.0f; q[1] = 0.0f; q[2] = mu;   // a, b, mu_r
    } else {
        q[3 * l] = 0.0f; q[3 * l + 1] = 0.0f; q[3 * l + 2] = mu;
    }
}

__device__ __forceinline__ void stage_get(const float* q, int stage, int l, float& c, float& d, float& mu) {
    if (stage == 0) { c = q[0]; d = q[1]; mu = q[2]; }
    else { c = q[3 * l]; d = q[3 * l + 1]; mu = q[3 * l + 2]; }
}

// Forward: residual r_t = f(x_t) - y_t of every sample under its model.
__global__ void k_model_forward(const float* x, const int32_t* leafid, i64 N, int p, int s, const void* model,
                                int stage, float* r) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const float* q = stage_params(const_cast<void*>(model), stage);
    float c, d, mu;
    stage_get(q, stage, leafid[t], c, d, mu);
    const float y = ((float)t + 0.5f) / ((float)p * (float)s);
    r[t] = c * (x[t] - mu) + d - y;
}

// Backward: per model, gradient of the loss and the Gram sums (all times 2/N),
// summed in sample order: g = (sum r dx, sum r), h = (sum dx^2, sum dx, count),
// dx = x - mu; also the model's share of the loss sum r^2.
__global__ void k_model_backward(const float* x, const float* r, const int32_t* lo, int nmod, i64 N,
                                 const void* model, int stage, float* g, float* hs, float* lossp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nmod) return;
    const float* q = stage_params(const_cast<void*>(model), stage);
    float c, d, mu;
    stage_get(q, stage, l, c, d, mu);
    float s_rx = 0, s_r = 0, s_xx = 0, s_x = 0, s_rr = 0;
    const int32_t a = lo[l], b = lo[l + 1];
    for (int32_t t = a; t < b; t++) {
        const float dx = x[t] - mu, rv = r[t];
        s_rx += rv * dx;
        s_r += rv;
        s_xx += dx * dx;
        s_x += dx;
        s_rr += rv * rv;
    }
    const float sc = N > 0 ? 2.0f / (float)N : 0.0f;
    g[2 * l] = s_rx * sc;
    g[2 * l + 1] = s_r * sc;
    hs[3 * l] = s_xx * sc;
    hs[3 * l + 1] = s_x * sc;
    hs[3 * l + 2] = (float)(b - a) * sc;
    lossp[l] = s_rr;
}

// Update: one Newton step per model (exact for a quadratic loss); a singular
// Gram matrix moves only the intercept; a model without samples keeps c = 0
// and predicts the fraction of samples below it.
__global__ void k_model_update(const float* g, const float* hs, const int32_t* lo, int nmod, int p, int s,
                               void* model, int stage) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nmod) return;
    float* q = stage_params(model, stage);
    float* c = stage == 0 ? &q[0] : &q[3 * l];
    float* d = stage == 0 ? &q[1] : &q[3 * l + 1];
    const float sxx = hs[3 * l], sx = hs[3 * l + 1], sn = hs[3 * l + 2];
    if (sn <= 0.0f) {
        *c = 0.0f;
        *d = (float)lo[l] / ((float)p * (float)s);
        return;
    }
    const float det = sxx * sn - sx * sx;
    if (sxx > 0.0f && det > 1e-6f * sxx * sn) {
        *c -= (sn * g[2 * l] - sx * g[2 * l + 1]) / det;
        *d -= (-sx * g[2 * l] + sxx * g[2 * l + 1]) / det;
    } else {
        *d -= g[2 * l + 1] / sn;
    }
}

// Root fitted: copy (a, b, mu_r) stays in the header; nothing else to do.
__global__ void k_sum_loss(const float* lossp, int nmod, i64 N, float* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float acc = 0;
    for (int l = 0; l < nmod; l++) acc += lossp[l];
    *out = N > 0 ? acc / (float)N : 0.0f;
}

// Keys and splitters of dtype dt (BSPS_DT_NONE: already order keys).
template <typename K, bool LEARNED>
__global__ __launch_bounds__(RANK_NT) void k_rank(const K* B, i64 n, int p, int tpb, const K* spk,
                                                      const u32* spp, int dt, const void* model, u32* bucket,
                                                      u32* counts, unsigned long long* lstats) {
    __shared__ K sk[MAXR];
    __shared__ u32 sp[MAXR];
    __shared__ u32 hist[MAXR];
    __shared__ float leaf[LEARNED ? 3 * 4096 : 1];
    __shared__ ModelHdr mh;
    __shared__ unsigned long long wst[2];
    const int t = threadIdx.x;
    const int k = blockIdx.x / tpb, tt = blockIdx.x % tpb;
    const i64 st = (i64)(((u64)k * (u64)n) / (u64)p), en = (i64)(((u64)(k + 1) * (u64)n) / (u64)p);
    const i64 base = st + (i64)tt * RANK_TILE;
    const i64 cnt64 = en - base;
    if (cnt64 <= 0) return;
    const int cnt = cnt64 > RANK_TILE ? RANK_TILE : (int)cnt64;
    int P2 = 1;
    while (P2 < p) P2 <<= 1;
    for (int i = t; i < P2; i += RANK_NT) {
        if (i < p - 1) {
            sk[i] = okey<K>(spk[i], dt);
            sp[i] = spp[i];
        } else {
            sk[i] = KeyMax<K>::v;
            sp[i] = 0xffffffffu;
        }
        if (i < p) hist[i] = 0;
    }
    if (LEARNED) {
        const ModelHdr* h = (const ModelHdr*)model;
        if (t == 0) {
            mh = *h;
            wst[0] = wst[1] = 0;
        }
        const float* lf = (const float*)(h + 1);
        for (int i = t; i < 3 * h->L; i += RANK_NT) leaf[i] = lf[i];
    }
    __syncthreads();
    unsigned long long miss = 0, dist = 0;
#pragma unroll 4
    for (int j = 0; j < RANK_IT; j++) {
        const int i = j * RANK_NT + t;
        if (i >= cnt) break;
        const i64 g = base + i;
        const K key = okey<K>(B[g], dt);
        const u32 pos = (u32)g;
        int b;
        if (!LEARNED) {
            b = 0;
            for (int hstep = P2 >> 1; hstep >= 1; hstep >>= 1) {
                const int q = b + hstep - 1;
                b += rec_lt<K>(sk[q], sp[q], key, pos) ? hstep : 0;
            }
        } else {
            const float x = model_x<K>(key, mh);
            const int pred = model_bucket(x, model_leaf(x, mh), leaf, p);
            b = pred;
            while (b > 0 && !rec_lt<K>(sk[b - 1], sp[b - 1], key, pos)) b--;
            while (b < p - 1 && rec_lt<K>(sk[b], sp[b], key, pos)) b++;
            miss += b != pred;
            dist += (unsigned long long)(b > pred ? b - pred : pred - b);
        }
        if (bucket) bucket[g] = (u32)b;
        atomicAdd(&hist[b], 1u);
    }
    if (LEARNED) {
        atomicAdd(&wst[0], miss);
        atomicAdd(&wst[1], dist);
    }
    __syncthreads();
    if (counts)
        for (int i = t; i < p; i += RANK_NT)
            if (hist[i]) atomicAdd(&counts[(i64)k * p + i], hist[i]);
    if (LEARNED && t == 0 && lstats) {
        atomicAdd(&lstats[0], wst[0]);
        atomicAdd(&lstats[1], wst[1]);
    }
}
