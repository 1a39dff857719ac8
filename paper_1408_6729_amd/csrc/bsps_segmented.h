// bsps_segmented.h -- batched sort of many independent segments.
//
// Segment i of n_i keys is sorted with its own p_i virtual processors and
// oversampling s_i (Figure SortD per segment). p_i is chosen so that every
// block fits one tile: each block is then sorted by one workgroup, and a
// segment with p_i = 1 is finished by that sort. The other steps run for all
// segments in one launch each, driven by tables:
//   seg[8*i .. 8*i+7] = start, n, p, s, first block, -, -, -
//   soff[i] / poff[i] / coff[i]: prefix offsets of the segments' samples
//   (p*s), splitters (p-1) and count rows ((p+1)*p); zero-sized for p = 1
//   btab[4*b ..]      = block start, size, segment, block-sample offset
#pragma once
#include "bsps_kernels.h"

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
