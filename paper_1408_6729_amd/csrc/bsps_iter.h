// bsps_iter.h -- kernels of the iterative Sort_Det_BSP (Section 5.1: m
// rounds of partitioning and merging, each round splitting every current
// bucket into k further buckets, p = k^m virtual processors).
//
// State between rounds: the array (order keys), its group table grp (G + 1
// starts; group g is the segment [grp[g], grp[g+1]) held by q = p / G
// processors) and the samples of every processor's share (every yb-th key,
// slot stride spb), written by the previous round's merge. Processor j of
// group g (global number g*q + j) owns the share [blk_start(z, q, j),
// blk_start(z, q, j + 1)) of the segment, z = its size; every share is sorted.
// Round r: regular sample of every share (k_it_sample), the sample of every
// group sorted (the block sort with one block per group), k - 1 splitters per
// group (k_it_splitters), each share cut by the splitters (k_it_count), the
// merge tables of the next round's shares (k_it_tables), and the multiway
// merge of those tables. A record's tag is its position in the round's input
// array; every round keeps equal keys in input order, so this orders exactly
// like the original (processor, index) tag.
#pragma once
#include "bsps_kernels.h"

// One group holding the whole array.
__global__ void k_it_groups_init(u32* grp, i64 n) {
    if (threadIdx.x == 0) {
        grp[0] = 0u;
        grp[1] = (u32)n;
    }
}

// Regular sample of every share (as Figure SortD step 4 inside each group):
// share j of a group of z records cut into s segments of x = ceil(ceil(z/q)/s)
// keys, the key closing each segment taken, positions past a short share
// clamped to its last key. No share is empty (a record fills at most s sample
// slots, so every sub-bucket keeps at least q/k records); the clamp into the
// array only keeps the read in bounds.
template <typename K>
__global__ void k_it_sample(const K* A, i64 n, const u32* grp, int q, int s, i64 ns, K* skey, u32* spos) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const int P = (int)(t / s), i = (int)(t % s) + 1;
    const int g = P / q, j = P % q;
    const i64 gs = grp[g], z = (i64)grp[g + 1] - gs;
    const i64 a = gs + blk_start(z, q, j), mj = blk_start(z, q, j + 1) - blk_start(z, q, j);
    const i64 xm = (z + q - 1) / q, x = (xm + s - 1) / s;
    i64 pos = a + max((i64)1, min((i64)i * x, mj)) - 1;
    pos = min(max(pos, (i64)0), n - 1);
    skey[t] = A[pos];
    spos[t] = (u32)pos;
}

// Splitters of every group: the records at 1-based ranks t, 2t, ..., (k-1)t of
// its sorted sample (q*s records), t = q*s/k.
template <typename K>
__global__ void k_it_splitters(const K* ssk, const u32* ssp, int G, int q, int s, int k, K* pk, u32* pp) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)G * (k - 1)) return;
    const int g = (int)(idx / (k - 1)), i = (int)(idx % (k - 1)) + 1;
    const i64 t = (i64)q * s / k;
    const i64 src = (i64)g * q * s + (i64)i * t - 1;
    pk[idx] = ssk[src];
    pp[idx] = ssp[src];
}

// cnt[b*p + P] = records of share P at or below splitter b of its group
// (b = 1..k-1; row 0 is 0 and row k the share size): share P's bucket b is
// [cnt[b][P], cnt[b+1][P]) within the sorted share.
template <typename K>
__global__ void k_it_count(const K* A, const u32* grp, int p, int q, int k, const K* pk, const u32* pp, u32* cnt) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)(k + 1) * p) return;
    const int b = (int)(idx / p), P = (int)(idx % p);
    const int g = P / q, j = P % q;
    const i64 gs = grp[g], z = (i64)grp[g + 1] - gs;
    const i64 st = gs + blk_start(z, q, j), mj = blk_start(z, q, j + 1) - blk_start(z, q, j);
    u32 res;
    if (b == 0) res = 0;
    else if (b == k) res = (u32)mj;
    else {
        const K sk = pk[(i64)g * (k - 1) + b - 1];
        const u32 sp = pp[(i64)g * (k - 1) + b - 1];
        u32 lo = 0, hi = (u32)mj;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (rec_le<K>(A[st + mid], (u32)(st + mid), sk, sp)) lo = mid + 1; else hi = mid;
        }
        res = lo;
    }
    cnt[idx] = res;
}

// Merge tables of the next round (routing fused into the merge): one
// workgroup per sub-bucket b of group g, which becomes group g*k + b. The
// sub-bucket is the concatenation, in processor order, of the q shares'
// runs of bucket b (run j: [c_j, c_j + len_j) of the concatenation); it
// starts after the group's records below splitter b. Its q/k new processors
// take even shares of it; new processor j' (merge group g2 = (g*k + b)*q/k +
// j') gets, as run slot j, the piece of run j inside its share, with the
// source samples (every yb-th key of the source share, slot stride spb,
// at most spb of them) that fall inside the piece.
constexpr int IT_NT = 256;

__global__ __launch_bounds__(IT_NT) void k_it_tables(const u32* grp, int G, int p, int q, int k, const u32* cnt,
                                                     u32 yb, u32 spb, u32* ngrp, u32* run_start, u32* run_len,
                                                     u32* out_base, u32* sdesc) {
    __shared__ u32 c[MAXR + 1];
    __shared__ u32 part[IT_NT];
    __shared__ u32 below_sum;
    const int t = threadIdx.x;
    const int g = blockIdx.x / k, b = blockIdx.x % k;
    const i64 gs = grp[g], z = (i64)grp[g + 1] - gs;
    const int q2 = q / k;
    // run lengths and the records below splitter b, per source share
    const int per = (q + IT_NT - 1) / IT_NT;
    u32 sl = 0, sb = 0;
    for (int e = 0; e < per; e++) {
        const int j = t * per + e;
        if (j < q) {
            const int P = g * q + j;
            const u32 lo = cnt[(i64)b * p + P], hi = cnt[(i64)(b + 1) * p + P];
            c[j] = hi - lo;
            sl += hi - lo;
            sb += lo;
        }
    }
    part[t] = sl;
    __syncthreads();
    if (t == 0) {
        u32 acc = 0;
        for (int i = 0; i < IT_NT; i++) {
            const u32 v = part[i];
            part[i] = acc;
            acc += v;
        }
        c[q] = acc;  // sub-bucket size (placed after the exclusive prefix below)
    }
    __syncthreads();
    {
        u32 acc = part[t];
        for (int e = 0; e < per; e++) {
            const int j = t * per + e;
            if (j < q) {
                const u32 v = c[j];
                c[j] = acc;
                acc += v;
            }
        }
    }
    // records of the group below splitter b: the sub-bucket's start
    for (int o = 32; o >= 1; o >>= 1) sb += __shfl_xor(sb, o, 64);
    if (t == 0) below_sum = 0;
    __syncthreads();
    if ((t & 63) == 0) atomicAdd(&below_sum, sb);
    __syncthreads();
    const u32 start = (u32)gs + below_sum, z2 = c[q];
    const int g2 = g * k + b;
    if (t == 0) {
        ngrp[g2] = start;
        if (g2 == G * k - 1) ngrp[G * k] = grp[G];
    }
    for (i64 e = t; e < (i64)q2 * q; e += IT_NT) {
        const int jn = (int)(e / q), j = (int)(e % q);
        const i64 P2 = (i64)g2 * q2 + jn, slot = P2 * q + j;
        const u32 u = (u32)blk_start(z2, q2, jn), v = (u32)blk_start(z2, q2, jn + 1);
        if (j == 0) out_base[P2] = start + u;
        const u32 cj = c[j], ej = j + 1 < q ? c[j + 1] : z2;
        const u32 lo = max(cj, u), hi = min(ej, v);
        u32* sd = sdesc + slot * 4;
        if (hi > lo) {
            const int P = g * q + j;
            const u32 a = (u32)(gs + blk_start(z, q, j));
            const u32 o0 = cnt[(i64)b * p + P] + (lo - cj), o1 = o0 + (hi - lo);
            run_start[slot] = a + o0;
            run_len[slot] = hi - lo;
            const u32 jlo = min(o0 / yb, spb), jhi = min(o1 / yb, spb);
            sd[0] = (u32)P * spb + jlo;
            sd[1] = jhi - jlo;
            sd[2] = a + (jlo + 1) * yb - 1;
            sd[3] = yb;
        } else {
            run_start[slot] = 0;
            run_len[slot] = 0;
            sd[0] = 0; sd[1] = 0; sd[2] = 0; sd[3] = yb;
        }
    }
}
