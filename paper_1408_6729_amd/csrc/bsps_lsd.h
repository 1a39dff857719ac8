// bsps_lsd.h -- the local block sort (Figure SortD / Figure SortRI, steps 2-3)
// as a least-significant-digit radix sort of every block through HBM.
//
// Each virtual processor's block is sorted by 8-bit digits of its order keys,
// lowest digit first. One pass moves every record once (read + write):
//   * k_lsd_hist reads every block once and counts, for every digit position,
//     how many of its keys have each digit value. The exclusive prefix of
//     those counts is where each digit's records start inside the block after
//     any pass over that position (the counts of a block do not depend on the
//     order of its records). A position at which all keys of the block share
//     one digit needs no pass and is skipped.
//   * k_lsd_pass (one launch per pass) hands each block to one workgroup,
//     which walks the block's tiles in order: a tile is sorted stably by the
//     pass's digit in LDS (two LDS ranking passes, 6 + 2 bits), and every
//     record goes to its digit's running offset. Walking the tiles in order
//     keeps every pass stable across tiles without any inter-workgroup
//     communication, so the final pass yields the stable sort of the block.
// The last pass writes the block-sorted array B (order keys) and the block
// samples (every ys-th key of a block) that the bucket boundaries and the
// bucket merge use.
#pragma once
#include "bsps_kernels.h"

constexpr int LSD_RADIX = 256;
constexpr int LSD_HIST_NT = 1024;

template <typename K>
struct LsdArgs {
    const K* in;       // source of the first pass (keys of dtype in_dt)
    const u32* inv;
    int in_dt;
    K* a;              // scratch buffers of the passes in between (order keys)
    u32* av;
    K* b;
    u32* bv;
    K* out;            // the block-sorted array (order keys)
    u32* outv;
    i64 n;
    int p, tpb;
    u32* dbase;        // [p][sizeof(K)][256] start of each digit inside the block, per position
    u32* plist;        // [p][sizeof(K) + 1]: passes c >= 1, then the c digit positions
    K* smp;            // block samples: key at block position (j+1)*ys - 1 -> smp[k*spb + j]
    u32 ys, spb;
};

// Digit counts of every block at every position, their exclusive prefixes and
// the list of positions the block needs a pass for. One workgroup per block.
template <typename K>
__global__ __launch_bounds__(LSD_HIST_NT) void k_lsd_hist(LsdArgs<K> a) {
    constexpr int NT = LSD_HIST_NT, DP = (int)sizeof(K), PER = 16 / (int)sizeof(K);
    constexpr int NV = DP * LSD_RADIX;  // counters
    __shared__ u32 h[NV];
    __shared__ u32 wt[NT / 64];
    __shared__ u32 trivial[DP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int k = blockIdx.x; k < a.p; k += gridDim.x) {
        __syncthreads();  // the previous block's reads of h are done
        for (int i = t; i < NV; i += NT) h[i] = 0u;
        if (t < DP) trivial[t] = 0u;
        __syncthreads();
        const i64 st = blk_start(a.n, a.p, k), en = blk_start(a.n, a.p, k + 1);
        auto count = [&](K raw) {
            const K u = okey<K>(raw, a.in_dt);
#pragma unroll
            for (int b = 0; b < DP; b++) atomicAdd(&h[b * LSD_RADIX + (u32)((u >> (8 * b)) & 255)], 1u);
        };
        // 16-byte loads over the aligned middle of the block, single keys at its ends
        const uintptr_t base = (uintptr_t)a.in;
        i64 vlo = st, vhi = st;
        if ((base & 15) == 0) {
            vlo = (st + PER - 1) / PER * PER;
            vhi = en / PER * PER;
            if (vhi < vlo) vhi = vlo;
        }
        // [st, vlo) and [vhi, en) single keys, [vlo, vhi) in 16-byte vectors
        for (i64 g = st + t; g < (vlo < en ? vlo : en); g += NT) count(a.in[g]);
        const uint4* vp = reinterpret_cast<const uint4*>(a.in);
        for (i64 q = vlo / PER + t; q < vhi / PER; q += NT) {
            const uint4 x = vp[q];
            const K* e = reinterpret_cast<const K*>(&x);
#pragma unroll
            for (int m = 0; m < PER; m++) count(e[m]);
        }
        for (i64 g = vhi + t; g < en; g += NT) count(a.in[g]);
        __syncthreads();
        const u32 mk = (u32)(en - st);
        // exclusive prefix of the 256 counts of each position: NT/256 positions
        // per round, 4 waves per position
        for (int r = 0; r < NV / NT; r++) {
            const int b = r * (NT / LSD_RADIX) + t / LSD_RADIX, d = t % LSD_RADIX;
            const u32 v = h[b * LSD_RADIX + d];
            if (v == mk) trivial[b] = 1u;  // every key of the block has digit d here
            const u32 inc = wave_incl_scan(v);
            if (lane == 63) wt[w] = inc;
            __syncthreads();
            u32 before = 0;
            for (int q = (w & ~3); q < w; q++) before += wt[q];
            a.dbase[((i64)k * DP + b) * LSD_RADIX + d] = before + inc - v;
            __syncthreads();
        }
        if (t == 0) {
            u32* pl = a.plist + (i64)k * (DP + 1);
            u32 c = 0;
            for (int b = 0; b < DP; b++)
                if (!trivial[b]) pl[1 + c++] = (u32)b;
            if (c == 0) pl[1 + c++] = 0u;  // all keys equal: one pass, which copies the block
            pl[0] = c;
        }
    }
}

// One pass of every block that needs it (pass < its pass count). Each
// workgroup takes whole blocks and walks their tiles in order, prefetching the
// next tile's keys while it sorts the current one. The exchange buffer has its
// own LDS region (SEP), so after the tile sort the counter region is free for
// the payloads' final exchange.
template <typename K, bool HASV>
__global__ __launch_bounds__(Shape<K>::NT, BSPS_WG_PER_CU) void k_lsd_pass(LsdArgs<K> a, int pass) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT, DP = (int)sizeof(K);
    __shared__ SortSmem<NT, (int)sizeof(K), IT, true> sm;
    __shared__ u32 off[LSD_RADIX], ts[LSD_RADIX], te[LSD_RADIX];
    static_assert(SortSmem<NT, (int)sizeof(K), IT, true>::CNTW >= NT * IT + NT * IT / 32, "payload exchange fits");
    K* exch = sm.template ex<K>();
    u32* vbuf = sm.cnt();
    const int t = threadIdx.x, i0 = t * IT;
    for (int k = blockIdx.x; k < a.p; k += gridDim.x) {
        const u32* pl = a.plist + (i64)k * (DP + 1);
        const int c = (int)uniform(pl[0]);
        if (pass >= c) continue;
        const int pos = (int)uniform(pl[1 + pass]);
        const int sh = 8 * pos;
        const bool first = pass == 0, last = pass == c - 1;
        const K* src = first ? a.in : ((pass & 1) ? a.a : a.b);
        const u32* srcv = first ? a.inv : ((pass & 1) ? a.av : a.bv);
        K* dst = last ? a.out : ((pass & 1) ? a.b : a.a);
        u32* dstv = last ? a.outv : ((pass & 1) ? a.bv : a.av);
        const int sdt = first ? a.in_dt : BSPS_DT_NONE;
        const i64 st = blk_start(a.n, a.p, k), en = blk_start(a.n, a.p, k + 1);
        if (t < LSD_RADIX) {
            off[t] = (u32)st + a.dbase[((i64)k * DP + pos) * LSD_RADIX + t];
            ts[t] = 0u;
            te[t] = 0u;
        }
        auto digit = [&](K u) { return (u32)(u >> sh) & 255u; };
        i64 base = st;
        int cnt = (int)min((i64)T, en - st);
        K nk[IT];
        load_blocked<K, IT>(src + base + i0, cnt - i0, nk);
        for (;;) {
            K kr[IT];
            u32 v[IT], rank[IT];
            const int valid = cnt - i0;
#pragma unroll
            for (int j = 0; j < IT; j++) kr[j] = j < valid ? okey<K>(nk[j], sdt) : KeyMax<K>::v;  // padding sorts last
            if (HASV) load_blocked<u32, IT>(srcv + base + i0, valid, v);
            const int ccnt = cnt;
            base += T;
            cnt = (int)min((i64)T, en - base);
            // the next tile's keys are in flight while this one is sorted
            if (cnt > 0) load_blocked<K, IT>(src + base + i0, cnt - i0, nk);
            wg_sort_regs<NT, IT, K, HASV, true, true>(kr, v, rank, 8, exch, sm.cnt(), sm.wsum, sh);
            // runs of equal digits in the sorted tile: where each starts and ends
#pragma unroll 4
            for (int j = 0; j < IT; j++) {
                const int i = j * NT + t;
                if (i < ccnt) {
                    const u32 d = digit(exch[padj<NT>(j, t)]);
                    const u32 dp = i > 0 ? digit(exch[padi(i - 1)]) : 256u;
                    if (d != dp) {
                        ts[d] = (u32)i;
                        if (i > 0) te[dp] = (u32)i;
                    }
                    if (i == ccnt - 1) te[d] = (u32)ccnt;
                }
            }
            if (HASV) {
                // the counters are free: the payloads go to their final slots there
#pragma unroll
                for (int j = 0; j < IT; j++) vbuf[padi((int)rank[j])] = v[j];
            }
            __syncthreads();
#pragma unroll 8
            for (int j = 0; j < IT; j++) {
                const int i = j * NT + t;
                if (i < ccnt) {
                    const K u = exch[padj<NT>(j, t)];
                    const u32 d = digit(u);
                    const u32 g = off[d] + ((u32)i - ts[d]);
                    dst[g] = u;
                    if (HASV) dstv[g] = vbuf[padj<NT>(j, t)];
                    if (last && a.smp) {
                        const u32 rel = g - (u32)st + 1u;
                        if ((rel & (a.ys - 1)) == 0 && rel / a.ys <= a.spb) a.smp[(i64)k * a.spb + rel / a.ys - 1] = u;
                    }
                }
            }
            __syncthreads();
            if (t < LSD_RADIX) {
                off[t] += te[t] - ts[t];
                ts[t] = 0u;
                te[t] = 0u;
            }
            if (cnt <= 0) break;
        }
        __syncthreads();  // off of this block is no longer read
    }
}
