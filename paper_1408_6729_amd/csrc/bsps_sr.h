// bsps_sr.h -- kernels of the Sort_Ran_BSP ordering (Section 5.2, Figure
// SortR): the sample is drawn from the unsorted input, every input key is
// ranked against the splitters and routed to its bucket, and the buckets are
// sorted last. The tags of the duplicate handling (Section 5.1.1) are the
// input positions: with no local sort before the sample, (processor, local
// index) orders exactly like the position in the input.
#pragma once
#include "bsps_kernels.h"

// Sample records (key, input position) of the unsorted input X (keys of dtype
// dt) at the given positions; keys become order keys.
template <typename K>
__global__ void k_gather_sample_in(const K* X, int dt, const u32* pos, i64 ns, K* skey) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    skey[t] = okey<K>(X[pos[t]], dt);
}

// Routing, order preserving (Figure SortR steps 10-11): the records of input
// block k (keys X of dtype dt, payloads Xv) go to their buckets, bucket b's
// run of block k starting at off[k*p + b], in input order. One workgroup per
// block walks the block's tiles in order and keeps each bucket's running
// offset: a tile is partitioned stably by bucket id in LDS (the sort key is
// bucket << 14 | tile position, sorted on the dbits bucket bits), then every
// record is read from its tile position (just loaded, so from the caches) and
// written, as an order key, to its bucket's running offset.
constexpr int SR_NT = 512, SR_IT = 32, SR_T = SR_NT * SR_IT;  // 14 bits of tile position
static_assert(SR_T == (1 << 14), "tile positions take the low 14 bits of the sort key");

template <typename K, bool HASV>
__global__ __launch_bounds__(SR_NT, BSPS_WG_PER_CU) void k_route_sr(const K* X, const u32* Xv, int dt,
                                                                    const u32* bucket, i64 n, int p, int dbits,
                                                                    const u32* off, K* Z, u32* Zv) {
    constexpr int NT = SR_NT, IT = SR_IT, T = SR_T;
    __shared__ SortSmem<NT, 4, IT, true> sm;
    __shared__ u32 offs[MAXR], ts[MAXR], te[MAXR];
    u32* exch = sm.template ex<u32>();
    const int t = threadIdx.x, i0 = t * IT;
    for (int k = blockIdx.x; k < p; k += gridDim.x) {
        const i64 st = blk_start(n, p, k), en = blk_start(n, p, k + 1);
        for (int b = t; b < p; b += NT) {
            offs[b] = off[(i64)k * p + b];
            ts[b] = 0u;
            te[b] = 0u;
        }
        i64 base = st;
        int cnt = (int)min((i64)T, en - st);
        u32 nb[IT];
        load_blocked<u32, IT>(bucket + base + i0, cnt - i0, nb);
        for (;;) {
            u32 sk[IT], v[IT], rank[IT];
            const int valid = cnt - i0;
#pragma unroll
            for (int j = 0; j < IT; j++) {
                sk[j] = j < valid ? (nb[j] << 14) | (u32)(i0 + j) : 0xFFFFFFFFu;  // padding sorts last
                v[j] = 0u;
            }
            const int ccnt = cnt;
            const i64 cbase = base;
            base += ccnt;
            cnt = (int)min((i64)T, en - base);
            if (cnt > 0) load_blocked<u32, IT>(bucket + base + i0, cnt - i0, nb);
            wg_sort_regs<NT, IT, u32, false, true, true>(sk, v, rank, dbits, exch, sm.cnt(), sm.wsum, 14);
            // runs of equal buckets in the partitioned tile
#pragma unroll 4
            for (int j = 0; j < IT; j++) {
                const int i = j * NT + t;
                if (i < ccnt) {
                    const u32 d = exch[padj<NT>(j, t)] >> 14;
                    const u32 dp = i > 0 ? exch[padi(i - 1)] >> 14 : 0xFFFFFFFFu;
                    if (d != dp) {
                        ts[d] = (u32)i;
                        if (i > 0) te[dp] = (u32)i;
                    }
                    if (i == ccnt - 1) te[d] = (u32)ccnt;
                }
            }
            __syncthreads();
#pragma unroll 8
            for (int j = 0; j < IT; j++) {
                const int i = j * NT + t;
                if (i < ccnt) {
                    const u32 e = exch[padj<NT>(j, t)];
                    const u32 d = e >> 14, o = e & (u32)(T - 1);
                    const u32 g = offs[d] + ((u32)i - ts[d]);
                    Z[g] = okey<K>(X[cbase + o], dt);
                    if (HASV) Zv[g] = Xv[cbase + o];
                }
            }
            __syncthreads();
            for (int b = t; b < p; b += NT) {
                offs[b] += te[b] - ts[b];
                ts[b] = 0u;
                te[b] = 0u;
            }
            if (cnt <= 0) break;
        }
        __syncthreads();  // offs of this block is no longer read
    }
}
