// bsps_lsd.h -- the local block sort (Figure SortD / Figure SortRI, steps 2-3)
// as a least-significant-digit radix sort of every block through HBM, and the
// sort of Sort_Ran_BSP's buckets (Figure SortR step 12), blocks of any sizes.
//
// Each block is sorted by 8-bit digits of its order keys, lowest digit first.
// One pass moves every record once (read + write). Everything is parallel over
// 16 Ki-key tiles, whatever the block sizes:
//   * k_lsd_tiles numbers every block's tiles; k_lsd_count counts, per tile,
//     how many keys have each digit value at every byte position and adds
//     that into its block's counts; k_lsd_scan takes their exclusive prefixes
//     per position (where each digit's records start inside the block after
//     any pass over that position: the counts of a block do not depend on the
//     order of its records) and lists the positions at which the block's keys
//     differ (the others need no pass).
//   * k_lsd_sweep (one launch per pass) sorts every tile stably by the pass's
//     digit in LDS (the tile sort's 6-bit and 2-bit ranking passes) and writes
//     every record to its digit's start in the block plus the count of that
//     digit in the block's earlier tiles, learnt by a decoupled look-back.
//     The passes are stable, so the last one yields the stable sort of the block.
// The last pass writes the block-sorted array (order keys, or raw keys for the
// buckets of Sort_Ran_BSP) and the block samples (every ys-th key of a block)
// that the bucket boundaries and the bucket merge use.
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
    const u32* blk;    // NULL: block k = [floor(k n/p), floor((k+1) n/p)); else [blk[k], blk[k+1]) (blk[p] = n
                       // implied), blocks of any sizes, empty ones included
    int out_dt;        // the last pass writes raw keys of this dtype (BSPS_DT_NONE: order keys)
};

template <typename K>
__device__ __forceinline__ void lsd_block(const LsdArgs<K>& a, int k, i64& st, i64& en) {
    if (a.blk) {
        st = a.blk[k];
        en = k + 1 < a.p ? (i64)a.blk[k + 1] : a.n;
    } else {
        st = blk_start(a.n, a.p, k);
        en = blk_start(a.n, a.p, k + 1);
    }
}

// ---------------------------------------------------------------- one sweep per pass, every tile in parallel
//
// The same pass with one workgroup per tile instead of one per block: a tile
// learns where each of its digits goes from the tiles before it in its block
// by a decoupled look-back. Every tile publishes, per digit, its count (flag
// A) and, once it knows the sum over all earlier tiles of the block, that
// inclusive prefix (flag P); a tile sums its predecessors' entries backwards
// until it meets a P. Tiles take tickets from a counter in the order they
// start, and a tile only ever waits on tiles with smaller tickets, which have
// all started before it: the smallest unfinished ticket never waits, so every
// wait ends. A spin limit bounds each wait all the same (an overrun is
// counted, and the host reports it as an error).
constexpr u32 LSD_FA = 1u << 30, LSD_FP = 2u << 30, LSD_CM = (1u << 30) - 1u;
constexpr int LSD_LB = 8;  // predecessors read per look-back step

struct LsdSweep {
    u32* status;     // [ntile][256]: 0 (not yet), LSD_FA | count, or LSD_FP | inclusive prefix
    u32* ctr;        // [0] ticket, [1] waits that hit the spin limit
    u32* tstart;     // [p + 1] first tile of every block (global tile numbers)
    u32* hist;       // [p][sizeof(K)][256] digit counts of every block
    u32 ntile;       // grid: at least the number of tiles
    u32 spin_limit;  // loads per wait before giving up
};

// tstart[k] = tiles of the blocks before k (a block of m keys has ceil(m/T)
// tiles, an empty one none). One workgroup; p <= 1024.
template <typename K>
__global__ __launch_bounds__(1024) void k_lsd_tiles(LsdArgs<K> a, LsdSweep w) {
    constexpr int T = Shape<K>::NT * Shape<K>::IT;
    __shared__ u32 wsum[1024 / 64 + 2];
    const int k = threadIdx.x;
    u32 nt = 0;
    if (k < a.p) {
        i64 st, en;
        lsd_block(a, k, st, en);
        nt = (u32)((en - st + T - 1) / T);
    }
    u32 total;
    const u32 ex = block_excl_scan<1024>(nt, total, wsum);
    if (k < a.p) w.tstart[k] = ex;
    if (k == 0) w.tstart[a.p] = total;
}

template <typename K, bool HASV>
__global__ __launch_bounds__(Shape<K>::NT, BSPS_WG_PER_CU) void k_lsd_sweep(LsdArgs<K> a, LsdSweep w, int pass) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT, DP = (int)sizeof(K);
    __shared__ SortSmem<NT, (int)sizeof(K), IT, true> sm;
    __shared__ u32 off[LSD_RADIX], ts[LSD_RADIX], te[LSD_RADIX];
    __shared__ u32 sh_tile;
    static_assert(SortSmem<NT, (int)sizeof(K), IT, true>::CNTW >= NT * IT + NT * IT / 32, "payload exchange fits");
    K* exch = sm.template ex<K>();
    u32* vbuf = sm.cnt();
    const int t = threadIdx.x, i0 = t * IT;
    if (t == 0) sh_tile = atomicAdd(&w.ctr[0], 1u);
    if (t < LSD_RADIX) {
        ts[t] = 0u;
        te[t] = 0u;
    }
    __syncthreads();
    const u32 tile = uniform(sh_tile);
    if (tile >= w.tstart[a.p]) return;  // past the last tile
    // the block of this tile: the last k with tstart[k] <= tile
    int lo = 0, hi = a.p - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (w.tstart[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const int k = uniform(lo);
    const u32 tt = tile - w.tstart[k];
    const u32* pl = a.plist + (i64)k * (DP + 1);
    const int c = (int)uniform(pl[0]);
    if (pass >= c) return;  // the block needs no pass here (none of its tiles waits)
    const int pos = (int)uniform(pl[1 + pass]);
    const int sh = 8 * pos;
    const bool first = pass == 0, last = pass == c - 1;
    const K* src = first ? a.in : ((pass & 1) ? a.a : a.b);
    const u32* srcv = first ? a.inv : ((pass & 1) ? a.av : a.bv);
    K* dst = last ? a.out : ((pass & 1) ? a.b : a.a);
    u32* dstv = last ? a.outv : ((pass & 1) ? a.bv : a.av);
    const int sdt = first ? a.in_dt : BSPS_DT_NONE;
    const int odt = last ? a.out_dt : BSPS_DT_NONE;
    i64 st, en;
    lsd_block(a, k, st, en);
    const i64 base = st + (i64)tt * T;
    const int cnt = (int)min((i64)T, en - base);
    auto digit = [&](K u) { return (u32)(u >> sh) & 255u; };
    K nk[IT], kr[IT];
    u32 v[IT], rank[IT];
    load_blocked<K, IT>(src + base + i0, cnt - i0, nk);
    const int valid = cnt - i0;
#pragma unroll
    for (int j = 0; j < IT; j++) kr[j] = j < valid ? okey<K>(nk[j], sdt) : KeyMax<K>::v;  // padding sorts last
    if (HASV) load_blocked<u32, IT>(srcv + base + i0, valid, v);
    wg_sort_regs<NT, IT, K, HASV, true, true>(kr, v, rank, 8, exch, sm.cnt(), sm.wsum, sh);
    // runs of equal digits in the sorted tile: where each starts and ends
#pragma unroll 4
    for (int j = 0; j < IT; j++) {
        const int i = j * NT + t;
        if (i < cnt) {
            const u32 d = digit(exch[padj<NT>(j, t)]);
            const u32 dp = i > 0 ? digit(exch[padi(i - 1)]) : 256u;
            if (d != dp) {
                ts[d] = (u32)i;
                if (i > 0) te[dp] = (u32)i;
            }
            if (i == cnt - 1) te[d] = (u32)cnt;
        }
    }
    if (HASV) {
        // the counters are free: the payloads go to their final slots there
#pragma unroll
        for (int j = 0; j < IT; j++) vbuf[padi((int)rank[j])] = v[j];
    }
    __syncthreads();
    if (t < LSD_RADIX) {
        // publish this tile's count of digit t, then look back for the sum
        // over the earlier tiles of the block
        const u32 mine = te[t] - ts[t];
        u32* sp = w.status + (u64)tile * LSD_RADIX + t;
        u32 before = 0;
        if (tt == 0) {
            __hip_atomic_store(sp, LSD_FP | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(sp, LSD_FA | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // look back LSD_LB tiles at a time (their loads in flight together):
            // add ready counts from the nearest tile on, up to a prefix; a tile
            // that is not ready yet is read again
            const u32 first_tile = w.tstart[k];
            u32 j = tile;  // tiles j, j+1, ..., tile-1 are summed into `before`
            u32 spins = 0;
            bool done = false;
            while (!done) {
                const u32 nw = min((u32)LSD_LB, j - first_tile);
                u32 sv[LSD_LB];
#pragma unroll
                for (int q = 0; q < LSD_LB; q++)
                    sv[q] = (u32)q < nw ? __hip_atomic_load(w.status + (u64)(j - 1 - q) * LSD_RADIX + t,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                        : 0u;
                u32 q = 0;
                for (; q < nw; q++) {
                    const u32 f = sv[q] & ~LSD_CM;
                    if (f == 0u) break;  // not ready yet
                    before += sv[q] & LSD_CM;
                    if (f == LSD_FP) {
                        done = true;
                        break;
                    }
                }
                if (done) break;
                j -= q;
                if (q == 0 && ++spins > w.spin_limit) {
                    atomicAdd(&w.ctr[1], 1u);
                    break;
                }
            }
            __hip_atomic_store(sp, LSD_FP | (before + mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        off[t] = (u32)st + a.dbase[((i64)k * DP + pos) * LSD_RADIX + t] + before;
    }
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < IT; j++) {
        const int i = j * NT + t;
        if (i < cnt) {
            const K u = exch[padj<NT>(j, t)];
            const u32 d = digit(u);
            const u32 g = off[d] + ((u32)i - ts[d]);
            dst[g] = rawkey<K>(u, odt);
            if (HASV) dstv[g] = vbuf[padj<NT>(j, t)];
            if (last && a.smp) {
                const u32 rel = g - (u32)st + 1u;
                if ((rel & (a.ys - 1)) == 0 && rel / a.ys <= a.spb) a.smp[(i64)k * a.spb + rel / a.ys - 1] = u;
            }
        }
    }
}

// ---------------------------------------------------------------- digit counts, every tile in parallel
//
// Every tile counts its digits in LDS and adds them to its block's counts in
// global memory (hist, zeroed before), so a large block (a large bucket of
// Sort_Ran_BSP) is spread over as many workgroups as it has tiles;
// k_lsd_scan then turns every block's counts into its digit starts and its
// pass list.
constexpr int LSD_COUNT_NT = 512;

template <typename K>
__global__ __launch_bounds__(LSD_COUNT_NT) void k_lsd_count(LsdArgs<K> a, LsdSweep w, u32* hist) {
    constexpr int NT = LSD_COUNT_NT, T = Shape<K>::NT * Shape<K>::IT, DP = (int)sizeof(K);
    constexpr int NV = DP * LSD_RADIX;
    __shared__ u32 h[NV];
    const int t = threadIdx.x;
    const u32 tile = blockIdx.x;
    if (tile >= w.tstart[a.p]) return;
    int lo = 0, hi = a.p - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (w.tstart[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const int k = lo;
    for (int i = t; i < NV; i += NT) h[i] = 0u;
    __syncthreads();
    i64 st, en;
    lsd_block(a, k, st, en);
    const i64 b0 = st + (i64)(tile - w.tstart[k]) * T, b1 = min(b0 + (i64)T, en);
    for (i64 g = b0 + t; g < b1; g += NT) {
        const K u = okey<K>(a.in[g], a.in_dt);
#pragma unroll
        for (int b = 0; b < DP; b++) atomicAdd(&h[b * LSD_RADIX + (u32)((u >> (8 * b)) & 255)], 1u);
    }
    __syncthreads();
    for (int i = t; i < NV; i += NT) {
        const u32 v = h[i];
        if (v) atomicAdd(&hist[(i64)k * NV + i], v);
    }
}

// Digit starts and pass list of every block from its counts. One workgroup
// per block.
template <typename K>
__global__ __launch_bounds__(LSD_HIST_NT) void k_lsd_scan(LsdArgs<K> a, const u32* hist) {
    constexpr int NT = LSD_HIST_NT, DP = (int)sizeof(K);
    constexpr int NV = DP * LSD_RADIX;
    __shared__ u32 wt[NT / 64];
    __shared__ u32 trivial[DP];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int k = blockIdx.x;
    if (t < DP) trivial[t] = 0u;
    __syncthreads();
    i64 st, en;
    lsd_block(a, k, st, en);
    const u32 mk = (u32)(en - st);
    for (int r = 0; r < NV / NT; r++) {
        const int b = r * (NT / LSD_RADIX) + t / LSD_RADIX, d = t % LSD_RADIX;
        const u32 v = hist[(i64)k * NV + b * LSD_RADIX + d];
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
