// bsps_kernels.h -- HIP kernels of the BSP sample sort for gfx950.
//
// Pipeline (Figure SortD / Figure SortRI, p virtual processors on one GPU):
//   A1 local block sort  = k_tile_sort (LDS radix sort of tiles) followed by a
//                          multiway merge of the tiles of every block (MWM)
//   A2 sample            = k_det_sample | k_ran_positions + k_gather_sample
//   A3 splitters         = sort of the sample (same A1 machinery, one block) +
//                          k_splitters
//   A4 bucket ranking    = k_count (splitters searched into each sorted block,
//                          the paper's Sort_IRan_BSP step 11) or k_rank (every
//                          key on its own, LDS splitter search or learned model)
//   A5 prefix + routing  = k_bucket_tables (+ k_route_offsets / k_scatter)
//   A6 per-bucket merge  = MWM over the p runs of every bucket, reading each run
//                          where it lies (fused routing) or from the routed array
//
// Multiway merge (MWM) of a group of R sorted runs (a block's tiles, or a
// bucket's runs): regular samples of the runs are sorted in one workgroup;
// every q-th sample becomes a chunk boundary record (key, position); each
// run is cut at every boundary by binary search on (key, position), so the
// cut is exact and ties follow position order; each chunk (the pieces of all
// runs between two boundaries) is gathered into LDS and sorted there. A chunk
// larger than the LDS tile is sorted by the same workgroup with LSD radix
// passes through global memory.
#pragma once
#include "bsps_device.h"

constexpr int MAXR = 1024;  // runs per merge group (tiles per block, or p)

#ifndef BSPS_GATHER_LDS
#define BSPS_GATHER_LDS 1  // merge gather through LDS-staged, position-striped loads
#endif

#ifdef BSPS_TIMING
// Per-phase cycle sums of the merge kernel: [0, 8) merges that emit output
// samples (block merges), [8, 16) the others (bucket merges).
__device__ unsigned long long g_phase[16];
#define PHASE(k)                                                               \
    do {                                                                       \
        __syncthreads();                                                       \
        if (threadIdx.x == 0) {                                                \
            const unsigned long long now = __builtin_amdgcn_s_memtime();       \
            atomicAdd(&g_phase[(k) + (a.osmp ? 0 : 8)], now - t_last);         \
            t_last = now;                                                      \
        }                                                                      \
    } while (0)
#define PHASE_START unsigned long long t_last = __builtin_amdgcn_s_memtime()
#else
#define PHASE(k) do {} while (0)
#define PHASE_START do {} while (0)
#endif

// Reference copy (attainable HBM bandwidth): every workgroup copies 1024
// consecutive 16-byte vectors, four per thread, position-striped, with
// nontemporal loads and stores (the data is not reused).
constexpr int COPY_NT = 256, COPY_PER = 4;

__global__ __launch_bounds__(COPY_NT) void k_stream_copy(const v4u32* __restrict__ src, v4u32* __restrict__ dst,
                                                         u64 n16) {
    const u64 b = (u64)blockIdx.x * (COPY_NT * COPY_PER) + threadIdx.x;
    v4u32 v[COPY_PER];
#pragma unroll
    for (int k = 0; k < COPY_PER; k++)
        if (b + (u64)k * COPY_NT < n16) v[k] = __builtin_nontemporal_load(src + b + (u64)k * COPY_NT);
#pragma unroll
    for (int k = 0; k < COPY_PER; k++)
        if (b + (u64)k * COPY_NT < n16) __builtin_nontemporal_store(v[k], dst + b + (u64)k * COPY_NT);
}

// ======================================================================= tables

template <typename K>
struct MwmArgs {
    const K* src;
    const u32* srcv;
    K* dst;           // output keys (order keys, or raw keys when out_dt >= 0)
    u32* dstv;
    K* scr;           // oversize-chunk scratch, indexed like dst
    u32* scrv;
    int G, R;
    const u32* run_start;  // [G*R] position of run r of group g in src
    const u32* run_len;    // [G*R]
    const u32* out_base;   // [G] output position of the group's first key
    const u32* sdesc;      // [G*R*4] sample runs: (index, count, first position, stride)
    const K* smp;          // sample keys
    u32 cap;               // largest chunk sorted in LDS
    u32 tavg;              // target chunk size
    u32* slot_count;       // [1] slots handed out (zeroed before the pick kernel)
    u32* oversize;         // [1] oversize chunks (statistics)
    u32* work;             // [1] next slot for the persistent merge workgroups
    u32* slot_group;       // [S]
    u32* grp_base;         // [G]
    u32* grp_nb;           // [G] boundaries of the group (chunks = nb + 1 when non-empty)
    K* bkey;               // [S] boundary records
    u32* bpos;
    u32* cuts;             // [S*R]
    u32* below;            // [S] keys of the group at or below each boundary (sum of its cuts)
    uint4* witem;          // [2S] work items of the merge, runs of consecutive chunks of one
                           // group that together fit the cap: {first slot, last slot, group,
                           // first chunk}, {last chunk, group boundaries, group output base, 0}
    u32* nwork;            // [1] work items
    u32* heavy;            // [G] groups with chunk boundaries (listed by k_mwm_size)
    u32* nheavy;           // [1] their number
    uint4* gpar;           // [2G] per listed group: {f, Sg, q, dsh}, {N, 0, 0, 0} (see k_mwm_size)
    u32 S;                 // slot capacity
    int out_dt;            // BSPS_DT_NONE: keep order keys; else write raw keys of this dtype
    K* osmp;               // output samples every oys-th key of each group (or NULL), at most
                           // ospb per group (later ones are not written)
    u32 oys, ospb;
    const u32* gsh;        // optional, per group: its runs sorted by key >> gsh[g] only (see TileArgs):
                           // boundaries then cut on that part alone, never inside a group of equal
                           // high parts
    u32 gsh_one;           // nonzero: every group's runs use the one shift gsh[0]
    u32 ggrow;             // keys a boundary gains over all runs when cut on a high part (estimate)
    u32 pack;              // nonzero: plan quarter-tile chunks where a lone chunk would fill the tile
                           // poorly (merges whose chunk sorts take many digit passes)
    // Optional [1]: with *ssh = D > 0 a chunk is sorted on key >> D only, when
    // no group of equal key >> D holds more than TRUNC_L of its records (else
    // in full), so the output is sorted on key >> D and every such group of
    // more than TRUNC_L records is exactly sorted. Needs boundaries on a part
    // at least as coarse (gsh >= D), so that no such group spans two chunks.
    const u32* ssh;
};

// Largest group of equal key >> D that a chunk sorted on key >> D may hold:
// one wave sorts such a group in place.
constexpr int TRUNC_L = 64;

// Per-tile sort arguments. Tile t of block k covers
// [start_k + t*T, min(start_k + (t+1)*T, end_k)).
template <typename K>
struct TileArgs {
    const K* in;
    const u32* inv;
    K* out;
    u32* outv;
    i64 n;
    int p, tpb;
    int in_dt, out_dt;
    K* smp;      // sample every ys-th key of each tile, tile slot stride spt
    u32 ys, spt;
    // Optional explicit tiles (segmented sorts): tile b covers
    // [btab[4b], btab[4b] + btab[4b+1]) of segment btab[4b+2]; its samples go to
    // smp[btab[4b+3] ...]. With dtab != NULL, a tile whose segment has
    // dtab[seg] != 0 is a whole segment: it is written as raw keys to outd.
    const u32* btab;
    const u32* dtab;
    K* outd;
    u32* outdv;
    // Keys only: a persistent grid loops over the ntile tiles (p*tpb, or the
    // btab entries) and loads each next tile while it sorts the current one.
    int persist;
    u32 ntile;
    // Optional (the tiles of multi-tile blocks, merged afterwards): gsh[k] > 0
    // sorts every tile of block k by the order key's bits from gsh[k] up only
    // (key >> gsh[k]), stably, so equal high parts keep their positions; the
    // merge then cuts the block's runs on that part and sorts each chunk in full.
    const u32* gsh;
};

// Processor k owns [floor(k n / p), floor((k+1) n / p)): blocks differ in size by at most one.
__device__ __forceinline__ i64 blk_start(i64 n, int p, int k) { return (i64)(((u64)k * (u64)n) / (u64)p); }

// Block merge tables: group = block k, run = tile t.
template <typename K>
__global__ void k_block_tables(i64 n, int p, int tpb, u32 T, u32 ys, u32 spt, u32* run_start, u32* run_len,
                               u32* out_base, u32* sdesc) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)p * tpb) return;
    const int k = (int)(idx / tpb), t = (int)(idx % tpb);
    const i64 st = blk_start(n, p, k), en = blk_start(n, p, k + 1);
    i64 a = st + (i64)t * T;
    i64 len = en - a;
    len = len < 0 ? 0 : (len > (i64)T ? (i64)T : len);
    run_start[idx] = (u32)(a < en ? a : en);
    run_len[idx] = (u32)len;
    if (t == 0) out_base[k] = (u32)st;
    sdesc[idx * 4 + 0] = (u32)idx * spt;
    sdesc[idx * 4 + 1] = (u32)(len / ys);
    sdesc[idx * 4 + 2] = (u32)(a + ys - 1);
    sdesc[idx * 4 + 3] = ys;
}

__global__ void k_zero_u32(u32* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_fill_u32(u32* p, int n, u32 v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ======================================================================= tile sort

// Stores the sorted tile held in the exchange buffer (rebased keys) to out and
// emits every ys-th key (ys a power of two) to the sample array.
template <typename K, typename SK, int NT, int IT>
__device__ __forceinline__ void store_sorted(const SK* ex, K mn, int cnt, K* out, int out_dt, K* smp, i64 sbase,
                                             u32 ysh) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const int i = j * NT + t;
        if (i < cnt) out[i] = rawkey<K>((K)ex[padj<NT>(j, t)] + mn, out_dt);
    }
    // samples: every (2^ysh)-th key, one strided pass over the sorted keys in LDS
    if (smp) {
        const int ns = cnt >> ysh;
        for (int k = t; k < ns; k += NT) smp[sbase + k] = (K)ex[padi(((k + 1) << ysh) - 1)] + mn;
    }
}

// Loads IT consecutive elements p[0..IT) (blocked order) into registers;
// 16-byte vector loads when the run is whole and aligned.
template <typename T, int IT>
__device__ __forceinline__ void load_blocked(const T* p, int valid, T (&r)[IT]) {
    static_assert((IT * sizeof(T)) % 16 == 0, "vector path needs whole 16-byte groups");
    if (valid >= IT && (((uintptr_t)p) & 15) == 0) {
        const uint4* q = reinterpret_cast<const uint4*>(p);
        constexpr int PER = 16 / sizeof(T);
#pragma unroll
        for (int k = 0; k < IT / PER; k++) {
            const uint4 w = q[k];
            const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
            for (int m = 0; m < PER; m++) r[k * PER + m] = e[m];
        }
    } else {
#pragma unroll
        for (int j = 0; j < IT; j++) r[j] = j < valid ? p[j] : (T)0;
    }
}

// Sorts one tile whose keys (raw, cnt of them from base; blocked order) are in
// kr, payloads in v, and writes it out with its samples.
template <typename K, bool HASV>
__device__ __forceinline__ void tile_sort_body(const TileArgs<K>& a, SortSmem<Shape<K>::NT, (int)sizeof(K), Shape<K>::IT, !HASV>& sm,
                                               K (&kr)[Shape<K>::IT], u32 (&v)[Shape<K>::IT], int cnt, i64 base,
                                               K* outk, u32* outv, int odt, K* smp, i64 sbase, int gsh = 0) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT;
    u32* vex = sm.template ex<u32>();
    const int t = threadIdx.x;
    const int valid = cnt - t * IT;  // items of this thread: positions t*IT .. t*IT+IT-1
    u32 rank[IT];
    K mn = KeyMax<K>::v, mx = 0;
#pragma unroll
    for (int j = 0; j < IT; j++) {
        kr[j] = okey<K>(kr[j], a.in_dt);
        if (j < valid) {
            mn = kr[j] < mn ? kr[j] : mn;
            mx = kr[j] > mx ? kr[j] : mx;
        }
    }
    block_minmax<NT, K>(mn, mx, sm.red64);
    // truncated sort (gsh > 0): the range starts at a multiple of 2^gsh, so
    // that (key - mn) >> gsh = (key >> gsh) - (mn >> gsh) orders like key >> gsh
    if (gsh > 0) mn &= ~(K)((((K)1) << gsh) - 1);
    const int nbits = bitwidth64((u64)(mx - mn));
    const int sbits = nbits > gsh ? nbits - gsh : 0;  // bits the passes sort on, from gsh up
    const u32 ysh = a.ys ? (u32)(__ffs(a.ys) - 1) : 0u;
    K* out = outk + base;
    if (sizeof(K) == 8 && nbits > 32) {
        u64 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = j < valid ? (u64)(kr[j] - mn) : (u64)(mx - mn);
        wg_sort_regs_top<NT, IT, HASV, (bool)BSPS_SMALLPASS, !HASV>(sk, v, rank, sbits, sm.template ex<u64>(),
                                                                    sm.cnt(), sm.wsum, gsh);
        store_sorted<K, u64, NT, IT>(sm.template ex<u64>(), mn, cnt, out, odt, smp, sbase, ysh);
    } else {
        u32 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = j < valid ? (u32)(kr[j] - mn) : (u32)(mx - mn);
        wg_sort_regs<NT, IT, u32, HASV, (bool)BSPS_SMALLPASS, !HASV>(sk, v, rank, sbits, vex, sm.cnt(), sm.wsum,
                                                                     gsh);
        store_sorted<K, u32, NT, IT>(vex, mn, cnt, out, odt, smp, sbase, ysh);
    }
    if (HASV) {
        wg_scatter_vals<NT, IT>(v, rank, vex);
        u32* ov = outv + base;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int i = j * NT + t;
            if (i < cnt) ov[i] = vex[padj<NT>(j, t)];
        }
    }
}

// Tile tt of block k: [blk_start(k) + tt*T, min(that + T, blk_start(k+1))).
template <typename K>
__device__ __forceinline__ void tile_range(const TileArgs<K>& a, u32 tile, i64& base, int& cnt) {
    constexpr int T = Shape<K>::NT * Shape<K>::IT;
    const int k = (int)(tile / (u32)a.tpb), tt = (int)(tile % (u32)a.tpb);
    const i64 st = blk_start(a.n, a.p, k), en = blk_start(a.n, a.p, k + 1);
    base = st + (i64)tt * T;
    const i64 c = en - base;
    cnt = c <= 0 ? 0 : (c > T ? T : (int)c);
}

// TT: the persistent loop reads its tiles from btab (compiled apart, so that
// the block-layout loop keeps its own register allocation).
template <typename K, bool HASV, bool TT = false>
__global__ __launch_bounds__(Shape<K>::NT, BSPS_WG_PER_CU) void k_tile_sort(TileArgs<K> a) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT;
    __shared__ SortSmem<NT, (int)sizeof(K), IT, !HASV> sm;
    const int t = threadIdx.x, i0 = t * IT;
    K kr[IT];
    u32 v[IT];
    if (!HASV && !TT && a.persist) {
        const u32 ntile = (u32)a.p * (u32)a.tpb;
        u32 tile = blockIdx.x;
        i64 base;
        int cnt;
        if (tile >= ntile) return;
        tile_range(a, tile, base, cnt);
        K nk[IT];
        // a tile's shift is read before its keys: loads complete in order, so
        // waiting for the shift never waits for the keys in flight behind it
        u32 ngsh = a.gsh ? a.gsh[tile / (u32)a.tpb] : 0u;
        load_blocked<K, IT>(a.in + base + i0, cnt - i0, nk);
#pragma unroll
        for (int j = 0; j < IT; j++) v[j] = 0;
        for (;;) {
#pragma unroll
            for (int j = 0; j < IT; j++) kr[j] = nk[j];
            const i64 cbase = base;
            const int ccnt = cnt;
            const u32 ctile = tile, cgsh = ngsh;
            tile += gridDim.x;
            // the next tile's keys are in flight while this one is sorted
            if (tile < ntile) {
                tile_range(a, tile, base, cnt);
                ngsh = a.gsh ? a.gsh[tile / (u32)a.tpb] : 0u;
                load_blocked<K, IT>(a.in + base + i0, cnt - i0, nk);
            }
            if (ccnt > 0)
                tile_sort_body<K, HASV>(a, sm, kr, v, ccnt, cbase, a.out, a.outv, a.out_dt, a.smp,
                                        (i64)ctile * a.spt, (int)uniform(cgsh));
            if (tile >= ntile) break;
            __syncthreads();
        }
        return;
    }
    if (!HASV && TT && a.persist) {
        // tile -> its keys [base, base + cnt), output, output type and samples
        auto info = [&](u32 tile, i64& base, int& cnt, K*& outk, int& odt, K*& smp, i64& sbase) {
            outk = a.out;
            odt = a.out_dt;
            smp = a.smp;
            if (TT) {
                const u32* bt = a.btab + 4 * (i64)tile;
                base = bt[0];
                cnt = bt[1] > (u32)(NT * IT) ? NT * IT : (int)bt[1];
                sbase = bt[3];
                if (a.dtab && a.dtab[bt[2]]) {
                    outk = a.outd;
                    odt = a.in_dt;
                    smp = nullptr;
                } else {
                    odt = BSPS_DT_NONE;
                }
            } else {
                tile_range(a, tile, base, cnt);
                sbase = (i64)tile * a.spt;
            }
        };
        u32 tile = blockIdx.x;
        if (tile >= a.ntile) return;
        i64 base, sbase;
        int cnt, odt;
        K *outk, *smp;
        info(tile, base, cnt, outk, odt, smp, sbase);
        K nk[IT];
        load_blocked<K, IT>(a.in + base + i0, cnt - i0, nk);
#pragma unroll
        for (int j = 0; j < IT; j++) v[j] = 0;
        for (;;) {
#pragma unroll
            for (int j = 0; j < IT; j++) kr[j] = nk[j];
            const i64 cbase = base, csbase = sbase;
            const int ccnt = cnt, codt = odt;
            K* const coutk = outk;
            K* const csmp = smp;
            tile += gridDim.x;
            // the next tile's keys are in flight while this one is sorted
            if (tile < a.ntile) {
                info(tile, base, cnt, outk, odt, smp, sbase);
                load_blocked<K, IT>(a.in + base + i0, cnt - i0, nk);
            }
            if (ccnt > 0) tile_sort_body<K, HASV>(a, sm, kr, v, ccnt, cbase, coutk, nullptr, codt, csmp, csbase);
            if (tile >= a.ntile) break;
            __syncthreads();
        }
        return;
    }
    i64 base, cnt64, sbase = (i64)blockIdx.x * a.spt;
    K* outk = a.out;
    u32* outv = a.outv;
    int odt = a.out_dt;
    K* smp = a.smp;
    if (a.btab) {
        const u32* bt = a.btab + 4 * (i64)blockIdx.x;
        base = bt[0];
        cnt64 = bt[1];
        sbase = bt[3];
        if (a.dtab && a.dtab[bt[2]]) {
            outk = a.outd;
            outv = a.outdv;
            odt = a.in_dt;
            smp = nullptr;
        } else {
            odt = BSPS_DT_NONE;
        }
    } else {
        int c;
        tile_range(a, blockIdx.x, base, c);
        cnt64 = c;
    }
    const int cnt = cnt64 <= 0 ? 0 : (cnt64 > NT * IT ? NT * IT : (int)cnt64);
    if (cnt == 0) return;
    // the shift is read first, so that its latency hides behind the key loads
    const u32 gsh = (a.gsh && !a.btab) ? a.gsh[blockIdx.x / (u32)a.tpb] : 0u;
    load_blocked<K, IT>(a.in + base + i0, cnt - i0, kr);
    if (HASV) load_blocked<u32, IT>(a.inv + base + i0, cnt - i0, v);
    tile_sort_body<K, HASV>(a, sm, kr, v, cnt, base, outk, outv, odt, smp, sbase, (int)uniform(gsh));
}

// ======================================================================= MWM: pick boundaries

// Chunking of every group, one light workgroup per group: the group's size N
// and sample count, the subsample factor f (at most T subsamples are sorted),
// the chunk target and the boundary count nb (below). Slots are allocated and
// mapped to the group; a group without boundaries gets its one work item here,
// the others are listed for k_mwm_pick and k_mwm_plan with their parameters.
//
// The chunk target leaves room for the spread of chunk sizes: a chunk holds q
// samples' worth of keys plus, per run, less than one sample stride y more or
// fewer, so its size varies by about y * sqrt(R / 3); the target is cap minus
// four such spreads (but at least a.tavg, the floor the slot capacity was
// sized for).
constexpr int SIZE_NT = 256;

// Subsample of the merge's boundary pick: run r takes its samples r mod f,
// r mod f + f, ... (of s_r samples). Its count, and their total over the R
// runs of a group (one workgroup).
__device__ __forceinline__ u32 mwm_sub_count(u32 s_r, int r, u32 f) {
    const u32 ph = (u32)r % f;
    return s_r > ph ? (s_r - 1u - ph) / f + 1u : 0u;
}
template <int NT>
__device__ u32 mwm_sub_total(const u32* sd, int R, u32 f, u32* wsum) {
    u32 my = 0;
    for (int r = threadIdx.x; r < R; r += NT) my += mwm_sub_count(sd[r * 4 + 1], r, f);
    u32 tot;
    __syncthreads();  // wsum is free
    (void)block_excl_scan<NT>(my, tot, wsum);
    return tot;
}

template <typename K>
__global__ __launch_bounds__(SIZE_NT) void k_mwm_size(MwmArgs<K> a) {
    constexpr int T = Shape<K>::NT * Shape<K>::IT;
    __shared__ u32 wsum[SIZE_NT / 64 + 2];
    __shared__ u32 sh_base;
    const int t = threadIdx.x, g = blockIdx.x, R = a.R;
    const u32* sd = a.sdesc + (i64)g * R * 4;
    u32 mys = 0, myn = 0;
    for (int r = t; r < R; r += SIZE_NT) {
        mys += sd[r * 4 + 1];
        myn += a.run_len[(i64)g * R + r];
    }
    u32 Sraw, N;
    (void)block_excl_scan<SIZE_NT>(mys, Sraw, wsum);
    __syncthreads();
    (void)block_excl_scan<SIZE_NT>(myn, N, wsum);
    u32 nb = 0, f = 1, Sg = 0, q = 1, dsh = 0;
    if (N > a.cap && Sraw > 0) {
        // Subsample: every f-th sample of each run, run r from its sample
        // r mod f on (mwm_sub_count). Every run's j-th sample sits near the
        // same quantile when the runs are alike (tiles of one block), so with
        // one phase for all runs the subsamples line up across runs near both
        // ends of the key range, and a boundary there takes the keys below a
        // whole row of them at once: chunks of up to R * f * ys keys. With
        // the phases staggered the rows interleave.
        f = (Sraw + T - 1) / T;
        Sg = mwm_sub_total<SIZE_NT>(sd, R, f, wsum);
        if (Sg > (u32)T) {  // a run's count rounds up by less than 1: one more step fits
            f++;
            Sg = mwm_sub_total<SIZE_NT>(sd, R, f, wsum);
        }
        if (Sg > (u32)T) Sg = 0;  // (R <= T / 3 rules it out) no boundaries: one chunk
    }
    if (N > a.cap && Sg > 0) {
        const float yeff = (float)N / (float)Sg;
        const float spread = 4.0f * yeff * sqrtf((float)R / 3.0f);
        float tgf = (float)a.cap - spread;
        // (MwmArgs.pack) A chunk's sort takes every digit pass over the whole
        // tile, however full, and k_mwm_plan packs consecutive chunks by their
        // exact sizes: when a lone chunk would fill under 3/4 of the tile,
        // chunks of a quarter tile pack it fuller, for more cuts (int64 blocks
        // of 128 tiles: 0.61 -> 0.87 of the tile per merge item).
        if (a.pack && tgf < 0.75f * (float)a.cap) tgf = (float)a.tavg;
        u32 tg = tgf < (float)a.tavg ? a.tavg : (u32)tgf;
        u64 qq = ((u64)tg * Sg + N - 1) / N;
        q = qq < 1 ? 1u : (u32)qq;
        // The keys at or below a boundary include, in every run, the keys
        // after its last subsample at or below it: about half a subsample
        // spacing (f samples of stride ys) per run. That offset cancels
        // between consecutive boundaries but not in the first chunk, so all
        // boundaries move down by it (in subsample ranks, at most q - 1).
        // Symmetrically every run ends with about half a spacing of keys
        // after its last subsample, which the last chunk holds: the boundary
        // count covers Sg + dsh ranks so that those keys are not left over.
        const float ys = (float)(sd[3] ? sd[3] : 1u);
        float off = 0.5f * (float)R * (float)f * ys / yeff;
        // Runs cut on a high part: every boundary moves to the end of its
        // group, about ggrow keys further over all runs, which again only the
        // first chunk keeps.
        if (a.ggrow && a.gsh && a.gsh[a.gsh_one ? 0u : g] > 0u) off += (float)a.ggrow / yeff;
        dsh = off >= (float)(q - 1) ? q - 1 : (u32)off;
        nb = (Sg + dsh) / q;
    }
    if (t == 0) {
        u32 slots = N > 0 ? nb + 1 : 0;
        u32 b = slots ? atomicAdd(a.slot_count, slots) : 0u;
        if (b + slots > a.S) { slots = 0; b = a.S; }  // cannot happen: capacity n/tavg + 2G + 1
        sh_base = b;
        a.grp_base[g] = b;
        a.grp_nb[g] = slots ? nb : 0u;
        if (slots && nb > 0) {
            const u32 h = atomicAdd(a.nheavy, 1u);
            a.heavy[h] = (u32)g;
            a.gpar[2 * (i64)g] = make_uint4(f, Sg, q, dsh);
            a.gpar[2 * (i64)g + 1] = make_uint4(N, 0u, 0u, 0u);
        } else if (slots) {  // one chunk: its work item
            const u32 w = atomicAdd(a.nwork, 1u);
            a.witem[2 * (i64)w] = make_uint4(b, b, (u32)g, 0u);
            a.witem[2 * (i64)w + 1] = make_uint4(0u, 0u, a.out_base[g], 0u);
        }
    }
    __syncthreads();
    const u32 gb = sh_base;
    if (N == 0 || gb >= a.S) return;
    for (u32 i = t; i <= nb; i += SIZE_NT) a.slot_group[gb + i] = (u32)g;
}

// Boundaries of the listed groups, workgroups looping over the list: sort (a
// regular subsample of) the group's samples and keep every q-th as a chunk
// boundary (parameters from k_mwm_size).
template <typename K>
__global__ __launch_bounds__(Shape<K>::NT) void k_mwm_pick(MwmArgs<K> a) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT;
    __shared__ SortSmem<NT, (int)sizeof(K), IT> sm;
    __shared__ u32 spre[MAXR + 1];
    __shared__ u32 sbase[MAXR];  // first sample index of each run
    __shared__ u32 spre2[MAXR + 1];  // prefix of the runs' subsample counts
    u32* vex = sm.template ex<u32>();
    const int t = threadIdx.x, R = a.R;
    const u32 nheavy = *a.nheavy;
    for (u32 h = blockIdx.x; h < nheavy; h += gridDim.x) {
        const u32 g = uniform(a.heavy[h]);
        const int gsh = a.gsh ? (int)uniform(a.gsh[a.gsh_one ? 0u : g]) : 0;
        const uint4 gp = a.gpar[2 * (i64)g];
        const u32 f = uniform(gp.x), Sg = uniform(gp.y), q = uniform(gp.z), dsh = uniform(gp.w);
        const u32 gb = uniform(a.grp_base[g]), nb = uniform(a.grp_nb[g]);
        const u32* sd = a.sdesc + (i64)g * R * 4;
        // exclusive prefixes of the runs' sample and subsample counts (runs in order)
        const int RPT = (R + NT - 1) / NT;
        u32 mys = 0, myq = 0;
        for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
            mys += sd[r * 4 + 1];
            myq += mwm_sub_count(sd[r * 4 + 1], r, f);
        }
        // one scan of both sums: sample counts (low 32 bits), subsample counts (high)
        u64 both;
        const u64 exb = block_excl_scan64<NT>(((u64)myq << 32) | mys, both, sm.red64);
        u32 ex = (u32)exb, ex2 = (u32)(exb >> 32);
        for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
            spre[r] = ex;
            spre2[r] = ex2;
            sbase[r] = sd[r * 4 + 0];
            ex += sd[r * 4 + 1];
            ex2 += mwm_sub_count(sd[r * 4 + 1], r, f);
        }
        if (t == 0) {
            spre[R] = (u32)both;
            spre2[R] = (u32)(both >> 32);  // = Sg
        }
        __syncthreads();
        // load the subsample: element i is run r's sample (r mod f) + (i -
        // spre2[r]) * f, r the run with spre2[r] <= i < spre2[r + 1]; c, its
        // concatenated sample index, increases with i. A thread's elements are
        // consecutive, so the run holding its first one is found by bisection
        // and the rest by walking; every sample index is formed first and all
        // loads are then issued together.
        K mn = KeyMax<K>::v, mx = 0;
        u32 v[IT], rank[IT];
        K key[IT];
        {
            const u32 i0 = (u32)(t * IT);
            int r = 0;
            if (i0 < Sg) {
                int lo = 0, hi = R;  // largest r with spre2[r] <= i0 (a run with subsamples)
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (spre2[mid] <= i0) lo = mid; else hi = mid;
                }
                r = lo;
            }
    #pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = i0 + (u32)j;
                v[j] = 0;
                key[j] = 0;
                if (i < Sg) {
                    while (spre2[r + 1] <= i) r++;  // stops at r < R: spre2[R] = Sg > i
                    const u32 c = spre[r] + (u32)r % f + (i - spre2[r]) * f;
                    key[j] = (K)(sbase[r] + (c - spre[r]));
                    v[j] = c;
                }
            }
    #pragma unroll
            for (int j = 0; j < IT; j++) {
                if (i0 + (u32)j < Sg) {
                    key[j] = a.smp[(u32)key[j]];
                    mn = key[j] < mn ? key[j] : mn;
                    mx = key[j] > mx ? key[j] : mx;
                }
            }
        }
        block_minmax<NT, K>(mn, mx, sm.red64);
        // with runs cut on key >> gsh a boundary takes the upper bound of its
        // high part, and the high part at a given rank does not depend on the
        // order inside equal high parts: the subsample is sorted on the high
        // part only (the minimum aligned down so that the order is key >> gsh's)
        const K mna = gsh > 0 ? (K)(mn & ~((((K)1) << gsh) - 1)) : mn;
        const int nbits = bitwidth64((u64)((mx - mna) >> gsh));
        if (sizeof(K) == 8 && nbits > 32) {
            u64 sk[IT];
    #pragma unroll
            for (int j = 0; j < IT; j++)
                sk[j] = (u64)(((u32)(t * IT + j) < Sg ? key[j] - mna : mx - mna) >> gsh);
            wg_sort_regs_top<NT, IT, true, false>(sk, v, rank, nbits, sm.template ex<u64>(), sm.cnt(), sm.wsum);
            u64* e = sm.template ex<u64>();
    #pragma unroll
            for (int j = 0; j < IT; j++) key[j] = (K)((e[padi(t * IT + j)] << gsh) + (u64)mna);
        } else {
            u32 sk[IT];
    #pragma unroll
            for (int j = 0; j < IT; j++)
                sk[j] = (u32)(((u32)(t * IT + j) < Sg ? key[j] - mna : mx - mna) >> gsh);
            wg_sort_regs<NT, IT, u32, true, false>(sk, v, rank, nbits, vex, sm.cnt(), sm.wsum);
    #pragma unroll
            for (int j = 0; j < IT; j++) key[j] = ((K)vex[padi(t * IT + j)] << gsh) + mna;
        }
        wg_scatter_vals<NT, IT>(v, rank, vex);
        // boundary b (1..nb) = sorted element b*q - 1 - dsh
    #pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(t * IT + j);
            if (i < Sg && (i + 1 + dsh) % q == 0 && (i + 1 + dsh) / q <= nb) {
                const u32 b = (i + 1 + dsh) / q;
                const u32 c = vex[padi((int)i)];
                int lo = 0, hi = R;
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (spre[mid] <= c) lo = mid; else hi = mid;
                }
                if (gsh > 0) {
                    // runs sorted by key >> gsh: the boundary is every record whose
                    // high part is at most this one's (largest key of that part,
                    // any position)
                    a.bkey[gb + b - 1] = key[j] | (K)((((K)1) << gsh) - 1);
                    a.bpos[gb + b - 1] = 0xFFFFFFFFu;
                } else {
                    a.bkey[gb + b - 1] = key[j];
                    a.bpos[gb + b - 1] = sd[lo * 4 + 2] + (c - spre[lo]) * sd[lo * 4 + 3];
                }
            }
        }
        __syncthreads();  // LDS is reused by the next listed group
    }
}

// ======================================================================= MWM: exact cuts

// cuts[slot*R + r] = number of records of run r that are <= the boundary record
// of that slot (key first, then position). One wave per (group, run, share of
// the group's boundaries): the run's samples (every stride-th key, stored
// compactly) are staged in LDS and each boundary is searched there (in global
// memory when the run has more samples than the stage holds); the cut then
// lies within one stride of the run, which is bisected in global memory. The
// kernel is bound by the number of scattered global requests per search, which
// the staging cuts from about lg(samples) + lg(stride) to lg(stride).
// gridDim.y splits the boundaries of a (group, run) over several waves when
// there are few runs.
constexpr int CUT_NT = 256, CUT_SMAX = 1024;
#ifndef BSPS_CUT_BP
#define BSPS_CUT_BP 8  // boundary pairs whose window loads are issued together
#endif

template <typename K, bool COOP>
__global__ __launch_bounds__(CUT_NT) void k_mwm_cuts(MwmArgs<K> a) {
    __shared__ K ls[CUT_NT / 64][CUT_SMAX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, R = a.R;
    const i64 gr = (i64)blockIdx.x * (CUT_NT / 64) + w;
    const bool live = gr < (i64)a.G * R;
    u32 nb = 0, gb = 0, rs = 0, len = 0, sidx = 0, scnt = 0, pb = 0, sstr = 1;
    if (live) {
        const u32 g = (u32)(gr / R);
        nb = a.grp_nb[g];
        gb = a.grp_base[g];
        rs = a.run_start[gr];
        len = a.run_len[gr];
        const u32* d = a.sdesc + gr * 4;
        sidx = d[0];
        scnt = d[1];
        pb = d[2];
        sstr = d[3];
    }
    nb = uniform(nb); gb = uniform(gb); rs = uniform(rs); len = uniform(len);
    sidx = uniform(sidx); scnt = uniform(scnt); pb = uniform(pb); sstr = uniform(sstr);
    const bool staged = scnt <= (u32)CUT_SMAX;
    K* st = ls[w];
    const u32 step = 64u * gridDim.y;
    // the boundaries of the wave's first pass load while the samples are
    // staged, and every pass loads the next pass's boundaries ahead
    K nbk = 0;
    u32 nbp = 0;
    if (live && blockIdx.y * 64u + (u32)lane < nb) {
        nbk = a.bkey[gb + blockIdx.y * 64u + (u32)lane];
        nbp = a.bpos[gb + blockIdx.y * 64u + (u32)lane];
    }
    if (live && nb > 0 && staged)
        for (u32 j = lane; j < scnt; j += 64) st[j] = a.smp[sidx + j];
    __syncthreads();
    if (!live || nb == 0) return;
    const u32 r = (u32)(gr % R);
    const int half = lane >> 5, hl = lane & 31;
    for (u32 c0 = blockIdx.y * 64u; c0 < nb; c0 += step) {
        const u32 c = c0 + (u32)lane;
        const bool act = c < nb;
        const u32 slot = gb + c;
        const K bk = nbk;
        const u32 bp = nbp;
        if (c + step < nb) {
            nbk = a.bkey[slot + step];
            nbp = a.bpos[slot + step];
        }
        u32 wlo = 0, whi = 0;
        if (act) {
            // J = samples of this run that are <= the boundary
            u32 lo = 0, hi = scnt;
            if (staged) {
                while (lo < hi) {
                    const u32 mid = (lo + hi) >> 1;
                    if (rec_le<K>(st[mid], pb + mid * sstr, bk, bp)) lo = mid + 1; else hi = mid;
                }
            } else {
                while (lo < hi) {
                    const u32 mid = (lo + hi) >> 1;
                    if (rec_le<K>(a.smp[sidx + mid], pb + mid * sstr, bk, bp)) lo = mid + 1; else hi = mid;
                }
            }
            const u32 J = lo;
            wlo = J > 0 ? pb + (J - 1) * sstr - rs + 1 : 0u;
            whi = J < scnt ? pb + J * sstr - rs : len;
        }
        // The cut lies in [wlo, whi): the records between two neighbouring
        // samples, fewer than the stride. COOP (4-byte keys, many boundaries per
        // group): when every window of the wave holds at most 32 records (stride
        // 32), a half-wave reads one boundary's window in one coalesced load and
        // counts the records at or below the boundary with a ballot (they are a
        // prefix of the window, the run being sorted): per boundary one request
        // for one or two cache lines instead of a bisection's five dependent
        // ones, each a line of its own. The windows of 2 BP boundaries are read
        // together so their loads are in flight at once. Only for boundaries on
        // a high part (runs sorted under a shift, which the probe allows only
        // without heavy duplicates): where many boundaries share a key, the
        // lanes' bisections read the same lines and are cheaper. With few
        // boundaries per wave the batch is mostly idle, so the bisection alone
        // is built there.
        const u32 wl = whi - wlo;
        constexpr int BP = BSPS_CUT_BP;  // boundary pairs per batch
        if (COOP && __all(!act || (wl <= 32u && bp == 0xFFFFFFFFu))) {
            const u32 nact = min(64u, nb - c0);
            u32 res = 0;
            for (u32 m0 = 0; m0 < nact; m0 += 2u * BP) {
                K v[BP];
                u32 pos[BP];
                bool in[BP];
#pragma unroll
                for (int q = 0; q < BP; q++) {
                    const int src = (int)m0 + 2 * q + half;
                    const u32 w0 = (u32)__shfl((int)wlo, src, 64), wn = (u32)__shfl((int)wl, src, 64);
                    in[q] = (u32)hl < wn;
                    pos[q] = rs + w0 + (u32)hl;
                    v[q] = in[q] ? a.src[pos[q]] : (K)0;
                }
#pragma unroll
                for (int q = 0; q < BP; q++) {
                    const int src = (int)m0 + 2 * q + half;
                    K kq;
                    if (sizeof(K) == 8) {
                        const u64 kb = (u64)bk;
                        const u32 lo32 = (u32)__shfl((int)(u32)kb, src, 64), hi32 = (u32)__shfl((int)(u32)(kb >> 32), src, 64);
                        kq = (K)(((u64)hi32 << 32) | lo32);
                    } else {
                        kq = (K)(u32)__shfl((int)(u32)bk, src, 64);
                    }
                    const u32 pq = (u32)__shfl((int)bp, src, 64);
                    const unsigned long long bal = __ballot(in[q] && rec_le<K>(v[q], pos[q], kq, pq));
                    const u32 m = m0 + 2u * (u32)q;
                    if ((u32)lane == m) res = (u32)__popcll(bal & 0xFFFFFFFFull);
                    if ((u32)lane == m + 1u) res = (u32)__popcll(bal >> 32);
                }
            }
            if (act) a.cuts[(i64)slot * R + r] = wlo + res;
        } else if (act) {
            while (wlo < whi) {
                const u32 mid = (wlo + whi) >> 1;
                if (rec_le<K>(a.src[rs + mid], rs + mid, bk, bp)) wlo = mid + 1; else whi = mid;
            }
            a.cuts[(i64)slot * R + r] = wlo;
        }
    }
}

// below[slot] = sum of the slot's cuts over the runs: the keys of its group at
// or below its boundary. One wave per slot.
template <typename K>
__global__ __launch_bounds__(256) void k_mwm_below(MwmArgs<K> a) {
    const u32 nslot = min(a.S, *a.slot_count);
    const int lane = threadIdx.x & 63, R = a.R;
    for (u32 slot = blockIdx.x * 4u + (threadIdx.x >> 6); slot < nslot; slot += gridDim.x * 4u) {
        const u32 g = a.slot_group[slot];
        if (slot - a.grp_base[g] >= a.grp_nb[g]) continue;  // a group's last chunk has no boundary
        const u32* row = a.cuts + (i64)slot * R;
        u32 v = 0;
        for (int i = lane; i < R; i += 64) v += row[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) a.below[slot] = v;
    }
}

// ======================================================================= MWM: work items

// The exact size of every chunk of a group follows from the cuts (the keys at
// or below boundary c are the sum of its cuts over the runs). Consecutive
// chunks are combined while they fit the cap, so that groups whose sample
// forced small chunks (large groups, few samples per key) still fill the LDS
// sort; a chunk above the cap stays alone. Workgroups loop over the groups
// listed by k_mwm_size (a group of one chunk got its work item there).
constexpr int PLAN_NT = 256, PLAN_MAXC = 4096;
template <typename K>
__global__ __launch_bounds__(PLAN_NT) void k_mwm_plan(MwmArgs<K> a) {
    __shared__ u32 P[PLAN_MAXC];
    __shared__ unsigned short itf[PLAN_MAXC], itl[PLAN_MAXC];
    __shared__ u32 sh_n, sh_base;
    const int t = threadIdx.x;
    const u32 nheavy = *a.nheavy;
    for (u32 h = blockIdx.x; h < nheavy; h += gridDim.x) {
        __syncthreads();  // LDS of the previous listed group is free
        const u32 g = uniform(a.heavy[h]);
        const u32 gb = uniform(a.grp_base[g]), nb = uniform(a.grp_nb[g]), ob = uniform(a.out_base[g]);
        const u32 N = uniform(a.gpar[2 * (i64)g + 1].x);
        auto item = [&](u32 i, u32 cf, u32 cl) {
            a.witem[2 * (i64)i] = make_uint4(gb + cf, gb + cl, g, cf);
            a.witem[2 * (i64)i + 1] = make_uint4(cl, nb, ob, 0u);
        };
        const u32 nch = nb + 1;
        if (nch > PLAN_MAXC) {  // not combined: one item per chunk
            if (t == 0) sh_base = atomicAdd(a.nwork, nch);
            __syncthreads();
            for (u32 c = t; c < nch; c += PLAN_NT) item(sh_base + c, c, c);
            continue;
        }
        for (u32 c = t; c < nb; c += PLAN_NT) P[c] = a.below[gb + c];
        __syncthreads();
        // greedy combination by wave 0: 64 chunk sizes at a time in registers,
        // walked in order with uniform (scalar) state
        if (t < 64) {
            u32 n = 0, first = 0, acc = 0, prev = 0;
            for (u32 c0 = 0; c0 < nch; c0 += 64) {
                const u32 mine = c0 + t < nb ? P[c0 + t] : N;
                const u32 cnt = min(64u, nch - c0);
                for (u32 j = 0; j < cnt; j++) {
                    const u32 below = (u32)__builtin_amdgcn_readlane((int)mine, (int)j);
                    const u32 sz = below - prev;
                    prev = below;
                    if (c0 + j > 0 && acc + sz > a.cap) {
                        if (t == 0) {
                            itf[n] = (unsigned short)first;
                            itl[n] = (unsigned short)(c0 + j - 1);
                        }
                        n++;
                        first = c0 + j;
                        acc = 0;
                    }
                    acc += sz;
                }
            }
            if (t == 0) {
                itf[n] = (unsigned short)first;
                itl[n] = (unsigned short)nb;
                sh_n = n + 1;
                sh_base = atomicAdd(a.nwork, n + 1);
            }
        }
        __syncthreads();
        for (u32 i = t; i < sh_n; i += PLAN_NT) item(sh_base + i, itf[i], itl[i]);
    }
}

// ======================================================================= MWM: chunk sort

template <typename K, bool HASV>
__device__ void mwm_emit(const MwmArgs<K>& a, u32 g, u32 o, K u, u32 gstart) {
    if (a.osmp) {
        const u32 rel = o - gstart + 1;
        if ((rel & (a.oys - 1)) == 0 && rel / a.oys <= a.ospb) a.osmp[(i64)g * a.ospb + rel / a.oys - 1] = u;
    }
}

// o[d] = h[0] + ... + h[d-1] for the RADIX digits, by wave 0 in steps of 64.
__device__ __forceinline__ void digit_excl_scan(const u32* h, u32* o, int t) {
    if (t < 64) {
        u32 carry = 0;
        for (int d0 = 0; d0 < RADIX; d0 += 64) {
            const u32 hv = d0 + t < RADIX ? h[d0 + t] : 0u;
            const u32 inc = wave_incl_scan(hv);
            if (d0 + t < RADIX) o[d0 + t] = carry + inc - hv;
            carry += (u32)__shfl((int)inc, 63, 64);
        }
    }
}

// Oversize chunk: LSD radix passes through global memory by one workgroup.
// Pieces are first copied (in run order) to scr[out .. out+N), then sorted by
// digit passes alternating scr <-> dst; the last step writes dst.
template <typename K, bool HASV>
__device__ void mwm_oversize(const MwmArgs<K>& a, u32 g, u32 slot, u32 c, u32 nb, const u32* ppre, u32 N,
                             u32 out, SortSmem<Shape<K>::NT, (int)sizeof(K), Shape<K>::IT>& sm, K* exch) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT;
    const int t = threadIdx.x, R = a.R;
    const int lane = t & 63, w = t >> 6, NW = NT / 64;
    __shared__ u32 hist[RADIX], doff[RADIX], tcnt[RADIX], tbase[RADIX];
    K mn = KeyMax<K>::v, mx = 0;
    for (int r = w; r < R; r += NW) {
        const u32 lo = c == 0 ? 0u : a.cuts[(i64)(slot - 1) * R + r];
        const u32 len = ppre[r + 1] - ppre[r];
        const u32 rs = a.run_start[(i64)g * R + r] + lo;
        for (u32 i = lane; i < len; i += 64) {
            K u = a.src[rs + i];
            a.scr[out + ppre[r] + i] = u;
            if (HASV) a.scrv[out + ppre[r] + i] = a.srcv[rs + i];
            mn = u < mn ? u : mn;
            mx = u > mx ? u : mx;
        }
    }
    block_minmax<NT, K>(mn, mx, sm.red64);
    __threadfence_block();
    const int nbits = bitwidth64((u64)(mx - mn));
    K* X = a.scr + out;
    u32* XV = a.scrv ? a.scrv + out : nullptr;
    K* Y = a.dst + out;
    u32* YV = a.dstv ? a.dstv + out : nullptr;
    for (int sh = 0; sh < nbits; sh += RB) {
        if (t < RADIX) hist[t] = 0;
        __syncthreads();
        for (u32 i = t; i < N; i += NT) atomicAdd(&hist[(u32)((u64)(X[i] - mn) >> sh) & (RADIX - 1)], 1u);
        __syncthreads();
        digit_excl_scan(hist, doff, t);
        __syncthreads();
        for (u32 b0 = 0; b0 < N; b0 += T) {
            u32 dig[IT], rank[IT];
            K kk[IT];
            u32 vv[IT];
            if (t < RADIX) tcnt[t] = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = b0 + t * IT + j;
                if (i < N) {
                    kk[j] = X[i];
                    if (HASV) vv[j] = XV[i];
                    dig[j] = (u32)((u64)(kk[j] - mn) >> sh) & (RADIX - 1);
                    atomicAdd(&tcnt[dig[j]], 1u);
                } else {
                    kk[j] = 0;
                    vv[j] = 0;
                    dig[j] = RADIX - 1;
                }
            }
            __syncthreads();
            digit_excl_scan(tcnt, tbase, t);
            radix_rank<NT, IT>([&](int j) { return dig[j]; }, [&](int j) { return (dig[j] >> (RB - 5)) & 16u; }, rank,
                               sm.cnt(), sm.wsum);
#pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = b0 + t * IT + j;
                if (i < N) {
                    const u32 d = dig[j];
                    const u32 dst = doff[d] + rank[j] - tbase[d];
                    Y[dst] = kk[j];
                    if (HASV) YV[dst] = vv[j];
                }
            }
            __syncthreads();
            if (t < RADIX) doff[t] += tcnt[t];
            __syncthreads();
        }
        __threadfence_block();
        K* tk = X; X = Y; Y = tk;
        u32* tv = XV; XV = YV; YV = tv;
        __syncthreads();
    }
    // X holds the sorted chunk; write dst (raw keys when requested) and samples.
    const u32 gstart = a.out_base[g];
    for (u32 i = t; i < N; i += NT) {
        K u = X[i];
        a.dst[out + i] = rawkey<K>(u, a.out_dt);
        if (HASV) a.dstv[out + i] = XV[i];
        mwm_emit<K, HASV>(a, g, out + i, u, gstart);
    }
    (void)exch;
    (void)nb;
}

template <typename K>
struct MergeSmem {
    static constexpr int NT = Shape<K>::NT, T = NT * Shape<K>::IT;
    SortSmem<NT, (int)sizeof(K), Shape<K>::IT> sm;
    u32 ppre[MAXR + 1];   // chunk offset of each piece
    u32 soff[MAXR];       // source position of each piece
    u32 slot;
};

template <typename K, bool HASV, bool TR>
__device__ __forceinline__ void mwm_merge_chunk(const MwmArgs<K>& a, const uint4 wi0, const uint4 wi1,
                                                MergeSmem<K>& S);

// Persistent merge: workgroups take work items (runs of chunks) one after
// another; the next item is claimed while the current one is merged. TR: the
// code for a sort shift (MwmArgs.ssh), left out of the other merges.
template <typename K, bool HASV, bool TR = false>
__global__ __launch_bounds__(Shape<K>::NT, BSPS_WG_PER_CU) void k_mwm_merge(MwmArgs<K> a) {
    __shared__ MergeSmem<K> S;
    // with a sort shift both variants are launched; the one for its value runs
    if (a.ssh && ((*a.ssh != 0u) != TR)) return;
    const u32 nwork = min(a.S, *a.nwork);
    if (threadIdx.x == 0) S.slot = atomicAdd(a.work, 1u);
    __syncthreads();
    u32 w = S.slot;
    for (;;) {
        __syncthreads();  // every thread has read S.slot
        if (w >= nwork) break;
        if (threadIdx.x == 0) S.slot = atomicAdd(a.work, 1u);
        mwm_merge_chunk<K, HASV, TR>(a, a.witem[2 * (i64)w], a.witem[2 * (i64)w + 1], S);
        __syncthreads();
        w = S.slot;
    }
}

// Merges the chunks slot .. slot_last of one group (one LDS sort).
template <typename K, bool HASV, bool TR>
__device__ __forceinline__ void mwm_merge_chunk(const MwmArgs<K>& a, const uint4 wi0, const uint4 wi1,
                                                MergeSmem<K>& S) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT;
    auto& sm = S.sm;
    u32* ppre = S.ppre;
    u32* soff = S.soff;
    K* exch = sm.template ex<K>();
    u32* vex = sm.template ex<u32>();
    const int t = threadIdx.x, R = a.R;
    PHASE_START;
    const u32 slot = uniform(wi0.x), slot_last = uniform(wi0.y), g = uniform(wi0.z), c = uniform(wi0.w);
    const u32 cl = uniform(wi1.x), nb = uniform(wi1.y), obase = uniform(wi1.z);
    const u32 dsh0 = (TR && a.ssh) ? *a.ssh : 0u;
    const u32* lorow = a.cuts + (i64)(slot - 1) * R;
    const u32* hirow = a.cuts + (i64)slot_last * R;
    const u32* rl = a.run_len + (i64)g * R;
    const u32* rsp = a.run_start + (i64)g * R;
    // piece lengths and their prefix (runs in order)
    const int RPT = (R + NT - 1) / NT;
    u32 mysum = 0, mylo = 0;
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
        const u32 lo = c == 0 ? 0u : lorow[r];
        const u32 hi = cl == nb ? rl[r] : hirow[r];
        mysum += hi - lo;
        mylo += lo;
    }
    // one scan of both sums: the chunk's piece lengths (low 32 bits; their
    // total N < 2^32) and the group's keys below the chunk (high 32 bits)
    u64 both;
    const u64 exb = block_excl_scan64<NT>(((u64)mylo << 32) | mysum, both, sm.red64);
    const u32 N = uniform((u32)both);
    u32 ex = (u32)exb;
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
        const u32 lo = c == 0 ? 0u : lorow[r];
        const u32 hi = cl == nb ? rl[r] : hirow[r];
        ppre[r] = ex;
        soff[r] = rsp[r] + lo;
        ex += hi - lo;
    }
    if (t == 0) ppre[R] = N;
    __syncthreads();
    const u32 out = uniform(obase + (u32)(both >> 32));
    if (N == 0) return;
    PHASE(0);
    if (N > a.cap) {
        if (t == 0) {
            atomicAdd(a.oversize, 1u);
            atomicMax(a.oversize + 2, N);  // largest oversize chunk (counters[3])
        }
        mwm_oversize<K, HASV>(a, g, slot, c, nb, ppre, N, out, sm, exch);
        return;
    }
    PHASE(1);
    // gather: item j of thread t holds chunk position t*IT + j (blocked order,
    // which the stable sort of payloads needs), or j*NT + t (striped:
    // keys-only merges through the LDS-staged gather)
    const u32 i0 = (u32)(t * IT);
    constexpr bool STRIPED = BSPS_GATHER_LDS && !HASV;
    auto item_ok = [&](int j) { return STRIPED ? (u32)(j * NT + t) < N : i0 + (u32)j < N; };
    K kr[IT];
    u32 v[IT], rank[IT];
    K mn = KeyMax<K>::v, mx = 0;
#if BSPS_GATHER_LDS
    // Every position's source index is written to LDS piece by piece; the
    // loads are then issued position-striped (consecutive lanes read
    // consecutive keys of a piece, coalesced). With payloads the keys are
    // turned back into blocked order through LDS, which the stable sort needs;
    // keys alone are sorted from the striped order, since the order of equal
    // keys cannot be seen in the output.
    {
        u32* srcidx = sm.template ex<u32>();
        if (N >= 48u * (u32)R) {
            // long pieces: each wave fills a contiguous range of pieces, 64 at
            // a time: lane l reads piece rb + l's table entries, then the wave
            // writes the pieces' positions one after another (no LDS read
            // waits on another)
            constexpr int NW = NT / 64;
            const int lane = t & 63, w = t >> 6;
            const int per = (R + NW - 1) / NW;
            const int r0 = w * per, r1 = min(R, r0 + per);
            for (int rb = r0; rb < r1; rb += 64) {
                const int r = rb + lane;
                u32 p0 = 0, len = 0, s0 = 0;
                if (r < r1) {
                    p0 = ppre[r];
                    len = ppre[r + 1] - p0;
                    s0 = soff[r];
                }
                const int nr = min(64, r1 - rb);
                for (int k = 0; k < nr; k++) {
                    const u32 q0 = (u32)__builtin_amdgcn_readlane((int)p0, k);
                    const u32 ql = (u32)__builtin_amdgcn_readlane((int)len, k);
                    const u32 qs = (u32)__builtin_amdgcn_readlane((int)s0, k);
                    for (u32 i = (u32)lane; i < ql; i += 64) srcidx[padi((int)(q0 + i))] = qs + i;
                }
            }
        } else if (i0 < N) {
            // short pieces: each thread walks its own positions from the piece
            // that holds its first one
            u32 lo = 0, hi = (u32)R - 1;
            while (lo < hi) {
                const u32 mid = (lo + hi + 1) >> 1;
                if (ppre[mid] <= i0) lo = mid; else hi = mid - 1;
            }
            u32 r = lo, nxt = ppre[lo + 1], sb = soff[lo] - ppre[lo];
#pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = i0 + j;
                if (i < N) {
                    while (i >= nxt) {
                        r++;
                        nxt = ppre[r + 1];
                        sb = soff[r] - ppre[r];
                    }
                    srcidx[padi((int)i)] = sb + i;
                }
            }
        }
        __syncthreads();
        PHASE(5);
        K ks[IT];
        u32 vs[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(j * NT + t);
            ks[j] = 0;
            vs[j] = 0;
            if (i < N) {
                const u32 si = srcidx[padj<NT>(j, t)];
                ks[j] = a.src[si];
                if (HASV) vs[j] = a.srcv[si];
            }
        }
        PHASE(6);
        if (HASV) {
            __syncthreads();
            K* exk = sm.template ex<K>();
#pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = (u32)(j * NT + t);
                if (i < N) exk[padj<NT>(j, t)] = ks[j];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) kr[j] = i0 + j < N ? exk[padi((int)(i0 + j))] : (K)0;
        } else {
#pragma unroll
            for (int j = 0; j < IT; j++) kr[j] = ks[j];
        }
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (item_ok(j)) {
                mn = kr[j] < mn ? kr[j] : mn;
                mx = kr[j] > mx ? kr[j] : mx;
            }
        }
        if (HASV) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) {
                const u32 i = (u32)(j * NT + t);
                if (i < N) srcidx[padj<NT>(j, t)] = vs[j];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = i0 + j < N ? srcidx[padi((int)(i0 + j))] : 0u;
        } else {
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = 0;
        }
        __syncthreads();
    }
#else
    if (i0 < N) {
        u32 lo = 0, hi = (u32)R - 1;  // largest piece r with ppre[r] <= i0 (a nonempty one)
        while (lo < hi) {
            const u32 mid = (lo + hi + 1) >> 1;
            if (ppre[mid] <= i0) lo = mid; else hi = mid - 1;
        }
        u32 r = lo, nxt = ppre[lo + 1], sb = soff[lo] - ppre[lo];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = i0 + j;
            kr[j] = 0;
            v[j] = 0;
            if (i < N) {
                while (i >= nxt) {
                    r++;
                    nxt = ppre[r + 1];
                    sb = soff[r] - ppre[r];
                }
                kr[j] = a.src[sb + i];
                if (HASV) v[j] = a.srcv[sb + i];
            }
        }
#pragma unroll
        for (int j = 0; j < IT; j++) {
            if (i0 + j < N) {
                mn = kr[j] < mn ? kr[j] : mn;
                mx = kr[j] > mx ? kr[j] : mx;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < IT; j++) { kr[j] = 0; v[j] = 0; }
    }
#endif
    block_minmax<NT, K>(mn, mx, sm.red64);
    PHASE(2);
    // sort on key >> dsh only when no group of equal key >> dsh holds more
    // than TRUNC_L of the chunk's records: each item is counted in an LDS
    // histogram of its high part (relative to the chunk's least, coarsened to
    // 2^13 bins, which only counts more)
    int dsh = (int)uniform(dsh0);
    if (TR && dsh > 0) {
        constexpr int TB = 1 << 13;
        u32* bins = sm.cnt();
        const K hlo = mn >> dsh;
        const int wb = bitwidth64((u64)((mx >> dsh) - hlo));
        const int cb = wb > 13 ? wb - 13 : 0;
        for (int i = t; i < TB; i += NT) bins[i] = 0u;
        if (t == 0) sm.misc[0] = 0u;
        __syncthreads();
        u32 big = 0;
#pragma unroll
        for (int j = 0; j < IT; j++)
            if (item_ok(j)) {
                const u32 e = (u32)((u64)((kr[j] >> dsh) - hlo) >> cb);
                big |= atomicAdd(&bins[e], 1u) >= (u32)TRUNC_L ? 1u : 0u;
            }
        if (big) sm.misc[0] = 1u;
        __syncthreads();
        if (sm.misc[0]) dsh = 0;
        // the range starts at a multiple of 2^dsh, so (key - mn) >> dsh orders like key >> dsh
        if (dsh > 0) mn &= ~(K)((((K)1) << dsh) - 1);
        // the padding needs a high part above every key's (see below): a key
        // range that leaves none sorts in full
        if (((u64)(mx - mn) >> dsh) + 1 > ((sizeof(K) == 4 ? 0xFFFFFFFFull : ~0ull) >> dsh)) dsh = 0;
    }
    // Sort keys are rebased on mn; the tail items past N are padding that must
    // sort after every key. Sorted in full it is the largest key (ties with it
    // are the same key); sorted on the high part it takes the next high part,
    // since keys-only merges rank items in an order where the padding is not
    // last and a tie by high part would push a key out of the chunk.
    const u64 top = dsh > 0 ? ((((u64)(mx - mn)) >> dsh) + 1) << dsh : (u64)(mx - mn);
    const int nbits = uniform(bitwidth64(top));
    const int sbits = nbits > dsh ? nbits - dsh : 0;
    const u32 gstart = obase;
    const u32 osh = a.oys ? (u32)(__ffs(a.oys) - 1) : 0u;
    const u32 om = (1u << osh) - 1;
    K* dst = a.dst + out;
    // output samples: the chunk positions whose rank in the group plus one is a
    // multiple of 2^osh, one strided pass over the sorted keys in LDS
    auto emit_samples = [&](auto* e) {
        if (a.osmp) {
            const u32 step = om + 1, first = (gstart - out - 1) & om;
            for (u32 i = first + (u32)t * step; i < N; i += (u32)NT * step) {
                const u32 si = (out + i - gstart + 1) >> osh;  // 1-based sample number in the group
                if (si <= a.ospb) a.osmp[(i64)g * a.ospb + si - 1] = (K)e[padi((int)i)] + mn;
            }
        }
    };
    if (sizeof(K) == 8 && nbits > 32) {
        u64 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = item_ok(j) ? (u64)(kr[j] - mn) : top;
        wg_sort_regs_top<NT, IT, HASV>(sk, v, rank, sbits, sm.template ex<u64>(), sm.cnt(), sm.wsum, dsh);
        const u64* e = sm.template ex<u64>();
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(j * NT + t);
            if (i < N) dst[i] = rawkey<K>((K)(e[padj<NT>(j, t)] + (u64)mn), a.out_dt);
        }
        emit_samples(e);
    } else {
        u32 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = item_ok(j) ? (u32)(kr[j] - mn) : (u32)top;
        wg_sort_regs<NT, IT, u32, HASV>(sk, v, rank, sbits, vex, sm.cnt(), sm.wsum, dsh);
        PHASE(3);
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(j * NT + t);
            if (i < N) dst[i] = rawkey<K>((K)vex[padj<NT>(j, t)] + mn, a.out_dt);
        }
        emit_samples(vex);
        PHASE(4);
    }
    if (HASV) {
        wg_scatter_vals<NT, IT>(v, rank, vex);
        u32* dv = a.dstv + out;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(j * NT + t);
            if (i < N) dv[i] = vex[padj<NT>(j, t)];
        }
    }
}

// ======================================================================= sample and splitters

// ======================================================================= high-part sorted blocks

// A block sorted on key >> D only (D > 0; the block merge with MwmArgs.ssh):
// every group of equal key >> D keeps its records in input order, and a group
// of more than TRUNC_L records is exactly sorted. Sorting every group stably
// by key gives the exactly sorted block, the same set of positions per group.
// block_key_at: the key at rank q of the exactly sorted block [st, st + mk)
// of B. The group around position q is found by scanning at most TRUNC_L
// records each way: a longer group is exact and holds that key at q; in a
// shorter one the key is the one with q - lo keys of the group below it.
template <typename K>
__device__ K block_key_at(const K* B, i64 st, i64 mk, i64 q, int D) {
    const K x = B[st + q];
    if (D <= 0) return x;
    const K h = x >> D;
    i64 lo = q, hi = q + 1;
    while (lo > 0 && q - lo < TRUNC_L && (B[st + lo - 1] >> D) == h) lo--;
    while (hi < mk && hi - lo <= TRUNC_L && (B[st + hi] >> D) == h) hi++;
    if (hi - lo > TRUNC_L) return x;
    const int g = (int)(hi - lo), r = (int)(q - lo);
    for (int i = 0; i < g; i++) {
        const K xi = B[st + lo + i];
        int less = 0, leq = 0;
        for (int j = 0; j < g; j++) {
            const K xj = B[st + lo + j];
            less += xj < xi ? 1 : 0;
            leq += xj <= xi ? 1 : 0;
        }
        if (less <= r && r < leq) return xi;
    }
    return x;  // not reached: the ranks of the group cover 0 .. g - 1
}

// The block shift D: the least fine shift of the probe over the blocks
// (fine[k] = gsh[p + 1 + k]; 0 when some block's tiles were fully sorted).
// One workgroup.
__global__ __launch_bounds__(256) void k_min_shift(const u32* fine, int p, u32* bsh) {
    __shared__ u32 red[4];
    u32 m = 0xFFFFFFFFu;
    for (int k = threadIdx.x; k < p; k += 256) m = min(m, fine[k]);
    for (int o = 32; o >= 1; o >>= 1) m = min(m, (u32)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *bsh = min(min(red[0], red[1]), min(red[2], red[3]));
}

// Counts under a block shift D = *bsh (cntT as k_count), on blocks sorted on
// key >> D only. One thread per (splitter i, block k). Records at or below a
// splitter and records above it mix only inside the group of records whose
// key >> D equals the splitter's. The thread of the first splitter with that
// high part sorts the group in place, stably by key with its payloads (2 ..
// TRUNC_L records; a longer group is exactly sorted already), then counts for
// every splitter sharing the group, by bisection from the group's start:
// "record <= splitter" by key then position is monotone along the fixed block.
// Other threads only compare high parts inside a group being sorted, which
// every record of it shares. With D = 0 every thread bisects for its own
// splitter, unless only_shift is set (then k_count_staged has counted).
template <typename K, bool HASV>
__global__ void k_count_fix(K* B, u32* Bv, i64 n, int p, const K* pk, const u32* pp, const u32* bsh, int only_shift,
                            u32* cntT) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)(p + 1) * p) return;
    const int D = (int)*bsh;
    if (D == 0 && only_shift) return;
    const int i = (int)(idx / p), k = (int)(idx % p);
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    if (i == 0 || i == p) {
        cntT[idx] = i == 0 ? 0u : (u32)mk;
        return;
    }
    // records <= splitter ii in [lo, hi) of the block, the predicate true before lo and false from hi
    auto count = [&](int ii, u32 lo, u32 hi) -> u32 {
        const K sk = pk[ii - 1];
        const u32 sp = pp[ii - 1];
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (rec_le<K>(B[st + mid], (u32)(st + mid), sk, sp)) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    if (D == 0) {
        cntT[idx] = count(i, 0u, (u32)mk);
        return;
    }
    const K h = pk[i - 1] >> D;
    if (i > 1 && (pk[i - 2] >> D) == h) return;  // counted with the first splitter of the group
    u32 lo = 0, hi = (u32)mk;  // the group's first record: the first whose high part is >= h
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if ((B[st + mid] >> D) < h) lo = mid + 1; else hi = mid;
    }
    const u32 glo = lo;
    u32 g = 0;
    while (glo + g < (u32)mk && g <= (u32)TRUNC_L && (B[st + glo + g] >> D) == h) g++;
    if (g >= 2 && g <= (u32)TRUNC_L) {
        K* bk = B + st + glo;
        u32* bv = HASV ? Bv + st + glo : nullptr;
        for (u32 a = 1; a < g; a++) {
            const K x = bk[a];
            const u32 v = HASV ? bv[a] : 0u;
            u32 b = a;
            for (; b > 0 && bk[b - 1] > x; b--) {
                bk[b] = bk[b - 1];
                if (HASV) bv[b] = bv[b - 1];
            }
            bk[b] = x;
            if (HASV) bv[b] = v;
        }
    }
    // past a group of at most TRUNC_L records every high part is above h
    const u32 gend = g <= (u32)TRUNC_L ? glo + g : (u32)mk;
    for (int ii = i; ii < p && (pk[ii - 1] >> D) == h; ii++) cntT[(i64)ii * p + k] = count(ii, glo, gend);
}

// Regular sample (Figure SortD step 4): block k contributes the keys closing
// its s segments of x = ceil(ceil(n/p)/s) keys; positions past a short
// block's end are clamped to its last key. Written in position order.
template <typename K>
__global__ void k_det_sample(const K* B, i64 n, int p, int s, const u32* bsh, K* skey, u32* spos) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)p * s) return;
    const int k = (int)(idx / s), j = (int)(idx % s) + 1;
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    const i64 m = (n + p - 1) / p, x = (m + s - 1) / s;
    const i64 q = ((i64)j * x < mk ? (i64)j * x : mk) - 1;
    skey[idx] = block_key_at<K>(B, st, mk, q, bsh ? (int)*bsh : 0);
    spos[idx] = (u32)(st + q);
}

// Shift of the truncated tile sort of every block (TileArgs.gsh): the tiles
// of a multi-tile block may be sorted on the order key's high part key >> gsh
// alone, which saves the LSD passes over the low gsh bits; the block merge
// then cuts the block's runs on the high part and sorts every chunk in full,
// so the block comes out exactly sorted whatever the shift. One workgroup per
// block samples TRUNC_S of its keys, evenly spread: the shift keeps `keep`
// bits of their range, so that groups of equal high parts hold a few keys of
// the block on average. A boundary of the merge moves to the end of its group,
// so a large group makes chunks overflow LDS (such a chunk is sorted through
// global memory): a high part seen TRUNC_DUP times or more among the samples
// makes the probe try smaller shifts (a few outlying keys widen the range and
// so every group), and switches the truncation off for the block when
// TRUNC_TRIES shifts all see one. Uniform keys repeat one of the
// block's m/4 high parts that often with odds below 1e-5 at m = 2^20; a group
// of 1/64 of the block is seen 16 times on average. The samples are counted in
// an LDS table of TRUNC_E 2-bit counters indexed by a multiplicative hash of
// the high part (Fibonacci hashing), whatever the range: distinct high parts
// share a counter only by collision, and four samples of four distinct high
// parts land on one counter with odds about C(1024, 4) / TRUNC_E^3 = 2.5e-6.
// A counter that reads 3 before its increment is the fourth hit (TRUNC_DUP);
// it carries into its neighbour only at the fifth, after the flag is set.
//
// That fine shift d (groups of about 4 keys of the block) is what the block
// shift needs (gsh[p + 1 + k]; k_min_shift takes their least into gsh[p]).
// The tiles themselves may be sorted on a coarser part: the block merge's
// chunk sort ranks every bit below it anyway, and its boundaries only need
// groups well inside a chunk. The tile shift gsh[k] keeps TRUNC_KEEPC bits of
// the range when that is fewer than `keep` (groups of m / 2^12 keys, 256 at
// m = 2^20: two 6-bit passes instead of three), unless a coarse group is seen
// TRUNC_DUPC times among the samples (a group of 6/1024 of the block on
// average; 4-bit counters, 2^TRUNC_LGC of them, hashed alike), and else is d.
constexpr int TRUNC_NT = 256, TRUNC_PER = 4, TRUNC_S = TRUNC_NT * TRUNC_PER, TRUNC_DUP = 4;
constexpr int TRUNC_LGE = 18, TRUNC_E = 1 << TRUNC_LGE;  // 2^18 counters, 64 KiB of LDS
constexpr int TRUNC_TRIES = 4;
constexpr int TRUNC_KEEPC = 12, TRUNC_DUPC = 6, TRUNC_LGC = 16;
static_assert(TRUNC_DUP == 4, "a 2-bit counter tells the fourth hit");
static_assert((1 << TRUNC_LGC) / 8 <= TRUNC_E / 16, "the coarse counters reuse the fine table");

template <typename K>
__global__ __launch_bounds__(TRUNC_NT) void k_trunc_probe(const K* in, int dt, i64 n, int p, int keep, u32* gsh) {
    __shared__ u32 tab[TRUNC_E / 16];
    __shared__ u64 red[TRUNC_NT / 64 * 2];
    __shared__ u32 dup;
    const int t = threadIdx.x, k = blockIdx.x;
    const i64 st = blk_start(n, p, k), m = blk_start(n, p, k + 1) - st;
    K u[TRUNC_PER];
    K mn = KeyMax<K>::v, mx = 0;
#pragma unroll
    for (int j = 0; j < TRUNC_PER; j++) {
        const i64 idx = st + (i64)(((u64)(t * TRUNC_PER + j) * (u64)m) / (u64)TRUNC_S);
        u[j] = m > 0 ? okey<K>(in[idx], dt) : (K)0;
        mn = u[j] < mn ? u[j] : mn;
        mx = u[j] > mx ? u[j] : mx;
    }
    block_minmax<TRUNC_NT, K>(mn, mx, red);
    const int bits = bitwidth64((u64)(mx - mn));
    const int d0 = bits > keep ? bits - keep : 0;
    // A few outlying keys widen the range and so the groups; when a group is
    // seen too often, smaller shifts are tried (TRUNC_TRIES in all).
    int d = d0;
    for (; d > 0 && d > d0 - TRUNC_TRIES; d--) {
        for (int i = t; i < TRUNC_E / 16; i += TRUNC_NT) tab[i] = 0u;
        if (t == 0) dup = 0u;
        __syncthreads();
        u32 hit = 0;
#pragma unroll
        for (int j = 0; j < TRUNC_PER; j++) {
            const u32 e = (u32)(((u64)(u[j] >> d) * 0x9E3779B97F4A7C15ull) >> (64 - TRUNC_LGE));
            const u32 sh = (e & 15u) * 2u;
            const u32 old = atomicAdd(&tab[e >> 4], 1u << sh);
            hit |= ((old >> sh) & 3u) == 3u ? 1u : 0u;
        }
        if (hit) dup = 1u;
        __syncthreads();
        const bool clean = dup == 0u;
        __syncthreads();  // every thread has read dup before the next try clears it
        if (clean) break;
    }
    const int dk = (d > 0 && d > d0 - TRUNC_TRIES) ? d : 0;
    int dc = dk;
    const int c = bits - TRUNC_KEEPC;
    if (dk > 0 && c > dk) {
        for (int i = t; i < (1 << TRUNC_LGC) / 8; i += TRUNC_NT) tab[i] = 0u;
        if (t == 0) dup = 0u;
        __syncthreads();
        u32 hit = 0;
#pragma unroll
        for (int j = 0; j < TRUNC_PER; j++) {
            const u32 e = (u32)(((u64)(u[j] >> c) * 0x9E3779B97F4A7C15ull) >> (64 - TRUNC_LGC));
            const u32 sh = (e & 7u) * 4u;
            const u32 old = atomicAdd(&tab[e >> 3], 1u << sh);
            hit |= ((old >> sh) & 15u) + 1u >= (u32)TRUNC_DUPC ? 1u : 0u;
        }
        if (hit) dup = 1u;
        __syncthreads();
        if (dup == 0u) dc = c;
    }
    if (t == 0) {
        gsh[k] = (u32)dc;
        gsh[p + 1 + k] = (u32)dk;
    }
}

// Random sample (Figure SortRI step 4): s*p - 1 distinct positions of the
// block-sorted array, the images of 0 .. s*p-2 under the keyed permutation.
__global__ void k_ran_positions(u64 seed, i64 n, i64 ns, u32* pos) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    pos[t] = (u32)feistel_perm(seed, (u64)n, (u64)t);
}

template <typename K>
__global__ void k_gather_sample(const K* B, i64 n, int p, const u32* bsh, const u32* pos, i64 ns, K* skey) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    const i64 q = pos[t];
    const int D = bsh ? (int)*bsh : 0;
    if (D == 0) {
        skey[t] = B[q];
        return;
    }
    // the block holding q: the largest k with floor(k n / p) <= q
    const int k = (int)(((u64)(q + 1) * (u64)p + (u64)n - 1) / (u64)n) - 1;
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    skey[t] = block_key_at<K>(B, st, mk, q - st, D);
}

// Splitters: sorted sample records at 1-based ranks s, 2s, ..., (p-1)s.
template <typename K>
__global__ void k_splitters(const K* skey, const u32* spos, int p, int s, K* pk, u32* pp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (i >= p) return;
    pk[i - 1] = skey[(i64)i * s - 1];
    pp[i - 1] = spos[(i64)i * s - 1];
}

// cntT[i*p + k] = keys of block k whose record is <= splitter i (i = 1..p-1);
// row 0 is 0 and row p is the block size. The bucket of a record is the
// number of splitters strictly below it, so bucket i of block k is
// [cntT[i][k], cntT[i+1][k]) within the sorted block.
template <typename K>
__global__ void k_count(const K* B, i64 n, int p, const K* pk, const u32* pp, u32* cntT) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)(p + 1) * p) return;
    const int i = (int)(idx / p), k = (int)(idx % p);
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    u32 res;
    if (i == 0) res = 0;
    else if (i == p) res = (u32)mk;
    else {
        const K sk = pk[i - 1];
        const u32 sp = pp[i - 1];
        u32 lo = 0, hi = (u32)mk;
        while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (rec_le<K>(B[st + mid], (u32)(st + mid), sk, sp)) lo = mid + 1; else hi = mid;
        }
        res = lo;
    }
    cntT[idx] = res;
}

// The same counts with one workgroup per block: the block's samples (every
// ys-th key, at block positions (j+1)*ys - 1; floor(mk/ys) of them) are staged
// in LDS and each splitter is bisected there, so only the last bisection,
// inside one sample stride, reads the block in global memory. For blocks of
// at most COUNT_SMAX samples. Under a block shift (bsh != NULL and *bsh > 0)
// it does nothing: k_count_fix counts.
constexpr int COUNT_NT = 256, COUNT_SMAX = 8192;

template <typename K>
__global__ __launch_bounds__(COUNT_NT) void k_count_staged(const K* B, i64 n, int p, const K* pk, const u32* pp,
                                                           const K* bsmp, u32 spb, u32 ys, const u32* bsh,
                                                           u32* cntT) {
    __shared__ K ls[COUNT_SMAX];
    const int k = blockIdx.x, t = threadIdx.x;
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    if (bsh && *bsh > 0u) return;
    const u32 ns = min((u32)(mk / ys), spb);
    for (u32 j = t; j < ns; j += COUNT_NT) ls[j] = bsmp[(i64)k * spb + j];
    __syncthreads();
    for (int i = t; i <= p; i += COUNT_NT) {
        u32 res;
        if (i == 0) res = 0;
        else if (i == p) res = (u32)mk;
        else {
            const K sk = pk[i - 1];
            const u32 sp = pp[i - 1];
            u32 lo = 0, hi = ns;  // samples <= the splitter
            while (lo < hi) {
                const u32 mid = (lo + hi) >> 1;
                if (rec_le<K>(ls[mid], (u32)(st + (u64)(mid + 1) * ys - 1), sk, sp)) lo = mid + 1; else hi = mid;
            }
            u32 wlo = lo * ys, whi = lo < ns ? (lo + 1) * ys - 1 : (u32)mk;
            while (wlo < whi) {
                const u32 mid = (wlo + whi) >> 1;
                if (rec_le<K>(B[st + mid], (u32)(st + mid), sk, sp)) wlo = mid + 1; else whi = mid;
            }
            res = wlo;
        }
        cntT[(i64)i * p + k] = res;
    }
}

// Bucket merge tables: group = bucket i, run = block k. One workgroup per
// bucket. out_base[i] = sum_k cntT[i][k] (keys in smaller buckets). Samples of
// the runs are the block samples every yb-th key that fall inside the run.
// When off != NULL the runs are read from the routed array instead, where run
// (k, i) starts at off[k*p + i].
__global__ __launch_bounds__(256) void k_bucket_tables(i64 n, int p, const u32* cntT, u32 yb, u32 spb,
                                                       const u32* off, u32* run_start, u32* run_len,
                                                       u32* out_base, u32* sdesc) {
    __shared__ u32 red[4];
    const int i = blockIdx.x, t = threadIdx.x;
    u32 acc = 0;
    for (int k = t; k < p; k += 256) {
        const i64 st = blk_start(n, p, k);
        const u32 a0 = cntT[(i64)i * p + k], a1 = cntT[(i64)(i + 1) * p + k];
        acc += a0;
        const u32 rs = (u32)st + a0, re = (u32)st + a1;
        const u32 jlo = a0 / yb, jhi = a1 / yb;
        const u32 shift = off ? off[(i64)k * p + i] - rs : 0u;
        run_start[(i64)i * p + k] = rs + shift;
        run_len[(i64)i * p + k] = a1 - a0;
        u32* d = sdesc + ((i64)i * p + k) * 4;
        d[0] = (u32)k * spb + jlo;
        d[1] = jhi - jlo;
        d[2] = (u32)st + (jlo + 1) * yb - 1 + shift;
        d[3] = yb;
        (void)re;
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) out_base[i] = red[0] + red[1] + red[2] + red[3];
}

// p == 1, or a final copy: order keys -> raw keys.
template <typename K>
__global__ void k_copy_out(const K* src, const u32* srcv, K* dst, u32* dstv, i64 n, int out_dt) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = rawkey<K>(src[i], out_dt);
    if (srcv) dstv[i] = srcv[i];
}

// ======================================================================= scatter routing

// From the count matrix C (row = block k, column = bucket i) to the
// boundaries used by the merge tables: cntT[i*p + k] = keys of block k in
// buckets below i (row p = block size). One workgroup per block.
__global__ __launch_bounds__(256) void k_counts_to_cntT(const u32* C, int p, u32* cntT) {
    __shared__ u32 wsum[8];
    const int k = blockIdx.x, t = threadIdx.x;
    const int per = (p + 255) / 256;
    u32 loc = 0;
    for (int i = t * per; i < (t + 1) * per && i < p; i++) loc += C[(i64)k * p + i];
    u32 tot;
    u32 ex = block_excl_scan<256>(loc, tot, wsum);
    for (int i = t * per; i < (t + 1) * per && i < p; i++) {
        cntT[(i64)i * p + k] = ex;
        ex += C[(i64)k * p + i];
    }
    if (t == 0) cntT[(i64)p * p + k] = tot;
}

// Routing offsets (the p independent prefix computations): bucket i starts
// after all smaller buckets, and within it the keys of block k follow those of
// blocks 0..k-1: off[k*p + i]. One workgroup per bucket.
__global__ __launch_bounds__(256) void k_route_offsets(const u32* C, const u32* cntT, int p, u32* off) {
    __shared__ u32 wsum[8];
    const int i = blockIdx.x, t = threadIdx.x;
    const int per = (p + 255) / 256;
    u32 loc = 0, lb = 0;
    for (int k = t * per; k < (t + 1) * per && k < p; k++) {
        loc += C[(i64)k * p + i];
        lb += cntT[(i64)i * p + k];
    }
    u32 tot, base;
    u32 ex = block_excl_scan<256>(loc, tot, wsum);
    __syncthreads();
    (void)block_excl_scan<256>(lb, base, wsum);
    for (int k = t * per; k < (t + 1) * per && k < p; k++) {
        off[(i64)k * p + i] = base + ex;
        ex += C[(i64)k * p + i];
    }
}

// Routing (Figure SortD steps 10-11): run (k, b), the keys of sorted block k
// that fall in bucket b (contiguous, since the block is sorted), moves to
// off[k*p + b] with its order kept. Each workgroup takes a share of one block:
// the block's run starts (the prefix of its count row) and destinations are
// staged in LDS, every key finds its run by a branch-free bisection there, and
// keys are read and written position-striped (coalesced within a run).
constexpr int SCAT_NT = 256, SCAT_IT = 16;

template <typename K, bool HASV>
__global__ __launch_bounds__(SCAT_NT) void k_scatter(const K* B, const u32* Bv, i64 n, int p, int wpb, const u32* C,
                                                     const u32* off, K* Z, u32* Zv) {
    constexpr int NT = SCAT_NT, TILE = SCAT_NT * SCAT_IT;
    __shared__ u32 rs[MAXR + 1], od[MAXR];
    __shared__ u32 wsum[NT / 64 + 2];
    const int k = blockIdx.x / wpb, w = blockIdx.x % wpb, t = threadIdx.x;
    const i64 st = blk_start(n, p, k), m = blk_start(n, p, k + 1) - st;
    const u32* crow = C + (i64)k * p;
    const int per = (p + NT - 1) / NT;
    u32 loc = 0;
    for (int b = t * per; b < (t + 1) * per && b < p; b++) loc += crow[b];
    u32 tot;
    u32 ex = block_excl_scan<NT>(loc, tot, wsum);
    for (int b = t * per; b < (t + 1) * per && b < p; b++) {
        rs[b] = ex;
        od[b] = off[(i64)k * p + b];
        ex += crow[b];
    }
    if (t == 0) rs[p] = tot;
    __syncthreads();
    int top = 1;  // largest power of two <= p - 1 (bisection steps)
    while (top * 2 <= p - 1) top *= 2;
    const i64 lo = m * w / wpb, hi = m * (w + 1) / wpb;
    for (i64 c0 = lo; c0 < hi; c0 += TILE) {
#pragma unroll
        for (int j = 0; j < SCAT_IT; j++) {
            const i64 c = c0 + j * NT + t;
            if (c < hi) {
                // run of position c: the largest b with rs[b] <= c
                int b = 0;
                for (int step = top; step > 0; step >>= 1)
                    if (b + step < p && rs[b + step] <= (u32)c) b += step;
                const u32 dst = od[b] + (u32)c - rs[b];
                Z[dst] = B[st + c];
                if (HASV) Zv[dst] = Bv[st + c];
            }
        }
    }
}
