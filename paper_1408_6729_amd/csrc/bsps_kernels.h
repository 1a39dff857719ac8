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

constexpr int MAXR = 4096;  // runs per merge group (tiles per block, or p)

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
    u32* slot_group;       // [S]
    u32* grp_base;         // [G]
    u32* grp_nb;           // [G] boundaries of the group (chunks = nb + 1 when non-empty)
    K* bkey;               // [S] boundary records
    u32* bpos;
    u32* cuts;             // [S*R]
    u32 S;                 // slot capacity
    int out_dt;            // BSPS_DT_NONE: keep order keys; else write raw keys of this dtype
    K* osmp;               // output samples every oys-th key of each group (or NULL)
    u32 oys, ospb;
};

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

// ======================================================================= tile sort

template <typename K, bool HASV>
__global__ __launch_bounds__(Shape<K>::NT) void k_tile_sort(TileArgs<K> a) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT;
    __shared__ SortSmem<NT> sm;
    __shared__ K exch[T + T / 32];
    const int t = threadIdx.x;
    const int k = blockIdx.x / a.tpb, tt = blockIdx.x % a.tpb;
    const i64 st = blk_start(a.n, a.p, k), en = blk_start(a.n, a.p, k + 1);
    const i64 base = st + (i64)tt * T;
    i64 cnt64 = en - base;
    const int cnt = cnt64 <= 0 ? 0 : (cnt64 > T ? T : (int)cnt64);
    if (cnt == 0) return;
    K mn = KeyMax<K>::v, mx = 0;
    for (int i = t; i < cnt; i += NT) {
        K u = okey<K>(a.in[base + i], a.in_dt);
        exch[padi(i)] = u;
        mn = u < mn ? u : mn;
        mx = u > mx ? u : mx;
    }
    block_minmax<NT, K>(mn, mx, sm.red64);  // includes barriers
    const int nbits = bitwidth64((u64)(mx - mn));
    u32 v[IT], rank[IT];
    u32* vex = reinterpret_cast<u32*>(exch);
    const bool wide = sizeof(K) == 8 && nbits > 32;
    if (wide) {
        u64 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int i = t * IT + j;
            sk[j] = i < cnt ? (u64)(exch[padi(i)] - mn) : (u64)(mx - mn);
        }
        __syncthreads();
        if (HASV) {
            for (int i = t; i < cnt; i += NT) vex[padi(i)] = a.inv[base + i];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = vex[padi(t * IT + j)];
            __syncthreads();
        }
        wg_sort_regs<NT, IT, u64, HASV>(sk, v, rank, nbits, reinterpret_cast<u64*>(exch), sm);
        u64* ex = reinterpret_cast<u64*>(exch);
        for (int i = t; i < cnt; i += NT) {
            K u = (K)(ex[padi(i)] + (u64)mn);
            a.out[base + i] = rawkey<K>(u, a.out_dt);
            if (a.smp && ((i + 1) % a.ys) == 0) a.smp[(i64)blockIdx.x * a.spt + (i + 1) / a.ys - 1] = u;
        }
    } else {
        u32 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int i = t * IT + j;
            sk[j] = i < cnt ? (u32)(exch[padi(i)] - mn) : (u32)(mx - mn);
        }
        __syncthreads();
        if (HASV) {
            for (int i = t; i < cnt; i += NT) vex[padi(i)] = a.inv[base + i];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = vex[padi(t * IT + j)];
            __syncthreads();
        }
        wg_sort_regs<NT, IT, u32, HASV>(sk, v, rank, nbits, vex, sm);
        for (int i = t; i < cnt; i += NT) {
            K u = (K)vex[padi(i)] + mn;
            a.out[base + i] = rawkey<K>(u, a.out_dt);
            if (a.smp && ((i + 1) % a.ys) == 0) a.smp[(i64)blockIdx.x * a.spt + (i + 1) / a.ys - 1] = u;
        }
    }
    if (HASV) {
        wg_scatter_vals<NT, IT>(v, rank, vex);
        for (int i = t; i < cnt; i += NT) a.outv[base + i] = vex[padi(i)];
    }
}

// ======================================================================= MWM: pick boundaries

// One workgroup per group: sort (a regular subsample of) the group's samples
// and keep every q-th as a chunk boundary.
template <typename K>
__global__ __launch_bounds__(Shape<K>::NT) void k_mwm_pick(MwmArgs<K> a) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT;
    __shared__ SortSmem<NT> sm;
    __shared__ K exch[T + T / 32];
    __shared__ u32 spre[MAXR + 1];
    __shared__ u32 sh_nb, sh_base;
    const int t = threadIdx.x, g = blockIdx.x, R = a.R;
    // prefix of the runs' sample counts, and the group size
    u32 locS = 0, locN = 0;
    for (int r = t; r < R; r += NT) {
        locS += a.sdesc[((i64)g * R + r) * 4 + 1];
        locN += a.run_len[(i64)g * R + r];
    }
    // chunked exclusive scan of sample counts in run order: thread t handles runs t*RPT..
    const int RPT = (R + NT - 1) / NT;
    u32 mys = 0;
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) mys += a.sdesc[((i64)g * R + r) * 4 + 1];
    u32 totS;
    u32 ex = block_excl_scan<NT>(mys, totS, sm.wsum);
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
        spre[r] = ex;
        ex += a.sdesc[((i64)g * R + r) * 4 + 1];
    }
    if (t == 0) spre[R] = totS;
    u32 totN;
    __syncthreads();
    (void)block_excl_scan<NT>(locN, totN, sm.wsum);
    (void)locS;
    const u32 Sraw = totS, N = totN;
    u32 nb = 0, f = 1, Sg = 0, q = 1;
    if (N > a.cap && Sraw > 0) {
        f = (Sraw + T - 1) / T;
        Sg = Sraw / f;
        u64 qq = ((u64)a.tavg * Sg + N - 1) / N;
        q = qq < 1 ? 1u : (u32)qq;
        nb = Sg / q;
    }
    if (t == 0) {
        u32 slots = N > 0 ? nb + 1 : 0;
        u32 b = slots ? atomicAdd(a.slot_count, slots) : 0u;
        if (b + slots > a.S) { slots = 0; nb = 0; b = a.S; }  // cannot happen: slot bound n/tavg + G
        sh_base = b;
        sh_nb = slots ? nb : 0u;
        a.grp_base[g] = b;
        a.grp_nb[g] = slots ? nb : 0u;
    }
    __syncthreads();
    const u32 gb = sh_base;
    nb = sh_nb;
    if (N == 0 || gb >= a.S) return;
    for (u32 i = t; i <= nb; i += NT) a.slot_group[gb + i] = g;
    if (nb == 0) return;
    // load the subsample: element i is concatenated sample index (i+1)*f - 1
    K mn = KeyMax<K>::v, mx = 0;
    u32 v[IT], rank[IT];
    K key[IT];
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const u32 i = (u32)(t * IT + j);
        v[j] = 0;
        key[j] = 0;
        if (i < Sg) {
            const u32 c = (i + 1) * f - 1;
            int lo = 0, hi = R;  // largest r with spre[r] <= c
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (spre[mid] <= c) lo = mid; else hi = mid;
            }
            const u32 si = a.sdesc[((i64)g * R + lo) * 4 + 0] + (c - spre[lo]);
            key[j] = a.smp[si];
            v[j] = c;
            mn = key[j] < mn ? key[j] : mn;
            mx = key[j] > mx ? key[j] : mx;
        }
    }
    block_minmax<NT, K>(mn, mx, sm.red64);
    const int nbits = bitwidth64((u64)(mx - mn));
    u32* vex = reinterpret_cast<u32*>(exch);
    if (sizeof(K) == 8 && nbits > 32) {
        u64 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = (u32)(t * IT + j) < Sg ? (u64)(key[j] - mn) : (u64)(mx - mn);
        wg_sort_regs<NT, IT, u64, true>(sk, v, rank, nbits, reinterpret_cast<u64*>(exch), sm);
        // keep the boundary keys in registers of the threads that own them
        u64* e = reinterpret_cast<u64*>(exch);
#pragma unroll
        for (int j = 0; j < IT; j++) key[j] = (K)(e[padi(t * IT + j)] + (u64)mn);
    } else {
        u32 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = (u32)(t * IT + j) < Sg ? (u32)(key[j] - mn) : (u32)(mx - mn);
        wg_sort_regs<NT, IT, u32, true>(sk, v, rank, nbits, vex, sm);
#pragma unroll
        for (int j = 0; j < IT; j++) key[j] = (K)vex[padi(t * IT + j)] + mn;
    }
    wg_scatter_vals<NT, IT>(v, rank, vex);
    // boundary b (1..nb) = sorted element b*q - 1
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const u32 i = (u32)(t * IT + j);
        if (i < Sg && (i + 1) % q == 0 && (i + 1) / q <= nb) {
            const u32 b = (i + 1) / q;
            const u32 c = vex[padi((int)i)];
            int lo = 0, hi = R;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (spre[mid] <= c) lo = mid; else hi = mid;
            }
            const u32* d = a.sdesc + ((i64)g * R + lo) * 4;
            a.bkey[gb + b - 1] = key[j];
            a.bpos[gb + b - 1] = d[2] + (c - spre[lo]) * d[3];
        }
    }
}

// ======================================================================= MWM: exact cuts

// cuts[slot*R + r] = number of records of run r that are <= the boundary record
// of that slot (key first, then position).
template <typename K>
__global__ void k_mwm_cuts(MwmArgs<K> a) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const u32 slot = (u32)(idx / a.R);
    const int r = (int)(idx % a.R);
    if (slot >= *a.slot_count || slot >= a.S) return;
    const u32 g = a.slot_group[slot];
    const u32 c = slot - a.grp_base[g];
    if (c >= a.grp_nb[g]) return;
    const K bk = a.bkey[slot];
    const u32 bp = a.bpos[slot];
    const u32 rs = a.run_start[(i64)g * a.R + r];
    u32 lo = 0, hi = a.run_len[(i64)g * a.R + r];
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (rec_le<K>(a.src[rs + mid], rs + mid, bk, bp)) lo = mid + 1; else hi = mid;
    }
    a.cuts[(i64)slot * a.R + r] = lo;
}

// ======================================================================= MWM: chunk sort

template <typename K, bool HASV>
__device__ void mwm_emit(const MwmArgs<K>& a, u32 g, u32 o, K u, u32 gstart) {
    if (a.osmp) {
        const u32 rel = o - gstart + 1;
        if (rel % a.oys == 0) a.osmp[(i64)g * a.ospb + rel / a.oys - 1] = u;
    }
}

// Oversize chunk: LSD radix passes through global memory by one workgroup.
// Pieces are first copied (in run order) to scr[out .. out+N), then sorted by
// digit passes alternating scr <-> dst; the last step writes dst.
template <typename K, bool HASV>
__device__ void mwm_oversize(const MwmArgs<K>& a, u32 g, u32 slot, u32 c, u32 nb, const u32* ppre, u32 N,
                             u32 out, SortSmem<Shape<K>::NT>& sm, K* exch) {
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
        if (t < 64) {
            u32 hv = hist[t];
            u32 inc = wave_incl_scan(hv);
            doff[t] = inc - hv;
        }
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
            if (t < 64) {
                u32 hv = tcnt[t];
                u32 inc = wave_incl_scan(hv);
                tbase[t] = inc - hv;
            }
            radix_rank<NT, IT>(dig, rank, sm);  // begins with a barrier-protected reset
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

template <typename K, bool HASV>
__global__ __launch_bounds__(Shape<K>::NT) void k_mwm_merge(MwmArgs<K> a) {
    constexpr int NT = Shape<K>::NT, IT = Shape<K>::IT, T = NT * IT;
    __shared__ SortSmem<NT> sm;
    __shared__ K exch[T + T / 32];
    __shared__ u32 ppre[MAXR + 1];
    const int t = threadIdx.x, R = a.R;
    const u32 slot = blockIdx.x;
    if (slot >= *a.slot_count || slot >= a.S) return;
    const u32 g = a.slot_group[slot];
    const u32 c = slot - a.grp_base[g];
    const u32 nb = a.grp_nb[g];
    // piece lengths and their prefix (runs in order)
    const int RPT = (R + NT - 1) / NT;
    u32 mysum = 0, mylo = 0;
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
        const u32 lo = c == 0 ? 0u : a.cuts[(i64)(slot - 1) * R + r];
        const u32 hi = c == nb ? a.run_len[(i64)g * R + r] : a.cuts[(i64)slot * R + r];
        mysum += hi - lo;
        mylo += lo;
    }
    u32 N;
    u32 ex = block_excl_scan<NT>(mysum, N, sm.wsum);
    for (int r = t * RPT; r < (t + 1) * RPT && r < R; r++) {
        const u32 lo = c == 0 ? 0u : a.cuts[(i64)(slot - 1) * R + r];
        const u32 hi = c == nb ? a.run_len[(i64)g * R + r] : a.cuts[(i64)slot * R + r];
        ppre[r] = ex;
        ex += hi - lo;
    }
    if (t == 0) ppre[R] = N;
    u32 LO;
    __syncthreads();
    (void)block_excl_scan<NT>(mylo, LO, sm.wsum);
    const u32 out = a.out_base[g] + LO;
    if (N == 0) return;
    if (N > a.cap) {
        if (t == 0) atomicAdd(a.oversize, 1u);
        mwm_oversize<K, HASV>(a, g, slot, c, nb, ppre, N, out, sm, exch);
        return;
    }
    // gather pieces into LDS in run order (one wave per piece)
    const int lane = t & 63, w = t >> 6, NW = NT / 64;
    K mn = KeyMax<K>::v, mx = 0;
    for (int r = w; r < R; r += NW) {
        const u32 lo = c == 0 ? 0u : a.cuts[(i64)(slot - 1) * R + r];
        const u32 len = ppre[r + 1] - ppre[r];
        const K* s = a.src + a.run_start[(i64)g * R + r] + lo;
        const u32 o = ppre[r];
        for (u32 i = lane; i < len; i += 64) {
            K u = s[i];
            exch[padi((int)(o + i))] = u;
            mn = u < mn ? u : mn;
            mx = u > mx ? u : mx;
        }
    }
    block_minmax<NT, K>(mn, mx, sm.red64);
    const int nbits = bitwidth64((u64)(mx - mn));
    u32 v[IT], rank[IT];
    u32* vex = reinterpret_cast<u32*>(exch);
    const u32 gstart = a.out_base[g];
    auto load_vals = [&]() {
        for (int r = w; r < R; r += NW) {
            const u32 lo = c == 0 ? 0u : a.cuts[(i64)(slot - 1) * R + r];
            const u32 len = ppre[r + 1] - ppre[r];
            const u32* s = a.srcv + a.run_start[(i64)g * R + r] + lo;
            const u32 o = ppre[r];
            for (u32 i = lane; i < len; i += 64) vex[padi((int)(o + i))] = s[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IT; j++) v[j] = vex[padi(t * IT + j)];
        __syncthreads();
    };
    if (sizeof(K) == 8 && nbits > 32) {
        u64 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(t * IT + j);
            sk[j] = i < N ? (u64)(exch[padi((int)i)] - mn) : (u64)(mx - mn);
        }
        __syncthreads();
        if (HASV) load_vals();
        wg_sort_regs<NT, IT, u64, HASV>(sk, v, rank, nbits, reinterpret_cast<u64*>(exch), sm);
        u64* e = reinterpret_cast<u64*>(exch);
        for (u32 i = t; i < N; i += NT) {
            K u = (K)(e[padi((int)i)] + (u64)mn);
            a.dst[out + i] = rawkey<K>(u, a.out_dt);
            mwm_emit<K, HASV>(a, g, out + i, u, gstart);
        }
    } else {
        u32 sk[IT];
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const u32 i = (u32)(t * IT + j);
            sk[j] = i < N ? (u32)(exch[padi((int)i)] - mn) : (u32)(mx - mn);
        }
        __syncthreads();
        if (HASV) load_vals();
        wg_sort_regs<NT, IT, u32, HASV>(sk, v, rank, nbits, vex, sm);
        for (u32 i = t; i < N; i += NT) {
            K u = (K)vex[padi((int)i)] + mn;
            a.dst[out + i] = rawkey<K>(u, a.out_dt);
            mwm_emit<K, HASV>(a, g, out + i, u, gstart);
        }
    }
    if (HASV) {
        wg_scatter_vals<NT, IT>(v, rank, vex);
        for (u32 i = t; i < N; i += NT) a.dstv[out + i] = vex[padi((int)i)];
    }
}

// ======================================================================= sample and splitters

// Regular sample (Figure SortD step 4): block k contributes the keys closing
// its s segments of x = ceil(ceil(n/p)/s) keys; positions past a short
// block's end are clamped to its last key. Written in position order.
template <typename K>
__global__ void k_det_sample(const K* B, i64 n, int p, int s, K* skey, u32* spos) {
    const i64 idx = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (i64)p * s) return;
    const int k = (int)(idx / s), j = (int)(idx % s) + 1;
    const i64 st = blk_start(n, p, k), mk = blk_start(n, p, k + 1) - st;
    const i64 m = (n + p - 1) / p, x = (m + s - 1) / s;
    const i64 q = ((i64)j * x < mk ? (i64)j * x : mk) - 1;
    skey[idx] = B[st + q];
    spos[idx] = (u32)(st + q);
}

// Random sample (Figure SortRI step 4): s*p - 1 distinct positions of the
// block-sorted array, the images of 0 .. s*p-2 under the keyed permutation.
__global__ void k_ran_positions(u64 seed, i64 n, i64 ns, u32* pos) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    pos[t] = (u32)feistel_perm(seed, (u64)n, (u64)t);
}

template <typename K>
__global__ void k_gather_sample(const K* B, const u32* pos, i64 ns, K* skey) {
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    skey[t] = B[pos[t]];
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
