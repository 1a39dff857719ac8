// bsps_device.h -- device building blocks for gfx950 (wave64, 160 KB LDS per CU).
//
// Keys are carried as unsigned "order keys" whose unsigned order is the key
// order (int: sign bit flipped; float32: IEEE-754 totalOrder of the bits).
// The workgroup sort below is a stable LSD radix sort held in registers and
// LDS: each thread owns IT consecutive tile positions ("blocked" order), ranks
// its items with private per-digit counters in LDS (two 16-bit counters per
// 32-bit word), and a raking scan over the counters in (digit, thread) order
// turns local counts into stable ranks. Only the bits in which the tile's
// keys differ are sorted: keys are rebased to (key - min) first.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;

#define BSPS_DT_I32 0
#define BSPS_DT_I64 1
#define BSPS_DT_F32 2
#define BSPS_DT_NONE (-1)  // input is already in order-key form

// ---------------------------------------------------------------- key maps

__device__ __forceinline__ u32 okey32(u32 raw, int dt) {
    if (dt == BSPS_DT_F32) return (raw & 0x80000000u) ? ~raw : (raw | 0x80000000u);
    if (dt == BSPS_DT_NONE) return raw;
    return raw ^ 0x80000000u;
}
__device__ __forceinline__ u32 rawkey32(u32 u, int dt) {
    if (dt == BSPS_DT_F32) return (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    if (dt == BSPS_DT_NONE) return u;
    return u ^ 0x80000000u;
}
__device__ __forceinline__ u64 okey64(u64 raw, int dt) {
    return dt == BSPS_DT_NONE ? raw : (raw ^ 0x8000000000000000ull);
}
__device__ __forceinline__ u64 rawkey64(u64 u, int dt) {
    return dt == BSPS_DT_NONE ? u : (u ^ 0x8000000000000000ull);
}
template <typename K> __device__ __forceinline__ K okey(K raw, int dt);
template <> __device__ __forceinline__ u32 okey<u32>(u32 raw, int dt) { return okey32(raw, dt); }
template <> __device__ __forceinline__ u64 okey<u64>(u64 raw, int dt) { return okey64(raw, dt); }
template <typename K> __device__ __forceinline__ K rawkey(K u, int dt);
template <> __device__ __forceinline__ u32 rawkey<u32>(u32 u, int dt) { return rawkey32(u, dt); }
template <> __device__ __forceinline__ u64 rawkey<u64>(u64 u, int dt) { return rawkey64(u, dt); }

template <typename K> struct KeyMax;
template <> struct KeyMax<u32> { static constexpr u32 v = 0xffffffffu; };
template <> struct KeyMax<u64> { static constexpr u64 v = 0xffffffffffffffffull; };

// Record order of the duplicate handling: key first, then the position tag.
template <typename K>
__device__ __forceinline__ bool rec_le(K k, u32 pos, K bk, u32 bpos) {
    return k < bk || (k == bk && pos <= bpos);
}
template <typename K>
__device__ __forceinline__ bool rec_lt(K k, u32 pos, K bk, u32 bpos) {
    return k < bk || (k == bk && pos < bpos);
}

__device__ __forceinline__ int bitwidth64(u64 v) { return v ? 64 - __clzll((long long)v) : 0; }

// ---------------------------------------------------------------- tile geometry

// Workgroup sort shapes: 4-byte keys use 512 threads x 32 items (16K keys),
// 8-byte keys 512 threads x 16 items (8K keys: half the items per thread keep
// the 64-bit keys, ranks and payloads in registers without spilling).
template <typename K> struct Shape;
#ifndef BSPS_NT32
#define BSPS_NT32 512
#endif
#ifndef BSPS_IT32
#define BSPS_IT32 32
#endif
template <> struct Shape<u32> { static constexpr int NT = BSPS_NT32, IT = BSPS_IT32; };
#ifndef BSPS_NT64
#define BSPS_NT64 512
#endif
#ifndef BSPS_IT64
#define BSPS_IT64 16
#endif
template <> struct Shape<u64> { static constexpr int NT = BSPS_NT64, IT = BSPS_IT64; };

#ifndef BSPS_DIG_RECOMPUTE
#define BSPS_DIG_RECOMPUTE 1  // recompute digits instead of keeping them in registers
#endif
#ifndef BSPS_WG_PER_CU
#define BSPS_WG_PER_CU 2      // occupancy target of the sorting kernels: minimum waves per SIMD (launch bound)
#endif

#ifndef BSPS_RB
#define BSPS_RB 6
#endif
constexpr int RB = BSPS_RB;           // radix bits per pass
constexpr int RADIX = 1 << RB;        // digits per pass
constexpr int HALF = RADIX / 2;       // digits d and d + HALF share one 32-bit counter word
static_assert(RB >= 5 && RB <= 8, "the half of a digit is its top bit shifted right to bit 4");

__device__ __forceinline__ int padi(int i) { return i + (i >> 5); }  // one pad word per 32
// padi(j*NT + t) for 0 <= t < NT, NT a multiple of 32: a fixed offset from
// padi(t), so striped accesses need no address arithmetic per item
template <int NT> __device__ __forceinline__ int padj(int j, int t) { return j * (NT + NT / 32) + padi(t); }

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// The digit counters and the key exchange buffer are never live at the same
// time (ranking ends with a barrier before keys are scattered), so they may
// share one LDS region: `u` holds HALF*NT counter words or NT*IT exchange
// slots of KB bytes, whichever is larger, each with one pad word per 32.
// SEP gives the exchange buffer its own region (twice the LDS), which lets a
// sort pass drop three of its barriers (see wg_sort_regs).
template <int NT, int KB, int IT, bool SEP = false> struct SortSmem {
    static constexpr int CNT = HALF * NT;
    static constexpr int CNTW = CNT + CNT / 32;
    static constexpr int EXW = (NT * IT + NT * IT / 32) * KB / 4;  // IT items of KB bytes per thread, padded
    static constexpr int UW = SEP ? CNTW : (CNTW > EXW ? CNTW : EXW);
    static constexpr int XW = SEP ? EXW : 1;
    u32 u[UW];
    u32 x[XW];
    u32 wsum[NT / 64 + 2];
    u32 misc[16];
    u64 red64[NT / 64 * 2];
    __device__ __forceinline__ u32* cnt() { return u; }
    template <typename T> __device__ __forceinline__ T* ex() { return reinterpret_cast<T*>(SEP ? x : u); }
};

// ---------------------------------------------------------------- scans

// Inclusive scan over the 64 lanes of a wave by DPP lane moves, all in
// registers: shifts by 1, 2, 4 and 8 lanes within each row of 16, then the
// broadcasts of lane 15 (into rows 1 and 3) and of lane 31 (into rows 2 and 3).
__device__ __forceinline__ u32 wave_incl_scan(u32 v) {
    const int lane = threadIdx.x & 63, rl = lane & 15;
    u32 y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    if (rl >= 1) v += y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    if (rl >= 2) v += y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    if (rl >= 4) v += y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    if (rl >= 8) v += y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x142, 0xf, 0xf, false);  // row_bcast:15
    if (lane & 16) v += y;
    y = (u32)__builtin_amdgcn_mov_dpp((int)v, 0x143, 0xf, 0xf, false);  // row_bcast:31
    if (lane >= 32) v += y;
    return v;
}

// Exclusive scan over the workgroup (u32 add, so packed 16-bit pairs work).
template <int NT>
__device__ __forceinline__ u32 block_excl_scan(u32 x, u32& total, u32* wsum) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u32 v = wave_incl_scan(x);
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        const u32 s = wave_incl_scan(lane < NW ? wsum[lane] : 0u);
        if (lane < NW) wsum[lane] = s;
    }
    __syncthreads();
    total = wsum[NW - 1];
    u32 before = w ? wsum[w - 1] : 0u;
    return before + v - x;
}

// The same two scans on 64-bit values (four packed 16-bit counts).
template <int CTRL> __device__ __forceinline__ u64 dpp_move64(u64 x) {
    const u32 lo = (u32)__builtin_amdgcn_mov_dpp((int)(u32)x, CTRL, 0xf, 0xf, false);
    const u32 hi = (u32)__builtin_amdgcn_mov_dpp((int)(u32)(x >> 32), CTRL, 0xf, 0xf, false);
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 wave_incl_scan64(u64 v) {
    const int lane = threadIdx.x & 63, rl = lane & 15;
    u64 y;
    y = dpp_move64<0x111>(v);
    if (rl >= 1) v += y;
    y = dpp_move64<0x112>(v);
    if (rl >= 2) v += y;
    y = dpp_move64<0x114>(v);
    if (rl >= 4) v += y;
    y = dpp_move64<0x118>(v);
    if (rl >= 8) v += y;
    y = dpp_move64<0x142>(v);
    if (lane & 16) v += y;
    y = dpp_move64<0x143>(v);
    if (lane >= 32) v += y;
    return v;
}

// ws holds NT/64 values; the caller puts a barrier between this scan and the
// next write of ws.
template <int NT>
__device__ __forceinline__ u64 block_excl_scan64(u64 x, u64& total, u64* ws) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const u64 v = wave_incl_scan64(x);
    if (lane == 63) ws[w] = v;
    __syncthreads();
    if (w == 0) {
        const u64 s = wave_incl_scan64(lane < NW ? ws[lane] : (u64)0);
        if (lane < NW) ws[lane] = s;
    }
    __syncthreads();
    total = ws[NW - 1];
    const u64 before = w ? ws[w - 1] : (u64)0;
    return before + v - x;
}

// A value every lane of the wave holds alike, moved to a scalar register
// (keeps workgroup-uniform values out of the vector registers).
__device__ __forceinline__ u32 uniform(u32 v) { return (u32)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ u64 uniform(u64 v) {
    const u32 lo = uniform((u32)v), hi = uniform((u32)(v >> 32));
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int NT, typename K>
__device__ __forceinline__ void block_minmax(K& mn, K& mx, u64* red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        K a = __shfl_xor(mn, o, 64);
        K b = __shfl_xor(mx, o, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (lane == 0) { red[w] = (u64)mn; red[NW + w] = (u64)mx; }
    __syncthreads();
    mn = (K)red[0];
    mx = (K)red[NW];
#pragma unroll
    for (int i = 1; i < NW; i++) {
        K a = (K)red[i], b = (K)red[NW + i];
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    mn = uniform(mn);
    mx = uniform(mx);
    __syncthreads();
}

// ---------------------------------------------------------------- stable rank

// rank[j] = position of item j (thread t, blocked position t*IT + j) after a
// stable sort by digit dig[j] in [0, RADIX). Counter word (h, t) sits at
// padi(h*NT + t) = h*ROW + padi(t) (row stride ROW = NT + NT/32): thread t's
// raking slice of HALF words in flattened (h, t) order is contiguous, and the
// per-item read-modify-writes of a wave hit consecutive banks. Digits d and
// d + HALF share word (d, t) as its low and high 16 bits; hsf(j) is the bit
// offset of item j's half, 16 * (dig[j] >= HALF).
//
// SEP (counters apart from the exchange buffer): each thread clears its own
// column (no other thread touches it between the scan of the last pass and
// the counting of this one), so neither the clear nor the end of the rank
// needs a barrier.
template <int NT, int IT, bool SEP = false, typename DF, typename HF>
__device__ __forceinline__ void radix_rank(DF digf, HF hsf, u32 (&rank)[IT], u32* cnt, u32* wsum) {
    constexpr u32 ROW = NT + NT / 32;
    const int t = threadIdx.x;
    const u32 padt = (u32)padi(t);
#if BSPS_DIG_RECOMPUTE
#define DIG(j) digf(j)
#else
    u32 dig[IT];
#pragma unroll
    for (int j = 0; j < IT; j++) dig[j] = digf(j);
#define DIG(j) dig[j]
#endif
    if (SEP) {
#pragma unroll
        for (int h = 0; h < HALF; h++) cnt[h * ROW + padt] = 0u;
    } else {
        // each thread clears its own raking slice
#pragma unroll
        for (int i = 0; i < HALF; i++) cnt[padi(t * HALF + i)] = 0u;
        __syncthreads();
    }
    u32 ai[IT];  // counter word of each item
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const u32 d = DIG(j);
        u32 a = (d & (HALF - 1)) * ROW + padt;
        asm volatile("" : "+v"(a));  // kept, not recomputed from the digit, for the second read
        const u32 sh = hsf(j);
        const u32 w = cnt[a];
        rank[j] = (w >> sh) & 0xffffu;
        cnt[a] = w + (1u << sh);
        ai[j] = a;
    }
    __syncthreads();
    u32 sum = 0;
#pragma unroll
    for (int i = 0; i < HALF; i++) sum += cnt[padi(t * HALF + i)];
    u32 total;
    u32 run = block_excl_scan<NT>(sum, total, wsum);
    // every item of a high digit follows all items of the low digits: the high
    // halves start at the low total (at most NT*IT, so neither half overflows)
    run += (total & 0xffffu) << 16;
#pragma unroll
    for (int i = 0; i < HALF; i++) {
        const int a = padi(t * HALF + i);
        const u32 v = cnt[a];
        cnt[a] = run;
        run += v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IT; j++) {
        rank[j] += (cnt[ai[j]] >> hsf(j)) & 0xffffu;
    }
#undef DIG
    if (!SEP) __syncthreads();
}

// The same rank for a pass of at most 2 bits (digits 0..3) without LDS
// counters: each thread counts its digits in one register (8 bits per digit;
// IT < 256), the four counts are widened to 16-bit fields of a 64-bit value,
// and one workgroup scan of those gives every digit's thread offsets. ws is
// LDS scratch for NT/64 64-bit values.
template <int NT, int IT, bool SEP = false, typename DF>
__device__ __forceinline__ void radix_rank4(DF digf, u32 (&rank)[IT], u64* ws) {
    static_assert(IT < 256 && NT * IT <= 65535, "8-bit thread counts, 16-bit totals");
    u32 c = 0;
#pragma unroll
    for (int j = 0; j < IT; j++) {
        const u32 sh = digf(j) << 3;
        rank[j] = (c >> sh) & 0xffu;
        c += 1u << sh;
    }
    const u64 x = (u64)(c & 0xffu) | ((u64)(c & 0xff00u) << 8) | ((u64)(c & 0xff0000u) << 16) |
                  ((u64)(c & 0xff000000u) << 24);
    u64 tot;
    const u64 ex = block_excl_scan64<NT>(x, tot, ws);
    // field d of base: items of the lower digits plus this digit's items in
    // the threads before this one (each field stays below 2^16)
    const u32 t0 = (u32)tot & 0xffffu, t1 = (u32)(tot >> 16) & 0xffffu, t2 = (u32)(tot >> 32) & 0xffffu;
    const u64 base = ex + (((u64)t0 << 16) | ((u64)(t0 + t1) << 32) | ((u64)(t0 + t1 + t2) << 48));
#pragma unroll
    for (int j = 0; j < IT; j++) rank[j] += (u32)(base >> (digf(j) << 4)) & 0xffffu;
    if (!SEP) __syncthreads();  // ws lies in the counter region
}

// ---------------------------------------------------------------- workgroup sort

// Sorts the NT*IT items held in registers (blocked order; unused tail items
// must hold the largest rebased key) by their rebased keys sk (nbits wide). Keys and payloads share one exchange buffer, one after
// the other. On return the sorted keys are in exch[padi(i)], i = 0..NT*IT-1,
// and rank[j] is the final position of item j, whose payload is still v[j];
// the caller stores the keys, then calls wg_scatter_vals() for the payloads.
// SK = u32 or u64; exch holds NT*IT + NT*IT/32 elements of SK.
// SMALLPASS: a last pass of at most 2 bits ranks without LDS counters (more
// code; kernels short of registers leave it off).
#ifndef BSPS_SMALLPASS
#define BSPS_SMALLPASS 1
#endif
// sh0: the sort key is bits [sh0, sh0 + nbits) of sk (0: the low nbits).
template <int NT, int IT, typename SK, bool HASV, bool SMALLPASS = (bool)BSPS_SMALLPASS, bool SEP = false>
__device__ __forceinline__ void wg_sort_regs(SK (&sk)[IT], u32 (&v)[IT], u32 (&rank)[IT], int nbits, SK* exch,
                                             u32* cnt, u32* wsum, int sh0 = 0) {
    const int t = threadIdx.x;
    u32* vex = reinterpret_cast<u32*>(exch);
    // all sort keys equal (nbits = 0): one pass over the all-zero digit, which
    // ranks every item at its own position
    const int npass = nbits <= 0 ? 1 : (nbits + RB - 1) / RB;
    for (int pass = 0; pass < npass; pass++) {
        const int sh = sh0 + pass * RB;
        const bool last = pass == npass - 1;
        if (SMALLPASS && nbits - pass * RB <= 2) {
            // a last pass of at most 2 bits (or all keys equal)
            radix_rank4<NT, IT, SEP>([&](int j) { return (u32)(sk[j] >> sh) & 3u; }, rank,
                                     reinterpret_cast<u64*>(cnt));
        } else {
            const int hsh = sh + RB - 5;  // moves the digit's top bit to bit 4
            radix_rank<NT, IT, SEP>([&](int j) { return (u32)(sk[j] >> sh) & (RADIX - 1); },
                                    [&](int j) { return (u32)(sk[j] >> hsh) & 16u; }, rank, cnt, wsum);
        }
#pragma unroll
        for (int j = 0; j < IT; j++) exch[padi((int)rank[j])] = sk[j];
        __syncthreads();
        if (last) break;
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = exch[padi(t * IT + j)];
        // with SEP the next write of exch (the next scatter) follows the rank's
        // barriers; payloads reuse exch at once
        if (!SEP || HASV) __syncthreads();
        if (HASV) {
#pragma unroll
            for (int j = 0; j < IT; j++) vex[padi((int)rank[j])] = v[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = vex[padi(t * IT + j)];
            __syncthreads();
        }
    }
}

// wg_sort_regs for wide 64-bit sort keys (bits [sh0, sh0 + nbits), nbits at
// least TOPW + 2 digits), ranked on their top TOPW bits first. When no two
// different keys share those top bits, that stable order is already the full
// order (equal top bits then mean equal keys, which keep their input order),
// and the passes over the lower bits are skipped: with at most 2^13 items and
// keys spread over their range, two of them meet in 2^30 top-bit classes with
// odds about 1/32, and inputs of few distinct keys (heavy duplicates) never.
// Otherwise the full sort runs on the top-ordered items; being stable, it
// keeps equal keys in the order the first sort left them, their input order.
// Same contract as wg_sort_regs on return.
constexpr int TOPW = 30;
template <int NT, int IT, bool HASV, bool SMALLPASS = (bool)BSPS_SMALLPASS, bool SEP = false>
__device__ __forceinline__ void wg_sort_regs_top(u64 (&sk)[IT], u32 (&v)[IT], u32 (&rank)[IT], int nbits, u64* exch,
                                                 u32* cnt, u32* wsum, int sh0 = 0) {
    const int t = threadIdx.x;
    const bool wide = nbits >= TOPW + 2 * RB;
    int nb = wide ? TOPW : nbits;
    const int tsh = wide ? sh0 + nbits - TOPW : sh0;
    // one sort call in a loop (the top bits, then if needed all bits), so that
    // the sort's code is instantiated once
    for (;;) {
        wg_sort_regs<NT, IT, u64, HASV, SMALLPASS, SEP>(sk, v, rank, nb, exch, cnt, wsum, nb == nbits ? sh0 : tsh);
        if (nb == nbits) return;
        // sorted keys are in exch[padi(i)]; a class of equal top bits must hold one key
        int mixed = 0;
#pragma unroll
        for (int j = 0; j < IT; j++) {
            const int i = t * IT + j;
            if (i + 1 < NT * IT) {
                const u64 x = exch[padi(i)], y = exch[padi(i + 1)];
                mixed |= ((x >> tsh) == (y >> tsh) && (x >> sh0) != (y >> sh0)) ? 1 : 0;
            }
        }
        if (!__syncthreads_or(mixed)) return;
        // the items in their top-bit order, payloads moved along, then the full sort
#pragma unroll
        for (int j = 0; j < IT; j++) sk[j] = exch[padi(t * IT + j)];
        __syncthreads();
        if (HASV) {
            u32* vex = reinterpret_cast<u32*>(exch);
#pragma unroll
            for (int j = 0; j < IT; j++) vex[padi((int)rank[j])] = v[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IT; j++) v[j] = vex[padi(t * IT + j)];
            __syncthreads();
        }
        nb = nbits;
    }
}

// Moves payloads to their final positions (after the keys were stored out of
// the exchange buffer): vex[padi(rank[j])] = v[j].
template <int NT, int IT>
__device__ __forceinline__ void wg_scatter_vals(const u32 (&v)[IT], const u32 (&rank)[IT], u32* vex) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IT; j++) vex[padi((int)rank[j])] = v[j];
    __syncthreads();
}

// ---------------------------------------------------------------- keyed permutation

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ u64 mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Image of t under a keyed permutation of [0, n): a balanced 4-round Feistel
// network on 2h >= ceil(log2 n) bits whose round function is mix64 of
// (seed + golden*(round+1) + right half), restricted to [0, n) by cycle
// walking (Black & Rogaway 2002).
__device__ __forceinline__ u64 feistel_perm(u64 seed, u64 n, u64 t) {
    if (n <= 1) return 0;
    int bits = 64 - __clzll((long long)(n - 1));
    int h = (bits + 1) >> 1;
    u64 mask = (1ull << h) - 1;
    u64 x = t;
    do {
        u64 L = x >> h, R = x & mask;
#pragma unroll
        for (u64 j = 0; j < 4; j++) {
            u64 f = mix64(seed + 0x9E3779B97F4A7C15ull * (j + 1) + R) & mask;
            u64 nl = R;
            R = L ^ f;
            L = nl;
        }
        x = (L << h) | R;
    } while (x >= n);
    return x;
}
