// bsps.hip -- host pipeline and C ABI of libbsps.so (see include/bsps.h).
//
// One call of bsps_sort enqueues, on the caller's stream:
//   A1 tile sort + block merge           -> B (every block sorted)
//   A2 DET regular / RAN keyed sample    -> sample records (key, position in B)
//   A3 sample sort + splitters           -> p-1 splitter records
//   A4 splitter search into each block   -> cntT (or per-key ranking, SCATTER route)
//   A5 bucket tables (prefix sums)       -> runs of every bucket
//   A6 per-bucket multiway merge         -> sorted keys back in the caller's buffer
// Every device buffer is carved from the caller's workspace; the library never
// allocates device memory on these paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/bsps.h"
#include "bsps_kernels.h"
#include "bsps_learned.h"
#include "bsps_lsd.h"
#include "bsps_sr.h"
#include "bsps_iter.h"
#include "bsps_segmented.h"

#include <map>
#include <mutex>
#include <string>
#include <type_traits>

// Scratch memory of the allocation-free entry point (bsps_sort_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never uses its name as an address: the per-device address comes
// from hipGetSymbolAddress (scratch_base below).
static __device__ __align__(256) unsigned char scratch[BSPS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr u32 kSampleStride = 32;  // tile and block samples for the merges: every 32nd key
constexpr int kMaxP = MAXR;  // p <= 1024
constexpr int kMaxRounds = 10;  // iterative rounds: p = k^m with k >= 2 and p <= 1024

// A failed HIP call maps to BSPS_EDEVICE; with BSPS_DEBUG set in the
// environment the call, the source line and HIP's message go to stderr.
bool debug_on() {
    static int v = -1;
    if (v < 0) v = std::getenv("BSPS_DEBUG") ? 1 : 0;
    return v == 1;
}
bsps_status hip_fail(hipError_t e, const char* what, int line) {
    if (debug_on()) std::fprintf(stderr, "[bsps] %s failed (bsps.hip:%d): %s\n", what, line, hipGetErrorString(e));
    return BSPS_EDEVICE;
}
#define HIP_OK(x)                                                      \
    do {                                                               \
        const hipError_t e_ = (x);                                     \
        if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__);       \
    } while (0)
#define LAUNCH_OK()                                                    \
    do {                                                               \
        if (t_dry) break;                                              \
        const hipError_t e_ = hipGetLastError();                       \
        if (e_ != hipSuccess) return hip_fail(e_, "launch", __LINE__); \
    } while (0)

// ------------------------------------------------------------------ host dry run
//
// With t_dry set (bsps_check_sort / bsps_check_segmented), the host pipeline
// plans and "launches" every kernel without touching the GPU: each launch's
// arguments are checked instead. Every pointer argument, and every pointer
// inside the argument structs, must be null or lie inside the caller's
// buffers or the workspace, and so must the whole extent of every table the
// kernel indexes by its sizes. Plans are made with fake buffer addresses.
struct DryRun {
    struct Range { uintptr_t lo, hi; };
    std::vector<Range> ranges;
    std::vector<std::string> errors;
    int launches = 0;
    u64 grid = 0;
    std::string kernel;
    void add(const void* p, size_t bytes) { ranges.push_back({(uintptr_t)p, (uintptr_t)p + bytes}); }
    void fail(const char* what, const void* p, size_t bytes) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "%s: %s = %p (+%zu bytes) outside every buffer", kernel.c_str(), what, p,
                      bytes);
        errors.push_back(buf);
    }
    // [p, p + bytes) inside one buffer (bytes 0: p may be one past the end)
    void span(const char* what, const void* p, size_t bytes) {
        if (!p) return;
        const uintptr_t a = (uintptr_t)p;
        for (auto& r : ranges)
            if (a >= r.lo && a + bytes <= r.hi) return;
        fail(what, p, bytes);
    }
};
thread_local DryRun* t_dry = nullptr;

inline u64 cdiv(u64 a, u64 b) { return (a + b - 1) / b; }
inline int bitw(u64 v) { int b = 0; while (v) { b++; v >>= 1; } return b; }
// The learned-rank counters (two u64, updated by 64-bit atomics) follow the
// p*p count matrix at the next 8-byte boundary.
inline size_t lstats_off(int p) { return ((size_t)p * p + 1) & ~(size_t)1; }
// Workspaces are carved into 256-byte aligned pieces and must start aligned.
inline bool ws_ok(const void* ws) { return ws && ((uintptr_t)ws & 255) == 0; }
inline i64 hblk(i64 n, int p, int k) { return (i64)(((u64)k * (u64)n) / (u64)p); }

// Bump allocator over the caller's workspace (256-byte aligned pieces). With
// base == nullptr it only measures.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(u64 count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
};

int key_bytes(int dt) { return dt == BSPS_I64 ? 8 : 4; }

// Argument checks of the dry run, by type: a plain pointer must lie inside a
// buffer (its extent is not known here); an argument struct's tables must fit
// inside a buffer at the extent the kernel indexes them with; scalars pass.
template <typename T>
void dry_check(T* p) {
    t_dry->span("pointer argument", p, 0);
}
template <typename T>
typename std::enable_if<std::is_arithmetic<T>::value || std::is_enum<T>::value>::type dry_check(T) {}
template <typename T>
void dry_span(const char* what, const T* p, u64 count) {
    t_dry->span(what, p, (size_t)count * sizeof(T));
}
template <typename K>
void dry_check(const TileArgs<K>& a) {
    const u64 n = (u64)std::max<i64>(a.n, 0);
    dry_span("TileArgs.gsh", a.gsh, a.btab ? 1 : (u64)a.p);
    dry_span("TileArgs.in", a.in, n);
    dry_span("TileArgs.inv", a.inv, n);
    dry_span("TileArgs.out", a.out, n);
    dry_span("TileArgs.outv", a.outv, n);
    const u64 ntile = a.persist ? a.ntile : t_dry->grid;
    if (a.btab) {
        dry_span("TileArgs.btab", a.btab, 4 * ntile);
        dry_span("TileArgs.dtab", a.dtab, 1);
        dry_span("TileArgs.outd", a.outd, n);
        dry_span("TileArgs.outdv", a.outdv, n);
        dry_span("TileArgs.smp", a.smp, 1);
    } else {
        dry_span("TileArgs.smp", a.smp, (u64)a.p * a.tpb * a.spt);
        if (a.dtab || a.outd || a.outdv) t_dry->fail("TileArgs: segment tables without btab", a.dtab, 0);
    }
}
template <typename K>
void dry_check(const MwmArgs<K>& a) {
    const u64 G = (u64)a.G, R = (u64)a.R, S = a.S;
    dry_span("MwmArgs.src", a.src, 0);
    dry_span("MwmArgs.srcv", a.srcv, 0);
    dry_span("MwmArgs.dst", a.dst, 0);
    dry_span("MwmArgs.dstv", a.dstv, 0);
    dry_span("MwmArgs.scr", a.scr, 0);
    dry_span("MwmArgs.scrv", a.scrv, 0);
    dry_span("MwmArgs.run_start", a.run_start, G * R);
    dry_span("MwmArgs.run_len", a.run_len, G * R);
    dry_span("MwmArgs.out_base", a.out_base, G);
    dry_span("MwmArgs.sdesc", a.sdesc, G * R * 4);
    dry_span("MwmArgs.smp", a.smp, 0);
    dry_span("MwmArgs.counters", a.slot_count, 6);
    dry_span("MwmArgs.slot_group", a.slot_group, S);
    dry_span("MwmArgs.grp_base", a.grp_base, G);
    dry_span("MwmArgs.grp_nb", a.grp_nb, G);
    dry_span("MwmArgs.bkey", a.bkey, S);
    dry_span("MwmArgs.gsh", a.gsh, a.gsh_one ? 1 : G);
    dry_span("MwmArgs.ssh", a.ssh, 1);
    dry_span("MwmArgs.bpos", a.bpos, S);
    dry_span("MwmArgs.cuts", a.cuts, S * R);
    dry_span("MwmArgs.below", a.below, S);
    dry_span("MwmArgs.witem", a.witem, 2 * S);
    dry_span("MwmArgs.heavy", a.heavy, G);
    dry_span("MwmArgs.gpar", a.gpar, 2 * G);
    dry_span("MwmArgs.osmp", a.osmp, G * a.ospb);
    if (a.R > MAXR || a.G < 0) t_dry->fail("MwmArgs: more runs per group than the merge holds", nullptr, 0);
}
template <typename K>
void dry_check(const LsdArgs<K>& a) {
    const u64 n = (u64)a.n, p = (u64)a.p, DP = sizeof(K);
    dry_span("LsdArgs.in", a.in, n);
    dry_span("LsdArgs.inv", a.inv, n);
    dry_span("LsdArgs.a", a.a, n);
    dry_span("LsdArgs.av", a.av, n);
    dry_span("LsdArgs.b", a.b, n);
    dry_span("LsdArgs.bv", a.bv, n);
    dry_span("LsdArgs.out", a.out, n);
    dry_span("LsdArgs.outv", a.outv, n);
    dry_span("LsdArgs.dbase", a.dbase, p * DP * LSD_RADIX);
    dry_span("LsdArgs.plist", a.plist, p * (DP + 1));
    dry_span("LsdArgs.smp", a.smp, p * a.spb);
    dry_span("LsdArgs.blk", a.blk, p);
    if (!a.inv != !a.outv || !a.av != !a.outv || !a.bv != !a.outv)
        t_dry->fail("LsdArgs: payload buffers given for some passes only", a.outv, 0);
}
void dry_check(const LsdSweep& w) {
    dry_span("LsdSweep.status", w.status, (u64)w.ntile * LSD_RADIX);
    dry_span("LsdSweep.ctr", w.ctr, 2);
    if (!w.hist) t_dry->fail("LsdSweep: missing digit counts", w.hist, 0);
    if (!w.status || !w.ctr || !w.tstart) t_dry->fail("LsdSweep: missing buffer", w.status, 0);
}
template <typename... A>
void dry_launch(const char* name, dim3 grid, dim3 block, const A&... args) {
    t_dry->kernel = name;
    t_dry->launches++;
    t_dry->grid = (u64)grid.x * grid.y * grid.z;
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x == 0 || block.x > 1024)
        t_dry->errors.push_back(std::string(name) + ": empty grid or bad workgroup size");
    (dry_check(args), ...);
}

// A kernel launch, or its argument check in a dry run.
#define LAUNCH(KER, GRID, BLOCK, SHMEM, STREAM, ...)                                    \
    do {                                                                                \
        if (t_dry)                                                                      \
            dry_launch(#KER, dim3(GRID), dim3(BLOCK), __VA_ARGS__);                     \
        else                                                                            \
            hipLaunchKernelGGL(KER, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);           \
    } while (0)

// Optional per-stage timing with HIP events recorded on the caller's stream
// around each stage (diagnostics and benchmarks only).
enum Stage {
    ST_TILE = 0,       // A1: tile sorts
    ST_BLOCK_MERGE,    // A1: block merge (pick + cuts + merge)
    ST_SAMPLE,         // A2 + A3: sample, sample sort, splitters
    ST_COUNT,          // A4: splitter search into blocks (or per-key ranking)
    ST_TABLES,         // A5: prefix sums / bucket tables (and scatter)
    ST_BUCKET_MERGE,   // A6: bucket merge (pick + cuts + merge)
    ST_BLOCK_MERGE_K,  // k_mwm_merge alone, block merge
    ST_BUCKET_MERGE_K, // k_mwm_merge alone, bucket merge
    ST_RANK_K,         // per-key rank kernel alone
    ST_LSD_K,          // A1 by LSD radix: the pass kernels alone
    ST_N
};
struct StageTimer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ST_N];
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
StageTimer g_timer;
// Set while an allocation-free call enqueues: no timing events are created.
thread_local bool t_no_events = false;
struct StageScope {
    int stage;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    StageScope(int s_, hipStream_t st_) : stage(s_), st(st_) {
        if (stage < ST_N && g_timer.on && !t_no_events && !t_dry && (e0 = g_timer.get()) &&
            hipEventRecord(e0, st) != hipSuccess)
            e0 = nullptr;
    }
    ~StageScope() {
        if (!e0) return;
        hipEvent_t e1 = g_timer.get();
        if (!e1 || hipEventRecord(e1, st) != hipSuccess) return;
        g_timer.ev[stage].push_back({e0, e1});
    }
};

template <typename K> constexpr u32 tileT() { return (u32)(Shape<K>::NT * Shape<K>::IT); }

// Device buffers of one multiway merge.
template <typename K>
struct MwmBufs {
    u32 *run_start, *run_len, *out_base, *sdesc, *counters, *slot_group, *grp_base, *grp_nb, *bpos, *cuts;
    u32 *below, *heavy;
    uint4 *witem, *gpar;
    K* bkey;
    u32 S;
    int G, R;
};

template <typename K>
void carve_mwm(Carver& c, MwmBufs<K>& m, int G, int R, u64 n, u32 tavg) {
    m.G = G;
    m.R = R;
    // chunks of a group of N > cap keys: at most N / tavg + 2 (k_mwm_pick)
    m.S = (u32)(n / tavg + 2 * (u64)G + 1);
    m.run_start = c.take<u32>((u64)G * R);
    m.run_len = c.take<u32>((u64)G * R);
    m.out_base = c.take<u32>(G);
    m.sdesc = c.take<u32>((u64)G * R * 4);
    m.counters = c.take<u32>(8);  // slots, oversize, merge claims, largest oversize, work items, listed groups
    m.slot_group = c.take<u32>(m.S);
    m.grp_base = c.take<u32>(G);
    m.grp_nb = c.take<u32>(G);
    m.bkey = c.take<K>(m.S);
    m.bpos = c.take<u32>(m.S);
    m.cuts = c.take<u32>((u64)m.S * R);
    m.below = c.take<u32>(m.S);
    m.witem = c.take<uint4>(2 * (u64)m.S);
    m.heavy = c.take<u32>(G);
    m.gpar = c.take<uint4>(2 * (u64)G);
}

template <typename K>
MwmArgs<K> mwm_args(const MwmBufs<K>& m, const K* src, const u32* srcv, K* dst, u32* dstv, K* scr, u32* scrv,
                    const K* smp, u32 cap, u32 tavg, int out_dt, K* osmp, u32 oys, u32 ospb) {
    MwmArgs<K> a{};
    a.src = src; a.srcv = srcv; a.dst = dst; a.dstv = dstv; a.scr = scr; a.scrv = scrv;
    a.G = m.G; a.R = m.R;
    a.run_start = m.run_start; a.run_len = m.run_len; a.out_base = m.out_base; a.sdesc = m.sdesc;
    a.smp = smp; a.cap = cap; a.tavg = tavg;
    a.slot_count = m.counters; a.oversize = m.counters + 1; a.work = m.counters + 2;
    a.slot_group = m.slot_group; a.grp_base = m.grp_base; a.grp_nb = m.grp_nb;
    a.bkey = m.bkey; a.bpos = m.bpos; a.cuts = m.cuts; a.below = m.below; a.S = m.S;
    a.witem = m.witem; a.nwork = m.counters + 4;
    a.heavy = m.heavy; a.nheavy = m.counters + 5; a.gpar = m.gpar;
    a.out_dt = out_dt; a.osmp = osmp; a.oys = oys; a.ospb = ospb;
    return a;
}

int device_cus() {
    if (t_dry) return 256;
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Per-key rank launch: every tile once, with at most as many workgroups as
// are resident at the same time (the kernel walks tiles with a stride).
template <typename K, bool LEARNED>
bsps_status launch_rank(const K* B, i64 n, int p, const K* spk, const u32* spp, int dt, int sdt, const void* model,
                        u32* bucket, u32* counts, unsigned long long* lstats, hipStream_t st) {
    typedef RankShape<LEARNED> RS;
    const int tpb = (int)cdiv(cdiv((u64)n, (u64)p), (u64)rank_tile<LEARNED>());
    const u32 grid = (u32)std::max<i64>(1, std::min<i64>((i64)p * tpb, (i64)device_cus() * RS::WG_PER_CU));
    LAUNCH((k_rank<K, LEARNED>), dim3(grid), dim3(RS::NT), 0, st, B, n, p, tpb, spk, spp, dt, sdt, model,
                       bucket, counts, lstats);
    LAUNCH_OK();
    return BSPS_OK;
}

template <typename K, bool HASV>
bsps_status mwm_run(const MwmArgs<K>& a, hipStream_t st, int kstage = ST_N) {
    constexpr int NT = Shape<K>::NT;
    const int cus = device_cus();
    LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, st, a.slot_count, 8);
    LAUNCH_OK();
    LAUNCH((k_mwm_size<K>), dim3(a.G), dim3(SIZE_NT), 0, st, a);
    LAUNCH_OK();
    // the groups with boundaries only (listed by k_mwm_size), in loops
    LAUNCH((k_mwm_pick<K>), dim3((u32)std::min<u64>(a.G, (u64)cus * 2)), dim3(NT), 0, st, a);
    LAUNCH_OK();
    // one wave per (group, run); with few runs the boundaries are split over
    // gridDim.y waves so that the launch still holds some 8K waves
    const u64 nwave = std::max<u64>(1, (u64)a.G * a.R);
    const u32 ysplit = (u32)std::min<u64>(64, std::max<u64>(1, cdiv(8192, nwave)));
    // window counts by half-waves pay off with 4-byte keys and some 32 or more
    // boundaries per group (chunks fill about 7/8 of the cap); the keys per
    // group follow from the slot capacity S = keys / tavg + 2 G + 1
    const u64 per_group = ((u64)a.S - 2ull * a.G - 1) * a.tavg / std::max<u64>(1, a.G);
    const bool coop = sizeof(K) == 4 && per_group >= 28ull * a.cap;
    if (coop)
        LAUNCH((k_mwm_cuts<K, sizeof(K) == 4>), dim3((u32)cdiv(nwave, CUT_NT / 64), ysplit), dim3(CUT_NT), 0, st, a);
    else
        LAUNCH((k_mwm_cuts<K, false>), dim3((u32)cdiv(nwave, CUT_NT / 64), ysplit), dim3(CUT_NT), 0, st, a);
    LAUNCH_OK();
    LAUNCH((k_mwm_below<K>), dim3((u32)std::min<u64>(cdiv(a.S, 4), (u64)cus * 16)), dim3(256), 0, st,
                       a);
    LAUNCH_OK();
    LAUNCH((k_mwm_plan<K>), dim3((u32)std::min<u64>(a.G, (u64)cus * 4)), dim3(PLAN_NT), 0, st, a);
    LAUNCH_OK();
#ifndef BSPS_MERGE_WGS_PER_CU
#define BSPS_MERGE_WGS_PER_CU 2
#endif
    const u32 gmerge = BSPS_MERGE_WGS_PER_CU > 0 ? (u32)std::min<u64>(a.S, (u64)cus * BSPS_MERGE_WGS_PER_CU) : a.S;
    {
        StageScope sc(kstage, st);
        // with a sort shift (known on the device only) both variants are
        // launched, and the one that does not fit its value returns at once
        if (a.ssh) {
            LAUNCH((k_mwm_merge<K, HASV, true>), dim3(gmerge), dim3(NT), 0, st, a);
            LAUNCH_OK();
        }
        LAUNCH((k_mwm_merge<K, HASV, false>), dim3(gmerge), dim3(NT), 0, st, a);
    }
    LAUNCH_OK();
    return BSPS_OK;
}

// ------------------------------------------------------------------ block sort (A1)

// Buffers of one "sort n keys split into p blocks" (the local sort of every
// virtual processor): tiles, tile samples and the block merge.
template <typename K>
struct BlockSortBufs {
    K* A;            // tile-sorted keys (NULL when every block fits one tile)
    u32* Av;
    K* tsmp;         // tile samples
    MwmBufs<K> mwm;
    int tpb;
    u32 spt;
};

template <typename K>
void carve_block_sort(Carver& c, BlockSortBufs<K>& b, u64 n, int p, bool hasv, u32 tavg, bool force_A) {
    const u32 T = tileT<K>();
    const u64 m = cdiv(n, (u64)p);
    b.tpb = (int)std::max<u64>(1, cdiv(m, T));
    b.spt = T / kSampleStride;
    b.A = nullptr;
    b.Av = nullptr;
    b.tsmp = nullptr;
    std::memset(&b.mwm, 0, sizeof(b.mwm));
    if (b.tpb > 1 || force_A) {
        b.A = c.take<K>(n);
        if (hasv) b.Av = c.take<u32>(n);
    }
    if (b.tpb > 1) {
        b.tsmp = c.take<K>((u64)p * b.tpb * b.spt);
        carve_mwm<K>(c, b.mwm, p, b.tpb, n, tavg);
    }
}

// Grid of a tile-sort launch over ntile tiles. Keys only: a persistent grid of
// the workgroups that are resident at once (ta.persist), each loading its next
// tile while it sorts the current one; with payloads one workgroup per tile.
template <typename K, bool HASV, bool TT = false>
u32 tile_grid(TileArgs<K>& ta, u32 ntile) {
    constexpr int NT = Shape<K>::NT;
    ta.ntile = ntile;
    if (HASV) return ntile;
    static int occ = -1;
    if (!t_dry && occ < 0 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_tile_sort<K, HASV, TT>, NT, 0) != hipSuccess)
        occ = 0;
    if (!t_dry && occ <= 0) return ntile;
    ta.persist = 1;
    return (u32)std::max<u64>(1, std::min<u64>(ntile, (u64)device_cus() * std::max(occ, 1)));
}

// in (dtype in_dt) -> out (order keys, or raw keys of out_dt), every block of
// the p-way split sorted. scr/scrv: n-element scratch for oversize chunks
// (may be the input). osmp: block samples every yb-th key (slot stride spb).
template <typename K, bool HASV>
bsps_status block_sort(const BlockSortBufs<K>& b, const K* in, const u32* inv, int in_dt, K* out, u32* outv,
                       int out_dt, K* scr, u32* scrv, i64 n, int p, u32 cap, u32 tavg, K* osmp, u32 yb, u32 spb,
                       hipStream_t st, int tstage = ST_N, int mstage = ST_N, int mkstage = ST_N,
                       u32* gsh = nullptr, int keep = 0, u32* bsh = nullptr) {
    constexpr int NT = Shape<K>::NT;
    const u32 T = tileT<K>();
    TileArgs<K> ta{};
    ta.in = in; ta.inv = inv; ta.n = n; ta.p = p; ta.tpb = b.tpb; ta.in_dt = in_dt;
    if (b.tpb == 1) {
        ta.out = out; ta.outv = outv; ta.out_dt = out_dt; ta.smp = osmp; ta.ys = yb; ta.spt = spb;
        StageScope sc(tstage, st);
        LAUNCH((k_tile_sort<K, HASV>), dim3(p), dim3(NT), 0, st, ta);
        LAUNCH_OK();
        return BSPS_OK;
    }
    ta.out = b.A; ta.outv = b.Av; ta.out_dt = BSPS_DT_NONE; ta.smp = b.tsmp; ta.ys = kSampleStride; ta.spt = b.spt;
    ta.gsh = gsh;  // tiles that are merged afterwards may be sorted on their high part only
    const u32 tgrid = tile_grid<K, HASV>(ta, (u32)(p * b.tpb));
    {
        StageScope sc(tstage, st);
        if (gsh) {
            LAUNCH((k_trunc_probe<K>), dim3((u32)p), dim3(TRUNC_NT), 0, st, in, in_dt, n, p, keep, gsh);
            LAUNCH_OK();
            if (bsh) {
                LAUNCH(k_min_shift, dim3(1), dim3(256), 0, st, (const u32*)(gsh + p + 1), p, bsh);
                LAUNCH_OK();
            }
        }
        LAUNCH((k_tile_sort<K, HASV>), dim3(tgrid), dim3(NT), 0, st, ta);
    }
    LAUNCH_OK();
    StageScope sc(mstage, st);
    const u64 nrun = (u64)p * b.tpb;
    LAUNCH((k_block_tables<K>), dim3((u32)cdiv(nrun, 256)), dim3(256), 0, st, n, p, b.tpb, T,
                       kSampleStride, b.spt, b.mwm.run_start, b.mwm.run_len, b.mwm.out_base, b.mwm.sdesc);
    LAUNCH_OK();
    MwmArgs<K> a = mwm_args<K>(b.mwm, b.A, b.Av, out, outv, scr, scrv, b.tsmp, cap, tavg, out_dt, osmp, yb, spb);
    a.gsh = gsh;
    a.ssh = gsh ? bsh : nullptr;  // blocks sorted on key >> *bsh only
    // a block's groups of equal tile-shift high parts: m / 2^TRUNC_KEEPC keys
    // on average, each boundary gaining about half of one (k_trunc_probe)
    if (gsh) a.ggrow = (u32)(cdiv(cdiv((u64)n, (u64)p), (u64)1 << TRUNC_KEEPC));
    // 8-byte keys: a block's chunks span wide key ranges (up to ten digit
    // passes each), so fuller merge items outweigh the extra cuts; the bucket
    // merge's narrower chunks do not gain
    a.pack = sizeof(K) == 8 ? 1u : 0u;
    return mwm_run<K, HASV>(a, st, mkstage);
}

// ------------------------------------------------------------------ block sort by LSD radix (A1)

// in (dtype in_dt, keys and payloads) -> out (order keys): every block of the
// p-way split sorted stably by LSD passes through HBM. A/Av and in/inv itself
// are the scratch of the passes in between (in is consumed). osmp: block
// samples every yb-th key (slot stride spb).
template <typename K, bool HASV>
bsps_status lsd_launch(const LsdArgs<K>& a, const LsdSweep& w, hipStream_t st);

// Buffers of the tile-parallel passes: per tile and digit one status word,
// the ticket and overrun counters, the first tile of every block.
template <typename K>
LsdSweep carve_sweep(Carver& c, i64 n, int p) {
    LsdSweep w{};
    w.ntile = (u32)(cdiv((u64)n, tileT<K>()) + (u64)p);
    w.status = c.take<u32>((u64)w.ntile * LSD_RADIX);
    w.ctr = c.take<u32>(8);
    w.tstart = c.take<u32>((u64)p + 1);
    w.hist = c.take<u32>((u64)p * sizeof(K) * LSD_RADIX);
    w.spin_limit = 1u << 16;  // a wait lasts about one tile sort; this is some 1000 times that
    return w;
}

template <typename K, bool HASV>
bsps_status lsd_block_sort(K* in, u32* inv, int in_dt, K* A, u32* Av, K* out, u32* outv, u32* dbase, u32* plist,
                           const LsdSweep& w, i64 n, int p, int tpb, K* osmp, u32 yb, u32 spb, hipStream_t st) {
    constexpr int NT = Shape<K>::NT;
    LsdArgs<K> a{};
    a.in = in; a.inv = inv; a.in_dt = in_dt;
    a.a = A; a.av = Av; a.b = in; a.bv = inv;
    a.out = out; a.outv = outv;
    a.n = n; a.p = p; a.tpb = tpb;
    a.dbase = dbase; a.plist = plist;
    a.smp = osmp; a.ys = yb; a.spb = spb;
    a.blk = nullptr;
    a.out_dt = BSPS_DT_NONE;
    return lsd_launch<K, HASV>(a, w, st);
}

// The digit counts of every block, then one tile-parallel launch per digit
// position (blocks that need fewer passes skip the later launches).
template <typename K, bool HASV>
bsps_status lsd_launch(const LsdArgs<K>& a, const LsdSweep& w, hipStream_t st) {
    constexpr int NT = Shape<K>::NT;
    const int p = a.p;
    StageScope sc(ST_TILE, st);
    // digit counts: every tile adds its own into its block's, then every block's are scanned
    LAUNCH((k_lsd_tiles<K>), dim3(1), dim3(1024), 0, st, a, w);
    LAUNCH_OK();
    const u64 nh = (u64)p * sizeof(K) * LSD_RADIX;
    LAUNCH(k_zero_u32, dim3((u32)cdiv(nh, 256)), dim3(256), 0, st, w.hist, (int)nh);
    LAUNCH_OK();
    LAUNCH((k_lsd_count<K>), dim3(w.ntile), dim3(LSD_COUNT_NT), 0, st, a, w, w.hist);
    LAUNCH_OK();
    LAUNCH((k_lsd_scan<K>), dim3((u32)p), dim3(LSD_HIST_NT), 0, st, a, (const u32*)w.hist);
    LAUNCH_OK();
    LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, st, w.ctr, 8);
    LAUNCH_OK();
    StageScope sk(ST_LSD_K, st);
    const u64 nstat = (u64)w.ntile * LSD_RADIX;
    for (int pass = 0; pass < (int)sizeof(K); pass++) {
        LAUNCH(k_zero_u32, dim3((u32)cdiv(nstat, 256)), dim3(256), 0, st, w.status, (int)nstat);
        LAUNCH_OK();
        LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, st, w.ctr, 1);  // the ticket
        LAUNCH_OK();
        (void)p;
        LAUNCH((k_lsd_sweep<K, HASV>), dim3(w.ntile), dim3(NT), 0, st, a, w, pass);
        LAUNCH_OK();
    }
    return BSPS_OK;
}


// ------------------------------------------------------------------ learned model

struct FitWs {
    float* x;
    int32_t* leafid;
    float* r;
    int32_t* lo;
    float *g, *hs, *lossp, *loss;
};

FitWs carve_fit(Carver& c, i64 N, int L) {
    FitWs f{};
    const i64 N1 = std::max<i64>(1, N);
    f.x = c.take<float>(N1);
    f.leafid = c.take<int32_t>(N1);
    f.r = c.take<float>(N1);
    f.lo = c.take<int32_t>((u64)L + 2);
    f.g = c.take<float>(2 * (u64)L);
    f.hs = c.take<float>(3 * (u64)L);
    f.lossp = c.take<float>(L);
    f.loss = c.take<float>(4);
    return f;
}

// Trains the two-stage model on the sorted sample (root, then leaves):
// forward (residuals), backward (gradient + Gram sums), Newton update, `iters`
// times per stage.
template <typename K>
bsps_status fit_model(const K* smp, i64 N, int dt, int p, int s, int L, int iters, void* model, void* ws,
                      hipStream_t st) {
    Carver c(ws);
    FitWs f = carve_fit(c, N, L);
    // root, leaf ranges, leaves: three launches
    LAUNCH((k_fit_root<K>), dim3(1), dim3(FIT_NT), 0, st, smp, N, dt, p, s, L, iters, model, f.x);
    LAUNCH_OK();
    LAUNCH(k_fit_ranges, dim3((u32)cdiv((u64)N + 1, 256)), dim3(256), 0, st, (const float*)f.x, N,
           (const void*)model, L, f.lo);
    LAUNCH_OK();
    LAUNCH(k_fit_leaves, dim3((u32)cdiv((u64)L, FIT_LEAF_NT / 64)), dim3(FIT_LEAF_NT), 0, st, (const float*)f.x,
           (const int32_t*)f.lo, N, L, p, s, iters, model);
    LAUNCH_OK();
    return BSPS_OK;
}

// ------------------------------------------------------------------ plan

struct Opts {
    u32 cap, tavg;
};

template <typename K>
Opts opts_for(const bsps_params* prm) {
    const u32 T = tileT<K>();
    Opts o{};
    o.cap = (prm && prm->chunk_cap > 0) ? std::min<u32>((u32)prm->chunk_cap, T) : T;
    o.tavg = std::max<u32>(1, o.cap / 4);  // floor of the adaptive chunk target
    return o;
}

template <typename K>
struct Plan {
    bool lsd;                // A1 by LSD radix through HBM (else tiles + multiway merge)
    u32* dbase;              // LSD: digit starts [p][sizeof(K)][256]
    u32* plist;              // LSD: passes of every block [p][sizeof(K) + 1]
    LsdSweep lsw;            // LSD: look-back status, tickets, tiles of every block
    BlockSortBufs<K> bs;     // main block sort
    u32* gsh;                // shift of its truncated tile sort (k_trunc_probe), or NULL
    u32* bsh;                // [1] the block shift D (blocks sorted on key >> D), or NULL
    K* B;
    u32* Bv;
    K* bsmp;                 // block samples (every kSampleStride-th key of each block)
    u32 spb;
    // sample
    i64 ns;
    K* skey;
    u32* spos;
    K* ssk;                  // sorted sample
    u32* ssp;
    K* sscr;
    u32* sscrv;
    BlockSortBufs<K> ss;     // sample sort
    u32* rpos;               // RAN positions and their sorted copy
    u32* rpos_s;
    u32* rpos_scr;
    BlockSortBufs<u32> rs;   // RAN position sort
    // splitters and counts
    K* pk;
    u32* pp;
    u32* pcmp;               // splitter tags the bucket searches compare with (all +inf when untagged)
    u32* cntT;
    MwmBufs<K> bm;           // bucket merge
    // scatter route
    u32* bucket;
    u32* C;
    u32* off;
    // learned
    void* model;
    void* fitws;
    size_t fitws_bytes;
    // iterative rounds (m >= 2): group tables, share samples, sample sorts
    int m, k;
    u32* grp0;
    u32* grp1;
    K* itsmp0;
    K* itsmp1;
    u32 itspb;
    BlockSortBufs<K> its[kMaxRounds];
};

// k with k^m = p (k >= 2), or 0 when p is not an m-th power (m >= 2).
int iter_k(int p, int m) {
    if (m <= 1) return p;
    for (int k = 2; k <= p; k++) {
        u64 v = 1;
        for (int r = 0; r < m && v <= (u64)p; r++) v *= (u64)k;
        if (v == (u64)p) return k;
        if (v > (u64)p) return 0;
    }
    return 0;
}

// Sample slots per share for the shares the non-final rounds produce: every
// kSampleStride-th key of the largest possible share. A sub-bucket of a group
// of z records on q processors holds at most (t + q - 1) x records (Lemma
// balance inside the group: t = q s / k sample ranks per sub-bucket, segments
// of x = ceil(ceil(z/q)/s) keys); a share of the next round is at most
// ceil(that / (q/k)). The merge writes no sample past the slots, so a share
// above the bound would only get a coarser merge plan.
u32 iter_spb(i64 n, int p, int s, int m, int k) {
    u64 z = (u64)n, q = (u64)p, best = 0;
    for (int r = 0; r + 1 < m; r++) {
        const u64 x = cdiv(cdiv(z, q), (u64)s);
        const u64 t = q * (u64)s / (u64)k;
        z = std::min<u64>((u64)n, (t + q - 1) * x);
        q /= (u64)k;
        best = std::max<u64>(best, cdiv(z, q));
    }
    return (u32)std::max<u64>(1, best / kSampleStride);
}

// Which local sort A1 uses (bsps_local_sort). Auto: the tile sort and merge,
// measured faster than the LSD passes on every workload.
template <typename K>
bool use_lsd(i64 n, const bsps_params* prm) {
    if (prm->local_sort == BSPS_LOCAL_LSD) return true;
    if (prm->local_sort == BSPS_LOCAL_MERGE) return false;
    // AUTO: tiles + merge, unless a block has more tiles than a merge group takes runs
    return cdiv(cdiv((u64)n, (u64)prm->p), tileT<K>()) > (u64)MAXR;
}

// Sort_Ran_BSP: the routed array Z (= B), the LSD scratch A and tables, the
// bucket of every key, the sample and its sorts, splitters and counts.
template <typename K>
size_t carve_plan_sr(Carver& c, Plan<K>& P, i64 n, bool hasv, const bsps_params* prm) {
    const int p = prm->p, s = prm->s;
    const Opts o = opts_for<K>(prm);
    P.lsd = true;
    std::memset(&P.bs, 0, sizeof(P.bs));
    P.bs.A = c.take<K>(n);
    P.bs.Av = hasv ? c.take<u32>(n) : nullptr;
    P.dbase = c.take<u32>((u64)p * sizeof(K) * LSD_RADIX);
    P.plist = c.take<u32>((u64)p * (sizeof(K) + 1));
    P.lsw = carve_sweep<K>(c, n, p);
    P.B = c.take<K>(n);
    P.Bv = hasv ? c.take<u32>(n) : nullptr;
    P.spb = 0;
    P.bsmp = nullptr;
    P.ns = (i64)p * s - 1;
    const i64 ns1 = std::max<i64>(1, P.ns);
    P.skey = c.take<K>(ns1);
    P.spos = c.take<u32>(ns1);
    P.ssk = c.take<K>(ns1);
    P.ssp = c.take<u32>(ns1);
    P.sscr = c.take<K>(ns1);
    P.sscrv = c.take<u32>(ns1);
    carve_block_sort<K>(c, P.ss, (u64)ns1, 1, true, o.tavg, false);
    P.rpos = c.take<u32>(ns1);
    P.rpos_s = c.take<u32>(ns1);
    P.rpos_scr = c.take<u32>(ns1);
    carve_block_sort<u32>(c, P.rs, (u64)ns1, 1, false, std::max<u32>(1, opts_for<u32>(prm).tavg), false);
    P.pk = c.take<K>(p);
    P.pp = c.take<u32>(p);
    P.pcmp = prm->untagged ? c.take<u32>(p) : P.pp;
    P.cntT = c.take<u32>((u64)(p + 1) * p);
    std::memset(&P.bm, 0, sizeof(P.bm));
    P.bucket = c.take<u32>(n);
    P.C = c.take<u32>(lstats_off(p) + 4);
    P.off = c.take<u32>((u64)p * p);
    P.model = P.fitws = nullptr;
    P.fitws_bytes = 0;
    if (prm->bucketing == BSPS_LEARNED) {
        const int L = prm->leaves > 0 ? prm->leaves : 4096;
        P.model = c.take<char>(bsps_model_bytes(L));
        P.fitws_bytes = bsps_fit_workspace_bytes(P.ns, L);
        P.fitws = c.take<char>(P.fitws_bytes);
    }
    return c.off + 256;
}

constexpr int kBlockShiftMaxP = 256;

template <typename K>
size_t carve_plan(Carver& c, Plan<K>& P, i64 n, bool hasv, const bsps_params* prm) {
    if (prm->variant == BSPS_RAN_SR) return carve_plan_sr<K>(c, P, n, hasv, prm);
    const int p = prm->p;
    const Opts o = opts_for<K>(prm);
    const bool scatter = prm->route == BSPS_ROUTE_SCATTER;
    P.lsd = use_lsd<K>(n, prm);
    P.dbase = P.plist = nullptr;
    if (P.lsd) {
        // A: pass scratch, then merge scratch / routed array
        std::memset(&P.bs, 0, sizeof(P.bs));
        P.bs.tpb = (int)std::max<u64>(1, cdiv(cdiv((u64)n, (u64)p), tileT<K>()));
        P.bs.A = c.take<K>(n);
        P.bs.Av = hasv ? c.take<u32>(n) : nullptr;
        P.dbase = c.take<u32>((u64)p * sizeof(K) * LSD_RADIX);
        P.plist = c.take<u32>((u64)p * (sizeof(K) + 1));
        P.lsw = carve_sweep<K>(c, n, p);
    } else {
        std::memset(&P.lsw, 0, sizeof(P.lsw));
        carve_block_sort<K>(c, P.bs, (u64)n, p, hasv, o.tavg, true);  // A doubles as merge scratch / routed array
    }
    // the tile shifts of the p blocks, the block shift, the p fine shifts
    P.gsh = (!P.lsd && P.bs.tpb > 1) ? c.take<u32>(2 * (u64)p + 1) : nullptr;
    P.B = c.take<K>(n);
    P.Bv = hasv ? c.take<u32>(n) : nullptr;
    const u64 m = cdiv((u64)n, (u64)p);
    P.spb = (u32)(m / kSampleStride);
    P.bsmp = c.take<K>((u64)p * std::max<u32>(1, P.spb));
    P.ns = prm->variant == BSPS_DET ? (i64)p * prm->s : (i64)p * prm->s - 1;
    const i64 ns1 = std::max<i64>(1, P.ns);
    P.skey = c.take<K>(ns1);
    P.spos = c.take<u32>(ns1);
    P.ssk = c.take<K>(ns1);
    P.ssp = c.take<u32>(ns1);
    P.sscr = c.take<K>(ns1);
    P.sscrv = c.take<u32>(ns1);
    carve_block_sort<K>(c, P.ss, (u64)ns1, 1, true, o.tavg, false);
    P.rpos = P.rpos_s = P.rpos_scr = nullptr;
    std::memset(&P.rs, 0, sizeof(P.rs));
    if (prm->variant == BSPS_RAN) {
        P.rpos = c.take<u32>(ns1);
        P.rpos_s = c.take<u32>(ns1);
        P.rpos_scr = c.take<u32>(ns1);
        carve_block_sort<u32>(c, P.rs, (u64)ns1, 1, false, std::max<u32>(1, opts_for<u32>(prm).tavg), false);
    }
    P.pk = c.take<K>(p);
    P.pp = c.take<u32>(p);
    P.pcmp = prm->untagged ? c.take<u32>(p) : P.pp;
    P.cntT = c.take<u32>((u64)(p + 1) * p);
    carve_mwm<K>(c, P.bm, p, p, (u64)n, o.tavg);
    P.bucket = P.C = P.off = nullptr;
    P.model = P.fitws = nullptr;
    P.fitws_bytes = 0;
    if (scatter) {
        P.bucket = c.take<u32>(n);
        P.C = c.take<u32>(lstats_off(p) + 4);
        P.off = c.take<u32>((u64)p * p);
        if (prm->bucketing == BSPS_LEARNED) {
            const int L = prm->leaves > 0 ? prm->leaves : 4096;
            P.model = c.take<char>(bsps_model_bytes(L));
            P.fitws_bytes = bsps_fit_workspace_bytes(P.ns, L);  // carve_fit layout
            P.fitws = c.take<char>(P.fitws_bytes);
        }
    }
    P.m = prm->rounds >= 2 && p > 1 ? prm->rounds : 1;
    P.k = iter_k(p, P.m);
    // Blocks left sorted on key >> D (the fused route of the one-round sort),
    // for p <= kBlockShiftMaxP: a boundary of the bucket merge then gains about
    // half a group of every one of the p runs, and the splitter groups are
    // fixed by p^2 threads; at p = 1024 (2^28 float keys) that cost more than
    // the block merge saved.
    P.bsh = (P.gsh && !scatter && P.m < 2 && p > 1 && p <= kBlockShiftMaxP) ? P.gsh + p : nullptr;
    P.grp0 = P.grp1 = nullptr;
    P.itsmp0 = P.itsmp1 = nullptr;
    P.itspb = 0;
    if (P.m >= 2) {
        P.grp0 = c.take<u32>((u64)p + 1);
        P.grp1 = c.take<u32>((u64)p + 1);
        P.itspb = iter_spb(n, p, prm->s, P.m, P.k);
        P.itsmp0 = c.take<K>((u64)p * P.itspb);
        P.itsmp1 = c.take<K>((u64)p * P.itspb);
        // round r sorts the p*s sample records as k^r blocks (one per group)
        P.its[0] = P.ss;
        u64 G = 1;
        for (int r = 1; r < P.m; r++) {
            G *= (u64)P.k;
            carve_block_sort<K>(c, P.its[r], (u64)ns1, (int)G, true, o.tavg, false);
        }
    }
    return c.off + 256;
}

bsps_status validate(i64 n, int dtype, const bsps_params* prm) {
    if (!prm) return BSPS_EINVAL;
    if (n < 0 || prm->p < 1 || prm->s < 1) return BSPS_EINVAL;
    if ((i64)prm->p > std::max<i64>(n, 1)) return BSPS_EINVAL;
    if (dtype < 0 || dtype > 2) return BSPS_EINVAL;
    if (prm->variant != BSPS_DET && prm->variant != BSPS_RAN && prm->variant != BSPS_RAN_SR) return BSPS_EINVAL;
    if (prm->route != BSPS_ROUTE_FUSED && prm->route != BSPS_ROUTE_SCATTER) return BSPS_EINVAL;
    if (prm->bucketing != BSPS_SPLITTER && prm->bucketing != BSPS_LEARNED) return BSPS_EINVAL;
    if (prm->leaves < 0 || prm->leaves > MAX_LEAVES || prm->chunk_cap < 0) return BSPS_EINVAL;
    if (prm->local_sort < BSPS_LOCAL_AUTO || prm->local_sort > BSPS_LOCAL_LSD) return BSPS_EINVAL;
    if (prm->untagged != 0 && prm->untagged != 1) return BSPS_EINVAL;
    for (int i = 0; i < 4; i++)
        if (prm->reserved[i]) return BSPS_EINVAL;
    if (prm->rounds < 0 || prm->rounds > kMaxRounds) return BSPS_EINVAL;
    if (prm->rounds >= 2 && prm->p > 1) {
        // the iterative version of Sort_Det_BSP: regular sample, splitter search, fused route
        if (prm->variant != BSPS_DET || prm->route != BSPS_ROUTE_FUSED || prm->bucketing != BSPS_SPLITTER ||
            prm->untagged)
            return BSPS_EINVAL;
        if (iter_k(prm->p, prm->rounds) < 2) return BSPS_EINVAL;
    }
    if (prm->variant != BSPS_DET && (i64)prm->s * prm->p - 1 > n) return BSPS_EINVAL;
    if (n >= (i64)0xFFFFFFFFll || prm->p > kMaxP) return BSPS_EUNSUPPORTED;
    // the merge of a block's tiles takes at most MAXR tiles (AUTO sorts larger
    // blocks by LSD passes, and Sort_Ran_BSP merges no tiles)
    const int kb = key_bytes(dtype);
    const u64 T = kb == 8 ? tileT<u64>() : tileT<u32>();
    if (n > 1 && prm->local_sort == BSPS_LOCAL_MERGE && prm->variant != BSPS_RAN_SR &&
        cdiv(cdiv((u64)n, (u64)prm->p), T) > (u64)MAXR)
        return BSPS_EUNSUPPORTED;
    const i64 ns = prm->variant == BSPS_DET ? (i64)prm->p * prm->s : (i64)prm->p * prm->s - 1;
    if (ns > (i64)MAXR * (i64)T || ns >= (i64)0xFFFFFFFFll) return BSPS_EUNSUPPORTED;
    if (prm->variant == BSPS_RAN_SR && prm->route != BSPS_ROUTE_FUSED) return BSPS_EINVAL;  // it has one route
    return BSPS_OK;
}

// ------------------------------------------------------------------ allocation-free entry point

// Address of `scratch` on the current device, looked up once per device with
// that device current and kept for later calls.
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

bsps_status scratch_base(void** out) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return BSPS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return BSPS_EDEVICE;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return BSPS_OK;
}

// ------------------------------------------------------------------ host conversions (stats)

template <typename K>
K raw_of(K u, int dt);
template <>
u32 raw_of<u32>(u32 u, int dt) {
    if (dt == BSPS_F32) return (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return u ^ 0x80000000u;
}
template <>
u64 raw_of<u64>(u64 u, int dt) { (void)dt; return u ^ 0x8000000000000000ull; }

// Device-to-host copy for the diagnostic paths. It goes through a small
// pinned buffer from hipHostMalloc, chunk by chunk, and never hands a large
// pageable host range to the runtime.
bsps_status d2h(void* host, const void* dev, size_t bytes, hipStream_t st) {
    if (!host || bytes == 0) return BSPS_OK;
    constexpr size_t CH = (size_t)8 << 20;
    void* pin = nullptr;
    HIP_OK(hipHostMalloc(&pin, std::min(bytes, CH), hipHostMallocDefault));
    bsps_status rc = BSPS_OK;
    for (size_t off = 0; off < bytes; off += CH) {
        const size_t b = std::min(CH, bytes - off);
        if (hipMemcpyAsync(pin, (const char*)dev + off, b, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = BSPS_EDEVICE;
            break;
        }
        std::memcpy((char*)host + off, pin, b);
    }
    if (hipHostFree(pin) != hipSuccess && rc == BSPS_OK) rc = BSPS_EDEVICE;
    return rc;
}

// Waits of the tile-parallel passes that hit their spin limit (diagnostic
// calls only: nonzero means the output cannot be trusted).
bsps_status sweep_overruns(const LsdSweep& w, hipStream_t st) {
    if (t_dry || !w.ctr) return BSPS_OK;
    u32 c[2];
    const bsps_status rc = d2h(c, w.ctr, 8, st);
    if (rc) return rc;
    return c[1] ? BSPS_EDEVICE : BSPS_OK;
}

template <typename K>
bsps_status copy_keys_out(void* host, const K* dev, i64 count, int dt, hipStream_t st) {
    if (!host || count <= 0) return BSPS_OK;
    std::vector<K> tmp((size_t)count);
    const bsps_status rc = d2h(tmp.data(), dev, sizeof(K) * (size_t)count, st);
    if (rc) return rc;
    K* h = (K*)host;
    for (i64 i = 0; i < count; i++) h[i] = raw_of<K>(tmp[i], dt);
    return BSPS_OK;
}

bsps_status copy_u32_to_i64(int64_t* host, const u32* dev, i64 count, hipStream_t st) {
    if (!host || count <= 0) return BSPS_OK;
    std::vector<u32> tmp((size_t)count);
    const bsps_status rc = d2h(tmp.data(), dev, sizeof(u32) * (size_t)count, st);
    if (rc) return rc;
    for (i64 i = 0; i < count; i++) host[i] = tmp[i];
    return BSPS_OK;
}

// ------------------------------------------------------------------ the sort

// Sort_Ran_BSP (Section 5.2, Figure SortR): sample the unsorted input, sort
// the sample, pick the splitters, rank every input record (key, position)
// against them (splitter search or the learned model with the exact check),
// route the records to their buckets in input order, then sort every bucket
// (a stable LSD sort through HBM, buckets of any size).
template <typename K, bool HASV>
bsps_status run_sort_sr(void* keys, u32* vals, i64 n, int dt, const bsps_params* prm, void* ws, size_t ws_bytes,
                        hipStream_t st, bsps_stats* stats) {
    const int p = prm->p, s = prm->s;
    Carver c(ws);
    Plan<K> P{};
    const size_t need = carve_plan<K>(c, P, n, HASV, prm);
    if (!ws_ok(ws) || ws_bytes < need) return BSPS_EWORKSPACE;
    const Opts o = opts_for<K>(prm);
    K* io = (K*)keys;
    const i64 ns = P.ns;
    const bool learned = prm->bucketing == BSPS_LEARNED;
    bsps_status rc;
    if (ns > 0) {  // (p = s = 1 draws no sample: one bucket, no splitters)
        StageScope sc(ST_SAMPLE, st);
        // step 2: s*p - 1 input positions without replacement, in position order
        LAUNCH(k_ran_positions, dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, (u64)prm->seed, n, ns, P.rpos);
        LAUNCH_OK();
        const Opts ou = opts_for<u32>(prm);
        rc = block_sort<u32, false>(P.rs, P.rpos, nullptr, BSPS_DT_NONE, P.spos, nullptr, BSPS_DT_NONE, P.rpos_scr,
                                    nullptr, ns, 1, ou.cap, ou.tavg, nullptr, 1, 1, st);
        if (rc) return rc;
        LAUNCH((k_gather_sample_in<K>), dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, io, dt, P.spos, ns, P.skey);
        LAUNCH_OK();
        // steps 5-6: sample sorted by (key, position), splitters at ranks s, 2s, ...
        rc = block_sort<K, true>(P.ss, P.skey, P.spos, BSPS_DT_NONE, P.ssk, P.ssp, BSPS_DT_NONE, P.sscr, P.sscrv, ns, 1,
                                 o.cap, o.tavg, nullptr, 1, 1, st);
        if (rc) return rc;
        LAUNCH((k_splitters<K>), dim3((u32)cdiv(p, 256)), dim3(256), 0, st, P.ssk, P.ssp, p, s, P.pk, P.pp);
        LAUNCH_OK();
        if (prm->untagged) {
            LAUNCH(k_fill_u32, dim3((u32)cdiv(p, 256)), dim3(256), 0, st, P.pcmp, p, 0xFFFFFFFFu);
            LAUNCH_OK();
        }
    }
    {
        // step 9: the bucket of every input record, and the counts C[k][i]
        StageScope sc(ST_COUNT, st);
        if (learned && ns > 0) {
            const int L = prm->leaves > 0 ? prm->leaves : 4096;
            rc = fit_model<K>(P.ssk, ns, BSPS_DT_NONE, p, s, L, 1, P.model, P.fitws, st);
            if (rc) return rc;
        }
        LAUNCH(k_zero_u32, dim3((u32)cdiv(lstats_off(p) + 4, 256)), dim3(256), 0, st, P.C, (int)(lstats_off(p) + 4));
        LAUNCH_OK();
        StageScope sk(ST_RANK_K, st);
        unsigned long long* lst = (unsigned long long*)(P.C + lstats_off(p));
        if (learned && ns > 0)
            rc = launch_rank<K, true>(io, n, p, P.pk, P.pcmp, dt, BSPS_DT_NONE, P.model, P.bucket, P.C, lst, st);
        else
            rc = launch_rank<K, false>(io, n, p, P.pk, P.pcmp, dt, BSPS_DT_NONE, nullptr, P.bucket, P.C, nullptr, st);
        if (rc) return rc;
    }
    {
        // steps 10-11: the p prefix computations, then the order-preserving route
        StageScope sc(ST_TABLES, st);
        LAUNCH(k_counts_to_cntT, dim3(p), dim3(256), 0, st, P.C, p, P.cntT);
        LAUNCH_OK();
        LAUNCH(k_route_offsets, dim3(p), dim3(256), 0, st, P.C, P.cntT, p, P.off);
        LAUNCH_OK();
        static int occ = -1;
        if (!t_dry && occ < 0 &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_route_sr<K, HASV>, SR_NT, 0) != hipSuccess)
            occ = 0;
        const u32 grid = (u32)std::max<i64>(1, std::min<i64>(p, (i64)device_cus() * std::max(occ, 1)));
        const int dbits = std::max(1, (int)bitw((u64)(p - 1)));
        LAUNCH((k_route_sr<K, HASV>), dim3(grid), dim3(SR_NT), 0, st, (const K*)io, (const u32*)vals, dt,
               (const u32*)P.bucket, n, p, dbits, (const u32*)P.off, P.B, P.Bv);
        LAUNCH_OK();
    }
    if (stats && stats->routed) {
        rc = copy_keys_out<K>(stats->routed, P.B, n, dt, st);
        if (rc) return rc;
    }
    if (stats && stats->buckets) {
        rc = d2h(stats->buckets, P.bucket, 4 * (size_t)n, st);
        if (rc) return rc;
    }
    {
        // step 12: every bucket sorted stably: Z -> the caller's buffer, raw keys.
        // Bucket i of Z starts at off[0][i] (block 0's run of it).
        StageScope sc(ST_BUCKET_MERGE, st);
        LsdArgs<K> a{};
        a.in = P.B; a.inv = P.Bv; a.in_dt = BSPS_DT_NONE;
        a.a = P.bs.A; a.av = P.bs.Av; a.b = P.B; a.bv = P.Bv;
        a.out = io; a.outv = vals;
        a.n = n; a.p = p; a.tpb = 0;
        a.dbase = P.dbase; a.plist = P.plist;
        a.smp = nullptr; a.ys = 1; a.spb = 0;
        a.blk = P.off;
        a.out_dt = dt;
        rc = lsd_launch<K, HASV>(a, P.lsw, st);
        if (rc) return rc;
    }
    if (stats) {
        HIP_OK(hipStreamSynchronize(st));
        rc = sweep_overruns(P.lsw, st);
        if (rc) return rc;
        rc = copy_keys_out<K>(stats->splitter_keys, P.pk, p - 1, dt, st);
        if (rc) return rc;
        rc = copy_u32_to_i64(stats->splitter_pos, P.pp, p - 1, st);
        if (rc) return rc;
        rc = copy_keys_out<K>(stats->sample_keys, P.ssk, ns, dt, st);
        if (rc) return rc;
        rc = copy_u32_to_i64(stats->sample_pos, P.ssp, ns, st);
        if (rc) return rc;
        std::vector<u32> ct((size_t)(p + 1) * p);
        rc = d2h(ct.data(), P.cntT, 4 * ct.size(), st);
        if (rc) return rc;
        double mx = 0;
        for (int i = 0; i < p; i++) {
            i64 bsz = 0;
            for (int k = 0; k < p; k++) {
                const i64 cki = (i64)ct[(size_t)(i + 1) * p + k] - (i64)ct[(size_t)i * p + k];
                if (stats->count_matrix) stats->count_matrix[(size_t)k * p + i] = cki;
                bsz += cki;
            }
            if (stats->bucket_sizes) stats->bucket_sizes[i] = bsz;
            mx = std::max(mx, (double)bsz);
        }
        stats->max_bucket_ratio = mx / ((double)n / p);
        stats->oversize_chunks = 0;
        if (learned) {
            unsigned long long ls[2];
            rc = d2h(ls, P.C + lstats_off(p), 16, st);
            if (rc) return rc;
            stats->mispredict_rate = (double)ls[0] / (double)n;
            stats->mean_fix_dist = (double)ls[1] / (double)n;
        }
    }
    return BSPS_OK;
}

// The iterative version of Sort_Det_BSP (Section 5.1), after the local sort
// (B, block samples): m rounds, each splitting every group into k sub-buckets
// and merging every processor's share of them. Round r reads the array the
// previous round wrote (B, then A and B in turn) and the last round writes
// raw keys into the caller's buffer; between rounds that buffer is the
// oversize-chunk scratch of the merge.
template <typename K, bool HASV>
bsps_status run_iter(Plan<K>& P, K* io, u32* vals, i64 n, int dt, const bsps_params* prm, const Opts& o,
                     hipStream_t st, bsps_stats* stats) {
    const int p = prm->p, s = prm->s, m = P.m, k = P.k;
    const i64 ns = (i64)p * s;
    bsps_status rc;
    LAUNCH(k_it_groups_init, dim3(1), dim3(64), 0, st, P.grp0, n);
    LAUNCH_OK();
    const K* src = P.B;
    const u32* srcv = P.Bv;
    const K* smp_in = P.bsmp;
    u32 spb_in = std::max<u32>(1, P.spb);
    u32* grp = P.grp0;
    u32* ngrp = P.grp1;
    int G = 1;
    u32 ctr[4] = {0, 0, 0, 0};
    for (int r = 0; r < m; r++) {
        const int q = p / G;
        const bool last = r == m - 1, even = r % 2 == 0;
        K* dst = last ? io : (even ? P.bs.A : P.B);
        u32* dstv = last ? vals : (even ? P.bs.Av : P.Bv);
        K* scr = last ? (even ? P.bs.A : P.B) : io;
        u32* scrv = last ? (even ? P.bs.Av : P.Bv) : vals;
        K* smp_out = last ? nullptr : (even ? P.itsmp0 : P.itsmp1);
        K* pk = P.pk + (G - 1);  // round r's splitters follow the k^r - 1 of earlier rounds
        u32* pp = P.pp + (G - 1);
        {
            StageScope sc(ST_SAMPLE, st);
            // regular sample of every share, sorted group by group, k - 1 splitters per group
            LAUNCH((k_it_sample<K>), dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, src, n, (const u32*)grp, q, s, ns,
                   P.skey, P.spos);
            LAUNCH_OK();
            rc = block_sort<K, true>(P.its[r], P.skey, P.spos, BSPS_DT_NONE, P.ssk, P.ssp, BSPS_DT_NONE, P.sscr,
                                     P.sscrv, ns, G, o.cap, o.tavg, nullptr, 1, 1, st);
            if (rc) return rc;
            LAUNCH((k_it_splitters<K>), dim3((u32)cdiv((u64)G * (k - 1), 256)), dim3(256), 0, st,
                   (const K*)P.ssk, (const u32*)P.ssp, G, q, s, k, pk, pp);
            LAUNCH_OK();
        }
        if (stats && r == 0) {
            rc = copy_keys_out<K>(stats->sample_keys, P.ssk, ns, dt, st);
            if (rc) return rc;
            rc = copy_u32_to_i64(stats->sample_pos, P.ssp, ns, st);
            if (rc) return rc;
        }
        {
            StageScope sc(ST_COUNT, st);
            LAUNCH((k_it_count<K>), dim3((u32)cdiv((u64)(k + 1) * p, 256)), dim3(256), 0, st, src,
                   (const u32*)grp, p, q, k, (const K*)pk, (const u32*)pp, P.cntT);
            LAUNCH_OK();
        }
        if (stats && stats->count_matrix) {
            std::vector<u32> ct((size_t)(k + 1) * p);
            rc = d2h(ct.data(), P.cntT, 4 * ct.size(), st);
            if (rc) return rc;
            for (int P_ = 0; P_ < p; P_++)
                for (int b = 0; b < k; b++)
                    stats->count_matrix[((size_t)r * p + P_) * k + b] =
                        (i64)ct[(size_t)(b + 1) * p + P_] - (i64)ct[(size_t)b * p + P_];
        }
        {
            StageScope sc(ST_TABLES, st);
            LAUNCH(k_it_tables, dim3((u32)(G * k)), dim3(IT_NT), 0, st, (const u32*)grp, G, p, q, k,
                   (const u32*)P.cntT, kSampleStride, spb_in, ngrp, P.bm.run_start, P.bm.run_len, P.bm.out_base,
                   P.bm.sdesc);
            LAUNCH_OK();
        }
        {
            StageScope sc(ST_BUCKET_MERGE, st);
            MwmArgs<K> a = mwm_args<K>(P.bm, src, srcv, dst, dstv, scr, scrv, smp_in, o.cap, o.tavg,
                                       last ? dt : BSPS_DT_NONE, smp_out, kSampleStride, P.itspb);
            a.R = q;  // run slot j of every share: the piece of source share j of its group
            rc = mwm_run<K, HASV>(a, st, ST_BUCKET_MERGE_K);
            if (rc) return rc;
        }
        if (stats) {
            u32 c4[4];
            rc = d2h(c4, P.bm.counters, 16, st);
            if (rc) return rc;
            ctr[1] += c4[1];
            ctr[3] = std::max(ctr[3], c4[3]);
        }
        src = dst;
        srcv = dstv;
        smp_in = smp_out;
        spb_in = P.itspb;
        std::swap(grp, ngrp);
        G *= k;
    }
    if (stats) {
        HIP_OK(hipStreamSynchronize(st));
        rc = copy_keys_out<K>(stats->splitter_keys, P.pk, p - 1, dt, st);
        if (rc) return rc;
        rc = copy_u32_to_i64(stats->splitter_pos, P.pp, p - 1, st);
        if (rc) return rc;
        std::vector<u32> g((size_t)p + 1);
        rc = d2h(g.data(), grp, 4 * g.size(), st);
        if (rc) return rc;
        double mx = 0;
        for (int i = 0; i < p; i++) {
            const i64 bsz = (i64)g[i + 1] - (i64)g[i];
            if (stats->bucket_sizes) stats->bucket_sizes[i] = bsz;
            mx = std::max(mx, (double)bsz);
        }
        stats->max_bucket_ratio = mx / ((double)n / p);
        u32 ctr2[4] = {0, 0, 0, 0};
        if (!P.lsd && P.bs.tpb > 1) {
            rc = d2h(ctr2, P.bs.mwm.counters, 16, st);
            if (rc) return rc;
        }
        stats->oversize_chunks = (i64)ctr[1] + (i64)ctr2[1];
        stats->reserved_i[0] = ctr2[1];                         // block merge
        stats->reserved_i[1] = ctr[1];                          // the rounds' merges
        stats->reserved_i[2] = (i64)std::max(ctr[3], ctr2[3]);  // largest oversize chunk
    }
    return BSPS_OK;
}

template <typename K, bool HASV>
bsps_status run_sort(void* keys, u32* vals, i64 n, int dt, const bsps_params* prm, void* ws, size_t ws_bytes,
                     hipStream_t st, bsps_stats* stats) {
    if (prm->variant == BSPS_RAN_SR) return run_sort_sr<K, HASV>(keys, vals, n, dt, prm, ws, ws_bytes, st, stats);
    const int p = prm->p, s = prm->s;
    Carver c(ws);
    Plan<K> P{};
    const size_t need = carve_plan<K>(c, P, n, HASV, prm);
    if (!ws_ok(ws) || ws_bytes < need) return BSPS_EWORKSPACE;
    const Opts o = opts_for<K>(prm);
    K* io = (K*)keys;
    bsps_status rc;
    // A1: every virtual processor sorts its block (stable).
    if (P.lsd)
        rc = lsd_block_sort<K, HASV>(io, vals, dt, P.bs.A, P.bs.Av, P.B, P.Bv, P.dbase, P.plist, P.lsw, n, p, P.bs.tpb,
                                     P.bsmp, kSampleStride, P.spb, st);
    else {
        // the shift of the truncated tile sort keeps lg(block) - 2 bits of the key range
        const int keep = std::max(12, bitw(cdiv((u64)n, (u64)p) - 1) - 2);
        rc = block_sort<K, HASV>(P.bs, io, vals, dt, P.B, P.Bv, BSPS_DT_NONE, io, vals, n, p, o.cap, o.tavg, P.bsmp,
                                 kSampleStride, std::max<u32>(1, P.spb), st, ST_TILE, ST_BLOCK_MERGE,
                                 ST_BLOCK_MERGE_K, P.gsh, keep, P.bsh);
    }
    if (rc) return rc;
    if (stats && P.gsh) {
        std::vector<u32> gs((size_t)p + 1);
        rc = d2h(gs.data(), P.gsh, 4 * gs.size(), st);
        if (rc) return rc;
        stats->reserved_i[3] = *std::max_element(gs.begin(), gs.begin() + p);
        if (P.bsh) stats->reserved_i[3] |= (i64)gs[(size_t)p] << 8;
    }
    if (stats && P.lsd) {
        rc = sweep_overruns(P.lsw, st);
        if (rc) return rc;
    }
    if (stats && stats->block_sorted) {
        rc = copy_keys_out<K>(stats->block_sorted, P.B, n, dt, st);
        if (rc) return rc;
    }
    if (stats && stats->block_sorted_values && HASV) {
        rc = d2h(stats->block_sorted_values, P.Bv, 4 * (size_t)n, st);
        if (rc) return rc;
    }
    if (p == 1) {
        LAUNCH((k_copy_out<K>), dim3((u32)cdiv(n, 256)), dim3(256), 0, st, P.B, HASV ? P.Bv : nullptr, io,
                           vals, n, dt);
        LAUNCH_OK();
        if (stats) {
            HIP_OK(hipStreamSynchronize(st));
            if (stats->bucket_sizes) stats->bucket_sizes[0] = n;
            if (stats->count_matrix) stats->count_matrix[0] = n;
            stats->max_bucket_ratio = 1.0;
        }
        return BSPS_OK;
    }
    if (P.m >= 2) return run_iter<K, HASV>(P, io, vals, n, dt, prm, o, st, stats);
    const i64 ns = P.ns;
    {
        StageScope sc(ST_SAMPLE, st);
        // A2: sample records (key, position in B), in position order.
        if (prm->variant == BSPS_DET) {
            LAUNCH((k_det_sample<K>), dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, P.B, n, p, s,
                   (const u32*)P.bsh, P.skey, P.spos);
            LAUNCH_OK();
        } else {
            LAUNCH(k_ran_positions, dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, (u64)prm->seed, n, ns,
                               P.rpos);
            LAUNCH_OK();
            const Opts ou = opts_for<u32>(prm);
            rc = block_sort<u32, false>(P.rs, P.rpos, nullptr, BSPS_DT_NONE, P.spos, nullptr, BSPS_DT_NONE, P.rpos_scr,
                                        nullptr, ns, 1, ou.cap, ou.tavg, nullptr, 1, 1, st);
            if (rc) return rc;
            LAUNCH((k_gather_sample<K>), dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, P.B, n, p,
                   (const u32*)P.bsh, P.spos, ns, P.skey);
            LAUNCH_OK();
        }
        // A3: sort the sample by (key, position): stable by key, input in position order.
        rc = block_sort<K, true>(P.ss, P.skey, P.spos, BSPS_DT_NONE, P.ssk, P.ssp, BSPS_DT_NONE, P.sscr, P.sscrv, ns, 1,
                                 o.cap, o.tavg, nullptr, 1, 1, st);
        if (rc) return rc;
        LAUNCH((k_splitters<K>), dim3((u32)cdiv(p, 256)), dim3(256), 0, st, P.ssk, P.ssp, p, s, P.pk, P.pp);
        LAUNCH_OK();
        if (prm->untagged) {
            // duplicate handling switched off: every splitter compares as (key, +inf)
            LAUNCH(k_fill_u32, dim3((u32)cdiv(p, 256)), dim3(256), 0, st, P.pcmp, p, 0xFFFFFFFFu);
            LAUNCH_OK();
        }
    }
    // A4: bucket boundaries inside every sorted block (splitters searched into it).
    {
        StageScope sc(ST_COUNT, st);
        const u64 ncnt = (u64)(p + 1) * p;
        const bool staged = P.spb > 0 && P.spb <= (u32)COUNT_SMAX;
        if (staged) {
            // (does nothing under a block shift)
            LAUNCH((k_count_staged<K>), dim3(p), dim3(COUNT_NT), 0, st, P.B, n, p, P.pk, P.pcmp, P.bsmp, P.spb,
                   kSampleStride, (const u32*)P.bsh, P.cntT);
            LAUNCH_OK();
        }
        if (P.bsh)  // blocks sorted on key >> D: the splitters' groups made exact as they are counted
            LAUNCH((k_count_fix<K, HASV>), dim3((u32)cdiv(ncnt, 256)), dim3(256), 0, st, P.B, HASV ? P.Bv : nullptr,
                   n, p, (const K*)P.pk, (const u32*)P.pcmp, (const u32*)P.bsh, staged ? 1 : 0, P.cntT);
        else if (!staged)
            LAUNCH((k_count<K>), dim3((u32)cdiv(ncnt, 256)), dim3(256), 0, st, P.B, n, p, P.pk, P.pcmp, P.cntT);
        LAUNCH_OK();
    }
    if (prm->route == BSPS_ROUTE_FUSED) {
        // A5: prefix sums -> runs of every bucket. A6: merge them (routing fused).
        {
            StageScope sc(ST_TABLES, st);
            LAUNCH(k_bucket_tables, dim3(p), dim3(256), 0, st, n, p, P.cntT, kSampleStride,
                   std::max<u32>(1, P.spb), (const u32*)nullptr, P.bm.run_start, P.bm.run_len, P.bm.out_base,
                   P.bm.sdesc);
            LAUNCH_OK();
        }
        {
            StageScope sc(ST_BUCKET_MERGE, st);
            MwmArgs<K> a =
                mwm_args<K>(P.bm, P.B, P.Bv, io, vals, P.bs.A, P.bs.Av, P.bsmp, o.cap, o.tavg, dt, nullptr, 1, 1);
            // runs sorted on key >> D: every bucket cuts them on that part; a
            // group of a block holds about 4 keys (the shift keeps lg(block) - 2
            // bits of its range), so a boundary gains about 2 keys per run
            a.gsh = P.bsh;
            a.gsh_one = 1u;
            a.ggrow = 2u * (u32)p;
            rc = mwm_run<K, HASV>(a, st, ST_BUCKET_MERGE_K);
            if (rc) return rc;
        }
    } else {
        // A5 with A4 per key: the p independent prefix computations, then the
        // routing into Z (= A), every key ranked on its own (splitter search
        // or the learned model with the exact check) as it is moved.
        if (prm->bucketing == BSPS_LEARNED) {
            StageScope sc(ST_COUNT, st);
            const int L = prm->leaves > 0 ? prm->leaves : 4096;
            // one Newton step per stage: the loss of each linear model is quadratic
            rc = fit_model<K>(P.ssk, ns, BSPS_DT_NONE, p, s, L, 1, P.model, P.fitws, st);
            if (rc) return rc;
        }
        {
            StageScope sc(ST_TABLES, st);
            LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, st, P.C + lstats_off(p), 4);
            LAUNCH_OK();
            LAUNCH(k_route_offsets_T, dim3(p), dim3(256), 0, st, P.cntT, p, P.off);
            LAUNCH_OK();
            // per-key bucket ids only for the diagnostic copy
            u32* bids = (stats && stats->buckets) ? P.bucket : nullptr;
            unsigned long long* lst = (unsigned long long*)(P.C + lstats_off(p));
            StageScope sk(ST_RANK_K, st);
            if (prm->bucketing == BSPS_LEARNED) {
                typedef RankShape<true> RS;
                const int wpb = (int)std::max<i64>(1, cdiv((u64)device_cus() * RS::WG_PER_CU * 2, (u64)p));
                LAUNCH((k_scatter_rank<K, true, HASV>), dim3((u32)(p * wpb)), dim3(RS::NT), 0, st, P.B, P.Bv, n, p,
                       wpb, P.pk, P.pcmp, (const void*)P.model, P.cntT, P.off, P.bs.A, P.bs.Av, bids, lst);
            } else {
                typedef RankShape<false> RS;
                const int wpb = (int)std::max<i64>(1, cdiv((u64)device_cus() * RS::WG_PER_CU * 2, (u64)p));
                LAUNCH((k_scatter_rank<K, false, HASV>), dim3((u32)(p * wpb)), dim3(RS::NT), 0, st, P.B, P.Bv, n,
                       p, wpb, P.pk, P.pcmp, (const void*)nullptr, P.cntT, P.off, P.bs.A, P.bs.Av, bids, lst);
            }
            LAUNCH_OK();
        }
        {
            StageScope sc(ST_TABLES, st);
            LAUNCH(k_bucket_tables, dim3(p), dim3(256), 0, st, n, p, P.cntT, kSampleStride,
                   std::max<u32>(1, P.spb), (const u32*)P.off, P.bm.run_start, P.bm.run_len, P.bm.out_base,
                   P.bm.sdesc);
            LAUNCH_OK();
        }
        if (stats && stats->routed) {
            rc = copy_keys_out<K>(stats->routed, P.bs.A, n, dt, st);
            if (rc) return rc;
        }
        if (stats && stats->buckets) {
            rc = d2h(stats->buckets, P.bucket, 4 * (size_t)n, st);
            if (rc) return rc;
        }
        // A6: per-bucket merge of the routed runs (B is free: oversize scratch).
        {
            StageScope sc(ST_BUCKET_MERGE, st);
            MwmArgs<K> a = mwm_args<K>(P.bm, P.bs.A, P.bs.Av, io, vals, P.B, P.Bv, P.bsmp, o.cap, o.tavg, dt,
                                       nullptr, 1, 1);
            rc = mwm_run<K, HASV>(a, st, ST_BUCKET_MERGE_K);
            if (rc) return rc;
        }
    }
    if (stats) {
        HIP_OK(hipStreamSynchronize(st));
        rc = copy_keys_out<K>(stats->splitter_keys, P.pk, p - 1, dt, st);
        if (rc) return rc;
        rc = copy_u32_to_i64(stats->splitter_pos, P.pp, p - 1, st);
        if (rc) return rc;
        rc = copy_keys_out<K>(stats->sample_keys, P.ssk, ns, dt, st);
        if (rc) return rc;
        rc = copy_u32_to_i64(stats->sample_pos, P.ssp, ns, st);
        if (rc) return rc;
        std::vector<u32> ct((size_t)(p + 1) * p);
        rc = d2h(ct.data(), P.cntT, 4 * ct.size(), st);
        if (rc) return rc;
        u32 ctr[4];
        rc = d2h(ctr, P.bm.counters, 16, st);
        if (rc) return rc;
        u32 ctr2[4] = {0, 0, 0, 0};
        if (!P.lsd && P.bs.tpb > 1) {
            rc = d2h(ctr2, P.bs.mwm.counters, 16, st);
            if (rc) return rc;
        }
        double mx = 0;
        for (int i = 0; i < p; i++) {
            i64 bsz = 0;
            for (int k = 0; k < p; k++) {
                const i64 cki = (i64)ct[(size_t)(i + 1) * p + k] - (i64)ct[(size_t)i * p + k];
                if (stats->count_matrix) stats->count_matrix[(size_t)k * p + i] = cki;
                bsz += cki;
            }
            if (stats->bucket_sizes) stats->bucket_sizes[i] = bsz;
            mx = std::max(mx, (double)bsz);
        }
        stats->max_bucket_ratio = mx / ((double)n / p);
        stats->oversize_chunks = (i64)ctr[1] + (i64)ctr2[1];
        stats->reserved_i[0] = ctr2[1];                            // block merge
        stats->reserved_i[1] = ctr[1];                             // bucket merge
        stats->reserved_i[2] = (i64)std::max(ctr[3], ctr2[3]);     // largest oversize chunk
        if (prm->route == BSPS_ROUTE_SCATTER && prm->bucketing == BSPS_LEARNED) {
            unsigned long long ls[2];
            rc = d2h(ls, P.C + lstats_off(p), 16, st);
            if (rc) return rc;
            stats->mispredict_rate = (double)ls[0] / (double)n;
            stats->mean_fix_dist = (double)ls[1] / (double)n;
        }
    }
    return BSPS_OK;
}

template <bool HASV>
bsps_status dispatch_sort(void* keys, u32* vals, i64 n, int dt, const bsps_params* prm, void* ws, size_t ws_bytes,
                          void* stream, bsps_stats* st) {
    bsps_status rc = validate(n, dt, prm);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n <= 1) {
        if (st) {
            if (st->bucket_sizes) st->bucket_sizes[0] = n;
            if (st->count_matrix) st->count_matrix[0] = n;
        }
        return BSPS_OK;
    }
    if (!keys || (HASV && !vals)) return BSPS_EINVAL;
    if (dt == BSPS_I64) return run_sort<u64, HASV>(keys, vals, n, dt, prm, ws, ws_bytes, s, st);
    return run_sort<u32, HASV>(keys, vals, n, dt, prm, ws, ws_bytes, s, st);
}

// ------------------------------------------------------------------ segmented sort (batch)

// Tuning: per size class (segments with n <= 2^max_log2, classes ascending),
// the block size (keys per virtual processor, at most one tile) and the
// oversampling s. p = ceil(n / block); s is clipped so that the segment's
// sample (p*s records) fits one tile.
struct TuneClass {
    int max_log2, block, s;
};
struct Tuning {
    std::vector<TuneClass> cls;
    int learned_log2 = 16;  // segments of more than 2^learned_log2 keys use learned bucketing (>= 32: none)
};

const char* kTuningFormat =
    "{\"classes\": [{\"max_log2\": L, \"block\": B, \"s\": S}, ...]} with classes in ascending L; a segment of n "
    "keys uses the first class with n <= 2^L (the last class beyond). B: keys per virtual processor, "
    "1 <= B <= tile (16384 for 4-byte keys, 8192 for int64); S >= 1 sample records per bucket. Optional "
    "\"learned_above_log2\": G (default 16): segments of more than 2^G keys that are split into blocks get "
    "their bucket counts from a learned model of their sample (G >= 32: never).";

// Built-in table (written by paper_1408_6729_amd/autotune.py on MI355X).
Tuning default_tuning() {
    Tuning t;
    t.cls = {{14, 16384, 1}, {17, 16384, 32}, {20, 16384, 16}, {40, 16384, 8}};
    return t;
}

// Minimal reader for the documented format (integers only).
bool parse_tuning(const char* js, Tuning& t) {
    t.cls.clear();
    if (!js) {
        t = default_tuning();
        return true;
    }
    const std::string s(js);
    {
        const size_t f = s.find("\"learned_above_log2\"");
        if (f != std::string::npos) {
            const size_t colon = s.find(':', f);
            if (colon == std::string::npos) return false;
            char* ep = nullptr;
            const long v = strtol(s.c_str() + colon + 1, &ep, 10);
            if (ep == s.c_str() + colon + 1 || v < 0 || v > 40) return false;
            t.learned_log2 = (int)v;
        }
    }
    size_t pos = s.find("\"classes\"");
    if (pos == std::string::npos) return false;
    pos = s.find('[', pos);
    if (pos == std::string::npos) return false;
    const size_t end = s.find(']', pos);
    if (end == std::string::npos) return false;
    while (true) {
        const size_t ob = s.find('{', pos);
        if (ob == std::string::npos || ob > end) break;
        const size_t cb = s.find('}', ob);
        if (cb == std::string::npos || cb > end) return false;
        const std::string obj = s.substr(ob, cb - ob);
        auto field = [&](const char* name, int& out) {
            const size_t f = obj.find(std::string("\"") + name + "\"");
            if (f == std::string::npos) return false;
            const size_t colon = obj.find(':', f);
            if (colon == std::string::npos) return false;
            char* ep = nullptr;
            const long v = strtol(obj.c_str() + colon + 1, &ep, 10);
            if (ep == obj.c_str() + colon + 1) return false;
            out = (int)v;
            return true;
        };
        TuneClass c;
        if (!field("max_log2", c.max_log2) || !field("block", c.block) || !field("s", c.s)) return false;
        if (c.block < 1 || c.s < 1 || c.max_log2 < 0 || c.max_log2 > 40) return false;
        if (!t.cls.empty() && c.max_log2 <= t.cls.back().max_log2) return false;
        t.cls.push_back(c);
        pos = cb + 1;
    }
    return !t.cls.empty();
}

struct SegPlan {
    int nseg = 0, NB = 0, nmerged = 0, nblocks_s = 0;
    int NL = 0;   // large segments (learned bucketing)
    u32 nls = 0;  // their sample records
    i64 n = 0;
    std::vector<u32> seg, soff, poff, coff, btab, dtab, btab_s;
    std::vector<u32> lseg, lcs, lblk;
    std::vector<std::vector<u32>> gtab;  // per merge class
    std::vector<int> cls_R;
    std::vector<i64> cls_n;
    u32 nbsmp = 0;
};

template <typename K>
bsps_status make_seg_plan(const int64_t* off, int nseg, const Tuning& tu, SegPlan& P) {
    const u32 T = tileT<K>();
    P = SegPlan();
    P.nseg = nseg;
    P.n = nseg ? off[nseg] : 0;
    P.seg.assign((size_t)SEGW * std::max(nseg, 1), 0);
    P.soff.assign(nseg + 1, 0);
    P.poff.assign(nseg + 1, 0);
    P.coff.assign(nseg + 1, 0);
    P.dtab.assign(std::max(nseg, 1), 0);
    std::vector<int> rclass;
    for (int i = 0; i < nseg; i++) {
        const i64 n = off[i + 1] - off[i];
        const TuneClass* c = &tu.cls.back();
        for (auto& cc : tu.cls)
            if (n <= ((i64)1 << cc.max_log2)) { c = &cc; break; }
        const i64 block = std::min<i64>(c->block, T);
        i64 p = std::max<i64>(1, (n + block - 1) / block);
        if (p > MAXR) return BSPS_EUNSUPPORTED;
        if (n <= 1) p = 1;
        i64 s = std::max<i64>(1, std::min<i64>(c->s, T / p));
        u32* d = &P.seg[(size_t)SEGW * i];
        d[0] = (u32)off[i];
        d[1] = (u32)n;
        d[2] = (u32)p;
        d[3] = (u32)s;
        d[4] = (u32)P.NB;
        for (i64 k = 0; k < p; k++) {
            const i64 a = (i64)(((u64)k * (u64)n) / (u64)p), b = (i64)(((u64)(k + 1) * (u64)n) / (u64)p);
            P.btab.push_back((u32)(off[i] + a));
            P.btab.push_back((u32)(b - a));
            P.btab.push_back((u32)i);
            P.btab.push_back(P.nbsmp);
            P.nbsmp += (u32)((b - a) / kSampleStride);
            P.NB++;
        }
        const bool merged = p >= 2;
        P.dtab[i] = merged ? 0u : 1u;
        P.soff[i + 1] = P.soff[i] + (merged ? (u32)(p * s) : 0u);
        P.poff[i + 1] = P.poff[i] + (merged ? (u32)(p - 1) : 0u);
        P.coff[i + 1] = P.coff[i] + (merged ? (u32)((p + 1) * p) : 0u);
        if (merged && tu.learned_log2 < 32 && n > ((i64)1 << tu.learned_log2)) {
            d[5] = 1;
            for (i64 k = 0; k < p; k++) {
                P.lblk.push_back(d[4] + (u32)k);
                P.lblk.push_back((u32)P.NL);
            }
            P.lseg.push_back((u32)i);
            P.NL++;
        }
        if (merged) {
            P.nmerged++;
            P.btab_s.push_back(P.soff[i]);
            P.btab_s.push_back((u32)(p * s));
            P.btab_s.push_back((u32)i);
            P.btab_s.push_back(0);
            int R = 2;
            while (R < p) R <<= 1;
            int ci = -1;
            for (size_t q = 0; q < P.cls_R.size(); q++)
                if (P.cls_R[q] == R) ci = (int)q;
            if (ci < 0) {
                ci = (int)P.cls_R.size();
                P.cls_R.push_back(R);
                P.cls_n.push_back(0);
                P.gtab.emplace_back();
            }
            P.cls_n[ci] += n;
            for (i64 b = 0; b < p; b++) {
                P.gtab[ci].push_back((u32)i);
                P.gtab[ci].push_back((u32)b);
            }
        }
    }
    if (P.btab.empty()) P.btab.assign(4, 0);
    if (P.btab_s.empty()) P.btab_s.assign(4, 0);
    P.lcs.assign(P.NL + 1, 0);
    for (int j = 0; j < P.NL; j++) {
        const u32 sg = P.lseg[j];
        P.lcs[j + 1] = P.lcs[j] + (P.soff[sg + 1] - P.soff[sg]);
    }
    P.nls = P.lcs[P.NL];
    if (P.lseg.empty()) P.lseg.assign(1, 0);
    if (P.lblk.empty()) P.lblk.assign(2, 0);
    return BSPS_OK;
}

template <typename K>
struct SegBufs {
    u32 *seg, *soff, *poff, *coff, *btab, *dtab, *btab_s;
    u32 *lseg, *lcs, *lblk;           // learned bucketing tables
    void* models;                     // learned models of the large segments
    float *fx, *fr, *fg, *fhs;        // their training buffers
    int32_t *fmid, *flo;
    unsigned long long* lst;          // mispredictions, total correction distance
    std::vector<u32*> gtab;
    K *B, *A, *bsmp, *skey, *ssk, *pk;
    u32 *Bv, *Av, *spos, *ssp, *pp, *cntT;
    std::vector<MwmBufs<K>> mw;
    char* tables;
    size_t tables_bytes;
};

template <typename K>
size_t carve_seg(Carver& c, const SegPlan& P, bool hasv, SegBufs<K>& b, u32 tavg) {
    const size_t t0 = (c.off + 255) & ~(size_t)255;
    b.seg = c.take<u32>(P.seg.size());
    b.soff = c.take<u32>(P.soff.size());
    b.poff = c.take<u32>(P.poff.size());
    b.coff = c.take<u32>(P.coff.size());
    b.btab = c.take<u32>(P.btab.size());
    b.dtab = c.take<u32>(P.dtab.size());
    b.btab_s = c.take<u32>(P.btab_s.size());
    b.gtab.clear();
    for (auto& g : P.gtab) b.gtab.push_back(c.take<u32>(g.size()));
    b.lseg = c.take<u32>(P.lseg.size());
    b.lcs = c.take<u32>(P.lcs.size());
    b.lblk = c.take<u32>(P.lblk.size());
    b.tables = c.base ? c.base + t0 : nullptr;
    b.tables_bytes = c.off - t0;
    const i64 n1 = std::max<i64>(1, P.n);
    b.B = c.take<K>(n1);
    b.Bv = hasv ? c.take<u32>(n1) : nullptr;
    b.A = c.take<K>(n1);
    b.Av = hasv ? c.take<u32>(n1) : nullptr;
    b.bsmp = c.take<K>(std::max<u32>(1, P.nbsmp));
    const u32 ns = std::max<u32>(1, P.soff.back());
    b.skey = c.take<K>(ns);
    b.spos = c.take<u32>(ns);
    b.ssk = c.take<K>(ns);
    b.ssp = c.take<u32>(ns);
    b.pk = c.take<K>(std::max<u32>(1, P.poff.back()));
    b.pp = c.take<u32>(std::max<u32>(1, P.poff.back()));
    b.cntT = c.take<u32>(std::max<u32>(1, P.coff.back()));
    {
        const u64 nl = std::max(P.NL, 1), nls = std::max<u32>(P.nls, 1), nm = nl * SEG_LEAVES;
        b.models = c.take<char>(nl * SEG_MODEL_BYTES);
        b.fx = c.take<float>(nls);
        b.fr = c.take<float>(nls);
        b.fmid = c.take<int32_t>(nls);
        b.flo = c.take<int32_t>(nm + 2);
        b.fg = c.take<float>(2 * nm);
        b.fhs = c.take<float>(3 * nm);
        b.lst = c.take<unsigned long long>(2);
    }
    b.mw.assign(P.cls_R.size(), MwmBufs<K>());
    for (size_t q = 0; q < P.cls_R.size(); q++)
        carve_mwm<K>(c, b.mw[q], (int)(P.gtab[q].size() / 2), P.cls_R[q], (u64)P.cls_n[q], tavg);
    return c.off + 256;
}

template <typename K, bool HASV>
bsps_status enqueue_segmented(const SegPlan& P, const SegBufs<K>& b, K* io, u32* vals, int dt, const Opts& o,
                              hipStream_t st) {
    constexpr int NT = Shape<K>::NT;
    if (P.NB == 0) return BSPS_OK;
    TileArgs<K> ta{};
    std::memset(&ta, 0, sizeof(ta));
    ta.in = io; ta.inv = vals; ta.n = P.n; ta.p = 1; ta.tpb = 1; ta.in_dt = dt;
    ta.out = b.B; ta.outv = b.Bv; ta.out_dt = BSPS_DT_NONE; ta.smp = b.bsmp; ta.ys = kSampleStride; ta.spt = 0;
    ta.btab = b.btab; ta.dtab = b.dtab; ta.outd = io; ta.outdv = vals;
    {
        StageScope sc(ST_TILE, st);
        LAUNCH((k_tile_sort<K, HASV, true>), dim3(tile_grid<K, HASV, true>(ta, P.NB)), dim3(NT), 0, st, ta);
        LAUNCH_OK();
    }
    if (P.nmerged == 0) return BSPS_OK;
    const u32 ns = P.soff.back(), np = P.poff.back(), nc = P.coff.back();
    {
        StageScope sc(ST_SAMPLE, st);
        LAUNCH((k_seg_det_sample<K>), dim3((u32)cdiv(ns, 256)), dim3(256), 0, st, b.B, b.seg, b.soff,
                           P.nseg, b.skey, b.spos);
        LAUNCH_OK();
        TileArgs<K> tb{};
        std::memset(&tb, 0, sizeof(tb));
        tb.in = b.skey; tb.inv = b.spos; tb.n = ns; tb.p = 1; tb.tpb = 1; tb.in_dt = BSPS_DT_NONE;
        tb.out = b.ssk; tb.outv = b.ssp; tb.out_dt = BSPS_DT_NONE; tb.smp = nullptr; tb.ys = 1;
        tb.btab = b.btab_s;
        LAUNCH((k_tile_sort<K, true>), dim3(P.nmerged), dim3(NT), 0, st, tb);
        LAUNCH_OK();
        if (np) {
            LAUNCH((k_seg_splitters<K>), dim3((u32)cdiv(np, 256)), dim3(256), 0, st, b.ssk, b.ssp, b.seg,
                               b.soff, b.poff, P.nseg, b.pk, b.pp);
            LAUNCH_OK();
        }
    }
    {
        StageScope sc(ST_COUNT, st);
        LAUNCH((k_seg_count<K>), dim3((u32)cdiv(nc, 256)), dim3(256), 0, st, b.B, b.seg, b.poff, b.coff,
                           P.nseg, b.pk, b.pp, b.cntT);
        LAUNCH_OK();
        if (P.NL > 0) {
            // large segments: train their models on their sorted samples, then
            // rank every key (learned prediction + exact splitter check)
            LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, st, (u32*)b.lst, 4);
            LAUNCH_OK();
            LAUNCH((k_sl_init<K>), dim3((u32)cdiv(P.NL, 64)), dim3(64), 0, st, b.ssk, b.seg, b.soff,
                               b.lseg, P.NL, b.models);
            LAUNCH_OK();
            const u32 gq = (u32)std::max<u64>(1, cdiv(P.nls, 256));
            for (int stage = 0; stage < 2; stage++) {
                const int nmod = stage == 0 ? P.NL : P.NL * SEG_LEAVES;
                LAUNCH((k_sl_x<K>), dim3(gq), dim3(256), 0, st, b.ssk, b.soff, b.lseg, b.lcs, P.NL,
                                   b.models, stage, b.fx, b.fmid);
                LAUNCH_OK();
                LAUNCH(k_model_ranges, dim3((u32)cdiv((u64)nmod + 1, 256)), dim3(256), 0, st, b.fmid,
                                   (i64)P.nls, nmod, b.flo);
                LAUNCH_OK();
                LAUNCH(k_sl_centres, dim3(nmod), dim3(64), 0, st, b.fx, b.flo, nmod, b.models, stage);
                LAUNCH_OK();
                LAUNCH(k_sl_forward, dim3(gq), dim3(256), 0, st, b.fx, b.fmid, b.lcs, P.NL, b.models,
                                   stage, b.fr);
                LAUNCH_OK();
                LAUNCH(k_sl_backward, dim3(nmod), dim3(64), 0, st, b.fx, b.fr, b.flo, nmod, b.lcs,
                                   b.models, stage, b.fg, b.fhs);
                LAUNCH_OK();
                LAUNCH(k_sl_update, dim3((u32)cdiv(nmod, 256)), dim3(256), 0, st, b.fg, b.fhs, b.flo,
                                   nmod, b.lcs, b.models, stage);
                LAUNCH_OK();
            }
            LAUNCH((k_sl_rank<K>), dim3((u32)(P.lblk.size() / 2)), dim3(SL_NT), 0, st, b.B, b.seg,
                               b.btab, b.lblk, b.poff, b.coff, b.pk, b.pp, b.models, b.cntT, b.lst);
            LAUNCH_OK();
        }
    }
    for (size_t q = 0; q < P.cls_R.size(); q++) {
        const int G = (int)(P.gtab[q].size() / 2);
        {
            StageScope sc(ST_TABLES, st);
            LAUNCH(k_seg_bucket_tables, dim3(G), dim3(256), 0, st, b.gtab[q], P.cls_R[q], b.seg, b.coff,
                               b.cntT, b.btab, kSampleStride, b.mw[q].run_start, b.mw[q].run_len, b.mw[q].out_base,
                               b.mw[q].sdesc);
            LAUNCH_OK();
        }
        StageScope sc(ST_BUCKET_MERGE, st);
        MwmArgs<K> a = mwm_args<K>(b.mw[q], b.B, b.Bv, io, vals, b.A, b.Av, b.bsmp, o.cap, o.tavg, dt, nullptr, 1, 1);
        const bsps_status rc = mwm_run<K, HASV>(a, st, ST_BUCKET_MERGE_K);
        if (rc) return rc;
    }
    return BSPS_OK;
}

// Cached graph executables, keyed by everything the captured launches depend on.
// Pinned host buffer the segmented sort's tables are uploaded from. The
// upload is asynchronous on the caller's stream; the next call waits for the
// previous upload (event `done`) before it refills the buffer.
struct TableStage {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
TableStage g_tstage;

bsps_status table_stage(size_t bytes, char** out) {
    if (g_tstage.done) HIP_OK(hipEventSynchronize(g_tstage.done));
    if (!g_tstage.done) {
        const hipError_t e = hipEventCreateWithFlags(&g_tstage.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            g_tstage.done = nullptr;
            return hip_fail(e, "hipEventCreateWithFlags", __LINE__);
        }
    }
    if (g_tstage.cap < bytes) {
        if (g_tstage.p) HIP_OK(hipHostFree(g_tstage.p));
        g_tstage.p = nullptr;
        g_tstage.cap = 0;
        const hipError_t e = hipHostMalloc(&g_tstage.p, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            g_tstage.p = nullptr;
            return hip_fail(e, "hipHostMalloc", __LINE__);
        }
        g_tstage.cap = bytes;
    }
    *out = (char*)g_tstage.p;
    return BSPS_OK;
}

struct GraphCache {
    std::map<std::string, hipGraphExec_t> execs;
    hipStream_t cap = nullptr;
};
GraphCache g_graphs;

std::string graph_key(const void* a, const void* b, const void* c, const int64_t* off, int nseg, int dt, bool hasv,
                      const Tuning& tu) {
    // The whole call signature, byte for byte (no hash: a collision would
    // replay another call's graph).
    std::string k;
    auto put = [&](u64 v) { k.append((const char*)&v, sizeof(v)); };
    put((u64)(uintptr_t)a); put((u64)(uintptr_t)b); put((u64)(uintptr_t)c); put((u64)nseg); put((u64)dt);
    put((u64)hasv);
    put((u64)tu.cls.size());
    put((u64)tu.learned_log2);
    for (auto& cc : tu.cls) { put((u64)cc.max_log2); put((u64)cc.block); put((u64)cc.s); }
    k.append((const char*)off, sizeof(int64_t) * ((size_t)nseg + 1));
    return k;
}

// Dry run: the segmented plan's tables are consistent (every block inside its
// segment and the key array, every group naming a merged segment and one of
// its buckets, every learned-bucketing entry naming a block of a large
// segment, the prefix tables matching the per-segment sizes).
void seg_plan_check(const SegPlan& P, u32 T) {
    auto bad = [&](const char* what, i64 a, i64 b) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "segmented plan: %s (%lld, %lld)", what, (long long)a, (long long)b);
        t_dry->errors.push_back(buf);
    };
    const i64 NB = P.NB;
    if ((i64)P.btab.size() < 4 * NB) bad("block table too short", (i64)P.btab.size(), NB);
    for (int i = 0; i < P.nseg; i++) {
        const u32* d = &P.seg[(size_t)SEGW * i];
        const i64 st = d[0], n = d[1], p = d[2], s = d[3], b0 = d[4];
        if (st + n > P.n) bad("segment past the end", i, st + n);
        if (p < 1 || p > MAXR || s < 1) bad("segment p or s out of range", p, s);
        if (b0 + p > NB) bad("segment blocks past the block table", i, b0 + p);
        i64 cover = st;
        for (i64 k = 0; k < p && b0 + k < NB; k++) {
            const u32* bt = &P.btab[(size_t)4 * (b0 + k)];
            if (bt[0] != cover || bt[1] > T || bt[2] != (u32)i) bad("block not contiguous inside its segment", i, k);
            cover = (i64)bt[0] + bt[1];
            if (bt[3] + bt[1] / kSampleStride > P.nbsmp) bad("block samples past the sample array", i, k);
        }
        if (cover != st + n) bad("blocks do not cover the segment", i, cover);
        const bool merged = p >= 2;
        if (P.soff[i + 1] - P.soff[i] != (merged ? (u32)(p * s) : 0u)) bad("sample prefix", i, P.soff[i + 1]);
        if (P.poff[i + 1] - P.poff[i] != (merged ? (u32)(p - 1) : 0u)) bad("splitter prefix", i, P.poff[i + 1]);
        if (P.coff[i + 1] - P.coff[i] != (merged ? (u32)((p + 1) * p) : 0u)) bad("count prefix", i, P.coff[i + 1]);
        if (P.dtab[i] != (merged ? 0u : 1u)) bad("direct flag", i, P.dtab[i]);
        if (merged && p * s > (i64)T) bad("segment sample larger than one tile", i, p * s);
    }
    for (size_t q = 0; q < P.gtab.size(); q++) {
        for (size_t e = 0; e + 1 < P.gtab[q].size(); e += 2) {
            const u32 sg = P.gtab[q][e], bk = P.gtab[q][e + 1];
            if ((int)sg >= P.nseg) { bad("group of a missing segment", (i64)q, sg); continue; }
            const i64 p = P.seg[(size_t)SEGW * sg + 2];
            if (p < 2 || bk >= p || p > P.cls_R[q]) bad("group bucket out of range", sg, bk);
        }
    }
    for (int j = 0; j < P.NL; j++) {
        const u32 sg = P.lseg[j];
        if ((int)sg >= P.nseg || !P.seg[(size_t)SEGW * sg + 5]) bad("learned entry of a segment not marked large", j, sg);
    }
    for (size_t e = 0; e + 1 < P.lblk.size() && P.NL > 0; e += 2)
        if ((i64)P.lblk[e] >= NB || (i64)P.lblk[e + 1] >= P.NL) bad("learned block entry out of range", (i64)P.lblk[e], P.lblk[e + 1]);
}

template <typename K, bool HASV>
bsps_status run_segmented(void* keys, u32* vals, const int64_t* off, int nseg, int dt, const Tuning& tu, void* ws,
                          size_t ws_bytes, hipStream_t st, bsps_stats* stats) {
    SegPlan P{};
    bsps_status rc = make_seg_plan<K>(off, nseg, tu, P);
    if (rc) return rc;
    bsps_params dp;
    std::memset(&dp, 0, sizeof(dp));
    const Opts o = opts_for<K>(&dp);
    SegBufs<K> b{};
    Carver c(ws);
    const size_t need = carve_seg<K>(c, P, HASV, b, o.tavg);
    if (!ws_ok(ws) || ws_bytes < need) return BSPS_EWORKSPACE;
    if (P.NB == 0) return BSPS_OK;
    if (t_dry) {
        // the plan's host tables index inside their arrays, the upload fits
        // the workspace, and then every launch of the eager enqueue is checked
        seg_plan_check(P, tileT<K>());
        t_dry->kernel = "segment table upload";
        t_dry->span("tables", b.tables, b.tables_bytes);
        return enqueue_segmented<K, HASV>(P, b, (K*)keys, vals, dt, o, st);
    }
    // tables -> workspace (pinned host staging in carve order, asynchronous)
    {
        char* stage = nullptr;
        rc = table_stage(b.tables_bytes, &stage);
        if (rc) return rc;
        std::memset(stage, 0, b.tables_bytes);
        Carver hc(stage);
        auto put = [&](const std::vector<u32>& v) {
            u32* d = hc.take<u32>(v.size());
            std::memcpy(d, v.data(), v.size() * sizeof(u32));
        };
        put(P.seg); put(P.soff); put(P.poff); put(P.coff); put(P.btab); put(P.dtab); put(P.btab_s);
        for (auto& g : P.gtab) put(g);
        put(P.lseg); put(P.lcs); put(P.lblk);
        HIP_OK(hipMemcpyAsync(b.tables, stage, b.tables_bytes, hipMemcpyHostToDevice, st));
        HIP_OK(hipEventRecord(g_tstage.done, st));
    }
    // capture every launch into one graph (on a private stream), launch it once
    (void)device_cus();  // device queries stay outside the graph capture
    const bool timed = g_timer.on;
    bool launched = false, cached = false;
    if (!timed && getenv("BSPS_NO_GRAPH") == nullptr) {
        const std::string key = graph_key(keys, vals, ws, off, nseg, dt, HASV, tu);
        auto it = g_graphs.execs.find(key);
        hipGraphExec_t exec = nullptr;
        if (it != g_graphs.execs.end()) {
            exec = it->second;
            cached = true;
        } else {
            if (!g_graphs.cap && hipStreamCreateWithFlags(&g_graphs.cap, hipStreamNonBlocking) != hipSuccess)
                g_graphs.cap = nullptr;
            hipGraph_t graph = nullptr;
            if (g_graphs.cap && hipStreamBeginCapture(g_graphs.cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const bsps_status erc = enqueue_segmented<K, HASV>(P, b, (K*)keys, vals, dt, o, g_graphs.cap);
                const hipError_t ec = hipStreamEndCapture(g_graphs.cap, &graph);
                hipError_t ei = hipErrorUnknown;
                if (erc == BSPS_OK && ec == hipSuccess && graph &&
                    (ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) == hipSuccess) {
                    g_graphs.execs[key] = exec;
                } else {
                    if (debug_on())
                        std::fprintf(stderr, "[bsps] graph capture not used (enqueue %d, end capture %s, "
                                     "instantiate %s); running eagerly\n", (int)erc, hipGetErrorString(ec),
                                     hipGetErrorString(ei));
                    exec = nullptr;
                }
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
            }
        }
        if (exec) {
            HIP_OK(hipGraphLaunch(exec, st));
            launched = true;
        }
    }
    if (!launched) {
        rc = enqueue_segmented<K, HASV>(P, b, (K*)keys, vals, dt, o, st);
        if (rc) return rc;
    }
    if (stats) {
        HIP_OK(hipStreamSynchronize(st));
        i64 over = 0;
        for (auto& m : b.mw) {
            u32 ctr[2];
            rc = d2h(ctr, m.counters, 8, st);
            if (rc) return rc;
            over += ctr[1];
        }
        stats->oversize_chunks = over;
        stats->reserved_i[0] = P.NB;
        stats->reserved_i[1] = P.nmerged;
        stats->reserved_i[2] = launched ? (cached ? 2 : 1) : 0;
        stats->reserved_i[3] = P.NL;
        stats->mispredict_rate = 0.0;
        stats->mean_fix_dist = 0.0;
        if (P.NL > 0 && stats->seg_capacity >= P.NL) {
            rc = d2h(stats->seg_models, b.models, (size_t)P.NL * SEG_MODEL_BYTES, st);
            if (rc) return rc;
            rc = d2h(stats->seg_grad, b.fg, sizeof(float) * 2 * (size_t)P.NL * SEG_LEAVES, st);
            if (rc) return rc;
            rc = d2h(stats->seg_gram, b.fhs, sizeof(float) * 3 * (size_t)P.NL * SEG_LEAVES, st);
            if (rc) return rc;
        }
        if (P.NL > 0) {
            unsigned long long ls[2];
            rc = d2h(ls, b.lst, 16, st);
            if (rc) return rc;
            i64 nlk = 0;  // keys ranked by the models
            for (int j = 0; j < P.NL; j++) nlk += P.seg[(size_t)SEGW * P.lseg[j] + 1];
            stats->mispredict_rate = (double)ls[0] / (double)std::max<i64>(1, nlk);
            stats->mean_fix_dist = (double)ls[1] / (double)std::max<i64>(1, nlk);
        }
    }
    return BSPS_OK;
}

bsps_status validate_segments(const int64_t* off, int nseg, int dtype, const char* tuning_json, Tuning& tu) {
    if (nseg < 0 || dtype < 0 || dtype > 2 || (nseg > 0 && !off)) return BSPS_EINVAL;
    if (!parse_tuning(tuning_json, tu)) return BSPS_EINVAL;
    if (nseg == 0) return BSPS_OK;
    if (off[0] != 0) return BSPS_EINVAL;
    for (int i = 0; i < nseg; i++)
        if (off[i + 1] < off[i]) return BSPS_EINVAL;
    if (off[nseg] >= (int64_t)0xFFFFFFFFll) return BSPS_EUNSUPPORTED;
    return BSPS_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

size_t bsps_workspace_bytes(int64_t n, int32_t dtype, int32_t with_values, const bsps_params* prm) {
    if (validate(n, dtype, prm) != BSPS_OK) return 0;
    if (n <= 1) return 256;
    Carver c(nullptr);
    if (dtype == BSPS_I64) {
        Plan<u64> P;
        return carve_plan<u64>(c, P, n, with_values != 0, prm);
    }
    Plan<u32> P;
    return carve_plan<u32>(c, P, n, with_values != 0, prm);
}

bsps_status bsps_sort(void* keys, int64_t n, int32_t dtype, const bsps_params* prm, void* ws, size_t ws_bytes,
                      void* stream, bsps_stats* st) {
    return dispatch_sort<false>(keys, nullptr, n, dtype, prm, ws, ws_bytes, stream, st);
}

bsps_status bsps_sort_kv(void* keys, uint32_t* values, int64_t n, int32_t dtype, const bsps_params* prm, void* ws,
                         size_t ws_bytes, void* stream, bsps_stats* st) {
    return dispatch_sort<true>(keys, values, n, dtype, prm, ws, ws_bytes, stream, st);
}

bsps_status bsps_sort_noalloc(void* keys, uint32_t* values, int64_t n, int32_t dtype, const bsps_params* prm,
                              void* stream) {
    bsps_status rc = validate(n, dtype, prm);
    if (rc) return rc;
    if (n <= 1) return BSPS_OK;
    if (!keys) return BSPS_EINVAL;
    const size_t need = bsps_workspace_bytes(n, dtype, values != nullptr, prm);
    if (need == 0) return BSPS_EINVAL;
    if (need > BSPS_NOALLOC_SCRATCH_BYTES) return BSPS_EUNSUPPORTED;
    void* ws = nullptr;
    rc = scratch_base(&ws);
    if (rc) return rc;
    // the sort clears every counter it reads before use, so the previous
    // call's contents of the scratch do not matter
    t_no_events = true;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == BSPS_I64)
        rc = values ? run_sort<u64, true>(keys, values, n, dtype, prm, ws, BSPS_NOALLOC_SCRATCH_BYTES, s, nullptr)
                    : run_sort<u64, false>(keys, nullptr, n, dtype, prm, ws, BSPS_NOALLOC_SCRATCH_BYTES, s, nullptr);
    else
        rc = values ? run_sort<u32, true>(keys, values, n, dtype, prm, ws, BSPS_NOALLOC_SCRATCH_BYTES, s, nullptr)
                    : run_sort<u32, false>(keys, nullptr, n, dtype, prm, ws, BSPS_NOALLOC_SCRATCH_BYTES, s, nullptr);
    t_no_events = false;
    return rc;
}

size_t bsps_fit_workspace_bytes(int64_t N, int32_t leaves) {
    Carver c(nullptr);
    (void)carve_fit(c, N, leaves > 0 ? leaves : 4096);
    return c.off + 256;
}

size_t bsps_rank_workspace_bytes(int64_t n, int32_t p) {
    (void)n;
    (void)p;
    return 256;
}

bsps_status bsps_rank(const void* keys, int64_t n, int32_t dtype, int32_t p, const void* spl_keys,
                      const uint32_t* spl_pos, int32_t bucketing, const void* model, uint32_t* out_bucket,
                      uint32_t* out_counts, void* ws, size_t ws_bytes, void* stream, bsps_stats* st) {
    if (n < 0 || p < 1 || (i64)p > std::max<i64>(n, 1) || dtype < 0 || dtype > 2) return BSPS_EINVAL;
    if (bucketing != BSPS_SPLITTER && bucketing != BSPS_LEARNED) return BSPS_EINVAL;
    if (bucketing == BSPS_LEARNED && !model) return BSPS_EINVAL;
    if (p > kMaxP || n >= (i64)0xFFFFFFFFll) return BSPS_EUNSUPPORTED;
    if (n > 0 && (!keys || (p > 1 && (!spl_keys || !spl_pos)))) return BSPS_EINVAL;
    if (!ws_ok(ws) || ws_bytes < bsps_rank_workspace_bytes(n, p)) return BSPS_EWORKSPACE;
    if (n == 0) return BSPS_OK;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* lst = (unsigned long long*)ws;
    LAUNCH(k_zero_u32, dim3(1), dim3(64), 0, s, (u32*)ws, 4);
    LAUNCH_OK();
    if (out_counts) {
        LAUNCH(k_zero_u32, dim3((u32)cdiv((u64)p * p, 256)), dim3(256), 0, s, out_counts, p * p);
        LAUNCH_OK();
    }
    {
        StageScope sc(ST_RANK_K, s);
        // keys and splitters arrive in dtype form; the kernel maps both to order keys
        bsps_status rc;
        if (dtype == BSPS_I64) {
            if (bucketing == BSPS_LEARNED)
                rc = launch_rank<u64, true>((const u64*)keys, n, p, (const u64*)spl_keys, spl_pos, dtype, dtype, model,
                                            out_bucket, out_counts, lst, s);
            else
                rc = launch_rank<u64, false>((const u64*)keys, n, p, (const u64*)spl_keys, spl_pos, dtype, dtype, model,
                                             out_bucket, out_counts, lst, s);
        } else {
            if (bucketing == BSPS_LEARNED)
                rc = launch_rank<u32, true>((const u32*)keys, n, p, (const u32*)spl_keys, spl_pos, dtype, dtype, model,
                                            out_bucket, out_counts, lst, s);
            else
                rc = launch_rank<u32, false>((const u32*)keys, n, p, (const u32*)spl_keys, spl_pos, dtype, dtype, model,
                                             out_bucket, out_counts, lst, s);
        }
        if (rc) return rc;
    }
    if (st) {
        unsigned long long h[2];
        const bsps_status rc = d2h(h, lst, 16, s);
        if (rc) return rc;
        st->mispredict_rate = (double)h[0] / (double)n;
        st->mean_fix_dist = (double)h[1] / (double)n;
    }
    return BSPS_OK;
}

bsps_status bsps_fit_model(const void* smp_keys, int64_t N, int32_t dtype, int32_t p, int32_t s, int32_t leaves,
                           int32_t iters, void* model, void* ws, size_t ws_bytes, void* stream) {
    if (N < 1 || p < 1 || s < 1 || leaves < 1 || leaves > MAX_LEAVES || iters < 1 || dtype < 0 || dtype > 2 ||
        !smp_keys || !model)
        return BSPS_EINVAL;
    if (!ws_ok(ws) || ws_bytes < bsps_fit_workspace_bytes(N, leaves)) return BSPS_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == BSPS_I64) return fit_model<u64>((const u64*)smp_keys, N, dtype, p, s, leaves, iters, model, ws, st);
    return fit_model<u32>((const u32*)smp_keys, N, dtype, p, s, leaves, iters, model, ws, st);
}

bsps_status bsps_model_grad(const void* smp_keys, int64_t N, int32_t dtype, int32_t p, int32_t s, int32_t leaves,
                            const void* model, int32_t* out_leaf, float* out_grad, float* out_gram, float* out_loss,
                            void* ws, size_t ws_bytes, void* stream) {
    if (N < 1 || p < 1 || s < 1 || leaves < 1 || leaves > MAX_LEAVES || dtype < 0 || dtype > 2 || !smp_keys || !model ||
        !out_leaf || !out_grad || !out_gram || !out_loss)
        return BSPS_EINVAL;
    if (!ws_ok(ws) || ws_bytes < bsps_fit_workspace_bytes(N, leaves)) return BSPS_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carver c(ws);
    FitWs f = carve_fit(c, N, leaves);
    const u32 gN = (u32)std::max<u64>(1, cdiv((u64)N, 256));
    if (dtype == BSPS_I64)
        LAUNCH((k_model_x<u64>), dim3(gN), dim3(256), 0, st, (const u64*)smp_keys, N, dtype, model, 1,
                           f.x, out_leaf);
    else
        LAUNCH((k_model_x<u32>), dim3(gN), dim3(256), 0, st, (const u32*)smp_keys, N, dtype, model, 1,
                           f.x, out_leaf);
    LAUNCH_OK();
    // leaf ranges and the forward / backward pass of the fit, at the given parameters
    LAUNCH(k_fit_ranges, dim3((u32)cdiv((u64)N + 1, 256)), dim3(256), 0, st, (const float*)f.x, N, model, leaves,
           f.lo);
    LAUNCH_OK();
    LAUNCH(k_grad_leaves, dim3((u32)cdiv((u64)leaves, FIT_LEAF_NT / 64)), dim3(FIT_LEAF_NT), 0, st,
           (const float*)f.x, (const int32_t*)f.lo, N, leaves, p, s, model, out_grad, out_gram, f.lossp);
    LAUNCH_OK();
    LAUNCH(k_sum_loss, dim3(1), dim3(256), 0, st, f.lossp, leaves, N, out_loss);
    LAUNCH_OK();
    return BSPS_OK;
}

size_t bsps_segmented_workspace_bytes(const int64_t* h_offsets, int32_t nseg, int32_t dtype, int32_t with_values,
                                      const char* tuning_json) {
    Tuning tu;
    if (validate_segments(h_offsets, nseg, dtype, tuning_json, tu) != BSPS_OK) return 0;
    SegPlan P{};
    bsps_params dp;
    std::memset(&dp, 0, sizeof(dp));
    Carver c(nullptr);
    if (dtype == BSPS_I64) {
        if (make_seg_plan<u64>(h_offsets, nseg, tu, P) != BSPS_OK) return 0;
        SegBufs<u64> b{};
        return carve_seg<u64>(c, P, with_values != 0, b, opts_for<u64>(&dp).tavg);
    }
    if (make_seg_plan<u32>(h_offsets, nseg, tu, P) != BSPS_OK) return 0;
    SegBufs<u32> b{};
    return carve_seg<u32>(c, P, with_values != 0, b, opts_for<u32>(&dp).tavg);
}

bsps_status bsps_sort_segmented(void* keys, uint32_t* values, const int64_t* h_offsets, int32_t nseg, int32_t dtype,
                                const char* tuning_json, void* ws, size_t ws_bytes, void* stream, bsps_stats* st) {
    Tuning tu;
    bsps_status rc = validate_segments(h_offsets, nseg, dtype, tuning_json, tu);
    if (rc) return rc;
    if (nseg == 0 || h_offsets[nseg] == 0) return BSPS_OK;
    if (!keys) return BSPS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == BSPS_I64)
        return values ? run_segmented<u64, true>(keys, values, h_offsets, nseg, dtype, tu, ws, ws_bytes, s, st)
                      : run_segmented<u64, false>(keys, values, h_offsets, nseg, dtype, tu, ws, ws_bytes, s, st);
    return values ? run_segmented<u32, true>(keys, values, h_offsets, nseg, dtype, tu, ws, ws_bytes, s, st)
                  : run_segmented<u32, false>(keys, values, h_offsets, nseg, dtype, tu, ws, ws_bytes, s, st);
}

const char* bsps_tuning_format(void) { return kTuningFormat; }

const char* bsps_status_string(int32_t status) {
    switch (status) {
        case BSPS_OK: return "ok";
        case BSPS_EINVAL: return "invalid argument";
        case BSPS_EWORKSPACE: return "workspace missing or too small";
        case BSPS_EDEVICE: return "HIP device error";
        case BSPS_EUNSUPPORTED: return "outside the library limits";
        default: return "unknown status";
    }
}

bsps_status bsps_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return BSPS_EINVAL;
    if (bytes == 0) return BSPS_OK;
    const u64 n16 = bytes / 16;
    const u64 grid = cdiv(n16, (u64)COPY_NT * COPY_PER);
    if (grid > 0x7fffffffull) return BSPS_EUNSUPPORTED;
    LAUNCH(k_stream_copy, dim3((u32)grid), dim3(COPY_NT), 0, (hipStream_t)stream, (const v4u32*)src,
                       (v4u32*)dst, n16);
    LAUNCH_OK();
    return BSPS_OK;
}

// Dry runs: report the checks' findings into `report` (HOST, may be NULL).
static int64_t dry_finish(DryRun& d, bsps_status rc, char* report, size_t report_len) {
    t_dry = nullptr;
    if (rc != BSPS_OK) return -(int64_t)rc;
    if (report && report_len) {
        std::string r;
        for (auto& e : d.errors) r += e + "\n";
        if (d.errors.empty()) r = "ok: " + std::to_string(d.launches) + " launches checked\n";
        std::snprintf(report, report_len, "%s", r.c_str());
    }
    return (int64_t)d.errors.size();
}

static void* const kFakeKeys = (void*)(uintptr_t)0x100000000000ull;
static void* const kFakeVals = (void*)(uintptr_t)0x200000000000ull;
static void* const kFakeWs = (void*)(uintptr_t)0x300000000000ull;

int64_t bsps_check_sort(int64_t n, int32_t dtype, int32_t with_values, const bsps_params* prm, char* report,
                        size_t report_len) {
    bsps_status rc = validate(n, dtype, prm);
    if (rc) return -(int64_t)rc;
    DryRun d;
    if (n <= 1) return dry_finish(d, BSPS_OK, report, report_len);
    const size_t ws_bytes = bsps_workspace_bytes(n, dtype, with_values, prm);
    d.add(kFakeKeys, (size_t)n * key_bytes(dtype));
    if (with_values) d.add(kFakeVals, (size_t)n * 4);
    d.add(kFakeWs, ws_bytes);
    u32* vals = with_values ? (u32*)kFakeVals : nullptr;
    t_dry = &d;
    if (dtype == BSPS_I64)
        rc = with_values ? run_sort<u64, true>(kFakeKeys, vals, n, dtype, prm, kFakeWs, ws_bytes, nullptr, nullptr)
                         : run_sort<u64, false>(kFakeKeys, vals, n, dtype, prm, kFakeWs, ws_bytes, nullptr, nullptr);
    else
        rc = with_values ? run_sort<u32, true>(kFakeKeys, vals, n, dtype, prm, kFakeWs, ws_bytes, nullptr, nullptr)
                         : run_sort<u32, false>(kFakeKeys, vals, n, dtype, prm, kFakeWs, ws_bytes, nullptr, nullptr);
    return dry_finish(d, rc, report, report_len);
}

int64_t bsps_check_segmented(const int64_t* h_offsets, int32_t nseg, int32_t dtype, int32_t with_values,
                             const char* tuning_json, char* report, size_t report_len) {
    Tuning tu;
    bsps_status rc = validate_segments(h_offsets, nseg, dtype, tuning_json, tu);
    if (rc) return -(int64_t)rc;
    DryRun d;
    if (nseg == 0 || h_offsets[nseg] == 0) return dry_finish(d, BSPS_OK, report, report_len);
    const i64 n = h_offsets[nseg];
    const size_t ws_bytes = bsps_segmented_workspace_bytes(h_offsets, nseg, dtype, with_values, tuning_json);
    d.add(kFakeKeys, (size_t)n * key_bytes(dtype));
    if (with_values) d.add(kFakeVals, (size_t)n * 4);
    d.add(kFakeWs, ws_bytes);
    u32* vals = with_values ? (u32*)kFakeVals : nullptr;
    t_dry = &d;
    if (dtype == BSPS_I64)
        rc = with_values ? run_segmented<u64, true>(kFakeKeys, vals, h_offsets, nseg, dtype, tu, kFakeWs, ws_bytes,
                                                    nullptr, nullptr)
                         : run_segmented<u64, false>(kFakeKeys, vals, h_offsets, nseg, dtype, tu, kFakeWs, ws_bytes,
                                                     nullptr, nullptr);
    else
        rc = with_values ? run_segmented<u32, true>(kFakeKeys, vals, h_offsets, nseg, dtype, tu, kFakeWs, ws_bytes,
                                                    nullptr, nullptr)
                         : run_segmented<u32, false>(kFakeKeys, vals, h_offsets, nseg, dtype, tu, kFakeWs, ws_bytes,
                                                     nullptr, nullptr);
    return dry_finish(d, rc, report, report_len);
}

void bsps_release_cache(void) {
    for (auto& kv : g_graphs.execs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.execs.clear();
    if (g_graphs.cap) (void)hipStreamDestroy(g_graphs.cap);
    g_graphs.cap = nullptr;
    if (g_tstage.done) {
        (void)hipEventSynchronize(g_tstage.done);
        (void)hipEventDestroy(g_tstage.done);
    }
    if (g_tstage.p) (void)hipHostFree(g_tstage.p);
    g_tstage = TableStage();
}

int bsps_timing(int enable) {
    g_timer.on = enable != 0;
    return BSPS_OK;
}

int bsps_timing_read(double* ms, int64_t* launches, int nstage, int reset) {
    for (int sg = 0; sg < ST_N; sg++) {
        double acc = 0;
        for (auto& pr : g_timer.ev[sg]) {
            float t = 0;
            if (hipEventSynchronize(pr.second) != hipSuccess) return BSPS_EDEVICE;
            if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess) return BSPS_EDEVICE;
            acc += t;
        }
        if (sg < nstage) {
            if (ms) ms[sg] = acc;
            if (launches) launches[sg] = (int64_t)g_timer.ev[sg].size();
        }
        if (reset) {
            for (auto& pr : g_timer.ev[sg]) {
                g_timer.pool.push_back(pr.first);
                g_timer.pool.push_back(pr.second);
            }
            g_timer.ev[sg].clear();
        }
    }
    return BSPS_OK;
}

#ifdef BSPS_TIMING
int bsps_debug_phases(unsigned long long* out, int reset) {
    unsigned long long h[16];
    if (hipMemcpyFromSymbol(h, HIP_SYMBOL(g_phase), sizeof(h)) != hipSuccess) return 1;
    for (int i = 0; i < 16; i++) out[i] = h[i];
    if (reset) {
        unsigned long long z[16] = {0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z)) != hipSuccess) return 1;
    }
    return 0;
}
#endif

}  // extern "C"
