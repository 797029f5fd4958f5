// Host side of the DFR sort: context, planner, level orchestration and the C ABI
// declared in include/dfr.h.
//
// One sort runs as a sequence of *levels* (Sec. 3: DFR recurses on large buckets).
// A level takes a list of segments -- ranges whose keys agree on every bit at and
// above the segment's hi_bit -- that all sit in the same buffer (the caller's or the
// temp buffer), and:
//   1. counts every 8-bit digit of every segment in one read (k_count), with the OR
//      and AND of the segment's keys, and reads the OR/AND back;
//   2. plans: digits that never vary inside a segment are skipped (Sec. 2.1 pass
//      skipping); the number d of top varying digits to deal is estimated so that the
//      expected bucket falls below the diversion threshold N_d (Sec. 3, Sec. 3.1);
//   3. deals those d digits least significant first (k_deal, ping-pong between the
//      two buffers);
//   4. finds the buckets of equal leading bits (k_heads), packs runs of small buckets
//      into local-sort chunks and lists large buckets (k_classify);
//   5. sorts every chunk inside LDS and writes it into the caller's buffer
//      (k_local_sort, the diversion);
//   6. reads back the large buckets, which become the next level's segments.
// Segments no larger than the local sort's capacity skip steps 1-4 and go straight to
// step 5.  The result always ends in the caller's buffers (Sec. 2.1: the last deal
// lands in the original space).
#include "dfr.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dfr_internal.h"

using namespace dfr;

namespace {

constexpr size_t ALIGN = 256;
static_assert((STAT_WORDS + LEVEL_WORDS) * 4 <= ALIGN, "status block and level counters fit one allocation");
inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct LSeg {
    uint64_t start;
    uint64_t len;
    int hi_bit;
};

enum Stage { ST_COUNT = 0, ST_DEAL, ST_BUCKETS, ST_LOCAL, ST_OTHER, ST_N };

// Largest segment, in tiles, whose bucket bases one block scans ahead of the deal.
constexpr uint64_t kSegScanTiles = 1024;
// Longest single segment (in tiles) whose bases one block walks.
constexpr uint64_t kSingleWalkTiles = 256;
// Most segments of a level whose tiles are scanned segment by segment with the
// one-segment scan when some segment is longer than kSegScanTiles.
constexpr size_t kPerSegScanMax = 16;
// Top digits with at most this many non-empty bins count as a skewed prefix.
constexpr uint32_t kFewTopValues = 16;
// Pinned host staging reserved by dfr_create (the allocation-free entry point's whole
// staging: tile and segment lists, plan and bucket read-backs of one level).
constexpr size_t kNoallocPinBytes = size_t(4) << 20;

}  // namespace

struct dfr_ctx {
    int device = 0;
    size_t budget = 0;
    bool failed = false;
    std::string err;

    uint32_t* err_dev = nullptr;  // device error word of the current call
    // Device scratch arena (bump allocation, reset per level).
    char* arena = nullptr;
    size_t arena_cap = 0;
    size_t arena_used = 0;
    // Cached temp buffer for calls with temp == NULL.
    void* tcache = nullptr;
    size_t tcache_cap = 0;
    size_t temp_slack = 0;   // extra fraction (in 1/8) allocated when the cache grows
    // Device (re)allocations made and host time spent in them.
    uint64_t n_allocs = 0;
    double ms_alloc = 0;
    // Pinned host staging (bump allocation, reset after each stream synchronisation).
    char* pin = nullptr;
    size_t pin_cap = 0;
    size_t pin_used = 0;
    // The allocation-free entry point: this device's fixed scratch array, and whether
    // the current call runs on it (then nothing may be allocated: the arena, the temp
    // buffer and the status block live in that array, and the pinned staging is the
    // one reserved at dfr_create).
    char* static_scratch = nullptr;
    bool static_mode = false;

    // Options.
    size_t divert = 0;  // 0 = default N_d
    int force_d = 0;
    int timing = 0;  // 1 every stage, 2 the deal launches only
    bool force_lookback = false;  // deal every level with decoupled look-back
    bool force_key_heads = false;  // find bucket heads from the keys on every level
    bool est_buckets = false;      // first level of plain sorts: Fast Radix estimated buckets
    uint64_t plan_lengths_max = 0;  // first levels of segments this short plan from their
                                    // lengths alone (0: never)
    int radix_bits = 0;           // 0 = tuned or default
    uint32_t tile_records = 0;
    size_t window = 0;
    std::map<uint32_t, dfr_tune> tunes;  // tuned settings per (kb, vb, size class)

    dfr_stats stats{};
    // Order between calls on different streams: every call records `done` on its
    // stream when it returns, and a call on another stream first makes its stream wait
    // for it, because calls share the arena, the temp cache and the pinned staging.
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    struct Ev {
        int stage;
        bool deal;
        hipEvent_t a, b;
    };
    std::vector<Ev> events;
    std::vector<hipEvent_t> event_pool;

    // Request serving (dfr_submit / dfr_poll), started by the first submit.
    std::mutex serve_mu;
    struct Server* server = nullptr;
    int serve_workers = 3;
    uint64_t serve_batch_records = 1ull << 25;
    uint64_t serve_gather_records = 1ull << 20;  // largest request gathered into a batch
    // Test hook: this many of the next serving batches report DFR_E_HIP once their
    // device work is queued, to exercise the failure path without a device fault.
    std::atomic<int> serve_fail_batches{0};
};

namespace {

dfr_status fail_hip(dfr_ctx* c, hipError_t e, const char* what) {
    c->failed = true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    c->err = buf;
    return DFR_E_HIP;
}

#define HIP_TRY(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return fail_hip(ctx, e_, #call); \
    } while (0)

// Make room for `bytes` more past the bump pointer, keeping [0, arena_used) intact:
// a larger arena is allocated, the used prefix copied over on the stream, and the old
// one freed once the stream has drained.  Pointers into the arena must be re-derived
// from offsets after a call that may grow it.
dfr_status arena_need(dfr_ctx* c, size_t bytes, hipStream_t s) {
    const size_t need = c->arena_used + bytes;
    if (need <= c->arena_cap) return DFR_OK;
    if (c->static_mode) {  // the fixed scratch does not grow
        c->err = "allocation-free sort: level scratch exceeds the fixed scratch array";
        return DFR_E_TOO_LARGE;
    }
    const size_t cap = std::max<size_t>(round_up(need + need / 4, 1 << 20), 16 << 20);
    const auto t0 = std::chrono::steady_clock::now();
    char* na = nullptr;
    hipError_t e = hipMalloc((void**)&na, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->err = "scratch allocation failed";
        return DFR_E_NO_MEMORY;
    }
    if (c->arena_used && c->arena)
        HIP_TRY(c, hipMemcpyAsync(na, c->arena, c->arena_used, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->arena) HIP_TRY(c, hipFree(c->arena));
    c->arena = na;
    c->arena_cap = cap;
    c->n_allocs += 1;
    c->ms_alloc += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return DFR_OK;
}

// Start a fresh level: everything in the arena may be overwritten (work already
// enqueued on the stream keeps its order against later uploads and kernels).
dfr_status arena_reserve(dfr_ctx* c, size_t bytes, hipStream_t s) {
    c->arena_used = 0;
    return arena_need(c, bytes, s);
}

template <typename T>
T* aalloc(dfr_ctx* c, size_t count) {
    size_t bytes = round_up(std::max<size_t>(count, 1) * sizeof(T), ALIGN);
    T* p = (T*)(c->arena + c->arena_used);
    c->arena_used += bytes;
    return p;
}

template <typename T>
size_t asize(size_t count) {
    return round_up(std::max<size_t>(count, 1) * sizeof(T), ALIGN);
}

// Pinned staging.  Host writes land in it immediately, so it is only reused after a
// synchronisation of the stream that consumes it.
dfr_status pin_reserve(dfr_ctx* c, size_t bytes, hipStream_t s) {
    if (c->pin_used + bytes <= c->pin_cap) return DFR_OK;
    HIP_TRY(c, hipStreamSynchronize(s));
    c->pin_used = 0;
    if (bytes <= c->pin_cap) return DFR_OK;
    if (c->static_mode) {  // no allocation: the staging reserved at dfr_create is all
        c->err = "allocation-free sort: host staging exceeds the reserved buffer";
        return DFR_E_TOO_LARGE;
    }
    if (c->pin) HIP_TRY(c, hipHostFree(c->pin));
    c->pin = nullptr;
    size_t cap = std::max<size_t>(round_up(bytes * 2, 1 << 20), 4 << 20);
    hipError_t e = hipHostMalloc((void**)&c->pin, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->pin_cap = 0;
        c->err = "pinned staging allocation failed";
        return DFR_E_NO_MEMORY;
    }
    c->pin_cap = cap;
    return DFR_OK;
}

template <typename T>
T* palloc(dfr_ctx* c, size_t count) {
    size_t bytes = round_up(std::max<size_t>(count, 1) * sizeof(T), 64);
    T* p = (T*)(c->pin + c->pin_used);
    c->pin_used += bytes;
    return p;
}

void synced(dfr_ctx* c) { c->pin_used = 0; }

// Optional per-stage kernel timing.
hipEvent_t get_event(dfr_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timed {
    dfr_ctx* c;
    hipStream_t s;
    int stage;
    bool deal;
    hipEvent_t a = nullptr;
    Timed(dfr_ctx* c_, hipStream_t s_, int st, bool d = false) : c(c_), s(s_), stage(st), deal(d) {
        if (!c->static_mode && (c->timing == 1 || (c->timing == 2 && deal))) {
            a = get_event(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Timed() {
        if (c->timing && a) {
            hipEvent_t b = get_event(c);
            if (b) {
                (void)hipEventRecord(b, s);
                c->events.push_back({stage, deal, a, b});
            }
        }
    }
};

void collect_events(dfr_ctx* c) {
    for (auto& e : c->events) {
        float ms = 0.f;
        if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            switch (e.stage) {
                case ST_COUNT: c->stats.ms_count += ms; break;
                case ST_DEAL: c->stats.ms_deal += ms; break;
                case ST_BUCKETS: c->stats.ms_buckets += ms; break;
                case ST_LOCAL: c->stats.ms_local_sort += ms; break;
                default: c->stats.ms_other += ms; break;
            }
            if (e.deal) c->stats.deal_launches_timed += 1;
        }
        c->event_pool.push_back(e.a);
        c->event_pool.push_back(e.b);
    }
    c->events.clear();
}

size_t local_cap(int kb, int vb) { return local_sort_capacity(kb, vb); }

// Default N_d: three quarters of the local sort's capacity.  A bucket whose expected
// size is N_d has a standard deviation near sqrt(N_d), so its largest siblings stay
// well inside the capacity and few buckets recurse.
size_t default_divert(int kb, int vb) { return local_cap(kb, vb) * 3 / 4; }

// ---------------------------------------------------------------------------------
// Planner (Sec. 3: estimate the number of most significant digits to deal so that
// diversion is reached; Sec. 3.1: the diversion threshold N_d).
// ---------------------------------------------------------------------------------

// Varying 8-bit digits of a segment, most significant first, from its OR and AND.
// Digits of `rb` bits, digit j holding key bits [j*rb, min((j+1)*rb, 8*kb)).
int num_digits(int kb, int rb) { return (8 * kb + rb - 1) / rb; }

// Digits on which some two keys differ, most significant first.
std::vector<int> varying_digits(uint64_t vor, uint64_t vand, int kb, int rb) {
    std::vector<int> v;
    const uint64_t var = vor ^ vand;
    const uint64_t mask = (1ull << rb) - 1;
    for (int j = num_digits(kb, rb) - 1; j >= 0; --j)
        if ((var >> (rb * j)) & mask) v.push_back(j);
    return v;
}

// Digits to deal for one segment of n records, from the collision probability of
// each of its digits, coll[j] = sum_v h_j[v]^2 / n^2: the chance that two random
// records share digit j.  With digits taken as independent, a random record's bucket
// after dealing the top digits holds about n * prod coll[j] records; d is the fewest
// top varying digits (V, most significant first) that bring this to N_d or below
// (Sec. 3; Sec. 3.1 for N_d).  When dealing every varying digit (plain LSD, Sec. 2.1)
// moves fewer bytes than DFR with that d, the plan deals them all.
int plan_segment(const double* coll, size_t n, int kb, int vb, size_t divert,
                 const std::vector<int>& V) {
    const int nv = (int)V.size();
    if (nv == 0) return 0;
    double expect = (double)n;
    int d = nv;
    for (int i = 0; i < nv; ++i) {
        expect *= coll[V[i]];
        if (expect <= (double)divert) {
            d = i + 1;
            break;
        }
    }
    const double rec = kb + vb, pass = 2 * rec;
    const double dfr_bytes = d * pass + kb + pass;
    const double lsd_bytes = nv * pass + ((nv % 2) ? pass : 0.0);
    if (d >= nv || lsd_bytes <= dfr_bytes) d = nv;
    return d;
}

// The same plan from the histograms of all kb digits (hist[j * 256 + v]).
int plan_from_hist(const uint32_t* hist, size_t n, int kb, int vb, size_t divert,
                   const std::vector<int>& V) {
    double coll[8] = {0};
    for (int j = 0; j < kb; ++j) {
        double c = 0;
        for (int v = 0; v < RADIX; ++v) c += (double)hist[j * RADIX + v] * (double)hist[j * RADIX + v];
        coll[j] = n ? c / ((double)n * (double)n) : 0.0;
    }
    return plan_segment(coll, n, kb, vb, divert, V);
}

// ---------------------------------------------------------------------------------
// Tuning: digit width, deal tile, diversion threshold and window width per (key
// bytes, value bytes, size class).  Explicit options override a tuned entry, which
// overrides the defaults.
// ---------------------------------------------------------------------------------
uint32_t tune_key(int kb, int vb, int cls) { return (uint32_t)(kb << 16 | vb << 8 | cls); }

dfr_tune default_tune(int kb, int vb) {
    dfr_tune t{};
    t.radix_bits = RADIX_BITS;
    t.tile_records = deal_tile_records(kb, vb);
    t.divert_records = default_divert(kb, vb);
    // Windows of half the bucketed local sort's capacity (rounded down to a power of
    // two): a window's chunk spans less than two windows, so it fits that kernel.
    uint64_t w = 16;
    while (2 * w <= local_bucket_capacity(kb, vb) / 2) w *= 2;
    t.window_records = w;
    return t;
}

// A tuning is usable when every kernel it selects exists and the local sort can hold
// every chunk it makes: a window's chunk spans less than two windows.
bool tune_valid(const dfr_tune& t, int kb, int vb) {
    const size_t cap = local_cap(kb, vb);
    return t.radix_bits >= 4 && t.radix_bits <= RADIX_BITS && num_digits(kb, t.radix_bits) <= MAX_PASSES &&
           deal_tile_supported(kb, vb, t.tile_records) && t.divert_records >= 1 &&
           t.divert_records <= cap && t.window_records >= 16 && t.window_records <= cap / 2;
}

// floor(log2) of the size-biased mean length of the segments that need sorting.
int size_class(const std::vector<LSeg>& segs) {
    double s1 = 0, s2 = 0;
    for (const LSeg& g : segs)
        if (g.len > 1) {
            s1 += (double)g.len;
            s2 += (double)g.len * (double)g.len;
        }
    if (s1 <= 0) return 0;
    return std::max(0, std::min(DFR_TUNE_CLASSES - 1, (int)std::floor(std::log2(s2 / s1))));
}

dfr_tune effective_tune(const dfr_ctx* c, int kb, int vb, int cls) {
    dfr_tune t = default_tune(kb, vb);
    auto it = c->tunes.find(tune_key(kb, vb, cls));
    if (it != c->tunes.end()) t = it->second;
    if (c->radix_bits) t.radix_bits = c->radix_bits;
    if (c->tile_records) t.tile_records = c->tile_records;
    if (c->divert) t.divert_records = c->divert;
    if (c->window) t.window_records = c->window;
    const size_t cap = local_cap(kb, vb);
    t.divert_records = std::min<uint64_t>(t.divert_records, cap);
    t.window_records = std::min<uint64_t>(t.window_records, cap / 2);
    if (!tune_valid(t, kb, vb)) t = default_tune(kb, vb);
    return t;
}

// ---------------------------------------------------------------------------------
// One sort (plain or segmented), level by level.
// ---------------------------------------------------------------------------------
struct Job {
    dfr_ctx* c;
    int kb, vb;
    void* k[2];  // [0] caller, [1] temp
    void* v[2];
    hipStream_t s;
    uint32_t tile;  // deal tile records
    int rb = RADIX_BITS;  // digit width of the deal passes
    size_t cap;     // local sort capacity
    size_t wsmall;  // small bucket limit = window width
    bool window_default = false;  // wsmall is the default, not an option or a tuning
    size_t divert;
    bool first_level = true;
    int top_d_forced = 0;
    uint32_t err_word_host = 0;
    bool err_known = false;  // err_word_host holds the word after the last error-setting kernel
    uint32_t stat_host[STAT_WORDS] = {};  // the status block as last read back
    uint32_t* err_dev = nullptr;
};

// Tiles of at most `tile` records over the given segments.
void build_tiles(const std::vector<LSeg>& segs, const std::vector<uint32_t>& ids, uint32_t tile,
                 std::vector<Tile>& tiles, std::vector<uint32_t>& first_tile) {
    tiles.clear();
    first_tile.assign(segs.size(), 0);
    for (uint32_t s : ids) {
        first_tile[s] = (uint32_t)tiles.size();
        for (uint64_t off = 0; off < segs[s].len; off += tile) {
            Tile t;
            t.start = segs[s].start + off;
            t.len = (uint32_t)std::min<uint64_t>(tile, segs[s].len - off);
            t.seg = s;
            tiles.push_back(t);
        }
    }
}

dfr_status upload(Job& j, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return DFR_OK;
    dfr_status st = pin_reserve(j.c, bytes, j.s);
    if (st) return st;
    char* p = palloc<char>(j.c, bytes);
    memcpy(p, src, bytes);
    HIP_TRY(j.c, hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, j.s));
    return DFR_OK;
}

// Copy finished ranges from the temp buffer into the caller's buffer.
dfr_status copy_back(Job& j, const std::vector<std::pair<uint64_t, uint64_t>>& ranges) {
    if (ranges.empty()) return DFR_OK;
    std::vector<Tile> tiles;
    for (auto& r : ranges)
        for (uint64_t off = 0; off < r.second; off += 65536)
            tiles.push_back(Tile{r.first + off, (uint32_t)std::min<uint64_t>(65536, r.second - off), 0});
    dfr_status st = arena_need(j.c, asize<Tile>(tiles.size()), j.s);
    if (st) return st;
    Tile* dt = aalloc<Tile>(j.c, tiles.size());
    st = upload(j, dt, tiles.data(), tiles.size() * sizeof(Tile));
    if (st) return st;
    Timed tm(j.c, j.s, ST_OTHER);
    HIP_TRY(j.c, launch_copy_tiles(j.kb, j.vb, j.k[1], j.v[1], j.k[0], j.v[0], dt, (uint32_t)tiles.size(), j.s));
    return DFR_OK;
}

// Buckets are known on the host (segments no larger than the local sort's capacity):
// each segment is one bucket and one local-sort chunk of its own.
dfr_status divert_level(Job& j, const std::vector<LSeg>& segs, int in) {
    dfr_ctx* c = j.c;
    j.err_known = false;
    const size_t S = segs.size();
    std::vector<Seg> hs(S);
    std::vector<uint64_t> bstart;
    std::vector<uint32_t> bseg;
    for (size_t i = 0; i < S; ++i) {
        Seg g{};
        g.start = segs[i].start;
        g.len = segs[i].len;
        g.lo_bit = segs[i].hi_bit;
        hs[i] = g;
        if (segs[i].len) {
            bstart.push_back(segs[i].start);
            bseg.push_back((uint32_t)i);
        }
    }
    const uint64_t nb = bstart.size();
    if (nb == 0) return DFR_OK;
    std::vector<uint32_t> med(nb);
    for (uint64_t i = 0; i < nb; ++i) med[i] = (uint32_t)i;
    // buckets, medium, spills, work, wide
    uint32_t counts3[5] = {(uint32_t)nb, (uint32_t)nb, 0, (uint32_t)nb, 0};
    const size_t need = asize<Seg>(S) + asize<uint64_t>(nb) + 2 * asize<uint32_t>(nb) +
                        3 * asize<ChunkDesc>(nb) + asize<uint32_t>(5) + asize<uint32_t>(1);
    dfr_status st = arena_reserve(c, need, j.s);
    if (st) return st;
    Seg* dsegs = aalloc<Seg>(c, S);
    uint64_t* dbstart = aalloc<uint64_t>(c, nb);
    uint32_t* dbseg = aalloc<uint32_t>(c, nb);
    uint32_t* dmed = aalloc<uint32_t>(c, nb);
    ChunkDesc* ddesc = aalloc<ChunkDesc>(c, nb);
    ChunkDesc* dspill = aalloc<ChunkDesc>(c, nb);
    ChunkDesc* dwide = aalloc<ChunkDesc>(c, nb);
    uint32_t* dcounts = aalloc<uint32_t>(c, 5);
    uint32_t* dnone = aalloc<uint32_t>(c, 1);
    st = upload(j, dsegs, hs.data(), S * sizeof(Seg));
    if (!st) st = upload(j, dbstart, bstart.data(), nb * sizeof(uint64_t));
    if (!st) st = upload(j, dbseg, bseg.data(), nb * sizeof(uint32_t));
    if (!st) st = upload(j, dmed, med.data(), nb * sizeof(uint32_t));
    if (!st) st = upload(j, dcounts, counts3, sizeof counts3);
    if (st) return st;
    {
        Timed tm(c, j.s, ST_LOCAL);
        LocalArgs la{};
        la.kin = j.k[in];
        la.vin = j.v[in];
        la.kout = j.k[0];
        la.vout = j.v[0];
        la.bstart = dbstart;
        la.bseg = dbseg;
        la.nbuckets = dcounts;
        la.bcap = nb;
        la.segs = dsegs;
        la.cfirst = dnone;
        la.clast = dnone;
        la.nslots = 0;
        la.med = dmed;
        la.nmed = dcounts + 1;
        la.medcap = (uint32_t)nb;
        la.work = dmed;  // medium index i is work item i (no window slots)
        la.nwork = dcounts + 3;
        la.workcap = (uint32_t)nb;
        la.desc = ddesc;
        la.spill = dspill;
        la.nspill = dcounts + 2;
        la.spillcap = (uint32_t)nb;
        la.wide = dwide;
        la.nwide = dcounts + 4;
        la.widecap = (uint32_t)nb;
        la.err = j.err_dev;
        la.stat = j.err_dev;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(nb, 8192);
        int max_lo = 0;
        for (const Seg& g : hs) max_lo = std::max(max_lo, (int)g.lo_bit);
        HIP_TRY(c, launch_local_sort(j.kb, j.vb, la, blocks,
                                     local_sort_first_form(j.kb, j.vb, max_lo, 0), j.s));
        c->stats.chunks += nb;
    }
    c->stats.used_diversion = 1;
    return DFR_OK;
}

// A level over segments larger than the local sort's capacity, all held in buffer
// `in`.  Appends the next level's segments (large buckets) to `next`, and sets
// *next_in to the buffer that holds them.
dfr_status deal_level(Job& j, const std::vector<LSeg>& segs, int in, std::vector<LSeg>& next,
                      int* next_in) {
    dfr_ctx* c = j.c;
    j.err_known = false;
    const size_t S = segs.size();
    const int kb = j.kb;
    const int rb = j.rb;
    const int ndig = num_digits(kb, rb);  // every digit of the key
    *next_in = in;
    std::vector<uint32_t> all_ids(S);
    for (size_t i = 0; i < S; ++i) all_ids[i] = (uint32_t)i;
    std::vector<Tile> tiles;
    std::vector<uint32_t> first_tile;
    build_tiles(segs, all_ids, j.tile, tiles, first_tile);

    // --- 1. count ---------------------------------------------------------------
    // Region A of the arena (kept for the whole level): histograms and OR/AND.
    const size_t hist_n = S * ndig * RADIX;
    // Levels are dealt without look-back where the tiles' bucket bases can be scanned
    // ahead of the deal: the count also keeps every tile's own digit counts.  One
    // segment: a three-kernel scan over all tiles; several segments of at most
    // kSegScanTiles tiles each: one block per segment walks its tiles.
    uint64_t max_seg_tiles = 0;
    for (const LSeg& g : segs) max_seg_tiles = std::max<uint64_t>(max_seg_tiles, (g.len + j.tile - 1) / j.tile);
    const bool single = S == 1 && !c->force_lookback;
    // A short single segment takes the one-block walk too: one launch instead of three.
    const bool segscan = !c->force_lookback && (S > 1 ? max_seg_tiles <= kSegScanTiles
                                                      : S == 1 && max_seg_tiles <= kSingleWalkTiles);
    const bool perseg = S > 1 && !segscan && S <= kPerSegScanMax && !c->force_lookback;
    const bool nolb = single || segscan || perseg;
    const size_t tcnt_n = nolb ? tiles.size() * ndig * RADIX : 0;
    dfr_status st = arena_reserve(c, asize<uint32_t>(hist_n) + 2 * asize<uint64_t>(S) +
                                         asize<double>(S * ndig) + 2 * asize<uint32_t>(S * ndig) +
                                         asize<uint32_t>(tcnt_n) +
                                         asize<Tile>(tiles.size()), j.s);
    if (st) return st;
    const size_t off_hist = c->arena_used;
    aalloc<uint32_t>(c, hist_n);
    const size_t off_coll = c->arena_used;
    aalloc<double>(c, S * ndig);
    const size_t off_nz = c->arena_used;
    aalloc<uint32_t>(c, S * ndig);
    const size_t off_ovf = c->arena_used;
    aalloc<uint32_t>(c, S * ndig);
    const size_t off_or = c->arena_used;
    aalloc<uint64_t>(c, S);
    const size_t off_and = c->arena_used;
    aalloc<uint64_t>(c, S);
    const size_t off_tcnt = c->arena_used;
    aalloc<uint32_t>(c, tcnt_n);
    const size_t off_ctiles = c->arena_used;  // the counting tile list, kept for reuse
    aalloc<Tile>(c, tiles.size());
    const size_t region_a = c->arena_used;
    Tile* dtiles = (Tile*)(c->arena + off_ctiles);
    uint32_t* dhist = (uint32_t*)(c->arena + off_hist);
    uint64_t* dor = (uint64_t*)(c->arena + off_or);
    uint64_t* dand = (uint64_t*)(c->arena + off_and);
    st = upload(j, dtiles, tiles.data(), tiles.size() * sizeof(Tile));
    if (st) return st;
    {
        Timed tm(c, j.s, ST_COUNT);
        FillSet fs{};
        fs.count = 3;
        fs.p[0] = dhist, fs.v[0] = 0, fs.n[0] = hist_n, fs.w[0] = 4;
        fs.p[1] = dor, fs.v[1] = 0, fs.n[1] = S, fs.w[1] = 8;
        fs.p[2] = dand, fs.v[2] = ~0ull, fs.n[2] = S, fs.w[2] = 8;
        HIP_TRY(c, launch_fill_set(fs, j.s));
        CountArgs ca{};
        ca.keys = j.k[in];
        ca.tiles = dtiles;
        ca.ntiles = (uint32_t)tiles.size();
        // Two rounds of blocks over the 256 CUs (8 resident each): the LDS-atomic-bound
        // count overlaps one block's tile flush with another's counting.
        const uint32_t blocks = (uint32_t)std::min<size_t>(tiles.size(), 4096);
        ca.tiles_per_block = (uint32_t)((tiles.size() + blocks - 1) / blocks);
        ca.base_shift = 0;
        ca.bits = rb;
        // Keys of a segment agree above its hi_bit (the digits its parent bucket was
        // dealt on, and the bits constant above them): only the digits below the
        // highest hi_bit are counted; the plan sees the others as constant from OR/AND.
        int top_bit = 0;
        for (const LSeg& g : segs) top_bit = std::max(top_bit, g.hi_bit);
        ca.ndig = std::max(1, std::min(ndig, (top_bit + rb - 1) / rb));
        ca.hist_digits = ndig;
        ca.hist = dhist;
        ca.seg_or = dor;
        ca.seg_and = dand;
        ca.tile_hist = nolb ? (uint32_t*)(c->arena + off_tcnt) : nullptr;
        const uint32_t grid = (uint32_t)((tiles.size() + ca.tiles_per_block - 1) / ca.tiles_per_block);
        HIP_TRY(c, launch_count(kb, ca, grid, j.s));
    }
    // Each segment's digit collision probabilities, then read them back with OR/AND.
    // The OR/AND words are key-sized: 32-bit keys use the low half of each 8-byte slot.
    double* dcoll = (double*)(c->arena + off_coll);
    uint32_t* dnz = (uint32_t*)(c->arena + off_nz);
    uint32_t* dovf = (uint32_t*)(c->arena + off_ovf);
    {
        Timed tm(c, j.s, ST_COUNT);
        HIP_TRY(c, launch_collisions(dhist, (uint32_t)S, ndig, rb, dcoll, dnz, dovf, j.s));
    }
    // Collision estimates, non-empty bins, overflow, OR and AND lie next to each other in
    // the arena: one copy brings them all back.
    const size_t readback = off_and + asize<uint64_t>(S) - off_coll;
    // A first level whose segments are all short plans from their lengths alone: every
    // digit taken as varying and uniform, the paper's estimate of the top digits for
    // uniform keys (Sec. 3, Sec. 3.1).  Nothing is read back before its deals, so a
    // one-level sort waits on the device only at its end.  A guess that leaves a bucket
    // too large for the local sort only sends it to the next level; a constant digit is
    // only a deal that moves nothing.
    uint64_t max_len = 0;
    for (const LSeg& g : segs) max_len = std::max<uint64_t>(max_len, g.len);
    const bool from_lengths = j.first_level && j.top_d_forced == 0 && c->plan_lengths_max > 0 &&
                              max_len <= c->plan_lengths_max;
    std::vector<uint64_t> vor(S), vand(S);
    std::vector<double> coll(S * ndig);
    std::vector<uint32_t> nonzero(S * ndig), overflow(S * ndig, 0);
    auto digit_width = [&](int dig) { return std::min(rb, 8 * kb - rb * dig); };
    if (from_lengths) {
        const uint64_t all = kb == 8 ? ~0ull : 0xffffffffull;
        for (size_t i = 0; i < S; ++i) {
            vor[i] = all;
            vand[i] = 0;
            for (int dg = 0; dg < ndig; ++dg) {
                coll[i * ndig + dg] = 1.0 / (double)(1u << digit_width(dg));
                nonzero[i * ndig + dg] = 1u << digit_width(dg);
            }
        }
        c->stats.plan_from_lengths = 1;
    } else {
        st = pin_reserve(c, readback + ALIGN, j.s);
        if (st) return st;
        char* h_rb = palloc<char>(c, readback);
        HIP_TRY(c, hipMemcpyAsync(h_rb, c->arena + off_coll, readback, hipMemcpyDeviceToHost, j.s));
        HIP_TRY(c, hipStreamSynchronize(j.s));
        const double* h_coll = (const double*)h_rb;
        const uint32_t* h_nz = (const uint32_t*)(h_rb + (off_nz - off_coll));
        const uint32_t* h_ovf = (const uint32_t*)(h_rb + (off_ovf - off_coll));
        const uint64_t* h_or = (const uint64_t*)(h_rb + (off_or - off_coll));
        const uint64_t* h_and = (const uint64_t*)(h_rb + (off_and - off_coll));
        for (size_t i = 0; i < S; ++i) {
            if (kb == 4) {
                vor[i] = ((const uint32_t*)h_or)[i];
                vand[i] = ((const uint32_t*)h_and)[i];
            } else {
                vor[i] = h_or[i];
                vand[i] = h_and[i];
            }
        }
        coll.assign(h_coll, h_coll + S * ndig);
        nonzero.assign(h_nz, h_nz + S * ndig);
        overflow.assign(h_ovf, h_ovf + S * ndig);
        synced(c);
    }

    // --- 2. plan ------------------------------------------------------------------
    // Per segment: its varying digits (from OR/AND) and the digits d_s to deal (forced
    // at the first level when asked).  The level deals d = max d_s passes.  A segment
    // that needs fewer sits out the first passes in pairs, so that it ends in the same
    // buffer as the others, and deals its lowest selected digit twice when d - d_s is
    // odd (a second deal on one digit changes nothing: the deal is stable).
    std::vector<std::vector<int>> V(S);
    std::vector<std::pair<uint64_t, uint64_t>> finished;  // all-equal segments
    std::vector<uint32_t> active;
    std::vector<int> dsel(S, 0);
    int d = 1;
    for (size_t i = 0; i < S; ++i) {
        V[i] = varying_digits(vor[i], vand[i], kb, rb);
        if (V[i].empty()) {
            finished.push_back({segs[i].start, segs[i].len});
            continue;
        }
        active.push_back((uint32_t)i);
        const int nv = (int)V[i].size();
        int di = (j.first_level && j.top_d_forced > 0)
                     ? j.top_d_forced
                     : plan_segment(&coll[i * ndig], segs[i].len, kb, j.vb, j.divert, V[i]);
        // Skewed prefix: when the top varying digit takes only a few values and its
        // buckets would still need several more digits, deal that digit alone and let
        // each bucket plan the rest with its own constant digits (digits that vary only
        // across the few groups of the prefix are then skipped; Sec. 3 recursion).
        const uint32_t nz_top = nonzero[i * ndig + V[i][0]];
        if (!(j.first_level && j.top_d_forced > 0) && nv > 1 && nz_top <= kFewTopValues &&
            (double)segs[i].len / nz_top > (double)j.divert * (double)(1u << rb))
            di = 1;
        di = std::max(1, std::min(std::min(di, nv), MAX_PASSES));
        dsel[i] = di;
        d = std::max(d, di);
    }
    c->arena_used = region_a;  // the rest of the arena is free again
    if (j.first_level && !from_lengths) {
        // What Fast Radix's estimated buckets would have overflowed on the top varying
        // digit of each segment (Sec. 3.1; Eq. 2 gives its expectation for uniform keys).
        double ov = 0, len = 0;
        for (uint32_t i : active) {
            ov += overflow[i * ndig + V[i][0]];
            len += (double)segs[i].len;
        }
        c->stats.estimated_overflow = len > 0 ? ov / len : 0.0;
    }
    if (in == 1) {
        st = copy_back(j, finished);
        if (st) return st;
    }
    if (active.empty()) return DFR_OK;
    if (j.first_level) c->stats.top_digits = d;
    auto skip_of = [&](uint32_t i) { return (d - dsel[i]) & ~1; };
    // Segments that sit out more passes come later, so pass p deals a prefix of tiles.
    std::stable_sort(active.begin(), active.end(),
                     [&](uint32_t x, uint32_t y) { return skip_of(x) < skip_of(y); });

    std::vector<Seg> hs(S);
    std::vector<char> full(S, 0);
    bool all_full = true;
    uint64_t nslots = 0, medcap = 0, bcap = 0, bigcap = 0;
    const std::vector<uint32_t> count_tile = first_tile;  // tiles of the counting list
    // When every segment is dealt, in its original order, the deal's tile list is the
    // counting list, already on the device.
    bool same_tiles = active.size() == S;
    for (size_t i = 0; same_tiles && i < S; ++i) same_tiles = active[i] == i;
    if (!same_tiles) build_tiles(segs, active, j.tile, tiles, first_tile);
    std::vector<uint32_t> pass_tiles(d, 0);  // tiles dealt in pass p
    // Window width of this level.  By default, where every dealt segment's buckets
    // average 512 records or more, windows of half the bucketed local sort's capacity
    // (a chunk spans less than two windows, so it still fits): fuller chunks, while a
    // chunk's buckets stay few enough for their index to fit beside the sort bits.
    size_t wsmall = j.wsmall;
    if (j.window_default) {
        const size_t half = local_bucket_capacity(kb, j.vb) / 2;
        bool large = true;
        for (uint32_t i : active) {
            const int bits = rb * dsel[i];
            large = large && bits < 64 && (segs[i].len >> bits) >= 512;
        }
        if (large && half > wsmall) wsmall = half;
    }
    for (uint32_t i : active) {
        const uint64_t nt = (segs[i].len + j.tile - 1) / j.tile;
        for (int p = skip_of(i); p < d; ++p) pass_tiles[p] += (uint32_t)nt;
        Seg g{};
        g.start = segs[i].start;
        g.len = segs[i].len;
        g.first_tile = first_tile[i];
        g.count_tile = count_tile[i];
        const int skip = skip_of(i), np = d - skip, di = dsel[i];
        g.first_pass = skip;
        g.npass = np;
        const std::vector<int>& v = V[i];
        const int nv = (int)v.size();
        // Selected digits, most significant first; the lowest once more if np > d_s.
        std::vector<int> sel(v.begin(), v.begin() + di);
        if (np > di) sel.push_back(sel.back());
        for (int p = 0; p < d; ++p) {  // LSD order: least significant selected first
            const int q = std::max(p, skip) - skip;
            const int dig = sel[np - 1 - q];
            g.shift[p] = (int8_t)(rb * dig);
            g.width[p] = (int8_t)std::min(rb, 8 * kb - rb * dig);
            g.hslot[p] = (int8_t)dig;
        }
        full[i] = nv <= di;
        g.lo_bit = full[i] ? 0 : rb * v[di - 1];
        if (!full[i]) {
            all_full = false;
            g.window_base = (uint32_t)nslots;
            nslots += (segs[i].len + wsmall - 1) / wsmall;
            medcap += segs[i].len / (wsmall + 1);
            bigcap += segs[i].len / (j.cap + 1);
            const uint64_t maxb = rb * di >= 64 ? ~0ull : (1ull << (rb * di));
            bcap += std::min<uint64_t>(segs[i].len, maxb);
        }
        hs[i] = g;
    }
    // Tiles whose buckets are found after the deals: those of segments not yet sorted
    // (the deal's list itself when no segment is).
    bool any_full = false;
    for (uint32_t i : active) any_full = any_full || full[i];
    std::vector<Tile> htiles;
    if (any_full)
        for (const Tile& t : tiles)
            if (!full[t.seg]) htiles.push_back(t);
    const uint64_t nht = any_full ? htiles.size() : tiles.size();

    // --- 3. deal ------------------------------------------------------------------
    const uint64_t ntiles = tiles.size();
    const size_t need_b = asize<Tile>(ntiles) + asize<Tile>(nht) + asize<Seg>(S) +
                          asize<uint64_t>(ntiles * RADIX + 1) +
                          asize<uint32_t>(nht) + asize<uint64_t>(nht) + asize<uint16_t>(nht * HEAD_SLOTS) +
                          asize<uint64_t>(bcap) + asize<uint32_t>(bcap) +
                          2 * asize<uint32_t>(nslots) + asize<uint32_t>(medcap) +
                          2 * asize<Big>(bigcap) + asize<uint32_t>(nslots + medcap) +
                          3 * asize<ChunkDesc>(nslots + medcap) +
                          asize<uint32_t>(8) + asize<uint32_t>(1u << (2 * RADIX_BITS)) +
                          asize<uint64_t>(RADIX) + 2 * asize<uint32_t>(S);
    const uint32_t scan_tpb = 128;
    const uint32_t scan_nb = (uint32_t)((ntiles + scan_tpb - 1) / scan_tpb);
    const size_t need_nolb = nolb ? asize<uint32_t>(ntiles * RADIX) * 2 +
                                        (single || perseg ? asize<uint32_t>((size_t)scan_nb * RADIX) : 0)
                                  : 0;
    st = arena_need(c, need_b + need_nolb, j.s);  // keeps region A
    if (st) return st;
    dhist = (uint32_t*)(c->arena + off_hist);
    uint32_t* tcnt = (uint32_t*)(c->arena + off_tcnt);
    uint32_t *toff = nullptr, *tone = nullptr, *tpart = nullptr;
    if (nolb) {
        toff = aalloc<uint32_t>(c, ntiles * RADIX);
        tone = aalloc<uint32_t>(c, ntiles * RADIX);
    }
    if (single || perseg) tpart = aalloc<uint32_t>(c, (size_t)scan_nb * RADIX);
    dtiles = same_tiles ? (Tile*)(c->arena + off_ctiles) : aalloc<Tile>(c, ntiles);
    Tile* dhtiles = any_full ? aalloc<Tile>(c, nht) : dtiles;
    Seg* dsegs = aalloc<Seg>(c, S);
    uint64_t* lb = aalloc<uint64_t>(c, ntiles * RADIX + 1);  // look-back words, then the ticket
    uint32_t* htcount = aalloc<uint32_t>(c, nht);
    uint64_t* htbase = aalloc<uint64_t>(c, nht);
    uint16_t* htslot = aalloc<uint16_t>(c, nht * HEAD_SLOTS);
    uint64_t* dbstart = aalloc<uint64_t>(c, bcap);
    uint32_t* dbseg = aalloc<uint32_t>(c, bcap);
    uint32_t* cfirst = aalloc<uint32_t>(c, nslots);
    uint32_t* clast = aalloc<uint32_t>(c, nslots);
    uint32_t* med = aalloc<uint32_t>(c, medcap);
    Big* big = aalloc<Big>(c, bigcap);
    Big* done = aalloc<Big>(c, bigcap);
    ChunkDesc* spill = aalloc<ChunkDesc>(c, nslots + medcap);
    uint32_t* work = aalloc<uint32_t>(c, nslots + medcap);
    ChunkDesc* wide = aalloc<ChunkDesc>(c, nslots + medcap);
    ChunkDesc* desc = aalloc<ChunkDesc>(c, nslots + medcap);
    uint32_t* counters = j.err_dev + STAT_WORDS;  // buckets, medium, big, done, spill, work, wide
    uint32_t* joint = aalloc<uint32_t>(c, 1u << (2 * RADIX_BITS));  // pair counts (heads from counts)
    uint64_t* joint_rows = aalloc<uint64_t>(c, RADIX);
    uint32_t* hh_ids = aalloc<uint32_t>(c, S);    // heads from histograms: segments,
    uint32_t* hh_first = aalloc<uint32_t>(c, S);  // and each one's first list index
    st = same_tiles ? DFR_OK : upload(j, dtiles, tiles.data(), ntiles * sizeof(Tile));
    if (!st && any_full) st = upload(j, dhtiles, htiles.data(), nht * sizeof(Tile));
    if (!st) st = upload(j, dsegs, hs.data(), S * sizeof(Seg));
    if (st) return st;

    int cur = in;
    for (int p = 0; p < d; ++p) {
        const uint32_t ntp = pass_tiles[p];
        if (nolb && p > 0) {
            // Per-tile counts of this pass's digit in the current order (the first
            // pass takes them from the level's count).
            Timed tc(c, j.s, ST_COUNT);
            CountArgs ca{};
            ca.keys = j.k[cur];
            ca.tiles = dtiles;
            ca.ntiles = ntp;
            const uint32_t blocks = std::min<uint32_t>(ntp, 4096);
            ca.tiles_per_block = (ntp + blocks - 1) / blocks;
            ca.base_shift = hs[active[0]].shift[p];
            ca.bits = rb;
            ca.ndig = 1;
            ca.tile_hist = tone;
            ca.segs = single ? nullptr : dsegs;  // several segments: each its own digit
            ca.pass = p;
            const uint32_t grid = (ntp + ca.tiles_per_block - 1) / ca.tiles_per_block;
            HIP_TRY(c, launch_count(kb, ca, grid, j.s));
        }
        if (segscan) {
            SegScanArgs sa{};
            sa.segs = dsegs;
            sa.nsegs = (uint32_t)S;
            sa.hist = dhist;
            sa.hist_digits = ndig;
            sa.cnt = p == 0 ? tcnt : tone;
            sa.cnt_ndig = p == 0 ? ndig : 1;
            sa.cnt_from_count_tiles = p == 0;
            sa.pass = p;
            sa.tile = j.tile;
            sa.off = toff;
            sa.ticket = lb + ntiles * RADIX;
            Timed ts(c, j.s, ST_OTHER);
            HIP_TRY(c, launch_seg_scan(sa, j.s));
        } else if (single) {
            const Seg& g = hs[active[0]];
            TileScanArgs ta{};
            ta.cnt = p == 0 ? tcnt : tone;
            ta.ndig = p == 0 ? ndig : 1;
            ta.slot = p == 0 ? g.hslot[0] : 0;
            ta.ntiles = (uint32_t)ntiles;
            ta.tiles_per_block = scan_tpb;
            ta.nblocks = scan_nb;
            ta.partial = tpart;
            ta.off = toff;
            ta.ticket = lb + ntiles * RADIX;
            Timed ts(c, j.s, ST_OTHER);
            HIP_TRY(c, launch_tile_scan(ta, j.s));
        } else if (perseg) {
            // A few long segments: the one-segment scan over each segment's tiles.
            Timed ts(c, j.s, ST_OTHER);
            for (uint32_t i : active) {
                const Seg& g = hs[i];
                if (p < g.first_pass) continue;
                const uint32_t nt = (uint32_t)((g.len + j.tile - 1) / j.tile);
                TileScanArgs ta{};
                ta.cnt = p == 0 ? tcnt + (size_t)g.count_tile * ndig * RADIX
                                : tone + (size_t)g.first_tile * RADIX;
                ta.ndig = p == 0 ? ndig : 1;
                ta.slot = p == 0 ? g.hslot[0] : 0;
                ta.ntiles = nt;
                ta.tiles_per_block = scan_tpb;
                ta.nblocks = (nt + scan_tpb - 1) / scan_tpb;
                ta.partial = tpart;
                ta.off = toff + (size_t)g.first_tile * RADIX;
                HIP_TRY(c, launch_tile_scan(ta, j.s));
            }
            HIP_TRY(c, launch_fill_u64(lb + ntiles * RADIX, 0, 1, j.s));  // tile ticket
        } else {
            HIP_TRY(c, launch_fill_u64(lb, 0, ntiles * RADIX + 1, j.s));
        }
        Timed tm(c, j.s, ST_DEAL, true);
        DealArgs da{};
        da.off = nolb ? toff : nullptr;
        da.tile = j.tile;
        da.kin = j.k[cur];
        da.vin = j.v[cur];
        da.kout = j.k[1 - cur];
        da.vout = j.v[1 - cur];
        da.tiles = dtiles;
        da.ntiles = ntp;
        da.segs = dsegs;
        da.hist = dhist;
        da.hist_digits = ndig;
        da.pass = p;
        da.lookback = lb;
        da.ticket = (uint32_t*)(lb + ntiles * RADIX);
        da.err = j.err_dev;
        HIP_TRY(c, launch_deal(kb, j.vb, da, j.s));
        cur = 1 - cur;
        c->stats.deal_passes += 1;
        if (nolb) c->stats.deal_passes_scanned += 1;
        else c->stats.deal_passes_lookback += 1;
    }
    *next_in = cur;

    // Segments whose every varying digit was dealt are sorted (plain LSD, Sec. 2.1).
    if (cur == 1) {
        std::vector<std::pair<uint64_t, uint64_t>> r;
        for (uint32_t i : active)
            if (full[i]) r.push_back({segs[i].start, segs[i].len});
        st = copy_back(j, r);
        if (st) return st;
    }
    if (all_full) return DFR_OK;

    // --- 4. buckets ---------------------------------------------------------------
    {
        Timed tm(c, j.s, ST_BUCKETS);
        FillSet fs{};
        fs.count = 3;
        fs.p[0] = counters, fs.v[0] = 0, fs.n[0] = 8, fs.w[0] = 4;
        fs.p[1] = cfirst, fs.v[1] = 0xffffffffu, fs.n[1] = nslots, fs.w[1] = 4;
        fs.p[2] = clast, fs.v[2] = 0, fs.n[2] = nslots, fs.w[2] = 4;
        HIP_TRY(c, launch_fill_set(fs, j.s));
        // One segment dealt on two digits, bases scanned ahead: its buckets are the
        // non-empty digit pairs, counted from the first digit's histogram and the second
        // deal's per-tile counts, so the keys need not be read again.
        const Seg& g0 = hs[active[0]];
        const bool from_counts = single && !c->force_key_heads && d == 2 && g0.first_pass == 0 &&
                                 g0.npass == 2 && g0.shift[0] != g0.shift[1] && !full[active[0]];
        if (from_counts) {
            JointArgs ja{};
            ja.keys = j.k[1 - cur];  // the first deal's output, intact after the second
            ja.seg_start = g0.start;
            ja.seg_len = g0.len;
            ja.h0 = dhist + ((size_t)active[0] * ndig + g0.hslot[0]) * RADIX;
            ja.tcnt = tone;
            ja.ntiles = (uint32_t)ntiles;
            ja.tile = j.tile;
            ja.shift1 = g0.shift[1];
            ja.width0 = g0.width[0];
            ja.width1 = g0.width[1];
            ja.joint = joint;
            ja.rows = joint_rows;
            ja.bstart = dbstart;
            ja.bseg = dbseg;
            ja.seg = active[0];
            ja.bcap = bcap;
            ja.nbuckets = counters;
            ja.err = j.err_dev;
            HIP_TRY(c, launch_joint_heads(kb, ja, j.s));
            c->stats.levels_heads_counts += 1;
        } else if (!c->force_key_heads && d == 1) {
            // Every segment dealt on one digit: its buckets are that digit's non-empty
            // values, from its histogram.
            std::vector<uint32_t> ids;
            for (uint32_t i : active)
                if (!full[i]) ids.push_back(i);
            st = upload(j, hh_ids, ids.data(), ids.size() * sizeof(uint32_t));
            if (st) return st;
            HistHeadArgs ha{};
            ha.segs = dsegs;
            ha.ids = hh_ids;
            ha.nids = (uint32_t)ids.size();
            ha.hist = dhist;
            ha.hist_digits = ndig;
            ha.first = hh_first;
            ha.bstart = dbstart;
            ha.bseg = dbseg;
            ha.bcap = bcap;
            ha.nbuckets = counters;
            ha.err = j.err_dev;
            HIP_TRY(c, launch_hist_heads(ha, j.s));
            c->stats.levels_heads_hist += 1;
        } else {
            HeadArgs ha{};
            ha.keys = j.k[cur];
            ha.tiles = dhtiles;
            ha.ntiles = (uint32_t)nht;
            ha.segs = dsegs;
            ha.tcount = htcount;
            ha.tbase = htbase;
            ha.tslot = htslot;
            ha.bstart = dbstart;
            ha.bseg = dbseg;
            ha.bcap = bcap;
            ha.nbuckets = counters;
            ha.err = j.err_dev;
            HIP_TRY(c, launch_heads(kb, ha, j.s));
            c->stats.levels_heads_keys += 1;
        }
        ClassifyArgs ca{};
        ca.bstart = dbstart;
        ca.bseg = dbseg;
        ca.nbuckets = counters;
        ca.bcap = bcap;
        ca.segs = dsegs;
        ca.wsmall = (uint32_t)wsmall;
        ca.cap = (uint32_t)j.cap;
        ca.kbits = 8 * kb;
        ca.cfirst = cfirst;
        ca.clast = clast;
        ca.nslots = (uint32_t)nslots;
        ca.med = med;
        ca.nmed = counters + 1;
        ca.medcap = (uint32_t)medcap;
        ca.big = big;
        ca.nbig = counters + 2;
        ca.bigcap = (uint32_t)bigcap;
        ca.done = done;
        ca.ndone = counters + 3;
        ca.donecap = (uint32_t)bigcap;
        ca.work = work;
        ca.nwork = counters + 5;
        ca.workcap = (uint32_t)(nslots + medcap);
        ca.err = j.err_dev;
        HIP_TRY(c, launch_classify(ca, (uint32_t)std::min<uint64_t>((bcap + 255) / 256, 4096), j.s));
    }
    // --- 5. local sort --------------------------------------------------------------
    {
        Timed tm(c, j.s, ST_LOCAL);
        LocalArgs la{};
        la.kin = j.k[cur];
        la.vin = j.v[cur];
        la.kout = j.k[0];
        la.vout = j.v[0];
        la.bstart = dbstart;
        la.bseg = dbseg;
        la.nbuckets = counters;
        la.bcap = bcap;
        la.segs = dsegs;
        la.cfirst = cfirst;
        la.clast = clast;
        la.nslots = (uint32_t)nslots;
        la.med = med;
        la.nmed = counters + 1;
        la.medcap = (uint32_t)medcap;
        la.work = work;
        la.nwork = counters + 5;
        la.workcap = (uint32_t)(nslots + medcap);
        la.desc = desc;
        la.spill = spill;
        la.nspill = counters + 4;
        la.spillcap = (uint32_t)(nslots + medcap);
        la.wide = wide;
        la.nwide = counters + 6;
        la.widecap = (uint32_t)(nslots + medcap);
        la.err = j.err_dev;
        la.stat = j.err_dev;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(nslots + medcap, 8192);
        // Bits a chunk's words need besides the position: the segment's lo_bit varying
        // bits, and the index of a bucket within a window's run of buckets (expected
        // from the buckets its dealt digits make, their values that occur, and the
        // window width).
        int max_lo = 0, max_index = 0;
        for (uint32_t i : active) {
            if (full[i]) continue;
            uint64_t nbk = 1;
            for (int p = 0; p < dsel[i] && p < (int)V[i].size(); ++p)
                nbk = std::min<uint64_t>(nbk * nonzero[i * ndig + V[i][p]], segs[i].len);
            const uint64_t per = std::max<uint64_t>(1, segs[i].len / std::max<uint64_t>(nbk, 1));
            const uint64_t run = std::max<uint64_t>(1, std::min<uint64_t>(wsmall / per, nbk));  // buckets per window
            const int ib = run > 1 ? 64 - __builtin_clzll(run - 1) : 0;
            max_lo = std::max(max_lo, (int)hs[i].lo_bit);
            max_index = std::max(max_index, (int)hs[i].lo_bit + ib);
        }
        HIP_TRY(c, launch_local_sort(kb, j.vb, la, blocks,
                                     local_sort_first_form(kb, j.vb, max_lo, max_index - max_lo), j.s));
    }
    c->stats.used_diversion = 1;

    // --- 6. large and finished buckets ----------------------------------------------
    st = pin_reserve(c, (STAT_WORDS + LEVEL_WORDS) * 4 + 2 * bigcap * sizeof(Big) + 256, j.s);
    if (st) return st;
    // The status block comes back with the counters, which follow it, in one copy: no
    // kernel after this point can change it unless another level runs (which clears
    // err_known).
    uint32_t* he = palloc<uint32_t>(c, STAT_WORDS + LEVEL_WORDS);
    uint32_t* hc = he + STAT_WORDS;
    HIP_TRY(c, hipMemcpyAsync(he, j.err_dev, (STAT_WORDS + LEVEL_WORDS) * 4, hipMemcpyDeviceToHost, j.s));
    // A level planned from its lengths brings its digit statistics back now, for the
    // estimated-bucket overflow of its top varying digit.
    char* h_plan = nullptr;
    if (from_lengths) {
        st = pin_reserve(c, readback + ALIGN, j.s);
        if (st) return st;
        h_plan = palloc<char>(c, readback);
        HIP_TRY(c, hipMemcpyAsync(h_plan, c->arena + off_coll, readback, hipMemcpyDeviceToHost, j.s));
    }
    HIP_TRY(c, hipStreamSynchronize(j.s));
    if (h_plan) {
        const uint32_t* h_ovf = (const uint32_t*)(h_plan + (off_ovf - off_coll));
        const uint64_t* h_or = (const uint64_t*)(h_plan + (off_or - off_coll));
        const uint64_t* h_and = (const uint64_t*)(h_plan + (off_and - off_coll));
        double ov = 0, len = 0;
        for (uint32_t i : active) {
            const uint64_t o = kb == 4 ? ((const uint32_t*)h_or)[i] : h_or[i];
            const uint64_t a = kb == 4 ? ((const uint32_t*)h_and)[i] : h_and[i];
            const std::vector<int> vv = varying_digits(o, a, kb, rb);
            if (!vv.empty()) ov += h_ovf[i * ndig + vv[0]];
            len += (double)segs[i].len;
        }
        c->stats.estimated_overflow = len > 0 ? ov / len : 0.0;
    }
    memcpy(j.stat_host, he, sizeof j.stat_host);
    j.err_word_host = he[STAT_ERR];
    j.err_known = true;
    const uint32_t nbig = std::min<uint32_t>(hc[2], (uint32_t)bigcap);
    const uint32_t ndone = std::min<uint32_t>(hc[3], (uint32_t)bigcap);
    c->stats.chunks += hc[5];  // work items listed by classify
    Big* hb = palloc<Big>(c, std::max<uint32_t>(nbig, 1));
    Big* hd = palloc<Big>(c, std::max<uint32_t>(ndone, 1));
    if (nbig) HIP_TRY(c, hipMemcpyAsync(hb, big, nbig * sizeof(Big), hipMemcpyDeviceToHost, j.s));
    if (ndone) HIP_TRY(c, hipMemcpyAsync(hd, done, ndone * sizeof(Big), hipMemcpyDeviceToHost, j.s));
    if (nbig || ndone) HIP_TRY(c, hipStreamSynchronize(j.s));
    std::vector<Big> bigs(hb, hb + nbig), dones(hd, hd + ndone);
    synced(c);
    c->stats.large_buckets += nbig;
    if (cur == 1 && !dones.empty()) {
        std::vector<std::pair<uint64_t, uint64_t>> r;
        for (auto& b : dones) r.push_back({b.start, b.len});
        st = copy_back(j, r);
        if (st) return st;
    }
    std::sort(bigs.begin(), bigs.end(), [](const Big& a, const Big& b) { return a.start < b.start; });
    for (auto& b : bigs) next.push_back(LSeg{b.start, b.len, (int)b.hi_bit});
    return DFR_OK;
}

// A first level dealt the Fast Radix way (Sec. 3): no count, the number of top digits
// estimated from n alone for uniform keys (Sec. 3.1: buckets of n / M^d records), and
// used only when that is two digits.  The lower digit is dealt into estimated buckets
// with an overflow area (k_deal_est), which also counts the upper digit; the upper
// digit is then dealt exactly, by decoupled look-back over the buckets in order, each
// bucket's estimated slots followed by its overflow slots.  Bucket heads come from the
// keys, then the runs of small buckets are diverted and the large ones recurse, as in
// deal_level.  *used is false (and nothing has been written) when the level does not
// qualify or a bucket outgrew its estimate and overflow slots: the caller then deals
// the level with counted buckets.
dfr_status est_level(Job& j, const LSeg& g, std::vector<LSeg>& next, bool* used) {
    dfr_ctx* c = j.c;
    *used = false;
    j.err_known = false;
    const int kb = j.kb, vb = j.vb, rb = j.rb;
    const int ndig = num_digits(kb, rb);
    const uint64_t n = g.len;
    if (g.start != 0 || g.hi_bit != 8 * kb || ndig < 2 || j.tile != deal_tile_records(kb, vb) ||
        n > DFR_MAX_SEGMENT_RECORDS)
        return DFR_OK;
    int d = 0;
    double expect = (double)n;
    while (d < ndig && expect > (double)j.divert) {
        expect /= (double)(1u << rb);
        ++d;
    }
    if (d != 2) return DFR_OK;
    const int du = ndig - 2, dw = ndig - 1;  // the two top digits: lower (estimated), upper (exact)
    const int su = rb * du, wu = std::min(rb, 8 * kb - su);
    const int sw = rb * dw, ww = std::min(rb, 8 * kb - sw);
    const uint32_t M = 1u << wu;
    const uint64_t E = n / M;
    // Overflow slots per bucket: four standard deviations of a bucket's count for
    // uniform keys, sqrt(E), at least 256; Eq. 2's expected overflow is far below that.
    const uint32_t C = (uint32_t)round_up(std::max<uint64_t>(256, (uint64_t)(4.0 * std::sqrt((double)E)) + 1), 64);
    const uint32_t T = j.tile;
    const uint64_t nt0 = (n + T - 1) / T;
    const uint64_t nt1 = nt0 + 2 * (uint64_t)M + 1;  // tiles of the exact pass, at most
    const uint64_t bcap = std::min<uint64_t>(n, (uint64_t)1 << (wu + ww));
    const size_t wsmall = j.wsmall;
    const uint64_t nslots = (n + wsmall - 1) / wsmall;
    const uint64_t medcap = n / (wsmall + 1), bigcap = n / (j.cap + 1);
    const size_t need = asize<uint64_t>(nt1 * RADIX + 1) + 3 * asize<uint32_t>(RADIX) + asize<uint32_t>(8) +
                        asize<char>((size_t)M * C * kb) + asize<char>((size_t)M * C * std::max(vb, 1)) +
                        asize<Tile>(nt1) + asize<Tile>(nt0) + asize<Seg>(1) + asize<uint32_t>(nt0) +
                        asize<uint64_t>(nt0) + asize<uint16_t>(nt0 * HEAD_SLOTS) + asize<uint64_t>(bcap) +
                        asize<uint32_t>(bcap) + 2 * asize<uint32_t>(nslots) + asize<uint32_t>(medcap) +
                        2 * asize<Big>(bigcap) + asize<uint32_t>(nslots + medcap) +
                        3 * asize<ChunkDesc>(nslots + medcap) + asize<uint32_t>(8);
    dfr_status st = arena_reserve(c, need, j.s);
    if (st) return st;
    uint64_t* lb = aalloc<uint64_t>(c, nt1 * RADIX + 1);
    uint32_t* cnt = aalloc<uint32_t>(c, RADIX);
    uint32_t* hist_w = aalloc<uint32_t>(c, RADIX);
    uint32_t* lost = aalloc<uint32_t>(c, 8);
    char* kovf = aalloc<char>(c, (size_t)M * C * kb);
    char* vovf = aalloc<char>(c, (size_t)M * C * std::max(vb, 1));
    Tile* tiles1 = aalloc<Tile>(c, nt1);
    Tile* htiles = aalloc<Tile>(c, nt0);
    Seg* dseg = aalloc<Seg>(c, 1);
    uint32_t* htcount = aalloc<uint32_t>(c, nt0);
    uint64_t* htbase = aalloc<uint64_t>(c, nt0);
    uint16_t* htslot = aalloc<uint16_t>(c, nt0 * HEAD_SLOTS);
    uint64_t* dbstart = aalloc<uint64_t>(c, bcap);
    uint32_t* dbseg = aalloc<uint32_t>(c, bcap);
    uint32_t* cfirst = aalloc<uint32_t>(c, nslots);
    uint32_t* clast = aalloc<uint32_t>(c, nslots);
    uint32_t* med = aalloc<uint32_t>(c, medcap);
    Big* big = aalloc<Big>(c, bigcap);
    Big* done = aalloc<Big>(c, bigcap);
    ChunkDesc* spill = aalloc<ChunkDesc>(c, nslots + medcap);
    uint32_t* work = aalloc<uint32_t>(c, nslots + medcap);
    ChunkDesc* wide = aalloc<ChunkDesc>(c, nslots + medcap);
    ChunkDesc* desc = aalloc<ChunkDesc>(c, nslots + medcap);
    uint32_t* counters = j.err_dev + STAT_WORDS;  // buckets, medium, big, done, spill, work, wide

    // --- the estimated deal of the lower digit into the temp buffer and overflow -----
    {
        Timed tz(c, j.s, ST_OTHER);
        FillSet fs{};
        fs.count = 4;
        fs.p[0] = lb, fs.v[0] = 0, fs.n[0] = nt0 * RADIX + 1, fs.w[0] = 8;
        fs.p[1] = cnt, fs.v[1] = 0, fs.n[1] = RADIX, fs.w[1] = 4;
        fs.p[2] = hist_w, fs.v[2] = 0, fs.n[2] = RADIX, fs.w[2] = 4;
        fs.p[3] = lost, fs.v[3] = 0, fs.n[3] = 8, fs.w[3] = 4;
        HIP_TRY(c, launch_fill_set(fs, j.s));
    }
    {
        Timed tm(c, j.s, ST_DEAL, true);
        EstArgs ea{};
        ea.kin = j.k[0];
        ea.vin = j.v[0];
        ea.kout = j.k[1];
        ea.vout = j.v[1];
        ea.kovf = kovf;
        ea.vovf = vovf;
        ea.n = n;
        ea.ntiles = (uint32_t)nt0;
        ea.tile = T;
        ea.shift = su;
        ea.width = wu;
        ea.nshift = sw;
        ea.nwidth = ww;
        ea.E = E;
        ea.C = C;
        ea.lookback = lb;
        ea.ticket = (uint32_t*)(lb + nt0 * RADIX);
        ea.cnt = cnt;
        ea.next_hist = hist_w;
        ea.lost = lost;
        ea.err = j.err_dev;
        HIP_TRY(c, launch_deal_est(kb, vb, ea, j.s));
    }
    // Bucket totals and lost records come back (the exact pass's tiles depend on them).
    st = pin_reserve(c, (RADIX + 8) * 4 + 64, j.s);
    if (st) return st;
    uint32_t* hcnt = palloc<uint32_t>(c, RADIX + 8);
    HIP_TRY(c, hipMemcpyAsync(hcnt, cnt, RADIX * 4, hipMemcpyDeviceToHost, j.s));
    HIP_TRY(c, hipMemcpyAsync(hcnt + RADIX, lost, 8 * 4, hipMemcpyDeviceToHost, j.s));
    HIP_TRY(c, hipStreamSynchronize(j.s));
    std::vector<uint32_t> bcount(hcnt, hcnt + M);
    const uint32_t nlost = hcnt[RADIX];
    synced(c);
    uint64_t total = 0, ovf = 0;
    for (uint32_t v = 0; v < M; ++v) {
        total += bcount[v];
        ovf += bcount[v] > E ? bcount[v] - E : 0;
    }
    if (nlost || total != n) return DFR_OK;  // a bucket outgrew its slots: deal it counted
    *used = true;
    c->stats.top_digits = 2;
    c->stats.deal_passes += 1;
    c->stats.deal_passes_estimated += 1;
    c->stats.estimated_overflow = (double)ovf / (double)n;

    // --- the exact deal of the upper digit, back into the caller's buffer --------------
    std::vector<Tile> t1;
    for (uint32_t v = 0; v < M; ++v) {
        const uint64_t inmain = std::min<uint64_t>(bcount[v], E), inovf = bcount[v] - inmain;
        for (uint64_t o = 0; o < inmain; o += T)
            t1.push_back(Tile{(uint64_t)v * E + o, (uint32_t)std::min<uint64_t>(T, inmain - o), 0});
        for (uint64_t o = 0; o < inovf; o += T)
            t1.push_back(Tile{(uint64_t)v * C + o, (uint32_t)std::min<uint64_t>(T, inovf - o), TILE_IN2});
    }
    Seg sg{};
    sg.start = 0;
    sg.len = n;
    sg.first_tile = 0;
    sg.npass = 1;
    sg.shift[0] = (int8_t)sw;
    sg.width[0] = (int8_t)ww;
    sg.hslot[0] = 0;
    sg.lo_bit = su;
    st = upload(j, tiles1, t1.data(), t1.size() * sizeof(Tile));
    if (!st) st = upload(j, dseg, &sg, sizeof sg);
    if (st) return st;
    HIP_TRY(c, launch_fill_u64(lb, 0, t1.size() * RADIX + 1, j.s));
    {
        Timed tm(c, j.s, ST_DEAL, true);
        DealArgs da{};
        da.off = nullptr;  // look-back
        da.tile = T;
        da.kin = j.k[1];
        da.vin = j.v[1];
        da.kin2 = kovf;
        da.vin2 = vb ? vovf : nullptr;
        da.kout = j.k[0];
        da.vout = j.v[0];
        da.tiles = tiles1;
        da.ntiles = (uint32_t)t1.size();
        da.segs = dseg;
        da.hist = hist_w;
        da.hist_digits = 1;
        da.pass = 0;
        da.lookback = lb;
        da.ticket = (uint32_t*)(lb + t1.size() * RADIX);
        da.err = j.err_dev;
        HIP_TRY(c, launch_deal(kb, vb, da, j.s));
    }
    c->stats.deal_passes += 1;
    c->stats.deal_passes_lookback += 1;

    // --- buckets (from the keys), classify, local sort ----------------------------------
    std::vector<Tile> ht;
    std::vector<uint32_t> ft;
    build_tiles(std::vector<LSeg>{LSeg{0, n, 8 * kb}}, std::vector<uint32_t>{0}, T, ht, ft);
    st = upload(j, htiles, ht.data(), ht.size() * sizeof(Tile));
    if (st) return st;
    {
        Timed tm(c, j.s, ST_BUCKETS);
        FillSet fs{};
        fs.count = 3;
        fs.p[0] = counters, fs.v[0] = 0, fs.n[0] = 8, fs.w[0] = 4;
        fs.p[1] = cfirst, fs.v[1] = 0xffffffffu, fs.n[1] = nslots, fs.w[1] = 4;
        fs.p[2] = clast, fs.v[2] = 0, fs.n[2] = nslots, fs.w[2] = 4;
        HIP_TRY(c, launch_fill_set(fs, j.s));
        HeadArgs ha{};
        ha.keys = j.k[0];
        ha.tiles = htiles;
        ha.ntiles = (uint32_t)ht.size();
        ha.segs = dseg;
        ha.tcount = htcount;
        ha.tbase = htbase;
        ha.tslot = htslot;
        ha.bstart = dbstart;
        ha.bseg = dbseg;
        ha.bcap = bcap;
        ha.nbuckets = counters;
        ha.err = j.err_dev;
        HIP_TRY(c, launch_heads(kb, ha, j.s));
        c->stats.levels_heads_keys += 1;
        ClassifyArgs ca{};
        ca.bstart = dbstart;
        ca.bseg = dbseg;
        ca.nbuckets = counters;
        ca.bcap = bcap;
        ca.segs = dseg;
        ca.wsmall = (uint32_t)wsmall;
        ca.cap = (uint32_t)j.cap;
        ca.kbits = 8 * kb;
        ca.cfirst = cfirst;
        ca.clast = clast;
        ca.nslots = (uint32_t)nslots;
        ca.med = med;
        ca.nmed = counters + 1;
        ca.medcap = (uint32_t)medcap;
        ca.big = big;
        ca.nbig = counters + 2;
        ca.bigcap = (uint32_t)bigcap;
        ca.done = done;
        ca.ndone = counters + 3;
        ca.donecap = (uint32_t)bigcap;
        ca.work = work;
        ca.nwork = counters + 5;
        ca.workcap = (uint32_t)(nslots + medcap);
        ca.err = j.err_dev;
        HIP_TRY(c, launch_classify(ca, (uint32_t)std::min<uint64_t>((bcap + 255) / 256, 4096), j.s));
    }
    {
        Timed tm(c, j.s, ST_LOCAL);
        LocalArgs la{};
        la.kin = j.k[0];
        la.vin = j.v[0];
        la.kout = j.k[0];
        la.vout = j.v[0];
        la.bstart = dbstart;
        la.bseg = dbseg;
        la.nbuckets = counters;
        la.bcap = bcap;
        la.segs = dseg;
        la.cfirst = cfirst;
        la.clast = clast;
        la.nslots = (uint32_t)nslots;
        la.med = med;
        la.nmed = counters + 1;
        la.medcap = (uint32_t)medcap;
        la.work = work;
        la.nwork = counters + 5;
        la.workcap = (uint32_t)(nslots + medcap);
        la.desc = desc;
        la.spill = spill;
        la.nspill = counters + 4;
        la.spillcap = (uint32_t)(nslots + medcap);
        la.wide = wide;
        la.nwide = counters + 6;
        la.widecap = (uint32_t)(nslots + medcap);
        la.err = j.err_dev;
        la.stat = j.err_dev;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(nslots + medcap, 8192);
        HIP_TRY(c, launch_local_sort(kb, vb, la, blocks, local_sort_first_form(kb, vb, su, 0), j.s));
    }
    c->stats.used_diversion = 1;
    // --- large buckets: the next level's segments --------------------------------------
    st = pin_reserve(c, (STAT_WORDS + LEVEL_WORDS) * 4 + bigcap * sizeof(Big) + 256, j.s);
    if (st) return st;
    uint32_t* he = palloc<uint32_t>(c, STAT_WORDS + LEVEL_WORDS);
    uint32_t* hc = he + STAT_WORDS;
    HIP_TRY(c, hipMemcpyAsync(he, j.err_dev, (STAT_WORDS + LEVEL_WORDS) * 4, hipMemcpyDeviceToHost, j.s));
    HIP_TRY(c, hipStreamSynchronize(j.s));
    memcpy(j.stat_host, he, sizeof j.stat_host);
    j.err_word_host = he[STAT_ERR];
    j.err_known = true;
    const uint32_t nbig = std::min<uint32_t>(hc[2], (uint32_t)bigcap);
    c->stats.chunks += hc[5];
    Big* hb = palloc<Big>(c, std::max<uint32_t>(nbig, 1));
    if (nbig) {
        HIP_TRY(c, hipMemcpyAsync(hb, big, nbig * sizeof(Big), hipMemcpyDeviceToHost, j.s));
        HIP_TRY(c, hipStreamSynchronize(j.s));
    }
    std::vector<Big> bigs(hb, hb + nbig);
    synced(c);
    c->stats.large_buckets += nbig;
    std::sort(bigs.begin(), bigs.end(), [](const Big& a, const Big& b) { return a.start < b.start; });
    for (auto& b : bigs) next.push_back(LSeg{b.start, b.len, (int)b.hi_bit});
    return DFR_OK;
}

dfr_status check_err(Job& j) {
    dfr_ctx* c = j.c;
    uint32_t e = j.err_word_host;
    if (!j.err_known) {
        dfr_status st = pin_reserve(c, 64 + STAT_WORDS * 4, j.s);
        if (st) return st;
        uint32_t* h = palloc<uint32_t>(c, STAT_WORDS);
        HIP_TRY(c, hipMemcpyAsync(h, j.err_dev, STAT_WORDS * 4, hipMemcpyDeviceToHost, j.s));
        HIP_TRY(c, hipStreamSynchronize(j.s));
        memcpy(j.stat_host, h, sizeof j.stat_host);
        e = h[STAT_ERR];
        synced(c);
    }
    c->stats.chunks_form0 = j.stat_host[STAT_FORM0];
    c->stats.chunks_form1 = j.stat_host[STAT_FORM0 + 1];
    c->stats.chunks_form2 = j.stat_host[STAT_FORM0 + 2];
    c->stats.chunks_general = j.stat_host[STAT_GENERAL];
    if (e) {
        char buf[128];
        snprintf(buf, sizeof buf, "device error word 0x%x", e);
        c->err = buf;
        return DFR_E_INTERNAL;
    }
    return DFR_OK;
}

dfr_status run_sort(dfr_ctx* c, int kb, int vb, void* keys, void* vals, const std::vector<LSeg>& segs0,
                    void* temp, hipStream_t s, const dfr_tune* forced = nullptr) {
    Job j;
    j.c = c;
    j.kb = kb;
    j.vb = vb;
    j.s = s;
    j.cap = local_cap(kb, vb);
    const dfr_tune t = forced ? *forced : effective_tune(c, kb, vb, size_class(segs0));
    j.tile = t.tile_records;
    j.rb = t.radix_bits;
    j.wsmall = t.window_records;
    j.window_default = !forced && !c->window &&
                       c->tunes.find(tune_key(kb, vb, size_class(segs0))) == c->tunes.end();
    j.divert = t.divert_records;
    j.top_d_forced = c->force_d;
    uint64_t n = 0;
    for (auto& g : segs0) n = std::max(n, g.start + g.len);
    j.k[0] = keys;
    j.v[0] = vals;
    j.k[1] = temp;
    j.v[1] = vb ? (char*)temp + round_up(n * kb, ALIGN) : nullptr;

    c->stats = dfr_stats{};
    c->events.clear();
    dfr_status st = DFR_OK;
    if (!c->err_dev) HIP_TRY(c, hipMalloc((void**)&c->err_dev, ALIGN));
    j.err_dev = c->err_dev;
    HIP_TRY(c, launch_fill_u32(j.err_dev, 0, STAT_WORDS, s));

    std::vector<LSeg> small, large;
    for (auto& g : segs0) {
        if (g.len <= 1) continue;  // one record is sorted where it is
        if (g.len <= j.cap) small.push_back(g);
        else large.push_back(g);
    }
    int level = 0;
    if (!small.empty()) {
        st = divert_level(j, small, 0);
        if (st) return st;
        level = 1;
    }
    int in = 0;
    while (!large.empty()) {
        std::vector<LSeg> next;
        int next_in = in;
        bool est = false;
        if (c->est_buckets && j.first_level && small.empty() && large.size() == 1 && !forced) {
            st = est_level(j, large[0], next, &est);
            if (st) return st;
        }
        if (!est) st = deal_level(j, large, in, next, &next_in);
        if (st) return st;
        j.first_level = false;
        ++level;
        large.swap(next);
        in = next_in;
        // Buckets of the next level that fit the local sort do not exist: every
        // listed bucket exceeds the capacity.
    }
    c->stats.levels = level;
    st = check_err(j);
    if (c->timing) collect_events(c);
    return st;
}

bool overlap(const void* a, size_t an, const void* b, size_t bn) {
    if (!a || !b || an == 0 || bn == 0) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

dfr_status validate(dfr_ctx* c, const void* keys, const void* vals, size_t n, int kb, int vb,
                    const void* temp, size_t temp_bytes) {
    if (!c) return DFR_E_INVALID_ARG;
    if (c->failed) return DFR_E_HIP;
    if (!(kb == 4 || kb == 8) || !(vb == 0 || vb == 4 || vb == 8)) return DFR_E_INVALID_ARG;
    if (n == 0) return DFR_OK;
    if (!keys) return DFR_E_INVALID_ARG;
    if ((uintptr_t)keys % kb) return DFR_E_INVALID_ARG;
    if (vb && (!vals || (uintptr_t)vals % vb)) return DFR_E_INVALID_ARG;
    if (temp) {
        if (temp_bytes < dfr_temp_bytes(n, kb, vb)) return DFR_E_INVALID_ARG;
        if ((uintptr_t)temp % 16) return DFR_E_INVALID_ARG;
        if (overlap(temp, temp_bytes, keys, n * kb) || (vb && overlap(temp, temp_bytes, vals, n * vb)))
            return DFR_E_INVALID_ARG;
    }
    if (vb && overlap(keys, n * kb, vals, n * vb)) return DFR_E_INVALID_ARG;
    return DFR_OK;
}

dfr_status get_temp(dfr_ctx* c, size_t n, int kb, int vb, void** temp, hipStream_t s) {
    if (*temp) return DFR_OK;
    const size_t need = dfr_temp_bytes(n, kb, vb);
    if (c->tcache_cap < need) {
        const auto t0 = std::chrono::steady_clock::now();
        HIP_TRY(c, hipStreamSynchronize(s));
        if (c->tcache) HIP_TRY(c, hipFree(c->tcache));
        c->tcache = nullptr;
        c->tcache_cap = 0;
        const size_t cap = round_up(need + need / 8 * c->temp_slack, 1 << 20);
        hipError_t e = hipMalloc(&c->tcache, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            c->err = "temp allocation failed";
            return DFR_E_NO_MEMORY;
        }
        c->tcache_cap = cap;
        c->n_allocs += 1;
        c->ms_alloc += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    *temp = c->tcache;
    return DFR_OK;
}

dfr_status set_device(dfr_ctx* c) {
    HIP_TRY(c, hipSetDevice(c->device));
    return DFR_OK;
}

// Stream order of one call against the context's previous call (see dfr_ctx::done).
struct CallOrder {
    dfr_ctx* c;
    hipStream_t s;
    dfr_status st = DFR_OK;
    CallOrder(dfr_ctx* c_, hipStream_t s_) : c(c_), s(s_) {
        if (c->have_last && c->last_stream != s) {
            const hipError_t e = hipStreamWaitEvent(s, c->done, 0);
            if (e != hipSuccess) st = fail_hip(c, e, "hipStreamWaitEvent");
        }
    }
    ~CallOrder() {
        if (hipEventRecord(c->done, s) == hipSuccess) {
            c->last_stream = s;
            c->have_last = true;
        } else {
            (void)hipGetLastError();
            c->have_last = false;
        }
    }
};

// run_sort between the in-place map of signed or float keys to unsigned ones and its
// inverse (mode 0: unsigned keys, no map).
dfr_status run_sort_mapped(dfr_ctx* c, int kb, int vb, int mode, void* keys, void* vals, size_t n,
                           const std::vector<LSeg>& segs, void* temp, hipStream_t s) {
    if (mode) {
        Timed tm(c, s, ST_OTHER);
        HIP_TRY(c, launch_key_transform(kb, mode, false, keys, n, s));
    }
    dfr_status st = run_sort(c, kb, vb, keys, vals, segs, temp, s);
    if (mode) {
        // Mapped back even after a failed sort, so the keys stay valid encodings.
        Timed tm(c, s, ST_OTHER);
        const hipError_t e = launch_key_transform(kb, mode, true, keys, n, s);
        if (!st && e != hipSuccess) return fail_hip(c, e, "key map");
    }
    return st;
}

dfr_status sort_plain(dfr_ctx* c, int kb, int vb, void* keys, void* vals, size_t n, void* temp,
                      size_t temp_bytes, void* stream, int mode = 0) {
    dfr_status st = validate(c, keys, vals, n, kb, vb, temp, temp_bytes);
    if (st) return st;
    if (n > DFR_MAX_SEGMENT_RECORDS) return DFR_E_TOO_LARGE;
    if (n <= 1) {
        c->stats = dfr_stats{};
        return DFR_OK;
    }
    st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    st = get_temp(c, n, kb, vb, &temp, s);
    if (st) return st;
    std::vector<LSeg> segs{LSeg{0, n, 8 * kb}};
    return run_sort_mapped(c, kb, vb, mode, keys, vb ? vals : nullptr, n, segs, temp, s);
}

// Segments from host offsets (S + 1 entries, [0] = 0, non-decreasing).
dfr_status parse_segments(const uint64_t* off, size_t S, int kb, std::vector<LSeg>& segs) {
    if (!off) return DFR_E_INVALID_ARG;
    if (off[0] != 0) return DFR_E_INVALID_ARG;
    for (size_t i = 0; i < S; ++i)
        if (off[i + 1] < off[i]) return DFR_E_INVALID_ARG;
    segs.clear();
    segs.reserve(S);
    for (size_t i = 0; i < S; ++i) {
        const uint64_t len = off[i + 1] - off[i];
        if (len > DFR_MAX_SEGMENT_RECORDS) return DFR_E_TOO_LARGE;
        segs.push_back(LSeg{off[i], len, 8 * kb});
    }
    return DFR_OK;
}

// Segment offsets as a host array: device memory is copied back after the work already
// queued on the stream (the caller's stream order), host memory is used as it is.
dfr_status host_offsets(dfr_ctx* c, const uint64_t* off, size_t S, hipStream_t s,
                        std::vector<uint64_t>& buf, const uint64_t** out) {
    *out = off;
    if (!off) return DFR_E_INVALID_ARG;
    hipPointerAttribute_t attr{};
    const hipError_t e = hipPointerGetAttributes(&attr, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // ordinary host memory is not known to HIP
        return DFR_OK;
    }
    if (attr.type != hipMemoryTypeDevice) return DFR_OK;
    buf.resize(S + 1);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(buf.data(), off, (S + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    *out = buf.data();
    return DFR_OK;
}

dfr_status sort_segmented(dfr_ctx* c, int kb, int vb, void* keys, void* vals, const uint64_t* off_in,
                          size_t S, void* temp, size_t temp_bytes, void* stream, int mode = 0) {
    if (!c) return DFR_E_INVALID_ARG;
    std::vector<LSeg> segs;
    std::vector<uint64_t> off_buf;
    const uint64_t* off = nullptr;
    dfr_status st0 = host_offsets(c, off_in, S, (hipStream_t)stream, off_buf, &off);
    if (st0) return st0;
    const size_t n = off[S];
    dfr_status st = validate(c, keys, vals, n, kb, vb, temp, temp_bytes);
    if (st) return st;
    st = parse_segments(off, S, kb, segs);
    if (st) return st;
    if (n <= 1) {
        c->stats = dfr_stats{};
        return DFR_OK;
    }
    st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    st = get_temp(c, n, kb, vb, &temp, s);
    if (st) return st;
    return run_sort_mapped(c, kb, vb, mode, keys, vb ? vals : nullptr, n, segs, temp, s);
}

// Key bytes and map mode (0 unsigned, 1 signed, 2 float) of a DFR_KEY_* code; false if
// the code is unknown.
bool key_type_info(int32_t key_type, int* kb, int* mode) {
    if (key_type < DFR_KEY_U32 || key_type > DFR_KEY_F64) return false;
    *kb = key_type % 2 == 0 ? 4 : 8;
    *mode = key_type / 2;
    return true;
}

// One timed sort of fresh copies of the caller's data under tuning t.
dfr_status time_sort(dfr_ctx* c, int kb, int vb, const void* keys, const void* vals, void* kw,
                     void* vw, size_t n, const std::vector<LSeg>& segs, void* temp, hipStream_t s,
                     const dfr_tune& t, int reps, hipEvent_t e0, hipEvent_t e1, double* ms) {
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(c, hipMemcpyAsync(kw, keys, n * kb, hipMemcpyDeviceToDevice, s));
        if (vb) HIP_TRY(c, hipMemcpyAsync(vw, vals, n * vb, hipMemcpyDeviceToDevice, s));
        HIP_TRY(c, hipEventRecord(e0, s));
        dfr_status st = run_sort(c, kb, vb, kw, vb ? vw : nullptr, segs, temp, s, &t);
        if (st) return st;
        HIP_TRY(c, hipEventRecord(e1, s));
        HIP_TRY(c, hipEventSynchronize(e1));
        float f = 0;
        HIP_TRY(c, hipEventElapsedTime(&f, e0, e1));
        best = std::min(best, (double)f);
    }
    *ms = best;
    return DFR_OK;
}

// Coordinate descent over the settings, two sweeps, from the defaults.
dfr_status autotune(dfr_ctx* c, int kb, int vb, const void* keys, const void* vals,
                    const std::vector<LSeg>& segs, size_t n, int reps, hipStream_t s, dfr_tune* out) {
    void* temp = nullptr;
    dfr_status st = get_temp(c, n, kb, vb, &temp, s);
    if (st) return st;
    void *kw = nullptr, *vw = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (kw) (void)hipFree(kw);
        if (vw) (void)hipFree(vw);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&kw, n * kb) != hipSuccess || (vb && hipMalloc(&vw, n * vb) != hipSuccess)) {
        (void)hipGetLastError();
        cleanup();
        c->err = "autotune: copy buffers";
        return DFR_E_NO_MEMORY;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail_hip(c, hipErrorUnknown, "autotune: events");
    }
    const int timing = c->timing;
    c->timing = 0;
    const size_t cap = local_cap(kb, vb);
    const uint32_t tile = deal_tile_records(kb, vb);
    std::vector<std::vector<uint64_t>> choices = {
        kb == 4 ? std::vector<uint64_t>{6, 7, 8} : std::vector<uint64_t>{8},
        {tile, tile / 2},
        {cap / 4, cap / 2, cap * 3 / 4, cap},
        {cap / 8, cap / 4, cap / 2},
    };
    auto with = [](dfr_tune t, int knob, uint64_t v) {
        if (knob == 0) t.radix_bits = (int32_t)v;
        else if (knob == 1) t.tile_records = (uint32_t)v;
        else if (knob == 2) t.divert_records = v;
        else t.window_records = v;
        return t;
    };
    auto get = [](const dfr_tune& t, int knob) -> uint64_t {
        return knob == 0 ? (uint64_t)t.radix_bits : knob == 1 ? t.tile_records
                                                 : knob == 2 ? t.divert_records : t.window_records;
    };
    dfr_tune best = default_tune(kb, vb);
    double best_ms = 0;
    st = time_sort(c, kb, vb, keys, vals, kw, vw, n, segs, temp, s, best, reps, e0, e1, &best_ms);
    const double default_ms = best_ms;
    for (int sweep = 0; sweep < 2 && !st; ++sweep) {
        for (int knob = 0; knob < 4 && !st; ++knob) {
            for (uint64_t v : choices[knob]) {
                if (v == get(best, knob)) continue;
                const dfr_tune t = with(best, knob, v);
                if (!tune_valid(t, kb, vb)) continue;
                double ms = 0;
                st = time_sort(c, kb, vb, keys, vals, kw, vw, n, segs, temp, s, t, reps, e0, e1, &ms);
                if (st) break;
                if (ms < best_ms * 0.99) {  // keep the incumbent on near ties
                    best = t;
                    best_ms = ms;
                }
            }
        }
    }
    c->timing = timing;
    cleanup();
    if (st) return st;
    best.ms = best_ms;
    best.ms_default = default_ms;
    c->tunes[tune_key(kb, vb, size_class(segs))] = best;
    if (out) *out = best;
    return DFR_OK;
}

}  // namespace

// =================================================================================
// Request serving: continuous batching of queued sort requests.
//
// Worker threads, each with its own stream and its own scratch (an internal context),
// take the oldest queued request and every later queued request of the same widths
// up to a record limit, and sort them as one segmented sort: the requests' records
// are gathered into one staging buffer, sorted segment by segment, and scattered back
// (a batch of one request is sorted in place).  While one worker's batch is on the
// device, another worker forms and launches the next one from requests that arrived
// meanwhile, so batches overlap on the device.  Device memory held by the workers
// (staging, temp and scratch) stays within the context's HBM budget: a batch shrinks,
// or a worker frees its caches, or it waits for another to finish, before it
// allocates past the budget.
// =================================================================================
struct Server {
    struct Req {
        uint64_t ticket;
        dfr_request r;
        std::chrono::steady_clock::time_point t_submit;
    };
    struct Done {
        dfr_status st;
        double latency;
    };
    struct Worker {
        dfr_ctx* w = nullptr;  // internal context: arena, pinned staging, temp cache
        hipStream_t s = nullptr;
        void* sk = nullptr;    // staging for gathered batches
        void* sv = nullptr;
        size_t skcap = 0, svcap = 0;
        size_t held = 0;       // device bytes counted against the budget
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // phase boundaries
    };
    dfr_ctx* owner = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, char> running;
    uint64_t next_ticket = 1;
    bool stop = false;
    size_t budget = 0;
    uint64_t batch_records = 0;
    uint64_t gather_records = 0;
    size_t held = 0;
    std::vector<Worker> workers;
    std::vector<std::thread> threads;
    dfr_serve_stats stats{};
};

namespace {

size_t worker_bytes(const Server::Worker& wk) {
    return wk.skcap + wk.svcap + (wk.w ? wk.w->arena_cap + wk.w->tcache_cap : 0);
}

// Device bytes a batch of `n` records may need: the temp buffer, staging when the
// records are gathered, and the sort's own scratch (lists of tiles, buckets and
// chunks: at most about 24 bytes per record, plus a fixed part).
size_t batch_bytes(uint64_t n, int kb, int vb, bool gather) {
    const size_t rec = (size_t)kb + vb;
    return n * rec * (gather ? 2 : 1) + n * 24 + (64u << 20);
}

void free_worker_buffers(Server::Worker& wk) {
    (void)hipStreamSynchronize(wk.s);
    if (wk.sk) (void)hipFree(wk.sk);
    if (wk.sv) (void)hipFree(wk.sv);
    wk.sk = wk.sv = nullptr;
    wk.skcap = wk.svcap = 0;
    dfr_ctx* w = wk.w;
    if (w->arena) (void)hipFree(w->arena);
    if (w->tcache) (void)hipFree(w->tcache);
    w->arena = nullptr;
    w->arena_cap = w->arena_used = 0;
    w->tcache = nullptr;
    w->tcache_cap = 0;
}

dfr_status grow(dfr_ctx* w, void** p, size_t* cap, size_t need) {
    if (need <= *cap) return DFR_OK;
    const auto t0 = std::chrono::steady_clock::now();
    if (*p) HIP_TRY(w, hipFree(*p));
    *p = nullptr;
    *cap = 0;
    const size_t c = round_up(need + need / 2, 1 << 20);
    if (hipMalloc(p, c) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        w->err = "staging allocation failed";
        return DFR_E_NO_MEMORY;
    }
    *cap = c;
    w->n_allocs += 1;
    w->ms_alloc += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return DFR_OK;
}

// Place of each request in the staging buffers: consecutive, each starting on a
// 256-byte boundary (segments of a sort need not be adjacent), so that the copies
// between a request's buffer and its place move aligned vectors.
std::vector<uint64_t> batch_places(const std::vector<Server::Req>& b, uint64_t* end) {
    std::vector<uint64_t> pos;
    uint64_t p = 0;
    for (const Server::Req& q : b) {
        const uint64_t align = ALIGN / q.r.key_bytes;  // records per 256 bytes
        p = (p + align - 1) / align * align;
        pos.push_back(p);
        p += q.r.n;
    }
    *end = p;
    return pos;
}

// Chunks of at most 2^13 records over the batch's requests, between the requests'
// buffers and their places in the staging buffers (one block copies one chunk).
void batch_chunks(const std::vector<Server::Req>& b, void* sk, void* sv, bool to_staging,
                  std::vector<CopyChunk>& out) {
    out.clear();
    uint64_t end = 0;
    const std::vector<uint64_t> place = batch_places(b, &end);
    for (size_t r = 0; r < b.size(); ++r) {
        const Server::Req& q = b[r];
        const int kb = q.r.key_bytes, vb = q.r.val_bytes;
        const uint64_t pos = place[r];
        for (uint64_t o = 0; o < q.r.n; o += 1u << 13) {
            const uint32_t len = (uint32_t)std::min<uint64_t>(1u << 13, q.r.n - o);
            char* rk = (char*)q.r.keys + o * kb;
            char* rv = vb ? (char*)q.r.vals + o * vb : nullptr;
            char* gk = (char*)sk + (pos + o) * kb;
            char* gv = vb ? (char*)sv + (pos + o) * vb : nullptr;
            CopyChunk ch{};
            ch.ksrc = to_staging ? rk : gk;
            ch.kdst = to_staging ? gk : rk;
            ch.vsrc = to_staging ? rv : gv;
            ch.vdst = to_staging ? gv : rv;
            ch.len = len;
            out.push_back(ch);
        }
    }
}

dfr_status copy_batch(Job& j, const std::vector<Server::Req>& b, void* sk, void* sv, bool to_staging) {
    std::vector<CopyChunk> ch;
    batch_chunks(b, sk, sv, to_staging, ch);
    if (ch.empty()) return DFR_OK;
    dfr_status st = arena_reserve(j.c, asize<CopyChunk>(ch.size()), j.s);
    if (st) return st;
    CopyChunk* d = aalloc<CopyChunk>(j.c, ch.size());
    st = upload(j, d, ch.data(), ch.size() * sizeof(CopyChunk));
    if (st) return st;
    HIP_TRY(j.c, launch_copy_chunks(j.kb, j.vb, d, (uint32_t)ch.size(), j.s));
    return DFR_OK;
}

// Sort one batch on the worker's stream and wait for it; ms[0..2] receive the device
// time of the gather, the sort and the scatter.  Once anything may have been queued the
// function always reaches the stream synchronisation, whatever fails; inject_fail marks
// the batch failed at that point (the serving test hook).
dfr_status run_batch(Server::Worker& wk, const std::vector<Server::Req>& b, double* ms, bool inject_fail) {
    dfr_ctx* w = wk.w;
    ms[0] = ms[1] = ms[2] = 0;
    const int kb = b[0].r.key_bytes, vb = b[0].r.val_bytes;
    uint64_t n = 0, records = 0;
    const std::vector<uint64_t> place = batch_places(b, &n);
    std::vector<LSeg> segs;
    for (size_t r = 0; r < b.size(); ++r) {
        segs.push_back(LSeg{place[r], b[r].r.n, 8 * kb});
        records += b[r].r.n;
    }
    if (records <= 1) return DFR_OK;
    void* temp = nullptr;
    dfr_status st = get_temp(w, n, kb, vb, &temp, wk.s);
    if (st) return st;
    const bool gather = b.size() > 1;
    if (gather) {
        st = grow(w, &wk.sk, &wk.skcap, n * kb);
        if (!st && vb) st = grow(w, &wk.sv, &wk.svcap, n * vb);
        if (st) return st;  // nothing of this batch is queued yet
    }
    auto mark = [&](int i) {
        const hipError_t e = hipEventRecord(wk.ev[i], wk.s);
        if (e != hipSuccess && !st) st = fail_hip(w, e, "hipEventRecord");
    };
    if (!gather) {
        mark(1);
        if (!st) st = run_sort(w, kb, vb, b[0].r.keys, vb ? b[0].r.vals : nullptr, segs, temp, wk.s);
        if (!st) mark(2);
    } else {
        Job j;
        j.c = w;
        j.kb = kb;
        j.vb = vb;
        j.s = wk.s;
        mark(0);
        if (!st) st = copy_batch(j, b, wk.sk, wk.sv, true);
        if (!st) mark(1);
        if (!st) st = run_sort(w, kb, vb, wk.sk, vb ? wk.sv : nullptr, segs, temp, wk.s);
        if (!st) mark(2);
        if (!st) st = copy_batch(j, b, wk.sk, wk.sv, false);
        if (!st) mark(3);
    }
    if (!st && inject_fail) {
        st = DFR_E_HIP;
        w->err = "failure injected by the serve_fail_batches option";
    }
    // Wait for the batch's device work whatever its status: the requests' buffers are
    // handed back to their callers once their tickets are done.
    const hipError_t sync_err = hipStreamSynchronize(wk.s);
    if (!st && sync_err != hipSuccess) st = fail_hip(w, sync_err, "hipStreamSynchronize");
    (void)hipGetLastError();
    synced(w);
    if (!st) {
        float f = 0;
        if (gather && hipEventElapsedTime(&f, wk.ev[0], wk.ev[1]) == hipSuccess) ms[0] = f;
        if (hipEventElapsedTime(&f, wk.ev[1], wk.ev[2]) == hipSuccess) ms[1] = f;
        if (gather && hipEventElapsedTime(&f, wk.ev[2], wk.ev[3]) == hipSuccess) ms[2] = f;
    }
    return st;
}

void worker_loop(Server* sv, int wi) {
    Server::Worker& wk = sv->workers[wi];
    (void)hipSetDevice(sv->owner->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
        if (sv->stop) break;
        // The oldest request, then later ones of the same widths, within the limit.  A
        // request above the gather limit is sorted alone, in place (gathering it would
        // copy it twice), and is not gathered into another's batch.
        const Server::Req& head = sv->pending.front();
        const int kb = head.r.key_bytes, vb = head.r.val_bytes;
        std::vector<size_t> pick{0};
        uint64_t total = head.r.n;
        for (size_t i = 1; i < sv->pending.size() && head.r.n <= sv->gather_records; ++i) {
            const Server::Req& q = sv->pending[i];
            if (q.r.key_bytes != kb || q.r.val_bytes != vb) continue;
            if (q.r.n > sv->gather_records || total + q.r.n > sv->batch_records) continue;
            pick.push_back(i);
            total += q.r.n;
        }
        // Budget: drop the newest picks until the batch fits beside the other
        // workers' memory; a lone request that does not fit frees this worker's
        // caches, then waits for the others.
        auto need_of = [&](uint64_t t, size_t cnt) { return batch_bytes(t, kb, vb, cnt > 1); };
        bool fits = false;
        while (!fits) {
            const size_t others = sv->held - wk.held;
            const size_t need = need_of(total, pick.size());
            if (!sv->budget || others + std::max(need, wk.held) <= sv->budget) {
                fits = true;
            } else if (pick.size() > 1) {
                total -= sv->pending[pick.back()].r.n;
                pick.pop_back();
            } else {
                break;
            }
        }
        if (!fits) {
            if (wk.held) {
                lk.unlock();
                free_worker_buffers(wk);
                lk.lock();
                sv->held -= wk.held;
                wk.held = 0;
                sv->cv.notify_all();
                continue;
            }
            sv->cv.wait(lk);
            continue;
        }
        std::vector<Server::Req> batch;
        for (size_t k = 0; k < pick.size(); ++k) batch.push_back(sv->pending[pick[k]]);
        for (size_t k = pick.size(); k-- > 0;) sv->pending.erase(sv->pending.begin() + pick[k]);
        for (const Server::Req& q : batch) sv->running[q.ticket] = 1;
        // Count the batch's memory before it is allocated.
        const size_t reserve = std::max(need_of(total, batch.size()), wk.held);
        sv->held += reserve - wk.held;
        wk.held = reserve;
        sv->stats.peak_held_bytes = std::max<uint64_t>(sv->stats.peak_held_bytes, sv->held);
        lk.unlock();

        const auto t_start = std::chrono::steady_clock::now();
        double ms[3];
        const uint64_t allocs0 = wk.w->n_allocs;
        const double ms_alloc0 = wk.w->ms_alloc;
        bool inject = false;
        for (int f = sv->owner->serve_fail_batches.load(); f > 0 && !inject;)
            inject = sv->owner->serve_fail_batches.compare_exchange_weak(f, f - 1);
        const dfr_status st = run_batch(wk, batch, ms, inject);
        const auto t_end = std::chrono::steady_clock::now();

        lk.lock();
        const size_t actual = worker_bytes(wk);
        sv->held = sv->held - wk.held + actual;
        wk.held = actual;
        sv->stats.peak_held_bytes = std::max<uint64_t>(sv->stats.peak_held_bytes, sv->held);
        sv->stats.batches += 1;
        sv->stats.requests += batch.size();
        sv->stats.max_batch_requests = std::max<uint64_t>(sv->stats.max_batch_requests, batch.size());
        sv->stats.records += total;
        sv->stats.allocs += wk.w->n_allocs - allocs0;
        sv->stats.ms_alloc += wk.w->ms_alloc - ms_alloc0;
        sv->stats.ms_batch_wall += std::chrono::duration<double, std::milli>(t_end - t_start).count();
        sv->stats.ms_gather += ms[0];
        sv->stats.ms_sort += ms[1];
        sv->stats.ms_scatter += ms[2];
        for (const Server::Req& q : batch) {
            sv->running.erase(q.ticket);
            sv->done[q.ticket] = Server::Done{
                st, std::chrono::duration<double>(t_end - q.t_submit).count()};
        }
        if (st) {
            // Record the failure on the owner for dfr_last_error.  The batch's device
            // work has finished (run_batch waits for it whatever its status); the
            // worker's context is cleared of its failed mark so later batches run.
            sv->owner->err = "serving batch: " + wk.w->err;
            wk.w->failed = false;
        }
        sv->cv.notify_all();
    }
}

dfr_status start_server(dfr_ctx* c) {
    Server* sv = new (std::nothrow) Server();
    if (!sv) return DFR_E_NO_MEMORY;
    sv->owner = c;
    sv->budget = c->budget;
    sv->batch_records = std::max<uint64_t>(c->serve_batch_records, 1);
    sv->gather_records = c->serve_gather_records;
    const int nw = std::max(1, std::min(c->serve_workers, 8));
    sv->workers.resize(nw);
    for (int i = 0; i < nw; ++i) {
        Server::Worker& wk = sv->workers[i];
        wk.w = new dfr_ctx();
        wk.w->device = c->device;
        wk.w->divert = c->divert;
        wk.w->radix_bits = c->radix_bits;
        wk.w->tile_records = c->tile_records;
        wk.w->window = c->window;
        wk.w->tunes = c->tunes;
        wk.w->temp_slack = 4;  // batches vary in size: grow the temp cache by half again
        bool ok = hipStreamCreateWithFlags(&wk.s, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&wk.w->done, hipEventDisableTiming) == hipSuccess;
        for (int e = 0; ok && e < 4; ++e) ok = hipEventCreate(&wk.ev[e]) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            for (int k = 0; k <= i; ++k) {
                if (sv->workers[k].s) (void)hipStreamDestroy(sv->workers[k].s);
                for (auto e : sv->workers[k].ev)
                    if (e) (void)hipEventDestroy(e);
                if (sv->workers[k].w->done) (void)hipEventDestroy(sv->workers[k].w->done);
                delete sv->workers[k].w;
            }
            delete sv;
            return DFR_E_HIP;
        }
    }
    for (int i = 0; i < nw; ++i) sv->threads.emplace_back(worker_loop, sv, i);
    c->server = sv;
    return DFR_OK;
}

void stop_server(dfr_ctx* c) {
    Server* sv = c->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    for (auto& t : sv->threads) t.join();
    for (auto& wk : sv->workers) {
        free_worker_buffers(wk);
        if (wk.w->err_dev) (void)hipFree(wk.w->err_dev);
        if (wk.w->pin) (void)hipHostFree(wk.w->pin);
        for (auto e : wk.w->event_pool) (void)hipEventDestroy(e);
        for (auto e : wk.ev) (void)hipEventDestroy(e);
        if (wk.w->done) (void)hipEventDestroy(wk.w->done);
        (void)hipStreamDestroy(wk.s);
        delete wk.w;
    }
    delete sv;
    c->server = nullptr;
}

}  // namespace

// =================================================================================
// C ABI
// =================================================================================
extern "C" {

dfr_status dfr_create(int hip_device, size_t hbm_budget_bytes, dfr_ctx** out) {
    if (!out) return DFR_E_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return DFR_E_HIP;
    }
    if (hip_device < 0 || hip_device >= count) return DFR_E_INVALID_ARG;
    dfr_ctx* c = new (std::nothrow) dfr_ctx();
    if (!c) return DFR_E_NO_MEMORY;
    c->device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete c;
        return DFR_E_HIP;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        total_b = 0;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : total_b / 4;
    if (hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return DFR_E_HIP;
    }
    // Set-up of the allocation-free entry point: this device's scratch array (looked
    // up once per device, this device current) and pinned staging reserved now.
    void* sp = nullptr;
    if (static_scratch_address(hip_device, &sp) != hipSuccess ||
        hipHostMalloc((void**)&c->pin, kNoallocPinBytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(c->done);
        delete c;
        return DFR_E_HIP;
    }
    c->static_scratch = (char*)sp;
    c->pin_cap = kNoallocPinBytes;
    *out = c;
    return DFR_OK;
}

void dfr_destroy(dfr_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    {
        std::lock_guard<std::mutex> g(c->serve_mu);
        stop_server(c);
    }
    (void)hipDeviceSynchronize();
    if (c->arena) (void)hipFree(c->arena);
    if (c->err_dev) (void)hipFree(c->err_dev);
    if (c->tcache) (void)hipFree(c->tcache);
    if (c->pin) (void)hipHostFree(c->pin);
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->done) (void)hipEventDestroy(c->done);
    delete c;
}

const char* dfr_status_string(dfr_status s) {
    switch (s) {
        case DFR_OK: return "ok";
        case DFR_E_INVALID_ARG: return "invalid argument";
        case DFR_E_TOO_LARGE: return "too large";
        case DFR_E_NO_MEMORY: return "out of device memory";
        case DFR_E_HIP: return "HIP runtime error";
        case DFR_E_PENDING: return "pending";
        case DFR_E_NOT_FOUND: return "not found";
        case DFR_E_BUDGET: return "exceeds memory budget";
        case DFR_E_UNSUPPORTED: return "unsupported";
        case DFR_E_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* dfr_last_error(const dfr_ctx* c) { return c ? c->err.c_str() : ""; }

size_t dfr_temp_bytes(size_t n, int key_bytes, int val_bytes) {
    if (!(key_bytes == 4 || key_bytes == 8) || !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return 0;
    return round_up(n * key_bytes, ALIGN) + round_up(n * val_bytes, ALIGN);
}

size_t dfr_local_sort_capacity(int key_bytes, int val_bytes) {
    if (!(key_bytes == 4 || key_bytes == 8) || !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return 0;
    return local_cap(key_bytes, val_bytes);
}

size_t dfr_deal_tile_records(int key_bytes, int val_bytes) {
    if (!(key_bytes == 4 || key_bytes == 8) || !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return 0;
    return deal_tile_records(key_bytes, val_bytes);
}

int32_t dfr_size_class(const uint64_t* seg_offsets, size_t num_segments) {
    std::vector<LSeg> segs;
    if (parse_segments(seg_offsets, num_segments, 4, segs) != DFR_OK) return -1;
    return size_class(segs);
}

dfr_status dfr_autotune(dfr_ctx* c, int key_bytes, int val_bytes, const void* keys,
                        const void* vals, const uint64_t* seg_offsets, size_t num_segments,
                        int reps, void* stream, dfr_tune* out) {
    if (!c || !seg_offsets) return DFR_E_INVALID_ARG;
    const size_t n = seg_offsets[num_segments];
    dfr_status st = validate(c, keys, vals, n, key_bytes, val_bytes, nullptr, 0);
    if (st) return st;
    std::vector<LSeg> segs;
    st = parse_segments(seg_offsets, num_segments, key_bytes, segs);
    if (st) return st;
    if (n <= 1) {
        if (out) *out = default_tune(key_bytes, val_bytes);
        return DFR_OK;
    }
    st = set_device(c);
    if (st) return st;
    CallOrder order(c, (hipStream_t)stream);
    if (order.st) return order.st;
    return autotune(c, key_bytes, val_bytes, keys, val_bytes ? vals : nullptr, segs, n,
                    reps > 0 ? reps : 2, (hipStream_t)stream, out);
}

dfr_status dfr_get_tune(const dfr_ctx* c, int key_bytes, int val_bytes, int32_t size_class,
                        dfr_tune* out) {
    if (!c || !out || size_class < 0 || size_class >= DFR_TUNE_CLASSES) return DFR_E_INVALID_ARG;
    auto it = c->tunes.find(tune_key(key_bytes, val_bytes, size_class));
    if (it == c->tunes.end()) return DFR_E_NOT_FOUND;
    *out = it->second;
    return DFR_OK;
}

dfr_status dfr_set_tune(dfr_ctx* c, int key_bytes, int val_bytes, int32_t size_class,
                        const dfr_tune* tune) {
    if (!c || size_class < 0 || size_class >= DFR_TUNE_CLASSES) return DFR_E_INVALID_ARG;
    if (!(key_bytes == 4 || key_bytes == 8) || !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return DFR_E_INVALID_ARG;
    const uint32_t k = tune_key(key_bytes, val_bytes, size_class);
    if (!tune) {
        c->tunes.erase(k);
        return DFR_OK;
    }
    if (!tune_valid(*tune, key_bytes, val_bytes)) return DFR_E_INVALID_ARG;
    c->tunes[k] = *tune;
    return DFR_OK;
}

dfr_status dfr_sort_u32(dfr_ctx* c, uint32_t* keys, uint32_t* vals, size_t n, void* temp,
                        size_t temp_bytes, void* stream) {
    return sort_plain(c, 4, vals ? 4 : 0, keys, vals, n, temp, temp_bytes, stream);
}

dfr_status dfr_sort_u64(dfr_ctx* c, uint64_t* keys, uint64_t* vals, size_t n, void* temp,
                        size_t temp_bytes, void* stream) {
    return sort_plain(c, 8, vals ? 8 : 0, keys, vals, n, temp, temp_bytes, stream);
}

dfr_status dfr_sort_noalloc(dfr_ctx* c, void* keys, void* vals, size_t n, int key_bytes,
                            int val_bytes, void* stream) {
    dfr_status st = validate(c, keys, vals, n, key_bytes, val_bytes, nullptr, 0);
    if (st) return st;
    if (n > NOALLOC_MAX_RECORDS) {
        c->err = "allocation-free sort: more records than its fixed scratch holds";
        return DFR_E_TOO_LARGE;
    }
    if (n <= 1) {
        c->stats = dfr_stats{};
        return DFR_OK;
    }
    if (!c->static_scratch) return DFR_E_UNSUPPORTED;
    st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    // Layout of the fixed scratch: the status block, the temp buffer, then the level
    // scratch (the arena).  Everything the kernels need zeroed is cleared per call.
    const size_t temp_bytes = dfr_temp_bytes(n, key_bytes, val_bytes);
    char* base = c->static_scratch;
    char* arena = base + ALIGN + temp_bytes;
    const size_t arena_cap = NOALLOC_SCRATCH_BYTES - ALIGN - temp_bytes;
    char* const saved_arena = c->arena;
    const size_t saved_cap = c->arena_cap, saved_used = c->arena_used;
    uint32_t* const saved_err = c->err_dev;
    c->arena = arena;
    c->arena_cap = arena_cap;
    c->arena_used = 0;
    c->err_dev = (uint32_t*)base;
    c->static_mode = true;
    const dfr_tune t = default_tune(key_bytes, val_bytes);  // options and tunings do not apply
    std::vector<LSeg> segs{LSeg{0, n, 8 * key_bytes}};
    st = run_sort(c, key_bytes, val_bytes, keys, val_bytes ? vals : nullptr, segs, base + ALIGN, s, &t);
    c->static_mode = false;
    c->arena = saved_arena;
    c->arena_cap = saved_cap;
    c->arena_used = saved_used;
    c->err_dev = saved_err;
    return st;
}

dfr_status dfr_sort_keys(dfr_ctx* c, int32_t key_type, void* keys, void* vals, int val_bytes,
                         size_t n, void* temp, size_t temp_bytes, void* stream) {
    int kb = 0, mode = 0;
    if (!key_type_info(key_type, &kb, &mode)) return DFR_E_INVALID_ARG;
    if (!(val_bytes == 0 || val_bytes == 4 || val_bytes == 8)) return DFR_E_INVALID_ARG;
    if ((val_bytes == 0) != (vals == nullptr)) return DFR_E_INVALID_ARG;
    return sort_plain(c, kb, val_bytes, keys, vals, n, temp, temp_bytes, stream, mode);
}

dfr_status dfr_sort_segmented_keys(dfr_ctx* c, int32_t key_type, void* keys, void* vals,
                                   int val_bytes, const uint64_t* seg_offsets, size_t num_segments,
                                   void* temp, size_t temp_bytes, void* stream) {
    int kb = 0, mode = 0;
    if (!key_type_info(key_type, &kb, &mode)) return DFR_E_INVALID_ARG;
    if (!(val_bytes == 0 || val_bytes == 4 || val_bytes == 8)) return DFR_E_INVALID_ARG;
    if ((val_bytes == 0) != (vals == nullptr)) return DFR_E_INVALID_ARG;
    return sort_segmented(c, kb, val_bytes, keys, vals, seg_offsets, num_segments, temp,
                          temp_bytes, stream, mode);
}

dfr_status dfr_sort_segmented_u32(dfr_ctx* c, uint32_t* keys, uint32_t* vals,
                                  const uint64_t* seg_offsets, size_t num_segments, void* temp,
                                  size_t temp_bytes, void* stream) {
    return sort_segmented(c, 4, vals ? 4 : 0, keys, vals, seg_offsets, num_segments, temp,
                          temp_bytes, stream);
}

dfr_status dfr_sort_segmented_u64(dfr_ctx* c, uint64_t* keys, uint64_t* vals,
                                  const uint64_t* seg_offsets, size_t num_segments, void* temp,
                                  size_t temp_bytes, void* stream) {
    return sort_segmented(c, 8, vals ? 8 : 0, keys, vals, seg_offsets, num_segments, temp,
                          temp_bytes, stream);
}

dfr_status dfr_count(dfr_ctx* c, const void* keys, int key_bytes, size_t n, int bits, int num_digits,
                     uint32_t* hist, void* stream) {
    if (!c) return DFR_E_INVALID_ARG;
    if (c->failed) return DFR_E_HIP;
    if (!(key_bytes == 4 || key_bytes == 8) || bits < 1 || bits > 8 || num_digits < 1 ||
        num_digits > MAX_PASSES || num_digits * bits > 8 * key_bytes || !hist)
        return DFR_E_INVALID_ARG;
    if (n > 0 && (!keys || (uintptr_t)keys % key_bytes)) return DFR_E_INVALID_ARG;
    if (n > DFR_MAX_SEGMENT_RECORDS) return DFR_E_TOO_LARGE;
    dfr_status st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    HIP_TRY(c, launch_fill_u32(hist, 0, (size_t)num_digits * RADIX, s));
    if (n == 0) return DFR_OK;
    std::vector<LSeg> segs{LSeg{0, n, 8 * key_bytes}};
    std::vector<uint32_t> ids{0};
    std::vector<Tile> tiles;
    std::vector<uint32_t> ft;
    Job j;
    j.c = c;
    j.s = s;
    build_tiles(segs, ids, deal_tile_records(key_bytes, 0), tiles, ft);
    st = arena_reserve(c, asize<Tile>(tiles.size()) + 2 * asize<uint64_t>(1), s);
    if (st) return st;
    Tile* dt = aalloc<Tile>(c, tiles.size());
    uint64_t* dor = aalloc<uint64_t>(c, 1);
    uint64_t* dand = aalloc<uint64_t>(c, 1);
    st = upload(j, dt, tiles.data(), tiles.size() * sizeof(Tile));
    if (st) return st;
    CountArgs ca{};
    ca.keys = keys;
    ca.tiles = dt;
    ca.ntiles = (uint32_t)tiles.size();
    const uint32_t blocks = (uint32_t)std::min<size_t>(tiles.size(), 2048);
    ca.tiles_per_block = (uint32_t)((tiles.size() + blocks - 1) / blocks);
    ca.base_shift = 0;
    ca.bits = bits;
    ca.ndig = num_digits;
    ca.hist = hist;
    ca.seg_or = dor;
    ca.seg_and = dand;
    const uint32_t grid = (uint32_t)((tiles.size() + ca.tiles_per_block - 1) / ca.tiles_per_block);
    HIP_TRY(c, launch_count(key_bytes, ca, grid, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    synced(c);
    return DFR_OK;
}

dfr_status dfr_deal(dfr_ctx* c, const void* keys_in, const void* vals_in, void* keys_out,
                    void* vals_out, int key_bytes, int val_bytes, size_t n, int shift, int bits,
                    void* stream) {
    if (!c) return DFR_E_INVALID_ARG;
    if (c->failed) return DFR_E_HIP;
    if (!(key_bytes == 4 || key_bytes == 8) || !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return DFR_E_INVALID_ARG;
    if (bits < 1 || bits > 8 || shift < 0 || shift + bits > 8 * key_bytes) return DFR_E_INVALID_ARG;
    if ((val_bytes == 0) != (vals_in == nullptr && vals_out == nullptr)) return DFR_E_INVALID_ARG;
    if (n == 0) return DFR_OK;
    if (!keys_in || !keys_out || (uintptr_t)keys_in % key_bytes || (uintptr_t)keys_out % key_bytes)
        return DFR_E_INVALID_ARG;
    if (val_bytes && (!vals_in || !vals_out || (uintptr_t)vals_in % val_bytes ||
                      (uintptr_t)vals_out % val_bytes))
        return DFR_E_INVALID_ARG;
    const size_t kbn = n * key_bytes, vbn = n * val_bytes;
    if (overlap(keys_in, kbn, keys_out, kbn) || (val_bytes && (overlap(vals_in, vbn, vals_out, vbn) ||
                                                               overlap(keys_in, kbn, vals_out, vbn) ||
                                                               overlap(vals_in, vbn, keys_out, kbn) ||
                                                               overlap(keys_out, kbn, vals_out, vbn))))
        return DFR_E_INVALID_ARG;
    if (n > DFR_MAX_SEGMENT_RECORDS) return DFR_E_TOO_LARGE;
    dfr_status st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    Job j;
    j.c = c;
    j.s = s;
    std::vector<LSeg> segs{LSeg{0, n, 8 * key_bytes}};
    std::vector<uint32_t> ids{0};
    std::vector<Tile> tiles;
    std::vector<uint32_t> ft;
    build_tiles(segs, ids, deal_tile_records(key_bytes, val_bytes), tiles, ft);
    const size_t nt = tiles.size();
    st = arena_reserve(c, asize<Tile>(nt) + asize<Seg>(1) + asize<uint32_t>(RADIX) +
                              2 * asize<uint64_t>(1) + asize<uint64_t>(nt * RADIX + 1) +
                              asize<uint32_t>(1),
                       s);
    if (st) return st;
    Tile* dt = aalloc<Tile>(c, nt);
    Seg* ds = aalloc<Seg>(c, 1);
    uint32_t* dh = aalloc<uint32_t>(c, RADIX);
    uint64_t* dor = aalloc<uint64_t>(c, 1);
    uint64_t* dand = aalloc<uint64_t>(c, 1);
    uint64_t* lb = aalloc<uint64_t>(c, nt * RADIX + 1);
    uint32_t* derr = aalloc<uint32_t>(c, 1);
    Seg g{};
    g.start = 0;
    g.len = n;
    g.first_tile = 0;
    g.npass = 1;
    g.shift[0] = (int8_t)shift;
    g.width[0] = (int8_t)bits;
    g.hslot[0] = 0;
    g.lo_bit = shift;
    st = upload(j, dt, tiles.data(), nt * sizeof(Tile));
    if (!st) st = upload(j, ds, &g, sizeof g);
    if (st) return st;
    HIP_TRY(c, launch_fill_u32(dh, 0, RADIX, s));
    HIP_TRY(c, launch_fill_u64(lb, 0, nt * RADIX + 1, s));
    HIP_TRY(c, launch_fill_u32(derr, 0, 1, s));
    CountArgs ca{};
    ca.keys = keys_in;
    ca.tiles = dt;
    ca.ntiles = (uint32_t)nt;
    const uint32_t blocks = (uint32_t)std::min<size_t>(nt, 2048);
    ca.tiles_per_block = (uint32_t)((nt + blocks - 1) / blocks);
    ca.base_shift = shift;
    ca.bits = bits;
    ca.ndig = 1;
    ca.hist = dh;
    ca.seg_or = dor;
    ca.seg_and = dand;
    HIP_TRY(c, launch_count(key_bytes, ca, (uint32_t)((nt + ca.tiles_per_block - 1) / ca.tiles_per_block), s));
    DealArgs da{};
    da.kin = keys_in;
    da.vin = vals_in;
    da.kout = keys_out;
    da.vout = vals_out;
    da.tiles = dt;
    da.ntiles = (uint32_t)nt;
    da.segs = ds;
    da.hist = dh;
    da.hist_digits = 1;
    da.pass = 0;
    da.lookback = lb;
    da.ticket = (uint32_t*)(lb + nt * RADIX);
    da.err = derr;
    da.tile = deal_tile_records(key_bytes, val_bytes);
    {
        Timed tm(c, s, ST_DEAL, true);
        HIP_TRY(c, launch_deal(key_bytes, val_bytes, da, s));
    }
    st = pin_reserve(c, 64, s);
    if (st) return st;
    uint32_t* he = palloc<uint32_t>(c, 1);
    HIP_TRY(c, hipMemcpyAsync(he, derr, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const uint32_t e = *he;
    synced(c);
    if (c->timing) collect_events(c);
    if (e) {
        c->err = "device error in deal";
        return DFR_E_INTERNAL;
    }
    return DFR_OK;
}

dfr_status dfr_stream_copy(dfr_ctx* c, const void* src, void* dst, size_t bytes, void* stream) {
    if (!c) return DFR_E_INVALID_ARG;
    if (c->failed) return DFR_E_HIP;
    if (bytes == 0) return DFR_OK;
    if (!src || !dst || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16 ||
        overlap(src, bytes, dst, bytes))
        return DFR_E_INVALID_ARG;
    dfr_status st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    HIP_TRY(c, launch_stream_copy(src, dst, bytes, s));
    return DFR_OK;
}

dfr_status dfr_stream_read(dfr_ctx* c, const void* src, size_t bytes, uint32_t* xor_out, void* stream) {
    if (!c) return DFR_E_INVALID_ARG;
    if (c->failed) return DFR_E_HIP;
    if (!xor_out || (uintptr_t)xor_out % 4 || bytes % 16 || (bytes && (!src || (uintptr_t)src % 16)) ||
        overlap(src, bytes, xor_out, 4))
        return DFR_E_INVALID_ARG;
    dfr_status st = set_device(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    if (order.st) return order.st;
    const uint64_t parts = stream_read_parts(bytes);
    st = arena_reserve(c, asize<uint32_t>(parts), s);
    if (st) return st;
    uint32_t* part = aalloc<uint32_t>(c, parts);
    HIP_TRY(c, launch_stream_read(src, bytes, part, xor_out, s));
    return DFR_OK;
}

dfr_status dfr_submit(dfr_ctx* c, const dfr_request* req, uint64_t* ticket) {
    if (!c || !req || !ticket) return DFR_E_INVALID_ARG;
    const int kb = req->key_bytes, vb = req->val_bytes;
    if (!(kb == 4 || kb == 8) || !(vb == 0 || vb == 4 || vb == 8)) return DFR_E_INVALID_ARG;
    if (vb && vb != kb) return DFR_E_INVALID_ARG;
    if (req->n > DFR_MAX_SEGMENT_RECORDS) return DFR_E_TOO_LARGE;
    if (req->n) {
        if (!req->keys || (uintptr_t)req->keys % kb) return DFR_E_INVALID_ARG;
        if (vb && (!req->vals || (uintptr_t)req->vals % vb)) return DFR_E_INVALID_ARG;
        if (vb && overlap(req->keys, req->n * kb, req->vals, req->n * vb)) return DFR_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> g(c->serve_mu);
    if (c->budget && batch_bytes(req->n, kb, vb, false) > c->budget) return DFR_E_BUDGET;
    if (!c->server) {
        dfr_status st = start_server(c);
        if (st) return st;
    }
    Server* sv = c->server;
    {
        std::lock_guard<std::mutex> l(sv->mu);
        Server::Req q;
        q.ticket = sv->next_ticket++;
        q.r = *req;
        if (!vb) q.r.vals = nullptr;
        q.t_submit = std::chrono::steady_clock::now();
        sv->pending.push_back(q);
        *ticket = q.ticket;
    }
    sv->cv.notify_all();
    return DFR_OK;
}

dfr_status dfr_poll(dfr_ctx* c, uint64_t ticket, double* latency_s) {
    if (!c) return DFR_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(c->serve_mu);
    Server* sv = c->server;
    if (!sv) return DFR_E_NOT_FOUND;
    std::lock_guard<std::mutex> l(sv->mu);
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        if (sv->running.count(ticket)) return DFR_E_PENDING;
        for (const auto& q : sv->pending)
            if (q.ticket == ticket) return DFR_E_PENDING;
        return DFR_E_NOT_FOUND;
    }
    const Server::Done d = it->second;
    sv->done.erase(it);
    if (latency_s) *latency_s = d.latency;
    return d.st;
}

dfr_status dfr_get_serve_stats(dfr_ctx* c, dfr_serve_stats* out) {
    if (!c || !out) return DFR_E_INVALID_ARG;
    std::lock_guard<std::mutex> g(c->serve_mu);
    *out = dfr_serve_stats{};
    if (!c->server) return DFR_OK;
    std::lock_guard<std::mutex> l(c->server->mu);
    *out = c->server->stats;
    out->workers = (int32_t)c->server->workers.size();
    out->budget_bytes = c->server->budget;
    out->held_bytes = c->server->held;
    out->queued = c->server->pending.size();
    return DFR_OK;
}

dfr_status dfr_set_option(dfr_ctx* c, const char* name, int64_t value) {
    if (!c || !name) return DFR_E_INVALID_ARG;
    if (!strcmp(name, "divert_records")) {
        if (value < 0) return DFR_E_INVALID_ARG;
        c->divert = (size_t)value;
        return DFR_OK;
    }
    if (!strcmp(name, "force_top_digits")) {
        if (value < 0 || value > MAX_PASSES) return DFR_E_INVALID_ARG;
        c->force_d = (int)value;
        return DFR_OK;
    }
    if (!strcmp(name, "timing")) {
        if (value < 0 || value > 2) return DFR_E_INVALID_ARG;
        c->timing = (int)value;
        return DFR_OK;
    }
    if (!strcmp(name, "force_lookback")) {
        c->force_lookback = value != 0;
        return DFR_OK;
    }
    if (!strcmp(name, "force_key_heads")) {
        c->force_key_heads = value != 0;
        return DFR_OK;
    }
    if (!strcmp(name, "estimated_buckets")) {
        c->est_buckets = value != 0;
        return DFR_OK;
    }
    if (!strcmp(name, "plan_lengths_records")) {
        if (value < 0) return DFR_E_INVALID_ARG;
        c->plan_lengths_max = (uint64_t)value;
        return DFR_OK;
    }
    if (!strcmp(name, "serve_fail_batches")) {
        if (value < 0 || value > 1000000) return DFR_E_INVALID_ARG;
        c->serve_fail_batches.store((int)value);
        return DFR_OK;
    }
    if (!strcmp(name, "serve_workers") || !strcmp(name, "serve_batch_records") ||
        !strcmp(name, "serve_gather_records")) {
        std::lock_guard<std::mutex> g(c->serve_mu);
        if (c->server) return DFR_E_UNSUPPORTED;  // fixed once serving has started
        if (!strcmp(name, "serve_workers")) {
            if (value < 1 || value > 8) return DFR_E_INVALID_ARG;
            c->serve_workers = (int)value;
        } else if (!strcmp(name, "serve_batch_records")) {
            if (value < 1) return DFR_E_INVALID_ARG;
            c->serve_batch_records = (uint64_t)value;
        } else {
            if (value < 0) return DFR_E_INVALID_ARG;
            c->serve_gather_records = value == 0 ? ~0ull : (uint64_t)value;
        }
        return DFR_OK;
    }
    if (!strcmp(name, "radix_bits")) {
        if (value != 0 && (value < 4 || value > RADIX_BITS)) return DFR_E_INVALID_ARG;
        c->radix_bits = (int)value;
        return DFR_OK;
    }
    if (!strcmp(name, "tile_records")) {
        if (value < 0 || value > (1 << 20)) return DFR_E_INVALID_ARG;
        c->tile_records = (uint32_t)value;
        return DFR_OK;
    }
    if (!strcmp(name, "window_records")) {
        if (value < 0) return DFR_E_INVALID_ARG;
        c->window = (size_t)value;
        return DFR_OK;
    }
    return DFR_E_UNSUPPORTED;
}

dfr_status dfr_get_stats(const dfr_ctx* c, dfr_stats* out) {
    if (!c || !out) return DFR_E_INVALID_ARG;
    *out = c->stats;
    return DFR_OK;
}

dfr_status dfr_plan_top_digits(const uint32_t* hist, size_t n, int key_bytes, int val_bytes,
                               size_t divert_records, int32_t* top_digits, int32_t* varying) {
    if (!hist || !top_digits || !(key_bytes == 4 || key_bytes == 8) ||
        !(val_bytes == 0 || val_bytes == 4 || val_bytes == 8))
        return DFR_E_INVALID_ARG;
    std::vector<int> V;
    for (int dgt = key_bytes - 1; dgt >= 0; --dgt) {
        int nz = 0;
        for (int v = 0; v < RADIX; ++v) nz += hist[(size_t)dgt * RADIX + v] != 0;
        if (nz > 1) V.push_back(dgt);
    }
    const size_t cap = local_cap(key_bytes, val_bytes);
    const size_t divert = divert_records ? std::min(divert_records, cap) : default_divert(key_bytes, val_bytes);
    *top_digits = n <= cap ? 0 : plan_from_hist(hist, n, key_bytes, val_bytes, divert, V);
    if (varying) *varying = (int32_t)V.size();
    return DFR_OK;
}

}  // extern "C"
