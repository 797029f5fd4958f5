// Internal declarations shared by the device kernels (kernels.hip) and the host
// orchestration (dfr.cpp).  Not part of the public ABI (include/dfr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfr {

// Radix width of the deal passes: 8-bit digits, 256 buckets per digit, as the
// paper's N/256 bucket estimate and its 256 amortised checks imply (Sec. 4).
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;

// Look-back words of the deal pass: a 2-bit status above a count of up to 62 bits (a
// segment holds fewer than 2^32 records, so every count fits).
constexpr uint64_t LB_AGG = 1ull << 62;  // tile's own count published
constexpr uint64_t LB_PRE = 2ull << 62;  // inclusive prefix through this tile published
constexpr uint64_t LB_COUNT = (1ull << 62) - 1;

// Bits of the device error word.
constexpr uint32_t ERR_SPIN = 1;        // a bounded look-back wait expired
constexpr uint32_t ERR_BUCKET_CAP = 2;  // more bucket heads than the list holds
constexpr uint32_t ERR_LIST_CAP = 4;    // a work list overflowed
constexpr uint32_t ERR_CHUNK = 8;       // a local-sort chunk exceeded its capacity
constexpr uint32_t ERR_RANGE = 16;      // a computed position fell outside its segment

constexpr int MAX_PASSES = 8;

// One segment of a level: a range of records whose keys agree on every bit at and
// above hi_bit, sorted independently of the others.
struct Seg {
    uint64_t start;
    uint64_t len;
    uint32_t first_tile;   // index of the segment's first tile in the level's tile list
    uint32_t window_base;  // first local-sort window slot of the segment
    int32_t lo_bit;        // after this level's deals, buckets agree on bits >= lo_bit
    int32_t npass;
    uint32_t count_tile;   // index of the segment's first tile in the counting tile list
    int32_t first_pass;    // deal passes before this one leave the segment where it is
    int8_t shift[MAX_PASSES];  // digit of deal pass j: (key >> shift[j]) mod 2^width[j]
    int8_t width[MAX_PASSES];
    int8_t hslot[MAX_PASSES];  // histogram slot holding that digit's counts
};

// A contiguous run of at most one tile's records inside one segment.
struct Tile {
    uint64_t start;
    uint32_t len;
    uint32_t seg;
};

// A bucket too large for the local sort, to be sorted by the next level.
struct Big {
    uint64_t start;
    uint32_t len;
    uint32_t hi_bit;
};

struct CountArgs {
    const void* keys;
    const Tile* tiles;
    uint32_t ntiles;
    uint32_t tiles_per_block;
    int32_t base_shift;  // digit j sits at base_shift + j * bits
    int32_t bits;
    int32_t ndig;        // digits counted, <= MAX_PASSES
    int32_t hist_digits; // digits per histogram row (0: ndig); rows past ndig are left as they are
    uint32_t* hist;      // [seg][hist_digits][RADIX]
    void* seg_or;        // [seg] key type, OR of the segment's keys
    void* seg_and;       // [seg] key type, AND of the segment's keys
    uint32_t* tile_hist; // optional [tile][hist_digits][RADIX]: each tile's own counts
    const Seg* segs;     // optional: digit shift per tile from segs[seg].shift[pass]
    int32_t pass;
};

// Per-tile bucket bases for many segments: one block per segment walks its tiles.
struct SegScanArgs {
    const Seg* segs;
    uint32_t nsegs;
    const uint32_t* hist;  // per-segment digit histograms [seg][hist_digits][RADIX]
    int32_t hist_digits;
    const uint32_t* cnt;   // per-tile counts cnt[(t * cnt_ndig + slot) * RADIX + v]
    int32_t cnt_ndig;
    int32_t cnt_from_count_tiles;  // 1: tiles indexed as in the counting list, slot = hslot
    int32_t pass;
    uint32_t tile;         // records per tile
    uint32_t* off;         // [tiles][RADIX], indexed by the deal's tile list
    uint64_t* ticket;      // if set, the deal's tile ticket, cleared by the scan
};

// Per-tile bucket bases from per-tile digit counts (one segment): off[t][v] is the
// position, relative to the segment start, of tile t's first record of digit v.
struct TileScanArgs {
    const uint32_t* cnt;  // cnt[(t * ndig + slot) * RADIX + v]
    int32_t ndig;
    int32_t slot;
    uint32_t ntiles;
    uint32_t tiles_per_block;
    uint32_t nblocks;
    uint32_t* partial;  // [nblocks][RADIX]
    uint32_t* off;      // [ntiles][RADIX]
    uint64_t* ticket;   // if set, the deal's tile ticket, cleared by the scan
};

struct DealArgs {
    const void* kin;
    const void* vin;
    void* kout;
    void* vout;
    const Tile* tiles;
    uint32_t ntiles;
    const Seg* segs;
    const uint32_t* hist;
    int32_t hist_digits;
    int32_t pass;
    uint64_t* lookback;  // [ntiles][RADIX]
    uint32_t* ticket;
    const uint32_t* off; // when set: per-tile bucket bases, and no look-back
    uint32_t tile;       // records per tile (selects the kernel; see deal_tile_supported)
    uint32_t* err;
    const void* kin2;    // tiles whose seg carries TILE_IN2 read from here (overflow areas)
    const void* vin2;
};

// Tile flag: the tile's records are in the deal's second input (kin2/vin2), at
// tile.start there; the segment index is the other bits.
constexpr uint32_t TILE_IN2 = 1u << 31;

// Fast Radix's deal into estimated buckets (Sec. 3; overflow, Sec. 3.1): one segment
// [0, n), bucket v's first E records at [v * E, v * E + E) of kout, the next C at
// [v * C, v * C + C) of kovf, in input order (decoupled look-back over the tiles).
struct EstArgs {
    const void* kin;
    const void* vin;
    void* kout;
    void* vout;
    void* kovf;
    void* vovf;
    uint64_t n;
    uint32_t ntiles;
    uint32_t tile;
    int32_t shift, width;    // the dealt digit
    int32_t nshift, nwidth;  // the next digit, counted for the exact pass that follows
    uint64_t E;              // estimated slots per bucket
    uint32_t C;              // overflow slots per bucket
    uint64_t* lookback;      // [ntiles][RADIX]
    uint32_t* ticket;
    uint32_t* cnt;           // [RADIX] records of each bucket, summed over the tiles
    uint32_t* next_hist;     // [RADIX] histogram of the next digit
    uint32_t* lost;          // records of buckets that outgrew E + C (then redone exactly)
    uint32_t* err;
};

// Bucket heads per tile, at most HEAD_SLOTS of them kept per tile as tile-relative
// positions; a tile with more is found again from its keys when the heads are listed.
constexpr uint32_t HEAD_SLOTS = 256;

struct HeadArgs {
    const void* keys;
    const Tile* tiles;
    uint32_t ntiles;
    const Seg* segs;
    uint32_t* tcount;    // [ntiles] heads in each tile
    uint64_t* tbase;     // [ntiles] index of each tile's first head in the bucket list
    uint16_t* tslot;     // [ntiles][HEAD_SLOTS] tile-relative positions of the heads
    uint64_t* bstart;
    uint32_t* bseg;
    uint64_t bcap;
    uint32_t* nbuckets;
    uint32_t* err;
};

// Bucket heads of a one-segment level dealt on two digits, from counts rather than the
// keys (see k_joint_counts).  u is the first deal's digit, v the second's.
struct JointArgs {
    const void* keys;       // the first deal's output (whole buffer)
    uint64_t seg_start;
    uint64_t seg_len;
    const uint32_t* h0;     // the segment's histogram of u
    const uint32_t* tcnt;   // the second deal's per-tile counts of v: tcnt[t * RADIX + v]
    uint32_t ntiles;        // tiles of the second deal: [t * tile, min((t + 1) * tile, seg_len))
    uint32_t tile;
    int32_t shift1;         // v = (key >> shift1) mod 2^width1
    int32_t width0;
    int32_t width1;
    uint32_t* joint;        // [2^width1][2^width0] record counts of each pair (v, u)
    uint64_t* rows;         // [2^width1] records | non-empty pairs << 32, of each row v
    uint64_t* bstart;
    uint32_t* bseg;
    uint32_t seg;           // the segment's index, written to bseg
    uint64_t bcap;
    uint32_t* nbuckets;
    uint32_t* err;
};

// Bucket heads of a level whose segments are all dealt on one digit: each segment's
// buckets are the non-empty values of that digit, from its histogram.
struct HistHeadArgs {
    const Seg* segs;
    const uint32_t* ids;    // the segments that need buckets, in list order
    uint32_t nids;
    const uint32_t* hist;   // per-segment digit histograms [seg][hist_digits][RADIX]
    int32_t hist_digits;
    uint32_t* first;        // [nids]: non-empty values, then each segment's first list index
    uint64_t* bstart;
    uint32_t* bseg;
    uint64_t bcap;
    uint32_t* nbuckets;
    uint32_t* err;
};

struct ClassifyArgs {
    const uint64_t* bstart;
    const uint32_t* bseg;
    const uint32_t* nbuckets;
    uint64_t bcap;
    const Seg* segs;
    uint32_t wsmall;  // largest "small" bucket, also the window width
    uint32_t cap;     // local sort capacity
    int32_t kbits;    // key bits
    uint32_t* cfirst;
    uint32_t* clast;
    uint32_t nslots;
    uint32_t* med;
    uint32_t* nmed;
    uint32_t medcap;
    uint32_t* work;    // non-empty local-sort work items, appended as found
    uint32_t* nwork;
    uint32_t workcap;
    Big* big;
    uint32_t* nbig;
    uint32_t bigcap;
    Big* done;
    uint32_t* ndone;
    uint32_t donecap;
    uint32_t* err;
};

// One local-sort chunk: consecutive buckets of one segment (or one medium bucket).
struct ChunkDesc {
    uint64_t start;  // its first record
    uint32_t len;    // records; 0 for a work item that holds no chunk
    uint32_t nbk;    // buckets in it
    uint32_t f;      // its first bucket
    int32_t lo;      // its records agree on the key bits >= lo
};

struct LocalArgs {
    const void* kin;
    const void* vin;
    void* kout;
    void* vout;
    const uint64_t* bstart;
    const uint32_t* bseg;
    const uint32_t* nbuckets;
    uint64_t bcap;
    const Seg* segs;
    const uint32_t* cfirst;
    const uint32_t* clast;
    uint32_t nslots;
    const uint32_t* med;
    const uint32_t* nmed;
    uint32_t medcap;
    const uint32_t* work;   // non-empty work items (window slots, then nslots + medium index)
    const uint32_t* nwork;
    uint32_t workcap;
    ChunkDesc* desc;        // the work items' chunks (workcap entries), decoded first
    ChunkDesc* spill;       // chunks the bucketed local sort hands to the general one
    uint32_t* nspill;       // zero before the launch
    uint32_t spillcap;
    ChunkDesc* wide;        // chunks a 32-bit-word form hands to the 64-bit-word form
    uint32_t* nwide;        // zero before the launch
    uint32_t widecap;
    // Set by the launcher: the list a bucketed kernel sorts (desc, or wide).
    const ChunkDesc* chunks;
    const uint32_t* nchunks;
    uint32_t chunkcap;
    uint32_t* err;
    uint32_t* stat;     // chunks sorted by forms 0, 1, 2 and by the general kernel
};

// Words of the per-call device status block: the error word, then kernel counters.
// The level's list counters follow it (LEVEL_WORDS words at STAT_WORDS), so one copy
// brings both back at a level's end.
constexpr int STAT_ERR = 0;
constexpr int STAT_FORM0 = 1;  // + form: chunks of the bucketed local sort, forms 0..2
constexpr int STAT_GENERAL = 4;  // chunks of the general local sort
constexpr int STAT_WORDS = 8;
constexpr int LEVEL_WORDS = 8;  // buckets, medium, big, done, spill, work, wide

// A run of at most 2^32 - 1 records copied between two places.
struct CopyChunk {
    const void* ksrc;
    const void* vsrc;
    void* kdst;
    void* vdst;
    uint32_t len;
};

// The allocation-free entry point's fixed device scratch (one array per GPU): the
// status block, the temp buffer of a sort of at most NOALLOC_MAX_RECORDS records of up
// to 16 bytes, and the level scratch such a sort needs at the default settings.
constexpr size_t NOALLOC_MAX_RECORDS = size_t(1) << 22;
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(192) << 20;
constexpr int MAX_DEVICES = 64;
// Address of this GPU's scratch array; `device` must be the current device.  Looked up
// once per device (hipGetSymbolAddress), then cached.
hipError_t static_scratch_address(int device, void** ptr);

// Tile and capacity choices per (key bytes, value bytes).
uint32_t deal_tile_records(int kb, int vb);  // the default tile
bool deal_tile_supported(int kb, int vb, uint32_t tile);  // the default or half of it
uint32_t local_sort_capacity(int kb, int vb);    // the general kernel's chunk capacity
uint32_t local_bucket_capacity(int kb, int vb);  // the bucketed kernels' chunk capacity

// Up to four fills in one launch: n[i] words of width w[i] (4 or 8 bytes) at p[i] set
// to v[i].
struct FillSet {
    void* p[4];
    uint64_t v[4];
    uint64_t n[4];
    int32_t w[4];
    int32_t count;
};

// Launchers (kernels.hip).  Each returns the launch's hipError_t.
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
hipError_t launch_fill_set(const FillSet& f, hipStream_t s);
hipError_t launch_count(int kb, const CountArgs& a, uint32_t blocks, hipStream_t s);
hipError_t launch_deal(int kb, int vb, const DealArgs& a, hipStream_t s);
hipError_t launch_deal_est(int kb, int vb, const EstArgs& a, hipStream_t s);
hipError_t launch_tile_scan(const TileScanArgs& a, hipStream_t s);
hipError_t launch_seg_scan(const SegScanArgs& a, hipStream_t s);
// For each segment's digit-j histogram h (digits of `bits` bits):
// coll[s * ndig + j] = sum_v h[v]^2 / (sum_v h[v])^2, nonzero[...] = its non-empty bins,
// overflow[...] = sum_v max(0, h[v] - ceil(len / 2^bits)).
hipError_t launch_collisions(const uint32_t* hist, uint32_t nsegs, int ndig, int bits, double* coll,
                             uint32_t* nonzero, uint32_t* overflow, hipStream_t s);
// In-place map of signed (mode 1) or floating-point (mode 2) keys to unsigned keys of
// the same order, or back (inverse).  Mode 0 does nothing.
hipError_t launch_key_transform(int kb, int mode, bool inverse, void* keys, size_t n,
                                hipStream_t s);
hipError_t launch_heads(int kb, const HeadArgs& a, hipStream_t s);
hipError_t launch_joint_heads(int kb, const JointArgs& a, hipStream_t s);
hipError_t launch_hist_heads(const HistHeadArgs& a, hipStream_t s);
hipError_t launch_classify(const ClassifyArgs& a, uint32_t blocks, hipStream_t s);
// Which form of the local sort runs first for chunks whose buckets agree on every bit
// >= max_lo_bit and whose bucket index is expected to take index_bits: 0 and 1 use
// 32-bit words (with and without the position inside), 2 64-bit words.
int local_sort_first_form(int kb, int vb, int max_lo_bit, int index_bits);
hipError_t launch_local_sort(int kb, int vb, const LocalArgs& a, uint32_t blocks,
                             int first_form, hipStream_t s);
hipError_t launch_copy_chunks(int kb, int vb, const CopyChunk* chunks, uint32_t nchunks,
                              hipStream_t s);
// Streaming copy of bytes / 16 vectors (both pointers 16-byte aligned).
hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);
// Words of partial results the streaming read needs for `bytes` (one per 32 KB block).
uint64_t stream_read_parts(uint64_t bytes);
hipError_t launch_stream_read(const void* src, uint64_t bytes, uint32_t* part, uint32_t* out, hipStream_t s);
hipError_t launch_copy_tiles(int kb, int vb, const void* kin, const void* vin, void* kout,
                             void* vout, const Tile* tiles, uint32_t ntiles, hipStream_t s);

}  // namespace dfr
