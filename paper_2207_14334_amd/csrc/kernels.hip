// Device kernels of the DFR sort for gfx950 (CDNA4, wave64).
//
// The paper's vocabulary (Sec. 2): a *count* tallies how often each value of one
// digit occurs; the counts become bucket indices by an exclusive prefix sum; a *deal*
// moves every record into its bucket, keeping input order among equal digits.  DFR
// (Sec. 3) deals the top digits least significant first, then diverts runs of small
// buckets to a simple stable sort and recurses on large buckets.
//
//   k_count        count: digit histograms of every digit in one read, plus the OR and
//                  AND of each segment's keys (digits that never vary are skipped); also
//                  each tile's own counts, for the deals' bucket bases.
//   k_tile_scan_*  per-tile bucket bases of one long segment (reduce, then scan);
//   k_seg_scan     the same for short segments, one block per segment.
//   k_deal         deal: one stable scatter pass.  Each tile ranks its records by digit
//                  with wave ballots and stages them in LDS in digit order, so each
//                  bucket's run is written contiguously; its bases come from the scans,
//                  or from decoupled look-back over the tiles before it.
//   k_deal_est     Fast Radix's deal into estimated buckets with overflow slots, without
//                  a count (Sec. 3); it counts the next digit on the way.
//   k_fill_*, k_stream_copy, k_stream_read, k_xor_fold
//                  fills of scratch (several ranges per launch); the streaming copy and
//                  read that are the passes' and the counts' bandwidth references.
//   k_heads*       bucket boundaries after the deals, from the keys: positions where
//                  the leading bits change, listed in order.
//   k_joint_*      the same without the keys, for one segment dealt on two digits:
//                  pair counts from the first digit's histogram and the second deal's
//                  per-tile counts.
//   k_hist_heads_* the same for segments dealt on one digit, from their histograms.
//   k_classify     buckets -> runs of small buckets packed per window, medium buckets,
//                  large buckets (recursion) and finished large buckets.
//   k_chunk_desc   the work list's runs of small buckets (and medium buckets) decoded
//                  into chunk descriptors ahead of the local sort.
//   k_local_sort_bucket, k_local_sort
//                  the diversion: each run of small buckets (or medium bucket) sorted
//                  in LDS by bucketing words and ranking them inside their bins, or by
//                  a stable LSD radix sort over only the bits that vary.
//   k_copy_tiles, k_copy_chunks
//                  copies of finished ranges, and the serving gather/scatter.
//   k_key_transform, k_collisions
//                  order-preserving maps of signed/float keys; the plan's collision
//                  estimates and overflow counts from the histograms.
#include "dfr_internal.h"

#include <algorithm>
#include <mutex>

namespace dfr {

template <int B>
struct uint_of {
    using type = uint32_t;
};
template <>
struct uint_of<8> {
    using type = uint64_t;
};

constexpr uint32_t SPIN_LIMIT = 1u << 22;


// Launch shapes.
constexpr int DEAL_THREADS = 512;
constexpr int DEAL_TILE_SMALL = 8192;  // records per deal tile when key + value <= 8 bytes
constexpr int DEAL_TILE_LARGE = 4096;  // records per deal tile for 12- and 16-byte records
constexpr int COUNT_THREADS = 256;
constexpr int COUNT_VECS = 8;          // 16-byte loads in flight per counting thread
constexpr int COUNT_MIN_WAVES = 8;     // waves per SIMD the 32-bit count of up to four digits fits
constexpr int LOCAL_THREADS = 512;
constexpr int LOCAL_CAP_SMALL = 8192;  // general local sort: records per chunk (<= 8-byte records)
constexpr int LOCAL_CAP_LARGE = 4096;  // the same for 12- and 16-byte records
constexpr int BUCKET_CAP_SMALL = 5120; // bucketed local sort: records per chunk (<= 8-byte records)
constexpr int BUCKET_CAP_LARGE = 4096;
constexpr int LOCAL_MIN_WAVES = 6;     // waves per SIMD local-sort forms 1 and 2 must fit (80 VGPRs)
constexpr int LOCAL_MIN_WAVES_FORM0 = 8;  // the same for form 0 (64 VGPRs)
constexpr int COPY_THREADS = 256;
constexpr int HEAD_THREADS = 512;
constexpr int GENERAL_THREADS = 256;
constexpr int LOCAL_RANK_WIN = 4;      // places of a bin the bucketed local sort compares unrolled
// Largest chunk any local-sort kernel accepts (the general kernel's capacity).
constexpr uint32_t LOCAL_CAP_ANY = LOCAL_CAP_SMALL;

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Bit b of d as 0 or ~0, and the lanes where it is set (the compare's lane mask taken on
// that value directly, one instruction for each).
__device__ __forceinline__ uint32_t digit_bit_mask(uint32_t d, int b, uint64_t* lanes) {
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
    *lanes = __builtin_amdgcn_uicmp(m, 0u, 33 /* not equal */);
    return m;
}

// Lanes of the wave (within `active`) whose digit equals this lane's, from one ballot
// per digit bit.  Lane order is input order, so lanes_below() of the result is this
// record's stable rank among equal digits in the wave.  Per bit: the bit as 0 / ~0,
// its ballot, and the lanes whose bit differs (ballot XOR own bit) folded into a
// mismatch mask.
template <int BITS>
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, uint64_t active) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        uint64_t bal;
        const uint32_t m = digit_bit_mask(d, b, &bal);
        lo |= (uint32_t)bal ^ m;
        hi |= (uint32_t)(bal >> 32) ^ m;
    }
    return active & ~(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t same_digit_lanes_rt(uint32_t d, uint64_t active, int bits) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
        if (b < bits) {
            uint64_t bal;
            const uint32_t m = digit_bit_mask(d, b, &bal);
            lo |= (uint32_t)bal ^ m;
            hi |= (uint32_t)(bal >> 32) ^ m;
        }
    }
    return active & ~(((uint64_t)hi << 32) | lo);
}

// Spin (bounded) until a look-back word carries a status.
__device__ __forceinline__ uint64_t wait_published(uint64_t* p, uint32_t* err) {
    uint64_t x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    while ((x & (LB_AGG | LB_PRE)) == 0) {
        if (++spins > SPIN_LIMIT) {
            atomicOr(err, ERR_SPIN);
            return LB_PRE;
        }
        __builtin_amdgcn_s_sleep(2);
        x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return x;
}

// Exclusive scan of one value per thread over threads 0..255 of the block (threads
// above 255 pass anything and ignore the result).  *total gets the sum of the 256.
// Every thread of the block must call it (it holds two barriers).
__device__ __forceinline__ uint32_t scan256_excl(uint32_t x, uint32_t* s_part, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (tid < RADIX && lane == 63) s_part[w] = incl;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < RADIX / 64; ++i) {
        const uint32_t p = s_part[i];
        before += (i < w) ? p : 0u;
        sum += p;
    }
    __syncthreads();
    *total = sum;
    return before + incl - x;
}

template <typename K>
__device__ __forceinline__ K wave_or(K x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}
template <typename K>
__device__ __forceinline__ K wave_and(K x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x &= __shfl_xor(x, o, 64);
    return x;
}

// ---------------------------------------------------------------------------------
// Fill.
// ---------------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// Several fills in one launch (blockIdx.y picks the range): fewer launches on the short
// sorts, where launches rather than bytes take the time.
__global__ void k_fill_set(FillSet f) {
    const int r = blockIdx.y;
    if (r >= f.count) return;
    const uint64_t n = f.n[r];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (f.w[r] == 8) ((uint64_t*)f.p[r])[i] = f.v[r];
        else ((uint32_t*)f.p[r])[i] = (uint32_t)f.v[r];
    }
}

// ---------------------------------------------------------------------------------
// Count (Sec. 2): per-segment digit histograms of up to MAX_PASSES digits, in one read.
// Keys arrive in 16-byte vector loads, all of a thread's share of a tile in flight at
// once.  Each wave keeps private LDS bins.  A digit on which a wave's first keys mostly
// agree (a skewed input) is added per group of equal lanes -- the lanes that share the
// first active lane's digit, or the first other lane's, add their number in one LDS
// atomic -- and otherwise one atomic per key.
// ---------------------------------------------------------------------------------
template <int KB, int THREADS, int NDIG>
__global__ __launch_bounds__(THREADS, KB == 4 && NDIG <= 4 ? COUNT_MIN_WAVES : 1) void k_count(CountArgs a) {
    using K = typename uint_of<KB>::type;
    constexpr int W = THREADS / 64;
    constexpr int SLICE = NDIG * RADIX;  // bins for up to NDIG digits
    constexpr int PER_VEC = 16 / KB;  // keys per 16-byte load
    // 16-byte loads in flight per thread; four for 64-bit keys, whose count otherwise
    // takes 128 VGPRs (four waves per SIMD; with four loads, six).
    constexpr int VECS = KB == 8 ? 4 : COUNT_VECS;
    // The waves' bins; between tiles (all zero) the first words also carry the waves'
    // OR and AND to the segment's flush.  With four digits the two arrays fill exactly
    // an eighth of the LDS, so eight blocks share a CU.
    __shared__ __align__(16) uint32_t s_h[W * SLICE];
    __shared__ uint32_t s_tot[SLICE];  // the block's counts for the current segment
    static_assert(2 * W * sizeof(K) <= sizeof(s_h), "room for the OR/AND words");
    K* const s_or = (K*)s_h;
    K* const s_and = s_or + W;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < W * SLICE; i += THREADS) s_h[i] = 0;
    for (int i = tid; i < SLICE; i += THREADS) s_tot[i] = 0;
    __syncthreads();

    const uint32_t t0 = blockIdx.x * a.tiles_per_block;
    if (t0 >= a.ntiles) return;
    const uint32_t t1 = a.ntiles - t0 < a.tiles_per_block ? a.ntiles : t0 + a.tiles_per_block;
    const int ndig = a.ndig < NDIG ? a.ndig : NDIG, bits = a.bits;
    const int nrow = a.hist_digits > 0 ? a.hist_digits : ndig;  // histogram row stride
    int base = a.base_shift;  // per tile from the segment when a.segs is set
    const uint32_t dmask = (1u << bits) - 1u;
    uint32_t* hw = s_h + w * SLICE;

    uint32_t cur = a.tiles[t0].seg;
    K vor = 0, vand = ~K(0);

    // End of a tile: fold the waves' bins into the block total (and write the tile's
    // own counts when asked).  Each thread owns the same entries in both arrays.
    auto end_tile = [&](uint32_t t) {
        __syncthreads();
        for (int idx = tid; idx < ndig * RADIX; idx += THREADS) {
            uint32_t sum = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                sum += s_h[ww * SLICE + idx];
                s_h[ww * SLICE + idx] = 0;
            }
            s_tot[idx] += sum;
            if (a.tile_hist) a.tile_hist[(size_t)t * nrow * RADIX + idx] = sum;
        }
        __syncthreads();  // bins are clear before any wave counts the next tile
    };
    auto flush = [&](uint32_t seg) {
        __syncthreads();
        for (int idx = tid; idx < ndig * RADIX; idx += THREADS) {
            const uint32_t sum = s_tot[idx];
            s_tot[idx] = 0;
            if (sum && a.hist) atomicAdd(&a.hist[(size_t)seg * nrow * RADIX + idx], sum);
        }
        if (!a.seg_or) {  // per-tile counts only
            __syncthreads();
            return;
        }
        const K o = wave_or(vor), n = wave_and(vand);
        if (lane == 0) {
            s_or[w] = o;
            s_and[w] = n;
        }
        __syncthreads();
        if (tid == 0) {
            K o2 = 0, n2 = ~K(0);
            for (int ww = 0; ww < W; ++ww) {
                o2 |= s_or[ww];
                n2 &= s_and[ww];
                s_or[ww] = 0;  // the bins are zero again before the next tile
                s_and[ww] = 0;
            }
            atomicOr(&((K*)a.seg_or)[seg], o2);
            atomicAnd(&((K*)a.seg_and)[seg], n2);
        }
        __syncthreads();
    };

    // One key into the wave's bins; `skew` marks digits added per group of lanes: the
    // lanes sharing the first active lane's digit, then those sharing the digit of the
    // first lane outside that group, each add their number in one LDS atomic (so a
    // value most lanes share is grouped even when the first lane holds another).
    auto add_key = [&](K key, uint32_t skew) {
        vor |= key;
        vand &= key;
        for (int j = 0; j < ndig; ++j) {
            const uint32_t d = (uint32_t)(key >> (base + j * bits)) & dmask;
            if ((skew >> j) & 1u) {
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                const uint64_t m0 = __ballot(d == d0);
                const uint64_t mo = __ballot(d != d0);
                uint32_t d1 = d0;
                uint64_t m1 = 0;
                if (mo) {
                    d1 = __builtin_amdgcn_readlane(d, __ffsll((unsigned long long)mo) - 1);
                    m1 = __ballot(d == d1);
                }
                if (d == d0) {
                    if (lanes_below(m0) == 0) atomicAdd(&hw[j * RADIX + d0], (uint32_t)__popcll(m0));
                } else if (d == d1) {
                    if (lanes_below(m1) == 0) atomicAdd(&hw[j * RADIX + d1], (uint32_t)__popcll(m1));
                } else {
                    atomicAdd(&hw[j * RADIX + d], 1u);
                }
            } else {
                atomicAdd(&hw[j * RADIX + d], 1u);
            }
        }
    };

    // One key, one atomic per digit (the digit loop unrolled): batches with no skewed
    // digit and no ragged end.
    auto add_plain = [&](K key) {
        vor |= key;
        vand &= key;
#pragma unroll
        for (int j = 0; j < NDIG; ++j)
            if (j < ndig) atomicAdd(&hw[j * RADIX + ((uint32_t)(key >> (base + j * bits)) & dmask)], 1u);
    };

    for (uint32_t t = t0; t < t1; ++t) {
        const Tile tl = a.tiles[t];
        if (tl.seg != cur) {
            flush(cur);
            cur = tl.seg;
            vor = 0;
            vand = ~K(0);
        }
        if (a.segs) base = a.segs[tl.seg].shift[a.pass];
        const K* kp = (const K*)a.keys + tl.start;
        // Unaligned head, 16-byte aligned body, tail.
        uint32_t head = (uint32_t)(((16u - ((uintptr_t)kp & 15u)) & 15u) / KB);
        if (head > tl.len) head = tl.len;
        const uint32_t nvec = (tl.len - head) / PER_VEC;
        const uint32_t tail = head + nvec * PER_VEC;
        for (uint32_t i = tid; i < head; i += THREADS) add_key(kp[i], 0u);
        for (uint32_t i = tail + tid; i < tl.len; i += THREADS) add_key(kp[i], 0u);
        const uint4* vp = (const uint4*)(kp + head);
        for (uint32_t v0 = 0; v0 < nvec; v0 += THREADS * VECS) {
            uint4 buf[VECS];
#pragma unroll
            for (int r = 0; r < VECS; ++r) {
                const uint32_t v = v0 + r * THREADS + tid;
                buf[r] = v < nvec ? vp[v] : make_uint4(0, 0, 0, 0);
            }
            // Skew test on each wave's first vector: digits on which more than a quarter
            // of the lanes share the first lane's value, or the value of the first lane
            // that differs from it.
            uint32_t skew = 0;
            {
                const K k0 = (K)buf[0].x | (KB == 8 ? ((K)buf[0].y << (8 * KB / 2)) : K(0));
                const bool ok0 = v0 + tid < nvec;
                for (int j = 0; j < ndig; ++j) {
                    const uint32_t d = (uint32_t)(k0 >> (base + j * bits)) & dmask;
                    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                    const uint64_t m0 = __ballot(ok0 && d == d0), mo = __ballot(ok0 && d != d0);
                    uint32_t most = (uint32_t)__popcll(m0);
                    if (mo) {
                        const uint32_t d1 = __builtin_amdgcn_readlane(d, __ffsll((unsigned long long)mo) - 1);
                        const uint32_t c1 = (uint32_t)__popcll(__ballot(ok0 && d == d1));
                        most = c1 > most ? c1 : most;
                    }
                    if (most > 16) skew |= 1u << j;
                }
            }
            if (skew == 0 && v0 + THREADS * VECS <= nvec) {
#pragma unroll
                for (int r = 0; r < VECS; ++r) {
                    if (KB == 4) {
                        add_plain((K)buf[r].x);
                        add_plain((K)buf[r].y);
                        add_plain((K)buf[r].z);
                        add_plain((K)buf[r].w);
                    } else {
                        add_plain((K)buf[r].x | ((K)buf[r].y << 32));
                        add_plain((K)buf[r].z | ((K)buf[r].w << 32));
                    }
                }
                continue;
            }
#pragma unroll
            for (int r = 0; r < VECS; ++r) {
                const uint32_t v = v0 + r * THREADS + tid;
                if (v < nvec) {
                    if (KB == 4) {
                        add_key((K)buf[r].x, skew);
                        add_key((K)buf[r].y, skew);
                        add_key((K)buf[r].z, skew);
                        add_key((K)buf[r].w, skew);
                    } else {
                        add_key((K)buf[r].x | ((K)buf[r].y << 32), skew);
                        add_key((K)buf[r].z | ((K)buf[r].w << 32), skew);
                    }
                }
            }
        }
        end_tile(t);
    }
    flush(cur);
}

// ---------------------------------------------------------------------------------
// Deal (Sec. 2; one pass of the LSD phase of Sec. 3).  One tile per block, tiles in
// ticket order so every tile it waits on is already running.
//
// Tile layout: wave w holds records [w*ITEMS*64, (w+1)*ITEMS*64) of the tile, item k
// of lane l being record w*ITEMS*64 + k*64 + l, so a wave meets its records in input
// order and the ballot ranks are stable.
// ---------------------------------------------------------------------------------
template <int KB, int VB, int THREADS, int ITEMS, bool LOOKBACK>
__global__ __launch_bounds__(THREADS) void k_deal(DealArgs a) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    constexpr int W = THREADS / 64;
    constexpr uint32_t T = THREADS * ITEMS;
    static_assert(THREADS >= RADIX, "one thread per digit value");

    __shared__ K s_keys[T];
    __shared__ V s_vals[VB ? T : 1];
    __shared__ uint32_t s_wcnt[W * RADIX];
    // Per digit: the place of the tile's first record of that digit in the segment,
    // minus that record's place in the staged tile, modulo 2^32 (a record at staged
    // index i of digit d goes to segment position s_delta[d] + i; a segment holds fewer
    // than 2^32 records, so the position is exact in 32-bit arithmetic).
    __shared__ uint32_t s_delta[RADIX];
    __shared__ uint32_t s_part[RADIX / 64];
    __shared__ uint32_t s_ticket;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (LOOKBACK && tid == 0) s_ticket = atomicAdd(a.ticket, 1u);
    for (int i = tid; i < W * RADIX; i += THREADS) s_wcnt[i] = 0;
    __syncthreads();
    uint32_t t;
    if (LOOKBACK) {
        t = s_ticket;
    } else {
        // Blocks are dealt to the 8 XCDs round-robin; give each XCD one contiguous
        // range of tiles, so the lines a bucket receives from neighbouring tiles are
        // written through one L2.
        const uint32_t nx = 8, b = blockIdx.x, per = (a.ntiles + nx - 1) / nx;
        const uint32_t full = a.ntiles - (per - 1) * nx;  // XCDs that get `per` tiles
        const uint32_t x = b % nx, i = b / nx;
        t = x < full ? x * per + i : full * per + (x - full) * (per - 1) + i;
        if (i >= (x < full ? per : per - 1)) t = a.ntiles;
    }
    if (t >= a.ntiles) return;

    const Tile tl = a.tiles[t];
    const uint32_t seg_id = tl.seg & ~TILE_IN2;
    const bool in2 = (tl.seg & TILE_IN2) != 0;  // a tile of an overflow area
    const Seg* sg = a.segs + seg_id;
    const uint64_t seg_start = sg->start, seg_end = sg->start + sg->len;
    const uint32_t first_tile = sg->first_tile;
    const int shift = sg->shift[a.pass];
    const uint32_t dmask = (1u << sg->width[a.pass]) - 1u;
    const int hslot = sg->hslot[a.pass];
    const uint32_t len = tl.len;
    const K* kin = (const K*)(in2 ? a.kin2 : a.kin) + tl.start;
    const V* vin = (const V*)(in2 ? a.vin2 : a.vin) + tl.start;

    K key[ITEMS];
    V val[ITEMS];
    uint32_t rnk[ITEMS];
    const uint32_t wbase = (uint32_t)w * ITEMS * 64;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        const bool ok = idx < len;
        key[k] = ok ? kin[idx] : K(0);
        if (VB) val[k] = ok ? vin[idx] : V(0);
    }

    // Stable rank of each record among equal digits, per wave.
    uint32_t* wc = s_wcnt + w * RADIX;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        const bool ok = idx < len;
        const uint64_t act = __ballot(ok);
        const uint32_t d = (uint32_t)(key[k] >> shift) & dmask;
        const uint64_t m = same_digit_lanes<RADIX_BITS>(d, act);
        const uint32_t below = lanes_below(m);
        const uint32_t base = wc[d];
        if (ok && below == 0) wc[d] = base + (uint32_t)__popcll(m);
        rnk[k] = base + below;
    }
    __syncthreads();

    // Per digit: offsets of each wave's run, the tile's count, and its publication.
    uint32_t tile_cnt = 0;
    if (tid < RADIX) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = s_wcnt[ww * RADIX + tid];
            s_wcnt[ww * RADIX + tid] = run;
            run += c;
        }
        tile_cnt = run;
        if (LOOKBACK)
            __hip_atomic_store(&a.lookback[(size_t)t * RADIX + tid],
                               (t == first_tile ? LB_PRE : LB_AGG) | (uint64_t)run, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t total;
    uint32_t seg_excl = 0;
    if (LOOKBACK) {
        const uint32_t hv =
            tid < RADIX ? a.hist[((size_t)seg_id * a.hist_digits + hslot) * RADIX + tid] : 0u;
        seg_excl = scan256_excl(hv, s_part, &total);
    }
    const uint32_t loc_excl = scan256_excl(tile_cnt, s_part, &total);

    if (!LOOKBACK && tid < RADIX) {
        for (int ww = 0; ww < W; ++ww) s_wcnt[ww * RADIX + tid] += loc_excl;  // wave runs from the tile start
        s_delta[tid] = a.off[(size_t)t * RADIX + tid] - loc_excl;
    }
    if (LOOKBACK && tid < RADIX) {
        for (int ww = 0; ww < W; ++ww) s_wcnt[ww * RADIX + tid] += loc_excl;  // wave runs from the tile start
        uint64_t excl = 0;
        if (t != first_tile) {
            uint32_t j = t - 1;
            for (;;) {
                const uint64_t x = wait_published(&a.lookback[(size_t)j * RADIX + tid], a.err);
                excl += x & LB_COUNT;
                if ((x & LB_PRE) || j <= first_tile) break;
                --j;
            }
            __hip_atomic_store(&a.lookback[(size_t)t * RADIX + tid], LB_PRE | (excl + tile_cnt),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_delta[tid] = seg_excl + (uint32_t)excl - loc_excl;
    }
    __syncthreads();

    // Stage the tile in LDS in digit order.
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        if (idx < len) {
            const uint32_t d = (uint32_t)(key[k] >> shift) & dmask;
            const uint32_t p = wc[d] + rnk[k];
            if (p < T) {
                s_keys[p] = key[k];
                if (VB) s_vals[p] = val[k];
            }
        }
    }
    __syncthreads();

    // Runs of equal digits go to consecutive addresses of their bucket.  Positions are
    // 32-bit offsets into the segment (a segment holds fewer than 2^32 records).
    K* kseg = (K*)a.kout + seg_start;
    V* vseg = (V*)a.vout + seg_start;
    const uint32_t seg_len = (uint32_t)(seg_end - seg_start);
    bool bad = false;
    if (len == T) {
        // A full tile: every staged place holds a record, so each step's LDS reads go
        // out for a group of up to eight items together before their stores (measured:
        // 16-byte records 10% faster than item by item).
        constexpr int G = ITEMS < 8 ? ITEMS : 8;
#pragma unroll
        for (int k0 = 0; k0 < ITEMS; k0 += G) {
            K kk[G];
            V vv[VB ? G : 1];
            uint32_t pp[G];
#pragma unroll
            for (int q = 0; q < G; ++q) kk[q] = s_keys[(uint32_t)(k0 + q) * THREADS + tid];
            if (VB) {
#pragma unroll
                for (int q = 0; q < G; ++q) vv[q] = s_vals[(uint32_t)(k0 + q) * THREADS + tid];
            }
#pragma unroll
            for (int q = 0; q < G; ++q)
                pp[q] = s_delta[(uint32_t)(kk[q] >> shift) & dmask] + (uint32_t)(k0 + q) * THREADS + tid;
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (pp[q] < seg_len) {
                    kseg[pp[q]] = kk[q];
                    if (VB) vseg[pp[q]] = vv[q];
                } else {
                    bad = true;
                }
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = (uint32_t)k * THREADS + tid;
            if (i < len) {
                const K kk = s_keys[i];
                const uint32_t d = (uint32_t)(kk >> shift) & dmask;
                const uint32_t p = s_delta[d] + i;
                if (p < seg_len) {
                    kseg[p] = kk;
                    if (VB) vseg[p] = s_vals[i];
                } else {
                    bad = true;
                }
            }
        }
    }
    if (bad) atomicOr(a.err, ERR_RANGE);
}

// ---------------------------------------------------------------------------------
// Fast Radix's deal without a count (Sec. 3): bucket v is estimated to hold E = n / 2^b
// records and gets the slots [v * E, v * E + E); records past its estimate go to its
// overflow slots [v * C, v * C + C) of a second area, where C is sized from the
// expected overflow (Eq. 2; a few standard deviations of a bucket's count).  Each
// record's rank in its bucket comes from decoupled look-back over the tiles (ticket
// order), so every bucket keeps input order: its estimated slots, then its overflow
// slots, in that order, are its records in input order.  The tile also counts the next
// digit of its records: that histogram gives the exact pass that follows its bucket
// starts (the penultimate pass counts the last digit, Sec. 3).  A record that finds no
// slot is counted in *lost; the caller then redoes the pass with counted buckets.
// ---------------------------------------------------------------------------------
template <int KB, int VB, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_deal_est(EstArgs a) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    constexpr int W = THREADS / 64;
    constexpr uint32_t T = THREADS * ITEMS;
    static_assert(THREADS >= RADIX, "one thread per digit value");
    __shared__ K s_keys[T];
    __shared__ V s_vals[VB ? T : 1];
    __shared__ uint32_t s_wcnt[W * RADIX];
    __shared__ uint32_t s_delta[RADIX];  // rank in the bucket of staged index 0, mod 2^32
    __shared__ uint32_t s_next[RADIX];
    __shared__ uint32_t s_part[RADIX / 64];
    __shared__ uint32_t s_ticket, s_lost;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) {
        s_ticket = atomicAdd(a.ticket, 1u);
        s_lost = 0;
    }
    for (int i = tid; i < W * RADIX; i += THREADS) s_wcnt[i] = 0;
    for (int i = tid; i < RADIX; i += THREADS) s_next[i] = 0;
    __syncthreads();
    const uint32_t t = s_ticket;
    if (t >= a.ntiles) return;
    const uint64_t start = (uint64_t)t * a.tile;
    const uint32_t len = (uint32_t)umin64(a.tile, a.n - start);
    const uint32_t dmask = (1u << a.width) - 1u, nmask = (1u << a.nwidth) - 1u;
    const K* kin = (const K*)a.kin + start;
    const V* vin = (const V*)a.vin + start;

    K key[ITEMS];
    V val[ITEMS];
    uint32_t rnk[ITEMS];
    const uint32_t wbase = (uint32_t)w * ITEMS * 64;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        const bool ok = idx < len;
        key[k] = ok ? kin[idx] : K(0);
        if (VB) val[k] = ok ? vin[idx] : V(0);
    }
    uint32_t* wc = s_wcnt + w * RADIX;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        const bool ok = idx < len;
        const uint64_t act = __ballot(ok);
        const uint32_t d = (uint32_t)(key[k] >> a.shift) & dmask;
        const uint64_t m = same_digit_lanes<RADIX_BITS>(d, act);
        const uint32_t below = lanes_below(m);
        const uint32_t base = wc[d];
        if (ok && below == 0) wc[d] = base + (uint32_t)__popcll(m);
        rnk[k] = base + below;
        if (ok) atomicAdd(&s_next[(uint32_t)(key[k] >> a.nshift) & nmask], 1u);
    }
    __syncthreads();

    // Per digit: offsets of each wave's run, the tile's count, its publication, and the
    // bucket totals; then the rank in the bucket of the tile's first record of the digit.
    uint32_t tile_cnt = 0;
    if (tid < RADIX) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = s_wcnt[ww * RADIX + tid];
            s_wcnt[ww * RADIX + tid] = run;
            run += c;
        }
        tile_cnt = run;
        __hip_atomic_store(&a.lookback[(size_t)t * RADIX + tid], (t == 0 ? LB_PRE : LB_AGG) | (uint64_t)run,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (run) atomicAdd(&a.cnt[tid], run);
        const uint32_t nx = s_next[tid];
        if (nx) atomicAdd(&a.next_hist[tid], nx);
    }
    uint32_t total;
    const uint32_t loc_excl = scan256_excl(tile_cnt, s_part, &total);
    if (tid < RADIX) {
        for (int ww = 0; ww < W; ++ww) s_wcnt[ww * RADIX + tid] += loc_excl;  // wave runs from the tile start
        uint64_t excl = 0;
        if (t != 0) {
            uint32_t j = t - 1;
            for (;;) {
                const uint64_t x = wait_published(&a.lookback[(size_t)j * RADIX + tid], a.err);
                excl += x & LB_COUNT;
                if ((x & LB_PRE) || j == 0) break;
                --j;
            }
            __hip_atomic_store(&a.lookback[(size_t)t * RADIX + tid], LB_PRE | (excl + tile_cnt),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_delta[tid] = (uint32_t)excl - loc_excl;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        if (idx < len) {
            const uint32_t d = (uint32_t)(key[k] >> a.shift) & dmask;
            const uint32_t p = wc[d] + rnk[k];
            if (p < T) {
                s_keys[p] = key[k];
                if (VB) s_vals[p] = val[k];
            }
        }
    }
    __syncthreads();
    // Runs of equal digits go to consecutive slots of their bucket (or of its overflow).
    K* kout = (K*)a.kout;
    V* vout = (V*)a.vout;
    K* kovf = (K*)a.kovf;
    V* vovf = (V*)a.vovf;
    uint32_t lost = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = (uint32_t)k * THREADS + tid;
        if (i < len) {
            const K kk = s_keys[i];
            const uint32_t d = (uint32_t)(kk >> a.shift) & dmask;
            const uint64_t r = (uint64_t)(s_delta[d] + i);  // rank in bucket d
            if (r < a.E) {
                kout[(uint64_t)d * a.E + r] = kk;
                if (VB) vout[(uint64_t)d * a.E + r] = s_vals[i];
            } else if (r - a.E < a.C) {
                const uint64_t q = (uint64_t)d * a.C + (r - a.E);
                kovf[q] = kk;
                if (VB) vovf[q] = s_vals[i];
            } else {
                ++lost;
            }
        }
    }
    if (lost) atomicAdd(&s_lost, lost);
    __syncthreads();
    if (tid == 0 && s_lost) atomicAdd(a.lost, s_lost);
}

// ---------------------------------------------------------------------------------
// Bucket heads (Sec. 2.2 buckets; Sec. 3: after the deals, the buckets are found so that
// those still too large for the diversion can be recursed on).
// After the deals, records of a segment are ordered by their bits >= lo_bit; a
// bucket starts where those bits change (or at the segment start).  Heads are
// written in position order: wave ballots inside the tile, look-back across tiles.
// ---------------------------------------------------------------------------------
template <int KB, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_heads(HeadArgs a) {
    using K = typename uint_of<KB>::type;
    constexpr int W = THREADS / 64;
    constexpr int KBITS = 8 * KB;
    __shared__ uint32_t s_wtot[W];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t t = blockIdx.x;
    if (t >= a.ntiles) return;
    const Tile tl = a.tiles[t];
    const Seg* sg = a.segs + tl.seg;
    const int lo = sg->lo_bit;
    const uint64_t seg_start = sg->start;
    const K* kp = (const K*)a.keys + tl.start;
    const uint32_t len = tl.len;
    const uint32_t wbase = (uint32_t)w * ITEMS * 64;

    // All loads first; a record's predecessor comes from the lane (or item) before.
    K key[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        key[k] = idx < len ? kp[idx] : K(0);
    }
    const uint64_t gpos0 = tl.start + wbase;  // position of the wave's first record
    K before = 0;
    if (lane == 0 && wbase < len && gpos0 > seg_start) before = kp[(int64_t)wbase - 1];

    uint32_t off[ITEMS];
    bool head[ITEMS];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t idx = wbase + k * 64 + lane;
        const bool ok = idx < len;
        const K up = __shfl_up(key[k], 1, 64);
        const K last = k > 0 ? __shfl(key[k > 0 ? k - 1 : 0], 63, 64) : before;
        const K prev = lane == 0 ? last : up;
        const uint64_t gpos = tl.start + idx;
        bool h = false;
        if (ok) {
            if (gpos == seg_start) h = true;
            else if (lo < KBITS) h = (key[k] >> lo) != (prev >> lo);
        }
        head[k] = h;
        const uint64_t hb = __ballot(h);
        off[k] = run + lanes_below(hb);
        run += (uint32_t)__popcll(hb);
    }
    if (lane == 0) s_wtot[w] = run;
    __syncthreads();
    uint32_t tot = 0, wexcl = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
        wexcl += ww < w ? s_wtot[ww] : 0u;
        tot += s_wtot[ww];
    }
    if (tid == 0) a.tcount[t] = tot;
    if (tot > HEAD_SLOTS) return;  // listed again from the keys (k_heads_emit)
    uint16_t* slot = a.tslot + (size_t)t * HEAD_SLOTS;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (head[k]) slot[wexcl + off[k]] = (uint16_t)(wbase + k * 64 + lane);
}

// Exclusive scan of the tiles' head counts (one block): tile bases in the bucket list.
// Each wave owns a contiguous range of tiles and reads it 64 tiles wide, eight loads in
// flight per lane.
__global__ __launch_bounds__(1024) void k_heads_scan(HeadArgs a) {
    constexpr uint32_t NW = 1024 / 64, U = 8;
    __shared__ uint64_t s_part[NW];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t per = ((a.ntiles + NW - 1) / NW + 63) / 64 * 64;
    const uint32_t w0 = w * per < a.ntiles ? w * per : a.ntiles;
    const uint32_t w1 = w0 + per < a.ntiles ? w0 + per : a.ntiles;
    uint64_t sum = 0;
    for (uint32_t b = w0; b < w1; b += 64 * U) {
        uint32_t c[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = b + u * 64 + lane;
            c[u] = i < w1 ? a.tcount[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) sum += c[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane == 0) s_part[w] = sum;
    __syncthreads();
    uint64_t run = 0, total = 0;
#pragma unroll
    for (uint32_t ww = 0; ww < NW; ++ww) {
        run += ww < w ? s_part[ww] : 0ull;
        total += s_part[ww];
    }
    for (uint32_t b = w0; b < w1; b += 64 * U) {
        uint32_t c[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = b + u * 64 + lane;
            c[u] = i < w1 ? a.tcount[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            uint64_t incl = c[u];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t y = __shfl_up(incl, o, 64);
                if ((int)lane >= o) incl += y;
            }
            const uint32_t i = b + u * 64 + lane;
            if (i < w1) a.tbase[i] = run + incl - c[u];
            run += __shfl(incl, 63, 64);
        }
    }
    if (threadIdx.x == 0) *a.nbuckets = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
}

// The bucket list in position order: one wave per tile copies the tile's kept heads,
// or finds them again from the keys when the tile had more than HEAD_SLOTS.
template <int KB>
__global__ __launch_bounds__(256) void k_heads_emit(HeadArgs a) {
    using K = typename uint_of<KB>::type;
    constexpr int KBITS = 8 * KB;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wid = (blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * 4;
    bool over = false;
    for (uint32_t t = wid; t < a.ntiles; t += nw) {
        const uint32_t n = a.tcount[t];
        const uint64_t base = a.tbase[t];
        const Tile tl = a.tiles[t];
        if (n <= HEAD_SLOTS) {
            const uint16_t* slot = a.tslot + (size_t)t * HEAD_SLOTS;
            for (uint32_t i = lane; i < n; i += 64) {
                const uint64_t gi = base + i;
                if (gi < a.bcap) {
                    a.bstart[gi] = tl.start + slot[i];
                    a.bseg[gi] = tl.seg;
                } else {
                    over = true;
                }
            }
            continue;
        }
        // More heads than slots: find them again, U rows of 64 keys per step (the loads
        // of a step issue together); a key's predecessor is the lane below, or the last
        // key of the row before.
        const Seg* sg = a.segs + tl.seg;
        const int lo = sg->lo_bit;
        const K* kp = (const K*)a.keys + tl.start;
        const bool seg_first = tl.start == sg->start;  // the tile opens its segment
        K carry = seg_first ? K(0) : kp[-1];
        uint64_t run = base;
        constexpr int U = 8;
        for (uint32_t i0 = 0; i0 < tl.len; i0 += 64 * U) {
            K x[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t idx = i0 + k * 64 + lane;
                x[k] = idx < tl.len ? kp[idx] : K(0);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const uint32_t idx = i0 + k * 64 + lane;
                K prev = __shfl_up(x[k], 1, 64);
                const K row_end = k > 0 ? __shfl(x[k > 0 ? k - 1 : 0], 63, 64) : carry;
                if (lane == 0) prev = row_end;
                bool h = false;
                if (idx < tl.len) {
                    if (idx == 0 && seg_first) h = true;
                    else if (lo < KBITS) h = (x[k] >> lo) != (prev >> lo);
                }
                const uint64_t hb = __ballot(h);
                if (h) {
                    const uint64_t gi = run + lanes_below(hb);
                    if (gi < a.bcap) {
                        a.bstart[gi] = tl.start + idx;
                        a.bseg[gi] = tl.seg;
                    } else {
                        over = true;
                    }
                }
                run += (uint64_t)__popcll(hb);
            }
            carry = __shfl(x[U - 1], 63, 64);
        }
    }
    if (over) atomicOr(a.err, ERR_BUCKET_CAP);
}

// ---------------------------------------------------------------------------------
// Bucket heads without reading the keys, for a one-segment level dealt on two digits
// (the lower, u, then the upper, v).  The level's buckets are the non-empty pairs
// (v, u), in that order, so their starts are an exclusive scan of the pair counts.
// After the first deal the records of each u fill one known range (the u histogram's
// prefix sum); the second deal's per-tile counts of v, summed over the tiles wholly
// inside that range, plus a direct count of the records of the range in the (at most
// two) tiles it shares with its neighbours, give the pair counts.
//
// k_joint_counts: one block per u; its four groups of RADIX threads sum a quarter of
// the range's tiles each, eight tiles in flight, and share the key counting.
// k_joint_rows: one block per v, the records and non-empty pairs of row v.
// k_joint_emit: one block per v, the row's pairs scanned after the rows before it; the
// non-empty ones are listed.
// ---------------------------------------------------------------------------------
constexpr int JOINT_GROUPS = 4;
template <int KB>
__global__ __launch_bounds__(JOINT_GROUPS * RADIX) void k_joint_counts(JointArgs a) {
    using K = typename uint_of<KB>::type;
    __shared__ uint32_t s_c[RADIX];
    __shared__ uint32_t s_g[JOINT_GROUPS][RADIX];
    __shared__ uint32_t s_sum[RADIX / 64];
    const uint32_t u = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t v = tid % RADIX, grp = tid / RADIX;
    const uint32_t n0 = 1u << a.width0, n1 = 1u << a.width1;
    // Start of u's range: the sum of the histogram below u.
    if (tid < RADIX) {
        uint32_t x = tid < u ? a.h0[tid] : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) s_sum[w] = x;
        s_c[tid] = 0;
    }
    __syncthreads();
    uint64_t lo = 0;
#pragma unroll
    for (int ww = 0; ww < RADIX / 64; ++ww) lo += s_sum[ww];
    const uint64_t hi = lo + a.h0[u];
    const uint64_t len = a.seg_len, T = a.tile;
    uint32_t sum = 0;
    if (hi > lo && hi <= len) {
        // Tiles t with t*T >= lo and min((t+1)*T, len) <= hi.
        const uint64_t t0 = (lo + T - 1) / T;
        const uint64_t t1 = hi == len ? (uint64_t)a.ntiles : hi / T;
        uint64_t p0 = lo, p1 = hi, q0 = hi, q1 = hi;  // ranges counted from the keys
        if (t0 < t1) {
            if (v < n1) {
                constexpr int U = 8;
                uint32_t acc[U] = {};
                uint64_t t = t0 + grp;
                for (; t + (U - 1) * JOINT_GROUPS < t1; t += U * JOINT_GROUPS) {
#pragma unroll
                    for (int r = 0; r < U; ++r) acc[r] += a.tcnt[(t + r * JOINT_GROUPS) * RADIX + v];
                }
                for (; t < t1; t += JOINT_GROUPS) acc[0] += a.tcnt[t * RADIX + v];
#pragma unroll
                for (int r = 0; r < U; ++r) sum += acc[r];
            }
            p1 = t0 * T;
            q0 = t1 * T < len ? t1 * T : len;
        }
        const K* kp = (const K*)a.keys + a.seg_start;
        const uint32_t m1 = n1 - 1;
        for (uint64_t i = p0 + tid; i < p1; i += JOINT_GROUPS * RADIX)
            atomicAdd(&s_c[(uint32_t)(kp[i] >> a.shift1) & m1], 1u);
        for (uint64_t i = q0 + tid; i < q1; i += JOINT_GROUPS * RADIX)
            atomicAdd(&s_c[(uint32_t)(kp[i] >> a.shift1) & m1], 1u);
    } else if (hi > len) {
        if (tid == 0) atomicOr(a.err, ERR_RANGE);
    }
    s_g[grp][v] = sum;
    __syncthreads();
    if (tid < n1) {
        uint32_t c = s_c[tid];
#pragma unroll
        for (int g = 0; g < JOINT_GROUPS; ++g) c += s_g[g][tid];
        a.joint[(size_t)tid * n0 + u] = c;
    }
}

// Exclusive scan of 64-bit values over a block of RADIX threads; returns the exclusive
// prefix and sets *total.
__device__ __forceinline__ uint64_t scan256_excl64(uint64_t x, uint64_t* s_part, uint64_t* total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint64_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += y;
    }
    if (lane == 63) s_part[w] = incl;
    __syncthreads();
    uint64_t run = incl - x, tot = 0;
#pragma unroll
    for (uint32_t ww = 0; ww < RADIX / 64; ++ww) {
        if (ww < w) run += s_part[ww];
        tot += s_part[ww];
    }
    *total = tot;
    return run;
}

// Records (low 32 bits) and non-empty pairs (high 32 bits) of one pair count.
__device__ __forceinline__ uint64_t pair_word(uint32_t c) {
    return (uint64_t)c | ((uint64_t)(c != 0) << 32);
}

__global__ __launch_bounds__(RADIX) void k_joint_rows(JointArgs a) {
    __shared__ uint64_t s_part[RADIX / 64];
    const uint32_t v = blockIdx.x, tid = threadIdx.x;
    const uint32_t n0 = 1u << a.width0;
    const uint64_t x = tid < n0 ? pair_word(a.joint[(size_t)v * n0 + tid]) : 0ull;
    uint64_t total;
    scan256_excl64(x, s_part, &total);
    if (tid == 0) a.rows[v] = total;
}

__global__ __launch_bounds__(RADIX) void k_joint_emit(JointArgs a) {
    __shared__ uint64_t s_part[RADIX / 64];
    const uint32_t v = blockIdx.x, tid = threadIdx.x;
    const uint32_t n0 = 1u << a.width0, n1 = 1u << a.width1;
    uint64_t before;
    scan256_excl64(tid < v ? a.rows[tid] : 0ull, s_part, &before);
    __syncthreads();  // s_part is used again
    const uint32_t c = tid < n0 ? a.joint[(size_t)v * n0 + tid] : 0u;
    uint64_t total;
    const uint64_t at = before + scan256_excl64(pair_word(c), s_part, &total);
    if (c) {
        const uint64_t idx = at >> 32;
        if (idx < a.bcap) {
            a.bstart[idx] = a.seg_start + (uint32_t)at;
            a.bseg[idx] = a.seg;
        } else {
            atomicOr(a.err, ERR_BUCKET_CAP);
        }
    }
    if (v == n1 - 1 && tid == 0) {
        const uint64_t all = before + total;
        *a.nbuckets = (uint32_t)(all >> 32);
        // Every record of the segment is in exactly one pair.
        if ((uint32_t)all != (uint32_t)a.seg_len) atomicOr(a.err, ERR_RANGE);
    }
}

// ---------------------------------------------------------------------------------
// Bucket heads of a level whose segments are all dealt on one digit, from the digit's
// histogram of each segment (no read of the keys): one block per segment counts its
// non-empty values, one block scans those counts into each segment's first list index,
// and one block per segment lists its buckets (exclusive scan of the histogram).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hist_value(const HistHeadArgs& a, uint32_t s, const Seg& sg,
                                               uint32_t v) {
    const uint32_t n0 = 1u << sg.width[0];
    return v < n0 ? a.hist[((size_t)s * a.hist_digits + sg.hslot[0]) * RADIX + v] : 0u;
}

__global__ __launch_bounds__(RADIX) void k_hist_heads_count(HistHeadArgs a) {
    __shared__ uint32_t s_n[RADIX / 64];
    const uint32_t i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t s = a.ids[i];
    const Seg sg = a.segs[s];
    const uint64_t m = __ballot(hist_value(a, s, sg, tid) != 0);
    if (lane == 0) s_n[w] = (uint32_t)__popcll(m);
    __syncthreads();
    if (tid == 0) {
        uint32_t n = 0;
        for (int ww = 0; ww < RADIX / 64; ++ww) n += s_n[ww];
        a.first[i] = n;
    }
}

constexpr int HIST_SCAN_THREADS = 1024;
__global__ __launch_bounds__(HIST_SCAN_THREADS) void k_hist_heads_scan(HistHeadArgs a) {
    __shared__ uint32_t s_part[HIST_SCAN_THREADS / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t per = (a.nids + HIST_SCAN_THREADS - 1) / HIST_SCAN_THREADS;
    const uint32_t i0 = tid * per < a.nids ? tid * per : a.nids;
    const uint32_t i1 = i0 + per < a.nids ? i0 + per : a.nids;
    uint32_t mine = 0;
    for (uint32_t i = i0; i < i1; ++i) mine += a.first[i];
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += y;
    }
    if (lane == 63) s_part[w] = incl;
    __syncthreads();
    uint32_t run = incl - mine, total = 0;
    for (uint32_t ww = 0; ww < HIST_SCAN_THREADS / 64; ++ww) {
        if (ww < w) run += s_part[ww];
        total += s_part[ww];
    }
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t c = a.first[i];
        a.first[i] = run;
        run += c;
    }
    if (tid == 0) *a.nbuckets = total;
}

__global__ __launch_bounds__(RADIX) void k_hist_heads_emit(HistHeadArgs a) {
    __shared__ uint64_t s_part[RADIX / 64];
    const uint32_t i = blockIdx.x, tid = threadIdx.x;
    const uint32_t s = a.ids[i];
    const Seg sg = a.segs[s];
    const uint32_t c = hist_value(a, s, sg, tid);
    uint64_t total;
    const uint64_t at = scan256_excl64(pair_word(c), s_part, &total);
    if (c) {
        const uint64_t idx = (uint64_t)a.first[i] + (at >> 32);
        if (idx < a.bcap) {
            a.bstart[idx] = sg.start + (uint32_t)at;
            a.bseg[idx] = s;
        } else {
            atomicOr(a.err, ERR_BUCKET_CAP);
        }
    }
    // Every record of the segment has one value of the digit.
    if (tid == 0 && (uint32_t)total != (uint32_t)sg.len) atomicOr(a.err, ERR_RANGE);
}

// ---------------------------------------------------------------------------------
// Classify buckets (Sec. 3: runs of small buckets are sorted in bulk, large buckets
// recursively).  Window width = wsmall <= cap/2: the small buckets starting in one
// window of a segment are contiguous (a bucket longer than wsmall is the last to start
// in its window) and span at most 2*wsmall records, so each window's run is one
// local-sort chunk.
// ---------------------------------------------------------------------------------
// Appends one entry for every lane of the wave that wants to, with one atomic on the
// list's counter; returns each such lane's index.  All lanes of the wave call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool want) {
    const uint64_t m = __ballot(want);
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
        base = __shfl(base, leader, 64);
    }
    return base + lanes_below(m);
}

// Buckets of a segment are listed in position order, so a window's first and last small
// bucket are found from the neighbours: a small bucket opens its window when the bucket
// before lies in another segment or window, and closes it when the bucket after lies in
// another segment or window or is not small.  (A bucket that is not small ends past its
// own window, so every bucket before it in that window is small and none comes after.)
constexpr uint32_t CLASSIFY_THREADS = 256;
constexpr uint32_t CLASSIFY_WBUF = 2048;  // work items a block gathers before listing them
__global__ __launch_bounds__(CLASSIFY_THREADS) void k_classify(ClassifyArgs a) {
    // Work items are gathered in LDS and listed with one atomic per CLASSIFY_WBUF of
    // them: a level with many windows would otherwise queue on the list's one counter.
    __shared__ uint32_t s_work[CLASSIFY_WBUF];
    __shared__ uint32_t s_nw, s_base;
    const uint64_t nb = umin64(*a.nbuckets, a.bcap);
    bool over = false;
    if (threadIdx.x == 0) s_nw = 0;
    __syncthreads();
    auto flush = [&]() {  // every thread of the block
        __syncthreads();
        const uint32_t cnt = s_nw;
        if (threadIdx.x == 0) s_base = cnt ? atomicAdd(a.nwork, cnt) : 0u;
        __syncthreads();
        const uint32_t base = s_base;
        for (uint32_t i = threadIdx.x; i < cnt; i += CLASSIFY_THREADS) {
            if ((uint64_t)base + i < a.workcap) a.work[base + i] = s_work[i];
            else over = true;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_nw = 0;
        __syncthreads();
    };
    const uint64_t stride = (uint64_t)gridDim.x * CLASSIFY_THREADS;
    for (uint64_t b0 = (uint64_t)blockIdx.x * CLASSIFY_THREADS; b0 < nb; b0 += stride) {
        const uint64_t b = b0 + threadIdx.x;
        int kind = 0;  // 1 medium, 2 small, 3 done, 4 large
        uint64_t start = 0, len = 0, slot = 0;
        bool first = false;
        int lo_bit = 0;
        if (b < nb) {
            const uint32_t s = a.bseg[b];
            const Seg* sg = a.segs + s;
            start = a.bstart[b];
            lo_bit = sg->lo_bit;
            const uint64_t seg_end = sg->start + sg->len;
            const bool next_same = b + 1 < nb && a.bseg[b + 1] == s;
            const uint64_t end = next_same ? a.bstart[b + 1] : seg_end;
            len = end - start;
            if (len <= a.cap && (len > a.wsmall || lo_bit >= a.kbits)) {
                // Medium bucket, or a bucket with no prefix bits to tell it from its
                // neighbours (a whole caller segment): a chunk of its own.
                kind = 1;
            } else if (len <= a.wsmall) {
                kind = 2;
                slot = sg->window_base + (start - sg->start) / a.wsmall;
                first = !(b > 0 && a.bseg[b - 1] == s &&
                          sg->window_base + (a.bstart[b - 1] - sg->start) / a.wsmall == slot);
                bool last = true;
                if (next_same) {
                    const uint64_t nend = (b + 2 < nb && a.bseg[b + 2] == s) ? a.bstart[b + 2] : seg_end;
                    last = sg->window_base + (end - sg->start) / a.wsmall != slot || nend - end > a.wsmall;
                }
                if (slot < a.nslots) {
                    if (first) a.cfirst[slot] = (uint32_t)b;
                    if (last) a.clast[slot] = (uint32_t)b;
                } else {
                    over = true;
                    first = false;
                }
            } else {
                kind = lo_bit == 0 ? 3 : 4;
            }
        }
        const uint32_t mi = wave_append(a.nmed, kind == 1);
        bool med = false;
        if (kind == 1) {
            if (mi < a.medcap) {
                a.med[mi] = (uint32_t)b;
                med = true;
            } else {
                over = true;
            }
        }
        // Work items: each medium bucket, and each window once (from its first bucket).
        const bool work = med || (kind == 2 && first);
        const uint32_t wp = wave_append(&s_nw, work);  // < CLASSIFY_WBUF: see the flush below
        if (work) s_work[wp] = med ? a.nslots + mi : (uint32_t)slot;
        const uint32_t di = wave_append(a.ndone, kind == 3);
        if (kind == 3) {
            if (di < a.donecap) a.done[di] = Big{start, (uint32_t)len, 0u};
            else over = true;
        }
        const uint32_t gi = wave_append(a.nbig, kind == 4);
        if (kind == 4) {
            if (gi < a.bigcap) a.big[gi] = Big{start, (uint32_t)len, (uint32_t)lo_bit};
            else over = true;
        }
        // A step adds at most CLASSIFY_THREADS items: list them while that still fits.
        __syncthreads();
        const bool full = s_nw > CLASSIFY_WBUF - CLASSIFY_THREADS;
        __syncthreads();  // every thread has read the count before the next step adds to it
        if (full) flush();
    }
    flush();
    if (over) atomicOr(a.err, ERR_LIST_CAP);
}


using Chunk = ChunkDesc;

// A local-sort work item is a window slot (a run of small buckets) or a medium bucket
// (item >= nslots).  Its chunk comes from the window's first and last bucket (or the
// medium bucket) and the bucket list; false for an empty window, and for a malformed
// item (reported when `report` is set).
__device__ __forceinline__ bool decode_chunk(const LocalArgs& a, uint32_t item, uint64_t nb,
                                             uint32_t cap, Chunk& ch, bool report) {
    uint32_t f, l;
    if (item < a.nslots) {
        f = a.cfirst[item];
        if (f == 0xffffffffu) return false;
        l = a.clast[item];
    } else {
        f = l = a.med[item - a.nslots];
    }
    if ((uint64_t)l >= nb || f > l) {
        if (report) atomicOr(a.err, ERR_CHUNK);
        return false;
    }
    const uint32_t s = a.bseg[f];
    const Seg* sg = a.segs + s;
    const uint64_t start = a.bstart[f];
    const uint64_t end =
        ((uint64_t)l + 1 < nb && a.bseg[l + 1] == s) ? a.bstart[l + 1] : sg->start + sg->len;
    const uint64_t len = end - start;
    if (len > cap || len == 0) {
        if (report) atomicOr(a.err, ERR_CHUNK);
        return false;
    }
    ch.start = start;
    ch.len = (uint32_t)len;
    ch.nbk = l - f + 1;
    ch.f = f;
    ch.lo = sg->lo_bit;
    return true;
}

// The work list's chunks, decoded ahead of the local sort (one item per thread): the
// dependent reads of the bucket lists then overlap across items, and each sorting
// block reads one descriptor per chunk.
__global__ __launch_bounds__(256) void k_chunk_desc(LocalArgs a) {
    const uint64_t nb = umin64(*a.nbuckets, a.bcap);
    const uint32_t nwork = *a.nwork < a.workcap ? *a.nwork : a.workcap;
    for (uint32_t it = blockIdx.x * 256u + threadIdx.x; it < nwork; it += gridDim.x * 256u) {
        Chunk ch{};
        if (!decode_chunk(a, a.work[it], nb, LOCAL_CAP_ANY, ch, true)) ch.len = 0;
        a.desc[it] = ch;
    }
}

// Offsets from per-wave digit counts (digit-major, then wave order), computed by wave 0
// alone; every thread calls it, only wave 0 works.
template <int W>
__device__ __forceinline__ void wave0_offsets(uint32_t* cnt, int w, int lane) {
    if (w != 0) return;
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < RADIX / 64; ++q) {
#pragma unroll
        for (int ww = 0; ww < W; ++ww) sum += cnt[ww * RADIX + lane * (RADIX / 64) + q];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int q = 0; q < RADIX / 64; ++q) {
        const int v = lane * (RADIX / 64) + q;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = cnt[ww * RADIX + v];
            cnt[ww * RADIX + v] = run;
            run += c;
        }
    }
}

// The sort phase of the bucketed local sort, on words of type WT: 32-bit when the
// sort bits and the position fit in 32 bits, else 64-bit.  Item k of thread tid is
// record k * THREADS + tid of the chunk, so every thread's first nfull items hold
// records and item nfull holds one for the threads below rem (item_valid).  x holds
// the chunk's keys as loaded; s_rel the buckets' starts relative to the chunk
// (nbk > 1).  Returns false, uniformly across the block, when the largest bin exceeds
// GMAX (the chunk then goes to the stable kernel); otherwise the chunk is sorted into
// kout/vout.
template <typename K, int MAXI>
struct Keys {
    K v[MAXI];
};

__device__ __forceinline__ bool item_valid(int k, uint32_t nfull, uint32_t rem, int tid) {
    return (uint32_t)k < nfull || ((uint32_t)k == nfull && (uint32_t)tid < rem);
}

template <typename WT, bool SEPPOS, bool WIDE, int KB, int VB, int THREADS, int CAP, int IB, int DB, int MAXI>
__device__ __forceinline__ bool bucket_sort_chunk(
    const Keys<typename uint_of<KB>::type, MAXI>& x, uint32_t len, uint32_t nfull, uint32_t rem, int lane, int w,
    int tid, uint32_t nbk, bool direct, int lo, int h, int B, typename uint_of<KB>::type key0,
    const typename uint_of<KB>::type* kin, const typename uint_of<VB>::type* vin,
    typename uint_of<KB>::type* kout, typename uint_of<VB>::type* vout, const uint32_t* s_rel,
    WT* s_w, uint16_t* s_pos, uint32_t* s_bin, uint32_t* s_part, uint32_t* s_max) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    constexpr int W = THREADS / 64;
    constexpr uint32_t GMAX = 64;
    constexpr int RANK_WIN = LOCAL_RANK_WIN;
    // With SEPPOS the words hold the sort bits only and the position sits beside them in
    // s_pos (ties broken by it); otherwise the words carry it in their low IB bits.
    constexpr int PB = SEPPOS ? 0 : IB;
    constexpr int KBITS = 8 * KB, WBITS = 8 * (int)sizeof(WT);
    const K mask_h = h >= KBITS ? ~K(0) : (K)((K(1) << h) - K(1));
    // The bucket index sits above the h sort bits.  h reaches WBITS only where that
    // index is 0 (the words then hold the sort bits alone), so shifts by h are taken
    // modulo WBITS and the bucket part is masked off in that case.
    const int hsh = h & (WBITS - 1);
    const WT bmask = h >= WBITS ? WT(0) : ~WT(0);
    WT xw[MAXI];

#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
        const uint32_t idx = (uint32_t)k * THREADS + tid;
        uint32_t bi = 0;
        if (direct) {
            bi = (uint32_t)((x.v[k] >> lo) - (key0 >> lo));
        } else if (nbk > 1) {
            uint32_t lo_i = 0, hi_i = nbk;  // last i with s_rel[i] <= idx
            while (hi_i - lo_i > 1) {
                const uint32_t mid = (lo_i + hi_i) >> 1;
                if (s_rel[mid] <= idx) lo_i = mid;
                else hi_i = mid;
            }
            bi = lo_i;
        }
        xw[k] = (WT)((((WT)(x.v[k] & mask_h) | ((WT)bi << hsh)) << PB) | (SEPPOS ? 0u : idx));
    }
    const int nbits = B < DB ? B : DB;
    const uint32_t nbins = 1u << nbits;
    const int dshift = PB + B - nbits;
    // Counters: one 32-bit word per bin (WIDE), or two 16-bit halves per word.
    if (nbk > 1 && !direct) __syncthreads();  // s_rel no longer needed
    // Slots inside the bins.
    uint32_t slot[MAXI];
#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
        slot[k] = 0;
        if (item_valid(k, nfull, rem, tid)) {
            const uint32_t d = (uint32_t)(xw[k] >> dshift) & (nbins - 1);
            if (WIDE) {
                slot[k] = atomicAdd(&s_bin[d], 1u);
            } else {
                const uint32_t sh = 16 * (d & 1);
                slot[k] = (atomicAdd(&s_bin[d >> 1], 1u << sh) >> sh) & 0xffffu;
            }
        }
    }
    __syncthreads();
    // Bin counts -> bin starts (exclusive scan, in place), and the largest bin.  Every
    // counter word is scanned, each thread taking PERW adjacent ones (vector LDS
    // accesses); words past nbins hold 0 and so take the start len.
    {
        constexpr int NW0 = WIDE ? (1 << DB) : (1 << DB) / 2;
        constexpr int PERW = NW0 / THREADS;
        static_assert(NW0 % THREADS == 0, "whole counter words per thread");
        uint32_t v[PERW];
#pragma unroll
        for (int j = 0; j < PERW; ++j) v[j] = s_bin[tid * PERW + j];
        uint32_t sum = 0, mx = 0;
#pragma unroll
        for (int j = 0; j < PERW; ++j) {
            const uint32_t c0 = WIDE ? v[j] : v[j] & 0xffffu, c1 = WIDE ? 0u : v[j] >> 16;
            sum += c0 + c1;
            mx = c0 > mx ? c0 : mx;
            mx = c1 > mx ? c1 : mx;
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t y = __shfl_xor(mx, o, 64);
            mx = y > mx ? y : mx;
        }
        if (lane == 63) s_part[w] = incl;
        if (lane == 0) s_max[w] = mx;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int ww = 0; ww < w; ++ww) run += s_part[ww];
#pragma unroll
        for (int j = 0; j < PERW; ++j) {
            if (WIDE) {
                s_bin[tid * PERW + j] = run;
                run += v[j];
            } else {
                const uint32_t c0 = v[j] & 0xffffu, c1 = v[j] >> 16;
                s_bin[tid * PERW + j] = run | ((run + c0) << 16);
                run += c0 + c1;
            }
        }
    }
    uint32_t gmax = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) gmax = s_max[ww] > gmax ? s_max[ww] : gmax;
    if (gmax > GMAX) return false;  // a big group of near-equal keys
    __syncthreads();
    // Each bin's start (a word, or a 16-bit half of the packed counters); entry nbins
    // holds len, so every bin's end is its successor's start.
    const uint16_t* s_start16 = (const uint16_t*)s_bin;
    auto bin_start = [&](uint32_t d) -> uint32_t { return WIDE ? s_bin[d] : (uint32_t)s_start16[d]; };
    if (tid == 0) {
        if (WIDE) s_bin[nbins] = len;
        else ((uint16_t*)s_bin)[nbins] = (uint16_t)len;
    }
#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
        const uint32_t idx = (uint32_t)k * THREADS + tid;
        if (item_valid(k, nfull, rem, tid)) {
            const uint32_t d = (uint32_t)(xw[k] >> dshift) & (nbins - 1);
            const uint32_t q = bin_start(d) + slot[k];
            if (q < CAP) {
                s_w[q] = xw[k];
                if (SEPPOS) s_pos[q] = (uint16_t)idx;
            }
        }
    }
    // Past the last word, RANK_WIN words above every word (ties lose on the position).
    if (tid < RANK_WIN) {
        s_w[len + tid] = ~WT(0);
        if (SEPPOS) s_pos[len + tid] = 0xffffu;
    }
    __syncthreads();
    // Rank inside the bin (its start plus the smaller words in it) and rebuild the
    // key; then the values are loaded (coalesced), and with every word ranked the
    // word buffer holds them by input position, so each is gathered from LDS by the
    // position its word carries.  All reads of the input happen before the barrier
    // that precedes the writes, since the output may be the input buffer itself.
    uint32_t pos[MAXI];  // destination in the low 16 bits, source above
    K ko[MAXI];
    // Bits in [h, lo) are the chunk's constant ones; bits >= lo are the bucket's.
    const K lowmask = lo >= KBITS ? ~K(0) : (K)((K(1) << lo) - K(1));
    const K mid0 = key0 & lowmask & ~mask_h;
    const K hi0 = key0 & ~mask_h;
    const K d0 = lo >= KBITS ? K(0) : (K)(key0 >> lo);
#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
        const uint32_t p = (uint32_t)k * THREADS + tid;
        pos[k] = 0xffffffffu;
        ko[k] = 0;
        if (item_valid(k, nfull, rem, tid)) {
            const WT me = s_w[p];
            const uint32_t d = (uint32_t)(me >> dshift) & (nbins - 1);
            const uint32_t gs = bin_start(d);
            const uint32_t ge = bin_start(d + 1);
            // The first RANK_WIN places from the bin's start are compared without a
            // bound: places past the bin hold larger words (later bins, or the
            // sentinels past the chunk), which add nothing.
            uint32_t r = 0, src;
            if (SEPPOS) {
                // Smaller words first; another word equal to this one (equal sort bits,
                // rare) sends the lane through the bin once more to break the tie by
                // input position.
                src = s_pos[p];
                bool tie = false;
#pragma unroll
                for (int i = 0; i < RANK_WIN; ++i) {
                    const WT o = s_w[gs + i];
                    r += o < me;
                    tie |= (o == me) & (gs + i != p);
                }
                for (uint32_t q = gs + RANK_WIN; q < ge; ++q) {
                    const WT o = s_w[q];
                    r += o < me;
                    tie |= (o == me) & (q != p);
                }
                if (tie)
                    for (uint32_t q = gs; q < ge; ++q) r += (s_w[q] == me) & (s_pos[q] < src);
            } else {
#pragma unroll
                for (int i = 0; i < RANK_WIN; ++i) r += s_w[gs + i] < me;
                for (uint32_t q = gs + RANK_WIN; q < ge; ++q) r += s_w[q] < me;
                src = (uint32_t)me & ((1u << IB) - 1u);
            }
            const uint32_t at = gs + r < len ? gs + r : len - 1;
            const WT sw = me >> PB;  // the sort bits, the bucket index above them
            K hi = hi0;
            // Direct bucket indices: lo < KBITS, so the shift by lo is in range.
            if (direct) hi = mid0 | (K)(((K)((sw >> hsh) & bmask) + d0) << lo);
            else if (nbk > 1) hi = kin[at] & ~mask_h;
            pos[k] = at | (src << 16);
            ko[k] = ((K)sw & mask_h) | hi;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    V vx[MAXI];
    if (VB) {
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = (uint32_t)k * THREADS + tid;
            vx[k] = item_valid(k, nfull, rem, tid) ? vin[idx] : V(0);
        }
    }
    __syncthreads();  // every word ranked: the word buffer takes the values
    V* s_v = (V*)s_w;
    if (VB) {
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = (uint32_t)k * THREADS + tid;
            if (item_valid(k, nfull, rem, tid)) s_v[idx] = vx[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
        if (pos[k] != 0xffffffffu) {
            const uint32_t at = pos[k] & 0xffffu, src = (pos[k] >> 16) < len ? pos[k] >> 16 : 0;
            kout[at] = ko[k];
            if (VB) vout[at] = s_v[src];
        }
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------------
// Local sort, bucketed form (the common case).
//
// Each record becomes one 64-bit word: its sort bits (the h bits that vary below
// lo_bit, with the bucket index above them) in the high part and its position in the
// chunk in the low IB bits.  Words are then distinct, and ordering them orders the
// records by (sort bits, input position) -- the stable order -- so no step needs to
// be stable.  The words are bucket-sorted in LDS by their top bits (LDS atomics hand
// out slots; ~one word per bin on average), and each word's final place is its bin's
// start plus the number of smaller words in its bin: the rank formula applied inside
// the bin, the small-group comparison sort of the diversion (Sec. 3; insertion sort
// in the paper).  Values are gathered by the carried position.  A chunk whose sort
// bits do not fit next to the position, or whose largest bin exceeds GMAX records,
// goes to the spill list for the stable radix kernel below.
// ---------------------------------------------------------------------------------
// FORM 0: 32-bit words with the position inside; 1: 32-bit words, position beside them;
// 2: 64-bit words with the position inside.  Forms 0 and 1 hand chunks that do not fit
// to the 64-bit form's list.
template <int KB, int VB, int THREADS, int CAP, int FORM>
__global__ __launch_bounds__(THREADS, FORM == 0 ? LOCAL_MIN_WAVES_FORM0 : LOCAL_MIN_WAVES) void k_local_sort_bucket(LocalArgs a) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    constexpr int W = THREADS / 64;
    constexpr int MAXI = CAP / THREADS;
    constexpr int KBITS = 8 * KB;
    constexpr int IB = CAP <= 4096 ? 12 : CAP <= 8192 ? 13 : 16;  // bits of a position
    constexpr int DB = IB - 1;  // most bin bits
    // Bin counters: 32-bit words where the LDS allows (32-bit words and records of at
    // most 8 bytes), else two 16-bit counters per word; one entry more for the end.
    constexpr bool WIDE = FORM == 0 && KB + VB <= 8;
    constexpr int NWORDS = (WIDE ? (1 << DB) : (1 << DB) / 2) + 1;
    static_assert(CAP % THREADS == 0 && CAP <= (1 << IB), "chunk layout");
    static_assert(CAP < (1 << 16), "a destination and a source share one 32-bit word");
    static_assert(VB <= 8, "values fit the word buffer");
    // Words, then (once ranked) values, share one buffer sized for the wider of the two.
    constexpr int WB = FORM < 2 ? 4 : 8;  // word bytes
    using SW = typename uint_of<(WB > VB ? WB : (VB > 4 ? 8 : 4))>::type;
    __shared__ SW s_w[CAP + LOCAL_RANK_WIN];
    __shared__ uint16_t s_pos[FORM == 1 ? CAP + LOCAL_RANK_WIN : 1];
    __shared__ __align__(16) uint32_t s_bin[NWORDS];
    __shared__ uint32_t s_part[W];
    __shared__ uint32_t s_max[W];
    __shared__ K s_red[W];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nitems = *a.nchunks < a.chunkcap ? *a.nchunks : a.chunkcap;
    const uint64_t nb = umin64(*a.nbuckets, a.bcap);
    uint32_t* s_rel = (uint32_t*)s_w;
    uint32_t sorted = 0;  // chunks this block finished (counted by thread 0)

    // Hand chunk `it` on to another list (its descriptor is read again there, so
    // nothing of it stays live across the sort).
    auto hand_on = [&](uint32_t it, ChunkDesc* list, uint32_t* count, uint32_t cap) {
        if (tid == 0) {
            const uint32_t m = atomicAdd(count, 1u);
            if (m < cap) list[m] = a.chunks[it];
            else atomicOr(a.err, ERR_LIST_CAP);
        }
        __syncthreads();
    };
    auto spill = [&](uint32_t it) { hand_on(it, a.spill, a.nspill, a.spillcap); };

    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        Chunk ch;
        if (FORM == 0) {
            // Form 0 decodes its work items itself (the pre-pass has reported bad ones):
            // at eight waves per SIMD its registers are full, and the decode leaves fewer
            // values live across the sort than a descriptor does.
            if (!decode_chunk(a, a.work[it], nb, LOCAL_CAP_ANY, ch, false)) continue;
        } else {
            ch = a.chunks[it];
            if (ch.len == 0) continue;
        }
        if (ch.len > CAP) {  // larger than this kernel's tile: the general kernel sorts it
            spill(it);
            continue;
        }
        const uint64_t start = ch.start;
        const uint32_t len = ch.len, nbk = ch.nbk;
        const int lo = ch.lo;
        const K* kin = (const K*)a.kin + start;
        const V* vin = (const V*)a.vin + start;
        K* kout = (K*)a.kout + start;
        V* vout = (V*)a.vout + start;
        const uint32_t nfull = len / THREADS, rem = len % THREADS;

        Keys<K, MAXI> xs;
        K* x = xs.v;
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = (uint32_t)k * THREADS + tid;
            x[k] = item_valid(k, nfull, rem, tid) ? kin[idx] : K(0);
        }
        for (int i = tid; i < NWORDS; i += THREADS) s_bin[i] = 0;
        const K lowmask = lo >= KBITS ? ~K(0) : (K)((K(1) << lo) - K(1));
        const K key0 = kin[0];
        K vary = 0;
#pragma unroll
        for (int k = 0; k < MAXI; ++k)
            if (item_valid(k, nfull, rem, tid)) vary |= (x[k] ^ key0) & lowmask;
        vary = wave_or(vary);
        if (lane == 0) s_red[w] = vary;
        __syncthreads();
        K all = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) all |= s_red[ww];
        int h = 0;
        while (h < KBITS && (all >> h) != 0) ++h;
        const int bb = nbk > 1 ? 32 - __clz(nbk - 1) : 0;
        const int B = h > 0 ? h + bb : 0;
        if (B + IB > 64) {
            spill(it);
            continue;
        }
        if (FORM < 2 && B + (FORM == 0 ? IB : 0) > 32) {  // the 64-bit form sorts it
            hand_on(it, a.wide, a.nwide, a.widecap);
            continue;
        }
        if (B == 0) {  // nothing varies: the chunk is in order already
#pragma unroll
            for (int k = 0; k < MAXI; ++k) {
                const uint32_t idx = (uint32_t)k * THREADS + tid;
                if (item_valid(k, nfull, rem, tid)) {
                    kout[idx] = x[k];
                    if (VB) vout[idx] = vin[idx];
                }
            }
            __syncthreads();
            ++sorted;
            continue;
        }
        // Bucket index from the key itself: the buckets' bits >= lo, less the first
        // bucket's.  Exact while the chunk's buckets span few more values than there
        // are buckets (dense digits); otherwise it is found from the bucket starts.
        bool direct = false;
        int Bw = B;
        if (nbk > 1 && lo < KBITS) {
            const uint64_t span = (uint64_t)((kin[len - 1] >> lo) - (key0 >> lo));
            const int sb = 64 - __clzll(span);
            const int Bd = h + sb;
            direct = sb <= bb + 1 && Bd + IB <= 64 && (FORM == 2 || Bd + (FORM == 0 ? IB : 0) <= 32);
            if (direct) Bw = Bd;
        }
        if (nbk > 1 && !direct) {
            for (uint32_t i = tid; i < nbk; i += THREADS) s_rel[i] = (uint32_t)(a.bstart[ch.f + i] - start);
            __syncthreads();
        }
        using WT = typename uint_of<WB>::type;
        const bool ok = bucket_sort_chunk<WT, FORM == 1, WIDE, KB, VB, THREADS, CAP, IB, DB, MAXI>(
            xs, len, nfull, rem, lane, w, tid, nbk, direct, lo, h, Bw, key0, kin, vin, kout, vout, s_rel,
            (WT*)s_w, s_pos, s_bin, s_part, s_max);
        if (!ok) spill(it);
        else ++sorted;
    }
    if (tid == 0 && sorted && a.stat) atomicAdd(&a.stat[STAT_FORM0 + FORM], sorted);
}

// ---------------------------------------------------------------------------------
// Local sort (the diversion of Sec. 3): one chunk of at most CAP records per step of
// a block-stride loop.  A chunk is a run of consecutive buckets of one segment (or one
// medium bucket).  Sorting the chunk stably by the pair (bucket index, bits below
// lo_bit) sorts each bucket stably by its full key and keeps the buckets in order.
// Only the bits that vary in the chunk are sorted on (pass skipping at bit
// granularity, Sec. 2.1), in LSD passes of at most 8 bits inside LDS.
//
// The pair is packed into the key word itself: the h varying low bits stay, and the
// bucket index goes right above them.  It fits, because distinct buckets differ in
// their bits >= lo_bit, so there are at most 2^(KBITS - lo_bit) of them and h <= lo_bit.
// On the way out the bits >= h are restored from the input record at the same
// position: it belongs to the same bucket (buckets keep their ranges), and bits in
// [h, lo_bit) do not vary in the chunk.
// ---------------------------------------------------------------------------------
template <int KB, int VB, int THREADS, int CAP>
__global__ __launch_bounds__(THREADS) void k_local_sort(LocalArgs a) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    constexpr int W = THREADS / 64;
    constexpr int MAXI = CAP / THREADS;
    constexpr int KBITS = 8 * KB;
    static_assert(CAP % THREADS == 0, "chunk layout");

    __shared__ K s_c[CAP];
    __shared__ V s_v[VB ? CAP : 1];
    __shared__ uint32_t s_wcnt[2][W * RADIX];  // per-wave digit counters, double-buffered
    __shared__ K s_red[W];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nitems = *a.nspill < a.spillcap ? *a.nspill : a.spillcap;
    uint32_t* s_rel = (uint32_t*)s_c;  // bucket starts, before records are staged

    uint32_t sorted = 0;  // chunks this block sorted (counted by thread 0)
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Chunk ch = a.spill[it];
        if (ch.len == 0) continue;
        if (ch.len > CAP) {  // larger than any local sort takes
            if (tid == 0) atomicOr(a.err, ERR_CHUNK);
            continue;
        }
        ++sorted;
        const uint64_t start = ch.start;
        const uint32_t len = ch.len;
        const uint32_t nbk = ch.nbk;
        const uint32_t f = ch.f;
        const int lo = ch.lo;
        const K* kin = (const K*)a.kin + start;
        const V* vin = (const V*)a.vin + start;
        const uint32_t iu = (len + THREADS - 1) / THREADS;  // items per thread in use
        const uint32_t wbase = (uint32_t)w * iu * 64;

        K key[MAXI];
        V val[MAXI];
        uint32_t rnk[MAXI];
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = wbase + k * 64 + lane;
            const bool ok = (uint32_t)k < iu && idx < len;
            key[k] = ok ? kin[idx] : K(0);
            val[k] = (VB && ok) ? vin[idx] : V(0);
            rnk[k] = 0;
        }
        for (int i = tid; i < W * RADIX; i += THREADS) s_wcnt[0][i] = 0;
        // Bits below lo_bit that vary within the chunk.
        const K lowmask = lo >= KBITS ? ~K(0) : (K)((K(1) << lo) - K(1));
        const K key0 = kin[0];
        K vary = 0;
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = wbase + k * 64 + lane;
            if ((uint32_t)k < iu && idx < len) vary |= (key[k] ^ key0) & lowmask;
        }
        vary = wave_or(vary);
        if (lane == 0) s_red[w] = vary;
        __syncthreads();
        K all = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) all |= s_red[ww];
        int h = 0;
        while (h < KBITS && (all >> h) != 0) ++h;  // bit width of `all`
        const int bb = nbk > 1 ? 32 - __clz(nbk - 1) : 0;
        const int B = h > 0 ? h + bb : 0;
        if (B > KBITS) {  // cannot happen for buckets told apart by their prefixes
            if (tid == 0) atomicOr(a.err, ERR_CHUNK);
            __syncthreads();
            continue;
        }
        const K mask_h = h >= KBITS ? ~K(0) : (K)((K(1) << h) - K(1));
        if (B > 0) {
            if (nbk > 1) {
                for (uint32_t i = tid; i < nbk; i += THREADS)
                    s_rel[i] = (uint32_t)(a.bstart[f + i] - start);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < MAXI; ++k) {
                    const uint32_t idx = wbase + k * 64 + lane;
                    uint32_t lo_i = 0, hi_i = nbk;  // last i with s_rel[i] <= idx
                    while (hi_i - lo_i > 1) {
                        const uint32_t mid = (lo_i + hi_i) >> 1;
                        if (s_rel[mid] <= idx) lo_i = mid;
                        else hi_i = mid;
                    }
                    key[k] = (key[k] & mask_h) | ((K)lo_i << h);
                }
                __syncthreads();
            } else {
#pragma unroll
                for (int k = 0; k < MAXI; ++k) key[k] &= mask_h;
            }
        }
        const int npass = (B + RADIX_BITS - 1) / RADIX_BITS;
        const int wd = npass ? (B + npass - 1) / npass : 0;

        for (int p = 0; p < npass; ++p) {
            const int plo = p * wd;
            const int pw = wd < B - plo ? wd : B - plo;
            const uint32_t pmask = (1u << pw) - 1u;
            uint32_t* cnt = s_wcnt[p & 1];
            uint32_t* wc = cnt + w * RADIX;
            // Rank: stable position of each record among equal digits in its wave.
#pragma unroll
            for (int k = 0; k < MAXI; ++k) {
                if ((uint32_t)k < iu) {
                    const uint32_t idx = wbase + k * 64 + lane;
                    const bool ok = idx < len;
                    const uint64_t act = __ballot(ok);
                    const uint32_t d = (uint32_t)(key[k] >> plo) & pmask;
                    const uint64_t m = same_digit_lanes_rt(d, act, pw);
                    const uint32_t below = lanes_below(m);
                    const uint32_t base = wc[d];
                    if (ok && below == 0) wc[d] = base + (uint32_t)__popcll(m);
                    rnk[k] = base + below;
                }
                __builtin_amdgcn_sched_barrier(0);  // one item at a time: bounded registers
            }
            __syncthreads();
            // Wave 0 turns the per-wave counts into block offsets, digit-major then wave
            // order; the other waves clear the counters of the next pass meanwhile.
            if (w == 0) {
                uint32_t tot[RADIX / 64];
                uint32_t sum = 0;
#pragma unroll
                for (int q = 0; q < RADIX / 64; ++q) {
                    uint32_t t = 0;
#pragma unroll
                    for (int ww = 0; ww < W; ++ww) t += cnt[ww * RADIX + lane * (RADIX / 64) + q];
                    tot[q] = t;
                    sum += t;
                }
                uint32_t incl = sum;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += y;
                }
                uint32_t run = incl - sum;
#pragma unroll
                for (int q = 0; q < RADIX / 64; ++q) {
                    const int v = lane * (RADIX / 64) + q;
#pragma unroll
                    for (int ww = 0; ww < W; ++ww) {
                        const uint32_t c = cnt[ww * RADIX + v];
                        cnt[ww * RADIX + v] = run;
                        run += c;
                    }
                }
            } else if (p + 1 < npass) {
                uint32_t* nxt = s_wcnt[(p + 1) & 1];
                for (int i = tid - 64; i < W * RADIX; i += THREADS - 64) nxt[i] = 0;
            }
            __syncthreads();
            // Stage in LDS in digit order.
#pragma unroll
            for (int k = 0; k < MAXI; ++k) {
                const uint32_t idx = wbase + k * 64 + lane;
                if ((uint32_t)k < iu && idx < len) {
                    const uint32_t d = (uint32_t)(key[k] >> plo) & pmask;
                    const uint32_t q = wc[d] + rnk[k];
                    if (q < CAP) {
                        s_c[q] = key[k];
                        if (VB) s_v[q] = val[k];
                    }
                }
            }
            __syncthreads();
            if (p + 1 < npass) {
#pragma unroll
                for (int k = 0; k < MAXI; ++k) {
                    const uint32_t idx = wbase + k * 64 + lane;
                    if ((uint32_t)k < iu && idx < len) {
                        key[k] = s_c[idx];
                        if (VB) val[k] = s_v[idx];
                    }
                }
            }
        }

        K* kout = (K*)a.kout + start;
        V* vout = (V*)a.vout + start;
        const K hi0 = key0 & ~mask_h;
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
            const uint32_t idx = wbase + k * 64 + lane;
            if ((uint32_t)k < iu && idx < len) {
                if (npass > 0) {
                    const K hi = nbk > 1 ? (kin[idx] & ~mask_h) : hi0;
                    kout[idx] = (s_c[idx] & mask_h) | hi;
                    if (VB) vout[idx] = s_v[idx];
                } else {
                    kout[idx] = key[k];
                    if (VB) vout[idx] = val[k];
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sorted && a.stat) atomicAdd(&a.stat[STAT_GENERAL], sorted);
}

// ---------------------------------------------------------------------------------
// Copy of whole tiles (finished ranges back into the caller's buffers).
// ---------------------------------------------------------------------------------
template <int KB, int VB, int THREADS>
__global__ __launch_bounds__(THREADS) void k_copy_tiles(const void* kin, const void* vin,
                                                        void* kout, void* vout,
                                                        const Tile* tiles, uint32_t ntiles) {
    using K = typename uint_of<KB>::type;
    using V = typename uint_of<VB>::type;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const K* ki = (const K*)kin + tl.start;
        K* ko = (K*)kout + tl.start;
        for (uint32_t i = threadIdx.x; i < tl.len; i += THREADS) ko[i] = ki[i];
        if (VB) {
            const V* vi = (const V*)vin + tl.start;
            V* vo = (V*)vout + tl.start;
            for (uint32_t i = threadIdx.x; i < tl.len; i += THREADS) vo[i] = vi[i];
        }
    }
}

// Copy of runs between arbitrary addresses (gathering requests into one batch and
// scattering the sorted batch back).  Runs are whole 4-byte words; where source and
// destination are both 16-byte aligned the body moves as 16-byte vectors, four loads in
// flight per thread before their stores.
typedef unsigned int copy4u __attribute__((ext_vector_type(4)));
template <int THREADS>
__device__ __forceinline__ void copy_run(const void* src, void* dst, uint64_t bytes) {
    const uint32_t tid = threadIdx.x;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) {
        const copy4u* s4 = (const copy4u*)src;
        copy4u* d4 = (copy4u*)dst;
        const uint64_t nvec = bytes >> 4;
        for (uint64_t i = tid; i < nvec; i += 4 * THREADS) {
            copy4u r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = i + u * THREADS < nvec ? s4[i + u * THREADS] : (copy4u)(0u);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + u * THREADS < nvec) d4[i + u * THREADS] = r[u];
        }
        const uint64_t done = nvec << 4;
        const uint32_t* sw = (const uint32_t*)((const char*)src + done);
        uint32_t* dw = (uint32_t*)((char*)dst + done);
        for (uint64_t i = tid; i < ((bytes - done) >> 2); i += THREADS) dw[i] = sw[i];
    } else {
        const uint32_t* sw = (const uint32_t*)src;
        uint32_t* dw = (uint32_t*)dst;
        const uint64_t nw = bytes >> 2;
        for (uint64_t i = tid; i < nw; i += 4 * THREADS) {
            uint32_t r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = i + u * THREADS < nw ? sw[i + u * THREADS] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + u * THREADS < nw) dw[i + u * THREADS] = r[u];
        }
    }
}

template <int KB, int VB, int THREADS>
__global__ __launch_bounds__(THREADS) void k_copy_chunks(const CopyChunk* chunks, uint32_t nchunks) {
    for (uint32_t t = blockIdx.x; t < nchunks; t += gridDim.x) {
        const CopyChunk ch = chunks[t];
        copy_run<THREADS>(ch.ksrc, ch.kdst, (uint64_t)ch.len * KB);
        if (VB) copy_run<THREADS>(ch.vsrc, ch.vdst, (uint64_t)ch.len * VB);
    }
}

// Streaming copy of 16-byte vectors, the bandwidth reference for the passes above (each
// of which reads and writes every record once).  Each block copies one contiguous run of
// STREAM_THREADS * STREAM_U vectors: all its loads issue before its stores, consecutive
// lanes touch consecutive vectors, and the lines are streamed past the caches
// (non-temporal), since nothing reads them again.
constexpr int STREAM_THREADS = 256, STREAM_U = 4;
typedef unsigned int vec4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_copy(const vec4u* __restrict__ src,
                                                                vec4u* __restrict__ dst, uint64_t nvec) {
    const uint64_t i0 = (uint64_t)blockIdx.x * STREAM_THREADS * STREAM_U + threadIdx.x;
    vec4u r[STREAM_U];
#pragma unroll
    for (int u = 0; u < STREAM_U; ++u) {
        const uint64_t i = i0 + (uint64_t)u * STREAM_THREADS;
        r[u] = i < nvec ? __builtin_nontemporal_load(src + i) : (vec4u)(0u);
    }
#pragma unroll
    for (int u = 0; u < STREAM_U; ++u) {
        const uint64_t i = i0 + (uint64_t)u * STREAM_THREADS;
        if (i < nvec) __builtin_nontemporal_store(r[u], dst + i);
    }
}

// Streaming read of 16-byte vectors, the bandwidth reference of the counts (which read
// every key once and write little): each block reads one contiguous run of
// STREAM_THREADS * STREAM_RU vectors, all its loads in flight together, and writes the
// XOR of its words to part[block]; one block then folds the parts into *out.  The result
// is the XOR of every 32-bit word read: a checksum that keeps the loads live and can be
// checked, at no more than one word written per 32 KB read.
constexpr int STREAM_RU = 8;
constexpr uint64_t STREAM_RUN = (uint64_t)STREAM_THREADS * STREAM_RU;  // vectors per block
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_read(const vec4u* __restrict__ src, uint64_t nvec,
                                                                uint32_t* __restrict__ part) {
    __shared__ uint32_t s_x[STREAM_THREADS / 64];
    const uint64_t i0 = (uint64_t)blockIdx.x * STREAM_RUN + threadIdx.x;
    vec4u r[STREAM_RU];
#pragma unroll
    for (int u = 0; u < STREAM_RU; ++u) {
        const uint64_t i = i0 + (uint64_t)u * STREAM_THREADS;
        r[u] = i < nvec ? src[i] : (vec4u)(0u);
    }
    uint32_t x = 0;
#pragma unroll
    for (int u = 0; u < STREAM_RU; ++u) x ^= r[u].x ^ r[u].y ^ r[u].z ^ r[u].w;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) s_x[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
#pragma unroll
        for (int w = 0; w < STREAM_THREADS / 64; ++w) b ^= s_x[w];
        part[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(1024) void k_xor_fold(const uint32_t* __restrict__ part, uint64_t n,
                                                   uint32_t* out) {
    __shared__ uint32_t s_x[16];
    uint32_t x = 0;
    // Sixteen independent loads in flight per thread and step.
    for (uint64_t i0 = threadIdx.x; i0 < n; i0 += 16 * 1024) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint64_t i = i0 + (uint64_t)u * 1024;
            v[u] = i < n ? part[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) x ^= v[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) s_x[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) b ^= s_x[w];
        *out = b;
    }
}

uint64_t stream_read_parts(uint64_t bytes) { return (bytes / 16 + STREAM_RUN - 1) / STREAM_RUN; }

hipError_t launch_stream_read(const void* src, uint64_t bytes, uint32_t* part, uint32_t* out, hipStream_t s) {
    const uint64_t nvec = bytes / 16, parts = stream_read_parts(bytes);
    if (parts > 0x7fffffffu) return hipErrorInvalidValue;
    if (parts)
        hipLaunchKernelGGL(k_stream_read, dim3((uint32_t)parts), dim3(STREAM_THREADS), 0, s,
                           (const vec4u*)src, nvec, part);
    hipLaunchKernelGGL(k_xor_fold, dim3(1), dim3(1024), 0, s, part, parts, out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
    const uint64_t nvec = bytes / 16;
    if (nvec == 0) return hipSuccess;
    const uint64_t per_block = (uint64_t)STREAM_THREADS * STREAM_U;
    const uint64_t blocks = (nvec + per_block - 1) / per_block;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)blocks), dim3(STREAM_THREADS), 0, s,
                       (const vec4u*)src, (vec4u*)dst, nvec);
    return hipGetLastError();
}

// Order-preserving maps from signed and floating-point encodings to unsigned integers
// (the paper sorts unsigned keys only).  Signed: flip the sign bit, so that negative
// values come first in two's-complement order.  Float: flip every bit of a negative
// value (larger magnitude first) and the sign bit of a positive one, which orders the
// encodings by IEEE 754 totalOrder.  `inverse` maps back.
template <int KB>
__global__ __launch_bounds__(256) void k_key_transform(void* keys, uint64_t n, int mode, int inverse) {
    using K = typename uint_of<KB>::type;
    constexpr K SIGN = K(1) << (8 * KB - 1);
    K* k = (K*)keys;
    const uint64_t stride = (uint64_t)gridDim.x * 256 * 4;
    for (uint64_t i0 = (uint64_t)blockIdx.x * 256 * 4 + threadIdx.x; i0 < n; i0 += stride) {
        K x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = i0 + u * 256 < n ? k[i0 + u * 256] : K(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (mode == 1) {
                x[u] ^= SIGN;
            } else {
                const bool top = (x[u] & SIGN) != 0;
                x[u] ^= (top != (inverse != 0)) ? ~K(0) : SIGN;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * 256 < n) k[i0 + u * 256] = x[u];
    }
}

// ---------------------------------------------------------------------------------
// Tile shapes and launchers.
// ---------------------------------------------------------------------------------
static_assert(DEAL_TILE_SMALL % DEAL_THREADS == 0 && DEAL_TILE_LARGE % DEAL_THREADS == 0, "tile");
static_assert(DEAL_TILE_SMALL >= DEAL_TILE_LARGE, "head kernel covers the larger tile");

uint32_t deal_tile_records(int kb, int vb) {
    return kb + vb <= 8 ? (uint32_t)DEAL_TILE_SMALL : (uint32_t)DEAL_TILE_LARGE;
}
bool deal_tile_supported(int kb, int vb, uint32_t tile) {
    const uint32_t t = deal_tile_records(kb, vb);
    return tile == t || tile == t / 2;
}
uint32_t local_sort_capacity(int kb, int vb) {
    return kb + vb <= 8 ? (uint32_t)LOCAL_CAP_SMALL : (uint32_t)LOCAL_CAP_LARGE;
}
uint32_t local_bucket_capacity(int kb, int vb) {
    return kb + vb <= 8 ? (uint32_t)BUCKET_CAP_SMALL : (uint32_t)BUCKET_CAP_LARGE;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_set(const FillSet& f, hipStream_t s) {
    uint64_t most = 0;
    for (int i = 0; i < f.count; ++i) most = std::max<uint64_t>(most, f.n[i]);
    if (f.count <= 0 || most == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((most + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_set, dim3(blocks, (uint32_t)f.count), dim3(256), 0, s, f);
    return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

template <int KB>
static void count_kb(const CountArgs& a, uint32_t blocks, hipStream_t s) {
    if (a.ndig <= 1)
        hipLaunchKernelGGL((k_count<KB, COUNT_THREADS, 1>), dim3(blocks), dim3(COUNT_THREADS), 0, s, a);
    else if (a.ndig <= 4)
        hipLaunchKernelGGL((k_count<KB, COUNT_THREADS, 4>), dim3(blocks), dim3(COUNT_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_count<KB, COUNT_THREADS, 8>), dim3(blocks), dim3(COUNT_THREADS), 0, s, a);
}

hipError_t launch_count(int kb, const CountArgs& a, uint32_t blocks, hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    if (a.ndig < 1 || a.ndig > MAX_PASSES) return hipErrorInvalidValue;
    if (kb == 4) count_kb<4>(a, blocks, s);
    else count_kb<8>(a, blocks, s);
    return hipGetLastError();
}

template <int KB, int VB, int ITEMS>
static void deal_items(const DealArgs& a, hipStream_t s) {
    if (a.off)
        hipLaunchKernelGGL((k_deal<KB, VB, DEAL_THREADS, ITEMS, false>), dim3(a.ntiles),
                           dim3(DEAL_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_deal<KB, VB, DEAL_THREADS, ITEMS, true>), dim3(a.ntiles),
                           dim3(DEAL_THREADS), 0, s, a);
}

// Two tile sizes per record size: the default and half of it.
template <int KB, int VB>
static bool deal_kb_vb(const DealArgs& a, hipStream_t s) {
    constexpr int ITEMS = (KB + VB <= 8 ? DEAL_TILE_SMALL : DEAL_TILE_LARGE) / DEAL_THREADS;
    static_assert(ITEMS % 2 == 0, "half tile");
    if (a.tile == (uint32_t)(ITEMS * DEAL_THREADS)) deal_items<KB, VB, ITEMS>(a, s);
    else if (a.tile == (uint32_t)(ITEMS / 2 * DEAL_THREADS)) deal_items<KB, VB, ITEMS / 2>(a, s);
    else return false;
    return true;
}

// ---------------------------------------------------------------------------------
// Per-tile bucket bases for one segment (reduce-then-scan): (a) each block of tiles
// sums its tiles' counts per digit; (b) one block scans those sums over blocks, and
// adds each digit's bucket start (exclusive scan of the digit totals); (c) each block
// walks its tiles in order, writing every tile's bases.
// ---------------------------------------------------------------------------------
constexpr int SCAN_BATCH = 16;  // independent loads in flight per thread

__global__ __launch_bounds__(RADIX) void k_tile_scan_a(TileScanArgs a) {
    const uint32_t b = blockIdx.x, v = threadIdx.x;
    const uint32_t t0 = b * a.tiles_per_block;
    const uint32_t t1 = a.ntiles - t0 < a.tiles_per_block ? a.ntiles : t0 + a.tiles_per_block;
    uint32_t sum = 0;
    for (uint32_t tb = t0; tb < t1; tb += SCAN_BATCH) {
        uint32_t c[SCAN_BATCH];
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i)
            c[i] = tb + i < t1 ? a.cnt[((size_t)(tb + i) * a.ndig + a.slot) * RADIX + v] : 0u;
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) sum += c[i];
    }
    a.partial[(size_t)b * RADIX + v] = sum;
}

// One block of 4 * RADIX threads: thread (q, v) scans part q of the block sums of
// digit v; the parts are then chained, and the digit totals turned into bucket starts.
__global__ __launch_bounds__(4 * RADIX) void k_tile_scan_b(TileScanArgs a) {
    __shared__ uint32_t s_q[4][RADIX];
    __shared__ uint32_t s_part[RADIX / 64];
    const uint32_t v = threadIdx.x % RADIX, q = threadIdx.x / RADIX;
    if (a.ticket && threadIdx.x == 0) *a.ticket = 0;
    const uint32_t per = (a.nblocks + 3) / 4;
    const uint32_t b0 = q * per, b1 = b0 + per < a.nblocks ? b0 + per : a.nblocks;
    uint32_t run = 0;
    for (uint32_t bb = b0; bb < b1; bb += SCAN_BATCH) {
        uint32_t c[SCAN_BATCH];
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) c[i] = bb + i < b1 ? a.partial[(size_t)(bb + i) * RADIX + v] : 0u;
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) {
            if (bb + i < b1) a.partial[(size_t)(bb + i) * RADIX + v] = run;
            run += c[i];
        }
    }
    s_q[q][v] = run;
    __syncthreads();
    uint32_t before = 0, total_v = 0;
    for (uint32_t i = 0; i < 4; ++i) {
        before += i < q ? s_q[i][v] : 0u;
        total_v += s_q[i][v];
    }
    uint32_t all;
    const uint32_t start = scan256_excl(threadIdx.x < RADIX ? total_v : 0u, s_part, &all);
    __shared__ uint32_t s_start[RADIX];
    if (threadIdx.x < RADIX) s_start[v] = start;
    __syncthreads();
    const uint32_t add = s_start[v] + before;
    for (uint32_t bb = b0; bb < b1; ++bb) a.partial[(size_t)bb * RADIX + v] += add;
}

__global__ __launch_bounds__(RADIX) void k_tile_scan_c(TileScanArgs a) {
    const uint32_t b = blockIdx.x, v = threadIdx.x;
    const uint32_t t0 = b * a.tiles_per_block;
    const uint32_t t1 = a.ntiles - t0 < a.tiles_per_block ? a.ntiles : t0 + a.tiles_per_block;
    uint32_t run = a.partial[(size_t)b * RADIX + v];
    for (uint32_t tb = t0; tb < t1; tb += SCAN_BATCH) {
        uint32_t c[SCAN_BATCH];
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i)
            c[i] = tb + i < t1 ? a.cnt[((size_t)(tb + i) * a.ndig + a.slot) * RADIX + v] : 0u;
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) {
            if (tb + i < t1) a.off[(size_t)(tb + i) * RADIX + v] = run;
            run += c[i];
        }
    }
}

// G groups of RADIX threads split the segment's tiles: each sums its share per digit,
// the shares are chained after the digit's bucket start, and each group writes its
// tiles' bases (few segments: G = 4, so the serial walks are a quarter as long).
template <int G>
__global__ __launch_bounds__(RADIX * G) void k_seg_scan(SegScanArgs a) {
    __shared__ uint32_t s_part[RADIX / 64];
    __shared__ uint32_t s_gsum[G][RADIX];
    __shared__ uint32_t s_start[RADIX];
    const uint32_t s = blockIdx.x, v = threadIdx.x % RADIX, g = threadIdx.x / RADIX;
    if (a.ticket && s == 0 && threadIdx.x == 0) *a.ticket = 0;
    const Seg* sg = a.segs + s;
    const uint64_t len = sg->len;
    if (len == 0 || a.pass < sg->first_pass) return;  // no tiles in this pass (whole block)
    const int slot = sg->hslot[a.pass];
    const uint32_t nt = (uint32_t)((len + a.tile - 1) / a.tile);
    const uint32_t per = (nt + G - 1) / G;
    const uint32_t t0 = g * per < nt ? g * per : nt, t1 = t0 + per < nt ? t0 + per : nt;
    const uint32_t ct = a.cnt_from_count_tiles ? sg->count_tile : sg->first_tile;
    const int cslot = a.cnt_from_count_tiles ? slot : 0;
    auto cnt_at = [&](uint32_t i) { return a.cnt[((size_t)(ct + i) * a.cnt_ndig + cslot) * RADIX + v]; };
    uint32_t sum = 0;
    if (G > 1) {
        for (uint32_t i0 = t0; i0 < t1; i0 += SCAN_BATCH) {
            uint32_t c[SCAN_BATCH];
#pragma unroll
            for (int i = 0; i < SCAN_BATCH; ++i) c[i] = i0 + i < t1 ? cnt_at(i0 + i) : 0u;
#pragma unroll
            for (int i = 0; i < SCAN_BATCH; ++i) sum += c[i];
        }
        s_gsum[g][v] = sum;
    }
    uint32_t total;
    const uint32_t start =
        scan256_excl(g == 0 ? a.hist[((size_t)s * a.hist_digits + slot) * RADIX + v] : 0u, s_part, &total);
    if (g == 0) s_start[v] = start;
    __syncthreads();
    uint32_t run = s_start[v];
    for (uint32_t gg = 0; gg < g; ++gg) run += s_gsum[gg][v];
    for (uint32_t i0 = t0; i0 < t1; i0 += SCAN_BATCH) {
        uint32_t c[SCAN_BATCH];
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) c[i] = i0 + i < t1 ? cnt_at(i0 + i) : 0u;
#pragma unroll
        for (int i = 0; i < SCAN_BATCH; ++i) {
            if (i0 + i < t1) a.off[(size_t)(sg->first_tile + i0 + i) * RADIX + v] = run;
            run += c[i];
        }
    }
}

// Collision probability of each segment's digits (the chance that two records drawn
// at random share the digit), the input of the plan's bucket-size estimate (Sec. 3).
__global__ __launch_bounds__(RADIX) void k_collisions(const uint32_t* hist, int ndig, int bits,
                                                      double* coll, uint32_t* nonzero,
                                                      uint32_t* overflow) {
    __shared__ double s_sq[RADIX / 64], s_n[RADIX / 64];
    __shared__ uint32_t s_nz[RADIX / 64];
    __shared__ uint32_t s_len;
    __shared__ uint32_t s_ov[RADIX / 64];
    const uint32_t s = blockIdx.x, v = threadIdx.x, lane = v & 63, w = v >> 6;
    for (int j = 0; j < ndig; ++j) {
        const uint32_t hv = hist[((size_t)s * ndig + j) * RADIX + v];
        const double h = (double)hv;
        double sq = h * h, n = h;
        for (int o = 32; o > 0; o >>= 1) {
            sq += __shfl_xor(sq, o);
            n += __shfl_xor(n, o);
        }
        const uint32_t nz = (uint32_t)__popcll(__ballot(hv != 0));
        if (lane == 0) {
            s_sq[w] = sq;
            s_n[w] = n;
            s_nz[w] = nz;
        }
        __syncthreads();
        if (v == 0) {
            double tsq = 0, tn = 0;
            uint32_t tnz = 0;
            for (int i = 0; i < RADIX / 64; ++i) {
                tsq += s_sq[i];
                tn += s_n[i];
                tnz += s_nz[i];
            }
            coll[(size_t)s * ndig + j] = tn > 0 ? tsq / (tn * tn) : 0.0;
            nonzero[(size_t)s * ndig + j] = tnz;
            s_len = (uint32_t)tn;
        }
        __syncthreads();
        // Records that estimated buckets of ceil(len / 2^bits) slots would not hold
        // (Fast Radix, Sec. 3.1): the measured counterpart of Eq. 2.
        const uint32_t m = 1u << bits, cap = s_len / m + (s_len % m != 0);
        uint32_t ov = v < m && hv > cap ? hv - cap : 0u;
        for (int o = 32; o > 0; o >>= 1) ov += __shfl_xor(ov, o);
        if (lane == 0) s_ov[w] = ov;
        __syncthreads();
        if (v == 0) {
            uint32_t t = 0;
            for (int i = 0; i < RADIX / 64; ++i) t += s_ov[i];
            overflow[(size_t)s * ndig + j] = t;
        }
        __syncthreads();
    }
}

hipError_t launch_collisions(const uint32_t* hist, uint32_t nsegs, int ndig, int bits, double* coll,
                             uint32_t* nonzero, uint32_t* overflow, hipStream_t s) {
    if (nsegs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_collisions, dim3(nsegs), dim3(RADIX), 0, s, hist, ndig, bits, coll, nonzero,
                       overflow);
    return hipGetLastError();
}

hipError_t launch_seg_scan(const SegScanArgs& a, hipStream_t s) {
    if (a.nsegs == 0) return hipSuccess;
    if (a.nsegs <= 64) hipLaunchKernelGGL(k_seg_scan<4>, dim3(a.nsegs), dim3(4 * RADIX), 0, s, a);
    else hipLaunchKernelGGL(k_seg_scan<1>, dim3(a.nsegs), dim3(RADIX), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tile_scan(const TileScanArgs& a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_scan_a, dim3(a.nblocks), dim3(RADIX), 0, s, a);
    hipLaunchKernelGGL(k_tile_scan_b, dim3(1), dim3(4 * RADIX), 0, s, a);
    hipLaunchKernelGGL(k_tile_scan_c, dim3(a.nblocks), dim3(RADIX), 0, s, a);
    return hipGetLastError();
}

template <int KB, int VB>
static void deal_est_kb_vb(const EstArgs& a, hipStream_t s) {
    constexpr int ITEMS = (KB + VB <= 8 ? DEAL_TILE_SMALL : DEAL_TILE_LARGE) / DEAL_THREADS;
    hipLaunchKernelGGL((k_deal_est<KB, VB, DEAL_THREADS, ITEMS>), dim3(a.ntiles), dim3(DEAL_THREADS), 0, s, a);
}

hipError_t launch_deal_est(int kb, int vb, const EstArgs& a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    if (a.tile != deal_tile_records(kb, vb)) return hipErrorInvalidValue;
    if (kb == 4) {
        if (vb == 0) deal_est_kb_vb<4, 0>(a, s);
        else if (vb == 4) deal_est_kb_vb<4, 4>(a, s);
        else deal_est_kb_vb<4, 8>(a, s);
    } else {
        if (vb == 0) deal_est_kb_vb<8, 0>(a, s);
        else if (vb == 4) deal_est_kb_vb<8, 4>(a, s);
        else deal_est_kb_vb<8, 8>(a, s);
    }
    return hipGetLastError();
}

hipError_t launch_deal(int kb, int vb, const DealArgs& a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    bool ok;
    if (kb == 4) {
        if (vb == 0) ok = deal_kb_vb<4, 0>(a, s);
        else if (vb == 4) ok = deal_kb_vb<4, 4>(a, s);
        else ok = deal_kb_vb<4, 8>(a, s);
    } else {
        if (vb == 0) ok = deal_kb_vb<8, 0>(a, s);
        else if (vb == 4) ok = deal_kb_vb<8, 4>(a, s);
        else ok = deal_kb_vb<8, 8>(a, s);
    }
    if (!ok) return hipErrorInvalidValue;  // no kernel for this tile size
    return hipGetLastError();
}

template <int KB, int VB>
static void copy_chunks_kb_vb(const CopyChunk* c, uint32_t n, hipStream_t s) {
    const uint32_t blocks = n < 8192 ? n : 8192;
    hipLaunchKernelGGL((k_copy_chunks<KB, VB, COPY_THREADS>), dim3(blocks), dim3(COPY_THREADS), 0, s, c, n);
}

hipError_t launch_copy_chunks(int kb, int vb, const CopyChunk* chunks, uint32_t nchunks,
                              hipStream_t s) {
    if (nchunks == 0) return hipSuccess;
    if (kb == 4) {
        if (vb == 0) copy_chunks_kb_vb<4, 0>(chunks, nchunks, s);
        else if (vb == 4) copy_chunks_kb_vb<4, 4>(chunks, nchunks, s);
        else copy_chunks_kb_vb<4, 8>(chunks, nchunks, s);
    } else {
        if (vb == 0) copy_chunks_kb_vb<8, 0>(chunks, nchunks, s);
        else if (vb == 4) copy_chunks_kb_vb<8, 4>(chunks, nchunks, s);
        else copy_chunks_kb_vb<8, 8>(chunks, nchunks, s);
    }
    return hipGetLastError();
}

hipError_t launch_key_transform(int kb, int mode, bool inverse, void* keys, size_t n,
                                hipStream_t s) {
    if (n == 0 || mode == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + 1023) / 1024, 8192);
    if (kb == 4) hipLaunchKernelGGL(k_key_transform<4>, dim3(blocks), dim3(256), 0, s, keys, (uint64_t)n, mode, inverse ? 1 : 0);
    else hipLaunchKernelGGL(k_key_transform<8>, dim3(blocks), dim3(256), 0, s, keys, (uint64_t)n, mode, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_heads(int kb, const HeadArgs& a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    // Tiles are the deal tiles of the level; the head kernel's block covers the
    // largest of them (8192 records).
    constexpr int ITEMS = DEAL_TILE_SMALL / HEAD_THREADS;
    static_assert(DEAL_TILE_SMALL <= 65536, "tile-relative head positions are 16-bit");
    const uint32_t emit_blocks = std::min<uint32_t>((a.ntiles + 3) / 4, 4096);
    if (kb == 4) {
        hipLaunchKernelGGL((k_heads<4, HEAD_THREADS, ITEMS>), dim3(a.ntiles), dim3(HEAD_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_heads_scan, dim3(1), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_heads_emit<4>, dim3(emit_blocks), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_heads<8, HEAD_THREADS, ITEMS>), dim3(a.ntiles), dim3(HEAD_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_heads_scan, dim3(1), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_heads_emit<8>, dim3(emit_blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_hist_heads(const HistHeadArgs& a, hipStream_t s) {
    if (a.nids == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist_heads_count, dim3(a.nids), dim3(RADIX), 0, s, a);
    hipLaunchKernelGGL(k_hist_heads_scan, dim3(1), dim3(HIST_SCAN_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_hist_heads_emit, dim3(a.nids), dim3(RADIX), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_joint_heads(int kb, const JointArgs& a, hipStream_t s) {
    const uint32_t n0 = 1u << a.width0, n1 = 1u << a.width1;
    if (kb == 4)
        hipLaunchKernelGGL(k_joint_counts<4>, dim3(n0), dim3(JOINT_GROUPS * RADIX), 0, s, a);
    else
        hipLaunchKernelGGL(k_joint_counts<8>, dim3(n0), dim3(JOINT_GROUPS * RADIX), 0, s, a);
    hipLaunchKernelGGL(k_joint_rows, dim3(n1), dim3(RADIX), 0, s, a);
    hipLaunchKernelGGL(k_joint_emit, dim3(n1), dim3(RADIX), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_classify(const ClassifyArgs& a, uint32_t blocks, hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3(blocks), dim3(CLASSIFY_THREADS), 0, s, a);
    return hipGetLastError();
}

template <int KB, int VB>
static void local_kb_vb(const LocalArgs& a, uint32_t blocks, int first_form, hipStream_t s) {
    constexpr int CAP = KB + VB <= 8 ? LOCAL_CAP_SMALL : LOCAL_CAP_LARGE;
    constexpr int BCAP = KB + VB <= 8 ? BUCKET_CAP_SMALL : BUCKET_CAP_LARGE;
    // The work items' chunks are decoded first.  A 32-bit form (first_form 0 or 1) then
    // sorts them, handing chunks that need more to the 64-bit form; or the 64-bit form
    // sorts every chunk (first_form 2).  Chunks none of them can take go to the general
    // kernel.  Every list but the work list holds descriptors.
    const uint32_t dblocks = std::min<uint32_t>((a.workcap + 255) / 256, 1024);
    if (dblocks) hipLaunchKernelGGL(k_chunk_desc, dim3(dblocks), dim3(256), 0, s, a);
    LocalArgs la = a;
    la.chunks = a.desc;
    la.nchunks = a.nwork;
    la.chunkcap = a.workcap;
    uint32_t wblocks = blocks;
    if (first_form < 2) {
        if (first_form == 0)
            hipLaunchKernelGGL((k_local_sort_bucket<KB, VB, LOCAL_THREADS, BCAP, 0>), dim3(blocks),
                               dim3(LOCAL_THREADS), 0, s, la);
        else
            hipLaunchKernelGGL((k_local_sort_bucket<KB, VB, LOCAL_THREADS, BCAP, 1>), dim3(blocks),
                               dim3(LOCAL_THREADS), 0, s, la);
        la.chunks = a.wide;
        la.nchunks = a.nwide;
        la.chunkcap = a.widecap;
        wblocks = blocks < 4096 ? blocks : 4096;
    }
    hipLaunchKernelGGL((k_local_sort_bucket<KB, VB, LOCAL_THREADS, BCAP, 2>), dim3(wblocks),
                       dim3(LOCAL_THREADS), 0, s, la);
    const uint32_t gblocks = blocks < 2048 ? blocks : 2048;
    hipLaunchKernelGGL((k_local_sort<KB, VB, GENERAL_THREADS, CAP>), dim3(gblocks),
                       dim3(GENERAL_THREADS), 0, s, a);
}

int local_sort_first_form(int kb, int vb, int max_lo_bit, int index_bits) {
    // A chunk's sort bits are at most its lo_bit varying bits plus the bits of its
    // buckets' index (index_bits as the level expects them).  With room for the position
    // as well, the 32-bit words carry it (form 0); else, while the sort bits fit 32, the
    // position goes beside them (form 1).  Otherwise the first form would only read
    // each chunk to hand it on to the 64-bit form.
    const int pb = local_bucket_capacity(kb, vb) <= 4096 ? 12 : 13;
    if (max_lo_bit + index_bits + pb <= 32) return 0;
    return max_lo_bit < 32 && max_lo_bit + index_bits <= 32 ? 1 : 2;
}

hipError_t launch_local_sort(int kb, int vb, const LocalArgs& a, uint32_t blocks,
                             int first_form, hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    if (kb == 4) {
        if (vb == 0) local_kb_vb<4, 0>(a, blocks, first_form, s);
        else if (vb == 4) local_kb_vb<4, 4>(a, blocks, first_form, s);
        else local_kb_vb<4, 8>(a, blocks, first_form, s);
    } else {
        if (vb == 0) local_kb_vb<8, 0>(a, blocks, first_form, s);
        else if (vb == 4) local_kb_vb<8, 4>(a, blocks, first_form, s);
        else local_kb_vb<8, 8>(a, blocks, first_form, s);
    }
    return hipGetLastError();
}

template <int KB, int VB>
static void copy_kb_vb(const void* kin, const void* vin, void* kout, void* vout, const Tile* tiles,
                       uint32_t ntiles, hipStream_t s) {
    const uint32_t blocks = std::min(ntiles, 8192u);
    hipLaunchKernelGGL((k_copy_tiles<KB, VB, COPY_THREADS>), dim3(blocks), dim3(COPY_THREADS), 0, s,
                       kin, vin, kout, vout, tiles, ntiles);
}

hipError_t launch_copy_tiles(int kb, int vb, const void* kin, const void* vin, void* kout,
                             void* vout, const Tile* tiles, uint32_t ntiles, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    if (kb == 4) {
        if (vb == 0) copy_kb_vb<4, 0>(kin, vin, kout, vout, tiles, ntiles, s);
        else if (vb == 4) copy_kb_vb<4, 4>(kin, vin, kout, vout, tiles, ntiles, s);
        else copy_kb_vb<4, 8>(kin, vin, kout, vout, tiles, ntiles, s);
    } else {
        if (vb == 0) copy_kb_vb<8, 0>(kin, vin, kout, vout, tiles, ntiles, s);
        else if (vb == 4) copy_kb_vb<8, 4>(kin, vin, kout, vout, tiles, ntiles, s);
        else copy_kb_vb<8, 8>(kin, vin, kout, vout, tiles, ntiles, s);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Fixed device scratch of the allocation-free entry point (dfr_sort_noalloc): one
// array per GPU, held until the process ends.  Host code never uses the array's name
// as an address: static_scratch_address() looks up this GPU's copy once (with that GPU
// current) and every later use goes through the pointer it returns.
// ---------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t static_scratch_address(int device, void** ptr) {
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes it current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace dfr
