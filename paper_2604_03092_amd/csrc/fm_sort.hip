// fm_sort.hip -- tile binning on gfx950: depth sort of the projected entries,
// pair emission, stable tile sort and per-tile ranges.
//
// The pair list must come out ordered by (tile, depth key, surfel index).
// Instead of one radix sort over 64-bit (tile, depth) keys of every pair, the
// entries are first sorted by their 32-bit depth key (a stable LSD radix sort,
// so equal keys keep entry order = surfel order), pairs are emitted in that
// order, and a second stable LSD radix sort over the tile id alone groups
// them by tile.  Both sorts are stable, so the result equals the 64-bit sort
// while moving only ceil(tile_bits/8) passes over the pairs.
//
// Every kernel runs on a fixed grid sized on the host from capacities; the
// actual pair count lives in device memory (Status), so nothing here needs a
// host read-back and the whole sequence can be graph-captured.
#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

// Item count of a pass: from device memory when n_dev is set, else n_host.
__device__ __forceinline__ uint32_t count_of(const uint32_t *n_dev, uint32_t n_host) {
    return n_dev ? *n_dev : n_host;
}
// Entries culled or off-screen, and pairs of tiles that the support ellipse
// misses, carry this key; the first pass of each sort drops them.
constexpr uint32_t kNoKey = 0xFFFFFFFFu;
// Items of the logical block handled by this workgroup: a fixed tile of
// kSortTile consecutive items.  Each XCD gets a contiguous run of tiles, so
// the neighbouring output runs of one digit stay in one L2, which merges
// their partial cache-line writes before they reach HBM.  The grid is sized
// for the capacity; only the first ga = ceil(n / kSortTile) workgroups hold
// items, and they are the ones spread over the XCDs (workgroups go to XCDs
// round-robin), so a pass over fewer items than the capacity still uses the
// whole chip.  The rest map to themselves and see empty tiles.
__device__ __forceinline__ uint32_t logical_block(uint32_t n, int G) {
    uint32_t ga = (uint32_t)(((uint64_t)n + kSortTile - 1) / kSortTile);
    if (ga > (uint32_t)G) ga = (uint32_t)G;
    return blockIdx.x < ga ? xcd_contiguous(blockIdx.x, ga) : blockIdx.x;
}
__device__ __forceinline__ void tile_of(uint32_t n, int G, uint32_t &lo, uint32_t &hi) {
    const uint64_t l = (uint64_t)logical_block(n, G) * kSortTile;
    lo = l < n ? (uint32_t)l : n;
    hi = l + kSortTile < n ? (uint32_t)(l + kSortTile) : n;
}

// Per-block digit histogram, written digit-major: hist[d * G + block].  With
// `drop`, items whose key is kNoKey are left out.  Each wave counts its run of
// 1024 items (all loads issued first); lanes with equal digits are matched
// through ballots and their lowest lane adds the group's size to the wave's
// LDS counters.
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                     uint32_t n_host, int shift, uint32_t *__restrict__ hist,
                                                     int G, int drop) {
    constexpr int IPT = kSortTile / 256;
    __shared__ uint32_t h[4][kRadix];
    const int w = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
    for (int k = 0; k < 4; ++k) h[k][threadIdx.x] = 0;
    const uint32_t n = count_of(n_dev, n_host);
    uint32_t lo, hi;
    tile_of(n, G, lo, hi);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t wbase = lo + (uint32_t)w * (kSortTile / 4);
    uint32_t key[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t i = wbase + (uint32_t)k * 64u + (uint32_t)lane;
        key[k] = i < hi ? keys[i] : kNoKey;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t i = wbase + (uint32_t)k * 64u + (uint32_t)lane;
        const bool ok = i < hi && !(drop && key[k] == kNoKey);
        if (ballot64(ok) == 0) continue;
        const uint32_t d = (key[k] >> shift) & 0xFFu;
        uint64_t m = ballot64(ok);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot64(bit);
            m &= bit ? bb : ~bb;
        }
        if (ok && (m & lt) == 0) atomicAdd(&h[w][d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    hist[threadIdx.x * G + logical_block(n, G)] = h[0][threadIdx.x] + h[1][threadIdx.x] + h[2][threadIdx.x] +
                                               h[3][threadIdx.x];
}

// Block d turns row d of the histogram into the exclusive prefix over the
// blocks (each block's start within the digit's run) and stores the digit's
// total in tot[d]; the scatter adds the digit's base (the sum of the totals
// of the smaller digits).
__global__ __launch_bounds__(256) void k_radix_rowscan(uint32_t *__restrict__ hist, int G,
                                                        uint32_t *__restrict__ tot) {
    __shared__ uint32_t wsum[4];
    const int d = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = lane_id();
    uint32_t carry = 0;
    uint32_t *row = hist + (size_t)d * G;
    // rounds of 256 x R columns, R consecutive ones per thread
    constexpr int R = 16;
    for (int base = 0; base < G; base += 256 * R) {
        const int b0 = base + (int)threadIdx.x * R;
        uint32_t c[R];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            c[i] = b0 + i < G ? row[b0 + i] : 0u;
            run += c[i];
        }
        uint32_t x = run;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t o = carry + x - run;
        for (int j = 0; j < w; ++j) o += wsum[j];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (b0 + i < G) row[b0 + i] = o;
            o += c[i];
        }
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[d] = carry;
}


// Stable scatter by digit through a local sort.  The block's tile of
// kSortTile items is split into one run of 1024 per wave; a wave ranks its
// items in order (16 steps of 64 lanes; lanes with equal digits are matched
// through ballots) against per-wave digit counters in LDS.  Per digit, the
// waves' counts give the wave offsets and a scan over the digits the
// block-local start of each digit's run.  The items are placed in LDS in
// (digit, original order) order and written out by consecutive threads, so
// each digit's run leaves the block as one contiguous, coalesced stream.
// The global start of the block's run of digit d is its row-scanned
// histogram entry plus the digit's base, the exclusive scan of the digit
// totals, which every block forms itself; block 0 also stores the number of
// items the pass keeps when n_kept is set.
// CARRY moves a second word per item along with the key and value, read at
// the item's input position from v2_in (so the first pass of a sort, whose
// input is in entry order, reads it coalesced): CARRY 1 writes it to v2_out
// at the output position, CARRY 2 writes it in place of the key (the last
// pass of a sort whose keys are not needed afterwards; the digits are kept
// in LDS).
// With RANGES (the last pass of the tile sort), the pass also finds the
// tile ranges [ts, te) of the sorted output: inside one of the block's
// digit runs the keys are sorted, so a key change there is a tile boundary
// of the whole output and is stored directly; at the ends of a run the
// neighbour belongs to another block, so the run's first position enters
// ts of its tile with an atomic min and its last position + 1 enters te
// with an atomic max (ts starts at 0xFFFFFFFF, te at 0: a tile without
// pairs keeps ts > te).
template <int CARRY, bool RANGES>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ keys_in,
                                                        const uint32_t *__restrict__ vals_in,
                                                        uint32_t *__restrict__ keys_out,
                                                        uint32_t *__restrict__ vals_out, const uint32_t *n_dev,
                                                        uint32_t n_host, int shift,
                                                        const uint32_t *__restrict__ hist, int G, int drop,
                                                        const uint32_t *__restrict__ tot, uint32_t *n_kept,
                                                        const uint32_t *__restrict__ v2_in,
                                                        uint32_t *__restrict__ v2_out,
                                                        uint32_t *__restrict__ ts, uint32_t *__restrict__ te,
                                                        uint32_t n_tiles) {
    constexpr int IPT = kSortTile / 256;   // items per lane
    constexpr int PER_WAVE = kSortTile / 4;
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint8_t s_dig[CARRY == 2 ? kSortTile : 1];
    __shared__ uint32_t s_v2[CARRY == 1 ? kSortTile : 1];
    __shared__ uint32_t s_wcnt[4][kRadix];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t s_start[kRadix];    // block-local start of each digit's run
    __shared__ uint32_t s_glob[kRadix];     // global start of this block's run of each digit
    __shared__ uint32_t s_wsum[4];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t n = count_of(n_dev, n_host);
    uint32_t lo, hi;
    tile_of(n, G, lo, hi);
    if (lo >= hi) return;  // uniform over the block (block 0 returns only when the pass has no items)
    {
        // thread = digit: base of the digit = exclusive scan of the totals
        const uint32_t t = tot[threadIdx.x];
        uint32_t x = t;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
        __syncthreads();
        uint32_t base = x - t;
        for (int j = 0; j < w; ++j) base += s_wsum[j];
        s_glob[threadIdx.x] = hist[threadIdx.x * G + logical_block(n, G)] + base;
        if (n_kept && blockIdx.x == 0 && threadIdx.x == kRadix - 1) *n_kept = base + t;
        __syncthreads();  // s_wsum is reused below
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wcnt[k][threadIdx.x] = 0u;
    uint32_t key[IPT], val[IPT];
    const uint32_t wbase = lo + (uint32_t)w * PER_WAVE;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t i = wbase + (uint32_t)k * 64u + (uint32_t)lane;
        const bool valid = i < hi;
        key[k] = valid ? keys_in[i] : kNoKey;
        val[k] = valid ? (vals_in ? vals_in[i] : i) : 0u;
    }
    uint32_t v2[CARRY ? IPT : 1];
    if (CARRY) {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint32_t i = wbase + (uint32_t)k * 64u + (uint32_t)lane;
            v2[k] = i < hi ? v2_in[i] : 0u;
        }
    }
    __syncthreads();
    uint32_t rank[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t i = wbase + (uint32_t)k * 64u + (uint32_t)lane;
        const bool ok = i < hi && !(drop && key[k] == kNoKey);
        const uint32_t d = (key[k] >> shift) & 0xFFu;
        uint64_t m = ballot64(ok);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot64(bit);
            m &= bit ? bb : ~bb;
        }
        // the wave's LDS accesses complete in order: every lane reads the
        // counter before its group's lowest lane advances it
        const uint32_t before = ok ? s_wcnt[w][d] : 0u;
        rank[k] = ok ? before + (uint32_t)__popcll(m & lt) : 0xFFFFFFFFu;
        if (ok && (m & lt) == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(m);
    }
    __syncthreads();
    {
        // thread = digit: wave offsets, then the block-wide exclusive scan of the totals
        const int d = threadIdx.x;
        const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        s_wcnt[0][d] = 0u;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
        const uint32_t all = c0 + c1 + c2 + c3;
        uint32_t x = all;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
        __syncthreads();
        uint32_t pre = x - all;
        for (int j = 0; j < w; ++j) pre += s_wsum[j];
        s_start[d] = pre;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        if (rank[k] == 0xFFFFFFFFu) continue;
        const uint32_t d = (key[k] >> shift) & 0xFFu;
        const uint32_t lp = s_start[d] + s_wcnt[w][d] + rank[k];
        if (lp < (uint32_t)kSortTile) {  // always holds; guards the LDS store
            if (CARRY == 2) {
                s_key[lp] = v2[k];
                s_dig[lp] = (uint8_t)d;
            } else {
                s_key[lp] = key[k];
            }
            if (CARRY == 1) s_v2[lp] = v2[k];
            s_val[lp] = val[k];
        }
    }
    __syncthreads();
    const uint32_t total = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    for (uint32_t i = threadIdx.x; i < total; i += 256) {
        const uint32_t k = s_key[i];
        const uint32_t d = CARRY == 2 ? (uint32_t)s_dig[i] : (k >> shift) & 0xFFu;
        const uint32_t g = s_glob[d] + (i - s_start[d]);
        if (g < n) {  // always holds; guards the store
            keys_out[g] = k;
            vals_out[g] = s_val[i];
            if (CARRY == 1) v2_out[g] = s_v2[i];
            if (RANGES && k < n_tiles) {
                if (i == s_start[d]) atomicMin(&ts[k], g);
                else if (s_key[i - 1] != k) ts[k] = g;
                const uint32_t kn = i + 1 < total ? s_key[i + 1] : kNoKey;
                if (i + 1 >= total || ((kn >> shift) & 0xFFu) != d) atomicMax(&te[k], g + 1u);
                else if (kn != k) te[k] = g + 1u;
            }
        }
    }
}

// ---- pair count scan and emission -----------------------------------------

// Block b sums the tile counts of sorted entries [b*kScanChunk, ...)
// (cnt_sorted: the counts in depth order, written by the last depth pass).
__global__ __launch_bounds__(256) void k_count_reduce(const uint32_t *__restrict__ cnt_sorted, const uint32_t *n_vis,
                                                       uint32_t *__restrict__ blk) {
    __shared__ uint32_t red[4];
    const int64_t E = *n_vis;
    const int64_t lo = (int64_t)blockIdx.x * kScanChunk;
    int64_t hi = lo + kScanChunk;
    if (hi > E) hi = E;
    // all of a thread's loads are issued before they are added
    uint32_t c[kScanChunk / 256];
#pragma unroll
    for (int u = 0; u < kScanChunk / 256; ++u) {
        const int64_t k = lo + threadIdx.x + u * 256;
        c[u] = k < hi ? cnt_sorted[k] : 0u;
    }
    uint32_t s = 0;
#pragma unroll
    for (int u = 0; u < kScanChunk / 256; ++u) s += c[u];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Which 8x8 pixel blocks (16x16 quadrants of a 32x32 tile) of the tile with
// origin (x0, y0) may hold a pixel
// centre inside the entry's culling ellipse.  Per block row, the x-extent of
// the ellipse over that row band is the hull of the slices at the clamped
// band edges and of the leftmost/rightmost points when they fall inside the
// band; it is widened by 0.01 px, which covers the FP32 rounding here
// (hardware square root and reciprocal, 1 ulp).
template <int TW, int TH> __device__ inline uint32_t block_mask(const Ell &el, int x0, int y0) {
    const float hy2 = el.hy * el.hy;
    constexpr int bs = (TW == 32 && TH == 32) ? 16 : 8;
    constexpr int bw = TW / bs, bh = TH / bs;
    constexpr float span = (float)bs - 0.5f;
    uint32_t mask = 0;
#pragma unroll
    for (int br = 0; br < bh; ++br) {
        float dy0 = (float)(y0 + bs * br) + 0.5f - el.ey - 0.01f;
        float dy1 = (float)(y0 + bs * br) + span - el.ey + 0.01f;
        dy0 = fmaxf(dy0, -el.hy);
        dy1 = fminf(dy1, el.hy);
        if (!(dy0 <= dy1)) continue;
        const float q0 = __builtin_amdgcn_sqrtf(fmaxf(el.k2 * (hy2 - dy0 * dy0), 0.f));
        const float q1 = __builtin_amdgcn_sqrtf(fmaxf(el.k2 * (hy2 - dy1 * dy1), 0.f));
        float xmax = fmaxf(el.k1 * dy0 + q0, el.k1 * dy1 + q1);
        float xmin = fminf(el.k1 * dy0 - q0, el.k1 * dy1 - q1);
        if (el.dyr >= dy0 && el.dyr <= dy1) xmax = el.hx;
        if (-el.dyr >= dy0 && -el.dyr <= dy1) xmin = -el.hx;
        xmax += el.ex + 0.01f;
        xmin += el.ex - 0.01f;
#pragma unroll
        for (int bc = 0; bc < bw; ++bc) {
            const float bx0 = (float)(x0 + bs * bc) + 0.5f, bx1 = (float)(x0 + bs * bc) + span;
            if (xmax >= bx0 && xmin <= bx1) mask |= 1u << (br * bw + bc);
        }
    }
    return mask;
}

// Pair offsets of the depth-sorted entries and the first entry of every
// emission chunk.  Block b owns sorted entries [b*kScanChunk, ...), thread t
// the kPer consecutive ones from b*kScanChunk + t*kPer; the exclusive scan of
// their tile counts, plus the block's offset, gives each entry's first pair.
// The block's offset is the sum of the block sums of blocks 0 .. b-1, which
// every block forms itself (64-bit); the block holding the last visible
// entry also records the batch's pair count, whether it exceeds the
// capacity, and the pairs stored (a batch without visible entries keeps the
// cleared status: no pairs).
// Offsets are clamped to the capacity (pairs beyond it are never emitted).
// Every entry that holds the first pair of a chunk of kEmitChunk pairs writes
// its sorted index into chunk_first.  Visible entries cover at least one
// tile, so chunk c's pairs belong to entries chunk_first[c] .. chunk_first[c+1].
// off32 may alias cnt_sorted: a thread reads its counts before it writes the
// same positions.
constexpr int kPer = kScanChunk / 256;
__global__ __launch_bounds__(256) void k_offsets(const uint32_t *cnt_sorted, const uint32_t *n_vis,
                                                  const uint32_t *__restrict__ blk, Status *st, uint64_t cap,
                                                  uint32_t *off32, uint32_t *__restrict__ chunk_first) {
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t wpre[4];
    const int64_t E = *n_vis;
    const int64_t lo = (int64_t)blockIdx.x * kScanChunk;
    if (lo >= E) return;
    const int w = threadIdx.x >> 6, lane = lane_id();
    uint64_t pre = 0;
    for (int i = (int)threadIdx.x; i < (int)blockIdx.x; i += 256) pre += blk[i];
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t l32 = __shfl_xor((uint32_t)pre, off), h32 = __shfl_xor((uint32_t)(pre >> 32), off);
        pre += ((uint64_t)h32 << 32) | l32;
    }
    if (lane == 0) wpre[w] = pre;
    const int64_t k0 = lo + (int64_t)threadIdx.x * kPer;
    uint32_t c[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) c[i] = k0 + i < E ? cnt_sorted[k0 + i] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) run += c[i];
    uint32_t x = run;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    const uint64_t base = wpre[0] + wpre[1] + wpre[2] + wpre[3];
    if (threadIdx.x == 0 && E - lo <= kScanChunk) {
        const uint64_t total = base + (uint64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
        st->required = total;
        st->overflow = total > cap ? 1u : 0u;
        st->n_pairs = (uint32_t)(total > cap ? cap : total);
    }
    uint64_t o = base + (x - run);
    for (int j = 0; j < w; ++j) o += wsum[j];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int64_t k = k0 + i;
        if (k < E) {
            off32[k] = (uint32_t)(o < cap ? o : cap);
            // chunk boundaries inside [o, o + c): the first multiple of kEmitChunk >= o, then every kEmitChunk
            for (uint64_t bnd = (o + kEmitChunk - 1) / kEmitChunk * kEmitChunk; bnd < o + c[i] && bnd < cap;
                 bnd += kEmitChunk)
                chunk_first[bnd / kEmitChunk] = (uint32_t)k;
        }
        o += c[i];
    }
}

// Pair emission balanced over pairs: each iteration of a block emits one
// chunk of kEmitChunk consecutive pairs.  The chunk's entries (at most
// kEmitChunk, each covering >= 1 tile) are staged in LDS; every entry marks
// the chunk position of its first pair with its local index and an inclusive
// max-scan over the chunk gives every pair its entry.  Consecutive threads
// write consecutive pairs.  With meta (deterministic gradients) the sorted
// value is the pair's emission index and meta holds its entry and mask.
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t x, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x = y > x ? y : x;
    }
    return x;
}

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ sorted_entry,
                                               const uint32_t *__restrict__ off32, const uint32_t *n_vis,
                                               const uint32_t *__restrict__ chunk_first, const Status *st,
                                               const Ell *__restrict__ ell,
                                               uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
                                               uint32_t *__restrict__ hist, int G,
                                               uint32_t *__restrict__ meta) {
    static_assert(2 * kEmitChunk == kSortTile && kRadix == 256, "two chunks make a tile of the first tile-sort pass");
    constexpr int PER = kEmitChunk / 256;
    __shared__ uint32_t s_own[kEmitChunk];
    __shared__ uint32_t s_ent[kEmitChunk];
    __shared__ uint32_t s_off[kEmitChunk];
    __shared__ uint32_t s_hist[kRadix];
    __shared__ uint32_t wmax[4];
    const uint32_t total = st->n_pairs;
    const uint32_t nv = *n_vis;
    const uint32_t nchunks = (total + kEmitChunk - 1) / kEmitChunk;
    const int w = threadIdx.x >> 6, lane = lane_id();
    // chunks 2t and 2t+1 make tile t of the first tile-sort pass: a block
    // emits both and writes the digit histogram of their kept keys (low 8
    // bits) to column t; the columns of the grid's tiles past the last chunk
    // are cleared
    for (uint32_t t = blockIdx.x; t < (uint32_t)G; t += gridDim.x) {
        if (2u * t >= nchunks) {  // uniform over the block
            hist[threadIdx.x * (uint32_t)G + t] = 0u;
            continue;
        }
        __syncthreads();  // the previous tile's histogram has been read
        s_hist[threadIdx.x] = 0u;
        for (uint32_t c = 2u * t; c < 2u * t + 2u && c < nchunks; ++c) {
            const uint32_t p0 = c * kEmitChunk;
            const uint32_t np = total - p0 < (uint32_t)kEmitChunk ? total - p0 : (uint32_t)kEmitChunk;
            const uint32_t first = chunk_first[c];
            const uint32_t lastx = c + 1 < nchunks ? chunk_first[c + 1] + 1 : nv;
            uint32_t n_ent = lastx > first ? lastx - first : 0u;
            if (n_ent > (uint32_t)kEmitChunk) n_ent = kEmitChunk;
            if (first >= nv || first + n_ent > nv) n_ent = 0;  // cannot happen; guards the loads
            __syncthreads();  // the previous chunk's readers are done with the LDS arrays
#pragma unroll
            for (int i = 0; i < PER; ++i) s_own[i * 256 + threadIdx.x] = 0u;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n_ent; i += 256) {
                const uint32_t o = off32[first + i];
                s_ent[i] = sorted_entry[first + i];
                s_off[i] = o;
                const uint32_t ls = o > p0 ? o - p0 : 0u;
                if (ls < np && i > 0) s_own[ls] = i;
            }
            __syncthreads();
            // inclusive max-scan of s_own: a thread owns PER consecutive positions
            uint32_t v[PER];
            uint32_t m = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint32_t y = s_own[threadIdx.x * PER + i];
                m = y > m ? y : m;
                v[i] = m;
            }
            const uint32_t incl = wave_incl_max_u32(m, lane);
            if (lane == 63) wmax[w] = incl;
            __syncthreads();
            uint32_t pre = __shfl_up(incl, 1);
            if (lane == 0) pre = 0;
            for (int j = 0; j < w; ++j) pre = wmax[j] > pre ? wmax[j] : pre;
#pragma unroll
            for (int i = 0; i < PER; ++i) s_own[threadIdx.x * PER + i] = v[i] > pre ? v[i] : pre;
            __syncthreads();
            for (uint32_t q = threadIdx.x; q < np; q += 256) {
                uint32_t i = s_own[q];
                if (i >= n_ent) i = 0;  // cannot happen; keeps the LDS read in range
                const uint32_t ent = s_ent[i];
                const uint32_t r = p0 + q - s_off[i];
                Ell el;  // the first 48 bytes (the padding is not read)
                {
                    const float4 *q = reinterpret_cast<const float4 *>(ell + ent);
                    const float4 a = q[0], b = q[1], c4 = q[2];
                    el.ex = a.x; el.ey = a.y; el.hx = a.z; el.hy = a.w;
                    el.k1 = b.x; el.k2 = b.y; el.dyr = b.z; el.tb = __float_as_uint(b.w);
                    el.t0 = __float_as_uint(c4.x); el.nt = __float_as_uint(c4.y);
                }
                const uint32_t ntx = el.nt & 0xFFFFu, tiles_x = el.nt >> 16;
                // r / ntx: r < 2^24, so the float estimate is off by at most one
                uint32_t ry = (uint32_t)((float)r * __builtin_amdgcn_rcpf((float)ntx));
                if (ry * ntx > r) --ry;
                else if ((ry + 1u) * ntx <= r) ++ry;
                const uint32_t rx = r - ry * ntx;
                const int tx = (int)(el.t0 & 0xFFFFu) + (int)rx, ty = (int)(el.t0 >> 16) + (int)ry;
                const uint32_t mask = block_mask<TW, TH>(el, tx * TW, ty * TH);
                // a tile of the rect that no block of reaches carries no pair: its
                // key drops it in the first tile-sort pass
                const uint32_t key = el.tb + ry * tiles_x + rx;
                pkey[p0 + q] = mask ? key : kNoKey;
                const uint32_t v = ent | (mask << kMaskShift);
                if (meta) {  // deterministic lists carry the emission index
                    pval[p0 + q] = p0 + q;
                    meta[p0 + q] = v;
                } else {
                    pval[p0 + q] = v;
                }
                if (mask) atomicAdd(&s_hist[key & 0xFFu], 1u);
            }
        }
        __syncthreads();
        hist[threadIdx.x * (uint32_t)G + t] = s_hist[threadIdx.x];
    }
}

__global__ __launch_bounds__(256) void k_init_ranges(uint32_t *__restrict__ status, int n_status,
                                                      uint32_t *__restrict__ tbucket,
                                                      uint32_t *__restrict__ ts, uint32_t *__restrict__ te,
                                                      int64_t n) {
    init_ranges_block(status, n_status, tbucket, ts, te, n);
}

// Blend order: a tile's cost bucket is 255 minus 16 log2(1 + list length)
// (capped); listing the tiles by increasing bucket puts the longest lists
// first, so the blend's workgroups (which take tiles in that order) start the
// long tiles early and the short ones fill the end of the launch.  Two
// kernels: a histogram of the buckets (LDS per block, one global atomic per
// bucket and block), then each block takes ranges of its buckets' slots with
// one atomic per bucket and places its tiles.  The order within a bucket
// depends on the schedule; nothing computed depends on the order.
__device__ __forceinline__ uint32_t tile_bucket(const uint32_t *ts, const uint32_t *te, int64_t i) {
    const uint32_t len = te[i] > ts[i] ? te[i] - ts[i] : 0u;  // an empty tile has ts > te
    const float lv = 16.f * __log2f((float)len + 1.f);
    return 255u - (lv < 255.f ? (uint32_t)lv : 255u);
}

__global__ __launch_bounds__(256) void k_tile_cost(const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                    int64_t n, uint32_t *__restrict__ bucket_count) {
    __shared__ uint32_t s_hist[kRadix];
    s_hist[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        atomicAdd(&s_hist[tile_bucket(ts, te, i)], 1u);
    __syncthreads();
    if (s_hist[threadIdx.x]) atomicAdd(&bucket_count[threadIdx.x], s_hist[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_tile_place(const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                     int64_t n, const uint32_t *__restrict__ bucket_count,
                                                     uint32_t *__restrict__ bucket_cursor,
                                                     uint32_t *__restrict__ order) {
    __shared__ uint32_t s_base[kRadix], s_cnt[kRadix], s_take[kRadix];
    // exclusive scan of the bucket counts (each block redundantly)
    const int lane = lane_id(), w = threadIdx.x >> 6;
    __shared__ uint32_t wsum[4];
    const uint32_t c = bucket_count[threadIdx.x];
    uint32_t x = c;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t base = x - c;
    for (int j = 0; j < w; ++j) base += wsum[j];
    s_base[threadIdx.x] = base;
    for (int64_t i0 = (int64_t)blockIdx.x * 256; i0 < n; i0 += (int64_t)gridDim.x * 256) {
        const int64_t i = i0 + threadIdx.x;
        __syncthreads();
        s_cnt[threadIdx.x] = 0u;
        __syncthreads();
        uint32_t b = 0, rank = 0;
        if (i < n) {
            b = tile_bucket(ts, te, i);
            rank = atomicAdd(&s_cnt[b], 1u);
        }
        __syncthreads();
        if (s_cnt[threadIdx.x]) s_take[threadIdx.x] = atomicAdd(&bucket_cursor[threadIdx.x], s_cnt[threadIdx.x]);
        __syncthreads();
        if (i < n) order[s_base[b] + s_take[b] + rank] = (uint32_t)i;
    }
}

void radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, const uint32_t *n_dev,
                uint32_t n_host, int shift, uint32_t *hist, int G, uint32_t *tot, int drop, uint32_t *n_kept,
                hipStream_t s, int carry = 0, const uint32_t *v2_in = nullptr, uint32_t *v2_out = nullptr,
                bool hist_ready = false, uint32_t *ts = nullptr, uint32_t *te = nullptr, uint32_t n_tiles = 0) {
    if (!hist_ready)
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(256), 0, s, kin, n_dev, n_host, shift, hist, G, drop);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadix), dim3(256), 0, s, hist, G, tot);
#define FM_SCATTER(C, R)                                                                                     \
    hipLaunchKernelGGL((k_radix_scatter<C, R>), dim3(G), dim3(256), 0, s, kin, vin, kout, vout, n_dev, n_host, \
                       shift, hist, G, drop, tot, n_kept, v2_in, v2_out, ts, te, n_tiles)
    if (carry == 1) FM_SCATTER(1, false);
    else if (carry == 2) FM_SCATTER(2, false);
    else if (ts) FM_SCATTER(0, true);
    else FM_SCATTER(0, false);
#undef FM_SCATTER
}

}  // namespace

int init_ranges_blocks(const Plan &p) {
    const int64_t b = (p.T + 255) / 256;
    return (int)(b < 1 ? 1 : (b < 4096 ? b : 4096));
}

hipError_t launch_init_ranges(const Plan &p, void *ws, hipStream_t st) {
    static_assert(sizeof(Status) / 4 <= 256, "status words are cleared by one block");
    hipLaunchKernelGGL(k_init_ranges, dim3(init_ranges_blocks(p)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t *>(at<Status>(ws, p.o_status)), (int)(sizeof(Status) / 4),
                       at<uint32_t>(ws, p.o_tbucket), at<uint32_t>(ws, p.o_tstart), at<uint32_t>(ws, p.o_tend), p.T);
    return hipGetLastError();
}

hipError_t launch_binning(const Plan &p, void *ws, hipStream_t st) {
    Status *status = at<Status>(ws, p.o_status);
    uint32_t *key = at<uint32_t>(ws, p.o_key), *key2 = at<uint32_t>(ws, p.o_key2);
    uint32_t *val = at<uint32_t>(ws, p.o_val), *val2 = at<uint32_t>(ws, p.o_val2);
    uint32_t *hist = at<uint32_t>(ws, p.o_hist);
    uint32_t *tot = at<uint32_t>(ws, p.o_tot);
    uint32_t *ts = at<uint32_t>(ws, p.o_tstart), *te = at<uint32_t>(ws, p.o_tend);
    // (the status words, the tile ranges and the order's buckets were
    // initialised by the setup of the call)
    // 1. stable sort of the entries by their 32-bit depth key (4 passes; the
    //    first pass starts from the identity permutation and drops the
    //    entries that cover no tile, so the later passes see only the
    //    visible ones)
    const uint32_t E = (uint32_t)p.E;
    uint32_t *n_vis = &status->n_vis;
    // each entry's tile count rides along (read coalesced by the first pass
    // in entry order) and the last pass outputs it in place of the key
    const uint32_t *cnt = at<uint32_t>(ws, p.o_cnt);
    uint32_t *ca = at<uint32_t>(ws, p.o_cnt2), *cb = at<uint32_t>(ws, p.o_cnt3);
    radix_pass(key, nullptr, key2, val2, nullptr, E, 0, hist, p.sortG_e, tot + 0 * kRadix, 1, n_vis, st, 1, cnt, ca);
    radix_pass(key2, val2, key, val, n_vis, 0, 8, hist, p.sortG_e, tot + 1 * kRadix, 0, nullptr, st, 1, ca, cb);
    radix_pass(key, val, key2, val2, n_vis, 0, 16, hist, p.sortG_e, tot + 2 * kRadix, 0, nullptr, st, 1, cb, ca);
    radix_pass(key2, val2, key, val, n_vis, 0, 24, hist, p.sortG_e, tot + 3 * kRadix, 0, nullptr, st, 2, ca);
    // 2. pair offsets in depth order and emission
    uint32_t *blk = at<uint32_t>(ws, p.o_scan);
    // the key buffer holds the counts in depth order
    uint32_t *cnt_sorted = key;
    hipLaunchKernelGGL(k_count_reduce, dim3(p.scan_blocks), dim3(256), 0, st, cnt_sorted, n_vis, blk);
    uint32_t *pkey = at<uint32_t>(ws, p.o_pkey), *pval = at<uint32_t>(ws, p.o_pval);
    uint32_t *pkey2 = at<uint32_t>(ws, p.o_pkey2), *pval2 = at<uint32_t>(ws, p.o_pval2);
    // the offsets replace the counts in place
    uint32_t *off32 = key;
    uint32_t *chunk_first = at<uint32_t>(ws, p.o_chunk);
    hipLaunchKernelGGL(k_offsets, dim3(p.scan_blocks), dim3(256), 0, st, cnt_sorted, n_vis, blk, status,
                       (uint64_t)p.cap, off32, chunk_first);
#define FM_EMIT(TW, TH)                                                                                        \
    hipLaunchKernelGGL((k_emit<TW, TH>), dim3(p.emit_blocks), dim3(256), 0, st, val, off32, n_vis, chunk_first,   \
                       status, at<Ell>(ws, p.o_ell), pkey, pval, hist, p.sortG_p,                    \
                       p.det ? at<uint32_t>(ws, p.o_meta) : nullptr)
    if (p.tile_w == 16 && p.tile_h == 16) FM_EMIT(16, 16);
    else if (p.tile_w == 8 && p.tile_h == 8) FM_EMIT(8, 8);
    else if (p.tile_w == 16 && p.tile_h == 8) FM_EMIT(16, 8);
    else if (p.tile_w == 32 && p.tile_h == 8) FM_EMIT(32, 8);
    else if (p.tile_w == 32 && p.tile_h == 32) FM_EMIT(32, 32);
    else return hipErrorInvalidValue;
#undef FM_EMIT
    // 3. stable sort of the pairs by tile id; the last pass also writes the
    //    per-tile ranges
    uint32_t *ka = pkey, *va = pval, *kb = pkey2, *vb = pval2;
    // (the first pass drops the pairs of missed tiles and counts the rest;
    // its histogram comes from the emission)
    for (int pass = 0; pass < p.pair_passes; ++pass) {
        const bool last = pass + 1 == p.pair_passes;
        radix_pass(ka, va, kb, vb, pass == 0 ? &status->n_pairs : &status->n_kept, 0, 8 * pass, hist, p.sortG_p,
                   tot + (4 + pass) * kRadix, pass == 0 ? 1 : 0, pass == 0 ? &status->n_kept : nullptr, st, 0,
                   nullptr, nullptr, pass == 0, last ? ts : nullptr, last ? te : nullptr, (uint32_t)p.T);
        uint32_t *t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    // 4. the longest-first tile order, written whichever order the blend
    //    uses, so that a later call on this workspace may choose either
    uint32_t *tb = at<uint32_t>(ws, p.o_tbucket);
    const int tblocks = (int)std::min<int64_t>((p.T + 255) / 256, 1024);
    hipLaunchKernelGGL(k_tile_cost, dim3(tblocks), dim3(256), 0, st, ts, te, p.T, tb);
    hipLaunchKernelGGL(k_tile_place, dim3(tblocks), dim3(256), 0, st, ts, te, p.T, tb, tb + kRadix,
                       at<uint32_t>(ws, p.o_torder));
    return hipGetLastError();
}

}  // namespace fm
