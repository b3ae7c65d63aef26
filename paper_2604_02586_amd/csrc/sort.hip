// Stable LSD radix sort of 32-bit keys (with optional 32-bit values) for
// gfx950, shared by the binning and the regularisation's neighbour grid.
//
// Per 8-bit pass: a histogram kernel (per block and digit), an exclusive scan
// of the digit-major histogram, and a scatter kernel whose block-local ranks
// are stable (wave64 ballot matching) and whose writes are staged in LDS so
// each digit's run leaves the block contiguously.
#include "tg_internal.h"

namespace {

// 8192 keys per block: a digit's run in the scatter's output averages 32
// keys (128 bytes, one cache line) for uniform digits; 4096-key tiles wrote
// 64-byte runs that straddle lines, about 1.6x the algorithmic write bytes.
// The scatter's LDS (64 KB of keys and values) still fits two blocks, 16
// waves, per CU.
constexpr int SORT_THREADS = 512;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;   // 8192 keys per block
constexpr int SORT_WAVES = SORT_THREADS / TG_WAVE;      // 8
constexpr int WAVE_ITEMS = SORT_TILE / SORT_WAVES;      // 1024 keys per wave
constexpr int DIGIT_WAVES = 256 / TG_WAVE;              // waves owning one digit per thread
static_assert(SORT_THREADS >= 256, "one thread per digit");

// Active length of a segment: fixed, or read from the device (single
// dynamic segment), 0 when the device count exceeds the capacity.
__device__ __forceinline__ int64_t seg_count(int64_t seg_len, const int64_t* dev_count) {
    if (!dev_count) return seg_len;
    int64_t n = *dev_count;
    return n > seg_len ? 0 : n;
}

// Adds one key's digit to the wave's sub-histogram.  FEW: the digit takes
// few distinct values (the top digit of depth keys or of the bin bits), so
// equal digits are first counted across the wave and the lowest lane of each
// group adds the count (one LDS atomic per distinct digit instead of a chain
// of colliding ones).
template <bool FEW>
__device__ __forceinline__ void hist_add(uint32_t* h, uint32_t d, bool active) {
    if (!FEW) {
        if (active) atomicAdd(&h[d], 1u);
        return;
    }
    uint64_t left = ballot64(active);
    while (left) {
        const int lead = __ffsll((unsigned long long)left) - 1;
        const uint32_t d0 = (uint32_t)__shfl((int)d, lead, 64);
        const uint64_t same = ballot64(active && d == d0);
        if ((int)(threadIdx.x & 63) == lead) atomicAdd(&h[d0], (uint32_t)__popcll(same));
        left &= ~same;
    }
}

// Whether the last pass of an LSD sort is the identity for a segment, from
// what the first histogram pass gathered (seginfo[4 seg + 0..3]: AND, OR and
// the largest lower bits -- the bits below the top digit within the sorted
// range -- of the keys that are not all ones, and how many keys are all
// ones, the "culled" sentinel of depth keys).  The last pass sorts by the top
// digit alone, after the earlier passes have sorted by the lower bits (stable
// throughout).  It changes nothing when every ordinary key has one top digit
// d and the sentinels either share it or follow every ordinary key already:
// their lower bits are all ones, so that holds when no ordinary key's lower
// bits are all ones too.
__device__ __forceinline__ bool top_constant(const uint32_t* __restrict__ seginfo, int seg, int bit0,
                                             int top_shift) {
    const uint32_t kand = seginfo[4 * seg], kor = seginfo[4 * seg + 1];
    const uint32_t maxlow = seginfo[4 * seg + 2], nsent = seginfo[4 * seg + 3];
    if (kand > kor) return true;                         // no ordinary key: all keys equal
    if ((((kand ^ kor) >> top_shift) & 255u) != 0u) return false;
    if (nsent == 0u) return true;
    const uint32_t d = (kor >> top_shift) & 255u, ds = (0xFFFFFFFFu >> top_shift) & 255u;
    const uint32_t lowmask = (1u << (top_shift - bit0)) - 1u;
    return d == ds || maxlow < lowmask;
}

constexpr int MODE_ANDOR = 1;     // first pass: AND/OR of the keys into seginfo
constexpr int MODE_SKIP = 2;      // last pass: nothing to do when the top digit is constant
constexpr int MODE_REDIRECT = 4;  // pass before the last: write the final outputs when it is

// Combines the per-block summaries of the first pass (four words per block:
// AND, OR, largest low part, sentinel count) into the segment's summary.
// One block per segment; plain stores from every block and one reduction
// here, since one-word global atomics from thousands of blocks on the same
// few cache lines serialise.
__global__ void __launch_bounds__(256) k_seginfo_reduce(const uint32_t* __restrict__ part, int nblk,
                                                        uint32_t* __restrict__ seginfo) {
    __shared__ uint32_t red[4][256 / TG_WAVE];
    const int seg = blockIdx.x, t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint4* pp = (const uint4*)(part + (int64_t)seg * nblk * 4);
    uint32_t kand = 0xFFFFFFFFu, kor = 0u, kmax = 0u, nsent = 0u;
    for (int b = t; b < nblk; b += 256) {
        const uint4 v = pp[b];
        kand &= v.x;
        kor |= v.y;
        kmax = max(kmax, v.z);
        nsent += v.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kand &= (uint32_t)__shfl_xor((int)kand, o, 64);
        kor |= (uint32_t)__shfl_xor((int)kor, o, 64);
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
        nsent += (uint32_t)__shfl_xor((int)nsent, o, 64);
    }
    if (l == 0) {
        red[0][w] = kand;
        red[1][w] = kor;
        red[2][w] = kmax;
        red[3][w] = nsent;
    }
    __syncthreads();
    if (t == 0) {
        for (int i = 1; i < 256 / TG_WAVE; ++i) {
            kand &= red[0][i];
            kor |= red[1][i];
            kmax = max(kmax, red[2][i]);
            nsent += red[3][i];
        }
        seginfo[4 * seg] = kand;
        seginfo[4 * seg + 1] = kor;
        seginfo[4 * seg + 2] = kmax;
        seginfo[4 * seg + 3] = nsent;
    }
}

// Folds one key into the per-thread summary of ordinary keys and sentinels.
__device__ __forceinline__ void summary_add(uint32_t k, int bit0, uint32_t lowmask, uint32_t& kand, uint32_t& kor,
                                            uint32_t& kmax, uint32_t& nsent) {
    // selects, not branches: the sentinel (all ones) is the identity of AND
    const bool sent = k == 0xFFFFFFFFu;
    kand &= k;
    kor |= sent ? 0u : k;
    kmax = max(kmax, sent ? 0u : (k >> bit0) & lowmask);
    nsent += sent ? 1u : 0u;
}

template <bool FEW, bool SUM>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, int64_t seg_len,
                                                             const int64_t* __restrict__ dev_count, int shift,
                                                             uint32_t* __restrict__ ghist, int nblk,
                                                             uint32_t* __restrict__ seginfo, int mode, int bit0,
                                                             int top_shift)
{
    // one sub-histogram per wave (fewer LDS atomic collisions), keys loaded
    // as uint4 where the block's range is whole and aligned.  With SUM,
    // seginfo is the [nseg][nblk] array of per-block summaries (uint4 each)
    __shared__ uint32_t h[SORT_WAVES][256];
    __shared__ uint32_t bsum[4];
    const int seg = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    if ((mode & MODE_SKIP) && top_constant(seginfo, seg, bit0, top_shift)) return;   // block-uniform
    const int w = t >> 6, l = t & 63;
    for (int i = t; i < SORT_WAVES * 256; i += SORT_THREADS) (&h[0][0])[i] = 0;
    if (t == 0) {
        bsum[0] = 0xFFFFFFFFu;
        bsum[1] = bsum[2] = bsum[3] = 0u;
    }
    __syncthreads();
    const int64_t n = seg_count(seg_len, dev_count);
    const int64_t base = (int64_t)b * SORT_TILE;
    const uint32_t* kp = keys + (int64_t)seg * seg_len;
    const uint32_t lowmask = (1u << (top_shift - bit0)) - 1u;
    uint32_t kand = 0xFFFFFFFFu, kor = 0u, kmax = 0u, nsent = 0u;
    if (base + SORT_TILE <= n && (((uintptr_t)(kp + base)) & 15u) == 0) {
        const uint4* k4 = (const uint4*)(kp + base);
        uint4 kk[SORT_ITEMS / 4];   // every load in flight before the first use
#pragma unroll
        for (int r = 0; r < SORT_ITEMS / 4; ++r) kk[r] = k4[r * SORT_THREADS + t];
#pragma unroll
        for (int r = 0; r < SORT_ITEMS / 4; ++r) {
            const uint4 k = kk[r];
            hist_add<FEW>(h[w], (k.x >> shift) & 255u, true);
            hist_add<FEW>(h[w], (k.y >> shift) & 255u, true);
            hist_add<FEW>(h[w], (k.z >> shift) & 255u, true);
            hist_add<FEW>(h[w], (k.w >> shift) & 255u, true);
            if constexpr (SUM) {
                summary_add(k.x, bit0, lowmask, kand, kor, kmax, nsent);
                summary_add(k.y, bit0, lowmask, kand, kor, kmax, nsent);
                summary_add(k.z, bit0, lowmask, kand, kor, kmax, nsent);
                summary_add(k.w, bit0, lowmask, kand, kor, kmax, nsent);
            }
        }
    } else if (base < n) {
#pragma unroll 4
        for (int r = 0; r < SORT_ITEMS; ++r) {
            int64_t idx = base + w * WAVE_ITEMS + r * TG_WAVE + l;
            const bool in = idx < n;
            const uint32_t k = in ? kp[idx] : 0u;
            hist_add<FEW>(h[w], in ? (k >> shift) & 255u : 0u, in);
            if (SUM && in) summary_add(k, bit0, lowmask, kand, kor, kmax, nsent);
        }
    }
    if (SUM) {
        // across the wave first (butterfly), then across the block's waves;
        // one plain 16-byte store of the block's summary (identity for a
        // block past the end of a counted segment)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kand &= (uint32_t)__shfl_xor((int)kand, o, 64);
            kor |= (uint32_t)__shfl_xor((int)kor, o, 64);
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
            nsent += (uint32_t)__shfl_xor((int)nsent, o, 64);
        }
        if (l == 0) {
            atomicAnd(&bsum[0], kand);
            atomicOr(&bsum[1], kor);
            atomicMax(&bsum[2], kmax);
            atomicAdd(&bsum[3], nsent);
        }
    }
    __syncthreads();
    if (SUM && t == 0)
        ((uint4*)seginfo)[(int64_t)seg * nblk + b] = make_uint4(bsum[0], bsum[1], bsum[2], bsum[3]);
    if (t < 256) {
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < SORT_WAVES; ++ww) c += h[ww][t];
        ghist[((int64_t)seg * 256 + t) * nblk + b] = c;
    }
}

// ---- exclusive scan of a [nseg][L] u32 array (three kernels) ------------
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[SCAN_THREADS / TG_WAVE];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint32_t inc = wave_scan_add_u32(v);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = l < SCAN_THREADS / TG_WAVE ? wsum[l] : 0u;
        uint32_t xi = wave_scan_add_u32(x);
        if (l < SCAN_THREADS / TG_WAVE) wsum[l] = xi - x;
        if (l == SCAN_THREADS / TG_WAVE - 1) *total = xi;
    }
    __syncthreads();
    uint32_t r = wsum[w] + inc - v;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t* __restrict__ in, int64_t L,
                                                              uint32_t* __restrict__ sums, int nchunk)
{
    __shared__ uint32_t tot;
    const int seg = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < L) s += in[(int64_t)seg * L + base + i];
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[(int64_t)seg * nchunk + blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(uint32_t* __restrict__ sums, int nchunk)
{
    // one block per segment; nchunk may exceed the block size
    __shared__ uint32_t tot;
    const int seg = blockIdx.x;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nchunk; c0 += SCAN_THREADS) {
        int c = c0 + threadIdx.x;
        uint32_t v = c < nchunk ? sums[(int64_t)seg * nchunk + c] : 0u;
        uint32_t ex = block_excl_scan(v, &tot);
        if (c < nchunk) sums[(int64_t)seg * nchunk + c] = ex + carry;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(uint32_t* __restrict__ data, int64_t L,
                                                            const uint32_t* __restrict__ sums, int nchunk)
{
    __shared__ uint32_t tot;
    const int seg = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < L ? data[(int64_t)seg * L + base + i] : 0u;
        s += v[i];
    }
    uint32_t ex = block_excl_scan(s, &tot) + sums[(int64_t)seg * nchunk + blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < L) data[(int64_t)seg * L + base + i] = ex;
        ex += v[i];
    }
}

// Exclusive scan of each segment's [L] u32 array in one block of
// SCAN_THREADS per segment (L <= SCAN_THREADS * ITEMS): thread t scans its
// ITEMS consecutive words in registers (16-byte loads), one block scan of
// the thread totals, then writes back.  Replaces the three-kernel scan when
// the segments are small (the radix histograms of per-view depth sorts).
template <int ITEMS>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_seg(uint32_t* __restrict__ data, int64_t L,
                                                           const uint32_t* __restrict__ seginfo, int skip, int bit0,
                                                           int top_shift)
{
    static_assert(ITEMS % 4 == 0, "16-byte chunks");
    // the last pass of a segment whose top digit is constant scatters
    // nothing, so its histogram needs no scan either
    if (skip && top_constant(seginfo, blockIdx.x, bit0, top_shift)) return;   // block-uniform
    __shared__ uint32_t tot;
    uint32_t* d = data + (int64_t)blockIdx.x * L;
    const int64_t i0 = (int64_t)threadIdx.x * ITEMS;
    uint32_t v[ITEMS];
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) {
        const int64_t i = i0 + 4 * q;
        uint4 x = make_uint4(0u, 0u, 0u, 0u);
        if (i + 4 <= L) {
            x = *(const uint4*)(d + i);
        } else {
            if (i < L) x.x = d[i];
            if (i + 1 < L) x.y = d[i + 1];
            if (i + 2 < L) x.z = d[i + 2];
        }
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t x = v[j];
        v[j] = sum;
        sum += x;
    }
    const uint32_t base = block_excl_scan(sum, &tot);
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) {
        const int64_t i = i0 + 4 * q;
        const uint4 x = make_uint4(v[4 * q] + base, v[4 * q + 1] + base, v[4 * q + 2] + base, v[4 * q + 3] + base);
        if (i + 4 <= L) {
            *(uint4*)(d + i) = x;
        } else {
            if (i < L) d[i] = x.x;
            if (i + 1 < L) d[i + 1] = x.y;
            if (i + 2 < L) d[i + 2] = x.z;
        }
    }
}

// ---- stable scatter --------------------------------------------------------
// Items of a block: wave w owns keys [w*1024, (w+1)*1024) of the block's 8192,
// visited in 16 rounds of 64 consecutive keys, so order within the block is
// (wave, round, lane) = input order.  Each key is first placed at its stable
// rank inside the block (digit-major) in LDS; the block then writes the LDS
// array out in order, so consecutive threads write consecutive addresses of
// one digit's run instead of 64 scattered words per instruction.
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t seg_len, const int64_t* __restrict__ dev_count, int shift,
    const uint32_t* __restrict__ goff, int nblk, const uint32_t* __restrict__ seginfo, int mode, int bit0,
    int top_shift, uint32_t* __restrict__ kalt, uint32_t* __restrict__ valt)
{
    if (mode & (MODE_SKIP | MODE_REDIRECT)) {
        // block-uniform: the segment's summary decides
        if (top_constant(seginfo, blockIdx.y, bit0, top_shift)) {
            if (mode & MODE_SKIP) return;
            kout = kalt;
            vout = valt;
        }
    }
    __shared__ uint32_t woff[SORT_WAVES][256];
    __shared__ uint32_t gdelta[256];     // global start of the digit minus its block-local start
    __shared__ uint32_t wtot[SORT_WAVES];
    __shared__ uint32_t LK[SORT_TILE];
    __shared__ uint32_t LV[SORT_TILE];
    const int seg = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    const int64_t n = seg_count(seg_len, dev_count);
    const int64_t base = (int64_t)b * SORT_TILE;
    if (base >= n) return;  // uniform per block
    const int nvalid = (int)((n - base) < SORT_TILE ? (n - base) : SORT_TILE);
    for (int i = t; i < SORT_WAVES * 256; i += SORT_THREADS) (&woff[0][0])[i] = 0;
    __syncthreads();
    const int64_t so = (int64_t)seg * seg_len;
    const bool with_v = vout != nullptr;
    uint32_t k[SORT_ITEMS], val[SORT_ITEMS];
    // every key and value load in flight before the first use (a load
    // followed by its LDS atomic item by item waits out 16 round trips)
    const int64_t i0 = base + w * WAVE_ITEMS + l;
    if (nvalid == SORT_TILE) {
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) k[r] = kin[so + i0 + r * TG_WAVE];
        if (vin) {
#pragma unroll
            for (int r = 0; r < SORT_ITEMS; ++r) val[r] = vin[so + i0 + r * TG_WAVE];
        } else {
#pragma unroll
            for (int r = 0; r < SORT_ITEMS; ++r) val[r] = (uint32_t)(i0 + r * TG_WAVE);
        }
    } else {
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const int64_t idx = i0 + r * TG_WAVE;
            k[r] = idx < n ? kin[so + idx] : 0u;
            val[r] = idx < n ? (vin ? vin[so + idx] : (uint32_t)idx) : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r)
        if (i0 + r * TG_WAVE < n) atomicAdd(&woff[w][(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    {
        // thread t < 256 owns digit t: block-local start of the digit
        // (exclusive scan of the digit totals), then each wave's start
        // inside it
        uint32_t c[SORT_WAVES], tot = 0;
        uint32_t inc = 0;
        if (t < 256) {
#pragma unroll
            for (int ww = 0; ww < SORT_WAVES; ++ww) {
                c[ww] = woff[ww][t];
                tot += c[ww];
            }
            inc = wave_scan_add_u32(tot);   // wave-uniform branch: waves 0..3
            if (l == 63) wtot[w] = inc;
        }
        __syncthreads();
        if (t < 256) {
            uint32_t start = inc - tot;
#pragma unroll
            for (int ww = 0; ww < DIGIT_WAVES; ++ww)
                if (ww < w) start += wtot[ww];
            gdelta[t] = goff[((int64_t)seg * 256 + t) * nblk + b] - start;
            uint32_t run = start;
#pragma unroll
            for (int ww = 0; ww < SORT_WAVES; ++ww) {
                woff[ww][t] = run;
                run += c[ww];
            }
        }
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        int64_t idx = base + w * WAVE_ITEMS + r * TG_WAVE + l;
        bool active = idx < n;
        uint32_t d = (k[r] >> shift) & 255u;
        const uint64_t m = match_digit8(d, active);
        if (active) {
            uint32_t rank = (uint32_t)__popcll(m & lt);
            uint32_t pos = woff[w][d] + rank;       // < nvalid for a consistent histogram
            if (pos < (uint32_t)nvalid) {
                LK[pos] = k[r];
                if (with_v) LV[pos] = val[r];
            }
            if (rank == 0) woff[w][d] += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    for (int i = t; i < nvalid; i += SORT_THREADS) {
        const uint32_t key = LK[i];
        const uint32_t pos = gdelta[(key >> shift) & 255u] + (uint32_t)i;
        if (pos < (uint64_t)n) {  // always true for a consistent histogram
            if (kout) kout[so + pos] = key;
            if (with_v) vout[so + pos] = LV[i];
        }
    }
}

}  // namespace

// ---- radix sort driver -------------------------------------------------------
struct SortBufs {
    uint32_t* hist;   // [nseg][256][nblk]
    uint32_t* sums;   // [nseg][nchunk]
};

size_t tg_sort_scratch_bytes(int64_t seg_len, int nseg) {
    int64_t nblk = (seg_len + SORT_TILE - 1) / SORT_TILE;
    int64_t L = 256 * nblk;
    int64_t nchunk = (L + SCAN_TILE - 1) / SCAN_TILE;
    // histograms, scan sums, segment summaries, per-block summaries
    return ((size_t)nseg * (size_t)(L + nchunk + 64) + 4 * (size_t)nseg * (size_t)nblk + 4) * sizeof(uint32_t);
}

// Sorts nseg segments of seg_len keys (or one segment of *dev_count keys) by
// bits [bit0, bit0 + 8*passes).  Buffers: ka/va hold the input; kb/vb are the
// ping-pong partner.  Final keys/values go to kfinal/vfinal (either may be
// null when not needed).  vin == null means values are the indices.
tg_status tg_radix_sort(const uint32_t* kin, const uint32_t* vin, uint32_t* ka, uint32_t* va, uint32_t* kb,
                     uint32_t* vb, uint32_t* kfinal, uint32_t* vfinal, int64_t seg_len, int nseg,
                     const int64_t* dev_count, int bit0, int passes, void* scratch, hipStream_t s)
{
    const int nblk = (int)((seg_len + SORT_TILE - 1) / SORT_TILE);
    if (nblk == 0) return TG_OK;
    const int64_t L = 256LL * nblk;
    const int nchunk = (int)((L + SCAN_TILE - 1) / SCAN_TILE);
    uint32_t* hist = (uint32_t*)scratch;
    uint32_t* sums = hist + (int64_t)nseg * L;
    // A summary of each segment's keys (first pass): when the last pass is
    // the identity for a segment (the sign and exponent bits of depth keys
    // within a factor of two, the high bits of few bins) the pass before it
    // writes the final outputs and the last pass does nothing for that
    // segment (decided on the device)
    uint32_t* seginfo = sums + (int64_t)nseg * nchunk;
    const int64_t part_off = ((int64_t)nseg * (L + nchunk + 4) + 3) & ~(int64_t)3;   // 16-byte aligned
    uint32_t* part = hist + part_off;
    const int top_shift = bit0 + 8 * (passes - 1);
    bool skip_top = passes >= 2 && top_shift < 32;
    if (skip_top) {
        // the redirected pass must not write a buffer it reads
        const int q = passes - 2;
        const void* in_k = q == 0 ? (const void*)kin : (((q - 1) & 1) ? (const void*)kb : (const void*)ka);
        const void* in_v = q == 0 ? (const void*)vin : (((q - 1) & 1) ? (const void*)vb : (const void*)va);
        for (const void* f : {(const void*)kfinal, (const void*)vfinal})
            if (f && (f == in_k || f == in_v)) skip_top = false;
    }
    const uint32_t* ck = kin;
    const uint32_t* cv = vin;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        uint32_t* ok = last ? kfinal : ((p & 1) ? kb : ka);
        uint32_t* ov = last ? vfinal : ((p & 1) ? vb : va);
        if (!last && !ok) return TG_ERR_INVALID_ARG;
        const int shift = bit0 + 8 * p;
        int mode = 0;
        if (skip_top) {
            if (p == 0) mode |= MODE_ANDOR;
            if (last) mode |= MODE_SKIP;
            if (p == passes - 2) mode |= MODE_REDIRECT;
        }
        // the top digit of a sort (the high exponent bits of depth keys, or
        // the high bits of the bin numbers) takes few distinct values
        if (last)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radix_hist<true, false>), dim3(nblk, nseg), dim3(SORT_THREADS), 0,
                               s, ck, seg_len, dev_count, shift, hist, nblk, seginfo, mode & MODE_SKIP, bit0,
                               top_shift);
        else if (mode & MODE_ANDOR)
        {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radix_hist<false, true>), dim3(nblk, nseg), dim3(SORT_THREADS), 0,
                               s, ck, seg_len, dev_count, shift, hist, nblk, part, mode, bit0, top_shift);
            hipLaunchKernelGGL(k_seginfo_reduce, dim3(nseg), dim3(256), 0, s, part, nblk, seginfo);
        }
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radix_hist<false, false>), dim3(nblk, nseg), dim3(SORT_THREADS), 0,
                               s, ck, seg_len, dev_count, shift, hist, nblk, seginfo, 0, bit0, top_shift);
        if (L <= (int64_t)SCAN_THREADS * 16) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_seg<16>), dim3(nseg), dim3(SCAN_THREADS), 0, s, hist, L,
                               seginfo, mode & MODE_SKIP, bit0, top_shift);
        } else if (L <= (int64_t)SCAN_THREADS * 32) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_seg<32>), dim3(nseg), dim3(SCAN_THREADS), 0, s, hist, L,
                               seginfo, mode & MODE_SKIP, bit0, top_shift);
        } else if (L <= (int64_t)SCAN_THREADS * 64) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_seg<64>), dim3(nseg), dim3(SCAN_THREADS), 0, s, hist, L,
                               seginfo, mode & MODE_SKIP, bit0, top_shift);
        } else {
            hipLaunchKernelGGL(k_scan_reduce, dim3(nchunk, nseg), dim3(SCAN_THREADS), 0, s, hist, L, sums, nchunk);
            hipLaunchKernelGGL(k_scan_sums, dim3(nseg), dim3(SCAN_THREADS), 0, s, sums, nchunk);
            hipLaunchKernelGGL(k_scan_down, dim3(nchunk, nseg), dim3(SCAN_THREADS), 0, s, hist, L, sums, nchunk);
        }
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk, nseg), dim3(SORT_THREADS), 0, s, ck, cv, ok,
                           (last && !vfinal) ? nullptr : ov, seg_len, dev_count, shift, hist, nblk, seginfo,
                           mode & (MODE_SKIP | MODE_REDIRECT), bit0, top_shift, kfinal, vfinal);
        TG_CHECK_LAUNCH();
        ck = ok;
        cv = ov;
    }
    return TG_OK;
}

// In-place exclusive scan of one u32 array of length L; scratch holds one
// u32 per SCAN_TILE elements.
void tg_exclusive_scan_u32(uint32_t* data, int64_t L, uint32_t* scratch, hipStream_t s) {
    if (L <= 0) return;
    const int nchunk = (int)((L + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nchunk, 1), dim3(SCAN_THREADS), 0, s, data, L, scratch, nchunk);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, s, scratch, nchunk);
    hipLaunchKernelGGL(k_scan_down, dim3(nchunk, 1), dim3(SCAN_THREADS), 0, s, data, L, scratch, nchunk);
}
