// tg_bin_sort / tg_bin_expand: depth ordering and coarse binning
// (TrackerSplat Sec. 3.1: blending follows the Gaussians' depth order).
//
// Design for CDNA4: instead of sorting one 64-bit (tile | depth) key per
// (tile, Gaussian) pair -- about 16M pairs per 1080p view at 1M Gaussians --
// we (1) radix-sort the N depth keys of each view once, then (2) emit one
// 32-bit key (coarse bin | Gaussian id) per (coarse bin, Gaussian) pair, with
// coarse bins of 8x8 tiles, written in (view, depth rank) order: a count
// pass, a scan of the per-block counts, and a write pass that places every
// block's pairs in rank order.  (3) A stable radix sort over the coarse-bin
// bits alone (two 8-bit passes for up to 65536 bins) then leaves each bin's
// ids in depth order, ties by id, so the low bits never need sorting.  The
// rasteriser streams its coarse bin's list in depth order and keeps the
// entries whose tile rectangle contains its tile, which is exactly the
// per-tile depth-ordered list.
//
// The radix sort (sort.hip) is LSD with 8-bit digits and stable ranks.
#include <algorithm>
#include <mutex>

#include "tg_internal.h"

namespace {

// ---- coarse-bin key emission ---------------------------------------------
// A block takes EMIT_RANKS consecutive depth ranks of one view.  Global
// loads and stores are item-major (rank = block base + item * 256 + thread,
// coalesced); the write pass transposes through LDS so that thread t owns the
// EMIT_ITEMS consecutive ranks [8t, 8t + 8), making rank order (thread, item)
// order and one block-wide exclusive scan enough to place every pair.
constexpr int EMIT_ITEMS = 8;
constexpr int EMIT_RANKS = 256 * EMIT_ITEMS;
constexpr int EMIT_STAGE = EMIT_RANKS * 3;   // keys staged in the write pass's 24 KB of LDS
constexpr int DIRECT_BINS = 256;   // coarse bins per view for the direct placement
constexpr int DIRECT_WIN = 2048;   // pairs per LDS window of the direct placement

// Coarse-bin rectangle of Gaussian g's tile rectangle (empty when culled).
// Coarse rectangle of a tile rectangle r (all zero when r is empty or the id
// was invalid), counting its coarse bins into cnt.
__device__ __forceinline__ ushort4 coarse_of(ushort4 r, bool valid, int cshift, uint32_t& cnt) {
    if (!valid || !(r.z > r.x && r.w > r.y)) return make_ushort4(0, 0, 0, 0);
    const ushort4 c = make_ushort4((unsigned short)(r.x >> cshift), (unsigned short)(r.y >> cshift),
                                   (unsigned short)(((r.z - 1) >> cshift) + 1),
                                   (unsigned short)(((r.w - 1) >> cshift) + 1));
    cnt += (uint32_t)((c.z - c.x) * (c.w - c.y));
    return c;
}

// Block sum and exclusive prefix of one u32 per thread (256 threads).
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x, uint32_t* wsum, uint32_t& total) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t inc = wave_scan_add_u32(x);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t c = wsum[i];
        before += i < w ? c : 0u;
        total += c;
    }
    return before + inc - x;
}

// Coarse rectangles of every (view, Gaussian) packed in 16 bits (x0, x1 - 1,
// y0, y1 - 1 in 4 bits each; 0x0001 when empty), for views of at most 16 x 16
// coarse bins: 2 MB per view at 1M Gaussians, small enough for the count
// pass's random gathers to stay in one XCD's L2 (8-byte tile rectangles are
// 8 MB per view).
constexpr uint16_t CRECT_EMPTY = 0x0001;

__device__ __forceinline__ uint32_t pack_crect(uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1, int cshift) {
    if (!(x1 > x0 && y1 > y0)) return CRECT_EMPTY;
    return (x0 >> cshift) | (((x1 - 1) >> cshift) << 4) | ((y0 >> cshift) << 8) | (((y1 - 1) >> cshift) << 12);
}

// VEC: four rectangles (two 16-byte loads) to one 8-byte store per thread
// (rect 16-byte aligned); the scalar form handles the rest.
template <bool VEC>
__global__ void __launch_bounds__(256) k_pack_crect(const ushort4* __restrict__ rect, int64_t VN, int cshift,
                                                    uint16_t* __restrict__ crect)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i0 = 0;
    if (VEC) {
        const int64_t nq = VN >> 2;
        const uint4* r4 = (const uint4*)rect;
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nq; q += stride) {
            const uint4 a = r4[2 * q], b = r4[2 * q + 1];
            const uint32_t p0 = pack_crect(a.x & 0xFFFFu, a.x >> 16, a.y & 0xFFFFu, a.y >> 16, cshift);
            const uint32_t p1 = pack_crect(a.z & 0xFFFFu, a.z >> 16, a.w & 0xFFFFu, a.w >> 16, cshift);
            const uint32_t p2 = pack_crect(b.x & 0xFFFFu, b.x >> 16, b.y & 0xFFFFu, b.y >> 16, cshift);
            const uint32_t p3 = pack_crect(b.z & 0xFFFFu, b.z >> 16, b.w & 0xFFFFu, b.w >> 16, cshift);
            ((uint2*)crect)[q] = make_uint2(p0 | (p1 << 16), p2 | (p3 << 16));
        }
        i0 = nq << 2;
    }
    for (int64_t i = i0 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < VN; i += stride) {
        const ushort4 r = rect[i];
        crect[i] = (uint16_t)pack_crect(r.x, r.y, r.z, r.w, cshift);
    }
}

__device__ __forceinline__ ushort4 unpack_crect(uint16_t p, uint32_t& cnt) {
    const unsigned x0 = p & 15u, x1 = (p >> 4) & 15u, y0 = (p >> 8) & 15u, y1 = (p >> 12) & 15u;
    if (x0 > x1) return make_ushort4(0, 0, 0, 0);   // empty
    cnt += (x1 + 1 - x0) * (y1 + 1 - y0);
    return make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)(x1 + 1), (unsigned short)(y1 + 1));
}

// Count pass: gathers each rank's coarse rectangle (the one random access of
// the emission), stores it in rank order for the write pass (unless PACKED:
// the placement then gathers the 2-byte form again from L2), and records the
// block's pair count -- or, for the direct placement (HIST), the block's pair
// count per coarse bin of its view, as the column hist[bin][block] of a
// bin-major matrix.  PACKED: the rectangles come from the 16-bit packed array
// and the blocks are remapped so that each XCD takes a contiguous range of
// views (launched as one dimension of nblk x V blocks, rounded up to 8).
template <bool HIST, bool PACKED>
__global__ void __launch_bounds__(256) k_emit_count(const uint32_t* __restrict__ order, const ushort4* __restrict__ rect,
                                                    const uint16_t* __restrict__ crect, int64_t N, int V,
                                                    int cshift, int nblk, GridPack gp, ushort4* __restrict__ crs,
                                                    uint16_t* __restrict__ prk, uint32_t* __restrict__ counts,
                                                    unsigned long long* __restrict__ n_pairs)
{
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t hist[HIST ? DIRECT_BINS : 1];
    int v, blk;
    if (PACKED) {
        const int64_t b = blockIdx.x;
        const int64_t per_xcd = (int64_t)gridDim.x >> 3;
        const int64_t Lb = (b & 7) * per_xcd + (b >> 3);
        if (Lb >= (int64_t)nblk * V) return;   // block-uniform
        v = (int)(Lb / nblk);
        blk = (int)(Lb - (int64_t)v * nblk);
    } else {
        v = blockIdx.y;
        blk = blockIdx.x;
    }
    const int t = threadIdx.x;
    const int64_t vN = (int64_t)v * N;
    const int64_t base = (int64_t)blk * EMIT_RANKS + t;
    const int cw = gp.cx[v], nbv = gp.cx[v] * gp.cy[v];
    if (HIST) {
        for (int c = t; c < nbv; c += 256) hist[c] = 0;
        __syncthreads();
    }
    uint32_t cnt = 0;
    if (PACKED) {
        // every id, then every gather, in flight before the first use
        uint32_t g[EMIT_ITEMS];
        uint16_t pk[EMIT_ITEMS];
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) g[i] = base + i * 256 < N ? order[vN + base + i * 256] : 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) pk[i] = g[i] < (uint64_t)N ? crect[vN + g[i]] : CRECT_EMPTY;
        // the gathered rectangles in rank order (coalesced): the placement
        // reads them back instead of gathering again
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i)
            if (base + i * 256 < N) prk[vN + base + i * 256] = pk[i];
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) {
            const ushort4 c = unpack_crect(pk[i], cnt);
            if (HIST)
                for (int y = c.y; y < c.w; ++y)
                    for (int x = c.x; x < c.z; ++x) atomicAdd(&hist[y * cw + x], 1u);
        }
    } else {
        // every id, then every rectangle, in flight before the first store
        // (a store between them would make each load wait for the one before)
        uint32_t g[EMIT_ITEMS];
        ushort4 c[EMIT_ITEMS];
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) g[i] = base + i * 256 < N ? order[vN + base + i * 256] : 0xFFFFFFFFu;
        ushort4 r[EMIT_ITEMS];
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) r[i] = rect[vN + (g[i] < (uint64_t)N ? g[i] : 0u)];
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) c[i] = coarse_of(r[i], g[i] < (uint64_t)N, cshift, cnt);
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) {
            const int64_t k = base + i * 256;
            if (k < N) {
                crs[vN + k] = c[i];
                if (HIST)
                    for (int y = c[i].y; y < c[i].w; ++y)
                        for (int x = c[i].x; x < c[i].z; ++x) atomicAdd(&hist[y * cw + x], 1u);
            }
        }
    }
    uint32_t total;
    (void)block_excl_scan_u32(cnt, wsum, total);
    if (HIST) {
        for (int c = t; c < nbv; c += 256)
            counts[(int64_t)(gp.cell_off[v] + c) * nblk + blk] = hist[c];
    } else if (t == 0) {
        counts[(int64_t)v * nblk + blk] = total;
    }
    if (t == 0 && total) atomicAdd(n_pairs, (unsigned long long)total);
}

// Direct placement: the block's pairs, already in (view, depth rank) order,
// are sorted by coarse bin inside the block (stable, in LDS, a window of
// DIRECT_WIN pairs at a time) and written straight to their final places in
// cell_ids: offsets[bin][block] (the scanned count matrix) is where the
// block's run of each bin starts.  This replaces a global radix sort of the
// pair keys.  Within a window, wave w ranks items [w*1024, w*1024+1024) in
// rounds of 64 consecutive items by ballot matching on the bin (stable), the
// window is placed bin-major in LDS and then written out as contiguous runs.
// The rectangles come in rank order: 8-byte coarse rectangles (crs), or with
// PACKED the 16-bit packed ones the count pass stored (crect, [V*N]).
template <bool PACKED>
__global__ void __launch_bounds__(256) k_emit_place(const uint32_t* __restrict__ order, const ushort4* __restrict__ crs,
                                                    const uint16_t* __restrict__ crect, int64_t N, int V, GridPack gp,
                                                    int nblk, const uint32_t* __restrict__ offsets,
                                                    uint32_t* __restrict__ cell_ids,
                                                    const int32_t* __restrict__ overflow)
{
    // 24 KB: the rank-major transpose of ids and rectangles, then the
    // window's ids (8 KB) and bins (2 KB)
    __shared__ uint4 lds[EMIT_RANKS * 12 / 16];
    __shared__ uint32_t sid[DIRECT_WIN];        // window sorted by bin
    __shared__ uint8_t sbin[DIRECT_WIN];
    __shared__ uint16_t cnt[4][DIRECT_BINS];    // per wave and bin (< DIRECT_WIN)
    __shared__ uint32_t boff[DIRECT_BINS];      // global start of the block's next pair per bin
    __shared__ uint32_t gofs[DIRECT_BINS];      // global position minus window position, per bin
    __shared__ uint32_t wsum[4];
    if (*overflow) return;   // block-uniform: the caller re-sizes and retries
    int v, blk;
    if (PACKED) {
        // each XCD takes a contiguous range of views (its L2 holds their
        // packed rectangles), as in the count pass
        const int64_t b = blockIdx.x;
        const int64_t per_xcd = (int64_t)gridDim.x >> 3;
        const int64_t Lb = (b & 7) * per_xcd + (b >> 3);
        if (Lb >= (int64_t)nblk * V) return;   // block-uniform
        v = (int)(Lb / nblk);
        blk = (int)(Lb - (int64_t)v * nblk);
    } else {
        v = blockIdx.y;
        blk = blockIdx.x;
    }
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int64_t vN = (int64_t)v * N;
    const int64_t rbase = (int64_t)blk * EMIT_RANKS;
    uint32_t* sg = (uint32_t*)lds;
    ushort4* sc = (ushort4*)(lds + EMIT_RANKS / 4);
    const int cw = gp.cx[v], nbv = gp.cx[v] * gp.cy[v];
    {
        // every load in flight before the first LDS store (a load followed by
        // its store, item by item, waits out each round trip)
        uint32_t og[EMIT_ITEMS];
        ushort4 oc[PACKED ? 1 : EMIT_ITEMS];
        const uint32_t bo = t < nbv ? offsets[(int64_t)(gp.cell_off[v] + t) * nblk + blk] : 0u;
        if (rbase + EMIT_RANKS <= N) {
#pragma unroll
            for (int i = 0; i < EMIT_ITEMS; ++i) og[i] = order[vN + rbase + i * 256 + t];
            if (!PACKED) {
#pragma unroll
                for (int i = 0; i < EMIT_ITEMS; ++i) oc[i] = crs[vN + rbase + i * 256 + t];
            }
        } else {
#pragma unroll
            for (int i = 0; i < EMIT_ITEMS; ++i) {
                const bool in = rbase + i * 256 + t < N;
                og[i] = in ? order[vN + rbase + i * 256 + t] : 0xFFFFFFFFu;
                if (!PACKED) oc[i] = in ? crs[vN + rbase + i * 256 + t] : make_ushort4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) {
            sg[i * 256 + t] = og[i];
            if (!PACKED) sc[i * 256 + t] = oc[i];
        }
        if (t < nbv) boff[t] = bo;   // nbv <= DIRECT_BINS = 256 = the block size
    }
    __syncthreads();
    uint32_t gid[EMIT_ITEMS];
    ushort4 cr[EMIT_ITEMS];
    {
        const uint4 a = lds[2 * t], b = lds[2 * t + 1];
        gid[0] = a.x; gid[1] = a.y; gid[2] = a.z; gid[3] = a.w;
        gid[4] = b.x; gid[5] = b.y; gid[6] = b.z; gid[7] = b.w;
    }
    uint32_t mine = 0;
    uint16_t pkr[EMIT_ITEMS];
    if (PACKED) {
        // the count pass stored each rank's packed rectangle in rank order;
        // ranks past the end hold no pairs
        const int64_t r0 = rbase + EMIT_ITEMS * t;
        if (r0 + EMIT_ITEMS <= N && ((vN + r0) & 7) == 0) {
            const uint4 q = *(const uint4*)(crect + vN + r0);
            pkr[0] = (uint16_t)q.x; pkr[1] = (uint16_t)(q.x >> 16);
            pkr[2] = (uint16_t)q.y; pkr[3] = (uint16_t)(q.y >> 16);
            pkr[4] = (uint16_t)q.z; pkr[5] = (uint16_t)(q.z >> 16);
            pkr[6] = (uint16_t)q.w; pkr[7] = (uint16_t)(q.w >> 16);
        } else {
#pragma unroll
            for (int i = 0; i < EMIT_ITEMS; ++i) pkr[i] = r0 + i < N ? crect[vN + r0 + i] : CRECT_EMPTY;
        }
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) cr[i] = unpack_crect(pkr[i], mine);
    } else {
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) {
            cr[i] = sc[EMIT_ITEMS * t + i];
            mine += (uint32_t)((cr[i].z - cr[i].x) * (cr[i].w - cr[i].y));
        }
    }
    uint32_t total;
    const uint32_t before = block_excl_scan_u32(mine, wsum, total);
    // PACKED keeps the ids and packed rectangles of every rank, and each
    // thread's first pair, in LDS for the balanced expansion below:
    // [0, 8 KB) ids by rank, [8, 12) rectangles by rank, [12, 13) starts,
    // then the window (ids 8 KB, bins 2 KB).  Otherwise the window reuses
    // the transpose area.
    constexpr int P_PK = EMIT_RANKS / 4, P_TST = P_PK + EMIT_RANKS / 8, P_WID = P_TST + 256 / 4;
    constexpr int P_WBIN = P_WID + DIRECT_WIN / 4;
    static_assert(P_WBIN + DIRECT_WIN / 16 <= EMIT_RANKS * 12 / 16, "LDS layout of the packed placement");
    static_assert(DIRECT_WIN / 256 == 8, "the balanced expansion stages 8 pairs per thread");
    uint16_t* pkl = (uint16_t*)(lds + P_PK);
    uint32_t* tst = (uint32_t*)(lds + P_TST);
    uint32_t* wid = PACKED ? (uint32_t*)(lds + P_WID) : (uint32_t*)lds;               // [DIRECT_WIN]
    uint8_t* wbin = PACKED ? (uint8_t*)(lds + P_WBIN) : (uint8_t*)(lds + DIRECT_WIN / 4);   // [DIRECT_WIN]
    if (PACKED) {
        // (the ids by rank in sg stay where the load phase put them)
        const uint4 pv = make_uint4(pkr[0] | ((uint32_t)pkr[1] << 16), pkr[2] | ((uint32_t)pkr[3] << 16),
                                    pkr[4] | ((uint32_t)pkr[5] << 16), pkr[6] | ((uint32_t)pkr[7] << 16));
        ((uint4*)pkl)[t] = pv;
        tst[t] = before;
    }
    const uint64_t lt = lanemask_lt();
    for (uint32_t w0 = 0; w0 < total; w0 += DIRECT_WIN) {
        __syncthreads();   // the previous window's LDS is free
        if (PACKED) {
            // Balanced expansion: thread t writes window pairs [8t, 8t + 8)
            // (pair order = rank order, then bin rows, then columns): find
            // the owning thread (the last whose first pair is <= p0; equal
            // starts belong to threads with no pairs before it), walk its
            // ranks to the pair, then step through pairs and ranks.  Every
            // lane does the same few steps, instead of each lane looping
            // over its own rectangles (as long as the largest of the wave).
            const uint32_t lim = total - w0 < DIRECT_WIN ? total - w0 : DIRECT_WIN;
            const uint32_t q0 = (uint32_t)t * (DIRECT_WIN / 256);
            if (q0 < lim) {
                const uint32_t p0 = w0 + q0;
                int lo = 0;
#pragma unroll
                for (int step = 128; step > 0; step >>= 1)
                    if (tst[lo + step] <= p0) lo += step;
                int r = lo * EMIT_ITEMS;
                uint32_t off = p0 - tst[lo];
                uint32_t pk = pkl[r];
                uint32_t np = 0;
                unpack_crect((uint16_t)pk, np);
                while (off >= np) {   // ends inside the owner's ranks
                    off -= np;
                    pk = pkl[++r];
                    np = 0;
                    unpack_crect((uint16_t)pk, np);
                }
                uint32_t x0 = pk & 15u, x1 = (pk >> 4) & 15u, y1 = (pk >> 12) & 15u;
                const uint32_t wdt = x1 + 1 - x0;
                // off < 256 and wdt <= 16: the reciprocal's error cannot
                // cross an integer ((off + 1/2) / wdt is >= 1/32 away from one)
                uint32_t dy = (uint32_t)(((float)off + 0.5f) * __builtin_amdgcn_rcpf((float)wdt));
                uint32_t x = x0 + (off - dy * wdt), y = ((pk >> 8) & 15u) + dy;
                uint32_t gcur = sg[r];
                const uint32_t qn = lim - q0 < (uint32_t)(DIRECT_WIN / 256) ? lim - q0 : (uint32_t)(DIRECT_WIN / 256);
                // the thread's 8 pairs go out as two 16-byte and one 8-byte
                // LDS store (8 scattered words per lane would hit the same
                // banks 16 ways); slots past qn hold junk the ranking never
                // reads (it stops at the window's pair count)
                uint32_t ids[DIRECT_WIN / 256];
                uint32_t bins2[2] = {0u, 0u};
#pragma unroll
                for (int j = 0; j < DIRECT_WIN / 256; ++j) ids[j] = 0u;
#pragma unroll
                for (uint32_t j = 0; j < (uint32_t)(DIRECT_WIN / 256); ++j) {
                    if (j >= qn) break;
                    ids[j] = gcur;
                    bins2[j >> 2] |= (y * cw + x) << (8 * (j & 3));
                    if (j + 1 == qn) break;
                    if (++x > x1) {
                        x = x0;
                        if (++y > y1) {
                            // next rank with pairs (one exists: more pairs follow)
                            do {
                                pk = pkl[++r];
                            } while ((pk & 15u) > ((pk >> 4) & 15u));
                            x0 = pk & 15u;
                            x1 = (pk >> 4) & 15u;
                            y1 = (pk >> 12) & 15u;
                            x = x0;
                            y = (pk >> 8) & 15u;
                            gcur = sg[r];
                        }
                    }
                }
                ((uint4*)wid)[q0 / 4] = make_uint4(ids[0], ids[1], ids[2], ids[3]);
                ((uint4*)wid)[q0 / 4 + 1] = make_uint4(ids[4], ids[5], ids[6], ids[7]);
                ((uint2*)wbin)[q0 / 8] = make_uint2(bins2[0], bins2[1]);
            }
        } else {
            uint32_t pidx = before;
#pragma unroll
            for (int i = 0; i < EMIT_ITEMS; ++i) {
                const ushort4 c = cr[i];
                for (int y = c.y; y < c.w; ++y)
                    for (int x = c.x; x < c.z; ++x, ++pidx)
                        if (pidx >= w0 && pidx < w0 + DIRECT_WIN) {
                            wid[pidx - w0] = gid[i];
                            wbin[pidx - w0] = (uint8_t)(y * cw + x);
                        }
            }
        }
        for (int k = t; k < 4 * DIRECT_BINS; k += 256) (&cnt[0][0])[k] = 0;
        __syncthreads();
        const uint32_t nwin = total - w0 < DIRECT_WIN ? total - w0 : DIRECT_WIN;
        uint32_t lrank[DIRECT_WIN / 256];
#pragma unroll
        for (int r = 0; r < DIRECT_WIN / 256; ++r) {
            const uint32_t idx = (uint32_t)(w * (DIRECT_WIN / 4) + r * 64 + lane);
            const bool act = idx < nwin;
            const uint32_t d = act ? wbin[idx] : 0u;
            const uint64_t m = match_digit8(d, act);
            const uint32_t rk = (uint32_t)__popcll(m & lt);
            const uint32_t b0 = act ? cnt[w][d] : 0u;
            lrank[r] = b0 + rk;
            if (act && rk == 0) cnt[w][d] = (uint16_t)(b0 + (uint32_t)__popcll(m));
        }
        __syncthreads();
        {
            // thread t owns bin t: window-local start (exclusive scan over
            // bins), the waves' starts inside it, and the global offset
            const int c = t;
            uint32_t cw4[4], tot = 0;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                cw4[ww] = cnt[ww][c];
                tot += cw4[ww];
            }
            uint32_t all;
            const uint32_t start = block_excl_scan_u32(tot, wsum, all);
            uint32_t run = start;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                cnt[ww][c] = (uint16_t)run;
                run += cw4[ww];
            }
            if (c < nbv) {
                gofs[c] = boff[c] - start;
                boff[c] += tot;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < DIRECT_WIN / 256; ++r) {
            const uint32_t idx = (uint32_t)(w * (DIRECT_WIN / 4) + r * 64 + lane);
            if (idx < nwin) {
                const uint32_t d = wbin[idx];
                const uint32_t sp = cnt[w][d] + lrank[r];
                sid[sp] = wid[idx];
                sbin[sp] = (uint8_t)d;
            }
        }
        __syncthreads();
        for (uint32_t i = t; i < nwin; i += 256) cell_ids[gofs[sbin[i]] + i] = sid[i];
    }
}

// Bin ranges of the direct placement from the scanned count matrix: bin c
// starts where its first block's run starts.
__global__ void k_bin_ranges(const uint32_t* __restrict__ offsets, int nblk, int64_t ncell,
                             const int64_t* __restrict__ n_pairs, int64_t capacity, uint2* __restrict__ ranges)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = *n_pairs;
    if (c >= ncell || n > capacity) return;
    const uint32_t start = offsets[c * nblk];
    const uint32_t end = c + 1 < ncell ? offsets[(c + 1) * nblk] : (uint32_t)n;
    ranges[c] = make_uint2(start, end);
}

// Write pass: the same ranks, coarse rectangles read back in rank order.
__global__ void __launch_bounds__(256) k_emit_write(const uint32_t* __restrict__ order, const ushort4* __restrict__ crs,
                                                    int64_t N, GridPack gp, int rbits, int nblk,
                                                    const uint32_t* __restrict__ offsets, uint32_t* __restrict__ keys,
                                                    int64_t capacity, const int32_t* __restrict__ overflow)
{
    // 24 KB: ids then coarse rectangles, rank-major; reused to stage keys
    __shared__ uint4 lds[EMIT_RANKS * 12 / 16];
    __shared__ uint32_t wsum[4];
    uint4* sg4 = lds;
    ushort4* sc = (ushort4*)(lds + EMIT_RANKS / 4);
    uint32_t* stage = (uint32_t*)lds;
    if (*overflow) return;   // block-uniform: the caller re-sizes and retries
    const int v = blockIdx.y, t = threadIdx.x;
    const int64_t vN = (int64_t)v * N;
    const int64_t base = (int64_t)blockIdx.x * EMIT_RANKS;
    uint32_t* sg = (uint32_t*)sg4;
#pragma unroll
    for (int i = 0; i < EMIT_ITEMS; ++i) {
        const int j = i * 256 + t;
        const bool in = base + j < N;
        sg[j] = in ? order[vN + base + j] : 0u;
        sc[j] = in ? crs[vN + base + j] : make_ushort4(0, 0, 0, 0);
    }
    __syncthreads();
    uint32_t gid[EMIT_ITEMS];
    ushort4 cr[EMIT_ITEMS];
    {
        const uint4 a = sg4[2 * t], b = sg4[2 * t + 1];
        gid[0] = a.x; gid[1] = a.y; gid[2] = a.z; gid[3] = a.w;
        gid[4] = b.x; gid[5] = b.y; gid[6] = b.z; gid[7] = b.w;
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < EMIT_ITEMS; ++i) {
        cr[i] = sc[EMIT_ITEMS * t + i];
        cnt += (uint32_t)((cr[i].z - cr[i].x) * (cr[i].w - cr[i].y));
    }
    uint32_t total;
    const uint32_t before = block_excl_scan_u32(cnt, wsum, total);
    const uint64_t off = (uint64_t)offsets[(int64_t)v * nblk + blockIdx.x];
    if (off + total > (uint64_t)capacity) return;   // unreachable without overflow
    const int cw = gp.cx[v];
    const uint32_t cbase = (uint32_t)gp.cell_off[v];
    if (total <= EMIT_STAGE) {
        // stage the block's keys in LDS (its ids and rectangles are in
        // registers now), then write them out contiguously
        __syncthreads();
        uint32_t pos = before;
#pragma unroll
        for (int i = 0; i < EMIT_ITEMS; ++i) {
            const ushort4 c = cr[i];
            for (int y = c.y; y < c.w; ++y)
                for (int x = c.x; x < c.z; ++x) stage[pos++] = ((cbase + (uint32_t)(y * cw + x)) << rbits) | gid[i];
        }
        __syncthreads();
        for (uint32_t j = t; j < total; j += 256) keys[off + j] = stage[j];
        return;
    }
    uint64_t pos = off + before;
#pragma unroll
    for (int i = 0; i < EMIT_ITEMS; ++i) {
        const ushort4 c = cr[i];
        for (int y = c.y; y < c.w; ++y)
            for (int x = c.x; x < c.z; ++x) keys[pos++] = ((cbase + (uint32_t)(y * cw + x)) << rbits) | gid[i];
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}
__global__ void k_zero_counters(unsigned long long* n_pairs, int32_t* overflow) {
    *n_pairs = 0ull;
    *overflow = 0;
}
__global__ void k_check_overflow(const unsigned long long* n_pairs, int64_t capacity, int32_t* overflow) {
    if (*n_pairs > (unsigned long long)capacity) *overflow = 1;
}

// Ids and bin ranges from the sorted keys; each thread takes four
// consecutive keys (one 16-byte load from the 256-byte aligned workspace).
__global__ void __launch_bounds__(256) k_cell_finalize(const uint32_t* __restrict__ skeys,
                                                       const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                       int rbits, int64_t N, uint32_t* __restrict__ cell_ids,
                                                       uint2* __restrict__ ranges, int64_t ncell)
{
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    int64_t n = *n_pairs;
    if (n > capacity) n = 0;
    if (i0 >= n) return;
    uint32_t k[6];   // k[0] = key i0 - 1, k[1..4] = keys i0..i0+3, k[5] = key i0 + 4
    if (i0 + 4 <= n) {
        const uint4 q = *(const uint4*)(skeys + i0);
        k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < n ? skeys[i0 + j] : 0u;
    }
    k[0] = i0 > 0 ? skeys[i0 - 1] : 0u;
    k[5] = i0 + 4 < n ? skeys[i0 + 4] : 0u;
    const uint32_t mask = (1u << rbits) - 1u;
#pragma unroll
    for (int j = 1; j <= 4; ++j) {
        const int64_t i = i0 + j - 1;
        if (i >= n) break;
        const uint32_t cell = k[j] >> rbits;
        const uint32_t id = k[j] & mask;
        if (cell >= (uint64_t)ncell || id >= (uint64_t)N) continue;  // consistent keys never hit this
        cell_ids[i] = id;
        if (i == 0 || (k[j - 1] >> rbits) != cell) ranges[cell].x = (uint32_t)i;
        if (i == n - 1 || (k[j + 1] >> rbits) != cell) ranges[cell].y = (uint32_t)(i + 1);
    }
}

inline int bitlen(uint64_t x) {  // number of bits to represent x-1 values [0, x)
    int b = 0;
    while (b < 63 && (1ull << b) < x) ++b;
    return b < 1 ? 1 : b;
}

struct BinPlan {
    int cshift, rbits, cbits, passes;
    int64_t ncell;
    GridPack gp;
};

tg_status plan_bins(const tg_camera* cams, int V, int64_t N, const tg_params* p, BinPlan* bp) {
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    int cs = p->coarse_shift < 0 ? 0 : p->coarse_shift;
    bp->rbits = bitlen((uint64_t)N);
    for (;; ++cs) {
        bp->ncell = fill_grid(cams, V, cs, &bp->gp);
        bp->cbits = bitlen((uint64_t)bp->ncell);
        if (bp->rbits + bp->cbits <= 32) break;
        if (cs > 12) return TG_ERR_UNSUPPORTED;
    }
    bp->cshift = cs;
    bp->passes = (bp->cbits + 7) / 8;   // the id bits are already in order
    return TG_OK;
}

// workspace layout
struct BinWs {
    uint32_t *dk_a, *dv_a, *dk_b, *dv_b;   // depth sort ping-pong [V*N]
    uint32_t *pk_a, *pk_b;                  // pair keys [capacity]
    uint32_t* counts;                       // per emission block pair counts [V*nblk]
    void* scratch;
    size_t bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

BinWs layout_ws(void* ws, int64_t N, int V, int64_t capacity) {
    BinWs L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    size_t vn = (size_t)V * (size_t)N * 4;
    // dk_a and dv_a are adjacent: after the depth sort the emission reuses
    // them as one [V*N] array of 8-byte coarse rectangles
    size_t a = take(vn), b = take(vn), c = take(vn), d = take(vn);
    size_t e = take((size_t)capacity * 4), f = take((size_t)capacity * 4);
    const int64_t ncount = (int64_t)V * ((N + EMIT_RANKS - 1) / EMIT_RANKS);
    size_t h = take((size_t)ncount * 4);
    size_t sc = tg_sort_scratch_bytes(N, V);
    size_t sc2 = tg_sort_scratch_bytes(capacity, 1);
    size_t g = take(sc > sc2 ? sc : sc2);
    char* base = (char*)ws;
    L.dk_a = (uint32_t*)(base + a);
    L.dv_a = (uint32_t*)(base + b);
    L.dk_b = (uint32_t*)(base + c);
    L.dv_b = (uint32_t*)(base + d);
    L.pk_a = (uint32_t*)(base + e);
    L.pk_b = (uint32_t*)(base + f);
    L.counts = (uint32_t*)(base + h);
    L.scratch = base + g;
    L.bytes = o;
    return L;
}

}  // namespace

extern "C" int64_t tg_num_cells(const tg_camera* cams, int32_t V, int64_t N, const tg_params* p) {
    if (!cams || !p || V < 1 || V > TG_MAX_VIEWS || N < 0) return -1;
    BinPlan bp;
    if (plan_bins(cams, V, N > 0 ? N : 1, p, &bp) != TG_OK) return -1;
    return bp.ncell;
}

extern "C" int64_t tg_num_tiles(const tg_camera* cams, int32_t V) {
    if (!cams || V < 1) return -1;
    int64_t t = 0;
    for (int v = 0; v < V; ++v) t += (int64_t)ceil_div(cams[v].width, TG_TILE) * ceil_div(cams[v].height, TG_TILE);
    return t;
}

extern "C" tg_status tg_bin_sort(const tg_splats* sp, int64_t N, const tg_camera* cams, int32_t V,
                                 const tg_params* p, tg_bins* bins, void* ws, size_t* ws_bytes, void* stream)
{
    if (!sp || !cams || !p || !bins || !ws_bytes || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (N > (int64_t)0xFFFFFFFF || bins->capacity < 0 || bins->capacity > (int64_t)0xFFFFFFFF)
        return TG_ERR_UNSUPPORTED;
    BinPlan bp;
    tg_status st = plan_bins(cams, V, N > 0 ? N : 1, p, &bp);
    if (st != TG_OK) return st;
    BinWs L = layout_ws(nullptr, N, V, bins->capacity);
    if (!ws) {
        *ws_bytes = L.bytes;
        return TG_OK;
    }
    if (*ws_bytes < L.bytes) return TG_ERR_WORKSPACE;
    if (!sp->key || !sp->rect || !bins->order || !bins->cell_ids || !bins->cell_ranges || !bins->n_pairs ||
        !bins->overflow)
        return TG_ERR_INVALID_ARG;
    L = layout_ws(ws, N, V, bins->capacity);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(1), 0, s, (unsigned long long*)bins->n_pairs, bins->overflow);
    {
        int64_t n = 2 * bp.ncell;
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bins->cell_ranges, n, 0u);
    }
    TG_CHECK_LAUNCH();
    if (N == 0) return TG_OK;
    // (1) depth order per view: 4 passes over the 32-bit depth keys
    st = tg_radix_sort(sp->key, nullptr, L.dk_a, L.dv_a, L.dk_b, L.dv_b, nullptr, bins->order, N, V, nullptr, 0, 4,
                    L.scratch, s);
    if (st != TG_OK) return st;
    // (2) emit the (coarse bin, Gaussian) pairs in (view, depth rank) order
    const int nblk = (int)((N + EMIT_RANKS - 1) / EMIT_RANKS);
    // coarse rectangles in rank order reuse the depth sort's first ping-pong
    // pair (8 B per (view, Gaussian) over two contiguous 4 B arrays)
    ushort4* crs = (ushort4*)L.dk_a;
    int max_bins = 0;
    for (int v = 0; v < V; ++v) max_bins = std::max(max_bins, bp.gp.cx[v] * bp.gp.cy[v]);
    const int64_t nmat = bp.ncell * (int64_t)nblk;
    if (max_bins <= DIRECT_BINS && nmat <= bins->capacity && nmat <= ((int64_t)1 << 26)) {
        // direct placement: per-(bin, block) counts, one scan, then each
        // block sorts its pairs by bin in LDS and writes the final lists
        uint32_t* mat = L.pk_a;   // [ncell][nblk], free on this path
        uint16_t* crect = nullptr;
        uint16_t* prk = nullptr;
        bool packed = false;
        int max_cx = 0, max_cy = 0;
        for (int v = 0; v < V; ++v) {
            max_cx = std::max(max_cx, bp.gp.cx[v]);
            max_cy = std::max(max_cy, bp.gp.cy[v]);
        }
        if (max_cx <= 16 && max_cy <= 16) {
            // packed coarse rectangles in the depth sort's second ping-pong
            // pair (free after the sort; 2 B of its 8 B per (view, Gaussian))
            crect = (uint16_t*)L.dk_b;
            const int64_t VN = (int64_t)V * N;
            const bool vec = (((uintptr_t)sp->rect) & 15u) == 0;
            const int64_t pgrid = std::min<int64_t>(((vec ? VN / 4 : VN) + 255) / 256, 65536);
            if (vec)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pack_crect<true>), dim3((unsigned)std::max<int64_t>(pgrid, 1)),
                                   dim3(256), 0, s, (const ushort4*)sp->rect, VN, bp.cshift, crect);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pack_crect<false>), dim3((unsigned)pgrid), dim3(256), 0, s,
                                   (const ushort4*)sp->rect, VN, bp.cshift, crect);
            const int64_t per_xcd = ((int64_t)nblk * V + 7) / 8;
            // packed rectangles in rank order for the placement: the depth
            // sort's first ping-pong key array (free once the order is out)
            prk = (uint16_t*)L.dk_a;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_emit_count<true, true>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0,
                               s, bins->order, (const ushort4*)sp->rect, (const uint16_t*)crect, N, V, bp.cshift,
                               nblk, bp.gp, crs, prk, mat, (unsigned long long*)bins->n_pairs);
            packed = true;
        } else {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_emit_count<true, false>), dim3((unsigned)nblk, V), dim3(256), 0, s,
                               bins->order, (const ushort4*)sp->rect, (const uint16_t*)nullptr, N, V, bp.cshift,
                               nblk, bp.gp, crs, (uint16_t*)nullptr, mat, (unsigned long long*)bins->n_pairs);
        }
        hipLaunchKernelGGL(k_check_overflow, dim3(1), dim3(1), 0, s, (const unsigned long long*)bins->n_pairs,
                           bins->capacity, bins->overflow);
        // with no overflow the total fits the capacity (< 2^32): u32 offsets
        tg_exclusive_scan_u32(mat, nmat, (uint32_t*)L.scratch, s);
        if (packed) {
            const int64_t per_xcd = ((int64_t)nblk * V + 7) / 8;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_emit_place<true>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0, s,
                               bins->order, (const ushort4*)nullptr, (const uint16_t*)prk, N, V, bp.gp, nblk, mat,
                               bins->cell_ids, bins->overflow);
        } else {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_emit_place<false>), dim3((unsigned)nblk, V), dim3(256), 0, s,
                               bins->order, (const ushort4*)crs, (const uint16_t*)nullptr, N, V, bp.gp, nblk, mat,
                               bins->cell_ids, bins->overflow);
        }
        hipLaunchKernelGGL(k_bin_ranges, dim3((unsigned)((bp.ncell + 255) / 256)), dim3(256), 0, s, mat, nblk,
                           bp.ncell, bins->n_pairs, bins->capacity, (uint2*)bins->cell_ranges);
        TG_CHECK_LAUNCH();
        return TG_OK;
    }
    // general path: keys (coarse bin | Gaussian id) written in rank order,
    // then a stable radix sort over the bin bits
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_emit_count<false, false>), dim3((unsigned)nblk, V), dim3(256), 0, s,
                       bins->order, (const ushort4*)sp->rect, (const uint16_t*)nullptr, N, V, bp.cshift, nblk, bp.gp,
                       crs, (uint16_t*)nullptr, L.counts, (unsigned long long*)bins->n_pairs);
    hipLaunchKernelGGL(k_check_overflow, dim3(1), dim3(1), 0, s, (const unsigned long long*)bins->n_pairs,
                       bins->capacity, bins->overflow);
    // with no overflow the total fits the capacity (< 2^32), so u32 offsets
    tg_exclusive_scan_u32(L.counts, (int64_t)V * nblk, (uint32_t*)L.scratch, s);
    hipLaunchKernelGGL(k_emit_write, dim3((unsigned)nblk, V), dim3(256), 0, s, bins->order, (const ushort4*)crs, N,
                       bp.gp, bp.rbits, nblk, L.counts, L.pk_a, bins->capacity, bins->overflow);
    TG_CHECK_LAUNCH();
    if (bins->capacity == 0) return TG_OK;
    // (3) stable sort of the pair keys over the coarse-bin bits
    uint32_t* final_keys = (bp.passes & 1) ? L.pk_b : L.pk_a;
    st = tg_radix_sort(L.pk_a, nullptr, L.pk_b, nullptr, L.pk_a, nullptr, final_keys, nullptr, bins->capacity, 1,
                       bins->n_pairs, bp.rbits, bp.passes, L.scratch, s);
    if (st != TG_OK) return st;
    // (4) ranges and ids
    hipLaunchKernelGGL(k_cell_finalize, dim3((unsigned)((bins->capacity + 1023) / 1024)), dim3(256), 0, s, final_keys,
                       bins->n_pairs, bins->capacity, bp.rbits, N, bins->cell_ids, (uint2*)bins->cell_ranges,
                       bp.ncell);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

// ---- expansion of coarse lists into per-tile lists (tests / tools) -----------
namespace {
// One wave per tile: stream the coarse list, keep entries whose rectangle
// contains the tile.  mode 0 counts, mode 1 writes.
__global__ void __launch_bounds__(64) k_expand(const ushort4* __restrict__ rect, const uint32_t* __restrict__ cell_ids,
                                               const uint2* __restrict__ ranges, const int32_t* __restrict__ overflow,
                                               int64_t N, int V, GridPack gp, int cshift, uint32_t* __restrict__ counts,
                                               const uint32_t* __restrict__ starts, uint32_t* __restrict__ out,
                                               int64_t capacity, int mode)
{
    const int64_t tile = blockIdx.x;
    if (*overflow) {
        if (mode == 0 && threadIdx.x == 0) counts[tile] = 0;
        return;
    }
    int v = 0;
    while (v + 1 < V && gp.tile_off[v + 1] <= tile) ++v;
    const int lt = (int)(tile - gp.tile_off[v]);
    const int tx = lt % gp.tx[v], ty = lt / gp.tx[v];
    const uint32_t cell = (uint32_t)gp.cell_off[v] + (uint32_t)((ty >> cshift) * gp.cx[v] + (tx >> cshift));
    const uint2 rg = ranges[cell];
    const int l = threadIdx.x;
    const uint64_t lt_mask = lanemask_lt();
    uint32_t n = 0;
    uint32_t wpos = mode ? starts[tile] : 0u;
    for (uint32_t i0 = rg.x; i0 < rg.y; i0 += 64) {
        uint32_t i = i0 + l;
        bool hit = false;
        uint32_t g = 0;
        if (i < rg.y) {
            g = cell_ids[i];
            if (g < (uint64_t)N) {
                ushort4 r = rect[(int64_t)v * N + g];
                hit = tx >= r.x && tx < r.z && ty >= r.y && ty < r.w;
            }
        }
        uint64_t m = ballot64(hit);
        if (mode && hit) {
            uint64_t o = (uint64_t)wpos + n + (uint64_t)__popcll(m & lt_mask);
            if (o < (uint64_t)capacity) out[o] = g;
        }
        n += (uint32_t)__popcll(m);
    }
    if (mode == 0 && l == 0) counts[tile] = n;
}

__global__ void k_ranges_from_starts(const uint32_t* __restrict__ starts, const uint32_t* __restrict__ counts,
                                     int64_t T, uint2* __restrict__ ranges, int64_t capacity, int64_t* n_out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) ranges[t] = make_uint2(starts[t], starts[t] + counts[t]);
    if (t == T - 1) *n_out = (int64_t)starts[t] + counts[t];
}
}  // namespace

extern "C" tg_status tg_bin_expand(const tg_splats* sp, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                   int32_t V, const tg_params* p, uint32_t* tile_ids, uint32_t* tile_ranges,
                                   int64_t capacity, int64_t* n_out, void* ws, size_t* ws_bytes, void* stream)
{
    if (!sp || !bins || !cams || !p || !ws_bytes || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    BinPlan bp;
    tg_status st = plan_bins(cams, V, N > 0 ? N : 1, p, &bp);
    if (st != TG_OK) return st;
    const int64_t T = bp.gp.tile_off[V];
    size_t need = align256((size_t)T * 4) * 2 + tg_sort_scratch_bytes(T, 1) + 256;
    if (!ws) {
        *ws_bytes = need;
        return TG_OK;
    }
    if (*ws_bytes < need) return TG_ERR_WORKSPACE;
    if (!tile_ids || !tile_ranges || !n_out) return TG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* counts = (uint32_t*)ws;
    uint32_t* starts = (uint32_t*)((char*)ws + align256((size_t)T * 4));
    uint32_t* scr = (uint32_t*)((char*)ws + 2 * align256((size_t)T * 4));
    hipLaunchKernelGGL(k_expand, dim3((unsigned)T), dim3(64), 0, s, (const ushort4*)sp->rect, bins->cell_ids,
                       (const uint2*)bins->cell_ranges, bins->overflow, N, V, bp.gp, bp.cshift, counts, nullptr,
                       nullptr, (int64_t)0, 0);
    if (hipMemcpyAsync(starts, counts, (size_t)T * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return TG_ERR_DEVICE;
    tg_exclusive_scan_u32(starts, T, scr, s);
    hipLaunchKernelGGL(k_ranges_from_starts, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, starts, counts, T,
                       (uint2*)tile_ranges, capacity, n_out);
    TG_CHECK_LAUNCH();
    // Entries beyond `capacity` are dropped; *n_out reports the full count so
    // the caller can re-size (counts are deterministic).
    hipLaunchKernelGGL(k_expand, dim3((unsigned)T), dim3(64), 0, s, (const ushort4*)sp->rect, bins->cell_ids,
                       (const uint2*)bins->cell_ranges, bins->overflow, N, V, bp.gp, bp.cshift, counts, starts,
                       tile_ids, capacity, 1);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

// ---- tg_bin_sort_static: the same binning with a library-owned scratch -------
// For callers that cannot allocate device memory.  The workspace is a
// file-scope device array; each device holds its own copy at its own address,
// which is looked up once per device (hipGetSymbolAddress with that device
// current) and used from then on: the array's name is a host-side stand-in
// and must never reach a kernel.  tg_bin_sort writes every workspace word it
// reads within the call, so nothing carries over between calls.
namespace {
constexpr int STATIC_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[TG_BIN_SORT_STATIC_BYTES];
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEVICES];

tg_status static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TG_ERR_DEVICE;
    if (dev >= STATIC_MAX_DEVICES) return TG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TG_ERR_DEVICE;
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return TG_OK;
}
}  // namespace

extern "C" tg_status tg_bin_sort_static(const tg_splats* sp, int64_t N, const tg_camera* cams, int32_t V,
                                        const tg_params* p, tg_bins* bins, void* stream)
{
    size_t need = 0;
    tg_status st = tg_bin_sort(sp, N, cams, V, p, bins, nullptr, &need, stream);
    if (st != TG_OK) return st;
    if (need > (size_t)TG_BIN_SORT_STATIC_BYTES) return TG_ERR_WORKSPACE;
    void* ws = nullptr;
    st = static_scratch(&ws);
    if (st != TG_OK) return st;
    size_t have = (size_t)TG_BIN_SORT_STATIC_BYTES;
    return tg_bin_sort(sp, N, cams, V, p, bins, ws, &have, stream);
}
