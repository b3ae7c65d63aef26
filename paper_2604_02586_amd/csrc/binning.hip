// tg_bin_sort / tg_bin_expand: depth ordering and coarse binning
// (TrackerSplat Sec. 3.1: blending follows the Gaussians' depth order).
//
// Design for CDNA4: instead of sorting one 64-bit (tile | depth) key per
// (tile, Gaussian) pair -- about 16M pairs per 1080p view at 1M Gaussians --
// we (1) radix-sort the N depth keys of each view once, giving every Gaussian
// a depth rank, then (2) emit one 32-bit key (coarse bin | depth rank) per
// (coarse bin, Gaussian) pair, with coarse bins of 8x8 tiles, and radix-sort
// those (about 2M pairs per view).  The rasteriser streams its coarse bin's
// list in depth order and keeps the entries whose tile rectangle contains its
// tile, which is exactly the per-tile depth-ordered list.
//
// The radix sort (sort.hip) is LSD with 8-bit digits and stable ranks.
#include "tg_internal.h"

namespace {

// ---- coarse-bin key emission ---------------------------------------------
// Each thread takes EMIT_ITEMS depth ranks (strided by the block size, so the
// order/rect reads stay coalesced), the block reserves its output range with
// one atomic on the pair counter, and each thread writes its keys into its
// own sub-range.  Key order is irrelevant here: the keys are sorted next.
constexpr int EMIT_ITEMS = 8;

__global__ void __launch_bounds__(256) k_emit(const uint32_t* __restrict__ order, const ushort4* __restrict__ rect,
                                              int64_t N, int V, GridPack gp, int cshift, int rbits,
                                              uint32_t* __restrict__ keys, int64_t capacity,
                                              unsigned long long* __restrict__ n_pairs, int32_t* __restrict__ overflow)
{
    __shared__ unsigned long long gbase;
    __shared__ uint32_t wsum[4];
    const int v = blockIdx.y;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int64_t base = (int64_t)blockIdx.x * (256 * EMIT_ITEMS);
    ushort4 cr[EMIT_ITEMS];
    uint32_t cnt = 0;
#pragma unroll
    for (int it = 0; it < EMIT_ITEMS; ++it) {
        const int64_t k = base + it * 256 + t;
        ushort4 c = make_ushort4(0, 0, 0, 0);
        if (k < N) {
            const uint32_t g = order[(int64_t)v * N + k];
            const ushort4 r = g < (uint64_t)N ? rect[(int64_t)v * N + g] : make_ushort4(0, 0, 0, 0);
            if (r.z > r.x && r.w > r.y) {
                c = make_ushort4((unsigned short)(r.x >> cshift), (unsigned short)(r.y >> cshift),
                                 (unsigned short)(((r.z - 1) >> cshift) + 1), (unsigned short)(((r.w - 1) >> cshift) + 1));
                cnt += (uint32_t)((c.z - c.x) * (c.w - c.y));
            }
        }
        cr[it] = c;
    }
    const uint32_t inc = wave_scan_add_u32(cnt);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    if (t == 0) {
        uint32_t s = 0;
        for (int i = 0; i < 4; ++i) { uint32_t c = wsum[i]; wsum[i] = s; s += c; }
        gbase = s ? atomicAdd(n_pairs, (unsigned long long)s) : 0ull;
    }
    __syncthreads();
    if (cnt == 0) return;
    unsigned long long pos = gbase + wsum[w] + inc - cnt;
    if (pos + cnt > (unsigned long long)capacity) {
        *overflow = 1;
        return;
    }
    const int cw = gp.cx[v];
    const uint32_t cbase = (uint32_t)gp.cell_off[v];
#pragma unroll
    for (int it = 0; it < EMIT_ITEMS; ++it) {
        const ushort4 c = cr[it];
        const uint32_t k = (uint32_t)(base + it * 256 + t);
        for (int y = c.y; y < c.w; ++y)
            for (int x = c.x; x < c.z; ++x) keys[pos++] = ((cbase + (uint32_t)(y * cw + x)) << rbits) | k;
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

__device__ __forceinline__ int view_of_cell(const GridPack& gp, int V, uint32_t cell) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((uint32_t)gp.cell_off[mid] <= cell) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_cell_finalize(const uint32_t* __restrict__ skeys,
                                                       const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                       int rbits, const uint32_t* __restrict__ order, int64_t N,
                                                       GridPack gp, int V, uint32_t* __restrict__ cell_ids,
                                                       uint2* __restrict__ ranges, int64_t ncell)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_pairs;
    if (n > capacity) n = 0;
    if (i >= n) return;
    const uint32_t key = skeys[i];
    const uint32_t cell = key >> rbits;
    const uint32_t rank = key & ((1u << rbits) - 1u);
    if (cell >= (uint64_t)ncell || rank >= (uint64_t)N) return;  // consistent keys never hit this
    const int v = view_of_cell(gp, V, cell);
    cell_ids[i] = order[(int64_t)v * N + rank];
    if (i == 0 || (skeys[i - 1] >> rbits) != cell) ranges[cell].x = (uint32_t)i;
    if (i == n - 1 || (skeys[i + 1] >> rbits) != cell) ranges[cell].y = (uint32_t)(i + 1);
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
    bp->passes = (bp->rbits + bp->cbits + 7) / 8;
    return TG_OK;
}

// workspace layout
struct BinWs {
    uint32_t *dk_a, *dv_a, *dk_b, *dv_b;   // depth sort ping-pong [V*N]
    uint32_t *pk_a, *pk_b;                  // pair keys [capacity]
    void* scratch;
    size_t bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

BinWs layout_ws(void* ws, int64_t N, int V, int64_t capacity) {
    BinWs L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    size_t vn = (size_t)V * (size_t)N * 4;
    size_t a = take(vn), b = take(vn), c = take(vn), d = take(vn);
    size_t e = take((size_t)capacity * 4), f = take((size_t)capacity * 4);
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
    // (2) emit (coarse bin | depth rank) keys
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((N + 256 * EMIT_ITEMS - 1) / (256 * EMIT_ITEMS)), V), dim3(256), 0, s,
                       bins->order,
                       (const ushort4*)sp->rect, N, V, bp.gp, bp.cshift, bp.rbits, L.pk_a, bins->capacity,
                       (unsigned long long*)bins->n_pairs, bins->overflow);
    hipLaunchKernelGGL(k_check_overflow, dim3(1), dim3(1), 0, s, (const unsigned long long*)bins->n_pairs,
                       bins->capacity, bins->overflow);
    TG_CHECK_LAUNCH();
    if (bins->capacity == 0) return TG_OK;
    // (3) sort pair keys over their used bits; final keys land in pk_b or pk_a
    uint32_t* final_keys = L.pk_b;
    uint32_t* other = L.pk_a;
    // ping-pong: pass p writes (p odd ? kb : ka) except the last -> kfinal.
    // Input lives in pk_a, so use ka = pk_b, kb = pk_a, final = whichever the
    // last pass would otherwise overwrite safely.
    final_keys = (bp.passes & 1) ? L.pk_b : L.pk_a;
    other = (bp.passes & 1) ? L.pk_a : L.pk_b;
    (void)other;
    st = tg_radix_sort(L.pk_a, nullptr, L.pk_b, nullptr, L.pk_a, nullptr, final_keys, nullptr, bins->capacity, 1,
                    bins->n_pairs, 0, bp.passes, L.scratch, s);
    if (st != TG_OK) return st;
    // (4) ranges and ids
    hipLaunchKernelGGL(k_cell_finalize, dim3((unsigned)((bins->capacity + 255) / 256)), dim3(256), 0, s, final_keys,
                       bins->n_pairs, bins->capacity, bp.rbits, bins->order, N, bp.gp, V, bins->cell_ids,
                       (uint2*)bins->cell_ranges, bp.ncell);
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
    hipMemcpyAsync(starts, counts, (size_t)T * 4, hipMemcpyDeviceToDevice, s);
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
