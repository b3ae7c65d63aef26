// Internal helpers shared by the libtg HIP sources (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tg.h"

#define TG_WAVE 64

// Cameras travel in the kernel-argument segment (no device allocation, no
// host->device copy): up to TG_MAX_VIEWS per launch.
struct CamPack {
    tg_camera cam[TG_MAX_VIEWS];
};

// Per-view geometry of the tile grid, packed alongside the cameras.
struct GridPack {
    int32_t tx[TG_MAX_VIEWS];        // tiles per row
    int32_t ty[TG_MAX_VIEWS];        // tiles per column
    int32_t cx[TG_MAX_VIEWS];        // coarse bins per row
    int32_t cy[TG_MAX_VIEWS];        // coarse bins per column
    int32_t cell_off[TG_MAX_VIEWS + 1];  // first coarse bin of each view
    int32_t tile_off[TG_MAX_VIEWS + 1];  // first tile of each view
};

__device__ __forceinline__ float bitsf(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint32_t fbits(float f) { return __builtin_bit_cast(uint32_t, f); }

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Lanes (among those where act holds) whose 8-bit value d equals this
// lane's: the stable-rank primitive of the sorts (rank = popcount of the
// result below this lane).  Eight ballots of the value's bits; each lane
// keeps the lanes that agree with it on a bit with one XNOR and one AND per
// mask half (against the bit spread over the word), instead of a per-lane
// select between a ballot and its complement.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, bool act) {
    const uint64_t a = __ballot(act);
    uint32_t mlo = (uint32_t)a, mhi = (uint32_t)(a >> 32);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const uint32_t sm = (uint32_t)(((int32_t)(d << (31 - bit))) >> 31);   // all ones where set
        const uint64_t bb = __ballot(sm != 0u);
        mlo &= ~((uint32_t)bb ^ sm);
        mhi &= ~((uint32_t)(bb >> 32) ^ sm);
    }
    return ((uint64_t)mhi << 32) | mlo;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ float writelane_f(float v, float val, int lane) {
    // returns v with lane `lane` replaced by val (val wave-uniform)
    return lane_id() == lane ? val : v;
}

// DPP moves (gfx9 encodings): row_shr:n = 0x110+n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.  Lanes without a source keep `old`.
template <int CTRL, int ROW, int BANK>
__device__ __forceinline__ float dpp_f(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, src), CTRL,
                                                                  ROW, BANK, false));
}

// Inclusive product scan across the 64 lanes of a wave.
__device__ __forceinline__ float wave_scan_mul(float v) {
    v *= dpp_f<0x111, 0xf, 0xf>(1.0f, v);
    v *= dpp_f<0x112, 0xf, 0xf>(1.0f, v);
    v *= dpp_f<0x114, 0xf, 0xe>(1.0f, v);
    v *= dpp_f<0x118, 0xf, 0xc>(1.0f, v);
    v *= dpp_f<0x142, 0xa, 0xf>(1.0f, v);
    v *= dpp_f<0x143, 0xc, 0xf>(1.0f, v);
    return v;
}
// Inclusive sum scan across the wave.
__device__ __forceinline__ float wave_scan_add(float v) {
    v += dpp_f<0x111, 0xf, 0xf>(0.0f, v);
    v += dpp_f<0x112, 0xf, 0xf>(0.0f, v);
    v += dpp_f<0x114, 0xf, 0xe>(0.0f, v);
    v += dpp_f<0x118, 0xf, 0xc>(0.0f, v);
    v += dpp_f<0x142, 0xa, 0xf>(0.0f, v);
    v += dpp_f<0x143, 0xc, 0xf>(0.0f, v);
    return v;
}
// Value of the previous lane (lane 0 gets `first`).
__device__ __forceinline__ float wave_shr1(float v, float first) { return dpp_f<0x138, 0xf, 0xf>(first, v); }

// Inclusive product scan across the wave as six fused v_mul_f32_dpp: lanes
// whose DPP source is outside the row/wave are not written (bound_ctrl off),
// which multiplies them by one.  Each step reads the previous VALU result, so
// two wait states precede it.  All 64 lanes must be active.
__device__ __forceinline__ float wave_scan_mul_fused(float x) {
    asm volatile(
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(x));
    return x;
}

// Three independent inclusive sum scans with their steps interleaved: each
// step reads its own previous result from three instructions back, which
// covers the two wait states a DPP read needs, so no s_nop is required.
// All 64 lanes must be active.
__device__ __forceinline__ void wave_scan_add_fused3(float& x, float& y, float& z) {
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_add_f32_dpp %2, %2, %2 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(x), "+v"(y), "+v"(z));
}

// Exact float of a wave-uniform integer n < 2^24, built on the scalar unit
// (exponent from the leading bit, mantissa by shifting): no VALU conversion.
__device__ __forceinline__ float uniform_u2f(uint32_t n) {
    if (n == 0) return 0.0f;
    const int e = 31 - __builtin_clz(n);
    const uint32_t bits = ((uint32_t)(127 + e) << 23) | ((n << (23 - e)) & 0x7FFFFFu);
    return __builtin_bit_cast(float, bits);
}

// Inclusive sum scan as six fused v_add_f32_dpp (lanes without a DPP source
// are not written, i.e. add zero).  All 64 lanes must be active.
__device__ __forceinline__ float wave_scan_add_fused(float x) {
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(x));
    return x;
}

// Exponent of alpha in log2 units at pixel offset (ux, uy) for a
// log2-prescaled conic (ca, cb, cc): ux (ca ux + cb uy) + cc uy^2.  The
// forward and backward rasterisers both call this one function, with the
// fused multiply-adds written out and contraction otherwise off, so the
// backward's replay of the forward's alpha decisions is bit-identical
// whatever the compiler does with the surrounding code.
__device__ __forceinline__ float raster_power(float ux, float uy, float ca, float cb, float cc) {
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(ca, ux, cb * uy);
    return __builtin_fmaf(ux, t, (cc * uy) * uy);
}

// Smallest value over the rectangle [x0,x1] x [y0,y1] of the positive-definite
// form q(p) = a dx^2 + 2 b dx dy + c dy^2, (dx, dy) = p - (mx, my): zero when the
// centre is inside, otherwise the least of the four edge minima (each a 1D
// quadratic minimised on its segment).
__device__ __forceinline__ float rect_min_form(float a, float b, float c, float mx, float my, float x0, float x1,
                                               float y0, float y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0f;
    const float dx0 = x0 - mx, dx1 = x1 - mx, dy0 = y0 - my, dy1 = y1 - my;
    // the hardware reciprocal (about 1 ulp) only moves each edge minimiser
    // slightly along its segment, where the form is flat to second order;
    // the caller's margin covers it
    const float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
    float best;
    {
        const float dy = fminf(dy1, fmaxf(dy0, -b * dx0 * ic));
        best = a * dx0 * dx0 + (2.0f * b * dx0 + c * dy) * dy;
    }
    {
        const float dy = fminf(dy1, fmaxf(dy0, -b * dx1 * ic));
        best = fminf(best, a * dx1 * dx1 + (2.0f * b * dx1 + c * dy) * dy);
    }
    {
        const float dx = fminf(dx1, fmaxf(dx0, -b * dy0 * ia));
        best = fminf(best, c * dy0 * dy0 + (2.0f * b * dy0 + a * dx) * dx);
    }
    {
        const float dx = fminf(dx1, fmaxf(dx0, -b * dy1 * ia));
        best = fminf(best, c * dy1 * dy1 + (2.0f * b * dy1 + a * dx) * dx);
    }
    return best;
}

// Does the splat (record r0 = {mx, my, conic a, b}, r1 = {conic c, opacity,..})
// reach alpha >= alpha_min anywhere on the tile's pixel centres?  Exact
// culling: q >= 2 ln(o / alpha_min) on the whole tile means alpha < alpha_min
// at every pixel (the Gaussian neither adds nor attenuates); the margin keeps
// the test conservative under FP32 rounding.
__device__ __forceinline__ bool splat_reaches_tile(float4 r0, float4 r1, float log_amin, float amin, float ex0,
                                                   float ex1, float ey0, float ey1) {
    const float tau = 2.0f * (__logf(r1.y) - log_amin);
    const float qmin = rect_min_form(r0.z, r0.w, r1.x, r0.x, r0.y, ex0, ex1, ey0, ey1);
    return r1.y >= amin && qmin <= tau + 1e-3f * (1.0f + fabsf(tau));
}

// Tile of a cell-major tile enumeration index L (coarse bins of k x k tiles,
// views back to back).  Returns false for enumerated tiles outside the image.
struct TileCoord {
    int v, tx, ty;
    uint32_t gcell;
};
__device__ __forceinline__ bool tile_of(int64_t L, int cshift, int V, const GridPack& gp, TileCoord* t) {
    const int k = 1 << cshift;
    const int kk = k * k;
    const uint32_t gcell = (uint32_t)(L / kk);
    const int ti = (int)(L % kk);
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((uint32_t)gp.cell_off[mid] <= gcell) lo = mid; else hi = mid - 1;
    }
    const int cl = (int)gcell - gp.cell_off[lo];
    t->v = lo;
    t->gcell = gcell;
    t->tx = (cl % gp.cx[lo]) * k + (ti % k);
    t->ty = (cl / gp.cx[lo]) * k + (ti / k);
    return t->tx < gp.tx[lo] && t->ty < gp.ty[lo];
}

// Integer inclusive sum scan across the wave (used by binning).
__device__ __forceinline__ uint32_t wave_scan_add_u32(uint32_t v) {
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane_id() >= o) v += t;
    }
    return v;
}

__host__ __device__ inline int32_t ceil_div(int32_t a, int32_t b) { return (a + b - 1) / b; }

// Host: fill grid metadata for V views; returns total coarse bins.
inline int64_t fill_grid(const tg_camera* cams, int32_t V, int cshift, GridPack* g) {
    int64_t cell = 0, tile = 0;
    for (int v = 0; v < V; ++v) {
        int TX = ceil_div(cams[v].width, TG_TILE), TY = ceil_div(cams[v].height, TG_TILE);
        int k = 1 << cshift;
        g->tx[v] = TX;
        g->ty[v] = TY;
        g->cx[v] = ceil_div(TX, k);
        g->cy[v] = ceil_div(TY, k);
        g->cell_off[v] = (int32_t)cell;
        g->tile_off[v] = (int32_t)tile;
        cell += (int64_t)g->cx[v] * g->cy[v];
        tile += (int64_t)TX * TY;
    }
    g->cell_off[V] = (int32_t)cell;
    g->tile_off[V] = (int32_t)tile;
    return cell;
}

// Same coarse plan as tg_bin_sort (coarse size grows until bin and rank bits
// fit 32); returns the number of coarse bins or -1.
inline int64_t coarse_plan(const tg_camera* cams, int32_t V, int64_t N, const tg_params* p, GridPack* gp,
                           int* cshift) {
    int cs = p->coarse_shift < 0 ? 0 : p->coarse_shift;
    int rbits = 1;
    while (rbits < 63 && (1ull << rbits) < (uint64_t)(N > 0 ? N : 1)) ++rbits;
    for (;; ++cs) {
        const int64_t ncell = fill_grid(cams, V, cs, gp);
        int cbits = 1;
        while (cbits < 63 && (1ull << cbits) < (uint64_t)ncell) ++cbits;
        if (rbits + cbits <= 32) {
            *cshift = cs;
            return ncell;
        }
        if (cs > 12) return -1;
    }
}

#define TG_CHECK_LAUNCH()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return TG_ERR_DEVICE; \
    } while (0)

static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Stable LSD radix sort (sort.hip).  Sorts nseg segments of seg_len keys (or
// one segment of *dev_count keys) by bits [bit0, bit0 + 8*passes).  ka/va
// receive the first pass, kb/vb are the ping-pong partner, kfinal/vfinal the
// last pass (either may be null when not needed); vin == null means values
// are the indices.  scratch: tg_sort_scratch_bytes(seg_len, nseg) bytes.
__attribute__((visibility("hidden"))) size_t tg_sort_scratch_bytes(int64_t seg_len, int nseg);
__attribute__((visibility("hidden"))) tg_status tg_radix_sort(const uint32_t* kin, const uint32_t* vin, uint32_t* ka, uint32_t* va, uint32_t* kb,
                        uint32_t* vb, uint32_t* kfinal, uint32_t* vfinal, int64_t seg_len, int nseg,
                        const int64_t* dev_count, int bit0, int passes, void* scratch, hipStream_t s);
// In-place exclusive scan of L u32 values; scratch: one u32 per 4096 values.
__attribute__((visibility("hidden"))) void tg_exclusive_scan_u32(uint32_t* data, int64_t L, uint32_t* scratch, hipStream_t s);
