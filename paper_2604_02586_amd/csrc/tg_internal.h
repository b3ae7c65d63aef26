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

#define TG_CHECK_LAUNCH()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return TG_ERR_DEVICE; \
    } while (0)

static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
