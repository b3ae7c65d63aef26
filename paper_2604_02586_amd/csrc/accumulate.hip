// tg_splat_accumulate: PWI-LS statistics inside the renderer
// (TrackerSplat Sec. 4.3.3-4.3.5, Eq. 4; static-pixel counters of Sec. 4.5.2).
//
// The paper accumulates w P_i and w Q_i per Gaussian with atomic additions
// from a modified 3DGS renderer (one thread per pixel).  On CDNA4 we turn the
// loop inside out so that the per-Gaussian sums never need a cross-lane
// reduction:
//
//  * one wave64 owns one 16x16 tile; its 256 pixels are wave-uniform scalars
//    (the pixel's transmittance, track and flags live in 4 VGPRs per quantity
//    and are read with v_readlane), visited with s_ff1 over an alive mask so
//    finished pixels cost nothing;
//  * the 64 lanes hold 64 consecutive Gaussians of the tile's depth-ordered
//    list; for a pixel, every lane evaluates its Gaussian's alpha, and the
//    transmittance in front of each lane is an exclusive product scan across
//    the wave (6 DPP row_shr/row_bcast steps), so termination is a ballot and
//    first-set-bit;
//  * each lane keeps its Gaussian's 15 running sums in registers over all
//    pixels of the tile, then adds them to HBM with one set of FP32 atomics
//    per (tile, Gaussian) -- no shuffle reduction, no LDS merge.
//
// The tile's list is read from its coarse bin (8x8 tiles) in depth order and
// filtered by the tile rectangle with a ballot/popcount compaction into a
// per-wave LDS queue.  Blocks are remapped so that each XCD receives a
// contiguous range of coarse bins (its L2 holds that bin's list and splats).
#include "tg_internal.h"

namespace {

constexpr int QCAP = 128;
constexpr float LOG2E = 1.4426950408889634f;

struct AccArgs {
    const float4* rec;
    const ushort4* rect;
    const uint32_t* cell_ids;
    const uint2* ranges;
    const int32_t* overflow;
    const uint8_t* vis;
    float* acc;
    float* t_final;
    unsigned long long* stats;
    int64_t N;
    int V, W, H, cshift;
    int64_t n_enum;          // tiles enumerated (cells * tiles per cell)
    int64_t blocks;          // logical blocks
    int64_t blocks_per_xcd;
    float alpha_min, alpha_max, t_min, static2;
};

// One wave (64 threads) per workgroup and per 16x16 tile, so tiles of very
// different work never hold each other's resources.
template <bool STATS>
__global__ void __launch_bounds__(64) k_accumulate(AccArgs a, GridPack gp, const float2* __restrict__ disp)
{
    // 3.5 KB of LDS per wave keeps 8 waves per SIMD resident:
    // queue of filtered list entries (ids), per-pixel column/row offsets
    // inside the tile (as floats) and per-pixel transmittance
    __shared__ uint32_t qi[QCAP];
    __shared__ float2 CR[256];
    __shared__ float T_[256];
    if (*a.overflow) return;
    // XCD-aware remap: hardware places workgroup b on XCD (b mod 8); give
    // each XCD a contiguous range of tiles (its L2 then holds those bins).
    const int64_t b = blockIdx.x;
    const int64_t L = (b & 7) * a.blocks_per_xcd + (b >> 3);
    if (L >= a.n_enum) return;
    const int lane = threadIdx.x;
    const int k = 1 << a.cshift;
    const int kk = k * k;
    const uint32_t gcell = (uint32_t)(L / kk);
    const int ti = (int)(L % kk);
    int v = 0;
    {
        int lo = 0, hi = a.V - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if ((uint32_t)gp.cell_off[mid] <= gcell) lo = mid; else hi = mid - 1;
        }
        v = lo;
    }
    const int cl = (int)gcell - gp.cell_off[v];
    const int tx = (cl % gp.cx[v]) * k + (ti % k);
    const int ty = (cl / gp.cx[v]) * k + (ti / k);
    if (tx >= gp.tx[v] || ty >= gp.ty[v]) return;
    const uint2 rg = a.ranges[gcell];
    const int64_t vN = (int64_t)v * a.N;
    const int px0 = tx * TG_TILE, py0 = ty * TG_TILE;
    const int64_t row_base = (int64_t)v * a.H;

    // pixel state: pixel j = g*64 + lane -> (px0 + (j&15), py0 + (j>>4))
    uint64_t alive[4], visb[4], statb[4];
    float dxg[4], dyg[4];   // track of pixel g*64 + lane
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int j = g * 64 + lane;
        const int px = px0 + (j & 15), py = py0 + (j >> 4);
        const bool in = px < a.W && py < a.H;
        float ddx = 0.f, ddy = 0.f;
        bool vv = false;
        if (in) {
            const int64_t pi = (row_base + py) * a.W + px;
            const float2 d = disp[pi];
            ddx = d.x;
            ddy = d.y;
            vv = a.vis ? a.vis[pi] != 0 : true;
        }
        CR[j] = make_float2((float)(j & 15), (float)(j >> 4));
        T_[j] = 1.0f;
        dxg[g] = ddx;
        dyg[g] = ddy;
        alive[g] = ballot64(in);
        visb[g] = ballot64(in && vv);
        float s2;
        {
#pragma clang fp contract(off)
            s2 = ddx * ddx;
            s2 = s2 + ddy * ddy;
        }
        statb[g] = ballot64(in && s2 < a.static2);
    }
    uint64_t n_eval = 0, n_contrib = 0, n_iter = 0, n_refill = 0;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min;
    const float log_amin = __logf(amin);
    const uint64_t ltmask = lanemask_lt();
    const bool lane0 = lane == 0;
    float pex_reg = 1.0f;   // lane 0 is never written by the wave shift below
    int qn = 0;
    uint32_t pos = rg.x;
    // pixel-centre extent of the tile (conservative for the ellipse test)
    const float ex0 = (float)px0, ex1 = (float)(px0 + TG_TILE - 1);
    const float ey0 = (float)py0, ey1 = (float)(py0 + TG_TILE - 1);
    // prefetched ids of the next 64 list entries
    uint32_t nid = (pos + lane < rg.y) ? a.cell_ids[pos + lane] : 0xFFFFFFFFu;

    while ((alive[0] | alive[1] | alive[2] | alive[3]) != 0ull) {
        // Refill: list entries whose rectangle contains this tile and whose
        // alpha >= alpha_min region can reach it.  The second test is exact
        // culling: q >= 2 ln(o / alpha_min) everywhere on the tile means
        // alpha < alpha_min at every pixel, so the Gaussian neither adds nor
        // attenuates (a margin keeps it conservative under FP32 rounding).
        while (qn < 64 && pos < rg.y) {
            const uint32_t gid = nid;
            const uint32_t i = pos + lane;
            pos += 64;
            nid = (pos + lane < rg.y) ? a.cell_ids[pos + lane] : 0xFFFFFFFFu;
            bool hit = false;
            if (i < rg.y && gid < (uint64_t)a.N) {
                const ushort4 r = a.rect[vN + gid];
                hit = tx >= r.x && tx < r.z && ty >= r.y && ty < r.w;
                if (hit)
                    hit = splat_reaches_tile(a.rec[2 * (vN + gid)], a.rec[2 * (vN + gid) + 1], log_amin, amin, ex0,
                                             ex1, ey0, ey1);
            }
            const uint64_t m = ballot64(hit);
            if (hit) qi[qn + __popcll(m & ltmask)] = gid;
            qn += __popcll(m);
            if (STATS) n_refill += 1;
        }
        if (qn == 0) break;
        const int nb = qn < 64 ? qn : 64;
        uint32_t gid = 0;
        float dxl = 0.f, dyl = 0.f, ca = 0.f, cb = 0.f, cc = 0.f, op = 0.f;
        if (lane < nb) {
            gid = qi[lane];
            const float4 r0 = a.rec[2 * (vN + gid)];
            const float4 r1 = a.rec[2 * (vN + gid) + 1];
            dxl = (float)px0 - r0.x;   // u = (px0 + column) - mu_x
            dyl = (float)py0 - r0.y;
            ca = -0.5f * LOG2E * r0.z;
            cb = -LOG2E * r0.w;
            cc = -0.5f * LOG2E * r1.x;
            op = r1.y;
        }
        if (lane + 64 < qn) {
            const uint32_t g2 = qi[lane + 64];
            qi[lane] = g2;
        }
        qn -= nb;

        float s_w = 0.f, s_ux = 0.f, s_uy = 0.f, s_xx = 0.f, s_xy = 0.f, s_yy = 0.f;
        float s_dx = 0.f, s_dy = 0.f, s_xdx = 0.f, s_xdy = 0.f, s_ydx = 0.f, s_ydy = 0.f;
        float s_n = 0.f, s_sn = 0.f, s_sa = 0.f;

#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint64_t m = alive[g];
            uint64_t dead = 0;
            const uint64_t vg = visb[g], sg = statb[g];
            // two pixels per step: their dependency chains interleave
            while (m) {
                const int j1 = __builtin_ctzll(m);
                m &= m - 1;
                const bool two = m != 0;
                const int j2 = two ? (int)__builtin_ctzll(m) : j1;
                if (two) m &= m - 1;
                const int p1 = g * 64 + j1, p2i = g * 64 + j2;
                const float2 cr1 = CR[p1], cr2 = CR[p2i];
                const float T1 = T_[p1], T2 = T_[p2i];
                const float ux1 = dxl + cr1.x, uy1 = dyl + cr1.y;
                const float ux2 = dxl + cr2.x, uy2 = dyl + cr2.y;
                const float q1 = ux1 * (ca * ux1 + cb * uy1) + cc * uy1 * uy1;
                const float q2 = ux2 * (ca * ux2 + cb * uy2) + cc * uy2 * uy2;
                // alpha = min(alpha_max, o e^power), clamped with one v_med3
                const float al1 = __builtin_amdgcn_fmed3f(op * __builtin_amdgcn_exp2f(q1), 0.0f, amax);
                const float al2 = __builtin_amdgcn_fmed3f(op * __builtin_amdgcn_exp2f(q2), 0.0f, amax);
                // valid lanes: power <= 0 and alpha >= alpha_min
                const uint64_t vm1 = ballot64(q1 <= 0.0f) & ballot64(al1 >= amin);
                const uint64_t vm2 = two ? (ballot64(q2 <= 0.0f) & ballot64(al2 >= amin)) : 0ull;
                float P1 = __builtin_amdgcn_inverse_ballot_w64(vm1) ? 1.0f - al1 : 1.0f;
                float P2 = __builtin_amdgcn_inverse_ballot_w64(vm2) ? 1.0f - al2 : 1.0f;
                wave_scan_mul_fused2(P1, P2);
                const uint64_t tm1 = ballot64(T1 * P1 < tmin) & vm1;
                const uint64_t tm2 = ballot64(T2 * P2 < tmin) & vm2;
                const int kt1 = (int)__builtin_ctzll(tm1 | (1ull << 63));
                const int kt2 = (int)__builtin_ctzll(tm2 | (1ull << 63));
                const uint64_t cm1 = vm1 & (tm1 ? ((1ull << kt1) - 1ull) : ~0ull);
                const uint64_t cm2 = vm2 & (tm2 ? ((1ull << kt2) - 1ull) : ~0ull);
                const float Pk1 = tm1 ? (kt1 == 0 ? 1.0f : readlane_f(P1, kt1 - 1)) : readlane_f(P1, 63);
                const float Pk2 = tm2 ? (kt2 == 0 ? 1.0f : readlane_f(P2, kt2 - 1)) : readlane_f(P2, 63);
                if (lane0) {
                    T_[p1] = T1 * Pk1;
                    if (two) T_[p2i] = T2 * Pk2;
                }
                if (tm1) dead |= 1ull << j1;
                if (tm2) dead |= 1ull << j2;
                if (STATS) {
                    n_eval += (uint64_t)(tm1 ? kt1 + 1 : nb);
                    n_contrib += (uint64_t)__popcll(cm1);
                    n_iter += 1;
                    if (two) {
                        n_eval += (uint64_t)(tm2 ? kt2 + 1 : nb);
                        n_contrib += (uint64_t)__popcll(cm2);
                        n_iter += 1;
                    }
                }
                // statistics of Eq. 4 for the lanes that contribute
                if (cm1 && ((vg >> j1) & 1ull)) {
                    const float tdx = readlane_f(dxg[g], j1), tdy = readlane_f(dyg[g], j1);
                    asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf"
                                 : "+v"(pex_reg) : "v"(P1));
                    if (__builtin_amdgcn_inverse_ballot_w64(cm1)) {
                        const float wgt = al1 * (T1 * pex_reg);
                        const float wx = wgt * ux1, wy = wgt * uy1;
                        s_w += wgt;
                        s_ux += wx;
                        s_uy += wy;
                        s_xx += wx * ux1;
                        s_xy += wx * uy1;
                        s_yy += wy * uy1;
                        s_dx += wgt * tdx;
                        s_dy += wgt * tdy;
                        s_xdx += wx * tdx;
                        s_xdy += wx * tdy;
                        s_ydx += wy * tdx;
                        s_ydy += wy * tdy;
                        s_n += 1.0f;
                        if ((sg >> j1) & 1ull) {
                            s_sn += 1.0f;
                            s_sa += al1;
                        }
                    }
                }
                if (cm2 && ((vg >> j2) & 1ull)) {
                    const float tdx = readlane_f(dxg[g], j2), tdy = readlane_f(dyg[g], j2);
                    asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf"
                                 : "+v"(pex_reg) : "v"(P2));
                    if (__builtin_amdgcn_inverse_ballot_w64(cm2)) {
                        const float wgt = al2 * (T2 * pex_reg);
                        const float wx = wgt * ux2, wy = wgt * uy2;
                        s_w += wgt;
                        s_ux += wx;
                        s_uy += wy;
                        s_xx += wx * ux2;
                        s_xy += wx * uy2;
                        s_yy += wy * uy2;
                        s_dx += wgt * tdx;
                        s_dy += wgt * tdy;
                        s_xdx += wx * tdx;
                        s_xdy += wx * tdy;
                        s_ydx += wy * tdx;
                        s_ydy += wy * tdy;
                        s_n += 1.0f;
                        if ((sg >> j2) & 1ull) {
                            s_sn += 1.0f;
                            s_sa += al2;
                        }
                    }
                }
            }
            alive[g] &= ~dead;
        }
        if (lane < nb && s_n > 0.0f) {
            float* dst = a.acc + (vN + gid) * TG_ACC_STRIDE;
            unsafeAtomicAdd(dst + 0, s_w);
            unsafeAtomicAdd(dst + 1, s_ux);
            unsafeAtomicAdd(dst + 2, s_uy);
            unsafeAtomicAdd(dst + 3, s_xx);
            unsafeAtomicAdd(dst + 4, s_xy);
            unsafeAtomicAdd(dst + 5, s_yy);
            unsafeAtomicAdd(dst + 6, s_dx);
            unsafeAtomicAdd(dst + 7, s_dy);
            unsafeAtomicAdd(dst + 8, s_xdx);
            unsafeAtomicAdd(dst + 9, s_xdy);
            unsafeAtomicAdd(dst + 10, s_ydx);
            unsafeAtomicAdd(dst + 11, s_ydy);
            unsafeAtomicAdd(dst + 12, s_n);
            if (s_sn > 0.0f) {
                unsafeAtomicAdd(dst + 13, s_sn);
                unsafeAtomicAdd(dst + 14, s_sa);
            }
        }
    }
    if (a.t_final) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int j = g * 64 + lane;
            const int px = px0 + (j & 15), py = py0 + (j >> 4);
            if (px < a.W && py < a.H) a.t_final[(row_base + py) * a.W + px] = T_[j];
        }
    }
    if (STATS && lane == 0) {
        atomicAdd(a.stats, (unsigned long long)n_eval);
        atomicAdd(a.stats + 1, (unsigned long long)n_contrib);
        atomicAdd(a.stats + 2, (unsigned long long)n_iter);
        atomicAdd(a.stats + 3, (unsigned long long)n_refill);
    }
}

}  // namespace

extern "C" tg_status tg_splat_accumulate(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                         int32_t V, const float* disp, const uint8_t* vis, const tg_params* p,
                                         float* acc, float* t_final, int64_t* stats, void* stream)
{
    if (!s || !bins || !cams || !p || !disp || !acc || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (!s->rec || !s->rect || !bins->cell_ids || !bins->cell_ranges || !bins->overflow) return TG_ERR_INVALID_ARG;
    if (!aligned16(s->rec) || !aligned16(acc) || ((uintptr_t)disp & 7u)) return TG_ERR_ALIGNMENT;
    for (int v = 1; v < V; ++v)
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) return TG_ERR_INVALID_ARG;
    if (N == 0) return TG_OK;
    if (N > (int64_t)0xFFFFFFFF) return TG_ERR_UNSUPPORTED;
    // same coarse plan as tg_bin_sort
    int cs = p->coarse_shift < 0 ? 0 : p->coarse_shift;
    int rbits = 1;
    while (rbits < 63 && (1ull << rbits) < (uint64_t)N) ++rbits;
    GridPack gp;
    int64_t ncell;
    for (;; ++cs) {
        ncell = fill_grid(cams, V, cs, &gp);
        int cbits = 1;
        while (cbits < 63 && (1ull << cbits) < (uint64_t)ncell) ++cbits;
        if (rbits + cbits <= 32) break;
        if (cs > 12) return TG_ERR_UNSUPPORTED;
    }
    AccArgs a;
    a.rec = (const float4*)s->rec;
    a.rect = (const ushort4*)s->rect;
    a.cell_ids = bins->cell_ids;
    a.ranges = (const uint2*)bins->cell_ranges;
    a.overflow = bins->overflow;
    a.vis = vis;
    a.acc = acc;
    a.t_final = t_final;
    a.stats = (unsigned long long*)stats;
    a.N = N;
    a.V = V;
    a.W = cams[0].width;
    a.H = cams[0].height;
    a.cshift = cs;
    a.n_enum = ncell << (2 * cs);
    a.blocks = a.n_enum;
    a.blocks_per_xcd = (a.n_enum + 7) / 8;
    a.alpha_min = p->alpha_min;
    a.alpha_max = p->alpha_max;
    a.t_min = p->t_min;
    a.static2 = p->static_px * p->static_px;
    const int64_t grid = a.blocks_per_xcd * 8;
    if (stats)
        hipLaunchKernelGGL(k_accumulate<true>, dim3((unsigned)grid), dim3(64), 0, (hipStream_t)stream, a, gp,
                           (const float2*)disp);
    else
        hipLaunchKernelGGL(k_accumulate<false>, dim3((unsigned)grid), dim3(64), 0, (hipStream_t)stream, a, gp,
                           (const float2*)disp);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
