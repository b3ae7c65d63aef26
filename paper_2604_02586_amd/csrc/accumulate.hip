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

constexpr int ACC_WAVES = 4;
constexpr int QCAP = 128;
constexpr float LOG2E = 1.4426950408889634f;

struct AccArgs {
    const float4* rec;
    const ushort4* rect;
    const uint32_t* cell_ids;
    const uint2* ranges;
    const int32_t* overflow;
    const float2* disp;
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

__global__ void __launch_bounds__(256) k_accumulate(AccArgs a, GridPack gp)
{
    __shared__ uint32_t queue[ACC_WAVES][QCAP];
    if (*a.overflow) return;
    // XCD-aware remap: hardware places block b on XCD (b mod 8).
    const int64_t b = blockIdx.x;
    const int64_t lb = (b & 7) * a.blocks_per_xcd + (b >> 3);
    if (lb >= a.blocks) return;
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t L = lb * ACC_WAVES + w;
    if (L >= a.n_enum) return;
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

    // pixel state: pixel j = g*64 + lane -> (tx*16 + (j&15), ty*16 + (j>>4))
    float Tg[4], dxg[4], dyg[4];
    uint64_t alive[4], visb[4], statb[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int j = g * 64 + lane;
        const int px = tx * TG_TILE + (j & 15), py = ty * TG_TILE + (j >> 4);
        const bool in = px < a.W && py < a.H;
        float ddx = 0.f, ddy = 0.f;
        bool vv = false;
        if (in) {
            const int64_t pi = ((int64_t)v * a.H + py) * a.W + px;
            float2 d = a.disp[pi];
            ddx = d.x;
            ddy = d.y;
            vv = a.vis ? a.vis[pi] != 0 : true;
        }
        Tg[g] = 1.0f;
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
    uint64_t n_eval = 0, n_contrib = 0;
    const bool want_stats = a.stats != nullptr;

    const uint64_t ltmask = lanemask_lt();
    uint32_t* q = queue[w];
    int qn = 0;
    uint32_t pos = rg.x;
    const float fx0 = (float)(tx * TG_TILE), fy0 = (float)(ty * TG_TILE);

    while ((alive[0] | alive[1] | alive[2] | alive[3]) != 0ull) {
        // refill the queue with list entries whose rectangle contains this tile
        while (qn < 64 && pos < rg.y) {
            const uint32_t i = pos + lane;
            bool hit = false;
            uint32_t gid = 0;
            if (i < rg.y) {
                gid = a.cell_ids[i];
                if (gid < (uint64_t)a.N) {
                    const ushort4 r = a.rect[vN + gid];
                    hit = tx >= r.x && tx < r.z && ty >= r.y && ty < r.w;
                }
            }
            const uint64_t m = ballot64(hit);
            if (hit) q[qn + __popcll(m & ltmask)] = gid;
            qn += __popcll(m);
            pos += 64;
        }
        if (qn == 0) break;
        const int nb = qn < 64 ? qn : 64;
        const uint32_t gid = lane < nb ? q[lane] : 0u;
        const uint32_t moved = (lane + 64 < qn) ? q[lane + 64] : 0u;
        if (lane + 64 < qn) q[lane] = moved;
        qn -= nb;

        float mx = 0.f, my = 0.f, ca = 0.f, cb = 0.f, cc = 0.f, op = 0.f;
        if (lane < nb) {
            const float4 r0 = a.rec[2 * (vN + gid)];
            const float4 r1 = a.rec[2 * (vN + gid) + 1];
            mx = r0.x;
            my = r0.y;
            ca = -0.5f * LOG2E * r0.z;
            cb = -LOG2E * r0.w;
            cc = -0.5f * LOG2E * r1.x;
            op = r1.y;
        }
        float s_w = 0.f, s_ux = 0.f, s_uy = 0.f, s_xx = 0.f, s_xy = 0.f, s_yy = 0.f;
        float s_dx = 0.f, s_dy = 0.f, s_xdx = 0.f, s_xdy = 0.f, s_ydx = 0.f, s_ydy = 0.f;
        float s_n = 0.f, s_sn = 0.f, s_sa = 0.f;

#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint64_t m = alive[g];
            while (m) {
                const int j = __builtin_ctzll(m);
                m &= m - 1;
                const int pj = g * 64 + j;
                const float T = readlane_f(Tg[g], j);
                const float ddx = readlane_f(dxg[g], j);
                const float ddy = readlane_f(dyg[g], j);
                const float ux = (fx0 + (float)(pj & 15)) - mx;
                const float uy = (fy0 + (float)(pj >> 4)) - my;
                const float p2 = ux * (ca * ux + cb * uy) + cc * uy * uy;
                const float al = fminf(a.alpha_max, op * __builtin_amdgcn_exp2f(p2));
                const bool valid = (p2 <= 0.0f) && (al >= a.alpha_min);
                const float qv = valid ? 1.0f - al : 1.0f;
                const float P = wave_scan_mul(qv);
                const uint64_t tm = ballot64(valid && (T * P < a.t_min));
                uint64_t cm = ballot64(valid);
                float Tn;
                if (tm) {
                    const int kt = __builtin_ctzll(tm);
                    cm &= (kt == 0) ? 0ull : (~0ull >> (64 - kt));
                    Tn = kt == 0 ? T : T * readlane_f(P, kt - 1);
                    alive[g] &= ~(1ull << j);
                    if (want_stats) n_eval += (uint64_t)(kt + 1);
                } else {
                    Tn = T * readlane_f(P, 63);
                    if (want_stats) n_eval += (uint64_t)nb;
                }
                Tg[g] = writelane_f(Tg[g], Tn, j);
                if (want_stats) n_contrib += (uint64_t)__popcll(cm);
                if (cm && ((visb[g] >> j) & 1ull)) {
                    const float Pex = wave_shr1(P, 1.0f);
                    if ((cm >> lane) & 1ull) {
                        const float wgt = al * (T * Pex);
                        const float wx = wgt * ux, wy = wgt * uy;
                        s_w += wgt;
                        s_ux += wx;
                        s_uy += wy;
                        s_xx += wx * ux;
                        s_xy += wx * uy;
                        s_yy += wy * uy;
                        s_dx += wgt * ddx;
                        s_dy += wgt * ddy;
                        s_xdx += wx * ddx;
                        s_xdy += wx * ddy;
                        s_ydx += wy * ddx;
                        s_ydy += wy * ddy;
                        s_n += 1.0f;
                        if ((statb[g] >> j) & 1ull) {
                            s_sn += 1.0f;
                            s_sa += al;
                        }
                    }
                }
            }
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
            const int px = tx * TG_TILE + (j & 15), py = ty * TG_TILE + (j >> 4);
            if (px < a.W && py < a.H) a.t_final[((int64_t)v * a.H + py) * a.W + px] = Tg[g];
        }
    }
    if (want_stats && lane == 0) {
        atomicAdd(a.stats, (unsigned long long)n_eval);
        atomicAdd(a.stats + 1, (unsigned long long)n_contrib);
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
    a.disp = (const float2*)disp;
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
    a.blocks = (a.n_enum + ACC_WAVES - 1) / ACC_WAVES;
    a.blocks_per_xcd = (a.blocks + 7) / 8;
    a.alpha_min = p->alpha_min;
    a.alpha_max = p->alpha_max;
    a.t_min = p->t_min;
    a.static2 = p->static_px * p->static_px;
    const int64_t grid = a.blocks_per_xcd * 8;
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, a, gp);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
