// Differentiable rasteriser for the post-relocation refinement
// (TrackerSplat Sec. 4.6: the relocated Gaussians are refined by training on
// the input frames with the 3DGS objective; here L1 + Adam, Sec. 5.2).
//
//   tg_raster_fwd   C(x) = sum_i c_i alpha_i T_i + T_final bg, depth order,
//                   same alpha / skip / termination rules as the motion path
//                   (Sec. 3.1).  Pixel-parallel: one 256-thread workgroup per
//                   16x16 tile; the block filters its coarse bin's depth-ordered
//                   list into LDS batches.  Per pixel it records how many
//                   filtered entries it processed, so the backward replays
//                   exactly the same set.
//   tg_raster_bwd   Gaussian-parallel within a tile (one wave64, 64
//                   consecutive Gaussians across the lanes, pixels as
//                   wave-uniform values), front to back: transmittance in
//                   front of a lane is a DPP product scan, and since every
//                   channel enters through its dot product with the pixel's
//                   dL/dC, one DPP sum scan of g . c_i w_i gives the colour in
//                   front and the final colour the colour behind:
//                   dL/dalpha_i = g . (c_i T_i - (C - front_i - c_i w_i) /
//                   (1 - alpha_i)).  The 9 gradients of
//                   each Gaussian's 2D splat stay in registers over the tile and
//                   go to HBM with one set of atomics per (tile, Gaussian).
//   tg_project_bwd  per Gaussian, over views: splat gradients -> mean,
//                   quaternion, log-scale, logit-opacity, SH coefficients.
//   tg_l1_loss_grad, tg_adam_step, tg_adam_step_rows: elementwise.
#include "tg_internal.h"

namespace {

constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.69314718055994531f;

struct RasterArgs {
    const float4* rec;
    const float* colors;
    const ushort4* rect;
    const uint32_t* cell_ids;
    const uint2* ranges;
    const int32_t* overflow;
    int64_t N;
    int V, W, H, cshift;
    int64_t n_enum;
    int64_t blocks_per_xcd;
    float alpha_min, alpha_max, t_min;
    float bg0, bg1, bg2;
};

// Sum over the wave of a per-lane count (a pixel's count is far below
// 2^26, so 64 of them fit 32 bits).
__device__ __forceinline__ uint64_t wave_sum_u64(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

// Filtered list entry staged in LDS: scaled conic (log2 units), centre,
// opacity, colour.
struct Entry {
    float mx, my, ca, cb, cc, op, r, g, b;
};

// STATS: adds (pairs evaluated, pairs contributing) to stats[0..1]; a
// pair is evaluated when the pixel, not yet terminated, tests the entry,
// and contributes when it passes every test and is composited.
template <bool STATS>
__global__ void __launch_bounds__(256) k_raster_fwd(RasterArgs a, GridPack gp, float* __restrict__ image,
                                                    float* __restrict__ t_final, int32_t* __restrict__ n_proc,
                                                    unsigned long long* __restrict__ stats)
{
    __shared__ Entry E[256];
    __shared__ uint32_t C[512];    // candidates passing the rectangle test
    __shared__ uint32_t wcount[4];
    if (*a.overflow) return;
    const int64_t b = blockIdx.x;
    const int64_t L = (b & 7) * a.blocks_per_xcd + (b >> 3);
    if (L >= a.n_enum) return;
    TileCoord tc;
    if (!tile_of(L, a.cshift, a.V, gp, &tc)) return;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    // wave w takes the 8x8 quadrant w of the tile: compact pixel blocks have
    // more alike list depths than 16x4 strips, and a wave runs as long as its
    // slowest pixel
    const int px = tc.tx * TG_TILE + 8 * (w & 1) + (lane & 7), py = tc.ty * TG_TILE + 8 * (w >> 1) + (lane >> 3);
    const bool inside = px < a.W && py < a.H;
    const float fx = (float)px, fy = (float)py;
    const uint2 rg = a.ranges[tc.gcell];
    const int64_t vN = (int64_t)tc.v * a.N;
    const float ex0 = (float)(tc.tx * TG_TILE), ex1 = ex0 + (float)(TG_TILE - 1);
    const float ey0 = (float)(tc.ty * TG_TILE), ey1 = ey0 + (float)(TG_TILE - 1);
    const float log_amin = __logf(a.alpha_min);
    const uint64_t ltmask = lanemask_lt();

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    bool done = !inside;
    int32_t nproc = -1;
    uint32_t n_ev = 0, n_co = 0;
    uint32_t idx = 0;  // filtered index of the current batch start
    uint32_t pos = rg.x;
    uint32_t cn = 0;   // candidates waiting in C (block-uniform)
    // Two filtering stages, in list order: the rectangle test streams 256
    // list entries per round into the candidate queue C, and the exact
    // culling test runs on 256 candidates at a time (one per thread).
    auto block_compact = [&](bool keep, uint32_t& before, uint32_t& total) {
        const uint64_t m = ballot64(keep);
        if (lane == 0) wcount[w] = (uint32_t)__popcll(m);
        __syncthreads();
        before = 0;
        total = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) before += wcount[k];
            total += wcount[k];
        }
        before += (uint32_t)__popcll(m & ltmask);
        __syncthreads();
    };
    while (pos < rg.y || cn > 0) {
        if (cn < 256 && pos < rg.y) {
            // pipelined: the next round's ids and rectangles are in flight
            // while a round is tested
            auto id_at = [&](uint32_t p) -> uint32_t {
                const uint32_t g = p + t < rg.y ? a.cell_ids[p + t] : 0xFFFFFFFFu;
                return g < (uint64_t)a.N ? g : 0xFFFFFFFFu;
            };
            auto rect_of = [&](uint32_t g) -> ushort4 {
                return g != 0xFFFFFFFFu ? a.rect[vN + g] : make_ushort4(0, 0, 0, 0);
            };
            uint32_t id0 = id_at(pos);
            ushort4 r0 = rect_of(id0);
            uint32_t id1 = id_at(pos + 256);
            while (true) {
                const ushort4 r1 = rect_of(id1);
                const uint32_t id2 = id_at(pos + 512);
                const bool hit = tc.tx >= r0.x && tc.tx < r0.z && tc.ty >= r0.y && tc.ty < r0.w;
                uint32_t before, nhit;
                block_compact(hit, before, nhit);
                if (hit) C[cn + before] = id0;
                cn += nhit;
                pos += 256;
                __syncthreads();
                if (!(cn < 256 && pos < rg.y)) break;
                id0 = id1;
                r0 = r1;
                id1 = id2;
            }
        }
        const uint32_t nc = cn < 256 ? cn : 256;
        bool ok = false;
        uint32_t gid = 0;
        if ((uint32_t)t < nc) {
            gid = C[t];
            ok = splat_reaches_tile(a.rec[2 * (vN + gid)], a.rec[2 * (vN + gid) + 1], log_amin, a.alpha_min, ex0,
                                    ex1, ey0, ey1);
        }
        const uint32_t moved = (uint32_t)t + 256 < cn ? C[t + 256] : 0u;
        uint32_t slot, nhit;
        block_compact(ok, slot, nhit);
        if ((uint32_t)t + 256 < cn) C[t] = moved;
        cn -= nc;
        if (ok) {
            const float4 r0 = a.rec[2 * (vN + gid)];
            const float4 r1 = a.rec[2 * (vN + gid) + 1];
            const float* c = a.colors + 3 * (vN + gid);
            E[slot] = Entry{r0.x, r0.y, -0.5f * LOG2E * r0.z, -LOG2E * r0.w, -0.5f * LOG2E * r1.x, r1.y, c[0], c[1],
                            c[2]};
        }
        __syncthreads();
        if (!done) {
            for (uint32_t e = 0; e < nhit; ++e) {
                const Entry en = E[e];
                if (STATS) ++n_ev;
                const float ux = fx - en.mx, uy = fy - en.my;
                const float p2 = raster_power(ux, uy, en.ca, en.cb, en.cc);
                if (p2 > 0.0f) continue;
                const float al = __builtin_amdgcn_fmed3f(en.op * __builtin_amdgcn_exp2f(p2), 0.0f, a.alpha_max);
                if (al < a.alpha_min) continue;
                const float test = T * (1.0f - al);
                if (test < a.t_min) {
                    done = true;
                    nproc = (int32_t)(idx + e);
                    break;
                }
                const float wgt = al * T;
                if (STATS) ++n_co;
                cr += en.r * wgt;
                cg += en.g * wgt;
                cb += en.b * wgt;
                T = test;
            }
        }
        idx += nhit;
        if (__syncthreads_and(done ? 1 : 0)) break;
    }
    if (STATS) {
        const uint64_t ev = wave_sum_u64(n_ev), co = wave_sum_u64(n_co);
        if (lane == 0) {
            atomicAdd(stats, (unsigned long long)ev);
            atomicAdd(stats + 1, (unsigned long long)co);
        }
    }
    if (!inside) return;
    if (nproc < 0) nproc = (int32_t)idx;
    const int64_t pi = ((int64_t)tc.v * a.H + py) * a.W + px;
    image[3 * pi] = cr + T * a.bg0;
    image[3 * pi + 1] = cg + T * a.bg1;
    image[3 * pi + 2] = cb + T * a.bg2;
    if (t_final) t_final[pi] = T;
    n_proc[pi] = nproc;
}

// ------------------------------------------------------------------ backward
constexpr int QCAP = 128;

// STATS: adds (pixel steps, pairs evaluated, pairs contributing) to
// stats[0..2]; a step is one pixel against one batch of 64 lanes, a pair is
// evaluated when the forward processed it for that pixel and contributes
// when it reaches the pixel (the lanes that carry gradient terms).
template <bool STATS>
__global__ void __launch_bounds__(64) k_raster_bwd(RasterArgs a, GridPack gp, const float* __restrict__ image,
                                                   const float* __restrict__ dimage,
                                                   const int32_t* __restrict__ n_proc, float* __restrict__ grad2d,
                                                   unsigned long long* __restrict__ stats)
{
    __shared__ uint32_t qi[QCAP];
    __shared__ uint32_t cq[QCAP];   // candidates passing the rectangle test
    // per pixel: the colour still to come (final colour minus the front
    // already composited) dotted with the pixel's dL/dC, the running
    // transmittance, and dL/dC itself.  Every channel enters dL/dalpha only
    // through that dot product, so one sum scan per step replaces three.
    __shared__ float2 RT[256];   // g . remaining colour, T
    // dL/dC per channel: three word arrays keep the wave's LDS at 6 KB (26
    // waves per CU; a float4 array would hold a dead word per pixel)
    __shared__ float GFr[256], GFg[256], GFb[256];
    if (*a.overflow) return;
    const int64_t b = blockIdx.x;
    const int64_t L = (b & 7) * a.blocks_per_xcd + (b >> 3);
    if (L >= a.n_enum) return;
    TileCoord tc;
    if (!tile_of(L, a.cshift, a.V, gp, &tc)) return;
    const int lane = threadIdx.x;
    const uint2 rg = a.ranges[tc.gcell];
    const int64_t vN = (int64_t)tc.v * a.N;
    const int px0 = tc.tx * TG_TILE, py0 = tc.ty * TG_TILE;
    const float ex0 = (float)px0, ex1 = ex0 + (float)(TG_TILE - 1);
    const float ey0 = (float)py0, ey1 = ey0 + (float)(TG_TILE - 1);
    const float log_amin = __logf(a.alpha_min);
    const float amin = a.alpha_min, amax = a.alpha_max;
    const uint64_t ltmask = lanemask_lt();

    uint64_t alive[4];
    int npg[4];  // n_proc of pixel g*64 + lane
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int j = g * 64 + lane;
        const int px = px0 + (j & 15), py = py0 + (j >> 4);
        const bool in = px < a.W && py < a.H;
        float4 cf = make_float4(0.f, 0.f, 0.f, 1.f), gf = make_float4(0.f, 0.f, 0.f, 0.f);
        int np = 0;
        if (in) {
            const int64_t pi = ((int64_t)tc.v * a.H + py) * a.W + px;
            cf = make_float4(image[3 * pi], image[3 * pi + 1], image[3 * pi + 2], 1.0f);
            gf = make_float4(dimage[3 * pi], dimage[3 * pi + 1], dimage[3 * pi + 2], 0.0f);
            np = n_proc[pi];
        }
        RT[j] = make_float2(fmaf(gf.z, cf.z, fmaf(gf.y, cf.y, gf.x * cf.x)), 1.0f);
        GFr[j] = gf.x;
        GFg[j] = gf.y;
        GFb[j] = gf.z;
        npg[g] = np;
        alive[g] = ballot64(in && np > 0);
    }
    float pex_reg = 1.0f;
    const bool lane0 = lane == 0;
    int qn = 0, cn = 0;
    uint32_t pos = rg.x;
    uint32_t bstart = 0;  // filtered index of the batch's first entry
    uint64_t n_st = 0, n_ev = 0, n_co = 0;   // wave-uniform

    while ((alive[0] | alive[1] | alive[2] | alive[3]) != 0ull) {
        // two stages, as in the forward's order: the rectangle test streams
        // the list into a candidate queue, the exact culling test runs on 64
        // candidates at a time (both queues keep list order)
        while (qn < 64 && (pos < rg.y || cn > 0)) {
            if (cn < 64 && pos < rg.y) {
                // pipelined two rounds deep, as in the accumulation
                auto id_at = [&](uint32_t p) -> uint32_t {
                    const uint32_t g = p + lane < rg.y ? a.cell_ids[p + lane] : 0xFFFFFFFFu;
                    return g < (uint64_t)a.N ? g : 0xFFFFFFFFu;
                };
                auto rect_of = [&](uint32_t g) -> ushort4 {
                    return g != 0xFFFFFFFFu ? a.rect[vN + g] : make_ushort4(0, 0, 0, 0);
                };
                uint32_t id0 = id_at(pos);
                ushort4 r0 = rect_of(id0);
                uint32_t id1 = id_at(pos + 64);
                while (true) {
                    const ushort4 r1 = rect_of(id1);
                    const uint32_t id2 = id_at(pos + 128);
                    const bool hit = tc.tx >= r0.x && tc.tx < r0.z && tc.ty >= r0.y && tc.ty < r0.w;
                    const uint64_t m = ballot64(hit);
                    if (hit) cq[cn + __popcll(m & ltmask)] = id0;
                    cn += __popcll(m);
                    pos += 64;
                    if (!(cn < 64 && pos < rg.y)) break;
                    id0 = id1;
                    r0 = r1;
                    id1 = id2;
                }
            }
            const int nc = cn < 64 ? cn : 64;
            bool ok = false;
            uint32_t cg = 0;
            if (lane < nc) {
                cg = cq[lane];
                ok = splat_reaches_tile(a.rec[2 * (vN + cg)], a.rec[2 * (vN + cg) + 1], log_amin, amin, ex0, ex1,
                                        ey0, ey1);
            }
            const uint64_t m = ballot64(ok);
            if (ok) qi[qn + __popcll(m & ltmask)] = cg;
            qn += __popcll(m);
            if (lane + 64 < cn) cq[lane] = cq[lane + 64];
            cn -= nc;
        }
        if (qn == 0) break;
        const int nb = qn < 64 ? qn : 64;
        uint32_t gid = 0;
        float mx = 0.f, my = 0.f, A = 0.f, B = 0.f, C = 0.f, op = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
        if (lane < nb) {
            gid = qi[lane];
            const float4 r0 = a.rec[2 * (vN + gid)];
            const float4 r1 = a.rec[2 * (vN + gid) + 1];
            mx = r0.x;
            my = r0.y;
            A = r0.z;
            B = r0.w;
            C = r1.x;
            op = r1.y;
            const float* c = a.colors + 3 * (vN + gid);
            c0 = c[0];
            c1 = c[1];
            c2 = c[2];
        }
        if (lane + 64 < qn) {
            const uint32_t g2 = qi[lane + 64];
            qi[lane] = g2;
        }
        qn -= nb;
        const float ca = -0.5f * LOG2E * A, cb = -LOG2E * B, cc = -0.5f * LOG2E * C;

        // per lane: sums over pixels of dpow u (s_x, s_y) and dpow u u^T
        // (s_xx, s_xy, s_yy), and the opacity and colour gradients
        float s_x = 0.f, s_y = 0.f, s_xx = 0.f, s_xy = 0.f, s_yy = 0.f, g_o = 0.f, g_r = 0.f, g_g = 0.f, g_b = 0.f;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint64_t m = alive[g];
            uint64_t dead = 0;
            while (m) {
                const int j = __builtin_ctzll(m);
                m &= m - 1;
                const int pj = g * 64 + j;
                const int np = __builtin_amdgcn_readlane(npg[g], j);
                if ((uint32_t)np <= bstart + (uint32_t)nb) dead |= 1ull << j;  // last batch for this pixel
                const float2 rt = RT[pj];
                const float3 gf = make_float3(GFr[pj], GFg[pj], GFb[pj]);
                // the pixel coordinate converted from the integer, as the
                // forward forms it, so alpha is bit-identical
                const float ux = (float)(px0 + (j & 15)) - mx, uy = (float)(py0 + 4 * g + (j >> 4)) - my;
                const float p2 = raster_power(ux, uy, ca, cb, cc);
                const float ex = __builtin_amdgcn_exp2f(p2);
                const float e2 = op * ex;
                const float al = __builtin_amdgcn_fmed3f(e2, 0.0f, amax);
                // lanes past the batch (opacity 0) fail alpha >= alpha_min;
                // the lanes the forward processed for this pixel are the
                // first np - bstart of the batch
                const uint32_t nfw = (uint32_t)np - bstart;
                const uint64_t fwm = nfw >= 64u ? ~0ull : ((1ull << nfw) - 1ull);
                const uint64_t vm = ballot64(p2 <= 0.0f) & ballot64(al >= amin) & fwm;
                if (STATS) {
                    n_st += 1;
                    n_ev += (uint64_t)(nfw < (uint32_t)nb ? nfw : (uint32_t)nb);
                    n_co += (uint64_t)__popcll(vm);
                }
                if (vm == 0ull) continue;   // no lane reaches the pixel: nothing changes
                const bool valid = __builtin_amdgcn_inverse_ballot_w64(vm);
                float P = valid ? 1.0f - al : 1.0f;
                P = wave_scan_mul_fused(P);
                asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf"
                             : "+v"(pex_reg) : "v"(P));
                const float Ti = rt.y * pex_reg;
                const float wgt = valid ? al * Ti : 0.0f;
                // the lane's colour dotted with the pixel's dL/dC
                const float dc = fmaf(gf.z, c2, fmaf(gf.y, c1, gf.x * c0));
                const float F = wave_scan_add_fused(dc * wgt);
                if (valid) {
                    // colour behind lane i (incl. background), dotted with
                    // dL/dC: (C - front - own) . g
                    const float S = rt.x - F;
                    // 1 - alpha >= 0.01 (alpha is clamped at 0.99): the
                    // hardware reciprocal's ulp error is far below the
                    // gradient's FP32 accumulation error
                    const float inv1m = __builtin_amdgcn_rcpf(1.0f - al);
                    const float dal = dc * Ti - S * inv1m;
                    g_r += gf.x * wgt;
                    g_g += gf.y * wgt;
                    g_b += gf.z * wgt;
                    if (e2 < amax) {  // not clamped: alpha = o e^power
                        // d power = dL/dalpha * alpha; the centre and conic
                        // gradients are linear in the moments of u = p - mu
                        // weighted by it, combined with the conic at the end
                        const float dpow = dal * al;
                        g_o += dal * ex;   // d alpha / d o = e^power when not clamped
                        const float tx = dpow * ux, ty = dpow * uy;
                        s_x += tx;
                        s_y += ty;
                        s_xx += tx * ux;
                        s_xy += tx * uy;
                        s_yy += ty * uy;
                    }
                }
                // advance this pixel's transmittance and remaining colour
                const float Tn = rt.y * readlane_f(P, 63);
                const float Rn = rt.x - readlane_f(F, 63);
                if (lane0) RT[pj] = make_float2(Rn, Tn);
            }
            alive[g] &= ~dead;
        }
        if (lane < nb) {
            float* dst = grad2d + (vN + gid) * 9;
            // power = -1/2 (A ux^2 + C uy^2) - B ux uy with u = p - mu
            unsafeAtomicAdd(dst + 0, A * s_x + B * s_y);
            unsafeAtomicAdd(dst + 1, C * s_y + B * s_x);
            unsafeAtomicAdd(dst + 2, -0.5f * s_xx);
            unsafeAtomicAdd(dst + 3, -s_xy);
            unsafeAtomicAdd(dst + 4, -0.5f * s_yy);
            unsafeAtomicAdd(dst + 5, g_o);
            unsafeAtomicAdd(dst + 6, g_r);
            unsafeAtomicAdd(dst + 7, g_g);
            unsafeAtomicAdd(dst + 8, g_b);
        }
        bstart += (uint32_t)nb;
    }
    if (STATS && lane0) {
        atomicAdd(stats, (unsigned long long)n_st);
        atomicAdd(stats + 1, (unsigned long long)n_ev);
        atomicAdd(stats + 2, (unsigned long long)n_co);
    }
}

// ------------------------------------------------------- projection backward
// Real SH basis Y_k (degree DEG) at a unit direction, and the direction
// gradient sum_k a_k dY_k/d(x, y, z) (polynomial form) without storing dY.
template <int DEG>
__device__ inline void sh_basis_dir_grad(float x, float y, float z, float Y[(DEG + 1) * (DEG + 1)],
                                         const float a[(DEG + 1) * (DEG + 1)], float g[3]) {
    const float c0 = 0.28209479177387814f, c1 = 0.48860251190291992f;
    const float k4 = 1.0925484305920792f, k6 = 0.31539156525252005f, k8 = 0.54627421529603959f;
    const float k9 = -0.59004358992664352f, k10 = 2.8906114426405538f, k11 = -0.45704579946446572f;
    const float k12 = 0.37317633259011540f, k13 = -0.45704579946446572f, k14 = 1.4453057213202769f;
    const float k15 = -0.59004358992664352f;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    Y[0] = c0;
    if constexpr (DEG > 0) {
        Y[1] = -c1 * y; gy -= c1 * a[1];
        Y[2] = c1 * z;  gz += c1 * a[2];
        Y[3] = -c1 * x; gx -= c1 * a[3];
    }
    if constexpr (DEG > 1) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = k4 * x * y;   gx += a[4] * k4 * y; gy += a[4] * k4 * x;
        Y[5] = -k4 * y * z;  gy -= a[5] * k4 * z; gz -= a[5] * k4 * y;
        Y[6] = k6 * (2.f * zz - xx - yy);
        gx -= a[6] * 2.f * k6 * x; gy -= a[6] * 2.f * k6 * y; gz += a[6] * 4.f * k6 * z;
        Y[7] = -k4 * x * z;  gx -= a[7] * k4 * z; gz -= a[7] * k4 * x;
        Y[8] = k8 * (xx - yy); gx += a[8] * 2.f * k8 * x; gy -= a[8] * 2.f * k8 * y;
        if constexpr (DEG > 2) {
            Y[9] = k9 * y * (3.f * xx - yy);
            gx += a[9] * 6.f * k9 * x * y; gy += a[9] * k9 * (3.f * xx - 3.f * yy);
            Y[10] = k10 * x * y * z;
            gx += a[10] * k10 * y * z; gy += a[10] * k10 * x * z; gz += a[10] * k10 * x * y;
            Y[11] = k11 * y * (4.f * zz - xx - yy);
            gx -= a[11] * 2.f * k11 * x * y; gy += a[11] * k11 * (4.f * zz - xx - 3.f * yy);
            gz += a[11] * 8.f * k11 * y * z;
            Y[12] = k12 * z * (2.f * zz - 3.f * xx - 3.f * yy);
            gx -= a[12] * 6.f * k12 * x * z; gy -= a[12] * 6.f * k12 * y * z;
            gz += a[12] * k12 * (6.f * zz - 3.f * xx - 3.f * yy);
            Y[13] = k13 * x * (4.f * zz - xx - yy);
            gx += a[13] * k13 * (4.f * zz - 3.f * xx - yy); gy -= a[13] * 2.f * k13 * x * y;
            gz += a[13] * 8.f * k13 * x * z;
            Y[14] = k14 * z * (xx - yy);
            gx += a[14] * 2.f * k14 * x * z; gy -= a[14] * 2.f * k14 * y * z; gz += a[14] * k14 * (xx - yy);
            Y[15] = k15 * x * (xx - 3.f * yy);
            gx += a[15] * k15 * (3.f * xx - 3.f * yy); gy -= a[15] * 6.f * k15 * x * y;
        }
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

struct ProjArgs {
    const float* means;
    const float* quats;
    const float* scales;   // log-scales when scale_mode == 1
    const float* opacity;  // logits when opacity_mode == 1
    const float* sh;
    int sh_deg, scale_mode, opacity_mode;
    const ushort4* rect;
    const uint8_t* clamped;
    const float* grad2d;
    float* g_means;
    float* g_quats;
    float* g_scales;
    float* g_opacity;
    float* g_sh;
    int64_t N;
    int V;
};

// DEG: SH degree (-1: no SH coefficients)
template <int DEG>
__global__ void __launch_bounds__(128) k_project_bwd(ProjArgs a, CamPack cams, tg_params prm)
{
    constexpr int NB = DEG >= 0 ? (DEG + 1) * (DEG + 1) : 1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N) return;
    const float m0 = a.means[3 * g], m1 = a.means[3 * g + 1], m2 = a.means[3 * g + 2];
    const float qw0 = a.quats[4 * g], qx0 = a.quats[4 * g + 1], qy0 = a.quats[4 * g + 2], qz0 = a.quats[4 * g + 3];
    float s[3] = {a.scales[3 * g], a.scales[3 * g + 1], a.scales[3 * g + 2]};
    if (a.scale_mode == 1)
        for (int i = 0; i < 3; ++i) s[i] = expf(s[i]);
    float o = a.opacity[g];
    if (a.opacity_mode == 1) o = 1.0f / (1.0f + expf(-o));
    // rotation of the normalised quaternion and Sigma_3D = M M^T, M = R S
    const float qn = sqrtf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const float w = qw0 / qn, x = qx0 / qn, y = qy0 / qn, z = qz0 / qn;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    float M[9], S3[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] * s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S3[i * 3 + j] = M[i * 3] * M[j * 3] + M[i * 3 + 1] * M[j * 3 + 1] + M[i * 3 + 2] * M[j * 3 + 2];

    float gS3[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float gmu[3] = {0.f, 0.f, 0.f};
    float go = 0.f;
    // the coefficients (read once) and their gradient, in registers
    float shc[3 * NB], gsh[3 * NB];
#pragma unroll
    for (int i = 0; i < 3 * NB; ++i) {
        shc[i] = DEG >= 0 ? a.sh[g * 3 * NB + i] : 0.f;
        gsh[i] = 0.f;
    }
    for (int v = 0; v < a.V; ++v) {
        const int64_t o_ = (int64_t)v * a.N + g;
        // every load of the view issued before the culling test (a culled
        // view reads its 40 unused bytes, but the view waits out one round
        // trip instead of one per test)
        const uint2 rr = *(const uint2*)(a.rect + o_);
        const float* gr = a.grad2d + o_ * 9;
        float gv[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) gv[i] = gr[i];
        uint8_t clp[3] = {0, 0, 0};
        if (DEG >= 0 && a.clamped) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) clp[ch] = a.clamped[3 * o_ + ch];
        }
        const uint32_t rx0 = rr.x & 0xFFFFu, ry0 = rr.x >> 16, rx1 = rr.y & 0xFFFFu, ry1 = rr.y >> 16;
        if (!((rx1 > rx0) & (ry1 > ry0))) continue;
        const float gmx = gv[0], gmy = gv[1], gA = gv[2], gB = gv[3], gC = gv[4], gop = gv[5];
        const float gcol[3] = {gv[6], gv[7], gv[8]};
        const tg_camera& c = cams.cam[v];
        const float* Rc = c.R;
        const float p0 = Rc[0] * m0 + Rc[1] * m1 + Rc[2] * m2 + c.t[0];
        const float p1 = Rc[3] * m0 + Rc[4] * m1 + Rc[5] * m2 + c.t[1];
        const float pz = Rc[6] * m0 + Rc[7] * m1 + Rc[8] * m2 + c.t[2];
        const float iz = 1.0f / pz;
        // --- 2D mean: mu = (fx p0/pz + cx, fy p1/pz + cy)
        float gp[3] = {gmx * c.fx * iz, gmy * c.fy * iz, -(gmx * c.fx * p0 + gmy * c.fy * p1) * iz * iz};
        // --- conic = inverse(Sigma_2D + dil I): dL/dSigma = -Q G Q (symmetric)
        const float limx = prm.j_clamp * ((0.5f * (float)c.width) / c.fx);
        const float limy = prm.j_clamp * ((0.5f * (float)c.height) / c.fy);
        const float ux = p0 * iz, uy = p1 * iz;
        const float tx = fminf(limx, fmaxf(-limx, ux)), ty = fminf(limy, fmaxf(-limy, uy));
        const bool clx = tx != ux, cly = ty != uy;
        const float J00 = c.fx * iz, J02 = -c.fx * tx * iz, J11 = c.fy * iz, J12 = -c.fy * ty * iz;
        float T0[3], T1[3];
        for (int j = 0; j < 3; ++j) {
            T0[j] = J00 * Rc[j] + J02 * Rc[6 + j];
            T1[j] = J11 * Rc[3 + j] + J12 * Rc[6 + j];
        }
        float U0[3], U1[3];
        for (int j = 0; j < 3; ++j) {
            U0[j] = T0[0] * S3[j] + T0[1] * S3[3 + j] + T0[2] * S3[6 + j];
            U1[j] = T1[0] * S3[j] + T1[1] * S3[3 + j] + T1[2] * S3[6 + j];
        }
        const float sa = U0[0] * T0[0] + U0[1] * T0[1] + U0[2] * T0[2] + prm.dilation;
        const float sb = U0[0] * T1[0] + U0[1] * T1[1] + U0[2] * T1[2];
        const float sc = U1[0] * T1[0] + U1[1] * T1[1] + U1[2] * T1[2] + prm.dilation;
        const float det = sa * sc - sb * sb;
        const float id = 1.0f / det;
        const float QA = sc * id, QB = -sb * id, QC = sa * id;
        // G = [[gA, gB/2], [gB/2, gC]]; dSigma = -Q G Q
        const float G01 = 0.5f * gB;
        const float X00 = QA * gA + QB * G01, X01 = QA * G01 + QB * gC;
        const float X10 = QB * gA + QC * G01, X11 = QB * G01 + QC * gC;
        const float dS00 = -(X00 * QA + X01 * QB), dS01 = -(X00 * QB + X01 * QC);
        const float dS10 = -(X10 * QA + X11 * QB), dS11 = -(X10 * QB + X11 * QC);
        // symmetric 2x2 gradient of Sigma_2D (full matrix form)
        const float H00 = dS00, H01 = 0.5f * (dS01 + dS10), H11 = dS11;
        // Sigma_2D = T S3 T^T: dS3 += T^T H T ; dT = 2 H T S3
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                gS3[i * 3 + j] += T0[i] * (H00 * T0[j] + H01 * T1[j]) + T1[i] * (H01 * T0[j] + H11 * T1[j]);
        float dT0[3], dT1[3];
        for (int j = 0; j < 3; ++j) {
            dT0[j] = 2.f * (H00 * U0[j] + H01 * U1[j]);
            dT1[j] = 2.f * (H01 * U0[j] + H11 * U1[j]);
        }
        // T = J W: dJ00 = dT0 . W row0, dJ02 = dT0 . W row2, dJ11 = dT1 . W row1, dJ12 = dT1 . W row2
        const float dJ00 = dT0[0] * Rc[0] + dT0[1] * Rc[1] + dT0[2] * Rc[2];
        const float dJ02 = dT0[0] * Rc[6] + dT0[1] * Rc[7] + dT0[2] * Rc[8];
        const float dJ11 = dT1[0] * Rc[3] + dT1[1] * Rc[4] + dT1[2] * Rc[5];
        const float dJ12 = dT1[0] * Rc[6] + dT1[1] * Rc[7] + dT1[2] * Rc[8];
        // J00 = fx/pz, J11 = fy/pz, J02 = -fx tx/pz (tx = p0/pz unless clamped)
        gp[2] += -dJ00 * c.fx * iz * iz - dJ11 * c.fy * iz * iz;
        if (clx) {
            gp[2] += dJ02 * c.fx * tx * iz * iz;
        } else {
            gp[0] += -dJ02 * c.fx * iz * iz;
            gp[2] += 2.f * dJ02 * c.fx * p0 * iz * iz * iz;
        }
        if (cly) {
            gp[2] += dJ12 * c.fy * ty * iz * iz;
        } else {
            gp[1] += -dJ12 * c.fy * iz * iz;
            gp[2] += 2.f * dJ12 * c.fy * p1 * iz * iz * iz;
        }
        // p = R mu + t
        for (int j = 0; j < 3; ++j) gmu[j] += Rc[j] * gp[0] + Rc[3 + j] * gp[1] + Rc[6 + j] * gp[2];
        go += gop;
        // --- colour: c = max(0, SH(dir) . coeffs + 0.5), dir = (mu - centre)/|mu - centre|
        if constexpr (DEG >= 0) {
            const float ccx = -(Rc[0] * c.t[0] + Rc[3] * c.t[1] + Rc[6] * c.t[2]);
            const float ccy = -(Rc[1] * c.t[0] + Rc[4] * c.t[1] + Rc[7] * c.t[2]);
            const float ccz = -(Rc[2] * c.t[0] + Rc[5] * c.t[1] + Rc[8] * c.t[2]);
            const float ex = m0 - ccx, ey = m1 - ccy, ez = m2 - ccz;
            const float il = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
            const float dx = ex * il, dy = ey * il, dz = ez * il;
            // clamped channels (colour = 0) pass no gradient
            float gc[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gc[ch] = clp[ch] ? 0.f : gcol[ch];
            float av[NB], Y[NB], gdir[3];
#pragma unroll
            for (int k = 0; k < NB; ++k)
                av[k] = gc[0] * shc[k * 3] + gc[1] * shc[k * 3 + 1] + gc[2] * shc[k * 3 + 2];
            sh_basis_dir_grad<DEG>(dx, dy, dz, Y, av, gdir);
#pragma unroll
            for (int k = 0; k < NB; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) gsh[k * 3 + ch] += gc[ch] * Y[k];
            // project out the radial part: d dir / d e = (I - d d^T) / |e|
            const float dd = gdir[0] * dx + gdir[1] * dy + gdir[2] * dz;
            gmu[0] += (gdir[0] - dd * dx) * il;
            gmu[1] += (gdir[1] - dd * dy) * il;
            gmu[2] += (gdir[2] - dd * dz) * il;
        }
    }
    // Sigma_3D = M M^T: dM = (G + G^T) M ; M = R S
    float gR[9], gs[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            float d = 0.f;
            for (int j = 0; j < 3; ++j) d += (gS3[i * 3 + j] + gS3[j * 3 + i]) * M[j * 3 + k];
            gR[i * 3 + k] = d * s[k];
            gs[k] += d * R[i * 3 + k];
        }
    // R(q): partial derivatives w.r.t. the normalised (w, x, y, z)
    const float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    const float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] -
                            2.f * x * gR[8]);
    const float gy = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] -
                            2.f * y * gR[8]);
    const float gz = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] + y * gR[5] +
                            x * gR[6] + y * gR[7]);
    // through the normalisation q / |q|
    const float dotg = gw * w + gx * x + gy * y + gz * z;
    a.g_quats[4 * g] = (gw - dotg * w) / qn;
    a.g_quats[4 * g + 1] = (gx - dotg * x) / qn;
    a.g_quats[4 * g + 2] = (gy - dotg * y) / qn;
    a.g_quats[4 * g + 3] = (gz - dotg * z) / qn;
    for (int k = 0; k < 3; ++k) a.g_scales[3 * g + k] = a.scale_mode == 1 ? gs[k] * s[k] : gs[k];
    a.g_means[3 * g] = gmu[0];
    a.g_means[3 * g + 1] = gmu[1];
    a.g_means[3 * g + 2] = gmu[2];
    a.g_opacity[g] = a.opacity_mode == 1 ? go * o * (1.f - o) : go;
    if constexpr (DEG >= 0) {
#pragma unroll
        for (int i = 0; i < 3 * NB; ++i) a.g_sh[g * 3 * NB + i] = gsh[i];
    }
}

// ------------------------------------------------------------ elementwise
__global__ void __launch_bounds__(256) k_l1(const float* __restrict__ img, const float* __restrict__ tgt, int64_t n,
                                            float scale, float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float red[4];
    // grid-stride: a bounded grid keeps the loss reduction to one atomic per
    // block (a few thousand) instead of one per 256 elements
    float l = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = img[i] - tgt[i];
        l += fabsf(d);
        grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    }
    // wave sums then one atomic per block
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) * scale);
}

// Adam over rows of `row` floats: the first `head` floats of each row step
// with lr_head, the rest with lr_tail (3DGS steps the DC colour coefficients
// and the higher SH bands at different rates).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, int row, int head, float lr_head, float lr_tail, float b1,
                       float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float lr = (int)(i % row) < head ? lr_head : lr_tail;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

tg_status raster_setup(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams, int32_t V,
                       const tg_params* p, RasterArgs* a, GridPack* gp) {
    if (!s || !bins || !cams || !p || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (!s->rec || !s->rect || !s->colors || !bins->cell_ids || !bins->cell_ranges || !bins->overflow)
        return TG_ERR_INVALID_ARG;
    if (!aligned16(s->rec)) return TG_ERR_ALIGNMENT;
    for (int v = 1; v < V; ++v)
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) return TG_ERR_INVALID_ARG;
    if (N > (int64_t)0xFFFFFFFF) return TG_ERR_UNSUPPORTED;
    int cs = 0;
    const int64_t ncell = coarse_plan(cams, V, N, p, gp, &cs);
    if (ncell < 0) return TG_ERR_UNSUPPORTED;
    a->rec = (const float4*)s->rec;
    a->colors = s->colors;
    a->rect = (const ushort4*)s->rect;
    a->cell_ids = bins->cell_ids;
    a->ranges = (const uint2*)bins->cell_ranges;
    a->overflow = bins->overflow;
    a->N = N;
    a->V = V;
    a->W = cams[0].width;
    a->H = cams[0].height;
    a->cshift = cs;
    a->n_enum = ncell << (2 * cs);
    a->blocks_per_xcd = (a->n_enum + 7) / 8;
    a->alpha_min = p->alpha_min;
    a->alpha_max = p->alpha_max;
    a->t_min = p->t_min;
    return TG_OK;
}

// out = in * factor (factor a device scalar: the upstream gradient of a
// loss, so the chain rule needs no host read)
__global__ void __launch_bounds__(256) k_scale_by(float* __restrict__ out, const float* __restrict__ in, int64_t n,
                                                  const float* __restrict__ factor) {
    const float f = *factor;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = in[i] * f;
}

// out[0] = c + sum_i w_i x[i] for a few device scalars x.
constexpr int AFFINE_MAX = 8;
struct AffineW {
    float w[AFFINE_MAX];
};
__global__ void k_scalar_affine(float* __restrict__ out, const float* __restrict__ x, int k, AffineW w, float c) {
    float r = c;
    for (int i = 0; i < k; ++i) r = fmaf(w.w[i], x[i], r);
    *out = r;
}

}  // namespace

extern "C" tg_status tg_raster_fwd_counted(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                           int32_t V, const float* bg, const tg_params* p, float* image,
                                           float* t_final, int32_t* n_proc, int64_t* stats, void* stream)
{
    RasterArgs a;
    GridPack gp;
    tg_status st = raster_setup(s, bins, N, cams, V, p, &a, &gp);
    if (st != TG_OK) return st;
    if (!image || !n_proc) return TG_ERR_INVALID_ARG;
    a.bg0 = bg ? bg[0] : 0.f;
    a.bg1 = bg ? bg[1] : 0.f;
    a.bg2 = bg ? bg[2] : 0.f;
    if (N == 0) return TG_OK;
    if (stats)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_raster_fwd<true>), dim3((unsigned)(a.blocks_per_xcd * 8)), dim3(256), 0,
                           (hipStream_t)stream, a, gp, image, t_final, n_proc, (unsigned long long*)stats);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_raster_fwd<false>), dim3((unsigned)(a.blocks_per_xcd * 8)), dim3(256),
                           0, (hipStream_t)stream, a, gp, image, t_final, n_proc, (unsigned long long*)nullptr);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_raster_fwd(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                   int32_t V, const float* bg, const tg_params* p, float* image, float* t_final,
                                   int32_t* n_proc, void* stream)
{
    return tg_raster_fwd_counted(s, bins, N, cams, V, bg, p, image, t_final, n_proc, nullptr, stream);
}

extern "C" tg_status tg_raster_bwd_counted(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                           int32_t V, const float* image, const float* dl_dimage,
                                           const int32_t* n_proc, const tg_params* p, float* grad2d, int64_t* stats,
                                           void* stream)
{
    RasterArgs a;
    GridPack gp;
    tg_status st = raster_setup(s, bins, N, cams, V, p, &a, &gp);
    if (st != TG_OK) return st;
    if (!image || !dl_dimage || !n_proc || !grad2d) return TG_ERR_INVALID_ARG;
    if (N == 0) return TG_OK;
    if (stats)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_raster_bwd<true>), dim3((unsigned)(a.blocks_per_xcd * 8)), dim3(64), 0,
                           (hipStream_t)stream, a, gp, image, dl_dimage, n_proc, grad2d, (unsigned long long*)stats);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_raster_bwd<false>), dim3((unsigned)(a.blocks_per_xcd * 8)), dim3(64), 0,
                           (hipStream_t)stream, a, gp, image, dl_dimage, n_proc, grad2d,
                           (unsigned long long*)nullptr);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_raster_bwd(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                   int32_t V, const float* image, const float* dl_dimage, const int32_t* n_proc,
                                   const tg_params* p, float* grad2d, void* stream)
{
    return tg_raster_bwd_counted(s, bins, N, cams, V, image, dl_dimage, n_proc, p, grad2d, nullptr, stream);
}

extern "C" tg_status tg_project_bwd(const tg_gaussians* g, const tg_splats* s, int64_t N, const tg_camera* cams,
                                    int32_t V, const float* grad2d, const tg_params* p, tg_gaussians* grads,
                                    void* stream)
{
    if (!g || !s || !cams || !grad2d || !p || !grads || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (!g->means || !g->quats || !g->scales || !g->opacity || !s->rect) return TG_ERR_INVALID_ARG;
    if (!grads->means || !grads->quats || !grads->scales || !grads->opacity) return TG_ERR_INVALID_ARG;
    if (g->sh && (g->sh_degree < 0 || g->sh_degree > 3 || !grads->sh)) return TG_ERR_INVALID_ARG;
    if (N == 0) return TG_OK;
    ProjArgs a;
    a.means = g->means;
    a.quats = g->quats;
    a.scales = g->scales;
    a.opacity = g->opacity;
    a.sh = g->sh;
    a.sh_deg = g->sh ? g->sh_degree : 0;
    a.scale_mode = g->scale_mode;
    a.opacity_mode = g->opacity_mode;
    a.rect = (const ushort4*)s->rect;
    a.clamped = s->clamped;
    a.grad2d = grad2d;
    a.g_means = grads->means;
    a.g_quats = grads->quats;
    a.g_scales = grads->scales;
    a.g_opacity = grads->opacity;
    a.g_sh = g->sh ? grads->sh : nullptr;
    a.N = N;
    a.V = V;
    CamPack cp;
    for (int v = 0; v < V; ++v) cp.cam[v] = cams[v];
    const dim3 grid((unsigned)((N + 127) / 128));
    switch (a.sh ? a.sh_deg : -1) {
        case 0: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project_bwd<0>), grid, dim3(128), 0, (hipStream_t)stream, a, cp, *p); break;
        case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project_bwd<1>), grid, dim3(128), 0, (hipStream_t)stream, a, cp, *p); break;
        case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project_bwd<2>), grid, dim3(128), 0, (hipStream_t)stream, a, cp, *p); break;
        case 3: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project_bwd<3>), grid, dim3(128), 0, (hipStream_t)stream, a, cp, *p); break;
        default: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_project_bwd<-1>), grid, dim3(128), 0, (hipStream_t)stream, a, cp, *p); break;
    }
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_l1_loss_grad(const float* image, const float* target, int64_t n, float scale, float* grad,
                                     float* loss_sum, void* stream)
{
    if (!image || !target || !grad || n < 0) return TG_ERR_INVALID_ARG;
    if (n == 0) return TG_OK;
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_l1, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, image, target, n, scale, grad,
                       loss_sum);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

static tg_status adam_launch(float* param, const float* grad, float* m, float* v, int64_t n, int32_t row,
                             int32_t head, float lr_head, float lr_tail, float beta1, float beta2, float eps,
                             int32_t step, void* stream)
{
    if (!param || !grad || !m || !v || n < 0 || step < 1 || row < 1 || head < 0 || head > row)
        return TG_ERR_INVALID_ARG;
    if (n % row) return TG_ERR_INVALID_ARG;
    if (n == 0) return TG_OK;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, param, grad, m, v,
                       n, row, head, lr_head, lr_tail, beta1, beta2, eps, c1, c2);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                                  float beta1, float beta2, float eps, int32_t step, void* stream)
{
    return adam_launch(param, grad, m, v, n, 1, 1, lr, lr, beta1, beta2, eps, step, stream);
}

extern "C" tg_status tg_adam_step_rows(float* param, const float* grad, float* m, float* v, int64_t n, int32_t row,
                                       int32_t head, float lr_head, float lr_tail, float beta1, float beta2,
                                       float eps, int32_t step, void* stream)
{
    return adam_launch(param, grad, m, v, n, row, head, lr_head, lr_tail, beta1, beta2, eps, step, stream);
}

extern "C" tg_status tg_scale_by(float* out, const float* in, int64_t n, const float* factor, void* stream)
{
    if (!out || !in || !factor || n < 0) return TG_ERR_INVALID_ARG;
    if (n == 0) return TG_OK;
    const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
    hipLaunchKernelGGL(k_scale_by, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, out, in, n, factor);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_scalar_affine(float* out, const float* x, int32_t k, const float* w, float c, void* stream)
{
    if (!out || k < 0 || (k > 0 && (!x || !w))) return TG_ERR_INVALID_ARG;
    if (k > AFFINE_MAX) return TG_ERR_UNSUPPORTED;
    AffineW aw;
    for (int i = 0; i < AFFINE_MAX; ++i) aw.w[i] = i < k ? w[i] : 0.0f;
    hipLaunchKernelGGL(k_scalar_affine, dim3(1), dim3(1), 0, (hipStream_t)stream, out, x, k, aw, c);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
