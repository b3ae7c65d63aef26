// tg_splat_accumulate: PWI-LS statistics inside the renderer
// (TrackerSplat Sec. 4.3.3-4.3.5, Eq. 4; static-pixel counters of Sec. 4.5.2).
//
// The paper accumulates w P_i and w Q_i per Gaussian with atomic additions
// from a modified 3DGS renderer (one thread per pixel).  On CDNA4 we turn the
// loop inside out so that the per-Gaussian sums never need a cross-lane
// reduction:
//
//  * one wave64 owns one 16x16 tile; its 256 pixels are wave-uniform scalars
//    (the transmittance in LDS, the flags in 4 VGPRs read with v_readlane,
//    the track fetched with a scalar load when the pixel contributes),
//    visited with s_ff1 over an alive mask so finished pixels cost nothing;
//  * the 64 lanes hold 64 consecutive Gaussians of the tile's depth-ordered
//    list; for a pixel, every lane evaluates its Gaussian's alpha, and the
//    transmittance in front of each lane is an exclusive product scan across
//    the wave (6 DPP row_shr/row_bcast steps), so termination is a ballot and
//    first-set-bit;
//  * each lane keeps its Gaussian's running sums in registers over all
//    pixels of the tile (per-row partial sums folded into the y terms at the
//    end of each row), then adds the 15-entry record to HBM with one set of
//    FP32 atomics per (tile, Gaussian) -- no shuffle reduction, no LDS merge.
//
// The tile's list is read from its coarse bin (8x8 tiles) in depth order and
// filtered by the tile rectangle with a ballot/popcount compaction into a
// per-wave LDS queue.  Blocks are remapped so that each XCD receives a
// contiguous range of coarse bins (its L2 holds that bin's list and splats).
//
// Batched form (tg_splat_accumulate_batch): one launch walks a ragged list of
// (slot, view, tile) work over up to TG_MAX_SLOTS slots, each slot one
// resident Gaussian set with its own size, views and resolution.  The frames
// of one slot share the reference Gaussians and hence every alpha and T
// (Sec. 4.7: each target frame is solved from the clip's first frame), so a
// tile evaluates alpha T once and adds each frame's track statistics: up to
// four frames ride on one evaluation, their sums side by side in registers.
#include "tg_internal.h"

namespace {

constexpr int QCAP = 128;
constexpr int SA_RECS = 8;    // records per round of the flush
constexpr float LOG2E = 1.4426950408889634f;

// One slot of a launch: a Gaussian set (splats + bins of one frame set)
// and F frames of tracks.  All views of a slot share one resolution, so the
// tile grid is uniform over its views.
struct SlotArgs {
    const float4* rec;
    const ushort4* rect;
    const uint32_t* cell_ids;
    const uint2* ranges;
    const int32_t* overflow;
    const float2* disp[TG_MAX_FRAMES];   // per frame [V,H,W]
    const uint8_t* vis[TG_MAX_FRAMES];   // per frame [V,H,W] or null
    float* acc[TG_MAX_FRAMES];           // per frame [V,N,16]
    float* t_final;          // [V,H,W] or null
    int64_t N;
    int64_t block0;          // first logical block of the slot
    int32_t W, H, F, cshift;
    int32_t cells_x, cells_pv, tiles_x, tiles_y;
};

struct BatchArgs {
    SlotArgs slot[TG_MAX_SLOTS];
    int32_t n_slots;
    int64_t n_enum;          // logical blocks over all slots
    int64_t blocks_per_xcd;
    float alpha_min, alpha_max, t_min, static2;
    unsigned long long* stats;
};

// Running sums of one frame for the lane's Gaussian.  With u = (ux, uy) the
// pixel's offset from the splat centre, the record of Eq. 4 needs sums of w,
// w u, w u u^T, w d, w u d^T.  Within a pixel row uy is constant, so the
// per-pixel work keeps only sums over the row's pixels (R0 = sum w,
// R1 = sum w c, RDX/RDY = sum w d), folded into the uy terms once per row.
// The x offsets are kept as ux = ax + c with c a small integer column offset
// from a per-lane anchor ax (|ax| <= 1/2 when the centre's column lies in the
// tile), so sum w ux^2 = C2 + 2 ax C1 + ax^2 W adds terms of one sign or of
// bounded ratio, never a large cancellation.
struct Sums {
    float W, C1, C2, N, DX, DY, CDX, CDY, UY, XY, YY, YDX, YDY, sn, sa;   // tile totals
    float R0, R1, RDX, RDY;                                               // current row
};

__device__ __forceinline__ void sums_zero(Sums& s) {
    s.W = s.C1 = s.C2 = s.N = s.DX = s.DY = s.CDX = s.CDY = 0.f;
    s.UY = s.XY = s.YY = s.YDX = s.YDY = s.sn = s.sa = 0.f;
    s.R0 = s.R1 = s.RDX = s.RDY = 0.f;
}

// One pixel: weight w, w c (c = column offset from the anchor), track d.
__device__ __forceinline__ void sums_add(Sums& s, float wgt, float wc, float cpp, float tdx, float tdy, bool stat,
                                         float al) {
    s.R0 += wgt;
    s.R1 += wc;
    s.C2 = fmaf(wc, cpp, s.C2);
    s.RDX = fmaf(wgt, tdx, s.RDX);
    s.RDY = fmaf(wgt, tdy, s.RDY);
    s.CDX = fmaf(wc, tdx, s.CDX);
    s.CDY = fmaf(wc, tdy, s.CDY);
    s.N += 1.0f;
    if (stat) {
        // static pixels are rare: a real (wave-uniform) branch, kept from
        // being turned into selects that would cost every pixel
        asm volatile("");
        s.sn += 1.0f;
        s.sa += al;
    }
}

// End of a pixel row at vertical offset uy.
__device__ __forceinline__ void sums_fold_row(Sums& s, float uy, float ax) {
    s.W += s.R0;
    s.C1 += s.R1;
    s.DX += s.RDX;
    s.DY += s.RDY;
    s.UY = fmaf(uy, s.R0, s.UY);
    s.XY = fmaf(uy, fmaf(ax, s.R0, s.R1), s.XY);
    s.YY = fmaf(uy * uy, s.R0, s.YY);
    s.YDX = fmaf(uy, s.RDX, s.YDX);
    s.YDY = fmaf(uy, s.RDY, s.YDY);
    s.R0 = s.R1 = s.RDX = s.RDY = 0.f;
}

// One wave (64 threads) per workgroup and per 16x16 tile, so tiles of very
// different work never hold each other's resources.  FM: frames per slot the
// launch is compiled for (a slot may carry fewer).
template <int FM, bool STATS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FM == 1 ? 7 : 1, 8)))
k_accumulate(BatchArgs a)
{
    // 5.5 KB of LDS per wave, allocated as 6 KB (512-byte granules), so 26
    // waves share a CU (the VGPRs would allow 28; a 5.5 KB variant that let
    // them in ran no faster, the VALU issuing every cycle already): queues
    // of candidate
    // and filtered list entries (ids), per-pixel records (transmittance, and for one frame the
    // track; a row of them is held in registers while the row is visited)
    // and the atomics' transpose buffer
    __shared__ uint32_t qi[QCAP];
    __shared__ uint32_t cq[QCAP];   // candidates passing the rectangle test
    __shared__ float4 PR[256];      // T, track x, track y, unused
    __shared__ float SA[SA_RECS * 17];
    // XCD-aware remap: hardware places workgroup b on XCD (b mod 8); give
    // each XCD a contiguous range of tiles (its L2 then holds those bins).
    const int64_t b = blockIdx.x;
    const int64_t L = (b & 7) * a.blocks_per_xcd + (b >> 3);
    if (L >= a.n_enum) return;
    int si = 0;
#pragma unroll
    for (int s = 1; s < TG_MAX_SLOTS; ++s)
        if (s < a.n_slots && L >= a.slot[s].block0) si = s;
    si = __builtin_amdgcn_readfirstlane(si);
    const SlotArgs& S = a.slot[si];
    if (*S.overflow) return;
    const int64_t N = S.N;
    const int W = S.W, H = S.H, F = S.F;
    const int k = 1 << S.cshift;
    const int kk = k * k;
    const int64_t Ll = L - S.block0;
    const uint32_t gcell = (uint32_t)(Ll / kk);
    const int ti = (int)(Ll % kk);
    const int v = (int)(gcell / (uint32_t)S.cells_pv);
    const int cl = (int)gcell - v * S.cells_pv;
    const int tx = (cl % S.cells_x) * k + (ti % k);
    const int ty = (cl / S.cells_x) * k + (ti / k);
    if (tx >= S.tiles_x || ty >= S.tiles_y) return;
    const float4* __restrict__ rec = S.rec;
    const ushort4* __restrict__ rect = S.rect;
    const uint32_t* __restrict__ cell_ids = S.cell_ids;
    const uint2 rg = S.ranges[gcell];
    const int64_t vN = (int64_t)v * N;
    const int px0 = tx * TG_TILE, py0 = ty * TG_TILE;
    const int64_t row_base = (int64_t)v * H;
    const int lane = threadIdx.x;

    // pixel state: pixel j = g*64 + lane -> (px0 + (j&15), py0 + (j>>4));
    // flags of pixel j: bit f = track visible in frame f, bit 8+f = static
    // in frame f
    constexpr uint32_t VISM = (1u << FM) - 1u;   // track-visible bits of the frames
    uint64_t alive[4];
    uint32_t flg[4];
    // tracks of pixel g*64 + lane per frame (in registers for several frames,
    // in the LDS records for one)
    float dxg[FM == 1 ? 1 : FM][4], dyg[FM == 1 ? 1 : FM][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int j = g * 64 + lane;
        const int px = px0 + (j & 15), py = py0 + (j >> 4);
        const bool in = px < W && py < H;
        uint32_t fl = 0;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            float ddx = 0.f, ddy = 0.f;
            if (in && f < F) {
                const int64_t pi = (row_base + py) * W + px;
                const float2 d = S.disp[f][pi];
                ddx = d.x;
                ddy = d.y;
                const bool vv = S.vis[f] ? S.vis[f][pi] != 0 : true;
                float s2;
                {
#pragma clang fp contract(off)
                    s2 = ddx * ddx;
                    s2 = s2 + ddy * ddy;
                }
                fl |= (vv ? 1u : 0u) << f;
                fl |= (s2 < a.static2 ? 1u : 0u) << (8 + f);
            }
            if constexpr (FM == 1) {
                PR[j] = make_float4(1.0f, ddx, ddy, 0.0f);
            } else {
                dxg[f][g] = ddx;
                dyg[f][g] = ddy;
            }
        }
        if constexpr (FM > 1) PR[j].x = 1.0f;
        flg[g] = fl;
        // a pixel whose track is hidden in every frame adds to no sum, so
        // unless its final transmittance is asked for it is never visited
        alive[g] = ballot64(in && (S.t_final != nullptr || (fl & VISM) != 0u));
    }
    uint64_t n_eval = 0, n_contrib = 0, n_iter = 0, n_refill = 0;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min;
    const float log_amin = __logf(amin);
    const uint64_t ltmask = lanemask_lt();
    const bool lane0 = lane == 0;
    float pex_reg = 1.0f;   // lane 0 is never written by the wave shift below
    int qn = 0, cn = 0;
    uint32_t pos = rg.x;
    // pixel-centre extent of the tile (conservative for the ellipse test)
    const float ex0 = (float)px0, ex1 = (float)(px0 + TG_TILE - 1);
    const float ey0 = (float)py0, ey1 = (float)(py0 + TG_TILE - 1);

    while ((alive[0] | alive[1] | alive[2] | alive[3]) != 0ull) {
        // Refill: list entries whose rectangle contains this tile and whose
        // alpha >= alpha_min region can reach it.  The second test is exact
        // culling: q >= 2 ln(o / alpha_min) everywhere on the tile means
        // alpha < alpha_min at every pixel, so the Gaussian neither adds nor
        // attenuates (a margin keeps it conservative under FP32 rounding).
        // Two stages keep the lanes busy: the rectangle test streams the
        // list (a few percent of a coarse bin's entries meet one tile) into
        // a candidate queue, and the exact test runs on 64 candidates at a
        // time.  Both queues keep list order.
        while (qn < 64 && (pos < rg.y || cn > 0)) {
            if (cn < 64 && pos < rg.y) {
                // a two-deep pipeline: the ids two rounds ahead and the
                // rectangles one round ahead are in flight while a round is
                // tested (entries fetched past the stopping point are read
                // again by the next refill)
                auto id_at = [&](uint32_t p) -> uint32_t {
                    const uint32_t g = p + lane < rg.y ? cell_ids[p + lane] : 0xFFFFFFFFu;
                    return g < (uint64_t)N ? g : 0xFFFFFFFFu;
                };
                auto rect_of = [&](uint32_t g) -> ushort4 {
                    return g != 0xFFFFFFFFu ? rect[vN + g] : make_ushort4(0, 0, 0, 0);
                };
                uint32_t id0 = id_at(pos);
                ushort4 r0 = rect_of(id0);
                uint32_t id1 = id_at(pos + 64);
                while (true) {
                    const ushort4 r1 = rect_of(id1);
                    const uint32_t id2 = id_at(pos + 128);
                    const bool hit = tx >= r0.x && tx < r0.z && ty >= r0.y && ty < r0.w;
                    const uint64_t m = ballot64(hit);
                    if (hit) cq[cn + __popcll(m & ltmask)] = id0;
                    cn += __popcll(m);
                    pos += 64;
                    if (STATS) n_refill += 1;
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
                ok = splat_reaches_tile(rec[2 * (vN + cg)], rec[2 * (vN + cg) + 1], log_amin, amin, ex0, ex1, ey0,
                                        ey1);
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
        float dxl = 0.f, dyl = 0.f, ca = 0.f, cb = 0.f, cc = 0.f, op = 0.f;
        if (lane < nb) {
            gid = qi[lane];
            const float4 r0 = rec[2 * (vN + gid)];
            const float4 r1 = rec[2 * (vN + gid) + 1];
            dxl = (float)px0 - r0.x;   // u = (px0 + column) - mu_x
            dyl = (float)py0 - r0.y;
            ca = -0.5f * LOG2E * r0.z;
            cb = -LOG2E * r0.w;
            cc = -0.5f * LOG2E * r1.x;
            op = r1.y;
        }
        // alpha = o 2^q = 2^(q + log2 o): the opacity rides in the row term
        // (log2 o = -inf for the empty lanes, whose alpha is then 0).  The
        // renderer's "skip if power > 0" test is not evaluated: the conic is
        // the inverse of the dilated covariance (determinant >= 0.09 px^4 for
        // any positive semi-definite Sigma_2D, FP32 rounding keeps it
        // positive definite), so power <= 0 everywhere but for rounding at
        // the splat centre, where alpha is o either way.
        const float lop = __builtin_amdgcn_logf(op);
        // column anchor: ux = ax + (column - o_x), o_x the column nearest the
        // centre, clamped to the tile
        const float o_x = fminf(fmaxf(rintf(-dxl), 0.0f), 15.0f);
        const float ax = dxl + o_x;
        if (lane + 64 < qn) {
            const uint32_t g2 = qi[lane + 64];
            qi[lane] = g2;
        }
        qn -= nb;

        Sums sm[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) sums_zero(sm[f]);

#pragma unroll
        for (int g = 0; g < 4; ++g) {
            // one frame: the group's visibility and static flags as
            // wave-uniform masks (one scalar bit test per pixel)
            uint64_t visg = 0, statg = 0;
            if constexpr (FM == 1) {
                visg = ballot64((flg[g] & 1u) != 0u);
                statg = ballot64((flg[g] & 0x100u) != 0u);
            }
            for (int rr = 0; rr < 4; ++rr) {
              uint32_t m = (uint32_t)(alive[g] >> (16 * rr)) & 0xFFFFu;
              if (m == 0u) continue;
              // the row's share of the quadratic form, common to its pixels:
              // q = ux (ca ux + cb uy) + cc uy^2 (+ log2 o)
              const float uy = dyl + (float)(4 * g + rr);
              const float brow = cb * uy;
              const float hrow = fmaf(cc * uy, uy, lop);
              // as a polynomial in the anchored column offset c'' = ux - ax:
              // q = (ca c'' + bq) c'' + cq, cq being q at the anchor column
              const float bq = fmaf(2.0f * ca, ax, brow);
              const float cq = fmaf(ax, fmaf(ca, ax, brow), hrow);
              // the row's pixel records live in lanes 0..15 (copied to every
              // 16-lane group) for the row: each step reads its pixel with
              // v_readlane and writes the new transmittance back with one
              // select, with no LDS traffic or address arithmetic per step
              const int rbase = (4 * g + rr) * 16;
              const float4 prow = PR[rbase + (lane & 15)];
              float Trow = prow.x;
              const float Xrow = prow.y, Yrow = prow.z;
              while (m) {
                const int c1 = __builtin_ctz(m);
                m &= m - 1;
                const int j1 = 16 * rr + c1;
                const float T1 = readlane_f(Trow, c1);
                const float cpp = (float)c1 - o_x;   // exact: small integers
                const float q1 = fmaf(fmaf(ca, cpp, bq), cpp, cq);
                // alpha = min(alpha_max, o e^power), clamped with one v_med3
                const float al1 = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(q1), 0.0f, amax);
                // valid lanes: alpha >= alpha_min
                const uint64_t vm1 = ballot64(al1 >= amin);
                // no Gaussian of the batch reaches the pixel: nothing changes
                if (vm1 == 0ull) {
                    if (STATS) {
                        n_eval += (uint64_t)nb;
                        n_iter += 1;
                    }
                    continue;
                }
                float P1 = __builtin_amdgcn_inverse_ballot_w64(vm1) ? 1.0f - al1 : 1.0f;
                P1 = wave_scan_mul_fused(P1);
                const uint64_t tm1 = ballot64(T1 * P1 < tmin) & vm1;
                // contributing lanes and the product of (1 - alpha) over them;
                // termination inside the batch is the rare case
                // A pixel that terminates stores its transmittance negated:
                // the row's dead pixels are then one ballot at the row's end.
                uint64_t cm1 = vm1;
                float Pk1 = readlane_f(P1, 63);
                if (__builtin_expect(tm1 != 0ull, 0)) {
                    const int kt1 = (int)__builtin_ctzll(tm1);
                    cm1 = vm1 & ((1ull << kt1) - 1ull);
                    Pk1 = -(kt1 == 0 ? 1.0f : readlane_f(P1, kt1 - 1));
                    if (STATS) n_eval += (uint64_t)(kt1 + 1 - nb);
                }
                const float Tn = Trow * Pk1;   // lane c1 holds T1
                Trow = __builtin_amdgcn_inverse_ballot_w64(1ull << c1) ? Tn : Trow;
                if (STATS) {
                    n_eval += (uint64_t)nb;
                    n_contrib += (uint64_t)__popcll(cm1);
                    n_iter += 1;
                }
                // statistics of Eq. 4 for the lanes that contribute, per frame
                // whose track at this pixel is visible: one exec mask, no
                // separate tests (the wave-wide reads come first)
                asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 wave_shr:1 row_mask:0xf bank_mask:0xf"
                             : "+v"(pex_reg) : "v"(P1));
                if constexpr (FM == 1) {
                    // one frame: a scalar bit test of the pixel's visibility
                    // (a wave-uniform branch, no selects), then the
                    // contributing lanes
                    if ((visg >> j1) & 1ull) {
                        const float2 td = make_float2(readlane_f(Xrow, c1), readlane_f(Yrow, c1));
                        if (__builtin_amdgcn_inverse_ballot_w64(cm1)) {
                            const float wgt = al1 * (T1 * pex_reg);
                            const float wc = wgt * cpp;
                            sums_add(sm[0], wgt, wc, cpp, td.x, td.y, (statg >> j1) & 1ull, al1);
                        }
                    }
                } else {
                    const uint32_t fl1 = (uint32_t)__builtin_amdgcn_readlane((int)flg[g], j1);
                    const uint64_t gate = (fl1 & VISM) ? cm1 : 0ull;
                    float2 td[FM];
#pragma unroll
                    for (int f = 0; f < FM; ++f)
                        td[f] = make_float2(readlane_f(dxg[f][g], j1), readlane_f(dyg[f][g], j1));
                    if (__builtin_amdgcn_inverse_ballot_w64(gate)) {
                        const float wgt = al1 * (T1 * pex_reg);
                        const float wc = wgt * cpp;
#pragma unroll
                        for (int f = 0; f < FM; ++f)
                            if ((fl1 >> f) & 1u)
                                sums_add(sm[f], wgt, wc, cpp, td[f].x, td[f].y, (fl1 >> (8 + f)) & 1u, al1);
                    }
                }
              }
              if (lane < 16) PR[rbase + lane].x = Trow;
              alive[g] &= ~((ballot64(Trow < 0.0f) & 0xFFFFull) << (16 * rr));
              // fold the row's partial sums unless no lane gathered any
              bool rowhit = false;
#pragma unroll
              for (int f = 0; f < FM; ++f) rowhit |= ballot64(sm[f].R0 != 0.0f) != 0ull;
              if (rowhit) {
#pragma unroll
                for (int f = 0; f < FM; ++f) sums_fold_row(sm[f], uy, ax);
              }
            }
        }
        // Flush through LDS: each lane's record is transposed so that one
        // atomic instruction adds 4 records (16 lanes each, one record per
        // 64-byte half line) instead of touching 64 lines.  Zero sums are
        // skipped (adding +0 never changes a sum that starts at +0), which
        // also skips lanes without contributions and the static slots when
        // no static pixel was seen.
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const Sums& s = sm[f];
            float* const accf = S.acc[f];
#pragma unroll
            for (int h = 0; h < 64 / SA_RECS; ++h) {
                if (SA_RECS * h >= nb) break;
                const int rl = lane - SA_RECS * h;
                if (rl >= 0 && rl < SA_RECS) {
                    // Eq. 4 record order: w, w ux, w uy, w ux^2, w ux uy,
                    // w uy^2, w dx, w dy, w ux dx, w ux dy, w uy dx, w uy dy,
                    // pixel count, static count, static alpha
                    float* r = SA + rl * 17;
                    r[0] = s.W;
                    r[1] = fmaf(ax, s.W, s.C1);
                    r[2] = s.UY;
                    r[3] = fmaf(ax, fmaf(ax, s.W, 2.0f * s.C1), s.C2);
                    r[4] = s.XY;
                    r[5] = s.YY;
                    r[6] = s.DX;
                    r[7] = s.DY;
                    r[8] = fmaf(ax, s.DX, s.CDX);
                    r[9] = fmaf(ax, s.DY, s.CDY);
                    r[10] = s.YDX;
                    r[11] = s.YDY;
                    r[12] = s.N;
                    r[13] = s.sn;
                    r[14] = s.sa;
                    r[15] = __builtin_bit_cast(float, gid);
                }
                __syncthreads();
                const int rec_n = min(SA_RECS, nb - SA_RECS * h);
                const int k = lane & 15;
                for (int q = 0; 4 * q < rec_n; ++q) {
                    const int gl = 4 * q + (lane >> 4);
                    const float val = SA[gl * 17 + k];
                    const uint32_t gg = __builtin_bit_cast(uint32_t, SA[gl * 17 + 15]);
                    if (k < 15 && gl < rec_n && val != 0.0f)
                        unsafeAtomicAdd(accf + (vN + gg) * TG_ACC_STRIDE + k, val);
                }
                __syncthreads();
            }
        }
    }
    if (S.t_final) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int j = g * 64 + lane;
            const int px = px0 + (j & 15), py = py0 + (j >> 4);
            // (terminated pixels hold their transmittance negated)
            if (px < W && py < H) S.t_final[(row_base + py) * W + px] = fabsf(PR[j].x);
        }
    }
    if (STATS && lane == 0) {
        atomicAdd(a.stats, (unsigned long long)n_eval);
        atomicAdd(a.stats + 1, (unsigned long long)n_contrib);
        atomicAdd(a.stats + 2, (unsigned long long)n_iter);
        atomicAdd(a.stats + 3, (unsigned long long)n_refill);
    }
}

// Validates one slot and fills its launch record; *blocks receives the
// slot's logical block count.
tg_status make_slot(const tg_acc_slot& in, const tg_params* p, SlotArgs* o, int64_t block0, int64_t* blocks) {
    const tg_splats* s = in.s;
    const tg_bins* bins = in.bins;
    if (!s || !bins || !in.cams || in.N < 0 || in.V < 1) return TG_ERR_INVALID_ARG;
    if (in.F < 1 || in.F > TG_MAX_FRAMES || in.V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (!s->rec || !s->rect || !bins->cell_ids || !bins->cell_ranges || !bins->overflow) return TG_ERR_INVALID_ARG;
    if (!aligned16(s->rec)) return TG_ERR_ALIGNMENT;
    for (int f = 0; f < in.F; ++f) {
        if (!in.disp[f] || !in.acc[f]) return TG_ERR_INVALID_ARG;
        if (!aligned16(in.acc[f]) || ((uintptr_t)in.disp[f] & 7u)) return TG_ERR_ALIGNMENT;
    }
    for (int v = 1; v < in.V; ++v)
        if (in.cams[v].width != in.cams[0].width || in.cams[v].height != in.cams[0].height)
            return TG_ERR_INVALID_ARG;
    if (in.cams[0].width < 1 || in.cams[0].height < 1) return TG_ERR_INVALID_ARG;
    if (in.N > (int64_t)0xFFFFFFFF) return TG_ERR_UNSUPPORTED;
    *blocks = 0;
    if (in.N == 0) return TG_OK;
    // same coarse plan as tg_bin_sort
    GridPack gp;
    int cs = 0;
    const int64_t ncell = coarse_plan(in.cams, in.V, in.N, p, &gp, &cs);
    if (ncell < 0) return TG_ERR_UNSUPPORTED;
    o->rec = (const float4*)s->rec;
    o->rect = (const ushort4*)s->rect;
    o->cell_ids = bins->cell_ids;
    o->ranges = (const uint2*)bins->cell_ranges;
    o->overflow = bins->overflow;
    for (int f = 0; f < TG_MAX_FRAMES; ++f) {
        const bool use = f < in.F;
        o->disp[f] = use ? (const float2*)in.disp[f] : nullptr;
        o->vis[f] = use ? in.vis[f] : nullptr;
        o->acc[f] = use ? in.acc[f] : nullptr;
    }
    o->t_final = in.t_final;
    o->N = in.N;
    o->W = in.cams[0].width;
    o->H = in.cams[0].height;
    o->F = in.F;
    o->cshift = cs;
    o->block0 = block0;
    o->cells_x = gp.cx[0];
    o->cells_pv = gp.cx[0] * gp.cy[0];
    o->tiles_x = gp.tx[0];
    o->tiles_y = gp.ty[0];
    *blocks = ncell << (2 * cs);
    return TG_OK;
}

template <int FM>
void launch(const BatchArgs& a, bool stats, hipStream_t st) {
    const int64_t grid = a.blocks_per_xcd * 8;
    if (stats)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_accumulate<FM, true>), dim3((unsigned)grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_accumulate<FM, false>), dim3((unsigned)grid), dim3(64), 0, st, a);
}

tg_status accumulate_slots(const tg_acc_slot* slots, int32_t n_slots, const tg_params* p, int64_t* stats,
                           void* stream) {
    if (!slots || !p || n_slots < 0) return TG_ERR_INVALID_ARG;
    if (n_slots > TG_MAX_SLOTS) return TG_ERR_UNSUPPORTED;
    BatchArgs a;
    int64_t total = 0;
    int fmax = 1, used = 0;
    for (int i = 0; i < n_slots; ++i) {
        int64_t nb = 0;
        const tg_status st = make_slot(slots[i], p, &a.slot[used], total, &nb);
        if (st != TG_OK) return st;
        if (nb == 0) continue;
        fmax = slots[i].F > fmax ? slots[i].F : fmax;
        total += nb;
        ++used;
    }
    if (used == 0) return TG_OK;
    if (total > (int64_t)0x7FFFFFF0) return TG_ERR_UNSUPPORTED;
    a.n_slots = used;
    a.n_enum = total;
    a.blocks_per_xcd = (total + 7) / 8;
    a.alpha_min = p->alpha_min;
    a.alpha_max = p->alpha_max;
    a.t_min = p->t_min;
    a.static2 = p->static_px * p->static_px;
    a.stats = (unsigned long long*)stats;
    const hipStream_t st = (hipStream_t)stream;
    if (fmax == 1)
        launch<1>(a, stats != nullptr, st);
    else if (fmax == 2)
        launch<2>(a, stats != nullptr, st);
    else
        launch<4>(a, stats != nullptr, st);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

}  // namespace

extern "C" tg_status tg_splat_accumulate(const tg_splats* s, const tg_bins* bins, int64_t N, const tg_camera* cams,
                                         int32_t V, const float* disp, const uint8_t* vis, const tg_params* p,
                                         float* acc, float* t_final, int64_t* stats, void* stream)
{
    if (!s || !bins || !cams || !p || !disp || !acc || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    tg_acc_slot one = {};
    one.s = s;
    one.bins = bins;
    one.cams = cams;
    one.N = N;
    one.V = V;
    one.F = 1;
    one.disp[0] = disp;
    one.vis[0] = vis;
    one.acc[0] = acc;
    one.t_final = t_final;
    return accumulate_slots(&one, 1, p, stats, stream);
}

extern "C" tg_status tg_splat_accumulate_batch(const tg_acc_slot* slots, int32_t n_slots, const tg_params* p,
                                               int64_t* stats, void* stream)
{
    return accumulate_slots(slots, n_slots, p, stats, stream);
}
