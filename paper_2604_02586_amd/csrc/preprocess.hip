// tg_preprocess: EWA projection of 3D Gaussians into every view
// (TrackerSplat Sec. 3.1, Eq. 1).
//
// One thread per Gaussian, looping over the views of the launch, so the
// Gaussian's parameters are read from HBM once and every per-view output is a
// coalesced store.  The integer-deciding quantities (splat centre, radius,
// tile rectangle, depth key) are FP32 in a fixed operation order with no
// contraction; the covariance and conic are formed in FP64 (the MI355X runs
// FP64 FMA at the FP32 non-packed rate, so this costs nothing in an
// HBM-bound kernel) and rounded once.
#include "tg_internal.h"

namespace {

// Per-view constants of the Jacobian clamp (the half field of view times
// j_clamp), formed once on the host with the same IEEE operations the
// kernel would use (no contraction), so the results are unchanged.
struct ClampPack {
    float limx[TG_MAX_VIEWS], limy[TG_MAX_VIEWS];
    double dlx[TG_MAX_VIEWS], dly[TG_MAX_VIEWS];
};

struct SplatOut {
    float4* rec;
    float* cov2d;
    ushort4* rect;
    uint32_t* key;
    float* colors;
    uint8_t* clamped;
};

// Real spherical harmonics up to degree DEG (Condon-Shortley phase) at a
// unit direction, dotted with the coefficients c[k*3 + ch] (held in
// registers: DEG is a compile-time constant, so every index is static).
template <int DEG>
__device__ inline void sh_color(const float* c, float x, float y, float z, float out[3]) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    float b[NB];
    b[0] = 0.28209479177387814f;
    if constexpr (DEG > 0) {
        const float c1 = 0.48860251190291992f;
        b[1] = -c1 * y;
        b[2] = c1 * z;
        b[3] = -c1 * x;
    }
    if constexpr (DEG > 1) {
        const float xx = x * x, yy = y * y, zz = z * z;
        b[4] = 1.0925484305920792f * x * y;
        b[5] = -1.0925484305920792f * y * z;
        b[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
        b[7] = -1.0925484305920792f * x * z;
        b[8] = 0.54627421529603959f * (xx - yy);
        if constexpr (DEG > 2) {
            b[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
            b[10] = 2.8906114426405538f * x * y * z;
            b[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
            b[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            b[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
            b[14] = 1.4453057213202769f * z * (xx - yy);
            b[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < NB; ++k) acc += b[k] * c[k * 3 + ch];
        out[ch] = acc + 0.5f;
    }
}

// DEG: SH degree of the colours (-1: no SH coefficients).
template <int DEG>
__global__ void __launch_bounds__(256) k_preprocess(
    const float* __restrict__ means, const float* __restrict__ quats,
    const float* __restrict__ scales, const float* __restrict__ opac,
    const float* __restrict__ sh, int scale_mode, int opacity_mode,
    int64_t N, int V, int64_t out_view0, CamPack cams, ClampPack clampk, tg_params prm, SplatOut out)
{
#pragma clang fp contract(off)
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const float m0 = means[3 * g], m1 = means[3 * g + 1], m2 = means[3 * g + 2];
    float qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
    float s0 = scales[3 * g], s1 = scales[3 * g + 1], s2 = scales[3 * g + 2];
    float o = opac[g];
    // a Gaussian with any non-finite parameter is culled in every view
    const bool finite_in = isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(qw) && isfinite(qx) &&
                           isfinite(qy) && isfinite(qz) && isfinite(s0) && isfinite(s1) && isfinite(s2) &&
                           isfinite(o);
    if (scale_mode == 1) { s0 = expf(s0); s1 = expf(s1); s2 = expf(s2); }
    if (opacity_mode == 1) o = 1.0f / (1.0f + expf(-o));

    // FP32 rotation of the normalised quaternion (fixed order).
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    float inv = 1.0f / sqrtf(n2);
    float w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
    float r[9];
    r[0] = 1.0f - 2.0f * (y * y + z * z);
    r[1] = 2.0f * (x * y - w * z);
    r[2] = 2.0f * (x * z + w * y);
    r[3] = 2.0f * (x * y + w * z);
    r[4] = 1.0f - 2.0f * (x * x + z * z);
    r[5] = 2.0f * (y * z - w * x);
    r[6] = 2.0f * (x * z - w * y);
    r[7] = 2.0f * (y * z + w * x);
    r[8] = 1.0f - 2.0f * (x * x + y * y);
    float M[9];
    const float sv[3] = {s0, s1, s2};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = r[i * 3 + j] * sv[j];
    float S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            S[i * 3 + j] = (M[i * 3] * M[j * 3] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];

    // FP64 copy of Sigma_3D (from the FP32 inputs).
    double dn = sqrt((double)qw * qw + (double)qx * qx + (double)qy * qy + (double)qz * qz);
    double dw = qw / dn, dx = qx / dn, dy = qy / dn, dz = qz / dn;
    double dr[9] = {1 - 2 * (dy * dy + dz * dz), 2 * (dx * dy - dw * dz), 2 * (dx * dz + dw * dy),
                    2 * (dx * dy + dw * dz), 1 - 2 * (dx * dx + dz * dz), 2 * (dy * dz - dw * dx),
                    2 * (dx * dz - dw * dy), 2 * (dy * dz + dw * dx), 1 - 2 * (dx * dx + dy * dy)};
    double ss[3] = {(double)s0 * s0, (double)s1 * s1, (double)s2 * s2};
    double D[6];  // S00 S01 S02 S11 S12 S22
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                D[k++] = dr[3 * i] * dr[3 * j] * ss[0] + dr[3 * i + 1] * dr[3 * j + 1] * ss[1] +
                         dr[3 * i + 2] * dr[3 * j + 2] * ss[2];
            }
    }

    // the Gaussian's SH coefficients, read once for all views
    constexpr int NC = DEG >= 0 ? 3 * (DEG + 1) * (DEG + 1) : 1;
    float shc[NC];
    if constexpr (DEG >= 0) {
        const float* src = sh + g * NC;
#pragma unroll
        for (int i = 0; i < NC; ++i) shc[i] = src[i];
    }

    for (int v = 0; v < V; ++v) {
        const tg_camera& c = cams.cam[v];
        const int64_t oi = (out_view0 + v) * N + g;
        const float* R = c.R;
        float px = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + c.t[0];
        float py = ((R[3] * m0 + R[4] * m1) + R[5] * m2) + c.t[1];
        float pz = ((R[6] * m0 + R[7] * m1) + R[8] * m2) + c.t[2];
        float4 rec0 = make_float4(0.f, 0.f, 0.f, 0.f), rec1 = make_float4(0.f, 0.f, 0.f, 0.f);
        ushort4 rc = make_ushort4(0, 0, 0, 0);
        uint32_t key = 0xFFFFFFFFu;
        float cov[3] = {0.f, 0.f, 0.f};
        bool ok = finite_in && pz > prm.near_z;
        if (ok) {
            float ux = px / pz, uy = py / pz;
            float mx = c.fx * ux + c.cx;
            float my = c.fy * uy + c.cy;
            const float limx = clampk.limx[v], limy = clampk.limy[v];
            float tx = fminf(limx, fmaxf(-limx, ux));
            float ty = fminf(limy, fmaxf(-limy, uy));
            float j00 = c.fx / pz, j02 = -(c.fx * tx) / pz;
            float j11 = c.fy / pz, j12 = -(c.fy * ty) / pz;
            float T0[3], T1[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T0[j] = j00 * R[j] + j02 * R[6 + j];
                T1[j] = j11 * R[3 + j] + j12 * R[6 + j];
            }
            float U0[3], U1[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                U0[j] = (T0[0] * S[j] + T0[1] * S[3 + j]) + T0[2] * S[6 + j];
                U1[j] = (T1[0] * S[j] + T1[1] * S[3 + j]) + T1[2] * S[6 + j];
            }
            float a = (U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2];
            float b = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
            float cc = (U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2];
            float ar = a + prm.dilation, cr = cc + prm.dilation;
            float det = ar * cr - b * b;
            ok = det > 0.0f;
            if (ok) {
                float mid = 0.5f * (ar + cr);
                float lmax = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
                float rad = ceilf(prm.extent * sqrtf(lmax));
                ok = isfinite(mx) && isfinite(my) && isfinite(rad);
                if (ok) {
                    float TX = (float)ceil_div(c.width, TG_TILE), TY = (float)ceil_div(c.height, TG_TILE);
                    float fx0 = floorf((mx - rad) * 0.0625f);
                    float fx1 = floorf((mx + rad) * 0.0625f) + 1.0f;
                    float fy0 = floorf((my - rad) * 0.0625f);
                    float fy1 = floorf((my + rad) * 0.0625f) + 1.0f;
                    fx0 = fminf(TX, fmaxf(0.0f, fx0));
                    fx1 = fminf(TX, fmaxf(0.0f, fx1));
                    fy0 = fminf(TY, fmaxf(0.0f, fy0));
                    fy1 = fminf(TY, fmaxf(0.0f, fy1));
                    int ix0 = (int)fx0, ix1 = (int)fx1, iy0 = (int)fy0, iy1 = (int)fy1;
                    ok = ix0 < ix1 && iy0 < iy1;
                    if (ok) {
                        rc = make_ushort4((unsigned short)ix0, (unsigned short)iy0, (unsigned short)ix1,
                                          (unsigned short)iy1);
                        key = fbits(pz);
                        // FP64 covariance and conic (Eq. 1), rounded once.
                        const double dpx = (double)R[0] * m0 + (double)R[1] * m1 + (double)R[2] * m2 + c.t[0];
                        const double dpy = (double)R[3] * m0 + (double)R[4] * m1 + (double)R[5] * m2 + c.t[1];
                        const double dpz = (double)R[6] * m0 + (double)R[7] * m1 + (double)R[8] * m2 + c.t[2];
                        // two FP64 reciprocals per view instead of nine divisions
                        // (each result is rounded to FP32 once afterwards)
                        const double idz = 1.0 / dpz;
                        double dtx = dpx * idz, dty = dpy * idz;
                        const double dlx = clampk.dlx[v], dly = clampk.dly[v];
                        dtx = fmin(dlx, fmax(-dlx, dtx));
                        dty = fmin(dly, fmax(-dly, dty));
                        double J00 = c.fx * idz, J02 = -c.fx * dtx * idz;
                        double J11 = c.fy * idz, J12 = -c.fy * dty * idz;
                        double A0[3], A1[3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            A0[j] = J00 * R[j] + J02 * R[6 + j];
                            A1[j] = J11 * R[3 + j] + J12 * R[6 + j];
                        }
                        // Sigma (symmetric) from D
                        double Sg[9] = {D[0], D[1], D[2], D[1], D[3], D[4], D[2], D[4], D[5]};
                        double B0[3], B1[3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            B0[j] = A0[0] * Sg[j] + A0[1] * Sg[3 + j] + A0[2] * Sg[6 + j];
                            B1[j] = A1[0] * Sg[j] + A1[1] * Sg[3 + j] + A1[2] * Sg[6 + j];
                        }
                        double ca = B0[0] * A0[0] + B0[1] * A0[1] + B0[2] * A0[2];
                        double cb = B0[0] * A1[0] + B0[1] * A1[1] + B0[2] * A1[2];
                        double ccc = B1[0] * A1[0] + B1[1] * A1[1] + B1[2] * A1[2];
                        double ra = ca + prm.dilation, rcc = ccc + prm.dilation;
                        double ddet = ra * rcc - cb * cb;
                        cov[0] = (float)ca;
                        cov[1] = (float)cb;
                        cov[2] = (float)ccc;
                        const double iddet = 1.0 / ddet;
                        rec0 = make_float4(mx, my, (float)(rcc * iddet), (float)(-cb * iddet));
                        rec1 = make_float4((float)(ra * iddet), o, pz, 0.0f);
                    }
                }
            }
        }
        out.rec[2 * oi] = rec0;
        out.rec[2 * oi + 1] = rec1;
        out.cov2d[3 * oi] = cov[0];
        out.cov2d[3 * oi + 1] = cov[1];
        out.cov2d[3 * oi + 2] = cov[2];
        out.rect[oi] = rc;
        out.key[oi] = key;
        if (out.colors) {
            float col[3] = {0.f, 0.f, 0.f};
            uint8_t cl[3] = {0, 0, 0};
            if (DEG >= 0 && ok) {
                // camera centre = -R^T t
                float ccx = -(R[0] * c.t[0] + R[3] * c.t[1] + R[6] * c.t[2]);
                float ccy = -(R[1] * c.t[0] + R[4] * c.t[1] + R[7] * c.t[2]);
                float ccz = -(R[2] * c.t[0] + R[5] * c.t[1] + R[8] * c.t[2]);
                float ex = m0 - ccx, ey = m1 - ccy, ez = m2 - ccz;
                float il = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
                if constexpr (DEG >= 0) sh_color<DEG>(shc, ex * il, ey * il, ez * il, col);
                for (int ch = 0; ch < 3; ++ch) {
                    if (col[ch] < 0.0f) { col[ch] = 0.0f; cl[ch] = 1; }
                }
            }
            out.colors[3 * oi] = col[0];
            out.colors[3 * oi + 1] = col[1];
            out.colors[3 * oi + 2] = col[2];
            if (out.clamped) {
                out.clamped[3 * oi] = cl[0];
                out.clamped[3 * oi + 1] = cl[1];
                out.clamped[3 * oi + 2] = cl[2];
            }
        }
    }
}

}  // namespace

extern "C" tg_status tg_preprocess(const tg_gaussians* g, int64_t N, const tg_camera* cams, int32_t V,
                                   const tg_params* p, tg_splats* out, void* stream)
{
    if (!g || !cams || !p || !out || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (N == 0) return TG_OK;
    if (!g->means || !g->quats || !g->scales || !g->opacity) return TG_ERR_INVALID_ARG;
    if (!out->rec || !out->cov2d || !out->rect || !out->key) return TG_ERR_INVALID_ARG;
    if (g->scale_mode < 0 || g->scale_mode > 1 || g->opacity_mode < 0 || g->opacity_mode > 1)
        return TG_ERR_INVALID_ARG;
    if (g->sh && (g->sh_degree < 0 || g->sh_degree > 3)) return TG_ERR_INVALID_ARG;
    if (!aligned16(out->rec)) return TG_ERR_ALIGNMENT;
    for (int v = 0; v < V; ++v)
        if (cams[v].width <= 0 || cams[v].height <= 0 || cams[v].width > 16 * 65535 ||
            cams[v].height > 16 * 65535)
            return TG_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    SplatOut so{(float4*)out->rec, out->cov2d, (ushort4*)out->rect, out->key, out->colors, out->clamped};
    const int threads = 256;
    const int64_t blocks = (N + threads - 1) / threads;
    for (int v0 = 0; v0 < V; v0 += TG_MAX_VIEWS) {
        int nv = V - v0 < TG_MAX_VIEWS ? V - v0 : TG_MAX_VIEWS;
        CamPack cp;
        ClampPack cl;
        for (int i = 0; i < nv; ++i) {
#pragma clang fp contract(off)
            const tg_camera& c = cams[v0 + i];
            cp.cam[i] = c;
            cl.limx[i] = p->j_clamp * ((0.5f * (float)c.width) / c.fx);
            cl.limy[i] = p->j_clamp * ((0.5f * (float)c.height) / c.fy);
            cl.dlx[i] = (double)p->j_clamp * (0.5 * c.width / (double)c.fx);
            cl.dly[i] = (double)p->j_clamp * (0.5 * c.height / (double)c.fy);
        }
        const int deg = (g->sh && out->colors) ? g->sh_degree : -1;
#define TG_PRE_LAUNCH(D)                                                                                        \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_preprocess<D>), dim3((unsigned)blocks), dim3(threads), 0, s, g->means, \
                       g->quats, g->scales, g->opacity, g->sh, g->scale_mode, g->opacity_mode, N, nv, (int64_t)v0, \
                       cp, cl, *p, so)
        switch (deg) {
            case 0: TG_PRE_LAUNCH(0); break;
            case 1: TG_PRE_LAUNCH(1); break;
            case 2: TG_PRE_LAUNCH(2); break;
            case 3: TG_PRE_LAUNCH(3); break;
            default: TG_PRE_LAUNCH(-1); break;
        }
#undef TG_PRE_LAUNCH
        TG_CHECK_LAUNCH();
    }
    return TG_OK;
}
