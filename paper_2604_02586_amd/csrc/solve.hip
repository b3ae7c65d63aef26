// tg_solve_views and tg_triangulate: the batched small solves of PWI-LS and
// of the multi-view update (TrackerSplat Sec. 4.2 Eq. 2, Sec. 4.3.4 Eq. 4,
// Sec. 4.4.1-4.4.3, thresholds of Sec. 5.2), in FP64.
//
// Both are one thread per (view, Gaussian) or per Gaussian and are bound by
// HBM traffic (the MI355X runs FP64 FMA at the rate of non-packed FP32, so a
// few thousand FP64 flops per Gaussian are free next to its 21 bytes x V of
// solved motions).  Eigen-decompositions use cyclic Jacobi, the covariance
// system a 6x6 Cholesky of the normal equations.
#include "tg_internal.h"

namespace {

// ---------------------------------------------------------------- per view
// Flags of one centred record and, when it is solved (flag 1), the FP64
// solution Theta = V1^{-1} V2 as th = [t0x, t0y, t1x, t1y, t2x, t2y]
// (rows of Theta: the x and y rows of G^T, then c^T).
__device__ __forceinline__ uint8_t solve_record(const float4 a0, const float4 a1, const float4 a2, const float4 a3,
                                                bool culled, const tg_params& prm, double th[6])
{
    // record: [Sw, Sux, Suy, Sxx, Sxy, Syy, Sdx, Sdy, Sxdx, Sxdy, Sydx, Sydy, n, ...]
    const double Sw = a0.x, Sux = a0.y, Suy = a0.z, Sxx = a0.w;
    const double Sxy = a1.x, Syy = a1.y, Sdx = a1.z, Sdy = a1.w;
    const double Sxdx = a2.x, Sxdy = a2.y, Sydx = a2.z, Sydy = a2.w;
    const double n = a3.x;
    // V1 = [[Sxx, Sxy, Sux], [Sxy, Syy, Suy], [Sux, Suy, Sw]]
    const double c00 = Syy * Sw - Suy * Suy;
    const double c01 = Sux * Suy - Sxy * Sw;
    const double c02 = Sxy * Suy - Syy * Sux;
    const double c11 = Sxx * Sw - Sux * Sux;
    const double c12 = Sxy * Sux - Sxx * Suy;
    const double c22 = Sxx * Syy - Sxy * Sxy;
    const double det = Sxx * c00 + Sxy * c01 + Sux * c02;
    uint8_t f = 0;
    if (culled) f |= 2;
    if (n < (double)prm.pix_min) f |= 4;
    if (!(Sw >= prm.wsum_min)) f |= 8;
    if (!(det >= prm.det_min)) f |= 16;
    // a non-finite track leaves non-finite sums in the record
    if (!(isfinite(a0.x) && isfinite(a0.y) && isfinite(a0.z) && isfinite(a0.w) && isfinite(a1.x) &&
          isfinite(a1.y) && isfinite(a1.z) && isfinite(a1.w) && isfinite(a2.x) && isfinite(a2.y) &&
          isfinite(a2.z) && isfinite(a2.w) && isfinite(a3.x)))
        f |= 32;
    {
        // scale-invariant near-singularity: pixel offsets (nearly) collinear
        const double iw = Sw > 0.0 ? 1.0 / Sw : 0.0;
        const double mx = Sux * iw, my = Suy * iw;
        const double ca = Sxx * iw - mx * mx, cb = Sxy * iw - mx * my, cc = Syy * iw - my * my;
        const double tr = ca + cc;
        if (!(tr > 0.0) || !(4.0 * (ca * cc - cb * cb) >= prm.iso_min * tr * tr)) f |= 16;
    }
    if (f != 0) return f;
    const double id = 1.0 / det;
    // inverse of V1 (symmetric): adj / det
    const double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    const double i11 = c11 * id, i12 = c12 * id, i22 = c22 * id;
    // Theta = V1^{-1} V2, V2 = [[Sxdx, Sxdy], [Sydx, Sydy], [Sdx, Sdy]]
    th[0] = i00 * Sxdx + i01 * Sydx + i02 * Sdx;
    th[1] = i00 * Sxdy + i01 * Sydy + i02 * Sdy;
    th[2] = i01 * Sxdx + i11 * Sydx + i12 * Sdx;
    th[3] = i01 * Sxdy + i11 * Sydy + i12 * Sdy;
    th[4] = i02 * Sxdx + i12 * Sydx + i22 * Sdx;
    th[5] = i02 * Sxdy + i12 * Sydy + i22 * Sdy;
    return 1;
}

// mu' = mu + c (Eq. 4's intercept in the centred frame), rounded to FP32.
__device__ __forceinline__ float2 moved_centre(const double th[6], float mux, float muy) {
    return make_float2((float)((double)mux + th[4]), (float)((double)muy + th[5]));
}

// Eq. 2: Sigma' = A Sigma A^T with A = I + G, rounded to FP32.
__device__ __forceinline__ void moved_cov(const double th[6], double sa, double sb, double sc, float co[3]) {
    const double A00 = 1.0 + th[0], A01 = th[2], A10 = th[1], A11 = 1.0 + th[3];
    const double m00 = A00 * sa + A01 * sb, m01 = A00 * sb + A01 * sc;
    const double m10 = A10 * sa + A11 * sb, m11 = A10 * sb + A11 * sc;
    co[0] = (float)(m00 * A00 + m01 * A01);
    co[1] = (float)(m00 * A10 + m01 * A11);
    co[2] = (float)(m10 * A10 + m11 * A11);
}

__global__ void __launch_bounds__(256) k_solve_views(const float4* __restrict__ acc, const float4* __restrict__ rec,
                                                     const float* __restrict__ cov2d, const ushort4* __restrict__ rect,
                                                     int64_t VN, tg_params prm, float2* __restrict__ mu_new,
                                                     float* __restrict__ cov_new, uint8_t* __restrict__ flags,
                                                     float2* __restrict__ wn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= VN) return;
    const float4 a0 = acc[4 * i], a1 = acc[4 * i + 1], a2 = acc[4 * i + 2], a3 = acc[4 * i + 3];
    const ushort4 r = rect[i];
    double th[6];
    const uint8_t f = solve_record(a0, a1, a2, a3, !(r.z > r.x && r.w > r.y), prm, th);
    float2 mo = make_float2(0.f, 0.f);
    float co[3] = {0.f, 0.f, 0.f};
    if (f == 1) {
        const float4 rc = rec[2 * i];
        mo = moved_centre(th, rc.x, rc.y);
        moved_cov(th, cov2d[3 * i], cov2d[3 * i + 1], cov2d[3 * i + 2], co);
    }
    mu_new[i] = mo;
    // accumulated alpha and pixel count, compact for the triangulation's
    // per-Gaussian totals (8 B instead of a 64-byte record per view)
    if (wn) wn[i] = make_float2(a0.x, a3.x);
    cov_new[3 * i] = co[0];
    cov_new[3 * i + 1] = co[1];
    cov_new[3 * i + 2] = co[2];
    flags[i] = f;
}

// ---------------------------------------------------------------- helpers
// Cyclic Jacobi for a symmetric n x n matrix (row-major, in place);
// eigenvectors in the columns of Vm.
template <int n>
__device__ void jacobi_eig(double* A, double* Vm) {
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) Vm[i * n + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 20; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i)
#pragma unroll
            for (int j = 0; j < n; ++j) {
                double x = A[i * n + j] * A[i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
#pragma unroll
        for (int p = 0; p < n - 1; ++p)
#pragma unroll
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    const double vkp = Vm[k * n + p], vkq = Vm[k * n + q];
                    Vm[k * n + p] = c * vkp - s * vkq;
                    Vm[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
}

__device__ void quat_from_rot(const double* R, double* q) {
    // Shepperd: pivot on the largest of tr, R00, R11, R22
    const double tr = R[0] + R[4] + R[8];
    double w, x, y, z;
    if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
        const double s = 2.0 * sqrt(fmax(1.0 + tr, 0.0));
        w = 0.25 * s;
        x = (R[7] - R[5]) / s;
        y = (R[2] - R[6]) / s;
        z = (R[3] - R[1]) / s;
    } else if (R[0] >= R[4] && R[0] >= R[8]) {
        const double s = 2.0 * sqrt(fmax(1.0 + R[0] - R[4] - R[8], 0.0));
        w = (R[7] - R[5]) / s;
        x = 0.25 * s;
        y = (R[1] + R[3]) / s;
        z = (R[2] + R[6]) / s;
    } else if (R[4] >= R[8]) {
        const double s = 2.0 * sqrt(fmax(1.0 - R[0] + R[4] - R[8], 0.0));
        w = (R[2] - R[6]) / s;
        x = (R[1] + R[3]) / s;
        y = 0.25 * s;
        z = (R[5] + R[7]) / s;
    } else {
        const double s = 2.0 * sqrt(fmax(1.0 - R[0] - R[4] + R[8], 0.0));
        w = (R[3] - R[1]) / s;
        x = (R[2] + R[6]) / s;
        y = (R[5] + R[7]) / s;
        z = 0.25 * s;
    }
    const double nn = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    const double sg = w < 0.0 ? -nn : nn;
    q[0] = w * sg;
    q[1] = x * sg;
    q[2] = y * sg;
    q[3] = z * sg;
}

// The Gaussians a multi-view update reads and writes.
struct GaussIO {
    const float* means_in;
    const float* quats_in;
    const float* scales_in;
    const float* opacity_in;
    float* means_out;
    float* quats_out;
    float* scales_out;
    uint32_t* status;
    int64_t N;
    int V;
    int scale_mode;
};

// Per-view results as tg_solve_views stored them.
struct StoredViews {
    const float2* mu_new;
    const float* cov_new;
    const uint8_t* vflags;
    const float2* wn;
    // totals (accumulated alpha, pixels) and flag of view record o
    __device__ __forceinline__ uint8_t screen(int64_t o, float2& t) const {
        t = wn[o];
        return vflags[o];
    }
    // the same in two halves: the loads (issued ahead), then the use
    struct Rec {
        float2 t;
        uint8_t f;
    };
    __device__ __forceinline__ Rec fetch(int64_t o) const { return Rec{wn[o], vflags[o]}; }
    __device__ __forceinline__ uint8_t screen_rec(const Rec& r, float2& t) const {
        t = r.t;
        return r.f;
    }
    __device__ __forceinline__ uint8_t view(int64_t o, float2& t, float2& mu) const {
        const uint8_t f = screen(o, t);
        if (f == 1) mu = mu_new[o];
        return f;
    }
    __device__ __forceinline__ void cov(int64_t o, float co[3]) const {
        co[0] = cov_new[3 * o];
        co[1] = cov_new[3 * o + 1];
        co[2] = cov_new[3 * o + 2];
    }
    // view() and, for a solved view, cov() at once
    __device__ __forceinline__ uint8_t view_cov(int64_t o, float2& t, float2& mu, float co[3]) const {
        const uint8_t f = view(o, t, mu);
        if (f == 1) cov(o, co);
        return f;
    }
};

// Per-view results solved on the fly from the accumulator records (the
// fused update): the same arithmetic as tg_solve_views, the same FP32
// rounding of mu' and Sigma', nothing stored in between.
struct RecordViews {
    const float4* acc;
    const float4* rec;
    const float* cov2d;
    const ushort4* rect;
    const tg_params* prm;
    __device__ __forceinline__ uint8_t solve(int64_t o, float2& t, double th[6]) const {
        const float4 a0 = acc[4 * o], a1 = acc[4 * o + 1], a2 = acc[4 * o + 2], a3 = acc[4 * o + 3];
        const ushort4 r = rect[o];
        t = make_float2(a0.x, a3.x);
        return solve_record(a0, a1, a2, a3, !(r.z > r.x && r.w > r.y), *prm, th);
    }
    __device__ __forceinline__ uint8_t screen(int64_t o, float2& t) const {
        double th[6];
        return solve(o, t, th);
    }
    // the same in two halves: the record's loads (issued ahead), then the solve
    struct Rec {
        float4 a0, a1, a2, a3;
        ushort4 r;
    };
    __device__ __forceinline__ Rec fetch(int64_t o) const {
        return Rec{acc[4 * o], acc[4 * o + 1], acc[4 * o + 2], acc[4 * o + 3], rect[o]};
    }
    __device__ __forceinline__ uint8_t screen_rec(const Rec& q, float2& t) const {
        double th[6];
        t = make_float2(q.a0.x, q.a3.x);
        return solve_record(q.a0, q.a1, q.a2, q.a3, !(q.r.z > q.r.x && q.r.w > q.r.y), *prm, th);
    }
    __device__ __forceinline__ uint8_t view(int64_t o, float2& t, float2& mu) const {
        double th[6];
        const uint8_t f = solve(o, t, th);
        if (f == 1) {
            const float4 rc = rec[2 * o];
            mu = moved_centre(th, rc.x, rc.y);
        }
        return f;
    }
    __device__ __forceinline__ void cov(int64_t o, float co[3]) const {
        double th[6];
        float2 t;
        solve(o, t, th);
        moved_cov(th, cov2d[3 * o], cov2d[3 * o + 1], cov2d[3 * o + 2], co);
    }
    // view() and, for a solved view, cov() from the same solve
    __device__ __forceinline__ uint8_t view_cov(int64_t o, float2& t, float2& mu, float co[3]) const {
        double th[6];
        const uint8_t f = solve(o, t, th);
        if (f == 1) {
            const float4 rc = rec[2 * o];
            mu = moved_centre(th, rc.x, rc.y);
            moved_cov(th, cov2d[3 * o], cov2d[3 * o + 1], cov2d[3 * o + 2], co);
        }
        return f;
    }
};

// Solved views whose Sigma' the DLT loop keeps in LDS for the covariance
// loop (views past these are solved again there): 20 x 3 floats x 256
// threads = 60 KB per block, so the two blocks a CU holds (256 VGPRs) fit.
constexpr int TRI_COV_SLOTS = 20;

// The full multi-view update of Gaussian g from the per-view results of
// `src`; cams holds the V cameras.  covs: this thread's LDS slots, slot k
// component c at covs[(3 * k + c) * stride].
template <class Src>
__device__ __forceinline__ void tri_one(const Src& src, const GaussIO& a, const tg_camera* cams,
                                        const tg_params& prm, int64_t g, float* covs, int stride)
{
    const float om0 = a.means_in[3 * g], om1 = a.means_in[3 * g + 1], om2 = a.means_in[3 * g + 2];
    const float oq0 = a.quats_in[4 * g], oq1 = a.quats_in[4 * g + 1], oq2 = a.quats_in[4 * g + 2],
                oq3 = a.quats_in[4 * g + 3];
    const float os0 = a.scales_in[3 * g], os1 = a.scales_in[3 * g + 1], os2 = a.scales_in[3 * g + 2];
    float nm[3] = {om0, om1, om2};
    float nq[4] = {oq0, oq1, oq2, oq3};
    float ns[3] = {os0, os1, os2};
    uint32_t st = 0;

    // ---- totals and DLT normal matrix (4x4)
    double M[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) M[i] = 0.0;
    int nv = 0;
    uint32_t solved = 0;   // bit v: view v solved (V <= 32)
    double sw = 0.0, nt = 0.0;
    for (int v = 0; v < a.V; ++v) {
        const int64_t o = (int64_t)v * a.N + g;
        // culled views accumulate nothing, so their totals are zero
        float2 t, mu;
        float co[3];
        const uint8_t f = nv < TRI_COV_SLOTS ? src.view_cov(o, t, mu, co) : src.view(o, t, mu);
        sw += (double)t.x;
        nt += (double)t.y;
        if (f & 32) st |= 256;
        if (f != 1) continue;
        if (nv < TRI_COV_SLOTS) {
#pragma unroll
            for (int c = 0; c < 3; ++c) covs[(3 * nv + c) * stride] = co[c];
        }
        ++nv;
        solved |= 1u << v;
        const tg_camera& c = cams[v];
        const double xn = ((double)mu.x - c.cx) / c.fx, yn = ((double)mu.y - c.cy) / c.fy;
        double r1[4], r2[4];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r1[j] = xn * c.R[6 + j] - c.R[j];
            r2[j] = yn * c.R[6 + j] - c.R[3 + j];
        }
        r1[3] = xn * c.t[2] - c.t[0];
        r2[3] = yn * c.t[2] - c.t[1];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) M[i * 4 + j] += r1[i] * r1[j] + r2[i] * r2[j];
    }
    if (nv < prm.views_min) st |= 4;
    if (!(sw >= prm.wsum_total_min)) st |= 8;
    if (nt < (double)prm.pix_total_min) st |= 16;
    if ((st & ~256u) == 0) {
        double E[16];
        jacobi_eig<4>(M, E);
        int kmin = 0;
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if (M[k * 4 + k] < M[kmin * 4 + kmin]) kmin = k;
        double h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = E[i * 4 + kmin];
        const double hn = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2] + h[3] * h[3]);
        if (!(fabs(h[3]) >= 1e-12 * hn)) st |= 64;
        double mu3[3] = {0, 0, 0};
        if ((st & ~256u) == 0) {
            mu3[0] = h[0] / h[3];
            mu3[1] = h[1] / h[3];
            mu3[2] = h[2] / h[3];
            for (uint32_t m = solved; m; m &= m - 1) {
                const tg_camera& c = cams[__builtin_ctz(m)];
                const double pz = c.R[6] * mu3[0] + c.R[7] * mu3[1] + c.R[8] * mu3[2] + c.t[2];
                if (!(pz > prm.near_z)) st |= 128;
            }
        }
        if ((st & ~256u) == 0) {
            st |= 1;
            nm[0] = (float)mu3[0];
            nm[1] = (float)mu3[1];
            nm[2] = (float)mu3[2];
            // ---- covariance system: unknowns (S00, S01, S02, S11, S12, S22)
            double AtA[36], Atb[6];
#pragma unroll
            for (int i = 0; i < 36; ++i) AtA[i] = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) Atb[i] = 0.0;
            int k = 0;   // solved views so far, in view order
            for (uint32_t m = solved; m; m &= m - 1, ++k) {
                const int v = __builtin_ctz(m);
                const int64_t o = (int64_t)v * a.N + g;
                const tg_camera& c = cams[v];
                double p[3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    p[i] = c.R[3 * i] * mu3[0] + c.R[3 * i + 1] * mu3[1] + c.R[3 * i + 2] * mu3[2] + c.t[i];
                const double limx = (double)prm.j_clamp * (0.5 * c.width / (double)c.fx);
                const double limy = (double)prm.j_clamp * (0.5 * c.height / (double)c.fy);
                const double ip2 = 1.0 / p[2];   // one FP64 reciprocal instead of six divisions
                const double tx = fmin(limx, fmax(-limx, p[0] * ip2));
                const double ty = fmin(limy, fmax(-limy, p[1] * ip2));
                const double J00 = c.fx * ip2, J02 = -c.fx * tx * ip2;
                const double J11 = c.fy * ip2, J12 = -c.fy * ty * ip2;
                double T0[3], T1[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    T0[j] = J00 * c.R[j] + J02 * c.R[6 + j];
                    T1[j] = J11 * c.R[3 + j] + J12 * c.R[6 + j];
                }
                float co[3];
                if (k < TRI_COV_SLOTS) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) co[e] = covs[(3 * k + e) * stride];
                } else {
                    src.cov(o, co);
                }
                const double rhs[3] = {co[0], co[1], co[2]};
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const double* Ta = e == 2 ? T1 : T0;
                    const double* Tb = e == 0 ? T0 : T1;
                    double row[6];
                    row[0] = Ta[0] * Tb[0];
                    row[1] = Ta[0] * Tb[1] + Ta[1] * Tb[0];
                    row[2] = Ta[0] * Tb[2] + Ta[2] * Tb[0];
                    row[3] = Ta[1] * Tb[1];
                    row[4] = Ta[1] * Tb[2] + Ta[2] * Tb[1];
                    row[5] = Ta[2] * Tb[2];
#pragma unroll
                    for (int i = 0; i < 6; ++i) {
                        Atb[i] += row[i] * rhs[e];
#pragma unroll
                        for (int j = 0; j < 6; ++j) AtA[i * 6 + j] += row[i] * row[j];
                    }
                }
            }
            // Cholesky AtA = L L^T
            double dmax = 0.0;
#pragma unroll
            for (int i = 0; i < 6; ++i) dmax = fmax(dmax, AtA[i * 6 + i]);
            // two solved views leave the 6-unknown system at rank 5 (the
            // symmetric product of the two viewing rays is seen by neither),
            // a structural fact that FP64 pivots cannot resolve (their
            // rounding floor sits near 1e-16 of the largest)
            bool pd = dmax > 0.0 && nv >= 3;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double d = AtA[j * 6 + j];
#pragma unroll
                for (int k = 0; k < j; ++k) d -= AtA[j * 6 + k] * AtA[j * 6 + k];
                if (!(d > 1e-24 * dmax)) pd = false;
                d = sqrt(fmax(d, 1e-300));
                AtA[j * 6 + j] = d;
#pragma unroll
                for (int i = j + 1; i < 6; ++i) {
                    double sacc = AtA[i * 6 + j];
#pragma unroll
                    for (int k = 0; k < j; ++k) sacc -= AtA[i * 6 + k] * AtA[j * 6 + k];
                    AtA[i * 6 + j] = sacc / d;
                }
            }
            double sol[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) {  // forward
                double sacc = Atb[i];
#pragma unroll
                for (int k = 0; k < i; ++k) sacc -= AtA[i * 6 + k] * sol[k];
                sol[i] = sacc / AtA[i * 6 + i];
            }
#pragma unroll
            for (int i = 5; i >= 0; --i) {  // backward
                double sacc = sol[i];
#pragma unroll
                for (int k = i + 1; k < 6; ++k) sacc -= AtA[k * 6 + i] * sol[k];
                sol[i] = sacc / AtA[i * 6 + i];
            }
            double S[9] = {sol[0], sol[1], sol[2], sol[1], sol[3], sol[4], sol[2], sol[4], sol[5]};
            double Ev[9];
            jacobi_eig<3>(S, Ev);
            double lam[3] = {S[0], S[4], S[8]};
            if (!pd || !(lam[0] > 0.0 && lam[1] > 0.0 && lam[2] > 0.0)) {
                st |= 32;
            } else {
                // ascending eigen-order (stable for ties)
                int ord[3] = {0, 1, 2};
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2 - i; ++j)
                        if (lam[ord[j + 1]] < lam[ord[j]]) {
                            int t = ord[j]; ord[j] = ord[j + 1]; ord[j + 1] = t;
                        }
                // rank of each old scale among the old scales (stable)
                const float so[3] = {os0, os1, os2};
                int rk[3];
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    int r = 0;
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        if (so[j] < so[kx] || (so[j] == so[kx] && j < kx)) ++r;
                    rk[kx] = r;
                }
                // old rotation (FP64, normalised quaternion)
                const double qn = sqrt((double)oq0 * oq0 + (double)oq1 * oq1 + (double)oq2 * oq2 + (double)oq3 * oq3);
                const double w = oq0 / qn, x = oq1 / qn, y = oq2 / qn, z = oq3 / qn;
                const double Ro[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                                      2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                                      2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
                double Rn[9], sc[3], dots[3];
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int e = ord[rk[kx]];
                    double dt = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        Rn[i * 3 + kx] = Ev[i * 3 + e];
                        dt += Ev[i * 3 + e] * Ro[i * 3 + kx];
                    }
                    if (dt < 0.0) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) Rn[i * 3 + kx] = -Rn[i * 3 + kx];
                        dt = -dt;
                    }
                    dots[kx] = dt;
                    sc[kx] = lam[e];
                }
                const double det = Rn[0] * (Rn[4] * Rn[8] - Rn[5] * Rn[7]) - Rn[1] * (Rn[3] * Rn[8] - Rn[5] * Rn[6]) +
                                   Rn[2] * (Rn[3] * Rn[7] - Rn[4] * Rn[6]);
                if (det < 0.0) {
                    int km = 0;
                    if (dots[1] < dots[km]) km = 1;
                    if (dots[2] < dots[km]) km = 2;
#pragma unroll
                    for (int i = 0; i < 3; ++i) Rn[i * 3 + km] = -Rn[i * 3 + km];
                }
                double qq[4];
                quat_from_rot(Rn, qq);
#pragma unroll
                for (int i = 0; i < 4; ++i) nq[i] = (float)qq[i];
#pragma unroll
                for (int i = 0; i < 3; ++i) ns[i] = a.scale_mode == 1 ? (float)(0.5 * log(sc[i])) : (float)sqrt(sc[i]);
                st |= 2;
            }
        }
    }
    a.means_out[3 * g] = nm[0];
    a.means_out[3 * g + 1] = nm[1];
    a.means_out[3 * g + 2] = nm[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a.quats_out[4 * g + i] = nq[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) a.scales_out[3 * g + i] = ns[i];
    if (a.status) a.status[g] = st;
}

// Status from the totals that decide whether a Gaussian is a candidate at
// all (views solved, accumulated alpha, pixels); a non-candidate is copied
// and done.
__device__ __forceinline__ uint32_t light_status(int nv, double sw, double nt, bool nonfinite, const tg_params& prm) {
    uint32_t st = nonfinite ? 256u : 0u;
    if (nv < prm.views_min) st |= 4;
    if (!(sw >= prm.wsum_total_min)) st |= 8;
    if (nt < (double)prm.pix_total_min) st |= 16;
    return st;
}

// A block first screens TRI_ITEMS x 256 Gaussians with the cheap totals and
// compacts the candidates in LDS, then runs the full update on the compacted
// list, so the register-heavy FP64 part runs in dense waves even when few
// Gaussians qualify.  A span of 1024 keeps the candidates of a block (about
// one in seven Gaussians on large scenes) within one pass of its 256 threads,
// so a block waits out one full update, not two (2048: 2 passes, 5% slower).
constexpr int TRI_THREADS = 256;
constexpr int TRI_ITEMS = 4;
constexpr int TRI_SPAN = TRI_THREADS * TRI_ITEMS;
constexpr int TRI_GROUP = 4;   // records in flight together in the screen

template <class Src>
__device__ __forceinline__ void tri_block(const Src& src, const GaussIO& a, const tg_camera* cams,
                                          const tg_params& prm, int64_t base, uint32_t* cand, uint32_t& cn,
                                          float* covs)
{
    const int t = threadIdx.x;
    if (t == 0) cn = 0;
    __syncthreads();
    // Screen: views outer, the thread's Gaussians inner in groups of
    // TRI_GROUP, so the group's records of one view are in flight together
    // (a view loop per Gaussian waits out one round trip per record).  The
    // totals add in view order, as one Gaussian's loop would.
    int nv[TRI_ITEMS];
    bool nonfinite[TRI_ITEMS];
    double sw[TRI_ITEMS], nt[TRI_ITEMS];
#pragma unroll
    for (int it = 0; it < TRI_ITEMS; ++it) {
        nv[it] = 0;
        nonfinite[it] = false;
        sw[it] = 0.0;
        nt[it] = 0.0;
    }
    for (int v = 0; v < a.V; ++v) {
#pragma unroll
        for (int i0 = 0; i0 < TRI_ITEMS; i0 += TRI_GROUP) {
            typename Src::Rec r[TRI_GROUP];
            // unconditional loads (past N: the last Gaussian's, unused), so
            // they issue together
#pragma unroll
            for (int j = 0; j < TRI_GROUP; ++j) {
                const int64_t g = base + (int64_t)(i0 + j) * TRI_THREADS + t;
                r[j] = src.fetch((int64_t)v * a.N + (g < a.N ? g : a.N - 1));
            }
#pragma unroll
            for (int j = 0; j < TRI_GROUP; ++j) {
                const int64_t g = base + (int64_t)(i0 + j) * TRI_THREADS + t;
                if (g < a.N) {
                    float2 tt;
                    const uint8_t f = src.screen_rec(r[j], tt);
                    sw[i0 + j] += (double)tt.x;
                    nt[i0 + j] += (double)tt.y;
                    if (f == 1) ++nv[i0 + j];
                    if (f & 32) nonfinite[i0 + j] = true;
                }
            }
        }
    }
    // Candidates go to the LDS list; every other Gaussian is copied through
    // (a Gaussian with a non-finite parameter is always copied, culled in
    // every view).  All the copied items' loads come before the first
    // store: the outputs may alias the inputs, so a store between loads
    // would make each load wait for the one before.
    float x[TRI_ITEMS][11];
    uint32_t stc[TRI_ITEMS];
    bool cp[TRI_ITEMS];
#pragma unroll
    for (int it = 0; it < TRI_ITEMS; ++it) {
        const int64_t g = base + (int64_t)it * TRI_THREADS + t;
        cp[it] = false;
        stc[it] = 0;
        if (g >= a.N) continue;
        const uint32_t st = light_status(nv[it], sw[it], nt[it], nonfinite[it], prm);
        if ((st & ~256u) == 0) {
            cand[atomicAdd(&cn, 1u)] = (uint32_t)(g - base);
        } else {
            cp[it] = true;
            stc[it] = st;
#pragma unroll
            for (int k = 0; k < 3; ++k) x[it][k] = a.means_in[3 * g + k];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[it][3 + k] = a.quats_in[4 * g + k];
#pragma unroll
            for (int k = 0; k < 3; ++k) x[it][7 + k] = a.scales_in[3 * g + k];
            x[it][10] = a.opacity_in[g];
        }
    }
#pragma unroll
    for (int it = 0; it < TRI_ITEMS; ++it) {
        if (!cp[it]) continue;
        const int64_t g = base + (int64_t)it * TRI_THREADS + t;
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 11; ++k) fin &= isfinite(x[it][k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) a.means_out[3 * g + k] = x[it][k];
#pragma unroll
        for (int k = 0; k < 4; ++k) a.quats_out[4 * g + k] = x[it][3 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) a.scales_out[3 * g + k] = x[it][7 + k];
        if (a.status) a.status[g] = fin ? stc[it] : (stc[it] | 256u);
    }
    __syncthreads();
    const uint32_t n = cn;
    for (uint32_t i = t; i < n; i += TRI_THREADS) tri_one(src, a, cams, prm, base + cand[i], covs + t, TRI_THREADS);
}

__global__ void __launch_bounds__(TRI_THREADS) k_triangulate(StoredViews src, GaussIO a, CamPack cams, tg_params prm)
{
    __shared__ uint32_t cand[TRI_SPAN];
    __shared__ uint32_t cn;
    __shared__ float covs[TRI_COV_SLOTS * 3 * TRI_THREADS];
    tri_block(src, a, cams.cam, prm, (int64_t)blockIdx.x * TRI_SPAN, cand, cn, covs);
}

// ---- fused per-view solve + multi-view update, batched over Gaussian sets
// and frames (one launch per serving step).
struct UpdSlotK {
    const float4* rec;
    const float* cov2d;
    const ushort4* rect;
    const tg_camera* cams;   // device [V]
    const float* means_in;
    const float* quats_in;
    const float* scales_in;
    const float* opacity_in;
    int64_t N;
    int32_t V;
    int32_t scale_mode;
};

struct UpdFrameK {
    const float4* acc;
    float* means_out;
    float* quats_out;
    float* scales_out;
    uint32_t* status;
    int32_t slot;
    int32_t blk0;            // first block of this frame in the launch
};

constexpr int UPD_MAX_ITEMS = TG_MAX_SLOTS * TG_MAX_FRAMES;

struct UpdBatchK {
    UpdSlotK slot[TG_MAX_SLOTS];
    UpdFrameK fr[UPD_MAX_ITEMS];
    int32_t n_fr;
};

__device__ __forceinline__ void update_item(const UpdSlotK& sl, const UpdFrameK& fr, const tg_camera* lcam,
                                            const tg_params& prm, int64_t blk, uint32_t* cand, uint32_t& cn,
                                            float* covs)
{
    RecordViews src{fr.acc, sl.rec, sl.cov2d, sl.rect, &prm};
    GaussIO a{sl.means_in, sl.quats_in, sl.scales_in, sl.opacity_in, fr.means_out, fr.quats_out, fr.scales_out,
              fr.status, sl.N, sl.V, sl.scale_mode};
    tri_block(src, a, lcam, prm, blk * TRI_SPAN, cand, cn, covs);
}

// One frame; cameras in the kernel arguments.
__global__ void __launch_bounds__(TRI_THREADS) k_update_one(UpdSlotK sl, UpdFrameK fr, CamPack cams, tg_params prm)
{
    __shared__ uint32_t cand[TRI_SPAN];
    __shared__ uint32_t cn;
    __shared__ float covs[TRI_COV_SLOTS * 3 * TRI_THREADS];
    update_item(sl, fr, cams.cam, prm, blockIdx.x, cand, cn, covs);
}

// Several (Gaussian set, frame) items; each set's cameras are copied from
// device memory into LDS by the block.
__global__ void __launch_bounds__(TRI_THREADS) k_update_batch(UpdBatchK b, tg_params prm)
{
    __shared__ uint32_t cand[TRI_SPAN];
    __shared__ uint32_t cn;
    __shared__ tg_camera lcam[TG_MAX_VIEWS];
    __shared__ float covs[TRI_COV_SLOTS * 3 * TRI_THREADS];
    int k = 0;
    while (k + 1 < b.n_fr && b.fr[k + 1].blk0 <= (int32_t)blockIdx.x) ++k;
    const UpdFrameK& fr = b.fr[k];
    const UpdSlotK& sl = b.slot[fr.slot];
    {
        const int nw = sl.V * (int)(sizeof(tg_camera) / 4);
        const uint32_t* src = (const uint32_t*)sl.cams;
        uint32_t* dst = (uint32_t*)lcam;
        for (int i = threadIdx.x; i < nw; i += TRI_THREADS) dst[i] = src[i];
    }
    __syncthreads();
    update_item(sl, fr, lcam, prm, (int64_t)blockIdx.x - fr.blk0, cand, cn, covs);
}

tg_status check_gauss(const tg_gaussians* g, bool in) {
    if (!g || !g->means || !g->quats || !g->scales || (in && !g->opacity)) return TG_ERR_INVALID_ARG;
    if (in && (g->scale_mode < 0 || g->scale_mode > 1)) return TG_ERR_INVALID_ARG;
    return TG_OK;
}

UpdSlotK slot_args(const tg_splats* s, const tg_gaussians* g_in, const tg_camera* cams_dev, int64_t N, int V) {
    UpdSlotK k;
    k.rec = (const float4*)s->rec;
    k.cov2d = s->cov2d;
    k.rect = (const ushort4*)s->rect;
    k.cams = cams_dev;
    k.means_in = g_in->means;
    k.quats_in = g_in->quats;
    k.scales_in = g_in->scales;
    k.opacity_in = g_in->opacity;
    k.N = N;
    k.V = V;
    k.scale_mode = g_in->scale_mode;
    return k;
}

UpdFrameK frame_args(const float* acc, tg_gaussians* g_out, uint32_t* status, int slot, int blk0) {
    UpdFrameK f;
    f.acc = (const float4*)acc;
    f.means_out = g_out->means;
    f.quats_out = g_out->quats;
    f.scales_out = g_out->scales;
    f.status = status;
    f.slot = slot;
    f.blk0 = blk0;
    return f;
}

}  // namespace

extern "C" tg_status tg_solve_views(const float* acc, const tg_splats* s, int64_t N, int32_t V, const tg_params* p,
                                    float* mu2d_new, float* cov2d_new, uint8_t* vflags, float* wn, void* stream)
{
    if (!acc || !s || !p || !mu2d_new || !cov2d_new || !vflags || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (!s->rec || !s->cov2d || !s->rect) return TG_ERR_INVALID_ARG;
    if (!aligned16(acc) || !aligned16(s->rec) || ((uintptr_t)mu2d_new & 7u) || ((uintptr_t)wn & 7u))
        return TG_ERR_ALIGNMENT;
    const int64_t VN = (int64_t)V * N;
    if (VN == 0) return TG_OK;
    hipLaunchKernelGGL(k_solve_views, dim3((unsigned)((VN + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const float4*)acc, (const float4*)s->rec, s->cov2d, (const ushort4*)s->rect, VN, *p,
                       (float2*)mu2d_new, cov2d_new, vflags, (float2*)wn);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_triangulate(const float* mu2d_new, const float* cov2d_new, const uint8_t* vflags,
                                    const float* wn, const tg_splats* s, const tg_gaussians* g_in, int64_t N,
                                    const tg_camera* cams, int32_t V, const tg_params* p, tg_gaussians* g_out,
                                    uint32_t* status, void* stream)
{
    if (!mu2d_new || !cov2d_new || !vflags || !wn || !s || !cams || !p || N < 0 || V < 1)
        return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (check_gauss(g_in, true) != TG_OK || check_gauss(g_out, false) != TG_OK) return TG_ERR_INVALID_ARG;
    if (((uintptr_t)mu2d_new & 7u) || ((uintptr_t)wn & 7u)) return TG_ERR_ALIGNMENT;
    if (N == 0) return TG_OK;
    StoredViews src{(const float2*)mu2d_new, cov2d_new, vflags, (const float2*)wn};
    GaussIO a{g_in->means, g_in->quats, g_in->scales, g_in->opacity, g_out->means, g_out->quats, g_out->scales,
              status, N, V, g_in->scale_mode};
    CamPack cp;
    for (int v = 0; v < V; ++v) cp.cam[v] = cams[v];
    hipLaunchKernelGGL(k_triangulate, dim3((unsigned)((N + TRI_SPAN - 1) / TRI_SPAN)), dim3(TRI_THREADS), 0,
                       (hipStream_t)stream, src, a, cp, *p);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_solve_triangulate(const float* acc, const tg_splats* s, const tg_gaussians* g_in, int64_t N,
                                          const tg_camera* cams, int32_t V, const tg_params* p, tg_gaussians* g_out,
                                          uint32_t* status, void* stream)
{
    if (!acc || !s || !cams || !p || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS) return TG_ERR_UNSUPPORTED;
    if (!s->rec || !s->cov2d || !s->rect) return TG_ERR_INVALID_ARG;
    if (check_gauss(g_in, true) != TG_OK || check_gauss(g_out, false) != TG_OK) return TG_ERR_INVALID_ARG;
    if (!aligned16(acc) || !aligned16(s->rec)) return TG_ERR_ALIGNMENT;
    if (N == 0) return TG_OK;
    if ((N + TRI_SPAN - 1) / TRI_SPAN > (int64_t)0x7FFFFFFF) return TG_ERR_UNSUPPORTED;
    CamPack cp;
    for (int v = 0; v < V; ++v) cp.cam[v] = cams[v];
    const UpdSlotK sl = slot_args(s, g_in, nullptr, N, V);
    const UpdFrameK fr = frame_args(acc, g_out, status, 0, 0);
    hipLaunchKernelGGL(k_update_one, dim3((unsigned)((N + TRI_SPAN - 1) / TRI_SPAN)), dim3(TRI_THREADS), 0,
                       (hipStream_t)stream, sl, fr, cp, *p);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_solve_triangulate_batch(const tg_upd_slot* slots, int32_t n_slots, const tg_params* p,
                                                void* stream)
{
    if (!p || n_slots < 0 || (n_slots > 0 && !slots)) return TG_ERR_INVALID_ARG;
    if (n_slots > TG_MAX_SLOTS) return TG_ERR_UNSUPPORTED;
    UpdBatchK b;
    b.n_fr = 0;
    int64_t blocks = 0;
    // every argument is checked before anything is launched
    for (int k = 0; k < n_slots; ++k) {
        const tg_upd_slot& u = slots[k];
        if (!u.s || !u.g_in || !u.cams || u.N < 0 || u.V < 1) return TG_ERR_INVALID_ARG;
        if (u.V > TG_MAX_VIEWS || u.F < 1 || u.F > TG_MAX_FRAMES) return TG_ERR_UNSUPPORTED;
        if (!u.s->rec || !u.s->cov2d || !u.s->rect || check_gauss(u.g_in, true) != TG_OK) return TG_ERR_INVALID_ARG;
        if (!aligned16(u.s->rec) || ((uintptr_t)u.cams & 3u)) return TG_ERR_ALIGNMENT;
        b.slot[k] = slot_args(u.s, u.g_in, u.cams, u.N, u.V);
        if (u.N == 0) continue;
        const int64_t nb = (u.N + TRI_SPAN - 1) / TRI_SPAN;
        for (int f = 0; f < u.F; ++f) {
            if (!u.acc[f] || check_gauss(u.g_out[f], false) != TG_OK) return TG_ERR_INVALID_ARG;
            if (!aligned16(u.acc[f])) return TG_ERR_ALIGNMENT;
            b.fr[b.n_fr++] = frame_args(u.acc[f], u.g_out[f], u.status[f], k, (int32_t)blocks);
            blocks += nb;
            if (blocks > (int64_t)0x7FFFFFFF) return TG_ERR_UNSUPPORTED;
        }
    }
    if (blocks == 0) return TG_OK;
    hipLaunchKernelGGL(k_update_batch, dim3((unsigned)blocks), dim3(TRI_THREADS), 0, (hipStream_t)stream, b, *p);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
