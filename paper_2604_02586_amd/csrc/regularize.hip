// tg_regularize: motion regularisation after the multi-view update
// (TrackerSplat Sec. 4.5; K = 8 neighbours, Sec. 5.2).
//
//   k_reg_classify  per Gaussian: static test over the views' pixel counts
//                   (Sec. 4.5.2), solved = position and covariance updated
//                   and not static; the change against the first frame
//                   (d_mu, Euler angles of R' R^T, d_S) of every solved
//                   Gaussian; bounding box and count of the solved set.
//   k_reg_grid      one thread: a uniform grid over the solved set (about two
//                   solved Gaussians per cell, at most 2^21 cells).
//   k_reg_keys + radix sort + k_reg_cells
//                   solved Gaussians sorted by grid cell; per-cell ranges and
//                   the sorted positions as float4 (coalesced reads).
//   k_reg_knn       per non-static Gaussian: exact K nearest solved
//                   Gaussians by expanding shells of cells, FP64 distances,
//                   ties by index; stops once no unvisited cell can hold a
//                   closer one.
//   k_reg_filter    per solved Gaussian: component-wise median of its
//                   neighbours' changes (itself included).
//   k_reg_apply     per Gaussian: static -> first frame; solved -> first
//                   frame + filtered change; other -> first frame + mean of
//                   the neighbours' filtered changes.
#include "tg_internal.h"

namespace {

constexpr int KMAX = TG_REG_K_MAX;
constexpr int CELL_BITS = 21;
constexpr uint32_t CELL_MAX = 1u << CELL_BITS;
constexpr uint32_t KEY_NONE = CELL_MAX;   // non-solved: sorts after every cell
constexpr int SORT_PASSES = 3;            // 22 key bits

enum : uint8_t { CLS_STATIC = 0, CLS_SOURCE = 1, CLS_TARGET = 2 };

struct GridInfo {
    float lo[3];
    float inv_h;
    double h;
    int32_t dim[3];
    uint32_t n_src;
    int32_t box[6];   // order-preserving integer images of min xyz, max xyz
};

__device__ __forceinline__ int32_t f2o(float f) {
    const int32_t i = __builtin_bit_cast(int32_t, f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float o2f(int32_t i) { return __builtin_bit_cast(float, i >= 0 ? i : i ^ 0x7FFFFFFF); }

__device__ inline void quat_rot64(const float* q, double R[9]) {
    const double n = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Rz(psi) Ry(theta) Rx(phi)
__device__ inline void rot_zyx(double phi, double theta, double psi, double Q[9]) {
    const double cx = cos(phi), sx = sin(phi), cy = cos(theta), sy = sin(theta), cz = cos(psi), sz = sin(psi);
    Q[0] = cz * cy; Q[1] = cz * sy * sx - sz * cx; Q[2] = cz * sy * cx + sz * sx;
    Q[3] = sz * cy; Q[4] = sz * sy * sx + cz * cx; Q[5] = sz * sy * cx - cz * sx;
    Q[6] = -sy;     Q[7] = cy * sx;                Q[8] = cy * cx;
}

// Rotation matrix -> unit quaternion (w, x, y, z), w >= 0 (Shepperd: pivot
// on the largest of w^2, x^2, y^2, z^2).
__device__ inline void rot_quat(const double R[9], double q[4]) {
    const double tr = R[0] + R[4] + R[8];
    int k = 0;
    double best = tr;
    if (R[0] > best) { best = R[0]; k = 1; }
    if (R[4] > best) { best = R[4]; k = 2; }
    if (R[8] > best) { best = R[8]; k = 3; }
    if (k == 0) {
        const double s = sqrt(fmax(1 + tr, 0.0)) * 2;
        q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
    } else if (k == 1) {
        const double s = sqrt(fmax(1 + R[0] - R[4] - R[8], 0.0)) * 2;
        q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
    } else if (k == 2) {
        const double s = sqrt(fmax(1 - R[0] + R[4] - R[8], 0.0)) * 2;
        q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
    } else {
        const double s = sqrt(fmax(1 - R[0] - R[4] + R[8], 0.0)) * 2;
        q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
    }
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = q[0] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < 4; ++i) q[i] = sg * q[i] / n;
}

struct RegArgs {
    const float* m0;   // first frame
    const float* q0;
    const float* s0;
    const float* m1;   // multi-view update
    const float* q1;
    const float* s1;
    const uint32_t* status;
    const float* acc;
    float* mo;         // output
    float* qo;
    float* so;
    uint32_t* reg;
    int64_t N;
    int V;
    int K;
    int static_min_pix;
    int static_views;
    double static_frac;
    // workspace
    uint8_t* cls;
    float* delta;      // [N,9]
    float* filt;       // [N,9]
    uint32_t* nbr;     // [N,KMAX] neighbour Gaussian indices
    uint8_t* ncnt;     // [N]
    uint32_t* keys;    // [N]
    const uint32_t* skeys;   // [N] sorted
    const uint32_t* svals;   // [N] Gaussian index of each sorted key
    uint2* ranges;     // [CELL_MAX]
    float4* spos;      // [N] sorted positions, index bits in w
    GridInfo* grid;
};

__global__ void k_reg_init(GridInfo* gi) {
    gi->n_src = 0;
    for (int i = 0; i < 3; ++i) {
        gi->box[i] = 0x7FFFFFFF;
        gi->box[3 + i] = (int32_t)0x80000000;
    }
}

__global__ void __launch_bounds__(256) k_reg_classify(RegArgs a) {
    __shared__ int32_t bmin[3], bmax[3];
    __shared__ uint32_t bcnt;
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) {
            bmin[i] = 0x7FFFFFFF;
            bmax[i] = (int32_t)0x80000000;
        }
        bcnt = 0;
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < a.N) {
        // static: more than static_min_pix pixels, more than static_frac of
        // them static, in at least static_views views (decided in FP64 on the
        // exact integer counts)
        int sv = 0;
        for (int v = 0; v < a.V; ++v) {
            const float* r = a.acc + ((int64_t)v * a.N + g) * TG_ACC_STRIDE;
            const double n = r[12], sn = r[13];
            if (n > (double)a.static_min_pix && sn > a.static_frac * n) ++sv;
        }
        const bool stat = sv >= a.static_views;
        const uint32_t st = a.status[g];
        const bool src = !stat && (st & 1u) && (st & 2u);
        a.cls[g] = stat ? CLS_STATIC : (src ? CLS_SOURCE : CLS_TARGET);
        if (src) {
            double R0[9], R1[9], Q[9];
            quat_rot64(a.q0 + 4 * g, R0);
            quat_rot64(a.q1 + 4 * g, R1);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    Q[i * 3 + j] = R1[i * 3] * R0[j * 3] + R1[i * 3 + 1] * R0[j * 3 + 1] + R1[i * 3 + 2] * R0[j * 3 + 2];
            float* d = a.delta + g * 9;
            for (int i = 0; i < 3; ++i) d[i] = (float)((double)a.m1[3 * g + i] - (double)a.m0[3 * g + i]);
            d[3] = (float)atan2(Q[7], Q[8]);
            d[4] = (float)asin(fmin(1.0, fmax(-1.0, -Q[6])));
            d[5] = (float)atan2(Q[3], Q[0]);
            for (int i = 0; i < 3; ++i) d[6 + i] = (float)((double)a.s1[3 * g + i] - (double)a.s0[3 * g + i]);
            for (int i = 0; i < 3; ++i) {
                const int32_t o = f2o(a.m0[3 * g + i]);
                atomicMin(&bmin[i], o);
                atomicMax(&bmax[i], o);
            }
            atomicAdd(&bcnt, 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && bcnt) {
        for (int i = 0; i < 3; ++i) {
            atomicMin(&a.grid->box[i], bmin[i]);
            atomicMax(&a.grid->box[3 + i], bmax[i]);
        }
        atomicAdd(&a.grid->n_src, bcnt);
    }
}

__global__ void k_reg_grid(GridInfo* gi) {
    if (gi->n_src == 0) {
        for (int i = 0; i < 3; ++i) {
            gi->lo[i] = 0.f;
            gi->dim[i] = 1;
        }
        gi->h = 1.0;
        gi->inv_h = 1.0f;
        return;
    }
    double lo[3], ext[3];
    for (int i = 0; i < 3; ++i) {
        lo[i] = o2f(gi->box[i]);
        ext[i] = fmax((double)o2f(gi->box[3 + i]) - lo[i], 1e-6);
    }
    const double vol = ext[0] * ext[1] * ext[2];
    double h = cbrt(vol / fmax(1.0, 0.5 * gi->n_src));
    h = fmax(h, fmax(ext[0], fmax(ext[1], ext[2])) / 1024.0);
    int64_t d[3];
    for (;;) {
        int64_t prod = 1;
        for (int i = 0; i < 3; ++i) {
            d[i] = (int64_t)(ext[i] / h) + 1;
            prod *= d[i];
        }
        if (prod <= (int64_t)CELL_MAX) break;
        h *= 1.25;
    }
    for (int i = 0; i < 3; ++i) {
        gi->lo[i] = (float)lo[i];
        gi->dim[i] = (int32_t)d[i];
    }
    gi->h = h;
    gi->inv_h = (float)(1.0 / h);
}

__device__ __forceinline__ int cell_coord(float p, float lo, float inv_h, int dim) {
    int c = (int)((p - lo) * inv_h);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

__global__ void __launch_bounds__(256) k_reg_keys(RegArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N) return;
    uint32_t key = KEY_NONE;
    if (a.cls[g] == CLS_SOURCE) {
        const GridInfo& gi = *a.grid;
        const int cx = cell_coord(a.m0[3 * g], gi.lo[0], gi.inv_h, gi.dim[0]);
        const int cy = cell_coord(a.m0[3 * g + 1], gi.lo[1], gi.inv_h, gi.dim[1]);
        const int cz = cell_coord(a.m0[3 * g + 2], gi.lo[2], gi.inv_h, gi.dim[2]);
        key = (uint32_t)((cz * gi.dim[1] + cy) * gi.dim[0] + cx);
    }
    a.keys[g] = key;
}

__global__ void __launch_bounds__(256) k_fill_ranges(uint2* r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = make_uint2(0u, 0u);
}

__global__ void __launch_bounds__(256) k_reg_cells(RegArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const uint32_t key = a.skeys[i];
    if (key >= KEY_NONE) return;
    const uint32_t g = a.svals[i];
    if (g >= (uint64_t)a.N) return;
    if (i == 0 || a.skeys[i - 1] != key) a.ranges[key].x = (uint32_t)i;
    if (i == a.N - 1 || a.skeys[i + 1] != key) a.ranges[key].y = (uint32_t)(i + 1);
    a.spos[i] = make_float4(a.m0[3 * g], a.m0[3 * g + 1], a.m0[3 * g + 2], __builtin_bit_cast(float, g));
}

// insert (d2, id) into the sorted top list (ascending by d2, then id)
__device__ __forceinline__ void topk_insert(double* bd, uint32_t* bi, int& cnt, int K, double d2, uint32_t id) {
    if (cnt == K && !(d2 < bd[K - 1] || (d2 == bd[K - 1] && id < bi[K - 1]))) return;
    int j = cnt < K ? cnt++ : K - 1;
    while (j > 0 && (d2 < bd[j - 1] || (d2 == bd[j - 1] && id < bi[j - 1]))) {
        bd[j] = bd[j - 1];
        bi[j] = bi[j - 1];
        --j;
    }
    bd[j] = d2;
    bi[j] = id;
}

__global__ void __launch_bounds__(128) k_reg_knn(RegArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N) return;
    if (a.cls[g] == CLS_STATIC) {
        a.ncnt[g] = 0;
        return;
    }
    const GridInfo& gi = *a.grid;
    const int K = (int)((uint32_t)a.K < gi.n_src ? (uint32_t)a.K : gi.n_src);
    if (K == 0) {
        a.ncnt[g] = 0;
        return;
    }
    const float px = a.m0[3 * g], py = a.m0[3 * g + 1], pz = a.m0[3 * g + 2];
    const int hx = cell_coord(px, gi.lo[0], gi.inv_h, gi.dim[0]);
    const int hy = cell_coord(py, gi.lo[1], gi.inv_h, gi.dim[1]);
    const int hz = cell_coord(pz, gi.lo[2], gi.inv_h, gi.dim[2]);
    const int rmax = max(gi.dim[0], max(gi.dim[1], gi.dim[2]));
    double bd[KMAX];
    uint32_t bi[KMAX];
    int cnt = 0;
    // cells were assigned in FP32 ((p - lo) / h up to ~1024 carries ~1e-4 of a
    // cell of rounding), so faces are moved in by a margin
    const double h = gi.h, margin = 1e-3 * h;
    for (int r = 0; r <= rmax; ++r) {
        const int z0 = max(hz - r, 0), z1 = min(hz + r, gi.dim[2] - 1);
        const int y0 = max(hy - r, 0), y1 = min(hy + r, gi.dim[1] - 1);
        const int x0 = max(hx - r, 0), x1 = min(hx + r, gi.dim[0] - 1);
        // the cells at Chebyshev distance exactly r from the home cell
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) {
                const bool face = r == 0 || z == hz - r || z == hz + r || y == hy - r || y == hy + r;
                const int xa = face ? x0 : hx - r, xb = face ? x1 : hx + r;
                const int step = face ? 1 : 2 * r;
                for (int x = xa; x <= xb; x += step) {
                    if (x < 0 || x >= gi.dim[0]) continue;
                    const uint2 rg = a.ranges[(z * gi.dim[1] + y) * gi.dim[0] + x];
                    for (uint32_t i = rg.x; i < rg.y; ++i) {
                        const float4 q = a.spos[i];
                        const double dx = (double)q.x - px, dy = (double)q.y - py, dz = (double)q.z - pz;
                        topk_insert(bd, bi, cnt, K, dx * dx + dy * dy + dz * dz, __builtin_bit_cast(uint32_t, q.w));
                    }
                }
            }
        if (cnt == K) {
            // distance from p to the nearest face of the visited block of
            // cells, ignoring faces on the grid boundary (nothing beyond)
            double bound = 1e300;
            const float pp[3] = {px, py, pz};
            const int hc[3] = {hx, hy, hz};
            for (int ax = 0; ax < 3; ++ax) {
                if (hc[ax] - r > 0) bound = fmin(bound, (double)pp[ax] - (gi.lo[ax] + (hc[ax] - r) * h));
                if (hc[ax] + r < gi.dim[ax] - 1) bound = fmin(bound, (gi.lo[ax] + (hc[ax] + r + 1) * h) - pp[ax]);
            }
            bound -= margin;
            if (bound > 0 && bd[K - 1] < bound * bound) break;
            if (bound >= 1e299) break;   // the whole grid has been visited
        }
    }
    for (int k = 0; k < K; ++k) a.nbr[g * KMAX + k] = bi[k];
    a.ncnt[g] = (uint8_t)K;
}

__global__ void __launch_bounds__(128) k_reg_filter(RegArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N || a.cls[g] != CLS_SOURCE) return;
    const int K = a.ncnt[g];
    uint32_t nb[KMAX];
    for (int k = 0; k < K; ++k) nb[k] = a.nbr[g * KMAX + k];
    for (int c = 0; c < 9; ++c) {
        float v[KMAX];
        for (int k = 0; k < K; ++k) v[k] = a.delta[(int64_t)nb[k] * 9 + c];
        for (int i = 1; i < K; ++i) {   // insertion sort
            const float x = v[i];
            int j = i;
            while (j > 0 && v[j - 1] > x) {
                v[j] = v[j - 1];
                --j;
            }
            v[j] = x;
        }
        a.filt[g * 9 + c] = (K & 1) ? v[K / 2] : (float)(0.5 * ((double)v[K / 2 - 1] + (double)v[K / 2]));
    }
}

__global__ void __launch_bounds__(128) k_reg_apply(RegArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N) return;
    const uint8_t cl = a.cls[g];
    const int K = a.ncnt[g];
    double d[9];
    uint32_t flag = 0;
    if (cl == CLS_STATIC) {
        flag = 1;
    } else if (cl == CLS_SOURCE && K > 0) {
        for (int c = 0; c < 9; ++c) d[c] = a.filt[g * 9 + c];
        flag = 2;
    } else if (cl == CLS_TARGET && K > 0) {
        for (int c = 0; c < 9; ++c) d[c] = 0.0;
        for (int k = 0; k < K; ++k) {
            const int64_t nbk = a.nbr[g * KMAX + k];
            for (int c = 0; c < 9; ++c) d[c] += a.filt[nbk * 9 + c];
        }
        for (int c = 0; c < 9; ++c) d[c] /= K;
        flag = 4;
    }
    a.reg[g] = flag;
    if (flag == 2 || flag == 4) {
        for (int i = 0; i < 3; ++i) a.mo[3 * g + i] = (float)((double)a.m0[3 * g + i] + d[i]);
        double Q[9], R0[9], R[9], q[4];
        rot_zyx(d[3], d[4], d[5], Q);
        quat_rot64(a.q0 + 4 * g, R0);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                R[i * 3 + j] = Q[i * 3] * R0[j] + Q[i * 3 + 1] * R0[3 + j] + Q[i * 3 + 2] * R0[6 + j];
        rot_quat(R, q);
        for (int i = 0; i < 4; ++i) a.qo[4 * g + i] = (float)q[i];
        for (int i = 0; i < 3; ++i) {
            const double s = (double)a.s0[3 * g + i] + d[6 + i];
            a.so[3 * g + i] = s > 0 ? (float)s : a.s0[3 * g + i];
        }
    } else {
        for (int i = 0; i < 3; ++i) a.mo[3 * g + i] = a.m0[3 * g + i];
        for (int i = 0; i < 4; ++i) a.qo[4 * g + i] = a.q0[4 * g + i];
        for (int i = 0; i < 3; ++i) a.so[3 * g + i] = a.s0[3 * g + i];
    }
}

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct RegLayout {
    size_t cls, delta, filt, nbr, ncnt, keys, ka, va, kb, vb, kf, vf, ranges, spos, grid, sort, total;
};

RegLayout reg_layout(int64_t N) {
    RegLayout L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t at = o; o += al256(b); return at; };
    L.cls = take((size_t)N);
    L.delta = take((size_t)N * 9 * 4);
    L.filt = take((size_t)N * 9 * 4);
    L.nbr = take((size_t)N * KMAX * 4);
    L.ncnt = take((size_t)N);
    L.keys = take((size_t)N * 4);
    L.ka = take((size_t)N * 4);
    L.va = take((size_t)N * 4);
    L.kb = take((size_t)N * 4);
    L.vb = take((size_t)N * 4);
    L.kf = take((size_t)N * 4);
    L.vf = take((size_t)N * 4);
    L.ranges = take((size_t)CELL_MAX * 8);
    L.spos = take((size_t)N * 16);
    L.grid = take(sizeof(GridInfo));
    L.sort = take(tg_sort_scratch_bytes(N, 1));
    L.total = o;
    return L;
}

}  // namespace

extern "C" tg_status tg_regularize(const tg_gaussians* g_ref, const tg_gaussians* g_upd, const uint32_t* status,
                                   const float* acc, int64_t N, int32_t V, const tg_params* p, void* ws,
                                   size_t* ws_bytes, tg_gaussians* g_out, uint32_t* reg_status, void* stream)
{
    if (!p || !ws_bytes || N < 0 || V < 1) return TG_ERR_INVALID_ARG;
    if (N > (int64_t)0x7FFFFFFF) return TG_ERR_UNSUPPORTED;
    const RegLayout L = reg_layout(N > 0 ? N : 1);
    if (!ws) {
        *ws_bytes = L.total;
        return TG_OK;
    }
    if (*ws_bytes < L.total) return TG_ERR_WORKSPACE;
    if (!g_ref || !g_upd || !status || !acc || !g_out || !reg_status) return TG_ERR_INVALID_ARG;
    if (!g_ref->means || !g_ref->quats || !g_ref->scales || !g_upd->means || !g_upd->quats || !g_upd->scales ||
        !g_out->means || !g_out->quats || !g_out->scales)
        return TG_ERR_INVALID_ARG;
    if (g_ref->scale_mode != 0 || g_upd->scale_mode != 0 || g_out->scale_mode != 0) return TG_ERR_UNSUPPORTED;
    if (p->reg_k < 1 || p->reg_k > KMAX) return TG_ERR_INVALID_ARG;
    if (N == 0) return TG_OK;
    char* w = (char*)ws;
    RegArgs a;
    a.m0 = g_ref->means;
    a.q0 = g_ref->quats;
    a.s0 = g_ref->scales;
    a.m1 = g_upd->means;
    a.q1 = g_upd->quats;
    a.s1 = g_upd->scales;
    a.status = status;
    a.acc = acc;
    a.mo = g_out->means;
    a.qo = g_out->quats;
    a.so = g_out->scales;
    a.reg = reg_status;
    a.N = N;
    a.V = V;
    a.K = p->reg_k;
    a.static_min_pix = p->static_min_pix;
    a.static_views = p->static_views;
    a.static_frac = p->static_frac;
    a.cls = (uint8_t*)(w + L.cls);
    a.delta = (float*)(w + L.delta);
    a.filt = (float*)(w + L.filt);
    a.nbr = (uint32_t*)(w + L.nbr);
    a.ncnt = (uint8_t*)(w + L.ncnt);
    a.keys = (uint32_t*)(w + L.keys);
    a.skeys = (const uint32_t*)(w + L.kf);
    a.svals = (const uint32_t*)(w + L.vf);
    a.ranges = (uint2*)(w + L.ranges);
    a.spos = (float4*)(w + L.spos);
    a.grid = (GridInfo*)(w + L.grid);
    hipStream_t s = (hipStream_t)stream;
    const unsigned b256 = (unsigned)((N + 255) / 256), b128 = (unsigned)((N + 127) / 128);
    hipLaunchKernelGGL(k_reg_init, dim3(1), dim3(1), 0, s, a.grid);
    hipLaunchKernelGGL(k_reg_classify, dim3(b256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reg_grid, dim3(1), dim3(1), 0, s, a.grid);
    hipLaunchKernelGGL(k_reg_keys, dim3(b256), dim3(256), 0, s, a);
    TG_CHECK_LAUNCH();
    tg_status st = tg_radix_sort(a.keys, nullptr, (uint32_t*)(w + L.ka), (uint32_t*)(w + L.va),
                                 (uint32_t*)(w + L.kb), (uint32_t*)(w + L.vb), (uint32_t*)(w + L.kf),
                                 (uint32_t*)(w + L.vf), N, 1, nullptr, 0, SORT_PASSES, w + L.sort, s);
    if (st != TG_OK) return st;
    hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)((CELL_MAX + 255) / 256)), dim3(256), 0, s, a.ranges,
                       (int64_t)CELL_MAX);
    hipLaunchKernelGGL(k_reg_cells, dim3(b256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_reg_knn, dim3(b128), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_reg_filter, dim3(b128), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_reg_apply, dim3(b128), dim3(128), 0, s, a);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
