// tg_regularize: motion regularisation after the multi-view update
// (TrackerSplat Sec. 4.5; K = 8 neighbours, Sec. 5.2).
//
//   k_reg_classify  per Gaussian: static test over the views' pixel counts
//                   (Sec. 4.5.2), solved = position and covariance updated
//                   and not static; the change against the first frame
//                   (d_mu, Euler angles of R' R^T, d_S) of every solved
//                   Gaussian; bounding box and count of the solved set.
//   k_reg_grid      one thread: a cubic grid of 2^B cells per axis over the
//                   solved set (about two solved Gaussians per finest cell,
//                   B <= 7), seen at levels L = 0..B (cells of 2^L finest
//                   cells per axis).
//   k_reg_keys + radix sort + k_reg_cells
//                   solved Gaussians sorted by the Morton code of their finest
//                   cell, so every cell of every level is one contiguous run;
//                   per-level cell ranges and the sorted positions as float4.
//   k_reg_qkeys + radix sort, k_reg_wkeys + radix sort
//                   the queries (all non-static Gaussians) in Morton order of
//                   their grid cell, so a wave's queries are neighbours; the
//                   waves with queries far from every solved Gaussian (the
//                   longest searches) launched first.
//   k_reg_knn       per non-static Gaussian: exact K nearest solved Gaussians
//                   (FP64 distances, ties by index); a wave answers 64
//                   neighbouring queries with one best-first descent of the
//                   implicit octree formed by the levels, pruning boxes
//                   farther from the queries' bounding box than the wave's
//                   largest current K-th neighbour distance, so queries far
//                   from every solved Gaussian (the occluded interior of a
//                   scene, say) share one traversal instead of diverging;
//                   leaf points screened on the matrix cores (|c'|^2 -
//                   2 c'.q' by FP32 MFMA against a conservative bound),
//                   the few candidates tested exactly in FP64.
//   k_reg_filter    per solved Gaussian (in Morton order): component-wise
//                   median of its neighbours' changes (itself included).
//   k_reg_apply     per Gaussian: static -> first frame; solved -> first
//                   frame + filtered change; other -> first frame + mean of
//                   the neighbours' filtered changes.
#include "tg_internal.h"

namespace {

constexpr int KMAX = TG_REG_K_MAX;
constexpr int BMAX = 7;                   // finest grid: up to 128^3 cells
constexpr uint32_t KEY_NONE = 1u << (3 * BMAX);   // non-solved: sorts after every cell
constexpr int SORT_PASSES = 3;            // 22 key bits
// cell ranges of all levels for B = BMAX: sum of 8^(BMAX - L), L = 0..BMAX
constexpr uint64_t RANGES_MAX = ((1ull << (3 * (BMAX + 1))) - 1) / 7;

enum : uint8_t { CLS_STATIC = 0, CLS_SOURCE = 1, CLS_TARGET = 2 };

struct GridInfo {
    float lo[3];
    float inv_h;
    double h;                 // finest cell size
    int32_t B;                // 2^B finest cells per axis
    uint32_t n_src;
    int32_t box[6];           // order-preserving integer images of min xyz, max xyz
    uint32_t lvl_off[BMAX + 2];   // first range entry of each level
};

// 10-bit coordinate -> every third bit (Morton interleave)
__device__ __forceinline__ uint32_t part1by2(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x30000ffu;
    x = (x | (x << 8)) & 0x300f00fu;
    x = (x | (x << 4)) & 0x30c30c3u;
    x = (x | (x << 2)) & 0x9249249u;
    return x;
}
__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

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
    uint2* ranges;     // [RANGES_MAX] cell ranges of every level
    const uint32_t* qorder;  // [N] Gaussians in the neighbour search's order
    const uint32_t* worder;  // [ceil(N / 64)] groups of 64 queries in launch order
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
        // The pixel counts of each record (slots 12 and 13, one 8-byte load),
        // eight views' loads issued together (views past V load the last
        // view's record again, unused) before the tests, which take both
        // comparisons without short-circuit so no load waits on another.
        const uint32_t st = a.status[g];   // in flight with the counts
        int sv = 0;
        for (int v0 = 0; v0 < a.V; v0 += 8) {
            float2 r[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int v = v0 + j < a.V ? v0 + j : a.V - 1;
                r[j] = *(const float2*)(a.acc + ((int64_t)v * a.N + g) * TG_ACC_STRIDE + 12);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double n = r[j].x, sn = r[j].y;
                const bool is_static = (n > (double)a.static_min_pix) & (sn > a.static_frac * n);
                sv += (v0 + j < a.V && is_static) ? 1 : 0;
            }
        }
        const bool stat = sv >= a.static_views;
        const bool src = !stat && (st & 1u) && (st & 2u);
        if (src) {
            // every input loaded before the first store (the change array
            // may alias them, and a store between loads would serialise them)
            float q0v[4], q1v[4], m0v[3], m1v[3], s0v[3], s1v[3];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                q0v[i] = a.q0[4 * g + i];
                q1v[i] = a.q1[4 * g + i];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                m0v[i] = a.m0[3 * g + i];
                m1v[i] = a.m1[3 * g + i];
                s0v[i] = a.s0[3 * g + i];
                s1v[i] = a.s1[3 * g + i];
            }
            double R0[9], R1[9], Q[9];
            quat_rot64(q0v, R0);
            quat_rot64(q1v, R1);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    Q[i * 3 + j] = R1[i * 3] * R0[j * 3] + R1[i * 3 + 1] * R0[j * 3 + 1] + R1[i * 3 + 2] * R0[j * 3 + 2];
            float* d = a.delta + g * 9;
            for (int i = 0; i < 3; ++i) d[i] = (float)((double)m1v[i] - (double)m0v[i]);
            d[3] = (float)atan2(Q[7], Q[8]);
            d[4] = (float)asin(fmin(1.0, fmax(-1.0, -Q[6])));
            d[5] = (float)atan2(Q[3], Q[0]);
            for (int i = 0; i < 3; ++i) d[6 + i] = (float)((double)s1v[i] - (double)s0v[i]);
            for (int i = 0; i < 3; ++i) {
                const int32_t o = f2o(m0v[i]);
                atomicMin(&bmin[i], o);
                atomicMax(&bmax[i], o);
            }
            atomicAdd(&bcnt, 1u);
        }
        a.cls[g] = stat ? CLS_STATIC : (src ? CLS_SOURCE : CLS_TARGET);
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
    double lo[3], ext = 1e-6;
    for (int i = 0; i < 3; ++i) {
        lo[i] = gi->n_src ? (double)o2f(gi->box[i]) : 0.0;
        if (gi->n_src) ext = fmax(ext, (double)o2f(gi->box[3 + i]) - lo[i]);
    }
    // about two solved Gaussians per finest cell
    int B = 0;
    while (B < BMAX && (double)(1ull << (3 * B)) * 2.0 < (double)gi->n_src) ++B;
    const double h = ext / (double)(1 << B) * (1.0 + 1e-6);
    for (int i = 0; i < 3; ++i) gi->lo[i] = (float)lo[i];
    gi->h = h;
    gi->inv_h = (float)(1.0 / h);
    gi->B = B;
    uint32_t off = 0;
    for (int L = 0; L <= B; ++L) {
        gi->lvl_off[L] = off;
        off += 1u << (3 * (B - L));
    }
    gi->lvl_off[B + 1] = off;
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
        const int dim = 1 << gi.B;
        const int cx = cell_coord(a.m0[3 * g], gi.lo[0], gi.inv_h, dim);
        const int cy = cell_coord(a.m0[3 * g + 1], gi.lo[1], gi.inv_h, dim);
        const int cz = cell_coord(a.m0[3 * g + 2], gi.lo[2], gi.inv_h, dim);
        key = morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
    }
    a.keys[g] = key;
}

// Query order for the neighbour search: every non-static Gaussian by the
// Morton code of the finest cell it falls in (clamped to the grid), so the
// 64 queries of a wave are spatial neighbours and walk the same octree nodes.
// Static Gaussians sort last.
__global__ void __launch_bounds__(256) k_reg_qkeys(RegArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.N) return;
    uint32_t key = KEY_NONE;
    const GridInfo& gi = *a.grid;
    if (a.cls[g] != CLS_STATIC && gi.n_src > 0) {
        const int dim = 1 << gi.B;
        const int cx = cell_coord(a.m0[3 * g], gi.lo[0], gi.inv_h, dim);
        const int cy = cell_coord(a.m0[3 * g + 1], gi.lo[1], gi.inv_h, dim);
        const int cz = cell_coord(a.m0[3 * g + 2], gi.lo[2], gi.inv_h, dim);
        key = morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
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
    const GridInfo& gi = *a.grid;
    const uint32_t prev = i > 0 ? a.skeys[i - 1] : KEY_NONE;
    const uint32_t next = i + 1 < a.N ? a.skeys[i + 1] : KEY_NONE;
    for (int L = 0; L <= gi.B; ++L) {
        const uint32_t c = key >> (3 * L);
        if (prev >= KEY_NONE || (prev >> (3 * L)) != c) a.ranges[gi.lvl_off[L] + c].x = (uint32_t)i;
        if (next >= KEY_NONE || (next >> (3 * L)) != c) a.ranges[gi.lvl_off[L] + c].y = (uint32_t)(i + 1);
    }
    a.spos[i] = make_float4(a.m0[3 * g], a.m0[3 * g + 1], a.m0[3 * g + 2], __builtin_bit_cast(float, g));
}

// Morton code -> one coordinate (every third bit)
__device__ __forceinline__ uint32_t compact1by2(uint32_t x) {
    x &= 0x9249249u;
    x = (x ^ (x >> 2)) & 0x30c30c3u;
    x = (x ^ (x >> 4)) & 0x300f00fu;
    x = (x ^ (x >> 8)) & 0x30000ffu;
    x = (x ^ (x >> 16)) & 0x3ffu;
    return x;
}

// squared distance between the box of cell `code` at level L (finest cells
// of size h from the corner lo) and the box [qlo, qhi] (FP64)
__device__ __forceinline__ double box_box_dist2(const double lo[3], double h, int L, uint32_t code,
                                                const double qlo[3], const double qhi[3]) {
    const double hL = h * (double)(1 << L);
    const uint32_t c[3] = {compact1by2(code), compact1by2(code >> 1), compact1by2(code >> 2)};
    double d2 = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double blo = lo[ax] + c[ax] * hL, bhi = blo + hL;
        const double d = fmax(0.0, fmax(blo - qhi[ax], qlo[ax] - bhi));
        d2 += d * d;
    }
    return d2;
}

// (d, i) before (e, j): by distance, ties by index
__device__ __forceinline__ bool nb_before(double d, uint32_t i, double e, uint32_t j) {
    return d < e || (d == e && i < j);
}

// sorted insert into the KMAX best (d, i) so far; fully unrolled, so the
// lists stay in registers
__device__ __forceinline__ void nb_insert(double (&bd)[KMAX], uint32_t (&bi)[KMAX], double d, uint32_t id) {
#pragma unroll
    for (int k = KMAX - 1; k >= 0; --k) {
        const bool here = nb_before(d, id, bd[k], bi[k]);
        const bool prev = k > 0 && nb_before(d, id, bd[k > 0 ? k - 1 : 0], bi[k > 0 ? k - 1 : 0]);
        if (here) {
            bd[k] = prev ? bd[k > 0 ? k - 1 : 0] : d;
            bi[k] = prev ? bi[k > 0 ? k - 1 : 0] : id;
        }
    }
}

__device__ __forceinline__ double bcast_f64(double x, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// largest value over the wave (DPP: prefix max within rows of 16, then the
// row maxima carried by row broadcasts to lane 63)
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x111, 0xf, 0xf, false));   // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x112, 0xf, 0xf, false));   // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x114, 0xf, 0xf, false));   // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x118, 0xf, 0xf, false));   // row_shr:8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x142, 0xa, 0xf, false));   // row_bcast:15
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// an FP32 value at least x >= 0
__device__ __forceinline__ float f32_up(double x) {
    const float f = (float)x;
    // below x: f is finite and non-negative, the next FP32 value is one up in its bits
    return (double)f < x ? __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u) : f;
}

__device__ __forceinline__ float wave_min_f32(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}

// FP32 screen of a squared distance against the K-th (FP64) wd: the FP32
// value of dx^2 + dy^2 + dz^2 from FP32 differences is within 5 units of
// 2^-24 (relative) of the exact one, plus a few units of 2^-149 where
// values are subnormal, so a point whose FP64 distance is at most wd has an
// FP32 distance at most wd (1 + 2^-18) rounded to FP32, plus 2^-126.
__device__ __forceinline__ float screen_bound(double wd) {
    return (float)(wd * (1.0 + 0x1p-18)) + 0x1p-126f;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// padding of a leaf chunk: infinitely far, index above every Gaussian's
constexpr uint32_t PAD_ID_U = 0xFFFFFFFFu;
#define PAD_ID __builtin_bit_cast(float, PAD_ID_U)

// first range entry of level L for 2^B finest cells per axis: the levels
// below hold 8^B + 8^(B-1) + ... + 8^(B-L+1) cells
__device__ __forceinline__ uint32_t level_offset(int B, int L) {
    return ((1u << (3 * (B + 1))) - (1u << (3 * (B + 1 - L)))) / 7u;
}

// Launch order of the neighbour search's waves (groups of 64 consecutive
// queries): by the level of the smallest cell around a query that holds K
// solved Gaussians, the largest over the group, largest first (stable).
// Queries far from every solved Gaussian have the longest searches; starting
// their waves first keeps them off the end of the launch.  One wave per group.
__global__ void __launch_bounds__(256) k_reg_wkeys(RegArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (((i >> 6) << 6) >= a.N) return;   // wave-uniform
    const GridInfo& gi = *a.grid;
    const uint32_t K = (uint32_t)a.K < gi.n_src ? (uint32_t)a.K : gi.n_src;
    uint32_t level = 0;   // deepest level + 1, 0 for no query
    if (i < a.N && K > 0) {
        const int64_t g = a.qorder[i];
        if (a.cls[g] != CLS_STATIC) {
            const int dim = 1 << gi.B;
            const int cx = cell_coord(a.m0[3 * g], gi.lo[0], gi.inv_h, dim);
            const int cy = cell_coord(a.m0[3 * g + 1], gi.lo[1], gi.inv_h, dim);
            const int cz = cell_coord(a.m0[3 * g + 2], gi.lo[2], gi.inv_h, dim);
            const uint32_t code = morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
            int L = 0;
            for (; L < gi.B; ++L) {
                const uint2 r = a.ranges[gi.lvl_off[L] + (code >> (3 * L))];
                if (r.y - r.x >= K) break;
            }
            level = (uint32_t)L + 1u;
        }
    }
    level = wave_max_u32(level);
    if ((threadIdx.x & 63) == 0) a.keys[i >> 6] = level == 0 ? 0xFFu : (uint32_t)(BMAX + 1) - level;
}

constexpr int KNN_WAVES = 4;   // independent waves per block
constexpr int STACK = 64;      // a descent of BMAX levels leaves at most 1 + 7 BMAX nodes
static_assert(STACK >= 1 + 7 * BMAX, "neighbour-search stack too small");
constexpr uint32_t LEAF = 256; // scan a cell's points directly at or below this count
constexpr int HEAVY_NODES = 64;   // a wave past this many nodes raises its issue priority
constexpr int SCREEN = 4;      // points screened together on the exact pass (divides 64)

__global__ void __launch_bounds__(64 * KNN_WAVES) __attribute__((amdgpu_waves_per_eu(4, 8))) k_reg_knn(RegArgs a) {
    // One wave answers 64 consecutive queries of the Morton order (spatial
    // neighbours) with one shared best-first descent of the implicit octree
    // (cells of every level are Morton runs): a node is skipped when its box
    // is farther from the queries' bounding box than the largest current
    // K-th neighbour distance of the wave, children are visited nearest
    // first, and every point of a visited leaf is offered to every lane
    // (an MFMA screen, then a per-lane FP32 screen, then the FP64 test).
    // The skipped points are farther than each lane's K-th neighbour and the
    // screens never reject a point the FP64 test would take, so every lane's
    // result is its exact K nearest.  Boxes are widened by a margin because
    // cells were assigned in FP32.
    __shared__ uint4 stk_all[KNN_WAVES][STACK];
    __shared__ float4 pts_all[KNN_WAVES][64];    // a leaf chunk: positions and indices
    __shared__ float4 rel_all[KNN_WAVES][64];    // the same relative to o, and |c - o|^2
    __shared__ float thr_all[KNN_WAVES][64];     // each query's screen threshold
    const uint32_t lane = threadIdx.x & 63;
    uint4* stk = stk_all[threadIdx.x >> 6];
    float4* pts = pts_all[threadIdx.x >> 6];
    float4* rel = rel_all[threadIdx.x >> 6];
    float* thr_l = thr_all[threadIdx.x >> 6];
    const int64_t wave = (int64_t)blockIdx.x * KNN_WAVES + (threadIdx.x >> 6);
    if (wave >= (a.N + 63) / 64) return;   // wave-uniform
    const int64_t qi = (int64_t)a.worder[wave] * 64 + lane;
    const GridInfo& gi = *a.grid;
    const int K = (int)((uint32_t)a.K < gi.n_src ? (uint32_t)a.K : gi.n_src);
    int64_t g = -1;
    if (qi < a.N) {
        g = a.qorder[qi];
        if (a.cls[g] == CLS_STATIC || K == 0) {
            a.ncnt[g] = 0;
            g = -1;
        }
    }
    const bool act = g >= 0;
    if (__ballot(act) == 0ull) return;   // wave-uniform
    double qlo[3], qhi[3];
    float pf[3];
    for (int ax = 0; ax < 3; ++ax) {
        const float x = act ? a.m0[3 * g + ax] : 0.0f;
        pf[ax] = x;
        qlo[ax] = wave_min_f32(act ? x : INFINITY);
        qhi[ax] = -wave_min_f32(act ? -x : INFINITY);
    }
    // grid in registers (the loop's wave barriers would reload it from memory)
    const double gh = gi.h, glo[3] = {gi.lo[0], gi.lo[1], gi.lo[2]};
    const double margin = 1e-3 * gh;
    // Matrix-core screen of a leaf chunk: with o the centre of the queries'
    // box, c' = c - o and q' = q - o in FP32, a 16x16x4 FP32 MFMA forms
    // |c'|^2 - 2 c'.q' for 16 points x 16 queries, i.e. |c - q|^2 - |q'|^2.
    // The FP32 roundings of c', q', |c'|^2 and the MFMA sums move this by
    // less than 2^-17 S^2 with S >= |c'| + |q'| (S from the grid's box and
    // the queries' box), so thr = wd (1 + 2^-18) - |q'|^2 + 2^-17 S^2
    // never rejects a point whose FP64 distance is at most wd.
    const float ofx = 0.5f * ((float)qlo[0] + (float)qhi[0]), ofy = 0.5f * ((float)qlo[1] + (float)qhi[1]),
                ofz = 0.5f * ((float)qlo[2] + (float)qhi[2]);
    double slack;
    {
        const double ext = gh * (double)(1 << gi.B);
        const double o3[3] = {ofx, ofy, ofz};
        double c2 = 0.0, q2 = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double c = fmax(fabs(glo[ax] - o3[ax]), fabs(glo[ax] + ext - o3[ax]));
            const double q = fmax(fabs(qlo[ax] - o3[ax]), fabs(qhi[ax] - o3[ax]));
            c2 += c * c;
            q2 += q * q;
        }
        const double S = (sqrt(c2) + sqrt(q2)) * (1.0 + 0x1p-20) + 1e-30;
        slack = 0x1p-17 * S * S;
    }
    const float qx = pf[0] - ofx, qy = pf[1] - ofy, qz = pf[2] - ofz;
    const double qq = (double)(qx * qx + qy * qy + qz * qz);
    auto screen_thr = [&](double w) {
        return act ? f32_up(w * (1.0 + 0x1p-18) - qq + slack) : -INFINITY;
    };
    // B operands (query columns): lane l holds component l / 16 of
    // (-2 q', 1) of query 16 qb + l % 16
    float bq[4];
    rel[lane] = act ? make_float4(-2.0f * qx, -2.0f * qy, -2.0f * qz, 1.0f) : make_float4(0.f, 0.f, 0.f, 1.0f);
    thr_l[lane] = screen_thr(INFINITY);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) bq[qb] = ((const float*)&rel[16 * qb + (lane & 15)])[lane >> 4];
    __builtin_amdgcn_wave_barrier();
    // every active lane's K-th neighbour distance^2 is at most R2 (wave-uniform);
    // pruned: a box at distance^2 d2 (to the queries' box) with d2 > Rm2 =
    // (sqrt(R2) + margin)^2, raised by 2^-40 for the rounding of this bound
    double Rm2 = INFINITY;
    auto pruned = [&](double d2) { return d2 > Rm2; };
    // the K best so far (the first K of KMAX sorted entries) and the K-th
    double bd[KMAX];
    uint32_t bi[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        bd[k] = INFINITY;
        bi[k] = 0xFFFFFFFFu;
    }
    double wd = INFINITY;
    uint32_t wi = 0xFFFFFFFFu;
    float wdf = INFINITY;
    // stack entries: node (level << 24 | Morton code), its point range and
    // its box distance^2 to the queries' box rounded toward zero
    const int B = gi.B;
    if (lane == 0) {
        const uint2 r0 = a.ranges[level_offset(B, B)];
        stk[0] = make_uint4((uint32_t)B << 24, r0.x, r0.y, 0u);
    }
    int sp = 1, visited = 0;
    auto is_leaf = [&](int L, uint2 r) { return L == 0 || r.y - r.x <= LEAF; };
    auto load_chunk = [&](uint32_t b, uint32_t end) {
        return lane < end - b ? a.spos[b + lane] : make_float4(INFINITY, INFINITY, INFINITY, PAD_ID);
    };
    // the first chunk of the leaf on top of the stack, loaded while the
    // previous leaf's last chunk is screened (pre_tag: that leaf's node,
    // wave-uniform)
    float4 pre = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t pre_tag = 0xFFFFFFFFu;
    auto prefetch_top = [&]() {
        if (sp == 0) return;
        const uint4 t = stk[sp - 1];
        const uint32_t tn = (uint32_t)__builtin_amdgcn_readfirstlane((int)t.x);
        const uint2 tr = make_uint2((uint32_t)__builtin_amdgcn_readfirstlane((int)t.y),
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)t.z));
        if (!is_leaf((int)(tn >> 24), tr)) return;
        pre = load_chunk(tr.x, tr.y - tr.x < 64u ? tr.y : tr.x + 64u);
        pre_tag = tn;
    };
    while (sp > 0) {
        __builtin_amdgcn_wave_barrier();
        const uint4 e = stk[--sp];
        const uint32_t node = (uint32_t)__builtin_amdgcn_readfirstlane((int)e.x);
        const uint2 rg = make_uint2((uint32_t)__builtin_amdgcn_readfirstlane((int)e.y),
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)e.z));
        if (pruned((double)__builtin_bit_cast(float, __builtin_amdgcn_readfirstlane((int)e.w)))) continue;
        const int L = (int)(node >> 24);
        const uint32_t code = node & 0xFFFFFFu;
        // the few long searches (queries far from every solved Gaussian) set
        // the launch's length: let them issue ahead of the short ones
        if (++visited == HEAVY_NODES) __builtin_amdgcn_s_setprio(2);
        if (is_leaf(L, rg)) {
            // per lane, against its own query and K-th neighbour (tighter
            // than the wave's bound): skip a leaf no lane can take a point from
            {
                const double pq[3] = {(double)pf[0], (double)pf[1], (double)pf[2]};
                const double r = sqrt(wd) + margin;
                const bool maybe = act && !(box_box_dist2(glo, gh, L, code, pq, pq) > r * r * (1.0 + 0x1p-40));
                if (__ballot(maybe) == 0ull) continue;
            }
            // the leaf's points in chunks of 64 through LDS, read back by
            // every lane SCREEN at a time (broadcast reads); an FP32 screen
            // (never below the FP64 distance, see wdf) sends the few points
            // that may enter a list to the exact FP64 test
            // (the next chunk, or the next leaf's first, is loaded while one
            // is screened)
            float4 cur = pre_tag == node ? pre : load_chunk(rg.x, rg.y - rg.x < 64u ? rg.y : rg.x + 64u);
            for (uint32_t b = rg.x; b < rg.y; b += 64) {
                const uint32_t m = rg.y - b < 64u ? rg.y - b : 64u;
                {
                    const float cx = cur.x - ofx, cy = cur.y - ofy, cz = cur.z - ofz;
                    pts[lane] = cur;
                    rel[lane] = lane < m ? make_float4(cx, cy, cz, cx * cx + cy * cy + cz * cz)
                                         : make_float4(0.f, 0.f, 0.f, INFINITY);
                }
                __builtin_amdgcn_wave_barrier();
                if (b + 64u < rg.y)
                    cur = load_chunk(b + 64u, rg.y - (b + 64u) < 64u ? rg.y : b + 128u);
                else
                    prefetch_top();
                // screen: rows = 16 points of block pb, columns = 16 queries of block qb
                float tq[4];
#pragma unroll
                for (int qb = 0; qb < 4; ++qb) tq[qb] = thr_l[16 * qb + (lane & 15)];
                uint32_t hit_blocks = 0;   // point blocks with a screen hit (wave-uniform)
                for (uint32_t pb = 0; pb < (m + 15) / 16; ++pb) {
                    const float av = ((const float*)&rel[16 * pb + (lane & 15)])[lane >> 4];
                    bool hit = false;
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb) {
                        const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bq[qb], f32x4{0.f, 0.f, 0.f, 0.f},
                                                                             0, 0, 0);
                        hit |= (d[0] <= tq[qb]) | (d[1] <= tq[qb]) | (d[2] <= tq[qb]) | (d[3] <= tq[qb]);
                    }
                    if (__ballot(hit) != 0ull) hit_blocks |= 1u << pb;
                }
                if (hit_blocks != 0u) {
                    // exact pass over the blocks with hits (per-lane FP32 screen, then FP64)
                    for (uint32_t t = 0; t < m; t += SCREEN) {
                        if (!((hit_blocks >> (t / 16)) & 1u)) continue;
                        bool h2 = false;
#pragma unroll
                        for (int u = 0; u < SCREEN; ++u) {
                            const float4 c = pts[t + u];
                            const float dx = c.x - pf[0], dy = c.y - pf[1], dz = c.z - pf[2];
                            h2 |= dx * dx + dy * dy + dz * dz <= wdf;
                        }
                        if (act && h2) {
#pragma unroll 1
                            for (int u = 0; u < SCREEN; ++u) {
                                const float4 cu = pts[t + u];
                                const double dx = (double)cu.x - (double)pf[0], dy = (double)cu.y - (double)pf[1],
                                             dz = (double)cu.z - (double)pf[2];
                                const double d2 = dx * dx + dy * dy + dz * dz;
                                const uint32_t id = __builtin_bit_cast(uint32_t, cu.w);
                                if (nb_before(d2, id, wd, wi)) {
                                    nb_insert(bd, bi, d2, id);
#pragma unroll
                                    for (int k = 0; k < KMAX; ++k)
                                        if (k == K - 1) {
                                            wd = bd[k];
                                            wi = bi[k];
                                        }
                                    wdf = screen_bound(wd);
                                }
                            }
                        }
                    }
                    thr_l[lane] = screen_thr(wd);
                }
                __builtin_amdgcn_wave_barrier();
            }
            // (non-negative FP32 values order as their bit patterns)
            const double R2 = (double)__builtin_bit_cast(
                float, wave_max_u32(__builtin_bit_cast(uint32_t, act ? f32_up(wd) : 0.0f)));
            if (R2 < INFINITY) {
                const double r = sqrt(R2) + margin;
                Rm2 = r * r * (1.0 + 0x1p-40);
            }
            continue;
        }
        // children on lanes 0..7, pushed farthest first so the nearest is
        // visited next (ties by child number)
        const uint2* rc = a.ranges + level_offset(B, L - 1);
        const uint32_t ch = (code << 3) | (lane & 7u);
        bool ok = false;
        double cd = INFINITY;
        uint2 r2 = make_uint2(0u, 0u);
        if (lane < 8) {
            r2 = rc[ch];
            if (r2.y > r2.x) {
                cd = box_box_dist2(glo, gh, L - 1, ch, qlo, qhi);
                ok = !pruned(cd);
            }
        }
        const uint64_t okm = __ballot(ok);
        const int nc = __popcll(okm);
        int rank = 0;
        for (int j = 0; j < 8; ++j) {
            const double dj = bcast_f64(cd, j);
            rank += (((okm >> j) & 1ull) && (dj < cd || (dj == cd && j < (int)lane))) ? 1 : 0;
        }
        if (ok)
            stk[sp + nc - 1 - rank] = make_uint4(((uint32_t)(L - 1) << 24) | ch, r2.x, r2.y,
                                                 __builtin_bit_cast(uint32_t, __double2float_rz(cd)));
        sp += nc;
    }
    if (act) {
        for (int k = 0; k < K; ++k) a.nbr[g * KMAX + k] = bi[k];
        a.ncnt[g] = (uint8_t)K;
    }
}

__global__ void __launch_bounds__(128) k_reg_filter(RegArgs a) {
    // one thread per solved Gaussian, in the Morton order of the sorted
    // positions (neighbouring threads gather neighbouring changes)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)a.grid->n_src) return;
    const int64_t g = __builtin_bit_cast(uint32_t, a.spos[i].w);
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
    // Every load before the first store (the outputs may alias the inputs,
    // so a store between loads would make each wait for the one before),
    // and a target's neighbour ids all loaded before their changes.
    const uint8_t cl = a.cls[g];
    const int K = a.ncnt[g];
    float m0v[3], q0v[4], s0v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) m0v[i] = a.m0[3 * g + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) q0v[i] = a.q0[4 * g + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) s0v[i] = a.s0[3 * g + i];
    double d[9];
    uint32_t flag = 0;
    if (cl == CLS_STATIC) {
        flag = 1;
    } else if (cl == CLS_SOURCE && K > 0) {
        for (int c = 0; c < 9; ++c) d[c] = a.filt[g * 9 + c];
        flag = 2;
    } else if (cl == CLS_TARGET && K > 0) {
        // unused slots (k >= K) gather Gaussian 0's changes, never added:
        // no load waits on a branch
        uint32_t nb[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t id = a.nbr[g * KMAX + k];
            nb[k] = k < K ? id : 0u;
        }
        float f[KMAX][9];
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
#pragma unroll
            for (int c = 0; c < 9; ++c) f[k][c] = a.filt[(int64_t)nb[k] * 9 + c];
        // the same summation order as one neighbour at a time
        for (int c = 0; c < 9; ++c) d[c] = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < K)
#pragma unroll
                for (int c = 0; c < 9; ++c) d[c] += f[k][c];
        for (int c = 0; c < 9; ++c) d[c] /= K;
        flag = 4;
    }
    a.reg[g] = flag;
    if (flag == 2 || flag == 4) {
        for (int i = 0; i < 3; ++i) a.mo[3 * g + i] = (float)((double)m0v[i] + d[i]);
        double Q[9], R0[9], R[9], q[4];
        rot_zyx(d[3], d[4], d[5], Q);
        quat_rot64(q0v, R0);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                R[i * 3 + j] = Q[i * 3] * R0[j] + Q[i * 3 + 1] * R0[3 + j] + Q[i * 3 + 2] * R0[6 + j];
        rot_quat(R, q);
        for (int i = 0; i < 4; ++i) a.qo[4 * g + i] = (float)q[i];
        for (int i = 0; i < 3; ++i) {
            const double s = (double)s0v[i] + d[6 + i];
            a.so[3 * g + i] = s > 0 ? (float)s : s0v[i];
        }
    } else {
        for (int i = 0; i < 3; ++i) a.mo[3 * g + i] = m0v[i];
        for (int i = 0; i < 4; ++i) a.qo[4 * g + i] = q0v[i];
        for (int i = 0; i < 3; ++i) a.so[3 * g + i] = s0v[i];
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
    L.ranges = take((size_t)RANGES_MAX * 8);
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
    a.qorder = nullptr;
    a.worder = nullptr;
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
    hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)((RANGES_MAX + 255) / 256)), dim3(256), 0, s, a.ranges,
                       (int64_t)RANGES_MAX);
    hipLaunchKernelGGL(k_reg_cells, dim3(b256), dim3(256), 0, s, a);
    // queries in Morton order (the sorted sources' buffers are free now:
    // the search reads the cell ranges and the sorted positions)
    hipLaunchKernelGGL(k_reg_qkeys, dim3(b256), dim3(256), 0, s, a);
    TG_CHECK_LAUNCH();
    st = tg_radix_sort(a.keys, nullptr, (uint32_t*)(w + L.ka), (uint32_t*)(w + L.va), (uint32_t*)(w + L.kb),
                       (uint32_t*)(w + L.vb), nullptr, (uint32_t*)(w + L.vf), N, 1, nullptr, 0, SORT_PASSES,
                       w + L.sort, s);
    if (st != TG_OK) return st;
    a.qorder = (const uint32_t*)(w + L.vf);
    const int64_t n_groups = (N + 63) / 64;
    hipLaunchKernelGGL(k_reg_wkeys, dim3(b256), dim3(256), 0, s, a);
    TG_CHECK_LAUNCH();
    st = tg_radix_sort(a.keys, nullptr, (uint32_t*)(w + L.ka), (uint32_t*)(w + L.va), (uint32_t*)(w + L.kb),
                       (uint32_t*)(w + L.vb), nullptr, (uint32_t*)(w + L.kf), n_groups, 1, nullptr, 0, 1,
                       w + L.sort, s);
    if (st != TG_OK) return st;
    a.worder = (const uint32_t*)(w + L.kf);
    hipLaunchKernelGGL(k_reg_knn, dim3((unsigned)((N + 64 * KNN_WAVES - 1) / (64 * KNN_WAVES))),
                       dim3(64 * KNN_WAVES), 0, s, a);
    hipLaunchKernelGGL(k_reg_filter, dim3(b128), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_reg_apply, dim3(b128), dim3(128), 0, s, a);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
