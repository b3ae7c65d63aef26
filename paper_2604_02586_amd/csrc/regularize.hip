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
//   k_reg_knn       per non-static Gaussian: exact K nearest solved Gaussians
//                   by a best-first descent of the implicit octree formed by
//                   the levels (FP64 distances, ties by index, boxes farther
//                   than the current K-th neighbour pruned), so queries far
//                   from every solved Gaussian (the occluded interior of a
//                   scene, say) cost about as much as queries among them.
//   k_reg_filter    per solved Gaussian: component-wise median of its
//                   neighbours' changes (itself included).
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

// Morton code -> one coordinate (every third bit)
__device__ __forceinline__ uint32_t compact1by2(uint32_t x) {
    x &= 0x9249249u;
    x = (x ^ (x >> 2)) & 0x30c30c3u;
    x = (x ^ (x >> 4)) & 0x300f00fu;
    x = (x ^ (x >> 8)) & 0x30000ffu;
    x = (x ^ (x >> 16)) & 0x3ffu;
    return x;
}

// squared distance from p to the box of cell `code` at level L (FP64)
__device__ __forceinline__ double box_dist2(const GridInfo& gi, int L, uint32_t code, const double p[3]) {
    const double hL = gi.h * (double)(1 << L);
    const uint32_t c[3] = {compact1by2(code), compact1by2(code >> 1), compact1by2(code >> 2)};
    double d2 = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double lo = (double)gi.lo[ax] + c[ax] * hL, hi = lo + hL;
        const double d = p[ax] < lo ? lo - p[ax] : (p[ax] > hi ? p[ax] - hi : 0.0);
        d2 += d * d;
    }
    return d2;
}

constexpr int KNN_THREADS = 128;
constexpr int STACK = 64;      // >= 1 + 7 B entries for B <= 7
constexpr uint32_t LEAF = 16;  // scan a cell's points directly at or below this count

__global__ void __launch_bounds__(KNN_THREADS) k_reg_knn(RegArgs a) {
    // Best-first descent of the implicit octree (cells of every level are
    // Morton runs): a node is skipped when its box is farther than the
    // current K-th neighbour, children are visited nearest first.  Boxes are
    // widened by a margin because cells were assigned in FP32.
    __shared__ uint32_t stk[KNN_THREADS * STACK];
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
    const double p[3] = {a.m0[3 * g], a.m0[3 * g + 1], a.m0[3 * g + 2]};
    const double margin = 1e-3 * gi.h;
    uint32_t* st = stk + threadIdx.x * STACK;
    double bd[KMAX];
    uint32_t bi[KMAX];
    int cnt = 0;
    int sp = 0;
    st[sp++] = ((uint32_t)gi.B << 24);
    while (sp > 0) {
        const uint32_t node = st[--sp];
        const int L = (int)(node >> 24);
        const uint32_t code = node & 0xFFFFFFu;
        const uint2 rg = a.ranges[gi.lvl_off[L] + code];
        if (rg.y <= rg.x) continue;
        if (cnt == K) {
            const double dn = sqrt(box_dist2(gi, L, code, p)) - margin;
            if (dn > 0.0 && dn * dn > bd[K - 1]) continue;
        }
        if (L == 0 || rg.y - rg.x <= LEAF) {
            for (uint32_t i = rg.x; i < rg.y; ++i) {
                const float4 q = a.spos[i];
                const double dx = (double)q.x - p[0], dy = (double)q.y - p[1], dz = (double)q.z - p[2];
                topk_insert(bd, bi, cnt, K, dx * dx + dy * dy + dz * dz, __builtin_bit_cast(uint32_t, q.w));
            }
            continue;
        }
        // children, pushed farthest first so the nearest is visited next
        double cd[8];
        uint32_t cc[8];
        int nc = 0;
        const uint2* rc = a.ranges + gi.lvl_off[L - 1];
        for (uint32_t k = 0; k < 8; ++k) {
            const uint32_t ch = (code << 3) | k;
            const uint2 r2 = rc[ch];
            if (r2.y <= r2.x) continue;
            const double d2 = box_dist2(gi, L - 1, ch, p);
            int j = nc++;
            while (j > 0 && cd[j - 1] < d2) {   // descending by distance
                cd[j] = cd[j - 1];
                cc[j] = cc[j - 1];
                --j;
            }
            cd[j] = d2;
            cc[j] = ch;
        }
        for (int k = 0; k < nc && sp < STACK; ++k) st[sp++] = ((uint32_t)(L - 1) << 24) | cc[k];
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
    hipLaunchKernelGGL(k_reg_knn, dim3(b128), dim3(KNN_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_reg_filter, dim3(b128), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_reg_apply, dim3(b128), dim3(128), 0, s, a);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
