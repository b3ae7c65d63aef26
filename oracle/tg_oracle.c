/*
 * CPU oracle for TrackerSplat motion transfer -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path never links or calls it.
 *
 * Plain, slow, obviously-correct loops.  Floating point is FP64 except the
 * "geometry decisions" (splat centre, tile rectangle, depth key, culling),
 * which decide integers and are therefore taken in the renderer's own
 * precision (FP32, IEEE round-to-nearest, no contraction, fixed order).
 * Build flags: -O2 -ffp-contract=off -fno-fast-math (no FMA contraction).
 *
 * Paper references (TrackerSplat, SIGGRAPH Asia 2025):
 *   Sec. 3.1, Eq. 1      EWA projection of a 3D Gaussian
 *   Sec. 3.1 (end)       depth-ordered alpha blending
 *   Sec. 4.3.3, 4.3.4    incremental + weighted LS statistics, w = alpha*T (Eq. 4)
 *   Sec. 4.5.2           static-pixel count and alpha per Gaussian
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    float pad[2];
} ocam;

#define O_TILE 16
static const float O_NEAR = 0.2f;
static const float O_DIL = 0.3f;
static const float O_EXTENT = 3.0f;
static const float O_JCLAMP = 1.3f;
static const double O_ALPHA_MIN = 1.0 / 255.0;
static const double O_ALPHA_MAX = 0.99;
static const double O_T_MIN = 1e-4;

int orc_abi(void) { return 3; }

/* ------------------------------------------------------------------------
 * FP32 geometry decisions (Sec. 3.1, Eq. 1; renderer tile binning).
 * The exact operation order is part of the definition.
 * ---------------------------------------------------------------------- */
static void geom_one(const float* m, const float* q, const float* s, const ocam* c,
                     float* mu_out, int32_t* rect_out, uint32_t* key_out, uint8_t* valid_out)
{
    const float* R = c->R;
    float px = ((R[0] * m[0] + R[1] * m[1]) + R[2] * m[2]) + c->t[0];
    float py = ((R[3] * m[0] + R[4] * m[1]) + R[5] * m[2]) + c->t[1];
    float pz = ((R[6] * m[0] + R[7] * m[1]) + R[8] * m[2]) + c->t[2];
    mu_out[0] = 0.0f; mu_out[1] = 0.0f;
    rect_out[0] = rect_out[1] = rect_out[2] = rect_out[3] = 0;
    *valid_out = 0;
    uint32_t kb; memcpy(&kb, &pz, 4);
    *key_out = kb;
    if (!(pz > O_NEAR)) { *key_out = 0xFFFFFFFFu; return; }
    float ux = px / pz, uy = py / pz;
    float mx = c->fx * ux + c->cx;
    float my = c->fy * uy + c->cy;
    /* rotation from the (normalised) quaternion */
    float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    float inv = 1.0f / sqrtf(n2);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    float r[9];
    r[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
    r[1] = 2.0f * (qx * qy - qw * qz);
    r[2] = 2.0f * (qx * qz + qw * qy);
    r[3] = 2.0f * (qx * qy + qw * qz);
    r[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
    r[5] = 2.0f * (qy * qz - qw * qx);
    r[6] = 2.0f * (qx * qz - qw * qy);
    r[7] = 2.0f * (qy * qz + qw * qx);
    r[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
    float M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = r[i * 3 + j] * s[j];
    float S[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            S[i * 3 + j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
    float limx = O_JCLAMP * ((0.5f * (float)c->W) / c->fx);
    float limy = O_JCLAMP * ((0.5f * (float)c->H) / c->fy);
    float tx = fminf(limx, fmaxf(-limx, ux));
    float ty = fminf(limy, fmaxf(-limy, uy));
    float j00 = c->fx / pz, j02 = -(c->fx * tx) / pz;
    float j11 = c->fy / pz, j12 = -(c->fy * ty) / pz;
    float T0[3], T1[3];
    for (int j = 0; j < 3; ++j) {
        T0[j] = j00 * R[0 + j] + j02 * R[6 + j];
        T1[j] = j11 * R[3 + j] + j12 * R[6 + j];
    }
    float U0[3], U1[3];
    for (int j = 0; j < 3; ++j) {
        U0[j] = (T0[0] * S[0 + j] + T0[1] * S[3 + j]) + T0[2] * S[6 + j];
        U1[j] = (T1[0] * S[0 + j] + T1[1] * S[3 + j]) + T1[2] * S[6 + j];
    }
    float a = (U0[0] * T0[0] + U0[1] * T0[1]) + U0[2] * T0[2];
    float b = (U0[0] * T1[0] + U0[1] * T1[1]) + U0[2] * T1[2];
    float cc = (U1[0] * T1[0] + U1[1] * T1[1]) + U1[2] * T1[2];
    float ar = a + O_DIL, cr = cc + O_DIL;
    float det = ar * cr - b * b;
    if (!(det > 0.0f)) return;
    float mid = 0.5f * (ar + cr);
    float lmax = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
    float rad = ceilf(O_EXTENT * sqrtf(lmax));
    if (!isfinite(mx) || !isfinite(my) || !isfinite(rad)) return;
    int TX = (c->W + O_TILE - 1) / O_TILE, TY = (c->H + O_TILE - 1) / O_TILE;
    float fx0 = floorf((mx - rad) * 0.0625f);
    float fx1 = floorf((mx + rad) * 0.0625f) + 1.0f;
    float fy0 = floorf((my - rad) * 0.0625f);
    float fy1 = floorf((my + rad) * 0.0625f) + 1.0f;
    fx0 = fminf((float)TX, fmaxf(0.0f, fx0));
    fx1 = fminf((float)TX, fmaxf(0.0f, fx1));
    fy0 = fminf((float)TY, fmaxf(0.0f, fy0));
    fy1 = fminf((float)TY, fmaxf(0.0f, fy1));
    int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
    if (x0 >= x1 || y0 >= y1) return;
    mu_out[0] = mx; mu_out[1] = my;
    rect_out[0] = x0; rect_out[1] = y0; rect_out[2] = x1; rect_out[3] = y1;
    *valid_out = 1;
}

/* mu[V][N][2], rect[V][N][4], key[V][N], valid[V][N] */
void orc_geometry_f32(int64_t N, const float* means, const float* quats, const float* scales,
                      int32_t V, const ocam* cams, float* mu, int32_t* rect, uint32_t* key,
                      uint8_t* valid)
{
    for (int v = 0; v < V; ++v) {
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < N; ++g) {
            int64_t o = (int64_t)v * N + g;
            geom_one(means + 3 * g, quats + 4 * g, scales + 3 * g, cams + v,
                     mu + 2 * o, rect + 4 * o, key + o, valid + o);
        }
    }
}

/* ------------------------------------------------------------------------
 * FP64 projection (Sec. 3.1, Eq. 1): undilated Sigma_2D and the conic of the
 * dilated one.  cov[V][N][3] = (a, b, c); conic[V][N][3].
 * ---------------------------------------------------------------------- */
void orc_project_f64(int64_t N, const float* means, const float* quats, const float* scales,
                     int32_t V, const ocam* cams, double* cov, double* conic)
{
    for (int v = 0; v < V; ++v) {
        const ocam* c = cams + v;
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < N; ++g) {
            int64_t o = (int64_t)v * N + g;
            const float* m = means + 3 * g;
            const float* q = quats + 4 * g;
            const float* s = scales + 3 * g;
            double R[9];
            for (int i = 0; i < 9; ++i) R[i] = c->R[i];
            double p[3];
            for (int i = 0; i < 3; ++i)
                p[i] = R[3 * i] * m[0] + R[3 * i + 1] * m[1] + R[3 * i + 2] * m[2] + (double)c->t[i];
            double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
            double n = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            qw /= n; qx /= n; qy /= n; qz /= n;
            double r[9] = {
                1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
            double S[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double acc = 0;
                    for (int k = 0; k < 3; ++k) acc += r[3 * i + k] * r[3 * j + k] * (double)s[k] * (double)s[k];
                    S[3 * i + j] = acc;
                }
            double pz = p[2];
            double limx = 1.3 * (0.5 * c->W / (double)c->fx), limy = 1.3 * (0.5 * c->H / (double)c->fy);
            double tx = p[0] / pz, ty = p[1] / pz;
            if (tx > limx) tx = limx;
            if (tx < -limx) tx = -limx;
            if (ty > limy) ty = limy;
            if (ty < -limy) ty = -limy;
            double J[6] = {c->fx / pz, 0.0, -c->fx * tx / pz, 0.0, c->fy / pz, -c->fy * ty / pz};
            double T[6];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    T[3 * i + j] = J[3 * i] * R[j] + J[3 * i + 1] * R[3 + j] + J[3 * i + 2] * R[6 + j];
            double C2[4];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    double acc = 0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) acc += T[3 * i + k] * S[3 * k + l] * T[3 * j + l];
                    C2[2 * i + j] = acc;
                }
            cov[3 * o] = C2[0]; cov[3 * o + 1] = C2[1]; cov[3 * o + 2] = C2[3];
            double ar = C2[0] + 0.3, br = C2[1], cr = C2[3] + 0.3;
            double det = ar * cr - br * br;
            conic[3 * o] = cr / det; conic[3 * o + 1] = -br / det; conic[3 * o + 2] = ar / det;
        }
    }
}

/* ------------------------------------------------------------------------
 * Brute-force per-tile lists: for every tile of view v, the Gaussians whose
 * rectangle (in units of `cell` tiles) contains it, ordered by (depth key,
 * index).  cell = 1 gives the 16x16-pixel tile lists; cell = 2^k gives the
 * coarse lists of 2^k x 2^k tiles.  Output is CSR over all views:
 * starts[T_total+1] and ids[].  Returns the number of ids, or -1 if ids_cap
 * is too small (call with ids == NULL to count).
 *
 * The Gaussians of a view are first put in (depth key, index) order; walking
 * them in that order and appending each to every tile its rectangle covers
 * leaves every tile's list in that order.
 * ---------------------------------------------------------------------- */
static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void cell_dims(const ocam* c, int32_t cell, int* CX, int* CY)
{
    int TX = (c->W + O_TILE - 1) / O_TILE, TY = (c->H + O_TILE - 1) / O_TILE;
    *CX = (TX + cell - 1) / cell;
    *CY = (TY + cell - 1) / cell;
}

int64_t orc_tile_lists(int64_t N, int32_t V, const ocam* cams, const int32_t* rect,
                       const uint32_t* key, const uint8_t* valid, int32_t cell,
                       int64_t* starts, uint32_t* ids, int64_t ids_cap)
{
    int64_t* view_base = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V + 1));
    view_base[0] = 0;
    for (int v = 0; v < V; ++v) {
        int CX, CY;
        cell_dims(cams + v, cell, &CX, &CY);
        view_base[v + 1] = view_base[v] + (int64_t)CX * CY;
    }
    const int64_t total_cells = view_base[V];
    int64_t* cnt = (int64_t*)calloc((size_t)total_cells + 1, sizeof(int64_t));
    /* count: views own disjoint ranges of cells */
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < V; ++v) {
        int CX, CY;
        cell_dims(cams + v, cell, &CX, &CY);
        for (int64_t g = 0; g < N; ++g) {
            int64_t o = (int64_t)v * N + g;
            if (!valid[o]) continue;
            const int32_t* r = rect + 4 * o;
            int x0 = r[0] / cell, y0 = r[1] / cell, x1 = (r[2] - 1) / cell + 1, y1 = (r[3] - 1) / cell + 1;
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x) cnt[view_base[v] + (int64_t)y * CX + x]++;
        }
    }
    int64_t run = 0;
    for (int64_t i = 0; i < total_cells; ++i) { int64_t c = cnt[i]; cnt[i] = run; run += c; }
    cnt[total_cells] = run;
    if (starts) memcpy(starts, cnt, sizeof(int64_t) * (size_t)(total_cells + 1));
    if (!ids || run > ids_cap) {
        free(cnt);
        free(view_base);
        return ids ? -1 : run;
    }
    /* fill in (depth key, index) order */
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < V; ++v) {
        int CX, CY;
        cell_dims(cams + v, cell, &CX, &CY);
        uint64_t* ord = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N > 0 ? N : 1));
        int64_t n = 0;
        for (int64_t g = 0; g < N; ++g)
            if (valid[(int64_t)v * N + g]) ord[n++] = ((uint64_t)key[(int64_t)v * N + g] << 32) | (uint64_t)g;
        qsort(ord, (size_t)n, sizeof(uint64_t), cmp_u64);
        int64_t* fill = cnt + view_base[v];     /* this view's cells only */
        for (int64_t i = 0; i < n; ++i) {
            uint32_t g = (uint32_t)(ord[i] & 0xFFFFFFFFu);
            const int32_t* r = rect + 4 * ((int64_t)v * N + g);
            int x0 = r[0] / cell, y0 = r[1] / cell, x1 = (r[2] - 1) / cell + 1, y1 = (r[3] - 1) / cell + 1;
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x) ids[fill[(int64_t)y * CX + x]++] = g;
        }
        free(ord);
    }
    free(cnt);
    free(view_base);
    return run;
}

/* ------------------------------------------------------------------------
 * Depth-ordered compositing with PWI-LS statistics (Sec. 3.1, Sec. 4.3.3,
 * Sec. 4.3.4 Eq. 4, Sec. 4.5.2), FP64.
 *
 * For pixel x (row r, col c at (c, r)) of view v, walk the tile's list:
 *   power = -1/2 d^T conic d, d = x - mu (mu = the FP32 splat centre);
 *   skip if power > 0; alpha = min(0.99, o e^power); skip if alpha < 1/255;
 *   stop if T (1 - alpha) < 1e-4 (that Gaussian is excluded); w = alpha T;
 *   if the pixel's track is visible: accumulate, with u = x - mu and
 *   dd = x' - x, the 16-entry record
 *     [w, w ux, w uy, w ux ux, w ux uy, w uy uy, w ddx, w ddy,
 *      w ux ddx, w ux ddy, w uy ddx, w uy ddy, 1, static, static*alpha, 0]
 *   (static: |dd| < 1 px), and the paper-literal raw V1, V2 of Eq. 4
 *   (V1 = sum w [x;1][x;1]^T, V2 = sum w [x;1] x'^T), row-major 3x3 + 3x2;
 *   T <- T (1 - alpha).
 *
 * Besides the sums, for every entry it returns sum |term| (absm) and a
 * "slack" bound covering decisions within a relative band of their
 * thresholds (alpha ~ 1/255, T(1-alpha) ~ 1e-4), where an FP32 renderer may
 * legitimately decide the other way; nmarg counts such own decisions.
 * pixmask (nullable, [V][H][W]) restricts which pixels are composited.
 * ---------------------------------------------------------------------- */
#define O_BAND_TILES 4   /* tile rows per compositing task */

void orc_composite(int32_t V, const ocam* cams, int64_t N,
                   const float* mu, const double* conic, const float* opacity,
                   const int64_t* tstarts, const uint32_t* tids,
                   const float* disp, const uint8_t* vis, const uint8_t* pixmask,
                   double band_alpha, double band_t,
                   double* mom, double* absm, double* slack, int32_t* nmarg, double* raw,
                   double* tfinal, uint8_t* pixmarg, int64_t* counters)
{
    /* per-view pixel and tile offsets; tasks are bands of tile rows */
    int64_t* pix_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V + 1));
    int64_t* tile_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V + 1));
    int64_t ntask = 0;
    pix_off[0] = 0; tile_off[0] = 0;
    for (int v = 0; v < V; ++v) {
        int TX = (cams[v].W + O_TILE - 1) / O_TILE, TY = (cams[v].H + O_TILE - 1) / O_TILE;
        pix_off[v + 1] = pix_off[v] + (int64_t)cams[v].W * cams[v].H;
        tile_off[v + 1] = tile_off[v] + (int64_t)TX * TY;
        ntask += (TY + O_BAND_TILES - 1) / O_BAND_TILES;
    }
    int32_t* task_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ntask > 0 ? ntask : 1));
    int32_t* task_r0 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ntask > 0 ? ntask : 1));
    {
        int64_t t = 0;
        for (int v = 0; v < V; ++v) {
            int TY = (cams[v].H + O_TILE - 1) / O_TILE;
            for (int b = 0; b < TY; b += O_BAND_TILES) { task_v[t] = v; task_r0[t] = b * O_TILE; ++t; }
        }
    }
    if (counters) memset(counters, 0, sizeof(int64_t) * 2 * (size_t)V);
#pragma omp parallel
    {
        /* this thread's sums for the band it composites, dense over the
         * Gaussians; `touched` lists the entries written */
        double* lm = (double*)calloc((size_t)N * 16 + 1, sizeof(double));
        double* la = (double*)calloc((size_t)N * 16 + 1, sizeof(double));
        double* ls = (double*)calloc((size_t)N * 16 + 1, sizeof(double));
        double* lr = raw ? (double*)calloc((size_t)N * 15 + 1, sizeof(double)) : NULL;
        int32_t* ln = (int32_t*)calloc((size_t)N + 1, sizeof(int32_t));
        uint8_t* seen = (uint8_t*)calloc((size_t)N + 1, 1);
        uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N + 1));
#pragma omp for ordered schedule(dynamic, 1)
        for (int64_t task = 0; task < ntask; ++task) {
            const int v = task_v[task];
            const ocam* c = cams + v;
            const int W = c->W, H = c->H, TX = (W + O_TILE - 1) / O_TILE;
            const int r0 = task_r0[task];
            const int r1 = r0 + O_BAND_TILES * O_TILE < H ? r0 + O_BAND_TILES * O_TILE : H;
            int64_t ev = 0, ec = 0, nt = 0;
            for (int r = r0; r < r1; ++r)
                for (int col = 0; col < W; ++col) {
                    int64_t pi = pix_off[v] + (int64_t)r * W + col;
                    if (pixmask && !pixmask[pi]) continue;
                    int64_t tile = tile_off[v] + (int64_t)(r / O_TILE) * TX + col / O_TILE;
                    double x = col, y = r;
                    double ddx = disp[2 * pi], ddy = disp[2 * pi + 1];
                    int visible = vis ? vis[pi] != 0 : 1;
                    /* static pixel (Sec. 4.5.2): |x' - x| < 1 px, decided in the
                     * renderer's FP32 (it decides an integer count) */
                    float fdx = disp[2 * pi], fdy = disp[2 * pi + 1];
                    float s2 = fdx * fdx;
                    s2 = s2 + fdy * fdy;
                    int is_static = s2 < 1.0f;
                    double T = 1.0, taint = 0.0;
                    int marg = 0;
                    for (int64_t k = tstarts[tile]; k < tstarts[tile + 1]; ++k) {
                        uint32_t g = tids[k];
                        int64_t o = (int64_t)v * N + g;
                        double dx = x - (double)mu[2 * o], dy = y - (double)mu[2 * o + 1];
                        const double* cn = conic + 3 * o;
                        double power = -0.5 * (cn[0] * dx * dx + cn[2] * dy * dy) - cn[1] * dx * dy;
                        ++ev;
                        if (power > 0.0) continue;
                        double alpha = (double)opacity[g] * exp(power);
                        if (alpha > O_ALPHA_MAX) alpha = O_ALPHA_MAX;
                        int own_marg = 0;
                        if (fabs(alpha - O_ALPHA_MIN) <= band_alpha * O_ALPHA_MIN) own_marg = 1;
                        double test = T * (1.0 - alpha);
                        double tband = (band_t + 1.5 * taint) * O_T_MIN;
                        int term_marg = alpha >= O_ALPHA_MIN && fabs(test - O_T_MIN) <= tband;
                        double w = alpha * T;
                        double term[16];
                        term[0] = w; term[1] = w * dx; term[2] = w * dy;
                        term[3] = w * dx * dx; term[4] = w * dx * dy; term[5] = w * dy * dy;
                        term[6] = w * ddx; term[7] = w * ddy;
                        term[8] = w * dx * ddx; term[9] = w * dx * ddy;
                        term[10] = w * dy * ddx; term[11] = w * dy * ddy;
                        term[12] = 1.0; term[13] = is_static ? 1.0 : 0.0;
                        term[14] = is_static ? alpha : 0.0; term[15] = 0.0;
                        int writes = ((own_marg || term_marg) && visible) ||
                                     (alpha >= O_ALPHA_MIN && test >= O_T_MIN && visible);
                        if (writes && !seen[g]) { seen[g] = 1; touched[nt++] = g; }
                        if ((own_marg || term_marg) && visible) {
                            for (int i = 0; i < 15; ++i) ls[16 * (int64_t)g + i] += fabs(term[i]);
                            ln[g] += 1;
                        }
                        if (own_marg || term_marg) marg = 1;
                        if (alpha < O_ALPHA_MIN) {
                            if (own_marg) taint += alpha / (1.0 - alpha);
                            continue;
                        }
                        if (test < O_T_MIN) break;
                        ++ec;
                        if (visible) {
                            double* m = lm + 16 * (int64_t)g;
                            double* a = la + 16 * (int64_t)g;
                            for (int i = 0; i < 15; ++i) { m[i] += term[i]; a[i] += fabs(term[i]); }
                            if (taint > 0.0)
                                for (int i = 0; i < 12; ++i) ls[16 * (int64_t)g + i] += taint * fabs(term[i]);
                            if (lr) {
                                double xv[3] = {x, y, 1.0}, xp[2] = {x + ddx, y + ddy};
                                double* rr = lr + 15 * (int64_t)g;
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 3; ++j) rr[3 * i + j] += w * xv[i] * xv[j];
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 2; ++j) rr[9 + 2 * i + j] += w * xv[i] * xp[j];
                            }
                        }
                        if (own_marg) taint += alpha / (1.0 - alpha);
                        T = test;
                    }
                    if (tfinal) tfinal[pi] = T;
                    if (pixmarg) pixmarg[pi] = (uint8_t)(marg || taint > 0.0);
                }
            /* add the band's sums to the view's records, bands in order
             * (the FP64 sums are then independent of the thread count) */
#pragma omp ordered
            {
                for (int64_t i = 0; i < nt; ++i) {
                    const uint32_t g = touched[i];
                    const int64_t o = (int64_t)v * N + g;
                    for (int k = 0; k < 16; ++k) {
                        mom[16 * o + k] += lm[16 * (int64_t)g + k];
                        absm[16 * o + k] += la[16 * (int64_t)g + k];
                        slack[16 * o + k] += ls[16 * (int64_t)g + k];
                        lm[16 * (int64_t)g + k] = la[16 * (int64_t)g + k] = ls[16 * (int64_t)g + k] = 0.0;
                    }
                    if (lr)
                        for (int k = 0; k < 15; ++k) {
                            raw[15 * o + k] += lr[15 * (int64_t)g + k];
                            lr[15 * (int64_t)g + k] = 0.0;
                        }
                    nmarg[o] += ln[g];
                    ln[g] = 0;
                    seen[g] = 0;
                }
                if (counters) { counters[2 * v] += ev; counters[2 * v + 1] += ec; }
            }
        }
        free(lm); free(la); free(ls); free(lr); free(ln); free(seen); free(touched);
    }
    free(task_v);
    free(task_r0);
    free(pix_off);
    free(tile_off);
}

/* Threads used by the parallel loops above (OpenMP's current setting), and a
 * way to change it (the CPU baseline times one thread as well as all). */
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
