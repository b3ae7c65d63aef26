// tg_ssim_loss_grad: the structural-similarity term of the 3DGS objective
// used by the refinement (Sec. 4.6 refines as the original 3DGS does:
// L = (1 - lambda) L1 + lambda (1 - SSIM), 11x11 Gaussian window, sigma 1.5).
//
// Both kernels are separable 11-tap blurs over a block tile of 64 pixels x 56
// rows, with the three channels interleaved as in memory (192 threads, one
// per (pixel column, channel)).  Input rows stream through LDS eleven at a
// time (a coalesced load of 222 floats per row, halo included); each thread
// blurs a row horizontally from LDS and adds the result to the eleven output
// rows it touches, kept in registers as a ring indexed modulo 11 (the row
// loop is unrolled by 11 so every ring index is static).  After input row i
// the output row i - 10 is complete: it is finished and its ring slot reused.
//   k_ssim_fwd  the five blurred moments (mu_x, mu_y, E[x^2], E[y^2], E[xy])
//               with zero padding, the SSIM value (summed into ssim_sum) and
//               its partial derivatives dS/dmu_x, dS/dE[x^2], dS/dE[xy]
//               (three maps in the workspace).
//   k_ssim_bwd  blurs the three maps (the window is symmetric, so the adjoint
//               of the blur is the blur) and adds
//               scale * (G*dmu + 2 x G*dExx + y G*dExy) to the gradient.
#include "tg_internal.h"

namespace {

constexpr int TW = 64;                 // tile width in pixels
constexpr int R = 5;                   // window radius
constexpr int NTAP = 2 * R + 1;        // 11 taps; also rows per LDS chunk
constexpr int TH = 6 * NTAP - 2 * R;   // 56 output rows: 66 input rows = 6 chunks
constexpr int NCHUNK = (TH + 2 * R) / NTAP;
constexpr int COLS = 3 * TW;           // threads per block
constexpr int PW = 3 * (TW + 2 * R);   // floats per staged row (222)
constexpr float C1 = 0.01f * 0.01f;
constexpr float C2 = 0.03f * 0.03f;

struct Win {
    float g[NTAP];
};

struct SsimArgs {
    const float* img;
    const float* tgt;
    float* grad;
    float* ssim_sum;
    float* dmu;    // [B,H,W,3] partial maps
    float* dxx;
    float* dxy;
    int B, H, W;
    float scale;
};

// Stage input rows [row0, row0 + NTAP) of the tile's patch (zero outside the
// image) from up to three [B,H,W,3] arrays into LDS.
template <int NA>
__device__ __forceinline__ void stage_rows(const float* const (&src)[NA], float (*dst)[NTAP * PW], const SsimArgs& a,
                                           int b, int x0, int gy0) {
    for (int i = threadIdx.x; i < NTAP * PW; i += COLS) {
        const int r = i / PW, f = i - r * PW;
        const int gy = gy0 + r, gx = x0 - R + f / 3;
        const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
        const int64_t o = (((int64_t)b * a.H + gy) * a.W + (x0 - R)) * 3 + f;
#pragma unroll
        for (int k = 0; k < NA; ++k) dst[k][i] = in ? src[k][o] : 0.f;
    }
}

__global__ void __launch_bounds__(COLS) k_ssim_fwd(SsimArgs a, Win win) {
    __shared__ float L[2][NTAP * PW];
    __shared__ float red[COLS / 64];
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, b = blockIdx.z;
    const bool colok = x0 + t / 3 < a.W;
    const float* const src[2] = {a.img, a.tgt};
    float acc[NTAP][5];
#pragma unroll
    for (int s = 0; s < NTAP; ++s)
#pragma unroll
        for (int m = 0; m < 5; ++m) acc[s][m] = 0.f;
    float ssum = 0.f;
    for (int q = 0; q < NCHUNK; ++q) {
        __syncthreads();
        stage_rows<2>(src, L, a, b, x0, y0 - R + q * NTAP);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NTAP; ++j) {
            float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f, h4 = 0.f;
#pragma unroll
            for (int k = 0; k < NTAP; ++k) {
                const float x = L[0][j * PW + t + 3 * k], y = L[1][j * PW + t + 3 * k];
                const float gx = win.g[k] * x, gy = win.g[k] * y;
                h0 += gx;
                h1 += gy;
                h2 += gx * x;
                h3 += gy * y;
                h4 += gx * y;
            }
            // input row i = q*11 + j feeds output rows i - k with weight g[k]
#pragma unroll
            for (int k = 0; k < NTAP; ++k) {
                float* A = acc[(j - k + NTAP) % NTAP];
                const float gk = win.g[k];
                A[0] += gk * h0;
                A[1] += gk * h1;
                A[2] += gk * h2;
                A[3] += gk * h3;
                A[4] += gk * h4;
            }
            const int o = q * NTAP + j - 2 * R;   // output row now complete
            if (o >= 0) {
                float* A = acc[(j + 1) % NTAP];
                const int py = y0 + o;
                if (py < a.H && colok) {
                    const float mx = A[0], my = A[1], exx = A[2], eyy = A[3], exy = A[4];
                    const float A1 = 2.f * mx * my + C1, A2 = 2.f * (exy - mx * my) + C2;
                    const float B1 = mx * mx + my * my + C1, B2 = (exx - mx * mx) + (eyy - my * my) + C2;
                    const float inv = 1.0f / (B1 * B2);
                    const float S = A1 * A2 * inv;
                    ssum += S;
                    const int64_t off = (((int64_t)b * a.H + py) * a.W + x0) * 3 + t;
                    a.dmu[off] = 2.f * my * (A2 - A1) * inv - S * (2.f * mx / B1 - 2.f * mx / B2);
                    a.dxx[off] = -S / B2;
                    a.dxy[off] = 2.f * A1 * inv;
                }
            }
            // the slot is free for output row o + 11 (rows before the first
            // output fill slots of rows -10..-1, cleared here too)
#pragma unroll
            for (int m = 0; m < 5; ++m) acc[(j + 1) % NTAP][m] = 0.f;
        }
    }
    for (int off = 32; off > 0; off >>= 1) ssum += __shfl_xor(ssum, off, 64);
    if ((t & 63) == 0) red[t >> 6] = ssum;
    __syncthreads();
    if (t == 0 && a.ssim_sum) atomicAdd(a.ssim_sum, red[0] + red[1] + red[2]);
}

__global__ void __launch_bounds__(COLS) k_ssim_bwd(SsimArgs a, Win win) {
    __shared__ float L[3][NTAP * PW];
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, b = blockIdx.z;
    const bool colok = x0 + t / 3 < a.W;
    const float* const src[3] = {a.dmu, a.dxx, a.dxy};
    float acc[NTAP][3];
#pragma unroll
    for (int s = 0; s < NTAP; ++s)
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[s][m] = 0.f;
    for (int q = 0; q < NCHUNK; ++q) {
        __syncthreads();
        stage_rows<3>(src, L, a, b, x0, y0 - R + q * NTAP);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NTAP; ++j) {
            float h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
            for (int k = 0; k < NTAP; ++k) {
                const float gk = win.g[k];
                h0 += gk * L[0][j * PW + t + 3 * k];
                h1 += gk * L[1][j * PW + t + 3 * k];
                h2 += gk * L[2][j * PW + t + 3 * k];
            }
#pragma unroll
            for (int k = 0; k < NTAP; ++k) {
                float* A = acc[(j - k + NTAP) % NTAP];
                const float gk = win.g[k];
                A[0] += gk * h0;
                A[1] += gk * h1;
                A[2] += gk * h2;
            }
            const int o = q * NTAP + j - 2 * R;
            if (o >= 0) {
                float* A = acc[(j + 1) % NTAP];
                const int py = y0 + o;
                if (py < a.H && colok) {
                    const int64_t off = (((int64_t)b * a.H + py) * a.W + x0) * 3 + t;
                    const float x = a.img[off], y = a.tgt[off];
                    a.grad[off] += a.scale * (A[0] + 2.f * x * A[1] + y * A[2]);
                }
            }
            // the slot is free for output row o + 11 (rows before the first
            // output fill slots of rows -10..-1, cleared here too)
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[(j + 1) % NTAP][m] = 0.f;
        }
    }
}

}  // namespace

extern "C" tg_status tg_ssim_loss_grad(const float* image, const float* target, int32_t B, int32_t H, int32_t W,
                                       float scale, float* grad, float* ssim_sum, void* ws, size_t* ws_bytes,
                                       void* stream)
{
    if (!ws_bytes || B < 0 || H < 0 || W < 0) return TG_ERR_INVALID_ARG;
    if (B > 65535) return TG_ERR_UNSUPPORTED;
    const size_t map = (size_t)B * H * W * 3 * sizeof(float);
    const size_t need = 3 * ((map + 255) & ~(size_t)255);
    if (!ws) {
        *ws_bytes = need;
        return TG_OK;
    }
    if (*ws_bytes < need) return TG_ERR_WORKSPACE;
    if (!image || !target || !grad) return TG_ERR_INVALID_ARG;
    if ((int64_t)B * H * W == 0) return TG_OK;
    SsimArgs a;
    a.img = image;
    a.tgt = target;
    a.grad = grad;
    a.ssim_sum = ssim_sum;
    const size_t step = (map + 255) & ~(size_t)255;
    a.dmu = (float*)ws;
    a.dxx = (float*)((char*)ws + step);
    a.dxy = (float*)((char*)ws + 2 * step);
    a.B = B;
    a.H = H;
    a.W = W;
    a.scale = scale;
    Win win;
    double g[2 * R + 1], sum = 0.0;
    for (int k = 0; k < 2 * R + 1; ++k) {
        const double x = k - R;
        g[k] = exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < 2 * R + 1; ++k) win.g[k] = (float)(g[k] / sum);
    const dim3 grid((unsigned)((W + TW - 1) / TW), (unsigned)((H + TH - 1) / TH), (unsigned)B);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(COLS), 0, (hipStream_t)stream, a, win);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(COLS), 0, (hipStream_t)stream, a, win);
    TG_CHECK_LAUNCH();
    return TG_OK;
}
