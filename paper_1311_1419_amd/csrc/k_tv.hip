// Total-variation recovery of block residuals (the TVAL3-style solver of
// Section 4, reference [14]), FP32, pixel domain, images as rows (nblk x n,
// each a BH x BW image row-major: a B x B block, or a whole frame):
//   min_x lam TV(x) + 1/2 ||Phi x - y^||^2,  TV(x) = sum_i ||D_i x||_2,
// by the linearised alternating-direction iteration, x_0 = 0, nu_0 = 0:
//   w   = shrink(D x + nu / beta, lam / beta)
//   x  <- x - alpha (Phi^T (Phi x - y^) + D^T (nu + beta (D x - w)))
//   nu <- nu + beta (D x - w)
// with alpha = 1 / (L + 8 beta), beta = 0.03 lam per block (1 if lam = 0),
// D the horizontal and vertical forward differences inside the block (zero
// across the last column and row).  One iteration is four launches: the
// dual step (the previous iteration's multiplier update, which needs the new
// x, then w and P = nu + beta (D x - w)), the forward product, the adjoint
// product, and the primal step.
#include <cmath>

#include "internal.h"
#include "tv_step.h"

namespace csv {

// One thread per pixel.  nu, w: (nblk x n) pairs (horizontal, vertical);
// on entry w holds the previous iteration's w (zero before the first).
__global__ __launch_bounds__(256) void tv_dual_kernel(const float* __restrict__ x,
                                                      float* __restrict__ nuh, float* __restrict__ nuv,
                                                      float* __restrict__ wh, float* __restrict__ wv,
                                                      float* __restrict__ ph, float* __restrict__ pv,
                                                      const float* __restrict__ lam, int nblk, int BH,
                                                      int BW) {
    const int n = BH * BW;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nblk * n) return;
    const int b = (int)(idx / n), k = (int)(idx - (size_t)b * n);
    const int i = k / BW, j = k - i * BW;
    tv_dual_at(x + (size_t)b * n, k, i, j, BH, BW, idx, lam[b], nuh, nuv, wh, wv, ph, pv);
}

// x <- x - alpha_b (g + D^T p), one thread per pixel (alpha per image).
__global__ __launch_bounds__(256) void tv_primal_kernel(float* __restrict__ x,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ ph,
                                                        const float* __restrict__ pv,
                                                        const float* __restrict__ alpha, int nblk,
                                                        int BH, int BW) {
    const int n = BH * BW;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nblk * n) return;
    const int b = (int)(idx / n), k = (int)(idx - (size_t)b * n);
    const int i = k / BW, j = k - i * BW;
    const float dt = tv_dtp_at(ph + (size_t)b * n, pv + (size_t)b * n, k, i, j, BH, BW);
    x[idx] -= alpha[b] * (g[idx] + dt);
}

// alpha_b = 1 / (L + 8 beta(lam_b)) for the images of one operator.
__global__ void tv_alpha_kernel(const double* __restrict__ lip, const float* __restrict__ lam,
                                int count, float* __restrict__ alpha) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) alpha[b] = tv_alpha(lip[0], tv_beta(lam[b]));
}

// FP64 check per block (one workgroup): r = s_Phi Q x - y^ with y^ =
// s_Phi c 2^e recomputed exactly; obj = 1/2 ||r||^2 + lam TV(x), ||r|| / ||y^||.
__global__ __launch_bounds__(256) void tv_final64_kernel(const int8_t* __restrict__ q,
                                                         const float* __restrict__ x,
                                                         const int8_t* __restrict__ codes,
                                                         const uint8_t* __restrict__ exps,
                                                         const float* __restrict__ lam, int M,
                                                         int B, double s_phi,
                                                         double* __restrict__ obj) {
    extern __shared__ double xs[];   // n
    __shared__ double red[3][256];
    const int n = B * B, b = blockIdx.x, tid = threadIdx.x;
    const float* xb = x + (size_t)b * n;
    double tvs = 0.0;
    for (int k = tid; k < n; k += 256) {
        const double v = xb[k];
        xs[k] = v;
        const int i = k / B, j = k - i * B;
        const double dh = j + 1 < B ? (double)xb[k + 1] - v : 0.0;
        const double dv = i + 1 < B ? (double)xb[k + B] - v : 0.0;
        tvs += sqrt(dh * dh + dv * dv);
    }
    __syncthreads();
    const int e = exps[b];
    double rr = 0.0, yy = 0.0;
    for (int m = tid; m < M; m += 256) {
        const int8_t* qr = q + (size_t)m * n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += (double)qr[k] * xs[k];
        const double yh = s_phi * ldexp((double)codes[(size_t)b * M + m], e);
        const double d = s_phi * acc - yh;
        rr += d * d;
        yy += yh * yh;
    }
    red[0][tid] = rr;
    red[1][tid] = yy;
    red[2][tid] = tvs;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
            red[2][tid] += red[2][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        obj[(size_t)b * 2 + 0] = 0.5 * red[0][0] + (double)lam[b] * red[2][0];
        obj[(size_t)b * 2 + 1] = red[1][0] > 0.0 ? sqrt(red[0][0]) / sqrt(red[1][0]) : 0.0;
    }
}

void launch_tv_dual(const float* x, float* nuh, float* nuv, float* wh, float* wv, float* ph,
                    float* pv, const float* lam, int nblk, int BH, int BW, hipStream_t st) {
    const size_t t = (size_t)nblk * BH * BW;
    if (!t) return;
    tv_dual_kernel<<<dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st>>>(x, nuh, nuv, wh, wv,
                                                                           ph, pv, lam, nblk, BH, BW);
    CSV_HIP(hipGetLastError());
}

void launch_tv_primal(float* x, const float* g, const float* ph, const float* pv,
                      const float* alpha, int nblk, int BH, int BW, hipStream_t st) {
    const size_t t = (size_t)nblk * BH * BW;
    if (!t) return;
    tv_primal_kernel<<<dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st>>>(x, g, ph, pv, alpha,
                                                                             nblk, BH, BW);
    CSV_HIP(hipGetLastError());
}

void launch_tv_alpha(const double* lip, const float* lam, int count, float* alpha,
                     hipStream_t st) {
    if (count <= 0) return;
    tv_alpha_kernel<<<dim3(ceil_div(count, 256)), dim3(256), 0, st>>>(lip, lam, count, alpha);
    CSV_HIP(hipGetLastError());
}

void launch_tv_final64(const int8_t* q, const float* x, const int8_t* codes, const uint8_t* exps,
                       const float* lam, int nblk, int M, int B, double s_phi, double* obj,
                       hipStream_t st) {
    if (nblk <= 0) return;
    tv_final64_kernel<<<dim3(nblk), dim3(256), (size_t)B * B * sizeof(double), st>>>(
        q, x, codes, exps, lam, M, B, s_phi, obj);
    CSV_HIP(hipGetLastError());
}

}  // namespace csv
