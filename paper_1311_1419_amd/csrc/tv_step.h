// Per-pixel steps of the total-variation iteration (the linearised
// alternating-direction solver of the TVAL3 style, Section 4, reference
// [14]) on row-major BH x BW images, shared by the block solver and the
// whole-frame solver so that both take the same arithmetic.
#pragma once
#include <hip/hip_runtime.h>

namespace csv {

constexpr float kTvBetaRatio = 0.03f;

__device__ inline float tv_beta(float lam) { return lam > 0.f ? kTvBetaRatio * lam : 1.f; }

// alpha = 1 / (L + 8 beta) (||D||^2 <= 8)
__device__ inline float tv_alpha(double L, float beta) {
    return (float)(1.0 / (L + 8.0 * (double)beta));
}

// Dual step at pixel k = (i, j) of image xb, state at index idx: the previous
// iteration's multiplier update with the current x, then w = shrink(D x +
// nu / beta, lam / beta) and P = nu + beta (D x - w).
__device__ inline void tv_dual_at(const float* __restrict__ xb, int k, int i, int j, int BH,
                                  int BW, size_t idx, float l, float* __restrict__ nuh,
                                  float* __restrict__ nuv, float* __restrict__ wh,
                                  float* __restrict__ wv, float* __restrict__ ph,
                                  float* __restrict__ pv) {
    // every load is issued unconditionally (a neighbour past the edge reads
    // the pixel itself, whose difference is then exactly zero)
    const int kr = j + 1 < BW ? k + 1 : k, kd = i + 1 < BH ? k + BW : k;
    const float xv = xb[k], xr = xb[kr], xd = xb[kd];
    const float nh0 = nuh[idx], nv0 = nuv[idx], wh0 = wh[idx], wv0 = wv[idx];
    const float dh = xr - xv, dv = xd - xv;
    const float beta = tv_beta(l);
    const float nh = nh0 + beta * (dh - wh0);
    const float nv = nv0 + beta * (dv - wv0);
    const float vh = dh + nh / beta, vv = dv + nv / beta;
    const float mag = sqrtf(vh * vh + vv * vv);
    const float sc = mag > 0.f ? fmaxf(mag - l / beta, 0.f) / mag : 0.f;
    const float w1 = sc * vh, w2 = sc * vv;
    nuh[idx] = nh;
    nuv[idx] = nv;
    wh[idx] = w1;
    wv[idx] = w2;
    ph[idx] = nh + beta * (dh - w1);
    pv[idx] = nv + beta * (dv - w2);
}

// D^T p at pixel k = (i, j): - ph(i, j)[j < BW-1] + ph(i, j-1)[j > 0]
// - pv(i, j)[i < BH-1] + pv(i-1, j)[i > 0]  (phb, pvb: the image's P).
__device__ inline float tv_dtp_at(const float* __restrict__ phb, const float* __restrict__ pvb,
                                  int k, int i, int j, int BH, int BW) {
    const float a = phb[k], b = phb[j > 0 ? k - 1 : k];
    const float c = pvb[k], d = pvb[i > 0 ? k - BW : k];
    float dt = 0.f;
    dt = j + 1 < BW ? dt - a : dt;
    dt = j > 0 ? dt + b : dt;
    dt = i + 1 < BH ? dt - c : dt;
    dt = i > 0 ? dt + d : dt;
    return dt;
}

}  // namespace csv
