// Householder QR fallback shared by the CholeskyQR kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace rh {

// Householder QR of Y (I x K) into Q (I x K), columns signed so that
// diag(R) >= 0.  Used when CholeskyQR breaks down even after the shift,
// i.e. when Y is numerically rank deficient (exact-rank data with p > 0).
__device__ inline void householder_qr(const double* __restrict__ y, int I, int K, double* A, double* Q,
                               double* tau_s, double* alpha_s, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < I * K; e += kBlock) A[e] = y[e];
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        double s = 0.0;
        for (int i = j + tid; i < I; i += kBlock) {
            const double v = A[static_cast<int64_t>(j) * I + i];
            s += v * v;
        }
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (tid == 0) {
            double n2 = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) n2 += red[w];
            const double a = A[static_cast<int64_t>(j) * I + j];
            const double alpha = (a > 0.0 ? -1.0 : 1.0) * sqrt(n2);
            const double v0 = a - alpha;
            const double vn2 = n2 - a * a + v0 * v0;
            A[static_cast<int64_t>(j) * I + j] = v0;
            tau_s[j] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
            alpha_s[j] = alpha;
        }
        __syncthreads();
        const double tau = tau_s[j];
        for (int c = j + 1 + wave; c < K; c += kBlock / kWave) {
            double w = 0.0;
            for (int i = j + lane; i < I; i += kWave)
                w += A[static_cast<int64_t>(j) * I + i] * A[static_cast<int64_t>(c) * I + i];
            w = wave_sum(w);
            for (int i = j + lane; i < I; i += kWave)
                A[static_cast<int64_t>(c) * I + i] -= tau * A[static_cast<int64_t>(j) * I + i] * w;
        }
        __syncthreads();
    }
    for (int e = tid; e < I * K; e += kBlock) {
        const int c = e / I, i = e - c * I;
        Q[e] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = K - 1; j >= 0; --j) {
        const double tau = tau_s[j];
        for (int c = wave; c < K; c += kBlock / kWave) {
            double w = 0.0;
            for (int i = j + lane; i < I; i += kWave)
                w += A[static_cast<int64_t>(j) * I + i] * Q[static_cast<int64_t>(c) * I + i];
            w = wave_sum(w);
            for (int i = j + lane; i < I; i += kWave)
                Q[static_cast<int64_t>(c) * I + i] -= tau * A[static_cast<int64_t>(j) * I + i] * w;
        }
        __syncthreads();
    }
    for (int e = tid; e < I * K; e += kBlock) {
        const int c = e / I;
        if (alpha_s[c] < 0.0) Q[e] = -Q[e];
    }
    __syncthreads();
}


}  // namespace rh
