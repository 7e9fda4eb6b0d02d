// Bookkeeping kernels of the batched decomposition: one workgroup per item
// of the batch (device tables of jobs), so that a whole batch needs one
// launch per step whatever its size.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

// report = zero, order, k_used (a negative entry marks a capped K)
__global__ void k_batch_report_init(const ReportJob* __restrict__ jobs) {
    const ReportJob& j = jobs[blockIdx.x];
    rhosvd_report* rep = j.rep;
    double* sg = &rep->sigma[0][0];
    for (int e = threadIdx.x; e < RHOSVD_MAX_ORDER * RHOSVD_MAX_K; e += blockDim.x) sg[e] = 0.0;
    if (threadIdx.x == 0) {
        uint32_t fl = 0;
        rep->norm_x2 = 0.0;
        rep->norm_core2 = 0.0;
        rep->resid2 = 0.0;
        rep->order = j.order;
        for (int n = 0; n < RHOSVD_MAX_ORDER; ++n) {
            const int k = j.k_used[n];
            if (k < 0) fl |= RHOSVD_FLAG_K_CAPPED;
            rep->k_used[n] = k < 0 ? -k : k;
        }
        rep->flags = fl;
    }
}

// report->norm_x2 = sum of the first pass's per-workgroup sums of squares
__global__ void k_batch_norm_x(const SumJob* __restrict__ jobs) {
    __shared__ double red[kBlock];
    const SumJob& j = jobs[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < j.G; i += kBlock) s += j.part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) j.rep->norm_x2 = red[0];
}

// report->norm_core2 = ||core||^2 (FP64, fixed order), then the report is
// copied to the caller's buffer
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_finish(const FinishJob* __restrict__ jobs) {
    __shared__ double red[kBlock];
    const FinishJob& j = jobs[blockIdx.x];
    const T* core = static_cast<const T*>(j.core);
    // eight loads in flight per thread, four accumulation chains (fixed order)
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t n = j.core_elems;
    int64_t e = threadIdx.x;
    for (; e + 7 * kBlock < n; e += 8 * kBlock) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = core[e + u * kBlock];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double d = static_cast<double>(v[u]);
            s4[u & 3] = fma(d, d, s4[u & 3]);
        }
    }
    for (; e < n; e += kBlock) {
        const double d = static_cast<double>(core[e]);
        s4[0] = fma(d, d, s4[0]);
    }
    red[threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) j.rep->norm_core2 = red[0];
    __syncthreads();
    if (j.out_report) {
        // 8-byte words when both ends allow them (the report's size is a
        // multiple of 8); the pointers do not alias, so every load of a thread
        // is issued before its stores
        constexpr int kWords = static_cast<int>(sizeof(rhosvd_report) / 8);
        static_assert(sizeof(rhosvd_report) % 8 == 0, "the report is copied in 8-byte words");
        if (((reinterpret_cast<uintptr_t>(j.rep) | reinterpret_cast<uintptr_t>(j.out_report)) & 7) == 0) {
            const uint64_t* __restrict__ src = reinterpret_cast<const uint64_t*>(j.rep);
            uint64_t* __restrict__ dst = static_cast<uint64_t*>(j.out_report);
            for (int e = threadIdx.x; e < kWords; e += kBlock) dst[e] = src[e];
        } else {
            const unsigned char* __restrict__ src = reinterpret_cast<const unsigned char*>(j.rep);
            unsigned char* __restrict__ dst = static_cast<unsigned char*>(j.out_report);
            for (int e = threadIdx.x; e < static_cast<int>(sizeof(rhosvd_report)); e += kBlock)
                dst[e] = src[e];
        }
    }
}

hipError_t launch_batch_report_init(const ReportJob* jobs, int njobs, hipStream_t s) {
    if (njobs < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_report_init, dim3(njobs), dim3(kBlock), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_batch_norm_x(const SumJob* jobs, int njobs, hipStream_t s) {
    if (njobs < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_norm_x, dim3(njobs), dim3(kBlock), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_batch_finish(bool dbl, const FinishJob* jobs, int njobs, hipStream_t s) {
    if (njobs < 1) return hipErrorInvalidValue;
    if (dbl)
        hipLaunchKernelGGL(k_batch_finish<double>, dim3(njobs), dim3(kBlock), 0, s, jobs);
    else
        hipLaunchKernelGGL(k_batch_finish<float>, dim3(njobs), dim3(kBlock), 0, s, jobs);
    return hipGetLastError();
}

}  // namespace rh
