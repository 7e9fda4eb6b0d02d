// Truncation of R-STHOSVD in the rotated layout (Algorithm 8 step 4 taken as
// Ubar_R^T B, the Lambda V^T shortcut of Section 4.1): out = M^T B for
// B = K x J column-major (the projection's output, K <= 64 rows per column)
// and M = K x R column-major, written rotated, out[r J + j].
//
// Each wave takes 64 consecutive columns of B at a time: their 64 K elements
// are contiguous, so the wave loads them with 16-byte buffer loads (the next
// chunk's loads in flight while the current one is computed; measured on
// this pass, buffer loads sustain about 1.4x the rate of 64-bit-addressed
// global loads) and stores them to its LDS slice.  The product runs on the
// matrix cores in the tensor's own precision (16x16x4 f32 or f64 steps): M^T
// is the A operand, held in registers for the whole kernel, and the slice
// supplies the B operand.  The contraction index is split over the four lane
// groups of a step as k = g KQ + s (g = lane / 16, s = step,
// KQ = ceil(K / 4)) in both operands, so each lane reads one column's
// elements in order.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

// Per wave a slice for the 64 columns in their own order.  A step's operand
// read touches 16 columns at pitch K and 4 runs of KQ: no bank conflict for
// odd K, at most 16-way for K = 64, where the matrix-core work per read is
// also the largest.
__host__ __device__ inline size_t trunc_slice_elems(int K) { return 64 * static_cast<size_t>(K); }
__host__ __device__ inline size_t trunc_lds_elems(int K) { return 4 * trunc_slice_elems(K); }

// RT row tiles of 16 output rows (R <= 16 RT), KQM >= ceil(K / 4) steps;
// a chunk is 64 K <= 256 KQM elements, NL 16-byte pieces per lane
template <typename T, int RT, int KQM>
__device__ __forceinline__ void trunc_body(const T* __restrict__ B, const T* __restrict__ M,
                                           T* __restrict__ out, int K, int R, int64_t J, int bidx,
                                           int nwg) {
    typedef __attribute__((ext_vector_type(4))) float vf4;
    typedef typename Mma<T>::acc_t acc_t;
    extern __shared__ __align__(16) unsigned char tsm[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n16 = lane & 15, g = lane >> 4;
    T* cs = reinterpret_cast<T*>(tsm) + static_cast<size_t>(wave) * trunc_slice_elems(K);
    const int KQ = (K + 3) >> 2;

    // A operand of step s, row tile t: A[m][g] = M(g KQ + s, 16 t + m), zero
    // past K and R
    T a[RT][KQM];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int r = 16 * t + n16;
#pragma unroll
        for (int s = 0; s < KQM; ++s) {
            const int k = g * KQ + s;
            a[t][s] = (s < KQ && k < K && r < R) ? M[static_cast<size_t>(r) * K + k] : T(0);
        }
    }

    // chunk c = 64 columns, elements B[64 c K .. 64 (c + 1) K); lane loads the
    // 16-byte pieces u = lane + 64 t of it
    constexpr int EPV = 16 / sizeof(T);                 // elements per 16-byte piece
    constexpr int NL = 4 * KQM / EPV;
    const int64_t nchunks = (J + 63) / 64;
    const int64_t total = J * K;                         // elements of B
    const int64_t wstride = static_cast<int64_t>(nwg) * (kBlock / kWave);
    int64_t c = static_cast<int64_t>(bidx) * (kBlock / kWave) + wave;
    const int pieces = 64 * K / EPV;                     // per chunk (64 K is a multiple of EPV)
    T buf[NL * EPV];
    auto load = [&](int64_t cc) {
        const int64_t e0 = cc * 64 * K;
        if (e0 + 64 * K <= total) {                      // uniform: a whole chunk
            // buffer loads from a range over the chunk: the 64-bit address
            // is formed once (uniform), the lanes add 32-bit offsets
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<T*>(B + e0), static_cast<short>(0), 64 * K * static_cast<int>(sizeof(T)), 0x00020000);
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                const int u = lane + 64 * t;
                if (u < pieces) {
                    const vf4 v = __builtin_bit_cast(vf4, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * lane, 1024 * t, 0));
                    const T* vp = reinterpret_cast<const T*>(&v);
#pragma unroll
                    for (int q = 0; q < EPV; ++q) buf[t * EPV + q] = vp[q];
                }
            }
        } else {                                         // the last, partial chunk
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                const int u = lane + 64 * t;
#pragma unroll
                for (int q = 0; q < EPV; ++q) {
                    const int64_t e = e0 + static_cast<int64_t>(u) * EPV + q;
                    buf[t * EPV + q] = (u < pieces && e < total) ? B[e] : T(0);
                }
            }
        }
    };
    if (c < nchunks) load(c);
    for (; c < nchunks; c += wstride) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int u = lane + 64 * t;
            if (u < pieces) {
                vf4 v;
                T* vp = reinterpret_cast<T*>(&v);
#pragma unroll
                for (int q = 0; q < EPV; ++q) vp[q] = buf[t * EPV + q];
                *reinterpret_cast<vf4*>(cs + u * EPV) = v;
            }
        }
        if (c + wstride < nchunks) load(c + wstride);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);              // lgkmcnt(0): the slice is written
        __builtin_amdgcn_wave_barrier();
        acc_t acc[4][RT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[q][t] = zero4<acc_t>();
#pragma unroll
        for (int s = 0; s < KQM; ++s) {
            if (s < KQ) {
                const int k = g * KQ + s;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // B operand: B[g][n] = B(k, 64 c + 16 q + n); past K zero
                    // (the word there is the next column's, or past the slice)
                    const T b = k < K ? cs[(16 * q + n16) * K + k] : T(0);
#pragma unroll
                    for (int t = 0; t < RT; ++t) acc[q][t] = Mma<T>::step(a[t][s], b, acc[q][t]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t j = c * 64 + 16 * q + n16;
            if (j < J) {
#pragma unroll
                for (int t = 0; t < RT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * t + Mma<T>::row(g, v);
                        if (r < R) __builtin_nontemporal_store(acc[q][t][v], out + static_cast<int64_t>(r) * J + j);
                    }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);              // reads of the slice done before it is refilled
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T, int RT, int KQM>
__global__ __launch_bounds__(kBlock) void k_trunc_rot(const T* __restrict__ B, const T* __restrict__ M,
                                                      T* __restrict__ out, int K, int R, int64_t J) {
    trunc_body<T, RT, KQM>(B, M, out, K, R, J, blockIdx.x, gridDim.x);
}

// Many truncations: job blockIdx.y on workgroups 0 .. units - 1 of grid x.
template <typename T, int RT, int KQM>
__global__ __launch_bounds__(kBlock) void k_trunc_batch(const TruncJob* __restrict__ jobs) {
    const TruncJob& j = jobs[blockIdx.y];
    if (static_cast<int>(blockIdx.x) >= j.units) return;
    trunc_body<T, RT, KQM>(static_cast<const T*>(j.b), static_cast<const T*>(j.m), static_cast<T*>(j.out),
                           j.K, j.R, j.J, blockIdx.x, j.units);
}

bool plan_trunc(bool dbl, int64_t I, int64_t T, int R, int num_cu, bool any_size, TruncGeom* g) {
    // I = K rows of B: FP32 up to K = 64 (four row tiles), FP64 up to K = 32
    if (I < 1 || I > (dbl ? 32 : 64) || R < 1 || R > I || T < 1) return false;
    // unless asked for at any size, only where every wave of the full grid
    // gets several chunks: measured against the column kernels'
    // truncation, this kernel wins at 8e6 columns (443 against 467 us at
    // K = 35, R = 25) and loses at 1e6 and below (68 against 61 us), where
    // each wave's first chunk waits for its loads with nothing to overlap
    const int64_t waves = 4 * 4 * static_cast<int64_t>(num_cu > 0 ? num_cu : 256);
    if (!any_size && (T + 63) / 64 < 8 * waves) return false;
    const size_t elem = dbl ? 8 : 4;
    g->K = static_cast<int>(I);
    g->R = R;
    g->J = T;
    g->rb = (R + 15) / 16;
    g->lds_bytes = trunc_lds_elems(g->K) * elem;
    if (g->lds_bytes + kStaticLdsMargin > kLdsLimit) return false;
    const int64_t chunks = (T + 63) / 64;
    const int64_t wgs = (chunks + 3) / 4;
    const int64_t cap = 4 * static_cast<int64_t>(num_cu > 0 ? num_cu : 256);
    g->grid = static_cast<int>(wgs < cap ? wgs : cap);
    return true;
}

template <typename T, int RT, int KQM>
static void launch_trunc_k(const TruncGeom& g, const void* B, const void* M, void* out, hipStream_t s) {
    hipLaunchKernelGGL((k_trunc_rot<T, RT, KQM>), dim3(g.grid), dim3(kBlock), g.lds_bytes, s,
                       static_cast<const T*>(B), static_cast<const T*>(M), static_cast<T*>(out), g.K, g.R,
                       g.J);
}

// the smallest step bound KQM in {4, 8, 12, 16} with 4 KQM >= K; RT <= KQM / 4
template <typename T, int KQM>
static hipError_t launch_trunc_q(const TruncGeom& g, const void* B, const void* M, void* out,
                                 hipStream_t s) {
    if (g.rb < 1 || 16 * g.rb > 4 * KQM) return hipErrorInvalidValue;
    if (g.rb == 1) launch_trunc_k<T, 1, KQM>(g, B, M, out, s);
    if constexpr (KQM >= 8) if (g.rb == 2) launch_trunc_k<T, 2, KQM>(g, B, M, out, s);
    if constexpr (KQM >= 12) if (g.rb == 3) launch_trunc_k<T, 3, KQM>(g, B, M, out, s);
    if constexpr (KQM >= 16) if (g.rb == 4) launch_trunc_k<T, 4, KQM>(g, B, M, out, s);
    return hipGetLastError();
}

hipError_t launch_trunc(bool dbl, const TruncGeom& g, const void* B, const void* M, void* out,
                        hipStream_t s) {
    const int kq = (g.K + 3) / 4;
    if (dbl) {
        if (kq <= 4) return launch_trunc_q<double, 4>(g, B, M, out, s);
        if (kq <= 8) return launch_trunc_q<double, 8>(g, B, M, out, s);
        return hipErrorInvalidValue;
    }
    if (kq <= 4) return launch_trunc_q<float, 4>(g, B, M, out, s);
    if (kq <= 8) return launch_trunc_q<float, 8>(g, B, M, out, s);
    if (kq <= 12) return launch_trunc_q<float, 12>(g, B, M, out, s);
    if (kq <= 16) return launch_trunc_q<float, 16>(g, B, M, out, s);
    return hipErrorInvalidValue;
}

// step bound of the batched instantiations: the smallest of 4, 8, 12, 16
// with 4 KQM >= K
size_t trunc_lds_bytes(int K, bool dbl) { return trunc_lds_elems(K) * (dbl ? 8 : 4); }

int trunc_kqm(int K) {
    const int kq = (K + 3) / 4;
    return kq <= 4 ? 4 : kq <= 8 ? 8 : kq <= 12 ? 12 : 16;
}

template <typename T, int RT, int KQM>
static void launch_trunc_batch_k(const TruncJob* jobs, int njobs, int max_units, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_trunc_batch<T, RT, KQM>), dim3(max_units, njobs), dim3(kBlock), lds, s, jobs);
}

template <typename T, int KQM>
static hipError_t launch_trunc_batch_q(int rt, const TruncJob* jobs, int njobs, int max_units, size_t lds,
                                       hipStream_t s) {
    if (rt < 1 || 16 * rt > 4 * KQM) return hipErrorInvalidValue;
    if (rt == 1) launch_trunc_batch_k<T, 1, KQM>(jobs, njobs, max_units, lds, s);
    if constexpr (KQM >= 8) if (rt == 2) launch_trunc_batch_k<T, 2, KQM>(jobs, njobs, max_units, lds, s);
    if constexpr (KQM >= 12) if (rt == 3) launch_trunc_batch_k<T, 3, KQM>(jobs, njobs, max_units, lds, s);
    if constexpr (KQM >= 16) if (rt == 4) launch_trunc_batch_k<T, 4, KQM>(jobs, njobs, max_units, lds, s);
    return hipGetLastError();
}

hipError_t launch_trunc_batch(bool dbl, int rt, int kqm, const TruncJob* jobs, int njobs, int max_units,
                              size_t lds, hipStream_t s) {
    if (njobs < 1 || max_units < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (dbl) {
        if (kqm == 4) return launch_trunc_batch_q<double, 4>(rt, jobs, njobs, max_units, lds, s);
        if (kqm == 8) return launch_trunc_batch_q<double, 8>(rt, jobs, njobs, max_units, lds, s);
        return hipErrorInvalidValue;
    }
    if (kqm == 4) return launch_trunc_batch_q<float, 4>(rt, jobs, njobs, max_units, lds, s);
    if (kqm == 8) return launch_trunc_batch_q<float, 8>(rt, jobs, njobs, max_units, lds, s);
    if (kqm == 12) return launch_trunc_batch_q<float, 12>(rt, jobs, njobs, max_units, lds, s);
    if (kqm == 16) return launch_trunc_batch_q<float, 16>(rt, jobs, njobs, max_units, lds, s);
    return hipErrorInvalidValue;
}

}  // namespace rh
