// Host-side interface of the kernels (launchers).  Every launcher enqueues on
// `stream` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rh {

enum StreamOp { OP_SKETCH = 0, OP_POWER = 1, OP_TTM = 2 };

// Geometry of one streaming pass over an n-unfolding view (L, I, T) of a
// first-index-fastest tensor: element (i, j = l + L t) at src[l + L (i + I t)].
struct StreamGeom {
    int64_t L, I, T, J;   // J = L T
    int K;                // sketch width (SKETCH/POWER) or output rows Kout (TTM)
    int I_pad, K_pad;     // rounded up to 16
    int P;                // LDS pitch of the tile (>= I_pad)
    int KW;               // LDS pitch of the K-wide operands (>= K_pad)
    int C;                // unfolding columns per tile (16, 32 or 64)
    int64_t ntiles;
    int grid;             // workgroups (each walks tiles grid-stride)
    size_t lds_bytes;
};

struct StreamArgs {
    const void* src;
    const void* mat;      // POWER: Q (I x K); TTM: M (I x Kout); column-major
    void* out;            // TTM: folded output
    void* part_y;         // [grid][K_pad][I_pad] partial sketches (SKETCH/POWER)
    void* part_g;         // [grid][K_pad][K_pad] partial Gram (TTM, optional)
    double* part_ss;      // [grid] partial sum of squares of src (optional)
    uint64_t seed;
    uint32_t mode, tag;
};

// Plan the geometry of a pass; returns false if the shape exceeds the
// implemented limits.  elem = sizeof(float) or sizeof(double).
bool plan_stream(int op, int elem, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                 StreamGeom* g);

hipError_t launch_stream(int op, bool dbl, const StreamGeom& g, const StreamArgs& a,
                         hipStream_t s);

// Fixed-order reductions of per-workgroup partials.
hipError_t launch_reduce_y(bool dbl, const void* part, int G, int I, int K, int I_pad, int K_pad,
                           double* y, hipStream_t s);
hipError_t launch_reduce_ss(const double* part, int G, double* out, hipStream_t s);

// CholeskyQR2 (shifted CholeskyQR3 when needed).  y is I x K double; work is
// I x K double scratch; q64 (may equal work) and q_out receive Q.
hipError_t launch_cqr(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                      uint32_t* flags, hipStream_t s);

hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s);

// U = Q V[:, :R] (V == nullptr means identity), canonical signs, M = V[:, :R] diag(s),
// sigma = sqrt(max(lambda, 0))[:R] (lambda may be nullptr).
hipError_t launch_factor(bool dbl, const void* q, const double* v, const double* lambda, int64_t I,
                         int K, int R, void* u_out, void* m_out, double* sigma_out, double* u64,
                         hipStream_t s);

hipError_t launch_sumsq(bool dbl, const void* x, int64_t n, double* part, int G, hipStream_t s);

hipError_t launch_omega_fill(bool dbl, uint64_t seed, int mode, int tag, int64_t J, int K,
                             void* out, hipStream_t s);

hipError_t launch_gram_reduce(bool dbl, const void* part, int G, int K, int K_pad, double* c,
                              hipStream_t s);

struct ReportInit {
    int32_t order;
    int32_t k_used[16];
};
hipError_t launch_report_init(void* rep, ReportInit ri, hipStream_t s);
hipError_t launch_copy_bytes(const void* src, void* dst, size_t n, hipStream_t s);

}  // namespace rh
