// Projection arithmetic of the reconstruction loops built on the simulator:
// the total weight of a (possibly signed) source, and a fixed-point tally
// scaled to activity units and optionally added to a running projection.
// Reuse of photon tracks (Sec. 5.3) needs both (the difference source's
// histories are proportional to sum |d|; the new projection is the old one
// plus the scaled difference projection); coarse-grid scatter modelling
// (Sec. 5.4) scales its expanded projection the same way.
#include "mc_internal.h"

namespace mcs {
namespace {

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0;
}

// sum over voxels of |act - prev| (act when prev is null): per-thread sums of
// a grid-strided range, a wavefront reduction, one atomic per wavefront
// (integer: the total does not depend on the order).
__global__ __launch_bounds__(256) void k_source_total(const uint32_t* __restrict__ act,
                                                      const uint32_t* __restrict__ prev, uint64_t n,
                                                      unsigned long long* total) {
    uint64_t s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        s += source_weight(act, prev, i);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, (unsigned long long)s);
}

// out[i] = (accumulate ? out[i] : 0) + tally[i] 2^-32 scale
__global__ __launch_bounds__(256) void k_scale_tally(const int64_t* __restrict__ tally, uint64_t n,
                                                     double scale, double* __restrict__ out,
                                                     int accumulate) {
    const double s = scale * (1.0 / 4294967296.0);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = (double)tally[i] * s;
        out[i] = accumulate ? out[i] + v : v;
    }
}

int grid_n(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

hipError_t launch_source_total(const uint32_t* act, const uint32_t* prev, uint64_t n,
                               unsigned long long* total, hipStream_t s) {
    k_zero_u64<<<1, 64, 0, s>>>(total);
    k_source_total<<<grid_n(n), 256, 0, s>>>(act, prev, n, total);
    return hipGetLastError();
}

hipError_t launch_scale_tally(const int64_t* tally, uint64_t n, double scale, double* out, int accumulate,
                              hipStream_t s) {
    k_scale_tally<<<grid_n(n), 256, 0, s>>>(tally, n, scale, out, accumulate);
    return hipGetLastError();
}

}  // namespace mcs
