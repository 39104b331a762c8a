// Coarse-grid scatter modelling (Sec. 5.4): the scatter projection is
// simulated with larger source voxels and larger detector pixels, then
// expanded and interpolated to the normal pixel size.
//
// k_block_activity gives every voxel the summed activity of its f^3 block,
// so the simulator's emission (voxel by activity, uniform inside it) is
// uniform over the block.  k_expand turns a coarse Q31.32 projection into
// counts per normal pixel: bilinear interpolation at the pixel centre of the
// coarse values read as samples at the coarse pixel centres (held constant
// beyond the outermost centres), divided by f^2 (and times a caller's scale,
// e.g. to activity units).  Both are HBM-bound passes.
#include "mc_internal.h"

namespace mcs {
namespace {

// one thread per block of f^3 voxels: sum in 64 bits, write the sum to the
// block's voxels (flag if it does not fit 32 bits)
__global__ __launch_bounds__(256) void k_block_activity(const uint32_t* __restrict__ act, int nx, int ny,
                                                        int nz, int f, uint32_t* __restrict__ out,
                                                        int64_t* status) {
    const int bx = nx / f, by = ny / f, bz = nz / f;
    const uint64_t nb = (uint64_t)bx * by * bz;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(b % bx), iy = (int)((b / bx) % by), iz = (int)(b / ((uint64_t)bx * by));
        uint64_t s = 0;
        for (int z = 0; z < f; ++z)
            for (int y = 0; y < f; ++y) {
                const uint64_t row = ((uint64_t)(iz * f + z) * ny + (iy * f + y)) * nx + (uint64_t)ix * f;
                for (int x = 0; x < f; ++x) s += act[row + x];
            }
        if (s > 0xFFFFFFFFull) {
            atomicOr((unsigned long long*)status, (unsigned long long)MC_STATUS_ACTIVITY_OVERFLOW);
            s = 0xFFFFFFFFull;
        }
        for (int z = 0; z < f; ++z)
            for (int y = 0; y < f; ++y) {
                const uint64_t row = ((uint64_t)(iz * f + z) * ny + (iy * f + y)) * nx + (uint64_t)ix * f;
                for (int x = 0; x < f; ++x) out[row + x] = (uint32_t)s;
            }
    }
}

__device__ inline void lerp_index(int i, int f, int n_c, int& i0, int& i1, double& t) {
    double x = (i + 0.5) / f - 0.5;
    x = fmin(fmax(x, 0.0), (double)(n_c - 1));
    i0 = (int)floor(x);
    i1 = min(i0 + 1, n_c - 1);
    t = x - i0;
}

// one thread per normal pixel of every plane
__global__ __launch_bounds__(256) void k_expand(const int64_t* __restrict__ coarse, uint64_t n_planes,
                                                int nu_c, int nv_c, int f, double user_scale,
                                                double* __restrict__ out) {
    const int nu = nu_c * f, nv = nv_c * f;
    const uint64_t n = n_planes * (uint64_t)nu * nv;
    const double scale = user_scale / (4294967296.0 * f * f);
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
         o += (uint64_t)gridDim.x * blockDim.x) {
        const int i = (int)(o % nu), j = (int)((o / nu) % nv);
        const uint64_t plane = o / ((uint64_t)nu * nv);
        int i0, i1, j0, j1;
        double tx, ty;
        lerp_index(i, f, nu_c, i0, i1, tx);
        lerp_index(j, f, nv_c, j0, j1, ty);
        const int64_t* c = coarse + plane * (uint64_t)nu_c * nv_c;
        const double c00 = (double)c[(uint64_t)j0 * nu_c + i0], c01 = (double)c[(uint64_t)j0 * nu_c + i1];
        const double c10 = (double)c[(uint64_t)j1 * nu_c + i0], c11 = (double)c[(uint64_t)j1 * nu_c + i1];
        out[o] = ((1.0 - ty) * ((1.0 - tx) * c00 + tx * c01) + ty * ((1.0 - tx) * c10 + tx * c11)) * scale;
    }
}

int grid_for_n(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

}  // namespace

hipError_t launch_block_activity(const uint32_t* act, int nx, int ny, int nz, int f, uint32_t* out,
                                 int64_t* status, hipStream_t s) {
    const uint64_t nb = (uint64_t)(nx / f) * (ny / f) * (nz / f);
    k_block_activity<<<grid_for_n(nb), 256, 0, s>>>(act, nx, ny, nz, f, out, status);
    return hipGetLastError();
}

hipError_t launch_expand(const int64_t* coarse, uint64_t n_planes, int nu_c, int nv_c, int f, double scale,
                         double* out, hipStream_t s) {
    const uint64_t n = n_planes * (uint64_t)nu_c * f * nv_c * f;
    k_expand<<<grid_for_n(n), 256, 0, s>>>(coarse, n_planes, nu_c, nv_c, f, scale, out);
    return hipGetLastError();
}

}  // namespace mcs
