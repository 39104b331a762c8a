// Adjoint of the projection tallies with respect to the 140 keV attenuation map.
//
// A tallied history sampled at mu0 is a path: emission point, Compton vertices,
// final flight out of the grid.  Under a change of mu its probability density
// changes by the factor
//     W_h(mu) = prod_{Compton vertices c} mu_{v_c}/mu0_{v_c}
//               * exp(-sum_v (mu_v - mu0_v) * lt_{h,v}),
//     lt_{h,v} = sum over segments of g(E_seg) * (length of the segment in v),
// (materials are density-scaled water, so the scatter and branch probabilities
// at a vertex do not depend on the magnitude of mu and cancel).  Hence
//     dL/dmu_v = sum_h G_{b(h)} * (c_{h,v}/mu0_v - lt_{h,v}),
// with G = dL/dtally.  The kernels here replay each tallied history from its
// Philox counter -- no path is stored -- and walk every segment voxel by voxel
// (Amanatides & Woo 1987 grid traversal), adding -G g(E) len to each crossed
// voxel and +G/mu0 at each Compton vertex.  A tallied history is replayed by
// a whole wavefront (every lane the same path), and each segment is cut into
// 64 equal pieces, one per lane, so a long walk is not one lane's serial
// chain.  Sums are 64-bit fixed point with frac_bits fractional bits:
// integer atomics, so the result is bit-exact from run to run and does not
// depend on the order of the additions.
#include <algorithm>

#include "history.h"

namespace mcs {
namespace {

__device__ inline void add_fixed(long long* grad, uint32_t v, double val, double scale,
                                 int64_t* status) {
    const double s = val * scale;
    if (!(fabs(s) < 4.0e18)) {
        atomicOr((unsigned long long*)status, (unsigned long long)MC_STATUS_GRAD_OVERFLOW);
        return;
    }
    atomicAdd((unsigned long long*)(grad + v), (unsigned long long)__double2ll_rn(s));
}

// Walk the ray a + t d over t in [t0, t1), adding w * (length in voxel) to
// every voxel the piece crosses; the piece starts in the voxel holding
// a + t0 d (clamped to the grid) and stops at t1 or at the grid edge.  The
// path itself (vertices, directions) is the FP32 replay's; the walk along it
// is in double precision, with every plane crossing computed from its plane
// index (t = (plane - p) / d) rather than accumulated step by step, so the
// lengths carry no error beyond that of the FP32 vertices.
__device__ void walk_piece(const Cst& C, double ax, double ay, double az, double dx, double dy,
                           double dz, double t0, double t1, double w, long long* grad, double scale,
                           int64_t* status) {
    if (!(t1 > t0)) return;
    const double vox = (double)C.vox;
    const double px = fma(t0, dx, ax) + (double)C.hx, py = fma(t0, dy, ay) + (double)C.hy,
                 pz = fma(t0, dz, az) + (double)C.hz;
    int ix = min(max((int)floor(px / vox), 0), C.nx - 1);
    int iy = min(max((int)floor(py / vox), 0), C.ny - 1);
    int iz = min(max((int)floor(pz / vox), 0), C.nz - 1);
    const int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1, sz = dz > 0.0 ? 1 : -1;
    const int ox = dx > 0.0 ? 1 : 0, oy = dy > 0.0 ? 1 : 0, oz = dz > 0.0 ? 1 : 0;
    const double inf = __builtin_huge_val();
    const double idx = dx != 0.0 ? 1.0 / dx : inf, idy = dy != 0.0 ? 1.0 / dy : inf,
                 idz = dz != 0.0 ? 1.0 / dz : inf;
    // parametric distance (from t0) to the next plane on each axis
    auto plane_t = [&](int i, int o, double p, double id, double d) {
        return d != 0.0 ? fmax(((double)(i + o) * vox - p) * id, 0.0) : inf;
    };
    double tx = plane_t(ix, ox, px, idx, dx), ty = plane_t(iy, oy, py, idy, dy),
           tz = plane_t(iz, oz, pz, idz, dz);
    const double t_end = t1 - t0;
    double t = 0.0;
    const int max_iter = C.nx + C.ny + C.nz + 3;
    for (int it = 0; it < max_iter; ++it) {
        const double tn = fmin(tx, fmin(ty, tz));
        const double te = fmin(tn, t_end);
        const uint32_t v = (uint32_t)ix + (uint32_t)C.nx * ((uint32_t)iy + (uint32_t)C.ny * (uint32_t)iz);
        if (te > t) add_fixed(grad, v, w * (te - t), scale, status);
        if (tn >= t_end) return;
        t = tn;
        if (tx <= ty && tx <= tz) {
            ix += sx;
            if (ix < 0 || ix >= C.nx) return;
            tx = plane_t(ix, ox, px, idx, dx);
        } else if (ty <= tz) {
            iy += sy;
            if (iy < 0 || iy >= C.ny) return;
            ty = plane_t(iy, oy, py, idy, dy);
        } else {
            iz += sz;
            if (iz < 0 || iz >= C.nz) return;
            tz = plane_t(iz, oz, pz, idz, dz);
        }
    }
}

// Walk the ray a + t d, t in [0, t_end) (t_end = +inf: to the grid exit), by
// the whole wavefront: the range is cut into 64 equal pieces, lane k walks
// piece k.  Every lane must call it with the same arguments.
__device__ void walk_wave(const Cst& C, double ax, double ay, double az, double dx, double dy,
                          double dz, double t_end, double w, long long* grad, double scale,
                          int64_t* status) {
    const double inf = __builtin_huge_val();
    const double px = ax + (double)C.hx, py = ay + (double)C.hy, pz = az + (double)C.hz;
    const double ex = dx > 0.0 ? ((double)C.lx - px) / dx : (dx < 0.0 ? -px / dx : inf);
    const double ey = dy > 0.0 ? ((double)C.ly - py) / dy : (dy < 0.0 ? -py / dy : inf);
    const double ez = dz > 0.0 ? ((double)C.lz - pz) / dz : (dz < 0.0 ? -pz / dz : inf);
    const double len = fmin(t_end, fmax(fmin(ex, fmin(ey, ez)), 0.0));
    const int lane = threadIdx.x & 63;
    const double piece = len * (1.0 / 64.0);
    const double t0 = (double)lane * piece;
    const double t1 = lane == 63 ? len : (double)(lane + 1) * piece;
    walk_piece(C, ax, ay, az, dx, dy, dz, t0, t1, w, grad, scale, status);
}

__device__ inline double g_of(const Cst& C, float e) {
    if (e == C.e0) return (double)C.g0;
    float a, b;
    return (double)energy_terms(C, e, a, b);
}

// Replay one history; if it ends TALLIED in `bin`, walk its path with weight G.
// walk_now = false: only report the fate/bin (first pass of replay-all mode);
// walk_now = true: every lane of the wavefront replays the same history (the
// walks are shared by the lanes).
__device__ int replay_path(const Cst& C, uint64_t hist, int view, bool walk_now, double G,
                           long long* grad, double scale, int64_t* status, uint32_t& bin_out) {
    Lane L;
    const Emission em = emit_history(C, (uint32_t)hist, (uint32_t)view);
    begin_history(C, L, (uint32_t)view, (uint32_t)hist, em);
    Acc A;
    acc_zero(A);
    double sx = L.x, sy = L.y, sz = L.z;   // start of the current segment
    for (;;) {
        uint32_t c0 = (uint32_t)L.hist, c1 = (uint32_t)L.view, c2, c3;
        counter_of(L, c2, c3);
        philox10(c0, c1, c2, c3, C.seed, C.pid);
        const int before = L.state;
        const float e_flight = L.e;
        int iu = -1, iv = -1;
        const int fate = advance(C, C.pal, L, c0, c1, c2, c3, A, iu, iv);
        if (fate == R_RUNNING) {
            if (walk_now && before == S_STEP && L.state == S_KAHN) {
                // Compton vertex at L.x: close the segment (its direction is
                // still the one it was flown in), add the collision term
                const double ex = (double)L.x - sx, ey = (double)L.y - sy, ez = (double)L.z - sz;
                const double len = ex * L.dx + ey * L.dy + ez * L.dz;
                walk_wave(C, sx, sy, sz, L.dx, L.dy, L.dz, len, -G * g_of(C, e_flight), grad, scale, status);
                if ((threadIdx.x & 63) == 0) {
                    const int ix = min((int)((L.x + C.hx) * C.inv_vox), C.nx - 1);
                    const int iy = min((int)((L.y + C.hy) * C.inv_vox), C.ny - 1);
                    const int iz = min((int)((L.z + C.hz) * C.inv_vox), C.nz - 1);
                    const uint32_t v = (uint32_t)ix + (uint32_t)C.nx * ((uint32_t)iy + (uint32_t)C.ny * (uint32_t)iz);
                    add_fixed(grad, v, G / (double)ldg(C.mu + v), scale, status);
                }
                sx = L.x; sy = L.y; sz = L.z;
            }
            continue;
        }
        if (fate == MC_TALLIED) {
            const int cls = L.n_scatter > 0 ? 1 : 0;
            bin_out = (uint32_t)((((uint32_t)L.view * 2u + cls) * (uint32_t)C.nv + iv) * (uint32_t)C.nu + iu);
            if (walk_now)
                walk_wave(C, sx, sy, sz, L.dx, L.dy, L.dz, __builtin_huge_val(), -G * g_of(C, L.e),
                          grad, scale, status);
        }
        return fate;
    }
}

// One listed tallied history per wavefront (grid-strided over the list).
__global__ __launch_bounds__(256) void k_adjoint_events(const ProbDesc* __restrict__ d,
                                                        const mc_event* __restrict__ events,
                                                        const unsigned long long* __restrict__ n_events,
                                                        uint64_t capacity, const double* __restrict__ dL,
                                                        long long* grad, double scale, int64_t* status) {
    const uint64_t n = min((uint64_t)*n_events, capacity);
    const Cst C = load_cst(d);
    if (C.flags) return;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const bool lead = (threadIdx.x & 63) == 0;
    for (uint64_t i = wave; i < n; i += n_waves) {
        const mc_event ev = events[i];
        if (ev.work >= d->work_count) {
            if (lead) atomicOr((unsigned long long*)status, (unsigned long long)MC_STATUS_BAD_EVENT);
            continue;
        }
        const double G = dL[C.tally_offset + ev.bin];
        if (G == 0.0) continue;
        uint64_t view, hist;
        split_work(C, C.work_begin + ev.work, view, hist);
        uint32_t bin = 0;
        const int fate = replay_path(C, hist, (int)view, true, G, grad, scale, status, bin);
        if (lead && (fate != MC_TALLIED || bin != ev.bin))
            atomicOr((unsigned long long*)status, (unsigned long long)MC_STATUS_BAD_EVENT);
    }
}

// Every history of the call's range: each lane replays its own to find the
// tallied ones, then the wavefront walks each of those together.
__global__ __launch_bounds__(256) void k_adjoint_all(const ProbDesc* __restrict__ d,
                                                     const double* __restrict__ dL, long long* grad,
                                                     double scale, int64_t* status) {
    const Cst C = load_cst(d);
    if (C.flags) return;
    const uint64_t cnt = d->work_count;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // wave-uniform loop bound: every lane stays for the shared walks
    const uint64_t first = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    for (uint64_t i0 = first; i0 < cnt; i0 += stride) {
        const uint64_t i = i0 + (threadIdx.x & 63);
        uint64_t view = 0, hist = 0;
        double G = 0.0;
        bool walk_it = false;
        if (i < cnt) {
            split_work(C, C.work_begin + i, view, hist);
            uint32_t bin = 0;
            const int fate = replay_path(C, hist, (int)view, false, 0.0, grad, scale, status, bin);
            if (fate == MC_TALLIED) {
                G = dL[C.tally_offset + bin];
                walk_it = G != 0.0;
            }
        }
        for (uint64_t m = __ballot(walk_it); m != 0; m &= m - 1) {
            const int src = __ffsll((unsigned long long)m) - 1;
            const uint64_t h = (uint64_t)__shfl((long long)hist, src, 64);
            const int v = __shfl((int)view, src, 64);
            const double g = __shfl(G, src, 64);
            uint32_t bin = 0;
            replay_path(C, h, v, true, g, grad, scale, status, bin);
        }
    }
}

__global__ __launch_bounds__(256) void k_zero_grad(long long* grad, uint64_t n, int64_t* status) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = tid; i < n; i += (uint64_t)gridDim.x * blockDim.x) grad[i] = 0;
    if (tid < 4) status[tid] = 0;
}

__global__ void k_adjoint_finalize(const ProbDesc* __restrict__ d, int64_t* status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) status[0] |= (int64_t)d->flags;
}

}  // namespace

hipError_t launch_adjoint(const ProbDesc* d, const mc_event* events, const uint64_t* n_events,
                          uint64_t capacity, const double* dL, int64_t* grad, uint64_t nvox,
                          int frac_bits, int64_t* status, int n_cu, hipStream_t s) {
    uint64_t gz = (nvox + 255) / 256;
    if (gz > 4096) gz = 4096;
    if (gz < 1) gz = 1;
    k_zero_grad<<<(int)gz, 256, 0, s>>>((long long*)grad, nvox, status);
    const double scale = ldexp(1.0, frac_bits);
    if (events) {
        if (capacity > 0) {
            // one wavefront per listed history, at most n_cu * 32 wavefronts (grid-strided)
            const uint64_t waves = std::min<uint64_t>(capacity, (uint64_t)n_cu * 32);
            k_adjoint_events<<<(int)((waves + 3) / 4), 256, 0, s>>>(
                d, events, (const unsigned long long*)n_events, capacity, dL, (long long*)grad, scale,
                status);
        }
    } else {
        k_adjoint_all<<<n_cu * 8, 256, 0, s>>>(d, dL, (long long*)grad, scale, status);
    }
    k_adjoint_finalize<<<1, 64, 0, s>>>(d, status);
    return hipGetLastError();
}

}  // namespace mcs
