// Convolution-based forced detection (CFD, paper Sec. 5.2): the collimator
// response of each depth layer, and the convolution of the sub-projection
// layers into the projection tally.
//
// A forced copy travels perpendicular to the detector and is stored, with
// its weight, in the layer of its depth (one pixel thick) at the pixel of its
// perpendicular hit (transport kernel).  The ideal cone collimator spreads a
// point at depth d over a disk of radius d tan(alpha) with plane density
// d / (2 pi (1 - cos alpha) (d^2 + r^2)^(3/2)) (directions uniform in the
// cone); integrated over each pixel (CFD_SUB^2 midpoint samples) and
// normalised, that is layer l's response at its centre depth.  The projection
// is the sum over layers of the layer convolved with its response, in FP64
// on the Q31.32 deposits, rounded once into the Q31.32 tally.
#include "mc_internal.h"

namespace mcs {
namespace {

constexpr double PI_D = 3.14159265358979323846;

__global__ __launch_bounds__(256) void k_cfd_half_widths(ProbDesc* pd) {
    for (int l = threadIdx.x; l < pd->cfd_L; l += blockDim.x)
        pd->cfd_h[l] = (uint32_t)min(cfd_half_width((l + 0.5) * pd->cfd_pix, pd->cfd_tan, pd->cfd_pix),
                                     pd->cfd_hmax);
}

// one block per layer; runs after k_cfd_half_widths
__global__ __launch_bounds__(256) void k_cfd_kernels(ProbDesc* pd) {
    const int l = blockIdx.x;
    if (l >= pd->cfd_L) return;
    const double pix = pd->cfd_pix, a = pd->alpha;
    const double d = (l + 0.5) * pix, rho = d * pd->cfd_tan, omc = 2.0 * sin(0.5 * a) * sin(0.5 * a);
    const int h = (int)pd->cfd_h[l], n = 2 * h + 1, nmax = 2 * pd->cfd_hmax + 1;
    double* k = pd->cfd_kern + (uint64_t)l * nmax * nmax;
    double part = 0.0;
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int b = idx / n - h, c = idx % n - h;
        double acc = 0.0;
        for (int t = 0; t < CFD_SUB; ++t)
            for (int u = 0; u < CFD_SUB; ++u) {
                const double x = (c + (u + 0.5) / CFD_SUB - 0.5) * pix;
                const double y = (b + (t + 0.5) / CFD_SUB - 0.5) * pix;
                const double r2 = x * x + y * y;
                if (r2 > rho * rho) continue;
                const double q = d * d + r2;
                acc += d / (2.0 * PI_D * omc * q * sqrt(q));
            }
        acc *= (pix / CFD_SUB) * (pix / CFD_SUB);
        k[idx] = acc;
        part += acc;
    }
    __shared__ double red[256];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double tot = red[0];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x)
        k[idx] = tot > 0.0 ? k[idx] / tot : (idx == h * n + h ? 1.0 : 0.0);
}

__global__ __launch_bounds__(256) void k_fill_i64(int64_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// One block (CFD_TILE^2 threads) per CFD_TILE x CFD_TILE output tile of one
// (view, class).  For each layer the block stages the tile with its halo of
// half-width h and the layer's response in LDS (sized at launch for the
// largest h), then every thread adds its output's (2h + 1)^2 products.  The
// next layer's values are loaded into registers while the current one is
// convolved, and a layer whose tile and halo are all zero is skipped (its
// products are exact zeros, so the sum is the same).  The responses are even
// in both offsets, so only their (b >= 0, a >= 0) quadrant is read.
// HMAX: the largest half-width the instance handles (sizes the prefetch).
constexpr int CFD_THREADS = CFD_TILE * CFD_TILE;
constexpr int CFD_SMALL_H = 8;

template <int HMAX>
__device__ __forceinline__ void cfd_convolve_body(const ProbDesc* __restrict__ pd, int64_t* tally) {
    constexpr int CFD_PF = ((CFD_TILE + 2 * HMAX) * (CFD_TILE + 2 * HMAX) + CFD_THREADS - 1) / CFD_THREADS;
    constexpr int CFD_KPF = ((2 * HMAX + 1) * (2 * HMAX + 1) + CFD_THREADS - 1) / CFD_THREADS;
    extern __shared__ double smem[];
    const int nu = pd->nu, nv = pd->nv, L = pd->cfd_L;
    const int hmax = pd->cfd_hmax, nmax = 2 * hmax + 1, wmax = CFD_TILE + 2 * hmax;
    double* tile = smem;                      // [wmax * wmax]
    double* kt = smem + wmax * wmax;          // [nmax * nmax]
    const int tu = (nu + CFD_TILE - 1) / CFD_TILE, tv = (nv + CFD_TILE - 1) / CFD_TILE;
    uint64_t b = blockIdx.x;
    const int bu = (int)(b % tu); b /= tu;
    const int bv = (int)(b % tv); b /= tv;
    const uint64_t vc = b;                       // view * 2 + class
    const uint64_t view = vc >> 1, cls = vc & 1;
    const int tid = (int)threadIdx.x;
    const int lu = tid % CFD_TILE, lv = tid / CFD_TILE;
    const int u0 = bu * CFD_TILE, v0 = bv * CFD_TILE;
    const int64_t* __restrict__ lay = pd->layers;
    const double* __restrict__ kern = pd->cfd_kern;
    const uint32_t* __restrict__ hl = pd->cfd_h;
    int64_t nx[CFD_PF];
    double kx[CFD_KPF];
    auto fetch = [&](int l, int h) {
        const int w = CFD_TILE + 2 * h, n = 2 * h + 1;
        const int64_t* base = lay + ((view * L + l) * 2 + cls) * (uint64_t)nv * nu;
        const double* kl = kern + (uint64_t)l * nmax * nmax;
#pragma unroll
        for (int k = 0; k < CFD_PF; ++k) {
            const int i = tid + k * CFD_THREADS;
            int64_t v = 0;
            if (i < w * w) {
                const int iv = v0 - h + i / w, iu = u0 - h + i % w;
                if (iv >= 0 && iv < nv && iu >= 0 && iu < nu) v = base[(uint64_t)iv * nu + iu];
            }
            nx[k] = v;
        }
#pragma unroll
        for (int k = 0; k < CFD_KPF; ++k) {
            const int i = tid + k * CFD_THREADS;
            kx[k] = i < n * n ? kl[i] : 0.0;
        }
    };
    int h_next = (int)hl[0];
    fetch(0, h_next);
    double acc = 0.0;
    for (int l = 0; l < L; ++l) {
        const int h = h_next, n = 2 * h + 1, w = CFD_TILE + 2 * h;
        __syncthreads();                         // the previous layer's reads are done
        bool any = false;
#pragma unroll
        for (int k = 0; k < CFD_PF; ++k) {
            const int i = tid + k * CFD_THREADS;
            if (i < w * w) {
                tile[i] = (double)nx[k];
                any |= nx[k] != 0;
            }
        }
#pragma unroll
        for (int k = 0; k < CFD_KPF; ++k) {
            const int i = tid + k * CFD_THREADS;
            if (i < n * n) kt[i] = kx[k];
        }
        if (l + 1 < L) {
            h_next = (int)hl[l + 1];
            fetch(l + 1, h_next);
        }
        if (!__syncthreads_or(any)) continue;
        // output (v, u) takes layer (v - b, u - a) times response (b, a).
        // The response is even in a and in b (the pixel samples are placed
        // symmetrically; the table is so up to rounding), so the four layer
        // values of (+-b, +-a) share one product.  Layer value (v - b, u - a) sits at tile row lv + h - b,
        // column lu + h - a.
        const double* c = tile + (lv + h) * w + lu + h;
        for (int bb = 0; bb <= h; ++bb) {
            const double* up = c - bb * w;
            const double* dn = c + bb * w;
            const double* kr = kt + (bb + h) * n + h;
            double s0 = bb ? up[0] + dn[0] : up[0];
            acc = fma(s0, kr[0], acc);
#pragma unroll 4
            for (int aa = 1; aa <= h; ++aa) {
                const double s = bb ? (up[-aa] + up[aa]) + (dn[-aa] + dn[aa]) : up[-aa] + up[aa];
                acc = fma(s, kr[aa], acc);
            }
        }
    }
    const int ou = u0 + lu, ov = v0 + lv;
    if (ou < nu && ov < nv)
        tally[pd->tally_offset + (vc * nv + ov) * (uint64_t)nu + ou] = (int64_t)llrint(acc);
}

// small responses: at most 64 VGPRs, so a CU holds 8 blocks
__global__ __launch_bounds__(CFD_THREADS) __attribute__((amdgpu_waves_per_eu(8)))
void k_cfd_convolve_small(const ProbDesc* __restrict__ pd, int64_t* tally) {
    cfd_convolve_body<CFD_SMALL_H>(pd, tally);
}

__global__ __launch_bounds__(CFD_THREADS) void k_cfd_convolve(const ProbDesc* __restrict__ pd, int64_t* tally) {
    cfd_convolve_body<CFD_MAX_H>(pd, tally);
}

int grid_cap(uint64_t n, int cap) {
    uint64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_cfd_setup(ProbDesc* d, const ProbDesc& h, hipStream_t s) {
    const uint64_t n_lay = (uint64_t)h.n_views * h.cfd_L * 2 * h.nv * h.nu;
    k_fill_i64<<<grid_cap(n_lay, 8192), 256, 0, s>>>(h.layers, n_lay);
    k_cfd_half_widths<<<1, 256, 0, s>>>(d);
    k_cfd_kernels<<<h.cfd_L, 256, 0, s>>>(d);
    return hipGetLastError();
}

hipError_t launch_cfd_convolve(const ProbDesc* d, const ProbDesc& h, int64_t* tally, hipStream_t s) {
    const uint64_t tiles = (uint64_t)h.n_views * 2 * ((h.nv + CFD_TILE - 1) / CFD_TILE) *
                           ((h.nu + CFD_TILE - 1) / CFD_TILE);
    const size_t w = CFD_TILE + 2 * (size_t)h.cfd_hmax, m = 2 * (size_t)h.cfd_hmax + 1;
    const size_t lds = 8 * (w * w + m * m);     // at most 51 KB (half-width 24)
    if (h.cfd_hmax <= CFD_SMALL_H)
        k_cfd_convolve_small<<<(unsigned)tiles, CFD_THREADS, lds, s>>>(d, tally);
    else
        k_cfd_convolve<<<(unsigned)tiles, CFD_THREADS, lds, s>>>(d, tally);
    return hipGetLastError();
}

}  // namespace mcs
