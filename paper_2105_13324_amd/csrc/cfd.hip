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

// One block per CFD_TILE x CFD_TILE output tile of one (view, class): for
// each layer the block stages the tile and its halo of half-width h in LDS,
// then every thread adds its output's (2h + 1)^2 products.  The response
// values are wave-uniform loads.
__global__ __launch_bounds__(256) void k_cfd_convolve(const ProbDesc* __restrict__ pd, int64_t* tally) {
    constexpr int W_MAX = CFD_TILE + 2 * CFD_MAX_H;
    __shared__ double tile[W_MAX * W_MAX];
    const int nu = pd->nu, nv = pd->nv, L = pd->cfd_L;
    const int tu = (nu + CFD_TILE - 1) / CFD_TILE, tv = (nv + CFD_TILE - 1) / CFD_TILE;
    uint64_t b = blockIdx.x;
    const int bu = (int)(b % tu); b /= tu;
    const int bv = (int)(b % tv); b /= tv;
    const uint64_t vc = b;                       // view * 2 + class
    const uint64_t view = vc >> 1, cls = vc & 1;
    const int lu = (int)threadIdx.x % CFD_TILE, lv = (int)threadIdx.x / CFD_TILE;
    const int u0 = bu * CFD_TILE, v0 = bv * CFD_TILE;
    const int64_t* __restrict__ lay = pd->layers;
    const double* __restrict__ kern = pd->cfd_kern;
    const uint32_t* __restrict__ hl = pd->cfd_h;
    const int nmax = 2 * pd->cfd_hmax + 1;
    double acc = 0.0;
    for (int l = 0; l < L; ++l) {
        const int h = (int)hl[l], n = 2 * h + 1, w = CFD_TILE + 2 * h;
        const int64_t* base = lay + ((view * L + l) * 2 + cls) * (uint64_t)nv * nu;
        __syncthreads();                         // the previous layer's reads are done
        for (int i = threadIdx.x; i < w * w; i += blockDim.x) {
            const int iv = v0 - h + i / w, iu = u0 - h + i % w;
            tile[i] = (iv >= 0 && iv < nv && iu >= 0 && iu < nu) ? (double)base[(uint64_t)iv * nu + iu]
                                                                   : 0.0;
        }
        __syncthreads();
        // output (v, u) takes layer (v - b, u - a) times response (b, a);
        // that layer value sits at tile row lv + 2h - (b + h)
        const double* k = kern + (uint64_t)l * nmax * nmax;
        for (int bb = 0; bb < n; ++bb) {
            const double* row = tile + (lv + 2 * h - bb) * w + lu + 2 * h;
            for (int aa = 0; aa < n; ++aa) acc = fma(row[-aa], k[bb * n + aa], acc);
        }
    }
    const int ou = u0 + lu, ov = v0 + lv;
    if (ou < nu && ov < nv)
        tally[pd->tally_offset + (vc * nv + ov) * (uint64_t)nu + ou] = (int64_t)llrint(acc);
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
    k_cfd_convolve<<<(unsigned)tiles, CFD_TILE * CFD_TILE, 0, s>>>(d, tally);
    return hipGetLastError();
}

}  // namespace mcs
