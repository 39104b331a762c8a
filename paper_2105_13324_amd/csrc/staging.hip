// Input staging: from the caller's attenuation and activity maps to the tables
// the transport kernels read.
//
//  * max mu, input validation and the activity total (one reduction pass);
//  * accept thresholds Q_v = ceil(mu_v 2^24 / max mu) in double precision, so
//    the real/virtual decision of Woodcock tracking is an exact integer compare;
//  * the inclusive prefix sum of activity (uint64) and a guide table over its
//    high bits, so that an emission voxel is found with one gather and a short
//    binary search (Chen & Asau 1974 guide tables; same result as a plain
//    inverse-CDF search);
//  * (cos, sin) of each view angle.
//
// Every pass streams the grid once with coalesced loads; the whole staging of
// a 128^3 phantom moves ~40 MB and is far below the transport cost.
#include "mc_internal.h"

namespace mcs {
namespace {

constexpr int RED_THREADS = 256;

__device__ inline uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ inline uint32_t wave_or_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o, 64);
    return v;
}

__global__ void k_write_desc(ProbDesc d, ProbDesc* out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = d;
}

// Max mu (as bits: order-preserving for non-negative floats), bad-value flags,
// activity total, view table.
__global__ __launch_bounds__(RED_THREADS) void k_reduce(ProbDesc* pd) {
    const uint64_t nvox = pd->nvox;
    const float* __restrict__ mu = pd->mu;
    const uint32_t* __restrict__ act = pd->act;
    uint32_t mx = 0, flags = 0;
    uint64_t sum = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float m = mu[i];
        if (!(m >= 0.0f) || !isfinite(m)) flags |= MC_STATUS_BAD_MU;
        else if (m > 0.0f) mx = max(mx, __float_as_uint(m));
        sum += act[i];
    }
    mx = wave_max_u32(mx);
    flags = wave_or_u32(flags);
    sum = wave_sum_u64(sum);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&pd->mu_hat_bits, mx);
        if (flags) atomicOr(&pd->flags, flags);
        atomicAdd((unsigned long long*)&pd->total, (unsigned long long)sum);
    }
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < pd->n_views; k += blockDim.x) {
            const double a = pd->angles[k];
            if (!isfinite(a)) atomicOr(&pd->flags, (uint32_t)MC_STATUS_BAD_ANGLE);
            pd->views[k] = make_float2((float)cos(a), (float)sin(a));
        }
    }
}

// Q_v in double precision: mu_v * 2^24 is exact, the division is correctly
// rounded, ceil is exact.
__global__ __launch_bounds__(RED_THREADS) void k_thresholds(ProbDesc* pd) {
    const uint64_t nvox = pd->nvox;
    const float mu_hat = __uint_as_float(pd->mu_hat_bits);
    const float* __restrict__ mu = pd->mu;
    uint32_t* __restrict__ q = pd->q32;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float m = mu[i];
        uint32_t v = 0;
        if (mu_hat > 0.0f && m > 0.0f) {
            double t = ceil((double)m * 16777216.0 / (double)mu_hat);
            v = t >= 16777216.0 ? 16777216u : (uint32_t)t;
        }
        q[i] = v;
    }
}

// --- three-pass inclusive scan of the activity map (uint64) ---

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(ProbDesc* pd) {
    const uint64_t nvox = pd->nvox;
    const uint32_t* __restrict__ act = pd->act;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
    for (int j = threadIdx.x; j < SCAN_ITEMS; j += SCAN_THREADS) {
        const uint64_t i = base + j;
        if (i < nvox) s += act[i];
    }
    s = wave_sum_u64(s);
    __shared__ uint64_t part[SCAN_THREADS / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) t += part[w];
        pd->block_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of the block sums, one block of 1024 threads, each thread a
// contiguous run.
__global__ __launch_bounds__(1024) void k_scan_top(ProbDesc* pd, int n_blocks) {
    __shared__ uint64_t tot[1024];
    uint64_t* __restrict__ bs = pd->block_sums;
    const int per = (n_blocks + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint64_t s = 0;
    for (int j = 0; j < per; ++j) if (b0 + j < n_blocks) s += bs[b0 + j];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = tot[threadIdx.x] - s;  // exclusive prefix of this thread's run
    for (int j = 0; j < per; ++j) {
        if (b0 + j < n_blocks) {
            const uint64_t v = bs[b0 + j];
            bs[b0 + j] = run;
            run += v;
        }
    }
}

// Per block: 16 consecutive items per thread, thread-local inclusive scan,
// block exclusive scan of thread totals, plus the block's offset.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_final(ProbDesc* pd) {
    constexpr int PER = SCAN_ITEMS / SCAN_THREADS;
    const uint64_t nvox = pd->nvox;
    const uint32_t* __restrict__ act = pd->act;
    uint64_t* __restrict__ cdf = pd->cdf;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_ITEMS + (uint64_t)threadIdx.x * PER;
    uint64_t v[PER];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t i = base + j;
        s += (i < nvox) ? act[i] : 0u;
        v[j] = s;
    }
    __shared__ uint64_t tot[SCAN_THREADS];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    const uint64_t off = pd->block_sums[blockIdx.x] + tot[threadIdx.x] - s;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t i = base + j;
        if (i < nvox) cdf[i] = off + v[j];
    }
}

// Guide table: bucket b covers t in [b 2^s, (b+1) 2^s); guide[b] is the first
// voxel whose cumulative activity exceeds b 2^s, guide[B] the last voxel.  The
// answer for any t in bucket b lies in [guide[b], guide[b+1]].
__global__ __launch_bounds__(RED_THREADS) void k_guide(ProbDesc* pd, uint64_t nb_cap) {
    const uint64_t total = pd->total;
    const uint64_t nvox = pd->nvox;
    if (total == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&pd->flags, (uint32_t)MC_STATUS_NO_ACTIVITY);
        return;
    }
    uint32_t s = 0;
    while (((total - 1) >> s) >= nb_cap) ++s;
    const uint64_t B = ((total - 1) >> s) + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        pd->shift = s;
        pd->n_buckets = (uint32_t)B;
    }
    const uint64_t* __restrict__ cdf = pd->cdf;
    uint32_t* __restrict__ guide = pd->guide;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= B;
         b += (uint64_t)gridDim.x * blockDim.x) {
        if (b == B) { guide[b] = (uint32_t)(nvox - 1); continue; }
        const uint64_t key = b << s;
        uint64_t lo = 0, hi = nvox - 1;   // first i with cdf[i] > key; cdf[nvox-1] = total > key
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (cdf[mid] > key) hi = mid; else lo = mid + 1;
        }
        guide[b] = (uint32_t)lo;
    }
}

int grid_for(uint64_t n, int threads, int cap) {
    uint64_t g = (n + threads - 1) / threads;
    if (g > (uint64_t)cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

uint64_t guide_capacity(uint64_t nvox) {
    uint64_t c = 1;
    while (c < nvox) c <<= 1;
    return c;
}

hipError_t launch_staging(ProbDesc* d, const ProbDesc& h, hipStream_t st) {
    const uint64_t nvox = h.nvox;
    k_write_desc<<<1, 64, 0, st>>>(h, d);
    k_reduce<<<grid_for(nvox, RED_THREADS, 2048), RED_THREADS, 0, st>>>(d);
    k_thresholds<<<grid_for(nvox, RED_THREADS, 8192), RED_THREADS, 0, st>>>(d);
    const int nb = (int)((nvox + SCAN_ITEMS - 1) / SCAN_ITEMS);
    k_scan_sums<<<nb, SCAN_THREADS, 0, st>>>(d);
    k_scan_top<<<1, 1024, 0, st>>>(d, nb);
    k_scan_final<<<nb, SCAN_THREADS, 0, st>>>(d);
    const uint64_t cap = guide_capacity(nvox);
    k_guide<<<grid_for(cap + 1, RED_THREADS, 8192), RED_THREADS, 0, st>>>(d, cap);
    return hipGetLastError();
}

}  // namespace mcs
