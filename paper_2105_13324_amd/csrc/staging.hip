// Input staging: from the caller's attenuation and activity maps to the tables
// the transport kernels read.
//
//  * max mu, input validation, the activity total and the attenuation box
//    (the voxel index range of mu > 0) in one reduction pass;
//  * accept thresholds Q_v = ceil(mu_v 2^24 / max mu) in double precision, so
//    the real/virtual decision of Woodcock tracking is an exact integer compare;
//    when the map has at most 256 distinct thresholds (segmented phantoms have
//    a handful) also one-byte codes into a palette of them, a table a quarter
//    the size that stays in L2;
//  * the runs of the activity map (maximal stretches of a grid row with one
//    weight), each with the cumulative activity before it (uint64), and a
//    table of buckets over the high bits of that sum with about two buckets
//    per run (after the guide tables of Chen & Asau 1974): an emission voxel
//    is one 8-byte bucket gather, one 16-byte run gather and a division
//    within the run, rarely a short search over runs -- the same voxel as a
//    plain inverse-CDF search over all voxels.  A segmented phantom has ~1e4
//    runs, so both tables stay in L2;
//  * (cos, sin) of each view angle;
//  * the Klein-Nishina attenuation shape sigma_KN(E)/sigma_KN(140) at 1/4 keV
//    steps, evaluated in double precision.
//
// Every pass streams the grid once with coalesced loads; the whole staging of
// a 128^3 phantom moves ~40 MB and is far below the transport cost.
#include <algorithm>

#include "mc_internal.h"

namespace mcs {
namespace {

constexpr int RED_THREADS = 256;
constexpr int ROWS = 4;        // grid rows a row pass loads at once
constexpr int REDUCE_BLOCKS = 512;      // most workgroups of k_reduce per problem
constexpr int REDUCE_PART_U64 = 4;      // partial results per workgroup

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
__global__ __launch_bounds__(RED_THREADS) void k_reduce(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const uint64_t nvox = pd->nvox;
    const float* __restrict__ mu = pd->mu;
    const uint32_t* __restrict__ act = pd->act;
    const uint32_t* __restrict__ prev = pd->act_prev;
    const uint32_t nx = (uint32_t)pd->nx, ny = (uint32_t)pd->ny;
    uint32_t mx = 0, flags = 0;
    uint64_t sum = 0;
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1};
    // grid rows (iy, iz) per block step, threads along x: no index division;
    // ROWS rows per step, their loads issued before any is used
    const uint32_t nrows = ny * (uint32_t)pd->nz;
    for (uint32_t r0 = blockIdx.x; r0 < nrows; r0 += ROWS * gridDim.x)
    for (uint32_t ix = threadIdx.x; ix < nx; ix += blockDim.x) {
        float m[ROWS];
        uint32_t w[ROWS];
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const uint32_t r = r0 + (uint32_t)u * gridDim.x;
            const uint64_t i = (uint64_t)r * nx + ix;
            m[u] = r < nrows ? mu[i] : 0.0f;
            w[u] = r < nrows ? source_weight(act, prev, i) : 0u;
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const uint32_t r = r0 + (uint32_t)u * gridDim.x;
            if (r >= nrows) break;
            const int iy = (int)(r % ny), iz = (int)(r / ny);
            if (!(m[u] >= 0.0f) || !isfinite(m[u])) flags |= MC_STATUS_BAD_MU;
            else if (m[u] > 0.0f) {
                mx = max(mx, __float_as_uint(m[u]));
                lo[0] = min(lo[0], (int)ix); hi[0] = max(hi[0], (int)ix);
                lo[1] = min(lo[1], iy); hi[1] = max(hi[1], iy);
                lo[2] = min(lo[2], iz); hi[2] = max(hi[2], iz);
            }
            sum += w[u];
        }
    }
    (void)nvox;
    mx = wave_max_u32(mx);
    flags = wave_or_u32(flags);
    sum = wave_sum_u64(sum);
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = max(hi[a], __shfl_xor(hi[a], o, 64));
        }
    }

    // per-block partials (the scan's block-sum scratch, idle until the scan):
    // k_reduce_final combines them.  One atomic per block on the same few
    // descriptor fields serialised in memory.
    __shared__ uint32_t s_mx[RED_THREADS / 64], s_fl[RED_THREADS / 64];
    __shared__ uint64_t s_sum[RED_THREADS / 64];
    __shared__ int s_lo[RED_THREADS / 64][3], s_hi[RED_THREADS / 64][3];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_mx[w] = mx; s_fl[w] = flags; s_sum[w] = sum;
        for (int a = 0; a < 3; ++a) { s_lo[w][a] = lo[a]; s_hi[w][a] = hi[a]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)((blockDim.x + 63) >> 6); ++k) {
            mx = max(mx, s_mx[k]); flags |= s_fl[k]; sum += s_sum[k];
            for (int a = 0; a < 3; ++a) { lo[a] = min(lo[a], s_lo[k][a]); hi[a] = max(hi[a], s_hi[k][a]); }
        }
        uint64_t lo_p = 0, hi_p = 0;     // 16 bits per axis: lo (0xFFFF: none), hi + 1 (0: none)
        for (int a = 0; a < 3; ++a) {
            lo_p |= (uint64_t)(hi[a] >= 0 ? (uint32_t)lo[a] : 0xFFFFu) << (16 * a);
            hi_p |= (uint64_t)(hi[a] >= 0 ? (uint32_t)hi[a] + 1u : 0u) << (16 * a);
        }
        uint64_t* part = pd->block_sums + (uint64_t)blockIdx.x * REDUCE_PART_U64;
        part[0] = (uint64_t)mx | ((uint64_t)flags << 32);
        part[1] = sum;
        part[2] = lo_p;
        part[3] = hi_p;
    }
    if (blockIdx.x == 0) {
        if (pd->pal_state == 0)
            for (int k = threadIdx.x; k < PALETTE_N; k += blockDim.x) pd->palette[k] = PALETTE_EMPTY;
        for (int k = threadIdx.x; k < pd->n_views; k += blockDim.x) {
            const double a = pd->angles[k];
            if (!isfinite(a)) atomicOr(&pd->flags, (uint32_t)MC_STATUS_BAD_ANGLE);
            pd->views[k] = make_float2((float)cos(a), (float)sin(a));
        }
    }
}

// Combine k_reduce's n_parts partials: max mu, flags, activity total and the
// attenuation box, written to the descriptor (one workgroup per problem).
__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(ProbDesc* descs, int n_parts) {
    ProbDesc* pd = descs + blockIdx.y;
    uint32_t mx = 0, flags = 0;
    uint64_t sum = 0;
    uint32_t lo[3] = {0xFFFFu, 0xFFFFu, 0xFFFFu}, hi[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < n_parts; b += blockDim.x) {
        const uint64_t* part = pd->block_sums + (uint64_t)b * REDUCE_PART_U64;
        const uint64_t p0 = part[0], p2 = part[2], p3 = part[3];
        mx = max(mx, (uint32_t)p0);
        flags |= (uint32_t)(p0 >> 32);
        sum += part[1];
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], (uint32_t)(p2 >> (16 * a)) & 0xFFFFu);
            hi[a] = max(hi[a], (uint32_t)(p3 >> (16 * a)) & 0xFFFFu);
        }
    }
    mx = wave_max_u32(mx);
    flags = wave_or_u32(flags);
    sum = wave_sum_u64(sum);
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], o, 64));
            hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], o, 64));
        }
    }
    __shared__ uint32_t s_mx[RED_THREADS / 64], s_fl[RED_THREADS / 64];
    __shared__ uint64_t s_sum[RED_THREADS / 64];
    __shared__ uint32_t s_lo[RED_THREADS / 64][3], s_hi[RED_THREADS / 64][3];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_mx[w] = mx; s_fl[w] = flags; s_sum[w] = sum;
        for (int a = 0; a < 3; ++a) { s_lo[w][a] = lo[a]; s_hi[w][a] = hi[a]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)((blockDim.x + 63) >> 6); ++k) {
            mx = max(mx, s_mx[k]); flags |= s_fl[k]; sum += s_sum[k];
            for (int a = 0; a < 3; ++a) { lo[a] = min(lo[a], s_lo[k][a]); hi[a] = max(hi[a], s_hi[k][a]); }
        }
        pd->mu_hat_bits = mx;
        if (flags) pd->flags |= flags;
        pd->total = sum;
        if (hi[0] > 0) {
            for (int a = 0; a < 3; ++a) {
                pd->bb_lo[a] = (int)lo[a];
                pd->bb_hi[a] = (int)hi[a] - 1;
            }
        }
    }
}

// True if the block has already put q in the palette; otherwise records it
// (a full block set records nothing and answers false).
__device__ inline bool block_seen(uint32_t* set, uint32_t q) {
    uint32_t h = palette_hash(q);
    for (int probe = 0; probe < PALETTE_N; ++probe, h = (h + 1) & (PALETTE_N - 1)) {
        const uint32_t cur = atomicCAS(set + h, PALETTE_EMPTY, q);
        if (cur == PALETTE_EMPTY) return false;
        if (cur == q) return true;
    }
    return false;
}

// Slot of q in the palette, inserting it if absent; PALETTE_N when full.
__device__ inline uint32_t palette_insert(uint32_t* pal, uint32_t q) {
    uint32_t h = palette_hash(q);
    for (int probe = 0; probe < PALETTE_N; ++probe, h = (h + 1) & (PALETTE_N - 1)) {
        uint32_t cur = __hip_atomic_load(pal + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == PALETTE_EMPTY) cur = atomicCAS(pal + h, PALETTE_EMPTY, q);
        if (cur == PALETTE_EMPTY || cur == q) return h;
    }
    return PALETTE_N;
}

// Q_v in double precision: mu_v * 2^24 is exact, the division is correctly
// rounded, ceil is exact.  Stored linear (b = 0) or in 2^b-voxel cubic bricks,
// so a brick is a few whole cache lines (the layout never changes a result).
// Each distinct Q also goes into the palette: a wavefront inserts each of its
// distinct values once (leader lane), so the table sees few atomics.
__global__ __launch_bounds__(RED_THREADS) void k_thresholds(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const uint64_t nvox = pd->nvox;
    const float mu_hat = __uint_as_float(pd->mu_hat_bits);
    const float* __restrict__ mu = pd->mu;
    uint32_t* __restrict__ q = pd->q32;
    const uint32_t nx = (uint32_t)pd->nx, ny = (uint32_t)pd->ny;
    const int b = pd->brick_log2;
    const uint32_t m = (1u << b) - 1u;
    const uint32_t nbx = (uint32_t)pd->nbx, nby = (uint32_t)pd->nby;
    const bool pal = pd->pal_state == 0;
    bool full = false;
    const uint32_t nrows = ny * (uint32_t)pd->nz;
    // the block's own set of the values it has put in the palette: a value
    // reaches the global table once per block, not once per wavefront
    __shared__ uint32_t seen[PALETTE_N];
    for (int k = threadIdx.x; k < PALETTE_N; k += blockDim.x) seen[k] = PALETTE_EMPTY;
    __syncthreads();
    // Q of one value, and its palette entry: a wavefront inserts each of its
    // distinct values once (leader lane); lanes with ok = false only vote.
    // The last four values the wavefront inserted are kept (wave-uniform):
    // a row whose values are all among them skips the insert loop.
    uint32_t recent[4] = {PALETTE_EMPTY, PALETTE_EMPTY, PALETTE_EMPTY, PALETTE_EMPTY};
    uint32_t n_recent = 0;
    auto threshold = [&](float mv, bool ok) -> uint32_t {
        uint32_t v = 0;
        if (ok && mu_hat > 0.0f && mv > 0.0f) {
            const double t = ceil((double)mv * 16777216.0 / (double)mu_hat);
            v = t >= 16777216.0 ? 16777216u : (uint32_t)t;
        }
        if (pal && !full) {
            const bool known = (v == recent[0]) | (v == recent[1]) | (v == recent[2]) | (v == recent[3]);
            bool todo = ok && !known;
            for (;;) {
                const uint64_t left = __ballot(todo);
                if (left == 0) break;
                const int leader = __ffsll((unsigned long long)left) - 1;
                const uint32_t lv = (uint32_t)__shfl((int)v, leader, 64);
                if ((int)(threadIdx.x & 63) == leader && !block_seen(seen, lv) &&
                    palette_insert(pd->palette, lv) == PALETTE_N)
                    full = true;
                if (v == lv) todo = false;
                recent[n_recent & 3u] = lv;   // lv is wave-uniform: so is the cache
                ++n_recent;
            }
        }
        return v;
    };
    if (b == 0) {
        // linear layout: the table index is the voxel index, so whole
        // wavefronts stream the grid, ROWS values per thread in flight
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nvox; i0 += ROWS * stride) {
            float mv[ROWS];
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint64_t i = i0 + (uint64_t)u * stride;
                mv[u] = i < nvox ? mu[i] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint64_t i = i0 + (uint64_t)u * stride;
                const uint32_t v = threshold(mv[u], i < nvox);
                if (i < nvox) q[i] = v;
            }
        }
    } else {
        for (uint32_t r0 = blockIdx.x; r0 < nrows; r0 += ROWS * gridDim.x)
        for (uint32_t ix = threadIdx.x; ix < nx; ix += blockDim.x) {
            // ROWS rows per step, their loads issued before any is used
            float mrow[ROWS];
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint32_t r = r0 + (uint32_t)u * gridDim.x;
                mrow[u] = r < nrows ? mu[(uint64_t)r * nx + ix] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint32_t r = r0 + (uint32_t)u * gridDim.x;
                if (r >= nrows) break;
                const uint32_t v = threshold(mrow[u], true);
                q[brick_index(ix, r % ny, r / ny, nx, ny, b, m, nbx, nby)] = v;
            }
        }
    }
    if (full) atomicOr(&pd->pal_state, 1u);
}

// One-byte palette codes in the threshold layout (skipped when the palette
// overflowed or was not requested: the kernels then read the 32-bit table).
__global__ __launch_bounds__(RED_THREADS) void k_codes(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    if (pd->pal_state != 0) return;
    const uint64_t nvox = pd->nvox;
    const uint32_t* __restrict__ q = pd->q32;
    const uint32_t* __restrict__ pal = pd->palette;
    uint8_t* __restrict__ code = pd->q8;
    const uint32_t nx = (uint32_t)pd->nx, ny = (uint32_t)pd->ny;
    const int b = pd->brick_log2;
    const uint32_t m = (1u << b) - 1u;
    const uint32_t nbx = (uint32_t)pd->nbx, nby = (uint32_t)pd->nby;
    const uint32_t nrows = ny * (uint32_t)pd->nz;
    auto code_of = [&](uint32_t v) {
        uint32_t h = palette_hash(v);
        for (int probe = 0; probe < PALETTE_N && pal[h] != v; ++probe) h = (h + 1) & (PALETTE_N - 1);
        return (uint8_t)h;
    };
    if (b == 0) {
        // linear layout: whole wavefronts stream the table, ROWS values per thread
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nvox; i0 += ROWS * stride) {
            uint32_t v[ROWS];
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint64_t i = i0 + (uint64_t)u * stride;
                v[u] = i < nvox ? q[i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < ROWS; ++u) {
                const uint64_t i = i0 + (uint64_t)u * stride;
                if (i < nvox) code[i] = code_of(v[u]);
            }
        }
        return;
    }
    for (uint32_t r0 = blockIdx.x; r0 < nrows; r0 += ROWS * gridDim.x)
    for (uint32_t ix = threadIdx.x; ix < nx; ix += blockDim.x) {
        // ROWS rows per step, their loads issued before any is used
        uint32_t k[ROWS], v[ROWS];
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const uint32_t r = r0 + (uint32_t)u * gridDim.x;
            k[u] = brick_index(ix, r % ny, r / ny, nx, ny, b, m, nbx, nby);
            v[u] = r < nrows ? q[k[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            if (r0 + (uint32_t)u * gridDim.x >= nrows) break;
            code[k[u]] = code_of(v[u]);
        }
    }
}

// --- three-pass scan of the activity map: uint64 sums of the source weight
// and the runs of equal weight, so the emission tables hold one entry per run
// (a segmented phantom has ~1e4 runs against ~1e6 active voxels) ---

// Voxel i starts a run: it is active and its row neighbour on the left (none
// at ix = 0) has a different weight.
__device__ inline bool run_start(uint32_t a, uint32_t a_left, uint64_t i, uint32_t nx) {
    return a > 0 && (i % nx == 0 || a_left != a);
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const uint64_t nvox = pd->nvox;
    if ((uint64_t)blockIdx.x * SCAN_ITEMS >= nvox) return;   // past this problem's blocks
    const uint32_t* __restrict__ act = pd->act;
    const uint32_t* __restrict__ prev = pd->act_prev;
    const uint32_t nx = (uint32_t)pd->nx;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
    uint32_t c = 0;
    for (int j = threadIdx.x; j < SCAN_ITEMS; j += SCAN_THREADS) {
        const uint64_t i = base + j;
        if (i < nvox) {
            const uint32_t a = source_weight(act, prev, i);
            const uint32_t l = i > 0 ? source_weight(act, prev, i - 1) : 0u;
            s += a;
            c += run_start(a, l, i, nx);
        }
    }
    s = wave_sum_u64(s);
    c = (uint32_t)wave_sum_u64(c);
    __shared__ uint64_t part[SCAN_THREADS / 64];
    __shared__ uint32_t partc[SCAN_THREADS / 64];
    if ((threadIdx.x & 63) == 0) { part[threadIdx.x >> 6] = s; partc[threadIdx.x >> 6] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        uint32_t tc = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) { t += part[w]; tc += partc[w]; }
        pd->block_sums[blockIdx.x] = t;
        pd->block_cnt[blockIdx.x] = tc;
    }
}

// Exclusive scan of the block sums and run counts, one block of 1024
// threads, each thread a contiguous stretch; also records the number of runs.
__global__ __launch_bounds__(1024) void k_scan_top(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const int n_blocks = (int)((pd->nvox + SCAN_ITEMS - 1) / SCAN_ITEMS);
    __shared__ uint64_t tot[1024];
    __shared__ uint32_t totc[1024];
    uint64_t* __restrict__ bs = pd->block_sums;
    uint32_t* __restrict__ bc = pd->block_cnt;
    const int per = (n_blocks + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint64_t s = 0;
    uint32_t c = 0;
    for (int j = 0; j < per; ++j) if (b0 + j < n_blocks) { s += bs[b0 + j]; c += bc[b0 + j]; }
    tot[threadIdx.x] = s;
    totc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        const uint32_t vc = threadIdx.x >= (unsigned)off ? totc[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += v;
        totc[threadIdx.x] += vc;
        __syncthreads();
    }
    if (threadIdx.x == 1023) pd->n_runs = totc[1023];
    uint64_t run = tot[threadIdx.x] - s;   // exclusive prefix of this thread's stretch
    uint32_t runc = totc[threadIdx.x] - c;
    for (int j = 0; j < per; ++j) {
        if (b0 + j < n_blocks) {
            const uint64_t v = bs[b0 + j];
            const uint32_t vc = bc[b0 + j];
            bs[b0 + j] = run;
            bc[b0 + j] = runc;
            run += v;
            runc += vc;
        }
    }
}

// Per block: 16 consecutive voxels per thread, thread-local scans, block
// exclusive scans of the thread totals, plus the block offsets; each voxel
// that starts a run writes the run (cumulative weight before it, its packed
// coordinates, its weight) at its compacted slot.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_final(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    constexpr int PER = SCAN_ITEMS / SCAN_THREADS;
    const uint64_t nvox = pd->nvox;
    if ((uint64_t)blockIdx.x * SCAN_ITEMS >= nvox) return;   // past this problem's blocks
    const uint32_t* __restrict__ act = pd->act;
    const uint32_t* __restrict__ prev = pd->act_prev;
    uint4* __restrict__ runs = pd->runs;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_ITEMS + (uint64_t)threadIdx.x * PER;
    const uint32_t nx = (uint32_t)pd->nx, ny = (uint32_t)pd->ny;
    uint32_t a[PER];
    const uint32_t left0 = (base > 0 && base < nvox) ? source_weight(act, prev, base - 1) : 0u;
    uint64_t s = 0;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t i = base + j;
        a[j] = (i < nvox) ? source_weight(act, prev, i) : 0u;
        s += a[j];
    }
    uint32_t starts = 0;        // bit j: voxel base + j starts a run
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t l = j > 0 ? a[j - 1] : left0;
        if (base + j < nvox && run_start(a[j], l, base + j, nx)) starts |= 1u << j;
    }
    c = __popc(starts);
    __shared__ uint64_t tot[SCAN_THREADS];
    __shared__ uint32_t totc[SCAN_THREADS];
    tot[threadIdx.x] = s;
    totc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        const uint32_t tc = threadIdx.x >= (unsigned)off ? totc[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        totc[threadIdx.x] += tc;
        __syncthreads();
    }
    uint64_t before = pd->block_sums[blockIdx.x] + tot[threadIdx.x] - s;   // weight before voxel base
    uint32_t k = pd->block_cnt[blockIdx.x] + totc[threadIdx.x] - c;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (starts & (1u << j)) {
            const uint32_t i = (uint32_t)(base + j);
            const uint32_t ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
            runs[k] = make_uint4((uint32_t)before, (uint32_t)(before >> 32),
                                 ix | (iy << 10) | (iz << 20), a[j]);   // packed 10 bits per axis
            ++k;
        }
        before += a[j];
    }
}

// Bucket table over the runs: bucket b covers t in [b 2^s, (b+1) 2^s), with
// about two buckets per run (after the guide tables of Chen & Asau 1974).
// Run r holds t in [c_r, c_{r+1}); the bucket's entry is the run holding its
// first t and the number of further runs starting inside it.
__device__ inline uint64_t run_c(const uint4* __restrict__ runs, uint64_t r) {
    const uint4 v = runs[r];
    return ((uint64_t)v.y << 32) | v.x;
}

// First run whose start is above key (R when none): the run holding key is
// the one before it (run 0 starts at 0 <= key).
__device__ inline uint64_t first_run_above(const uint4* __restrict__ runs, uint64_t R, uint64_t key) {
    uint64_t lo = 0, hi = R;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (run_c(runs, mid) > key) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(RED_THREADS) void k_guide(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const uint64_t nb_cap = guide_capacity(pd->nvox);
    const uint64_t total = pd->total;
    const uint64_t R = pd->n_runs;
    if (total == 0 || R == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&pd->flags, (uint32_t)MC_STATUS_NO_ACTIVITY);
        return;
    }
    uint64_t cap = 1;
    while (cap < 2 * R) cap <<= 1;
    if (cap > nb_cap) cap = nb_cap;
    uint32_t s = 0;
    while (((total - 1) >> s) >= cap) ++s;
    const uint64_t B = ((total - 1) >> s) + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        pd->shift = s;
        pd->n_buckets = (uint32_t)B;
    }
    const uint4* __restrict__ runs = pd->runs;
    uint2* __restrict__ guide = pd->guide;
    // bucket b's first t lies in run lo(b) = first_run_above(b 2^s) - 1 and
    // its last t = (b + 1) 2^s - 1 in run hi(b) = (first run starting at or
    // above (b + 1) 2^s) - 1, which is lo(b + 1), or one less when a run
    // starts exactly at (b + 1) 2^s.  A wavefront finds lo for 64
    // consecutive buckets, one search per lane, and completes 63 of them with
    // its neighbour's.
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t grp = wave; grp * 63 < B; grp += n_waves) {
        const uint64_t b = grp * 63 + (uint64_t)lane;
        const uint64_t fa = b < B ? first_run_above(runs, R, b << s) : R;   // >= 1
        const uint32_t nl = (uint32_t)__shfl_down((int)(uint32_t)fa, 1, 64);
        const uint32_t nh = (uint32_t)__shfl_down((int)(uint32_t)(fa >> 32), 1, 64);
        if (lane == 63 || b >= B) continue;
        const uint64_t lo = fa - 1;
        uint64_t hi;
        if (b + 1 < B) {
            const uint64_t fa1 = (uint64_t)nl | ((uint64_t)nh << 32);
            hi = fa1 - 1;
            if (run_c(runs, hi) == ((b + 1) << s)) --hi;
        } else {
            hi = R - 1;                        // the last bucket ends at total - 1
        }
        guide[b] = make_uint2((uint32_t)lo, (uint32_t)(hi - lo));
    }
}

// Klein-Nishina total cross-section per electron over 2 pi r_e^2 (closed form).
__device__ double kn_bracket(double e) {
    const double k = e / 510.99895;
    const double a = 1.0 + 2.0 * k;
    const double la = log(a);
    return (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - la / k) + la / (2.0 * k)
           - (1.0 + 3.0 * k) / (a * a);
}

__global__ void k_kn_table(ProbDesc* descs) {
    ProbDesc* pd = descs + blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KN_TABLE_N) return;
    const double e = fmax((double)pd->e0 - 0.25 * i, 0.5);
    pd->kn_table[i] = (float)(kn_bracket(e) / kn_bracket(140.0));
}

int grid_for(uint64_t n, int threads, int cap) {
    uint64_t g = (n + threads - 1) / threads;
    if (g > (uint64_t)cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace


// The problems' descriptors are written one by one (by value, so the launch
// can be captured in a graph); every other pass is one launch for all
// problems, blockIdx.y picking the problem and each block walking that
// problem's share, so small problems overlap instead of queueing.
hipError_t launch_staging_batch(ProbDesc* d, const ProbDesc* h, int n, hipStream_t st) {
    uint64_t max_rows = 1, max_nb = 1, max_cap = 1;
    int max_nx = 1;
    for (int i = 0; i < n; ++i) {
        k_write_desc<<<1, 64, 0, st>>>(h[i], d + i);
        max_rows = std::max<uint64_t>(max_rows, (uint64_t)h[i].ny * h[i].nz);
        max_nx = std::max(max_nx, h[i].nx);
        max_nb = std::max<uint64_t>(max_nb, (h[i].nvox + SCAN_ITEMS - 1) / SCAN_ITEMS);
        max_cap = std::max<uint64_t>(max_cap, guide_capacity(h[i].nvox));
    }
    // row-per-block passes: a block walks grid rows (iy, iz), threads along x
    const int row_threads = (int)std::min<uint64_t>(RED_THREADS, ((uint64_t)max_nx + 63) / 64 * 64);
    const unsigned ny = (unsigned)n;
    const unsigned red_blocks = (unsigned)std::min<uint64_t>(max_rows, REDUCE_BLOCKS);
    k_reduce<<<dim3(red_blocks, ny), row_threads, 0, st>>>(d);
    k_reduce_final<<<dim3(1, ny), RED_THREADS, 0, st>>>(d, (int)red_blocks);
    const unsigned row_blocks = (unsigned)std::min<uint64_t>((max_rows + ROWS - 1) / ROWS, 8192);
    // each workgroup puts each threshold value it meets into the palette once
    // (a round trip to memory): fewer, larger workgroups for this pass
    k_thresholds<<<dim3(std::min(row_blocks, 1024u), ny), row_threads, 0, st>>>(d);
    k_codes<<<dim3(row_blocks, ny), row_threads, 0, st>>>(d);
    k_scan_sums<<<dim3((unsigned)max_nb, ny), SCAN_THREADS, 0, st>>>(d);
    k_scan_top<<<dim3(1, ny), 1024, 0, st>>>(d);
    k_scan_final<<<dim3((unsigned)max_nb, ny), SCAN_THREADS, 0, st>>>(d);
    k_guide<<<dim3((unsigned)grid_for(max_cap, RED_THREADS, 8192), ny), RED_THREADS, 0, st>>>(d);
    k_kn_table<<<dim3((KN_TABLE_N + 255) / 256, ny), 256, 0, st>>>(d);
    return hipGetLastError();
}

// Entries (uint64) of a problem's block-sum scratch: the scan's block sums,
// and before them k_reduce's partials.
size_t staging_block_scratch_u64(uint64_t nvox) {
    const uint64_t nb = (nvox + SCAN_ITEMS - 1) / SCAN_ITEMS;
    const uint64_t red = (uint64_t)REDUCE_BLOCKS * REDUCE_PART_U64;
    return (size_t)(nb > red ? nb : red);
}

hipError_t launch_staging(ProbDesc* d, const ProbDesc& h, hipStream_t st) {
    return launch_staging_batch(d, &h, 1, st);
}

}  // namespace mcs
