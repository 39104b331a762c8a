// Monte Carlo response matrix and MLEM (paper Sec. 5.1, Eq. IMC and Eq. MLEM).
//
// Response matrix.  Each tally contribution of the forward call is an event
// (projection bin j, phantom voxel of emission, weight: 1 for an analog
// arrival, the score of a forced-detection copy).  With i the image voxel of
// the emission (phantom voxel / image_factor per axis),
//     T_ij = c_ij / n_i(j),   n_i(j) = N_view(j) * A_i / A,
// c_ij the summed weight of the events (i, j), N_view(j) the histories of bin j's view,
// A_i the activity in image voxel i and A the total: the estimated probability
// that a photon emitted in image voxel i is counted in bin j.  Bins merge the
// primary and scatter classes (the camera cannot tell them apart): j =
// (view * nv + iv) * nu + iu.  The projection P_j = sum_i c_ij is the same
// run's counts, so P = T n exactly.
//
// Both orientations are built as CSR (bins x voxels and voxels x bins): the
// events are radix-sorted by (row, column), runs of equal keys merged, and
// the weights summed as Q31.32 integers, so the result does not depend on the
// order of the event list.
//
// MLEM.  S_i <- S_i / sens_i * sum_j T_ij P_j / y_j, y = T S, sens_i =
// sum_j T_ij; FP32 matrix values, FP64 accumulation; bins with y_j = 0 add
// nothing; voxels with sens_i = 0 stay 0.  Rows are swept by groups of 1 to
// 64 lanes sized to the mean row length; on large detectors the
// backprojection works on one bin slice per XCD so its gathers hit L2.
#include <algorithm>

#include "mc_internal.h"

namespace mcs {
namespace {

constexpr int T256 = 256;
constexpr int SCAN_PER = 16;                     // items per thread in the block scan
constexpr int SCAN_BLOCK = T256 * SCAN_PER;      // items per scan block

int grid_for(uint64_t n, int threads, int cap) {
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

__device__ inline uint64_t wave_sum64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---- generic exclusive scan: uint32 counts -> uint64 offsets [n + 1] ----

// n_dev (nullable): a device-side count below n; items from it on are taken
// as 0 without being read, and outputs past it are not written.
__device__ inline uint64_t scan_limit(uint64_t n, const uint64_t* n_dev) {
    if (!n_dev) return n;
    const uint64_t m = *n_dev;
    return m < n ? m : n;
}

__global__ __launch_bounds__(T256) void k_sum_blocks(const uint32_t* __restrict__ in, uint64_t n_host,
                                                     const uint64_t* __restrict__ n_dev,
                                                     uint64_t* __restrict__ bsum) {
    const uint64_t n = scan_limit(n_host, n_dev);
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK;
    uint64_t s = 0;
    for (int j = threadIdx.x; j < SCAN_BLOCK; j += T256) {
        const uint64_t i = base + j;
        if (i < n) s += in[i];
    }
    s = wave_sum64(s);
    __shared__ uint64_t part[T256 / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < T256 / 64; ++w) t += part[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint64_t* bsum, int nb) {
    __shared__ uint64_t tot[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint64_t s = 0;
    for (int j = 0; j < per; ++j) if (b0 + j < nb) s += bsum[b0 + j];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = tot[threadIdx.x] - s;
    for (int j = 0; j < per; ++j) {
        if (b0 + j < nb) {
            const uint64_t v = bsum[b0 + j];
            bsum[b0 + j] = run;
            run += v;
        }
    }
}

// out[i] = sum_{k<i} in[k] for i in [0, n]; out[n] = total.
__global__ __launch_bounds__(T256) void k_scan_write(const uint32_t* __restrict__ in, uint64_t n_host,
                                                     const uint64_t* __restrict__ n_dev,
                                                     const uint64_t* __restrict__ bsum,
                                                     uint64_t* __restrict__ out) {
    const uint64_t n = scan_limit(n_host, n_dev);
    if ((uint64_t)blockIdx.x * SCAN_BLOCK > n) return;   // past the limit: no output here
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK + (uint64_t)threadIdx.x * SCAN_PER;
    uint32_t v[SCAN_PER];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const uint64_t i = base + j;
        v[j] = i < n ? in[i] : 0u;
        s += v[j];
    }
    __shared__ uint64_t tot[T256];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < T256; off <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    uint64_t run = bsum[blockIdx.x] + tot[threadIdx.x] - s;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const uint64_t i = base + j;
        if (i <= n) out[i] = run;   // i == n: the total
        run += v[j];
    }
}

// out[i] = sum_{k<i} in[k] for i in [0, min(n, *n_dev)] (n_dev nullable).
hipError_t exclusive_scan(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* bsum,
                          hipStream_t s, const uint64_t* n_dev = nullptr) {
    // one extra item so the block holding index n writes the total
    const int nb = (int)((n + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK);
    k_sum_blocks<<<nb, T256, 0, s>>>(in, n, n_dev, bsum);
    k_scan_blocks<<<1, 1024, 0, s>>>(bsum, nb);
    k_scan_write<<<nb, T256, 0, s>>>(in, n, n_dev, bsum, out);
    return hipGetLastError();
}

// ---- response matrix ----

struct SysArgs {
    const mc_event* events;
    const unsigned long long* n_events;
    uint64_t capacity;
    uint32_t class_mask;     // bit 0: primary events, bit 1: scattered events
    uint32_t nv_nu;          // bins per view and class
    uint32_t nx, ny, f, mx, my;
    uint64_t q_per_view, r_extra;
};

__device__ inline uint64_t n_events_of(const SysArgs& a) {
    const uint64_t n = *a.n_events;
    return n < a.capacity ? n : a.capacity;
}

// projection bin (classes merged) and image voxel of event e; false if the
// event's class is filtered out
__device__ inline bool event_rc(const SysArgs& a, const mc_event& ev, uint32_t& bin, uint32_t& img) {
    const uint32_t per_view = 2u * a.nv_nu;
    const uint32_t cls = (ev.bin / a.nv_nu) & 1u;
    if (!((a.class_mask >> cls) & 1u)) return false;
    const uint32_t view = ev.bin / per_view;
    bin = view * a.nv_nu + (ev.bin % a.nv_nu);
    const uint32_t v = ev.emit_voxel;
    const uint32_t ix = v % a.nx, iy = (v / a.nx) % a.ny, iz = v / (a.nx * a.ny);
    img = (ix / a.f) + a.mx * ((iy / a.f) + a.my * (iz / a.f));
    return true;
}

__global__ __launch_bounds__(T256) void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

// activity per image voxel, and the total
__global__ __launch_bounds__(T256) void k_image_activity(const uint32_t* __restrict__ act,
                                                         uint32_t nx, uint32_t ny, uint32_t nz,
                                                         uint32_t f, uint32_t mx, uint32_t my,
                                                         unsigned long long* __restrict__ a_img,
                                                         unsigned long long* __restrict__ total) {
    const uint64_t n = (uint64_t)nx * ny * nz;
    uint64_t sum = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t a = act[i];
        if (!a) continue;
        sum += a;
        const uint32_t ix = (uint32_t)(i % nx), iy = (uint32_t)((i / nx) % ny), iz = (uint32_t)(i / ((uint64_t)nx * ny));
        atomicAdd(a_img + (ix / f) + mx * ((iy / f) + my * (iz / f)), (unsigned long long)a);
    }
    sum = wave_sum64(sum);
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(total, (unsigned long long)sum);
}

// ---- response matrix rows by LSD radix sort ----
//
// Each orientation sorts the events by the key (row << col_bits) | col with
// a least-significant-digit radix sort (8-bit digits, stable), so a row's
// events end up together, ordered by column, with duplicates adjacent.  A
// pass is three launches: per-tile digit histograms (LDS counters), one
// exclusive scan of the histograms in digit-major order (the global output
// offset of every (digit, tile)), and a stable scatter: within a tile, items
// are ranked round by round (256 consecutive items), inside a wavefront by
// matching digits with eight ballots and across the four wavefronts through
// LDS counts.  No global atomics: the per-event atomics of a counting sort
// contend on the rows that collect many events.  The event count is read on
// the device, so nothing waits on the host; tiles past it do no work.
// Events of a filtered class take row n_rows and sort last.

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;              // digits per pass (= T256)
constexpr int RADIX_ITEMS = 16;                     // items per thread and tile
constexpr uint64_t RADIX_TILE = (uint64_t)T256 * RADIX_ITEMS;
static_assert(RADIX == T256, "one digit counter per thread");

int bit_width(uint64_t v) {
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

// Tile of workgroup b.  Workgroups are dealt to the 8 XCDs in turn; the
// tiles that hold items (the first `used`) are remapped so that each XCD
// takes a contiguous run of them, so neighbouring tiles share one L2 (their
// histogram and offset lines, and the adjacent digit runs they write).
// Empty tiles keep their own index.
__device__ inline uint32_t tile_of(uint32_t b, uint64_t n) {
    const uint32_t used = (uint32_t)((n + RADIX_TILE - 1) / RADIX_TILE);
    if (b >= used) return b;
    const uint32_t per = used / 8, rem = used % 8, x = b % 8, q = b / 8;
    return x * per + (x < rem ? x : rem) + q;
}

__global__ __launch_bounds__(T256) void k_make_keys(SysArgs a, int transpose, uint64_t n_rows,
                                                    int col_bits, uint64_t* __restrict__ keys,
                                                    int64_t* __restrict__ vals) {
    const uint64_t n = n_events_of(a);
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t bin, img;
        const mc_event ev = a.events[e];
        if (event_rc(a, ev, bin, img)) {
            const uint64_t r = transpose ? img : bin, c = transpose ? bin : img;
            keys[e] = (r << col_bits) | c;
            vals[e] = ev.weight;
        } else {
            keys[e] = n_rows << col_bits;
            vals[e] = 0;
        }
    }
}

// hist[d * n_tiles + t]: items of tile t (one workgroup per tile) with digit d
__global__ __launch_bounds__(T256) void k_radix_hist(const uint64_t* __restrict__ keys, SysArgs a,
                                                     int shift, uint32_t n_tiles,
                                                     uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[RADIX];
    const uint64_t n = n_events_of(a);
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t tile = tile_of(blockIdx.x, n);
    const uint64_t base = (uint64_t)tile * RADIX_TILE;
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const uint64_t i = base + (uint64_t)j * T256 + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * n_tiles + tile] = cnt[threadIdx.x];
}

// Stable scatter of tile t's items to offs[d * n_tiles + t] + their rank
// among the tile's items of digit d.  Each wavefront takes a quarter of the
// tile (1024 consecutive items, 16 per lane, loaded at once) and ranks it on
// its own, 64 items per round: lanes with equal digits found with eight
// ballots, and a running count per digit kept in the wavefront's row of LDS.
// After one barrier, the earlier wavefronts' counts place each item in a
// digit-ordered copy of the tile in LDS (keys, then values through the same
// 32 KB), which is written out so that each digit's run from this tile (16
// items on average) goes to consecutive addresses.
constexpr uint32_t RADIX_WAVE_ITEMS = (uint32_t)(RADIX_TILE / (T256 / 64));

__global__ __launch_bounds__(T256) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                        const int64_t* __restrict__ vin,
                                                        uint64_t* __restrict__ kout,
                                                        int64_t* __restrict__ vout, SysArgs a,
                                                        int shift, uint32_t n_tiles,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint64_t* __restrict__ offs) {
    __shared__ uint64_t stage[RADIX_TILE];         // the tile's keys, then values, in digit order
    __shared__ uint16_t sdig[RADIX_TILE];          // the digit of each staged slot
    __shared__ uint64_t gbase[RADIX];              // global slot of each digit's first item
    __shared__ uint32_t lstart[RADIX];             // tile slot of each digit's first item
    __shared__ uint32_t wcnt[T256 / 64][RADIX];    // items of each digit per wavefront
    __shared__ uint32_t wsum[T256 / 64];
    const uint64_t n = n_events_of(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    const uint32_t tile = tile_of(blockIdx.x, n);
    const uint64_t base = (uint64_t)tile * RADIX_TILE;
    if (base >= n) return;       // an empty tile (the whole workgroup leaves)
    const uint64_t wbase = base + (uint64_t)wave * RADIX_WAVE_ITEMS;

    uint64_t k[RADIX_ITEMS];
    int64_t v[RADIX_ITEMS];
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const uint64_t i = wbase + (uint64_t)j * 64 + lane;
        k[j] = i < n ? kin[i] : 0;
        v[j] = i < n ? vin[i] : 0;
    }
    // tile slots: exclusive scan of this tile's digit counts
    const uint32_t c = hist[(uint64_t)threadIdx.x * n_tiles + tile];
    gbase[threadIdx.x] = offs[(uint64_t)threadIdx.x * n_tiles + tile];
#pragma unroll
    for (int w = 0; w < T256 / 64; ++w) wcnt[w][threadIdx.x] = 0;
    uint32_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    lstart[threadIdx.x] = pre + x - c;

    // rank within this wavefront: items of the same digit in earlier rounds
    // (the running count) plus lower lanes of this round
    uint32_t rk[RADIX_ITEMS];
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const bool ok = wbase + (uint64_t)j * 64 + lane < n;
        const uint32_t d = ok ? (uint32_t)(k[j] >> shift) & (RADIX - 1) : 0;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lane_lt);
        const uint32_t before = ok ? wcnt[wave][d] : 0;
        rk[j] = before + rank;
        if (ok && rank == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // tile slots of this lane's items (kept for the second staging)
    uint32_t slot[RADIX_ITEMS];
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        slot[j] = RADIX_TILE;
        if (wbase + (uint64_t)j * 64 + lane >= n) continue;
        const uint32_t d = (uint32_t)(k[j] >> shift) & (RADIX - 1);
        uint32_t sl = lstart[d] + rk[j];
        for (int w = 0; w < wave; ++w) sl += wcnt[w][d];
        slot[j] = sl;
        if (sl < RADIX_TILE) {
            stage[sl] = k[j];
            sdig[sl] = (uint16_t)d;
        }
    }
    __syncthreads();
    const uint64_t in_tile = n - base < RADIX_TILE ? n - base : RADIX_TILE;
    for (uint32_t t = threadIdx.x; t < in_tile; t += T256) {
        const uint32_t d = sdig[t];
        const uint64_t pos = gbase[d] + (t - lstart[d]);
        if (pos < a.capacity) kout[pos] = stage[t];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j)
        if (slot[j] < RADIX_TILE) stage[slot[j]] = (uint64_t)v[j];
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < in_tile; t += T256) {
        const uint32_t d = sdig[t];
        const uint64_t pos = gbase[d] + (t - lstart[d]);
        if (pos < a.capacity) vout[pos] = (int64_t)stage[t];
    }
}

// start[r] (r = 0..n_rows): first sorted position whose row is >= r (a
// binary search, so start is non-decreasing and within [0, n] whatever the
// keys hold); the filtered events (row n_rows) follow start[n_rows].
__global__ __launch_bounds__(T256) void k_row_starts(const uint64_t* __restrict__ keys, SysArgs a,
                                                     int col_bits, uint64_t n_rows,
                                                     uint64_t* __restrict__ start) {
    const uint64_t n = n_events_of(a);
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n_rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = r << col_bits;
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (keys[mid] < key) lo = mid + 1; else hi = mid;
        }
        start[r] = lo;
    }
}

// flag[i] = 1 where a run of equal keys starts, for the valid (unfiltered)
// items i < start[n_rows] (the scan below reads no further)
__global__ __launch_bounds__(T256) void k_run_heads(const uint64_t* __restrict__ keys,
                                                    const uint64_t* __restrict__ start,
                                                    uint64_t n_rows, uint64_t capacity,
                                                    uint32_t* __restrict__ flag) {
    const uint64_t n_valid = start[n_rows] < capacity ? start[n_rows] : capacity;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_valid;
         i += (uint64_t)gridDim.x * blockDim.x)
        flag[i] = i == 0 || keys[i] != keys[i - 1];
}

// rowptr[r] = distinct entries before row r (head_pos: exclusive scan of the run heads)
__global__ __launch_bounds__(T256) void k_rows_from_runs(const uint64_t* __restrict__ start,
                                                         const uint64_t* __restrict__ head_pos,
                                                         uint64_t n_rows, int64_t* __restrict__ rowptr) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n_rows;
         r += (uint64_t)gridDim.x * blockDim.x)
        rowptr[r] = (int64_t)head_pos[start[r]];
}

// Each run of equal keys (one distinct (row, column)) becomes CSR entry
// head_pos[i] of its first item i: the column and T = c / n_i(j), with c the
// run's summed weight.
__global__ __launch_bounds__(T256) void k_emit_runs(SysArgs a, int transpose,
                                                    const uint64_t* __restrict__ keys,
                                                    const int64_t* __restrict__ w,
                                                    const uint64_t* __restrict__ start,
                                                    const uint64_t* __restrict__ head_pos,
                                                    uint64_t n_rows, int col_bits,
                                                    int32_t* __restrict__ col, float* __restrict__ val,
                                                    const unsigned long long* __restrict__ a_img,
                                                    const unsigned long long* __restrict__ total_p) {
    const uint64_t n_valid = start[n_rows];
    const double total = (double)*total_p;
    const uint64_t mask = (1ull << col_bits) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_valid;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        if (i > 0 && keys[i - 1] == k) continue;
        long long cw = 0;
        for (uint64_t j = i; j < n_valid && keys[j] == k; ++j) cw += w[j];
        const uint32_t r = (uint32_t)(k >> col_bits), c = (uint32_t)(k & mask);
        const uint32_t bin = transpose ? c : r;
        const uint32_t img = transpose ? r : c;
        const uint64_t view = bin / a.nv_nu;
        const double n_view = (double)(a.q_per_view + (view < a.r_extra ? 1u : 0u));
        const double n_i = n_view * (double)a_img[img] / total;
        const uint64_t o = head_pos[i];
        col[o] = (int32_t)c;
        val[o] = (float)((double)cw * 0x1p-32 / n_i);
    }
}

// P_j = the summed weight of bin row j's events (all its items)
__global__ __launch_bounds__(T256) void k_proj_rows(const int64_t* __restrict__ w,
                                                    const uint64_t* __restrict__ start,
                                                    uint64_t n_rows, float* __restrict__ proj) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        long long tot = 0;
        for (uint64_t i = start[r]; i < start[r + 1]; ++i) tot += w[i];
        proj[r] = (float)((double)tot * 0x1p-32);
    }
}

// ---- MLEM ----
//
// Row kernels: a matrix whose rows hold on average at least WAVE_ROW_MIN
// entries (forced-detection matrices) is read one wavefront per row --
// coalesced loads, FP64 wavefront reduction -- and a sparse one (analog
// matrices: far fewer entries than rows) one thread per row.  The choice
// depends only on the matrix, so results are deterministic.

constexpr int64_t WAVE_ROW_MIN = 8;

__device__ inline double wave_sum_f64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// For each row r: done(r, sum over the row's entries of term(k)).
template <class Term, class Done>
__device__ inline void for_rows(int64_t n_rows, const int64_t* __restrict__ rp, Term term, Done done) {
    const bool wave_mode = rp[n_rows] >= WAVE_ROW_MIN * n_rows;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    if (wave_mode) {
        const int lane = threadIdx.x & 63;
        for (int64_t r = tid >> 6; r < n_rows; r += nt >> 6) {
            double acc = 0.0;
            for (int64_t k = rp[r] + lane; k < rp[r + 1]; k += 64) acc += term(k);
            acc = wave_sum_f64(acc);
            if (lane == 0) done(r, acc);
        }
    } else {
        for (int64_t r = tid; r < n_rows; r += nt) {
            double acc = 0.0;
            for (int64_t k = rp[r]; k < rp[r + 1]; ++k) acc += term(k);
            done(r, acc);
        }
    }
}

__global__ __launch_bounds__(T256) void k_row_sums(int64_t n_rows, const int64_t* __restrict__ rp,
                                                   const float* __restrict__ v, double* __restrict__ out) {
    for_rows(n_rows, rp, [&](int64_t k) { return (double)v[k]; },
             [&](int64_t r, double acc) { out[r] = acc; });
}

__global__ __launch_bounds__(T256) void k_mlem_init(int64_t n_vox, const float* __restrict__ img,
                                                    const double* __restrict__ sens,
                                                    double* __restrict__ S) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * blockDim.x)
        S[i] = sens[i] > 0.0 ? (double)img[i] : 0.0;
}

// Lanes that share one row in the MLEM sweeps: the smallest group of 1, 4, 16
// or 64 lanes for which four entries per lane cover the mean row (nnz /
// n_rows entries), so that short rows do not leave most of a wavefront idle.
__device__ inline int lanes_per_row(int64_t nnz, int64_t n_rows) {
    if (nnz <= 4 * n_rows) return 1;
    if (nnz <= 16 * n_rows) return 4;
    if (nnz <= 64 * n_rows) return 16;
    return 64;
}

// The rows a group of GS lanes visits: row g, g + n_groups, ... (g: the
// group's index among n_groups); every lane of a group sees the same rows.
template <int GS>
struct RowGroups {
    int64_t first, step;
    int sub;
    __device__ RowGroups(int64_t block, int64_t n_blocks) {
        const int64_t t = block * blockDim.x + threadIdx.x;
        first = t / GS;
        step = n_blocks * blockDim.x / GS;
        sub = (int)(threadIdx.x & (GS - 1));
    }
};

// Sum over k in [k0, k1) of term(k, valid) by a group of GS lanes (sub: the
// lane's index in the group).  Indices past the end are clamped to k1 - 1 so
// every load is in bounds and issued unconditionally; term() zeroes them.
// Each lane adds its four terms in order, then a butterfly over the group:
// the summation order depends only on the row and GS.
template <int GS, class Term>
__device__ inline double group_row_sum(int64_t k0, int64_t k1, int sub, Term term) {
    double acc = 0.0;
    for (int64_t k = k0 + sub; k < k1; k += 4 * GS) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t kk = k + (int64_t)u * GS;
            t[u] = term(kk < k1 ? kk : k1 - 1, kk < k1);
        }
        acc += t[0];
        acc += t[1];
        acc += t[2];
        acc += t[3];
    }
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, GS);
    return acc;
}

// A group's rows of n, four per pass: bounds(q, lo, hi) loads the entry
// ranges of four rows before any of them is summed (row by row, with
// group_row_sum), so a sparse matrix (most rows empty or one entry long)
// keeps four row-pointer loads in flight per lane.  done(q, lo, len, sum)
// runs for every row q < n; the test is group-uniform.  (Summing the four
// rows interleaved was slower on forced-detection matrices: a pass then
// lasts as long as the longest of the four rows.)
template <int GS, class Bounds, class Term, class Done>
__device__ inline void sweep_rows(const RowGroups<GS>& G, int64_t n, Bounds bounds, Term term,
                                  Done done) {
    for (int64_t r = G.first; r < n; r += 4 * G.step) {
        int64_t lo[4], hi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = r + u * G.step;
            bounds(q < n ? q : n - 1, lo[u], hi[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (r + u * G.step < n)
                done(r + u * G.step, lo[u], hi[u] - lo[u], group_row_sum<GS>(lo[u], hi[u], G.sub, term));
    }
}

// y_j = sum_i T_ij S_i; ratio_j = P_j / y_j (0 when y_j = 0).  An empty bin
// row is skipped: no entry of T^T refers to it, so its ratio is never read.
template <int GS>
__device__ inline void mlem_forward_rows(int64_t n_bins, const int64_t* __restrict__ rp,
                                         const int32_t* __restrict__ col,
                                         const float* __restrict__ val,
                                         const double* __restrict__ S,
                                         const float* __restrict__ P, double* __restrict__ ratio) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_rows(G, n_bins, [&](int64_t j, int64_t& lo, int64_t& hi) { lo = rp[j]; hi = rp[j + 1]; },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * S[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int64_t j, int64_t, int64_t len, double y) {
                   if (len > 0 && G.sub == 0) ratio[j] = y > 0.0 ? (double)P[j] / y : 0.0;
               });
}

__global__ __launch_bounds__(T256) void k_mlem_forward(int64_t n_bins, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const double* __restrict__ S,
                                                       const float* __restrict__ P,
                                                       double* __restrict__ ratio) {
    switch (lanes_per_row(rp[n_bins], n_bins)) {
        case 1: mlem_forward_rows<1>(n_bins, rp, col, val, S, P, ratio); break;
        case 4: mlem_forward_rows<4>(n_bins, rp, col, val, S, P, ratio); break;
        case 16: mlem_forward_rows<16>(n_bins, rp, col, val, S, P, ratio); break;
        default: mlem_forward_rows<64>(n_bins, rp, col, val, S, P, ratio); break;
    }
}

// Backprojection by bin slices.  When the ratio vector is larger than one
// XCD's L2 (4 MB) and T^T has at least 16 entries per voxel row, the bin
// range is cut into MLEM_SEGS equal slices and workgroup b works on slice
// b mod MLEM_SEGS only: workgroups are handed to the 8 XCDs in turn, so each
// XCD gathers from one slice of ratio (under 4 MB at 2^22 bins) that stays in
// its L2, instead of every gather missing to HBM.  Each voxel row is cut at
// the slice boundaries (binary search over its ascending columns, once per
// call); the MLEM_SEGS partial sums are added in slice order.  Any cut is
// correct (the pieces always partition the row), so rows whose columns are
// not ascending lose only the locality.
constexpr int MLEM_SEGS = 8;
constexpr int64_t MLEM_SEG_MIN_BINS = (int64_t)1 << 19;

__host__ __device__ inline bool mlem_sliced(int64_t n_bins, int64_t nnz, int64_t n_vox) {
    return n_bins >= MLEM_SEG_MIN_BINS && nnz >= 16 * n_vox;
}

// sb[i][s] (s = 0..MLEM_SEGS): first entry of voxel row i in slice s, with
// sb[i][0] = rp[i] and sb[i][MLEM_SEGS] = rp[i + 1]; non-decreasing in s.
__global__ __launch_bounds__(T256) void k_mlem_slices(int64_t n_vox, int64_t n_bins,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      int64_t* __restrict__ sb) {
    if (!mlem_sliced(n_bins, rp[n_vox], n_vox)) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = rp[i];
        const int64_t hi = rp[i + 1];
        int64_t* out = sb + i * (MLEM_SEGS + 1);
        out[0] = lo;
        for (int s = 1; s < MLEM_SEGS; ++s) {
            const int64_t bound = n_bins * s / MLEM_SEGS;
            int64_t a = lo, b = hi;
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if ((int64_t)col[mid] < bound) a = mid + 1; else b = mid;
            }
            out[s] = a;
            lo = a;
        }
        out[MLEM_SEGS] = hi;
    }
}

// S_i <- S_i * (sum_j T_ij ratio_j) / sens_i over whole voxel rows.  An
// empty row has sens_i = 0, so its S_i is already 0 and is skipped.
template <int GS>
__device__ inline void mlem_update_rows(int64_t n_vox, const int64_t* __restrict__ rp,
                                        const int32_t* __restrict__ col,
                                        const float* __restrict__ val,
                                        const double* __restrict__ ratio,
                                        const double* __restrict__ sens, double* __restrict__ S) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_rows(G, n_vox, [&](int64_t i, int64_t& lo, int64_t& hi) { lo = rp[i]; hi = rp[i + 1]; },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * ratio[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int64_t i, int64_t, int64_t len, double b) {
                   if (len > 0 && G.sub == 0) {
                       const double si = sens[i];
                       S[i] = si > 0.0 ? S[i] * b / si : 0.0;
                   }
               });
}

// part[s][i] = sum over the entries of voxel row i in slice s of T_ij ratio_j,
// slice s = blockIdx.x mod MLEM_SEGS (gridDim.x is a multiple of MLEM_SEGS).
template <int GS>
__device__ inline void mlem_back_slices(int64_t n_vox, const int64_t* __restrict__ sb,
                                        const int32_t* __restrict__ col,
                                        const float* __restrict__ val,
                                        const double* __restrict__ ratio,
                                        double* __restrict__ part) {
    const int seg = (int)(blockIdx.x % MLEM_SEGS);
    const RowGroups<GS> G(blockIdx.x / MLEM_SEGS, gridDim.x / MLEM_SEGS);
    sweep_rows(G, n_vox,
               [&](int64_t i, int64_t& lo, int64_t& hi) {
                   const int64_t* b = sb + i * (MLEM_SEGS + 1) + seg;
                   lo = b[0];
                   hi = b[1];
               },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * ratio[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int64_t i, int64_t, int64_t, double acc) {
                   if (G.sub == 0) part[(int64_t)seg * n_vox + i] = acc;
               });
}

__global__ __launch_bounds__(T256) void k_mlem_update(int64_t n_vox, int64_t n_bins,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ val,
                                                      const double* __restrict__ ratio,
                                                      const double* __restrict__ sens,
                                                      double* __restrict__ S,
                                                      const int64_t* __restrict__ sb,
                                                      double* __restrict__ part) {
    const int64_t nnz = rp[n_vox];
    if (mlem_sliced(n_bins, nnz, n_vox)) {
        switch (lanes_per_row(nnz, n_vox * MLEM_SEGS)) {
            case 1: mlem_back_slices<1>(n_vox, sb, col, val, ratio, part); break;
            case 4: mlem_back_slices<4>(n_vox, sb, col, val, ratio, part); break;
            case 16: mlem_back_slices<16>(n_vox, sb, col, val, ratio, part); break;
            default: mlem_back_slices<64>(n_vox, sb, col, val, ratio, part); break;
        }
        return;
    }
    switch (lanes_per_row(nnz, n_vox)) {
        case 1: mlem_update_rows<1>(n_vox, rp, col, val, ratio, sens, S); break;
        case 4: mlem_update_rows<4>(n_vox, rp, col, val, ratio, sens, S); break;
        case 16: mlem_update_rows<16>(n_vox, rp, col, val, ratio, sens, S); break;
        default: mlem_update_rows<64>(n_vox, rp, col, val, ratio, sens, S); break;
    }
}

// Sliced backprojection, second half: S_i <- S_i * (sum_s part[s][i]) / sens_i.
__global__ __launch_bounds__(T256) void k_mlem_combine(int64_t n_vox, int64_t n_bins,
                                                       const int64_t* __restrict__ rp,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ sens,
                                                       double* __restrict__ S) {
    if (!mlem_sliced(n_bins, rp[n_vox], n_vox)) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * blockDim.x) {
        double b = 0.0;
#pragma unroll
        for (int s = 0; s < MLEM_SEGS; ++s) b += part[(int64_t)s * n_vox + i];
        const double si = sens[i];
        S[i] = si > 0.0 ? S[i] * b / si : 0.0;
    }
}

__global__ __launch_bounds__(T256) void k_mlem_out(int64_t n_vox, const double* __restrict__ S,
                                                   float* __restrict__ img) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * blockDim.x)
        img[i] = (float)S[i];
}

// ---- ordered subsets (OSEM; dual matrix, Eq. DMOS; additive scatter, the
// Sohlberg OS-EM equation).  Subset k holds the views v with v mod n_sub == k.

// sens[k][i] = sum over the bins j of subset k of b_ij (row i of B^T)
__global__ __launch_bounds__(T256) void k_subset_sens(int64_t n_vox, const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ val,
                                                      int32_t bins_per_view, int32_t n_sub,
                                                      double* __restrict__ sens) {
    for (int k = 0; k < n_sub; ++k)
        for_rows(n_vox, rp,
                 [&](int64_t e) { return (col[e] / bins_per_view) % n_sub == k ? (double)val[e] : 0.0; },
                 [&](int64_t i, double acc) { sens[(int64_t)k * n_vox + i] = acc; });
}

__global__ __launch_bounds__(T256) void k_os_init(int64_t n_vox, int32_t n_sub,
                                                  const float* __restrict__ img,
                                                  const double* __restrict__ sens,
                                                  double* __restrict__ S) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * blockDim.x) {
        double tot = 0.0;
        for (int k = 0; k < n_sub; ++k) tot += sens[(int64_t)k * n_vox + i];
        S[i] = tot > 0.0 ? (double)img[i] : 0.0;
    }
}

// subset k: y_j = sum_i c_ij S_i + s_j, ratio_j = P_j / y_j on the subset's
// bins (row t of the subset is bin j of view k + n_sub * (t / bins_per_view));
// rows swept as in MLEM, the group size following the whole matrix's density
template <int GS>
__device__ inline void os_forward_rows(int64_t n_sub_bins, int32_t bins_per_view, int32_t n_sub,
                                       int32_t k, const int64_t* __restrict__ rp,
                                       const int32_t* __restrict__ col,
                                       const float* __restrict__ val,
                                       const double* __restrict__ S, const float* __restrict__ P,
                                       const float* __restrict__ scat, double* __restrict__ ratio) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    auto bin_of = [&](int64_t t) {
        const int64_t view = k + (int64_t)n_sub * (t / bins_per_view);
        return view * bins_per_view + t % bins_per_view;
    };
    sweep_rows(G, n_sub_bins,
               [&](int64_t t, int64_t& lo, int64_t& hi) {
                   const int64_t j = bin_of(t);
                   lo = rp[j];
                   hi = rp[j + 1];
               },
               [&](int64_t e, bool ok) {
                   const double x = (double)val[e] * S[col[e]];
                   return ok ? x : 0.0;
               },
               [&](int64_t t, int64_t, int64_t, double y) {
                   if (G.sub != 0) return;
                   const int64_t j = bin_of(t);
                   y += scat ? (double)scat[j] : 0.0;
                   ratio[j] = y > 0.0 ? (double)P[j] / y : 0.0;
               });
}

__global__ __launch_bounds__(T256) void k_os_forward(int64_t n_sub_bins, int32_t bins_per_view,
                                                     int32_t n_sub, int32_t k,
                                                     const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ val,
                                                     const double* __restrict__ S,
                                                     const float* __restrict__ P,
                                                     const float* __restrict__ scat,
                                                     double* __restrict__ ratio, int64_t n_bins) {
    switch (lanes_per_row(rp[n_bins], n_bins)) {
        case 1: os_forward_rows<1>(n_sub_bins, bins_per_view, n_sub, k, rp, col, val, S, P, scat, ratio); break;
        case 4: os_forward_rows<4>(n_sub_bins, bins_per_view, n_sub, k, rp, col, val, S, P, scat, ratio); break;
        case 16: os_forward_rows<16>(n_sub_bins, bins_per_view, n_sub, k, rp, col, val, S, P, scat, ratio); break;
        default: os_forward_rows<64>(n_sub_bins, bins_per_view, n_sub, k, rp, col, val, S, P, scat, ratio); break;
    }
}

// subset k: S_i <- S_i * (sum_{j in k} b_ij ratio_j) / sens_k,i (unchanged where sens_k,i = 0)
template <int GS>
__device__ inline void os_update_rows(int64_t n_vox, int32_t bins_per_view, int32_t n_sub, int32_t k,
                                      const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                      const float* __restrict__ val,
                                      const double* __restrict__ ratio,
                                      const double* __restrict__ sens, double* __restrict__ S) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_rows(G, n_vox, [&](int64_t i, int64_t& lo, int64_t& hi) { lo = rp[i]; hi = rp[i + 1]; },
               [&](int64_t e, bool ok) {
                   // every entry gathers its ratio (loads issued together);
                   // entries outside subset k then count 0.  Masking the
                   // gather instead serialises the loads and was slower.
                   const int32_t j = col[e];
                   const bool in_k = (j / bins_per_view) % n_sub == k;
                   const double x = (double)val[e] * ratio[j];
                   return ok && in_k ? x : 0.0;
               },
               [&](int64_t i, int64_t, int64_t, double bsum) {
                   if (G.sub != 0) return;
                   const double si = sens[(int64_t)k * n_vox + i];
                   if (si > 0.0) S[i] = S[i] * bsum / si;
               });
}

__global__ __launch_bounds__(T256) void k_os_update(int64_t n_vox, int32_t bins_per_view,
                                                    int32_t n_sub, int32_t k,
                                                    const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const double* __restrict__ ratio,
                                                    const double* __restrict__ sens,
                                                    double* __restrict__ S) {
    switch (lanes_per_row(rp[n_vox], n_vox)) {
        case 1: os_update_rows<1>(n_vox, bins_per_view, n_sub, k, rp, col, val, ratio, sens, S); break;
        case 4: os_update_rows<4>(n_vox, bins_per_view, n_sub, k, rp, col, val, ratio, sens, S); break;
        case 16: os_update_rows<16>(n_vox, bins_per_view, n_sub, k, rp, col, val, ratio, sens, S); break;
        default: os_update_rows<64>(n_vox, bins_per_view, n_sub, k, rp, col, val, ratio, sens, S); break;
    }
}

}  // namespace


size_t osem_workspace(uint64_t n_bins, uint64_t n_vox, uint32_t n_sub) {
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    return al(8 * n_vox * n_sub) /* sens per subset */ + al(8 * n_vox) /* S */ + al(8 * n_bins);
}

hipError_t launch_osem(int64_t n_bins, int64_t n_vox, int32_t bins_per_view, int32_t n_sub,
                       const int64_t* C_rp, const int32_t* C_col, const float* C_val,
                       const int64_t* Bt_rp, const int32_t* Bt_col, const float* Bt_val,
                       const float* proj, const float* scatter, float* image, int32_t n_iter,
                       void* workspace, hipStream_t s) {
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    char* w = (char*)workspace;
    double* sens = (double*)w;  w += al(8 * (uint64_t)n_vox * n_sub);
    double* S = (double*)w;     w += al(8 * (uint64_t)n_vox);
    double* ratio = (double*)w;
    const int64_t n_views = n_bins / bins_per_view;
    const int gv = grid_for((uint64_t)n_vox, T256, 8192);
    k_subset_sens<<<gv, T256, 0, s>>>(n_vox, Bt_rp, Bt_col, Bt_val, bins_per_view, n_sub, sens);
    k_os_init<<<gv, T256, 0, s>>>(n_vox, n_sub, image, sens, S);
    for (int it = 0; it < n_iter; ++it) {
        for (int k = 0; k < n_sub; ++k) {
            const int64_t views_k = (n_views - k + n_sub - 1) / n_sub;
            const int64_t nb = views_k * bins_per_view;
            if (nb <= 0) continue;
            k_os_forward<<<grid_for((uint64_t)nb, T256, 16384), T256, 0, s>>>(
                nb, bins_per_view, n_sub, k, C_rp, C_col, C_val, S, proj, scatter, ratio, n_bins);
            k_os_update<<<gv, T256, 0, s>>>(n_vox, bins_per_view, n_sub, k, Bt_rp, Bt_col, Bt_val,
                                            ratio, sens, S);
        }
    }
    k_mlem_out<<<gv, T256, 0, s>>>(n_vox, S, image);
    return hipGetLastError();
}

// Workspace of the response-matrix build, in bytes (layout below).
// Workspace of the response-matrix build (layout in sysmat_layout).
struct SysLayout {
    uint64_t* start;       // [nr + 1] row starts in the sorted items
    uint64_t* bsum;        // scan block sums
    uint32_t* hist;        // [RADIX * n_tiles] digit histograms
    uint64_t* offs;        // [RADIX * n_tiles + 1] their exclusive scan
    uint64_t* keys[2];     // [cap + 1] sort keys (double buffer; the spare one
                           //  then holds the run-head positions)
    int64_t* vals[2];      // [cap] weights, Q31.32
    uint32_t* flag;        // [cap] run heads
    unsigned long long* a_img;   // [n_img + 1] activity per image voxel, then the total
    size_t bytes;
};

SysLayout sysmat_layout(char* w, uint64_t n_bins, uint64_t n_img, uint64_t capacity) {
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    const uint64_t nr = n_bins > n_img ? n_bins : n_img;
    const uint64_t cap = capacity ? capacity : 1;
    const uint64_t n_tiles = (cap + RADIX_TILE - 1) / RADIX_TILE;
    uint64_t scan_n = nr;
    if (cap > scan_n) scan_n = cap;
    if (RADIX * n_tiles > scan_n) scan_n = RADIX * n_tiles;
    const uint64_t nb = (scan_n + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK;
    SysLayout L;
    char* p = w;
    auto take = [&](uint64_t bytes) { char* q = p; p += al(bytes); return q; };
    L.start = (uint64_t*)take(8 * (nr + 1));
    L.bsum = (uint64_t*)take(8 * nb);
    L.hist = (uint32_t*)take(4 * RADIX * n_tiles);
    L.offs = (uint64_t*)take(8 * (RADIX * n_tiles + 1));
    L.keys[0] = (uint64_t*)take(8 * (cap + 1));
    L.keys[1] = (uint64_t*)take(8 * (cap + 1));
    L.vals[0] = (int64_t*)take(8 * cap);
    L.vals[1] = (int64_t*)take(8 * cap);
    L.flag = (uint32_t*)take(4 * cap);
    L.a_img = (unsigned long long*)take(8 * (n_img + 1));
    L.bytes = (size_t)(p - w);
    return L;
}

size_t sysmat_workspace_bytes(uint64_t n_bins, uint64_t n_img, uint64_t capacity) {
    return sysmat_layout(nullptr, n_bins, n_img, capacity).bytes;
}

hipError_t launch_sysmat(const mc_event* events, const unsigned long long* n_events, uint64_t capacity,
                         uint32_t nx, uint32_t ny, uint32_t nz, uint32_t f, uint32_t n_views,
                         uint32_t nu, uint32_t nv, uint64_t n_hist, const uint32_t* activity,
                         uint32_t class_mask, int64_t* T_rp, int32_t* T_col, float* T_val,
                         int64_t* Tt_rp, int32_t* Tt_col, float* Tt_val, float* proj,
                         void* workspace, hipStream_t s) {
    const uint64_t n_bins = (uint64_t)n_views * nu * nv;
    const uint32_t mx = nx / f, my = ny / f, mz = nz / f;
    const uint64_t n_img = (uint64_t)mx * my * mz;
    const SysLayout L = sysmat_layout((char*)workspace, n_bins, n_img, capacity);
    const uint64_t cap = capacity ? capacity : 1;
    const uint32_t n_tiles = (uint32_t)((cap + RADIX_TILE - 1) / RADIX_TILE);
    unsigned long long* a_img = L.a_img;
    unsigned long long* total = a_img + n_img;

    SysArgs a;
    a.events = events; a.n_events = n_events; a.capacity = capacity;
    a.class_mask = class_mask;
    a.nv_nu = nu * nv;
    a.nx = nx; a.ny = ny; a.f = f; a.mx = mx; a.my = my;
    a.q_per_view = n_hist / n_views; a.r_extra = n_hist % n_views;

    k_fill_u64<<<grid_for(n_img + 1, T256, 4096), T256, 0, s>>>((uint64_t*)a_img, n_img + 1, 0);
    k_image_activity<<<grid_for((uint64_t)nx * ny * nz, T256, 8192), T256, 0, s>>>(
        activity, nx, ny, nz, f, mx, my, a_img, total);
    const int ge = grid_for(cap, T256, 8192);
    for (int transpose = 0; transpose < 2; ++transpose) {
        const uint64_t n_rows = transpose ? n_img : n_bins;
        const uint64_t n_cols = transpose ? n_bins : n_img;
        // rows 0..n_rows (n_rows: filtered events), columns 0..n_cols - 1
        const int col_bits = std::max(1, bit_width(n_cols - 1));
        const int key_bits = col_bits + bit_width(n_rows);
        k_make_keys<<<ge, T256, 0, s>>>(a, transpose, n_rows, col_bits, L.keys[0], L.vals[0]);
        int cur = 0;
        for (int shift = 0; shift < key_bits; shift += RADIX_BITS) {
            k_radix_hist<<<n_tiles, T256, 0, s>>>(L.keys[cur], a, shift, n_tiles, L.hist);
            hipError_t e = exclusive_scan(L.hist, (uint64_t)RADIX * n_tiles, L.offs, L.bsum, s);
            if (e != hipSuccess) return e;
            k_radix_scatter<<<n_tiles, T256, 0, s>>>(L.keys[cur], L.vals[cur], L.keys[cur ^ 1],
                                                     L.vals[cur ^ 1], a, shift, n_tiles, L.hist, L.offs);
            cur ^= 1;
        }
        const uint64_t* keys = L.keys[cur];
        const int64_t* w = L.vals[cur];
        uint64_t* head_pos = L.keys[cur ^ 1];
        k_row_starts<<<grid_for(n_rows + 1, T256, 8192), T256, 0, s>>>(keys, a, col_bits, n_rows, L.start);
        k_run_heads<<<ge, T256, 0, s>>>(keys, L.start, n_rows, cap, L.flag);
        hipError_t e = exclusive_scan(L.flag, cap, head_pos, L.bsum, s, L.start + n_rows);
        if (e != hipSuccess) return e;
        k_rows_from_runs<<<grid_for(n_rows + 1, T256, 8192), T256, 0, s>>>(
            L.start, head_pos, n_rows, transpose ? Tt_rp : T_rp);
        k_emit_runs<<<ge, T256, 0, s>>>(a, transpose, keys, w, L.start, head_pos, n_rows, col_bits,
                                        transpose ? Tt_col : T_col, transpose ? Tt_val : T_val,
                                        a_img, total);
        if (!transpose && proj)
            k_proj_rows<<<grid_for(n_rows, T256, 8192), T256, 0, s>>>(w, L.start, n_rows, proj);
    }
    return hipGetLastError();
}

size_t mlem_workspace(uint64_t n_bins, uint64_t n_vox) {
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    size_t b = al(8 * n_vox) /* sens */ + al(8 * n_vox) /* S */ + al(8 * n_bins) /* ratio */;
    if ((int64_t)n_bins >= MLEM_SEG_MIN_BINS)
        b += al(8 * (MLEM_SEGS + 1) * n_vox) /* slice cuts */ + al(8 * MLEM_SEGS * n_vox) /* partials */;
    return b;
}

hipError_t launch_mlem(int64_t n_bins, int64_t n_vox, const int64_t* T_rp, const int32_t* T_col,
                       const float* T_val, const int64_t* Tt_rp, const int32_t* Tt_col,
                       const float* Tt_val, const float* proj, float* image, int32_t n_iter,
                       void* workspace, hipStream_t s) {
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    char* w = (char*)workspace;
    double* sens = (double*)w;  w += al(8 * n_vox);
    double* S = (double*)w;     w += al(8 * n_vox);
    double* ratio = (double*)w; w += al(8 * n_bins);
    // slicing is decided on the device from nnz; n_bins alone rules it out
    const bool may_slice = n_bins >= MLEM_SEG_MIN_BINS;
    int64_t* sb = nullptr;
    double* part = nullptr;
    if (may_slice) {
        sb = (int64_t*)w;       w += al(8 * (MLEM_SEGS + 1) * (uint64_t)n_vox);
        part = (double*)w;
    }
    const int gv = grid_for((uint64_t)n_vox, T256, 8192);
    // The sweeps are grid-strided: one resident round of workgroups at most
    // (more only costs dispatch time and a ragged last round).
    int dev = 0, n_cu = 0, bpc_f = 0, bpc_u = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc_f, k_mlem_forward, T256, 0)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc_u, k_mlem_update, T256, 0)) != hipSuccess)
        return e;
    const int gb = grid_for((uint64_t)n_bins, T256, std::max(1, n_cu * bpc_f));
    const int gu = MLEM_SEGS * grid_for((uint64_t)n_vox, T256, std::max(1, n_cu * bpc_u / MLEM_SEGS));
    k_row_sums<<<gv, T256, 0, s>>>(n_vox, Tt_rp, Tt_val, sens);
    k_mlem_init<<<gv, T256, 0, s>>>(n_vox, image, sens, S);
    if (may_slice) k_mlem_slices<<<gv, T256, 0, s>>>(n_vox, n_bins, Tt_rp, Tt_col, sb);
    for (int it = 0; it < n_iter; ++it) {
        k_mlem_forward<<<gb, T256, 0, s>>>(n_bins, T_rp, T_col, T_val, S, proj, ratio);
        k_mlem_update<<<gu, T256, 0, s>>>(n_vox, n_bins, Tt_rp, Tt_col, Tt_val, ratio, sens, S, sb, part);
        if (may_slice) k_mlem_combine<<<gv, T256, 0, s>>>(n_vox, n_bins, Tt_rp, part, sens, S);
    }
    k_mlem_out<<<gv, T256, 0, s>>>(n_vox, S, image);
    return hipGetLastError();
}

}  // namespace mcs
