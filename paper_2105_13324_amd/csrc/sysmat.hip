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
// nothing; voxels with sens_i = 0 stay 0.  The non-empty rows are listed
// once per call and only they are swept, by groups of 1 to 64 lanes sized to
// their mean length; on large detectors the backprojection works on one bin
// slice per XCD so its gathers hit L2.
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
    for (uint64_t i = (uint64_t)blockIdx.x * T256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * T256) p[i] = v;
}

// activity per image voxel, and the total
__global__ __launch_bounds__(T256) void k_image_activity(const uint32_t* __restrict__ act,
                                                         uint32_t nx, uint32_t ny, uint32_t nz,
                                                         uint32_t f, uint32_t mx, uint32_t my,
                                                         unsigned long long* __restrict__ a_img,
                                                         unsigned long long* __restrict__ total) {
    const uint64_t n = (uint64_t)nx * ny * nz;
    uint64_t sum = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * T256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * T256) {
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
    for (uint64_t e = (uint64_t)blockIdx.x * T256 + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * T256) {
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
    for (uint64_t r = (uint64_t)blockIdx.x * T256 + threadIdx.x; r <= n_rows;
         r += (uint64_t)gridDim.x * T256) {
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
    for (uint64_t i = (uint64_t)blockIdx.x * T256 + threadIdx.x; i < n_valid;
         i += (uint64_t)gridDim.x * T256)
        flag[i] = i == 0 || keys[i] != keys[i - 1];
}

// rowptr[r] = distinct entries before row r (head_pos: exclusive scan of the run heads)
__global__ __launch_bounds__(T256) void k_rows_from_runs(const uint64_t* __restrict__ start,
                                                         const uint64_t* __restrict__ head_pos,
                                                         uint64_t n_rows, int64_t* __restrict__ rowptr) {
    for (uint64_t r = (uint64_t)blockIdx.x * T256 + threadIdx.x; r <= n_rows;
         r += (uint64_t)gridDim.x * T256)
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
    // a list that lost events (count above the capacity) gives no matrix
    const bool lost = *a.n_events > a.capacity;
    for (uint64_t i = (uint64_t)blockIdx.x * T256 + threadIdx.x; i < n_valid;
         i += (uint64_t)gridDim.x * T256) {
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
        val[o] = lost ? __builtin_nanf("") : (float)((double)cw * 0x1p-32 / n_i);
    }
}

// P_j = the summed weight of bin row j's events (all its items); NaN when
// the list lost events
__global__ __launch_bounds__(T256) void k_proj_rows(const int64_t* __restrict__ w,
                                                    const uint64_t* __restrict__ start,
                                                    uint64_t n_rows, const unsigned long long* n_events,
                                                    uint64_t capacity, float* __restrict__ proj) {
    const bool lost = *n_events > capacity;
    for (uint64_t r = (uint64_t)blockIdx.x * T256 + threadIdx.x; r < n_rows;
         r += (uint64_t)gridDim.x * T256) {
        long long tot = 0;
        for (uint64_t i = start[r]; i < start[r + 1]; ++i) tot += w[i];
        proj[r] = lost ? __builtin_nanf("") : (float)((double)tot * 0x1p-32);
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
    const int64_t tid = (int64_t)blockIdx.x * T256 + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * T256;
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

// MLEM state in the workspace (device uint32 [ST_WORDS]), written by the
// set-up of a matrix and kept for every later call on it: the lengths of the
// two row lists; a flag set when the entry count the caller gave is not the
// matrix's own; a flag set by each call when it does not match the set-up
// (its sizes differ from the fingerprint); for the compact layout, per
// matrix and per (group, length class) key (2 x 32), the rows counted, their
// first list position and an append cursor; the fingerprint (n_bins, n_vox,
// nnz).  With either flag set the iterations sweep nothing and the image is
// NaN.
enum {
    ST_BINS = 0, ST_VOXS = 1, ST_BAD = 2, ST_CALL_BAD = 3, ST_HIST = 4, ST_OFF = 68, ST_CUR = 132,
    ST_FP = 196, ST_WORDS = 200
};

// Set-up: the state zeroed, the entry count checked against both row-pointer
// arrays, the fingerprint stored (one workgroup).
__global__ __launch_bounds__(T256) void k_mlem_setup(int64_t n_bins, int64_t n_vox, int64_t nnz,
                                                     const int64_t* __restrict__ T_rp,
                                                     const int64_t* __restrict__ Tt_rp,
                                                     uint32_t* __restrict__ st) {
    const uint32_t t = threadIdx.x;
    if (t >= ST_WORDS) return;
    uint32_t v = 0;
    if (t == ST_BAD) v = (T_rp[n_bins] != nnz || Tt_rp[n_vox] != nnz) ? 1u : 0u;
    else if (t == ST_FP) v = (uint32_t)n_bins;
    else if (t == ST_FP + 1) v = (uint32_t)n_vox;
    else if (t == ST_FP + 2) v = (uint32_t)(uint64_t)nnz;
    else if (t == ST_FP + 3) v = (uint32_t)((uint64_t)nnz >> 32);
    st[t] = v;
}

// A call's sizes against the set-up's fingerprint (and its entry-count flag).
__device__ inline bool mlem_call_bad(const uint32_t* __restrict__ st, int64_t n_bins, int64_t n_vox,
                                     int64_t nnz) {
    return st[ST_BAD] != 0 || st[ST_FP] != (uint32_t)n_bins || st[ST_FP + 1] != (uint32_t)n_vox ||
           st[ST_FP + 2] != (uint32_t)(uint64_t)nnz || st[ST_FP + 3] != (uint32_t)((uint64_t)nnz >> 32);
}

// A non-empty row of a CSR matrix: its index and entry range.
struct RowRef {
    int64_t lo;
    int32_t row, len;
};

// The non-empty rows of T (bins[], length st[ST_BINS]) and of T^T (voxs[],
// length st[ST_VOXS]): only these are swept by the iterations (an empty bin
// row has no ratio to compute, an empty voxel row has sens_i = 0 and
// S_i = 0).  A workgroup takes 4096 consecutive rows of one matrix at a time
// and appends their non-empty ones in row order with one atomic; the order
// of the workgroups' runs varies from call to call, which changes no result,
// since every row is summed by one group of lanes on its own.  bin_pos /
// vox_pos (nullable): each row's list position, -1 for an empty row.
constexpr int ROWS_PER_THREAD = 16;
constexpr int ROW_CHUNK = T256 * ROWS_PER_THREAD;

__global__ __launch_bounds__(T256) void k_mlem_rows(int64_t n_bins, int64_t n_vox,
                                                    const int64_t* __restrict__ T_rp,
                                                    const int64_t* __restrict__ Tt_rp,
                                                    RowRef* __restrict__ bins,
                                                    RowRef* __restrict__ voxs,
                                                    int32_t* __restrict__ bin_pos,
                                                    int32_t* __restrict__ vox_pos,
                                                    uint32_t* __restrict__ st) {
    constexpr int WAVES = T256 / 64;
    __shared__ uint32_t before[ROWS_PER_THREAD * WAVES];
    __shared__ uint32_t base_s;
    if (st[ST_BAD]) return;
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const uint64_t lane_lt = (1ull << lane) - 1;
    const int64_t nbc = (n_bins + ROW_CHUNK - 1) / ROW_CHUNK;
    const int64_t nvc = (n_vox + ROW_CHUNK - 1) / ROW_CHUNK;
    for (int64_t c = blockIdx.x; c < nbc + nvc; c += gridDim.x) {
        const bool vox = c >= nbc;
        const int64_t r0 = (vox ? c - nbc : c) * ROW_CHUNK;
        const int64_t nr = vox ? n_vox : n_bins;
        const int64_t* rp = vox ? Tt_rp : T_rp;
        int32_t* pos = vox ? vox_pos : bin_pos;
        int64_t lo[ROWS_PER_THREAD];
        int32_t len[ROWS_PER_THREAD];
        uint64_t m[ROWS_PER_THREAD];
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) {
            const int64_t r = r0 + k * T256 + threadIdx.x;
            lo[k] = 0;
            len[k] = 0;
            if (r < nr) {
                lo[k] = rp[r];
                len[k] = (int32_t)(rp[r + 1] - lo[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) {
            m[k] = __ballot(len[k] > 0);
            if (lane == 0) before[k * WAVES + w] = (uint32_t)__popcll(m[k]);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // rows r0 + k * 256 + w * 64 + lane in (k, w, lane) order: row order
            uint32_t tot = 0;
            for (int q = 0; q < ROWS_PER_THREAD * WAVES; ++q) {
                const uint32_t x = before[q];
                before[q] = tot;
                tot += x;
            }
            base_s = tot ? atomicAdd(&st[vox ? ST_VOXS : ST_BINS], tot) : 0u;
        }
        __syncthreads();
        RowRef* out = vox ? voxs : bins;
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) {
            const int64_t r = r0 + k * T256 + threadIdx.x;
            const uint32_t slot = base_s + before[k * WAVES + w] + (uint32_t)__popcll(m[k] & lane_lt);
            if (len[k] > 0) out[slot] = RowRef{lo[k], (int32_t)r, len[k]};
            if (pos && r < nr) pos[r] = len[k] > 0 ? (int32_t)slot : -1;
        }
        __syncthreads();     // before[] and base_s are rewritten for the next chunk
    }
}

// Lanes that share one row in the MLEM sweeps: the smallest group of 1, 4, 16
// or 64 lanes for which four entries per lane cover the mean row (nnz /
// n_rows entries), so that short rows do not leave most of a wavefront idle.
// The kernel instantiated for lane-group size gs (1, 4, 16 or 64).
template <class K>
K by_group(int gs, K k1, K k4, K k16, K k64) {
    return gs == 1 ? k1 : gs == 4 ? k4 : gs == 16 ? k16 : k64;
}

__host__ __device__ inline int lanes_per_row(int64_t nnz, int64_t n_rows) {
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
        const int64_t t = block * T256 + threadIdx.x;
        first = t / GS;
        step = n_blocks * T256 / GS;
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

// A group's share of a row list: entries q = G.first + k G.step (k = 0, 1,
// ...), four per pass.  The first four entries are loaded together with the
// list's length (those past it are read from the list's spare capacity, cap
// entries in all, and dropped), so a sweep of short rows waits for three
// dependent loads (list entry, matrix entry, gathered vector entry), not
// four.  aux(q, valid, ref) loads a row's own operands (q clamped below cap)
// before its sum; done(q, ref, aux, sum) runs for every listed row.
template <int GS, class Aux, class Term, class Done>
__device__ inline void sweep_list(const RowGroups<GS>& G, const RowRef* __restrict__ L, int64_t cap,
                                  const uint32_t* __restrict__ count, const uint32_t* __restrict__ call_bad,
                                  Aux aux, Term term, Done done) {
    if (G.first >= cap) return;
    RowRef ref[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t q = G.first + u * G.step;
        ref[u] = L[q < cap ? q : cap - 1];
    }
    const uint32_t n_listed = *count, bad = *call_bad;
    // all six loads in flight before any is used (the compiler would
    // otherwise issue the rows' loads only once the length test has passed)
    asm volatile("" ::"v"(ref[0].lo), "v"(ref[1].lo), "v"(ref[2].lo), "v"(ref[3].lo), "s"(n_listed),
                 "s"(bad));
    const uint32_t n32 = bad ? 0u : n_listed;   // a call that does not match the set-up sweeps nothing
    const int64_t n = n32;
    for (int64_t r = G.first; r < n; r += 4 * G.step) {
        if (r != G.first) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = r + u * G.step;
                ref[u] = L[q < n ? q : n - 1];
            }
        }
        bool ok[4];
        decltype(aux(0, false, ref[0])) a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t q = r + u * G.step;
            ok[u] = q < n;
            a[u] = aux(q < cap ? q : cap - 1, ok[u], ref[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u])
                done(r + u * G.step, ref[u], a[u],
                     group_row_sum<GS>(ref[u].lo, ref[u].lo + ref[u].len, G.sub, term));
    }
}

// y_j = sum_i T_ij S_i; ratio_j = P_j / y_j (0 when y_j = 0), over the
// non-empty bin rows (an empty one is referred to by no entry of T^T, so its
// ratio is never read).
template <int GS>
__global__ __launch_bounds__(T256) void k_mlem_forward(const RowRef* __restrict__ L, int64_t cap,
                                                       const uint32_t* __restrict__ count,
                                                       const uint32_t* __restrict__ call_bad,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const double* __restrict__ S,
                                                       const float* __restrict__ P,
                                                       double* __restrict__ ratio) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_list(G, L, cap, count, call_bad,
               [&](int64_t, bool ok, const RowRef& r) { return P[ok ? r.row : 0]; },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * S[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int64_t, const RowRef& r, float p, double y) {
                   if (G.sub == 0) ratio[r.row] = y > 0.0 ? (double)p / y : 0.0;
               });
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

inline bool mlem_sliced(int64_t n_bins, int64_t nnz, int64_t n_vox) {
    return n_bins >= MLEM_SEG_MIN_BINS && nnz >= 16 * n_vox;
}

// sb[i][s] (s = 0..MLEM_SEGS): first entry of voxel row i in slice s, with
// sb[i][0] = rp[i] and sb[i][MLEM_SEGS] = rp[i + 1]; non-decreasing in s.
__global__ __launch_bounds__(T256) void k_mlem_slices(int64_t n_vox, int64_t n_bins,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      int64_t* __restrict__ sb) {
    for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * T256) {
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

// S_i <- S_i * (sum_j T_ij ratio_j) / sens_i over the non-empty voxel rows
// (an empty row has sens_i = 0, so its S_i is already 0).
template <int GS>
__global__ __launch_bounds__(T256) void k_mlem_update(const RowRef* __restrict__ L, int64_t cap,
                                                       const uint32_t* __restrict__ count,
                                                       const uint32_t* __restrict__ call_bad,
                                                      const int32_t* __restrict__ col,
                                                      const float* __restrict__ val,
                                                      const double* __restrict__ ratio,
                                                      const double* __restrict__ sens,
                                                      double* __restrict__ S) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_list(G, L, cap, count, call_bad,
               [&](int64_t, bool ok, const RowRef& r) {
                   const int64_t i = ok ? r.row : 0;
                   return double2{S[i], sens[i]};
               },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * ratio[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int64_t, const RowRef& r, double2 ss, double b) {
                   if (G.sub == 0) S[r.row] = ss.y > 0.0 ? ss.x * b / ss.y : 0.0;
               });
}

// ---- compact layout.  The non-empty rows of both matrices are listed in
// (group, length class) order; the list position of a row is the index of
// its entries in the iterated vectors.
//
// Groups.  Workgroups are handed to the 8 XCDs in turn, and workgroup b of a
// sweep works on group b mod 8, so the rows of one group are swept, and
// their vector entries written, by one XCD.  A voxel row's group is its
// eighth of the voxel index range (contiguous index ranges are slabs of
// planes); a bin row's group is that of the voxel of its first entry (for a
// parallel-hole camera, the slab its ray crosses).  Gathers then mostly read
// entries that the same XCD wrote in the previous sweep, still in its L2,
// rather than lines written back by other XCDs.  Any grouping is correct.
//
// Length classes.  Rows of at most 4, 16, 64 entries and longer ones are
// swept by groups of 1, 4, 16 and 64 lanes, one row per group and pass, so a
// row of up to 4 GS entries takes one load round of its group and a long row
// does not hold one lane for many rounds.  The lane-group size, and with it
// the summation order, depends only on the row's length.
constexpr int N_CLASS = 4;
constexpr int N_GROUP = 8;
constexpr int N_KEY = N_CLASS * N_GROUP;     // per matrix

__host__ __device__ inline int length_class(int64_t len) {
    return len <= 4 ? 0 : len <= 16 ? 1 : len <= 64 ? 2 : 3;
}

// The most rows class c can hold, of n rows and at most nnz entries.
__host__ __device__ inline int64_t class_capacity(int c, int64_t n, int64_t nnz) {
    const int64_t min_len[N_CLASS] = {1, 5, 17, 65};
    const int64_t m = nnz / min_len[c];
    return m < n ? m : n;
}

// A listed row of the compact layout (at its list position): its index and
// entry range.
struct ClassRef {
    int32_t row;
    uint32_t lo;
    int32_t len, pad;
};

// The entries of a listed row of at most four (length class 0), copied at
// its list position with columns renumbered: a sweep loads them together
// with the row's ClassRef instead of after it (one dependent load fewer).
// Slots past the row's length are unused.
struct alignas(16) ShortRow {
    int32_t col[4];
    float val[4];
};

// Compact layout (sparse matrices, nnz <= n_bins + n_vox): the iterations
// keep S, sens, P and the ratio in list order, and the column indices of both
// matrices are renumbered to list positions (Tc: voxel positions, Ttc: bin
// positions), so every gather falls in a vector of the non-empty rows only
// (a few MB at most, L2-resident) instead of a sparse scattering over the
// full bin and voxel ranges.  A column whose row in the other orientation is
// empty (the two orientations disagree) sets the bad flag.
__global__ __launch_bounds__(T256) void k_mlem_compact(int64_t nnz, const int32_t* __restrict__ T_col,
                                                       const int32_t* __restrict__ Tt_col,
                                                       const int32_t* __restrict__ bin_pos,
                                                       const int32_t* __restrict__ vox_pos,
                                                       int32_t* __restrict__ Tc, int32_t* __restrict__ Ttc,
                                                       const ClassRef* __restrict__ bins,
                                                       const ClassRef* __restrict__ voxs,
                                                       const float* __restrict__ T_val,
                                                       const float* __restrict__ Tt_val,
                                                       ShortRow* __restrict__ bin_short,
                                                       ShortRow* __restrict__ vox_short,
                                                       const double* __restrict__ sens,
                                                       double* __restrict__ sens_l, uint32_t* __restrict__ st) {
    if (st[ST_BAD]) return;
    const int64_t nb = st[ST_BINS], nv = st[ST_VOXS];
    const int64_t n = std::max(nnz, std::max(nb, nv));
    bool bad = false;
    // a short row's entries with the renumbering of Tc / Ttc (from the
    // original columns: Tc and Ttc are written by other threads of this pass)
    auto copy_short = [](const ClassRef& r, const int32_t* __restrict__ c, const float* __restrict__ v,
                         const int32_t* __restrict__ pos, ShortRow* __restrict__ out) {
        ShortRow e;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t p = k < r.len ? pos[c[r.lo + k]] : 0;
            e.col[k] = p < 0 ? 0 : p;
            e.val[k] = k < r.len ? v[r.lo + k] : 0.0f;
        }
        *out = e;
    };
    for (int64_t t = (int64_t)blockIdx.x * T256 + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * T256) {
        if (t < nnz) {
            const int32_t pv = vox_pos[T_col[t]], pb = bin_pos[Tt_col[t]];
            bad |= pv < 0 || pb < 0;
            Tc[t] = pv < 0 ? 0 : pv;
            Ttc[t] = pb < 0 ? 0 : pb;
        }
        if (t < nv) {
            const ClassRef r = voxs[t];
            sens_l[t] = sens[r.row];
            if (r.len <= 4) copy_short(r, Tt_col, Tt_val, bin_pos, vox_short + t);
        }
        if (t < nb) {
            const ClassRef r = bins[t];
            if (r.len <= 4) copy_short(r, T_col, T_val, vox_pos, bin_short + t);
        }
    }
    if (bad) atomicOr(&st[ST_BAD], 1u);
}

// Per call: the call checked against the set-up (ST_CALL_BAD), then the
// iterated vectors loaded: S = img where sens > 0, else 0, and for the
// compact layout P in list order (voxs / bins non-null).  In row order S and
// sens are indexed by voxel; in list order by list position.
__global__ __launch_bounds__(T256) void k_mlem_load(int64_t n_bins, int64_t n_vox, int64_t nnz,
                                                    const float* __restrict__ img,
                                                    const double* __restrict__ sens,
                                                    double* __restrict__ S, const float* __restrict__ P,
                                                    const ClassRef* __restrict__ bins,
                                                    const ClassRef* __restrict__ voxs,
                                                    float* __restrict__ P_l, uint32_t* __restrict__ st) {
    const bool bad = mlem_call_bad(st, n_bins, n_vox, nnz);
    if (blockIdx.x == 0 && threadIdx.x == 0) st[ST_CALL_BAD] = bad ? 1u : 0u;
    if (bad) return;
    const int64_t nv = voxs ? (int64_t)st[ST_VOXS] : n_vox, nb = bins ? (int64_t)st[ST_BINS] : 0;
    const int64_t n = std::max(nv, nb);
    for (int64_t t = (int64_t)blockIdx.x * T256 + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * T256) {
        if (t < nv) S[t] = sens[t] > 0.0 ? (double)img[voxs ? voxs[t].row : t] : 0.0;
        if (t < nb) P_l[t] = P[bins[t].row];
    }
}

// (group, class) key of a non-empty row: group by voxel index (a voxel row's
// own, a bin row's first column), class by length.
__device__ inline int row_key(int64_t vox, int64_t n_vox, int64_t len) {
    const int g = (int)(((uint64_t)vox * N_GROUP) / (uint64_t)n_vox);
    return g * N_CLASS + length_class(len);
}

// One matrix's rows in chunks of 4096 per workgroup: for each non-empty row,
// f(row, lo, len, key).  Rows of the bin matrix (col: its columns) take the
// group of their first column.
template <class F>
__device__ inline void for_listed_rows(int64_t r0, int64_t nr, const int64_t* __restrict__ rp,
                                       const int32_t* __restrict__ col, int64_t n_vox, F f) {
    // all row bounds, then all first columns, in flight before any is used
    int64_t lo[ROWS_PER_THREAD], len[ROWS_PER_THREAD];
    int32_t c0[ROWS_PER_THREAD];
#pragma unroll
    for (int k = 0; k < ROWS_PER_THREAD; ++k) {
        const int64_t r = r0 + k * T256 + threadIdx.x;
        lo[k] = 0;
        len[k] = 0;
        if (r < nr) {
            lo[k] = rp[r];
            len[k] = rp[r + 1] - lo[k];
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS_PER_THREAD; ++k) c0[k] = (col && len[k] > 0) ? col[lo[k]] : 0;
#pragma unroll
    for (int k = 0; k < ROWS_PER_THREAD; ++k) {
        const int64_t r = r0 + k * T256 + threadIdx.x;
        if (len[k] > 0) f(r, lo[k], len[k], row_key(col ? (int64_t)c0[k] : r, n_vox, len[k]));
    }
}

// Pass 1: rows per (matrix, key), one workgroup histogram per chunk.
__global__ __launch_bounds__(T256) void k_mlem_count(int64_t n_bins, int64_t n_vox,
                                                     const int64_t* __restrict__ T_rp,
                                                     const int32_t* __restrict__ T_col,
                                                     const int64_t* __restrict__ Tt_rp,
                                                     uint32_t* __restrict__ st) {
    __shared__ uint32_t h[N_KEY];
    if (st[ST_BAD]) return;
    const int64_t nbc = (n_bins + ROW_CHUNK - 1) / ROW_CHUNK, nvc = (n_vox + ROW_CHUNK - 1) / ROW_CHUNK;
    for (int64_t c = blockIdx.x; c < nbc + nvc; c += gridDim.x) {
        const bool vox = c >= nbc;
        if (threadIdx.x < N_KEY) h[threadIdx.x] = 0;
        __syncthreads();
        for_listed_rows((vox ? c - nbc : c) * ROW_CHUNK, vox ? n_vox : n_bins, vox ? Tt_rp : T_rp,
                        vox ? nullptr : T_col, n_vox,
                        [&](int64_t, int64_t, int64_t, int key) { atomicAdd(&h[key], 1u); });
        __syncthreads();
        if (threadIdx.x < N_KEY && h[threadIdx.x])
            atomicAdd(&st[ST_HIST + (vox ? N_KEY : 0) + threadIdx.x], h[threadIdx.x]);
        __syncthreads();
    }
}

// Pass 2 (one thread): each key's first list position, the list lengths,
// cursors zeroed.
__global__ void k_mlem_offsets(uint32_t* __restrict__ st) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st[ST_BAD]) return;
    for (int m = 0; m < 2; ++m) {
        uint32_t at = 0;
        for (int k = 0; k < N_KEY; ++k) {
            st[ST_OFF + m * N_KEY + k] = at;
            st[ST_CUR + m * N_KEY + k] = 0;
            at += st[ST_HIST + m * N_KEY + k];
        }
        st[m == 0 ? ST_BINS : ST_VOXS] = at;
    }
}

// Pass 3: each non-empty row at the next position of its key (one atomic per
// key and workgroup chunk; the order within a key varies from call to call,
// which changes no result: every row is summed by one lane group on its
// own); pos[row] = its position, -1 for an empty row.
__global__ __launch_bounds__(T256) void k_mlem_place(int64_t n_bins, int64_t n_vox,
                                                     const int64_t* __restrict__ T_rp,
                                                     const int32_t* __restrict__ T_col,
                                                     const int64_t* __restrict__ Tt_rp,
                                                     ClassRef* __restrict__ bins, ClassRef* __restrict__ voxs,
                                                     int32_t* __restrict__ bin_pos, int32_t* __restrict__ vox_pos,
                                                     uint32_t* __restrict__ st) {
    __shared__ uint32_t h[N_KEY], base[N_KEY];
    if (st[ST_BAD]) return;
    const int64_t nbc = (n_bins + ROW_CHUNK - 1) / ROW_CHUNK, nvc = (n_vox + ROW_CHUNK - 1) / ROW_CHUNK;
    for (int64_t c = blockIdx.x; c < nbc + nvc; c += gridDim.x) {
        const bool vox = c >= nbc;
        const int64_t r0 = (vox ? c - nbc : c) * ROW_CHUNK, nr = vox ? n_vox : n_bins;
        const int64_t* rp = vox ? Tt_rp : T_rp;
        int32_t* pos = vox ? vox_pos : bin_pos;
        ClassRef* out = vox ? voxs : bins;
        const uint32_t* off = st + ST_OFF + (vox ? N_KEY : 0);
        if (threadIdx.x < N_KEY) h[threadIdx.x] = 0;
        __syncthreads();
        // rank within the chunk's rows of the same key (packed: key << 16 | rank)
        uint32_t kr[ROWS_PER_THREAD];
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) kr[k] = 0xFFFFFFFFu;
        for_listed_rows(r0, nr, rp, vox ? nullptr : T_col, n_vox, [&](int64_t r, int64_t, int64_t, int key) {
            kr[(r - r0) / T256] = ((uint32_t)key << 16) | atomicAdd(&h[key], 1u);
        });
        __syncthreads();
        if (threadIdx.x < N_KEY)
            base[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&st[ST_CUR + (vox ? N_KEY : 0) + threadIdx.x],
                                                           h[threadIdx.x])
                                               : 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) {
            const int64_t r = r0 + k * T256 + threadIdx.x;
            if (r < nr) {
                int32_t q = -1;
                if (kr[k] != 0xFFFFFFFFu) {
                    const uint32_t key = kr[k] >> 16;
                    q = (int32_t)(off[key] + base[key] + (kr[k] & 0xFFFFu));
                    const int64_t lo = rp[r];
                    out[q] = ClassRef{(int32_t)r, (uint32_t)lo, (int32_t)(rp[r + 1] - lo), 0};
                }
                pos[r] = q;
            }
        }
        __syncthreads();     // h and base are rewritten for the next chunk
    }
}

// One (group, class) list by lane groups of GS (workgroup `block` of n_blocks
// for it), one row per group and pass.  aux(q) loads the row's own operands,
// done(q, aux, sum) runs on the group's first lane; q is the list position.
template <int GS, class Aux, class Term, class Done>
__device__ inline void sweep_key(int64_t block, int64_t n_blocks, const ClassRef* __restrict__ L,
                                 uint32_t first, uint32_t n, Aux aux, Term term, Done done) {
    const RowGroups<GS> G(block, n_blocks);
    for (int64_t r = G.first; r < (int64_t)n; r += G.step) {
        const ClassRef ref = L[first + r];
        const uint32_t q = first + (uint32_t)r;
        const auto a = aux(q);
        const double sum = group_row_sum<GS>(ref.lo, (int64_t)ref.lo + ref.len, G.sub, term);
        if (G.sub == 0) done(q, a, sum);
    }
}

// Class 0 (rows of at most four entries), one lane per row: the row's
// ClassRef and its ShortRow load together, then its (up to) four gathers.
// The terms are added in group_row_sum<1>'s order (a term past the row's
// length is 0), so the sum is the same bit for bit.
template <class Aux, class Gather, class Done>
__device__ inline void sweep_key_short(int64_t block, int64_t n_blocks, const ClassRef* __restrict__ L,
                                       const ShortRow* __restrict__ E, uint32_t first, uint32_t n, Aux aux,
                                       Gather gather, Done done) {
    const RowGroups<1> G(block, n_blocks);
    for (int64_t r = G.first; r < (int64_t)n; r += G.step) {
        const uint32_t q = first + (uint32_t)r;
        const int32_t len = L[q].len;
        const ShortRow e = E[q];
        const auto a = aux(q);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double x = (double)e.val[k] * gather(e.col[k]);
            acc += k < len ? x : 0.0;
        }
        done(q, a, acc);
    }
}

// The (group, class) lists of one matrix in one launch: workgroups [b.x, b.y)
// sweep class 0, [b.y, b.z) class 1, [b.z, b.w) class 2, [b.w, gridDim.x)
// class 3 (every range a multiple of N_GROUP); within a class, workgroup b
// works on group b mod N_GROUP.  key_st: that matrix's counts (ST_HIST) and
// first positions (ST_OFF).
template <class Aux, class Term, class Gather, class Done>
__device__ inline void sweep_keys(const ClassRef* __restrict__ L, const ShortRow* __restrict__ E,
                                  const uint32_t* __restrict__ hist, const uint32_t* __restrict__ off,
                                  const uint32_t* __restrict__ call_bad, int4 b, Aux aux, Term term,
                                  Gather gather, Done done) {
    const int64_t k = blockIdx.x;
    const int g = (int)(k % N_GROUP);
    int c;
    int64_t lo, hi;
    if (k < b.y) { c = 0; lo = b.x; hi = b.y; }
    else if (k < b.z) { c = 1; lo = b.y; hi = b.z; }
    else if (k < b.w) { c = 2; lo = b.z; hi = b.w; }
    else { c = 3; lo = b.w; hi = gridDim.x; }
    const int key = g * N_CLASS + c;
    // a call that does not match the set-up sweeps nothing (the three loads
    // are independent)
    const uint32_t first = off[key], n = *call_bad ? 0u : hist[key];
    const int64_t blk = (k - lo) / N_GROUP, nblk = (hi - lo) / N_GROUP;
    if (c == 0) sweep_key_short(blk, nblk, L, E, first, n, aux, gather, done);
    else if (c == 1) sweep_key<4>(blk, nblk, L, first, n, aux, term, done);
    else if (c == 2) sweep_key<16>(blk, nblk, L, first, n, aux, term, done);
    else sweep_key<64>(blk, nblk, L, first, n, aux, term, done);
}

// Compact forward: ratio_q = P_q / (sum_k val_k S[col_k]) over the bin rows,
// S, P, ratio in list order and col renumbered to voxel list positions.
__global__ __launch_bounds__(T256) void k_mlem_forward_c(const ClassRef* __restrict__ L,
                                                         const ShortRow* __restrict__ E,
                                                         const uint32_t* __restrict__ st, int4 b,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ val,
                                                         const double* __restrict__ S,
                                                         const float* __restrict__ P,
                                                         double* __restrict__ ratio) {
    sweep_keys(L, E, st + ST_HIST, st + ST_OFF, st + ST_CALL_BAD, b, [&](uint32_t q) { return P[q]; },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * S[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int32_t c) { return S[c]; },
               [&](uint32_t q, float p, double y) { ratio[q] = y > 0.0 ? (double)p / y : 0.0; });
}

// Compact update: S_q <- S_q (sum_k val_k ratio[col_k]) / sens_q over the
// voxel rows, in list order, col renumbered to bin list positions.
__global__ __launch_bounds__(T256) void k_mlem_update_c(const ClassRef* __restrict__ L,
                                                        const ShortRow* __restrict__ E,
                                                        const uint32_t* __restrict__ st, int4 b,
                                                        const int32_t* __restrict__ col,
                                                        const float* __restrict__ val,
                                                        const double* __restrict__ ratio,
                                                        const double* __restrict__ sens,
                                                        double* __restrict__ S) {
    sweep_keys(L, E, st + ST_HIST + N_KEY, st + ST_OFF + N_KEY, st + ST_CALL_BAD, b,
               [&](uint32_t q) { return double2{S[q], sens[q]}; },
               [&](int64_t k, bool ok) {
                   const double x = (double)val[k] * ratio[col[k]];
                   return ok ? x : 0.0;
               },
               [&](int32_t c) { return ratio[c]; },
               [&](uint32_t q, double2 ss, double v) { S[q] = ss.y > 0.0 ? ss.x * v / ss.y : 0.0; });
}

// part[s][i] = sum over the entries of voxel row i in slice s of T_ij ratio_j,
// slice s = blockIdx.x mod MLEM_SEGS (gridDim.x is a multiple of MLEM_SEGS).
template <int GS>
__global__ __launch_bounds__(T256) void k_mlem_back_slices(int64_t n_vox,
                                                           const int64_t* __restrict__ sb,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           const double* __restrict__ ratio,
                                                           double* __restrict__ part,
                                                           const uint32_t* __restrict__ call_bad) {
    if (*call_bad) return;   // the slices are the set-up's: a mismatched call reads none
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

// Sliced backprojection, second half: S_i <- S_i * (sum_s part[s][i]) / sens_i.
__global__ __launch_bounds__(T256) void k_mlem_combine(int64_t n_vox, const double* __restrict__ part,
                                                       const double* __restrict__ sens,
                                                       double* __restrict__ S,
                                                       const uint32_t* __restrict__ call_bad) {
    if (*call_bad) return;
    for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * T256) {
        double b = 0.0;
#pragma unroll
        for (int s = 0; s < MLEM_SEGS; ++s) b += part[(int64_t)s * n_vox + i];
        const double si = sens[i];
        S[i] = si > 0.0 ? S[i] * b / si : 0.0;
    }
}

// image_i = S_i (row order; vox_pos given: S in list order, 0 for an empty
// row), NaN throughout when the bad flag of st (nullable) is set.
__global__ __launch_bounds__(T256) void k_mlem_out(int64_t n_vox, const double* __restrict__ S,
                                                   const int32_t* __restrict__ vox_pos,
                                                   const uint32_t* __restrict__ st,
                                                   float* __restrict__ img) {
    const bool bad = st && (st[ST_BAD] != 0 || st[ST_CALL_BAD] != 0);
    for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * T256) {
        float v;
        if (bad) {
            v = __builtin_nanf("");
        } else if (vox_pos) {
            const int32_t p = vox_pos[i];
            v = p >= 0 ? (float)S[p] : 0.0f;
        } else {
            v = (float)S[i];
        }
        img[i] = v;
    }
}

// ---- ordered subsets (OSEM; dual matrix, Eq. DMOS; additive scatter, the
// Sohlberg OS-EM equation).  Subset k holds the views v with v mod n_sub == k.

// The backprojector split by subset, built once per call: for subset k and
// voxel i, the entries of row i of B^T whose bin lies in subset k, in their
// order in the row, at rows k * n_vox + i of one CSR (offsets off[], k-major),
// so that a subset's backprojection reads that subset's entries only instead
// of the whole of B^T once per subset.  One wavefront per row: 64 entries at
// a time, the distinct subsets among them taken in turn (a ballot matches
// the lanes of one subset); lane k of the wavefront keeps subset k's count
// (hence at most 64 subsets).

// st[2] (as for MLEM: the image is NaN when set): the entry count the caller
// gave is not B^T's own.
__global__ void k_os_check(int64_t n_vox, const int64_t* __restrict__ rp, int64_t nnz,
                           uint32_t* __restrict__ st) {
    if (blockIdx.x == 0 && threadIdx.x < 4) st[threadIdx.x] = threadIdx.x == 2 ? (rp[n_vox] != nnz) : 0u;
}

__device__ __forceinline__ int os_subset_of(int32_t bin, int32_t bins_per_view, int32_t n_sub) {
    return (bin / bins_per_view) % n_sub;
}

// cnt[k * n_vox + i] = entries of row i in subset k (all 0 when st[2] is set).
__global__ __launch_bounds__(T256) void k_os_split_count(int64_t n_vox, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         int32_t bins_per_view, int32_t n_sub,
                                                         uint32_t* __restrict__ cnt,
                                                         const uint32_t* __restrict__ st) {
    const bool bad = st[2] != 0;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t waves = (int64_t)gridDim.x * (T256 / 64);
    for (int64_t i = (int64_t)blockIdx.x * (T256 / 64) + (threadIdx.x >> 6); i < n_vox; i += waves) {
        uint32_t c = 0;                    // lane k: entries of subset k so far
        if (!bad) {
            const int64_t lo = rp[i], hi = rp[i + 1];
            for (int64_t e0 = lo; e0 < hi; e0 += 64) {
                const int64_t e = e0 + lane;
                const bool valid = e < hi;
                const int k = valid ? os_subset_of(col[e], bins_per_view, n_sub) : -1;
                uint64_t m = __ballot(valid);
                while (m != 0) {
                    const int kk = __builtin_amdgcn_readlane(k, __builtin_ctzll(m));
                    const uint64_t grp = __ballot(k == kk) & m;
                    if (lane == kk) c += (uint32_t)__popcll(grp);
                    m &= ~grp;
                }
            }
        }
        if (lane < n_sub) cnt[(int64_t)lane * n_vox + i] = c;
    }
}

// The entries moved to their subset rows: off[k * n_vox + i] is the first
// slot of subset k's row i (an exclusive scan of cnt).
__global__ __launch_bounds__(T256) void k_os_split_scatter(int64_t n_vox, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           int32_t bins_per_view, int32_t n_sub,
                                                           const uint64_t* __restrict__ off,
                                                           int32_t* __restrict__ col_s,
                                                           float* __restrict__ val_s,
                                                           const uint32_t* __restrict__ st) {
    if (st[2] != 0) return;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t waves = (int64_t)gridDim.x * (T256 / 64);
    for (int64_t i = (int64_t)blockIdx.x * (T256 / 64) + (threadIdx.x >> 6); i < n_vox; i += waves) {
        const int64_t lo = rp[i], hi = rp[i + 1];
        if (lo == hi) continue;           // wave-uniform
        // lane k: the next free slot of subset k's row i
        uint64_t next = lane < n_sub ? off[(int64_t)lane * n_vox + i] : 0;
        for (int64_t e0 = lo; e0 < hi; e0 += 64) {
            const int64_t e = e0 + lane;
            const bool valid = e < hi;
            const int32_t c = valid ? col[e] : 0;
            const float v = valid ? val[e] : 0.0f;
            const int k = valid ? os_subset_of(c, bins_per_view, n_sub) : -1;
            uint64_t m = __ballot(valid);
            while (m != 0) {
                const int kk = __builtin_amdgcn_readlane(k, __builtin_ctzll(m));
                const uint64_t grp = __ballot(k == kk) & m;
                const uint32_t lo32 = __builtin_amdgcn_readlane((uint32_t)next, kk);
                const uint32_t hi32 = __builtin_amdgcn_readlane((uint32_t)(next >> 32), kk);
                const uint64_t base = ((uint64_t)hi32 << 32) | lo32;
                if (k == kk) {
                    const uint64_t at = base + (uint64_t)__popcll(grp & ((1ull << lane) - 1ull));
                    col_s[at] = c;
                    val_s[at] = v;
                }
                if (lane == kk) next += (uint64_t)__popcll(grp);
                m &= ~grp;
            }
        }
    }
}

__global__ __launch_bounds__(T256) void k_os_init(int64_t n_vox, int32_t n_sub,
                                                  const float* __restrict__ img,
                                                  const double* __restrict__ sens,
                                                  double* __restrict__ S) {
    for (int64_t i = (int64_t)blockIdx.x * T256 + threadIdx.x; i < n_vox;
         i += (int64_t)gridDim.x * T256) {
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

// subset k: S_i <- S_i * (sum_{j in k} b_ij ratio_j) / sens_k,i (unchanged
// where sens_k,i = 0), over subset k's rows of the split backprojector
// (rp = off + k n_vox: row i spans [rp[i], rp[i + 1])).
template <int GS>
__global__ __launch_bounds__(T256) void k_os_update(int64_t n_vox, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const double* __restrict__ ratio,
                                                    const double* __restrict__ sens_k,
                                                    double* __restrict__ S) {
    const RowGroups<GS> G(blockIdx.x, gridDim.x);
    sweep_rows(G, n_vox, [&](int64_t i, int64_t& lo, int64_t& hi) { lo = rp[i]; hi = rp[i + 1]; },
               [&](int64_t e, bool ok) {
                   const double x = (double)val[e] * ratio[col[e]];
                   return ok ? x : 0.0;
               },
               [&](int64_t i, int64_t, int64_t, double bsum) {
                   if (G.sub != 0) return;
                   const double si = sens_k[i];
                   if (si > 0.0) S[i] = S[i] * bsum / si;
               });
}

}  // namespace


// OSEM workspace: per-subset sensitivities, S, the ratio, the check word,
// and the subset-split backprojector (counts, their scan and its block sums,
// columns and values).
struct OsemLayout {
    size_t sens, S, ratio, st, cnt, off, bsum, col_s, val_s, total;
};

OsemLayout osem_layout(uint64_t n_bins, uint64_t n_vox, uint32_t n_sub, uint64_t nnz) {
    OsemLayout L{};
    size_t o = 0;
    auto take = [&](uint64_t bytes) {
        const size_t at = o;
        o += (bytes + 255) & ~(uint64_t)255;
        return at;
    };
    const uint64_t rows = (uint64_t)n_sub * n_vox;
    L.sens = take(8 * rows);
    L.S = take(8 * n_vox);
    L.ratio = take(8 * n_bins);
    L.st = take(16);
    L.cnt = take(4 * rows);
    L.off = take(8 * (rows + 1));
    L.bsum = take(8 * ((rows + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK));
    L.col_s = take(4 * nnz);
    L.val_s = take(4 * nnz);
    L.total = o;
    return L;
}

size_t osem_workspace(uint64_t n_bins, uint64_t n_vox, uint32_t n_sub, uint64_t bt_nnz) {
    return osem_layout(n_bins, n_vox, n_sub, bt_nnz).total;
}

hipError_t launch_osem(int64_t n_bins, int64_t n_vox, int32_t bins_per_view, int32_t n_sub,
                       const int64_t* C_rp, const int32_t* C_col, const float* C_val,
                       const int64_t* Bt_rp, const int32_t* Bt_col, const float* Bt_val, int64_t bt_nnz,
                       const float* proj, const float* scatter, float* image, int32_t n_iter,
                       void* workspace, hipStream_t s) {
    const OsemLayout L = osem_layout((uint64_t)n_bins, (uint64_t)n_vox, (uint32_t)n_sub, (uint64_t)bt_nnz);
    char* w = (char*)workspace;
    double* sens = (double*)(w + L.sens);
    double* S = (double*)(w + L.S);
    double* ratio = (double*)(w + L.ratio);
    uint32_t* st = (uint32_t*)(w + L.st);
    uint32_t* cnt = (uint32_t*)(w + L.cnt);
    uint64_t* off = (uint64_t*)(w + L.off);
    int32_t* col_s = (int32_t*)(w + L.col_s);
    float* val_s = (float*)(w + L.val_s);
    const int64_t n_views = n_bins / bins_per_view;
    const uint64_t rows = (uint64_t)n_sub * (uint64_t)n_vox;
    const int gv = grid_for((uint64_t)n_vox, T256, 8192);
    const int gw = grid_for((uint64_t)n_vox, T256 / 64, 8192);     // one wavefront per row
    hipError_t e;
    k_os_check<<<1, 64, 0, s>>>(n_vox, Bt_rp, bt_nnz, st);
    k_os_split_count<<<gw, T256, 0, s>>>(n_vox, Bt_rp, Bt_col, bins_per_view, n_sub, cnt, st);
    if ((e = exclusive_scan(cnt, rows, off, (uint64_t*)(w + L.bsum), s)) != hipSuccess) return e;
    k_os_split_scatter<<<gw, T256, 0, s>>>(n_vox, Bt_rp, Bt_col, Bt_val, bins_per_view, n_sub, off, col_s,
                                           val_s, st);
    k_row_sums<<<grid_for(rows, T256, 8192), T256, 0, s>>>((int64_t)rows, (const int64_t*)off, val_s, sens);
    k_os_init<<<gv, T256, 0, s>>>(n_vox, n_sub, image, sens, S);
    // lanes per subset row from the mean subset row length
    const int gs_u = lanes_per_row(bt_nnz / n_sub, n_vox);
    auto ku = by_group(gs_u, k_os_update<1>, k_os_update<4>, k_os_update<16>, k_os_update<64>);
    for (int it = 0; it < n_iter; ++it) {
        for (int k = 0; k < n_sub; ++k) {
            const int64_t views_k = (n_views - k + n_sub - 1) / n_sub;
            const int64_t nb = views_k * bins_per_view;
            if (nb <= 0) continue;
            k_os_forward<<<grid_for((uint64_t)nb, T256, 16384), T256, 0, s>>>(
                nb, bins_per_view, n_sub, k, C_rp, C_col, C_val, S, proj, scatter, ratio, n_bins);
            ku<<<gv, T256, 0, s>>>(n_vox, (const int64_t*)(off + (uint64_t)k * (uint64_t)n_vox), col_s, val_s,
                                   ratio, sens + (uint64_t)k * (uint64_t)n_vox, S);
        }
    }
    k_mlem_out<<<gv, T256, 0, s>>>(n_vox, S, nullptr, st, image);
    return hipGetLastError();
}

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
            k_proj_rows<<<grid_for(n_rows, T256, 8192), T256, 0, s>>>(w, L.start, n_rows, n_events, capacity,
                                                                      proj);
    }
    return hipGetLastError();
}

namespace {

// Byte offsets of mlem_iterate's workspace, for n_bins x n_vox (every array
// 256-byte aligned).  The compact layout's arrays are sized for its largest
// entry count, n_bins + n_vox; the slice arrays exist for n_bins >= 2^19.
struct MlemLayout {
    size_t sens, S, ratio, bin_rows, vox_rows, st, sens_l, P_l, bin_pos, vox_pos, Tc, Ttc, bin_short, vox_short;
    size_t sb, part, total;
};

MlemLayout mlem_layout(uint64_t nb, uint64_t nv) {
    MlemLayout L{};
    size_t o = 0;
    auto take = [&](uint64_t bytes) {
        const size_t at = o;
        o += (bytes + 255) & ~(uint64_t)255;
        return at;
    };
    L.sens = take(8 * nv);
    L.S = take(8 * nv);
    L.ratio = take(8 * nb);
    L.bin_rows = take(16 * nb);
    L.vox_rows = take(16 * nv);
    L.st = take(4 * ST_WORDS);
    L.sens_l = take(8 * nv);
    L.P_l = take(4 * nb);
    L.bin_pos = take(4 * nb);
    L.vox_pos = take(4 * nv);
    L.Tc = take(4 * (nb + nv));
    L.Ttc = take(4 * (nb + nv));
    L.bin_short = take(sizeof(ShortRow) * nb);
    L.vox_short = take(sizeof(ShortRow) * nv);
    if ((int64_t)nb >= MLEM_SEG_MIN_BINS) {
        L.sb = take(8 * (MLEM_SEGS + 1) * nv);
        L.part = take(8 * MLEM_SEGS * nv);
    }
    L.total = o;
    return L;
}

}  // namespace

size_t mlem_workspace(uint64_t n_bins, uint64_t n_vox) { return mlem_layout(n_bins, n_vox).total; }

namespace {

// Workgroups for a sweep of at most `rows` rows by groups of gs lanes, four
// rows per group and pass: one pass when the device holds it, else one
// resident round (the sweeps are grid-strided; more workgroups would only
// cost dispatch time and a ragged last round).
template <class K>
hipError_t sweep_grid(K kernel, int64_t rows, int gs, int n_cu, int* grid) {
    int bpc = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, kernel, T256, 0);
    if (e != hipSuccess) return e;
    const uint64_t threads = ((uint64_t)std::max<int64_t>(rows, 1) + 3) / 4 * (uint64_t)gs;
    *grid = grid_for(threads, T256, std::max(1, n_cu * bpc));
    return hipSuccess;
}

}  // namespace

hipError_t launch_mlem(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rp,
                       const int32_t* T_col, const float* T_val, const int64_t* Tt_rp,
                       const int32_t* Tt_col, const float* Tt_val, const float* proj, float* image,
                       int32_t n_iter, void* workspace, int phases, hipStream_t s) {
    const uint64_t nb = (uint64_t)n_bins, nv = (uint64_t)n_vox;
    const MlemLayout Lo = mlem_layout(nb, nv);
    char* w = (char*)workspace;
    double* sens = (double*)(w + Lo.sens);
    double* S = (double*)(w + Lo.S);
    double* ratio = (double*)(w + Lo.ratio);
    RowRef* bin_rows = (RowRef*)(w + Lo.bin_rows);
    RowRef* vox_rows = (RowRef*)(w + Lo.vox_rows);
    uint32_t* st = (uint32_t*)(w + Lo.st);
    const bool setup = (phases & MLEM_SETUP) != 0, iterate = (phases & MLEM_ITERATE) != 0;
    // Layout: compact when the matrix is sparse (its renumbered columns fit
    // the workspace), else bin slices on large detectors, else row order.
    const bool compact = nnz <= n_bins + n_vox;
    const bool sliced = !compact && mlem_sliced(n_bins, nnz, n_vox);
    int dev = 0, n_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int gv = grid_for(nv, T256, 8192);
    const int gr = grid_for((nb + ROW_CHUNK - 1) / ROW_CHUNK + (nv + ROW_CHUNK - 1) / ROW_CHUNK, 1, 2048);
    if (setup) {
        k_row_sums<<<gv, T256, 0, s>>>(n_vox, Tt_rp, Tt_val, sens);
        k_mlem_setup<<<1, T256, 0, s>>>(n_bins, n_vox, nnz, T_rp, Tt_rp, st);
    }
    if (compact) {
        double* sens_l = (double*)(w + Lo.sens_l);
        float* P_l = (float*)(w + Lo.P_l);
        int32_t* bin_pos = (int32_t*)(w + Lo.bin_pos);
        int32_t* vox_pos = (int32_t*)(w + Lo.vox_pos);
        int32_t* Tc = (int32_t*)(w + Lo.Tc);
        int32_t* Ttc = (int32_t*)(w + Lo.Ttc);
        ClassRef* bin_list = (ClassRef*)(w + Lo.bin_rows);
        ClassRef* vox_list = (ClassRef*)(w + Lo.vox_rows);
        ShortRow* bin_short = (ShortRow*)(w + Lo.bin_short);
        ShortRow* vox_short = (ShortRow*)(w + Lo.vox_short);
        if (setup) {
            k_mlem_count<<<gr, T256, 0, s>>>(n_bins, n_vox, T_rp, T_col, Tt_rp, st);
            k_mlem_offsets<<<1, 64, 0, s>>>(st);
            k_mlem_place<<<gr, T256, 0, s>>>(n_bins, n_vox, T_rp, T_col, Tt_rp, bin_list, vox_list, bin_pos,
                                              vox_pos, st);
            k_mlem_compact<<<grid_for(std::max<uint64_t>((uint64_t)nnz, std::max(nb, nv)), T256, 8192), T256, 0,
                             s>>>(nnz, T_col, Tt_col, bin_pos, vox_pos, Tc, Ttc, bin_list, vox_list, T_val, Tt_val,
                                  bin_short, vox_short, sens, sens_l, st);
        }
        if (!iterate) return hipGetLastError();
        // Workgroups per class: each of the N_GROUP groups gets one pass over
        // a quarter of the rows the class can hold with nnz entries (groups
        // are uneven; the sweeps are grid-strided, so any count is correct),
        // the whole launch at most one resident round.
        int bpc_f = 0, bpc_u = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc_f, k_mlem_forward_c, T256, 0)) != hipSuccess)
            return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc_u, k_mlem_update_c, T256, 0)) != hipSuccess)
            return e;
        auto ranges = [&](int64_t n_rows, int bpc, int4* b) {
            const int gs[N_CLASS] = {1, 4, 16, 64};
            const int cap = std::max(1, n_cu * bpc / (N_CLASS * N_GROUP));
            int at = 0, start[N_CLASS];
            for (int c = 0; c < N_CLASS; ++c) {
                start[c] = at;
                const uint64_t lanes = ((uint64_t)class_capacity(c, n_rows, nnz) + 3) / 4 * gs[c];
                at += N_GROUP * grid_for(lanes, T256, cap);
            }
            *b = make_int4(start[0], start[1], start[2], start[3]);
            return at;
        };
        int4 bf, bu;
        const int gf = ranges(n_bins, bpc_f, &bf), gu = ranges(n_vox, bpc_u, &bu);
        k_mlem_load<<<grid_for(std::max(nb, nv), T256, 8192), T256, 0, s>>>(n_bins, n_vox, nnz, image, sens_l, S,
                                                                            proj, bin_list, vox_list, P_l, st);
        for (int it = 0; it < n_iter; ++it) {
            k_mlem_forward_c<<<gf, T256, 0, s>>>(bin_list, bin_short, st, bf, Tc, T_val, S, P_l, ratio);
            k_mlem_update_c<<<gu, T256, 0, s>>>(vox_list, vox_short, st, bu, Ttc, Tt_val, ratio, sens_l, S);
        }
        k_mlem_out<<<gv, T256, 0, s>>>(n_vox, S, vox_pos, st, image);
        return hipGetLastError();
    }
    int64_t* sb = sliced ? (int64_t*)(w + Lo.sb) : nullptr;
    double* part = sliced ? (double*)(w + Lo.part) : nullptr;
    if (setup) {
        k_mlem_rows<<<gr, T256, 0, s>>>(n_bins, n_vox, T_rp, Tt_rp, bin_rows, vox_rows, nullptr, nullptr, st);
        if (sliced) k_mlem_slices<<<gv, T256, 0, s>>>(n_vox, n_bins, Tt_rp, Tt_col, sb);
    }
    if (!iterate) return hipGetLastError();
    // Group sizes from the mean row length over all rows that can be
    // non-empty (at most nnz of them): the summation order depends only on
    // the matrix.
    const int64_t bin_rows_max = std::min(n_bins, std::max<int64_t>(nnz, 1));
    const int64_t vox_rows_max = std::min(n_vox, std::max<int64_t>(nnz, 1));
    const int gs_f = lanes_per_row(nnz, bin_rows_max);
    const int gs_u = sliced ? lanes_per_row(nnz, n_vox * MLEM_SEGS) : lanes_per_row(nnz, vox_rows_max);
    auto kf = by_group(gs_f, k_mlem_forward<1>, k_mlem_forward<4>, k_mlem_forward<16>, k_mlem_forward<64>);
    auto ku = by_group(gs_u, k_mlem_update<1>, k_mlem_update<4>, k_mlem_update<16>, k_mlem_update<64>);
    auto kb = by_group(gs_u, k_mlem_back_slices<1>, k_mlem_back_slices<4>, k_mlem_back_slices<16>,
                       k_mlem_back_slices<64>);
    int gb = 1, gu = 1;
    if ((e = sweep_grid(kf, bin_rows_max, gs_f, n_cu, &gb)) != hipSuccess) return e;
    if (sliced) {
        // one grid of slices: workgroup b on slice b mod MLEM_SEGS
        int per = 1;
        if ((e = sweep_grid(kb, n_vox, gs_u, std::max(1, n_cu / MLEM_SEGS), &per)) != hipSuccess) return e;
        gu = MLEM_SEGS * per;
    } else if ((e = sweep_grid(ku, vox_rows_max, gs_u, n_cu, &gu)) != hipSuccess) {
        return e;
    }
    k_mlem_load<<<gv, T256, 0, s>>>(n_bins, n_vox, nnz, image, sens, S, nullptr, nullptr, nullptr, nullptr, st);
    for (int it = 0; it < n_iter; ++it) {
        kf<<<gb, T256, 0, s>>>(bin_rows, n_bins, st + ST_BINS, st + ST_CALL_BAD, T_col, T_val, S, proj, ratio);
        if (sliced) {
            kb<<<gu, T256, 0, s>>>(n_vox, sb, Tt_col, Tt_val, ratio, part, st + ST_CALL_BAD);
            k_mlem_combine<<<gv, T256, 0, s>>>(n_vox, part, sens, S, st + ST_CALL_BAD);
        } else {
            ku<<<gu, T256, 0, s>>>(vox_rows, n_vox, st + ST_VOXS, st + ST_CALL_BAD, Tt_col, Tt_val, ratio, sens, S);
        }
    }
    k_mlem_out<<<gv, T256, 0, s>>>(n_vox, S, nullptr, st, image);
    return hipGetLastError();
}

}  // namespace mcs
