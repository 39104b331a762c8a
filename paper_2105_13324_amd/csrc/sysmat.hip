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
// Both orientations are built as CSR (bins x voxels and voxels x bins) by a
// deterministic counting sort: rows counted with integer atomics, scanned,
// scattered, each row's columns sorted and merged.  Weights are summed as
// Q31.32 integers, so the result does not depend on the atomics' order.
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

__global__ __launch_bounds__(T256) void k_sum_blocks(const uint32_t* __restrict__ in, uint64_t n,
                                                     uint64_t* __restrict__ bsum) {
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
__global__ __launch_bounds__(T256) void k_scan_write(const uint32_t* __restrict__ in, uint64_t n,
                                                     const uint64_t* __restrict__ bsum,
                                                     uint64_t* __restrict__ out) {
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

hipError_t exclusive_scan(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* bsum,
                          hipStream_t s) {
    // one extra item so the block holding index n writes the total
    const int nb = (int)((n + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK);
    k_sum_blocks<<<nb, T256, 0, s>>>(in, n, bsum);
    k_scan_blocks<<<1, 1024, 0, s>>>(bsum, nb);
    k_scan_write<<<nb, T256, 0, s>>>(in, n, bsum, out);
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

__global__ __launch_bounds__(T256) void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
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

// count events per row (transpose = 0: rows are bins, 1: rows are image voxels)
__global__ __launch_bounds__(T256) void k_count_rows(SysArgs a, int transpose, uint32_t* cnt) {
    const uint64_t n = n_events_of(a);
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t bin, img;
        if (!event_rc(a, a.events[e], bin, img)) continue;
        atomicAdd(cnt + (transpose ? img : bin), 1u);
    }
}

__global__ __launch_bounds__(T256) void k_scatter(SysArgs a, int transpose, const uint64_t* start,
                                                  uint32_t* fill, uint32_t* tmp_col, int64_t* tmp_w) {
    const uint64_t n = n_events_of(a);
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t bin, img;
        const mc_event ev = a.events[e];
        if (!event_rc(a, ev, bin, img)) continue;
        const uint32_t r = transpose ? img : bin, c = transpose ? bin : img;
        const uint32_t k = atomicAdd(fill + r, 1u);
        tmp_col[start[r] + k] = c;
        tmp_w[start[r] + k] = ev.weight;
    }
}

// Sift-down of heap node i over [0, n) of the row (col keys, weights carried).
__device__ inline void sift(uint32_t* col, int64_t* w, uint64_t i, uint64_t n) {
    for (;;) {
        uint64_t m = i;
        const uint64_t l = 2 * i + 1, r = l + 1;
        if (l < n && col[l] > col[m]) m = l;
        if (r < n && col[r] > col[m]) m = r;
        if (m == i) return;
        const uint32_t tc = col[i]; col[i] = col[m]; col[m] = tc;
        const int64_t tw = w[i]; w[i] = w[m]; w[m] = tw;
        i = m;
    }
}

constexpr uint64_t ROW_SHORT = 32;      // rows up to this length: one thread, insertion sort
constexpr uint64_t ROW_LDS = 4096;      // rows up to this length: one wavefront, LDS bitonic sort
constexpr uint64_t ROW_BIG = 8192;      // rows up to this length: one 256-thread block, LDS bitonic sort

// sort each row's (column, weight) pairs by column and count the distinct
// columns: short rows (analog lists) by insertion sort here; longer rows are
// left to k_sort_rows_wave and k_sort_rows_block.  With heap = 1 the kernel
// instead heapsorts the rows k_sort_rows_block could not take (marked
// ROW_OVERFLOW in row_nnz).
constexpr uint32_t ROW_OVERFLOW = 0xFFFFFFFFu;

__global__ __launch_bounds__(T256) void k_sort_rows(uint64_t n_rows, const uint64_t* start,
                                                    uint32_t* tmp_col, int64_t* tmp_w,
                                                    uint32_t* row_nnz, int heap) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = start[r], e = start[r + 1], n = e - b;
        uint32_t* col = tmp_col + b;
        int64_t* w = tmp_w + b;
        if (heap ? row_nnz[r] != ROW_OVERFLOW : n > ROW_SHORT) continue;
        if (n <= ROW_SHORT) {
            for (uint64_t i = 1; i < n; ++i) {
                const uint32_t v = col[i];
                const int64_t wv = w[i];
                uint64_t j = i;
                while (j > 0 && col[j - 1] > v) { col[j] = col[j - 1]; w[j] = w[j - 1]; --j; }
                col[j] = v;
                w[j] = wv;
            }
        } else {
            for (uint64_t i = n / 2; i-- > 0;) sift(col, w, i, n);
            for (uint64_t k = n - 1; k > 0; --k) {
                const uint32_t tc = col[0]; col[0] = col[k]; col[k] = tc;
                const int64_t tw = w[0]; w[0] = w[k]; w[k] = tw;
                sift(col, w, 0, k);
            }
        }
        uint32_t d = 0;
        for (uint64_t i = b; i < e; ++i) d += (i == b || tmp_col[i] != tmp_col[i - 1]);
        row_nnz[r] = d;
    }
}

// one wavefront per row of ROW_SHORT < length <= 1024 (two classes):
// bitonic sort of the (column, weight) pairs in LDS, padded to a power of
// two, then the count of distinct columns
// Instantiated per length class (LO, HI] so that the LDS a wavefront holds
// (12 B per entry) fits the class and short-row classes keep many
// wavefronts resident per CU.
template <uint32_t LO, uint32_t HI>
__global__ __launch_bounds__(64) void k_sort_rows_wave(uint64_t n_rows, const uint64_t* start,
                                                       uint32_t* tmp_col, int64_t* tmp_w,
                                                       uint32_t* row_nnz) {
    __shared__ uint32_t key[HI];
    __shared__ int64_t wt[HI];
    const uint32_t lane = threadIdx.x;
    // 64 rows are screened at once (a lane each; rows gridDim.x apart, so
    // runs of long rows spread over the grid); the wavefront then sorts the
    // ones of this length class in turn
    const uint64_t stride = gridDim.x;
    for (uint64_t r0 = blockIdx.x; r0 < n_rows; r0 += stride * 64) {
        bool need = false;
        const uint64_t rl = r0 + lane * stride;
        if (rl < n_rows) {
            const uint64_t len = start[rl + 1] - start[rl];
            need = len > LO && len <= HI;
        }
        for (uint64_t todo = __ballot(need); todo != 0; todo &= todo - 1) {
            const uint64_t r = r0 + (uint64_t)(__ffsll((unsigned long long)todo) - 1) * stride;
            const uint64_t b = start[r], n = start[r + 1] - b;
            uint32_t m = 1;
            while (m < n) m <<= 1;
            for (uint32_t i = lane; i < m; i += 64) {
                key[i] = i < n ? tmp_col[b + i] : 0xFFFFFFFFu;
                wt[i] = i < n ? tmp_w[b + i] : 0;
            }
            __syncthreads();
            for (uint32_t k = 2; k <= m; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = lane; i < m; i += 64) {
                        const uint32_t x = i ^ j;
                        if (x > i) {
                            const bool up = (i & k) == 0;
                            const uint32_t ki = key[i], kx = key[x];
                            if ((ki > kx) == up) {
                                key[i] = kx; key[x] = ki;
                                const int64_t t = wt[i]; wt[i] = wt[x]; wt[x] = t;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            uint32_t d = 0;
            for (uint32_t i = lane; i < n; i += 64) {
                tmp_col[b + i] = key[i];
                tmp_w[b + i] = wt[i];
                d += (i == 0 || key[i] != key[i - 1]);
            }
            for (int o = 32; o > 0; o >>= 1) d += (uint32_t)__shfl_xor((int)d, o, 64);
            if (lane == 0) row_nnz[r] = d;
            __syncthreads();
        }
    }
}

// one 256-thread block per row longer than 1024 entries (the dense voxel
// rows of forced-detection matrices), in 48 KB of LDS up to ROW_LDS entries
// and 96 KB up to ROW_BIG: the same bitonic sort.  Longer rows: their
// entries are first summed per
// column in an LDS hash table of ROW_BIG slots (64-bit integer adds: exact,
// so the order does not matter), the table is sorted, and the row is
// rewritten as its distinct columns with their sums followed by copies of
// the last column with weight 0 (which the merge adds as 0); a row with more
// than ROW_BIG distinct columns is marked ROW_OVERFLOW for the heapsort.  A
// block screens 256 rows per step (rows gridDim.x apart), lists the long
// ones and sorts them in turn.
// Instantiated per class: rows of (LO, CAP] entries are sorted in CAP
// slots; with AGG also every longer row goes through the column sums.
__device__ inline uint32_t col_hash(uint32_t c) { return (c * 2654435761u) >> 19; }   // 13 bits

template <uint32_t LO, uint32_t CAP, bool AGG>
__global__ __launch_bounds__(T256) void k_sort_rows_block(uint64_t n_rows, const uint64_t* start,
                                                          uint32_t* tmp_col, int64_t* tmp_w,
                                                          uint32_t* row_nnz) {
    static_assert(!AGG || CAP == 8192, "col_hash gives 13 bits");
    __shared__ uint32_t key[CAP];
    __shared__ int64_t wt[CAP];
    __shared__ uint32_t list[T256];
    __shared__ uint32_t n_list, n_distinct, overflow;
    const uint32_t t = threadIdx.x;
    const uint64_t stride = gridDim.x;
    for (uint64_t r0 = blockIdx.x; r0 < n_rows; r0 += stride * T256) {
        if (t == 0) n_list = 0;
        __syncthreads();
        const uint64_t rl = r0 + t * stride;
        if (rl < n_rows) {
            const uint64_t len = start[rl + 1] - start[rl];
            if (len > LO && (AGG || len <= CAP)) list[atomicAdd(&n_list, 1u)] = t;
        }
        __syncthreads();
        const uint32_t nl = n_list;
        for (uint32_t q = 0; q < nl; ++q) {
            const uint64_t r = r0 + (uint64_t)list[q] * stride;
            const uint64_t b = start[r], n = start[r + 1] - b;
            const bool agg = AGG && n > CAP;
            uint32_t m = CAP;
            if (!agg) {
                m = 1;
                while (m < n) m <<= 1;
                for (uint32_t i = t; i < m; i += T256) {
                    key[i] = i < n ? tmp_col[b + i] : 0xFFFFFFFFu;
                    wt[i] = i < n ? tmp_w[b + i] : 0;
                }
            } else {
                for (uint32_t i = t; i < CAP; i += T256) { key[i] = 0xFFFFFFFFu; wt[i] = 0; }
            }
            if (t == 0) { n_distinct = 0; overflow = 0; }
            __syncthreads();
            if (agg) {
                for (uint64_t i = t; i < n; i += T256) {
                    const uint32_t c = tmp_col[b + i];
                    const int64_t w = tmp_w[b + i];
                    uint32_t h = col_hash(c);
                    uint32_t probe = 0;
                    for (; probe < CAP; ++probe, h = (h + 1) & (CAP - 1)) {
                        const uint32_t cur = atomicCAS(&key[h], 0xFFFFFFFFu, c);
                        if (cur == 0xFFFFFFFFu || cur == c) {
                            atomicAdd((unsigned long long*)&wt[h], (unsigned long long)w);
                            break;
                        }
                    }
                    if (probe == CAP) overflow = 1;
                }
                __syncthreads();
                if (overflow) {                   // left to the heapsort
                    if (t == 0) row_nnz[r] = ROW_OVERFLOW;
                    __syncthreads();
                    continue;
                }
            }
            for (uint32_t k = 2; k <= m; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = t; i < m; i += T256) {
                        const uint32_t x = i ^ j;
                        if (x > i) {
                            const bool up = (i & k) == 0;
                            const uint32_t ki = key[i], kx = key[x];
                            if ((ki > kx) == up) {
                                key[i] = kx; key[x] = ki;
                                const int64_t tw = wt[i]; wt[i] = wt[x]; wt[x] = tw;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            if (!agg) {
                uint32_t d = 0;
                for (uint32_t i = t; i < n; i += T256) {
                    tmp_col[b + i] = key[i];
                    tmp_w[b + i] = wt[i];
                    d += (i == 0 || key[i] != key[i - 1]);
                }
                atomicAdd(&n_distinct, d);
            } else {
                // distinct columns: the slots before the first empty one
                uint32_t d = 0;
                for (uint32_t i = t; i < CAP; i += T256) d += key[i] != 0xFFFFFFFFu;
                atomicAdd(&n_distinct, d);
                __syncthreads();
                const uint32_t nd = n_distinct;
                for (uint64_t i = t; i < n; i += T256) {
                    tmp_col[b + i] = i < nd ? key[i] : key[nd - 1];
                    tmp_w[b + i] = i < nd ? wt[i] : 0;
                }
            }
            __syncthreads();
            if (t == 0) row_nnz[r] = n_distinct;
            __syncthreads();
        }
    }
}

// distinct columns with their counts -> CSR column and value arrays
__global__ __launch_bounds__(T256) void k_emit_rows(SysArgs a, int transpose, uint64_t n_rows,
                                                    const uint64_t* start, const uint32_t* tmp_col,
                                                    const int64_t* tmp_w,
                                                    const uint64_t* rowptr_u, int64_t* rowptr,
                                                    int32_t* col, float* val,
                                                    const unsigned long long* a_img,
                                                    const unsigned long long* total_p, float* proj) {
    const double total = (double)*total_p;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n_rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        rowptr[r] = (int64_t)rowptr_u[r];
        if (r == n_rows) continue;
        const uint64_t b = start[r], e = start[r + 1];
        if (e - b > ROW_SHORT) continue;          // k_emit_rows_wave
        uint64_t o = rowptr_u[r];
        if (!transpose && proj) {
            long long tot = 0;
            for (uint64_t i = b; i < e; ++i) tot += tmp_w[i];
            proj[r] = (float)((double)tot * 0x1p-32);
        }
        uint64_t i = b;
        while (i < e) {
            const uint32_t c = tmp_col[i];
            uint64_t j = i;
            long long cw = 0;
            while (j < e && tmp_col[j] == c) { cw += tmp_w[j]; ++j; }
            const uint32_t bin = transpose ? c : (uint32_t)r;
            const uint32_t img = transpose ? (uint32_t)r : c;
            const uint64_t view = bin / a.nv_nu;
            const double n_view = (double)(a.q_per_view + (view < a.r_extra ? 1u : 0u));
            const double n_i = n_view * (double)a_img[img] / total;
            col[o] = (int32_t)c;
            val[o] = (float)((double)cw * 0x1p-32 / n_i);
            ++o;
            i = j;
        }
    }
}


// The same for rows longer than ROW_SHORT, one wavefront per row: the lanes
// take 64 consecutive entries at a time, each entry that starts a run of
// equal columns gets its output slot from a ballot and sums its run (runs
// are short), so the reads are coalesced.  Rows are screened 64 at a time,
// gridDim.x apart.
__global__ __launch_bounds__(64) void k_emit_rows_wave(SysArgs a, int transpose, uint64_t n_rows,
                                                       const uint64_t* start, const uint32_t* tmp_col,
                                                       const int64_t* tmp_w, const uint64_t* rowptr_u,
                                                       int32_t* col, float* val,
                                                       const unsigned long long* a_img,
                                                       const unsigned long long* total_p, float* proj) {
    const double total = (double)*total_p;
    const uint32_t lane = threadIdx.x;
    const uint64_t lane_lt = (1ull << lane) - 1ull;
    const uint64_t stride = gridDim.x;
    for (uint64_t r0 = blockIdx.x; r0 < n_rows; r0 += stride * 64) {
        bool need = false;
        const uint64_t rl = r0 + lane * stride;
        if (rl < n_rows) need = start[rl + 1] - start[rl] > ROW_SHORT;
        for (uint64_t todo = __ballot(need); todo != 0; todo &= todo - 1) {
            const uint64_t r = r0 + (uint64_t)(__ffsll((unsigned long long)todo) - 1) * stride;
            const uint64_t b = start[r], e = start[r + 1];
            uint64_t o = rowptr_u[r];
            long long tot = 0;
            for (uint64_t c0 = b; c0 < e; c0 += 64) {
                const uint64_t i = c0 + lane;
                const bool valid = i < e;
                uint32_t c = 0;
                bool first = false;
                if (valid) {
                    c = tmp_col[i];
                    tot += tmp_w[i];
                    first = i == b || tmp_col[i - 1] != c;
                }
                const uint64_t m = __ballot(first);
                if (first) {
                    long long cw = 0;
                    for (uint64_t j = i; j < e && tmp_col[j] == c; ++j) cw += tmp_w[j];
                    const uint32_t bin = transpose ? c : (uint32_t)r;
                    const uint32_t img = transpose ? (uint32_t)r : c;
                    const uint64_t view = bin / a.nv_nu;
                    const double n_view = (double)(a.q_per_view + (view < a.r_extra ? 1u : 0u));
                    const double n_i = n_view * (double)a_img[img] / total;
                    const uint64_t slot = o + (uint64_t)__popcll(m & lane_lt);
                    col[slot] = (int32_t)c;
                    val[slot] = (float)((double)cw * 0x1p-32 / n_i);
                }
                o += (uint64_t)__popcll(m);
            }
            if (!transpose && proj) {
                for (int k = 32; k > 0; k >>= 1) tot += __shfl_xor(tot, k, 64);
                if (lane == 0) proj[r] = (float)((double)tot * 0x1p-32);
            }
        }
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
// bins (row t of the subset is bin j of view k + n_sub * (t / bins_per_view))
__global__ __launch_bounds__(T256) void k_os_forward(int64_t n_sub_bins, int32_t bins_per_view,
                                                     int32_t n_sub, int32_t k,
                                                     const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const float* __restrict__ val,
                                                     const double* __restrict__ S,
                                                     const float* __restrict__ P,
                                                     const float* __restrict__ scat,
                                                     double* __restrict__ ratio, int64_t n_bins) {
    // the mode follows the whole matrix's density (the subset rows are a
    // view-interleaved part of it)
    const bool wave_mode = rp[n_bins] >= WAVE_ROW_MIN * n_bins;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    const int64_t step = wave_mode ? 64 : 1;
    const int64_t first = wave_mode ? lane : 0;
    for (int64_t t = wave_mode ? tid >> 6 : tid; t < n_sub_bins; t += wave_mode ? nt >> 6 : nt) {
        const int64_t view = k + (int64_t)n_sub * (t / bins_per_view);
        const int64_t j = view * bins_per_view + t % bins_per_view;
        double y = 0.0;
        for (int64_t e = rp[j] + first; e < rp[j + 1]; e += step) y += (double)val[e] * S[col[e]];
        if (wave_mode) y = wave_sum_f64(y);
        if (!wave_mode || lane == 0) {
            y += scat ? (double)scat[j] : 0.0;
            ratio[j] = y > 0.0 ? (double)P[j] / y : 0.0;
        }
    }
}

// subset k: S_i <- S_i * (sum_{j in k} b_ij ratio_j) / sens_k,i (unchanged where sens_k,i = 0)
__global__ __launch_bounds__(T256) void k_os_update(int64_t n_vox, int32_t bins_per_view,
                                                    int32_t n_sub, int32_t k,
                                                    const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const double* __restrict__ ratio,
                                                    const double* __restrict__ sens,
                                                    double* __restrict__ S) {
    for_rows(n_vox, rp,
             [&](int64_t e) {
                 const int32_t j = col[e];
                 return (j / bins_per_view) % n_sub == k ? (double)val[e] * ratio[j] : 0.0;
             },
             [&](int64_t i, double bsum) {
                 const double si = sens[(int64_t)k * n_vox + i];
                 if (si > 0.0) S[i] = S[i] * bsum / si;
             });
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
size_t sysmat_workspace_bytes(uint64_t n_bins, uint64_t n_img, uint64_t capacity) {
    const uint64_t nr = n_bins > n_img ? n_bins : n_img;
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    const uint64_t nb = (nr + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK;
    return al(4 * nr) /* cnt */ + al(4 * nr) /* fill */ + al(8 * (nr + 1)) /* start */
         + al(8 * (nr + 1)) /* rowptr_u */ + al(4 * nr) /* row_nnz */ + al(8 * nb) /* bsum */
         + al(4 * (capacity ? capacity : 1)) /* tmp_col */ + al(8 * (capacity ? capacity : 1)) /* tmp_w */
         + al(8 * (n_img + 1)) /* a_img, total */;
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
    const uint64_t nr = n_bins > n_img ? n_bins : n_img;
    auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    char* w = (char*)workspace;
    uint32_t* cnt = (uint32_t*)w;          w += al(4 * nr);
    uint32_t* fill = (uint32_t*)w;         w += al(4 * nr);
    uint64_t* start = (uint64_t*)w;        w += al(8 * (nr + 1));
    uint64_t* rowptr_u = (uint64_t*)w;     w += al(8 * (nr + 1));
    uint32_t* row_nnz = (uint32_t*)w;      w += al(4 * nr);
    const uint64_t nb = (nr + 1 + SCAN_BLOCK - 1) / SCAN_BLOCK;
    uint64_t* bsum = (uint64_t*)w;         w += al(8 * nb);
    uint32_t* tmp_col = (uint32_t*)w;      w += al(4 * (capacity ? capacity : 1));
    int64_t* tmp_w = (int64_t*)w;          w += al(8 * (capacity ? capacity : 1));
    unsigned long long* a_img = (unsigned long long*)w;   // n_img entries, then the total
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
    const int ge = grid_for(capacity ? capacity : 1, T256, 8192);
    for (int transpose = 0; transpose < 2; ++transpose) {
        const uint64_t n_rows = transpose ? n_img : n_bins;
        k_fill_u32<<<grid_for(n_rows, T256, 4096), T256, 0, s>>>(cnt, n_rows, 0);
        k_fill_u32<<<grid_for(n_rows, T256, 4096), T256, 0, s>>>(fill, n_rows, 0);
        k_count_rows<<<ge, T256, 0, s>>>(a, transpose, cnt);
        hipError_t e = exclusive_scan(cnt, n_rows, start, bsum, s);
        if (e != hipSuccess) return e;
        k_scatter<<<ge, T256, 0, s>>>(a, transpose, start, fill, tmp_col, tmp_w);
        k_sort_rows<<<grid_for(n_rows, T256, 8192), T256, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz, 0);
        const int gw = (int)std::min<uint64_t>(n_rows ? (n_rows + 63) / 64 : 1, 16384);
        k_sort_rows_wave<ROW_SHORT, 256><<<gw, 64, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz);
        k_sort_rows_wave<256, 1024><<<gw, 64, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz);
        // rows of 1025..4096 entries: one 256-thread block each (below)
        const int gb = (int)std::min<uint64_t>(n_rows ? (n_rows + T256 - 1) / T256 : 1, 4096);
        k_sort_rows_block<1024, ROW_LDS, false><<<gb, T256, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz);
        k_sort_rows_block<ROW_LDS, ROW_BIG, true><<<gb, T256, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz);
        k_sort_rows<<<grid_for(n_rows, T256, 8192), T256, 0, s>>>(n_rows, start, tmp_col, tmp_w, row_nnz, 1);
        e = exclusive_scan(row_nnz, n_rows, rowptr_u, bsum, s);
        if (e != hipSuccess) return e;
        k_emit_rows<<<grid_for(n_rows + 1, T256, 8192), T256, 0, s>>>(
            a, transpose, n_rows, start, tmp_col, tmp_w, rowptr_u, transpose ? Tt_rp : T_rp,
            transpose ? Tt_col : T_col, transpose ? Tt_val : T_val, a_img, total,
            transpose ? nullptr : proj);
        k_emit_rows_wave<<<gw, 64, 0, s>>>(a, transpose, n_rows, start, tmp_col, tmp_w, rowptr_u,
                                           transpose ? Tt_col : T_col, transpose ? Tt_val : T_val,
                                           a_img, total, transpose ? nullptr : proj);
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
