// Internal definitions shared by the HIP translation units of libmcspect.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcspect.h"

namespace mcs {

// ---------------------------------------------------------------------------
// Region profile of the transport loop (measurement build only: compiled with
// -DMC_REGION_PROFILE into libmcspect_prof.so).  Each marker charges the
// shader-clock time since the wave's previous marker to the previous region
// and counts one wave-level entry of the new one, in LDS per wave; the
// transport kernel adds the totals to a device array at its end
// (mc_region_profile).  The markers cost about as much as a short region, so
// the entry counts are exact while the times carry that overhead.
// ---------------------------------------------------------------------------
enum Region : int {
    RG_LOOP = 0, RG_REFILL, RG_EMIT, RG_BEGIN, RG_EXIT_TEST, RG_PHILOX, RG_STEP, RG_ESCAPE, RG_GATHER,
    RG_KAHN, RG_KAHN_ACCEPT, RG_ACCEPT_TEST, RG_REAL, RG_ENERGY_TERMS, RG_FATE_ENERGY, RG_WORK_COUNT,
    RG_FATES, RG_TALLY, RG_FORCED, RG_COUNT
};
#ifdef MC_REGION_PROFILE
constexpr int RG_SLOTS = RG_COUNT + 1;      // + the time before the first marker
static __device__ unsigned long long g_region_count[RG_SLOTS];
static __device__ unsigned long long g_region_cycles[RG_SLOTS];
// k >= 0: enter region k; -1: start (zero the wave's LDS totals); -2: add them
// to the device totals.  Kernels other than the transport loop that share the
// marked functions only touch their own LDS copy, which is never read back.
__device__ inline void region_mark(int k) {
    __shared__ unsigned long long rg_cyc[4][RG_SLOTS], rg_cnt[4][RG_SLOTS], rg_last[4];
    __shared__ int rg_cur[4];
    const unsigned long long m = __ballot(1);
    const int w = (int)(threadIdx.x >> 6);
    if (w >= 4 || (threadIdx.x & 63) != (unsigned)(__ffsll((long long)m) - 1)) return;
    const unsigned long long t = __builtin_amdgcn_s_memtime();
    if (k == -1) {
        for (int i = 0; i < RG_SLOTS; ++i) rg_cyc[w][i] = rg_cnt[w][i] = 0;
        rg_cur[w] = RG_COUNT;
    } else {
        const int c = (unsigned)rg_cur[w] < (unsigned)RG_SLOTS ? rg_cur[w] : RG_COUNT;
        rg_cyc[w][c] += t - rg_last[w];
        if (k == -2) {
            for (int i = 0; i < RG_SLOTS; ++i) {
                atomicAdd(&g_region_cycles[i], rg_cyc[w][i]);
                atomicAdd(&g_region_count[i], rg_cnt[w][i]);
            }
        } else {
            rg_cnt[w][k] += 1;
            rg_cur[w] = k;
        }
    }
    rg_last[w] = t;
}
#define MC_REGION(k) ::mcs::region_mark(k)
#else
#define MC_REGION(k) ((void)0)
#endif

// Everything a kernel needs about one problem.  Host-filled fields come from
// mc_problem; the staging kernels fill the rest on the device.
struct ProbDesc {
    // grid
    int32_t nx, ny, nz, source_mode;
    float hx, hy, hz, vox;          // half widths, voxel edge
    float lx, ly, lz, inv_vox;      // full widths, 1/voxel
    // camera
    int32_t nu, nv, n_views, image_factor;
    float pix, inv_pix, radius, cos_alpha;
    float wu, wv, e_lo, e_hi;
    float e_cut, f_pe;
    uint32_t max_steps;
    int32_t brick_log2;             // threshold layout: 0 linear, b > 0: 2^b-voxel cubic bricks
    int32_t nbx, nby, nbz, pad0;    // bricks per axis
    uint32_t seed, problem_id;
    int32_t img_nx, img_ny;
    double kn140;                   // Klein-Nishina bracket at 140 keV
    uint64_t nvox;
    uint64_t q_per_view, r_extra;   // N / V and N mod V
    uint64_t work_begin;            // first work index of this call (within the problem)
    uint64_t work_count;            // work indices of this call
    uint64_t tally_offset;          // element offset of this problem's tally block
    // inputs and staged tables (device pointers)
    const float* mu;
    const uint32_t* act;
    const double* angles;
    uint32_t* q32;                  // accept thresholds (linear or bricked layout)
    uint8_t* q8;                    // palette codes, same layout (when pal_state == 0)
    uint32_t* palette;              // PALETTE_N thresholds, open-addressing hash table
    uint4* runs;                    // emission runs (EmitRun layout), n_runs entries
    uint64_t* block_sums;           // scan scratch: activity per block
    uint32_t* block_cnt;            // scan scratch: runs starting in each block
    uint2* guide;                   // emission buckets (EmitBucket layout), n_buckets entries
    float2* views;                  // (cos, sin) per view
    float* kn_table;                // sigma_KN(e0 - i/4 keV) / sigma_KN(140), i < KN_TABLE_N
    // filled on the device by staging
    uint32_t mu_hat_bits;           // max mu, as float bits (mu >= 0)
    uint32_t flags;                 // MC_STATUS_* bits found during staging
    uint64_t total;                 // sum of activity
    uint32_t shift;                 // bucket = t >> shift
    uint32_t n_buckets;
    uint32_t n_runs;                // emission runs
    uint32_t pal_state;             // 0: palette in use; 1: 32-bit thresholds (host request
                                    // or more than PALETTE_N distinct values, set by staging)
    float omc_alpha;                // 1 - cos(alpha), from double precision (forced detection)
    uint32_t pad2;
    int32_t bb_lo[3], bb_hi[3];     // attenuation box: voxel index range of mu > 0 (staging)
    // convolution-based forced detection (layers null otherwise)
    int64_t* layers;                // [V][cfd_L][2][nv][nu] deposits, Q31.32
    double* cfd_kern;               // [cfd_L][2 cfd_hmax + 1]^2 collimator responses
    uint32_t* cfd_h;                // [cfd_L] response half-width per layer
    int32_t cfd_L, cfd_hmax;        // depth layers (one pixel thick); largest half-width
    double alpha, cfd_pix, cfd_tan; // collimator half-angle (rad), pixel (cm), tan(alpha)
    const uint32_t* act_prev;       // nullable: the source is act - act_prev (signed)
    float e0;                       // emission line energy (keV)
    uint32_t pad4;
};

// Emission weight of voxel i: the activity, or for a difference source the
// magnitude of act - act_prev.
__device__ inline uint32_t source_weight(const uint32_t* __restrict__ act,
                                         const uint32_t* __restrict__ prev, uint64_t i) {
    const uint32_t a = act[i];
    if (!prev) return a;
    const uint32_t b = prev[i];
    return a >= b ? a - b : b - a;
}

// Fixed-point weight of one contribution from a history emitted in voxel v:
// negative where a difference source is negative.
__device__ inline long long signed_weight(const ProbDesc* __restrict__ d, uint32_t v, long long w) {
    const uint32_t* prev = d->act_prev;
    return (prev && d->act[v] < prev[v]) ? -w : w;
}

// Convolution-based forced detection geometry (host and device agree):
// L = ceil(2 D / pixel) layers of one pixel's depth; layer l's response is
// evaluated at depth (l + 1/2) pixel with half-width h_l = ceil(d tan a /
// pixel + 1/2) pixels and CFD_SUB x CFD_SUB samples per pixel.
constexpr int CFD_SUB = 8;
constexpr int CFD_MAX_H = 24;     // largest response half-width (pixels) accepted
constexpr int CFD_TILE = 16;      // output tile edge of the convolution
__host__ __device__ inline int cfd_half_width(double depth, double tan_a, double pix) {
    return (int)ceil(depth * tan_a / pix + 0.5);
}

// Emission tables.  A run is a maximal stretch of consecutive voxels of one
// grid row (x fastest) with the same nonzero source weight a; EmitRun, as a
// uint4 (x, y, z, w): (y:x) the cumulative weight of all voxels before the
// run (c), z the run's first voxel as packed coordinates ix | iy << 10 |
// iz << 20, w its weight a.  The voxel of t in [c, c + a len) is the run's
// j-th, j = floor((t - c) / a), exactly the voxel a plain inverse-CDF search
// over all voxels finds.  EmitBucket b covers t in [b << shift, (b + 1) <<
// shift); as a uint2: x the run holding the bucket's first t, y how many
// further runs it meets (0: none, the run is known without a search).

// Threshold palette: a 256-slot open-addressing table keyed by Q (Q <= 2^24,
// so the all-ones word marks an empty slot); a voxel's code is its slot.
constexpr int PALETTE_N = 256;
constexpr uint32_t PALETTE_EMPTY = 0xFFFFFFFFu;
__host__ __device__ inline uint32_t palette_hash(uint32_t q) { return (q * 2654435761u) >> 24; }

constexpr int SCAN_ITEMS = 4096;    // activity values per scan block
constexpr int KN_TABLE_N = 2048;    // entries of the Klein-Nishina shape table (>= 4*500 + 2)
constexpr double MAX_LINE_KEV = 500.0;   // highest emission line accepted
constexpr int MAX_AXIS = 1024;      // voxel indices are packed 10 bits per axis
constexpr int SCAN_THREADS = 256;

// Index of voxel (ix, iy, iz) in the threshold array: linear for b = 0, else
// brick-major over nbx x nby x nbz bricks of 2^b voxels per side.  Every
// factor is below 2^24 (axes of at most 1024 voxels), so the products take
// the full-rate 24-bit multiplier.
__device__ inline uint32_t brick_index(uint32_t ix, uint32_t iy, uint32_t iz, uint32_t nx,
                                       uint32_t ny, int b, uint32_t m, uint32_t nbx, uint32_t nby) {
    if (b == 0) return ix + __umul24(nx, iy + __umul24(ny, iz));
    const uint32_t brick = __umul24(__umul24(iz >> b, nby) + (iy >> b), nbx) + (ix >> b);
    const uint32_t local = (((iz & m) << b | (iy & m)) << b) | (ix & m);
    return (brick << (3 * b)) | local;
}

// Global counters of one call (in the workspace).
struct CallState {
    unsigned long long next_chunk;
    unsigned long long pad[7];
};

// Host launchers (cgsm.hip): block-summed source; coarse projection expanded
// to the normal pixels.
hipError_t launch_block_activity(const uint32_t* act, int nx, int ny, int nz, int f, uint32_t* out,
                                 int64_t* status, hipStream_t s);
hipError_t launch_expand(const int64_t* coarse, uint64_t n_planes, int nu_c, int nv_c, int f, double scale,
                         double* out, hipStream_t s);

// Host launchers (compose.hip): total source weight (sum of |act - prev|)
// into a device uint64; a Q31.32 tally times scale into (or added to) FP64.
hipError_t launch_source_total(const uint32_t* act, const uint32_t* prev, uint64_t n,
                               unsigned long long* total, hipStream_t s);
hipError_t launch_scale_tally(const int64_t* tally, uint64_t n, double scale, double* out, int accumulate,
                              hipStream_t s);

// Host launchers (cfd.hip): zero the layers and build the responses (per call,
// before transport); convolve the layers into the tally (after transport).
// The host sizes the response table with cfd_hmax; each layer's half-width is
// capped at it, so the table is never overrun.
hipError_t launch_cfd_setup(ProbDesc* d, const ProbDesc& h, hipStream_t s);
hipError_t launch_cfd_convolve(const ProbDesc* d, const ProbDesc& h, int64_t* tally, hipStream_t s);

// Host launchers (staging.hip)
hipError_t launch_staging(ProbDesc* d_desc, const ProbDesc& h_desc, hipStream_t s);
// emission buckets reserved: the power of two >= nvox (the staging uses the
// power of two >= 2 x the number of runs, up to this)
__host__ __device__ inline uint64_t guide_capacity(uint64_t nvox) {
    uint64_t c = 2;
    while (c < nvox) c <<= 1;
    return c;
}
hipError_t launch_staging_batch(ProbDesc* d_descs, const ProbDesc* h_descs, int n, hipStream_t s);

// Host launchers (transport.hip)
struct TransportArgs {
    const ProbDesc* descs;
    int32_t n_problems;
    const uint64_t* work_prefix;    // [n_problems + 1], device
    uint64_t total_work;
    uint32_t chunk;                 // work indices per claim (per wave)
    int32_t forced_detection;       // 1: forced detection in the tally; 2: into CFD layers
    CallState* state;
    int64_t* tally;
    int64_t* tally_sq;
    int64_t* fates;
    int64_t* energy;
    int64_t* counters;
    mc_event* events;
    uint64_t event_capacity;
    unsigned long long* n_events;
    int64_t* status;
    int32_t vr_flags;               // VR_FORCED_DIRECTION | VR_FORCED_INTERACTION (weighted analog)
    float vr_omc;                   // forced direction: 1 - cos(cone half-angle)
};
constexpr int32_t VR_FORCED_DIRECTION = 1, VR_FORCED_INTERACTION = 2;
hipError_t launch_transport(const TransportArgs& a, int grid, int block, hipStream_t s);
// After every tally writer of a forward call: MC_STATUS_TALLY_OVERFLOW when a
// problem's tally may have left the Q31.32 range.
hipError_t launch_tally_check(const ProbDesc* d_desc, int n_problems, const int64_t* tally,
                              const int64_t* fates, int64_t* status, hipStream_t s);
hipError_t launch_replay(const ProbDesc* d_desc, const int32_t* views, const uint64_t* hists,
                         int64_t n, mc_record* out, int64_t* status, int block, int32_t vr_flags,
                         float vr_omc, hipStream_t s);
hipError_t launch_prepare_call(const ProbDesc* descs, int32_t n_problems, uint64_t* work_prefix,
                               CallState* state, int64_t* status, unsigned long long* n_events,
                               int64_t* tally, uint64_t tally_elems, int64_t* tally_sq,
                               int64_t* fates, int64_t* energy, int64_t* counters,
                               uint32_t chunk, hipStream_t s);

// Host launcher (adjoint.hip)
hipError_t launch_adjoint(const ProbDesc* d, const mc_event* events, const uint64_t* n_events,
                          uint64_t capacity, const double* dL, int64_t* grad, uint64_t nvox,
                          int frac_bits, int64_t* status, int n_cu, hipStream_t s);

// Host launchers (sysmat.hip)
size_t sysmat_workspace_bytes(uint64_t n_bins, uint64_t n_img, uint64_t capacity);
hipError_t launch_sysmat(const mc_event* events, const unsigned long long* n_events, uint64_t capacity,
                         uint32_t nx, uint32_t ny, uint32_t nz, uint32_t f, uint32_t n_views,
                         uint32_t nu, uint32_t nv, uint64_t n_hist, const uint32_t* activity,
                         uint32_t class_mask, int64_t* T_rp, int32_t* T_col, float* T_val,
                         int64_t* Tt_rp, int32_t* Tt_col, float* Tt_val, float* proj,
                         void* workspace, hipStream_t s);
size_t mlem_workspace(uint64_t n_bins, uint64_t n_vox);
// launch_mlem phases: the matrix's set-up (row sums, row lists, renumbered
// columns, kept in the workspace) and the call (load, iterations, image out).
enum : int { MLEM_SETUP = 1, MLEM_ITERATE = 2 };
hipError_t launch_mlem(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rp,
                       const int32_t* T_col, const float* T_val, const int64_t* Tt_rp,
                       const int32_t* Tt_col, const float* Tt_val, const float* proj, float* image,
                       int32_t n_iter, void* workspace, int phases, hipStream_t s);

constexpr int32_t OSEM_MAX_SUBSETS = 64;   // one lane of a wavefront per subset in the split
size_t osem_workspace(uint64_t n_bins, uint64_t n_vox, uint32_t n_sub, uint64_t bt_nnz);
hipError_t launch_osem(int64_t n_bins, int64_t n_vox, int32_t bins_per_view, int32_t n_sub,
                       const int64_t* C_rp, const int32_t* C_col, const float* C_val,
                       const int64_t* Bt_rp, const int32_t* Bt_col, const float* Bt_val, int64_t bt_nnz,
                       const float* proj, const float* scatter, float* image, int32_t n_iter,
                       void* workspace, hipStream_t s);

// Occupancy of the transport kernel (blocks per CU at this block size).
int transport_blocks_per_cu(int block, int forced_detection, int vr_flags);

}  // namespace mcs
