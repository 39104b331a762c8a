// Host side of the C ABI: argument checks, workspace layout, launches.
// No device memory is allocated here; no exception leaves this file.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "mc_internal.h"

using namespace mcs;

namespace mcs {
size_t staging_block_scratch_u64(uint64_t nvox);   // staging.hip
}

namespace {

thread_local int g_last_hip = 0;

constexpr uint32_t DEFAULT_MAX_STEPS = 1000;
constexpr int DEFAULT_BLOCK = 256;
constexpr int DEFAULT_HIST_PER_LANE = 16;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int MAX_BRICK_LOG2 = 3;

// Threshold storage for the largest brick size (grid padded to whole bricks).
uint64_t padded_voxels(const mc_problem& p) {
    const uint64_t b = 1u << MAX_BRICK_LOG2;
    const uint64_t px = (p.nx + b - 1) / b * b, py = (p.ny + b - 1) / b * b, pz = (p.nz + b - 1) / b * b;
    return px * py * pz;
}

double kn_bracket(double e) {
    // Klein-Nishina total cross-section per electron over 2 pi r_e^2.
    const double k = e / 510.99895;
    const double a = 1.0 + 2.0 * k;
    const double la = std::log(a);
    return (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - la / k) + la / (2.0 * k)
           - (1.0 + 3.0 * k) / (a * a);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host-visible checks of one problem.
bool check_problem(const mc_problem& p) {
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return false;
    if (p.nx > MAX_AXIS || p.ny > MAX_AXIS || p.nz > MAX_AXIS) return false;
    const uint64_t nvox = (uint64_t)p.nx * p.ny * p.nz;
    if (nvox >= (1ull << 31)) return false;
    if (p.source_mode != MC_SOURCE_VOXELS && p.source_mode != MC_SOURCE_POINT) return false;
    if (!finite_pos(p.voxel_cm)) return false;
    if (!p.mu140 || !p.activity || !p.angle_rad) return false;
    if (p.n_views < 1 || p.nu < 1 || p.nv < 1) return false;
    if ((uint64_t)p.nu * p.nv * 2 * p.n_views >= (1ull << 32)) return false;
    if (!finite_pos(p.pixel_cm) || !std::isfinite(p.radius_cm)) return false;
    const double lx = p.nx * p.voxel_cm, ly = p.ny * p.voxel_cm;
    if (p.radius_cm <= 0.5 * std::sqrt(lx * lx + ly * ly)) return false;   // plane outside the grid
    if (!(p.accept_half_angle_rad > 0.0 && p.accept_half_angle_rad < 1.5707963267948966)) return false;
    if (!std::isfinite(p.e_lo_kev) || !std::isfinite(p.e_hi_kev) || p.e_lo_kev > p.e_hi_kev) return false;
    const double e0 = p.e0_kev > 0.0 ? p.e0_kev : 140.0;
    if (!(e0 <= MAX_LINE_KEV) || (double)(float)e0 != e0) return false;
    if (!std::isfinite(p.e_cut_kev) || p.e_cut_kev < 1.0 || p.e_cut_kev > e0) return false;
    if (!(p.pe_fraction >= 0.0 && p.pe_fraction <= 1.0)) return false;
    if (p.n_histories < 1) return false;
    if (p.n_histories / (uint64_t)p.n_views >= (1ull << 32) - 1) return false;
    if (p.history_offset > p.n_histories) return false;
    const uint64_t cnt = p.history_count ? p.history_count : p.n_histories - p.history_offset;
    if (p.history_offset + cnt > p.n_histories) return false;
    if (p.image_factor < 0) return false;
    if (p.image_factor > 0 &&
        (p.nx % p.image_factor || p.ny % p.image_factor || p.nz % p.image_factor)) return false;
    return true;
}

// Convolution-based forced detection geometry: layers of one pixel's depth
// over [0, 2 D]; the largest response half-width is the deepest layer's.
int cfd_layers(const mc_problem& p) { return (int)std::ceil(2.0 * p.radius_cm / p.pixel_cm); }
int cfd_hmax(const mc_problem& p) {
    const int nl = cfd_layers(p);
    return cfd_half_width((nl - 0.5) * p.pixel_cm, std::tan(p.accept_half_angle_rad), p.pixel_cm);
}
bool cfd_ok(const mc_problem& p) { return cfd_layers(p) >= 1 && cfd_hmax(p) <= CFD_MAX_H; }

struct Layout {
    size_t desc, prefix, state;
    std::vector<size_t> q, q8, pal, runs, bsum, bcnt, guide, views, kn, lay, kern, hw;
    size_t total;
};

bool plan(const mc_problem* probs, int n, Layout& L, bool cfd = false) {
    size_t off = 0;
    L.desc = off;   off += align256(sizeof(ProbDesc) * (size_t)n);
    L.prefix = off; off += align256(sizeof(uint64_t) * 2 * ((size_t)n + 1));
    L.state = off;  off += align256(sizeof(CallState));
    L.q.resize(n); L.q8.resize(n); L.pal.resize(n); L.runs.resize(n); L.bsum.resize(n); L.bcnt.resize(n);
    L.guide.resize(n); L.views.resize(n); L.kn.resize(n);
    L.lay.assign(n, 0); L.kern.assign(n, 0); L.hw.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const mc_problem& p = probs[i];
        const uint64_t nvox = (uint64_t)p.nx * p.ny * p.nz;
        L.q[i] = off;     off += align256(4 * padded_voxels(p));
        L.q8[i] = off;    off += align256(padded_voxels(p));
        L.pal[i] = off;   off += align256(4 * (size_t)PALETTE_N);
        L.runs[i] = off;  off += align256(16 * nvox);
        L.bsum[i] = off;  off += align256(8 * staging_block_scratch_u64(nvox));
        L.bcnt[i] = off;  off += align256(4 * ((nvox + SCAN_ITEMS - 1) / SCAN_ITEMS));
        L.guide[i] = off; off += align256(8 * guide_capacity(nvox));
        L.views[i] = off; off += align256(8 * (size_t)p.n_views);
        L.kn[i] = off;    off += align256(4 * (size_t)KN_TABLE_N);
        if (cfd) {
            const size_t nl = (size_t)cfd_layers(p), m = 2 * (size_t)cfd_hmax(p) + 1;
            L.lay[i] = off;  off += align256(8 * nl * 2 * p.n_views * (size_t)p.nv * p.nu);
            L.kern[i] = off; off += align256(8 * nl * m * m);
            L.hw[i] = off;   off += align256(4 * nl);
        }
    }
    L.total = off;
    return true;
}

ProbDesc host_desc(const mc_problem& p, char* ws, const Layout& L, int i, uint64_t tally_offset,
                   int brick_log2, int threshold_bytes, bool cfd = false) {
    ProbDesc d;
    std::memset(&d, 0, sizeof(d));
    d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.source_mode = p.source_mode;
    const double vox = p.voxel_cm;
    d.vox = (float)vox;
    d.inv_vox = (float)(1.0 / vox);
    d.lx = (float)(p.nx * vox); d.ly = (float)(p.ny * vox); d.lz = (float)(p.nz * vox);
    d.hx = (float)(0.5 * p.nx * vox); d.hy = (float)(0.5 * p.ny * vox); d.hz = (float)(0.5 * p.nz * vox);
    d.nu = p.nu; d.nv = p.nv; d.n_views = p.n_views;
    d.image_factor = p.image_factor;
    d.pix = (float)p.pixel_cm;
    d.inv_pix = (float)(1.0 / p.pixel_cm);
    d.radius = (float)p.radius_cm;
    d.cos_alpha = (float)std::cos(p.accept_half_angle_rad);
    d.omc_alpha = (float)(2.0 * std::sin(0.5 * p.accept_half_angle_rad) * std::sin(0.5 * p.accept_half_angle_rad));
    d.wu = (float)(p.nu * p.pixel_cm);
    d.wv = (float)(p.nv * p.pixel_cm);
    d.e_lo = (float)p.e_lo_kev; d.e_hi = (float)p.e_hi_kev; d.e_cut = (float)p.e_cut_kev;
    d.f_pe = (float)p.pe_fraction;
    d.max_steps = p.max_steps ? p.max_steps : DEFAULT_MAX_STEPS;
    d.brick_log2 = brick_log2;
    const int b = 1 << brick_log2;
    d.nbx = (p.nx + b - 1) / b; d.nby = (p.ny + b - 1) / b; d.nbz = (p.nz + b - 1) / b;
    d.seed = p.seed; d.problem_id = p.problem_id;
    if (p.image_factor > 0) { d.img_nx = p.nx / p.image_factor; d.img_ny = p.ny / p.image_factor; }
    d.kn140 = kn_bracket(140.0);
    d.nvox = (uint64_t)p.nx * p.ny * p.nz;
    d.q_per_view = p.n_histories / (uint64_t)p.n_views;
    d.r_extra = p.n_histories % (uint64_t)p.n_views;
    d.work_begin = p.history_offset;
    d.work_count = p.history_count ? p.history_count : p.n_histories - p.history_offset;
    d.tally_offset = tally_offset;
    d.mu = p.mu140; d.act = p.activity; d.angles = p.angle_rad;
    d.act_prev = p.activity_prev;
    d.e0 = (float)(p.e0_kev > 0.0 ? p.e0_kev : 140.0);
    d.q32 = (uint32_t*)(ws + L.q[i]);
    d.q8 = (uint8_t*)(ws + L.q8[i]);
    d.palette = (uint32_t*)(ws + L.pal[i]);
    d.pal_state = threshold_bytes == 4 ? 1u : 0u;
    for (int a = 0; a < 3; ++a) { d.bb_lo[a] = INT32_MAX; d.bb_hi[a] = -1; }
    d.runs = (uint4*)(ws + L.runs[i]);
    d.block_sums = (uint64_t*)(ws + L.bsum[i]);
    d.block_cnt = (uint32_t*)(ws + L.bcnt[i]);
    d.guide = (uint2*)(ws + L.guide[i]);
    d.views = (float2*)(ws + L.views[i]);
    d.kn_table = (float*)(ws + L.kn[i]);
    if (cfd) {
        d.layers = (int64_t*)(ws + L.lay[i]);
        d.cfd_kern = (double*)(ws + L.kern[i]);
        d.cfd_h = (uint32_t*)(ws + L.hw[i]);
        d.cfd_L = cfd_layers(p);
        d.cfd_hmax = cfd_hmax(p);
        d.alpha = p.accept_half_angle_rad;
        d.cfd_pix = p.pixel_cm;
        d.cfd_tan = std::tan(p.accept_half_angle_rad);
    }
    return d;
}

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return MC_EDEVICE;
}

void resolve(const mc_options* opt, int& block, int& hpl, int& bpc, int& brick, int& qbytes) {
    block = DEFAULT_BLOCK;
    hpl = DEFAULT_HIST_PER_LANE;
    bpc = 0;
    brick = 0;
    qbytes = 0;
    if (opt) {
        if (opt->block_size > 0) block = opt->block_size;
        if (opt->hist_per_lane > 0) hpl = opt->hist_per_lane;
        if (opt->blocks_per_cu > 0) bpc = opt->blocks_per_cu;
        if (opt->brick_log2 > 0) brick = opt->brick_log2;
        qbytes = opt->threshold_bytes;
    }
}

// Variance-reduction options (weighted analog): flags in [0, 3], a forced-
// direction cone in (0, pi], and not together with forced detection.
bool vr_ok(const mc_options* opt) {
    if (!opt) return true;
    const int v = opt->variance_reduction;
    if (v < 0 || v > 3) return false;
    if ((v & VR_FORCED_DIRECTION) &&
        !(opt->forced_direction_half_angle_rad > 0.0 && opt->forced_direction_half_angle_rad <= 3.14159265358979323846))
        return false;
    if (v && opt->forced_detection) return false;
    return true;
}
float vr_omc(const mc_options* opt) {
    if (!opt || !(opt->variance_reduction & VR_FORCED_DIRECTION)) return 0.0f;
    const double h = 0.5 * opt->forced_direction_half_angle_rad;
    return (float)(2.0 * std::sin(h) * std::sin(h));
}

bool options_ok(int block, int hpl, int brick, int qbytes) {
    if (block < 64 || block > 256 || block % 64 != 0) return false;
    if (hpl < 1 || hpl > (1 << 20)) return false;
    if (brick < 0 || brick > MAX_BRICK_LOG2 || brick == 1) return false;
    if (qbytes != 0 && qbytes != 1 && qbytes != 4) return false;
    return true;
}

}  // namespace

extern "C" {

size_t mc_workspace_bytes(const mc_problem* problems, int32_t n_problems, const mc_options* opt) {
    if (!problems || n_problems < 1) return 0;
    const bool cfd = opt && opt->forced_detection == 2;
    for (int i = 0; i < n_problems; ++i)
        if (!check_problem(problems[i]) || (cfd && !cfd_ok(problems[i]))) return 0;
    Layout L;
    plan(problems, n_problems, L, cfd);
    return L.total;
}

}  // extern "C"

namespace {

int simulate_impl(const mc_problem* problems, int32_t n_problems, const mc_options* opt,
                  int64_t* tally, int64_t* tally_sq, int64_t* fates, int64_t* energy,
                  int64_t* counters, mc_event* events, uint64_t event_capacity,
                  uint64_t* n_events, int64_t* status, void* workspace,
                  size_t workspace_bytes, void* stream) {
    if (!problems || n_problems < 1 || !tally || !fates || !status || !workspace) return MC_EINVAL;
    if (opt && (opt->forced_detection < 0 || opt->forced_detection > 2)) return MC_EINVAL;
    if (!vr_ok(opt)) return MC_EINVAL;
    const bool cfd = opt && opt->forced_detection == 2;
    if (events && !n_events) return MC_EINVAL;
    if (cfd && events) return MC_EINVAL;   // convolved tallies have no per-copy bins
    for (int i = 0; i < n_problems; ++i)
        if (!check_problem(problems[i]) || (cfd && !cfd_ok(problems[i]))) return MC_EINVAL;
    int block, hpl, bpc, brick, qbytes;
    resolve(opt, block, hpl, bpc, brick, qbytes);
    if (!options_ok(block, hpl, brick, qbytes)) return MC_EINVAL;
    Layout L;
    plan(problems, n_problems, L, cfd);
    if (workspace_bytes < L.total) return MC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    ProbDesc* d_desc = (ProbDesc*)(ws + L.desc);
    uint64_t tally_elems = 0;
    std::vector<ProbDesc> hd;
    hd.reserve(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        const mc_problem& p = problems[i];
        hd.push_back(host_desc(p, ws, L, i, tally_elems, brick, qbytes, cfd));
        tally_elems += (uint64_t)p.n_views * 2 * p.nv * p.nu;
    }
    {
        hipError_t e = launch_staging_batch(d_desc, hd.data(), n_problems, st);
        if (e != hipSuccess) return hip_fail(e);
        for (int i = 0; cfd && i < n_problems; ++i)
            if ((e = launch_cfd_setup(d_desc + i, hd[i], st)) != hipSuccess) return hip_fail(e);
    }
    hipError_t e = hipSuccess;
    int dev = 0, n_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e);
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e);
    const int fd = opt ? opt->forced_detection : 0;
    const int vr = opt ? opt->variance_reduction : 0;
    if (bpc <= 0) bpc = transport_blocks_per_cu(block, fd, vr);
    if (!(opt && opt->hist_per_lane > 0)) {
        // automatic claim size (results do not depend on it): half the
        // default when there are fewer than 2048 histories per resident
        // wavefront, which spreads small calls better (measured: 1e6
        // histories on one view 0.33 against 0.35 ms; 1e7 and more: 16 best)
        uint64_t work = 0;
        for (int i = 0; i < n_problems; ++i) work += hd[i].work_count;
        const uint64_t waves = (uint64_t)n_cu * (uint64_t)bpc * (uint64_t)(block / 64);
        hpl = work < 2048ull * (waves ? waves : 1) ? DEFAULT_HIST_PER_LANE / 2 : DEFAULT_HIST_PER_LANE;
    }
    const uint32_t chunk = (uint32_t)(64 * hpl);
    e = launch_prepare_call(d_desc, n_problems, (uint64_t*)(ws + L.prefix),
                            (CallState*)(ws + L.state), status,
                            (unsigned long long*)n_events, tally, tally_elems, tally_sq,
                            fates, energy, counters, chunk, st);
    if (e != hipSuccess) return hip_fail(e);
    TransportArgs a;
    a.descs = d_desc;
    a.n_problems = n_problems;
    a.work_prefix = (const uint64_t*)(ws + L.prefix);
    a.total_work = 0;
    a.chunk = chunk;
    a.state = (CallState*)(ws + L.state);
    a.tally = tally;
    a.tally_sq = tally_sq;
    a.fates = fates;
    a.energy = energy;
    a.counters = counters;
    a.events = events;
    a.event_capacity = events ? event_capacity : 0;
    a.n_events = (unsigned long long*)n_events;
    a.status = status;
    a.forced_detection = fd;
    a.vr_flags = vr;
    a.vr_omc = vr_omc(opt);
    hipEvent_t ev0 = opt ? (hipEvent_t)opt->kernel_events[0] : nullptr;
    hipEvent_t ev1 = opt ? (hipEvent_t)opt->kernel_events[1] : nullptr;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return hip_fail(e);
    e = launch_transport(a, n_cu * bpc, block, st);
    if (e != hipSuccess) return hip_fail(e);
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return hip_fail(e);
    for (int i = 0; cfd && i < (int)hd.size(); ++i)
        if ((e = launch_cfd_convolve(d_desc + i, hd[i], tally, st)) != hipSuccess) return hip_fail(e);
    if ((e = launch_tally_check(d_desc, n_problems, tally, fates, status, st)) != hipSuccess) return hip_fail(e);
    return MC_OK;
}

// Scratch of the no-allocation entry point: one array per device, placed by
// the code-object loader, shared by every call on that device.  Its host-side
// name is not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[MC_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up once per
// device, with that device current).  Returns MC_OK or an error code.
int scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= MAX_DEVICES) return MC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p) return MC_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MC_OK;
}

}  // namespace

extern "C" {

int mc_simulate_projections(const mc_problem* problems, int32_t n_problems, const mc_options* opt,
                            int64_t* tally, int64_t* tally_sq, int64_t* fates, int64_t* energy,
                            int64_t* counters, mc_event* events, uint64_t event_capacity,
                            uint64_t* n_events, int64_t* status, void* workspace,
                            size_t workspace_bytes, void* stream) {
    return simulate_impl(problems, n_problems, opt, tally, tally_sq, fates, energy, counters, events,
                         event_capacity, n_events, status, workspace, workspace_bytes, stream);
}

int mc_simulate_projections_static(const mc_problem* problems, int32_t n_problems,
                                   const mc_options* opt, int64_t* tally, int64_t* tally_sq,
                                   int64_t* fates, int64_t* energy, int64_t* counters,
                                   mc_event* events, uint64_t event_capacity, uint64_t* n_events,
                                   int64_t* status, void* stream) {
    if (!problems || n_problems < 1) return MC_EINVAL;
    const size_t need = mc_workspace_bytes(problems, n_problems, opt);
    if (need == 0) return MC_EINVAL;
    if (need > (size_t)MC_STATIC_SCRATCH_BYTES) return MC_ENOMEM;
    void* ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc != MC_OK) return rc;
    return simulate_impl(problems, n_problems, opt, tally, tally_sq, fates, energy, counters, events,
                         event_capacity, n_events, status, ws, (size_t)MC_STATIC_SCRATCH_BYTES, stream);
}

int mc_replay_histories(const mc_problem* problem, const mc_options* opt, const int32_t* views,
                        const uint64_t* hists, int64_t n, mc_record* records, int64_t* status,
                        void* workspace, size_t workspace_bytes, void* stream) {
    if (!problem || !status || !workspace || n < 0) return MC_EINVAL;
    if (n > 0 && (!views || !hists || !records)) return MC_EINVAL;
    if (!check_problem(*problem)) return MC_EINVAL;
    int block, hpl, bpc, brick, qbytes;
    resolve(opt, block, hpl, bpc, brick, qbytes);
    if (!options_ok(block, hpl, brick, qbytes) || !vr_ok(opt)) return MC_EINVAL;
    Layout L;
    plan(problem, 1, L);
    if (workspace_bytes < L.total) return MC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    ProbDesc* d_desc = (ProbDesc*)(ws + L.desc);
    const ProbDesc h = host_desc(*problem, ws, L, 0, 0, brick, qbytes);
    hipError_t e = launch_staging(d_desc, h, st);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_replay(d_desc, views, hists, n, records, status, block, opt ? opt->variance_reduction : 0,
                      vr_omc(opt), st);
    if (e != hipSuccess) return hip_fail(e);
    return MC_OK;
}

int mc_adjoint_mu(const mc_problem* problem, const mc_options* opt, const double* dL_dtally,
                  const mc_event* events, const uint64_t* n_events, uint64_t event_capacity,
                  int64_t* dL_dmu, int32_t frac_bits, int64_t* status, void* workspace,
                  size_t workspace_bytes, void* stream) {
    if (!problem || !dL_dtally || !dL_dmu || !status || !workspace) return MC_EINVAL;
    if (events && !n_events) return MC_EINVAL;
    if (frac_bits < 0 || frac_bits > 62) return MC_EINVAL;
    if (opt && (opt->forced_detection || opt->variance_reduction))
        return MC_EINVAL;                                  // adjoint of analog tallies only
    if (problem->activity_prev) return MC_EINVAL;         // and of plain sources
    if (!check_problem(*problem)) return MC_EINVAL;
    int block, hpl, bpc, brick, qbytes;
    resolve(opt, block, hpl, bpc, brick, qbytes);
    if (!options_ok(block, hpl, brick, qbytes)) return MC_EINVAL;
    Layout L;
    plan(problem, 1, L);
    if (workspace_bytes < L.total) return MC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    ProbDesc* d_desc = (ProbDesc*)(ws + L.desc);
    const ProbDesc h = host_desc(*problem, ws, L, 0, 0, brick, qbytes);
    hipError_t e = hipSuccess;
    if (!(opt && opt->reuse_staging)) {
        e = launch_staging(d_desc, h, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    int dev = 0, n_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e);
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e);
    e = launch_adjoint(d_desc, events, n_events, events ? event_capacity : 0, dL_dtally, dL_dmu,
                       h.nvox, frac_bits, status, n_cu, st);
    if (e != hipSuccess) return hip_fail(e);
    return MC_OK;
}

size_t mc_system_matrix_workspace_bytes(const mc_problem* problem, uint64_t event_capacity) {
    if (!problem || !check_problem(*problem) || problem->image_factor < 1) return 0;
    const mc_problem& p = *problem;
    const uint64_t n_bins = (uint64_t)p.n_views * p.nu * p.nv;
    const uint64_t f = (uint64_t)p.image_factor;
    const uint64_t n_img = (p.nx / f) * (p.ny / f) * (p.nz / f);
    return sysmat_workspace_bytes(n_bins, n_img, event_capacity);
}

int mc_system_matrix(const mc_problem* problem, const mc_event* events, const uint64_t* n_events,
                     uint64_t event_capacity, int32_t class_mask, int64_t* T_rowptr, int32_t* T_col,
                     float* T_val,
                     int64_t* Tt_rowptr, int32_t* Tt_col, float* Tt_val, float* proj,
                     void* workspace, size_t workspace_bytes, void* stream) {
    if (!problem || !events || !n_events || !T_rowptr || !T_col || !T_val || !Tt_rowptr ||
        !Tt_col || !Tt_val || !workspace)
        return MC_EINVAL;
    if (!check_problem(*problem) || problem->image_factor < 1) return MC_EINVAL;
    if (problem->activity_prev) return MC_EINVAL;   // normalised by a plain source's activity
    // N_view is the view's share of all n_histories: the forward call must
    // have covered the whole work range
    if (problem->history_offset != 0 ||
        (problem->history_count != 0 && problem->history_count != problem->n_histories))
        return MC_EINVAL;
    if (event_capacity < 1 || event_capacity >= (1ull << 31)) return MC_EINVAL;
    if (class_mask < 1 || class_mask > 3) return MC_EINVAL;
    const mc_problem& p = *problem;
    if ((uint64_t)p.n_views * p.nu * p.nv >= (1ull << 31)) return MC_EINVAL;
    if (workspace_bytes < mc_system_matrix_workspace_bytes(problem, event_capacity)) return MC_ENOMEM;
    hipError_t e = launch_sysmat(events, (const unsigned long long*)n_events, event_capacity,
                                 (uint32_t)p.nx, (uint32_t)p.ny, (uint32_t)p.nz,
                                 (uint32_t)p.image_factor, (uint32_t)p.n_views, (uint32_t)p.nu,
                                 (uint32_t)p.nv, p.n_histories, p.activity, (uint32_t)class_mask,
                                 T_rowptr, T_col, T_val,
                                 Tt_rowptr, Tt_col, Tt_val, proj, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return MC_OK;
}

size_t mlem_workspace_bytes(int64_t n_bins, int64_t n_vox) {
    if (n_bins < 1 || n_vox < 1) return 0;
    return mlem_workspace((uint64_t)n_bins, (uint64_t)n_vox);
}

static int mlem_call(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rowptr,
                     const int32_t* T_col, const float* T_val, const int64_t* Tt_rowptr,
                     const int32_t* Tt_col, const float* Tt_val, const float* proj, float* image,
                     int32_t n_iter, void* workspace, size_t workspace_bytes, void* stream, int phases) {
    const bool iterate = (phases & MLEM_ITERATE) != 0;
    if (n_bins < 1 || n_vox < 1 || nnz < 0 || n_iter < 0) return MC_EINVAL;
    if (n_bins >= (1ll << 31) || n_vox >= (1ll << 31)) return MC_EINVAL;
    if (!T_rowptr || !T_col || !T_val || !Tt_rowptr || !Tt_col || !Tt_val || !workspace) return MC_EINVAL;
    if (iterate && (!proj || !image)) return MC_EINVAL;
    if (workspace_bytes < mlem_workspace((uint64_t)n_bins, (uint64_t)n_vox)) return MC_ENOMEM;
    hipError_t e = launch_mlem(n_bins, n_vox, nnz, T_rowptr, T_col, T_val, Tt_rowptr, Tt_col, Tt_val,
                               proj, image, n_iter, workspace, phases, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return MC_OK;
}

int mlem_iterate(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rowptr,
                 const int32_t* T_col, const float* T_val, const int64_t* Tt_rowptr,
                 const int32_t* Tt_col, const float* Tt_val, const float* proj, float* image,
                 int32_t n_iter, void* workspace, size_t workspace_bytes, void* stream) {
    return mlem_call(n_bins, n_vox, nnz, T_rowptr, T_col, T_val, Tt_rowptr, Tt_col, Tt_val, proj, image,
                     n_iter, workspace, workspace_bytes, stream, MLEM_SETUP | MLEM_ITERATE);
}

int mlem_prepare(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rowptr,
                 const int32_t* T_col, const float* T_val, const int64_t* Tt_rowptr,
                 const int32_t* Tt_col, const float* Tt_val, void* workspace, size_t workspace_bytes,
                 void* stream) {
    return mlem_call(n_bins, n_vox, nnz, T_rowptr, T_col, T_val, Tt_rowptr, Tt_col, Tt_val, nullptr, nullptr,
                     0, workspace, workspace_bytes, stream, MLEM_SETUP);
}

int mlem_iterate_prepared(int64_t n_bins, int64_t n_vox, int64_t nnz, const int64_t* T_rowptr,
                          const int32_t* T_col, const float* T_val, const int64_t* Tt_rowptr,
                          const int32_t* Tt_col, const float* Tt_val, const float* proj, float* image,
                          int32_t n_iter, void* workspace, size_t workspace_bytes, void* stream) {
    return mlem_call(n_bins, n_vox, nnz, T_rowptr, T_col, T_val, Tt_rowptr, Tt_col, Tt_val, proj, image,
                     n_iter, workspace, workspace_bytes, stream, MLEM_ITERATE);
}

size_t osem_workspace_bytes(int64_t n_bins, int64_t n_vox, int32_t n_subsets, int64_t bt_nnz) {
    if (n_bins < 1 || n_vox < 1 || n_subsets < 1 || n_subsets > OSEM_MAX_SUBSETS || bt_nnz < 0) return 0;
    return osem_workspace((uint64_t)n_bins, (uint64_t)n_vox, (uint32_t)n_subsets, (uint64_t)bt_nnz);
}

int osem_iterate(int64_t n_bins, int64_t n_vox, int32_t bins_per_view, int32_t n_subsets,
                 const int64_t* C_rowptr, const int32_t* C_col, const float* C_val,
                 const int64_t* Bt_rowptr, const int32_t* Bt_col, const float* Bt_val, int64_t bt_nnz,
                 const float* proj, const float* scatter, float* image, int32_t n_iter,
                 void* workspace, size_t workspace_bytes, void* stream) {
    if (n_bins < 1 || n_vox < 1 || n_iter < 0 || bins_per_view < 1 || n_subsets < 1 || bt_nnz < 0)
        return MC_EINVAL;
    if (n_bins >= (1ll << 31) || n_vox >= (1ll << 31) || n_bins % bins_per_view != 0) return MC_EINVAL;
    if (n_subsets > n_bins / bins_per_view || n_subsets > OSEM_MAX_SUBSETS) return MC_EINVAL;
    if (!C_rowptr || !C_col || !C_val || !Bt_rowptr || !Bt_col || !Bt_val || !proj || !image ||
        !workspace)
        return MC_EINVAL;
    if (workspace_bytes < osem_workspace((uint64_t)n_bins, (uint64_t)n_vox, (uint32_t)n_subsets, (uint64_t)bt_nnz))
        return MC_ENOMEM;
    hipError_t e = launch_osem(n_bins, n_vox, bins_per_view, n_subsets, C_rowptr, C_col, C_val,
                               Bt_rowptr, Bt_col, Bt_val, bt_nnz, proj, scatter, image, n_iter, workspace,
                               (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return MC_OK;
}

int mc_block_activity(const uint32_t* act, int32_t nx, int32_t ny, int32_t nz, int32_t factor,
                      uint32_t* out, int64_t* status, void* stream) {
    if (!act || !out || !status || act == out) return MC_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || factor < 1) return MC_EINVAL;
    if (nx % factor || ny % factor || nz % factor) return MC_EINVAL;
    if ((uint64_t)nx * ny * nz >= (1ull << 40)) return MC_EINVAL;
    const hipError_t e = launch_block_activity(act, nx, ny, nz, factor, out, status, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_expand_projection(const int64_t* coarse, int64_t n_planes, int32_t nu_c, int32_t nv_c,
                         int32_t factor, double scale, double* out, void* stream) {
    if (!coarse || !out || n_planes < 1 || nu_c < 1 || nv_c < 1 || factor < 1) return MC_EINVAL;
    if (!std::isfinite(scale)) return MC_EINVAL;
    if ((uint64_t)nu_c * factor >= (1ull << 20) || (uint64_t)nv_c * factor >= (1ull << 20)) return MC_EINVAL;
    if ((uint64_t)n_planes * nu_c * factor * nv_c * factor >= (1ull << 40)) return MC_EINVAL;
    const hipError_t e = launch_expand(coarse, (uint64_t)n_planes, nu_c, nv_c, factor, scale, out,
                                       (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_source_total(const uint32_t* activity, const uint32_t* activity_prev, int64_t n_vox,
                    uint64_t* total, void* stream) {
    if (!activity || !total || n_vox < 1) return MC_EINVAL;
    const hipError_t e = launch_source_total(activity, activity_prev, (uint64_t)n_vox,
                                             (unsigned long long*)total, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_scale_tally(const int64_t* tally, int64_t n, double scale, double* out, int32_t accumulate,
                   void* stream) {
    if (!tally || !out || n < 1 || !std::isfinite(scale)) return MC_EINVAL;
    if (accumulate != 0 && accumulate != 1) return MC_EINVAL;
    const hipError_t e = launch_scale_tally(tally, (uint64_t)n, scale, out, accumulate, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

}  // extern "C"

struct mc_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int mc_graph_begin(void* stream) {
    if (!stream) return MC_EINVAL;   // the legacy default stream cannot be captured
    const hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_graph_end(void* stream, mc_graph* out) {
    if (!stream || !out) return MC_EINVAL;
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
    if (e != hipSuccess) return hip_fail(e);
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e);
    }
    mc_graph h = new (std::nothrow) mc_graph_s;
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return MC_ENOMEM;
    }
    h->graph = g;
    h->exec = x;
    *out = h;
    return MC_OK;
}

int mc_graph_launch(mc_graph graph, void* stream) {
    if (!graph) return MC_EINVAL;
    const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_graph_destroy(mc_graph graph) {
    if (!graph) return MC_OK;
    hipError_t e = hipGraphExecDestroy(graph->exec);
    const hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? MC_OK : hip_fail(e);
}

int mc_autotune(const mc_problem* problems, int32_t n_problems, const mc_options* candidates,
                int32_t n_candidates, int32_t reps, int64_t* tally, int64_t* fates, int64_t* status,
                void* workspace, size_t workspace_bytes, void* stream, int32_t* best, float* times_ms) {
    if (!problems || n_problems < 1 || !candidates || n_candidates < 1 || reps < 1 || !best)
        return MC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return hip_fail(e);
    }
    int rc = MC_OK;
    float best_ms = 0.0f;
    *best = -1;
    for (int32_t c = 0; c < n_candidates && rc == MC_OK; ++c) {
        mc_options o = candidates[c];
        o.kernel_events[0] = nullptr;
        o.kernel_events[1] = nullptr;
        rc = simulate_impl(problems, n_problems, &o, tally, nullptr, fates, nullptr, nullptr, nullptr, 0,
                           nullptr, status, workspace, workspace_bytes, stream);     // untimed
        o.kernel_events[0] = ev[0];
        o.kernel_events[1] = ev[1];
        float t_c = 0.0f;
        for (int32_t r = 0; r < reps && rc == MC_OK; ++r) {
            rc = simulate_impl(problems, n_problems, &o, tally, nullptr, fates, nullptr, nullptr, nullptr,
                               0, nullptr, status, workspace, workspace_bytes, stream);
            if (rc != MC_OK) break;
            float ms = 0.0f;
            if ((e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                rc = hip_fail(e);
                break;
            }
            if (r == 0 || ms < t_c) t_c = ms;
        }
        if (rc != MC_OK) break;
        if (times_ms) times_ms[c] = t_c;
        if (*best < 0 || t_c < best_ms) {
            *best = c;
            best_ms = t_c;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    (void)st;
    return rc;
}

int mc_check_status(const int64_t* status, void* stream) {
    if (!status) return MC_EINVAL;
    int64_t st = 0;
    hipError_t e = hipMemcpyAsync(&st, status, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    if (st & (MC_STATUS_BAD_MU | MC_STATUS_NO_ACTIVITY | MC_STATUS_BAD_ANGLE | MC_STATUS_BAD_EVENT))
        return MC_EINVAL;
    if (st & (MC_STATUS_GRAD_OVERFLOW | MC_STATUS_TALLY_OVERFLOW | MC_STATUS_ACTIVITY_OVERFLOW))
        return MC_EOVERFLOW;
    if (st & MC_STATUS_LIST_OVERFLOW) return MC_ENOMEM;
    if (st & MC_STATUS_CAPPED) return MC_ECAPPED;
    return MC_OK;
}

const char* mc_error_string(int code) {
    switch (code) {
        case MC_OK: return "ok";
        case MC_EINVAL: return "invalid argument";
        case MC_ENOMEM: return "workspace or capacity too small";
        case MC_EDEVICE: return "HIP error";
        case MC_EOVERFLOW: return "fixed-point overflow";
        case MC_ECAPPED: return "history step cap reached";
        default: return "unknown error";
    }
}

int mc_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
