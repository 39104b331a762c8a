// FP64 CPU oracle for Monte Carlo SPECT photon transport.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU library is checked against.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the product path never does.
// It shares no code, header or table with the GPU library.
//
// What it computes (paper: Zhou et al., "Application of Monte Carlo algorithms
// to cardiac imaging reconstruction"):
//  * history-by-history photon transport, each photon followed from emission to
//    absorption, energy cut or escape, with tallies and their second moments
//    (Sec. 2);
//  * a rotating parallel-hole camera that accepts photons travelling
//    perpendicular to its face, with a photopeak energy window (Sec. 3);
//  * Monte Carlo estimates of the response matrix T_ij, the probability that a
//    photon emitted in source voxel i is counted in projection bin j (Sec. 5.1,
//    Eq. IMC);
//  * the path-frozen likelihood-ratio gradient of the tallies with respect to
//    the attenuation map, and its finite-difference check;
//  * forced detection (Sec. 5.2): at emission and at every interaction a copy
//    forced to the detector, weighted by the probabilities of not being
//    absorbed there, of leaving in a direction the collimator passes and of
//    crossing the rest of the object.
//
// The paper gives no cross-section model, tracking scheme, sampler or random
// number generator.  The readings used here:
//  * attenuation mu_v(E) = mu_v * g(E) (density-scaled water);
//    g(E) = (1-f) sigma_KN(E)/sigma_KN(140) + f (140/E)^3, f = photoelectric
//    share at 140 keV; p_pe(E) = f (140/E)^3 / g(E);
//  * Woodcock (delta) tracking against mu_max(E) = max_v mu_v * g(E); a
//    tentative collision in voxel v is real iff (r >> 8) < Q_v with
//    Q_v = ceil(mu_v 2^24 / max mu), computed in FP64;
//  * Compton polar angle by Kahn's rejection sampler for the Klein-Nishina
//    distribution (Kahn 1954), azimuth uniform;
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key (seed, problem),
//    counter (history, view, event, sub-draw);
//  * uniform u(r) = ((r >> 9) + 1/2) 2^-23, exactly representable in FP32 and
//    FP64;
//  * ideal collimator: accept iff d . n_view >= cos(alpha).
//
// Everything is double precision except the integer work (Philox, the activity
// CDF, the accept thresholds), which is exact.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 from its published definition: 10 rounds, each round two
// 32x32->64 products of counter words 0 and 2 with fixed multipliers, output
// words mixed with the other counter words and the key; the key advances by the
// Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Words { uint32_t r[4]; };

Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                    uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n1 = lo1;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        const uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    Words w;
    w.r[0] = c0; w.r[1] = c1; w.r[2] = c2; w.r[3] = c3;
    return w;
}

// Uniform on (0,1) from the top 23 bits of a word: (2m+1) / 2^24.
double uniform(uint32_t r) { return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0); }

// ---------------------------------------------------------------------------
// Physics (double precision).
// ---------------------------------------------------------------------------
const double E0_KEV = 140.0;        // energy the attenuation map is given at (and Tc-99m line)
const double MEC2_KEV = 510.99895;  // electron rest energy (CODATA 2018)
const double PI = 3.14159265358979323846;

// Klein-Nishina total cross-section per electron, in units of 2 pi r_e^2.
double kn_total(double e_kev) {
    const double k = e_kev / MEC2_KEV;
    const double a = 1.0 + 2.0 * k;
    const double l = std::log(a);
    return (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k) + l / (2.0 * k)
           - (1.0 + 3.0 * k) / (a * a);
}

struct XS {
    double f_pe, kn140;
    // g(E): total attenuation at E relative to 140 keV.
    double g(double e) const {
        const double r = E0_KEV / e;
        return (1.0 - f_pe) * kn_total(e) / kn140 + f_pe * r * r * r;
    }
    double p_pe(double e) const {
        const double r = E0_KEV / e;
        return f_pe * r * r * r / g(e);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Problem description (mirrors the Python ctypes structure field by field).
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
    int32_t nx, ny, nz, source_mode;
    double voxel_cm;
    const float* mu140;          // [nz][ny][nx], 1/cm at 140 keV
    const uint32_t* activity;    // [nz][ny][nx]
    int32_t n_views, nu, nv, image_factor;
    const double* angle_rad;     // [n_views]
    double pixel_cm, radius_cm, accept_half_angle_rad;
    double e_lo_kev, e_hi_kev, e_cut_kev, pe_fraction;
    uint64_t n_histories, history_offset, history_count;
    uint32_t seed, problem_id, max_steps, n_threads;
    const uint32_t* activity_prev;   // nullable: the source is activity - activity_prev
    double e0_kev;                   // emission line energy (0: 140 keV)
    int32_t vr_flags;                // VR_FORCED_DIRECTION | VR_FORCED_INTERACTION
    int32_t escape_shortcut;         // 0 (default): plain Woodcock walk to the grid edge;
                                     // 1: escape at once outside the attenuation box
    double vr_cone_rad;              // forced direction: cone half-angle about the view normal
} orc_problem;

typedef struct {
    int64_t fates[8];       // ABSORBED CUT ESCAPED ESCAPED_FOV OUT_OF_WINDOW TALLIED CAPPED spare
    double energy[4];       // deposited, escaped, capped, spare (keV)
    int64_t n_tent, n_real, n_kahn, n_hist;
} orc_result;

typedef struct {
    int32_t fate, view, iu, iv, n_scatter, n_tent, emit_voxel, cls;
    double e_final;
} orc_record;

}  // extern "C"

namespace {

enum Fate { ABSORBED = 0, CUT = 1, ESCAPED = 2, ESCAPED_FOV = 3, OUT_OF_WINDOW = 4,
            TALLIED = 5, CAPPED = 6 };

const uint32_t KAHN_MAX_ATTEMPTS = 64;

// Everything derived from the inputs before any history runs.
struct Setup {
    const orc_problem* p;
    double H[3], L[3];
    double mu_hat;                 // max_v mu_v
    std::vector<uint32_t> Q;       // accept thresholds
    std::vector<uint64_t> cdf;     // inclusive prefix sum of activity
    uint64_t total;
    XS xs;
    double cos_alpha;
    std::vector<double> nvec_x, nvec_y;  // view normals
    uint64_t q_per_view, r_extra;
    uint64_t begin, end;           // global work range
    int box_first[3], box_last[3]; // attenuation box: voxel index range of mu > 0
    bool box_empty;
};


// Reuse of photon tracks (Sec. 5.3): the projection of the new estimate is
// the old projection plus the projection of the difference d = lambda(k) -
// lambda(k-1) (activity - activity_prev), a source of signed activity.  Its
// histories are drawn from |d| and every tally contribution carries the sign
// of d at the emitting voxel.
double source_sign(const orc_problem* p, int32_t vox) {
    return (p->activity_prev && p->activity[vox] < p->activity_prev[vox]) ? -1.0 : 1.0;
}

// Emission line (Sec. 3: Tc-99m emits at 140 keV, Tl-201 at 71 and 167 keV;
// a multi-line source is one problem per line).  The attenuation map stays
// given at 140 keV and g(E) scales it to any energy.
double emission_energy(const orc_problem* p) { return p->e0_kev > 0.0 ? p->e0_kev : E0_KEV; }

// Variance reduction by weighting (Sec. 5.2).  Forced direction: every
// photon leaves in the cone of half-angle beta about the view normal, with
// weight Omega / (4 pi) = (1 - cos beta) / 2 (unbiased for the photons that
// start inside the cone; the scatter of those emitted outside it is left
// out).  Forced interaction: a real collision is always a Compton scatter and
// the weight takes the factor sigma_C / sigma_tot = 1 - p_pe(E).  A tallied
// photon adds its weight (tally) and its squared weight (tally_sq).
const int32_t VR_FORCED_DIRECTION = 1, VR_FORCED_INTERACTION = 2;

bool build_setup(const orc_problem* p, Setup& s) {
    s.p = p;
    const double e0 = emission_energy(p);
    if (!(e0 >= p->e_cut_kev && e0 <= 500.0)) return false;
    if (p->vr_flags < 0 || p->vr_flags > 3) return false;
    if ((p->vr_flags & VR_FORCED_DIRECTION) && !(p->vr_cone_rad > 0.0 && p->vr_cone_rad <= PI)) return false;
    const size_t nvox = (size_t)p->nx * p->ny * p->nz;
    s.L[0] = p->nx * p->voxel_cm; s.L[1] = p->ny * p->voxel_cm; s.L[2] = p->nz * p->voxel_cm;
    for (int a = 0; a < 3; ++a) s.H[a] = 0.5 * s.L[a];
    s.mu_hat = 0.0;
    for (size_t i = 0; i < nvox; ++i) {
        const double m = p->mu140[i];
        if (!(m >= 0.0) || !std::isfinite(m)) return false;
        s.mu_hat = std::max(s.mu_hat, m);
    }
    s.Q.assign(nvox, 0);
    for (size_t i = 0; i < nvox; ++i) {
        if (s.mu_hat > 0.0) {
            double q = std::ceil((double)p->mu140[i] * 16777216.0 / s.mu_hat);
            q = std::min(std::max(q, 0.0), 16777216.0);
            s.Q[i] = (uint32_t)q;
        }
    }
    int lo[3] = {p->nx, p->ny, p->nz}, hi[3] = {-1, -1, -1};
    for (size_t i = 0; i < nvox; ++i) {
        if (!(p->mu140[i] > 0.0f)) continue;
        const int c[3] = {(int)(i % p->nx), (int)((i / p->nx) % p->ny), (int)(i / ((size_t)p->nx * p->ny))};
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], c[a]); hi[a] = std::max(hi[a], c[a]); }
    }
    s.box_empty = hi[0] < 0;
    for (int a = 0; a < 3; ++a) { s.box_first[a] = lo[a]; s.box_last[a] = hi[a]; }
    // a difference source (reuse of photon tracks) emits in proportion to
    // the magnitude of the difference
    s.cdf.assign(nvox, 0);
    uint64_t acc = 0;
    for (size_t i = 0; i < nvox; ++i) {
        const int64_t a = (int64_t)p->activity[i] - (p->activity_prev ? (int64_t)p->activity_prev[i] : 0);
        acc += (uint64_t)(a < 0 ? -a : a);
        s.cdf[i] = acc;
    }
    s.total = acc;
    if (s.total == 0) return false;
    s.xs.f_pe = p->pe_fraction;
    s.xs.kn140 = kn_total(E0_KEV);
    s.cos_alpha = std::cos(p->accept_half_angle_rad);
    s.nvec_x.resize(p->n_views); s.nvec_y.resize(p->n_views);
    for (int k = 0; k < p->n_views; ++k) {
        s.nvec_x[k] = std::cos(p->angle_rad[k]);
        s.nvec_y[k] = std::sin(p->angle_rad[k]);
    }
    // Histories per view: N_k = floor(N/V) + [k < N mod V]; work index g runs
    // view-major over (view, history id).
    s.q_per_view = p->n_histories / (uint64_t)p->n_views;
    s.r_extra = p->n_histories % (uint64_t)p->n_views;
    s.begin = p->history_offset;
    s.end = p->history_count ? p->history_offset + p->history_count : p->n_histories;
    if (s.end > p->n_histories || s.begin > s.end) return false;
    return true;
}

void work_to_view_hist(const Setup& s, uint64_t g, int32_t& view, uint64_t& hist) {
    const uint64_t big = s.q_per_view + 1;
    if (g < s.r_extra * big) {
        view = (int32_t)(g / big);
        hist = g % big;
    } else {
        const uint64_t g2 = g - s.r_extra * big;
        view = (int32_t)(s.r_extra + g2 / s.q_per_view);
        hist = g2 % s.q_per_view;
    }
}

// One real collision / segment end, kept for the adjoint.
struct Vertex { double x[3]; double e_after; };

struct History {
    int32_t fate = -1, view = 0, iu = -1, iv = -1, n_scatter = 0, n_tent = 0, n_real = 0,
            n_kahn = 0, emit_voxel = -1, cls = 0;
    double e = E0_KEV, dep = 0.0, esc = 0.0, capped = 0.0;
    double sign = 1.0;           // of the emitting voxel's activity (signed source)
    double w = 1.0;              // statistical weight (forced direction / interaction)
    // path (only filled when requested)
    std::vector<Vertex> verts;   // emission point, then each Compton vertex
    double dfinal[3] = {0, 0, 0};
};

bool voxel_of(const Setup& s, const double x[3], int idx[3]) {
    for (int a = 0; a < 3; ++a) {
        const double t = x[a] + s.H[a];
        if (!(t >= 0.0 && t < s.L[a])) return false;
    }
    const int n[3] = {s.p->nx, s.p->ny, s.p->nz};
    for (int a = 0; a < 3; ++a) {
        int i = (int)std::floor((x[a] + s.H[a]) / s.p->voxel_cm);
        idx[a] = std::min(i, n[a] - 1);
    }
    return true;
}

// True if voxel idx lies outside the attenuation box on some axis and d does
// not point back towards the box on that axis: the ray can never enter the
// box again, so every later collision would be virtual.
bool leaves_box(const Setup& s, const int idx[3], const double d[3]) {
    if (s.box_empty) return false;   // no attenuation anywhere: no shortcut
    for (int a = 0; a < 3; ++a) {
        if (idx[a] < s.box_first[a] && d[a] <= 0.0) return true;
        if (idx[a] > s.box_last[a] && d[a] >= 0.0) return true;
    }
    return false;
}

// Rotate direction d by polar angle (cos_t) and azimuth phi.
void rotate(double d[3], double cos_t, double phi) {
    const double sin_t = std::sqrt(std::max(0.0, 1.0 - cos_t * cos_t));
    const double cp = std::cos(phi), sp = std::sin(phi);
    const double u = d[0], v = d[1], w = d[2];
    if (std::fabs(w) > 0.99999) {
        d[0] = sin_t * cp;
        d[1] = sin_t * sp;
        d[2] = (w > 0 ? 1.0 : -1.0) * cos_t;
    } else {
        const double t = std::sqrt(1.0 - w * w);
        d[0] = sin_t * (u * w * cp - v * sp) / t + u * cos_t;
        d[1] = sin_t * (v * w * cp + u * sp) / t + v * cos_t;
        d[2] = -sin_t * cp * t + w * cos_t;
    }
}

void segment_voxels(const Setup& s, const double a[3], const double b[3],
                    std::vector<std::pair<size_t, double>>& out);

// ---------------------------------------------------------------------------
// Forced detection (Sec. 5.2).  At the emission point and at every real
// collision a copy of the photon is forced towards this view's detector and
// scored with the weight the paper lists: the probability that it is not
// absorbed at the point, that it leaves in a direction the collimator passes,
// and that it crosses the rest of the object without interacting.  The
// direction is drawn uniformly in the collimator cone (Philox event of the
// point, sub-draw FD_SUB, words 0 and 1), so
//   w = Omega_cone * pdf(direction) * exp(-g(E') * integral of mu140 on the ray)
// with pdf = 1/(4 pi) at emission and (1 - p_pe(E)) * Klein-Nishina angular pdf
// at a collision, and the expected score equals the expected analog count in
// every bin.  A copy whose energy would be cut or falls outside the window, or
// that misses the detector, scores nothing.
// ---------------------------------------------------------------------------
const uint32_t FD_SUB = 0x80000000u;

// Klein-Nishina angular density per steradian at energy e (normalised over
// the sphere): (r_e^2/2) eps^2 (eps + 1/eps - sin^2) / sigma_KN(e).
double kn_pdf(double e, double cos_t) {
    const double k = e / MEC2_KEV;
    const double eps = 1.0 / (1.0 + k * (1.0 - cos_t));
    return eps * eps * (eps + 1.0 / eps - (1.0 - cos_t * cos_t)) / (4.0 * PI * kn_total(e));
}

// Integral of mu140 along the ray x + t d, t >= 0, to where it leaves the grid.
double ray_mu_integral(const Setup& s, const double x[3], const double d[3]) {
    const double far = 4.0 * (s.L[0] + s.L[1] + s.L[2]);
    const double b[3] = {x[0] + far * d[0], x[1] + far * d[1], x[2] + far * d[2]};
    std::vector<std::pair<size_t, double>> pieces;
    segment_voxels(s, x, b, pieces);
    double sum = 0.0;
    for (auto& pc : pieces) sum += (double)s.p->mu140[pc.first] * pc.second;
    return sum;
}

int32_t image_voxel(const orc_problem* p, int32_t vox);

struct FdSink {
    std::vector<double>* tally;
    std::vector<double>* tally_sq;
    bool cfd = false;              // convolution-based: deposit into depth layers
    std::vector<std::pair<size_t, double>> layer_dep;   // (layer bin, weight)
    bool want_trip = false;
    int32_t emit_img = 0;          // image voxel of the current history's emission
    double sign = 1.0;             // sign of its source (signed source)
    int64_t work = 0;              // its work index relative to history_offset
    std::vector<int64_t> ti, tj, tg;
    std::vector<double> tw;
};

// ---------------------------------------------------------------------------
// Convolution-based forced detection (CFD, Sec. 5.2).  The forced copy goes
// along the perpendicular n_k to the detector: its weight is the forced-
// detection weight with the direction at the cone axis, Omega_cone * pdf(n_k)
// * exp(-g(E') * integral of mu140 along n_k), and instead of being followed
// it is stored in a sub-projection layer: layer l = floor(d / pixel) of the
// depth d = D - n_k . x, pixel of the perpendicular hit (u_k . x, z).  After
// all histories each layer is convolved with the collimator response at its
// depth (cfd_kernel) and the layers are summed into the projection.
// ---------------------------------------------------------------------------
int cfd_layers(const orc_problem* p) {
    return (int)std::ceil(2.0 * p->radius_cm / p->pixel_cm);
}

// Collimator response at depth d (cm) on the pixel grid: a cone of half-angle
// alpha with directions uniform in solid angle spreads a point's photons over
// a disk of radius d tan(alpha) with plane density d / (2 pi (1 - cos a)
// (d^2 + r^2)^(3/2)).  Integrated over each pixel with CFD_SUB x CFD_SUB
// midpoint samples, normalised to sum 1; offsets -h..h.  Returns h.
const int CFD_SUB = 8;
int cfd_half_width(double d, double tan_a, double pix) {
    return (int)std::ceil(d * tan_a / pix + 0.5);
}
void cfd_kernel(double d, double alpha, double pix, int h, std::vector<double>& k) {
    const int n = 2 * h + 1;
    k.assign((size_t)n * n, 0.0);
    const double rho = d * std::tan(alpha), omc = 1.0 - std::cos(alpha);
    double tot = 0.0;
    for (int b = -h; b <= h; ++b)
        for (int a = -h; a <= h; ++a) {
            double acc = 0.0;
            for (int t = 0; t < CFD_SUB; ++t)
                for (int u = 0; u < CFD_SUB; ++u) {
                    const double x = (a + (u + 0.5) / CFD_SUB - 0.5) * pix;
                    const double y = (b + (t + 0.5) / CFD_SUB - 0.5) * pix;
                    const double r2 = x * x + y * y;
                    if (r2 > rho * rho) continue;
                    acc += d / (2.0 * PI * omc * std::pow(d * d + r2, 1.5));
                }
            acc *= (pix / CFD_SUB) * (pix / CFD_SUB);
            k[(size_t)(b + h) * n + (a + h)] = acc;
            tot += acc;
        }
    if (tot > 0.0) for (auto& v : k) v /= tot;
    else k[(size_t)h * n + h] = 1.0;
}

void cfd_score(const Setup& s, int32_t view, const double x[3], const double* d_in, double e,
               int cls, FdSink& sink) {
    const orc_problem* p = s.p;
    const double nx = s.nvec_x[view], ny = s.nvec_y[view];
    const double o[3] = {nx, ny, 0.0};
    const double omega = 2.0 * PI * (1.0 - s.cos_alpha);
    double weight, e2;
    if (!d_in) {
        weight = omega / (4.0 * PI);
        e2 = e;
    } else {
        const double ct = d_in[0] * nx + d_in[1] * ny;
        e2 = e / (1.0 + (e / MEC2_KEV) * (1.0 - ct));
        weight = (1.0 - s.xs.p_pe(e)) * omega * kn_pdf(e, ct);
    }
    if (e2 < p->e_cut_kev || !(e2 >= p->e_lo_kev && e2 <= p->e_hi_kev)) return;
    const double wu = p->nu * p->pixel_cm, wv = p->nv * p->pixel_cm;
    const double au = (-ny * x[0] + nx * x[1]) + 0.5 * wu;
    const double av = x[2] + 0.5 * wv;
    if (!(au >= 0.0 && au < wu && av >= 0.0 && av < wv)) return;
    const int iu = std::min((int)std::floor(au / p->pixel_cm), p->nu - 1);
    const int iv = std::min((int)std::floor(av / p->pixel_cm), p->nv - 1);
    const int L = cfd_layers(p);
    const double depth = p->radius_cm - (x[0] * nx + x[1] * ny);
    const int l = std::min(std::max((int)std::floor(depth / p->pixel_cm), 0), L - 1);
    const double score = sink.sign * weight * std::exp(-s.xs.g(e2) * ray_mu_integral(s, x, o));
    const size_t b = ((((size_t)view * L + l) * 2 + cls) * p->nv + iv) * p->nu + iu;
    sink.layer_dep.emplace_back(b, score);
}

void fd_score(const Setup& s, int32_t view, uint64_t hist, uint32_t event, const double x[3],
              const double* d_in, double e, int cls, FdSink& sink) {
    const orc_problem* p = s.p;
    if (sink.cfd) { cfd_score(s, view, x, d_in, e, cls, sink); return; }
    const Words w = philox4x32_10((uint32_t)hist, (uint32_t)view, event, FD_SUB, p->seed,
                                  p->problem_id);
    const double cos_b = 1.0 - uniform(w.r[0]) * (1.0 - s.cos_alpha);
    const double nx = s.nvec_x[view], ny = s.nvec_y[view];
    double o[3] = {nx, ny, 0.0};
    rotate(o, cos_b, 2.0 * PI * uniform(w.r[1]));
    const double omega = 2.0 * PI * (1.0 - s.cos_alpha);
    double weight, e2;
    if (!d_in) {
        weight = omega / (4.0 * PI);
        e2 = e;
    } else {
        const double ct = d_in[0] * o[0] + d_in[1] * o[1] + d_in[2] * o[2];
        e2 = e / (1.0 + (e / MEC2_KEV) * (1.0 - ct));
        weight = (1.0 - s.xs.p_pe(e)) * omega * kn_pdf(e, ct);
    }
    if (e2 < p->e_cut_kev || !(e2 >= p->e_lo_kev && e2 <= p->e_hi_kev)) return;
    const double dn = o[0] * nx + o[1] * ny;
    const double tp = (p->radius_cm - (x[0] * nx + x[1] * ny)) / dn;
    const double px = x[0] + tp * o[0], py = x[1] + tp * o[1], pz = x[2] + tp * o[2];
    const double wu = p->nu * p->pixel_cm, wv = p->nv * p->pixel_cm;
    const double au = (-ny * px + nx * py) + 0.5 * wu;
    const double av = pz + 0.5 * wv;
    if (!(au >= 0.0 && au < wu && av >= 0.0 && av < wv)) return;
    const int iu = std::min((int)std::floor(au / p->pixel_cm), p->nu - 1);
    const int iv = std::min((int)std::floor(av / p->pixel_cm), p->nv - 1);
    const double score = sink.sign * weight * std::exp(-s.xs.g(e2) * ray_mu_integral(s, x, o));
    const size_t b = (((size_t)view * 2 + cls) * p->nv + iv) * p->nu + iu;
    (*sink.tally)[b] += score;
    (*sink.tally_sq)[b] += score * score;
    if (sink.want_trip) {
        sink.ti.push_back(sink.emit_img);
        sink.tj.push_back((int64_t)b);
        sink.tw.push_back(score);
        sink.tg.push_back(sink.work);
    }
}

// Kahn's rejection sampler (Kahn 1954) for x = E/E' of a Compton scatter at
// energy e, x on [1, 1+2k] with k = e / m_e c^2: attempt a takes its three
// uniforms from Philox counter (c0, c1, event, 1 + a).  With probability
// (1+2k)/(9+2k) the candidate is x = 1 + 2k rho2, kept if rho3 <= 4 (1/x -
// 1/x^2); otherwise x = (1+2k)/(1 + 2k rho2), kept if rho3 <= (c^2 + 1/x)/2
// with c = 1 - (x-1)/k.  Returns x, or NaN when KAHN_MAX_ATTEMPTS attempts
// all fail; *attempts receives the number of attempts made.  The transport
// and the sampler check below both call this one function.
double kahn_sample(double e, uint32_t c0, uint32_t c1, uint32_t event, uint32_t k0, uint32_t k1,
                   int32_t* attempts) {
    const double k = e / MEC2_KEV;
    for (uint32_t a = 0; a < KAHN_MAX_ATTEMPTS; ++a) {
        *attempts = (int32_t)a + 1;
        const Words wk = philox4x32_10(c0, c1, event, 1 + a, k0, k1);
        const double r1 = uniform(wk.r[0]), r2 = uniform(wk.r[1]), r3 = uniform(wk.r[2]);
        if (r1 <= (1.0 + 2.0 * k) / (9.0 + 2.0 * k)) {
            const double xx = 1.0 + 2.0 * k * r2;
            if (r3 <= 4.0 * (1.0 / xx - 1.0 / (xx * xx))) return xx;
        } else {
            const double xx = (1.0 + 2.0 * k) / (1.0 + 2.0 * k * r2);
            const double c = 1.0 - (xx - 1.0) / k;
            if (r3 <= 0.5 * (c * c + 1.0 / xx)) return xx;
        }
    }
    return NAN;
}

// Transport one history.  view/hist identify its random stream.
void run_history(const Setup& s, int32_t view, uint64_t hist, bool keep_path, History& h,
                 FdSink* fd = nullptr) {
    const orc_problem* p = s.p;
    const uint32_t k0 = p->seed, k1 = p->problem_id;
    const uint32_t c0 = (uint32_t)hist, c1 = (uint32_t)view;
    h.view = view;

    // --- emission: event 0, sub-draws 0 and 1 ---
    const Words w0 = philox4x32_10(c0, c1, 0, 0, k0, k1);
    const Words w1 = philox4x32_10(c0, c1, 0, 1, k0, k1);
    const uint64_t R = ((uint64_t)w0.r[0] << 32) | w0.r[1];
    const uint64_t t = (uint64_t)(((unsigned __int128)R * s.total) >> 64);
    // voxel i with cdf[i-1] <= t < cdf[i]
    const size_t vox = (size_t)(std::upper_bound(s.cdf.begin(), s.cdf.end(), t) - s.cdf.begin());
    h.emit_voxel = (int32_t)vox;
    h.sign = source_sign(p, (int32_t)vox);
    double x[3];
    if (p->source_mode == 1) {
        x[0] = x[1] = x[2] = 0.0;
    } else {
        const int ix = (int)(vox % p->nx);
        const int iy = (int)((vox / p->nx) % p->ny);
        const int iz = (int)(vox / ((size_t)p->nx * p->ny));
        x[0] = -s.H[0] + (ix + uniform(w0.r[2])) * p->voxel_cm;
        x[1] = -s.H[1] + (iy + uniform(w0.r[3])) * p->voxel_cm;
        x[2] = -s.H[2] + (iz + uniform(w1.r[0])) * p->voxel_cm;
    }
    double d[3];
    if (p->vr_flags & VR_FORCED_DIRECTION) {
        // forced direction: uniform in the cone of half-angle beta about the
        // view normal (the same two words), weight Omega / (4 pi)
        const double cb = std::cos(p->vr_cone_rad);
        d[0] = s.nvec_x[view]; d[1] = s.nvec_y[view]; d[2] = 0.0;
        rotate(d, 1.0 - uniform(w1.r[1]) * (1.0 - cb), 2.0 * PI * uniform(w1.r[2]));
        h.w = 0.5 * (1.0 - cb);
    } else {
        const double cos_t = 2.0 * uniform(w1.r[1]) - 1.0;
        const double phi = 2.0 * PI * uniform(w1.r[2]);
        const double sin_t = std::sqrt(std::max(0.0, 1.0 - cos_t * cos_t));
        d[0] = sin_t * std::cos(phi); d[1] = sin_t * std::sin(phi); d[2] = cos_t;
    }
    double e = emission_energy(p);
    double mu_max = s.mu_hat * s.xs.g(e);
    double p_pe = s.xs.p_pe(e);
    if (keep_path) h.verts.push_back(Vertex{{x[0], x[1], x[2]}, e});
    if (fd) {
        fd->emit_img = image_voxel(p, (int32_t)vox);
        fd->sign = h.sign;
        fd_score(s, view, hist, 0, x, nullptr, e, 0, *fd);
    }

    // --- Woodcock loop: event n = 1, 2, ... ---
    uint32_t n = 0;
    for (;;) {
        ++n;
        if (n > p->max_steps) { h.fate = CAPPED; h.capped = e; break; }
        h.n_tent = (int32_t)n;
        const Words w = philox4x32_10(c0, c1, n, 0, k0, k1);
        const double step = -std::log(uniform(w.r[0])) / mu_max;
        const double xn[3] = {x[0] + step * d[0], x[1] + step * d[1], x[2] + step * d[2]};
        int idx[3];
        const bool in_grid = voxel_of(s, xn, idx);
        // Optional shortcut (off unless the problem asks for it): in the air
        // outside the attenuation box and moving away from it, every remaining
        // collision would be virtual, so the photon escapes along the same ray.
        // Exact in real arithmetic; it only drops the remaining virtual steps.
        const bool box_exit = in_grid && p->escape_shortcut && leaves_box(s, idx, d);
        if (box_exit) { x[0] = xn[0]; x[1] = xn[1]; x[2] = xn[2]; }
        if (!in_grid || box_exit) {
            // Escape: the photon leaves the grid along d from x (last inside point).
            h.esc = e;
            const double nx = s.nvec_x[view], ny = s.nvec_y[view];
            const double dn = d[0] * nx + d[1] * ny;
            if (dn < s.cos_alpha) { h.fate = ESCAPED; break; }
            const double tp = (p->radius_cm - (x[0] * nx + x[1] * ny)) / dn;
            const double px = x[0] + tp * d[0], py = x[1] + tp * d[1], pz = x[2] + tp * d[2];
            const double wu = p->nu * p->pixel_cm, wv = p->nv * p->pixel_cm;
            const double au = (-ny * px + nx * py) + 0.5 * wu;   // u_k = (-sin, cos, 0)
            const double av = pz + 0.5 * wv;
            if (!(au >= 0.0 && au < wu && av >= 0.0 && av < wv)) { h.fate = ESCAPED_FOV; break; }
            h.iu = std::min((int)std::floor(au / p->pixel_cm), p->nu - 1);
            h.iv = std::min((int)std::floor(av / p->pixel_cm), p->nv - 1);
            if (!(e >= p->e_lo_kev && e <= p->e_hi_kev)) { h.fate = OUT_OF_WINDOW; break; }
            h.fate = TALLIED;
            h.cls = h.n_scatter > 0 ? 1 : 0;
            for (int a = 0; a < 3; ++a) h.dfinal[a] = d[a];
            break;
        }
        x[0] = xn[0]; x[1] = xn[1]; x[2] = xn[2];
        const size_t v = (size_t)idx[0] + (size_t)p->nx * ((size_t)idx[1] + (size_t)p->ny * idx[2]);
        if ((w.r[1] >> 8) >= s.Q[v]) continue;           // virtual collision
        h.n_real++;
        if (fd) fd_score(s, view, hist, n, x, d, e, 1, *fd);
        if (p->vr_flags & VR_FORCED_INTERACTION) {
            h.w *= 1.0 - p_pe;                            // forced interaction: always Compton
        } else if (uniform(w.r[2]) < p_pe) {              // photoelectric absorption
            h.dep += e; h.fate = ABSORBED; break;
        }
        // Compton: Kahn's sampler for x = E/E' on [1, 1+2k].
        const double k = e / MEC2_KEV;
        int32_t attempts = 0;
        const double xr = kahn_sample(e, c0, c1, n, k0, k1, &attempts);
        h.n_kahn += attempts;
        if (std::isnan(xr)) { h.fate = CAPPED; h.capped = e; break; }
        const double cos_s = 1.0 - (xr - 1.0) / k;
        const double e_new = e / xr;
        h.dep += e - e_new;
        e = e_new;
        h.n_scatter++;
        rotate(d, cos_s, 2.0 * PI * uniform(w.r[3]));
        if (keep_path) h.verts.push_back(Vertex{{x[0], x[1], x[2]}, e});
        if (e < p->e_cut_kev) { h.fate = CUT; h.dep += e; break; }
        mu_max = s.mu_hat * s.xs.g(e);
        p_pe = s.xs.p_pe(e);
    }
    h.e = e;
}

size_t n_threads_for(const orc_problem* p) {
    size_t t = p->n_threads ? p->n_threads : std::max(1u, std::thread::hardware_concurrency());
    return std::max<size_t>(1, t);
}

template <class F>
void parallel_ranges(uint64_t begin, uint64_t end, size_t nt, F f) {
    std::vector<std::thread> th;
    const uint64_t n = end - begin;
    for (size_t t = 0; t < nt; ++t) {
        const uint64_t b = begin + n * t / nt, e = begin + n * (t + 1) / nt;
        th.emplace_back([=, &f]() { f(t, b, e); });
    }
    for (auto& x : th) x.join();
}

struct Acc {
    std::vector<double> tally, tally_sq;
    int64_t fates[8] = {0};
    double energy[4] = {0, 0, 0, 0};
    int64_t n_tent = 0, n_real = 0, n_kahn = 0, n_hist = 0;
    std::vector<int64_t> trip_i, trip_j, trip_g;
};

size_t bin_index(const orc_problem* p, int view, int cls, int iv, int iu) {
    return (((size_t)view * 2 + cls) * p->nv + iv) * p->nu + iu;
}

int32_t image_voxel(const orc_problem* p, int32_t vox) {
    const int f = p->image_factor;
    if (f <= 0) return vox;
    const int ix = vox % p->nx, iy = (vox / p->nx) % p->ny, iz = vox / (p->nx * p->ny);
    const int mx = p->nx / f, my = p->ny / f;
    return (ix / f) + mx * ((iy / f) + my * (iz / f));
}

void accumulate(const orc_problem* p, const History& h, Acc& a, bool want_tally, bool want_trip,
                uint64_t g = 0) {
    a.fates[h.fate]++;
    a.energy[0] += h.dep;
    if (h.fate == CAPPED) a.energy[2] += h.capped;
    else a.energy[1] += h.esc;
    a.n_tent += h.n_tent; a.n_real += h.n_real; a.n_kahn += h.n_kahn; a.n_hist++;
    if (h.fate == TALLIED) {
        const size_t b = bin_index(p, h.view, h.cls, h.iv, h.iu);
        if (want_tally) { a.tally[b] += h.sign * h.w; a.tally_sq[b] += h.w * h.w; }
        if (want_trip) {
            a.trip_i.push_back(image_voxel(p, h.emit_voxel));
            a.trip_j.push_back((int64_t)b);
            a.trip_g.push_back((int64_t)(g - p->history_offset));
        }
    }
}

// Exact intersection lengths of segment a->b with the voxels of the grid
// (all crossings of grid planes, sorted; the voxel of each piece is the one
// containing its midpoint).  Appends (voxel, length) pairs.
void segment_voxels(const Setup& s, const double a[3], const double b[3],
                    std::vector<std::pair<size_t, double>>& out) {
    const orc_problem* p = s.p;
    const int n[3] = {p->nx, p->ny, p->nz};
    double dir[3], len2 = 0;
    for (int k = 0; k < 3; ++k) { dir[k] = b[k] - a[k]; len2 += dir[k] * dir[k]; }
    const double len = std::sqrt(len2);
    if (len <= 0) return;
    // parameter range inside the box
    double t0 = 0.0, t1 = 1.0;
    for (int k = 0; k < 3; ++k) {
        const double lo = -s.H[k], hi = s.H[k];
        if (dir[k] == 0.0) {
            if (a[k] < lo || a[k] >= hi) return;
        } else {
            double ta = (lo - a[k]) / dir[k], tb = (hi - a[k]) / dir[k];
            if (ta > tb) std::swap(ta, tb);
            t0 = std::max(t0, ta); t1 = std::min(t1, tb);
        }
    }
    if (t1 <= t0) return;
    std::vector<double> ts;
    ts.push_back(t0); ts.push_back(t1);
    for (int k = 0; k < 3; ++k) {
        if (dir[k] == 0.0) continue;
        for (int i = 0; i <= n[k]; ++i) {
            const double plane = -s.H[k] + i * p->voxel_cm;
            const double t = (plane - a[k]) / dir[k];
            if (t > t0 && t < t1) ts.push_back(t);
        }
    }
    std::sort(ts.begin(), ts.end());
    for (size_t i = 0; i + 1 < ts.size(); ++i) {
        const double ta = ts[i], tb = ts[i + 1];
        if (tb <= ta) continue;
        const double tm = 0.5 * (ta + tb);
        int idx[3];
        bool in = true;
        for (int k = 0; k < 3; ++k) {
            const double x = a[k] + tm * dir[k];
            int ii = (int)std::floor((x + s.H[k]) / p->voxel_cm);
            if (ii < 0 || ii >= n[k]) { in = false; break; }
            idx[k] = ii;
        }
        if (!in) continue;
        const size_t v = (size_t)idx[0] + (size_t)p->nx * ((size_t)idx[1] + (size_t)p->ny * idx[2]);
        out.emplace_back(v, (tb - ta) * len);
    }
}

// The two parts of a tallied path's likelihood-ratio derivative: the
// energy-weighted length g(E_seg) len(seg n v) of every segment piece (from
// the emission point to each Compton vertex in turn, then from the last
// vertex to beyond the grid along the final direction), and the voxel of
// every Compton vertex.
void path_terms(const Setup& s, const History& h, std::vector<std::pair<size_t, double>>& pieces,
                std::vector<std::pair<size_t, double>>& lv, std::vector<size_t>& cv) {
    const orc_problem* p = s.p;
    for (size_t k = 0; k < h.verts.size(); ++k) {
        const double* a = h.verts[k].x;
        double bpt[3];
        if (k + 1 < h.verts.size()) {
            for (int c = 0; c < 3; ++c) bpt[c] = h.verts[k + 1].x[c];
        } else {
            const double far = 4.0 * (s.L[0] + s.L[1] + s.L[2]);
            for (int c = 0; c < 3; ++c) bpt[c] = a[c] + far * h.dfinal[c];
        }
        pieces.clear();
        segment_voxels(s, a, bpt, pieces);
        const double ge = s.xs.g(h.verts[k].e_after);
        for (auto& pc : pieces) lv.emplace_back(pc.first, ge * pc.second);
        if (k + 1 < h.verts.size()) {
            int idx[3];
            voxel_of(s, h.verts[k + 1].x, idx);
            cv.push_back((size_t)idx[0] + (size_t)p->nx * ((size_t)idx[1] + (size_t)p->ny * idx[2]));
        }
    }
}

}  // namespace

extern "C" {

// ---- small pieces, exposed for the closed-form checks ----
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const Words w = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = w.r[i];
}
double orc_uniform(uint32_t r) { return uniform(r); }
void orc_uniform_array(const uint32_t* r, uint64_t n, double* out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = uniform(r[i]);
}
double orc_kn_total(double e_kev) { return kn_total(e_kev); }
double orc_g(double e_kev, double f_pe) { XS xs{f_pe, kn_total(E0_KEV)}; return xs.g(e_kev); }
double orc_p_pe(double e_kev, double f_pe) { XS xs{f_pe, kn_total(E0_KEV)}; return xs.p_pe(e_kev); }

// Kahn samples of x = E/E' at energy e_kev through the transport's own
// sampler (kahn_sample): sample h uses the Philox counters of collision 1 of
// history (h mod 2^32) in "view" h >> 32 under key (seed, 0).  Returns the
// total attempt count in *attempts.
void orc_kahn_samples(double e_kev, uint32_t seed, uint64_t n, double* x_out, int64_t* attempts) {
    int64_t att = 0;
    for (uint64_t h = 0; h < n; ++h) {
        int32_t a = 0;
        x_out[h] = kahn_sample(e_kev, (uint32_t)h, (uint32_t)(h >> 32), 1, seed, 0, &a);
        att += a;
    }
    *attempts = att;
}

// Direction rotation by (cos_t, phi), exposed for checks.
void orc_rotate(double d[3], double cos_t, double phi) { rotate(d, cos_t, phi); }

// Accept thresholds as the transport uses them (exposed for checks).
int orc_thresholds(const orc_problem* p, uint32_t* q_out, double* mu_hat) {
    Setup s;
    if (!build_setup(p, s)) return -1;
    std::memcpy(q_out, s.Q.data(), s.Q.size() * sizeof(uint32_t));
    *mu_hat = s.mu_hat;
    return 0;
}

// Forward simulation.  tally / tally_sq: [V][2][nv][nu] (nullable).
// Per tallied history (capacity cap, nullable): trip_i image voxel of emission
// (phantom voxel when image_factor is 0), trip_j bin, trip_g work index
// relative to history_offset, in work-index order.
int orc_simulate(const orc_problem* p, double* tally, double* tally_sq, orc_result* res,
                 int64_t* trip_i, int64_t* trip_j, int64_t* trip_g, uint64_t trip_cap,
                 uint64_t* n_trip) {
    Setup s;
    if (!build_setup(p, s)) return -1;
    const size_t nbins = (size_t)p->n_views * 2 * p->nv * p->nu;
    const bool want_tally = tally != nullptr;
    const bool want_trip = trip_i != nullptr;
    const size_t nt = n_threads_for(p);
    std::vector<Acc> acc(nt);
    for (auto& a : acc) if (want_tally) { a.tally.assign(nbins, 0.0); a.tally_sq.assign(nbins, 0.0); }
    parallel_ranges(s.begin, s.end, nt, [&](size_t t, uint64_t b, uint64_t e) {
        for (uint64_t g = b; g < e; ++g) {
            int32_t view; uint64_t hist;
            work_to_view_hist(s, g, view, hist);
            History h;
            run_history(s, view, hist, false, h);
            accumulate(p, h, acc[t], want_tally, want_trip, g);
        }
    });
    std::memset(res, 0, sizeof(*res));
    if (want_tally) {
        std::fill(tally, tally + nbins, 0.0);
        if (tally_sq) std::fill(tally_sq, tally_sq + nbins, 0.0);
    }
    uint64_t nt_out = 0;
    for (auto& a : acc) {
        for (int i = 0; i < 8; ++i) res->fates[i] += a.fates[i];
        for (int i = 0; i < 4; ++i) res->energy[i] += a.energy[i];
        res->n_tent += a.n_tent; res->n_real += a.n_real; res->n_kahn += a.n_kahn;
        res->n_hist += a.n_hist;
        if (want_tally) for (size_t b = 0; b < nbins; ++b) {
            tally[b] += a.tally[b];
            if (tally_sq) tally_sq[b] += a.tally_sq[b];
        }
        if (want_trip) for (size_t i = 0; i < a.trip_i.size(); ++i) {
            if (nt_out < trip_cap) {
                trip_i[nt_out] = a.trip_i[i];
                trip_j[nt_out] = a.trip_j[i];
                if (trip_g) trip_g[nt_out] = a.trip_g[i];
            }
            ++nt_out;
        }
    }
    if (n_trip) *n_trip = nt_out;
    return (want_trip && nt_out > trip_cap) ? -2 : 0;
}

// Forced-detection forward simulation: the same analog histories (fates,
// energies and counters as orc_simulate), but the tally is the forced-
// detection estimate, scored at emission (class 0) and at every real collision
// (class 1); tally_sq sums the squared scores.  Analog arrivals are not tallied.
int orc_simulate_fd(const orc_problem* p, double* tally, double* tally_sq, orc_result* res,
                    int64_t* trip_i, int64_t* trip_j, double* trip_w, int64_t* trip_g,
                    uint64_t trip_cap, uint64_t* n_trip) {
    Setup s;
    if (p->vr_flags) return -1;          // forced detection runs the analog histories
    if (!build_setup(p, s)) return -1;
    const size_t nbins = (size_t)p->n_views * 2 * p->nv * p->nu;
    const size_t nt = n_threads_for(p);
    const bool want_trip = trip_i != nullptr;
    std::vector<Acc> acc(nt);
    std::vector<FdSink> sinks(nt);
    for (size_t t = 0; t < nt; ++t) {
        acc[t].tally.assign(nbins, 0.0);
        acc[t].tally_sq.assign(nbins, 0.0);
        sinks[t].tally = &acc[t].tally;
        sinks[t].tally_sq = &acc[t].tally_sq;
        sinks[t].want_trip = want_trip;
    }
    parallel_ranges(s.begin, s.end, nt, [&](size_t t, uint64_t b, uint64_t e) {
        FdSink& sink = sinks[t];
        for (uint64_t g = b; g < e; ++g) {
            int32_t view; uint64_t hist;
            work_to_view_hist(s, g, view, hist);
            History h;
            sink.work = (int64_t)(g - p->history_offset);
            run_history(s, view, hist, false, h, &sink);
            accumulate(p, h, acc[t], false, false, g);
        }
    });
    uint64_t n_out = 0;
    for (auto& k : sinks) {
        for (size_t i = 0; i < k.ti.size(); ++i) {
            if (want_trip && n_out < trip_cap) {
                trip_i[n_out] = k.ti[i]; trip_j[n_out] = k.tj[i];
                trip_w[n_out] = k.tw[i]; trip_g[n_out] = k.tg[i];
            }
            ++n_out;
        }
    }
    if (n_trip) *n_trip = n_out;
    std::memset(res, 0, sizeof(*res));
    std::fill(tally, tally + nbins, 0.0);
    if (tally_sq) std::fill(tally_sq, tally_sq + nbins, 0.0);
    for (auto& a : acc) {
        for (int i = 0; i < 8; ++i) res->fates[i] += a.fates[i];
        for (int i = 0; i < 4; ++i) res->energy[i] += a.energy[i];
        res->n_tent += a.n_tent; res->n_real += a.n_real; res->n_kahn += a.n_kahn;
        res->n_hist += a.n_hist;
        for (size_t b = 0; b < nbins; ++b) {
            tally[b] += a.tally[b];
            if (tally_sq) tally_sq[b] += a.tally_sq[b];
        }
    }
    return (want_trip && n_out > trip_cap) ? -2 : 0;
}

// Convolution-based forced detection (see cfd_score): the same analog
// histories; tally [V][2][nv][nu] = sum over depth layers of the layer
// deposits convolved with the collimator response at the layer's centre
// depth; layers (nullable) [V][L][2][nv][nu] returns the deposits.
int orc_simulate_cfd(const orc_problem* p, double* tally, double* layers, orc_result* res) {
    Setup s;
    if (p->vr_flags) return -1;
    if (!build_setup(p, s)) return -1;
    const size_t nbins = (size_t)p->n_views * 2 * p->nv * p->nu;
    const int L = cfd_layers(p);
    const size_t nlay = nbins * (size_t)L;
    const size_t nt = n_threads_for(p);
    std::vector<Acc> acc(nt);
    std::vector<FdSink> sinks(nt);
    std::vector<std::vector<double>> dummy(nt);
    for (size_t t = 0; t < nt; ++t) {
        sinks[t].tally = &dummy[t];
        sinks[t].tally_sq = &dummy[t];
        sinks[t].cfd = true;
    }
    parallel_ranges(s.begin, s.end, nt, [&](size_t t, uint64_t b, uint64_t e) {
        for (uint64_t g = b; g < e; ++g) {
            int32_t view; uint64_t hist;
            work_to_view_hist(s, g, view, hist);
            History h;
            run_history(s, view, hist, false, h, &sinks[t]);
            accumulate(p, h, acc[t], false, false, g);
        }
    });
    std::vector<double> lay(nlay, 0.0);
    for (auto& k : sinks) for (auto& d : k.layer_dep) lay[d.first] += d.second;
    if (layers) std::copy(lay.begin(), lay.end(), layers);
    std::fill(tally, tally + nbins, 0.0);
    std::vector<double> ker;
    const double tan_a = std::tan(p->accept_half_angle_rad);
    for (int l = 0; l < L; ++l) {
        const double d = (l + 0.5) * p->pixel_cm;
        const int h = cfd_half_width(d, tan_a, p->pixel_cm);
        cfd_kernel(d, p->accept_half_angle_rad, p->pixel_cm, h, ker);
        const int n = 2 * h + 1;
        for (int v = 0; v < p->n_views; ++v)
            for (int c = 0; c < 2; ++c)
                for (int iv = 0; iv < p->nv; ++iv)
                    for (int iu = 0; iu < p->nu; ++iu) {
                        const double w = lay[((((size_t)v * L + l) * 2 + c) * p->nv + iv) * p->nu + iu];
                        if (w == 0.0) continue;
                        for (int b = -h; b <= h; ++b) {
                            const int ov = iv + b;
                            if (ov < 0 || ov >= p->nv) continue;
                            for (int a = -h; a <= h; ++a) {
                                const int ou = iu + a;
                                if (ou < 0 || ou >= p->nu) continue;
                                tally[(((size_t)v * 2 + c) * p->nv + ov) * p->nu + ou] +=
                                    w * ker[(size_t)(b + h) * n + (a + h)];
                            }
                        }
                    }
    }
    std::memset(res, 0, sizeof(*res));
    for (auto& a : acc) {
        for (int i = 0; i < 8; ++i) res->fates[i] += a.fates[i];
        for (int i = 0; i < 4; ++i) res->energy[i] += a.energy[i];
        res->n_tent += a.n_tent; res->n_real += a.n_real; res->n_kahn += a.n_kahn;
        res->n_hist += a.n_hist;
    }
    return 0;
}

// Collimator response at depth d (see cfd_kernel): writes (2h+1)^2 values.
int orc_cfd_kernel(double depth_cm, double alpha, double pixel_cm, double* out, int32_t* half) {
    const int h = cfd_half_width(depth_cm, std::tan(alpha), pixel_cm);
    std::vector<double> k;
    cfd_kernel(depth_cm, alpha, pixel_cm, h, k);
    if (out) std::copy(k.begin(), k.end(), out);
    *half = h;
    return 0;
}

int32_t orc_cfd_layers(const orc_problem* p) { return cfd_layers(p); }

double orc_kn_pdf(double e_kev, double cos_t) { return kn_pdf(e_kev, cos_t); }

// Integral of mu140 from x along d to the grid edge (exact voxel pieces).
int orc_ray_integral(const orc_problem* p, const double x[3], const double d[3], double* out) {
    Setup s;
    if (!build_setup(p, s)) return -1;
    *out = ray_mu_integral(s, x, d);
    return 0;
}

// Per-history records for the listed (view, history id) pairs.
int orc_replay(const orc_problem* p, const int32_t* views, const uint64_t* hists, int64_t n,
               orc_record* out) {
    Setup s;
    if (!build_setup(p, s)) return -1;
    const size_t nt = n_threads_for(p);
    parallel_ranges(0, (uint64_t)n, nt, [&](size_t, uint64_t b, uint64_t e) {
        for (uint64_t i = b; i < e; ++i) {
            History h;
            run_history(s, views[i], hists[i], false, h);
            orc_record& r = out[i];
            r.fate = h.fate; r.view = h.view; r.iu = h.iu; r.iv = h.iv; r.n_scatter = h.n_scatter;
            r.n_tent = h.n_tent; r.emit_voxel = h.emit_voxel; r.cls = h.cls; r.e_final = h.e;
        }
    });
    return 0;
}

// Path-frozen likelihood-ratio gradient of sum_b G_b * tally_b with respect to
// the 140 keV attenuation map, and central finite differences of the Poisson
// log-likelihood L = sum_b [lam_b - y_b ln(lam_b + eps)] on listed voxels.
//
// A tallied history h sampled at mu0 has weight
//   W_h(mu) = prod_{real c} mu_{v_c}/mu0_{v_c} * exp(-sum_v (mu_v - mu0_v) lt_{h,v}),
//   lt_{h,v} = sum_seg g(E_seg) len(seg n v),
// so dW_h/dmu_v at mu0 = c_{h,v}/mu0_v - lt_{h,v}.  Segments run from the
// emission point to each Compton vertex in turn and from the last vertex to
// the grid exit along the final direction.
//
// G: [V][2][nv][nu].  grad: [nvox] (accumulated into, caller zeroes).
// n_contrib: [nvox] tallied histories touching each voxel (nullable).
// FD part (n_pert > 0): lam/y over loss bins [V][nv][nu] (classes summed),
// eps, delta; fd_out[n_pert].
int orc_adjoint(const orc_problem* p, const double* G, double* grad, int64_t* n_contrib,
                int32_t n_pert, const int32_t* pert_voxel, double delta,
                const double* lam, const double* y, double eps, double* fd_out,
                orc_result* res) {
    Setup s;
    if (p->activity_prev || p->vr_flags) return -1;   // the adjoint is of plain analog sources
    if (!build_setup(p, s)) return -1;
    const size_t nvox = (size_t)p->nx * p->ny * p->nz;
    const size_t nloss = (size_t)p->n_views * p->nv * p->nu;
    const size_t nt = n_threads_for(p);
    struct TAcc {
        std::vector<double> grad; std::vector<int64_t> contrib;
        std::vector<std::vector<std::pair<size_t, double>>> dplus, dminus;  // per pert: (loss bin, W-1)
        Acc acc;
    };
    std::vector<TAcc> ta(nt);
    for (auto& t : ta) {
        t.grad.assign(nvox, 0.0);
        if (n_contrib) t.contrib.assign(nvox, 0);
        t.dplus.resize(n_pert); t.dminus.resize(n_pert);
    }
    parallel_ranges(s.begin, s.end, nt, [&](size_t ti, uint64_t b, uint64_t e) {
        TAcc& T = ta[ti];
        std::vector<std::pair<size_t, double>> pieces;
        for (uint64_t g = b; g < e; ++g) {
            int32_t view; uint64_t hist;
            work_to_view_hist(s, g, view, hist);
            History h;
            run_history(s, view, hist, true, h);
            accumulate(p, h, T.acc, false, false);
            if (h.fate != TALLIED) continue;
            const size_t bin = bin_index(p, h.view, h.cls, h.iv, h.iu);
            const double Gb = G[bin];
            std::vector<std::pair<size_t, double>> lv;   // (voxel, g*len)
            std::vector<size_t> cv;                       // collision voxels
            path_terms(s, h, pieces, lv, cv);
            for (auto& q : lv) T.grad[q.first] -= Gb * q.second;
            for (size_t v : cv) T.grad[v] += Gb / (double)p->mu140[v];
            if (n_contrib) {
                std::vector<size_t> touched;
                for (auto& q : lv) touched.push_back(q.first);
                for (size_t v : cv) touched.push_back(v);
                std::sort(touched.begin(), touched.end());
                touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
                for (size_t v : touched) T.contrib[v]++;
            }
            const size_t lb = ((size_t)h.view * p->nv + h.iv) * p->nu + h.iu;
            for (int32_t q = 0; q < n_pert; ++q) {
                const size_t v = (size_t)pert_voxel[q];
                double L = 0.0; int c = 0;
                for (auto& x : lv) if (x.first == v) L += x.second;
                for (size_t vc : cv) if (vc == v) ++c;
                if (L == 0.0 && c == 0) continue;
                const double m0 = p->mu140[v];
                const double lp = (c ? c * std::log1p(delta / m0) : 0.0) - delta * L;
                const double lm = (c ? c * std::log1p(-delta / m0) : 0.0) + delta * L;
                T.dplus[q].emplace_back(lb, std::expm1(lp));
                T.dminus[q].emplace_back(lb, std::expm1(lm));
            }
        }
    });
    std::memset(res, 0, sizeof(*res));
    for (auto& t : ta) {
        for (size_t v = 0; v < nvox; ++v) grad[v] += t.grad[v];
        if (n_contrib) for (size_t v = 0; v < nvox; ++v) n_contrib[v] += t.contrib[v];
        for (int i = 0; i < 8; ++i) res->fates[i] += t.acc.fates[i];
        for (int i = 0; i < 4; ++i) res->energy[i] += t.acc.energy[i];
        res->n_tent += t.acc.n_tent; res->n_real += t.acc.n_real; res->n_kahn += t.acc.n_kahn;
        res->n_hist += t.acc.n_hist;
    }
    if (n_pert > 0 && lam && y && fd_out) {
        for (int32_t q = 0; q < n_pert; ++q) {
            std::vector<double> dp(nloss, 0.0), dm(nloss, 0.0);
            std::vector<char> touched(nloss, 0);
            for (auto& t : ta) {
                for (auto& x : t.dplus[q]) { dp[x.first] += x.second; touched[x.first] = 1; }
                for (auto& x : t.dminus[q]) { dm[x.first] += x.second; touched[x.first] = 1; }
            }
            // L(+) - L(-) over the bins the voxel touches
            double diff = 0.0;
            for (size_t b = 0; b < nloss; ++b) {
                if (!touched[b]) continue;
                diff += (dp[b] - dm[b]) - y[b] * std::log1p((dp[b] - dm[b]) / (lam[b] + dm[b] + eps));
            }
            fd_out[q] = diff / (2.0 * delta);
        }
    }
    return 0;
}

// The same gradient over a given list of histories: each listed (view,
// history id) is replayed and, if the oracle tallies it, adds
// G_b (c_{h,v}/mu0_v - lt_{h,v}) to grad (accumulated into; caller zeroes).
// tallied_bin[i] (nullable) receives the listed history's global bin
// (view, class, iv, iu) in the tally layout, or -1 if it is not tallied.
int orc_adjoint_list(const orc_problem* p, const double* G, const int32_t* views,
                     const uint64_t* hists, int64_t n, double* grad, int64_t* tallied_bin) {
    Setup s;
    if (p->activity_prev || p->vr_flags) return -1;
    if (!build_setup(p, s)) return -1;
    const size_t nvox = (size_t)p->nx * p->ny * p->nz;
    const size_t nt = n_threads_for(p);
    std::vector<std::vector<double>> tg(nt, std::vector<double>(nvox, 0.0));
    parallel_ranges(0, (uint64_t)n, nt, [&](size_t ti, uint64_t b, uint64_t e) {
        std::vector<std::pair<size_t, double>> pieces, lv;
        std::vector<size_t> cv;
        for (uint64_t i = b; i < e; ++i) {
            History h;
            run_history(s, views[i], hists[i], true, h);
            if (h.fate != TALLIED) {
                if (tallied_bin) tallied_bin[i] = -1;
                continue;
            }
            const size_t bin = bin_index(p, h.view, h.cls, h.iv, h.iu);
            if (tallied_bin) tallied_bin[i] = (int64_t)bin;
            lv.clear(); cv.clear();
            path_terms(s, h, pieces, lv, cv);
            const double Gb = G[bin];
            for (auto& q : lv) tg[ti][q.first] -= Gb * q.second;
            for (size_t v : cv) tg[ti][v] += Gb / (double)p->mu140[v];
        }
    });
    for (auto& t : tg) for (size_t v = 0; v < nvox; ++v) grad[v] += t[v];
    return 0;
}

}  // extern "C"
