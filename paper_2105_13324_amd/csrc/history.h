// Device-side photon history: Philox stream, physics steps and the per-lane
// state machine shared by the transport, replay and adjoint kernels.
//
// Every branch below runs for the lanes of a wavefront that are in that state
// while the others wait, so each tail is kept short: no integer division, no
// double precision, hardware transcendentals (v_log, v_sin/v_cos in
// revolutions, v_rcp, v_sqrt), and the Klein-Nishina part of the attenuation
// from a small table.  Emission is a separate, converged function: the
// kernels emit histories in batches outside the per-lane state machine.
#pragma once

#include "mc_internal.h"

namespace mcs {
namespace {

constexpr uint32_t KAHN_MAX = 64;
constexpr float MEC2_F = 510.99895f;
constexpr float INV_MEC2 = (float)(1.0 / 510.99895);
constexpr float LN2_F = 0.693147180559945f;

enum : int { S_IDLE = 0, S_STEP = 3, S_KAHN = 4 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// (words 0 and 2), xor-mixed with words 1 and 3 and the key; the key takes a
// Weyl step after every round.  The key is wave-uniform, so its steps are
// scalar adds.  Each three-way xor is one gfx950 v_bitop3_b32 (truth table
// 0x96 = a ^ b ^ c), so a round is two v_mad_u64_u32 and two bitwise ops.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// (2m+1) 2^-24 with m the top 23 bits: exact in FP32, strictly inside (0,1).
__device__ __forceinline__ float unif(uint32_t r) {
    return fmaf((float)(r >> 9), 0x1p-23f, 0x1p-24f);
}

// Load through a global (address space 1) pointer: a global_load, where a
// flat load of a pointer read from the descriptor would also wait on LDS.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ uint4 ldg(const uint4* p) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u v = *(const __attribute__((address_space(1))) v4u*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ldg(const uint2* p) {
    typedef uint32_t v2u __attribute__((ext_vector_type(2)));
    const v2u v = *(const __attribute__((address_space(1))) v2u*)p;
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float2 ldg(const float2* p) {
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = *(const __attribute__((address_space(1))) v2f*)p;
    return make_float2(v.x, v.y);
}

// A wave-uniform pointer moved to scalar registers.
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const void*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrtf_hw(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqf_hw(float x) { return __builtin_amdgcn_rsqf(x); }
// sin(2 pi u), cos(2 pi u): the hardware instructions take revolutions.
__device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }
__device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }

// Table of the Klein-Nishina attenuation shape sigma_KN(E)/sigma_KN(140 keV)
// at E = 140 - i/4 keV (filled in double precision during staging).
constexpr float KN_TABLE_STEP_INV = 4.0f;

// Problem constants a wavefront works with (wave-uniform).
struct Cst {
    const float* mu;
    const uint32_t* q32;
    const uint8_t* q8;
    const uint32_t* pal;
    const uint4* runs;
    const uint2* guide;
    const float2* views;
    const float* kn_table;
    int nx, ny, nz, source_mode;
    float hx, hy, hz, lx, ly, lz, inv_vox, vox;
    uint32_t bbx, bby, bbz;   // attenuation box per axis: first | last voxel << 16
    uint32_t box_margin;      // the box leaves air on some side of the grid
    int nu, nv, n_views;
    float inv_pix, radius, cos_alpha, wu, wv, e_lo, e_hi, e_cut;
    float f_pe, mu_hat, ln2_mm0, p_pe0, e0, g0;   // attenuation terms at the line e0
    float ln2_mu;                                 // ln 2 / max mu
    uint32_t seed, pid, max_steps, shift;
    uint64_t total, q_per_view, r_extra, work_begin, tally_offset;
    uint32_t flags, use_pal;
    int brick;
    uint32_t bmask, nbx, nby;
};

// Attenuation at energy e relative to 140 keV, g(E) = (1-f) KN(E)/KN(140) +
// f (140/E)^3, the flight scale ln2/(max mu g) (a flight is -log2(u) times
// it, with the hardware log2) and the photoelectric share f (140/E)^3 / g.
// The KN ratio is linearly interpolated (error below 1e-6 relative over the
// table range), the photoelectric term is exact.
__device__ inline float kn_ratio(const Cst& C, float e) {
    const float t = (C.e0 - e) * KN_TABLE_STEP_INV;
    const int i = (int)t;
    const float fr = t - (float)i;
    const float k0 = ldg(C.kn_table + i), k1 = ldg(C.kn_table + i + 1);
    return fmaf(fr, k1 - k0, k0);
}

// The same, given the KN table pair and fraction of e (read earlier).
__device__ inline float energy_terms_kn(const Cst& C, float e, float fr, float k0, float k1, float& ln2_mm,
                                        float& p_pe) {
    const float kn = fmaf(fr, k1 - k0, k0);
    const float x = 140.0f * rcpf(e);
    const float pe = C.f_pe * x * x * x;
    const float g = fmaf(1.0f - C.f_pe, kn, pe);
    const float ig = rcpf(g);
    ln2_mm = C.ln2_mu * ig;
    p_pe = pe * ig;
    return g;
}

__device__ inline float energy_terms(const Cst& C, float e, float& ln2_mm, float& p_pe) {
    const float kn = kn_ratio(C, e);
    const float x = 140.0f * rcpf(e);
    const float pe = C.f_pe * x * x * x;
    const float g = fmaf(1.0f - C.f_pe, kn, pe);
    const float ig = rcpf(g);
    ln2_mm = C.ln2_mu * ig;
    p_pe = pe * ig;
    return g;
}

__device__ inline Cst load_cst(const ProbDesc* __restrict__ d) {
    Cst c;
    c.mu = d->mu;
    c.q32 = d->q32; c.q8 = d->q8; c.pal = d->palette; c.runs = d->runs; c.guide = d->guide; c.views = d->views;
    c.kn_table = d->kn_table;
    c.nx = d->nx; c.ny = d->ny; c.nz = d->nz; c.source_mode = d->source_mode;
    c.hx = d->hx; c.hy = d->hy; c.hz = d->hz;
    c.lx = d->lx; c.ly = d->ly; c.lz = d->lz;
    c.inv_vox = d->inv_vox; c.vox = d->vox;
    if (d->bb_hi[0] >= 0) {
        c.bbx = (uint32_t)d->bb_lo[0] | (uint32_t)d->bb_hi[0] << 16;
        c.bby = (uint32_t)d->bb_lo[1] | (uint32_t)d->bb_hi[1] << 16;
        c.bbz = (uint32_t)d->bb_lo[2] | (uint32_t)d->bb_hi[2] << 16;
    } else {   // no attenuation anywhere: first 0, last 0xFFFF, so no shortcut
        c.bbx = c.bby = c.bbz = 0xFFFF0000u;
    }
    c.box_margin = (c.bbx != ((uint32_t)(c.nx - 1) << 16)) | (c.bby != ((uint32_t)(c.ny - 1) << 16)) |
                   (c.bbz != ((uint32_t)(c.nz - 1) << 16));
    if (d->bb_hi[0] < 0) c.box_margin = 0;
    c.nu = d->nu; c.nv = d->nv; c.n_views = d->n_views;
    c.inv_pix = d->inv_pix; c.radius = d->radius; c.cos_alpha = d->cos_alpha;
    c.wu = d->wu; c.wv = d->wv; c.e_lo = d->e_lo; c.e_hi = d->e_hi; c.e_cut = d->e_cut;
    c.f_pe = d->f_pe;
    c.mu_hat = __uint_as_float(d->mu_hat_bits);
    c.ln2_mu = (float)(0.69314718055994531 / (double)c.mu_hat);
    c.e0 = d->e0;
    if (c.e0 == 140.0f) {
        // g(140 keV) = 1 by construction: mu_max(140) = max mu, p_pe(140) = f.
        c.g0 = 1.0f;
        c.ln2_mm0 = c.ln2_mu;
        c.p_pe0 = c.f_pe;
    } else {
        c.g0 = energy_terms(c, c.e0, c.ln2_mm0, c.p_pe0);
    }
    c.seed = d->seed; c.pid = d->problem_id; c.max_steps = d->max_steps; c.shift = d->shift;
    c.total = d->total; c.q_per_view = d->q_per_view; c.r_extra = d->r_extra;
    c.work_begin = d->work_begin; c.tally_offset = d->tally_offset;
    c.flags = d->flags;
    c.use_pal = d->pal_state == 0;
    c.brick = d->brick_log2;
    c.bmask = (1u << c.brick) - 1u;
    c.nbx = (uint32_t)d->nbx; c.nby = (uint32_t)d->nby;
    return c;
}

struct Lane {
    uint32_t hist;      // history id within its view (< 2^32 by the problem checks)
    int view, state;
    uint32_t n, a, phi_word, emit_voxel;
    int n_scatter;
    float x, y, z, dx, dy, dz, e, ln2_mm, p_pe, vc, vs;
    float w;            // statistical weight (forced direction / interaction)
};

// Per-lane work counters: tentative collisions, real collisions, Kahn
// attempts (per history in replay and adjoint; the transport kernel keeps
// them over all of a lane's histories and sums them over the wave).
struct Acc {
    uint32_t n_tent, n_real, n_kahn;
};

__device__ inline void acc_zero(Acc& A) {
    A.n_tent = A.n_real = A.n_kahn = 0;
}

// keV -> Q40.23 fixed point, rounded to nearest even; |kev| < 256 fits int32.
// A history's energy is booked once: what leaves the grid (escape) or is left
// at the step cap is its outgoing energy; the rest of the 140 keV was
// deposited (the Compton deposits telescope).
__device__ __forceinline__ long long to_q23(float kev) {
    return (long long)__float2int_rn(kev * 8388608.0f);
}

// Outcome of one iteration.
enum : int { R_RUNNING = -1 };

// Voxel (ix, iy, iz) inside the attenuation box.
__device__ inline bool in_box(const Cst& C, int ix, int iy, int iz) {
    return ((uint32_t)(ix - (int)(C.bbx & 0xFFFFu)) <= (uint32_t)((int)(C.bbx >> 16) - (int)(C.bbx & 0xFFFFu))) &
           ((uint32_t)(iy - (int)(C.bby & 0xFFFFu)) <= (uint32_t)((int)(C.bby >> 16) - (int)(C.bby & 0xFFFFu))) &
           ((uint32_t)(iz - (int)(C.bbz & 0xFFFFu)) <= (uint32_t)((int)(C.bbz >> 16) - (int)(C.bbz & 0xFFFFu)));
}

// Voxel (ix, iy, iz) outside the attenuation box on some axis with the
// direction not pointing back towards the box on that axis: the ray never
// enters the box again, so every later collision would be virtual.
__device__ inline bool leaves_box(const Cst& C, int ix, int iy, int iz, float dx, float dy, float dz) {
    const int x0 = (int)(C.bbx & 0xFFFFu), x1 = (int)(C.bbx >> 16);
    const int y0 = (int)(C.bby & 0xFFFFu), y1 = (int)(C.bby >> 16);
    const int z0 = (int)(C.bbz & 0xFFFFu), z1 = (int)(C.bbz >> 16);
    return ((ix < x0) & (dx <= 0.0f)) | ((ix > x1) & (dx >= 0.0f)) |
           ((iy < y0) & (dy <= 0.0f)) | ((iy > y1) & (dy >= 0.0f)) |
           ((iz < z0) & (dz <= 0.0f)) | ((iz > z1) & (dz >= 0.0f));
}

// Per-lane escape: collimator, detector bin, window.  Returns the fate; sets iu, iv.
__device__ inline int escape(const Cst& C, const Lane& L, int& iu, int& iv) {
    const float dn = L.dx * L.vc + L.dy * L.vs;
    if (dn < C.cos_alpha) return MC_ESCAPED;
    const float tp = (C.radius - (L.x * L.vc + L.y * L.vs)) * rcpf(dn);
    const float px = fmaf(tp, L.dx, L.x);
    const float py = fmaf(tp, L.dy, L.y);
    const float pz = fmaf(tp, L.dz, L.z);
    const float au = (-L.vs * px + L.vc * py) + 0.5f * C.wu;
    const float av = pz + 0.5f * C.wv;
    if (!(au >= 0.0f && au < C.wu && av >= 0.0f && av < C.wv)) return MC_ESCAPED_FOV;
    iu = min((int)(au * C.inv_pix), C.nu - 1);
    iv = min((int)(av * C.inv_pix), C.nv - 1);
    if (!(L.e >= C.e_lo && L.e <= C.e_hi)) return MC_OUT_OF_WINDOW;
    return MC_TALLIED;
}

// Rotate unit direction (u, v, w) by polar cosine ct and azimuth phi_u (in
// revolutions): the standard formula, with the near-pole branch for
// |w| > 0.99999 (the direction then taken as +-z).
__device__ inline void rotate_dir(float& u, float& v, float& w, float ct, float phi_u) {
    const float sp = sin_rev(phi_u), cp = cos_rev(phi_u);
    const float st = sqrtf_hw(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float u0 = u, v0 = v, w0 = w;
    if (fabsf(w0) > 0.99999f) {
        u = st * cp;
        v = st * sp;
        w = w0 > 0.0f ? ct : -ct;
    } else {
        const float t2 = (1.0f - w0) * (1.0f + w0);
        const float it = rsqf_hw(t2);
        const float a = st * it;
        u = fmaf(a, u0 * w0 * cp - v0 * sp, u0 * ct);
        v = fmaf(a, v0 * w0 * cp + u0 * sp, v0 * ct);
        w = fmaf(-st * cp, t2 * it, w0 * ct);
    }
}

// rotate_dir on a lane's direction.
__device__ inline void rotate(Lane& L, float ct, float phi_u) {
    const float sp = sin_rev(phi_u), cp = cos_rev(phi_u);
    const float st = sqrtf_hw(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float u = L.dx, v = L.dy, w = L.dz;
    if (fabsf(w) > 0.99999f) {
        L.dx = st * cp;
        L.dy = st * sp;
        L.dz = w > 0.0f ? ct : -ct;
    } else {
        const float t2 = (1.0f - w) * (1.0f + w);
        const float it = rsqf_hw(t2);
        const float a = st * it;
        L.dx = fmaf(a, u * w * cp - v * sp, u * ct);
        L.dy = fmaf(a, v * w * cp + u * sp, v * ct);
        L.dz = fmaf(-st * cp, t2 * it, w * ct);
    }
}

// Philox counter words 2 and 3 of a lane's next draw: tentative collision n+1
// (sub-draw 0) or Kahn attempt a of collision n (sub-draw 1+a).
__device__ __forceinline__ void counter_of(const Lane& L, uint32_t& c2, uint32_t& c3) {
    const bool kahn = L.state == S_KAHN;
    c2 = kahn ? L.n : L.n + 1;
    c3 = kahn ? 1 + L.a : 0;
}

// Histories in view v: N_v = floor(N/V) + [v < N mod V].
__device__ __forceinline__ uint64_t hists_in_view(const Cst& C, uint64_t v) {
    return C.q_per_view + (v < C.r_extra ? 1u : 0u);
}

// Split a problem-local work index into (view, history id).  Uses 64-bit
// division: call it wave-uniformly (once per claimed chunk), not per lane.
__device__ inline void split_work(const Cst& C, uint64_t g, uint64_t& view, uint64_t& hist) {
    const uint64_t big = C.q_per_view + 1;
    if (g < C.r_extra * big) { view = g / big; hist = g - view * big; }
    else {
        const uint64_t g2 = g - C.r_extra * big;
        view = C.r_extra + g2 / C.q_per_view;
        hist = g2 - (view - C.r_extra) * C.q_per_view;
    }
}

// Move (view, hist) forward by k histories (k small): no division.
__device__ inline void advance_cursor(const Cst& C, uint64_t& view, uint64_t& hist, uint64_t k,
                                      int n_views) {
    hist += k;
    uint64_t n = hists_in_view(C, view);
    while (hist >= n && (int)view < n_views - 1) {
        hist -= n;
        ++view;
        n = hists_in_view(C, view);
    }
}

// floor(d / a) for d < 1024 a (t - c within one run, and a run lies in one
// grid row): a float estimate, within one of the quotient (its relative error
// is a few 2^-24 and the quotient is below 1024), then one integer
// correction.
__device__ __forceinline__ uint32_t div_in_run(uint64_t d, uint32_t a) {
    uint32_t q = (uint32_t)((float)d * rcpf((float)a));
    const uint64_t p = (uint64_t)q * a;
    if (p > d) --q;
    else if (p + a <= d) ++q;
    return q;
}

// Emission of history (view, hist): Philox event 0, sub-draws 0 and 1.
// Sub-draw 0: words 0-1 pick the voxel by inverse CDF, words 2-3 the x and y
// offsets in it; sub-draw 1: word 0 the z offset, word 1 cos(theta), word 2
// the azimuth.  Runs with the wavefront converged (no per-lane branches
// except the search of a bucket that meets several runs).
struct Emission {
    float x, y, z, dx, dy, dz;
    uint32_t voxel;
};

// vr_dir: forced direction (Sec. 5.2): the direction is drawn uniformly in
// the cone about the view normal with 1 - cos(half-angle) = omc, from the
// same two words that otherwise give a direction on the sphere.
__device__ inline Emission emit_history(const Cst& C, uint32_t hist, uint32_t view, bool vr_dir = false,
                                        float omc = 0.0f) {
    uint32_t a0 = hist, a1 = view, a2 = 0, a3 = 0;
    philox10(a0, a1, a2, a3, C.seed, C.pid);
    uint32_t b0 = hist, b1 = view, b2 = 0, b3 = 1;
    philox10(b0, b1, b2, b3, C.seed, C.pid);
    // voxel: t = floor(R * total / 2^64) with R the 64-bit word pair; the run
    // holding t (its bucket, rarely a search over the runs the bucket
    // meets), then the voxel within the run
    const uint64_t R = ((uint64_t)a0 << 32) | a1;
    const uint64_t t = __umul64hi(R, C.total);
    const uint2 g = ldg(C.guide + (t >> C.shift));
    uint32_t r = g.x;
    if (g.y != 0) {
        // the last run starting at or below t among runs g.x .. g.x + g.y
        uint32_t lo = g.x, hi = g.x + g.y;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            const uint2 c = ldg((const uint2*)(C.runs + mid));
            if ((((uint64_t)c.y << 32) | c.x) <= t) lo = mid; else hi = mid - 1;
        }
        r = lo;
    }
    const uint4 run = ldg(C.runs + r);
    const uint32_t packed = run.z + div_in_run(t - (((uint64_t)run.y << 32) | run.x), run.w);
    const uint32_t ix = packed & 1023u, iy = (packed >> 10) & 1023u, iz = packed >> 20;
    Emission e;
    e.voxel = ix + (uint32_t)C.nx * (iy + (uint32_t)C.ny * iz);
    if (C.source_mode == MC_SOURCE_POINT) {
        e.x = 0.0f; e.y = 0.0f; e.z = 0.0f;
    } else {
        e.x = -C.hx + ((float)ix + unif(a2)) * C.vox;
        e.y = -C.hy + ((float)iy + unif(a3)) * C.vox;
        e.z = -C.hz + ((float)iz + unif(b0)) * C.vox;
    }
    if (vr_dir) {
        const float2 vw = ldg(C.views + view);
        e.dx = vw.x; e.dy = vw.y; e.dz = 0.0f;
        rotate_dir(e.dx, e.dy, e.dz, fmaf(-unif(b1), omc, 1.0f), unif(b2));
        return e;
    }
    const float ct = fmaf(2.0f, unif(b1), -1.0f);
    const float st = sqrtf_hw((1.0f - ct) * (1.0f + ct));
    const float u = unif(b2);
    e.dx = st * cos_rev(u); e.dy = st * sin_rev(u); e.dz = ct;
    return e;
}

// Lane state at the start of transport (after emission).
__device__ inline void begin_history(const Cst& C, Lane& L, uint32_t view, uint32_t hist,
                                     const Emission& e) {
    L.hist = hist;
    L.view = (int)view;
    L.state = S_STEP;
    L.n = 0; L.a = 0; L.n_scatter = 0;
    L.emit_voxel = e.voxel;
    L.x = e.x; L.y = e.y; L.z = e.z;
    L.dx = e.dx; L.dy = e.dy; L.dz = e.dz;
    L.e = C.e0;
    L.ln2_mm = C.ln2_mm0;
    L.p_pe = C.p_pe0;
    const float2 cs = ldg(C.views + view);
    L.vc = cs.x; L.vs = cs.y;
    L.w = 1.0f;
}

// One iteration of a lane's history (tentative collision or Kahn attempt)
// given its Philox words.  Returns the fate when the history ends (iu/iv set
// for escapes), else R_RUNNING.  pal: the problem's threshold palette (global,
// or a copy in LDS), read when C.use_pal.
// fi: forced interaction (Sec. 5.2): a real collision is always a Compton
// scatter and the weight takes the factor 1 - p_pe(E).
//
// Every lane runs exactly one of the two states; the body is laid out in
// four phases so that a wavefront holding lanes of both states overlaps the
// latency of the threshold gather with the Kahn arithmetic: (1) tentative
// collision up to the gather of the voxel's threshold code (lanes that leave
// escape here), (2) the Kahn attempt and, on acceptance, the new direction
// and energy (arithmetic only), (3) the accept test of the tentative
// collision, (4) the attenuation terms at a new energy (table reads).
__device__ inline int advance(const Cst& C, const uint32_t* pal, Lane& L, uint32_t w0, uint32_t w1,
                              uint32_t w2, uint32_t w3, Acc& A, int& iu, int& iv, bool fi = false) {
    const int state = L.state;
    int fate = R_RUNNING;
    // (1) tentative collision n + 1: flight -log(u)/mu_max, the new point
    bool pending = false;
    uint32_t raw;               // set, with xn..zn, wherever pending is
    float xn, yn, zn;
    if (state == S_STEP) {
        MC_REGION(RG_STEP);
        L.n += 1;
        if (L.n > C.max_steps) {
            L.n -= 1;
            fate = MC_CAPPED_FATE;
        } else {
            A.n_tent++;
            const float s = -__builtin_amdgcn_logf(unif(w0)) * L.ln2_mm;
            xn = fmaf(s, L.dx, L.x);
            yn = fmaf(s, L.dy, L.y);
            zn = fmaf(s, L.dz, L.z);
            const float tx = xn + C.hx, ty = yn + C.hy, tz = zn + C.hz;
            // the voxel by floor (negative below the grid), inside iff every
            // index is in range: one test per axis decides both
            const int ix = (int)floorf(tx * C.inv_vox);
            const int iy = (int)floorf(ty * C.inv_vox);
            const int iz = (int)floorf(tz * C.inv_vox);
            const bool inside = ((uint32_t)ix < (uint32_t)C.nx) & ((uint32_t)iy < (uint32_t)C.ny) &
                                ((uint32_t)iz < (uint32_t)C.nz);
            // in the air outside the attenuation box, moving away from it, every
            // later collision would be virtual: the photon escapes along this ray
            // from the new point (one escape path for both ways out, so the
            // wavefront runs it once when lanes leave both ways)
            const bool box_exit = inside && C.box_margin && leaves_box(C, ix, iy, iz, L.dx, L.dy, L.dz);
            if (!inside || box_exit) {
                MC_REGION(RG_ESCAPE);
                if (box_exit) { L.x = xn; L.y = yn; L.z = zn; }
                fate = escape(C, L, iu, iv);
            }
            // the gather comes last in this phase, so nothing after it in the
            // phase can reuse its destination register while it is in flight
            pending = inside && !box_exit;
            if (pending) {
                MC_REGION(RG_GATHER);
                const uint32_t k = brick_index((uint32_t)ix, (uint32_t)iy, (uint32_t)iz, (uint32_t)C.nx,
                                               (uint32_t)C.ny, C.brick, C.bmask, C.nbx, C.nby);
                raw = C.use_pal ? (uint32_t)ldg(C.q8 + k) : ldg(C.q32 + k);
            }
        }
    }
    // (2) Kahn's rejection sampler for x = E/E' on [1, 1+2k], k = E / m_e c^2
    bool new_energy = false;
    float kn_fr, kn0, kn1;      // set with new_energy
    if (state == S_KAHN) {
        MC_REGION(RG_KAHN);
        A.n_kahn++;
        const float k = L.e * INV_MEC2;
        const float ik = MEC2_F * rcpf(L.e);
        const float tk = 2.0f * k;
        const float r1 = unif(w0), r2 = unif(w1), r3 = unif(w2);
        const float den = fmaf(tk, r2, 1.0f);
        const float r_den = rcpf(den);
        // both candidates from one reciprocal each; the first branch of
        // Kahn's method is x = den, the second x = (1 + 2k) / den
        const bool first = r1 * (9.0f + tk) <= 1.0f + tk;
        const float xx = first ? den : (1.0f + tk) * r_den;
        const float ixx = first ? r_den : den * rcpf(1.0f + tk);
        const float c = 1.0f - (xx - 1.0f) * ik;
        const bool acc = first ? (r3 <= 4.0f * (ixx - ixx * ixx)) : (r3 <= 0.5f * fmaf(c, c, ixx));
        if (!acc) {
            L.a += 1;
            if (L.a >= KAHN_MAX) fate = MC_CAPPED_FATE;
        } else {
            MC_REGION(RG_KAHN_ACCEPT);
            const float ct = 1.0f - (xx - 1.0f) * ik;
            L.e = L.e * ixx;
            {
                // the KN table pair of the new energy, read before the
                // rotation so the load is in flight during it
                const float t = (C.e0 - L.e) * KN_TABLE_STEP_INV;
                const int i = (int)t;
                kn_fr = t - (float)i;
                kn0 = ldg(C.kn_table + i);
                kn1 = ldg(C.kn_table + i + 1);
            }
            L.n_scatter += 1;
            rotate(L, ct, unif(L.phi_word));
            if (L.e < C.e_cut) {
                fate = MC_CUT;
            } else {
                new_energy = true;
                L.state = S_STEP;
            }
        }
    }
    // (3) the tentative collision is real iff (r >> 8) < Q_v
    if (pending) {
        MC_REGION(RG_ACCEPT_TEST);
        const uint32_t q = C.use_pal ? pal[raw] : raw;
        L.x = xn; L.y = yn; L.z = zn;
        if ((w1 >> 8) < q) {
            MC_REGION(RG_REAL);
            A.n_real++;
            if (fi) L.w *= 1.0f - L.p_pe;
            else if (unif(w2) < L.p_pe) fate = MC_ABSORBED;
            if (fate == R_RUNNING) {
                L.phi_word = w3;
                L.a = 0;
                L.state = S_KAHN;
            }
        }
    }
    // (4) flight scale and photoelectric share at the new energy
    if (new_energy) {
        MC_REGION(RG_ENERGY_TERMS);
        energy_terms_kn(C, L.e, kn_fr, kn0, kn1, L.ln2_mm, L.p_pe);
    }
    return fate;
}

// ---------------------------------------------------------------------------
// Forced detection (Sec. 5.2).  At the emission point and at every real
// collision a copy of the photon is forced to this view's detector, with the
// weight the paper lists: the probabilities of not being absorbed there, of
// leaving in a direction the collimator passes, and of crossing the rest of
// the object.  The copy's direction is uniform in the collimator cone (Philox
// event of the point, sub-draw FD_SUB, words 0 and 1):
//   w = Omega_cone pdf(direction) exp(-g(E') integral of mu140 on the ray),
// pdf = 1/(4 pi) at emission, (1 - p_pe(E)) times the Klein-Nishina angular
// density at a collision; the expected score in each bin is the expected
// analog count.  No score if E' is cut or outside the window, or the ray
// misses the detector.
// ---------------------------------------------------------------------------
constexpr uint32_t FD_SUB = 0x80000000u;
constexpr float FOUR_PI_F = 12.566370614359172f;
constexpr float TWO_PI_F = 6.283185307179586f;

struct FdPoint {
    float x, y, z;       // scoring point
    float dx, dy, dz;    // direction before the collision (unused at emission)
    float e;             // energy before the collision
    uint32_t view, hist, event;   // event 0: emission
    uint32_t voxel;      // phantom voxel of the history's emission
};

constexpr int RAY_BATCH = 8;

// State of a voxel walk: the current voxel (linear index), the planes
// crossed, the ray parameter reached, the next plane per axis, and whether
// it has ended.
struct RayWalk {
    int v;
    uint32_t n;
    float t, tx, ty, tz;
    bool done;
};
// What the walk does not change: linear voxel step per axis, plane spacing
// in t per axis, the exit parameter, the last voxel index.
struct RaySteps {
    int stx, sty, stz;
    float ddx, ddy, ddz, t_exit;
    uint32_t vmax;
};

// RAY_BATCH pieces of the walk: piece k is voxel v from t to min(next plane,
// exit); a finished walk repeats its last voxel with length 0.  The walk ends
// when the next plane lies at or beyond the exit (the grid's, or the
// attenuation box's); the voxels are not tracked per axis.  Where rounding
// puts the grid's last plane just before t_exit, the walk takes one more
// step, past the grid edge, whose piece is as short as that rounding
// difference: its index is clamped into the map (any voxel's mu times a
// length of rounding size).  The pieces' mu gathers are issued at the end
// (byte offsets below 2^32: axes of at most 1024 voxels).
__device__ __forceinline__ void ray_batch(const Cst& C, const RaySteps& s, RayWalk& w,
                                          const float* __restrict__ mu_map, float (&mu)[RAY_BATCH],
                                          float (&lb)[RAY_BATCH]) {
    uint32_t vb[RAY_BATCH];
#pragma unroll
    for (int k = 0; k < RAY_BATCH; ++k) {
        const float tn = fminf(w.tx, fminf(w.ty, w.tz));
        vb[k] = min((uint32_t)w.v, s.vmax);
        lb[k] = w.done ? 0.0f : fminf(tn, s.t_exit) - w.t;
        const bool bx = (w.tx <= w.ty) & (w.tx <= w.tz);
        const bool by = !bx & (w.ty <= w.tz);
        const bool bz = !bx & !by;
        w.done = w.done | (tn >= s.t_exit);
        if (!w.done) {
            w.t = tn;
            w.n += 1;
            w.tx += bx ? s.ddx : 0.0f; w.ty += by ? s.ddy : 0.0f; w.tz += bz ? s.ddz : 0.0f;
            // one term per axis (selects against 0, not between the steps)
            w.v += (bx ? s.stx : 0) + (by ? s.sty : 0) + (bz ? s.stz : 0);
        }
    }
#pragma unroll
    for (int k = 0; k < RAY_BATCH; ++k) mu[k] = ldg((const float*)((const char*)mu_map + vb[k] * 4u));
}

__device__ __forceinline__ void ray_add(float& sum, const float (&mu)[RAY_BATCH], const float (&lb)[RAY_BATCH]) {
#pragma unroll
    for (int k = 0; k < RAY_BATCH; ++k) sum = fmaf(mu[k], lb[k], sum);
}

// Integral of mu140 along p + t o (t >= 0, o a unit vector) to the grid edge:
// voxel walk (Amanatides & Woo 1987) with the advancing axis chosen by
// selects, so the lanes of a wavefront stay together.  The walk runs
// RAY_BATCH crossings of pure arithmetic and issues their RAY_BATCH mu
// gathers together; two batches alternate buffers, so a batch's gathered
// values are summed after the next batch has been walked and its gathers
// issued, and a gather's latency overlaps a whole batch of work (the sum is
// still taken piece by piece in walk order).  Plane parameters use the
// reciprocals of the direction's components (one division per axis); the
// gathers take a 32-bit offset from the map's base in scalar registers.
__device__ inline float ray_mu(const Cst& C, float x, float y, float z, float ox, float oy, float oz,
                               uint32_t& pieces) {
    const float px = x + C.hx, py = y + C.hy, pz = z + C.hz;
    RayWalk w;
    const int ix = min(max((int)(px * C.inv_vox), 0), C.nx - 1);
    const int iy = min(max((int)(py * C.inv_vox), 0), C.ny - 1);
    const int iz = min(max((int)(pz * C.inv_vox), 0), C.nz - 1);
    const float inf = __builtin_huge_valf();
    // 1 / o per axis (inf for a zero component: never selected)
    const float rx = ox != 0.0f ? 1.0f / ox : inf, ry = oy != 0.0f ? 1.0f / oy : inf;
    const float rz = oz != 0.0f ? 1.0f / oz : inf;
    RaySteps s;
    w.tx = ox != 0.0f ? fmaxf(((float)(ix + (ox > 0.0f)) * C.vox - px) * rx, 0.0f) : inf;
    w.ty = oy != 0.0f ? fmaxf(((float)(iy + (oy > 0.0f)) * C.vox - py) * ry, 0.0f) : inf;
    w.tz = oz != 0.0f ? fmaxf(((float)(iz + (oz > 0.0f)) * C.vox - pz) * rz, 0.0f) : inf;
    s.ddx = ox != 0.0f ? C.vox * fabsf(rx) : inf;
    s.ddy = oy != 0.0f ? C.vox * fabsf(ry) : inf;
    s.ddz = oz != 0.0f ? C.vox * fabsf(rz) : inf;
    // exit of the grid, and of the attenuation box (mu is zero outside it):
    // per axis the far plane, (plane - p) / o; the nearest of the three
    const float ex = ox > 0.0f ? (C.lx - px) * rx : (ox < 0.0f ? -px * rx : inf);
    const float ey = oy > 0.0f ? (C.ly - py) * ry : (oy < 0.0f ? -py * ry : inf);
    const float ez = oz > 0.0f ? (C.lz - pz) * rz : (oz < 0.0f ? -pz * rz : inf);
    s.t_exit = fmaxf(fminf(ex, fminf(ey, ez)), 0.0f);
    if (in_box(C, ix, iy, iz)) {
        const float bx = ox > 0.0f ? ((float)((C.bbx >> 16) + 1u) * C.vox - px) * rx
                                   : (ox < 0.0f ? ((float)(C.bbx & 0xFFFFu) * C.vox - px) * rx : inf);
        const float by = oy > 0.0f ? ((float)((C.bby >> 16) + 1u) * C.vox - py) * ry
                                   : (oy < 0.0f ? ((float)(C.bby & 0xFFFFu) * C.vox - py) * ry : inf);
        const float bz = oz > 0.0f ? ((float)((C.bbz >> 16) + 1u) * C.vox - pz) * rz
                                   : (oz < 0.0f ? ((float)(C.bbz & 0xFFFFu) * C.vox - pz) * rz : inf);
        s.t_exit = fminf(s.t_exit, fmaxf(fminf(bx, fminf(by, bz)), 0.0f));
    }
    s.stx = ox > 0.0f ? 1 : -1;
    s.sty = oy > 0.0f ? C.nx : -C.nx;
    s.stz = oz > 0.0f ? C.nx * C.ny : -(C.nx * C.ny);
    s.vmax = (uint32_t)(C.nx * C.ny * C.nz - 1);
    w.v = ix + C.nx * (iy + C.ny * iz);
    w.n = 0;
    w.t = 0.0f;
    w.done = false;
    float sum = 0.0f;
    const int max_batches = (C.nx + C.ny + C.nz + 3) / RAY_BATCH + 1;
    const float* __restrict__ mu_map = (const float*)uniform_ptr(C.mu);
    float mu_a[RAY_BATCH], lb_a[RAY_BATCH], mu_b[RAY_BATCH], lb_b[RAY_BATCH];
    ray_batch(C, s, w, mu_map, mu_a, lb_a);
    int it = 1;
    for (; it + 1 < max_batches && !w.done; it += 2) {
        ray_batch(C, s, w, mu_map, mu_b, lb_b);
        ray_add(sum, mu_a, lb_a);
        ray_batch(C, s, w, mu_map, mu_a, lb_a);
        ray_add(sum, mu_b, lb_b);
    }
    if (it < max_batches && !w.done) {     // one batch left (max_batches even)
        ray_batch(C, s, w, mu_map, mu_b, lb_b);
        ray_add(sum, mu_a, lb_a);
        ray_add(sum, mu_b, lb_b);
    } else {
        ray_add(sum, mu_a, lb_a);
    }
    // voxels the walk visited: one per plane crossed, plus the first
    pieces = w.n + 1;
    return sum;
}

// A forced copy that scores, up to its ray walk: start point, direction,
// weight before transmission, the attenuation scale g(E') of the walk's
// integral, its target (tally bin, or index in the CFD depth layers), and
// what the tally and the event list take from the copy (view, history id,
// emission voxel).  Score = w exp(-g integral of mu140 along the ray).
struct FdJob {
    float x, y, z, ox, oy, oz, w, g;
    uint32_t bin_lo, bin_hi;
    uint32_t view, hist, voxel;
};

__device__ inline float fd_walk_score(const Cst& C, const FdJob& j, uint32_t& pieces) {
    return j.w * __expf(-j.g * ray_mu(C, j.x, j.y, j.z, j.ox, j.oy, j.oz, pieces));
}

// Set-up of one forced copy: false if it scores nothing (energy out of the
// window or cut, or the ray misses the detector), else its job with the
// tally bin in bin_lo.  d: the problem's descriptor (cone and Klein-Nishina
// constants).
__device__ inline bool fd_setup(const Cst& C, const ProbDesc* __restrict__ d, const FdPoint& q, FdJob& j) {
    const float omc = d->omc_alpha, kn140 = (float)d->kn140;
    uint32_t r0 = q.hist, r1 = q.view, r2 = q.event, r3 = FD_SUB;
    philox10(r0, r1, r2, r3, C.seed, C.pid);
    const float2 vw = ldg(C.views + q.view);
    float ox = vw.x, oy = vw.y, oz = 0.0f;
    rotate_dir(ox, oy, oz, fmaf(-unif(r0), omc, 1.0f), unif(r1));
    float w, e2;
    if (q.event == 0) {
        w = 0.5f * omc;
        e2 = q.e;
    } else {
        const float ct = q.dx * ox + q.dy * oy + q.dz * oz;
        const float eps = rcpf(fmaf(q.e * INV_MEC2, 1.0f - ct, 1.0f));
        e2 = q.e * eps;
        float l2, ppe;
        energy_terms(C, q.e, l2, ppe);
        const float pdf = eps * eps * (eps + rcpf(eps) - (1.0f - ct * ct)) *
                          rcpf(FOUR_PI_F * kn140 * kn_ratio(C, q.e));
        w = (1.0f - ppe) * (TWO_PI_F * omc) * pdf;
    }
    if (!(e2 >= C.e_cut && e2 >= C.e_lo && e2 <= C.e_hi)) return false;
    const float dn = ox * vw.x + oy * vw.y;
    const float tp = (C.radius - (q.x * vw.x + q.y * vw.y)) * rcpf(dn);
    const float px = fmaf(tp, ox, q.x), py = fmaf(tp, oy, q.y), pz = fmaf(tp, oz, q.z);
    const float au = (-vw.y * px + vw.x * py) + 0.5f * C.wu;
    const float av = pz + 0.5f * C.wv;
    if (!(au >= 0.0f && au < C.wu && av >= 0.0f && av < C.wv)) return false;
    const int iu = min((int)(au * C.inv_pix), C.nu - 1);
    const int iv = min((int)(av * C.inv_pix), C.nv - 1);
    float l2, ppe;
    j.g = e2 == C.e0 ? C.g0 : energy_terms(C, e2, l2, ppe);
    j.x = q.x; j.y = q.y; j.z = q.z;
    j.ox = ox; j.oy = oy; j.oz = oz;
    j.w = w;
    const uint32_t cls = q.event == 0 ? 0u : 1u;
    j.bin_lo = ((q.view * 2u + cls) * (uint32_t)C.nv + (uint32_t)iv) * (uint32_t)C.nu + (uint32_t)iu;
    j.bin_hi = 0;
    j.view = q.view; j.hist = q.hist; j.voxel = q.voxel;
    return true;
}

// Convolution-based forced detection (Sec. 5.2): the forced copy goes along
// the detector normal n_k instead of a direction drawn in the cone, with the
// weight above taken at that direction, and is stored in the sub-projection
// layer of its depth D - n_k . x (one pixel per layer, clamped to the layer
// range) at the pixel of its perpendicular hit.  The set-up: false if it
// scores nothing, else its job with the index in the problem's layers
// [V][L][2][nv][nu] in (bin_lo, bin_hi).  The layers are convolved with the
// collimator response of their depth after transport.
__device__ inline bool cfd_setup(const Cst& C, const ProbDesc* __restrict__ d, const FdPoint& q, FdJob& j) {
    const float omc = d->omc_alpha, kn140 = (float)d->kn140;
    const float2 vw = ldg(C.views + q.view);
    float w, e2;
    if (q.event == 0) {
        w = 0.5f * omc;
        e2 = q.e;
    } else {
        const float ct = q.dx * vw.x + q.dy * vw.y;
        const float eps = rcpf(fmaf(q.e * INV_MEC2, 1.0f - ct, 1.0f));
        e2 = q.e * eps;
        float l2, ppe;
        energy_terms(C, q.e, l2, ppe);
        const float pdf = eps * eps * (eps + rcpf(eps) - (1.0f - ct * ct)) *
                          rcpf(FOUR_PI_F * kn140 * kn_ratio(C, q.e));
        w = (1.0f - ppe) * (TWO_PI_F * omc) * pdf;
    }
    if (!(e2 >= C.e_cut && e2 >= C.e_lo && e2 <= C.e_hi)) return false;
    const float au = (-vw.y * q.x + vw.x * q.y) + 0.5f * C.wu;
    const float av = q.z + 0.5f * C.wv;
    if (!(au >= 0.0f && au < C.wu && av >= 0.0f && av < C.wv)) return false;
    const int iu = min((int)(au * C.inv_pix), C.nu - 1);
    const int iv = min((int)(av * C.inv_pix), C.nv - 1);
    const int nl = d->cfd_L;
    const float depth = C.radius - (q.x * vw.x + q.y * vw.y);
    const int l = min(max((int)floorf(depth * C.inv_pix), 0), nl - 1);
    float l2, ppe;
    j.g = e2 == C.e0 ? C.g0 : energy_terms(C, e2, l2, ppe);
    j.x = q.x; j.y = q.y; j.z = q.z;
    j.ox = vw.x; j.oy = vw.y; j.oz = 0.0f;
    j.w = w;
    const uint32_t cls = q.event == 0 ? 0u : 1u;
    const uint64_t lbin = ((((uint64_t)q.view * (uint64_t)nl + (uint64_t)l) * 2u + cls) * (uint64_t)C.nv +
                           (uint64_t)iv) * (uint64_t)C.nu + (uint64_t)iu;
    j.bin_lo = (uint32_t)lbin;
    j.bin_hi = (uint32_t)(lbin >> 32);
    j.view = q.view; j.hist = q.hist; j.voxel = q.voxel;
    return true;
}

}  // namespace
}  // namespace mcs
